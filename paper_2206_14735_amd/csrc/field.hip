// Fused per-sample field kernels: multi-level trilinear gather, geometry and
// colour decoders on MFMA, d(phi)/dx, and (backward) decoder weight gradients,
// the double backward of the gradient terms and the grid scatter.
//
// Work decomposition (one wave = 64 lanes):
//   a wave-tile is 16 consecutive samples; lane l serves sample l % 16 and
//   grid level q = l / 16.  Each lane gathers only its level's 8 corners, and
//   the 16-d feature z lands directly in the B-operand layout of the
//   16x16x4 MFMA (lane q holds rows 4q..4q+3 = level q's four features).
//   Decoder activations stay in MFMA accumulator layout between layers
//   ([neuron][sample], lane (q, j) holds rows 16b + 4q + r of sample j), so
//   layers chain in registers; weights are pre-arranged per lane in LDS.
//   Weight gradients (sums over samples) are MFMAs with the sample axis as K;
//   their operands are transposed through a small per-wave LDS scratch.
#include "args.h"
#include "gather.h"
#include "mfma.h"

namespace gs {

// ---------------------------------------------------------------- A-operand tables in LDS
// slot = table base + out_block * (4 * in_blocks) + step; 64 floats per slot.
enum : int {
  T_L1 = 0,    // W1       out 32 (2 blk), in 16 (1 blk)
  T_L2 = 8,    // W2       out 32, in 32
  T_L3 = 24,   // W3       out 16, in 32
  T_C1 = 32,   // U1       out 32, in o-index 16 (row 0 = phi -> 0)
  T_C2 = 40,   // U2       out 16 (rows 0..2), in 32
  T_C2T = 48,  // U2^T     out 32, in 16 (rows 0..2)
  T_C1T = 56,  // U1^T     out o-index 16, in 32
  T_L3T = 64,  // W3^T     out 32, in 16
  T_L2T = 72,  // W2^T     out 32, in 32
  T_L1T = 88,  // W1^T     out 16, in 32
  T_END = 96
};

__device__ float table_value(const float* __restrict__ P, int slot, int l) {
  int tb, nbi;
  if (slot < T_L2) { tb = T_L1; nbi = 1; }
  else if (slot < T_L3) { tb = T_L2; nbi = 2; }
  else if (slot < T_C1) { tb = T_L3; nbi = 2; }
  else if (slot < T_C2) { tb = T_C1; nbi = 1; }
  else if (slot < T_C2T) { tb = T_C2; nbi = 2; }
  else if (slot < T_C1T) { tb = T_C2T; nbi = 1; }
  else if (slot < T_L3T) { tb = T_C1T; nbi = 2; }
  else if (slot < T_L2T) { tb = T_L3T; nbi = 1; }
  else if (slot < T_L1T) { tb = T_L2T; nbi = 2; }
  else { tb = T_L1T; nbi = 2; }
  int rel = slot - tb;
  int bo = rel / (4 * nbi), s = rel % (4 * nbi);
  int i = 16 * bo + (l & 15);                       // output row
  int k = 16 * (s >> 2) + 4 * (l >> 4) + (s & 3);   // input row
  switch (tb) {
    case T_L1: return P[oW1 + i * 16 + k];
    case T_L2: return P[oW2 + i * 32 + k];
    case T_L3: return P[oW3 + i * 32 + k];
    case T_C1: return k >= 1 ? P[oU1 + i * 15 + (k - 1)] : 0.f;
    case T_C2: return i < 3 ? P[oU2 + i * 32 + k] : 0.f;
    case T_C2T: return k < 3 ? P[oU2 + k * 32 + i] : 0.f;
    case T_C1T: return i >= 1 ? P[oU1 + k * 15 + (i - 1)] : 0.f;
    case T_L3T: return P[oW3 + k * 32 + i];
    case T_L2T: return P[oW2 + k * 32 + i];
    default: return P[oW1 + k * 16 + i];
  }
}

// out[bo] = sum over input blocks/steps of A(slot) * in   (NBO output blocks of 16 rows).
// FP32: 4 steps of 16x16x4 per input block; BF16: one 16x16x16 per input block
// whose A operand packs the four fp32 steps' values of the same lane.
template <bool BF, int NBO, int NBI, class Smem>
__device__ __forceinline__ void layer(const Smem& sm, int base, const v4f* in, v4f* out, int lane) {
#pragma unroll
  for (int bo = 0; bo < NBO; ++bo) out[bo] = v4f{0.f, 0.f, 0.f, 0.f};
  if constexpr (BF) {
#pragma unroll
    for (int bi = 0; bi < NBI; ++bi) {
      const v4s b = pack_bf16(in[bi]);
#pragma unroll
      for (int bo = 0; bo < NBO; ++bo)
        out[bo] = mfma16_bf16(as_v4s(sm.tabbf[(base / 4 + bo * NBI + bi) * 64 + lane]), b, out[bo]);
    }
  } else {
    layer_f32<NBO, NBI>(sm.tab, base, in, out, lane);
  }
}

// One step of the segmented sum inside a 16-lane level group: lanes of the
// same run (equal cell) add their right neighbour's partial at distance D.
// The partial is taken as a multiply by 0 or 1, which folds into one
// v_fmac_f32 with a DPP source per value (the values are finite).
template <int CTRL, int D>
__device__ __forceinline__ void run_step(float (&val)[8][4], int segid, int j) {
  const int so = dpp_i<CTRL>(segid);
  const float take = (j + D < 16) && so == segid ? 1.f : 0.f;
#pragma unroll
  for (int c = 0; c < 8; ++c)
#pragma unroll
    for (int k = 0; k < 4; ++k) val[c][k] = fmaf(dpp_f<CTRL>(val[c][k]), take, val[c][k]);
}

// Per-wave LDS staging of the scatter, indexed by the writer's rank among the
// wave's writers (lane order), so that job k (writer k / 4, segment k % 4)
// finds its 8 floats at val[8 k] and its destination at dst[k].
struct ScatterStage {
  float* val;   // [64][32]: per writer, 4 segments (by, bz) of 8 floats (bx, feature)
  int* dst;     // [64][4]: vertex row of the segment's x = 0 corner, or, for a
                // level accumulated in LDS, ~(float offset in the block's copy)
};

// grid scatter: dL/dtheta_c,k = w_c dz_k + a_k (J_c . gvec) / v.
// 1. The 16 lanes of a level group hold 16 consecutive samples, so runs of
//    samples in the same cell sit in neighbouring lanes: a segmented sum
//    merges each run into its first lane (the writer).
// 2. Each writer's 32 values are 4 segments of 8 contiguous floats (the two
//    x-neighbour vertices of one (by, bz) edge, 4 features each).  Writers
//    stage them in LDS; then 8 lanes handle one segment, so every atomic
//    instruction covers 8 contiguous 32-byte segments instead of 64
//    scattered words (the memory system processes atomics per segment).
// 3. Small levels go to the block's LDS copy, the others to HBM.  The
//    writers compute their segments' destinations, so the atomic loop reads
//    only LDS (po >= 0: this lane's level has its LDS copy at float offset po).
// BF: the BF16 kernel (decoders in bf16), which keeps fewer atomics in flight.
// 4. With gradient copies (cpb >= 0: this lane's level scatters into four
//    x/y-parity copies), the writer of cell (i, j, k) uses copy (i & 1, j & 1),
//    where the cell's four corners at one z are one aligned 64-byte unit
//    [dy][dx][feature]: its four segments are two such units, one request each
//    instead of about five for the segments of the single layout.
template <bool HAS_DZ, bool HAS_GV, bool BF, bool COPIES>
__device__ __forceinline__ void scatter(const FieldArgs& A, float* priv, const ScatterStage& S, int lane, int q,
                                        int j, const LevelSample& ls, const LevelConst& lc, int po, int cpb,
                                        bool valid, const float dz[4], const float a[4], const float gv[3]) {
  // an invalid lane's inputs are zeroed (and its weights kept finite), so
  // its 32 values are exact zeros
  const float fx = valid ? ls.f[0] : 0.f, fy = valid ? ls.f[1] : 0.f, fz = valid ? ls.f[2] : 0.f;
  float dzv[4], av[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    dzv[k] = valid ? dz[k] : 0.f;
    av[k] = valid ? a[k] : 0.f;
  }
  float val[8][4];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const float wx = bx ? fx : 1.f - fx, wy = by ? fy : 1.f - fy, wz = bz ? fz : 1.f - fz;
    float jg = 0.f;
    if (HAS_GV) {
      const float jx = (bx ? 1.f : -1.f) * wy * wz, jy = (by ? 1.f : -1.f) * wx * wz,
                  jz = (bz ? 1.f : -1.f) * wx * wy;
      jg = (jx * gv[0] + jy * gv[1] + jz * gv[2]) * ls.inv_v;
    }
    const float w = wx * wy * wz;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float v = 0.f;
      if (HAS_DZ) v += w * dzv[k];
      if (HAS_GV) v += av[k] * jg;
      val[c][k] = v;
    }
  }
  // runs of equal cells (invalid lanes form runs of their own and never write)
  const int key = valid ? (int)ls.row : -1 - j;
  const int kprev = dpp_i<kRowShr1>(key);
  const bool head = (j == 0) || key != kprev;
  const unsigned long long hm = __ballot(head);
  const unsigned g = (unsigned)(hm >> (16 * q)) & 0xffffu;
  const int segid = __popc(g & ((2u << j) - 1u));
  run_step<kRowShl1, 1>(val, segid, j);
  run_step<kRowShl2, 2>(val, segid, j);
  run_step<kRowShl4, 4>(val, segid, j);
  run_step<kRowShl8, 8>(val, segid, j);

  const bool writer = head && valid;
  const unsigned long long wm = __ballot(writer);
  const int nw = __popcll(wm);
  if (writer) {
    const int rank = __popcll(wm & ((1ull << lane) - 1ull));
    float* st = S.val + rank * 32;
    int unit = 0, plane = 0;
    if (COPIES && cpb >= 0) {
      const int ci = ls.cell & 2047, cj = (ls.cell >> 11) & 2047, ck = ls.cell >> 22;
      const int mx = (lc.n[0] >> 1) + 1, my = (lc.n[1] >> 1) + 1;
      plane = mx * my * 16;
      unit = cpb + ((ci & 1) + 2 * (cj & 1)) * (lc.n[2] * plane) + ck * plane + ((cj >> 1) * mx + (ci >> 1)) * 16;
    }
#pragma unroll
    for (int sg = 0; sg < 4; ++sg) {
      const int c0 = sg, c1 = 4 + sg;   // corners (0, by, bz) and (1, by, bz), sg = 2 by + bz
      *reinterpret_cast<float4*>(st + 8 * sg) = make_float4(val[c0][0], val[c0][1], val[c0][2], val[c0][3]);
      *reinterpret_cast<float4*>(st + 8 * sg + 4) = make_float4(val[c1][0], val[c1][1], val[c1][2], val[c1][3]);
      const long long row = ls.row + (long long)(sg >> 1) * ls.sy + (long long)(sg & 1) * ls.sz;
      S.dst[4 * rank + sg] = po >= 0   ? ~(po + 4 * (int)(row - lc.off))
                             : COPIES && cpb >= 0 ? unit + (sg & 1) * plane + (sg >> 1) * 8
                                       : (int)row;
    }
  }
  wave_lds_fence();
  // Eight lanes per job, eight jobs per atomic instruction.  The next
  // instruction's values are read from LDS before the wait below, so the LDS
  // latency overlaps the memory system's.
  const int jobs = 4 * nw;
  const int f = lane & 7;
  int k = lane >> 3;
  float v = 0.f;
  int d = 0;
  if (k < jobs) { v = S.val[8 * k + f]; d = S.dst[k]; }
  for (int base = 0; base < jobs; base += 8) {
    const int kn = k + 8;
    float vn = 0.f;
    int dn = 0;
    if (kn < jobs) { vn = S.val[8 * kn + f]; dn = S.dst[kn]; }
    // At most two (FP32) or one (BF16) atomic instructions of this wave in
    // flight: issued back to back, a tile's atomics queue in the memory system
    // ahead of the other waves' gathers.  Measured on MI355X, backward kernel
    // on the room batch in FP32: 0.43 ms unthrottled, 0.44 ms with one, 0.39
    // ms with two, 0.39 ms with four in flight; at 65536 rays in BF16, whose
    // decoders take less time per tile: 3.13 ms with one, 3.30 ms with two.
    if constexpr (BF) wait_vmem_at_most<0>();
    else wait_vmem_at_most<1>();
    if (k < jobs) {
      if (d < 0) atomic_add_lds(priv + (~d) + f, v);
      else if constexpr (COPIES) atomic_add_global(A.copies + d + f, v);   // every level not in LDS has copies
      else atomic_add_global(A.grad_grid + (long long)d * 4 + f, v);
    }
    k = kn;
    v = vn;
    d = dn;
  }
  wave_lds_fence();
}

__device__ __forceinline__ v4f relu_mask(v4f x, v4f h) {
  return v4f{h[0] > 0.f ? x[0] : 0.f, h[1] > 0.f ? x[1] : 0.f, h[2] > 0.f ? x[2] : 0.f,
             h[3] > 0.f ? x[3] : 0.f};
}

// LDS footprint of one block.  The fp32 kernels keep one float per lane per
// MFMA step, the bf16 kernels four packed bf16 values per lane per input block;
// only the backward kernels need the per-wave scratch.
template <bool BF, bool BWD>
struct FieldSmem {
  float tab[BF ? 1 : T_END * 64];
  uint2 tabbf[BF ? (T_END / 4) * 64 : 1];
  float bias[32 + 32 + 16 + 32 + 16];   // b1, b2, b3, c1, c2(pad 16)
  float w3row0[32];
  float scr[kWavesPerBlock][BWD ? 2048 : 1];   // operand transposes, then scatter staging
  int dst[kWavesPerBlock][BWD ? 256 : 1];
};
constexpr int kRedFloats = kWavesPerBlock * kMlpNumel;
// the area is reused at the end for the per-wave block partials
template <bool BF, bool BWD>
constexpr int smem_bytes() {
  constexpr int red = BWD ? kRedFloats * 4 : kWavesPerBlock * 4;
  return (sizeof(FieldSmem<BF, BWD>) > red) ? (int)sizeof(FieldSmem<BF, BWD>) : red;
}
constexpr int kPrivMaxFloats = 4096;
constexpr int kFieldMaxBlocksFwd = 4096;   // rows of the smoothness partials in the workspace
constexpr int kFieldMaxBlocksBwd = 2048;   // rows of the decoder / level partials in the workspace   // LDS budget for privatised levels (1024 vertices)

// One wave-tile: MODE 0 = 16 ray samples, MODE 1 = 8 smoothness pairs (lanes
// j < 8 hold x, lanes j >= 8 hold x + eps of the same pair).  POSE (backward
// only): also dL/dx of every ray sample, for camera pose refinement.
template <int MODE, bool BWD, bool BF, bool POSE, bool COPIES, class Smem>
__device__ __forceinline__ void field_tile(const FieldArgs& A, const Smem& sm, int tile, int total, int lane, int q,
                                           int j, const LevelConst& lc, int po, int cpb, float* scrA, float* scrB,
                                           const ScatterStage& stage, float* priv,
                                           v4f (&aW1)[2], v4f (&aW2)[4], v4f (&aW3)[2], v4f (&aU1)[2], v4f& aS,
                                           float& smooth_acc) {
  // ---------------- sample position
  int item;
  float px, py, pz;
  bool live;
  float4 seed_in = make_float4(0.f, 0.f, 0.f, 0.f);   // backward: dL/dphi, dL/dc of the sample
  float ew_in = 0.f;                                   // backward: its Eikonal weight
  float b_fs = 0.f;                                    // forward: D - t of the sample (-1 without depth)
  if (MODE == 0) {
    item = tile * 16 + j;
    live = item < total;
    px = py = pz = 0.f;
    if (live) {
      if constexpr (BWD) {
        // position and seeds in one round of independent loads
        const float4 p4 = *reinterpret_cast<const float4*>(A.posw + 4 * (size_t)item);
        seed_in = *reinterpret_cast<const float4*>(A.seed4 + 4 * (size_t)item);
        px = p4.x; py = p4.y; pz = p4.z; ew_in = p4.w;
      } else {
        const int ray = A.ray_of[item];
        const float tt = A.t[item];
        px = mad_norm(tt, A.r[3 * ray + 0], A.o[3 * ray + 0]);
        py = mad_norm(tt, A.r[3 * ray + 1], A.o[3 * ray + 1]);
        pz = mad_norm(tt, A.r[3 * ray + 2], A.o[3 * ray + 2]);
        if (A.depth) {
          const float D = A.depth[ray];
          b_fs = D > 0.f ? D - tt : -1.f;
        }
      }
    }
  } else {
    const int pair = tile * 8 + (j & 7);
    item = pair;
    live = pair < A.S;
    px = py = pz = 0.f;
    if (live) {
      px = A.xs[3 * pair + 0];
      py = A.xs[3 * pair + 1];
      pz = A.xs[3 * pair + 2];
      if (j >= 8) {
        px = __fadd_rn(px, A.eps[3 * pair + 0]);
        py = __fadd_rn(py, A.eps[3 * pair + 1]);
        pz = __fadd_rn(pz, A.eps[3 * pair + 2]);
      }
    }
  }
  const bool valid = live && inside_box(A.g, px, py, pz);
  // d(phi)/dx is needed at smoothness points, for pose refinement, and for
  // the Eikonal term, which only samples of S_fs = {D - t > trunc} (decided in
  // float32 as the render decides it) carry.  A wave-tile with no such sample
  // skips the gradient of the interpolation and the decoders' d(phi)/dz,
  // which contribute exactly zero there.
  bool need_g = (MODE == 1) || POSE;
  if (MODE == 0 && !POSE && A.need_gx) {
    bool lane_fs;
    if constexpr (BWD) lane_fs = valid && ew_in != 0.f;
    else lane_fs = A.grad_phi != nullptr || A.depth == nullptr || (valid && b_fs > A.trunc);
    need_g = __ballot(lane_fs) != 0ull;
  }
  LevelSample ls;
  locate(A.g, lc, px, py, pz, ls);
  float zl[4], G[4][3];
  LevelHess hs;   // second derivatives of this level's features (pose refinement)
  if constexpr (POSE && MODE == 0) interp<true, BF, true>(A.grid, A.grid_bf16, ls, valid, zl, G, &hs);
  else if (need_g) interp<true, BF>(A.grid, A.grid_bf16, ls, valid, zl, G);
  else interp<false, BF>(A.grid, A.grid_bf16, ls, valid, zl, G);

  // ---------------- geometry decoder
  v4f zb = v4f{zl[0], zl[1], zl[2], zl[3]};
  v4f h1[2], h2[2], ob, hc[2], cb;
  layer<BF, 2, 1>(sm, T_L1, &zb, h1, lane);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[b][r] = fmaxf(h1[b][r] + sm.bias[16 * b + 4 * q + r], 0.f);
  layer<BF, 2, 2>(sm, T_L2, h1, h2, lane);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[b][r] = fmaxf(h2[b][r] + sm.bias[32 + 16 * b + 4 * q + r], 0.f);
  layer<BF, 1, 2>(sm, T_L3, h2, &ob, lane);
#pragma unroll
  for (int r = 0; r < 4; ++r) ob[r] += sm.bias[64 + 4 * q + r];

  // ---------------- colour decoder (ray mode)
  if (MODE == 0 && A.colour) {
    layer<BF, 2, 1>(sm, T_C1, &ob, hc, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) hc[b][r] = fmaxf(hc[b][r] + sm.bias[80 + 16 * b + 4 * q + r], 0.f);
    layer<BF, 1, 2>(sm, T_C2, hc, &cb, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) cb[r] = sigmoidf_(cb[r] + sm.bias[112 + 4 * q + r]);
  } else {
    cb = v4f{0.f, 0.f, 0.f, 0.f};
  }

  // ---------------- d phi / d x
  v4f e2[2], e1[2], ab;
  float gx[3] = {0.f, 0.f, 0.f};
  if (need_g) {
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) e2[b][r] = h2[b][r] > 0.f ? sm.w3row0[16 * b + 4 * q + r] : 0.f;
    layer<BF, 2, 2>(sm, T_L2T, e2, e1, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b) e1[b] = relu_mask(e1[b], h1[b]);
    layer<BF, 1, 2>(sm, T_L1T, e1, &ab, lane);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float v = ab[0] * G[0][a] + ab[1] * G[1][a] + ab[2] * G[2][a] + ab[3] * G[3][a];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      gx[a] = v;
    }
  }

  if constexpr (!BWD) {
    if (MODE == 0) {
      if (q == 0 && live) {
        *reinterpret_cast<float4*>(A.out4 + 4 * (size_t)item) = make_float4(ob[0], cb[0], cb[1], cb[2]);
        if (A.need_gx) {
          // (a tile that skipped d(phi)/dx holds no S_fs sample: its residuals are not read)
          const float n = sqrtf(gx[0] * gx[0] + gx[1] * gx[1] + gx[2] * gx[2]);
          A.eik[item] = need_g ? (1.f - n) * (1.f - n) : 0.f;
          if (A.grad_phi) {
            float* gp = A.grad_phi + 3 * (size_t)item;
            gp[0] = gx[0]; gp[1] = gx[1]; gp[2] = gx[2];
          }
        }
      }
    } else {
      if (A.grad_phi && q == 0 && live) {
        float* gp = A.grad_phi + 3 * ((size_t)A.total + 2 * (size_t)item + (j >> 3));
        gp[0] = gx[0]; gp[1] = gx[1]; gp[2] = gx[2];
      }
      // pair partner is lane j ^ 8 of the same level group
      float d0 = gx[0] - __shfl_xor(gx[0], 8, 64);
      float d1 = gx[1] - __shfl_xor(gx[1], 8, 64);
      float d2 = gx[2] - __shfl_xor(gx[2], 8, 64);
      const bool pv = valid && __shfl_xor((int)valid, 8, 64);
      const float sq = d0 * d0 + d1 * d1 + d2 * d2;
      if (q == 0 && j < 8 && pv) smooth_acc += sq;
      if (A.pair_terms && q == 0 && j < 8 && live) A.pair_terms[item] = pv ? sq : 0.f;
    }
    return;
  } else {

  // ================================================================ backward
  float gv[3] = {0.f, 0.f, 0.f};   // dL / d(grad phi)
  if (MODE == 0) {
    const float4 sd = valid ? seed_in : make_float4(0.f, 0.f, 0.f, 0.f);
    const float ew = valid && A.need_gx ? ew_in : 0.f;
    if (A.need_gx && ew != 0.f) {
      const float n = sqrtf(gx[0] * gx[0] + gx[1] * gx[1] + gx[2] * gx[2]);
      const float c = n > 0.f ? ew * 2.f * (n - 1.f) / n : 0.f;
      gv[0] = c * gx[0]; gv[1] = c * gx[1]; gv[2] = c * gx[2];
    }
    // colour: dL/d(pre-sigmoid) for rows 0..2 held by level-group 0
    const bool col = A.colour != 0;
    v4f dc2 = v4f{0, 0, 0, 0};
    if (q == 0 && col) {
      dc2[0] = sd.y * cb[0] * (1.f - cb[0]);
      dc2[1] = sd.z * cb[1] * (1.f - cb[1]);
      dc2[2] = sd.w * cb[2] * (1.f - cb[2]);
    }
    v4f dhc[2], dob = v4f{0, 0, 0, 0};
    if (col) {
      layer<BF, 2, 1>(sm, T_C2T, &dc2, dhc, lane);
#pragma unroll
      for (int b = 0; b < 2; ++b) dhc[b] = relu_mask(dhc[b], hc[b]);
      layer<BF, 1, 2>(sm, T_C1T, dhc, &dob, lane);
    }
    if (q == 0) dob[0] += sd.x;
    v4f dh2[2], dh1[2], dz;
    layer<BF, 2, 1>(sm, T_L3T, &dob, dh2, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b) dh2[b] = relu_mask(dh2[b], h2[b]);
    layer<BF, 2, 2>(sm, T_L2T, dh2, dh1, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b) dh1[b] = relu_mask(dh1[b], h1[b]);
    layer<BF, 1, 2>(sm, T_L1T, dh1, &dz, lane);

    if constexpr (POSE) {
      // dL/dx = sum over levels and features of dL/dz_k dz_k/dx, plus, through
      // the Eikonal residual, (d^2 phi/dx^2) dL/d(grad phi) with
      // d^2 phi/dx^2 = sum_k (df/dz_k) d^2 z_k/dx^2 (the decoder's own second
      // derivative vanishes for ReLU units; supplementary Eq.
      // second_sdf_grad_x and the h12, h13, h23 block)
      float dxv[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) dxv[a] = dz[0] * G[0][a] + dz[1] * G[1][a] + dz[2] * G[2][a] + dz[3] * G[3][a];
      if (A.need_gx) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const float ak = ab[k], h12 = hs.h[k][0], h13 = hs.h[k][1], h23 = hs.h[k][2];
          dxv[0] += ak * (h12 * gv[1] + h13 * gv[2]);
          dxv[1] += ak * (h12 * gv[0] + h23 * gv[2]);
          dxv[2] += ak * (h13 * gv[0] + h23 * gv[1]);
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        dxv[a] += __shfl_xor(dxv[a], 16, 64);
        dxv[a] += __shfl_xor(dxv[a], 32, 64);
      }
      // the seeds of this sample were read at the start of the tile by this wave
      // alone; their slot takes dL/dx
      if (q == 0 && live) *reinterpret_cast<float4*>(A.grad_x + 4 * (size_t)item) = make_float4(dxv[0], dxv[1], dxv[2], 0.f);
    }

    // weight gradients (sums over the tile's samples, the MFMA K axis)
    float4 tX[2], tY[2];
    if (col) {
      // U2 and c2: U2[c][k] = sum_s dc2[c][s] hc[k][s] goes to column 10 + 3b + c
      // of aS (row k - 16b), with hc as the A operand and dc2 row c as the B
      // operand of exactly those columns
      rows_to_lanes<2>(scrA, hc, tX, q, j);
      rows_to_lanes<1>(scrB, &dc2, tY, q, j);
      colsum_into(tY[0], 5, aS, j);
      {
        const int c = j >= 13 ? j - 13 : (j >= 10 ? j - 10 : 0);
        const float4 d = *reinterpret_cast<const float4*>(scrB + c * RSR + 4 * q);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const bool on = j >= 10 + 3 * b && j < 13 + 3 * b;
          aS = mfma4(tX[b].x, on ? d.x : 0.f, aS);
          aS = mfma4(tX[b].y, on ? d.y : 0.f, aS);
          aS = mfma4(tX[b].z, on ? d.z : 0.f, aS);
          aS = mfma4(tX[b].w, on ? d.w : 0.f, aS);
        }
      }
      // U1 and c1: o-index 0 (phi) does not feed the colour decoder; its
      // operand row is replaced by ones, so column 0 of aU1 sums dhc (= dc1)
      rows_to_lanes<2>(scrA, dhc, tX, q, j);
      rows_to_lanes<1>(scrB, &ob, tY, q, j);
      if (j == 0) tY[0] = make_float4(1.f, 1.f, 1.f, 1.f);
      outer_lanes<BF, 2, 1>(tX, tY, aU1);
    }
    // W3 and b3
    rows_to_lanes<1>(scrA, &dob, tX, q, j);
    rows_to_lanes<2>(scrB, h2, tY, q, j);
    outer_lanes<BF, 1, 2>(tX, tY, aW3);
    colsum_into(tX[0], 4, aS, j);
    // W2 and b2
    rows_to_lanes<2>(scrA, dh2, tX, q, j);
    rows_to_lanes<2>(scrB, h1, tY, q, j);
    outer_lanes<BF, 2, 2>(tX, tY, aW2);
    colsum_into(tX[0], 2, aS, j);
    colsum_into(tX[1], 3, aS, j);
    // W1 and b1
    rows_to_lanes<2>(scrA, dh1, tX, q, j);
    rows_to_lanes<1>(scrB, &zb, tY, q, j);
    outer_lanes<BF, 2, 1>(tX, tY, aW1);
    colsum_into(tX[0], 0, aS, j);
    colsum_into(tX[1], 1, aS, j);

    const float dzl[4] = {dz[0], dz[1], dz[2], dz[3]};
    if (need_g && A.need_gx) {
      // second-order terms of the Eikonal residual
      v4f qv;
#pragma unroll
      for (int k = 0; k < 4; ++k) qv[k] = gv[0] * G[k][0] + gv[1] * G[k][1] + gv[2] * G[k][2];
      v4f r1[2], w2r1[2];
      layer<BF, 2, 1>(sm, T_L1, &qv, r1, lane);
#pragma unroll
      for (int b = 0; b < 2; ++b) r1[b] = relu_mask(r1[b], h1[b]);
      layer<BF, 2, 2>(sm, T_L2, r1, w2r1, lane);
#pragma unroll
      for (int b = 0; b < 2; ++b) w2r1[b] = relu_mask(w2r1[b], h2[b]);
      float4 tX[2], tY[2];
      rows_to_lanes<2>(scrA, w2r1, tX, q, j);
      colsum_into(tX[0], 6, aS, j);
      colsum_into(tX[1], 7, aS, j);
      rows_to_lanes<2>(scrA, e2, tX, q, j);
      rows_to_lanes<2>(scrB, r1, tY, q, j);
      outer_lanes<BF, 2, 2>(tX, tY, aW2);
      rows_to_lanes<2>(scrA, e1, tX, q, j);
      rows_to_lanes<1>(scrB, &qv, tY, q, j);
      outer_lanes<BF, 2, 1>(tX, tY, aW1);
      const float al[4] = {ab[0], ab[1], ab[2], ab[3]};
      scatter<true, true, BF, COPIES>(A, priv, stage, lane, q, j, ls, lc, po, cpb, valid, dzl, al, gv);
    } else {
      const float al[4] = {0, 0, 0, 0};
      scatter<true, false, BF, COPIES>(A, priv, stage, lane, q, j, ls, lc, po, cpb, valid, dzl, al, gv);
    }
  } else {
    // smoothness pair: d|g(x) - g(x+eps)|^2 / dg at either point is
    // 2 (own gradient - partner's gradient); smooth_coef carries the 2.
    const bool pv = valid && __shfl_xor((int)valid, 8, 64);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float d = gx[a] - __shfl_xor(gx[a], 8, 64);
      gv[a] = pv ? A.smooth_coef * d : 0.f;
    }
    v4f qv;
#pragma unroll
    for (int k = 0; k < 4; ++k) qv[k] = gv[0] * G[k][0] + gv[1] * G[k][1] + gv[2] * G[k][2];
    v4f r1[2], w2r1[2];
    layer<BF, 2, 1>(sm, T_L1, &qv, r1, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b) r1[b] = relu_mask(r1[b], h1[b]);
    layer<BF, 2, 2>(sm, T_L2, r1, w2r1, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b) w2r1[b] = relu_mask(w2r1[b], h2[b]);
    float4 tX[2], tY[2];
    rows_to_lanes<2>(scrA, w2r1, tX, q, j);
    colsum_into(tX[0], 6, aS, j);
    colsum_into(tX[1], 7, aS, j);
    rows_to_lanes<2>(scrA, e2, tX, q, j);
    rows_to_lanes<2>(scrB, r1, tY, q, j);
    outer_lanes<BF, 2, 2>(tX, tY, aW2);
    rows_to_lanes<2>(scrA, e1, tX, q, j);
    rows_to_lanes<1>(scrB, &qv, tY, q, j);
    outer_lanes<BF, 2, 1>(tX, tY, aW1);
    const float al[4] = {ab[0], ab[1], ab[2], ab[3]};
    const float dzl[4] = {0, 0, 0, 0};
    scatter<false, true, BF, COPIES>(A, priv, stage, lane, q, j, ls, lc, po, cpb, pv, dzl, al, gv);
  }
  }
}

// Pair tiles come first, then ray tiles, in one launch: the few pair tiles
// overlap with the ray tiles of other waves.
// At least two waves per SIMD: the backward kernels then fit 256 registers
// without spilling, and a second wave hides the gather and atomic latency.
template <bool BWD, bool BF, bool POSE, bool COPIES>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void field_kernel(FieldArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FieldSmem<BF, BWD>& sm = *reinterpret_cast<FieldSmem<BF, BWD>*>(smem_raw);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;

  if constexpr (BF) {
    // two entries (8 loads) per thread and pass, loaded before either is stored
    for (int e0 = tid; e0 < (T_END / 4) * 64; e0 += 2 * kBlock) {
      float v[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = e0 + u * kBlock, slot = e >> 6, l = e & 63;
#pragma unroll
        for (int c = 0; c < 4; ++c) v[u][c] = e < (T_END / 4) * 64 ? table_value(A.mlp, 4 * slot + c, l) : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int e = e0 + u * kBlock;
        if (e < (T_END / 4) * 64) sm.tabbf[e] = make_uint2(f2bf2(v[u][0], v[u][1]), f2bf2(v[u][2], v[u][3]));
      }
    }
  } else {
    fill_batched<kBlock>(sm.tab, T_END * 64, tid, [&](int e) { return table_value(A.mlp, e >> 6, e & 63); });
  }
  if (tid < 32) {
    sm.bias[tid] = A.mlp[oB1 + tid];
    sm.bias[32 + tid] = A.mlp[oB2 + tid];
    sm.bias[80 + tid] = A.mlp[oC1 + tid];
    sm.w3row0[tid] = A.mlp[oW3 + tid];
  }
  if (tid < 16) {
    sm.bias[64 + tid] = A.mlp[oB3 + tid];
    sm.bias[112 + tid] = tid < 3 ? A.mlp[oC2 + tid] : 0.f;
  }
  float* scrA = BWD ? sm.scr[wave] : nullptr;
  float* scrB = BWD ? sm.scr[wave] + 32 * RSR : nullptr;
  const ScatterStage stage{scrA, BWD ? sm.dst[wave] : nullptr};
  // this lane's grid level (q) in registers; po >= 0 if the level is accumulated in LDS
  const LevelConst lc = level_const(A.g, q);
  const int po = ((uniform_i(A.priv_mask) >> q) & 1) ? pick_level(A.priv_off, q) : -1;
  const int cpb = COPIES ? pick_level(A.copy_base, q) : -1;
  float* priv = reinterpret_cast<float*>(smem_raw + smem_bytes<BF, BWD>());
  if (BWD)
    for (int e = tid; e < A.priv_floats; e += kBlock) priv[e] = 0.f;
  __syncthreads();

  // the device sample count never exceeds the capacity the workspace and the
  // forward outputs were sized for
  const int total = A.seg_end ? min(*A.seg_end, A.total) : A.total;
  const int n_pair_tiles = (A.S + 7) / 8;
  const int n_tiles = n_pair_tiles + (total + 15) / 16;

  // accumulators of the decoder gradients (backward), in MFMA accumulator layout:
  // aW1 [32 x 16], aW2 [32 x 32], aW3 [16 x 32], aU1 [32 x 16 o-index; column 0
  // holds c1]; aS [16 x 16] gathers the small ones by column: 0-1 b1, 2-3 b2,
  // 4 b3, 5 c2, 6-7 the Eikonal part of W3 row 0, 10-15 U2 (column 10 + 3b + c
  // holds U2[c][16b + row]).
  v4f aW1[2], aW2[4], aW3[2], aU1[2], aS;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    aW1[b] = aW3[b] = aU1[b] = v4f{0, 0, 0, 0};
    aW2[b] = aW2[b + 2] = v4f{0, 0, 0, 0};
  }
  aS = v4f{0, 0, 0, 0};
  float smooth_acc = 0.f;

  for (int tile = blockIdx.x * kWavesPerBlock + wave; tile < n_tiles; tile += gridDim.x * kWavesPerBlock) {
    if (tile < n_pair_tiles)
      field_tile<1, BWD, BF, POSE, COPIES>(A, sm, tile, total, lane, q, j, lc, po, cpb, scrA, scrB, stage, priv, aW1, aW2, aW3,
                                   aU1, aS, smooth_acc);
    else
      field_tile<0, BWD, BF, POSE, COPIES>(A, sm, tile - n_pair_tiles, total, lane, q, j, lc, po, cpb, scrA, scrB, stage, priv,
                                   aW1, aW2, aW3, aU1, aS, smooth_acc);
  }

  if constexpr (!BWD) {
    if (A.S > 0) {
      // block partial of the smoothness sum (fixed order: lanes, then waves)
      float v = wave_sum(smooth_acc);
      __syncthreads();
      float* red = reinterpret_cast<float*>(smem_raw);
      if (lane == 0) red[wave] = v;
      __syncthreads();
      if (tid == 0) {
        float s = 0.f;
        for (int w = 0; w < kWavesPerBlock; ++w) s += red[w];
        A.smooth_partial[blockIdx.x] = s;
      }
    }
    return;
  }

  // ---------------- block partial of the privatised levels' gradients
  __syncthreads();
  if (A.priv_floats > 0) {
    float* dst = A.priv_partial + (size_t)blockIdx.x * A.priv_floats;
    for (int e = tid; e < A.priv_floats; e += kBlock) dst[e] = priv[e];
  }
  // ---------------- block partial of the decoder gradients (deterministic)
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem_raw) + wave * kMlpNumel;
  for (int e = lane; e < kMlpNumel; e += 64) red[e] = 0.f;
  wave_lds_fence();
#pragma unroll
  for (int ba = 0; ba < 2; ++ba)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * ba + 4 * q + r;
      red[oW1 + row * 16 + j] = aW1[ba][r];
      red[oW2 + row * 32 + j] = aW2[ba * 2 + 0][r];
      red[oW2 + row * 32 + 16 + j] = aW2[ba * 2 + 1][r];
      if (j >= 1) red[oU1 + row * 15 + j - 1] = aU1[ba][r];
      else red[oC1 + row] = aU1[ba][r];
    }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = 4 * q + r;
    red[oW3 + row * 32 + j] = aW3[0][r];
    red[oW3 + row * 32 + 16 + j] = aW3[1][r];
  }
  wave_lds_fence();
  // the columns of aS (lane j holds column j, rows 4q..4q+3)
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 4 * q + r;
    const float v = aS[r];
    if (j < 2) red[oB1 + 16 * j + i] = v;
    else if (j < 4) red[oB2 + 16 * (j - 2) + i] = v;
    else if (j == 4) red[oB3 + i] = v;
    else if (j == 5) { if (i < 3) red[oC2 + i] = v; }
    else if (j < 8) red[oW3 + 16 * (j - 6) + i] += v;
    else if (j >= 10) {
      const int b = (j - 10) / 3, c = (j - 10) % 3;
      red[oU2 + c * 32 + 16 * b + i] = v;
    }
  }
  __syncthreads();
  const float* red0 = reinterpret_cast<const float*>(smem_raw);
  float* out = A.mlp_partial + (size_t)blockIdx.x * kMlpNumel;
  for (int e = tid; e < kMlpNumel; e += kBlock) {
    float s = 0.f;
    for (int w = 0; w < kWavesPerBlock; ++w) s += red0[w * kMlpNumel + e];
    out[e] = s;
  }
}


// sum of the block partials of the privatised levels into the grid gradient
// (one writer per entry, fixed block order)
struct PrivMap {
  int mask;
  int po[4], pc[4];
  long long go[4];
};

__global__ __launch_bounds__(256) void priv_stage2_kernel(const float* __restrict__ tmp, int floats, PrivMap pm,
                                                          float* __restrict__ grad) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= floats) return;
  float s = 0.f;
#pragma unroll 8
  for (int y = 0; y < 64; ++y) s += tmp[(size_t)y * floats + e];
  for (int l = 0; l < 4; ++l)
    if (((pm.mask >> l) & 1) && e >= pm.po[l] && e < pm.po[l] + pm.pc[l]) grad[pm.go[l] * 4 + (e - pm.po[l])] += s;
}

hipError_t launch_colsum_stage1(const float* part, int rows, int cols, float* tmp, hipStream_t st);
int colsum_rows();

hipError_t launch_priv_reduce(const FieldArgs& a, int n_part, const int counts[4], float* tmp, hipStream_t st) {
  if (a.priv_floats <= 0) return hipSuccess;
  if (colsum_rows() != 64) return hipErrorInvalidValue;
  PrivMap pm;
  pm.mask = a.priv_mask;
  for (int l = 0; l < 4; ++l) {
    pm.po[l] = a.priv_off[l];
    pm.pc[l] = counts[l];
    pm.go[l] = a.g.off[l];
  }
  hipError_t e = launch_colsum_stage1(a.priv_partial, n_part, a.priv_floats, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(priv_stage2_kernel, dim3((a.priv_floats + 255) / 256), dim3(256), 0, st, tmp, a.priv_floats,
                     pm, a.grad_grid);
  return hipGetLastError();
}

void plan_privatised_levels(FieldArgs& a, int counts[4]) {
  a.priv_mask = 0;
  a.priv_floats = 0;
  for (int l = 0; l < 4; ++l) {
    const long long nv = (long long)a.g.nx[l] * a.g.ny[l] * a.g.nz[l];
    counts[l] = 0;
    a.priv_off[l] = 0;
    if (a.priv_floats + 4 * nv <= kPrivMaxFloats) {
      a.priv_mask |= 1 << l;
      a.priv_off[l] = a.priv_floats;
      counts[l] = (int)(4 * nv);
      a.priv_floats += (int)(4 * nv);
    }
  }
}

int priv_max_floats() { return kPrivMaxFloats; }

// Copy layout of one level with (nx, ny, nz) vertices: four copies (px, py),
// each [nz][my][mx][dy][dx][feature] with mx = nx / 2 + 1, my = ny / 2 + 1;
// vertex (x, y, z) sits in copy (px, py) at pair (x - px) / 2, (y - py) / 2
// with dx = (x - px) & 1, dy = (y - py) & 1 (for x >= px, y >= py).
static long long copy_level_floats(int nx, int ny, int nz) {
  return 4LL * nz * ((nx >> 1) + 1) * ((ny >> 1) + 1) * 16;
}

// Gradient copies for every level not accumulated in LDS (call after
// plan_privatised_levels).  Returns the floats of all copies, or -1 where a
// level is too large for the packed cell index or the 32-bit offsets.
long long plan_copies(FieldArgs& a) {
  long long n = 0;
  for (int l = 0; l < 4; ++l) {
    a.copy_base[l] = -1;
    if ((a.priv_mask >> l) & 1) continue;
    if (a.g.nx[l] > 2048 || a.g.ny[l] > 2048 || a.g.nz[l] > 512) return -1;
    a.copy_base[l] = (int)n;
    n += copy_level_floats(a.g.nx[l], a.g.ny[l], a.g.nz[l]);
    if (n >= (1LL << 31) - 64) return -1;
  }
  return n;
}

// grad[level] += the level's four copies (one thread per vertex, fixed order).
// A block covers 64 x 4 vertices of one z-slice: a 64-byte unit holds two
// rows of the copy, so the rows that share units are read by one block (one
// XCD's L2) instead of by blocks that the dispatcher spreads over the XCDs.
__global__ __launch_bounds__(256) void copy_fold_kernel(const float* __restrict__ copies, int base, int nx, int ny,
                                                        int nz, long long off, float* __restrict__ grad) {
  const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y, z = blockIdx.z;
  if (x >= nx || y >= ny) return;
  const int mx = (nx >> 1) + 1, my = (ny >> 1) + 1, plane = mx * my * 16, csize = nz * plane;
  float4* gp = reinterpret_cast<float4*>(grad) + off + ((long long)z * ny + y) * nx + x;
  float4 acc = *gp;
#pragma unroll
  for (int py = 0; py < 2; ++py)
#pragma unroll
    for (int px = 0; px < 2; ++px) {
      if (x < px || y < py) continue;
      const int ux = x - px, uy = y - py;
      const float4 c = *reinterpret_cast<const float4*>(copies + base + (px + 2 * py) * csize + z * plane +
                                                        ((uy >> 1) * mx + (ux >> 1)) * 16 + (uy & 1) * 8 +
                                                        (ux & 1) * 4);
      acc.x += c.x; acc.y += c.y; acc.z += c.z; acc.w += c.w;
    }
  *gp = acc;
}

hipError_t launch_copy_fold(const FieldArgs& a, hipStream_t st) {
  for (int l = 0; l < 4; ++l) {
    if (a.copy_base[l] < 0) continue;
    hipLaunchKernelGGL(copy_fold_kernel, dim3((unsigned)((a.g.nx[l] + 63) / 64), (unsigned)((a.g.ny[l] + 3) / 4),
                                              a.g.nz[l]),
                       dim3(64, 4), 0, st, a.copies, a.copy_base[l], a.g.nx[l], a.g.ny[l], a.g.nz[l],
                       (long long)a.g.off[l], a.grad_grid);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <bool BWD, bool BF>
static size_t field_smem(const FieldArgs& a) {
  return (size_t)smem_bytes<BF, BWD>() + (BWD ? (size_t)a.priv_floats * sizeof(float) : 0);
}

// Blocks that are resident at once on the current device for this kernel and
// LDS size (CUs x blocks per CU), queried once per (device, kernel, LDS size).
template <bool BWD, bool BF, bool POSE, bool COPIES>
static int resident_blocks(size_t smem) {
  struct Entry { int dev; size_t smem; int blocks; };
  thread_local Entry cache[8];
  thread_local int n_cached = 0;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  for (int i = 0; i < n_cached; ++i)
    if (cache[i].dev == dev && cache[i].smem == smem) return cache[i].blocks;
  const void* fn = reinterpret_cast<const void*>(&field_kernel<BWD, BF, POSE, COPIES>);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return 0;
  int cus = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, smem) != hipSuccess) return 0;
  const int blocks = cus * (per_cu > 0 ? per_cu : 1);
  if (n_cached < 8) cache[n_cached++] = Entry{dev, smem, blocks};
  return blocks;
}

// Grid of a field launch over `total` ray samples (16 per tile) and `S` pairs
// (8 per tile): one block per 4 tiles, at most one resident round (the tile
// loop covers the rest; a partial second round leaves the machine half
// empty), and at most the workspace's partial rows.  0 on a HIP error.
int field_grid(const FieldArgs& a, bool bwd) {
  const bool bf = a.grid_bf16 != nullptr;
  const int tiles = (a.total + 15) / 16 + (a.S + 7) / 8;
  int blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  int resident;
  const bool pose = bwd && a.grad_x != nullptr, copies = bwd && a.copies != nullptr;
  if (!bwd) resident = bf ? resident_blocks<false, true, false, false>(field_smem<false, true>(a))
                          : resident_blocks<false, false, false, false>(field_smem<false, false>(a));
  else if (bf) resident = pose ? (copies ? resident_blocks<true, true, true, true>(field_smem<true, true>(a))
                                         : resident_blocks<true, true, true, false>(field_smem<true, true>(a)))
                               : (copies ? resident_blocks<true, true, false, true>(field_smem<true, true>(a))
                                         : resident_blocks<true, true, false, false>(field_smem<true, true>(a)));
  else resident = pose ? (copies ? resident_blocks<true, false, true, true>(field_smem<true, false>(a))
                                 : resident_blocks<true, false, true, false>(field_smem<true, false>(a)))
                       : (copies ? resident_blocks<true, false, false, true>(field_smem<true, false>(a))
                                 : resident_blocks<true, false, false, false>(field_smem<true, false>(a)));
  if (resident <= 0) return 0;
  const int cap = bwd ? kFieldMaxBlocksBwd : kFieldMaxBlocksFwd;
  if (blocks > resident) blocks = resident;
  if (blocks > cap) blocks = cap;
  return blocks < 1 ? 1 : blocks;
}

template <bool BWD, bool BF, bool POSE, bool COPIES>
static hipError_t launch_field_t(const FieldArgs& a, int blocks, hipStream_t st) {
  const size_t smem = field_smem<BWD, BF>(a);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&field_kernel<BWD, BF, POSE, COPIES>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((field_kernel<BWD, BF, POSE, COPIES>), dim3(blocks), dim3(kBlock), smem, st, a);
  return hipGetLastError();
}

template <bool BF>
static hipError_t launch_field_bwd(const FieldArgs& a, int blocks, hipStream_t st) {
  const bool pose = a.grad_x != nullptr, copies = a.copies != nullptr;
  if (pose) return copies ? launch_field_t<true, BF, true, true>(a, blocks, st)
                          : launch_field_t<true, BF, true, false>(a, blocks, st);
  return copies ? launch_field_t<true, BF, false, true>(a, blocks, st)
                : launch_field_t<true, BF, false, false>(a, blocks, st);
}

hipError_t launch_field(const FieldArgs& a, bool bwd, int blocks, hipStream_t st) {
  const bool bf = a.grid_bf16 != nullptr;
  if (bwd) return bf ? launch_field_bwd<true>(a, blocks, st) : launch_field_bwd<false>(a, blocks, st);
  return bf ? launch_field_t<false, true, false, false>(a, blocks, st)
            : launch_field_t<false, false, false, false>(a, blocks, st);
}

}  // namespace gs
