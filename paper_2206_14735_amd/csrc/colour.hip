// The paper's colour path (Sec. 3.1, Eq. COLOR_MLP): colour decoded from a
// 6-channel colour grid at the finest level and the viewing direction by a
// decoder with two hidden layers of 32, (6 + 3) -> 32 -> 32 -> 3.  Colour
// does not depend on the geometry features on this path, so it runs as a
// kernel of its own beside the geometry field kernel: the forward writes the
// colour of every sample, the backward takes the samples' colour seeds,
// scatters into the colour grid and sums the decoder's weight gradients.
//
// Work decomposition as in the field kernels: a wave-tile is 16 samples,
// lane (q, j) serves sample j; lane group q gathers corners 2q and 2q + 1
// of the sample's finest cell, and the four partial feature vectors are
// summed across the groups.  The decoder input (16 rows: 6 features, the
// unit view direction, zeros) sits in the B-operand layout of the 16x16x4
// MFMA; weights are pre-arranged per lane in LDS.
#include "args.h"
#include "gather.h"
#include "mfma.h"

namespace gs {

// One step of the segmented sum inside a 16-lane group: lanes of the same run
// add the partial of the lane D to their right (a multiply by 0 or 1, folded
// into one v_fmac_f32 with a DPP source; the values are finite).
template <int CTRL, int D>
__device__ __forceinline__ void merge_step(float (&val)[12], int segid, int j) {
  const int so = dpp_i<CTRL>(segid);
  const float take = (j + D < 16) && so == segid ? 1.f : 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) val[c] = fmaf(dpp_f<CTRL>(val[c]), take, val[c]);
}

// packed V1[32][9] e1[32] V2[32][32] e2[32] V3[3][32] e3[3]
constexpr int oV1 = 0, oE1 = 288, oV2 = 320, oE2 = 1344, oV3 = 1376, oE3 = 1472, kColourNumel = 1475;
static_assert(kColourNumel == GOSURF_COLOUR_MLP_NUMEL, "colour decoder layout");

// A-operand slots (64 floats each): base + out_block * 4 * in_blocks + step
enum : int {
  CV1 = 0,     // V1    out 32, in 16 (9 used)
  CV2 = 8,     // V2    out 32, in 32
  CV3 = 24,    // V3    out 16 (3 used), in 32
  CV3T = 32,   // V3^T  out 32, in 16 (3 used)
  CV2T = 40,   // V2^T  out 32, in 32
  CV1T = 56,   // V1^T  out 16 (9 used), in 32
  CV_END = 64
};

__device__ float colour_table_value(const float* __restrict__ P, int slot, int l) {
  int tb, nbi;
  if (slot < CV2) { tb = CV1; nbi = 1; }
  else if (slot < CV3) { tb = CV2; nbi = 2; }
  else if (slot < CV3T) { tb = CV3; nbi = 2; }
  else if (slot < CV2T) { tb = CV3T; nbi = 1; }
  else if (slot < CV1T) { tb = CV2T; nbi = 2; }
  else { tb = CV1T; nbi = 2; }
  const int rel = slot - tb;
  const int bo = rel / (4 * nbi), s = rel % (4 * nbi);
  const int i = 16 * bo + (l & 15);                       // output row
  const int k = 16 * (s >> 2) + 4 * (l >> 4) + (s & 3);   // input row
  switch (tb) {
    case CV1: return k < 9 ? P[oV1 + i * 9 + k] : 0.f;
    case CV2: return P[oV2 + i * 32 + k];
    case CV3: return i < 3 ? P[oV3 + i * 32 + k] : 0.f;
    case CV3T: return k < 3 ? P[oV3 + k * 32 + i] : 0.f;
    case CV2T: return P[oV2 + k * 32 + i];
    default: return i < 9 ? P[oV1 + k * 9 + i] : 0.f;
  }
}

struct ColourSmem {
  float tab[CV_END * 64];
  float bias[32 + 32 + 16];         // e1, e2, e3 (padded to 16)
};
constexpr int kColourScrFloats = 2048;   // per wave: operand transposes (backward)
constexpr int kColourMaxBlocks = 2048;   // rows of the weight-gradient partials

template <bool BWD>
__device__ __forceinline__ void colour_tile(const ColourArgs& A, const ColourSmem& sm, int tile, int total,
                                            const LevelConst& lc, int lane, int q, int j, float* scrA, float* scrB,
                                            v4f (&aV1)[2], v4f (&aV2)[4], v4f (&aV3)[2], v4f& aS) {
  const int item = tile * 16 + j;
  const bool live = item < total;
  float px = 0.f, py = 0.f, pz = 0.f, rx = 0.f, ry = 0.f, rz = 1.f;
  float4 sd = make_float4(0.f, 0.f, 0.f, 0.f);
  if (live) {
    const int ray = A.ray_of[item];
    rx = A.r[3 * ray + 0]; ry = A.r[3 * ray + 1]; rz = A.r[3 * ray + 2];
    if constexpr (BWD) {
      const float4 p4 = *reinterpret_cast<const float4*>(A.posw + 4 * (size_t)item);
      sd = *reinterpret_cast<const float4*>(A.seed4 + 4 * (size_t)item);
      px = p4.x; py = p4.y; pz = p4.z;
    } else {
      const float tt = A.t[item];
      px = mad_norm(tt, rx, A.o[3 * ray + 0]);
      py = mad_norm(tt, ry, A.o[3 * ray + 1]);
      pz = mad_norm(tt, rz, A.o[3 * ray + 2]);
    }
  }
  const bool valid = live && inside_box(A.g, px, py, pz);
  LevelSample ls;
  locate(A.g, lc, px, py, pz, ls);
  const long long row0 = ls.row - lc.off;        // colour-grid row of corner 000
  // this lane group's two corners
  float cf[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  float wc[2] = {0.f, 0.f};
  long long crow[2] = {0, 0};
#pragma unroll
  for (int cc = 0; cc < 2; ++cc) {
    const int c = 2 * q + cc;
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const float wx = bx ? ls.f[0] : 1.f - ls.f[0], wy = by ? ls.f[1] : 1.f - ls.f[1],
                wz = bz ? ls.f[2] : 1.f - ls.f[2];
    wc[cc] = valid ? wx * wy * wz : 0.f;
    crow[cc] = row0 + bx + (long long)by * ls.sy + (long long)bz * ls.sz;
    if (valid) {
      const float4 lo = *reinterpret_cast<const float4*>(A.cgrid + 8 * crow[cc]);
      const float2 hi = *reinterpret_cast<const float2*>(A.cgrid + 8 * crow[cc] + 4);
      cf[0] += wc[cc] * lo.x; cf[1] += wc[cc] * lo.y; cf[2] += wc[cc] * lo.z; cf[3] += wc[cc] * lo.w;
      cf[4] += wc[cc] * hi.x; cf[5] += wc[cc] * hi.y;
    }
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    cf[k] += __shfl_xor(cf[k], 16, 64);
    cf[k] += __shfl_xor(cf[k], 32, 64);
  }
  const float rn = sqrtf(rx * rx + ry * ry + rz * rz);
  const float d0 = rx / rn, d1 = ry / rn, d2 = rz / rn;
  v4f in0 = v4f{0.f, 0.f, 0.f, 0.f};
  if (valid) {
    if (q == 0) in0 = v4f{cf[0], cf[1], cf[2], cf[3]};
    else if (q == 1) in0 = v4f{cf[4], cf[5], d0, d1};
    else if (q == 2) in0 = v4f{d2, 0.f, 0.f, 0.f};
  }
  v4f h1[2], h2[2], ob;
  layer_f32<2, 1>(sm.tab, CV1, &in0, h1, lane);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) h1[b][r] = fmaxf(h1[b][r] + sm.bias[16 * b + 4 * q + r], 0.f);
  layer_f32<2, 2>(sm.tab, CV2, h1, h2, lane);
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[b][r] = fmaxf(h2[b][r] + sm.bias[32 + 16 * b + 4 * q + r], 0.f);
  layer_f32<1, 2>(sm.tab, CV3, h2, &ob, lane);
  v4f cb;
#pragma unroll
  for (int r = 0; r < 4; ++r) cb[r] = sigmoidf_(ob[r] + sm.bias[64 + 4 * q + r]);

  if constexpr (!BWD) {
    if (q == 0 && live) {
      float* o4 = A.out4 + 4 * (size_t)item;
      o4[1] = cb[0]; o4[2] = cb[1]; o4[3] = cb[2];
    }
  } else {
    // dL/d(pre-sigmoid) of the three channels (rows 0..2, lane group 0)
    v4f dc = v4f{0.f, 0.f, 0.f, 0.f};
    if (q == 0 && valid) {
      dc[0] = sd.y * cb[0] * (1.f - cb[0]);
      dc[1] = sd.z * cb[1] * (1.f - cb[1]);
      dc[2] = sd.w * cb[2] * (1.f - cb[2]);
    }
    v4f dh2[2], dh1[2], din;
    layer_f32<2, 1>(sm.tab, CV3T, &dc, dh2, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dh2[b][r] = h2[b][r] > 0.f ? dh2[b][r] : 0.f;
    layer_f32<2, 2>(sm.tab, CV2T, dh2, dh1, lane);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) dh1[b][r] = h1[b][r] > 0.f ? dh1[b][r] : 0.f;
    layer_f32<1, 2>(sm.tab, CV1T, dh1, &din, lane);

    // weight gradients: sums over the tile's samples (the MFMA K axis)
    float4 tX[2], tY[2];
    rows_to_lanes<1>(scrA, &dc, tX, q, j);
    rows_to_lanes<2>(scrB, h2, tY, q, j);
    outer_lanes<false, 1, 2>(tX, tY, aV3);
    colsum_into(tX[0], 4, aS, j);
    rows_to_lanes<2>(scrA, dh2, tX, q, j);
    rows_to_lanes<2>(scrB, h1, tY, q, j);
    outer_lanes<false, 2, 2>(tX, tY, aV2);
    colsum_into(tX[0], 2, aS, j);
    colsum_into(tX[1], 3, aS, j);
    rows_to_lanes<2>(scrA, dh1, tX, q, j);
    rows_to_lanes<1>(scrB, &in0, tY, q, j);
    outer_lanes<false, 2, 1>(tX, tY, aV1);
    colsum_into(tX[0], 0, aS, j);
    colsum_into(tX[1], 1, aS, j);

    // dL/d(colour features): rows 0..3 in lane group 0, rows 4..5 in group 1
    float g[6];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = __shfl(din[k], j, 64);
    g[4] = __shfl(din[0], 16 + j, 64);
    g[5] = __shfl(din[1], 16 + j, 64);
    // Consecutive samples of a ray often share the finest cell: a segmented
    // sum over the 16 lanes of the group (DPP row shifts) merges each run of
    // equal cells into its first lane, which alone writes its two corners.
    float val[12];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
      for (int k = 0; k < 6; ++k) val[6 * cc + k] = valid ? wc[cc] * g[k] : 0.f;
    const int key = valid ? (int)row0 : -1 - j;   // an invalid lane is a run of its own
    const bool head = (j == 0) || key != dpp_i<kRowShr1>(key);
    const unsigned grp = (unsigned)(__ballot(head) >> (16 * q)) & 0xffffu;
    const int segid = __popc(grp & ((2u << j) - 1u));
    merge_step<kRowShl1, 1>(val, segid, j);
    merge_step<kRowShl2, 2>(val, segid, j);
    merge_step<kRowShl4, 4>(val, segid, j);
    merge_step<kRowShl8, 8>(val, segid, j);
    // The writers stage their two corners by rank in the wave's scratch (8
    // floats per corner, 6 used), then 8 lanes write one corner: the 6
    // features of a vertex lie in one aligned 32-byte row, so each corner is
    // one request of an atomic instruction instead of six.
    const bool writer = head && valid;
    const unsigned long long wm = __ballot(writer);
    const int nw = __popcll(wm);
    int* dsti = reinterpret_cast<int*>(scrA + 1024);   // [128] rows, after the [128][8] values
    wave_lds_fence();   // the transposes' reads of the scratch are complete
    if (writer) {
      const int rank = __popcll(wm & ((1ull << lane) - 1ull));
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
        for (int k = 0; k < 6; ++k) scrA[16 * rank + 8 * cc + k] = val[6 * cc + k];
        dsti[2 * rank + cc] = (int)crow[cc];
      }
    }
    wave_lds_fence();
    const int jobs = 2 * nw, f = lane & 7;
    for (int base = 0; base < jobs; base += 8) {
      const int k = base + (lane >> 3);
      wait_vmem_at_most<1>();   // as in the field kernel's scatter: a bounded number in flight
      if (k < jobs && f < 6) atomic_add_global(A.grad_cgrid + 8 * (long long)dsti[k] + f, scrA[8 * k + f]);
    }
    wave_lds_fence();   // the next tile reuses the scratch
  }
}

template <bool BWD>
__global__ __launch_bounds__(256) void colour_kernel(ColourArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  ColourSmem& sm = *reinterpret_cast<ColourSmem*>(smem_raw);
  float* scr = reinterpret_cast<float*>(smem_raw + sizeof(ColourSmem));
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;
  fill_batched<256>(sm.tab, CV_END * 64, tid, [&](int e) { return colour_table_value(A.cmlp, e >> 6, e & 63); });
  if (tid < 32) {
    sm.bias[tid] = A.cmlp[oE1 + tid];
    sm.bias[32 + tid] = A.cmlp[oE2 + tid];
  }
  if (tid < 16) sm.bias[64 + tid] = tid < 3 ? A.cmlp[oE3 + tid] : 0.f;
  __syncthreads();
  const int total = A.seg_end ? min(*A.seg_end, A.total) : A.total;
  const int n_tiles = (total + 15) / 16;
  const LevelConst lc = level_const(A.g, GOSURF_LEVELS - 1);
  float* scrA = BWD ? scr + wave * kColourScrFloats : nullptr;
  float* scrB = BWD ? scrA + 32 * RSR : nullptr;
  v4f aV1[2], aV2[4], aV3[2], aS;
#pragma unroll
  for (int b = 0; b < 2; ++b) aV1[b] = aV3[b] = aV2[b] = aV2[b + 2] = v4f{0.f, 0.f, 0.f, 0.f};
  aS = v4f{0.f, 0.f, 0.f, 0.f};
  for (int tile = blockIdx.x * 4 + wave; tile < n_tiles; tile += gridDim.x * 4)
    colour_tile<BWD>(A, sm, tile, total, lc, lane, q, j, scrA, scrB, aV1, aV2, aV3, aS);
  if constexpr (BWD) {
    // block partial of the decoder gradients (fixed order: waves in LDS, then summed)
    __syncthreads();
    float* red = reinterpret_cast<float*>(smem_raw) + wave * kColourNumel;
    for (int e = lane; e < kColourNumel; e += 64) red[e] = 0.f;
    wave_lds_fence();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int ba = 0; ba < 2; ++ba) {
        const int row = 16 * ba + 4 * q + r;
        if (j < 9) red[oV1 + row * 9 + j] = aV1[ba][r];
        red[oV2 + row * 32 + j] = aV2[2 * ba][r];
        red[oV2 + row * 32 + 16 + j] = aV2[2 * ba + 1][r];
      }
      const int i = 4 * q + r;
      if (i < 3) {
        red[oV3 + i * 32 + j] = aV3[0][r];
        red[oV3 + i * 32 + 16 + j] = aV3[1][r];
      }
      const float v = aS[r];
      if (j < 2) red[oE1 + 16 * j + i] = v;
      else if (j < 4) red[oE2 + 16 * (j - 2) + i] = v;
      else if (j == 4 && i < 3) red[oE3 + i] = v;
    }
    __syncthreads();
    const float* red0 = reinterpret_cast<const float*>(smem_raw);
    float* out = A.partial + (size_t)blockIdx.x * kColourNumel;
    for (int e = tid; e < kColourNumel; e += 256) {
      float s = 0.f;
      for (int w = 0; w < 4; ++w) s += red0[w * kColourNumel + e];
      out[e] = s;
    }
  }
}

template <bool BWD>
static size_t colour_smem() {
  const size_t a = sizeof(ColourSmem) + (BWD ? sizeof(float) * 4 * kColourScrFloats : 0);
  const size_t red = BWD ? sizeof(float) * 4 * kColourNumel : 0;
  return a > red ? a : red;
}

// blocks of a colour launch: one per 4 tiles, at most the resident count and
// the partial rows; 0 on a HIP error
int colour_grid_blocks(int total, bool bwd) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const void* fn = bwd ? reinterpret_cast<const void*>(&colour_kernel<true>)
                       : reinterpret_cast<const void*>(&colour_kernel<false>);
  const size_t smem = bwd ? colour_smem<true>() : colour_smem<false>();
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, smem) != hipSuccess) return 0;
  int blocks = ((total + 15) / 16 + 3) / 4;
  const int resident = cus * (per_cu > 0 ? per_cu : 1);
  if (blocks > resident) blocks = resident;
  if (blocks > kColourMaxBlocks) blocks = kColourMaxBlocks;
  return blocks < 1 ? 1 : blocks;
}

hipError_t launch_colour(const ColourArgs& a, bool bwd, int blocks, hipStream_t st) {
  if (bwd) {
    hipLaunchKernelGGL(colour_kernel<true>, dim3(blocks), dim3(256), colour_smem<true>(), st, a);
  } else {
    hipLaunchKernelGGL(colour_kernel<false>, dim3(blocks), dim3(256), colour_smem<false>(), st, a);
  }
  return hipGetLastError();
}

int colour_numel() { return kColourNumel; }

}  // namespace gs
