// Learned proposal sampler: inference, training (forward + loss + backward
// with MFMA weight gradients) and training targets from logged weights.
//
// Wave tile = 16 rays; lane (q, j) serves ray j and gathers the level-1
// features of bin centres q and 4 + q, so the 38 inputs (padded to 48) land
// in MFMA B layout: block 0 rows 4q..4q+3 = point q, block 1 = point 4 + q,
// block 2 rows 32..37 = ray origin and direction.  The 38-64-64-3 network
// runs on 16x16x4 fp32 MFMA with activations chained in accumulator layout.
#include "args.h"
#include "gather.h"
#include "mfma.h"

namespace gs {

// packed proposal parameters: P1[64][38] q1[64] P2[64][64] q2[64] P3[3][64] q3[3]
constexpr int pP1 = 0, pQ1 = 2432, pP2 = 2496, pQ2 = 6592, pP3 = 6656, pQ3 = 6848, kPropNumel = 6851;
static_assert(kPropNumel == GOSURF_PROPOSAL_NUMEL, "proposal layout");
constexpr int kPropLevel = 1;     // grid level whose features feed the network
constexpr int kPropPoints = 8;

enum : int {
  PT_1 = 0,     // P1     out 64 (4 blk), in 48 (3 blk; rows >= 38 are 0)
  PT_2 = 48,    // P2     out 64, in 64
  PT_3 = 112,   // P3     out 16 (rows 0..2), in 64
  PT_3T = 128,  // P3^T   out 64, in 16 (rows 0..2)
  PT_2T = 144,  // P2^T   out 64, in 64
  PT_END = 208
};

__device__ float prop_table_value(const float* __restrict__ P, int slot, int l) {
  int tb, nbi;
  if (slot < PT_2) { tb = PT_1; nbi = 3; }
  else if (slot < PT_3) { tb = PT_2; nbi = 4; }
  else if (slot < PT_3T) { tb = PT_3; nbi = 4; }
  else if (slot < PT_2T) { tb = PT_3T; nbi = 1; }
  else { tb = PT_2T; nbi = 4; }
  const int rel = slot - tb;
  const int bo = rel / (4 * nbi), s = rel % (4 * nbi);
  const int i = 16 * bo + (l & 15);
  const int k = 16 * (s >> 2) + 4 * (l >> 4) + (s & 3);
  switch (tb) {
    case PT_1: return k < 38 ? P[pP1 + i * 38 + k] : 0.f;
    case PT_2: return P[pP2 + i * 64 + k];
    case PT_3: return i < 3 ? P[pP3 + i * 64 + k] : 0.f;
    case PT_3T: return k < 3 ? P[pP3 + k * 64 + i] : 0.f;
    default: return P[pP2 + k * 64 + i];
  }
}

// only the training form transposes operands through the per-wave scratch
template <bool TRAIN>
struct PropSmem {
  float tab[PT_END * 64];
  float bias[64 + 64 + 16];
  float scr[kWavesPerBlock][TRAIN ? 2 * 64 * RSR : 1];
};
template <bool TRAIN>
constexpr size_t prop_smem_bytes() {
  return (TRAIN && sizeof(PropSmem<TRAIN>) < (kPropNumel + 1) * sizeof(float)) ? (kPropNumel + 1) * sizeof(float)
                                                                               : sizeof(PropSmem<TRAIN>);
}

__device__ __forceinline__ float smooth_l1_grad(float x, float beta) {
  return fabsf(x) < beta ? x / beta : (x > 0.f ? 1.f : -1.f);
}
__device__ __forceinline__ float smooth_l1(float x, float beta) {
  const float a = fabsf(x);
  return a < beta ? 0.5f * x * x / beta : a - 0.5f * beta;
}

// TRAIN = false: near/far/confidence per ray; TRAIN = true: additionally the
// loss and the gradient of the mean loss w.r.t. the proposal parameters
// (block partials, reduced in a fixed order afterwards).
template <bool TRAIN>
__global__ __launch_bounds__(kBlock) void proposal_kernel(PropArgs A) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  PropSmem<TRAIN>& sm = *reinterpret_cast<PropSmem<TRAIN>*>(smem_raw);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63, q = lane >> 4, j = lane & 15;
  fill_batched<kBlock>(sm.tab, PT_END * 64, tid, [&](int e) { return prop_table_value(A.prop, e >> 6, e & 63); });
  if (tid < 64) {
    sm.bias[tid] = A.prop[pQ1 + tid];
    sm.bias[64 + tid] = A.prop[pQ2 + tid];
  }
  if (tid < 16) sm.bias[128 + tid] = tid < 3 ? A.prop[pQ3 + tid] : 0.f;
  __syncthreads();
  float* scrA = TRAIN ? sm.scr[wave] : nullptr;
  float* scrB = TRAIN ? sm.scr[wave] + 64 * RSR : nullptr;

  v4f aP1[12], aP2[16], aP3[4], gq1[4], gq2[4], gq3;
  if (TRAIN) {
#pragma unroll
    for (int b = 0; b < 16; ++b) aP2[b] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 12; ++b) aP1[b] = v4f{0, 0, 0, 0};
#pragma unroll
    for (int b = 0; b < 4; ++b) aP3[b] = gq1[b] = gq2[b] = v4f{0, 0, 0, 0};
    gq3 = v4f{0, 0, 0, 0};
  }
  float loss_acc = 0.f;
  const float invM = 1.f / (float)A.M;
  const int n_tiles = (A.M + 15) / 16;
  const LevelConst lc = level_const(A.g, kPropLevel);

  for (int tile = blockIdx.x * kWavesPerBlock + wave; tile < n_tiles; tile += gridDim.x * kWavesPerBlock) {
    const int m = tile * 16 + j;
    const bool live = m < A.M;
    float o[3] = {0.f, 0.f, 0.f}, r[3] = {0.f, 0.f, 1.f};
    if (live) {
#pragma unroll
      for (int a = 0; a < 3; ++a) { o[a] = A.o[3 * m + a]; r[a] = A.r[3 * m + a]; }
    }
    float tn, tf;
    ray_span(A.g, o, r, A.span_mode, A.near_t, A.far_t, tn, tf);
    const float dt = (tf - tn) / (float)kPropPoints;
    v4f in[3];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int b = q + 4 * h;
      const float tb = tn + ((float)b + 0.5f) * dt;
      const float px = mad_norm(tb, r[0], o[0]), py = mad_norm(tb, r[1], o[1]), pz = mad_norm(tb, r[2], o[2]);
      const bool ok = live && inside_box(A.g, px, py, pz);
      LevelSample ls;
      locate(A.g, lc, px, py, pz, ls);
      float z[4], G[4][3];
      interp<false, false>(A.grid, nullptr, ls, ok, z, G);
      in[h] = v4f{z[0], z[1], z[2], z[3]};
    }
    in[2] = v4f{0.f, 0.f, 0.f, 0.f};
    if (live && q == 0) in[2] = v4f{o[0], o[1], o[2], r[0]};
    if (live && q == 1) in[2] = v4f{r[1], r[2], 0.f, 0.f};

    v4f h1[4], h2[4], ob;
    layer_f32<4, 3>(sm.tab, PT_1, in, h1, lane);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) h1[b][rr] = fmaxf(h1[b][rr] + sm.bias[16 * b + 4 * q + rr], 0.f);
    layer_f32<4, 4>(sm.tab, PT_2, h1, h2, lane);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) h2[b][rr] = fmaxf(h2[b][rr] + sm.bias[64 + 16 * b + 4 * q + rr], 0.f);
    layer_f32<1, 4>(sm.tab, PT_3, h2, &ob, lane);
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) ob[rr] += sm.bias[128 + 4 * q + rr];

    // interval and confidence (outputs 0..2 live in lane group 0)
    const float s0 = sigmoidf_(ob[0]), s1 = sigmoidf_(ob[1]), s2 = sigmoidf_(ob[2]);
    const float near = tn + (tf - tn) * s0;
    const float far = near + (tf - near) * s1;
    if (q == 0 && live && A.out3) {
      A.out3[3 * m + 0] = near;
      A.out3[3 * m + 1] = far;
      A.out3[3 * m + 2] = s2;
    }
    if (!TRAIN) continue;

    v4f dob = v4f{0, 0, 0, 0};
    if (q == 0 && live) {
      const float c = A.tgt[3 * m + 2];
      const float en = near - A.tgt[3 * m + 0], ef = far - A.tgt[3 * m + 1];
      // confidence label: a ray with a logged surface whose interval covers the target
      const bool cov = near <= A.tgt[3 * m + 0] + A.cover_tol && far >= A.tgt[3 * m + 1] - A.cover_tol;
      const float k = (c > 0.5f && cov) ? 1.f : 0.f;
      const float x = ob[2];
      const float bce = fmaxf(x, 0.f) - k * x + log1pf(__expf(-fabsf(x)));
      loss_acc += (c * (smooth_l1(en, A.beta) + smooth_l1(ef, A.beta)) + bce) * invM;
      const float g_far = c * smooth_l1_grad(ef, A.beta);
      const float g_near = c * smooth_l1_grad(en, A.beta) + g_far * (1.f - s1);
      dob[0] = g_near * (tf - tn) * s0 * (1.f - s0) * invM;
      dob[1] = g_far * (tf - near) * s1 * (1.f - s1) * invM;
      dob[2] = (s2 - k) * invM;
    }
    v4f dh2[4], dh1[4];
    layer_f32<4, 1>(sm.tab, PT_3T, &dob, dh2, lane);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) dh2[b][rr] = h2[b][rr] > 0.f ? dh2[b][rr] : 0.f;
    layer_f32<4, 4>(sm.tab, PT_2T, dh2, dh1, lane);
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) dh1[b][rr] = h1[b][rr] > 0.f ? dh1[b][rr] : 0.f;
    outer_acc<false, 1, 4>(scrA, scrB, &dob, h2, aP3, q, j);
    outer_acc<false, 4, 4>(scrA, scrB, dh2, h1, aP2, q, j);
    outer_acc<false, 4, 3>(scrA, scrB, dh1, in, aP1, q, j);
#pragma unroll
    for (int b = 0; b < 4; ++b) { gq1[b] += dh1[b]; gq2[b] += dh2[b]; }
    gq3 += dob;
  }
  if (!TRAIN) return;

  // ---------------- block partials (waves add in turn: fixed order)
  __syncthreads();
  float* red = reinterpret_cast<float*>(smem_raw);
  for (int e = tid; e < kPropNumel + 1; e += kBlock) red[e] = 0.f;
  const float ls_w = wave_sum(loss_acc);
  for (int w = 0; w < kWavesPerBlock; ++w) {
    __syncthreads();
    if (wave != w) continue;
#pragma unroll
    for (int bo = 0; bo < 4; ++bo)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 16 * bo + 4 * q + rr;
#pragma unroll
        for (int bi = 0; bi < 3; ++bi) {
          const int col = 16 * bi + j;
          if (col < 38) red[pP1 + row * 38 + col] += aP1[bo * 3 + bi][rr];
        }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) red[pP2 + row * 64 + 16 * bi + j] += aP2[bo * 4 + bi][rr];
      }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int row = 4 * q + rr;
      if (row < 3)
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) red[pP3 + row * 64 + 16 * bi + j] += aP3[bi][rr];
    }
    wave_lds_fence();
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 16 * b + 4 * q + rr;
        float v1 = gq1[b][rr], v2 = gq2[b][rr];
        v1 += __shfl_xor(v1, 1, 64); v1 += __shfl_xor(v1, 2, 64); v1 += __shfl_xor(v1, 4, 64); v1 += __shfl_xor(v1, 8, 64);
        v2 += __shfl_xor(v2, 1, 64); v2 += __shfl_xor(v2, 2, 64); v2 += __shfl_xor(v2, 4, 64); v2 += __shfl_xor(v2, 8, 64);
        if (j == 0) { red[pQ1 + row] += v1; red[pQ2 + row] += v2; }
      }
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      float v3 = gq3[rr];
      v3 += __shfl_xor(v3, 1, 64); v3 += __shfl_xor(v3, 2, 64); v3 += __shfl_xor(v3, 4, 64); v3 += __shfl_xor(v3, 8, 64);
      const int row = 4 * q + rr;
      if (j == 0 && row < 3) red[pQ3 + row] += v3;
    }
    if (lane == 0) red[kPropNumel] += ls_w;
    wave_lds_fence();
  }
  __syncthreads();
  float* out = A.grad_partial + (size_t)blockIdx.x * (kPropNumel + 1);
  for (int e = tid; e < kPropNumel + 1; e += kBlock) out[e] = red[e];
}

// ---------------------------------------------------------------- targets from logged weights
// One wave per ray: normalised weights, their inclusive prefix sum (the CDF
// through (t_i, C_i) starting from (t_0, 0)), first crossings of the two
// quantile levels with linear interpolation, widening and clipping to the span.
__global__ __launch_bounds__(256) void proposal_targets_kernel(TargetArgs A) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= A.M) return;
  const int s0 = A.seg[m], n = A.seg[m + 1] - s0;
  float o[3], r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) { o[a] = A.o[3 * m + a]; r[a] = A.r[3 * m + a]; }
  float tn, tf;
  ray_span(A.g, o, r, A.span_mode, A.near_t, A.far_t, tn, tf);
  float w[kChunks], t[kChunks];
  float tot = 0.f;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int k = 64 * c + lane;
    w[c] = k < n ? A.w[s0 + k] : 0.f;
    t[c] = k < n ? A.t[s0 + k] : 0.f;
    tot += w[c];
  }
  tot = wave_sum(tot);
  if (tot <= 0.f) {
    if (lane == 0) { A.tgt[3 * m] = tn; A.tgt[3 * m + 1] = tf; A.tgt[3 * m + 2] = 0.f; }
    return;
  }
  // inclusive prefix sums of p_i = w_i / tot
  float cdf[kChunks];
  float carry = 0.f;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    float v = w[c] / tot;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float u = __shfl_up(v, d, 64);
      if (lane >= d) v += u;
    }
    cdf[c] = carry + v;
    carry = __shfl(cdf[c], 63, 64);
  }
  float qv[2];
  const float levels[2] = {A.q_lo, A.q_hi};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    int first = -1;
#pragma unroll
    for (int c = kChunks - 1; c >= 0; --c) {
      const int k = 64 * c + lane;
      const unsigned long long bm = __ballot(k < n && cdf[c] >= levels[h]);
      if (bm) first = 64 * c + __ffsll((long long)bm) - 1;
    }
    if (first < 0) first = n - 1;
    // values at `first` and `first - 1`
    const int cf = first >> 6, lf = first & 63;
    float tf_ = 0.f, cf_ = 0.f, tp = 0.f, cp = 0.f;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const float tt = __shfl(t[c], lf, 64), cc = __shfl(cdf[c], lf, 64);
      if (c == cf) { tf_ = tt; cf_ = cc; }
    }
    const int pidx = first - 1 < 0 ? 0 : first - 1;
    const int cpc = pidx >> 6, lp = pidx & 63;
#pragma unroll
    for (int c = 0; c < kChunks; ++c) {
      const float tt = __shfl(t[c], lp, 64), cc = __shfl(cdf[c], lp, 64);
      if (c == cpc) { tp = tt; cp = cc; }
    }
    float val;
    if (first == 0) val = tf_;
    else if (cf_ <= cp) val = tf_;
    else val = tp + (levels[h] - cp) / (cf_ - cp) * (tf_ - tp);
    qv[h] = val;
  }
  if (lane == 0) {
    const float a = fminf(fmaxf(qv[0] - A.widen, tn), tf);
    const float b = fminf(fmaxf(qv[1] + A.widen, a), tf);
    A.tgt[3 * m] = a;
    A.tgt[3 * m + 1] = b;
    A.tgt[3 * m + 2] = tot >= A.conf_min ? 1.f : 0.f;
  }
}

// samples per ray from the confidences, and their exclusive prefix sum (one block)
// Segment offsets of the proposal-driven batch: ray m gets n_prop samples if
// its confidence reaches thr, else n_plain.  With depth_check, a confident ray
// with an observed depth D > 0 outside [near, far] gets its interval extended
// to D in prop3 if D lies within `extend` of it, and is rejected otherwise: its
// confidence is negated in prop3 (thr > 0), which the sample generator reads.
// With edge > 0 (and depth_check) a confident ray whose pixel has a
// 4-neighbour in its frame with valid depth differing from D by more than
// edge is rejected the same way: at a depth discontinuity the interval
// around D would leave the grazed surface in front of it unsampled.
// Block b scans rays [8192 b, 8192 (b + 1)): lengths are read
// coalesced into LDS, each thread sums 8 consecutive rays, the 1024 partial
// sums are scanned in LDS and the chunk-local offsets written out coalesced
// with the chunk total in block_total[b]; a second pass adds the totals of
// the preceding chunks.
constexpr int kSegChunk = 8192;

// true if a 4-neighbour of pixel p (frame-major index into [T][H][W]) has a
// valid depth (> 0) that differs from D by more than ec.edge
__device__ __forceinline__ bool at_depth_edge(const EdgeCheck& ec, long long p, float D) {
  const long long hw = (long long)ec.H * ec.W;
  const long long f = p / hw;
  const int rem = (int)(p - f * hw), y = rem / ec.W, x = rem - (rem / ec.W) * ec.W;
  const float* img = ec.depth + f * hw;
  const int nx[4] = {x - 1, x + 1, x, x}, ny[4] = {y, y, y - 1, y + 1};
  bool edge = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (nx[i] < 0 || nx[i] >= ec.W || ny[i] < 0 || ny[i] >= ec.H) continue;
    const float Dn = img[(long long)ny[i] * ec.W + nx[i]];
    if (Dn > 0.f && fabsf(Dn - D) > ec.edge) edge = true;
  }
  return edge;
}
__global__ __launch_bounds__(1024) void proposal_seg_local_kernel(float* __restrict__ prop3,
                                                                  const float* __restrict__ depth, int depth_check,
                                                                  float extend, EdgeCheck ec, int M, float thr,
                                                                  int n_prop, int n_plain, int* __restrict__ seg,
                                                                  int* __restrict__ block_total) {
  __shared__ int len[kSegChunk];
  __shared__ int part[1024];
  const int tid = threadIdx.x;
  constexpr int per = kSegChunk / 1024;
  const int c0 = blockIdx.x * kSegChunk;
  const int n = min(kSegChunk, M - c0);
  for (int m = tid; m < kSegChunk; m += 1024) {
    int l = 0;
    if (m < n) {
      const size_t k = (size_t)(c0 + m);
      const float conf = prop3[3 * k + 2];
      bool acc = conf >= thr;
      if (acc && depth_check && ec.edge > 0.f && depth[k] > 0.f && at_depth_edge(ec, ec.pixel[k], depth[k])) {
        acc = false;
        prop3[3 * k + 2] = -conf;
      }
      if (acc && depth_check) {
        const float D = depth[k], nr = prop3[3 * k], fr = prop3[3 * k + 1];
        if (D > 0.f && !(nr <= D && D <= fr)) {
          if (nr - extend <= D && D <= fr + extend) {
            prop3[3 * k] = fminf(nr, D);
            prop3[3 * k + 1] = fmaxf(fr, D);
          } else {
            acc = false;
            prop3[3 * k + 2] = -conf;
          }
        }
      }
      l = acc ? n_prop : n_plain;
    }
    len[m] = l;
  }
  __syncthreads();
  int s = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) s += len[tid * per + k];
  part[tid] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const int v = tid >= d ? part[tid - d] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  int run = part[tid] - s;   // exclusive prefix of this thread's first ray in the chunk
#pragma unroll
  for (int k = 0; k < per; ++k) {
    const int l = len[tid * per + k];
    len[tid * per + k] = run;
    run += l;
  }
  __syncthreads();
  for (int m = tid; m < n; m += 1024) seg[c0 + m] = len[m];
  if (tid == 0) block_total[blockIdx.x] = part[1023];
}

__global__ __launch_bounds__(1024) void proposal_seg_add_kernel(int M, int* __restrict__ seg,
                                                                const int* __restrict__ block_total) {
  __shared__ int off;
  if (threadIdx.x == 0) {
    int o = 0;
    for (int b = 0; b < (int)blockIdx.x; ++b) o += block_total[b];
    off = o;
    if (blockIdx.x == gridDim.x - 1) seg[M] = o + block_total[blockIdx.x];
  }
  __syncthreads();
  const int c0 = blockIdx.x * kSegChunk;
  const int n = min(kSegChunk, M - c0);
  if (blockIdx.x > 0)
    for (int m = threadIdx.x; m < n; m += 1024) seg[c0 + m] += off;
}

int proposal_blocks(int M) {
  int blocks = ((M + 15) / 16 + kWavesPerBlock - 1) / kWavesPerBlock;
  if (blocks > 512) blocks = 512;
  return blocks < 1 ? 1 : blocks;
}

template <bool TRAIN>
static hipError_t launch_proposal_t(const PropArgs& a, int blocks, hipStream_t st) {
  const size_t smem = prop_smem_bytes<TRAIN>();
  const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&proposal_kernel<TRAIN>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(proposal_kernel<TRAIN>, dim3(blocks), dim3(kBlock), smem, st, a);
  return hipGetLastError();
}

hipError_t launch_proposal(const PropArgs& a, bool train, int blocks, hipStream_t st) {
  return train ? launch_proposal_t<true>(a, blocks, st) : launch_proposal_t<false>(a, blocks, st);
}

hipError_t launch_proposal_targets(const TargetArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(proposal_targets_kernel, dim3((a.M + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

// block_total: scratch of ceil(M / 8192) ints (the batch's ray_of, which the
// sample generator overwrites afterwards)
hipError_t launch_proposal_seg(float* prop3, const float* depth, int depth_check, float extend, const EdgeCheck& ec,
                               int M, float thr, int n_prop, int n_plain, int* seg, int* block_total, hipStream_t st) {
  const int nb = (M + kSegChunk - 1) / kSegChunk;
  hipLaunchKernelGGL(proposal_seg_local_kernel, dim3(nb), dim3(1024), 0, st, prop3, depth, depth_check, extend, ec,
                     M, thr, n_prop, n_plain, seg, block_total);
  hipLaunchKernelGGL(proposal_seg_add_kernel, dim3(nb), dim3(1024), 0, st, M, seg, block_total);
  return hipGetLastError();
}

int proposal_numel() { return kPropNumel; }

}  // namespace gs
