// Hierarchical importance sampling along rays (Sec. 3.2, last paragraph): the
// samples of a ray grow from the coarse set in steps, each drawing n_add new
// depths from the rendering weights (Eqs. volume_rendering and
// volume_rendering_alpha) of the samples it has so far.
//
// importance_step_kernel: one wave per ray.  Opacities and the exclusive
// transmittance product run over 64-sample chunks with a carry; the interval
// probabilities w_i + eps and their running sum (the unnormalised CDF) go to
// LDS; n_add lanes then each draw one stratified uniform and invert the CDF by
// binary search.
// importance_merge_kernel: one wave per ray; every entry finds its place in
// the merged list by counting (binary search in the sorted current list), so
// the merge is stable (current samples first on ties) and needs no sort.
#include "device.h"

#include "args.h"

namespace gs {

constexpr int kImpWaves = 4;

__global__ __launch_bounds__(kImpWaves * 64) void importance_step_kernel(ImpArgs A) {
  __shared__ float cdf_s[kImpWaves][kChunks * 64 + 1];
  __shared__ float pdf_s[kImpWaves][kChunks * 64];
  __shared__ float t_s[kImpWaves][kChunks * 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = blockIdx.x * kImpWaves + wv;
  if (m >= A.M) return;   // whole waves
  float* cdf = cdf_s[wv];
  float* pdf = pdf_s[wv];
  float* ts = t_s[wv];
  const int n = A.n;
  const size_t base = (size_t)m * n;
  const float s = __expf(10.f * A.mlp[oV]);
  const float o[3] = {A.o[3 * m], A.o[3 * m + 1], A.o[3 * m + 2]};
  const float r[3] = {A.r[3 * m], A.r[3 * m + 1], A.r[3 * m + 2]};

  float ph[kChunks];
  int val[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int i = 64 * c + lane;
    ph[c] = 0.f;
    val[c] = 0;
    if (i < n) {
      const float tt = A.t[base + i];
      ts[i] = tt;
      ph[c] = A.phi[(base + i) * A.phi_stride];
      val[c] = inside_box(A.g, mad_norm(tt, r[0], o[0]), mad_norm(tt, r[1], o[1]), mad_norm(tt, r[2], o[2]));
      if (!val[c]) ph[c] = 0.f;
    }
  }
  const int nch = (n + 63) >> 6;
  float carry_t = 1.f, carry_c = 0.f;
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    if (c >= nch) break;
    const int i = 64 * c + lane;
    float nphi = __shfl_down(ph[c], 1, 64);
    int nval = __shfl_down(val[c], 1, 64);
    if (c + 1 < kChunks) {
      const float p0 = __shfl(ph[c + 1], 0, 64);
      const int v0 = __shfl(val[c + 1], 0, 64);
      if (lane == 63) { nphi = p0; nval = v0; }
    } else if (lane == 63) {
      nval = 0;
    }
    float a = 0.f;
    if (val[c] && nval && i + 1 < n && nphi < ph[c]) a = sigmoidf_(-s * nphi) * -expm1f(s * (nphi - ph[c]));
    // exclusive product of (1 - alpha): inclusive scan, shifted by one lane
    float v = 1.f - a;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float u = __shfl_up(v, d, 64);
      if (lane >= d) v *= u;
    }
    float T = __shfl_up(v, 1, 64);
    if (lane == 0) T = 1.f;
    T *= carry_t;
    carry_t *= __shfl(v, 63, 64);
    // interval probability (unnormalised) and its running sum
    const float p = (i + 1 < n) ? T * a + A.eps : 0.f;
    float q = p;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const float u = __shfl_up(q, d, 64);
      if (lane >= d) q += u;
    }
    if (i < n) {
      pdf[i] = p;
      cdf[i + 1] = carry_c + q;
    }
    carry_c += __shfl(q, 63, 64);
  }
  if (lane == 0) cdf[0] = 0.f;
  wave_lds_fence();

  if (lane < A.n_add) {
    const U4 w = philox((uint32_t)m, A.iteration, A.stream, (uint32_t)(lane >> 2), A.k0, A.k1);
    const uint32_t word = (lane & 3) == 0 ? w.x : (lane & 3) == 1 ? w.y : (lane & 3) == 2 ? w.z : w.w;
    const float u = ((float)lane + u01(word)) / (float)A.n_add;
    const float target = u * cdf[n - 1];
    // last interval i in [0, n - 2] whose CDF start is <= target
    int lo = 0, hi = n - 2;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cdf[mid] <= target) lo = mid;
      else hi = mid - 1;
    }
    float frac = pdf[lo] > 0.f ? (target - cdf[lo]) / pdf[lo] : 0.f;
    frac = fminf(fmaxf(frac, 0.f), 1.f);
    const float tn = ts[lo] + frac * (ts[lo + 1] - ts[lo]);
    A.t_new[(size_t)m * A.n_add + lane] = tn;
    if (A.ray_of_new) A.ray_of_new[(size_t)m * A.n_add + lane] = m;
  }
}

__global__ __launch_bounds__(kImpWaves * 64) void importance_merge_kernel(ImpMergeArgs A) {
  __shared__ float ta_s[kImpWaves][kChunks * 64];
  __shared__ float tb_s[kImpWaves][kImpMaxAdd];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = blockIdx.x * kImpWaves + wv;
  if (m >= A.M) return;
  float* ta = ta_s[wv];
  float* tb = tb_s[wv];
  const int na = A.na, nb = A.nb, no = na + nb;
  const size_t ba = (size_t)m * na, bb = (size_t)m * nb, bo = (size_t)m * no;
  for (int i = lane; i < na; i += 64) ta[i] = A.ta[ba + i];
  if (lane < nb) tb[lane] = A.tb[bb + lane];
  wave_lds_fence();
  // current samples: rank = own index + new samples strictly before
  for (int i = lane; i < na; i += 64) {
    const float x = ta[i];
    int cnt = 0;
    for (int j = 0; j < nb; ++j) cnt += tb[j] < x;
    const size_t dst = bo + i + cnt;
    A.t_out[dst] = x;
    if (A.p_out) A.p_out[dst] = A.pa[(ba + i) * A.pa_stride];
    if (A.ray_of_out) A.ray_of_out[dst] = m;
  }
  // new samples: rank among the new ones (by value, then index) + current samples at or before
  if (lane < nb) {
    const float y = tb[lane];
    int own = 0;
    for (int j = 0; j < nb; ++j) own += (tb[j] < y) || (tb[j] == y && j < lane);
    int lo = 0, hi = na;   // first index with ta > y
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ta[mid] <= y) lo = mid + 1;
      else hi = mid;
    }
    const size_t dst = bo + own + lo;
    A.t_out[dst] = y;
    if (A.p_out) A.p_out[dst] = A.pb[(bb + lane) * A.pb_stride];
    if (A.ray_of_out) A.ray_of_out[dst] = m;
  }
  if (A.seg_out && lane == 0) {
    A.seg_out[m] = (int)bo;
    if (m == A.M - 1) A.seg_out[A.M] = (int)(bo + no);
  }
}

hipError_t launch_importance_step(const ImpArgs& a, hipStream_t st) {
  if (a.M < 1 || a.n < 2 || a.n > kChunks * 64 || a.n_add < 1 || a.n_add > kImpMaxAdd) return hipErrorInvalidValue;
  const int blocks = (a.M + kImpWaves - 1) / kImpWaves;
  hipLaunchKernelGGL(importance_step_kernel, dim3(blocks), dim3(kImpWaves * 64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_importance_merge(const ImpMergeArgs& a, hipStream_t st) {
  if (a.M < 1 || a.na < 1 || a.nb < 1 || a.nb > kImpMaxAdd || a.na + a.nb > kChunks * 64) return hipErrorInvalidValue;
  const int blocks = (a.M + kImpWaves - 1) / kImpWaves;
  hipLaunchKernelGGL(importance_merge_kernel, dim3(blocks), dim3(kImpWaves * 64), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
