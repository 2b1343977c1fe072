// Ray batch and smoothness-point sampling on the device.
//
// Ray m is built by one wave: Philox picks a pixel of any frame, the pixel is
// back-projected through the pinhole, and its samples are the stratified list
// over the span merged in order with the stratified list around the observed
// depth.  Smoothness pairs are built one per thread.
#include "args.h"

namespace gs {


struct PixelRay {
  float o[3], r[3];
};

__device__ __forceinline__ PixelRay pixel_ray(const SampleArgs& A, unsigned long long pix) {
  const unsigned long long hw = (unsigned long long)A.H * A.W;
  const int f = (int)(pix / hw);
  const int rem = (int)(pix - (unsigned long long)f * hw);
  const int v = rem / A.W, u = rem - v * A.W;
  const float* M = A.c2w + 16 * (size_t)f;
  const float dx = ((float)u + 0.5f - A.cx) / A.fx;
  const float dy = ((float)v + 0.5f - A.cy) / A.fy;
  PixelRay pr;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    pr.r[a] = M[4 * a + 0] * dx + M[4 * a + 1] * dy + M[4 * a + 2];
    pr.o[a] = M[4 * a + 3];
  }
  return pr;
}

__device__ __forceinline__ unsigned long long pick_pixel(uint32_t x, unsigned long long thw) {
  return ((unsigned long long)x * thw) >> 32;
}

// uniform number i of stream `stream` for index `idx`, caching one Philox block
struct UniformStream {
  uint32_t idx, step, stream, k0, k1;
  int block;
  U4 words;
  __device__ float get(int i) {
    const int b = i >> 2;
    if (b != block) {
      words = philox(idx, step, stream, (uint32_t)b, k0, k1);
      block = b;
    }
    const int w = i & 3;
    const uint32_t x = w == 0 ? words.x : (w == 1 ? words.y : (w == 2 ? words.z : words.w));
    return u01(x);
  }
};

// One wave per ray.  Every sample value is computed by one lane; its place
// in the merged order is its index in its own list plus the number of values
// of the other list that precede it (stratified first on ties), counted on the
// same float32 values by every lane, so the ranks form a permutation.
// RAY: pick the pixel and write the ray; GEN: write the ray's samples (with a
// proposal, confident rays get n_prop stratified samples in [near, far] and
// their first sample comes from the precomputed seg).
template <bool RAY, bool GEN>
__global__ __launch_bounds__(256) void sample_rays_kernel(SampleArgs A) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= A.M) return;
  float o[3], r[3], D;
  if (RAY) {
    const unsigned long long thw = (unsigned long long)A.T * A.H * A.W;
    const U4 w0 = philox((uint32_t)m, A.step, 0u, 0u, A.k0, A.k1);
    const unsigned long long pix = pick_pixel(w0.x, thw);
    const PixelRay pr = pixel_ray(A, pix);
    D = A.depth[pix];
#pragma unroll
    for (int a = 0; a < 3; ++a) { o[a] = pr.o[a]; r[a] = pr.r[a]; }
    if (lane < 3) {
      A.o[3 * m + lane] = pr.o[lane];
      A.r[3 * m + lane] = pr.r[lane];
      A.rgb_out[3 * m + lane] = (float)A.rgb[3 * pix + lane] / 255.f;
    }
    if (lane == 0) {
      A.depth_out[m] = D;
      if (A.pixel) A.pixel[m] = (long long)pix;
    }
  } else {
#pragma unroll
    for (int a = 0; a < 3; ++a) { o[a] = A.o[3 * m + a]; r[a] = A.r[3 * m + a]; }
    D = A.depth_out[m];
  }
  if (!GEN) return;
  float tn, tf;
  ray_span(A.g, o, r, A.span_mode, A.near_t, A.far_t, tn, tf);
  const int n_tot = A.n_strat + A.n_near;
  const bool proposed = A.prop3 != nullptr && A.prop3[3 * m + 2] >= A.conf_thr;
  const bool two = !proposed && D > 0.f && A.n_near > 0;
  // list a (stratified stream): the span, or a confident ray's interval;
  // list b (near-depth stream): around the observed depth, or a confident
  // ray's free space [t_lo, near] before its interval
  const int ns = proposed ? A.n_prop : (two ? A.n_strat : n_tot);
  const int nn = proposed ? A.n_free : (two ? A.n_near : 0);
  float lo = D - A.trunc, dn = (2.f * A.trunc) / (float)(nn > 0 ? nn : 1);
  if (proposed) {
    const float pn = A.prop3[3 * m], pf = A.prop3[3 * m + 1];
    lo = tn;
    dn = (pn - tn) / (float)(nn > 0 ? nn : 1);
    tn = pn;
    tf = pf;
  }
  const float ds = (tf - tn) / (float)ns;
  const size_t base = A.prop3 != nullptr ? (size_t)A.seg[m] : (size_t)m * n_tot;
  float av[kChunks], bv[kChunks];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int i = 64 * c + lane;
    av[c] = bv[c] = 0.f;
    if (i < ns) {
      const U4 w = philox((uint32_t)m, A.step, 1u, (uint32_t)(i >> 2), A.k0, A.k1);
      const uint32_t x = (i & 3) == 0 ? w.x : ((i & 3) == 1 ? w.y : ((i & 3) == 2 ? w.z : w.w));
      av[c] = tn + ((float)i + u01(x)) * ds;
    }
    if (i < nn) {
      const U4 w = philox((uint32_t)m, A.step, 2u, (uint32_t)(i >> 2), A.k0, A.k1);
      const uint32_t x = (i & 3) == 0 ? w.x : ((i & 3) == 1 ? w.y : ((i & 3) == 2 ? w.z : w.w));
      bv[c] = lo + ((float)i + u01(x)) * dn;
    }
  }
  // ranks: stratified value a_i precedes near value b_j iff a_i <= b_j.  Both
  // lists are non-decreasing in float32 (each value is a monotone rounding of
  // an increasing exact value), so a binary search over the other list in LDS
  // gives the same counts as comparing with every value.
  int ra[kChunks], rb[kChunks];
  __shared__ float lists[4][2][kChunks * 64];   // per wave: the ray's two lists
  float* la = lists[threadIdx.x >> 6][0];
  float* lb = lists[threadIdx.x >> 6][1];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int i = 64 * c + lane;
    if (i < ns) la[i] = av[c];
    if (i < nn) lb[i] = bv[c];
  }
  wave_lds_fence();
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int i = 64 * c + lane;
    ra[c] = rb[c] = i;
    if (i < ns) {   // near values strictly below a_i
      int lo_ = 0, hi_ = nn;
      while (lo_ < hi_) {
        const int mid = (lo_ + hi_) >> 1;
        if (lb[mid] < av[c]) lo_ = mid + 1;
        else hi_ = mid;
      }
      ra[c] += lo_;
    }
    if (i < nn) {   // stratified values at or below b_j
      int lo_ = 0, hi_ = ns;
      while (lo_ < hi_) {
        const int mid = (lo_ + hi_) >> 1;
        if (la[mid] <= bv[c]) lo_ = mid + 1;
        else hi_ = mid;
      }
      rb[c] += lo_;
    }
  }
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    const int i = 64 * c + lane;
    if (i < ns) A.t[base + ra[c]] = av[c];
    if (i < nn) A.t[base + rb[c]] = bv[c];
    if (i < ns + nn) A.ray_of[base + i] = m;
  }
  if (lane == 0 && A.prop3 == nullptr) {
    A.seg[m] = (int)base;
    if (m == A.M - 1) A.seg[A.M] = (int)((size_t)A.M * n_tot);
  }
}

// Rays only (proposal mode, before the proposal runs): one thread per ray picks
// the pixel and writes the ray, its colour and depth, exactly as the
// wave-per-ray kernel does.
__global__ __launch_bounds__(256) void sample_pixels_kernel(SampleArgs A) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= A.M) return;
  const unsigned long long thw = (unsigned long long)A.T * A.H * A.W;
  const U4 w0 = philox((uint32_t)m, A.step, 0u, 0u, A.k0, A.k1);
  const unsigned long long pix = pick_pixel(w0.x, thw);
  const PixelRay pr = pixel_ray(A, pix);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    A.o[3 * m + a] = pr.o[a];
    A.r[3 * m + a] = pr.r[a];
    A.rgb_out[3 * m + a] = (float)A.rgb[3 * pix + a] / 255.f;
  }
  A.depth_out[m] = A.depth[pix];
  if (A.pixel) A.pixel[m] = (long long)pix;
}

// One thread per smoothness pair.
__global__ __launch_bounds__(256) void sample_points_kernel(SampleArgs A) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= A.S) return;
  const unsigned long long thw = (unsigned long long)A.T * A.H * A.W;
  int found = -1;
  U4 wf{};
  unsigned long long pix = 0;
  for (int att = 0; att < 8; ++att) {
    const U4 w = philox((uint32_t)p, A.step, 3u, (uint32_t)att, A.k0, A.k1);
    const unsigned long long c = pick_pixel(w.x, thw);
    if (A.depth[c] > 0.f) { found = att; wf = w; pix = c; break; }
  }
  if (found < 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      A.xs[3 * p + a] = 0.5f * (A.g.p0[a] + A.g.p1[a]);
      A.eps[3 * p + a] = 0.f;
    }
    return;
  }
  const PixelRay pr = pixel_ray(A, pix);
  const float d = A.depth[pix] + (2.f * u01(wf.y) - 1.f) * A.trunc;
  const float zc = 1.f - 2.f * u01(wf.z);
  const float ph = 6.283185307179586f * u01(wf.w);
  const float rr = sqrtf(fmaxf(0.f, 1.f - zc * zc));
  float sn, cs;
  sincosf(ph, &sn, &cs);
  const float e[3] = {rr * cs, rr * sn, zc};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    A.xs[3 * p + a] = pr.o[a] + d * pr.r[a];
    A.eps[3 * p + a] = A.delta_s * e[a];
  }
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((sample_rays_kernel<true, true>), dim3((a.M + 3) / 4), dim3(256), 0, st, a);
  if (a.S > 0) hipLaunchKernelGGL(sample_points_kernel, dim3((a.S + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

// proposal mode: rays first, then (after inference and the seg scan) samples
hipError_t launch_sample_rays_only(const SampleArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(sample_pixels_kernel, dim3((a.M + 255) / 256), dim3(256), 0, st, a);
  if (a.S > 0) hipLaunchKernelGGL(sample_points_kernel, dim3((a.S + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_sample_gen_only(const SampleArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((sample_rays_kernel<false, true>), dim3((a.M + 3) / 4), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
