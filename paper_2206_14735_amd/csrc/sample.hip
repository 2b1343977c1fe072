// Ray batch and smoothness-point sampling on the device.
//
// Thread m < M builds ray m: Philox picks a pixel of any frame, the pixel is
// back-projected through the pinhole, and its samples are generated in order
// by merging the stratified list over the span with the stratified list
// around the observed depth.  Threads M .. M+S-1 build the smoothness pairs.
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

__global__ __launch_bounds__(256) void sample_kernel(SampleArgs A) {
  const int gid = blockIdx.x * 256 + threadIdx.x;
  const unsigned long long thw = (unsigned long long)A.T * A.H * A.W;
  if (gid < A.M) {
    const int m = gid;
    const U4 w0 = philox((uint32_t)m, A.step, 0u, 0u, A.k0, A.k1);
    const unsigned long long pix = pick_pixel(w0.x, thw);
    const PixelRay pr = pixel_ray(A, pix);
    const float D = A.depth[pix];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      A.o[3 * m + a] = pr.o[a];
      A.r[3 * m + a] = pr.r[a];
      A.rgb_out[3 * m + a] = (float)A.rgb[3 * pix + a] / 255.f;
    }
    A.depth_out[m] = D;
    if (A.pixel) A.pixel[m] = (long long)pix;
    float tn = A.near_t, tf = A.far_t;
    if (A.span_mode == GOSURF_SPAN_BOX) {
      float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float ta = (A.g.p0[a] - pr.o[a]) / pr.r[a];
        const float tb = (A.g.p1[a] - pr.o[a]) / pr.r[a];
        tmin = fmaxf(tmin, fminf(ta, tb));   // NaN (0/0) is ignored by fmin/fmax
        tmax = fminf(tmax, fmaxf(ta, tb));
      }
      tn = fmaxf(tmin, A.near_t);
      tf = fmaxf(fminf(tmax, A.far_t), tn);
    }
    const int n_tot = A.n_strat + A.n_near;
    const size_t base = (size_t)m * n_tot;
    UniformStream us{(uint32_t)m, A.step, 1u, A.k0, A.k1, -1, {}};
    UniformStream un{(uint32_t)m, A.step, 2u, A.k0, A.k1, -1, {}};
    if (D > 0.f && A.n_near > 0) {
      const float ds = (tf - tn) / (float)A.n_strat;
      const float lo = D - A.trunc, dn = (2.f * A.trunc) / (float)A.n_near;
      int i = 0, jn = 0;
      float a = tn + ((float)0 + us.get(0)) * ds;
      float b = lo + ((float)0 + un.get(0)) * dn;
      for (int k = 0; k < n_tot; ++k) {
        const bool take_a = jn >= A.n_near || (i < A.n_strat && a <= b);
        if (take_a) {
          A.t[base + k] = a;
          ++i;
          if (i < A.n_strat) a = tn + ((float)i + us.get(i)) * ds;
        } else {
          A.t[base + k] = b;
          ++jn;
          if (jn < A.n_near) b = lo + ((float)jn + un.get(jn)) * dn;
        }
        A.ray_of[base + k] = m;
      }
    } else {
      const float ds = (tf - tn) / (float)n_tot;
      for (int k = 0; k < n_tot; ++k) {
        A.t[base + k] = tn + ((float)k + us.get(k)) * ds;
        A.ray_of[base + k] = m;
      }
    }
    A.seg[m] = (int)base;
    if (m == A.M - 1) A.seg[A.M] = (int)((size_t)A.M * n_tot);
  } else if (gid < A.M + A.S) {
    const int p = gid - A.M;
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
}

hipError_t launch_sample(const SampleArgs& a, hipStream_t st) {
  const int n = a.M + a.S;
  hipLaunchKernelGGL(sample_kernel, dim3((n + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
