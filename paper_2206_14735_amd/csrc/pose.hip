// Camera pose refinement (Sec. 3 and 3.5; the implementation details give a
// pose as a translation and an so(3) rotation): the refined camera-to-world
// poses, the per-ray gradients of the loss with respect to ray origin and
// direction (from the per-sample dL/dx of the backward field kernel), and the
// per-frame pose gradient.
#include "args.h"

namespace gs {

// sin(t)/t, (1 - cos t)/t^2 and (t - sin t)/t^3 of t = |nu|; below t = 0.1
// by their Taylor series to t^6 (whose remainder is then below 1e-13), where
// the closed forms would lose digits to cancellation in float32
__device__ __forceinline__ void so3_coefficients(float t2, float& a, float& b, float& c) {
  if (t2 < 1e-2f) {
    a = 1.f - t2 * (1.f / 6.f - t2 * (1.f / 120.f - t2 * (1.f / 5040.f)));
    b = 0.5f - t2 * (1.f / 24.f - t2 * (1.f / 720.f - t2 * (1.f / 40320.f)));
    c = (1.f / 6.f) - t2 * (1.f / 120.f - t2 * (1.f / 5040.f - t2 * (1.f / 362880.f)));
  } else {
    const float t = sqrtf(t2);
    const float s = sinf(t), co = cosf(t);
    a = s / t;
    b = (1.f - co) / t2;
    c = (t - s) / (t2 * t);
  }
}

// K = [nu]_x; out = I + p K + q K^2
__device__ __forceinline__ void so3_poly(const float nu[3], float p, float q, float out[3][3]) {
  const float K[3][3] = {{0.f, -nu[2], nu[1]}, {nu[2], 0.f, -nu[0]}, {-nu[1], nu[0], 0.f}};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float k2 = 0.f;
#pragma unroll
      for (int l = 0; l < 3; ++l) k2 += K[i][l] * K[l][j];
      out[i][j] = (i == j ? 1.f : 0.f) + p * K[i][j] + q * k2;
    }
}

// c2w[t] = [Exp(nu_t) R0_t | c0_t + tau_t; 0 0 0 1], pose[t] = (tau, nu)
__global__ __launch_bounds__(256) void pose_apply_kernel(const float* __restrict__ c2w0,
                                                         const float* __restrict__ pose, int T,
                                                         float* __restrict__ c2w) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= T) return;
  const float* P0 = c2w0 + 16 * (size_t)t;
  const float* p = pose + 6 * (size_t)t;
  const float nu[3] = {p[3], p[4], p[5]};
  float a, b, c;
  so3_coefficients(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2], a, b, c);
  float E[3][3];
  so3_poly(nu, a, b, E);
  float* out = c2w + 16 * (size_t)t;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) out[4 * i + j] = E[i][0] * P0[j] + E[i][1] * P0[4 + j] + E[i][2] * P0[8 + j];
    out[4 * i + 3] = P0[4 * i + 3] + p[i];
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) out[12 + j] = P0[12 + j];
}

// Per ray: dL/do = sum_i dL/dx_i and dL/dr = sum_i t_i dL/dx_i over its
// samples (x_i = o + t_i r); ADDED to grad_o, grad_r.  One wave per ray.
__global__ __launch_bounds__(256) void ray_xgrad_kernel(const float* __restrict__ dx, const float* __restrict__ t,
                                                        const int* __restrict__ seg, int M, int total,
                                                        float* __restrict__ grad_o, float* __restrict__ grad_r) {
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (m >= M) return;
  const int s0 = min(max(seg[m], 0), total);
  const int n = max(min(seg[m + 1], total) - s0, 0);
  float go[3] = {0.f, 0.f, 0.f}, gr[3] = {0.f, 0.f, 0.f};
  for (int k = lane; k < n; k += 64) {
    const float4 d = *reinterpret_cast<const float4*>(dx + 4 * (size_t)(s0 + k));
    const float tt = t[s0 + k];
    go[0] += d.x; go[1] += d.y; go[2] += d.z;
    gr[0] += tt * d.x; gr[1] += tt * d.y; gr[2] += tt * d.z;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    go[a] = wave_sum_dpp(go[a]);
    gr[a] = wave_sum_dpp(gr[a]);
  }
  if (lane == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      grad_o[3 * (size_t)m + a] += go[a];
      grad_r[3 * (size_t)m + a] += gr[a];
    }
  }
}

// Per ray of frame f = pixel / HW: grad_pose[f][0..2] += dL/do and
// grad_pose[f][3..5] += J_l(nu_f)^T (r x dL/dr).  Rays whose pixel index
// names no frame of [0, T) are skipped.
__global__ __launch_bounds__(256) void pose_grad_kernel(const float* __restrict__ pose, int T,
                                                        const long long* __restrict__ pixel, long long HW,
                                                        const float* __restrict__ r, const float* __restrict__ grad_o,
                                                        const float* __restrict__ grad_r, int M,
                                                        float* __restrict__ grad_pose) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= M) return;
  const long long px = pixel[m];
  if (px < 0) return;
  const long long f = px / HW;
  if (f >= T) return;
  const float* p = pose + 6 * f;
  const float nu[3] = {p[3], p[4], p[5]};
  float a, b, c;
  so3_coefficients(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2], a, b, c);
  float J[3][3];
  so3_poly(nu, b, c, J);
  const float rr[3] = {r[3 * (size_t)m], r[3 * (size_t)m + 1], r[3 * (size_t)m + 2]};
  const float g[3] = {grad_r[3 * (size_t)m], grad_r[3 * (size_t)m + 1], grad_r[3 * (size_t)m + 2]};
  const float cr[3] = {rr[1] * g[2] - rr[2] * g[1], rr[2] * g[0] - rr[0] * g[2], rr[0] * g[1] - rr[1] * g[0]};
  float* out = grad_pose + 6 * f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    atomic_add_global(out + i, grad_o[3 * (size_t)m + i]);
    atomic_add_global(out + 3 + i, J[0][i] * cr[0] + J[1][i] * cr[1] + J[2][i] * cr[2]);
  }
}

hipError_t launch_pose_apply(const float* c2w0, const float* pose, int T, float* c2w, hipStream_t st) {
  hipLaunchKernelGGL(pose_apply_kernel, dim3((T + 255) / 256), dim3(256), 0, st, c2w0, pose, T, c2w);
  return hipGetLastError();
}

hipError_t launch_ray_xgrad(const float* dx, const float* t, const int* seg, int M, int total, float* grad_o,
                            float* grad_r, hipStream_t st) {
  hipLaunchKernelGGL(ray_xgrad_kernel, dim3((M + 3) / 4), dim3(256), 0, st, dx, t, seg, M, total, grad_o, grad_r);
  return hipGetLastError();
}

hipError_t launch_pose_grad(const float* pose, int T, const long long* pixel, long long HW, const float* r,
                            const float* grad_o, const float* grad_r, int M, float* grad_pose, hipStream_t st) {
  hipLaunchKernelGGL(pose_grad_kernel, dim3((M + 255) / 256), dim3(256), 0, st, pose, T, pixel, HW, r, grad_o,
                     grad_r, M, grad_pose);
  return hipGetLastError();
}

}  // namespace gs
