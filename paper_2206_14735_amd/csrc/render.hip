// Per-ray volume rendering, loss terms and their backward seeds.
//
// One wave owns one ray: lane k holds samples k, k+64, k+128, k+192, so every
// per-sample array is read coalesced; two neighbouring rays of at most 32
// samples share a wave, one half each.  The transmittance is an exclusive
// product scan over the ray and the backward recurrence of the opacities is a
// suffix scan of affine maps, both on DPP row shifts and row broadcasts.
#include "args.h"

namespace gs {



// Cross-lane steps of the per-ray scans, on DPP row shifts and readlane.  A
// ray occupies a segment of W lanes: a whole wave (W = 64), or one half of it
// (W = 32, two rays of at most 32 samples per wave).  sl is the lane's index
// in its segment.

// lane sl reads lane sl + 1 of its segment (the last lane reads 0)
template <int W>
__device__ __forceinline__ float seg_next(float v, int sl) {
  const float x = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));  // wave_shl:1
  return (W == 32 && sl == 31) ? 0.f : x;
}
template <int W>
__device__ __forceinline__ int seg_next_i(int v, int sl) {
  const int x = __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true);
  return (W == 32 && sl == 31) ? 0 : x;
}
// lane sl reads lane sl - 1 of its segment (the first lane reads 0)
template <int W>
__device__ __forceinline__ float seg_prev(float v, int sl) {
  const float x = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));  // wave_shr:1
  return (W == 32 && sl == 0) ? 0.f : x;
}
__device__ __forceinline__ float lane_at(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
// the value of the segment's first / last lane
template <int W>
__device__ __forceinline__ float seg_first(float v, int lane) {
  if constexpr (W == 64) return lane_at(v, 0);
  else return lane < 32 ? lane_at(v, 0) : lane_at(v, 32);
}
template <int W>
__device__ __forceinline__ float seg_last(float v, int lane) {
  if constexpr (W == 64) return lane_at(v, 63);
  else return lane < 32 ? lane_at(v, 31) : lane_at(v, 63);
}

// Inclusive scan over the segment (op: sum or product): inside each row of
// 16 lanes by row shifts (lanes without a source keep their value), then the
// row totals carried on by row broadcasts (lane 15 into row 1 and lane 47
// into row 3; for W = 64, then lane 31 into rows 2 and 3).  Rows that a
// broadcast does not write take the identity.
template <int CTRL, int D, bool PROD>
__device__ __forceinline__ float scan_step(float v, int lane) {
  const float u = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
  if ((lane & 15) < D) return v;
  return PROD ? v * u : v + u;
}
template <int W, bool PROD>
__device__ __forceinline__ float seg_scan(float v, int lane) {
  constexpr float id = PROD ? 1.f : 0.f;
  v = scan_step<0x111, 1, PROD>(v, lane);   // row_shr:1
  v = scan_step<0x112, 2, PROD>(v, lane);   // row_shr:2
  v = scan_step<0x114, 4, PROD>(v, lane);   // row_shr:4
  v = scan_step<0x118, 8, PROD>(v, lane);   // row_shr:8
  const float b15 =
      __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(v), 0x142, 0xA, 0xF, false));
  v = PROD ? v * b15 : v + b15;
  if constexpr (W == 64) {
    const float b31 =
        __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(id), __float_as_int(v), 0x143, 0xC, 0xF, false));
    v = PROD ? v * b31 : v + b31;
  }
  return v;
}
// the segment's sum, in every lane of the segment
template <int W>
__device__ __forceinline__ float seg_sum(float v, int lane) {
  return seg_last<W>(seg_scan<W, false>(v, lane), lane);
}

// Suffix composition of the affine maps x -> b_j + a_j x over lanes j..end
// of the segment: on return lane j holds the maps of lanes j..end composed
// (the map of lane j applied last).  Inside each row by row shifts towards
// lower lanes; the later rows of the segment are composed from their first
// lanes and applied.
template <int CTRL, int D>
__device__ __forceinline__ void affine_step(float& a, float& b, int lane) {
  const float a2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(a), CTRL, 0xF, 0xF, true));
  const float b2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(b), CTRL, 0xF, 0xF, true));
  if ((lane & 15) + D < 16) {
    b = b + a * b2;
    a = a * a2;
  }
}
template <int W>
__device__ __forceinline__ void seg_affine_suffix(float& a, float& b, int lane) {
  affine_step<0x101, 1>(a, b, lane);   // row_shl:1
  affine_step<0x102, 2>(a, b, lane);   // row_shl:2
  affine_step<0x104, 4>(a, b, lane);   // row_shl:4
  affine_step<0x108, 8>(a, b, lane);   // row_shl:8
  const int row = lane >> 4;
  float ca = 1.f, cb = 0.f;   // the maps of the segment's later rows: x -> cb + ca x
  if constexpr (W == 64) {
    const float a1 = lane_at(a, 16), b1 = lane_at(b, 16);
    const float a2 = lane_at(a, 32), b2 = lane_at(b, 32);
    const float a3 = lane_at(a, 48), b3 = lane_at(b, 48);
    if (row < 3) { ca = a3; cb = b3; }
    if (row < 2) { cb = b2 + a2 * cb; ca = a2 * ca; }
    if (row < 1) { cb = b1 + a1 * cb; ca = a1 * ca; }
  } else {
    const float a1 = lane_at(a, 16), b1 = lane_at(b, 16);
    const float a3 = lane_at(a, 48), b3 = lane_at(b, 48);
    if (row == 0) { ca = a1; cb = b1; }
    if (row == 2) { ca = a3; cb = b3; }
  }
  b = b + a * cb;
  a = a * ca;
}

struct RayState {
  int n, s0;
  float s;              // sharpness
  float o[3], r[3];     // ray origin and direction
  float D, I[3];
  float phi[kChunks], tt[kChunks], col[kChunks][3];
  float da[kChunks];    // depth attributed to each sample in d_hat (its t, or the interval midpoint)
  bool valid[kChunks];
  float alpha[kChunks], T[kChunks], w[kChunks];
  float c_hat[3], d_hat, wsum;
};

// Chunks of W samples per ray: 4 of 64 (up to GOSURF_MAX_SAMPLES_PER_RAY
// samples) for a whole wave, 1 of 32 for a half.
template <int W>
constexpr int seg_chunks() { return W == 64 ? kChunks : 1; }

template <int W>
__device__ __forceinline__ void ray_forward(const RenderArgs& A, int m, int lane, RayState& R) {
  constexpr int NC = seg_chunks<W>();
  const int sl = lane & (W - 1);
  // offsets clamped to the batch's capacity (the segment array lives on the
  // device and is not validated by the host)
  R.s0 = min(max(A.seg[m], 0), A.total);
  R.n = max(min(A.seg[m + 1], A.total) - R.s0, 0);
  R.s = __expf(10.f * A.mlp[oV]);
  const float ox = A.o[3 * m], oy = A.o[3 * m + 1], oz = A.o[3 * m + 2];
  const float rx = A.r[3 * m], ry = A.r[3 * m + 1], rz = A.r[3 * m + 2];
  R.o[0] = ox; R.o[1] = oy; R.o[2] = oz;
  R.r[0] = rx; R.r[1] = ry; R.r[2] = rz;
  R.D = A.depth[m];
  R.I[0] = A.rgb[3 * m]; R.I[1] = A.rgb[3 * m + 1]; R.I[2] = A.rgb[3 * m + 2];
#pragma unroll
  for (int c = 0; c < kChunks; ++c) {
    R.valid[c] = false;
    R.phi[c] = 0.f; R.tt[c] = 0.f;
    R.col[c][0] = R.col[c][1] = R.col[c][2] = 0.f;
    R.alpha[c] = R.T[c] = R.w[c] = 0.f;
    R.da[c] = 0.f;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int k = W * c + sl;
    if (k < R.n) {
      const int sidx = R.s0 + k;
      const float tt = A.t[sidx];
      R.tt[c] = tt;
      const float px = mad_norm(tt, rx, ox), py = mad_norm(tt, ry, oy), pz = mad_norm(tt, rz, oz);
      R.valid[c] = inside_box(A.g, px, py, pz);
      if (R.valid[c]) {
        const float4 v = *reinterpret_cast<const float4*>(A.out4 + 4 * (size_t)sidx);
        R.phi[c] = v.x; R.col[c][0] = v.y; R.col[c][1] = v.z; R.col[c][2] = v.w;
      }
    }
  }
  // opacities: alpha_k uses sample k+1 (next lane, or the first lane of the next chunk).
  // 1 - Phi(b)/Phi(a) = Phi(-b) * (1 - e^{-(a - b)}) with a = s phi_k, b = s phi_{k+1}:
  // no difference of nearly equal logarithms, so small opacities keep their
  // relative accuracy.  With W = 64 the chunks past the ray's end are skipped
  // (nch is wave-uniform); with W = 32 there is one chunk.
  const int nch = W == 64 ? (R.n + 63) >> 6 : 1;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R.da[c] = R.tt[c];
    if (c >= nch) continue;
    float nphi = seg_next<W>(R.phi[c], sl);
    float ntt = seg_next<W>(R.tt[c], sl);
    int nval = seg_next_i<W>((int)R.valid[c], sl);
    if (c + 1 < NC && c + 1 < nch) {
      const float p0 = lane_at(R.phi[c + 1], 0);
      const float t0 = lane_at(R.tt[c + 1], 0);
      const int v0 = __builtin_amdgcn_readlane((int)R.valid[c + 1], 0);
      if (lane == 63) { nphi = p0; ntt = t0; nval = v0; }
    }
    const int k = W * c + sl;
    float a = 0.f;
    if (R.valid[c] && nval && k + 1 < R.n && nphi < R.phi[c]) {
      a = sigmoidf_(-R.s * nphi) * -expm1f(R.s * (nphi - R.phi[c]));
      // alpha_k belongs to the interval [t_k, t_k+1]; the midpoint variant
      // attributes its weight to the interval's centre
      if (A.depth_mid) R.da[c] = 0.5f * (R.tt[c] + ntt);
    }
    R.alpha[c] = a;
  }
  // transmittance: exclusive product of (1 - alpha)
  float carry = 1.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    float Tc = 0.f;
    if (c < nch) {
      const float v = seg_scan<W, true>(1.f - R.alpha[c], lane);
      float ex = seg_prev<W>(v, sl);
      if (sl == 0) ex = 1.f;
      Tc = carry * ex;
      if (c + 1 < NC) carry *= lane_at(v, 63);
    }
    R.T[c] = Tc;
    R.w[c] = Tc * R.alpha[c];
  }
  float cr = 0.f, cg = 0.f, cbl = 0.f, dd = 0.f, ws = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    cr += R.w[c] * R.col[c][0];
    cg += R.w[c] * R.col[c][1];
    cbl += R.w[c] * R.col[c][2];
    dd += R.w[c] * R.da[c];
    ws += R.w[c];
  }
  R.c_hat[0] = seg_sum<W>(cr, lane);
  R.c_hat[1] = seg_sum<W>(cg, lane);
  R.c_hat[2] = seg_sum<W>(cbl, lane);
  R.d_hat = seg_sum<W>(dd, lane);
  R.wsum = seg_sum<W>(ws, lane);
}

template <int W>
__device__ __forceinline__ void render_fwd_ray(const RenderArgs& A, int m, int lane) {
  constexpr int NC = seg_chunks<W>();
  const int sl = lane & (W - 1);
  RayState R;
  ray_forward<W>(A, m, lane, R);
  const bool has_d = R.D > 0.f;
  float sdf = 0.f, fs = 0.f, ek = 0.f, ntr = 0.f, nfs = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int k = W * c + sl;
    if (A.weights && k < R.n) A.weights[R.s0 + k] = R.w[c];
    if (!(R.valid[c] && has_d)) continue;
    const float b = R.D - R.tt[c];
    if (fabsf(b) <= A.trunc) {
      sdf += fabsf(R.phi[c] - b);
      ntr += 1.f;
    } else if (b > A.trunc) {
      const float e = __expf(-A.alpha_fs * R.phi[c]) - 1.f;
      fs += fmaxf(fmaxf(0.f, e), R.phi[c] - b);
      if (A.eik) ek += A.eik[R.s0 + k];
      nfs += 1.f;
    }
  }
  // a ray ends at its GOSURF_MAX_SAMPLES_PER_RAY-th sample: later samples are
  // not rendered and get weight 0 (a half-wave ray holds at most 32)
  if (W == 64 && A.weights)
    for (int k = kChunks * 64 + lane; k < R.n; k += 64) A.weights[R.s0 + k] = 0.f;
  sdf = seg_sum<W>(sdf, lane); fs = seg_sum<W>(fs, lane); ek = seg_sum<W>(ek, lane);
  ntr = seg_sum<W>(ntr, lane); nfs = seg_sum<W>(nfs, lane);
  if (sl == 0) {
    A.rgb_hat[3 * m] = R.c_hat[0];
    A.rgb_hat[3 * m + 1] = R.c_hat[1];
    A.rgb_hat[3 * m + 2] = R.c_hat[2];
    A.depth_hat[m] = R.d_hat;
    A.wsum[m] = R.wsum;
    float* p = A.ray_partial + 8 * (size_t)m;
    p[0] = (fabsf(R.I[0] - R.c_hat[0]) + fabsf(R.I[1] - R.c_hat[1]) + fabsf(R.I[2] - R.c_hat[2])) / 3.f;
    p[1] = has_d ? fabsf(R.D - R.d_hat) : 0.f;
    p[2] = ntr > 0.f ? sdf / ntr : 0.f;
    p[3] = nfs > 0.f ? fs / nfs : 0.f;
    p[4] = nfs > 0.f ? ek / nfs : 0.f;
    p[5] = has_d ? 1.f : 0.f;
    p[6] = 0.f;
    p[7] = 0.f;
  }
}

template <int W>
__device__ __forceinline__ void render_bwd_ray(const RenderArgs& A, int m, int lane) {
  constexpr int NC = seg_chunks<W>();
  const int sl = lane & (W - 1);
  RayState R;
  ray_forward<W>(A, m, lane, R);
  const bool has_d = R.D > 0.f;
  const float invM = 1.f / (float)A.M;
  const float nd = *A.n_depth_rays;
  const float sc = A.loss_scale;
  float gc[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) gc[ch] = -signf_(R.I[ch] - R.c_hat[ch]) * A.lam[0] * invM * (1.f / 3.f);
  const float gd = (has_d && nd > 0.f) ? -signf_(R.D - R.d_hat) * A.lam[1] / nd : 0.f;

  // subset sizes
  float ntr = 0.f, nfs = 0.f;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (!(R.valid[c] && has_d)) continue;
    const float b = R.D - R.tt[c];
    if (fabsf(b) <= A.trunc) ntr += 1.f;
    else if (b > A.trunc) nfs += 1.f;
  }
  ntr = seg_sum<W>(ntr, lane);
  nfs = seg_sum<W>(nfs, lane);
  const int nch = W == 64 ? (R.n + 63) >> 6 : 1;   // chunks holding samples (uniform over the segment's wave)

  // dL/dw_k and the suffix recurrence Q_i = g_i alpha_i + (1 - alpha_i) Q_{i+1}
  float g[kChunks], Q[kChunks];
#pragma unroll
  for (int c = 0; c < NC; ++c)
    g[c] = gc[0] * R.col[c][0] + gc[1] * R.col[c][1] + gc[2] * R.col[c][2] + gd * R.da[c];
  float carry = 0.f;   // Q just past the current chunk
#pragma unroll
  for (int c = NC - 1; c >= 0; --c) {
    if (c >= nch) {
      Q[c] = 0.f;
      continue;
    }
    float a = 1.f - R.alpha[c], b = g[c] * R.alpha[c];
    seg_affine_suffix<W>(a, b, lane);
    Q[c] = b + a * carry;
    carry = seg_first<W>(Q[c], lane);
  }
  float dv_acc = 0.f;
  float dalpha[kChunks], act_next[kChunks];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c >= nch) {
      dalpha[c] = 0.f;
      continue;
    }
    // R_k = Q_{k+1}
    float Rk = seg_next<W>(Q[c], sl);
    if (c + 1 < NC && c + 1 < nch) {
      const float q0 = lane_at(Q[c + 1], 0);
      if (lane == 63) Rk = q0;
    }
    dalpha[c] = R.alpha[c] > 0.f ? R.T[c] * (g[c] - Rk) : 0.f;
  }
  const float s = R.s;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c >= nch) {
      act_next[c] = 0.f;
      continue;
    }
    const int k = W * c + sl;
    // this interval's derivative factors (active only when alpha > 0)
    const float om = 1.f - R.alpha[c];
    const float q_here = sigmoidf_(-s * R.phi[c]);           // 1 - Phi_s(phi_k)
    float nphi = seg_next<W>(R.phi[c], sl);
    if (c + 1 < NC && c + 1 < nch) {
      const float p0 = lane_at(R.phi[c + 1], 0);
      if (lane == 63) nphi = p0;
    }
    const float q_next = sigmoidf_(-s * nphi);
    // 1 - alpha = Phi(phi_{k+1}) / Phi(phi_k) exactly when alpha > 0
    const float ratio = R.alpha[c] > 0.f ? om : 0.f;
    const float d_self = dalpha[c] * s * ratio * q_here;      // d alpha_k / d phi_k
    const float d_next = -dalpha[c] * s * ratio * q_next;     // d alpha_k / d phi_{k+1}
    dv_acc += dalpha[c] * ratio * (R.phi[c] * q_here - nphi * q_next);
    // contribution of interval k-1 to phi_k
    float from_prev = seg_prev<W>(d_next, sl);
    if (c > 0) {
      const float p63 = lane_at(act_next[c - 1], 63);
      if (lane == 0) from_prev = p63;
    }
    act_next[c] = d_next;
    float dphi = d_self + from_prev;
    float ew = 0.f;
    if (R.valid[c] && has_d) {
      const float b = R.D - R.tt[c];
      if (fabsf(b) <= A.trunc) {
        dphi += A.lam[2] * invM / ntr * signf_(R.phi[c] - b);
      } else if (b > A.trunc) {
        const float ex = __expf(-A.alpha_fs * R.phi[c]);
        const float e = ex - 1.f, lin = R.phi[c] - b;
        const float inner = fmaxf(0.f, e);
        float dl = 0.f;
        if (lin > inner) dl = 1.f;
        else if (e > 0.f) dl = -A.alpha_fs * ex;
        dphi += A.lam[3] * invM / nfs * dl;
        ew = A.lam[4] * invM / nfs;
      }
    }
    if (k < R.n) {
      const size_t sidx = R.s0 + k;
      const float wk = R.w[c];
      float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
      if (R.valid[c]) out = make_float4(dphi * sc, gc[0] * wk * sc, gc[1] * wk * sc, gc[2] * wk * sc);
      *reinterpret_cast<float4*>(A.seed4 + 4 * sidx) = out;
      // the position again (same rounding as the forward), so that the field
      // backward reads it with the seeds instead of through ray_of, t, o, r
      const float tt = R.tt[c];
      *reinterpret_cast<float4*>(A.posw + 4 * sidx) =
          make_float4(mad_norm(tt, R.r[0], R.o[0]), mad_norm(tt, R.r[1], R.o[1]), mad_norm(tt, R.r[2], R.o[2]),
                      R.valid[c] ? ew * sc : 0.f);
    }
  }
  // samples past the per-ray cap are not rendered: zero seeds and a position
  // outside the box, so that the field backward neither gathers nor scatters
  // for them (instead of reading what an earlier call left in the workspace)
  if (W == 64)
    for (int k = kChunks * 64 + lane; k < R.n; k += 64) {
      const size_t sidx = R.s0 + k;
      *reinterpret_cast<float4*>(A.seed4 + 4 * sidx) = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<float4*>(A.posw + 4 * sidx) =
          make_float4(A.g.p0[0] - 1.f, A.g.p0[1] - 1.f, A.g.p0[2] - 1.f, 0.f);
    }
  dv_acc = seg_sum<W>(dv_acc, lane);
  // d s / d v = 10 s
  if (sl == 0) A.ray_dv[m] = dv_acc * 10.f * s * sc;
}

// One wave per ray, except that two neighbouring rays (2i, 2i + 1) of at most
// 32 samples each share the wave of ray 2i, one half each, and the wave of
// ray 2i + 1 ends at once: a wave's time is mostly memory latency, which the
// two rays then share.  Both waves take the decision from the same offsets.
__device__ __forceinline__ int ray_len(const RenderArgs& A, int m) {
  const int s0 = min(max(A.seg[m], 0), A.total);
  return max(min(A.seg[m + 1], A.total) - s0, 0);
}
__device__ __forceinline__ bool short_pair(const RenderArgs& A, int pm) {
  return pm + 1 < A.M && ray_len(A, pm) <= 32 && ray_len(A, pm + 1) <= 32;
}

__global__ __launch_bounds__(256) void render_fwd_kernel(RenderArgs A) {
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (m >= A.M) return;
  if (short_pair(A, m & ~1)) {
    if ((m & 1) == 0) render_fwd_ray<32>(A, m + (lane >> 5), lane);
    return;
  }
  render_fwd_ray<64>(A, m, lane);
}

__global__ __launch_bounds__(256) void render_bwd_kernel(RenderArgs A) {
  const int lane = threadIdx.x & 63;
  const int m = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (m >= A.M) return;
  if (short_pair(A, m & ~1)) {
    if ((m & 1) == 0) render_bwd_ray<32>(A, m + (lane >> 5), lane);
    return;
  }
  render_bwd_ray<64>(A, m, lane);
}

// ---------------------------------------------------------------- reductions (fixed order)
// Sums over rays in two fixed-order stages.  Stage 1: block b adds columns
// 0..NCOL-1 of rays b*256 + t, b*256 + t + 256*gridDim, ... per thread, then
// over its 256 threads in a fixed tree, into part[b][0..NCOL-1] (rows of 8).
constexpr int kRaySumBlocks = 64;
template <int NCOL>
__global__ __launch_bounds__(256) void ray_sum_stage1_kernel(const float* __restrict__ x, int M, int stride,
                                                             float* __restrict__ part) {
  __shared__ float red[NCOL][256];
  float acc[NCOL];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) acc[c] = 0.f;
  for (int m = blockIdx.x * 256 + threadIdx.x; m < M; m += gridDim.x * 256)
#pragma unroll
    for (int c = 0; c < NCOL; ++c) acc[c] += x[(size_t)m * stride + c];
#pragma unroll
  for (int c = 0; c < NCOL; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int c = 0; c < NCOL; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < NCOL) part[8 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

int ray_sum_blocks(int M) {
  const int b = (M + 255) / 256;
  return b < 1 ? 1 : (b > kRaySumBlocks ? kRaySumBlocks : b);
}

// Stage 2 of the loss: the block partials of the six per-ray columns (rgb,
// depth, sdf, fs, eik, rays with depth) in block order, the smoothness block
// partials in a fixed tree; then the set means and the weighted total.
__global__ __launch_bounds__(256) void loss_final_kernel(const float* __restrict__ part, int nb,
                                                         const float* __restrict__ smooth_partial, int n_sp, int M,
                                                         int S, float l0, float l1, float l2, float l3, float l4,
                                                         float l5, float* __restrict__ losses) {
  __shared__ float sred[256];
  float sm = 0.f;
  for (int i = threadIdx.x; i < n_sp; i += 256) sm += smooth_partial[i];
  sred[threadIdx.x] = sm;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sred[threadIdx.x] += sred[threadIdx.x + w];
    __syncthreads();
  }
  // block partials: lane b of wave 0 holds block b's row (nb <= 64), summed
  // over the wave in a fixed order
  float col[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (threadIdx.x < 64) {
#pragma unroll
    for (int c = 0; c < 6; ++c) col[c] = wave_sum_dpp((int)threadIdx.x < nb ? part[8 * threadIdx.x + c] : 0.f);
  }
  if (threadIdx.x == 0) {
    const float invM = 1.f / (float)M;
    const float nd = col[5];
    const float L[6] = {col[0] * invM, nd > 0.f ? col[1] / nd : 0.f, col[2] * invM,
                        col[3] * invM, col[4] * invM, S > 0 ? sred[0] / (float)S : 0.f};
    const float lam[6] = {l0, l1, l2, l3, l4, l5};
    float tot = 0.f;
    for (int k = 0; k < 6; ++k) { losses[k] = L[k]; tot += lam[k] * L[k]; }
    losses[6] = tot;
    losses[7] = nd;
  }
}

// Column sums of a [rows][cols] matrix of block partials, in two fixed-order
// stages: block (x, y) sums rows y, y + R1, y + 2 R1, ... of columns
// 256x .. 256x + 255 into tmp[y][col]; the second stage sums the R1 rows of tmp.
constexpr int kR1 = 64;

__global__ __launch_bounds__(256) void colsum_stage1_kernel(const float* __restrict__ part, int rows, int cols,
                                                            float* __restrict__ tmp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y;
  if (e >= cols) return;
  float s0 = 0.f, s1 = 0.f;
  int r = y;
  for (; r + kR1 < rows; r += 2 * kR1) {
    s0 += part[(size_t)r * cols + e];
    s1 += part[(size_t)(r + kR1) * cols + e];
  }
  if (r < rows) s0 += part[(size_t)r * cols + e];
  tmp[(size_t)y * cols + e] = s0 + s1;
}

__device__ __forceinline__ float colsum_stage2(const float* __restrict__ tmp, int cols, int e) {
  float s = 0.f;
#pragma unroll 8
  for (int y = 0; y < kR1; ++y) s += tmp[(size_t)y * cols + e];
  return s;
}

// grads.mlp += column sums; entry v gets the per-ray dL/dv sums instead (the
// nb block partials of ray_sum_stage1, in block order)
__global__ __launch_bounds__(256) void grad_stage2_kernel(const float* __restrict__ tmp, const float* __restrict__ dv_part,
                                                          int nb, float* __restrict__ grad_mlp) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= kMlpNumel) return;
  if (blockIdx.x == 0 && threadIdx.x < 64) {   // wave 0 of block 0: the nb <= 64 dL/dv partials
    const float s = wave_sum_dpp((int)threadIdx.x < nb ? dv_part[8 * threadIdx.x] : 0.f);
    if (threadIdx.x == 0) grad_mlp[oV] += s;
  }
  if (e == oV) return;
  grad_mlp[e] += colsum_stage2(tmp, kMlpNumel, e);
}

hipError_t launch_colsum_stage1(const float* part, int rows, int cols, float* tmp, hipStream_t st) {
  hipLaunchKernelGGL(colsum_stage1_kernel, dim3((cols + 255) / 256, kR1), dim3(256), 0, st, part, rows, cols, tmp);
  return hipGetLastError();
}

hipError_t launch_grad_reduce(const float* partial, int n_part, const float* ray_dv, int M, float* grad_mlp,
                              float* tmp, float* ray_part, hipStream_t st) {
  hipError_t e = launch_colsum_stage1(partial, n_part, kMlpNumel, tmp, st);
  if (e != hipSuccess) return e;
  const int nb = ray_sum_blocks(M);
  hipLaunchKernelGGL(ray_sum_stage1_kernel<1>, dim3(nb), dim3(256), 0, st, ray_dv, M, 1, ray_part);
  hipLaunchKernelGGL(grad_stage2_kernel, dim3((kMlpNumel + 255) / 256), dim3(256), 0, st, tmp, ray_part, nb,
                     grad_mlp);
  return hipGetLastError();
}

int colsum_rows() { return kR1; }

// dst[e] += column sum e for e < n_add; set_dst = column sum `set_col`
__global__ __launch_bounds__(256) void colsum_stage2_kernel(const float* __restrict__ tmp, int cols,
                                                            float* __restrict__ add_dst, int n_add,
                                                            float* __restrict__ set_dst, int set_col) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= cols) return;
  const float v = colsum_stage2(tmp, cols, e);
  if (e < n_add) add_dst[e] += v;
  if (e == set_col && set_dst) *set_dst = v;
}

hipError_t launch_colsum(const float* part, int rows, int cols, float* tmp, float* add_dst, int n_add,
                         float* set_dst, int set_col, hipStream_t st) {
  hipError_t e = launch_colsum_stage1(part, rows, cols, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(colsum_stage2_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, tmp, cols, add_dst, n_add,
                     set_dst, set_col);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Adam
// Streaming accesses: every parameter, gradient and moment is touched once
// per step, so the loads and stores bypass the caches' retention (non-temporal).
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4* a) {
  const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(a));
  return make_float4(x[0], x[1], x[2], x[3]);
}
__device__ __forceinline__ void st_stream(float4 v, float4* a) {
  const f4v x = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(a));
}

struct AdamGroup {
  float4* p;
  float4* g;
  float4* m;
  float4* v;
  uint2* bf;   // optional bfloat16 mirror of p (4 values per entry)
  long long n4;
  float lr;
};

// Two float4 per thread and pass, both loaded before either is updated.  The
// grid group comes first in the flattened index, then the decoder group.
constexpr int kAdamUnroll = 2;
// skip (optional device flag, nonzero = skip): the step is dropped on the
// device, only the gradients are zeroed.
__global__ __launch_bounds__(256) void adam_kernel(AdamGroup G0, AdamGroup G1, float b1, float b2, float eps,
                                                   float inv_bc1, float inv_sqrt_bc2, float inv_scale,
                                                   const int* __restrict__ skip) {
  const long long n4 = G0.n4 + G1.n4;
  const long long stride = (long long)gridDim.x * 256 * kAdamUnroll;
  if (skip && __builtin_amdgcn_readfirstlane(*skip) != 0) {
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n4; i += (long long)gridDim.x * 256) {
      const AdamGroup& Gr = i < G0.n4 ? G0 : G1;
      st_stream(make_float4(0.f, 0.f, 0.f, 0.f), Gr.g + (i < G0.n4 ? i : i - G0.n4));
    }
    return;
  }
  for (long long base = (long long)blockIdx.x * 256 * kAdamUnroll + threadIdx.x; base < n4; base += stride) {
    float4 p[kAdamUnroll], g[kAdamUnroll], m[kAdamUnroll], v[kAdamUnroll];
#pragma unroll
    for (int u = 0; u < kAdamUnroll; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n4) {
        const AdamGroup& Gr = i < G0.n4 ? G0 : G1;
        const long long k = i < G0.n4 ? i : i - G0.n4;
        p[u] = ld_stream(Gr.p + k);
        g[u] = ld_stream(Gr.g + k);
        m[u] = ld_stream(Gr.m + k);
        v[u] = ld_stream(Gr.v + k);
      }
    }
#pragma unroll
    for (int u = 0; u < kAdamUnroll; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n4) {
        const AdamGroup& Gr = i < G0.n4 ? G0 : G1;
        const long long k = i < G0.n4 ? i : i - G0.n4;
        float pa[4] = {p[u].x, p[u].y, p[u].z, p[u].w}, ga[4] = {g[u].x, g[u].y, g[u].z, g[u].w};
        float ma[4] = {m[u].x, m[u].y, m[u].z, m[u].w}, va[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float gs_ = ga[c] * inv_scale;
          ma[c] = b1 * ma[c] + (1.f - b1) * gs_;
          va[c] = b2 * va[c] + (1.f - b2) * gs_ * gs_;
          const float den = sqrtf(va[c]) * inv_sqrt_bc2 + eps;
          pa[c] -= Gr.lr * (ma[c] * inv_bc1) / den;
        }
        st_stream(make_float4(pa[0], pa[1], pa[2], pa[3]), Gr.p + k);
        st_stream(make_float4(ma[0], ma[1], ma[2], ma[3]), Gr.m + k);
        st_stream(make_float4(va[0], va[1], va[2], va[3]), Gr.v + k);
        st_stream(make_float4(0.f, 0.f, 0.f, 0.f), Gr.g + k);
        if (Gr.bf) {
          const uint32_t lo = f2bf2(pa[0], pa[1]);
          const uint32_t hi = f2bf2(pa[2], pa[3]);
          Gr.bf[k] = make_uint2(lo, hi);
        }
      }
    }
  }
}

hipError_t launch_render(const RenderArgs& a, bool bwd, hipStream_t st) {
  const int blocks = (a.M + 3) / 4;
  if (bwd) hipLaunchKernelGGL(render_bwd_kernel, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(render_fwd_kernel, dim3(blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_loss_reduce(const float* ray_partial, int M, const float* smooth_partial, int n_sp, int S,
                              const float lam[6], float* losses, float* ray_part, hipStream_t st) {
  const int nb = ray_sum_blocks(M);
  hipLaunchKernelGGL(ray_sum_stage1_kernel<6>, dim3(nb), dim3(256), 0, st, ray_partial, M, 8, ray_part);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, ray_part, nb, smooth_partial, n_sp, M, S, lam[0],
                     lam[1], lam[2], lam[3], lam[4], lam[5], losses);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float4* __restrict__ src, uint2* __restrict__ dst,
                                                      long long n4) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n4; i += (long long)gridDim.x * 256) {
    const float4 v = src[i];
    dst[i] = make_uint2(f2bf2(v.x, v.y), f2bf2(v.z, v.w));
  }
}

hipError_t launch_to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t st) {
  const long long n4 = n / 4;
  long long blocks = (n4 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(to_bf16_kernel, dim3((unsigned)blocks), dim3(256), 0, st, reinterpret_cast<const float4*>(src),
                     reinterpret_cast<uint2*>(dst), n4);
  return hipGetLastError();
}

// the last numel % 4 entries of a group (scalar)
__global__ void adam_tail_kernel(float* __restrict__ p, float* __restrict__ g, float* __restrict__ m,
                                 float* __restrict__ v, int n, float lr, float b1, float b2, float eps, float inv_bc1,
                                 float inv_sqrt_bc2, float inv_scale, const int* __restrict__ skip) {
  const int i = threadIdx.x;
  if (i >= n) return;
  if (skip && *skip != 0) {
    g[i] = 0.f;
    return;
  }
  const float gg = g[i] * inv_scale;
  m[i] = b1 * m[i] + (1.f - b1) * gg;
  v[i] = b2 * v[i] + (1.f - b2) * gg * gg;
  p[i] -= lr * (m[i] * inv_bc1) / (sqrtf(v[i]) * inv_sqrt_bc2 + eps);
  g[i] = 0.f;
}

hipError_t launch_adam(const gosurf_adam_cfg& c, gosurf_adam_state& s, const int* skip, hipStream_t st) {
  const long long n4g = s.grid_numel / 4;
  const int n4m = s.mlp_numel / 4;
  const int tail = s.mlp_numel - 4 * n4m;
  const double bc1 = 1.0 - pow((double)c.beta1, (double)c.step);
  const double bc2 = 1.0 - pow((double)c.beta2, (double)c.step);
  const AdamGroup G0{reinterpret_cast<float4*>(s.grid), reinterpret_cast<float4*>(s.grid_grad),
                     reinterpret_cast<float4*>(s.grid_m), reinterpret_cast<float4*>(s.grid_v),
                     reinterpret_cast<uint2*>(s.grid_bf16), n4g, c.lr_grid};
  const AdamGroup G1{reinterpret_cast<float4*>(s.mlp), reinterpret_cast<float4*>(s.mlp_grad),
                     reinterpret_cast<float4*>(s.mlp_m), reinterpret_cast<float4*>(s.mlp_v), nullptr, n4m, c.lr_mlp};
  // one pass: each thread takes kAdamUnroll float4 (the loop covers larger sizes)
  long long blocks = (n4g + n4m + 256 * kAdamUnroll - 1) / (256 * kAdamUnroll);
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  if (n4g + n4m > 0)
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G0, G1, c.beta1, c.beta2, c.eps,
                       (float)(1.0 / bc1), (float)(1.0 / sqrt(bc2)), c.inv_loss_scale, skip);
  if (tail > 0) {
    const size_t o = 4 * (size_t)n4m;
    hipLaunchKernelGGL(adam_tail_kernel, dim3(1), dim3(64), 0, st, s.mlp + o, s.mlp_grad + o, s.mlp_m + o,
                       s.mlp_v + o, tail, c.lr_mlp, c.beta1, c.beta2, c.eps, (float)(1.0 / bc1),
                       (float)(1.0 / sqrt(bc2)), c.inv_loss_scale, skip);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- non-finite gradient check
// A float is non-finite when its exponent bits are all ones (inf or NaN);
// tested on the bits so that no compiler flag can fold the test away.
__device__ __forceinline__ bool nonfinite(float x) { return (__float_as_uint(x) & 0x7f800000u) == 0x7f800000u; }

__global__ void set_flag_kernel(int* flag, int value) { *flag = value; }

// *flag = 1 if any of a[0 .. n) is inf or NaN (a is 16-byte aligned); the
// flag is cleared on the stream beforehand, and every writer stores the same value
__global__ __launch_bounds__(256) void nonfinite_kernel(const float* __restrict__ a, long long n,
                                                        int* __restrict__ flag) {
  const long long n4 = n / 4;
  const float4* a4 = reinterpret_cast<const float4*>(a);
  bool bad = false;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n4; i += (long long)gridDim.x * 256) {
    const float4 v = a4[i];
    bad |= nonfinite(v.x) | nonfinite(v.y) | nonfinite(v.z) | nonfinite(v.w);
  }
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) bad |= nonfinite(a[4 * n4 + threadIdx.x]);
  if (bad) flag[0] = 1;
}

__global__ __launch_bounds__(256) void zero_kernel(float* __restrict__ a, long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) a[i] = 0.f;
}

static unsigned stream_blocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

hipError_t launch_nonfinite_check(const float* grid_grad, long long n_grid, const float* mlp_grad, long long n_mlp,
                                  int* flag, hipStream_t st) {
  hipLaunchKernelGGL(set_flag_kernel, dim3(1), dim3(1), 0, st, flag, 0);
  if (n_grid > 0)
    hipLaunchKernelGGL(nonfinite_kernel, dim3(stream_blocks(n_grid / 4)), dim3(256), 0, st, grid_grad, n_grid, flag);
  if (n_mlp > 0)
    hipLaunchKernelGGL(nonfinite_kernel, dim3(stream_blocks(n_mlp / 4)), dim3(256), 0, st, mlp_grad, n_mlp, flag);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void zero4_kernel(float4* __restrict__ a, long long n4) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n4; i += (long long)gridDim.x * 256)
    a[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

hipError_t launch_zero(float* a, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n % 4 == 0 && reinterpret_cast<uintptr_t>(a) % 16 == 0)
    hipLaunchKernelGGL(zero4_kernel, dim3(stream_blocks(n / 4)), dim3(256), 0, st, reinterpret_cast<float4*>(a),
                       n / 4);
  else
    hipLaunchKernelGGL(zero_kernel, dim3(stream_blocks(n)), dim3(256), 0, st, a, n);
  return hipGetLastError();
}

}  // namespace gs
