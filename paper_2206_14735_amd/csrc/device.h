// Device helpers shared by the gfx950 kernels of the GO-Surf hot path.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gosurf.h"

namespace gs {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;
constexpr int kTile = 16;          // samples per wave-tile (one 16-wide MFMA column block)
constexpr int kBlock = 256;        // threads per block of the field kernels (4 waves)
constexpr int kWavesPerBlock = kBlock / kWave;

// ---------------------------------------------------------------- packed decoder offsets
// W1[32][16] b1[32] W2[32][32] b2[32] W3[16][32] b3[16] U1[32][15] c1[32] U2[3][32] c2[3] v[1]
constexpr int oW1 = 0, oB1 = 512, oW2 = 544, oB2 = 1568, oW3 = 1600, oB3 = 2112;
constexpr int oU1 = 2128, oC1 = 2608, oU2 = 2640, oC2 = 2736, oV = 2739, kMlpNumel = 2740;
static_assert(kMlpNumel == GOSURF_MLP_NUMEL, "decoder layout");

// ---------------------------------------------------------------- grid description (by value)
struct Grid {
  float p0[3], p1[3];
  float voxel[4];
  int nx[4], ny[4], nz[4];
  long long off[4];   // first vertex row of each level
};

// ---------------------------------------------------------------- Philox4x32-10 (Salmon et al. SC'11)
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return U4{c0, c1, c2, c3};
}

__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------- exact-rounding helpers
// o + t*r with the product and the sum rounded separately, so that the box
// test and the cell choice take the same decisions as a plain float32
// evaluation.  The pragma matters: hipcc fuses even __fadd_rn(__fmul_rn())
// into one v_fmac_f32 (a single rounding) under its default contraction.
__device__ __forceinline__ float mad_norm(float t, float r, float o) {
#pragma clang fp contract(off)
  return t * r + o;
}

__device__ __forceinline__ bool inside_box(const Grid& g, float x, float y, float z) {
  return x >= g.p0[0] && x <= g.p1[0] && y >= g.p0[1] && y <= g.p1[1] && z >= g.p0[2] &&
         z <= g.p1[2];
}

// The plain sampler's span of a ray: fixed [near, far], or its passage
// through the grid box clipped to [near, far] (slab test; 0/0 -> NaN is
// ignored by fminf/fmaxf).
__device__ __forceinline__ void ray_span(const Grid& g, const float o[3], const float r[3], int mode, float near_t,
                                         float far_t, float& tn, float& tf) {
  tn = near_t;
  tf = far_t;
  if (mode == GOSURF_SPAN_BOX) {
    float tmin = -INFINITY, tmax = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const float ta = (g.p0[a] - o[a]) / r[a];
      const float tb = (g.p1[a] - o[a]) / r[a];
      tmin = fmaxf(tmin, fminf(ta, tb));
      tmax = fminf(tmax, fmaxf(ta, tb));
    }
    tn = fmaxf(tmin, near_t);
    tf = fmaxf(fminf(tmax, far_t), tn);
  }
}

// ---------------------------------------------------------------- numerics
__device__ __forceinline__ float log_sigmoid(float x) {
  // log(1 / (1 + e^-x)) = -softplus(-x), evaluated without overflow
  return x >= 0.f ? -log1pf(__expf(-x)) : x - log1pf(__expf(x));
}
__device__ __forceinline__ float sigmoidf_(float x) {
  return x >= 0.f ? 1.f / (1.f + __expf(-x)) : __expf(x) / (1.f + __expf(x));
}
__device__ __forceinline__ float signf_(float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); }

// float -> bfloat16, round to nearest even (the hardware conversion; NaN stays
// NaN; float32 subnormals are flushed like all float32 arithmetic here)
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
// two values in one 32-bit word, a in the low half
__device__ __forceinline__ uint32_t f2bf2(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2_t{a, b}, bf16x2_t));
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------- MFMA (CDNA3/4 16x16x4 fp32)
// D[16x16] += A[16x4] B[4x16].  Lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the result holds D[4*(l/16) + r][l%16] in component r.
__device__ __forceinline__ v4f mfma4(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// bf16 16x16x16: lane l supplies A[l%16][4(l/16)+0..3] and B[4(l/16)+0..3][l%16].
__device__ __forceinline__ v4f mfma16_bf16(v4s a, v4s b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// DPP moves inside one 16-lane row; lanes whose source lies outside the row read 0.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int kRowShl1 = 0x101, kRowShl2 = 0x102, kRowShl4 = 0x104, kRowShl8 = 0x108;  // lane j <- j + d
constexpr int kRowShr1 = 0x111;                                                        // lane j <- j - 1

// Float atomics with the address space stated: a generic (flat) atomic would
// also count against the LDS wait counter, so every LDS fence after a scatter
// would wait for the scatter's atomics in memory.
typedef __attribute__((address_space(1))) float global_float;
typedef __attribute__((address_space(3))) float lds_float;
__device__ __forceinline__ void atomic_add_global(float* p, float v) {
  __hip_atomic_fetch_add((global_float*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_add_lds(float* p, float v) {
  __hip_atomic_fetch_add((lds_float*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until at most N vector-memory operations of this wave are outstanding
// (s_waitcnt: vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt at their
// maxima, so they are not waited on).
template <int N>
__device__ __forceinline__ void wait_vmem_at_most() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fills tab[0 .. n) with value(e), a value loaded from global memory, in
// batches of 8 entries per thread: each thread then waits for 8 loads in
// flight at once instead of one after another (block of NT threads).
template <int NT, class F>
__device__ __forceinline__ void fill_batched(float* tab, int n, int tid, F value) {
  for (int e0 = tid; e0 < n; e0 += 8 * NT) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      v[u] = e < n ? value(e) : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * NT;
      if (e < n) tab[e] = v[u];
    }
  }
}

// Sum over the 64 lanes of a wave with every lane active, in a fixed order:
// prefix sums inside each row of 16 lanes by DPP row shifts, then the row
// totals carried on by row broadcasts (lane 15 into row 1 and lane 47 into
// row 3, then lane 31 into rows 2-3); lane 63 ends with the total, which is
// returned to every lane.  Six VALU steps instead of six LDS-crossbar shuffles.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f<0x111>(v);   // row_shr:1
  v += dpp_f<0x112>(v);   // row_shr:2
  v += dpp_f<0x114>(v);   // row_shr:4
  v += dpp_f<0x118>(v);   // row_shr:8
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x142, 0xA, 0xF, false));   // row_bcast:15
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x143, 0xC, 0xF, false));   // row_bcast:31
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

}  // namespace gs
