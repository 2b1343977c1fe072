// MFMA operand helpers shared by the field and proposal kernels.
#pragma once
#include "device.h"

namespace gs {

__device__ __forceinline__ v4s pack_bf16(v4f x) {
  const uint2 u = make_uint2(f2bf2(x[0], x[1]), f2bf2(x[2], x[3]));
  return __builtin_bit_cast(v4s, u);
}
__device__ __forceinline__ v4s pack_bf16(float4 x) {
  const uint2 u = make_uint2(f2bf2(x.x, x.y), f2bf2(x.z, x.w));
  return __builtin_bit_cast(v4s, u);
}
__device__ __forceinline__ v4s as_v4s(uint2 u) {
  v4s r;
  __builtin_memcpy(&r, &u, sizeof(r));
  return r;
}

// fp32 layer: out[bo] = sum over input blocks and steps of A(slot) * in, with
// the A operands pre-arranged per lane in `tab` (slot = base + bo*4*NBI + bi*4 + r).
template <int NBO, int NBI>
__device__ __forceinline__ void layer_f32(const float* __restrict__ tab, int base, const v4f* in, v4f* out,
                                          int lane) {
#pragma unroll
  for (int bo = 0; bo < NBO; ++bo) out[bo] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int bi = 0; bi < NBI; ++bi)
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int bo = 0; bo < NBO; ++bo)
        out[bo] = mfma4(tab[(base + bo * 4 * NBI + bi * 4 + r) * 64 + lane], in[bi][r], out[bo]);
}

// LDS scratch of one operand: [row][sample], 16 samples + 4 floats of padding
// per row (rows of the four lane groups land in different banks).
constexpr int RSR = 20;

template <int NB>
__device__ __forceinline__ void store_rows(float* scr, const v4f* X, int q, int j) {
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) scr[(16 * b + 4 * q + r) * RSR + j] = X[b][r];
}

// X (NB blocks of 16 rows in accumulator layout, [row][sample]) passed through
// the wave's LDS scratch so that lane (q, j) receives row 16b + j at samples
// 4q..4q+3: the operand layout of a product that contracts over the samples.
template <int NB>
__device__ __forceinline__ void rows_to_lanes(float* scr, const v4f* X, float4* out, int q, int j) {
  wave_lds_fence();
  store_rows<NB>(scr, X, q, j);
  wave_lds_fence();
#pragma unroll
  for (int b = 0; b < NB; ++b) out[b] = *reinterpret_cast<const float4*>(scr + (16 * b + j) * RSR + 4 * q);
}

// acc[a][b] += sum over the tile's 16 samples of A[16a + i][s] * B[16b + n][s],
// with both operands from rows_to_lanes.
template <bool BF, int NA, int NB>
__device__ __forceinline__ void outer_lanes(const float4* av, const float4* bv, v4f* acc) {
  if constexpr (BF) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a * NB + b] = mfma16_bf16(pack_bf16(av[a]), pack_bf16(bv[b]), acc[a * NB + b]);
  } else {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[a * NB + b] = mfma4(av[a].x, bv[b].x, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].y, bv[b].y, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].z, bv[b].z, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].w, bv[b].w, acc[a * NB + b]);
      }
  }
}

// Column `col` of the 16x16 accumulator gains the sums over the tile's samples
// of the 16 rows in av (from rows_to_lanes); the other columns are unchanged.
// The B operand is the indicator of column `col`, so one MFMA sums the four
// lane groups' partial sums.
__device__ __forceinline__ void colsum_into(const float4& av, int col, v4f& acc, int j) {
  acc = mfma4((av.x + av.y) + (av.z + av.w), j == col ? 1.f : 0.f, acc);
}

// acc[ba][bb] += sum over the tile's 16 samples of A[16ba + i][s] * B[16bb + n][s].
// The sample axis is the MFMA K axis; lane group q supplies samples 4q..4q+3
// (one 16-byte LDS read per operand block).
template <bool BF, int NA, int NB>
__device__ __forceinline__ void outer_acc(float* scrA, float* scrB, const v4f* A, const v4f* B, v4f* acc,
                                          int q, int j) {
  store_rows<NA>(scrA, A, q, j);
  store_rows<NB>(scrB, B, q, j);
  wave_lds_fence();
  float4 av[NA], bv[NB];
#pragma unroll
  for (int a = 0; a < NA; ++a) av[a] = *reinterpret_cast<const float4*>(scrA + (16 * a + j) * RSR + 4 * q);
#pragma unroll
  for (int b = 0; b < NB; ++b) bv[b] = *reinterpret_cast<const float4*>(scrB + (16 * b + j) * RSR + 4 * q);
  if constexpr (BF) {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a * NB + b] = mfma16_bf16(pack_bf16(av[a]), pack_bf16(bv[b]), acc[a * NB + b]);
  } else {
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[a * NB + b] = mfma4(av[a].x, bv[b].x, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].y, bv[b].y, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].z, bv[b].z, acc[a * NB + b]);
        acc[a * NB + b] = mfma4(av[a].w, bv[b].w, acc[a * NB + b]);
      }
  }
  wave_lds_fence();
}

}  // namespace gs
