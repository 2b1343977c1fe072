// Trilinear gather of one grid level for one lane (Sec. 3.1; coefficient
// vector and Jacobian of the supplementary "Second-order Grid Sampler").
#pragma once
#include "device.h"

namespace gs {

// per-lane gather state of one level
struct LevelSample {
  float f[3];
  long long row;   // corner 000
  int sy, sz;      // row strides of +y, +z corners
  int cell;        // cell indices i | j << 11 | k << 22 (each below 2048 where gradient copies are used)
  float inv_v;
};

// Sizes of the grid level one lane works on.  The by-value grid description
// lives in the kernel-argument segment; indexing its per-level arrays with a
// per-lane level makes the compiler read them from memory at every use, and
// such a read waits for all earlier memory operations of the wave (the
// scatter's atomics included, which share the vector-memory counter).  So each
// entry is read once as a wave-uniform scalar and the lane's value selected in
// registers.
struct LevelConst {
  int n[3];
  float voxel;
  long long off;
};

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int pick_level(const int (&a)[4], int q) {
  const int v0 = uniform_i(a[0]), v1 = uniform_i(a[1]), v2 = uniform_i(a[2]), v3 = uniform_i(a[3]);
  return q == 0 ? v0 : q == 1 ? v1 : q == 2 ? v2 : v3;
}

__device__ __forceinline__ LevelConst level_const(const Grid& g, int q) {
  LevelConst c;
  c.n[0] = pick_level(g.nx, q);
  c.n[1] = pick_level(g.ny, q);
  c.n[2] = pick_level(g.nz, q);
  const int vb[4] = {__float_as_int(g.voxel[0]), __float_as_int(g.voxel[1]), __float_as_int(g.voxel[2]),
                     __float_as_int(g.voxel[3])};
  c.voxel = __int_as_float(pick_level(vb, q));
  const int lo[4] = {(int)g.off[0], (int)g.off[1], (int)g.off[2], (int)g.off[3]};
  const int hi[4] = {(int)(g.off[0] >> 32), (int)(g.off[1] >> 32), (int)(g.off[2] >> 32), (int)(g.off[3] >> 32)};
  c.off = (long long)(((unsigned long long)(unsigned)pick_level(hi, q) << 32) | (unsigned)pick_level(lo, q));
  return c;
}

__device__ __forceinline__ void locate(const Grid& g, const LevelConst& lc, float x, float y, float z,
                                       LevelSample& ls) {
  const float xyz[3] = {x, y, z};
  const float v = lc.voxel;
  int i0[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    float u = (xyz[a] - g.p0[a]) / v;
    int c = (int)floorf(u);
    c = c < 0 ? 0 : (c > lc.n[a] - 2 ? lc.n[a] - 2 : c);
    i0[a] = c;
    ls.f[a] = u - (float)c;
  }
  ls.sy = lc.n[0];
  ls.sz = lc.n[0] * lc.n[1];
  ls.row = lc.off + ((long long)i0[2] * lc.n[1] + i0[1]) * lc.n[0] + i0[0];
  ls.cell = i0[0] | (i0[1] << 11) | (i0[2] << 22);
  ls.inv_v = 1.f / v;
}

__device__ __forceinline__ float comp(const float4& v, int k) {
  return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
}

// Off-diagonal second derivatives d^2 z_k / dx_a dx_b of one level (the
// supplementary's h12, h13, h23; the diagonal is zero), in world units.
struct LevelHess {
  float h[4][3];   // [feature][h12, h13, h23]
};

// trilinear value (z) and, optionally, dz/dx (G[k][axis]) and the second
// derivatives (H) of one level
template <bool NEED_G, bool BF, bool NEED_H = false>
__device__ __forceinline__ void interp(const float* __restrict__ grid, const uint16_t* __restrict__ grid_bf,
                                       const LevelSample& ls, bool valid, float z[4], float G[4][3],
                                       LevelHess* H = nullptr) {
#pragma unroll
  for (int k = 0; k < 4; ++k) { z[k] = 0.f; G[k][0] = G[k][1] = G[k][2] = 0.f; }
  if constexpr (NEED_H) {
#pragma unroll
    for (int k = 0; k < 4; ++k) H->h[k][0] = H->h[k][1] = H->h[k][2] = 0.f;
  }
  if (!valid) return;
  const float fx = ls.f[0], fy = ls.f[1], fz = ls.f[2];
  float4 th[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const long long row = ls.row + bx + (long long)by * ls.sy + (long long)bz * ls.sz;
    if constexpr (BF) {
      const uint2 u = *reinterpret_cast<const uint2*>(grid_bf + row * 4);
      th[c] = make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                          __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
    } else {
      th[c] = *reinterpret_cast<const float4*>(grid + row * 4);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int bx = (c >> 2) & 1, by = (c >> 1) & 1, bz = c & 1;
    const float wx = bx ? fx : 1.f - fx, wy = by ? fy : 1.f - fy, wz = bz ? fz : 1.f - fz;
    const float w = wx * wy * wz;
    const float tv[4] = {th[c].x, th[c].y, th[c].z, th[c].w};
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] += w * tv[k];
    if (NEED_G) {
      const float jx = (bx ? 1.f : -1.f) * wy * wz, jy = (by ? 1.f : -1.f) * wx * wz,
                  jz = (bz ? 1.f : -1.f) * wx * wy;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        G[k][0] += jx * tv[k];
        G[k][1] += jy * tv[k];
        G[k][2] += jz * tv[k];
      }
    }
  }
  if (NEED_G) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { G[k][0] *= ls.inv_v; G[k][1] *= ls.inv_v; G[k][2] *= ls.inv_v; }
  }
  if constexpr (NEED_H) {
    // corner c = 4 bx + 2 by + bz; h12 mixes x and y at the two z faces, etc.
    const float iv2 = ls.inv_v * ls.inv_v;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float t0 = comp(th[0], k), t1 = comp(th[1], k), t2 = comp(th[2], k), t3 = comp(th[3], k);
      const float t4 = comp(th[4], k), t5 = comp(th[5], k), t6 = comp(th[6], k), t7 = comp(th[7], k);
      H->h[k][0] = ((1.f - fz) * (t0 + t6 - t2 - t4) + fz * (t1 + t7 - t3 - t5)) * iv2;
      H->h[k][1] = ((1.f - fy) * (t0 + t5 - t1 - t4) + fy * (t2 + t7 - t3 - t6)) * iv2;
      H->h[k][2] = ((1.f - fx) * (t0 + t3 - t1 - t2) + fx * (t4 + t7 - t5 - t6)) * iv2;
    }
  }
}

}  // namespace gs
