// Surface extraction: the reconstructed surface is the zero level set of phi
// (Sec. 3.1).  The SDF is evaluated on a regular lattice by the forward field
// kernel (each lattice row along x is a ray with direction (1, 0, 0) and
// samples t_i = i h), and the surface is extracted by marching tetrahedra:
// every cube of 8 lattice points is split into the six tetrahedra around its
// main diagonal (corners c = bx + 2 by + 4 bz), so neighbouring cubes split
// their shared faces the same way and the surface is closed.
#include "device.h"

#include "args.h"

namespace gs {

// rows (j, k0 + kk) of a slab of `layers` z-layers as rays; lattice point
// x = p0 + h (i, j, k) rounded as the field kernel forms o + t r
__global__ __launch_bounds__(256) void lattice_rays_kernel(LatticeArgs A) {
  const long long n = (long long)A.nx * A.ny * A.layers;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(e % A.nx);
    const long long row = e / A.nx;
    A.t[e] = __fmul_rn((float)i, A.h);
    A.ray_of[e] = (int)row;
    if (i == 0) {
      const int j = (int)(row % A.ny), k = A.k0 + (int)(row / A.ny);
      A.o[3 * row + 0] = A.p0[0];
      A.o[3 * row + 1] = mad_norm((float)j, A.h, A.p0[1]);
      A.o[3 * row + 2] = mad_norm((float)k, A.h, A.p0[2]);
      A.r[3 * row + 0] = 1.f;
      A.r[3 * row + 1] = 0.f;
      A.r[3 * row + 2] = 0.f;
    }
  }
}

__global__ __launch_bounds__(256) void phi_copy_kernel(const float* __restrict__ out4, long long n,
                                                       float* __restrict__ phi) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    phi[e] = out4[4 * e];
}

__global__ void zero_count_kernel(unsigned* count) { *count = 0u; }

// tetrahedra of a cube around its main diagonal 0-7
__device__ __forceinline__ int tet_corner(int t, int q) {
  constexpr int T[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7}, {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};
  return T[t][q];
}

__device__ __forceinline__ void crossing(const float pa[3], const float pb[3], float fa, float fb, float* out) {
  const float w = fa / (fa - fb);
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = pa[a] + w * (pb[a] - pa[a]);
}

// one thread per cube; a wave reserves space for all its triangles with one
// atomic and each lane writes at its prefix
__global__ __launch_bounds__(256) void marching_tets_kernel(MtArgs A) {
  const int lane = threadIdx.x & 63;
  const long long cx = A.nx - 1, cy = A.ny - 1, cz = A.nz - 1;
  const long long ncubes = cx * cy * cz;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long base = (long long)blockIdx.x * blockDim.x; base < ncubes; base += stride) {
    const long long e = base + threadIdx.x;
    const bool live = e < ncubes;
    float v[8], p[8][3];
    int ntri = 0;
    if (live) {
      const int i = (int)(e % cx);
      const int j = (int)((e / cx) % cy);
      const int k = (int)(e / (cx * cy));
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
        v[c] = A.phi[((long long)(k + bz) * A.ny + (j + by)) * A.nx + (i + bx)];
        p[c][0] = A.p0[0] + A.h * (float)(i + bx);
        p[c][1] = A.p0[1] + A.h * (float)(j + by);
        p[c][2] = A.p0[2] + A.h * (float)(k + bz);
      }
#pragma unroll
      for (int t = 0; t < 6; ++t) {
        int nin = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) nin += v[tet_corner(t, q)] < 0.f;
        ntri += (nin == 1 || nin == 3) ? 1 : (nin == 2 ? 2 : 0);
      }
    }
    // wave prefix of the triangle counts
    int incl = ntri;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int u = __shfl_up(incl, d, 64);
      if (lane >= d) incl += u;
    }
    const int total = __shfl(incl, 63, 64);
    unsigned off = 0u;
    if (lane == 63 && total > 0) off = atomicAdd(A.count, (unsigned)total);
    off = (unsigned)__shfl((int)off, 63, 64);
    if (!live || ntri == 0) continue;
    long long slot = (long long)off + incl - ntri;
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      int c4[4], nin = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c4[q] = tet_corner(t, q);
        nin += v[c4[q]] < 0.f;
      }
      if (nin == 0 || nin == 4) continue;
      if (nin == 1 || nin == 3) {
        // the corner alone on its side, then the other three in order
        int lone = 0;
#pragma unroll
        for (int q = 3; q >= 0; --q)
          if ((v[c4[q]] < 0.f) == (nin == 1)) lone = q;
        if (slot < A.max_tris) {
          float* out = A.tris + 9 * slot;
          int w = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            if (q == lone) continue;
            crossing(p[c4[lone]], p[c4[q]], v[c4[lone]], v[c4[q]], out + 3 * w);
            ++w;
          }
        }
        ++slot;
      } else {
        // inside corners a0 < a1, outside corners b0 < b1 (tetrahedron order)
        int a[2], b[2], na = 0, nb = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (v[c4[q]] < 0.f) a[na++ & 1] = c4[q];
          else b[nb++ & 1] = c4[q];
        }
        float e00[3], e01[3], e11[3], e10[3];
        crossing(p[a[0]], p[b[0]], v[a[0]], v[b[0]], e00);
        crossing(p[a[0]], p[b[1]], v[a[0]], v[b[1]], e01);
        crossing(p[a[1]], p[b[1]], v[a[1]], v[b[1]], e11);
        crossing(p[a[1]], p[b[0]], v[a[1]], v[b[0]], e10);
        if (slot < A.max_tris) {
          float* out = A.tris + 9 * slot;
#pragma unroll
          for (int x = 0; x < 3; ++x) { out[x] = e00[x]; out[3 + x] = e01[x]; out[6 + x] = e11[x]; }
        }
        if (slot + 1 < A.max_tris) {
          float* out = A.tris + 9 * (slot + 1);
#pragma unroll
          for (int x = 0; x < 3; ++x) { out[x] = e00[x]; out[3 + x] = e11[x]; out[6 + x] = e10[x]; }
        }
        slot += 2;
      }
    }
  }
}

static int grid_for(long long n) {
  const long long b = (n + 255) / 256;
  return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

hipError_t launch_lattice_rays(const LatticeArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(lattice_rays_kernel, dim3(grid_for((long long)a.nx * a.ny * a.layers)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_phi_copy(const float* out4, long long n, float* phi, hipStream_t st) {
  hipLaunchKernelGGL(phi_copy_kernel, dim3(grid_for(n)), dim3(256), 0, st, out4, n, phi);
  return hipGetLastError();
}

hipError_t launch_marching_tets(const MtArgs& a, hipStream_t st) {
  if (a.nx < 2 || a.ny < 2 || a.nz < 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(1), 0, st, a.count);
  const long long ncubes = (long long)(a.nx - 1) * (a.ny - 1) * (a.nz - 1);
  hipLaunchKernelGGL(marching_tets_kernel, dim3(grid_for(ncubes)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace gs
