// Kernel argument blocks (passed by value to the kernels).
#pragma once
#include "device.h"

namespace gs {

constexpr int kChunks = GOSURF_MAX_SAMPLES_PER_RAY / 64;

// Depth-edge test of the proposal's segment pass: the frames' depth images
// [T][H][W], each ray's pixel, the threshold (metres; 0 = off).
struct EdgeCheck {
  const float* depth;
  int H, W;
  const long long* pixel;
  float edge;
};

struct FieldArgs {
  Grid g;
  const float* grid;
  const uint16_t* grid_bf16;   // non-null: BF16 decoders and gathers from this mirror
  const float* mlp;
  // ray samples
  const float* o;
  const float* r;
  const float* t;
  const int* ray_of;
  int total;
  // smoothness pairs
  const float* xs;
  const float* eps;
  int S;
  // forward outputs
  float* out4;            // [total][4] phi, c
  float* eik;             // [total] (1 - |grad phi|)^2
  float* smooth_partial;  // [gridDim.x]
  float* grad_phi;        // [total + 2 S][3] d(phi)/dx (forward, optional; total = the capacity)
  float* pair_terms;      // [S] per-pair smoothness value (forward, optional)
  // backward
  const float* seed4;     // [total][4] dL/dphi, dL/dc (scaled)
  const float* posw;      // [total][4]: sample position (as the forward computed it), Eikonal
                          // weight (scaled, 0 outside S_fs)
  float smooth_coef;      // 2 * lambda_smooth * loss_scale / S
  float* grad_grid;       // [V][4]
  float* mlp_partial;     // [gridDim.x][kMlpNumel]
  int need_gx;            // ray mode: compute grad phi for the Eikonal term
  const float* depth;     // forward, optional: [M] observed depth per ray; with it, wave-tiles
                          // with no sample in S_fs = {D - t > trunc} skip grad phi
  float trunc;
  float* grad_x;          // backward, optional: [total][4] dL/dx of each sample (x, y, z, 0)
  int colour;             // ray mode: 1 = colour from the geometry decoder's features; 0 = no colour
                          // here (the paper's colour path runs in its own kernel)
  const int* seg_end;     // ray mode: device copy of the sample count (seg[M]); total is then a capacity
  // levels whose gradient is accumulated in LDS per block (bit l) and the
  // float offset of each such level inside the block's LDS area
  int priv_mask;
  int priv_off[4];
  int priv_floats;        // floats of the LDS area
  float* priv_partial;    // [gridDim.x][priv_floats] block partials
  // gradient copies (optional): the levels not accumulated in LDS scatter into
  // four x/y-parity copies instead of grad_grid; copy_base[l] is the float
  // offset of level l's four copies in `copies` (-1: no copies)
  float* copies;
  int copy_base[4];
};

// the paper's colour path (colour grid at the finest level + view direction)
struct ColourArgs {
  Grid g;
  const float* cgrid;     // [V_finest][8]: 6 features, 2 unused
  const float* cmlp;      // packed V1 e1 V2 e2 V3 e3
  const float* o;
  const float* r;
  const float* t;
  const int* ray_of;
  int total;
  const int* seg_end;     // device copy of the sample count (seg[M]); total is then a capacity
  float* out4;            // forward: colour into components 1..3 of [total][4]
  const float* seed4;     // backward: [total][4] seeds (components 1..3: dL/dc, scaled)
  const float* posw;      // backward: [total][4] sample positions
  float* grad_cgrid;      // backward: [V_finest][8]
  float* partial;         // backward: [gridDim.x][colour decoder size] block partials
};

struct RenderArgs {
  Grid g;
  const float* o;
  const float* r;
  const float* rgb;
  const float* depth;
  const float* t;
  const int* seg;
  int M;
  int total;            // sample capacity of the batch
  const float* mlp;
  const float* out4;    // [total][4]
  const float* eik;     // [total] or null
  float trunc, alpha_fs;
  float lam[6];
  int depth_mid;        // d_hat attributes w_i to (t_i + t_i+1) / 2 instead of t_i
  // forward outputs
  float* rgb_hat;
  float* depth_hat;
  float* wsum;
  float* weights;       // or null
  float* ray_partial;   // [M][8]
  // backward
  const float* n_depth_rays;  // device scalar (losses[7])
  float loss_scale;
  float* seed4;         // [total][4]
  float* posw;          // [total][4]: sample position, Eikonal weight
  float* ray_dv;        // [M]
};

// proposal network over a set of rays
struct PropArgs {
  Grid g;
  const float* grid;
  const float* prop;     // packed proposal parameters
  const float* o;
  const float* r;
  int M;
  int span_mode;
  float near_t, far_t;
  float* out3;           // [M][3] near, far, confidence (or null)
  const float* tgt;      // [M][3] training targets
  float beta;            // smooth-L1 transition
  float cover_tol;       // confidence label: interval covers the target within this
  float* grad_partial;   // [gridDim.x][numel + 1] (last entry: loss)
};

// training targets from logged per-sample weights
struct TargetArgs {
  Grid g;
  const float* t;
  const float* w;
  const int* seg;
  const float* o;
  const float* r;
  int M;
  int span_mode;
  float near_t, far_t;
  float widen, q_lo, q_hi, conf_min;
  float* tgt;            // [M][3]
};

struct SampleArgs {
  Grid g;
  const uint8_t* rgb;
  const float* depth;
  const float* c2w;
  int T, H, W;
  float fx, fy, cx, cy;
  int M, n_strat, n_near, span_mode;
  float near_t, far_t, trunc;
  int S;
  float delta_s;
  uint32_t k0, k1, step;
  float* o;
  float* r;
  float* rgb_out;
  float* depth_out;
  float* t;
  int* seg;
  int* ray_of;
  float* xs;
  float* eps;
  long long* pixel;
  // proposal-driven sampling: per-ray (near, far, confidence); rays with
  // confidence >= conf_thr get n_free samples on [t_lo, near] and n_prop in
  // [near, far], the others the plain n_strat + n_near; seg is then filled
  // beforehand by the scan
  const float* prop3;
  float conf_thr;
  int n_prop;
  int n_free;
};


// Hierarchical importance sampling: one step (new depths from the current
// samples of every ray, all rays with n samples) and the merge of the new
// depths into the sorted lists.
constexpr int kImpMaxAdd = 64;   // samples added per ray and step
struct ImpArgs {
  Grid g;
  const float* o;
  const float* r;
  const float* t;        // [M][n] sorted
  const float* phi;      // SDF of sample i at phi[i * phi_stride]
  int phi_stride;
  const float* mlp;      // sharpness s = exp(10 v)
  int M, n, n_add;
  float eps;             // added to every interval weight
  uint32_t k0, k1, iteration, stream;   // Philox key and counter words
  float* t_new;          // [M][n_add]
  int* ray_of_new;       // [M][n_add] or null
};
struct ImpMergeArgs {
  const float* ta;       // [M][na] sorted
  const float* pa;       // value carried with ta: pa[i * pa_stride]
  int pa_stride, na;
  const float* tb;       // [M][nb]
  const float* pb;
  int pb_stride, nb;
  int M;
  float* t_out;          // [M][na + nb]
  float* p_out;          // or null
  int* ray_of_out;       // or null
  int* seg_out;          // [M + 1] or null
};

// Surface extraction: lattice rows as rays for the forward field kernel, and
// marching tetrahedra over the SDF lattice.
struct LatticeArgs {
  float p0[3];
  float h;
  int nx, ny, k0, layers;   // a slab of `layers` z-layers starting at k0
  float* t;                 // [nx * ny * layers]
  int* ray_of;              // [nx * ny * layers]
  float* o;                 // [ny * layers][3]
  float* r;                 // [ny * layers][3]
};
struct MtArgs {
  const float* phi;         // [nz][ny][nx]
  float p0[3];
  float h;
  int nx, ny, nz;
  float* tris;              // [max_tris][3][3]
  long long max_tris;
  unsigned* count;          // triangles found (may exceed max_tris)
};

}  // namespace gs
