/*
 * gosurf.h - C ABI of the GO-Surf optimisation hot path for MI355X (gfx950).
 *
 * One optimisation iteration of GO-Surf (Wang, Bleja, Agapito 2022) over a
 * dense multi-level feature grid is four asynchronous calls on one HIP stream:
 *
 *   gosurf_sample_rays  rays from all pixels of all frames and the points along
 *                       them (Sec. 3.2 "Depth and Color Rendering", Sec. 3.5),
 *                       plus the smoothness points and perturbations (Sec. 3.4)
 *   gosurf_forward      grid interpolation (Sec. 3.1, Eq. SDF_MLP), decoders,
 *                       volume rendering (Eqs. volume_rendering,
 *                       volume_rendering_alpha) and the six loss terms with
 *                       their weighted total (Sec. 3.3-3.5)
 *   gosurf_backward     exact gradients of that total with respect to every
 *                       grid feature and decoder parameter, including the
 *                       second-order grid-sampler blocks that the Eikonal and
 *                       smoothness terms need (supplementary "Second-order Grid
 *                       Sampler", Eqs. second_sdf_grad_theta, second_sdf_grad_omega)
 *   gosurf_adam_step    Adam over all parameters (implementation details);
 *                       gosurf_adam_step_checked skips a step whose
 *                       gradients hold an inf or NaN
 *
 * A precision variant runs the decoders in bfloat16 on the matrix cores with
 * float32 accumulation and reads grid features from a bfloat16 mirror of the
 * float32 master table (GOSURF_BF16); rendering, losses, gradient
 * accumulation and Adam stay float32.
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array pointers are DEVICE pointers to caller-owned memory, contiguous,
 *   row-major, float32 unless stated.  The library allocates nothing on these
 *   paths; scratch memory is a caller-supplied workspace sized by
 *   gosurf_workspace_bytes().
 * - Every call only validates its arguments on the host and enqueues kernels
 *   on `stream` (a hipStream_t; NULL = the default stream).  It returns
 *   GOSURF_OK or an error status and never blocks.  Device faults surface at
 *   the caller's next synchronisation.  On error nothing has been enqueued
 *   and gosurf_last_error() (thread-local) describes the problem.
 * - No C++ exception crosses this interface.  Calls are re-entrant; calls that
 *   share output or workspace buffers must be ordered by the caller.
 *
 * Grid layout (Sec. 3.1; readings stated where the paper is silent)
 * -----------------------------------------------------------------
 * GOSURF_LEVELS = 4 levels, coarsest first (z = [V^0 .. V^3]), 4 features per
 * vertex (h_g = 4).  All levels share the box [p0, p1].  Level l has voxel
 * edge voxel[l] and dims[l] = (nx, ny, nz) vertices; vertex (i, j, k) of level
 * l is row offset[l] + (k*ny + j)*nx + i of the concatenated float32 table
 * grid[n_vertices][4] (16-byte aligned).  Interpolation uses the eight
 * vertices of the cell with origin clamp(floor((x - p0)/voxel), 0, n - 2) and
 * the supplementary's coefficient vector (bit order theta_xyz).  A point
 * outside [p0, p1] (decided in float32 on o + t*r, product and sum rounded
 * separately) is masked: it has no SDF, the opacities of both intervals that
 * touch it are 0 and it receives no loss and no gradient.
 *
 * Decoder parameters: one float32 vector of GOSURF_MLP_NUMEL entries, each
 * matrix row-major [out][in]:
 *   W1[32][16] b1[32] W2[32][32] b2[32] W3[16][32] b3[16]    geometry 16-32-32-16
 *   U1[32][15] c1[32] U2[3][32] c2[3]                        colour   15-32-3
 *   v[1]                                                     sharpness s = exp(10 v)
 * Hidden layers use ReLU (derivative 0 at 0); output 0 of the geometry decoder
 * is the SDF, outputs 1..15 feed the colour decoder, whose output is a sigmoid.
 */
#ifndef GOSURF_H
#define GOSURF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GOSURF_LEVELS 4
#define GOSURF_FEAT 4
#define GOSURF_MLP_NUMEL 2740
#define GOSURF_MAX_SAMPLES_PER_RAY 256
#define GOSURF_N_LOSSES 8
#define GOSURF_PROPOSAL_NUMEL 6851
#define GOSURF_STATIC_MAX_RAYS 65536
#define GOSURF_COLOUR_FEAT 6
#define GOSURF_COLOUR_MLP_NUMEL 1475

typedef enum {
  GOSURF_OK = 0,
  GOSURF_ERR_NULL = 1,       /* a required pointer is NULL */
  GOSURF_ERR_SHAPE = 2,      /* a size is out of range or inconsistent */
  GOSURF_ERR_ALIGN = 3,      /* a pointer is not suitably aligned */
  GOSURF_ERR_VALUE = 4,      /* a scalar argument is invalid (NaN, <= 0, ...) */
  GOSURF_ERR_WORKSPACE = 5,  /* workspace missing or smaller than required */
  GOSURF_ERR_HIP = 6,        /* a kernel launch failed */
  GOSURF_ERR_NONFINITE = 7   /* reserved (no call returns it: gosurf_adam_step_checked reports through its flag) */
} gosurf_status;

typedef enum { GOSURF_FP32 = 0, GOSURF_BF16 = 1 } gosurf_precision;
typedef enum { GOSURF_SPAN_FIXED = 0, GOSURF_SPAN_BOX = 1 } gosurf_span_mode;
/* Where colour comes from.  DECODED: from the geometry decoder's outputs
   1..15 through the colour decoder 15-32-3 (the layout below).  GRID: the
   paper's path (Sec. 3.1, Eq. COLOR_MLP and the architecture details): a
   colour grid W_beta of GOSURF_COLOUR_FEAT features per vertex of the finest
   level, stored float32 [V_finest][8] (features 0..5, then two entries that
   are never read), trilinearly interpolated at the sample and decoded with
   the viewing direction d = r / |r| by g_gamma: (6 + 3) -> 32 -> 32 -> 3,
   ReLU hidden, sigmoid output, packed V1[32][9] e1[32] V2[32][32] e2[32]
   V3[3][32] e3[3] (GOSURF_COLOUR_MLP_NUMEL; inputs: the 6 features, then
   d).  On the GRID path the geometry decoder's outputs 1..15 and the
   DECODED colour decoder's parameters feed nothing (zero gradient).  GRID
   needs precision GOSURF_FP32. */
typedef enum { GOSURF_COLOUR_DECODED = 0, GOSURF_COLOUR_GRID = 1 } gosurf_colour_mode;

/* Geometry of the grid (see "Grid layout" above). */
typedef struct {
  float p0[3];                        /* box minimum (world units, metres) */
  float p1[3];                        /* box maximum */
  float voxel[GOSURF_LEVELS];         /* voxel edge per level, coarsest first */
  int32_t dims[GOSURF_LEVELS][3];     /* (nx, ny, nz) per level, each >= 2 */
  int64_t offset[GOSURF_LEVELS];      /* first vertex row of each level */
  int64_t n_vertices;                 /* rows of the concatenated table */
  int32_t precision;                  /* gosurf_precision of decoders and grid reads */
  int32_t colour_mode;                /* gosurf_colour_mode */
  int32_t grad_copies;                /* 0: the backward scatters into grads->grid; 1: it scatters the
                                         levels it does not accumulate on chip into four gradient copies
                                         in the workspace and adds them into grads->grid before it
                                         returns (see gosurf_backward) */
} gosurf_model;

/* Parameters read by forward/backward. */
typedef struct {
  const float* grid;          /* [n_vertices][4] float32 master features */
  const uint16_t* grid_bf16;  /* [n_vertices][4] bfloat16 mirror; required for GOSURF_BF16 */
  const float* mlp;           /* [GOSURF_MLP_NUMEL] decoder parameters and v */
  const float* colour_grid;   /* GOSURF_COLOUR_GRID: [V_finest][8], 16-byte aligned; else unused */
  const float* colour_mlp;    /* GOSURF_COLOUR_GRID: [GOSURF_COLOUR_MLP_NUMEL]; else unused */
} gosurf_params;

/* An RGB-D sequence {I_t, D_t} with camera-to-world poses (Sec. 3, first para.). */
typedef struct {
  const uint8_t* rgb;   /* [T][H][W][3] */
  const float* depth;   /* [T][H][W], z-depth in metres, <= 0 means missing */
  const float* c2w;     /* [T][4][4] camera-to-world, OpenCV camera axes */
  int32_t T, H, W;
  float fx, fy, cx, cy; /* pinhole intrinsics; pixel (u, v) looks along
                           R [(u + .5 - cx)/fx, (v + .5 - cy)/fy, 1] */
} gosurf_frames;

/* How a batch is drawn.  Every random number is Philox4x32-10 keyed by `seed`
   with counter (index, step, stream, block): stream 0 picks the pixel
   (floor(u32 * T*H*W / 2^32)), 1 the stratified jitter, 2 the near-depth
   jitter, 3 the smoothness points; u = (u32 >> 8) * 2^-24. */
typedef struct {
  int32_t M;            /* rays, >= 1 */
  int32_t n_strat;      /* stratified samples per ray over the span, >= 1 */
  int32_t n_near;       /* extra samples on [D - trunc, D + trunc] for rays with depth */
  int32_t span_mode;    /* GOSURF_SPAN_FIXED: [near, far]; GOSURF_SPAN_BOX: the
                           ray's passage through the grid box, clipped to [near, far] */
  float near_t, far_t;  /* span limits (ray parameter = camera z-depth) */
  float trunc;          /* truncation t of the SDF terms (metres) */
  int32_t S;            /* smoothness pairs, >= 0 */
  float delta_s;        /* perturbation length (metres) */
  uint64_t seed;
  uint32_t step;
  /* Learned proposal (optional).  With proposal != NULL each ray first gets
     (near, far, confidence) from the proposal network (see
     gosurf_proposal_forward); rays with confidence >= conf_threshold get
     n_free stratified samples on [t_lo, near] (the span before the interval,
     near-depth jitter stream) followed by n_proposal stratified samples in
     [near, far] (stratified stream); the others fall back to the plain
     n_strat + n_near samples.  Rays then have different lengths. */
  const float* proposal;   /* [GOSURF_PROPOSAL_NUMEL] network parameters, or NULL */
  const float* grid;       /* float32 grid features read by the proposal (its level 1) */
  int32_t n_proposal;      /* interval samples per confident ray (>= 1) */
  float conf_threshold;
  int32_t n_free;          /* free-space samples per confident ray before its interval (>= 0) */
  int32_t depth_check;     /* nonzero: a confident ray with observed depth D > 0 and D outside
                              [near, far] has its interval extended to reach D if D lies within
                              depth_extend of it, and falls back to plain samples otherwise
                              (needs conf_threshold > 0) */
  float depth_extend;      /* metres, >= 0 */
  float depth_edge;        /* with depth_check, metres (0: off): a confident ray whose pixel has a
                              4-neighbour in its frame with valid depth differing from D by more
                              than depth_edge (a depth discontinuity, e.g. a silhouette) falls back
                              to plain samples (needs out->pixel) */
} gosurf_sample_cfg;

/* A ray batch.  Written by gosurf_sample_rays, read by forward/backward.
   Samples are stored ray-major: the samples of ray m are
   t[seg[m] .. seg[m+1]-1], sorted ascending, at most
   GOSURF_MAX_SAMPLES_PER_RAY per ray (a longer ray is cut to that many by
   forward and backward); ray_of[s] is the ray of sample s. */
typedef struct {
  int32_t M;            /* rays, >= 1 (an empty batch is rejected with GOSURF_ERR_SHAPE) */
  int32_t total;        /* samples, = seg[M], M <= total < 2^29 (else GOSURF_ERR_SHAPE); with
                           a proposal the capacity (seg[M], on the device, is then the
                           actual count) */
  int32_t S;            /* smoothness pairs */
  float* o;             /* [M][3] ray origin (camera centre) */
  float* r;             /* [M][3] ray direction (camera-z component 1) */
  float* rgb;           /* [M][3] observed colour in [0, 1] */
  float* depth;         /* [M] observed depth, 0 = missing */
  float* t;             /* [total] sample depths along the ray */
  int32_t* seg;         /* [M + 1] CSR offsets */
  int32_t* ray_of;      /* [total] */
  float* xs;            /* [S][3] smoothness points */
  float* eps;           /* [S][3] perturbations; the pair is (x, x + eps rounded to float32) */
  int64_t* pixel;       /* [M] flat pixel index of each ray (output only; may be NULL) */
  float* prop;          /* [M][3] proposal near, far, confidence (written with a proposal; the
                           confidence is negated where the depth check rejected the interval) */
} gosurf_ray_batch;

/* Loss configuration (Sec. 3.3-3.5 and implementation details). */
typedef struct {
  float lambda[6];      /* weights of rgb, depth, sdf, free-space, Eikonal, smoothness */
  float trunc;          /* truncation t: S_tr = {|D - d| <= t}, S_fs = {D - d > t} */
  float alpha_fs;       /* exponent of the free-space term (5) */
  int32_t depth_midpoint; /* 0: d_hat = sum w_i t_i (Eq. volume_rendering; w_i belongs to the interval
                             [t_i, t_i+1], so a sharp surface renders about half a spacing short);
                             1: d_hat = sum w_i (t_i + t_i+1) / 2 (unbiased for any spacing) */
} gosurf_loss_cfg;

/* Forward outputs.  losses[] = {L_rgb, L_d, L_sdf, L_fs, L_eik, L_smooth,
   weighted total, number of rays with valid depth}.  `saved` holds what the
   backward needs and must be passed to it unchanged. */
typedef struct {
  float* rgb_hat;       /* [M][3] rendered colour */
  float* depth_hat;     /* [M] rendered depth */
  float* wsum;          /* [M] sum of the ray's weights */
  float* losses;        /* [GOSURF_N_LOSSES] */
  float* saved;         /* [total][4]: phi, colour per sample; then [total] eik residual */
  float* weights;       /* [total] per-sample weights w_i, or NULL */
  float* grad_phi;      /* [total + 2 S][3] d(phi)/dx, or NULL (inspection output): row s < total
                           for sample s (written when the Eikonal weight is nonzero), rows
                           total + 2p and total + 2p + 1 for the points x and x + eps of
                           smoothness pair p (written when the smoothness weight is nonzero) */
  float* ray_terms;     /* [M][8] per-ray terms, or NULL (inspection output): the channel-mean
                           |I - c_hat|, |D - d_hat| (0 without depth), the means of |phi - b| over
                           S_tr, of the free-space term and of the Eikonal residual over S_fs,
                           1 if the ray has depth, then two zeros */
  float* pair_terms;    /* [S] |grad phi(x) - grad phi(x + eps)|^2 per smoothness pair (0 for a
                           pair leaving the box), or NULL; written when the smoothness weight
                           is nonzero */
} gosurf_fwd_out;

/* Gradient accumulators (caller zeroes them once; Adam re-zeroes them). */
typedef struct {
  float* grid;          /* [n_vertices][4] */
  float* mlp;           /* [GOSURF_MLP_NUMEL] */
  float* ray_o;         /* [M][3] dL/d(ray origin), or NULL (camera pose refinement; with ray_r) */
  float* ray_r;         /* [M][3] dL/d(ray direction), or NULL */
  float* colour_grid;   /* GOSURF_COLOUR_GRID: [V_finest][8] (entries 6, 7 untouched); else unused */
  float* colour_mlp;    /* GOSURF_COLOUR_GRID: [GOSURF_COLOUR_MLP_NUMEL]; else unused */
} gosurf_grads;

typedef struct {
  float lr_grid;        /* 1e-2 in the paper */
  float lr_mlp;         /* 1e-3 in the paper (decoders and v) */
  float beta1, beta2, eps;
  int32_t step;         /* 1-based Adam step */
  float inv_loss_scale; /* gradients are multiplied by this before use */
} gosurf_adam_cfg;

/* Parameters, gradients and Adam moments of both groups (a group with 0
   entries may pass NULL pointers). */
typedef struct {
  float* grid; float* grid_grad; float* grid_m; float* grid_v;
  uint16_t* grid_bf16;  /* refreshed bfloat16 mirror of grid, or NULL */
  int64_t grid_numel;   /* multiple of 4 */
  float* mlp; float* mlp_grad; float* mlp_m; float* mlp_v;
  int32_t mlp_numel;    /* any size (e.g. the decoders' 2740 or the proposal's 6851) */
} gosurf_adam_state;

/* Kernels that can be timed individually (see gosurf_time_kernel). */
typedef enum {
  GOSURF_KERNEL_NONE = 0,
  GOSURF_KERNEL_FIELD_FWD = 1,     /* forward field kernel of gosurf_forward (samples and smoothness pairs) */
  GOSURF_KERNEL_FIELD_BWD = 2,     /* backward field kernel of gosurf_backward (samples and smoothness pairs) */
  GOSURF_KERNEL_ADAM = 4           /* the dense Adam kernel of gosurf_adam_step */
} gosurf_kernel_id;

/* Measurement hook (this thread only): the next launch of `kernel` is
   bracketed by hipEventRecord(start) and hipEventRecord(stop) on the launch
   stream, after which the hook clears itself; start/stop are caller-created
   hipEvent_t handles.  kernel = GOSURF_KERNEL_NONE (or NULL events) clears
   it.  Errors: VALUE. */
gosurf_status gosurf_time_kernel(int32_t kernel, void* start_event, void* stop_event);

/* Thread-local description of the last error on this thread ("" if none). */
const char* gosurf_last_error(void);

/* Sample capacity of a batch drawn with `cfg`: M * (n_strat + n_near), or
   M * max(n_strat + n_near, n_free + n_proposal) with a proposal (the actual count is
   then seg[M], on the device). */
int64_t gosurf_batch_samples(const gosurf_sample_cfg* cfg);

/* Draw a ray batch (Sec. 3.2, 3.4, 3.5).  `out` arrays must be sized for
   cfg->M rays, gosurf_batch_samples(cfg) samples and cfg->S pairs; out->M,
   out->total and out->S are set by the caller to those sizes.  Pixels are
   drawn uniformly from all pixels of all frames, including those without
   depth.  Rays with depth get n_strat stratified samples over the span and
   n_near stratified samples on [D - trunc, D + trunc], merged in order
   (stratified first on ties); rays without depth get n_strat + n_near
   stratified samples.  A smoothness point tries up to 8 pixels and keeps the
   first with depth, at depth D + (2u - 1) trunc along its ray; eps is delta_s
   times a uniform unit vector; with no valid pixel the point is the box
   centre with eps = 0.  With a proposal (see gosurf_sample_cfg) the rays are
   drawn first, the proposal runs on them, the depth check and the segment
   offsets follow on the device, and then each ray's samples are written.
   Errors: NULL, SHAPE (sizes, T*H*W >= 2^32), VALUE. */
gosurf_status gosurf_sample_rays(const gosurf_model* model, const gosurf_frames* frames,
                                 const gosurf_sample_cfg* cfg, gosurf_ray_batch* out,
                                 void* stream);

/* Workspace bytes needed by forward/backward for a batch of these sizes.  With
   model->grad_copies = 1 this includes the gradient copies, about 64 bytes
   per vertex of every level the backward does not accumulate on chip (levels
   are accumulated on chip, coarsest first, while their vertices add up to at
   most 1024).
   Returns 0 for negative sizes or a model the copies cannot serve. */
size_t gosurf_workspace_bytes(const gosurf_model* model, int32_t M, int32_t total, int32_t S);

/* Hierarchical importance sampling (Sec. 3.2, last paragraph: starting from
   the coarse samples, each step adds n_add samples per ray drawn from the
   weights of Eq. volume_rendering computed with the samples so far; the
   implementation details use 96 coarse samples and 3 steps of 12).
   One step: interval i = [t_i, t_{i+1}] of a ray gets probability
   proportional to w_i + weight_eps, with w_i = T_i alpha_i (Eq.
   volume_rendering_alpha at the model's sharpness s = exp(10 v); an interval
   touching a sample outside the grid box has alpha = 0), uniform within the
   interval; the draws are u_j = (j + xi_j) / n_add, xi_j from Philox4x32-10
   keyed by seed with counter (ray, step, 8 + step index, j / 4), word j % 4;
   the new samples are merged into the ray's sorted list, existing samples
   first on ties. */
typedef struct {
  int32_t steps;       /* importance steps, 1..8 (3 in the paper) */
  int32_t n_add;       /* samples added per ray and step, 1..64 (12 in the paper) */
  float weight_eps;    /* added to every interval weight, > 0 (1e-5) */
  uint64_t seed;       /* Philox key */
  int64_t step;        /* iteration number (Philox counter word, low 32 bits) */
} gosurf_importance_cfg;

/* Workspace bytes for gosurf_importance_sample on M rays with n_coarse
   samples each. */
size_t gosurf_importance_workspace_bytes(int32_t M, int32_t n_coarse, const gosurf_importance_cfg* cfg);

/* The full sampler: the SDF of the coarse samples (the forward field kernel,
   at the model's precision), then `steps` times one importance step, the SDF
   at the new samples and the merge.  `coarse` must hold the same number n0 of
   sorted samples on every ray (a batch of gosurf_sample_rays without a
   proposal: total = M * n0).  Writes out->t [M * nf], out->seg [M + 1] and
   out->ray_of [M * nf] with nf = n0 + steps * n_add <=
   GOSURF_MAX_SAMPLES_PER_RAY; out->M must be M and out->total M * nf; the
   other arrays of `out` are not touched (point them at the coarse batch's).
   Errors: NULL, SHAPE, VALUE, WORKSPACE, HIP. */
gosurf_status gosurf_importance_sample(const gosurf_model* model, const gosurf_params* params,
                                       const gosurf_ray_batch* coarse, const gosurf_importance_cfg* cfg,
                                       gosurf_ray_batch* out, void* workspace, size_t workspace_bytes,
                                       void* stream);

/* One importance step on given SDF values: rays->t holds n = total / M sorted
   samples per ray (n >= 2, total = M * n), phi [total] their SDF values, and
   step_index selects the Philox stream; writes t_new [M * n_add], each ray's
   new samples in draw order (u_j increasing).  Errors: NULL, SHAPE, VALUE, HIP. */
gosurf_status gosurf_importance_step(const gosurf_model* model, const float* mlp, const gosurf_ray_batch* rays,
                                     const float* phi, const gosurf_importance_cfg* cfg, int32_t step_index,
                                     float* t_new, void* stream);

/* Forward pass and loss (Sec. 3.1-3.5).  Per-ray opacities
   alpha_i = max(1 - Phi_s(phi_{i+1}) / Phi_s(phi_i), 0), alpha_last = 0,
   w_i = T_i alpha_i; colour/depth = sum w_i c_i / sum w_i t_i.  Loss terms:
   L_rgb = mean over rays of the channel-mean |I - c_hat|; L_d = mean over rays
   with depth of |D - d_hat|; L_sdf, L_fs, L_eik = (1/M) sum over rays of the
   per-ray mean over S_tr / S_fs (empty: 0) of |phi - b|,
   max(0, e^{-alpha phi} - 1, phi - b), (1 - |grad phi|)^2 with b = D - t; only
   rays with depth have S_tr and S_fs, and membership is decided in float32;
   L_smooth = (1/S) sum over pairs of |grad phi(x) - grad phi(x + eps)|^2
   (a pair leaving the box contributes 0).  The Eikonal and smoothness terms
   are not evaluated, and reported as 0, when their weight lambda is 0.
   Errors: NULL, SHAPE, VALUE, WORKSPACE, HIP. */
gosurf_status gosurf_forward(const gosurf_model* model, const gosurf_params* params,
                             const gosurf_ray_batch* batch, const gosurf_loss_cfg* loss,
                             gosurf_fwd_out* out, void* workspace, size_t workspace_bytes,
                             void* stream);

/* gosurf_forward for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
   the same computation and outputs, with the workspace replaced by a scratch
   array that the library holds on each GPU it runs on until the process
   ends (2.1 MB: sized for GOSURF_STATIC_MAX_RAYS rays).  The caller still
   passes every input and output; nothing is allocated and no workspace
   argument is taken.  Every call on a GPU uses that GPU's one scratch array,
   so calls whose work overlaps on one GPU (other threads, other streams)
   race and must be ordered by the caller; each call writes every scratch
   entry it reads, so nothing carries over between calls.  The first call on
   a device looks up the array's device address (device to be current).
   Errors: as gosurf_forward; SHAPE if M > GOSURF_STATIC_MAX_RAYS. */
gosurf_status gosurf_forward_static(const gosurf_model* model, const gosurf_params* params,
                                    const gosurf_ray_batch* batch, const gosurf_loss_cfg* loss,
                                    gosurf_fwd_out* out, void* stream);

/* Backward pass: ADDS loss_scale * d(total)/d(params) into grads (loss_scale
   any finite value: a negative one gives the gradient of -scale * total, 0
   adds zeros).  Must follow the gosurf_forward call that produced `fwd` with
   the same params, batch, loss config and workspace.  Grid gradients are
   accumulated with float32 atomics (summation order varies between runs);
   decoder gradients are reduced in a fixed order.  With grads.ray_o and
   grads.ray_r, the derivatives of the same scaled total with respect to each
   ray's origin and direction are ADDED there too (sample points o + t r; the
   Eikonal term contributes through the second derivatives of the
   interpolation, supplementary Eq. second_sdf_grad_x).  A ray holding more than
   GOSURF_MAX_SAMPLES_PER_RAY samples ends at that many: forward and backward
   treat it as the ray of its first GOSURF_MAX_SAMPLES_PER_RAY samples (the
   rest get weight 0, no loss and no gradient).  Device offsets seg[] beyond
   `total` are clamped to it.
   Gradient copies (model->grad_copies = 1): grid-gradient atomics are
   processed per aligned 64-byte chunk, and in the grid layout a sample's eight
   corners span about five.  With copies, the levels not accumulated on chip
   are scattered into four copies held in the workspace, one per parity of the
   cell's (x, y) index, laid out so a cell's four corners at one z are one
   aligned 64-byte unit (two chunks per sample and level).  The backward zeroes
   the copies first and adds them into grads->grid before it returns, so the
   result is the same gradient up to the order of float32 additions.  It needs
   each such level to have at most 2048 x 2048 x 512 vertices and all copies
   to fit 2^31 floats (else VALUE).
   Errors: NULL, SHAPE, VALUE, WORKSPACE, HIP. */
gosurf_status gosurf_backward(const gosurf_model* model, const gosurf_params* params,
                              const gosurf_ray_batch* batch, const gosurf_loss_cfg* loss,
                              const gosurf_fwd_out* fwd, float loss_scale, gosurf_grads* grads,
                              void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Camera pose refinement (Sec. 3, first paragraph, and Sec. 3.5: the poses are
 * optimised with the grids and decoders; the implementation details give a
 * pose as a translation t and a rotation nu in so(3), learning rate 5e-4).
 * Each frame carries a correction pose[t] = (tau, nu) (float32 [T][6], zero
 * at the start) of its initial camera-to-world pose: R = Exp(nu) R0 and
 * c = c0 + tau, Exp the exponential map of so(3).  One step with refinement:
 * gosurf_pose_apply, gosurf_sample_rays on the refined poses (with
 * out.pixel), gosurf_forward, gosurf_backward with grads.ray_o/ray_r,
 * gosurf_pose_backward, and gosurf_adam_step on the pose group.  The
 * smoothness points are inputs of the step and carry no pose gradient.
 * ------------------------------------------------------------------------- */

/* c2w[t] = [Exp(nu_t) R0_t | c0_t + tau_t; 0 0 0 1] for t < T (row-major
   [T][4][4], last row copied from c2w0).  Errors: NULL, SHAPE, HIP. */
gosurf_status gosurf_pose_apply(const float* c2w0, const float* pose, int32_t T, float* c2w, void* stream);

/* ADDS the pose gradient of the rays of a batch to grad_pose [T][6]: ray m of
   frame f = pixel[m] / HW (pixel as written by gosurf_sample_rays; rays whose
   index names no frame below T are skipped) contributes dL/do to
   grad_pose[f][0..2] and J_l(nu_f)^T (r_m x dL/dr) to grad_pose[f][3..5],
   J_l the left Jacobian of SO(3).  r [M][3] are the batch's ray directions,
   grad_o and grad_r [M][3] what gosurf_backward accumulated in grads.ray_o
   and grads.ray_r.  Float32 atomics: the summation order varies.
   Errors: NULL, SHAPE, HIP. */
gosurf_status gosurf_pose_backward(const float* pose, int32_t T, const int64_t* pixel, int64_t HW, const float* r,
                                   const float* grad_o, const float* grad_r, int32_t M, float* grad_pose,
                                   void* stream);

/* ---------------------------------------------------------------------------
 * Learned proposal sampler.  Not part of the paper: a small network trained
 * on the per-ray weight distributions that plain sampling produces, which
 * predicts a narrow depth interval per ray.  Input (38): the 4 features of
 * grid level 1 at the 8 bin centres t_lo + (b + 1/2)(t_hi - t_lo)/8 of the
 * ray's span (0 outside the box), then o and r.  Network 38-64-64-3 (ReLU),
 * parameters packed P1[64][38] q1[64] P2[64][64] q2[64] P3[3][64] q3[3].
 * near = t_lo + (t_hi - t_lo) sigmoid(o0); far = near + (t_hi - near)
 * sigmoid(o1); confidence = sigmoid(o2).  The span [t_lo, t_hi] is the plain
 * sampler's (span_mode, near_t, far_t of `span`).
 * ------------------------------------------------------------------------- */

/* out3[M][3] = (near, far, confidence) for the rays of `rays` (uses M, o, r). */
gosurf_status gosurf_proposal_forward(const gosurf_model* model, const float* grid, const float* proposal,
                                      const gosurf_ray_batch* rays, const gosurf_sample_cfg* span, float* out3,
                                      void* stream);

/* Training targets from a logged plain batch and its forward weights: per ray
   p_i = w_i / sum w; the 0.5 % and 99.5 % first crossings of the piecewise-
   linear CDF through (t_0, p_0), (t_1, p_0 + p_1), ..., widened by `widen`
   and clipped to the span; confidence target = [sum w >= 0.5].
   targets[M][3] = (near*, far*, conf*). */
gosurf_status gosurf_proposal_targets(const gosurf_model* model, const gosurf_ray_batch* rays,
                                      const gosurf_sample_cfg* span, const float* weights, float widen,
                                      float* targets, void* stream);

size_t gosurf_proposal_workspace_bytes(int32_t M);

/* Mean over rays of conf* (smoothL1(near - near*) + smoothL1(far - far*)) +
   BCE(confidence, k) (smooth-L1 transition `beta`), with the confidence label
   k = conf* [near <= near* + cover_tol] [far >= far* - cover_tol] (the current
   interval covers the target one; a decision, not differentiated).  *loss is
   set to it and its gradient is ADDED to grad[GOSURF_PROPOSAL_NUMEL]
   (fixed-order sums).  The grid is not differentiated. */
gosurf_status gosurf_proposal_backward(const gosurf_model* model, const float* grid, const float* proposal,
                                       const gosurf_ray_batch* rays, const gosurf_sample_cfg* span,
                                       const float* targets, float beta, float cover_tol, float* grad,
                                       float* loss, void* workspace, size_t workspace_bytes, void* stream);

/* Surface extraction (evaluation, not part of an optimisation step).  The
   reconstructed surface is the zero level set of phi (Sec. 3.1); the paper
   meshes it on a 1 cm lattice.

   The SDF on the lattice p0 + h (i, j, k), i < nx, j < ny, k < nz, stored in
   phi [nz][ny][nx] (x fastest), evaluated by the forward field kernel at the
   model's precision (lattice point x = p0 + i h rounded as float32 i*h + p0).
   Points outside the grid box get the decoder's value at zero features.  The
   lattice is processed in z-slabs as large as the workspace allows
   (gosurf_lattice_workspace_bytes(nx, ny, layers) bytes hold `layers`
   z-layers; at least one layer is needed).
   Errors: NULL, SHAPE, VALUE, WORKSPACE, HIP. */
size_t gosurf_lattice_workspace_bytes(int32_t nx, int32_t ny, int32_t layers);
gosurf_status gosurf_sdf_lattice(const gosurf_model* model, const gosurf_params* params, const float p0[3],
                                 float h, int32_t nx, int32_t ny, int32_t nz, float* phi, void* workspace,
                                 size_t workspace_bytes, void* stream);

/* Marching tetrahedra on phi [nz][ny][nx] (lattice as above): each cube is
   split into the six tetrahedra around its main diagonal (corner c = bx +
   2 by + 4 bz: (0,1,3,7) (0,3,2,7) (0,2,6,7) (0,6,4,7) (0,4,5,7)
   (0,5,1,7)); a corner is inside when phi < 0; a tetrahedron with one corner
   on one side gives one triangle, one with two on each side two; an edge
   (p, q) crosses at p + phi_p / (phi_p - phi_q) (q - p).  Writes up to
   max_triangles triangles to triangles [max_triangles][3][3] (vertex
   positions, unordered, orientation not fixed) and the number found (which
   may exceed max_triangles; the rest are then not written) to the device
   *count (at most 12 per cube; (nx-1)(ny-1)(nz-1) * 12 < 2^32 is required).
   Errors: NULL, SHAPE, VALUE, HIP. */
gosurf_status gosurf_marching_tetrahedra(const float* phi, const float p0[3], float h, int32_t nx, int32_t ny,
                                         int32_t nz, float* triangles, int64_t max_triangles, uint32_t* count,
                                         void* stream);

/* Round the float32 grid to its bfloat16 mirror (round to nearest even), as
   gosurf_adam_step does after every update; call once before the first
   GOSURF_BF16 forward.  numel = 4 * n_vertices.  Errors: NULL, SHAPE, ALIGN,
   HIP. */
gosurf_status gosurf_refresh_bf16(const float* grid, uint16_t* grid_bf16, int64_t numel, void* stream);

/* Adam (Kingma & Ba) with bias correction over both groups, dense: every
   entry is updated, touched or not.  g = grad * inv_loss_scale;
   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
   p -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps).
   Gradients are zeroed and the bfloat16 mirror (if any) refreshed in the same
   pass.  Errors: NULL, SHAPE, ALIGN, VALUE, HIP. */
gosurf_status gosurf_adam_step(const gosurf_adam_cfg* cfg, gosurf_adam_state* state, void* stream);

/* gosurf_adam_step behind a guard against non-finite gradients, for callers
   that scale the loss (the BF16 precision variant) or otherwise want a step
   with an inf or NaN gradient discarded rather than written into the
   parameters and moments.  Enqueues, on the stream: clearing *flag (a
   caller-owned device int32), setting it to 1 if any entry of grid_grad or
   mlp_grad is inf or NaN, and the update, which reads the flag on the device:
   flag 0 gives exactly gosurf_adam_step; flag 1 leaves the parameters,
   moments and bfloat16 mirror unchanged and only zeroes both gradient arrays.
   Nothing waits on the host: the caller reads *flag after the stream has
   reached it to learn whether the step was taken (the step number passed in
   `cfg` is the caller's to keep or repeat).  Extra traffic: one read of the
   gradients (4 B per parameter).  Errors: NULL, SHAPE, ALIGN, VALUE, HIP. */
gosurf_status gosurf_adam_step_checked(const gosurf_adam_cfg* cfg, gosurf_adam_state* state, int32_t* flag,
                                       void* stream);

#ifdef __cplusplus
}
#endif
#endif /* GOSURF_H */
