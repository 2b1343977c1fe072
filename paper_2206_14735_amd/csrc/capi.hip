// C ABI of the GO-Surf hot path: host-side validation, workspace layout and
// kernel launches.  Every entry point validates on the host, enqueues on the
// caller's stream and returns without synchronising.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "device.h"

#include "args.h"

namespace gs {

hipError_t launch_field(const FieldArgs& a, bool bwd, int blocks, hipStream_t st);
hipError_t launch_priv_reduce(const FieldArgs& a, int n_part, const int counts[4], float* tmp, hipStream_t st);
void plan_privatised_levels(FieldArgs& a, int counts[4]);
long long plan_copies(FieldArgs& a);
hipError_t launch_copy_fold(const FieldArgs& a, hipStream_t st);
int priv_max_floats();
int field_grid(const FieldArgs& a, bool bwd);
hipError_t launch_render(const RenderArgs& a, bool bwd, hipStream_t st);
hipError_t launch_loss_reduce(const float* ray_partial, int M, const float* smooth_partial, int n_sp, int S,
                              const float lam[6], float* losses, float* ray_part, hipStream_t st);
hipError_t launch_grad_reduce(const float* partial, int n_part, const float* ray_dv, int M, float* grad_mlp,
                              float* tmp, float* ray_part, hipStream_t st);
hipError_t launch_adam(const gosurf_adam_cfg& c, gosurf_adam_state& s, const int* skip, hipStream_t st);
hipError_t launch_nonfinite_check(const float* grid_grad, long long n_grid, const float* mlp_grad, long long n_mlp,
                                  int* flag, hipStream_t st);
hipError_t launch_zero(float* a, long long n, hipStream_t st);
hipError_t launch_sample(const SampleArgs& a, hipStream_t st);
hipError_t launch_to_bf16(const float* src, uint16_t* dst, long long n, hipStream_t st);
hipError_t launch_sample_rays_only(const SampleArgs& a, hipStream_t st);
hipError_t launch_sample_gen_only(const SampleArgs& a, hipStream_t st);
hipError_t launch_proposal(const PropArgs& a, bool train, int blocks, hipStream_t st);
hipError_t launch_proposal_targets(const TargetArgs& a, hipStream_t st);
hipError_t launch_proposal_seg(float* prop3, const float* depth, int depth_check, float extend, const EdgeCheck& ec,
                               int M, float thr, int n_prop, int n_plain, int* seg, int* block_total, hipStream_t st);
int proposal_blocks(int M);
int proposal_numel();
hipError_t launch_colsum(const float* part, int rows, int cols, float* tmp, float* add_dst, int n_add,
                         float* set_dst, int set_col, hipStream_t st);
hipError_t launch_importance_step(const ImpArgs& a, hipStream_t st);
hipError_t launch_importance_merge(const ImpMergeArgs& a, hipStream_t st);
hipError_t launch_lattice_rays(const LatticeArgs& a, hipStream_t st);
hipError_t launch_phi_copy(const float* out4, long long n, float* phi, hipStream_t st);
hipError_t launch_marching_tets(const MtArgs& a, hipStream_t st);
hipError_t launch_pose_apply(const float* c2w0, const float* pose, int T, float* c2w, hipStream_t st);
hipError_t launch_colour(const ColourArgs& a, bool bwd, int blocks, hipStream_t st);
int colour_grid_blocks(int total, bool bwd);
int colour_numel();
hipError_t launch_ray_xgrad(const float* dx, const float* t, const int* seg, int M, int total, float* grad_o,
                            float* grad_r, hipStream_t st);
hipError_t launch_pose_grad(const float* pose, int T, const long long* pixel, long long HW, const float* r,
                            const float* grad_o, const float* grad_r, int M, float* grad_pose, hipStream_t st);

}  // namespace gs

namespace {

// last error text of this thread: a fixed buffer, so that recording an error
// never allocates and nothing can throw across the C interface
thread_local char g_err[512];

// optional event pair recorded around one kernel (measurement hook)
thread_local int g_timed_kernel = GOSURF_KERNEL_NONE;
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

// One shot: the first launch of the named kernel after gosurf_time_kernel is
// bracketed, later launches are not (a step may launch a kernel more than once,
// e.g. Adam once per parameter group).
void mark(int kernel, bool start, hipStream_t s) {
  if (kernel != g_timed_kernel || !g_ev_start || !g_ev_stop) return;
  hipEventRecord(start ? g_ev_start : g_ev_stop, s);
  if (!start) g_timed_kernel = GOSURF_KERNEL_NONE;
}

gosurf_status fail(gosurf_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
gosurf_status fail(gosurf_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

gosurf_status ok() {
  g_err[0] = '\0';
  return GOSURF_OK;
}

gosurf_status hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) return fail(GOSURF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
  return GOSURF_OK;
}

bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

gosurf_status check_model(const gosurf_model* m) {
  if (!m) return fail(GOSURF_ERR_NULL, "model is NULL");
  if (m->precision != GOSURF_FP32 && m->precision != GOSURF_BF16)
    return fail(GOSURF_ERR_VALUE, "precision %d is not GOSURF_FP32 or GOSURF_BF16", m->precision);
  if (m->colour_mode != GOSURF_COLOUR_DECODED && m->colour_mode != GOSURF_COLOUR_GRID)
    return fail(GOSURF_ERR_VALUE, "colour_mode %d is not GOSURF_COLOUR_DECODED or GOSURF_COLOUR_GRID",
                m->colour_mode);
  if (m->colour_mode == GOSURF_COLOUR_GRID && m->precision != GOSURF_FP32)
    return fail(GOSURF_ERR_VALUE, "the colour-grid path runs in GOSURF_FP32 only");
  if (m->grad_copies != 0 && m->grad_copies != 1)
    return fail(GOSURF_ERR_VALUE, "grad_copies %d is not 0 or 1", m->grad_copies);
  long long rows = 0;
  for (int l = 0; l < GOSURF_LEVELS; ++l) {
    if (!(m->voxel[l] > 0.f) || !std::isfinite(m->voxel[l]))
      return fail(GOSURF_ERR_VALUE, "voxel[%d] must be positive and finite", l);
    for (int a = 0; a < 3; ++a)
      if (m->dims[l][a] < 2) return fail(GOSURF_ERR_SHAPE, "dims[%d][%d] = %d < 2", l, a, m->dims[l][a]);
    const long long n = (long long)m->dims[l][0] * m->dims[l][1] * m->dims[l][2];
    if (m->offset[l] < 0 || m->offset[l] + n > m->n_vertices)
      return fail(GOSURF_ERR_SHAPE, "level %d rows [%lld, %lld) exceed n_vertices %lld", l,
                  (long long)m->offset[l], (long long)(m->offset[l] + n), (long long)m->n_vertices);
    rows += n;
  }
  if (m->n_vertices >= (1LL << 31) - 1) return fail(GOSURF_ERR_SHAPE, "grid has more than 2^31 vertices");
  for (int a = 0; a < 3; ++a)
    if (!(m->p1[a] > m->p0[a])) return fail(GOSURF_ERR_VALUE, "box is empty along axis %d", a);
  (void)rows;
  return GOSURF_OK;
}

gs::Grid to_grid(const gosurf_model* m) {
  gs::Grid g;
  for (int a = 0; a < 3; ++a) { g.p0[a] = m->p0[a]; g.p1[a] = m->p1[a]; }
  for (int l = 0; l < 4; ++l) {
    g.voxel[l] = m->voxel[l];
    g.nx[l] = m->dims[l][0];
    g.ny[l] = m->dims[l][1];
    g.nz[l] = m->dims[l][2];
    g.off[l] = m->offset[l];
  }
  return g;
}

constexpr size_t kAlign = 256;
size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Workspace {
  float* ray_partial;     // [M][8]
  float* smooth_partial;  // [4096]
  float* seed4;           // [total][4]
  float* posw;            // [total][4]: sample position, Eikonal weight
  float* ray_dv;          // [M]
  float* mlp_partial;     // [2048][kMlpNumel]
  float* priv_partial;    // [2048][priv_max_floats]
  float* colsum_tmp;      // [64][max(kMlpNumel, priv_max_floats)]
  float* ray_part;        // [64][8] block partials of sums over rays
  float* copies;          // gradient copies (grad_copies), else NULL
  size_t bytes;
};

Workspace layout(char* base, int M, int total, int S, long long copy_floats) {
  (void)S;
  Workspace w{};
  size_t off = 0;
  auto take = [&](size_t n) { char* p = base ? base + off : nullptr; off += up(n); return p; };
  w.ray_partial = reinterpret_cast<float*>(take(sizeof(float) * 8 * (size_t)M));
  w.smooth_partial = reinterpret_cast<float*>(take(sizeof(float) * 4096));
  w.seed4 = reinterpret_cast<float*>(take(sizeof(float) * 4 * (size_t)total));
  w.posw = reinterpret_cast<float*>(take(sizeof(float) * 4 * (size_t)total));
  w.ray_dv = reinterpret_cast<float*>(take(sizeof(float) * (size_t)M));
  w.mlp_partial = reinterpret_cast<float*>(take(sizeof(float) * 2048 * (size_t)gs::kMlpNumel));
  w.priv_partial = reinterpret_cast<float*>(take(sizeof(float) * 2048 * (size_t)gs::priv_max_floats()));
  w.ray_part = reinterpret_cast<float*>(take(sizeof(float) * 64 * 8));
  w.colsum_tmp = reinterpret_cast<float*>(
      take(sizeof(float) * 64 * (size_t)(gs::priv_max_floats() > gs::kMlpNumel ? gs::priv_max_floats() : gs::kMlpNumel)));
  w.copies = copy_floats > 0 ? reinterpret_cast<float*>(take(sizeof(float) * (size_t)copy_floats)) : nullptr;
  w.bytes = off;
  return w;
}

// Floats of the model's gradient copies: 0 without copies, -1 if the model's
// levels are too large for them.
long long model_copy_floats(const gosurf_model* m) {
  if (!m->grad_copies) return 0;
  gs::FieldArgs fa{};
  fa.g = to_grid(m);
  int counts[4];
  gs::plan_privatised_levels(fa, counts);
  return gs::plan_copies(fa);
}

gosurf_status check_batch(const gosurf_ray_batch* b, bool need_outputs) {
  if (!b) return fail(GOSURF_ERR_NULL, "batch is NULL");
  if (b->M < 1) return fail(GOSURF_ERR_SHAPE, "batch M = %d < 1", b->M);
  if (b->total < b->M) return fail(GOSURF_ERR_SHAPE, "batch total = %d < M", b->total);
  if ((long long)b->total * 4 >= (1LL << 31)) return fail(GOSURF_ERR_SHAPE, "too many samples (%d)", b->total);
  if (b->S < 0) return fail(GOSURF_ERR_SHAPE, "S = %d < 0", b->S);
  if (!b->o || !b->r || !b->rgb || !b->depth || !b->t || !b->seg || !b->ray_of)
    return fail(GOSURF_ERR_NULL, "a ray-batch array is NULL");
  if (b->S > 0 && (!b->xs || !b->eps)) return fail(GOSURF_ERR_NULL, "smoothness arrays are NULL");
  (void)need_outputs;
  return GOSURF_OK;
}

gosurf_status check_loss(const gosurf_loss_cfg* l) {
  if (!l) return fail(GOSURF_ERR_NULL, "loss config is NULL");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(l->lambda[k]) || l->lambda[k] < 0.f)
      return fail(GOSURF_ERR_VALUE, "lambda[%d] must be finite and >= 0", k);
  if (!(l->trunc > 0.f) || !std::isfinite(l->trunc)) return fail(GOSURF_ERR_VALUE, "trunc must be > 0");
  if (!std::isfinite(l->alpha_fs)) return fail(GOSURF_ERR_VALUE, "alpha_fs must be finite");
  if (l->depth_midpoint != 0 && l->depth_midpoint != 1)
    return fail(GOSURF_ERR_VALUE, "depth_midpoint %d is not 0 or 1", l->depth_midpoint);
  return GOSURF_OK;
}

gosurf_status check_params(const gosurf_model* m, const gosurf_params* p) {
  if (!p) return fail(GOSURF_ERR_NULL, "params is NULL");
  if (!p->grid || !p->mlp) return fail(GOSURF_ERR_NULL, "params.grid / params.mlp is NULL");
  if (!aligned(p->grid, 16)) return fail(GOSURF_ERR_ALIGN, "params.grid must be 16-byte aligned");
  if (m->colour_mode == GOSURF_COLOUR_GRID) {
    if (!p->colour_grid || !p->colour_mlp)
      return fail(GOSURF_ERR_NULL, "params.colour_grid and params.colour_mlp are required for GOSURF_COLOUR_GRID");
    if (!aligned(p->colour_grid, 16)) return fail(GOSURF_ERR_ALIGN, "params.colour_grid must be 16-byte aligned");
  }
  if (m->precision == GOSURF_BF16) {
    if (!p->grid_bf16) return fail(GOSURF_ERR_NULL, "params.grid_bf16 is required for GOSURF_BF16");
    if (!aligned(p->grid_bf16, 8)) return fail(GOSURF_ERR_ALIGN, "params.grid_bf16 must be 8-byte aligned");
  }
  return GOSURF_OK;
}

}  // namespace

extern "C" {

const char* gosurf_last_error(void) { return g_err; }

gosurf_status gosurf_time_kernel(int32_t kernel, void* start_event, void* stop_event) {
  if (kernel != GOSURF_KERNEL_NONE && kernel != GOSURF_KERNEL_FIELD_FWD && kernel != GOSURF_KERNEL_FIELD_BWD &&
      kernel != GOSURF_KERNEL_ADAM)
    return fail(GOSURF_ERR_VALUE, "unknown kernel %d", kernel);
  g_timed_kernel = (start_event && stop_event) ? kernel : GOSURF_KERNEL_NONE;
  g_ev_start = static_cast<hipEvent_t>(start_event);
  g_ev_stop = static_cast<hipEvent_t>(stop_event);
  return ok();
}

int64_t gosurf_batch_samples(const gosurf_sample_cfg* cfg) {
  if (!cfg) return -1;
  int64_t n = cfg->n_strat + cfg->n_near;
  if (cfg->proposal && cfg->n_free + cfg->n_proposal > n) n = cfg->n_free + cfg->n_proposal;
  return (int64_t)cfg->M * n;
}

size_t gosurf_workspace_bytes(const gosurf_model* model, int32_t M, int32_t total, int32_t S) {
  if (M < 0 || total < 0 || S < 0) return 0;
  long long cf = 0;
  if (model) {
    if (check_model(model) != GOSURF_OK) return 0;
    cf = model_copy_floats(model);
    if (cf < 0) return 0;
  }
  return layout(nullptr, M, total, S, cf).bytes;
}

gosurf_status gosurf_sample_rays(const gosurf_model* model, const gosurf_frames* fr, const gosurf_sample_cfg* c,
                                 gosurf_ray_batch* out, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if (!fr || !c || !out) return fail(GOSURF_ERR_NULL, "frames, cfg and out must not be NULL");
  if (!fr->rgb || !fr->depth || !fr->c2w) return fail(GOSURF_ERR_NULL, "frame arrays must not be NULL");
  if (fr->T < 1 || fr->H < 1 || fr->W < 1) return fail(GOSURF_ERR_SHAPE, "frames must be non-empty");
  const unsigned long long thw = (unsigned long long)fr->T * fr->H * fr->W;
  if (thw >= (1ULL << 32)) return fail(GOSURF_ERR_SHAPE, "T*H*W = %llu must be < 2^32", thw);
  if (!(fr->fx > 0.f) || !(fr->fy > 0.f)) return fail(GOSURF_ERR_VALUE, "focal lengths must be > 0");
  if (c->M < 1 || c->n_strat < 1 || c->n_near < 0 || c->S < 0)
    return fail(GOSURF_ERR_SHAPE, "need M >= 1, n_strat >= 1, n_near >= 0, S >= 0");
  if (c->n_strat + c->n_near > GOSURF_MAX_SAMPLES_PER_RAY)
    return fail(GOSURF_ERR_SHAPE, "n_strat + n_near = %d exceeds %d", c->n_strat + c->n_near,
                GOSURF_MAX_SAMPLES_PER_RAY);
  const long long total = gosurf_batch_samples(c);
  if (total * 4 >= (1LL << 31)) return fail(GOSURF_ERR_SHAPE, "too many samples (%lld)", total);
  if (c->proposal) {
    if (!c->grid) return fail(GOSURF_ERR_NULL, "the proposal needs the grid");
    if (!out->prop) return fail(GOSURF_ERR_NULL, "out.prop must hold [M][3] with a proposal");
    if (c->n_proposal < 1 || c->n_free < 0 || c->n_free + c->n_proposal > GOSURF_MAX_SAMPLES_PER_RAY)
      return fail(GOSURF_ERR_SHAPE, "need n_proposal >= 1, n_free >= 0 and n_free + n_proposal = %d <= %d",
                  c->n_free + c->n_proposal, GOSURF_MAX_SAMPLES_PER_RAY);
    if (!std::isfinite(c->conf_threshold)) return fail(GOSURF_ERR_VALUE, "conf_threshold must be finite");
    if (c->depth_check && !(c->conf_threshold > 0.f))
      return fail(GOSURF_ERR_VALUE, "the depth check needs conf_threshold > 0");
    if (c->depth_check && !(c->depth_extend >= 0.f && std::isfinite(c->depth_extend)))
      return fail(GOSURF_ERR_VALUE, "depth_extend must be finite and >= 0");
    if (!(c->depth_edge >= 0.f && std::isfinite(c->depth_edge)))
      return fail(GOSURF_ERR_VALUE, "depth_edge must be finite and >= 0");
    if (c->depth_edge > 0.f && !c->depth_check) return fail(GOSURF_ERR_VALUE, "depth_edge needs depth_check");
    if (c->depth_edge > 0.f && !out->pixel) return fail(GOSURF_ERR_NULL, "depth_edge needs out.pixel");
  }
  if (out->M != c->M || out->total != total || out->S != c->S)
    return fail(GOSURF_ERR_SHAPE, "out sizes (M=%d total=%d S=%d) do not match cfg (M=%d total=%lld S=%d)",
                out->M, out->total, out->S, c->M, total, c->S);
  if (c->span_mode != GOSURF_SPAN_FIXED && c->span_mode != GOSURF_SPAN_BOX)
    return fail(GOSURF_ERR_VALUE, "unknown span_mode %d", c->span_mode);
  if (!(c->far_t >= c->near_t) || !std::isfinite(c->near_t))
    return fail(GOSURF_ERR_VALUE, "need finite near <= far");
  if (!(c->trunc > 0.f) || c->delta_s < 0.f) return fail(GOSURF_ERR_VALUE, "need trunc > 0, delta_s >= 0");
  if (!out->o || !out->r || !out->rgb || !out->depth || !out->t || !out->seg || !out->ray_of)
    return fail(GOSURF_ERR_NULL, "an output array is NULL");
  if (c->S > 0 && (!out->xs || !out->eps)) return fail(GOSURF_ERR_NULL, "smoothness outputs are NULL");
  gs::SampleArgs a{};
  a.g = to_grid(model);
  a.rgb = fr->rgb; a.depth = fr->depth; a.c2w = fr->c2w;
  a.T = fr->T; a.H = fr->H; a.W = fr->W;
  a.fx = fr->fx; a.fy = fr->fy; a.cx = fr->cx; a.cy = fr->cy;
  a.M = c->M; a.n_strat = c->n_strat; a.n_near = c->n_near; a.span_mode = c->span_mode;
  a.near_t = c->near_t; a.far_t = c->far_t; a.trunc = c->trunc; a.S = c->S; a.delta_s = c->delta_s;
  a.k0 = (uint32_t)(c->seed & 0xffffffffu); a.k1 = (uint32_t)(c->seed >> 32); a.step = c->step;
  a.o = out->o; a.r = out->r; a.rgb_out = out->rgb; a.depth_out = out->depth; a.t = out->t;
  a.seg = out->seg; a.ray_of = out->ray_of; a.xs = out->xs; a.eps = out->eps;
  a.pixel = reinterpret_cast<long long*>(out->pixel);
  hipStream_t s = (hipStream_t)stream;
  if (!c->proposal) {
    if ((st = hip_check(gs::launch_sample(a, s), "sample_kernel")) != GOSURF_OK) return st;
    return ok();
  }
  if ((st = hip_check(gs::launch_sample_rays_only(a, s), "sample rays")) != GOSURF_OK) return st;
  gs::PropArgs pa{};
  pa.g = a.g; pa.grid = c->grid; pa.prop = c->proposal; pa.o = out->o; pa.r = out->r; pa.M = c->M;
  pa.span_mode = c->span_mode; pa.near_t = c->near_t; pa.far_t = c->far_t; pa.out3 = out->prop;
  if ((st = hip_check(gs::launch_proposal(pa, false, gs::proposal_blocks(c->M), s), "proposal")) != GOSURF_OK)
    return st;
  gs::EdgeCheck ec{fr->depth, fr->H, fr->W, reinterpret_cast<const long long*>(out->pixel),
                   c->depth_check ? c->depth_edge : 0.f};
  if ((st = hip_check(gs::launch_proposal_seg(out->prop, out->depth, c->depth_check, c->depth_extend, ec, c->M,
                                              c->conf_threshold,
                                              c->n_free + c->n_proposal,
                                              c->n_strat + c->n_near, out->seg, out->ray_of, s),
                      "proposal seg")) != GOSURF_OK)
    return st;
  a.prop3 = out->prop; a.conf_thr = c->conf_threshold; a.n_prop = c->n_proposal; a.n_free = c->n_free;
  if ((st = hip_check(gs::launch_sample_gen_only(a, s), "proposal samples")) != GOSURF_OK) return st;
  return ok();
}

}  // extern "C"

namespace {

// The forward's scratch: per-ray loss partials [M][8], the field kernel's
// per-block smoothness partials [4096] and the block partials of the sums
// over rays [64][8].  Every entry that is read is written first by the same
// call, so nothing needs clearing.
struct FwdScratch {
  float* ray_partial;
  float* smooth_partial;
  float* ray_part;
};

gosurf_status forward_checks(const gosurf_model* model, const gosurf_params* params, const gosurf_ray_batch* b,
                             const gosurf_loss_cfg* loss, const gosurf_fwd_out* out) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_params(model, params)) != GOSURF_OK) return st;
  if ((st = check_batch(b, false)) != GOSURF_OK) return st;
  if ((st = check_loss(loss)) != GOSURF_OK) return st;
  if (!out || !out->rgb_hat || !out->depth_hat || !out->wsum || !out->losses || !out->saved)
    return fail(GOSURF_ERR_NULL, "a forward output array is NULL");
  if (!aligned(out->saved, 16)) return fail(GOSURF_ERR_ALIGN, "out.saved must be 16-byte aligned");
  return GOSURF_OK;
}

gosurf_status forward_launch(const gosurf_model* model, const gosurf_params* params, const gosurf_ray_batch* b,
                             const gosurf_loss_cfg* loss, gosurf_fwd_out* out, const FwdScratch& w, hipStream_t s) {
  gosurf_status st;
  const gs::Grid g = to_grid(model);
  const bool need_gx = loss->lambda[4] != 0.f;
  float* eik = out->saved + 4 * (size_t)b->total;

  gs::FieldArgs fa{};
  fa.g = g; fa.grid = params->grid; fa.mlp = params->mlp;
  fa.grid_bf16 = model->precision == GOSURF_BF16 ? params->grid_bf16 : nullptr;
  fa.o = b->o; fa.r = b->r; fa.t = b->t; fa.ray_of = b->ray_of; fa.total = b->total;
  fa.xs = b->xs; fa.eps = b->eps; fa.S = b->S; fa.seg_end = b->seg + b->M;
  fa.out4 = out->saved; fa.eik = eik; fa.smooth_partial = w.smooth_partial; fa.need_gx = need_gx;
  fa.depth = b->depth; fa.trunc = loss->trunc;   // residuals are needed only in S_fs
  fa.grad_phi = out->grad_phi; fa.pair_terms = out->pair_terms;
  fa.colour = model->colour_mode == GOSURF_COLOUR_DECODED;
  if (loss->lambda[5] == 0.f) fa.S = 0;   // the smoothness pairs are skipped
  const int nb = gs::field_grid(fa, false);
  if (nb <= 0) return fail(GOSURF_ERR_HIP, "field grid: the occupancy query failed");
  mark(GOSURF_KERNEL_FIELD_FWD, true, s);
  if ((st = hip_check(gs::launch_field(fa, false, nb, s), "field fwd")) != GOSURF_OK) return st;
  mark(GOSURF_KERNEL_FIELD_FWD, false, s);
  if (model->colour_mode == GOSURF_COLOUR_GRID) {
    gs::ColourArgs ca{};
    ca.g = g; ca.cgrid = params->colour_grid; ca.cmlp = params->colour_mlp;
    ca.o = b->o; ca.r = b->r; ca.t = b->t; ca.ray_of = b->ray_of; ca.total = b->total; ca.seg_end = b->seg + b->M;
    ca.out4 = out->saved;
    const int cb = gs::colour_grid_blocks(b->total, false);
    if (cb <= 0) return fail(GOSURF_ERR_HIP, "colour grid: the occupancy query failed");
    if ((st = hip_check(gs::launch_colour(ca, false, cb, s), "colour fwd")) != GOSURF_OK) return st;
  }
  const int n_sp = fa.S > 0 ? nb : 0;
  gs::RenderArgs ra{};
  ra.g = g; ra.o = b->o; ra.r = b->r; ra.rgb = b->rgb; ra.depth = b->depth; ra.t = b->t; ra.seg = b->seg;
  ra.M = b->M; ra.total = b->total; ra.mlp = params->mlp; ra.out4 = out->saved; ra.eik = need_gx ? eik : nullptr;
  ra.trunc = loss->trunc; ra.alpha_fs = loss->alpha_fs; ra.depth_mid = loss->depth_midpoint;
  for (int k = 0; k < 6; ++k) ra.lam[k] = loss->lambda[k];
  ra.rgb_hat = out->rgb_hat; ra.depth_hat = out->depth_hat; ra.wsum = out->wsum; ra.weights = out->weights;
  ra.ray_partial = out->ray_terms ? out->ray_terms : w.ray_partial;
  if ((st = hip_check(gs::launch_render(ra, false, s), "render fwd")) != GOSURF_OK) return st;
  if ((st = hip_check(gs::launch_loss_reduce(ra.ray_partial, b->M, w.smooth_partial, n_sp, b->S, loss->lambda,
                                             out->losses, w.ray_part, s),
                      "loss reduce")) != GOSURF_OK)
    return st;
  return ok();
}

// ---------------------------------------------------------------- allocation-free forward
// The scratch of gosurf_forward_static: a file-scope device array, one copy
// per GPU, sized for GOSURF_STATIC_MAX_RAYS rays.  In host code its name
// stands for a host-side shadow, so its device address is looked up once per
// device (hipGetSymbolAddress, with that device current) and only that
// address is handed to kernels.
constexpr size_t kStaticRayPartialBytes = (size_t)32 * GOSURF_STATIC_MAX_RAYS;
constexpr size_t kStaticSmoothBytes = (size_t)4 * 4096;
constexpr size_t kStaticRayPartBytes = (size_t)4 * 64 * 8;
constexpr size_t kStaticScratchBytes = kStaticRayPartialBytes + kStaticSmoothBytes + kStaticRayPartBytes;
static_assert(kStaticRayPartialBytes % 256 == 0 && kStaticSmoothBytes % 256 == 0, "scratch alignment");

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

gosurf_status static_scratch(void** out) {
  int dev = 0;
  gosurf_status st;
  if ((st = hip_check(hipGetDevice(&dev), "hipGetDevice")) != GOSURF_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) return fail(GOSURF_ERR_VALUE, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if ((st = hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch address")) != GOSURF_OK) return st;
    if (!p) return fail(GOSURF_ERR_HIP, "scratch address: null");
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return GOSURF_OK;
}

}  // namespace

extern "C" {

gosurf_status gosurf_forward(const gosurf_model* model, const gosurf_params* params, const gosurf_ray_batch* b,
                             const gosurf_loss_cfg* loss, gosurf_fwd_out* out, void* ws, size_t ws_bytes,
                             void* stream) {
  gosurf_status st;
  if ((st = forward_checks(model, params, b, loss, out)) != GOSURF_OK) return st;
  // the forward uses the part before the gradient copies
  const Workspace w = layout(static_cast<char*>(ws), b->M, b->total, b->S, 0);
  if (!ws || ws_bytes < w.bytes)
    return fail(GOSURF_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                w.bytes);
  return forward_launch(model, params, b, loss, out, FwdScratch{w.ray_partial, w.smooth_partial, w.ray_part},
                        (hipStream_t)stream);
}

gosurf_status gosurf_forward_static(const gosurf_model* model, const gosurf_params* params,
                                    const gosurf_ray_batch* b, const gosurf_loss_cfg* loss, gosurf_fwd_out* out,
                                    void* stream) {
  gosurf_status st;
  if ((st = forward_checks(model, params, b, loss, out)) != GOSURF_OK) return st;
  if (b->M > GOSURF_STATIC_MAX_RAYS)
    return fail(GOSURF_ERR_SHAPE, "gosurf_forward_static: %d rays exceed its scratch of %d rays", b->M,
                GOSURF_STATIC_MAX_RAYS);
  void* base = nullptr;
  if ((st = static_scratch(&base)) != GOSURF_OK) return st;
  char* c = static_cast<char*>(base);
  const FwdScratch w{reinterpret_cast<float*>(c), reinterpret_cast<float*>(c + kStaticRayPartialBytes),
                     reinterpret_cast<float*>(c + kStaticRayPartialBytes + kStaticSmoothBytes)};
  return forward_launch(model, params, b, loss, out, w, (hipStream_t)stream);
}

gosurf_status gosurf_backward(const gosurf_model* model, const gosurf_params* params, const gosurf_ray_batch* b,
                              const gosurf_loss_cfg* loss, const gosurf_fwd_out* fwd, float loss_scale,
                              gosurf_grads* grads, void* ws, size_t ws_bytes, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_params(model, params)) != GOSURF_OK) return st;
  if ((st = check_batch(b, false)) != GOSURF_OK) return st;
  if ((st = check_loss(loss)) != GOSURF_OK) return st;
  if (!fwd || !fwd->saved || !fwd->losses) return fail(GOSURF_ERR_NULL, "forward outputs are NULL");
  if (!grads || !grads->grid || !grads->mlp) return fail(GOSURF_ERR_NULL, "gradient buffers are NULL");
  if (model->colour_mode == GOSURF_COLOUR_GRID && (!grads->colour_grid || !grads->colour_mlp))
    return fail(GOSURF_ERR_NULL, "grads.colour_grid and grads.colour_mlp are required for GOSURF_COLOUR_GRID");
  if ((grads->ray_o == nullptr) != (grads->ray_r == nullptr))
    return fail(GOSURF_ERR_NULL, "grads.ray_o and grads.ray_r are both given or both NULL");
  if (!aligned(grads->grid, 16)) return fail(GOSURF_ERR_ALIGN, "grads.grid must be 16-byte aligned");
  if (!std::isfinite(loss_scale)) return fail(GOSURF_ERR_VALUE, "loss_scale must be finite");
  const long long copy_floats = model_copy_floats(model);
  if (copy_floats < 0)
    return fail(GOSURF_ERR_VALUE, "gradient copies need levels of at most 2048 x 2048 x 512 vertices and 2^31 floats");
  const Workspace w = layout(static_cast<char*>(ws), b->M, b->total, b->S, copy_floats);
  if (!ws || ws_bytes < w.bytes)
    return fail(GOSURF_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes,
                w.bytes);
  hipStream_t s = (hipStream_t)stream;
  const gs::Grid g = to_grid(model);
  const bool need_gx = loss->lambda[4] != 0.f;

  gs::RenderArgs ra{};
  ra.g = g; ra.o = b->o; ra.r = b->r; ra.rgb = b->rgb; ra.depth = b->depth; ra.t = b->t; ra.seg = b->seg;
  ra.M = b->M; ra.total = b->total; ra.mlp = params->mlp; ra.out4 = fwd->saved; ra.eik = nullptr;
  ra.trunc = loss->trunc; ra.alpha_fs = loss->alpha_fs; ra.depth_mid = loss->depth_midpoint;
  for (int k = 0; k < 6; ++k) ra.lam[k] = loss->lambda[k];
  ra.n_depth_rays = fwd->losses + 7;
  ra.loss_scale = loss_scale; ra.seed4 = w.seed4; ra.posw = w.posw; ra.ray_dv = w.ray_dv;
  if ((st = hip_check(gs::launch_render(ra, true, s), "render bwd")) != GOSURF_OK) return st;

  gs::FieldArgs fa{};
  fa.g = g; fa.grid = params->grid; fa.mlp = params->mlp;
  fa.grid_bf16 = model->precision == GOSURF_BF16 ? params->grid_bf16 : nullptr;
  fa.o = b->o; fa.r = b->r; fa.t = b->t; fa.ray_of = b->ray_of; fa.total = b->total;
  fa.xs = b->xs; fa.eps = b->eps; fa.S = b->S; fa.seg_end = b->seg + b->M;
  fa.seed4 = w.seed4; fa.posw = w.posw; fa.need_gx = need_gx;
  const bool ray_grads = grads->ray_o != nullptr;
  const bool cgrid = model->colour_mode == GOSURF_COLOUR_GRID;
  fa.colour = !cgrid;
  // dL/dx per sample replaces the sample's seeds once read (the colour kernel,
  // which also reads the seeds, runs first then)
  fa.grad_x = ray_grads ? w.seed4 : nullptr;
  if (cgrid && ray_grads)
    return fail(GOSURF_ERR_VALUE, "ray gradients (pose refinement) are not built for the colour-grid path");
  fa.grad_grid = grads->grid; fa.mlp_partial = w.mlp_partial;
  fa.smooth_coef = b->S > 0 ? 2.f * loss->lambda[5] * loss_scale / (float)b->S : 0.f;
  if (loss->lambda[5] == 0.f) fa.S = 0;   // the smoothness pairs are skipped
  int counts[4];
  gs::plan_privatised_levels(fa, counts);
  fa.priv_partial = w.priv_partial;
  if (copy_floats > 0) {
    fa.copies = w.copies;
    gs::plan_copies(fa);
    if ((st = hip_check(gs::launch_zero(w.copies, copy_floats, s), "zero gradient copies")) != GOSURF_OK) return st;
  }
  const int nb = gs::field_grid(fa, true);
  if (nb <= 0) return fail(GOSURF_ERR_HIP, "field grid: the occupancy query failed");
  mark(GOSURF_KERNEL_FIELD_BWD, true, s);
  if ((st = hip_check(gs::launch_field(fa, true, nb, s), "field bwd")) != GOSURF_OK) return st;
  mark(GOSURF_KERNEL_FIELD_BWD, false, s);
  if (copy_floats > 0 && (st = hip_check(gs::launch_copy_fold(fa, s), "fold gradient copies")) != GOSURF_OK)
    return st;
  if ((st = hip_check(gs::launch_priv_reduce(fa, nb, counts, w.colsum_tmp, s), "level reduce")) != GOSURF_OK)
    return st;
  if (ray_grads &&
      (st = hip_check(gs::launch_ray_xgrad(w.seed4, b->t, b->seg, b->M, b->total, grads->ray_o, grads->ray_r, s),
                      "ray gradients")) != GOSURF_OK)
    return st;
  if ((st = hip_check(gs::launch_grad_reduce(w.mlp_partial, nb, w.ray_dv, b->M, grads->mlp, w.colsum_tmp,
                                             w.ray_part, s),
                      "grad reduce")) != GOSURF_OK)
    return st;
  if (cgrid) {
    // the colour path: its own kernel on the colour seeds; its decoder partials
    // reuse the decoder-partial rows, whose reduction above is already enqueued
    gs::ColourArgs ca{};
    ca.g = g; ca.cgrid = params->colour_grid; ca.cmlp = params->colour_mlp;
    ca.o = b->o; ca.r = b->r; ca.t = b->t; ca.ray_of = b->ray_of; ca.total = b->total; ca.seg_end = b->seg + b->M;
    ca.seed4 = w.seed4; ca.posw = w.posw; ca.grad_cgrid = grads->colour_grid; ca.partial = w.mlp_partial;
    const int cb = gs::colour_grid_blocks(b->total, true);
    if (cb <= 0) return fail(GOSURF_ERR_HIP, "colour grid: the occupancy query failed");
    if ((st = hip_check(gs::launch_colour(ca, true, cb, s), "colour bwd")) != GOSURF_OK) return st;
    const int cn = gs::colour_numel();
    if ((st = hip_check(gs::launch_colsum(w.mlp_partial, cb, cn, w.colsum_tmp, grads->colour_mlp, cn, nullptr, -1, s),
                        "colour reduce")) != GOSURF_OK)
      return st;
  }
  return ok();
}

static gosurf_status check_rays(const gosurf_ray_batch* r, const gosurf_sample_cfg* span) {
  if (!r || !span) return fail(GOSURF_ERR_NULL, "rays and span must not be NULL");
  if (r->M < 1) return fail(GOSURF_ERR_SHAPE, "M = %d < 1", r->M);
  if (!r->o || !r->r) return fail(GOSURF_ERR_NULL, "rays.o / rays.r are NULL");
  if (span->span_mode != GOSURF_SPAN_FIXED && span->span_mode != GOSURF_SPAN_BOX)
    return fail(GOSURF_ERR_VALUE, "unknown span_mode %d", span->span_mode);
  if (!(span->far_t >= span->near_t)) return fail(GOSURF_ERR_VALUE, "need near <= far");
  return GOSURF_OK;
}

gosurf_status gosurf_proposal_forward(const gosurf_model* model, const float* grid, const float* proposal,
                                      const gosurf_ray_batch* rays, const gosurf_sample_cfg* span, float* out3,
                                      void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_rays(rays, span)) != GOSURF_OK) return st;
  if (!grid || !proposal || !out3) return fail(GOSURF_ERR_NULL, "grid, proposal and out3 must not be NULL");
  if (!aligned(grid, 16)) return fail(GOSURF_ERR_ALIGN, "grid must be 16-byte aligned");
  gs::PropArgs pa{};
  pa.g = to_grid(model); pa.grid = grid; pa.prop = proposal; pa.o = rays->o; pa.r = rays->r; pa.M = rays->M;
  pa.span_mode = span->span_mode; pa.near_t = span->near_t; pa.far_t = span->far_t; pa.out3 = out3;
  if ((st = hip_check(gs::launch_proposal(pa, false, gs::proposal_blocks(rays->M), (hipStream_t)stream),
                      "proposal forward")) != GOSURF_OK)
    return st;
  return ok();
}

gosurf_status gosurf_proposal_targets(const gosurf_model* model, const gosurf_ray_batch* rays,
                                      const gosurf_sample_cfg* span, const float* weights, float widen,
                                      float* targets, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_rays(rays, span)) != GOSURF_OK) return st;
  if (!rays->t || !rays->seg || !weights || !targets)
    return fail(GOSURF_ERR_NULL, "rays.t, rays.seg, weights and targets must not be NULL");
  if (!(widen >= 0.f) || !std::isfinite(widen)) return fail(GOSURF_ERR_VALUE, "widen must be >= 0");
  gs::TargetArgs ta{};
  ta.g = to_grid(model); ta.t = rays->t; ta.w = weights; ta.seg = rays->seg; ta.o = rays->o; ta.r = rays->r;
  ta.M = rays->M; ta.span_mode = span->span_mode; ta.near_t = span->near_t; ta.far_t = span->far_t;
  ta.widen = widen; ta.q_lo = 0.005f; ta.q_hi = 0.995f; ta.conf_min = 0.5f; ta.tgt = targets;
  if ((st = hip_check(gs::launch_proposal_targets(ta, (hipStream_t)stream), "proposal targets")) != GOSURF_OK)
    return st;
  return ok();
}

size_t gosurf_proposal_workspace_bytes(int32_t M) {
  if (M < 1) return 0;
  const size_t cols = (size_t)gs::proposal_numel() + 1;
  return up(sizeof(float) * (size_t)gs::proposal_blocks(M) * cols) + up(sizeof(float) * 64 * cols);
}

gosurf_status gosurf_proposal_backward(const gosurf_model* model, const float* grid, const float* proposal,
                                       const gosurf_ray_batch* rays, const gosurf_sample_cfg* span,
                                       const float* targets, float beta, float cover_tol, float* grad,
                                       float* loss, void* ws, size_t ws_bytes, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_rays(rays, span)) != GOSURF_OK) return st;
  if (!grid || !proposal || !targets || !grad || !loss)
    return fail(GOSURF_ERR_NULL, "grid, proposal, targets, grad and loss must not be NULL");
  if (!aligned(grid, 16)) return fail(GOSURF_ERR_ALIGN, "grid must be 16-byte aligned");
  if (!(beta > 0.f) || !std::isfinite(beta)) return fail(GOSURF_ERR_VALUE, "beta must be > 0");
  if (!(cover_tol >= 0.f) || !std::isfinite(cover_tol)) return fail(GOSURF_ERR_VALUE, "cover_tol must be >= 0");
  const size_t need = gosurf_proposal_workspace_bytes(rays->M);
  if (!ws || ws_bytes < need)
    return fail(GOSURF_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
  const int blocks = gs::proposal_blocks(rays->M);
  const int cols = gs::proposal_numel() + 1;
  float* part = static_cast<float*>(ws);
  float* tmp = reinterpret_cast<float*>(static_cast<char*>(ws) + up(sizeof(float) * (size_t)blocks * cols));
  gs::PropArgs pa{};
  pa.g = to_grid(model); pa.grid = grid; pa.prop = proposal; pa.o = rays->o; pa.r = rays->r; pa.M = rays->M;
  pa.span_mode = span->span_mode; pa.near_t = span->near_t; pa.far_t = span->far_t; pa.out3 = nullptr;
  pa.tgt = targets; pa.beta = beta; pa.cover_tol = cover_tol; pa.grad_partial = part;
  hipStream_t s = (hipStream_t)stream;
  if ((st = hip_check(gs::launch_proposal(pa, true, blocks, s), "proposal backward")) != GOSURF_OK) return st;
  if ((st = hip_check(gs::launch_colsum(part, blocks, cols, tmp, grad, cols - 1, loss, cols - 1, s),
                      "proposal reduce")) != GOSURF_OK)
    return st;
  return ok();
}

gosurf_status gosurf_refresh_bf16(const float* grid, uint16_t* grid_bf16, int64_t numel, void* stream) {
  if (!grid || !grid_bf16) return fail(GOSURF_ERR_NULL, "grid and grid_bf16 must not be NULL");
  if (numel < 0 || numel % 4) return fail(GOSURF_ERR_SHAPE, "numel must be a non-negative multiple of 4");
  if (!aligned(grid, 16) || !aligned(grid_bf16, 8)) return fail(GOSURF_ERR_ALIGN, "grid 16-B, mirror 8-B aligned");
  gosurf_status st;
  if ((st = hip_check(gs::launch_to_bf16(grid, grid_bf16, numel, (hipStream_t)stream), "bf16 refresh")) !=
      GOSURF_OK)
    return st;
  return ok();
}

}  // extern "C"

namespace {

gosurf_status check_adam(const gosurf_adam_cfg* c, const gosurf_adam_state* s) {
  if (!c || !s) return fail(GOSURF_ERR_NULL, "cfg and state must not be NULL");
  if (s->grid_numel > 0 && (!s->grid || !s->grid_grad || !s->grid_m || !s->grid_v))
    return fail(GOSURF_ERR_NULL, "a grid-group Adam array is NULL");
  if (s->mlp_numel > 0 && (!s->mlp || !s->mlp_grad || !s->mlp_m || !s->mlp_v))
    return fail(GOSURF_ERR_NULL, "a decoder-group Adam array is NULL");
  if (s->grid_numel < 0 || s->grid_numel % 4 || s->mlp_numel < 0)
    return fail(GOSURF_ERR_SHAPE, "grid group: non-negative multiple of 4; decoder group: non-negative");
  const void* ptrs[] = {s->grid, s->grid_grad, s->grid_m, s->grid_v, s->mlp, s->mlp_grad, s->mlp_m, s->mlp_v};
  for (const void* p : ptrs)
    if (!aligned(p, 16)) return fail(GOSURF_ERR_ALIGN, "Adam arrays must be 16-byte aligned");
  if (s->grid_bf16 && !aligned(s->grid_bf16, 8)) return fail(GOSURF_ERR_ALIGN, "grid_bf16 must be 8-byte aligned");
  if (c->step < 1) return fail(GOSURF_ERR_VALUE, "step must be >= 1");
  if (!(c->beta1 >= 0.f && c->beta1 < 1.f && c->beta2 >= 0.f && c->beta2 < 1.f))
    return fail(GOSURF_ERR_VALUE, "betas must lie in [0, 1)");
  if (!(c->eps > 0.f) || !std::isfinite(c->lr_grid) || !std::isfinite(c->lr_mlp) ||
      !std::isfinite(c->inv_loss_scale))
    return fail(GOSURF_ERR_VALUE, "eps must be > 0 and rates finite");
  return GOSURF_OK;
}

}  // namespace

extern "C" {

gosurf_status gosurf_adam_step(const gosurf_adam_cfg* c, gosurf_adam_state* s, void* stream) {
  gosurf_status st;
  if ((st = check_adam(c, s)) != GOSURF_OK) return st;
  gosurf_adam_state copy = *s;
  mark(GOSURF_KERNEL_ADAM, true, (hipStream_t)stream);
  if ((st = hip_check(gs::launch_adam(*c, copy, nullptr, (hipStream_t)stream), "adam")) != GOSURF_OK) return st;
  mark(GOSURF_KERNEL_ADAM, false, (hipStream_t)stream);
  return ok();
}

gosurf_status gosurf_adam_step_checked(const gosurf_adam_cfg* c, gosurf_adam_state* s, int32_t* flag,
                                       void* stream) {
  gosurf_status st;
  if ((st = check_adam(c, s)) != GOSURF_OK) return st;
  if (!flag) return fail(GOSURF_ERR_NULL, "flag is NULL");
  if (!aligned(flag, 4)) return fail(GOSURF_ERR_ALIGN, "flag must be 4-byte aligned");
  hipStream_t h = (hipStream_t)stream;
  // the check writes the flag on the stream; the update kernels read it there
  // and skip the step on the device, so nothing waits on the host
  if ((st = hip_check(gs::launch_nonfinite_check(s->grid_grad, s->grid_numel, s->mlp_grad, s->mlp_numel, flag, h),
                      "non-finite check")) != GOSURF_OK)
    return st;
  gosurf_adam_state copy = *s;
  mark(GOSURF_KERNEL_ADAM, true, h);
  if ((st = hip_check(gs::launch_adam(*c, copy, flag, h), "adam")) != GOSURF_OK) return st;
  mark(GOSURF_KERNEL_ADAM, false, h);
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- camera pose refinement
extern "C" {

gosurf_status gosurf_pose_apply(const float* c2w0, const float* pose, int32_t T, float* c2w, void* stream) {
  if (!c2w0 || !pose || !c2w) return fail(GOSURF_ERR_NULL, "c2w0, pose and c2w must not be NULL");
  if (T < 1) return fail(GOSURF_ERR_SHAPE, "T = %d < 1", T);
  gosurf_status st;
  if ((st = hip_check(gs::launch_pose_apply(c2w0, pose, T, c2w, (hipStream_t)stream), "pose apply")) != GOSURF_OK)
    return st;
  return ok();
}

gosurf_status gosurf_pose_backward(const float* pose, int32_t T, const int64_t* pixel, int64_t HW, const float* r,
                                   const float* grad_o, const float* grad_r, int32_t M, float* grad_pose,
                                   void* stream) {
  if (!pose || !pixel || !r || !grad_o || !grad_r || !grad_pose)
    return fail(GOSURF_ERR_NULL, "a pose-gradient array is NULL");
  if (T < 1 || M < 1 || HW < 1) return fail(GOSURF_ERR_SHAPE, "need T, M, HW >= 1 (got %d, %d, %lld)", T, M,
                                           (long long)HW);
  gosurf_status st;
  if ((st = hip_check(gs::launch_pose_grad(pose, T, reinterpret_cast<const long long*>(pixel), HW, r, grad_o,
                                           grad_r, M, grad_pose, (hipStream_t)stream),
                      "pose gradient")) != GOSURF_OK)
    return st;
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- hierarchical importance sampling
namespace {

constexpr uint32_t kImpStream = 8;   // Philox stream of importance step k: 8 + k

gosurf_status check_importance_cfg(const gosurf_importance_cfg* c) {
  if (!c) return fail(GOSURF_ERR_NULL, "importance config is NULL");
  if (c->steps < 1 || c->steps > 8) return fail(GOSURF_ERR_VALUE, "importance steps = %d (1..8)", c->steps);
  if (c->n_add < 1 || c->n_add > gs::kImpMaxAdd)
    return fail(GOSURF_ERR_VALUE, "n_add = %d (1..%d)", c->n_add, gs::kImpMaxAdd);
  if (!(c->weight_eps > 0.f) || !std::isfinite(c->weight_eps))
    return fail(GOSURF_ERR_VALUE, "weight_eps must be finite and > 0");
  return GOSURF_OK;
}

struct ImpWorkspace {
  float* ta;        // [M][nf] current depths (two buffers, alternating)
  float* pa;        // [M][nf] their SDF values
  float* tb;
  float* pb;
  float* t_new;     // [M][n_add]
  int* ray_new;     // [M][n_add]
  float* out_c;     // [M][n0][4] forward outputs at the coarse samples
  float* out_n;     // [M][n_add][4] forward outputs at the new samples
  size_t bytes;
};

ImpWorkspace imp_layout(char* base, int M, int n0, int n_add, int steps) {
  ImpWorkspace w{};
  const size_t nf = (size_t)n0 + (size_t)steps * n_add;
  size_t off = 0;
  auto take = [&](size_t n) { char* p = base ? base + off : nullptr; off += up(n); return p; };
  w.ta = reinterpret_cast<float*>(take(sizeof(float) * M * nf));
  w.pa = reinterpret_cast<float*>(take(sizeof(float) * M * nf));
  w.tb = reinterpret_cast<float*>(take(sizeof(float) * M * nf));
  w.pb = reinterpret_cast<float*>(take(sizeof(float) * M * nf));
  w.t_new = reinterpret_cast<float*>(take(sizeof(float) * M * (size_t)n_add));
  w.ray_new = reinterpret_cast<int*>(take(sizeof(int) * M * (size_t)n_add));
  w.out_c = reinterpret_cast<float*>(take(sizeof(float) * 4 * M * (size_t)n0));
  w.out_n = reinterpret_cast<float*>(take(sizeof(float) * 4 * M * (size_t)n_add));
  w.bytes = off;
  return w;
}

// SDF (with colour) of `total` samples given by (t, ray_of) through the forward field kernel
gosurf_status field_phi(const gosurf_model* model, const gosurf_params* params, const gosurf_ray_batch* rays,
                        const float* t, const int* ray_of, int total, float* out4, hipStream_t s) {
  gs::FieldArgs fa{};
  fa.g = to_grid(model); fa.grid = params->grid; fa.mlp = params->mlp;
  fa.grid_bf16 = model->precision == GOSURF_BF16 ? params->grid_bf16 : nullptr;
  fa.o = rays->o; fa.r = rays->r; fa.t = t; fa.ray_of = ray_of; fa.total = total;
  fa.S = 0; fa.out4 = out4; fa.need_gx = 0;
  const int nb = gs::field_grid(fa, false);
  if (nb <= 0) return fail(GOSURF_ERR_HIP, "field grid: the occupancy query failed");
  return hip_check(gs::launch_field(fa, false, nb, s), "field fwd (importance)");
}

}  // namespace

extern "C" {

size_t gosurf_importance_workspace_bytes(int32_t M, int32_t n_coarse, const gosurf_importance_cfg* cfg) {
  if (!cfg || M < 1 || n_coarse < 1) return 0;
  return imp_layout(nullptr, M, n_coarse, cfg->n_add, cfg->steps).bytes;
}

gosurf_status gosurf_importance_step(const gosurf_model* model, const float* mlp, const gosurf_ray_batch* rays,
                                     const float* phi, const gosurf_importance_cfg* cfg, int32_t step_index,
                                     float* t_new, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_importance_cfg(cfg)) != GOSURF_OK) return st;
  if (!mlp || !rays || !phi || !t_new || !rays->o || !rays->r || !rays->t)
    return fail(GOSURF_ERR_NULL, "an importance-step array is NULL");
  if (rays->M < 1 || rays->total % rays->M != 0)
    return fail(GOSURF_ERR_SHAPE, "total = %d is not a multiple of M = %d", rays->total, rays->M);
  const int n = rays->total / rays->M;
  if (n < 2 || n > GOSURF_MAX_SAMPLES_PER_RAY)
    return fail(GOSURF_ERR_SHAPE, "%d samples per ray (2..%d)", n, GOSURF_MAX_SAMPLES_PER_RAY);
  if (step_index < 0) return fail(GOSURF_ERR_VALUE, "step_index = %d < 0", step_index);
  gs::ImpArgs a{};
  a.g = to_grid(model); a.o = rays->o; a.r = rays->r; a.t = rays->t; a.phi = phi; a.phi_stride = 1;
  a.mlp = mlp; a.M = rays->M; a.n = n; a.n_add = cfg->n_add; a.eps = cfg->weight_eps;
  a.k0 = (uint32_t)(cfg->seed & 0xffffffffu); a.k1 = (uint32_t)(cfg->seed >> 32);
  a.iteration = (uint32_t)cfg->step; a.stream = kImpStream + (uint32_t)step_index;
  a.t_new = t_new; a.ray_of_new = nullptr;
  if ((st = hip_check(gs::launch_importance_step(a, (hipStream_t)stream), "importance step")) != GOSURF_OK)
    return st;
  return ok();
}

gosurf_status gosurf_importance_sample(const gosurf_model* model, const gosurf_params* params,
                                       const gosurf_ray_batch* coarse, const gosurf_importance_cfg* cfg,
                                       gosurf_ray_batch* out, void* ws, size_t ws_bytes, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_params(model, params)) != GOSURF_OK) return st;
  if ((st = check_batch(coarse, false)) != GOSURF_OK) return st;
  if ((st = check_importance_cfg(cfg)) != GOSURF_OK) return st;
  const int M = coarse->M;
  if (coarse->total % M != 0)
    return fail(GOSURF_ERR_SHAPE, "coarse total = %d is not a multiple of M = %d", coarse->total, M);
  const int n0 = coarse->total / M;
  const long long nf = (long long)n0 + (long long)cfg->steps * cfg->n_add;
  if (n0 < 2 || nf > GOSURF_MAX_SAMPLES_PER_RAY)
    return fail(GOSURF_ERR_SHAPE, "%d coarse + %d x %d samples per ray (at most %d)", n0, cfg->steps, cfg->n_add,
                GOSURF_MAX_SAMPLES_PER_RAY);
  if (!out || !out->t || !out->seg || !out->ray_of) return fail(GOSURF_ERR_NULL, "an output array is NULL");
  if (out->M != M || (long long)out->total != (long long)M * nf)
    return fail(GOSURF_ERR_SHAPE, "out has M = %d, total = %d; expected %d, %lld", out->M, out->total, M,
                (long long)M * nf);
  if ((long long)M * nf * 4 >= (1LL << 31)) return fail(GOSURF_ERR_SHAPE, "too many samples");
  const ImpWorkspace w = imp_layout(static_cast<char*>(ws), M, n0, cfg->n_add, cfg->steps);
  if (!ws || ws_bytes < w.bytes)
    return fail(GOSURF_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, w.bytes);
  hipStream_t s = (hipStream_t)stream;

  if ((st = field_phi(model, params, coarse, coarse->t, coarse->ray_of, M * n0, w.out_c, s)) != GOSURF_OK)
    return st;
  const float* t_cur = coarse->t;
  const float* p_cur = w.out_c;
  int p_stride = 4, n = n0;
  float* t_dst = w.tb;
  float* p_dst = w.pb;
  for (int k = 0; k < cfg->steps; ++k) {
    gs::ImpArgs a{};
    a.g = to_grid(model); a.o = coarse->o; a.r = coarse->r; a.t = t_cur; a.phi = p_cur; a.phi_stride = p_stride;
    a.mlp = params->mlp; a.M = M; a.n = n; a.n_add = cfg->n_add; a.eps = cfg->weight_eps;
    a.k0 = (uint32_t)(cfg->seed & 0xffffffffu); a.k1 = (uint32_t)(cfg->seed >> 32);
    a.iteration = (uint32_t)cfg->step; a.stream = kImpStream + (uint32_t)k;
    a.t_new = w.t_new; a.ray_of_new = w.ray_new;
    if ((st = hip_check(gs::launch_importance_step(a, s), "importance step")) != GOSURF_OK) return st;
    if ((st = field_phi(model, params, coarse, w.t_new, w.ray_new, M * cfg->n_add, w.out_n, s)) != GOSURF_OK)
      return st;
    const bool last = k + 1 == cfg->steps;
    gs::ImpMergeArgs mg{};
    mg.ta = t_cur; mg.pa = p_cur; mg.pa_stride = p_stride; mg.na = n;
    mg.tb = w.t_new; mg.pb = w.out_n; mg.pb_stride = 4; mg.nb = cfg->n_add; mg.M = M;
    mg.t_out = last ? out->t : t_dst;
    mg.p_out = last ? nullptr : p_dst;
    mg.ray_of_out = last ? out->ray_of : nullptr;
    mg.seg_out = last ? out->seg : nullptr;
    if ((st = hip_check(gs::launch_importance_merge(mg, s), "importance merge")) != GOSURF_OK) return st;
    t_cur = t_dst; p_cur = p_dst; p_stride = 1; n += cfg->n_add;
    t_dst = (t_dst == w.tb) ? w.ta : w.tb;
    p_dst = (p_dst == w.pb) ? w.pa : w.pb;
  }
  return ok();
}

}  // extern "C"

// ---------------------------------------------------------------- surface extraction
namespace {

struct LatWorkspace {
  float* t;
  int* ray_of;
  float* out4;
  float* o;
  float* r;
  size_t bytes;
};

LatWorkspace lat_layout(char* base, long long nx, long long ny, long long layers) {
  LatWorkspace w{};
  size_t off = 0;
  const size_t n = (size_t)(nx * ny * layers), rows = (size_t)(ny * layers);
  auto take = [&](size_t b) { char* p = base ? base + off : nullptr; off += up(b); return p; };
  w.t = reinterpret_cast<float*>(take(sizeof(float) * n));
  w.ray_of = reinterpret_cast<int*>(take(sizeof(int) * n));
  w.out4 = reinterpret_cast<float*>(take(sizeof(float) * 4 * n));
  w.o = reinterpret_cast<float*>(take(sizeof(float) * 3 * rows));
  w.r = reinterpret_cast<float*>(take(sizeof(float) * 3 * rows));
  w.bytes = off;
  return w;
}

gosurf_status check_lattice(const float* p0, float h, int nx, int ny, int nz) {
  if (!p0) return fail(GOSURF_ERR_NULL, "p0 is NULL");
  if (nx < 2 || ny < 2 || nz < 2) return fail(GOSURF_ERR_SHAPE, "lattice %d x %d x %d (at least 2 each)", nx, ny, nz);
  if (!(h > 0.f) || !std::isfinite(h)) return fail(GOSURF_ERR_VALUE, "lattice spacing must be finite and > 0");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p0[a])) return fail(GOSURF_ERR_VALUE, "p0 must be finite");
  return GOSURF_OK;
}

}  // namespace

extern "C" {

size_t gosurf_lattice_workspace_bytes(int32_t nx, int32_t ny, int32_t layers) {
  if (nx < 1 || ny < 1 || layers < 1) return 0;
  return lat_layout(nullptr, nx, ny, layers).bytes;
}

gosurf_status gosurf_sdf_lattice(const gosurf_model* model, const gosurf_params* params, const float p0[3],
                                 float h, int32_t nx, int32_t ny, int32_t nz, float* phi, void* ws,
                                 size_t ws_bytes, void* stream) {
  gosurf_status st;
  if ((st = check_model(model)) != GOSURF_OK) return st;
  if ((st = check_params(model, params)) != GOSURF_OK) return st;
  if ((st = check_lattice(p0, h, nx, ny, nz)) != GOSURF_OK) return st;
  if (!phi || !ws) return fail(GOSURF_ERR_NULL, "phi or the workspace is NULL");
  // the largest slab that fits the workspace and the field kernel's sample indexing
  long long layers = 0;
  for (long long lo = 1, hi = nz; lo <= hi;) {
    const long long mid = (lo + hi) / 2;
    if (lat_layout(nullptr, nx, ny, mid).bytes <= ws_bytes && (long long)nx * ny * mid * 4 < (1LL << 31)) {
      layers = mid;
      lo = mid + 1;
    } else {
      hi = mid - 1;
    }
  }
  if (layers < 1)
    return fail(GOSURF_ERR_WORKSPACE, "workspace of %zu bytes holds no z-layer (%zu needed)", ws_bytes,
                lat_layout(nullptr, nx, ny, 1).bytes);
  const LatWorkspace w = lat_layout(static_cast<char*>(ws), nx, ny, layers);
  hipStream_t s = (hipStream_t)stream;
  for (int k0 = 0; k0 < nz; k0 += (int)layers) {
    const int L = (int)((nz - k0) < layers ? (nz - k0) : layers);
    gs::LatticeArgs la{};
    for (int a = 0; a < 3; ++a) la.p0[a] = p0[a];
    la.h = h; la.nx = nx; la.ny = ny; la.k0 = k0; la.layers = L;
    la.t = w.t; la.ray_of = w.ray_of; la.o = w.o; la.r = w.r;
    if ((st = hip_check(gs::launch_lattice_rays(la, s), "lattice rays")) != GOSURF_OK) return st;
    gs::FieldArgs fa{};
    fa.g = to_grid(model); fa.grid = params->grid; fa.mlp = params->mlp;
    fa.grid_bf16 = model->precision == GOSURF_BF16 ? params->grid_bf16 : nullptr;
    fa.o = w.o; fa.r = w.r; fa.t = w.t; fa.ray_of = w.ray_of; fa.total = nx * ny * L;
    fa.S = 0; fa.out4 = w.out4; fa.need_gx = 0;
    const int nb = gs::field_grid(fa, false);
    if (nb <= 0) return fail(GOSURF_ERR_HIP, "field grid: the occupancy query failed");
    if ((st = hip_check(gs::launch_field(fa, false, nb, s), "field fwd (lattice)")) != GOSURF_OK) return st;
    if ((st = hip_check(gs::launch_phi_copy(w.out4, (long long)nx * ny * L, phi + (size_t)k0 * nx * ny, s),
                        "lattice copy")) != GOSURF_OK)
      return st;
  }
  return ok();
}

gosurf_status gosurf_marching_tetrahedra(const float* phi, const float p0[3], float h, int32_t nx, int32_t ny,
                                         int32_t nz, float* triangles, int64_t max_triangles, uint32_t* count,
                                         void* stream) {
  gosurf_status st;
  if ((st = check_lattice(p0, h, nx, ny, nz)) != GOSURF_OK) return st;
  if (!phi || !count || (max_triangles > 0 && !triangles)) return fail(GOSURF_ERR_NULL, "an array is NULL");
  if (max_triangles < 0) return fail(GOSURF_ERR_VALUE, "max_triangles < 0");
  if ((long long)(nx - 1) * (ny - 1) * (nz - 1) * 12 >= (1LL << 32))
    return fail(GOSURF_ERR_SHAPE, "lattice too large for a 32-bit triangle count");
  gs::MtArgs a{};
  a.phi = phi;
  for (int q = 0; q < 3; ++q) a.p0[q] = p0[q];
  a.h = h; a.nx = nx; a.ny = ny; a.nz = nz; a.tris = triangles; a.max_tris = max_triangles;
  a.count = reinterpret_cast<unsigned*>(count);
  if ((st = hip_check(gs::launch_marching_tets(a, (hipStream_t)stream), "marching tetrahedra")) != GOSURF_OK)
    return st;
  return ok();
}

}  // extern "C"

