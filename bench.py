"""Throughput of the GO-Surf optimisation step on one MI355X.

One step = gosurf_sample_rays + gosurf_forward + gosurf_backward +
gosurf_adam_step over one batch of the room workload (8 x 6 x 3 m room,
1000 synthetic RGB-D frames of 640 x 480, 6144 rays x (64 stratified + 32
near-depth) samples, 16384 smoothness pairs, 4-level grid at
0.03/0.06/0.24/0.96 m = 37.9 M parameters, FP32).  Inputs are generated on the
device before timing; the timed region contains only library calls.

Prints one JSON line: ray-samples/s (rays x samples per ray / step time),
the roofline of the dominant kernel measured with HIP events on the launch
stream, the FP64 oracle timed on a bounded sample on the host cores, and a
comparison of plain FP32 steps with BF16 + learned-proposal steps at 65536
rays on the same trained field (iterations/s and rendered depth error).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_MFMA_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="room")
    ap.add_argument("--frames", type=int, default=None, help="override the number of frames")
    ap.add_argument("--poses", action="store_true",
                    help="optimise per-frame camera poses with the field (pose refinement, Adam at 5e-4)")
    ap.add_argument("--colour-grid", action="store_true",
                    help="the paper's colour path: colour grid at the finest level + view direction, 9-32-32-3")
    ap.add_argument("--grad-copies", action="store_true",
                    help="the backward scatters the large levels into x/y-parity gradient copies")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=0,
                    help="rays of the oracle baseline's sample (0: the workload's whole batch)")
    ap.add_argument("--cpu-reps", type=int, default=7, help="oracle baseline steps timed")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for memory counters)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain FP32 vs BF16 + proposal comparison")
    ap.add_argument("--compare-seeds", type=int, default=3, help="seeds of the comparison")
    ap.add_argument("--proposal-samples", type=int, default=None,
                    help="samples in the predicted interval per confident ray (default: the workload's)")
    ap.add_argument("--depth-midpoint", action="store_true",
                    help="comparison: render depth with each weight at its interval's midpoint (unbiased) in both arms")
    ap.add_argument("--depth-edge", type=float, default=0.0,
                    help="proposal rays at a depth discontinuity larger than this (m) fall back to plain samples")
    ap.add_argument("--free-samples", type=int, default=None,
                    help="samples on the free space before the interval per confident ray (default: the workload's)")
    ap.add_argument("--compare-phase1", type=int, default=600,
                    help="shared plain FP32 steps (65536 rays) before the two continuations")
    ap.add_argument("--compare-phase2", type=int, default=600, help="steps of each continuation (timed)")
    ap.add_argument("--sequential", type=int, default=0,
                    help="also run sequential (online) mapping over this many frames of the room sequence")
    ap.add_argument("--seq-iters", type=int, default=10, help="sequential mapping: steps after each new frame")
    ap.add_argument("--seq-rays", type=int, default=4096, help="sequential mapping: rays per step")
    ap.add_argument("--mesh", type=float, default=0.0,
                    help="also extract the surface on a lattice of this spacing (m) after --mesh-train more steps")
    ap.add_argument("--mesh-train", type=int, default=10000,
                    help="training steps before the extraction (10k: the paper's iteration count)")
    return ap.parse_args()


# Algorithmic bytes per unit of work of the timed kernels.  The field kernels
# process ray samples and smoothness pairs in one launch; a corner is 16 B in
# FP32 and 8 B when the gathers read the bfloat16 mirror (BF16 workloads), so
# one point's 4 levels x 8 corners are g = 512 B (256 B BF16):
#   backward, per sample: g gathered + 128 float atomic adds of 4 B (512 B) +
#   seeds (16 B) + position and Eikonal weight (16 B) = 1056 B (800 B BF16);
#   per pair: 2 g + 2 x 512 B atomics + position and perturbation (24 B)
#   = 2072 B (1560 B BF16);
#   forward, per sample: g + t and ray index (8 B) + outputs (20 B) = 540 B
#   (284 B BF16); per pair: 2 g + 24 B = 1048 B (536 B BF16);
#   Adam, per parameter: p, g, m, v read and written (32 B).
CORNER_BYTES = {"fp32": 16.0, "bf16": 8.0}

# Algorithmic decoder FLOPs of the field kernels (2 per multiply-add; the
# 16-32-32-16 geometry and 15-32-3 colour decoders of Sec. 3.1):
#   forward, per sample: geometry 4096 + colour 1152, plus 3072 for d(phi)/dz
#   through W3 row 0, W2^T and W1^T when the Eikonal term is on; per pair
#   point: 4096 + 3072 (no colour);
#   backward, per sample: the recomputed forward + input gradients of both
#   decoders (5248) + their weight gradients (5248), plus the double
#   backward of the Eikonal term (W1, W2 products 3072 and their weight
#   gradients 3072) when it is on; per pair point: 7168 + 3072 + 3072.
MFMA_PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}   # dense, MI355X


def field_unit_flops(kernel, eikonal):
    """(FLOPs per ray sample, FLOPs per smoothness pair) of one field kernel."""
    fwd = 5248.0 + (3072.0 if eikonal else 0.0)
    pair_point = 7168.0
    if kernel == "field_bwd":
        return fwd + 5248.0 + 5248.0 + (6144.0 if eikonal else 0.0), 2 * (pair_point + 6144.0)
    return fwd, 2 * pair_point


def field_unit_bytes(kernel, precision):
    """(bytes per ray sample, bytes per smoothness pair) of one field kernel."""
    g = 32 * CORNER_BYTES[precision]            # 4 levels x 8 corners
    if kernel == "field_bwd":
        return g + 512.0 + 32.0, 2 * g + 1024.0 + 24.0
    return g + 28.0, 2 * g + 24.0


BYTES_PER_PARAM_ADAM = 32.0


def source_digest():
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2206_14735_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:12]


def measured_mfma(kernel, workload):
    """(issued MFMA FLOPs per launch, MFMA busy fraction) from the committed
    counter summary, if it was taken on the current kernel sources and on
    this workload (else (None, None))."""
    path = os.path.join(ROOT, "profiles", "mfma.json")
    if not os.path.exists(path):
        return None, None
    entry = json.load(open(path)).get(f"{kernel}@{workload}")
    if not entry or entry.get("source_digest") != source_digest():
        return None, None
    return entry.get("flops_per_launch"), entry.get("busy_frac")


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources and on this workload (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    entry = json.load(open(path)).get(f"{kernel}@{workload}")
    if not entry or entry.get("source_digest") != source_digest():
        return None
    return entry.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or '' if unreadable."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def cpu_baseline(w, frames_cpu, grid, mlp, n_rays, reps=1):
    """FP64 oracle on a bounded sample of the same workload: `reps` steps,
    each a forward+backward on `n_rays` rays (with the proportional share of
    smoothness pairs) over the full grid and one dense Adam update of all
    parameters; the forward+backward time is scaled to the full batch."""
    import numpy as np
    import torch

    from oracle import sampler, step as ostep
    from tests.helpers import f32_layout
    L = f32_layout(w.layout())
    S = max(1, round(w.S * n_rays / w.M))
    b, _, _ = sampler.sample_batch(frames_cpu, L, n_rays, w.n_strat, w.n_near, w.span, w.near, w.far, w.trunc,
                                   S, w.delta_s, seed=0, step=0)
    g64 = grid.double().numpy()
    m64 = mlp.double().numpy()
    t_fb = t_adam = 0.0
    for _ in range(reps):
        t0 = time.perf_counter()
        res = ostep.evaluate(g64, m64, L, b, ostep.LossCfg(w.lambdas, w.trunc, w.alpha_fs))
        t_fb += time.perf_counter() - t0
        t0 = time.perf_counter()
        ostep.adam(g64, res["grad_grid"].numpy(), np.zeros_like(g64), np.zeros_like(g64), 1, w.lr_grid)
        ostep.adam(m64, res["grad_mlp"].numpy(), np.zeros_like(m64), np.zeros_like(m64), 1, w.lr_mlp)
        t_adam += time.perf_counter() - t0
        del res
    t_step = (t_fb * (w.M / n_rays) + t_adam) / reps
    scaled = f", scaled by {w.M}/{n_rays}" if n_rays != w.M else ""
    return {"value": w.M * w.n_samples / t_step, "unit": "ray-samples/s", "cores": torch.get_num_threads(),
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"{reps} step(s) of {n_rays} rays x {w.n_samples} samples + {S} smoothness pairs fwd+bwd "
                      f"over the full grid ({t_fb:.1f} s){scaled}, each with one dense Adam step over all "
                      f"{grid.numel() + mlp.numel()} parameters ({t_adam:.1f} s in all)"}


def sequential_measure(a, G, synth, frames, torch):
    """Online mapping over the first a.sequential frames of the room sequence
    with the 3-level grid of the sequential mode (96, 24, 6 cm): frames/s of
    the whole loop (a.seq_iters steps of a.seq_rays rays after each frame),
    then the depth error of the resulting field on the received frames,
    rendered with 64 + 32 samples against the noise-free depth."""
    from paper_2206_14735_amd.train import Reconstruction, SequentialMapper
    n = min(a.sequential, frames.depth.shape[0])
    sm = SequentialMapper(frames, (0.0, 0.0, 0.0), (8.0, 6.0, 3.0), M=a.seq_rays, S=1024,
                          iters_per_frame=a.seq_iters, seed=0)
    sm.add_frame()                       # warm-up: first frame, kernels loaded
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n - 1):
        sm.add_frame()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rec = sm.rec
    seen = sm._frames(n)
    ev = Reconstruction(sm.layout, seen, 64, 32, 16384, 0, G.SPAN_BOX, 0.1, 1e9, 0.1, seed=5, grid=rec.grid,
                        mlp=rec.mlp)
    errs = []
    for k in range(4):
        ev.it = 400_000 + k
        ev.sample()
        ev.forward()
        ok = ev.batch.depth > 0
        errs.append((ev.fwd.depth_hat[ok] - seen.depth_gt.reshape(-1)[ev.batch.pixel][ok]).abs())
    e = torch.cat(errs)
    n_par = rec.grid.numel() + rec.mlp.numel()
    return {"frames": n, "frames_per_s": round((n - 1) / dt, 2), "ms_per_frame": round(1e3 * dt / (n - 1), 3),
            "steps_per_frame": a.seq_iters, "rays_per_step": a.seq_rays, "smoothness_pairs": 1024,
            "ms_per_step": round(1e3 * dt / ((n - 1) * a.seq_iters), 4),
            "grid": "3 levels, 0.96 / 0.24 / 0.06 m", "params": n_par,
            "depth_l1_mm_on_received_frames": {"mean": round(1e3 * e.mean().item(), 3),
                                               "median": round(1e3 * e.median().item(), 3)}}


def mesh_measure(a, G, rec, w, scene, frames, torch):
    """SDF lattice over the grid box and marching tetrahedra on it, timed with
    HIP events; then culling of unobserved surface and the reconstruction
    metrics against the analytic scene (evaluation protocol of the paper's
    supplementary), and |scene SDF| at triangle centroids before culling."""
    from paper_2206_14735_amd import mesh_eval
    for _ in range(a.mesh_train):
        rec.step()
    torch.cuda.synchronize()
    lay = rec.layout
    h = a.mesh
    dims = tuple(int((lay.p1[q] - lay.p0[q]) / h) + 1 for q in range(3))
    nx, ny, nz = dims
    n_pts = nx * ny * nz
    layers = min(nz, 64)
    ws = torch.empty(G.gosurf_lattice_workspace_bytes(nx, ny, layers), dtype=torch.uint8, device="cuda")
    phi = torch.empty(nz, ny, nx, device="cuda")
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    G.gosurf_sdf_lattice(rec.model, rec.grid, rec.mlp, lay.p0, h, dims, phi=phi, workspace=ws,
                         grid_bf16=rec.grid_bf16)              # warm-up
    ev[0].record()
    G.gosurf_sdf_lattice(rec.model, rec.grid, rec.mlp, lay.p0, h, dims, phi=phi, workspace=ws,
                         grid_bf16=rec.grid_bf16)
    ev[1].record()
    cap = 80_000_000
    tris = torch.empty(cap, 3, 3, device="cuda")
    count = torch.empty(1, device="cuda", dtype=torch.int32)
    G.gosurf_marching_tetrahedra(phi, lay.p0, h, cap, triangles=tris, count=count)   # warm-up
    ev[2].record()
    G.gosurf_marching_tetrahedra(phi, lay.p0, h, cap, triangles=tris, count=count)
    ev[3].record()
    torch.cuda.synchronize()
    sdf_ms, mt_ms = ev[0].elapsed_time(ev[1]), ev[2].elapsed_time(ev[3])
    n_tri = G.triangle_count(count)
    kept = min(n_tri, cap)
    gen = torch.Generator(device="cuda").manual_seed(0)
    pick = torch.randint(0, max(kept, 1), (min(kept, 1_000_000),), device="cuda", generator=gen)
    cen = tris[pick].double().mean(1)
    err = scene.sdf(cen).abs() if kept else torch.zeros(1, device="cuda", dtype=torch.float64)
    # per lattice point: 4 levels x 8 corners x 16 B gathered, t and ray index in, 4 outputs out, phi copied
    # Per lattice point the kernel runs the geometry decoder (16-32-32-16: 4096 FLOPs, the colour decoder
    # is skipped) on 4 levels x 8 corners gathered from the caches (neighbouring points share corners),
    # so its bound is the matrix cores; the compulsory HBM bytes are t and the ray index in, the 16-byte
    # output and the phi copy (36 B per point) plus one read of the grid.
    flops_pt = 4096.0
    tfs = flops_pt * n_pts / (sdf_ms * 1e-3) / 1e12
    comp_bytes = 36.0 * n_pts + 4.0 * rec.grid.numel()
    gbs = comp_bytes / (sdf_ms * 1e-3) / 1e9
    t0 = time.perf_counter()
    tk = tris[:kept]
    seen = mesh_eval.visible(tk.mean(1), frames)
    pred, pred_n = mesh_eval.sample_triangles(tk[seen], 1e4, seed=0, normals=True)
    gt = scene.surface_samples(1e4, seed=0).to("cuda")
    gt = gt[mesh_eval.visible(gt, frames)]
    gt_n = scene.normals(gt)
    torch.cuda.synchronize()
    t_cull = time.perf_counter() - t0
    m = mesh_eval.metrics(pred, gt, 0.05, pred_normals=pred_n, gt_normals=gt_n)
    t_eval = time.perf_counter() - t0
    quality = {"culled_triangles_kept": int(seen.sum()), "points_per_cm2": 1,
               **{k: (round(1e3 * v, 3) if k in ("accuracy", "completion", "chamfer_l1") else v) for k, v in m.items()},
               "distance_unit": "mm", "threshold": "5 cm", "cull_s": round(t_cull, 2), "eval_s": round(t_eval, 2)}
    return {"spacing_m": h, "lattice": list(dims), "points": n_pts, "train_steps_before": a.mesh_train,
            "sdf_lattice_ms": round(sdf_ms, 3), "lattice_points_per_s": round(n_pts / (sdf_ms * 1e-3)),
            "sdf_lattice_roofline": {"bound": "mfma", "achieved": round(tfs, 2), "peak": MFMA_PEAK_TFLOPS[w.precision],
                                     "unit": "TFLOP/s", "frac": round(tfs / MFMA_PEAK_TFLOPS[w.precision], 4),
                                     "flops_per_point": flops_pt,
                                     "compulsory_hbm_gb_per_s": round(gbs, 1)},
            "marching_ms": round(mt_ms, 3), "cubes_per_s": round((nx - 1) * (ny - 1) * (nz - 1) / (mt_ms * 1e-3)),
            "triangles": n_tri, "triangle_capacity": cap,
            "unculled_centroid_sdf_mm": {"mean": round(1e3 * float(err.mean()), 3),
                                         "median": round(1e3 * float(err.median()), 3), "centroids": int(pick.numel())},
            "reconstruction": quality}


def subset_frames(synth, fr, idx):
    """The frames `idx` of a sequence (device tensors)."""
    return synth.Frames(fr.rgb[idx].contiguous(), fr.depth[idx].contiguous(), fr.c2w[idx].contiguous(), fr.fx, fr.fy,
                        fr.cx, fr.cy, None if fr.depth_gt is None else fr.depth_gt[idx].contiguous())


def compare(a, G, synth, Reconstruction, torch):
    """Plain FP32 against BF16 + learned proposal on the proposal workload
    (65536 rays per step, 2000 frames).

    Every 50th frame (40 of 2000) is held out: the training steps draw rays
    from the other 1960, and depth errors are measured on the held-out frames
    against their noise-free depth.  Per seed: plain FP32 steps train the
    field (phase 1); about 49k rays' weight distributions are logged from it
    and the proposal is trained on them; then the same state continues for
    the same number of steps once with plain FP32 steps and once with BF16 +
    proposal steps (confident rays: 24 samples in the predicted interval, the
    others the plain 64 + 32).  Reported per seed and summarised over the
    seeds: iterations/s of the two continuations, the held-out depth error
    of the two resulting fields rendered by the same plain FP32 renderer (the
    reconstruction error the proposal adds), and the held-out depth error of
    the proposal-sampled render itself."""
    from paper_2206_14735_amd.proposal import ProposalLog, ProposalTrainer
    wp = synth.configs.ROOM_PROPOSAL
    lay = wp.layout()
    M, S = wp.M, wp.S
    n_prop = wp.extra["proposal_samples"] if a.proposal_samples is None else a.proposal_samples
    n_free = wp.extra["free_samples"] if a.free_samples is None else a.free_samples
    depth_check = wp.extra["depth_check"]
    depth_extend = wp.extra["depth_extend"]
    thr = wp.extra["conf_threshold"]
    cover_tol = wp.extra["cover_tol"]
    span = G.SPAN_BOX
    t0 = time.time()
    frames_all, _ = synth.room_frames(wp.n_frames, H=wp.H, W=wp.W, f=wp.f, seed=1, device="cuda")
    T = wp.n_frames
    held_idx = torch.arange(0, T, 50, device="cuda")
    keep = torch.ones(T, dtype=torch.bool, device="cuda")
    keep[held_idx] = False
    frames = subset_frames(synth, frames_all, torch.nonzero(keep)[:, 0])
    held = subset_frames(synth, frames_all, held_idx)
    del frames_all
    torch.cuda.synchronize()
    print(f"# compare: {T} frames in {time.time() - t0:.1f} s ({len(held_idx)} held out)", file=sys.stderr,
          flush=True)
    dgt = held.depth_gt.reshape(-1)

    def new_rec(bf16, seed, src=None):
        rec = Reconstruction(lay, frames, 64, 32, M, S, span, wp.near, wp.far, wp.trunc, seed=seed,
                             precision=G.BF16 if bf16 else G.FP32, loss_scale=wp.loss_scale if bf16 else 1.0,
                             grid=None if src is None else src.grid.clone(),
                             mlp=None if src is None else src.mlp.clone())
        rec.loss_cfg.depth_midpoint = 1 if a.depth_midpoint else 0
        if src is not None:
            for n in ("grid_m", "grid_v", "mlp_m", "mlp_v"):
                getattr(rec, n).copy_(getattr(src, n))
            rec.it = src.it
            if bf16:
                G.gosurf_refresh_bf16(rec.grid, rec.grid_bf16)
        return rec

    def run(rec, steps):
        for _ in range(3):
            rec.step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        spr = 0.0
        for k in range(steps):
            rec.step()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t) / steps
        # per-call split over a few further steps (HIP events on the launch stream)
        st = torch.cuda.current_stream()
        names = ("sample_rays", "forward", "backward", "adam_step")
        acc = dict.fromkeys(names, 0.0)
        n = 5
        for _ in range(n):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            ev[0].record(st)
            rec.sample()
            ev[1].record(st)
            rec.forward()
            ev[2].record(st)
            spr += rec.batch.n_samples() / M
            rec.backward()
            ev[3].record(st)
            rec.adam()
            ev[4].record(st)
            rec.it += 1
            torch.cuda.synchronize()
            for i, nm in enumerate(names):
                acc[nm] += ev[i].elapsed_time(ev[i + 1]) / n
        return ms, {k: round(v, 4) for k, v in acc.items()}, spr / n

    def one_seed(seed):
        base = new_rec(False, seed)
        t0 = time.time()
        for _ in range(a.compare_phase1):
            base.step()
        torch.cuda.synchronize()
        print(f"# compare seed {seed}: phase 1, {a.compare_phase1} plain steps in {time.time() - t0:.1f} s, "
              f"losses {base.losses()}", file=sys.stderr, flush=True)
        # proposal: log weights of plain forwards on the training frames, train on the device
        logger = Reconstruction(lay, frames, 64, 32, 4096, 0, span, wp.near, wp.far, wp.trunc, seed=7 + 100 * seed,
                                grid=base.grid, mlp=base.mlp)
        log = ProposalLog()
        for k in range(12):
            logger.it = 50_000 + k
            logger.sample()
            log.add(logger, widen=0.05)
        del logger
        trainer = ProposalTrainer(base.model, base.cfg, synth.init_proposal(1 + seed), lr=3e-3, batch=8192,
                                  cover_tol=cover_tol)
        t0 = time.time()
        ploss = trainer.fit(base.grid, log, steps=12000)
        torch.cuda.synchronize()
        n_logged = log.tensors()[0].shape[0]
        print(f"# compare seed {seed}: proposal trained on {n_logged} rays in {time.time() - t0:.1f} s "
              f"(loss {ploss:.4f})", file=sys.stderr, flush=True)
        evaluator = Reconstruction(lay, held, 64, 32, M, 0, span, wp.near, wp.far, wp.trunc, seed=11 + 100 * seed,
                                   grid=base.grid, mlp=base.mlp)
        evaluator.loss_cfg.depth_midpoint = 1 if a.depth_midpoint else 0

        def surface_depth(grid, mlp, b, n1=256, n2=64):
            """Depth of the learned surface along each ray of batch b (sampler-free): the first + to -
            sign change of phi on n1 even samples over the ray's span, then on n2 even samples inside
            that bracket, linearly interpolated.  NaN where phi does not cross zero."""
            Mb = b.M
            seg = b.seg.long()
            lo, hi = b.t[seg[:-1]], b.t[seg[1:] - 1]
            t = lo[:, None] + (hi - lo)[:, None] * torch.linspace(0, 1, n1, device="cuda")[None]
            lc = evaluator.loss_cfg
            for n, last in ((n1, False), (n2, True)):
                sb = G.RayBatch(b.o, b.r, b.rgb, b.depth, t.reshape(-1).contiguous(),
                                (torch.arange(Mb + 1, device="cuda", dtype=torch.int32) * n),
                                torch.arange(Mb, device="cuda", dtype=torch.int32).repeat_interleave(n),
                                torch.zeros(0, 3, device="cuda"), torch.zeros(0, 3, device="cuda"))
                ws = G.workspace_for(evaluator.model, Mb, Mb * n, 0)
                fo = G.gosurf_forward(evaluator.model, grid, mlp, sb, lc, ws)
                phi = fo.sample_values(Mb * n)[0].view(Mb, n)
                cross = (phi[:, :-1] > 0) & (phi[:, 1:] <= 0)
                has = cross.any(1)
                k = cross.float().argmax(1)
                r_ = torch.arange(Mb, device="cuda")
                t0, t1 = t[r_, k], t[r_, k + 1]
                p0, p1 = phi[r_, k], phi[r_, k + 1]
                if not last:
                    t = t0[:, None] + (t1 - t0)[:, None] * torch.linspace(0, 1, n2, device="cuda")[None]
                    found = has
            d = t0 + (t1 - t0) * p0 / (p0 - p1)
            return torch.where(found & has, d, torch.full_like(d, float("nan")))

        def depth_error(grid, mlp, proposal=None, n_batches=4):
            """Rendered depth against the noise-free depth of the held-out frames, on rays with observed depth
            (and, for the plain render, the depth of the learned surface along the same rays)."""
            evaluator.grid, evaluator.mlp = grid, mlp
            evaluator.use_proposal(proposal, n_proposal=n_prop, conf_threshold=thr, n_free=n_free,
                                   depth_check=depth_check, depth_extend=depth_extend, depth_edge=a.depth_edge)
            errs, spr, conf, net_conf, serrs = [], [], [], [], []
            for k in range(n_batches):
                evaluator.it = 300_000 + k
                evaluator.sample()
                evaluator.forward()
                ok = evaluator.batch.depth > 0
                errs.append((evaluator.fwd.depth_hat[ok] - dgt[evaluator.batch.pixel][ok]).abs())
                if proposal is None:
                    sd = surface_depth(grid, mlp, evaluator.batch)
                    serrs.append((sd[ok] - dgt[evaluator.batch.pixel][ok]).abs())
                spr.append(evaluator.batch.n_samples() / M)
                if proposal is not None:
                    conf.append((evaluator.batch.prop[:, 2] >= thr).float().mean().item())
                    net_conf.append((evaluator.batch.prop[:, 2].abs() >= thr).float().mean().item())
            e = torch.cat(errs)
            out = {"depth_l1_mm": {"mean": round(1e3 * e.mean().item(), 3),
                                   "median": round(1e3 * e.median().item(), 3),
                                   "p90": round(1e3 * torch.quantile(e, 0.9).item(), 3),
                                   "p99": round(1e3 * torch.quantile(e, 0.99).item(), 3),
                                   "over_50mm": round((e > 0.05).float().mean().item(), 5)},
                   "samples_per_ray": round(sum(spr) / len(spr), 2)}
            if serrs:
                se = torch.cat(serrs)
                miss = torch.isnan(se)
                sv = se[~miss]
                out["surface_depth_l1_mm"] = {"mean": round(1e3 * sv.mean().item(), 3),
                                              "median": round(1e3 * sv.median().item(), 3),
                                              "p90": round(1e3 * torch.quantile(sv, 0.9).item(), 3),
                                              "over_50mm": round((sv > 0.05).float().mean().item(), 5),
                                              "no_crossing": round(miss.float().mean().item(), 5)}
            if conf:
                out["confident_fraction"] = round(sum(conf) / len(conf), 4)
                out["network_confident_fraction"] = round(sum(net_conf) / len(net_conf), 4)
            return out

        res = {}
        for name, bf16, prop in (("plain_fp32", False, None), ("bf16_proposal", True, trainer.prop)):
            rec = new_rec(bf16, 3 + seed, base)
            if prop is not None:
                rec.use_proposal(prop, n_proposal=n_prop, conf_threshold=thr, n_free=n_free, depth_check=depth_check,
                                 depth_extend=depth_extend, depth_edge=a.depth_edge)
            t0 = time.time()
            ms, per_call, spr = run(rec, a.compare_phase2)
            r = {"ms_per_step": round(ms, 4), "iterations_per_s": round(1e3 / ms, 2), "per_call_ms": per_call,
                 "samples_per_ray": round(spr, 2), "ray_samples_per_s": round(M * spr / (ms * 1e-3)),
                 "plain_equivalent_ray_samples_per_s": round(M * 96 / (ms * 1e-3)),
                 "field": depth_error(rec.grid, rec.mlp)}
            if prop is not None:
                r["proposal_render"] = depth_error(rec.grid, rec.mlp, prop)
            res[name] = r
            print(f"# compare seed {seed} {name}: {r} ({time.time() - t0:.1f} s)", file=sys.stderr, flush=True)
            del rec
            torch.cuda.empty_cache()
        p, b = res["plain_fp32"], res["bf16_proposal"]
        fp, fb = p["field"]["depth_l1_mm"], b["field"]["depth_l1_mm"]
        res["iterations_speedup"] = round(p["ms_per_step"] / b["ms_per_step"], 3)
        res["field_depth_l1_gap_mm"] = {k: round(fb[k] - fp[k], 3) for k in ("mean", "median", "p90")}
        sp, sb_ = p["field"]["surface_depth_l1_mm"], b["field"]["surface_depth_l1_mm"]
        res["surface_depth_l1_gap_mm"] = {k: round(sb_[k] - sp[k], 3) for k in ("mean", "median", "p90")}
        res["n_logged"] = n_logged
        return res

    seeds = [one_seed(k) for k in range(a.compare_seeds)]

    def summary(get):
        v = [get(r) for r in seeds]
        return {"mean": round(sum(v) / len(v), 3), "min": round(min(v), 3), "max": round(max(v), 3)}

    return {
        "workload": f"{wp.name}: {M} rays per step, plain 64+32 vs proposal {n_prop} in the interval + "
                    f"{n_free} on the free space before it per confident ray (confidence >= {thr}"
                    f"{f' and the observed depth within {depth_extend} m of the interval (stretched to it)' if depth_check else ''}"
                    f"{f' and no depth step above {a.depth_edge} m to a neighbouring pixel' if a.depth_edge > 0 else ''}, else plain "
                    f"64+32){'; depth rendered at interval midpoints in both arms' if a.depth_midpoint else ''}, "
                    f"{S} smoothness pairs, {T} frames {wp.W}x{wp.H} of which every 50th is held out "
                    f"for the depth error; per seed {a.compare_phase1} shared plain steps, then "
                    f"{a.compare_phase2} steps of each; proposal trained for 12000 steps on "
                    f"{seeds[0]['n_logged']} logged rays; {a.compare_seeds} seeds",
        "plain_fp32": seeds[0]["plain_fp32"],
        "bf16_proposal": seeds[0]["bf16_proposal"],
        "iterations_speedup": summary(lambda r: r["iterations_speedup"]),
        "field_depth_l1_gap_mm": {k: summary(lambda r, k=k: r["field_depth_l1_gap_mm"][k])
                                  for k in ("mean", "median", "p90")},
        "surface_depth_l1_gap_mm": {k: summary(lambda r, k=k: r["surface_depth_l1_gap_mm"][k])
                                    for k in ("mean", "median", "p90")},
        "held_out_depth_l1_mm": {
            "plain_field": summary(lambda r: r["plain_fp32"]["field"]["depth_l1_mm"]["mean"]),
            "proposal_trained_field": summary(lambda r: r["bf16_proposal"]["field"]["depth_l1_mm"]["mean"]),
            "proposal_render": summary(lambda r: r["bf16_proposal"]["proposal_render"]["depth_l1_mm"]["mean"])},
        "seeds": [{k: v for k, v in r.items() if k != "n_logged"} for r in seeds],
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}): the step's sharding over several GPUs "
              f"is not implemented.", file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2206_14735_amd import gosurf as G
    from paper_2206_14735_amd.train import Reconstruction

    G.lib()
    w = synth.configs.ALL[a.workload]
    n_frames = a.frames or w.n_frames
    t0 = time.time()
    frames, scene = synth.room_frames(n_frames, H=w.H, W=w.W, f=w.f, seed=0, device="cuda") \
        if w.scene == "room" else (synth.sphere_frames().to("cuda"), None)
    torch.cuda.synchronize()
    print(f"# frames ready: {n_frames} x {w.H}x{w.W} in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    grid, mlp = synth.init_params(w.layout(), seed=0)
    rec = Reconstruction.from_workload(w, frames, seed=0, grid=grid.clone(), mlp=mlp.clone(),
                                       grad_copies=a.grad_copies)
    if a.poses:
        rec.use_pose_refinement(lr_pose=5e-4)
    if a.colour_grid:
        rec.use_colour_grid(seed=0)

    t0 = time.time()
    for _ in range(a.warmup):
        rec.step()
    torch.cuda.synchronize()
    print(f"# warmup done ({a.warmup} steps, {time.time() - t0:.2f} s), losses {rec.losses()}", file=sys.stderr,
          flush=True)

    # timed region: K whole steps, with an event between consecutive steps on
    # the launch stream for the distribution of single-step times
    st = torch.cuda.current_stream()
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(a.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev[0].record(st)
    for k in range(a.steps):
        rec.step()
        step_ev[k + 1].record(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / a.steps
    step_ms = sorted(step_ev[k].elapsed_time(step_ev[k + 1]) for k in range(a.steps))
    q = lambda f: step_ms[min(len(step_ms) - 1, int(round(f * (len(step_ms) - 1))))]  # noqa: E731
    step_dist = {"median": round(q(0.5), 4), "p10": round(q(0.1), 4), "p90": round(q(0.9), 4), "steps": a.steps}
    print(f"# timed {a.steps} steps: {ms:.3f} ms/step (median {step_dist['median']}, p10 {step_dist['p10']}, "
          f"p90 {step_dist['p90']})", file=sys.stderr, flush=True)

    # per-call breakdown with HIP events on the launch stream (separate pass)
    names = ["sample_rays", "forward", "backward", "adam_step"]
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(a.steps)]
    for k in range(a.steps):
        e = evs[k]
        e[0].record(st)
        rec.sample()
        e[1].record(st)
        rec.forward()
        e[2].record(st)
        rec.backward()
        e[3].record(st)
        rec.adam()
        e[4].record(st)
        rec.it += 1
    torch.cuda.synchronize()
    per = {n: sum(evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(a.steps)) / a.steps
           for i, n in enumerate(names)}
    print(f"# per call (ms): {per}", file=sys.stderr, flush=True)

    # per-kernel durations: HIP events recorded by the library around each launch
    kern = {}
    for name, kid in (("field_fwd", G.KERNEL_FIELD_FWD), ("field_bwd", G.KERNEL_FIELD_BWD),
                      ("adam", G.KERNEL_ADAM)):
        pairs = []
        for _ in range(a.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)   # creates the events; the library re-records them around the kernel
            e1.record(st)
            G.gosurf_time_kernel(kid, e0, e1)
            rec.step()
            pairs.append((e0, e1))
        G.gosurf_time_kernel(0)
        torch.cuda.synchronize()
        kern[name] = sum(x.elapsed_time(y) for x, y in pairs) / len(pairs)
    print(f"# per kernel (ms): {kern}", file=sys.stderr, flush=True)

    n_par = rec.grid.numel() + rec.mlp.numel() + (0 if rec.cgrid is None else rec.cgrid.numel() + rec.cmlp.numel())
    losses = rec.losses()
    grid_numel = rec.grid.numel()
    samples_now = rec.batch.n_samples()

    def roofline(name, bytes_per_launch, ms, label):
        gbs = bytes_per_launch / (ms * 1e-3) / 1e9
        traffic = measured_traffic(name, w.name + ("+copies" if a.grad_copies else ""))
        return {"kernel": label, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes_per_launch, "ms_per_launch": round(ms, 4)}

    pairs = w.S

    def field_bytes(k):
        per_sample, per_pair = field_unit_bytes(k, w.precision)
        return per_sample * samples_now + per_pair * pairs

    roofs = {
        "field_bwd": roofline("field_bwd", field_bytes("field_bwd"), kern["field_bwd"],
                              "field_kernel<backward> (gosurf_backward: samples and smoothness pairs)"),
        "field_fwd": roofline("field_fwd", field_bytes("field_fwd"), kern["field_fwd"],
                              "field_kernel<forward> (gosurf_forward: samples and smoothness pairs)"),
        # the timed launch is the step's first Adam call: the geometry grid and the decoders
        "adam": roofline("adam", BYTES_PER_PARAM_ADAM * (rec.grid.numel() + rec.mlp.numel()), kern["adam"],
                         "adam_kernel (gosurf_adam_step)"),
    }
    eikonal = w.lambdas[4] > 0

    def mfma_roofline(k, label):
        per_sample, per_pair = field_unit_flops(k, eikonal)
        flops = per_sample * samples_now + per_pair * pairs
        tfs = flops / (kern[k] * 1e-3) / 1e12
        peak = MFMA_PEAK_TFLOPS[w.precision]
        issued, busy = measured_mfma(k, w.name + ("+copies" if a.grad_copies else ""))
        return {"kernel": label, "bound": "mfma", "achieved": round(tfs, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(tfs / peak, 4), "algorithmic_flops_per_launch": flops, "issued_flops_per_launch": issued,
                "mfma_busy": busy, "ms_per_launch": round(kern[k], 4)}

    mfma_roofs = {
        "field_bwd_mfma": mfma_roofline("field_bwd", "field_kernel<backward>: decoder FLOPs on MFMA"),
        "field_fwd_mfma": mfma_roofline("field_fwd", "field_kernel<forward>: decoder FLOPs on MFMA"),
    }
    dominant = max(("field_fwd", "field_bwd", "adam"), key=lambda k: kern[k])
    roof = roofs[dominant]

    if a.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)   # elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        print("# calibration copy: 1 GiB read + 1 GiB written", file=sys.stderr, flush=True)

    cpu = None
    if "importance_steps" in w.extra and not a.no_cpu_baseline:
        # the oracle baseline covers the stratified step; this workload's step also samples by importance
        print("# oracle baseline: not run for the importance-sampling workload", file=sys.stderr, flush=True)
    elif a.poses or a.colour_grid:
        print("# oracle baseline: not run with --poses or --colour-grid (it times the plain step)", file=sys.stderr,
              flush=True)
    elif not a.no_cpu_baseline:
        fr_cpu = synth.Frames(frames.rgb.cpu(), frames.depth.cpu(), frames.c2w.cpu(), frames.fx, frames.fy,
                              frames.cx, frames.cy)
        n_cpu = a.cpu_rays if 0 < a.cpu_rays < w.M else w.M
        print(f"# oracle baseline: {a.cpu_reps} step(s) on {n_cpu} rays ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, fr_cpu, grid, mlp, n_cpu, a.cpu_reps)
        print(f"# oracle baseline: {cpu['sample']}", file=sys.stderr, flush=True)

    spr = rec.total // w.M                 # samples per ray of the batch the step trains on
    mesh = None
    if a.mesh > 0:
        if scene is None:
            raise SystemExit("--mesh needs a room workload (its analytic scene judges the accuracy)")
        mesh = mesh_measure(a, G, rec, w, scene, frames, torch)
        print(f"# mesh: {mesh}", file=sys.stderr, flush=True)
    sequential = None
    if a.sequential > 0:
        if scene is None:
            raise SystemExit("--sequential needs a room workload")
        sequential = sequential_measure(a, G, synth, frames, torch)
        print(f"# sequential: {sequential}", file=sys.stderr, flush=True)
    comparison = None
    if not a.no_compare:
        del rec
        torch.cuda.empty_cache()
        comparison = compare(a, G, synth, Reconstruction, torch)

    samples = w.M * spr
    if "importance_steps" in w.extra:
        sampling = (f"({w.n_strat} stratified + {w.extra['importance_steps']} importance steps of "
                    f"{w.extra['importance_add']}) samples")
    else:
        sampling = f"({w.n_strat}+{w.n_near}) samples"
    out = {
        "metric": "ray-samples/s per fwd+bwd step, plain FP32 vs BF16+proposal at equal depth L1",
        "value": samples / (ms * 1e-3), "unit": "ray-samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "step_ms": step_dist, "iterations_per_s": 1e3 / ms,
        "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if w.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.M} rays x {sampling}, {w.S} smoothness "
                               f"pairs, grid {'/'.join(str(v) for v in sorted(w.voxels))} m "
                               f"({n_par / 1e6:.2f} M params), {n_frames} frames {w.W}x{w.H}, {w.precision}"
                               + (", with camera pose refinement" if a.poses else "")
                               + (", colour from the colour grid (the paper's colour path)" if a.colour_grid else "")
                               + (", gradient copies" if a.grad_copies else ""),
                   "rays": w.M, "samples_per_ray": spr, "smoothness_pairs": w.S,
                   "grid_params": grid_numel, "frames": n_frames},
        "per_call_ms": {k: round(v, 4) for k, v in per.items()},
        "per_kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "roofline": roof,
        "other_rooflines": {**{k: v for k, v in roofs.items() if k != dominant}, **mfma_roofs},
        "source_digest": source_digest(),
        "cpu_baseline": cpu,
        "losses": losses,
        "comparison": comparison,
    }
    if mesh is not None:
        out["mesh"] = mesh
    if sequential is not None:
        out["sequential_mapping"] = sequential
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
