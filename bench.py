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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="room")
    ap.add_argument("--frames", type=int, default=None, help="override the number of frames")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rays", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 1 GiB device copy (reference for memory counters)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain FP32 vs BF16 + proposal comparison")
    ap.add_argument("--compare-pretrain", type=int, default=3000,
                    help="plain steps that train the field before the comparison")
    ap.add_argument("--compare-steps", type=int, default=10, help="timed steps of each compared variant")
    return ap.parse_args()


# Algorithmic bytes per unit of work of the timed kernels (FP32).  The field
# kernels process ray samples and smoothness pairs in one launch:
#   backward, per sample: 4 levels x 8 corners x 16 B gathered (512 B) + 128
#   float atomic adds of 4 B (512 B) + backward seeds (20 B) + depth and ray
#   index (8 B) = 1052 B; per pair: two points of 512 B gathered + 512 B
#   atomics + 12 B position / perturbation = 2072 B;
#   forward, per sample: 512 B gathered + 8 B in + 20 B out = 540 B; per pair:
#   two points of 512 B gathered + 12 B = 1048 B;
#   Adam, per parameter: p, g, m, v read and written (32 B).
BYTES_PER_SAMPLE = {"field_bwd": 1052.0, "field_fwd": 540.0}
BYTES_PER_PAIR = {"field_bwd": 2072.0, "field_fwd": 1048.0}
BYTES_PER_PARAM_ADAM = 32.0


def source_digest():
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2206_14735_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:12]


def measured_traffic(kernel):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    data = json.load(open(path))
    entry = data.get(kernel)
    if not entry or entry.get("source_digest") != source_digest():
        return None
    return entry.get("bytes_per_launch")


def cpu_baseline(w, frames_cpu, grid, mlp, n_rays):
    """FP64 oracle on a bounded sample of the same workload: one step's
    forward+backward on `n_rays` rays (with the proportional share of
    smoothness pairs) over the full grid, plus one dense Adam update of all
    parameters; scaled to the full batch."""
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
    t0 = time.perf_counter()
    res = ostep.evaluate(g64, m64, L, b, ostep.LossCfg(w.lambdas, w.trunc, w.alpha_fs))
    t_fb = time.perf_counter() - t0
    t0 = time.perf_counter()
    ostep.adam(g64, res["grad_grid"].numpy(), np.zeros_like(g64), np.zeros_like(g64), 1, w.lr_grid)
    ostep.adam(m64, res["grad_mlp"].numpy(), np.zeros_like(m64), np.zeros_like(m64), 1, w.lr_mlp)
    t_adam = time.perf_counter() - t0
    t_step = t_fb * (w.M / n_rays) + t_adam
    return {"value": w.M * w.n_samples / t_step, "unit": "ray-samples/s", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"{n_rays} rays x {w.n_samples} samples + {S} smoothness pairs fwd+bwd over the full "
                      f"grid ({t_fb:.1f} s), scaled by {w.M}/{n_rays}, plus one dense Adam step over all "
                      f"{grid.numel() + mlp.numel()} parameters ({t_adam:.1f} s)"}


def compare(a, G, synth, Reconstruction, torch):
    """Plain FP32 against BF16 + learned proposal at the proposal workload's
    batch (65536 rays): the same trained field, iterations/s of whole steps
    and the rendered depth error of each against the noise-free depth.

    The field is trained by plain FP32 steps (6144 rays x (64 + 32)); about
    49k rays' weight distributions are then logged and the proposal trained
    on them; plain rays get 64 + 32 samples, confident proposal rays 24 in the
    predicted interval and the others the plain 96."""
    from paper_2206_14735_amd.proposal import ProposalLog, ProposalTrainer
    wp = synth.configs.ROOM_PROPOSAL
    lay = wp.layout()
    t0 = time.time()
    frames, _ = synth.room_frames(wp.n_frames, H=wp.H, W=wp.W, f=wp.f, seed=1, device="cuda")
    torch.cuda.synchronize()
    print(f"# compare: {wp.n_frames} frames in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)
    span = G.SPAN_BOX
    base = Reconstruction(lay, frames, 64, 32, 6144, 16384, span, wp.near, wp.far, wp.trunc, seed=0)
    t0 = time.time()
    for _ in range(a.compare_pretrain):
        base.step()
    torch.cuda.synchronize()
    print(f"# compare: {a.compare_pretrain} plain steps in {time.time() - t0:.1f} s, losses {base.losses()}",
          file=sys.stderr, flush=True)
    logger = Reconstruction(lay, frames, 64, 32, 4096, 0, span, wp.near, wp.far, wp.trunc, seed=7,
                            grid=base.grid.clone(), mlp=base.mlp.clone())
    log = ProposalLog()
    for k in range(12):
        logger.it = 50_000 + k
        logger.sample()
        log.add(logger, widen=0.05)
    del logger
    trainer = ProposalTrainer(base.model, base.cfg, synth.init_proposal(1), lr=3e-3, batch=8192, cover_tol=0.02)
    t0 = time.time()
    ploss = trainer.fit(base.grid, log, steps=12000)
    torch.cuda.synchronize()
    print(f"# compare: proposal trained on {log.tensors()[0].shape[0]} rays in {time.time() - t0:.1f} s "
          f"(loss {ploss:.4f})", file=sys.stderr, flush=True)

    M, S = wp.M, wp.S
    n_prop = wp.extra["proposal_samples"]
    thr = wp.extra["conf_threshold"]
    dgt = frames.depth_gt.reshape(-1)

    def make(bf16, proposal):
        rec = Reconstruction(lay, frames, 64, 32, M, S, span, wp.near, wp.far, wp.trunc, seed=3,
                             precision=G.BF16 if bf16 else G.FP32, loss_scale=wp.loss_scale if bf16 else 1.0,
                             grid=base.grid.clone(), mlp=base.mlp.clone())
        rec.it = base.it
        if proposal is not None:
            rec.use_proposal(proposal, n_proposal=n_prop, conf_threshold=thr)
        return rec

    def depth_error(rec, n_batches=4):
        errs, samples, conf = [], [], []
        saved_it = rec.it
        for k in range(n_batches):
            rec.it = 200_000 + k
            rec.sample()
            rec.forward()
            ok = rec.batch.depth > 0
            errs.append((rec.fwd.depth_hat[ok] - dgt[rec.batch.pixel][ok]).abs())
            samples.append(rec.batch.n_samples() / M)
            if rec.batch.prop is not None:
                conf.append((rec.batch.prop[:, 2] >= thr).float().mean().item())
        rec.it = saved_it
        e = torch.cat(errs)
        out = {"mean": round(1e3 * e.mean().item(), 3), "median": round(1e3 * e.median().item(), 3)}
        return out, float(sum(samples) / len(samples)), (float(sum(conf) / len(conf)) if conf else None)

    def timed(rec, steps, warmup=3):
        for _ in range(warmup):
            rec.step()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            rec.step()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps

    res = {}
    for name, bf16, prop in (("plain_fp32", False, None), ("bf16_proposal", True, trainer.prop)):
        rec = make(bf16, prop)
        err, spr, conf = depth_error(rec)
        ms = timed(rec, a.compare_steps)
        res[name] = {"ms_per_step": round(ms, 4), "iterations_per_s": round(1e3 / ms, 2),
                     "samples_per_ray": round(spr, 2), "depth_l1_mm": err,
                     "ray_samples_per_s": round(M * spr / (ms * 1e-3)),
                     "plain_equivalent_ray_samples_per_s": round(M * 96 / (ms * 1e-3))}
        if conf is not None:
            res[name]["confident_fraction"] = round(conf, 4)
        print(f"# compare {name}: {res[name]}", file=sys.stderr, flush=True)
        del rec
        torch.cuda.empty_cache()
    p, b = res["plain_fp32"], res["bf16_proposal"]
    return {
        "workload": f"{wp.name}: {M} rays, plain 64+32 vs proposal {n_prop} (fallback 96 below confidence "
                    f"{thr}), {S} smoothness pairs, {wp.n_frames} frames {wp.W}x{wp.H}; field trained by "
                    f"{a.compare_pretrain} plain steps, proposal by 12000 steps on ~49k logged rays",
        **res,
        "iterations_speedup": round(p["ms_per_step"] / b["ms_per_step"], 3),
        "depth_l1_gap_mm": {k: round(b["depth_l1_mm"][k] - p["depth_l1_mm"][k], 3) for k in ("mean", "median")},
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {a.gpus}); the multi-GPU sharding is a design "
              f"described in DESIGN.md and is not run here.", file=sys.stderr)
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
    rec = Reconstruction.from_workload(w, frames, seed=0, grid=grid.clone(), mlp=mlp.clone())

    t0 = time.time()
    for _ in range(a.warmup):
        rec.step()
    torch.cuda.synchronize()
    print(f"# warmup done ({a.warmup} steps, {time.time() - t0:.2f} s), losses {rec.losses()}", file=sys.stderr,
          flush=True)

    # timed region: K whole steps
    t0 = time.perf_counter()
    for _ in range(a.steps):
        rec.step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms = 1e3 * dt / a.steps
    print(f"# timed {a.steps} steps: {ms:.3f} ms/step", file=sys.stderr, flush=True)

    # per-call breakdown with HIP events on the launch stream (separate pass)
    st = torch.cuda.current_stream()
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

    n_par = rec.grid.numel() + rec.mlp.numel()
    losses = rec.losses()
    grid_numel = rec.grid.numel()
    samples_now = rec.batch.n_samples()

    def roofline(name, bytes_per_launch, ms, label):
        gbs = bytes_per_launch / (ms * 1e-3) / 1e9
        traffic = measured_traffic(name)
        return {"kernel": label, "bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes_per_launch, "ms_per_launch": round(ms, 4)}

    pairs = w.S

    def field_bytes(k):
        return BYTES_PER_SAMPLE[k] * samples_now + BYTES_PER_PAIR[k] * pairs

    roofs = {
        "field_bwd": roofline("field_bwd", field_bytes("field_bwd"), kern["field_bwd"],
                              "field_kernel<backward> (gosurf_backward: samples and smoothness pairs)"),
        "field_fwd": roofline("field_fwd", field_bytes("field_fwd"), kern["field_fwd"],
                              "field_kernel<forward> (gosurf_forward: samples and smoothness pairs)"),
        "adam": roofline("adam", BYTES_PER_PARAM_ADAM * n_par, kern["adam"], "adam_kernel (gosurf_adam_step)"),
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
    if not a.no_cpu_baseline:
        fr_cpu = synth.Frames(frames.rgb.cpu(), frames.depth.cpu(), frames.c2w.cpu(), frames.fx, frames.fy,
                              frames.cx, frames.cy)
        print(f"# oracle baseline on {a.cpu_rays} rays ...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(w, fr_cpu, grid, mlp, a.cpu_rays)
        print(f"# oracle baseline: {cpu['sample']}", file=sys.stderr, flush=True)

    comparison = None
    if not a.no_compare:
        del rec
        torch.cuda.empty_cache()
        comparison = compare(a, G, synth, Reconstruction, torch)

    samples = w.M * w.n_samples
    out = {
        "metric": "ray-samples/s per fwd+bwd step, plain FP32 vs BF16+proposal at equal depth L1",
        "value": samples / (ms * 1e-3), "unit": "ray-samples/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms, "iterations_per_s": 1e3 / ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if w.precision == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.M} rays x ({w.n_strat}+{w.n_near}) samples, {w.S} smoothness "
                               f"pairs, grid {'/'.join(str(v) for v in sorted(w.voxels))} m "
                               f"({n_par / 1e6:.2f} M params), {n_frames} frames {w.W}x{w.H}, {w.precision}",
                   "rays": w.M, "samples_per_ray": w.n_samples, "smoothness_pairs": w.S,
                   "grid_params": grid_numel, "frames": n_frames},
        "per_call_ms": {k: round(v, 4) for k, v in per.items()},
        "per_kernel_ms": {k: round(v, 4) for k, v in kern.items()},
        "roofline": roof,
        "other_rooflines": {k: v for k, v in roofs.items() if k != dominant},
        "source_digest": source_digest(),
        "cpu_baseline": cpu,
        "losses": losses,
        "comparison": comparison,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
