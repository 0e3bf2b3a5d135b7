#!/usr/bin/env python3
"""CTV-FGP throughput on one MI355X.

Workload (one "step"): the masked 2048 x 2048 complex64 denoising problem
(200 random disks/rectangles, noise sigma 0.15, lambda 0.08, |x| <= 1 with a
square support covering 70 % of the pixels), solved with 200 FGP iterations for
each of the four complex TV kinds (type-I/II, isotropic/anisotropic), the four
solves submitted as one batched plan (one HIP graph). Inputs are synthetic and
seeded, resident in HBM before timing starts.

Prints one JSON line: Mpixel-iterations/s over the timed steps, the roofline
record of the dominant kernel (the batched fused FGP tile kernel; average
launch duration from HIP events on the stream the graph runs on), the same
solves as four plain calls and with every tile run, and the FP64 CPU oracle
timed on a bounded sample of the same workload.

Each problem runs in the launch configuration (tile shape, iterations fused
per launch) the library's autotuner chose for it: from the saved tuning table
of this GPU model, or tuned live before the warm-up when the table lacks it.
The fused kernel performs several iterations per launch, so its real memory
traffic is far below the per-iteration algorithmic bytes: it is bound by VALU
issue. `roofline` reports the algorithmic FP32 FLOP/s (FMA = 2) against the
published 157.3 TFLOP/s vector peak; as secondary fields the algorithmic
operations per second against the VALU issue peak of the library's code (it is
compiled without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz), the measured HBM traffic of the
committed PMC profile per second against the 8 TB/s peak (the metric's "%HBM",
when the kernel sources are unchanged since the profile was taken) and the
bytes an unfused solver would move (57 B per pixel-iteration), whose ratio to
the HBM peak exceeds 1 because of fusion.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1] [--tuning auto|live|off] [--save-tuning PATH]
"""
import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
FP32_VECTOR_PEAK_TFLOPS = 157.3
# VALU issue peak without packed FP32 (the library is compiled with packed-FP32
# code generation disabled): 256 CUs x 4 SIMDs x 16 lanes, one operation per
# lane per cycle at 2.4 GHz.
VALU_OPS_PEAK_GOPS = 256 * 4 * 16 * 2.4
BYTES_PER_PX_IT_MASKED = 57    # read b 8 + q 16 + r 16 + mask 1, write q 16 (per pixel-iteration)
FLOPS_PER_PX_IT = {"1i": 52, "1a": 52, "2i": 52, "2a": 44}
# Arithmetic operations of one pixel-iteration as written in the per-pixel
# operators (a fused multiply-add, a reciprocal square root, a min or a max
# each count once): L^T and w 8, P_C with the modulus bound and the support 7,
# the dual step 8, the P_S scale or clip 6 / 8 / 10 / 8, the in-place update 12.
OPS_PER_PX_IT = {"1i": 41, "1a": 43, "2i": 45, "2a": 43}
KIND_INDEX = {"1i": 0, "1a": 1, "2i": 2, "2a": 3}
# Unfused algorithmic bytes of the secondary workloads: the backward per
# pixel-iteration (recompute 56 + r history 16 + reverse step 120 - rounded
# to 190), and one phase-retrieval outer iteration per pixel (FGP 20 x 56 +
# 10 FFT2 x 2 passes x 16 B + H 64 + y 16 + the sum over distances 64 + FISTA
# 48), of which the FFT side (everything but the FGP prox) is 464 B.
ADJ_BYTES_PER_PX_IT = 190
PR_BYTES_PER_PX_OUTER = 1640
PR_FFT_BYTES_PER_PX_OUTER = 464
ADJ_PROFILES = ("adjoint_16x512sq_K50_ckpt10_stats.md", "adjoint_16x512sq_K50_ckpt10_pmc.md")
PR_PROFILES = ("pr_1024sq_D4_100x20_stats.md", "pr_1024sq_D4_100x20_pmc.md")
PMC_PROFILE = "fgp_batched_kernel_2048sq_masked_4kinds_K200_pmc.md"
ROOT = os.path.dirname(os.path.abspath(__file__))
TUNING_TABLE = os.path.join(ROOT, "paper_2109_05496_amd", "tuning", "mi355x.jsonl")


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--fuse", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=20)
    ap.add_argument("--pr-oracle", action="store_true",
                    help="also run the full phase-retrieval problem in the FP64 oracle (minutes) and report the "
                         "GPU's end-to-end error against it")
    ap.add_argument("--cpu-batch-iters", type=int, default=4,
                    help="iterations per image of the all-cores oracle run over the ragged batch")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the secondary measurements (batched ragged workload, ...)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run three 1 GiB device-to-device copies (byte-counter calibration under rocprofv3)")
    ap.add_argument("--tuning", choices=("auto", "live", "off"), default="auto",
                    help="launch configuration: auto = the saved tuning table, and the autotuner (untimed, "
                         "before the warm-up) for problems it does not cover; live = autotune every problem; "
                         "off = the library default")
    ap.add_argument("--tuning-table", default=TUNING_TABLE)
    ap.add_argument("--save-tuning", default=None, help="write the tuning table here at the end")
    ap.add_argument("--only", choices=("adjoint", "pr", "small"), default=None,
                    help="run only this secondary measurement, timed part only (for profiling it); prints "
                         "{\"only\": ..., <entry>: {...}} instead of the result line")
    return ap.parse_args()


class Tuner:
    """Chooses the launch configuration of each benchmarked problem with the
    library's autotuner (outside every timed region)."""

    def __init__(self, ctv, mode, table):
        self.ctv, self.mode, self.table = ctv, mode, None
        if mode == "auto" and table and os.path.exists(table):
            ctv.tune_cache_load(table)
            self.table = os.path.relpath(table, ROOT)

    def plain(self, b, lam, kind, alpha, constraint, support, iters, out=None, workspace=None):
        if self.mode == "off":
            return "default"
        if self.mode == "auto" and self.ctv.tuned(b.shape[-2], b.shape[-1], batch=1 if b.dim() == 2 else b.shape[0],
                                                  kind=kind, constraint=constraint, iters=iters) is not None:
            return "table"
        self.ctv.autotune(b, lam, kind=kind, alpha=alpha, constraint=constraint, support=support, iters=iters,
                          reps=3, out=out, workspace=workspace)
        return "live"

    def batched(self, images, b_packed, support_packed=None):
        if self.mode == "off":
            return "default"
        if self.mode == "auto" and self.ctv.batched_tuned(images) is not None:
            return "table"
        self.ctv.autotune_batched(images, b_packed, support_packed, reps=2)
        return "live"


def _oracle_kind(args):
    """One kind of the sample in a worker process: the worker builds the same
    seeded input itself (outside the timing) and returns the oracle's time."""
    kind, iters, size = args
    import numpy as np

    import synth
    from oracle import tv
    c = synth.config2(0, size=size)
    b = c["b"].astype(np.complex128)
    t0 = time.perf_counter()
    tv.fgp(b, c["lam"], iters, kind, c["alpha"], c["constraint"], c["mask"])
    return time.perf_counter() - t0


def _cpu_model():
    """The host CPU as /proc/cpuinfo names it, with family / model / stepping
    (some hosts report only a short model name)."""
    info = {}
    try:
        for line in open("/proc/cpuinfo"):
            if ":" in line:
                k, v = (t.strip() for t in line.split(":", 1))
                if k in ("model name", "cpu family", "model", "stepping", "vendor_id") and k not in info:
                    info[k] = v
            if not line.strip() and info:
                break
    except OSError:
        pass
    if not info:
        return "unknown"
    return (f"{info.get('model name', '?')} (vendor {info.get('vendor_id', '?')}, family {info.get('cpu family', '?')}, "
            f"model {info.get('model', '?')}, stepping {info.get('stepping', '?')})")


def _oracle_image(args):
    """One image of the ragged batch in a pool worker: (index, seconds of the
    oracle's solve at `iters` iterations); the worker rebuilds the seeded batch
    itself, outside the timing."""
    idx, iters = args
    import numpy as np

    import synth
    from oracle import tv
    global _BATCH3
    try:
        _BATCH3
    except NameError:
        _BATCH3 = synth.config3(0)
    d = _BATCH3[idx]
    t0 = time.perf_counter()
    tv.fgp(d["b"].astype(np.complex128), d["lam"], iters, d["kind"])
    return idx, time.perf_counter() - t0


def cpu_batched_pool(iters):
    """The oracle over all 256 ragged images on every host core: a process pool
    of len(sched_getaffinity) workers, images handed out largest first (LPT by
    m n), `iters` iterations each (a bounded sample of the 150)."""
    import multiprocessing as mp

    import synth
    imgs = synth.config3(0)
    order = sorted(range(len(imgs)), key=lambda i: -imgs[i]["b"].size)
    px_it = sum(d["b"].size for d in imgs) * iters
    workers = len(os.sched_getaffinity(0))
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_image, [(i, 0) for i in range(workers)], chunksize=1)   # workers build the batch first
        t0 = time.perf_counter()
        pool.map(_oracle_image, [(i, iters) for i in order], chunksize=1)
        dt = time.perf_counter() - t0
    return {"value": round(px_it / dt / 1e6, 2), "unit": "Mpixel-iters/s", "cores": workers,
            "sample": f"256 ragged images (sides 128..1024), {iters} FGP iterations each, "
                      f"largest first over {workers} worker processes ({dt:.1f} s)"}


def cpu_baseline(c, sample_iters):
    """The FP64 numpy oracle, as it stands, on a bounded sample of the same
    workload: every kind on the full image for `sample_iters` iterations, once
    on one core (the kinds in sequence) and once with the four kinds, which are
    independent problems, in four worker processes (started fresh, so they
    share nothing with this process's GPU context). The parallel figure is
    the reported value."""
    import multiprocessing as mp

    import numpy as np
    from oracle import tv
    b = c["b"].astype(np.complex128)
    n_px = b.size
    kinds = list(c["kinds"])
    work = len(kinds) * n_px * sample_iters
    t0 = time.perf_counter()
    for kind in kinds:
        tv.fgp(b, c["lam"], sample_iters, kind, c["alpha"], c["constraint"], c["mask"])
    dt1 = time.perf_counter() - t0
    workers = min(len(kinds), os.cpu_count() or 1)
    with mp.get_context("spawn").Pool(workers) as pool:
        # the kinds run concurrently; the slowest worker's oracle time is the sample's duration
        dtp = max(pool.map(_oracle_kind, [(k, sample_iters, b.shape[0]) for k in kinds], chunksize=1))
    threads = int(os.environ.get("OMP_NUM_THREADS", "1") or 1)
    return {"value": work / dtp / 1e6, "unit": "Mpixel-iters/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(kinds)} kinds x {sample_iters} FGP iterations on the full {b.shape[0]}x{b.shape[1]} "
                      f"masked image, one kind per worker process ({dtp:.1f} s, slowest worker; numpy float64, "
                      f"single-threaded elementwise; OMP_NUM_THREADS={threads})",
            "single_core": {"value": work / dt1 / 1e6, "cores": 1, "seconds": round(dt1, 2)},
            "host_cores": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model(), "numpy": np.__version__}


def pr_end_to_end(ctv, synth, torch, dev):
    """The full phase-retrieval run (1024^2, D = 4, 100 x 20, FISTA) on the GPU
    and in the FP64 oracle on the same measurements (simulated with the
    oracle's propagator): the end-to-end relative L2 error of x, and the
    oracle's time on one core. Minutes of CPU work, so only with --pr-oracle."""
    import numpy as np
    from oracle import pr as opr
    P = synth.PR_DEFAULTS
    truth = synth.config5_object(seed=0)
    m = truth.shape[0]
    Hs = [opr.transfer(m, m, d, P["wavelength"], P["pixel"]) for d in P["distances"]]
    rng = np.random.default_rng(0)
    y = np.stack([synth.poisson_measure(np.abs(opr.A(truth, H)) ** 2, P["photons"], rng) for H in Hs])
    xg = ctv.phase_retrieval(torch.as_tensor(y).to(dev), P["distances"], P["wavelength"], P["pixel"], tau=P["tau"],
                             gamma=P["gamma"], outer=P["outer"], inner=P["inner"]).cpu().numpy()
    t0 = time.perf_counter()
    xo, _ = opr.fista(y.astype(np.float64), P["distances"], P["wavelength"], P["pixel"], P["outer"], P["inner"],
                      P["tau"], P["gamma"])
    dt = time.perf_counter() - t0
    px_it = m * m * P["outer"] * P["inner"]
    return {"workload": "1024^2, D=4, 100 outer x 20 FGP iterations (FISTA), same measurements on both sides",
            "rel_l2_x": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
            "elementwise_x": float(np.abs(xg - xo).max() / np.abs(xo).max()),
            "phase_rmse_gpu": phase_rmse(xg, truth), "phase_rmse_oracle": phase_rmse(xo, truth),
            "oracle_seconds": round(dt, 1), "oracle_fgp_Mpx_it_s_equiv": round(px_it / dt / 1e6, 2), "cores": 1}


def timed(fn, reps, torch, stream):
    """Average milliseconds of fn() over reps, bracketed by HIP events."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def bench_batched(ctv, synth, torch, dev, tuner, reps=3):
    """Ragged batch: 256 images with sides ~ U{128..1024}, per-image lambda and
    kind, 150 iterations, as one HIP-graph launch vs 256 plain calls."""
    imgs = synth.config3(0)
    descs = [dict(m=d["b"].shape[0], n=d["b"].shape[1], lam=d["lam"], kind=d["kind"], alpha=0.5,
                  iters=d["iters"]) for d in imgs]
    plan = ctv.BatchedPlan(descs)
    bp = plan.pack([d["b"] for d in imgs], device=dev)
    source = tuner.batched(descs, bp)
    if source == "live":
        plan.close()
        plan = ctv.BatchedPlan(descs)
    tiling = plan.tiling
    xp = torch.empty_like(bp)
    stream = torch.cuda.current_stream(dev)
    ms_graph = timed(lambda: plan.run(bp, out=xp), reps, torch, stream)
    bs = [torch.as_tensor(d["b"]).to(dev) for d in imgs]
    xs = [torch.empty_like(t) for t in bs]
    ws = torch.empty(max(ctv.workspace_size(d["m"], d["n"], 1, iters=d["iters"])[0] for d in descs),
                     dtype=torch.uint8, device=dev)

    def plain_all():
        for d, t, x in zip(imgs, bs, xs):
            ctv.denoise(t, d["lam"], kind=d["kind"], iters=d["iters"], out=x, workspace=ws)

    ms_plain = timed(plain_all, reps, torch, stream)
    same = all(torch.equal(a.view(torch.float32), x.view(torch.float32)) for a, x in zip(plan.unpack(xp), xs))
    px_it = sum(d["b"].size * d["iters"] for d in imgs)
    plan.close()
    return {"workload": "256 complex64 images, sides ~ U{128..1024}, lambda log-U[0.01,0.2], kinds 1i/1a, K=150",
            "tuning": {"fuse": tiling[0], "tile": list(tiling[1:]), "source": source}, "px_iters": px_it, "graph_ms": round(ms_graph, 3), "plain_256_calls_ms": round(ms_plain, 3),
            "speedup": round(ms_plain / ms_graph, 3), "graph_Mpx_it_s": round(px_it / ms_graph / 1e3, 1),
            "plain_Mpx_it_s": round(px_it / ms_plain / 1e3, 1), "bitwise_equal_to_plain": bool(same)}


def profile_figures(names, marker, keep):
    """Per-kernel figures of a secondary workload from its committed rocprofv3
    summaries (kernel-trace statistics and PMC counters of `bench.py --only`):
    launches per unit (the launches of the kernel whose name contains `marker`
    run once per unit), average duration, measured traffic per launch and its
    rate, VALU issue utilisation. Kernels whose names contain none of `keep` are
    left out. None while the kernel sources differ from the profiled ones."""
    from paper_2109_05496_amd import prof_summary
    st = prof_summary.load_summary(os.path.join(ROOT, "profiles", names[0]))
    pm = prof_summary.load_summary(os.path.join(ROOT, "profiles", names[1]))
    if not st:
        return None
    per_unit = next((v["calls"] for k, v in st["kernels"].items() if marker in k), None)
    if not per_unit:
        return None
    out = {}
    for k, v in st["kernels"].items():
        if not any(s in k for s in keep):
            continue
        p = pm["kernels"].get(k) if pm else None
        d = {"launches_per_unit": round(v["calls"] / per_unit, 3), "avg_us": v["avg_us"],
             "traffic_bytes": p["traffic_bytes"] if p else None,
             "valu_issue_frac": p["valu_issue_frac"] if p else None}
        if p and p["traffic_bytes"]:
            gbs = p["traffic_bytes"] / (v["avg_us"] * 1e-6) / 1e9
            d["hbm"] = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(gbs / HBM_PEAK_GBS, 4)}
        out[k] = d
    return out


def _per_unit(figs, select, field):
    """Sum over the selected kernels of launches per unit x field (None if any is missing)."""
    tot = 0.0
    for k, d in figs.items():
        if select(k):
            if d.get(field) is None:
                return None
            tot += d["launches_per_unit"] * d[field]
    return tot


def bench_adjoint(ctv, synth, torch, dev, reps=3):
    """16 x 512^2, type-1i, lambda 0.05, K = 50 with checkpoints every 10:
    forward (storing checkpoints) and hand-written backward."""
    c = synth.config4(0)
    b = torch.as_tensor(c["b"]).to(dev)
    B, m, n = b.shape
    K, ck = c["iters"], c["ckpt_every"]
    gx = torch.ones_like(b)
    stream = torch.cuda.current_stream(dev)
    state = {}

    def fwd():
        state["x"], state["saved"] = ctv.denoise(b, c["lam"], kind="1i", iters=K, ckpt_every=ck)

    def bwd():
        ctv.denoise_backward(b, [c["lam"]] * B, gx, state["saved"], kind="1i", iters=K, ckpt_every=ck)

    ms_f = timed(fwd, reps, torch, stream)
    ms_b = timed(bwd, reps, torch, stream)
    px_it = B * m * n * K
    # roofline of the backward: the unfused algorithmic bytes per backward
    # pixel-iteration over the live backward time, and (from the committed
    # profiles) each backward kernel's duration, measured traffic and VALU issue;
    # launches per unit = per backward call
    figs = profile_figures(ADJ_PROFILES, "adj_output_kernel", ("adj_", "lam_final", ", true>("))
    alg_gbs = ADJ_BYTES_PER_PX_IT * px_it / (ms_b * 1e-3) / 1e9
    traffic = _per_unit(figs, lambda k: True, "traffic_bytes") if figs else None
    kern_us = _per_unit(figs, lambda k: True, "avg_us") if figs else None
    step_k = next((k for k in figs if "adj_step_kernel" in k), None) if figs else None
    sk = figs[step_k] if step_k else None
    # the block prices the backward against HBM (its unfused byte model); the
    # profiles say which unit of the dominant (reverse-step) kernel is busier:
    # VALU issue or HBM
    limiter = None
    if sk and sk.get("valu_issue_frac") is not None and sk.get("hbm"):
        limiter = {"valu_issue_frac": sk["valu_issue_frac"], "hbm_frac": sk["hbm"]["frac"],
                   "busier": "VALU issue" if sk["valu_issue_frac"] > sk["hbm"]["frac"] else "HBM"}
    roof = {"bound": "hbm", "achieved": round(alg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(alg_gbs / HBM_PEAK_GBS, 4), "bytes_per_px_it": ADJ_BYTES_PER_PX_IT,
            "basis": "unfused model (recompute 56 + r history 16 + reverse step ~120 B per backward px-it) over "
                     "the live backward time; fusion keeps the real traffic below it",
            "traffic": round(traffic) if traffic is not None else None,
            "hbm": ({"achieved": round(traffic / (ms_b * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(traffic / (ms_b * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "what": "measured bytes of one backward (profiles) over the live backward time"}
                    if traffic is not None else None),
            "dominant_kernel": step_k, "dominant_kernel_limiter": limiter,
            "profiled_kernel_time_ms": round(kern_us / 1e3, 3) if kern_us is not None else None,
            "kernels": figs}
    return {"workload": "16 x 512^2 complex64, type-1i, lambda 0.05, K=50, checkpoints every 10",
            "forward_ms": round(ms_f, 3), "backward_ms": round(ms_b, 3),
            "forward_Mpx_it_s": round(px_it / ms_f / 1e3, 1), "backward_Mpx_it_s": round(px_it / ms_b / 1e3, 1),
            "backward_over_forward": round(ms_b / ms_f, 2), "roofline": roof}


def bench_pr(ctv, synth, torch, dev, tuner, reps=2, extras=True):
    """1024^2 object, 4 distances (1.0-2.5 mm, 532 nm, 4 um), Poisson 1000
    photons/pixel; 100 FISTA iterations x 20 FGP iterations (tau 0.01, gamma 1/4).
    The measurements are simulated with the library's own propagator."""
    import numpy as np
    P = synth.PR_DEFAULTS
    truth = synth.config5_object(seed=0)
    m = truth.shape[0]
    fields = ctv.pr_forward(torch.as_tensor(truth.astype(np.complex64)).to(dev), P["distances"],
                            P["wavelength"], P["pixel"])
    inten = (fields.abs() ** 2).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    y = torch.as_tensor(np.stack([synth.poisson_measure(I, P["photons"], rng) for I in inten])).to(dev)
    stream = torch.cuda.current_stream(dev)
    out = {}
    # the prox is ctv_denoise's problem class (1i, |x| <= 1, batch 1, m x m, K_in)
    source = tuner.plain(torch.as_tensor(truth.astype(np.complex64)).to(dev), P["tau"] * P["gamma"], "1i", 0.5,
                         "modulus", None, P["inner"])
    T, _, tw, tr = ctv.tiling(0, P["inner"], m, m, detail=True)

    def run():
        out["x"] = ctv.phase_retrieval(y, P["distances"], P["wavelength"], P["pixel"], tau=P["tau"],
                                       gamma=P["gamma"], outer=P["outer"], inner=P["inner"])

    ms = timed(run, reps, torch, stream)
    fgp_px_it = m * m * P["outer"] * P["inner"]
    outer_us = ms * 1e3 / P["outer"]
    # roofline of an outer iteration: the unfused algorithmic bytes per pixel
    # over the live time, and per kernel (committed profiles; launches per unit
    # = per outer iteration, whose gradient runs the accumulate-inverse pass
    # once) the FFT side against its own 464 B per pixel
    figs = profile_figures(PR_PROFILES, "fft_acc_inverse_kernel", ("fft_", "fgp_", "transpose", "loss_final"))
    is_fft = lambda k: "fft_" in k or "transpose" in k  # noqa: E731
    alg_gbs = PR_BYTES_PER_PX_OUTER * m * m / (outer_us * 1e-6) / 1e9
    fft_us = _per_unit(figs, is_fft, "avg_us") if figs else None
    all_us = _per_unit(figs, lambda k: True, "avg_us") if figs else None
    fft_traffic = _per_unit(figs, is_fft, "traffic_bytes") if figs else None
    traffic = _per_unit(figs, lambda k: True, "traffic_bytes") if figs else None
    fft = None
    if fft_us:
        fft_gbs = PR_FFT_BYTES_PER_PX_OUTER * m * m / (fft_us * 1e-6) / 1e9
        fft = {"bound": "hbm", "achieved": round(fft_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(fft_gbs / HBM_PEAK_GBS, 4), "bytes_per_px": PR_FFT_BYTES_PER_PX_OUTER,
               "traffic": round(fft_traffic) if fft_traffic is not None else None,
               "hbm": ({"achieved": round(fft_traffic / (fft_us * 1e-6) / 1e9, 1),
                        "frac": round(fft_traffic / (fft_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
                       if fft_traffic is not None else None),
               "us_per_outer_iteration": round(fft_us, 2),
               "share_of_outer_iteration": round(fft_us / all_us, 4)}
    roof = {"bound": "hbm", "achieved": round(alg_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(alg_gbs / HBM_PEAK_GBS, 4), "bytes_per_px_outer": PR_BYTES_PER_PX_OUTER,
            "basis": "unfused model per outer iteration (FGP 20 x 56, FFT side 464 B per pixel) over the live time; "
                     "the fused prox moves far less, so this ratio can exceed 1",
            "traffic": round(traffic) if traffic is not None else None,
            "hbm": ({"achieved": round(traffic / (all_us * 1e-6) / 1e9, 1),
                     "frac": round(traffic / (all_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "what": "measured bytes of one outer iteration over its profiled kernel time"}
                    if traffic is not None else None),
            "fft": fft, "profiled_kernel_us_per_outer_iteration": round(all_us, 2) if all_us else None,
            "kernels": figs}
    if not extras:
        return {"ms": round(ms, 3), "ms_per_outer_iteration": round(ms / P["outer"], 4), "roofline": roof}

    def loss_trace(accelerate):
        """Data term F after outer iterations 1, 10, 50, 100 (Algorithm 1 vs
        the plain proximal gradient of Eq. 14, the comparison of Fig. 5)."""
        _, lt = ctv.phase_retrieval(y, P["distances"], P["wavelength"], P["pixel"], tau=P["tau"], gamma=P["gamma"],
                                    outer=P["outer"], inner=P["inner"], accelerate=accelerate, loss=True)
        lt = lt.cpu().numpy()
        return {f"F_{k}": float(lt[k - 1]) for k in (1, 10, 50, P["outer"]) if k <= len(lt)}

    ks = (10, 50, P["outer"])

    def rmse_trace(run):
        """Phase RMSE (rad, best global phase removed, Section VI-A) of the
        estimate after 10, 50 and 100 iterations of `run(k)`."""
        return {f"rmse_{k}": round(phase_rmse(run(k).cpu().numpy(), truth), 5) for k in ks}

    def fista_run(constraint, accelerate=True):
        return lambda k: ctv.phase_retrieval(y, P["distances"], P["wavelength"], P["pixel"], tau=P["tau"],
                                             gamma=P["gamma"], outer=k, inner=P["inner"], constraint=constraint,
                                             accelerate=accelerate)

    def ip_run(k):
        return ctv.phase_retrieval_ip(y, P["distances"], P["wavelength"], P["pixel"], iters=k)

    ms_ip = timed(lambda: ip_run(P["outer"]), reps, torch, stream)
    x0 = ctv.phase_retrieval_ip(y, P["distances"], P["wavelength"], P["pixel"], iters=0)

    def kind_run(kind, constraint):
        return ctv.phase_retrieval(y, P["distances"], P["wavelength"], P["pixel"], tau=P["tau"], gamma=P["gamma"],
                                   outer=P["outer"], inner=P["inner"], kind=kind, alpha=P["alpha"],
                                   constraint=constraint)

    by_kind = {"what": "phase RMSE (rad) after 100 outer iterations with each TV kind, without (TV) and with (CTV) "
                       "the constraint |x| <= 1: the comparison of Fig. 4 on the synthetic object",
               **{k: {c_name: round(phase_rmse(kind_run(k, c).cpu().numpy(), truth), 5)
                      for c_name, c in (("tv", "none"), ("ctv", "modulus"))} for k in ("1i", "1a", "2i", "2a")}}
    return {"workload": "1024^2, D=4, 100 outer x 20 FGP iterations, type-1i, |x|<=1",
            "prox_tuning": {"fuse": T, "tile": [tw, tr], "source": source}, "ms": round(ms, 3),
            "ms_per_outer_iteration": round(ms / P["outer"], 4), "roofline": roof,
            "fgp_Mpx_it_s_equiv": round(fgp_px_it / ms / 1e3, 1), "fft2_per_outer_iteration": 2 * len(P["distances"]) + 2,
            "data_term_fista_vs_ista": {"fista": loss_trace(True), "ista": loss_trace(False)},
            "phase_rmse_fista_vs_ista": {"fista": rmse_trace(fista_run("modulus")),
                                         "ista": rmse_trace(fista_run("modulus", accelerate=False))},
            "tv_ctv_ip": {"what": "phase RMSE (rad) on the same measurements: CTV = Algorithm 1 with the "
                                  "constrained prox (|x| <= 1), TV = the same with C = C^{m x n}, IP = iterative "
                                  "projections (each distance's modulus set in turn, then |x| <= 1), all from the "
                                  "back-propagated field",
                          "backprop_rmse": round(phase_rmse(x0.cpu().numpy(), truth), 5),
                          "ctv": rmse_trace(fista_run("modulus")), "tv": rmse_trace(fista_run("none")),
                          "ip": rmse_trace(ip_run), "ip_ms_100_iterations": round(ms_ip, 3),
                          "ip_fft2_per_iteration": 4 * len(P["distances"])},
            "tv_ctv_by_kind": by_kind,
            "paper_simulation": paper_simulation(ctv, synth, torch, dev)}


def paper_simulation(ctv, synth, torch, dev):
    """The simulated experiment of Section VI-A with synthetic stand-ins: a
    256^2 pure phase object (phase in [0, pi)), pixel 5 um, 500 nm, one
    distance of 5 mm, 10 % Gaussian intensity noise; IP, TV and CTV (type-I
    anisotropic, 10 FGP iterations per prox) from the back-propagated field,
    phase RMSE after 10 / 50 / 100 iterations (Fig. 2's comparison), and CTV
    after 100 iterations for several tau (Fig. 6's question)."""
    import numpy as np
    S = synth.PR_PAPER_SIM
    truth = synth.phase_object(seed=0, size=S["size"])
    fields = ctv.pr_forward(torch.as_tensor(truth.astype(np.complex64)).to(dev), S["distances"], S["wavelength"],
                            S["pixel"])
    inten = (fields.abs() ** 2).cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(0)
    y = torch.as_tensor(np.stack([synth.gaussian_measure(I, S["noise"], rng) for I in inten])).to(dev)
    geo = (y, S["distances"], S["wavelength"], S["pixel"])

    def fista(constraint, tau=S["tau"]):
        return lambda k: ctv.phase_retrieval(*geo, tau=tau, gamma=S["gamma"], outer=k, inner=S["inner"],
                                             kind=S["kind"], alpha=S["alpha"], constraint=constraint)

    def rmse(run, ks=(10, 50, S["outer"])):
        return {f"rmse_{k}": round(phase_rmse(run(k).cpu().numpy(), truth), 5) for k in ks}

    return {"what": "Section VI-A's simulated setup on a synthetic pure phase object: phase RMSE (rad) of IP, TV "
                    "and CTV (type-I anisotropic, 10 FGP iterations per prox, gamma 1) at tau 0.01 and 0.1",
            "backprop_rmse": round(phase_rmse(ctv.phase_retrieval_ip(*geo, iters=0).cpu().numpy(), truth), 5),
            "ip": rmse(lambda k: ctv.phase_retrieval_ip(*geo, iters=k)),
            "tv": rmse(fista("none")), "ctv": rmse(fista("modulus")),
            "tv_tau_0.1": rmse(fista("none", 0.1)), "ctv_tau_0.1": rmse(fista("modulus", 0.1)),
            "ctv_rmse_100_by_tau": {str(t): rmse(fista("modulus", t), (S["outer"],))[f"rmse_{S['outer']}"]
                                    for t in (0.003, 0.01, 0.03, 0.1, 0.3, 1.0)}}


def phase_rmse(x, truth):
    """Phase RMSE with the global phase removed (the error measure of Section
    VI-A): x is first rotated by the unit phasor of sum(conj(x) * truth), the
    rotation that brings x closest to the truth in the L2 sense."""
    import numpy as np
    c = np.vdot(x, truth)
    rot = c / abs(c) if abs(c) > 0 else 1.0
    d = np.angle(x * rot * np.conj(truth))
    return float(np.sqrt(np.mean(d * d)))


def median_ms(fn, reps, torch, stream, before=None):
    """Median milliseconds of fn() over reps, each bracketed by its own HIP
    events; before() (untimed) runs ahead of every repetition."""
    fn()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        if before is not None:
            before()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def live_tile_px(mask, halo, rows):
    """Output pixels of the tiles that ctv_denoise runs for a support (cold
    start, column tiles of rows x 64 with this halo): a tile runs if its output
    holds a pixel that is in the support or has a support pixel below or to the
    right. Returns (live tiles, tiles, live output pixels)."""
    import numpy as np
    mk = np.asarray(mask).astype(bool)
    m, n = mk.shape
    live = mk.copy()
    live[:-1, :] |= mk[1:, :]
    live[:, :-1] |= mk[:, 1:]
    OW, OH = 64 - 2 * halo, rows - 2 * halo
    ty, tx = -(-m // OH), -(-n // OW)
    pad = np.zeros((ty * OH, tx * OW), bool)
    pad[:m, :n] = live
    tl = pad.reshape(ty, OH, tx, OW).any(axis=(1, 3))
    hr = np.minimum(OH, m - OH * np.arange(ty))
    wc = np.minimum(OW, n - OW * np.arange(tx))
    return int(tl.sum()), int(tl.size), int((np.outer(hr, wc) * tl).sum())


def bench_plain_calls(ctv, c, torch, dev, b, mask, x_plan, tuner, args):
    """The same four solves as four ctv_denoise calls (each in its own tuned
    configuration), and as the same calls with every tile run: a warm start from
    an all-zero dual state is the cold start's iteration, but ctv_denoise builds
    live-tile lists only for cold starts. Both must equal the plan bit for bit."""
    m, n = c["b"].shape
    K = args.iters
    ws = torch.empty(ctv.workspace_size(m, n, 1, iters=K, fuse=args.fuse)[0], dtype=torch.uint8, device=dev)
    zero = torch.zeros((1, 2, m, n, 4), dtype=torch.float32, device=dev)
    x = torch.empty_like(b)
    stream = torch.cuda.current_stream(dev)
    reps = max(1, args.steps)
    plain_ms, every_ms, same_plain, same_every, tuning = {}, {}, True, True, {}
    for i, kind in enumerate(c["kinds"]):
        kw = dict(kind=kind, alpha=c["alpha"], constraint=c["constraint"], support=mask, iters=K, fuse=args.fuse,
                  out=x, workspace=ws)
        source = tuner.plain(b, c["lam"], kind, c["alpha"], c["constraint"], mask, K, out=x, workspace=ws)
        T, _, tw, tr = ctv.tiling(args.fuse, K, m, n, detail=True, kind=kind, constraint=c["constraint"])
        tuning[kind] = {"fuse": T, "tile": [tw, tr], "source": source}
        plain_ms[kind] = timed(lambda: ctv.denoise(b, c["lam"], **kw), reps, torch, stream)
        same_plain = same_plain and torch.equal(x.view(torch.float32), x_plan[i].view(torch.float32))
        every_ms[kind] = timed(lambda: ctv.denoise(b, c["lam"], state=zero, k0=0, **kw), reps, torch, stream)
        same_every = same_every and torch.equal(x.view(torch.float32), x_plan[i].view(torch.float32))
    px_it = len(c["kinds"]) * m * n * K
    pm, em = sum(plain_ms.values()), sum(every_ms.values())
    plain = {"workload": "the same four solves as four ctv_denoise calls", "tuning": tuning,
             "ms": round(pm, 3), "per_kind_ms": {k: round(v, 3) for k, v in plain_ms.items()},
             "Mpx_it_s": round(px_it / pm / 1e3, 1), "bitwise_equal_to_plan": bool(same_plain)}
    every = {"workload": "the four calls with every tile run (no live-tile lists)", "ms": round(em, 3),
             "Mpx_it_s": round(px_it / em / 1e3, 1), "bitwise_equal_to_plan": bool(same_every)}
    return plain, every


def bench_small(ctv, synth, torch, dev, tuner, reps=20):
    """64 x 64, type-1i, lambda 0.05, K = 100: latency of one solve."""
    c = synth.config1(0)
    b = torch.as_tensor(c["b"]).to(dev)
    x = torch.empty_like(b)
    ws = torch.empty(ctv.workspace_size(64, 64, 1, iters=c["iters"])[0], dtype=torch.uint8, device=dev)
    source = tuner.plain(b, c["lam"], "1i", 0.5, "modulus", None, c["iters"], out=x, workspace=ws)
    T, _, tw, tr = ctv.tiling(0, c["iters"], 64, 64, detail=True)
    stream = torch.cuda.current_stream(dev)
    ms = median_ms(lambda: ctv.denoise(b, c["lam"], kind="1i", iters=c["iters"], out=x, workspace=ws),
                   reps, torch, stream)
    return {"workload": "64x64 complex64, type-1i, lambda 0.05, K=100, |x|<=1",
            "tuning": {"fuse": T, "tile": [tw, tr], "source": source}, "us_per_solve": round(ms * 1e3, 1),
            "Mpx_it_s": round(64 * 64 * c["iters"] / ms / 1e3, 1)}


def bench_out_of_cache(ctv, synth, torch, dev, tuner, size=8192, iters=48, reps=7):
    """The masked configuration at 8192^2 (about 5.4 GB resident: b, x, two
    dual-state buffers, mask), type-1i: warm median, and median with a 512 MB
    write ahead of every repetition so the 256 MB Infinity Cache holds none of
    the working set."""
    c = synth.config2(0, size=size)
    b = torch.as_tensor(c["b"]).to(dev)
    mask = torch.as_tensor(c["mask"]).to(dev)
    x = torch.empty_like(b)
    ws = torch.empty(ctv.workspace_size(size, size, 1, iters=iters)[0], dtype=torch.uint8, device=dev)
    flush = torch.empty(1 << 27, dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream(dev)
    source = tuner.plain(b, c["lam"], "1i", c["alpha"], "modulus", mask, iters, out=x, workspace=ws)
    T, _, tw, tr = ctv.tiling(0, iters, size, size, detail=True)

    def run():
        ctv.denoise(b, c["lam"], kind="1i", support=mask, iters=iters, out=x, workspace=ws)

    warm = median_ms(run, reps, torch, stream)
    cold = median_ms(run, reps, torch, stream, before=lambda: flush.fill_(1.0))
    px_it = size * size * iters
    _, _, live_px = live_tile_px(c["mask"], T, tw * tr)
    run_px_it = live_px * iters       # pixel-iterations actually computed (tiles outside the support skipped)
    return {"workload": f"masked {size}x{size} complex64, type-1i, K={iters}",
            "tuning": {"fuse": T, "tile": [tw, tr], "source": source}, "warm_ms": round(warm, 3),
            "cold_ms": round(cold, 3), "warm_Mpx_it_s": round(px_it / warm / 1e3, 1),
            "cold_Mpx_it_s": round(px_it / cold / 1e3, 1), "computed_px_frac": round(live_px / (size * size), 4),
            "cold_modelled_unfused_bytes_ratio": round(run_px_it * BYTES_PER_PX_IT_MASKED / (cold * 1e-3) / 1e9
                                                       / HBM_PEAK_GBS, 3)}


def copy_probe(torch, dev):
    """Three 1 GiB device-to-device copies: the calibration of the byte
    counters under rocprofv3. Returns the bytes copied each way."""
    src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 4


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs on one MI355X; multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2109_05496_amd as ctv
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        # one secondary measurement alone (what its profiles are taken on)
        tuner = Tuner(ctv, args.tuning, args.tuning_table)
        if args.only == "adjoint":
            res = bench_adjoint(ctv, synth, torch, dev)
        elif args.only == "small":
            res = bench_small(ctv, synth, torch, dev, tuner)
        else:
            res = bench_pr(ctv, synth, torch, dev, tuner, extras=False)
        if args.copy_probe:
            copy_probe(torch, dev)
        print(json.dumps({"only": args.only, args.only: res}), flush=True)
        return
    c = synth.config2(0, size=args.size)
    m, n = c["b"].shape
    K = args.iters
    b = torch.as_tensor(c["b"]).to(dev)
    mask = torch.as_tensor(c["mask"]).to(dev)
    kinds = list(c["kinds"])

    # One step: the four solves submitted as one batched plan (one HIP graph;
    # four images' live tiles per fused step fill the GPU far better than one).
    from paper_2109_05496_amd import prof_summary
    tuner = Tuner(ctv, "off" if args.fuse else args.tuning, args.tuning_table)
    descs = [dict(m=m, n=n, lam=c["lam"], kind=k, alpha=c["alpha"], iters=K, has_support=True) for k in kinds]
    plan = ctv.BatchedPlan(descs, constraint=c["constraint"], fuse=args.fuse)
    bp = plan.pack([c["b"]] * len(kinds), device=dev)
    sp = plan.pack_support([c["mask"]] * len(kinds), device=dev)
    source = tuner.batched(descs, bp, sp) if not args.fuse else "fixed"
    if source == "live":
        plan.close()
        plan = ctv.BatchedPlan(descs, constraint=c["constraint"], fuse=args.fuse)
    T, tw, tr = plan.tiling
    launch_cfg = {"four_kinds_plan": {"fuse": T, "tile": [tw, tr], "source": source}}
    xp = torch.empty_like(bp)

    def step():
        plan.run(bp, sp, out=xp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for s in range(args.steps):
        step()
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = [ev[s].elapsed_time(ev[s + 1]) for s in range(args.steps)]
    ms_per_step = sum(step_ms) / args.steps
    px_iters_step = len(kinds) * m * n * K
    value = px_iters_step / (ms_per_step * 1e-3) / 1e6

    # Roofline of the dominant kernel, the batched fused tile kernel: every
    # launch of a step is one of its ceil(K / T) graph nodes (plus one small scan
    # and one list node, whose time the event average also holds). The work of
    # a launch is what it computes: the output pixels of the live tiles of the
    # four images (tiles outside the support are not run) times T.
    launches = math.ceil(K / T)
    kname = f"void ctv::fgp_batched_kernel<1, {tw}, {tr}>(ctv::FgpBatchedArgs)"
    avg_launch_s = ms_per_step / launches * 1e-3
    live_tiles, all_tiles, live_px = live_tile_px(c["mask"], T, tw * tr)
    run_px_it = live_px * K                   # computed pixel-iterations of one kind
    alg_bytes_launch = BYTES_PER_PX_IT_MASKED * run_px_it * len(kinds) / launches
    alg_flops_launch = sum(FLOPS_PER_PX_IT[k] for k in kinds) * run_px_it / launches
    alg_ops_launch = sum(OPS_PER_PX_IT[k] for k in kinds) * run_px_it / launches
    achieved_gbs = alg_bytes_launch / avg_launch_s / 1e9
    achieved_tflops = alg_flops_launch / avg_launch_s / 1e12
    achieved_gops = alg_ops_launch / avg_launch_s / 1e9
    pmc = prof_summary.load_pmc(os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", PMC_PROFILE))
    # the profile counts only while it was taken with the same launch configuration
    same_config = bool(pmc) and pmc.get("tuning") == prof_summary.tuning_signature(launch_cfg)
    kp = pmc["kernels"].get(kname) if (same_config and args.size == 2048 and K == 200 and args.fuse == 0) else None
    traffic_gbs = kp["traffic_bytes"] / avg_launch_s / 1e9 if kp else None
    roof = {"bound": "alu", "achieved": round(achieved_tflops, 2), "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": kp["traffic_bytes"] if kp else None,
            "kernel": kname, "fused_iters": T, "avg_launch_us": round(avg_launch_s * 1e6, 2),
            "alg_flops_per_launch": int(alg_flops_launch),
            "flops_per_px_it": {k: FLOPS_PER_PX_IT[k] for k in kinds},
            "live_tiles": [len(kinds) * live_tiles, len(kinds) * all_tiles],
            "computed_px_frac": round(live_px / (m * n), 4),
            # the same work against the VALU issue rate of the library's code (non-packed FP32:
            # one lane-operation per lane per cycle), counting an FMA, a min, a max or
            # a reciprocal square root as one operation
            "valu_issue": {"achieved": round(achieved_gops, 1), "peak": round(VALU_OPS_PEAK_GOPS, 1), "unit": "Gop/s",
                           "frac": round(achieved_gops / VALU_OPS_PEAK_GOPS, 4),
                           "ops_per_px_it": {k: OPS_PER_PX_IT[k] for k in kinds},
                           "alg_ops_per_launch": int(alg_ops_launch),
                           "pmc_issue_utilisation": kp["valu_issue_frac"] if kp else None},
            # measured HBM/fabric bytes of the committed PMC profile per launch over the
            # launch time: the "%HBM peak" of the metric
            "hbm": ({"achieved": round(traffic_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(traffic_gbs / HBM_PEAK_GBS, 4)} if kp else None),
            # algorithmic bytes of an unfused iteration (57 B/px-it) per second: what a
            # one-iteration-per-launch solver would have to move; fusion keeps the real
            # traffic far below it, so this ratio exceeds 1 and is no bandwidth fraction
            "modelled_unfused_bytes": {"GBs": round(achieved_gbs, 1), "bytes_per_px_it": BYTES_PER_PX_IT_MASKED,
                                       "ratio_to_hbm_peak": round(achieved_gbs / HBM_PEAK_GBS, 3),
                                       "alg_bytes_per_launch": int(alg_bytes_launch)}}

    computed = len(kinds) * live_px * K / (ms_per_step * 1e-3) / 1e6
    out = {"metric": "CTV-FGP Mpixel-iters/s & %HBM peak", "value": round(value, 1),
           "unit": "Mpixel-iters/s",
           # `value` counts every pixel-iteration of the four problems (dense equivalent);
           # this counts only the pixels of the tiles that run (the others provably keep
           # a zero dual and x = 0)
           "computed_Mpx_it_s": round(computed, 1),
           "hbm_peak_frac": roof["hbm"]["frac"] if roof["hbm"] else None,
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"masked {m}x{n} complex64 CTV denoise, all four TV kinds x {K} FGP iterations: "
                                  "the four plain solves submitted together as one batched plan (one HIP graph); "
                                  "the same solves as four ctv_denoise calls are timed in four_plain_calls",
                      "size": [m, n], "kinds": kinds, "iters": K, "lambda": c["lam"], "alpha": c["alpha"],
                      "constraint": "|x|<=1 + 70% square support",
                      "tiles": "live only: tiles whose output lies where the dual stays zero are not run "
                               "(results bitwise those of running every tile)"},
           "tuning": {"mode": tuner.mode, "table": tuner.table, "launch": launch_cfg},
           "wall_s": round(wall, 3),
           "roofline": roof}
    if not args.no_extras:
        x_plan = [t.reshape(m, n) for t in plan.unpack(xp)]
        out["four_plain_calls"], out["every_tile"] = bench_plain_calls(ctv, c, torch, dev, b, mask, x_plan, tuner,
                                                                       args)
        out["small_64"] = bench_small(ctv, synth, torch, dev, tuner)
        out["out_of_cache_8192"] = bench_out_of_cache(ctv, synth, torch, dev, tuner)
        out["batched"] = bench_batched(ctv, synth, torch, dev, tuner)
        out["adjoint"] = bench_adjoint(ctv, synth, torch, dev)
        out["phase_retrieval"] = bench_pr(ctv, synth, torch, dev, tuner)
    if args.copy_probe:
        out["copy_probe_bytes_each_way"] = copy_probe(torch, dev)
    if args.save_tuning:
        ctv.tune_cache_save(args.save_tuning)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, args.cpu_sample_iters)
        out["cpu_baseline"]["ragged_batch_all_cores"] = cpu_batched_pool(args.cpu_batch_iters)
        if args.pr_oracle:
            out["cpu_baseline"]["phase_retrieval_end_to_end"] = pr_end_to_end(ctv, synth, torch, dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
