"""Benchmark: streaming Tucker updates per second on one MI355X.

Workload: the advecting-blob stream with 128 x 128 x 128 spatial slices and 16
variables (4-way slices, d = 5), 400 slices, tau = 1e-4, initial ST-HOSVD on
the first 20 slices. A step is one streaming update (Alg. 5) of one slice. All
slices are generated on the GPU and resident in HBM before the timed region;
the timed region covers exactly the last --steps updates of the stream (the
steady state, at the largest ranks); the --warmup updates before it, and all
earlier ones, run untimed.

Prints one JSON line with the throughput, a roofline entry for the kernel group
that takes the most device time (from HIP events recorded by the library on its
own stream), and the FP64 CPU oracle timed on a bounded sample of the same
stream on the host cores.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "slices/s at eps-bounded error: bf16x3 MFMA vs FP32 path; TTM/Gram % roofline"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0 / 3.0, "fp64": 78.6}
# MFMA type of the residual Gram's products per path precision
GRAM_PREC = {"fp32": "fp32", "bf16x3": "bf16x3", "fp64": "fp64"}
GOLDEN = os.path.join(ROOT, "tests", "golden", "blobs128_oracle_trajectory.json")
GOLDEN_FACTORED = os.path.join(ROOT, "tests", "golden", "blobs128_oracle_trajectory_factored.json")

WORKLOAD = dict(space=(128, 128, 128), n_vars=16, n_blobs=32, n_slices=400, n_init=20,
                tau=1e-4, seed=1001)

# HBM bytes per launch of the dominant kernel of a run, from the two counter
# passes (FETCH_SIZE, WRITE_SIZE; calibrated on a 1 GiB copy) recorded under
# profiles/. Keyed by (precision, core update, kernel group, timed steps); only
# reported for the kernel and timed window the counters were taken on.
MEASURED_TRAFFIC = {
    # V rotation, default timed window (slices 210..399): FETCH_SIZE 492782.1
    # KiB x 2.000 + WRITE_SIZE 974950.2 KiB x 1.000 per launch
    ("fp32", "literal", "rot_v", 190): 2.0076e9,
}

# Differentiation workload: a 96^3 x 8 variables x 16-slice window, ranks
# (24, 24, 24, 6, 8).
GRAD_DIMS, GRAD_RANKS = (96, 96, 96, 8, 16), (24, 24, 24, 6, 8)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def roofline(prof, precision, core="literal", steps=None):
    """Roofline entry of the group with the most device time."""
    group = max(prof, key=lambda g: prof[g]["ms"])
    p = prof[group]
    if p["ms"] <= 0 or p["launches"] == 0:
        return group, None
    sec = p["ms"] / 1e3
    ai = p["flops"] / p["bytes"] if p["bytes"] else float("inf")
    prec_key = "fp64" if group in ("eig", "svd", "ud", "rot_v", "rot_c", "isvd") else precision
    peak_f = PEAK_TFLOPS[prec_key]
    ridge = peak_f * 1e12 / (PEAK_HBM_GBS * 1e9)
    if ai >= ridge:
        achieved = p["flops"] / sec / 1e12
        entry = dict(bound="mfma", achieved=round(achieved, 3), peak=peak_f, unit="TFLOP/s",
                     frac=round(achieved / peak_f, 4))
    else:
        achieved = p["bytes"] / sec / 1e9
        entry = dict(bound="hbm", achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                     frac=round(achieved / PEAK_HBM_GBS, 4))
    entry.update(kernel=group, launches=p["launches"], avg_ms=round(p["ms"] / p["launches"], 5),
                 flops_per_launch=p["flops"] / p["launches"],
                 bytes_per_launch=p["bytes"] / p["launches"],
                 traffic=MEASURED_TRAFFIC.get((precision, core, group, steps)))
    return group, entry


def ttm_roofline(prof, precision):
    """Roofline of the mode-1 TTM with its fused residual (the largest contraction)."""
    p = prof["ttm1"]
    if not p["launches"] or p["ms"] <= 0:
        return None
    sec = p["ms"] / 1e3
    peak_f = PEAK_TFLOPS[precision]
    ridge = peak_f * 1e12 / (PEAK_HBM_GBS * 1e9)
    ai = p["flops"] / p["bytes"]
    t_floor = max(p["flops"] / (peak_f * 1e12), p["bytes"] / (PEAK_HBM_GBS * 1e9))
    return dict(kernel="ttm1", bound="mfma" if ai >= ridge else "hbm",
                achieved_tflops=round(p["flops"] / sec / 1e12, 3),
                achieved_gbs=round(p["bytes"] / sec / 1e9, 1),
                avg_ms=round(p["ms"] / p["launches"], 5), frac=round(t_floor / sec, 4))


def gram_roofline(prof, precision):
    """Roofline of the residual Gram over every growth of the stream's updates
    (growth is rare, so the timed window may hold none; the Grams of the
    initial ST-HOSVD, FP64 products of the data, are not included)."""
    p = prof["gram"]
    if not p["launches"] or p["ms"] <= 0:
        return None
    sec = p["ms"] / 1e3
    peak_f = PEAK_TFLOPS[GRAM_PREC.get(precision, precision)]
    t_floor = max(p["flops"] / (peak_f * 1e12), p["bytes"] / (PEAK_HBM_GBS * 1e9))
    return dict(kernel="gram", launches=p["launches"], scope="all updates (not the init)",
                achieved_tflops=round(p["flops"] / sec / 1e12, 3),
                achieved_gbs=round(p["bytes"] / sec / 1e9, 1),
                avg_ms=round(p["ms"] / p["launches"], 5), peak_tflops=peak_f,
                frac=round(t_floor / sec, 4))


def ttm_chain_flops(shape, modes_to):
    """Flops of the mode-by-mode TTM chain changing shape[k] to modes_to[k]."""
    shape = list(shape)
    total = 0.0
    for k, m in enumerate(modes_to):
        total += 2.0 * math.prod(shape) * m
        shape[k] = m
    return total


def large_bench(n_init=20, warmup=3, steps=30):
    """FP32 vs bf16x3 products on the 512 x 512 x 256 Fourier stream (tau 1e-4),
    factored core form: updates per second and the mode-1 TTM roofline."""
    import torch

    import paper_2308_16395_amd as pkg
    from synth import make_stream

    s = make_stream(4)
    dev = torch.device("cuda:0")
    total = n_init + warmup + steps
    data = torch.empty((total, math.prod(s.dims)), dtype=torch.float32, device=dev)
    for t in range(total):
        data[t] = s.slice_torch(t, dev, torch.float32)
    torch.cuda.synchronize()
    out = dict(workload="random-Fourier 512x512x256, tau 1e-4, init 20 slices, "
                        f"{steps} timed updates after {warmup}, factored core form")
    for prec in ("fp32", "bf16x3"):
        st = pkg.StreamingTucker(s.dims, 1e-4, precision=prec, profile=True,
                                 core_update="factored")
        st.init(data[:n_init].reshape(-1), n_init)
        for t in range(n_init, n_init + warmup):
            st.update(data[t])
        st.profile(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(n_init + warmup, total):
            st.update(data[t])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = st.profile()
        out[prec] = dict(value=round(steps / dt, 2), ranks=list(st.ranks),
                         recon_error_bound=st.recon_error()[0],
                         ttm_roofline=ttm_roofline(prof, prec),
                         ttm_ms_per_step=round((prof["ttm1"]["ms"] + prof["ttm"]["ms"]) / steps,
                                               4))
        st.close()
        log(f"large stream {prec}: {out[prec]}")
    del data
    torch.cuda.empty_cache()
    return out


def symeig_bench():
    """The library's small symmetric eigensolver (st_symeig: the step of Alg. 1
    after the Gram) at the Gram orders of the blob stream (16, 64, 128) keeping
    k = 1, 2, 8 eigenvectors, on seeded Gram matrices X X^T (X: n x 4n, columns
    scaled by a decaying spectrum) resident in HBM; wall time per call,
    including its workspace allocation and the final synchronisation."""
    import numpy as np
    import torch

    import paper_2308_16395_amd.binding as bd

    out = dict(workload="st_symeig on seeded Gram matrices X X^T, X: n x 4n, column "
                        "scales 10^(-4 j / 4n); wall ms per call")
    rng = np.random.default_rng(2308)
    for n in (16, 64, 128):
        x = rng.standard_normal((n, 4 * n)) * np.logspace(0, -4, 4 * n)[None, :]
        g = torch.from_numpy(x @ x.T).cuda()
        for k in (1, 2, 8):
            for _ in range(3):
                bd.symeig(g, k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                bd.symeig(g, k)
            torch.cuda.synchronize()
            out[f"n{n}_k{k}"] = round((time.perf_counter() - t0) / 20 * 1e3, 3)
    log(f"symeig: {out}")
    return out


def sine_bench():
    """The sine-wave experiment of Sec. 5.1 (100 x 100 x 5000, rank bump at slice
    2500, eta 1e-3, tau 1e-2): the streaming path (initial ST-HOSVD on 200
    slices, then 4800 updates, FP32 products, literal core update) and the batch
    ST-HOSVD of all 5000 slices at once, slices resident in HBM, whole-run wall
    times."""
    import numpy as np
    import torch

    import paper_2308_16395_amd as pkg
    from synth import SINE_WAVE, make_stream

    s = make_stream(SINE_WAVE)
    tau, n_init, n = SINE_WAVE["eps"], SINE_WAVE["n_init"], s.n_slices
    data = torch.from_numpy(
        np.stack([s.slice_flat(t).astype(np.float32) for t in range(n)])).cuda()
    out = dict(workload="sine wave 100x100x5000 (ranks (11,11,11) then (11,11,15)), "
                        "eta 1e-3, tau 1e-2, FP32")
    st = pkg.StreamingTucker(s.dims, tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.init(data[:n_init].reshape(-1), n_init)
    r3 = {}
    for t in range(n_init, n):
        st.update(data[t])
        if t in (s.n_half - 1, s.n_half):
            r3[t] = st.ranks[2]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["stream"] = dict(seconds=round(dt, 3), slices_per_s=round((n - n_init) / dt, 1),
                         ranks=list(st.ranks), recon_error_bound=st.recon_error()[0],
                         r3_before_after_bump=[r3[s.n_half - 1], r3[s.n_half]])
    st.close()
    st = pkg.StreamingTucker(s.dims, tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.init(data.reshape(-1), n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out["batch"] = dict(seconds=round(dt, 3), ranks=list(st.ranks),
                        recon_error_bound=st.recon_error()[0])
    st.close()
    log(f"sine wave: {out}")
    del data
    torch.cuda.empty_cache()
    return out


def grad_bench(reps=5):
    """Reconstruct / Project forward and VJPs at GRAD_DIMS, FP32 products."""
    import numpy as np
    import torch

    import paper_2308_16395_amd.autodiff as ad

    rng = np.random.default_rng(7)
    facs = [ad.colmajor(torch.from_numpy(np.linalg.qr(rng.standard_normal((n, r)))[0]
                                         .astype(np.float32)).cuda())
            for n, r in zip(GRAD_DIMS, GRAD_RANKS)]
    core = torch.randn(math.prod(GRAD_RANKS), device="cuda")
    xhat = ad.tucker_reconstruct(core, facs)
    x = xhat + 0.01 * torch.randn_like(xhat)
    upstream = 2.0 * (xhat - x)
    gbar = torch.randn_like(core)
    ops = {
        "reconstruct": lambda: ad.tucker_reconstruct(core, facs),
        "reconstruct_vjp": lambda: ad.tucker_reconstruct_vjp(core, facs, upstream),
        "project": lambda: ad.tucker_project(x, facs),
        "project_vjp": lambda: ad.tucker_project_vjp(x, facs, gbar),
    }
    f_rec = ttm_chain_flops(GRAD_RANKS, GRAD_DIMS)
    f_proj = ttm_chain_flops(GRAD_DIMS, GRAD_RANKS)
    out = {}
    for name, fn in ops.items():
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        flops = f_rec if name == "reconstruct" else f_proj if name == "project" else None
        out[name] = dict(ms=round(ms, 3))
        if flops:
            out[name]["tflops"] = round(flops / ms / 1e9, 2)
    return dict(workload="Reconstruct/Project and VJPs, 96x96x96 x 8 variables x 16-slice "
                         "window, ranks (24, 24, 24, 6, 8), FP32 MFMA, wall time per call",
                **out)


def cpu_info():
    """CPU model and thread counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        avail = os.cpu_count() or 1
    return dict(model=model, blas_threads=int(threads), cpus_available=int(avail),
                os_cpu_count=os.cpu_count())


def cpu_baseline(host_slice, n_init, tau, n_updates, dims):
    """The FP64 oracle on the host: init on the first slices (untimed), then
    `n_updates` timed updates of the same stream. `host_slice(t)` returns slice
    t in float64 (the float32 values the GPU consumes)."""
    import numpy as np

    from oracle import StreamingTucker as Oracle

    info = cpu_info()
    t0 = time.perf_counter()
    x0 = np.stack([host_slice(t).reshape(dims, order="F") for t in range(n_init)], axis=-1)
    orc = Oracle(x0, tau)
    init_s = time.perf_counter() - t0
    del x0
    slices = [host_slice(t).reshape(dims, order="F") for t in range(n_init, n_init + n_updates)]
    t0 = time.perf_counter()
    for y in slices:
        orc.update(y)
    dt = time.perf_counter() - t0
    return dict(value=round(n_updates / dt, 4), unit="slices/s", cores=info["blas_threads"],
                kind="oracle",
                sample=f"FP64 oracle updates of slices {n_init}..{n_init + n_updates - 1} of the "
                       f"same stream after its own init on slices 0..{n_init - 1} "
                       f"({init_s:.1f} s, untimed); {dt:.1f} s timed; ranks after the sample "
                       f"{list(orc.ranks)} (the GPU figure is taken at the end of the stream, "
                       "where ranks are larger)",
                cpu_model=info["model"], cpus_available=info["cpus_available"])


def cpu_baseline_cfg0():
    """The oracle on the 32 x 32 x 100 exactly-low-rank stream (tau 1e-3, init
    10 slices), on one BLAS thread and on all of them."""
    import numpy as np

    from oracle import StreamingTucker as Oracle
    from synth import CONFIGS, make_stream

    c = CONFIGS[0]
    s = make_stream(0)
    sl = [s.slice_flat(t).astype(np.float32).astype(np.float64).reshape(s.dims, order="F")
          for t in range(s.n_slices)]

    def once():
        orc = Oracle(np.stack(sl[:c["n_init"]], axis=-1), c["eps"])
        t0 = time.perf_counter()
        for t in range(c["n_init"], s.n_slices):
            orc.update(sl[t])
        return (s.n_slices - c["n_init"]) / (time.perf_counter() - t0), orc.ranks

    out = dict(workload="32x32x100 exact rank (4,4,6) + noise, tau 1e-3, init 10 slices, "
                        "90 updates")
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            v1, ranks = once()
        out["one_thread"] = dict(value=round(v1, 2), unit="slices/s", cores=1)
    except Exception as exc:  # pragma: no cover
        out["one_thread"] = dict(error=repr(exc))
    vall, ranks = once()
    out["all_threads"] = dict(value=round(vall, 2), unit="slices/s",
                              cores=cpu_info()["blas_threads"])
    out["ranks"] = list(ranks)
    return out


def plan_window(n_slices, n_init, steps, warmup):
    """Slice ranges of a benchmark run over the whole stream.

    The initial ST-HOSVD takes slices [0, n_init); every later slice is one
    update. The timed window is the LAST `steps` updates (the steady state, at
    the largest ranks); the `warmup` updates just before it are the warm-up,
    and all earlier updates run untimed (the state must go through them).
    """
    updates = n_slices - n_init
    if steps < 1:
        raise ValueError("--steps must be at least 1")
    if warmup < 0:
        raise ValueError("--warmup must be non-negative")
    if steps + warmup > updates:
        raise ValueError(f"--steps + --warmup = {steps + warmup} exceeds the {updates} updates "
                         f"of the {n_slices}-slice stream (init {n_init})")
    t0 = n_slices - steps
    return dict(init=(0, n_init), untimed=(n_init, t0), warmup=(t0 - warmup, t0),
                timed=(t0, n_slices))


def probe_errors(st, golden_ck, pos_t):
    """Element-wise comparison of GPU reconstructions with the oracle's at the
    sampled positions of one golden checkpoint: max over its probe slices of
    ||x^_gpu - x^_oracle|| / ||Y_t|| on the sample."""
    import numpy as np

    worst = 0.0
    per = {}
    for pr in golden_ck["probes"]:
        rec = st.reconstruct_slice(pr["t"])
        g = rec[pos_t].double().cpu().numpy()
        o = np.asarray(pr["recon"])
        x = np.asarray(pr["data"])
        err = float(np.linalg.norm(g - o) / np.linalg.norm(x))
        per[pr["t"]] = err
        worst = max(worst, err)
    return worst, per


def guarded(name, fn, result):
    """Run an optional benchmark leg; a failure is recorded, not fatal."""
    try:
        result[name] = fn()
    except Exception as exc:  # the headline must survive an optional leg
        log(f"{name} failed: {exc!r}")
        result[name] = dict(error=repr(exc))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=190,
                    help="timed updates: the last STEPS updates of the 400-slice stream")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", choices=["fp32", "bf16x3", "fp64"], default="fp32")
    ap.add_argument("--core-update", choices=["literal", "factored"], default="literal",
                    help="literal: Alg. 5 as stated (V and core rotated per slice); factored: "
                         "V = V0 M and C = V x_d S")
    ap.add_argument("--cpu-updates", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-grad", action="store_true",
                    help="skip the Reconstruct/Project forward and VJP timings")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the FP32 vs bf16x3 comparison on the 512x512x256 stream")
    ap.add_argument("--no-block", action="store_true",
                    help="skip the block-update leg (b slices per call)")
    ap.add_argument("--no-sine", action="store_true",
                    help="skip the sine-wave stream and batch run (100x100x5000)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline run (for profiling it alone)")
    ap.add_argument("--sine-only", action="store_true",
                    help="run only the sine-wave stream and batch run and print their "
                         "JSON (for profiling that workload alone)")
    ap.add_argument("--symeig-only", action="store_true",
                    help="run only the small symmetric eigensolver timings and print "
                         "their JSON (for profiling its kernels alone)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (a known-size "
                         "kernel against which HBM byte counters are calibrated)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the streaming update is sequential along the "
              "stream and this build measures one GPU's share (see DESIGN.md on sharding).",
              file=sys.stderr)
        sys.exit(2)
    if args.sine_only:
        print(json.dumps(dict(sine_wave=sine_bench())), flush=True)
        return
    if args.symeig_only:
        print(json.dumps(dict(symeig=symeig_bench())), flush=True)
        return
    w = WORKLOAD
    n_init, n_slices = w["n_init"], w["n_slices"]
    try:
        plan = plan_window(n_slices, n_init, args.steps, args.warmup)
    except ValueError as exc:
        raise SystemExit(str(exc))
    if args.headline_only:
        args.no_variants = args.no_cpu_baseline = args.no_large = True
        args.no_sine = args.no_grad = args.no_block = True

    import numpy as np
    import torch

    import paper_2308_16395_amd as pkg
    from synth import BlobStream

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.copy_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 1 GiB read + 1 GiB written by one copy kernel")
        del src, dst
    stream = BlobStream(w["space"], w["n_vars"], w["n_blobs"], n_slices=n_slices,
                        seed=w["seed"])
    ny = math.prod(stream.dims)
    log(f"generating {n_slices} slices of {ny} elements on {torch.cuda.get_device_name(0)}")
    data = torch.empty((n_slices, ny), dtype=torch.float32, device=dev)
    for t in range(n_slices):
        data[t] = stream.slice_torch(t, dev, torch.float32)
    torch.cuda.synchronize()
    log(f"plan: {plan}")

    golden = None
    if os.path.exists(GOLDEN):
        with open(GOLDEN) as f:
            golden = json.load(f)
    # oracle reconstructions at sampled positions, per core update
    pos_t = None
    checkpoints = {"literal": {}, "factored": {}}
    if golden is not None and golden.get("probe_positions"):
        pos_t = torch.tensor(golden["probe_positions"], dtype=torch.long, device=dev)
        checkpoints["literal"] = {ck["after"]: ck for ck in golden["checkpoints"]}
    if os.path.exists(GOLDEN_FACTORED):
        with open(GOLDEN_FACTORED) as f:
            gf = json.load(f)
        if gf.get("probe_positions") == (golden or {}).get("probe_positions"):
            checkpoints["factored"] = {ck["after"]: ck for ck in gf["checkpoints"]}
    t_begin, t_end = plan["timed"]

    def run(precision, core_update):
        cks = checkpoints[core_update]
        st = pkg.StreamingTucker(stream.dims, w["tau"], precision=precision, profile=True,
                                 core_update=core_update)
        t0 = time.perf_counter()
        st.init(data[:n_init].reshape(-1), n_init)
        init_s = time.perf_counter() - t0
        st.profile(reset=True)  # the update groups below count updates only
        traj, guard, probe = [], 0, {}
        for t in range(n_init, t_begin):
            st.update(data[t])
            traj.append(st.ranks)
            guard += st.stats()["guard_hits"]
            if t in cks and pos_t is not None:
                probe[t] = probe_errors(st, cks[t], pos_t)[0]
        prof_untimed = st.profile(reset=True)
        ranks = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(t_begin, t_end):
            st.update(data[t])
            ranks.append(st.ranks)  # host-side counters only, no device sync
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        traj += ranks
        prof = st.profile()
        whole = {g: {k: prof_untimed[g][k] + prof[g][k] for k in prof[g]} for g in prof}
        info = dict(value=round(args.steps / dt, 3), ms_per_step=round(1e3 * dt / args.steps, 4),
                    init_s=round(init_s, 3), ranks_final=list(st.ranks),
                    recon_error_bound=st.recon_error()[0], guard_hits_untimed=guard,
                    qr_fixes=st.stats()["qr_total"])
        if golden is not None:
            ref = [tuple(x["ranks"]) for x in golden["slices"]][:len(traj)]
            bad = [n_init + i for i, (a, b) in enumerate(zip(traj, ref)) if tuple(a) != b]
            info["ranks_match_oracle"] = not bad
            info["rank_divergent_slices"] = len(bad)
            info["first_rank_divergence_slice"] = bad[0] if bad else None
            if cks.get(t_end - 1) is not None and pos_t is not None:
                probe[t_end - 1], per = probe_errors(st, cks[t_end - 1], pos_t)
                info["oracle_error_final_probes"] = {str(k): v for k, v in per.items()}
            if probe:
                info["oracle_error_max_over_checkpoints"] = max(probe.values())
                info["oracle_error_checkpoints"] = {str(k): v for k, v in probe.items()}
        if not args.no_accuracy:
            err2 = nrm2 = 0.0
            for t in range(n_slices):
                rec = st.reconstruct_slice(t)
                err2 += torch.sum((rec.double() - data[t].double()) ** 2).item()
                nrm2 += torch.sum(data[t].double() ** 2).item()
            info["true_rel_error"] = math.sqrt(err2 / nrm2)
            info["eps_met"] = info["true_rel_error"] <= w["tau"]
        st.close()
        log(f"{precision} {core_update}: {info}")
        return info, prof, whole

    head, prof, whole = run(args.precision, args.core_update)
    group, roof = roofline(prof, args.precision, args.core_update, args.steps)
    result = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "slices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16x3": "bf16x3", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {
            "workload": "advecting-blobs 128x128x128 x 16 variables, 400 slices, tau 1e-4, "
                        f"init 20 slices; timed: updates of slices {t_begin}..{t_end - 1} "
                        "(the last steps of the stream), all slices resident in HBM",
            "slice_dims": list(stream.dims), "n_slices": n_slices, "n_init": n_init,
            "eps": w["tau"], "precision": args.precision, "core_update": args.core_update,
            "seed": w["seed"], "timed_slices": [t_begin, t_end - 1],
        },
        "roofline": roof,
        "ttm_roofline": ttm_roofline(prof, args.precision),
        "gram_roofline": gram_roofline(whole, args.precision),
        "kernels": {g: dict(launches=p["launches"], ms=round(p["ms"], 3),
                            tflops=round(p["flops"] / p["ms"] / 1e9, 3) if p["ms"] else None,
                            gbs=round(p["bytes"] / p["ms"] / 1e6, 1) if p["ms"] else None)
                    for g, p in prof.items() if p["launches"]},
    }
    result.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step")})
    if not args.no_cpu_baseline:
        k = max(1, min(args.cpu_updates, n_slices - n_init))

        def host_slice(t):
            return data[t].cpu().numpy().astype(np.float64)

        log(f"timing the FP64 oracle on {k} updates")
        guarded("cpu_baseline",
                lambda: cpu_baseline(host_slice, n_init, w["tau"], k, stream.dims), result)
        guarded("cpu_baseline_cfg0", cpu_baseline_cfg0, result)
    if not args.no_variants:
        result["variants"] = {}
        for core in ("literal", "factored"):
            for prec in ("fp64", "bf16x3", "fp32"):
                if (prec, core) == (args.precision, args.core_update):
                    continue

                def variant(prec=prec, core=core):
                    info, vprof, vwhole = run(prec, core)
                    info["roofline"] = roofline(vprof, prec, core, args.steps)[1]
                    info["ttm_roofline"] = ttm_roofline(vprof, prec)
                    info["gram_roofline"] = gram_roofline(vwhole, prec)
                    info["ttm_ms"] = round(vprof["ttm1"]["ms"] + vprof["ttm"]["ms"], 3)
                    info["kernels_ms"] = {g: round(p["ms"], 2) for g, p in vprof.items()
                                          if p["launches"]}
                    return info

                guarded(f"{prec}_{core}", variant, result["variants"])
    if not args.no_block:
        log("block updates (b slices per call) over the timed window")

        def block_leg():
            out = dict(workload=f"same stream and window (slices {t_begin}..{t_end - 1}); "
                                "blocks of b slices per st_update_block call, "
                                f"{args.precision}; literal core (bN) and factored core "
                                "(bN_factored)")
            for bsz, core in ((4, "literal"), (16, "literal"), (4, "factored"),
                              (16, "factored")):
                st = pkg.StreamingTucker(stream.dims, w["tau"], precision=args.precision,
                                         core_update=core)
                st.init(data[:n_init].reshape(-1), n_init)
                t = n_init
                while t < t_begin:
                    b = min(bsz, t_begin - t)
                    st.update_block(data[t:t + b].reshape(-1), b)
                    t += b
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                while t < t_end:
                    b = min(bsz, t_end - t)
                    st.update_block(data[t:t + b].reshape(-1), b)
                    t += b
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                err2 = nrm2 = 0.0
                for tt in range(n_slices):
                    rec = st.reconstruct_slice(tt)
                    err2 += torch.sum((rec.double() - data[tt].double()) ** 2).item()
                    nrm2 += torch.sum(data[tt].double() ** 2).item()
                key = f"b{bsz}" if core == "literal" else f"b{bsz}_factored"
                out[key] = dict(value=round((t_end - t_begin) / dt, 3),
                                      ms_per_block=round(1e3 * dt / ((t_end - t_begin) / bsz), 3),
                                      ranks_final=list(st.ranks),
                                      recon_error_bound=st.recon_error()[0],
                                      true_rel_error=math.sqrt(err2 / nrm2),
                                      qr_fixes=st.stats()["qr_total"])
                st.close()
            return out

        guarded("block_updates", block_leg, result)
    del data
    torch.cuda.empty_cache()
    if not args.no_large:
        log("FP32 vs bf16x3 on the 512x512x256 stream")
        guarded("large_stream", large_bench, result)
    if not args.no_sine:
        log("sine-wave stream and batch ST-HOSVD (100x100x5000)")
        guarded("sine_wave", sine_bench, result)
    if not args.no_grad:
        log("timing Reconstruct/Project forward and VJPs")
        guarded("differentiation", grad_bench, result)
    if not args.headline_only:
        guarded("symeig", symeig_bench, result)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
