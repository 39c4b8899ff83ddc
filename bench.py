"""Benchmark of the coupled LB-FD-PF step on one MI355X.

Default workload: the D3Q19 packed sphere bed of 256x128x128 cells, FP32
populations and fields, one-step F + O -> 2P chemistry (4 species).  A step
is one launch of the fused kernel (LB collide+stream with interface drag, FD
transport of T and Y_k with interface heat exchange, Arrhenius reaction
sub-steps, FP64 conservation partials) followed by the FP64 reaction-island
kernel for cells above the ignition threshold.  Inputs are resident in HBM
before the timed region; the timed region is K steps bracketed by stream
synchronisation, timed with HIP events on the stream the kernels run on.
A second pass of K steps brackets every step-kernel launch with HIP events:
their mean is the kernel duration the roofline figure divides by.

The same line carries the chemistry surrogate against exact chemistry on the
9-species sphere bed: ms per step of both paths, their ratio, and the maximum
relative temperature difference after 1000 steps from the same state.

Prints one JSON line.  --gpus above 1 is refused: this runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("coupled MLUPS + % HBM roofline; surrogate vs exact-chemistry speedup "
          "@≤1% T err")
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2310_17214_amd/csrc/lbfd_kernels.inc",
                  "paper_2310_17214_amd/csrc/lbfd_device.h"]


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def make_workload(name):
    from paper_2310_17214_amd import workloads as W

    def log(m):
        print("bench:", m, file=sys.stderr, flush=True)

    if name == "sphere_bed":
        return W.bed_one_step(precision="fp32")
    if name == "sphere_bed_fp64":
        return W.bed_one_step(precision="fp64")
    if name == "cylinder":
        return W.cylinder_channel()
    if name == "sphere_bed_9sp":
        return W.bed_sphere_9sp(precision="fp32")
    if name == "superquadric_bed":
        return W.bed_superquadric_9sp(precision="fp32")
    if name == "sphere_bed_closed":
        # the one-step sphere bed as a closed box: walls where the inlet and
        # outlet were, P0(t) from the fixed mass, r = cp (gamma - 1) / gamma
        # with gamma = 1.4
        wl = W.bed_one_step(precision="fp32")
        s = wl.setup
        s["lb_bc"] = ["wall" if b in ("inlet", "outlet") else b for b in s["lb_bc"]]
        s["u_in"] = [0.0, 0.0, 0.0]
        s["closed"], s["r_gas"] = 1, s["cp"] * 0.4 / 1.4
        wl.name = wl.name.replace("sphere_bed", "sphere_bed_closed")
        return wl
    if name == "elongated_bed_slab":
        # one GPU's share (third of eight 128-cell slabs, with a halo plane
        # on each side) of the 1024x256x256 elongated bed
        return W.bed_elongated_9sp(window=(255, 385), log=log)
    if name == "elongated_bed":
        return W.bed_elongated_9sp(log=log)
    raise SystemExit(f"unknown workload {name}")


def _counter_summary(workload_name, bytes_alg):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_hash") != kernel_hash() or d.get("bytes_per_launch_alg") != bytes_alg:
        return None
    return d


def traffic_from_profiles(workload_name, bytes_alg):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current kernel sources (else None)."""
    d = _counter_summary(workload_name, bytes_alg)
    return None if d is None else d.get("bytes_per_launch")


# wave64 VALU instructions the chip can issue per second without packed FP32:
# 256 CUs x 4 SIMDs, one wave64 instruction every 4 cycles each, at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4 / 1e9


def alu_from_profiles(workload_name, bytes_alg, kernel_ms):
    """The step kernel against the vector-ALU issue rate: SQ_INSTS_VALU per
    launch from the committed counter summary (current kernel sources only)
    over the live mean launch duration."""
    d = _counter_summary(workload_name, bytes_alg)
    if d is None or "valu_insts_per_launch" not in d:
        return None
    achieved = d["valu_insts_per_launch"] / (kernel_ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": VALU_ISSUE_PEAK,
            "unit": "G wave64 VALU instructions/s", "frac": round(achieved / VALU_ISSUE_PEAK, 4),
            "valu_insts_per_launch": d["valu_insts_per_launch"], "summary": d.get("summary")}


XGMI_LINK_GBS = 153.0


def halo_measure(ctx, stream, reps=50):
    """Pack and unpack of the halo planes of both x faces of a slab, timed
    with HIP events on the context's stream: the copies a slab decomposition
    adds to each step, and the time one xGMI link would take to move the
    packed bytes."""
    import torch

    nb = ctx.halo_bytes()
    elem = 4 if ctx.precision == "fp32" else 8
    dt = torch.float32 if elem == 4 else torch.float64
    bufs = [torch.empty(nb // elem, dtype=dt, device="cuda") for _ in range(2)]
    faces = (-1, 1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    for _ in range(3):
        for f, b in zip(faces, bufs):
            ctx.halo_pack(f, b)
    ev[0].record(stream)
    for _ in range(reps):
        for f, b in zip(faces, bufs):
            ctx.halo_pack(f, b)
    ev[1].record(stream)
    for _ in range(reps):
        for f, b in zip(faces, bufs):
            ctx.halo_unpack(f, b)
    ev[2].record(stream)
    ctx.synchronize()
    pack_us = ev[0].elapsed_time(ev[1]) * 1e3 / reps
    unpack_us = ev[1].elapsed_time(ev[2]) * 1e3 / reps
    moved = 2 * 2 * nb  # both faces, read + write
    return {"bytes_per_face": nb, "planes_per_face": nb // (elem * ctx.shape[0] * ctx.shape[1]),
            "pack_both_faces_us": round(pack_us, 2),
            "unpack_both_faces_us": round(unpack_us, 2),
            "pack_GBps": round(moved / (pack_us * 1e-6) / 1e9, 1),
            "unpack_GBps": round(moved / (unpack_us * 1e-6) / 1e9, 1),
            "xgmi_one_link_us_per_face": round(nb / (XGMI_LINK_GBS * 1e9) * 1e6, 2),
            "note": "halo copies only; the transfers between GPUs are not run"}


def cpu_baseline(wl, target_s=15.0, one_thread_s=8.0):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the same
    workload: whole-grid steps from the initial state, as many as fit in about
    `target_s` seconds (at least two) on every host thread, then about
    `one_thread_s` seconds of the following steps on one thread."""
    from oracle import oracle as O

    wl64 = dict(wl.setup)
    wl64["precision"] = "fp64"
    orc = O.Oracle(wl64, wl.phi)
    orc.init_state(wl.T0, wl.Y0 if wl.setup["ns"] else None)
    threads = O.nthreads()
    t0 = time.perf_counter()
    orc.step(1)
    first = time.perf_counter() - t0
    more = max(1, int(target_s / max(first, 1e-3)) - 1)
    orc.step(more)
    dt = time.perf_counter() - t0
    steps = 1 + more
    mlups = wl.cells * steps / dt / 1e6
    # one thread: as many steps as the all-thread rate says fit
    O.set_threads(1)
    n1 = max(1, int(one_thread_s * mlups / threads * 1e6 / wl.cells))
    t1 = time.perf_counter()
    orc.step(n1)
    dt1 = time.perf_counter() - t1
    O.set_threads(threads)
    grid = f"{wl.setup['nx']}x{wl.setup['ny']}x{wl.setup['nz']}"
    return {"value": round(mlups, 3), "unit": "MLUPS",
            "cores": threads, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{steps} steps of the full {grid} grid from the initial state, "
                      f"{dt:.1f} s on {threads} threads",
            "one_thread": {"value": round(wl.cells * n1 / dt1 / 1e6, 3), "unit": "MLUPS",
                           "cores": 1, "sample": f"the next {n1} steps, {dt1:.1f} s"}}


MLP_FLOP_PER_CELL = 2 * (11 * 256 + 256 * 256 + 256 * 9)   # 141,312 (9 species)
BF16_PEAK_TFLOPS = 2500.0


def surrogate_measure(wl=None, steps=200, seed=4, log=None, sample_steps=5000, every=25,
                      per_snapshot=10000, err_steps=1000, sweep=True, epochs=20):
    """Surrogate against exact chemistry, by default on the 9-species sphere
    bed (256x128x128): train on pairs sampled from an exact run (every 25th
    step of 5000, 10,000 cells each, 90/10 split), then time both paths and
    compare T after `err_steps` steps from the same initial state."""
    import torch

    from paper_2310_17214_amd import lbfd, surrogate as SG, workloads as W

    t0 = time.perf_counter()
    if wl is None:
        wl = W.bed_sphere_9sp(precision="fp32")
    ns = wl.setup["ns"]
    x, y = SG.sample_run(wl, steps=sample_steps, every=every, per_snapshot=per_snapshot,
                         seed=seed)
    t_sample = time.perf_counter() - t0
    if log:
        log(f"sampled {x.shape[0]} pairs in {t_sample:.1f} s")
    (xt, yt), (xh, yh) = SG.split(x, y, 0.1, seed=seed + 1)
    n_pairs = int(x.shape[0])
    del x, y
    t1 = time.perf_counter()
    w, nrm, env, losses = SG.train(xt, yt, ns, epochs=epochs, batch=8192, seed=seed + 2, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    res = {}
    for mode in ("exact", "surrogate"):
        ctx = lbfd.Context(wl.setup, wl.phi)
        if mode == "surrogate":
            ctx.set_surrogate(w, nrm, env)
            rmse, rel, fb_ho = SG.heldout_rmse(ctx, xh, yh)
        ctx.init_state(wl.T0, wl.Y0)
        ctx.step(20)
        ctx.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.step(steps)
        e1.record(ctx.stream)
        ctx.synchronize()
        ms = e0.elapsed_time(e1) / steps
        ctx.set_timing(True)
        ctx.step(steps)
        kt = {k: ctx.kernel_time(i) for i, k in enumerate(("step", "island", "mlp"))}
        ctx.set_timing(False)
        ctx.step(err_steps - 20 - 2 * steps)
        d = ctx.diagnostics()
        res[mode] = {"ms": ms, "kt": kt, "T": ctx.read(lbfd.F_T), "diag": d}
        del ctx
        if log:
            log(f"{mode}: {ms:.3f} ms per step")
    ex, su = res["exact"], res["surrogate"]
    err = float(np.max(np.abs(su["T"] - ex["T"]) / ex["T"]))
    # cost of the exact path against the number of reaction sub-steps (same
    # mechanism and state, n_sub overridden): where the surrogate would pay
    by_nsub = {}
    for k in ((3, 6, 12, 24) if sweep else ()):
        s = dict(wl.setup)
        s["n_sub"] = k
        ctx = lbfd.Context(s, wl.phi)
        ctx.init_state(wl.T0, wl.Y0)
        ctx.step(10)
        ctx.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.step(50)
        e1.record(ctx.stream)
        ctx.synchronize()
        by_nsub[k] = e0.elapsed_time(e1) / 50
        del ctx
    # the stiff reaction schemes on the same bed: every cell's reaction step
    # in the FP64 island (linearly implicit Euler at one sub-step, adaptive
    # explicit sub-steps up to 8); T after err_steps against the explicit run
    stiff = {}
    for name, scheme, nsub in ((("linearly_implicit", 1, 1), ("adaptive_explicit", 2, 8))
                               if sweep else ()):
        s = dict(wl.setup, chem_scheme=scheme, n_sub=nsub)
        ctx = lbfd.Context(s, wl.phi)
        ctx.init_state(wl.T0, wl.Y0)
        ctx.step(10)
        ctx.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.step(50)
        e1.record(ctx.stream)
        ctx.synchronize()
        ms_s = e0.elapsed_time(e1) / 50
        ctx.step(err_steps - 60)
        Ts = ctx.read(lbfd.F_T)
        stiff[name] = {"chem_scheme": scheme, "n_sub": nsub, "ms_per_step": round(ms_s, 5),
                       f"max_rel_T_err_vs_explicit_{err_steps}_steps":
                           float(np.max(np.abs(Ts - ex["T"]) / ex["T"]))}
        del ctx
        if log:
            log(f"{name}: {ms_s:.3f} ms per step")
    ks = sorted(by_nsub)
    even = None
    for a, b in zip(ks, ks[1:]):
        ya, yb = by_nsub[a], by_nsub[b]
        if ya <= su["ms"] <= yb:
            even = a + (b - a) * (su["ms"] - ya) / (yb - ya)
            break
    mlp_ms = su["kt"]["mlp"][1]
    tflops = MLP_FLOP_PER_CELL * wl.cells / (mlp_ms * 1e-3) / 1e12
    return {
        "workload": wl.name, "species": ns, "reactions": len(wl.setup["mech"]["A"]),
        "n_sub": int(wl.setup["n_sub"]),
        "exact_ms_per_step": round(ex["ms"], 5), "surrogate_ms_per_step": round(su["ms"], 5),
        "speedup": round(ex["ms"] / su["ms"], 4),
        f"max_rel_T_err_{err_steps}_steps": err, "T_err_bar": 0.01,
        "fallback_share": su["diag"]["n_fallback"] / (float(err_steps) * wl.cells),
        "fallback_reason_share": {k: v / (float(err_steps) * wl.cells)
                                  for k, v in su["diag"]["n_fallback_reason"].items()},
        "kernels_ms": {"exact": {k: round(v[1], 5) for k, v in ex["kt"].items()},
                       "surrogate": {k: round(v[1], 5) for k, v in su["kt"].items()}},
        "mlp_roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": BF16_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / BF16_PEAK_TFLOPS, 4),
                         "flop_per_cell": MLP_FLOP_PER_CELL},
        "training": {"pairs": n_pairs, "train_pairs": int(xt.shape[0]),
                     "sample_s": round(t_sample, 2), "train_s": round(t_train, 2),
                     "epochs": len(losses), "final_loss": losses[-1]},
        "heldout_rel_rmse": [None if not np.isfinite(v) else round(float(v), 5) for v in rel],
        "heldout_fallback_share": fb_ho,
        "exact_ms_per_step_by_n_sub": {str(k): round(v, 5) for k, v in by_nsub.items()} or None,
        "break_even_n_sub": None if even is None else round(even, 2),
        "stiff_schemes": stiff or None,
    }


def mlp_probe(steps):
    """The in-step surrogate alone on the 9-species sphere bed (freshly
    initialised weights: the kernel's work does not depend on them), for
    counter runs; prints the surrogate kernel's mean launch time."""
    import torch  # noqa: F401

    from paper_2310_17214_amd import lbfd, surrogate as SG, workloads as W

    wl = W.bed_sphere_9sp(precision="fp32")
    ns = wl.setup["ns"]
    ni = ns + 2
    w = SG.initial_weights(ns, 1)
    norm = np.concatenate([[700.0, 1.0] + [0.1] * ns, [300.0, 1e-12] + [0.1] * ns,
                           [0.0] * ns, [1e-3] * ns]).astype(np.float32)
    env = np.concatenate([[0.0, 1.0] + [0.0] * ns, [5000.0, 1.0] + [1.0] * ns]).astype(np.float32)
    assert len(norm) == 2 * ni + 2 * ns and len(env) == 2 * ni
    ctx = lbfd.Context(wl.setup, wl.phi)
    ctx.set_surrogate(w, norm, env)
    ctx.init_state(wl.T0, wl.Y0)
    ctx.set_timing(True)
    ctx.step(steps)
    n, ms = ctx.kernel_time(lbfd.LBFD_KERNEL_SURROGATE)
    print(json.dumps({"mlp_probe_steps": steps, "mlp_kernel_ms": ms,
                      "tflops": MLP_FLOP_PER_CELL * wl.cells / (ms * 1e-3) / 1e12}))


def copy_probe():
    """A plain device copy of 1 GiB, run under the HBM counters to calibrate
    FETCH_SIZE / WRITE_SIZE."""
    import torch

    a = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written":
                      b.numel() * 4}))


def method_bytes_per_cell(setup):
    """Algorithmic bytes per cell and step of the method, each array moved
    once: the LB part reads and writes the Q populations in place and reads
    rho, T, phi_s and divu and writes u; the FD + chemistry part reads T, Y_k,
    u and phi_s and writes T, Y_k, rho and divu: s (2Q + 4 + d) + s (5 + 2 ns
    + d) with s the storage size (244 B for D3Q19, FP32, 4 species; 284 B
    with 9; 248 B for D2Q9 in FP64 without species)."""
    d = setup["dim"]
    Q = 9 if d == 2 else 19
    s = 4 if setup.get("precision", "fp64") == "fp32" else 8
    return float(s * ((2 * Q + 4 + d) + (5 + 2 * setup["ns"] + d)))


def measure(wl, steps, warmup, settle_ms, stream=None, timing=True):
    """MLUPS of `steps` coupled steps after `warmup` untimed steps (HIP events
    on the context's stream), then the same number of steps again with every
    kernel launch timed, for the kernels' own mean durations.  Before the
    warm-up the context steps for `settle_ms` of wall time (untimed) so that
    the GPU's clocks have ramped up as in a long run."""
    import torch

    from paper_2310_17214_amd import lbfd

    ctx = lbfd.Context(wl.setup, wl.phi, stream=stream)
    ctx.init_state(wl.T0, wl.Y0 if wl.setup["ns"] else None)
    settle = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < settle_ms:
        ctx.step(10)
        ctx.synchronize()
        settle += 10
    ctx.step(warmup)
    ctx.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(ctx.stream)
    ctx.step(steps)
    e1.record(ctx.stream)
    ctx.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    diag = ctx.diagnostics()
    out = {"ctx": ctx, "ms": ms, "ms_step": ms / steps, "wall": wall, "settle": settle,
           "mlups": wl.cells * steps / (ms * 1e-3) / 1e6, "diag": diag}
    if timing:
        ctx.set_timing(True)
        ctx.step(steps)
        out["step_kernel"] = ctx.kernel_time(lbfd.LBFD_KERNEL_STEP)
        out["island_kernel"] = ctx.kernel_time(lbfd.LBFD_KERNEL_ISLAND)
        ctx.set_timing(False)
    return out


def roofline(wl, m, traffic=None, alu=None):
    """The step kernel against the HBM roofline: achieved = the method's
    algorithmic bytes per cell (method_bytes_per_cell) x cells / the kernel's
    mean launch duration; the kernel's own count of what it moves beside it."""
    bpc = method_bytes_per_cell(wl.setup)
    kbpc = m["ctx"].bytes_per_cell()
    n, kms = m["step_kernel"]
    achieved = bpc * wl.cells / (kms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "bytes_per_cell": bpc, "bytes_per_launch": bpc * wl.cells,
            "bytes_per_cell_kernel": kbpc,
            "frac_kernel_bytes": round(kbpc * wl.cells / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel": "step_kernel (fused LB+FD+chemistry+partials)",
            "kernel_ms": round(kms, 5), "kernel_launches": n,
            "island_ms": round(m["island_kernel"][1], 5), "island_launches": m["island_kernel"][0],
            "alu": alu}


def config_line(name, steps, warmup, settle_ms, log):
    """One more workload of the method at its own size: MLUPS and the step
    kernel's roofline."""
    import torch

    t0 = time.perf_counter()
    wl = make_workload(name)
    gen = time.perf_counter() - t0
    log(f"config {wl.name}: {wl.cells} cells (inputs built in {gen:.1f} s)")
    m = measure(wl, steps, warmup, settle_ms)
    bytes_alg = m["ctx"].bytes_per_cell() * wl.cells
    traffic = traffic_from_profiles(name, bytes_alg)
    alu = alu_from_profiles(name, bytes_alg, m["step_kernel"][1])
    line = {"workload": wl.name, "cells": wl.cells,
            "lattice": "D2Q9" if wl.setup["dim"] == 2 else "D3Q19",
            "species": wl.setup["ns"], "reactions": len(wl.setup["mech"]["A"]),
            "precision": wl.setup.get("precision", "fp64"),
            "value": round(m["mlups"], 2), "unit": "MLUPS", "ms_per_step": round(m["ms_step"], 5),
            "steps": steps, "warmup": warmup, "settle_steps": m["settle"],
            "roofline": roofline(wl, m, traffic, alu),
            "diagnostics": {"Tmax": m["diag"]["Tmax"], "umax": m["diag"]["umax"],
                            "n_flagged_fp64": m["diag"]["n_flagged_fp64"],
                            "n_nonfinite": m["diag"]["n_nonfinite"]}}
    del m
    torch.cuda.empty_cache()
    return line


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-ms", type=float, default=300.0)
    ap.add_argument("--workload", default="sphere_bed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--mlp-probe", type=int, default=0, metavar="STEPS")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported: the benchmark runs on one GPU "
              "(the slab decomposition over several GPUs is described, not built)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return
    if args.mlp_probe:
        mlp_probe(args.mlp_probe)
        return

    import torch

    blog = lambda m: print("bench:", m, file=sys.stderr, flush=True)  # noqa: E731
    blog(f"building workload {args.workload}")
    wl = make_workload(args.workload)
    blog(f"{wl.name}, {wl.cells} cells, warmup {args.warmup}, steps {args.steps}")
    stream = torch.cuda.current_stream()
    m = measure(wl, args.steps, args.warmup, args.settle_ms, stream=stream)
    ctx, diag = m["ctx"], m["diag"]
    bpc = method_bytes_per_cell(wl.setup)
    traffic = traffic_from_profiles(args.workload, ctx.bytes_per_cell() * wl.cells)
    alu = alu_from_profiles(args.workload, ctx.bytes_per_cell() * wl.cells, m["step_kernel"][1])
    prec = wl.setup.get("precision", "fp64")
    out = {
        "metric": METRIC,
        "value": round(m["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(m["ms_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "cells": wl.cells,
                   "lattice": "D2Q9" if wl.setup["dim"] == 2 else "D3Q19",
                   "species": wl.setup["ns"], "reactions": len(wl.setup["mech"]["A"]),
                   "precision": prec, "parallelism": "single GPU"},
        "settle_steps": m["settle"],
        "roofline": roofline(wl, m, traffic, alu),
        "diagnostics": {"mass": diag["mass"], "Tmax": diag["Tmax"], "umax": diag["umax"],
                        "n_flagged_fp64": diag["n_flagged_fp64"],
                        "n_nonfinite": diag["n_nonfinite"]},
        "wall_s": round(m["wall"], 3),
    }
    if wl.name.startswith("elongated_bed") and "_slab_" in wl.name:
        blog("halo planes")
        out["halo"] = halo_measure(ctx, stream)
        out["halo"]["step_ms"] = round(m["ms_step"], 4)
    del m, ctx
    torch.cuda.empty_cache()
    if not args.no_surrogate and args.workload == "sphere_bed":
        blog("surrogate vs exact chemistry (9-species bed)")
        out["surrogate"] = surrogate_measure(log=blog)
    elif not args.no_surrogate and args.workload == "elongated_bed":
        # the elongated bed's own surrogate: pairs from 2000 exact steps of it
        blog("surrogate vs exact chemistry (elongated bed)")
        out["surrogate"] = surrogate_measure(wl, steps=20, log=blog, sample_steps=2000,
                                             every=25, per_snapshot=25000, err_steps=200,
                                             sweep=False)
    if not args.no_configs and args.workload == "sphere_bed":
        # the other workloads of the method at their own sizes: the cylinder
        # channel (D2Q9, FP64), the superquadric bed and the 67 M-cell
        # elongated bed (9 species, FP32)
        out["configs"] = [config_line(n, args.steps, args.warmup, args.settle_ms, blog)
                          for n in ("cylinder", "superquadric_bed", "elongated_bed")]
    if not args.no_cpu_baseline:
        blog("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
