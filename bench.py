"""Benchmark of the 3D eighth-order immersed-boundary step on one MI355X.

Workload: 401 x 401 x 301 grid, 10 m, space order 8, seeded fractal free surface
(spectral exponent -2, 300 m relief), depth-gradient velocity with a 5 % random
perturbation, 40-cell damping layer, one Ricker 10 Hz source, 201 x 201 receivers.
A step is one pass of the hot path: interior stencil + damping, IB patch, source
injection, receiver sampling.  Inputs are generated on the host, the stencil table is
built on the GPU, then W warm-up steps and K timed steps run with every input resident
in HBM.  Prints one JSON line.

Roofline: HIP events (torch.cuda.Event on the stream the library launches on) time
each kernel over its own launches; algorithmic bytes per launch, counted over the
physical (interior) nodes, whose exterior neighbours hold zeros that need no traffic:
  interior: FP32 (increment form) 20 B per node: read p^n, d^n, K, write p^{n+1}, d^{n+1};
            FP64 32 B per node: read p^n, p^{n-1}, K, write p^{n+1};
  IB patch: 4 B per weight + 21 B per IB point (FP32: 5 B record, read-modify-write of
            p^{n+1} and d^{n+1}), 8 B per weight + 21 B (FP64: 5 B record, 16 B p^{n+1}).
The accuracy figure comes from its own full-length runs (FP32 and FP64, every step of the
workload), not from the timed window.  "achievable" is a 1 GiB device-to-device copy
timed the same way.
HBM traffic per launch comes from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this script
(``--calibrate`` adds a 1 GiB device copy whose counters give the scale factors), turned
into profiles/traffic.json by ``--summarize-counters FETCH_DIR WRITE_DIR``.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNELS = {"interior": "k_interior3d_p", "patch": "k_patch_cols"}
TRAFFIC_FILE = "hbm_traffic_interior_patch_config3.json"
# (OUT: any output folder)
PROFILE_CMDS = [
    "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/prof_f -o f -- "
    "python3 bench.py --steps 20 --warmup 5 --no-cpu --no-accuracy --calibrate",
    "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/prof_w -o w -- "
    "python3 bench.py --steps 20 --warmup 5 --no-cpu --no-accuracy --calibrate",
    "python3 bench.py --summarize-counters OUT/prof_f OUT/prof_w",
]
CALIB_BYTES = 1 << 30


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step.hip", "step.h", "io.h"):
        h.update(open(os.path.join(ROOT, "paper_2309_03600_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per launch measured with rocprofv3 counters (profiles/traffic.json),
    valid only for the kernel source they were taken on."""
    p = os.path.join(ROOT, "profiles", TRAFFIC_FILE)
    if not os.path.exists(p):
        return {}
    d = json.load(open(p))
    if d.get("source_hash") != kernel_source_hash():
        return {}
    return d.get("kernels", {})


def time_kernel(st, which, count, torch):
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    st.run_kernel(which, 2)                      # warm
    e0.record(s)
    st.run_kernel(which, count)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / count           # ms per launch


def summarize_counters(fetch_dir, write_dir):
    """profiles/traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per
    dispatch) of ``bench.py --calibrate``: each kernel's mean per dispatch, scaled by what
    the same counter reads for the 1 GiB calibration copy."""
    import csv
    import glob

    def per_kernel(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    rows.append((int(r["Dispatch_Id"]), r["Kernel_Name"], float(r["Counter_Value"]) * 1024.0))
        out = {}
        for i, k, v in sorted(rows):
            out.setdefault(k, []).append((i, v))
        return out

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")

    def copy_value(tab):
        vals = [v for k, vs in tab.items() if "copy" in k.lower() or "elementwise" in k.lower() for _, v in vs]
        vals = [v for v in vals if v > 0.25 * CALIB_BYTES]
        return float(np.median(vals)) if vals else None

    cf, cw = copy_value(fetch), copy_value(write)
    res = {"source_hash": kernel_source_hash(), "commands": PROFILE_CMDS, "calibration": {
        "copy_bytes_each_way": CALIB_BYTES, "fetch_reads": cf, "write_reads": cw,
        "fetch_factor": CALIB_BYTES / cf if cf else None, "write_factor": CALIB_BYTES / cw if cw else None},
        "kernels": {}}
    def launches(tab, sym, tname, last):
        # dispatches in launch order; the interior kernel's autotuning launches (other
        # variants and depth chunks) precede the timed ones, so only the trailing ``last``
        # dispatches (as many as the patch kernel had: one per step or timing launch) count
        rows = sorted((i, v) for k, vs in tab.items() if sym + "<" + tname in k for i, v in vs)
        return [v for _, v in rows[-last:]] if last else [v for _, v in rows]

    for short, sym in KERNELS.items():
        for prec, tname in (("f32", "float"), ("f64", "double")):
            npatch = len([v for k, vs in fetch.items() if KERNELS["patch"] + "<" + tname in k for v in vs])
            fk = launches(fetch, sym, tname, npatch)
            wk = launches(write, sym, tname, npatch)
            if not fk or not wk or not cf or not cw:
                continue
            rd = float(np.mean(fk)) * CALIB_BYTES / cf
            wr = float(np.mean(wk)) * CALIB_BYTES / cw
            res["kernels"][f"{sym}/{prec}"] = {"read_bytes_per_launch": rd, "write_bytes_per_launch": wr,
                                              "bytes_per_launch": rd + wr, "dispatches": len(fk)}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", TRAFFIC_FILE), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res, indent=1))


_ORACLE = {}


def _oracle_init(sim, wav):
    _ORACLE.update(sim=sim, wav=wav)


def _oracle_steps(nsteps):
    """One worker's share of the CPU baseline: the oracle's own stepping, timed."""
    t0 = time.perf_counter()
    _ORACLE["sim"].run(_ORACLE["wav"], nsteps)
    return time.perf_counter() - t0


def cpu_baseline(budget_steps=5000):
    """The FP64 oracle on a bounded sample: a 24 x 24 x 301 grid with the same recipe
    (fractal free surface, M = 8, damping), weights from a process pool (untimed), then
    ``budget_steps`` oracle steps in each of as many processes as the host has cores (up
    to 16), all at once: the host's aggregate oracle throughput."""
    import multiprocessing as mp

    from paper_2309_03600_amd import workloads as W
    from oracle import stepper
    from oracle.parallel import solve_points
    from oracle.weights import IBModel
    procs = min(16, os.cpu_count() or 1)
    wl = dataclasses.replace(W.small3d(cfg=95, n=24, nz=301, relief=50.0, nt=budget_steps, z_top_cells=20),
                             eta=W.config3(nt=1, with_velocity=False).eta)
    t0 = time.time()
    m = IBModel(wl.heights, wl.h, wl.shape, M=wl.M, surface=wl.surface, eta=wl.eta)
    sols = solve_points(m, procs=procs)
    L = stepper.assemble_laplacian(m, sols)
    sim = stepper.Simulation(m, L, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, damp_R=wl.damp_R)
    t_build = time.time() - t0
    wav = wl.wavelets(np.float64)
    saved = {k: os.environ.get(k) for k in ("OPENBLAS_NUM_THREADS", "OMP_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(procs, initializer=_oracle_init, initargs=(sim, wav)) as pool:
            pool.map(abs, range(procs))          # the workers are up before the clock starts
            t0 = time.perf_counter()
            times = pool.map(_oracle_steps, [budget_steps] * procs, chunksize=1)
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    npts = int(np.prod(wl.shape))
    return {"value": npts * budget_steps * procs / wall / 1e9, "unit": "Gpts/s", "cores": procs, "kind": "oracle",
            "sample": f"oracle FP64 stepping of a {wl.shape[0]}x{wl.shape[1]}x{wl.shape[2]} grid "
                      f"(same recipe, {len(sols)} IB points) for {budget_steps} steps in each of {procs} processes "
                      f"at once, {wall:.1f} s wall (each process {min(times):.1f}-{max(times):.1f} s, "
                      f"{npts * budget_steps / max(times) / 1e9:.3f} Gpts/s or more); its weight build took "
                      f"{t_build:.1f} s over {procs} processes"}


def copy_bandwidth(torch):
    """GB/s of a 1 GiB device-to-device copy (read + write), timed with HIP events: the
    measured "achievable" HBM bandwidth beside the 8 TB/s peak.  Its dispatches also
    calibrate the rocprofv3 traffic counters (``--summarize-counters``)."""
    a = torch.ones(CALIB_BYTES // 4, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(10):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    del a, b
    return 2 * CALIB_BYTES / (ms * 1e-3) / 1e9


def accuracy_full_length(torch, ib, w, stats, nt=3000):
    """Per-trace ||d32 - d64|| / max(||d64||, 1e-3 max ||d64||) over all ``nt`` steps of the
    headline workload (FP32 increment form against FP64, graph replay)."""
    from paper_2309_03600_amd import workloads as W
    wl = W.config3(nt=nt)
    tr = {}
    for prec in ("f32", "f64"):
        dt = torch.float32 if prec == "f32" else torch.float64
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        wav = torch.tensor(wl.wavelets(np.float64), dtype=dt, device="cuda")
        tr[prec] = st.step(nt, wav, use_graph=True)[0].double().cpu().numpy()
        st.close()
        del wav
    num = np.linalg.norm(tr["f32"] - tr["f64"], axis=0)
    nrm = np.linalg.norm(tr["f64"], axis=0)
    e = num / np.maximum(nrm, 1e-3 * nrm.max())
    strong = nrm >= 2.5e-3 * nrm.max()
    out = {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "median": float(np.median(e)),
           "traces_above_1e-4": int((e > 1e-4).sum()), "traces": int(e.size),
           "max_over_traces_at_least_2.5e-3_of_largest": float(e[strong].max()),
           "abs_error_max_over_largest_trace": float(num.max() / nrm.max()),
           "over": f"all {nt} steps of the workload, FP32 (increment form) GPU vs FP64 GPU; the FP64 path "
                   "matches the FP64 oracle to 1e-9"}
    log(f"[bench] accuracy over {nt} steps: max {out['max']:.2e} p99 {out['p99']:.2e} median {out['median']:.2e}, "
        f"{out['traces_above_1e-4']} of {e.size} traces above 1e-4")
    return out


def _time_steps(torch, st, wav, K, Wm, graph=True):
    """Wm untimed steps, then K steps between HIP events; returns (ms per step, traces)."""
    tr_w = torch.empty((st.nshots, Wm, st.nrec), dtype=wav.dtype, device="cuda") if st.nrec else None
    tr = torch.empty((st.nshots, K, st.nrec), dtype=wav.dtype, device="cuda") if st.nrec else None
    st.step(Wm, wav, tr_w, use_graph=graph)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    st.step(K, wav, tr, use_graph=graph)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K, tr


def _trace_err(a, b):
    num = np.linalg.norm(a - b, axis=0)
    den = np.linalg.norm(b, axis=0)
    den = np.maximum(den, 1e-3 * den.max())
    e = num / den
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)), "median": float(np.median(e))}


def bench_config2(args):
    """2D 801x401, M = 8: both forms (second-order p; first-order staggered p-v), free and
    rigid surfaces (the first-order form is built for the free surface), FP32 and FP64."""
    import torch

    import paper_2309_03600_amd as ib
    from paper_2309_03600_amd import workloads as W
    K, Wm = args.steps, args.warmup
    rows = []
    for form, surface in (("p2", "free"), ("p2", "rigid"), ("pv1", "free")):
        wl = W.config2(surface=surface, nt=K + Wm + 8)
        w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta,
                                form=form)
        N = int(np.prod(wl.shape))
        tr = {}
        row = {"form": form, "surface": surface, "rows_or_ib_points": w.stats()["n_ib"]}
        for prec in ("f32", "f64"):
            tdt = torch.float32 if prec == "f32" else torch.float64
            st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
            wav = torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda")
            ms, t = _time_steps(torch, st, wav, K, Wm)
            tr[prec] = t.double().cpu().numpy()[0]
            row[prec] = {"ms_per_step": ms, "gpts": N / (ms * 1e-3) / 1e9}
            st.close()
        row["fp32_vs_fp64_trace_relL2"] = _trace_err(tr["f32"], tr["f64"])
        log(f"[bench config2] {form} {surface}: FP32 {row['f32']['gpts']:.2f} Gpts/s, FP64 {row['f64']['gpts']:.2f}"
            f" Gpts/s, FP32 vs FP64 max {row['fp32_vs_fp64_trace_relL2']['max']:.2e}")
        rows.append(row)
        w.close()
    out = {"metric": "Gpts/s, 2D eighth-order IB step (second-order and first-order forms)",
           "value": rows[0]["f32"]["gpts"], "unit": "Gpts/s", "n_gpus": 1, "steps": K, "warmup": Wm,
           "ms_per_step": rows[0]["f32"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "2D 801x401, dx=5 m, space order 8, Gaussian hill 150 m / 400 m, "
                                  "1 Ricker source, 161 receivers, 40-cell damping"},
           "results": rows}
    print(json.dumps(out))


def bench_config4(args):
    """64 shots over one 301x301x201 topography (FP32, one batched state, graph replay)
    against the plain single-shot FP64 path, with the FP32 error on a shot."""
    import torch

    import paper_2309_03600_amd as ib
    from paper_2309_03600_amd import workloads as W
    K, Wm = args.steps, args.warmup
    wl = W.config4(nt=K + Wm + 8)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    N = int(np.prod(wl.shape))
    S = wl.src.shape[0]
    st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision="f32")
    wav = torch.tensor(wl.wavelets(np.float64), dtype=torch.float32, device="cuda")
    ms_b, tr_b = _time_steps(torch, st, wav, K, Wm)
    tr_b0 = tr_b[0].double().cpu().numpy()
    st.close()
    del tr_b
    single = {}
    for prec in ("f64", "f32"):
        tdt = torch.float64 if prec == "f64" else torch.float32
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src[:1], wl.rec, damp_width=wl.damp_width, precision=prec)
        ms, tr = _time_steps(torch, st, wav[:1].to(tdt).contiguous(), K, Wm)
        single[prec] = {"ms_per_step": ms, "gpts": N / (ms * 1e-3) / 1e9, "tr": tr[0].double().cpu().numpy()}
        st.close()
    gb = N * S / (ms_b * 1e-3) / 1e9
    err = _trace_err(tr_b0, single["f64"]["tr"])
    log(f"[bench config4] batched {S} shots FP32: {gb:.1f} Gpts/s ({ms_b:.3f} ms/step); single-shot FP64 "
        f"{single['f64']['gpts']:.1f}, FP32 {single['f32']['gpts']:.1f} Gpts/s; shot 0 FP32 vs FP64 max {err['max']:.2e}")
    out = {"metric": "Gpts/s (shot-points per second), batched shots, 3D eighth-order IB step", "value": gb,
           "unit": "Gpts/s", "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": ms_b, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3D 301x301x201, dx=10 m, space order 8, {S} shots in one state, "
                                  "shared fractal topography and weights, hipGraph replay, 151x151 receivers"},
           "single_shot_fp64": {k: v for k, v in single["f64"].items() if k != "tr"},
           "single_shot_fp32": {k: v for k, v in single["f32"].items() if k != "tr"},
           "speedup_vs_single_shot_fp64": gb / single["f64"]["gpts"],
           "shot0_fp32_batched_vs_fp64_single_trace_relL2": err}
    print(json.dumps(out))


def bench_config5(args):
    """FWI gradient: forward with checkpoints every 50 steps and the discrete adjoint, 16
    shots FP32 over 256^3 for the workload's 1500 steps (the velocity anomaly 900 m down is
    reached and its reflection recorded only after about 1000 steps; a shorter run
    differentiates rounding noise), with the FP32 vs FP64 gradient error on four shots and
    the FP64 throughput of the same four shots batched."""
    import torch

    import paper_2309_03600_amd as ib
    from paper_2309_03600_amd import workloads as W
    nt = args.nt
    wl = W.config5(nt=nt)
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    N = int(np.prod(wl.shape))
    res = {}
    grads = {}
    for prec, shots in (("f32", slice(0, 16)), ("f64_4", slice(0, 4)), ("f32_4", slice(0, 4)), ("f64", slice(5, 6)),
                        ("f32_1", slice(5, 6))):
        p = prec[:3]
        tdt = torch.float32 if p == "f32" else torch.float64
        src = wl.src[shots]
        S = src.shape[0]
        wav = torch.tensor(wl.wavelets(np.float64)[shots], dtype=tdt, device="cuda").contiguous()
        obs = ib.ib_state_create(w, wl.extra["v_true"], wl.dt, src, wl.rec, damp_width=wl.damp_width, precision=p)
        dobs = obs.forward(nt, wav, ckpt_every=50)
        obs.close()
        st = ib.ib_state_create(w, wl.vel, wl.dt, src, wl.rec, damp_width=wl.damp_width, precision=p)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = st.forward(nt, wav, ckpt_every=50)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = st.adjoint(d - dobs, wav)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st.close()
        grads[prec] = g.cpu().numpy()
        del d, dobs, g
        torch.cuda.empty_cache()
        res[prec] = {"shots": S, "forward_s": t1 - t0, "adjoint_s": t2 - t1,
                     "forward_gpts": N * S * nt / (t1 - t0) / 1e9,
                     "gradient_gpts": N * S * nt / (t2 - t0) / 1e9}
        log(f"[bench config5] {prec}: {S} shots, forward {t1 - t0:.2f} s, adjoint {t2 - t1:.2f} s, "
            f"gradient {res[prec]['gradient_gpts']:.2f} Gpts/s")
    e = float(np.linalg.norm(grads["f32_1"] - grads["f64"]) / np.linalg.norm(grads["f64"]))
    e4 = float(np.linalg.norm(grads["f32_4"] - grads["f64_4"]) / np.linalg.norm(grads["f64_4"]))
    e4max = float(np.abs(grads["f32_4"] - grads["f64_4"]).max() / np.abs(grads["f64_4"]).max())
    out = {"metric": "Gpts/s (shot-points per second of forward + adjoint), FWI gradient, 3D eighth-order IB",
           "value": res["f32"]["gradient_gpts"], "unit": "Gpts/s", "n_gpus": 1, "steps": nt, "warmup": 0,
           "ms_per_step": (res["f32"]["forward_s"] + res["f32"]["adjoint_s"]) / nt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "3D 256^3, dx=10 m, space order 8, rigid fractal surface, 16 shots, "
                                  "64x64 receivers, +3% Gaussian velocity anomaly, checkpoints every 50 steps"},
           "results": res, "single_shot_fp32_vs_fp64_gradient_relL2": e,
           "fp32_vs_fp64_gradient_4_shots": {"relL2": e4, "max_over_max": e4max},
           "fp64_4_shot_gradient_gpts": res["f64_4"]["gradient_gpts"],
           "speedup_vs_single_shot_fp64": res["f32"]["gradient_gpts"] / res["f64"]["gradient_gpts"]}
    print(json.dumps(out))


def bench_pv3d(args):
    """3D first-order p-v form, fourth order (the order of the paper's examples), over the
    401x401x301 fractal free surface of the headline workload; FP32 and FP64."""

    import torch

    import paper_2309_03600_amd as ib
    from paper_2309_03600_amd import workloads as W
    K, Wm = args.steps, args.warmup
    wl = dataclasses.replace(W.config3(nt=K + Wm + 8, lateral=args.lateral, depth=args.depth), M=4, eta=0.5)
    t0 = time.time()
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=4, surface=wl.surface, eta=wl.eta, form="pv1")
    torch.cuda.synchronize()
    build_s = time.time() - t0
    N = int(np.prod(wl.shape))
    res, tr = {}, {}
    for prec in ("f32", "f64"):
        tdt = torch.float32 if prec == "f32" else torch.float64
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        wav = torch.tensor(wl.wavelets(np.float64), dtype=tdt, device="cuda")
        ms, t = _time_steps(torch, st, wav, K, Wm)
        tr[prec] = t.double().cpu().numpy()[0]
        res[prec] = {"ms_per_step": ms, "gpts": N / (ms * 1e-3) / 1e9}
        st.close()
    err = _trace_err(tr["f32"], tr["f64"])
    log(f"[bench pv3d] rows {w.stats()['n_ib']} built in {build_s:.1f} s; FP32 {res['f32']['gpts']:.1f} Gpts/s, "
        f"FP64 {res['f64']['gpts']:.1f} Gpts/s; FP32 vs FP64 max {err['max']:.2e}")
    out = {"metric": "Gpts/s, 3D fourth-order first-order (p-v) IB step", "value": res["f32"]["gpts"],
           "unit": "Gpts/s", "n_gpus": 1, "steps": K, "warmup": Wm, "ms_per_step": res["f32"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3D first-order form {wl.shape[0]}x{wl.shape[1]}x{wl.shape[2]}, dx=10 m, "
                                  "space order 4, fractal free surface, 40-cell damping, 201x201 receivers"},
           "results": res, "fp32_vs_fp64_trace_relL2": err, "modified_rows": w.stats()["n_ib"],
           "weights_build_s": build_s}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--lateral", type=int, default=401)
    ap.add_argument("--depth", type=int, default=301)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--zchunk", type=int, default=-1)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--graph", type=int, default=1)
    ap.add_argument("--patch-variant", type=int, default=-1)
    ap.add_argument("--calibrate", action="store_true", help="(kept for the profiling commands: the 1 GiB "
                    "device copy that calibrates the counters always runs)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the full-length FP32 vs FP64 accuracy runs")
    ap.add_argument("--nt", type=int, default=1500, help="steps of the gradient workload (config5)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--workload", default="config3", choices=["config3", "config2", "config4", "config5", "pv3d"],
                    help="config3 is the headline benchmark; the others report the secondary workloads")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters)
        return
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; sharding shots or a slab decomposition over "
              "several GPUs is not implemented (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "config3":
        {"config2": bench_config2, "config4": bench_config4, "config5": bench_config5,
         "pv3d": bench_pv3d}[args.workload](args)
        return
    import torch

    import paper_2309_03600_amd as ib
    from paper_2309_03600_amd import workloads as W

    K, Wm = args.steps, args.warmup
    t0 = time.time()
    wl = W.config3(nt=K + Wm + 8, lateral=args.lateral, depth=args.depth)
    log(f"[bench] inputs {wl.name} generated in {time.time() - t0:.1f} s")
    torch.cuda.synchronize()
    t0 = time.time()
    w = ib.ib_build_weights(wl.heights, wl.h, wl.shape, space_order=wl.M, surface=wl.surface, eta=wl.eta)
    torch.cuda.synchronize()
    setup_s = time.time() - t0
    stats = w.stats()
    log(f"[bench] weights built in {setup_s:.1f} s: n_ib={stats['n_ib']} sum_nw={stats['sum_nw']} "
        f"max_cond={stats['max_cond']:.3g} radius_hist={stats['radius_hist']} order_hist={stats['order_hist']}")
    N = int(np.prod(wl.shape))
    results = {}
    traces = {}
    for prec in (["f32"] if args.no_fp64 else ["f32", "f64"]):
        dt = torch.float32 if prec == "f32" else torch.float64
        st = ib.ib_state_create(w, wl.vel, wl.dt, wl.src, wl.rec, damp_width=wl.damp_width, precision=prec)
        if args.zchunk >= 0 or args.variant >= 0 or args.patch_variant >= 0:
            st.set_tuning(args.variant if args.variant >= 0 else 1, max(args.zchunk, 0), args.patch_variant)
        wav = torch.tensor(wl.wavelets(np.float64), dtype=dt, device="cuda")
        tr_w = torch.empty((1, Wm, st.nrec), dtype=dt, device="cuda")
        tr = torch.empty((1, K, st.nrec), dtype=dt, device="cuda")
        st.step(Wm, wav, tr_w, use_graph=bool(args.graph))
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t_host = time.perf_counter()
        e0.record(s)
        st.step(K, wav, tr, use_graph=bool(args.graph))
        e1.record(s)
        torch.cuda.synchronize()
        t_host = time.perf_counter() - t_host
        ms = e0.elapsed_time(e1) / K
        traces[prec] = tr.double().cpu().numpy()[0]
        nrep = max(20, min(200, K))
        ms_int = time_kernel(st, 0, nrep, torch)
        ms_patch = time_kernel(st, 1, nrep, torch)
        esz = 4 if prec == "f32" else 8
        # interior kernel at each physical-side node (exterior nodes hold zeros that need no
        # traffic): FP32 reads p^n, d^n, K and writes p^{n+1}, d^{n+1}; FP64 reads p^n,
        # p^{n-1}, K and writes p^{n+1}
        b_int = (5 * esz if prec == "f32" else 4 * esz) * stats["n_interior"]
        b_patch = esz * stats["sum_nw"] + 21 * stats["n_ib"]
        results[prec] = dict(ms_per_step=ms, host_ms_per_step=t_host * 1e3 / K, gpts=N / (ms * 1e-3) / 1e9,
                             gpts_physical=stats["n_interior"] / (ms * 1e-3) / 1e9,
                             interior_ms=ms_int, patch_ms=ms_patch,
                             interior_GBs=b_int / (ms_int * 1e-3) / 1e9, patch_GBs=b_patch / (ms_patch * 1e-3) / 1e9,
                             interior_bytes=b_int, patch_bytes=b_patch,
                             step_alg_GBs=(b_int + b_patch) / (ms * 1e-3) / 1e9)
        log(f"[bench] {prec}: {ms:.4f} ms/step, {results[prec]['gpts']:.1f} Gpts/s; interior {ms_int:.4f} ms "
            f"({results[prec]['interior_GBs']:.0f} GB/s), patch {ms_patch:.4f} ms ({results[prec]['patch_GBs']:.0f} GB/s)")
        st.close()
        del wav, tr, tr_w
        torch.cuda.synchronize()
    r = results["f32"]
    dom = "interior" if r["interior_ms"] >= r["patch_ms"] else "patch"
    traffic = load_traffic()
    tkey = KERNELS[dom]
    roof = {"bound": "hbm", "achieved": r[f"{dom}_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": r[f"{dom}_GBs"] / HBM_PEAK_GBS,
            "traffic": traffic.get(tkey + "/f32", {}).get("bytes_per_launch"), "kernel": tkey,
            "algorithmic_bytes": r[f"{dom}_bytes"], "ms_per_launch": r[f"{dom}_ms"]}
    other = "patch" if dom == "interior" else "interior"
    roof_other = {"kernel": KERNELS[other], "achieved": r[f"{other}_GBs"], "frac": r[f"{other}_GBs"] / HBM_PEAK_GBS,
                  "traffic": traffic.get(KERNELS[other] + "/f32", {}).get("bytes_per_launch"),
                  "algorithmic_bytes": r[f"{other}_bytes"], "ms_per_launch": r[f"{other}_ms"]}
    acc = None
    if not args.no_accuracy and not args.no_fp64:
        acc = accuracy_full_length(torch, ib, w, stats)
    achievable = copy_bandwidth(torch)
    roof["achievable"] = achievable
    roof["frac_of_achievable"] = r[f"{dom}_GBs"] / achievable
    cpu = None
    if not args.no_cpu:
        t0 = time.time()
        cpu = cpu_baseline()
        log(f"[bench] cpu baseline {cpu['value']:.4g} Gpts/s ({time.time() - t0:.1f} s)")
    out = {
        "metric": "Gpts/s & % HBM roofline, 3D 8th-order IB step, FP32 vs FP64 @1e-4 trace err",
        "value": r["gpts"], "unit": "Gpts/s", "n_gpus": 1, "steps": K, "warmup": Wm,
        "ms_per_step": r["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "value_counts": "all grid nodes (air included) per second; gpts_physical counts the physical-side nodes",
        "gpts_physical": r["gpts_physical"],
        "config": {"workload": f"3D second-order acoustic IB step, {wl.shape[0]}x{wl.shape[1]}x{wl.shape[2]}, "
                               "dx=10 m, space order 8, seeded fractal free surface (300 m relief), "
                               "40-cell damping, 1 Ricker source, 201x201 receivers",
                   "grid": list(wl.shape), "space_order": wl.M, "shots": 1, "hip_graph": bool(args.graph)},
        "roofline": roof,
        "roofline_other_kernel": roof_other,
        "cpu_baseline": cpu,
        "kernels": results,
        "fp64": results.get("f64"),
        "fp32_vs_fp64_trace_relL2": acc,
        "setup": {"weights_build_s": setup_s, "n_ib": stats["n_ib"], "sum_nw": stats["sum_nw"],
                  "max_nw": stats["max_nw"], "radius_hist": stats["radius_hist"],
                  "order_hist": stats["order_hist"], "max_cond": stats["max_cond"],
                  "table_bytes_f32": stats["table_bytes_f32"], "dense_weights": stats["dense_weights"],
                  "col_weights": stats["col_weights"]},
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
