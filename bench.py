"""Benchmark: coupled D3Q19 LBM + rigid-fiber time steps on one MI355X.

Workload (default): 256^3 shear cell (walls at the z ends moving at -/+0.01),
64 rigid cylinder fibers, lengths U[24, 40], diameters U[4, 6], uniform
non-overlapping positions, orientations uniform on the sphere (seed 0),
TRT tau = 0.8 with Lambda = 3/16, FP32 deviation storage.  A step is the
whole hot path: fused AA stream-collide with wall and fiber bounce-back,
momentum exchange, rigid-body update, remap with refill, boundary-list
rebuild.  Inputs are synthetic and resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line: MLUPS (all cells x steps / s), the roofline of the
dominant kernel (the bulk stream-collide sweep, timed live with HIP events
on the stream it runs on), and the FP64 oracle's rate on bounded samples on
the host cores (the same workload on all cores; the 32^3 single-fiber cell
in full on all cores and on one core).  The FP16/BF16 deviation-storage
forms of the same workload, the batched form (512 independent one-fiber
shear cells of uneven size, edges 24..64, in one persistent graph-captured
launch with autotuned workgroup size and bin count), and the learned-coarse
form (128^3, 200 under-resolved fibers with the trained closure attached,
beside the same run without it) are timed too and reported under "forms",
each with its error: the storage forms against the FP64 oracle on the 32^3
single-fiber cell (velocity, force and torque after 3000 steps; tumbling
period), the learned form against the resolved fine run (single-fiber
tumbling period).
"""
import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "D3Q19 MLUPS & %HBM peak; FP32 vs FP16-storage vs learned-coarse at fixed error"
HBM_PEAK_GBS = 8000.0
# HBM traffic of the FP32 bulk sweep on this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE passes (profiles/sweep_bulk_256cube_64fibers_traffic.md),
# scaled by the counters' readings for a plain copy of known size.  Valid only
# for the sources it was measured on (SHA-1 of sweep.hip followed by
# lbm_sweep_dev.h, below); otherwise reported null.
SWEEP_TRAFFIC = {"sweep_sha1": "0faaf7ca95c52b06ca254e84f08c38c1ffc95d3a",
                 "bytes_per_launch": 2.5726e+09}
# algorithmic bytes per lattice update of the bulk sweep: 19 loads + 19
# stores of the population type + the 1-byte cell flag
BYTES_PER_LUP = {"f32": 19 * 4 * 2 + 1, "f16": 19 * 2 * 2 + 1, "bf16": 19 * 2 * 2 + 1,
                 "f64": 19 * 8 * 2 + 1}


def build_context(sc, storage, stream, stabilize=False):
    from paper_1503_06869_amd import lbm
    g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u,
                    init_couette=True, storage=storage, stream=stream, stabilize=stabilize)
    for f in sc.fibers:
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    return g


def time_form(sc, storage, steps, warmup, torch, stabilize=False):
    """Whole-step throughput and the bulk sweep's live event timing."""
    stream = torch.cuda.Stream()          # default priority; the context runs on it
    g = build_context(sc, storage, stream.cuda_stream, stabilize)
    g.step(warmup)
    g.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    g.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    g.sync()
    ms = t0.elapsed_time(t1)
    # dominant kernel: bulk sweep, bracketed by events on the context stream
    nsw = max(20, min(steps, 200))
    g.enable_sweep_timing(True)
    g.step(nsw)
    sweep_ms, n = g.sweep_time()
    g.enable_sweep_timing(False)
    info = g.info()
    _, _, flags, _ = g.fields()
    n_solid = int(flags.sum())
    g.close()
    ncell = sc.ncell
    n_bulk = ncell - n_solid - int(info["boundary_cells"])
    bytes_launch = n_bulk * (BYTES_PER_LUP[storage] - 1) + ncell * 1
    avg = sweep_ms / n
    return {
        "ms_per_step": ms / steps,
        "mlups": ncell * steps / (ms * 1e-3) / 1e6,
        "sweep_ms": avg,
        "sweep_gbs": bytes_launch / (avg * 1e-3) / 1e9,
        "sweep_bytes": bytes_launch,
        "bulk_cells": n_bulk,
        "boundary_cells": int(info["boundary_cells"]),
        "solid_cells": n_solid,
    }


def time_batched(steps, warmup, torch, trial_steps=6):
    """Batched form: 512 cases, one persistent launch of `steps` steps."""
    from paper_1503_06869_amd import lbm, scenarios
    cases = scenarios.batched_cases(seed=0)
    stream = torch.cuda.Stream()
    b = lbm.Batch(cases, stream=stream.cuda_stream)
    cache = os.environ.get("LBM_TUNE_CACHE", os.path.join(tempfile.gettempdir(), "lbm_batch_tune.txt"))
    tune = b.autotune(trial_steps=trial_steps, cache_path=cache)
    b.step(warmup)
    b.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    b.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    b.sync()
    ms = t0.elapsed_time(t1) / steps
    info = b.info()
    solid = 0
    for c in range(len(cases)):
        solid += int(b.fields(c)[2].sum())
    b.close()
    cells = info["cells"]
    bytes_step = (cells - solid) * (BYTES_PER_LUP["f32"] - 1) + cells
    return {"mlups": round(cells / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
            "steps_per_launch": steps, "cases": len(cases), "cells": cells,
            "gbs": round(bytes_step / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(bytes_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "threads": tune["threads"], "bins": tune["bins"], "tuning_trials": tune["trials"]}


CLOSURE_NET = os.path.join(ROOT, "paper_1503_06869_amd", "closure_net.npz")


def time_learned(steps, warmup, torch):
    """Learned-coarse form: 128^3, 200 under-resolved fibers (d = 2, AR 4-12),
    with the closure attached, beside the same run without it.  One coarse
    step stands for 2^3 fine cells x 4 fine steps of the resolved run."""
    from paper_1503_06869_amd import closure, lbm, scenarios
    sc = scenarios.learned_coarse(seed=0)
    out = {"cells": sc.ncell, "fibers": len(sc.fibers)}
    if os.path.exists(CLOSURE_NET):
        mlp, _ = closure.load(CLOSURE_NET)
        out["network"] = "trained (paper_1503_06869_amd/closure_net.npz)"
    else:
        mlp = lbm.Mlp(seed=0)
        out["network"] = "untrained (no closure_net.npz): cost only"
    for name, m in (("plain", None), ("learned", mlp)):
        stream = torch.cuda.Stream()
        g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True,
                        stream=stream.cuda_stream)
        for f in sc.fibers:
            g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        if m is not None:
            g.set_closure(m)
        g.step(warmup)
        g.sync()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(stream)
        g.step(steps)
        t1.record(stream)
        torch.cuda.synchronize()
        g.sync()
        ms = t0.elapsed_time(t1) / steps
        out[name] = {"mlups": round(sc.ncell / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4)}
        if m is not None:
            a, fb = g.closure_stats()
            out[name]["fallback_frac"] = round(fb / max(1, a + fb), 4)
        g.close()
    # error at matched physical time: the free tumbling period of one fiber
    # (seed 0) coarse, coarse + closure, and resolved (fine twin, diameter 4,
    # diffusive scaling: 4 fine steps per coarse step)
    from paper_1503_06869_amd import jeffery
    pr = closure.tumble_pair(seed=0)
    nc = 25000
    per = {}
    for name, scn, n, m in (("fine", pr.fine, 4 * nc, None), ("plain", pr.coarse, nc, None),
                            ("learned", pr.coarse, nc, mlp)):
        h, _ = closure.run_free(scn, n, mlp=m)
        T, _ = jeffery.period(jeffery.axis_from_quat(h[:, 9:13])[:, 0], min_crossings=3)
        per[name] = T / (4.0 if name == "fine" else 1.0)
    for name in ("plain", "learned"):
        out[name]["single_fiber_period_rel_error_vs_fine"] = float("%.3g" % (per[name] / per["fine"] - 1))
    out["single_fiber_periods_coarse_steps"] = {k: round(v, 1) for k, v in per.items()}
    mlp.close()
    return out


FP64_VECTOR_PEAK_TFLOPS = 78.6


def time_sbf(torch, m=1024, steps=10, warmup=2):
    """Slender-body form (Sec. 3): a sedimenting cloud of m fibers (1/eps =
    12, N = 5 Legendre modes, 48 quadrature points per fiber, the paper's
    parameters) in free space; a step is the moments of every fiber pair,
    GMRES to 1e-10, the velocities and the Adams-Bashforth-2 update.
    Roofline of its two kernels: the moments (FP64 ALU: per pair
    Q^2 (33 + 15 (N + 1)) + 21 Q (N + 1)^2 flops over m (m - 1)/2 pairs) and
    the product with the symmetric moment matrix (HBM: its D (D + 1)/2
    distinct entries x 8 bytes, D = 3 m (N + 1))."""
    from paper_1503_06869_amd import scenarios, sbf
    N, nq = 5, 16
    sc = scenarios.sbf_cloud(seed=0, m=m)
    stream = torch.cuda.Stream()
    g = sbf.SBF(m, sc.length, sc.eps, nmodes=N, nq=nq, gmres_tol=1e-10, stream=stream.cuda_stream)
    g.set_fibers(sc.X, sc.p, sc.F, sc.M)
    dt = 10.0    # relative displacements of a fraction of a fiber radius per step (speeds ~1e-2)
    g.step(warmup, dt)
    g.enable_timing(True)
    t = time.perf_counter()
    g.step(steps, dt)
    wall = (time.perf_counter() - t) / steps
    tm, nm, tg, ng = g.timing()
    st = g.stats()
    X, _ = g.state()
    g.close()
    Q, NP1 = 3 * nq, N + 1
    flops = (m * (m - 1) / 2) * (Q * Q * (33 + 15 * NP1) + 21 * Q * NP1 * NP1)
    D = 3 * m * NP1
    th_ms, gv_ms = tm / nm, tg / ng
    return {"fibers": m, "modes": N, "quadrature_points": Q, "ms_per_step": round(wall * 1e3, 3),
            "steps_per_s": round(1.0 / wall, 1), "gmres_iterations_last_solve": st["iterations"],
            "finite": bool(np.isfinite(X).all()),
            "moments": {"bound": "alu", "ms": round(th_ms, 4), "achieved_tflops": round(flops / (th_ms * 1e-3) / 1e12, 2),
                        "peak_tflops": FP64_VECTOR_PEAK_TFLOPS,
                        "frac": round(flops / (th_ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS, 4)},
            "gemv": {"bound": "hbm", "ms": round(gv_ms, 4), "launches_per_step": round(ng / steps, 1),
                     "achieved_gbs": round(D * (D + 1) / 2 * 8 / (gv_ms * 1e-3) / 1e9, 1),
                     "frac": round(D * (D + 1) / 2 * 8 / (gv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}


def sweep_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for name in ("sweep.hip", "lbm_sweep_dev.h"):
        h.update(open(os.path.join(ROOT, "paper_1503_06869_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def sweep_traffic():
    return SWEEP_TRAFFIC["bytes_per_launch"] if sweep_sources_sha1() == SWEEP_TRAFFIC["sweep_sha1"] else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_c1(threads, steps):
    """The FP64 oracle on the 32^3 single-fiber shear cell (seed 0, U 0.005)
    on `threads` host threads; returns the sim and the seconds of its step loop."""
    from oracle import pyoracle as O
    from paper_1503_06869_amd import scenarios
    sc = scenarios.single_fiber(seed=0)
    f = sc.fibers[0]
    O.set_threads(threads)
    o = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u, init_couette=True)
    o.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    t = time.perf_counter()
    o.step(steps)
    return o, time.perf_counter() - t


def cpu_baseline(sc, c1_steps=3000, c1_one_core_steps=300, c2_steps=10):
    """FP64 oracle on the host: the 256^3 64-fiber workload (value, all
    cores, c2_steps steps after set-up, per-step rate extrapolated), the
    32^3 single-fiber cell in full (3000 steps, all cores) and on one core
    (c1_one_core_steps, extrapolated).  Returns the record and the all-core
    32^3 oracle run (used for the storage forms' errors)."""
    from oracle import pyoracle as O
    threads = O.get_threads()
    o_c1, t_all = oracle_c1(threads, c1_steps)
    _, t_one = oracle_c1(1, c1_one_core_steps)
    O.set_threads(threads)
    s = O.Sim(sc.nx, sc.ny, sc.nz, tau=sc.tau, magic=sc.magic, wall_u=sc.wall_u, init_couette=True)
    for f in sc.fibers:
        s.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
    t = time.perf_counter()
    s.step(c2_steps)
    dt = time.perf_counter() - t
    del s
    c1 = 32 ** 3
    rec = {"value": round(sc.ncell * c2_steps / dt / 1e6, 2), "unit": "MLUPS", "cores": threads,
           "kind": "oracle",
           "sample": "%d steps of the 256^3 64-fiber shear cell after set-up (FP64, %d OpenMP threads, "
                     "%.1f s; per-step rate extrapolated to the 5000-step run)" % (c2_steps, threads, dt),
           "cpu_model": cpu_model(),
           "c1_32cube_all_cores": {"mlups": round(c1 * c1_steps / t_all / 1e6, 3), "steps": c1_steps,
                                   "seconds": round(t_all, 2), "threads": threads},
           "c1_32cube_one_core": {"mlups": round(c1 * c1_one_core_steps / t_one / 1e6, 3),
                                  "steps": c1_one_core_steps, "seconds": round(t_one, 2), "threads": 1,
                                  "seconds_for_3000_steps_extrapolated": round(t_one * 3000 / c1_one_core_steps, 1)}}
    return rec, o_c1


def _ft_rel(hg, ho, length):
    """Force and torque errors over a run, max over steps, relative to the
    fiber's load (F to max(|F|, |M|/L), M to max(|M|, L|F|))."""
    dF = np.linalg.norm(hg[:, 0:3] - ho[:, 0:3], axis=1).max()
    dM = np.linalg.norm(hg[:, 3:6] - ho[:, 3:6], axis=1).max()
    nF = np.linalg.norm(ho[:, 0:3], axis=1).max()
    nM = np.linalg.norm(ho[:, 3:6], axis=1).max()
    return float(dF / max(nF, nM / length)), float(dM / max(nM, nF * length))


def storage_errors(o_c1, storage, torch, c1_steps=3000, period_steps=124000):
    """Error of a storage form against the FP64 oracle: the 32^3 single-fiber
    cell (U 0.005) after 3000 steps (fluid velocity relative L2, force and
    torque over the run), and its tumbling period over 124,000 steps against
    the oracle's (tests/golden/jeffery_single_fiber.json, written from the
    oracle alone)."""
    from paper_1503_06869_amd import jeffery, lbm, scenarios
    sc = scenarios.single_fiber(seed=0)
    f = sc.fibers[0]
    out = {}
    if o_c1 is not None:
        g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True,
                        storage=storage, history_capacity=c1_steps)
        g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
        g.step(c1_steps)
        _, ug, flg, _ = g.fields()
        hg = g.history(0, c1_steps)[:, 0, :]
        g.close()
        _, uo, flo, _ = o_c1.fields()
        fl = (flo == 0) & (flg == 0)
        eu = float(np.linalg.norm((ug.astype(np.float64) - uo)[:, fl]) / np.linalg.norm(uo[:, fl]))
        eF, eM = _ft_rel(hg, o_c1.history()[:, 0, :], f.length)
        out["c1_3000_steps"] = {"velocity_rel_l2": float("%.3g" % eu), "force_rel": float("%.3g" % eF),
                                "torque_rel": float("%.3g" % eM)}
    gold_path = os.path.join(ROOT, "tests", "golden", "jeffery_single_fiber.json")
    if period_steps > 0 and os.path.exists(gold_path):
        gold = json.load(open(gold_path)).get("U0.005/seed0")
        if gold:
            g = lbm.Context(sc.nx, sc.ny, sc.nz, tau=sc.tau, wall_u=sc.wall_u, init_couette=True,
                            storage=storage, history_capacity=period_steps)
            g.add_fiber(f.X, f.q, f.length, f.radius, f.density_ratio, f.V, f.W)
            g.step(period_steps)
            h = g.history(0, period_steps)
            g.close()
            T, _ = jeffery.period(jeffery.axis_from_quat(h[:, 0, 9:13])[:, 0])
            out["c1_tumbling_period"] = {"steps": round(T, 1), "oracle_steps": round(gold["period"], 1),
                                         "rel_error": float("%.3g" % (T / gold["period"] - 1))}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--forms", default="f16,bf16,stab",
                    help="extra forms to time: storage types, and stab (FP32 with momentum stabilization)")
    ap.add_argument("--batched-steps", type=int, default=200,
                    help="steps of the batched form's timed launch (0: skip it)")
    ap.add_argument("--learned-steps", type=int, default=500,
                    help="steps of the learned-coarse form (0: skip it)")
    ap.add_argument("--sbf-fibers", type=int, default=1024,
                    help="fibers of the slender-body form (0: skip it)")
    ap.add_argument("--no-error-checks", dest="error_checks", action="store_false",
                    help="skip the storage forms' errors against the FP64 oracle")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run the plain copy kernel (traffic-counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(the slab decomposition over xGMI is a design, not code)", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("run with one process per node: --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1503_06869_amd import lbm, scenarios
    lbm.load()
    torch.cuda.set_device(0)
    if a.copy_calib:
        nbytes = 1 << 30
        src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        st = torch.cuda.Stream()
        for _ in range(3):
            lbm.copy_bytes(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(10):
            lbm.copy_bytes(dst.data_ptr(), src.data_ptr(), nbytes, st.cuda_stream)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        print(json.dumps({"copy_bytes_per_launch": 2 * nbytes, "copy_ms": ms,
                          "copy_gbs": 2 * nbytes / (ms * 1e-3) / 1e9}))
        return
    sc = scenarios.many_fibers(seed=0)
    main_form = time_form(sc, "f32", a.steps, a.warmup, torch)
    forms = {"f32": {"mlups": round(main_form["mlups"], 1),
                     "sweep_hbm_frac": round(main_form["sweep_gbs"] / HBM_PEAK_GBS, 4)}}
    cpu, o_c1 = (None, None) if a.no_cpu else cpu_baseline(sc)
    if a.error_checks:
        forms["f32"]["error_vs_fp64_oracle"] = storage_errors(o_c1, "f32", torch)
    for st in [s for s in a.forms.split(",") if s]:
        if st == "stab":
            # the same step with the momentum stabilization's bookkeeping
            r = time_form(sc, "f32", max(100, a.steps // 2), a.warmup, torch, stabilize=True)
            forms["f32_stabilized"] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                                       "sweep_ms": round(r["sweep_ms"], 4),
                                       "step_time_vs_f32": round(r["ms_per_step"] / main_form["ms_per_step"], 4)}
            continue
        r = time_form(sc, st, max(100, a.steps // 2), a.warmup, torch)
        forms[st] = {"mlups": round(r["mlups"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                     "sweep_gbs": round(r["sweep_gbs"], 1),
                     "sweep_hbm_frac": round(r["sweep_gbs"] / HBM_PEAK_GBS, 4)}
        if a.error_checks:
            forms[st]["error_vs_fp64_oracle"] = storage_errors(o_c1, st, torch)
    if a.batched_steps > 0:
        forms["batched_512_cases"] = time_batched(a.batched_steps, 10, torch)
    if a.learned_steps > 0:
        forms["learned_coarse_128cube_200fibers"] = time_learned(a.learned_steps, 20, torch)
    if a.sbf_fibers > 0:
        forms["slender_body_cloud"] = time_sbf(torch, m=a.sbf_fibers)
    out = {
        "metric": METRIC,
        "value": round(main_form["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_form["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "256^3 shear cell, 64 rigid cylinder fibers (L 24-40, d 4-6), "
                               "TRT tau 0.8, U 0.01, FP32 deviation storage, seed 0",
                   "cells": sc.ncell, "fibers": len(sc.fibers),
                   "bulk_cells": main_form["bulk_cells"],
                   "boundary_cells": main_form["boundary_cells"],
                   "solid_cells": main_form["solid_cells"]},
        "roofline": {"bound": "hbm", "achieved": round(main_form["sweep_gbs"], 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(main_form["sweep_gbs"] / HBM_PEAK_GBS, 4),
                     "traffic": sweep_traffic(),
                     "kernel": "k_sweep_bulk (even/odd AA)",
                     "kernel_ms": round(main_form["sweep_ms"], 5),
                     "algorithmic_bytes_per_launch": main_form["sweep_bytes"]},
        "forms": forms,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
