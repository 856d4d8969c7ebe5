"""Benchmark of the explicit hot path on one MI355X.

A step = one fused velocity-Verlet step over the whole mesh: bond-force
gather + critical-stretch damage test + half-kicks + drift + boundary data
(pd_verlet_step).  Default workload: the jittered 100^3 cube (1M nodes,
delta = 3h, damage on, velocity-driven uniaxial tension) in mixed precision.  Inputs are synthetic and
resident in HBM before the timed region; the neighbour build is one-off and
reported separately.  "fp64" and "mixed" compute the bond terms in float64;
"mixed" takes 1/|xi| from the hardware reciprocal-square-root estimate without
refinement; "fp32" (timed beside them) computes the bond terms in float32 after
float64 differences, with compensated float32 sums per node.

Then (unless --no-law) the other material laws: NP explicit steps on the
notched 512^2 plate, linear-peridynamic-solid steps on the cube, and the NP
Newton-Krylov solve of the 400 x 40 bar ("law" object).
Then (unless --no-serve) the serving workload: independent notched-plate
requests through pd_server_* under a device-memory budget, first all at
once (saturated throughput), then with Poisson arrivals at a fraction of that
rate; completion latency (arrival to result) p50/p99 and aggregate bond
evaluations per second go into the line's "serving" object.

Prints one JSON line.  `roofline` prices the step kernel against HBM with the
algorithmic byte model B = nnz * 5 + n * (93 | 133) bytes (2-d | 3-d):
per bond a 4-byte column index and a 1-byte flag, per node the row offset,
X, V, u, v, the boundary kind read once and u', v' written once.  The other
laws' step figures carry a `roofline` of the whole step by the same model
(the solid: two passes, plus 32 B of coefficients per node written by the
first and read by the second).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the sources of the dominant kernel (stream_kernel): its traffic record is
# valid only while these are unchanged
KERNEL_SOURCES = ["pd_kernels.hpp", "pd_stream.hip", "pd_internal.hpp"]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "stream_kernel_cube100_traffic.md")
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "stream_kernel_cube100_counters.md")
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3   # packed; scalar FP32 issues at the FP64 rate


def kernel_source_hash():
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1806_06917_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_profile(path, workload, precision, launch=None):
    """The JSON record of a committed rocprofv3 summary -- only if the kernel
    sources are unchanged since the counters were taken and (launch given)
    the counters were taken at the same tile size and lane count."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"```json\n(.*?)```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    if rec.get("workload") != workload or rec.get("precision") != precision:
        return None
    if launch is not None and (rec.get("tile"), rec.get("lanes")) != (launch.get("tile"),
                                                                       launch.get("lanes")):
        return None
    return rec


def recorded_traffic(workload, precision, launch=None):
    """HBM bytes per launch measured with rocprofv3 (FETCH_SIZE + WRITE_SIZE,
    scaled by a plain copy kernel), under the conditions of recorded_profile."""
    rec = recorded_profile(TRAFFIC_SUMMARY, workload, precision, launch)
    return rec.get("hbm_bytes_per_launch") if rec else None


def recorded_valu(workload, precision, launch, nnz):
    """VALU figures of the step kernel from the committed SQ counters (same
    conditions): busy fraction of the SIMDs, FP64 rate against the vector
    FP64 peak, and lane-instructions per bond."""
    rec = recorded_profile(COUNTER_SUMMARY, workload, precision, launch)
    if not rec:
        return None
    k32 = rec.get("fp32_mode_kernel", {})
    return {"valu_busy": rec["valu_busy"], "fp64_tflops": rec["fp64_tflops"],
            "fp64_peak_tflops": FP64_PEAK_TFLOPS,
            "fp64_frac": rec["fp64_tflops"] / FP64_PEAK_TFLOPS,
            "fp32_tflops": rec.get("fp32_tflops"),
            "fp32_peak_tflops": FP32_PEAK_TFLOPS,
            "lane_instr_per_bond": rec["valu_lane_instr_per_bond"],
            "fp32_mode_kernel": {"valu_busy": k32.get("valu_busy"),
                                 "fp32_tflops": k32.get("fp32_tflops"),
                                 "fp32_frac": (k32["fp32_tflops"] / FP32_PEAK_TFLOPS
                                               if k32 else None),
                                 "lane_instr_per_bond": k32.get("valu_lane_instr_per_bond")},
            "source": os.path.relpath(COUNTER_SUMMARY, ROOT)}


def algorithmic_bytes(n, nnz, dim):
    per_node = 4 + 3 * dim * 8 + 8 + 1 + 2 * dim * 8
    return nnz * 5 + n * per_node


def lps_algorithmic_bytes(n, nnz, dim):
    """The solid's step is two passes over the bonds: the state pass reads the
    bonds, row offsets, X and u and writes 32 B of coefficients per node; the
    force pass is the linear law's step plus those coefficients read once."""
    state = nnz * 5 + n * (4 + 2 * dim * 8 + 32)
    return state + algorithmic_bytes(n, nnz, dim) + n * 32


def step_roofline(bytes_per_step, ms):
    """Algorithmic bytes of one step over its measured time, priced against
    HBM (the whole step: both passes where there are two)."""
    gbs = bytes_per_step / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_step": bytes_per_step}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="cube100",
                    choices=["cube100", "notched512", "plate32", "paper443"])
    ap.add_argument("--precision", default=None, choices=["fp64", "mixed", "fp32"])
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--kernel", default="auto", choices=["auto", "gather", "tile"])
    ap.add_argument("--tile", type=int, default=0, help="nodes per tile (0 = automatic)")
    ap.add_argument("--block", type=int, default=0, help="threads per tile workgroup (0 = auto)")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed windows of --steps steps each; the median is reported")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 512^2 / 32^2 / 443^2 plates and the implicit bar")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-validation", action="store_true",
                    help="skip the 2-d and 1-d convergence studies")
    ap.add_argument("--no-law", action="store_true",
                    help="skip the NP-law measurements (explicit steps, Newton-Krylov)")
    ap.add_argument("--convergence", action="store_true",
                    help="run only the 2-d convergence study (LP and NP, both initial "
                         "conditions, t = 0..2) and print its rates")
    ap.add_argument("--convergence-t", type=float, default=2.0)
    ap.add_argument("--no-autotune", action="store_true",
                    help="built-in launch heuristics instead of the autotuner's choice")
    ap.add_argument("--serve-count", type=int, default=256)
    ap.add_argument("--serve-budget-gib", type=float, default=4.0)
    ap.add_argument("--serve-chunk", type=int, default=100)
    ap.add_argument("--serve-load", type=float, default=0.8,
                    help="Poisson arrival rate as a fraction of the saturated request rate")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times "
                         "(reference kernel for scaling the HBM byte counters)")
    return ap.parse_args()


def progress(*args):
    print("[bench]", *args, file=sys.stderr, flush=True)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def timed_windows(torch, ctx, work, reps):
    """Times `work` (a fixed number of steps) reps times with HIP events on the
    context's stream, each window bracketed by device synchronisation;
    returns the window times (ms) and the wall time of all of them."""
    stream = ctx.stream
    out = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        work()
        e1.record(stream)
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return out, time.perf_counter() - t0


def run_gpu(torch, pd, w, precision, steps, warmup, lanes, tuning=("auto", 0, 0), tune=True,
            reps=5):
    ctx = pd.Context(0)
    if lanes:
        ctx.set_lanes(lanes)
    ctx.set_tuning(*tuning)
    Xd = dev(torch, w.X)
    tuned = None
    progress(w.name, precision, "neighbours, tuning, timing")
    if tune and not lanes and tuning == ("auto", 0, 0):
        # launch shape from the autotuner (cached in ctx for this mesh's kind)
        t0 = time.perf_counter()
        best, table = ctx.autotune(Xd, dev(torch, w.V), w.delta, precision, steps=20)
        tuned = {"best": best, "candidates": table, "search_s": time.perf_counter() - t0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb = pd.Neighbors(ctx, Xd, w.delta)
    t_nbr = time.perf_counter() - t0
    c = pd.micromodulus(w.dim, w.E, w.delta)
    mat = pd.material(w.dim, c, w.rho, w.s_c, precision)
    sim = pd.Simulation(ctx, nb, mat, Xd, dev(torch, w.V), dev(torch, w.u0), dev(torch, w.v0),
                        bc_kind=dev(torch, w.bc_kind), bc_vel=dev(torch, w.bc_vel),
                        notch=w.notch, ramp_steps=w.ramp_steps)
    sim.step(warmup, w.dt)
    windows, wall = timed_windows(torch, ctx, lambda: sim.step(steps, w.dt), reps)
    info = sim.get(energies=True)
    res = {"ms_total": float(np.median(windows)), "windows_ms": windows, "wall_s": wall,
           "nnz": nb.nnz, "t_nbr_s": t_nbr, "ke": info["ke"], "pe": info["pe"],
           "step": info["step"], "launch": sim.info(), "autotune": tuned}
    sim.close()
    nb.close()
    ctx.close()
    return res


def serve(pd, reqs, budget, chunk, rate=None, tile=0, precision="mixed"):
    """Runs the requests through pd_server_* with arrivals at their Poisson
    times (rate given) or all at once; returns completion-latency statistics
    and the aggregate bond-evaluation rate.  tile: nodes per tile of the
    requests' simulations (0: automatic)."""
    from paper_1806_06917_amd import inputs
    progress("serving", len(reqs), "requests", "burst" if rate is None else f"rate {rate:.1f}/s")
    loads = []
    for q in reqs:
        w = inputs.serving_workload(q)
        loads.append((w, pd.micromodulus(w.dim, w.E, w.delta)))
    ctx = pd.Context(0)
    ctx.set_tuning("auto", tile, 0)
    srv = pd.Server(ctx, budget, chunk_steps=chunk, lanes=4)
    t0 = pd.Server.clock()
    ids, k, most, rounds = [], 0, 0, 0
    while True:
        now = pd.Server.clock() - t0
        while k < len(reqs) and (rate is None or reqs[k].arrival <= now):
            w, c = loads[k]
            t_arr = t0 + (reqs[k].arrival if rate is not None else 0.0)
            ids.append(srv.submit(w.X, w.V, pd.material(w.dim, c, w.rho, w.s_c, precision),
                                  w.delta, w.dt, w.steps, bc_kind=w.bc_kind, bc_vel=w.bc_vel,
                                  notch=w.notch, ramp_steps=w.ramp_steps,
                                  t_arrival=max(t_arr, 1e-9)))
            k += 1
        running, queued = srv.pump()
        rounds += 1
        most = max(most, running)
        if running == 0 and queued == 0:
            if k == len(reqs):
                break
            wait = t0 + reqs[k].arrival - pd.Server.clock()
            if wait > 0:
                time.sleep(wait)
    t_end = pd.Server.clock()
    infos = [srv.info(i) for i in ids]
    _, peak = srv.usage()
    stats = srv.stats()
    srv.close()
    ctx.close()
    ok = [f for f in infos if f["state"] == pd.PD_REQ_DONE]
    lat = np.array([f["t_done"] - f["t_submit"] for f in ok])
    queue = np.array([f["t_admit"] - f["t_submit"] for f in ok])
    evals = sum(f["bonds"] * q.steps for f, q in zip(infos, reqs)
                if f["state"] == pd.PD_REQ_DONE)
    span = t_end - t0
    # host time of admission and retirement that the device did not hide
    # (admission during a running chunk overlaps it)
    exposed = stats["admit_s"] - stats["admit_overlap_s"] + stats["retire_s"]
    return {"requests": len(reqs), "completed": len(ok), "makespan_s": span,
            "admit_retire_exposed_s": exposed, "admit_retire_exposed_frac": exposed / span,
            "bond_evals_per_s": evals / span, "requests_per_s": len(ok) / span,
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "queue_p50_s": float(np.percentile(queue, 50)),
            "max_running": most, "rounds": rounds, "peak_bytes": peak, "server": stats}


def config_runs(torch, pd, steps, warmup):
    """The other explicit workloads in the linearised law, timed like the
    headline one: the 512^2 notched plate (notch, collars, damage) in each
    precision, the 32^2 free plate (100 steps per window, FP64) and the
    paper's benchmark shape, the 443^2 plate with a 20-cell horizon (mixed
    and FP64, 100 steps per window)."""
    from paper_1806_06917_amd import inputs
    out = {}
    for name, precs, k in (("notched512", ("mixed", "fp64", "fp32"), steps),
                           ("plate32", ("fp64",), 100),
                           ("paper443", ("mixed", "fp64"), 100)):
        w = inputs.CONFIGS[name]()
        for prec in precs:
            r = run_gpu(torch, pd, w, prec, k, warmup, 0)
            ms = r["ms_total"] / k
            out[f"{name}_{prec}"] = {
                "workload": w.name, "nodes": w.n, "bonds": r["nnz"], "precision": prec,
                "steps": k, "ms_per_step": ms,
                "windows_ms_per_step": [x / k for x in r["windows_ms"]],
                "bond_evals_per_s": r["nnz"] / (ms * 1e-3), "launch": r["launch"],
                "neighbor_build_s": r["t_nbr_s"],
                "roofline": step_roofline(algorithmic_bytes(w.n, r["nnz"], w.dim), ms)}
    return out


def implicit_runs(torch, pd):
    """Time to solution of the linear quasi-static 400 x 40 bar (relative
    residual 1e-10) in FP64 and in mixed precision."""
    from paper_1806_06917_amd import inputs
    wb = inputs.CONFIGS["bar400x40"]()
    progress("implicit bar", wb.name)
    ctx = pd.Context(0)
    Xb, Vb, bb = dev(torch, wb.X), dev(torch, wb.V), dev(torch, wb.b)
    fixed = dev(torch, wb.fixed)
    nb = pd.Neighbors(ctx, Xb, wb.delta)
    cb = pd.micromodulus(2, wb.E, wb.delta)
    out = {}
    for prec in ("fp64", "mixed", "fp64", "mixed"):      # the first pair warms up
        u = dev(torch, wb.u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pd.solve_implicit(ctx, nb, pd.material(2, cb, precision=prec), Xb, Vb, bb, u,
                                fixed=fixed, rtol=1e-10)
        t = time.perf_counter() - t0
        out[prec] = {"workload": wb.name, "seconds": t, "outer_iterations": res.outer,
                     "cg_iterations": res.inner, "rel_residual": res.rel_residual,
                     "bonds": nb.nnz}
    nb.close()
    ctx.close()
    return out


def law_runs(torch, pd, steps, tuned=None):
    """The other material laws: NP explicit steps on the notched 512^2 plate
    and linear-peridynamic-solid steps (two passes per step) on the 1M-node
    cube, both on the streamed kernel, and the NP Newton-Krylov solve of the
    400 x 40 bar (beta set so that beta |xi| S^2 reaches 0.1 at the linear
    solution).  The step timings are the median of five windows after 20
    warm-up steps (the first milliseconds of a run are slower while the
    device clock ramps up).  tuned: (dim, mean neighbours, precision, tile,
    lanes) entries of the autotuner to seed this context with."""
    from paper_1806_06917_amd import inputs
    out = {}
    ctx = pd.Context(0)
    for t in tuned or ():
        ctx.tune_set(*t)
    w = inputs.CONFIGS["notched512"]()
    progress("NP law, explicit steps,", w.name)
    X = dev(torch, w.X)
    nb = pd.Neighbors(ctx, X, w.delta)
    c = pd.micromodulus(w.dim, w.E, w.delta)
    for prec in ("mixed", "fp64"):
        mat = pd.material(w.dim, c, w.rho, 0.0, prec, law="np", beta=1e3)
        sim = pd.Simulation(ctx, nb, mat, X, dev(torch, w.V), dev(torch, w.u0),
                            dev(torch, w.v0), bc_kind=dev(torch, w.bc_kind),
                            bc_vel=dev(torch, w.bc_vel), notch=w.notch,
                            ramp_steps=w.ramp_steps)
        sim.step(20, w.dt)
        windows, _ = timed_windows(torch, ctx, lambda: sim.step(steps, w.dt), 5)
        ms = float(np.median(windows)) / steps
        out[f"np_step_{prec}"] = {"workload": w.name, "ms_per_step": ms,
                                  "windows_ms_per_step": [x / steps for x in windows],
                                  "bond_evals_per_s": nb.nnz / (ms * 1e-3),
                                  "launch": sim.info(), "beta": 1e3,
                                  "roofline": step_roofline(
                                      algorithmic_bytes(w.n, nb.nnz, w.dim), ms)}
        sim.close()
    nb.close()
    wc = inputs.CONFIGS["cube100"]()
    progress("linear peridynamic solid, explicit steps,", wc.name)
    Xc = dev(torch, wc.X)
    nb = pd.Neighbors(ctx, Xc, wc.delta)
    K, mu = wc.E / (3 * (1 - 2 * 0.25)), wc.E / (2 * (1 + 0.25))
    for prec in ("mixed", "fp64"):
        mat = pd.material(3, 0.0, wc.rho, 0.0, prec, law="lps", bulk=K, shear=mu)
        sim = pd.Simulation(ctx, nb, mat, Xc, dev(torch, wc.V), dev(torch, wc.u0),
                            dev(torch, wc.v0), bc_kind=dev(torch, wc.bc_kind),
                            bc_vel=dev(torch, wc.bc_vel), ramp_steps=wc.ramp_steps)
        sim.step(20, wc.dt)
        k = steps // 4
        windows, _ = timed_windows(torch, ctx, lambda: sim.step(k, wc.dt), 5)
        ms = float(np.median(windows)) / k
        out[f"lps_step_{prec}"] = {"workload": wc.name, "ms_per_step": ms,
                                   "windows_ms_per_step": [x / k for x in windows],
                                   "bond_evals_per_s": nb.nnz / (ms * 1e-3),
                                   "launch": sim.info(), "nu": 0.25,
                                   "roofline": step_roofline(
                                       lps_algorithmic_bytes(wc.n, nb.nnz, wc.dim), ms)}
        sim.close()
    nb.close()
    wb = inputs.CONFIGS["bar400x40"]()
    progress("NP law, Newton-Krylov,", wb.name)
    Xb, Vb, bb = dev(torch, wb.X), dev(torch, wb.V), dev(torch, wb.b)
    fixed = dev(torch, wb.fixed)
    nb = pd.Neighbors(ctx, Xb, wb.delta)
    cb = pd.micromodulus(2, wb.E, wb.delta)
    u = dev(torch, wb.u0)
    pd.solve_implicit(ctx, nb, pd.material(2, cb), Xb, Vb, bb, u, fixed=fixed, rtol=1e-10)
    rp, col = nb.export()
    ul = u.cpu().numpy()
    i = np.repeat(np.arange(wb.n), np.diff(rp))
    xi = wb.X[col] - wb.X[i]
    S = np.sum(xi * (ul[col] - ul[i]), 1) / np.sum(xi * xi, 1)
    beta = 0.1 / float(np.max(np.sqrt(np.sum(xi * xi, 1)) * S * S))
    for prec in ("fp64", "mixed"):
        u = dev(torch, wb.u0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = pd.solve_implicit(ctx, nb, pd.material(2, cb, precision=prec, law="np", beta=beta),
                                Xb, Vb, bb, u, fixed=fixed, rtol=1e-10)
        t = time.perf_counter() - t0
        out[f"np_newton_{prec}"] = {"workload": wb.name, "seconds": t, "newton_steps": res.outer,
                                    "cg_iterations": res.inner,
                                    "rel_residual": res.rel_residual, "beta": beta}
    nb.close()
    ctx.close()
    return out


def convergence(torch, pd, law, ic, t_end=2.0, every=0.25, chunk=500):
    """The paper's 2-d convergence study on the GPU: the plate with the
    clamped collar at h = delta/2, delta/4, delta/8, stepped together in
    batched launches; at every checkpoint the rate
    alpha = (log||u1 - u2|| - log||u2 - u3||) / log 2, the norms over [0,1]^2
    on the coarser grid of each pair (finer solution averaged onto it)."""
    from paper_1806_06917_amd import inputs
    ws = [inputs.convergence_plate(m, ic) for m in (2, 4, 8)]
    delta = ws[0].delta
    c = 4.0 / (np.pi * delta ** 3)          # 4 psi'(0)/(delta |B_delta|), psi'(0) = C beta = 1
    ctx = pd.Context(0)
    ctx.set_lanes(8)              # one launch shape for the three meshes
    ctx.set_tuning("auto", 64, 0)
    made = []
    for w in ws:
        nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta)
        mat = pd.material(2, c, 1.0, 0.0, "fp64", law=law, beta=1.0)
        sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                            dev(torch, w.v0), bc_kind=dev(torch, w.bc_kind),
                            bc_vel=dev(torch, w.bc_vel))
        made.append((nb, sim))
    sims = [s for _, s in made]
    batch = pd.Batch(ctx)
    dt = ws[0].dt
    per = int(round(every / dt))
    rows = []
    t0 = time.perf_counter()
    step = 0
    while step * dt < t_end - 1e-12:
        for _ in range(per // chunk):
            batch.step(sims, [chunk] * 3, [dt] * 3, chunk)
        step += per
        us = []
        for w, (nb, s) in zip(ws, made):
            u = torch.zeros((w.n, 2), dtype=torch.float64, device="cuda")
            s.get(u)
            us.append(u.cpu().numpy())
        norms = []
        for k in range(2):
            N = ws[k].shape[0]
            d = us[k] - inputs.coarsen(us[k + 1], N)
            inside = ws[k].bc_kind == inputs.BC_FREE
            norms.append(float(np.sqrt(np.sum(d[inside] ** 2) * ws[k].h ** 2)))
        rows.append({"t": round(step * dt, 6), "diff12": norms[0], "diff23": norms[1],
                     "alpha": float(np.log(norms[0] / norms[1]) / np.log(2.0))})
    secs = time.perf_counter() - t0
    batch.close()
    for nb, s in made:
        s.close()
        nb.close()
    ctx.close()
    return {"law": law, "ic": ic, "steps": step, "dt": dt, "seconds": secs,
            "nodes": [w.n for w in ws], "rates": rows}


def convergence_1d(torch, pd, law, ic, t_end=2.0, every=0.25, pv=False):
    """The paper's 1-d convergence study on the GPU: the bar [0,1] with the
    clamped collars [-delta, 0] and [1, 1+delta], delta = 0.01, influence
    function J(r) = r exp(-r^2/0.4), psi(r) = 1 - exp(-r) (NP) or its
    linearisation (LP), force (2/delta^2) J psi'(r) S per unit length, at
    h = delta/2, delta/4, delta/8, delta/16 (a line of nodes in 2-d, gather
    kernel, one simulation per mesh); at every checkpoint the rate of the
    two sets {h1, h2, h3} and {h2, h3, h4}, norms over [0,1] on the coarser
    line of each pair (finer solution averaged onto it).  pv: partial volumes
    (neighbours out to delta + h/2, the node at distance delta weighted 1/2)."""
    from paper_1806_06917_amd import inputs
    ws = [inputs.convergence_line(m, ic) for m in (2, 4, 8, 16)]
    delta = ws[0].delta
    c = 2.0 / delta ** 2                    # (2/delta^2) psi'(0), psi'(0) = C beta = 1
    ctx = pd.Context(0)
    made = []
    for w in ws:
        pv_h = w.h if pv else 0.0
        nb = pd.Neighbors(ctx, dev(torch, w.X), w.delta + pv_h / 2)
        mat = pd.material(2, c, 1.0, 0.0, "fp64", law=law, beta=1.0, j=inputs.INFLUENCE_1D,
                          pv_h=pv_h)
        sim = pd.Simulation(ctx, nb, mat, dev(torch, w.X), dev(torch, w.V), dev(torch, w.u0),
                            dev(torch, w.v0), bc_kind=dev(torch, w.bc_kind),
                            bc_vel=dev(torch, w.bc_vel))
        made.append((nb, sim))
    dt = ws[0].dt
    per = int(round(every / dt))
    rows = []
    t0 = time.perf_counter()
    step = 0
    while step * dt < t_end - 1e-12:
        for _, s in made:
            s.step(per, dt)
        step += per
        us = []
        for w, (nb, s) in zip(ws, made):
            u = torch.zeros((w.n, 2), dtype=torch.float64, device="cuda")
            s.get(u)
            us.append(u.cpu().numpy())
        norms = []
        for k in range(3):
            d = us[k] - inputs.coarsen_line(us[k + 1], ws[k].n)
            inside = ws[k].bc_kind == inputs.BC_FREE
            norms.append(float(np.sqrt(np.sum(d[inside] ** 2) * ws[k].h)))
        rows.append({"t": round(step * dt, 6), "diff": norms,
                     "alpha_set1": float(np.log(norms[0] / norms[1]) / np.log(2.0)),
                     "alpha_set2": float(np.log(norms[1] / norms[2]) / np.log(2.0))})
    secs = time.perf_counter() - t0
    for nb, s in made:
        s.close()
        nb.close()
    ctx.close()
    return {"law": law, "ic": ic, "steps": step, "dt": dt, "seconds": secs,
            "nodes": [w.n for w in ws], "rates": rows}


def copy_probe(torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rate of this GPU (read + write bytes over the
    copy's time, median of reps), the attainable-bandwidth context for the
    8 TB/s peak."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    del a, b
    return 2 * nbytes / (float(np.median(ts)) * 1e-3) / 1e9


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, steps, steps_1t):
    """The FP64 oracle, as it stands, on the same workload: `steps` velocity-
    Verlet steps on all the host's cores (OpenMP over nodes), then
    `steps_1t` on one thread."""
    from oracle import oracle as orc
    progress("oracle on the host,", steps, "steps on all cores,", steps_1t, "on one")
    mesh = orc.Mesh(w.X, w.V, w.delta)
    c = orc.micromodulus(w.dim, w.E, w.delta)
    cores = orc.num_threads()

    def run(k):
        st = mesh.start(w.u0, w.v0, c, w.s_c)
        t0 = time.perf_counter()
        mesh.verlet(st, c, w.rho, w.s_c, w.dt, k, w.bc_kind, w.bc_vel, None, w.ramp_steps)
        return time.perf_counter() - t0

    dt = run(steps)
    orc.set_threads(1)
    try:
        dt1 = run(steps_1t)
    finally:
        orc.set_threads(cores)
    return {"value": mesh.nnz * steps / dt, "unit": "bond evals/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} velocity-Verlet steps of the full workload ({mesh.n} nodes, "
                      f"{mesh.nnz} bonds), FP64, OpenMP over nodes on {cores} threads, "
                      f"{dt:.2f} s; then {steps_1t} steps on one thread, {dt1:.2f} s",
            "ms_per_step": 1e3 * dt / steps,
            "single_thread": {"value": mesh.nnz * steps_1t / dt1, "unit": "bond evals/s",
                              "ms_per_step": 1e3 * dt1 / steps_1t, "steps": steps_1t},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_config_baselines(gpu_configs, gpu_implicit):
    """The FP64 oracle on the other workloads, on all the host's cores: 100
    velocity-Verlet steps of the 512^2 notched plate (notch, collars,
    damage) and of the 32^2 free plate, 5 of the 443^2 plate with a 20-cell
    horizon, and the 400 x 40 bar's quasi-static
    solve to a relative residual of 1e-10; each beside the GPU's time for
    the same work when that was measured in this run."""
    from oracle import oracle as orc
    from paper_1806_06917_amd import inputs
    out = {}
    for name, k in (("notched512", 100), ("plate32", 100), ("paper443", 5)):
        w = inputs.CONFIGS[name]()
        progress("oracle on the host,", name, k, "steps")
        mesh = orc.Mesh(w.X, w.V, w.delta)
        c = orc.micromodulus(w.dim, w.E, w.delta)
        alive = mesh.notch_cut(w.notch, mesh.all_alive()) if w.notch is not None else None
        st = mesh.start(w.u0, w.v0, c, w.s_c, alive)
        t0 = time.perf_counter()
        mesh.verlet(st, c, w.rho, w.s_c, w.dt, k, w.bc_kind, w.bc_vel, None, w.ramp_steps)
        ms = 1e3 * (time.perf_counter() - t0) / k
        rec = {"workload": w.name, "steps": k, "ms_per_step": ms,
               "bond_evals_per_s": mesh.nnz / (ms * 1e-3)}
        for prec in ("mixed", "fp64"):
            g = (gpu_configs or {}).get(f"{name}_{prec}")
            if g:
                rec[f"gpu_speedup_{prec}"] = ms / g["ms_per_step"]   # oracle time over GPU time
        out[name] = rec
    wb = inputs.CONFIGS["bar400x40"]()
    progress("oracle on the host, implicit bar", wb.name)
    mesh = orc.Mesh(wb.X, wb.V, wb.delta)
    c = orc.micromodulus(2, wb.E, wb.delta)
    t0 = time.perf_counter()
    _, info = mesh.solve_implicit(wb.u0, c, wb.b, wb.fixed, rtol=1e-10, inner_rtol=1e-10)
    sec = time.perf_counter() - t0
    rec = {"workload": wb.name, "seconds": sec, "cg_iterations": info["inner"],
           "rel_residual": info["relres"]}
    for prec in ("fp64", "mixed"):
        g = (gpu_implicit or {}).get(prec)
        if g:
            rec[f"gpu_speedup_{prec}"] = sec / g["seconds"]
    out["bar400x40"] = rec
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                          "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8, "launches": 5}))
        return

    from paper_1806_06917_amd import inputs
    from paper_1806_06917_amd import pd

    if args.convergence:
        res = []
        for law in ("linear", "np"):
            for ic in (1, 2):
                progress("convergence study", law, "IC", ic)
                res.append(convergence(torch, pd, law, ic, args.convergence_t))
        res1 = []
        for pv in (False, True):
            for law in ("linear", "np"):
                for ic in (1, 2):
                    progress("1-d convergence study", law, "IC", ic, "pv" if pv else "")
                    r = convergence_1d(torch, pd, law, ic, args.convergence_t, pv=pv)
                    res1.append(dict(r, partial_volumes=pv))
        print(json.dumps({"validation": "convergence studies", "runs_2d": res,
                          "runs_1d": res1}), flush=True)
        return

    w = inputs.CONFIGS[args.config]()
    precision = args.precision or ("mixed" if args.config == "cube100" else "fp64")
    tuning = (args.kernel, args.tile, args.block)
    r = run_gpu(torch, pd, w, precision, args.steps, args.warmup, args.lanes, tuning,
                not args.no_autotune, args.reps)
    ms_step = r["ms_total"] / args.steps           # median window
    bonds_per_s = r["nnz"] / (ms_step * 1e-3)
    B = algorithmic_bytes(w.n, r["nnz"], w.dim)
    achieved = B / (ms_step * 1e-3) / 1e9
    traffic = recorded_traffic(w.name, precision, r["launch"])
    copy_gbs = copy_probe(torch)
    out = {
        "metric": "bond evals/sec + ms/explicit step at 1M nodes",
        "value": bonds_per_s,
        "unit": "bond evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": w.n, "bonds": r["nnz"], "dim": w.dim,
                   "horizon": f"{round(w.delta / w.h)}h", "damage_s_c": w.s_c,
                   "precision": precision, "dt": w.dt, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic,
                     "traffic_gbs": traffic / (ms_step * 1e-3) / 1e9 if traffic else None,
                     "traffic_frac": (traffic / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS
                                      if traffic else None),
                     "valu": recorded_valu(w.name, precision, r["launch"], r["nnz"]),
                     "copy_probe_gbs": copy_gbs,
                     "frac_of_copy_probe": achieved / copy_gbs,
                     "algorithmic_bytes_per_launch": B,
                     "kernel_source_hash": kernel_source_hash()},
        "timing": {"windows": args.reps, "steps_per_window": args.steps,
                   "windows_ms_per_step": [x / args.steps for x in r["windows_ms"]],
                   "statistic": "median window"},
        "neighbor_build_s": r["t_nbr_s"],
        "launch": r["launch"],
        "autotune": r["autotune"],
    }
    if not args.no_fp64_compare and precision == "mixed":
        r64 = run_gpu(torch, pd, w, "fp64", args.steps, args.warmup, args.lanes, tuning,
                      not args.no_autotune, args.reps)
        out["fp64_ms_per_step"] = r64["ms_total"] / args.steps
        out["fp64_launch"] = r64["launch"]
        r32 = run_gpu(torch, pd, w, "fp32", args.steps, args.warmup, args.lanes, tuning,
                      not args.no_autotune, args.reps)
        out["fp32_ms_per_step"] = r32["ms_total"] / args.steps
        out["fp32_launch"] = r32["launch"]
    if not args.no_configs:
        out["configs"] = config_runs(torch, pd, 200, 20)
        out["implicit"] = implicit_runs(torch, pd)
    if not args.no_law:
        # the solid's cube steps use the autotuner's shape for this mesh kind
        seeds = []
        for prec, rr in ((precision, r), ("fp64", r64 if "fp64_launch" in out else None)):
            if rr is not None and rr["autotune"]:
                b = rr["autotune"]["best"]
                seeds.append((w.dim, rr["nnz"] / w.n, b["tile"], b["lanes"], prec))
        out["law"] = law_runs(torch, pd, 200, seeds)
    if not args.no_serve:
        from paper_1806_06917_amd import inputs
        budget = int(args.serve_budget_gib * (1 << 30))
        per = {}
        for prec in ("mixed", "fp64"):
            burst = serve(pd, inputs.serving_requests(args.serve_count), budget,
                          args.serve_chunk, precision=prec)
            rate = args.serve_load * burst["requests_per_s"]
            poisson = serve(pd, inputs.serving_requests(args.serve_count, rate=rate), budget,
                            args.serve_chunk, rate, precision=prec)
            per[prec] = {"burst": burst,
                         "poisson": dict(poisson, rate_per_s=rate, load=args.serve_load),
                         "p50_s": poisson["p50_s"], "p99_s": poisson["p99_s"],
                         "bond_evals_per_s": poisson["bond_evals_per_s"]}
        out["serving"] = dict(
            per["mixed"],
            workload=f"{args.serve_count} notched plates, side U{{64..512}}, delta in "
                     "{3h,4h}, s_c ~ U[5e-4,2e-3], 1k-5k steps, lanes 4; the top-level "
                     "figures are the mixed-precision service, `fp64` the same requests "
                     "served in FP64",
            budget_bytes=budget, chunk_steps=args.serve_chunk, fp64=per["fp64"])
    if not args.no_law and not args.no_validation:
        runs = []
        for law, ic in (("linear", 1), ("np", 2)):
            progress("convergence study", law, "IC", ic)
            r = convergence(torch, pd, law, ic, args.convergence_t)
            runs.append({"law": law, "ic": ic, "seconds": r["seconds"], "steps": r["steps"],
                         "alpha": [round(x["alpha"], 3) for x in r["rates"]],
                         "t": [x["t"] for x in r["rates"]]})
        runs1 = []
        for pv in (False, True):
            progress("1-d convergence study, linear, IC 1", "partial volumes" if pv else "")
            r = convergence_1d(torch, pd, "linear", 1, args.convergence_t, pv=pv)
            runs1.append({"law": "linear", "ic": 1, "partial_volumes": pv,
                          "seconds": r["seconds"], "steps": r["steps"],
                          "alpha_set1": [round(x["alpha_set1"], 3) for x in r["rates"]],
                          "alpha_set2": [round(x["alpha_set2"], 3) for x in r["rates"]],
                          "t": [x["t"] for x in r["rates"]]})
        out["validation"] = {"study": "2-d convergence, h = delta/2, delta/4, delta/8",
                             "runs": runs,
                             "study_1d": "1-d convergence, h = delta/2 ... delta/16, sets "
                                         "{h1,h2,h3} and {h2,h3,h4}",
                             "runs_1d": runs1}
    if not args.no_cpu_baseline:
        steps = args.cpu_steps or (180 if w.n > 100000 else 600)
        out["cpu_baseline"] = cpu_baseline(w, steps, max(1, steps // 18))
        if not args.no_configs:
            out["cpu_baseline"]["configs"] = cpu_config_baselines(out.get("configs"),
                                                                  out.get("implicit"))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
