"""Benchmark: DoFs/s per semi-implicit time step of the SIPDG monodomain
solver (ionic update + load vector + PCG with one agglomerated-multigrid
V-cycle per iteration, to relative residual 1e-8) on one MI355X.

Workload: [0,1]^2, 256x256 quadrilaterals with seeded +-0.2h nodal jitter,
DG Q2 (589,824 DoFs), Aliev-Panfilov ionic model, three agglomerated levels
(4x4 grouping twice), dt = 1e-2.  The headline value is the mixed-precision
solver (FP32 V-cycle, FP64 outer PCG); the FP64 solver is reported beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
Prints one JSON line.
"""
import argparse
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DoFs/s per time step (PCG+V-cycle to 1e-8), mixed vs FP64; iters; HBM GB/s"
WORKLOADS = {
    "c2": "256x256 jittered Q2 SIPDG monodomain, Aliev-Panfilov, "
          "3-level agglomerated V-cycle PCG to rel. residual 1e-8",
    "c3": "64^3 Q2 SIPDG monodomain cube, rotating fibres, Bueno-Orovio, "
          "4-level agglomerated V-cycle PCG to rel. residual 1e-8",
    "c4": "1.0M-hex jittered ellipsoidal shell, Q1, transmural fibres, Bueno-Orovio, "
          "5-level STR R-tree agglomerated V-cycle PCG to rel. residual 1e-8, apex stimulus",
    "c4x8": "1.0M-hex jittered ellipsoidal shell, Q1, transmural fibres, Bueno-Orovio, "
            "5-level STR R-tree agglomerated V-cycle, 8 simulations (8 stimulus sites) "
            "solved together by 8-column PCG to rel. residual 1e-8 per column",
    "c5": "gradient of a 64-sensor misfit over 50 steps of the 256x256 Q2 Aliev-Panfilov "
          "problem w.r.t. 65,536 cell conductivity scalings: forward, checkpointed replay "
          "and discrete adjoint (FP64, PCG to rel. residual 1e-13)",
}
MFMA_F32_PEAK_TFLOPS = 157.3
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _stats(v):
    import numpy as np
    a = np.asarray(v, dtype=float)
    return dict(mean=float(a.mean()), std=float(a.std()), min=int(a.min()), max=int(a.max()))


def cheb_step_bytes(info, prec_bytes, nrhs=1):
    """Algorithmic bytes of one fused Chebyshev step on level 0: every face
    block once (its nonzero part in the sparse-face form) and every cell block once (the axis layout: its upper
    triangle, the block being symmetric; matrix-free: the packed
    conductivity of every cell instead), the adjacency lists, and the
    vector streams of every column (gather d, x r/w, r r/w, new d) plus
    D^-1 once."""
    b = info["b"]
    n, nf = info["n_cells"][0], info["n_faces"][0]
    N = n * b
    if info.get("fine_layout") == "matrix_free":
        d = info["dim"]
        return n * (d * (d + 1) // 2) * prec_bytes + 2 * d * 4 * n + (6 * nrhs + 1) * prec_bytes * N
    blocks = (n * cell_block_values(info) + nf * face_block_values(info)) * prec_bytes
    adjacency = 4 * (n + 1) + 2 * 2 * 4 * nf
    vectors = (6 * nrhs + 1) * prec_bytes * N
    return blocks + adjacency + vectors


def cell_block_values(info):
    """Values a level-0 cell block needs: the upper triangle of the symmetric
    block on the axis layout (which stores b/2 + 1 cyclic planes of b, the
    entries at distance b/2 twice when b is even), the full b x b block on
    the tile layout."""
    b = info["b"]
    return b * (b + 1) // 2 if info.get("fine_layout") == "axis_ell" else b * b


def face_block_values(info):
    """Values a level-0 face block needs: b^2, or on a nodal fine level in
    the sparse-face form the entries whose row or column node lies on the
    face (nF = b / q of each, q nodes per axis): 2 nF b - nF^2."""
    b, d = info["b"], info["dim"]
    if not info.get("sparse_faces"):
        return b * b
    q = round(b ** (1.0 / d))
    nf_ = b // q
    return 2 * nf_ * b - nf_ * nf_


def level0_working_set(info, prec_bytes, nrhs=1):
    """Bytes of the level-0 data the V-cycle's smoother touches: the stored
    operator (or the matrix-free coefficients) and adjacency, the inverse
    diagonal and the level's six work vectors (right-hand side, two x, r,
    two d).  The same count as one step's algorithmic bytes, whose seven
    vector streams are these seven vectors."""
    b = info["b"]
    n, nf = info["n_cells"][0], info["n_faces"][0]
    N = n * b
    if info.get("fine_layout") == "matrix_free":
        d = info["dim"]
        ops = n * (d * (d + 1) // 2) * prec_bytes + 2 * d * 4 * n
    else:
        ops = (n * cell_block_values(info) + nf * face_block_values(info)) * prec_bytes + 4 * (n + 1) + 2 * 2 * 4 * nf
    return ops + (6 * nrhs + 1) * prec_bytes * N


INFINITY_CACHE_BYTES = 256 * 1024 * 1024


def host_description():
    """Logical CPUs available to this process, physical cores and model name
    of the host (from the scheduler affinity and /proc/cpuinfo)."""
    desc = {"nproc": len(os.sched_getaffinity(0))}
    try:
        txt = open("/proc/cpuinfo").read()
    except OSError:
        return desc
    cores, model = set(), None
    phys = core = None
    for line in txt.splitlines():
        if ":" not in line:
            continue
        k, v = [x.strip() for x in line.split(":", 1)]
        if k == "model name" and model is None:
            model = v
        elif k == "physical id":
            phys = v
        elif k == "core id":
            core = v
            cores.add((phys, core))
    desc["physical_cores"] = len(cores) if cores else None
    desc["model"] = model
    return desc


def cheb_step_flops(info, nrhs):
    """Multiply-adds of the block products of one Chebyshev step, as flops:
    each stored block is used twice for a face (both orientations)."""
    b = info["b"]
    n, nf = info["n_cells"][0], info["n_faces"][0]
    return 2.0 * (n + 2 * nf) * b * b * nrhs


COUNTER_FILES = {
    "c2": "k_cheb_step_f32_b9_c2_counters.md",
    "c3": "k_cheb_step_mf_f32_b27_c3_counters.md",
    "c4": "k_cheb_step_f32_b8_c4_counters.md",
    "c4x8": "k_cheb_step_mfma8_c4x8_counters.md",
}


def kernel_source_sha():
    """sha256 over the device kernel sources (the counters are only valid for
    the kernels they were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hpp", "kernels_multi.hpp", "kernels_mf.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2602_16312_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def profiled_counters(workload):
    """Values of the committed counter summary of the dominant kernel
    (traffic_bytes_per_launch, flops_per_launch), or {} when there is none or
    the kernel sources changed since it was taken."""
    if workload not in COUNTER_FILES:
        return {}
    try:
        txt = open(os.path.join(ROOT, "profiles", COUNTER_FILES[workload])).read()
    except OSError:
        return {}
    vals = dict(l.split(": ", 1) for l in txt.splitlines() if ": " in l and not l.startswith(" "))
    if vals.get("kernel_source_sha256", "").strip() != kernel_source_sha():
        return {}
    return {k: float(vals[k]) for k in ("traffic_bytes_per_launch", "flops_per_launch") if k in vals}


def _iapp(pr, t, nrhs):
    """Nodal applied current at time t: one column, or one column per
    stimulus site (column-minor), or None when no stimulus is on."""
    import numpy as np
    from workloads.configs import iapp_nodal
    if nrhs == 1:
        a = iapp_nodal(pr, t)
        return a if a.any() else None
    if t > pr["stim_tend"] + 1e-12:
        return None
    a = np.zeros((pr["N"], nrhs))
    for c in range(nrhs):
        a[np.repeat(pr["stim_masks"][c], pr["b"]), c] = pr["stim_amp"]
    return a.ravel()


def run_gpu(pr, precision, steps, warmup, tol, profile_kind=None, nrhs=1, mfma=False,
            fine_layout="auto", setup="device", jacobi="point", step_log=None, workload=None):
    import numpy as np
    import torch
    from paper_2602_16312_amd import api, problem

    t0 = time.perf_counter()
    # the solver's device memory comes from torch's caching allocator
    h, s = problem.build(pr, precision=precision, max_rhs=nrhs, mfma=mfma,
                         fine_layout=fine_layout, setup=setup, allocator="torch", jacobi=jacobi)
    setup_s = time.perf_counter() - t0
    log(f"{precision}: setup {setup_s:.1f} s")
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    N, S = pr["N"], pr["S"]
    U0 = np.repeat(pr["U0"][:, None], nrhs, axis=1).ravel()
    W0 = np.repeat(pr["W0"].reshape(S, N)[:, :, None], nrhs, axis=2).ravel()
    st = api.State(dev(U0), dev(U0), dev(W0), dev(W0),
                   torch.empty(N * nrhs, dtype=torch.float64, device="cuda"))
    step = api.time_step if nrhs == 1 else api.time_step_multi
    # applied current per step, uploaded before the timed region (identical
    # vectors share one device copy)
    ia, cache = {}, {}
    for k in range(1, warmup + 2 * steps + 1):
        a = _iapp(pr, k * pr["dt"], nrhs)
        key = None if a is None else hash(a.tobytes())
        if key not in cache:
            cache[key] = None if a is None else dev(a)
        ia[k] = cache[key]
    k = 0
    for _ in range(warmup):
        k += 1
        step(s, st, k * pr["dt"], iapp=ia[k], tol=tol)
    torch.cuda.synchronize()
    its = []
    t0 = time.perf_counter()
    for _ in range(steps):
        k += 1
        r = step(s, st, k * pr["dt"], iapp=ia[k], tol=tol)
        its.append(r["its"] if nrhs == 1 else max(c["its"] for c in r))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    U = st.U.cpu().numpy()
    log(f"{precision}: {steps} steps in {wall:.3f} s, its {its[:10]}...")
    prof = None
    if profile_kind:
        # the dominant kernel: HIP events around each of its launches during
        # a further `steps` time steps (same stream), and around back-to-back
        # launches on the same level data
        api.profile_begin(s, profile_kind, 0)
        for _ in range(steps):
            k += 1
            step(s, st, k * pr["dt"], iapp=ia[k], tol=tol)
        n, ms = api.profile_end(s)
        b2b = api.kernel_bench(s, profile_kind, 0, 200, nrhs=nrhs)
        prof = dict(launches=n, in_run_ms=ms / max(1, n), back_to_back_ms=b2b)
    if step_log is not None:
        write_step_log(step_log, workload, precision, s, st, step, pr, k, steps, tol, nrhs, setup_s, dev)
    return dict(wall=wall, its=its, setup_s=setup_s, info=s.info(), prof=prof, U=U)


def write_step_log(f, workload, precision, s, st, step, pr, k, steps, tol, nrhs, setup_s, dev):
    """One JSON line for the set-up (phase buckets, operator complexity,
    level sizes) and one per time step of a further `steps` steps after the
    timed and profiled ones (iterations, initial and final residual norms,
    wall time, the ionic / load-vector / PCG phase times from HIP events on
    the solver's stream, DoFs/s).  The logged steps synchronise after every
    step and carry the phase events, so they are not the timed ones."""
    import torch
    from paper_2602_16312_amd import api
    info = s.info()
    f.write(json.dumps({"record": "setup", "workload": workload, "precision": precision,
                        "setup_s": round(setup_s, 4),
                        "phases_s": {a: round(b, 4) for a, b in info["t_setup"].items()},
                        "op_complexity": info["op_complexity"], "cells_per_level": info["n_cells"],
                        "n_dofs": int(pr["N"]), "rhs": nrhs}) + "\n")
    api.set_phase_timing(s, True)
    try:
        for _ in range(steps):
            k += 1
            a = _iapp(pr, k * pr["dt"], nrhs)
            ia = None if a is None else dev(a)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = step(s, st, k * pr["dt"], iapp=ia, tol=tol)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            cols = [r] if nrhs == 1 else r
            rec = {"record": "step", "workload": workload, "precision": precision, "step": k,
                   "t": k * pr["dt"], "its": [c["its"] for c in cols], "r0": [c["r0"] for c in cols],
                   "r_final": [c["rfin"] for c in cols], "converged": all(c["converged"] for c in cols),
                   "ms": round(ms, 4), "dofs_per_s": pr["N"] * nrhs / (ms / 1e3)}
            if nrhs == 1:
                rec["phase_ms"] = {a: round(b, 4) for a, b in api.step_phase_ms(s).items()}
            f.write(json.dumps(rec) + "\n")
    finally:
        api.set_phase_timing(s, False)
    f.flush()


def run_adjoint(args):
    """Times forward + backward of the sensor-misfit gradient (set-up included)
    and compares loss and gradient with the stored FP64 oracle values."""
    import numpy as np
    import torch
    from paper_2602_16312_amd.adjoint import sensor_misfit_loss
    from workloads import make_problem
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "c5_adjoint.json")))
    pr = make_problem("c5")
    steps, tol = g["steps"], g["tol"]
    targets = torch.tensor(np.array(g["targets"]), dtype=torch.float64, device="cuda")
    runs = []
    for k in range(args.warmup + args.steps):
        s = torch.ones(pr["n_cells"], dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss = sensor_misfit_loss(s, pr, targets, steps, tol=tol, checkpoint=10)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k >= args.warmup:
            runs.append((t1 - t0, t2 - t1))
        log(f"adjoint run {k}: forward {t1 - t0:.3f} s, backward {t2 - t1:.3f} s")
    grad = s.grad.cpu().numpy()
    fwd = float(np.mean([r[0] for r in runs]))
    bwd = float(np.mean([r[1] for r in runs]))
    gn = g["grad_norm"]
    rng = np.random.default_rng(g["dir_seed"])
    dir_err = 0.0
    for k in range(len(g["grad_dot_dirs"])):
        d = rng.standard_normal(pr["n_cells"])
        d /= np.linalg.norm(d)
        dir_err = max(dir_err, abs(float(grad @ d) - g["grad_dot_dirs"][k]) / gn)
    cells = np.array(g["sample_cells"])
    out = {
        "metric": METRIC, "value": pr["N"] * steps / (fwd + bwd), "unit": "DoFs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": (fwd + bwd) / steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"], "n_dofs": int(pr["N"]), "time_steps": steps,
                   "checkpoint_every": 10, "tol": tol,
                   "value_is": "DoFs x time steps / (forward + backward seconds), set-up included"},
        "forward_s": fwd, "backward_s": bwd,
        "loss_rel_err_vs_oracle": abs(loss.item() - g["loss"]) / g["loss"],
        "grad_rel_err_vs_oracle": {
            "at_64_cells": float(np.abs(grad[cells] - np.array(g["grad_at_cells"])).max() / gn),
            "projections_16_dirs": dir_err,
            "norm": abs(float(np.linalg.norm(grad)) - gn) / gn},
        "roofline": None,
    }
    print(json.dumps(out))


def _its_stats(pr, precision, tol, tol_mode, **mg):
    """Runs pr's time steps through the library; PCG iteration statistics."""
    import numpy as np
    import torch
    from paper_2602_16312_amd import api, problem
    t0 = time.perf_counter()
    mg.setdefault("setup", "device")
    mg.setdefault("allocator", "torch")
    h, s = problem.build(pr, precision=precision, **mg)
    setup = time.perf_counter() - t0
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    st = api.State(dev(pr["U0"]), dev(pr["U0"]), dev(pr["W0"].ravel()), dev(pr["W0"].ravel()),
                   torch.empty(pr["N"], dtype=torch.float64, device="cuda"))
    on = _iapp(pr, pr["dt"], 1)
    on = None if on is None else dev(on)
    its = []
    t0 = time.perf_counter()
    for k in range(pr["steps"]):
        t = (k + 1) * pr["dt"]
        r = api.time_step(s, st, t, iapp=on if t <= pr["stim_tend"] + 1e-12 else None,
                          tol=tol, tol_mode=tol_mode)
        if not r["converged"]:
            raise RuntimeError(f"step {k} did not converge: {r}")
        its.append(r["its"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = s.info()
    return dict(its=_stats(its), its_per_step=its, levels=info["n_cells"], n_dofs=int(pr["N"]),
                setup_s=setup,
                ms_per_step=wall / pr["steps"] * 1e3, u_max=float(st.U.max()))


def run_sweep(kind, precision, fine_layout="auto", mesh="c4"):
    """Iteration-count sweeps in the shape of the paper's tables: "e1" the
    two-dimensional FitzHugh-Nagumo test for p = 1..4 (iterations per step
    over T = 0.4 s); "levels" (number of multigrid levels) and "dt" (time
    step) over 5 ms of simulated time on the full 1.0M-hex shell (mesh "c4",
    p = 1), the 64^3 Q2 cube (mesh "c3") or the 125k-hex shell (mesh
    "c4half", p = 1 and 2).  The coarsest level is solved with its dense
    inverse, so the level counts start where that fits."""
    from workloads import make_problem
    rows = []
    if kind == "e1":
        for p in (1, 2, 3, 4):
            pr = make_problem("e1", p=p)
            r = _its_stats(pr, precision, pr["tol"], pr["tol_mode"], fine_layout=fine_layout)
            r.update(p=p)
            rows.append(r)
            log(f"e1 p={p}: {r['its']}")
        desc = ("128x128 Q1-Q4 FitzHugh-Nagumo, shock on [0.4,0.6]^2, dt 1e-4 s, 4000 steps, "
                "PCG to absolute residual 1e-14, 3 grid-grouped levels (4x4)")
    elif kind in ("levels", "dt"):
        if mesh == "c3":
            # 2x2x2 grid grouping: 64^3 -> 32^3 -> ... ; L levels in all
            cases = ([(2, L, 0.05) for L in (4, 5, 6)] if kind == "levels" else
                     [(2, 4, dt) for dt in (0.5, 0.1, 0.05)])
            mk = lambda p, L, dt: make_problem("c3", p=p, group=[2] * (L - 1), dt=dt,
                                               steps=int(round(5.0 / dt)))
            desc = ("64^3 Q2 cube (7.08M DoFs), rotating fibres, Bueno-Orovio, corner stimulus, "
                    "2x2x2 grid levels, 5 ms of simulated time, PCG to relative residual 1e-8")
        elif mesh == "c4":
            cases = ([(1, L, 0.05) for L in (4, 5, 6)] if kind == "levels" else
                     [(1, 5, dt) for dt in (0.5, 0.1, 0.05)])
            mk = lambda p, L, dt: make_problem("c4", p=p, agglo=("rtree_str", 8, L), dt=dt,
                                               steps=int(round(5.0 / dt)))
            desc = ("1.0M-hex shell (h 0.0147, 8.0M DoFs), Bueno-Orovio, apex stimulus, STR levels, "
                    "5 ms of simulated time, PCG to relative residual 1e-8")
        else:
            cases = ([(1, 3, 0.05), (1, 4, 0.05), (1, 5, 0.05), (2, 4, 0.05), (2, 5, 0.05)]
                     if kind == "levels" else
                     [(p, 5, dt) for p in (1, 2) for dt in (0.5, 0.1, 0.05)])
            mk = lambda p, L, dt: make_problem("c4", h=0.0294, p=p, agglo=("rtree_str", 8, L), dt=dt,
                                               steps=int(round(5.0 / dt)))
            desc = ("125k-hex shell (h 0.0294), Bueno-Orovio, apex stimulus, STR levels, 5 ms of "
                    "simulated time, PCG to relative residual 1e-8")
        for p, L, dt in cases:
            pr = mk(p, L, dt)
            r = _its_stats(pr, precision, 1e-8, "rel_r0", fine_layout=fine_layout)
            r.update(p=p, n_levels=L, dt=dt)
            rows.append(r)
            log(f"{kind} {mesh} p={p} L={L} dt={dt}: {r['its']}")
    else:
        raise SystemExit(f"unknown sweep {kind}")
    print(json.dumps({"sweep": kind, "mesh": mesh, "precision": precision,
                      "fine_layout": fine_layout, "workload": desc, "rows": rows}))


def cpu_baseline(pr, tol, nsteps):
    """The oracle timed on the host cores over the first `nsteps` steps;
    also returns its solution after those steps."""
    from oracle.stepper import Simulation
    from workloads.configs import iapp_nodal
    log("cpu baseline: oracle setup")
    sim = Simulation(pr)
    log("cpu baseline: timing steps")
    r0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    state, _, stats = sim.run(nsteps, tol, iapp_fn=lambda t: iapp_nodal(pr, t), record=False)
    wall = time.perf_counter() - t0
    r1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (r1.ru_utime - r0.ru_utime) + (r1.ru_stime - r0.ru_stime)
    # cores: the threads the oracle kept busy on average (process CPU time
    # over wall time; scipy's sparse products run on one thread, numpy's
    # dense kernels on the BLAS pool)
    return dict(value=pr["N"] / (wall / nsteps), unit="DoFs/s", cores=max(1, round(cpu / wall)),
                kind="oracle", cpu_seconds=round(cpu, 3), wall_seconds=round(wall, 3),
                host=host_description(),
                sample=f"first {nsteps} time steps of the same workload (scipy CSR PCG + "
                       f"V-cycle, FP64, tol {tol}); oracle setup excluded; "
                       f"its={[s['its'] for s in stats]}"), state[0]


def measure(workload, pr, args, steps, warmup, nrhs):
    """Mixed-precision time stepping of one workload (throughput, iteration
    statistics, roofline of the level-0 Chebyshev step from HIP events on the
    solver's stream) and, unless disabled, the FP64 solver beside it."""
    import numpy as np
    mfma = nrhs > 1 and not args.no_mfma
    res = run_gpu(pr, "mixed", steps, warmup, args.tol, profile_kind="cheb_step",
                  step_log=args.step_log_file, workload=workload,
                  nrhs=nrhs, mfma=mfma, fine_layout=args.fine_layout, setup=args.setup,
                  jacobi=args.jacobi)
    info = res["info"]
    prof = res["prof"]
    # the committed counter summaries profile the default configuration
    # (point Jacobi, automatic fine layout, the MFMA step for 8 columns)
    default_cfg = args.jacobi == "point" and args.fine_layout == "auto" and not args.no_mfma
    counters = profiled_counters(workload) if default_cfg else {}
    in_run_s = prof["in_run_ms"] / 1e3
    b2b_s = prof["back_to_back_ms"] / 1e3
    alg = cheb_step_bytes(info, 4, nrhs)
    ws = level0_working_set(info, 4, nrhs)
    b_ = info["b"]
    achieved = alg / in_run_s / 1e9
    if nrhs == 1:
        kname = f"k_cheb_step<float,{b_},{info['fine_layout']}{', sparse faces' if info.get('sparse_faces') else ''}> (level 0)"
    elif mfma:
        kname = f"k_cheb_step_mfma8<{info['fine_layout']}> (level 0, 8 columns, v_mfma_f32_4x4x1f32)"
    else:
        kname = f"k_cheb_step_m<float,{b_},8,{info['fine_layout']}> (level 0, 8 columns)"
    m = {
        "value": pr["N"] * nrhs / (res["wall"] / steps),
        "ms_per_step": res["wall"] / steps * 1e3,
        "config": {"workload": WORKLOADS[workload],
                   "n_dofs": int(pr["N"]), "rhs": nrhs, "cells_per_level": info["n_cells"],
                   "precision": "mixed: FP32 V-cycle (coarse inverse computed in FP64, stored in FP32), FP64 PCG",
                   "smoother": f"Chebyshev degree 3, 3 sweeps, {args.jacobi.replace('_', '-')} Jacobi",
                   "dt": pr["dt"], "tol": args.tol},
        "iters": _stats(res["its"]),
        "setup_s": res["setup_s"],
        "setup": {"where": args.setup,
                  "phases_s": {k: round(v, 4) for k, v in info["t_setup"].items()}},
        # achieved / frac: algorithmic bytes over the kernel's mean duration
        # across its launches in time steps (HIP events on the solver's
        # stream); the back-to-back figure repeats one launch on the same data
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counters.get("traffic_bytes_per_launch"),
                     "kernel": kname,
                     "alg_bytes_per_launch": alg, "avg_launch_us": in_run_s * 1e6,
                     "launches": prof["launches"],
                     "avg_launch_us_back_to_back": b2b_s * 1e6,
                     "frac_back_to_back": alg / b2b_s / 1e9 / HBM_PEAK_GBS,
                     "working_set_bytes": ws,
                     "residency": ("infinity_cache" if ws < INFINITY_CACHE_BYTES else "hbm")},
    }
    if m["roofline"]["residency"] == "infinity_cache":
        m["roofline"]["note"] = ("the level-0 working set fits the 256 MB Infinity Cache: "
                                 "the HBM peak is a reference, not the bound")
    if info["fine_layout"] == "matrix_free":
        # the sum-factorised kernel trades bytes for arithmetic: the binding
        # roofline is the one whose peak takes longer for the launch's work,
        # its FP32 vector work (counted by rocprofv3) at the FP32 vector peak
        # or its algorithmic bytes at the HBM peak; the other stays alongside
        fl = counters.get("flops_per_launch")
        if fl is not None:
            tf = fl / in_run_s / 1e12
            alu = {"achieved": tf, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                   "frac": tf / FP32_VECTOR_PEAK_TFLOPS, "flops_per_launch": fl}
            if fl / (FP32_VECTOR_PEAK_TFLOPS * 1e12) > alg / (HBM_PEAK_GBS * 1e9):
                hbm = {k: m["roofline"][k] for k in ("achieved", "peak", "unit", "frac")}
                m["roofline"].update(dict(alu, bound="alu", hbm=hbm))
            else:
                m["roofline"]["alu"] = alu
    if nrhs > 1:
        fl = cheb_step_flops(info, nrhs) / in_run_s / 1e12
        m["roofline"]["mfma" if mfma else "valu"] = {
            "achieved_tflops": fl, "peak_tflops": MFMA_F32_PEAK_TFLOPS,
            "utilisation": fl / MFMA_F32_PEAK_TFLOPS}
    if not args.no_fp64:
        r64 = run_gpu(pr, "fp64", steps, warmup, args.tol, nrhs=nrhs,
                      fine_layout=args.fine_layout, setup=args.setup, jacobi=args.jacobi,
                      step_log=args.step_log_file, workload=workload)
        m["fp64"] = {"value": pr["N"] * nrhs / (r64["wall"] / steps),
                     "ms_per_step": r64["wall"] / steps * 1e3,
                     "iters": _stats(r64["its"])}
        m["mixed_vs_fp64_rel_diff"] = float(np.abs(res["U"] - r64["U"]).max()
                                            / np.abs(r64["U"]).max())
    return res, m


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--step-log", default=None, metavar="PATH",
                    help="write JSON lines to PATH: one per solver set-up (phase buckets, operator "
                         "complexity), one per time step of a further --steps logged steps after the "
                         "timed ones (iterations, r0, r_final, phase times, DoFs/s), one for the run")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-c4", action="store_true",
                    help="default line without the 1.0M-hex shell sub-record")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline", action="store_true",
                    help="time the oracle on the 3D workloads too (its set-up alone takes minutes "
                         "there; the default line, c2, always carries it)")
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--workload", default="c2", choices=list(WORKLOADS),
                    help="c2: 256x256 Q2 (default bench line); c3: 64^3 Q2 cube; "
                         "c4: 1.0M-hex Q1 shell; c4x8: the shell with 8 simulations")
    ap.add_argument("--fine-layout", default="auto",
                    choices=["auto", "tile_ell", "axis_ell", "matrix_free"],
                    help="device storage of the fine operator (auto: each face block once; "
                         "matrix_free: sum factorisation, meshes of identical boxes only)")
    ap.add_argument("--jacobi", default="point", choices=["point", "cell_block"],
                    help="Jacobi matrix of the Chebyshev smoother: the diagonal (the paper's) or "
                         "the cells' inverted diagonal blocks")
    ap.add_argument("--setup", default="device", choices=["host", "device"],
                    help="where the prolongations, Galerkin products and Lanczos estimates "
                         "are computed (outside the timed region either way)")
    ap.add_argument("--sweep", choices=["e1", "levels", "dt"],
                    help="print PCG iteration statistics of a sweep instead of the bench line")
    ap.add_argument("--sweep-precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--sweep-mesh", default="c4", choices=["c4", "c3", "c4half"],
                    help="mesh of the levels/dt sweeps: the full shell, the 64^3 cube or the "
                         "125k-hex shell")
    ap.add_argument("--no-mfma", action="store_true",
                    help="c4x8: keep the 8-column Chebyshev step on the vector ALUs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    args.step_log_file = open(args.step_log, "w") if args.step_log else None

    import numpy as np
    import torch
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "launches": 5}))
        return

    if args.sweep:
        run_sweep(args.sweep, args.sweep_precision, args.fine_layout, args.sweep_mesh)
        return
    if args.workload == "c5":
        run_adjoint(args)
        return
    from workloads import make_problem
    nrhs = 8 if args.workload == "c4x8" else 1
    pr = make_problem("c4" if args.workload == "c4x8" else args.workload)
    out = {
        "metric": METRIC, "value": None, "unit": "DoFs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
    }
    res, m = measure(args.workload, pr, args, args.steps, args.warmup, nrhs)
    out["value"], out["ms_per_step"] = m.pop("value"), m.pop("ms_per_step")
    out.update(m)
    if args.workload == "c2" and not args.no_c4:
        # the same measurement on the 1.0M-hex shell (HBM-resident level 0),
        # single column, 20 time steps
        log("shell sub-record")
        pr4 = make_problem("c4")
        k4 = min(args.steps, 20)
        _, m4 = measure("c4", pr4, args, k4, min(args.warmup, 2), 1)
        m4["steps"], m4["warmup"] = k4, min(args.warmup, 2)
        out["c4"] = m4
        del pr4
    if not args.no_cpu_baseline and args.workload != "c2" and not args.cpu_baseline:
        out["cpu_baseline"] = {"skipped": "the oracle's set-up on this 3D workload takes minutes; "
                                          "pass --cpu-baseline to time it (the c2 line carries it)"}
    elif not args.no_cpu_baseline:
        out["cpu_baseline"], U_oracle = cpu_baseline(pr, args.tol, args.cpu_steps)
        if nrhs == 1:
            # error of each GPU solver against the oracle over the same steps
            # (all stopped at the same relative residual)
            err = {"steps": args.cpu_steps, "tol": args.tol}
            for prec in ("mixed",) + (() if args.no_fp64 else ("fp64",)):
                rg = run_gpu(pr, prec, args.cpu_steps, 0, args.tol, fine_layout=args.fine_layout,
                             setup=args.setup, jacobi=args.jacobi)
                err[prec] = float(np.linalg.norm(rg["U"] - U_oracle) / np.linalg.norm(U_oracle))
            out["rel_err_vs_oracle"] = err
    print(json.dumps(out))
    if args.step_log_file:
        args.step_log_file.write(json.dumps({"record": "run", **out}) + "\n")
        args.step_log_file.close()


if __name__ == "__main__":
    main()
