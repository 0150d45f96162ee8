"""Benchmark of the JFNK hot path on one MI355X.

Workload: 3D linear-elastic manufactured trigonometric solution on the unit
cube, 64^3 hexahedra with interior vertices perturbed by up to +-20 % of the
spacing (seed 0), 4th order (p = 3, cubic least squares, |S| = 85, 2x2 Gauss
points per face), alpha = 0.1, FP64 residual and J.v, FP32 preconditioner
sweeps.  One step = one J.v = (R(u + eps v) - R(u)) / eps with eps from device
norms, at u = the manufactured field and v = standard normal (seed 1000).
Reported: J.v Mcells/s (the headline value), residual Mcells/s, the roofline
of the dominant kernel from per-kernel HIP events recorded on the launch
stream over the timed region, the time of a Newton solve to 1e-8 with the plain
compact preconditioner (sweeps), its V-cycle application and the learned
correction, and the CPU oracle timed on a bounded sample (one thread and all
cores) with its time to tolerance on the 2D 32x32 problem.  A second leg runs
the 128^3 p = 3 cube on an unseen seed: J.v throughput and kernel HBM fractions,
the GPU's error against the oracle on sampled cells, and Newton to 1e-8 with
the plain sweeps and with the learned correction of the committed model
(trained on 2D squares and neo-Hookean beams).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per k_face_le launch on this workload from two rocprofv3 --pmc
# passes (FETCH_SIZE x 2.0 and WRITE_SIZE x 1.0, factors from a plain 512 MiB
# elementwise copy), valid only for the kernel and table-layout sources whose
# combined sha256 has this prefix.
MEASURED_TRAFFIC = {"kernel": "k_face_le", "n": 64, "p": 3, "bytes": 1934204633.0,
                    "kernels_sha256": "b021e324ca743f5b"}
TRAFFIC_SOURCES = ("kernels.hip", "common.h", "setup_blocks.cpp", "setup_tables.cpp")


def sources_sha():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2601_18417_amd", "csrc", name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, n, p):
    sha = sources_sha()
    t = MEASURED_TRAFFIC
    if t["kernel"] == kernel and t["n"] == n and t["p"] == p and t["kernels_sha256"] == sha:
        return t["bytes"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


_WORKER = {}


def _named_problem(spec):
    """The workloads the oracle is timed on: ("cube", n, p), the perturbed n^3
    cube of the benchmark; ("square", n, p), the 2D n^2 manufactured problem;
    ("cantilever", n, p), the 200x20x20 neo-Hookean cantilever."""
    import workloads as w
    name, n, p = spec
    if name == "cube":
        return w.cube_mms(n, p, perturb=0.2, seed=0)
    if name == "square":
        return w.square_mms(n, p)
    if name == "cantilever":
        return w.cantilever(p=p)
    raise ValueError(name)


def _oracle_state(prob):
    """The throughput state: the manufactured field, or the cantilever's bent
    state u_y = -0.3 x^2 / L; v standard normal (seed 1000)."""
    from oracle import geometry as geo
    m = prob.mesh
    _, cen = geo.cell_volume_centroid(m.verts[m.cells])
    if prob.loads.exact is not None:
        u = prob.loads.exact.value(cen)
    else:
        u = np.zeros((m.n_cells, prob.dim))
        u[:, 1] = -0.3 * cen[:, 0] ** 2 / m.lengths[0]
    v = np.random.default_rng(1000).standard_normal((prob.dim, m.n_cells)).T.copy()
    return u, v


def _oracle_worker_setup(args):
    """Worker process: build the oracle's discretisation for its block of cells."""
    prob_spec, cells, u, v = args
    from oracle import residual as ores
    from oracle import jacobian as ojac
    prob = _named_problem(prob_spec)
    disc = ores.build(prob, active=cells)
    Ru = ores.residual(disc, u)
    _WORKER.update(disc=disc, u=u, v=v, Ru=Ru, eps=ojac.default_eps(u, v))
    return len(cells)


def _oracle_worker_jvp(reps):
    from oracle import jacobian as ojac
    d = _WORKER
    for _ in range(reps):
        ojac.jvp(d["disc"], d["u"], d["v"], d["Ru"], d["eps"])
    return reps


def cpu_study(args):
    """The oracle's residual and J.v throughput on the host, one core and all
    cores (one process per core on its own block of cells), on bounded samples
    of each workload: the 2D 32^2 p = 2 square, the 64^3 p = 3 cube,
    the 200x20x20 p = 2 cantilever and the 128^3 cube at p = 1 and 2 (1000
    contiguous cells each; the oracle's setup for them is not timed)."""
    import multiprocessing as mp
    from oracle import jacobian as ojac
    from oracle import residual as ores
    named = {"square32p2": ("square", 32, 2), "cube64p3": ("cube", 64, 3), "cantilever": ("cantilever", 0, 2),
             "cube128p1": ("cube", 128, 1), "cube128p2": ("cube", 128, 2)}
    specs = [named[k] for k in args.cpu_workloads.split(",")]
    nw = min(16, os.cpu_count() or 1)
    rows = []
    for spec in specs:
        log(f"cpu study: {spec} setup")
        t0 = time.perf_counter()
        prob = _named_problem(spec)
        n = prob.mesh.n_cells
        u, v = _oracle_state(prob)
        ns = min(1000, n)
        rng = np.random.default_rng(0)
        start = int(rng.integers(0, n - ns)) if n > ns else 0
        cells = np.arange(start, start + ns)
        disc = ores.build(prob, active=cells)
        t_setup = time.perf_counter() - t0
        eps = ojac.default_eps(u, v)
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < 5.0:
            Ru = ores.residual(disc, u)
            reps += 1
        t_res = (time.perf_counter() - t0) / reps
        reps, t0 = 0, time.perf_counter()
        while reps < 3 or time.perf_counter() - t0 < 5.0:
            ojac.jvp(disc, u, v, Ru, eps)
            reps += 1
        t_jvp = (time.perf_counter() - t0) / reps
        row = {"workload": f"{spec[0]} n={spec[1] or '200x20x20'} p={spec[2]}", "n_cells": n, "sample_cells": ns,
               "setup_seconds": t_setup, "residual_mcells_s_1core": ns / t_res / 1e6,
               "jvp_mcells_s_1core": ns / t_jvp / 1e6}
        if n > 1_000_000:
            # every worker would rebuild the whole mesh's face geometry (6.2 M faces
            # at 128^3) for its block: one core only
            row["jvp_mcells_s_all_cores"] = None
        elif n >= nw * ns:
            blocks = [np.arange(b0, b0 + ns) for b0 in np.linspace(0, n - ns, nw).astype(np.int64)]
            log(f"cpu study: {spec} one core done, {nw} worker setups")
            with mp.get_context("spawn").Pool(nw) as pool:
                for k, _ in enumerate(pool.imap_unordered(_oracle_worker_setup,
                                                          [(spec, blk, u, v) for blk in blocks], chunksize=1)):
                    log(f"cpu study: worker setup {k + 1}/{nw}")
                t0 = time.perf_counter()
                pool.map(_oracle_worker_jvp, [reps] * nw, chunksize=1)
                t_all = time.perf_counter() - t0
            row["jvp_mcells_s_all_cores"] = nw * ns * reps / t_all / 1e6
            row["cores"] = nw
        log(json.dumps(row))
        rows.append(row)
    print(json.dumps({"study": "cpu", "kind": "oracle", "host_cores": os.cpu_count(), "rows": rows}), flush=True)


def cpu_baseline(prob, n_sample: int, u, v, ctx, torch, label, seed: int = 0, cube=None):
    """The FP64 oracle's J.v on n_sample cells of the same mesh at the bench's
    state (setup excluded), on one thread and on all host cores (one worker
    process per core, each on its own contiguous block of cells); the error of
    the GPU's R and J.v against it on those cells (same u, v and eps); and the
    oracle's time to 1e-10 on the 2D 32x32 p = 2 manufactured problem."""
    from oracle import jacobian as ojac
    from oracle import newton as onw
    from oracle import residual as ores
    import workloads as w
    rng = np.random.default_rng(seed)
    n = prob.mesh.n_cells
    # a contiguous block of cells (lexicographic), which is what a CPU would sweep
    start = int(rng.integers(0, n - n_sample))
    cells = np.arange(start, start + n_sample)
    t0 = time.perf_counter()
    disc = ores.build(prob, active=cells)
    t_setup = time.perf_counter() - t0
    Ru = ores.residual(disc, u)
    eps = ojac.default_eps(u, v)
    reps = 0
    t0 = time.perf_counter()
    while reps < 3 or time.perf_counter() - t0 < 5.0:
        Jo = ojac.jvp(disc, u, v, Ru, eps)
        reps += 1
    t_jvp = (time.perf_counter() - t0) / reps
    ud = torch.tensor(u.T.copy(), device="cuda:0")
    vd = torch.tensor(v.T.copy(), device="cuda:0")
    Rg = torch.empty_like(ud)
    Jg = torch.empty_like(ud)
    ctx.residual(ud, Rg)
    ctx.jvp(ud, Rg, vd, Jg, eps=eps)
    Rg = Rg.cpu().numpy().T[cells]
    Jg = Jg.cpu().numpy().T[cells]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))

    out = {"value": n_sample / t_jvp / 1e6, "unit": "Mcells/s", "cores": 1, "kind": "oracle",
           "sample": f"J.v at {n_sample} contiguous cells of the same {label} mesh, {reps} repetitions "
                     f"(numpy fp64, one thread; its setup for those cells, {t_setup:.1f}s, not timed)",
           "seconds_per_jvp": t_jvp,
           "gpu_error_vs_oracle": {"residual_rel_l2": rel(Rg, Ru[cells]), "jvp_rel_l2": rel(Jg, Jo[cells]),
                                   "cells": n_sample}}
    try:
        import platform
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")),
                     platform.processor())
    except OSError:
        model = "unknown"
    out["cpu_model"] = model
    out["host_cores"] = os.cpu_count()
    if cube is not None:
        # all cores: one spawned process per core (none touches the GPU), each
        # with its own block of n_sample cells; the J.v phase is timed after
        # every worker has set up
        import multiprocessing as mp
        nw = min(16, os.cpu_count() or 1)
        blocks = [np.arange(b0, b0 + n_sample) for b0 in
                  np.linspace(0, n - n_sample, nw).astype(np.int64)]
        with mp.get_context("spawn").Pool(nw) as pool:
            pool.map(_oracle_worker_setup, [(cube, blk, u, v) for blk in blocks], chunksize=1)
            t0 = time.perf_counter()
            pool.map(_oracle_worker_jvp, [reps] * nw, chunksize=1)
            t_all = time.perf_counter() - t0
        out["all_cores"] = {"value": nw * n_sample * reps / t_all / 1e6, "unit": "Mcells/s", "cores": nw,
                            "sample": f"J.v, {nw} processes x {n_sample} contiguous cells x {reps} repetitions"}
    # time to tolerance of the whole oracle solve on the 2D 32x32 p = 2 problem
    sq = w.square_mms(32, 2)
    t0 = time.perf_counter()
    dsq = ores.build(sq)
    t_sq_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, st = onw.newton(dsq, np.zeros((dsq.n_cells, 2)), tol=1e-10, eta=1e-4)
    out["time_to_tol_square32_p2"] = {"seconds": time.perf_counter() - t0, "tol": 1e-10, "cores": 1,
                                      "newton_iters": st["newton"], "krylov_iters": st["krylov"],
                                      "setup_seconds": t_sq_setup}
    return out


MIXED_MODEL = os.path.join(ROOT, "paper_2601_18417_amd", "weights", "mixed_sweeps.hofvnn")
MIXED_TRAIN_CMD = ("python bench.py --study train --train-set mixed --mg-base 0 --train-seeds 0-49 --harvest-starts 2 "
                "--harvest-length 9 --restart 300 --learned-epochs 30 --model paper_2601_18417_amd/weights/"
                "mixed_sweeps.hofvnn")


def big_leg(args, torch, api, w, dev):
    """The 128^3 perturbed cube at p = 3 on an unseen seed: J.v and residual
    throughput with the face and extrapolation kernels' HBM fractions, the
    GPU's R and J.v against the oracle on sampled cells, and Newton to 1e-8
    with the plain sweeps and with the learned correction of the committed
    model (trained on 2D squares and neo-Hookean beams), each solution's
    oracle residual on the sampled cells."""
    from oracle import jacobian as ojac
    from oracle import residual as ores
    t0 = time.perf_counter()
    prob = w.cube_mms(args.big_n, 3, perturb=0.2, seed=args.big_seed)
    ctx = api.context_for(prob)
    t_setup = time.perf_counter() - t0
    log(f"128^3 setup {t_setup:.1f}s")
    nc = prob.mesh.n_cells
    cen = ctx.cell_centroids()
    u = torch.tensor(prob.loads.exact.value(cen).T.copy(), device=dev)
    v = torch.tensor(np.random.default_rng(1000).standard_normal((3, nc)), device=dev)
    Ru = torch.empty_like(u)
    Jv = torch.empty_like(u)
    ctx.residual(u, Ru)
    for _ in range(3):
        ctx.jvp(u, Ru, v, Jv)
    steps = 10
    # the step with events around the face kernel only, then a breakdown with
    # every kernel timed
    ctx.set_timing(True, only="k_face_le")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.jvp(u, Ru, v, Jv)
    torch.cuda.synchronize()
    ms_jvp = (time.perf_counter() - t0) / steps * 1e3
    ctx.set_timing(True)
    for _ in range(steps):
        ctx.jvp(u, Ru, v, Jv)
    torch.cuda.synchronize()
    kern = {}
    for name in ("k_face_le", "k_extrap", "k_cell_sum", "k_pack", "k_sumsq2"):
        ms, cnt = ctx.kernel_time(name)
        if cnt:
            kern[name] = {"avg_ms": ms / cnt}
            if name in ("k_face_le", "k_extrap", "k_cell_sum"):  # the kernels with a byte model
                kern[name]["GBps"] = ctx.kernel_bytes(name) / (ms / cnt * 1e-3) / 1e9
                kern[name]["frac_of_hbm_peak"] = kern[name]["GBps"] / HBM_PEAK_GBS
    ctx.set_timing(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.residual(u, Ru)
    torch.cuda.synchronize()
    ms_res = (time.perf_counter() - t0) / steps * 1e3
    # the oracle on sampled cells: corners, boundary-face cells and random ones
    ijk = w.cell_ijk(prob.mesh)
    top = np.array(prob.mesh.shape) - 1
    rng = np.random.default_rng(77)
    sample = np.unique(np.concatenate([rng.choice(nc, 12, replace=False),
                                       np.nonzero(np.all((ijk == 0) | (ijk == top), axis=1))[0][:4],
                                       np.nonzero(ijk[:, 0] == 0)[0][:3], np.nonzero(ijk[:, 2] == top[2])[0][:3]]))
    t0 = time.perf_counter()
    disc = ores.build(prob, active=sample)
    uh = u.cpu().numpy().T
    vh = v.cpu().numpy().T
    eps = ojac.default_eps(uh, vh)
    ctx.residual(u, Ru)
    ctx.jvp(u, Ru, v, Jv, eps=eps)
    Rg, Jg = Ru.cpu().numpy().T[sample], Jv.cpu().numpy().T[sample]
    Ro = ores.residual(disc, uh)
    Jo = (ores.residual(disc, uh + eps * vh) - Ro) / eps
    Ff, Fd = ores.face_fluxes(disc, uh)
    scale = np.zeros_like(Ro)
    np.add.at(scale, disc.f_own, np.abs(Ff))
    np.add.at(scale, disc.f_nei, np.abs(Ff))
    np.add.at(scale, disc.d_own, np.abs(Fd))
    scale += np.abs(disc.b_body)
    err = {"cells": int(sample.size),
           "residual_max_over_flux_scale": float(np.max(np.abs(Rg - Ro[sample]) / scale[sample])),
           "jvp_rel_l2": float(np.linalg.norm(Jg - Jo[sample]) / np.linalg.norm(Jo[sample])),
           "oracle_seconds": time.perf_counter() - t0}
    R0o = ores.residual(disc, np.zeros_like(uh))[sample]
    out = {"workload": f"3D linear elastic MMS, unit cube {args.big_n}^3 hex perturbed +-20% (seed {args.big_seed}), "
                       f"p=3, |S|={ctx.report['stencil_size']}, 2x2 Gauss/face, alpha=0.1",
           "n_cells": nc, "setup_seconds": t_setup, "jvp_ms": ms_jvp, "jvp_mcells_s": nc / (ms_jvp * 1e-3) / 1e6,
           "residual_mcells_s": nc / (ms_res * 1e-3) / 1e6, "kernels": kern, "gpu_error_vs_oracle": err}
    log(f"128^3 J.v {out['jvp_mcells_s']:.0f} Mcells/s, kernels {kern}, oracle {err}")
    if not args.big_solve:
        ctx.close()
        return out
    # time to 1e-8 from u = 0: plain sweeps, then the learned correction
    res = {}
    model = api.Model(0)
    model.load(args.learned_model)
    ctx.attach(model)
    z = torch.empty_like(u)
    ctx.precond_apply(v, z, learned=True)  # the network's workspace
    for name, learned in (("plain", False), ("learned", True)):
        uu = torch.zeros_like(u)
        st = newton_run(torch, ctx, prob, nc, learned, 1e-8, args.max_krylov, u_out=uu)
        ug = uu.cpu().numpy().T
        st["oracle_rel_residual_sampled"] = float(np.linalg.norm(ores.residual(disc, ug)[sample]) /
                                                  np.linalg.norm(R0o))
        ue = prob.loads.exact.value(cen)
        st["rms_error_vs_manufactured"] = float(np.sqrt(np.mean(np.sum((ug - ue) ** 2, axis=1))))
        res[name] = st
        log(f"128^3 {name} solve {st}")
    res["speedup"] = res["plain"]["seconds"] / res["learned"]["seconds"]
    res["krylov_ratio"] = res["learned"]["krylov_iters"] / max(res["plain"]["krylov_iters"], 1)
    res["model"] = os.path.relpath(args.learned_model, ROOT)
    res["training_command"] = MIXED_TRAIN_CMD
    res["training"] = ("2,000 pairs: 2D 32x32 p=2 squares and 60x6x6 p=2 neo-Hookean beams, perturbation seeds 0-49; "
                       "evaluated on an unseen seed")
    ctx.attach(None)
    ctx.close()
    return out, res


def parse_seeds(s):
    out = []
    for part in s.split(","):
        a, _, b = part.partition("-")
        out += list(range(int(a), int(b) + 1)) if b else [int(a)]
    return out


KRYLOV = {"eta": 1e-4, "restart": 30, "line_search": 10, "forcing": 0, "predictor": 0, "side": 0, "gs_passes": 0,
          "graphs": 0}  # Newton's Krylov options (set from the arguments)


def forcing_term(rn, rprev, eta_prev, eta_max, tol, r0):
    """The library's Eisenstat-Walker rule (forcing = 1), applied here across
    one-step library calls."""
    e = 0.9 * (rn / rprev) ** 2
    if 0.9 * eta_prev ** 2 > 0.1:
        e = max(e, 0.9 * eta_prev ** 2)
    return max(min(e, eta_max), 0.5 * tol * r0 / rn)


def newton_stepwise(torch, ctx, uu, learned, tol, max_krylov, max_newton, label):
    """One library Newton step per call, each logged as it ends (long solves
    stay visible); stops at ||R|| <= tol ||R_0||."""
    R = torch.empty_like(uu)
    ctx.residual(uu, R)
    r0 = float(torch.linalg.norm(R))
    tot = {"newton_iters": 0, "krylov_iters": 0, "fallbacks": 0, "converged": False, "rel_residual": 1.0}
    t0 = time.perf_counter()
    eta, rn, rprev = KRYLOV["eta"], r0, r0
    for step in range(max_newton):
        if KRYLOV["forcing"] and step > 0:
            eta = forcing_term(rn, rprev, eta, KRYLOV["eta"], tol, r0)
        rprev = rn
        st = ctx.newton_solve(uu, tol=1e-300, eta=eta, max_newton=1, max_krylov=max_krylov, n_sweeps=2,
                              learned=learned, check=False, n_increments=0, restart=KRYLOV["restart"],
                              max_line_search=KRYLOV["line_search"], side=KRYLOV["side"],
                              gs_passes=KRYLOV["gs_passes"], graphs=KRYLOV["graphs"])
        for key in ("newton_iters", "krylov_iters", "fallbacks"):
            tot[key] += st[key]
        ctx.residual(uu, R)
        rn = float(torch.linalg.norm(R))
        tot["rel_residual"] = rn / r0
        log(f"{label} step {step}: {st['krylov_iters']} Krylov (eta {eta:.1e}), rel {tot['rel_residual']:.2e}, "
            f"{time.perf_counter() - t0:.1f}s")
        if tot["rel_residual"] <= tol:
            tot["converged"] = True
            break
    return tot


def newton_run(torch, ctx, prob, nc, learned, tol, max_krylov, u_out=None, stepwise=0):
    """Newton from u = 0 through the problem's load increments (each one a
    library Newton solve at its load factor, logged as it ends; with
    stepwise > 0, one logged call per Newton step, at most that many steps)."""
    uu = torch.zeros((prob.dim, nc), device="cuda:0", dtype=torch.float64) if u_out is None else u_out.zero_()
    ninc = max(1, prob.n_increments)
    out = {"newton_iters": 0, "krylov_iters": 0, "fallbacks": 0, "converged": True, "rel_residual": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if KRYLOV["predictor"] and ninc > 1:
        # the predictor spans increments: one library call for all of them
        st = ctx.newton_solve(uu, tol=tol, eta=KRYLOV["eta"], max_krylov=max_krylov, n_sweeps=2, learned=learned,
                              check=False, n_increments=ninc, restart=KRYLOV["restart"],
                              max_line_search=KRYLOV["line_search"], forcing=KRYLOV["forcing"], predictor=1, side=KRYLOV["side"],
                              gs_passes=KRYLOV["gs_passes"], graphs=KRYLOV["graphs"])
        torch.cuda.synchronize()
        out.update({key: st[key] for key in ("newton_iters", "krylov_iters", "fallbacks", "rel_residual")})
        out["converged"] = bool(st["converged"])
        out["seconds"] = time.perf_counter() - t0
        log(f"{'learned' if learned else 'plain'} {ninc} increments with the predictor: {out}")
        return out
    for inc in range(1, ninc + 1):
        ctx.set_load_scale(inc / ninc)
        if stepwise:
            st = newton_stepwise(torch, ctx, uu, learned, tol, max_krylov, stepwise,
                                 f"{'learned' if learned else 'plain'} increment {inc}")
        else:
            st = ctx.newton_solve(uu, tol=tol, eta=KRYLOV["eta"], max_krylov=max_krylov, n_sweeps=2,
                                  learned=learned, check=False, n_increments=0, restart=KRYLOV["restart"],
                                  max_line_search=KRYLOV["line_search"], forcing=KRYLOV["forcing"], side=KRYLOV["side"],
                              gs_passes=KRYLOV["gs_passes"], graphs=KRYLOV["graphs"])
        for key in ("newton_iters", "krylov_iters", "fallbacks"):
            out[key] += st[key]
        out["rel_residual"] = st["rel_residual"]
        if ninc > 1:
            log(f"{'learned' if learned else 'plain'} increment {inc}/{ninc}: {st['newton_iters']} Newton, "
                f"{st['krylov_iters']} Krylov, rel {st['rel_residual']:.2e}, {time.perf_counter() - t0:.1f}s")
        if not st["converged"]:
            out["converged"] = False
            break
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    return out


def column_steps(args, torch, ctx, prob, cen):
    """BDF2 time steps of the vibrating column from rest under the sudden end
    traction; the transverse displacement of the loaded end is sampled every
    10 steps."""
    nc = prob.mesh.n_cells
    rho, dt = prob.meta["rho"], prob.meta["dt"]
    ctx.set_dynamics(rho, dt)
    u = torch.zeros((3, nc), device="cuda:0", dtype=torch.float64)
    ctx.dyn_reset(u, u.clone())
    L = prob.mesh.lengths[0]
    end = np.nonzero(cen[:, 0] > L - L / prob.mesh.shape[0])[0]
    tol = args.tol if args.tol > 0 else 1e-8
    out = {"rho": rho, "dt": dt, "steps": args.time_steps, "newton_iters": 0, "krylov_iters": 0,
           "tol": tol, "end_displacement": []}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, args.time_steps + 1):
        st = ctx.dyn_step(u, tol=tol, eta=KRYLOV["eta"], restart=KRYLOV["restart"], max_krylov=args.max_krylov,
                          max_line_search=KRYLOV["line_search"], forcing=KRYLOV["forcing"], check=False)
        out["newton_iters"] += st["newton_iters"]
        out["krylov_iters"] += st["krylov_iters"]
        if not st["converged"]:
            out["failed_step"] = k
            break
        if k % 10 == 0:
            ue = u[1:, end].mean(dim=1).cpu().numpy()
            out["end_displacement"].append([k * dt, float(ue[0]), float(ue[1])])
            log(f"column step {k}: t = {k * dt:.3f} s, end (u_y, u_z) = ({ue[0]:.4f}, {ue[1]:.4f}) m, "
                f"{out['newton_iters']} Newton, {out['krylov_iters']} Krylov, {time.perf_counter() - t0:.1f}s")
    torch.cuda.synchronize()
    out["seconds"] = time.perf_counter() - t0
    out["ms_per_step"] = 1e3 * out["seconds"] / max(k, 1)
    ctx.set_dynamics(0.0, 0.0)
    return out


def study(args):
    """The learned-preconditioner study: 'train' harvests pairs on seeded
    meshes (--train-set) and trains a model (saved with hofv_nn_save); 'eval'
    times plain vs learned Newton solves to the tolerance on an unseen mesh;
    'nn' times the learned application alone."""
    import torch

    import workloads as w
    from paper_2601_18417_amd import api
    from paper_2601_18417_amd import learned as lrn
    dev = torch.device("cuda:0")
    if args.study == "nn":
        # the learned preconditioner's application alone (a seeded untrained
        # model runs every kernel of the forward pass), for kernel traces
        prob = w.cube_mms(args.n, args.p, perturb=0.2, seed=0)
        ctx = api.context_for(prob)
        model = api.Model(7)
        ctx.attach(model)
        nc = prob.mesh.n_cells
        r = torch.randn((3, nc), device=dev, dtype=torch.float64, generator=torch.Generator(device=dev).manual_seed(5))
        z = torch.empty_like(r)
        for _ in range(args.warmup):
            ctx.precond_apply(r, z, learned=True)
        ctx.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.precond_apply(r, z, learned=True)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        lay_ms, lay_n = ctx.kernel_time("k_nn_layer")
        ctx.set_timing(False)
        print(json.dumps({"study": "nn", "n_cells": nc, "learned_apply_ms": ms,
                          "k_nn_layer_avg_ms": lay_ms / max(lay_n, 1), "k_nn_layer_launches": lay_n}), flush=True)
        return
    if args.study == "train":
        t0 = time.perf_counter()
        data, keep = [], []
        kinds = {"mixed": ["square", "beam"], "cube": ["cube"], "cantilever": ["beam"]}[args.train_set]
        for seed in parse_seeds(args.train_seeds):
            for kind in kinds:
                if kind == "beam":
                    # a short beam with the cantilever's cells (0.05 cubes) and slenderness
                    # (10), perturbed by seed; the same tip traction bends it by the same
                    # fraction of its length (the sweeps alone do not solve it: V-cycle)
                    nx = args.learned_size if args.train_set == "cantilever" else 60
                    shape, lengths = (nx, nx // 10, nx // 10), (0.05 * nx, 0.005 * nx, 0.005 * nx)
                    tp = w.cantilever(shape=shape, p=2 if args.train_set == "mixed" else args.p)
                    tp.mesh = w.box_mesh(shape, lengths=lengths, perturb=0.1, seed=seed)
                    tp.loads = w.fields.cantilever_loads(lengths[0], (0.0, -2.18e-3, 0.0))
                    mg = True
                elif kind == "square":  # the 2D 32x32 p = 2 manufactured problem, perturbed by seed
                    tp = w.square_mms(32, 2, perturb=0.2, seed=seed)
                    mg = args.mg_base
                else:
                    tp = w.cube_mms(args.learned_size, args.p, perturb=0.2, seed=seed)
                    mg = args.mg_base
                tctx = api.context_for(tp, precond_levels=8 if mg else 1)
                if mg:
                    tctx.set_multigrid(True)
                if kind == "beam":
                    tctx.set_load_scale(0.3)
                u0 = torch.zeros((tp.dim, tp.mesh.n_cells), device=dev, dtype=torch.float64)
                data.append(lrn.harvest(tctx, u0, n_starts=args.harvest_starts, length=args.harvest_length,
                                        newton_steps=2, seed=seed, restart=args.restart))
                if mg and not args.mg_base:
                    # e came from V-cycle-preconditioned solves; the network learns to
                    # correct the sweeps' output
                    tctx.set_multigrid(False)
                keep.append(tctx)
                log(f"harvested {kind} seed {seed}: {len(data[-1])} pairs, {time.perf_counter() - t0:.0f}s")
        t_harvest = time.perf_counter() - t0
        model = api.Model(7)
        hist = lrn.train(model, data, epochs=args.learned_epochs, lr=2e-3, batch=4, seed=args.train_order_seed)
        for ep, l in enumerate(hist):
            log(f"epoch {ep} loss {l:.4f}")
        model.save(args.model)
        meshes = {"mixed": "2D 32x32 p=2 perturbed squares and 60x6x6 p=2 perturbed neo-Hookean beams (the beams' "
                        "e solved with the V-cycle), network inputs from the "
                        + ("V-cycle" if args.mg_base else "sweeps"),
                  "cube": f"{args.learned_size}^3 p={args.p} perturbed cubes" + (" (V-cycle inputs)" if args.mg_base
                                                                                    else ""),
                  "cantilever": f"{args.learned_size}x{args.learned_size // 10}x{args.learned_size // 10} "
                                f"p={args.p} perturbed neo-Hookean beams (V-cycle inputs)"}[args.train_set]
        out = {"study": "train", "pairs": int(sum(len(d) for d in data)),
               "meshes": meshes + f", seeds {args.train_seeds}",
               "epochs": args.learned_epochs, "harvest_seconds": t_harvest,
               "train_seconds": time.perf_counter() - t0 - t_harvest, "loss_first_epoch": hist[0],
               "loss_last_epoch": hist[-1], "model": args.model}
    else:
        model = api.Model(0)
        model.load(args.model)
        t0 = time.perf_counter()
        if args.workload == "cantilever":
            prob = w.cantilever(p=args.p)
            desc = f"neo-Hookean cantilever 200x20x20, p={args.p}, 10 increments"
        else:
            lz = args.lz
            prob = w.cube_mms(args.n, args.p, perturb=0.2, seed=args.seed, lengths=(1.0, 1.0, lz))
            desc = (f"LE MMS {args.n}^3 perturbed +-20% (seed {args.seed}) on [0,1]^2 x [0,{lz}] "
                    f"(cell aspect {1.0 / lz:g}), p={args.p}")
        log(f"mesh generated {time.perf_counter() - t0:.0f}s")
        nc = prob.mesh.n_cells
        t0 = time.perf_counter()
        ctx = api.context_for(prob, precond_levels=args.precond_levels,
                              progress=lambda s: log(f"  {s} {time.perf_counter() - t0:.0f}s"))
        t_setup = time.perf_counter() - t0
        multigrid = args.precond_levels >= 2
        if multigrid:
            try:
                ctx.set_multigrid(False)
            except api.HofvError:
                multigrid = False
        ctx.attach(model)
        tol = args.tol if args.tol > 0 else 1e-8
        r = torch.randn((prob.dim, nc), device=dev, dtype=torch.float64)
        z = torch.empty_like(r)
        ctx.precond_apply(r, z, learned=True)  # allocates the network's workspace
        solvers = set(args.solvers.split(","))
        out = {"study": "eval", "workload": desc, "n_cells": nc, "tol": tol, "setup_seconds": t_setup,
               "krylov": {"eta": args.eta, "forcing": args.forcing, "restart": args.restart,
                          "line_search": args.line_search}}
        if "plain" in solvers:
            out["plain"] = newton_run(torch, ctx, prob, nc, False, tol, args.max_krylov, stepwise=args.max_newton)
            log(f"plain {out['plain']}")
        if "learned" in solvers:
            out["learned"] = newton_run(torch, ctx, prob, nc, True, tol, args.max_krylov, stepwise=args.max_newton)
            log(f"learned {out['learned']}")
        if "plain" in out and "learned" in out:
            out["speedup"] = out["plain"]["seconds"] / out["learned"]["seconds"]
            out["krylov_ratio"] = out["learned"]["krylov_iters"] / max(out["plain"]["krylov_iters"], 1)
        if multigrid and "multigrid" in solvers:
            ctx.set_multigrid(True)
            out["multigrid"] = newton_run(torch, ctx, prob, nc, False, tol, args.max_krylov, stepwise=args.max_newton)
            log(f"multigrid {out['multigrid']}")
        if multigrid and "mglearned" in solvers:
            # the network's correction of the V-cycle's output
            ctx.set_multigrid(True)
            out["mglearned"] = newton_run(torch, ctx, prob, nc, True, tol, args.max_krylov, stepwise=args.max_newton)
            log(f"multigrid + learned {out['mglearned']}")
            if "multigrid" in out:
                out["mglearned_speedup"] = out["multigrid"]["seconds"] / out["mglearned"]["seconds"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cube",
                    choices=["cube", "cantilever", "square", "plane", "column", "symmetric", "tets", "poly"],
                    help="cube: 3D LE manufactured solution on a perturbed n^3 mesh (default); cantilever: "
                         "3D neo-Hookean 200x20x20 beam, 10 load increments; square: 2D 32x32 LE, p=2; "
                         "column: the vibrating neo-Hookean column, BDF2 time steps; symmetric: a polynomial "
                         "field symmetric about x = 0 on a tensor-perturbed n^3 box whose x = 0 faces are "
                         "symmetry planes; tets: the cube's hexahedra split into 6 tetrahedra; poly: the cube's "
                         "problem on the n^3 grid with every other 2x2x2 block merged into one 24-face cell")
    ap.add_argument("--column-cells", default="50x5x5", help="cells of the column (length x width x depth)")
    ap.add_argument("--time-steps", type=int, default=100, help="BDF2 steps of the column (dt = 1 ms)")
    ap.add_argument("--n", type=int, default=64, help="cells per axis")
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=1000, help="cells for the CPU oracle (0: skip)")
    ap.add_argument("--solve", type=int, default=1, help="also time a Newton solve to 1e-8")
    ap.add_argument("--learned", type=int, default=1,
                    help="train the learned correction and time the learned Newton solve")
    ap.add_argument("--learned-size", type=int, default=24, help="cells per axis of the training meshes")
    ap.add_argument("--nej-inner", type=int, default=4,
                    help="inner GMRES iterations per application of the near-exact Jacobian (solver nej)")
    ap.add_argument("--learned-epochs", type=int, default=60)
    ap.add_argument("--tol", type=float, default=0.0, help="Newton tolerance (default 1e-8; 1e-10 for square)")
    ap.add_argument("--max-krylov", type=int, default=4000, help="Krylov iterations per Newton step")
    ap.add_argument("--calib", type=int, default=0,
                    help="run a plain 512 MiB elementwise copy first (counter calibration)")
    ap.add_argument("--precond-levels", type=int, default=None,
                    help="multigrid levels built for the approximate Jacobian (1: sweeps only); the plain and "
                         "learned solves use the sweeps, a third solve the V-cycle")
    ap.add_argument("--study", choices=["train", "eval", "nn", "cpu"], default=None,
                    help="learned-preconditioner study instead of the benchmark: train a model on "
                         "--train-seeds (saved to --model), evaluate --model on one mesh, or time the "
                         "learned application alone (nn)")
    ap.add_argument("--cpu-workloads", default="square32p2,cube64p3,cantilever,cube128p1,cube128p2",
                    help="workloads of --study cpu")
    ap.add_argument("--train-seeds", default="0-49")
    ap.add_argument("--train-set", choices=["mixed", "cube", "cantilever"], default="cube",
                    help="training meshes of --study train: mixed = 2D squares and neo-Hookean beams (the learned-"
                         "preconditioner configuration), cube = perturbed cubes of --learned-size, cantilever = beams")
    ap.add_argument("--mg-base", type=int, default=0,
                    help="1: the network corrects the V-cycle's output (training and evaluation contexts build the "
                         "multigrid hierarchy); 0: the sweeps'")
    ap.add_argument("--train-order-seed", type=int, default=0, help="seed of the training loop's pair order")
    ap.add_argument("--harvest-starts", type=int, default=4)
    ap.add_argument("--harvest-length", type=int, default=9)
    ap.add_argument("--model", default="learned_model.hofvnn",
                    help="weights file (hofv_nn_save format) written by --study train, read by eval")
    ap.add_argument("--seed", type=int, default=50, help="mesh seed of --study eval")
    ap.add_argument("--max-newton", type=int, default=10, help="Newton steps per increment in --study eval")
    ap.add_argument("--eta", type=float, default=None,
                    help="Krylov tolerance of each Newton step (default 1e-4; cantilever 0.5 with --forcing 1)")
    ap.add_argument("--restart", type=int, default=None,
                    help="FGMRES cycle length, at most 2048 (default 30; cantilever 250)")
    ap.add_argument("--line-search", type=int, default=None,
                    help="Newton backtracking halvings; -1: full steps (halved only at an inverted cell)")
    ap.add_argument("--forcing", type=int, default=None,
                    help="0: Krylov tolerance --eta on every Newton step; 1: Eisenstat-Walker from --eta")
    ap.add_argument("--predictor", type=int, default=None,
                    help="1: start each load increment from the secant prediction (one library call for "
                         "all increments)")
    ap.add_argument("--side", type=int, default=0,
                    help="0: right-preconditioned FGMRES; 1: left-preconditioned GMRES as eq. jfnk prints it "
                         "(its tolerance is on the preconditioned residual)")
    ap.add_argument("--solvers", default=None,
                    help="time-to-tolerance solves to run: any of plain, multigrid, learned (learned needs plain), "
                         "nej / nejmg (the near-exact Jacobian of App. C over the sweeps / the V-cycle, linear elastic law)")
    ap.add_argument("--stepwise", type=int, default=0,
                    help="time-to-tolerance solves as one logged library Newton step per call, at most this many "
                         "steps per increment (0: one library call per increment)")
    ap.add_argument("--lz", type=float, default=1.0, help="z extent of the evaluation cube (cell aspect 1/lz)")
    ap.add_argument("--gs-passes", type=int, default=None,
                    help="classical Gram-Schmidt passes per Arnoldi step: 1 once (PETSc's default orthogonalisation; "
                         "the default here), 2 twice (the default for the cantilever's 250-vector cycles)")
    ap.add_argument("--graphs", type=int, default=None,
                    help="1: replay each Arnoldi step as a HIP graph after its first run (captured in the "
                         "first solve that reaches it: time a solve after a warm-up on the same state tensor), "
                         "0: launch one by one (default)")
    ap.add_argument("--stencil-grow", type=int, default=0,
                    help="grow stencils that fail the pivot test by this many cells at a time (0: such a "
                         "stencil is an error)")
    ap.add_argument("--big", type=int, default=1,
                    help="1: also the 128^3 p = 3 leg (J.v throughput, sampled oracle error, plain and learned "
                         "Newton with the committed model) after the cube workload")
    ap.add_argument("--big-n", type=int, default=128)
    ap.add_argument("--big-seed", type=int, default=50, help="mesh seed of the 128^3 leg (unseen in training)")
    ap.add_argument("--big-solve", type=int, default=1, help="time-to-tolerance solves in the 128^3 leg")
    ap.add_argument("--learned-model", default=MIXED_MODEL, help="weights of the learned correction for the 128^3 leg")
    args = ap.parse_args()
    # solver settings per workload, where not given: the slender cantilever needs long
    # cycles, full Newton steps, the forcing term and the predictor (its sweeps-only
    # solve does not converge, so it runs the multigrid one)
    defaults = {"eta": 1e-4, "restart": 30, "line_search": 10, "forcing": 0, "predictor": 0,
                "solvers": "plain,multigrid,learned", "precond_levels": 8, "gs_passes": 1, "graphs": 0}
    if args.workload == "cantilever":
        defaults.update(eta=0.5, restart=250, line_search=-1, forcing=1, predictor=1, solvers="multigrid",
                        gs_passes=2)
    elif args.workload == "column":  # the mass term keeps each step well conditioned
        defaults.update(eta=0.1, restart=60, line_search=-1, forcing=1, precond_levels=1)
    for key, val in defaults.items():
        if getattr(args, key) is None:
            setattr(args, key, val)
    KRYLOV.update(eta=args.eta, restart=args.restart, line_search=args.line_search, forcing=args.forcing,
                  predictor=args.predictor, side=args.side, gs_passes=args.gs_passes, graphs=args.graphs)
    solvers = set(args.solvers.split(","))
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not built",
              file=sys.stderr)
        sys.exit(2)

    if args.study == "cpu":
        cpu_study(args)
        return
    if args.study:
        study(args)
        return

    import torch

    import workloads as w
    from paper_2601_18417_amd import api

    dev = torch.device("cuda:0")
    if args.calib:
        # plain read-8-bytes/write-8-bytes kernel over 512 MiB, for scaling HBM counters
        xa = torch.ones(1 << 26, dtype=torch.float64, device=dev)
        ya = torch.empty_like(xa)
        torch.mul(xa, 1.0, out=ya)
        torch.cuda.synchronize()
        del xa, ya
    if args.workload == "cube":
        prob = w.cube_mms(args.n, args.p, perturb=0.2, seed=0)
    elif args.workload == "cantilever":
        prob = w.cantilever(p=args.p)
    elif args.workload == "column":
        prob = w.vibrating_column(tuple(int(x) for x in args.column_cells.split("x")), p=args.p)
    elif args.workload == "tets":
        prob = w.tet_mms(args.n, args.p, perturb=0.2, seed=0)
    elif args.workload == "poly":
        prob = w.split_mms((args.n // 2,) * 3, args.p, perturb=0.2, seed=0)
    elif args.workload == "symmetric":
        prob = w.poly_patch(w.box_mesh((args.n,) * 3, perturb=0.2, seed=0, mode="tensor"), args.p, args.p, seed=1,
                            symmetric=True)
    elif args.workload == "plane":  # the square's problem at n^2 perturbed cells
        prob = w.square_mms(args.n, args.p, perturb=0.2, seed=0)
    else:
        prob = w.square_mms(32, args.p)
    prob.stencil_grow = args.stencil_grow
    nc, D = prob.mesh.n_cells, prob.dim
    t0 = time.perf_counter()
    ctx = api.context_for(prob, precond_levels=args.precond_levels)
    t_setup = time.perf_counter() - t0
    log(f"setup {t_setup:.1f}s report {ctx.report}")
    multigrid = args.precond_levels >= 2
    if multigrid:
        try:
            ctx.set_multigrid(False)  # the plain preconditioner is the sweeps
        except api.HofvError:
            multigrid = False  # too small a mesh for a second level

    cen = ctx.cell_centroids()
    if prob.loads.exact is not None:
        u = torch.tensor(prob.loads.exact.value(cen).T.copy(), device=dev)
    else:  # a bent state of the beam: u_y = -0.3 x^2 / L (0.03 for the column), the throughput state
        L = prob.mesh.lengths[0]
        st = np.zeros((nc, 3))
        st[:, 1] = -(0.03 if args.workload == "column" else 0.3) * cen[:, 0] ** 2 / L
        u = torch.tensor(st.T.copy(), device=dev)
    v = torch.tensor(np.random.default_rng(1000).standard_normal((D, nc)), device=dev)
    Ru = torch.empty_like(u)
    Jv = torch.empty_like(u)
    stream = torch.cuda.current_stream()

    JVP_KERNELS = ("k_face_le", "k_face_q", "k_face_nh", "k_extrap", "k_cell_sum", "k_pack", "k_sumsq2")

    def kernel_times():
        out = {}
        for name in JVP_KERNELS:
            ms, cnt = ctx.kernel_time(name)
            if cnt:
                out[name] = {"avg_ms": ms / cnt, "launches": cnt}
        return out

    # warm-up, every kernel timed: finds the dominant kernel
    ctx.residual(u, Ru)
    ctx.set_timing(True)
    for _ in range(max(args.warmup, 1)):
        ctx.jvp(u, Ru, v, Jv)
    torch.cuda.synchronize()
    warm = kernel_times()
    dom = max(warm, key=lambda k: warm[k]["avg_ms"])

    # headline: J.v, events around the dominant kernel only (events around every
    # kernel would add their own gaps to the step)
    ctx.set_timing(True, only=dom)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.jvp(u, Ru, v, Jv)
    torch.cuda.synchronize()
    t_jvp = time.perf_counter() - t0
    dom_ms, dom_n = ctx.kernel_time(dom)
    ms_step = 1e3 * t_jvp / args.steps

    # per-kernel breakdown: the same steps again with every kernel timed
    ctx.set_timing(True)
    for _ in range(args.steps):
        ctx.jvp(u, Ru, v, Jv)
    torch.cuda.synchronize()
    kernels = kernel_times()
    ctx.set_timing(False)

    # residual alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.residual(u, Ru)
    torch.cuda.synchronize()
    ms_res = 1e3 * (time.perf_counter() - t0) / args.steps

    byts = ctx.kernel_bytes(dom)
    dom_avg = dom_ms / dom_n
    achieved = byts / (dom_avg * 1e-3) / 1e9
    for k in kernels:
        try:
            b = ctx.kernel_bytes(k)
            kernels[k]["GBps"] = b / (kernels[k]["avg_ms"] * 1e-3) / 1e9
        except Exception:
            pass
    log(f"kernels {json.dumps(kernels)}")
    jvp_bytes = sum(ctx.kernel_bytes(k) for k in kernels if k in ("k_face_le", "k_face_q", "k_face_nh", "k_extrap",
                                                                  "k_cell_sum"))

    def newton(learned):
        uu = torch.zeros_like(u)
        out = newton_run(torch, ctx, prob, nc, learned,
                         args.tol if args.tol > 0 else (1e-10 if args.workload == "square" else 1e-8),
                         args.max_krylov, u_out=uu, stepwise=args.stepwise)
        ctx.set_load_scale(1.0)
        if args.workload == "cantilever":
            # mean transverse displacement of the last layer of cells / length
            L = prob.mesh.lengths[0]
            tip = np.nonzero(cen[:, 0] > L - L / prob.mesh.shape[0])[0]
            uy = uu[1].cpu().numpy()[tip]
            out["tip_deflection_over_length"] = float(abs(uy.mean()) / L)
        return out

    solve = None
    if args.solve and args.workload == "column":
        solve = {"dynamics": column_steps(args, torch, ctx, prob, cen)}
    elif args.solve:
        solve = {"krylov": {"eta": args.eta, "forcing": args.forcing, "restart": args.restart,
                            "line_search": args.line_search, "predictor": args.predictor, "side": args.side,
                            "gs_passes": 1 if args.gs_passes == 1 else 2, "graphs": args.graphs}}
        if "plain" in solvers:
            if prob.n_increments == 1:
                newton(False)  # warm-up (allocates the Krylov workspace)
            solve["plain"] = newton(False)
            solve["plain_preconditioner"] = "compact approximate Jacobian, 2 FP32 symmetric Gauss-Seidel sweeps"
            log(f"plain solve {solve['plain']}")
        if multigrid and "multigrid" in solvers:
            ctx.set_multigrid(True)
            if prob.n_increments == 1:
                newton(False)
            solve["multigrid"] = newton(False)
            solve["multigrid_preconditioner"] = ("the same matrix by a smoothed-aggregation V-cycle "
                                                 "(2 sweeps on the cell level, 2 Jacobi steps on coarser ones)")
            ctx.set_multigrid(False)
            log(f"multigrid solve {solve['multigrid']}")
        for name, inner_mg in (("nej", False), ("nejmg", True)):
            if name not in solvers or prob.material != w.LINEAR_ELASTIC or (inner_mg and not multigrid):
                continue
            ctx.set_multigrid(inner_mg)
            ctx.set_nej(args.nej_inner)
            if prob.n_increments == 1:
                newton(False)
            solve[name] = newton(False)
            solve[name + "_preconditioner"] = (f"near-exact Jacobian (App. C): {args.nej_inner} GMRES iterations on "
                                               "the stabilisation-free operator, right-preconditioned by the "
                                               + ("V-cycle" if inner_mg else "sweeps"))
            ctx.set_nej(0)
            ctx.set_multigrid(False)
            log(f"{name} solve {solve[name]}")
        # one application of each preconditioner, host-timed over 20 calls
        rr = torch.randn((D, nc), device=dev, dtype=torch.float64, generator=torch.Generator(device=dev).manual_seed(5))
        zz = torch.empty_like(rr)
        for mode in (["plain", "multigrid"] if multigrid else ["plain"]):
            ctx.set_multigrid(mode == "multigrid") if multigrid else None
            for _ in range(3):
                ctx.precond_apply(rr, zz)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                ctx.precond_apply(rr, zz)
            torch.cuda.synchronize()
            solve["precond_ms_" + mode] = (time.perf_counter() - t0) / 20 * 1e3
        if multigrid:
            ctx.set_multigrid(False)
        if args.learned and args.workload == "cube" and {"plain", "learned"} <= solvers:
            from paper_2601_18417_amd import learned as lrn
            t0 = time.perf_counter()
            data = []
            for seed in (1, 2, 3):  # training meshes: seeds other than the benchmark's
                tp = w.cube_mms(args.learned_size, args.p, perturb=0.2, seed=seed)
                tctx = api.context_for(tp)
                u0 = torch.zeros((3, tp.mesh.n_cells), device=dev, dtype=torch.float64)
                data.append(lrn.harvest(tctx, u0, n_starts=4, length=6, newton_steps=2, seed=seed))
            t_harvest = time.perf_counter() - t0
            model = api.Model(7)
            hist = lrn.train(model, data, epochs=args.learned_epochs, lr=2e-3, batch=4)
            t_train = time.perf_counter() - t0 - t_harvest
            ctx.attach(model)
            newton(True)
            solve["learned"] = newton(True)
            solve["learned_training"] = {
                "pairs": int(sum(len(d) for d in data)), "meshes": f"3 x {args.learned_size}^3 p={args.p} "
                "perturbed cubes, seeds 1-3", "epochs": args.learned_epochs, "harvest_seconds": t_harvest,
                "train_seconds": t_train, "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]}
            solve["learned_speedup"] = solve["plain"]["seconds"] / solve["learned"]["seconds"]
            r = torch.randn((3, nc), device=dev, dtype=torch.float64, generator=torch.Generator(device=dev).manual_seed(5))
            z = torch.empty_like(r)
            for _ in range(3):
                ctx.precond_apply(r, z, learned=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                ctx.precond_apply(r, z, learned=True)
            torch.cuda.synchronize()
            solve["precond_ms_learned"] = (time.perf_counter() - t0) / 20 * 1e3
            log(f"learned solve {solve['learned']} training {solve['learned_training']}")

    cpu = None
    if args.cpu_sample > 0:
        label = {"cube": f"{args.n}^3 p={args.p}", "cantilever": f"cantilever p={args.p}",
                 "square": f"32^2 p={args.p}", "plane": f"{args.n}^2 p={args.p}"}.get(
                     args.workload, f"{args.workload} p={args.p}")
        cpu = cpu_baseline(prob, min(args.cpu_sample, nc // 2), u.cpu().numpy().T.copy(),
                           v.cpu().numpy().T.copy(), ctx, torch, label,
                           cube=("cube", args.n, args.p) if args.workload == "cube" else None)
        log(f"cpu {cpu}")

    big, learned_big = None, None
    if args.big and args.workload == "cube":
        r = big_leg(args, torch, api, w, dev)
        big, learned_big = r if isinstance(r, tuple) else (r, None)

    out = {
        "metric": "J.v Mcells/s (FP64) & time-to-1e-8 residual, learned vs plain precond",
        "value": nc / (ms_step * 1e-3) / 1e6,
        "unit": "Mcells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": {"cube": f"3D linear elastic MMS, unit cube {args.n}^3 hex perturbed +-20% (seed 0), "
                                        f"p={args.p}, |S|={ctx.report['stencil_size']}, 2x2 Gauss/face, alpha=0.1",
                                "cantilever": f"3D neo-Hookean cantilever 200x20x20 hex (mu=1, lambda=10), p={args.p}, "
                                              f"|S|={ctx.report['stencil_size']}, 10 load increments",
                                "square": f"2D plane-strain LE MMS, 32x32 quads, p={args.p}, "
                                          f"|S|={ctx.report['stencil_size']}",
                                "plane": f"2D plane-strain LE MMS, unit square {args.n}^2 quads perturbed +-20% "
                                         f"(seed 0), p={args.p}, |S|={ctx.report['stencil_size']}",
                                "column": f"3D neo-Hookean vibrating column 6 x 0.2 x 0.2 m, {args.column_cells} hex, "
                                          f"p={args.p}, |S|={ctx.report['stencil_size']}, BDF2 dt = 1 ms",
                                "tets": f"3D linear elastic MMS, unit cube, {args.n}^3 hex perturbed +-20% (seed 0) "
                                        f"each split into 6 tetrahedra, p={args.p}, |S|={ctx.report['stencil_size']}",
                                "symmetric": f"3D LE polynomial (degree p) symmetric about x = 0, {args.n}^3 hex "
                                             f"tensor-perturbed +-20%, symmetry planes on x = 0, p={args.p}, "
                                             f"|S|={ctx.report['stencil_size']}",
                                "poly": f"3D linear elastic MMS, unit cube, {args.n}^3 hex perturbed +-20% (seed 0) "
                                        f"with every other 2x2x2 block merged into one 24-face polyhedron, "
                                        f"p={args.p}, |S|={ctx.report['stencil_size']}, fan-triangulated faces"
                                }[args.workload],
                   "n_cells": nc, "global_batch": nc, "parallelism": "single GPU",
                   **({"stencil_grow": args.stencil_grow, "grown_stencils": ctx.report["n_grown_stencils"]}
                      if args.stencil_grow else {})},
        "residual_mcells_s": nc / (ms_res * 1e-3) / 1e6,
        "jvp_algorithmic_GBps": jvp_bytes / (ms_step * 1e-3) / 1e9,
        "jvp_frac_of_hbm_peak": jvp_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(dom, args.n, args.p) if args.workload == "cube" else None,
                     "bytes_per_launch": byts, "avg_ms": dom_avg, "launches": dom_n},
        "kernels": kernels,
        "time_to_tol": solve,
        "cpu_baseline": cpu,
        "setup_seconds": t_setup,
        "precision_study_128": big,
        "learned_128": learned_big,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
