#!/usr/bin/env python3
"""Benchmark of the DG S_N sweep + VEF-moment path on one MI355X.

One step = one full pass of the hot path over the synthetic workload with all
inputs already in HBM: for the default workload (64x64 quadrilaterals, p = 2,
level-symmetric S8 = 40 directions, sigma_t log-uniform in [0.1, 100] per 8x8
block, scattering ratio 0.9, isotropic source 1, vacuum boundaries) that is 50
source iterations -- each a full transport sweep (assembly + local solve of
every element-direction pair in upwind order), the angular moments, the
boundary sums and the max-norm residual -- followed by the VEF closures.
The handle (host plan + upload) is created outside the timed region.

Prints one JSON line.  Metric: element-direction solves per second
(elements x directions x sweeps / time).  The roofline object refers to the
dominant kernel (the sweep kernel), timed with HIP events on its own stream.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "element-direction solves/sec and HBM GB/s; FP32 batched vs FP64 sweep at 1e-5"
FP64_PEAK_TFLOPS = 78.6    # MI355X vector FP64 (256 CU x 2.4 GHz x 128 flop/clk)
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32
HBM_PEAK_GBS = 8000.0


def sweep_flops_per_solve(p):
    """Algorithmic flops of one element-direction solve in the sweep kernel:
    LU with pivoting (2/3 n^3) + two triangular solves (2 n^2) + A = sigma_t M +
    Omega_x G^x + Omega_y G^y (6 n^2) + b = M s (2 n^2) + four face terms (12 (p+1)^2)."""
    n = (p + 1) ** 2
    return (2.0 / 3.0) * n ** 3 + 2 * n * n + 6 * n * n + 2 * n * n + 12 * (p + 1) ** 2


def sweep_bytes_per_solve(p, m, n_dir, s):
    """Algorithmic HBM bytes of one solve in the sweep kernel: psi write (n s),
    upwind trace read (2 (p+1) s), and the element data (control points,
    cross sections, scalar-flux coefficients) amortised over the n_dir/4
    directions of a quadrant that visit the element together."""
    n = (p + 1) ** 2
    return n * s + 2 * (p + 1) * s + ((m + 1) ** 2 * 16 + 16 + 8 * n) / (n_dir / 4.0)


def workload(name):
    from paper_2301_04758_amd import problems as P
    probs, run = P.make_config(name)
    return probs, run


def describe(name, probs, run):
    pr = probs[0]
    if name == "c2":
        return ("64x64 quads, p=2, S8 (40 dirs), sigma_t log-uniform [0.1,100] per 8x8 block, c=0.9, "
                "isotropic source 1, vacuum; 50 source iterations + closures")
    return "%s: %d problems, first %dx%d p=%d n_dir=%d" % (name, len(probs), pr.nx, pr.ny, pr.p, pr.n_dir)


TIMING_STRIDE = 10  # HIP events around every 10th sweep of a step (each event costs device time)


def run_gpu(probs, n_iter, precision, steps, warmup, timing=True, schedule="auto", tune=True):
    import torch
    from paper_2301_04758_amd import vef
    sw = vef.Sweep(probs, precision=precision, timing=TIMING_STRIDE if timing else 0, schedule=schedule)
    io = sw.buffers(n_iter=n_iter, store_psi=True)
    mio = sw.moment_buffers(io)
    stream = torch.cuda.current_stream()
    tuned = sw.autotune(io, n_iter=n_iter, reps=1, stream=stream) if tune and schedule == "auto" else None

    def step():
        sw.run(io, n_iter=n_iter, stream=stream)
        sw.moments(mio, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    sweep_ms = 0.0
    launches = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if timing:
        # HIP events of the last timed step around every TIMING_STRIDE-th
        # sweep (the handle reuses them per run, so reading them after every
        # step would stall the queue)
        sweep_ms, launches = sw.timing()
    sw.check()
    out = dict(seconds=t1 - t0, sweep_ms=sweep_ms, launches=launches,
               schedule=vef.SCHEDULE_NAMES[sw.info[0]["schedule"]], kernel=sw.info[0]["kernel"],
               n_levels=sw.info[0]["n_levels"], tuned=tuned,
               phi=[b["mom"][0].double().cpu().numpy() for b in io],
               resid=[b["resid"].cpu().numpy() for b in io])
    sw.close()
    return out


PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                       "k_sweep_pipe_c2_64x64_p2_S8_fp64.md")
KERNEL_SOURCES = ["paper_2301_04758_amd/csrc/sweep_device.h", "paper_2301_04758_amd/csrc/sweep_p2.hip",
                  "paper_2301_04758_amd/csrc/kernels.h"]


def measured_traffic(kernel):
    """HBM bytes per launch of the C2 pipelined kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel),
    or None when the kernel differs or its sources changed since then."""
    import hashlib
    import re
    if kernel != "k_sweep_pipe<2, 3, double, false, false>" or not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    m = re.search(r"traffic_bytes_per_launch=([0-9.e+]+) kernel_sources_sha256_16=([0-9a-f]+)", text)
    if not m:
        return None
    h = hashlib.sha256()
    root = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(root, f), "rb").read())
    return float(m.group(1)) if h.hexdigest()[:16] == m.group(2) else None


def kernel_name(g, pr):
    """Name of the sweep kernel that ran (as the profiler lists it)."""
    nq = pr.nq or pr.p + pr.m
    if g["schedule"] == "dir_resident" and g["kernel"] in (3, 4):
        return "k_sweep_pipe<%d, %d, double, false, %s>" % (pr.p, nq, "true" if g["kernel"] == 4 else "false")
    kind = "dir" if g["schedule"] == "dir_resident" else "level"
    return "k_sweep_%s<%d, %d, double, %d>" % (kind, pr.p, nq, g["kernel"])


def fixup_leg(probs, n_iter, steps, ms_plain):
    """The same FP64 workload with the negative-flux fixup inside the sweep:
    time per step, and the smallest angular flux with and without it."""
    import torch
    from paper_2301_04758_amd import vef
    out = {}
    for fix in (False, True):
        sw = vef.Sweep(probs, precision="fp64", fixup=fix)
        io = sw.buffers(n_iter=n_iter, store_psi=True)
        sw.autotune(io, n_iter=n_iter, reps=1)
        sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        sw.check()
        out["fixed" if fix else "plain"] = dict(ms=ms, min_psi=float(io[0]["psi_out"].min().item()),
                                                phi=io[0]["mom"][0].cpu().numpy())
        sw.close()
        del io
    import numpy as np
    p, f = out["plain"], out["fixed"]
    return {"ms_per_step": f["ms"], "overhead_vs_plain": f["ms"] / p["ms"], "min_psi_plain": p["min_psi"],
            "min_psi_fixed": f["min_psi"],
            "rel_inf_phi_change": float(np.abs(f["phi"] - p["phi"]).max() / np.abs(p["phi"]).max())}


def lagged_leg(steps, n_iter=5):
    """The 64x64 random mesh with reflex corners (p = 2, S8, cyclic upwind
    graphs, about an eighth of the element-direction pairs with a lagged
    inflow face): source iterations with lagged couplings, FP64 and
    FP32-local, time per sweep."""
    import numpy as np
    import torch
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd import vef
    pr = P.reentrant_quads(64)
    out = {"workload": "64x64 straight-sided quads, interior vertices moved up to 0.45 h (reflex corners), "
                       "p=2, S8, sigma_t log-uniform [0.1,100] per 8x8 block, c=0.9; %d sweeps per step" % n_iter}
    phi = {}
    for prec in ("fp64", "fp32"):
        sw = vef.Sweep([pr], precision=prec, lag_cycles=True)
        io = sw.buffers(n_iter=n_iter, store_psi=True)
        tuned = sw.autotune(io, n_iter=n_iter, reps=1)
        io[0]["psi_out"].zero_()
        sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / (steps * n_iter)
        sw.check()
        inf = sw.info[0]
        phi[prec] = io[0]["mom"][0].cpu().numpy()
        out[prec] = {"ms_per_sweep": ms, "solves_per_s": pr.n_elem * pr.n_dir / (ms * 1e-3),
                     "schedule": vef.SCHEDULE_NAMES[inf["schedule"]], "kernel": vef.KERNEL_NAMES[inf["kernel"]],
                     "tuning": tuned}
        out.update(n_lagged=inf["n_lagged"], lagged_frac=inf["n_lagged"] / (pr.n_elem * pr.n_dir),
                   n_levels=inf["n_levels"])
        sw.close()
        del io
    out["fp32_rel_inf_phi_vs_fp64"] = float(np.abs(phi["fp32"] - phi["fp64"]).max() / np.abs(phi["fp64"]).max())
    return out


def pointwise_leg(steps, n_iter=5):
    """Pointwise against whole-face upwinding on a curved mesh: the 64x64
    cubic Taylor-Green mesh (t = 0.3 pi), p = 2, S8, sigma_t log-uniform
    [0.1, 100] per 8x8 block, c = 0.9.  Whole-face upwinding gives acyclic
    graphs there; the pointwise rule couples both elements of every face
    along which Omega . n changes sign, and those couplings are lagged.  FP64
    source iterations, time per sweep."""
    import numpy as np
    import torch
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd import vef
    cp, ec = P.taylor_green_mesh(64, 3, t_final=0.3 * math.pi)
    om, wt = P.level_symmetric_2d(8)
    rng = np.random.Generator(np.random.PCG64(P.SEED_BASE + 13))
    st = P.block_log_uniform(64, 64, 8, 0.1, 100.0, rng)
    pr = P.Problem("tg64_m3_p2_S8", 2, 3, cp, ec, om, wt, st, 0.9 * st, nx=64, ny=64)
    pr.q_iso = np.ones((pr.n_elem, 9))
    out = {"workload": "64x64 cubic Taylor-Green mesh (t = 0.3 pi), p=2, S8, sigma_t log-uniform [0.1,100] per "
                       "8x8 block, c=0.9, FP64; %d sweeps per step" % n_iter}
    phi = {}
    for rule, pointwise in (("whole_face", False), ("pointwise", True)):
        sw = vef.Sweep([pr], precision="fp64", lag_cycles=True, pointwise=pointwise)
        io = sw.buffers(n_iter=n_iter, store_psi=True)
        tuned = sw.autotune(io, n_iter=n_iter, reps=1)
        io[0]["psi_out"].zero_()
        sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / (steps * n_iter)
        sw.check()
        inf = sw.info[0]
        phi[rule] = io[0]["mom"][0].cpu().numpy()
        out[rule] = {"ms_per_sweep": ms, "solves_per_s": pr.n_elem * pr.n_dir / (ms * 1e-3),
                     "schedule": vef.SCHEDULE_NAMES[inf["schedule"]], "kernel": vef.KERNEL_NAMES[inf["kernel"]],
                     "n_lagged": inf["n_lagged"], "lagged_frac": inf["n_lagged"] / (pr.n_elem * pr.n_dir),
                     "n_levels": inf["n_levels"], "tuning": tuned}
        sw.close()
        del io
    out["rel_inf_phi_pointwise_vs_whole_face"] = float(np.abs(phi["pointwise"] - phi["whole_face"]).max()
                                                       / np.abs(phi["whole_face"]).max())
    return out


def hrt_flops_bytes(p, nq):
    """Algorithmic flops and HBM bytes of one element of the HRT local block
    inverse on an affine element: the G block summed over the Gauss points
    (2 Q nv nphi: E varies from point to point), A and Ma scaled from reference
    matrices (nv^2 + nphi^2), in-place Gauss-Jordan 2 N^3; bytes: the N x N
    inverse written, the element's moments, geometry, cross sections and
    neighbours read."""
    nv, nphi = 2 * (p + 1) * (p + 2), (p + 1) ** 2
    n = nv + nphi
    Q = nq * nq
    return (2 * Q * nv * nphi + nv * nv + nphi * nphi + 2 * n ** 3,
            8 * n * n + 6 * (p + 1) ** 2 * 8 + 13 * 8 + 16 + 16)


def hrt_leg(reps=5):
    """Element-local HRT VEF block inverse (W, X, Y, Z) on the C2 mesh and a
    512x512 affine mesh, p = 2, nq = 4, E from the moments of one transport
    sweep: time per launch from HIP events on the launch stream."""
    import numpy as np
    import torch
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd import vef
    (c2,), _ = P.make_config("c2")
    big = P.make_problem("affine_512", 512, 512, 2, 1, 8, 1.0, 0.9)
    rng = np.random.Generator(np.random.PCG64(P.SEED_BASE + 11))
    big.sigma_t = P.block_log_uniform(512, 512, 8, 0.1, 100.0, rng)
    big.sigma_s = 0.9 * big.sigma_t
    out = {}
    for name, pr in (("c2_64x64", c2), ("affine_512x512", big)):
        pr.nq = 4
        sw = vef.Sweep([pr], precision="fp64")
        io = sw.buffers(n_iter=1, store_psi=False)
        sw.run(io, n_iter=1)
        mio = sw.moment_buffers(io)
        sw.moments(mio)
        inv = sw.hrt_local_inverse(0, io[0]["mom"], mio[0]["Eb"])
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            sw.hrt_local_inverse(0, io[0]["mom"], mio[0]["Eb"])
        b.record()
        torch.cuda.synchronize()
        sw.check()
        ms = a.elapsed_time(b) / reps
        F, B = hrt_flops_bytes(pr.p, pr.nq)
        tf = F * pr.n_elem / (ms * 1e-3) / 1e12
        gbs = B * pr.n_elem / (ms * 1e-3) / 1e9
        out[name] = {"elements": pr.n_elem, "n": inv.shape[1], "ms_per_launch": ms,
                     "elements_per_s": pr.n_elem / (ms * 1e-3),
                     "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                  "frac": tf / FP64_PEAK_TFLOPS, "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                                  "algorithmic_flops_per_element": F, "algorithmic_bytes_per_element": B}}
        # the element-local reduction of the hybridized solve from these inverses
        red = sw.hrt_reduce(0, io[0]["mom"], mio[0], inv)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            sw.hrt_reduce(0, io[0]["mom"], mio[0], inv)
        b.record()
        torch.cuda.synchronize()
        out[name]["reduce_ms_per_launch"] = a.elapsed_time(b) / reps
        del inv, red
        sw.close()
        del io, mio
    return out


def outer_leg():
    """Transport / hybridized-RT VEF outer iteration in the thick diffusion
    limit (Sec. 8): 64x64 unit square, p = 2, S8, sigma_t = 1/eps, sigma_a =
    eps, q = eps, eps = 1e-3, vacuum; outer iterations to a relative change of
    1e-8, plain and with two Anderson vectors (the paper's outer solver), with
    the time split between the transport / element-local stage and the
    lambda solve; the lambda system solved on the device (re-factorisation
    with the pivot order of one host factorisation) and, for comparison, on
    the host (SuperLU every iteration)."""
    import numpy as np
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd.vef_outer import VefOuter
    eps = 1e-3
    pr = P.make_problem("tdl_64", 64, 64, 2, 1, 8, 1.0 / eps, 1.0 / eps - eps, q=eps / (4 * math.pi))
    res = {"workload": "64x64, p=2, S8, sigma_t=1/eps, sigma_a=eps, q=eps, eps=1e-3 (thick diffusion limit)"}
    for mode in ("device", "host"):
        drv = VefOuter(pr, lambda_solve=mode)
        try:
            drv.step(None)  # warm-up (tables, geometry, allocations, the host factorisation)
            t0 = time.perf_counter()
            out = drv.solve(max_outer=20, tol=1e-8)
            total = time.perf_counter() - t0
            stage, solve = [], []
            phi = None
            for _ in range(3):
                phi, _, _ = drv.step(phi)
                stage.append(drv.last_times["stage_s"])
                solve.append(drv.last_times["solve_s"])
            r = {"outer_iterations": out["iterations"], "history": out["history"], "seconds_total": total,
                 "ms_per_outer_iteration": 1e3 * total / out["iterations"],
                 "stage_ms": 1e3 * float(np.median(stage)), "lambda_solve_ms": 1e3 * float(np.median(solve))}
            if mode == "device":
                acc = drv.solve(max_outer=20, tol=1e-8, anderson=2)
                diff = float(np.abs(acc["phi_leg"] - out["phi_leg"]).max() / np.abs(out["phi_leg"]).max())
                r["anderson2"] = {"outer_iterations": acc["iterations"], "history": acc["history"],
                                  "rel_diff_vs_plain": diff}
                r["host_factorisations"] = drv.host_factorisations
                r["last_rel_residual"] = drv.last_resid
                res.update(r)
                res["lambda_unknowns"] = drv.n_faces * (pr.p + 1)
                phi_dev = out["phi_leg"]
            else:
                r["rel_diff_vs_device_lambda"] = float(np.abs(out["phi_leg"] - phi_dev).max() /
                                                       np.abs(phi_dev).max())
                res["host_lambda_solve"] = r
        finally:
            drv.close()
    return res


def tdl_table(tol=1e-6):
    """The thick-diffusion-limit experiment of Sec. 8 (its table of
    fixed-point iteration counts): 8x8 orthogonal mesh of the unit square,
    p = 2, S4, sigma_t = 1/eps, sigma_a = eps, q = eps, vacuum; plain fixed
    point until the relative change of the VEF scalar flux is <= tol."""
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd.vef_outer import VefOuter
    out = {"workload": "8x8 unit square, p=2, S4, sigma_t=1/eps, sigma_a=eps, q=eps, vacuum; fixed point to a "
                       "change of successive iterates of %g, relative and in the max norm" % tol,
           "iterations": {}, "iterations_max_norm": {}, "paper_hrt": {"1e-1": 8, "1e-2": 6, "1e-3": 4, "1e-4": 3}}
    for eps in (1e-1, 1e-2, 1e-3, 1e-4):
        pr = P.make_problem("tdl_8", 8, 8, 2, 1, 4, 1.0 / eps, 1.0 / eps - eps, q=eps)
        drv = VefOuter(pr)
        try:
            r = drv.solve(max_outer=40, tol=tol)
            m = drv.solve(max_outer=40, tol=tol, stop="max_norm")
        finally:
            drv.close()
        out["iterations"]["%g" % eps] = r["iterations"]
        out["iterations_max_norm"]["%g" % eps] = m["iterations"]
    return out


def c4_batched(reps=3):
    """The 64-problem batch: plain FP64 level-synchronous sweeps one problem at
    a time, against all 64 in one FP32-local handle whose run is captured in a
    HIP graph and replayed.  Error: rel_inf of phi against the FP64 runs."""
    import numpy as np
    import torch
    from paper_2301_04758_amd import problems as P
    from paper_2301_04758_amd import vef
    probs, _ = P.make_config("c4")
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    t_plain, phi64 = 0.0, []
    for pr in probs:
        sw = vef.Sweep([pr], precision="fp64", schedule="level")
        io = sw.buffers(n_iter=1, store_psi=False)
        sw.run(io, n_iter=1)
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record()
        for _ in range(reps):
            sw.run(io, n_iter=1)
        b.record()
        torch.cuda.synchronize()
        sw.check()
        t_plain += a.elapsed_time(b) / reps
        phi64.append(io[0]["mom"][0].cpu().numpy())
        sw.close()
        del io
    sw = vef.Sweep(probs, precision="fp32")
    io = sw.buffers(n_iter=1, store_psi=False)
    tuned = sw.autotune(io, n_iter=1, reps=2)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sw.run(io, n_iter=1)
    g.replay()
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record()
    for _ in range(reps):
        g.replay()
    b.record()
    torch.cuda.synchronize()
    sw.check()
    t_batch = a.elapsed_time(b) / reps
    err = max(float(np.abs(io[k]["mom"][0].cpu().numpy() - phi64[k]).max() / np.abs(phi64[k]).max())
              for k in range(len(probs)))
    solves = sum(p.n_elem * p.n_dir for p in probs)
    out = {"problems": len(probs), "solves_per_sweep": solves, "plain_fp64_one_by_one_ms": t_plain,
           "batched_fp32_graph_ms": t_batch, "schedule": vef.SCHEDULE_NAMES[sw.info[0]["schedule"]],
           "tuning": tuned,
           "rel_inf_phi_vs_fp64": err, "within_1e-5": err <= 1e-5,
           "speedup": (t_plain / t_batch) if err <= 1e-5 else None,
           "batched_solves_per_s": solves / (t_batch * 1e-3)}
    del g
    sw.close()
    return out


def cpu_baseline(probs, iters):
    """The oracle (serial double-precision C, gcc -O2) on the host, on the first
    `iters` source iterations of the same workload."""
    from oracle import oracle as O
    pr = probs[0]
    t0 = time.perf_counter()
    r = O.source_iteration(pr, iters)
    dt = time.perf_counter() - t0
    solves = pr.n_elem * pr.n_dir * r["iters"]
    return dict(value=solves / dt, unit="element-direction solves/s", cores=1, kind="oracle",
                sample="first %d of the 50 source iterations of the same workload (%d solves, %.1f s)"
                % (r["iters"], solves, dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=30)
    ap.add_argument("--schedule", default="auto", choices=["auto", "level", "dir"],
                    help="auto: the library's autotuner picks schedule and kernel before the timed steps")
    ap.add_argument("--no-c4", action="store_true", help="skip the 64-problem batched FP32 vs one-by-one FP64 block")
    ap.add_argument("--no-fixup", action="store_true", help="skip the negative-flux fixup leg")
    ap.add_argument("--no-lagged", action="store_true", help="skip the re-entrant-mesh lagged-sweep leg")
    ap.add_argument("--no-pointwise", action="store_true", help="skip the pointwise-upwinding leg")
    ap.add_argument("--no-hrt", action="store_true", help="skip the HRT local block inverse leg")
    ap.add_argument("--no-outer", action="store_true", help="skip the transport / VEF outer iteration leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of 256 MiB (three times), the reference kernel "
                         "for scaling HBM byte counters")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the sweep library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    probs, run = workload(args.workload)
    n_iter = run["n_iter"]
    pr = probs[0]
    solves_per_step = sum(p.n_elem * p.n_dir for p in probs) * n_iter

    from paper_2301_04758_amd import vef
    machine = vef.vef_probe_machine()
    g64 = run_gpu(probs, n_iter, "fp64", args.steps, args.warmup, schedule=args.schedule)
    ms_step = 1e3 * g64["seconds"] / args.steps
    value = solves_per_step * args.steps / g64["seconds"]

    # dominant kernel: the sweep kernel, timed by events on the run's stream
    # over the last timed step
    F = sweep_flops_per_solve(pr.p)
    B = sweep_bytes_per_solve(pr.p, pr.m, pr.n_dir, 8)
    launches = max(g64["launches"], 1)
    avg_launch_s = g64["sweep_ms"] * 1e-3 / launches
    n_timed = sum(1 for it in range(n_iter) if (it + 1) % TIMING_STRIDE == 0 or it == n_iter - 1)
    solves_per_launch = solves_per_step / n_iter * n_timed / launches
    achieved_tf = F * solves_per_launch / avg_launch_s / 1e12
    kname = kernel_name(g64, pr)
    sweeps_per_launch = solves_per_launch / sum(p.n_elem * p.n_dir for p in probs)
    t_bw = B * solves_per_launch / (HBM_PEAK_GBS * 1e9)
    t_flop = F * solves_per_launch / (FP64_PEAK_TFLOPS * 1e12)
    # the chain of dependent levels can go no faster than one measured
    # wave-to-wave hand-off per level (vef_probe_machine)
    t_cp = g64["n_levels"] * sweeps_per_launch * machine["lds_handoff_ns"] * 1e-9
    roofline = {"bound": "alu", "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved_tf / FP64_PEAK_TFLOPS, "traffic": measured_traffic(kname),
                "kernel": kname, "avg_launch_us": avg_launch_s * 1e6,
                "levels_per_sweep": g64["n_levels"],
                "us_per_level": avg_launch_s * 1e6 / (g64["n_levels"] * sweeps_per_launch),
                "lower_bounds_us": {"hbm": t_bw * 1e6, "fp64_alu": t_flop * 1e6,
                                    "critical_path_handoff": t_cp * 1e6},
                "binding": "critical path: %d dependent upwind levels per sweep" % g64["n_levels"],
                "frac_of_critical_path_bound": t_cp / avg_launch_s,
                "measured_peak": machine["fp64_fma_tflops"],
                "frac_of_measured_peak": achieved_tf / machine["fp64_fma_tflops"],
                "launches_per_step": launches / n_timed * n_iter,
                "algorithmic_flops_per_solve": F, "algorithmic_bytes_per_solve": B,
                "hbm_frac": (B * solves_per_launch / avg_launch_s / 1e9) / HBM_PEAK_GBS}
    hbm_gbs = B * solves_per_step / (ms_step * 1e-3) / 1e9

    result = {
        "metric": METRIC, "value": value, "unit": "element-direction solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": describe(args.workload, probs, run), "n_elem": pr.n_elem, "p": pr.p,
                   "n_dir": pr.n_dir, "sweeps_per_step": n_iter,
                   "schedule": ("autotuned: " if g64["tuned"] else "") + g64["schedule"],
                   "tuning": g64["tuned"],
                   "precision": "fp64"},
        "hbm_gbs_algorithmic": hbm_gbs,
        "roofline": roofline,
        "machine": machine,
    }
    if not args.no_fp32:
        g32 = run_gpu(probs, n_iter, "fp32", args.steps, args.warmup, schedule=args.schedule)
        ms32 = 1e3 * g32["seconds"] / args.steps
        err = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(g32["phi"], g64["phi"]))
        result["fp32_local"] = {"ms_per_step": ms32, "value": solves_per_step / (ms32 * 1e-3),
                                "speedup_vs_fp64": ms_step / ms32,
                                "rel_inf_phi_vs_fp64_path": err, "within_1e-5": err <= 1e-5}
    if not args.no_fixup:
        result["fixup_fp64"] = fixup_leg(probs, n_iter, args.steps, ms_step)
    if not args.no_lagged:
        result["lagged_reentrant"] = lagged_leg(args.steps)
    if not args.no_pointwise:
        result["pointwise_upwinding"] = pointwise_leg(args.steps)
    if not args.no_hrt:
        result["hrt_local_inverse"] = hrt_leg()
    if not args.no_outer:
        result["vef_outer_thick_limit"] = outer_leg()
        result["vef_outer_thick_limit"]["eps_table"] = tdl_table()
    if not args.no_c4:
        result["c4_batched_fp32_vs_plain_fp64"] = c4_batched()
    if args.copy_calibration:
        n = 256 << 20
        src = torch.ones(n // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration"] = {"bytes_read": n, "bytes_written": n, "launches": 3,
                                      "gbs": 2 * n * 3 / (time.perf_counter() - t0) / 1e9}
        del src, dst
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(probs, args.cpu_iters)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
