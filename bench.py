#!/usr/bin/env python3
"""Benchmark of the DG S_N sweep + VEF-moment path on one MI355X.

One step = one full pass of the hot path over the synthetic workload with all
inputs already in HBM.  The default workload is the largest single-GPU
configuration, the thick diffusive regime: 512x512 quadrilaterals, p = 4 (25
unknowns per element), the 144-direction level-symmetric S16 set,
sigma_t = 1000, sigma_s = 999.9, isotropic source 1, vacuum boundaries; a step
is one transport sweep (assembly + local solve of every element-direction
pair in upwind order) with the angular moments, the boundary sums, the
max-norm residual and the VEF closures.  The handle (host plan + upload) is
created outside the timed region.

Prints one JSON line.  Metric: element-direction solves per second
(elements x directions x sweeps / time).  The roofline object refers to the
sweep kernel, timed with HIP events on the stream it is launched on; its
algorithmic flops and bytes per solve are those of the method (pivoted LU,
two triangular solves, assembly from element matrices, face terms, moments),
not of the implementation.
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
FP32_PEAK_TFLOPS = 157.3   # MI355X vector FP32 (packed forms)
HBM_PEAK_GBS = 8000.0
GOLDEN = os.path.join(ROOT, "tests", "golden")

WORKLOADS = {
    "c5": dict(n_iter=1, fixture="c5_full.json",
               text="512x512 straight quads, p=4 (25 unknowns/element), S16 (144 directions, LS16-moment set), "
                    "sigma_t=1000, sigma_s=999.9 (c=0.9999), isotropic source 1, vacuum; one transport sweep "
                    "with moments, boundary sums, residual and VEF closures per step"),
    "c3": dict(n_iter=1, fixture="c3_full.json",
               text="256x256 quads curved by 0.1 sin(pi x) sin(pi y)(1,1) (quadratic geometry), p=3, S12 "
                    "(84 directions), sigma_t U[1,10] per element, c=0.5, isotropic source 1, vacuum; one sweep "
                    "with moments and closures per step"),
    "c2": dict(n_iter=50, fixture="c2_full.json",
               text="64x64 quads, p=2, S8 (40 directions), sigma_t log-uniform [0.1,100] per 8x8 block, c=0.9, "
                    "isotropic source 1, vacuum; 50 source iterations + closures per step"),
}


def flops_per_solve(p):
    """Algorithmic flops of one element-direction solve: LU (2/3 n^3), two
    triangular solves (2 n^2), A = sigma_t M + Omega_x G^x + Omega_y G^y
    (6 n^2), b = M s (2 n^2), two outflow and two inflow face terms
    (12 (p+1)^2) and the six angular moments (12 n)."""
    n = (p + 1) ** 2
    return (2.0 / 3.0) * n ** 3 + 2 * n * n + 6 * n * n + 2 * n * n + 12 * (p + 1) ** 2 + 12 * n


def flops_per_solve_shared(p):
    """Algorithmic flops of one solve by the matrix K = A^-1 R of its class of
    shared local matrices: the product with the nodal source (n columns) and
    with the traces of the two inflow faces (2 (p+1) columns),
    2 n (n + 2 (p+1)), and the six angular moments (12 n).  Forming K once
    per class and run (O(n^3)) is amortised over the class's solves and left
    out (under one flop per solve at 512x512, S16)."""
    n = (p + 1) ** 2
    return 2 * n * (n + 2 * (p + 1)) + 12 * n


def bytes_per_solve(p, m, n_dir, s):
    """Algorithmic HBM bytes of one solve: the angular flux written (n s), the
    upwind trace read (2 (p+1) s), and per element the control points, cross
    sections, scalar-flux coefficients and six moments (48 n), amortised over
    the n_dir / 4 directions of a quadrant that visit the element together.
    s = 8 (double) or 4 (float angular flux)."""
    n = (p + 1) ** 2
    return n * s + 2 * (p + 1) * s + ((m + 1) ** 2 * 16 + 16 + 8 * n + 48 * n) / (n_dir / 4.0)


def roofline(probs, s, sweep_s, launches_per_sweep, kernel, alu_peak, traffic=None, shared=False):
    """Roofline of the sweep kernel over one sweep of probs: algorithmic flops
    and bytes per launch against the average launch duration; the bound is
    the ALU when F/B exceeds the machine balance, else HBM.  shared: the
    solves go through their class matrices (flops_per_solve_shared)."""
    fps = flops_per_solve_shared if shared else flops_per_solve
    F = sum(pr.n_elem * pr.n_dir * fps(pr.p) for pr in probs)
    B = sum(pr.n_elem * pr.n_dir * bytes_per_solve(pr.p, pr.m, pr.n_dir, s) for pr in probs)
    solves = sum(pr.n_elem * pr.n_dir for pr in probs)
    L = max(launches_per_sweep, 1)
    avg = sweep_s / L
    balance = alu_peak * 1e12 / (HBM_PEAK_GBS * 1e9)
    if F / B > balance:
        out = {"bound": "alu", "achieved": F / L / avg / 1e12, "peak": alu_peak, "unit": "TFLOP/s"}
    else:
        out = {"bound": "hbm", "achieved": B / L / avg / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    out["frac"] = out["achieved"] / out["peak"]
    out["traffic"] = traffic
    out.update(kernel=kernel, launches_per_sweep=L, avg_launch_us=avg * 1e6,
               algorithmic_flops_per_solve=F / solves, algorithmic_bytes_per_solve=B / solves,
               flop_per_byte=F / B, machine_balance_flop_per_byte=balance,
               algorithmic_hbm_gbs=B / sweep_s / 1e9, hbm_frac=B / sweep_s / 1e9 / HBM_PEAK_GBS,
               alu_tflops=F / sweep_s / 1e12, alu_frac=F / sweep_s / 1e12 / alu_peak)
    return out


def workload(name):
    from paper_2301_04758_amd import problems as P
    probs, run = P.make_config(name)
    return probs, run


def fixture_error(name, mom_list):
    """rel_inf of the moments against the oracle's sampled values of the same
    workload (tests/golden, written from oracle/ only): max over the six
    moments of max|gpu - oracle| at the sampled nodes / max|oracle phi|."""
    import numpy as np
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    idx = np.asarray(g["index"])
    flat = mom_list[0].reshape(6, -1)
    scale = g["mom_absmax"][0]
    phi_err = float(np.abs(flat[0, idx] - np.asarray(g["mom"][0])).max() / scale)
    all_err = max(float(np.abs(flat[k, idx] - np.asarray(g["mom"][k])).max() / scale) for k in range(6))
    return {"phi": phi_err, "all_moments": all_err, "fixture": "tests/golden/" + name}


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
    n_timed = sum(1 for it in range(n_iter) if (it + 1) % TIMING_STRIDE == 0 or it == n_iter - 1)
    out = dict(seconds=t1 - t0, sweep_ms=sweep_ms / n_timed, launches=launches / n_timed,
               schedule=vef.SCHEDULE_NAMES[sw.info[0]["schedule"]], kernel=sw.info[0]["kernel"],
               n_levels=sw.info[0]["n_levels"], tuned=tuned,
               mom=[b["mom"].cpu().numpy() for b in io],
               phi=[b["mom"][0].double().cpu().numpy() for b in io],
               resid=[b["resid"].cpu().numpy() for b in io])
    sw.close()
    return out


PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2301_04758_amd/csrc/sweep_device.h", "paper_2301_04758_amd/csrc/kernels.h"]


def sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by what the same counters read for a
    plain copy kernel), or None when none covers it or the kernel sources
    changed since it was taken."""
    import re
    if not os.path.isdir(PROFILES):
        return None
    want = sources_hash()
    for f in sorted(os.listdir(PROFILES)):
        text = open(os.path.join(PROFILES, f)).read()
        for m in re.finditer(r"traffic kernel=(\S+) traffic_bytes_per_launch=([0-9.e+]+) "
                             r"kernel_sources_sha256_16=([0-9a-f]+)", text):
            if m.group(1) == kernel.replace(" ", "") and m.group(3) == want:
                return float(m.group(2))
    return None


def kernel_name(g, pr, dtype="double", single=True):
    """Name of the sweep kernel that ran (as the profiler lists it); single:
    the handle holds one problem (the level-synchronous row-set LU then runs
    in its streaming form)."""
    nq = pr.nq or pr.p + pr.m
    if g["schedule"] == "dir_resident" and g["kernel"] in (3, 4):
        return "k_sweep_pipe<%d, %d, %s, false, %s>" % (pr.p, nq, dtype, "true" if g["kernel"] == 4 else "false")
    if g["kernel"] in (5, 7):
        level = "level_lus" if single else "level_lu"
        kind = {"dir_resident": "dir_lu", "persistent": "flow", "level_sync": level}[g["schedule"]]
        if kind == "flow":
            return "k_sweep_flow<%d, %d, %s, 5>" % (pr.p, nq, dtype)
        if kind == "level_lus":
            # last template argument: solves by the class inverses
            return "k_sweep_level_lus<%d, %d, %s, false, %s>" % (pr.p, nq, dtype,
                                                                 "true" if g["kernel"] == 7 else "false")
        return "k_sweep_%s<%d, %d, %s, false>" % (kind, pr.p, nq, dtype)
    kind = {"dir_resident": "dir", "persistent": "flow", "level_sync": "level"}[g["schedule"]]
    return "k_sweep_%s<%d, %d, %s, %d>" % (kind, pr.p, nq, dtype, g["kernel"])


def workload_leg(name, steps, warmup, schedule):
    """FP64 and FP32-local runs of one configuration: time per step, solves/s,
    roofline of the sweep kernel, error of the moments against the oracle's
    sampled values."""
    probs, _ = workload(name)
    cfg = WORKLOADS[name]
    n_iter = cfg["n_iter"]
    solves = sum(p.n_elem * p.n_dir for p in probs) * n_iter
    out = {"workload": cfg["text"]}
    for prec, s, peak, dt in (("fp64", 8, FP64_PEAK_TFLOPS, "double"), ("fp32", 4, FP32_PEAK_TFLOPS, "float")):
        g = run_gpu(probs, n_iter, prec, steps, warmup, schedule=schedule)
        ms = 1e3 * g["seconds"] / steps
        kname = kernel_name(g, probs[0], dt, single=len(probs) == 1)
        out[prec] = {"ms_per_step": ms, "solves_per_s": solves / (ms * 1e-3), "schedule": g["schedule"],
                     "tuning": g["tuned"], "sweep_ms": g["sweep_ms"],
                     "roofline": roofline(probs, s, g["sweep_ms"] * 1e-3, g["launches"], kname, peak,
                                          measured_traffic(kname), shared=g["kernel"] == 7),
                     "rel_inf_vs_oracle": fixture_error(cfg["fixture"], g["mom"])}
    out["fp32_speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["fp32"]["ms_per_step"]
    return out


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
    # error of the batch (and of the plain runs) against the oracle's sampled
    # values of the problems the fixture holds
    ora = {}
    path = os.path.join(GOLDEN, "c4_some.json")
    if os.path.exists(path):
        g = json.load(open(path))
        e32 = e64 = 0.0
        for item in g["problems"]:
            k, idx = item["problem"], np.asarray(item["index"])
            ref, scale = np.asarray(item["mom"][0]), item["mom_absmax"][0]
            e32 = max(e32, float(np.abs(io[k]["mom"][0].cpu().numpy().reshape(-1)[idx] - ref).max() / scale))
            e64 = max(e64, float(np.abs(phi64[k].reshape(-1)[idx] - ref).max() / scale))
        ora = {"batched_fp32": e32, "plain_fp64": e64, "problems_checked": len(g["problems"]),
               "fixture": "tests/golden/c4_some.json"}
    out = {"problems": len(probs), "solves_per_sweep": solves, "plain_fp64_one_by_one_ms": t_plain,
           "batched_fp32_graph_ms": t_batch, "schedule": vef.SCHEDULE_NAMES[sw.info[0]["schedule"]],
           "tuning": tuned,
           "rel_inf_phi_vs_fp64": err, "within_1e-5": err <= 1e-5, "rel_inf_phi_vs_oracle": ora,
           "speedup": (t_plain / t_batch) if err <= 1e-5 else None,
           "batched_solves_per_s": solves / (t_batch * 1e-3),
           # the replayed graph holds the sweep kernels and the moment kernels of all 64 problems
           "roofline_graph": roofline(probs, 4, t_batch * 1e-3, 1, "graph replay (sweep + moments, 64 problems)",
                                      FP32_PEAK_TFLOPS)}
    del g
    sw.close()
    return out


def cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(probs, n_dirs=16, max_threads=16):
    """The oracle (double-precision C, gcc -O2, OpenMP over directions) on the
    host cores, on a bounded sample of the same workload: one sweep of n_dirs
    of its directions (evenly spaced over the set, so every quadrant is in it)
    from phi = 0, all cores; and one direction on one core."""
    import numpy as np
    from oracle import oracle as O
    pr = probs[0]
    threads = max(1, min(max_threads, os.cpu_count() or 1, n_dirs))
    dirs = np.linspace(0, pr.n_dir - 1, n_dirs).round().astype(np.int32)
    t0 = time.perf_counter()
    O.sweep(pr, dirs=dirs, want_psi=False, threads=threads)
    dt = time.perf_counter() - t0
    solves = pr.n_elem * len(dirs)
    t0 = time.perf_counter()
    O.sweep(pr, dirs=dirs[:1], want_psi=False, threads=1)
    dt1 = time.perf_counter() - t0
    out = dict(value=solves / dt, unit="element-direction solves/s", cores=threads, kind="oracle",
               sample="one sweep of %d of the %d directions of the same workload from phi = 0 (%d solves, "
                      "%.1f s, %d OpenMP threads, one direction per thread)" % (len(dirs), pr.n_dir, solves, dt,
                                                                               threads),
               serial={"value": pr.n_elem / dt1, "cores": 1, "sample": "one direction (%d solves, %.1f s)"
                       % (pr.n_elem, dt1)})
    out.update(cpu_info())
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--schedule", default="auto", choices=["auto", "level", "dir", "persistent"],
                    help="auto: the library's autotuner picks schedule and kernel before the timed steps")
    ap.add_argument("--legs", default="c3,c2,c4,fixup,lagged,pointwise,hrt,outer",
                    help="comma-separated extra legs (c3, c2: the same measurements on those configurations; "
                         "c4: 64-problem batched FP32 graph vs one-by-one FP64; fixup, lagged, pointwise, hrt, "
                         "outer); 'none' for the headline only")
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
    legs = set() if args.legs == "none" else set(args.legs.split(","))

    cfg = WORKLOADS[args.workload]
    probs, _ = workload(args.workload)
    n_iter = cfg["n_iter"]
    pr = probs[0]
    solves_per_step = sum(p.n_elem * p.n_dir for p in probs) * n_iter

    from paper_2301_04758_amd import vef
    machine = vef.vef_probe_machine()
    g64 = run_gpu(probs, n_iter, "fp64", args.steps, args.warmup, schedule=args.schedule)
    ms_step = 1e3 * g64["seconds"] / args.steps
    value = solves_per_step * args.steps / g64["seconds"]
    kname = kernel_name(g64, pr)
    roof = roofline(probs, 8, g64["sweep_ms"] * 1e-3, g64["launches"], kname, FP64_PEAK_TFLOPS,
                    measured_traffic(kname), shared=g64["kernel"] == 7)
    roof.update(levels_per_sweep=g64["n_levels"], measured_peak=machine["fp64_fma_tflops"],
                frac_of_measured_peak=roof["alu_tflops"] / machine["fp64_fma_tflops"],
                # lower bounds of one sweep: HBM traffic, FP64 ALU work, and the chain of dependent
                # levels at one measured wave-to-wave hand-off each
                lower_bounds_us={"hbm": 1e6 * roof["algorithmic_bytes_per_solve"] * solves_per_step / n_iter
                                 / (HBM_PEAK_GBS * 1e9),
                                 "fp64_alu": 1e6 * roof["algorithmic_flops_per_solve"] * solves_per_step / n_iter
                                 / (FP64_PEAK_TFLOPS * 1e12),
                                 "critical_path_handoff": g64["n_levels"] * machine["lds_handoff_ns"] * 1e-3})
    result = {
        "metric": METRIC, "value": value, "unit": "element-direction solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": cfg["text"], "name": args.workload, "n_elem": pr.n_elem, "p": pr.p,
                   "n_dir": pr.n_dir, "sweeps_per_step": n_iter,
                   "schedule": ("autotuned: " if g64["tuned"] else "") + g64["schedule"],
                   "kernel": vef.KERNEL_NAMES[g64["kernel"]],
                   "tuning": g64["tuned"], "precision": "fp64"},
        "rel_inf_vs_oracle": fixture_error(cfg["fixture"], g64["mom"]),
        "roofline": roof,
        "machine": machine,
    }
    if not args.no_fp32:
        g32 = run_gpu(probs, n_iter, "fp32", args.steps, args.warmup, schedule=args.schedule)
        ms32 = 1e3 * g32["seconds"] / args.steps
        err = max(float(np.abs(a - b).max() / np.abs(b).max()) for a, b in zip(g32["phi"], g64["phi"]))
        ora = fixture_error(cfg["fixture"], g32["mom"])
        k32 = kernel_name(g32, pr, "float")
        result["fp32_local"] = {"ms_per_step": ms32, "value": solves_per_step / (ms32 * 1e-3),
                                "speedup_vs_fp64": ms_step / ms32, "schedule": g32["schedule"],
                                "rel_inf_vs_oracle": ora,
                                "within_1e-5_of_oracle": (ora["phi"] <= 1e-5) if ora else None,
                                "rel_inf_phi_vs_fp64_path": err,
                                "roofline": roofline(probs, 4, g32["sweep_ms"] * 1e-3, g32["launches"], k32,
                                                     FP32_PEAK_TFLOPS, measured_traffic(k32),
                                                     shared=g32["kernel"] == 7)}
    for leg in ("c3", "c2"):
        if leg in legs and leg != args.workload:
            result["workload_" + leg] = workload_leg(leg, args.steps, args.warmup, args.schedule)
    if "fixup" in legs:
        p2, r2 = workload("c2")
        result["fixup_fp64"] = fixup_leg(p2, r2["n_iter"], args.steps, None)
    if "lagged" in legs:
        result["lagged_reentrant"] = lagged_leg(args.steps)
    if "pointwise" in legs:
        result["pointwise_upwinding"] = pointwise_leg(args.steps)
    if "hrt" in legs:
        result["hrt_local_inverse"] = hrt_leg()
    if "outer" in legs:
        result["vef_outer_thick_limit"] = outer_leg()
        result["vef_outer_thick_limit"]["eps_table"] = tdl_table()
    if "c4" in legs:
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
        result["cpu_baseline"] = cpu_baseline(probs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
