"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Bar: rel_inf(x, ref) = max|x - ref| / max|ref| <= 1e-12 for the all-double
path and <= 1e-5 for float local solves with double moments, residuals and
closures (tolerances of the target; the float bound covers float rounding of
the local assembly/solve accumulated along upwind chains).
"""
import numpy as np
import pytest

import dg_numpy as D
import mms
from oracle import oracle as O
from paper_2301_04758_amd import problems as P

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def rel_inf(x, ref, scale=None):
    """max|x - ref| / max|ref|, or / scale for quantities that vanish up to roundoff."""
    s = np.abs(ref).max() if scale is None else scale
    return float(np.abs(np.asarray(x) - ref).max() / max(s, 1e-300))


def closure_scales(cl):
    """Natural magnitude of each closure output: Q1 vanishes for isotropic sources, so it
    is measured against Q0; the others against themselves."""
    return {"E": None, "Eb": None, "Jin": None, "Q0": None, "Q1": np.abs(cl["Q0"]).max()}


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def gpu_run(torch, problems, precision, n_iter=1, phi_in=None, tol=0.0, store_psi=True, closures=False,
            schedule="auto", pipeline_waves=0, pipeline_ring=0):
    from paper_2301_04758_amd import vef
    print("gpu_run", [p.name for p in problems][:3], precision, schedule, "n_iter", n_iter,
          "pipeline", pipeline_waves, pipeline_ring, flush=True)
    sw = vef.Sweep(problems, precision=precision, schedule=schedule, pipeline_waves=pipeline_waves,
                   pipeline_ring=pipeline_ring)
    io = sw.buffers(n_iter=n_iter, store_psi=store_psi, phi_in=phi_in)
    iters = torch.zeros(1, dtype=torch.int32, device="cuda")
    sw.run(io, n_iter=n_iter, tol=tol, iters_done=iters)
    out = dict(io=io, iters=None)
    if closures:
        mio = sw.moment_buffers(io)
        sw.moments(mio)
        out["mio"] = mio
    torch.cuda.synchronize()
    sw.check()
    out["iters"] = int(iters.item())
    out["info"] = sw.info
    res = []
    for k in range(len(problems)):
        r = {key: (v.cpu().numpy() if hasattr(v, "cpu") else v) for key, v in io[k].items() if v is not None}
        if closures:
            r.update({"cl_" + key: v.cpu().numpy() for key, v in out["mio"][k].items() if v is not None})
        res.append(r)
    sw.close()
    return res, out


def _small(nx, ny, p, m, N, st=1.0, ss=0.0, warp=0.0, q=1.0, seed=0):
    cp, ec = P.quad_mesh(nx, ny, m)
    if warp:
        cp = P.sine_warp(cp, warp)
    om, wt = P.level_symmetric_2d(N)
    ne = nx * ny
    rng = np.random.default_rng(seed)
    st = np.broadcast_to(np.asarray(st, float), (ne,)).copy() if not callable(st) else st(rng, ne)
    ss = np.broadcast_to(np.asarray(ss, float), (ne,)).copy() if not callable(ss) else ss(rng, ne)
    pr = P.Problem("small_%dx%d_p%d_m%d_S%d" % (nx, ny, p, m, N), p, m, cp, ec, om, wt, st, ss, nx=nx, ny=ny)
    pr.q_iso = np.full((ne, (p + 1) ** 2), float(q))
    return pr


SCHEDULES = ["level", "dir"]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_single_sweep(torch, precision, schedule):
    (pr,), _ = P.make_config("c1")
    (g,), _ = gpu_run(torch, [pr], precision, closures=True, schedule=schedule)
    ref = O.sweep(pr)
    tol = TOL[precision]
    assert rel_inf(g["psi_out"], ref["psi"]) <= tol
    for k in range(6):
        assert rel_inf(g["mom"][k], ref["mom"][k]) <= tol or np.abs(ref["mom"][k]).max() < 1e-12
    cl = O.closures(pr, ref["mom"], ref["bnd"])
    sc = closure_scales(cl)
    for key in ("E", "Eb", "Q0", "Q1"):
        assert rel_inf(g["cl_" + key], cl[key], sc[key]) <= tol, key
    assert np.abs(g["cl_Jin"]).max() == 0 and np.abs(cl["Jin"]).max() == 0  # vacuum inflow
    assert int(g["cl_n_nonpos"][0]) == cl["n_nonpos"]
    # the residual of one sweep from phi_in = 0 is max |phi|
    assert abs(g["resid"][0] - np.abs(ref["mom"][0]).max()) <= tol * np.abs(ref["mom"][0]).max()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c2_scaled_source_iteration(torch, precision, schedule):
    (pr,), _ = P.make_config("c2", scale=16)
    n_iter = 12
    (g,), out = gpu_run(torch, [pr], precision, n_iter=n_iter, schedule=schedule)
    ref = O.source_iteration(pr, n_iter)
    tol = TOL[precision]
    assert out["iters"] == n_iter
    for k in range(6):
        assert rel_inf(g["mom"][k], ref["mom"][k]) <= tol
    assert np.abs(g["resid"] - ref["resid"]).max() <= tol * ref["resid"].max()


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(12, 12, 3, 2, 12), (7, 5, 2, 2, 8), (9, 4, 1, 3, 6), (6, 6, 4, 2, 4)])
def test_curved_meshes(torch, precision, shape, schedule):
    nx, ny, p, m, N = shape
    pr = _small(nx, ny, p, m, N, st=lambda r, n: r.uniform(1, 10, n), warp=0.1 if m == 2 else 0.05)
    pr.sigma_s = 0.5 * pr.sigma_t
    phi = np.random.default_rng(1).uniform(0, 3, (pr.n_elem, (p + 1) ** 2))
    (g,), _ = gpu_run(torch, [pr], precision, phi_in=phi, closures=True, schedule=schedule)
    ref = O.sweep(pr, phi_in=phi)
    tol = TOL[precision]
    assert rel_inf(g["psi_out"], ref["psi"]) <= tol
    assert rel_inf(g["mom"][0], ref["mom"][0]) <= tol
    cl = O.closures(pr, ref["mom"], ref["bnd"])
    assert rel_inf(g["cl_E"], cl["E"]) <= 10 * tol
    assert rel_inf(g["cl_Eb"], cl["Eb"]) <= 10 * tol


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_straight_non_affine_mesh(torch, precision, p, schedule):
    """Trapezoids (straight faces, varying J): the general pivot-free path."""
    from test_library_host import _trapezoids
    cp, ec = _trapezoids(7, 0.2, seed=p)
    om, wt = P.level_symmetric_2d(6)
    ne = ec.shape[0]
    rng = np.random.default_rng(p)
    st = rng.uniform(0.5, 20, ne)
    pr = P.Problem("trap", p, 1, cp, ec, om, wt, st, 0.7 * st, q_iso=rng.uniform(0, 1, (ne, (p + 1) ** 2)))
    nb = O.n_boundary_faces(pr)
    pr.psi_bc = rng.uniform(0, 1, (pr.n_dir, nb, p + 1))
    phi = rng.uniform(0, 2, (ne, (p + 1) ** 2))
    (g,), _ = gpu_run(torch, [pr], precision, phi_in=phi, schedule=schedule)
    ref = O.sweep(pr, phi_in=phi)
    assert rel_inf(g["psi_out"], ref["psi"]) <= TOL[precision]
    assert rel_inf(g["mom"][0], ref["mom"][0]) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p,m,warp", [(2, 2, 0.08), (3, 1, 0.0), (1, 2, 0.05), (4, 1, 0.0), (2, 2, 0.0)])
def test_mms_inputs(torch, precision, p, m, warp):
    """Direction-dependent source at volume points and non-isotropic inflow data."""
    pr = _small(8, 8, p, m, 4, warp=warp, q=0.0)
    pr.q_iso = None
    vxy, bxy, _ = O.qp_coords(pr)
    mms.attach(pr, vxy, bxy)
    (g,), _ = gpu_run(torch, [pr], precision, closures=True)
    ref = O.sweep(pr)
    tol = TOL[precision]
    assert rel_inf(g["psi_out"], ref["psi"]) <= tol
    for k in range(6):
        assert rel_inf(g["mom"][k], ref["mom"][k]) <= tol
    cl = O.closures(pr, ref["mom"], ref["bnd"])
    sc = closure_scales(cl)
    for key in ("E", "Eb", "Jin", "Q0", "Q1"):
        assert rel_inf(g["cl_" + key], cl[key], sc[key]) <= 10 * tol, key


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thick_p4_scaled(torch, precision, schedule):
    """C5-like thick diffusive cells (sigma_t = 1000, c = 0.9999), p = 4, S16."""
    (pr,), _ = P.make_config("c5", scale=10)
    n_iter = 3
    (g,), _ = gpu_run(torch, [pr], precision, n_iter=n_iter, schedule=schedule)
    ref = O.source_iteration(pr, n_iter)
    tol = TOL[precision]
    assert rel_inf(g["mom"][0], ref["mom"][0]) <= tol
    assert np.abs(g["resid"] - ref["resid"]).max() <= tol * ref["resid"].max()


def test_edge_cases_single_element_and_ragged(torch):
    # one element, every face on the boundary, non-vacuum inflow
    pr = _small(1, 1, 3, 1, 8, st=2.0, ss=1.0)
    pr.psi_bc = np.random.default_rng(5).uniform(0, 1, (pr.n_dir, 4, 4))
    (g,), _ = gpu_run(torch, [pr], "fp64")
    ref = O.sweep(pr)
    assert rel_inf(g["psi_out"], ref["psi"]) <= 1e-12
    # a long thin strip: levels with a ragged number of solves
    pr = _small(37, 3, 2, 1, 6, st=lambda r, n: r.uniform(0.1, 50, n))
    (g,), _ = gpu_run(torch, [pr], "fp64")
    ref = O.sweep(pr)
    assert rel_inf(g["psi_out"], ref["psi"]) <= 1e-12


def test_zero_scattering_source_and_internal_psi(torch):
    """psi_out = NULL keeps the angular flux inside the library: same moments."""
    pr = _small(10, 9, 2, 1, 6, st=lambda r, n: r.uniform(0.5, 5, n))
    pr.sigma_s = 0.8 * pr.sigma_t
    (a,), _ = gpu_run(torch, [pr], "fp64", n_iter=4)
    (b,), _ = gpu_run(torch, [pr], "fp64", n_iter=4, store_psi=False)
    assert np.array_equal(a["mom"], b["mom"])
    assert np.array_equal(a["resid"], b["resid"])


def test_repeat_runs_bitwise(torch):
    (pr,), _ = P.make_config("c2", scale=16)
    (a,), _ = gpu_run(torch, [pr], "fp64", n_iter=3)
    (b,), _ = gpu_run(torch, [pr], "fp64", n_iter=3)
    assert np.array_equal(a["psi_out"], b["psi_out"])
    assert np.array_equal(a["mom"], b["mom"])


def test_device_side_tolerance_stop(torch):
    pr = _small(6, 6, 1, 1, 4, st=lambda r, n: r.uniform(1, 4, n))
    pr.sigma_s = 0.5 * pr.sigma_t
    (g,), out = gpu_run(torch, [pr], "fp64", n_iter=60, tol=1e-9)
    ref = O.source_iteration(pr, 60, tol=1e-9)
    assert out["iters"] == ref["iters"] < 60
    assert rel_inf(g["mom"][0], ref["mom"][0]) <= 1e-12
    assert np.abs(g["resid"][:ref["iters"]] - ref["resid"]).max() <= 1e-12 * ref["resid"].max()
    assert np.all(g["resid"][ref["iters"]:] == 0)


def test_nonpositive_flux_count(torch):
    pr = _small(4, 4, 1, 1, 4, st=200.0, q=0.0)
    pr.q_iso[0] = 50.0
    (g,), _ = gpu_run(torch, [pr], "fp64", closures=True)
    ref = O.sweep(pr)
    cl = O.closures(pr, ref["mom"], ref["bnd"])
    assert cl["n_nonpos"] > 0
    assert int(g["cl_n_nonpos"][0]) == cl["n_nonpos"]


def test_invalid_problem_rejected_before_launch(torch):
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c1")
    pr.weight = pr.weight * 2
    with pytest.raises(vef.VefError):
        vef.Sweep([pr])


@pytest.mark.parametrize("p,m,warp,kernel", [(3, 2, 0.05, "general_mat"), (2, 2, 0.05, None),
                                             (1, 1, 0.0, None)])
def test_level_lists_start_problems_on_whole_waves(torch, p, m, warp, kernel):
    """Three problems of one kernel variant in one handle, with level widths
    that leave partial waves: the level kernel takes each wave's problem from
    its first slot, so every problem's solves start on a whole wave (padding
    entries between them).  Each problem gives the bits it gives alone."""
    from paper_2301_04758_amd import vef
    probs = [_small(5, 3, p, m, 4, st=2.0, ss=0.3, warp=warp, seed=1),
             _small(3, 7, p, m, 4, st=0.5, ss=0.3, warp=warp, seed=2),
             _small(7, 5, p, m, 4, st=lambda r, n: r.uniform(0.5, 5.0, n), ss=0.3, warp=warp, seed=3)]
    batch, out = gpu_run(torch, probs, "fp64", n_iter=2, schedule="level")
    kinds = {vef.KERNEL_NAMES[i["kernel"]] for i in out["info"]}
    assert len(kinds) == 1 and (kernel is None or kinds == {kernel}), kinds
    for k, pr in enumerate(probs):
        (alone,), _ = gpu_run(torch, [pr], "fp64", n_iter=2, schedule="level")
        for key in ("psi_out", "mom", "resid"):
            assert np.array_equal(batch[k][key], alone[key]), (k, key)
        ref = O.source_iteration(pr, 2)
        assert rel_inf(batch[k]["mom"][0], ref["mom"][0]) <= TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg,scale", [("c2", 24), ("c3", 10), ("c5", 12)])
def test_schedules_agree(torch, precision, cfg, scale):
    """The schedules run the same per-solve arithmetic in a different order
    and must agree bit for bit (any race or stale read would show), except
    for affine elements of degree <= 2, where the direction-resident schedule
    factors each local matrix once (LU, then substitution) instead of
    Gauss-Jordan, and for the solves of curved degree-3 elements that are not
    certified for elimination in natural order, which the direction-resident
    schedule pivots as it eliminates while the others take the rows in the
    pivoting order formed beforehand: there they agree to rounding."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config(cfg, scale=scale)
    (a,), _ = gpu_run(torch, [pr], precision, n_iter=2, schedule="level")
    (b,), _ = gpu_run(torch, [pr], precision, n_iter=2, schedule="dir")
    # the persistent schedule runs the level-synchronous kernels' arithmetic
    (c,), _ = gpu_run(torch, [pr], precision, n_iter=2, schedule="persistent")
    for key in ("psi_out", "mom", "resid"):
        assert np.array_equal(a[key], c[key]), key
    info = vef.vef_plan_query(pr)
    if info["affine"] and pr.p <= 2:
        assert rel_inf(b["psi_out"], a["psi_out"]) <= TOL[precision]
        assert rel_inf(b["mom"][0], a["mom"][0]) <= TOL[precision]
        return
    if not info["affine"] and pr.p == 3 and info["n_pivoting"] > 0:
        tol = 1e-13 if precision == "fp64" else 2e-6
        assert rel_inf(b["psi_out"], a["psi_out"]) <= tol
        assert rel_inf(b["mom"][0], a["mom"][0]) <= tol
        return
    assert np.array_equal(a["psi_out"], b["psi_out"])
    assert np.array_equal(a["mom"], b["mom"])
    assert np.array_equal(a["resid"], b["resid"])


PIPE_CASES = [(1, 4), (8, 4), (3, 2), (8, 1), (2, 1)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["c2", "p1", "strip"])
def test_pipeline_depths_bitwise(torch, precision, case):
    """The pipelined kernel with 1..8 waves and 1..4 ring levels: identical
    bits (one wave is the serial order; ring depth 1 hands every upwind trace
    over through global memory) and oracle parity."""
    if case == "c2":
        (pr,), _ = P.make_config("c2", scale=20)
        n_iter = 3
    elif case == "p1":
        pr = _small(33, 29, 1, 1, 8, st=lambda r, n: r.uniform(0.2, 30, n), ss=0.0)
        n_iter = 1
    else:  # levels wider than one wave and a ragged last chunk
        pr = _small(150, 70, 2, 1, 4, st=lambda r, n: r.uniform(0.5, 8, n))
        pr.sigma_s = 0.3 * pr.sigma_t
        n_iter = 2
    runs = [gpu_run(torch, [pr], precision, n_iter=n_iter, schedule="dir", pipeline_waves=w,
                    pipeline_ring=r)[0][0] for w, r in PIPE_CASES]
    for k in range(1, len(runs)):
        assert np.array_equal(runs[0]["psi_out"], runs[k]["psi_out"]), PIPE_CASES[k]
        assert np.array_equal(runs[0]["mom"], runs[k]["mom"]), PIPE_CASES[k]
        assert np.array_equal(runs[0]["resid"], runs[k]["resid"]), PIPE_CASES[k]
    ref = O.source_iteration(pr, n_iter) if n_iter > 1 else O.sweep(pr)
    assert rel_inf(runs[0]["mom"][0], ref["mom"][0]) <= TOL[precision]
    if n_iter == 1:
        assert rel_inf(runs[0]["psi_out"], ref["psi"]) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("p,nx,N", [(1, 23, 6), (2, 90, 4), (2, 7, 8)])
def test_bilinear_pipeline(torch, precision, p, nx, N):
    """Straight-sided bilinear elements (trapezoids) on the direction-resident
    schedule: the pipelined kernel with quadrature assembly, identical bits for
    1..8 waves and ring depths 1..4, and oracle parity with a direction
    dependent source and boundary inflow (nx = 90: levels wider than one wave,
    ragged last chunks)."""
    from test_library_host import _trapezoids
    from paper_2301_04758_amd import vef
    cp, ec = _trapezoids(nx, 0.2, seed=nx)
    om, wt = P.level_symmetric_2d(N)
    ne = ec.shape[0]
    rng = np.random.default_rng(p + nx)
    st = rng.uniform(0.5, 20, ne)
    nq = p + 2 if nx == 7 else p + 1
    pr = P.Problem("trap_pipe", p, 1, cp, ec, om, wt, st, 0.7 * st, q_iso=rng.uniform(0, 1, (ne, (p + 1) ** 2)),
                   nq=nq)
    pr.q_dir = rng.uniform(0, 1, (pr.n_dir, ne, nq * nq))
    pr.psi_bc = rng.uniform(0, 1, (pr.n_dir, O.n_boundary_faces(pr), nq))
    phi = rng.uniform(0, 2, (ne, (p + 1) ** 2))
    runs = []
    for w, r in PIPE_CASES:
        (g,), out = gpu_run(torch, [pr], precision, phi_in=phi, schedule="dir", pipeline_waves=w, pipeline_ring=r)
        assert out["info"][0]["kernel"] == vef.VEF_KERNEL_BILINEAR_PIPELINE
        runs.append(g)
    for k in range(1, len(runs)):
        assert np.array_equal(runs[0]["psi_out"], runs[k]["psi_out"]), PIPE_CASES[k]
        assert np.array_equal(runs[0]["mom"], runs[k]["mom"]), PIPE_CASES[k]
    ref = O.sweep(pr, phi_in=phi, nq=nq)
    assert rel_inf(runs[0]["psi_out"], ref["psi"]) <= TOL[precision]
    assert rel_inf(runs[0]["mom"][0], ref["mom"][0]) <= TOL[precision]
    # the row-per-lane kernel of the same problem (pipelining off)
    (g,), out = gpu_run(torch, [pr], precision, phi_in=phi, schedule="dir", pipeline_waves=-1)
    assert out["info"][0]["kernel"] == vef.VEF_KERNEL_NOPIVOT
    assert rel_inf(g["psi_out"], runs[0]["psi_out"]) <= TOL[precision]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("p,m,warp", [(3, 2, 0.08), (2, 1, 0.0), (1, 3, 0.05)])
def test_translation_invariance(torch, schedule, p, m, warp):
    """A mesh on a 2^-30 grid shifted by 2^10 is the same problem: the
    library evaluates the geometry from coordinate differences, so the bits
    agree (absolute coordinates would cost about eps * 2^10 / h)."""
    pr = _small(20, 20, p, m, 6, st=lambda r, n: r.uniform(0.5, 8, n), warp=warp)
    pr.sigma_s = 0.5 * pr.sigma_t
    pr.cp_xy = np.round(pr.cp_xy * 2.0 ** 30) / 2.0 ** 30
    (a,), _ = gpu_run(torch, [pr], "fp64", n_iter=2, schedule=schedule)
    pr.cp_xy = pr.cp_xy + 2.0 ** 10
    (b,), _ = gpu_run(torch, [pr], "fp64", n_iter=2, schedule=schedule)
    assert np.array_equal(a["psi_out"], b["psi_out"])
    assert np.array_equal(a["mom"], b["mom"])


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_capture_replays(torch, precision, schedule):
    """After one eager run, a run with the same arguments issues only kernel
    launches, so it can be captured in a HIP graph.  Every replay, with eager
    work on the same buffers in between, gives the bits of the eager run."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c2", scale=16)
    pr.sigma_s = 0.9 * pr.sigma_t
    small = _small(9, 7, 1, 1, 4, st=lambda r, n: r.uniform(0.5, 5, n))
    small.sigma_s = 0.5 * small.sigma_t
    print("graph capture", precision, schedule, flush=True)
    sw = vef.Sweep([pr, small], precision=precision, schedule=schedule)
    io = sw.buffers(n_iter=3)
    sw.run(io, n_iter=3)
    torch.cuda.synchronize()
    sw.check()
    ref = [{k: b[k].clone() for k in ("mom", "psi_out", "resid")} for b in io]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sw.run(io, n_iter=3)
    for rep in range(3):
        for b in io:  # eager work between replays
            b["mom"].fill_(-1.0)
            b["psi_out"].zero_()
            b["resid"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sw.check()
        for k, b in enumerate(io):
            for key in ("mom", "psi_out", "resid"):
                assert torch.equal(b[key], ref[k][key]), (rep, k, key)
    del g
    sw.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_choice_keeps_parity(torch, precision):
    """vef_sweep_autotune times every schedule/kernel candidate and keeps the
    fastest; the handle then reports it and still matches the oracle."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c2", scale=20)
    small = _small(11, 6, 3, 1, 6, st=lambda r, n: r.uniform(0.5, 5, n))
    small.sigma_s = 0.5 * small.sigma_t
    probs = [pr, small]
    print("autotune", precision, flush=True)
    sw = vef.Sweep(probs, precision=precision)
    io = sw.buffers(n_iter=2)
    res = sw.autotune(io, n_iter=2, reps=2)
    assert res["n_candidates"] >= 4
    assert 0 < res["best_ms"] <= res["before_ms"]
    assert sw.info[0]["schedule"] == res["schedule"]
    if res["schedule"] == vef.VEF_DIR_RESIDENT and res["pipeline_waves"] >= 0:
        assert sw.info[0]["kernel"] == vef.VEF_KERNEL_AFFINE_PIPELINE
    else:
        assert sw.info[0]["kernel"] == vef.VEF_KERNEL_AFFINE
    sw.run(io, n_iter=2)
    torch.cuda.synchronize()
    sw.check()
    for k, p in enumerate(probs):
        ref = O.source_iteration(p, 2)
        assert rel_inf(io[k]["mom"][0].cpu().numpy(), ref["mom"][0]) <= TOL[precision]
    with pytest.raises(vef.VefError):
        sw.autotune(io, n_iter=1, reps=0)
    sw.close()


def test_probe_machine(torch):
    """Measured roofline denominators are in a plausible range for MI355X
    (published: 8 TB/s HBM, 78.6 TFLOP/s FP64 vector)."""
    from paper_2301_04758_amd import vef
    m = vef.vef_probe_machine()
    print("machine", m, flush=True)
    assert m["compute_units"] >= 1
    assert 500 < m["hbm_copy_gbs"] < 9000
    assert 1 < m["fp64_fma_tflops"] < 90
    assert 1 < m["fp32_fma_tflops"] < 180
    assert 1 < m["lds_handoff_ns"] < 100000


@pytest.mark.parametrize("schedule", ["level", "dir"])
def test_timing_stride(torch, schedule):
    """vef_options.timing = k times the sweep kernels of every k-th source
    iteration and of the last one; k = 1 times all.  Results do not depend
    on it."""
    from paper_2301_04758_amd import vef
    pr = _small(12, 12, 2, 1, 4, st=2.0, ss=1.0)
    out = {}
    for k in (1, 3):
        sw = vef.Sweep([pr], precision="fp64", schedule=schedule, timing=k)
        io = sw.buffers(n_iter=7, store_psi=False)
        sw.run(io, n_iter=7)
        ms, nl = sw.timing()
        sw.check()
        out[k] = (ms, nl, io[0]["mom"].cpu().numpy())
        sw.close()
    per_sweep = out[1][1] // 7
    assert out[1][1] == 7 * per_sweep and per_sweep >= 1
    assert out[3][1] == 3 * per_sweep  # iterations 3, 6 and the last (7)
    assert out[1][0] > 0 and out[3][0] > 0
    assert np.array_equal(out[1][2], out[3][2])


def _negative_flux_case(kind):
    """Thick cells with a source in one corner element: the unfixed solution
    dips below zero.  kind selects the kernel family that solves it."""
    if kind in ("trap", "trap1"):  # straight, non-affine (bilinear elements)
        from test_library_host import _trapezoids
        p = 2 if kind == "trap" else 1
        cp, ec = _trapezoids(7, 0.2, seed=4)
        om, wt = P.level_symmetric_2d(4)
        ne = ec.shape[0]
        pr = P.Problem("trap_fix", p, 1, cp, ec, om, wt, np.full(ne, 200.0), np.zeros(ne))
        pr.q_iso = np.zeros((ne, (p + 1) ** 2))
    else:
        p, m, warp = {"p1": (1, 1, 0.0), "p2": (2, 1, 0.0), "p4": (4, 1, 0.0), "curved": (3, 2, 0.06)}[kind]
        pr = _small(7, 7, p, m, 4, st=200.0, warp=warp, q=0.0)
    pr.q_iso[0] = 50.0
    return pr


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("kind", ["p1", "p2", "p4", "trap", "trap1", "curved"])
def test_fixup_parity(torch, precision, kind, schedule):
    """Set-to-zero-and-scale fixup inside the sweep against the oracle's, on
    problems whose unfixed solution is negative somewhere (pipelined kernel
    for affine and bilinear elements with p <= 2 under the direction-resident
    schedule, row-per-lane kernels otherwise, pivoting on the curved mesh)."""
    from paper_2301_04758_amd import vef
    pr = _negative_flux_case(kind)
    ref = O.sweep(pr, fixup=True)
    assert O.sweep(pr)["psi"].min() < 0  # the case needs the fixup
    print("fixup", kind, precision, schedule, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule=schedule, fixup=True)
    io = sw.buffers(n_iter=1)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    psi = io[0]["psi_out"].double().cpu().numpy()
    kernel = sw.info[0]["kernel"]
    sw.close()
    if schedule == "dir" and kind in ("p1", "p2", "trap", "trap1"):
        assert kernel == (vef.VEF_KERNEL_BILINEAR_PIPELINE if kind.startswith("trap")
                          else vef.VEF_KERNEL_AFFINE_PIPELINE)
    assert psi.min() >= 0.0
    assert rel_inf(psi, ref["psi"]) <= TOL[precision]


@pytest.mark.parametrize("schedule", SCHEDULES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_fixup_noop_without_negative_values(torch, precision, schedule):
    (pr,), _ = P.make_config("c1")
    (a,), _ = gpu_run(torch, [pr], precision, schedule=schedule)
    assert a["psi_out"].min() >= 0
    from paper_2301_04758_amd import vef
    sw = vef.Sweep([pr], precision=precision, schedule=schedule, fixup=True)
    io = sw.buffers(n_iter=1)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    assert np.array_equal(io[0]["psi_out"].cpu().numpy(), a["psi_out"])
    sw.close()
