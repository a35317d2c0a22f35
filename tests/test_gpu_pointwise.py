"""GPU parity of pointwise upwinding (vef_options.upwind = VEF_UPWIND_POINT,
with lagged sweeps for the faces whose points have both signs) against the
oracle with the same rule, on curved Taylor-Green meshes.  Bound: the bar
(1e-12 FP64, 1e-5 FP32-local) or 4 eps kappa_max where the local systems
are ill-conditioned (kappa_max from the diagonal blocks of the independent
dense pointwise system)."""
import math

import numpy as np
import pytest

import dg_numpy as D
import mms
from oracle import oracle as O
from paper_2301_04758_amd import problems as P

pytestmark = pytest.mark.gpu

BAR = {"fp64": 1e-12, "fp32": 1e-5}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _tg(n, m, p, N=4, st=2.0, c=0.0):
    cp, ec = P.taylor_green_mesh(n, m, t_final=0.3 * math.pi)
    om, wt = P.level_symmetric_2d(N)
    ne = ec.shape[0]
    sig = np.random.default_rng(n + 10 * m).uniform(0.5 * st, 2 * st, ne)
    pr = P.Problem("tg_%dx%d_m%d_p%d" % (n, n, m, p), p, m, cp, ec, om, wt, sig, c * sig, nx=n, ny=n)
    pr.q_iso = np.ones((ne, (p + 1) ** 2))
    return pr


def _tol(pr, precision):
    """The stated bar against the oracle (1e-5) for FP32-local; for FP64 the
    bar or 4 eps kappa_max of the local blocks, whichever is larger (two
    backward-stable double solves differ by a few eps kappa)."""
    if precision == "fp32":
        return BAR[precision]
    k = 0.0
    n = (pr.p + 1) ** 2
    for d in range(pr.n_dir):
        A, _ = D.global_system(pr, d, pointwise=True)
        for e in range(pr.n_elem):
            k = max(k, np.linalg.cond(A[e * n:(e + 1) * n, e * n:(e + 1) * n]))
    eps = np.finfo(np.float64 if precision == "fp64" else np.float32).eps
    return max(BAR[precision], 4 * eps * k)


def _rel(x, ref):
    return float(np.abs(x - ref).max() / np.abs(ref).max())


def _gpu(torch, pr, precision, schedule, n_iter):
    from paper_2301_04758_amd import vef
    print("pointwise run", pr.name, precision, schedule, n_iter, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule=schedule, lag_cycles=True, pointwise=True)
    try:
        assert sw.info[0]["n_lagged"] > 0
        io = sw.buffers(n_iter=n_iter, store_psi=True)
        sw.run(io, n_iter=n_iter)
        torch.cuda.synchronize()
        sw.check()
        return {k: v.cpu().numpy() for k, v in io[0].items() if v is not None and hasattr(v, "cpu")}
    finally:
        sw.close()


@pytest.mark.parametrize("schedule", ["level", "dir"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n,m,p", [(3, 2, 1), (4, 2, 2), (4, 3, 2), (3, 3, 3)])
def test_pointwise_lagged_sweep(torch, precision, schedule, n, m, p):
    """One sweep from zero (lagged reads see zero) and three source
    iterations with scattering."""
    pr = _tg(n, m, p, c=0.5)
    tol = _tol(pr, precision)
    g = _gpu(torch, pr, precision, schedule, 1)
    ref = O.sweep(pr, lag=True, pointwise=True)
    e1 = _rel(g["psi_out"], ref["psi"])
    g3 = _gpu(torch, pr, precision, schedule, 3)
    ref3 = O.source_iteration(pr, 3, lag=True, pointwise=True)
    e3 = _rel(g3["mom"][0], ref3["mom"][0])
    print("sweep %.2e, 3 iterations %.2e (bound %.1e)" % (e1, e3, tol), flush=True)
    assert e1 <= tol and e3 <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_pointwise_inflow_data_and_directional_source(torch, precision):
    pr = _tg(4, 2, 2)
    pr.q_iso = None
    vxy, bxy, _ = O.qp_coords(pr)
    mms.attach(pr, vxy, bxy)
    tol = _tol(pr, precision)
    g = _gpu(torch, pr, precision, "dir", 1)
    ref = O.sweep(pr, lag=True, pointwise=True)
    assert _rel(g["psi_out"], ref["psi"]) <= tol
