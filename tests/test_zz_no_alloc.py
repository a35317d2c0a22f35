"""vef_sweep_run_static (the run entry point that allocates nothing) against
vef_sweep_run, through the C ABI: identical moments, angular flux and
stop-test iteration counts on two calls in a row, the second on a smaller
problem; and its argument checks (no internal angular flux yet, residuals
beyond the static array)."""
import numpy as np
import pytest

from paper_2301_04758_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def _problem(side, p, n_sn, seed):
    rng = np.random.Generator(np.random.PCG64(P.SEED_BASE + seed))
    pr = P.make_problem("static_%d" % side, side, side, p, 1, n_sn, 1.0, 0.9)
    pr.sigma_t = P.block_log_uniform(side, side, min(8, side), 0.1, 100.0, rng)
    pr.sigma_s = 0.9 * pr.sigma_t
    return pr


def _run(torch, pr, n_iter, tol, static):
    from paper_2301_04758_amd import vef
    print("static-run case", pr.name, "n_iter", n_iter, "tol", tol, "static", static, flush=True)
    sw = vef.Sweep([pr], precision="fp64")
    io = sw.buffers(n_iter=n_iter, store_psi=True)
    io[0]["resid"] = None  # residuals in library memory: the static array for the static run
    iters = torch.zeros(1, dtype=torch.int32, device="cuda")
    fn = vef.vef_sweep_run_static if static else vef.vef_sweep_run
    fn(sw.h, io, n_iter, tol, iters)
    torch.cuda.synchronize()
    sw.check()
    out = dict(mom=io[0]["mom"].cpu().numpy(), psi=io[0]["psi_out"].cpu().numpy(), iters=int(iters.item()))
    sw.close()
    return out


def _tol_stopping_early(torch, pr, n_iter):
    """A tolerance between two residuals of the history, so that the
    device-side stop test (which reads the residual array) ends the run early."""
    from paper_2301_04758_amd import vef
    sw = vef.Sweep([pr], precision="fp64")
    io = sw.buffers(n_iter=n_iter, store_psi=False)
    sw.run(io, n_iter=n_iter)
    torch.cuda.synchronize()
    r = io[0]["resid"].cpu().numpy()
    sw.close()
    k = n_iter // 2
    return float(np.sqrt(r[k] * r[k - 1]))


def test_static_run_equals_run_two_calls(torch):
    big = _problem(32, 2, 8, 21)
    small = _problem(8, 1, 4, 22)
    cases = [(big, 12), (small, 5)]
    tols = [_tol_stopping_early(torch, pr, n) for pr, n in cases]
    # two static calls in a row (the second on the smaller problem), then the
    # reference entry point on the same inputs
    got = [_run(torch, pr, n, tol, True) for (pr, n), tol in zip(cases, tols)]
    ref = [_run(torch, pr, n, tol, False) for (pr, n), tol in zip(cases, tols)]
    for (pr, n), g, r in zip(cases, got, ref):
        assert g["iters"] == r["iters"] and 1 <= r["iters"] < n, (g["iters"], r["iters"])
        # same kernels on the same inputs: equal bit for bit
        assert np.array_equal(g["mom"], r["mom"])
        assert np.array_equal(g["psi"], r["psi"])


def test_static_run_argument_checks(torch):
    from paper_2301_04758_amd import vef
    pr = _problem(8, 1, 4, 23)
    sw = vef.Sweep([pr], precision="fp64")
    io = sw.buffers(n_iter=1, store_psi=False)
    io[0]["resid"] = None
    # no caller angular flux and none held by the handle yet
    with pytest.raises(vef.VefError) as e:
        vef.vef_sweep_run_static(sw.h, io, 1)
    assert e.value.code == vef.VEF_ERR_INVALID
    # an ordinary run with psi_out NULL gives the handle its own angular flux,
    # after which the static run accepts psi_out NULL
    sw.run(io, n_iter=1)
    vef.vef_sweep_run_static(sw.h, io, 1)
    torch.cuda.synchronize()
    sw.check()
    phi = io[0]["mom"][0].cpu().numpy()
    assert np.isfinite(phi).all() and phi.max() > 0
    # residuals beyond the static array
    io2 = sw.buffers(n_iter=1, store_psi=True)
    io2[0]["resid"] = None
    with pytest.raises(vef.VefError) as e:
        vef.vef_sweep_run_static(sw.h, io2, vef.VEF_STATIC_RESID_MAX + 1)
    assert e.value.code == vef.VEF_ERR_INVALID
    sw.close()
