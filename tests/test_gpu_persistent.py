"""The persistent schedule (VEF_PERSISTENT: one launch per sweep and kernel
variant, tasks in upwind-level order on every resident wave, dependency
counters in global memory) against the level-synchronous schedule, which runs
the same per-solve arithmetic one launch per level: equal bit for bit, so a
missing wait or a stale read of an upwind flux would show.  Also the
device-side stop, a cyclic mesh with lagged couplings, a batch of problems of
different degrees, graph capture, and the bounded wait forced to expire from
the host."""
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


def _run(torch, probs, precision, schedule, n_iter=2, tol=0.0, lag=False):
    from paper_2301_04758_amd import vef
    print("persistent-test run", [p.name for p in probs][:3], precision, schedule, n_iter, flush=True)
    sw = vef.Sweep(probs, precision=precision, schedule=schedule, lag_cycles=lag)
    io = sw.buffers(n_iter=n_iter, store_psi=True)
    iters = torch.zeros(1, dtype=torch.int32, device="cuda")
    sw.run(io, n_iter=n_iter, tol=tol, iters_done=iters)
    torch.cuda.synchronize()
    sw.check()
    out = [{k: v.cpu().numpy() for k, v in b.items() if v is not None and hasattr(v, "cpu")} for b in io]
    info = sw.info
    sw.close()
    return out, int(iters.item()), info


def _equal(a, b):
    for x, y in zip(a, b):
        for key in ("psi_out", "mom", "resid"):
            assert np.array_equal(x[key], y[key]), key


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("cfg,scale", [("c3", 24), ("c5", 40), ("c3", 7), ("c5", 3)])
def test_persistent_equals_level(torch, precision, cfg, scale):
    (pr,), _ = P.make_config(cfg, scale=scale)
    a, _, _ = _run(torch, [pr], precision, "level")
    b, _, info = _run(torch, [pr], precision, "persistent")
    assert info[0]["schedule"] == 3
    _equal(a, b)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_persistent_batch_of_degrees(torch, precision):
    """Problems of degree 1 to 4 in one handle: the degree 3 and 4 ones run
    persistent launches, the others level-synchronous ones."""
    probs, _ = P.make_config("c4", scale=20)
    a, _, _ = _run(torch, probs[:12], precision, "level")
    b, _, _ = _run(torch, probs[:12], precision, "persistent")
    _equal(a, b)


def test_persistent_stop_rule(torch):
    (pr,), _ = P.make_config("c3", scale=16)
    a, _, _ = _run(torch, [pr], "fp64", "level", n_iter=6)
    tol = float(np.sqrt(a[0]["resid"][2] * a[0]["resid"][3]))
    b, it_l, _ = _run(torch, [pr], "fp64", "level", n_iter=6, tol=tol)
    c, it_p, _ = _run(torch, [pr], "fp64", "persistent", n_iter=6, tol=tol)
    assert it_l == it_p == 4
    _equal(b, c)


def test_persistent_lagged_cycles(torch):
    """A mesh with re-entrant faces swept with lagged couplings: a lagged read
    must see the previous sweep, which the level order of the plan guarantees
    in both schedules."""
    pr = P.reentrant_quads(24)
    a, _, _ = _run(torch, [pr], "fp64", "level", n_iter=3, lag=True)
    b, _, _ = _run(torch, [pr], "fp64", "persistent", n_iter=3, lag=True)
    _equal(a, b)


def test_persistent_graph_replays(torch):
    """A captured persistent run replayed several times, with eager work in
    between, equals the eager run each time."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c5", scale=24)
    sw = vef.Sweep([pr], precision="fp64", schedule="persistent")
    io = sw.buffers(n_iter=2, store_psi=True)
    sw.run(io, n_iter=2)
    torch.cuda.synchronize()
    ref = io[0]["mom"].cpu().numpy()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        sw.run(io, n_iter=2, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            sw.run(io, n_iter=2, stream=s)
    for _ in range(3):
        io[0]["mom"].zero_()
        g.replay()
        torch.cuda.synchronize()
        sw.check()
        assert np.array_equal(io[0]["mom"].cpu().numpy(), ref)
        sw.run(io, n_iter=2)  # eager work between replays
        torch.cuda.synchronize()
    del g
    sw.close()


def test_persistent_wait_bound_gives_timeout(torch):
    """wait_polls = 1: the first dependency wait that is not met at once gives
    up; every wave leaves the kernel, the run reports VEF_ERR_TIMEOUT, and a
    default handle afterwards matches the level-synchronous result."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c3", scale=12)
    sw = vef.Sweep([pr], precision="fp64", schedule="persistent", wait_polls=1)
    io = sw.buffers(n_iter=1)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    with pytest.raises(vef.VefError) as e:
        sw.check()
    assert e.value.code == vef.VEF_ERR_TIMEOUT
    sw.close()
    a, _, _ = _run(torch, [pr], "fp64", "level", n_iter=1)
    b, _, _ = _run(torch, [pr], "fp64", "persistent", n_iter=1)
    _equal(a, b)
