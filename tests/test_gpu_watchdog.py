"""The bounded device-side waits of the pipelined sweep, forced to expire from
the host (vef_options.wait_polls = 1 poll): the kernel's own wait gives up,
every wave leaves the kernel normally, vef_sweep_check reports
VEF_ERR_TIMEOUT, the status word is cleared by the next run, and a handle with
the default bound on the same device still matches the oracle afterwards."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_04758_amd import problems as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def test_wait_bound_gives_timeout_status(torch):
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c2")
    print("watchdog: c2 pipelined kernel with a 1-poll wait bound", flush=True)
    sw = vef.Sweep([pr], precision="fp64", schedule="dir", wait_polls=1)
    assert sw.info[0]["kernel"] == vef.VEF_KERNEL_AFFINE_PIPELINE
    io = sw.buffers(n_iter=2)
    for _ in range(2):  # the status word is set again by each run that times out
        sw.run(io, n_iter=2)
        torch.cuda.synchronize()
        with pytest.raises(vef.VefError) as e:
            sw.check()
        assert e.value.code == vef.VEF_ERR_TIMEOUT
    sw.close()
    # the device is healthy: a default handle sweeps C1 to oracle parity, and
    # its status is clean
    (c1,), _ = P.make_config("c1")
    sw = vef.Sweep([c1], precision="fp64")
    io = sw.buffers(n_iter=1)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    ref = O.sweep(c1)
    got = io[0]["psi_out"].cpu().numpy()
    assert np.abs(got - ref["psi"]).max() <= 1e-12 * np.abs(ref["psi"]).max()
    sw.close()


def test_status_cleared_by_next_run(torch):
    """A run that times out, then an ordinary run on a handle with the
    default bound: each run's status reflects that run only."""
    from paper_2301_04758_amd import vef
    (pr,), _ = P.make_config("c2", scale=16)
    bad = vef.Sweep([pr], precision="fp64", schedule="dir", wait_polls=1)
    io = bad.buffers(n_iter=1)
    bad.run(io, n_iter=1)
    torch.cuda.synchronize()
    with pytest.raises(vef.VefError):
        bad.check()
    bad.close()
    good = vef.Sweep([pr], precision="fp64", schedule="dir")
    io = good.buffers(n_iter=1)
    good.run(io, n_iter=1)
    torch.cuda.synchronize()
    good.check()
    good.close()
