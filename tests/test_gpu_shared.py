"""Affine elements of degree 3 and 4 whose local matrices repeat (uniform
grids with a few materials): each run forms one matrix per class of
(direction, element) pairs that share their local matrix A, K = A^-1 R with R
the map from a solve's inputs to its right-hand side, and the
level-synchronous sweep computes each local solution as K times the solve's
inputs.  Checked
against the oracle and against the row-set LU (shared_matrices=False) on the
same inputs, with the paths that feed the right-hand side: a scalar flux and
isotropic source, the direction-dependent source and boundary inflow data,
scattering over several source iterations, and the fixup.
"""
import numpy as np
import pytest

import mms
from oracle import oracle as O
from paper_2301_04758_amd import problems as P
from test_gpu_parity import TOL, _small, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def _blocks(n, values):
    """sigma per element of an n x n grid: values cycled over 2 x 2 blocks."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    blk = (i // 2 + (j // 2) * (n // 2)).ravel()
    return np.asarray(values, float)[blk % len(values)]


def _uniform_case(p, N=6, seed=1, with_mms=True):
    """8 x 8 grid of equal squares (an exactly representable spacing), three
    materials; returns the problem and a scalar flux input."""
    st = _blocks(8, [0.7, 4.0, 25.0])
    pr = _small(8, 8, p, 1, N, st=st, ss=0.5 * st, seed=seed)
    if with_mms:
        pr.q_iso = None
        vxy, bxy, _ = O.qp_coords(pr)
        mms.attach(pr, vxy, bxy)
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0, (pr.n_elem, (p + 1) ** 2))
    return pr, phi


def _run(torch, pr, precision, shared, phi=None, n_iter=1, fixup=False, schedule="level"):
    from paper_2301_04758_amd import vef
    print("shared run", pr.name, precision, schedule, "shared", shared, "n_iter", n_iter, "fixup", fixup, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule=schedule, shared_matrices=shared, fixup=fixup)
    io = sw.buffers(n_iter=n_iter, phi_in=phi)
    sw.run(io, n_iter=n_iter)
    torch.cuda.synchronize()
    sw.check()
    out = dict(psi=io[0]["psi_out"].double().cpu().numpy(), mom=io[0]["mom"].cpu().numpy(),
               kernel=vef.KERNEL_NAMES[sw.info[0]["kernel"]], n_classes=sw.info[0]["n_classes"])
    sw.close()
    return out


@pytest.mark.parametrize("p", [3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_matrices_match_oracle_and_lu(torch, precision, p):
    pr, phi = _uniform_case(p)
    ref = O.sweep(pr, phi_in=phi)
    a = _run(torch, pr, precision, True, phi)
    b = _run(torch, pr, precision, False, phi)
    assert a["kernel"] == "affine_shared" and a["n_classes"] == 3 * pr.n_dir
    assert b["kernel"] == "affine_lu" and b["n_classes"] == 0
    tol = TOL[precision]
    assert rel_inf(a["psi"], ref["psi"]) <= tol
    assert rel_inf(b["psi"], ref["psi"]) <= tol
    for k in range(6):
        assert rel_inf(a["mom"][k], ref["mom"][k], np.abs(ref["mom"][0]).max()) <= tol
    # the same systems solved by elimination and by the class matrices
    assert rel_inf(a["psi"], b["psi"]) <= (1e-13 if precision == "fp64" else tol)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_matrices_source_iteration(torch, precision):
    """Four source iterations: the class matrices formed before the first
    sweep serve every sweep of the run."""
    pr, _ = _uniform_case(4, seed=6, with_mms=False)
    pr.sigma_s = 0.95 * pr.sigma_t
    ref = O.source_iteration(pr, 4)
    a = _run(torch, pr, precision, True, n_iter=4)
    assert a["kernel"] == "affine_shared"
    assert rel_inf(a["mom"][0], ref["mom"][0]) <= TOL[precision]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_matrices_fixup(torch, precision):
    """Thick cells with a source in one corner: negative values are zeroed
    and the rest scaled, after the product with the class matrix."""
    pr = _small(8, 8, 4, 1, 4, st=200.0, q=0.0)
    pr.q_iso[0] = 50.0
    ref = O.sweep(pr, fixup=True)
    assert O.sweep(pr)["psi"].min() < 0  # the case needs the fixup
    a = _run(torch, pr, precision, True, fixup=True)
    assert a["kernel"] == "affine_shared" and a["n_classes"] == pr.n_dir
    assert a["psi"].min() >= 0.0
    assert rel_inf(a["psi"], ref["psi"]) <= TOL[precision]


def test_shared_matrices_only_where_they_repeat(torch):
    """sigma_t different on every element gives one class per solve: the
    row-set LU; the direction-resident schedule keeps the row-set LU too."""
    pr = _small(8, 8, 4, 1, 4, st=lambda r, n: r.uniform(0.5, 5.0, n), seed=3)
    a = _run(torch, pr, "fp64", True)
    assert a["kernel"] == "affine_lu" and a["n_classes"] == 0
    pr2, phi = _uniform_case(3, with_mms=False)
    b = _run(torch, pr2, "fp64", True, phi, schedule="dir")
    assert b["kernel"] == "affine_lu" and b["n_classes"] == 3 * pr2.n_dir
    ref = O.sweep(pr2, phi_in=phi)
    assert rel_inf(b["psi"], ref["psi"]) <= TOL["fp64"]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_weighs_shared_matrices_against_lu(torch, precision):
    """The autotuner times the level-synchronous kernels with the class
    matrices and with the row-set LU; the handle then runs what it reports."""
    from paper_2301_04758_amd import vef
    pr, phi = _uniform_case(4, seed=2)
    ref = O.sweep(pr, phi_in=phi)
    print("autotune shared", precision, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule="level")
    io = sw.buffers(n_iter=1, phi_in=phi)
    res = sw.autotune(io, n_iter=1, reps=2)
    assert res["shared_matrices"] in (0, 1)
    assert res["n_candidates"] >= 6  # level x 2 blocks x 2 solvers, dir, persistent
    info = vef.vef_problem_info(sw.h, 0)
    kernel = vef.KERNEL_NAMES[info["kernel"]]
    assert (kernel == "affine_shared") == (res["shared_matrices"] == 1), (kernel, res)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    psi = io[0]["psi_out"].double().cpu().numpy()
    sw.close()
    assert rel_inf(psi, ref["psi"]) <= TOL[precision]


def test_shared_matrices_runs_are_deterministic(torch):
    """Two runs of one handle give the same bits (the class matrices are
    formed again by the second run)."""
    from paper_2301_04758_amd import vef
    pr, phi = _uniform_case(4, seed=9)
    sw = vef.Sweep([pr], precision="fp64", schedule="level")
    outs = []
    for _ in range(2):
        io = sw.buffers(n_iter=2, phi_in=phi)
        sw.run(io, n_iter=2)
        torch.cuda.synchronize()
        sw.check()
        outs.append(io[0]["psi_out"].cpu().numpy().copy())
    sw.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_shared_matrices_graph_replays(torch, precision):
    """A run with class matrices (their formation included) captured in a HIP
    graph: every replay, with eager work on the same buffers in between,
    gives the bits of the eager run."""
    from paper_2301_04758_amd import vef
    pr, phi = _uniform_case(4, seed=4, with_mms=False)
    pr.sigma_s = 0.9 * pr.sigma_t
    print("shared graph capture", precision, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule="level")
    assert vef.KERNEL_NAMES[sw.info[0]["kernel"]] == "affine_shared"
    io = sw.buffers(n_iter=3, phi_in=phi)
    sw.run(io, n_iter=3)
    torch.cuda.synchronize()
    sw.check()
    ref = {k: io[0][k].clone() for k in ("mom", "psi_out", "resid")}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sw.run(io, n_iter=3)
    for rep in range(3):
        io[0]["mom"].fill_(-1.0)  # eager work between replays
        io[0]["psi_out"].zero_()
        io[0]["resid"].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        sw.check()
        for key in ("mom", "psi_out", "resid"):
            assert torch.equal(io[0][key], ref[key]), (rep, key)
    del g
    sw.close()
    assert rel_inf(ref["mom"][0].cpu().numpy(), O.source_iteration(pr, 3, phi0=phi)["mom"][0]) <= TOL[precision]


@pytest.mark.parametrize("p,nq", [(3, 5), (3, 6), (4, 7)])
def test_shared_matrices_more_face_points(torch, p, nq):
    """More quadrature points than face nodes: the class matrix's trace
    block carries padding columns and its boundary-data block more entries
    than a face has nodes; direction-dependent source and inflow data at
    those points (FP64 against the oracle and the row-set LU, FP32 against
    the oracle)."""
    st = _blocks(8, [0.7, 4.0, 25.0])
    pr = _small(8, 8, p, 1, 6, st=st, ss=0.5 * st, seed=11)
    pr.nq = nq
    pr.q_iso = None
    vxy, bxy, _ = O.qp_coords(pr)
    mms.attach(pr, vxy, bxy)
    phi = np.random.default_rng(11).uniform(0.0, 2.0, (pr.n_elem, (p + 1) ** 2))
    ref = O.sweep(pr, phi_in=phi)
    a = _run(torch, pr, "fp64", True, phi)
    b = _run(torch, pr, "fp64", False, phi)
    c = _run(torch, pr, "fp32", True, phi)
    assert a["kernel"] == "affine_shared" and c["kernel"] == "affine_shared"
    assert rel_inf(a["psi"], ref["psi"]) <= TOL["fp64"]
    assert rel_inf(a["psi"], b["psi"]) <= 1e-13
    assert rel_inf(c["psi"], ref["psi"]) <= TOL["fp32"]
