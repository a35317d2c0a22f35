"""Curved elements of degree 3 solved from precomputed element matrices.

The element matrices (mass, the two streaming matrices, the face matrices
weighted by each normal component) are formed once per handle on the matrix
cores; every local system is then assembled from them.  Checked here against
the oracle and against the quadrature-assembly kernel (elem_matrices=False)
on the same inputs, in every schedule and precision, with the paths that
read more than the matrices: the direction-dependent source at the volume
points, inflow data on boundary faces, a scalar flux input, the fixup, and
uncertified solves that pivot.
"""
import numpy as np
import pytest

import mms
from oracle import oracle as O
from paper_2301_04758_amd import problems as P
from test_gpu_parity import TOL, _negative_flux_case, _small, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    if not T.cuda.is_available():
        pytest.skip("no GPU")
    return T


def _run(torch, pr, precision, schedule, elem_matrices, phi=None, fixup=False, n_iter=1):
    from paper_2301_04758_amd import vef
    print("elem_mat run", pr.name, precision, schedule, "elem_matrices", elem_matrices, "fixup", fixup, flush=True)
    sw = vef.Sweep([pr], precision=precision, schedule=schedule, elem_matrices=elem_matrices, fixup=fixup)
    io = sw.buffers(n_iter=n_iter, phi_in=phi)
    sw.run(io, n_iter=n_iter)
    torch.cuda.synchronize()
    sw.check()
    out = dict(psi=io[0]["psi_out"].double().cpu().numpy(), mom=io[0]["mom"].cpu().numpy(),
               kernel=vef.KERNEL_NAMES[sw.info[0]["kernel"]])
    sw.close()
    return out


def _curved_case(seed=3, with_mms=True):
    pr = _small(9, 7, 3, 2, 6, st=lambda r, n: r.uniform(0.2, 20.0, n), ss=lambda r, n: r.uniform(0.0, 0.1, n),
                warp=0.07, seed=seed)
    if with_mms:
        pr.q_iso = None
        vxy, bxy, _ = O.qp_coords(pr)
        mms.attach(pr, vxy, bxy)  # direction-dependent volume source and boundary inflow data
    rng = np.random.default_rng(seed)
    phi = rng.uniform(0.0, 2.0, (pr.n_elem, 16))
    return pr, phi


@pytest.mark.parametrize("schedule", ["level", "dir", "persistent"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_elem_matrices_match_oracle_and_quadrature(torch, precision, schedule):
    pr, phi = _curved_case()
    ref = O.sweep(pr, phi_in=phi)
    a = _run(torch, pr, precision, schedule, True, phi)
    b = _run(torch, pr, precision, schedule, False, phi)
    assert a["kernel"] == "general_mat"
    assert b["kernel"] in ("pivot", "nopivot")
    tol = TOL[precision]
    assert rel_inf(a["psi"], ref["psi"]) <= tol
    assert rel_inf(b["psi"], ref["psi"]) <= tol
    for k in range(6):
        assert rel_inf(a["mom"][k], ref["mom"][k], np.abs(ref["mom"][0]).max()) <= tol
    # the two assemblies are the same sums in another order
    assert rel_inf(a["psi"], b["psi"]) <= (1e-13 if precision == "fp64" else 2e-6)


@pytest.mark.parametrize("fixup", [False, True])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_elem_matrices_uncertified_solves(torch, precision, fixup):
    """A strongly warped mesh where about one solve in 19 is not certified
    for elimination in natural order.  The level-synchronous kernel takes
    those rows in the order of partial pivoting formed when the handle is
    created and eliminates in natural order; the direction-resident and
    persistent kernels pivot during the solve; the quadrature kernel
    assembles without the matrices.  All against the oracle, and the two
    eliminations against each other."""
    from paper_2301_04758_amd import vef
    pr = _small(9, 7, 3, 2, 6, st=lambda r, n: r.uniform(0.2, 20.0, n), ss=lambda r, n: r.uniform(0.0, 0.1, n),
                warp=0.15, seed=5)
    if fixup:
        pr.q_iso = np.zeros_like(pr.q_iso)
        pr.q_iso[0] = 50.0
        pr.sigma_t = pr.sigma_t * 20.0
    else:
        pr.q_iso = None
        vxy, bxy, _ = O.qp_coords(pr)
        mms.attach(pr, vxy, bxy)
    assert vef.vef_plan_query(pr)["n_pivoting"] == 80
    ref = O.sweep(pr, fixup=fixup)
    lvl = _run(torch, pr, precision, "level", True, fixup=fixup)
    dr = _run(torch, pr, precision, "dir", True, fixup=fixup)
    per = _run(torch, pr, precision, "persistent", True, fixup=fixup)
    quad = _run(torch, pr, precision, "level", False, fixup=fixup)
    assert lvl["kernel"] == dr["kernel"] == per["kernel"] == "general_mat"
    tol = TOL[precision]
    for out in (lvl, dr, per, quad):
        assert rel_inf(out["psi"], ref["psi"]) <= tol
    if fixup:
        assert lvl["psi"].min() >= 0.0
    assert rel_inf(lvl["psi"], dr["psi"]) <= (1e-13 if precision == "fp64" else 2e-6)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_elem_matrices_source_iteration(torch, precision):
    """Three source iterations with scattering (the nodal source from the
    previous iterate goes through M)."""
    pr, _ = _curved_case(seed=8, with_mms=False)
    pr.sigma_s = 0.9 * pr.sigma_t
    ref = O.source_iteration(pr, 3)
    a = _run(torch, pr, precision, "level", True, n_iter=3)
    assert a["kernel"] == "general_mat"
    assert rel_inf(a["mom"][0], ref["mom"][0]) <= TOL[precision]


@pytest.mark.parametrize("schedule", ["level", "dir"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_elem_matrices_fixup(torch, precision, schedule):
    """The fixup's balance weights from the matrices: sigma_t times a row sum
    of M plus the outflow face rows."""
    pr = _negative_flux_case("curved")
    ref = O.sweep(pr, fixup=True)
    a = _run(torch, pr, precision, schedule, True, fixup=True)
    assert a["kernel"] == "general_mat"
    assert a["psi"].min() >= 0.0
    assert rel_inf(a["psi"], ref["psi"]) <= TOL[precision]


def test_elem_matrices_only_where_they_apply(torch):
    """Degree 3 on general elements only: affine meshes keep the row-set LU,
    other degrees the quadrature kernels, and pointwise upwinding the
    quadrature kernel (its face terms change sign inside a face)."""
    from paper_2301_04758_amd import vef
    cases = [(_small(4, 4, 3, 1, 4), {}, "affine_lu"), (_small(4, 4, 2, 2, 4, warp=0.05), {}, None),
             (_small(4, 4, 3, 2, 4, warp=0.05), {"pointwise": True, "lag_cycles": True}, None),
             (_small(4, 4, 3, 2, 4, warp=0.05), {}, "general_mat")]
    for pr, kw, want in cases:
        sw = vef.Sweep([pr], precision="fp64", **kw)
        got = vef.KERNEL_NAMES[sw.info[0]["kernel"]]
        sw.close()
        if want is None:
            assert got != "general_mat", pr.name
        else:
            assert got == want, pr.name


def test_c3_sized_elem_matrices_agree_with_fixture(torch):
    """The 256 x 256 curved configuration on the element-matrix kernel (its
    default) against the oracle fixture, FP64, one sweep."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "c3_full.json")
    g = json.load(open(path))
    (pr,), _ = P.make_config("c3")
    a = _run(torch, pr, "fp64", "level", True)
    assert a["kernel"] == "general_mat"
    idx = np.asarray(g["index"])
    flat = a["mom"].reshape(6, -1)
    scale = g["mom_absmax"][0]
    for k in range(6):
        assert np.abs(flat[k, idx] - np.asarray(g["mom"][k])).max() / scale <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_autotune_weighs_element_matrices_against_quadrature(torch, precision):
    """The autotuner times every schedule with the element-matrix kernel and
    with the quadrature kernel; the handle then runs what it reports, and
    stays at the bar against the oracle."""
    from paper_2301_04758_amd import vef
    pr, phi = _curved_case(seed=5)
    ref = O.sweep(pr, phi_in=phi)
    print("autotune elem_mat", precision, flush=True)
    sw = vef.Sweep([pr], precision=precision)
    io = sw.buffers(n_iter=1, phi_in=phi)
    res = sw.autotune(io, n_iter=1, reps=2)
    assert res["elem_matrices"] in (0, 1)
    assert res["n_candidates"] >= 7  # level x 2 blocks, dir, persistent; each with both assemblies
    kernel = vef.KERNEL_NAMES[sw.info[0]["kernel"]]
    assert (kernel == "general_mat") == (res["elem_matrices"] == 1), (kernel, res)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    psi = io[0]["psi_out"].double().cpu().numpy()
    sw.close()
    assert rel_inf(psi, ref["psi"]) <= TOL[precision]
