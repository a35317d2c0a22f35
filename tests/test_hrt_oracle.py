"""Pins of the HRT element-local oracle (oracle/hrt_oracle.py) against what
the mathematics fixes, independent of the oracle's own formulas:

  * nodal RT_p basis: interpolation property; the divergence maps onto Q_p;
  * divergence theorem per basis function (volume D against face fluxes);
  * E = I/3 gives G = -D^T / 3 (grad v : I = div v), on sheared elements;
  * the RT mass at nq = p + 2 equals a higher-order rule (exact on affine
    elements), and is symmetric positive definite;
  * the boundary term through the reference normal component (the Piola
    transform preserves v . n ds), for E = I/3;
  * local exactness: for a constant Eddington tensor E0 (isotropic and
    anisotropic), a linear phi and the constant current -E0 grad phi /
    sigma_t solve the element-local problem with lambda = phi on every face,
    so the inverse maps the right-hand side back to them;
  * the block formulas of Sec. 7 for W, X, Y, Z equal the blocks of the
    plain inverse;
  * E from moments of an isotropic flux is I/3.
"""
import numpy as np
import pytest

from oracle import hrt_oracle as H
from oracle import oracle as O
from paper_2301_04758_amd import problems as P

RNG = np.random.default_rng(77)


def _sheared(nx, ny, p, shear=0.35, stretch=1.7, st=1.0, ss=0.4, m=1, seed=0):
    """Parallelogram mesh: the unit-square grid mapped by a fixed linear map."""
    cp, ec = P.quad_mesh(nx, ny, m)
    Mlin = np.array([[stretch, shear], [0.2, 1.0]])
    cp = cp @ Mlin.T + np.array([3.0, -1.0])
    om, wt = P.level_symmetric_2d(4)
    ne = ec.shape[0]
    rng = np.random.default_rng(seed)
    sig_t = rng.uniform(0.5, 3.0, ne) * st
    pr = P.Problem("sheared", p, m, cp, ec, om, wt, sig_t, ss * sig_t, nx=nx, ny=ny)
    return pr


def _iso(ne, npt):
    E = np.zeros((ne, npt, 2, 2))
    E[..., 0, 0] = E[..., 1, 1] = 1.0 / 3.0
    return E


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rt_basis_nodal_and_divergence(p):
    lob, leg = O.gl_nodes(p + 1), H.legendre_points(p + 1)
    X, Y = np.meshgrid(lob, leg, indexing="xy")
    vx, _ = H.rt_basis(p, X.ravel(), Y.ravel())
    nx = (p + 2) * (p + 1)
    assert np.allclose(vx[:, :nx, 0], np.eye(nx), atol=1e-13) and np.allclose(vx[:, :nx, 1], 0, atol=1e-13)
    X, Y = np.meshgrid(leg, lob, indexing="xy")
    vy, _ = H.rt_basis(p, X.ravel(), Y.ravel())
    assert np.allclose(vy[:, nx:, 1], np.eye(nx), atol=1e-13) and np.allclose(vy[:, nx:, 0], 0, atol=1e-13)
    pr = _sheared(1, 1, p)
    blk = H.local_blocks(pr, p + 2, _iso(1, (p + 2) ** 2))
    assert np.linalg.matrix_rank(blk["D"][0]) == (p + 1) ** 2  # div maps onto Q_p


@pytest.mark.parametrize("p", [1, 2, 3])
def test_divergence_theorem(p):
    pr = _sheared(2, 1, p)
    nq = p + 2
    blk = H.local_blocks(pr, nq, _iso(pr.n_elem, nq * nq))
    x0, F = H.affine_frames(pr)
    gx, gw = O.gauss_rule(nq)
    for e in range(pr.n_elem):
        J = np.linalg.det(F[e])
        flux = np.zeros(blk["A"].shape[1])
        for f in range(4):
            fx, fy = H.face_points(f, gx)
            vb, _ = H.rt_basis(p, fx, fy)
            v = np.einsum("kl,qil->qik", F[e], vb) / J
            tang = {0: F[e][:, 0], 1: F[e][:, 1], 2: -F[e][:, 0], 3: -F[e][:, 1]}[f]
            nds = np.array([tang[1], -tang[0]])
            flux += np.einsum("q,qik,k->i", gw, v, nds)
        ones = np.ones((p + 1) ** 2)  # the nodal phi basis sums to one
        assert np.allclose(ones @ blk["D"][e], flux, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_isotropic_G_is_minus_D_transpose_over_three(p):
    pr = _sheared(2, 2, p)
    nq = p + 2
    blk = H.local_blocks(pr, nq, _iso(pr.n_elem, nq * nq))
    assert np.allclose(blk["G"], -np.transpose(blk["D"], (0, 2, 1)) / 3.0, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_rt_mass_exact_and_spd(p):
    pr = _sheared(2, 2, p)
    a = H.local_blocks(pr, p + 2, _iso(pr.n_elem, (p + 2) ** 2))["A"]
    b = H.local_blocks(pr, p + 5, _iso(pr.n_elem, (p + 5) ** 2))["A"]
    assert np.allclose(a, b, rtol=1e-13, atol=1e-14)
    assert np.allclose(a, np.transpose(a, (0, 2, 1)), atol=1e-14)
    assert (np.linalg.eigvalsh(a) > 0).all()


@pytest.mark.parametrize("p", [1, 2])
def test_boundary_term_through_reference_normals(p):
    """With E = I/3 and E_b = 1/2 the boundary term is (2/3) int (v.n)(J.n) ds;
    v . n ds = v_hat . n_hat ds_hat, so on face f with chord length |N_f| it
    is (2/3) sum_q w_q (vh_i . nh)(vh_j . nh) / |N_f|."""
    pr = _sheared(2, 2, p)
    nq = p + 2
    bf = O.boundary_faces(pr)
    E_b = np.full((len(bf), nq), 0.5)
    E_bnd = _iso(len(bf), nq)
    with_b = H.local_blocks(pr, nq, _iso(pr.n_elem, nq * nq), E_bnd, E_b)["A"]
    without = H.local_blocks(pr, nq, _iso(pr.n_elem, nq * nq))["A"]
    x0, F = H.affine_frames(pr)
    gx, gw = O.gauss_rule(nq)
    ref_n = {0: (0, -1), 1: (1, 0), 2: (0, 1), 3: (-1, 0)}
    want = without.copy()
    for e, f in bf:
        fx, fy = H.face_points(f, gx)
        vb, _ = H.rt_basis(p, fx, fy)
        vn = vb @ np.array(ref_n[f], dtype=float)
        tang = {0: F[e][:, 0], 1: F[e][:, 1], 2: -F[e][:, 0], 3: -F[e][:, 1]}[f]
        want[e] += (2.0 / 3.0) * np.einsum("q,qi,qj->ij", gw, vn, vn) / np.hypot(*tang)
    assert np.allclose(with_b, want, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("E0", [((1 / 3, 0.0), (0.0, 1 / 3)), ((0.5, 0.12), (0.12, 0.25))])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_local_problem_reproduces_linear_solution(p, E0):
    """Constant Eddington tensor E0, phi = c0 + c . x, J = -E0 c / sigma_t:
    the first moment equation div(E0 phi) + sigma_t J = Q1 holds with Q1 = 0
    and the zeroth with Q0 = sigma_a phi.  With lambda = phi on every face
    (numerical flux E0 n lambda) the element-local system is satisfied by the
    interpolants, so [J; phi] = inv [-C2 lambda; f].  With E0 not a multiple
    of I this pins the Piola gradient (only its trace enters for I/3)."""
    E0 = np.array(E0)
    pr = _sheared(1, 1, p)
    nq = p + 2
    E = np.broadcast_to(E0, (1, nq * nq, 2, 2)).copy()
    blk = H.local_blocks(pr, nq, E)
    inv = np.linalg.inv(H.assemble_full(blk))[0]
    x0, F = H.affine_frames(pr)
    x0, F = x0[0], F[0]
    J = np.linalg.det(F)
    st, sa = pr.sigma_t[0], pr.sigma_t[0] - pr.sigma_s[0]
    c0, c = 0.7, np.array([0.3, -0.45])
    Jex = -E0 @ c / st
    phi_ex = lambda x: c0 + x @ c  # noqa: E731
    gx, gw = O.gauss_rule(nq)
    # right-hand side: -C2 lambda (every face) and f = int u sigma_a phi
    rhs_v = np.zeros(blk["A"].shape[1])
    for f in range(4):
        fx, fy = H.face_points(f, gx)
        vb, _ = H.rt_basis(p, fx, fy)
        v = np.einsum("kl,qil->qik", F, vb) / J
        tang = {0: F[:, 0], 1: F[:, 1], 2: -F[:, 0], 3: -F[:, 1]}[f]
        nds = np.array([tang[1], -tang[0]])
        xq = x0 + np.stack([fx, fy], 1) @ F.T
        rhs_v -= np.einsum("q,qik,k,q->i", gw, v, E0 @ nds, phi_ex(xq))
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    xi, eta = XI.ravel(), ETA.ravel()
    W = np.outer(gw, gw).ravel()
    u = H.phi_basis(p, xi, eta)
    xq = x0 + np.stack([xi, eta], 1) @ F.T
    rhs_u = np.einsum("q,qi,q->i", W * J * sa, u, phi_ex(xq))
    sol = inv @ np.concatenate([rhs_v, rhs_u])
    # interpolants: RT dofs are components of v_hat = J F^{-1} J_ex at the nodes
    vhat = J * np.linalg.solve(F, Jex)
    nx = (p + 2) * (p + 1)
    want_J = np.concatenate([np.full(nx, vhat[0]), np.full(nx, vhat[1])])
    leg = H.legendre_points(p + 1)
    LX, LY = np.meshgrid(leg, leg, indexing="xy")
    want_phi = phi_ex(x0 + np.stack([LX.ravel(), LY.ravel()], 1) @ F.T)
    assert np.allclose(sol[:2 * nx], want_J, rtol=1e-12, atol=1e-13)
    assert np.allclose(sol[2 * nx:], want_phi, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("p", [1, 2])
def test_block_formulas_equal_the_inverse(p):
    pr = _sheared(2, 2, p)
    nq = p + 2
    E = _iso(pr.n_elem, nq * nq)
    E[..., 0, 1] = E[..., 1, 0] = RNG.uniform(-0.1, 0.1, E.shape[:2])
    E[..., 0, 0] += RNG.uniform(0, 0.2, E.shape[:2])
    blk = H.local_blocks(pr, nq, E)
    inv = np.linalg.inv(H.assemble_full(blk))
    W, X, Y, Z = H.schur_blocks(blk)
    nv = blk["A"].shape[1]
    for got, want in ((W, inv[:, :nv, :nv]), (X, inv[:, :nv, nv:]), (Y, inv[:, nv:, :nv]), (Z, inv[:, nv:, nv:])):
        assert np.allclose(got, want, rtol=1e-11, atol=1e-12 * np.abs(inv).max())


def test_eddington_of_an_isotropic_flux_is_a_third():
    pr = _sheared(2, 2, 2)
    n = 9
    mom = np.zeros((6, pr.n_elem, n))
    mom[0] = RNG.uniform(1.0, 2.0, (pr.n_elem, n))
    mom[3] = mom[5] = mom[0] / 3.0
    gx, _ = O.gauss_rule(4)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    E = H.eddington_from_moments(pr, mom, XI.ravel(), ETA.ravel())
    assert np.allclose(E[..., 0, 0], 1 / 3, rtol=1e-14) and np.allclose(E[..., 0, 1], 0, atol=1e-15)
    mom[0, 0] = -1.0  # non-positive phi: isotropic fallback
    E = H.eddington_from_moments(pr, mom, XI.ravel(), ETA.ravel())
    assert np.allclose(E[0, :, 0, 0], 1 / 3) and np.allclose(E[0, :, 1, 1], 1 / 3)


def test_non_affine_rejected():
    cp, ec = P.quad_mesh(2, 2, 1)
    cp = cp.copy()
    cp[4] += [0.05, 0.02]
    om, wt = P.level_symmetric_2d(2)
    pr = P.Problem("t", 1, 1, cp, ec, om, wt, np.ones(4), np.zeros(4))
    with pytest.raises(ValueError):
        H.affine_frames(pr)
