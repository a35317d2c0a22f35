"""Pins of the oracle's hybridized-RT VEF global solve and outer iteration
(oracle/vef_outer_oracle.py):

  * exactness: with a constant Eddington tensor E0 (isotropic or not) and
    constant sigma_t, phi = c0 + c . x and J = -E0 c / sigma_t solve the
    VEF equations with Q1 = 0, Q0 = sigma_a phi, and the Miften-Larsen
    boundary condition holds when J_in = (J . n - E_b phi) / 2; the discrete
    solution reproduces them (and lambda = phi on interior faces) on sheared
    meshes, which pins C1, C2, the boundary terms and the global assembly;
  * the global solve equals the element-local elimination through the
    block inverse (the paper's reduced system for lambda), computed here
    with numpy from the oracle's blocks;
  * thick diffusion limit: the outer iteration converges in a handful of
    iterations where plain source iteration would need thousands.
"""
import math

import numpy as np
import pytest

from oracle import hrt_oracle as H
from oracle import oracle as O
from oracle import vef_outer_oracle as V
from paper_2301_04758_amd import problems as P


def _sheared(n, p, st=2.0, sa=0.3, nq=None, graded=False):
    cp, ec = P.quad_mesh(n, n, 1)
    if graded:  # rectangles of different sizes: the Jacobian varies by element
        cp = cp.copy()
        cp[:, 0] = cp[:, 0] ** 1.7
        cp[:, 1] = 0.5 * (cp[:, 1] + cp[:, 1] ** 2)
    cp = cp @ np.array([[1.3, 0.3], [0.15, 1.0]]).T + np.array([0.5, 0.25])
    om, wt = P.level_symmetric_2d(4)
    ne = ec.shape[0]
    pr = P.Problem("sheared", p, 1, cp, ec, om, wt, np.full(ne, st), np.full(ne, st - sa), nx=n, ny=n,
                   nq=nq or p + 2)
    return pr


def _linear_case(pr, E0, c0=0.8, c=(0.25, -0.4)):
    nq = pr.nq
    c = np.asarray(c)
    st = pr.sigma_t[0]
    sa = pr.sigma_t - pr.sigma_s
    Jex = -E0 @ c / st
    x0, F = H.affine_frames(pr)
    gx, gw = O.gauss_rule(nq)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    xi, eta = XI.ravel(), ETA.ravel()
    ne = pr.n_elem
    xq = x0[:, None, :] + np.einsum("ekl,ql->eqk", F, np.stack([xi, eta], 1))
    phi_q = c0 + xq @ c
    E_vol = np.broadcast_to(E0, (ne, nq * nq, 2, 2)).copy()
    bfs = O.boundary_faces(pr)
    Eb = np.full((len(bfs), nq), 0.55)
    Jin = np.zeros((len(bfs), nq))
    for k, (e, f) in enumerate(bfs):
        fx, fy = H.face_points(f, gx)
        x = x0[e] + np.stack([fx, fy], 1) @ F[e].T
        tang = {0: F[e][:, 0], 1: F[e][:, 1], 2: -F[e][:, 0], 3: -F[e][:, 1]}[f]
        n = np.array([tang[1], -tang[0]]) / np.hypot(*tang)
        Jin[k] = (Jex @ n - Eb[k] * (c0 + x @ c)) / 2.0
    Q0 = sa[:, None] * phi_q
    Q1 = np.zeros((2, ne, nq * nq))
    out = V.global_solve(pr, nq, E_vol, lambda e, f: np.broadcast_to(E0, (nq, 2, 2)), Eb, Jin, Q0, Q1)
    return out, Jex, c0, c, x0, F


@pytest.mark.parametrize("graded", [False, True])
@pytest.mark.parametrize("E0", [((1 / 3, 0), (0, 1 / 3)), ((0.45, 0.1), (0.1, 0.3))])
@pytest.mark.parametrize("p", [1, 2])
def test_global_solve_reproduces_linear_solution(p, E0, graded):
    E0 = np.array(E0, float)
    pr = _sheared(3, p, graded=graded)
    out, Jex, c0, c, x0, F = _linear_case(pr, E0)
    leg = H.legendre_points(p + 1)
    LX, LY = np.meshgrid(leg, leg, indexing="xy")
    nodes = np.stack([LX.ravel(), LY.ravel()], 1)
    for e in range(pr.n_elem):
        want_phi = c0 + (x0[e] + nodes @ F[e].T) @ c
        assert np.allclose(out["phi"][e], want_phi, rtol=1e-11, atol=1e-12)
        vhat = np.linalg.det(F[e]) * np.linalg.solve(F[e], Jex)
        nx = (p + 2) * (p + 1)
        assert np.allclose(out["J"][e], np.concatenate([np.full(nx, vhat[0]), np.full(nx, vhat[1])]),
                           rtol=1e-11, atol=1e-12)
    # lambda = phi at the face nodes
    nbr, interior = V._faces(pr)
    for k, (e1, f1, e2, f2) in enumerate(interior):
        fx, fy = H.face_points(f1, leg)
        x = x0[e1] + np.stack([fx, fy], 1) @ F[e1].T
        assert np.allclose(out["lam"][k], c0 + x @ c, rtol=1e-11, atol=1e-12)


def test_global_solve_equals_local_elimination():
    """The direct solve and the reduced lambda system through the block
    inverse (Sec. 7: H lambda = C1 (W g + X f)) give the same phi."""
    p = 2
    pr = _sheared(3, p, st=1.5, sa=0.2)
    pr.sigma_t = pr.sigma_t * np.linspace(0.8, 1.6, pr.n_elem)
    pr.sigma_s = pr.sigma_t - 0.2
    pr.q_iso = np.ones((pr.n_elem, 9))
    nq = pr.nq
    r = O.sweep(pr, want_psi=False, nq=nq)
    cl = O.closures(pr, r["mom"], r["bnd"], nq=nq)
    gx, _ = O.gauss_rule(nq)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    E_vol = H.eddington_from_moments(pr, r["mom"], XI.ravel(), ETA.ravel())

    def E_face(e, f):
        fx, fy = H.face_points(f, gx)
        return H.eddington_from_moments(pr, r["mom"][:, e:e + 1], fx, fy)[0]

    d = V.global_solve(pr, nq, E_vol, E_face, cl["Eb"], cl["Jin"], cl["Q0"], cl["Q1"], return_system=True)
    M, b, nloc = d["M"], d["b"], d["nloc"]
    ne = pr.n_elem
    nl = M.shape[0] - ne * nloc
    inv, _ = H.local_inverse(pr, nq, r["mom"], cl["Eb"])
    Hred = np.zeros((nl, nl))
    rhs = np.zeros(nl)
    for e in range(ne):
        sl = slice(e * nloc, (e + 1) * nloc)
        C2 = M[sl, ne * nloc:]          # [[C2], [0]] columns of element e
        C1 = M[ne * nloc:, sl]          # [C1, 0] rows
        Hred += C1 @ inv[e] @ C2
        rhs += C1 @ inv[e] @ b[sl]
    lam = np.linalg.solve(Hred, rhs)
    assert np.allclose(lam, d["lam"].ravel(), rtol=1e-10, atol=1e-12 * np.abs(lam).max())
    for e in range(ne):
        sl = slice(e * nloc, (e + 1) * nloc)
        x = inv[e] @ (b[sl] - M[sl, ne * nloc:] @ lam)
        assert np.allclose(x[nloc - (p + 1) ** 2:], d["phi"][e], rtol=1e-10, atol=1e-12)


def test_thick_diffusion_limit_converges_fast():
    """sigma_t = 1/eps, sigma_a = eps, q = eps on an 8x8 unit square (Sec. 8,
    thick diffusion limit): the outer iteration settles within a few
    iterations for eps = 1e-2, where source iteration's spectral radius is
    1 - eps^2."""
    eps = 1e-2
    cp, ec = P.quad_mesh(8, 8, 1)
    om, wt = P.level_symmetric_2d(4)
    ne = ec.shape[0]
    pr = P.Problem("tdl", 1, 1, cp, ec, om, wt, np.full(ne, 1 / eps), np.full(ne, 1 / eps - eps), nx=8, ny=8, nq=3)
    pr.q_iso = np.full((ne, 4), eps / (4 * math.pi))
    hist = V.outer_iteration(pr, 3, 10)
    changes = [np.abs(hist[k + 1] - hist[k]).max() / np.abs(hist[k + 1]).max() for k in range(len(hist) - 1)]
    assert changes[-1] < 1e-6, changes
    assert all(np.isfinite(h).all() for h in hist)


# --------------------------------------------------------------- Anderson
def test_anderson_scalar_linear_map_is_exact_after_one_secant_step():
    """x = a x + b with memory 1: the constrained weights make the affine
    residual vanish, so the second iterate is the fixed point b / (1 - a)."""
    a, b, x0 = 0.9, 0.7, np.array([0.3])
    xs, _ = V.anderson(lambda x: a * x + b, x0, 1, 3)
    assert abs(xs[0][0] - (a * 0.3 + b)) < 1e-15
    assert abs(xs[1][0] - b / (1 - a)) < 1e-13


def _gmres_iterate(A, rhs, x0, k):
    """The GMRES iterate by its definition: x0 + z, z in the Krylov space
    K_k(A, r0), minimising |rhs - A x|_2 (plain least squares on the
    orthonormalised Krylov basis)."""
    r0 = rhs - A @ x0
    K = np.stack([np.linalg.matrix_power(A, j) @ r0 for j in range(k)], axis=1)
    Qk, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Qk, r0, rcond=None)
    return x0 + Qk @ y


def test_anderson_on_a_linear_map_is_G_of_the_gmres_iterate():
    """Walker and Ni (2011), Sec. 4: on G(x) = M x + b with unbounded memory,
    x_{k+1} = G(xbar_k) with xbar_k the k-th GMRES iterate of (I - M) x = b
    from x0; after n steps that is the fixed point itself."""
    rng = np.random.default_rng(2)
    n = 6
    M = rng.standard_normal((n, n))
    M *= 0.8 / max(abs(np.linalg.eigvals(M)))
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    G = lambda x: M @ x + b  # noqa: E731
    xs, gs = V.anderson(G, x0, n, n + 1)
    A = np.eye(n) - M
    for k in range(1, n):
        want = G(_gmres_iterate(A, b, x0, k))
        assert np.allclose(xs[k], want, rtol=0, atol=1e-10 * np.abs(want).max()), k
    xstar = np.linalg.solve(A, b)
    assert np.abs(xs[n] - xstar).max() < 1e-9 * np.abs(xstar).max()
    # memory 0 is the plain iteration
    xp, _ = V.anderson(G, x0, 0, 3)
    assert np.allclose(xp[2], G(G(G(x0))), rtol=0, atol=1e-15)


def test_anderson_outer_iteration_converges_no_slower():
    """On the thick-diffusion-limit problem (eps = 1e-2, 8x8) the outer
    iteration with two Anderson vectors reaches a relative change of 1e-8 in
    no more iterations than the plain one, to the same flux."""
    eps = 1e-2
    cp, ec = P.quad_mesh(8, 8, 1)
    om, wt = P.level_symmetric_2d(4)
    ne = ec.shape[0]
    pr = P.Problem("tdl", 1, 1, cp, ec, om, wt, np.full(ne, 1 / eps), np.full(ne, 1 / eps - eps), nx=8, ny=8, nq=3)
    pr.q_iso = np.full((ne, 4), eps / (4 * math.pi))

    def first_below(hist, tol=1e-8):
        for k in range(1, len(hist)):
            if np.abs(hist[k] - hist[k - 1]).max() <= tol * np.abs(hist[k]).max():
                return k + 1
        return None

    plain = V.outer_iteration(pr, 3, 10)
    acc = V.outer_iteration(pr, 3, 10, m_anderson=2)
    kp, ka = first_below(plain), first_below(acc)
    assert kp is not None and ka is not None and ka <= kp, (kp, ka)
    assert np.abs(acc[ka - 1] - plain[-1]).max() <= 1e-7 * np.abs(plain[-1]).max()


def _paper_tdl_table():
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_tdl_iterations.txt")):
        line = line.split("#")[0].split()
        if line:
            rows.append((float(line[0]), int(line[1])))
    return rows


def _tdl8(eps):
    pr = P.make_problem("tdl_8", 8, 8, 2, 1, 4, 1.0 / eps, 1.0 / eps - eps, q=eps)
    pr.nq = 4
    return pr


def test_thick_limit_iteration_counts_match_the_paper_table():
    """The oracle's fixed point on the paper's thick-diffusion-limit setup
    (8x8 orthogonal mesh, p = 2, S4) converges to a relative change of 1e-6
    within one iteration of the paper's HRT counts (tests/golden)."""
    for eps, want in _paper_tdl_table():
        pr = _tdl8(eps)
        hist = V.outer_iteration(pr, pr.nq, want + 2)
        got = None
        for k in range(1, len(hist)):
            if np.abs(hist[k] - hist[k - 1]).max() <= 1e-6 * np.abs(hist[k]).max():
                got = k + 1
                break
        assert got is not None and abs(got - want) <= 1, (eps, got, want)
