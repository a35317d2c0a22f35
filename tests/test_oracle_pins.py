"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the part of the oracle it pins:
  tables (Gauss rule, Gauss-Lobatto nodes), geometry, constant preservation,
  polynomial patch test, per-element balance, an independent brute-force
  global solve, the Pade outflow of pure absorption, manufactured-solution
  convergence order, symmetry of the square, moment closed forms, quadrature
  rule independence, the source-iteration fixed point, and error paths.
"""
import math
import os

import numpy as np
import pytest

import dg_numpy as D
import mms
from oracle import oracle as O
from paper_2301_04758_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(230104758)


def _problem(nx, ny, p, m, N, st=1.0, ss=0.0, warp=0.0, q=None):
    cp, ec = P.quad_mesh(nx, ny, m)
    if warp:
        cp = P.sine_warp(cp, warp)
    om, wt = P.level_symmetric_2d(N)
    ne = ec.shape[0]
    st = np.broadcast_to(np.asarray(st, float), (ne,)).copy()
    ss = np.broadcast_to(np.asarray(ss, float), (ne,)).copy()
    pr = P.Problem("t", p, m, cp, ec, om, wt, st, ss, nx=nx, ny=ny)
    if q is not None:
        pr.q_iso = np.full((ne, (p + 1) ** 2), float(q))
    return pr


# ---------------------------------------------------------------- tables


@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_rule_exact_for_monomials(n):
    x, w = O.gauss_rule(n)
    assert np.all(np.diff(x) > 0) and abs(w.sum() - 1) < 1e-15
    for k in range(2 * n):
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14
    # not exact one degree higher (sanity of the degree claim)
    assert abs(np.dot(w, x ** (2 * n)) - 1.0 / (2 * n + 1)) > 1e-12
    xr, wr = D.gauss01(n)
    assert np.allclose(x, xr, atol=1e-15) and np.allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_gauss_lobatto_nodes(k):
    z = O.gl_nodes(k)
    assert np.allclose(z, D.gl_points(k), atol=1e-15)
    closed = {1: [0, 1], 2: [0, .5, 1], 3: [0, (1 - 5 ** -.5) / 2, (1 + 5 ** -.5) / 2, 1],
              4: [0, (1 - (3 / 7) ** .5) / 2, .5, (1 + (3 / 7) ** .5) / 2, 1]}[k]
    assert np.allclose(z, closed, atol=1e-16)
    B = D.Basis1D(z)
    t = np.linspace(0, 1, 17)
    assert np.allclose(B.val(t).sum(-1), 1.0, atol=1e-13)  # partition of unity


# ---------------------------------------------------------------- geometry


@pytest.mark.parametrize("m,warp", [(1, 0.0), (2, 0.1), (3, 0.05)])
def test_geometry_area_closure_and_face_match(m, warp):
    pr = _problem(6, 5, 2, m, 4, warp=warp)
    area, closure, mismatch = O.geometry_report(pr)
    assert abs(area - 1.0) < 1e-14
    assert closure < 1e-15
    assert mismatch < 1e-15
    assert O.n_boundary_faces(pr) == 2 * (6 + 5)


def test_boundary_face_numbering_is_element_face_order():
    pr = _problem(3, 2, 1, 1, 4)
    bf = O.boundary_faces(pr)
    keys = [tuple(r) for r in bf]
    assert keys == sorted(keys)
    # 1 + 2 faces on a 3x2 grid's corner elements etc.
    assert len(bf) == 10


# ---------------------------------------------------------------- invariants



def _random_st(ne):
    return np.random.default_rng(7).uniform(0.5, 5.0, ne)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_translation_invariance(m):
    """Geometry: the discrete problem is invariant under a translation of the
    mesh.  Control points on a 2^-30 grid stay exact when shifted by 2^10, so
    the translated problem is the same problem; only an evaluation of the map
    derivatives from absolute coordinates (cancellation of domain-size
    numbers down to element size) could tell them apart, by about
    eps * 2^10 / h = 5e-12 here."""
    pr = _problem(24, 24, 3, m, 4, st=_random_st(24 * 24), ss=0.0, warp=0.08 if m > 1 else 0.0, q=1.0)
    if m == 1:  # straight but non-affine: move interior vertices
        cp = pr.cp_xy.copy()
        inner = (cp > 1e-12).all(1) & (cp < 1 - 1e-12).all(1)
        cp[inner] += RNG.uniform(-0.01, 0.01, (inner.sum(), 2))
        pr.cp_xy = cp
    pr.cp_xy = np.round(pr.cp_xy * 2.0 ** 30) / 2.0 ** 30
    a = O.sweep(pr)
    pr.cp_xy = pr.cp_xy + 2.0 ** 10
    b = O.sweep(pr)
    assert np.abs(b["psi"] - a["psi"]).max() <= 4e-16 * np.abs(a["psi"]).max()


@pytest.mark.parametrize("p,m,warp", [(1, 1, 0.0), (3, 1, 0.0), (2, 2, 0.1), (3, 2, 0.1), (4, 1, 0.0)])
def test_constant_preservation(p, m, warp):
    """sigma_s = 0, q const, inflow q/sigma_t: psi == q/sigma_t (Piola identity keeps
    the discrete streaming of a constant zero on curved maps)."""
    st = 2.5
    pr = _problem(5, 4, p, m, 6, st=st, warp=warp, q=3.0)
    nb = O.n_boundary_faces(pr)
    pr.psi_bc = np.full((pr.n_dir, nb, p + m), 3.0 / st)
    r = O.sweep(pr)
    assert np.abs(r["psi"] - 3.0 / st).max() < 1e-13
    # with scattering: phi_in = 4 pi q / sigma_a, inflow q / sigma_a
    sa = 0.7
    pr.sigma_s = np.full(pr.n_elem, st - sa)
    pr.psi_bc = np.full((pr.n_dir, nb, p + m), 3.0 / sa)
    phi = np.full((pr.n_elem, (p + 1) ** 2), 4 * np.pi * 3.0 / sa)
    r = O.sweep(pr, phi_in=phi)
    assert np.abs(r["psi"] - 3.0 / sa).max() < 1e-12 * 3.0 / sa


@pytest.mark.parametrize("p,m,warp", [(1, 1, 0.0), (2, 2, 0.1), (3, 2, 0.1), (3, 3, 0.05)])
def test_linear_patch(p, m, warp):
    """psi_d = a_d + b_d . x is reproduced to roundoff when p >= m."""
    pr = _problem(4, 4, p, m, 4, st=1.7, warp=warp)
    vxy, bxy, _ = O.qp_coords(pr)
    a = RNG.uniform(1, 2, pr.n_dir)
    b = RNG.uniform(-1, 1, (pr.n_dir, 2))
    pr.q_dir = np.stack([pr.omega[d] @ b[d] + 1.7 * (a[d] + vxy @ b[d]) for d in range(pr.n_dir)])
    pr.psi_bc = np.stack([a[d] + bxy @ b[d] for d in range(pr.n_dir)])
    r = O.sweep(pr)
    X = D.Mesh(pr).node_coords()
    exact = np.stack([a[d] + X @ b[d] for d in range(pr.n_dir)])
    assert np.abs(r["psi"] - exact).max() < 1e-12


@pytest.mark.parametrize("p,m,warp", [(1, 1, 0.0), (2, 1, 0.0), (2, 2, 0.1), (3, 2, 0.08)])
def test_element_balance_and_brute_force(p, m, warp):
    """Per-element particle balance (test function 1) and equality with an
    independent dense global solve of the upwind DG system per direction."""
    pr = _problem(3, 4, p, m, 4, st=RNG.uniform(0.3, 4.0, 12), warp=warp)
    pr.sigma_s = 0.6 * pr.sigma_t
    n = (p + 1) ** 2
    nq = p + m
    nb = O.n_boundary_faces(pr)
    pr.q_iso = RNG.uniform(0, 1, (12, n))
    pr.q_dir = RNG.uniform(0, 1, (pr.n_dir, 12, nq * nq))
    pr.psi_bc = RNG.uniform(0, 1, (pr.n_dir, nb, nq))
    phi = RNG.uniform(0, 2, (12, n))
    r = O.sweep(pr, phi_in=phi)
    for d in range(pr.n_dir):
        g = D.global_solve(pr, d, phi, pr.q_iso, pr.q_dir, pr.psi_bc)
        assert np.abs(g - r["psi"][d]).max() <= 1e-13 * np.abs(g).max()
        res, sc = D.balance_residuals(pr, r["psi"][d], d, phi, pr.q_iso, pr.q_dir, pr.psi_bc)
        assert np.abs(res).max() <= 1e-13 * sc.max()


def _pade(p, z):
    L, M = p, p + 1
    f = math.factorial
    num = sum(f(L + M - j) * f(L) / (f(L + M) * f(j) * f(L - j)) * (-z) ** j for j in range(L + 1))
    den = sum(f(L + M - j) * f(M) / (f(L + M) * f(j) * f(M - j)) * z ** j for j in range(M + 1))
    return num / den


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("mu,st", [(0.7, 2.3), (0.3, 9.0)])
def test_pure_absorber_pade_outflow(p, mu, st):
    """Direction (mu, 0), unit inflow on x = 0: each cell multiplies the outflow
    by the [p/(p+1)] Pade approximant of exp(-sigma_t h / mu), the known
    outflow map of upwind DG of degree p."""
    nx = 6
    cp, ec = P.quad_mesh(nx, 2, 1)
    ne = ec.shape[0]
    pr = P.Problem("pade", p, 1, cp, ec, np.array([[mu, 0.0]]), np.array([4 * np.pi]),
                   np.full(ne, st), np.zeros(ne))
    bf = O.boundary_faces(pr)
    bc = np.zeros((1, len(bf), p + 1))
    bc[0, bf[:, 1] == 3] = 1.0
    pr.psi_bc = bc
    psi = O.sweep(pr)["psi"][0]
    R = _pade(p, st / nx / mu)
    for j in range(2):
        for i in range(nx):
            for b in range(p + 1):
                v = psi[i + nx * j, p + (p + 1) * b]
                assert abs(v - R ** (i + 1)) < 1e-13
    # exponential attenuation: R differs from exp at O(z^(2p+2))
    z = st / nx / mu
    assert abs(R - math.exp(-z)) < 0.2 * z ** (2 * p + 2) / math.factorial(2 * p + 1)


def _mms_error(p, m, warp, nx):
    pr = _problem(nx, nx, p, m, 4, st=1.0, warp=warp)
    vxy, bxy, _ = O.qp_coords(pr)
    mms.attach(pr, vxy, bxy)
    r = O.sweep(pr)
    M = D.Mesh(pr)
    err = 0.0
    for e in range(pr.n_elem):
        xi, eta, W, x, F, J, v, gxi, geta = M.volume_data(e)
        ex = mms.moments_closed_form(x[:, 0], x[:, 1])[0]
        err += np.sum(W * J * (v @ r["mom"][0][e] - ex) ** 2)
    return math.sqrt(err)


@pytest.mark.parametrize("p,m,warp", [(1, 1, 0.0), (2, 1, 0.0), (3, 1, 0.0), (1, 2, 0.05), (2, 2, 0.05)])
def test_mms_convergence_order(p, m, warp):
    """Manufactured solution of Sec. 8.1 on straight and sine-curved meshes:
    the L2 error of the scalar flux decreases at order p+1 (log fit, 4 meshes)."""
    hs = [1 / 4, 1 / 8, 1 / 16, 1 / 32]
    errs = [_mms_error(p, m, warp, int(round(1 / h))) for h in hs]
    order = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert order > p + 1 - 0.2, (errs, order)


def test_c1_square_symmetry():
    """C1 (8x8, S4, vacuum, uniform data): phi is invariant under the symmetries of the square."""
    (pr,), _ = P.make_config("c1")
    phi = O.sweep(pr, want_psi=False)["mom"][0].reshape(8, 8, 2, 2)  # [j, i, b, a]
    full = phi.transpose(0, 2, 1, 3).reshape(16, 16)  # rows y nodes, cols x nodes
    scale = np.abs(full).max()
    for g in (full[:, ::-1], full[::-1, :], full.T, full[::-1, ::-1].T):
        assert np.abs(g - full).max() < 1e-14 * scale


# ---------------------------------------------------------------- moments / closures


def test_moments_of_mms_psi_match_paper_closed_forms():
    """Moments of the manufactured psi sampled per direction equal the paper's
    phi, J and P (S4 integrates these angular polynomials exactly).  The
    printed off-diagonal P uses a factor 1/15; direct integration gives 2/15,
    recorded in tests/golden/paper_closures.txt."""
    gold = {}
    for line in open(os.path.join(GOLD, "paper_closures.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            gold[k] = float(v)
    assert (gold["mms_delta"], gold["mms_zeta"], gold["mms_omega"]) == (mms.DELTA, mms.ZETA, mms.OMEGA)
    pr = _problem(3, 3, 2, 2, 4, warp=0.1)
    X = D.Mesh(pr).node_coords()
    psi = np.stack([mms.psi(X[..., 0], X[..., 1], *pr.omega[d])[0] for d in range(pr.n_dir)])
    mom = O.moments_from_psi(pr, psi)
    phi, J, Pm = mms.moments_closed_form(X[..., 0], X[..., 1])
    assert np.abs(mom[0] - phi).max() < 1e-13
    assert np.abs(mom[1] - J[0]).max() < 1e-13 and np.abs(mom[2] - J[1]).max() < 1e-13
    assert np.abs(mom[3] - Pm[0]).max() < 1e-13
    assert np.abs(mom[4] - gold["mms_P_offdiag_factor"] * mms.fields(X[..., 0], X[..., 1])["t12"][0] / 15).max() < 1e-13
    assert np.abs(mom[5] - Pm[2]).max() < 1e-13


@pytest.mark.parametrize("N", [4, 12])
def test_isotropic_closures(N):
    """Constant psi: phi = 4 pi c, J = 0, E = I/3 exactly; E_b tends to 1/2
    (continuous value) and J_in to -pi c for isotropic inflow c; Q0 = 4 pi q,
    Q1 = 0."""
    c = 0.8
    pr = _problem(4, 4, 2, 2, N, st=2.0, warp=0.08, q=2.0 * c)
    nb = O.n_boundary_faces(pr)
    pr.psi_bc = np.full((pr.n_dir, nb, 4), c)
    r = O.sweep(pr)
    assert np.abs(r["mom"][0] - 4 * np.pi * c).max() < 1e-12
    assert np.abs(r["mom"][1:3]).max() < 1e-12
    cl = O.closures(pr, r["mom"], r["bnd"])
    assert cl["n_nonpos"] == 0
    assert np.abs(cl["E"][0] - 1 / 3).max() < 1e-13 and np.abs(cl["E"][2] - 1 / 3).max() < 1e-13
    assert np.abs(cl["E"][1]).max() < 1e-13
    tol = {4: 0.03, 12: 0.005}[N]
    assert np.abs(cl["Eb"] - 0.5).max() < tol
    assert np.abs(cl["Jin"] + np.pi * c).max() < 2 * np.pi * c * tol
    # J_in = -(c/2) sum w |Omega.n| = -2 pi c E_b for a set symmetric under Omega -> -Omega
    assert np.abs(cl["Jin"] + 2 * np.pi * c * cl["Eb"]).max() < 1e-12
    assert np.abs(cl["Q0"] - 4 * np.pi * 2.0 * c).max() < 1e-12
    assert np.abs(cl["Q1"]).max() < 1e-12


def test_closure_flags_nonpositive_flux():
    """Thick cells with p = 1 produce negative DG angular flux; where the scalar
    flux is not positive the Eddington tensor is left 0 and counted."""
    pr = _problem(4, 4, 1, 1, 4, st=1.0)
    pr.q_iso = np.zeros((16, 4))
    pr.q_iso[0] = 50.0
    pr.sigma_t[:] = 200.0
    r = O.sweep(pr)
    cl = O.closures(pr, r["mom"], r["bnd"])
    phiq_neg = cl["n_nonpos"]
    assert phiq_neg > 0
    assert np.all(cl["E"][:, cl["E"][0] == 0] == 0)


# ---------------------------------------------------------------- rule independence, SI


def test_quadrature_rule_independence_straight():
    """On straight meshes with element-constant data the default n_q = p + m
    integrates every term exactly: one more point changes nothing."""
    pr = _problem(5, 5, 3, 1, 6, st=RNG.uniform(0.5, 5, 25), q=1.0)
    pr.sigma_s = 0.5 * pr.sigma_t
    phi = RNG.uniform(0, 1, (25, 16))
    r1 = O.sweep(pr, phi_in=phi, nq=4)
    r2 = O.sweep(pr, phi_in=phi, nq=5)
    assert np.abs(r1["psi"] - r2["psi"]).max() < 1e-13 * np.abs(r1["psi"]).max()


def test_source_iteration_converges_to_coupled_solve():
    """Source iteration reaches the fixed point of the fully coupled
    (all directions, implicit scattering) discrete system; residuals are the
    max norm of successive scalar-flux iterates."""
    pr = _problem(2, 3, 1, 1, 4, st=RNG.uniform(1, 3, 6), q=1.0)
    pr.sigma_s = 0.5 * pr.sigma_t
    si = O.source_iteration(pr, 80, tol=1e-15)
    ref = D.coupled_scattering_solve(pr, pr.q_iso)
    assert np.abs(si["mom"][0] - ref).max() < 1e-12 * np.abs(ref).max()
    r = si["resid"]
    assert r[-1] < 1e-13 and np.all(np.diff(np.log(r[:20])) < 0)
    # same residual history when run by single sweeps
    phi = np.zeros_like(ref)
    for k in range(5):
        mom = O.sweep(pr, phi_in=phi, want_psi=False)["mom"]
        assert abs(np.abs(mom[0] - phi).max() - r[k]) < 1e-15 * abs(r[k]) + 1e-300
        phi = mom[0]


# ---------------------------------------------------------------- error paths


def test_negative_jacobian_rejected():
    pr = _problem(2, 2, 1, 1, 4)
    ec = pr.elem_cp.copy()
    ec[0] = ec[0][[1, 0, 3, 2]]  # mirror element 0 in xi
    pr.elem_cp = ec
    with pytest.raises(O.OracleError) as ei:
        O.sweep(pr)
    assert ei.value.code == O.ERR_JACOBIAN


def test_invalid_order_rejected():
    pr = _problem(2, 2, 1, 1, 4)
    pr.p = 7
    with pytest.raises(O.OracleError):
        O.sweep(pr)


def test_levels_cartesian():
    """On an nx x ny Cartesian mesh every direction has nx + ny - 1 levels."""
    pr = _problem(7, 5, 1, 1, 8)
    assert np.all(O.levels(pr) == 11)


# ---------------------------------------------------------------- negative-flux fixup

def _negative_flux_problem(p, m, warp, n=6):
    """Thick cells with a source in one corner element only: the unfixed DG
    solution dips below zero downstream of the source."""
    pr = _problem(n, n, p, m, 4, st=200.0, ss=0.0, warp=warp, q=0.0)
    pr.q_iso[0] = 50.0
    return pr


def test_fixup_is_noop_without_negative_values():
    pr = _problem(6, 6, 1, 1, 4, st=1.0, ss=0.0, q=1.0)  # p = 1, optically thin: no dip below zero
    a = O.sweep(pr)
    assert a["psi"].min() >= 0.0
    b = O.sweep(pr, fixup=True)
    assert np.array_equal(a["psi"], b["psi"])


@pytest.mark.parametrize("p,m,warp", [(1, 1, 0.0), (2, 1, 0.0), (3, 2, 0.06)])
def test_fixup_positive_and_element_balance(p, m, warp):
    """Set to zero and scale: no negative nodal value remains, and every
    element still satisfies its particle balance (outflow + absorption =
    inflow + source, checked with the independent numpy DG model)."""
    pr = _negative_flux_problem(p, m, warp)
    raw = O.sweep(pr)
    assert raw["psi"].min() < 0.0  # the case needs the fixup
    fx = O.sweep(pr, fixup=True)
    assert fx["psi"].min() >= 0.0
    assert not np.array_equal(raw["psi"], fx["psi"])
    for d in range(pr.n_dir):
        res, sc = D.balance_residuals(pr, fx["psi"][d], d, q_iso=pr.q_iso)
        rel = np.abs(res).max() / sc.max()
        assert rel <= 1e-12, (d, rel)
    # moments are those of the fixed angular flux
    assert np.allclose(O.moments_from_psi(pr, fx["psi"]), fx["mom"], rtol=0, atol=1e-13 * np.abs(fx["mom"]).max())


def test_threaded_oracle_sweep_is_bitwise_serial():
    """Directions swept on several OpenMP threads and summed in direction
    order afterwards: the same bits as the serial sweep (moments, angular
    flux, boundary sums, levels) and the same source-iteration history."""
    from paper_2301_04758_amd import problems as P
    (pr,), _ = P.make_config("c3", scale=6)
    a = O.sweep(pr)
    b = O.sweep(pr, threads=5)
    for k in ("psi", "mom", "bnd", "levels"):
        assert np.array_equal(a[k], b[k]), k
    r1 = O.source_iteration(pr, 3)
    r2 = O.source_iteration(pr, 3, threads=3)
    assert np.array_equal(r1["mom"], r2["mom"]) and np.array_equal(r1["resid"], r2["resid"])
