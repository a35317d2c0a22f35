"""Hybridized-RT VEF solve and the transport/VEF outer iteration -- TEST
INFRASTRUCTURE ONLY (numpy, double precision, small meshes).

Assembles the whole hybridized system of Sec. 7 (Eq. eq:hyb_form) and solves
it directly, without the element-by-element elimination: unknowns J (broken
RT_p), phi (Q_p per element) and lambda (degree p per interior face):

  rows of J_K:  A_K J_K + G_K phi_K + sum_{F in dK interior} C2_{K,F} lambda_F = g_K
  rows of phi_K:  D_K J_K + Ma_K phi_K = f_K
  rows of lambda_F:  sum_{K adjacent to F} C1_{F,K} J_K = 0

with  v^T C2 lambda = int_F v . <E n_K> lambda ds  (<E n_K> the average of E
n_K from both sides), mu^T C1 J = int_F mu (J . n_K) ds, g = int v . Q1 +
2 int_{Gamma_b} (1/E_b) v . E n J_in ds and f = int u Q0 (Eq. eq:g, eq:f).
Bases and readings as in hrt_oracle; lambda is Lagrange through the
Gauss-Legendre points in the counter-clockwise parameter of the face's lower
numbered element.  The outer iteration (Sec. 2) alternates an oracle
transport sweep driven by the VEF scalar flux with this solve, plain or
Anderson-accelerated (Sec. 8).
"""
from __future__ import annotations

import numpy as np

from . import hrt_oracle as H
from . import oracle as O


def _faces(pr):
    m = pr.m
    ec = np.asarray(pr.elem_cp)
    corner = {0: (0, m), 1: (m, (m + 1) ** 2 - 1), 2: ((m + 1) ** 2 - 1, m * (m + 1)), 3: (m * (m + 1), 0)}
    table = {}
    for e in range(pr.n_elem):
        for f in range(4):
            key = frozenset((int(ec[e, corner[f][0]]), int(ec[e, corner[f][1]])))
            table.setdefault(key, []).append((e, f))
    nbr = {}
    interior = []
    for lst in table.values():
        if len(lst) == 2:
            (e1, f1), (e2, f2) = sorted(lst)
            nbr[(e1, f1)] = (e2, f2)
            nbr[(e2, f2)] = (e1, f1)
            interior.append((e1, f1, e2, f2))
    interior.sort()
    return nbr, interior


def global_solve(pr, nq, E_vol, E_face, Eb, Jin, Q0, Q1, return_system=False):
    """Dense solve of the hybridized system.  E_vol [ne, nq^2, 2, 2] at the
    volume points; E_face(e, f) -> [nq, 2, 2] at the points of face f of
    element e (counter-clockwise parameter at the Gauss points); Eb, Jin
    [n_bf, nq]; Q0 [ne, nq^2]; Q1 [2, ne, nq^2].  Returns dict(J [ne, nv],
    phi [ne, nphi] (Gauss-Legendre nodal), lam [n_faces, p+1])."""
    p = pr.p
    nv, nphi = H.sizes(p)
    ne = pr.n_elem
    P1 = p + 1
    x0, F = H.affine_frames(pr)
    Jd = np.linalg.det(F)
    gx, gw = O.gauss_rule(nq)
    bfs = O.boundary_faces(pr)
    bf_index = {(int(e), int(f)): k for k, (e, f) in enumerate(bfs)}
    E_bnd = np.stack([E_face(int(e), int(f)) for e, f in bfs]) if len(bfs) else None
    blk = H.local_blocks(pr, nq, E_vol, E_bnd, Eb)
    nbr, interior = _faces(pr)
    fid = {}
    for k, (e1, f1, e2, f2) in enumerate(interior):
        fid[(e1, f1)] = k
        fid[(e2, f2)] = k
    nloc = nv + nphi
    N = ne * nloc + len(interior) * P1
    M = np.zeros((N, N))
    b = np.zeros(N)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    xi, eta = XI.ravel(), ETA.ravel()
    Wq = np.outer(gw, gw).ravel()
    vh, _ = H.rt_basis(p, xi, eta)
    u = H.phi_basis(p, xi, eta)
    leg = H.legendre_points(P1)
    for e in range(ne):
        o = e * nloc
        M[o:o + nv, o:o + nv] = blk["A"][e]
        M[o:o + nv, o + nv:o + nloc] = blk["G"][e]
        M[o + nv:o + nloc, o:o + nv] = blk["D"][e]
        M[o + nv:o + nloc, o + nv:o + nloc] = blk["Ma"][e]
        v = np.einsum("kl,qil->qik", F[e], vh) / Jd[e]
        b[o:o + nv] += np.einsum("q,qik,kq->i", Wq * Jd[e], v, Q1[:, e])
        b[o + nv:o + nloc] += np.einsum("q,qi,q->i", Wq * Jd[e], u, Q0[e])
        for f in range(4):
            fx, fy = H.face_points(f, gx)
            vb = np.einsum("kl,qil->qik", F[e], H.rt_basis(p, fx, fy)[0]) / Jd[e]
            tang = {0: F[e][:, 0], 1: F[e][:, 1], 2: -F[e][:, 0], 3: -F[e][:, 1]}[f]
            nds = np.array([tang[1], -tang[0]])
            length = np.hypot(*nds)
            n = nds / length
            if (e, f) not in nbr:
                k = bf_index[(e, f)]
                eb = np.where(Eb[k] > 0, Eb[k], 0.5)
                vEn = np.einsum("qik,qkl,l->qi", vb, E_face(e, f), n)
                b[o:o + nv] += np.einsum("q,qi,q->i", 2.0 * gw * length / eb, vEn, Jin[k])
                continue
            e2, f2 = nbr[(e, f)]
            En = 0.5 * np.einsum("qkl,l->qk", E_face(e, f) + E_face(e2, f2)[::-1], n)
            s = gx if e < e2 else 1.0 - gx
            lam = np.stack([np.prod([(s - leg[c]) / (leg[t] - leg[c]) for c in range(P1) if c != t], axis=0)
                            for t in range(P1)], axis=1)
            col = ne * nloc + fid[(e, f)] * P1
            M[o:o + nv, col:col + P1] += np.einsum("q,qik,qk,qt->it", gw * length, vb, En, lam)
            M[col:col + P1, o:o + nv] += np.einsum("q,qt,qik,k->ti", gw * length, lam, vb, n)
    sol = np.linalg.solve(M, b)
    loc = sol[:ne * nloc].reshape(ne, nloc)
    out = dict(J=loc[:, :nv], phi=loc[:, nv:], lam=sol[ne * nloc:].reshape(-1, P1))
    if return_system:
        out.update(M=M, b=b, nloc=nloc)
    return out


def legendre_to_lobatto(p):
    """[nT, nphi]: the Gauss-Legendre nodal Q_p basis at the transport's
    Gauss-Lobatto nodes (node a + (p+1) b)."""
    lob = O.gl_nodes(p)
    X, Y = np.meshgrid(lob, lob, indexing="xy")
    return H.phi_basis(p, X.ravel(), Y.ravel())


def outer_step(pr, nq, phi_lob):
    """One outer iteration: oracle sweep with scattering flux phi_lob
    (Gauss-Lobatto nodal, None = 0), closures, hybridized VEF solve.
    Returns (phi at the Lobatto nodes, dict of the solve)."""
    r = O.sweep(pr, phi_in=phi_lob, want_psi=False, nq=nq)
    cl = O.closures(pr, r["mom"], r["bnd"], nq=nq)
    mom = r["mom"]
    gx, _ = O.gauss_rule(nq)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    E_vol = H.eddington_from_moments(pr, mom, XI.ravel(), ETA.ravel())

    def E_face(e, f):
        fx, fy = H.face_points(f, gx)
        return H.eddington_from_moments(pr, mom[:, e:e + 1], fx, fy)[0]

    Q0 = cl["Q0"]
    Q1 = cl["Q1"]
    out = global_solve(pr, nq, E_vol, E_face, cl["Eb"], cl["Jin"], Q0, Q1)
    return out["phi"] @ legendre_to_lobatto(pr.p).T, out


def anderson(G, x0, m, n_iter):
    """Anderson-accelerated fixed-point iteration for x = G(x) with memory m
    (the outer solver the paper takes from KINSOL, Sec. 8; algorithm of
    Walker and Ni, SIAM J. Numer. Anal. 49 (2011)): with residuals
    f_i = G(x_i) - x_i, the weights alpha minimise |sum_i alpha_i f_i|_2 over
    the last min(m, k) + 1 residuals subject to sum_i alpha_i = 1, and
    x_{k+1} = sum_i alpha_i G(x_i).  m = 0 is the plain iteration
    x_{k+1} = G(x_k).  Returns the iterates [x_1, ..., x_n_iter] and the
    evaluations [G(x_0), ..., G(x_{n_iter-1})]."""
    xs = [np.asarray(x0, dtype=float)]
    gs, fs = [], []
    for k in range(n_iter):
        gs.append(np.asarray(G(xs[k]), dtype=float))
        fs.append(gs[k] - xs[k])
        mk = min(m, k)
        if mk == 0:
            xs.append(gs[k])
            continue
        Fm = np.stack(fs[k - mk:k + 1], axis=1)            # [n, mk + 1]
        # equality-constrained least squares through its KKT system
        K = np.zeros((mk + 2, mk + 2))
        K[:mk + 1, :mk + 1] = 2.0 * Fm.T @ Fm
        K[:mk + 1, mk + 1] = 1.0
        K[mk + 1, :mk + 1] = 1.0
        rhs = np.zeros(mk + 2)
        rhs[mk + 1] = 1.0
        alpha = np.linalg.solve(K, rhs)[:mk + 1]
        xs.append(sum(alpha[i] * gs[k - mk + i] for i in range(mk + 1)))
    return xs[1:], gs


def outer_iteration(pr, nq, n_outer, phi0=None, m_anderson=0):
    """n_outer outer iterations on the VEF scalar flux (Gauss-Legendre nodal,
    phi0 None = 0), Anderson-accelerated with memory m_anderson (0 = the
    plain fixed point of Sec. 2); returns the list of iterates."""
    L = legendre_to_lobatto(pr.p)
    shape = (pr.n_elem, (pr.p + 1) ** 2)

    def G(x):
        _, out = outer_step(pr, nq, x.reshape(shape) @ L.T)
        return out["phi"].ravel()

    x0 = np.zeros(shape) if phi0 is None else np.asarray(phi0, dtype=float)
    xs, _ = anderson(G, x0.ravel(), m_anderson, n_outer)
    return [x.reshape(shape) for x in xs]
