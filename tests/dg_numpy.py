"""Independent numpy implementation of the upwind DG S_N discretisation, used only to pin the oracle.

Built from numpy library routines (Gauss rule from numpy.polynomial.legendre,
Gauss-Lobatto points as roots of P_k', Lagrange polynomials as numpy
polynomials) and assembled *globally*: one dense (n_elem*n)^2 system per
direction, solved with numpy.linalg.solve.  It shares the weak-form definition
with the oracle but none of its code, ordering or indexing, so it checks face
matching, orientation, upwind ordering and the local assembly of the sweep.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def gl_points(k):
    """Gauss-Lobatto points of degree k on [0,1] from the roots of P_k'."""
    if k == 1:
        return np.array([0.0, 1.0])
    c = np.zeros(k + 1)
    c[k] = 1.0
    r = np.sort(npleg.legroots(npleg.legder(c)).real)
    return np.concatenate([[0.0], 0.5 * (r + 1.0), [1.0]])


def gauss01(n):
    x, w = npleg.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_polys(z):
    """numpy power-series coefficients of the Lagrange polynomials through z."""
    out = []
    for a in range(len(z)):
        others = np.delete(z, a)
        c = nppoly.polyfromroots(others)
        c = c / nppoly.polyval(z[a], c)
        out.append(c)
    return out


class Basis1D:
    def __init__(self, z):
        self.z = np.asarray(z, dtype=float)
        self.c = lagrange_polys(self.z)
        self.dc = [nppoly.polyder(c) for c in self.c]

    def val(self, x):
        x = np.asarray(x, dtype=float)
        return np.stack([nppoly.polyval(x, c) for c in self.c], axis=-1)

    def der(self, x):
        x = np.asarray(x, dtype=float)
        return np.stack([nppoly.polyval(x, c) for c in self.dc], axis=-1)


def tensor_vals(B: Basis1D, xi, eta):
    """values, d/dxi, d/deta of the tensor basis (index a + (k+1) b) at points."""
    vx, vy = B.val(xi), B.val(eta)
    dx, dy = B.der(xi), B.der(eta)
    v = (vy[..., :, None] * vx[..., None, :]).reshape(*np.shape(xi), -1)
    gxi = (vy[..., :, None] * dx[..., None, :]).reshape(*np.shape(xi), -1)
    geta = (dy[..., :, None] * vx[..., None, :]).reshape(*np.shape(xi), -1)
    return v, gxi, geta


FACE_LOCAL = {  # reference point of face f at parameter s (counter-clockwise)
    0: lambda s: (s, 0.0 * s),
    1: lambda s: (1.0 + 0.0 * s, s),
    2: lambda s: (1.0 - s, 1.0 + 0.0 * s),
    3: lambda s: (0.0 * s, 1.0 - s),
}


class Mesh:
    def __init__(self, pr, nq=None):
        self.pr = pr
        self.p, self.m = pr.p, pr.m
        self.nq = nq or pr.p + pr.m
        self.n = (pr.p + 1) ** 2
        self.Bp = Basis1D(gl_points(pr.p))
        self.Bm = Basis1D(gl_points(pr.m))
        self.gx, self.gw = gauss01(self.nq)
        self.cp = np.asarray(pr.cp_xy, dtype=float)
        self.ec = np.asarray(pr.elem_cp)
        m = self.m
        corners = {0: (0, m), 1: (m, (m + 1) ** 2 - 1), 2: ((m + 1) ** 2 - 1, m * (m + 1)), 3: (m * (m + 1), 0)}
        self.corners = corners
        # face matching by an (unordered) pair of corner ids
        table = {}
        for e in range(pr.n_elem):
            for f in range(4):
                a, b = self.ec[e, corners[f][0]], self.ec[e, corners[f][1]]
                table.setdefault(frozenset((int(a), int(b))), []).append((e, f))
        self.nbr = {}
        for key, lst in table.items():
            assert len(lst) <= 2
            if len(lst) == 2:
                (e1, f1), (e2, f2) = lst
                self.nbr[(e1, f1)] = (e2, f2)
                self.nbr[(e2, f2)] = (e1, f1)
        self.bfaces = [(e, f) for e in range(pr.n_elem) for f in range(4) if (e, f) not in self.nbr]
        self.bf_index = {ef: i for i, ef in enumerate(self.bfaces)}

    def start_end(self, e, f):
        a, b = self.corners[f]
        return int(self.ec[e, a]), int(self.ec[e, b])

    def geom(self, e, xi, eta):
        """x, y, F (..., 2, 2) at reference points."""
        v, gxi, geta = tensor_vals(self.Bm, xi, eta)
        X = self.cp[self.ec[e]]
        x = v @ X
        Fxi = gxi @ X  # (x_xi, y_xi)
        Feta = geta @ X
        F = np.stack([np.stack([Fxi[..., 0], Feta[..., 0]], -1), np.stack([Fxi[..., 1], Feta[..., 1]], -1)], -2)
        return x, F

    def chord(self, e, f):
        s, t = self.start_end(e, f)
        d = self.cp[t] - self.cp[s]
        return np.array([d[1], -d[0]])

    def upwind_is_self(self, e, f, om):
        val = om @ self.chord(e, f)
        if (e, f) in self.nbr:
            if val > 0:
                return True
            if val < 0:
                return False
            return e < self.nbr[(e, f)][0]
        return not (val < 0)

    def face_data(self, e, f):
        s = self.gx
        xi, eta = FACE_LOCAL[f](s)
        x, F = self.geom(e, xi, eta)
        t = {0: F[:, :, 0], 1: F[:, :, 1], 2: -F[:, :, 0], 3: -F[:, :, 1]}[f]
        nds = np.stack([t[:, 1], -t[:, 0]], -1)
        return xi, eta, x, nds

    def neighbour_points(self, e, f):
        e2, f2 = self.nbr[(e, f)]
        s_start, _ = self.start_end(e, f)
        s2_start, _ = self.start_end(e2, f2)
        s = self.gx if s_start == s2_start else 1.0 - self.gx
        xi2, eta2 = FACE_LOCAL[f2](s)
        return e2, xi2, eta2

    def volume_data(self, e):
        XI, ETA = np.meshgrid(self.gx, self.gx, indexing="xy")  # qx fastest after ravel
        xi, eta = XI.ravel(), ETA.ravel()
        W = np.outer(self.gw, self.gw).ravel()
        x, F = self.geom(e, xi, eta)
        J = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
        v, gxi, geta = tensor_vals(self.Bp, xi, eta)
        return xi, eta, W, x, F, J, v, gxi, geta

    def node_coords(self):
        z = self.Bp.z
        XI, ETA = np.meshgrid(z, z, indexing="xy")
        out = np.zeros((self.pr.n_elem, self.n, 2))
        for e in range(self.pr.n_elem):
            out[e] = self.geom(e, XI.ravel(), ETA.ravel())[0]
        return out


def global_solve(pr, d, phi_in=None, q_iso=None, q_dir=None, psi_bc=None, nq=None, pointwise=False):
    """Dense global upwind-DG system for direction d, solved directly. Returns psi [n_elem, n]."""
    A, b = global_system(pr, d, phi_in, q_iso, q_dir, psi_bc, nq, pointwise=pointwise)
    return np.linalg.solve(A, b).reshape(pr.n_elem, -1)


def mass_matrices(pr, nq=None):
    M = Mesh(pr, nq)
    out = np.zeros((pr.n_elem, M.n, M.n))
    for e in range(pr.n_elem):
        xi, eta, W, x, F, J, v, gxi, geta = M.volume_data(e)
        out[e] = np.einsum("q,qi,qj->ij", W * J, v, v)
    return out


def coupled_scattering_solve(pr, q_iso=None, q_dir=None, psi_bc=None, nq=None):
    """All directions at once with the scattering source sigma_s/(4 pi) sum_d w_d psi_d
    kept implicit: the fixed point that source iteration converges to.  Returns phi [n_elem, n]."""
    nd, ne = pr.n_dir, pr.n_elem
    blocks = [global_system(pr, d, None, q_iso, q_dir, psi_bc, nq) for d in range(nd)]
    N = blocks[0][1].size
    n = N // ne
    Mm = mass_matrices(pr, nq)
    S = np.zeros((N, N))
    for e in range(ne):
        S[e * n:(e + 1) * n, e * n:(e + 1) * n] = pr.sigma_s[e] / (4 * np.pi) * Mm[e]
    big = np.zeros((nd * N, nd * N))
    rhs = np.zeros(nd * N)
    for d in range(nd):
        big[d * N:(d + 1) * N, d * N:(d + 1) * N] = blocks[d][0]
        rhs[d * N:(d + 1) * N] = blocks[d][1]
        for d2 in range(nd):
            big[d * N:(d + 1) * N, d2 * N:(d2 + 1) * N] -= pr.weight[d2] * S
    psi = np.linalg.solve(big, rhs).reshape(nd, ne, n)
    return np.einsum("d,den->en", pr.weight, psi)


def global_system(pr, d, phi_in=None, q_iso=None, q_dir=None, psi_bc=None, nq=None, pointwise=False):
    """Dense global upwind-DG matrix and right-hand side for direction d.
    pointwise: the upwind side is taken at each face point from the sign of
    Omega . n there (else for the whole face, from the rotated chord)."""
    M = Mesh(pr, nq)
    n, ne = M.n, pr.n_elem
    om = np.asarray(pr.omega[d], dtype=float)
    A = np.zeros((ne * n, ne * n))
    b = np.zeros(ne * n)
    for e in range(ne):
        xi, eta, W, x, F, J, v, gxi, geta = M.volume_data(e)
        adj = np.stack([np.stack([F[:, 1, 1], -F[:, 0, 1]], -1), np.stack([-F[:, 1, 0], F[:, 0, 0]], -1)], -2)
        g = adj @ om  # (Q, 2)
        stream = g[:, 0:1] * gxi + g[:, 1:2] * geta
        blk = np.einsum("q,qi,qj->ij", W * J * pr.sigma_t[e], v, v) - np.einsum("q,qi,qj->ij", W, stream, v)
        src = np.zeros(len(W))
        if phi_in is not None:
            src += pr.sigma_s[e] / (4 * np.pi) * (v @ phi_in[e])
        if q_iso is not None:
            src += v @ q_iso[e]
        if q_dir is not None:
            src += q_dir[d, e]
        b[e * n:(e + 1) * n] += np.einsum("q,qi->i", W * J * src, v)
        for f in range(4):
            fxi, feta, fx, nds = M.face_data(e, f)
            on = nds @ om
            vf = tensor_vals(M.Bp, fxi, feta)[0]
            if pointwise:
                own = (on >= 0).astype(float)
            else:
                own = np.full(len(on), 1.0 if M.upwind_is_self(e, f, om) else 0.0)
            blk += np.einsum("q,qi,qj->ij", M.gw * on * own, vf, vf)
            up = 1.0 - own
            if (e, f) in M.nbr:
                e2, xi2, eta2 = M.neighbour_points(e, f)
                v2 = tensor_vals(M.Bp, xi2, eta2)[0]
                A[e * n:(e + 1) * n, e2 * n:(e2 + 1) * n] += np.einsum("q,qi,qj->ij", M.gw * on * up, vf, v2)
            elif psi_bc is not None:
                bf = M.bf_index[(e, f)]
                b[e * n:(e + 1) * n] -= np.einsum("q,qi->i", M.gw * on * up * psi_bc[d, bf], vf)
        A[e * n:(e + 1) * n, e * n:(e + 1) * n] += blk
    return A, b


def balance_residuals(pr, psi, d, phi_in=None, q_iso=None, q_dir=None, psi_bc=None, nq=None, pointwise=False):
    """Per-element particle balance (test function u = 1) for direction d:
    outflow - inflow + absorption - source, relative to the source scale
    (pointwise: upwind trace chosen at each face point)."""
    M = Mesh(pr, nq)
    om = np.asarray(pr.omega[d], dtype=float)
    res = np.zeros(pr.n_elem)
    scale = np.zeros(pr.n_elem)
    for e in range(pr.n_elem):
        xi, eta, W, x, F, J, v, gxi, geta = M.volume_data(e)
        val = v @ psi[e]
        src = np.zeros(len(W))
        if phi_in is not None:
            src += pr.sigma_s[e] / (4 * np.pi) * (v @ phi_in[e])
        if q_iso is not None:
            src += v @ q_iso[e]
        if q_dir is not None:
            src += q_dir[d, e]
        tot = np.sum(W * J * pr.sigma_t[e] * val) - np.sum(W * J * src)
        sc = abs(np.sum(W * J * pr.sigma_t[e] * val)) + abs(np.sum(W * J * src))
        for f in range(4):
            fxi, feta, fx, nds = M.face_data(e, f)
            on = nds @ om
            mine = tensor_vals(M.Bp, fxi, feta)[0] @ psi[e]
            if (e, f) in M.nbr:
                e2, xi2, eta2 = M.neighbour_points(e, f)
                other = tensor_vals(M.Bp, xi2, eta2)[0] @ psi[e2]
            else:
                other = psi_bc[d, M.bf_index[(e, f)]] if psi_bc is not None else np.zeros(M.nq)
            if pointwise:
                tr = np.where(on >= 0, mine, other)
            else:
                tr = mine if M.upwind_is_self(e, f, om) else other
            flux = np.sum(M.gw * on * tr)
            tot += flux
            sc += abs(flux)
        res[e] = tot
        scale[e] = sc
    return res, scale
