"""Element-local blocks of the hybridized Raviart-Thomas (HRT) VEF method and
their inverse -- TEST INFRASTRUCTURE ONLY (plain numpy, double precision).

Follows Sec. 7 (hybridization, "Implementation Details"): on each element K
the local VEF problem couples the current J in D_p(K) (the RT_p space of
Sec. 4: reference space Q_{p+1,p} x Q_{p,p+1} mapped by the contravariant
Piola transform, Eq. eq:piola) and the scalar flux phi in Q_p(K):

  A[i][j] = int_K sigma_t v_i . v_j dx
            + int_{dK cap Gamma_b} (1/E_b) (v_i . E n)(v_j . n) ds     (Eq. eq:A)
  G[i][j] = - int_K grad v_i : E phi_j dx                             (hat G)
  D[i][j] = int_K u_i div v_j dx                                      (Eq. eq:D)
  Ma[i][j] = int_K sigma_a u_i u_j dx                                 (Eq. eq:Ma)

and the inverse of [[A, G], [D, Ma]] has the blocks W, X, Y, Z of Eq.
eq:block_inv.  Everything is evaluated in physical form at each quadrature
point: v = F v_hat / J and grad v = F (grad_hat v_hat) F^{-1} / J (Eq.
eq:piola_grad; the correction term B_hat vanishes on affine elements, the
only ones treated here), integrated with the Jacobian.

Readings fixed here (shared with the library, which computes the same
quantities its own way):
  * RT nodal basis: Gauss-Lobatto points in the component's own direction,
    Gauss-Legendre points across it (the figure of Sec. 4); xi component
    functions first (node a + (p+2) b), then eta component (a + (p+1) b);
  * phi basis: Lagrange through the tensor Gauss-Legendre points (Sec. 8
    intro), node a + (p+1) b;
  * E = P / phi at each point from the transport moments (Lagrange basis
    through Gauss-Lobatto points), the isotropic I/3 where phi <= 0; E_b as
    given, 1/2 where it is not positive;
  * quadrature: the tensor Gauss-Legendre rule of the transport tables
    (nq >= p + 2 points per direction, exact for the RT mass on affine
    elements); boundary faces use the same nq points, ascending in the
    counter-clockwise face parameter.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def _lagrange(z, x):
    """Values and derivatives of the Lagrange polynomials through nodes z at
    points x: ([len(x), len(z)], [len(x), len(z)]), product forms."""
    z = np.asarray(z, dtype=float)
    x = np.asarray(x, dtype=float)
    k = len(z)
    val = np.ones((len(x), k))
    der = np.zeros((len(x), k))
    for a in range(k):
        others = [b for b in range(k) if b != a]
        den = np.prod([z[a] - z[b] for b in others])
        for b in others:
            val[:, a] *= (x - z[b])
        for c in others:
            term = np.ones(len(x))
            for b in others:
                if b != c:
                    term *= (x - z[b])
            der[:, a] += term
        val[:, a] /= den
        der[:, a] /= den
    return val, der


def legendre_points(k):
    """k Gauss-Legendre points on [0,1]."""
    return O.gauss_rule(k)[0]


def sizes(p):
    nx = (p + 2) * (p + 1)
    return 2 * nx, (p + 1) ** 2


def rt_basis(p, xi, eta):
    """Reference RT_p basis at points: values [npt, n_v, 2] and gradients
    [npt, n_v, 2, 2] (component, derivative direction)."""
    lob = O.gl_nodes(p + 1)
    leg = legendre_points(p + 1)
    Lx, dLx = _lagrange(lob, xi)
    Gx, dGx = _lagrange(leg, xi)
    Ly, dLy = _lagrange(lob, eta)
    Gy, dGy = _lagrange(leg, eta)
    n_v, _ = sizes(p)
    npt = len(xi)
    val = np.zeros((npt, n_v, 2))
    grad = np.zeros((npt, n_v, 2, 2))
    i = 0
    for b in range(p + 1):
        for a in range(p + 2):  # xi component: Lobatto in xi, Legendre in eta
            val[:, i, 0] = Lx[:, a] * Gy[:, b]
            grad[:, i, 0, 0] = dLx[:, a] * Gy[:, b]
            grad[:, i, 0, 1] = Lx[:, a] * dGy[:, b]
            i += 1
    for b in range(p + 2):
        for a in range(p + 1):  # eta component: Legendre in xi, Lobatto in eta
            val[:, i, 1] = Gx[:, a] * Ly[:, b]
            grad[:, i, 1, 0] = dGx[:, a] * Ly[:, b]
            grad[:, i, 1, 1] = Gx[:, a] * dLy[:, b]
            i += 1
    return val, grad


def phi_basis(p, xi, eta):
    leg = legendre_points(p + 1)
    Gx, _ = _lagrange(leg, xi)
    Gy, _ = _lagrange(leg, eta)
    return np.einsum("qa,qb->qba", Gx, Gy).reshape(len(xi), -1)


def transport_basis(p, xi, eta):
    lob = O.gl_nodes(p)
    Lx, _ = _lagrange(lob, xi)
    Ly, _ = _lagrange(lob, eta)
    return np.einsum("qa,qb->qba", Lx, Ly).reshape(len(xi), -1)


def face_points(f, s):
    """Reference points of face f at counter-clockwise parameter s."""
    s = np.asarray(s, dtype=float)
    one, zero = np.ones_like(s), np.zeros_like(s)
    return {0: (s, zero), 1: (one, s), 2: (1 - s, one), 3: (zero, 1 - s)}[f]


def affine_frames(pr):
    """(x0 [ne,2], F [ne,2,2]) of affine element maps x = x0 + F xi, from the
    corner control points; raises if an element is not a parallelogram."""
    m = pr.m
    ec = np.asarray(pr.elem_cp)
    cp = np.asarray(pr.cp_xy, dtype=float)
    x00 = cp[ec[:, 0]]
    x10 = cp[ec[:, m]]
    x01 = cp[ec[:, m * (m + 1)]]
    x11 = cp[ec[:, (m + 1) ** 2 - 1]]
    scale = np.abs(cp).max() + 1.0
    if np.abs(x11 - x10 - x01 + x00).max() > 1e-12 * scale:
        raise ValueError("HRT local blocks are defined here for affine (parallelogram) elements only")
    F = np.stack([x10 - x00, x01 - x00], axis=-1)  # columns t1, t2
    return x00, F


def eddington_from_moments(pr, mom, xi, eta):
    """E [ne, npt, 2, 2] = P / phi at reference points from nodal transport
    moments mom [6, ne, (p+1)^2]; I/3 where phi <= 0."""
    B = transport_basis(pr.p, xi, eta)
    ph = np.einsum("qj,ej->eq", B, mom[0])
    pxx = np.einsum("qj,ej->eq", B, mom[3])
    pxy = np.einsum("qj,ej->eq", B, mom[4])
    pyy = np.einsum("qj,ej->eq", B, mom[5])
    E = np.zeros(ph.shape + (2, 2))
    pos = ph > 0
    safe = np.where(pos, ph, 1.0)
    E[..., 0, 0] = np.where(pos, pxx / safe, 1.0 / 3.0)
    E[..., 0, 1] = E[..., 1, 0] = np.where(pos, pxy / safe, 0.0)
    E[..., 1, 1] = np.where(pos, pyy / safe, 1.0 / 3.0)
    return E


def local_blocks(pr, nq, E_vol, E_bnd=None, Eb=None):
    """A, G, D, Ma of every element.

    E_vol [ne, nq*nq, 2, 2] at the volume Gauss points (index qx + nq qy);
    E_bnd [n_bf, nq, 2, 2] and Eb [n_bf, nq] at the boundary-face points
    (faces in ascending (element, face) order); boundary terms are skipped
    when E_bnd is None.  Returns dict(A [ne,nv,nv], G [ne,nv,nphi],
    D [ne,nphi,nv], Ma [ne,nphi,nphi])."""
    p = pr.p
    x0, F = affine_frames(pr)
    J = F[:, 0, 0] * F[:, 1, 1] - F[:, 0, 1] * F[:, 1, 0]
    Finv = np.linalg.inv(F)
    gx, gw = O.gauss_rule(nq)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    xi, eta = XI.ravel(), ETA.ravel()
    W = np.outer(gw, gw).ravel()
    vh, gh = rt_basis(p, xi, eta)
    u = phi_basis(p, xi, eta)
    st = np.asarray(pr.sigma_t, dtype=float)
    sa = st - np.asarray(pr.sigma_s, dtype=float)
    # physical values (Piola): v = F vh / J, grad v = F gh F^{-1} / J
    v = np.einsum("ekl,qil->eqik", F, vh) / J[:, None, None, None]
    gv = np.einsum("ekl,qilm,emn->eqikn", F, gh, Finv) / J[:, None, None, None, None]
    wJ = W[None, :] * J[:, None]
    A = np.einsum("eq,e,eqik,eqjk->eij", wJ, st, v, v)
    G = -np.einsum("eq,eqikn,eqkn,qj->eij", wJ, gv, E_vol, u)
    div = np.einsum("eqikk->eqi", gv)
    D = np.einsum("eq,qi,eqj->eij", wJ, u, div)
    Ma = np.einsum("eq,e,qi,qj->eij", wJ, sa, u, u)
    if E_bnd is not None:
        bf = O.boundary_faces(pr)
        for k, (e, f) in enumerate(bf):
            fx, fy = face_points(f, gx)
            vb, _ = rt_basis(p, fx, fy)
            vph = np.einsum("kl,qil->qik", F[e], vb) / J[e]
            # outward n ds: clockwise rotation of the face tangent d x / d s
            tang = {0: F[e][:, 0], 1: F[e][:, 1], 2: -F[e][:, 0], 3: -F[e][:, 1]}[f]
            nds = np.array([tang[1], -tang[0]])
            length = np.hypot(*nds)
            n = nds / length
            eb = np.where(Eb[k] > 0, Eb[k], 0.5)
            vEn = np.einsum("qik,qkl,l->qi", vph, E_bnd[k], n)
            vn = np.einsum("qik,k->qi", vph, n)
            A[e] += np.einsum("q,qi,qj->ij", gw * length / eb, vEn, vn)
    return dict(A=A, G=G, D=D, Ma=Ma)


def assemble_full(blk):
    top = np.concatenate([blk["A"], blk["G"]], axis=2)
    bot = np.concatenate([blk["D"], blk["Ma"]], axis=2)
    return np.concatenate([top, bot], axis=1)


def local_inverse(pr, nq, mom, Eb):
    """The inverse [[W, X], [Y, Z]] of every element's local block matrix,
    [ne, n, n], with E from the transport moments (volume and boundary-face
    points) and E_b as given [n_bf, nq]."""
    gx, _ = O.gauss_rule(nq)
    XI, ETA = np.meshgrid(gx, gx, indexing="xy")
    E_vol = eddington_from_moments(pr, mom, XI.ravel(), ETA.ravel())
    bf = O.boundary_faces(pr)
    E_bnd = np.zeros((len(bf), nq, 2, 2))
    for k, (e, f) in enumerate(bf):
        fx, fy = face_points(f, gx)
        E_bnd[k] = eddington_from_moments(pr, mom[:, e:e + 1], fx, fy)[0]
    blk = local_blocks(pr, nq, E_vol, E_bnd, np.asarray(Eb, dtype=float))
    return np.linalg.inv(assemble_full(blk)), blk


def schur_blocks(blk):
    """W, X, Y, Z by the formulas of Sec. 7 (S = Ma - D A^{-1} G)."""
    Ai = np.linalg.inv(blk["A"])
    S = blk["Ma"] - blk["D"] @ Ai @ blk["G"]
    Si = np.linalg.inv(S)
    W = Ai @ (np.eye(Ai.shape[-1]) + blk["G"] @ Si @ blk["D"] @ Ai)
    X = -Ai @ blk["G"] @ Si
    Y = -Si @ blk["D"] @ Ai
    return W, X, Y, Si
