"""Seeded synthetic inputs for the DG S_N sweep (meshes, angular sets, materials).

This module only *describes problems*: control points and connectivity of
quadrilateral meshes (Sec. 3.1: elements are images of [0,1]^2 under a map
built from global control points and a Gauss-Lobatto nodal basis of order m),
level-symmetric discrete-ordinates sets (Sec. 5 uses level-symmetric S_N sets
without listing them), and per-element cross sections and sources (Eq.
eq:transport).  It holds none of the sweep's arithmetic; both the CPU oracle
and the HIP library consume the arrays produced here.

Conventions shared by every consumer of these arrays:
  * reference element [0,1]^2, coordinates (xi, eta);
  * element control points are listed lexicographically, xi fastest, at the
    Gauss-Lobatto points of order m; neighbouring elements share control
    points, so the mesh is conforming;
  * element e = i + nx*j on structured meshes;
  * the 2D angular set is the upper hemisphere (z > 0) of a 3D set, projected
    on the plane; weights sum to 4*pi.
"""
from __future__ import annotations

import dataclasses
import functools
import math
from typing import Optional

import numpy as np

SEED_BASE = 230104758

# Gauss-Lobatto points of order m on [0,1] used to place geometry control
# points (closed forms; these are the nodal points of the map, Sec. 3.1).
_GEOM_NODES = {
    1: (0.0, 1.0),
    2: (0.0, 0.5, 1.0),
    3: (0.0, 0.5 * (1.0 - 1.0 / math.sqrt(5.0)), 0.5 * (1.0 + 1.0 / math.sqrt(5.0)), 1.0),
}


@dataclasses.dataclass
class Problem:
    """One fixed-source transport problem (Eq. eq:transport, eq:trans_bc).

    Arrays (all numpy, C-contiguous):
      cp_xy   [n_cp, 2]       float64  control points
      elem_cp [n_elem, (m+1)^2] int32  element -> control point ids
      omega   [n_dir, 2]      float64  in-plane direction components
      weight  [n_dir]         float64  angular weights, sum 4*pi
      sigma_t [n_elem]        float64  total cross section
      sigma_s [n_elem]        float64  scattering cross section
      q_iso   [n_elem, n]     float64  isotropic source per steradian, nodal
                                       coefficients in the degree-p space
                                       (None = 0)
      q_dir   [n_dir, n_elem, Q] float64 direction-dependent source at volume
                                       quadrature points (None = 0)
      psi_bc  [n_dir, n_bf, nq] float64 inflow values at boundary-face
                                       quadrature points (None = vacuum)
    """

    name: str
    p: int
    m: int
    cp_xy: np.ndarray
    elem_cp: np.ndarray
    omega: np.ndarray
    weight: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q_iso: Optional[np.ndarray] = None
    q_dir: Optional[np.ndarray] = None
    psi_bc: Optional[np.ndarray] = None
    nq: int = 0
    nx: int = 0
    ny: int = 0

    @property
    def n_elem(self) -> int:
        return int(self.elem_cp.shape[0])

    @property
    def n_dir(self) -> int:
        return int(self.omega.shape[0])

    @property
    def n(self) -> int:
        return (self.p + 1) ** 2

    @property
    def nq_eff(self) -> int:
        return self.nq if self.nq > 0 else self.p + self.m

    @property
    def n_solves(self) -> int:
        return self.n_elem * self.n_dir


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------

def quad_mesh(nx: int, ny: int, m: int = 1, x0: float = 0.0, x1: float = 1.0,
              y0: float = 0.0, y1: float = 1.0):
    """Structured nx-by-ny mesh of [x0,x1]x[y0,y1] with order-m control points.

    Returns (cp_xy [n_cp,2] float64, elem_cp [n_elem,(m+1)^2] int32).
    """
    if m not in _GEOM_NODES:
        raise ValueError("geometry order m must be 1, 2 or 3")
    g = np.asarray(_GEOM_NODES[m])
    hx = (x1 - x0) / nx
    hy = (y1 - y0) / ny
    npx = m * nx + 1
    npy = m * ny + 1
    # 1D control point coordinates along each axis
    xs = np.empty(npx)
    ys = np.empty(npy)
    for i in range(nx):
        xs[m * i:m * i + m + 1] = x0 + (i + g) * hx
    for j in range(ny):
        ys[m * j:m * j + m + 1] = y0 + (j + g) * hy
    xs[-1] = x1
    ys[-1] = y1
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # [npy, npx]
    cp_xy = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    a = np.arange(m + 1)
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    bb, aa = np.meshgrid(a, a, indexing="ij")  # local index aa + (m+1)*bb
    aa = aa.ravel()
    bb = bb.ravel()
    elem_cp = ((m * ii[:, None] + aa[None, :]) + npx * (m * jj[:, None] + bb[None, :]))
    return cp_xy, np.ascontiguousarray(elem_cp.astype(np.int32))


def sine_warp(cp_xy: np.ndarray, amp: float, k: float = 1.0) -> np.ndarray:
    """Displace control points by amp*sin(k pi x) sin(k pi y) * (1, 1).

    Same family as the sine distortion of Sec. 8 (curved-mesh solver study);
    on the unit square the boundary is invariant for integer k.
    """
    x = cp_xy[:, 0]
    y = cp_xy[:, 1]
    s = amp * np.sin(k * np.pi * x) * np.sin(k * np.pi * y)
    out = cp_xy.copy()
    out[:, 0] = x + s
    out[:, 1] = y + s
    return out


def taylor_green_mesh(n: int, m: int = 3, t_final: float = 0.3 * math.pi, steps: int = 300,
                      vortices: int = 1):
    """n-by-n order-m mesh of the unit square distorted by the Taylor-Green
    vortex (Sec. 8, method of manufactured solutions): every control point is
    advected by v = (sin x cos y, -cos x sin y) up to t_final with `steps`
    forward Euler steps.

    The printed velocity has no factor pi while the domain is the unit square;
    the reading used here advects on [0, pi]^2, where v . n = 0 on the
    boundary, and maps back to [0,1]^2, so the printed velocity and final
    time stand and boundary points slide along the boundary.  `vortices` > 1
    tiles vortices-by-vortices such cells (alternating sense of rotation), each
    covering n/vortices elements per side.  Longer t_final on coarse cells
    gives re-entrant faces (cyclic upwind graphs) but also nearly degenerate
    elements.  Returns (cp_xy, elem_cp) like quad_mesh."""
    cp, ec = quad_mesh(n, n, m)
    scale = math.pi * vortices
    y = cp * scale
    dt = t_final / steps
    for _ in range(steps):
        v = np.stack([np.sin(y[:, 0]) * np.cos(y[:, 1]), -np.cos(y[:, 0]) * np.sin(y[:, 1])], axis=1)
        y = y + dt * v
    out = y / scale
    # boundary points stay on their side (v . n = 0 there up to rounding)
    for k in range(2):
        out[np.abs(cp[:, k]) == 0.0, k] = 0.0
        out[cp[:, k] == 1.0, k] = 1.0
    return np.ascontiguousarray(out), ec


# --------------------------------------------------------------------------
# level-symmetric angular sets
# --------------------------------------------------------------------------

_LS16_MU1 = 0.1389568  # standard first cosine of the S16 level-symmetric set


def _ls_octant(N: int):
    """Index triples (i, j, k), 1-based, with i + j + k = N/2 + 2, lexicographic in (i, j)."""
    h = N // 2
    pts = []
    for i in range(1, h + 1):
        for j in range(1, h + 1):
            k = h + 2 - i - j
            if k >= 1:
                pts.append((i, j, k))
    return pts


def _ls_cosines(N: int, a: float) -> np.ndarray:
    """mu_i for i = 1..N/2 given a = mu_1^2 (equal spacing of mu_i^2)."""
    h = N // 2
    d = 2.0 * (1.0 - 3.0 * a) / (N - 2)
    return np.sqrt(a + d * np.arange(h))


def _ls_moment_matrix(N: int, mu: np.ndarray, classes, ks):
    pts = _ls_octant(N)
    M = np.zeros((len(ks), len(classes)))
    for (i, j, k) in pts:
        c = classes.index(tuple(sorted((i, j, k))))
        for r, kk in enumerate(ks):
            M[r, c] += mu[i - 1] ** (2 * kk)
    rhs = np.array([1.0 / (2 * kk + 1) for kk in ks])
    return M, rhs


@functools.lru_cache(maxsize=None)
def level_symmetric_octant(N: int):
    """Octant points and normalised weights (sum 1) of the level-symmetric S_N set.

    The cosines satisfy mu_i^2 = mu_1^2 + (i-1) * 2(1 - 3 mu_1^2)/(N-2); one
    weight per permutation class; the even moment conditions
    sum w mu^(2k) = 1/(2k+1), k = 0, 2, 3, ..., N/2 fix mu_1 and the weights
    for N <= 12.  For N = 16 the conditions leave freedom: mu_1 is set to the
    standard 0.1389568 and the minimum-norm weights are taken.
    Returns (mu [N/2], pts [(i,j,k)], w_point [len(pts)]).
    """
    if N < 2 or N % 2:
        raise ValueError("N must be even")
    if N == 2:
        mu = np.array([1.0 / math.sqrt(3.0)])
        return mu, [(1, 1, 1)], np.array([1.0])
    pts = _ls_octant(N)
    classes = sorted({tuple(sorted(t)) for t in pts})
    h = N // 2
    ks_all = [0] + list(range(2, h + 1))
    if N <= 12:
        ks_sq = ks_all[:len(classes)]
        ks_last = ks_all[len(classes):]
        assert len(ks_last) == 1

        def resid(a):
            mu = _ls_cosines(N, a)
            M, rhs = _ls_moment_matrix(N, mu, classes, ks_sq)
            try:
                w = np.linalg.solve(M, rhs)
            except np.linalg.LinAlgError:
                return float("nan"), None
            Ml, rl = _ls_moment_matrix(N, mu, classes, ks_last)
            return float((Ml @ w - rl)[0]), w

        # scan for sign changes of the last moment residual in a = mu_1^2
        grid = np.linspace(1e-4, 1.0 / 3.0 - 1e-4, 4001)
        vals = np.array([resid(a)[0] for a in grid])
        roots = []
        for t in range(len(grid) - 1):
            if not (np.isfinite(vals[t]) and np.isfinite(vals[t + 1])):
                continue
            if vals[t] == 0.0 or vals[t] * vals[t + 1] < 0:
                lo, hi = grid[t], grid[t + 1]
                flo = vals[t]
                for _ in range(200):
                    mid = 0.5 * (lo + hi)
                    fm = resid(mid)[0]
                    if fm == 0.0:
                        lo = hi = mid
                        break
                    if (fm < 0) == (flo < 0):
                        lo, flo = mid, fm
                    else:
                        hi = mid
                a = 0.5 * (lo + hi)
                _, w = resid(a)
                if w is not None and np.all(w > 0):
                    roots.append((a, w))
        if not roots:
            raise RuntimeError("no positive level-symmetric set for N=%d" % N)
        # the standard set is the one with the largest mu_1 among positive solutions
        a, wc = max(roots, key=lambda t: t[0])
        mu = _ls_cosines(N, a)
    else:
        a = _LS16_MU1 ** 2 if N == 16 else None
        if a is None:
            raise ValueError("level-symmetric sets provided for N = 2..12 and 16")
        mu = _ls_cosines(N, a)
        M, rhs = _ls_moment_matrix(N, mu, classes, ks_all)
        wc = np.linalg.lstsq(M, rhs, rcond=None)[0]
        if not np.all(wc > 0):
            raise RuntimeError("LS16 minimum-norm weights not positive")
    w_pt = np.array([wc[classes.index(tuple(sorted(t)))] for t in pts])
    return mu, pts, w_pt


def level_symmetric_2d(N: int):
    """2D S_N set: the four upper octants, weights summing to 4 pi.

    Order: octants (+,+), (-,+), (-,-), (+,-); inside an octant lexicographic
    in (i, j).  Omega = (sx mu_i, sy mu_j); the dropped z component is mu_k.
    Returns (omega [N(N+2)/2, 2], weight [N(N+2)/2]).
    """
    mu, pts, w_pt = level_symmetric_octant(N)
    mu = np.array(mu)
    om = []
    wt = []
    for sx, sy in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        for (i, j, k), w in zip(pts, w_pt):
            om.append((sx * mu[i - 1], sy * mu[j - 1]))
            wt.append(w * math.pi)
    return np.array(om, dtype=np.float64), np.array(wt, dtype=np.float64)


# --------------------------------------------------------------------------
# materials and configurations
# --------------------------------------------------------------------------

def block_log_uniform(nx, ny, block, lo, hi, rng):
    """sigma per element, log-uniform in [lo, hi] per block x block tile (tile-major draws)."""
    nbx = (nx + block - 1) // block
    nby = (ny + block - 1) // block
    draws = 10.0 ** rng.uniform(math.log10(lo), math.log10(hi), size=nbx * nby)
    i = np.arange(nx)[None, :] // block
    j = np.arange(ny)[:, None] // block
    return np.ascontiguousarray(draws[(i + nbx * j)].ravel().astype(np.float64))


def _const_source(n_elem, p, value=1.0):
    return np.full((n_elem, (p + 1) ** 2), value, dtype=np.float64)


def make_problem(name, nx, ny, p, m, N, sigma_t, sigma_s, q=1.0, warp=0.0):
    cp, ec = quad_mesh(nx, ny, m)
    if warp:
        cp = sine_warp(cp, warp, 1.0)
    om, wt = level_symmetric_2d(N)
    st = np.broadcast_to(np.asarray(sigma_t, dtype=np.float64), (nx * ny,)).copy()
    ss = np.broadcast_to(np.asarray(sigma_s, dtype=np.float64), (nx * ny,)).copy()
    return Problem(name=name, p=p, m=m, cp_xy=cp, elem_cp=ec, omega=om, weight=wt,
                   sigma_t=st, sigma_s=ss, q_iso=_const_source(nx * ny, p, q), nx=nx, ny=ny)


def make_tg_problem(name, n, p, m, N, sigma_t, sigma_s, q=1.0, t_final=0.3 * math.pi, vortices=1):
    """Problem on taylor_green_mesh(n, m, t_final, vortices=vortices) with an
    isotropic source q and vacuum inflow."""
    cp, ec = taylor_green_mesh(n, m, t_final, vortices=vortices)
    om, wt = level_symmetric_2d(N)
    st = np.broadcast_to(np.asarray(sigma_t, dtype=np.float64), (n * n,)).copy()
    ss = np.broadcast_to(np.asarray(sigma_s, dtype=np.float64), (n * n,)).copy()
    return Problem(name=name, p=p, m=m, cp_xy=cp, elem_cp=ec, omega=om, weight=wt,
                   sigma_t=st, sigma_s=ss, q_iso=_const_source(n * n, p, q), nx=n, ny=n)


def nonconvex_quad_mesh(n: int, amp: float, max_reflex: float, rng) -> tuple:
    """n-by-n straight-sided (m = 1) mesh of the unit square whose interior
    vertices are moved by independent uniform offsets in [-amp h, amp h]^2.
    Quads may have one reflex corner, which makes some upwind graphs cyclic
    (re-entrant faces, as on the Lagrangian-hydrodynamics mesh of the
    thick-diffusion-limit study); a quad whose most negative corner area (the
    cross product of the two edges leaving a corner) is below -max_reflex
    times the mean of its four corner areas has the offsets of its vertices
    halved, until none is.  Returns (cp_xy, elem_cp) like quad_mesh."""
    cp, ec = quad_mesh(n, n, 1)
    h = 1.0 / n
    inner = (cp[:, 0] > 0.0) & (cp[:, 0] < 1.0) & (cp[:, 1] > 0.0) & (cp[:, 1] < 1.0)
    disp = np.zeros_like(cp)
    disp[inner] = rng.uniform(-amp * h, amp * h, size=(int(inner.sum()), 2))
    ccw = ec[:, [0, 1, 3, 2]]
    for _ in range(64):
        x = (cp + disp)[ccw]
        nxt = np.roll(x, -1, axis=1) - x
        prv = np.roll(x, 1, axis=1) - x
        area = nxt[..., 0] * prv[..., 1] - nxt[..., 1] * prv[..., 0]
        bad = area.min(axis=1) < -max_reflex * area.mean(axis=1)
        if not bad.any():
            return np.ascontiguousarray(cp + disp), ec
        disp[np.unique(ccw[bad])] *= 0.5
    raise RuntimeError("nonconvex_quad_mesh: offsets did not settle")


def reentrant_quads(n: int = 64, p: int = 2, N: int = 8, seed: Optional[int] = None):
    """Workload with re-entrant faces: nonconvex_quad_mesh(n, 0.45, 0.2), p,
    S_N, sigma_t log-uniform [0.1, 100] per 8x8 block, c = 0.9, unit
    isotropic source, vacuum.  At 64x64 and S8 about an eighth of the
    element-direction pairs have a lagged inflow face."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7 if seed is None else seed))
    cp, ec = nonconvex_quad_mesh(n, 0.45, 0.2, rng)
    om, wt = level_symmetric_2d(N)
    st = block_log_uniform(n, n, 8, 0.1, 100.0, rng)
    return Problem(name="reentrant_%d" % n, p=p, m=1, cp_xy=cp, elem_cp=ec, omega=om, weight=wt,
                   sigma_t=st, sigma_s=0.9 * st, q_iso=_const_source(n * n, p, 1.0), nx=n, ny=n)


CONFIG_NAMES = ("c1", "c2", "c3", "c4", "c5")


def make_config(name: str, seed: Optional[int] = None, scale: Optional[int] = None):
    """The five benchmark/parity workloads as lists of Problems.

    c1: 8x8 unit square, p=1, S4, sigma_t=1, sigma_s=0, q=1, vacuum, one sweep
    c2: 64x64, p=2, S8, sigma_t log-uniform [0.1,100] per 8x8 block, c=0.9,
        50 source iterations
    c3: 256x256, m=2 curved by 0.1 sin(pi x) sin(pi y)(1,1), p=3, S12,
        sigma_t ~ U[1,10] per element, c=0.5
    c4: 64 problems, sides U{16..128}, p U{1..4}, S_N with N U{4..12 even},
        sigma_t log-uniform [0.1,100] per 8x8 block, c=0.9
    c5: 512x512, p=4, S16, sigma_t=1000, sigma_s=999.9
    `scale` (optional) replaces the mesh side, for reduced-size parity runs.
    Returns (problems, run) where run = dict(n_iter=..., precision=...).
    """
    idx = CONFIG_NAMES.index(name)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + idx if seed is None else seed))
    if name == "c1":
        n = scale or 8
        pr = make_problem("c1", n, n, 1, 1, 4, 1.0, 0.0)
        return [pr], dict(n_iter=1, precision="fp64")
    if name == "c2":
        n = scale or 64
        st = block_log_uniform(n, n, 8, 0.1, 100.0, rng)
        pr = make_problem("c2", n, n, 2, 1, 8, st, 0.9 * st)
        return [pr], dict(n_iter=50, precision="fp64")
    if name == "c3":
        n = scale or 256
        st = rng.uniform(1.0, 10.0, size=n * n)
        pr = make_problem("c3", n, n, 3, 2, 12, st, 0.5 * st, warp=0.1)
        return [pr], dict(n_iter=1, precision="fp32")
    if name == "c4":
        probs = []
        count = 64
        for k in range(count):
            side = int(rng.integers(16, 129)) if scale is None else int(rng.integers(2, scale + 1))
            p = int(rng.integers(1, 5))
            N = int(rng.choice([4, 6, 8, 10, 12]))
            st = block_log_uniform(side, side, 8, 0.1, 100.0, rng)
            probs.append(make_problem("c4_%02d" % k, side, side, p, 1, N, st, 0.9 * st))
        return probs, dict(n_iter=1, precision="fp32")
    if name == "c5":
        n = scale or 512
        pr = make_problem("c5", n, n, 4, 1, 16, 1000.0, 999.9)
        return [pr], dict(n_iter=1, precision="fp32")
    raise ValueError(name)
