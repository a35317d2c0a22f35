"""Host outer iteration of the transport / hybridized-RT VEF method (Sec. 2's
three-stage fixed point, with the hybridized discretisation of Sec. 7).

Each outer iteration:
  1. one transport sweep on the GPU (vef_sweep_run) whose scattering source
     is the previous VEF scalar flux, then the closures (vef_moments: E_b,
     J_in, Q_0, Q_1);
  2. the element-local HRT blocks and their inverse [[W, X], [Y, Z]] on the
     GPU (vef_hrt_local_inverse), E = P / phi from the sweep's moments;
  3. on the host: the interior-face couplings C_1 (Eq. eq:hyb_cts_n_vef) and
     C_2 (the lambda term of the local first-moment equation, with the
     average of E n from both sides), the right-hand sides g (Q_1 and the
     Miften-Larsen inflow term with J_in) and f (Q_0), the reduced system
     H lambda = sum_K C_1 (W g + X f), H = sum_K C_1 W C_2 (scipy sparse
     direct solve in place of the paper's AMG), and per element
     [J; phi] = [[W, X], [Y, Z]] [g - C_2 lambda; f];
  4. phi (Gauss-Legendre nodal Q_p) evaluated at the transport's
     Gauss-Lobatto nodes (the same polynomial) becomes the next scattering
     source.
Affine meshes only, like vef_hrt_local_inverse.  The lambda space on each
interior face is Lagrange of degree p through the Gauss-Legendre points in the
counter-clockwise parameter of the face's lower-numbered element.
"""
from __future__ import annotations

import numpy as np

from . import vef


def _gauss(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def _lobatto(k):
    inner = np.polynomial.legendre.Legendre.basis(k).deriv().roots()
    return np.sort(np.concatenate([[0.0], 0.5 * (np.real(inner) + 1.0), [1.0]]))


def _lagrange(z, x):
    """Values and derivatives [len(x), len(z)] (barycentric form)."""
    z = np.asarray(z, float)
    x = np.atleast_1d(np.asarray(x, float))
    k = len(z)
    bw = np.array([1.0 / np.prod([z[j] - z[l] for l in range(k) if l != j]) for j in range(k)])
    val = np.zeros((len(x), k))
    der = np.zeros((len(x), k))
    for i, xi in enumerate(x):
        d = xi - z
        hit = np.nonzero(d == 0.0)[0]
        if len(hit):
            j = hit[0]
            val[i, j] = 1.0
            for l in range(k):
                if l != j:
                    der[i, l] = (bw[l] / bw[j]) / (z[j] - z[l])
            der[i, j] = -der[i].sum()
            continue
        t = bw / d
        val[i] = t / t.sum()
        for j in range(k):
            der[i, j] = val[i, j] * sum(1.0 / d[l] for l in range(k) if l != j)
    return val, der


class _Ref:
    """Reference tables of degree p with nq Gauss points per direction."""

    def __init__(self, p, nq):
        self.p, self.nq = p, nq
        self.gx, self.gw = _gauss(nq)
        self.lob1 = _lobatto(p + 1)
        self.lob = _lobatto(p)
        self.leg, _ = _gauss(p + 1)
        self.nx = (p + 2) * (p + 1)
        self.nv = 2 * self.nx
        self.nphi = (p + 1) ** 2
        XI, ETA = np.meshgrid(self.gx, self.gx, indexing="xy")
        self.vxi, self.veta = XI.ravel(), ETA.ravel()
        self.W = np.outer(self.gw, self.gw).ravel()
        self.rt_vol = self.rt(self.vxi, self.veta)
        self.u_vol = self.tensor(self.leg, self.vxi, self.veta)
        self.leg_at_lob = self.tensor(self.leg, *self._grid(self.lob))  # [nT, nphi]

    @staticmethod
    def _grid(z):
        X, Y = np.meshgrid(z, z, indexing="xy")
        return X.ravel(), Y.ravel()

    def rt(self, x, y):
        """Reference RT_p vectors [npt, nv, 2] (xi-component functions first)."""
        p = self.p
        Lx, _ = _lagrange(self.lob1, x)
        Ly, _ = _lagrange(self.lob1, y)
        Gx, _ = _lagrange(self.leg, x)
        Gy, _ = _lagrange(self.leg, y)
        v = np.zeros((len(x), self.nv, 2))
        i = 0
        for b in range(p + 1):
            for a in range(p + 2):
                v[:, i, 0] = Lx[:, a] * Gy[:, b]
                i += 1
        for b in range(p + 2):
            for a in range(p + 1):
                v[:, i, 1] = Gx[:, a] * Ly[:, b]
                i += 1
        return v

    @staticmethod
    def tensor(z, x, y):
        Lx, _ = _lagrange(z, x)
        Ly, _ = _lagrange(z, y)
        return (Ly[:, :, None] * Lx[:, None, :]).reshape(len(x), -1)

    @staticmethod
    def face_xy(f, s):
        s = np.asarray(s, float)
        return {0: (s, 0 * s), 1: (1 + 0 * s, s), 2: (1 - s, 1 + 0 * s), 3: (0 * s, 1 - s)}[f]


class VefOuter:
    """Transport + HRT VEF outer iteration for one affine problem."""

    # normwise backward error of the device lambda solve above which its
    # re-used pivot order is replaced by a new host factorisation (a stable
    # LU stays within a small multiple of the unit round-off)
    REFACTOR_RESID = 1e-12

    def __init__(self, problem, nq=None, precision="fp64", device_reduce=True, lambda_solve="device"):
        p = problem.p
        if nq is None:
            nq = p + 2
        problem.nq = nq
        self.pr = problem
        self.ref = _Ref(p, nq)
        self.device_reduce = device_reduce
        if lambda_solve not in ("device", "host"):
            raise ValueError("lambda_solve is 'device' or 'host'")
        self.lambda_solve = lambda_solve
        self._lam = None
        self.host_factorisations = 0
        self.last_resid = None
        self.sw = vef.Sweep([problem], precision=precision)
        import scipy.sparse  # noqa: F401  (after the device is set up; fail early if missing)
        if not self.sw.info[0]["affine"]:
            self.sw.close()
            raise ValueError("the HRT outer iteration needs an affine mesh")
        self._setup_host(vef.vef_boundary_faces(self.sw.h, 0))
        self.history = []

    @classmethod
    def host_only(cls, problem, bf, nq=None):
        """The host stage alone (host_stage), with no device handle: for
        driving it from closures and block inverses computed elsewhere."""
        self = cls.__new__(cls)
        self.device_reduce = False
        self.lambda_solve = "host"
        self._lam = None
        problem.nq = nq or problem.p + 2
        self.pr = problem
        self.ref = _Ref(problem.p, problem.nq)
        self.sw = None
        self._setup_host(bf)
        self.history = []
        return self

    def _setup_host(self, bf):
        """Geometry and face numbering of the host stage; bf [n_bf, 2] the
        boundary faces (element, face) in the order of the closures."""
        problem = self.pr
        m = problem.m
        ec = np.asarray(problem.elem_cp)
        cp = np.asarray(problem.cp_xy, float)
        x00, x10, x01 = cp[ec[:, 0]], cp[ec[:, m]], cp[ec[:, m * (m + 1)]]
        self.F = np.stack([x10 - x00, x01 - x00], axis=-1)
        self.J = np.linalg.det(self.F)
        corner = {0: (0, m), 1: (m, (m + 1) ** 2 - 1), 2: ((m + 1) ** 2 - 1, m * (m + 1)), 3: (m * (m + 1), 0)}
        first = {}
        self.nbr = -np.ones((problem.n_elem, 4), dtype=np.int64)
        self.nbr_face = -np.ones((problem.n_elem, 4), dtype=np.int64)
        for e in range(problem.n_elem):
            for f in range(4):
                key = frozenset((int(ec[e, corner[f][0]]), int(ec[e, corner[f][1]])))
                if key in first:
                    e2, f2 = first.pop(key)
                    self.nbr[e, f], self.nbr_face[e, f] = e2, f2
                    self.nbr[e2, f2], self.nbr_face[e2, f2] = e, f
                else:
                    first[key] = (e, f)
        # interior faces, numbered by (lower element, its face)
        self.face_id = -np.ones((problem.n_elem, 4), dtype=np.int64)
        nf = 0
        for e in range(problem.n_elem):
            for f in range(4):
                e2 = self.nbr[e, f]
                if e2 > e:
                    self.face_id[e, f] = nf
                    self.face_id[e2, self.nbr_face[e, f]] = nf
                    nf += 1
        self.n_faces = nf
        self.bf = np.asarray(bf)
        self.bf_of = -np.ones((problem.n_elem, 4), dtype=np.int64)
        for k, (e, f) in enumerate(self.bf):
            self.bf_of[int(e), int(f)] = k

    def close(self):
        if getattr(self, "_lam", None) is not None:
            self._lam.close()
            self._lam = None
        if self.sw is not None:
            self.sw.close()

    # ------------------------------------------------------------ geometry
    @staticmethod
    def _eddington_all(Tb, mom):
        """E [ne, npt, 2, 2] = P / phi from basis values Tb [npt, nT] and
        moments [6, ne, nT]; I/3 where phi <= 0."""
        ph = np.einsum("qj,ej->eq", Tb, mom[0])
        pxx = np.einsum("qj,ej->eq", Tb, mom[3])
        pxy = np.einsum("qj,ej->eq", Tb, mom[4])
        pyy = np.einsum("qj,ej->eq", Tb, mom[5])
        E = np.zeros(ph.shape + (2, 2))
        pos = ph > 0
        safe = np.where(pos, ph, 1.0)
        E[..., 0, 0] = np.where(pos, pxx / safe, 1 / 3)
        E[..., 1, 1] = np.where(pos, pyy / safe, 1 / 3)
        E[..., 0, 1] = E[..., 1, 0] = np.where(pos, pxy / safe, 0.0)
        return E

    def _tb(self, f, s):
        return _Ref.tensor(self.ref.lob, *_Ref.face_xy(f, s))

    # ------------------------------------------------------------- one step
    def step(self, phi_lob=None):
        """One outer iteration from the transport scattering flux phi_lob
        [n_elem, (p+1)^2] (Gauss-Lobatto nodal; None = 0).  Returns the VEF
        scalar flux at the Gauss-Lobatto nodes and at the Gauss-Legendre
        nodes, and the current."""
        import time
        t0 = time.perf_counter()
        on_device = self.device_reduce and self.lambda_solve == "device" and self.n_faces > 0
        d = self._device_stage(phi_lob, keep_device=on_device)
        if on_device:
            import torch
            torch.cuda.synchronize()
        t1 = time.perf_counter()
        if on_device:
            out = self._solve_device(d)
        else:
            out = self._solve_reduced(**d) if "hloc" in d else self.host_stage(**d)
        # wall time of the transport and element-local stage (sweep,
        # closures, block inverses, reduction, and copies to the host where
        # the lambda system is solved there) and of the lambda solve with the
        # recovery of [J; phi]
        self.last_times = dict(stage_s=t1 - t0, solve_s=time.perf_counter() - t1)
        return out

    def _device_stage(self, phi_lob, keep_device=False):
        """Sweep, closures and block inverses on the GPU, and with
        device_reduce the element-local reduction too (vef_hrt_reduce);
        copied to the host unless keep_device (reduction results only)."""
        import torch
        io = self.sw.buffers(n_iter=1, store_psi=False, phi_in=phi_lob)
        self.sw.run(io, n_iter=1)
        mio = self.sw.moment_buffers(io)
        self.sw.moments(mio)
        inv = self.sw.hrt_local_inverse(0, io[0]["mom"], mio[0]["Eb"])
        if self.device_reduce:
            red = self.sw.hrt_reduce(0, io[0]["mom"], mio[0], inv)
            if keep_device:
                return red
            torch.cuda.synchronize()
            self.sw.check()
            return {k: v.cpu().numpy() for k, v in red.items()}
        torch.cuda.synchronize()
        self.sw.check()
        inv = inv.cpu().numpy()
        mom = io[0]["mom"].cpu().numpy()
        Eb = mio[0]["Eb"].cpu().numpy()
        Jin = mio[0]["Jin"].cpu().numpy()
        Q0 = mio[0]["Q0"].cpu().numpy()
        Q1 = mio[0]["Q1"].cpu().numpy()
        return dict(inv=inv, mom=mom, Eb=Eb, Jin=Jin, Q0=Q0, Q1=Q1)

    def host_stage(self, inv, mom, Eb, Jin, Q0, Q1):
        """Face couplings, right-hand sides, the reduced lambda system and its
        solve, and the element-by-element recovery of [J; phi].  inv
        [ne, n, n] the block inverses; mom [6, ne, (p+1)^2] the transport
        moments; Eb, Jin [n_bf, nq]; Q0 [ne, nq^2]; Q1 [2, ne, nq^2]."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spl
        pr, ref = self.pr, self.ref
        p, nv = pr.p, ref.nv
        ne = pr.n_elem
        P1 = p + 1
        # right-hand sides g, f and the face couplings C1_K, C2_K (local slots f*(p+1)+t)
        # The Piola map v = F v_hat / J gives v . a = v_hat . (F^T a) / J, so
        # every integral below is a product with the reference RT table
        # R [(q, l), i] of the physical vectors pulled back by F^T / J.
        Jinv = 1.0 / self.J
        Rvol = ref.rt_vol.transpose(0, 2, 1).reshape(-1, nv)
        FQ = np.einsum("ekl,keq->eql", self.F, Q1) * ref.W[None, :, None]
        g = FQ.reshape(ne, -1) @ Rvol
        fr = (ref.W[None, :] * self.J[:, None] * Q0) @ ref.u_vol
        C1 = np.zeros((ne, 4 * P1, nv))
        C2 = np.zeros((ne, nv, 4 * P1))
        lam_fwd, _ = _lagrange(ref.leg, ref.gx)
        lam_rev, _ = _lagrange(ref.leg, 1.0 - ref.gx)
        ids = np.arange(ne)
        for f in range(4):
            fx, fy = _Ref.face_xy(f, ref.gx)
            R = ref.rt(fx, fy).transpose(0, 2, 1).reshape(-1, nv)          # [(q, l), i]
            tang = self.F[:, :, f % 2] * (1.0 if f < 2 else -1.0)
            N = np.stack([tang[:, 1], -tang[:, 0]], axis=1)
            length = np.hypot(N[:, 0], N[:, 1])
            n = N / length[:, None]
            w = ref.gw[None, :] * length[:, None]
            E = self._eddington_all(self._tb(f, ref.gx), mom)
            bnd = self.nbr[:, f] < 0
            if bnd.any():
                e = ids[bnd]
                k = self.bf_of[e, f]
                eb = np.where(Eb[k] > 0, Eb[k], 0.5)
                FtEn = np.einsum("ekl,eqkm,em->eql", self.F[e], E[e], n[e])
                c = (2.0 * w[e] / eb * Jin[k] * Jinv[e][:, None])[:, :, None]
                g[e] += (c * FtEn).reshape(len(e), -1) @ R
            Ftn = np.einsum("ekl,ek->el", self.F, n)  # (the 1 / J is in lam below)
            for f2 in range(4):
                sel = (~bnd) & (self.nbr_face[:, f] == f2)
                if not sel.any():
                    continue
                e = ids[sel]
                e2 = self.nbr[e, f]
                E2 = self._eddington_all(self._tb(f2, 1.0 - ref.gx), mom[:, e2])
                FtEn = np.einsum("ekl,eqkm,em->eql", self.F[e], 0.5 * (E[e] + E2), n[e])
                lam = np.where((e < e2)[:, None, None], lam_fwd[None], lam_rev[None]) \
                    * (w[e] * Jinv[e][:, None])[:, :, None]                       # [e, q, t]
                T = (FtEn[:, :, :, None] * lam[:, :, None, :]).reshape(len(e), -1, P1)
                C2[e, :, f * P1:(f + 1) * P1] = np.matmul(R.T[None], T)
                U = (lam[:, :, None, :] * Ftn[e][:, None, :, None]).reshape(len(e), -1, P1)
                C1[e, f * P1:(f + 1) * P1, :] = np.matmul(U.transpose(0, 2, 1), R[None])
        # sol0 = inv [g; f], resp = inv [C2; 0]: the element's [J; phi] is
        # sol0 - resp lambda; H and r collect C1 W C2 and C1 (W g + X f)
        sol0 = np.matmul(inv, np.concatenate([g, fr], axis=1)[:, :, None])[:, :, 0]
        resp = np.matmul(inv[:, :, :nv], C2)
        return self._solve_reduced(hloc=np.matmul(C1, resp[:, :nv]), rloc=np.matmul(C1, sol0[:, :nv, None])[:, :, 0],
                                   sol0=sol0, resp=resp)

    def _gidx(self):
        """[ne, 4(p+1)]: the lambda unknown of each element slot f(p+1)+t
        (-1 on boundary faces)."""
        P1 = self.pr.p + 1
        fid = self.face_id[:, :, None]
        g = np.where(fid >= 0, fid * P1 + np.arange(P1)[None, None, :], -1)
        return g.reshape(self.pr.n_elem, 4 * P1)

    def _assemble_host(self, hloc, rloc):
        """H [n, n] (CSR) and r from the element contributions."""
        import scipy.sparse as sp
        P1 = self.pr.p + 1
        gidx = self._gidx()
        ok = gidx >= 0
        rows = np.repeat(gidx[:, :, None], 4 * P1, axis=2)
        cols = np.repeat(gidx[:, None, :], 4 * P1, axis=1)
        mask = ok[:, :, None] & ok[:, None, :]
        nl = self.n_faces * P1
        H = sp.csr_matrix((hloc[mask], (rows[mask], cols[mask])), shape=(nl, nl))
        rhs = np.zeros(nl)
        np.add.at(rhs, gidx[ok], rloc[ok])
        return H, rhs

    def _solve_device(self, red):
        """The reduced system on the device (vef.LambdaSolver): the first
        call factorises H on the host (SuperLU, fill-reducing column order)
        and later calls re-factorise with that pivot order; a relative
        residual above REFACTOR_RESID factorises the current H on the host
        again."""
        import scipy.sparse.linalg as spl
        ref = self.ref

        def factorise():
            H, _ = self._assemble_host(red["hloc"].cpu().numpy(), red["rloc"].cpu().numpy())
            lu = spl.splu(H.tocsc(), permc_spec="MMD_AT_PLUS_A")
            if self._lam is not None:
                self._lam.close()
            self._lam = vef.LambdaSolver(self._gidx(), ref.nv + ref.nphi, lu, red["hloc"], red["rloc"])
            self.host_factorisations += 1

        if self._lam is None:
            factorise()
        _, sol, resid = self._lam.solve(red["hloc"], red["rloc"], red["sol0"], red["resp"])
        if not resid <= self.REFACTOR_RESID:
            factorise()
            _, sol, resid = self._lam.solve(red["hloc"], red["rloc"], red["sol0"], red["resp"])
        self.sw.check()
        self.last_resid = resid
        sol = sol.cpu().numpy()
        Jc, phi_leg = sol[:, :ref.nv], sol[:, ref.nv:]
        return phi_leg @ ref.leg_at_lob.T, phi_leg, Jc

    def _solve_reduced(self, hloc, rloc, sol0, resp):
        """Assemble H lambda = r from the elements' hloc [ne, 4(p+1), 4(p+1)]
        and rloc [ne, 4(p+1)] by interior-face slot, solve it (scipy sparse
        LU), and recover [J; phi] = sol0 - resp lambda per element."""
        import scipy.sparse.linalg as spl
        pr, ref = self.pr, self.ref
        ne, P1, nv = pr.n_elem, pr.p + 1, ref.nv
        gidx = self._gidx()
        ok = gidx >= 0
        nl = self.n_faces * P1
        H, rhs = self._assemble_host(hloc, rloc)
        lam_g = spl.spsolve(H.tocsc(), rhs, permc_spec="MMD_AT_PLUS_A") if nl else np.zeros(0)
        lam_loc = np.where(ok, lam_g[np.where(ok, gidx, 0)] if nl else 0.0, 0.0)
        sol = sol0 - np.matmul(resp, lam_loc[:, :, None])[:, :, 0]
        Jc, phi_leg = sol[:, :nv], sol[:, nv:]
        phi_lob = phi_leg @ ref.leg_at_lob.T
        return phi_lob, phi_leg, Jc

    def solve(self, max_outer=50, tol=1e-8, phi0=None, anderson=0, stop="relative"):
        """Outer iterations on the VEF scalar flux x (Gauss-Legendre nodal;
        phi0 None = 0) until max|x_new - x_old| <= tol max|x_new| (stop =
        "relative"), or until max|x_new - x_old| <= tol (stop = "max_norm":
        the max norm of the difference of successive iterates, the paper's
        termination rule in Sec. 8).  anderson
        > 0 accelerates the fixed point x = G(x) (G: sweep, closures, VEF
        solve) with that many difference vectors, as the paper's outer solver
        does (Sec. 8 uses two): x_new = G(x) - dG gamma, gamma the least-squares
        fit of the residual f = G(x) - x by the last differences dF of
        residuals (dG the differences of G values).  anderson = 0 is the plain
        fixed point of Sec. 2.  Returns dict(phi_leg, phi_lob, J (of the last
        evaluation of G), iterations, history)."""
        if stop not in ("relative", "max_norm"):
            raise ValueError("stop must be 'relative' or 'max_norm'")
        ref = self.ref
        shape = (self.pr.n_elem, ref.nphi)
        x = np.zeros(shape) if phi0 is None else np.asarray(phi0, dtype=float).reshape(shape)
        dF, dG = [], []
        f_prev = g_prev = None
        self.history = []
        for it in range(1, max_outer + 1):
            _, g, Jc = self.step(None if (it == 1 and phi0 is None) else x @ ref.leg_at_lob.T)
            f = g - x
            x_new = g
            if anderson > 0 and f_prev is not None:
                dF.append((f - f_prev).ravel())
                dG.append((g - g_prev).ravel())
                if len(dF) > anderson:
                    dF.pop(0)
                    dG.pop(0)
                gamma = np.linalg.lstsq(np.stack(dF, axis=1), f.ravel(), rcond=None)[0]
                x_new = g - (np.stack(dG, axis=1) @ gamma).reshape(shape)
            f_prev, g_prev = f, g
            done = False
            if it > 1:
                r = float(np.abs(x_new - x).max())
                if stop == "relative":
                    r /= max(float(np.abs(x_new).max()), 1e-300)
                self.history.append(r)
                done = r <= tol
            x = x_new
            if done:
                break
        return dict(phi_leg=x, phi_lob=x @ ref.leg_at_lob.T, J=Jc, iterations=it, history=self.history)
