"""ctypes wrapper of the serial FP64 oracle (oracle/vef_oracle.c).

Test infrastructure only.  Every function takes a `Problem` from
paper_2301_04758_amd.problems (the shared seeded input generator) and returns
numpy arrays.  The C source is compiled with gcc -O2 (no fast-math) into
oracle/liboracle.so by build_oracle(); the loader builds it only when it is
missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vef_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
ERR_INVALID = -1
ERR_CYCLE = -2
ERR_JACOBIAN = -3


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with status %d" % (what, code))
        self.code = code


def build_oracle(out=_LIB):
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fopenmp", "-fPIC", "-shared", "-o", out, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        _lib = C.CDLL(_LIB)
        _setup(_lib)
    return _lib


class _Prob(C.Structure):
    _fields_ = [("p", C.c_int), ("m", C.c_int), ("nq", C.c_int),
                ("n_elem", C.c_int), ("n_cp", C.c_int),
                ("cp_xy", C.c_void_p), ("elem_cp", C.c_void_p),
                ("n_dir", C.c_int), ("omega", C.c_void_p), ("weight", C.c_void_p),
                ("sigma_t", C.c_void_p), ("sigma_s", C.c_void_p), ("fixup", C.c_int), ("lag", C.c_int),
                ("pointwise", C.c_int), ("threads", C.c_int)]


_DP = C.POINTER(C.c_double)
_IP = C.POINTER(C.c_int)


def _setup(L):
    P = C.POINTER(_Prob)
    L.oracle_gl_nodes.argtypes = [C.c_int, _DP]
    L.oracle_gauss_rule.argtypes = [C.c_int, _DP, _DP]
    L.oracle_sweep.argtypes = [P, _DP, _DP, _DP, _DP, _IP, C.c_int, _DP, _DP, _DP, _DP, _IP]
    L.oracle_boundary_faces.argtypes = [P, _IP]
    L.oracle_qp_coords.argtypes = [P, _DP, _DP, _DP]
    L.oracle_geometry_report.argtypes = [P, _DP, _DP, _DP]
    L.oracle_levels.argtypes = [P, _IP, _IP]
    L.oracle_moments_from_psi.argtypes = [P, _DP, _DP]
    L.oracle_closures.argtypes = [P, _DP, _DP, _DP, _DP, _DP, _DP, _DP, _DP, _DP, _DP, _IP]
    L.oracle_source_iteration.argtypes = [P, _DP, _DP, _DP, _DP, C.c_int, C.c_double, _DP, _DP,
                                          _DP, _IP, _DP]
    for f in ("oracle_gl_nodes", "oracle_gauss_rule", "oracle_sweep", "oracle_boundary_faces",
              "oracle_qp_coords", "oracle_geometry_report", "oracle_levels",
              "oracle_moments_from_psi", "oracle_closures", "oracle_source_iteration"):
        getattr(L, f).restype = C.c_int


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_DP)


def _iptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_IP)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class _Bound:
    """Keeps the numpy arrays behind an oracle_problem struct alive."""

    def __init__(self, pr, nq=None, fixup=False, lag=False, pointwise=False, threads=1):
        self.cp = np.ascontiguousarray(pr.cp_xy, dtype=np.float64)
        self.ec = np.ascontiguousarray(pr.elem_cp, dtype=np.int32)
        self.om = np.ascontiguousarray(pr.omega, dtype=np.float64)
        self.wt = np.ascontiguousarray(pr.weight, dtype=np.float64)
        self.st = np.ascontiguousarray(pr.sigma_t, dtype=np.float64)
        self.ss = np.ascontiguousarray(pr.sigma_s, dtype=np.float64)
        self.s = _Prob(pr.p, pr.m, int(pr.nq if nq is None else nq), self.ec.shape[0], self.cp.shape[0],
                       self.cp.ctypes.data, self.ec.ctypes.data, self.om.shape[0], self.om.ctypes.data,
                       self.wt.ctypes.data, self.st.ctypes.data, self.ss.ctypes.data, 1 if fixup else 0,
                       1 if lag else 0, 1 if pointwise else 0, int(threads))
        self.nq = self.s.nq if self.s.nq > 0 else pr.p + pr.m
        self.n = (pr.p + 1) ** 2
        self.Q = self.nq * self.nq

    @property
    def ref(self):
        return C.byref(self.s)


def _check(rc, what):
    if rc < 0:
        raise OracleError(rc, what)
    return rc


def gl_nodes(k):
    z = np.zeros(k + 1)
    _check(lib().oracle_gl_nodes(k, _dptr(z)), "gl_nodes")
    return z


def gauss_rule(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().oracle_gauss_rule(n, _dptr(x), _dptr(w)), "gauss_rule")
    return x, w


def n_boundary_faces(pr, nq=None):
    b = _Bound(pr, nq)
    return _check(lib().oracle_boundary_faces(b.ref, None), "boundary_faces")


def boundary_faces(pr, nq=None):
    b = _Bound(pr, nq)
    nb = n_boundary_faces(pr, nq)
    out = np.zeros((nb, 2), dtype=np.int32)
    _check(lib().oracle_boundary_faces(b.ref, _iptr(out)), "boundary_faces")
    return out


def qp_coords(pr, nq=None):
    """(vol_xy [n_elem,Q,2], bnd_xy [n_bf,nq,2], bnd_normal [n_bf,nq,2])."""
    b = _Bound(pr, nq)
    nb = n_boundary_faces(pr, nq)
    v = np.zeros((pr.n_elem, b.Q, 2))
    bx = np.zeros((nb, b.nq, 2))
    bn = np.zeros((nb, b.nq, 2))
    _check(lib().oracle_qp_coords(b.ref, _dptr(v), _dptr(bx), _dptr(bn)), "qp_coords")
    return v, bx, bn


def geometry_report(pr, nq=None):
    b = _Bound(pr, nq)
    a = C.c_double()
    c = C.c_double()
    m = C.c_double()
    _check(lib().oracle_geometry_report(b.ref, C.byref(a), C.byref(c), C.byref(m)), "geometry_report")
    return a.value, c.value, m.value


def levels(pr, nq=None, lag=False, pointwise=False):
    b = _Bound(pr, nq, lag=lag, pointwise=pointwise)
    out = np.zeros(pr.n_dir, dtype=np.int32)
    _check(lib().oracle_levels(b.ref, _iptr(out), None), "levels")
    return out


def lagged_couplings(pr, nq=None, pointwise=False):
    """Lagged (element, face) couplings per direction of the lagged sweep order."""
    b = _Bound(pr, nq, lag=True, pointwise=pointwise)
    lv = np.zeros(pr.n_dir, dtype=np.int32)
    out = np.zeros(pr.n_dir, dtype=np.int32)
    _check(lib().oracle_levels(b.ref, _iptr(lv), _iptr(out)), "levels")
    return out


def sweep(pr, phi_in=None, dirs=None, want_psi=True, nq=None, q_iso="problem", q_dir="problem",
          psi_bc="problem", fixup=False, lag=False, psi_prev=None, pointwise=False, threads=1):
    """One sweep.  Returns dict(psi [n_sel,n_elem,n] or None, mom [6,n_elem,n],
    bnd [n_bf,nq,2], levels [n_sel]).  fixup: set-to-zero-and-scale
    negative-flux fixup after each local solve.  lag: cyclic upwind graphs
    are swept with lagged couplings, which read psi_prev [n_sel,n_elem,n]
    (None = 0).  pointwise: the upwind side is chosen at each face point
    (faces with both signs need lag).  threads > 1: that many directions at
    a time on OpenMP threads (same results, summed in direction order)."""
    b = _Bound(pr, nq, fixup, lag, pointwise, threads)
    psi_prev = _f64(psi_prev)
    q_iso = _f64(pr.q_iso if isinstance(q_iso, str) else q_iso)
    q_dir = _f64(pr.q_dir if isinstance(q_dir, str) else q_dir)
    psi_bc = _f64(pr.psi_bc if isinstance(psi_bc, str) else psi_bc)
    phi_in = _f64(phi_in)
    dl = None if dirs is None else np.ascontiguousarray(dirs, dtype=np.int32)
    n_sel = pr.n_dir if dl is None else len(dl)
    nb = n_boundary_faces(pr, nq)
    psi = np.zeros((n_sel, pr.n_elem, b.n)) if want_psi else None
    mom = np.zeros((6, pr.n_elem, b.n))
    bnd = np.zeros((nb, b.nq, 2))
    lv = np.zeros(n_sel, dtype=np.int32)
    rc = lib().oracle_sweep(b.ref, _dptr(phi_in), _dptr(q_iso), _dptr(q_dir), _dptr(psi_bc), _iptr(dl),
                            n_sel, _dptr(psi_prev), _dptr(psi), _dptr(mom), _dptr(bnd), _iptr(lv))
    _check(rc, "sweep")
    return dict(psi=psi, mom=mom, bnd=bnd, levels=lv)


def moments_from_psi(pr, psi, nq=None):
    b = _Bound(pr, nq)
    psi = _f64(psi)
    mom = np.zeros((6, pr.n_elem, b.n))
    _check(lib().oracle_moments_from_psi(b.ref, _dptr(psi), _dptr(mom)), "moments_from_psi")
    return mom


def closures(pr, mom, bnd, nq=None, q_iso="problem", q_dir="problem", psi_bc="problem"):
    """dict(E [3,n_elem,Q], Eb [n_bf,nq], Jin [n_bf,nq], Q0 [n_elem,Q], Q1 [2,n_elem,Q], n_nonpos)."""
    b = _Bound(pr, nq)
    q_iso = _f64(pr.q_iso if isinstance(q_iso, str) else q_iso)
    q_dir = _f64(pr.q_dir if isinstance(q_dir, str) else q_dir)
    psi_bc = _f64(pr.psi_bc if isinstance(psi_bc, str) else psi_bc)
    nb = n_boundary_faces(pr, nq)
    E = np.zeros((3, pr.n_elem, b.Q))
    Eb = np.zeros((nb, b.nq))
    Jin = np.zeros((nb, b.nq))
    Q0 = np.zeros((pr.n_elem, b.Q))
    Q1 = np.zeros((2, pr.n_elem, b.Q))
    nn = C.c_int()
    rc = lib().oracle_closures(b.ref, _dptr(_f64(mom)), _dptr(_f64(bnd)), _dptr(q_iso), _dptr(q_dir),
                               _dptr(psi_bc), _dptr(E), _dptr(Eb), _dptr(Jin), _dptr(Q0), _dptr(Q1),
                               C.byref(nn))
    _check(rc, "closures")
    return dict(E=E, Eb=Eb, Jin=Jin, Q0=Q0, Q1=Q1, n_nonpos=nn.value)


def source_iteration(pr, n_iter, tol=0.0, phi0=None, nq=None, fixup=False, lag=False, psi0=None,
                     want_psi=False, pointwise=False, threads=1):
    """dict(mom [6,n_elem,n] of the last sweep, bnd, resid [iters], iters, psi).
    lag: lagged sweeps of cyclic graphs; their first sweep reads psi0
    [n_dir,n_elem,n] (None = 0).  psi: the last sweep's angular flux when
    want_psi, else None.  pointwise, threads: as in sweep."""
    b = _Bound(pr, nq, fixup, lag, pointwise, threads)
    psi = None
    if want_psi or psi0 is not None:
        psi = np.zeros((pr.n_dir, pr.n_elem, b.n)) if psi0 is None else np.array(psi0, dtype=np.float64)
    nb = n_boundary_faces(pr, nq)
    mom = np.zeros((6, pr.n_elem, b.n))
    bnd = np.zeros((nb, b.nq, 2))
    res = np.zeros(n_iter)
    it = C.c_int()
    rc = lib().oracle_source_iteration(b.ref, _dptr(_f64(phi0)), _dptr(_f64(pr.q_iso)), _dptr(_f64(pr.q_dir)),
                                       _dptr(_f64(pr.psi_bc)), int(n_iter), float(tol), _dptr(mom),
                                       _dptr(bnd), _dptr(res), C.byref(it), _dptr(psi))
    _check(rc, "source_iteration")
    return dict(mom=mom, bnd=bnd, resid=res[:it.value], iters=it.value, psi=psi if want_psi else None)
