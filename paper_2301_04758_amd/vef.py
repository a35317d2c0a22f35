"""Thin ctypes binding of the C ABI in include/vef_sweep.h (argument marshalling only).

The functions vef_sweep_create / vef_sweep_run / vef_moments / vef_sweep_destroy
and the queries keep the C names and argument order.  Device buffers are
PyTorch tensors on the current HIP device (only their data pointers cross the
boundary); streams are torch streams (their hipStream_t handle crosses).
Every step of the sweep runs in the HIP library: if libvefsweep.so is missing
the import of this module fails.  There is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvefsweep.so")

VEF_OK = 0
VEF_ERR_INVALID = -1
VEF_ERR_CYCLE = -2
VEF_ERR_JACOBIAN = -3
VEF_ERR_HIP = -4
VEF_ERR_OOM = -5
VEF_ERR_TIMEOUT = -6
VEF_STATIC_RESID_MAX = 65536  # doubles of the static residual array (vef_sweep_run_static)
VEF_FP64 = 0
VEF_FP32_LOCAL = 1
VEF_CYCLES_REJECT = 0
VEF_CYCLES_LAG = 1
VEF_UPWIND_FACE, VEF_UPWIND_POINT = 0, 1
VEF_SCHEDULE_AUTO = 0
VEF_LEVEL_SYNC = 1
VEF_DIR_RESIDENT = 2
VEF_PERSISTENT = 3
SCHEDULES = {"auto": VEF_SCHEDULE_AUTO, "level": VEF_LEVEL_SYNC, "dir": VEF_DIR_RESIDENT, "persistent": VEF_PERSISTENT}
SCHEDULE_NAMES = {VEF_LEVEL_SYNC: "level_sync", VEF_DIR_RESIDENT: "dir_resident", VEF_PERSISTENT: "persistent"}
VEF_KERNEL_PIVOT, VEF_KERNEL_NOPIVOT, VEF_KERNEL_AFFINE, VEF_KERNEL_AFFINE_PIPELINE = 0, 1, 2, 3
VEF_KERNEL_BILINEAR_PIPELINE = 4
VEF_KERNEL_AFFINE_LU = 5
VEF_KERNEL_GENERAL_MAT = 6
VEF_KERNEL_AFFINE_SHARED = 7
KERNEL_NAMES = {VEF_KERNEL_PIVOT: "pivot", VEF_KERNEL_NOPIVOT: "nopivot", VEF_KERNEL_AFFINE: "affine",
                VEF_KERNEL_AFFINE_PIPELINE: "affine_pipeline", VEF_KERNEL_BILINEAR_PIPELINE: "bilinear_pipeline",
                VEF_KERNEL_AFFINE_LU: "affine_lu", VEF_KERNEL_GENERAL_MAT: "general_mat",
                VEF_KERNEL_AFFINE_SHARED: "affine_shared"}

EXPORTED = ("vef_sweep_create", "vef_sweep_run", "vef_sweep_run_static", "vef_moments", "vef_sweep_destroy", "vef_plan_query",
            "vef_problem_info", "vef_boundary_faces", "vef_sweep_check", "vef_sweep_timing",
            "vef_sweep_autotune", "vef_probe_machine", "vef_hrt_local_inverse", "vef_hrt_reduce", "vef_last_error",
            "vef_status_string", "vef_lambda_create", "vef_lambda_solve", "vef_lambda_destroy", "vef_lambda_error")


class vef_problem_desc(C.Structure):
    _fields_ = [("p", C.c_int), ("m", C.c_int), ("nq", C.c_int), ("n_elem", C.c_int), ("n_cp", C.c_int),
                ("cp_xy", C.c_void_p), ("elem_cp", C.c_void_p), ("n_dir", C.c_int),
                ("omega", C.c_void_p), ("weight", C.c_void_p), ("sigma_t", C.c_void_p),
                ("sigma_s", C.c_void_p)]


class vef_options(C.Structure):
    _fields_ = [("precision", C.c_int), ("schedule", C.c_int), ("block", C.c_int), ("timing", C.c_int),
                ("pipeline_waves", C.c_int), ("pipeline_ring", C.c_int), ("fixup", C.c_int),
                ("cycles", C.c_int), ("upwind", C.c_int), ("wait_polls", C.c_longlong),
                ("elem_matrices", C.c_int), ("shared_matrices", C.c_int)]


class vef_problem_io(C.Structure):
    _fields_ = [("phi_in", C.c_void_p), ("q_iso", C.c_void_p), ("q_dir", C.c_void_p),
                ("psi_bc", C.c_void_p), ("mom", C.c_void_p), ("psi_out", C.c_void_p),
                ("resid", C.c_void_p)]


class vef_run_args(C.Structure):
    _fields_ = [("io", C.POINTER(vef_problem_io)), ("n_iter", C.c_int), ("tol", C.c_double),
                ("iters_done", C.c_void_p)]


class vef_moment_io(C.Structure):
    _fields_ = [("mom", C.c_void_p), ("q_iso", C.c_void_p), ("q_dir", C.c_void_p), ("psi_bc", C.c_void_p),
                ("E", C.c_void_p), ("Eb", C.c_void_p), ("Jin", C.c_void_p), ("Q0", C.c_void_p),
                ("Q1", C.c_void_p), ("n_nonpos", C.c_void_p)]


class vef_info(C.Structure):
    _fields_ = [("n", C.c_int), ("nq", C.c_int), ("Q", C.c_int), ("n_bf", C.c_int), ("n_levels", C.c_int),
                ("n_groups", C.c_int), ("pivoting", C.c_int), ("affine", C.c_int), ("n_solves", C.c_longlong),
                ("schedule", C.c_int), ("kernel", C.c_int), ("n_lagged", C.c_longlong),
                ("n_pivoting", C.c_longlong), ("n_classes", C.c_int)]


def _load():
    # The library and torch must share one HIP runtime: torch ships its own,
    # so it is loaded first and the library's HIP dependency resolves to it
    # (with the library loaded first, the process holds two runtimes and the
    # library's finds no device).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError("libvefsweep.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2301_04758_amd.build)")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.vef_sweep_create.argtypes = [C.POINTER(vef_problem_desc), C.c_int, C.POINTER(vef_options), C.POINTER(H)]
    L.vef_sweep_run.argtypes = [H, C.POINTER(vef_run_args), C.c_void_p]
    L.vef_sweep_run_static.argtypes = [H, C.POINTER(vef_run_args), C.c_void_p]
    L.vef_moments.argtypes = [H, C.POINTER(vef_moment_io), C.c_void_p]
    L.vef_sweep_destroy.argtypes = [H]
    L.vef_plan_query.argtypes = [C.POINTER(vef_problem_desc), C.POINTER(vef_options), C.POINTER(vef_info)]
    L.vef_problem_info.argtypes = [H, C.c_int, C.POINTER(vef_info)]
    L.vef_boundary_faces.argtypes = [H, C.c_int, C.c_void_p]
    L.vef_sweep_check.argtypes = [H]
    L.vef_sweep_timing.argtypes = [H, C.POINTER(C.c_double), C.POINTER(C.c_int)]
    L.vef_sweep_autotune.argtypes = [H, C.POINTER(vef_run_args), C.c_void_p, C.c_int, C.c_void_p]
    L.vef_probe_machine.argtypes = [C.c_void_p, C.c_void_p]
    L.vef_hrt_local_inverse.argtypes = [H, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    L.vef_hrt_reduce.argtypes = [H, C.c_int] + [C.c_void_p] * 11
    L.vef_lambda_create.argtypes = [C.c_int] * 4 + [C.c_void_p, C.c_int] + [C.c_void_p] * 8 + [C.POINTER(H)]
    L.vef_lambda_solve.argtypes = [H] + [C.c_void_p] * 6 + [C.POINTER(C.c_double), C.c_void_p]
    L.vef_lambda_destroy.argtypes = [H]
    L.vef_lambda_error.argtypes = [H]
    L.vef_lambda_error.restype = C.c_char_p
    L.vef_last_error.argtypes = [H]
    L.vef_last_error.restype = C.c_char_p
    L.vef_status_string.argtypes = [C.c_int]
    L.vef_status_string.restype = C.c_char_p
    for f in ("vef_sweep_create", "vef_sweep_run", "vef_sweep_run_static", "vef_moments", "vef_sweep_destroy", "vef_plan_query",
              "vef_problem_info", "vef_boundary_faces", "vef_sweep_check", "vef_sweep_timing",
              "vef_sweep_autotune", "vef_probe_machine", "vef_hrt_local_inverse", "vef_hrt_reduce",
              "vef_lambda_create", "vef_lambda_solve", "vef_lambda_destroy"):
        getattr(L, f).restype = C.c_int
    return L


lib = _load()


class VefError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (status %d: %s)" % (msg, code, lib.vef_status_string(code).decode()))
        self.code = code


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


class _Desc:
    """A vef_problem_desc plus the numpy arrays its pointers refer to."""

    def __init__(self, pr):
        self.cp = np.ascontiguousarray(pr.cp_xy, dtype=np.float64)
        self.ec = np.ascontiguousarray(pr.elem_cp, dtype=np.int32)
        self.om = np.ascontiguousarray(pr.omega, dtype=np.float64)
        self.wt = np.ascontiguousarray(pr.weight, dtype=np.float64)
        self.st = np.ascontiguousarray(pr.sigma_t, dtype=np.float64)
        self.ss = np.ascontiguousarray(pr.sigma_s, dtype=np.float64)
        self.s = vef_problem_desc(pr.p, pr.m, int(pr.nq), self.ec.shape[0], self.cp.shape[0], self.cp.ctypes.data,
                                  self.ec.ctypes.data, self.om.shape[0], self.om.ctypes.data, self.wt.ctypes.data,
                                  self.st.ctypes.data, self.ss.ctypes.data)


# ------------------------------------------------------------------ C names


def vef_plan_query(problem, lag_cycles: bool = False, pointwise: bool = False, precision: int = VEF_FP64,
                   shared_matrices: bool = True) -> dict:
    d = _Desc(problem)
    info = vef_info()
    opt = vef_options()
    opt.precision = precision
    opt.cycles = VEF_CYCLES_LAG if lag_cycles else VEF_CYCLES_REJECT
    opt.upwind = VEF_UPWIND_POINT if pointwise else VEF_UPWIND_FACE
    opt.shared_matrices = 0 if shared_matrices else -1
    rc = lib.vef_plan_query(C.byref(d.s), C.byref(opt), C.byref(info))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(None).decode())
    return {f: getattr(info, f) for f, _ in vef_info._fields_}


def vef_sweep_create(problems: Sequence, precision: int = VEF_FP64, schedule: int = VEF_SCHEDULE_AUTO,
                     block: int = 0, timing: int = 0, pipeline_waves: int = 0,
                     pipeline_ring: int = 0, fixup: bool = False, lag_cycles: bool = False,
                     pointwise: bool = False, wait_polls: int = 0, elem_matrices: bool = True,
                     shared_matrices: bool = True) -> int:
    descs = [_Desc(p) for p in problems]
    arr = (vef_problem_desc * len(descs))(*[d.s for d in descs])
    opt = vef_options(precision, schedule, block, int(timing), pipeline_waves, pipeline_ring,
                      1 if fixup else 0, VEF_CYCLES_LAG if lag_cycles else VEF_CYCLES_REJECT,
                      VEF_UPWIND_POINT if pointwise else VEF_UPWIND_FACE, int(wait_polls),
                      0 if elem_matrices else -1, 0 if shared_matrices else -1)
    h = C.c_void_p()
    rc = lib.vef_sweep_create(arr, len(descs), C.byref(opt), C.byref(h))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(None).decode())
    return h.value


def _run_args(io, n_iter, tol, iters_done):
    arr = (vef_problem_io * len(io))()
    for k, b in enumerate(io):
        arr[k] = vef_problem_io(_ptr(b.get("phi_in")), _ptr(b.get("q_iso")), _ptr(b.get("q_dir")),
                                _ptr(b.get("psi_bc")), _ptr(b["mom"]), _ptr(b.get("psi_out")), _ptr(b.get("resid")))
    return vef_run_args(arr, int(n_iter), float(tol), _ptr(iters_done)), arr


def vef_sweep_run(h: int, io: Sequence[dict], n_iter: int = 1, tol: float = 0.0, iters_done=None, stream=None):
    args, _keep = _run_args(io, n_iter, tol, iters_done)
    rc = lib.vef_sweep_run(C.c_void_p(h), C.byref(args), C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


def vef_sweep_run_static(h: int, io: Sequence[dict], n_iter: int = 1, tol: float = 0.0, iters_done=None,
                         stream=None):
    """The run of vef_sweep_run without any device allocation (residuals of
    problems without a "resid" buffer in the library's static array)."""
    args, _keep = _run_args(io, n_iter, tol, iters_done)
    rc = lib.vef_sweep_run_static(C.c_void_p(h), C.byref(args), C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


def vef_moments(h: int, io: Sequence[dict], stream=None):
    arr = (vef_moment_io * len(io))()
    for k, b in enumerate(io):
        arr[k] = vef_moment_io(*[_ptr(b.get(f)) for f, _ in vef_moment_io._fields_])
    rc = lib.vef_moments(C.c_void_p(h), arr, C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


def vef_sweep_destroy(h: Optional[int]):
    lib.vef_sweep_destroy(C.c_void_p(h) if h else None)


def vef_problem_info(h: int, k: int) -> dict:
    info = vef_info()
    rc = lib.vef_problem_info(C.c_void_p(h), int(k), C.byref(info))
    if rc != VEF_OK:
        raise VefError(rc, "vef_problem_info")
    return {f: getattr(info, f) for f, _ in vef_info._fields_}


def vef_boundary_faces(h: int, k: int) -> np.ndarray:
    nbf = vef_problem_info(h, k)["n_bf"]
    out = np.zeros((nbf, 2), dtype=np.int32)
    rc = lib.vef_boundary_faces(C.c_void_p(h), int(k), out.ctypes.data)
    if rc != VEF_OK:
        raise VefError(rc, "vef_boundary_faces")
    return out


def vef_sweep_timing(h: int):
    """(summed sweep-kernel device time in ms of the last run, number of sweep launches)."""
    ms = C.c_double()
    n = C.c_int()
    rc = lib.vef_sweep_timing(C.c_void_p(h), C.byref(ms), C.byref(n))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())
    return ms.value, n.value


class vef_tune_result(C.Structure):
    _fields_ = [("schedule", C.c_int), ("pipeline_waves", C.c_int), ("block", C.c_int),
                ("elem_matrices", C.c_int), ("shared_matrices", C.c_int), ("n_candidates", C.c_int),
                ("best_ms", C.c_double),
                ("before_ms", C.c_double)]


def vef_sweep_autotune(h: int, io: Sequence[dict], n_iter: int = 1, reps: int = 3, stream=None) -> dict:
    arr = (vef_problem_io * len(io))()
    for k, b in enumerate(io):
        arr[k] = vef_problem_io(_ptr(b.get("phi_in")), _ptr(b.get("q_iso")), _ptr(b.get("q_dir")),
                                _ptr(b.get("psi_bc")), _ptr(b.get("mom")), _ptr(b.get("psi_out")), _ptr(b.get("resid")))
    args = vef_run_args(arr, n_iter, 0.0, None)
    res = vef_tune_result()
    rc = lib.vef_sweep_autotune(C.c_void_p(h), C.byref(args), C.c_void_p(_stream_handle(stream)), int(reps),
                                C.cast(C.byref(res), C.c_void_p))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())
    return {f: getattr(res, f) for f, _ in vef_tune_result._fields_}


class vef_machine(C.Structure):
    _fields_ = [("compute_units", C.c_int), ("hbm_copy_gbs", C.c_double), ("fp64_fma_tflops", C.c_double),
                ("fp32_fma_tflops", C.c_double), ("lds_handoff_ns", C.c_double)]


def vef_probe_machine(stream=None) -> dict:
    m = vef_machine()
    rc = lib.vef_probe_machine(C.cast(C.byref(m), C.c_void_p), C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(None).decode())
    return {f: getattr(m, f) for f, _ in vef_machine._fields_}


def vef_hrt_local_inverse(h: int, k: int, mom, Eb, inv, stream=None):
    """Device pointers (int) or torch tensors; see include/vef_sweep.h."""
    rc = lib.vef_hrt_local_inverse(C.c_void_p(h), int(k), C.c_void_p(_ptr(mom)), C.c_void_p(_ptr(Eb)),
                                   C.c_void_p(_ptr(inv)), C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


def vef_hrt_reduce(h: int, k: int, mom, Eb, Jin, Q0, Q1, inv, hloc, rloc, sol0, resp, stream=None):
    """Device pointers (int) or torch tensors; see include/vef_sweep.h."""
    rc = lib.vef_hrt_reduce(C.c_void_p(h), int(k), *[C.c_void_p(_ptr(x)) for x in
                                                     (mom, Eb, Jin, Q0, Q1, inv, hloc, rloc, sol0, resp)],
                            C.c_void_p(_stream_handle(stream)))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


class LambdaSolver:
    """The reduced hybridized system H lambda = r on the device
    (vef_lambda_create / vef_lambda_solve, include/vef_sweep.h).  gidx [ne,
    k] the unknown of each element slot (-1: boundary); the factors of one
    matrix H0 of the pattern as a scipy LU (splu) of H0 assembled from the
    same gidx; hloc0, rloc0 its element contributions (device tensors)."""

    def __init__(self, gidx, nloc, lu, hloc0, rloc0, stream=None):
        import numpy as np
        import scipy.sparse as sp
        gidx = np.ascontiguousarray(gidx, dtype=np.int32)
        ne, k = gidx.shape
        n = lu.shape[0]
        Lc, Uc = lu.L.tocoo(), lu.U.tocoo()
        low = Lc.col < Lc.row
        T = sp.csr_matrix((np.concatenate([Lc.data[low], Uc.data]), (np.concatenate([Lc.row[low], Uc.row]),
                          np.concatenate([Lc.col[low], Uc.col]))), shape=(n, n))
        T.sort_indices()
        ptr = np.ascontiguousarray(T.indptr, dtype=np.int32)
        ind = np.ascontiguousarray(T.indices, dtype=np.int32)
        val = np.ascontiguousarray(T.data, dtype=np.float64)
        piv_p = np.ascontiguousarray(np.argsort(lu.perm_r), dtype=np.int32)
        piv_q = np.ascontiguousarray(np.argsort(lu.perm_c), dtype=np.int32)
        self.n, self.ne, self.k, self.nloc = n, ne, k, nloc
        h = C.c_void_p()
        rc = lib.vef_lambda_create(n, ne, k, nloc, gidx.ctypes.data, int(T.nnz), ptr.ctypes.data, ind.ctypes.data,
                                   val.ctypes.data, piv_p.ctypes.data, piv_q.ctypes.data, _ptr(hloc0.contiguous()),
                                   _ptr(rloc0.contiguous()), _stream_handle(stream), C.byref(h))
        if rc != VEF_OK:
            raise VefError(rc, lib.vef_lambda_error(None).decode())
        self.h = h

    def solve(self, hloc, rloc, sol0=None, resp=None, want_resid=True, stream=None):
        """Returns (lam [n], sol [ne, nloc] or None, relative residual or
        None) as device tensors."""
        import torch
        dev = hloc.device
        lam = torch.empty(self.n, dtype=torch.float64, device=dev)
        sol = torch.empty((self.ne, self.nloc), dtype=torch.float64, device=dev) if sol0 is not None else None
        r = C.c_double(0.0)
        rc = lib.vef_lambda_solve(self.h, _ptr(hloc.contiguous()), _ptr(rloc.contiguous()),
                                  _ptr(sol0.contiguous()) if sol0 is not None else None,
                                  _ptr(resp.contiguous()) if resp is not None else None, _ptr(lam), _ptr(sol),
                                  C.byref(r) if want_resid else None, _stream_handle(stream))
        if rc != VEF_OK:
            raise VefError(rc, lib.vef_lambda_error(self.h).decode())
        return lam, sol, (r.value if want_resid else None)

    def close(self):
        if getattr(self, "h", None):
            lib.vef_lambda_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vef_sweep_check(h: int):
    rc = lib.vef_sweep_check(C.c_void_p(h))
    if rc != VEF_OK:
        raise VefError(rc, lib.vef_last_error(C.c_void_p(h)).decode())


# ------------------------------------------------------------------ convenience


class Sweep:
    """Owns one handle; allocates device buffers with torch for convenience."""

    def __init__(self, problems, precision="fp64", block=0, device=None, timing=False, schedule="auto",
                 pipeline_waves=0, pipeline_ring=0, fixup=False, lag_cycles=False, pointwise=False, wait_polls=0,
                 elem_matrices=True, shared_matrices=True):
        import torch
        self.torch = torch
        self.problems = list(problems)
        self.fp32 = precision == "fp32"
        self.device = torch.device("cuda" if device is None else device)
        with torch.cuda.device(self.device):
            self.h = vef_sweep_create(self.problems, VEF_FP32_LOCAL if self.fp32 else VEF_FP64,
                                      SCHEDULES[schedule], block, timing, pipeline_waves, pipeline_ring,
                                      fixup, lag_cycles, pointwise, wait_polls, elem_matrices,
                                      shared_matrices)
        self.info = [vef_problem_info(self.h, k) for k in range(len(self.problems))]

    def close(self):
        if self.h:
            vef_sweep_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _t(self, a, dtype=None):
        if a is None:
            return None
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(self.device).contiguous()
        return t.as_tensor(np.ascontiguousarray(a), dtype=dtype or t.float64, device=self.device)

    def buffers(self, n_iter=1, store_psi=True, phi_in=None):
        """Device buffers for every problem: inputs from the Problem arrays, zeroed outputs."""
        t = self.torch
        out = []
        for pr, inf in zip(self.problems, self.info):
            n = inf["n"]
            b = dict(q_iso=self._t(pr.q_iso), q_dir=self._t(pr.q_dir), psi_bc=self._t(pr.psi_bc),
                     phi_in=self._t(phi_in) if phi_in is not None else None,
                     mom=t.zeros((6, pr.n_elem, n), dtype=t.float64, device=self.device),
                     resid=t.zeros(n_iter, dtype=t.float64, device=self.device))
            if store_psi:
                b["psi_out"] = t.zeros((pr.n_dir, pr.n_elem, n), dtype=t.float32 if self.fp32 else t.float64,
                                       device=self.device)
            out.append(b)
        return out

    def run(self, io, n_iter=1, tol=0.0, iters_done=None, stream=None):
        vef_sweep_run(self.h, io, n_iter, tol, iters_done, stream)

    def moment_buffers(self, io):
        t = self.torch
        out = []
        for b, pr, inf in zip(io, self.problems, self.info):
            Q, nbf, nq = inf["Q"], inf["n_bf"], inf["nq"]
            out.append(dict(mom=b["mom"], q_iso=b.get("q_iso"), q_dir=b.get("q_dir"), psi_bc=b.get("psi_bc"),
                            E=t.zeros((3, pr.n_elem, Q), dtype=t.float64, device=self.device),
                            Eb=t.zeros((nbf, nq), dtype=t.float64, device=self.device),
                            Jin=t.zeros((nbf, nq), dtype=t.float64, device=self.device),
                            Q0=t.zeros((pr.n_elem, Q), dtype=t.float64, device=self.device),
                            Q1=t.zeros((2, pr.n_elem, Q), dtype=t.float64, device=self.device),
                            n_nonpos=t.zeros(1, dtype=t.int32, device=self.device)))
        return out

    def moments(self, mio, stream=None):
        vef_moments(self.h, mio, stream)

    def hrt_local_inverse(self, k, mom, Eb=None, stream=None):
        """[[W, X], [Y, Z]] of every element of problem k: a [n_elem, n, n]
        float64 tensor, n = 2(p+1)(p+2) + (p+1)^2 (vef_hrt_local_inverse)."""
        t = self.torch
        pr = self.problems[k]
        p = pr.p
        n = 2 * (p + 1) * (p + 2) + (p + 1) ** 2
        out = t.empty((pr.n_elem, n, n), dtype=t.float64, device=self.device)
        mom = mom.contiguous()
        Eb = None if Eb is None else Eb.contiguous()
        vef_hrt_local_inverse(self.h, k, mom, Eb, out, stream)
        return out

    def hrt_reduce(self, k, mom, mio, inv, stream=None):
        """Element-local part of the hybridized solve (vef_hrt_reduce) from the
        run's moments, the closures of moment_buffers()[k] and the block
        inverses: dict of tensors hloc [n_elem, 4(p+1), 4(p+1)], rloc
        [n_elem, 4(p+1)], sol0 [n_elem, n], resp [n_elem, n, 4(p+1)]."""
        t = self.torch
        pr = self.problems[k]
        p = pr.p
        n = 2 * (p + 1) * (p + 2) + (p + 1) ** 2
        nl = 4 * (p + 1)
        kw = dict(dtype=t.float64, device=self.device)
        out = dict(hloc=t.empty((pr.n_elem, nl, nl), **kw), rloc=t.empty((pr.n_elem, nl), **kw),
                   sol0=t.empty((pr.n_elem, n), **kw), resp=t.empty((pr.n_elem, n, nl), **kw))
        vef_hrt_reduce(self.h, k, mom.contiguous(), mio["Eb"], mio["Jin"], mio["Q0"], mio["Q1"], inv.contiguous(),
                       out["hloc"], out["rloc"], out["sol0"], out["resp"], stream)
        return out

    def check(self):
        vef_sweep_check(self.h)

    def autotune(self, io, n_iter=1, reps=3, stream=None):
        """Time every schedule/kernel candidate on these buffers and keep the
        fastest (vef_sweep_autotune); refreshes self.info."""
        res = vef_sweep_autotune(self.h, io, n_iter, reps, stream)
        self.info = [vef_problem_info(self.h, k) for k in range(len(self.problems))]
        return res

    def timing(self):
        return vef_sweep_timing(self.h)
