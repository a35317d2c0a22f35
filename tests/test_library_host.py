"""CPU-side checks of the HIP library: it loads, exports every declared entry
point, and its host planner (validation, face matching, upwind levels) agrees
with the oracle.  No kernel is launched here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2301_04758_amd import problems as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vef_sweep.h")


def _vef():
    from paper_2301_04758_amd import vef
    return vef


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(vef_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    vef = _vef()
    names = declared_functions()
    assert {"vef_sweep_create", "vef_sweep_run", "vef_moments", "vef_sweep_destroy"} <= set(names)
    lib = C.CDLL(vef.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(vef.EXPORTED)


def test_status_strings():
    vef = _vef()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert vef.lib.vef_status_string(code)
    vef.vef_sweep_destroy(None)  # NULL is a no-op


@pytest.mark.parametrize("cfg,scale", [("c1", None), ("c2", 16), ("c3", 12), ("c5", 8)])
def test_plan_matches_oracle_levels_and_faces(cfg, scale):
    vef = _vef()
    (pr,), _ = P.make_config(cfg, scale=scale)
    info = vef.vef_plan_query(pr)
    assert info["n"] == (pr.p + 1) ** 2
    assert info["nq"] == pr.p + pr.m
    assert info["n_bf"] == O.n_boundary_faces(pr)
    assert info["n_levels"] == int(O.levels(pr).max())
    assert info["n_solves"] == pr.n_elem * pr.n_dir
    if pr.m == 1:
        assert info["n_groups"] == 4  # straight Cartesian mesh: one upwind graph per quadrant
        assert info["pivoting"] == 0  # straight faces, sigma_t > 0: natural-order elimination
    else:
        assert info["pivoting"] == 1  # curved faces keep partial pivoting


def test_pivoting_choice():
    vef = _vef()
    import copy
    (pr,), _ = P.make_config("c1")
    assert vef.vef_plan_query(pr)["pivoting"] == 0
    q = copy.deepcopy(pr)
    q.sigma_t = q.sigma_t.copy()
    q.sigma_t[5] = 0.0  # a purely streaming element: symmetric part only semidefinite
    assert vef.vef_plan_query(q)["pivoting"] == 1
    # straight but m = 2 (midpoint control points on the chords): still natural order
    cp, ec = P.quad_mesh(4, 4, 2)
    q = P.Problem("m2", 2, 2, cp, ec, pr.omega, pr.weight, np.ones(16), np.zeros(16))
    assert vef.vef_plan_query(q)["pivoting"] == 0


def _certification_count(pr):
    """Pairs (direction, element) whose local system the plan may not eliminate
    in natural order, counted from the independent numpy geometry: sigma_t = 0,
    or a face quadrature point where Omega . n ds has the sign of the other
    role (inflow faces need <= 0, outflow faces >= 0)."""
    import dg_numpy as D
    mesh = D.Mesh(pr)
    faces = {(e, f): mesh.face_data(e, f)[3] for e in range(pr.n_elem) for f in range(4)}
    n = 0
    for om in np.asarray(pr.omega):
        for e in range(pr.n_elem):
            ok = pr.sigma_t[e] > 0.0
            for f in range(4):
                on = faces[(e, f)] @ om
                inflow = not mesh.upwind_is_self(e, f, om)
                ok = ok and bool(np.all(on <= 0.0) if inflow else np.all(on >= 0.0))
            n += 0 if ok else 1
    return n


def test_pivoting_certification_counts():
    """vef_info.n_pivoting against a count from the definition, on straight,
    curved and sigma_t = 0 inputs."""
    import copy
    vef = _vef()
    (pr,), _ = P.make_config("c1")
    assert vef.vef_plan_query(pr)["n_pivoting"] == 0
    q = copy.deepcopy(pr)
    q.sigma_t = q.sigma_t.copy()
    q.sigma_t[5] = 0.0
    assert vef.vef_plan_query(q)["n_pivoting"] == q.n_dir == _certification_count(q)
    for warp, N in ((0.12, 8), (0.2, 12)):
        cp, ec = P.quad_mesh(10, 9, 2)
        cp = P.sine_warp(cp, warp)
        om, wt = P.level_symmetric_2d(N)
        c = P.Problem("warp", 3, 2, cp, ec, om, wt, np.ones(90), np.zeros(90), nx=10, ny=9)
        got = vef.vef_plan_query(c)["n_pivoting"]
        want = _certification_count(c)
        assert got == want, (warp, N, got, want)
        assert 0 < got < c.n_elem * c.n_dir


def _shared_class_count(pr, s=8):
    """Classes of (direction, element) pairs with equal local matrices, from
    the definition on numpy geometry: equal sigma_t, an equal element shape
    (the corners' offsets from the first corner, compared exactly) and the
    same direction, which then fixes the inflow faces.  0 where the
    library's rule declines them (more than 4096 element classes, fewer than
    8 solves per class, or more than 16 MiB of class matrices)."""
    xy = pr.cp_xy[pr.elem_cp]  # [ne][(m+1)^2][2]
    shape = xy - xy[:, :1, :]
    keys = {}
    for e in range(pr.n_elem):
        keys.setdefault((pr.sigma_t[e],) + tuple(shape[e].ravel()), len(keys))
    n_cls = len(keys) * pr.n_dir
    n, nq = (pr.p + 1) ** 2, pr.nq or pr.p + pr.m
    tw = max(pr.p + 1, nq)
    inv_bytes = (n + 8 * tw + nq * nq) * 16 * ((n + 15) // 16) * s
    if len(keys) > 4096 or n_cls * 8 > pr.n_elem * pr.n_dir or n_cls * inv_bytes > (16 << 20):
        return 0
    return n_cls


def test_shared_matrix_class_counts():
    """vef_info.n_classes of vef_plan_query against a count from the
    definition: uniform grids with one or a few materials (one class per
    material and direction), sigma_t on every element different (declined),
    spacings that are not exact in binary (element shapes differ in the last
    bit: many classes, declined), degrees without the row-set LU and the
    option off."""
    vef = _vef()

    def grid(n, p, N, st):
        cp, ec = P.quad_mesh(n, n, 1)
        om, wt = P.level_symmetric_2d(N)
        st = np.broadcast_to(np.asarray(st, float), (n * n,)).copy()
        return P.Problem("grid", p, 1, cp, ec, om, wt, st, 0.5 * st, nx=n, ny=n)

    rng = np.random.default_rng(5)
    cases = [grid(8, 4, 8, 1.0), grid(16, 3, 6, rng.choice([0.5, 3.0, 40.0], 256)), grid(8, 4, 4, rng.uniform(1, 2, 64)),
             grid(12, 4, 4, 2.0), grid(32, 3, 12, 1000.0)]
    for c in cases:
        want = _shared_class_count(c)
        assert vef.vef_plan_query(c)["n_classes"] == want, c.sigma_t[:3]
        assert vef.vef_plan_query(c, shared_matrices=False)["n_classes"] == 0
        assert vef.vef_plan_query(c, precision=vef.VEF_FP32_LOCAL)["n_classes"] == _shared_class_count(c, 4)
    assert _shared_class_count(cases[0]) == cases[0].n_dir
    assert _shared_class_count(cases[1]) == 3 * cases[1].n_dir
    assert _shared_class_count(cases[2]) == 0
    assert _shared_class_count(cases[4]) == cases[4].n_dir
    assert vef.vef_plan_query(grid(8, 2, 8, 1.0))["n_classes"] == 0  # p = 2: no row-set LU
    (c3,), _ = P.make_config("c3")
    assert vef.vef_plan_query(c3)["n_classes"] == 0  # curved


def _bad(pr, code):
    vef = _vef()
    with pytest.raises(vef.VefError) as ei:
        vef.vef_plan_query(pr)
    assert ei.value.code == code
    return str(ei.value)


def test_plan_rejects_bad_inputs():
    vef = _vef()
    base, _ = P.make_config("c1")
    pr = base[0]
    import copy
    q = copy.deepcopy(pr)
    q.p = 5
    _bad(q, vef.VEF_ERR_INVALID)
    q = copy.deepcopy(pr)
    q.weight = q.weight * 1.001
    assert "4 pi" in _bad(q, vef.VEF_ERR_INVALID)
    q = copy.deepcopy(pr)
    q.sigma_t = q.sigma_t.copy()
    q.sigma_t[3] = np.nan
    _bad(q, vef.VEF_ERR_INVALID)
    q = copy.deepcopy(pr)
    q.elem_cp = q.elem_cp.copy()
    q.elem_cp[0, 0] = 10 ** 6
    _bad(q, vef.VEF_ERR_INVALID)
    q = copy.deepcopy(pr)
    q.nq = pr.p + 5
    _bad(q, vef.VEF_ERR_INVALID)
    # mirrored element: negative Jacobian
    q = copy.deepcopy(pr)
    ec = q.elem_cp.copy()
    ec[0] = ec[0][[1, 0, 3, 2]]
    q.elem_cp = ec
    _bad(q, vef.VEF_ERR_JACOBIAN)


def test_plan_detects_cycle():
    """A mesh whose upwind graph has a cycle for some direction is rejected
    before any launch (the fixture is a 3x3 curved mesh with non-convex chord quadrilaterals)."""
    vef = _vef()
    from cyclic_mesh import reentrant_problem
    pr = reentrant_problem()
    with pytest.raises(O.OracleError) as oe:
        O.levels(pr)
    assert oe.value.code == O.ERR_CYCLE
    msg = _bad(pr, vef.VEF_ERR_CYCLE)
    assert "cycle" in msg


def _trapezoids(n=6, amp=0.15, seed=3):
    """Straight-sided, non-affine mesh: interior vertices of an m = 1 grid moved at random."""
    cp, ec = P.quad_mesh(n, n, 1)
    cp = cp.copy()
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    inner = (cp[:, 0] > 1e-12) & (cp[:, 0] < 1 - 1e-12) & (cp[:, 1] > 1e-12) & (cp[:, 1] < 1 - 1e-12)
    cp[inner] += rng.uniform(-amp * h, amp * h, (inner.sum(), 2))
    return cp, ec


def test_affine_classification():
    vef = _vef()
    (c1,), _ = P.make_config("c1")
    assert vef.vef_plan_query(c1)["affine"] == 1
    (c3,), _ = P.make_config("c3", scale=6)
    i3 = vef.vef_plan_query(c3)
    assert i3["affine"] == 0 and i3["pivoting"] == 1
    cp, ec = P.quad_mesh(4, 4, 2)  # straight, uniformly placed midpoints: affine
    q = P.Problem("m2", 2, 2, cp, ec, c1.omega, c1.weight, np.ones(16), np.zeros(16))
    assert vef.vef_plan_query(q)["affine"] == 1
    cp, ec = _trapezoids()
    q = P.Problem("trap", 2, 1, cp, ec, c1.omega, c1.weight, np.ones(36), np.zeros(36))
    i = vef.vef_plan_query(q)
    assert i["affine"] == 0 and i["pivoting"] == 0


@pytest.mark.parametrize("n,m,shift", [(1024, 1, 0.0), (512, 2, 0.0), (300, 1, 1000.0)])
def test_affine_classification_fine_meshes(n, m, shift):
    """Rounding of the geometry grows with coordinate size / element size:
    fine uniform meshes, also far from the origin, stay affine; a corner
    moved by 1e-9 of the element size (1e-7 far from the origin, where
    1e-9 is within a few ulps of the coordinates) makes it non-affine."""
    vef = _vef()
    cp, ec = P.quad_mesh(n, n, m)
    cp = cp + shift
    om, wt = P.level_symmetric_2d(4)
    ne = n * n
    q = P.Problem("fine", 1, m, cp, ec, om, wt, np.ones(ne), np.zeros(ne))
    i = vef.vef_plan_query(q)
    assert i["affine"] == 1 and i["pivoting"] == 0
    if m == 1:
        cp2 = cp.copy()
        k = (n + 1) * (n // 2) + n // 2  # an interior vertex
        cp2[k, 0] += (1e-9 if shift == 0 else 1e-7) / n
        i2 = vef.vef_plan_query(P.Problem("fine", 1, m, cp2, ec, om, wt, np.ones(ne), np.zeros(ne)))
        assert i2["affine"] == 0


def test_lambda_create_rejects_bad_arguments():
    """vef_lambda_create checks its host arrays before any device call:
    slot indices out of range, pivots that are not permutations and an
    unsorted factor pattern are rejected with VEF_ERR_INVALID."""
    vef = _vef()
    n, ne, k = 4, 2, 4
    gidx = np.array([[0, 1, -1, -1], [2, 3, 0, -1]], dtype=np.int32)
    ptr = np.array([0, 1, 2, 3, 4], dtype=np.int32)
    ind = np.array([0, 1, 2, 3], dtype=np.int32)
    val = np.ones(4)
    piv = np.arange(4, dtype=np.int32)

    def create(g=gidx, pt=ptr, it=ind, pp=piv, pq=piv):
        h = C.c_void_p()
        rc = vef.lib.vef_lambda_create(n, ne, k, 3, g.ctypes.data, int(it.size), pt.ctypes.data, it.ctypes.data,
                                       val.ctypes.data, pp.ctypes.data, pq.ctypes.data, 16, 16, None, C.byref(h))
        return rc, vef.lib.vef_lambda_error(None).decode()

    bad = gidx.copy()
    bad[0, 0] = 4
    assert create(g=bad)[0] == vef.VEF_ERR_INVALID
    assert create(pp=np.array([0, 1, 1, 3], dtype=np.int32))[0] == vef.VEF_ERR_INVALID
    assert create(pq=np.array([0, 1, 2, 4], dtype=np.int32))[0] == vef.VEF_ERR_INVALID
    rc, msg = create(pt=np.array([0, 2, 2, 3, 4], dtype=np.int32), it=np.array([1, 0, 2, 3], dtype=np.int32))
    assert rc == vef.VEF_ERR_INVALID and "CSR" in msg
    assert vef.lib.vef_lambda_destroy(None) == vef.VEF_OK


def test_static_resid_limit_matches_header():
    """The binding's copy of VEF_STATIC_RESID_MAX (vef_sweep_run_static) is
    the header's."""
    vef = _vef()
    m = re.search(r"#define\s+VEF_STATIC_RESID_MAX\s+(\d+)", open(HEADER).read())
    assert m and int(m.group(1)) == vef.VEF_STATIC_RESID_MAX
