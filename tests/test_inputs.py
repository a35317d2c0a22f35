"""Pins of the seeded input generator: level-symmetric sets and meshes."""
import os

import numpy as np
import pytest

from paper_2301_04758_amd import problems as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _mu1_table():
    out = {}
    for line in open(os.path.join(GOLD, "ls_first_cosine.txt")):
        if line.startswith("#") or not line.strip():
            continue
        n, v = line.split()
        out[int(n)] = float(v)
    return out


@pytest.mark.parametrize("N", [4, 6, 8, 10, 12, 16])
def test_level_symmetric_moments(N):
    om, w = P.level_symmetric_2d(N)
    assert len(w) == N * (N + 2) // 2
    fp = 4 * np.pi
    assert abs(w.sum() - fp) < 1e-12 * fp
    assert np.all(w > 0)
    ox, oy = om[:, 0], om[:, 1]
    tol = 1e-11
    assert abs((w * ox).sum()) < tol and abs((w * oy).sum()) < tol
    assert abs((w * ox * oy).sum()) < tol
    assert abs((w * ox ** 2).sum() - fp / 3) < tol
    assert abs((w * oy ** 2).sum() - fp / 3) < tol
    assert abs((w * ox ** 4).sum() - fp / 5) < tol
    assert abs((w * ox ** 2 * oy ** 2).sum() - fp / 15) < tol
    # in-plane components lie inside the unit disc (dropped z component > 0)
    assert np.all(ox ** 2 + oy ** 2 < 1.0)
    # symmetric under x <-> y and sign flips
    key = {(round(a, 12), round(b, 12)): ww for (a, b), ww in zip(om, w)}
    for (a, b), ww in zip(om, w):
        for t in ((b, a), (-a, b), (a, -b)):
            assert abs(key[(round(t[0], 12), round(t[1], 12))] - ww) < 1e-12


def test_level_symmetric_first_cosine_matches_tables():
    for N, mu1 in _mu1_table().items():
        mu, _, _ = P.level_symmetric_octant(N)
        assert abs(mu[0] - mu1) < 1.5e-7, (N, mu[0], mu1)


def test_ls4_closed_form():
    # S4: a = mu_1^2 solves 6 a^2 - 4 a + 2/5 = 0 (smaller root)
    a = (4 - np.sqrt(16 - 9.6)) / 12
    mu, _, w = P.level_symmetric_octant(4)
    assert abs(mu[0] ** 2 - a) < 1e-13
    assert np.allclose(w, 1.0 / 3.0)


def test_direction_order_octants():
    om, _ = P.level_symmetric_2d(8)
    q = len(om) // 4
    signs = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    for k, (sx, sy) in enumerate(signs):
        blk = om[k * q:(k + 1) * q]
        assert np.all(np.sign(blk[:, 0]) == sx) and np.all(np.sign(blk[:, 1]) == sy)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_quad_mesh_conforming(m):
    cp, ec = P.quad_mesh(3, 2, m)
    assert ec.shape == (6, (m + 1) ** 2)
    assert cp.shape[0] == (3 * m + 1) * (2 * m + 1)
    # element 0 lower-left corner at origin, last element upper-right at (1,1)
    assert np.allclose(cp[ec[0, 0]], [0, 0])
    assert np.allclose(cp[ec[-1, -1]], [1, 1])
    # neighbours share the whole face column of control points
    assert np.all(ec[0, m::m + 1] == ec[1, 0::m + 1])


def test_sine_warp_keeps_boundary():
    cp, ec = P.quad_mesh(6, 6, 2)
    w = P.sine_warp(cp, 0.1)
    on_b = (np.isclose(cp[:, 0], 0) | np.isclose(cp[:, 0], 1) | np.isclose(cp[:, 1], 0) | np.isclose(cp[:, 1], 1))
    assert np.allclose(w[on_b], cp[on_b], atol=1e-15)
    assert np.abs(w - cp).max() > 0.05


def test_configs_shapes_and_seeds():
    (c1,), r1 = P.make_config("c1")
    assert c1.n_elem == 64 and c1.n_dir == 12 and c1.p == 1 and r1["n_iter"] == 1
    (c2,), r2 = P.make_config("c2")
    assert c2.n_elem == 4096 and c2.n_dir == 40 and c2.p == 2 and r2["n_iter"] == 50
    assert np.allclose(c2.sigma_s, 0.9 * c2.sigma_t)
    assert c2.sigma_t.min() >= 0.1 and c2.sigma_t.max() <= 100
    # constant per 8x8 block
    st = c2.sigma_t.reshape(64, 64)
    assert np.all(st[:8, :8] == st[0, 0])
    (c2b,), _ = P.make_config("c2")
    assert np.array_equal(c2.sigma_t, c2b.sigma_t)
    probs, r4 = P.make_config("c4")
    assert len(probs) == 64
    assert {p.p for p in probs} <= {1, 2, 3, 4}
    assert all(16 <= p.nx <= 128 for p in probs)
