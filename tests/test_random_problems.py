"""Randomized coverage.

CPU (hypothesis): the library's host plan agrees with the oracle on random
meshes: unknowns, quadrature, boundary faces, upwind level depth, and the
classification (pivoting / affine) follows from the geometry.

GPU: a seeded family of random problems (order, geometry order, warp,
vertex jitter, cross sections, angular order, isotropic and direction-
dependent sources, inflow data, scattering input) against the oracle through
every schedule, at the double and float bars.
"""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from oracle import oracle as O
from paper_2301_04758_amd import problems as P


def random_problem(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(1, 5))
    m = int(rng.integers(1, 4))
    nx, ny = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    cp, ec = P.quad_mesh(nx, ny, m)
    kind = rng.integers(0, 3)
    if kind == 1 and m > 1:
        cp = P.sine_warp(cp, float(rng.uniform(0.01, 0.08)))
    elif kind == 2 and m == 1 and nx > 1 and ny > 1:
        h = 1.0 / max(nx, ny)
        cp = cp.copy()
        inner = (cp > 1e-12).all(1) & (cp < 1 - 1e-12).all(1)
        cp[inner] += rng.uniform(-0.15 * h, 0.15 * h, (inner.sum(), 2))
    N = int(rng.choice([2, 4, 6, 8]))
    om, wt = P.level_symmetric_2d(N)
    ne = nx * ny
    st_ = 10 ** rng.uniform(-1, 2, ne)
    ss = rng.uniform(0, 0.95, ne) * st_
    pr = P.Problem("rand%d" % seed, p, m, cp, ec, om, wt, st_, ss, nx=nx, ny=ny)
    n = (p + 1) ** 2
    pr.q_iso = rng.uniform(0, 2, (ne, n))
    if rng.uniform() < 0.5:
        nq = p + m
        pr.q_dir = rng.uniform(0, 1, (pr.n_dir, ne, nq * nq))
    if rng.uniform() < 0.5:
        nb = O.n_boundary_faces(pr)
        pr.psi_bc = rng.uniform(0, 1, (pr.n_dir, nb, p + m))
    phi = rng.uniform(0, 3, (ne, n)) if rng.uniform() < 0.5 else None
    return pr, phi


@settings(max_examples=40, deadline=None)
@given(st.integers(min_value=0, max_value=10 ** 6))
def test_plan_agrees_with_oracle_on_random_meshes(seed):
    from paper_2301_04758_amd import vef
    pr, _ = random_problem(seed)
    info = vef.vef_plan_query(pr)
    assert info["n"] == (pr.p + 1) ** 2
    assert info["nq"] == pr.p + pr.m
    assert info["Q"] == info["nq"] ** 2
    assert info["n_bf"] == O.n_boundary_faces(pr)
    assert info["n_levels"] == int(O.levels(pr).max())
    assert info["n_solves"] == pr.n_elem * pr.n_dir
    if info["affine"]:
        assert info["pivoting"] == 0  # affine maps are straight-sided (and sigma_t > 0 here)


SEEDS = [11, 23, 37, 41, 59, 67, 73, 89, 97, 101, 131, 157, 207, 244, 246]


@pytest.mark.gpu
@pytest.mark.parametrize("schedule", ["level", "dir"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("seed", SEEDS)
def test_random_problem_parity(seed, precision, schedule):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2301_04758_amd import vef
    pr, phi = random_problem(seed)
    print("random problem", seed, pr.name, "p", pr.p, "m", pr.m, pr.nx, pr.ny, "N", pr.n_dir, precision, schedule,
          flush=True)
    ref = O.sweep(pr, phi_in=phi)
    sw = vef.Sweep([pr], precision=precision, schedule=schedule)
    io = sw.buffers(n_iter=1, phi_in=phi)
    sw.run(io, n_iter=1)
    torch.cuda.synchronize()
    sw.check()
    psi = io[0]["psi_out"].double().cpu().numpy()
    mom = io[0]["mom"].cpu().numpy()
    sw.close()
    tol = 1e-12 if precision == "fp64" else 1e-5
    assert np.abs(psi - ref["psi"]).max() <= tol * np.abs(ref["psi"]).max()
    assert np.abs(mom[0] - ref["mom"][0]).max() <= tol * np.abs(ref["mom"][0]).max()
