"""A valid curved mesh whose upwind graph is cyclic for some directions.

3x3 quadratic (m = 2) mesh of the unit square whose four interior corner
control points are moved (mid-edge control points stay put, so the faces
bend).  The Jacobian is positive at every Gauss point, but the chord
quadrilaterals are not convex, and for directions near 49.5 and 229.5
degrees the chord-based upwind relation of three elements closes a cycle
(a re-entrant configuration in the sense of the triple-point discussion of
Sec. 8, thick-diffusion-limit study).  Found by a seeded random search over
perturbations; stored here as plain coordinates.
"""
import numpy as np

from paper_2301_04758_amd import problems as P

MOVED = {  # control point id -> new (x, y)
    16: (0.4796345942313551, 0.30796490832127377),
    18: (0.5714672620839093, 0.4179576514645563),
    30: (0.26484903403928095, 0.6863930859171834),
    32: (0.7104711906340646, 0.5765698441125696),
}
CYCLIC_ANGLE_DEG = 49.5


def reentrant_problem(p=1):
    cp, ec = P.quad_mesh(3, 3, 2)
    cp = cp.copy()
    for k, xy in MOVED.items():
        cp[k] = xy
    t = np.radians(CYCLIC_ANGLE_DEG)
    om = np.array([[0.99 * np.cos(t), 0.99 * np.sin(t)], [0.99, 0.0]])
    wt = np.array([2 * np.pi, 2 * np.pi])
    return P.Problem("cyclic", p, 2, cp, ec, om, wt, np.ones(9), np.zeros(9))
