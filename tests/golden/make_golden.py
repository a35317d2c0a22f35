#!/usr/bin/env python3
"""Write the full-size reference fixtures of tests/golden/ from the CPU oracle.

Every value stored here is computed by oracle/ (serial double precision) on
the seeded inputs of paper_2301_04758_amd.problems; nothing comes from the
GPU library.  Each fixture holds sampled outputs (indices drawn from a seeded
generator and stored with the values), so that GPU runs at the benchmark
sizes can be checked element by element:

  c2_full.json  64x64, p=2, S8, 50 source iterations: residual history and
                the six moments at sampled nodes after the last sweep
  c3_full.json  256x256 curved (m=2), p=3, S12, one sweep from phi = 0:
                moments at sampled nodes and angular flux at sampled
                (direction, element, node) triples
  c5_dirs.json  512x512, p=4, S16, one sweep from phi = 0, two sampled
                directions swept in full: angular flux at sampled nodes
  c4_some.json  the 64-problem batch, one sweep from phi = 0, for a subset
                of the problems: moments at sampled nodes

Usage: python tests/golden/make_golden.py [c2 c3 c4 c5]   (all by default)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2301_04758_amd import problems as P  # noqa: E402

SAMPLE_SEED = 20230111


def _sample_nodes(rng, ne, n, k):
    idx = rng.choice(ne * n, size=min(k, ne * n), replace=False)
    return np.sort(idx)


def _write(name, obj):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(obj, f, separators=(",", ":"))
    print("wrote", path, flush=True)


def _header(cfg, what):
    return {"generated_by": "tests/golden/make_golden.py (oracle/, serial double precision)",
            "inputs": "paper_2301_04758_amd.problems.make_config(%r)" % cfg, "content": what}


def make_c2():
    (pr,), run = P.make_config("c2")
    t = time.time()
    r = O.source_iteration(pr, run["n_iter"])
    rng = np.random.default_rng(SAMPLE_SEED + 2)
    idx = _sample_nodes(rng, pr.n_elem, pr.n, 400)
    mom = r["mom"].reshape(6, -1)
    out = _header("c2", "50 source iterations from phi = 0; moments at sampled flat (element*n + node) indices")
    out.update(n_iter=run["n_iter"], resid=r["resid"].tolist(), index=idx.tolist(),
               mom=[mom[k, idx].tolist() for k in range(6)], mom_absmax=[float(np.abs(mom[k]).max()) for k in range(6)],
               oracle_seconds=time.time() - t)
    _write("c2_full.json", out)


def make_c3():
    (pr,), _ = P.make_config("c3")
    t = time.time()
    rng = np.random.default_rng(SAMPLE_SEED + 3)
    dsel = np.sort(rng.choice(pr.n_dir, size=6, replace=False))
    r = O.sweep(pr, want_psi=False)
    # angular flux of the sampled directions (a second pass over those directions only)
    rd = O.sweep(pr, dirs=dsel)
    idx = _sample_nodes(rng, pr.n_elem, pr.n, 400)
    mom = r["mom"].reshape(6, -1)
    psi = rd["psi"].reshape(len(dsel), -1)
    pidx = _sample_nodes(rng, pr.n_elem, pr.n, 150)
    out = _header("c3", "one sweep from phi = 0; moments at sampled flat indices; angular flux of "
                        "sampled directions at sampled flat indices")
    out.update(index=idx.tolist(), mom=[mom[k, idx].tolist() for k in range(6)],
               mom_absmax=[float(np.abs(mom[k]).max()) for k in range(6)],
               dirs=dsel.tolist(), psi_index=pidx.tolist(), psi=[psi[i, pidx].tolist() for i in range(len(dsel))],
               psi_absmax=[float(np.abs(psi[i]).max()) for i in range(len(dsel))],
               levels=O.levels(pr).tolist(), oracle_seconds=time.time() - t)
    _write("c3_full.json", out)


def make_c5():
    (pr,), _ = P.make_config("c5")
    t = time.time()
    dsel = np.array([5, 101])
    rd = O.sweep(pr, dirs=dsel)
    rng = np.random.default_rng(SAMPLE_SEED + 5)
    pidx = _sample_nodes(rng, pr.n_elem, pr.n, 300)
    psi = rd["psi"].reshape(len(dsel), -1)
    out = _header("c5", "one sweep from phi = 0 for two directions; angular flux at sampled flat indices")
    out.update(dirs=dsel.tolist(), psi_index=pidx.tolist(), psi=[psi[i, pidx].tolist() for i in range(len(dsel))],
               psi_absmax=[float(np.abs(psi[i]).max()) for i in range(len(dsel))], oracle_seconds=time.time() - t)
    _write("c5_dirs.json", out)


def make_c4():
    probs, _ = P.make_config("c4")
    t = time.time()
    rng = np.random.default_rng(SAMPLE_SEED + 4)
    # a spread of sizes and orders, kept cheap enough for the oracle
    cost = [p.n_solves * p.n ** 2 for p in probs]
    order = np.argsort(cost)
    high = [k for k in order if probs[k].p >= 3][:2]  # the two cheapest problems of degree 3-4
    pick = sorted(set(order[[0, 5, 12, 20, 31, 44]].tolist()) | set(int(k) for k in high))
    items = []
    for k in pick:
        pr = probs[k]
        r = O.sweep(pr, want_psi=False)
        idx = _sample_nodes(rng, pr.n_elem, pr.n, 60)
        mom = r["mom"].reshape(6, -1)
        items.append(dict(problem=int(k), p=pr.p, side=pr.nx, n_dir=pr.n_dir, index=idx.tolist(),
                          mom=[mom[j, idx].tolist() for j in range(6)],
                          mom_absmax=[float(np.abs(mom[j]).max()) for j in range(6)]))
        print("c4 problem", k, "side", pr.nx, "p", pr.p, "N", pr.n_dir, flush=True)
    out = _header("c4", "one sweep from phi = 0 of selected problems; moments at sampled flat indices")
    out.update(problems=items, oracle_seconds=time.time() - t)
    _write("c4_some.json", out)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2", "c4", "c5", "c3"]
    for w in which:
        globals()["make_" + w]()
