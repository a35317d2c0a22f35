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
  c5_full.json  512x512, p=4, S16, one sweep of all 144 directions from
                phi = 0: moments at sampled nodes
  c5_si5.json   the same, 5 source iterations: residual history and moments
                at sampled nodes after each iteration
  c3_si10.json  256x256 curved, p=3, S12, 10 source iterations: residual
                history and scalar flux at sampled nodes after the last

Usage: python tests/golden/make_golden.py [--threads T] [c2 c3 c4 c5 c5_full c5_si5 c3_si10]
(c2 c4 c5 c3 by default).  --threads sweeps T directions at a time on OpenMP
threads; the oracle sums them in direction order, so the values do not
depend on T.
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


THREADS = 1


def make_c5_full():
    (pr,), _ = P.make_config("c5")
    t = time.time()
    r = O.sweep(pr, want_psi=False, threads=THREADS)
    rng = np.random.default_rng(SAMPLE_SEED + 51)
    idx = _sample_nodes(rng, pr.n_elem, pr.n, 400)
    mom = r["mom"].reshape(6, -1)
    out = _header("c5", "one sweep of every direction from phi = 0; moments at sampled flat indices")
    out.update(index=idx.tolist(), mom=[mom[k, idx].tolist() for k in range(6)],
               mom_absmax=[float(np.abs(mom[k]).max()) for k in range(6)], oracle_seconds=time.time() - t)
    _write("c5_full.json", out)


def _si_fixture(cfg, n_iter, seed, name, what):
    (pr,), _ = P.make_config(cfg)
    t = time.time()
    rng = np.random.default_rng(seed)
    idx = _sample_nodes(rng, pr.n_elem, pr.n, 400)
    phi_hist, mom = [], None
    phi = None
    resid = []
    for k in range(n_iter):
        r = O.source_iteration(pr, 1, phi0=phi, threads=THREADS)
        mom = r["mom"]
        resid.append(float(r["resid"][0]))
        phi = mom[0].copy()
        phi_hist.append(phi.reshape(-1)[idx].tolist())
        print(name, "iteration", k + 1, "resid %.6e" % resid[-1], "%.0f s" % (time.time() - t), flush=True)
    flat = mom.reshape(6, -1)
    out = _header(cfg, what)
    out.update(n_iter=n_iter, resid=resid, index=idx.tolist(), phi=phi_hist,
               phi_absmax=float(np.abs(flat[0]).max()), mom=[flat[k, idx].tolist() for k in range(6)],
               mom_absmax=[float(np.abs(flat[k]).max()) for k in range(6)], oracle_seconds=time.time() - t)
    _write(name, out)


def make_c5_si5():
    _si_fixture("c5", 5, SAMPLE_SEED + 52, "c5_si5.json",
                "5 source iterations from phi = 0; residual history, scalar flux at sampled flat indices after "
                "each iteration, moments of the last")


def make_c3_si10():
    _si_fixture("c3", 10, SAMPLE_SEED + 31, "c3_si10.json",
                "10 source iterations from phi = 0; residual history, scalar flux at sampled flat indices after "
                "each iteration, moments of the last")


if __name__ == "__main__":
    args = sys.argv[1:]
    if args[:1] == ["--threads"]:
        THREADS = int(args[1])
        args = args[2:]
    which = args or ["c2", "c4", "c5", "c3"]
    for w in which:
        globals()["make_" + w]()
