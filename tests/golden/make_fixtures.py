"""Writes the stored oracle results that the full-size GPU parity tests compare against.

Run from the repository root:  python tests/golden/make_fixtures.py [name ...]
(no name: all).  Only the FP64 oracle (``oracle/``) and the seeded input generator
(``paper_1910_13908_amd.synth``, which holds no calibration arithmetic) are called: every
stored value is the oracle's.  The tests rebuild the same inputs from the same seeds.

Fixtures (one ``.npz`` each, loaded with ``numpy.load`` without pickles):

* ``lm_n512_k1_seed0``: one cluster of 50 sources at the SKA1-LOW station count (N = 512,
  130816 baselines, T = 10, F = 1, 20 km disk, J = I + 0.2 CN(0,1), sigma = 0.01 Jy), ten
  FP64 Levenberg-Marquardt iterations from identity Jones: the 8N = 4096 normal matrix of
  the paper's largest array (Section 2).  Stores the final Jones and the per-iteration
  cost, damping and accept trace.
* ``sage_n128_k10_seed0``: the N = 128 mixed-precision workload (8128 baselines, K = 10
  clusters x 20 sources, T = 10, F = 4 channels over 140-160 MHz), 5 SAGE sweeps x 10 LM
  iterations in FP64 from identity Jones.  Stores the final Jones of every cluster, the
  per-visit costs and the final total cost.
* ``sage_n512_k4_seed0``: SAGE at the SKA1-LOW station count with the bench workload's
  cluster size and schedule (N = 512, 50 sources per cluster, T = 10, 20 km disk,
  J = I + 0.2 CN(0,1), 3 sweeps x 10 LM iterations) on four clusters, in FP64 from identity
  Jones.  Stored like the N = 128 run.
"""
from __future__ import annotations

import dataclasses
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import rime, lm  # noqa: E402
from paper_1910_13908_amd import synth  # noqa: E402

# The problems, named by what they are; the tests import these definitions.
LM_N512 = synth.ObsConfig(512, 1, 50, 10, (150e6,), disk_radius_m=20000.0, jones_amp=0.2,
                          n_sweeps=1, n_lm=10)
SAGE_N128 = synth.CONFIGS["n128_k10"]
# the SKA1-LOW workload's station count, cluster size and schedule with four of its clusters
SAGE_N512 = synth.ObsConfig(512, 4, 50, 10, (150e6,), disk_radius_m=20000.0, jones_amp=0.2,
                            n_sweeps=3, n_lm=10)

FIXTURES = {
    "lm_n512_k1_seed0": (LM_N512, 0),
    "sage_n128_k10_seed0": (SAGE_N128, 0),
    "sage_n512_k4_seed0": (SAGE_N512, 0),
}


def path(name: str) -> str:
    return os.path.join(HERE, name + ".npz")


def write_lm(name, cfg, seed):
    ob = synth.make_obs(cfg, seed=seed)
    t0 = time.time()
    V, C = rime.make_vis(ob)
    t1 = time.time()
    J0 = synth.identity_jones(1, ob.N)[0]
    J, info = lm.lm_solve(V, C[0], J0, ob.ant_p, ob.ant_q, n_iter=cfg.n_lm)
    t2 = time.time()
    np.savez(path(name), jones=J, cost0=info.cost0, costs=np.array(info.costs),
             accepted=np.array(info.accepted), mu_effs=np.array(info.mu_effs),
             mus=np.array(info.mus), nus=np.array(info.nus),
             trial_costs=np.array(info.trial_costs),
             config=repr(dataclasses.asdict(cfg)), seed=seed)
    print(f"{name}: predict {t1 - t0:.1f} s, {cfg.n_lm} LM iterations {t2 - t1:.1f} s, "
          f"cost {info.cost0:.6f} -> {info.cost:.6f}, accepted {info.accepted}", flush=True)


def write_sage(name, cfg, seed):
    ob = synth.make_obs(cfg, seed=seed)
    t0 = time.time()
    V, C = rime.make_vis(ob)
    t1 = time.time()
    J0 = synth.identity_jones(ob.K, ob.N)
    J, R, infos, totals = lm.calibrate(V, C, J0, ob.ant_p, ob.ant_q, n_sweeps=cfg.n_sweeps,
                                       n_lm=cfg.n_lm, track_total_cost=True)
    t2 = time.time()
    cost0 = np.array([[i.cost0 for i in row] for row in infos])
    cost = np.array([[i.cost for i in row] for row in infos])
    n_acc = np.array([[i.n_accept for i in row] for row in infos])
    np.savez(path(name), jones=J, visit_cost0=cost0, visit_cost=cost, visit_accepts=n_acc,
             totals=np.array(totals), final_cost=float(rime.cost(R)),
             config=repr(dataclasses.asdict(cfg)), seed=seed)
    print(f"{name}: predict {t1 - t0:.1f} s, calibrate {t2 - t1:.1f} s, total cost "
          f"{totals[0]:.6f} -> {totals[-1]:.6f}", flush=True)


def main(names):
    for name in names or list(FIXTURES):
        cfg, seed = FIXTURES[name]
        if cfg.n_clusters == 1:
            write_lm(name, cfg, seed)
        else:
            write_sage(name, cfg, seed)


if __name__ == "__main__":
    main(sys.argv[1:])
