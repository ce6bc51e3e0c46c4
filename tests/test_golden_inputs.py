"""The stored oracle runs in tests/golden still describe the inputs the tests rebuild: for
each fixture, the problem definition it records equals today's, and the cost at the identity
start recomputed from the seeded generator equals the stored one.  (A change to the
generator would otherwise leave the full-size GPU parity tests comparing against runs on
other data.)"""
import dataclasses
import os
import sys

import numpy as np
import pytest

from oracle import rime
from paper_1910_13908_amd import synth

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_fixtures as mf  # noqa: E402


@pytest.mark.parametrize("name", sorted(mf.FIXTURES))
def test_fixture_inputs_are_reproduced(name):
    cfg, seed = mf.FIXTURES[name]
    d = np.load(mf.path(name))
    assert str(d["config"]) == repr(dataclasses.asdict(cfg))
    assert int(d["seed"]) == seed
    ob = synth.make_obs(cfg, seed=seed)
    V, C = rime.make_vis(ob)
    f0 = rime.cost(V - rime.model(C, synth.identity_jones(ob.K, ob.N), ob.ant_p, ob.ant_q))
    stored = float(d["cost0"]) if cfg.n_clusters == 1 else float(d["totals"][0])
    assert abs(f0 - stored) <= 1e-12 * stored, (f0, stored)
