"""Pin of the oracle's multi-cluster cost gradient against central finite differences."""
import numpy as np

from oracle import rime, adjoint, normal_eq as ne
from paper_1910_13908_amd import synth


def test_gradient_matches_central_differences():
    cfg = synth.ObsConfig(5, 3, 3, 2, (145e6, 155e6), polarised=True, jones_amp=0.2)
    ob = synth.make_obs(cfg, seed=11)
    V, C = rime.make_vis(ob)
    rng = np.random.default_rng(12)
    J = ob.jones_true + 0.1 * (rng.normal(size=ob.jones_true.shape) + 1j * rng.normal(size=ob.jones_true.shape))
    f, grad = adjoint.cost_and_gradient(V, C, J, ob.ant_p, ob.ant_q)
    assert abs(f - rime.cost(rime.residual(V, C, J, ob.ant_p, ob.ant_q))) <= 1e-13 * f
    h = 1e-6
    x = ne.to_real8(J)                          # [K, N, 8]
    fd = np.empty_like(x)
    for idx in np.ndindex(x.shape):
        e = np.zeros_like(x)
        e[idx] = h
        fp = rime.cost(rime.residual(V, C, ne.from_real8(x + e), ob.ant_p, ob.ant_q))
        fm = rime.cost(rime.residual(V, C, ne.from_real8(x - e), ob.ant_p, ob.ant_q))
        fd[idx] = (fp - fm) / (2 * h)
    assert np.max(np.abs(grad - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_gradient_vanishes_at_noiseless_truth():
    cfg = synth.ObsConfig(6, 2, 3, 2, (150e6,))
    ob = synth.make_obs(cfg, seed=13, with_noise=False)
    V, C = rime.make_vis(ob)
    f, grad = adjoint.cost_and_gradient(V, C, ob.jones_true, ob.ant_p, ob.ant_q)
    assert f < 1e-24 and np.max(np.abs(grad)) < 1e-10
