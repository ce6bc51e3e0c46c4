"""The oracle's CPU pins fail on plausible mistakes.  Each case plants one mistake in a copy
of ``oracle/`` (never in the oracle itself) and runs the pin module that should catch it;
the unmodified copy passes the same modules.  The mistakes are the kinds a reimplementation
from the definitions could make: a sign, a conjugate or a transpose, a dropped term, an
index, a factor, and the steps of the damping schedule."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# (oracle file, text, planted text, pin module)
MISTAKES = {
    "phase sign": ("rime.py", "np.exp(-2j * np.pi * geo", "np.exp(2j * np.pi * geo",
                   "test_oracle_predict.py"),
    "n - 1 sign": ("rime.py", "return -r2 / (1.0 + np.sqrt(1.0 - r2))",
                   "return r2 / (1.0 + np.sqrt(1.0 - r2))", "test_oracle_predict.py"),
    "brightness U + iV": ("rime.py", "out[..., 0, 1] = U + 1j * V", "out[..., 0, 1] = U - 1j * V",
                          "test_oracle_predict.py"),
    "first channel's frequency": ("rime.py", "geo * freqs[f] / C_LIGHT", "geo * freqs[0] / C_LIGHT",
                                  "test_oracle_predict.py"),
    "J_q not conjugated": ("rime.py", "Jp, C, Jq.conj()", "Jp, C, Jq", "test_oracle_model.py"),
    "cost without imaginary parts": (
        "rime.py", "return float(np.sum(R.real * R.real + R.imag * R.imag))",
        "return float(np.sum(R.real * R.real))", "test_oracle_model.py"),
    "q-columns without conjugate": (
        "normal_eq.py", "A_q[..., :, j] = to_real8(Hm @ np.conj(E[j].T))",
        "A_q[..., :, j] = to_real8(Hm @ E[j].T)", "test_oracle_normal_eq.py"),
    "cross block not transposed": (
        "normal_eq.py", "H[8 * q:8 * q + 8, 8 * p:8 * p + 8] = Hpq[b].T",
        "H[8 * q:8 * q + 8, 8 * p:8 * p + 8] = Hpq[b]", "test_oracle_normal_eq.py"),
    "square for cube": ("lm.py", "1.0 - (2.0 * rho - 1.0) ** 3", "1.0 - (2.0 * rho - 1.0) ** 2",
                        "test_oracle_lm_damping.py"),
    "halved denominator": ("lm.py", "denom = float(d @ (mu_eff * d + g))",
                           "denom = 0.5 * float(d @ (mu_eff * d + g))", "test_oracle_lm_damping.py"),
    "acceptance threshold": ("lm.py", "if rho > 0.0:", "if rho > 0.25:", "test_oracle_lm_damping.py"),
    "nu not doubled": ("lm.py", "            nu = 2.0 * nu", "            nu = 4.0 * nu",
                       "test_oracle_lm_damping.py"),
    "failed factorisation not counted": ("lm.py", "            info.n_notpd += 1", "            pass",
                                         "test_oracle_lm_damping.py"),
    "SAGE without the cluster's model": (
        "lm.py", "            Y = R + model_cluster(C[k], J[k], ant_p, ant_q)", "            Y = R",
        "test_oracle_lm.py"),
    "gradient sign": ("adjoint.py", "grad[k] = -2.0 * g.reshape(N, 8)", "grad[k] = 2.0 * g.reshape(N, 8)",
                      "test_oracle_adjoint.py"),
    "Procrustes order": ("align.py", "return W @ Zh", "return Zh @ W", "test_oracle_model.py"),
}


@pytest.fixture(scope="module")
def sandbox(tmp_path_factory):
    box = tmp_path_factory.mktemp("oracle_copy")
    shutil.copytree(os.path.join(ROOT, "oracle"), box / "oracle",
                    ignore=shutil.ignore_patterns("__pycache__"))
    (box / "tests").mkdir()
    (box / "paper_1910_13908_amd").mkdir()
    for f in ("conftest.py",) + tuple(sorted({m[3] for m in MISTAKES.values()})):
        shutil.copy(os.path.join(ROOT, "tests", f), box / "tests" / f)
    for f in ("__init__.py", "synth.py"):
        shutil.copy(os.path.join(ROOT, "paper_1910_13908_amd", f), box / "paper_1910_13908_amd" / f)
    shutil.copy(os.path.join(ROOT, "pytest.ini"), box / "pytest.ini")
    return box


def _run(box, module):
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join("tests", module), "-x", "-q",
                        "-p", "no:cacheprovider"], cwd=box, capture_output=True, text=True,
                       timeout=600, env={**os.environ, "PYTHONDONTWRITEBYTECODE": "1"})
    return r.returncode, (r.stdout.strip().splitlines() or [""])[-1]


def test_unmodified_copy_passes(sandbox):
    for module in sorted({m[3] for m in MISTAKES.values()}):
        rc, last = _run(sandbox, module)
        assert rc == 0, (module, last)


@pytest.mark.parametrize("name", sorted(MISTAKES))
def test_planted_mistake_fails_a_pin(sandbox, name):
    fname, text, planted, module = MISTAKES[name]
    path = sandbox / "oracle" / fname
    src = path.read_text()
    assert src.count(text) == 1, (name, src.count(text))
    try:
        path.write_text(src.replace(text, planted))
        rc, last = _run(sandbox, module)
    finally:
        path.write_text(src)
    assert rc != 0, (name, last)
