"""The C-ABI library loads on the CPU and exports every function include/ddcal.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    hdr = open(os.path.join(ROOT, "include", "ddcal.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = sorted(set(re.findall(r"\b(ddc_[a-z_]+)\s*\(", hdr)))
    assert len(names) >= 15
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1910_13908_amd", "libddcal.so"))
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_imports_without_gpu():
    from paper_1910_13908_amd import ddcal
    assert set(ddcal.EXPORTS) >= {"ddc_predict", "ddc_residual", "ddc_build_normal_eq",
                                  "ddc_lm_solve", "ddc_calibrate"}
    o = ddcal.default_lm_opts()
    assert o.n_iter == 10 and o.tau == 1e-3 and o.mu_floor == 1e-6 and o.refine_max == 5


def test_binding_round_trips_layouts():
    import numpy as np
    from paper_1910_13908_amd import ddcal
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 4, 5, 2, 2)) + 1j * rng.normal(size=(2, 3, 4, 5, 2, 2))
    assert np.array_equal(ddcal.unplanes(ddcal.planes(x)), x)
    J = rng.normal(size=(3, 7, 2, 2)) + 1j * rng.normal(size=(3, 7, 2, 2))
    assert np.array_equal(ddcal.jones_complex(ddcal.jones_real(J)), J)
    assert ddcal.planes(x)[0, 1, 2, 3, 4] == x[0, 2, 3, 4, 0, 0].imag


def test_binding_without_the_library_raises(tmp_path):
    # the package's Python files without libddcal.so: importing the binding fails loudly
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_1910_13908_amd"
    pkg.mkdir()
    for f in ("__init__.py", "ddcal.py", "synth.py"):
        shutil.copy(os.path.join(ROOT, "paper_1910_13908_amd", f), pkg / f)
    r = subprocess.run([sys.executable, "-c", "import paper_1910_13908_amd.ddcal"],
                       cwd=tmp_path, capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "libddcal.so is missing" in r.stderr


def test_the_package_never_reaches_the_oracle():
    # only the tests, smoke() and the benchmark's CPU baseline may use oracle/
    pkg = os.path.join(ROOT, "paper_1910_13908_amd")
    for f in sorted(os.listdir(pkg)):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
