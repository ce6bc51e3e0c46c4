"""Direction-dependent calibration hot path (SAGECal-style) for AMD MI355X (gfx950).

The compute path lives in a HIP/C++ shared library (``csrc/``) with a C ABI declared in
``include/ddcal.h``; :mod:`paper_1910_13908_amd.ddcal` is the thin ctypes binding that
marshals torch device tensors into it.  :mod:`paper_1910_13908_amd.synth` draws seeded
synthetic observations.  Importing this package loads nothing native: the binding loads
the library on first use and raises if it is missing.
"""
__all__ = ["synth", "ddcal"]
