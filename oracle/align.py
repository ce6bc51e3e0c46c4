"""Unitary alignment of gain solutions (test infrastructure only, see ``oracle/__init__``).

For an unpolarised cluster the cost is unchanged under J_p -> J_p U for any U in U(2)
(a 4-D gauge), and for any cluster under a common phase e^{i theta}; gains are therefore
compared after removing that freedom.  The unitary that best maps J onto J_ref in the
Frobenius norm is the orthogonal Procrustes solution (Schoenemann 1966): with
M = sum_p J_p^H J_ref,p = W S Z^H (SVD), U = W Z^H.
"""
from __future__ import annotations

import numpy as np


def procrustes_unitary(J, J_ref):
    """U in U(2) minimising sum_p ||J_p U - J_ref,p||_F^2.  J, J_ref: [N, 2, 2]."""
    M = np.einsum("pji,pjk->ik", np.conj(J), J_ref)
    W, _, Zh = np.linalg.svd(M)
    return W @ Zh


def phase_only(J, J_ref):
    """e^{i theta} I minimising the same cost over a common phase only."""
    M = np.einsum("pji,pjk->ik", np.conj(J), J_ref)
    return np.exp(1j * np.angle(np.trace(M))) * np.eye(2)


def align_error(J, J_ref, polarised=False):
    """||J U - J_ref||_F / ||J_ref||_F after the best U (unitary or phase only)."""
    U = phase_only(J, J_ref) if polarised else procrustes_unitary(J, J_ref)
    return float(np.linalg.norm(J @ U - J_ref) / np.linalg.norm(J_ref))
