"""Gauss-Newton normal equations of one cluster, built by brute force in FP64.

Test infrastructure only (see ``oracle/__init__``).

Parameters (a reading; the paper gives no layout): x in R^{8N}, with
x[8p + 2e + 0] = Re (J_p)_e and x[8p + 2e + 1] = Im (J_p)_e, where e = 0..3 walks the
entries 00, 01, 10, 11 of the 2x2 Jones matrix in row-major order.  The residual of one
visibility is flattened the same way (entry e, then re/im).

For one cluster the model of baseline (p, q) is M = J_p C J_q^H.  It is linear in J_p and
in J_q^H, so the real Jacobian A = dM/dx is written out column by column:

* column (p, j):  vec(E_j G)       with G  = C J_q^H
* column (q, j):  vec(Hm E_j^H)    with Hm = J_p C

where E_j runs over the eight real/imaginary unit matrices (1 or i at entry e).  The normal
matrix is H = A^T A and the right-hand side is g = A^T r with r = Y - M, so that the
Gauss-Newton step d solves H d = g.  Everything here is the plain definition: the per-
visibility 8x16 Jacobian block is materialised and multiplied out.
"""
from __future__ import annotations

import numpy as np

from .rime import model_cluster, cost


def unit_matrices():
    """E_j, j = 2e + c: 1 (c = 0) or i (c = 1) at entry e = 2a + b of a 2x2 matrix."""
    E = np.zeros((8, 2, 2), dtype=np.complex128)
    for e in range(4):
        a, b = divmod(e, 2)
        E[2 * e, a, b] = 1.0
        E[2 * e + 1, a, b] = 1.0j
    return E


def to_real8(M):
    """[..., 2, 2] complex -> [..., 8] real in (entry row-major, re/im) order."""
    M = np.asarray(M)
    flat = M.reshape(M.shape[:-2] + (4,))
    out = np.empty(M.shape[:-2] + (8,), dtype=np.float64)
    out[..., 0::2] = flat.real
    out[..., 1::2] = flat.imag
    return out


def from_real8(x):
    """[..., 8] real -> [..., 2, 2] complex (inverse of ``to_real8``)."""
    x = np.asarray(x, dtype=np.float64)
    z = x[..., 0::2] + 1j * x[..., 1::2]
    return z.reshape(x.shape[:-1] + (2, 2))


def pack_jones(J):
    """[N, 2, 2] complex -> x [8N]."""
    return to_real8(J).reshape(-1)


def unpack_jones(x):
    """x [8N] -> [N, 2, 2] complex."""
    x = np.asarray(x, dtype=np.float64)
    return from_real8(x.reshape(-1, 8))


def jacobian_blocks(C, Jp, Jq):
    """Per-visibility real Jacobian blocks of M = J_p C J_q^H.

    C: [..., 2, 2]; Jp, Jq: broadcastable [..., 2, 2].  Returns (A_p, A_q), each
    [..., 8 (residual), 8 (parameter)].
    """
    E = unit_matrices()
    G = C @ np.conj(np.swapaxes(Jq, -1, -2))        # C J_q^H
    Hm = Jp @ C                                     # J_p C
    shp = np.broadcast_shapes(G.shape, Hm.shape)[:-2]
    A_p = np.empty(shp + (8, 8))
    A_q = np.empty(shp + (8, 8))
    for j in range(8):
        A_p[..., :, j] = to_real8(E[j] @ G)
        A_q[..., :, j] = to_real8(Hm @ np.conj(E[j].T))
    return A_p, A_q


def normal_equations(Y, C, J, ant_p, ant_q, chunk_times=1):
    """(H, g, f) of one cluster at Jones J.

    Y, C: [T, F, B, 2, 2] complex (data for this cluster, its coherencies); J: [N, 2, 2].
    H: [8N, 8N] = A^T A; g: [8N] = A^T r with r = Y - J_p C J_q^H; f = ||r||^2.
    """
    T, F, B = C.shape[:3]
    N = J.shape[0]
    ant_p = np.asarray(ant_p)
    ant_q = np.asarray(ant_q)
    H = np.zeros((8 * N, 8 * N))
    g = np.zeros(8 * N)
    Hpp = np.zeros((B, 8, 8))
    Hqq = np.zeros((B, 8, 8))
    Hpq = np.zeros((B, 8, 8))
    gp = np.zeros((B, 8))
    gq = np.zeros((B, 8))
    f = 0.0
    Jp = J[ant_p]
    Jq = J[ant_q]
    for t0 in range(0, T, chunk_times):
        Cc = C[t0:t0 + chunk_times]
        Yc = Y[t0:t0 + chunk_times]
        R = Yc - model_cluster(Cc, J, ant_p, ant_q)
        f += cost(R)
        r = to_real8(R)                                   # [t, F, B, 8]
        A_p, A_q = jacobian_blocks(Cc, Jp, Jq)             # [t, F, B, 8, 8]
        Hpp += np.einsum("tfbri,tfbrj->bij", A_p, A_p, optimize=True)
        Hqq += np.einsum("tfbri,tfbrj->bij", A_q, A_q, optimize=True)
        Hpq += np.einsum("tfbri,tfbrj->bij", A_p, A_q, optimize=True)
        gp += np.einsum("tfbri,tfbr->bi", A_p, r, optimize=True)
        gq += np.einsum("tfbri,tfbr->bi", A_q, r, optimize=True)
    Hd = np.zeros((N, 8, 8))
    np.add.at(Hd, ant_p, Hpp)
    np.add.at(Hd, ant_q, Hqq)
    gd = np.zeros((N, 8))
    np.add.at(gd, ant_p, gp)
    np.add.at(gd, ant_q, gq)
    for n in range(N):
        H[8 * n:8 * n + 8, 8 * n:8 * n + 8] = Hd[n]
    for b in range(B):
        p, q = int(ant_p[b]), int(ant_q[b])
        H[8 * p:8 * p + 8, 8 * q:8 * q + 8] = Hpq[b]
        H[8 * q:8 * q + 8, 8 * p:8 * p + 8] = Hpq[b].T
    g[:] = gd.reshape(-1)
    return H, g, f
