"""Predict, model, residual and cost: the measurement equation in FP64.

Test infrastructure only (see ``oracle/__init__``).

Measurement equation (Hamaker, Bregman & Sault 1996) for the paper's problem: N stations,
baselines p<q (Section 3: N(N-1)/2 of them), a sky grouped into K clusters with one 2x2
Jones matrix per station per cluster (Section 2):

    V_pq(t, f) = sum_k J_{p,k} C_{pq,k}(t, f) J_{q,k}^H + noise
    C_{pq,k}(t, f) = sum_{s in k} B_s exp(-2 pi i (u l_s + v m_s + w (n_s - 1)) f / c)

with (u, v, w) the baseline p - q in metres at timeslot t, (l, m) the source direction
cosines and B_s the source brightness matrix for linear feeds.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299_792_458.0


def n_minus_1(l, m):
    """n - 1 = sqrt(1 - l^2 - m^2) - 1, written without cancellation."""
    l = np.asarray(l, dtype=np.float64)
    m = np.asarray(m, dtype=np.float64)
    r2 = l * l + m * m
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def brightness(I, Q, U, V):
    """Brightness matrix of a source for linear feeds: [[I+Q, U+iV], [U-iV, I-Q]].

    No factor 1/2: a 1 Jy unpolarised source gives XX = YY = 1 (a reading; the paper
    gives no convention).  Returns [..., 2, 2] complex128.
    """
    I, Q, U, V = (np.asarray(a, dtype=np.float64) for a in (I, Q, U, V))
    out = np.empty(I.shape + (2, 2), dtype=np.complex128)
    out[..., 0, 0] = I + Q
    out[..., 0, 1] = U + 1j * V
    out[..., 1, 0] = U - 1j * V
    out[..., 1, 1] = I - Q
    return out


def predict(u, v, w, freqs, l, m, I, Q, U, V, cluster_offset, baselines=None):
    """Model coherencies of every cluster, C[k, t, f, b, 2, 2] (complex128).

    u, v, w: [T, B] metres; freqs: [F] Hz; sky arrays: [S]; cluster_offset: [K+1].
    ``baselines`` optionally restricts the output to a subset of baseline columns (used to
    check full-size runs on a sample).  Each term is evaluated straight from its definition.
    """
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    if baselines is not None:
        u, v, w = u[:, baselines], v[:, baselines], w[:, baselines]
    T, B = u.shape
    freqs = np.asarray(freqs, dtype=np.float64)
    F = freqs.shape[0]
    K = len(cluster_offset) - 1
    n1 = n_minus_1(l, m)
    Bs = brightness(I, Q, U, V)
    out = np.zeros((K, T, F, B, 2, 2), dtype=np.complex128)
    for k in range(K):
        for s in range(int(cluster_offset[k]), int(cluster_offset[k + 1])):
            geo = u * l[s] + v * m[s] + w * n1[s]                 # [T, B] metres
            for f in range(F):
                ph = np.exp(-2j * np.pi * geo * freqs[f] / C_LIGHT)  # [T, B]
                out[k, :, f, :, :, :] += ph[:, :, None, None] * Bs[s]
    return out


def model_cluster(C, J, ant_p, ant_q):
    """J_p C J_q^H for one cluster.  C: [T, F, B, 2, 2]; J: [N, 2, 2] -> [T, F, B, 2, 2]."""
    Jp = J[ant_p]
    Jq = J[ant_q]
    # (J_q^H)_{jl} = conj(J_q)_{lj}
    return np.einsum("bij,tfbjk,blk->tfbil", Jp, C, Jq.conj(), optimize=True)


def model(C, J, ant_p, ant_q):
    """sum_k J_{p,k} C_k J_{q,k}^H.  C: [K, T, F, B, 2, 2]; J: [K, N, 2, 2]."""
    out = np.zeros(C.shape[1:], dtype=np.complex128)
    for k in range(C.shape[0]):
        out += model_cluster(C[k], J[k], ant_p, ant_q)
    return out


def residual(Vis, C, J, ant_p, ant_q):
    """R = V - sum_k J_{p,k} C_k J_{q,k}^H."""
    return Vis - model(C, J, ant_p, ant_q)


def cost(R):
    """f = sum over baselines, timeslots, channels of ||R||_F^2 (unit weights, no 1/2)."""
    R = np.asarray(R)
    return float(np.sum(R.real * R.real + R.imag * R.imag))


def make_vis(obs):
    """Synthetic data from a ``synth.Obs``: V = sum_k J_true C_k J_true^H + noise."""
    C = predict(obs.u, obs.v, obs.w, obs.freqs, obs.l, obs.m, obs.I, obs.Q, obs.U, obs.V,
                obs.cluster_offset)
    return model(C, obs.jones_true, obs.ant_p, obs.ant_q) + obs.noise, C
