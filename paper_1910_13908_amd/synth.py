"""Seeded synthetic observations for direction-dependent calibration.

This module only draws inputs: station layouts, uvw tracks, clustered point-source
skies, planted Jones matrices, noise draws and request arrival times.  It holds none of
the calibration arithmetic (no phase, coherency, model or residual): the visibilities
themselves are formed from these draws by whichever implementation consumes them.

The workloads follow the paper's problem statement: N stations with N(N-1)/2 baselines
(Section 3), a sky grouped into clusters with one calibration solution per cluster
(Section 2), on N in {64, 128, 256, 384, 512} (Section 2, SKA1-LOW = 512).  The paper's
artificial data sets are not available, so these draws stand in for them.

Random streams: ``np.random.SeedSequence(seed).spawn(5)`` gives independent streams for
stations, sky, Jones, noise and arrivals, so changing one part leaves the others intact.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

C_LIGHT = 299_792_458.0            # m/s
SIDEREAL_DAY_S = 86_164.0905       # s
DEG = math.pi / 180.0


@dataclasses.dataclass(frozen=True)
class ObsConfig:
    """Shape and distributions of one synthetic calibration problem."""
    n_stations: int
    n_clusters: int
    sources_per_cluster: int
    n_times: int
    freqs_hz: tuple
    disk_radius_m: float = 3000.0
    height_m: float = 10.0             # station heights uniform in [-h, h]
    jones_amp: float = 0.1             # planted J = I + a * CN(0, 1)
    sigma_jy: float = 0.01             # visibility noise CN(0, sigma^2) per correlation
    dec_deg: float = 52.0
    lat_deg: float = 52.9
    ha0_rad: float = 0.0
    dt_s: float = 10.0
    source_radius_deg: float = 3.0     # sources uniform in a disk about the cluster centre
    centre_radius_deg: float = 5.0     # cluster centres uniform in a disk (K > 1)
    flux_log10_range: tuple = (-1.0, 1.0)
    polarised: bool = False            # draw Q, U, V as well (tests only)
    n_sweeps: int = 1
    n_lm: int = 20

    @property
    def n_baselines(self) -> int:
        return self.n_stations * (self.n_stations - 1) // 2

    @property
    def n_chans(self) -> int:
        return len(self.freqs_hz)

    @property
    def n_sources(self) -> int:
        return self.n_clusters * self.sources_per_cluster

    @property
    def n_vis(self) -> int:
        return self.n_baselines * self.n_times * self.n_chans


# The paper's station grid and cluster counts set these workloads; the per-config
# schedules (sweeps x LM iterations) split the iteration totals of each workload.
CONFIGS: Dict[str, ObsConfig] = {
    # N=64 (LOFAR-sized), one cluster of 10 sources, plain FP64 LM, 20 iterations.
    "n64_k1": ObsConfig(64, 1, 10, 10, (150e6,), n_sweeps=1, n_lm=20),
    # N=128, 10 clusters x 20 sources, 4 channels over 140-160 MHz, 5 sweeps x 10 LM.
    "n128_k10": ObsConfig(128, 10, 20, 10, (142.5e6, 147.5e6, 152.5e6, 157.5e6),
                          n_sweeps=5, n_lm=10),
    # N=512 (SKA1-LOW), 20 clusters x 50 sources, 20 km disk, J = I + 0.2 CN(0,1),
    # 3 sweeps x 10 LM.
    "n512_k20": ObsConfig(512, 20, 50, 10, (150e6,), disk_radius_m=20000.0,
                          jones_amp=0.2, n_sweeps=3, n_lm=10),
    # N=256, 10 clusters x 20 sources, 2 channels (differentiable-cost workload).
    "n256_k10": ObsConfig(256, 10, 20, 10, (145e6, 155e6), n_sweeps=5, n_lm=10),
}


@dataclasses.dataclass
class Obs:
    """One synthetic problem.  All arrays are float64 / complex128 / int32 NumPy."""
    cfg: ObsConfig
    seed: int
    ant_p: np.ndarray          # [B] int32, canonical p<q, p-major
    ant_q: np.ndarray          # [B] int32
    enu: np.ndarray            # [N, 3] station east/north/up, metres
    u: np.ndarray              # [T, B] metres, baseline p - q
    v: np.ndarray
    w: np.ndarray
    freqs: np.ndarray          # [F] Hz
    l: np.ndarray              # [S] direction cosines (radians, small field)
    m: np.ndarray
    I: np.ndarray              # [S] Jy
    Q: np.ndarray
    U: np.ndarray
    V: np.ndarray
    cluster_offset: np.ndarray  # [K+1] int32
    jones_true: np.ndarray     # [K, N, 2, 2] complex128
    noise: np.ndarray          # [T, F, B, 2, 2] complex128 (already scaled by sigma)
    suvw: Optional[np.ndarray] = None   # [T, N, 3] station (u, v, w), metres; baseline = p - q

    @property
    def N(self) -> int:
        return self.cfg.n_stations

    @property
    def B(self) -> int:
        return self.cfg.n_baselines

    @property
    def T(self) -> int:
        return self.cfg.n_times

    @property
    def F(self) -> int:
        return self.cfg.n_chans

    @property
    def K(self) -> int:
        return len(self.cluster_offset) - 1


def canonical_baselines(n_stations: int):
    """Baseline index b <-> (p, q), p < q, p-major: b = p(2N-p-1)/2 + (q-p-1)."""
    p, q = np.triu_indices(n_stations, k=1)
    return p.astype(np.int32), q.astype(np.int32)


def _complex_normal(rng: np.random.Generator, shape) -> np.ndarray:
    """CN(0, 1): real and imaginary parts N(0, 1/2), so E|z|^2 = 1."""
    s = math.sqrt(0.5)
    return rng.normal(0.0, s, shape) + 1j * rng.normal(0.0, s, shape)


def _disk(rng: np.random.Generator, n: int, radius: float):
    r = radius * np.sqrt(rng.random(n))
    th = 2.0 * math.pi * rng.random(n)
    return r * np.cos(th), r * np.sin(th)


def stations_enu(cfg: ObsConfig, rng: np.random.Generator) -> np.ndarray:
    e, n = _disk(rng, cfg.n_stations, cfg.disk_radius_m)
    up = rng.uniform(-cfg.height_m, cfg.height_m, cfg.n_stations)
    return np.stack([e, n, up], axis=1)


def station_uvw(cfg: ObsConfig, enu: np.ndarray) -> np.ndarray:
    """Per-station (u, v, w) in metres for each timeslot, shape [T, N, 3].

    Local east/north/up is rotated to equatorial (X, Y, Z) at latitude phi and then
    projected on the (u, v, w) frame of a field at declination delta and hour angle H
    (Thompson, Moran & Swenson, Interferometry and Synthesis in Radio Astronomy, ch. 4).
    The hour angle steps by dt seconds of sidereal time per timeslot.
    """
    lat, dec = cfg.lat_deg * DEG, cfg.dec_deg * DEG
    e, n, up = enu[:, 0], enu[:, 1], enu[:, 2]
    X = -math.sin(lat) * n + math.cos(lat) * up
    Y = e
    Z = math.cos(lat) * n + math.sin(lat) * up
    out = np.empty((cfg.n_times, cfg.n_stations, 3))
    for t in range(cfg.n_times):
        H = cfg.ha0_rad + t * cfg.dt_s * 2.0 * math.pi / SIDEREAL_DAY_S
        sH, cH = math.sin(H), math.cos(H)
        sd, cd = math.sin(dec), math.cos(dec)
        out[t, :, 0] = sH * X + cH * Y
        out[t, :, 1] = -sd * cH * X + sd * sH * Y + cd * Z
        out[t, :, 2] = cd * cH * X - cd * sH * Y + sd * Z
    return out


def make_sky(cfg: ObsConfig, rng: np.random.Generator):
    K, S = cfg.n_clusters, cfg.sources_per_cluster
    ls, ms = [], []
    if K == 1:
        cl, cm = np.zeros(1), np.zeros(1)
    else:
        cl, cm = _disk(rng, K, cfg.centre_radius_deg * DEG)
    for k in range(K):
        dl, dm = _disk(rng, S, cfg.source_radius_deg * DEG)
        ls.append(cl[k] + dl)
        ms.append(cm[k] + dm)
    l = np.concatenate(ls)
    m = np.concatenate(ms)
    lo, hi = cfg.flux_log10_range
    I = 10.0 ** rng.uniform(lo, hi, K * S)
    if cfg.polarised:
        # fractional polarisation up to 30 %, so the brightness matrix stays positive
        frac = 0.3 * rng.random(K * S)
        d = rng.normal(size=(K * S, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        Q, U, V = (I * frac) * d[:, 0], (I * frac) * d[:, 1], (I * frac) * d[:, 2]
    else:
        Q = np.zeros(K * S)
        U = np.zeros(K * S)
        V = np.zeros(K * S)
    offs = np.arange(K + 1, dtype=np.int32) * S
    return l, m, I, Q, U, V, offs


def make_obs(cfg: ObsConfig, seed: int = 0, with_noise: bool = True) -> Obs:
    ss = np.random.SeedSequence(seed).spawn(5)
    r_st, r_sky, r_jones, r_noise = (np.random.default_rng(s) for s in ss[:4])
    enu = stations_enu(cfg, r_st)
    suvw = station_uvw(cfg, enu)
    ap, aq = canonical_baselines(cfg.n_stations)
    buvw = suvw[:, ap, :] - suvw[:, aq, :]
    l, m, I, Q, U, V, offs = make_sky(cfg, r_sky)
    K, N = cfg.n_clusters, cfg.n_stations
    J = np.broadcast_to(np.eye(2), (K, N, 2, 2)) + cfg.jones_amp * _complex_normal(r_jones, (K, N, 2, 2))
    shape = (cfg.n_times, cfg.n_chans, cfg.n_baselines, 2, 2)
    if with_noise and cfg.sigma_jy > 0:
        noise = cfg.sigma_jy * _complex_normal(r_noise, shape)
    else:
        noise = np.zeros(shape, dtype=np.complex128)
    return Obs(cfg=cfg, seed=seed, ant_p=ap, ant_q=aq, enu=enu,
               u=np.ascontiguousarray(buvw[..., 0]), v=np.ascontiguousarray(buvw[..., 1]),
               w=np.ascontiguousarray(buvw[..., 2]), freqs=np.asarray(cfg.freqs_hz, dtype=np.float64),
               l=l, m=m, I=I, Q=Q, U=U, V=V, cluster_offset=offs,
               jones_true=np.ascontiguousarray(J), noise=noise, suvw=np.ascontiguousarray(suvw))


SERVE_N = (64, 128, 256, 384, 512)
SERVE_K = (1, 5, 10, 20)


def serving_configs(n_requests: int = 200, seed: int = 0):
    """Request mix of the serving workload: N uniform over the paper's station counts, K uniform
    over {1, 5, 10, 20} clusters of 20 sources, T=10, F=1, 3 km disk, J = I + 0.1 CN(0,1).
    Schedules: K = 1 runs 1 sweep x 20 LM iterations, otherwise 2 sweeps x 10."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(5)[4])
    out = []
    for i in range(n_requests):
        N = int(rng.choice(SERVE_N))
        K = int(rng.choice(SERVE_K))
        sweeps, n_lm = (1, 20) if K == 1 else (2, 10)
        out.append((ObsConfig(N, K, 20, 10, (150e6,), n_sweeps=sweeps, n_lm=n_lm), 1000 + i))
    return out


def identity_jones(n_clusters: int, n_stations: int) -> np.ndarray:
    return np.ascontiguousarray(np.broadcast_to(np.eye(2, dtype=np.complex128),
                                                (n_clusters, n_stations, 2, 2)))


def poisson_arrivals(rate_hz: float, n: int, seed: int = 0) -> np.ndarray:
    """Arrival times (s) of n requests of a Poisson process; rate 0 = all at t = 0."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(5)[4])
    if rate_hz <= 0:
        return np.zeros(n)
    return np.cumsum(rng.exponential(1.0 / rate_hz, n))
