#!/usr/bin/env python3
"""Benchmark of the calibration hot path on one MI355X.

One step = one full calibration of the N=512 (SKA1-LOW scale) workload through the C ABI:
predict of all 20 clusters x 50 sources, then 3 SAGE sweeps x 20 clusters x 10 LM
iterations (600 LM iterations, each: normal-equation build over 1,308,160 visibilities,
4096 x 4096 damped Cholesky, triangular solves, FP64 refinement, trial cost, accept/reject).
Inputs (uvw, sky, noisy visibilities) are resident in HBM before the timed region; the Jones
start from identity at the beginning of every step.

Prints ONE JSON line (metric = LM iterations per second, mixed precision).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma_tflops": 157.3, "fp64_mfma_tflops": 78.6, "hbm_gbs": 8000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="n512_k20")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--mode", default="lm", choices=["lm", "serve", "lbfgs", "copy", "scan", "predict"],
                    help="lm: the headline calibration step; serve: the request stream; "
                         "lbfgs: gradient-based solve vs LM; copy: a plain device copy of "
                         "known size (reference for the HBM byte counters); scan: calibration "
                         "runtime over the station-count x cluster-count grid; predict: the "
                         "direct predict of the workload alone (for counter runs)")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the served stream (mixed and FP64) in the lm mode")
    return ap.parse_args()


def _progress(msg):
    """Progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = int(np.floor(k)), int(np.ceil(k))
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def serve_measure(n_requests=200, n_slots=4, seed=0, precision="mixed"):
    """Served stream: closed loop (all at t=0) for the saturation rate, then Poisson arrivals
    at 0.5x and 0.9x that rate; solves/s and p50/p99 latency from submit to completion."""
    import threading
    import queue
    import torch
    from paper_1910_13908_amd import synth, ddcal as dd
    prec = dd.MIXED if precision == "mixed" else dd.FP64
    dt = torch.float32 if prec == dd.MIXED else torch.float64
    ctx = dd.Context(0)
    reqs = []
    gen = torch.Generator(device="cuda")
    for cfg, rseed in synth.serving_configs(n_requests, seed):
        ob = synth.make_obs(cfg, seed=rseed, with_noise=False)
        obs, sky = dd.device_obs(ob), dd.device_sky(ob)
        gen.manual_seed(rseed)
        noise = (cfg.sigma_jy * np.sqrt(0.5)) * torch.randn((8, ob.T, ob.F, ob.B), generator=gen,
                                                            device="cuda", dtype=torch.float64)
        noise = noise.to(dt).contiguous()
        coh = ctx.predict(obs, sky, prec)
        Jt = torch.as_tensor(dd.jones_real(ob.jones_true), device="cuda").contiguous()
        V = torch.empty_like(noise)
        ctx.add_model(obs, ob.K, noise, coh, Jt, 1.0, prec, V)
        del coh, noise
        J0 = torch.as_tensor(dd.jones_real(synth.identity_jones(ob.K, ob.N)), device="cuda").contiguous()
        reqs.append(dict(cfg=cfg, obs=obs, sky=sky, V=V, J0=J0, J=J0.clone(), K=ob.K, N=ob.N))
    torch.cuda.synchronize()
    ctx.close()
    foot = max(dd.calibrate_footprint(r["obs"], r["K"], r["cfg"].n_sweeps, r["cfg"].n_lm, prec)
               for r in reqs)
    budget = int(n_slots * foot * 1.05) + (64 << 20)
    srv = dd.Server(0, n_slots=n_slots, hbm_budget_bytes=budget)

    def run(arrivals, subset=None):
        rs = reqs if subset is None else reqs[:subset]
        for r in rs:
            r["J"].copy_(r["J0"])
        torch.cuda.synchronize()
        q = queue.Queue()
        lat = []

        def collector():
            while True:
                item = q.get()
                if item is None:
                    return
                _, l, _ = srv.wait(item)
                lat.append(l)

        th = threading.Thread(target=collector)
        th.start()
        t0 = time.perf_counter()
        for r, ta in zip(rs, arrivals):
            dtw = t0 + ta - time.perf_counter()
            if dtw > 0:
                time.sleep(dtw)
            lm = dd.default_lm_opts(n_iter=r["cfg"].n_lm, precision=prec)
            q.put(srv.submit(r["obs"], r["sky"], r["V"], r["J"], r["cfg"].n_sweeps, lm))
        q.put(None)
        th.join()
        el = time.perf_counter() - t0
        return {"solves_per_s": len(rs) / el, "p50_latency_s": _percentile(lat, 0.5),
                "p99_latency_s": _percentile(lat, 0.99), "elapsed_s": el}

    run(np.zeros(len(reqs)), subset=24)      # warm-up pass (code objects, every request shape)
    closed = run(np.zeros(len(reqs)))
    _progress(f"serve {precision}: closed loop {closed['solves_per_s']:.2f} solves/s")
    sat = closed["solves_per_s"]
    out = {"requests": len(reqs), "slots": n_slots, "arena_bytes": budget,
           "mix": "N in {64,128,256,384,512}, K in {1,5,10,20} x 20 sources, T=10, F=1",
           "closed_loop": closed}
    for frac in (0.5, 0.9):
        arr = synth.poisson_arrivals(frac * sat, len(reqs), seed=seed + 7)
        out[f"poisson_{frac}x"] = dict(run(arr), rate_hz=frac * sat)
        _progress(f"serve {precision}: Poisson {frac}x p50 {out[f'poisson_{frac}x']['p50_latency_s']:.3f} s")
    out["server"] = srv.stats()
    srv.close()
    return out


def lbfgs_measure(seed=0, n_iter=200):
    """Gradient-based solve (adjoint kernel + torch L-BFGS, plain and with a diagonal Jacobi
    change of variables) vs LM on the N=256 workload."""
    import torch
    from paper_1910_13908_amd import synth, ddcal as dd, autograd as ag
    cfg = synth.CONFIGS["n256_k10"]
    ob = synth.make_obs(cfg, seed=seed)
    ctx = dd.Context(0)
    obs, sky = dd.device_obs(ob), dd.device_sky(ob)
    out = {"workload": "n256_k10: N=256, K=10 x 20 sources, T=10, F=2"}
    for pname, prec, dt in (("mixed", dd.MIXED, torch.float32), ("fp64", dd.FP64, torch.float64)):
        noise = torch.as_tensor(dd.planes(ob.noise), dtype=dt, device="cuda").contiguous()
        coh = ctx.predict(obs, sky, prec)
        Jt = torch.as_tensor(dd.jones_real(ob.jones_true), device="cuda").contiguous()
        V = torch.empty_like(noise)
        ctx.add_model(obs, ob.K, noise, coh, Jt, 1.0, prec, V)
        J0 = torch.as_tensor(dd.jones_real(synth.identity_jones(ob.K, ob.N)), device="cuda").contiguous()
        prob = ag.Problem(ctx, obs, ob.K, V, coh, prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Jl, costs = ag.lbfgs_calibrate(prob, J0, n_iter=n_iter)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t0
        t0 = time.perf_counter()
        scale = ag.jacobi_scaling(prob, J0)
        Jp, costs_p = ag.lbfgs_calibrate(prob, J0, n_iter=n_iter, scaling=scale)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t0
        J = J0.clone()
        t0 = time.perf_counter()
        infos = ctx.calibrate(obs, sky, V, J, cfg.n_sweeps, dd.default_lm_opts(n_iter=cfg.n_lm, precision=prec))
        torch.cuda.synchronize()
        t_m = time.perf_counter() - t0
        f0 = ctx.residual(obs, ob.K, V, coh, J0, prec, None)
        out[pname] = {"cost_at_start": f0,
                      "lbfgs_final_cost": costs[-1], "lbfgs_s": t_l, "lbfgs_iters": n_iter,
                      "lbfgs_cost_trace": [costs[i] for i in (0, 9, 49, 99, n_iter - 1)],
                      "jacobi_lbfgs_final_cost": costs_p[-1], "jacobi_lbfgs_s": t_p,
                      "jacobi_lbfgs_cost_trace": [costs_p[i] for i in (0, 9, 49, 99, n_iter - 1)],
                      "lm_final_cost": infos[-1][-1].cost, "lm_s": t_m,
                      "lm_iters": cfg.n_sweeps * ob.K * cfg.n_lm,
                      "cost_at_truth": ctx.residual(obs, ob.K, V, coh, Jt, prec, None)}
        del V, coh, noise
        torch.cuda.empty_cache()
    ctx.close()
    return out


def scan_measure(seed=0, n_lm=10, oracle_max_n=512):
    """Calibration runtime over the paper's station grid and cluster counts (its runtime-vs-N
    and runtime-vs-K experiments, Section 3): N in {64, 128, 256, 384, 512} x K in
    {1, 5, 10, 20, 50} clusters of 20 sources, T=10, F=1, one SAGE sweep of n_lm LM iterations
    per cluster, mixed and FP64.  The time covers predict + calibrate with data resident in
    HBM.  The CPU line is the FP64 oracle's time for one LM iteration of one cluster (at K = 1,
    for N <= oracle_max_n; seconds per iteration at N = 512)."""
    import torch
    from paper_1910_13908_amd import synth, ddcal as dd
    ctx = dd.Context(0)
    rows = []
    for N in synth.SERVE_N:
        for K in (1, 5, 10, 20, 50):
            cfg = synth.ObsConfig(N, K, 20, 10, (150e6,), n_sweeps=1, n_lm=n_lm)
            ob = synth.make_obs(cfg, seed=seed)
            obs, sky = dd.device_obs(ob), dd.device_sky(ob)
            row = {"N": N, "K": K, "vis": ob.B * ob.T * ob.F}
            for pname, prec, dt in (("mixed", dd.MIXED, torch.float32), ("fp64", dd.FP64, torch.float64)):
                noise = torch.as_tensor(dd.planes(ob.noise), dtype=dt, device="cuda").contiguous()
                coh = ctx.predict(obs, sky, prec)
                Jt = torch.as_tensor(dd.jones_real(ob.jones_true), device="cuda").contiguous()
                V = torch.empty_like(noise)
                ctx.add_model(obs, K, noise, coh, Jt, 1.0, prec, V)
                del coh, noise
                J0 = torch.as_tensor(dd.jones_real(synth.identity_jones(K, N)), device="cuda").contiguous()
                J = J0.clone()
                lm = dd.default_lm_opts(n_iter=n_lm, precision=prec)
                ctx.calibrate(obs, sky, V, J, 1, lm, want_info=False)     # warm-up
                torch.cuda.synchronize()
                reps = 3 if N * K <= 2560 else 1
                ts = []
                for _ in range(reps):
                    J.copy_(J0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    ctx.calibrate(obs, sky, V, J, 1, lm, want_info=False)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                row[f"{pname}_s"] = float(np.median(ts))
                row[f"{pname}_lm_iters_per_s"] = K * n_lm / row[f"{pname}_s"]
                del V, J, J0
                torch.cuda.empty_cache()
            if K == 1 and N <= oracle_max_n:
                row["oracle_lm_iter_s"] = _oracle_lm_iteration_s(ob)
            rows.append(row)
            print(json.dumps({"scan_row": row}), file=sys.stderr, flush=True)
    ctx.close()
    return rows


def _oracle_lm_iteration_s(ob):
    """Host time of one FP64 oracle LM iteration of cluster 0 (normal equations, damped solve,
    trial cost)."""
    from oracle import rime, normal_eq as ne, lm as olm
    from paper_1910_13908_amd import synth
    offs = ob.cluster_offset[:2]
    C0 = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, offs)[0]
    Y = rime.model_cluster(C0, ob.jones_true[0], ob.ant_p, ob.ant_q) + ob.noise
    J = synth.identity_jones(1, ob.N)[0]
    t0 = time.perf_counter()
    H, g, f = ne.normal_equations(Y, C0, J, ob.ant_p, ob.ant_q)
    mu = max(1e-3, 1e-6) * float(np.max(np.diag(H)))
    d = olm.damped_solve(H, g, mu)
    rime.cost(Y - rime.model_cluster(C0, ne.unpack_jones(ne.pack_jones(J) + d), ob.ant_p, ob.ant_q))
    return time.perf_counter() - t0


def predict_measure(config="n512_k20", precision="mixed", reps=5, seed=0):
    """The direct predict of a workload, alone: `reps` launches after one warm-up, timed with
    events on the stream it runs on (the unit of the predict counter runs in profiles/)."""
    import torch
    from paper_1910_13908_amd import synth, ddcal as dd
    cfg = synth.CONFIGS[config]
    ob = synth.make_obs(cfg, seed=seed, with_noise=False)
    prec = dd.MIXED if precision == "mixed" else dd.FP64
    ctx = dd.Context(0)
    obs, sky = dd.device_obs(ob), dd.device_sky(ob)
    coh = ctx.predict(obs, sky, prec)
    torch.cuda.synchronize()
    ctx.enable_timing(True, timers=[dd.TIMER_PREDICT])
    for _ in range(reps):
        ctx.predict(obs, sky, prec, out=coh)
    n, ms, terms = ctx.timing(dd.TIMER_PREDICT)
    ctx.enable_timing(False)
    vis = ob.K * ob.B * ob.T * ob.F
    out = {"config": config, "precision": precision, "launches": n, "avg_us": 1e3 * ms / max(n, 1),
           "gvis_per_s": n * vis / (ms * 1e-3) / 1e9, "gterms_per_s": terms / (ms * 1e-3) / 1e9,
           "roofline": _predict_roofline(terms / (ms * 1e-3) / 1e9) if prec == dd.MIXED else None}
    ctx.close()
    return out


# Issue cost of the mixed-precision predict's Stokes-I inner loop, per source-visibility term,
# from the instructions of the generated code (the loop is unrolled by four): 1/4 VGPR move,
# 4 FP64 (multiply, two FMA, fract), 1 FP64->FP32 conversion, 2 transcendental (sin, cos in
# turns) and 2 FP32 FMA.  Lanes per clock per CU from the chip's published vector rates at
# 2.4 GHz on 256 CUs (FP64 78.6 TFLOP/s -> 64 FMA lanes; FP32 157.3 TFLOP/s -> 128 lanes) and,
# for the transcendental unit, a quarter of the FP32 rate (32 lanes); the conversion issues at
# the FP64 rate.  The roof is the term rate at which these issue slots are full.
PREDICT_LANE_CLOCKS_PER_TERM = 0.25 / 128 + 4 / 64 + 1 / 64 + 2 / 32 + 2 / 128
PREDICT_TERM_PEAK_G = 256 * 2.4e9 / PREDICT_LANE_CLOCKS_PER_TERM / 1e9


def _predict_roofline(gterms):
    return {"bound": "alu", "kernel": "k_predict", "unit": "Gterm/s", "achieved": gterms,
            "peak": PREDICT_TERM_PEAK_G, "frac": gterms / PREDICT_TERM_PEAK_G,
            "per_term": "1/4 move + 4 FP64 + 1 cvt + 2 transcendental + 2 FP32 FMA issue slots"}


def copy_measure(mib=1024, reps=5):
    """A plain device-to-device copy of `mib` MiB, `reps` times: the known-size reference that
    scales FETCH_SIZE / WRITE_SIZE counter readings into bytes."""
    import torch
    n = (mib << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"bytes_read_per_copy": n * 4, "bytes_written_per_copy": n * 4, "copies": reps + 1,
            "gbs": 2 * n * 4 * reps / el / 1e9}


def _hbm_roofline(kernel, launches, total_ms, algo_bytes):
    """Achieved algorithmic GB/s of an HBM-bound kernel from the live event timers, with the
    HBM bytes per launch measured by rocprofv3 (profiles/) while that kernel's source is the one
    profiled, else traffic null."""
    import hashlib
    out = {"bound": "hbm", "kernel": kernel, "unit": "GB/s", "peak": PEAK["hbm_gbs"],
           "achieved": None, "frac": None, "traffic": None}
    if launches and total_ms > 0:
        out["achieved"] = algo_bytes / (total_ms * 1e-3) / 1e9
        out["frac"] = out["achieved"] / PEAK["hbm_gbs"]
        out["avg_us"] = 1e3 * total_ms / launches
    try:
        prof = json.load(open(os.path.join(ROOT, "profiles", "hbm_traffic_n512_k20_mixed.json")))
        k = prof["kernels"][kernel]
        src = open(os.path.join(ROOT, k["source"]), "rb").read()
        if hashlib.sha256(src).hexdigest() == k["sha256"]:
            out["traffic"] = k["fetch_bytes"] + k["write_bytes"]
            out["traffic_source"] = "profiles/hbm_traffic_n512_k20_mixed.json"
    except (OSError, KeyError, ValueError):
        pass
    return out


def cpu_baseline(cfg, seed):
    """The FP64 oracle on the host: one LM iteration of cluster 0 at full size."""
    from oracle import rime, normal_eq as ne, lm as olm
    from paper_1910_13908_amd import synth
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    ob = synth.make_obs(cfg, seed=seed)
    offs = ob.cluster_offset[:2]
    t0 = time.perf_counter()
    C0 = rime.predict(ob.u, ob.v, ob.w, ob.freqs, ob.l, ob.m, ob.I, ob.Q, ob.U, ob.V, offs)[0]
    t_pred = time.perf_counter() - t0
    Y = rime.model_cluster(C0, ob.jones_true[0], ob.ant_p, ob.ant_q) + ob.noise
    J = synth.identity_jones(1, ob.N)[0]
    t0 = time.perf_counter()
    H, g, f = ne.normal_equations(Y, C0, J, ob.ant_p, ob.ant_q)
    mu = 1e-3 * float(np.max(np.diag(H)))
    mu_eff = max(mu, 1e-6 * float(np.max(np.diag(H))))
    d = olm.damped_solve(H, g, mu_eff)
    f_new = rime.cost(Y - rime.model_cluster(C0, ne.unpack_jones(ne.pack_jones(J) + d), ob.ant_p, ob.ant_q))
    t_iter = time.perf_counter() - t0
    vis = ob.B * ob.T * ob.F
    return {
        "value": 1.0 / t_iter, "unit": "LM iters/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"one FP64 LM iteration of cluster 0 at N={ob.N} (8N={8 * ob.N}): brute-force "
                   f"normal equations over {vis} visibilities, LAPACK Cholesky solve, trial cost; "
                   f"{t_iter:.1f} s"),
        "predict_gvis_per_s": vis / t_pred / 1e9,
        "predict_sample": f"predict of cluster 0 ({ob.cluster_offset[1]} sources): {t_pred:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU layout is "
              "designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1910_13908_amd import synth, ddcal as dd

    if args.mode == "serve":
        res = serve_measure(args.requests, args.slots, args.seed, args.precision)
        c = res["closed_loop"]
        print(json.dumps({"metric": "served solves/s", "value": c["solves_per_s"], "unit": "solves/s",
                          "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "serve": res}),
              flush=True)
        return
    if args.mode == "scan":
        print(json.dumps({"metric": "calibration runtime scan", "data": "synthetic",
                          "scan": scan_measure(args.seed)}), flush=True)
        return
    if args.mode == "copy":
        print(json.dumps({"metric": "device copy", "copy": copy_measure()}), flush=True)
        return
    if args.mode == "predict":
        print(json.dumps({"metric": "predict", "predict": predict_measure(args.config, args.precision,
                                                                           seed=args.seed)}), flush=True)
        return
    if args.mode == "lbfgs":
        print(json.dumps({"metric": "L-BFGS vs LM", "lbfgs": lbfgs_measure(args.seed)}), flush=True)
        return

    cfg = synth.CONFIGS[args.config]
    prec = dd.MIXED if args.precision == "mixed" else dd.FP64
    dt = torch.float32 if prec == dd.MIXED else torch.float64
    ob = synth.make_obs(cfg, seed=args.seed)
    ctx = dd.Context(0)
    obs = dd.device_obs(ob)
    sky = dd.device_sky(ob)
    K, N = ob.K, ob.N

    def make_vis(p, dtype):
        noise = torch.as_tensor(dd.planes(ob.noise), dtype=dtype, device="cuda").contiguous()
        coh = ctx.predict(obs, sky, p)
        Jt = torch.as_tensor(dd.jones_real(ob.jones_true), device="cuda").contiguous()
        V = torch.empty_like(noise)
        ctx.add_model(obs, K, noise, coh, Jt, 1.0, p, V)
        del coh, noise
        torch.cuda.synchronize()
        return V

    V = make_vis(prec, dt)
    J0 = torch.as_tensor(dd.jones_real(synth.identity_jones(K, N)), device="cuda").contiguous()
    J = J0.clone()
    lm = dd.default_lm_opts(n_iter=cfg.n_lm, precision=prec)
    n_lm_per_step = cfg.n_sweeps * K * cfg.n_lm

    def step(want_info=False):
        J.copy_(J0)
        return ctx.calibrate(obs, sky, V, J, cfg.n_sweeps, lm, want_info=want_info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the timed steps bracket only the kernels reported from them (the factorisation for the
    # roofline, the predict): every event pair adds a stream marker that waits for its launch
    ctx.enable_timing(True, timers=[dd.TIMER_CHOLESKY, dd.TIMER_PREDICT])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    _progress(f"{args.steps} timed steps: {elapsed:.1f} s")
    timer_names = ["cholesky", "predict", "build", "trsv", "trial", "model", "refine", "adjoint"]
    timers = {name: ctx.timing(i) for i, name in enumerate(timer_names)}
    # one more step with every kernel class timed: the per-kernel breakdown, and the LM info
    ctx.enable_timing(True)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    infos = step(want_info=True)
    torch.cuda.synchronize()
    elapsed_b = time.perf_counter() - tb0
    breakdown = {name: ctx.timing(i) for i, name in enumerate(timer_names)}
    ctx.enable_timing(False)
    final_cost = infos[-1][-1].cost if infos else None   # residual cost after the last visit
    visits = [i for row in (infos or []) for i in row]
    lm_stats = {
        "accepted": int(sum(i.n_accept for i in visits)),
        "rejected": int(sum(i.n_reject for i in visits)),
        "failed_factorisations": int(sum(i.n_notpd for i in visits)),
        "max_refinement_steps": int(max((i.max_refine for i in visits), default=0)),
        "note": "over the 600 LM iterations of the step that collects the kernel breakdown; "
                "refinement steps are the FP64 corrections of one iteration (at most refine_max)",
    }

    ms_per_step = 1e3 * elapsed / args.steps
    value = n_lm_per_step * args.steps / elapsed
    n_ch, ms_ch, fl_ch = timers["cholesky"]
    peak = PEAK["fp32_mfma_tflops"] if prec == dd.MIXED else PEAK["fp64_mfma_tflops"]
    achieved = fl_ch / (ms_ch * 1e-3) / 1e12 if ms_ch > 0 else 0.0
    n_pr, ms_pr, terms = timers["predict"]
    vis_per_predict = K * ob.B * ob.T * ob.F
    gvis = (n_pr * vis_per_predict) / (ms_pr * 1e-3) / 1e9 if ms_pr > 0 else 0.0
    kernel_ms = {k: {"launches": v[0], "avg_us": 1e3 * v[1] / max(v[0], 1),
                     "share_of_step": v[1] / (1e3 * elapsed_b) if elapsed_b > 0 else 0.0}
                 for k, v in breakdown.items()}
    n_tr, ms_tr, by_tr = breakdown["trial"]

    out = {
        "metric": "LM iters/s", "value": value, "unit": "LM iters/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if prec == dd.MIXED else "f64",
        "data": "synthetic (seeded generator; the paper's data sets are not available)",
        "config": {"workload": f"{args.config}: N={N} stations, B={ob.B} baselines, K={K} clusters x "
                               f"{cfg.sources_per_cluster} sources, T={ob.T}, F={ob.F}, "
                               f"{cfg.n_sweeps} SAGE sweeps x {cfg.n_lm} LM iterations, "
                               f"{'mixed' if prec == dd.MIXED else 'fp64'} precision",
                   "n_stations": N, "n_clusters": K, "lm_iters_per_step": n_lm_per_step,
                   "precision": args.precision},
        "roofline": {"bound": "mfma", "kernel": "k_cholesky", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None,
                     "traffic_note": "HBM counters could not be collected on this kernel (the "
                                     "profiler process dies at the next launch); see "
                                     "roofline_hbm and profiles/ for measured traffic",
                     "per_launch": f"(8N)^3/3 = {(8 * N) ** 3 / 3:.3e} flop per factorisation, "
                                   f"avg {1e3 * ms_ch / max(n_ch, 1):.1f} us over {n_ch} launches"},
        "predict_gvis_per_s": gvis,
        "predict_gterms_per_s": terms / (ms_pr * 1e-3) / 1e9 if ms_pr > 0 else 0.0,
        "roofline_predict": (_predict_roofline(terms / (ms_pr * 1e-3) / 1e9)
                             if ms_pr > 0 and prec == dd.MIXED else None),
        # the trial cost runs in every LM iteration (the build is skipped after a rejection,
        # so its average over launches would not be a bandwidth)
        "roofline_hbm": _hbm_roofline("k_trial_cost", n_tr, ms_tr, by_tr),
        "kernels": kernel_ms,
        "kernels_note": "per-kernel HIP-event times from one extra step with every kernel class "
                        "timed (the timed steps time only the factorisation and the predict)",
        "final_total_cost": final_cost,
        "lm": lm_stats,
    }

    # station-factorised predict of the same sky (same coherencies; reported beside the
    # direct predict, which the calibration step uses)
    su, sv, sw = dd.device_station_uvw(ob)
    coh_f = ctx.predict_factored(obs, su, sv, sw, sky, prec)
    torch.cuda.synchronize()
    del coh_f
    ctx.enable_timing(True)
    for _ in range(3):
        coh_f = ctx.predict_factored(obs, su, sv, sw, sky, prec)
        del coh_f
    torch.cuda.synchronize()
    n_pf, ms_pf, vis_pf = ctx.timing(dd.TIMER_PREDICT_FACTORED)
    ctx.enable_timing(False)
    out["predict_factored_gvis_per_s"] = vis_pf / (ms_pf * 1e-3) / 1e9 if ms_pf > 0 else 0.0
    out["predict_factored_us"] = 1e3 * ms_pf / max(n_pf, 1)
    torch.cuda.empty_cache()

    # the residual kernel on its own (ddc_residual: R = V - sum_k J_k C_k J_k^H over all K
    # clusters at the calibrated Jones, with the cost): its algorithmic bytes are the data,
    # K coherency planes and the residual written, (16 + 8K) elements per visibility; the
    # timed region also holds the small launch that lays the Jones out as component planes
    coh = ctx.predict(obs, sky, prec)
    Rres = torch.empty_like(V)
    ctx.residual(obs, K, V, coh, J, prec, res=Rres)
    torch.cuda.synchronize()
    ctx.enable_timing(True, timers=[dd.TIMER_MODEL])
    for _ in range(5):
        ctx.residual(obs, K, V, coh, J, prec, res=Rres, want_cost=False)
    n_rs, ms_rs, _ = ctx.timing(dd.TIMER_MODEL)
    ctx.enable_timing(False)
    es = 4 if prec == dd.MIXED else 8
    res_bytes = (16 + 8 * K) * es * ob.B * ob.T * ob.F
    out["roofline_residual"] = {
        "bound": "hbm", "kernel": "k_jones_planes + k_add_model (ddc_residual, all clusters)", "unit": "GB/s",
        "peak": PEAK["hbm_gbs"], "achieved": n_rs * res_bytes / (ms_rs * 1e-3) / 1e9,
        "frac": n_rs * res_bytes / (ms_rs * 1e-3) / 1e9 / PEAK["hbm_gbs"],
        "avg_us": 1e3 * ms_rs / max(n_rs, 1), "traffic": None,
        "per_launch": f"(16 + 8K) x {es} B x {ob.B * ob.T * ob.F} visibilities = {res_bytes / 1e6:.1f} MB"}
    del coh, Rres
    torch.cuda.empty_cache()

    if prec == dd.MIXED and not args.no_fp64_compare:
        V = None
        torch.cuda.empty_cache()
        V64 = make_vis(dd.FP64, torch.float64)
        J64 = J0.clone()
        lm64 = dd.default_lm_opts(n_iter=cfg.n_lm, precision=dd.FP64)
        ctx.calibrate(obs, sky, V64, J64, cfg.n_sweeps, lm64, want_info=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J64.copy_(J0)
        ctx.calibrate(obs, sky, V64, J64, cfg.n_sweeps, lm64, want_info=False)
        torch.cuda.synchronize()
        out["fp64_path_lm_iters_per_s"] = n_lm_per_step / (time.perf_counter() - t0)
        V64 = None
        _progress("FP64 path timed")

    if not args.no_serve:
        # the served stream of calibration requests, in both precisions: solves/s at
        # saturation (all requests at t = 0) and p50/p99 latency under Poisson arrivals at
        # 0.5x and 0.9x that rate
        V = None
        torch.cuda.empty_cache()
        served = {}
        for p in ("mixed", "fp64"):
            served[p] = serve_measure(args.requests, args.slots, args.seed, p)
            torch.cuda.empty_cache()
        served["mixed_over_fp64_solves_per_s"] = (served["mixed"]["closed_loop"]["solves_per_s"] /
                                                  served["fp64"]["closed_loop"]["solves_per_s"])
        out["served"] = served

    if not args.no_cpu_baseline:
        _progress("oracle on the host")
        out["cpu_baseline"] = cpu_baseline(cfg, args.seed)

    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
