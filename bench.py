#!/usr/bin/env python3
"""Throughput of the Artificial Retina hot path on one MI355X.

One step = Algorithm 1 over the whole batch through the C-ABI: hit staging,
seeds, truncated-Newton ascents with sigma continuation, FP64 polish,
clustering and selection.  Two seedings of the same batch are timed:

  lattice  retina_find_tracks with the workload's uniform (tx, ty) lattice
  learned  retina_find_tracks_learned: the trained proposer network picks the
           seeds on the device (lattice fallback per event), then the same
           ascent, polish and merge

`value` is the learned path's events/s.  The lattice baseline is the fastest
lattice of the workload's sweep (`lattice_sweep`) that reaches >= 95% track
efficiency; every swept size is reported, with the qualities against
generator truth and the speedup.  The standalone response kernel
(retina_response: R only and R + gradient + Hessian) is timed on the
workload's shapes for the response evals/s and %FP32 peak figures.
Inputs are resident in device memory before the timed regions; each timed
region brackets exactly --steps calls with device synchronisation.  `value`
and `ms_per_step` come from the library's default mode, each call replaying
its captured hipGraph.  A second timed region runs the same steps with the
library's HIP-event profiling on (eager launches: events cannot sit inside a
graph), which gives the per-kernel times on the library's stream and the
dominant kernel's (the ascent's) average duration for the roofline
(`ms_per_step_profiled`).
The FP64 CPU oracle is timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector peak: 256 CU x 4 SIMD x 32 lanes x 2.4 GHz x 2 (FMA)
PEAK_BF16_TFLOPS = 2500.0      # MI355X dense BF16 MFMA
# algorithmic FP32 flops (FMA = 2, exp2 not counted) per hit-candidate pair,
# meas_dim 2, per-plane factored sums
FLOP_RGH_PAIR = 21
FLOP_R_PAIR = 11
FLOP_POLISH_PAIR = 25          # RGH pair with the two-float residual (4 more)
FLOP_FOLD = 26                 # per (candidate, plane) per derivative pass
# proposer network: 2 x 16384 pixels x (9 x (2x64 + 64x128 + 128x96 + 96x1)) per event
FLOP_NET_EVENT = 2 * 16384 * 9 * (2 * 64 + 64 * 128 + 128 * 96 + 96 * 1)
# HBM bytes per launch of the ascent kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (profiles/k_ascent_c3_learned.md), each scaled
# by the counter's reading for a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0).  Valid only for the kernel source they were taken with (hash of
# csrc/hot.hip + csrc/rt_internal.h); reported as null otherwise.
MEASURED_TRAFFIC = {("c3", "learned"): {"bytes": 154.6e6, "fetch": 146.8e6, "write": 7.8e6,
                                         "source_sha256_16": "685acee4fc24cad6"}}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("hot.hip", "rt_internal.h"):
        with open(os.path.join(ROOT, "paper_1709_08610_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    m = MEASURED_TRAFFIC.get((workload, "learned"))
    if m is None or m["source_sha256_16"] != kernel_source_hash():
        return None
    return m["bytes"]


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def algorithmic_flops(P, ev_hits, ev_seeds, nreval_per_event, n_planes):
    n_steps = len(P["sigma"]) + P["n_final_steps"]
    fl = 0.0
    pairs = 0.0
    for nh, ns, nr in zip(ev_hits, ev_seeds, nreval_per_event):
        fl += nh * ns * (n_steps * FLOP_RGH_PAIR + P["n_polish"] * FLOP_POLISH_PAIR)
        fl += nh * nr * FLOP_R_PAIR
        fl += ns * n_planes * FLOP_FOLD * (n_steps + P["n_polish"])
        pairs += nh * (ns * (n_steps + P["n_polish"]) + nr)
    return fl, pairs


def _sample_size(run_one, target_s, cap):
    """Events for a CPU sample of about target_s seconds (one event timed first)."""
    t0 = time.perf_counter()
    run_one()
    dt = max(time.perf_counter() - t0, 1e-3)
    return int(max(1, min(cap, target_s / dt)))


def cpu_baseline(cfg, P, target_s=12.0, cap=256):
    import oracle
    from paper_1709_08610_amd import events
    threads = os.cpu_count() or 1
    n_events = _sample_size(lambda: oracle.find_tracks(events.make_batch(cfg, 1), P, n_threads=threads),
                            target_s, cap)
    b = events.make_batch(cfg, n_events)
    t0 = time.perf_counter()
    ref = oracle.find_tracks(b, P, n_threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n_events / dt, unit="events/s", cores=threads, kind="oracle",
                sample="first %d of %d events of the %s workload, full method with the %dx%d lattice "
                       "(FP64, OpenMP over seeds), %.1f s"
                       % (n_events, cfg["n_events"], cfg["name"], P["lattice_n"][0], P["lattice_n"][1], dt)), ref


def cpu_baseline_learned(cfg, LS, model, target_s=12.0, cap=256):
    """The oracle's own learned path on the host cores: the FP64 network forward
    (numpy, BF16 at the device's storage points) and seed selection of
    oracle/proposer.py on the same weights, then oracle_find_tracks on those
    seeds."""
    import numpy as np
    import oracle
    from oracle import proposer as op
    from paper_1709_08610_amd import events
    layers = op.unpack_params(model.retina_model_get_params())
    lat = oracle.lattice(2, LS["params"])
    threads = os.cpu_count() or 1

    def run(b):
        seeds, off = [], [0]
        for e in range(b.n_events):
            ev = b.event(e)
            _, z = op.forward(op.bin_image(ev.x, ev.y, ev.plane, b.plane_z), layers)
            picks = op.seed_bins(z, LS["tau"], LS["k_max"], nms=LS["nms"])
            fb = not picks or z.max() < op.logit_threshold(LS["conf_min"])
            s = lat if fb else op.seeds_from_pixels(picks)
            seeds.append(s)
            off.append(off[-1] + len(s))
        return oracle.find_tracks(b, LS["params"], np.concatenate(seeds), np.array(off, np.int64),
                                  n_threads=threads)

    n_events = _sample_size(lambda: run(events.make_batch(cfg, 1)), target_s, cap)
    b = events.make_batch(cfg, n_events)
    t0 = time.perf_counter()
    ref = run(b)
    dt = time.perf_counter() - t0
    return dict(value=n_events / dt, unit="events/s", cores=threads, kind="oracle",
                sample="first %d of %d events of the %s workload, oracle proposer (numpy FP64 forward) + full "
                       "method on its seeds (FP64, OpenMP over seeds), %.1f s" % (n_events, cfg["n_events"],
                                                                               cfg["name"], dt)), ref


def fp32_vs_fp64(D, gpu_theta, gpu_R, gpu_toff, ref, d_merge, z0, z1):
    """The GPU's FP32 track sets against the FP64 oracle's on the oracle's
    sample events: tracks matched within d_merge, the largest parameter error
    |dp| / max(|p|, s_p) (s_p = 0.05 mm for offsets, 0.01 for slopes) and the
    largest |dR| / R over the matched tracks, and the tracks on one side only."""
    import numpy as np
    from oracle.evaluate import match_tracks
    s_p = np.array([0.05, 0.05, 0.01, 0.01]) if D == 2 else np.array([0.01, 0.01])
    rto = ref["track_offsets"]
    n_ev = len(rto) - 1
    matched = only_gpu = only_ref = 0
    dth = dR = 0.0
    for e in range(n_ev):
        g = np.asarray(gpu_theta[gpu_toff[e]:gpu_toff[e + 1]], np.float64)[:, :2 * D]
        gR = np.asarray(gpu_R[gpu_toff[e]:gpu_toff[e + 1]], np.float64)
        r = np.asarray(ref["theta"][rto[e]:rto[e + 1]], np.float64)
        rR = np.asarray(ref["R"][rto[e]:rto[e + 1]], np.float64)
        f2t, t2f, _ = match_tracks(D, g, r, d_merge, z0, z1)
        m = t2f >= 0
        matched += int(m.sum())
        only_ref += int((~m).sum())
        only_gpu += int((f2t < 0).sum())
        if m.any():
            dth = max(dth, float((np.abs(g[t2f[m]] - r[m]) / np.maximum(np.abs(r[m]), s_p)).max()))
            dR = max(dR, float((np.abs(gR[t2f[m]] - rR[m]) / np.abs(rR[m])).max()))
    return dict(events=n_ev, matched_tracks=matched, gpu_only=only_gpu, oracle_only=only_ref,
                max_rel_dtheta=dth, max_rel_dR=dR)


def response_throughput(ctx, retina, cfg, b, torch, np):
    """retina_response alone (R only, and R + gradient + Hessian) on the
    workload's events with its lattice as the candidate lines: pair
    evaluations per second and the algorithmic FP32 rate."""
    P = cfg["params"]
    D = b.meas_dim
    n0, n1 = P["lattice_n"]
    i0, i1 = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    v0 = (P["lattice_lo"][0] + (i0.ravel() + 0.5) * (P["lattice_hi"][0] - P["lattice_lo"][0]) / n0)
    v1 = (P["lattice_lo"][1] + (i1.ravel() + 0.5) * (P["lattice_hi"][1] - P["lattice_lo"][1]) / n1)
    th = np.zeros((n0 * n1, 2 * D), np.float32)
    if D == 2:
        th[:, 2], th[:, 3] = v0, v1
    else:
        th[:, 0], th[:, 1] = v1, v0
    dev = torch.device("cuda:0")
    E = b.n_events
    theta = torch.from_numpy(np.tile(th, (E, 1))).to(dev)
    toff = torch.from_numpy(np.arange(E + 1, dtype=np.int64) * len(th)).to(dev)
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    hits = (tin(b.event_offsets), tin(b.x), tin(b.y) if D == 2 else None, tin(b.plane))
    pairs = float(len(th)) * float(b.x.shape[0])
    out = {"candidates_per_event": len(th), "events": E, "hits": int(b.x.shape[0])}
    for name, want, fl in (("R", retina.WANT_R, FLOP_R_PAIR if D == 2 else 6),
                           ("RGH", retina.WANT_R | retina.WANT_GRAD | retina.WANT_HESS, FLOP_RGH_PAIR if D == 2 else 10)):
        f = lambda: ctx.retina_response(D, b.plane_z, *hits, theta, toff, sigma=P["sigma_final"], want=want)
        f()
        torch.cuda.synchronize()
        ctx.retina_set_profiling(True)
        ctx.retina_profile_reset()
        for _ in range(3):
            f()
        torch.cuda.synchronize()
        pr = ctx.retina_get_profile()
        ctx.retina_set_profiling(False)
        ms = pr["ms_hot"] / max(pr["calls"], 1)
        rate = pairs / (ms * 1e-3)
        out[name] = {"ms": ms, "pair_evals_per_s": rate, "tflops": rate * fl / 1e12,
                     "frac_fp32_peak": rate * fl / 1e12 / PEAK_FP32_TFLOPS}
        log("response %s: %.3f ms, %.3g pair evals/s, %.1f%% of FP32 peak" % (name, ms, rate,
                                                                              100 * rate * fl / 1e12 / PEAK_FP32_TFLOPS))
    return out


def timed(ctx, step, steps):
    """Run `steps` calls with HIP-event profiling on; then the same through the
    graph path without events.  Returns (s per step, profile per call, graph s per step)."""
    import torch
    ctx.retina_set_profiling(True)
    ctx.retina_profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    prof = ctx.retina_get_profile()
    ctx.retina_set_profiling(False)
    n = max(prof["calls"], 1)
    prof = {k: (v / n if k != "calls" else v) for k, v in prof.items()}
    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return dt, prof, (time.perf_counter() - t0) / steps


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="approximate length of each CPU oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-budget", action="store_true",
                    help="skip the grid-search vs multi-start comparison (c7 track-count scan)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one plain device-to-device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one device per context and "
              "has no multi-GPU launcher (events would shard across GPUs with no exchange). "
              "Use --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1709_08610_amd import events, learned, metrics, retina

    cfg = events.load_config(args.workload)
    P = cfg["params"]
    LS = learned.settings(cfg)
    PL = LS["params"]
    log("generating %s (%d events)" % (cfg["name"], cfg["n_events"]))
    b = events.make_batch(cfg)
    D = b.meas_dim
    E = b.n_events
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    off_d, x_d, y_d, pl_d = tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane)
    ctx = retina.Context(0)
    model = ctx.retina_model_load(LS["model"])
    torch.cuda.synchronize()
    z0, z1 = float(b.plane_z.min()), float(b.plane_z.max())
    ev_hits = np.diff(b.event_offsets)

    def quality(tracks_theta, toff):
        return metrics.batch_quality(D, tracks_theta, toff, b.truth, b.truth_nhits, cfg["match_tol"], z0, z1)

    def lattice_step(want_seeds=False):
        return ctx.retina_find_tracks(D, b.plane_z, off_d, x_d, y_d, pl_d, P, want_seeds=want_seeds)

    def learned_step():
        return ctx.retina_find_tracks_learned(model, b.plane_z, off_d, x_d, y_d, pl_d, PL, LS["k_max"],
                                              LS["tau"], LS["conf_min"], nms=LS["nms"])

    # ---- lattice sweep: the fastest lattice reaching the efficiency bar is the baseline
    sweep = []
    for n in cfg.get("lattice_sweep", [P["lattice_n"][0]]):
        Pn = dict(P, lattice_n=[n, n])
        f = lambda: ctx.retina_find_tracks(D, b.plane_z, off_d, x_d, y_d, pl_d, Pn)
        r = f()
        torch.cuda.synchronize()
        qn = quality(retina.tracks_from_device(r)["theta"][:, :2 * D], r["track_offsets"].cpu().numpy())
        del r
        t0 = time.perf_counter()
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        tn = (time.perf_counter() - t0) / 2
        sweep.append(dict(lattice_n=n, ms_per_step=tn * 1e3, events_per_s=E / tn,
                          efficiency=round(qn["efficiency"], 5), fake_rate=round(qn["fake_rate"], 5)))
        log("lattice %dx%d: %.2f ms, efficiency %.4f fake %.4f" % (n, n, tn * 1e3, qn["efficiency"], qn["fake_rate"]))
    ok = [r for r in sweep if r["efficiency"] >= 0.95]
    best = min(ok, key=lambda r: r["ms_per_step"]) if ok else max(sweep, key=lambda r: r["efficiency"])
    P = dict(P, lattice_n=[best["lattice_n"], best["lattice_n"]])
    log("lattice baseline: %dx%d" % (best["lattice_n"], best["lattice_n"]))

    # ---- quality + work accounting (untimed)
    log("lattice: quality + work accounting run")
    res = lattice_step(want_seeds=True)
    torch.cuda.synchronize()
    tl = retina.tracks_from_device(res)
    toff_lat = res["track_offsets"].cpu().numpy()
    q_lat = quality(tl["theta"][:, :2 * D], toff_lat)
    ns = P["lattice_n"][0] * P["lattice_n"][1]
    nre = res["seed_nreval"].cpu().numpy().astype(np.int64).reshape(E, ns).sum(axis=1)
    fl_lat, pairs_lat = algorithmic_flops(P, ev_hits, [ns] * E, nre, len(b.plane_z))
    del res
    log("lattice efficiency %.4f fake %.4f" % (q_lat["efficiency"], q_lat["fake_rate"]))

    log("learned: quality + work accounting run (proposer seeds -> explicit-seed ascent)")
    prop = ctx.retina_propose_seeds(model, b.plane_z, off_d, x_d, y_d, pl_d, LS["k_max"], LS["tau"],
                                    LS["conf_min"], PL, nms=LS["nms"])
    so = prop["seed_offsets"]
    res = ctx.retina_find_tracks(D, b.plane_z, off_d, x_d, y_d, pl_d, PL, seeds=prop["seeds"].contiguous(),
                                 seed_offsets=so, want_seeds=True)
    torch.cuda.synchronize()
    so_h = so.cpu().numpy()
    seeds_ev = np.diff(so_h)
    nre_s = res["seed_nreval"].cpu().numpy().astype(np.int64)
    cs = np.concatenate([[0], np.cumsum(nre_s)])
    nre_ev = cs[so_h[1:]] - cs[so_h[:-1]]
    fl_lrn, pairs_lrn = algorithmic_flops(PL, ev_hits, seeds_ev, nre_ev, len(b.plane_z))
    res2 = learned_step()
    torch.cuda.synchronize()
    tr = retina.tracks_from_device(res2)
    toff_lrn = res2["track_offsets"].cpu().numpy()
    q_lrn = quality(tr["theta"][:, :2 * D], toff_lrn)
    fb_rate = float(((res2["event_flags"] >> 4) & 1).float().mean().item())
    assert np.array_equal(res["track_offsets"].cpu().numpy(), res2["track_offsets"].cpu().numpy())
    del res, res2, prop
    log("learned efficiency %.4f fake %.4f, %.1f seeds/event, fallback %.3f" % (
        q_lrn["efficiency"], q_lrn["fake_rate"], seeds_ev.mean(), fb_rate))

    for i in range(args.warmup):
        lattice_step()
        learned_step()
        log("warmup %d done" % (i + 1))
    dt_lat, prof_lat, g_lat = timed(ctx, lattice_step, args.steps)
    log("lattice: %.2f ms/step (profiled, eager: %.2f), ascent %.2f ms" % (g_lat * 1e3, dt_lat * 1e3, prof_lat["ms_hot"]))
    dt_lrn, prof_lrn, g_lrn = timed(ctx, learned_step, args.steps)
    log("learned: %.2f ms/step (profiled, eager: %.2f), proposer %.2f ms, ascent %.2f ms" % (
        g_lrn * 1e3, dt_lrn * 1e3, prof_lrn["ms_propose"], prof_lrn["ms_hot"]))

    # ---- locality-pruned passes (prune_u = 30: each skipped term < 1e-13), both
    # seedings: the lattice sweep again (pruning favours compact waves, so the
    # fastest lattice reaching the bar may change) and the learned seeds
    PU = 30.0
    sweep_p = []
    for n in cfg.get("lattice_sweep", [P["lattice_n"][0]]):
        Pn = dict(P, lattice_n=[n, n], prune_u=PU)
        f = lambda: ctx.retina_find_tracks(D, b.plane_z, off_d, x_d, y_d, pl_d, Pn)
        r = f()
        torch.cuda.synchronize()
        qn = quality(retina.tracks_from_device(r)["theta"][:, :2 * D], r["track_offsets"].cpu().numpy())
        del r
        t0 = time.perf_counter()
        for _ in range(2):
            f()
        torch.cuda.synchronize()
        tn = (time.perf_counter() - t0) / 2
        sweep_p.append(dict(lattice_n=n, ms_per_step=tn * 1e3, events_per_s=E / tn,
                            efficiency=round(qn["efficiency"], 5), fake_rate=round(qn["fake_rate"], 5)))
        log("pruned lattice %dx%d: %.2f ms, efficiency %.4f" % (n, n, tn * 1e3, qn["efficiency"]))
    ok_p = [r for r in sweep_p if r["efficiency"] >= 0.95]
    best_p = min(ok_p, key=lambda r: r["ms_per_step"]) if ok_p else max(sweep_p, key=lambda r: r["efficiency"])
    PLp = dict(PL, prune_u=PU)

    def learned_pruned():
        return ctx.retina_find_tracks_learned(model, b.plane_z, off_d, x_d, y_d, pl_d, PLp, LS["k_max"],
                                              LS["tau"], LS["conf_min"], nms=LS["nms"])
    r = learned_pruned()
    torch.cuda.synchronize()
    q_lp = quality(retina.tracks_from_device(r)["theta"][:, :2 * D], r["track_offsets"].cpu().numpy())
    del r
    dt_lp, prof_lp, g_lp = timed(ctx, learned_pruned, args.steps)
    log("pruned learned: %.2f ms/step, ascent %.2f ms, efficiency %.4f; pruned lattice %dx%d %.2f ms" % (
        g_lp * 1e3, prof_lp["ms_hot"], q_lp["efficiency"], best_p["lattice_n"], best_p["lattice_n"],
        best_p["ms_per_step"]))
    pruned = {"prune_u": PU, "lattice_sweep": sweep_p, "lattice_best": best_p,
              "learned": {"events_per_s": E / g_lp, "ms_per_step": g_lp * 1e3, "ms_per_step_profiled": dt_lp * 1e3, "ascent_ms": prof_lp["ms_hot"],
                          "efficiency": round(q_lp["efficiency"], 5), "fake_rate": round(q_lp["fake_rate"], 5)},
              "speedup_vs_lattice": best_p["ms_per_step"] / (g_lp * 1e3)}

    # end to end from host memory (hits H2D, tracks D2H included)
    hb = (b.event_offsets, b.x, b.y, b.plane)
    ctx.retina_find_tracks_learned(model, b.plane_z, *hb, PL, LS["k_max"], LS["tau"], LS["conf_min"], nms=LS["nms"])
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.retina_find_tracks_learned(model, b.plane_z, *hb, PL, LS["k_max"], LS["tau"], LS["conf_min"],
                                       nms=LS["nms"])
    ms_host = (time.perf_counter() - t0) / args.steps * 1e3
    log("learned, host memory end to end: %.2f ms/step" % ms_host)

    resp = response_throughput(ctx, retina, cfg, b, torch, np)
    # the other response shapes: one c2 event (4096 lattice lines x 5.6k hits,
    # occupancy-limited) and the c1 brute-force grid (400 x 400 lines x 130
    # hits, meas_dim 1)
    c2 = events.load_config("c2")
    resp_c2 = response_throughput(ctx, retina, c2, events.make_batch(c2, 1), torch, np)
    c1 = events.load_config("c1")
    c1g = dict(c1, params=dict(c1["params"], lattice_n=[400, 400]))
    resp_c1 = response_throughput(ctx, retina, c1g, events.make_batch(c1, 1), torch, np)

    # Section 3's comparison: multi-start at 1/3 and 1/10 of the grid search's
    # measured cost, efficiency against the number of tracks (Fig. 3)
    alpha = alpha_sv = upd = None
    if not args.no_budget:
        from paper_1709_08610_amd import budget
        alpha = budget.run(ctx, events.load_config("c7"), log=log)
        # the same on the paper's simplified VELO (tracks from the origin, prior-drawn seeds)
        alpha_sv = budget.run(ctx, events.load_config("c8"), log=log)
        # Section 3's choice of update rule: truncated Newton against the
        # normalised gradient and BFGS from the same seeds
        upd = {name: budget.compare_updates(ctx, events.load_config(name), log=log) for name in ("c7", "c8")}

    cpu = cpu_l = prec = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, %dx%d lattice)" % tuple(P["lattice_n"]))
        cpu, ref_lat = cpu_baseline(cfg, P, args.cpu_seconds)
        log("cpu baseline (oracle, learned seeds)")
        cpu_l, ref_lrn = cpu_baseline_learned(cfg, LS, model, args.cpu_seconds)
        # FP32 GPU against the FP64 oracle on the baseline's sample events
        prec = {"lattice": fp32_vs_fp64(D, tl["theta"], tl["R"], toff_lat, ref_lat, P["d_merge"], z0, z1),
                "learned": fp32_vs_fp64(D, tr["theta"], tr["R"], toff_lrn, ref_lrn, PL["d_merge"], z0, z1)}
        log("fp32 vs fp64 (oracle sample): %s" % prec)

    hot = prof_lrn["ms_hot"]
    achieved = fl_lrn / (hot * 1e-3) / 1e12
    net_tflops = FLOP_NET_EVENT * E / (prof_lrn["ms_propose"] * 1e-3) / 1e12
    rq = lambda q: {k: (round(v, 5) if isinstance(v, float) else v) for k, v in q.items()}
    kms = lambda p: {"stage": p["ms_stage"], "plan": p["ms_plan"], "ascent": p["ms_hot"], "merge": p["ms_merge"]}
    out = {
        "metric": "events/sec at >=95% track eff (learned vs lattice seeds); response evals/s, %FP32 peak",
        "value": E / g_lrn,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": g_lrn * 1e3,
        "ms_per_step_profiled": dt_lrn * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (cfg["name"], cfg["description"]), "events": E,
                   "hits": int(b.x.shape[0]),
                   "seeds": "learned: %s, k_max %d, tau %g, conf_min %g, nms %d; lattice %dx%d fallback"
                            % (os.path.basename(LS["model"]), LS["k_max"], LS["tau"], LS["conf_min"],
                               int(LS["nms"]), P["lattice_n"][0], P["lattice_n"][1]),
                   "parallelism": "single GPU"},
        "quality": rq(q_lrn),
        "learned": {"seeds_per_event": float(seeds_ev.mean()), "fallback_rate": fb_rate,
                    "kernel_ms": dict(kms(prof_lrn), proposer=prof_lrn["ms_propose"]),
                    "response_evals_per_s": pairs_lrn / (hot * 1e-3),
                    "proposer_net_tflops": net_tflops},
        "lattice": {"lattice_n": best["lattice_n"], "events_per_s": E / g_lat, "ms_per_step": g_lat * 1e3, "ms_per_step_profiled": dt_lat * 1e3,
                    "quality": rq(q_lat), "kernel_ms": kms(prof_lat),
                    "response_evals_per_s": pairs_lat / (prof_lat["ms_hot"] * 1e-3),
                    "ascent_tflops": fl_lat / (prof_lat["ms_hot"] * 1e-3) / 1e12,
                    "pairs_per_launch": {"algorithmic": pairs_lat, "executed": prof_lat["exec_pairs"],
                                         "executed_line_search": prof_lat["exec_rpairs"]}},
        "lattice_sweep": sweep,
        "speedup_vs_lattice": g_lat / g_lrn,
        "pruned": pruned,
        "end_to_end_host_ms_per_step": ms_host,
        "response": resp,
        "response_c2_event": resp_c2,
        "response_c1_grid": resp_c1,
        "response_evals_per_s": pairs_lrn / (hot * 1e-3),
        "pairs_per_launch": {"algorithmic": pairs_lrn, "executed": prof_lrn["exec_pairs"],
                             "executed_line_search": prof_lrn["exec_rpairs"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(cfg["name"]), "traffic_unit": "bytes per launch", "kernel": "k_ascent (persistent truncated-Newton ascent, learned seeds)",
                     "flops_per_launch": fl_lrn},
        "roofline_proposer": {"bound": "mfma", "achieved": net_tflops, "peak": PEAK_BF16_TFLOPS,
                              "unit": "TFLOP/s", "frac": net_tflops / PEAK_BF16_TFLOPS,
                              "kernel": "binning + four conv layers + seed selection (network flops only)",
                              "flops_per_launch": FLOP_NET_EVENT * E},
        "alpha_budget": alpha,
        "alpha_budget_svelo": alpha_sv,
        "update_rules": upd,
        "cpu_baseline": cpu,
        "cpu_baseline_learned": cpu_l,
        "fp32_vs_fp64": prec,
    }
    print(json.dumps(out))
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))


if __name__ == "__main__":
    main()
