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
lattice of the workload's sweep that reaches >= 95% track efficiency.

Timing.  Inputs are resident in device memory before any timed region.  After
--warmup untimed steps, exactly --steps calls are timed in the library's
default mode (each call replays its captured hipGraph): the wall clock
brackets the K calls with device synchronisation on both sides
(`ms_per_step`, `value`), and HIP events recorded on the library's stream
around each call give the per-step device time (`ms_per_step_events_median`,
the median of the K steps).  A further profiled run (eager launches with the
library's per-kernel HIP events on its stream) gives the dominant kernel's
(the ascent's) average duration for the roofline.

Cost model of Section 3, measured: T0 = time of R at one line over an event's
hits (the standalone response kernel, R only, the workload's batch and
lattice lines), C = time of R + gradient + Hessian / T0, and C0 = time of
one optimisation step per seed / T0, where a seed's steps are its sigma
stages, final steps and FP64 polish iterations (lattice ascent).

The FP64 CPU oracle is timed on a bounded sample of the same workload
(`cpu_baseline`, the learned path; `cpu_baseline_lattice`), and the GPU's
FP32 track sets are compared with the oracle's on that sample
(`fp32_vs_fp64`).

Output: the LAST stdout line is one compact JSON object (the headline).  The
full report (lattice sweep, per-kernel times, response shapes, optional
studies) goes to stderr as one line starting with "[bench] detail " and, with
--detail-out PATH, to that file.  --studies adds the locality-pruned
comparison, Section 3's alpha-budget scans and the update-rule comparison.
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
# meas_dim 2, per-plane factored sums.  The polish evaluates the same
# R + gradient + Hessian sums (its two-float residual is implementation work,
# not counted).
FLOP_RGH_PAIR = 21
FLOP_R_PAIR = 11
FLOP_POLISH_PAIR = FLOP_RGH_PAIR
FLOP_FOLD = 26                 # per (candidate, plane) per derivative pass
# proposer network: 2 x 16384 pixels x (9 x (2x64 + 64x128 + 128x96 + 96x1)) per event
FLOP_NET_EVENT = 2 * 16384 * 9 * (2 * 64 + 64 * 128 + 128 * 96 + 96 * 1)
# HBM bytes per launch of the ascent kernel from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE runs of this script (profiles/k_ascent_c3_learned.md), each scaled
# by the counter's reading for a 1 GiB device copy (FETCH_SIZE x 2.0, WRITE_SIZE
# x 1.0).  Valid only for the kernel source they were taken with (hash of
# csrc/hot.hip + csrc/rt_internal.h + csrc/stage.hip, the kernel and the plan
# that orders its work); reported as null otherwise.
MEASURED_TRAFFIC = {("c3", "learned"): {"bytes": 80.82e6, "fetch": 72.24e6, "write": 8.58e6,
                                         "source_sha256_16": "aa016066931a8bce"}}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("hot.hip", "rt_internal.h", "stage.hip"):
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
    """FP32 flops of one ascent launch by the method's own work: per seed and
    event hit, one R + gradient + Hessian pair per step and per polish
    iteration, one R pair per line-search evaluation, and one fold per
    (seed, plane) of every derivative pass."""
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
    """Events for a CPU sample of about target_s seconds (one event timed
    first); a negative target_s fixes the sample at -target_s events."""
    if target_s < 0:
        return int(-target_s)
    t0 = time.perf_counter()
    run_one()
    dt = max(time.perf_counter() - t0, 1e-3)
    return int(max(1, min(cap, target_s / dt)))


def _timed_in_parts(cfg, n_events, run, label, parts=8):
    """run(batch) over the first n_events events of cfg, as up to `parts`
    consecutive sub-batches (generated before the clock starts; one progress
    line per sub-batch); returns the summed run time and the joined tracks
    (theta, R, track_offsets)."""
    import numpy as np
    from paper_1709_08610_amd import events
    k = -(-n_events // parts)
    subs = [events.make_batch(cfg, min(k, n_events - s), start=s) for s in range(0, n_events, k)]
    theta, R, off, dt = [], [], [np.zeros(1, np.int64)], 0.0
    for i, sb in enumerate(subs):
        t0 = time.perf_counter()
        r = run(sb)
        dt += time.perf_counter() - t0
        theta.append(r["theta"])
        R.append(r["R"])
        off.append(off[-1][-1] + r["track_offsets"][1:])
        log("%s: %d of %d sub-batches, %.1f s" % (label, i + 1, len(subs), dt))
    return dt, dict(theta=np.concatenate(theta), R=np.concatenate(R), track_offsets=np.concatenate(off))


def cpu_baseline(cfg, P, target_s=12.0, cap=256):
    import oracle
    from paper_1709_08610_amd import events
    threads = os.cpu_count() or 1
    n_events = _sample_size(lambda: oracle.find_tracks(events.make_batch(cfg, 1), P, n_threads=threads),
                            target_s, cap)
    dt, ref = _timed_in_parts(cfg, n_events, lambda b: oracle.find_tracks(b, P, n_threads=threads),
                              "cpu lattice")
    return dict(value=n_events / dt, unit="events/s", cores=threads, kind="oracle",
                sample="first %d of %d %s events, FP64 oracle, %dx%d lattice, %.1f s"
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
    dt, ref = _timed_in_parts(cfg, n_events, run, "cpu learned")
    return dict(value=n_events / dt, unit="events/s", cores=threads, kind="oracle",
                sample="first %d of %d %s events, FP64 oracle proposer (numpy) + FP64 method on its "
                       "seeds, %.1f s" % (n_events, cfg["n_events"], cfg["name"], dt)), ref


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


def response_throughput(ctx, retina, cfg, b, torch, np, reps=3):
    """retina_response alone (R only, and R + gradient + Hessian) on the
    workload's events with its lattice as the candidate lines: pair
    evaluations per second, the algorithmic FP32 rate, and the kernel time
    per candidate line (T0 for R only)."""
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
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        pr = ctx.retina_get_profile()
        ctx.retina_set_profiling(False)
        ms = pr["ms_hot"] / max(pr["calls"], 1)
        rate = pairs / (ms * 1e-3)
        out[name] = {"ms": ms, "ns_per_candidate": ms * 1e6 / (len(th) * E), "pair_evals_per_s": rate,
                     "tflops": rate * fl / 1e12, "frac_fp32_peak": rate * fl / 1e12 / PEAK_FP32_TFLOPS}
        log("response %s (%s): %.3f ms, %.3g pair evals/s, %.1f%% of FP32 peak" % (
            name, cfg["name"], ms, rate, 100 * rate * fl / 1e12 / PEAK_FP32_TFLOPS))
    return out


def timed_graph(step, steps):
    """`steps` calls in the library's default mode (graph replay): wall-clock
    mean over the bracketed region and the median of per-call HIP-event
    times on the library's stream (the binding runs the library on torch's
    current stream)."""
    import numpy as np
    import torch
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        step()
        b.record(st)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ev_ms = [a.elapsed_time(b) for a, b in evs]
    return wall, float(np.median(ev_ms)), ev_ms


def profiled(ctx, step, steps):
    """`steps` eager calls with the library's per-kernel HIP events on its
    stream; returns the per-call average of each profile field."""
    import torch
    ctx.retina_set_profiling(True)
    ctx.retina_profile_reset()
    torch.cuda.synchronize()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    prof = ctx.retina_get_profile()
    ctx.retina_set_profiling(False)
    n = max(prof["calls"], 1)
    return {k: (v / n if k != "calls" else v) for k, v in prof.items()}


def shape_sweep(ctx, D, learned_step, lattice_step, steps):
    """Ascent launch time (library HIP events, mean of `steps` eager calls) of
    the learned step over the sparse shape's hit tiles (one candidate per lane,
    several lanes per seed) and of the lattice step over the dense shape's
    tiles and candidates per lane; the tunings in force are restored."""
    out = {"sparse": [], "dense": []}
    for kernel, key, step, shapes in ((2, "sparse", learned_step, [(1, t) for t in (2048, 4096, 5632, 6144, 8192)]),
                                      (0, "dense", lattice_step,
                                       [(c, t) for c in (1, 2) for t in (2048, 4096, 5632, 8192)])):
        old = ctx.retina_get_tuning(D, kernel)
        try:
            for cand, tile in shapes:
                ctx.retina_set_tuning(D, kernel, cand, tile)
                step()
                pr = profiled(ctx, step, max(1, steps))
                tn = ctx.retina_get_tuning(D, kernel)
                out[key].append({"cand": cand, "tile_hits": tile, "grid": tn["grid"], "ascent_ms": pr["ms_hot"]})
                log("shape sweep %s: cand %d tile %d (grid %d): ascent %.3f ms" % (key, cand, tile, tn["grid"],
                                                                                  pr["ms_hot"]))
        finally:
            ctx.retina_set_tuning(D, kernel, old["cand"], old["tile_hits"])
    return out


def lattice_sweep(ctx, retina, b, dev_hits, P, sizes, quality, reps=2, prune_u=0.0):
    import torch
    D = b.meas_dim
    E = b.n_events
    rows = []
    for n in sizes:
        Pn = dict(P, lattice_n=[n, n], prune_u=prune_u)
        f = lambda: ctx.retina_find_tracks(D, b.plane_z, *dev_hits, Pn)
        r = f()
        torch.cuda.synchronize()
        qn = quality(retina.tracks_from_device(r)["theta"][:, :2 * D], r["track_offsets"].cpu().numpy())
        del r
        t0 = time.perf_counter()
        for _ in range(reps):
            f()
        torch.cuda.synchronize()
        tn = (time.perf_counter() - t0) / reps
        rows.append(dict(lattice_n=n, ms_per_step=tn * 1e3, events_per_s=E / tn,
                         efficiency=round(qn["efficiency"], 5), fake_rate=round(qn["fake_rate"], 5)))
        log("%slattice %dx%d: %.2f ms, efficiency %.4f fake %.4f" % (
            "pruned " if prune_u else "", n, n, tn * 1e3, qn["efficiency"], qn["fake_rate"]))
    ok = [r for r in rows if r["efficiency"] >= 0.95]
    best = min(ok, key=lambda r: r["ms_per_step"]) if ok else max(rows, key=lambda r: r["efficiency"])
    return rows, best


def r5(v):
    return None if v is None else float("%.5g" % v)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--lattice-sweep", type=int, nargs="*", default=None,
                    help="lattice sides to sweep for the baseline (default: the workload's list)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="approximate length of each CPU oracle sample")
    ap.add_argument("--cpu-max-events", type=int, default=256)
    ap.add_argument("--cpu-events", type=int, default=0,
                    help="fixed CPU oracle sample (first N events) instead of one sized by --cpu-seconds")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--studies", action="store_true",
                    help="also run the pruned comparison, the alpha-budget scans and the update rules")
    ap.add_argument("--shape-sweep", action="store_true",
                    help="also time both ascent launch shapes over hit tiles and candidates per lane")
    ap.add_argument("--detail-out", default=None, help="write the full report (JSON) to this file")
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
    dev_hits = (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))
    ctx = retina.Context(0)
    model = ctx.retina_model_load(LS["model"])
    torch.cuda.synchronize()
    z0, z1 = float(b.plane_z.min()), float(b.plane_z.max())
    ev_hits = np.diff(b.event_offsets)

    def quality(tracks_theta, toff):
        return metrics.batch_quality(D, tracks_theta, toff, b.truth, b.truth_nhits, cfg["match_tol"], z0, z1)

    # ---- lattice sweep: the fastest lattice reaching the efficiency bar is the baseline
    sizes = args.lattice_sweep or cfg.get("lattice_sweep", [P["lattice_n"][0]])
    sweep, best = lattice_sweep(ctx, retina, b, dev_hits, P, sizes, quality)
    P = dict(P, lattice_n=[best["lattice_n"], best["lattice_n"]])
    log("lattice baseline: %dx%d" % (best["lattice_n"], best["lattice_n"]))

    def lattice_step(want_seeds=False):
        return ctx.retina_find_tracks(D, b.plane_z, *dev_hits, P, want_seeds=want_seeds)

    def learned_step():
        return ctx.retina_find_tracks_learned(model, b.plane_z, *dev_hits, PL, LS["k_max"],
                                              LS["tau"], LS["conf_min"], nms=LS["nms"])

    # ---- quality + work accounting (untimed)
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

    prop = ctx.retina_propose_seeds(model, b.plane_z, *dev_hits, LS["k_max"], LS["tau"],
                                    LS["conf_min"], PL, nms=LS["nms"])
    so = prop["seed_offsets"]
    res = ctx.retina_find_tracks(D, b.plane_z, *dev_hits, PL, seeds=prop["seeds"].contiguous(),
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
    assert np.array_equal(res["track_offsets"].cpu().numpy(), toff_lrn)
    del res, res2, prop
    log("learned efficiency %.4f fake %.4f, %.1f seeds/event, fallback %.3f" % (
        q_lrn["efficiency"], q_lrn["fake_rate"], seeds_ev.mean(), fb_rate))

    # ---- timed regions
    for i in range(args.warmup):
        lattice_step()
        learned_step()
    log("%d warmup steps done" % args.warmup)
    wall_lrn, med_lrn, evs_lrn = timed_graph(learned_step, args.steps)
    log("learned: %.3f ms/step (wall mean), %.3f ms (HIP-event median)" % (wall_lrn * 1e3, med_lrn))
    wall_lat, med_lat, evs_lat = timed_graph(lattice_step, args.steps)
    log("lattice %dx%d: %.3f ms/step (wall mean), %.3f ms (HIP-event median)" % (
        P["lattice_n"][0], P["lattice_n"][1], wall_lat * 1e3, med_lat))
    nprof = max(1, min(args.steps, 5))
    prof_lrn = profiled(ctx, learned_step, nprof)
    prof_lat = profiled(ctx, lattice_step, nprof)
    log("profiled: learned proposer %.3f ms, ascent %.3f ms, merge %.3f ms; lattice ascent %.3f ms" % (
        prof_lrn["ms_propose"], prof_lrn["ms_hot"], prof_lrn["ms_merge"], prof_lat["ms_hot"]))

    # end to end from host memory (hits H2D, tracks D2H included)
    hb = (b.event_offsets, b.x, b.y, b.plane)
    ctx.retina_find_tracks_learned(model, b.plane_z, *hb, PL, LS["k_max"], LS["tau"], LS["conf_min"], nms=LS["nms"])
    nh = max(1, min(args.steps, 5))
    t0 = time.perf_counter()
    for _ in range(nh):
        ctx.retina_find_tracks_learned(model, b.plane_z, *hb, PL, LS["k_max"], LS["tau"], LS["conf_min"],
                                       nms=LS["nms"])
    ms_host = (time.perf_counter() - t0) / nh * 1e3
    log("learned, host memory end to end: %.2f ms/step" % ms_host)

    # ---- standalone response kernel; the cost model's T0, C and C0
    resp = response_throughput(ctx, retina, cfg, b, torch, np)
    resp_c2 = resp_c1 = None
    if args.workload == "c3":
        c2 = events.load_config("c2")
        resp_c2 = response_throughput(ctx, retina, c2, events.make_batch(c2, 1), torch, np)
        c1 = events.load_config("c1")
        c1g = dict(c1, params=dict(c1["params"], lattice_n=[400, 400]))
        resp_c1 = response_throughput(ctx, retina, c1g, events.make_batch(c1, 1), torch, np)
    T0_ns = resp["R"]["ns_per_candidate"]
    C = resp["RGH"]["ms"] / resp["R"]["ms"]
    q_steps = len(P["sigma"]) + P["n_final_steps"] + P["n_polish"]
    step_ns = prof_lat["ms_hot"] * 1e6 / (E * ns * q_steps)
    C0 = step_ns / T0_ns
    q_steps_l = len(PL["sigma"]) + PL["n_final_steps"] + PL["n_polish"]
    C0_learned = prof_lrn["ms_hot"] * 1e6 / (float(seeds_ev.sum()) * q_steps_l) / T0_ns
    log("cost model: T0 %.3f ns per line, C = %.3f (paper: 3), C0 = %.2f lattice, %.2f learned (paper: ~30)" % (
        T0_ns, C, C0, C0_learned))

    studies = {}
    if args.studies:
        studies = run_studies(ctx, retina, events, cfg, b, dev_hits, P, PL, LS, model, sizes, quality, args)
    if args.shape_sweep:
        studies["shape_sweep"] = shape_sweep(ctx, D, learned_step, lattice_step, args.steps)

    cpu = cpu_l = prec = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, learned seeds)")
        cpu_target = -float(args.cpu_events) if args.cpu_events > 0 else args.cpu_seconds
        cpu_l, ref_lrn = cpu_baseline_learned(cfg, LS, model, cpu_target, args.cpu_max_events)
        log("cpu baseline: %s" % cpu_l)
        log("cpu baseline (oracle, %dx%d lattice)" % tuple(P["lattice_n"]))
        cpu, ref_lat = cpu_baseline(cfg, P, cpu_target, args.cpu_max_events)
        log("cpu baseline lattice: %s" % cpu)
        prec = {"lattice": fp32_vs_fp64(D, tl["theta"], tl["R"], toff_lat, ref_lat, P["d_merge"], z0, z1),
                "learned": fp32_vs_fp64(D, tr["theta"], tr["R"], toff_lrn, ref_lrn, PL["d_merge"], z0, z1)}
        log("fp32 vs fp64 (oracle sample): %s" % prec)

    hot = prof_lrn["ms_hot"]
    achieved = fl_lrn / (hot * 1e-3) / 1e12
    net_tflops = FLOP_NET_EVENT * E / (prof_lrn["ms_propose"] * 1e-3) / 1e12
    rq = lambda q: {k: (round(v, 5) if isinstance(v, float) else v) for k, v in q.items()}
    kms = lambda p: {"stage": p["ms_stage"], "plan": p["ms_plan"], "ascent": p["ms_hot"], "merge": p["ms_merge"]}
    value = E / wall_lrn
    roofline = {"bound": "alu", "achieved": r5(achieved), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": r5(achieved / PEAK_FP32_TFLOPS), "traffic": measured_traffic(cfg["name"]),
                "kernel": "k_ascent (learned seeds)", "ms": r5(hot), "flops_per_launch": r5(fl_lrn)}
    prec_short = None
    if prec is not None:
        prec_short = {k: {"events": v["events"], "tracks": v["matched_tracks"], "gpu_only": v["gpu_only"],
                          "oracle_only": v["oracle_only"], "max_rel_dtheta": r5(v["max_rel_dtheta"]),
                          "max_rel_dR": r5(v["max_rel_dR"])} for k, v in prec.items()}
    headline = {
        "metric": "events/sec at >=95% track eff (learned vs lattice seeds); response evals/s, %FP32 peak",
        "value": r5(value),
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r5(wall_lrn * 1e3),
        "ms_per_step_events_median": r5(med_lrn),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d events, %d hits, learned seeds (lattice %dx%d fallback)"
                               % (cfg["name"], E, int(b.x.shape[0]), P["lattice_n"][0], P["lattice_n"][1]),
                   "parallelism": "single GPU"},
        "quality": {"efficiency": round(q_lrn["efficiency"], 5), "fake_rate": round(q_lrn["fake_rate"], 5),
                    "seeds_per_event": r5(float(seeds_ev.mean())), "fallback_rate": r5(fb_rate)},
        "lattice": {"n": best["lattice_n"], "events_per_s": r5(E / wall_lat), "ms_per_step": r5(wall_lat * 1e3),
                    "efficiency": round(q_lat["efficiency"], 5), "fake_rate": round(q_lat["fake_rate"], 5)},
        "speedup_vs_lattice": r5(wall_lat / wall_lrn),
        "roofline": roofline,
        "roofline_proposer": {"bound": "mfma", "achieved": r5(net_tflops), "peak": PEAK_BF16_TFLOPS,
                              "unit": "TFLOP/s", "frac": r5(net_tflops / PEAK_BF16_TFLOPS),
                              "ms": r5(prof_lrn["ms_propose"])},
        "response": {"RGH_pair_evals_per_s": r5(resp["RGH"]["pair_evals_per_s"]),
                     "RGH_frac_fp32_peak": r5(resp["RGH"]["frac_fp32_peak"]),
                     "R_pair_evals_per_s": r5(resp["R"]["pair_evals_per_s"]),
                     "R_frac_fp32_peak": r5(resp["R"]["frac_fp32_peak"])},
        "cost_model": {"T0_ns": r5(T0_ns), "C": r5(C), "C_paper": 3, "C0": r5(C0),
                       "C0_learned": r5(C0_learned), "C0_paper": 30, "q": q_steps},
        "cpu_baseline": (dict(cpu_l, value=r5(cpu_l["value"])) if cpu_l else None),
        "cpu_baseline_lattice": ({"value": r5(cpu["value"]), "cores": cpu["cores"]} if cpu else None),
        "fp32_vs_fp64": prec_short,
    }
    detail = dict(headline)
    detail.update({
        "ms_per_step_events": evs_lrn,
        "lattice_detail": {"ms_per_step_events": evs_lat, "ms_per_step_events_median": med_lat,
                           "kernel_ms": kms(prof_lat), "response_evals_per_s": pairs_lat / (prof_lat["ms_hot"] * 1e-3),
                           "ascent_tflops": fl_lat / (prof_lat["ms_hot"] * 1e-3) / 1e12,
                           "quality": rq(q_lat),
                           "pairs_per_launch": {"algorithmic": pairs_lat, "executed": prof_lat["exec_pairs"],
                                                "executed_line_search": prof_lat["exec_rpairs"]}},
        "learned_detail": {"kernel_ms": dict(kms(prof_lrn), proposer=prof_lrn["ms_propose"]),
                           "response_evals_per_s": pairs_lrn / (hot * 1e-3), "quality": rq(q_lrn),
                           "pairs_per_launch": {"algorithmic": pairs_lrn, "executed": prof_lrn["exec_pairs"],
                                                "executed_line_search": prof_lrn["exec_rpairs"]}},
        "roofline_proposer": {"bound": "mfma", "achieved": net_tflops, "peak": PEAK_BF16_TFLOPS,
                              "unit": "TFLOP/s", "frac": net_tflops / PEAK_BF16_TFLOPS,
                              "kernel": "binning + four conv layers + seed selection (network flops only)",
                              "flops_per_launch": FLOP_NET_EVENT * E},
        "lattice_sweep": sweep,
        "end_to_end_host_ms_per_step": ms_host,
        "response_detail": resp, "response_c2_event": resp_c2, "response_c1_grid": resp_c1,
        "cpu_baseline_lattice_detail": cpu,
        "fp32_vs_fp64_detail": prec,
        "studies": studies,
    })
    dj = json.dumps(detail)
    sys.stderr.write("[bench] detail %s\n" % dj)
    sys.stderr.flush()
    if args.detail_out:
        with open(args.detail_out, "w") as fh:
            fh.write(dj + "\n")
    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d MiB read + %d MiB written" % (args.calib_copy_mib, args.calib_copy_mib))
    line = json.dumps(headline, separators=(",", ":"))
    sys.stdout.write(line + "\n")
    sys.stdout.flush()


def run_studies(ctx, retina, events, cfg, b, dev_hits, P, PL, LS, model, sizes, quality, args):
    """Locality-pruned passes on both seedings, Section 3's alpha-budget scans
    (c7, c8) and the update-rule comparison."""
    import torch
    D = b.meas_dim
    E = b.n_events
    PU = 30.0
    sweep_p, best_p = lattice_sweep(ctx, retina, b, dev_hits, P, sizes, quality, prune_u=PU)
    PLp = dict(PL, prune_u=PU)

    def learned_pruned():
        return ctx.retina_find_tracks_learned(model, b.plane_z, *dev_hits, PLp, LS["k_max"],
                                              LS["tau"], LS["conf_min"], nms=LS["nms"])
    r = learned_pruned()
    torch.cuda.synchronize()
    q_lp = quality(retina.tracks_from_device(r)["theta"][:, :2 * D], r["track_offsets"].cpu().numpy())
    del r
    learned_pruned()
    wall, med, _ = timed_graph(learned_pruned, args.steps)
    log("pruned learned: %.2f ms/step, efficiency %.4f; pruned lattice %dx%d %.2f ms" % (
        wall * 1e3, q_lp["efficiency"], best_p["lattice_n"], best_p["lattice_n"], best_p["ms_per_step"]))
    out = {"pruned": {"prune_u": PU, "lattice_sweep": sweep_p, "lattice_best": best_p,
                      "learned": {"events_per_s": E / wall, "ms_per_step": wall * 1e3, "ms_events_median": med,
                                  "efficiency": round(q_lp["efficiency"], 5), "fake_rate": round(q_lp["fake_rate"], 5)},
                      "speedup_vs_lattice": best_p["ms_per_step"] / (wall * 1e3)}}
    from paper_1709_08610_amd import budget
    out["alpha_budget"] = budget.run(ctx, events.load_config("c7"), log=log)
    out["alpha_budget_svelo"] = budget.run(ctx, events.load_config("c8"), log=log)
    out["update_rules"] = {name: budget.compare_updates(ctx, events.load_config(name), log=log)
                           for name in ("c7", "c8")}
    return out


if __name__ == "__main__":
    main()
