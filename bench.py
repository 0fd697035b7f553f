#!/usr/bin/env python3
"""Throughput of the Artificial Retina hot path on one MI355X.

One step = Algorithm 1 over the whole batch through the C-ABI: hit staging,
seeds, truncated-Newton ascents with sigma continuation, FP64 polish,
clustering and selection.  Two seedings of the same batch are timed:

  lattice  retina_find_tracks with the workload's uniform (tx, ty) lattice
  learned  retina_find_tracks_learned: the trained proposer network picks the
           seeds on the device (lattice fallback per event), then the same
           ascent, polish and merge

`value` is the learned path's events/s; the lattice figure, both track
qualities against generator truth, and the speedup are reported beside it.
Inputs are resident in device memory before the timed regions; each timed
region brackets exactly --steps calls with device synchronisation and runs
with the library's HIP-event profiling on (eager launches), which gives the
dominant kernel's (the ascent's) average duration on the library's stream.
The same steps replayed through the captured hipGraph are timed as well.
The FP64 CPU oracle is timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3       # MI355X FP32 vector peak (packed)
PEAK_FP32_UNPACKED = 78.6      # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz x 2 (FMA)
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
MEASURED_TRAFFIC = {("c3", "learned"): {"bytes": 83.2e6, "fetch": 75.7e6, "write": 7.3e6,
                                         "source_sha256_16": "670bf742c546b5b0"}}


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


def cpu_baseline(cfg, n_events):
    import oracle
    from paper_1709_08610_amd import events
    b = events.make_batch(cfg, n_events)
    threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    oracle.find_tracks(b, cfg["params"], n_threads=threads)
    dt = time.perf_counter() - t0
    return dict(value=n_events / dt, unit="events/s", cores=threads, kind="oracle",
                sample="first %d of %d events of the %s workload, full method with the %dx%d lattice "
                       "(FP64, OpenMP over seeds), %.1f s"
                       % (n_events, cfg["n_events"], cfg["name"], cfg["params"]["lattice_n"][0],
                          cfg["params"]["lattice_n"][1], dt))


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
    ap.add_argument("--cpu-events", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, one plain device-to-device copy of this many MiB (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(events shard across GPUs with no exchange; see DESIGN.md). Use --gpus 1.")
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

    # ---- quality + work accounting (untimed)
    log("lattice: quality + work accounting run")
    res = lattice_step(want_seeds=True)
    torch.cuda.synchronize()
    tl = retina.tracks_from_device(res)
    q_lat = quality(tl["theta"][:, :2 * D], res["track_offsets"].cpu().numpy())
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
    q_lrn = quality(tr["theta"][:, :2 * D], res2["track_offsets"].cpu().numpy())
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
    log("lattice: %.2f ms/step (graph replay %.2f), ascent %.2f ms" % (dt_lat * 1e3, g_lat * 1e3, prof_lat["ms_hot"]))
    dt_lrn, prof_lrn, g_lrn = timed(ctx, learned_step, args.steps)
    log("learned: %.2f ms/step (graph replay %.2f), proposer %.2f ms, ascent %.2f ms" % (
        dt_lrn * 1e3, g_lrn * 1e3, prof_lrn["ms_propose"], prof_lrn["ms_hot"]))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on %d events" % args.cpu_events)
        cpu = cpu_baseline(cfg, args.cpu_events)

    hot = prof_lrn["ms_hot"]
    achieved = fl_lrn / (hot * 1e-3) / 1e12
    net_tflops = FLOP_NET_EVENT * E / (prof_lrn["ms_propose"] * 1e-3) / 1e12
    rq = lambda q: {k: (round(v, 5) if isinstance(v, float) else v) for k, v in q.items()}
    kms = lambda p: {"stage": p["ms_stage"], "plan": p["ms_plan"], "ascent": p["ms_hot"], "merge": p["ms_merge"]}
    out = {
        "metric": "events/sec at >=95% track eff (learned vs lattice seeds); response evals/s, %FP32 peak",
        "value": E / dt_lrn,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt_lrn * 1e3,
        "ms_per_step_graph_replay": g_lrn * 1e3,
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
        "lattice": {"events_per_s": E / dt_lat, "ms_per_step": dt_lat * 1e3, "ms_per_step_graph_replay": g_lat * 1e3,
                    "quality": rq(q_lat), "kernel_ms": kms(prof_lat),
                    "response_evals_per_s": pairs_lat / (prof_lat["ms_hot"] * 1e-3),
                    "ascent_tflops": fl_lat / (prof_lat["ms_hot"] * 1e-3) / 1e12,
                    "pairs_per_launch": {"algorithmic": pairs_lat, "executed": prof_lat["exec_pairs"],
                                         "executed_line_search": prof_lat["exec_rpairs"]}},
        "speedup_vs_lattice": dt_lat / dt_lrn,
        "response_evals_per_s": pairs_lrn / (hot * 1e-3),
        "pairs_per_launch": {"algorithmic": pairs_lrn, "executed": prof_lrn["exec_pairs"],
                             "executed_line_search": prof_lrn["exec_rpairs"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "frac_unpacked_peak": achieved / PEAK_FP32_UNPACKED,
                     "traffic": measured_traffic(cfg["name"]), "traffic_unit": "bytes per launch", "kernel": "k_ascent (persistent truncated-Newton ascent, learned seeds)",
                     "flops_per_launch": fl_lrn},
        "roofline_proposer": {"bound": "mfma", "achieved": net_tflops, "peak": PEAK_BF16_TFLOPS,
                              "unit": "TFLOP/s", "frac": net_tflops / PEAK_BF16_TFLOPS,
                              "kernel": "binning + four conv layers + seed selection (network flops only)",
                              "flops_per_launch": FLOP_NET_EVENT * E},
        "cpu_baseline": cpu,
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
