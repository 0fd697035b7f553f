#!/usr/bin/env python3
"""Throughput of the Artificial Retina hot path on one MI355X.

One step = Algorithm 1 over the whole batch through the C-ABI
(retina_find_tracks): hit staging, seeds, truncated-Newton ascents with sigma
continuation, FP64 polish, clustering and selection.  Inputs are resident in
device memory before the timed region; the timed region brackets exactly
--steps calls with device synchronisation.

The JSON line reports events/s (value), the track quality of the same
configuration against generator truth, the dominant kernel's (ascent) time
from HIP events on the library's stream, its algorithmic FP32 work per launch
against the FP32 vector peak, and the FP64 CPU oracle timed on a bounded
sample of the same workload.
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
# algorithmic FP32 flops (FMA = 2, exp2 not counted) per hit-candidate pair,
# meas_dim 2, per-plane factored sums
FLOP_RGH_PAIR = 21
FLOP_R_PAIR = 11
FLOP_POLISH_PAIR = 25          # RGH pair with the two-float residual (4 more)
FLOP_FOLD = 26                 # per (candidate, plane) per derivative pass


def log(msg):
    sys.stderr.write("[bench] %s\n" % msg)
    sys.stderr.flush()


def algorithmic_flops(P, ev_hits, ev_seeds, nreval_per_event, n_planes):
    n_steps = len(P["sigma"]) + P["n_final_steps"]
    fl = 0.0
    for nh, ns, nr in zip(ev_hits, ev_seeds, nreval_per_event):
        fl += nh * ns * (n_steps * FLOP_RGH_PAIR + P["n_polish"] * FLOP_POLISH_PAIR)
        fl += nh * nr * FLOP_R_PAIR
        fl += ns * n_planes * FLOP_FOLD * (n_steps + P["n_polish"])
    pairs = 0.0
    for nh, ns, nr in zip(ev_hits, ev_seeds, nreval_per_event):
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
                sample="first %d of %d events of the %s workload, full method (FP64, OpenMP over seeds), %.1f s"
                % (n_events, cfg["n_events"], cfg["name"], dt))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--cpu-events", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(events shard across GPUs with no exchange; see DESIGN.md). Use --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1709_08610_amd import events, metrics, retina

    cfg = events.load_config(args.workload)
    P = cfg["params"]
    log("generating %s (%d events)" % (cfg["name"], cfg["n_events"]))
    b = events.make_batch(cfg)
    D = b.meas_dim
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    off_d, x_d, pl_d = tin(b.event_offsets), tin(b.x), tin(b.plane)
    y_d = tin(b.y) if D == 2 else None
    ctx = retina.Context(0)
    torch.cuda.synchronize()

    def step(want_seeds=False):
        return ctx.retina_find_tracks(D, b.plane_z, off_d, x_d, y_d, pl_d, P, want_seeds=want_seeds)

    log("quality + work accounting run")
    res = step(want_seeds=True)
    torch.cuda.synchronize()
    tracks = retina.tracks_from_device(res)
    toff = res["track_offsets"].cpu().numpy()
    z0, z1 = float(b.plane_z.min()), float(b.plane_z.max())
    q = metrics.batch_quality(D, tracks["theta"][:, :2 * D], toff, b.truth, b.truth_nhits,
                              cfg["match_tol"], z0, z1)
    nre = res["seed_nreval"].cpu().numpy().astype(np.int64)
    ns = P["lattice_n"][0] * P["lattice_n"][1]
    ev_hits = np.diff(b.event_offsets)
    nre_ev = nre.reshape(b.n_events, ns).sum(axis=1)
    flops, pairs = algorithmic_flops(P, ev_hits, [ns] * b.n_events, nre_ev, len(b.plane_z))
    log("efficiency %.4f fake %.4f clone %.4f tracks %d" % (q["efficiency"], q["fake_rate"],
                                                            q["clone_rate"], int(toff[-1])))
    del res

    for i in range(args.warmup):
        step()
        log("warmup %d done" % (i + 1))
    ctx.retina_set_profiling(True)
    ctx.retina_profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.retina_get_profile()
    ctx.retina_set_profiling(False)
    dt = t1 - t0
    # the same steps replayed through the captured graph (no per-kernel events)
    step()
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - tg0) / args.steps * 1e3
    ms_step = dt / args.steps * 1e3
    hot_ms = prof["ms_hot"] / max(prof["calls"], 1)
    achieved = flops / (hot_ms * 1e-3) / 1e12
    log("timed %d steps: %.2f ms/step, ascent kernel %.2f ms" % (args.steps, ms_step, hot_ms))

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) on %d events" % args.cpu_events)
        cpu = cpu_baseline(cfg, args.cpu_events)

    out = {
        "metric": "events/sec at >=95% track eff (lattice seeds); response evals/s, %FP32 peak",
        "value": b.n_events * args.steps / dt,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_graph_replay": ms_graph,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %s" % (cfg["name"], cfg["description"]), "events": b.n_events,
                   "hits": int(b.x.shape[0]), "seeds": "lattice %dx%d" % tuple(P["lattice_n"]),
                   "parallelism": "single GPU"},
        "quality": {k: (round(v, 5) if isinstance(v, float) else v) for k, v in q.items()},
        "kernel_ms": {"stage": prof["ms_stage"] / max(prof["calls"], 1),
                      "plan": prof["ms_plan"] / max(prof["calls"], 1), "ascent": hot_ms,
                      "merge": prof["ms_merge"] / max(prof["calls"], 1)},
        "response_evals_per_s": pairs / (hot_ms * 1e-3),
        "pairs_per_launch": {"algorithmic": pairs,
                             "executed": prof["exec_pairs"] / max(prof["calls"], 1),
                             "executed_line_search": prof["exec_rpairs"] / max(prof["calls"], 1)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "frac_unpacked_peak": achieved / PEAK_FP32_UNPACKED,
                     "traffic": None, "kernel": "k_ascent (persistent truncated-Newton ascent)",
                     "flops_per_launch": flops},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
