"""Multi-start at a fraction alpha of the grid search's cost (Section 3, the
comparison of Fig. 3), both methods on the same GPU.

  python -m paper_1709_08610_amd.budget [--events 16] [--counts 50 200 350]

Section 3 sets the number of seeds to n = alpha * n_grid / (C0 * q): n_grid
cells give the grid search its epsilon resolution, each seed makes q
optimisation steps, and one step costs C0 response evaluations T0.  Every
quantity is measured here on the device that runs both methods:
  T0    grid-search time per cell (the response of one line against the event,
        plus the cell's share of the peak passes)
  q     steps per seed: the sigma stages, the final steps and the FP64 polish
  C0    multi-start time per seed and step, divided by T0, calibrated on a
        reference lattice at the middle track count
Both are throughput figures: each track count is a batch of hundreds of events,
so that even the smallest seed lattice keeps the GPU busy (a few events with a
few hundred seeds each would time the latency of one seed's twelve sequential
steps, not the cost the formula counts).
Seeds: a square lattice of floor(sqrt(n)) per side over the prior box, or,
for a config with "seeding": "prior", round(n) draws per event from the track
prior (Algorithm 1's first step), passed in as explicit seeds.
Workloads: the c7 track-count scan (c2 geometry, 50..350 tracks per event;
efficiency by the paper's 1e-3 criterion on the slopes, eff_eps) and the c8
scan on the simplified VELO of Section 3 (tracks from the origin; 1e-3 rad
between directions, eff_angle).  The multi-start is also scored with the
end-plane criterion of the benchmark (the grid estimates carry slopes only).
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import events, metrics, retina


def _median_time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _tracks(res, E):
    toff = res["track_offsets"].cpu().numpy()
    tr = res["tracks_bytes"].cpu().numpy()[: int(toff[-1]) * 48].view(retina.TRACK_DTYPE)
    return tr["theta"], toff


def run(ctx, cfg=None, counts=None, events_per_point=None, reps=3, log=print):
    """The alpha-budget comparison; returns a JSON-ready dict."""
    import torch
    cfg = cfg or events.load_config("c7")
    P = dict(cfg["params"])
    G = cfg["grid"]
    n_grid = int(G["n"][0]) * int(G["n"][1])
    q = len(P["sigma"]) + int(P["n_final_steps"]) + int(P["n_polish"])
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pts = events.scan_batches(cfg, counts, events_per_point)
    z0, z1 = float(cfg["planes"]["z_first"]), float(cfg["planes"]["z_last"])

    def prep(b):
        return b, (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))

    pts = [(n, *prep(b)) for n, b in pts]

    def grid_call(b, d):
        E = b.n_events
        return ctx.retina_grid_search(2, b.plane_z, *d, G, capacity=E * 4096)

    prior = cfg.get("seeding") == "prior"
    qkey = cfg.get("quality_key", "eff_eps")

    def seeds_for(b, n):
        """(find_tracks keyword arguments, seeds per event) for about n seeds per event."""
        if prior:
            k = max(1, int(round(n)))
            s, o = events.prior_seeds(cfg, k, b.index)
            return dict(params=P, seeds=tin(s), seed_offsets=tin(o)), k
        side = max(1, int(math.floor(math.sqrt(n))))
        return dict(params=dict(P, lattice_n=[side, side])), side * side

    def ms_call(b, d, kw, k):
        return ctx.retina_find_tracks(2, b.plane_z, *d, kw["params"], seeds=kw.get("seeds"),
                                      seed_offsets=kw.get("seed_offsets"), capacity=b.n_events * k)

    def quality(b, theta, toff):
        return metrics.batch_quality(2, theta, toff, b.truth, b.truth_nhits, cfg["match_tol"], z0, z1)

    # calibration at the middle count: T0 from the grid search, C0 from a reference lattice
    n_mid, b_mid, d_mid = pts[len(pts) // 2]
    E = b_mid.n_events
    t_grid = _median_time(lambda: grid_call(b_mid, d_mid), reps)
    T0 = t_grid / (E * n_grid)
    side_ref = int(cfg.get("calibration_lattice", 48))
    kw_ref, k_ref = seeds_for(b_mid, side_ref * side_ref)
    t_ref = _median_time(lambda: ms_call(b_mid, d_mid, kw_ref, k_ref), reps)
    C0 = t_ref / (E * k_ref * q) / T0
    log("alpha budget (%s): n_grid %d, q %d, T0 %.3g ns per cell, C0 %.2f (%d seeds at %d tracks)"
        % (cfg["name"], n_grid, q, T0 * 1e9, C0, k_ref, n_mid))
    out = dict(workload="%s: %s" % (cfg["name"], cfg["description"]), events_per_point=E, grid=G, n_grid=n_grid,
               q=q, T0_ns=T0 * 1e9, C0=C0, C0_calibration=dict(n_tracks=n_mid, seeds=k_ref),
               seeding="prior draws" if prior else "lattice", efficiency_criterion=qkey,
               paper=dict(C0=30, q=3), points=[])
    for n_tr, b, d in pts:
        E = b.n_events
        t_g = _median_time(lambda: grid_call(b, d), reps)
        qg = quality(b, *_tracks(grid_call(b, d), E))
        row = dict(n_tracks=n_tr, hits_per_event=float(np.mean(np.diff(b.event_offsets))),
                   grid=dict(ms_per_event=1e3 * t_g / E, eff=qg[qkey], eff_eps=qg["eff_eps"],
                             eff_angle=qg["eff_angle"], fake_rate_eps=qg["fake_rate_eps"],
                             peaks_per_event=qg["n_found"] / E))
        for a in cfg["alphas"]:
            n = a * n_grid / (C0 * q)
            kw, k = seeds_for(b, n)
            t_m = _median_time(lambda: ms_call(b, d, kw, k), reps)
            qm = quality(b, *_tracks(ms_call(b, d, kw, k), E))
            row["alpha_%.4g" % a] = dict(alpha=a, seeds=k, seeds_formula=n, ms_per_event=1e3 * t_m / E,
                                         cost_ratio=t_m / t_g, eff=qm[qkey], eff_eps=qm["eff_eps"],
                                         eff_angle=qm["eff_angle"], efficiency=qm["efficiency"],
                                         fake_rate=qm["fake_rate"], fake_rate_eps=qm["fake_rate_eps"])
        out["points"].append(row)
        log("  %3d tracks: grid %s %.3f (%.3f ms/event) | %s" % (
            n_tr, qkey, qg[qkey], 1e3 * t_g / E,
            " | ".join("alpha %.3g: %d seeds, %s %.3f, eff %.3f, cost %.2f" % (
                r["alpha"], r["seeds"], qkey, r["eff"], r["efficiency"], r["cost_ratio"])
                for k, r in row.items() if k.startswith("alpha_"))))
    return out


def compare_updates(ctx, cfg=None, n_tracks=200, events_per_point=None, seeds=2304, reps=3, log=print):
    """Section 3's choice among update rules: truncated Newton, the normalised
    gradient and BFGS from the same seeds on the same events (the middle point
    of a scan), with the same steps, line search and FP64 polish: efficiency
    and measured time per seed and step (in units of T0, the grid-search cost
    per cell, as C0)."""
    import torch
    cfg = cfg or events.load_config("c7")
    P = dict(cfg["params"])
    G = cfg["grid"]
    n_grid = int(G["n"][0]) * int(G["n"][1])
    q = len(P["sigma"]) + int(P["n_final_steps"]) + int(P["n_polish"])
    qkey = cfg.get("quality_key", "eff_eps")
    dev = torch.device("cuda:0")
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    (_, b), = events.scan_batches(cfg, [n_tracks], events_per_point)
    E = b.n_events
    d = (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))
    z0, z1 = float(cfg["planes"]["z_first"]), float(cfg["planes"]["z_last"])
    t_grid = _median_time(lambda: ctx.retina_grid_search(2, b.plane_z, *d, G, capacity=E * 4096), reps)
    T0 = t_grid / (E * n_grid)
    if cfg.get("seeding") == "prior":
        s, o = events.prior_seeds(cfg, seeds, b.index)
        kw = dict(seeds=tin(s), seed_offsets=tin(o))
        k = seeds
    else:
        side = int(round(math.sqrt(seeds)))
        P = dict(P, lattice_n=[side, side])
        kw = {}
        k = side * side
    out = dict(workload="%s, %d tracks per event, %d events" % (cfg["name"], n_tracks, E), seeds=k, q=q,
               T0_ns=T0 * 1e9, efficiency_criterion=qkey, rules={})
    for rule in ("newton", "gradient", "bfgs"):
        Pr = dict(P, update=rule)
        call = lambda: ctx.retina_find_tracks(2, b.plane_z, *d, Pr, capacity=E * k, **kw)
        t = _median_time(call, reps)
        theta, toff = _tracks(call(), E)
        qm = metrics.batch_quality(2, theta, toff, b.truth, b.truth_nhits, cfg["match_tol"], z0, z1)
        out["rules"][rule] = dict(ms_per_event=1e3 * t / E, C0=t / (E * k * q) / T0, eff=qm[qkey],
                                  efficiency=qm["efficiency"], fake_rate=qm["fake_rate"],
                                  tracks_per_event=qm["n_found"] / E)
        log("  update %-8s: %s %.3f, eff %.3f, C0 %.2f, %.3f ms/event" % (
            rule, qkey, qm[qkey], qm["efficiency"], out["rules"][rule]["C0"], 1e3 * t / E))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--events", type=int, default=None, help="events per track count (default: the config's)")
    ap.add_argument("--counts", type=int, nargs="*", default=None)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--config", default="c7", help="c7 (c2 geometry) or c8 (simplified VELO)")
    ap.add_argument("--updates", action="store_true", help="compare the update rules instead of the scan")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("budget needs a GPU")
    ctx = retina.Context(0)
    lg = lambda m: print(m, file=sys.stderr, flush=True)
    if a.updates:
        out = compare_updates(ctx, events.load_config(a.config), events_per_point=a.events, reps=a.reps, log=lg)
    else:
        out = run(ctx, events.load_config(a.config), counts=a.counts, events_per_point=a.events, reps=a.reps, log=lg)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
