"""Bandwidth-schedule search (Section 3: sigma is updated with each
optimisation step; the paper's own values 0.3, 0.175, 0.05 belong to its
geometry and units).

  python -m paper_1709_08610_amd.sigma_search [--reps 3] [--out FILE]

Candidates form a geometric family: stages sigma_1 r^k for every k with
sigma_1 r^k > 2 sigma_final, then n_final steps at sigma_final, then the FP64
polish; sigma_1 in {0.5, 1, 2, 4, 8} mm, r in {0.5, 0.35, 0.25}, n_final in
{2, 3}.  The schedule each workload runs today and the paper's three values
(read as mm) are scored beside them.  Stages of at least 0.5 mm move the slopes
only (offsets stay at the seed's x0 = y0 = 0, as the configured schedules do),
except on the simplified VELO, whose tracks come from the origin.

Workloads, each one batch on the GPU through retina_find_tracks:
  c2-like   the c7 scan point of 200 tracks (c2's generator), 512 events, the
            configured 64 x 64 lattice
  c3-learned  the 1024 c3 events from the trained proposer's seeds (lattice
            fallback included), the headline path
  c5-learned  the first 512 c5 events (about 800 tracks each) from the
            high-multiplicity proposer's seeds
  c8        the simplified VELO at 200 tracks, 512 events, 2304 draws per
            event from the track prior (Algorithm 1's first step)
Scores per (workload, schedule): the workload's efficiency and fake rate, the
time per event (median of --reps graph replays), q (optimisation steps per
seed) and C0 = time per seed and step / T0, where T0 is the standalone
response kernel's time for R at one line against one event's hits.
Choice (choose()): the fastest schedule whose efficiency is at most 0.005
below the current schedule's (and at least 0.95 where the current one reaches
0.95) and whose fake rate is at most 0.001 above it: a schedule may only buy
time at a quality the workload already has.  The output is one JSON object.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import events, learned, metrics, retina

SIGMA1 = (0.5, 1.0, 2.0, 4.0, 8.0)
RATIOS = (0.5, 0.35, 0.25)
N_FINAL = (2, 3)
PAPER = (0.3, 0.175, 0.05)
SLOPE_ONLY_MIN_SIGMA = 0.5   # mm: stages at or above move the slopes only
EFF_BAR = 0.95
EFF_SLACK = 0.005
FAKE_SLACK = 0.001


def choose(rows: list):
    """The fastest acceptable row (rows[0] is the current schedule), or None."""
    cur = rows[0]
    floor = cur["efficiency"] - EFF_SLACK
    if cur["efficiency"] >= EFF_BAR:
        floor = max(floor, EFF_BAR)
    ok = [r for r in rows if r["efficiency"] >= floor and r["fake_rate"] <= cur["fake_rate"] + FAKE_SLACK]
    return min(ok, key=lambda r: r["ms_per_event"]) if ok else None


def geometric(s1: float, r: float, sigma_final: float) -> list:
    out = []
    s = s1
    while s > 2.0 * sigma_final and len(out) < 16:
        out.append(float("%.6g" % s))
        s *= r
    return out


def candidates(base: dict) -> list:
    """(name, params) pairs: the current schedule first."""
    sf = float(base["sigma_final"])
    cur = dict(base)
    out = [("current", cur)]
    seen = {(tuple(cur["sigma"]), int(cur["n_final_steps"]))}

    def add(name, sig, nf):
        key = (tuple(sig), nf)
        if not sig or key in seen:
            return
        seen.add(key)
        p = dict(base, sigma=list(sig), n_final_steps=int(nf))
        if base.get("n_slope_steps", 0) < 99:
            p["n_slope_steps"] = sum(1 for s in sig if s >= SLOPE_ONLY_MIN_SIGMA)
        out.append((name, p))

    add("paper 0.3, 0.175, 0.05", list(PAPER), int(base["n_final_steps"]))
    for s1 in SIGMA1:
        for r in RATIOS:
            for nf in N_FINAL:
                add("s1=%g r=%g nf=%d" % (s1, r, nf), geometric(s1, r, sf), nf)
    return out


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


def _t0_ns(ctx, b, d, sigma, lines=4096):
    """R at `lines` lattice lines per event, standalone kernel: ns per line per event."""
    import torch
    rng = np.random.default_rng(0)
    th = np.zeros((lines, 4), np.float32)
    th[:, 2:] = rng.uniform(-0.3, 0.3, (lines, 2))
    E = b.n_events
    theta = torch.from_numpy(np.tile(th, (E, 1))).cuda()
    toff = torch.from_numpy(np.arange(E + 1, dtype=np.int64) * lines).cuda()
    f = lambda: ctx.retina_response(2, b.plane_z, *d, theta, toff, sigma=sigma, want=retina.WANT_R)
    ctx.retina_set_profiling(True)
    ctx.retina_profile_reset()
    for _ in range(3):
        f()
    torch.cuda.synchronize()
    pr = ctx.retina_get_profile()
    ctx.retina_set_profiling(False)
    return pr["ms_hot"] / max(pr["calls"], 1) * 1e6 / (lines * E)


def score(ctx, name, b, d, schedules, seeds_kw, n_seeds, qkey, tol, reps, log):
    import torch
    E = b.n_events
    z0, z1 = float(b.plane_z.min()), float(b.plane_z.max())
    fkey = {"eff_angle": "fake_rate_angle", "eff_eps": "fake_rate_eps"}.get(qkey, "fake_rate")
    t0 = _t0_ns(ctx, b, d, float(schedules[0][1]["sigma_final"]))
    rows = []
    for label, P in schedules:
        call = lambda: ctx.retina_find_tracks(2, b.plane_z, *d, P, capacity=E * 4096, **seeds_kw)
        t = _median_time(call, reps)
        res = call()
        torch.cuda.synchronize()
        tr = retina.tracks_from_device(res)
        qm = metrics.batch_quality(2, tr["theta"][:, :4], res["track_offsets"].cpu().numpy(), b.truth,
                                   b.truth_nhits, tol, z0, z1)
        q = len(P["sigma"]) + int(P["n_final_steps"]) + int(P["n_polish"])
        row = dict(schedule=label, sigma=P["sigma"], n_final=int(P["n_final_steps"]),
                   n_slope_steps=int(P.get("n_slope_steps", 0)), q=q, ms_per_event=1e3 * t / E,
                   efficiency=round(qm[qkey], 5), fake_rate=round(qm[fkey], 5),
                   C0=round(t * 1e9 / (n_seeds * q) / t0, 4))
        rows.append(row)
        log("  %-10s %-24s q %2d  %.4f ms/event  eff %.4f  fake %.4f  C0 %.2f" % (
            name, label, q, row["ms_per_event"], row["efficiency"], row["fake_rate"], row["C0"]))
    cur = rows[0]
    best = choose(rows)
    return dict(workload=name, events=E, seeds=int(n_seeds), T0_ns=t0, efficiency_key=qkey, fake_key=fkey, rows=rows,
                chosen=best, current=cur,
                speedup_vs_current=(cur["ms_per_event"] / best["ms_per_event"]) if best else None)


def run(ctx, reps=3, log=print):
    import torch
    tin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dev = lambda b: (tin(b.event_offsets), tin(b.x), tin(b.y), tin(b.plane))
    out = {"rule": "fastest with efficiency >= current - %.3f (>= %.2f where the current reaches it) and fake "
                   "rate <= current + %.3f" % (EFF_SLACK, EFF_BAR, FAKE_SLACK),
           "workloads": []}

    c7 = events.load_config("c7")
    (_, b7), = events.scan_batches(c7, [200], 512)
    d7 = dev(b7)
    n7 = c7["params"]["lattice_n"][0] * c7["params"]["lattice_n"][1]
    out["workloads"].append(score(ctx, "c2-like", b7, d7, candidates(c7["params"]), {}, E_seeds(b7, n7),
                                  "efficiency", c7["match_tol"], reps, log))

    c3 = events.load_config("c3")
    LS = learned.settings(c3)
    b3 = events.make_batch(c3)
    d3 = dev(b3)
    model = ctx.retina_model_load(LS["model"])
    prop = ctx.retina_propose_seeds(model, b3.plane_z, *d3, LS["k_max"], LS["tau"], LS["conf_min"],
                                    LS["params"], nms=LS["nms"])
    torch.cuda.synchronize()
    kw = dict(seeds=prop["seeds"].contiguous(), seed_offsets=prop["seed_offsets"])
    n3 = int(prop["seed_offsets"][-1].item())
    out["workloads"].append(score(ctx, "c3-learned", b3, d3, candidates(LS["params"]), kw, n3,
                                  "efficiency", c3["match_tol"], reps, log))

    c5 = events.load_config("c5")
    L5 = learned.settings(c5)
    b5 = events.make_batch(c5, 512)
    d5 = dev(b5)
    m5 = ctx.retina_model_load(L5["model"])
    p5 = ctx.retina_propose_seeds(m5, b5.plane_z, *d5, L5["k_max"], L5["tau"], L5["conf_min"],
                                  L5["params"], nms=L5["nms"])
    torch.cuda.synchronize()
    kw5 = dict(seeds=p5["seeds"].contiguous(), seed_offsets=p5["seed_offsets"])
    out["workloads"].append(score(ctx, "c5-learned", b5, d5, candidates(L5["params"]), kw5,
                                  int(p5["seed_offsets"][-1].item()), "efficiency", c5["match_tol"], reps, log))

    c8 = events.load_config("c8")
    (_, b8), = events.scan_batches(c8, [200], 512)
    d8 = dev(b8)
    k = 2304
    s, o = events.prior_seeds(c8, k, b8.index)
    out["workloads"].append(score(ctx, "c8", b8, d8, candidates(c8["params"]),
                                  dict(seeds=tin(s), seed_offsets=tin(o)), k * b8.n_events,
                                  c8.get("quality_key", "efficiency"), c8["match_tol"], reps, log))
    return out


def E_seeds(b, per_event):
    return int(per_event) * b.n_events


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="also write the JSON here")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("sigma_search needs a GPU")
    ctx = retina.Context(0)
    out = run(ctx, a.reps, log=lambda m: print(m, file=sys.stderr, flush=True))
    js = json.dumps(out)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(js + "\n")
    print(js)


if __name__ == "__main__":
    main()
