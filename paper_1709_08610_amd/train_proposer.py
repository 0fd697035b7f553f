"""Training driver of the learned seed proposer (runs on one gfx950 GPU).

  python -m paper_1709_08610_amd.train_proposer --events 100000 --epochs 2 \\
      --out paper_1709_08610_amd/models/proposer_c4.bin

1. Events of the training workload (c4: the generator of the 1024-event batch
   with its own key; c6: likewise for the high-multiplicity batch) are drawn
   on the host cores in parallel and moved to the GPU once.
2. Labels: the maxima the plain method finds, i.e. the tracks of
   retina_find_tracks with the workload's seed lattice (Algorithm 1 with its
   FP64 polish and merge); their slopes (tx, ty) mark the target heatmap.
3. Adam on the weighted binary cross-entropy through retina_train_step, batches
   of consecutive events visited in a seeded random order per epoch, cosine
   learning-rate decay after a short linear warm-up.
4. The model file (weights, Adam moments, step) is written at the end of every
   epoch; --resume continues from one (the step fixes the data position).

Everything numeric runs in libretina; torch only holds device memory.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

from . import events, retina


def _gen_chunk(args):
    name, lo, hi = args
    cfg = events.load_config(name)
    zp = events.plane_z(cfg)
    evs = [events.make_event(cfg, i, zp) for i in range(lo, hi)]
    nh = np.array([e.n_hits for e in evs], np.int64)
    return (np.concatenate([e.x for e in evs]), np.concatenate([e.y for e in evs]),
            np.concatenate([e.plane for e in evs]).astype(np.int32), nh)


def generate(name: str, n_events: int, start: int = 0, workers: int = 0):
    """Events [start, start + n_events) of a workload as flat host arrays."""
    workers = workers or min(16, os.cpu_count() or 1)
    step = 2000
    chunks = [(name, a, min(a + step, start + n_events)) for a in range(start, start + n_events, step)]
    if workers > 1 and len(chunks) > 1:
        with mp.get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_gen_chunk, chunks)
    else:
        parts = [_gen_chunk(c) for c in chunks]
    x = np.concatenate([p[0] for p in parts])
    y = np.concatenate([p[1] for p in parts])
    plane = np.concatenate([p[2] for p in parts])
    off = np.concatenate([[0], np.cumsum(np.concatenate([p[3] for p in parts]))]).astype(np.int64)
    return x, y, plane, off


class DeviceEvents:
    """A batch of events resident in device memory, sliceable by event range."""

    def __init__(self, x, y, plane, off, device="cuda:0"):
        import torch
        self.x = torch.from_numpy(x).to(device)
        self.y = torch.from_numpy(y).to(device)
        self.plane = torch.from_numpy(plane).to(device)
        self.off_host = off
        self.off = torch.from_numpy(off).to(device)
        self.n_events = off.shape[0] - 1

    def slice(self, e0, e1):
        a, b = int(self.off_host[e0]), int(self.off_host[e1])
        return self.off[e0:e1 + 1] - a, self.x[a:b], self.y[a:b], self.plane[a:b]


def label(ctx, zp, dev: DeviceEvents, params: dict, chunk: int = 4096):
    """Slopes of the tracks found with the lattice, per event (device tensors)."""
    import torch
    tg, counts = [], []
    for e0 in range(0, dev.n_events, chunk):
        e1 = min(e0 + chunk, dev.n_events)
        off, x, y, pl = dev.slice(e0, e1)
        res = ctx.retina_find_tracks(2, zp, off, x, y, pl, params)
        toff = res["track_offsets"]
        n = int(toff[-1].item())
        th = res["tracks_bytes"][: n * 48].view(torch.float64).view(n, 6)[:, 2:4].clone()
        tg.append(th)
        counts.append(toff.diff())
        print("labelled events %d..%d: %d tracks" % (e0, e1 - 1, n), flush=True)
    cnt = torch.cat(counts)
    toff = torch.zeros(dev.n_events + 1, dtype=torch.int64, device=cnt.device)
    toff[1:] = torch.cumsum(cnt, 0)
    return torch.cat(tg).contiguous(), toff


def lr_at(step: int, total: int, lr: float, warmup: int = 100, floor: float = 0.05) -> float:
    if step < warmup:
        return lr * (step + 1) / warmup
    t = min(1.0, (step - warmup) / max(1, total - warmup))
    return lr * (floor + (1 - floor) * 0.5 * (1 + math.cos(math.pi * t)))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--config", default="c4")
    ap.add_argument("--events", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--pos-weight", type=float, default=10.0)
    ap.add_argument("--init-key", type=int, default=20170925)
    ap.add_argument("--order-key", type=int, default=1709)
    ap.add_argument("--out", required=True)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--log-every", type=int, default=200)
    a = ap.parse_args(argv)

    cfg = events.load_config(a.config)
    zp = events.plane_z(cfg)
    t0 = time.time()
    # host worker processes start before this process touches the GPU
    x, y, plane, off = generate(a.config, a.events)
    print("generated %d events (%d hits) in %.1f s" % (a.events, x.shape[0], time.time() - t0), flush=True)
    import torch
    if not torch.cuda.is_available():
        sys.exit("train_proposer needs a GPU")
    dev = DeviceEvents(x, y, plane, off)
    del x, y, plane
    ctx = retina.Context(0)
    ctx.set_stream(torch.cuda.current_stream().cuda_stream)
    t0 = time.time()
    tg, toff = label(ctx, zp, dev, cfg["params"])
    torch.cuda.synchronize()
    toff_host = toff.cpu().numpy()
    print("labelled: %d tracks (%.1f per event) in %.1f s" % (toff_host[-1], toff_host[-1] / a.events,
                                                               time.time() - t0), flush=True)

    model = ctx.retina_model_load(a.resume) if a.resume else ctx.retina_model_create(a.init_key)
    n_batches = a.events // a.batch
    total = n_batches * a.epochs
    rng = np.random.default_rng(a.order_key)
    orders = [rng.permutation(n_batches) for _ in range(a.epochs)]
    t0 = time.time()
    run = []
    for step in range(model.step, total):
        ep, i = divmod(step, n_batches)
        b = int(orders[ep][i])
        e0, e1 = b * a.batch, (b + 1) * a.batch
        eoff, xs, ys, ps = dev.slice(e0, e1)
        ta, tb = int(toff_host[e0]), int(toff_host[e1])
        loss, _ = ctx.retina_train_step(model, zp, eoff, xs, ys, ps, tg[ta:tb], toff[e0:e1 + 1] - ta,
                                        lr_at(step, total, a.lr), a.pos_weight)
        run.append(loss)
        if (step + 1) % a.log_every == 0 or step + 1 == total:
            dt = time.time() - t0
            print(json.dumps(dict(step=step + 1, epoch=ep, loss=float(np.mean(run)), lr=lr_at(step, total, a.lr),
                                  events_per_s=round(a.log_every * a.batch / dt, 1))), flush=True)
            run = []
            t0 = time.time()
        if (step + 1) % n_batches == 0 or step + 1 == total:
            model.retina_model_save(a.out)
    print("saved %s at step %d" % (a.out, model.step), flush=True)


if __name__ == "__main__":
    main()
