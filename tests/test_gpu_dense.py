"""GPU parity at high multiplicity (Algorithm 1's last two steps on dense
events): the merge's paths for events too large for its LDS caches, against
the FP64 oracle.

The merge kernel sorts an event's candidate keys in LDS when the event has at
most 8,192 seeds (1,024 in the shape used when a batch averages at most 1,024
seeds per event) and otherwise in a global scratch; it caches the first 1,024
cluster leaders in LDS (256 in that small shape) and reads later leaders from
global memory.  Each case below is built to reach one of those paths, and
asserts that it does:

  * the first two events of the 4096-event high-multiplicity batch with its
    configured 128 x 128 lattice (16,384 seeds per event: global key sort);
  * the same two events on the seeds the oracle's own proposer picks with the
    high-multiplicity weights (the learned path at that density);
  * a batch averaging few seeds per event (small shape) with one event of
    ~1,600 seeds and ~800 clusters (global key sort and global leaders);
  * one event of 1,600 tracks seeded at its true lines and a perturbed copy
    of each (~3,200 seeds, ~1,500 clusters: global leaders in the large shape);
  * a learned batch of seven ordinary events and one noise-only event, which
    falls back to the 4,096-seed lattice while the batch average stays in the
    small shape.

Expected tracks of the slow cases come from tests/golden/dense_oracle.npz,
written by tests/golden/make_dense_oracle.py (oracle only); the others run
the oracle here.  Bar: track sets identical after matching within d_merge,
parameters within 1e-4 relative (scale floors), R within 1e-5 relative."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from oracle import proposer as op
from paper_1709_08610_amd import events, learned, retina

from gpu_util import assert_tracks_match, event_tracks
from proposer_util import _logit_bound, _oracle_images

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dense_oracle.npz")
MERGE_KEYS, MERGE_LEADERS = 8192, 1024           # LDS capacities of the merge (large shape)
SMALL_KEYS, SMALL_LEADERS = 1024, 256            # ... and of the small shape


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


@pytest.fixture(scope="module")
def gold():
    with np.load(GOLD, allow_pickle=False) as f:
        return {k: f[k] for k in f.files}


def _compare(res, gold, prefix, d_merge, z0, z1):
    toff = gold[prefix + "_toff"]
    E = len(toff) - 1
    for e in range(E):
        a, c = int(toff[e]), int(toff[e + 1])
        gt, gR = event_tracks(res, e, 2)
        assert_tracks_match(2, gt, gR, gold[prefix + "_theta"][a:c], gold[prefix + "_R"][a:c], d_merge, z0, z1)
    return int(toff[-1])


def test_c5_lattice_global_key_sort(ctx, gold):
    cfg = events.load_config("c5")
    P = cfg["params"]
    n = P["lattice_n"][0] * P["lattice_n"][1]
    assert n > MERGE_KEYS  # dense shape, keys sorted in the global scratch
    _say("c5 events 0-1, %dx%d lattice (%d seeds per event)" % (P["lattice_n"][0], P["lattice_n"][1], n))
    b = events.make_batch(cfg, 2)
    res = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P)
    nt = _compare(res, gold, "c5lat", P["d_merge"], float(b.plane_z[0]), float(b.plane_z[-1]))
    _say("  %d tracks match" % nt)


def test_c5_learned_seeds(ctx):
    """The proposer with the high-multiplicity weights on the first two events:
    the device's seed bins equal the oracle's (FP64 forward, same weights) up
    to bins whose logit lies within the forward error bound of the threshold;
    the ascent on the oracle's seeds matches the oracle's tracks, and where the
    seed sets are identical so does the whole learned entry point."""
    cfg = events.load_config("c5")
    LS = learned.settings(cfg)
    b = events.make_batch(cfg, 2)
    model = ctx.retina_model_load(LS["model"])
    layers = op.unpack_params(model.retina_model_get_params())
    _say("c5 events 0-1, learned seeds (k_max %d, tau %g)" % (LS["k_max"], LS["tau"]))
    res = ctx.retina_propose_seeds(model, b.plane_z, b.event_offsets, b.x, b.y, b.plane, LS["k_max"], LS["tau"],
                                   LS["conf_min"], LS["params"], nms=LS["nms"])
    thr = op.logit_threshold(LS["tau"])
    lo = float(np.float32(op.SLOPE_LO))
    w = (float(np.float32(op.SLOPE_HI)) - lo) / op.IMG
    ref_seeds, ref_off, same = [], [0], True
    for e, img in enumerate(_oracle_images(b)):
        _, z = op.forward(img, layers, store_bf16=True)
        picks = op.seed_bins(z, LS["tau"], LS["k_max"], nms=LS["nms"])
        assert res["fallback"][e] == 0 and z.max() >= op.logit_threshold(LS["conf_min"])
        a, c = int(res["seed_offsets"][e]), int(res["seed_offsets"][e + 1])
        s = res["seeds"][a:c]
        gpix = set((np.floor((s[:, 2] - lo) / w).astype(int) * op.IMG + np.floor((s[:, 3] - lo) / w).astype(int)))
        diff = gpix ^ set(picks)
        if diff:
            bound = _logit_bound(img, layers).ravel()
            zf = z.ravel()
            marginal = [p for p in diff if abs(zf[p] - thr) <= 1.5 * bound[p] + 1e-6]
            assert len(marginal) == len(diff), "event %d: seed bins differ beyond the error bound: %s" % (
                e, sorted(set(diff) - set(marginal))[:10])
            same = False
        ref_seeds.append(op.seeds_from_pixels(picks))
        ref_off.append(ref_off[-1] + len(picks))
        _say("  event %d: %d seeds, %d differing (marginal) bins" % (e, len(picks), len(diff)))
    seeds, soff = np.concatenate(ref_seeds), np.array(ref_off, np.int64)
    ref = oracle.find_tracks(b, LS["params"], seeds, soff)
    z0, z1 = float(b.plane_z[0]), float(b.plane_z[-1])
    got = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, LS["params"], seeds=seeds,
                                 seed_offsets=soff)
    runs = [("explicit oracle seeds", got)]
    if same:
        runs.append(("learned entry point", ctx.retina_find_tracks_learned(
            model, b.plane_z, b.event_offsets, b.x, b.y, b.plane, LS["params"], LS["k_max"], LS["tau"],
            LS["conf_min"], nms=LS["nms"])))
    for name, r in runs:
        for e in range(b.n_events):
            a, c = int(ref["track_offsets"][e]), int(ref["track_offsets"][e + 1])
            gt, gR = event_tracks(r, e, 2)
            assert_tracks_match(2, gt, gR, ref["theta"][a:c], ref["R"][a:c], LS["params"]["d_merge"], z0, z1)
        _say("  %s: %d tracks match" % (name, int(ref["track_offsets"][-1])))


def _mixed_batch():
    c5, c3 = events.load_config("c5"), events.load_config("c3")
    zp = events.plane_z(c3)
    evs = [events.make_event(c5, 0, zp)] + [events.make_event(c3, i, zp) for i in range(7)]
    return events.batch_from_events(2, zp, evs), learned.settings(c3)["params"]


def test_small_shape_global_keys_and_leaders(ctx, gold):
    b, P = _mixed_batch()
    seeds, soff = gold["mix_seeds"], gold["mix_soff"]
    E = b.n_events
    assert soff[-1] <= SMALL_KEYS * E                      # the small merge shape
    assert soff[1] - soff[0] > SMALL_KEYS                   # event 0: keys in the global scratch
    toff = gold["mix_toff"]
    assert toff[1] - toff[0] > SMALL_LEADERS                # event 0: leaders past the LDS cache
    _say("mixed batch: %d seeds (%d in event 0), %d clusters in event 0" % (soff[-1], soff[1], toff[1]))
    res = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P, seeds=seeds,
                                 seed_offsets=soff)
    nt = _compare(res, gold, "mix", P["d_merge"], float(b.plane_z[0]), float(b.plane_z[-1]))
    _say("  %d tracks match" % nt)


def test_large_shape_global_leaders(ctx, gold):
    c5 = events.load_config("c5")
    wide = json.loads(json.dumps(c5))
    wide["tracks"]["count"] = {"kind": "fixed", "n": 1600}
    zp = events.plane_z(c5)
    b = events.batch_from_events(2, zp, [events.make_event(wide, 100000, zp)])
    seeds, soff = gold["wide_seeds"], gold["wide_soff"]
    assert soff[-1] > SMALL_KEYS                            # the large merge shape
    assert gold["wide_toff"][-1] > MERGE_LEADERS            # leaders past the LDS cache
    P = learned.settings(c5)["params"]
    _say("1600-track event: %d hits, %d seeds, %d clusters" % (b.x.shape[0], soff[-1], gold["wide_toff"][-1]))
    res = ctx.retina_find_tracks(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, P, seeds=seeds,
                                 seed_offsets=soff)
    nt = _compare(res, gold, "wide", P["d_merge"], float(zp[0]), float(zp[-1]))
    _say("  %d tracks match" % nt)


def test_learned_batch_with_fallback_event(ctx):
    """Seven events of the 1024-event batch and one event made of another
    event's noise hits only: the network is not confident there, so that event
    takes the 64 x 64 lattice (4,096 seeds) while the batch averages fewer than
    1,024 seeds per event (small merge shape, global key sort for that event).
    The oracle runs its own proposer and the same fallback rule."""
    cfg = events.load_config("c3")
    LS = learned.settings(cfg)
    zp = events.plane_z(cfg)
    evs = [events.make_event(cfg, i, zp) for i in range(7)]
    src = events.make_event(cfg, 7, zp)
    m = src.label < 0
    evs.append(events.Event(src.x[m], src.y[m], src.plane[m], src.label[m], np.zeros((0, 4)),
                            np.zeros(0, np.int32)))
    b = events.batch_from_events(2, zp, evs)
    model = ctx.retina_model_load(LS["model"])
    layers = op.unpack_params(model.retina_model_get_params())
    lat = oracle.lattice(2, LS["params"])
    seeds, off, fb = [], [0], []
    for e, img in enumerate(_oracle_images(b)):
        _, z = op.forward(img, layers, store_bf16=True)
        picks = op.seed_bins(z, LS["tau"], LS["k_max"], nms=LS["nms"])
        f = (not picks) or z.max() < op.logit_threshold(LS["conf_min"])
        s = lat if f else op.seeds_from_pixels(picks)
        seeds.append(s)
        off.append(off[-1] + len(s))
        fb.append(f)
    assert fb == [False] * 7 + [True], "the noise-only event must be the only fallback (%s)" % fb
    assert off[-1] <= SMALL_KEYS * b.n_events and off[-1] - off[-2] > SMALL_KEYS
    _say("learned batch with a fallback event: %d seeds, %d in the fallback event" % (off[-1], off[-1] - off[-2]))
    ref = oracle.find_tracks(b, LS["params"], np.concatenate(seeds), np.array(off, np.int64))
    got = ctx.retina_find_tracks_learned(model, b.plane_z, b.event_offsets, b.x, b.y, b.plane, LS["params"],
                                         LS["k_max"], LS["tau"], LS["conf_min"], nms=LS["nms"])
    flags = np.asarray(got["event_flags"])
    assert list((flags >> 4) & 1) == [0] * 7 + [1]
    z0, z1 = float(zp[0]), float(zp[-1])
    for e in range(b.n_events):
        a, c = int(ref["track_offsets"][e]), int(ref["track_offsets"][e + 1])
        gt, gR = event_tracks(got, e, 2)
        assert_tracks_match(2, gt, gR, ref["theta"][a:c], ref["R"][a:c], LS["params"]["d_merge"], z0, z1)
    _say("  %d tracks match (fallback event: %d)" % (int(ref["track_offsets"][-1]),
                                                   int(ref["track_offsets"][-1] - ref["track_offsets"][-2])))


def _label_sets_match(tg, toff, ref):
    """Label slopes (tx, ty) per event against the oracle's track slopes: same
    count, and each pairs off with one oracle track within 1e-4 relative
    (scale floor 0.01) in both slopes."""
    for e in range(len(toff) - 1):
        g = np.asarray(tg[toff[e]:toff[e + 1]], np.float64)
        a, c = int(ref["track_offsets"][e]), int(ref["track_offsets"][e + 1])
        r = np.asarray(ref["theta"][a:c], np.float64)[:, 2:4]
        assert len(g) == len(r), "event %d: %d labels, oracle %d tracks" % (e, len(g), len(r))
        if not len(r):
            continue
        tol = 1e-4 * np.maximum(np.abs(r), 0.01)
        d = np.abs(g[:, None, :] - r[None, :, :]) <= tol[None, :, :]
        ok = d.all(axis=2)
        assert ok.any(axis=1).all() and ok.any(axis=0).all(), "event %d: unmatched labels" % e


def test_training_labels_match_oracle(ctx, gold):
    """The training labels (train_proposer.label: the slopes of the tracks the
    plain method finds with the lattice) are the oracle's maxima: three events
    of the 100k-event training workload, and event 0 of the high-multiplicity
    one (its oracle tracks from the golden file)."""
    import torch
    from paper_1709_08610_amd import train_proposer as tp
    for name, n in (("c4", 3), ("c6", 1)):
        cfg = events.load_config(name)
        b = events.make_batch(cfg, n)
        dev = tp.DeviceEvents(b.x, b.y, b.plane, b.event_offsets)
        tg, toff = tp.label(ctx, b.plane_z, dev, cfg["params"])
        torch.cuda.synchronize()
        tg, toff = tg.cpu().numpy(), toff.cpu().numpy()
        if name == "c6":
            ref = dict(track_offsets=gold["c6lab_toff"], theta=gold["c6lab_theta"])
        else:
            ref = oracle.find_tracks(b, cfg["params"])
        _label_sets_match(tg, toff, ref)
        _say("%s: %d labels on %d events match the oracle's tracks" % (name, int(toff[-1]), n))
