"""GPU parity of the learned seed proposer against the FP64 proposer oracle.

* binned images: bit-exact (same FP32 bin decision, BF16 of log1p(count));
* logits: within a forward error bound that propagates one BF16 rounding
  (2^-8 relative, doubled because two roundings of nearly equal values may
  straddle a rounding boundary) of every stored activation through the
  absolute-value network, plus FP32 accumulation;
* gradients of the mean loss: every entry within 8 standard deviations of a
  rounding model propagated through the forward and backward passes (FP32
  accumulation as sqrt(K) u of the products' root sum of squares; a stored
  BF16 value taking its neighbour with a probability set by its source's
  deviation; the loss gradient's sensitivity to the logits; ReLU masks that
  may flip where a pre-activation lies within 8 spreads of zero), a few
  percent of |g| for most entries; per-layer relative L2 below 1e-3 and
  cosine above 0.99999 as diagnostics beside it;
* seed proposal on a network whose logits are exact in FP32: bit-exact seeds,
  counts and fallback flags;
* Adam's first step against its closed form on the oracle's gradient, checkpoint save / load / resume
  bit-exact."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle
from oracle import proposer as op
from paper_1709_08610_amd import events, retina

from gpu_util import assert_tracks_match, event_tracks
from proposer_util import U_BF16, _bf16_bits_to_f64, _grad_spread, _logit_bound, _oracle_images

pytestmark = pytest.mark.gpu

INIT_KEY = 20170925
GRAD_K = 8.0   # standard deviations of the gradient rounding model allowed per entry


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


@pytest.fixture(scope="module")
def batch():
    """Three training-workload events (ragged hit counts) plus an empty event."""
    cfg = events.load_config("c4")
    evs = [events.make_event(cfg, i) for i in range(3)]
    empty = events.Event(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32),
                         np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros(0, np.int32))
    return events.batch_from_events(2, events.plane_z(cfg), evs + [empty])


def _targets(b):
    t = [np.asarray(b.truth[e], np.float64)[:, 2:4] for e in range(b.n_events)]
    off = np.concatenate([[0], np.cumsum([len(a) for a in t])]).astype(np.int64)
    return np.concatenate(t), off


# ------------------------------------------------------------------ images
def test_bin_image_exact(ctx, batch):
    _say("proposer: bin image")
    m = ctx.retina_model_create(INIT_KEY)
    img, _ = ctx.retina_model_forward(m, batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane)
    ref = _oracle_images(batch)
    for e in range(batch.n_events):
        want = op.bf16_round(ref[e])
        got = _bf16_bits_to_f64(img[e])
        assert np.array_equal(got, want), "event %d: %d bins differ" % (e, int((got != want).sum()))
    assert not _bf16_bits_to_f64(img[3]).any()


def test_bin_image_large_counts_and_events(ctx):
    """Bin counts above the 256-entry table of BF16(log1p(count)) (300 hits on
    every plane of one line through the origin: 3,900 per plane group in one
    bin) and an event of more than 65,535 hits (two passes, one per plane
    group, 16-bit counts no longer packed in pairs), against the oracle's
    binning bit for bit."""
    _say("proposer: bin image, large counts and events")
    cfg = events.load_config("c4")
    z = events.plane_z(cfg)
    P = len(z)
    rng = np.random.default_rng(23)
    w = (0.35 - (-0.35)) / 128
    tx, ty = -0.35 + 40.5 * w, -0.35 + 90.5 * w  # bin centres: every plane's hit lands in bin (40, 90)
    pl = np.repeat(np.arange(P, dtype=np.int32), 300)
    zz = z[pl].astype(np.float64)
    line = events.Event((tx * zz).astype(np.float32), (ty * zz).astype(np.float32), pl,
                        np.zeros(len(pl), np.int32), np.array([[0.0, 0.0, tx, ty]]), np.array([len(pl)], np.int32))
    n = 70_000
    pl2 = np.sort(rng.integers(0, P, n)).astype(np.int32)
    z2 = z[pl2].astype(np.float64)
    wide = events.Event((rng.uniform(-0.34, 0.34, n) * z2).astype(np.float32),
                        (rng.uniform(-0.34, 0.34, n) * z2).astype(np.float32), pl2,
                        np.full(n, -1, np.int32), np.zeros((0, 4)), np.zeros(0, np.int32))
    b = events.batch_from_events(2, z, [line, wide])
    m = ctx.retina_model_create(INIT_KEY)
    img, _ = ctx.retina_model_forward(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane)
    ref = _oracle_images(b)
    cnt = op.bin_counts(*(lambda ev: (ev.x, ev.y, ev.plane))(b.event(0)), b.plane_z)
    assert cnt.max() > 255, "the line's bin should exceed the table"
    assert b.event_offsets[2] - b.event_offsets[1] > 0xFFFF
    for e in range(b.n_events):
        want = op.bf16_round(ref[e])
        got = _bf16_bits_to_f64(img[e])
        assert np.array_equal(got, want), "event %d: %d bins differ" % (e, int((got != want).sum()))


def test_model_params_round_trip(ctx):
    m = ctx.retina_model_create(INIT_KEY)
    p = m.retina_model_get_params()
    assert p.shape == (retina.MODEL_PARAMS,) and np.isfinite(p).all()
    layers = op.unpack_params(p)
    for l, (W, bb) in enumerate(layers):
        sd = np.sqrt(2.0 / (9 * op.CHANNELS[l]))
        assert abs(W.std() / sd - 1) < 0.1 and abs(W.mean()) < 0.1 * sd
        assert np.all(bb == (0 if l < 3 else np.float32(np.log(0.01 / 0.99))))
    q = np.random.default_rng(1).normal(size=p.shape).astype(np.float32)
    m.retina_model_set_params(q)
    assert np.array_equal(m.retina_model_get_params(), q)
    m2 = ctx.retina_model_create(INIT_KEY)
    assert np.array_equal(m2.retina_model_get_params(), p)   # same key, same weights


# ------------------------------------------------------------------ forward
def test_forward_logits_parity(ctx, batch):
    _say("proposer: forward logits")
    m = ctx.retina_model_create(INIT_KEY)
    # a model with non-trivial biases so every layer's bias path is exercised
    p = m.retina_model_get_params()
    rng = np.random.default_rng(7)
    layers = op.unpack_params(p)
    q = np.concatenate([np.concatenate([W.ravel(), rng.normal(0, 0.05, bb.shape)]) for W, bb in layers])
    m.retina_model_set_params(q.astype(np.float32))
    params = op.unpack_params(m.retina_model_get_params())
    _, logits = ctx.retina_model_forward(m, batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane)
    for e, img in enumerate(_oracle_images(batch)):
        _, zr = op.forward(img, params, store_bf16=True)
        bound = _logit_bound(img, params)
        d = np.abs(logits[e].astype(np.float64) - zr)
        bad = d > 1.5 * bound + 1e-6
        assert not bad.any(), "event %d: %d logits outside the bound (max excess %g)" % (
            e, int(bad.sum()), float((d - 1.5 * bound).max()))
        rel = np.linalg.norm(d) / np.linalg.norm(zr)
        assert rel < 1e-3, "event %d: relative L2 error %g" % (e, rel)


def test_forward_logits_many_bands_per_work_group(ctx):
    """40 events: 1280 bands of four rows over at most 256 persistent
    work-groups, so a work-group runs several consecutive bands (taking the
    act1 rows a band shares with the previous one of its event) and some
    cross an event boundary.  Every event's logits equal, bit for bit, those
    of the event run alone (one band per work-group), and three events stay
    within the oracle's bound."""
    _say("proposer: forward logits, consecutive bands per work-group")
    cfg = events.load_config("c4")
    evs = [events.make_event(cfg, 100 + i) for i in range(40)]
    evs[17] = events.Event(np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.int32),
                           np.zeros(0, np.int32), np.zeros((0, 4)), np.zeros(0, np.int32))
    z = events.plane_z(cfg)
    big = events.batch_from_events(2, z, evs)
    m = ctx.retina_model_create(INIT_KEY)
    p = m.retina_model_get_params()
    rng = np.random.default_rng(11)
    layers = op.unpack_params(p)
    q = np.concatenate([np.concatenate([W.ravel(), rng.normal(0, 0.05, bb.shape)]) for W, bb in layers])
    m.retina_model_set_params(q.astype(np.float32))
    params = op.unpack_params(m.retina_model_get_params())
    _, logits = ctx.retina_model_forward(m, big.plane_z, big.event_offsets, big.x, big.y, big.plane)
    for e in range(len(evs)):
        one = events.batch_from_events(2, z, [evs[e]])
        _, l1 = ctx.retina_model_forward(m, one.plane_z, one.event_offsets, one.x, one.y, one.plane)
        assert np.array_equal(logits[e].view(np.uint32), l1[0].view(np.uint32)), \
            "event %d: logits differ from the event run alone (%d entries)" % (e, int((logits[e] != l1[0]).sum()))
    imgs = _oracle_images(big)
    for e in (0, 17, 39):
        _, zr = op.forward(imgs[e], params, store_bf16=True)
        bound = _logit_bound(imgs[e], params)
        d = np.abs(logits[e].astype(np.float64) - zr)
        assert not (d > 1.5 * bound + 1e-6).any(), "event %d: logits outside the bound" % e


# ------------------------------------------------------------------ gradients
def _oracle_loss_grad(b, params, pos_weight, want_bound=False):
    """Loss and gradient of the FP64 oracle; with want_bound also the
    elementwise bar for the device's deviation: GRAD_K standard deviations of
    the propagated rounding model (proposer_util._grad_spread), plus a floor of
    1e-9 of the largest gradient entry."""
    tg, toff = _targets(b)
    imgs = _oracle_images(b)
    outs = [op.forward(img, params, store_bf16=True) for img in imgs]
    z = np.stack([o[1] for o in outs])
    y = np.stack([op.target_image(tg[toff[e]:toff[e + 1]]) for e in range(b.n_events)])
    loss, dz = op.bce_logits(z, y, pos_weight)
    grads = None
    for e, (acts, _) in enumerate(outs):
        g = op.backward(acts, params, dz[e], store_bf16=True)
        grads = g if grads is None else [(a[0] + c[0], a[1] + c[1]) for a, c in zip(grads, g)]
    g = op.pack_grads(grads)
    bound = None
    if want_bound:
        bound = GRAD_K * _grad_spread(imgs, list(y), params, pos_weight, z.size, k=GRAD_K) + 1e-9 * np.abs(g).max()
    return loss, g, y, bound


def _layer_slices():
    out, q = [], 0
    for l in range(4):
        ci, co = op.CHANNELS[l], op.CHANNELS[l + 1]
        out.append((slice(q, q + 9 * ci * co), slice(q + 9 * ci * co, q + 9 * ci * co + co)))
        q += 9 * ci * co + co
    return out


def test_train_step_gradient_parity(ctx, batch):
    _say("proposer: gradient")
    pw = 20.0
    m = ctx.retina_model_create(INIT_KEY)
    p0 = m.retina_model_get_params()
    params = op.unpack_params(p0)
    tg, toff = _targets(batch)
    loss, grad = ctx.retina_train_step(m, batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane,
                                       tg, toff, 0.0, pw, want_grad=True)
    assert m.step == 0
    lref, gref, y, bound = _oracle_loss_grad(batch, params, pw, want_bound=True)
    assert y.sum() > 100
    assert loss == pytest.approx(lref, rel=1e-3)
    g = grad.astype(np.float64)
    # every gradient entry within GRAD_K standard deviations of the propagated
    # rounding model (a few percent of |g| for most entries): a wrong index,
    # sign or transposition breaks it by O(|g|)
    d = np.abs(g - gref)
    bad = d > bound
    for l, (sw, sb) in enumerate(_layer_slices()):
        for name, s in (("W", sw), ("b", sb)):
            a, r = g[s], gref[s]
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r))
            _say("  layer %d %s: %d entries, outside the bound %d, max |d|/bound %.3f, rel L2 %.2e cos %.7f" % (
                l, name, a.size, int(bad[s].sum()), float((d[s] / np.maximum(bound[s], 1e-300)).max()), rel, cos))
    assert not bad.any(), "%d gradient entries outside the bound (first %s)" % (int(bad.sum()), np.nonzero(bad)[0][:8])
    # diagnostics beside the elementwise bar
    for l, (sw, sb) in enumerate(_layer_slices()):
        for name, s in (("W", sw), ("b", sb)):
            a, r = g[s], gref[s]
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r))
            assert rel < 1e-3 and cos > 0.99999, "layer %d %s: rel %g cos %g" % (l, name, rel, cos)
    # an lr = 0 call leaves the weights alone
    assert np.array_equal(m.retina_model_get_params(), p0)


def test_adam_first_step_closed_form(ctx, batch):
    """From zero moments Adam's first step is lr g / (|g| + eps) (bias
    corrections cancel), with g the oracle's gradient: wherever the oracle's
    gradient exceeds the device's error bound (so its sign is certain) the
    weight moves by lr g / (|g| + eps) up to that bound's effect; elsewhere
    by at most lr.  The device's own gradient gives the same step to FP32
    rounding."""
    _say("proposer: adam step")
    lr, pw = 1e-3, 20.0
    m = ctx.retina_model_create(INIT_KEY)
    w0 = m.retina_model_get_params().astype(np.float64)
    params = op.unpack_params(w0)
    tg, toff = _targets(batch)
    _, g = ctx.retina_train_step(m, batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane,
                                 tg, toff, 0.0, pw, want_grad=True)
    ctx.retina_train_step(m, batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane,
                          tg, toff, lr, pw)
    assert m.step == 1
    w1 = m.retina_model_get_params().astype(np.float64)
    ulp = 2 * np.abs(w0).max() * 2 ** -24
    _, gref, _, bound = _oracle_loss_grad(batch, params, pw, want_bound=True)
    eps = 1e-8
    sure = np.abs(gref) > bound
    assert sure.mean() > 0.9
    want = w0 - lr * gref / (np.abs(gref) + eps)
    # d/dg [g / (|g| + eps)] = eps / (|g| + eps)^2: the step moves by at most
    # lr eps dg / (|g| - dg + eps)^2 where the gradient is off by dg
    dg = bound
    tol = lr * eps * dg / np.maximum(np.abs(gref) - dg + eps, eps) ** 2 + 4e-6 * lr + ulp
    np.testing.assert_array_less(np.abs(w1 - want)[sure], tol[sure])
    assert np.all(np.abs(w1 - w0) <= lr * (1 + 1e-5) + ulp)
    np.testing.assert_allclose(w1, w0 - lr * g / (np.abs(g.astype(np.float64)) + eps), rtol=0,
                               atol=4e-6 * lr + ulp)


def test_training_reduces_loss(ctx, batch):
    _say("proposer: training")
    m = ctx.retina_model_create(INIT_KEY)
    tg, toff = _targets(batch)
    args = (batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane, tg, toff)
    losses = [ctx.retina_train_step(m, *args, 1e-3, 20.0)[0] for _ in range(30)]
    _say("  loss %.4f -> %.4f" % (losses[0], losses[-1]))
    assert m.step == 30
    assert losses[-1] < 0.5 * losses[0]


def test_save_load_resume_bit_exact(ctx, batch):
    _say("proposer: save/load")
    tg, toff = _targets(batch)
    args = (batch.plane_z, batch.event_offsets, batch.x, batch.y, batch.plane, tg, toff)
    m = ctx.retina_model_create(INIT_KEY)
    for _ in range(2):
        ctx.retina_train_step(m, *args, 1e-3, 20.0)
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "m.bin")
        m.retina_model_save(path)
        m2 = ctx.retina_model_load(path)
        assert m2.step == 2
        assert np.array_equal(m2.retina_model_get_params(), m.retina_model_get_params())
        l1 = ctx.retina_train_step(m, *args, 1e-3, 20.0)[0]
        l2 = ctx.retina_train_step(m2, *args, 1e-3, 20.0)[0]
        assert l1 == l2
        assert np.array_equal(m2.retina_model_get_params(), m.retina_model_get_params())
        raw = bytearray(open(path, "rb").read())
        raw[100] ^= 1
        open(path, "wb").write(bytes(raw))
        with pytest.raises(retina.RetinaError, match="checksum"):
            ctx.retina_model_load(path)


# ------------------------------------------------------------------ proposal
def _exact_net(bias=-3.0):
    """Weights under which the logits are exact in FP32: the centre taps carry
    channel 0 + channel 1 through three ReLU layers, the last bias is `bias`,
    so logit = bf16(img0 + img1) + bias at every bin."""
    layers = []
    for l in range(4):
        ci, co = op.CHANNELS[l], op.CHANNELS[l + 1]
        W = np.zeros((co, 9, ci))
        W[0, 4, 0] = 1.0
        if l == 0:
            W[0, 4, 1] = 1.0
        b = np.zeros(co)
        if l == 3:
            b[0] = bias
        layers.append((W, b))
    return layers


def _pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)


@pytest.fixture(scope="module")
def prop_batch():
    """Two training-workload events, an empty event and a one-hit event."""
    cfg = events.load_config("c4")
    evs = [events.make_event(cfg, 10 + i) for i in range(2)]
    z = np.zeros(0)
    empty = events.Event(z.astype(np.float32), z.astype(np.float32), z.astype(np.int32), z.astype(np.int32),
                         np.zeros((0, 4)), z.astype(np.int32))
    one = events.Event(np.array([3.0], np.float32), np.array([-2.0], np.float32), np.array([7], np.int32),
                       np.array([-1], np.int32), np.zeros((0, 4)), z.astype(np.int32))
    return events.batch_from_events(2, events.plane_z(cfg), evs + [empty, one])


TAU, CONF_MIN, K_MAX = 0.07, 0.11, 48


def _oracle_seeds(b, layers, lattice_params, nms, k_max=K_MAX, tau=TAU, conf_min=CONF_MIN):
    seeds, off, conf, fb = [], [0], [], []
    lat = oracle.lattice(2, lattice_params)
    for e, img in enumerate(_oracle_images(b)):
        _, z = op.forward(img, layers, store_bf16=True)
        picks = op.seed_bins(z, tau, k_max, nms=nms)
        conf.append(1.0 / (1.0 + np.exp(-z.max())))
        if not picks or z.max() < op.logit_threshold(conf_min):
            fb.append(1)
            s = lat
        else:
            fb.append(0)
            s = op.seeds_from_pixels(picks)
        seeds.append(s)
        off.append(off[-1] + len(s))
    return np.concatenate(seeds), np.array(off, np.int64), np.array(conf), np.array(fb)


@pytest.mark.parametrize("nms", [True, False])
def test_propose_seeds_exact(ctx, prop_batch, nms):
    _say("proposer: seeds nms=%d" % nms)
    b = prop_batch
    params = dict(events.load_config("c4")["params"])
    layers = _exact_net()
    m = ctx.retina_model_create(INIT_KEY)
    m.retina_model_set_params(_pack(layers))
    _, logits = ctx.retina_model_forward(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane)
    # the logits are exact: the oracle's FP64 values are the same numbers
    for e, img in enumerate(_oracle_images(b)):
        assert np.array_equal(logits[e].astype(np.float64), op.forward(img, layers)[1])
    res = ctx.retina_propose_seeds(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane, K_MAX, TAU, CONF_MIN, params,
                                   nms=nms)
    s_ref, off_ref, conf_ref, fb_ref = _oracle_seeds(b, layers, params, nms)
    assert list(fb_ref) == [0, 0, 1, 1]
    np.testing.assert_array_equal(res["fallback"], fb_ref)
    np.testing.assert_array_equal(res["seed_offsets"], off_ref)
    np.testing.assert_array_equal(res["seeds"], s_ref)
    np.testing.assert_allclose(res["confidence"], conf_ref, rtol=1e-6)
    # too small a buffer reports the size it needs
    with pytest.raises(retina.RetinaError) as ei:
        ctx.retina_propose_seeds(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane, K_MAX, TAU, CONF_MIN,
                                 params, capacity=5, nms=nms)
    assert ei.value.code == retina.ERR_CAPACITY and ei.value.required == off_ref[-1]


@pytest.mark.parametrize("k_max", [4096, 77])
def test_propose_seeds_more_candidates_than_fit(ctx, prop_batch, k_max):
    """Every bin above the threshold (16,384 candidates, long runs of equal
    logits): the selection of the k_max best must still follow (score desc,
    index asc) exactly."""
    _say("proposer: selection overflow k_max=%d" % k_max)
    b = prop_batch
    params = dict(events.load_config("c4")["params"])
    layers = _exact_net(bias=3.0)
    m = ctx.retina_model_create(INIT_KEY)
    m.retina_model_set_params(_pack(layers))
    res = ctx.retina_propose_seeds(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane, k_max, TAU, CONF_MIN, params,
                                   nms=False)
    s_ref, off_ref, _, fb_ref = _oracle_seeds(b, layers, params, False, k_max=k_max)
    assert not fb_ref.any()
    np.testing.assert_array_equal(res["seed_offsets"], off_ref)
    np.testing.assert_array_equal(res["seeds"], s_ref)


def test_find_tracks_learned_parity(ctx, prop_batch):
    """Algorithm 1 on the proposer's seeds (device hand-off) against the oracle
    on the oracle's seeds."""
    _say("proposer: learned find_tracks")
    b = prop_batch
    cfg = events.load_config("c4")
    params = dict(cfg["params"])
    params.update(sigma=[2.0, 1.0, 0.5, 0.25, 0.125, 0.0625], n_slope_steps=3)
    layers = _exact_net()
    m = ctx.retina_model_create(INIT_KEY)
    m.retina_model_set_params(_pack(layers))
    res = ctx.retina_find_tracks_learned(m, b.plane_z, b.event_offsets, b.x, b.y, b.plane, params,
                                         K_MAX, TAU, CONF_MIN, nms=True)
    s_ref, off_ref, _, fb_ref = _oracle_seeds(b, layers, params, True)
    ref = oracle.find_tracks(b, params, s_ref, off_ref)
    assert list((res["event_flags"] >> 4) & 1) == list(fb_ref)
    z0, z1 = float(b.plane_z[0]), float(b.plane_z[-1])
    for e in range(b.n_events):
        a, c = int(ref["track_offsets"][e]), int(ref["track_offsets"][e + 1])
        gt, gR = event_tracks(res, e, 2)
        assert_tracks_match(2, gt, gR, ref["theta"][a:c], ref["R"][a:c], params["d_merge"], z0, z1)
    assert int(res["track_offsets"][2]) > 50
