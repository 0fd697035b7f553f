"""Edge cases of the learned-seed entry points: a bin holding more hits than a
16-bit count, empty batches, and arguments rejected before any work."""
import ctypes
import sys

import numpy as np
import pytest

from oracle import proposer as op
from paper_1709_08610_amd import events, retina

from proposer_util import _bf16_bits_to_f64

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    return retina.Context(0)


@pytest.fixture(scope="module")
def model(ctx):
    return ctx.retina_model_create(7)


def _zp():
    return events.plane_z(events.load_config("c4"))


def test_bin_counts_beyond_16_bits(ctx, model):
    """70,000 hits in one slope bin of the first plane group and 3 in the second:
    the count must not spill into the other channel."""
    _say("proposer edges: bin overflow")
    zp = _zp()
    n = 70000
    x = np.full(n + 3, np.float32(0.1) * zp[2], np.float32)
    y = np.full(n + 3, np.float32(-0.05) * zp[2], np.float32)
    plane = np.full(n + 3, 2, np.int32)
    plane[-3:] = 20
    x[-3:] = np.float32(0.2) * zp[20]
    y[-3:] = np.float32(0.0)
    off = np.array([0, n + 3], np.int64)
    img, _ = ctx.retina_model_forward(model, zp, off, x, y, plane)
    want = op.bf16_round(op.bin_image(x, y, plane, zp))
    got = _bf16_bits_to_f64(img[0])
    assert np.array_equal(got, want)
    cnt = op.bin_counts(x, y, plane, zp)
    assert cnt.max() == n and cnt[..., 1].sum() == 3


def test_empty_batches(ctx, model):
    _say("proposer edges: empty batches")
    params = events.load_config("c4")["params"]
    zp = _zp()
    z = np.zeros(0, np.float32)
    off = np.zeros(1, np.int64)
    res = ctx.retina_propose_seeds(model, zp, off, z, z, z.astype(np.int32), 16, 0.5, 0.5, params)
    assert res["seed_offsets"].tolist() == [0] and res["seeds"].shape[0] == 0
    out = ctx.retina_find_tracks_learned(model, zp, off, z, z, z.astype(np.int32), params, 16, 0.5, 0.5)
    assert out["track_offsets"].tolist() == [0]


def test_invalid_arguments_are_rejected(ctx, model):
    _say("proposer edges: invalid arguments")
    cfg = events.load_config("c4")
    params = cfg["params"]
    b = events.make_batch(cfg, 1)
    args = (b.plane_z, b.event_offsets, b.x, b.y, b.plane)
    for k_max, tau, conf in ((0, 0.5, 0.5), (4097, 0.5, 0.5), (16, 0.0, 0.5), (16, 1.0, 0.5), (16, 0.5, 1.5)):
        with pytest.raises(retina.RetinaError) as ei:
            ctx.retina_propose_seeds(model, *args, k_max, tau, conf, params)
        assert ei.value.code == retina.ERR_INVALID_ARG
    # nms must be 0 or 1 (raw call)
    g, zk = ctx._geometry(2, b.plane_z)
    hits, keep, _ = ctx._hits(2, b.event_offsets, b.x, b.y, b.plane)
    P, pk, _ = ctx._params(params, None, None, retina.MEM_HOST, 4, 1)
    pr = retina.Proposal(16, 0.5, 0.5, 2)
    seeds = np.zeros((4096, 4))
    so = np.zeros(2, np.int64)
    rc = ctx.lib.retina_propose_seeds(ctx.h, ctypes.byref(g), ctypes.byref(hits), model.h, ctypes.byref(pr),
                                      ctypes.byref(P), retina._ptr(seeds), 4096, retina._ptr(so), None, None)
    assert rc == retina.ERR_INVALID_ARG and "nms" in ctx.lib.retina_last_error(ctx.h).decode()
    # the proposer needs two measured coordinates (raw call with meas_dim 1)
    c1 = events.load_config("c1")
    b1 = events.make_batch(c1, 1)
    g1, zk1 = ctx._geometry(1, b1.plane_z)
    hits1, keep1, _ = ctx._hits(1, b1.event_offsets, b1.x, None, b1.plane)
    rc = ctx.lib.retina_model_forward(ctx.h, model.h, ctypes.byref(g1), ctypes.byref(hits1), None, None)
    assert rc == retina.ERR_INVALID_ARG and "meas_dim 2" in ctx.lib.retina_last_error(ctx.h).decode()
    # a parameter vector of the wrong length / non-finite values
    with pytest.raises(ValueError):
        model.retina_model_set_params(np.zeros(10, np.float32))
    bad = model.retina_model_get_params()
    bad[5] = np.nan
    with pytest.raises(retina.RetinaError):
        model.retina_model_set_params(bad)
