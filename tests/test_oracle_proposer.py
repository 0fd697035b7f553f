"""Pins of the proposer oracle (oracle/proposer.py) against textbook routines,
finite differences, closed forms and hand-worked cases."""
import numpy as np
import pytest

from oracle import proposer as op


def _rand(shape, seed):
    return np.random.default_rng(seed).normal(size=shape)


def test_conv_matches_im2col_matmul():
    x = _rand((9, 7, 5), 1)
    W = _rand((4, 9, 5), 2)
    b = _rand(4, 3)
    xp = np.zeros((11, 9, 5))
    xp[1:-1, 1:-1] = x
    cols = np.zeros((9 * 7, 9 * 5))
    for r in range(9):
        for c in range(7):
            patch = xp[r:r + 3, c:c + 3]  # rows r-1..r+1, cols c-1..c+1 -> tap = 3 dr' + dc'
            cols[r * 7 + c] = patch.reshape(9, 5).ravel()
    ref = (cols @ W.reshape(4, 45).T + b).reshape(9, 7, 4)
    np.testing.assert_allclose(op.conv3x3(x, W, b), ref, rtol=1e-12, atol=1e-12)


def test_conv_backward_finite_differences():
    x = _rand((6, 5, 3), 4)
    W = _rand((2, 9, 3), 5)
    b = _rand(2, 6)
    R = _rand((6, 5, 2), 7)
    L = lambda x_, W_, b_: float(np.sum(R * op.conv3x3(x_, W_, b_)))
    dx, dW, db = op.conv3x3_back(x, W, R)
    eps = 1e-6
    rng = np.random.default_rng(8)
    for _ in range(10):
        i = tuple(rng.integers(0, s) for s in x.shape)
        xp, xm = x.copy(), x.copy()
        xp[i] += eps
        xm[i] -= eps
        assert (L(xp, W, b) - L(xm, W, b)) / (2 * eps) == pytest.approx(dx[i], rel=1e-6, abs=1e-8)
        j = tuple(rng.integers(0, s) for s in W.shape)
        Wp, Wm = W.copy(), W.copy()
        Wp[j] += eps
        Wm[j] -= eps
        assert (L(x, Wp, b) - L(x, Wm, b)) / (2 * eps) == pytest.approx(dW[j], rel=1e-6, abs=1e-8)
    for k in range(2):
        bp, bm = b.copy(), b.copy()
        bp[k] += eps
        bm[k] -= eps
        assert (L(x, W, bp) - L(x, W, bm)) / (2 * eps) == pytest.approx(db[k], rel=1e-6)


def test_bce_hand_values_and_gradient():
    loss, g = op.bce_logits(np.array([0.0]), np.array([1.0]), 10.0)
    assert loss == pytest.approx(10 * np.log(2))
    assert g[0] == pytest.approx((10 + 0) * 0.5 - 10)
    loss, g = op.bce_logits(np.array([0.0]), np.array([0.0]), 10.0)
    assert loss == pytest.approx(np.log(2)) and g[0] == pytest.approx(0.5)
    z = _rand(50, 9)
    y = (np.random.default_rng(10).random(50) < 0.2).astype(float)
    l0, g0 = op.bce_logits(z, y, 7.0)
    eps = 1e-6
    for i in range(0, 50, 7):
        zp, zm = z.copy(), z.copy()
        zp[i] += eps
        zm[i] -= eps
        fd = (op.bce_logits(zp, y, 7.0)[0] - op.bce_logits(zm, y, 7.0)[0]) / (2 * eps)
        assert fd == pytest.approx(g0[i], rel=1e-6, abs=1e-10)


def test_adam_first_step_closed_form():
    """From zero moments the bias corrections cancel: w1 = w0 - lr g / (|g| + eps)."""
    w = _rand(20, 11)
    g = _rand(20, 12)
    w1, m1, v1 = op.adam_step(w, np.zeros(20), np.zeros(20), g, lr=1e-3, step=1)
    np.testing.assert_allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g)
    np.testing.assert_allclose(v1, 0.001 * g * g)


def test_nms_hand_cases():
    z = np.full((5, 6), -10.0)
    z[1, 1] = 3.0               # isolated peak
    z[3, 4] = 2.0
    z[3, 5] = 2.0               # plateau: the lower flat index (3, 4) wins
    z[0, 5] = 1.0               # border peak
    z[4, 0] = -1.0              # below a tau of 0.5 (logit 0)
    got = op.nms_topk(z, 0.5, 10)
    assert got == [1 * 6 + 1, 3 * 6 + 4, 0 * 6 + 5]
    assert op.nms_topk(z, 0.5, 2) == [7, 22]
    # a value exactly at the threshold is not above it
    z2 = np.full((3, 3), -5.0)
    z2[1, 1] = 0.0
    assert op.nms_topk(z2, 0.5, 5) == []


def test_bin_counts_hand_case():
    zp = np.array([100.0, 200.0, 300.0, 400.0], np.float32)
    w = 0.7 / 128
    # hits exactly at bin centres: (tx, ty) = centre of bins (10, 20) and (64, 127)
    def centre(i):
        return -0.35 + (i + 0.5) * w
    x = np.array([centre(10) * 100, centre(10) * 400, centre(64) * 200, 0.36 * 300], np.float32)
    y = np.array([centre(20) * 100, centre(20) * 400, centre(127) * 200, 0.0], np.float32)
    pl = np.array([0, 3, 1, 2], np.int32)
    cnt = op.bin_counts(x, y, pl, zp)
    assert cnt.sum() == 3                     # the last hit (slope 0.36) is out of range
    assert cnt[10, 20, 0] == 1 and cnt[10, 20, 1] == 1   # plane 0 -> group 0, plane 3 -> group 1
    assert cnt[64, 127, 0] == 1


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3], np.float32)
    r = op.bf16_round(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                           # tie -> even
    assert r[2] == 1.0 + 4 * 2 ** -8             # tie -> even (up)
    assert r[3] == -2.5
    assert abs(r[4] - 3.0e-3) <= 3.0e-3 * 2 ** -8


def test_network_gradient_finite_differences():
    """End-to-end FP64 (no BF16 storage): backward matches central differences of
    the loss on a few parameters of every layer."""
    rng = np.random.default_rng(13)
    params = [(rng.normal(0, np.sqrt(2 / (9 * ci)), (co, 9, ci)), rng.normal(0, 0.1, co))
              for ci, co in zip(op.CHANNELS[:-1], op.CHANNELS[1:])]
    img = np.zeros((128, 128, 2))
    img[40:60, 30:70] = rng.random((20, 40, 2))
    y = np.zeros((128, 128))
    y[50, 50] = 1
    y[45, 60] = 1

    def loss(ps):
        _, z = op.forward(img, ps, store_bf16=False)
        return op.bce_logits(z, y, 10.0)

    acts, z = op.forward(img, params, store_bf16=False)
    l0, dz = op.bce_logits(z, y, 10.0)
    grads = op.backward(acts, params, dz, store_bf16=False)
    eps = 1e-5
    for l in range(4):
        W, b = params[l]
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in W.shape)
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = list(params)
            pm = list(params)
            pp[l] = (Wp, b)
            pm[l] = (Wm, b)
            fd = (loss(pp)[0] - loss(pm)[0]) / (2 * eps)
            assert fd == pytest.approx(grads[l][0][idx], rel=2e-4, abs=1e-9)


def test_target_image_and_seed_centres_round_trip():
    """A seed at a bin's centre lands back in that bin; values on the edges of
    the range follow the half-open rule."""
    pix = np.array([0, 127, 128 * 64 + 5, 128 * 128 - 1])
    s = op.seeds_from_pixels(pix)
    assert np.all(s[:, :2] == 0)
    assert s[0, 2] == pytest.approx(-0.35 + 0.7 / 256, abs=1e-7)
    assert s[3, 3] == pytest.approx(0.35 - 0.7 / 256, abs=1e-7)
    y = op.target_image(s[:, 2:])
    assert y.sum() == 4 and all(y.ravel()[p] == 1 for p in pix)
    edge = op.target_image([[np.float32(0.35), 0.0], [np.float32(-0.35), 0.0]])
    assert edge.sum() == 1 and edge[0, 64] == 1


def test_topk_without_nms_is_a_sort():
    """Without suppression the selection is the k largest values above the
    threshold, ties to the lower index: a stable argsort of -z."""
    z = np.round(np.random.default_rng(3).normal(size=(12, 10)), 1)   # many ties
    thr = op.logit_threshold(0.4)
    flat = z.ravel()
    order = [i for i in np.argsort(-flat, kind="stable") if flat[i] > thr]
    assert op.nms_topk(z, 0.4, 30, nms=False) == order[:30]
    assert op.nms_topk(z, 0.4, 1000, nms=False) == order


def test_logit_threshold():
    assert op.logit_threshold(0.5) == 0.0
    assert op.logit_threshold(0.0) == -np.inf and op.logit_threshold(1.0) == np.inf
    assert op.logit_threshold(0.9) == pytest.approx(np.log(9), rel=1e-7)
    assert op.logit_threshold(0.9) == float(np.float32(op.logit_threshold(0.9)))


def test_seed_bins_are_the_selection_in_bin_order():
    z = np.round(np.random.default_rng(9).normal(size=(16, 16)), 1)
    for nms in (False, True):
        sel = op.nms_topk(z, 0.3, 20, nms=nms)
        got = op.seed_bins(z, 0.3, 20, nms=nms)
        assert got == sorted(sel) and len(got) == len(set(got))
