"""FP64 oracle of the learned seed proposer (test infrastructure only).

Plain numpy, direct definitions:
  * bin_image      slope histogram (x/z, y/z) -> log1p counts, two plane groups;
                   the bin index is decided in FP32 exactly as a kernel would
                   (same operations, same order), the rest in FP64
  * conv3x3        zero-padded 3x3 correlation, out[r, c, co] =
                   b[co] + sum_{dr, dc, ci} in[r + dr, c + dc, ci] W[co, tap, ci]
                   with tap = 3 (dr + 1) + (dc + 1)
  * conv3x3_back   gradients of a scalar loss through conv3x3
  * bce_logits     weighted binary cross-entropy on logits, mean over pixels
  * adam_step      Kingma & Ba's update with bias correction
  * nms_topk       bins above a threshold (optionally strict 3x3 local
                   maxima), best k
  * seed_bins      those bins in bin order (the order seeds are handed to
                   the ascent)
  * target_image / seeds_from_pixels   slope pair <-> bin maps
  * forward / backward of the four-layer network, optionally rounding the
    stored activations and gradients to BF16 where the device stores them

No code is shared with the HIP library.
"""
from __future__ import annotations

import numpy as np

IMG = 128
CHANNELS = (2, 64, 128, 96, 1)
SLOPE_LO, SLOPE_HI = -0.35, 0.35


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    a32 = np.asarray(a, np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bin_counts(x, y, plane, plane_z):
    """[128, 128, 2] integer counts of hits per slope bin and plane group."""
    P = len(plane_z)
    z = np.asarray(plane_z, np.float32)[plane]
    lo = np.float32(SLOPE_LO)
    w = np.float32((np.float32(SLOPE_HI) - lo) / np.float32(IMG))
    u = (np.asarray(x, np.float32) / z - lo) / w
    v = (np.asarray(y, np.float32) / z - lo) / w
    ok = (u >= 0) & (u < IMG) & (v >= 0) & (v < IMG)
    ch = (np.asarray(plane) >= P // 2).astype(np.int64)
    cnt = np.zeros((IMG, IMG, 2), np.int64)
    np.add.at(cnt, (u[ok].astype(np.int64), v[ok].astype(np.int64), ch[ok]), 1)
    return cnt


def bin_image(x, y, plane, plane_z):
    return np.log1p(bin_counts(x, y, plane, plane_z).astype(np.float64))


def target_image(targets):
    """[128, 128] 0/1 image with a 1 at the bin of every (tx, ty) pair (FP64 bin
    decision; pairs outside the image range are dropped)."""
    lo = float(np.float32(SLOPE_LO))
    w = (float(np.float32(SLOPE_HI)) - lo) / IMG
    t = np.asarray(targets, np.float64).reshape(-1, 2)
    u = (t[:, 0] - lo) / w
    v = (t[:, 1] - lo) / w
    ok = (u >= 0) & (u < IMG) & (v >= 0) & (v < IMG)
    y = np.zeros((IMG, IMG))
    y[u[ok].astype(np.int64), v[ok].astype(np.int64)] = 1.0
    return y


def seeds_from_pixels(pix):
    """Seeds (x0, y0, tx, ty) = (0, 0, bin centre) of flat pixel indices, the
    centre computed in FP64 and rounded to FP32."""
    lo = float(np.float32(SLOPE_LO))
    w = (float(np.float32(SLOPE_HI)) - lo) / IMG
    pix = np.asarray(pix, np.int64)
    out = np.zeros((pix.shape[0], 4))
    out[:, 2] = np.float32(lo + (pix // IMG + 0.5) * w)
    out[:, 3] = np.float32(lo + (pix % IMG + 0.5) * w)
    return out


def conv3x3(x, W, b):
    """x [H, W, Cin], W [Cout, 9, Cin], b [Cout] -> [H, W, Cout] (FP64)."""
    H, Wd, Cin = x.shape
    xp = np.zeros((H + 2, Wd + 2, Cin))
    xp[1:-1, 1:-1] = x
    out = np.broadcast_to(np.asarray(b, np.float64), (H, Wd, W.shape[0])).copy()
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            tap = 3 * (dr + 1) + (dc + 1)
            shifted = xp[1 + dr:1 + dr + H, 1 + dc:1 + dc + Wd]
            out += shifted @ W[:, tap, :].T
    return out


def conv3x3_back(x, W, dy):
    """Given dL/dy, return (dL/dx, dL/dW, dL/db) of y = conv3x3(x, W, b)."""
    H, Wd, Cin = x.shape
    xp = np.zeros((H + 2, Wd + 2, Cin))
    xp[1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W, dtype=np.float64)
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            tap = 3 * (dr + 1) + (dc + 1)
            sl = (slice(1 + dr, 1 + dr + H), slice(1 + dc, 1 + dc + Wd))
            dxp[sl] += dy @ W[:, tap, :]
            dW[:, tap, :] = dy.reshape(-1, dy.shape[-1]).T @ xp[sl].reshape(-1, Cin)
    return dxp[1:-1, 1:-1], dW, dy.sum(axis=(0, 1))


def bce_logits(z, y, pos_weight):
    """Mean of w y softplus(-z) + (1 - y) softplus(z) and its gradient."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    sp = np.logaddexp(0.0, z)       # softplus(z)
    spn = np.logaddexp(0.0, -z)     # softplus(-z)
    n = z.size
    loss = np.sum(pos_weight * y * spn + (1 - y) * sp) / n
    sig = 1.0 / (1.0 + np.exp(-z))
    grad = ((pos_weight * y + 1 - y) * sig - pos_weight * y) / n
    return loss, grad


def adam_step(w, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return w, m, v


def logit_threshold(p):
    """logit(p) computed in FP64 and rounded to FP32: the threshold a bin's
    FP32 logit is compared with (p = 0 and 1 give -inf and +inf)."""
    if p <= 0:
        return -np.inf
    if p >= 1:
        return np.inf
    return float(np.float32(np.log(p / (1 - p))))


def nms_topk(z, tau, k_max, nms=True):
    """Candidate bins: logit above logit_threshold(tau) and, with nms, above
    every 8-neighbour (equal neighbours: the lower flat index wins); the best
    k_max by value (ties: lower index).  Returns flat indices."""
    z = np.asarray(z)
    H, Wd = z.shape
    thr = logit_threshold(tau)
    cands = []
    for r in range(H):
        for c in range(Wd):
            v = z[r, c]
            if not v > thr:
                continue
            peak = True
            for dr in (-1, 0, 1):
                for dc in (-1, 0, 1):
                    if not nms or (dr == 0 and dc == 0):
                        continue
                    rr, cc = r + dr, c + dc
                    if 0 <= rr < H and 0 <= cc < Wd:
                        u = z[rr, cc]
                        j = rr * Wd + cc
                        if u > v or (u == v and j < r * Wd + c):
                            peak = False
            if peak:
                cands.append((-float(v), r * Wd + c))
    cands.sort()
    return [i for _, i in cands[:k_max]]


def seed_bins(z, tau, k_max, nms=True):
    """The proposal's seed bins: the set nms_topk selects, emitted in ascending
    bin index (tx bin major), so that consecutive seeds are neighbours in tx."""
    return sorted(nms_topk(z, tau, k_max, nms))


def unpack_params(flat):
    """Logical flat parameter vector -> list of (W [Cout, 9, Cin], b [Cout])."""
    out, q = [], 0
    for l in range(4):
        cin, cout = CHANNELS[l], CHANNELS[l + 1]
        W = np.asarray(flat[q:q + cout * 9 * cin], np.float64).reshape(cout, 9, cin)
        q += cout * 9 * cin
        b = np.asarray(flat[q:q + cout], np.float64)
        q += cout
        out.append((W, b))
    return out


def pack_grads(grads):
    return np.concatenate([np.concatenate([dW.ravel(), db.ravel()]) for dW, db in grads])


def forward(image, params, store_bf16=True):
    """Four-layer network on one image [128, 128, 2].  With store_bf16 the
    input, weights and the stored post-ReLU activations are BF16 values (the
    device's storage points); arithmetic stays FP64.  Returns (acts, logits)."""
    q = bf16_round if store_bf16 else (lambda a: np.asarray(a, np.float64))
    acts = [q(image)]
    for l, (W, b) in enumerate(params):
        y = conv3x3(acts[-1], q(W), np.asarray(b, np.float32).astype(np.float64))
        if l < 3:
            acts.append(q(np.maximum(y, 0.0)))
        else:
            logits = y[..., 0]
    return acts, logits


def backward(acts, params, dlogits, store_bf16=True):
    """Gradients of the loss given dL/dlogits; dz (gradient w.r.t. each layer's
    pre-activation) is stored in BF16 where the device stores it."""
    q = bf16_round if store_bf16 else (lambda a: np.asarray(a, np.float64))
    grads = [None] * 4
    dz = q(dlogits[..., None])
    for l in range(3, -1, -1):
        W, _ = params[l]
        dx, dW, db = conv3x3_back(acts[l], q(W), dz)
        grads[l] = (dW, db)
        if l > 0:
            dz = q(dx * (acts[l] > 0))
    return grads
