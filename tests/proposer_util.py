"""Helpers shared by the proposer GPU tests (oracle-side computations only)."""
import numpy as np

from oracle import proposer as op

U_BF16 = 2.0 ** -8


def _bf16_bits_to_f64(u16):
    return (np.asarray(u16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _oracle_images(b):
    return [op.bin_image(*(lambda ev: (ev.x, ev.y, ev.plane))(b.event(e)), b.plane_z) for e in range(b.n_events)]


def _logit_bound(img, params):
    """Elementwise bound on |logits_gpu - logits_oracle|: one BF16 rounding
    (2^-8 relative, doubled for two roundings of nearly equal values that may
    straddle a rounding boundary) of every stored activation, propagated
    through the absolute-value network, plus FP32 accumulation error."""
    acts, _ = op.forward(img, params, store_bf16=True)
    absW = [(np.abs(op.bf16_round(W)), np.zeros_like(bb)) for W, bb in params]
    err = np.zeros_like(acts[0])
    mag = np.abs(acts[0])
    for l in range(4):
        err = op.conv3x3(err, absW[l][0], absW[l][1])
        mag = op.conv3x3(mag, absW[l][0], np.abs(np.asarray(params[l][1], np.float64)))
        err = err + 1e-5 * mag                           # FP32 accumulation (K <= 1152)
        if l < 3:
            err = err + 2 * U_BF16 * acts[l + 1]         # rounding of the stored activation
            mag = acts[l + 1]
    return err[..., 0]




def _round_var(v_pre, s):
    """Variance of the deviation of a stored BF16 value whose FP32 source
    deviates with variance v_pre from the oracle's (FP64) one: the two round to
    different neighbours with probability about sqrt(v_pre) / ulp, and then
    differ by about one ulp (ulp = 2^-7 |s|); never more than v_pre + ulp^2."""
    ulp = 2 * U_BF16 * np.abs(s)
    return v_pre + np.minimum(np.sqrt(v_pre) * ulp, ulp ** 2)


def _act_spread(img, params):
    """Oracle activations (BF16 at the storage points), pre-activations and the
    variance of the device's deviation from each of them, treating the
    deviations as independent zero-mean errors: an FP32 accumulation over K
    products deviates by about sqrt(K) u of their root sum of squares, a
    deviation travels through a layer as the root sum of squares of the
    weighted deviations, and a stored BF16 value takes the neighbouring value
    with a probability set by its source's deviation (_round_var).  Returns
    (acts, pre, var) with var[l] for stored activation l (l = 0: the image,
    exact) and var[4] for the logits."""
    acts, _ = op.forward(img, params, store_bf16=True)
    Wq = [op.bf16_round(W) for W, _ in params]
    pre = [None] + [op.conv3x3(acts[l], Wq[l], np.asarray(params[l][1], np.float32).astype(np.float64))
                    for l in range(4)]
    u32 = 2.0 ** -24
    var = [np.zeros_like(acts[0])]
    for l in range(4):
        W2 = Wq[l] ** 2
        zero_b = np.zeros(W2.shape[0])
        K = 9 * W2.shape[2]
        v = op.conv3x3(var[l], W2, zero_b) + K * u32 ** 2 * op.conv3x3(acts[l] ** 2, W2, zero_b)
        if l < 3:
            v = _round_var(v * (pre[l + 1] > 0), acts[l + 1])
        var.append(v)
    return acts, pre, var


def _grad_spread(imgs, targets, params, pos_weight, n_total, k=8.0, chunk_pixels=2048):
    """Standard deviation of grad_gpu - grad_oracle of the mean weighted BCE
    over a batch (n_total pixels), propagated backward like _act_spread:
      * the logits deviate with the forward spread; dL/dz = ((w y + 1 - y)
        sigmoid(z) - w y) / n has slope at most (w y + 1 - y) / (4 n) in z,
        plus its FP32 evaluation; then the stored BF16 value (_round_var);
      * a weight gradient sum_pixels x dz deviates by the root sum of squares
        of x e_dz and e_x dz, plus FP32 accumulation over the pixels;
      * the data gradient (W^T dz, masked by the ReLU of the layer below)
        deviates by the root sum of squares of W e_dz plus accumulation, and by
        its whole value wherever the device's activation may lie on the other
        side of zero (|pre-activation| within k spreads), then the stored BF16
        value.
    Returns the flat spread (standard deviation) in the logical layout."""
    u32 = 2.0 ** -24
    Wq = [op.bf16_round(W) for W, _ in params]
    W2 = [W ** 2 for W in Wq]
    vsum = None
    for img, y in zip(imgs, targets):
        acts, pre, var = _act_spread(img, params)
        z = pre[4][..., 0]
        wy = pos_weight * y + 1.0 - y
        sig = 1.0 / (1.0 + np.exp(-z))
        dz = op.bf16_round((wy * sig - pos_weight * y) / n_total)
        v_pre = (wy / (4.0 * n_total)) ** 2 * var[4][..., 0] + (4 * u32 * (wy * sig + pos_weight * y) / n_total) ** 2
        dz, v_dz = dz[..., None], _round_var(v_pre, dz)[..., None]
        grads = [None] * 4
        n_acc = chunk_pixels + n_total // chunk_pixels
        for l in range(3, -1, -1):
            x2, vx = acts[l] ** 2, var[l]
            zero = np.zeros_like(Wq[l])
            _, a1, _ = op.conv3x3_back(x2, zero, v_dz)          # sum x^2 v_dz
            _, a2, _ = op.conv3x3_back(vx, zero, dz ** 2)       # sum v_x dz^2
            _, a3, _ = op.conv3x3_back(x2, zero, dz ** 2)       # sum x^2 dz^2
            vW = a1 + a2 + n_acc * u32 ** 2 * a3
            vb = v_dz.sum(axis=(0, 1)) + n_acc * u32 ** 2 * (dz ** 2).sum(axis=(0, 1))
            grads[l] = (vW, vb)
            if l > 0:
                d1, _, _ = op.conv3x3_back(x2, W2[l], v_dz)     # sum W^2 v_dz
                d2, _, _ = op.conv3x3_back(x2, W2[l], dz ** 2)  # sum W^2 dz^2
                dxo, _, _ = op.conv3x3_back(acts[l], Wq[l], dz)
                mask = acts[l] > 0
                flip = np.abs(pre[l]) <= k * np.sqrt(var[l]) + 1e-30
                dz_new = op.bf16_round(dxo * mask)
                v_pre = (d1 + 9 * W2[l].shape[0] * u32 ** 2 * d2) * mask + dxo ** 2 * flip
                dz, v_dz = dz_new, _round_var(v_pre, dz_new)
        vflat = op.pack_grads(grads)
        vsum = vflat if vsum is None else vsum + vflat
    return np.sqrt(vsum)
