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
