"""retina_response_noalloc (the fixed-workspace variant of retina_response)
against retina_response through the C-ABI.

Both entry points run the same kernels; the variant takes its workspace from
the library's per-device fixed array instead of the context's pool.  Checked:
two calls in a row (the second on a smaller batch, so stale workspace contents
from the first call are present), each against retina_response at the parity
bar (R 1e-5 relative, gradient / Hessian 1e-4 relative with a floor) and, as
the part split is the same here, bit for bit; a context whose pool may not
grow at all still serves the variant; host memory and an oversized batch are
refused before any device work."""
import sys

import numpy as np
import pytest

import oracle
from paper_1709_08610_amd import events, retina

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(b):
    import torch
    return (torch.from_numpy(b.event_offsets).cuda(), torch.from_numpy(b.x).cuda(),
            torch.from_numpy(b.y).cuda(), torch.from_numpy(b.plane).cuda())


def _close(a, b, rtol):
    a = a.cpu().numpy().astype(np.float64)
    b = b.cpu().numpy().astype(np.float64)
    floor = 1e-6 * max(np.abs(b).max(), 1e-30)
    np.testing.assert_array_less(np.abs(a - b), rtol * np.abs(b) + floor)


def _compare(ctx, b, theta, theta_off, sigma):
    import torch
    off, x, y, pl = _dev(b)
    th = torch.from_numpy(np.ascontiguousarray(theta, np.float32)).cuda()
    to = None if theta_off is None else torch.from_numpy(np.asarray(theta_off, np.int64)).cuda()
    want = retina.WANT_R | retina.WANT_GRAD | retina.WANT_HESS
    R1, G1, H1 = ctx.retina_response(2, b.plane_z, off, x, y, pl, th, to, sigma=sigma, want=want)
    R2, G2, H2 = ctx.retina_response_noalloc(2, b.plane_z, off, x, y, pl, th, to, sigma=sigma, want=want)
    torch.cuda.synchronize()
    _close(R2, R1, 1e-5)
    _close(G2, G1, 1e-4)
    _close(H2, H1, 1e-4)
    for a, c in ((R1, R2), (G1, G2), (H1, H2)):
        assert torch.equal(a, c), "same kernels, same part split: results must be bit-identical"
    return R2


def test_noalloc_two_calls_second_smaller():
    _say("noalloc: c2 event (4096 lattice lines + near lines), then 3 ragged c3 events")
    ctx = retina.Context(0)
    cfg2 = events.load_config("c2")
    b2 = events.make_batch(cfg2, 1)
    ev = b2.event(0)
    rng = np.random.default_rng(5)
    lat = oracle.lattice(2, cfg2["params"])
    near = ev.truth[rng.integers(0, len(ev.truth), 1024)] + rng.normal(0, 1, (1024, 4)) * np.array(
        [0.03, 0.03, 1e-4, 1e-4])
    theta = np.concatenate([lat, near]).astype(np.float32)
    R = _compare(ctx, b2, theta, None, 0.03)
    # the first call's values against the oracle on a sample (the variant is
    # the response itself, not only equal to the pooled call)
    idx = rng.choice(theta.shape[0], 64, replace=False)
    Rr, _, _ = oracle.response(2, b2.plane_z, ev.x, ev.y, ev.plane, theta[idx].astype(np.float64), 0.03)
    got = R.cpu().numpy()[idx].astype(np.float64)
    np.testing.assert_array_less(np.abs(got - Rr), 1e-5 * np.abs(Rr) + 1e-30)

    cfg3 = events.load_config("c3")
    evs = [events.make_event(cfg3, i) for i in range(3)]
    b3 = events.batch_from_events(2, events.plane_z(cfg3), evs)
    counts = [700, 0, 129]
    th3 = np.concatenate([e.truth[rng.integers(0, len(e.truth), n)] if n else np.zeros((0, 4))
                          for e, n in zip(evs, counts)]).astype(np.float32)
    th3 += (rng.normal(0, 1, th3.shape) * np.array([0.03, 0.03, 1e-4, 1e-4])).astype(np.float32)
    toff = np.concatenate([[0], np.cumsum(counts)])
    _compare(ctx, b3, th3, toff, 0.25)
    ctx.close()


def test_noalloc_needs_no_pool():
    """A fresh context whose pool may not grow by a single byte: the pooled
    call fails for want of memory, the variant does not."""
    import torch
    _say("noalloc: pool limited to 1 byte")
    ctx = retina.Context(0)
    ctx.set_max_device_bytes(1)
    cfg = events.load_config("c3")
    b = events.batch_from_events(2, events.plane_z(cfg), [events.make_event(cfg, 7)])
    off, x, y, pl = _dev(b)
    th = torch.from_numpy(b.event(0).truth.astype(np.float32)).cuda()
    with pytest.raises(retina.RetinaError) as ei:
        ctx.retina_response(2, b.plane_z, off, x, y, pl, th, sigma=0.03)
    assert ei.value.code == retina.ERR_OUT_OF_MEMORY
    R, G, H = ctx.retina_response_noalloc(2, b.plane_z, off, x, y, pl, th, sigma=0.03)
    torch.cuda.synchronize()
    ev = b.event(0)
    Rr, _, _ = oracle.response(2, b.plane_z, ev.x, ev.y, ev.plane, th.cpu().numpy().astype(np.float64), 0.03)
    np.testing.assert_array_less(np.abs(R.cpu().numpy() - Rr), 1e-5 * np.abs(Rr) + 1e-30)
    ctx.close()


def test_noalloc_refusals():
    import torch
    _say("noalloc: host memory and an oversized batch are refused")
    ctx = retina.Context(0)
    cfg = events.load_config("c3")
    b = events.batch_from_events(2, events.plane_z(cfg), [events.make_event(cfg, 0)])
    th = b.event(0).truth.astype(np.float32)
    with pytest.raises(retina.RetinaError) as ei:
        ctx.retina_response_noalloc(2, b.plane_z, b.event_offsets, b.x, b.y, b.plane, th, sigma=0.03)
    assert ei.value.code == retina.ERR_INVALID_ARG
    # more staged hits than the workspace holds (8 bytes per hit): refused with
    # the sizes, before any kernel reads the (zero) hit arrays
    n = (64 << 20) // 8 + 4096  # RETINA_NOALLOC_SCRATCH_BYTES / (8 bytes per staged hit), plus some
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    x = torch.zeros(n, dtype=torch.float32, device="cuda")
    y = torch.zeros(n, dtype=torch.float32, device="cuda")
    pl = torch.zeros(n, dtype=torch.int32, device="cuda")
    thd = torch.from_numpy(th).cuda()
    with pytest.raises(retina.RetinaError) as ei:
        ctx.retina_response_noalloc(2, b.plane_z, off, x, y, pl, thd, sigma=0.03)
    assert ei.value.code == retina.ERR_CAPACITY
    assert "workspace" in str(ei.value)
    ctx.close()
