"""Allocation-free one-shot detection (mpnl_detect_static) against mpnl_detect.

The static entry point runs the same kernels with its buffers in the
library's fixed device scratch area; its decisions must equal those of
mpnl_detect on the same inputs, bit for bit, call after call (the second
call smaller than the first, so stale contents of the area would show), and
it must leave the context's memory pool untouched.
"""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _inputs(S, T, M, N, bits, snr, seed, channel="iid"):
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=seed, channel=channel,
                         rho_rx=0.5, rho_tx=0.3)
    return torch.from_numpy(sl.H).to(DEV), torch.from_numpy(sl.y).to(DEV)


def _compare(ctx_static, ctx_ref, H, y, bits, K, label):
    import paper_2409_14355_amd as mp
    S, M, N = H.shape
    T = y.shape[0]
    out_s = torch.full((T, S, N), -7, dtype=torch.int32, device=DEV)
    out_r = torch.full((T, S, N), -9, dtype=torch.int32, device=DEV)
    print(f"[no-alloc] {label}: S={S} T={T} M={M} N={N} bits={bits} K={K}", flush=True)
    mp.mpnl_detect_static(ctx_static.handle, H, y, S, T, M, N, bits, K, out_s)
    mp.mpnl_detect(ctx_ref.handle, H, y, S, T, M, N, bits, K, out_r)
    torch.cuda.synchronize()
    a, b = out_s.cpu().numpy(), out_r.cpu().numpy()
    n_bad = int(np.any(a != b, axis=-1).sum())
    print(f"[no-alloc] {label}: {n_bad} of {T * S} vectors differ", flush=True)
    assert n_bad == 0
    return a


def test_static_equals_detect_two_calls_shrinking():
    import paper_2409_14355_amd as mp
    ctx_s = mp.Context(0)
    ctx_r = mp.Context(0)
    try:
        # first call: a full 16 x 16 16-QAM slot, 256 paths (four path groups)
        H, y = _inputs(1200, 14, 16, 16, 4, 12.0, (70, 0))
        _compare(ctx_s, ctx_r, H, y, 4, 256, "call 1")
        # second, smaller call with more than 256 paths (the other position-set
        # kernel and more path groups) on a different shape
        H2, y2 = _inputs(77, 5, 8, 6, 6, 18.0, (70, 1))
        _compare(ctx_s, ctx_r, H2, y2, 6, 1000, "call 2")
        # the pool of the context that ran only static calls is untouched
        assert ctx_s.memory_usage() == (0, 0)
    finally:
        ctx_s.close()
        ctx_r.close()


def test_static_reduced_precision_and_limits():
    import paper_2409_14355_amd as mp
    ctx_s = mp.Context(0)
    ctx_r = mp.Context(0)
    try:
        for prec in (mp.MPNL_PREC_FP16, mp.MPNL_PREC_BF16):
            ctx_s.set_precision(prec)
            ctx_r.set_precision(prec)
            H, y = _inputs(300, 14, 24, 24, 4, 18.0, (71, prec), channel="kron")
            _compare(ctx_s, ctx_r, H, y, 4, 256, f"precision {prec}")
        ctx_s.set_precision(mp.MPNL_PREC_FP32)
        ctx_r.set_precision(mp.MPNL_PREC_FP32)
        H, y = _inputs(64, 1, 4, 4, 2, 10.0, (71, 9))
        _compare(ctx_s, ctx_r, H, y, 2, 16, "4x4 QPSK, one symbol")
        # a slot larger than the scratch area is refused before anything runs
        S, T, M, N = 3276, 14, 32, 32
        Hb = torch.zeros((S, M, N), dtype=torch.complex64, device=DEV)
        yb = torch.zeros((T, S, M), dtype=torch.complex64, device=DEV)
        ob = torch.full((T, S, N), -3, dtype=torch.int32, device=DEV)
        with pytest.raises(mp.MpnlError) as ei:
            mp.mpnl_detect_static(ctx_s.handle, Hb, yb, S, T, M, N, 6, 256, ob)
        assert ei.value.code == mp.MPNL_E_NOMEM
        torch.cuda.synchronize()
        assert bool((ob == -3).all())
        assert ctx_s.memory_usage() == (0, 0)
    finally:
        ctx_s.close()
        ctx_r.close()
