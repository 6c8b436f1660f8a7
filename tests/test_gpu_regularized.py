"""Regularised MPNL (MMSE-extended system) on the GPU against the oracle on
the same extended system, including overloaded slots with N > M."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def mp():
    import paper_2409_14355_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


CASES = [  # S, T, M, N, bits, paths, snr
    (40, 14, 8, 12, 2, 64, 12.0),    # overloaded 1.5x
    (30, 14, 4, 8, 4, 256, 18.0),    # overloaded 2x, 16-QAM
    (25, 5, 12, 16, 4, 128, 16.0),   # M + N = 28
    (20, 14, 16, 16, 4, 256, 14.0),  # M + N = 32, square
    (33, 3, 6, 2, 6, 100, 20.0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[3]}u-{c[2]}a-b{c[4]}-K{c[5]}")
def test_regularized_matches_oracle(ctx, case):
    S, T, M, N, bits, K, snr = case
    _say("regularized", case)
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=(600, M, N))
    got = ctx.detect_regularized(_dev(sl.H), _dev(sl.y), bits, K, sl.sigma2)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    Hx, yx = oracle.regularized_system(sl.H, sl.y, float(np.sqrt(np.float32(sl.sigma2))))
    ref, diag = oracle.detect_slot("mpnl", Hx, yx, bits, n_paths=K, want_diag=True, nthreads=8)
    check(Hx, yx, got, ref, diag, bits, label=str(case))
    ber_reg = synth.bit_errors(got, sl.s_idx, bits) / (sl.s_idx.size * bits)
    print("BER", ber_reg, flush=True)


def test_zero_sigma_is_plain_detect(ctx):
    _say("regularized sigma2 = 0")
    sl = synth.make_slot(S=30, T=7, M=12, N=10, bits=4, snr_db=15, seed=(601,))
    H, y = _dev(sl.H), _dev(sl.y)
    a = ctx.detect_regularized(H, y, 4, 128, 0.0)
    b = ctx.detect(H, y, 4, 128)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_overloaded_regularized_beats_mmse(ctx):
    """Directional: on an overloaded 12-user, 8-antenna QPSK slot the
    regularised MPNL makes fewer bit errors than linear MMSE."""
    _say("regularized vs mmse")
    sl = synth.make_slot(S=300, T=14, M=8, N=12, bits=2, snr_db=14, seed=(602,))
    H, y = _dev(sl.H), _dev(sl.y)
    a = ctx.detect_regularized(H, y, 2, 256, sl.sigma2)
    b = ctx.mmse(H, y, 2, sl.sigma2)
    torch.cuda.synchronize()
    ea = synth.bit_errors(a.cpu().numpy(), sl.s_idx, 2)
    eb = synth.bit_errors(b.cpu().numpy(), sl.s_idx, 2)
    print("errors regularized MPNL", ea, "MMSE", eb, flush=True)
    assert ea < eb


def test_regularized_error_codes(ctx, mp):
    _say("regularized error codes")
    H = torch.zeros((4, 4, 8), dtype=torch.complex64, device="cuda:0")
    y = torch.zeros((1, 4, 4), dtype=torch.complex64, device="cuda:0")
    out = torch.zeros((1, 4, 8), dtype=torch.int32, device="cuda:0")
    L, h = mp.lib(), ctx.handle
    hp, yp, op = H.data_ptr(), y.data_ptr(), out.data_ptr()
    assert L.mpnl_detect_regularized(h, hp, yp, 4, 1, 4, 8, 2, 16, 0.0, op, None) == mp.MPNL_E_INVAL
    assert L.mpnl_detect_regularized(h, hp, yp, 4, 1, 4, 8, 2, 16, -0.5, op, None) == mp.MPNL_E_INVAL
    assert L.mpnl_detect_regularized(h, hp, yp, 4, 1, 28, 8, 2, 16, 0.1, op, None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_detect_regularized(h, hp, yp, 4, 1, 4, 8, 5, 16, 0.1, op, None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_detect_regularized(h, hp, yp, 4, 1, 4, 8, 2, 0, 0.1, op, None) == mp.MPNL_E_INVAL
