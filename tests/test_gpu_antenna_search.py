"""The antenna-count search (the procedure behind the paper's antenna
results, Sec. III-B and Fig. 3: raise the number of receive antennas one at
a time until the error target is met) run with the GPU detectors, every
detector output checked against the FP64 oracle on the same inputs, and the
antenna counts it finds equal to the ones the oracle's own decisions give."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from parity_util import check

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
from bench import antenna_search  # noqa: E402  (the host loop bench.py runs)

# users, detector, paths; 16-QAM at 20 dB, 24 subcarriers x 14 symbols per
# antenna count, BER target 1e-3
BITS, SNR, S, T, TARGET = 4, 20.0, 24, 14, 1e-3
MMSE_TAU = 1e-2  # relative gap of the two nearest points under which float32 may flip a decision


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import paper_2409_14355_amd as m
    c = m.Context(0)
    yield c
    c.close()


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda:0")


def _mmse_check(sl, got):
    """GPU MMSE decisions equal the oracle's except for users whose FP64
    estimate lies within MMSE_TAU of a decision boundary."""
    pts = oracle.constellation(BITS)
    ref = np.empty_like(got)
    n_diff = 0
    for s in range(sl.H.shape[0]):
        for t in range(sl.y.shape[0]):
            ref[t, s] = oracle.mmse(sl.H[s], sl.y[t, s], BITS, sl.sigma2)
            diff = ref[t, s] != got[t, s]
            if diff.any():
                x = oracle.mmse_estimate(sl.H[s], sl.y[t, s], sl.sigma2)
                d = np.sort(np.abs(x[:, None] - pts[None, :]) ** 2, axis=1)
                near = (d[:, 1] - d[:, 0]) / np.maximum(d[:, 1], 1e-300) < MMSE_TAU
                assert near[diff].all(), (s, t, ref[t, s], got[t, s])
                n_diff += int(diff.sum())
    assert n_diff <= max(2, 0.01 * got.size)
    return ref


@pytest.mark.parametrize("users,det", [(2, "mpnl64"), (4, "mpnl64"), (4, "mpnl256"), (2, "mmse"),
                                       (4, "mmse")])
def test_antenna_search_matches_oracle(ctx, users, det):
    _say("antenna search", users, det)
    ber_gpu, ber_ref = {}, {}

    def run(M):
        sl = synth.make_slot(S=S, T=T, M=M, N=users, bits=BITS, snr_db=SNR, seed=(700, users, M))
        H, y = _dev(sl.H), _dev(sl.y)
        if det == "mmse":
            got = ctx.mmse(H, y, BITS, sl.sigma2)
            torch.cuda.synchronize()
            got = got.cpu().numpy()
            ref = _mmse_check(sl, got)
        else:
            K = int(det[4:])
            got = ctx.detect_regularized(H, y, BITS, K, sl.sigma2)
            torch.cuda.synchronize()
            got = got.cpu().numpy()
            Hx, yx = oracle.regularized_system(sl.H, sl.y, float(np.sqrt(np.float32(sl.sigma2))))
            ref, diag = oracle.detect_slot("mpnl", Hx, yx, BITS, n_paths=K, want_diag=True, nthreads=8)
            check(Hx, yx, got, ref, diag, BITS, label=f"{det} {users} users {M} antennas")
        nb = sl.s_idx.size * BITS
        ber_gpu[M] = synth.bit_errors(got, sl.s_idx, BITS) / nb
        ber_ref[M] = synth.bit_errors(ref, sl.s_idx, BITS) / nb
        return ber_gpu[M]

    m_hi = 16 if det == "mmse" else 32 - users
    M_gpu, trace = antenna_search(run, 1, m_hi, TARGET)
    M_ref, _ = antenna_search(lambda M: ber_ref[M] if M in ber_ref else 1.0, 1, m_hi, TARGET)
    print(f"{det}, {users} users: {M_gpu} antennas (trace {trace})", flush=True)
    assert M_gpu is not None
    assert M_gpu == M_ref
