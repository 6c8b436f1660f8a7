"""GPU parity of the MPNL hot path against the FP64 oracle, through the C ABI.

Every case prints its name, shape and seed before touching the GPU.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL, check

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


def _run(ctx, sl, n_paths):
    out = ctx.detect(_dev(sl.H), _dev(sl.y), sl.bits, n_paths)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _assert_parity(sl, got, n_paths, nthreads=8, label=""):
    ref, diag = oracle.detect_slot("mpnl", sl.H, sl.y, sl.bits, n_paths=n_paths,
                                   want_diag=True, nthreads=nthreads)
    n_bad, _ = check(sl.H, sl.y, got, ref, diag, sl.bits, label=label)
    return ref, n_bad


# ------------------------------------------------------------------ a1 / a2 ---
@pytest.mark.parametrize("S,M,N,bits,ch", [(37, 4, 4, 2, "iid"), (16, 16, 16, 4, "iid"),
                                           (9, 24, 24, 4, "kron"), (11, 32, 12, 6, "iid"),
                                           (5, 7, 3, 4, "iid"), (4, 32, 32, 6, "iid")])
def test_sorted_qr_stage(ctx, S, M, N, bits, ch):
    _say("sqrd", S, M, N, bits, ch)
    sl = synth.make_slot(S=S, T=1, M=M, N=N, bits=bits, snr_db=18, seed=(201, S, M, N), channel=ch,
                         rho_rx=0.5, rho_tx=0.3)
    slot = ctx.slot_prepare(_dev(sl.H), bits, 64)
    ex = slot.export()
    torch.cuda.synchronize()
    perm = ex["perm"].cpu().numpy()
    w = ex["w"].cpu().numpy()
    roff = ex["roff"].cpu().numpy()
    slot.release()
    for s in range(S):
        Q, R, operm, pm = oracle.sqrd(sl.H[s])
        operm_d = operm[::-1]          # depth order
        if not np.array_equal(perm[s], operm_d):
            assert pm < TOL, (s, perm[s], operm_d, pm)
            continue
        rd = np.real(np.diag(R))[::-1]
        scale = np.abs(sl.H[s]).max()
        assert np.allclose(np.sqrt(w[s]), rd, rtol=1e-5, atol=1e-5 * scale)
        for d in range(N):
            for d2 in range(d + 1, N):
                ref = R[N - 1 - d2, N - 1 - d]
                assert abs(roff[s, d, d2] - ref) < 2e-5 * max(1.0, scale * math.sqrt(M)), (s, d, d2)


@pytest.mark.parametrize("S,M,N,bits,K", [(20, 4, 4, 2, 16), (12, 16, 16, 4, 256), (6, 24, 24, 4, 256),
                                          (8, 8, 8, 6, 128), (4, 3, 3, 4, 4096), (6, 12, 10, 4, 1000),
                                          (5, 4, 2, 6, 4096), (7, 6, 5, 2, 100)])
def test_position_set_stage(ctx, S, M, N, bits, K):
    """a2 on the GPU's own float64 weights equals the oracle's best-first set,
    entry for entry and in order: both sides round every score the same way
    (product and sum of each term separately, in depth order)."""
    _say("posvec", S, M, N, bits, K)
    sl = synth.make_slot(S=S, T=1, M=M, N=N, bits=bits, snr_db=15, seed=(202, S, N, K))
    slot = ctx.slot_prepare(_dev(sl.H), bits, K)
    ex = slot.export()
    torch.cuda.synchronize()
    w = ex["w"].cpu().numpy()
    P = ex["P"].cpu().numpy()
    slot.release()
    for s in range(S):
        Pr, _, bmargin = oracle.position_set(w[s], 1 << bits, K)
        assert P.shape[1] == Pr.shape[0]
        assert np.array_equal(P[s], Pr), (s, bmargin)


def test_position_set_large_slot(ctx):
    """A slot of 3276 subcarriers with 24 users and 256 paths, where the
    position-set kernel keeps its back pointers in global memory (fewer rounds
    of workgroups than with them in LDS on this device): the sets of sampled
    subcarriers equal the oracle's entry for entry, and equal those of the
    same subcarriers prepared in a small slot (back pointers in LDS)."""
    S, M, N, bits, K = 3276, 24, 24, 4, 256
    _say("posvec large slot", S, N, K)
    sl = synth.make_slot(S=S, T=1, M=M, N=N, bits=bits, snr_db=18, seed=(203, S, N))
    slot = ctx.slot_prepare(_dev(sl.H), bits, K)
    ex = slot.export()
    torch.cuda.synchronize()
    w = ex["w"].cpu().numpy()
    P = ex["P"].cpu().numpy()
    slot.release()
    sub = np.sort(np.random.default_rng(204).choice(S, size=24, replace=False))
    small = ctx.slot_prepare(_dev(np.ascontiguousarray(sl.H[sub])), bits, K)
    ex_small = small.export()
    torch.cuda.synchronize()
    P_small = ex_small["P"].cpu().numpy()
    small.release()
    assert np.array_equal(P[sub], P_small)
    for i, s in enumerate(sub):
        Pr, _, bmargin = oracle.position_set(w[s], 1 << bits, K)
        assert np.array_equal(P[s], Pr), (int(s), bmargin)


@pytest.mark.parametrize("M,N,bits,K", [(4, 4, 2, 200), (6, 6, 4, 256), (5, 5, 2, 64), (8, 8, 6, 1000)])
def test_position_set_exact_ties(ctx, M, N, bits, K):
    """Identity channels give exactly equal weights (all 1.0) and zeroed
    columns give zero weights: the set and its order are then decided by the
    lexicographic rule alone."""
    _say("posvec ties", M, N, bits, K)
    H = np.zeros((3, M, N), np.complex64)
    for s in range(3):
        H[s, :N, :N] = np.eye(N)
    H[1, :, 1] = 0
    H[2, :, 0] = 0
    H[2, :, N - 1] = 0
    slot = ctx.slot_prepare(_dev(H), bits, K)
    ex = slot.export()
    torch.cuda.synchronize()
    w = ex["w"].cpu().numpy()
    P = ex["P"].cpu().numpy()
    slot.release()
    assert np.all(np.isin(w, [0.0, 1.0]))
    for s in range(3):
        Pr, _, _ = oracle.position_set(w[s], 1 << bits, K)
        assert np.array_equal(P[s], Pr), s


# ------------------------------------------------------------- end to end ---
CASES = [
    # name, S, T, M, N, bits, snr, K, channel
    ("4x4-qpsk-S64-T1-K16", 64, 1, 4, 4, 2, 10, 16, "iid"),
    ("16x16-qam16-K64", 40, 14, 16, 16, 4, 14, 64, "iid"),
    ("16x16-qam16-K256", 24, 14, 16, 16, 4, 20, 256, "iid"),
    ("24x24-qam16-kron-K256", 12, 14, 24, 24, 4, 18, 256, "kron"),
    ("8x8-qam64-K128", 30, 5, 8, 8, 6, 22, 128, "iid"),
    ("32x12-qam64-K256", 10, 3, 32, 12, 6, 20, 256, "iid"),
    ("32x32-qpsk-K64", 6, 2, 32, 32, 2, 8, 64, "iid"),
    ("6x5-qam16-K1000", 9, 17, 6, 5, 4, 12, 1000, "iid"),
    ("3x1-qam64-K8", 33, 3, 3, 1, 6, 15, 8, "iid"),
    ("7x3-qpsk-K100-odd", 15, 2, 7, 3, 2, 5, 100, "iid"),
    ("12x8-qam16-K1-sic", 50, 7, 12, 8, 4, 16, 1, "iid"),      # path 0 alone: ordered SIC
    ("6x6-qpsk-K2", 40, 5, 6, 6, 2, 6, 2, "kron"),
    ("4x3-qam16-K4096-all", 12, 3, 4, 3, 4, 8, 4096, "iid"),  # every vector: ML
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_detect_parity(ctx, case):
    name, S, T, M, N, bits, snr, K, ch = case
    _say("detect", name)
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=(203, S, T, M, N, K),
                         channel=ch, rho_rx=0.5, rho_tx=0.3)
    got = _run(ctx, sl, K)
    assert got.min() >= 0 and got.max() < (1 << bits)
    _assert_parity(sl, got, K, label=name)


@pytest.mark.parametrize("M,N,bits,S", [(4, 4, 2, 40), (3, 3, 4, 12), (2, 2, 6, 24), (6, 4, 2, 30)])
def test_enough_paths_is_ml(ctx, M, N, bits, S):
    """With N_p >= |Q|^N the detector is exact ML (clamped path count)."""
    _say("ml", M, N, bits, S)
    sl = synth.make_slot(S=S, T=2, M=M, N=N, bits=bits, snr_db=6, seed=(204, M, N, bits))
    got = _run(ctx, sl, 10 ** 6)
    ref = oracle.detect_slot("ml", sl.H, sl.y, bits, nthreads=8)
    mism = np.any(got != ref, axis=-1)
    for t, s in zip(*np.nonzero(mism)):
        r_got = oracle.residual_norm2(sl.H[s], sl.y[t, s], bits, got[t, s])
        r_ref = oracle.residual_norm2(sl.H[s], sl.y[t, s], bits, ref[t, s])
        assert abs(r_got - r_ref) <= TOL * r_ref, (t, s)


def test_noise_free_and_one_path(ctx):
    _say("noise-free")
    sl = synth.make_slot(S=50, T=3, M=10, N=8, bits=4, snr_db=0, seed=(205,), noise=False)
    got = _run(ctx, sl, 1)
    assert np.array_equal(got, sl.s_idx)


def test_zero_column_channel(ctx):
    _say("zero-column")
    sl = synth.make_slot(S=20, T=2, M=6, N=4, bits=4, snr_db=12, seed=(206,))
    sl.H[:, :, 2] = 0
    sl.y[...] = np.einsum("smn,tsn->tsm", sl.H.astype(np.complex128),
                          synth._tx_points(4)[sl.s_idx]).astype(np.complex64) + sl.y * 0.01
    got = _run(ctx, sl, 64)
    # every point ties at the zero column's depth and paths that differ only
    # there tie in metric: both sides take index order and the lowest path,
    # so no vector may differ at all
    ref = oracle.detect_slot("mpnl", sl.H, sl.y, sl.bits, n_paths=64, nthreads=8)
    n_bad = int(np.any(got != ref, axis=-1).sum())
    print(f"zero-column: {n_bad} of {got.shape[0] * got.shape[1]} vectors differ", flush=True)
    assert n_bad == 0
    assert np.all(got[:, :, 2] == 0)


def test_full_size_sampled_24x24_kron(ctx):
    """24x24 16-QAM Kronecker slot of 3276 subcarriers x 14 symbols, 256 paths,
    in the launch configuration the benchmark times; the oracle checks a sample."""
    _say("full-size 24x24 S3276 T14 K256")
    S, T, M, N, bits, K = 3276, 14, 24, 24, 4, 256
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=18, seed=(3, 0, 0, 0), channel="kron",
                         rho_rx=0.5, rho_tx=0.3)
    got = _run(ctx, sl, K)
    rng = np.random.default_rng(0)
    sub = np.sort(rng.choice(S, size=24, replace=False))
    sub_sl = synth.Slot(H=sl.H[sub], y=sl.y[:, sub], s_idx=sl.s_idx[:, sub], sigma2=sl.sigma2, bits=bits)
    _assert_parity(sub_sl, got[:, sub], K, nthreads=16, label="24x24 kron S3276 T14 sample")


def test_full_size_sampled_16x16(ctx):
    _say("full-size 16x16 S1200 T14 K256")
    S, T, M, N, bits, K = 1200, 14, 16, 16, 4, 256
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=16, seed=(2, 3, 0, 0))
    got = _run(ctx, sl, K)
    sub = np.arange(0, S, 60)
    sub_sl = synth.Slot(H=sl.H[sub], y=sl.y[:, sub], s_idx=sl.s_idx[:, sub], sigma2=sl.sigma2, bits=bits)
    _assert_parity(sub_sl, got[:, sub], K, nthreads=16, label="16x16 S1200 T14 sample")


def test_paired_ber_matches_oracle(ctx):
    """BER of the GPU and of the FP64 oracle on the same samples agree within
    the Wilson interval."""
    _say("paired BER")
    S, T, M, N, bits, K = 60, 14, 16, 16, 4, 64
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=6, seed=(207,))
    got = _run(ctx, sl, K)
    ref = oracle.detect_slot("mpnl", sl.H, sl.y, bits, n_paths=K, nthreads=16)
    n = sl.s_idx.size * bits
    e_gpu = synth.bit_errors(got, sl.s_idx, bits)
    e_ref = synth.bit_errors(ref, sl.s_idx, bits)
    assert e_ref >= 100
    lo, hi = synth.wilson(e_ref, n)
    assert lo <= e_gpu / n <= hi


# ---------------------------------------------------------- API behaviour ---
def test_slot_reuse_equals_one_shot(ctx):
    _say("slot reuse")
    sl = synth.make_slot(S=30, T=14, M=12, N=10, bits=4, snr_db=14, seed=(208,))
    sl2 = synth.make_slot(S=30, T=5, M=12, N=10, bits=4, snr_db=14, seed=(209,))
    Hd = _dev(sl.H)
    slot = ctx.slot_prepare(Hd, 4, 128)
    a = slot.detect(_dev(sl.y))
    y2 = _dev(sl2.y)
    b = slot.detect(y2)
    torch.cuda.synchronize()
    one = ctx.detect(Hd, _dev(sl.y), 4, 128)
    two = ctx.detect(Hd, y2, 4, 128)
    torch.cuda.synchronize()
    slot.release()
    assert torch.equal(a, one) and torch.equal(b, two)


def test_workspace_reuse_across_streams(ctx):
    """One-shot and slot calls on the default stream hand their workspace back
    to the pool without a stream event; a call on another stream that wants
    that memory must still wait for the work that used it.  Calls alternate
    between the default stream and a side stream with similar sizes (so the
    pool hands the same blocks around), the side stream's calls running while
    the default stream still works; every result must equal the first one."""
    _say("workspace across streams")
    sls = [synth.make_slot(S=S, T=14, M=16, N=16, bits=4, snr_db=14, seed=(211, S)) for S in (300, 280)]
    dev = [(_dev(sl.H), _dev(sl.y)) for sl in sls]
    refs = [ctx.detect(H, y, 4, 256) for H, y in dev]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    outs = [(j, torch.full_like(refs[j], -1)) for _ in range(8) for j in range(len(dev))]
    torch.cuda.synchronize()
    for i in range(8):
        st = None if i % 2 == 0 else side
        for j, (H, y) in enumerate(dev):
            out = outs[i * len(dev) + j][1]
            if i % 4 == 3:
                slot = ctx.slot_prepare(H, 4, 256, stream=st)
                slot.detect(y, out=out, stream=st)
                slot.release()
            else:
                ctx.detect(H, y, 4, 256, out=out, stream=st)
    torch.cuda.synchronize()
    for j, out in outs:
        assert torch.equal(out, refs[j]), j


def test_deterministic_and_batch_equals_alone(ctx):
    _say("batch vs alone")
    shapes = [(120, 14, 8, 6, 2, 64), (75, 14, 16, 16, 4, 128), (40, 14, 32, 20, 6, 256),
              (33, 3, 5, 5, 4, 256), (64, 14, 12, 12, 4, 64)]
    jobs, alone = [], []
    for i, (S, T, M, N, bits, K) in enumerate(shapes):
        sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=20, seed=(210, i))
        H, y = _dev(sl.H), _dev(sl.y)
        jobs.append(dict(H=H, y=y, mod=bits, n_paths=K, out=None))
        a1 = ctx.detect(H, y, bits, K)
        a2 = ctx.detect(H, y, bits, K)
        torch.cuda.synchronize()
        assert torch.equal(a1, a2)
        alone.append(a1)
    outs = ctx.detect_batch(jobs)
    torch.cuda.synchronize()
    for a, b in zip(alone, outs):
        assert torch.equal(a, b)


def test_error_codes(ctx, mp):
    _say("error codes")
    H = torch.zeros((4, 4, 4), dtype=torch.complex64, device="cuda:0")
    y = torch.zeros((1, 4, 4), dtype=torch.complex64, device="cuda:0")
    out = torch.zeros((1, 4, 4), dtype=torch.int32, device="cuda:0")
    h = ctx.handle
    L = mp.lib()
    assert L.mpnl_detect(h, None, y.data_ptr(), 4, 1, 4, 4, 2, 16, out.data_ptr(), None) == mp.MPNL_E_INVAL
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 0, 1, 4, 4, 2, 16, out.data_ptr(), None) == mp.MPNL_E_INVAL
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 4, 1, 4, 4, 2, 0, out.data_ptr(), None) == mp.MPNL_E_INVAL
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 4, 1, 4, 4, 3, 16, out.data_ptr(), None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 4, 1, 3, 4, 2, 16, out.data_ptr(), None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 4, 1, 40, 33, 2, 16, out.data_ptr(), None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_detect(h, H.data_ptr(), y.data_ptr(), 4, 1, 8, 8, 4, 5000, out.data_ptr(), None) == mp.MPNL_E_UNSUPPORTED
    assert L.mpnl_set_precision(h, 7) == mp.MPNL_E_INVAL
    assert L.mpnl_slot_release(h, 12345) == mp.MPNL_E_INVAL


def test_hbm_budget_admission(mp):
    _say("budget")
    small = mp.Context(0, hbm_budget_bytes=1 << 20)
    sl = synth.make_slot(S=3000, T=14, M=24, N=24, bits=4, snr_db=18, seed=(211,))
    with pytest.raises(mp.MpnlError) as ei:
        small.slot_prepare(_dev(sl.H), 4, 256)
    assert ei.value.code == mp.MPNL_E_NOMEM
    sl2 = synth.make_slot(S=4, T=1, M=4, N=4, bits=2, snr_db=18, seed=(212,))
    s2 = small.slot_prepare(_dev(sl2.H), 2, 16)
    held, used = small.memory_usage()
    assert 0 < used <= held <= (1 << 20)
    s2.release()
    small.close()


# --------------------------------------------------------- precision ---
@pytest.mark.parametrize("prec", [1, 2], ids=["fp16", "bf16"])
def test_reduced_precision_close_to_fp64(ctx, mp, prec):
    """FP16 / BF16 path-metric operands with FP32 accumulation: the decision
    mismatch against the FP64 oracle stays small and the BER stays inside the
    oracle's Wilson interval."""
    _say("precision", prec)
    S, T, M, N, bits, K = 40, 14, 24, 24, 4, 256
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=8, seed=(213,), channel="kron",
                         rho_rx=0.5, rho_tx=0.3)
    ctx.set_precision(prec)
    try:
        got = _run(ctx, sl, K)
    finally:
        ctx.set_precision(0)
    ref = oracle.detect_slot("mpnl", sl.H, sl.y, bits, n_paths=K, nthreads=16)
    frac = np.mean(np.any(got != ref, axis=-1))
    n = sl.s_idx.size * bits
    e_gpu, e_ref = synth.bit_errors(got, sl.s_idx, bits), synth.bit_errors(ref, sl.s_idx, bits)
    lo, hi = synth.wilson(e_ref, n)
    print(f"prec {prec}: vector mismatch {frac:.4f}, BER gpu {e_gpu / n:.3e} oracle {e_ref / n:.3e}",
          flush=True)
    # about twice the measured mismatch (FP16: 1 of 560 vectors, BF16: 7)
    assert frac <= {1: 0.006, 2: 0.025}[prec]
    assert lo <= e_gpu / n <= hi or abs(e_gpu - e_ref) <= 3 * math.sqrt(max(e_ref, 1))


@pytest.mark.parametrize("prec", [1, 2])
def test_reduced_precision_24x24_kron_slot(ctx, prec):
    """The 24-user Kronecker slot at its full size and SNR (3276 subcarriers
    x 14 symbols, rho 0.5 / 0.3, 18 dB, 256 paths) in FP16 / BF16 path
    metrics, against the FP64 oracle on the first 128 subcarriers."""
    _say("precision full 24x24 slot", prec)
    S, T, M, N, bits, K, n_sub = 3276, 14, 24, 24, 4, 256, 128
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=18, seed=(1, 0, 0, 0), channel="kron",
                         rho_rx=0.5, rho_tx=0.3)
    ctx.set_precision(prec)
    try:
        got = _run(ctx, sl, K)[:, :n_sub]
    finally:
        ctx.set_precision(0)
    ref = oracle.detect_slot("mpnl", sl.H[:n_sub], np.ascontiguousarray(sl.y[:, :n_sub]), bits, n_paths=K,
                             nthreads=16)
    n_mis = int(np.sum(np.any(got != ref, axis=-1)))
    s_idx = sl.s_idx[:, :n_sub]
    n = s_idx.size * bits
    e_gpu, e_ref = synth.bit_errors(got, s_idx, bits), synth.bit_errors(ref, s_idx, bits)
    print(f"prec {prec}: {n_mis} of {ref.shape[0] * ref.shape[1]} vectors differ, bit errors gpu {e_gpu} "
          f"oracle {e_ref} of {n}", flush=True)
    assert n_mis <= 0.005 * ref.shape[0] * ref.shape[1]
    lo, hi = synth.wilson(e_ref, n)
    assert lo <= e_gpu / n <= hi or abs(e_gpu - e_ref) <= 3 * math.sqrt(max(e_ref, 1))


# ---------------------------------------------------------- soft output ---
@pytest.mark.parametrize("snr,K,bits", [(10, 64, 4), (0, 200, 4), (2, 300, 6), (-3, 256, 2)])
def test_soft_output_matches_oracle(ctx, snr, K, bits):
    """Max-log LLRs use every path's metric, so they check the k-th-best
    choice of all paths, including received points far outside the
    constellation (low SNR) and more paths than one workgroup."""
    _say("soft", snr, K, bits)
    S, T, M, N = 12, 3, 6, 4
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=(214, snr + 100, K))
    slot = ctx.slot_prepare(_dev(sl.H), bits, K)
    out = torch.empty((T, S, N), dtype=torch.int32, device="cuda:0")
    llr = slot.detect_soft(_dev(sl.y), sl.sigma2, 50.0, out=out)
    torch.cuda.synchronize()
    slot.release()
    llr = llr.cpu().numpy()
    got = out.cpu().numpy()
    ref, diag = oracle.detect_slot("mpnl", sl.H, sl.y, bits, n_paths=K, want_diag=True)
    check(sl.H, sl.y, got, ref, diag, bits, label=f"soft {snr} dB")
    n_skip = 0
    for s in range(S):
        Q, R, perm, _ = oracle.sqrd(sl.H[s])
        P, _, _ = oracle.position_set(oracle.depth_weights(R), 1 << bits, K)
        for t in range(T):
            r = oracle.mpnl_vector(Q, R, perm, P, sl.y[t, s], bits)
            ol = oracle.llr_from_paths(r["metrics"], r["paths"], bits, sl.sigma2, 50.0)
            # every path's metric enters the LLRs: a near-tie on any path counts
            if r["kth_margin_all"] < TOL:
                n_skip += 1
                continue
            assert np.allclose(llr[t, s], ol, rtol=1e-3, atol=2e-3 * max(1.0, np.abs(ol).max())), (t, s)
    print(f"soft {snr} dB: {n_skip} of {S * T} vectors skipped for a near-tie on some path", flush=True)
    assert n_skip <= max(1, 0.05 * S * T)


@pytest.mark.parametrize("shape", [(400, 14, 16, 16, 4, 256, 16.0, "iid"), (300, 14, 24, 24, 4, 256, 18.0, "kron"),
                                   (200, 14, 30, 28, 6, 128, 20.0, "iid"), (150, 14, 8, 8, 2, 300, 6.0, "iid"),
                                   (300, 3, 12, 12, 4, 64, 10.0, "iid")])
def test_pruning_changes_no_decision(mp, shape):
    """Pruned search (waves stop once every path exceeds path 0's metric) and
    the full search give identical symbols, in every precision and through
    the batched and planned launches."""
    S, T, M, N, bits, K, snr, ch = shape
    _say("pruning", shape)
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=(230, S, N), channel=ch,
                         rho_rx=0.5, rho_tx=0.3)
    H, y = _dev(sl.H), _dev(sl.y)
    full = mp.Context(0, prune=False)
    pruned = mp.Context(0)
    try:
        for prec in (0, 1, 2):
            full.set_precision(prec)
            pruned.set_precision(prec)
            a = full.detect(H, y, bits, K)
            b = pruned.detect(H, y, bits, K)
            c = pruned.detect_batch([dict(H=H, y=y, mod=bits, n_paths=K, out=None)])[0]
            torch.cuda.synchronize()
            assert torch.equal(a, b), prec
            assert torch.equal(a, c), prec
            if K <= 256:
                plan = pruned.batch_plan([dict(S=S, T=T, M=M, N=N, mod=bits, n_paths=K)])
                try:
                    out = torch.full((T, S, N), -1, dtype=torch.int32, device="cuda:0")
                    plan.run([dict(H=H, y=y, mod=bits, n_paths=K, out=out)])
                    torch.cuda.synchronize()
                    assert torch.equal(a, out), prec
                finally:
                    plan.close()
    finally:
        full.close()
        pruned.close()


def test_near_ml_at_16_users(ctx):
    """16 users x 16 antennas, 16-QAM, 10 dB, 256 paths: the GPU decisions
    follow the FP64 oracle (parity protocol) and leave the exact ML decision
    (sphere decoder) on at most 0.5% of the vectors, each time for a vector
    with a larger residual."""
    _say("near-ML 16x16")
    S, T, M, N, bits, K = 150, 14, 16, 16, 4, 256
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=10.0, seed=(804,))
    got = _run(ctx, sl, K)
    _assert_parity(sl, got, K, nthreads=16, label="16x16 10 dB")
    ml = oracle.detect_slot("sphere", sl.H, sl.y, bits, nthreads=16)
    off = np.any(got != ml, axis=-1)
    for t, s in zip(*np.nonzero(off)):
        assert oracle.residual_norm2(sl.H[s], sl.y[t, s], bits, got[t, s]) >= \
            oracle.residual_norm2(sl.H[s], sl.y[t, s], bits, ml[t, s]) * (1 - 1e-12)
    nb = sl.s_idx.size * bits
    print(f"off ML: {off.sum()} of {off.size} vectors; bit errors GPU {synth.bit_errors(got, sl.s_idx, bits)}, "
          f"ML {synth.bit_errors(ml, sl.s_idx, bits)} of {nb}", flush=True)
    assert off.mean() <= 0.005
