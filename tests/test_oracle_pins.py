"""Pins of the FP64 oracle against facts fixed by the mathematics.

The paper prints no worked detection example, so each oracle function is tied
to something other than itself: an independent evaluation of a definition,
an identity between two different algorithms, a closed form, an invariant or
a brute-force enumeration.  A dropped term, a wrong sign or index, or a
transposed operand in the oracle breaks at least one of these.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.filterwarnings("ignore")


def _brute_ml_numpy(H, y, bits):
    """Independent numpy evaluation of argmin ||y - H s||^2 over Q^N."""
    pts = synth._tx_points(bits)
    M, N = H.shape
    nq = len(pts)
    allidx = np.array(list(itertools.product(range(nq), repeat=N)), np.int64)
    S = pts[allidx]                                   # (|Q|^N, N)
    r = y.astype(np.complex128)[None, :] - S @ H.astype(np.complex128).T
    m = np.sum(np.abs(r) ** 2, axis=1)
    k = int(np.argmin(m))                             # first minimum = lexicographic
    return allidx[k].astype(np.int32), float(m[k]), m, allidx


# --------------------------------------------------------------------- ML ---
@pytest.mark.parametrize("M,N,bits", [(4, 4, 2), (3, 2, 4), (2, 2, 6), (6, 4, 2)])
def test_ml_equals_numpy_brute_force(M, N, bits):
    sl = synth.make_slot(S=6, T=1, M=M, N=N, bits=bits, snr_db=8, seed=(101, M, N, bits))
    for s in range(6):
        idx, met = oracle.ml(sl.H[s], sl.y[0, s], bits)
        ref, rmet, _, _ = _brute_ml_numpy(sl.H[s], sl.y[0, s], bits)
        assert np.array_equal(idx, ref)
        assert abs(met - rmet) <= 1e-12 * max(1.0, rmet)


def test_ml_qr_form_same_argmin():
    """||y-Hs||^2 = sum_l |yt_l - sum_{j>=l} R_lj s'_j|^2 + ||(I-QQ^H) y||^2,
    evaluated with numpy's own (unsorted) QR: same argmin, same metric."""
    bits = 4
    sl = synth.make_slot(S=5, T=1, M=4, N=3, bits=bits, snr_db=12, seed=(102,))
    pts = synth._tx_points(bits)
    for s in range(5):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        Qn, Rn = np.linalg.qr(H)
        yt = Qn.conj().T @ y
        const = np.linalg.norm(y - Qn @ yt) ** 2
        allidx = np.array(list(itertools.product(range(16), repeat=3)))
        m = np.sum(np.abs(yt[None] - pts[allidx] @ Rn.T) ** 2, axis=1) + const
        idx, met = oracle.ml(H, y, bits)
        assert np.array_equal(idx, allidx[np.argmin(m)])
        assert abs(met - m.min()) < 1e-10


# ------------------------------------------------------------------- SQRD ---
@pytest.mark.parametrize("M,N,ch", [(4, 4, "iid"), (16, 16, "iid"), (32, 12, "iid"), (24, 24, "kron")])
def test_sqrd_properties(M, N, ch):
    sl = synth.make_slot(S=4, T=1, M=M, N=N, bits=4, snr_db=18, seed=(103, M, N),
                         channel=ch, rho_rx=0.5, rho_tx=0.3)
    for s in range(4):
        H = sl.H[s].astype(np.complex128)
        Q, R, perm, margin = oracle.sqrd(H)
        assert sorted(perm.tolist()) == list(range(N))
        assert np.abs(Q.conj().T @ Q - np.eye(N)).max() < 1e-12
        assert np.abs(Q @ R - H[:, perm]).max() < 1e-12 * np.abs(H).max()
        assert np.allclose(np.tril(R, -1), 0)
        assert np.all(np.abs(np.imag(np.diag(R))) == 0) and np.all(np.real(np.diag(R)) > 0)
        assert margin > 0
        # greedy property, checked with independent least-squares projections
        for i in range(N):
            placed = H[:, perm[:i]]

            def resid(col):
                if i == 0:
                    return np.linalg.norm(col) ** 2
                c, *_ = np.linalg.lstsq(placed, col, rcond=None)
                return np.linalg.norm(col - placed @ c) ** 2

            chosen = resid(H[:, perm[i]])
            assert abs(chosen - R[i, i].real ** 2) < 1e-9 * max(1.0, chosen)
            for k in perm[i + 1:]:
                assert chosen <= resid(H[:, k]) * (1 + 1e-9)


def test_sqrd_tie_goes_to_lower_column():
    # two columns of identical norm and orthogonal: pivot order must follow the index
    H = np.array([[2, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 0]], np.complex128)
    _, R, perm, margin = oracle.sqrd(H)
    assert perm.tolist() == [1, 2, 0]
    assert margin == 0.0


# ------------------------------------------------------------ position set ---
@pytest.mark.parametrize("N,nq,K,seed", [(4, 4, 256, 1), (3, 16, 200, 2), (2, 64, 4096, 3),
                                         (5, 4, 700, 4), (4, 16, 4096, 5)])
def test_position_set_equals_brute_force(N, nq, K, seed):
    rng = np.random.default_rng(seed)
    w = rng.exponential(size=N)
    P, sc, _ = oracle.position_set(w, nq, K)
    P2, sc2 = oracle.position_set_brute(w, nq, K)
    assert np.array_equal(P, P2)
    assert np.array_equal(sc, sc2)
    assert np.all(np.diff(sc) >= 0)
    assert P[0].tolist() == [1] * N


@pytest.mark.parametrize("w", [[1.0, 1.0, 1.0], [0.0, 2.0, 0.0], [0.0, 0.0, 0.0], [3.0, 1.5, 0.5]])
def test_position_set_ties_by_prefix_costs_then_lexicographic(w):
    w = np.array(w)
    P, sc, bm = oracle.position_set(w, 4, 64)
    P2, sc2 = oracle.position_set_brute(w, 4, 64)
    assert np.array_equal(P, P2)
    # explicit check of the order: (C_N, C_{N-1}, ..., C_1, p lexicographic),
    # C_j the cost of the first j depths, from the integer depth costs
    c = [round(x / max(w) * 2 ** 20) if max(w) > 0 else 0 for x in w]
    def key(p):
        pre = [sum(c[e] * (p[e] - 1) for e in range(j)) for j in range(len(p), 0, -1)]
        return tuple(pre) + tuple(p)
    keys = [key(p) for p in P.tolist()]
    assert keys == sorted(keys)
    assert [k[0] for k in keys] == sc.tolist()


@pytest.mark.parametrize("w,c1", [([1.0, 2.5 * 2.0 ** -20], 2),    # 2.5 units: half to even, down
                                   ([1.0, 3.5 * 2.0 ** -20], 4),    # 3.5 units: half to even, up
                                   ([4.0, 1.0], 2 ** 18),           # a quarter of the largest
                                   ([2.0, float("nan")], 0),        # not a number: cost 0
                                   ([0.0, 0.0], 0)])                # no positive weight: all 0
def test_position_set_integer_depth_costs(w, c1):
    """The scores are sums of integer depth costs: the weights in units of
    2^-20 of the largest, rounded half to even.  With two depths the second
    vector of the set is (1, 2), whose score is the cost of depth 1."""
    P, sc, _ = oracle.position_set(np.array(w), 4, 3)
    c0 = 2 ** 20 if max([x for x in w if x == x]) > 0 else 0
    if c1 > 0:
        assert P[:2].tolist() == [[1, 1], [1, 2]] and sc[1] == c1
    assert sc[0] == 0
    # every score is the integer combination sum_d c_d (p_d - 1)
    assert np.array_equal(sc, (P.astype(np.int64) - 1) @ np.array([c0, c1]))


def test_position_set_nested_and_clamped():
    w = np.array([0.3, 1.7, 0.9, 2.2])
    P64, _, _ = oracle.position_set(w, 4, 64)
    P200, _, _ = oracle.position_set(w, 4, 200)
    assert np.array_equal(P200[:64], P64)
    Pall, _, bm = oracle.position_set(w, 4, 10 ** 6)
    assert Pall.shape == (256, 4) and math.isinf(bm)
    assert len({tuple(p) for p in Pall.tolist()}) == 256


# -------------------------------------------------------------------- MPNL ---
def _mpnl(H, y, bits, n_paths):
    Q, R, perm, _ = oracle.sqrd(H)
    P, _, _ = oracle.position_set(oracle.depth_weights(R), 1 << bits, n_paths)
    return oracle.mpnl_vector(Q, R, perm, P, y, bits)


@pytest.mark.parametrize("M,N,bits,nvec", [(4, 4, 2, 24), (2, 2, 4, 24), (3, 3, 4, 6),
                                           (2, 2, 6, 6), (6, 4, 2, 12), (4, 4, 4, 2)])
def test_mpnl_all_paths_is_ml(M, N, bits, nvec):
    """With every position vector the path list is all of Q^N: exactly ML."""
    sl = synth.make_slot(S=nvec, T=1, M=M, N=N, bits=bits, snr_db=6, seed=(104, M, N, bits))
    total = (1 << bits) ** N
    for s in range(nvec):
        H, y = sl.H[s], sl.y[0, s]
        r = _mpnl(H, y, bits, total)
        ml, mlm = oracle.ml(H, y, bits)
        assert np.array_equal(r["idx"], ml)
        Q, _, _, _ = oracle.sqrd(H)
        yy = y.astype(np.complex128)
        const = np.linalg.norm(yy - Q @ (Q.conj().T @ yy)) ** 2
        assert abs(r["metric"] + const - mlm) < 1e-9 * max(1, mlm)
        # every symbol vector appears exactly once among the paths
        assert len({tuple(p) for p in r["paths"].tolist()}) == total


@pytest.mark.parametrize("M,N,bits,ch", [(4, 4, 2, "iid"), (16, 16, 4, "iid"), (24, 24, 4, "kron"),
                                         (12, 8, 6, "iid"), (1, 1, 4, "iid")])
def test_mpnl_one_path_is_ordered_zfsic(M, N, bits, ch):
    sl = synth.make_slot(S=12, T=1, M=M, N=N, bits=bits, snr_db=10, seed=(105, M, N),
                         channel=ch, rho_rx=0.5, rho_tx=0.3)
    for s in range(12):
        H, y = sl.H[s], sl.y[0, s]
        Q, R, perm, _ = oracle.sqrd(H)
        r = _mpnl(H, y, bits, 1)
        assert np.array_equal(r["idx"], oracle.zfsic(H, y, bits, perm))


def test_mpnl_monotone_in_paths():
    bits = 4
    sl = synth.make_slot(S=8, T=1, M=8, N=8, bits=bits, snr_db=8, seed=(106,))
    for s in range(8):
        H, y = sl.H[s], sl.y[0, s]
        prev = np.inf
        for n_paths in (1, 4, 16, 64, 256):
            m = _mpnl(H, y, bits, n_paths)["metric"]
            assert m <= prev
            prev = m


def test_mpnl_metric_lower_bounded_by_ml():
    bits = 2
    sl = synth.make_slot(S=10, T=1, M=5, N=5, bits=bits, snr_db=4, seed=(107,))
    for s in range(10):
        H, y = sl.H[s], sl.y[0, s]
        Q, _, _, _ = oracle.sqrd(H)
        yy = y.astype(np.complex128)
        const = np.linalg.norm(yy - Q @ (Q.conj().T @ yy)) ** 2
        _, mlm = oracle.ml(H, y, bits)
        for n_paths in (1, 8, 64):
            assert _mpnl(H, y, bits, n_paths)["metric"] + const >= mlm - 1e-9


def test_paths_are_distinct_symbol_vectors():
    bits = 4
    sl = synth.make_slot(S=3, T=1, M=8, N=6, bits=bits, snr_db=10, seed=(108,))
    for s in range(3):
        r = _mpnl(sl.H[s], sl.y[0, s], bits, 256)
        assert len({tuple(p) for p in r["paths"].tolist()}) == 256
        # each path's metric equals the QR-form residual of its own symbol vector
        Q, R, perm, _ = oracle.sqrd(sl.H[s])
        yy = sl.y[0, s].astype(np.complex128)
        const = np.linalg.norm(yy - Q @ (Q.conj().T @ yy)) ** 2
        for k in (0, 17, 255):
            full = oracle.residual_norm2(sl.H[s], sl.y[0, s], bits, r["paths"][k])
            assert abs(r["metrics"][k] + const - full) < 1e-9 * max(1, full)


# --------------------------------------------------------- special cases ---
@pytest.mark.parametrize("bits", [2, 4, 6])
def test_single_user_is_mrc_slicing(bits):
    sl = synth.make_slot(S=40, T=1, M=3, N=1, bits=bits, snr_db=10, seed=(109, bits))
    pts = synth._tx_points(bits)
    for s in range(40):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        x = (H[:, 0].conj() @ y) / np.linalg.norm(H[:, 0]) ** 2
        ref = int(np.argmin(np.abs(x - pts) ** 2))
        for det in (oracle.zf(H, y, bits)[0], oracle.ml(H, y, bits)[0][0],
                    _mpnl(H, y, bits, 1)["idx"][0], oracle.zfsic(H, y, bits, [0])[0]):
            assert det == ref
        g = np.linalg.norm(H[:, 0]) ** 2
        # unbiased MMSE scales the MRC estimate by a positive real: same slice
        assert oracle.mmse(H, y, bits, 0.3)[0] == ref or abs(g) < 1e-9


def test_orthogonal_channel_all_detectors_agree():
    bits = 4
    rng = np.random.default_rng(110)
    for trial in range(10):
        A = rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))
        U, _ = np.linalg.qr(A)
        H = 1.7 * U
        s = rng.integers(0, 16, 4)
        y = H @ synth._tx_points(bits)[s] + 0.3 * (rng.standard_normal(6) + 1j * rng.standard_normal(6))
        ml, _ = oracle.ml(H, y, bits)
        Q, R, perm, _ = oracle.sqrd(H)
        for det in (oracle.zf(H, y, bits), oracle.mmse(H, y, bits, 0.5), oracle.zfsic(H, y, bits, perm),
                    _mpnl(H, y, bits, 1)["idx"]):
            assert np.array_equal(det, ml)


def test_noise_free_recovers_symbols():
    for bits, M, N in ((2, 4, 4), (4, 16, 16), (6, 8, 6)):
        sl = synth.make_slot(S=6, T=1, M=M, N=N, bits=bits, snr_db=0, seed=(111, bits), noise=False)
        for s in range(6):
            r = _mpnl(sl.H[s], sl.y[0, s], bits, 16)
            assert np.array_equal(r["idx"], sl.s_idx[0, s])
            assert r["metric"] < 1e-10
            assert r["metrics"][0] == r["metric"]


def test_phase_and_scale_invariance():
    bits = 4
    sl = synth.make_slot(S=8, T=1, M=8, N=8, bits=bits, snr_db=10, seed=(112,))
    for s in range(8):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        base = _mpnl(H, y, bits, 64)
        ph = np.exp(1j * 0.7)
        rot = _mpnl(ph * H, ph * y, bits, 64)
        sc = _mpnl(2.5 * H, 2.5 * y, bits, 64)
        assert np.array_equal(base["idx"], rot["idx"])
        assert np.array_equal(base["idx"], sc["idx"])


def test_column_permutation_permutes_decisions():
    bits = 4
    sl = synth.make_slot(S=8, T=1, M=6, N=5, bits=bits, snr_db=12, seed=(113,))
    rng = np.random.default_rng(113)
    for s in range(8):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        pi = rng.permutation(5)
        a = _mpnl(H, y, bits, 32)["idx"]
        b = _mpnl(H[:, pi], y, bits, 32)["idx"]
        assert np.array_equal(b, a[pi])


def test_zero_column_ties_follow_index_order():
    bits = 2
    sl = synth.make_slot(S=4, T=1, M=4, N=3, bits=bits, snr_db=10, seed=(114,))
    for s in range(4):
        H = sl.H[s].astype(np.complex128).copy()
        H[:, 1] = 0
        y = sl.y[0, s]
        Q, R, perm, _ = oracle.sqrd(H)
        assert perm[0] == 1 and R[0, 0] == 0
        r = _mpnl(H, y, bits, 64)
        ml, _ = oracle.ml(H, y, bits)
        assert np.array_equal(r["idx"], ml)
        assert r["idx"][1] == 0


# --------------------------------------------------------------- linear ---
def test_mmse_matches_direct_solve_and_zf_limit():
    bits = 4
    sl = synth.make_slot(S=10, T=1, M=8, N=6, bits=bits, snr_db=5, seed=(115,))
    pts = synth._tx_points(bits)
    for s in range(10):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        s2 = sl.sigma2
        W = np.linalg.solve(H.conj().T @ H + s2 * np.eye(6), H.conj().T)
        x = (W @ y) / np.real(np.diag(W @ H))
        ref = np.argmin(np.abs(x[:, None] - pts[None]) ** 2, axis=1)
        assert np.array_equal(oracle.mmse(H, y, bits, s2), ref)
        xz = np.linalg.lstsq(H, y, rcond=None)[0]
        refz = np.argmin(np.abs(xz[:, None] - pts[None]) ** 2, axis=1)
        assert np.array_equal(oracle.zf(H, y, bits), refz)
        assert np.array_equal(oracle.mmse(H, y, bits, 1e-12), refz)


def test_mmse_estimate_closed_forms():
    """The unbiased estimate equals W y / (W H)_kk from numpy's solve, and
    (W H)_kk = 1 - s2 (G^-1)_kk with G = H^H H + s2 I (the identity the GPU
    MMSE uses); overloaded N > M works with s2 > 0."""
    for (M, N, seed) in ((8, 6, 116), (16, 16, 117), (4, 8, 118)):
        sl = synth.make_slot(S=4, T=1, M=M, N=N, bits=4, snr_db=8, seed=(seed,)) if N <= M else None
        rng = np.random.default_rng(seed)
        for s in range(4):
            if sl is not None:
                H = sl.H[s].astype(np.complex128)
                y = sl.y[0, s].astype(np.complex128)
            else:
                H = (rng.normal(size=(M, N)) + 1j * rng.normal(size=(M, N))) / np.sqrt(2)
                y = rng.normal(size=M) + 1j * rng.normal(size=M)
            s2 = 0.2
            G = H.conj().T @ H + s2 * np.eye(N)
            W = np.linalg.solve(G, H.conj().T)
            g = np.diag(W @ H)
            x = oracle.mmse_estimate(H, y, s2)
            assert np.allclose(x, (W @ y) / g, rtol=1e-10, atol=1e-12)
            assert np.allclose(g, 1 - s2 * np.diag(np.linalg.inv(G)), rtol=1e-10, atol=1e-12)


def test_regularized_mpnl_all_paths_is_regularized_ml():
    """Overloaded N > M: MPNL on [H; sigma I] with every path minimises
    ||y - H s||^2 + sigma^2 ||s||^2 exactly (numpy brute force)."""
    rng = np.random.default_rng(119)
    for (M, N, bits) in ((2, 3, 2), (1, 2, 4), (3, 4, 2)):
        pts = synth._tx_points(bits)
        nq = len(pts)
        cands = np.array(np.meshgrid(*[np.arange(nq)] * N, indexing="ij")).reshape(N, -1).T
        for trial in range(5):
            H = (rng.normal(size=(1, M, N)) + 1j * rng.normal(size=(1, M, N))) / np.sqrt(2)
            s_true = rng.integers(0, nq, size=N)
            y = (H[0] @ pts[s_true] + 0.3 * (rng.normal(size=M) + 1j * rng.normal(size=M)))[None, None, :]
            sigma = 0.4
            Hx, yx = oracle.regularized_system(H, y, sigma)
            got = oracle.detect_slot("mpnl", Hx, yx, bits, n_paths=nq ** N)[0, 0]
            X = pts[cands]  # (C, N)
            cost = np.sum(np.abs(y[0, 0][None, :] - X @ H[0].T) ** 2, axis=1) + sigma ** 2 * np.sum(np.abs(X) ** 2, axis=1)
            best = cands[np.argmin(cost)]
            assert np.array_equal(got, best), (M, N, bits, trial)


def test_regularized_with_zero_sigma_is_plain_mpnl():
    sl = synth.make_slot(S=6, T=3, M=8, N=6, bits=4, snr_db=12, seed=(120,))
    Hx, yx = oracle.regularized_system(sl.H, sl.y, 0.0)
    a = oracle.detect_slot("mpnl", Hx, yx, 4, n_paths=32)
    b = oracle.detect_slot("mpnl", sl.H, sl.y, 4, n_paths=32)
    assert np.array_equal(a, b)


def test_zfsic_against_projection():
    """Independent ZF-SIC: null each stream with the least-squares residual."""
    bits = 4
    sl = synth.make_slot(S=6, T=1, M=8, N=6, bits=bits, snr_db=12, seed=(116,))
    pts = synth._tx_points(bits)
    for s in range(6):
        H = sl.H[s].astype(np.complex128)
        y = sl.y[0, s].astype(np.complex128)
        perm = np.random.default_rng(s).permutation(6)
        r = y.copy()
        ref = np.zeros(6, np.int64)
        for k in range(5, -1, -1):
            x = np.linalg.lstsq(H[:, perm[:k + 1]], r, rcond=None)[0][k]
            c = int(np.argmin(np.abs(x - pts) ** 2))
            ref[perm[k]] = c
            r = r - H[:, perm[k]] * pts[c]
        assert np.array_equal(oracle.zfsic(H, y, bits, perm), ref)


# -------------------------------------------------------------- soft out ---
def test_llr_all_paths_is_exact_maxlog():
    bits = 4
    sl = synth.make_slot(S=4, T=1, M=3, N=2, bits=bits, snr_db=6, seed=(117,))
    for s in range(4):
        H, y = sl.H[s], sl.y[0, s]
        r = _mpnl(H, y, bits, 256)
        llr = oracle.llr_from_paths(r["metrics"], r["paths"], bits, sl.sigma2, 1e9)
        _, _, m, allidx = _brute_ml_numpy(H, y, bits)
        b = synth.index_bits(allidx, bits)      # (|Q|^N, N, bits)
        for u in range(2):
            for k in range(bits):
                m1 = m[b[:, u, k] == 1].min()
                m0 = m[b[:, u, k] == 0].min()
                assert abs(llr[u, k] - (m1 - m0) / sl.sigma2) < 1e-6 * max(1, abs(llr[u, k]))


def test_llr_clips_missing_hypothesis():
    mets = np.array([1.0, 2.0])
    paths = np.array([[0], [1]], np.int32)     # QPSK: first bit always 0
    llr = oracle.llr_from_paths(mets, paths, 2, 0.5, 7.0)
    assert llr[0, 0] == 7.0
    assert llr[0, 1] == pytest.approx(2.0)


# ------------------------------------------------------------ harness ---
def test_siso_awgn_qpsk_ber_closed_form():
    bits, snr_db = 2, 6.0
    S = 50000
    rng = np.random.default_rng(118)
    sl = synth.make_slot(S=S, T=1, M=1, N=1, bits=bits, snr_db=snr_db, seed=(118,))
    # AWGN: replace the fading draw by a unit channel, keeping the same symbols
    H = np.ones((S, 1, 1), np.complex64)
    x = synth._tx_points(bits)[sl.s_idx[0, :, 0]]
    n = (rng.standard_normal(S) + 1j * rng.standard_normal(S)) * math.sqrt(sl.sigma2 / 2)
    y = (x + n).astype(np.complex64)[None, :, None]
    det = oracle.detect_slot("zf", H, y, bits)
    errs = synth.bit_errors(det, sl.s_idx, bits)
    lo, hi = synth.wilson(errs, S * bits)
    assert lo <= synth.qfunc(math.sqrt(10 ** (snr_db / 10))) <= hi


def test_siso_rayleigh_qpsk_ber_closed_form():
    bits, snr_db = 2, 10.0
    S = 60000
    sl = synth.make_slot(S=S, T=1, M=1, N=1, bits=bits, snr_db=snr_db, seed=(119,))
    det = oracle.detect_slot("ml", sl.H, sl.y, bits)
    errs = synth.bit_errors(det, sl.s_idx, bits)
    g = 10 ** (snr_db / 10)
    lo, hi = synth.wilson(errs, S * bits)
    assert lo <= 0.5 * (1 - math.sqrt(g / (2 + g))) <= hi


def test_generator_constellation_unit_energy_and_gray():
    for bits in (2, 4, 6):
        pts = synth._tx_points(bits)
        assert np.allclose(oracle.constellation(bits), pts)
        assert abs(np.mean(np.abs(pts) ** 2) - 1) < 1e-12
        # Gray: nearest neighbours differ in exactly one bit
        b = synth.index_bits(np.arange(1 << bits), bits)
        dmin = np.min(np.abs(pts[:, None] - pts[None])[~np.eye(1 << bits, dtype=bool)])
        for i in range(1 << bits):
            for j in range(1 << bits):
                if i != j and abs(abs(pts[i] - pts[j]) - dmin) < 1e-9:
                    assert np.sum(b[i] != b[j]) == 1


def test_slot_driver_matches_vector_calls():
    bits = 4
    sl = synth.make_slot(S=5, T=3, M=6, N=5, bits=bits, snr_db=10, seed=(120,))
    out, diag = oracle.detect_slot("mpnl", sl.H, sl.y, bits, n_paths=32, want_diag=True, nthreads=2)
    for t in range(3):
        for s in range(5):
            r = _mpnl(sl.H[s], sl.y[t, s], bits, 32)
            assert np.array_equal(out[t, s], r["idx"])
            assert diag[t, s, 2] == r["kth_margin"]


# ------------------------------------------------------- worked example ---
def test_worked_example_diagonal_2x2_qpsk():
    """A 2x2 QPSK case small enough to derive by hand.

    H = diag(2, 1): SQRD takes the weaker column first, so perm = [1, 0],
    R = diag(1, 2) and depth 0 detects user 0 (R_11 = 2), depth 1 user 1.
    Depth weights are (4, 1), integer depth costs (2^20, 2^18) (the weights
    in units of 2^-20 of the largest), so the four cheapest position vectors
    are (1,1), (1,2), (1,3), (1,4) with scores 0, 1, 2, 3 times 2^18: every
    path keeps user 0 at its nearest point and walks user 1 through its
    1st..4th nearest.
    QPSK points: index 0 = (-D,-D), 1 = (-D,+D), 2 = (+D,-D), 3 = (+D,+D),
    D = 1/sqrt(2).  With y = (1 + 0.3j, -0.2 + 0.9j):
      user 0: z = y0 / 2 = 0.5 + 0.15j, nearest is index 3;
      user 1: z = -0.2 + 0.9j, order by distance 1, 3, 0, 2.
    The metric of each path is |y0 - 2 c0|^2 + |y1 - c1|^2.
    """
    D = 1 / math.sqrt(2)
    H = np.array([[2, 0], [0, 1]], np.complex128)
    y = np.array([1 + 0.3j, -0.2 + 0.9j])
    Q, R, perm, _ = oracle.sqrd(H)
    assert perm.tolist() == [1, 0]
    assert np.allclose(R, np.diag([1, 2]))
    w = oracle.depth_weights(R)
    assert np.allclose(w, [4, 1])
    P, sc, _ = oracle.position_set(w, 4, 4)
    assert P.tolist() == [[1, 1], [1, 2], [1, 3], [1, 4]]
    assert sc.tolist() == [0, 2 ** 18, 2 * 2 ** 18, 3 * 2 ** 18]
    r = oracle.mpnl_vector(Q, R, perm, P, y, 2)
    assert r["paths"][:, 0].tolist() == [3, 3, 3, 3]
    assert r["paths"][:, 1].tolist() == [1, 3, 0, 2]
    d0 = 4 * ((0.5 - D) ** 2 + (0.15 - D) ** 2)
    d1 = [(-0.2 + D) ** 2 + (0.9 - D) ** 2, (-0.2 - D) ** 2 + (0.9 - D) ** 2,
          (-0.2 + D) ** 2 + (0.9 + D) ** 2, (-0.2 - D) ** 2 + (0.9 + D) ** 2]
    assert np.allclose(r["metrics"], [d0 + v for v in d1], rtol=1e-14)
    assert r["idx"].tolist() == [3, 1]
