"""Pins of the oracle's near-tie margins (the four parity classes).

The parity tests excuse a GPU decision that differs from the oracle's only
where one of the oracle's margins is below 1e-5: the sorted-QR pivot, the
position-set boundary, a k-th-best choice that could still change the
result, and best versus second-best path metric.  Those margins decide which
mismatches pass, so they are recomputed here independently of the oracle's C
code, in numpy, from the definitions:

* pivot    -- greedy column order from least-squares residuals (numpy lstsq)
              at every step, smallest relative gap between the chosen
              residual and any other remaining one;
* boundary -- all |Q|^N position vectors scored and sorted (score, then
              lexicographic), relative gap between ranks K and K + 1;
* kth      -- every path's descent with a full stable sort of all
              constellation distances at each depth (numpy QR for R), the
              relative gap of the chosen rank to its neighbours over the
              (path, depth) pairs whose partial metric is not above the
              final minimum (padded by 1e-3) and whose R_ll is not zero;
* metric   -- relative gap between the smallest and second smallest path
              metric.

Each must match the oracle to 1e-12 on >= 50 vectors at three sizes, and
planted ties must show a margin below 1e-5 (Sec. II: the N_p candidates and
the selection of the best are what these margins guard).
"""
import itertools

import numpy as np
import pytest

import oracle
import synth

TOL = 1e-5
KTH_REACH = 1e-3


def rel_gap(a, b):
    m = max(abs(a), abs(b))
    return 0.0 if m == 0.0 else abs(a - b) / m


def gray_points(bits):
    """Square QAM, unit energy; index = (Gray(I level) << h) | Gray(Q level)."""
    h = bits // 2
    L = 1 << h
    delta = np.sqrt(3.0 / (2.0 * (L * L - 1)))
    level_of_label = np.zeros(L, np.int64)
    for m in range(L):
        level_of_label[m ^ (m >> 1)] = m
    idx = np.arange(1 << bits)
    mi = level_of_label[idx >> h]
    mq = level_of_label[idx & (L - 1)]
    return ((2 * mi - L + 1) + 1j * (2 * mq - L + 1)) * delta


def np_sqrd(H):
    """Greedy order by least-squares residuals, then numpy QR of the permuted
    channel with the diagonal of R made real positive."""
    M, N = H.shape
    placed, margin = [], np.inf
    for _ in range(N):
        rest = [k for k in range(N) if k not in placed]
        res = {}
        for k in rest:
            h = H[:, k]
            if placed:
                A = H[:, placed]
                coef = np.linalg.lstsq(A, h, rcond=None)[0]
                h = h - A @ coef
            res[k] = float(np.vdot(h, h).real)
        kmin = min(rest, key=lambda k: (res[k], k))
        for k in rest:
            if k != kmin:
                margin = min(margin, rel_gap(res[kmin], res[k]))
        placed.append(kmin)
    perm = np.array(placed)
    Hp = H[:, perm]
    # exactly zero columns (residual 0) come first; they get a zero column of
    # Q and a zero row of R, the factorisation of the others is unchanged
    z = int(np.sum(~np.any(Hp != 0, axis=0)))
    assert np.all(np.any(Hp[:, z:] != 0, axis=0))
    Q = np.zeros((M, N), np.complex128)
    R = np.zeros((N, N), np.complex128)
    if z < N:
        Qn, Rn = np.linalg.qr(Hp[:, z:])
        ph = np.diag(Rn) / np.abs(np.diag(Rn))
        Q[:, z:] = Qn * ph[None, :]
        R[z:, z:] = np.conj(ph)[:, None] * Rn
    return Q, R, perm, margin


def np_depth_costs(w_depth):
    """Integer depth costs: each weight in units of 2^-20 of the largest,
    rounded half to even (0 for a weight that is not a number, or when the
    largest is not positive and finite)."""
    w = np.asarray(w_depth, np.float64)
    wmax = max([0.0] + [x for x in w.tolist() if x > 0.0])
    if not (0.0 < wmax < np.inf):
        return np.zeros_like(w)
    with np.errstate(invalid="ignore"):
        x = (w / wmax) * float(1 << 20)
        ok = (x >= 0.0) & (x <= float(1 << 20))
    return np.where(ok, np.rint(np.where(ok, x, 0.0)), 0.0)


def np_position_set(w_depth, nq, K):
    """All |Q|^N vectors (depth order, entries 1..nq), sorted by integer cost,
    equal costs by the costs of the prefixes (longest first), then
    lexicographically; -> (first K vectors, boundary margin)."""
    N = len(w_depth)
    P = np.array(list(itertools.product(range(1, nq + 1), repeat=N)), dtype=np.int64)
    terms = (P - 1) * np_depth_costs(w_depth).astype(np.int64)[None, :]
    prefix = np.cumsum(terms, axis=1)          # prefix[:, j - 1] = cost of the first j depths
    score = prefix[:, -1].astype(np.float64)
    # np.lexsort: the last key is the primary one
    keys = [P[:, d] for d in range(N - 1, -1, -1)] + [prefix[:, j] for j in range(N)]
    order = np.lexsort(keys)
    P, score = P[order], score[order]
    K = min(K, len(P))
    boundary = rel_gap(score[K - 1], score[K]) if K < len(P) else np.inf
    return P[:K], boundary


def np_mpnl(Q, R, perm, P, y, bits):
    """Every path's descent; -> (decisions in user order, kth margin, metric margin)."""
    pts = gray_points(bits)
    nq = len(pts)
    N = R.shape[0]
    K = P.shape[0]
    yt = np.conj(Q).T @ y
    s = np.zeros((K, N), np.complex128)
    sidx = np.zeros((K, N), np.int64)
    metric = np.zeros(K)
    gaps = np.full((K, N), np.inf)
    partial = np.zeros((K, N))
    rows = np.arange(K)
    for d in range(N):
        l = N - 1 - d
        b = yt[l] - s[:, l + 1:] @ R[l, l + 1:]
        dist = np.abs(b[:, None] - R[l, l] * pts[None, :]) ** 2
        order = np.argsort(dist, axis=1, kind="stable")  # (distance, index)
        sd = np.take_along_axis(dist, order, axis=1)
        k = P[:, d] - 1
        c = order[rows, k]
        if R[l, l] != 0:
            g = np.full(K, np.inf)
            lo = k > 0
            g[lo] = np.minimum(g[lo], [rel_gap(a, b_) for a, b_ in zip(sd[rows[lo], k[lo] - 1], sd[rows[lo], k[lo]])])
            hi = k + 1 < nq
            g[hi] = np.minimum(g[hi], [rel_gap(a, b_) for a, b_ in zip(sd[rows[hi], k[hi]], sd[rows[hi], k[hi] + 1])])
            gaps[:, d] = g
        s[:, l] = pts[c]
        sidx[:, l] = c
        metric = metric + dist[rows, c]
        partial[:, d] = metric
    best_r = int(np.argmin(metric))
    best = metric[best_r]
    reach = partial <= best * (1.0 + KTH_REACH)
    kth = float(gaps[reach].min()) if reach.any() else np.inf
    if K > 1:
        second = np.min(np.delete(metric, best_r))
        met = rel_gap(best, second)
    else:
        met = np.inf
    out = np.zeros(N, np.int64)
    out[perm] = sidx[best_r]
    np_mpnl.kth_all = float(gaps.min())
    return out, kth, met


def np_margins_slot(H, y, bits, K):
    """-> decisions (T,S,N) and margins (T,S,4) [pivot, boundary, kth, metric]."""
    S, M, N = H.shape
    T = y.shape[0]
    nq = 1 << bits
    dec = np.zeros((T, S, N), np.int64)
    mg = np.zeros((T, S, 4))
    for s_ in range(S):
        Q, R, perm, piv = np_sqrd(H[s_].astype(np.complex128))
        w = np.abs(np.diag(R))[::-1] ** 2
        P, bnd = np_position_set(w, nq, K)
        for t in range(T):
            o, kth, met = np_mpnl(Q, R, perm, P, y[t, s_].astype(np.complex128), bits)
            dec[t, s_] = o
            mg[t, s_] = (piv, bnd, kth, met)
    return dec, mg


CASES = [
    # (S, T, M, N, bits, K, snr dB)
    (20, 3, 3, 3, 4, 64, 12.0),   # 16-QAM 3x3, 64 of 4096 vectors
    (25, 2, 6, 4, 2, 16, 6.0),    # QPSK 4 users on 6 antennas, 16 of 256
    (30, 2, 2, 2, 6, 100, 20.0),  # 64-QAM 2x2, 100 of 4096
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"S{c[0]}T{c[1]}M{c[2]}N{c[3]}b{c[4]}K{c[5]}")
def test_margins_match_independent_numpy(case):
    S, T, M, N, bits, K, snr = case
    sl = synth.make_slot(S=S, T=T, M=M, N=N, bits=bits, snr_db=snr, seed=(80, N, bits))
    ref, diag = oracle.detect_slot("mpnl", sl.H, sl.y, bits, n_paths=K, want_diag=True)
    dec, mg = np_margins_slot(sl.H, sl.y, bits, K)
    assert S * T >= 50
    assert np.array_equal(dec, ref)
    both_inf = np.isinf(diag) & np.isinf(mg)
    assert np.array_equal(np.isinf(diag), np.isinf(mg))
    err = np.where(both_inf, 0.0, np.abs(np.where(both_inf, 0.0, diag) - np.where(both_inf, 0.0, mg)))
    assert err.max() <= 1e-12, (err.max(), np.unravel_index(np.argmax(err), err.shape))
    # the margins are informative: generic inputs are rarely near ties
    assert np.mean(diag.min(axis=-1) < TOL) < 0.05


def test_planted_pivot_and_boundary_ties():
    # two orthogonal columns of equal norm: the pivot order is a tie, and
    # with equal weights ranks 2 and 3 of the position set tie (scores w, w)
    H = np.eye(2, dtype=np.complex64)[None]
    y = np.array([[[0.3 + 0.2j, -0.6 + 0.1j]]], np.complex64)
    _, diag = oracle.detect_slot("mpnl", H, y, 2, n_paths=2, want_diag=True)
    assert diag[0, 0, 0] < TOL and diag[0, 0, 1] < TOL
    _, mg = np_margins_slot(H, y, 2, 2)
    assert mg[0, 0, 0] < TOL and mg[0, 0, 1] < TOL


def test_planted_kth_and_metric_ties_on_the_winner():
    # user 1 (detected first) received exactly between two QPSK points on the
    # in-phase axis: the winner's first choice is a tie, and the path taking
    # the other point (position vector (2, 1), rank 3) has the same metric
    a = 1 / np.sqrt(2)
    H = np.diag([1.0, 1.3]).astype(np.complex64)[None]
    y = np.array([[[a + 1j * a, 1.3 * (0.0 + 1j * a)]]], np.complex64)
    _, diag = oracle.detect_slot("mpnl", H, y, 2, n_paths=4, want_diag=True)
    assert diag[0, 0, 2] < TOL
    assert diag[0, 0, 3] < TOL
    _, mg = np_margins_slot(H, y, 2, 4)
    assert mg[0, 0, 2] < TOL and mg[0, 0, 3] < TOL


def test_tie_on_a_path_that_cannot_win_is_not_a_near_tie():
    # noise-free y on a constellation point: the winner has metric 0, and the
    # tie between ranks 2 and 3 (the in-phase and quadrature neighbours) on
    # other paths happens where their partial metric is already above 0
    a = 1 / np.sqrt(2)
    H = np.diag([1.0, 1.3]).astype(np.complex64)[None]
    y = np.array([[[a + 1j * a, 1.3 * (-a + 1j * a)]]], np.complex64)
    _, diag = oracle.detect_slot("mpnl", H, y, 2, n_paths=16, want_diag=True)
    assert diag[0, 0, 2] > 0.5
    _, mg = np_margins_slot(H, y, 2, 16)
    assert abs(mg[0, 0, 2] - diag[0, 0, 2]) <= 1e-12


def test_zero_diagonal_depth_is_not_a_near_tie():
    # a zero column: every point ties at its depth; both sides take the k-th
    # in index order there by rule, so it is not counted as a near-tie
    rng = np.random.default_rng(5)
    H = (rng.standard_normal((1, 4, 3)) + 1j * rng.standard_normal((1, 4, 3))).astype(np.complex64)
    H[:, :, 1] = 0
    y = (rng.standard_normal((2, 1, 4)) + 1j * rng.standard_normal((2, 1, 4))).astype(np.complex64)
    _, diag = oracle.detect_slot("mpnl", H, y, 4, n_paths=16, want_diag=True)
    _, mg = np_margins_slot(H, y, 4, 16)
    fin = np.isfinite(diag[..., 2])
    assert np.array_equal(fin, np.isfinite(mg[..., 2]))
    assert np.all(np.abs(diag[..., 2][fin] - mg[..., 2][fin]) <= 1e-12)


def test_all_paths_kth_margin_matches_numpy():
    """The margin over every (path, depth) pair, which soft output needs."""
    sl = synth.make_slot(S=6, T=3, M=5, N=3, bits=4, snr_db=4.0, seed=(81,))
    for s_ in range(6):
        Q, R, perm, _ = oracle.sqrd(sl.H[s_])
        P, _, _ = oracle.position_set(oracle.depth_weights(R), 16, 40)
        Qn, Rn, permn, _ = np_sqrd(sl.H[s_].astype(np.complex128))
        Pn, _ = np_position_set(np.abs(np.diag(Rn))[::-1] ** 2, 16, 40)
        for t in range(3):
            r = oracle.mpnl_vector(Q, R, perm, P, sl.y[t, s_], 4)
            np_mpnl(Qn, Rn, permn, Pn, sl.y[t, s_].astype(np.complex128), 4)
            assert abs(r["kth_margin_all"] - np_mpnl.kth_all) <= 1e-12
            assert r["kth_margin_all"] <= r["kth_margin"]
