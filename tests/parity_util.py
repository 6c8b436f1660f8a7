"""Shared helpers of the GPU parity tests (oracle side only; no HIP code).

Decisions must equal the FP64 oracle's except for vectors whose oracle
diagnostics show a relative margin below TOL in one of the four places where
floating point decides an integer: the sorted-QR pivot, the position-set
boundary, a k-th-best ordering on any path, or best versus second-best path
metric.  As a last escape hatch the two decisions' FP64 ||y - H s||^2 may lie
within TOL of each other.  Anything else is a bug.
"""
import numpy as np

import oracle

TOL = 1e-5
CLASSES = ("pivot", "boundary", "kth", "metric")
# Near-ties are rare with continuous noise: at most this fraction of the
# vectors of a case may be excused, so a widened margin cannot hide a bug.
MAX_EXCUSED_FRAC = 0.005


def classify(H, y, got, ref, diag, bits, tol=TOL):
    """H (S,M,N), y (T,S,M), got/ref (T,S,N), diag (T,S,4).

    Returns (n_mismatch, counts per class, list of unexplained mismatches)."""
    bad_t, bad_s = np.nonzero(np.any(got != ref, axis=-1))
    counts = {c: 0 for c in CLASSES + ("residual",)}
    unexplained = []
    for t, s in zip(bad_t, bad_s):
        d = diag[t, s]
        k = int(np.argmin(d))
        if d[k] < tol:
            counts[CLASSES[k]] += 1
            continue
        r_got = oracle.residual_norm2(H[s], y[t, s], bits, got[t, s])
        r_ref = oracle.residual_norm2(H[s], y[t, s], bits, ref[t, s])
        if abs(r_got - r_ref) <= tol * max(r_got, r_ref):
            counts["residual"] += 1
            continue
        unexplained.append(dict(t=int(t), s=int(s), margins=d.tolist(), r_ref=r_ref, r_got=r_got,
                                got=got[t, s].tolist(), ref=ref[t, s].tolist()))
    return len(bad_t), counts, unexplained


def check(H, y, got, ref, diag, bits, label="", tol=TOL, max_excused_frac=MAX_EXCUSED_FRAC):
    """classify(), print the counts, and fail on any unexplained mismatch or
    when more than max_excused_frac of the vectors (at least one allowed)
    needed an excuse.
    -> (n_mismatch, n_excused)."""
    n_bad, counts, unexplained = classify(H, y, got, ref, diag, bits, tol)
    n_vec = int(np.prod(ref.shape[:-1]))
    n_exc = n_bad - len(unexplained)
    print(f"{label}: {n_bad} of {n_vec} vectors differ, {n_exc} excused ({counts})", flush=True)
    assert not unexplained, unexplained[:3]
    assert n_exc <= max(1.0, max_excused_frac * n_vec), (n_exc, n_vec, counts)
    return n_bad, n_exc
