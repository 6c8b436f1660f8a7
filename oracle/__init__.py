"""FP64 CPU oracle for MPNL uplink detection (arXiv 2409.14355, Sec. II).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline may import this module; the product library never does.  The oracle
is plain C (``mpnl_oracle.c``) driven through ctypes; this file only marshals
NumPy arrays.  It shares no code with the HIP library.

Parity status of each function (what pins it is in ``tests/test_oracle_*``):
  ml              pinned (two independent evaluations, closed forms)
  sphere          pinned (= exhaustive ML on every vector of small systems,
                  never above any other detector's metric at 16 users)
  zf, mmse        pinned (direct solve, special cases)
  sqrd            pinned (orthonormality, reconstruction, greedy property)
  position_set    pinned (brute-force sort on tiny sizes)
  mpnl            pinned (= ML when every vector is used, = ZF-SIC with one path)
  zfsic           pinned (independent projection at each step)
  llr_from_paths  pinned (brute-force max-log over explicit hypotheses)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpnl_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

METHOD = {"mpnl": 0, "ml": 1, "zf": 2, "mmse": 3, "zfsic": 4, "sphere": 5}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no HIP involved)."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)
    ):
        tmp = _LIB_PATH + ".tmp"
        cmd = [
            "gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
            "-ffp-contract=off", "-fopenmp", _SRC, "-lm", "-o", tmp,
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        vp, ip, dp = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
        L.orc_constellation.argtypes = [ip, vp]
        L.orc_residual_norm2.argtypes = [vp, vp, ip, ip, ip, vp]
        L.orc_residual_norm2.restype = dp
        L.orc_ml_vector.argtypes = [vp, vp, ip, ip, ip, vp, vp]
        L.orc_zf_vector.argtypes = [vp, vp, ip, ip, ip, vp]
        L.orc_mmse_vector.argtypes = [vp, vp, ip, ip, ip, dp, vp]
        L.orc_mmse_estimate.argtypes = [vp, vp, ip, ip, dp, vp]
        L.orc_sqrd.argtypes = [vp, ip, ip, vp, vp, vp, vp]
        L.orc_num_vectors.argtypes = [ip, ip]
        L.orc_num_vectors.restype = ctypes.c_long
        L.orc_position_set.argtypes = [vp, ip, ip, ip, vp, vp, vp]
        L.orc_position_set_brute.argtypes = [vp, ip, ip, ip, vp, vp]
        L.orc_mpnl_vector.argtypes = [vp, vp, vp, vp, ip, vp, ip, ip, ip, vp, vp, vp, vp, vp]
        L.orc_zfsic_vector.argtypes = [vp, vp, ip, ip, ip, vp, vp]
        L.orc_sphere_vector.argtypes = [vp, vp, vp, vp, ip, ip, ip, ctypes.c_long, vp, vp, vp]
        L.orc_llr_from_paths.argtypes = [vp, vp, ip, ip, ip, dp, dp, vp]
        L.orc_detect_slot.argtypes = [ip, vp, vp, ip, ip, ip, ip, ip, ip, dp, vp, vp, ip]
        _lib = L
    return _lib


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _check(rc: int, what: str) -> None:
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def constellation(bits: int) -> np.ndarray:
    pts = np.zeros(1 << bits, np.complex128)
    _check(lib().orc_constellation(bits, _ptr(pts)), "constellation")
    return pts


def residual_norm2(H, y, bits: int, idx) -> float:
    H, y = _c128(H), _c128(y)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    M, N = H.shape
    return lib().orc_residual_norm2(_ptr(H), _ptr(y), M, N, bits, _ptr(idx))


def ml(H, y, bits: int):
    """Exhaustive ML for one vector -> (indices, metric)."""
    H, y = _c128(H), _c128(y)
    M, N = H.shape
    out = np.zeros(N, np.int32)
    met = ctypes.c_double()
    _check(lib().orc_ml_vector(_ptr(H), _ptr(y), M, N, bits, _ptr(out), ctypes.addressof(met)), "ml")
    return out, met.value


def zf(H, y, bits: int) -> np.ndarray:
    H, y = _c128(H), _c128(y)
    M, N = H.shape
    out = np.zeros(N, np.int32)
    _check(lib().orc_zf_vector(_ptr(H), _ptr(y), M, N, bits, _ptr(out)), "zf")
    return out


def mmse(H, y, bits: int, sigma2: float) -> np.ndarray:
    H, y = _c128(H), _c128(y)
    M, N = H.shape
    out = np.zeros(N, np.int32)
    _check(lib().orc_mmse_vector(_ptr(H), _ptr(y), M, N, bits, float(sigma2), _ptr(out)), "mmse")
    return out


def mmse_estimate(H, y, sigma2: float) -> np.ndarray:
    """Unbiased MMSE estimate x_k / (W H)_kk before slicing (complex, N)."""
    H, y = _c128(H), _c128(y)
    M, N = H.shape
    out = np.zeros(N, np.complex128)
    _check(lib().orc_mmse_estimate(_ptr(H), _ptr(y), M, N, float(sigma2), _ptr(out)), "mmse_estimate")
    return out


def sqrd(H):
    """Sorted QR -> (Q, R, perm, pivot_margin) with H[:, perm] = Q R."""
    H = _c128(H)
    M, N = H.shape
    Q = np.zeros((M, N), np.complex128)
    R = np.zeros((N, N), np.complex128)
    perm = np.zeros(N, np.int32)
    marg = ctypes.c_double()
    _check(lib().orc_sqrd(_ptr(H), M, N, _ptr(Q), _ptr(R), _ptr(perm), ctypes.addressof(marg)), "sqrd")
    return Q, R, perm, marg.value


def depth_weights(R) -> np.ndarray:
    """w_d = R_{l,l}^2 with l = N-1-d (depth order)."""
    d = np.real(np.diag(R))[::-1]
    return np.ascontiguousarray(d * d, dtype=np.float64)


def num_vectors(nq: int, N: int) -> int:
    return int(lib().orc_num_vectors(nq, N))


def position_set(w_depth, nq: int, n_paths: int):
    """Best-first position-vector set -> (P (K,N) uint8, scores (K,), boundary_margin)."""
    w = np.ascontiguousarray(w_depth, dtype=np.float64)
    N = w.shape[0]
    K = min(n_paths, num_vectors(nq, N))
    P = np.zeros((K, N), np.uint8)
    sc = np.zeros(K, np.float64)
    marg = ctypes.c_double()
    k = lib().orc_position_set(_ptr(w), N, nq, n_paths, _ptr(P), _ptr(sc), ctypes.addressof(marg))
    _check(k, "position_set")
    return P[:k], sc[:k], marg.value


def position_set_brute(w_depth, nq: int, n_paths: int):
    w = np.ascontiguousarray(w_depth, dtype=np.float64)
    N = w.shape[0]
    K = min(n_paths, num_vectors(nq, N))
    P = np.zeros((K, N), np.uint8)
    sc = np.zeros(K, np.float64)
    k = lib().orc_position_set_brute(_ptr(w), N, nq, n_paths, _ptr(P), _ptr(sc))
    _check(k, "position_set_brute")
    return P[:k], sc[:k]


def mpnl_vector(Q, R, perm, P, y, bits: int):
    """One MPNL detection -> dict(idx, metric, kth_margin, metric_margin, kth_margin_all,
    metrics, paths).  kth_margin covers the paths that could still reach the
    minimum; kth_margin_all every path (for outputs built from all paths)."""
    Q, R, y = _c128(Q), _c128(R), _c128(y)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    P = np.ascontiguousarray(P, dtype=np.uint8)
    M, N = Q.shape
    K = P.shape[0]
    out = np.zeros(N, np.int32)
    best = ctypes.c_double()
    diag = np.full(5, np.inf)
    mets = np.zeros(K, np.float64)
    paths = np.zeros((K, N), np.int32)
    _check(lib().orc_mpnl_vector(_ptr(Q), _ptr(R), _ptr(perm), _ptr(P), K, _ptr(y), M, N, bits,
                                 _ptr(out), ctypes.addressof(best), _ptr(diag), _ptr(mets),
                                 _ptr(paths)), "mpnl")
    return dict(idx=out, metric=best.value, kth_margin=diag[2], metric_margin=diag[3],
                kth_margin_all=diag[4], metrics=mets, paths=paths)


def sphere(H, y, bits: int, max_nodes: int = 200_000_000):
    """Exact ML by sphere decoding on the sorted QR of H.
    -> dict(idx (N,) int32, metric (QR form), nodes visited)."""
    H, y = _c128(H), _c128(y)
    M, N = H.shape
    Q, R, perm, _ = sqrd(H)
    out = np.zeros(N, np.int32)
    met = ctypes.c_double()
    nodes = ctypes.c_long()
    _check(lib().orc_sphere_vector(_ptr(Q), _ptr(R), _ptr(perm), _ptr(y), M, N, bits, int(max_nodes), _ptr(out),
                                   ctypes.addressof(met), ctypes.addressof(nodes)), "sphere")
    return dict(idx=out, metric=met.value, nodes=nodes.value)


def zfsic(H, y, bits: int, perm) -> np.ndarray:
    H, y = _c128(H), _c128(y)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    M, N = H.shape
    out = np.zeros(N, np.int32)
    _check(lib().orc_zfsic_vector(_ptr(H), _ptr(y), M, N, bits, _ptr(perm), _ptr(out)), "zfsic")
    return out


def llr_from_paths(metrics, paths, bits: int, sigma2: float, clip: float) -> np.ndarray:
    mets = np.ascontiguousarray(metrics, dtype=np.float64)
    paths = np.ascontiguousarray(paths, dtype=np.int32)
    K, N = paths.shape
    out = np.zeros((N, bits), np.float64)
    _check(lib().orc_llr_from_paths(_ptr(mets), _ptr(paths), K, N, bits, float(sigma2),
                                    float(clip), _ptr(out)), "llr")
    return out


def detect_slot(method: str, H, y, bits: int, n_paths: int = 1, sigma2: float = 0.0,
                nthreads: int = 1, want_diag: bool = False):
    """Whole slot: H (S,M,N), y (T,S,M) -> out (T,S,N) int32 [, diag (T,S,4)]."""
    H, y = _c128(H), _c128(y)
    S, M, N = H.shape
    T = y.shape[0]
    assert y.shape == (T, S, M)
    out = np.zeros((T, S, N), np.int32)
    diag = np.zeros((T, S, 4), np.float64) if want_diag else None
    rc = lib().orc_detect_slot(METHOD[method], _ptr(H), _ptr(y), S, T, M, N, bits, n_paths,
                               float(sigma2), _ptr(out), _ptr(diag) if want_diag else None,
                               int(nthreads))
    _check(rc, "detect_slot")
    return (out, diag) if want_diag else out


def regularized_system(H, y, sigma: float):
    """The MMSE-extended system of an overloaded (or any) slot:
    H_x = [H; sigma I_N] (S, M+N, N) and y_x = [y; 0] (T, S, M+N), so that
    ||y_x - H_x s||^2 = ||y - H s||^2 + sigma^2 ||s||^2.  MPNL on it is the
    regularised detector for N > M (the paper's overloaded regime,
    Secs. III-IV, for which it gives no method)."""
    H, y = _c128(H), _c128(y)
    S, M, N = H.shape
    T = y.shape[0]
    Hx = np.zeros((S, M + N, N), np.complex128)
    Hx[:, :M] = H
    Hx[:, M:] = sigma * np.eye(N)
    yx = np.zeros((T, S, M + N), np.complex128)
    yx[:, :, :M] = y
    return Hx, yx
