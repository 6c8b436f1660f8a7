"""Seeded synthetic uplink slots (inputs only; no detection arithmetic).

The paper evaluates on MATLAB CDL-D channels with LDPC-coded packets (Sec.
III-A/B), which are not available here.  These generators stand in for them
with the slot shape of Sec. III-B (14 OFDM symbols sharing one channel per
subcarrier) and the MIMO orders of Sec. III-A:

* H i.i.d. CN(0, 1):  (randn + j randn) / sqrt(2) per entry, or
* Kronecker exponential correlation: H = L_rx H_w L_tx^T with
  L = chol([rho^|i-j|]) over the receive antennas / users;
* s uniform over constellation indices, n ~ CN(0, sigma^2 I),
  sigma^2 = 10^(-SNR/10) (unit-energy symbols, E|h_ij|^2 = 1, so SNR is the
  per-user receive SNR);
* y = H s + n evaluated in float64, then H and y rounded once to complex64.
  Every detector (oracle or GPU) is handed the same complex64 arrays.

Seeding: NumPy PCG64 from ``SeedSequence(seed)`` where ``seed`` is a tuple of
ints such as (config, snr_index, cell, trial).

The transmit-side symbol table below is the square-QAM / per-axis Gray
mapping that both detectors implement independently.  Bit labels for BER
counting are the index bits, most significant first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Sequence

import numpy as np

MOD_BITS = {"qpsk": 2, "qam16": 4, "qam64": 6}


def _tx_points(bits: int) -> np.ndarray:
    half = bits // 2
    L = 1 << half
    delta = math.sqrt(3.0 / (2.0 * (L * L - 1)))
    level_of_gray = np.zeros(L, np.int64)
    for m in range(L):
        level_of_gray[m ^ (m >> 1)] = m
    idx = np.arange(1 << bits)
    mI = level_of_gray[idx >> half]
    mQ = level_of_gray[idx & (L - 1)]
    return ((2 * mI - L + 1) + 1j * (2 * mQ - L + 1)) * delta


def index_bits(idx: np.ndarray, bits: int) -> np.ndarray:
    """Constellation index -> bit array (..., bits), most significant first."""
    idx = np.asarray(idx, np.int64)
    sh = np.arange(bits - 1, -1, -1)
    return ((idx[..., None] >> sh) & 1).astype(np.uint8)


def _rng(seed: Sequence[int] | int) -> np.random.Generator:
    if isinstance(seed, (int, np.integer)):
        seed = [int(seed)]
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def exp_corr_chol(n: int, rho: float) -> np.ndarray:
    i = np.arange(n)
    C = rho ** np.abs(i[:, None] - i[None, :])
    return np.linalg.cholesky(C)


@dataclass
class Slot:
    H: np.ndarray        # (S, M, N) complex64
    y: np.ndarray        # (T, S, M) complex64
    s_idx: np.ndarray    # (T, S, N) int32 transmitted indices
    sigma2: float
    bits: int


def make_slot(S: int, T: int, M: int, N: int, bits: int, snr_db: float,
              seed: Sequence[int] | int, channel: str = "iid",
              rho_rx: float = 0.0, rho_tx: float = 0.0,
              noise: bool = True) -> Slot:
    rng = _rng(seed)
    Hw = (rng.standard_normal((S, M, N)) + 1j * rng.standard_normal((S, M, N))) / math.sqrt(2.0)
    if channel == "iid":
        H = Hw
    elif channel == "kron":
        Lr = exp_corr_chol(M, rho_rx)
        Lt = exp_corr_chol(N, rho_tx)
        H = Lr[None] @ Hw @ Lt.T[None]
    else:
        raise ValueError(channel)
    H = H.astype(np.complex64)
    s_idx = rng.integers(0, 1 << bits, size=(T, S, N)).astype(np.int32)
    pts = _tx_points(bits)
    x = pts[s_idx]                                   # (T,S,N)
    y = np.einsum("smn,tsn->tsm", H.astype(np.complex128), x)
    sigma2 = 10.0 ** (-snr_db / 10.0)
    if noise:
        n = (rng.standard_normal(y.shape) + 1j * rng.standard_normal(y.shape)) * math.sqrt(sigma2 / 2)
        y = y + n
    return Slot(H=H, y=y.astype(np.complex64), s_idx=s_idx, sigma2=sigma2, bits=bits)


def bit_errors(det_idx: np.ndarray, tx_idx: np.ndarray, bits: int) -> int:
    return int(np.sum(index_bits(det_idx, bits) != index_bits(tx_idx, bits)))


def wilson(k: int, n: int, z: float = 1.959964) -> tuple[float, float]:
    """Wilson score interval for a binomial proportion k / n."""
    if n == 0:
        return 0.0, 1.0
    p = k / n
    den = 1 + z * z / n
    c = (p + z * z / (2 * n)) / den
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / den
    return max(0.0, c - h), min(1.0, c + h)


def qfunc(x: float) -> float:
    return 0.5 * math.erfc(x / math.sqrt(2.0))


# Workload draws for the multi-cell batch (uneven cells).
@dataclass
class CellShape:
    N: int
    M: int
    bits: int
    S: int
    n_paths: int


def draw_cells(n_cells: int, seed: Sequence[int] | int, *, n_min=4, n_max=32,
               s_min=300, s_max=3276, paths=(64, 128, 256)) -> list[CellShape]:
    rng = _rng(seed)
    cells = []
    for _ in range(n_cells):
        N = int(rng.integers(n_min, n_max + 1))
        M = int(rng.integers(N, n_max + 1))
        bits = int(rng.choice([2, 4, 6]))
        S = int(rng.integers(s_min, s_max + 1))
        npth = int(rng.choice(list(paths)))
        cells.append(CellShape(N=N, M=M, bits=bits, S=S, n_paths=npth))
    return cells
