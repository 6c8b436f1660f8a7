"""MI355X (gfx950) MPNL uplink MIMO detection, arXiv 2409.14355 Sec. II.

Thin ctypes binding of the C ABI in ``include/mpnl.h``: the functions named
``mpnl_*`` take the same arguments as their C counterparts (torch tensors
stand in for device pointers, a torch stream or None for ``hipStream_t``) and
only marshal them.  Every step of detection runs in the HIP kernels of
``libmpnl.so``; there is no CPU fallback: if the library is missing or no GPU
is present the calls raise.

Convenience layer: :class:`Context`, :class:`Slot` and :func:`detect`.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpnl.so")

MPNL_OK = 0
MPNL_E_INVAL = -1
MPNL_E_UNSUPPORTED = -2
MPNL_E_NOMEM = -3
MPNL_E_HIP = -4
MPNL_MAX_USERS = 32
MPNL_MAX_ANTENNAS = 32
MPNL_MAX_PATHS = 4096
MPNL_STATIC_SCRATCH_BYTES = 128 << 20
MPNL_QPSK, MPNL_QAM16, MPNL_QAM64 = 2, 4, 6
MPNL_PREC_FP32, MPNL_PREC_FP16, MPNL_PREC_BF16 = 0, 1, 2

EXPORTED = (
    "mpnl_create", "mpnl_destroy", "mpnl_strerror", "mpnl_last_hip_error",
    "mpnl_set_precision", "mpnl_memory_usage", "mpnl_detect", "mpnl_slot_prepare",
    "mpnl_slot_detect", "mpnl_slot_detect_soft", "mpnl_slot_release", "mpnl_slot_export",
    "mpnl_slot_info", "mpnl_detect_batch", "mpnl_profile_enable", "mpnl_profile_collect",
    "mpnl_batch_create", "mpnl_batch_run", "mpnl_batch_info", "mpnl_batch_destroy",
    "mpnl_job_bytes", "mpnl_server_create", "mpnl_server_now_us", "mpnl_server_submit",
    "mpnl_server_poll", "mpnl_server_pending", "mpnl_server_run_poisson", "mpnl_server_destroy",
    "mpnl_sched_simulate", "mpnl_mmse_detect", "mpnl_detect_regularized", "mpnl_detect_static",
    "mpnl_diag_valu_rate",
)
MPNL_JOB_DONE, MPNL_JOB_REJECTED, MPNL_JOB_DROPPED, MPNL_JOB_FAILED = 0, 1, 2, 3
MPNL_CREATE_NO_PRUNE = 1
MPNL_BATCH_AUTOTUNE = 1
MPNL_BATCH_SERIAL = 2
MPNL_STAGE_SQRD, MPNL_STAGE_POSVEC, MPNL_STAGE_ROTATE, MPNL_STAGE_PATHS, MPNL_STAGE_BOUND = 0, 1, 2, 3, 4
MPNL_STAGE_PATH_WINDOW = 5
STAGE_NAMES = ("sqrd", "posvec", "rotate", "paths", "bound", "path_window")


class mpnl_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_batch_jobs", ctypes.c_int),
                ("max_inflight", ctypes.c_int), ("max_queue", ctypes.c_int),
                ("deadline_us", ctypes.c_double), ("drop_late", ctypes.c_int), ("policy", ctypes.c_int),
                ("split_vectors", ctypes.c_int64), ("est_fixed_us", ctypes.c_double),
                ("est_us_per_gflop", ctypes.c_double)]


class mpnl_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int), ("error", ctypes.c_int),
                ("arrival_us", ctypes.c_double), ("start_us", ctypes.c_double),
                ("done_us", ctypes.c_double)]


class mpnl_sim_job(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("arrival_us", ctypes.c_double), ("bytes", ctypes.c_size_t),
                ("vectors", ctypes.c_int64), ("gflop", ctypes.c_double)]


class mpnl_sim_device(ctypes.Structure):
    _fields_ = [("launch_us", ctypes.c_double), ("per_vector_us", ctypes.c_double),
                ("fail_launch", ctypes.c_int), ("slow_job", ctypes.c_int64),
                ("slow_extra_us", ctypes.c_double)]


class MpnlError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {code} ({strerror(code)})")


class mpnl_job(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_void_p), ("y", ctypes.c_void_p), ("out", ctypes.c_void_p),
        ("S", ctypes.c_int), ("T", ctypes.c_int), ("M", ctypes.c_int), ("N", ctypes.c_int),
        ("mod", ctypes.c_int), ("n_paths", ctypes.c_int),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libmpnl.so (built by ``paper_2409_14355_amd/build.py``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    vp, ip, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_size_t
    L.mpnl_create.argtypes = [ctypes.POINTER(vp), ip, sz, ctypes.c_uint]
    L.mpnl_destroy.argtypes = [vp]
    L.mpnl_strerror.argtypes = [ip]
    L.mpnl_strerror.restype = ctypes.c_char_p
    L.mpnl_last_hip_error.argtypes = [vp]
    L.mpnl_set_precision.argtypes = [vp, ip]
    L.mpnl_memory_usage.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    L.mpnl_detect.argtypes = [vp, vp, vp, ip, ip, ip, ip, ip, ip, vp, vp]
    L.mpnl_detect_static.argtypes = [vp, vp, vp, ip, ip, ip, ip, ip, ip, vp, vp]
    L.mpnl_slot_prepare.argtypes = [vp, vp, ip, ip, ip, ip, ip, vp, ctypes.POINTER(vp)]
    L.mpnl_slot_detect.argtypes = [vp, vp, vp, ip, vp, vp]
    L.mpnl_slot_detect_soft.argtypes = [vp, vp, vp, ip, ctypes.c_float, ctypes.c_float, vp, vp, vp]
    L.mpnl_slot_release.argtypes = [vp, vp]
    L.mpnl_slot_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.mpnl_slot_info.argtypes = [vp] + [ctypes.POINTER(ip)] * 5
    L.mpnl_detect_batch.argtypes = [vp, ctypes.POINTER(mpnl_job), ip, vp]
    L.mpnl_batch_create.argtypes = [vp, ctypes.POINTER(mpnl_job), ip, ctypes.c_uint, ctypes.POINTER(vp)]
    L.mpnl_batch_run.argtypes = [vp, vp, ctypes.POINTER(mpnl_job), vp]
    L.mpnl_batch_info.argtypes = [vp, ctypes.POINTER(ip), ctypes.POINTER(ip), ip]
    L.mpnl_batch_destroy.argtypes = [vp, vp]
    L.mpnl_diag_valu_rate.argtypes = [ip, ip, ip, ip, ctypes.POINTER(ctypes.c_double)]
    L.mpnl_mmse_detect.argtypes = [vp, vp, vp, ip, ip, ip, ip, ip, ctypes.c_float, vp, vp]
    L.mpnl_detect_regularized.argtypes = [vp, vp, vp, ip, ip, ip, ip, ip, ip, ctypes.c_float, vp, vp]
    cfgp = ctypes.POINTER(mpnl_server_config)
    compp = ctypes.POINTER(mpnl_completion)
    L.mpnl_job_bytes.argtypes = [ip] * 6
    L.mpnl_job_bytes.restype = sz
    L.mpnl_server_create.argtypes = [vp, cfgp, ctypes.POINTER(vp)]
    L.mpnl_server_now_us.argtypes = [vp]
    L.mpnl_server_now_us.restype = ctypes.c_double
    L.mpnl_server_submit.argtypes = [vp, ctypes.POINTER(mpnl_job), ctypes.c_int64, ctypes.c_double]
    L.mpnl_server_poll.argtypes = [vp, compp, ip, ctypes.POINTER(ip)]
    L.mpnl_server_pending.argtypes = [vp]
    L.mpnl_server_run_poisson.argtypes = [vp, ctypes.POINTER(mpnl_job), ip, ip, ctypes.c_double,
                                          ctypes.c_uint64, compp, ctypes.POINTER(ctypes.c_int32)]
    L.mpnl_server_destroy.argtypes = [vp]
    L.mpnl_sched_simulate.argtypes = [cfgp, ctypes.POINTER(mpnl_sim_device), ctypes.POINTER(mpnl_sim_job),
                                      ip, compp, ctypes.POINTER(ip)]
    L.mpnl_profile_enable.argtypes = [vp, ip]
    L.mpnl_profile_collect.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ip)]
    _lib = L
    return L


def strerror(code: int) -> str:
    try:
        return lib().mpnl_strerror(code).decode()
    except RuntimeError:
        return "library not loaded"


def _check(rc: int, what: str) -> None:
    if rc != MPNL_OK:
        raise MpnlError(rc, what)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("device buffers are passed as torch tensors")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> Optional[int]:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- same-named wrappers of the C ABI -------------------------------------------

def mpnl_create(device: int = 0, hbm_budget_bytes: int = 0, flags: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().mpnl_create(ctypes.byref(h), device, hbm_budget_bytes, flags), "mpnl_create")
    return h.value


def mpnl_destroy(ctx: int) -> None:
    _check(lib().mpnl_destroy(ctx), "mpnl_destroy")


def mpnl_strerror(code: int) -> str:
    return strerror(code)


def mpnl_last_hip_error(ctx: int) -> int:
    return lib().mpnl_last_hip_error(ctx)


def mpnl_set_precision(ctx: int, precision: int) -> None:
    _check(lib().mpnl_set_precision(ctx, precision), "mpnl_set_precision")


def mpnl_memory_usage(ctx: int) -> tuple[int, int]:
    held, used = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().mpnl_memory_usage(ctx, ctypes.byref(held), ctypes.byref(used)), "mpnl_memory_usage")
    return held.value, used.value


def mpnl_detect(ctx: int, H, y, S: int, T: int, M: int, N: int, mod: int, n_paths: int, out,
                stream=None) -> None:
    _check(lib().mpnl_detect(ctx, _ptr(H), _ptr(y), S, T, M, N, mod, n_paths, _ptr(out),
                             _stream(stream)), "mpnl_detect")


def mpnl_detect_static(ctx: int, H, y, S: int, T: int, M: int, N: int, mod: int, n_paths: int, out,
                       stream=None) -> None:
    _check(lib().mpnl_detect_static(ctx, _ptr(H), _ptr(y), S, T, M, N, mod, n_paths, _ptr(out),
                                    _stream(stream)), "mpnl_detect_static")


def mpnl_slot_prepare(ctx: int, H, S: int, M: int, N: int, mod: int, n_paths: int,
                      stream=None) -> int:
    h = ctypes.c_void_p()
    _check(lib().mpnl_slot_prepare(ctx, _ptr(H), S, M, N, mod, n_paths, _stream(stream),
                                   ctypes.byref(h)), "mpnl_slot_prepare")
    return h.value


def mpnl_slot_detect(ctx: int, slot: int, y, T: int, out, stream=None) -> None:
    _check(lib().mpnl_slot_detect(ctx, slot, _ptr(y), T, _ptr(out), _stream(stream)),
           "mpnl_slot_detect")


def mpnl_slot_detect_soft(ctx: int, slot: int, y, T: int, sigma2: float, clip: float, llr,
                          out=None, stream=None) -> None:
    _check(lib().mpnl_slot_detect_soft(ctx, slot, _ptr(y), T, sigma2, clip, _ptr(llr), _ptr(out),
                                       _stream(stream)), "mpnl_slot_detect_soft")


def mpnl_slot_release(ctx: int, slot: int) -> None:
    _check(lib().mpnl_slot_release(ctx, slot), "mpnl_slot_release")


def mpnl_slot_export(ctx: int, slot: int, perm=None, w=None, roff=None, P=None,
                     stream=None) -> None:
    _check(lib().mpnl_slot_export(ctx, slot, _ptr(perm), _ptr(w), _ptr(roff), _ptr(P),
                                  _stream(stream)), "mpnl_slot_export")


def mpnl_slot_info(slot: int) -> dict:
    v = [ctypes.c_int() for _ in range(5)]
    _check(lib().mpnl_slot_info(slot, *[ctypes.byref(x) for x in v]), "mpnl_slot_info")
    return dict(zip(("S", "M", "N", "mod", "K"), (x.value for x in v)))


def _job_array(jobs: Sequence[dict]):
    """Jobs as dicts {H, y, out, mod, n_paths}; a dict without tensors may give
    the sizes S, T, M, N directly (shapes of a batch plan)."""
    arr = (mpnl_job * len(jobs))()
    for i, j in enumerate(jobs):
        if "H" in j:
            S, M, N = j["H"].shape
            T = j["y"].shape[0]
        else:
            S, T, M, N = j["S"], j["T"], j["M"], j["N"]
        arr[i] = mpnl_job(_ptr(j.get("H")), _ptr(j.get("y")), _ptr(j.get("out")), S, T, M, N,
                          j["mod"], j["n_paths"])
    return arr


def mpnl_detect_batch(ctx: int, jobs: Sequence[dict], stream=None) -> None:
    arr = _job_array(jobs)
    _check(lib().mpnl_detect_batch(ctx, arr, len(jobs), _stream(stream)), "mpnl_detect_batch")


def mpnl_batch_create(ctx: int, shapes: Sequence[dict], flags: int = 0) -> int:
    arr = _job_array(shapes)
    h = ctypes.c_void_p()
    _check(lib().mpnl_batch_create(ctx, arr, len(shapes), flags, ctypes.byref(h)), "mpnl_batch_create")
    return h.value


def mpnl_batch_run(ctx: int, batch: int, jobs: Sequence[dict], stream=None) -> None:
    arr = _job_array(jobs)
    _check(lib().mpnl_batch_run(ctx, batch, arr, _stream(stream)), "mpnl_batch_run")


def mpnl_batch_info(batch: int, max_launches: int = 128) -> list[dict]:
    """-> launch shape of every path-search launch of the plan."""
    n = ctypes.c_int()
    v = (ctypes.c_int * (7 * max_launches))()
    _check(lib().mpnl_batch_info(batch, ctypes.byref(n), v, max_launches), "mpnl_batch_info")
    keys = ("N", "mod", "lanes", "group_lanes", "items_per_workgroup", "group_major", "workgroups")
    return [dict(zip(keys, v[7 * i:7 * i + 7])) for i in range(min(n.value, max_launches))]


def mpnl_diag_valu_rate(device: int, kind: int, waves: int, iters: int) -> float:
    """-> milliseconds of the VALU issue probe launch (see mpnl.h)."""
    ms = ctypes.c_double()
    _check(lib().mpnl_diag_valu_rate(device, kind, waves, iters, ctypes.byref(ms)), "mpnl_diag_valu_rate")
    return ms.value


def mpnl_batch_destroy(ctx: int, batch: int) -> None:
    _check(lib().mpnl_batch_destroy(ctx, batch), "mpnl_batch_destroy")


def mpnl_mmse_detect(ctx: int, H, y, S: int, T: int, M: int, N: int, mod: int, sigma2: float, out,
                     stream=None) -> None:
    _check(lib().mpnl_mmse_detect(ctx, _ptr(H), _ptr(y), S, T, M, N, mod, float(sigma2), _ptr(out),
                                  _stream(stream)), "mpnl_mmse_detect")


def mpnl_detect_regularized(ctx: int, H, y, S: int, T: int, M: int, N: int, mod: int, n_paths: int,
                            sigma2: float, out, stream=None) -> None:
    _check(lib().mpnl_detect_regularized(ctx, _ptr(H), _ptr(y), S, T, M, N, mod, n_paths, float(sigma2),
                                         _ptr(out), _stream(stream)), "mpnl_detect_regularized")


def mpnl_profile_enable(ctx: int, enable: bool) -> None:
    _check(lib().mpnl_profile_enable(ctx, 1 if enable else 0), "mpnl_profile_enable")


def mpnl_profile_collect(ctx: int) -> dict:
    """-> {stage name: (total milliseconds, launches)} since the last collect."""
    ns = len(STAGE_NAMES)
    ms = (ctypes.c_double * ns)()
    n = (ctypes.c_int * ns)()
    _check(lib().mpnl_profile_collect(ctx, ms, n), "mpnl_profile_collect")
    return {STAGE_NAMES[i]: (ms[i], n[i]) for i in range(ns)}


# ---- convenience layer ------------------------------------------------------------

def _shapes(H, y):
    if H.dim() != 3 or y.dim() != 3:
        raise ValueError("H must be (S, M, N) and y (T, S, M)")
    S, M, N = H.shape
    T = y.shape[0]
    if y.shape[1] != S or y.shape[2] != M:
        raise ValueError(f"y shape {tuple(y.shape)} does not match H {tuple(H.shape)}")
    return S, T, M, N


class Slot:
    """Channel state of one slot kept on the device (a1 + a2 done)."""

    def __init__(self, ctx: "Context", handle: int, S: int, M: int, N: int, mod: int):
        self.ctx, self.handle, self.S, self.M, self.N, self.mod = ctx, handle, S, M, N, mod

    def detect(self, y, out=None, stream=None):
        import torch
        T = y.shape[0]
        if out is None:
            out = torch.empty((T, self.S, self.N), dtype=torch.int32, device=y.device)
        mpnl_slot_detect(self.ctx.handle, self.handle, y, T, out, stream)
        return out

    def detect_soft(self, y, sigma2: float, clip: float = 1e4, out=None, stream=None):
        import torch
        T = y.shape[0]
        llr = torch.empty((T, self.S, self.N, self.mod), dtype=torch.float32, device=y.device)
        mpnl_slot_detect_soft(self.ctx.handle, self.handle, y, T, sigma2, clip, llr, out, stream)
        return llr

    def export(self, stream=None) -> dict:
        import torch
        info = mpnl_slot_info(self.handle)
        S, N, K = info["S"], info["N"], info["K"]
        dev = f"cuda:{self.ctx.device}"
        perm = torch.empty((S, N), dtype=torch.int32, device=dev)
        w = torch.empty((S, N), dtype=torch.float64, device=dev)
        roff = torch.empty((S, N, N), dtype=torch.complex64, device=dev)
        P = torch.empty((S, K, N), dtype=torch.uint8, device=dev)
        mpnl_slot_export(self.ctx.handle, self.handle, perm, w, roff, P, stream)
        return dict(perm=perm, w=w, roff=roff, P=P, K=K)

    def release(self):
        if self.handle:
            mpnl_slot_release(self.ctx.handle, self.handle)
            self.handle = 0


class Context:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, prune: bool = True):
        self.device = device
        self.handle = mpnl_create(device, hbm_budget_bytes, 0 if prune else MPNL_CREATE_NO_PRUNE)

    def close(self):
        if self.handle:
            mpnl_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, precision: int):
        mpnl_set_precision(self.handle, precision)

    def memory_usage(self):
        return mpnl_memory_usage(self.handle)

    def profile(self, enable: bool = True):
        mpnl_profile_enable(self.handle, enable)

    def profile_collect(self) -> dict:
        return mpnl_profile_collect(self.handle)

    def detect(self, H, y, mod: int, n_paths: int, out=None, stream=None):
        import torch
        S, T, M, N = _shapes(H, y)
        if out is None:
            out = torch.empty((T, S, N), dtype=torch.int32, device=H.device)
        mpnl_detect(self.handle, H, y, S, T, M, N, mod, n_paths, out, stream)
        return out

    def detect_static(self, H, y, mod: int, n_paths: int, out=None, stream=None):
        """As detect(), with no device allocation (the library's static scratch area)."""
        import torch
        S, T, M, N = _shapes(H, y)
        if out is None:
            out = torch.empty((T, S, N), dtype=torch.int32, device=H.device)
        mpnl_detect_static(self.handle, H, y, S, T, M, N, mod, n_paths, out, stream)
        return out

    def detect_regularized(self, H, y, mod: int, n_paths: int, sigma2: float, out=None, stream=None):
        """MPNL on [H; sqrt(sigma2) I] (overloaded N > M allowed) -> (T, S, N) int32."""
        import torch
        S, T, M, N = _shapes(H, y)
        if out is None:
            out = torch.empty((T, S, N), dtype=torch.int32, device=H.device)
        mpnl_detect_regularized(self.handle, H, y, S, T, M, N, mod, n_paths, sigma2, out, stream)
        return out

    def mmse(self, H, y, mod: int, sigma2: float, out=None, stream=None):
        """Linear MMSE detection -> (T, S, N) int32 indices."""
        import torch
        S, T, M, N = _shapes(H, y)
        if out is None:
            out = torch.empty((T, S, N), dtype=torch.int32, device=H.device)
        mpnl_mmse_detect(self.handle, H, y, S, T, M, N, mod, sigma2, out, stream)
        return out

    def slot_prepare(self, H, mod: int, n_paths: int, stream=None) -> Slot:
        S, M, N = H.shape
        h = mpnl_slot_prepare(self.handle, H, S, M, N, mod, n_paths, stream)
        return Slot(self, h, S, M, N, mod)

    def detect_batch(self, jobs: Sequence[dict], stream=None):
        import torch
        for j in jobs:
            if j.get("out") is None:
                S, T, M, N = _shapes(j["H"], j["y"])
                j["out"] = torch.empty((T, S, N), dtype=torch.int32, device=j["H"].device)
        mpnl_detect_batch(self.handle, jobs, stream)
        return [j["out"] for j in jobs]

    def batch_plan(self, shapes: Sequence[dict], autotune: bool = False, serial: bool = False) -> "BatchPlan":
        return BatchPlan(self, shapes, autotune, serial)


class BatchPlan:
    """A fixed set of job shapes whose whole pipeline (every stage of every
    job) replays as one captured graph; each run takes new tensors of the
    same shapes."""

    def __init__(self, ctx: Context, shapes: Sequence[dict], autotune: bool = False, serial: bool = False):
        self.ctx = ctx
        self.shapes = [dict(s) for s in shapes]
        flags = (MPNL_BATCH_AUTOTUNE if autotune else 0) | (MPNL_BATCH_SERIAL if serial else 0)
        self.handle = mpnl_batch_create(ctx.handle, self.shapes, flags)

    def run(self, jobs: Sequence[dict], stream=None):
        mpnl_batch_run(self.ctx.handle, self.handle, jobs, stream)
        return [j["out"] for j in jobs]

    def launch_shapes(self) -> list[dict]:
        return mpnl_batch_info(self.handle)

    def close(self):
        if self.handle and self.ctx.handle:
            mpnl_batch_destroy(self.ctx.handle, self.handle)
        self.handle = 0


MPNL_SCHED_FIFO, MPNL_SCHED_SLACK = 0, 1


def server_config(hbm_budget: int = 0, max_batch_jobs: int = 8, max_inflight: int = 2,
                  max_queue: int = 0, deadline_us: float = 500.0, drop_late: bool = False,
                  policy: int = MPNL_SCHED_FIFO, split_vectors: int = 0, est_fixed_us: float = 40.0,
                  est_us_per_gflop: float = 20.0):
    return mpnl_server_config(hbm_budget, max_batch_jobs, max_inflight, max_queue, deadline_us,
                              1 if drop_late else 0, policy, split_vectors, est_fixed_us, est_us_per_gflop)


def _completions(arr) -> list[dict]:
    return [dict(id=c.id, status=c.status, error=c.error, arrival_us=c.arrival_us, start_us=c.start_us,
                 done_us=c.done_us) for c in arr]


def mpnl_job_bytes(S: int, T: int, M: int, N: int, mod: int, n_paths: int) -> int:
    return int(lib().mpnl_job_bytes(S, T, M, N, mod, n_paths))


def mpnl_sched_simulate(cfg: mpnl_server_config, jobs: Sequence[dict], launch_us: float = 5.0,
                        per_vector_us: float = 0.0, fail_launch: int = -1, slow_job: int = -1,
                        slow_extra_us: float = 0.0):
    """Scheduler on a virtual clock with a modelled device.  jobs: dicts
    {arrival_us, bytes, vectors, gflop} in arrival order (ids are their
    positions).  -> (completions by id, number of launches)."""
    arr = (mpnl_sim_job * len(jobs))()
    for i, j in enumerate(jobs):
        arr[i] = mpnl_sim_job(i, j["arrival_us"], j.get("bytes", 0), j.get("vectors", 0), j.get("gflop", 0.0))
    dev = mpnl_sim_device(launch_us, per_vector_us, fail_launch, slow_job, slow_extra_us)
    out = (mpnl_completion * max(len(jobs), 1))()
    n = ctypes.c_int()
    _check(lib().mpnl_sched_simulate(ctypes.byref(cfg), ctypes.byref(dev), arr, len(jobs), out,
                                     ctypes.byref(n)), "mpnl_sched_simulate")
    return _completions(out[:len(jobs)]), n.value


class Server:
    """Continuous-batching detection service on one context."""

    def __init__(self, ctx: "Context", cfg: mpnl_server_config):
        self.ctx = ctx
        self.cfg = cfg
        h = ctypes.c_void_p()
        _check(lib().mpnl_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)), "mpnl_server_create")
        self.handle = h.value

    def now_us(self) -> float:
        return lib().mpnl_server_now_us(self.handle)

    def submit(self, job: dict, id: int, arrival_us: Optional[float] = None):
        arr = _job_array([job])
        t = self.now_us() if arrival_us is None else arrival_us
        _check(lib().mpnl_server_submit(self.handle, arr, id, t), "mpnl_server_submit")

    def poll(self, max_n: int = 256) -> list[dict]:
        out = (mpnl_completion * max_n)()
        n = ctypes.c_int()
        _check(lib().mpnl_server_poll(self.handle, out, max_n, ctypes.byref(n)), "mpnl_server_poll")
        return _completions(out[:n.value])

    def pending(self) -> int:
        return lib().mpnl_server_pending(self.handle)

    def drain(self) -> list[dict]:
        got = []
        while self.pending() > 0:
            got += self.poll()
        return got

    def run_poisson(self, pool: Sequence[dict], n_jobs: int, rate_hz: float, seed: int) -> list[dict]:
        """-> completions by job id, each with the pool index of the job ("entry")."""
        arr = _job_array(pool)
        out = (mpnl_completion * max(n_jobs, 1))()
        ent = (ctypes.c_int32 * max(n_jobs, 1))()
        _check(lib().mpnl_server_run_poisson(self.handle, arr, len(pool), n_jobs, rate_hz, seed, out, ent),
               "mpnl_server_run_poisson")
        comp = _completions(out[:n_jobs])
        for c, e in zip(comp, ent[:n_jobs]):
            c["entry"] = e
        return comp

    def close(self):
        if self.handle:
            lib().mpnl_server_destroy(self.handle)
        self.handle = 0


_default_ctx: Optional[Context] = None


def detect(H, y, mod: int, n_paths: int, out=None, stream=None):
    """detect(H (S,M,N) c64, y (T,S,M) c64, mod, n_paths) -> (T,S,N) int32 indices."""
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context(H.device.index or 0)
    return _default_ctx.detect(H, y, mod, n_paths, out, stream)
