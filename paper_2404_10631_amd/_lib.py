"""ctypes binding of ``libknnf.so`` (the C-ABI declared in include/knnf.h).

Argument marshalling only: every step of the filter runs in the HIP kernels.
The functions keep the C names (``knnf_create``, ``knnf_filter``, ...).  Device
buffers are passed as integer addresses (``tensor.data_ptr()``) and streams as
integer handles (``torch.cuda.current_stream().cuda_stream``).

The library is loaded after torch so that both use the one HIP runtime
(torch's ``libamdhip64.so`` carries the same SONAME the library links against).
If ``libknnf.so`` is missing the import fails loudly: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libknnf.so")

KNNF_OK = 0
KNNF_EINVAL = -1
KNNF_ENOMEM = -2
KNNF_EDEVICE = -3
KNNF_EAGAIN = -4
KNNF_ESTATE = -5

KNNF_SEARCH_EXHAUSTIVE = 0
KNNF_SEARCH_PRUNED = 1

KNNF_MAX_K = 64
KNNF_MAX_C = 16

_STATUS_NAMES = {0: "KNNF_OK", -1: "KNNF_EINVAL", -2: "KNNF_ENOMEM", -3: "KNNF_EDEVICE",
                 -4: "KNNF_EAGAIN", -5: "KNNF_ESTATE"}


class knnf_frame(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
        ("K", ctypes.c_int32), ("R", ctypes.c_int32), ("lam", ctypes.c_float),
        ("pc1", ctypes.c_void_p), ("prob", ctypes.c_void_p),
        ("out_prob", ctypes.c_void_p), ("out_class", ctypes.c_void_p),
        ("out_nbr", ctypes.c_void_p), ("out_dist", ctypes.c_void_p),
    ]


KNNF_LAUNCH_DEFAULT = 0
KNNF_LAUNCH_PERSISTENT = 1
KNNF_LAUNCH_GRID = 2


KNNF_PLAN_NO_INPUT_CHECK = 1


class knnf_plan(ctypes.Structure):
    _fields_ = [("search", ctypes.c_int32), ("tile_rows", ctypes.c_int32),
                ("tile_cols", ctypes.c_int32), ("waves", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("chunk_rows", ctypes.c_int32),
                ("flags", ctypes.c_int32)]

    def as_dict(self):
        return {"search": self.search, "tile_rows": self.tile_rows,
                "tile_cols": self.tile_cols, "waves": self.waves, "launch": self.launch,
                "chunk_rows": self.chunk_rows, "flags": self.flags}


def make_plan(plan) -> "knnf_plan":
    if isinstance(plan, knnf_plan):
        return plan
    return knnf_plan(int(plan.get("search", 0)), int(plan.get("tile_rows", 0)),
                     int(plan.get("tile_cols", 0)), int(plan.get("waves", 0)),
                     int(plan.get("launch", 0)), int(plan.get("chunk_rows", 0)),
                     int(plan.get("flags", 0)))


KNNF_SERVE_BATCHED = 0
KNNF_SERVE_PLAIN = 1


class knnf_server_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("max_queue", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("step_tiles", ctypes.c_int32),
                ("plan", knnf_plan)]


class knnf_host_frame(ctypes.Structure):
    _fields_ = [
        ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
        ("K", ctypes.c_int32), ("R", ctypes.c_int32), ("lam", ctypes.c_float),
        ("pc1", ctypes.c_void_p), ("prob", ctypes.c_void_p),
        ("with_nbr", ctypes.c_int32), ("t_arrival", ctypes.c_double),
    ]


class knnf_ticket_info(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("released", ctypes.c_int32),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class KnnfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# Every symbol include/knnf.h declares, with its ctypes signature.
_P = ctypes.c_void_p
_I = ctypes.c_int
_SIGS = {
    "knnf_create": (_I, [ctypes.POINTER(_P), _I]),
    "knnf_destroy": (_I, [_P]),
    "knnf_ctx_status": (_I, [_P]),
    "knnf_inject_fault": (_I, [_P]),
    "knnf_tune_lookup": (_I, [_P, ctypes.POINTER(knnf_frame), _I, ctypes.POINTER(knnf_plan)]),
    "knnf_set_default_plan": (_I, [_P, ctypes.POINTER(knnf_plan)]),
    "knnf_get_default_plan": (_I, [_P, ctypes.POINTER(knnf_plan)]),
    "knnf_validate": (_I, [ctypes.POINTER(knnf_frame)]),
    "knnf_filter": (_I, [_P, ctypes.POINTER(knnf_frame), ctypes.POINTER(knnf_plan), _P]),
    "knnf_filter_batch": (_I, [_P, ctypes.POINTER(knnf_frame), _I, ctypes.POINTER(knnf_plan), _P]),
    "knnf_tune": (_I, [_P, ctypes.POINTER(knnf_frame), _I, _I, _P, ctypes.POINTER(knnf_plan)]),
    "knnf_frame_bytes": (ctypes.c_size_t, [_I, _I, _I, _I, _I]),
    "knnf_stats_enable": (_I, [_P, _I]),
    "knnf_stats_read": (_I, [_P, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64), _I]),
    "knnf_last_error": (ctypes.c_char_p, []),
    "knnf_server_clock": (ctypes.c_double, []),
    "knnf_server_create": (_I, [ctypes.POINTER(_P), _P, _P, ctypes.c_size_t,
                                ctypes.POINTER(knnf_server_opts)]),
    "knnf_server_submit": (_I, [_P, ctypes.POINTER(knnf_host_frame), ctypes.POINTER(ctypes.c_uint64)]),
    "knnf_server_poll": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(knnf_ticket_info)]),
    "knnf_server_result": (_I, [_P, ctypes.c_uint64, ctypes.POINTER(knnf_frame)]),
    "knnf_server_release": (_I, [_P, ctypes.c_uint64]),
    "knnf_server_drain": (_I, [_P, ctypes.c_double]),
    "knnf_server_destroy": (_I, [_P]),
    "knnf_version": (ctypes.c_char_p, []),
    "knnf_pc1": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P]),
    "knnf_pc1_noalloc": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P, _P, ctypes.c_int32,
                              _P]),
    "knnf_svm": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P,
                      _P]),
    "knnf_svm_pc1": (_I, [_P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P,
                          _P, _P, _P, _P, ctypes.c_int32, _P]),
}

_lib = None


def load():
    """Load libknnf.so (after torch) and set the signatures.  Raises if unbuilt."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  -- the HIP runtime torch uses must be loaded first

    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python -m paper_2404_10631_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


def last_error() -> str:
    return load().knnf_last_error().decode()


def check(status: int) -> None:
    if status != KNNF_OK:
        raise KnnfError(status, last_error())


def _plan_ptr(plan):
    if plan is None:
        return None
    return ctypes.byref(make_plan(plan))


def knnf_version() -> str:
    return load().knnf_version().decode()


def knnf_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    check(load().knnf_create(ctypes.byref(h), int(device)))
    return h.value


def knnf_destroy(ctx: int) -> None:
    check(load().knnf_destroy(ctx))


def knnf_ctx_status(ctx: int) -> int:
    """KNNF_OK, or KNNF_EDEVICE once the context has failed (returned, not raised)."""
    return int(load().knnf_ctx_status(ctx))


def knnf_inject_fault(ctx: int) -> None:
    check(load().knnf_inject_fault(ctx))


def knnf_tune_lookup(ctx: int, frames) -> tuple[int, knnf_plan]:
    """(status, plan): KNNF_OK and the cached plan, or KNNF_ESTATE and the
    context's default plan."""
    arr, n = _frames_arg(frames)
    p = knnf_plan()
    st = load().knnf_tune_lookup(ctx, arr, n, ctypes.byref(p))
    if st not in (KNNF_OK, KNNF_ESTATE):
        check(st)
    return int(st), p


def knnf_set_default_plan(ctx: int, plan) -> None:
    check(load().knnf_set_default_plan(ctx, _plan_ptr(plan)))


def knnf_get_default_plan(ctx: int) -> knnf_plan:
    p = knnf_plan()
    check(load().knnf_get_default_plan(ctx, ctypes.byref(p)))
    return p


def knnf_validate(frame: knnf_frame) -> int:
    return int(load().knnf_validate(ctypes.byref(frame)))


def knnf_filter(ctx: int, frame: knnf_frame, plan=None, stream: int = 0) -> None:
    check(load().knnf_filter(ctx, ctypes.byref(frame), _plan_ptr(plan), stream))


def frame_array(frames):
    """A C array of knnf_frame, built once for repeated batched calls over
    the same frames (building it costs ~0.1-0.2 us per frame in Python)."""
    return (knnf_frame * len(frames))(*frames)


def _frames_arg(frames):
    arr = frames if isinstance(frames, ctypes.Array) else frame_array(frames)
    return arr, len(arr)


def knnf_filter_batch(ctx: int, frames, plan=None, stream: int = 0) -> None:
    """frames: a list of knnf_frame or an array from frame_array()."""
    arr, n = _frames_arg(frames)
    check(load().knnf_filter_batch(ctx, arr, n, _plan_ptr(plan), stream))


def knnf_tune(ctx: int, frames, reps: int = 3, stream: int = 0) -> knnf_plan:
    arr, n = _frames_arg(frames)
    best = knnf_plan()
    check(load().knnf_tune(ctx, arr, n, int(reps), stream, ctypes.byref(best)))
    return best


def knnf_stats_enable(ctx: int, on: bool) -> None:
    check(load().knnf_stats_enable(ctx, 1 if on else 0))


def knnf_stats_read(ctx: int, reset: bool = True) -> tuple[int, int]:
    p, t = ctypes.c_uint64(), ctypes.c_uint64()
    check(load().knnf_stats_read(ctx, ctypes.byref(p), ctypes.byref(t), 1 if reset else 0))
    return p.value, t.value


def knnf_frame_bytes(H: int, W: int, C: int, K: int, with_nbr: bool) -> int:
    return int(load().knnf_frame_bytes(H, W, C, K, 1 if with_nbr else 0))


def knnf_server_clock() -> float:
    return float(load().knnf_server_clock())


def knnf_server_create(ctx: int, pool_ptr: int, pool_bytes: int, opts: knnf_server_opts | None = None) -> int:
    h = ctypes.c_void_p()
    check(load().knnf_server_create(ctypes.byref(h), ctx, pool_ptr, pool_bytes,
                                    ctypes.byref(opts) if opts is not None else None))
    return h.value


def knnf_server_submit(srv: int, frame: knnf_host_frame) -> tuple[int, int]:
    """Returns (status, ticket); KNNF_EAGAIN is returned, not raised."""
    t = ctypes.c_uint64()
    st = load().knnf_server_submit(srv, ctypes.byref(frame), ctypes.byref(t))
    if st not in (KNNF_OK, KNNF_EAGAIN):
        check(st)
    return st, t.value


def knnf_server_poll(srv: int, ticket: int) -> knnf_ticket_info:
    info = knnf_ticket_info()
    check(load().knnf_server_poll(srv, ticket, ctypes.byref(info)))
    return info


def knnf_server_result(srv: int, ticket: int) -> knnf_frame:
    v = knnf_frame()
    check(load().knnf_server_result(srv, ticket, ctypes.byref(v)))
    return v


def knnf_server_release(srv: int, ticket: int) -> None:
    check(load().knnf_server_release(srv, ticket))


def knnf_server_drain(srv: int, timeout_s: float = 0.0) -> None:
    check(load().knnf_server_drain(srv, float(timeout_s)))


def knnf_server_destroy(srv: int) -> None:
    check(load().knnf_server_destroy(srv))


def knnf_pc1(ctx: int, cube_ptr: int, npix: int, bands: int, mean_ptr: int, vec_ptr: int,
             out_ptr: int, normalize: bool = True, stream: int = 0) -> None:
    """PC1 projection of a device cube (see include/knnf.h); device pointers."""
    check(load().knnf_pc1(ctx, cube_ptr, int(npix), int(bands), mean_ptr, vec_ptr, out_ptr,
                          1 if normalize else 0, stream))


KNNF_PC1_NOALLOC_MAX_PIXELS = 1 << 20


def knnf_pc1_noalloc(ctx: int, cube_ptr: int, npix: int, bands: int, mean_ptr: int, vec_ptr: int,
                     out_ptr: int, normalize: bool = True, stream: int = 0) -> None:
    """knnf_pc1 on the library's static scratch: allocates nothing (see include/knnf.h)."""
    check(load().knnf_pc1_noalloc(ctx, cube_ptr, int(npix), int(bands), mean_ptr, vec_ptr,
                                  out_ptr, 1 if normalize else 0, stream))


def knnf_svm(ctx: int, cube_ptr: int, npix: int, bands: int, classes: int, w_ptr: int,
             bias_ptr: int, a_ptr: int, b_ptr: int, out_ptr: int, stream: int = 0) -> None:
    """SVM probability maps of a device cube (see include/knnf.h); device pointers."""
    check(load().knnf_svm(ctx, cube_ptr, int(npix), int(bands), int(classes), w_ptr, bias_ptr,
                          a_ptr, b_ptr, out_ptr, stream))


def knnf_svm_pc1(ctx: int, cube_ptr: int, npix: int, bands: int, classes: int, w_ptr: int,
                 bias_ptr: int, a_ptr: int, b_ptr: int, mean_ptr: int, vec_ptr: int,
                 prob_ptr: int, band_ptr: int, normalize: bool = True, stream: int = 0) -> None:
    """SVM maps and the PC1 band from one read of a device cube (see include/knnf.h)."""
    check(load().knnf_svm_pc1(ctx, cube_ptr, int(npix), int(bands), int(classes), w_ptr, bias_ptr,
                              a_ptr, b_ptr, mean_ptr, vec_ptr, prob_ptr, band_ptr,
                              1 if normalize else 0, stream))
