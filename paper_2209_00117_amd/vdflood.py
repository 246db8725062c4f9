"""Python binding of libvdflood.so (C ABI in include/vdflood.h).

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides the device workspace (a uint8 CUDA tensor) and
the stream (torch's current stream).  If the library is missing this module
raises; there is no fallback.

The functions carry the C names without the ``vd_`` prefix; :class:`Sim`
bundles a handle with the workspace tensor that must outlive it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LABEL_ID32, LABEL_XY16 = 0, 1
EUCLID, MANHATTAN = 0, 1
EMPTY = -1
MAX_SIDE = 16368

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvdflood.so")


class VdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"vdflood status {status}: {message}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("num_seeds", ctypes.c_int32),
        ("disp_lo", ctypes.c_int32), ("disp_hi", ctypes.c_int32), ("label", ctypes.c_int32),
        ("metric", ctypes.c_int32), ("vn_passes", ctypes.c_int32),
        ("extra_passes", ctypes.c_int32), ("dmax_override", ctypes.c_int32),
        ("sim_seed", ctypes.c_uint64),
    ]


class SimInfo(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("num_seeds", ctypes.c_int32),
        ("label", ctypes.c_int32), ("metric", ctypes.c_int32), ("k1", ctypes.c_int32),
        ("delta1", ctypes.c_int32), ("passes_jfa", ctypes.c_int32),
        ("passes_djfa", ctypes.c_int32), ("t", ctypes.c_int64),
    ]


class Timing(ctypes.Structure):
    _fields_ = [
        ("flood_launches", ctypes.c_int64), ("flood_ms", ctypes.c_double),
        ("flood_pixels", ctypes.c_int64), ("step_count", ctypes.c_int64),
        ("step_ms", ctypes.c_double),
    ]


# name -> (restype, argtypes); the exported symbols of include/vdflood.h
_P = ctypes.c_void_p
SIGNATURES = {
    "vd_config_default": (None, [ctypes.POINTER(Config)]),
    "vd_footprint_bytes": (ctypes.c_size_t, [ctypes.POINTER(Config)]),
    "vd_init_sim": (ctypes.c_int, [ctypes.POINTER(Config), _P, _P, ctypes.c_size_t, _P,
                                   ctypes.POINTER(_P)]),
    "vd_move_seeds": (ctypes.c_int, [_P]),
    "vd_jfa_step": (ctypes.c_int, [_P]),
    "vd_djfa_step": (ctypes.c_int, [_P]),
    "vd_read_map": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_read_seeds": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_map_device": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "vd_get_info": (ctypes.c_int, [_P, ctypes.POINTER(SimInfo)]),
    "vd_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(Timing)]),
    "vd_set_flood_variant": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_destroy": (None, [_P]),
    "vd_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """Loads libvdflood.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2209_00117_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != 0:
        raise VdError(status, lib().vd_last_error().decode())


def config(width, height, num_seeds, disp_lo=-1, disp_hi=1, label=LABEL_ID32, metric=EUCLID,
           vn_passes=2, extra_passes=0, dmax_override=0, sim_seed=1) -> Config:
    c = Config()
    lib().vd_config_default(ctypes.byref(c))
    c.width, c.height, c.num_seeds = width, height, num_seeds
    c.disp_lo, c.disp_hi, c.label, c.metric = disp_lo, disp_hi, label, metric
    c.vn_passes, c.extra_passes, c.dmax_override, c.sim_seed = (vn_passes, extra_passes,
                                                                dmax_override, sim_seed)
    return c


def footprint_bytes(cfg: Config) -> int:
    return int(lib().vd_footprint_bytes(ctypes.byref(cfg)))


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def init_sim(cfg: Config, xy: np.ndarray, workspace, stream=None) -> ctypes.c_void_p:
    """Raw vd_init_sim; `workspace` is a uint8 CUDA tensor the caller keeps."""
    xy = np.ascontiguousarray(xy, dtype=np.int32)
    if xy.shape != (cfg.num_seeds, 2):
        raise ValueError(f"positions must be ({cfg.num_seeds}, 2) int32, got {xy.shape}")
    h = ctypes.c_void_p()
    _check(lib().vd_init_sim(ctypes.byref(cfg), xy.ctypes.data_as(_P),
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                             _stream_ptr(stream), ctypes.byref(h)))
    return h


def move_seeds(h):
    _check(lib().vd_move_seeds(h))


def jfa_step(h):
    _check(lib().vd_jfa_step(h))


def djfa_step(h):
    _check(lib().vd_djfa_step(h))


def get_info(h) -> SimInfo:
    info = SimInfo()
    _check(lib().vd_get_info(h, ctypes.byref(info)))
    return info


def read_map(h) -> np.ndarray:
    info = get_info(h)
    out = np.empty((info.height, info.width), np.int32)
    _check(lib().vd_read_map(h, out.ctypes.data_as(_P), out.size))
    return out


def read_seeds(h) -> np.ndarray:
    info = get_info(h)
    out = np.empty((info.num_seeds, 2), np.int32)
    _check(lib().vd_read_seeds(h, out.ctypes.data_as(_P), out.size))
    return out


def map_device(h) -> int:
    p = ctypes.c_void_p()
    _check(lib().vd_map_device(h, ctypes.byref(p)))
    return int(p.value or 0)


def set_timing(h, enable: bool):
    _check(lib().vd_set_timing(h, int(bool(enable))))


def get_timing(h) -> Timing:
    t = Timing()
    _check(lib().vd_get_timing(h, ctypes.byref(t)))
    return t


def set_flood_variant(h, variant: int):
    _check(lib().vd_set_flood_variant(h, variant))


def destroy(h):
    if h:
        lib().vd_destroy(h)


def last_error() -> str:
    return lib().vd_last_error().decode()


class Sim:
    """A simulation and the workspace tensor it lives in."""

    def __init__(self, width, height, xy, device="cuda", stream=None, **kw):
        import torch
        self.cfg = config(width, height, int(np.asarray(xy).shape[0]), **kw)
        nbytes = footprint_bytes(self.cfg)
        if nbytes == 0:
            raise VdError(-1, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.handle = init_sim(self.cfg, xy, self.workspace, stream)

    def move_seeds(self):
        move_seeds(self.handle)

    def jfa_step(self):
        jfa_step(self.handle)

    def djfa_step(self):
        djfa_step(self.handle)

    def read_map(self) -> np.ndarray:
        return read_map(self.handle)

    def read_seeds(self) -> np.ndarray:
        return read_seeds(self.handle)

    def info(self) -> SimInfo:
        return get_info(self.handle)

    def close(self):
        if self.handle:
            destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
