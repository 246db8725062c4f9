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
DMAX_MEASURED = -1     # dmax_override: d_max measured per dJFA step

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
    "vd_jfa_noalloc": (ctypes.c_int, [ctypes.POINTER(Config), _P, _P, _P]),
    "vd_set_seeds": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_remove_seeds": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_set_tail_fusion": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_server_set_policy": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vd_server_set_solo": (ctypes.c_int, [_P, ctypes.c_int64]),
    "vd_get_tail_fusion": (ctypes.c_int, [_P, _P, _P]),
    "vd_insert_seeds": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "vd_get_seed_set": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P, _P]),
    "vd_jfa_step": (ctypes.c_int, [_P]),
    "vd_djfa_step": (ctypes.c_int, [_P]),
    "vd_read_map": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_read_seeds": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "vd_map_device": (ctypes.c_int, [_P, ctypes.POINTER(_P)]),
    "vd_get_info": (ctypes.c_int, [_P, ctypes.POINTER(SimInfo)]),
    "vd_place_seeds": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_uint64, _P]),
    "vd_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(Timing)]),
    "vd_set_flood_variant": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_destroy": (None, [_P]),
    "vd_last_error": (ctypes.c_char_p, []),
    "vd_batch_footprint_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "vd_batch_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, _P, ctypes.c_size_t,
                                       _P, ctypes.POINTER(_P)]),
    "vd_batch_step": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "vd_batch_set_graph": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_batch_set_shape": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vd_batch_set_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "vd_batch_get_timing": (ctypes.c_int, [_P, ctypes.POINTER(Timing)]),
    "vd_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "vd_batch_destroy": (None, [_P]),
    "vd_batch_autotune": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vd_batch_set_solo": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64]),
    "vd_autotune": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vd_get_tuning": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32]),
    "vd_get_tuning_us": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "vd_tuning_export": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "vd_tuning_import": (ctypes.c_int, [ctypes.c_char_p]),
    "vd_tuning_clear": (ctypes.c_int, []),
}

STEP_JFA, STEP_DJFA = 0, 1
SERVE_STEPS, SERVE_PASSES = 0, 1


class ServerStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("pixel_updates", ctypes.c_int64), ("ticks", ctypes.c_int64),
        ("elapsed_s", ctypes.c_double), ("mean_ms", ctypes.c_double),
        ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("max_ms", ctypes.c_double),
        ("resident", ctypes.c_int32), ("waiting_admission", ctypes.c_int32),
    ]


SIGNATURES.update({
    "vd_server_footprint_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
    "vd_server_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_size_t, _P,
                                        ctypes.POINTER(_P)]),
    "vd_server_add_sim": (ctypes.c_int, [_P, ctypes.POINTER(Config), _P,
                                         ctypes.POINTER(ctypes.c_int32)]),
    "vd_server_submit": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(ctypes.c_int64)]),
    "vd_server_wait": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_double,
                                      ctypes.POINTER(ctypes.c_double)]),
    "vd_server_drain": (ctypes.c_int, [_P, ctypes.c_double]),
    "vd_server_remove_sim": (ctypes.c_int, [_P, ctypes.c_int32]),
    "vd_server_read_map": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_size_t]),
    "vd_server_sim_state": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "vd_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats), ctypes.c_int]),
    "vd_server_destroy": (None, [_P]),
})

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


NOALLOC_SCRATCH_BYTES = 72 << 20


def jfa_noalloc(cfg: Config, dev_xy: int, dev_map: int, stream=None):
    """vd_jfa_noalloc: the JFA diagram of the (x, y) int32 pairs at device
    address dev_xy into the width*height int32 map at device address
    dev_map (vd_read_map's encoding), queued on the stream; no allocation."""
    _check(lib().vd_jfa_noalloc(ctypes.byref(cfg), ctypes.c_void_p(dev_xy),
                                ctypes.c_void_p(dev_map), _stream_ptr(stream)))


def place_seeds(width: int, height: int, num_seeds: int, seed: int) -> np.ndarray:
    """vd_place_seeds: the (num_seeds, 2) int32 positions vd_init_sim draws
    from `seed` when it is given none (host only)."""
    out = np.empty((num_seeds, 2), dtype=np.int32)
    _check(lib().vd_place_seeds(width, height, num_seeds, seed, out.ctypes.data_as(_P)))
    return out


def init_sim(cfg: Config, xy, workspace, stream=None) -> ctypes.c_void_p:
    """Raw vd_init_sim; `workspace` is a uint8 CUDA tensor the caller keeps.
    xy None: the library draws the positions from cfg.sim_seed."""
    ptr = None
    if xy is not None:
        xy = np.ascontiguousarray(xy, dtype=np.int32)
        if xy.shape != (cfg.num_seeds, 2):
            raise ValueError(f"positions must be ({cfg.num_seeds}, 2) int32, got {xy.shape}")
        ptr = xy.ctypes.data_as(_P)
    h = ctypes.c_void_p()
    _check(lib().vd_init_sim(ctypes.byref(cfg), ptr,
                             ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
                             _stream_ptr(stream), ctypes.byref(h)))
    return h


def move_seeds(h):
    _check(lib().vd_move_seeds(h))


def set_seeds(h, xy):
    """Moves every seed to the given (S, 2) positions (one time step)."""
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    _check(lib().vd_set_seeds(h, a.ctypes.data_as(_P), a.size))


def remove_seeds(h, ids):
    """Removes the given present seeds from the seed set."""
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.int32).reshape(-1))
    _check(lib().vd_remove_seeds(h, a.ctypes.data_as(_P), a.size))


def insert_seeds(h, xy) -> np.ndarray:
    """Inserts seeds at the given (n, 2) positions into the lowest free
    slots; returns their indices."""
    a = np.ascontiguousarray(np.asarray(xy, dtype=np.int32).reshape(-1, 2))
    ids = np.empty(a.shape[0], np.int32)
    _check(lib().vd_insert_seeds(h, a.ctypes.data_as(_P), a.shape[0], ids.ctypes.data_as(_P)))
    return ids


def seed_set(h):
    """(present mask as bool array, number present, JFA fallbacks so far)."""
    info = get_info(h)
    m = np.empty(info.num_seeds, np.uint8)
    n = ctypes.c_int32()
    fb = ctypes.c_int64()
    _check(lib().vd_get_seed_set(h, m.ctypes.data_as(_P), m.size, ctypes.byref(n),
                                 ctypes.byref(fb)))
    return m.astype(bool), int(n.value), int(fb.value)


def set_tail_fusion(h, mode: int):
    """16, 24 or 32: fuse each step's last passes into one launch with tiles
    of that many rows (1: 16), 0: do not, -1: the default or the autotuner's
    choice."""
    _check(lib().vd_set_tail_fusion(h, int(mode)))


def get_tail_fusion(h):
    """(passes fused in a JFA step, in a dJFA step)."""
    j, d = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().vd_get_tail_fusion(h, ctypes.byref(j), ctypes.byref(d)))
    return int(j.value), int(d.value)


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


def read_map_into(h, host_ptr: int, count: int):
    """vd_read_map into caller-owned host memory of `count` int32 (for
    instance a pinned tensor's data_ptr())."""
    _check(lib().vd_read_map(h, ctypes.c_void_p(host_ptr), count))


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


def autotune(h, reps: int = 3):
    _check(lib().vd_autotune(h, reps))


def get_tuning(h):
    """[(variant, seg_rows)] per pass, JFA passes first, then dJFA."""
    info = get_info(h)
    n = info.passes_jfa + info.passes_djfa
    v = np.zeros(max(n, 1), np.int32)
    r = np.zeros(max(n, 1), np.int32)
    _check(lib().vd_get_tuning(h, v.ctypes.data_as(_P), r.ctypes.data_as(_P), n))
    return list(zip(v[:n].tolist(), r[:n].tolist()))


def get_tuning_us(h):
    """Best measured microseconds per launch of each pass's tuned choice
    (0 where never tuned), JFA passes first, then dJFA."""
    info = get_info(h)
    n = info.passes_jfa + info.passes_djfa
    us = np.zeros(max(n, 1), np.float32)
    _check(lib().vd_get_tuning_us(h, us.ctypes.data_as(_P), n))
    return us[:n].tolist()


def tuning_export() -> dict:
    """The process-wide tuning table as {key: [variant, seg_rows]}."""
    need = ctypes.c_size_t()
    _check(lib().vd_tuning_export(None, 0, ctypes.byref(need)))
    buf = ctypes.create_string_buffer(need.value)
    _check(lib().vd_tuning_export(buf, need.value, ctypes.byref(need)))
    out = {}
    for line in buf.value.decode().splitlines():
        key, v, r = line.rsplit("|", 2)
        out[key] = [int(v), int(r)]
    return out


def tuning_import(table: dict):
    text = "".join(f"{k}|{v[0]}|{v[1]}\n" for k, v in table.items())
    _check(lib().vd_tuning_import(text.encode()))


def tuning_clear():
    _check(lib().vd_tuning_clear())


def save_tuning(path: str):
    """Writes the tuning table as JSON."""
    import json
    with open(path, "w") as f:
        json.dump(tuning_export(), f, indent=1, sort_keys=True)


def load_tuning(path: str):
    import json
    with open(path) as f:
        tuning_import(json.load(f))


def batch_autotune(b, reps: int = 3):
    _check(lib().vd_batch_autotune(b, reps))


def destroy(h):
    if h:
        lib().vd_destroy(h)


def last_error() -> str:
    return lib().vd_last_error().decode()


class Sim:
    """A simulation and the workspace tensor it lives in."""

    def __init__(self, width, height, xy, device="cuda", stream=None, num_seeds=None, **kw):
        """xy None: num_seeds positions drawn by the library from sim_seed."""
        import torch
        n = num_seeds if xy is None else int(np.asarray(xy).shape[0])
        if n is None:
            raise ValueError("give positions or num_seeds")
        self.cfg = config(width, height, n, **kw)
        nbytes = footprint_bytes(self.cfg)
        if nbytes == 0:
            raise VdError(-1, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream
        self.handle = init_sim(self.cfg, xy, self.workspace, stream)

    def move_seeds(self):
        move_seeds(self.handle)

    def set_seeds(self, xy):
        set_seeds(self.handle, xy)

    def remove_seeds(self, ids):
        remove_seeds(self.handle, ids)

    def insert_seeds(self, xy) -> np.ndarray:
        return insert_seeds(self.handle, xy)

    def seed_set(self):
        return seed_set(self.handle)

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


# --- batches ----------------------------------------------------------------
def batch_footprint_bytes(n: int) -> int:
    return int(lib().vd_batch_footprint_bytes(n))


def batch_create(handles, workspace, stream=None) -> ctypes.c_void_p:
    arr = (ctypes.c_void_p * len(handles))(*[h.value if isinstance(h, ctypes.c_void_p) else h
                                             for h in handles])
    out = ctypes.c_void_p()
    _check(lib().vd_batch_create(arr, len(handles), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel(), _stream_ptr(stream), ctypes.byref(out)))
    return out


def batch_step(b, mode: int, move: bool):
    _check(lib().vd_batch_step(b, mode, int(bool(move))))


def batch_set_graph(b, enable: bool):
    _check(lib().vd_batch_set_graph(b, int(bool(enable))))


def batch_set_shape(b, wg_per_cu: int):
    _check(lib().vd_batch_set_shape(b, wg_per_cu))


def batch_set_timing(b, enable: bool):
    _check(lib().vd_batch_set_timing(b, int(bool(enable))))


def batch_get_timing(b) -> Timing:
    t = Timing()
    _check(lib().vd_batch_get_timing(b, ctypes.byref(t)))
    return t


def batch_info(b):
    lj, ld, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().vd_batch_info(b, ctypes.byref(lj), ctypes.byref(ld), ctypes.byref(g)))
    return lj.value, ld.value, g.value


def batch_destroy(b):
    if b:
        lib().vd_batch_destroy(b)


class Batch:
    """Simulations advanced together (vd_batch_*); keeps them and the
    batch workspace alive."""

    def __init__(self, sims, device="cuda", stream=None):
        import torch
        self.sims = list(sims)
        n = len(self.sims)
        self.workspace = torch.empty(batch_footprint_bytes(n), dtype=torch.uint8, device=device)
        self.handle = batch_create([s.handle for s in self.sims], self.workspace, stream)

    def step(self, mode: int, move: bool = True):
        batch_step(self.handle, mode, move)

    def set_graph(self, enable: bool):
        batch_set_graph(self.handle, enable)

    def set_shape(self, wg_per_cu: int):
        batch_set_shape(self.handle, wg_per_cu)

    def autotune(self, reps: int = 3):
        batch_autotune(self.handle, reps)

    def set_solo(self, mode: int, min_pixels: int):
        """Members of at least min_pixels pixels (<= 0: none) run `mode`
        steps' passes with their own launches."""
        _check(lib().vd_batch_set_solo(self.handle, mode, int(min_pixels)))

    def info(self):
        return batch_info(self.handle)

    def close(self):
        if self.handle:
            batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --- serving ----------------------------------------------------------------
class Server:
    """A serving loop over resident simulations (vd_server_*): time-step
    requests are queued per simulation and run on the GPU by the library's
    scheduler thread, as batched ticks (SERVE_PASSES, the default:
    continuous batching) or whole steps (SERVE_STEPS)."""

    def __init__(self, max_sims: int, pool_bytes: int, metric=EUCLID, device="cuda",
                 stream=None):
        import torch
        self.pool = torch.empty(pool_bytes, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().vd_server_create(max_sims, metric, ctypes.c_void_p(self.pool.data_ptr()),
                                      pool_bytes, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.shapes = {}

    @staticmethod
    def footprint_bytes(max_sims: int) -> int:
        return int(lib().vd_server_footprint_bytes(max_sims))

    def add_sim(self, width, height, xy, num_seeds=None, **kw) -> int:
        """xy None: num_seeds positions drawn by the library from sim_seed."""
        n = num_seeds if xy is None else int(np.asarray(xy).shape[0])
        if n is None:
            raise ValueError("give positions or num_seeds")
        cfg = config(width, height, n, **kw)
        ptr = None
        if xy is not None:
            xy = np.ascontiguousarray(xy, dtype=np.int32)
            ptr = xy.ctypes.data_as(_P)
        sid = ctypes.c_int32()
        _check(lib().vd_server_add_sim(self.handle, ctypes.byref(cfg), ptr, ctypes.byref(sid)))
        self.shapes[sid.value] = (height, width)
        return sid.value

    def set_policy(self, policy: int):
        _check(lib().vd_server_set_policy(self.handle, int(policy)))

    def set_solo(self, min_pixels: int):
        """Batched ticks: simulations of at least min_pixels pixels run
        alone (<= 0: all of them)."""
        _check(lib().vd_server_set_solo(self.handle, int(min_pixels)))

    def submit(self, sim_id: int, mode: int) -> int:
        t = ctypes.c_int64()
        _check(lib().vd_server_submit(self.handle, sim_id, mode, ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> float:
        lat = ctypes.c_double()
        _check(lib().vd_server_wait(self.handle, ticket, timeout_ms, ctypes.byref(lat)))
        return lat.value

    def drain(self, timeout_ms: float = -1.0):
        _check(lib().vd_server_drain(self.handle, timeout_ms))

    def remove_sim(self, sim_id: int):
        _check(lib().vd_server_remove_sim(self.handle, sim_id))

    def read_map(self, sim_id: int) -> np.ndarray:
        out = np.empty(self.shapes[sim_id], np.int32)
        _check(lib().vd_server_read_map(self.handle, sim_id, out.ctypes.data_as(_P), out.size))
        return out

    def sim_state(self, sim_id: int):
        r, t, p = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().vd_server_sim_state(self.handle, sim_id, ctypes.byref(r), ctypes.byref(t),
                                         ctypes.byref(p)))
        return {"resident": bool(r.value), "t": t.value, "pending": p.value}

    def stats(self, reset: bool = False) -> dict:
        st = ServerStats()
        _check(lib().vd_server_stats(self.handle, ctypes.byref(st), int(bool(reset))))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self.handle:
            lib().vd_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
