"""CPU oracle for JFA / dJFA -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does, and this package imports nothing from it.

The arithmetic lives in ``oracle.c`` (plain scalar C, int64); this module
loads ``liboracle.so`` with ctypes and composes its calls into the per-step
API the tests use.  Each wrapped C function cites its passage of the paper
("GPU Voronoi Diagrams for Random Moving Seeds") in ``oracle.c``.

Conventions: seed positions are int32 arrays of shape (S, 2) holding (x, y);
maps are int32 arrays of shape (H, W), row-major; EMPTY is -1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

EMPTY = -1
EUCLID, MANHATTAN = 0, 1
LABEL_ID, LABEL_XY = 0, 1
DMAX_MEASURED = -1
MOORE, VN = 0, 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (no GPU involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                        "-pthread", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        _declare(_lib)
    return _lib


_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
_p = ctypes.c_void_p


def _declare(L):
    sig = {
        "orc_mix64": (_u64, [_u64]),
        "orc_stream_out": (_u64, [_u64, _u64]),
        "orc_bounded": (_u32, [_u64, _u32]),
        "orc_move_seeds": (None, [_i32, _i32, _i32, _u64, _i64, _i32, _i32, _p]),
        "orc_k1": (_i32, [_i32, _i32]),
        "orc_delta1": (_i32, [_i32, _i32, _i32, _i32]),
        "orc_brute_force": (None, [_i32, _i32, _i32, _p, _i32, _p]),
        "orc_nearest_scan": (None, [_i32, _p, _i64, _p, _p, _p, _p]),
        "orc_nearest_bucketed": (None, [_i32, _i32, _i32, _p, _i64, _p, _p, _p, _p]),
        "orc_fill_empty": (None, [_i64, _p]),
        "orc_splat": (None, [_i32, _i32, _p, _i32, _p]),
        "orc_relabel_xy": (None, [_i32, _i32, _i32, _p, _p, _p]),
        "orc_pass": (None, [_i32, _i32, _p, _p, _p, _i32, _i32, _i32, _i32, _i32]),
        "orc_schedule": (_i32, [_i32, _i32, _i32, _i32, _i32, _i32, _i32, _p, _p, _i32]),
        "orc_run_passes": (None, [_i32, _i32, _p, _p, _p, _p, _i32, _i32, _i32, _i32]),
        "orc_jfa_step": (None, [_i32, _i32, _i32, _p, _i32, _i32, _i32, _p, _i32]),
        "orc_djfa_step": (None, [_i32, _i32, _i32, _p, _p, _i32, _i32, _i32, _i32, _i32, _p, _i32]),
        "orc_splat_active": (None, [_i32, _i32, _p, _p, _i32, _p]),
        "orc_relabel_xy_active": (None, [_i32, _i32, _i32, _p, _p, _p, _p]),
        "orc_purge_id": (None, [_i64, _p, _p]),
        "orc_jfa_step_active": (None, [_i32, _i32, _i32, _p, _p, _i32, _i32, _i32, _p, _i32]),
        "orc_djfa_step_active": (_i32, [_i32, _i32, _i32, _p, _p, _p, _p, _i32, _i32, _i32,
                                        _i32, _i32, _p, _i32]),
        "orc_count_equal": (_i64, [_i64, _p, _p]),
        "orc_count_exact": (_i64, [_i32, _p, _i32, _p, _i64, _p, _p, _p]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    return a.ctypes.data_as(ctypes.c_void_p)


def _xy(xy) -> np.ndarray:
    a = np.ascontiguousarray(xy, dtype=np.int32)
    assert a.ndim == 2 and a.shape[1] == 2, "seed positions are (S, 2) int32 (x, y)"
    return a


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --- RNG -----------------------------------------------------------------
def mix64(z: int) -> int:
    return lib().orc_mix64(z)


def stream_out(seed: int, n: int) -> int:
    return lib().orc_stream_out(seed, n)


def bounded(r: int, m: int) -> int:
    return lib().orc_bounded(r, m)


# --- schedules ----------------------------------------------------------
def k1(W: int, H: int) -> int:
    return lib().orc_k1(W, H)


def delta1(W: int, H: int, S: int, dmax: int) -> int:
    return lib().orc_delta1(W, H, S, dmax)


def schedule(W, H, S, dynamic, dmax=0, vn_passes=2, extra_passes=0):
    """[(k, nbhd), ...] of one JFA (dynamic=False) or dJFA (dynamic=True) step."""
    ks = np.zeros(80, np.int32)
    nb = np.zeros(80, np.int32)
    n = lib().orc_schedule(W, H, S, int(bool(dynamic)), dmax, vn_passes, extra_passes,
                           _ptr(ks), _ptr(nb), 80)
    return [(int(ks[i]), int(nb[i])) for i in range(n)]


# --- primitives ---------------------------------------------------------
def move_seeds(xy, W, H, sim_seed, t, lo, hi) -> np.ndarray:
    """Positions after the move of time step t >= 1 (returns a new array)."""
    a = _xy(xy).copy()
    lib().orc_move_seeds(W, H, a.shape[0], sim_seed, t, lo, hi, _ptr(a))
    return a


def brute_force(xy, W, H, metric=EUCLID) -> np.ndarray:
    a = _xy(xy)
    m = np.empty((H, W), np.int32)
    lib().orc_brute_force(W, H, a.shape[0], _ptr(a), metric, _ptr(m))
    return m


def nearest(xy, W, H, px, py, bucketed=True):
    """Exact Euclidean nearest seed (lowest index on ties) of sampled pixels."""
    a = _xy(xy)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    ids = np.empty(px.shape[0], np.int32)
    ds = np.empty(px.shape[0], np.int64)
    if bucketed:
        lib().orc_nearest_bucketed(W, H, a.shape[0], _ptr(a), px.shape[0], _ptr(px), _ptr(py),
                                   _ptr(ids), _ptr(ds))
    else:
        lib().orc_nearest_scan(a.shape[0], _ptr(a), px.shape[0], _ptr(px), _ptr(py),
                               _ptr(ids), _ptr(ds))
    return ids, ds


def splat(m: np.ndarray, xy, label_mode=LABEL_ID) -> np.ndarray:
    a = _xy(xy)
    out = np.ascontiguousarray(m, np.int32).copy()
    lib().orc_splat(out.shape[1], a.shape[0], _ptr(a), label_mode, _ptr(out))
    return out


def relabel_xy(m: np.ndarray, old_xy, new_xy) -> np.ndarray:
    o, n = _xy(old_xy), _xy(new_xy)
    out = np.ascontiguousarray(m, np.int32).copy()
    H, W = out.shape
    lib().orc_relabel_xy(W, H, o.shape[0], _ptr(o), _ptr(n), _ptr(out))
    return out


def flood_pass(m: np.ndarray, xy, k, nbhd=MOORE, metric=EUCLID, label_mode=LABEL_ID,
               nthreads=1) -> np.ndarray:
    a = _xy(xy)
    src = np.ascontiguousarray(m, np.int32)
    H, W = src.shape
    out = np.empty_like(src)
    lib().orc_pass(W, H, _ptr(a), _ptr(src), _ptr(out), k, nbhd, metric, label_mode, nthreads)
    return out


def run_passes(m: np.ndarray, xy, passes, metric=EUCLID, label_mode=LABEL_ID,
               nthreads=1) -> np.ndarray:
    a = _xy(xy)
    out = np.ascontiguousarray(m, np.int32).copy()
    H, W = out.shape
    ks = np.array([p[0] for p in passes] or [0], np.int32)
    nb = np.array([p[1] for p in passes] or [0], np.int32)
    lib().orc_run_passes(W, H, _ptr(a), _ptr(out), _ptr(ks), _ptr(nb), len(passes), metric,
                         label_mode, nthreads)
    return out


def jfa(xy, W, H, metric=EUCLID, label_mode=LABEL_ID, extra_passes=0, nthreads=None):
    a = _xy(xy)
    m = np.empty((H, W), np.int32)
    lib().orc_jfa_step(W, H, a.shape[0], _ptr(a), metric, label_mode, extra_passes, _ptr(m),
                       nthreads or default_threads())
    return m


def djfa(prev_map, old_xy, xy, dmax, metric=EUCLID, label_mode=LABEL_ID, vn_passes=2,
         extra_passes=0, nthreads=None):
    o, a = _xy(old_xy), _xy(xy)
    m = np.ascontiguousarray(prev_map, np.int32).copy()
    H, W = m.shape
    lib().orc_djfa_step(W, H, a.shape[0], _ptr(o), _ptr(a), dmax, metric, label_mode,
                        vn_passes, extra_passes, _ptr(m), nthreads or default_threads())
    return m


# --- a changing seed set (insertion and removal) ----------------------------
def _mask(m, S):
    if m is None:
        return None
    a = np.ascontiguousarray(m, dtype=np.uint8)
    assert a.shape == (S,), "a seed mask holds one byte per seed"
    return a


def splat_active(m: np.ndarray, xy, active, label_mode=LABEL_ID) -> np.ndarray:
    a = _xy(xy)
    act = _mask(active, a.shape[0])
    out = np.ascontiguousarray(m, np.int32).copy()
    lib().orc_splat_active(out.shape[1], a.shape[0], _ptr(a), None if act is None else _ptr(act),
                           label_mode, _ptr(out))
    return out


def relabel_xy_active(m: np.ndarray, old_xy, keep, new_xy) -> np.ndarray:
    o, n = _xy(old_xy), _xy(new_xy)
    kp = _mask(keep, o.shape[0])
    out = np.ascontiguousarray(m, np.int32).copy()
    H, W = out.shape
    lib().orc_relabel_xy_active(W, H, o.shape[0], _ptr(o), None if kp is None else _ptr(kp),
                                _ptr(n), _ptr(out))
    return out


def purge_id(m: np.ndarray, keep) -> np.ndarray:
    kp = np.ascontiguousarray(keep, dtype=np.uint8)
    out = np.ascontiguousarray(m, np.int32).copy()
    lib().orc_purge_id(out.size, _ptr(kp), _ptr(out))
    return out


def jfa_active(xy, active, W, H, metric=EUCLID, label_mode=LABEL_ID, extra_passes=0,
               nthreads=None):
    a = _xy(xy)
    act = _mask(active, a.shape[0])
    m = np.empty((H, W), np.int32)
    lib().orc_jfa_step_active(W, H, a.shape[0], _ptr(a), None if act is None else _ptr(act),
                              metric, label_mode, extra_passes, _ptr(m),
                              nthreads or default_threads())
    return m


def djfa_active(prev_map, old_xy, xy, keep, active, dmax, metric=EUCLID, label_mode=LABEL_ID,
                vn_passes=2, extra_passes=0, nthreads=None):
    """dJFA step after the seed set changed; returns (map, fell_back)."""
    o, a = _xy(old_xy), _xy(xy)
    kp, act = _mask(keep, a.shape[0]), _mask(active, a.shape[0])
    m = np.ascontiguousarray(prev_map, np.int32).copy()
    H, W = m.shape
    fb = lib().orc_djfa_step_active(W, H, a.shape[0], _ptr(o), _ptr(a),
                                    None if kp is None else _ptr(kp),
                                    None if act is None else _ptr(act), dmax, metric,
                                    label_mode, vn_passes, extra_passes, _ptr(m),
                                    nthreads or default_threads())
    return m, bool(fb)


def count_equal(a: np.ndarray, b: np.ndarray) -> int:
    a = np.ascontiguousarray(a, np.int32)
    b = np.ascontiguousarray(b, np.int32)
    assert a.shape == b.shape
    return int(lib().orc_count_equal(a.size, _ptr(a), _ptr(b)))


def count_exact(m: np.ndarray, xy, px, py, nearest_d, label_mode=LABEL_ID) -> int:
    a = _xy(xy)
    m = np.ascontiguousarray(m, np.int32)
    px = np.ascontiguousarray(px, np.int32)
    py = np.ascontiguousarray(py, np.int32)
    nd = np.ascontiguousarray(nearest_d, np.int64)
    return int(lib().orc_count_exact(m.shape[1], _ptr(a), label_mode, _ptr(m), px.shape[0],
                                     _ptr(px), _ptr(py), _ptr(nd)))


# --- a whole simulation -------------------------------------------------
class Sim:
    """One simulation as the oracle runs it: positions, time step, and the
    diagram carried from step to step (Alg. 1's VD).  ``init`` computes
    VD_0 by a full JFA on the initial positions; ``move`` advances t and
    moves the seeds; ``jfa_step`` and ``djfa_step`` replace the diagram."""

    def __init__(self, W, H, xy, sim_seed, disp_lo, disp_hi, label_mode=LABEL_ID,
                 metric=EUCLID, vn_passes=2, extra_passes=0, dmax=None, nthreads=None):
        self.W, self.H = W, H
        self.xy = _xy(xy).copy()
        self.S = self.xy.shape[0]
        self.sim_seed, self.lo, self.hi = sim_seed, disp_lo, disp_hi
        self.label_mode, self.metric = label_mode, metric
        self.vn_passes, self.extra_passes = vn_passes, extra_passes
        # dmax == DMAX_MEASURED: each dJFA step takes d_max from the moves
        # since the previous step (the sum of each move's largest per-axis
        # displacement), the bound on how far a seed got from the position
        # the diagram refers to
        self.measured = dmax == DMAX_MEASURED
        self.dmax = max(abs(disp_lo), abs(disp_hi)) if dmax is None or dmax <= 0 else dmax
        self.moved = 0
        self.nthreads = nthreads or default_threads()
        self.t = 0
        self.map = jfa(self.xy, W, H, metric, label_mode, extra_passes, self.nthreads)
        self.map_xy = self.xy          # positions the current diagram's labels refer to
        # The seed set: active[i] -- seed i is present now; keep[i] -- present
        # when the diagram was made and ever since; changed -- a seed was
        # inserted or removed since then.  A seed index is a slot of a table
        # of S entries; removal frees the slot, insertion takes free ones
        # (see insert).  Removed seeds neither move nor take part in a step.
        self.active = np.ones(self.S, bool)
        self.keep = np.ones(self.S, bool)
        self.removed = np.zeros(self.S, bool)     # removed since the diagram was made
        self.changed = False
        self.fell_back = False

    def _displace(self, new_xy):
        d = np.abs(new_xy.astype(np.int64) - self.xy)[self.active]
        self.moved += int(d.max()) if d.size else 0
        self.xy = new_xy

    def move(self):
        self.t += 1
        new = move_seeds(self.xy, self.W, self.H, self.sim_seed, self.t, self.lo, self.hi)
        new[~self.active] = self.xy[~self.active]
        self._displace(new)

    def remove(self, ids):
        """Removes the given present seeds (distinct indices)."""
        ids = np.asarray(ids, np.int64)
        assert len(set(ids.tolist())) == ids.size and self.active[ids].all()
        assert self.active.sum() > ids.size, "at least one seed stays"
        self.active[ids] = False
        self.keep[ids] = False
        self.removed[ids] = True
        self.changed = True

    def insert(self, xy):
        """Inserts seeds at the given positions into free slots, in ascending
        index order: first the slots free since before the diagram was made,
        then (if those run out) slots removed since, whose old labels the
        next dJFA step must purge; returns their indices."""
        a = _xy(xy)
        cold = np.flatnonzero(~self.active & ~self.removed)
        hot = np.flatnonzero(~self.active & self.removed)
        free = np.concatenate([cold, hot])[:a.shape[0]]
        assert free.size == a.shape[0], "not enough free slots"
        self.xy = self.xy.copy()
        self.xy[free] = a
        self.active[free] = True
        self.changed = True
        return free.astype(np.int32)

    def set_positions(self, xy):
        """Moves every seed to caller-given positions: one time step."""
        a = _xy(xy).copy()
        assert a.shape == self.xy.shape
        self.t += 1
        self._displace(a)

    def _settle(self):
        self.map_xy = self.xy
        self.moved = 0
        self.keep = self.active.copy()
        self.removed[:] = False
        self.changed = False

    def jfa_step(self):
        act = None if self.active.all() else self.active
        self.map = jfa_active(self.xy, act, self.W, self.H, self.metric, self.label_mode,
                              self.extra_passes, self.nthreads)
        self.fell_back = False
        self._settle()
        return self.map

    def djfa_step(self):
        dmax = self.moved if self.measured else self.dmax
        if self.changed or not self.active.all():
            self.map, self.fell_back = djfa_active(
                self.map, self.map_xy, self.xy, self.keep, self.active, dmax, self.metric,
                self.label_mode, self.vn_passes, self.extra_passes, self.nthreads)
        else:
            self.map = djfa(self.map, self.map_xy, self.xy, dmax, self.metric,
                            self.label_mode, self.vn_passes, self.extra_passes, self.nthreads)
            self.fell_back = False
        self._settle()
        return self.map
