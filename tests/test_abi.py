"""The C-ABI library loads and exports what include/vdflood.h declares;
argument validation that needs no device (no compute calls here)."""
import ctypes
import os
import re

import pytest

from paper_2209_00117_amd import vdflood as V

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vdflood.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b(vd_[a-z_]+)\s*\(", src))


def test_library_exports_every_declared_symbol():
    L = V.lib()
    declared = _declared()
    assert {"vd_init_sim", "vd_move_seeds", "vd_jfa_step", "vd_djfa_step",
            "vd_read_map"} <= declared
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(V.SIGNATURES), declared ^ set(V.SIGNATURES)


def test_binding_struct_layout_matches_header():
    # vd_config: 10 int32 then one uint64 -> 48 bytes with alignment
    assert ctypes.sizeof(V.Config) == 48
    assert ctypes.sizeof(V.SimInfo) == 48
    assert ctypes.sizeof(V.Timing) == 40


def test_footprint():
    c = V.config(512, 512, 256)
    npix = 512 * 512 * 4
    # two maps, the seed table with its sentinel entry (256-B aligned), step
    # counters (256 B), seed-set state (1 B per seed, 256-B aligned), ID
    # mode: parked positions (4 B per seed), slack (256 B)
    assert V.footprint_bytes(c) == 2 * npix + 1280 + 256 + 256 + 1024 + 256
    cx = V.config(512, 512, 256, label=V.LABEL_XY16)
    # XY mode: a third map (the old-position index of dJFA steps) and the
    # positions the diagram refers to instead of the parked positions
    assert V.footprint_bytes(cx) == 3 * npix + 1280 + 1280 + 256 + 256 + 256
    big = V.config(8192, 8192, 1 << 20)
    assert V.footprint_bytes(big) == (2 * 8192 * 8192 * 4 + 4 * (1 << 20) + 256 + 256
                                      + (1 << 20) + 4 * (1 << 20) + 256)
    assert V.footprint_bytes(V.config(16368, 16368, 1)) > 0
    assert V.footprint_bytes(V.config(16369, 8, 1)) == 0


@pytest.mark.parametrize("kw", [
    dict(width=0, height=8, num_seeds=1), dict(width=8, height=16369, num_seeds=1),
    dict(width=8, height=8, num_seeds=0), dict(width=8, height=8, num_seeds=65),
    dict(width=8, height=8, num_seeds=2, disp_lo=2, disp_hi=1),
    dict(width=8, height=8, num_seeds=2, label=7), dict(width=8, height=8, num_seeds=2, metric=3),
    dict(width=8, height=8, num_seeds=2, extra_passes=3),
    dict(width=8, height=8, num_seeds=2, vn_passes=-1),
    dict(width=8, height=8, num_seeds=2, dmax_override=-2),
])
def test_invalid_config_rejected_before_device_work(kw):
    w, h, s = kw.pop("width"), kw.pop("height"), kw.pop("num_seeds")
    c = V.config(w, h, s, **kw)
    assert V.footprint_bytes(c) == 0
    out = ctypes.c_void_p()
    xy = (ctypes.c_int32 * 4)(0, 0, 1, 1)
    st = V.lib().vd_init_sim(ctypes.byref(c), ctypes.cast(xy, ctypes.c_void_p),
                             ctypes.c_void_p(0x1000), 1 << 30, None, ctypes.byref(out))
    assert st == -1 and not out.value
    assert V.last_error()


def test_null_and_small_workspace():
    c = V.config(8, 8, 2)
    xy = (ctypes.c_int32 * 4)(0, 0, 1, 1)
    out = ctypes.c_void_p()
    L = V.lib()
    # positions drawn by the library (host_xy NULL) still need a valid
    # config and a large enough workspace before any device work
    bad_cfg = V.config(8, 8, 65)
    assert L.vd_init_sim(ctypes.byref(bad_cfg), None, ctypes.c_void_p(0x1000), 1 << 20, None,
                         ctypes.byref(out)) == -1
    assert L.vd_init_sim(ctypes.byref(c), None, ctypes.c_void_p(0x1000), 100, None,
                         ctypes.byref(out)) == -2
    assert L.vd_init_sim(ctypes.byref(c), ctypes.cast(xy, ctypes.c_void_p), None, 1 << 20, None,
                         ctypes.byref(out)) == -1
    assert L.vd_init_sim(ctypes.byref(c), ctypes.cast(xy, ctypes.c_void_p),
                         ctypes.c_void_p(0x1000), 100, None, ctypes.byref(out)) == -2
    assert "workspace" in V.last_error()
    bad = (ctypes.c_int32 * 4)(0, 0, 8, 1)       # x = 8 is off an 8-wide grid
    assert L.vd_init_sim(ctypes.byref(c), ctypes.cast(bad, ctypes.c_void_p),
                         ctypes.c_void_p(0x1000), 1 << 20, None, ctypes.byref(out)) == -1
    assert "outside" in V.last_error()
    for fn in ("vd_move_seeds", "vd_jfa_step", "vd_djfa_step"):
        assert getattr(L, fn)(None) == -1
    ids = (ctypes.c_int32 * 2)(0, 1)
    assert L.vd_remove_seeds(None, ctypes.cast(ids, ctypes.c_void_p), 2) == -1
    assert L.vd_insert_seeds(None, ctypes.cast(xy, ctypes.c_void_p), 2,
                             ctypes.cast(ids, ctypes.c_void_p)) == -1
    assert L.vd_get_seed_set(None, None, 0, None, None) == -1
    L.vd_destroy(None)


def test_tuning_table_round_trip():
    """The tuning table's text form (no device work involved)."""
    V.tuning_import({"gfx950 64x64 S10 id euclid k32 moore": [3, 16],
                     "gfx950 64x64 S10 xy euclid k1 vn": [1, 0]})
    t = V.tuning_export()
    assert t["gfx950 64x64 S10 id euclid k32 moore"] == [3, 16]
    assert t["gfx950 64x64 S10 xy euclid k1 vn"] == [1, 0]
    for bad in ("no separators\n", "k|99|0\n", "k|-1|0\n", "k|1|999\n"):
        assert V.lib().vd_tuning_import(bad.encode()) == -1


# vd_place_seeds is host code: the library draws the same initial positions
# as the input generator the tests and the oracle use (shapes: one pixel, a
# saturated grid, a single row and column, the 4096^2 and 8192^2 workloads).
@pytest.mark.parametrize("W,H,S,seed", [(1, 1, 1, 5), (64, 64, 4096, 3), (1000, 1, 700, 9),
                                        (1, 900, 899, 2), (1000, 700, 5000, 17),
                                        (4096, 4096, 65536, 1), (8192, 8192, 1 << 20, 1)])
def test_place_seeds_matches_input_generator(W, H, S, seed):
    from paper_2209_00117_amd import inputs
    got = V.place_seeds(W, H, S, seed)
    want = inputs.place_seeds(W, H, S, seed)
    assert got.shape == want.shape and (got == want).all()
    assert len({(int(x), int(y)) for x, y in got}) == S


def test_place_seeds_rejects_bad_arguments():
    out = (ctypes.c_int32 * 16)()
    L = V.lib()
    for w, h, s in ((0, 4, 1), (4, 16369, 1), (2, 2, 0), (2, 2, 5)):
        assert L.vd_place_seeds(w, h, s, 1, ctypes.cast(out, ctypes.c_void_p)) == -1
        assert V.last_error()
    assert L.vd_place_seeds(2, 2, 1, 1, None) == -1
