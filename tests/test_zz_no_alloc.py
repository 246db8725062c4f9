"""vd_jfa_noalloc, the allocation-free entry point, against the path it
mirrors: a simulation's VD_0 (vd_init_sim, a full JFA step on the given
positions) read back with vd_read_map.  Both are exact integer maps, so
they must be equal element by element.  Called through the C ABI."""
import numpy as np
import pytest

from paper_2209_00117_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_00117_amd import vdflood
    vdflood.lib()                    # fails loudly if the library is missing
    return torch, vdflood


def _reference(V, W, H, xy, **kw):
    s = V.Sim(W, H, xy, **kw)
    m = s.read_map()
    s.close()
    return m


def _noalloc(torch, V, W, H, xy, **kw):
    cfg = V.config(W, H, len(xy), **kw)
    dxy = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.int32)).cuda()
    dmap = torch.full((H, W), 12345, dtype=torch.int32, device="cuda")   # overwritten
    V.jfa_noalloc(cfg, dxy.data_ptr(), dmap.data_ptr())
    torch.cuda.synchronize()
    return dmap.cpu().numpy()


@pytest.mark.parametrize("label", [0, 1])
def test_noalloc_twice_second_smaller(env, label):
    """Two calls in a row, the second on a smaller map with fewer seeds (the
    scratch array still holds the first call's contents)."""
    torch, V = env
    for W, H, S, seed, kw in ((2000, 1500, 12000, 3, {}),
                              (333, 171, 700, 4, dict(metric=1, extra_passes=2))):
        xy = inputs.place_seeds(W, H, S, seed)
        print(f"[noalloc] {W}x{H} S={S} label={label} {kw}", flush=True)
        got = _noalloc(torch, V, W, H, xy, label=label, **kw)
        want = _reference(V, W, H, xy, label=label, **kw)
        assert np.array_equal(got, want), f"{W}x{H}: differs on {(got != want).sum()} pixels"


def test_noalloc_largest_and_degenerate(env):
    """The largest map the fixed scratch allows (4096 x 4096, 2^18 seeds),
    then a single pixel, a single row and coincident seeds."""
    torch, V = env
    cases = [(4096, 4096, inputs.place_seeds(4096, 4096, 1 << 18, 5)),
             (1, 1, np.array([[0, 0]], np.int32)),
             (97, 1, inputs.place_seeds(97, 1, 5, 6)),
             (64, 48, np.array([[10, 10], [10, 10], [50, 40], [10, 10]], np.int32))]
    for W, H, xy in cases:
        for label in (0, 1):
            print(f"[noalloc] {W}x{H} S={len(xy)} label={label}", flush=True)
            got = _noalloc(torch, V, W, H, xy, label=label)
            want = _reference(V, W, H, xy, label=label)
            assert np.array_equal(got, want), f"{W}x{H}: differs on {(got != want).sum()} pixels"


def test_noalloc_seeds_off_the_grid_take_no_part(env):
    """XY labels: seeds off the grid leave the map of the others unchanged."""
    torch, V = env
    W, H = 640, 480
    xy = inputs.place_seeds(W, H, 2000, 8)
    bad = np.array([[-1, 5], [W, 0], [3, H], [7, -9]], np.int32)
    mixed = np.concatenate([xy[:700], bad, xy[700:]])
    got = _noalloc(torch, V, W, H, mixed, label=1)
    assert np.array_equal(got, _reference(V, W, H, xy, label=1))


def test_noalloc_rejects_oversize(env):
    torch, V = env
    cfg = V.config(8192, 4096, 1000)           # 128 MiB partner map > 72 MiB
    dxy = torch.zeros((1000, 2), dtype=torch.int32, device="cuda")
    import ctypes
    rc = V.lib().vd_jfa_noalloc(ctypes.byref(cfg), dxy.data_ptr(), dxy.data_ptr(), None)
    assert rc == -1                              # VD_EINVAL, nothing launched
    assert b"scratch" in V.lib().vd_last_error()
