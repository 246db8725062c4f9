"""GPU parity of a changing seed set (insertion and removal between steps).

The HIP path and the oracle run the same script of removals, insertions
(the same slots: the lowest free ones), moves and JFA / dJFA steps; the
bar is exact equality of positions, present masks, fallback counts and
every map after every step.  Cases cover both label encodings, both
metrics, ragged widths (single-column kernels) and widths divisible by 4
(four-column kernels), measured d_max, a slot removed and inserted again
before one step, a hole too wide for the dJFA passes (the step redone as
JFA), the full-size single workload, and the argument checks.
"""
import numpy as np
import pytest

import oracle as O
from paper_2209_00117_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_00117_amd import vdflood
    vdflood.lib()
    return vdflood


def _pair(V, W, H, xy, lo, hi, sim_seed=1, label=0, metric=0, vn=2, dmax=0, variant=None):
    kw = dict(disp_lo=lo, disp_hi=hi, label=label, metric=metric, vn_passes=vn,
              dmax_override=dmax, sim_seed=sim_seed)
    g = V.Sim(W, H, xy, **kw)
    if variant is not None:
        V.set_flood_variant(g.handle, variant)
    o = O.Sim(W, H, xy, sim_seed, lo, hi, label_mode=label, metric=metric, vn_passes=vn,
              dmax=dmax if dmax != 0 else None)
    return g, o


def _same(g, o, tag):
    pres, n, fb = g.seed_set()
    assert np.array_equal(pres, o.active), f"{tag}: present masks differ"
    assert n == int(o.active.sum())
    assert np.array_equal(g.read_seeds(), o.xy), f"{tag}: positions differ"
    m = g.read_map()
    bad = int((m != o.map).sum())
    assert bad == 0, f"{tag}: map differs on {bad} pixels"
    return fb


def run_script(V, W, H, S, steps, lo, hi, label=0, metric=0, vn=2, dmax=0, variant=None,
               seed=5, remove_frac=0.1, insert_frac=0.08, tag=""):
    """Each step: remove a share of the present seeds, insert into free
    slots, move, then a dJFA step (a JFA step every third step); the JFA and
    dJFA twins both follow the script."""
    print(f"[seedset] {tag} W={W} H={H} S={S} steps={steps} disp=[{lo},{hi}] label={label} "
          f"metric={metric} vn={vn} dmax={dmax} variant={variant}", flush=True)
    xy = inputs.place_seeds(W, H, S, seed)
    g, o = _pair(V, W, H, xy, lo, hi, seed, label, metric, vn, dmax, variant)
    rng = np.random.default_rng(seed)
    fallbacks = 0
    for t in range(1, steps + 1):
        on = np.flatnonzero(o.active)
        k = min(int(remove_frac * S), on.size - 1)
        if k > 0:
            gone = rng.choice(on, size=k, replace=False).astype(np.int32)
            g.remove_seeds(gone)
            o.remove(gone)
        free = int((~o.active).sum())
        m = min(int(insert_frac * S) + (t % 2), free)
        if m > 0:
            new = np.stack([rng.integers(0, W, m), rng.integers(0, H, m)], 1).astype(np.int32)
            ids = g.insert_seeds(new)
            assert np.array_equal(ids, o.insert(new)), f"{tag}: inserted slots differ"
        g.move_seeds(), o.move()
        if t % 3 == 0:
            g.jfa_step(), o.jfa_step()
        else:
            g.djfa_step(), o.djfa_step()
            fallbacks += int(o.fell_back)
        fb = _same(g, o, f"{tag} t={t}")
        assert fb == fallbacks, f"{tag} t={t}: {fb} fallbacks, oracle {fallbacks}"
    g.close()
    return fallbacks


@pytest.mark.parametrize("label", [0, 1])
@pytest.mark.parametrize("metric", [0, 1])
@pytest.mark.parametrize("W,H,S,lo,hi", [(512, 512, 256, -1, 1), (301, 177, 120, -2, 2),
                                         (1024, 96, 900, -3, 3)])
def test_script_parity(V, W, H, S, lo, hi, label, metric):
    run_script(V, W, H, S, 6, lo, hi, label=label, metric=metric, tag="script")


@pytest.mark.parametrize("variant", [1, 3, 4, 10])
def test_script_parity_variants(V, variant):
    for label in (0, 1):
        run_script(V, 640, 384, 500, 4, -2, 2, label=label, variant=variant, tag="variant")


@pytest.mark.parametrize("label", [0, 1])
def test_script_measured_dmax(V, label):
    run_script(V, 512, 320, 300, 6, -3, 3, label=label, dmax=O.DMAX_MEASURED, tag="measured")


@pytest.mark.parametrize("label", [0, 1])
def test_heavy_churn(V, label):
    """Half the present seeds removed before each step on a sparse grid;
    the fallback counts must agree, whatever they are."""
    fb = run_script(V, 256, 256, 40, 4, -1, 1, label=label, remove_frac=0.5, insert_frac=0.3,
                    tag="churn")
    print(f"[seedset] churn label={label}: {fb} fallbacks", flush=True)


@pytest.mark.parametrize("label", [0, 1])
def test_reinserted_slot(V, label):
    """A slot removed and inserted again elsewhere before one dJFA step."""
    W, H = 200, 160
    xy = inputs.place_seeds(W, H, 60, 3)
    g, o = _pair(V, W, H, xy, -1, 1, 3, label)
    for ids in ([6], [6, 7, 30]):
        g.remove_seeds(ids), o.remove(ids)
        new = np.array([[190, 5], [3, 150], [100, 80]][:len(ids)], np.int32)
        assert np.array_equal(g.insert_seeds(new), o.insert(new))
        g.move_seeds(), o.move()
        g.djfa_step(), o.djfa_step()
        _same(g, o, "reinserted")
    g.close()


@pytest.mark.parametrize("label", [0, 1])
def test_insert_prefers_cold_slots(V, label):
    """Slots free since before the last step are taken first; a slot freed
    since is reused (and its old labels purged) only when they run out."""
    W, H = 96, 64
    xy = inputs.place_seeds(W, H, 10, 2)
    g, o = _pair(V, W, H, xy, -1, 1, 2, label)
    g.remove_seeds([8, 4]), o.remove([8, 4])
    g.djfa_step(), o.djfa_step()
    g.remove_seeds([1, 6]), o.remove([1, 6])
    new = np.array([[1, 1], [2, 2], [3, 3]], np.int32)
    ids = g.insert_seeds(new)
    assert ids.tolist() == [4, 8, 1] and np.array_equal(ids, o.insert(new))
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    _same(g, o, "cold")
    g.close()


@pytest.mark.parametrize("label", [0, 1])
def test_set_seeds_with_absent_seeds(V, label):
    """Caller-given positions for every slot, absent ones included (they
    keep the new position while absent and count towards no displacement),
    with measured d_max; then the absent slots are inserted again."""
    W, H = 160, 120
    xy = inputs.place_seeds(W, H, 50, 8)
    g, o = _pair(V, W, H, xy, -1, 1, 8, label, dmax=O.DMAX_MEASURED)
    g.remove_seeds([1, 2, 40]), o.remove([1, 2, 40])
    rng = np.random.default_rng(8)
    for _ in range(2):
        new = np.clip(o.xy + rng.integers(-3, 4, o.xy.shape), 0, [W - 1, H - 1]).astype(np.int32)
        g.set_seeds(new), o.set_positions(new)
        g.djfa_step(), o.djfa_step()
        _same(g, o, "set_seeds")
    back = np.array([[5, 5], [150, 110], [80, 60]], np.int32)
    assert np.array_equal(g.insert_seeds(back), o.insert(back))
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    _same(g, o, "set_seeds+insert")
    g.close()


@pytest.mark.parametrize("label", [0, 1])
def test_unrefillable_hole_falls_back(V, label):
    W = H = 256
    rng = np.random.default_rng(1)
    crowd = np.stack([rng.integers(0, 20, 300), rng.integers(0, 20, 300)], 1)
    xy = np.concatenate([crowd, [[240, 240]]]).astype(np.int32)
    g, o = _pair(V, W, H, xy, -1, 1, 3, label)
    g.remove_seeds([300]), o.remove([300])
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    assert o.fell_back
    assert _same(g, o, "hole") == 1
    # the next step, with nothing changed, is a plain dJFA step
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    assert not o.fell_back and _same(g, o, "hole+1") == 1
    g.close()


def test_single_full_size_with_churn(V):
    """4096^2, 65536 seeds: 10% removed, 5% inserted, one move, one dJFA
    step, compared in full with the threaded oracle."""
    spec = inputs.single().sims[0]
    W, H = spec.width, spec.height
    xy = spec.positions()
    g, o = _pair(V, W, H, xy, spec.disp_lo, spec.disp_hi, spec.sim_seed)
    rng = np.random.default_rng(2)
    gone = rng.choice(len(xy), size=len(xy) // 10, replace=False).astype(np.int32)
    g.remove_seeds(gone), o.remove(gone)
    new = np.stack([rng.integers(0, W, len(xy) // 20), rng.integers(0, H, len(xy) // 20)],
                   1).astype(np.int32)
    assert np.array_equal(g.insert_seeds(new), o.insert(new))
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    _same(g, o, "single")
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    _same(g, o, "single+1")
    g.close()


def test_seed_set_rejects_bad_input(V):
    W, H = 64, 64
    xy = inputs.place_seeds(W, H, 8, 1)
    g = V.Sim(W, H, xy)
    with pytest.raises(V.VdError):
        g.remove_seeds(list(range(8)))              # none would stay
    with pytest.raises(V.VdError):
        g.remove_seeds([3, 3])                      # named twice
    with pytest.raises(V.VdError):
        g.remove_seeds([8])                         # out of range
    with pytest.raises(V.VdError):
        g.insert_seeds([[1, 1]])                    # no free slot
    assert g.seed_set()[1] == 8
    g.remove_seeds([2, 5])
    with pytest.raises(V.VdError):
        g.remove_seeds([2])                         # already removed
    with pytest.raises(V.VdError):
        g.insert_seeds([[1, 1], [64, 0]])           # off the grid
    with pytest.raises(V.VdError):
        g.insert_seeds([[1, 1], [2, 2], [3, 3]])    # two free slots
    pres, n, fb = g.seed_set()
    assert n == 6 and not pres[2] and not pres[5] and fb == 0
    # a batch refuses a simulation with a changed seed set
    import torch
    ws = torch.empty(V.batch_footprint_bytes(1), dtype=torch.uint8, device="cuda")
    with pytest.raises(V.VdError):
        V.batch_create([g.handle], ws)
    assert list(g.insert_seeds([[1, 1], [2, 2]])) == [2, 5]
    g.djfa_step()
    g.close()
