"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every map is integer labels, so the bar is exact equality at every time
step, for both the JFA and the dJFA simulation of each case.  The cases span
several tiles with ragged tails, degenerate grids (1 pixel, 1 row, 1
column), one seed, a saturated grid (S = W*H), heavy seed collisions, both
label encodings, both metrics and every pass option; the full-size
workloads run a few steps each in the launch configuration the benchmark
uses.
"""
import sys

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
    vdflood.lib()                    # fails loudly if the library is missing
    return vdflood


def _seed_pixels_ok(m, xy, label_mode):
    first = {}
    for i, (x, y) in enumerate(xy.tolist()):
        first.setdefault((x, y), i)
    for (x, y), i in first.items():
        want = i if label_mode == 0 else (y << 16 | x)
        if m[y, x] != want:
            return False
    return True


def run_twin(V, W, H, xy, steps, lo, hi, sim_seed=1, label=0, metric=0, vn=2, extra=0,
             dmax=0, tag="", variant=None, fuse=None, tune=False, tune_reps=1):
    """Runs a JFA and a dJFA simulation side by side on the GPU and in the
    oracle; asserts equal positions and maps at every step.  `variant` runs
    every pass on one kernel variant; the step's last passes are then fused
    only if `fuse` is 1 (otherwise `fuse` sets tail fusion, None: default).
    `tune` autotunes the first simulation before the second is made (which
    adopts the table), as bench.py does before it times."""
    if variant is not None and fuse is None:
        fuse = 0
    print(f"[parity] {tag} W={W} H={H} S={len(xy)} steps={steps} disp=[{lo},{hi}] "
          f"label={label} metric={metric} vn={vn} extra={extra} variant={variant} fuse={fuse} "
          f"tune={tune}", flush=True)
    kw = dict(disp_lo=lo, disp_hi=hi, label=label, metric=metric, vn_passes=vn,
              extra_passes=extra, dmax_override=dmax, sim_seed=sim_seed)
    gj = V.Sim(W, H, xy, **kw)
    if tune:
        V.autotune(gj.handle, tune_reps)
    gd = V.Sim(W, H, xy, **kw)
    if tune:
        assert V.get_tuning(gd.handle) == V.get_tuning(gj.handle)
    if variant is not None:
        V.set_flood_variant(gj.handle, variant)
        V.set_flood_variant(gd.handle, variant)
    if fuse is not None:
        V.set_tail_fusion(gj.handle, fuse)
        V.set_tail_fusion(gd.handle, fuse)
    okw = dict(label_mode=label, metric=metric, vn_passes=vn, extra_passes=extra,
               dmax=dmax if dmax > 0 else None)
    oj = O.Sim(W, H, xy, sim_seed, lo, hi, **okw)
    od = O.Sim(W, H, xy, sim_seed, lo, hi, **okw)
    m0 = gj.read_map()
    assert np.array_equal(m0, oj.map), f"{tag}: VD_0 differs"
    assert np.array_equal(gd.read_map(), oj.map)
    info = gd.info()
    assert info.passes_jfa == len(O.schedule(W, H, len(xy), False, extra_passes=extra))
    assert info.passes_djfa == len(O.schedule(W, H, len(xy), True, od.dmax, vn, extra))
    for t in range(1, steps + 1):
        gj.move_seeds(), gd.move_seeds(), oj.move(), od.move()
        gj.jfa_step(), gd.djfa_step()
        oj.jfa_step(), od.djfa_step()
        assert np.array_equal(gj.read_seeds(), oj.xy), f"{tag}: positions differ at t={t}"
        mj, md = gj.read_map(), gd.read_map()
        nj = int((mj != oj.map).sum())
        nd = int((md != od.map).sum())
        assert nj == 0, f"{tag}: JFA map differs at t={t} on {nj} pixels"
        assert nd == 0, f"{tag}: dJFA map differs at t={t} on {nd} pixels"
        assert _seed_pixels_ok(md, od.xy, label) and _seed_pixels_ok(mj, oj.xy, label)
    gj.close(), gd.close()
    return oj, od


def test_small_workload_id(V):
    spec = inputs.small().sims[0]
    oj, od = run_twin(V, spec.width, spec.height, spec.positions(), spec.steps, spec.disp_lo,
                      spec.disp_hi, tag="small")
    sim = O.count_equal(oj.map, od.map) / oj.map.size
    print(f"[parity] small: dJFA vs JFA similarity at last step {100 * sim:.3f}%")


def test_small_workload_xy(V):
    spec = inputs.small().sims[0]
    run_twin(V, spec.width, spec.height, spec.positions(), spec.steps, spec.disp_lo,
             spec.disp_hi, label=1, tag="small-xy")


@pytest.mark.parametrize("W,H,S,steps,lo,hi", [
    (1000, 1000, 50, 3, -2, 2),       # 50 seeds on 1000 x 1000, as in Fig. 6
    (1, 1, 1, 2, -1, 1),
    (1, 37, 5, 3, -1, 1),
    (53, 1, 3, 3, -2, 2),
    (333, 77, 1000, 3, -1, 1),
    (64, 64, 4096, 2, -1, 1),         # every pixel a seed
    (257, 129, 300, 6, -1, 3),        # drift piles seeds onto the far borders
    (130, 200, 1, 3, -5, 5),          # one seed: dJFA equals the exact diagram
])
@pytest.mark.parametrize("label", [0, 1])
def test_ragged_and_degenerate(V, W, H, S, steps, lo, hi, label):
    xy = inputs.place_seeds(W, H, S, W * 7 + H)
    run_twin(V, W, H, xy, steps, lo, hi, sim_seed=W + H, label=label, tag="ragged")


# Degenerate shapes for the four-column kernels (widths divisible by 4):
# one column group, one row, short chains (k >= H), a second tile holding a
# single group, every pixel a seed, seeds piled on the borders by drift.
@pytest.mark.parametrize("variant", [4, 5, 10, 11])
@pytest.mark.parametrize("W,H,S,steps,lo,hi", [
    (4, 4, 1, 2, -1, 1),
    (4, 37, 5, 3, -1, 1),
    (8, 1, 3, 3, -2, 2),
    (1024, 3, 50, 2, -2, 2),
    (1028, 64, 500, 2, -1, 1),
    (64, 64, 4096, 2, -1, 1),
    (260, 129, 300, 5, -1, 3),
])
@pytest.mark.parametrize("label", [0, 1])
def test_quad_degenerate(V, W, H, S, steps, lo, hi, label, variant):
    xy = inputs.place_seeds(W, H, S, W * 5 + H)
    run_twin(V, W, H, xy, steps, lo, hi, sim_seed=W + 2 * H, label=label, variant=variant,
             tag="quad")


@pytest.mark.parametrize("variant", [None, 4, 5, 10])
@pytest.mark.parametrize("metric,vn,extra", [
    (1, 2, 0), (0, 0, 0), (0, 1, 1), (0, 2, 2), (1, 1, 2), (0, 5, 0),
])
def test_pass_options(V, metric, vn, extra, variant):
    xy = inputs.place_seeds(700, 450, 900, 3)
    for label in (0, 1):
        run_twin(V, 700, 450, xy, 3, -2, 2, sim_seed=5, label=label, metric=metric, vn=vn,
                 extra=extra, tag="options", variant=variant)


# Widths: below, at and across the 256- and 1024-column tiles, one not a
# multiple of 4 (the four-column kernels then fall back); heights with
# ragged chains.
@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5, 6, 9, 10, 11])
@pytest.mark.parametrize("W,H,S", [(100, 90, 40), (700, 450, 900), (1100, 300, 5000),
                                   (257, 1200, 600), (2060, 340, 3000), (1024, 1030, 700)])
def test_flood_variants(V, variant, W, H, S):
    """Every kernel variant writes the same maps (k from 1 to 1024, widths
    below, at and across the 256-column tile, heights with ragged chains)."""
    xy = inputs.place_seeds(W, H, S, W + 3 * H)
    for label in (0, 1):
        run_twin(V, W, H, xy, 2, -2, 2, sim_seed=7, label=label, variant=variant,
                 tag="variant")


# Variants 4 and 5 (and 10, 11) at a step of at least half of both sides --
# a step's first pass when it starts at k1 -- run one lane per 2 x 2 block
# of four-column groups.  d_max is overridden so that dJFA steps start at k1
# too, with Von Neumann first passes; the shapes give blocks cut by both
# edges, one row, one group, and a width that is not a power of two.
@pytest.mark.parametrize("variant", [4, 11])
@pytest.mark.parametrize("W,H,S", [(700, 450, 900), (1028, 64, 300), (8, 1, 3), (4, 37, 5),
                                   (2060, 2000, 4000)])
@pytest.mark.parametrize("metric,vn", [(0, 2), (1, 1)])
@pytest.mark.parametrize("label", [0, 1])
def test_block_first_pass(V, variant, W, H, S, metric, vn, label):
    xy = inputs.place_seeds(W, H, S, W + 11 * H)
    run_twin(V, W, H, xy, 2, -3, 3, sim_seed=17, label=label, metric=metric, vn=vn,
             dmax=max(W, H), variant=variant, tag="block")


# Variant 4 (and 10) at steps of 128 and up where one column class (the
# columns congruent mod k) fits 16 lanes of two or four groups: lanes hold
# whole classes and swap their end groups over DPP.  The widths give 1 to 16
# lanes per class, both group counts, a last lane past the grid and classes
# cut by the width; d_max is overridden so that dJFA steps start at k1 with
# five Von Neumann passes, which reach these steps.
@pytest.mark.parametrize("variant", [4, 10])
@pytest.mark.parametrize("W,H,S", [(2060, 2000, 4000), (4100, 700, 3000), (1100, 300, 2000),
                                   (8188, 600, 6000)])
@pytest.mark.parametrize("metric,vn", [(0, 0), (1, 5)])
@pytest.mark.parametrize("label", [0, 1])
def test_class_tile(V, variant, W, H, S, metric, vn, label):
    xy = inputs.place_seeds(W, H, S, W + 13 * H)
    run_twin(V, W, H, xy, 2, -3, 3, sim_seed=19, label=label, metric=metric, vn=vn,
             dmax=max(W, H), variant=variant, tag="class")


# Tail fusion (the last passes of a step in one LDS-tiled launch): tiles of
# 48 x 32 outputs with up to 8 pixels of halo, so the shapes span one tile,
# ragged last tiles, grids smaller than the halo, and fused runs whose
# passes use the Von Neumann neighbourhood (dJFA with delta_1 <= 4).
@pytest.mark.parametrize("W,H,S,steps,lo,hi", [
    (1, 1, 1, 2, -1, 1),
    (2, 1, 2, 2, -1, 1),
    (3, 5, 4, 2, -1, 1),
    (7, 40, 9, 3, -1, 1),
    (48, 32, 30, 3, -1, 1),
    (49, 33, 60, 3, -2, 2),
    (100, 90, 40, 3, -2, 2),
    (64, 64, 1024, 3, -1, 1),         # delta_1 = 4: the fused passes 4, 2 are Von Neumann
    (333, 77, 1000, 3, -1, 1),
    (1000, 1000, 50, 2, -2, 2),
    (64, 64, 4096, 2, -1, 1),
    (257, 129, 300, 5, -1, 3),
])
@pytest.mark.parametrize("label", [0, 1])
def test_tail_fusion(V, W, H, S, steps, lo, hi, label):
    xy = inputs.place_seeds(W, H, S, W * 3 + H)
    run_twin(V, W, H, xy, steps, lo, hi, sim_seed=W + 5 * H, label=label, fuse=1, tag="tail")


@pytest.mark.parametrize("metric,vn,extra", [
    (1, 2, 0), (0, 0, 0), (0, 1, 1), (0, 2, 2), (1, 1, 2), (0, 5, 0), (1, 5, 1),
])
def test_tail_fusion_options(V, metric, vn, extra):
    """Manhattan, every Von Neumann count, JFA+1 / +2 (four fused passes:
    4, 2, 1, 1 or 2, 1, 2, 1), with the non-temporal store form too."""
    for S, variant in ((900, None), (5000, 10)):
        xy = inputs.place_seeds(700, 450, S, 3)
        for label in (0, 1):
            run_twin(V, 700, 450, xy, 3, -2, 2, sim_seed=5, label=label, metric=metric, vn=vn,
                     extra=extra, tag="tail-options", variant=variant, fuse=1)


def test_dmax_override(V):
    xy = inputs.place_seeds(512, 512, 4000, 9)
    run_twin(V, 512, 512, xy, 3, -1, 1, dmax=40, tag="dmax")


def _full_size(V, spec, steps, label=0, tune=False, tune_reps=1):
    """A full-size workload for a few steps; positions and maps compared in
    full against the threaded oracle."""
    return run_twin(V, spec.width, spec.height, spec.positions(), steps, spec.disp_lo,
                    spec.disp_hi, sim_seed=spec.sim_seed, label=label,
                    tag=f"{spec.width}x{spec.height}", tune=tune, tune_reps=tune_reps)


def test_single_full_size(V):
    """The 4096^2 workload with the autotuned kernels bench.py times."""
    oj, od = _full_size(V, inputs.single().sims[0], 2, tune=True)
    print(f"[parity] 4096^2: dJFA vs JFA similarity {100 * O.count_equal(oj.map, od.map) / oj.map.size:.4f}%")


@pytest.mark.parametrize("label", [0, 1])
def test_band_full_size(V, label):
    """One of eight row bands of 8192^2 with its halo rows (8192 x 1056),
    autotuned as bench.py runs it."""
    _full_size(V, inputs.band().sims[0], 2, label=label, tune=True)


@pytest.mark.parametrize("label", [0, 1])
def test_large_full_size(V, label):
    """The 8192^2 workload (2^20 seeds, moves in [-4, 4]) for two steps with
    the kernels bench.py times there: autotuned with its repetitions."""
    _full_size(V, inputs.large().sims[0], 2, label=label, tune=True, tune_reps=3)


def _arch():
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


@pytest.mark.parametrize("label", [0, 1])
def test_large_every_kernel(V, label):
    """Every choice the autotuner has at the 8192^2 workload's full size --
    kernel variants 0-11 x segment lengths (automatic, 8, 16, 64 rows) -- on
    real passes: ten runs, each giving the passes of VD_0 and of one JFA and
    one dJFA step other choices by a cyclic rotation (injected as a tuning
    table), so that every choice runs on JFA passes at two or more k and on
    at least one dJFA pass; maps compared in full with the oracle."""
    spec = inputs.large().sims[0]
    W, H, S = spec.width, spec.height, spec.num_seeds
    xy = spec.positions()
    print(f"[parity] every-kernel {W}x{H} S={S} label={label}", flush=True)
    oj = O.Sim(W, H, xy, spec.sim_seed, spec.disp_lo, spec.disp_hi, label_mode=label)
    od = O.Sim(W, H, xy, spec.sim_seed, spec.disp_lo, spec.disp_hi, label_mode=label)
    map0 = oj.map.copy()
    oj.move(), od.move()
    oj.jfa_step(), od.djfa_step()
    jfa_k = [k for k, _ in O.schedule(W, H, S, False)]
    djfa = O.schedule(W, H, S, True, od.dmax)
    choices = [(v, r) for v in range(12) for r in (0, 8, 16, 64)]
    arch, lab = _arch(), ("xy" if label else "id")
    kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed, label=label)
    try:
        for run in range(10):
            table = {}
            for i, k in enumerate(jfa_k):
                c = choices[(run * len(jfa_k) + i) % len(choices)]
                table[f"{arch} {W}x{H} S{S} {lab} euclid k{k} moore jfa"] = list(c)
            for j, (k, nb) in enumerate(djfa):
                c = choices[(run * len(djfa) + j) % len(choices)]
                table[f"{arch} {W}x{H} S{S} {lab} euclid k{k} {'vn' if nb else 'moore'} djfa"] = \
                    list(c)
            V.tuning_import(table)
            gj, gd = V.Sim(W, H, xy, **kw), V.Sim(W, H, xy, **kw)
            want = [tuple(table[key]) for key in table]
            assert V.get_tuning(gd.handle) == want, f"run {run}: table not adopted"
            assert np.array_equal(gj.read_map(), map0), f"run {run}: VD_0 differs"
            gj.move_seeds(), gd.move_seeds()
            gj.jfa_step(), gd.djfa_step()
            nj = int((gj.read_map() != oj.map).sum())
            nd = int((gd.read_map() != od.map).sum())
            gj.close(), gd.close()
            assert nj == 0 and nd == 0, f"run {run}: JFA differs on {nj}, dJFA on {nd} pixels"
    finally:
        V.tuning_clear()


@pytest.mark.parametrize("label", [0, 1])
def test_max_side_full_size(V, label):
    """The largest grid the library accepts (16368^2, 1 GiB per map): the
    squared distance from the sentinel to the far corner is the largest key
    the passes see, and byte offsets reach 2^30.  2^20 seeds; VD_0 (a full
    JFA step) and one dJFA step, compared in full."""
    W = H = 16368
    xy = inputs.place_seeds(W, H, 1 << 20, 17)
    print(f"[parity] max-side {W}x{H} S={len(xy)} label={label}", flush=True)
    g = V.Sim(W, H, xy, disp_lo=-4, disp_hi=4, sim_seed=17, label=label)
    o = O.Sim(W, H, xy, 17, -4, 4, label_mode=label)
    bad = int((g.read_map() != o.map).sum())            # VD_0: a full JFA step
    assert bad == 0, f"max-side: VD_0 differs on {bad} pixels"
    g.move_seeds(), o.move()
    g.djfa_step(), o.djfa_step()
    assert np.array_equal(g.read_seeds(), o.xy)
    bad = int((g.read_map() != o.map).sum())
    assert bad == 0, f"max-side: dJFA map differs on {bad} pixels"
    g.close()


@pytest.mark.parametrize("W,H", [(16367, 33), (33, 16367), (16368, 2), (1, 16368)])
def test_max_side_thin_grids(V, W, H):
    """One side at (or next to) the maximum, the other tiny: the first jump
    is 8192 along the long side and every candidate across the short side
    falls off the grid."""
    S = max(1, min(W * H // 50, 3000))
    xy = inputs.place_seeds(W, H, S, W + H)
    for label in (0, 1):
        run_twin(V, W, H, xy, 3, -3, 3, sim_seed=W, label=label, tag="thin")


@pytest.mark.parametrize("label", [0, 1])
def test_autotune_keeps_results(V, label):
    """Tuned kernel variants and segment lengths change speed only: a tuned
    simulation, a new one that adopts the table, and an untuned one stay
    bit-identical to each other and to the oracle.  Tuning replays a JFA and
    a dJFA step and then puts the diagram (and in XY mode the table it
    refers to) back, so it is run mid-trajectory here."""
    W, H, S = 700, 500, 2000
    xy = inputs.place_seeds(W, H, S, 4)
    kw = dict(disp_lo=-2, disp_hi=2, sim_seed=3, label=label)
    a = V.Sim(W, H, xy, **kw)
    b = V.Sim(W, H, xy, **kw)
    o = O.Sim(W, H, xy, 3, -2, 2, label_mode=label)
    for s in (a, b):
        s.move_seeds()
        s.djfa_step()
    o.move()
    o.djfa_step()
    m_before = a.read_map()
    V.autotune(a.handle, 2)
    assert np.array_equal(a.read_map(), m_before)          # tuning leaves the state alone
    tuned = V.get_tuning(a.handle)
    assert all(0 <= v < 12 and r in (0, 8, 16, 64) for v, r in tuned)
    assert all(us > 0 for us in V.get_tuning_us(a.handle))
    c = V.Sim(W, H, xy, **kw)                               # adopts the process-wide table
    assert V.get_tuning(c.handle) == tuned
    assert V.get_tail_fusion(c.handle) == V.get_tail_fusion(a.handle)
    c.move_seeds()
    c.djfa_step()
    for mode in (1, 1, 0, 1):
        for s in (a, b, c):
            s.move_seeds()
            s.djfa_step() if mode else s.jfa_step()
        o.move()
        o.djfa_step() if mode else o.jfa_step()
        for s in (a, b, c):
            assert np.array_equal(s.read_map(), o.map)


@pytest.mark.parametrize("label", [0, 1])
def test_measured_dmax_and_set_seeds(V, label):
    """dmax_override = DMAX_MEASURED: every dJFA step takes d_max from the
    displacement the moves since the previous step recorded on the device
    (vd_set_seeds moves seeds anywhere).  Positions, maps and the chosen
    first jump equal the oracle's at every step."""
    W, H, S = 600, 400, 800
    xy = inputs.place_seeds(W, H, S, 21)
    g = V.Sim(W, H, xy, disp_lo=-2, disp_hi=2, sim_seed=5, label=label,
              dmax_override=V.DMAX_MEASURED)
    o = O.Sim(W, H, xy, 5, -2, 2, label_mode=label, dmax=O.DMAX_MEASURED)
    rng = np.random.default_rng(3)

    def jump(n, reach):
        a = o.xy.copy()
        idx = rng.choice(S, n, replace=False)
        a[idx, 0] = np.clip(a[idx, 0] + rng.integers(-reach, reach + 1, n), 0, W - 1)
        a[idx, 1] = np.clip(a[idx, 1] + rng.integers(-reach, reach + 1, n), 0, H - 1)
        return a

    plan = ["move", "djfa", "jump150", "djfa", "move", "move", "djfa", "djfa", "jump3",
            "jfa", "move", "djfa", "jump40", "move", "djfa"]
    for i, op in enumerate(plan):
        print(f"[parity] measured label={label} op {i} {op}", flush=True)
        if op == "move":
            g.move_seeds(), o.move()
        elif op.startswith("jump"):
            a = jump(10, int(op[4:]))
            g.set_seeds(a), o.set_positions(a)
        elif op == "djfa":
            want = O.delta1(W, H, S, o.moved)
            g.djfa_step(), o.djfa_step()
            assert g.info().delta1 == want, (i, g.info().delta1, want)
        else:
            g.jfa_step(), o.jfa_step()
        assert np.array_equal(g.read_seeds(), o.xy), f"positions differ after op {i}"
        if op in ("djfa", "jfa"):
            diff = int((g.read_map() != o.map).sum())
            assert diff == 0, f"map differs after op {i} ({op}) on {diff} px"
        assert g.info().t == o.t


@pytest.mark.parametrize("label", [0, 1])
def test_library_placement(V, label):
    """vd_init_sim with no positions draws them from sim_seed exactly as the
    input generator does; the simulation then matches the oracle's."""
    W, H, S, seed = 700, 450, 900, 13
    print(f"[parity] library placement W={W} H={H} S={S} seed={seed} label={label}", flush=True)
    g = V.Sim(W, H, None, num_seeds=S, sim_seed=seed, disp_lo=-2, disp_hi=2, label=label)
    xy = inputs.place_seeds(W, H, S, seed)
    assert np.array_equal(g.read_seeds(), xy)
    o = O.Sim(W, H, xy, seed, -2, 2, label_mode=label)
    assert np.array_equal(g.read_map(), o.map)
    for _ in range(2):
        g.move_seeds(), o.move()
        g.djfa_step(), o.djfa_step()
        assert np.array_equal(g.read_seeds(), o.xy)
        assert np.array_equal(g.read_map(), o.map)
    g.close()


def test_set_seeds_rejects_bad_input(V):
    g = V.Sim(64, 64, inputs.place_seeds(64, 64, 10, 1))
    with pytest.raises(V.VdError):
        g.set_seeds(np.zeros((9, 2), np.int32))                      # wrong count
    bad = g.read_seeds().copy()
    bad[3] = (64, 0)                                                 # off the grid
    with pytest.raises(V.VdError):
        g.set_seeds(bad)
    assert g.info().t == 0                                           # nothing changed


def test_read_map_into_caller_memory(V):
    """vd_read_map into pinned and pageable caller memory gives the same
    diagram as the binding's own array (ID and XY labels)."""
    import torch
    W, H = 300, 200
    xy = inputs.place_seeds(W, H, 150, 6)
    for label in (0, 1):
        g = V.Sim(W, H, xy, label=label)
        g.move_seeds(), g.djfa_step()
        ref = g.read_map()
        pinned = torch.zeros(W * H, dtype=torch.int32, pin_memory=True)
        V.read_map_into(g.handle, pinned.data_ptr(), W * H)
        assert np.array_equal(pinned.numpy().reshape(H, W), ref)
        plain = np.zeros(W * H, np.int32)
        V.read_map_into(g.handle, plain.ctypes.data, W * H)
        assert np.array_equal(plain.reshape(H, W), ref)
        with pytest.raises(V.VdError):
            V.read_map_into(g.handle, plain.ctypes.data, W * H - 1)
        g.close()


@pytest.mark.parametrize("fill", [0x00, 0x01, 0xFF])
def test_xy_index_in_dirty_workspace(V, fill):
    """XY dJFA steps in a workspace whose bytes all start as `fill` (0 and
    small values lie below every seed label, so an old-position index built
    by atomic minima must not trust what the workspace held), with
    coincident seeds and a removed seed: every map equals the oracle's."""
    import torch
    W, H, S = 256, 192, 300
    xy = inputs.place_seeds(W, H, S, 21)
    xy[7] = xy[3]                    # coincident seeds from the start
    xy[150] = xy[3]
    kw = dict(disp_lo=-2, disp_hi=2, label=1)
    g = V.Sim.__new__(V.Sim)
    g.cfg = V.config(W, H, S, **kw)
    g.workspace = torch.full((V.footprint_bytes(g.cfg),), fill, dtype=torch.uint8,
                             device="cuda")
    g.stream = None
    g.handle = V.init_sim(g.cfg, xy, g.workspace, None)
    o = O.Sim(W, H, xy, 1, -2, 2, label_mode=1)
    assert np.array_equal(g.read_map(), o.map)
    for t in range(1, 7):
        if t == 3:
            g.remove_seeds([3, 40]), o.remove([3, 40])
        g.move_seeds(), o.move()
        if t == 5:                   # a JFA step starting from the previous diagram
            g.jfa_step(), o.jfa_step()
        else:
            g.djfa_step(), o.djfa_step()
        nd = int((g.read_map() != o.map).sum())
        assert nd == 0, f"fill={fill:#x}: map differs at t={t} on {nd} pixels"
    g.close()


def test_xy_index_epochs_and_batch(V):
    """An XY simulation through more dJFA steps than the index has epoch
    values (so the index is refilled and its epochs restart), with three
    batched steps in between (the batch keeps its own form of the index in
    the same memory): every map equals the oracle's."""
    W, H, S = 64, 48, 40
    xy = inputs.place_seeds(W, H, S, 9)
    xy[5] = xy[1]
    g = V.Sim(W, H, xy, disp_lo=-1, disp_hi=1, label=1)
    o = O.Sim(W, H, xy, 1, -1, 1, label_mode=1)
    for t in range(1, 271):
        if t == 120:
            b = V.Batch([g])
            for _ in range(3):
                b.step(V.STEP_DJFA)
                o.move(), o.djfa_step()
            b.close()
            assert np.array_equal(g.read_map(), o.map), "after the batched steps"
        g.move_seeds(), o.move()
        if t in (121, 200):
            g.jfa_step(), o.jfa_step()
        else:
            g.djfa_step(), o.djfa_step()
        nd = int((g.read_map() != o.map).sum())
        assert nd == 0, f"map differs at step {t} on {nd} pixels"
    g.close()


@pytest.mark.parametrize("d,moves", [(7, 1), (8, 1), (3, 2), (4, 2), (1, 9)])
def test_xy_index_move_reach(V, d, moves):
    """XY dJFA steps after `moves` moves of up to d pixels per axis: up to 7
    pixels in all the index codes each seed's move, beyond that the step
    relabels in a pass of its own; both give the oracle's maps."""
    W, H, S = 192, 160, 200
    xy = inputs.place_seeds(W, H, S, 33)
    xy[9] = xy[2]
    g = V.Sim(W, H, xy, disp_lo=-d, disp_hi=d, label=1, sim_seed=4)
    o = O.Sim(W, H, xy, 4, -d, d, label_mode=1)
    for t in range(1, 5):
        for _ in range(moves):
            g.move_seeds(), o.move()
        g.djfa_step(), o.djfa_step()
        nd = int((g.read_map() != o.map).sum())
        assert nd == 0, f"d={d} moves={moves}: dJFA map differs at step {t} on {nd} pixels"
    g.close()


@pytest.mark.parametrize("label", [0, 1])
def test_djfa_splat_over_stale_labels(V, label):
    """Seeds moved (vd_set_seeds) onto pixels that hold smaller labels of
    seeds now elsewhere, and two seeds onto one pixel: the dJFA splat must
    replace the stale labels and leave the lowest coincident label, as the
    oracle's splat of the present seeds does."""
    W = H = 48
    xy = np.array([[2, 2], [40, 40], [10, 30], [30, 10], [24, 24]], np.int32)
    g = V.Sim(W, H, xy, label=label, dmax_override=40)
    o = O.Sim(W, H, xy, 1, -1, 1, label_mode=label, dmax=40)
    # seed 4 and seed 3 onto the pixel seed 1 labelled, seed 2 onto seed 0's cell
    new = xy.copy()
    new[4] = [36, 36]
    new[3] = [36, 36]
    new[2] = [4, 3]
    g.set_seeds(new), o.set_positions(new)
    g.djfa_step(), o.djfa_step()
    m = g.read_map()
    assert np.array_equal(m, o.map)
    if label == 0:
        assert m[36, 36] == 3 and m[3, 4] == 2 and m[2, 2] == 0
    g.close()
