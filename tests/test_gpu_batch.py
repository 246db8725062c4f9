"""Batched steps (vd_batch_*): every member of a batch ends each step with
exactly the map and positions it has when it is stepped alone, in both
modes, with and without moves, with launches or replayed graphs; and the
alone runs equal the CPU oracle."""
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


# uneven members: sizes below, at and across the 256-column tile, tall,
# wide, one pixel, one seed, dense and sparse (so pass counts differ)
SHAPES = [(300, 200, 120, -2, 2), (64, 64, 4096, -1, 1), (1, 1, 1, -1, 1), (1000, 37, 50, -1, 3),
          (37, 900, 400, -2, 2), (512, 512, 256, -1, 1), (1024, 700, 30000, -3, 3),
          (257, 257, 1, -5, 5), (2048, 256, 2000, -1, 3)]


def _make(V, specs, metric=0, labels=None):
    out = []
    for j, (W, H, S, lo, hi) in enumerate(specs):
        xy = inputs.place_seeds(W, H, S, 50 + j)
        label = labels[j % len(labels)] if labels else 0
        out.append((xy, dict(disp_lo=lo, disp_hi=hi, sim_seed=900 + j, metric=metric,
                             label=label)))
    return out


def _run(V, specs, plan, metric=0, graph=False, tune=False, solo=None, variant=None, fuse=None,
         labels=None):
    made = _make(V, specs, metric, labels)
    members = [V.Sim(s[0], s[1], xy, **kw) for s, (xy, kw) in zip(specs, made)]
    alone = [V.Sim(s[0], s[1], xy, **kw) for s, (xy, kw) in zip(specs, made)]
    if variant is not None:
        for m in members:
            V.set_flood_variant(m.handle, variant)
    if fuse is not None:                 # solo members run their last passes fused or not
        for m in members:
            V.set_tail_fusion(m.handle, fuse)
    b = V.Batch(members)
    if tune:
        b.autotune(2)
    if solo is not None:
        for mode in (V.STEP_JFA, V.STEP_DJFA):
            b.set_solo(mode, solo)
    b.set_graph(graph)
    for t, (mode, move) in enumerate(plan):
        print(f"[batch] n={len(specs)} step={t} mode={mode} move={move} graph={graph}", flush=True)
        b.step(mode, move)
        for a in alone:
            if move:
                a.move_seeds()
            a.djfa_step() if mode == V.STEP_DJFA else a.jfa_step()
        for j, (m, a) in enumerate(zip(members, alone)):
            assert np.array_equal(m.read_seeds(), a.read_seeds()), (j, t)
            diff = int((m.read_map() != a.read_map()).sum())
            assert diff == 0, f"member {j} {specs[j]} differs from alone on {diff} px at step {t}"
            assert m.info().t == a.info().t
    b.close()
    return members, alone, made


def test_batch_equals_alone(V):
    plan = [(1, True), (1, True), (0, True), (1, False), (0, False), (1, True)]
    _run(V, SHAPES, plan)


def test_batch_graph_replays(V):
    """Graphs are captured on first use and replayed; eager reads between
    replays; every replay matches the alone runs."""
    plan = [(1, True)] * 4 + [(0, True)] * 2 + [(1, True)] * 2
    _run(V, SHAPES[:6], plan, graph=True)


def test_batch_autotuned(V):
    """The tuned persistent grid changes speed only."""
    _run(V, SHAPES, [(1, True), (0, True), (1, True)], graph=True, tune=True)


@pytest.mark.parametrize("fuse", [None, 0, 24])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("solo", [1, 100000])
def test_batch_solo_members(V, graph, solo, fuse):
    """Members of at least `solo` pixels run their passes with their own
    launches (all members for 1; the larger ones for 100000, the rest in the
    persistent levels), their last passes fused as the member's own steps
    would fuse them (default, off, 24-row tiles).  Mixed step kinds change
    which maps are current, so graphs are captured per parity
    configuration; every step still equals the alone runs."""
    plan = [(1, True), (1, True), (0, True), (1, True), (0, False), (1, True), (1, True)]
    _run(V, SHAPES, plan, graph=graph, solo=solo, variant=4, fuse=fuse)


def test_batch_manhattan(V):
    _run(V, SHAPES[:5], [(1, True), (0, True), (1, True)], metric=1)


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("solo", [-1, 60000])
def test_batch_xy_members(V, graph, solo):
    """XY and ID members mixed in one batch (their relabel, index and table
    copy run batched), fused or solo, every step equal to the lone runs."""
    plan = [(1, True), (0, True), (1, False), (1, True), (0, False), (1, True)]
    _run(V, SHAPES, plan, graph=graph, solo=solo, labels=[1, 0, 1])


def test_batch_xy_all_variants(V):
    _run(V, SHAPES, [(1, True), (1, True), (0, True)], variant=4, labels=[1])
    _run(V, SHAPES, [(1, True), (0, True), (1, True)], metric=1, labels=[1, 1, 0])


@pytest.mark.parametrize("label", [0, 1])
def test_batch_members_equal_oracle(V, label):
    specs = SHAPES[:5]
    members, _, made = _run(V, specs, [(1, True), (1, True), (0, True)], labels=[label])
    for (W, H, S, lo, hi), m, (xy, kw) in zip(specs, members, made):
        o = O.Sim(W, H, xy, kw["sim_seed"], lo, hi, label_mode=label)
        for mode in (1, 1, 0):
            o.move()
            o.djfa_step() if mode == 1 else o.jfa_step()
        assert np.array_equal(m.read_map(), o.map)


def test_batch_rejects_misuse(V):
    xy = inputs.place_seeds(100, 100, 10, 3)
    a = V.Sim(100, 100, xy)
    b = V.Batch([a])
    with pytest.raises(V.VdError):
        a.djfa_step()                      # driven by the batch
    with pytest.raises(V.VdError):
        V.Batch([a])                       # already in a batch
    with pytest.raises(V.VdError):
        V.set_tail_fusion(a.handle, 0)     # fixed while batched
    b.close()
    a.djfa_step()                          # free again
    # a member destroyed while batched is only marked; the batch keeps
    # stepping it and releases it when it is destroyed
    c = V.Sim(100, 100, xy)
    d = V.Sim(100, 100, xy, label=V.LABEL_XY16)
    bc = V.Batch([c, d])
    c.close()
    bc.step(V.STEP_DJFA, True)
    assert d.info().t == 1
    bc.close()


def test_batched_workload_subset(V):
    """The batched recipe's members at their real sizes (first 12 of 64)."""
    wl = inputs.batched()
    specs = [(s.width, s.height, s.num_seeds, s.disp_lo, s.disp_hi) for s in wl.sims[:12]]
    _run(V, specs, [(1, True), (0, True), (1, True)], graph=True)
