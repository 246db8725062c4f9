"""Randomised GPU parity: seeded draws over every option at once.

Each case draws a grid (1..2052 columns, so up to three workgroups across,
and 1..399 rows), a seed count (up to the pixel count), a move range, the
label encoding, the metric, the Von Neumann and extra pass counts, d_max
(bound, measured or overridden), a forced kernel variant or the defaults,
tail fusion, and a changing seed set or not; a JFA
and a dJFA twin then run four steps on the GPU and in the oracle, and
positions, present masks and every map must agree exactly.  Random batches
and random servers are drawn the same way and compared with the oracle
after every step or drain.  The draws are fixed by the case number, so a
failure names a reproducible configuration.
"""
import numpy as np
import pytest

import oracle as O
from paper_2209_00117_amd import inputs

pytestmark = pytest.mark.gpu

N_CASES = 160


@pytest.fixture(scope="module")
def V():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2209_00117_amd import vdflood
    vdflood.lib()
    return vdflood


def draw(case: int) -> dict:
    r = np.random.default_rng(1000 + case)
    W = int(r.choice([1, 2, 3, 4, 7, 16, 33, 64, 100, 128, 255, 256, 300, 400, 1028, 1100,
                      2052]))
    H = int(r.choice([1, 2, 5, 8, 31, 64, 97, 128, 200, 256, 399]))
    S = int(min(W * H, max(1, int(r.integers(1, 2000)))))
    lo = int(r.integers(-4, 3))
    hi = int(r.integers(lo, 5))
    dm = int(r.integers(0, 3))
    return dict(W=W, H=H, S=S, lo=lo, hi=hi, label=int(r.integers(0, 2)),
                metric=int(r.integers(0, 2)), vn=int(r.integers(0, 4)),
                extra=int(r.integers(0, 3)),
                dmax=(0, O.DMAX_MEASURED, int(r.integers(1, 20)))[dm],
                variant=int(r.integers(-1, 12)), fuse=int(r.choice([-1, 0, 1, 24])),
                churn=bool(r.integers(0, 2)) and S >= 4, seed=int(r.integers(1, 1 << 30)))


@pytest.mark.parametrize("case", range(N_CASES))
def test_random_configuration(V, case):
    c = draw(case)
    print(f"[random] case {case}: {c}", flush=True)
    W, H, S = c["W"], c["H"], c["S"]
    xy = inputs.place_seeds(W, H, S, c["seed"])
    kw = dict(disp_lo=c["lo"], disp_hi=c["hi"], label=c["label"], metric=c["metric"],
              vn_passes=c["vn"], extra_passes=c["extra"], dmax_override=c["dmax"],
              sim_seed=c["seed"])
    okw = dict(label_mode=c["label"], metric=c["metric"], vn_passes=c["vn"],
               extra_passes=c["extra"], dmax=c["dmax"] if c["dmax"] != 0 else None)
    gj, gd = V.Sim(W, H, xy, **kw), V.Sim(W, H, xy, **kw)
    for g in (gj, gd):
        V.set_flood_variant(g.handle, c["variant"])
        V.set_tail_fusion(g.handle, c["fuse"])
    oj = O.Sim(W, H, xy, c["seed"], c["lo"], c["hi"], **okw)
    od = O.Sim(W, H, xy, c["seed"], c["lo"], c["hi"], **okw)
    assert np.array_equal(gj.read_map(), oj.map), f"case {case}: VD_0 differs"
    rng = np.random.default_rng(case)
    for t in range(1, 5):
        if c["churn"]:
            on = np.flatnonzero(od.active)
            k = min(max(1, S // 8), on.size - 1)
            if k > 0:
                gone = rng.choice(on, size=k, replace=False).astype(np.int32)
                for s in (gj, gd, oj, od):
                    (s.remove_seeds if hasattr(s, "remove_seeds") else s.remove)(gone)
            m = min(max(1, S // 10), int((~od.active).sum()))
            if m > 0:
                new = np.stack([rng.integers(0, W, m), rng.integers(0, H, m)],
                               1).astype(np.int32)
                ids = [gj.insert_seeds(new), gd.insert_seeds(new), oj.insert(new),
                       od.insert(new)]
                assert all(np.array_equal(ids[0], i) for i in ids[1:]), \
                    f"case {case}: slots differ"
        for s in (gj, gd):
            s.move_seeds()
        oj.move(), od.move()
        gj.jfa_step(), gd.djfa_step()
        oj.jfa_step(), od.djfa_step()
        for g, o, kind in ((gj, oj, "JFA"), (gd, od, "dJFA")):
            assert np.array_equal(g.read_seeds(), o.xy), f"case {case} t={t}: positions differ"
            assert np.array_equal(g.seed_set()[0], o.active)
            bad = int((g.read_map() != o.map).sum())
            assert bad == 0, f"case {case} t={t}: {kind} map differs on {bad} pixels"
    gj.close(), gd.close()


N_BATCH_CASES = 64


def draw_batch(case: int) -> dict:
    r = np.random.default_rng(5000 + case)
    members = []
    for j in range(int(r.integers(1, 11))):
        W = int(r.choice([1, 5, 64, 100, 256, 300, 1024, 1030]))
        H = int(r.choice([1, 7, 64, 200, 333]))
        lo = int(r.integers(-4, 3))
        members.append(dict(W=W, H=H, S=int(min(W * H, int(r.integers(1, 3000)))), lo=lo,
                            hi=int(r.integers(lo, 5)), vn=int(r.integers(0, 4)),
                            extra=int(r.integers(0, 3)),
                            dmax=int(r.choice([0, 0, int(r.integers(1, 20))])),
                            variant=int(r.integers(-1, 12)),
                            fuse=int(r.choice([-1, 0, 1, 24])),
                            seed=int(r.integers(1, 1 << 30))))
    plan = [(int(r.integers(0, 2)), bool(r.integers(0, 4))) for _ in range(6)]
    rl = np.random.default_rng(7000 + case)    # label encodings, drawn apart from the rest
    for m in members:
        m["label"] = int(rl.integers(0, 2))
    return dict(members=members, metric=int(r.integers(0, 2)), graph=bool(r.integers(0, 2)),
                shape=int(r.choice([0, 1, 2, 4, 8])),
                solo=int(r.choice([-1, 0, 1, 20000, 60000])), plan=plan)


@pytest.mark.parametrize("case", range(N_BATCH_CASES))
def test_random_batch(V, case):
    """A batch of 1..10 uneven members (ID or XY labels, one metric) with
    random per-member options, persistent grid shape, graphs on or off and
    solo members or not, over six random steps (JFA or dJFA, with or without
    moves); every member equals its oracle after every step."""
    c = draw_batch(case)
    print(f"[random-batch] case {case}: {c}", flush=True)
    sims, orcs = [], []
    for m in c["members"]:
        xy = inputs.place_seeds(m["W"], m["H"], m["S"], m["seed"])
        g = V.Sim(m["W"], m["H"], xy, disp_lo=m["lo"], disp_hi=m["hi"], metric=c["metric"],
                  vn_passes=m["vn"], extra_passes=m["extra"], dmax_override=m["dmax"],
                  sim_seed=m["seed"], label=m["label"])
        V.set_flood_variant(g.handle, m["variant"])
        V.set_tail_fusion(g.handle, m["fuse"])
        sims.append(g)
        orcs.append(O.Sim(m["W"], m["H"], xy, m["seed"], m["lo"], m["hi"], metric=c["metric"],
                          vn_passes=m["vn"], extra_passes=m["extra"],
                          dmax=m["dmax"] if m["dmax"] > 0 else None, label_mode=m["label"]))
    b = V.Batch(sims)
    b.set_shape(c["shape"])
    if c["solo"] >= 0:
        for mode in (V.STEP_JFA, V.STEP_DJFA):
            b.set_solo(mode, c["solo"])
    b.set_graph(c["graph"])
    for t, (mode, move) in enumerate(c["plan"]):
        b.step(mode, move)
        for o in orcs:
            if move:
                o.move()
            o.djfa_step() if mode == V.STEP_DJFA else o.jfa_step()
        for j, (g, o) in enumerate(zip(sims, orcs)):
            assert np.array_equal(g.read_seeds(), o.xy), f"case {case} t={t} member {j}"
            bad = int((g.read_map() != o.map).sum())
            assert bad == 0, f"case {case} t={t} member {j}: map differs on {bad} pixels"
    b.close()
    for g in sims:
        g.close()


N_SERVER_CASES = 12


@pytest.mark.parametrize("case", range(N_SERVER_CASES))
def test_random_server(V, case):
    """A server with 2..8 uneven simulations (random labels and pass
    options, one metric) takes 40 random requests in bursts, switching policy at random
    and draining at random points (every resident simulation is then read
    and compared); at the end every simulation equals its oracle run of the
    same request sequence."""
    r = np.random.default_rng(9000 + case)
    rl = np.random.default_rng(9500 + case)    # label encodings, drawn apart from the rest
    metric = int(r.integers(0, 2))
    sv = V.Server(8, 1 << 31, metric=metric)
    sv.set_policy(int(r.integers(0, 2)))
    sv.set_solo(int(rl.choice([0, 1 << 16, 1 << 40])))   # which simulations share pass levels
    ids, orcs = [], {}
    for j in range(int(r.integers(2, 9))):
        W = int(r.choice([1, 40, 256, 300, 1024, 1100]))
        H = int(r.choice([1, 9, 128, 333]))
        S = int(min(W * H, int(r.integers(1, 4000))))
        lo = int(r.integers(-3, 2))
        hi = int(r.integers(lo, 4))
        vn, extra = int(r.integers(0, 3)), int(r.integers(0, 3))
        seed = int(r.integers(1, 1 << 30))
        label = int(rl.integers(0, 2))
        xy = inputs.place_seeds(W, H, S, seed)
        i = sv.add_sim(W, H, xy, disp_lo=lo, disp_hi=hi, metric=metric, vn_passes=vn,
                       extra_passes=extra, sim_seed=seed, label=label)
        ids.append(i)
        orcs[i] = O.Sim(W, H, xy, seed, lo, hi, metric=metric, vn_passes=vn,
                        extra_passes=extra, label_mode=label)
    print(f"[random-server] case {case}: {len(ids)} sims, metric {metric}", flush=True)
    for n in range(40):
        if r.random() < 0.1:
            sv.set_policy(int(r.integers(0, 2)))
        i = int(r.choice(ids))
        mode = V.STEP_DJFA if r.random() < 0.7 else V.STEP_JFA
        sv.submit(i, mode)
        orcs[i].move()
        orcs[i].djfa_step() if mode == V.STEP_DJFA else orcs[i].jfa_step()
        if r.random() < 0.1 or n == 39:
            sv.drain(60000)
            for k in ids:
                bad = int((sv.read_map(k) != orcs[k].map).sum())
                assert bad == 0, f"case {case} request {n}: sim {k} differs on {bad} pixels"
    st = sv.stats()
    assert st["completed"] == st["submitted"] == 40
    sv.close()
