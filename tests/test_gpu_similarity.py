"""Similarity of the GPU diagrams (Sec. VI-A), reported per workload.

sim_bf: share of (sampled) pixels whose label's seed is at the exact nearest
distance, from the oracle's exact nearest-seed search (all pixels of the
small workload; 2^20 sampled pixels of the single and large workloads).
sim_jfa: share of pixels whose dJFA label equals the JFA label (the paper's
metric).  The same two figures are reported for dJFAm, a Manhattan-metric
dJFA twin on the same seed trajectory, against the Euclidean references.  The paper finds dJFAe agreeing with JFA on close to all pixels (Sec. VI-B);
the assertions hold the GPU to 99%.  The numbers are printed, and written
as JSON into the folder VD_RESULTS_DIR names when it is set.
"""
import json
import os

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


RESULTS = {}


@pytest.mark.parametrize("name,steps", [("small", 5), ("single", 4), ("large", 2)])
def test_similarity_per_workload(V, name, steps):
    wl = inputs.WORKLOADS[name]()
    spec = wl.sims[0]
    W, H = spec.width, spec.height
    xy = spec.positions()
    kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed)
    sj, sd = V.Sim(W, H, xy, **kw), V.Sim(W, H, xy, **kw)
    sm = V.Sim(W, H, xy, metric=V.MANHATTAN, **kw)      # dJFAm (Sec. V-C), same trajectory
    if wl.sample_pixels:
        px, py = inputs.sample_pixels(W, H, wl.sample_pixels, seed=7)
    else:
        yy, xx = np.mgrid[0:H, 0:W]
        px, py = xx.ravel().astype(np.int32), yy.ravel().astype(np.int32)
    rows = []
    for t in range(1, steps + 1):
        sj.move_seeds(), sd.move_seeds(), sm.move_seeds()
        sj.jfa_step(), sd.djfa_step(), sm.djfa_step()
        pos = sd.read_seeds()
        _, nd = O.nearest(pos, W, H, px, py)
        md, mj, mm = sd.read_map(), sj.read_map(), sm.read_map()
        bf_d = O.count_exact(md, pos, px, py, nd) / len(px)
        bf_j = O.count_exact(mj, pos, px, py, nd) / len(px)
        bf_m = O.count_exact(mm, pos, px, py, nd) / len(px)
        sim_jfa = O.count_equal(md, mj) / md.size
        sim_m = O.count_equal(mm, mj) / mm.size
        rows.append({"t": t, "djfa_vs_exact": bf_d, "jfa_vs_exact": bf_j, "djfa_vs_jfa": sim_jfa,
                     "djfam_vs_exact": bf_m, "djfam_vs_jfa": sim_m})
        print(f"[similarity] {name} t={t} dJFA vs exact {100 * bf_d:.4f}%  JFA vs exact "
              f"{100 * bf_j:.4f}%  dJFA vs JFA {100 * sim_jfa:.4f}%  dJFAm vs exact "
              f"{100 * bf_m:.4f}%  dJFAm vs JFA {100 * sim_m:.4f}%", flush=True)
        assert bf_d >= 0.99 and sim_jfa >= 0.99
        # dJFAm is reported, not held to a bound from the paper (which shows it
        # well below dJFAe); this only catches a broken diagram
        assert bf_m >= 0.5 and sim_m >= 0.5
    RESULTS[name] = {"workload": wl.name, "sampled_pixels": int(len(px)), "steps": rows}
    out = os.environ.get("VD_RESULTS_DIR")
    if out and os.path.isdir(out):
        with open(os.path.join(out, "similarity.json"), "w") as f:
            json.dump(RESULTS, f, indent=1)


def test_similarity_sweep_vn_extra(V):
    """Similarity to the exact diagram of JFA+e and of dJFA with v leading
    Von Neumann passes and e extra passes, v, e in {0, 1, 2} (small and
    single workloads, 3 steps).  Reported, and written to sweep.json in the
    folder VD_RESULTS_DIR names; each configuration is held to 99%."""
    out = {}
    for name, steps in (("small", 3), ("single", 3)):
        wl = inputs.WORKLOADS[name]()
        spec = wl.sims[0]
        W, H = spec.width, spec.height
        xy = spec.positions()
        kw = dict(disp_lo=spec.disp_lo, disp_hi=spec.disp_hi, sim_seed=spec.sim_seed)
        if wl.sample_pixels:
            px, py = inputs.sample_pixels(W, H, wl.sample_pixels, seed=7)
        else:
            yy, xx = np.mgrid[0:H, 0:W]
            px, py = xx.ravel().astype(np.int32), yy.ravel().astype(np.int32)
        rows = []
        for e in (0, 1, 2):
            sims = {("jfa", 0): V.Sim(W, H, xy, extra_passes=e, **kw)}
            for v in (0, 1, 2):
                sims[("djfa", v)] = V.Sim(W, H, xy, vn_passes=v, extra_passes=e, **kw)
            for _ in range(steps):
                for (kind, _v), sm in sims.items():
                    sm.move_seeds()
                    sm.djfa_step() if kind == "djfa" else sm.jfa_step()
            pos = sims[("jfa", 0)].read_seeds()
            _, nd = O.nearest(pos, W, H, px, py)
            for (kind, v), sm in sims.items():
                r = O.count_exact(sm.read_map(), pos, px, py, nd) / len(px)
                rows.append({"kind": kind, "vn_passes": v, "extra_passes": e, "vs_exact": r})
                print(f"[sweep] {name} {kind} vn={v} extra={e}: {100 * r:.4f}% exact", flush=True)
                assert r >= 0.99
                sm.close()
        out[name] = rows
    d = os.environ.get("VD_RESULTS_DIR")
    if d and os.path.isdir(d):
        with open(os.path.join(d, "sweep.json"), "w") as f:
            json.dump(out, f, indent=1)
