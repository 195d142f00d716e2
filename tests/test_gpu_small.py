"""Small systems (a few thousand atoms) on the graph path: binning, list build
and density pass of a step run in one kernel, and the autotuner times that
kernel.  Timing the schedules must leave the state as it was, and the run
after it must be bitwise the run of a fresh context given the same schedules;
both follow the FP64 oracle (1e-9 A)."""
import sys

import numpy as np
import pytest

from workloads import configs, potential as P

pytestmark = pytest.mark.gpu

RC, SKIN = P.RC, configs.SKIN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _system(md, tabs, box, lpa):
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                       ftm2v=configs.FTM2V, chunk_steps=50, lanes_per_atom=lpa)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    return s


def test_autotune_on_a_small_box_keeps_state_and_trajectory(oracle_lib):
    """The exported on-step velocity is the stored half-step one plus half a
    kick from forces recomputed with the current lanes per atom, so the state
    is compared under the schedule it was exported with (4), and the fresh
    context starts under that schedule too (its first half-kick)."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    box = configs.small_box(10, seed=71, temperature=1500.0, sigma_x=0.03)
    _say(f"[gpu] small-box autotune n={box.n}")
    s = _system(md, tabs, box, 4)
    x0, v0, _ = (t.cpu().numpy() for t in s.get_state())
    lpa, us = s.autotune(5)
    assert lpa in (1, 2, 4, 8) and us > 0
    s.set_schedule(4)
    x1, v1, _ = (t.cpu().numpy() for t in s.get_state())
    assert np.array_equal(x0, x1) and np.array_equal(v0, v1)
    s.set_schedule(lpa)
    s.step(120)
    xa, va, _ = (t.cpu().numpy() for t in s.get_state())
    sa = s.stats()
    s.close()
    t = _system(md, tabs, box, 4)
    t.set_schedule(lpa)
    t.step(120)
    xb, vb, _ = (u.cpu().numpy() for u in t.get_state())
    sb = t.stats()
    t.close()
    assert np.array_equal(xa, xb) and np.array_equal(va, vb)
    assert sa["rebuilds"] == sb["rebuilds"] and sa["steps"] == sb["steps"] == 120
    assert sa["rebuilds"] > 0
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 120, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    d = xa - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(va - out["v"])) < 1e-11
