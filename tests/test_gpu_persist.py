"""The persistent launch (one cooperative kernel per chunk, grid barriers
between phases) runs the same device code as the graph path: trajectories,
forces, counters and error handling must be bitwise those of the graph.

Systems whose atom tiles fit one thread slot each on the workgroups of one XCD
run the small-system kernel (state in registers, slot barriers on one L2);
the cases named all_xcds_* are too large for it (8,192 atoms at 8 lanes per
atom: 128 tiles for at most 32 workgroups) and run the kernel that spreads
its workgroups over every XCD."""
import sys

import numpy as np
import pytest

from workloads import configs, potential as P

pytestmark = pytest.mark.gpu

RC, SKIN = P.RC, configs.SKIN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def md():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_07898_amd import md as mdmod

    mdmod.lib()
    return mdmod


@pytest.fixture(scope="module")
def tabs():
    return P.md_tables()


def _run(md, tabs, boxes, steps, mode, check=True, **kw):
    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                launch_mode=mode)
    base.update(kw)
    s = md.System(md.make_params(**base), tabs, [b.n for b in boxes],
                  np.stack([b.box for b in boxes]))
    s.set_state(np.concatenate([b.x for b in boxes]), np.concatenate([b.v for b in boxes]))
    s.build_neighbors()
    rc = s.step(steps, check=check)
    x, v, f = (t.cpu().numpy() for t in s.get_state())
    pe, ke = s.energy()
    st = s.stats()
    s.close()
    return rc, x, v, f, pe, ke, st


CASES = [
    ("c1_2000", lambda: [configs.config_small()], 100, dict(chunk_steps=50)),
    ("hot_8cells_rebuilds", lambda: [configs.small_box(8, seed=41, temperature=2000.0,
                                                       sigma_x=0.05)], 60, dict(chunk_steps=20)),
    ("lpa1", lambda: [configs.small_box(7, seed=42, temperature=900.0)], 40,
     dict(chunk_steps=20, lanes_per_atom=1)),
    ("mixed", lambda: [configs.small_box(8, seed=43, temperature=1200.0)], 40,
     dict(chunk_steps=20, precision=1)),
    ("replicas", lambda: [configs.small_box(n, seed=44 + n, temperature=1500.0) for n in (5, 6, 7)],
     60, dict(chunk_steps=20)),
    ("slab_open", lambda: [configs.slab(8, 8, 5, seed=31)], 60, dict(chunk_steps=20)),
    ("resort_every_chunk", lambda: [configs.small_box(8, seed=45, temperature=2500.0)], 80,
     dict(chunk_steps=20, sort_every=1)),
    ("all_xcds_8192", lambda: [configs.small_box(16, seed=47, temperature=2500.0)], 60,
     dict(chunk_steps=20, lanes_per_atom=8)),
    ("all_xcds_mixed", lambda: [configs.small_box(16, seed=48, temperature=2500.0)], 40,
     dict(chunk_steps=20, lanes_per_atom=8, precision=1)),
]


@pytest.mark.parametrize("name,make,steps,kw", CASES, ids=[c[0] for c in CASES])
def test_persistent_equals_graph(md, tabs, name, make, steps, kw):
    boxes = make()
    _say(f"[gpu] persistent vs graph case={name} n={sum(b.n for b in boxes)} steps={steps}")
    g = _run(md, tabs, boxes, steps, md.MD_LAUNCH_GRAPH, **kw)
    p = _run(md, tabs, boxes, steps, md.MD_LAUNCH_PERSISTENT, **kw)
    for a, b in zip(g[1:4], p[1:4]):
        assert np.array_equal(a, b)
    assert np.array_equal(g[4], p[4]) and np.array_equal(g[5], p[5])
    for key in ("steps", "rebuilds", "list_entries", "max_list", "max_cell", "status_bits"):
        assert g[6][key] == p[6][key], key
    assert p[6]["steps"] == steps


def test_persistent_matches_oracle(md, tabs, oracle_lib):
    box = configs.config_small()
    _say(f"[gpu] persistent vs oracle n={box.n}")
    _, x, v, f, _, _, _ = _run(md, tabs, [box], 100, md.MD_LAUNCH_PERSISTENT, chunk_steps=50)
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    d = x - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v - out["v"])) < 1e-11


# list capacities just above each box's initial longest list (29 and 31 entries)
@pytest.mark.parametrize("cells,lpa,cap", [(8, 0, 30), (16, 8, 32)], ids=["small_kernel", "all_xcds"])
def test_persistent_overflow_rolls_back_like_the_graph(md, tabs, cells, lpa, cap):
    """A list overflow in a rebuild inside the chunk stops every workgroup at
    the same barrier; the chunk rolls back to its snapshot, as in the graph."""
    box = configs.small_box(cells, seed=46, temperature=2500.0, sigma_x=0.05)
    _say(f"[gpu] persistent overflow n={box.n} lpa={lpa}")
    g = _run(md, tabs, [box], 60, md.MD_LAUNCH_GRAPH, check=False, chunk_steps=20,
             nbr_capacity=cap, lanes_per_atom=lpa)
    p = _run(md, tabs, [box], 60, md.MD_LAUNCH_PERSISTENT, check=False, chunk_steps=20,
             nbr_capacity=cap, lanes_per_atom=lpa)
    assert g[0] == md.MD_E_NBR_OVERFLOW and p[0] == md.MD_E_NBR_OVERFLOW
    for a, b in zip(g[1:3], p[1:3]):
        assert np.array_equal(a, b)
    assert g[6]["steps"] == p[6]["steps"]
