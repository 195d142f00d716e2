"""Mixed-precision form (float32 pair terms, compensated float32 sums, float64
state) against the float64 oracle on identical positions, within the error
bound derived term by term in mixed_bound.py (float32 separation, r^2, rsqrt,
segment and Horner cubic; their effect on each term is its size plus r times
its slope)."""
import sys

import numpy as np
import pytest

from mixed_bound import pair_bounds
from workloads import configs, potential as P

pytestmark = pytest.mark.gpu
RC, SKIN = P.RC, configs.SKIN
U = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


MIXED_CASES = [
    ("box_6cells_300K", lambda: configs.small_box(6, seed=61, temperature=300.0, sigma_x=0.02)),
    ("box_8cells_2500K", lambda: configs.small_box(8, seed=62, temperature=2500.0,
                                                   sigma_x=0.02 * np.sqrt(2500.0 / 300))),
    ("slab_open_xy", lambda: configs.slab(7, 7, 5, seed=63, sigma_x=0.05, vacuum=6.0)),
    ("ortho_5x6x7", lambda: configs.ortho_box(5, 6, 7, seed=64, sigma_x=0.05)),
]


@pytest.mark.parametrize("name,make", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_forces_within_float32_bound(oracle_lib, name, make):
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    box = make()
    _say(f"[gpu] mixed precision case={name} n={box.n}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       precision=md.MD_MIXED)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    f, rho, fp = (t.cpu().numpy() for t in s.compute_forces())
    s.close()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    cnt, nbr, _ = oracle_lib.neighbor_list(box.x, box.box, RC + SKIN, cap=128)
    rho_bound, f_bound = pair_bounds(box.x, box.box, ref["fp"], cnt, nbr)
    assert np.all(np.abs(rho - ref["rho"]) <= rho_bound), np.max(np.abs(rho - ref["rho"]) / rho_bound)
    err = np.linalg.norm(f - ref["f"], axis=1)
    assert np.all(err <= f_bound), np.max(err / f_bound)
    # and it is not accidentally the float64 path: errors are of float32 size
    assert np.max(err) > 1e-12


def _forces_vs_oracle(oracle_lib, tabs, s, box):
    """The form's forces at its own current state against the oracle's at the
    exported positions, within the float32 bound."""
    x, _, _ = s.get_state(want_f=False)
    f, rho, _ = (t.cpu().numpy() for t in s.compute_forces())
    x = x.cpu().numpy()
    ref = oracle_lib.forces_at(x, box.box, tabs, RC, SKIN)
    cnt, nbr, _ = oracle_lib.neighbor_list(x, box.box, RC + SKIN, cap=128)
    rho_bound, f_bound = pair_bounds(x, box.box, ref["fp"], cnt, nbr)
    assert np.all(np.abs(rho - ref["rho"]) <= rho_bound), np.max(np.abs(rho - ref["rho"]) / rho_bound)
    err = np.linalg.norm(f - ref["f"], axis=1)
    assert np.all(err <= f_bound), np.max(err / f_bound)
    assert np.max(err) > 1e-12


@pytest.mark.parametrize("launch", ["graph", "persistent"])
def test_mixed_records_follow_the_trajectory(oracle_lib, launch):
    """The mixed form's 16-byte records (fixed-point position and F') are
    rewritten by every kernel that moves atoms: after 73 steps of a hot box
    (list rebuilds, a re-sort by cell before every chunk, the odd position
    buffer current at the end) the forces at the state reached are within the
    float32 bound of the oracle's at the exported positions."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    box = configs.small_box(7, seed=91, temperature=2500.0, sigma_x=0.05)
    _say(f"[gpu] mixed records along a trajectory ({launch}), n={box.n}")
    mode = md.MD_LAUNCH_GRAPH if launch == "graph" else md.MD_LAUNCH_PERSISTENT
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       precision=md.MD_MIXED, chunk_steps=20, sort_every=1, launch_mode=mode)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    s.step(73)
    st = s.stats()
    assert st["steps"] == 73 and st["rebuilds"] >= 3, st
    _forces_vs_oracle(oracle_lib, tabs, s, box)
    s.close()


def test_mixed_records_after_a_rollback(oracle_lib):
    """A binning overflow at a re-sort (the configuration of the float64
    rollback test) in the mixed form: the state rolls back to the last
    snapshot, records included, and the forces there are within the float32
    bound of the oracle's at the returned positions."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    box = configs.small_box(9, seed=72, temperature=4000.0, sigma_x=0.05)
    skin = 2.0
    _say(f"[gpu] mixed rollback, n={box.n}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=skin, ftm2v=configs.FTM2V,
                       precision=md.MD_MIXED, chunk_steps=10, sort_every=1, cell_capacity=29,
                       nbr_capacity=256)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    rc = s.step(100, check=False)
    assert rc == md.MD_E_CELL_OVERFLOW, rc
    st = s.stats()
    assert st["steps"] in (10, 20, 30), st
    x, _, _ = s.get_state(want_f=False)
    f, rho, _ = (t.cpu().numpy() for t in s.compute_forces())
    s.close()
    x = x.cpu().numpy()
    ref = oracle_lib.forces_at(x, box.box, tabs, RC, skin)
    cnt, nbr, _ = oracle_lib.neighbor_list(x, box.box, RC + skin, cap=256)
    rho_bound, f_bound = pair_bounds(x, box.box, ref["fp"], cnt, nbr)
    assert np.all(np.abs(rho - ref["rho"]) <= rho_bound)
    err = np.linalg.norm(f - ref["f"], axis=1)
    assert np.all(err <= f_bound), np.max(err / f_bound)
