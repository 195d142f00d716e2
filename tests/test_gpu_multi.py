"""Several atom types (Sec. II-A: rho_j, F_i, phi_ij per type) on the GPU
against the oracle's multi-species functions, through the C ABI.

Bars as for one species: rho_i and F' within 1e-12 relative, forces within
1e-10 relative (max-norm over atoms, relative to the largest force), energy
1e-12 relative; trajectories within 1e-9 A (positions) and 1e-11 A/fs
(velocities) of the oracle's velocity-Verlet run with per-type masses.
"""
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
def atabs():
    return P.alloy_tables()


def _system(md, tabs, box, masses=P.ALLOY_MASS, **kw):
    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                n_types=2)
    base.update(kw)
    s = md.System(md.make_params(**base), tabs, [box.n], box.box[None, :], masses=masses)
    s.set_state(box.x, box.v)
    s.set_types(box.types)
    return s


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _disp(a, b, box):
    d = a - b
    per = box > 0
    d[:, per] -= box[per] * np.round(d[:, per] / box[per])
    return d


def _alloy_slab():
    """A thin slab (open in x and y) whose sites are type 1 with probability 1/2."""
    b = configs.slab(6, 7, 5, seed=77, sigma_x=0.05, vacuum=6.0)
    b.types = (np.random.default_rng(78).random(b.n) < 0.5).astype(np.int32)
    return b


CASES = [
    ("alloy_6cells", lambda: configs.alloy_box(6, 71)),
    ("alloy_slab_open_xy", _alloy_slab),
    ("alloy_hot_8cells", lambda: configs.alloy_box(8, 72, sigma_x=0.2, temperature=2000.0)),
    ("dilute_5cells", lambda: configs.alloy_box(5, 73, frac_1=0.1)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lpa", [1, 4])
def test_multi_forces_match_oracle(md, atabs, oracle_lib, name, make, lpa):
    box = make()
    _say(f"[gpu] multi-species forces case={name} n={box.n} lpa={lpa}")
    s = _system(md, atabs, box, lanes_per_atom=lpa)
    s.build_neighbors()
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at_multi(box.x, box.box, box.types, atabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    pe, _ = s.energy()
    assert abs(pe[0] - ref["pe"]) <= 1e-12 * abs(ref["pe"])
    s.close()


@pytest.mark.parametrize("name,make,steps,chunk,sort_every", [
    ("alloy_6cells", lambda: configs.alloy_box(6, 71), 100, 50, 1),
    ("alloy_hot_8cells", lambda: configs.alloy_box(8, 72, sigma_x=0.05, temperature=2000.0), 61,
     10, 1),
], ids=["alloy_6cells", "alloy_hot_8cells"])
def test_multi_trajectory_matches_oracle(md, atabs, oracle_lib, name, make, steps, chunk,
                                         sort_every):
    """Graph-captured steps with rebuilds and re-sorts (the types move with
    their atoms) and per-type masses in the update."""
    box = make()
    _say(f"[gpu] multi-species trajectory case={name} n={box.n} steps={steps}")
    s = _system(md, atabs, box, chunk_steps=chunk, sort_every=sort_every)
    s.build_neighbors()
    s.step(steps)
    x, v, f = s.get_state()
    pe, ke = s.energy()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run_multi(box.x, box.v, box.box, box.types, atabs, P.ALLOY_MASS, steps,
                                  dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                                  want_energy=True)
    assert out["code"] == 0
    assert np.max(np.abs(_disp(x.cpu().numpy(), out["x"], box.box))) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11
    assert _rel(f.cpu().numpy(), out["f"]) < 1e-8
    e_or = out["energy"][-1]
    assert abs(pe[0] - e_or[0]) < 1e-8 * abs(e_or[0])
    assert abs(ke[0] - e_or[1]) < 1e-8 * abs(e_or[1])
    assert st["steps"] == steps
    if name == "alloy_hot_8cells":
        assert st["rebuilds"] >= 2


def test_types_set_before_or_after_the_state(md, atabs, oracle_lib):
    box = configs.alloy_box(5, 74)
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       n_types=2)
    out = []
    for order in ("types_first", "state_first"):
        s = md.System(p, atabs, [box.n], box.box[None, :], masses=P.ALLOY_MASS)
        if order == "types_first":
            s.set_types(box.types)
            s.set_state(box.x, box.v)
        else:
            s.set_state(box.x, box.v)
            s.build_neighbors()  # slots sorted by cell: types go through the slot map
            s.set_types(box.types)
        s.build_neighbors()
        out.append(s.compute_forces()[0].cpu().numpy())
        s.close()
    assert np.array_equal(out[0], out[1])
    ref = oracle_lib.forces_at_multi(box.x, box.box, box.types, atabs, RC, SKIN)
    assert _rel(out[0], ref["f"]) < 1e-10


def test_bad_types_and_tables_are_rejected(md, atabs):
    box = configs.alloy_box(5, 75)
    s = _system(md, atabs, box)
    bad = box.types.copy()
    bad[7] = 2
    with pytest.raises(md.MDError) as e:
        s.set_types(bad)
    assert e.value.code == md.MD_E_ARG
    s.close()
    phi, rho, emb = atabs
    asym = ([[phi[0][0], phi[0][1]], [phi[1][1], phi[1][1]]], rho, emb)
    with pytest.raises(md.MDError) as e:
        _system(md, asym, box)
    assert e.value.code == md.MD_E_TABLE


def test_two_types_with_one_species_tables_match_one_species(md, md_tables):
    """Both types carrying the same tables and mass: the one-species path's forces."""
    box = configs.alloy_box(6, 76, sigma_x=0.1)
    phi, rho, emb = md_tables
    s = _system(md, ([[phi, phi], [phi, phi]], [rho, rho], [emb, emb]), box,
                masses=(configs.MASS, configs.MASS))
    s.build_neighbors()
    fm = s.compute_forces()[0].cpu().numpy()
    s.step(20)
    xm = s.get_state()[0].cpu().numpy()
    s.close()
    p1 = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    s1 = md.System(p1, md_tables, [box.n], box.box[None, :])
    s1.set_state(box.x, box.v)
    s1.build_neighbors()
    f1 = s1.compute_forces()[0].cpu().numpy()
    s1.step(20)
    x1 = s1.get_state()[0].cpu().numpy()
    s1.close()
    assert _rel(fm, f1) < 1e-13
    assert np.max(np.abs(_disp(xm, x1, box.box))) < 1e-11


def test_multi_batch_equals_alone(md, atabs):
    reps = [configs.alloy_box(n, 80 + n, temperature=900.0) for n in (5, 6, 7)]
    _say(f"[gpu] multi-species batch sizes {[b.n for b in reps]}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       n_types=2, chunk_steps=20)
    batch = md.System(p, atabs, [b.n for b in reps], np.stack([b.box for b in reps]),
                      masses=P.ALLOY_MASS)
    batch.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    batch.set_types(np.concatenate([b.types for b in reps]))
    batch.build_neighbors()
    batch.step(41)
    xb, vb, _ = (t.cpu().numpy() for t in batch.get_state())
    batch.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        alone = md.System(p, atabs, [b.n], b.box[None, :], masses=P.ALLOY_MASS)
        alone.set_state(b.x, b.v)
        alone.set_types(b.types)
        alone.build_neighbors()
        alone.step(41)
        xa, va, _ = (t.cpu().numpy() for t in alone.get_state())
        alone.close()
        sl = slice(off[r], off[r + 1])
        assert np.array_equal(xb[sl], xa) and np.array_equal(vb[sl], va)


def test_multi_full_size_128k(md, atabs, oracle_lib):
    """The 128,000-atom binary alloy in the benchmark's launch configuration:
    forces, then 100 graph steps, against the oracle."""
    box = configs.config_alloy_128k()
    _say(f"[gpu] multi-species full size n={box.n}")
    s = _system(md, atabs, box, chunk_steps=100, nbr_capacity=128, cell_capacity=64, sort_every=2)
    s.build_neighbors()
    s.autotune(5)
    f, rho, _ = s.compute_forces()
    ref = oracle_lib.forces_at_multi(box.x, box.box, box.types, atabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    s.step(100)
    x, v, _ = s.get_state()
    s.close()
    out = oracle_lib.md_run_multi(box.x, box.v, box.box, box.types, atabs, P.ALLOY_MASS, 100,
                                  dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    assert np.max(np.abs(_disp(x.cpu().numpy(), out["x"], box.box))) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11


@pytest.mark.parametrize("nt", [3, 4])
@pytest.mark.parametrize("lpa", [1, 4])
def test_three_and_four_types(md, oracle_lib, nt, lpa):
    """More than two types: the pair-table rows (one per unordered type pair),
    density rows that no longer fit the LDS (read from global memory), and
    force rows mostly outside the LDS window.  rho, F', forces and energy
    against the oracle, then a hot 41-step trajectory with rebuilds."""
    tabs = P.alloy_tables(n_types=nt)
    masses = P.MULTI_MASS[:nt]
    box = configs.multi_box(6, 80 + nt, masses, sigma_x=0.1, temperature=1500.0)
    assert set(np.unique(box.types).tolist()) == set(range(nt))
    _say(f"[gpu] {nt} types n={box.n} lpa={lpa}")
    s = _system(md, tabs, box, masses=masses, n_types=nt, lanes_per_atom=lpa, chunk_steps=20)
    s.build_neighbors()
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at_multi(box.x, box.box, box.types, tabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    pe, _ = s.energy()
    assert abs(pe[0] - ref["pe"]) <= 1e-12 * abs(ref["pe"])
    s.step(41)
    x, v, _ = s.get_state()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run_multi(box.x, box.v, box.box, box.types, tabs, masses, 41,
                                  dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    assert np.max(np.abs(_disp(x.cpu().numpy(), out["x"], box.box))) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11
    assert st["rebuilds"] >= 1
