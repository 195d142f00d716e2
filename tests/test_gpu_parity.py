"""GPU path vs the FP64 CPU oracle, element by element, through the C ABI.

Bars: cell ids and neighbour sets bit-exact; float64 forces within 1e-10
relative (max-norm over atoms, relative to the largest force); energies to
1e-12 relative; 100-step trajectories within 1e-9 A; bitwise repeatability.
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
def tabs():
    return P.md_tables()


def _params(md, **kw):
    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    base.update(kw)
    return md.make_params(**base)


def _system(md, tabs, box, **kw):
    s = md.System(_params(md, **kw), tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    return s


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


CASES = [
    ("c1_2000", lambda: configs.config_small()),
    ("ragged_6cells_vac", lambda: configs.small_box(6, seed=31, vacancy_fraction=0.03,
                                                   sigma_x=0.05, temperature=900.0)),
    ("min_3cells", lambda: configs.small_box(5, seed=32, sigma_x=0.2, temperature=300.0)),
    ("hot_12cells", lambda: configs.small_box(12, seed=33, sigma_x=0.25, temperature=2500.0)),
    ("ortho_5x6x7", lambda: configs.ortho_box(5, 6, 7, seed=36, sigma_x=0.1, temperature=900.0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lpa", [1, 4])
def test_cells_lists_forces(md, tabs, oracle_lib, name, make, lpa):
    box = make()
    _say(f"[gpu] cells/lists/forces case={name} n={box.n} lpa={lpa}")
    s = _system(md, tabs, box, lanes_per_atom=lpa)
    s.build_neighbors()
    cell_gpu = s.cells().cpu().numpy()
    cell_or, nc, _ = oracle_lib.cell_ids(box.x, box.box, RC + SKIN)
    assert np.array_equal(cell_gpu, cell_or)
    cnt_g, nbr_g = s.neighbors(128)
    cnt_g, nbr_g = cnt_g.cpu().numpy(), nbr_g.cpu().numpy()
    cnt_o, nbr_o, _ = oracle_lib.neighbor_list(box.x, box.box, RC + SKIN, cap=128)
    assert np.array_equal(cnt_g, cnt_o)
    assert oracle_lib.neighbor_sets(cnt_g, nbr_g) == oracle_lib.neighbor_sets(cnt_o, nbr_o)
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    pe, ke = s.energy()
    pe_o, ke_o = oracle_lib.energy(box.x, box.v, box.box, cnt_o, nbr_o, RC, *tabs, configs.MASS,
                                   configs.FTM2V)
    assert abs(pe[0] - pe_o) <= 1e-12 * abs(pe_o)
    assert abs(ke[0] - ke_o) <= 1e-12 * abs(ke_o) + 1e-300
    s.close()


def test_trajectory_100_steps_c1(md, tabs, oracle_lib):
    box = configs.config_small()
    _say(f"[gpu] trajectory c1 n={box.n} 100 steps")
    s = _system(md, tabs, box, chunk_steps=50)
    s.build_neighbors()
    s.step(100)
    x, v, f = s.get_state()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V, want_energy=True)
    d = x.cpu().numpy() - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11
    assert _rel(f.cpu().numpy(), out["f"]) < 1e-8
    pe, ke = s.energy()
    e_or = out["energy"][-1]
    assert abs(pe[0] - e_or[0]) < 1e-8 * abs(e_or[0])
    assert abs(ke[0] - e_or[1]) < 1e-8 * abs(e_or[1])
    st = s.stats()
    assert st["steps"] == 100
    s.close()


def test_hot_run_rebuilds_and_matches(md, tabs, oracle_lib):
    """Rebuilds inside the captured graph (odd remainder too) keep the oracle trajectory."""
    box = configs.small_box(8, seed=41, temperature=2000.0, sigma_x=0.05)
    _say(f"[gpu] hot run n={box.n} 61 steps")
    s = _system(md, tabs, box, chunk_steps=20)
    s.build_neighbors()
    s.step(61)
    x, v, f = s.get_state()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 61, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    d = x.cpu().numpy() - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    st = s.stats()
    assert st["rebuilds"] >= 2 and out["stats"]["rebuilds"] >= 2
    # after the run the GPU list equals the oracle list on the same positions
    fr = oracle_lib.forces_at(x.cpu().numpy(), box.box, tabs, RC, SKIN)
    assert _rel(f.cpu().numpy(), fr["f"]) < 1e-10
    s.close()


def test_orthorhombic_hot_run(md, tabs, oracle_lib):
    """Three different periodic edge lengths, hot enough to cross the faces and
    rebuild: the oracle trajectory."""
    box = configs.ortho_box(5, 6, 7, seed=37, sigma_x=0.05, temperature=3000.0)
    _say(f"[gpu] orthorhombic hot run n={box.n} box={box.box.tolist()}")
    s = _system(md, tabs, box, chunk_steps=20)
    s.build_neighbors()
    s.step(61)
    x, v, _ = s.get_state()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 61, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    d = x.cpu().numpy() - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-10
    assert st["rebuilds"] >= 2


def test_calls_between_steps_keep_the_trajectory(md, tabs, oracle_lib):
    """A hot box rebuilds every few steps; list builds, binning passes, the
    step's own kernels as timing passes, energy and force evaluations between
    short step calls (eager steps and graph chunks) leave the oracle trajectory
    unchanged, also when a rebuild is already due at the next step."""
    box = configs.small_box(8, seed=42, temperature=6000.0, sigma_x=0.05)
    _say(f"[gpu] calls between steps n={box.n}")
    s = _system(md, tabs, box, chunk_steps=20)
    s.build_neighbors()
    calls = [
        lambda: s.launch_pass(md.PASS_BUILD, 1),
        lambda: s.energy(),
        lambda: s.launch_pass(md.PASS_BIN, 2),
        lambda: s.compute_forces(),
        lambda: s.launch_pass(md.PASS_DENSITY, 2),
        lambda: s.launch_pass(md.PASS_FORCE, 1),
    ]
    total = 0
    for k in range(12):
        n = 20 if k % 4 == 3 else 3 + (k % 3)
        s.step(n)
        total += n
        calls[k % len(calls)]()
    x, v, f = s.get_state()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, total, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    d = x.cpu().numpy() - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-10
    # the list builds between calls reset the skin reference, so fewer fall due in md_step
    assert st["steps"] == total and st["rebuilds"] >= 8


def test_bitwise_repeatable(md, tabs):
    box = configs.small_box(10, seed=51, temperature=1500.0)
    _say(f"[gpu] determinism n={box.n}")
    res = []
    for _ in range(2):
        s = _system(md, tabs, box, chunk_steps=10)
        s.build_neighbors()
        s.step(40)
        x, v, f = s.get_state()
        res.append((x.cpu().numpy(), v.cpu().numpy(), f.cpu().numpy()))
        s.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_lanes_per_atom_agree(md, tabs):
    box = configs.small_box(8, seed=52, temperature=800.0, sigma_x=0.1)
    _say(f"[gpu] lanes-per-atom agreement n={box.n}")
    fs = []
    for lpa in (1, 2, 4, 8):
        s = _system(md, tabs, box, lanes_per_atom=lpa)
        s.build_neighbors()
        fs.append(s.compute_forces()[0].cpu().numpy())
        s.close()
    for f in fs[1:]:
        assert _rel(f, fs[0]) < 1e-13


def test_density_past_the_f_table(md, tabs, oracle_lib):
    """A compressed lattice (a = 2.2 A) puts every rho_i above the F table's
    end (40): F' comes from the end tangent on both sides, and the library
    reports the range warning."""
    box = configs.small_box(8, seed=55, a=2.2, sigma_x=0.02)
    _say(f"[gpu] density past the F table n={box.n}")
    s = _system(md, tabs, box)
    s.build_neighbors()
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN, cap=256)
    assert ref["rho"].min() > tabs[2].x1
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    assert s.stats()["status_bits"] & 256
    s.close()


def test_maximum_capacities(md, tabs, oracle_lib):
    """Both capacities at their documented maxima (nbr_capacity 1024,
    cell_capacity 256): a lattice compressed to a = 1.5 A holds up to ~140
    atoms per cell and ~340 list entries per atom, so a cell's ~3,500
    candidates are staged in 14 batches.  Cells and neighbour sets bit-exact, forces 1e-10,
    a short trajectory 1e-9 A."""
    box = configs.small_box(12, seed=56, a=1.5, sigma_x=0.01)
    _say(f"[gpu] maximum capacities n={box.n}")
    s = _system(md, tabs, box, nbr_capacity=1024, cell_capacity=256, chunk_steps=10)
    s.build_neighbors()
    st = s.stats()
    assert 64 < st["max_cell"] <= 256 and 300 < st["max_list"] <= 1024
    cell_gpu = s.cells().cpu().numpy()
    cell_o, _, _ = oracle_lib.cell_ids(box.x, box.box, RC + SKIN)
    assert np.array_equal(cell_gpu, cell_o)
    cnt_g, nbr_g = (t.cpu().numpy() for t in s.neighbors(1024))
    cnt_o, nbr_o, _ = oracle_lib.neighbor_list(box.x, box.box, RC + SKIN, cap=1024)
    assert np.array_equal(cnt_g, cnt_o)
    assert oracle_lib.neighbor_sets(cnt_g, nbr_g) == oracle_lib.neighbor_sets(cnt_o, nbr_o)
    f, _, _ = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN, cap=1024)
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    s.step(10)
    x, _, _ = s.get_state()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 10, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V, cap=1024)
    assert out["code"] == 0
    d = x.cpu().numpy() - out["x"]
    d -= box.box * np.round(d / box.box)
    assert np.max(np.abs(d)) < 1e-9


def test_error_paths(md, tabs):
    box = configs.small_box(6, seed=53)
    _say("[gpu] error paths")
    s = _system(md, tabs, box, nbr_capacity=8)
    with pytest.raises(md.MDError) as e:
        s.build_neighbors()
    assert e.value.code == md.MD_E_NBR_OVERFLOW
    s.close()
    s = _system(md, tabs, box)
    with pytest.raises(md.MDError) as e:
        s.step(1)
    assert e.value.code == md.MD_E_ORDER
    s.close()
    tiny = configs.small_box(3, seed=54)
    with pytest.raises(md.MDError) as e:
        md.System(_params(md), tabs, [tiny.n], tiny.box[None, :])
    assert e.value.code == md.MD_E_BOX
    s = _system(md, tabs, box, cell_capacity=4)
    with pytest.raises(md.MDError) as e:
        s.build_neighbors()
    assert e.value.code == md.MD_E_CELL_OVERFLOW
    s.close()
    # two coincident atoms: r = 0 gives a non-finite force (every table index
    # stays clamped to its table)
    x = box.x.copy()
    x[5] = x[4]
    s = md.System(_params(md), tabs, [box.n], box.box[None, :])
    s.set_state(x, box.v)
    with pytest.raises(md.MDError) as e:
        s.build_neighbors()
    assert e.value.code == md.MD_E_NONFINITE
    s.close()
