"""Open boundaries on the GPU vs the FP64 oracle: thin slabs with free lateral
surfaces, periodic through the thickness (the geometry of the paper's
benchmarks, Sec. IV-B), and boxes open in every dimension.

A negative box length marks an open dimension (no wrap, no image; its
magnitude is the extent of the cell grid).  Same bars as the periodic parity
tests: cell ids and neighbour sets bit-exact; forces 1e-10 relative; energy
1e-12 relative; 100-step trajectories within 1e-9 A.
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


def _system(md, tabs, box, **kw):
    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    base.update(kw)
    s = md.System(md.make_params(**base), tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    return s


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _disp(a, b, box):
    """a - b with the minimum image along periodic dimensions only."""
    d = a - b
    per = box > 0
    d[:, per] -= box[per] * np.round(d[:, per] / box[per])
    return d


def _strays():
    """A slab flush with the low x and y grid edges (face atoms below 0) plus two
    isolated atoms outside the grid, one on each side: they bin into edge cells."""
    b = configs.slab(6, 5, 5, seed=34, vacuum=0.0, sigma_x=0.05)
    extra = np.array([[-20.0, -20.0, 1.0], [-b.box[0] + 15.0, 3.0, 9.0]])
    x = np.vstack([b.x, extra])
    rng = np.random.default_rng(35)
    v = np.vstack([b.v, 1e-3 * rng.standard_normal((2, 3))])
    return configs.Box(x=x, v=v, box=b.box, n_cells=b.n_cells, temperature=b.temperature,
                       site_ids=np.arange(x.shape[0], dtype=np.int64))


def _dimer():
    x = np.array([[1.0, 1.0, 1.0], [3.6, 1.0, 1.0]])
    return configs.Box(x=x, v=np.zeros_like(x), box=-np.array([6.0, 3.0, 3.0]), n_cells=1,
                       temperature=0.0, site_ids=np.arange(2, dtype=np.int64))


CASES = [
    ("slab_8x8x5", lambda: configs.slab(8, 8, 5, seed=31)),
    ("slab_rough", lambda: configs.slab(7, 9, 6, seed=32, sigma_x=0.2, vacuum=6.0,
                                        temperature=900.0)),
    ("film_1cell", lambda: configs.slab(1, 6, 5, seed=33, vacuum=0.5)),
    ("strays", _strays),
    ("dimer_all_open", _dimer),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("lpa", [1, 4])
def test_open_cells_lists_forces(md, tabs, oracle_lib, name, make, lpa):
    box = make()
    _say(f"[gpu] open box case={name} n={box.n} box={box.box.tolist()} lpa={lpa}")
    s = _system(md, tabs, box, lanes_per_atom=lpa)
    s.build_neighbors()
    cell_g = s.cells().cpu().numpy()
    cell_o, _, _ = oracle_lib.cell_ids(box.x, box.box, RC + SKIN)
    assert np.array_equal(cell_g, cell_o)
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
    pe, _ = s.energy()
    assert abs(pe[0] - ref["pe"]) <= 1e-12 * abs(ref["pe"])
    # positions along open dimensions come back as given, periodic ones wrapped
    x, _, _ = s.get_state()
    assert np.array_equal(x.cpu().numpy()[:, box.box < 0], box.x[:, box.box < 0])
    s.close()


@pytest.mark.parametrize("name,make,steps,chunk", [
    ("slab_8x8x5", lambda: configs.slab(8, 8, 5, seed=31), 100, 50),
    ("strays_hot", lambda: _strays(), 61, 20),
], ids=["slab_8x8x5", "strays_hot"])
def test_open_trajectory(md, tabs, oracle_lib, name, make, steps, chunk):
    box = make()
    if name == "strays_hot":
        box.v[:] *= np.sqrt(2000.0 / 300.0)
    _say(f"[gpu] open box trajectory case={name} n={box.n} steps={steps}")
    s = _system(md, tabs, box, chunk_steps=chunk)
    s.build_neighbors()
    s.step(steps)
    x, v, f = s.get_state()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, steps, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    assert np.max(np.abs(_disp(x.cpu().numpy(), out["x"], box.box))) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11
    assert _rel(f.cpu().numpy(), out["f"]) < 1e-8
    assert st["steps"] == steps
    if name == "strays_hot":
        assert st["rebuilds"] >= 1 and out["stats"]["rebuilds"] >= 1


def test_open_dimer_closed_form(md, tabs):
    """All dimensions open: the dimer's force is the closed form with no image,
    in a box shorter than twice the list radius (one cell per dimension)."""
    box = _dimer()
    s = _system(md, tabs, box)
    s.build_neighbors()
    f, _, _ = s.compute_forces()
    s.close()
    r = 2.6
    g = P.dphi(r) + 2 * P.demb(P.rho(r)) * P.drho(r)
    np.testing.assert_allclose(f.cpu().numpy(), [[g, 0, 0], [-g, 0, 0]], atol=1e-6)


def test_periodic_edge_still_rejected(md, tabs):
    """A periodic edge below twice the list radius is still an error when the
    other dimensions are open."""
    box = _dimer()
    bad = box.box.copy()
    bad[2] = 6.0
    with pytest.raises(Exception):
        md.System(md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                                 ftm2v=configs.FTM2V), tabs, [box.n], bad[None, :])


def test_open_cluster_trajectory_and_momenta(md, tabs, oracle_lib):
    """A rotating cluster in a box open in every dimension: the oracle's
    trajectory, and linear and angular momentum kept to rounding."""
    x = configs.bcc_block(3, 3, 3) + 10.0
    rng = np.random.default_rng(91)
    x = x + 0.02 * rng.standard_normal(x.shape)
    v = configs.maxwell_boltzmann(rng, x.shape[0], 100.0)
    c = x.mean(axis=0)
    v = v + np.cross(np.array([0.3, -0.5, 1.0]) * 0.002, x - c)
    box = configs.Box(x=x, v=v, box=-np.full(3, 40.0), n_cells=3, temperature=100.0,
                      site_ids=np.arange(x.shape[0], dtype=np.int64))
    _say(f"[gpu] open cluster n={box.n}")
    s = _system(md, tabs, box, chunk_steps=100)
    s.build_neighbors()
    s.step(400)
    xg, vg, _ = (t.cpu().numpy() for t in s.get_state())
    s.close()
    out = oracle_lib.md_run(x, v, box.box, tabs, 400, mass=configs.MASS, dt=configs.DT, r_cut=RC,
                            skin=SKIN, ftm2v=configs.FTM2V)
    assert np.max(np.abs(xg - out["x"])) < 1e-9
    assert np.max(np.abs(vg - out["v"])) < 1e-11

    def ang(xx, vv):
        return configs.MASS * np.cross(xx - xx.mean(axis=0), vv).sum(axis=0)

    l0 = ang(x, v)
    assert np.max(np.abs(ang(xg, vg) - l0)) < 1e-9 * np.linalg.norm(l0)
    assert np.max(np.abs(vg.sum(axis=0) - v.sum(axis=0))) < 1e-12 * np.abs(v).sum()
