"""Parity at the benchmark's full sizes, in the benchmark's launch configuration.

The 128,000-atom and 802,344-atom periodic boxes and the 801,792-atom slab
(open in x and y) are built with the same parameters as
bench.py (hipGraph chunks of 100 steps, list capacity 128, cell capacity 64,
lanes per atom from the autotuner).  Against the FP64 oracle:
- cell ids, list lengths and neighbour sets of every atom: bit-exact (each
  atom's set compared as its sorted row);
- rho_i, F'(rho_i): 1e-12 relative; forces: 1e-10 relative (max-norm over
  atoms, relative to the largest force); potential energy: 1e-12 relative;
- after 100 graph-captured steps: positions within 1e-9 A, velocities within
  1e-11 A/fs of the oracle's velocity-Verlet run.
"""
import sys

import numpy as np
import pytest

import bench
from mixed_bound import pair_bounds
from workloads import configs, potential as P

pytestmark = pytest.mark.gpu

RC, SKIN = P.RC, configs.SKIN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _sorted_rows(nbr, cnt):
    """Each atom's neighbour set as its sorted row (unused slots last)."""
    valid = np.arange(nbr.shape[1])[None, :] < cnt[:, None]
    return np.sort(np.where(valid, nbr, np.iinfo(np.int32).max), axis=1)


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


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


SIZES = [("128k", configs.config_128k), ("810k", configs.config_810k),
         ("slab_801792", configs.config_slab_801792)]


@pytest.mark.parametrize("name,make", SIZES, ids=[s[0] for s in SIZES])
def test_full_size_cells_lists_forces(md, tabs, oracle_lib, name, make):
    box = make()
    _say(f"[gpu] full size {name}: n={box.n} cells/lists/forces")
    s = bench.make_system(md, box, tabs, precision=md.MD_FP64, chunk=100)
    lpa, _ = s.autotune(5)
    _say(f"[gpu]   lanes per atom {lpa}")
    cell_g = s.cells().cpu().numpy()
    cell_o, _, _ = oracle_lib.cell_ids(box.x, box.box, RC + SKIN)
    assert np.array_equal(cell_g, cell_o)
    cnt_g, nbr_g = s.neighbors(128)
    cnt_g, nbr_g = cnt_g.cpu().numpy(), nbr_g.cpu().numpy()
    cnt_o, nbr_o, _ = oracle_lib.neighbor_list(box.x, box.box, RC + SKIN, cap=128)
    assert np.array_equal(cnt_g, cnt_o)
    assert np.array_equal(_sorted_rows(nbr_g, cnt_g), _sorted_rows(nbr_o, cnt_o))
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    pe, _ = s.energy()
    assert abs(pe[0] - ref["pe"]) <= 1e-12 * abs(ref["pe"])
    s.close()


@pytest.mark.parametrize("name,make", SIZES, ids=[s[0] for s in SIZES])
def test_full_size_trajectory_100_steps(md, tabs, oracle_lib, name, make):
    box = make()
    _say(f"[gpu] full size {name}: n={box.n} 100 graph steps")
    s = bench.make_system(md, box, tabs, precision=md.MD_FP64, chunk=100)
    s.autotune(5)
    s.step(100)
    x, v, _ = s.get_state()
    st = s.stats()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    d = x.cpu().numpy() - out["x"]
    per = box.box > 0  # minimum image along periodic dimensions only
    d[:, per] -= box.box[per] * np.round(d[:, per] / box.box[per])
    assert np.max(np.abs(d)) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11
    assert st["steps"] == 100


def test_full_size_mixed_810k_within_float32_bound(md, tabs, oracle_lib):
    """The mixed form at 802,344 atoms, launched as the benchmark launches it:
    every rho_i and force within the float32 bound (mixed_bound.py) of the
    float64 oracle."""
    box = configs.config_810k()
    _say(f"[gpu] full size mixed: n={box.n}")
    s = bench.make_system(md, box, tabs, precision=md.MD_MIXED, chunk=100)
    s.autotune(5)
    f, rho, _ = (t.cpu().numpy() for t in s.compute_forces())
    s.close()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    cnt, nbr, _ = oracle_lib.neighbor_list(box.x, box.box, RC + SKIN, cap=128)
    rho_bound, f_bound = pair_bounds(box.x, box.box, ref["fp"], cnt, nbr)
    assert np.all(np.abs(rho - ref["rho"]) <= rho_bound)
    err = np.linalg.norm(f - ref["f"], axis=1)
    assert np.all(err <= f_bound), float(np.max(err / f_bound))
    assert np.max(err) > 1e-12  # float32 arithmetic, not the float64 path


def test_full_batch_256_replicas_sampled(md, tabs, oracle_lib):
    """All 256 replicas (1.5 M atoms) in one context, launched as the benchmark
    launches them (100-step graph chunk, autotuned lanes per atom); 8 replicas,
    drawn with a fixed seed, follow the oracle's own runs."""
    reps = configs.config_batch(256)
    _say(f"[gpu] full batch: {len(reps)} replicas, n={sum(b.n for b in reps)}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       chunk_steps=100, nbr_capacity=128, cell_capacity=64)
    s = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    s.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    s.build_neighbors()
    s.autotune(5)
    s.step(100)
    x, v, _ = (t.cpu().numpy() for t in s.get_state())
    assert s.stats()["steps"] == 100
    s.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r in np.sort(np.random.default_rng(11).choice(len(reps), 8, replace=False)):
        b = reps[r]
        out = oracle_lib.md_run(b.x, b.v, b.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                                r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
        assert out["code"] == 0
        d = x[off[r]:off[r + 1]] - out["x"]
        d -= b.box * np.round(d / b.box)
        assert np.max(np.abs(d)) < 1e-9, r
        assert np.max(np.abs(v[off[r]:off[r + 1]] - out["v"])) < 1e-11, r


def test_full_batch_256_replicas_mixed_within_float32_bound(md, tabs, oracle_lib):
    """The mixed form of all 256 replicas in one context, launched as the
    benchmark launches it (autotuned lanes per atom): for 8 replicas drawn with
    a fixed seed, every rho_i and force within the float32 bound
    (mixed_bound.py) of the float64 oracle on the same positions."""
    reps = configs.config_batch(256)
    _say(f"[gpu] full batch mixed: {len(reps)} replicas, n={sum(b.n for b in reps)}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       precision=md.MD_MIXED, chunk_steps=100, nbr_capacity=128,
                       cell_capacity=64)
    s = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    s.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    s.build_neighbors()
    lpa, _ = s.autotune(5)
    _say(f"[gpu]   lanes per atom {lpa}")
    f, rho, _ = (t.cpu().numpy() for t in s.compute_forces())
    s.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r in np.sort(np.random.default_rng(12).choice(len(reps), 8, replace=False)):
        b = reps[r]
        ref = oracle_lib.forces_at(b.x, b.box, tabs, RC, SKIN)
        cnt, nbr, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, cap=128)
        rho_bound, f_bound = pair_bounds(b.x, b.box, ref["fp"], cnt, nbr)
        sl = slice(off[r], off[r + 1])
        assert np.all(np.abs(rho[sl] - ref["rho"]) <= rho_bound), r
        err = np.linalg.norm(f[sl] - ref["f"], axis=1)
        assert np.all(err <= f_bound), (r, float(np.max(err / f_bound)))
        assert np.max(err) > 1e-12  # float32 arithmetic, not the float64 path
