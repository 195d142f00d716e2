"""The half-list form (force symmetry, each pair evaluated once; two-phase
deterministic reduction) against the FP64 oracle and against the full-list
form, through the C ABI.

Bars as for the full list: rho_i and F' within 1e-12 relative, forces within
1e-10 relative (max-norm over atoms, relative to the largest force), energy
1e-12 relative, trajectories within 1e-9 A of the oracle's velocity-Verlet
run; bitwise repeatable; a batch of replicas equals each replica alone.
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
    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                list_mode=md.MD_LIST_HALF)
    base.update(kw)
    return md.make_params(**base)


def _system(md, tabs, box, **kw):
    s = md.System(_params(md, **kw), tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    return s


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _disp(a, b, box):
    d = a - b
    per = box > 0
    d[:, per] -= box[per] * np.round(d[:, per] / box[per])
    return d


CASES = [
    ("c1_2000", lambda: configs.config_small()),
    ("ragged_6cells_vac", lambda: configs.small_box(6, seed=31, vacancy_fraction=0.03,
                                                   sigma_x=0.05, temperature=900.0)),
    ("min_3cells", lambda: configs.small_box(5, seed=32, sigma_x=0.2, temperature=300.0)),
    ("hot_12cells", lambda: configs.small_box(12, seed=33, sigma_x=0.25, temperature=2500.0)),
    ("slab_open", lambda: configs.slab(7, 9, 6, seed=32, sigma_x=0.2, vacuum=6.0)),
    ("ortho_5x6x7", lambda: configs.ortho_box(5, 6, 7, seed=38, sigma_x=0.1, temperature=900.0)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_half_forces_match_oracle(md, tabs, oracle_lib, name, make):
    box = make()
    _say(f"[gpu] half list forces case={name} n={box.n}")
    s = _system(md, tabs, box)
    s.build_neighbors()
    f, rho, fp = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(fp.cpu().numpy(), ref["fp"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    pe, _ = s.energy()
    assert abs(pe[0] - ref["pe"]) <= 1e-12 * abs(ref["pe"])
    # the pair force on the j side is minus the one on the i side: the net
    # force vanishes up to the rounding of the per-atom sums
    fa = f.cpu().numpy()
    assert np.all(np.abs(fa.sum(axis=0)) <= 1e-12 * np.abs(fa).sum())
    s.close()


@pytest.mark.parametrize("name,make,steps,chunk", [
    ("c1_2000", lambda: configs.config_small(), 100, 50),
    ("hot_8cells", lambda: configs.small_box(8, seed=41, temperature=2000.0, sigma_x=0.05), 61, 20),
    ("slab_open", lambda: configs.slab(8, 8, 5, seed=31), 100, 50),
], ids=["c1_2000", "hot_8cells", "slab_open"])
def test_half_trajectory_matches_oracle(md, tabs, oracle_lib, name, make, steps, chunk):
    """Graph-captured steps, rebuilds (and the half-list re-derivation that
    follows each) inside the graph."""
    box = make()
    _say(f"[gpu] half list trajectory case={name} n={box.n} steps={steps}")
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
    if name == "hot_8cells":
        assert st["rebuilds"] >= 2


def test_half_equals_full_trajectory(md, tabs):
    box = configs.small_box(10, seed=51, temperature=1500.0)
    _say(f"[gpu] half vs full n={box.n}")
    out = []
    for mode in (md.MD_LIST_FULL, md.MD_LIST_HALF):
        s = _system(md, tabs, box, chunk_steps=10, list_mode=mode)
        s.build_neighbors()
        s.step(40)
        out.append([t.cpu().numpy() for t in s.get_state()])
        s.close()
    assert np.max(np.abs(_disp(out[0][0], out[1][0], box.box))) < 1e-9
    assert _rel(out[1][2], out[0][2]) < 1e-8


def test_half_bitwise_repeatable(md, tabs):
    """The reverse slots arrive in a varying order and are sorted: two runs
    give the same bits."""
    box = configs.small_box(8, seed=41, temperature=2000.0, sigma_x=0.05)
    _say(f"[gpu] half list determinism n={box.n}")
    res = []
    for _ in range(2):
        s = _system(md, tabs, box, chunk_steps=20)
        s.build_neighbors()
        s.step(61)
        res.append([t.cpu().numpy() for t in s.get_state()])
        assert s.stats()["rebuilds"] >= 2
        s.close()
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_half_batch_equals_alone(md, tabs):
    reps = []
    for r in range(4):
        rng = np.random.default_rng([42, r])
        n = int(rng.integers(5, 9))
        reps.append(configs.make_box(n, rng, vacancy_fraction=float(rng.uniform(0, 0.02)),
                                     temperature=float(rng.uniform(300, 2000))))
    _say(f"[gpu] half list batch sizes {[b.n for b in reps]}")
    p = _params(md, chunk_steps=20)
    batch = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    batch.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    batch.build_neighbors()
    batch.step(41)
    xb, vb, fb = (t.cpu().numpy() for t in batch.get_state())
    batch.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        alone = md.System(p, tabs, [b.n], b.box[None, :])
        alone.set_state(b.x, b.v)
        alone.build_neighbors()
        alone.step(41)
        xa, va, fa = (t.cpu().numpy() for t in alone.get_state())
        alone.close()
        sl = slice(off[r], off[r + 1])
        assert np.array_equal(xb[sl], xa) and np.array_equal(vb[sl], va)
        assert np.array_equal(fb[sl], fa)


def test_half_full_size_128k(md, tabs, oracle_lib):
    """The 128,000-atom box: forces at the start, then 100 graph steps, against
    the oracle."""
    box = configs.config_128k()
    _say(f"[gpu] half list full size n={box.n}")
    s = _system(md, tabs, box, chunk_steps=100, nbr_capacity=128, cell_capacity=64, sort_every=2)
    s.build_neighbors()
    f, rho, _ = s.compute_forces()
    ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
    assert _rel(rho.cpu().numpy(), ref["rho"]) < 1e-12
    assert _rel(f.cpu().numpy(), ref["f"]) < 1e-10
    s.step(100)
    x, v, _ = s.get_state()
    s.close()
    out = oracle_lib.md_run(box.x, box.v, box.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                            r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
    assert np.max(np.abs(_disp(x.cpu().numpy(), out["x"], box.box))) < 1e-9
    assert np.max(np.abs(v.cpu().numpy() - out["v"])) < 1e-11


def test_half_overflow_is_reported(md, tabs):
    box = configs.small_box(6, seed=53)
    s = _system(md, tabs, box, nbr_capacity=8)
    with pytest.raises(md.MDError) as e:
        s.build_neighbors()
    assert e.value.code == md.MD_E_NBR_OVERFLOW
    s.close()
