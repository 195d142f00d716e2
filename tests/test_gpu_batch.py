"""Batched replicas: each replica of a batch equals the same replica run alone
(bitwise, same schedule) and follows the oracle trajectory."""
import sys

import numpy as np
import pytest

from mixed_bound import pair_bounds
from workloads import configs, potential as P

pytestmark = pytest.mark.gpu
RC, SKIN = P.RC, configs.SKIN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _replicas(n_rep):
    reps = []
    for r in range(n_rep):
        rng = np.random.default_rng([40, r])
        n = int(rng.integers(5, 9))
        reps.append(configs.make_box(n, rng, vacancy_fraction=float(rng.uniform(0, 0.02)),
                                     temperature=float(rng.uniform(300, 2000))))
    return reps


def _params(md, lpa):
    return md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                          ftm2v=configs.FTM2V, chunk_steps=20, lanes_per_atom=lpa)


@pytest.mark.parametrize("lpa", [1, 4])
def test_batch_equals_alone_and_oracle(oracle_lib, lpa):
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    reps = _replicas(5)
    steps = 61
    _say(f"[gpu] batch of {len(reps)} replicas sizes {[b.n for b in reps]} lpa={lpa}")
    batch = md.System(_params(md, lpa), tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    batch.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    batch.build_neighbors()
    batch.step(steps)
    xb, vb, fb = (t.cpu().numpy() for t in batch.get_state())
    peb, keb = batch.energy()
    batch.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        alone = md.System(_params(md, lpa), tabs, [b.n], b.box[None, :])
        alone.set_state(b.x, b.v)
        alone.build_neighbors()
        alone.step(steps)
        xa, va, fa = (t.cpu().numpy() for t in alone.get_state())
        pea, kea = alone.energy()
        alone.close()
        sl = slice(off[r], off[r + 1])
        assert np.array_equal(xb[sl], xa) and np.array_equal(vb[sl], va)
        assert np.array_equal(fb[sl], fa)
        assert peb[r] == pea[0] and keb[r] == kea[0]
        out = oracle_lib.md_run(b.x, b.v, b.box, tabs, steps, mass=configs.MASS, dt=configs.DT,
                                r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
        d = xa - out["x"]
        d -= b.box * np.round(d / b.box)
        assert np.max(np.abs(d)) < 1e-9, (r, np.max(np.abs(d)))


@pytest.mark.parametrize("lpa", [1, 4])
def test_batch_mixed_equals_alone_and_within_float32_bound(oracle_lib, lpa):
    """Mixed precision in a batch: each replica's forces bitwise equal to the
    replica alone, and every rho_i and force of every replica within the
    float32 bound (mixed_bound.py) of the float64 oracle."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    reps = _replicas(5)
    _say(f"[gpu] mixed batch of {len(reps)} replicas sizes {[b.n for b in reps]} lpa={lpa}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       chunk_steps=20, lanes_per_atom=lpa, precision=md.MD_MIXED)
    batch = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    batch.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    batch.build_neighbors()
    fb, rb, _ = (t.cpu().numpy() for t in batch.compute_forces())
    batch.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        alone = md.System(p, tabs, [b.n], b.box[None, :])
        alone.set_state(b.x, b.v)
        alone.build_neighbors()
        fa, ra, _ = (t.cpu().numpy() for t in alone.compute_forces())
        alone.close()
        sl = slice(off[r], off[r + 1])
        assert np.array_equal(fb[sl], fa) and np.array_equal(rb[sl], ra), r
        ref = oracle_lib.forces_at(b.x, b.box, tabs, RC, SKIN)
        cnt, nbr, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, cap=128)
        rho_bound, f_bound = pair_bounds(b.x, b.box, ref["fp"], cnt, nbr)
        assert np.all(np.abs(rb[sl] - ref["rho"]) <= rho_bound), r
        err = np.linalg.norm(fb[sl] - ref["f"], axis=1)
        assert np.all(err <= f_bound), (r, float(np.max(err / f_bound)))


@pytest.mark.parametrize("prec", [0, 1], ids=["fp64", "mixed"])
def test_replica_schedule_equals_alone(oracle_lib, prec):
    """A per-replica schedule (each replica its own lanes per atom, one launch
    per pass): every replica bitwise equal to the same replica run alone with
    its value, over a 61-step run with rebuilds; float64 also follows the
    oracle trajectory."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    reps = _replicas(5)
    lanes = [1, 8, 2, 4, 8]
    steps = 61
    _say(f"[gpu] replica schedule {lanes} sizes {[b.n for b in reps]} precision={prec}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       chunk_steps=20, precision=prec)
    batch = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    batch.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    batch.build_neighbors()
    batch.set_replica_schedule(lanes)
    assert list(batch.replica_schedule()) == lanes
    batch.step(steps)
    xb, vb, fb = (t.cpu().numpy() for t in batch.get_state())
    batch.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        alone = md.System(p, tabs, [b.n], b.box[None, :])
        alone.set_state(b.x, b.v)
        alone.build_neighbors()
        alone.set_schedule(lanes[r])
        alone.step(steps)
        xa, va, fa = (t.cpu().numpy() for t in alone.get_state())
        alone.close()
        sl = slice(off[r], off[r + 1])
        assert np.array_equal(xb[sl], xa) and np.array_equal(vb[sl], va), r
        assert np.array_equal(fb[sl], fa), r
        if prec == 0:
            out = oracle_lib.md_run(b.x, b.v, b.box, tabs, steps, mass=configs.MASS,
                                    dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
            d = xa - out["x"]
            d -= b.box * np.round(d / b.box)
            assert np.max(np.abs(d)) < 1e-9, (r, np.max(np.abs(d)))


def test_autotune_per_size_class_keeps_the_trajectory(oracle_lib):
    """The autotuner's per-size-class search on replicas of 250 to 3,456
    atoms leaves a valid schedule (one value per size class) and the state it
    started from: the run after it follows the oracle."""
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    reps = []
    for r, n in enumerate([5, 12, 6, 9, 5, 12]):
        rng = np.random.default_rng([43, r])
        reps.append(configs.make_box(n, rng, temperature=float(rng.uniform(300, 1500))))
    _say(f"[gpu] autotune per size class, sizes {[b.n for b in reps]}")
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                       chunk_steps=20)
    s = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
    s.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
    s.build_neighbors()
    lpa, us = s.autotune(3)
    sched = s.replica_schedule()
    assert lpa in (1, 2, 4, 8) and us > 0
    assert set(sched.tolist()) <= {1, 2, 4, 8}
    cls = [0 if b.n <= 2048 else (1 if b.n <= 8192 else 2) for b in reps]
    for a in range(len(reps)):
        for b in range(len(reps)):
            if cls[a] == cls[b]:
                assert sched[a] == sched[b]
    s.step(41)
    x, _, _ = (t.cpu().numpy() for t in s.get_state())
    assert s.stats()["steps"] == 41
    s.close()
    off = np.concatenate([[0], np.cumsum([b.n for b in reps])])
    for r, b in enumerate(reps):
        out = oracle_lib.md_run(b.x, b.v, b.box, tabs, 41, mass=configs.MASS, dt=configs.DT,
                                r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V)
        d = x[off[r]:off[r + 1]] - out["x"]
        d -= b.box * np.round(d / b.box)
        assert np.max(np.abs(d)) < 1e-9, r
