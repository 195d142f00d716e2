"""Degenerate inputs on the GPU: the smallest system (one atom, no neighbour:
zero force, so uniform straight-line motion with periodic wrap, a closed form),
one-atom replicas inside a batch, and a zero-step call.

Bars: the closed form to 1e-12 A in position and bit-exact velocities (no
force acts); the batch's other replicas bit-identical to the same replicas run
alone; md_step(0) changes nothing.
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
                chunk_steps=20)
    base.update(kw)
    return md.make_params(**base)


# one atom in a 16 A periodic box (3 cells of 5.33 A per edge): its nearest
# image is 16 A away, beyond r_c + skin
L1 = 16.0
X1 = np.array([[15.7, 0.2, 8.0]])
V1 = np.array([[0.05, -0.03, 0.011]])  # A/fs: a rebuild every 3 steps, 1 wrap in x and y

VARIANTS = [
    ("fp64", {}),
    ("mixed", {"precision": 1}),
    ("half", {"list_mode": 1}),
    ("persistent", {"launch_mode": 1}),
]


@pytest.mark.parametrize("name,kw", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_one_atom_moves_in_a_straight_line(md, tabs, oracle_lib, name, kw):
    steps = 130
    _say(f"[gpu] one atom variant={name} steps={steps}")
    box = np.full(3, L1)
    s = md.System(_params(md, **kw), tabs, [1], box[None, :])
    s.set_state(X1, V1)
    s.build_neighbors()
    cnt, _ = s.neighbors(8)
    assert int(cnt.cpu().numpy()[0]) == 0
    pe0, ke0 = s.energy()
    s.step(steps)
    x, v, f = (t.cpu().numpy() for t in s.get_state())
    st = s.stats()
    pe1, ke1 = s.energy()
    s.close()
    want = np.mod(X1 + steps * configs.DT * V1, L1)
    assert np.max(np.abs(x - want)) < 1e-12
    assert np.array_equal(v, V1)
    assert np.array_equal(f, np.zeros((1, 3)))
    assert st["steps"] == steps and st["rebuilds"] >= steps // 4
    ref = oracle_lib.forces_at(X1, box, tabs, RC, SKIN)
    # the embedding energy of an empty neighbourhood, F(0), and no pair term
    assert pe0[0] == pe1[0]
    assert abs(pe0[0] - ref["pe"]) <= 1e-12 * max(1.0, abs(ref["pe"]))
    ke = 0.5 * configs.MASS * float(np.sum(V1 ** 2)) / configs.FTM2V
    assert abs(ke0[0] - ke) <= 1e-14 * ke and ke1[0] == ke0[0]
    out = oracle_lib.md_run(X1, V1, box, tabs, steps, mass=configs.MASS, dt=configs.DT, r_cut=RC,
                            skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    assert np.max(np.abs(out["x"] - want)) < 1e-12


@pytest.mark.parametrize("kw", [{}, {"list_mode": 1}], ids=["full", "half"])
def test_one_atom_replicas_in_a_batch(md, tabs, kw):
    """Replicas of 1, 250 (ragged: 4 tiles minus 6), 1 and 128 atoms in one
    context: each equals the same replica run alone, bit for bit."""
    b250 = configs.small_box(5, seed=71, sigma_x=0.05, temperature=600.0)
    b250 = configs.Box(x=b250.x[:250], v=b250.v[:250], box=b250.box, n_cells=5,
                       temperature=600.0, site_ids=b250.site_ids[:250])
    b128 = configs.small_box(4, seed=72, sigma_x=0.05)
    b128 = configs.Box(x=b128.x[:128], v=b128.v[:128], box=np.full(3, 16.5), n_cells=4,
                       temperature=300.0, site_ids=b128.site_ids[:128])
    one_a = (X1, V1, np.full(3, L1))
    one_b = (X1[:, ::-1].copy(), -V1, np.full(3, 17.0))
    reps = [one_a, (b250.x, b250.v, b250.box), one_b, (b128.x, b128.v, b128.box)]
    steps = 60
    _say(f"[gpu] one-atom replicas in a batch kw={kw}")
    sizes = [r[0].shape[0] for r in reps]
    s = md.System(_params(md, **kw), tabs, sizes, np.stack([r[2] for r in reps]))
    s.set_state(np.concatenate([r[0] for r in reps]), np.concatenate([r[1] for r in reps]))
    s.build_neighbors()
    s.step(steps)
    xb, vb, fb = (t.cpu().numpy() for t in s.get_state())
    peb, keb = s.energy()
    s.close()
    off = 0
    for k, (x, v, bx) in enumerate(reps):
        n = x.shape[0]
        a = md.System(_params(md, **kw), tabs, [n], bx[None, :])
        a.set_state(x, v)
        a.build_neighbors()
        a.step(steps)
        xa, va, fa = (t.cpu().numpy() for t in a.get_state())
        pea, kea = a.energy()
        a.close()
        assert np.array_equal(xb[off:off + n], xa), k
        assert np.array_equal(vb[off:off + n], va), k
        assert np.array_equal(fb[off:off + n], fa), k
        assert peb[k] == pea[0] and keb[k] == kea[0], k
        off += n


def test_zero_steps_change_nothing(md, tabs):
    box = configs.small_box(6, seed=73, sigma_x=0.1, temperature=900.0)
    _say("[gpu] zero steps")
    s = md.System(_params(md), tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    s.step(7)
    before = [t.cpu().numpy() for t in s.get_state()]
    st0 = s.stats()
    assert s.step(0) == 0
    after = [t.cpu().numpy() for t in s.get_state()]
    st1 = s.stats()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)
    assert st0 == st1
    assert s.step(-1, check=False) == md.MD_E_ARG
    s.close()
