"""Mixed-precision form (float32 pair terms, compensated float32 sums, float64
state) against the float64 oracle on identical positions.

Bound: each pair term carries a relative error of at most about 16 u
(u = 2^-24: rounding of the separation, r^2, the hardware rsqrt, the
spline segment and the products), and the TwoSum accumulation adds
O(n u^2).  The pair force f_ij = (F'_i + F'_j) rho'(r) + phi'(r) is a sum of
an embedding and a pair term that cancel in part (exactly so in the
lattice-sum sense at zero pressure), and each carries its error relative to
its own size, so |dF_i| <= 16 u sum_j (|(F'_i + F'_j) rho'(r_ij)| + |phi'(r_ij)|)
and |d rho_i| <= 16 u rho_i.  The sums are computed here by numpy from the
analytic potential (a bound on the tabulated one within 1e-6)."""
import sys

import numpy as np
import pytest

from workloads import configs, potential as P

pytestmark = pytest.mark.gpu
RC, SKIN = P.RC, configs.SKIN
U = 2.0 ** -24


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair_force_sums(x, box, fp):
    d = x[None, :, :] - x[:, None, :]
    per = box > 0  # minimum image along periodic dimensions only
    d[..., per] -= box[per] * np.round(d[..., per] / box[per])
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    m = r < RC
    rr = np.where(m, r, 1.0)
    s = np.where(m, np.abs((fp[:, None] + fp[None, :]) * P.drho(rr)) + np.abs(P.dphi(rr)), 0.0)
    return s.sum(1) * 1.000001


MIXED_CASES = [
    ("box_6cells_300K", lambda: configs.small_box(6, seed=61, temperature=300.0, sigma_x=0.02)),
    ("box_8cells_2500K", lambda: configs.small_box(8, seed=62, temperature=2500.0,
                                                   sigma_x=0.02 * np.sqrt(2500.0 / 300))),
    ("slab_open_xy", lambda: configs.slab(7, 7, 5, seed=63, sigma_x=0.05, vacuum=6.0)),
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
    assert np.all(np.abs(rho - ref["rho"]) <= 16 * U * ref["rho"] + 1e-12)
    bound = 16 * U * _pair_force_sums(box.x, box.box, ref["fp"])
    err = np.linalg.norm(f - ref["f"], axis=1)
    assert np.all(err <= bound), np.max(err / bound)
    # and it is not accidentally the float64 path: errors are of float32 size
    assert np.max(err) > 1e-12
