"""Pins of the oracle's multi-species EAM (Sec. II-A: rho_j, F_i and phi_ij depend
on the atom types) against closed forms and invariants, not against itself."""
import numpy as np
import pytest

from workloads import configs, potential as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")

RC, SKIN = P.RC, configs.SKIN


@pytest.fixture(scope="module")
def alloy_tabs():
    return P.alloy_tables()


@pytest.mark.parametrize("r", [2.3, 2.6])
@pytest.mark.parametrize("pair", [(0, 1), (1, 0), (1, 1)])
def test_binary_dimer_closed_form(oracle_lib, alloy_tabs, r, pair):
    """Energy phi_ab(r) + F_a(rho_b(r)) + F_b(rho_a(r)); force along the bond
    phi'_ab + F'_a(rho_b) rho'_b + F'_b(rho_a) rho'_a (each atom embeds the
    density the other one emits)."""
    a, b = pair
    x = np.array([[6.0, 6.0, 6.0], [6.0 + r, 6.0, 6.0]])
    box = np.array([20.0, 20.0, 20.0])
    res = oracle_lib.forces_at_multi(x, box, [a, b], alloy_tabs, RC, SKIN)
    e = P.alloy_phi(r, a, b) + P.alloy_emb(P.alloy_rho(r, b), a) + P.alloy_emb(P.alloy_rho(r, a), b)
    s = (P.alloy_dphi(r, a, b) + P.alloy_demb(P.alloy_rho(r, b), a) * P.alloy_drho(r, b)
         + P.alloy_demb(P.alloy_rho(r, a), b) * P.alloy_drho(r, a))
    # tolerance from the cubic-spline error bound of the F tables' slopes,
    # |F' - S'| <= h^3/24 max|F''''| (F'''' = (15/16) E_t rho^-7/2), times rho'
    h = alloy_tabs[2][0].dx
    bound = 1e-7
    for t, rho_src in ((a, b), (b, a)):
        rr = P.alloy_rho(r, rho_src) - h
        bound += h ** 3 / 24 * (15 / 16) * P.ALLOY_EMB_A[t] * rr ** -3.5 * abs(P.alloy_drho(r, rho_src))
    assert abs(res["pe"] - e) < 1e-6
    np.testing.assert_allclose(res["rho"], [P.alloy_rho(r, b), P.alloy_rho(r, a)], rtol=1e-7)
    np.testing.assert_allclose(res["f"][0], [s, 0, 0], atol=bound)
    np.testing.assert_allclose(res["f"][1], [-s, 0, 0], atol=bound)
    assert bound < 1e-4  # the bound itself stays tight


def test_alloy_forces_are_minus_gradient(oracle_lib, alloy_tabs):
    box = configs.alloy_box(4, 61, sigma_x=0.12)
    res = oracle_lib.forces_at_multi(box.x, box.box, box.types, alloy_tabs, RC, SKIN)
    assert np.all(np.abs(res["f"].sum(axis=0)) <= 1e-12 * np.abs(res["f"]).sum())
    rng = np.random.default_rng(62)
    h = 1e-4
    picks = np.concatenate([rng.choice(np.nonzero(box.types == 0)[0], 3),
                            rng.choice(np.nonzero(box.types == 1)[0], 3)])
    for i in picks:
        for d in range(3):
            xp, xm = box.x.copy(), box.x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            ep = oracle_lib.forces_at_multi(xp, box.box, box.types, alloy_tabs, RC, SKIN)["pe"]
            em = oracle_lib.forces_at_multi(xm, box.box, box.types, alloy_tabs, RC, SKIN)["pe"]
            assert abs(-(ep - em) / (2 * h) - res["f"][i, d]) < 1e-7


def test_one_species_in_two_types_is_the_single_species_model(oracle_lib, md_tables):
    """Two types carrying the same tables reproduce the (separately pinned)
    single-species oracle."""
    phi, rho, emb = md_tables
    tabs = ([[phi, phi], [phi, phi]], [rho, rho], [emb, emb])
    box = configs.alloy_box(5, 63, sigma_x=0.1)
    multi = oracle_lib.forces_at_multi(box.x, box.box, box.types, tabs, RC, SKIN)
    single = oracle_lib.forces_at(box.x, box.box, md_tables, RC, SKIN)
    assert np.array_equal(multi["rho"], single["rho"])
    assert np.array_equal(multi["fp"], single["fp"])
    np.testing.assert_allclose(multi["f"], single["f"], rtol=0, atol=1e-13)
    assert abs(multi["pe"] - single["pe"]) <= 1e-13 * abs(single["pe"])


def test_relabelling_the_types_changes_nothing(oracle_lib, alloy_tabs):
    phi, rho, emb = alloy_tabs
    swapped = ([[phi[1][1], phi[1][0]], [phi[0][1], phi[0][0]]], [rho[1], rho[0]], [emb[1], emb[0]])
    box = configs.alloy_box(5, 64, sigma_x=0.1)
    a = oracle_lib.forces_at_multi(box.x, box.box, box.types, alloy_tabs, RC, SKIN)
    b = oracle_lib.forces_at_multi(box.x, box.box, 1 - box.types, swapped, RC, SKIN)
    for k in ("f", "rho", "fp"):
        assert np.array_equal(a[k], b[k])
    assert a["pe"] == b["pe"]


def test_alloy_nve_second_order_and_momentum(oracle_lib, alloy_tabs):
    """Per-type masses: total energy is conserved to second order in dt and the
    mass-weighted momentum stays zero (a mass taken from the wrong atom breaks both)."""
    box = configs.alloy_box(5, 65, temperature=600.0)
    m = np.asarray(P.ALLOY_MASS)[box.types]
    assert np.all(np.abs((m[:, None] * box.v).sum(axis=0)) < 1e-12)
    errs, e0 = [], None
    for dt, steps in ((1.0, 200), (0.5, 400)):
        out = oracle_lib.md_run_multi(box.x, box.v, box.box, box.types, alloy_tabs, P.ALLOY_MASS,
                                      steps, dt=dt, r_cut=RC, skin=SKIN, ftm2v=configs.FTM2V,
                                      want_energy=True)
        assert out["code"] == 0
        e = out["energy"].sum(axis=1)
        e0 = e[0]
        errs.append(np.max(np.abs(e - e[0])))
        p = (m[:, None] * out["v"]).sum(axis=0)
        assert np.all(np.abs(p) < 1e-9)
    # the lattice collapses and heats by ~270 eV here; the energy error stays
    # below 1e-4 of the total and falls 4x when dt halves
    assert errs[0] < 1e-4 * abs(e0)
    assert 3.5 < errs[0] / errs[1] < 4.5


@pytest.fixture(scope="module")
def tabs3():
    return P.alloy_tables(n_types=3)


@pytest.mark.parametrize("pair", [(0, 2), (2, 1), (2, 2)])
def test_three_type_dimer_closed_form(oracle_lib, tabs3, pair):
    """A third type: energy and force of a dimer against the closed forms (the
    same bound as the binary dimers' tables)."""
    a, b = pair
    r = 2.5
    x = np.array([[6.0, 6.0, 6.0], [6.0 + r, 6.0, 6.0]])
    res = oracle_lib.forces_at_multi(x, np.full(3, 20.0), [a, b], tabs3, RC, SKIN)
    e = P.alloy_phi(r, a, b) + P.alloy_emb(P.alloy_rho(r, b), a) + P.alloy_emb(P.alloy_rho(r, a), b)
    s = (P.alloy_dphi(r, a, b) + P.alloy_demb(P.alloy_rho(r, b), a) * P.alloy_drho(r, b)
         + P.alloy_demb(P.alloy_rho(r, a), b) * P.alloy_drho(r, a))
    assert abs(res["pe"] - e) < 1e-6
    np.testing.assert_allclose(res["rho"], [P.alloy_rho(r, b), P.alloy_rho(r, a)], rtol=1e-7)
    np.testing.assert_allclose(res["f"][0], [s, 0, 0], atol=1e-4)
    np.testing.assert_allclose(res["f"][1], [-s, 0, 0], atol=1e-4)


def test_three_types_relabelled_by_a_cycle(oracle_lib, tabs3):
    """Relabelling the types by the cycle 0 -> 1 -> 2 -> 0, with the tables
    permuted to match, changes no bit."""
    phi, rho, emb = tabs3
    perm = [1, 2, 0]  # new label of old type t
    inv = [2, 0, 1]   # old type of new label u
    phi_p = [[phi[inv[u]][inv[v]] for v in range(3)] for u in range(3)]
    rho_p = [rho[inv[u]] for u in range(3)]
    emb_p = [emb[inv[u]] for u in range(3)]
    box = configs.multi_box(5, 66, P.MULTI_MASS[:3], sigma_x=0.1)
    a = oracle_lib.forces_at_multi(box.x, box.box, box.types, tabs3, RC, SKIN)
    b = oracle_lib.forces_at_multi(box.x, box.box, np.asarray(perm)[box.types], (phi_p, rho_p, emb_p),
                                   RC, SKIN)
    for k in ("f", "rho", "fp"):
        assert np.array_equal(a[k], b[k])
    assert a["pe"] == b["pe"]


def test_three_type_forces_are_minus_gradient(oracle_lib, tabs3):
    box = configs.multi_box(4, 67, P.MULTI_MASS[:3], sigma_x=0.12)
    res = oracle_lib.forces_at_multi(box.x, box.box, box.types, tabs3, RC, SKIN)
    h = 1e-4
    for t in range(3):
        i = int(np.nonzero(box.types == t)[0][0])
        for d in range(3):
            xp, xm = box.x.copy(), box.x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            ep = oracle_lib.forces_at_multi(xp, box.box, box.types, tabs3, RC, SKIN)["pe"]
            em = oracle_lib.forces_at_multi(xm, box.box, box.types, tabs3, RC, SKIN)["pe"]
            assert abs(-(ep - em) / (2 * h) - res["f"][i, d]) < 1e-7
