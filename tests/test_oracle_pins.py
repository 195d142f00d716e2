"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms
on lattices, dimers and trimers, brute force, finite differences of the
energy, a reduction to a pair potential, and the integrator's stated
properties (Sec. II-A: second order, momentum conserving, time reversible).
"""
import numpy as np
import pytest

from workloads import configs, potential as P

RC, SKIN = 5.0, 0.3
A = configs.A_LAT


def bcc_shell_distances(a, rc):
    out = []
    for i in range(-3, 4):
        for j in range(-3, 4):
            for k in range(-3, 4):
                for b in (0.0, 0.5):
                    v = np.array([i + b, j + b, k + b]) * a
                    r = float(np.sqrt(v @ v))
                    if 0.0 < r < rc:
                        out.append(r)
    return np.array(out)


# ----------------------------------------------------------------- tables

def test_spline_tables_match_analytic(oracle_lib, md_tables):
    """Natural cubic 2000-knot tables reproduce the analytic functions (value and slope)."""
    phi_t, rho_t, emb_t = md_tables
    r = np.linspace(1.5, 4.999, 20001)
    for tab, f, df in ((phi_t, P.phi, P.dphi), (rho_t, P.rho, P.drho)):
        v, d, _ = oracle_lib.spline_eval(tab, r)
        # cubic-spline interpolation bounds (Hall and Meyer, 1976):
        # |s - f| <= 5/384 h^4 max|f''''|, |s' - f'| <= 1/24 h^3 max|f''''|
        q = 1e-3
        rr = np.linspace(1.5 - 2 * q, 5.0 - 2 * q, 7001)
        f4 = np.max(np.abs(f(rr - 2 * q) - 4 * f(rr - q) + 6 * f(rr) - 4 * f(rr + q)
                           + f(rr + 2 * q))) / q ** 4
        h = tab.dx
        assert np.max(np.abs(v - f(r))) < 5.0 / 384.0 * h ** 4 * f4 * 1.01
        assert np.max(np.abs(d - df(r))) < h ** 3 * f4 / 24.0 * 1.01
    p = np.linspace(0.5, 39.99, 20001)
    v, d, dd = oracle_lib.spline_eval(emb_t, p)
    # Two error sources.  Interior: the Hall-Meyer bounds with max|F''''| on
    # [0.5, 40] (value, slope) or [1, 40] (curvature, 3/8 h^2 max|F''''|).  End:
    # the natural condition sets s'' = 0 at rho = 40 where F'' = M; that moment
    # defect, spread over the last interval, moves s by at most M h^2 (t^3 - t)/6
    # (max 0.065 M h^2), s' by M h / 3 and s'' by M.
    h = emb_t.dx
    m_end = abs(float(P.ddemb(emb_t.x1)))
    f4 = lambda lo: 15.0 / 16.0 * P.EMB_A * lo ** -3.5  # F = -A sqrt(rho): |F''''| largest at lo
    assert np.max(np.abs(v - P.emb(p))) < 0.065 * m_end * h ** 2 + 5.0 / 384.0 * h ** 4 * f4(0.5)
    assert np.max(np.abs(d - P.demb(p))) < m_end * h / 3.0 + h ** 3 * f4(0.5) / 24.0
    assert np.max(np.abs(dd - P.ddemb(p))[p > 1.0]) < m_end + 3.0 / 8.0 * h ** 2 * f4(1.0)


def test_table_continues_along_end_tangent(oracle_lib, md_tables):
    """Past the last knot a table is the straight line tangent at that knot:
    value and slope continuous at the end, slope constant and curvature zero
    beyond (the reading for densities above the F table, e.g. a compressed
    cluster at rho > 40)."""
    _, _, emb_t = md_tables
    end = emb_t.x1
    e = 1e-7
    v0, d0, _ = oracle_lib.spline_eval(emb_t, np.array([end - e, end]))
    assert abs(v0[1] - v0[0] - d0[1] * e) < 1e-12 and abs(d0[1] - d0[0]) < 1e-9
    x = end + np.array([0.5, 3.0, 17.0, 260.0])
    v, d, dd = oracle_lib.spline_eval(emb_t, x)
    assert np.all(d == d0[1]) and np.all(dd == 0.0)
    np.testing.assert_allclose(v, v0[1] + d0[1] * (x - end), rtol=1e-14, atol=1e-12)


def test_spline_knots_interpolate(oracle_lib, md_tables):
    """At the knots the tables return the sampled analytic values to rounding."""
    phi_t, _, _ = md_tables
    k = np.arange(300, 1999, 97)
    r = k * phi_t.dx
    v, _, _ = oracle_lib.spline_eval(phi_t, r)
    np.testing.assert_allclose(v, P.phi(r), rtol=1e-12, atol=1e-14)


# ----------------------------------------------------------------- lattice closed form

def test_perfect_lattice_energy_density_forces(oracle_lib, md_tables):
    """Perfect BCC: rho_i, E/atom equal the closed-form shell sums; all forces vanish."""
    n = 10
    x = configs.bcc_sites(n)
    box = np.full(3, n * A)
    shells = bcc_shell_distances(A, RC)
    assert shells.size == 26
    rho_lat = P.rho(shells).sum()
    e_lat = 0.5 * P.phi(shells).sum() + P.emb(rho_lat)
    res = oracle_lib.forces_at(x, box, md_tables, RC, SKIN)
    assert np.max(np.abs(res["rho"] - rho_lat)) < 1e-9
    assert abs(res["pe"] / x.shape[0] - e_lat) < 1e-9
    np.testing.assert_allclose(res["fp"], P.demb(rho_lat), atol=1e-6)
    assert np.max(np.linalg.norm(res["f"], axis=1)) < 1e-12


def test_net_force_zero(oracle_lib, md_tables):
    b = configs.small_box(6, seed=11, sigma_x=0.1)
    res = oracle_lib.forces_at(b.x, b.box, md_tables, RC, SKIN)
    net = np.abs(res["f"].sum(axis=0))
    assert np.all(net <= 1e-12 * np.abs(res["f"]).sum())


# ----------------------------------------------------------------- F = -grad U

def test_forces_are_negative_energy_gradient(oracle_lib, md_tables):
    b = configs.small_box(6, seed=12, sigma_x=0.05)
    res = oracle_lib.forces_at(b.x, b.box, md_tables, RC, SKIN)
    rng = np.random.default_rng(0)
    h = 1e-4
    for _ in range(12):
        i, d = int(rng.integers(b.n)), int(rng.integers(3))
        xp, xm = b.x.copy(), b.x.copy()
        xp[i, d] += h
        xm[i, d] -= h
        ep = oracle_lib.forces_at(xp, b.box, md_tables, RC, SKIN)["pe"]
        em = oracle_lib.forces_at(xm, b.box, md_tables, RC, SKIN)["pe"]
        fd = -(ep - em) / (2 * h)
        assert abs(fd - res["f"][i, d]) < 1e-7, (i, d, fd, res["f"][i, d])


# ----------------------------------------------------------------- neighbour lists

@pytest.mark.parametrize("ncell,seed,sigma", [(6, 1, 0.01), (10, 2, 0.2), (4, 3, 0.3)])
def test_cell_list_equals_brute_force(oracle_lib, ncell, seed, sigma):
    b = configs.small_box(ncell, seed=seed, sigma_x=sigma)
    c1, n1, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method="cells")
    c2, n2, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method="brute")
    assert np.array_equal(c1, c2)
    assert oracle_lib.neighbor_sets(c1, n1) == oracle_lib.neighbor_sets(c2, n2)


def test_lattice_list_length_is_26(oracle_lib):
    x = configs.bcc_sites(6)
    cnt, _, _ = oracle_lib.neighbor_list(x, np.full(3, 6 * A), RC + SKIN)
    assert np.all(cnt == 26)


def test_neighbor_list_brute_pairs_by_numpy(oracle_lib):
    """Brute-force list against an independent numpy all-pairs minimum-image distance."""
    b = configs.small_box(4, seed=5, sigma_x=0.3)
    cnt, nbr, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method="brute")
    d = b.x[None, :, :] - b.x[:, None, :]
    d -= b.box * np.round(d / b.box)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    want = [frozenset(np.nonzero(r[i] < RC + SKIN - 1e-9)[0].tolist()) for i in range(b.n)]
    got = oracle_lib.neighbor_sets(cnt, nbr)
    near = np.abs(r - (RC + SKIN)) < 1e-9
    assert not near.any()
    assert got == want


@pytest.mark.parametrize("method", ["cells", "brute"])
def test_orthorhombic_lists_by_numpy(oracle_lib, method):
    """Three different periodic edge lengths: both list builders against numpy
    all-pairs distances under the minimum image of each dimension."""
    b = configs.ortho_box(5, 6, 7, seed=6, sigma_x=0.3)
    assert len(set(b.box.tolist())) == 3
    cnt, nbr, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method=method)
    d = b.x[None, :, :] - b.x[:, None, :]
    d -= b.box * np.round(d / b.box)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    assert not (np.abs(r - (RC + SKIN)) < 1e-9).any()
    want = [frozenset(np.nonzero(r[i] < RC + SKIN)[0].tolist()) for i in range(b.n)]
    assert oracle_lib.neighbor_sets(cnt, nbr) == want


def test_orthorhombic_forces_are_negative_energy_gradient(oracle_lib, md_tables):
    """Central differences of the energy for atoms next to each periodic face."""
    b = configs.ortho_box(5, 6, 7, seed=7, sigma_x=0.1)
    res = oracle_lib.forces_at(b.x, b.box, md_tables, RC, SKIN)
    h = 1e-5
    picks = [int(np.argmin(b.x[:, d])) for d in range(3)] + \
            [int(np.argmax(b.x[:, d])) for d in range(3)]
    for i in picks:
        for d in range(3):
            xp, xm = b.x.copy(), b.x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            ep = oracle_lib.forces_at(xp, b.box, md_tables, RC, SKIN)["pe"]
            em = oracle_lib.forces_at(xm, b.box, md_tables, RC, SKIN)["pe"]
            assert abs(-(ep - em) / (2 * h) - res["f"][i, d]) < 1e-5


def test_cell_assignment_properties(oracle_lib):
    b = configs.small_box(10, seed=7, sigma_x=0.3)
    cell, nc, ic = oracle_lib.cell_ids(b.x, b.box, RC + SKIN)
    assert list(nc) == [6, 6, 6]
    cx = cell % nc[0]
    cy = (cell // nc[0]) % nc[1]
    cz = cell // (nc[0] * nc[1])
    w = b.box / nc
    for c, k in ((cx, 0), (cy, 1), (cz, 2)):
        assert np.all(b.x[:, k] >= c * w[k] - 1e-12)
        assert np.all(b.x[:, k] <= (c + 1) * w[k] + 1e-12)
    start, order = oracle_lib.cell_sort(cell, int(np.prod(nc)))
    assert start[-1] == b.n and np.all(np.diff(start) >= 0)
    assert sorted(order.tolist()) == list(range(b.n))
    for q in range(int(np.prod(nc))):
        seg = order[start[q]:start[q + 1]]
        assert np.all(cell[seg] == q) and np.all(np.diff(seg) > 0)


def test_wrap_rule(oracle_lib):
    box = np.array([10.0, 10.0, 10.0])
    x = np.array([[10.0, -1e-18, 3.0], [-2.5, 12.0, 9.999999999999998]])
    w, bad = oracle_lib.wrap(x, box)
    assert bad == 0
    assert w[0, 0] == 0.0 and w[0, 1] == 0.0 and w[0, 2] == 3.0
    assert w[1, 0] == 7.5 and w[1, 1] == 2.0
    assert np.all((w >= 0) & (w < box))


# ----------------------------------------------------------------- many-body closed forms

def _isolated(points, L=20.0):
    x = np.asarray(points, dtype=np.float64) + L / 2
    return x, np.full(3, L)


# rho(r) >= 0.5 here: the F table interpolates a sqrt, poorly resolved near rho = 0
@pytest.mark.parametrize("r", [2.3, 2.6, 2.86, 2.95])
def test_dimer(oracle_lib, md_tables, r):
    x, box = _isolated([[0, 0, 0], [r, 0, 0]])
    res = oracle_lib.forces_at(x, box, md_tables, RC, SKIN)
    e = P.phi(r) + 2 * P.emb(P.rho(r))
    s = P.dphi(r) + 2 * P.demb(P.rho(r)) * P.drho(r)
    assert abs(res["pe"] - e) < 1e-6
    # F' table error near small rho (dx = 0.02 on a sqrt) is ~4e-6 relative
    np.testing.assert_allclose(res["f"][0], [s, 0, 0], rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(res["f"][1], [-s, 0, 0], rtol=2e-5, atol=1e-7)


def test_equilateral_trimer(oracle_lib, md_tables):
    r = 2.9
    pts = np.array([[0, 0, 0], [r, 0, 0], [r / 2, r * np.sqrt(3) / 2, 0]])
    x, box = _isolated(pts)
    res = oracle_lib.forces_at(x, box, md_tables, RC, SKIN)
    rho_i = 2 * P.rho(r)
    assert abs(res["pe"] - (3 * P.phi(r) + 3 * P.emb(rho_i))) < 1e-6
    s = P.dphi(r) + 2 * P.demb(rho_i) * P.drho(r)
    centroid = pts.mean(0)
    for i in range(3):
        u = (centroid - pts[i]) / np.linalg.norm(centroid - pts[i])
        np.testing.assert_allclose(res["f"][i], np.sqrt(3) * s * u, atol=1e-5)


def test_linear_trimer(oracle_lib, md_tables):
    r = 2.7
    pts = np.array([[-r, 0, 0], [0, 0, 0], [r, 0, 0]])
    x, box = _isolated(pts)
    res = oracle_lib.forces_at(x, box, md_tables, RC, SKIN)
    re, rm = P.rho(r) + P.rho(2 * r), 2 * P.rho(r)
    e = 2 * P.phi(r) + P.phi(2 * r) + 2 * P.emb(re) + P.emb(rm)
    assert abs(res["pe"] - e) < 1e-6
    assert np.allclose(res["f"][1], 0.0, atol=1e-12)
    s1 = P.dphi(r) + (P.demb(re) + P.demb(rm)) * P.drho(r)
    s2 = P.dphi(2 * r) + 2 * P.demb(re) * P.drho(2 * r)
    np.testing.assert_allclose(res["f"][2, 0], -(s1 + s2), atol=1e-5)


def test_linear_embedding_reduces_to_pair_potential(oracle_lib):
    """F(rho) = c rho makes EAM the pair potential phi + 2 c rho (energy and forces)."""
    c = -0.7
    phi_t = P.tabulate(P.phi, RC, 2000)
    rho_t = P.tabulate(P.rho, RC, 2000)
    lin_t = P.tabulate(lambda p: c * p, 40.0, 2000)
    b = configs.small_box(4, seed=9, sigma_x=0.25)
    res = oracle_lib.forces_at(b.x, b.box, (phi_t, rho_t, lin_t), RC, SKIN)
    d = b.x[None, :, :] - b.x[:, None, :]
    d -= b.box * np.round(d / b.box)
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    m = r < RC
    rr = np.where(m, r, 1.0)
    psi = np.where(m, P.phi(rr) + 2 * c * P.rho(rr), 0.0)
    dpsi = np.where(m, P.dphi(rr) + 2 * c * P.drho(rr), 0.0)
    e = 0.5 * psi.sum()
    f = (dpsi[:, :, None] * d / rr[:, :, None]).sum(1)
    assert abs(res["pe"] - e) < 1e-6
    np.testing.assert_allclose(res["f"], f, atol=2e-6)


def test_tabulated_forces_match_analytic(oracle_lib, md_tables):
    b = configs.small_box(6, seed=13, sigma_x=0.08)
    res = oracle_lib.forces_at(b.x, b.box, md_tables, RC, SKIN)
    fa, ea = oracle_lib.forces_analytic(b.x, b.box, P.analytic_params())
    assert np.max(np.abs(res["f"] - fa)) < 5e-6
    assert abs(res["pe"] - ea) < 1e-6


# ----------------------------------------------------------------- integrator

def _run(b, tables, nsteps, dt, **kw):
    return configs, __import__("oracle").md_run(
        b.x, b.v, b.box, tables, nsteps, mass=configs.MASS, dt=dt, r_cut=RC, skin=SKIN,
        ftm2v=configs.FTM2V, **kw)


def test_nve_energy_and_momentum(oracle_lib, md_tables):
    b = configs.small_box(6, seed=21, temperature=300.0)
    _, out = _run(b, md_tables, 200, 1.0, want_energy=True)
    assert out["code"] == 0 and out["stats"]["steps"] == 200
    e = out["energy"].sum(1)
    assert np.max(np.abs(e - e[0])) / b.n < 2e-4
    p = out["v"].sum(0) * configs.MASS
    assert np.max(np.abs(out["v"].sum(0))) < 1e-12
    assert np.all(np.isfinite(p))


def test_energy_error_is_second_order(oracle_lib, md_tables):
    """Halving dt cuts the total-energy fluctuation by about 4 (second-order scheme)."""
    b = configs.small_box(6, seed=22, temperature=600.0)
    _, o1 = _run(b, md_tables, 100, 1.0, want_energy=True)
    _, o2 = _run(b, md_tables, 200, 0.5, want_energy=True)
    e1 = o1["energy"].sum(1)
    e2 = o2["energy"].sum(1)[::2]
    a1 = np.max(np.abs(e1 - e1[0]))
    a2 = np.max(np.abs(e2 - e2[0]))
    assert 3.0 < a1 / a2 < 5.0, (a1, a2)


def test_time_reversal(oracle_lib, md_tables):
    b = configs.small_box(6, seed=23, temperature=300.0)
    _, fw = _run(b, md_tables, 100, 1.0)
    back = configs.Box(x=fw["x"], v=-fw["v"], box=b.box, n_cells=6, temperature=0, site_ids=None)
    _, bw = _run(back, md_tables, 100, 1.0)
    d = bw["x"] - b.x
    d -= b.box * np.round(d / b.box)
    assert np.max(np.abs(d)) < 1e-9
    np.testing.assert_allclose(-bw["v"], b.v, atol=1e-12)


def test_rebuilds_happen_and_list_stays_valid(oracle_lib, md_tables):
    """A hot run triggers rebuilds; the final forces equal forces from a fresh list."""
    b = configs.small_box(6, seed=24, temperature=2000.0)
    _, out = _run(b, md_tables, 150, 1.0)
    assert out["stats"]["rebuilds"] >= 2
    fresh = oracle_lib.forces_at(out["x"], b.box, md_tables, RC, 0.0)
    np.testing.assert_allclose(out["f"], fresh["f"], rtol=0, atol=1e-12)


def test_thread_count_does_not_change_bits(oracle_lib, md_tables):
    b = configs.small_box(8, seed=25, temperature=900.0)
    oracle_lib.set_threads(1)
    _, a = _run(b, md_tables, 20, 1.0)
    oracle_lib.set_threads(4)
    _, c = _run(b, md_tables, 20, 1.0)
    assert np.array_equal(a["x"], c["x"]) and np.array_equal(a["f"], c["f"])


def test_overflow_and_box_errors(oracle_lib, md_tables):
    b = configs.small_box(6, seed=26)
    _, out = _run(b, md_tables, 1, 1.0, cap=8)
    assert out["code"] == oracle_lib.OR_E_OVERFLOW
    tiny = configs.small_box(3, seed=27)
    _, out = _run(tiny, md_tables, 1, 1.0)
    assert out["code"] == oracle_lib.OR_E_BOX


# ----------------------------------------------------------------- open boundaries

def _numpy_sets(x, box, rlist):
    """All-pairs neighbour sets by numpy: minimum image only where box > 0."""
    d = x[None, :, :] - x[:, None, :]
    per = box > 0
    L = np.abs(box)
    d[..., per] -= L[per] * np.round(d[..., per] / L[per])
    r = np.sqrt((d ** 2).sum(-1))
    np.fill_diagonal(r, np.inf)
    return [frozenset(np.nonzero(r[i] < rlist)[0].tolist()) for i in range(x.shape[0])], r


@pytest.mark.parametrize("sigma", [0.01, 0.2])
def test_open_slab_lists(oracle_lib, sigma):
    """Open x, y (negative box lengths), periodic z: cell list = brute force =
    numpy all-pairs with the minimum image in z only; no pair across the open
    edges."""
    b = configs.slab(7, 6, 5, seed=21, sigma_x=sigma, vacuum=6.0)
    c1, n1, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method="cells")
    c2, n2, _ = oracle_lib.neighbor_list(b.x, b.box, RC + SKIN, method="brute")
    want, r = _numpy_sets(b.x, b.box, RC + SKIN)
    assert not np.any(np.abs(r - (RC + SKIN)) < 1e-9)
    assert oracle_lib.neighbor_sets(c1, n1) == want
    assert oracle_lib.neighbor_sets(c2, n2) == want
    # an atom on the low-x face has no neighbour on the high-x face
    lo = np.argmin(b.x[:, 0])
    hi = set(np.nonzero(b.x[:, 0] > b.x[:, 0].max() - 1.0)[0].tolist())
    assert not (want[lo] & hi)


def test_open_slab_forces(oracle_lib, md_tables):
    """Open slab: net force zero (Newton's third law holds pair by pair) and
    F = -grad U by central differences, surface atoms included."""
    b = configs.slab(6, 6, 5, seed=22, sigma_x=0.05, vacuum=6.0)
    res = oracle_lib.forces_at(b.x, b.box, md_tables, RC, SKIN)
    net = np.abs(res["f"].sum(axis=0))
    assert np.all(net <= 1e-12 * np.abs(res["f"]).sum())
    # surface atoms carry a net inward force of order eV/A, interior ones ~0
    assert np.abs(res["f"][:, 0]).max() > 0.1
    rng = np.random.default_rng(3)
    h = 1e-4
    for i in np.concatenate([[int(np.argmin(b.x[:, 0]))], rng.integers(b.n, size=6)]):
        for d in range(3):
            xp, xm = b.x.copy(), b.x.copy()
            xp[i, d] += h
            xm[i, d] -= h
            ep = oracle_lib.forces_at(xp, b.box, md_tables, RC, SKIN)["pe"]
            em = oracle_lib.forces_at(xm, b.box, md_tables, RC, SKIN)["pe"]
            assert abs(-(ep - em) / (2 * h) - res["f"][i, d]) < 1e-7


# rho(r) >= 0.5, as for the periodic dimer
@pytest.mark.parametrize("r", [2.3, 2.6])
def test_dimer_in_open_box(oracle_lib, md_tables, r):
    """All three dimensions open: a dimer is the closed form with no image at all,
    even when the open box is shorter than twice the list radius."""
    x = np.array([[1.0, 1.0, 1.0], [1.0 + r, 1.0, 1.0]])
    box = -np.array([6.0, 3.0, 3.0])
    res = oracle_lib.forces_at(x, box, md_tables, RC, SKIN)
    e = P.phi(r) + 2 * P.emb(P.rho(r))
    s = P.dphi(r) + 2 * P.demb(P.rho(r)) * P.drho(r)
    assert abs(res["pe"] - e) < 1e-6
    np.testing.assert_allclose(res["f"][0], [s, 0, 0], atol=1e-6)
    np.testing.assert_allclose(res["f"][1], [-s, 0, 0], atol=1e-6)


def _cluster(n_cells=3, seed=91, temperature=100.0, omega=0.002):
    """A small BCC cluster in a box open in every dimension, with thermal
    velocities plus a rigid rotation about its centre (rad/fs)."""
    x = configs.bcc_block(n_cells, n_cells, n_cells) + 10.0
    rng = np.random.default_rng(seed)
    x = x + 0.02 * rng.standard_normal(x.shape)
    v = configs.maxwell_boltzmann(rng, x.shape[0], temperature)
    c = x.mean(axis=0)
    v = v + np.cross(np.array([0.3, -0.5, 1.0]) * omega, x - c)
    return x, v, -np.full(3, 40.0)


def _angular_momentum(x, v):
    c = x.mean(axis=0)
    return configs.MASS * np.cross(x - c, v).sum(axis=0)


def test_open_cluster_conserves_momenta(oracle_lib, md_tables):
    """No images in any dimension: the forces are central and pairwise opposite,
    so velocity Verlet keeps the linear and the angular momentum to rounding."""
    x, v, box = _cluster()
    p0, l0 = configs.MASS * v.sum(axis=0), _angular_momentum(x, v)
    out = oracle_lib.md_run(x, v, box, md_tables, 400, mass=configs.MASS, dt=configs.DT, r_cut=RC,
                            skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == 0
    p1 = configs.MASS * out["v"].sum(axis=0)
    # the centre of mass moves with the (conserved) momentum; the angular
    # momentum is taken about it
    l1 = _angular_momentum(out["x"], out["v"])
    assert np.max(np.abs(p1 - p0)) < 1e-12 * configs.MASS * np.abs(v).sum()
    assert np.max(np.abs(l1 - l0)) < 1e-9 * np.linalg.norm(l0)
    assert np.linalg.norm(l0) > 1.0  # the rotation is not negligible


def test_coincident_atoms_are_reported_nonfinite(oracle_lib, md_tables):
    b = configs.small_box(6, seed=92)
    x = b.x.copy()
    x[5] = x[4]
    out = oracle_lib.md_run(x, b.v, b.box, md_tables, 2, mass=configs.MASS, dt=configs.DT, r_cut=RC,
                            skin=SKIN, ftm2v=configs.FTM2V)
    assert out["code"] == oracle_lib.OR_E_NONFINITE
