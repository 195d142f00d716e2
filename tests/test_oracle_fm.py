"""Pins of the oracle's force-matching loss gradient.

The predicted forces are linear in the phi and F spline coefficients (at fixed
rho coefficients), so the loss is exactly quadratic in them and a central
difference is exact up to rounding; rho directions are checked with central
differences at two step sizes.  Segments that no pair visits must get an
exact zero, the gradient must add over configurations, and the chain rule to
knot values must match differences taken on the knot values themselves.
"""
import numpy as np
import pytest

from workloads import configs, potential as P


@pytest.fixture(scope="module")
def fm_problem(oracle_lib):
    boxes = [configs.small_box(5, seed=100 + c, sigma_x=0.12, temperature=0.0) for c in range(2)]
    x = np.concatenate([b.x for b in boxes])
    off = np.array([0, boxes[0].n, boxes[0].n + boxes[1].n], np.int64)
    bx = np.stack([b.box for b in boxes])
    fref = np.concatenate([oracle_lib.forces_analytic(b.x, b.box, P.analytic_params())[0] for b in boxes])
    tabs = P.fm_tables()
    return dict(x=x, off=off, boxes=bx, fref=fref, tabs=tabs)


def _loss(oracle_lib, pb, tabs):
    return oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], tabs, pb["fref"],
                                   want_grad=False)[0]


def _with(tabs, which, q, delta):
    out = []
    for k, t in enumerate(tabs):
        c = t.coef.copy()
        if k == which:
            c.ravel()[q] += delta
        out.append(P.SplineTable(x0=t.x0, dx=t.dx, coef=c))
    return tuple(out)


def test_loss_is_positive_and_forces_close(oracle_lib, fm_problem):
    pb = fm_problem
    loss, grads, f = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"],
                                             pb["fref"])
    assert loss > 0 and np.isfinite(loss)
    assert np.isclose(loss, np.sum((f - pb["fref"]) ** 2), rtol=1e-12)


@pytest.mark.parametrize("which", [0, 2])
def test_grad_phi_and_F_exact_by_central_difference(oracle_lib, fm_problem, which):
    pb = fm_problem
    _, grads, _ = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"], pb["fref"])
    g = grads[which].ravel()
    nz = np.nonzero(g)[0]
    assert nz.size > 8
    rng = np.random.default_rng(which)
    pick = np.unique(np.concatenate([nz[np.argsort(-np.abs(g[nz]))[:6]],
                                     rng.choice(nz, 10, replace=False)]))
    h = 1e-6
    loss0 = _loss(oracle_lib, pb, pb["tabs"])
    # the loss is quadratic in these coefficients: only rounding of the two losses remains
    tol = 8 * np.finfo(float).eps * loss0 / h
    for q in pick:
        lp = _loss(oracle_lib, pb, _with(pb["tabs"], which, q, h))
        lm = _loss(oracle_lib, pb, _with(pb["tabs"], which, q, -h))
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[q]) <= tol, (which, q, fd, g[q], tol)


def test_grad_rho_by_central_difference(oracle_lib, fm_problem):
    pb = fm_problem
    _, grads, _ = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"], pb["fref"])
    g = grads[1].ravel()
    nz = np.nonzero(g)[0]
    rng = np.random.default_rng(7)
    pick = np.unique(np.concatenate([nz[np.argsort(-np.abs(g[nz]))[:6]],
                                     rng.choice(nz, 8, replace=False)]))
    scale = np.max(np.abs(g))
    h = 1e-6
    for q in pick:
        fds = []
        for hh in (h, 2 * h):
            lp = _loss(oracle_lib, pb, _with(pb["tabs"], 1, q, hh))
            lm = _loss(oracle_lib, pb, _with(pb["tabs"], 1, q, -hh))
            fds.append((lp - lm) / (2 * hh))
        # fd(h) = g + c h^2 + rounding; |fd(2h) - fd(h)| = 3 c h^2 estimates the truncation
        trunc = abs(fds[1] - fds[0]) / 3.0
        assert abs(fds[0] - g[q]) <= 2.0 * trunc + 2e-9 * scale, (q, fds, g[q])
        assert trunc <= 1e-7 * scale


def test_unvisited_segments_are_exactly_zero(oracle_lib, fm_problem):
    pb = fm_problem
    _, grads, _ = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"], pb["fref"])
    phi_t = pb["tabs"][0]
    # no pair is closer than 1.5 A: phi segments below 1.5 A are never evaluated
    k_lo = int(1.5 / phi_t.dx)
    assert np.all(grads[0][:k_lo] == 0.0) and np.all(grads[1][:k_lo] == 0.0)
    # F segments far above any rho_i
    emb_t = pb["tabs"][2]
    k_hi = int(6.0 / emb_t.dx)
    assert np.all(grads[2][k_hi:] == 0.0)


def test_gradient_adds_over_configurations(oracle_lib, fm_problem):
    pb = fm_problem
    _, g_all, _ = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"], pb["fref"])
    parts = []
    for c in range(2):
        a, b = pb["off"][c], pb["off"][c + 1]
        _, g, _ = oracle_lib.fm_loss_grad(pb["x"][a:b], np.array([0, b - a]), pb["boxes"][c:c + 1],
                                          pb["tabs"], pb["fref"][a:b])
        parts.append(g)
    for k in range(3):
        np.testing.assert_allclose(g_all[k], parts[0][k] + parts[1][k], rtol=1e-12, atol=1e-12)


def test_knot_value_chain_rule(oracle_lib, fm_problem):
    """dL/dy = M^T dL/dc, checked by central differences on the knot values of phi."""
    pb = fm_problem
    _, grads, _ = oracle_lib.fm_loss_grad(pb["x"], pb["off"], pb["boxes"], pb["tabs"], pb["fref"])
    M = P.spline_value_map(P.FM_KNOTS)
    gy = M.T @ grads[0].ravel()
    kv = P.fm_knot_values()
    x1, y = kv[0]
    dx = x1 / (P.FM_KNOTS - 1)
    for k in (40, 45, 50, 55):
        vals = []
        for s in (+1, -1):
            yy = y.copy()
            yy[k] += s * 1e-6
            t0 = P.natural_spline_from_values(0.0, dx, yy)
            vals.append(_loss(oracle_lib, pb, (t0, pb["tabs"][1], pb["tabs"][2])))
        fd = (vals[0] - vals[1]) / 2e-6
        assert abs(fd - gy[k]) <= 1e-6 * np.max(np.abs(gy)), (k, fd, gy[k])


def test_orthorhombic_configurations_by_central_difference(oracle_lib):
    """Configurations with three different periodic edge lengths: the phi
    gradient against central differences (exact up to rounding, the loss being
    quadratic in those coefficients)."""
    boxes = [configs.ortho_box(5, 6, 7, seed=110, sigma_x=0.12, temperature=0.0),
             configs.ortho_box(6, 5, 5, seed=111, sigma_x=0.12, temperature=0.0)]
    x = np.concatenate([b.x for b in boxes])
    off = np.array([0, boxes[0].n, boxes[0].n + boxes[1].n], np.int64)
    bx = np.stack([b.box for b in boxes])
    fref = np.concatenate([oracle_lib.forces_analytic(b.x, b.box, P.analytic_params())[0]
                           for b in boxes])
    pb = dict(x=x, off=off, boxes=bx, fref=fref, tabs=P.fm_tables())
    _, grads, _ = oracle_lib.fm_loss_grad(x, off, bx, pb["tabs"], fref)
    g = grads[0].ravel()
    nz = np.nonzero(g)[0]
    pick = nz[np.argsort(-np.abs(g[nz]))[:8]]
    h = 1e-6
    loss0 = _loss(oracle_lib, pb, pb["tabs"])
    tol = 8 * np.finfo(float).eps * loss0 / h
    for q in pick:
        lp = _loss(oracle_lib, pb, _with(pb["tabs"], 0, q, h))
        lm = _loss(oracle_lib, pb, _with(pb["tabs"], 0, q, -h))
        assert abs((lp - lm) / (2 * h) - g[q]) <= tol


def test_open_slab_configuration_by_central_difference(oracle_lib):
    """A configuration with open x and y (a slab) next to a periodic one: the
    phi gradient against central differences."""
    boxes = [configs.slab(6, 6, 5, seed=112, sigma_x=0.12, vacuum=3.0, temperature=0.0),
             configs.small_box(5, seed=113, sigma_x=0.12, temperature=0.0)]
    x = np.concatenate([b.x for b in boxes])
    off = np.array([0, boxes[0].n, boxes[0].n + boxes[1].n], np.int64)
    bx = np.stack([b.box for b in boxes])
    assert bx[0, 0] < 0 and bx[0, 1] < 0
    fref = np.concatenate([oracle_lib.forces_analytic(b.x, b.box, P.analytic_params())[0]
                           for b in boxes])
    pb = dict(x=x, off=off, boxes=bx, fref=fref, tabs=P.fm_tables())
    _, grads, _ = oracle_lib.fm_loss_grad(x, off, bx, pb["tabs"], fref)
    g = grads[0].ravel()
    nz = np.nonzero(g)[0]
    pick = nz[np.argsort(-np.abs(g[nz]))[:8]]
    h = 1e-6
    loss0 = _loss(oracle_lib, pb, pb["tabs"])
    tol = 8 * np.finfo(float).eps * loss0 / h
    for q in pick:
        lp = _loss(oracle_lib, pb, _with(pb["tabs"], 0, q, h))
        lm = _loss(oracle_lib, pb, _with(pb["tabs"], 0, q, -h))
        assert abs((lp - lm) / (2 * h) - g[q]) <= tol
