"""Force-matching loss and adjoint on the GPU vs the FP64 CPU oracle."""
import sys

import numpy as np
import pytest

from workloads import configs, potential as P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _problem(oracle_lib, boxes):
    x = np.concatenate([b.x for b in boxes])
    off = np.concatenate([[0], np.cumsum([b.n for b in boxes])]).astype(np.int64)
    bx = np.stack([b.box for b in boxes])
    fref = np.concatenate([oracle_lib.forces_analytic(b.x, b.box, P.analytic_params())[0] for b in boxes])
    return x, off, bx, fref


@pytest.fixture(scope="module")
def fm():
    import torch

    assert torch.cuda.is_available()
    from paper_2405_07898_amd import fm as fmmod

    return fmmod


@pytest.mark.parametrize("n_cfg,ncell", [(3, 5), (64, 10)])
def test_loss_forces_gradient_match_oracle(fm, oracle_lib, n_cfg, ncell):
    import torch

    boxes = configs.config_fm(n_cfg, ncell)
    x, off, bx, fref = _problem(oracle_lib, boxes)
    tabs = P.fm_tables()
    _say(f"[gpu] force matching n_cfg={n_cfg} n={x.shape[0]}")
    prob = fm.ForceMatch(x, fref, np.diff(off), bx, tabs)
    coefs = [torch.as_tensor(t.coef, device="cuda") for t in tabs]
    loss, f = prob.forward(*coefs, want_forces=True)
    g = [t.cpu().numpy() for t in prob.backward()]
    loss_o, g_o, f_o = oracle_lib.fm_loss_grad(x, off, bx, tabs, fref)
    assert abs(loss - loss_o) <= 1e-12 * abs(loss_o)
    fe = f.cpu().numpy()
    assert np.max(np.abs(fe - f_o)) <= 1e-10 * np.max(np.abs(f_o))
    scale = max(np.max(np.abs(a)) for a in g_o)
    for a, b in zip(g, g_o):
        assert np.max(np.abs(a - b)) <= 1e-9 * scale
        # segments no pair visits are exactly zero on both sides
        assert np.all(a[b == 0.0] == 0.0)
    prob.close()


def test_orthorhombic_and_open_configurations(fm, oracle_lib):
    """Configurations with three different periodic edge lengths, and a slab
    open in x and y (the adjoint kernels apply image shifts of their own)."""
    import torch

    boxes = [configs.ortho_box(5, 6, 7, seed=120, sigma_x=0.1, temperature=0.0),
             configs.ortho_box(7, 5, 6, seed=121, sigma_x=0.1, temperature=0.0),
             configs.slab(6, 6, 5, seed=122, sigma_x=0.1, vacuum=3.0, temperature=0.0)]
    x, off, bx, fref = _problem(oracle_lib, boxes)
    tabs = P.fm_tables()
    _say(f"[gpu] force matching orthorhombic n={x.shape[0]}")
    prob = fm.ForceMatch(x, fref, np.diff(off), bx, tabs)
    coefs = [torch.as_tensor(t.coef, device="cuda") for t in tabs]
    loss, f = prob.forward(*coefs, want_forces=True)
    g = [t.cpu().numpy() for t in prob.backward()]
    prob.close()
    loss_o, g_o, f_o = oracle_lib.fm_loss_grad(x, off, bx, tabs, fref)
    assert abs(loss - loss_o) <= 1e-12 * abs(loss_o)
    assert np.max(np.abs(f.cpu().numpy() - f_o)) <= 1e-10 * np.max(np.abs(f_o))
    scale = max(np.max(np.abs(a)) for a in g_o)
    for a, b in zip(g, g_o):
        assert np.max(np.abs(a - b)) <= 1e-9 * scale


def test_adjoint_is_deterministic_and_autograd_consistent(fm, oracle_lib):
    import torch

    boxes = configs.config_fm(4, 6)
    x, off, bx, fref = _problem(oracle_lib, boxes)
    tabs = P.fm_tables()
    _say(f"[gpu] force matching determinism n={x.shape[0]}")
    prob = fm.ForceMatch(x, fref, np.diff(off), bx, tabs)
    coefs = [torch.as_tensor(t.coef, device="cuda").clone().requires_grad_(True) for t in tabs]
    prob.forward(*[c.detach() for c in coefs])
    g1 = [t.cpu().numpy() for t in prob.backward()]
    g2 = [t.cpu().numpy() for t in prob.backward()]
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)
    loss = fm.eam_force_match(*coefs, prob)
    (2.0 * loss).backward()
    for c, a in zip(coefs, g1):
        np.testing.assert_allclose(c.grad.cpu().numpy(), 2.0 * a, rtol=0, atol=0)
    # central differences in phi and F coefficients (loss is quadratic in them)
    base = [c.detach().clone() for c in coefs]
    h = 1e-6
    L0 = prob.forward(*base)[0]
    tol = 8 * np.finfo(float).eps * L0 / h
    for which in (0, 2):
        flat = g1[which].ravel()
        for q in np.argsort(-np.abs(flat))[:4]:
            vals = []
            for sgn in (1, -1):
                cs = [b.clone() for b in base]
                cs[which].view(-1)[q] += sgn * h
                vals.append(prob.forward(*cs)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - flat[q]) <= tol + 1e-9 * np.max(np.abs(flat)), (which, q, fd, flat[q])
    prob.close()


def test_async_calls_equal_the_synchronous_ones(fm, oracle_lib):
    """md_fm_forward_async / md_fm_backward_async (no host synchronisation, the
    loss and the seed on the device) give bitwise the loss and gradients of
    the synchronous calls; a non-finite evaluation stays latched until
    md_fm_check, which reports it once and clears it."""
    import torch

    from paper_2405_07898_amd import md

    boxes = configs.config_fm(3, 5)
    x, off, bx, fref = _problem(oracle_lib, boxes)
    tabs = P.fm_tables()
    _say(f"[gpu] force matching async calls n={x.shape[0]}")
    prob = fm.ForceMatch(x, fref, np.diff(off), bx, tabs)
    coefs = [torch.as_tensor(t.coef, device="cuda") for t in tabs]
    loss_s, _ = prob.forward(*coefs)
    g_s = [t.cpu().numpy() for t in prob.backward(0.5)]
    loss_a, _ = prob.forward_async(*coefs)
    g_a = [t.cpu().numpy() for t in prob.backward_async(torch.tensor(0.5, dtype=torch.float64))]
    prob.check()
    assert loss_a.item() == loss_s
    for a, b in zip(g_a, g_s):
        assert np.array_equal(a, b)
    bad = [c.clone() for c in coefs]
    bad[0].fill_(float("nan"))  # every phi segment, so the visited ones too
    prob.forward_async(*bad)
    prob.backward_async(torch.tensor(1.0, dtype=torch.float64))
    with pytest.raises(md.MDError) as err:
        prob.check()
    assert err.value.code == md.MD_E_NONFINITE
    prob.check()  # cleared
    loss_b, _ = prob.forward(*coefs)
    assert loss_b == loss_s
    prob.close()
