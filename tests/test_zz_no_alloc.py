"""md_forces_static, the entry point that allocates nothing (its scratch is a
fixed device array), against the workspace path it stands in for
(md_create + md_set_state + md_build_neighbors + md_compute_forces) on the
same boxes, through the C ABI.  Consecutive calls share the array, so the
calls run in a row with the box shrinking: 16,000 atoms, then 432, in float64
and in the mixed form.  The same kernels run in the same order on the same
inputs, so forces, rho_i and F'_i are bitwise equal; the float64 forces are
also within 1e-10 of the oracle's."""
import ctypes as C
import sys

import numpy as np
import pytest

from workloads import configs, potential as P

RC, SKIN = P.RC, configs.SKIN


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _params(md, prec):
    return md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                          ftm2v=configs.FTM2V, precision=prec, nbr_capacity=128,
                          cell_capacity=64)


def _device_spline(md, torch, tab):
    """md_spline whose coefficients live in device memory (kept alive by the tensor)."""
    coef = torch.as_tensor(np.ascontiguousarray(tab.coef), device="cuda")
    sp = md.md_spline(tab.coef.shape[0] + 1, 0, float(tab.x0), float(1.0 / tab.dx),
                      C.cast(C.c_void_p(coef.data_ptr()), C.POINTER(C.c_double)))
    return sp, coef


def _static_forces(md, torch, p, box, dev_tabs):
    n = box.n
    x = torch.as_tensor(box.x, device="cuda")
    f = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    rho = torch.empty(n, dtype=torch.float64, device="cuda")
    fp = torch.empty(n, dtype=torch.float64, device="cuda")
    b = np.ascontiguousarray(box.box, dtype=np.float64)
    torch.cuda.synchronize()
    rc = md.lib().md_forces_static(C.byref(p), n, b.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(dev_tabs[0][0]), C.byref(dev_tabs[1][0]),
                                   C.byref(dev_tabs[2][0]), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(f.data_ptr()), C.c_void_p(rho.data_ptr()),
                                   C.c_void_p(fp.data_ptr()),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == md.MD_OK, rc
    return f.cpu().numpy(), rho.cpu().numpy(), fp.cpu().numpy()


def _workspace_forces(md, p, tabs, box):
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    out = tuple(t.cpu().numpy() for t in s.compute_forces())
    s.close()
    return out


@pytest.mark.gpu
def test_static_forces_equal_the_workspace_path(oracle_lib):
    import torch

    from paper_2405_07898_amd import md

    assert torch.cuda.is_available()
    tabs = P.md_tables()
    dev_tabs = [_device_spline(md, torch, t) for t in tabs]
    big = configs.small_box(20, seed=91, temperature=900.0, sigma_x=0.05)   # 16,000 atoms
    small = configs.small_box(6, seed=92, temperature=1500.0, sigma_x=0.05)  # 432 atoms
    assert big.n <= md.MD_STATIC_MAX_ATOMS
    for prec in (md.MD_FP64, md.MD_MIXED):
        p = _params(md, prec)
        for box in (big, small):
            _say(f"[gpu] md_forces_static precision={prec} n={box.n}")
            fs, rs, ps = _static_forces(md, torch, p, box, dev_tabs)
            fw, rw, pw = _workspace_forces(md, p, tabs, box)
            assert np.array_equal(fs, fw) and np.array_equal(rs, rw) and np.array_equal(ps, pw)
            if prec == md.MD_FP64:
                ref = oracle_lib.forces_at(box.x, box.box, tabs, RC, SKIN)
                err = np.max(np.abs(fs - ref["f"])) / np.max(np.abs(ref["f"]))
                assert err < 1e-10, err


def test_static_forces_reject_sizes_past_the_limits_without_gpu():
    """Sizes past the fixed array's limits (atoms, cells, table knots) and the
    forms it does not run are rejected on the host, before any device call."""
    from paper_2405_07898_amd import md

    lib = md.lib()
    fake = C.cast(C.c_void_p(256), C.POINTER(C.c_double))  # never dereferenced on the host

    def spline(n_knots):
        return md.md_spline(n_knots, 0, 0.0, (n_knots - 1) / 5.0, fake)

    def call(p, n, box, knots=2000):
        b = np.ascontiguousarray(box, dtype=np.float64)
        sp = [spline(knots), spline(knots), spline(knots)]
        return lib.md_forces_static(C.byref(p), n, b.ctypes.data_as(C.POINTER(C.c_double)),
                                    C.byref(sp[0]), C.byref(sp[1]), C.byref(sp[2]),
                                    C.c_void_p(256), C.c_void_p(256), None, None, None)

    p = _params(md, md.MD_FP64)
    ok_box = [66.08, 66.08, 66.08]
    assert call(p, md.MD_STATIC_MAX_ATOMS + 1, ok_box) == md.MD_E_ARG
    assert call(p, 0, ok_box) == md.MD_E_ARG
    assert call(p, 1000, [400.0, 400.0, 400.0]) == md.MD_E_ARG       # 75^3 cells
    assert call(p, 1000, ok_box, knots=md.MD_STATIC_MAX_KNOTS + 1) == md.MD_E_TABLE
    assert call(p, 1000, [10.0, 66.08, 66.08]) == md.MD_E_BOX        # below 2 (r_cut + skin)
    half = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                          ftm2v=configs.FTM2V, list_mode=md.MD_LIST_HALF)
    assert call(half, 1000, ok_box) == md.MD_E_ARG
    big_cap = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=RC, skin=SKIN,
                             ftm2v=configs.FTM2V, nbr_capacity=256)
    assert call(big_cap, 1000, ok_box) == md.MD_E_ARG
