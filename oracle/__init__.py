"""ctypes binding of the plain FP64 CPU oracle (oracle/eam_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports or calls it.
All arrays are numpy float64 AoS (N, 3) in original atom order.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "eam_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK, OR_E_BOX, OR_E_OVERFLOW, OR_E_NONFINITE, OR_E_LOST = 0, -2, -4, -6, -9


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Spline(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("reserved", C.c_int32), ("x0", C.c_double),
                ("inv_dx", C.c_double), ("coef", C.POINTER(C.c_double))]


class MDParams(C.Structure):
    _fields_ = [("box", C.c_double * 3), ("mass", C.c_double), ("dt", C.c_double),
                ("r_cut", C.c_double), ("skin", C.c_double), ("ftm2v", C.c_double),
                ("cap", C.c_int32), ("reserved", C.c_int32)]


class MDStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("list_entries", C.c_int64),
                ("max_count", C.c_int32), ("flags", C.c_int32)]


class Analytic(C.Structure):
    _fields_ = [("rc", C.c_double), ("r0", C.c_double), ("phi_a", C.c_double),
                ("phi_b", C.c_double), ("rho_b", C.c_double), ("emb_a", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        pd, pi = P(d), P(i32)
        sig = {
            "or_set_threads": (None, [i32]),
            "or_get_threads": (i32, []),
            "or_spline_eval": (None, [P(Spline), i64, pd, pd, pd, pd]),
            "or_wrap": (i64, [i64, pd, pd]),
            "or_cell_grid": (i32, [pd, d, pi, pd]),
            "or_cell_ids": (None, [i64, pd, pi, pd, pi]),
            "or_cell_sort": (None, [i64, pi, i32, pi, pi]),
            "or_list_brute": (i32, [i64, pd, pd, d, i32, pi, pi]),
            "or_list_cells": (i32, [i64, pd, pd, d, i32, pi, pi]),
            "or_density": (i32, [i64, pd, pd, pi, pi, i32, d, P(Spline), P(Spline), pd, pd, pd]),
            "or_forces": (None, [i64, pd, pd, pi, pi, i32, d, P(Spline), P(Spline), pd, pd]),
            "or_energy_atoms": (None, [i64, pd, pd, pd, pi, pi, i32, d, P(Spline), P(Spline), pd,
                                       d, d, pd, pd]),
            "or_energy": (None, [i64, pd, pd, pd, pi, pi, i32, d, P(Spline), P(Spline), P(Spline),
                                 d, d, pd, pd]),
            "or_md_run": (i32, [i64, pd, pd, pd, P(MDParams), P(Spline), P(Spline), P(Spline), i64,
                                pd, P(MDStats)]),
            "or_forces_at": (i32, [i64, pd, pd, d, d, i32, P(Spline), P(Spline), P(Spline), pd, pd,
                                   pd, pd]),
            "or_forces_analytic": (i32, [i64, pd, pd, P(Analytic), pd, pd]),
            "or_forces_at_multi": (i32, [i64, pd, pd, d, d, i32, i32, pi, P(Spline), P(Spline),
                                         P(Spline), pd, pd, pd, pd]),
            "or_md_run_multi": (i32, [i64, pd, pd, pd, P(MDParams), i32, pi, pd, P(Spline),
                                      P(Spline), P(Spline), i64, pd, P(MDStats)]),
            "or_fm_loss_grad": (d, [i32, P(i64), pd, pd, d, P(Spline), P(Spline), P(Spline), pd,
                                    pd, pd, pd, pd]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def _pd(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _pi(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class _SplineRef:
    """Keeps the coefficient array alive next to its ctypes struct."""

    def __init__(self, table):
        self.coef = np.ascontiguousarray(table.coef, dtype=np.float64)
        self.s = Spline(self.coef.shape[0] + 1, 0, float(table.x0), float(1.0 / table.dx),
                        self.coef.ctypes.data_as(C.POINTER(C.c_double)))

    @property
    def ref(self):
        return C.byref(self.s)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def spline_eval(table, s):
    s = _f64(s).ravel()
    f, df, ddf = (np.empty_like(s) for _ in range(3))
    sp = _SplineRef(table)
    lib().or_spline_eval(sp.ref, s.size, _pd(s), _pd(f), _pd(df), _pd(ddf))
    return f, df, ddf


def wrap(x, box):
    x = _f64(x).copy()
    box = _f64(box)
    bad = lib().or_wrap(x.shape[0], _pd(x), _pd(box))
    return x, int(bad)


def cell_grid(box, rlist):
    nc = np.zeros(3, np.int32)
    ic = np.zeros(3, np.float64)
    rc = lib().or_cell_grid(_pd(_f64(box)), float(rlist), _pi(nc), _pd(ic))
    return rc, nc, ic


def cell_ids(x, box, rlist):
    x = _f64(x)
    rc, nc, ic = cell_grid(box, rlist)
    if rc != OR_OK:
        raise ValueError("box too small for a 3x3x3 cell grid")
    cell = np.empty(x.shape[0], np.int32)
    lib().or_cell_ids(x.shape[0], _pd(x), _pi(nc), _pd(ic), _pi(cell))
    return cell, nc, ic


def cell_sort(cell, ncells):
    cell = np.ascontiguousarray(cell, np.int32)
    start = np.empty(ncells + 1, np.int32)
    order = np.empty(cell.size, np.int32)
    lib().or_cell_sort(cell.size, _pi(cell), int(ncells), _pi(start), _pi(order))
    return start, order


def neighbor_list(x, box, rlist, cap=128, method="cells"):
    x = _f64(x)
    n = x.shape[0]
    cnt = np.empty(n, np.int32)
    nbr = np.full((n, cap), -1, np.int32)
    fn = lib().or_list_cells if method == "cells" else lib().or_list_brute
    mx = fn(n, _pd(x), _pd(_f64(box)), float(rlist), int(cap), _pi(cnt), _pi(nbr))
    return cnt, nbr, int(mx)


def neighbor_sets(cnt, nbr):
    return [frozenset(nbr[i, : cnt[i]].tolist()) for i in range(cnt.size)]


def density(x, box, cnt, nbr, rc, rho_t, emb_t):
    x = _f64(x)
    n = x.shape[0]
    cap = nbr.shape[1]
    r, fp, fpp = np.empty(n), np.empty(n), np.empty(n)
    a, b = _SplineRef(rho_t), _SplineRef(emb_t)
    nbr = np.ascontiguousarray(nbr, np.int32)
    cnt = np.ascontiguousarray(cnt, np.int32)
    flag = lib().or_density(n, _pd(x), _pd(_f64(box)), _pi(cnt), _pi(nbr), cap, float(rc), a.ref,
                            b.ref, _pd(r), _pd(fp), _pd(fpp))
    return r, fp, fpp, int(flag)


def forces(x, box, cnt, nbr, rc, phi_t, rho_t, fp):
    x = _f64(x)
    n = x.shape[0]
    f = np.empty((n, 3))
    a, b = _SplineRef(phi_t), _SplineRef(rho_t)
    nbr = np.ascontiguousarray(nbr, np.int32)
    cnt = np.ascontiguousarray(cnt, np.int32)
    lib().or_forces(n, _pd(x), _pd(_f64(box)), _pi(cnt), _pi(nbr), nbr.shape[1], float(rc), a.ref,
                    b.ref, _pd(_f64(fp)), _pd(f))
    return f


def energy(x, v, box, cnt, nbr, rc, phi_t, rho_t, emb_t, mass, ftm2v):
    x = _f64(x)
    pe, ke = C.c_double(), C.c_double()
    a, b, e = _SplineRef(phi_t), _SplineRef(rho_t), _SplineRef(emb_t)
    nbr = np.ascontiguousarray(nbr, np.int32)
    cnt = np.ascontiguousarray(cnt, np.int32)
    vv = None if v is None else _f64(v)
    lib().or_energy(x.shape[0], _pd(x), _pd(vv), _pd(_f64(box)), _pi(cnt), _pi(nbr), nbr.shape[1],
                    float(rc), a.ref, b.ref, e.ref, float(mass), float(ftm2v), C.byref(pe),
                    C.byref(ke))
    return pe.value, ke.value


def forces_at(x, box, tables, rc, skin=0.0, cap=256):
    """Forces, rho, F' and potential energy of a configuration (list built at rc + skin)."""
    x = _f64(x)
    n = x.shape[0]
    f, r, fp = np.empty((n, 3)), np.empty(n), np.empty(n)
    pe = C.c_double()
    refs = [_SplineRef(t) for t in tables]
    code = lib().or_forces_at(n, _pd(x), _pd(_f64(box)), float(rc), float(skin), int(cap),
                              refs[0].ref, refs[1].ref, refs[2].ref, _pd(f), _pd(r), _pd(fp),
                              C.byref(pe))
    if code < 0:
        raise RuntimeError(f"oracle forces_at failed: {code}")
    return dict(f=f, rho=r, fp=fp, pe=pe.value, flags=code)


def forces_analytic(x, box, params):
    """Forces and energy of the closed-form potential; params holds rc, r0, phi_a,
    phi_b, rho_b, emb_a (the synthetic potential's constants)."""
    x = _f64(x)
    f = np.empty_like(x)
    pe = C.c_double()
    an = Analytic(*[float(params[k]) for k in ("rc", "r0", "phi_a", "phi_b", "rho_b", "emb_a")])
    code = lib().or_forces_analytic(x.shape[0], _pd(x), _pd(_f64(box)), C.byref(an), _pd(f),
                                    C.byref(pe))
    if code != OR_OK:
        raise RuntimeError(f"oracle forces_analytic failed: {code}")
    return f, pe.value


def md_run(x, v, box, tables, nsteps, *, mass, dt, r_cut, skin, ftm2v, cap=128,
           want_energy=False):
    """Velocity-Verlet run; returns dict(x, v, f, energy (nsteps+1, 2) or None, stats, code)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[0]
    f = np.empty_like(x)
    p = MDParams((C.c_double * 3)(*[float(b) for b in box]), mass, dt, r_cut, skin, ftm2v, cap, 0)
    st = MDStats()
    en = np.empty((nsteps + 1, 2)) if want_energy else None
    refs = [_SplineRef(t) for t in tables]
    code = lib().or_md_run(n, _pd(x), _pd(v), _pd(f), C.byref(p), refs[0].ref, refs[1].ref,
                           refs[2].ref, int(nsteps), _pd(en), C.byref(st))
    stats = dict(steps=st.steps, rebuilds=st.rebuilds, list_entries=st.list_entries,
                 max_count=st.max_count, flags=st.flags)
    return dict(x=x, v=v, f=f, energy=en, stats=stats, code=int(code))


def fm_loss_grad(x, offsets, boxes, tables, fref, rc=5.0, want_grad=True):
    """Force-matching loss and gradient w.r.t. the per-segment coefficients of (phi, rho, F)."""
    x = _f64(x)
    off = np.ascontiguousarray(offsets, np.int64)
    boxes = _f64(boxes)
    fref = _f64(fref)
    refs = [_SplineRef(t) for t in tables]
    grads = [np.zeros_like(r.coef) for r in refs] if want_grad else [None, None, None]
    f = np.empty_like(x)
    loss = lib().or_fm_loss_grad(int(off.size - 1), off.ctypes.data_as(C.POINTER(C.c_int64)),
                                 _pd(x), _pd(boxes), float(rc), refs[0].ref, refs[1].ref,
                                 refs[2].ref, _pd(fref), _pd(grads[0]), _pd(grads[1]),
                                 _pd(grads[2]), _pd(f))
    return float(loss), grads, f


# ---------------------------------------------------------------- several atom types

class _SplineArray:
    """A contiguous C array of spline structs (and the coefficient arrays behind it)."""

    def __init__(self, tables):
        self.refs = [_SplineRef(t) for t in tables]
        self.arr = (Spline * len(self.refs))(*[r.s for r in self.refs])

    @property
    def ptr(self):
        return C.cast(self.arr, C.POINTER(Spline))


def _multi_tables(tabs):
    """tabs = (phi[a][b], rho[t], emb[t]) -> (n_types, phi array (row-major a, b), rho, emb)."""
    phi, rho, emb = tabs
    nt = len(rho)
    assert len(emb) == nt and len(phi) == nt and all(len(row) == nt for row in phi)
    return nt, _SplineArray([phi[a][b] for a in range(nt) for b in range(nt)]), \
        _SplineArray(rho), _SplineArray(emb)


def forces_at_multi(x, box, types, tabs, rc, skin=0.0, cap=256):
    """Multi-species forces, rho, F' and potential energy (list built at rc + skin)."""
    x = _f64(x)
    n = x.shape[0]
    t = np.ascontiguousarray(types, np.int32)
    nt, ph, rh, em = _multi_tables(tabs)
    assert t.shape == (n,) and (n == 0 or (t.min() >= 0 and t.max() < nt))
    f, r, fp = np.empty((n, 3)), np.empty(n), np.empty(n)
    pe = C.c_double()
    code = lib().or_forces_at_multi(n, _pd(x), _pd(_f64(box)), float(rc), float(skin), int(cap),
                                    nt, _pi(t), ph.ptr, rh.ptr, em.ptr, _pd(f), _pd(r), _pd(fp),
                                    C.byref(pe))
    if code < 0:
        raise RuntimeError(f"oracle forces_at_multi failed: {code}")
    return dict(f=f, rho=r, fp=fp, pe=pe.value, flags=code)


def md_run_multi(x, v, box, types, tabs, masses, nsteps, *, dt, r_cut, skin, ftm2v, cap=128,
                 want_energy=False):
    """Multi-species velocity-Verlet run (per-type masses)."""
    x = _f64(x).copy()
    v = _f64(v).copy()
    n = x.shape[0]
    t = np.ascontiguousarray(types, np.int32)
    nt, ph, rh, em = _multi_tables(tabs)
    m = _f64(masses)
    assert m.shape == (nt,)
    f = np.empty_like(x)
    p = MDParams((C.c_double * 3)(*[float(b) for b in box]), 1.0, dt, r_cut, skin, ftm2v, cap, 0)
    st = MDStats()
    en = np.empty((nsteps + 1, 2)) if want_energy else None
    code = lib().or_md_run_multi(n, _pd(x), _pd(v), _pd(f), C.byref(p), nt, _pi(t), _pd(m),
                                 ph.ptr, rh.ptr, em.ptr, int(nsteps), _pd(en), C.byref(st))
    stats = dict(steps=st.steps, rebuilds=st.rebuilds, list_entries=st.list_entries,
                 max_count=st.max_count, flags=st.flags)
    return dict(x=x, v=v, f=f, energy=en, stats=stats, code=int(code))
