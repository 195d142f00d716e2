"""Thin ctypes binding of libmdeam.so (C ABI in include/md.h).

Functions keep the C names; arguments are marshalled from torch tensors
(device memory, streams) and numpy arrays (host tables).  Every step of the
computation runs in the library's HIP kernels; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdeam.so")

MD_OK = 0
MD_E_ARG, MD_E_BOX, MD_E_TABLE, MD_E_NBR_OVERFLOW, MD_E_CELL_OVERFLOW = -1, -2, -3, -4, -5
MD_E_NONFINITE, MD_E_HIP, MD_E_ORDER, MD_E_LOST_ATOM, MD_E_WORKSPACE = -6, -7, -8, -9, -10
MD_E_STALL = -11
MD_W_RHO_RANGE = 1
MD_STATIC_MAX_ATOMS, MD_STATIC_MAX_CELLS, MD_STATIC_MAX_KNOTS = 16384, 4096, 2048
MD_FP64, MD_MIXED = 0, 1
MD_LIST_FULL, MD_LIST_HALF = 0, 1
MD_LAUNCH_GRAPH, MD_LAUNCH_PERSISTENT = 0, 1
PASS_DENSITY, PASS_FORCE, PASS_BUILD, PASS_BIN, PASS_FORCE_RAW = 0, 1, 2, 3, 4


class MDError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code}) {detail}".strip())


class md_spline(C.Structure):
    _fields_ = [("n_knots", C.c_int32), ("reserved", C.c_int32), ("x0", C.c_double),
                ("inv_dx", C.c_double), ("coef", C.POINTER(C.c_double))]


class md_params(C.Structure):
    _fields_ = [("mass", C.c_double), ("dt", C.c_double), ("r_cut", C.c_double),
                ("skin", C.c_double), ("ftm2v", C.c_double), ("kboltz", C.c_double),
                ("precision", C.c_int32), ("nbr_capacity", C.c_int32),
                ("cell_capacity", C.c_int32), ("chunk_steps", C.c_int32),
                ("lanes_per_atom", C.c_int32), ("sort_every", C.c_int32),
                ("list_mode", C.c_int32), ("n_types", C.c_int32),
                ("launch_mode", C.c_int32), ("reserved", C.c_int32)]


class md_stats_t(C.Structure):
    _fields_ = [("steps", C.c_int64), ("rebuilds", C.c_int64), ("list_entries", C.c_int64),
                ("max_list", C.c_int32), ("max_cell", C.c_int32), ("status_bits", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None

EXPORTED = [
    "md_workspace_size", "md_workspace_bytes", "md_init", "md_init_batch", "md_create",
    "md_set_state", "md_build_neighbors", "md_step", "md_prepare",
    "md_energy", "md_get_state", "md_compute_forces", "md_stats", "md_get_cells",
    "md_get_neighbors", "md_launch_pass", "md_set_schedule", "md_set_replica_schedule",
    "md_get_replica_schedule", "md_autotune", "md_last_error",
    "md_status_string", "md_destroy", "md_create_multi", "md_set_types",
    "md_fm_workspace_size", "md_fm_create", "md_fm_forward", "md_fm_backward", "md_fm_destroy",
    "md_fm_forward_async", "md_fm_backward_async", "md_fm_check",
    "md_forces_static",
]


def lib():
    """Load the in-tree library; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        P, vp = C.POINTER, C.c_void_p
        i32, i64, d, sz = C.c_int32, C.c_int64, C.c_double, C.c_size_t
        sig = {
            "md_workspace_size": (i32, [P(md_params), i32, P(i64), P(d), P(sz)]),
            "md_workspace_bytes": (sz, [P(md_params), i32, P(i64), P(d)]),
            "md_init": (i32, [P(vp), P(md_params), i64, P(d), P(md_spline), P(md_spline),
                              P(md_spline), vp, vp, vp, sz, vp]),
            "md_init_batch": (i32, [P(vp), P(md_params), i32, P(i64), P(d), P(md_spline),
                                    P(md_spline), P(md_spline), vp, vp, vp, sz, vp]),
            "md_create": (i32, [P(vp), P(md_params), i32, P(i64), P(d), P(md_spline),
                                P(md_spline), P(md_spline), vp, sz, vp]),
            "md_create_multi": (i32, [P(vp), P(md_params), i32, P(i64), P(d), P(md_spline),
                                      P(md_spline), P(md_spline), P(d), vp, sz, vp]),
            "md_set_types": (i32, [vp, vp]),
            "md_set_state": (i32, [vp, vp, vp]),
            "md_build_neighbors": (i32, [vp]),
            "md_step": (i32, [vp, i64]),
            "md_prepare": (i32, [vp, i64]),
            "md_energy": (i32, [vp, P(d), P(d)]),
            "md_get_state": (i32, [vp, vp, vp, vp]),
            "md_compute_forces": (i32, [vp, vp, vp, vp]),
            "md_stats": (i32, [vp, P(md_stats_t)]),
            "md_get_cells": (i32, [vp, vp]),
            "md_get_neighbors": (i32, [vp, vp, vp, i32]),
            "md_launch_pass": (i32, [vp, i32, i32]),
            "md_set_schedule": (i32, [vp, i32]),
            "md_set_replica_schedule": (i32, [vp, P(i32)]),
            "md_get_replica_schedule": (i32, [vp, P(i32)]),
            "md_autotune": (i32, [vp, i32, P(i32), P(C.c_float)]),
            "md_last_error": (C.c_char_p, [vp]),
            "md_status_string": (C.c_char_p, [i32]),
            "md_destroy": (None, [vp]),
            "md_fm_workspace_size": (i32, [i32, P(i64), P(d), d, i32, P(i32), P(sz)]),
            "md_fm_create": (i32, [P(vp), i32, P(i64), P(d), d, i32, P(md_spline), P(md_spline),
                                   P(md_spline), vp, vp, vp, sz, vp]),
            "md_fm_forward": (i32, [vp, vp, vp, vp, P(d), vp]),
            "md_fm_backward": (i32, [vp, d, vp, vp, vp]),
            "md_fm_forward_async": (i32, [vp, vp, vp, vp, vp, vp]),
            "md_fm_backward_async": (i32, [vp, vp, vp, vp, vp]),
            "md_fm_check": (i32, [vp]),
            "md_fm_destroy": (None, [vp]),
            "md_forces_static": (i32, [P(md_params), i64, P(d), P(md_spline), P(md_spline),
                                       P(md_spline), vp, vp, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().md_status_string(int(code)).decode()
    except ImportError:
        return "library not loaded"


def _check(code: int, where: str, ctx=None) -> int:
    if code < 0:
        detail = ""
        if code == MD_E_HIP:
            detail = lib().md_last_error(ctx).decode()
        raise MDError(code, where, detail)
    return code


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _stream_handle(stream) -> int:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Spline:
    """Keeps a host coefficient array alive next to its md_spline struct."""

    def __init__(self, table):
        self.coef = np.ascontiguousarray(table.coef, dtype=np.float64)
        self.s = md_spline(self.coef.shape[0] + 1, 0, float(table.x0), float(1.0 / table.dx),
                           self.coef.ctypes.data_as(C.POINTER(C.c_double)))


def make_params(*, mass, dt, r_cut, skin, ftm2v, kboltz=8.617333262e-5, precision=MD_FP64,
                nbr_capacity=128, cell_capacity=64, chunk_steps=100, lanes_per_atom=0,
                sort_every=1, list_mode=0, n_types=0, launch_mode=0) -> md_params:
    return md_params(mass, dt, r_cut, skin, ftm2v, kboltz, precision, nbr_capacity, cell_capacity,
                     chunk_steps, lanes_per_atom, sort_every, list_mode, n_types, launch_mode, 0)


class System:
    """One context: n_rep boxes advanced together on one GPU.

    A box length L > 0 makes that dimension periodic; L < 0 makes it open
    with a cell grid of extent |L|.

    x, v: (N, 3) float64 (numpy or torch); boxes: (n_rep, 3); rep_atoms: (n_rep,).
    tables: (phi, rho, F) for one species; with params.n_types = T > 1,
    (phi[a][b], rho[t], F[t]) and `masses` (T,) for the multi-species form.
    Device memory (workspace, state staging) is allocated through torch.
    """

    def __init__(self, params: md_params, tables: Sequence, rep_atoms, boxes, *, stream=None,
                 device="cuda", masses=None):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.params = params
        self.rep_atoms = np.ascontiguousarray(rep_atoms, dtype=np.int64).ravel()
        self.boxes = np.ascontiguousarray(boxes, dtype=np.float64).reshape(-1, 3)
        self.n_rep = int(self.rep_atoms.size)
        self.n = int(self.rep_atoms.sum())
        nt = int(params.n_types)
        if nt > 1:
            phi, rho, emb = tables
            flat = [phi[a][b] for a in range(nt) for b in range(nt)]
            self.multi = [(md_spline * len(ts))() for ts in (flat, rho, emb)]
            self.splines = []
            for arr, ts in zip(self.multi, (flat, rho, emb)):
                for k, tab in enumerate(ts):
                    sp = Spline(tab)
                    self.splines.append(sp)
                    arr[k] = sp.s
            self.masses = np.ascontiguousarray(masses, dtype=np.float64)
            assert self.masses.shape == (nt,)
        else:
            self.splines = [Spline(t) for t in tables]
        # a stream of its own (default priority): graphs cannot be captured on the
        # legacy default stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        L = lib()
        nbytes = C.c_size_t()
        _check(L.md_workspace_size(C.byref(params), self.n_rep,
                                   self.rep_atoms.ctypes.data_as(C.POINTER(C.c_int64)),
                                   self.boxes.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(nbytes)), "md_workspace_size")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        if nt > 1:
            sp = C.POINTER(md_spline)
            _check(L.md_create_multi(C.byref(ctx), C.byref(params), self.n_rep,
                                     self.rep_atoms.ctypes.data_as(C.POINTER(C.c_int64)),
                                     self.boxes.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.cast(self.multi[0], sp), C.cast(self.multi[1], sp),
                                     C.cast(self.multi[2], sp),
                                     self.masses.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.c_void_p(self.workspace.data_ptr()), nbytes.value,
                                     C.c_void_p(self.stream.cuda_stream)), "md_create_multi")
        else:
            _check(L.md_create(C.byref(ctx), C.byref(params), self.n_rep,
                               self.rep_atoms.ctypes.data_as(C.POINTER(C.c_int64)),
                               self.boxes.ctypes.data_as(C.POINTER(C.c_double)),
                               C.byref(self.splines[0].s), C.byref(self.splines[1].s),
                               C.byref(self.splines[2].s), C.c_void_p(self.workspace.data_ptr()),
                               nbytes.value, C.c_void_p(self.stream.cuda_stream)), "md_create")
        self.ctx = ctx

    # -- lifecycle -----------------------------------------------------------
    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.float64).contiguous()
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    def set_state(self, x, v):
        xd, vd = self._dev(x).reshape(self.n, 3), self._dev(v).reshape(self.n, 3)
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        rc = lib().md_set_state(self.ctx, C.c_void_p(xd.data_ptr()), C.c_void_p(vd.data_ptr()))
        return _check(rc, "md_set_state", self.ctx)

    def set_types(self, types):
        """Atom types (original order, int32 in [0, n_types)); md_build_neighbors must follow."""
        t = self.torch
        td = t.as_tensor(np.ascontiguousarray(types, dtype=np.int32), device=self.device)
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        rc = lib().md_set_types(self.ctx, C.c_void_p(td.data_ptr()))
        self.stream.synchronize()
        return _check(rc, "md_set_types", self.ctx)

    def build_neighbors(self):
        return _check(lib().md_build_neighbors(self.ctx), "md_build_neighbors", self.ctx)

    def step(self, n: int, check: bool = True):
        rc = lib().md_step(self.ctx, int(n))
        return _check(rc, "md_step", self.ctx) if check else rc

    def prepare(self, n: int):
        """Capture the graphs step(n) will launch, so that step(n) only launches them."""
        return _check(lib().md_prepare(self.ctx, int(n)), "md_prepare", self.ctx)

    def energy(self):
        pe = np.zeros(self.n_rep)
        ke = np.zeros(self.n_rep)
        _check(lib().md_energy(self.ctx, pe.ctypes.data_as(C.POINTER(C.c_double)),
                               ke.ctypes.data_as(C.POINTER(C.c_double))), "md_energy", self.ctx)
        return pe, ke

    def get_state(self, want_f: bool = True):
        t = self.torch
        x = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        v = t.empty_like(x)
        f = t.empty_like(x) if want_f else None
        _check(lib().md_get_state(self.ctx, C.c_void_p(x.data_ptr()), C.c_void_p(v.data_ptr()),
                                  C.c_void_p(_ptr(f)) if f is not None else None),
               "md_get_state", self.ctx)
        return x, v, f

    def compute_forces(self):
        t = self.torch
        f = t.empty((self.n, 3), dtype=t.float64, device=self.device)
        rho = t.empty(self.n, dtype=t.float64, device=self.device)
        fp = t.empty_like(rho)
        rc = lib().md_compute_forces(self.ctx, C.c_void_p(f.data_ptr()), C.c_void_p(rho.data_ptr()),
                                     C.c_void_p(fp.data_ptr()))
        _check(rc, "md_compute_forces", self.ctx)
        return f, rho, fp

    def stats(self) -> dict:
        st = md_stats_t()
        _check(lib().md_stats(self.ctx, C.byref(st)), "md_stats", self.ctx)
        return dict(steps=st.steps, rebuilds=st.rebuilds, list_entries=st.list_entries,
                    max_list=st.max_list, max_cell=st.max_cell, status_bits=st.status_bits)

    def cells(self):
        t = self.torch
        c = t.empty(self.n, dtype=t.int32, device=self.device)
        _check(lib().md_get_cells(self.ctx, C.c_void_p(c.data_ptr())), "md_get_cells", self.ctx)
        return c

    def neighbors(self, cap_out: int = 128):
        t = self.torch
        cnt = t.empty(self.n, dtype=t.int32, device=self.device)
        nbr = t.empty((self.n, cap_out), dtype=t.int32, device=self.device)
        _check(lib().md_get_neighbors(self.ctx, C.c_void_p(cnt.data_ptr()),
                                      C.c_void_p(nbr.data_ptr()), int(cap_out)),
               "md_get_neighbors", self.ctx)
        return cnt, nbr

    def launch_pass(self, which: int, reps: int):
        return _check(lib().md_launch_pass(self.ctx, int(which), int(reps)), "md_launch_pass",
                      self.ctx)

    def set_schedule(self, lanes_per_atom: int):
        return _check(lib().md_set_schedule(self.ctx, int(lanes_per_atom)), "md_set_schedule",
                      self.ctx)

    def set_replica_schedule(self, lanes):
        """Lanes per atom of each replica (n_rep values of 1, 2, 4 or 8)."""
        a = np.ascontiguousarray(lanes, dtype=np.int32)
        assert a.shape == (self.n_rep,)
        return _check(lib().md_set_replica_schedule(self.ctx, a.ctypes.data_as(C.POINTER(C.c_int32))),
                      "md_set_replica_schedule", self.ctx)

    def replica_schedule(self):
        a = np.zeros(self.n_rep, dtype=np.int32)
        _check(lib().md_get_replica_schedule(self.ctx, a.ctypes.data_as(C.POINTER(C.c_int32))),
               "md_get_replica_schedule", self.ctx)
        return a

    def autotune(self, reps: int = 20):
        lpa = C.c_int32()
        us = C.c_float()
        _check(lib().md_autotune(self.ctx, int(reps), C.byref(lpa), C.byref(us)), "md_autotune",
               self.ctx)
        return int(lpa.value), float(us.value)

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            lib().md_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
