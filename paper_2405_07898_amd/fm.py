"""Force matching on the GPU: loss, adjoint, and a torch autograd wrapper.

The loss is L = sum over configurations and atoms of |F_i - Fref_i|^2 with
forces from the EAM force expression (paper Sec. II-A, Eq. EAMforce); its
gradient with respect to the per-segment cubic coefficients of phi, rho and
F comes from the hand-written adjoint kernels in libmdeam.so
(md_fm_forward / md_fm_backward).
"""
from __future__ import annotations

import ctypes as C
from typing import Sequence

import numpy as np

from . import md as _md


class ForceMatch:
    """Static configurations (concatenated (N, 3) positions, per-config boxes)
    and reference forces; coefficient grids fixed by `grid_tables`."""

    def __init__(self, x, fref, cfg_atoms, cfg_boxes, grid_tables: Sequence, *, r_cut=5.0,
                 nbr_capacity=128, stream=None, device="cuda"):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        L = _md.lib()
        self.cfg_atoms = np.ascontiguousarray(cfg_atoms, dtype=np.int64).ravel()
        self.cfg_boxes = np.ascontiguousarray(cfg_boxes, dtype=np.float64).reshape(-1, 3)
        self.n_cfg = int(self.cfg_atoms.size)
        self.n = int(self.cfg_atoms.sum())
        self.grids = [_md.Spline(t) for t in grid_tables]
        self.shapes = [s.coef.shape for s in self.grids]
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        nk = (C.c_int32 * 3)(*[s.coef.shape[0] + 1 for s in self.grids])
        nbytes = C.c_size_t()
        pa = self.cfg_atoms.ctypes.data_as(C.POINTER(C.c_int64))
        pb = self.cfg_boxes.ctypes.data_as(C.POINTER(C.c_double))
        _md._check(L.md_fm_workspace_size(self.n_cfg, pa, pb, float(r_cut), int(nbr_capacity), nk,
                                          C.byref(nbytes)), "md_fm_workspace_size")
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        xd = self._dev(x).reshape(self.n, 3)
        fd = self._dev(fref).reshape(self.n, 3)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        ctx = C.c_void_p()
        _md._check(L.md_fm_create(C.byref(ctx), self.n_cfg, pa, pb, float(r_cut), int(nbr_capacity),
                                  C.byref(self.grids[0].s), C.byref(self.grids[1].s),
                                  C.byref(self.grids[2].s), C.c_void_p(xd.data_ptr()),
                                  C.c_void_p(fd.data_ptr()), C.c_void_p(self.workspace.data_ptr()),
                                  nbytes.value, C.c_void_p(self.stream.cuda_stream)),
                   "md_fm_create")
        self.ctx = ctx
        self._last = None

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device=self.device, dtype=t.float64).contiguous()
        return t.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=self.device)

    def forward(self, coef_phi, coef_rho, coef_emb, want_forces: bool = False):
        cs = [self._dev(c).contiguous() for c in (coef_phi, coef_rho, coef_emb)]
        for c, shp in zip(cs, self.shapes):
            if tuple(c.shape) != tuple(shp):
                raise ValueError(f"coefficient shape {tuple(c.shape)} != {tuple(shp)}")
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        f = self.torch.empty((self.n, 3), dtype=self.torch.float64, device=self.device) \
            if want_forces else None
        loss = C.c_double()
        rc = _md.lib().md_fm_forward(self.ctx, *[C.c_void_p(c.data_ptr()) for c in cs],
                                     C.byref(loss), C.c_void_p(f.data_ptr()) if f is not None else None)
        _md._check(rc, "md_fm_forward")
        self._last = cs  # keeps the coefficients alive for the backward pass
        return loss.value, f

    def backward(self, seed: float = 1.0):
        t = self.torch
        gs = [t.empty(shp, dtype=t.float64, device=self.device) for shp in self.shapes]
        rc = _md.lib().md_fm_backward(self.ctx, float(seed), *[C.c_void_p(g.data_ptr()) for g in gs])
        _md._check(rc, "md_fm_backward")
        return gs

    def forward_async(self, coef_phi, coef_rho, coef_emb, want_forces: bool = False):
        """The loss as a device tensor, with no host synchronisation; errors stay
        latched until check()."""
        t = self.torch
        cs = [self._dev(c).contiguous() for c in (coef_phi, coef_rho, coef_emb)]
        for c, shp in zip(cs, self.shapes):
            if tuple(c.shape) != tuple(shp):
                raise ValueError(f"coefficient shape {tuple(c.shape)} != {tuple(shp)}")
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        f = t.empty((self.n, 3), dtype=t.float64, device=self.device) if want_forces else None
        loss = t.empty((), dtype=t.float64, device=self.device)
        _md._check(_md.lib().md_fm_forward_async(
            self.ctx, *[C.c_void_p(c.data_ptr()) for c in cs], C.c_void_p(loss.data_ptr()),
            C.c_void_p(f.data_ptr()) if f is not None else None), "md_fm_forward_async")
        self._last = cs
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return loss, f

    def backward_async(self, seed):
        """Gradients for the last forward, scaled by the device scalar `seed`,
        with no host synchronisation."""
        t = self.torch
        seed = self._dev(seed).reshape(())
        self.stream.wait_stream(t.cuda.current_stream(self.device))
        gs = [t.empty(shp, dtype=t.float64, device=self.device) for shp in self.shapes]
        _md._check(_md.lib().md_fm_backward_async(self.ctx, C.c_void_p(seed.data_ptr()),
                                                  *[C.c_void_p(g.data_ptr()) for g in gs]),
                   "md_fm_backward_async")
        self._seed = seed  # alive until the stream has read it
        t.cuda.current_stream(self.device).wait_stream(self.stream)
        return gs

    def check(self):
        """Raises if any call since the last check met a non-finite value."""
        _md._check(_md.lib().md_fm_check(self.ctx), "md_fm_check")

    def close(self):
        if getattr(self, "ctx", None):
            self.stream.synchronize()
            _md.lib().md_fm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _autograd():
    import torch

    class EamForceMatch(torch.autograd.Function):
        """loss = EamForceMatch.apply(coef_phi, coef_rho, coef_emb, problem)."""

        @staticmethod
        def forward(ctx, coef_phi, coef_rho, coef_emb, problem):
            # no host synchronisation: the loss stays on the device, and errors
            # stay latched until problem.check()
            loss, _ = problem.forward_async(coef_phi.detach(), coef_rho.detach(),
                                            coef_emb.detach())
            ctx.problem = problem
            ctx.coefs = (coef_phi.detach(), coef_rho.detach(), coef_emb.detach())
            return loss

        @staticmethod
        def backward(ctx, grad_loss):
            p = ctx.problem
            # the adjoint needs the forward state of these coefficients
            if p._last is None or any(a.data_ptr() != b.data_ptr() for a, b in zip(p._last, ctx.coefs)):
                p.forward_async(*ctx.coefs)
            g = p.backward_async(grad_loss.detach())
            return g[0], g[1], g[2], None

    return EamForceMatch


_EFM = None


def eam_force_match(coef_phi, coef_rho, coef_emb, problem: ForceMatch):
    """Differentiable force-matching loss (torch autograd)."""
    global _EFM
    if _EFM is None:
        _EFM = _autograd()
    return _EFM.apply(coef_phi, coef_rho, coef_emb, problem)
