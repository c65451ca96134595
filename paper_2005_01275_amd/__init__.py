"""spfas: nonlinear spectral multigrid (FAS) for heterogeneous nonlinear
diffusion on MI355X.

Python side of the C ABI in include/spfas.h.  ``Hierarchy`` wraps a handle;
arrays are marshalled from numpy (host) or torch tensors (device).  PyTorch
is used for device memory and streams only; all arithmetic runs in the HIP
library, which must be built (``paper_2005_01275_amd/build.py``).
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Optional

import numpy as np

from . import _native as N
from ._native import (SPFAS_OK, SPFAS_NOT_CONVERGED, SPFAS_MEM_HOST, SPFAS_MEM_DEVICE, SPFAS_NEWTON,
                      SPFAS_PICARD, SPFAS_PREC_FP64, SPFAS_PREC_MIXED, SpfasError)

__all__ = ["Hierarchy", "SolveOpts", "SpfasError", "SPFAS_NEWTON", "SPFAS_PICARD", "lib"]


def lib():
    return N.lib()


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclasses.dataclass
class SolveOpts:
    smoother: int = SPFAS_NEWTON
    rtol: float = 1e-8
    atol: float = 1e-10
    max_it: int = 50
    bt_nmax: int = 4
    bt_theta: float = 0.9
    dp_cap: float = 0.0
    coarsest_max_steps: int = 10
    lin_rtol: float = 1e-8
    lin_max_it: int = 500
    x0_given: int = 0
    lin_rtol_coarse: float = 0.0
    lin_target: float = 0.0
    newton_pcg: int = 0
    amg_reuse: int = 0
    lin_max_it_coarse: int = 0
    coarsest_atol: float = -1.0
    precision: int = N.SPFAS_PREC_FP64

    def c(self):
        o = N.spfas_solve_opts()
        for f in dataclasses.fields(self):
            setattr(o, f.name, getattr(self, f.name))
        return o


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except Exception:
            pass
        return C.c_void_p(0)
    return C.c_void_p(int(stream))


def _mesh_struct(mesh):
    """spfas_mesh over contiguous copies of a ``problems.Mesh`` (the copies
    are returned to keep them alive)."""
    cen = np.ascontiguousarray(mesh.cell_centroid, dtype=np.float64)
    k0 = np.ascontiguousarray(mesh.cell_k0, dtype=np.float64)
    vol = np.ascontiguousarray(mesh.cell_volume, dtype=np.float64)
    fc = np.ascontiguousarray(mesh.face_cells, dtype=np.int32)
    area = np.ascontiguousarray(mesh.face_area, dtype=np.float64)
    nrm = np.ascontiguousarray(mesh.face_normal, dtype=np.float64)
    pt = np.ascontiguousarray(mesh.face_point, dtype=np.float64)
    kind = np.ascontiguousarray(mesh.face_bc, dtype=np.int8)
    ms = N.spfas_mesh(dim=mesh.dim, n_cells=vol.size, n_faces=area.size, cell_volume=_dptr(vol),
                      cell_centroid=_dptr(cen), cell_k0=_dptr(k0),
                      face_cells=fc.ctypes.data_as(C.POINTER(C.c_int32)), face_area=_dptr(area),
                      face_normal=_dptr(nrm), face_point=_dptr(pt),
                      face_kind=kind.ctypes.data_as(C.POINTER(C.c_int8)))
    return ms, (cen, k0, vol, fc, area, nrm, pt, kind)


class Hierarchy:
    """Owns an spfas_hierarchy built from a mesh with the fields of
    ``problems.Mesh`` (numpy host arrays)."""

    def __init__(self, mesh, n_levels: int, box=(), m: int = 1, host_only: bool = False, stream=None,
                 agg_kind: int = N.SPFAS_AGG_BOX, user_agg=None, greedy_size: int = 0, allocator=None,
                 eig_threshold: float = 0.0, m_min: int = 2, m_f: int = 1, greedy_size_coarse: int = 0):
        """allocator: None (hipMalloc) or "torch" (PyTorch's caching
        allocator owns the hierarchy's device memory).  user_agg: for
        agg_kind USER, the aggregation of every coarsened level,
        concatenated.  eig_threshold > 0: eigenvectors per aggregate by the
        eigenvalue threshold, between m_min and m.  greedy_size_coarse:
        the greedy target on levels 1 and up (0: greedy_size)."""
        L = N.lib()
        self._keep = []
        ms, arrays = _mesh_struct(mesh)
        vol, area = arrays[2], arrays[4]
        box = tuple(box) + (1,) * (3 - len(box))
        ua = None
        if user_agg is not None:
            ua = np.ascontiguousarray(user_agg, dtype=np.int32)
            self._keep.append(ua)
        op = N.spfas_coarsen_opts(n_levels=n_levels, box=(C.c_int32 * 3)(*box), m=m, host_only=int(host_only),
                                  agg_kind=agg_kind,
                                  user_agg=ua.ctypes.data_as(C.POINTER(C.c_int32)) if ua is not None else None,
                                  user_agg_len=0 if ua is None else ua.size, greedy_size=greedy_size,
                                  eig_threshold=float(eig_threshold), m_min=int(m_min), m_f=int(m_f),
                                  greedy_size_coarse=int(greedy_size_coarse))
        if allocator not in (None, "torch"):
            raise ValueError("allocator must be None or 'torch'")
        alloc = C.byref(N.TORCH_ALLOCATOR) if allocator == "torch" else None
        h = C.c_void_p()
        N.check(L.spfas_setup_hierarchy(C.byref(ms), C.byref(op), alloc, _stream_handle(stream) if not host_only
                                        else C.c_void_p(0), C.byref(h)))
        self.h = h
        self.n_cells = vol.size
        self.n_faces = area.size
        self.n_levels = n_levels
        self.host_only = host_only

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            N.lib().spfas_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- problem
    @staticmethod
    def _problem(prob, device: bool):
        """spfas_problem for a ``problems.Problem``; device=True passes
        torch CUDA tensors (kept alive by the returned tuple)."""
        kind = N.KAPPA_KINDS[getattr(prob, "kappa_kind", "exp")]
        ka, kb = float(getattr(prob, "kappa_a", 1.0)), float(getattr(prob, "kappa_beta", 2.0))
        shift = getattr(prob, "shift", None)
        if device:
            import torch
            src = torch.as_tensor(prob.source, dtype=torch.float64, device="cuda")
            gd = torch.as_tensor(prob.g_dirichlet, dtype=torch.float64, device="cuda")
            gn = torch.as_tensor(prob.g_neumann, dtype=torch.float64, device="cuda")
            sh = None if shift is None else torch.as_tensor(shift, dtype=torch.float64, device="cuda")
            cp = N.spfas_problem(alpha=prob.alpha, source=src.data_ptr(), g_dirichlet=gd.data_ptr(),
                                 g_neumann=gn.data_ptr(), mem=SPFAS_MEM_DEVICE, kappa_kind=kind, kappa_a=ka,
                                 kappa_beta=kb, shift=None if sh is None else sh.data_ptr())
            return cp, (src, gd, gn, sh)
        src = np.ascontiguousarray(prob.source, dtype=np.float64)
        gd = np.ascontiguousarray(prob.g_dirichlet, dtype=np.float64)
        gn = np.ascontiguousarray(prob.g_neumann, dtype=np.float64)
        sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
        cp = N.spfas_problem(alpha=prob.alpha, source=src.ctypes.data, g_dirichlet=gd.ctypes.data,
                             g_neumann=gn.ctypes.data, mem=SPFAS_MEM_HOST, kappa_kind=kind, kappa_a=ka,
                             kappa_beta=kb, shift=None if sh is None else sh.ctypes.data)
        return cp, (src, gd, gn, sh)

    def eval_residual(self, prob, p, sigma):
        """Fine residual at host arrays (p [n_cells], sigma [n_faces])."""
        cp, keep = self._problem(prob, device=False)
        p = np.ascontiguousarray(p, dtype=np.float64)
        s = np.ascontiguousarray(sigma, dtype=np.float64)
        rp = np.zeros(self.n_cells)
        rs = np.zeros(self.n_faces)
        N.check(N.lib().spfas_eval_residual(self.h, C.byref(cp), p.ctypes.data, s.ctypes.data, rp.ctypes.data,
                                            rs.ctypes.data, SPFAS_MEM_HOST, _stream_handle(None)))
        return rp, rs

    def eval_residual_device(self, cprob, p, sigma, rp, rs, stream=None):
        """Device variant on torch tensors (all float64, CUDA)."""
        N.check(N.lib().spfas_eval_residual(self.h, C.byref(cprob), p.data_ptr(), sigma.data_ptr(),
                                            rp.data_ptr(), rs.data_ptr(), SPFAS_MEM_DEVICE,
                                            _stream_handle(stream)))

    # ---------------------------------------------------------------- solves
    def _solve(self, fn, prob, opts: SolveOpts, p0=None, sigma0=None, device=False, cprob=None, stream=None,
               out=None, extra=()):
        L = N.lib()
        st = N.spfas_stats()
        o = opts.c()
        if device:
            import torch
            if cprob is None:
                cprob, keep = self._problem(prob, device=True)
            if out is None:
                p = torch.zeros(self.n_cells, dtype=torch.float64, device="cuda")
                s = torch.zeros(self.n_faces, dtype=torch.float64, device="cuda")
            else:
                p, s = out
            if p0 is not None:
                p.copy_(torch.as_tensor(p0, dtype=torch.float64))
                s.copy_(torch.as_tensor(sigma0, dtype=torch.float64))
                o.x0_given = 1
            rc = getattr(L, fn)(self.h, C.byref(cprob), C.byref(o), p.data_ptr(), s.data_ptr(), SPFAS_MEM_DEVICE,
                                C.byref(st), *extra, _stream_handle(stream))
        else:
            cprob, keep = self._problem(prob, device=False)
            p = np.zeros(self.n_cells) if p0 is None else np.array(p0, dtype=np.float64)
            s = np.zeros(self.n_faces) if sigma0 is None else np.array(sigma0, dtype=np.float64)
            if p0 is not None:
                o.x0_given = 1
            rc = getattr(L, fn)(self.h, C.byref(cprob), C.byref(o), p.ctypes.data, s.ctypes.data, SPFAS_MEM_HOST,
                                C.byref(st), *extra, _stream_handle(stream))
        N.check(rc)
        stats = {f: getattr(st, f) for f, _ in N.spfas_stats._fields_}
        stats["converged"] = rc == SPFAS_OK
        return p, s, stats

    def fas_solve(self, prob, opts: SolveOpts, **kw):
        return self._solve("spfas_fas_solve", prob, opts, **kw)

    def picard_solve(self, prob, opts: SolveOpts, **kw):
        return self._solve("spfas_picard_solve", prob, opts, **kw)

    def newton_solve(self, prob, opts: SolveOpts, **kw):
        return self._solve("spfas_newton_solve", prob, opts, **kw)

    def cascadic_solve(self, prob, opts: SolveOpts, **kw):
        """Nonlinear cascadic multigrid (spfas_cascadic_solve); starts from
        zero, so p0/sigma0 are not accepted.  stats["level_steps"] lists the
        smoothing steps per level, finest first."""
        if kw.get("p0") is not None or kw.get("sigma0") is not None:
            raise ValueError("the cascadic solve starts from zero on the coarsest level")
        steps = (C.c_int32 * self.n_levels)()
        p, s, stats = self._solve("spfas_cascadic_solve", prob, opts, extra=(steps,), **kw)
        stats["level_steps"] = list(steps)
        return p, s, stats

    # ---------------------------------------------------------------- parity hooks
    def level_sizes(self, level):
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        N.check(N.lib().spfas_level_sizes(self.h, level, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def aggregation(self, level):
        n, _, _ = self.level_sizes(level)
        out = np.zeros(n, dtype=np.int32)
        N.check(N.lib().spfas_get_aggregation(self.h, level, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def permutation(self, level):
        n, _, nf = self.level_sizes(level)
        co = np.zeros(n, dtype=np.int32)
        fo = np.zeros(nf, dtype=np.int32)
        N.check(N.lib().spfas_get_permutation(self.h, level, co.ctypes.data_as(C.POINTER(C.c_int32)),
                                              fo.ctypes.data_as(C.POINTER(C.c_int32))))
        return co, fo

    def profile_enable(self, on=True):
        N.check(N.lib().spfas_profile_enable(self.h, int(on)))

    def profile_read(self):
        """{kernel name: (launches, total ms, algorithmic bytes)}"""
        out = {}
        for k, name in N.PROF_NAMES.items():
            a, b, c = C.c_int64(), C.c_double(), C.c_double()
            N.check(N.lib().spfas_profile_read(self.h, k, C.byref(a), C.byref(b), C.byref(c)))
            out[name] = (a.value, b.value, c.value)
        return out

    def device_bytes(self):
        """(bytes held now, peak) of the hierarchy's device memory."""
        a, b = C.c_int64(), C.c_int64()
        N.check(N.lib().spfas_hierarchy_device_bytes(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def level_operator(self, level, what, count):
        out = np.zeros(count)
        N.check(N.lib().spfas_get_level_operator(self.h, level, what, _dptr(out), count))
        return out
