"""Python side of the library's serving runtime (spfas_server_* in
include/spfas.h): continuous batching of solve requests with a cache of
device-resident hierarchies and admission by device-memory footprint.
Argument marshalling only; the queue, the workers and the cache are native."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _native as N
from . import _mesh_struct, SolveOpts

FAS, NEWTON, PICARD = N.SPFAS_SOLVE_FAS, N.SPFAS_SOLVE_NEWTON, N.SPFAS_SOLVE_PICARD


class ServerError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"spfas server error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc < 0:
        raise ServerError(rc, N.lib().spfas_server_last_error().decode())
    return rc


class Server:
    """n_slots solves in flight, each on its own worker thread and HIP
    stream; hbm_budget bytes for cached hierarchies (0: 80% of free)."""

    def __init__(self, n_slots: int = 4, hbm_budget: int = 0, device: int = 0):
        self._L = N.lib()
        o = N.spfas_server_opts(n_slots=n_slots, hbm_budget=hbm_budget, device=device)
        s = C.c_void_p()
        _check(self._L.spfas_server_create(C.byref(o), C.byref(s)))
        self.s = s
        self.n_slots = n_slots
        self._models = {}
        self._pending = {}

    def add_model(self, mesh, n_levels, box=(), m=1, agg_kind=N.SPFAS_AGG_BOX, greedy_size=0, user_agg=None,
                  greedy_size_coarse=0):
        ms, keep = _mesh_struct(mesh)
        ua = None if user_agg is None else np.ascontiguousarray(user_agg, dtype=np.int32)
        box = tuple(box) + (1,) * (3 - len(box))
        co = N.spfas_coarsen_opts(n_levels=n_levels, box=(C.c_int32 * 3)(*box), m=m, host_only=0, agg_kind=agg_kind,
                                  user_agg=ua.ctypes.data_as(C.POINTER(C.c_int32)) if ua is not None else None,
                                  user_agg_len=0 if ua is None else ua.size, greedy_size=greedy_size,
                                  eig_threshold=0.0, m_min=1, greedy_size_coarse=greedy_size_coarse)
        mid = C.c_int64()
        _check(self._L.spfas_server_add_model(self.s, C.byref(ms), C.byref(co), C.byref(mid)))
        self._models[mid.value] = (mesh.n_cells, mesh.n_faces)
        return mid.value

    def submit(self, model_id, prob, opts: SolveOpts, kind=FAS):
        src = np.ascontiguousarray(prob.source, dtype=np.float64)
        gd = np.ascontiguousarray(prob.g_dirichlet, dtype=np.float64)
        gn = np.ascontiguousarray(prob.g_neumann, dtype=np.float64)
        shift = getattr(prob, "shift", None)
        sh = None if shift is None else np.ascontiguousarray(shift, dtype=np.float64)
        cp = N.spfas_problem(alpha=prob.alpha, source=src.ctypes.data, g_dirichlet=gd.ctypes.data,
                             g_neumann=gn.ctypes.data, mem=N.SPFAS_MEM_HOST,
                             kappa_kind=N.KAPPA_KINDS[getattr(prob, "kappa_kind", "exp")],
                             kappa_a=float(getattr(prob, "kappa_a", 1.0)),
                             kappa_beta=float(getattr(prob, "kappa_beta", 2.0)),
                             shift=None if sh is None else sh.ctypes.data)
        o = opts.c()
        t = C.c_int64()
        _check(self._L.spfas_server_submit(self.s, model_id, C.byref(cp), C.byref(o), kind, C.byref(t)))
        self._pending[t.value] = model_id
        return t.value

    def wait(self, ticket):
        """(p, sigma, stats, info) of a ticket; raises ServerError on a
        failed solve."""
        n, nf = self._models[self._pending.pop(ticket)]
        p = np.zeros(n)
        s = np.zeros(nf)
        st = N.spfas_stats()
        info = N.spfas_request_info()
        rc = _check(self._L.spfas_server_wait(self.s, ticket, p.ctypes.data, s.ctypes.data, C.byref(st),
                                              C.byref(info)))
        stats = {f: getattr(st, f) for f, _ in N.spfas_stats._fields_}
        stats["converged"] = rc == N.SPFAS_OK
        inf = {f: getattr(info, f) for f, _ in N.spfas_request_info._fields_}
        return p, s, stats, inf

    def counters(self):
        c = N.spfas_server_counters()
        _check(self._L.spfas_server_counters_get(self.s, C.byref(c)))
        return {f: getattr(c, f) for f, _ in N.spfas_server_counters._fields_}

    def close(self):
        if getattr(self, "s", None) is not None and self.s.value:
            for t in list(self._pending):
                try:
                    self.wait(t)
                except ServerError:
                    pass
            self._L.spfas_server_destroy(self.s)
            self.s = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
