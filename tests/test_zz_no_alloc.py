"""spfas_eval_residual_noalloc (GPU): the residual entry point that stages
its work in a static device array instead of allocating, called through the
C ABI twice in a row -- a 40x32 problem, then a smaller 12x8 one that reuses
the same array -- and compared with spfas_eval_residual on the same inputs
(same kernels and summation order: identical bits)."""
import ctypes as C

import numpy as np
import pytest

from problems import small_problem

pytestmark = pytest.mark.gpu


def _device_inputs(H, prob, seed):
    import torch
    rng = np.random.default_rng(seed)
    p = torch.tensor(0.3 * rng.standard_normal(H.n_cells), dtype=torch.float64, device="cuda")
    s = torch.tensor(rng.standard_normal(H.n_faces), dtype=torch.float64, device="cuda")
    return p, s


def test_noalloc_residual_matches_eval_residual():
    import torch
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    L = pk.lib()
    cases = []
    for shape, seed in (((40, 32), 1), ((12, 8), 2)):
        print("case", shape, flush=True)
        prob = small_problem(shape, seed=seed, box=(4, 4), m=2, n_levels=2, g_d_scale=0.3, g_n_scale=0.2,
                             permute=True)
        H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
        cp, keep = H._problem(prob, device=True)
        p, s = _device_inputs(H, prob, seed)
        rp_ref = torch.empty(H.n_cells, dtype=torch.float64, device="cuda")
        rs_ref = torch.empty(H.n_faces, dtype=torch.float64, device="cuda")
        H.eval_residual_device(cp, p, s, rp_ref, rs_ref)
        torch.cuda.synchronize()
        cases.append((prob, H, cp, keep, p, s, rp_ref, rs_ref))
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    # two calls in a row, the second on the smaller problem
    outs = []
    for prob, H, cp, keep, p, s, _, _ in cases:
        rp = torch.full((H.n_cells,), float("nan"), dtype=torch.float64, device="cuda")
        rs = torch.full((H.n_faces,), float("nan"), dtype=torch.float64, device="cuda")
        N.check(L.spfas_eval_residual_noalloc(H.h, C.byref(cp), p.data_ptr(), s.data_ptr(), rp.data_ptr(),
                                              rs.data_ptr(), stream))
        outs.append((rp, rs))
    torch.cuda.synchronize()
    for (prob, H, cp, keep, p, s, rp_ref, rs_ref), (rp, rs) in zip(cases, outs):
        assert torch.equal(rp, rp_ref) and torch.equal(rs, rs_ref)
        # Neumann faces carry no flux unknown: their residual entries are zero
        nm = torch.as_tensor(prob.mesh.face_bc == 2, device="cuda")
        assert bool(torch.all(rs[nm] == 0.0))
        # and the values are the oracle's fine residual
        from oracle.fv import FineSystem
        fs = FineSystem(prob)
        ff = fs.fm.flux_face
        ref_s, ref_p = fs.residual(s.cpu().numpy()[ff], p.cpu().numpy())
        np.testing.assert_allclose(rp.cpu().numpy(), ref_p, rtol=1e-13, atol=1e-14 * np.abs(ref_p).max())
        np.testing.assert_allclose(rs.cpu().numpy()[ff], ref_s, rtol=1e-13, atol=1e-14 * np.abs(ref_s).max())


def test_noalloc_rejects_host_problem_data():
    import torch
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    L = pk.lib()
    prob = small_problem((8, 8), seed=3, box=(4, 4), m=2, n_levels=2)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    cp, keep = H._problem(prob, device=False)
    p = torch.zeros(H.n_cells, dtype=torch.float64, device="cuda")
    s = torch.zeros(H.n_faces, dtype=torch.float64, device="cuda")
    rc = L.spfas_eval_residual_noalloc(H.h, C.byref(cp), p.data_ptr(), s.data_ptr(), p.data_ptr(), s.data_ptr(),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == N.SPFAS_ERR_INVALID
    assert b"device memory" in L.spfas_last_error()


def test_noalloc_rejects_a_kappa_shift():
    """A shift of the kappa argument would need a device buffer of its own:
    the no-allocation entry point refuses it before any work."""
    import dataclasses
    import torch
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    L = pk.lib()
    base = small_problem((8, 8), seed=3, box=(4, 4), m=2, n_levels=2)
    prob = dataclasses.replace(base, shift=np.linspace(0.0, 1.0, base.mesh.n_cells))
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    cp, keep = H._problem(prob, device=True)
    p = torch.zeros(H.n_cells, dtype=torch.float64, device="cuda")
    s = torch.zeros(H.n_faces, dtype=torch.float64, device="cuda")
    rc = L.spfas_eval_residual_noalloc(H.h, C.byref(cp), p.data_ptr(), s.data_ptr(), p.data_ptr(), s.data_ptr(),
                                       C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == N.SPFAS_ERR_INVALID
    assert b"shift" in L.spfas_last_error()
