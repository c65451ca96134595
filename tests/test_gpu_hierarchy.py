"""Hierarchy built by the HIP setup kernels against the oracle (GPU):
spectra of the local Laplacians, P_A, P_sigma, Q_sigma, the static coarse
local matrices M^{l+1}_A and D^{l+1}_A (Prop. 1) and the projector weights
(Appendix B), in canonical order.  Eigenvalues agree to 1e-12 of each
aggregate's largest eigenvalue, the other operators element by element to
1e-10 of their largest entry."""
import numpy as np
import pytest

from problems import small_problem, c1_problem
from oracle.coarsen import build_hierarchy

pytestmark = pytest.mark.gpu

CASES = [
    dict(shape=(8, 8), box=(4, 4), m=2, n_levels=2, seed=1),
    dict(shape=(12, 8), box=(4, 4), m=3, n_levels=3, seed=2, g_d_scale=0.3, g_n_scale=0.2,
         dirichlet=((0, 0), (1, 1)), permute=True),
    dict(shape=(6, 4, 4), box=(2, 2, 2), m=3, n_levels=3, seed=3, anisotropic=True, permute=True),
    dict(shape=(9, 7), box=(4, 3), m=2, n_levels=3, seed=4, sigma=1.5),
    # level-1 -> 2 local problems of 64 coarse cells (192 pressure unknowns,
    # interface problems of 384): the blocked dense routines of the setup
    dict(shape=(32, 16, 16), box=(4, 4, 4), m=3, n_levels=3, seed=5, anisotropic=True, permute=True),
    # the largest aggregates the batched workload draws: 8^3 = 512 cells
    # (interface problems over 1,024 cells), and 6^3 / 7^3 boxes with
    # remainder blocks merged into their neighbours
    dict(shape=(16, 16, 16), box=(8, 8, 8), m=3, n_levels=2, seed=6, sigma=2.0, permute=True),
    dict(shape=(16, 13, 9), box=(6, 6, 6), m=3, n_levels=2, seed=7, sigma=2.0),
    dict(shape=(14, 11, 7), box=(7, 7, 7), m=3, n_levels=2, seed=8, sigma=1.5, anisotropic=True),
]


def build_pair(prob):
    import paper_2005_01275_amd as pk
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    h = build_hierarchy(prob)
    return H, h


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kw", CASES + ["c1"])
def test_hierarchy_parity(kw):
    from paper_2005_01275_amd import _native as N
    print("case", kw, flush=True)
    prob = c1_problem() if kw == "c1" else small_problem(**kw)
    H, h = build_pair(prob)
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        assert H.level_sizes(l + 1) == (clev.n_cells, clev.n_p, clev.n_flux)
        # the m_A smallest eigenvalues of every local Laplacian (all the method uses)
        ms = [ad.P.shape[1] for ad in tr.aggs]
        lam = np.concatenate([ad.lam[:m] for ad, m in zip(tr.aggs, ms)])
        g = H.level_operator(l, N.SPFAS_OP_EIGVALS, lam.size)
        for ad, m, seg in zip(tr.aggs, ms, np.split(g, np.cumsum(ms)[:-1])):
            np.testing.assert_allclose(seg, ad.lam[:m], rtol=0.0, atol=1e-12 * max(1e-300, abs(ad.lam[-1])))
        P = np.concatenate([ad.P.ravel() for ad in tr.aggs])
        gP = H.level_operator(l, N.SPFAS_OP_PP, P.size)
        assert rel(gP, P) <= 1e-10, rel(gP, P)
        Ps = tr.P_sig.toarray()
        gPs = H.level_operator(l, N.SPFAS_OP_PSIGMA, Ps.size).reshape(Ps.shape)
        assert rel(gPs, Ps) <= 1e-10, rel(gPs, Ps)
        Qs = tr.Q_sig.toarray()
        gQs = H.level_operator(l, N.SPFAS_OP_QSIGMA, Qs.size).reshape(Qs.shape)
        assert rel(gQs, Qs) <= 1e-10, rel(gQs, Qs)
        M = np.concatenate([m.ravel() for m in clev.M_loc])
        gM = H.level_operator(l, N.SPFAS_OP_MLOC, M.size)
        assert rel(gM, M) <= 1e-10, rel(gM, M)
        D = np.concatenate([d.ravel() for d in clev.D_loc])
        gD = H.level_operator(l, N.SPFAS_OP_DLOC, D.size)
        assert rel(gD, D) <= 1e-10, rel(gD, D)
        w = np.concatenate(clev.w)
        gw = H.level_operator(l, N.SPFAS_OP_W, w.size)
        assert rel(gw, w) <= 1e-11, rel(gw, w)
