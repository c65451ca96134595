"""Fine-level residual of the HIP library against the oracle (eq. FV_matrix),
element by element, on seeded states (GPU)."""
import numpy as np
import pytest

from problems import small_problem, c1_problem, c2_problem
from oracle.fv import FineSystem

pytestmark = pytest.mark.gpu


def check_residual(prob, seed=0, scale=0.5):
    import paper_2005_01275_amd as pk
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    rng = np.random.default_rng(seed)
    n, nf = prob.mesh.n_cells, prob.mesh.n_faces
    p = scale * rng.standard_normal(n)
    s = rng.standard_normal(nf)
    rp, rs = H.eval_residual(prob, p, s)
    fs = FineSystem(prob)
    ff = fs.fm.flux_face
    ref_s, ref_p = fs.residual(s[ff], p)
    # row scales of the two equation blocks
    a = prob.alpha
    Li = np.where(fs.inner, fs.L, 0)
    m = np.exp(-a * p[fs.K]) / fs.TK + np.where(fs.inner, np.exp(-a * p[Li]) / np.where(fs.inner, fs.TL, 1), 0)
    sc_s = np.abs(m * s[ff]) + np.abs(p[fs.K]) + np.abs(np.where(fs.inner, p[Li], 0)) + np.abs(fs.g)
    absdiv = np.zeros(n)
    np.add.at(absdiv, fs.K, np.abs(s[ff]))
    np.add.at(absdiv, fs.L[fs.inner], np.abs(s[ff][fs.inner]))
    sc_p = absdiv + np.abs(fs.f)
    assert np.all(np.abs(rs[ff] - ref_s) <= 4e-15 * sc_s + 1e-300)
    assert np.all(np.abs(rp - ref_p) <= 4e-15 * sc_p + 1e-300)
    nn = np.setdiff1d(np.arange(nf), ff)
    assert np.all(rs[nn] == 0.0)
    return H


@pytest.mark.parametrize("kw", [
    dict(shape=(8, 8), box=(4, 4), m=2, n_levels=2, seed=1, g_d_scale=0.3, g_n_scale=0.2),
    dict(shape=(13, 7), box=(4, 3), m=2, n_levels=3, seed=2, permute=True, dirichlet=((0, 0), (1, 1)),
         g_d_scale=0.5, g_n_scale=0.4, anisotropic=True),
    dict(shape=(7, 6, 5), box=(2, 2, 2), m=3, n_levels=2, seed=3, permute=True, g_n_scale=0.3, alpha=2.0),
    dict(shape=(5, 3), box=(2, 2), m=1, n_levels=1, seed=4),
])
def test_residual_small(kw):
    print("case", kw, flush=True)
    check_residual(small_problem(**kw))


def test_residual_c1():
    check_residual(c1_problem())


def test_residual_c2_full():
    print("case c2 full", flush=True)
    check_residual(c2_problem(), scale=0.3)
