"""Fine-level TPFA discretisation in mixed form (oracle; test infrastructure only).

Section 2.1 of the paper: one pressure per cell, one flux per interface,
TPFA flux (eq. TPFA_flux) with half-transmissibilities (eq.
half-transmissibility), written as the augmented system (eq. FV_matrix)

    [ M(p)  D^T ] [sigma]     [ g ]
    [ D     0   ] [ p   ] = - [ f ],

    M_ii = 1/(kappa(p_K) Tb_K) + 1/(kappa(p_L) Tb_L)   interior face (K, L)
    M_ii = 1/(kappa(p_K) Tb_K)                         Dirichlet face of K
    D^T_{i,.} = e_L - e_K (interior), -e_K (Dirichlet)
    g_i = g_D on Dirichlet faces, 0 on interior faces
    f_K = |tau_K| f_K + sum over Neumann faces of K of |eps| g_N.

Neumann faces carry the prescribed flux sigma = -|eps| g_N; their row is
decoupled (M_ii = 1, no D entry), so they are kept out of the unknowns and
their flux is folded into f_K as the definition of f already does.  (The
index in the printed definition of D^T reads delta_iL - delta_iK where the
column index is meant; the flux row then gives sigma = Upsilon_KL (p_K - p_L),
which is eq. TPFA_flux.)
"""
from __future__ import annotations

import numpy as np

from .levels import Level, INTERIOR, DIRICHLET


def half_transmissibilities(mesh):
    """Tb_{i,eps} = |eps| n_i . K0_i . (x_eps - x_i) / ||x_eps - x_i||^2
    (eq. half-transmissibility), with n_K = n_eps and n_L = -n_eps.
    Returns (Tb_K [nf], Tb_L [nf]); Tb_L is 0 on boundary faces."""
    fc = mesh.face_cells.astype(np.int64)
    K, L = fc[:, 0], fc[:, 1]
    n = mesh.face_normal
    dK = mesh.face_point - mesh.cell_centroid[K]
    TK = mesh.face_area * np.einsum("fi,fij,fj->f", n, mesh.cell_k0[K], dK) / np.einsum("fi,fi->f", dK, dK)
    TL = np.zeros_like(TK)
    inner = L >= 0
    Li = L[inner]
    dL = mesh.face_point[inner] - mesh.cell_centroid[Li]
    TL[inner] = mesh.face_area[inner] * np.einsum("fi,fij,fj->f", -n[inner], mesh.cell_k0[Li], dL) \
        / np.einsum("fi,fi->f", dL, dL)
    return TK, TL


def lattice_from_centroids(centroid: np.ndarray):
    """Lattice coordinates of a Cartesian mesh recovered from cell centroids:
    per axis, the rank of the centroid coordinate among the distinct values
    (exact comparison).  Returns (shape, index) with index = i + nx*(j + ny*k)."""
    n, dim = centroid.shape
    shape, coords = [], []
    for a in range(dim):
        vals, inv = np.unique(centroid[:, a], return_inverse=True)
        shape.append(int(vals.size))
        coords.append(inv.astype(np.int64))
    index = np.zeros(n, dtype=np.int64)
    stride = 1
    for a in range(dim):
        index += coords[a] * stride
        stride *= shape[a]
    return tuple(shape), index


class FineMap:
    """Correspondence between input faces and level-0 flux unknowns."""

    def __init__(self, mesh):
        bc = mesh.face_bc
        self.flux_face = np.nonzero(bc != 2)[0]           # flux dof -> input face (input order)
        self.neumann_faces = np.nonzero(bc == 2)[0]
        self.n_faces = mesh.n_faces


def fine_level(prob):
    """Level 0 of the hierarchy plus the right-hand side b^0 = -[g; f]
    (eq. fine_level_operators).  Returns (level, b0, finemap)."""
    mesh = prob.mesh
    fm = FineMap(mesh)
    TK, TL = half_transmissibilities(mesh)
    fc = mesh.face_cells.astype(np.int64)
    ff = fm.flux_face
    nflux = ff.size
    n = mesh.n_cells
    K = fc[ff, 0]
    L = fc[ff, 1]
    kind = np.where(mesh.face_bc[ff] == 1, DIRICHLET, INTERIOR).astype(np.int8)
    if np.any((kind == INTERIOR) & (L < 0)) or np.any((kind == DIRICHLET) & (L >= 0)):
        raise ValueError("interior faces need two cells, boundary faces one")
    # cell -> (flux dof, Tb of that side, sign of D)
    cj = np.concatenate([np.arange(nflux), np.nonzero(L >= 0)[0]])
    cc = np.concatenate([K, L[L >= 0]])
    ct = np.concatenate([TK[ff], TL[ff][L >= 0]])
    cs = np.concatenate([-np.ones(nflux), np.ones(int((L >= 0).sum()))])
    order = np.lexsort((cj, cc))
    cj, cc, ct, cs = cj[order], cc[order], ct[order], cs[order]
    ptr = np.searchsorted(cc, np.arange(n + 1))
    cell_flux, M_loc, D_loc, w = [], [], [], []
    for c in range(n):
        s = slice(ptr[c], ptr[c + 1])
        cell_flux.append(cj[s].copy())
        M_loc.append(np.diag(1.0 / ct[s]))        # Prop. 1 on level 0: diag(1/Tb_{K,eps})
        D_loc.append(cs[s][None, :].copy())
        w.append(np.ones(1))
    shape, index = lattice_from_centroids(mesh.cell_centroid)
    if int(np.prod(np.array(shape, dtype=np.float64))) != n or np.unique(index).size != n:
        shape, index = None, None   # not a Cartesian lattice (box aggregation unavailable)
    lev = Level(n_cells=n, pdof_ptr=np.arange(n + 1), n_flux=nflux, flux_kind=kind,
                flux_cells=np.stack([K, np.where(L >= 0, L, -1)], axis=1),
                cell_flux=cell_flux, M_loc=M_loc, D_loc=D_loc, w=w,
                ones=np.ones(n), u=mesh.cell_volume.copy(), vol=mesh.cell_volume.copy(),
                lattice_shape=shape, lattice_index=index).finalize()
    sh = getattr(prob, "shift", None)
    lev.shift = None if sh is None else np.asarray(sh, dtype=np.float64).copy()
    # right-hand side
    g = np.where(kind == DIRICHLET, prob.g_dirichlet[ff], 0.0)
    f = mesh.cell_volume * prob.source
    nf_ = fm.neumann_faces
    np.add.at(f, fc[nf_, 0], mesh.face_area[nf_] * prob.g_neumann[nf_])
    b0 = -np.concatenate([g, f])
    return lev, b0, fm


def full_flux(prob, fm: FineMap, sig_dofs: np.ndarray) -> np.ndarray:
    """Flux on every input face: the unknowns, and sigma = -|eps| g_N on
    Neumann faces (eq. TPFA_flux, third case)."""
    out = np.zeros(fm.n_faces)
    out[fm.flux_face] = sig_dofs
    nf_ = fm.neumann_faces
    out[nf_] = -prob.mesh.face_area[nf_] * prob.g_neumann[nf_]
    return out


class FineSystem:
    """The level-0 system written face by face, directly from eq. FV_matrix
    (vectorised; used at sizes where per-cell assembly is too slow)."""

    def __init__(self, prob):
        mesh = prob.mesh
        self.fm = FineMap(mesh)
        TK, TL = half_transmissibilities(mesh)
        ff = self.fm.flux_face
        fc = mesh.face_cells.astype(np.int64)
        self.K = fc[ff, 0]
        self.L = fc[ff, 1]
        self.inner = self.L >= 0
        self.TK = TK[ff]
        self.TL = TL[ff]
        self.n_cells = mesh.n_cells
        self.n_flux = ff.size
        from .levels import kappa_of
        self.alpha = kappa_of(prob)
        sh = getattr(prob, "shift", None)
        self.shift = np.zeros(mesh.n_cells) if sh is None else np.asarray(sh, dtype=np.float64)
        self.g = np.where(self.inner, 0.0, prob.g_dirichlet[ff])
        f = mesh.cell_volume * prob.source
        nf_ = self.fm.neumann_faces
        np.add.at(f, fc[nf_, 0], mesh.face_area[nf_] * prob.g_neumann[nf_])
        self.f = f

    def residual(self, sigma, p):
        """r_sigma = M(p) sigma + D^T p + g, r_p = D sigma + f."""
        from .levels import kinv
        a = self.alpha
        Li = np.where(self.inner, self.L, 0)
        psi = p - self.shift
        m = kinv(psi[self.K], a) / self.TK
        m = m + np.where(self.inner, kinv(psi[Li], a) / np.where(self.inner, self.TL, 1.0), 0.0)
        dtp = np.where(self.inner, p[Li], 0.0) - p[self.K]
        r_sig = m * sigma + dtp + self.g
        div = np.zeros(self.n_cells)
        np.add.at(div, self.K, -sigma)
        np.add.at(div, self.L[self.inner], sigma[self.inner])
        return r_sig, div + self.f


def linear_pressure(prob):
    """Pressure of the linear problem (kappa = 1) from the reduced cell
    system of the remark after eq. FV_matrix: eliminating sigma with the
    diagonal M gives D M^{-1} D^T p = f - D M^{-1} g (sign of g as it follows
    from the first block row M sigma + D^T p = -g).  Sparse direct solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    fs = FineSystem(prob)
    n = fs.n_cells
    w = 1.0 / (1.0 / fs.TK + np.where(fs.inner, 1.0 / np.where(fs.inner, fs.TL, 1.0), 0.0))
    K, L, inner = fs.K, fs.L, fs.inner
    rows = np.concatenate([K, L[inner], K[inner], L[inner]])
    cols = np.concatenate([K, L[inner], L[inner], K[inner]])
    vals = np.concatenate([w, w[inner], -w[inner], -w[inner]])
    S = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    # D M^{-1} g: Dirichlet faces carry g on the K side with D = -1
    dmg = np.zeros(n)
    np.add.at(dmg, K[~inner], -w[~inner] * fs.g[~inner])
    return spla.spsolve(S.tocsc(), fs.f - dmg)
