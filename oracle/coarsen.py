"""Hierarchy construction (oracle; test infrastructure only).

Section 3.1 and Appendix A of the paper, level l -> l+1:

* aggregates of level-l cells (connected, non-overlapping; here boxes on the
  level lattice, see ``box_aggregate``),
* local spectral problem D|_A M|_A^{-1} D|_A^T q = lambda q on each aggregate
  (eq. local-eigenvalue-problem) and P_A = [q_PV, P_NPV] with
  q_PV = 1^l|_A / ||1^l|_A|| (eqs. structure_pressure_interpolation,
  definition_q_pv),
* sigma_PV on each coarse interface from the local mixed problem on the union
  of its two aggregates (eq. local_problem_to_define_sigma_pv) -- with one
  flux per interface (m_f = 1) this is the only trace kept,
* extension of each trace into the neighbouring aggregates by the local
  Neumann problem (eq. local_neumann_boundary_value_problem),
* bubbles: the same problem with right-hand side [0; q] for each NPV column,
* P_sigma = [P^TR 0; P^E P^B], P_p = blockdiag(P_A), Q_p = P_p^T,
* static coarse local matrices M^{l+1}_A = P_sigma,A^T M^l_A P_sigma,A (proof
  of Prop. 1) and D^{l+1} = P_p^T D^l P_sigma (Section 3.1),
* weights of the piecewise-constant projector (Appendix B).

Readings taken where the paper is silent (each restated at its code):
  * the eigenproblem uses the static matrices (kappa = 1) on the aggregate
    itself, not the extended aggregate N(A) -- with one flux per interface the
    traces of the eigenvectors are discarded, so N(A) is not needed;
  * eigenvector sign: the first local entry with |v_k| > 1e-8 max|v| is made
    positive (local order = ascending cell id, then coefficient index);
  * a group of Dirichlet faces of an aggregate is one coarse flux with a
    one-sided PV trace (unit total outflow) from the same mixed problem on A;
  * Q_sigma (deferred by the paper to the spectral-coarsening reference) is
    the flux-moment projection: phi_F = q_PV^T D|_{A,F} sigma / q_PV^T D|_{A,F} t_F
    on coarse interfaces and beta_j = v_j^T (D sigma)|_A on bubbles, which
    satisfies Q P = I and D^{l+1} Q_sigma = Q_p D^l.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np
import scipy.sparse as sp

from .levels import Level, INTERIOR, DIRICHLET, BUBBLE, kappa_of


# ------------------------------------------------------------- aggregation

def box_blocks(n: int, a: int) -> int:
    """Number of boxes of edge a along an axis of n cells: a remainder block
    with fewer than a/2 cells merges into the previous block."""
    nb, rem = divmod(n, a)
    if rem == 0:
        return max(nb, 1)
    if 2 * rem < a:
        return max(nb, 1)
    return nb + 1


def box_aggregate(shape, index, box):
    """Box aggregates on a lattice; ids lexicographic with x fastest.
    Returns (agg [n], coarse lattice shape)."""
    dim = len(shape)
    index = np.asarray(index, dtype=np.int64)
    agg = np.zeros(index.size, dtype=np.int64)
    rem = index.copy()
    stride = 1
    cshape = []
    for a in range(dim):
        coord = rem % shape[a]
        rem //= shape[a]
        nb = box_blocks(shape[a], box[a])
        blk = np.minimum(coord // box[a], nb - 1)
        agg += blk * stride
        stride *= nb
        cshape.append(nb)
    return agg, tuple(cshape)


def greedy_aggregate(level: Level, target: int) -> np.ndarray:
    """Greedy graph aggregation of a level (the paper partitions with METIS;
    this rule is the build's deterministic stand-in for unstructured meshes):
    seeds in ascending cell id grow breadth first, visiting neighbours in
    ascending id, until the aggregate holds ``target`` cells; then every
    aggregate with fewer than target/2 cells, in ascending id, joins the
    neighbouring aggregate with which it shares the most interior flux
    unknowns (ties: the lower id); ids are renumbered in ascending order of
    the surviving aggregates.  Neighbours are cells that share an interior
    flux unknown of the level."""
    from collections import deque
    n = level.n_cells
    fc = level.flux_cells
    inner = np.nonzero((level.flux_kind == INTERIOR) & (fc[:, 1] >= 0))[0]
    nbr = [set() for _ in range(n)]
    for j in inner:
        a, b = int(fc[j, 0]), int(fc[j, 1])
        nbr[a].add(b)
        nbr[b].add(a)
    nbr = [sorted(x) for x in nbr]
    agg = np.full(n, -1, dtype=np.int64)
    members = []
    for seed in range(n):
        if agg[seed] >= 0:
            continue
        A = len(members)
        group = [seed]
        agg[seed] = A
        queue = deque([seed])
        while queue and len(group) < target:
            u = queue.popleft()
            for v in nbr[u]:
                if len(group) >= target:
                    break
                if agg[v] < 0:
                    agg[v] = A
                    group.append(v)
                    queue.append(v)
        members.append(group)
    na0 = len(members)
    label = np.arange(na0)
    size = np.array([len(g) for g in members])
    for A in range(na0):
        if label[A] != A or 2 * size[A] >= target:
            continue
        la = label[agg[fc[inner, 0]]]
        lb = label[agg[fc[inner, 1]]]
        shared = {}
        for x, y in zip(la, lb):
            if x == A and y != A:
                shared[int(y)] = shared.get(int(y), 0) + 1
            elif y == A and x != A:
                shared[int(x)] = shared.get(int(x), 0) + 1
        if not shared:
            continue
        best = min(shared, key=lambda B: (-shared[B], B))
        label[label == A] = best
        size[best] += size[A]
        size[A] = 0
    survivors = np.unique(label)
    newid = np.full(na0, -1, dtype=np.int64)
    newid[survivors] = np.arange(survivors.size)
    return newid[label[agg]]


def renumber(level: Level, agg: np.ndarray):
    """Cells contiguous per aggregate (stable by (aggregate, id)); flux
    unknowns grouped [inside each aggregate] [per coarse interface, by
    (lower, higher) aggregate] [Dirichlet, per aggregate]; inside a group by
    (face before bubble, lower renumbered cell, higher renumbered cell, id).
    Returns (cell_order, flux_order): position -> canonical id."""
    n = level.n_cells
    cell_order = np.lexsort((np.arange(n), agg))
    pos = np.empty(n, dtype=np.int64)
    pos[cell_order] = np.arange(n)
    kind = level.flux_kind
    c1 = level.flux_cells[:, 0]
    c2 = level.flux_cells[:, 1]
    two = c2 >= 0
    a1 = agg[c1]
    a2 = np.where(two, agg[np.maximum(c2, 0)], -1)
    inside = (kind == BUBBLE) | ((kind == INTERIOR) & (a1 == a2))
    cross = (kind == INTERIOR) & (a1 != a2)
    g0 = np.where(inside, 0, np.where(cross, 1, 2))
    g1 = np.where(cross, np.minimum(a1, a2), a1)
    g2 = np.where(cross, np.maximum(a1, a2), 0)
    kr = (kind == BUBBLE).astype(np.int64)
    p1 = pos[c1]
    p2 = np.where(two, pos[np.maximum(c2, 0)], p1)
    lo = np.minimum(p1, p2)
    hi = np.maximum(p1, p2)
    flux_order = np.lexsort((np.arange(level.n_flux), hi, lo, kr, g2, g1, g0))
    return cell_order, flux_order


# ------------------------------------------------------------- local pieces

def assemble_local(level: Level, cells, dofs):
    """Static M^l restricted to the flux unknowns ``dofs`` and assembled from
    the local matrices of ``cells`` (Prop. 1), and D^l[pdofs(cells), dofs]."""
    dofs = np.asarray(dofs, dtype=np.int64)
    where = {int(j): i for i, j in enumerate(dofs)}
    pd = np.concatenate([level.pdofs(c) for c in cells])
    prow = {int(j): i for i, j in enumerate(pd)}
    M = np.zeros((dofs.size, dofs.size))
    D = np.zeros((pd.size, dofs.size))
    for c in cells:
        loc = np.array([where.get(int(j), -1) for j in level.cell_flux[c]], dtype=np.int64)
        keep = loc >= 0
        li = loc[keep]
        M[np.ix_(li, li)] += level.M_loc[c][np.ix_(keep, keep)]
        rows = np.array([prow[int(j)] for j in level.pdofs(c)], dtype=np.int64)
        D[np.ix_(rows, li)] += level.D_loc[c][:, keep]
    return M, D, pd


def saddle_solve(M, D, a, b, kernel=None):
    """Solve [M D^T; D 0][s; q] = [a; b].  When the pressure block is
    singular (pure Neumann local problem), ``kernel`` spans its null space
    and q is fixed by kernel^T q = 0; s is unique either way."""
    n, m = M.shape[0], D.shape[0]
    if kernel is None:
        K = np.block([[M, D.T], [D, np.zeros((m, m))]])
        sol = np.linalg.solve(K, np.concatenate([a, b]))
        return sol[:n], sol[n:]
    u = kernel.reshape(-1, 1)
    K = np.block([[M, D.T, np.zeros((n, 1))],
                  [D, np.zeros((m, m)), u],
                  [np.zeros((1, n)), u.T, np.zeros((1, 1))]])
    sol = np.linalg.solve(K, np.concatenate([a, b, [0.0]]))
    return sol[:n], sol[n:n + m]


def sign_fix(v: np.ndarray) -> np.ndarray:
    """First local entry with |v_k| > 1e-8 max|v| made positive."""
    thr = 1e-8 * np.max(np.abs(v))
    k = int(np.argmax(np.abs(v) > thr))
    return -v if v[k] < 0 else v


@dataclasses.dataclass
class AggData:
    cells: np.ndarray
    pd: np.ndarray                 # p unknowns of the aggregate (ascending)
    int_dofs: np.ndarray           # int(A)
    faces: Dict[int, np.ndarray]   # neighbour aggregate -> flux unknowns of F_AB
    dir_dofs: np.ndarray           # Dirichlet flux unknowns of A
    dofs: np.ndarray               # int(A) ++ F (by neighbour) ++ Dirichlet
    M: np.ndarray                  # static M^l_A over dofs
    D: np.ndarray                  # D^l[pd, dofs]
    lam: np.ndarray = None         # eigenvalues of L_A (ascending)
    V: np.ndarray = None           # eigenvectors of L_A
    P: np.ndarray = None           # P_A = [q_PV, v_2..v_m]


def aggregate_data(level: Level, agg: np.ndarray, A: int, cells) -> AggData:
    js = np.unique(np.concatenate([level.cell_flux[c] for c in cells]))
    kind = level.flux_kind[js]
    c1 = level.flux_cells[js, 0]
    c2 = level.flux_cells[js, 1]
    a1 = agg[c1]
    a2 = np.where(c2 >= 0, agg[np.maximum(c2, 0)], -1)
    is_int = (kind == BUBBLE) | ((kind == INTERIOR) & (a1 == a2))
    is_face = (kind == INTERIOR) & (a1 != a2)
    is_dir = kind == DIRICHLET
    other = np.where(a1 == A, a2, a1)
    faces = {int(B): js[is_face & (other == B)] for B in np.unique(other[is_face])}
    int_dofs = js[is_int]
    dir_dofs = js[is_dir]
    dofs = np.concatenate([int_dofs] + [faces[B] for B in sorted(faces)] + [dir_dofs]).astype(np.int64)
    M, D, pd = assemble_local(level, cells, dofs)
    return AggData(cells=np.asarray(cells), pd=pd, int_dofs=int_dofs, faces=faces,
                   dir_dofs=dir_dofs, dofs=dofs, M=M, D=D)


def eig_count(lam: np.ndarray, m: int, threshold: float = 0.0, m_min: int = 2) -> int:
    """Number of local eigenvectors kept for an aggregate whose ascending
    eigenvalues are lam.  threshold <= 0: the uniform count m (the paper's
    m_A).  threshold > 0: the eigenvalues up to threshold times the largest
    (lambda_1 = 0 included), clamped to [m_min, m]; either way at most the
    number of pressure unknowns of the aggregate."""
    if threshold > 0.0:
        cnt = int(np.count_nonzero(lam <= threshold * lam[-1]))
        mA = min(max(cnt, m_min), m)
    else:
        mA = m
    return min(mA, lam.size)


def local_spectral(level: Level, ad: AggData, m: int, threshold: float = 0.0, m_min: int = 2):
    """Eigen-decomposition of L_A = D|_A (M|_int(A))^{-1} D|_A^T with the
    static (kappa = 1) matrices (eq. local-eigenvalue-problem) and
    P_A = [q_PV, v_2, ..., v_m] (eqs. structure_pressure_interpolation and
    definition_q_pv); m per eig_count."""
    ni = ad.int_dofs.size
    Mi = ad.M[:ni, :ni]
    Di = ad.D[:, :ni]
    if ni:
        L = Di @ np.linalg.solve(Mi, Di.T)
        L = 0.5 * (L + L.T)
    else:
        L = np.zeros((ad.pd.size, ad.pd.size))
    lam, V = np.linalg.eigh(L)
    one = level.ones[ad.pd]
    q = one / np.linalg.norm(one)
    mA = eig_count(lam, m, threshold, m_min)
    cols = [q]
    for i in range(1, mA):
        v = V[:, i] - (q @ V[:, i]) * q
        v = v / np.linalg.norm(v)
        cols.append(sign_fix(v))
    ad.lam, ad.V, ad.P = lam, V, np.stack(cols, axis=1)
    return ad


def pos_in(dofs: np.ndarray, sub: np.ndarray) -> np.ndarray:
    where = {int(j): i for i, j in enumerate(dofs)}
    return np.array([where[int(j)] for j in sub], dtype=np.int64)


def pv_trace(level: Level, ads: Dict[int, AggData], A: int, B: int):
    """sigma_PV of the coarse interface between A < B: local mixed problem
    on A u B with right-hand side [0; -1|_A/||1|_A||^2 ; +1|_B/||1|_B||^2]
    (eq. local_problem_to_define_sigma_pv); returns its restriction to F_AB
    (which carries unit total flux from A to B)."""
    a, b = ads[A], ads[B]
    F = a.faces[B]
    dofs = np.concatenate([a.int_dofs, b.int_dofs, F])
    cells = np.concatenate([a.cells, b.cells])
    M, D, pd = assemble_local(level, cells, dofs)
    oa, ob = level.ones[a.pd], level.ones[b.pd]
    f = np.concatenate([-oa / (oa @ oa), ob / (ob @ ob)])
    s, _ = saddle_solve(M, D, np.zeros(dofs.size), f, kernel=level.ones[pd])
    return s[dofs.size - F.size:]


def pv_trace_dirichlet(level: Level, ad: AggData):
    """One-sided PV trace on the Dirichlet faces of an aggregate (reading:
    the same mixed problem on A with right-hand side [0; -1|_A/||1|_A||^2],
    nonsingular because of the Dirichlet faces); unit total outflow."""
    F = ad.dir_dofs
    dofs = np.concatenate([ad.int_dofs, F])
    M, D, pd = assemble_local(level, ad.cells, dofs)
    oa = level.ones[pd]
    s, _ = saddle_solve(M, D, np.zeros(dofs.size), -oa / (oa @ oa))
    return s[dofs.size - F.size:]


def extension(level: Level, ad: AggData, F: np.ndarray, t: np.ndarray):
    """Extension of the trace t on F into int(A): local Neumann problem
    [M_int D_int^T; D_int 0][s; p] = [-M_{int,F} t; c q_PV - D_{A,F} t] with
    c = q_PV^T D_{A,F} t (eq. local_neumann_boundary_value_problem)."""
    ni = ad.int_dofs.size
    fpos = pos_in(ad.dofs, F)
    q = ad.P[:, 0]
    DF = ad.D[:, fpos] @ t
    c = q @ DF
    if ni == 0:
        return np.zeros(0), c
    s, _ = saddle_solve(ad.M[:ni, :ni], ad.D[:, :ni], -ad.M[:ni, fpos] @ t, c * q - DF,
                        kernel=level.ones[ad.pd])
    return s, c


def bubble(level: Level, ad: AggData, v: np.ndarray):
    """Bubble of an NPV column v: the same local problem with right-hand side [0; v]."""
    ni = ad.int_dofs.size
    s, _ = saddle_solve(ad.M[:ni, :ni], ad.D[:, :ni], np.zeros(ni), v, kernel=level.ones[ad.pd])
    return s


# ------------------------------------------------------------- one coarsening

@dataclasses.dataclass
class Transfer:
    P_sig: sp.csr_matrix
    P_p: sp.csr_matrix
    Q_sig: sp.csr_matrix
    agg: np.ndarray
    cell_order: np.ndarray
    flux_order: np.ndarray
    aggs: List[AggData]
    coarse_faces: List[Tuple[int, int]]      # (A, B) with A < B; B = -1 for Dirichlet
    traces: List[np.ndarray]

    @property
    def Q_p(self):
        return self.P_p.T.tocsr()

    def P(self, e, nf_c):
        return np.concatenate([self.P_sig @ e[:nf_c], self.P_p @ e[nf_c:]])

    def Q(self, x, nf):
        return np.concatenate([self.Q_sig @ x[:nf], self.Q_p @ x[nf:]])

    def R(self, r, nf):
        """R = P^T (Section 3)."""
        return np.concatenate([self.P_sig.T @ r[:nf], self.P_p.T @ r[nf:]])


def coarsen(level: Level, agg: np.ndarray, cshape, m: int, threshold: float = 0.0, m_min: int = 2):
    n_agg = int(agg.max()) + 1
    cell_order, flux_order = renumber(level, agg)
    members = [np.sort(np.nonzero(agg == A)[0]) for A in range(n_agg)]
    ads = {}
    for A in range(n_agg):
        if members[A].size == 0:
            raise ValueError("empty aggregate")
        ads[A] = local_spectral(level, aggregate_data(level, agg, A, members[A]), m, threshold, m_min)
    # coarse flux numbering: interior interfaces (A<B), Dirichlet groups, bubbles
    pairs = sorted({(A, B) for A in range(n_agg) for B in ads[A].faces if A < B})
    dirs = [A for A in range(n_agg) if ads[A].dir_dofs.size]
    faces = pairs + [(A, -1) for A in dirs]
    nF = len(faces)
    mA = [ads[A].P.shape[1] for A in range(n_agg)]
    bub_ptr = np.concatenate([[0], np.cumsum([k - 1 for k in mA])]) + nF
    nfc = int(bub_ptr[-1])
    traces, exts = [], []
    for (A, B) in faces:
        if B >= 0:
            t = pv_trace(level, ads, A, B)
            F = ads[A].faces[B]
            eA, cA = extension(level, ads[A], F, t)
            eB, cB = extension(level, ads[B], F, t)
            exts.append({A: (eA, cA), B: (eB, cB)})
        else:
            t = pv_trace_dirichlet(level, ads[A])
            eA, cA = extension(level, ads[A], ads[A].dir_dofs, t)
            exts.append({A: (eA, cA)})
        traces.append(t)
    bubs = {A: [bubble(level, ads[A], ads[A].P[:, j]) for j in range(1, mA[A])] for A in range(n_agg)}
    # P_sigma
    rows, cols, vals = [], [], []
    for fi, (A, B) in enumerate(faces):
        F = ads[A].faces[B] if B >= 0 else ads[A].dir_dofs
        rows.append(F); cols.append(np.full(F.size, fi)); vals.append(traces[fi])
        for X, (e, _) in exts[fi].items():
            rows.append(ads[X].int_dofs); cols.append(np.full(e.size, fi)); vals.append(e)
    for A in range(n_agg):
        for j, bj in enumerate(bubs[A]):
            rows.append(ads[A].int_dofs); cols.append(np.full(bj.size, bub_ptr[A] + j)); vals.append(bj)
    P_sig = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(level.n_flux, nfc))
    # P_p and coarse pressure numbering
    pptr = np.concatenate([[0], np.cumsum(mA)])
    pr, pc, pv = [], [], []
    for A in range(n_agg):
        rr, cc = np.meshgrid(ads[A].pd, np.arange(pptr[A], pptr[A + 1]), indexing="ij")
        pr.append(rr.ravel()); pc.append(cc.ravel()); pv.append(ads[A].P.ravel())
    P_p = sp.csr_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))),
                        shape=(level.n_p, int(pptr[-1])))
    # Q_sigma: flux moments on interfaces, divergence moments on bubbles
    qr, qc, qv = [], [], []
    for fi, (A, B) in enumerate(faces):
        ad = ads[A]
        F = ad.faces[B] if B >= 0 else ad.dir_dofs
        row = ad.P[:, 0] @ ad.D[:, pos_in(ad.dofs, F)]
        qr.append(np.full(F.size, fi)); qc.append(F); qv.append(row / (row @ traces[fi]))
    for A in range(n_agg):
        ad = ads[A]
        for j in range(1, mA[A]):
            qr.append(np.full(ad.dofs.size, bub_ptr[A] + j - 1)); qc.append(ad.dofs)
            qv.append(ad.P[:, j] @ ad.D)
    Q_sig = sp.csr_matrix((np.concatenate(qv), (np.concatenate(qr), np.concatenate(qc))),
                          shape=(nfc, level.n_flux))
    # coarse level: local flux lists, static local matrices, projector weights
    fkind = np.concatenate([np.full(len(pairs), INTERIOR), np.full(len(dirs), DIRICHLET),
                            np.full(nfc - nF, BUBBLE)]).astype(np.int8)
    fcells = np.full((nfc, 2), -1, dtype=np.int64)
    for fi, (A, B) in enumerate(faces):
        fcells[fi] = (A, B)
    for A in range(n_agg):
        fcells[bub_ptr[A]:bub_ptr[A + 1], 0] = A
    cell_flux, M_loc, D_loc, w = [], [], [], []
    ones_c = np.zeros(int(pptr[-1]))
    u_c = np.zeros(int(pptr[-1]))
    vol_c = np.zeros(n_agg)
    for A in range(n_agg):
        ad = ads[A]
        mine = [fi for fi, (X, Y) in enumerate(faces) if X == A or Y == A]
        lf = np.array(mine + list(range(bub_ptr[A], bub_ptr[A + 1])), dtype=np.int64)
        # P_sigma restricted to dofs(A) and the coarse unknowns of A
        Ploc = np.asarray(P_sig[ad.dofs][:, lf].todense())
        M_loc.append(Ploc.T @ ad.M @ Ploc)
        D_loc.append(ad.P.T @ ad.D @ Ploc)
        cell_flux.append(lf)
        ones_c[pptr[A]:pptr[A + 1]] = ad.P.T @ level.ones[ad.pd]
        u_c[pptr[A]:pptr[A + 1]] = ad.P.T @ level.u[ad.pd]
        vol_c[A] = level.vol[ad.cells].sum()
        w.append(u_c[pptr[A]:pptr[A + 1]] / vol_c[A])
    coarse = Level(n_cells=n_agg, pdof_ptr=pptr, n_flux=nfc, flux_kind=fkind, flux_cells=fcells,
                   cell_flux=cell_flux, M_loc=M_loc, D_loc=D_loc, w=w, ones=ones_c, u=u_c,
                   vol=vol_c, lattice_shape=tuple(cshape),
                   lattice_index=np.arange(n_agg)).finalize()
    if level.shift is not None:
        # volume-weighted mean of the level-0 shift over each coarse cell
        coarse.shift = np.array([(level.vol[ads[A].cells] * level.shift[ads[A].cells]).sum() / vol_c[A]
                                 for A in range(n_agg)])
    tr = Transfer(P_sig=P_sig, P_p=P_p, Q_sig=Q_sig, agg=agg, cell_order=cell_order,
                  flux_order=flux_order, aggs=[ads[A] for A in range(n_agg)],
                  coarse_faces=faces, traces=traces)
    return coarse, tr


# ------------------------------------------------------------- hierarchy

@dataclasses.dataclass
class Hierarchy:
    levels: List[Level]
    transfers: List[Transfer]
    b0: np.ndarray
    alpha: object                  # exponent of kappa = exp(alpha p), or a levels.Kappa
    finemap: object


def build_hierarchy(prob, n_levels=None, box=None, m=None, greedy_size=None, user_agg=None,
                    eig_threshold=None, m_min=None, greedy_size_coarse=None) -> Hierarchy:
    """Levels and transfers of ``prob``.  Aggregation: boxes on the level
    lattice by default; ``greedy_size`` > 0 selects ``greedy_aggregate``
    (with the target ``greedy_size_coarse`` on levels 1 and up when that is
    > 0);
    ``user_agg`` (one array per coarsened level) gives it explicitly.
    ``eig_threshold`` > 0 selects the eigenvalue-threshold count of
    ``eig_count`` (m is then the upper clamp).  Defaults come from the
    problem's own configuration."""
    from .fv import fine_level
    n_levels = prob.n_levels if n_levels is None else n_levels
    box = prob.box if box is None else box
    m = prob.m if m is None else m
    if greedy_size is None:
        greedy_size = getattr(prob, "greedy_size", 0)
    if greedy_size_coarse is None:
        greedy_size_coarse = getattr(prob, "greedy_size_coarse", 0)
    if eig_threshold is None:
        eig_threshold = getattr(prob, "eig_threshold", 0.0)
    if m_min is None:
        m_min = getattr(prob, "m_min", 2)
    lev, b0, fm = fine_level(prob)
    levels, transfers = [lev], []
    for l in range(n_levels - 1):
        cur = levels[-1]
        if user_agg is not None:
            agg, cshape = np.asarray(user_agg[l], dtype=np.int64), ()
        elif greedy_size:
            target = greedy_size_coarse if l > 0 and greedy_size_coarse > 0 else greedy_size
            agg, cshape = greedy_aggregate(cur, target), ()
        else:
            if cur.lattice_shape is None:
                raise ValueError("box aggregation needs a Cartesian lattice")
            agg, cshape = box_aggregate(cur.lattice_shape, cur.lattice_index, box)
        coarse, tr = coarsen(cur, agg, cshape, m, eig_threshold, m_min)
        levels.append(coarse)
        transfers.append(tr)
    return Hierarchy(levels=levels, transfers=transfers, b0=b0, alpha=kappa_of(prob), finemap=fm)
