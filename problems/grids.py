"""Cartesian meshes, permeability fields, boundary data and sources.

Every function here is seeded and deterministic.  The arrays describe the
boundary-value problem of Section 2 of the paper (mass conservation with
Darcy's law, K(x, p) = K0(x) kappa(p), kappa(p) = exp(alpha p), Dirichlet and
Neumann data; or the Richards-type family of Example 3, kappa evaluated at
p - z with a per-cell shift z) on a conforming mesh given as cells and an unstructured face
list.  Nothing here evaluates the finite-volume scheme itself.

Conventions shared by both consumers of these arrays:
  * ``face_cells[f] = (K, L)``; ``L = -1`` on a boundary face.
  * ``face_normal[f]`` is the unit normal pointing out of cell K.
  * ``face_point[f]`` is the collocation point x_eps (Section 2.1, remark on
    collocation points): the face centre for these Cartesian meshes.
  * ``face_bc``: 0 interior, 1 Dirichlet, 2 Neumann.
  * ``source`` is the density f of the mass-conservation equation (not yet
    multiplied by the cell measure); ``g_neumann`` is g_N = -q.n.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Mesh:
    dim: int
    cell_volume: np.ndarray        # [n] float64
    cell_centroid: np.ndarray      # [n, dim] float64
    cell_k0: np.ndarray            # [n, dim, dim] float64, K0 tensor
    face_cells: np.ndarray         # [nf, 2] int32
    face_area: np.ndarray          # [nf] float64
    face_normal: np.ndarray        # [nf, dim] float64, out of K
    face_point: np.ndarray         # [nf, dim] float64
    face_bc: np.ndarray            # [nf] int8
    shape: Optional[tuple] = None  # lattice shape when structured (informational)

    @property
    def n_cells(self) -> int:
        return int(self.cell_volume.shape[0])

    @property
    def n_faces(self) -> int:
        return int(self.face_area.shape[0])


@dataclasses.dataclass
class Problem:
    mesh: Mesh
    alpha: float                   # kappa(p) = exp(alpha p)
    source: np.ndarray             # [n] density f
    g_dirichlet: np.ndarray        # [nf] used where face_bc == 1
    g_neumann: np.ndarray          # [nf] used where face_bc == 2
    name: str = ""
    # hierarchy configuration of the workload (box edge per axis, number of
    # local eigenvectors per aggregate, number of levels)
    box: tuple = ()
    m: int = 1
    n_levels: int = 2
    dp_cap_c: float = 5.0          # cap constant c: max |dp| <= ln(c)/alpha
    greedy_size: int = 0           # > 0: greedy aggregates of about this many cells (unstructured meshes)
    greedy_size_coarse: int = 0    # > 0: the greedy target on levels 1 and up
    # > 0: eigenvectors per aggregate by the eigenvalue threshold (lambda <=
    # eig_threshold * lambda_max), clamped to [m_min, m]
    eig_threshold: float = 0.0
    m_min: int = 2
    # kappa family: "exp" (exp(alpha psi)) or "richards" (a / (a + |psi|^beta)),
    # evaluated at psi = p - shift (shift per cell, None = 0)
    kappa_kind: str = "exp"
    kappa_a: float = 1.0
    kappa_beta: float = 2.0
    shift: Optional[np.ndarray] = None


# ---------------------------------------------------------------- meshes

def cartesian_mesh(shape, spacing, k_cells, dirichlet=((0, 0),)) -> Mesh:
    """Uniform Cartesian mesh with cell id = i + nx*(j + ny*k).

    ``k_cells`` is [n] (isotropic K0 = k I) or [n, dim] (diagonal K0).
    ``dirichlet`` lists (axis, side) boundary sides that carry Dirichlet
    data; all other boundary sides are Neumann.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    h = np.asarray(spacing, dtype=np.float64)
    assert h.shape == (dim,)
    n = int(np.prod(shape))
    idx = np.arange(n)
    # lattice coordinates, x fastest
    coords = []
    rem = idx.copy()
    for a in range(dim):
        coords.append(rem % shape[a])
        rem //= shape[a]
    coords = np.stack(coords, axis=1)
    centroid = (coords.astype(np.float64) + 0.5) * h[None, :]
    vol = np.full(n, float(np.prod(h)))
    k = np.asarray(k_cells, dtype=np.float64)
    k0 = np.zeros((n, dim, dim))
    if k.ndim == 1:
        for a in range(dim):
            k0[:, a, a] = k
    else:
        for a in range(dim):
            k0[:, a, a] = k[:, a]

    strides = [1]
    for a in range(1, dim):
        strides.append(strides[-1] * shape[a - 1])

    fK, fL, farea, fnorm, fpt, fbc = [], [], [], [], [], []
    dset = set(tuple(d) for d in dirichlet)
    for a in range(dim):
        area = float(np.prod(h)) / h[a]
        e = np.zeros(dim)
        e[a] = 1.0
        inner = coords[:, a] < shape[a] - 1
        K = idx[inner]
        fK.append(K)
        fL.append(K + strides[a])
        farea.append(np.full(K.size, area))
        fnorm.append(np.tile(e, (K.size, 1)))
        pt = centroid[K].copy()
        pt[:, a] = (coords[K, a] + 1).astype(np.float64) * h[a]
        fpt.append(pt)
        fbc.append(np.zeros(K.size, dtype=np.int8))
    for a in range(dim):
        area = float(np.prod(h)) / h[a]
        for side in (0, 1):
            sel = coords[:, a] == (0 if side == 0 else shape[a] - 1)
            K = idx[sel]
            e = np.zeros(dim)
            e[a] = -1.0 if side == 0 else 1.0
            fK.append(K)
            fL.append(np.full(K.size, -1))
            farea.append(np.full(K.size, area))
            fnorm.append(np.tile(e, (K.size, 1)))
            pt = centroid[K].copy()
            pt[:, a] = 0.0 if side == 0 else shape[a] * h[a]
            fpt.append(pt)
            fbc.append(np.full(K.size, 1 if (a, side) in dset else 2, dtype=np.int8))
    face_cells = np.stack([np.concatenate(fK), np.concatenate(fL)], axis=1).astype(np.int32)
    return Mesh(dim=dim, cell_volume=vol, cell_centroid=centroid, cell_k0=k0,
                face_cells=face_cells, face_area=np.concatenate(farea),
                face_normal=np.concatenate(fnorm), face_point=np.concatenate(fpt),
                face_bc=np.concatenate(fbc), shape=shape)


def voronoi_mesh(points: np.ndarray, k_cells: np.ndarray, dirichlet_x0: bool = True,
                 band: Optional[float] = None) -> Mesh:
    """Bounded Voronoi tessellation of the unit square from generator
    points: points are mirrored across the four sides, so the cells of the
    original points are clipped to the square (qhull through SciPy).

    Only the points within ``band`` of a side are mirrored (default 8 point
    spacings; ``band`` >= 1 mirrors all of them).  Within the square a point
    is never farther from an original generator than from that generator's
    mirror image, so a cell computed with a subset of the mirrors contains
    the exact clipped cell, and equals it once it lies inside the square;
    when some cell does not, the band is doubled and the diagram recomputed.

    Geometry as the two-point flux needs it on a Voronoi mesh: the cell
    "centroid" is its generator point (the face between two cells is then
    perpendicular to the segment joining them), the face point is the
    midpoint of that segment (on the bisector), the normal points from K to
    L, the face measure is the Voronoi edge length.  Boundary faces are the
    edges shared with a mirror point.  Dirichlet on the side x = 0 when
    ``dirichlet_x0``, Neumann elsewhere.  Cell volumes are polygon areas,
    summed as the triangles between the generator and each edge (a Voronoi
    cell is convex and holds its generator)."""
    from scipy.spatial import Voronoi
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    h = 8.0 / math.sqrt(max(n, 1)) if band is None else float(band)
    while True:
        sides = [(pts[:, 0] < h, lambda q: np.c_[-q[:, 0], q[:, 1]]),
                 (pts[:, 0] > 1.0 - h, lambda q: np.c_[2.0 - q[:, 0], q[:, 1]]),
                 (pts[:, 1] < h, lambda q: np.c_[q[:, 0], -q[:, 1]]),
                 (pts[:, 1] > 1.0 - h, lambda q: np.c_[q[:, 0], 2.0 - q[:, 1]])]
        allp = np.concatenate([pts] + [f(pts[sel]) for sel, f in sides])
        vor = Voronoi(allp)
        V = vor.vertices
        rp = vor.ridge_points
        rv = np.asarray(vor.ridge_vertices, dtype=np.int64)
        keep = (rp[:, 0] < n) | (rp[:, 1] < n)
        if h >= 1.0:
            break
        # every original cell bounded and inside the square: the diagram is exact
        rk = rv[keep]
        if (rk >= 0).all():
            xy = V[np.unique(rk)]
            if (xy >= -1e-9).all() and (xy <= 1.0 + 1e-9).all():
                break
        h *= 2.0
    a, b, rv = rp[keep, 0], rp[keep, 1], rv[keep]
    # orient every ridge with an original point first
    sw = a >= n
    a, b = np.where(sw, b, a), np.where(sw, a, b)
    v0, v1 = V[rv[:, 0]], V[rv[:, 1]]
    length = np.linalg.norm(v0 - v1, axis=1)

    def fan(c):   # area of the triangle (generator c, edge end points)
        e0, e1 = v0 - pts[c], v1 - pts[c]
        return 0.5 * np.abs(e0[:, 0] * e1[:, 1] - e0[:, 1] * e1[:, 0])

    vol = np.zeros(n)
    np.add.at(vol, a, fan(a))
    inner = b < n
    np.add.at(vol, b[inner], fan(np.where(inner, b, 0))[inner])
    # drop degenerate ridges (zero length) between two original cells
    ok = length > 1e-14
    a, b, length, inner = a[ok], b[ok], length[ok], inner[ok]
    other = allp[b]   # the neighbour's generator (or the mirror image across the boundary)
    d = other - pts[a]
    normal = d / np.linalg.norm(d, axis=1)[:, None]
    point = 0.5 * (pts[a] + other)
    L = np.where(inner, b, -1)
    bc = np.zeros(a.size, dtype=np.int8)
    on_x0 = (~inner) & (np.abs(point[:, 0]) < 1e-12)
    bc[~inner] = 2
    if dirichlet_x0:
        bc[on_x0] = 1
    k = np.asarray(k_cells, dtype=np.float64)
    k0 = np.zeros((n, 2, 2))
    k0[:, 0, 0] = k
    k0[:, 1, 1] = k
    return Mesh(dim=2, cell_volume=vol, cell_centroid=pts.copy(), cell_k0=k0,
                face_cells=np.stack([a, L], axis=1).astype(np.int32), face_area=length,
                face_normal=normal, face_point=point, face_bc=bc, shape=None)


def permute_mesh(prob: Problem, seed: int) -> Problem:
    """Seeded random cell permutation, face shuffle and orientation flips.

    The result is the same boundary-value problem written as an unstructured
    face list: cell ids are scrambled, faces are listed in random order and
    each interior face is oriented K->L or L->K at random.
    """
    rng = np.random.default_rng(seed)
    m = prob.mesh
    n, nf = m.n_cells, m.n_faces
    new_of_old = rng.permutation(n)
    old_of_new = np.empty(n, dtype=np.int64)
    old_of_new[new_of_old] = np.arange(n)
    forder = rng.permutation(nf)
    flip = rng.random(nf) < 0.5
    fc = m.face_cells[forder].astype(np.int64)
    fl = flip[forder] & (fc[:, 1] >= 0)
    K = np.where(fc[:, 0] >= 0, new_of_old[fc[:, 0]], -1)
    L = np.where(fc[:, 1] >= 0, new_of_old[np.maximum(fc[:, 1], 0)], -1)
    K2 = np.where(fl, L, K)
    L2 = np.where(fl, K, L)
    normal = m.face_normal[forder].copy()
    normal[fl] *= -1.0
    mesh = Mesh(dim=m.dim, cell_volume=m.cell_volume[old_of_new],
                cell_centroid=m.cell_centroid[old_of_new], cell_k0=m.cell_k0[old_of_new],
                face_cells=np.stack([K2, L2], axis=1).astype(np.int32),
                face_area=m.face_area[forder], face_normal=normal,
                face_point=m.face_point[forder], face_bc=m.face_bc[forder], shape=m.shape)
    return dataclasses.replace(prob, mesh=mesh, source=prob.source[old_of_new],
                               g_dirichlet=prob.g_dirichlet[forder],
                               g_neumann=prob.g_neumann[forder],
                               shift=None if prob.shift is None else prob.shift[old_of_new])


# ---------------------------------------------------------------- fields

def gaussian_field(shape, corr_len, rng) -> np.ndarray:
    """Standardised Gaussian random field: white noise on a 2x padded
    lattice, smoothed by a Gaussian kernel whose standard deviation is
    ``corr_len`` cells (product of 1-D kernels applied through FFT), cropped,
    then shifted/scaled to sample mean 0 and standard deviation 1.  Returned
    array is indexed [i, j(, k)] with x first."""
    shape = tuple(int(s) for s in shape)
    pad = tuple(2 * s for s in shape)
    w = rng.standard_normal(pad)
    spec = np.fft.fftn(w)
    for a, s in enumerate(pad):
        freq = np.fft.fftfreq(s)  # cycles per cell
        filt = np.exp(-2.0 * (math.pi * corr_len * freq) ** 2)
        sh = [1] * len(pad)
        sh[a] = s
        spec = spec * filt.reshape(sh)
    g = np.real(np.fft.ifftn(spec))
    g = g[tuple(slice(0, s) for s in shape)]
    g = (g - g.mean()) / g.std()
    return g


def channel_field(nx, ny, nlayers, rng, k_in=1e3, k_out=1e-3, group=5) -> np.ndarray:
    """Binary sinuous channels along y, indexed [i, j, layer].

    Per group of ``group`` layers: 4..8 channels with centre
    x_c(y) = x0 + A sin(2 pi y / lam + phi), x0 ~ U[0, nx), A ~ U[3, 12],
    lam ~ U[40, 120], phi ~ U[0, 2 pi), half-width ~ U[1.5, 4] cells, and x0
    jittered by U[-1, 1] per layer.  k = k_in inside a channel, k_out outside.
    """
    k = np.full((nx, ny, nlayers), k_out)
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    for g0 in range(0, nlayers, group):
        nch = int(rng.integers(4, 9))
        chans = []
        for _ in range(nch):
            chans.append((rng.uniform(0, nx), rng.uniform(3, 12), rng.uniform(40, 120),
                          rng.uniform(0, 2 * math.pi), rng.uniform(1.5, 4.0)))
        for lay in range(g0, min(g0 + group, nlayers)):
            for (x0, A, lam, phi, hw) in chans:
                jit = rng.uniform(-1.0, 1.0)
                xc = x0 + jit + A * np.sin(2 * math.pi * y / lam + phi)  # [ny]
                inside = np.abs(x[:, None] - xc[None, :]) <= hw          # [nx, ny]
                k[:, :, lay][inside] = k_in
    return k


# ---------------------------------------------------------------- workloads

def _flat(field):
    """[i, j(, k)] array -> cell-id order (x fastest)."""
    return np.asarray(field).transpose(tuple(range(field.ndim))[::-1]).reshape(-1)


def c1_problem(seed: int = 0) -> Problem:
    """2D unit square, 32x32 cells, cell id = i + 32 j; log10 k ~ N(0,1) per
    cell in cell-id order; kappa = exp(p); source density +1 in cell (0,0)
    and -1 in cell (31,31); p = 0 on x = 0, no flow elsewhere; 2 levels of
    4x4 aggregates with 2 local eigenvectors each."""
    rng = np.random.default_rng(seed)
    n = 32
    z = rng.standard_normal(n * n)
    k = 10.0 ** z
    mesh = cartesian_mesh((n, n), (1.0 / n, 1.0 / n), k, dirichlet=((0, 0),))
    src = np.zeros(n * n)
    src[0] = 1.0
    src[n * n - 1] = -1.0
    return Problem(mesh=mesh, alpha=1.0, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=np.zeros(mesh.n_faces), name="c1_2d_32x32",
                   box=(4, 4), m=2, n_levels=2, dp_cap_c=5.0)


# Total well rate of the 60x220x85 workload (seed 0).  Chosen so that the
# linear (kappa = 1) pressure has max |p| = 0.5 (stronger sinks can leave the
# exp(p) problem without a solution); written by the calibration script
# tests/golden/calibrate_c2_rate.py (stored in tests/golden/c2_rate.json).
C2_WELL_RATE = 0.033890383672807535


def c2_problem(seed: int = 0, rate: Optional[float] = None, permute: bool = True,
               shape=(60, 220, 85), spacing=(6.1, 3.05, 0.61), top_layers: int = 35) -> Problem:
    """3D 60x220x85 hex grid (cells 6.1 x 3.05 x 0.61 m): top 35 layers
    log-normal (ln k = 2 G, correlation length 5 cells), bottom layers binary
    sinuous channels (k = 1e3 / 1e-3); p = 0 on y = 0, no flow elsewhere;
    injector column at (0, 0) and producer column at (nx-1, ny-1) over all
    layers; kappa = exp(p); stored as an unstructured face list after a seeded
    random cell permutation.  4 levels of 4x4x4 aggregates, 3 eigenvectors."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    ktop = np.exp(2.0 * gaussian_field((nx, ny, min(top_layers, nz)), 5.0, rng))
    kbot = channel_field(nx, ny, nz - min(top_layers, nz), rng) if nz > top_layers else None
    kf = ktop if kbot is None else np.concatenate([ktop, kbot], axis=2)
    k = _flat(kf)
    mesh = cartesian_mesh(shape, spacing, k, dirichlet=((1, 0),))
    q = C2_WELL_RATE if rate is None else rate
    vol = float(mesh.cell_volume[0])
    src = np.zeros(mesh.n_cells)
    for kz in range(nz):
        src[0 + nx * (0 + ny * kz)] += q / (nz * vol)
        src[(nx - 1) + nx * ((ny - 1) + ny * kz)] -= q / (nz * vol)
    prob = Problem(mesh=mesh, alpha=1.0, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=np.zeros(mesh.n_faces), name="c2_3d_60x220x85",
                   box=(4, 4, 4), m=3, n_levels=4, dp_cap_c=5.0)
    if permute:
        prob = permute_mesh(prob, seed + 1)
    return prob


def bilinear_sample(field: np.ndarray, xy: np.ndarray) -> np.ndarray:
    """Values of a field given on the cell centres of a uniform lattice over
    the unit square ([i, j], x first) at points xy, by bilinear
    interpolation (clamped at the border)."""
    nx, ny = field.shape
    fx = np.clip(xy[:, 0] * nx - 0.5, 0.0, nx - 1.0)
    fy = np.clip(xy[:, 1] * ny - 0.5, 0.0, ny - 1.0)
    i0 = np.minimum(np.floor(fx).astype(np.int64), nx - 2)
    j0 = np.minimum(np.floor(fy).astype(np.int64), ny - 2)
    tx, ty = fx - i0, fy - j0
    return ((1 - tx) * (1 - ty) * field[i0, j0] + tx * (1 - ty) * field[i0 + 1, j0]
            + (1 - tx) * ty * field[i0, j0 + 1] + tx * ty * field[i0 + 1, j0 + 1])


def voronoi_problem(n_points: int = 2000, seed: int = 0, sigma: float = 3.0, corr_len: float = 0.01,
                    alpha: float = 2.0, lattice: int = 0, rate: Optional[float] = None, n_levels: int = 3,
                    greedy_size: int = 64, m: int = 3, eig_threshold: float = 0.0, m_min: int = 2,
                    greedy_size_coarse: int = 0) -> Problem:
    """Unstructured 2-D problem on the Voronoi mesh of ``n_points`` seeded
    uniform points in the unit square: ln k = sigma G, G a standardised
    Gaussian random field of correlation length ``corr_len`` (in units of
    the square) sampled from a lattice of ``lattice``^2 cells (default: 4
    cells per point spacing, at most 4096) by bilinear interpolation;
    kappa = exp(alpha p); p = 0 on x = 0, no flow elsewhere; a source and a
    sink of equal total rate in the cells whose generators are nearest to
    (0.05, 0.05) and (0.95, 0.95).  The caller chooses the rate (default
    1.0): with kappa = exp(alpha p) a strong sink leaves the problem without a
    solution, and the rule used with these meshes is alpha max|p| = 0.5 for
    the kappa = 1 pressure (p is linear in the rate there).  Greedy
    aggregates of about ``greedy_size`` cells, m local eigenvectors (with
    eig_threshold > 0: those with eigenvalue up to eig_threshold times the
    largest, between m_min and m)."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n_points, 2))
    if lattice <= 0:
        lattice = int(min(4096, max(64, 4 * math.sqrt(n_points))))
    g = gaussian_field((lattice, lattice), corr_len * lattice, rng)
    k = np.exp(sigma * bilinear_sample(g, pts))
    mesh = voronoi_mesh(pts, k)
    src = np.zeros(n_points)
    q = 1.0 if rate is None else rate
    i_in = int(np.argmin(np.sum((pts - np.array([0.05, 0.05])) ** 2, axis=1)))
    i_out = int(np.argmin(np.sum((pts - np.array([0.95, 0.95])) ** 2, axis=1)))
    src[i_in] += q / mesh.cell_volume[i_in]
    src[i_out] -= q / mesh.cell_volume[i_out]
    prob = Problem(mesh=mesh, alpha=alpha, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=np.zeros(mesh.n_faces), name=f"voronoi_2d_{n_points}", box=(), m=m,
                   n_levels=n_levels, dp_cap_c=5.0)
    return dataclasses.replace(prob, greedy_size=greedy_size, eig_threshold=eig_threshold, m_min=m_min,
                               greedy_size_coarse=greedy_size_coarse)


def served_problem(seed: int, n_min: int = 32 ** 2, n_max: int = 64 ** 3, dims=(2, 3), sigma: float = 2.0,
                   corr_len: float = 3.0) -> Problem:
    """One model of the served and batched workloads: dimension drawn from
    ``dims``, cell count log-uniform in [n_min, n_max], side = round(N^(1/d))
    on the unit square / cube; ln k = sigma G, G a standardised Gaussian
    random field of correlation length ``corr_len`` cells; kappa = exp(p);
    p = 0 on x = 0, no flow elsewhere; zero-mean random source density (the
    caller scales it: a strong sink can leave exp(p) without a root, and the
    rule used is max|p| = 0.5 for the kappa = 1 pressure); box aggregates of 4 cells per axis with 2 local eigenvectors, levels
    until the coarsest has at most a few hundred cells."""
    rng = np.random.default_rng(seed)
    d = int(rng.choice(dims))
    n = math.exp(rng.uniform(math.log(n_min), math.log(n_max)))
    side = max(8, int(round(n ** (1.0 / d))))
    shape = (side,) * d
    nc = side ** d
    k = np.exp(sigma * _flat(gaussian_field(shape, corr_len, rng)))
    mesh = cartesian_mesh(shape, tuple(1.0 / side for _ in shape), k, dirichlet=((0, 0),))
    src = rng.standard_normal(nc)
    src -= src.mean()
    levels, c = 1, nc
    while c > 400 and levels < 8:
        c //= 4 ** d
        levels += 1
    return Problem(mesh=mesh, alpha=1.0, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=np.zeros(mesh.n_faces), name=f"served_{d}d_{side}_s{seed}", box=(4,) * d, m=2,
                   n_levels=levels, dp_cap_c=5.0)


def _c4_shape(rng):
    """Aggregate edge a ~ U{4..8}, then the three box edges from U{16..96},
    an edge drawn again when the box rule would merge its remainder into a
    block of more than 8 cells."""
    a = int(rng.integers(4, 9))
    shape = []
    while len(shape) < 3:
        n = int(rng.integers(16, 97))
        r = n % a
        if 0 < r and 2 * r < a and a + r > 8:
            continue
        shape.append(n)
    return tuple(shape), a


def c4_shape(i: int, seed: int = 4):
    """(shape, a) of instance i of the batched workload, without its mesh."""
    return _c4_shape(np.random.default_rng([seed, i]))


def c4_problem(i: int, seed: int = 4) -> Problem:
    """Instance i of the batched workload (512 instances): a box of
    n_x x n_y x n_z cubic cells with every edge drawn from U{16..96}, ln k =
    2G with correlation length 5 cells, kappa = exp(p), p = 0 on x = 0, no
    flow elsewhere, a zero-mean random source density (the caller scales
    it: the rule used is max|p| = 0.25 for the kappa = 1 pressure); box
    aggregates of edge a ~ U{4..8} (64 to 512 cells) with 3 local
    eigenvectors; 2 levels when a >= 5 (a coarse aggregate of up to
    (a + 2)^3 coarse cells of 3 unknowns each would exceed the 512 unknowns
    the local dense solvers take), else levels until the coarsest has at
    most 400 cells (at most 4).  An edge
    whose remainder the box rule would merge into a block of more than 8
    cells (a = 7 or 8 with 0 < n mod a < a/2) is drawn again, so that no
    aggregate exceeds 512 cells."""
    rng = np.random.default_rng([seed, i])
    shape, a = _c4_shape(rng)
    h = 1.0 / max(shape)
    k = np.exp(2.0 * _flat(gaussian_field(shape, 5.0, rng)))
    mesh = cartesian_mesh(shape, (h, h, h), k, dirichlet=((0, 0),))
    n = mesh.n_cells
    src = rng.standard_normal(n)
    src -= src.mean()
    if a >= 5:
        levels = 2
    else:
        levels, c = 1, n
        while c > 400 and levels < 4:
            c //= a ** 3
            levels += 1
    return Problem(mesh=mesh, alpha=1.0, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=np.zeros(mesh.n_faces), name=f"c4_{i}_{'x'.join(map(str, shape))}_a{a}",
                   box=(a, a, a), m=3, n_levels=levels, dp_cap_c=5.0)


# Source rate of the 2,000,000-point Voronoi workload (seed 3), chosen so that
# alpha max |p| = 0.5 for the linear (kappa = 1) pressure; written by the
# calibration script tests/golden/calibrate_c3_rate.py (stored in
# tests/golden/c3_rate.json).
C3_RATE = 0.17304720191344097


def c3_problem(rate: Optional[float] = None) -> Problem:
    """The unstructured workload: the Voronoi mesh of 2,000,000 seeded uniform
    points in the unit square (seed 3), ln k = 3G with correlation length
    0.01, kappa = exp(2p), p = 0 on x = 0, a source pair near (0.05, 0.05)
    and (0.95, 0.95); greedy aggregates of about 64 cells on 2 levels, 2 to 6
    eigenvectors per aggregate by the threshold 0.1."""
    q = C3_RATE if rate is None else rate
    if q is None:
        raise ValueError("C3_RATE is not calibrated")
    return voronoi_problem(n_points=2000000, seed=3, sigma=3.0, corr_len=0.01, alpha=2.0, rate=q, n_levels=2,
                           greedy_size=64, m=6, eig_threshold=0.1, m_min=2)


def small_problem(shape, seed=0, sigma=1.0, alpha=1.0, dirichlet=((0, 0),), box=None, m=2,
                  n_levels=2, spacing=None, g_d_scale=0.0, g_n_scale=0.0, src_scale=1.0,
                  anisotropic=False, permute=False, dp_cap_c=5.0) -> Problem:
    """Small seeded test problem: ln k = sigma * N(0,1) i.i.d. per cell,
    zero-mean random source density, optional random Dirichlet and Neumann
    data, optional diagonal anisotropic K0 and optional permutation."""
    rng = np.random.default_rng(seed)
    shape = tuple(shape)
    dim = len(shape)
    n = int(np.prod(shape))
    if spacing is None:
        spacing = tuple(1.0 / s for s in shape)
    if anisotropic:
        k = np.exp(sigma * rng.standard_normal((n, dim)))
    else:
        k = np.exp(sigma * rng.standard_normal(n))
    mesh = cartesian_mesh(shape, spacing, k, dirichlet=dirichlet)
    src = rng.standard_normal(n)
    src -= src.mean()
    src *= src_scale
    gd = g_d_scale * rng.standard_normal(mesh.n_faces)
    gn = g_n_scale * rng.standard_normal(mesh.n_faces)
    gd[mesh.face_bc != 1] = 0.0
    gn[mesh.face_bc != 2] = 0.0
    if box is None:
        box = tuple(min(2, s) for s in shape)
    prob = Problem(mesh=mesh, alpha=alpha, source=src, g_dirichlet=gd, g_neumann=gn,
                   name=f"small_{'x'.join(map(str, shape))}_s{seed}", box=tuple(box), m=m,
                   n_levels=n_levels, dp_cap_c=dp_cap_c)
    if permute:
        prob = permute_mesh(prob, seed + 7)
    return prob


# Hydraulic parameters of Example 3's table (a, beta, k0 in cm/day).
RICHARDS_MEDIA = {"loam": (1.246e2, 1.77, 1.067), "sand": (1.175e6, 4.74, 8.160e2)}


def richards_problem(shape=(40, 10), size=(400.0, 100.0), medium="loam", seed=0, sigma=0.0,
                     psi_dry=-300.0, psi_wet=-20.0, wet_frac=0.25, box=(4, 4), m=2, n_levels=2,
                     permute=False) -> Problem:
    """Static Richards-type problem on a vertical 2-D section (cm): the
    conductivity K0 kappa(psi) with kappa = a / (a + |psi|^beta) of the
    medium, the pressure head psi = p - z and z the height (cell centroid).
    Zero source; water table psi = 0 on the bottom (p = 0); on the top the
    head psi_wet over the first wet_frac of the width and psi_dry elsewhere
    (p = psi + height); no flow through the sides.  K0 = k0 exp(sigma G)
    with G i.i.d. standard normal (sigma = 0: the homogeneous medium).  The
    paper's boundary layout is given only as a figure, so this one is a
    stand-in with the same kind of wet/dry contrast."""
    a, beta, k0 = RICHARDS_MEDIA[medium]
    rng = np.random.default_rng(seed)
    shape = tuple(int(v) for v in shape)
    spacing = tuple(size[d] / shape[d] for d in range(2))
    n = shape[0] * shape[1]
    k = k0 * np.exp(sigma * rng.standard_normal(n))
    mesh = cartesian_mesh(shape, spacing, k, dirichlet=((1, 0), (1, 1)))
    gd = np.zeros(mesh.n_faces)
    top = (mesh.face_bc == 1) & (mesh.face_point[:, 1] > 0.5 * size[1])
    wet = top & (mesh.face_point[:, 0] < wet_frac * size[0])
    gd[top] = psi_dry + size[1]
    gd[wet] = psi_wet + size[1]
    prob = Problem(mesh=mesh, alpha=0.0, source=np.zeros(n), g_dirichlet=gd, g_neumann=np.zeros(mesh.n_faces),
                   name=f"richards_{medium}_{shape[0]}x{shape[1]}_s{seed}", box=tuple(box), m=m,
                   n_levels=n_levels, kappa_kind="richards", kappa_a=a, kappa_beta=beta,
                   shift=mesh.cell_centroid[:, 1].copy())
    if permute:
        prob = permute_mesh(prob, seed + 7)
    return prob
