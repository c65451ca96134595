"""The bounded Voronoi mesh of the unstructured workloads: mirroring only
the points near the sides gives the same cells, faces and geometry as
mirroring every point (up to face order and orientation), the cell areas
tile the unit square, and each boundary face lies on a side."""
import numpy as np
import pytest

from problems.grids import voronoi_mesh


def canon(m):
    fc = m.face_cells.astype(np.int64).copy()
    nrm = m.face_normal.copy()
    flip = (fc[:, 1] >= 0) & (fc[:, 0] > fc[:, 1])
    fc[flip] = fc[flip][:, ::-1]
    nrm[flip] *= -1.0
    P = m.face_point
    o = np.lexsort((np.round(P[:, 1], 9), np.round(P[:, 0], 9), fc[:, 1], fc[:, 0]))
    return fc[o], P[o], m.face_area[o], m.face_bc[o], nrm[o]


@pytest.mark.parametrize("n,seed", [(40, 0), (3000, 1)])
def test_band_mirrors_match_full_mirrors(n, seed):
    pts = np.random.default_rng(seed).random((n, 2))
    k = np.ones(n)
    full = voronoi_mesh(pts, k, band=1.0)
    fast = voronoi_mesh(pts, k)
    a, b = canon(full), canon(fast)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[3], b[3])
    for x, y in zip((a[1], a[2], a[4]), (b[1], b[2], b[4])):
        np.testing.assert_allclose(y, x, rtol=0.0, atol=1e-13)
    np.testing.assert_allclose(fast.cell_volume, full.cell_volume, rtol=1e-12, atol=0.0)


def test_band_too_narrow_is_widened():
    # a band far below the point spacing: cells reach outside the square
    # until the band has been doubled enough times
    pts = np.random.default_rng(2).random((500, 2))
    narrow = voronoi_mesh(pts, np.ones(500), band=1e-4)
    full = voronoi_mesh(pts, np.ones(500), band=1.0)
    np.testing.assert_allclose(narrow.cell_volume, full.cell_volume, rtol=1e-12, atol=0.0)
    assert narrow.n_faces == full.n_faces


def test_areas_tile_the_square_and_boundary_faces_lie_on_sides():
    pts = np.random.default_rng(4).random((5000, 2))
    m = voronoi_mesh(pts, np.ones(5000))
    assert abs(m.cell_volume.sum() - 1.0) < 1e-12
    assert (m.cell_volume > 0).all()
    bnd = m.face_cells[:, 1] < 0
    P = m.face_point[bnd]
    on_side = np.minimum.reduce([np.abs(P[:, 0]), np.abs(P[:, 0] - 1), np.abs(P[:, 1]), np.abs(P[:, 1] - 1)])
    assert on_side.max() < 1e-12
    # total boundary length is the perimeter
    assert abs(m.face_area[bnd].sum() - 4.0) < 1e-12
    # Dirichlet exactly on x = 0
    dir_ = m.face_bc == 1
    assert np.all(np.abs(m.face_point[dir_, 0]) < 1e-12)
    assert abs(m.face_area[dir_].sum() - 1.0) < 1e-12
