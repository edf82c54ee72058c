"""Pins of the CPU oracle's periodic Becke weights (Sec. 2.8, eqs.
becke_weight_definition, becke_vicinity_definition, becke_mu_definition,
becke_switch_definition, becke_grid_integrate_one) against values that
symmetry and the integral of the partition fix, independently of the
formulas:

- a point at an atom belongs wholly to it; the centroid of an equilateral
  triangle or a regular tetrahedron of atoms is shared equally; any point of
  the bisecting plane of two atoms is shared half and half (cells far larger
  than the cutoff sphere: the molecular case);
- one atom in a cubic cell: the face centre, edge centre and corner of its
  Wigner-Seitz cube are shared by 2, 4 and 8 images (large cutoff);
- the grid weights integrate the unit function to the cell volume within the
  excess the paper reports for a 17 bohr sphere (0.01-0.25 %; 0.27 % here
  with a product grid);
- rotating or translating the whole system changes no weight.
"""
import numpy as np

from oracle import becke
from paper_2410_22278_amd import inputs

BIG = np.eye(3) * 300.0


def _w(cell, xyz, pts, origin, **kw):
    return becke.becke_weights(cell, xyz, np.atleast_2d(pts), np.atleast_1d(origin), **kw)


def test_point_at_atom_is_its_own():
    xyz = np.array([[0.0, 0.0, 0.0], [2.1, 0.3, -0.4], [-1.0, 1.9, 0.8]])
    for a in range(3):
        assert _w(BIG, xyz, xyz[a], a)[0] == 1.0
        for b in range(3):
            if b != a:
                assert _w(BIG, xyz, xyz[a], b)[0] == 0.0


def test_centroids_shared_equally():
    tri = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0], [1.0, np.sqrt(3.0), 0.0]])
    c = tri.mean(axis=0)
    w = [_w(BIG, tri, c, a)[0] for a in range(3)]
    assert np.allclose(w, 1.0 / 3.0, rtol=0, atol=1e-14)
    tet = np.array([[1.0, 1.0, 1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]]) * 1.3
    w = [_w(BIG, tet, np.zeros(3), a)[0] for a in range(4)]
    assert np.allclose(w, 0.25, rtol=0, atol=1e-14)


def test_bisecting_plane_half_and_half():
    rng = np.random.default_rng(3)
    xyz = np.array([[0.0, 0.0, 0.0], [2.4, 0.0, 0.0]])
    pts = np.column_stack([np.full(20, 1.2), rng.uniform(-3, 3, 20), rng.uniform(-3, 3, 20)])
    for a in range(2):
        assert np.allclose(becke.becke_weights(BIG, xyz, pts, np.full(20, a)), 0.5, rtol=0, atol=1e-14)


def test_wigner_seitz_points_of_one_atom():
    a = 5.0
    cell = np.eye(3) * a
    xyz = np.zeros((1, 3))
    pts = np.array([[a / 2, 0, 0], [a / 2, a / 2, 0], [a / 2, a / 2, a / 2]])
    w = becke.becke_weights(cell, xyz, pts, np.zeros(3, int), rcut=25.0)
    assert abs(w[0] - 0.5) < 2e-4
    assert abs(w[1] - 0.25) < 1e-3
    assert abs(w[2] - 0.125) < 2e-3


def test_grid_integrates_the_cell_volume():
    cell = np.eye(3) * 5.0
    cell[1, 0] = 0.4
    cell[2, 1] = -0.3
    xyz = np.array([[0.1, 0.2, 0.3]])
    pts, wq, org = inputs.atom_grid(xyz, 40, 12, 24, 1.0)
    w = becke.becke_weights(cell, xyz, pts, org, rcut=17.0)
    ratio = float((wq * w).sum()) / abs(np.linalg.det(cell))
    assert 1.0 < ratio < 1.005, ratio


def test_rotation_and_translation_invariance():
    rng = np.random.default_rng(5)
    cell = np.array([[6.0, 0.0, 0.0], [1.1, 5.5, 0.0], [0.4, -0.7, 6.2]])
    xyz = np.array([[0.3, 0.2, 0.1], [2.9, 2.4, 3.3]])
    pts = np.concatenate([xyz[0] + rng.normal(0, 1.5, (30, 3)), xyz[1] + rng.normal(0, 1.5, (30, 3))])
    org = np.repeat([0, 1], 30)
    w0 = becke.becke_weights(cell, xyz, pts, org, rcut=10.0)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    w1 = becke.becke_weights(cell @ q, xyz @ q, pts @ q, org, rcut=10.0)
    t = np.array([3.7, -1.2, 0.5])
    w2 = becke.becke_weights(cell, xyz + t, pts + t, org, rcut=10.0)
    assert np.abs(w0).max() > 0.1
    assert np.allclose(w1, w0, rtol=0, atol=1e-12)
    assert np.allclose(w2, w0, rtol=0, atol=1e-12)


def test_point_inside_another_atom_gets_zero():
    xyz = np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 0.0]])
    # next to atom 1, far from atom 0: one switching factor underflows delta
    assert _w(BIG, xyz, [2.99, 0.0, 0.0], 0, delta=1e-14)[0] == 0.0


def test_switch_range():
    u = np.linspace(-1, 1, 201)
    s = becke.switch(u)
    assert s[0] == 1.0 and s[-1] == 0.0 and s[100] == 0.5
    assert np.all(np.diff(s) <= 0)
    assert np.allclose(s + s[::-1], 1.0, rtol=0, atol=1e-15)
