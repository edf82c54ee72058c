"""Pins of the oracle's Gamma-point one-electron terms (overlap S, kinetic T,
nuclear attraction V, nuclear repulsion E_nuc) against what the mathematics
fixes:

- T: the 1-D integrals <g_i| d^2/dx^2 |g_j> of monomial Gaussians by
  Gauss-Hermite quadrature (exact for polynomial times Gaussian) with the
  analytic second derivative, and the s closed form
  T = (ab/p)(3 - 2 ab/p |A-B|^2) S;
- V: independence of omega (the Ewald split of the point-charge potential,
  Sec. 2.3, is exact), and the compact-charge limit: a normalised s Gaussian
  of exponent a at A, away from the charges, sees
  q (phi(A - C) + pi/(2 a V)), phi the Ewald pair potential of the
  point-charge energy (pinned separately by the NaCl Madelung constant) and
  pi/(2 a V) the spread of the Gaussian in the mean-zero potential, whose
  Laplacian away from the charges is 4 pi/V;
- S: the same Gamma overlap as the one pinned by T S T^T = I.
"""
import math

import numpy as np

from paper_2410_22278_amd.inputs import Thresholds
from tests._systems import make_system


def _dfact(n):
    return 1.0 if n <= 0 else n * _dfact(n - 2)


def _norm(a, c):
    return (2 * a / math.pi) ** 0.75 * math.sqrt((4 * a) ** sum(c) / (_dfact(2 * c[0] - 1) * _dfact(2 * c[1] - 1)
                                                                    * _dfact(2 * c[2] - 1)))


def _quad_1d(i, a, A, j, b, B, deriv2=False):
    """int (x-A)^i e^{-a(x-A)^2} [d^2/dx^2] (x-B)^j e^{-b(x-B)^2} dx by
    Gauss-Hermite quadrature on the product Gaussian."""
    p = a + b
    P = (a * A + b * B) / p
    K = math.exp(-a * b / p * (A - B) ** 2)
    xs, ws = np.polynomial.hermite.hermgauss(30)
    x = P + xs / math.sqrt(p)
    u, v = x - A, x - B
    if deriv2:
        g = j * (j - 1) * v ** (j - 2) if j >= 2 else 0.0 * v
        g = g - 2 * b * (2 * j + 1) * v ** j + 4 * b * b * v ** (j + 2)
    else:
        g = v ** j
    return K * float(np.sum(ws * u ** i * g)) / math.sqrt(p)


def _comps(l):
    """Cartesian components in the library's order x^l, x^(l-1) y, ..."""
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def test_kinetic_vs_quadrature(oracle_mod):
    rng = np.random.default_rng(5)
    shells, xyz = [], np.array([[0.3, -0.2, 0.1], [1.1, 0.7, -0.9]])
    for atom in range(2):
        for l in (0, 1, 2):
            shells.append((atom, l, [rng.uniform(0.3, 3.0)], [1.0]))
    s = make_system(np.eye(3) * 40.0, xyz, shells, 0.3)
    r = oracle_mod.one_electron(s, parts="self")
    T = r["Tc"]
    offs = np.cumsum([0] + [(l + 1) * (l + 2) // 2 for _, l, _, _ in shells])
    worst = 0.0
    for A, (ia, la, ea, _) in enumerate(shells):
        for B, (ib, lb, eb, _) in enumerate(shells):
            a, b = ea[0], eb[0]
            for i, ci in enumerate(_comps(la)):
                for j, cj in enumerate(_comps(lb)):
                    ov = [_quad_1d(ci[x], a, xyz[ia][x], cj[x], b, xyz[ib][x]) for x in range(3)]
                    d2 = [_quad_1d(ci[x], a, xyz[ia][x], cj[x], b, xyz[ib][x], deriv2=True) for x in range(3)]
                    ref = -0.5 * (d2[0] * ov[1] * ov[2] + ov[0] * d2[1] * ov[2] + ov[0] * ov[1] * d2[2])
                    ref *= _norm(a, ci) * _norm(b, cj)
                    worst = max(worst, abs(T[offs[A] + i, offs[B] + j] - ref))
    assert worst < 1e-12


def test_kinetic_s_closed_form(oracle_mod):
    xyz = np.array([[0.0, 0.0, 0.0], [0.8, -0.5, 1.2]])
    a, b = 0.7, 1.9
    s = make_system(np.eye(3) * 40.0, xyz, [(0, 0, [a], [1.0]), (1, 0, [b], [1.0])], 0.3)
    r = oracle_mod.one_electron(s, parts="self")
    p, R2 = a + b, float(np.sum((xyz[0] - xyz[1]) ** 2))
    S01 = r["S"][0, 1]
    assert abs(r["T"][0, 1] - (a * b / p) * (3 - 2 * a * b / p * R2) * S01) < 1e-14
    assert abs(r["T"][0, 0] - 1.5 * a) < 1e-14       # <g|-1/2 lap|g> = 3a/2 for a normalised s


def test_overlap_same_as_gamma_overlap(oracle_mod):
    from paper_2410_22278_amd import inputs
    s = inputs.small_cell(21, natom=2, recipe=((0, 0), (1, 0), (2, 1)), a_ang=3.2, lo=0.3, hi=4.0)
    r = oracle_mod.one_electron(s, parts="self")
    assert np.abs(r["Sc"] - oracle_mod.overlap_cart(s)).max() < 1e-15


def test_nuclear_attraction_omega_invariance(oracle_mod):
    from paper_2410_22278_amd import inputs
    s = inputs.small_cell(23, natom=3, recipe=((0, 0), (1, 0), (2, 1)), a_ang=3.4, lo=0.3, hi=4.0, skew=0.1,
                          delta=1e-14)
    s.charge = np.array([3.0, 1.0, 2.0])
    v = [oracle_mod.one_electron(s, omega=w)["V"] for w in (0.35, 0.6, 1.1)]
    e = [oracle_mod.one_electron(s, omega=w)["E_nuc"] for w in (0.35, 0.6, 1.1)]
    assert np.abs(v[0] - v[1]).max() < 1e-10 and np.abs(v[0] - v[2]).max() < 1e-10
    assert abs(e[0] - e[1]) < 1e-10 and abs(e[0] - e[2]) < 1e-10


def test_nuclear_attraction_compact_charge_limit(oracle_mod):
    L = 9.0
    a = 4.0e3
    A = np.array([1.0, 2.0, 3.0])
    Cs = np.array([[5.5, 1.0, 7.0], [2.0, 6.5, 0.5]])
    q = np.array([1.5, -0.7])
    xyz = np.vstack([A, Cs])
    s = make_system(np.eye(3) * L, xyz, [(0, 0, [a], [1.0])], 0.5, thr=Thresholds.uniform(1e-15))
    s.charge = np.zeros(3)
    V = oracle_mod.one_electron(s, charges=np.array([0.0, *q]))["V"][0, 0]
    # Ewald pair potential phi(A - C) from the point-charge energy of A and C
    cell = np.eye(3) * L
    ref = 0.0
    for C, qc in zip(Cs, q):
        two = np.vstack([A, C])
        e11 = oracle_mod.ewald_energy(two, np.array([1.0, 1.0]), cell, 0.5, 1e-16, 1e-16)
        e10 = oracle_mod.ewald_energy(two, np.array([1.0, 0.0]), cell, 0.5, 1e-16, 1e-16)
        e01 = oracle_mod.ewald_energy(two, np.array([0.0, 1.0]), cell, 0.5, 1e-16, 1e-16)
        ref += qc * (e11 - e10 - e01 + math.pi / (2 * a * L ** 3))
    assert abs(V - ref) < 1e-9, (V, ref)
