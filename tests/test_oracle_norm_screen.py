"""Pins of the oracle's basis normalisation, spherical-d transform and
short-range Cauchy-Schwarz factors against what the mathematics fixes.

- Single-centre overlap: every contracted shell is rescaled to unit
  single-centre self-overlap (Sec. 2.1, eq. local_normalization and the note
  that the crystalline function itself is not normalised), and the real solid
  harmonics of a spherical d shell are orthonormal and orthogonal to the s and
  p shells of the same atom.  In a 60-bohr cell the images do not contribute,
  so T S T^T of one atom must be the identity on those blocks; a wrong
  normalisation, renormalisation or transform coefficient breaks it.
  Normalised Cartesian d functions have the textbook overlaps
  <xx|xx> = 1, <xx|yy> = 1/3 and vanishing mixed overlaps.
- Short-range Cauchy-Schwarz factor (Sec. 2.4, eq. local_cauchy_schwarz_bound
  with the erfc kernel): closed form for s pairs, the component maximum of
  the oracle's own diagonal integrals for p and d pairs, and the inequality
  itself on random quartets.
"""
import math

import numpy as np
import pytest

from paper_2410_22278_amd.inputs import Thresholds
from tests._systems import make_system


def _dfact(n):
    return 1.0 if n <= 0 else n * _dfact(n - 2)


def _cart_norm(a, c):
    """Normalisation of x^i y^j z^k e^{-a r^2} (textbook)."""
    l = sum(c)
    return (2 * a / math.pi) ** 0.75 * math.sqrt((4 * a) ** l / (_dfact(2 * c[0] - 1) * _dfact(2 * c[1] - 1)
                                                              * _dfact(2 * c[2] - 1)))


def _one_atom(pure_d, seed=7):
    rng = np.random.default_rng(seed)
    shells = []
    pure = []
    for l in (0, 1, 2):
        e = np.exp(rng.uniform(np.log(0.15), np.log(12.0), 3))
        c = rng.uniform(0.1, 1.0, 3)
        shells.append((0, l, e, c))
        pure.append(1 if (l == 2 and pure_d) else 0)
    return make_system(np.eye(3) * 60.0, np.array([[1.0, -2.0, 0.5]]), shells, 0.3,
                       thr=Thresholds.uniform(1e-14), pure=pure)


def test_single_centre_overlap_spherical_is_identity(oracle_mod):
    s = _one_atom(pure_d=True)
    S = oracle_mod.overlap_cart(s)
    T = oracle_mod.sph_transform(s)
    M = T @ S @ T.T
    assert M.shape == (9, 9)          # s (1) + p (3) + spherical d (5)
    assert np.abs(M - np.eye(9)).max() < 1e-12


def test_single_centre_overlap_cartesian_d(oracle_mod):
    s = _one_atom(pure_d=False)
    S = oracle_mod.overlap_cart(s)
    T = oracle_mod.sph_transform(s)
    M = T @ S @ T.T
    assert M.shape == (10, 10)        # s + p + 6 Cartesian d
    # s and p: unit self-overlap, mutually orthogonal (parity)
    assert np.abs(M[:4, :4] - np.eye(4)).max() < 1e-12
    assert np.abs(M[1:4, 4:]).max() < 1e-12            # p with d: odd parity
    d = M[4:, 4:]
    comps = [(2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    for i, ci in enumerate(comps):
        for j, cj in enumerate(comps):
            if i == j:
                ref = 1.0
            elif max(ci) == 2 and max(cj) == 2:
                ref = 1.0 / 3.0          # <xx|yy> of normalised Cartesian d
            else:
                ref = 0.0
            assert abs(d[i, j] - ref) < 1e-12, (ci, cj, d[i, j])


def _pairs_of(oracle_mod, s):
    pl = oracle_mod.pair_list(s)
    offs = np.cumsum([0] + list(s.shell_nprim))
    return pl, offs


def test_sr_schwarz_factor_s_closed_form(oracle_mod):
    """(ss|ss)_SR at zero separation is 2 pi^{5/2}/(p^2 sqrt(2p)) K^2 (1 - c),
    c = w/sqrt(p/2 + w^2) (the erfc difference of the Boys split at T = 0)."""
    rng = np.random.default_rng(3)
    w = 0.35
    shells = [(0, 0, [rng.uniform(0.2, 5.0)], [1.0]), (1, 0, [rng.uniform(0.2, 5.0)], [1.0])]
    s = make_system(np.eye(3) * 40.0, np.array([[0.0, 0.0, 0.0], [0.9, -0.4, 0.3]]), shells, w)
    pl, offs = _pairs_of(oracle_mod, s)
    for k in range(len(pl["Q"])):
        if np.any(pl["n2"][k] != 0):
            continue
        sa, sb = int(pl["sa"][k]), int(pl["sb"][k])
        a, b = s.exps[offs[sa]], s.exps[offs[sb]]
        p = a + b
        d = s.xyz[s.shell_atom[sa]] - s.xyz[s.shell_atom[sb]]
        K = math.exp(-a * b / p * float(d @ d))
        c = w / math.sqrt(p / 2 + w * w)
        ref = _cart_norm(a, (0, 0, 0)) * _cart_norm(b, (0, 0, 0)) * math.sqrt(
            2 * math.pi ** 2.5 / (p * p * math.sqrt(2 * p)) * K * K * (1 - c))
        assert abs(pl["Q"][k] - ref) <= 1e-13 * ref, (sa, sb)


def test_sr_schwarz_factor_p_d_and_inequality(oracle_mod):
    """p and d pairs: Q equals the largest normalised diagonal element of the
    oracle's primitive SR integrals (pinned separately by closed forms and the
    centre-derivative identity), and |(ab|cd)_SR| <= Q_ab Q_cd holds for
    random quartets of such pairs, component by component."""
    rng = np.random.default_rng(11)
    w = 0.3
    xyz = np.array([[0.0, 0.0, 0.0], [1.1, 0.6, -0.8], [-0.7, 1.3, 0.9]])
    shells = []
    for atom in range(3):
        for l in (0, 1, 2):
            shells.append((atom, l, [rng.uniform(0.3, 4.0)], [1.0]))
    s = make_system(np.eye(3) * 40.0, xyz, shells, w)
    pl, offs = _pairs_of(oracle_mod, s)
    recs = []
    for k in range(len(pl["Q"])):
        if np.any(pl["n2"][k] != 0):
            continue
        sa, sb = int(pl["sa"][k]), int(pl["sb"][k])
        la, lb = int(s.shell_l[sa]), int(s.shell_l[sb])
        a, b = float(s.exps[offs[sa]]), float(s.exps[offs[sb]])
        A, B = s.xyz[s.shell_atom[sa]], s.xyz[s.shell_atom[sb]]
        blk = oracle_mod.eri_prim(1, (la, lb, la, lb), (a, b, a, b), (A, B, A, B), w)
        ca, cb = oracle_mod.cart_components(la), oracle_mod.cart_components(lb)
        best = 0.0
        for i, ci in enumerate(ca):
            for j, cj in enumerate(cb):
                v = blk[i, j, i, j] * (_cart_norm(a, ci) * _cart_norm(b, cj)) ** 2
                assert v > 0
                best = max(best, v)
        assert abs(pl["Q"][k] - math.sqrt(best)) <= 1e-12 * math.sqrt(best), (la, lb)
        recs.append((la, lb, a, b, A, B, pl["Q"][k]))
    assert {(r[0], r[1]) for r in recs} == {(x, y) for x in range(3) for y in range(3)}
    worst = 0.0
    for _ in range(60):
        r1, r2 = recs[rng.integers(len(recs))], recs[rng.integers(len(recs))]
        la, lb, a, b, A, B, Q1 = r1
        lc, ld, c, d, C, D, Q2 = r2
        shift = rng.uniform(-1.5, 1.5, 3)
        blk = oracle_mod.eri_prim(1, (la, lb, lc, ld), (a, b, c, d), (A, B, C + shift, D + shift), w)
        na = [_cart_norm(a, x) for x in oracle_mod.cart_components(la)]
        nb = [_cart_norm(b, x) for x in oracle_mod.cart_components(lb)]
        nc = [_cart_norm(c, x) for x in oracle_mod.cart_components(lc)]
        nd = [_cart_norm(d, x) for x in oracle_mod.cart_components(ld)]
        val = np.abs(np.einsum("ijkl,i,j,k,l->ijkl", blk, na, nb, nc, nd)).max()
        worst = max(worst, val / (Q1 * Q2))
    assert worst <= 1.0 + 1e-12
    assert worst > 1e-3              # the bound is not vacuous


def test_d_shell_screening_truncation(oracle_mod):
    """What the quartet screen drops on a d-shell cell (2 atoms, 2s+1p+1d
    spherical, exponents down to 0.15, omega 0.4, delta 1e-11): the
    short-range Cauchy-Schwarz factors with the six-block density weight
    (and the local-pair Cauchy-Schwarz cutoff) at delta against delta/100.
    The change must stay below the 1e-7 matrix tolerance and 1e-6 Eh per
    atom (measured 6e-10)."""
    from paper_2410_22278_amd import inputs
    s = inputs.small_cell(41, natom=2, a_ang=3.2, recipe=((0, 0), (1, 0), (2, 1)), lo=0.15, hi=8.0,
                          nprim=2, omega=0.4, delta=1e-11)
    r = oracle_mod.jk(s)
    tight = Thresholds.uniform(1e-11)
    tight.schwarz = 1e-13
    tight.pair_cs = 1e-13
    c = oracle_mod.jk(s, thr=tight)
    assert np.abs(r["J"] - c["J"]).max() < 1e-7
    assert np.abs(r["K"] - c["K"]).max() < 1e-7
    assert abs(r["E_J"] - c["E_J"]) / s.natom < 1e-6
    assert abs(r["E_K"] - c["E_K"]) / s.natom < 1e-6
