"""Seeded synthetic workloads for the Gamma-point periodic J/K build.

This module only draws numbers: cells, atom positions, shell recipes with raw
exponents and contraction coefficients, and density matrices.  It holds none
of the method's arithmetic (no normalisation, no integrals, no screening), so
that both the CPU oracle and the HIP library can consume the same inputs.

Every random number comes from ``numpy.random.default_rng(seed)`` (PCG64) and
is drawn in the order documented on each generator.  All lengths are bohr,
exponents bohr^-2.

The workloads stand in for the paper's crystals (ice, benzene, Si, ZnO,
LiF; def2-SVP), which are not reproduced: they keep the shapes that matter
for the integral engine (cell size, atom density, shell mix, exponent range,
density-matrix rank).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BOHR_PER_ANGSTROM = 1.0 / 0.529177210903  # CODATA 2018 Bohr radius


@dataclass
class Thresholds:
    """Screening thresholds (see include/pbcjk.h for the meaning of each)."""
    pair_R: float = 1e-14
    pair_cs: float = 1e-14
    ewald_R: float = 1e-14
    ewald_K: float = 1e-14
    schwarz: float = 1e-14
    fp32_below: float = 0.0
    r_cut: float = 0.0
    g_cut: float = 0.0

    @classmethod
    def uniform(cls, delta: float, **kw) -> "Thresholds":
        return cls(pair_R=delta, pair_cs=delta, ewald_R=delta, ewald_K=delta,
                   schwarz=delta, **kw)


@dataclass
class System:
    """One periodic cell with a Gaussian basis and a density matrix."""
    name: str
    cell: np.ndarray            # (3, 3) rows = lattice vectors a, b, c
    xyz: np.ndarray             # (natom, 3)
    charge: np.ndarray          # (natom,)
    shell_atom: np.ndarray      # (nshell,) int32
    shell_l: np.ndarray         # (nshell,) int32
    shell_pure: np.ndarray      # (nshell,) int32
    shell_nprim: np.ndarray     # (nshell,) int32
    exps: np.ndarray            # (sum nprim,)
    coefs: np.ndarray           # (sum nprim,) raw contraction coefficients
    omega: float
    thr: Thresholds
    D: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def natom(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def nshell(self) -> int:
        return int(self.shell_l.shape[0])

    @property
    def nbf(self) -> int:
        return int(sum(shell_size(int(l), int(p))
                       for l, p in zip(self.shell_l, self.shell_pure)))

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.cell)))


def shell_size(l: int, pure: int) -> int:
    """Number of functions in a shell: 2l+1 spherical or (l+1)(l+2)/2 Cartesian."""
    return 2 * l + 1 if pure else (l + 1) * (l + 2) // 2


# --------------------------------------------------------------------------
# helpers (geometry drawing only)
# --------------------------------------------------------------------------

def _min_image_dist(cell: np.ndarray, x: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Distances from x to each row of ys under the minimum-image convention."""
    if ys.shape[0] == 0:
        return np.zeros(0)
    inv = np.linalg.inv(cell.T)
    d = ys - x[None, :]
    f = d @ inv.T
    f -= np.round(f)
    d = f @ cell
    # a 27-image check guards against skewed cells
    best = np.full(d.shape[0], np.inf)
    for i in (-1, 0, 1):
        for j in (-1, 0, 1):
            for k in (-1, 0, 1):
                s = d + i * cell[0] + j * cell[1] + k * cell[2]
                best = np.minimum(best, np.linalg.norm(s, axis=1))
    return best


def _uniform_points(rng, cell, n, min_sep, max_tries=200000):
    pts = []
    tries = 0
    while len(pts) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place points with the requested separation")
        f = rng.random(3)
        x = f @ cell
        if pts and np.min(_min_image_dist(cell, x, np.array(pts))) < min_sep:
            continue
        pts.append(x)
    return np.array(pts)


def _haar_rotation(rng) -> np.ndarray:
    """Haar-random rotation: QR of a Gaussian matrix with the sign fix, det +1."""
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _draw_shells(rng, recipe, lo, hi, nprim=3):
    """recipe: list of (l, pure).  Exponents log-uniform in [lo, hi], then
    raw coefficients U(0.1, 1.0), per shell in recipe order."""
    out = []
    for (l, pure) in recipe:
        e = np.exp(rng.uniform(np.log(lo), np.log(hi), nprim))
        c = rng.uniform(0.1, 1.0, nprim)
        out.append((l, pure, e, c))
    return out


def _assemble(name, cell, xyz, charge, atom_shells, omega, thr, meta=None):
    """atom_shells[i] = list of (l, pure, exps, coefs) for atom i."""
    sa, sl, sp, sn, ex, co = [], [], [], [], [], []
    for ia, shells in enumerate(atom_shells):
        for (l, pure, e, c) in shells:
            sa.append(ia); sl.append(l); sp.append(pure); sn.append(len(e))
            ex.extend(e); co.extend(c)
    return System(name=name, cell=np.asarray(cell, float), xyz=np.asarray(xyz, float),
                  charge=np.asarray(charge, float),
                  shell_atom=np.array(sa, np.int32), shell_l=np.array(sl, np.int32),
                  shell_pure=np.array(sp, np.int32), shell_nprim=np.array(sn, np.int32),
                  exps=np.array(ex, float), coefs=np.array(co, float),
                  omega=float(omega), thr=thr, meta=meta or {})


def density_from_orbitals(rng, nbf: int, nocc: int) -> np.ndarray:
    """D = C C^T with C (nbf x nocc) entries N(0,1)/sqrt(nbf)."""
    C = rng.standard_normal((nbf, nocc)) / np.sqrt(nbf)
    D = C @ C.T
    return 0.5 * (D + D.T)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def cfg1(seed: int = 1) -> System:
    """Tiny FP64 case: cubic a = 5.0 A, 8 atoms (one element), 2 s + 1 p
    shells per atom, 3 primitives, exponents log-uniform [0.1, 20]; nbf 40.
    omega 0.3, every delta 1e-10, image cap 10 A, |G| cap 3 bohr^-1.
    Draw order: positions (rejection, min-image separation >= 1.2 A),
    element basis, then C (40 x 8)."""
    rng = np.random.default_rng(seed)
    a = 5.0 * BOHR_PER_ANGSTROM
    cell = np.eye(3) * a
    xyz = _uniform_points(rng, cell, 8, 1.2 * BOHR_PER_ANGSTROM)
    basis = _draw_shells(rng, [(0, 0), (0, 0), (1, 0)], 0.1, 20.0)
    sysm = _assemble("cfg1", cell, xyz, np.ones(8), [basis] * 8, 0.3,
                     Thresholds.uniform(1e-10, r_cut=10.0 * BOHR_PER_ANGSTROM, g_cut=3.0))
    sysm.D = density_from_orbitals(rng, sysm.nbf, 8)
    return sysm


_WATER_OH = 0.96
_WATER_ANGLE = np.deg2rad(104.5)


def water_box(seed: int = 2, nmol: int = 64, a_ang: float = 12.4, omega: float = 0.3,
              delta: float = 1e-10, nocc: int = 320, fp32_below: float = 0.0,
              name: str = "cfg2") -> System:
    """Molecular-liquid cell: nmol rigid H2O (O-H 0.96 A, 104.5 deg) in a cubic
    box; O-O minimum-image separation >= 2.5 A is the only constraint.
    O: 3 s + 2 p, H: 2 s, 3 primitives each, log-uniform [0.1, 50], one basis
    per element.  Draw order: O basis, H basis, then for each molecule the
    O position (rejection) and a Haar rotation, then C (nbf x nocc)."""
    rng = np.random.default_rng(seed)
    a = a_ang * BOHR_PER_ANGSTROM
    cell = np.eye(3) * a
    bO = _draw_shells(rng, [(0, 0), (0, 0), (0, 0), (1, 0), (1, 0)], 0.1, 50.0)
    bH = _draw_shells(rng, [(0, 0), (0, 0)], 0.1, 50.0)
    roh = _WATER_OH * BOHR_PER_ANGSTROM
    h1 = roh * np.array([np.sin(_WATER_ANGLE / 2), 0.0, np.cos(_WATER_ANGLE / 2)])
    h2 = roh * np.array([-np.sin(_WATER_ANGLE / 2), 0.0, np.cos(_WATER_ANGLE / 2)])
    xyz, chg, shells = [], [], []
    oxy = []
    minsep = 2.5 * BOHR_PER_ANGSTROM
    tries = 0
    while len(oxy) < nmol:
        tries += 1
        if tries > 100000:
            raise RuntimeError("water packing failed")
        x = rng.random(3) @ cell
        if oxy and np.min(_min_image_dist(cell, x, np.array(oxy))) < minsep:
            continue
        Rm = _haar_rotation(rng)
        oxy.append(x)
        xyz += [x, x + Rm @ h1, x + Rm @ h2]
        chg += [8.0, 1.0, 1.0]
        shells += [bO, bH, bH]
    thr = Thresholds.uniform(delta, fp32_below=fp32_below)
    sysm = _assemble(name, cell, np.array(xyz), np.array(chg), shells, omega, thr)
    sysm.D = density_from_orbitals(rng, sysm.nbf, nocc)
    return sysm


def cfg2(seed: int = 2) -> System:
    """64 waters, a = 12.4 A, nbf 832, omega 0.3, delta 1e-10, FP64."""
    return water_box(seed=seed)


def cfg3(seed: int = 2) -> System:
    """cfg2 evaluated in mixed precision: FP32 quartets below a bound of 1e-6."""
    return water_box(seed=seed, fp32_below=1e-6, name="cfg3")


_DIAMOND = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0],
                     [.25, .25, .25], [.25, .75, .75], [.75, .25, .75], [.75, .75, .25]])


def diamond(seed: int = 4, reps: int = 4, a_conv_ang: float = 5.43, omega: float = 0.2,
            delta: float = 1e-11, nocc: Optional[int] = 1024, fp32_below: float = 0.0,
            name: str = "cfg4") -> System:
    """Diamond-lattice supercell (reps^3 conventional cells) with N(0, 0.05 A)
    displacements; 2 s + 2 p + 1 spherical d per atom, 3 primitives,
    log-uniform [0.08, 10], one element basis.  Draw order: displacements,
    basis, C."""
    rng = np.random.default_rng(seed)
    ac = a_conv_ang * BOHR_PER_ANGSTROM
    cell = np.eye(3) * ac * reps
    frac = []
    for i in range(reps):
        for j in range(reps):
            for k in range(reps):
                for f in _DIAMOND:
                    frac.append((f + np.array([i, j, k])) / reps)
    xyz = np.array(frac) @ cell
    xyz = xyz + rng.normal(0.0, 0.05 * BOHR_PER_ANGSTROM, xyz.shape)
    basis = _draw_shells(rng, [(0, 0), (0, 0), (1, 0), (1, 0), (2, 1)], 0.08, 10.0)
    natom = xyz.shape[0]
    thr = Thresholds.uniform(delta, fp32_below=fp32_below)
    sysm = _assemble(name, cell, xyz, np.full(natom, 14.0), [basis] * natom, omega, thr)
    if nocc is None:
        nocc = sysm.nbf // 6
    sysm.D = density_from_orbitals(rng, sysm.nbf, nocc)
    return sysm


def cfg4(seed: int = 4, mixed: bool = False) -> System:
    """512-atom diamond, a = 21.72 A, nbf 6656, omega 0.2, delta 1e-11."""
    return diamond(seed=seed, fp32_below=1e-6 if mixed else 0.0,
                   name="cfg4m" if mixed else "cfg4")


# Serving-stream elements: H: 2 s [0.1, 50]; O: 3 s + 2 p [0.1, 50];
# C: 2 s + 2 p + 1 d (spherical) [0.08, 10].
_SERVE_RECIPES = {
    "H": ([(0, 0), (0, 0)], 0.1, 50.0, 1.0),
    "C": ([(0, 0), (0, 0), (1, 0), (1, 0), (2, 1)], 0.08, 10.0, 6.0),
    "O": ([(0, 0), (0, 0), (0, 0), (1, 0), (1, 0)], 0.1, 50.0, 8.0),
}


def serving_request(i: int, base_seed: int = 1000, n_atoms: Optional[int] = None) -> System:
    """Request i of the serving stream: N ~ log-uniform[8, 216] atoms of
    H/C/O (p = 0.5/0.3/0.2) at 0.1 atoms/A^3 in a cubic cell, uniform
    positions with separation >= 1.2 A, element bases drawn per request,
    omega 0.3, delta 1e-10, FP32 below 1e-6, nocc = max(1, nbf // 4).
    Draw order: N, species, positions, H/C/O bases, C."""
    rng = np.random.default_rng(base_seed + i)
    n = int(round(np.exp(rng.uniform(np.log(8), np.log(216))))) if n_atoms is None else n_atoms
    species = rng.choice(["H", "C", "O"], size=n, p=[0.5, 0.3, 0.2])
    L = (n / 0.1) ** (1.0 / 3.0) * BOHR_PER_ANGSTROM
    cell = np.eye(3) * L
    xyz = _uniform_points(rng, cell, n, 1.2 * BOHR_PER_ANGSTROM)
    bases = {}
    for el in ("H", "C", "O"):
        rec, lo, hi, _z = _SERVE_RECIPES[el]
        bases[el] = _draw_shells(rng, rec, lo, hi)
    chg = np.array([_SERVE_RECIPES[s][3] for s in species])
    sysm = _assemble(f"req{i}", cell, xyz, chg, [bases[s] for s in species], 0.3,
                     Thresholds.uniform(1e-10, fp32_below=1e-6))
    sysm.D = density_from_orbitals(rng, sysm.nbf, max(1, sysm.nbf // 4))
    return sysm


def serving_arrivals(n: int = 256, rate: float = 1.0, seed: int = 500) -> np.ndarray:
    """Poisson arrival times (seconds) of n requests at the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg4": cfg4,
           "cfg4m": lambda: cfg4(mixed=True)}


def small_cell(seed: int, natom: int = 2, a_ang: float = 3.0, recipe=((0, 0), (1, 0)),
               lo: float = 0.3, hi: float = 5.0, omega: float = 0.5, delta: float = 1e-12,
               nprim: int = 2, per_atom_basis: bool = True, skew: float = 0.0,
               nocc: Optional[int] = None, r_cut: float = 0.0, g_cut: float = 0.0) -> System:
    """Small test cell with an optional triclinic skew; each atom draws its
    own basis when per_atom_basis.  Draw order: cell skew, positions,
    bases, C."""
    rng = np.random.default_rng(seed)
    a = a_ang * BOHR_PER_ANGSTROM
    cell = np.eye(3) * a
    if skew:
        cell = cell + skew * a * rng.uniform(-1, 1, (3, 3)) * (1 - np.eye(3))
    xyz = _uniform_points(rng, cell, natom, 0.8 * BOHR_PER_ANGSTROM)
    shells = []
    shared = None
    for _ in range(natom):
        if per_atom_basis or shared is None:
            b = []
            for (l, pure) in recipe:
                e = np.exp(rng.uniform(np.log(lo), np.log(hi), nprim))
                c = rng.uniform(0.1, 1.0, nprim)
                b.append((l, pure, e, c))
            shared = b
        shells.append(shared)
    sysm = _assemble(f"small{seed}", cell, xyz, np.ones(natom), shells, omega,
                     Thresholds.uniform(delta, r_cut=r_cut, g_cut=g_cut))
    nbf = sysm.nbf
    sysm.D = density_from_orbitals(rng, nbf, nocc if nocc else max(1, nbf // 2))
    return sysm


# ---------------------------------------------------------------- integration grids
def atom_grid(xyz, nrad: int = 40, ntheta: int = 12, nphi: int = 24, rscale: float = 1.0):
    """Atom-centred product grids (inputs of the Becke-weight kernel): per
    atom, radial Gauss-Legendre nodes x mapped by r = rscale (1 + x)/(1 - x),
    Gauss-Legendre nodes in cos(theta) and uniform phi.  Returns the points
    (N x 3), their quadrature weights (r^2 dr dcos(theta) dphi) and the index
    of each point's origin atom; points are grouped by atom."""
    xyz = np.asarray(xyz, float)
    xr, wr = np.polynomial.legendre.leggauss(nrad)
    r = rscale * (1.0 + xr) / (1.0 - xr)
    wr = wr * 2.0 * rscale / (1.0 - xr) ** 2 * r * r
    ct, wt = np.polynomial.legendre.leggauss(ntheta)
    st = np.sqrt(1.0 - ct * ct)
    ph = (np.arange(nphi) + 0.5) * (2.0 * np.pi / nphi)
    wp = 2.0 * np.pi / nphi
    dirs = np.stack([np.outer(st, np.cos(ph)).ravel(), np.outer(st, np.sin(ph)).ravel(),
                     np.repeat(ct, nphi)], axis=1)
    wang = np.repeat(wt, nphi) * wp
    off = (r[:, None, None] * dirs[None, :, :]).reshape(-1, 3)
    wq1 = (wr[:, None] * wang[None, :]).ravel()
    pts = np.concatenate([a + off for a in xyz])
    wq = np.tile(wq1, len(xyz))
    origin = np.repeat(np.arange(len(xyz), dtype=np.int32), len(off))
    return pts, wq, origin
