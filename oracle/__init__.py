"""CPU oracle for the Gamma-point periodic J/K build (TEST INFRASTRUCTURE).

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP
library: the C part (oracle.c) evaluates local primitive pairs, short-range
quartets and pair structure factors in plain FP64 loops; this module adds the
reciprocal-space and self terms with numpy matrix products and the spherical
transform of d shells.

Pieces and the passages they follow:
  J, K at the Gamma point            Sec. 2.5-2.6 (eqs. pbc_j_definition_k_sample,
                                     pbc_k_definition with k = 0, weight 1)
  periodic ERI split                  Sec. 2.4, eq. pbc_eri_general_final:
                                     real-space erfc sum + reciprocal sum over
                                     G != 0 + self term
  reciprocal sum                      the Gaussian factors of that equation,
                                     split into bra and ket structure factors
  self term                           -(2 pi^{3/2}/V) sqrt(1/p+1/q)/(4 w^2) x
                                     prefactor x E_0...E_0, which equals
                                     -(pi/(V w^2)) S_bra S_ket
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from ctypes import POINTER, c_double, c_int, c_long, c_ubyte
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

SQRT3_2 = np.sqrt(3.0) / 2.0


def build(force: bool = True) -> str:
    """Compile oracle.c (plain -O2, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = POINTER(c_double)
        ip = POINTER(c_int)
        lib.orc_boys.argtypes = [c_int, c_double, dp]
        lib.orc_eri_prim.argtypes = [c_int] + [c_int] * 4 + [c_double] * 4 + [dp] * 4 + [c_double, dp]
        lib.orc_overlap_prim.argtypes = [c_int, c_int, c_double, c_double, dp, dp, dp]
        lib.orc_sr_jk.argtypes = [POINTER(OrcSys), dp, POINTER(c_ubyte), dp, dp, dp]
        lib.orc_sr_jk.restype = c_int
        lib.orc_sr_tensor.argtypes = [POINTER(OrcSys), dp]
        lib.orc_glist.argtypes = [POINTER(OrcSys), c_int, dp, dp]
        lib.orc_glist.restype = c_int
        lib.orc_nbf_cart.argtypes = [POINTER(OrcSys)]
        lib.orc_nbf_cart.restype = c_int
        lib.orc_sfac.argtypes = [POINTER(OrcSys), c_int, dp, dp, dp]
        lib.orc_sfac.restype = c_int
        lib.orc_ctx_new.argtypes = [POINTER(OrcSys)]
        lib.orc_ctx_new.restype = ctypes.c_void_p
        lib.orc_ctx_free.argtypes = [ctypes.c_void_p]
        lib.orc_ctx_sfac.argtypes = [ctypes.c_void_p, c_int, dp, dp, dp]
        lib.orc_overlap.argtypes = [POINTER(OrcSys), dp]
        lib.orc_overlap.restype = c_int
        lib.orc_pair_list.argtypes = [POINTER(OrcSys), c_long, ip, ip, ip, ip, ip, dp]
        lib.orc_pair_list.restype = c_long
        lib.orc_min_image.argtypes = [dp, dp, dp]
        lib.orc_lattice_sphere.argtypes = [dp, dp, c_double, c_long, ip]
        lib.orc_lattice_sphere.restype = c_long
        lib.orc_ewald_energy.argtypes = [c_int, dp, dp, dp, c_double, c_double, c_double]
        lib.orc_ewald_energy.restype = c_double
        lib.orc_one_electron.argtypes = [POINTER(OrcSys), dp, dp, dp, dp]
        lib.orc_one_electron.restype = c_int
        _lib = lib
    return _lib


class OrcSys(ctypes.Structure):
    _fields_ = [("cell", c_double * 9), ("natom", c_int), ("xyz", POINTER(c_double)),
                ("nshell", c_int), ("sh_atom", POINTER(c_int)), ("sh_l", POINTER(c_int)),
                ("sh_pure", POINTER(c_int)), ("sh_nprim", POINTER(c_int)),
                ("exps", POINTER(c_double)), ("coefs", POINTER(c_double)),
                ("omega", c_double), ("d_pair_R", c_double), ("d_pair_cs", c_double),
                ("d_ewald_R", c_double), ("d_ewald_K", c_double), ("d_schwarz", c_double),
                ("r_cut", c_double), ("g_cut", c_double)]


def _dp(a):
    return a.ctypes.data_as(POINTER(c_double))


def _ip(a):
    return a.ctypes.data_as(POINTER(c_int))


class _Sys:
    """Keeps the numpy buffers alive while the C struct points at them."""

    def __init__(self, s, omega=None, thr=None):
        self.cell = np.ascontiguousarray(s.cell, dtype=np.float64)
        self.xyz = np.ascontiguousarray(s.xyz, dtype=np.float64)
        self.sa = np.ascontiguousarray(s.shell_atom, dtype=np.int32)
        self.sl = np.ascontiguousarray(s.shell_l, dtype=np.int32)
        self.sp = np.ascontiguousarray(s.shell_pure, dtype=np.int32)
        self.sn = np.ascontiguousarray(s.shell_nprim, dtype=np.int32)
        self.ex = np.ascontiguousarray(s.exps, dtype=np.float64)
        self.co = np.ascontiguousarray(s.coefs, dtype=np.float64)
        t = thr if thr is not None else s.thr
        self.c = OrcSys()
        self.c.cell[:] = self.cell.ravel().tolist()
        self.c.natom = self.xyz.shape[0]
        self.c.xyz = _dp(self.xyz)
        self.c.nshell = self.sl.shape[0]
        self.c.sh_atom = _ip(self.sa)
        self.c.sh_l = _ip(self.sl)
        self.c.sh_pure = _ip(self.sp)
        self.c.sh_nprim = _ip(self.sn)
        self.c.exps = _dp(self.ex)
        self.c.coefs = _dp(self.co)
        self.c.omega = float(s.omega if omega is None else omega)
        self.c.d_pair_R = t.pair_R
        self.c.d_pair_cs = t.pair_cs
        self.c.d_ewald_R = t.ewald_R
        self.c.d_ewald_K = t.ewald_K
        self.c.d_schwarz = t.schwarz
        self.c.r_cut = t.r_cut
        self.c.g_cut = t.g_cut
        self.volume = abs(np.linalg.det(self.cell))
        self.omega = self.c.omega


# --------------------------------------------------------------------------
# primitive-level entry points (used by the pins)
# --------------------------------------------------------------------------

def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    _load().orc_boys(mmax, float(T), _dp(out))
    return out


def ncart(l: int) -> int:
    return (l + 1) * (l + 2) // 2


def cart_components(l: int):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def eri_prim(kind: int, ls, exps, centers, omega: float = 0.0) -> np.ndarray:
    """Molecular primitive ERI block over monomial Cartesian Gaussians.
    kind 0 = 1/r, 1 = erfc(w r)/r, 2 = erf(w r)/r."""
    la, lb, lc, ld = ls
    out = np.zeros(ncart(la) * ncart(lb) * ncart(lc) * ncart(ld))
    cs = [np.ascontiguousarray(c, dtype=np.float64) for c in centers]
    _load().orc_eri_prim(kind, la, lb, lc, ld, *[float(e) for e in exps], *[_dp(c) for c in cs],
                         float(omega), _dp(out))
    return out.reshape(ncart(la), ncart(lb), ncart(lc), ncart(ld))


def overlap_prim(la: int, lb: int, a: float, b: float, A, B) -> np.ndarray:
    out = np.zeros(ncart(la) * ncart(lb))
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    _load().orc_overlap_prim(la, lb, float(a), float(b), _dp(A), _dp(B), _dp(out))
    return out.reshape(ncart(la), ncart(lb))


def min_image(cell, x) -> np.ndarray:
    out = np.zeros(3)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    xx = np.ascontiguousarray(x, dtype=np.float64)
    _load().orc_min_image(_dp(c), _dp(xx), _dp(out))
    return out


def lattice_sphere(cell, center, r: float) -> np.ndarray:
    c = np.ascontiguousarray(cell, dtype=np.float64)
    ce = np.ascontiguousarray(center, dtype=np.float64)
    n = _load().orc_lattice_sphere(_dp(c), _dp(ce), float(r), 0, _ip(np.zeros(3, np.int32)))
    buf = np.zeros(3 * max(n, 1), np.int32)
    _load().orc_lattice_sphere(_dp(c), _dp(ce), float(r), n, _ip(buf))
    return buf[:3 * n].reshape(n, 3)


def ewald_energy(xyz, q, cell, omega: float, dR: float = 1e-16, dK: float = 1e-16) -> float:
    """Point-charge Ewald energy with the background term (Sec. 2.8)."""
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    qq = np.ascontiguousarray(q, dtype=np.float64)
    c = np.ascontiguousarray(cell, dtype=np.float64)
    return _load().orc_ewald_energy(x.shape[0], _dp(x), _dp(qq), _dp(c), float(omega), dR, dK)


# --------------------------------------------------------------------------
# system-level entry points
# --------------------------------------------------------------------------

def sph_transform(system) -> np.ndarray:
    """T (nbf x nbf_cart): identity on Cartesian shells; real solid harmonics
    m = -2..2 on spherical d shells, built from P:normalised Cartesian
    components (xx, xy, xz, yy, yz, zz):
      d-2 = xy, d-1 = yz, d0 = zz - xx/2 - yy/2, d1 = xz, d2 = (sqrt3/2)(xx - yy)."""
    rows = []
    nbc = sum(ncart(int(l)) for l in system.shell_l)
    off = 0
    for l, pure in zip(system.shell_l, system.shell_pure):
        l = int(l)
        nc = ncart(l)
        if pure and l == 2:
            blk = np.zeros((5, 6))
            blk[0, 1] = 1.0
            blk[1, 4] = 1.0
            blk[2, 5] = 1.0
            blk[2, 0] = -0.5
            blk[2, 3] = -0.5
            blk[3, 2] = 1.0
            blk[4, 0] = SQRT3_2
            blk[4, 3] = -SQRT3_2
        else:
            blk = np.eye(nc)
        for r in blk:
            row = np.zeros(nbc)
            row[off:off + nc] = r
            rows.append(row)
        off += nc
    return np.array(rows)


def glist(system, omega=None, thr=None):
    s = _Sys(system, omega, thr)
    lib = _load()
    n = lib.orc_glist(ctypes.byref(s.c), 0, _dp(np.zeros(3)), _dp(np.zeros(1)))
    G = np.zeros((max(n, 1), 3))
    w = np.zeros(max(n, 1))
    lib.orc_glist(ctypes.byref(s.c), n, _dp(G), _dp(w))
    return G[:n], w[:n]


def pair_list(system, omega=None, thr=None):
    s = _Sys(system, omega, thr)
    lib = _load()
    z = np.zeros(1, np.int32)
    n = lib.orc_pair_list(ctypes.byref(s.c), 0, _ip(z), _ip(z), _ip(z), _ip(z), _ip(z),
                          _dp(np.zeros(1)))
    arrs = [np.zeros(max(n, 1), np.int32) for _ in range(4)]
    n2 = np.zeros(3 * max(n, 1), np.int32)
    Q = np.zeros(max(n, 1))
    lib.orc_pair_list(ctypes.byref(s.c), n, *[_ip(a) for a in arrs], _ip(n2), _dp(Q))
    return dict(sa=arrs[0][:n], sb=arrs[1][:n], ia=arrs[2][:n], ib=arrs[3][:n],
                n2=n2[:3 * n].reshape(n, 3), Q=Q[:n])


def overlap_cart(system, omega=None, thr=None) -> np.ndarray:
    s = _Sys(system, omega, thr)
    lib = _load()
    nbc = lib.orc_nbf_cart(ctypes.byref(s.c))
    S = np.zeros((nbc, nbc))
    if lib.orc_overlap(ctypes.byref(s.c), _dp(S)) != 0:
        raise ValueError("oracle rejected the basis")
    return S


def structure_factors(system, G, omega=None, thr=None) -> np.ndarray:
    """Complex pair structure factors F[g, mu, nu] (Cartesian)."""
    s = _Sys(system, omega, thr)
    lib = _load()
    nbc = lib.orc_nbf_cart(ctypes.byref(s.c))
    G = np.ascontiguousarray(G, dtype=np.float64)
    ng = G.shape[0]
    fr = np.zeros((ng, nbc, nbc))
    fi = np.zeros((ng, nbc, nbc))
    if ng:
        lib.orc_sfac(ctypes.byref(s.c), ng, _dp(G), _dp(fr), _dp(fi))
    return fr + 1j * fi


def sr_jk_cart(system, Dc, bra_shells: Optional[Sequence[int]] = None, omega=None, thr=None):
    """Short-range J, K (Cartesian) and counts from the C loops."""
    s = _Sys(system, omega, thr)
    lib = _load()
    nbc = lib.orc_nbf_cart(ctypes.byref(s.c))
    Dc = np.ascontiguousarray(Dc, dtype=np.float64)
    J = np.zeros((nbc, nbc))
    K = np.zeros((nbc, nbc))
    counts = np.zeros(3)
    mask = None
    if bra_shells is not None:
        m = np.zeros(system.nshell, np.uint8)
        m[list(bra_shells)] = 1
        mask = m
    mp = mask.ctypes.data_as(POINTER(c_ubyte)) if mask is not None else None
    rc = lib.orc_sr_jk(ctypes.byref(s.c), _dp(Dc), mp, _dp(J), _dp(K), _dp(counts))
    if rc != 0:
        raise ValueError("oracle rejected the basis")
    return J, K, counts


def sr_tensor_cart(system, omega=None, thr=None) -> np.ndarray:
    s = _Sys(system, omega, thr)
    lib = _load()
    nbc = lib.orc_nbf_cart(ctypes.byref(s.c))
    T = np.zeros((nbc,) * 4)
    lib.orc_sr_tensor(ctypes.byref(s.c), _dp(T))
    return T


def cart_rows(system, shells: Sequence[int]) -> np.ndarray:
    off = np.cumsum([0] + [ncart(int(l)) for l in system.shell_l])
    return np.concatenate([np.arange(off[s], off[s + 1]) for s in shells]).astype(np.int64)


def ao_rows(system, shells: Sequence[int]) -> np.ndarray:
    sizes = [(2 * int(l) + 1) if (p and int(l) == 2) else ncart(int(l))
             for l, p in zip(system.shell_l, system.shell_pure)]
    off = np.cumsum([0] + sizes)
    return np.concatenate([np.arange(off[s], off[s + 1]) for s in shells]).astype(np.int64)


def jk(system, D=None, omega=None, thr=None, bra_shells: Optional[Sequence[int]] = None,
       parts: str = "sr,lr,self", g_chunk: int = 64, g_range=None) -> dict:
    """Gamma-point J and K of `system` (spherical where the basis says so).

    With bra_shells set, only the rows of J and K belonging to those shells
    are exact (the others are left partial); energies are then not formed.
    g_range = (start, stop) restricts the reciprocal sum to a slice of the
    G list (for timing samples only).
    Returns a dict with J, K, E_J, E_K, the parts, and counts."""
    D = system.D if D is None else D
    s = _Sys(system, omega, thr)
    T = sph_transform(system)
    Dc = T.T @ D @ T
    nbc = Dc.shape[0]
    want = set(parts.split(","))
    out = {}
    rows = None if bra_shells is None else cart_rows(system, bra_shells)
    Jsr = np.zeros((nbc, nbc)); Ksr = np.zeros((nbc, nbc)); counts = np.zeros(3)
    if "sr" in want:
        Jsr, Ksr, counts = sr_jk_cart(system, Dc, bra_shells, omega, thr)
    Jlr = np.zeros((nbc, nbc)); Klr = np.zeros((nbc, nbc))
    nG = 0
    if "lr" in want:
        G, w = glist(system, omega, thr)
        if g_range is not None:
            G, w = G[g_range[0]:g_range[1]], w[g_range[0]:g_range[1]]
        nG = G.shape[0]
        lib = _load()
        ctx = lib.orc_ctx_new(ctypes.byref(s.c))
        if not ctx:
            raise ValueError("oracle rejected the basis")
        fr = np.zeros((g_chunk, nbc, nbc))
        fi = np.zeros((g_chunk, nbc, nbc))
        for g0 in range(0, nG, g_chunk):
            Gc = np.ascontiguousarray(G[g0:g0 + g_chunk])
            ng = Gc.shape[0]
            lib.orc_ctx_sfac(ctx, ng, _dp(Gc), _dp(fr), _dp(fi))
            F = fr[:ng] + 1j * fi[:ng]
            for k in range(F.shape[0]):
                Fg = F[k]
                wg = w[g0 + k]
                rhoD = np.sum(Dc * Fg)                    # sum_{la si} D F_G[la si]
                if rows is None:
                    Jlr += wg * np.real(np.conj(Fg) * rhoD)
                    Klr += wg * np.real(np.conj(Fg) @ Dc @ Fg.T)
                else:
                    Jlr[rows] += wg * np.real(np.conj(Fg[rows]) * rhoD)
                    Klr[rows] += wg * np.real(np.conj(Fg[rows]) @ Dc @ Fg.T)
        lib.orc_ctx_free(ctx)
    Jself = np.zeros((nbc, nbc)); Kself = np.zeros((nbc, nbc))
    if "self" in want:
        S = overlap_cart(system, omega, thr)
        f = -np.pi / (s.volume * s.omega ** 2)
        Jself = f * S * np.sum(S * Dc)
        Kself = f * (S @ Dc @ S)
    Jc = Jsr + Jlr + Jself
    Kc = Ksr + Klr + Kself
    J = T @ Jc @ T.T
    K = T @ Kc @ T.T
    out.update(J=J, K=K, Jc=Jc, Kc=Kc, J_sr=T @ Jsr @ T.T, K_sr=T @ Ksr @ T.T,
               J_lr=T @ Jlr @ T.T, K_lr=T @ Klr @ T.T, J_self=T @ Jself @ T.T,
               K_self=T @ Kself @ T.T, n_quartets=counts[0], n_terms=counts[1],
               n_pairs=counts[2], n_G=nG)
    if bra_shells is None:
        out["E_J"] = 0.5 * float(np.sum(D * J))
        out["E_K"] = -0.25 * float(np.sum(D * K))
    else:
        out["rows"] = ao_rows(system, bra_shells)
    return out


def eri_tensor(system, omega=None, thr=None) -> np.ndarray:
    """Full Gamma ERI tensor (nbf^4, spherical where the basis says so) for
    tiny systems: SR part from the C loops (Schwarz screen without density),
    LR from structure factors, self from the overlap."""
    s = _Sys(system, omega, thr)
    Tsr = sr_tensor_cart(system, omega, thr)
    G, w = glist(system, omega, thr)
    F = structure_factors(system, G, omega, thr)
    Tlr = np.real(np.einsum("g,gij,gkl->ijkl", w, np.conj(F), F))
    S = overlap_cart(system, omega, thr)
    Tself = -np.pi / (s.volume * s.omega ** 2) * np.einsum("ij,kl->ijkl", S, S)
    Tc = Tsr + Tlr + Tself
    T = sph_transform(system)
    return np.einsum("ai,bj,ck,dl,ijkl->abcd", T, T, T, T, Tc, optimize=True)


def one_electron(system, omega=None, thr=None, charges=None, parts: str = "sr,lr,self") -> dict:
    """Gamma-point overlap S, kinetic T, nuclear attraction V and the nuclear
    repulsion energy E_nuc of `system` (spherical where the basis says so).

    V_{mu nu} = sum_C q_C <mu| v(r - C) |nu> with q_C = -Z_C (electrons
    attracted by nuclei of charge Z = system.charge unless `charges` is
    given) and v the Ewald-split periodic Coulomb potential of a point charge
    with its G = 0 term removed (Sec. 2.3, eq. pbc_v1e_general_final):
    real-space erfc sum (the C loops), reciprocal sum over the same G list as
    the ERIs, and the self term -(pi/(V w^2)) sum_C q_C S.  E_nuc is the
    Ewald energy of the nuclei (Sec. 2.9, eq. nuclear_repulsion_energy)."""
    s = _Sys(system, omega, thr)
    lib = _load()
    Z = np.ascontiguousarray(system.charge, dtype=np.float64)
    q = -Z if charges is None else np.ascontiguousarray(charges, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    nbc = lib.orc_nbf_cart(ctypes.byref(s.c))
    S = np.zeros((nbc, nbc)); T = np.zeros((nbc, nbc)); Vsr = np.zeros((nbc, nbc))
    if lib.orc_one_electron(ctypes.byref(s.c), _dp(q), _dp(S), _dp(T), _dp(Vsr)) != 0:
        raise ValueError("oracle rejected the basis")
    want = set(parts.split(","))
    if "sr" not in want:
        Vsr[:] = 0.0
    Vlr = np.zeros((nbc, nbc))
    if "lr" in want:
        G, w = glist(system, omega, thr)
        xyz = np.asarray(system.xyz, dtype=np.float64)
        for g0 in range(0, G.shape[0], 64):
            Gc = np.ascontiguousarray(G[g0:g0 + 64])
            F = structure_factors(system, Gc, omega, thr)
            for k in range(Gc.shape[0]):
                # rho_n(G) = sum_C q_C e^{-i G.C}; v's Fourier sum gives
                # sum_G w_G Re(conj(F_G) rho_n(G))
                rho_n = np.sum(q * np.exp(-1j * (xyz @ Gc[k])))
                Vlr += w[g0 + k] * np.real(np.conj(F[k]) * rho_n)
    Vself = np.zeros((nbc, nbc))
    if "self" in want:
        Vself = -np.pi / (s.volume * s.omega ** 2) * np.sum(q) * S
    Vc = Vsr + Vlr + Vself
    Tm = sph_transform(system)
    out = dict(S=Tm @ S @ Tm.T, T=Tm @ T @ Tm.T, V=Tm @ Vc @ Tm.T, V_sr=Tm @ Vsr @ Tm.T,
               V_lr=Tm @ Vlr @ Tm.T, V_self=Tm @ Vself @ Tm.T, Sc=S, Tc=T, Vc=Vc)
    t = thr if thr is not None else system.thr
    out["E_nuc"] = ewald_energy(system.xyz, Z, system.cell, s.omega, t.ewald_R, t.ewald_K)
    return out

