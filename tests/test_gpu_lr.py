"""GPU parity of the two forms of the reciprocal exchange.

K_LR = sum_G W_G (A_G D A_G + B_G D B_G) is evaluated either densely or, for
a positive semidefinite density of low rank, through a device pivoted
Cholesky factor D = L L^T as sum_G W_G (A_G L)(A_G L)^T + (B_G L)(B_G L)^T.
The factor is accepted only after an entrywise check of D - L L^T, so both
forms must agree with the oracle to the FP64 bar; the counters say which
form ran.  The 144-AO cell spans two 128-wide output tiles, so the dense
form's upper-tile-only accumulation and its symmetric read-back are
exercised; the low-rank form forms three of the four half blocks of each
Y Y^T and reads K back by upper half blocks, which the 25-AO cell (odd, so
the two halves differ in size) checks as well.
"""
import numpy as np
import pytest

from paper_2410_22278_amd import inputs

pytestmark = pytest.mark.gpu

CELL144 = dict(seed=41, natom=36, a_ang=7.0, recipe=((0, 0), (1, 0)), delta=1e-10, g_cut=2.0, r_cut=8.0)
CELL_D = dict(seed=21, natom=2, recipe=((0, 0), (1, 0), (2, 1)), a_ang=3.2, lo=0.3, hi=4.0)
CELL_ODD = dict(seed=7, natom=5, recipe=((0, 0), (0, 0), (1, 0)), a_ang=5.0, delta=1e-10, g_cut=2.0, r_cut=8.0)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_22278_amd import pbcjk
    pbcjk.load()
    return pbcjk


def _lr(lib, s, D, mode, parts=2 | 4):
    with lib.Handle(s) as h:
        h.set_parts(parts)
        h.set_lr(mode)
        J, K, _, _ = h.build(D)
        st = h.stats()
    return J, K, st


def _cmp(tag, J, K, ref):
    dJ = np.abs(J - ref["J"]).max()
    dK = np.abs(K - ref["K"]).max()
    print(f"{tag}: max|dJ|={dJ:.3e} max|dK|={dK:.3e} (max|K|={np.abs(ref['K']).max():.3e})", flush=True)
    return dJ, dK


@pytest.mark.parametrize("mode", ["auto", "dense"])
def test_lr_forms_multi_tile(lib, oracle_mod, mode):
    s = inputs.small_cell(**CELL144)
    ref = oracle_mod.jk(s, parts="lr,self")
    m = lib.LR_AUTO if mode == "auto" else lib.LR_DENSE
    J, K, st = _lr(lib, s, s.D, m)
    dJ, dK = _cmp(f"lr+self {mode} nbf={s.nbf} rank={st['lr_rank']:.0f}", J, K, ref)
    assert dJ < 1e-9 and dK < 1e-9
    assert np.abs(K - K.T).max() < 1e-13
    if mode == "auto":
        assert st["lr_rank"] == s.nbf // 2      # D = C C^T with nbf/2 orbitals
    else:
        assert st["lr_rank"] == -1


@pytest.mark.parametrize("mode", ["auto", "dense"])
def test_lr_forms_odd_size(lib, oracle_mod, mode):
    s = inputs.small_cell(**CELL_ODD)
    assert s.nbf % 2 == 1
    ref = oracle_mod.jk(s, parts="lr,self")
    m = lib.LR_AUTO if mode == "auto" else lib.LR_DENSE
    J, K, st = _lr(lib, s, s.D, m)
    dJ, dK = _cmp(f"lr+self {mode} nbf={s.nbf} rank={st['lr_rank']:.0f}", J, K, ref)
    assert dJ < 1e-9 and dK < 1e-9
    assert np.abs(K - K.T).max() < 1e-13
    assert (st["lr_rank"] > 0) if mode == "auto" else (st["lr_rank"] == -1)


def test_lr_d_shells_scaled_basis(lib, oracle_mod):
    """Spherical d: the factor is taken of the density in the scaled
    Cartesian basis, whose rank equals that of D."""
    s = inputs.small_cell(**CELL_D)
    ref = oracle_mod.jk(s, parts="lr")
    J, K, st = _lr(lib, s, s.D, lib.LR_AUTO, parts=2)
    dJ, dK = _cmp(f"lr d auto rank={st['lr_rank']:.0f}", J, K, ref)
    assert dJ < 1e-9 and dK < 1e-9
    assert st["lr_rank"] == s.nbf // 2


def test_lr_fallbacks_and_switching(lib, oracle_mod):
    """One handle, densities in turn: indefinite (dense form), full-rank
    semidefinite (rank above the cap: dense form), low rank (factor), zero
    (rank 0).  The control block is rebuilt every time."""
    s = inputs.small_cell(**CELL144)
    n = s.nbf
    rng = np.random.default_rng(77)
    X = rng.standard_normal((n, n)) / n
    D_indef = X + X.T
    C = rng.standard_normal((n, n)) / np.sqrt(n)
    D_full = C @ C.T
    D_full = 0.5 * (D_full + D_full.T)
    cases = [("indefinite", D_indef, -1), ("full rank", D_full, -1), ("low rank", s.D, n // 2),
             ("zero", np.zeros((n, n)), 0), ("indefinite again", D_indef, -1)]
    with lib.Handle(s) as h:
        h.set_parts(2)
        for tag, D, rank in cases:
            ref = oracle_mod.jk(s, D=D, parts="lr")
            J, K, _, _ = h.build(D)
            st = h.stats()
            dJ, dK = _cmp(f"{tag}: rank={st['lr_rank']:.0f}", J, K, ref)
            assert st["lr_rank"] == rank, tag
            scale = max(1.0, np.abs(ref["K"]).max())
            assert dJ < 1e-9 * scale and dK < 1e-9 * scale, tag
