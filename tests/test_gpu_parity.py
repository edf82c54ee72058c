"""GPU parity: the HIP library through its C ABI against the CPU oracle.

FP64 path: the two implementations apply the same written truncation rules,
so they differ only by rounding and by screening decisions that sit exactly
at a threshold (contributions of size ~delta * |D|).  The bar is the stated
matrix tolerance 1e-7 and 1e-6 Eh/atom; the FP64 cases are asserted tighter
(1e-9) to catch any systematic error.
"""
import numpy as np
import pytest

from paper_2410_22278_amd import inputs
from paper_2410_22278_amd.inputs import Thresholds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_22278_amd import pbcjk
    pbcjk.load()
    return pbcjk


def _report(tag, J, K, ref, natom, EJ=None, EK=None):
    rows = ref.get("rows")
    if rows is not None:
        dJ = np.abs(J[rows] - ref["J"][rows]).max()
        dK = np.abs(K[rows] - ref["K"][rows]).max()
    else:
        dJ = np.abs(J - ref["J"]).max()
        dK = np.abs(K - ref["K"]).max()
    msg = f"{tag}: max|dJ|={dJ:.3e} max|dK|={dK:.3e}"
    dEJ = dEK = 0.0
    if EJ is not None and "E_J" in ref:
        dEJ = abs(EJ - ref["E_J"]) / natom
        dEK = abs(EK - ref["E_K"]) / natom
        msg += f" dE_J/atom={dEJ:.3e} dE_K/atom={dEK:.3e}"
    print(msg, flush=True)
    return dJ, dK, dEJ, dEK


SMALL = [
    dict(seed=3, natom=2, recipe=((0, 0), (1, 0))),
    dict(seed=5, natom=3, recipe=((0, 0), (0, 0), (1, 0)), skew=0.15, omega=0.35),
    dict(seed=6, natom=2, recipe=((1, 0), (1, 0)), lo=0.2, hi=8.0, a_ang=2.8, delta=1e-10),
    dict(seed=13, natom=4, recipe=((0, 0), (1, 0)), nprim=3, a_ang=3.5, omega=0.8),
]


@pytest.mark.parametrize("case", SMALL, ids=[f"small{c['seed']}" for c in SMALL])
def test_small_cells(lib, oracle_mod, case):
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D)
    dJ, dK, dEJ, dEK = _report(s.name, J, K, ref, s.natom, EJ, EK)
    assert dJ < 1e-9 and dK < 1e-9 and dEJ < 1e-9 and dEK < 1e-9


PART_CASES = [dict(seed=5, natom=3, recipe=((0, 0), (0, 0), (1, 0)), skew=0.15, omega=0.35),
              dict(seed=3, natom=2, recipe=((0, 0), (1, 0)))]


@pytest.mark.parametrize("mask,key", [(1, "sr"), (2, "lr"), (4, "self")])
@pytest.mark.parametrize("case", PART_CASES, ids=["nbf15", "nbf8"])
def test_parts(lib, oracle_mod, mask, key, case):
    """Each part alone: partial 16-row matrix-core tiles (nbf 8 and 15) make
    any lane-layout mistake in the reciprocal and self GEMMs visible."""
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s, parts=key)
    with lib.Handle(s) as h:
        h.set_parts(mask)
        J, K, _, _ = h.build(s.D)
    dJ, dK, _, _ = _report(f"part {key}", J, K, ref, s.natom)
    assert dJ < 1e-9 and dK < 1e-9


def test_device_path_and_repeatability(lib, oracle_mod):
    import torch
    s = inputs.small_cell(13, natom=4, recipe=((0, 0), (1, 0)), nprim=3, a_ang=3.5)
    with lib.Handle(s) as h:
        J0, K0, EJ0, EK0 = h.build(s.D)
        dD = torch.from_numpy(s.D).cuda()
        dJ = torch.empty_like(dD)
        dK = torch.empty_like(dD)
        spread = 0.0
        for _ in range(3):
            EJ, EK = h.build_device(dD, dJ, dK)
            torch.cuda.synchronize()
            spread = max(spread, np.abs(dJ.cpu().numpy() - J0).max(), np.abs(dK.cpu().numpy() - K0).max())
        # J only and K only
        h.build_device(dD, dJ, None, energies=False)
        torch.cuda.synchronize()
        Jonly = dJ.cpu().numpy()
    print(f"device path: run-to-run spread {spread:.3e}", flush=True)
    assert spread < 1e-12
    assert np.abs(Jonly - J0).max() < 1e-12
    assert abs(EJ - EJ0) < 1e-12 and abs(EK - EK0) < 1e-12


def test_cfg1_full(lib, oracle_mod):
    """Tiny FP64 workload (8 atoms, nbf 40) at its own thresholds."""
    s = inputs.cfg1()
    ref = oracle_mod.jk(s)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    dJ, dK, dEJ, dEK = _report("cfg1", J, K, ref, s.natom, EJ, EK)
    print(f"cfg1 stats: pairs={st['n_pairs']} groups={st['n_groups']} G={st['n_gvec']} "
          f"quartets={st['quartets']:.0f} terms={st['terms']:.0f} "
          f"oracle ordered quartets={ref['n_quartets']:.0f} terms={ref['n_terms']:.0f}", flush=True)
    assert dJ < 1e-9 and dK < 1e-9 and dEJ < 1e-9 and dEK < 1e-9
    assert np.abs(J - J.T).max() < 1e-13 and np.abs(K - K.T).max() < 1e-13


def test_cfg2_sampled_rows(lib, oracle_mod):
    """64-water cell (nbf 832) at full size: every row of three bra shells
    (an O s, an O p and an H s shell) against the oracle's exact rows."""
    s = inputs.cfg2()
    shells = [0, 3, 5 + 2]   # O 1st s, O 1st p, first H s
    ref = oracle_mod.jk(s, bra_shells=shells)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    print(f"cfg2: E_J={EJ:.10f} E_K={EK:.10f} build {st['t_build_ms']:.1f} ms "
          f"(sr {st['t_sr_ms']:.1f} lr {st['t_lr_ms']:.1f} other {st['t_other_ms']:.1f})", flush=True)
    dJ, dK, _, _ = _report("cfg2 rows", J, K, ref, s.natom)
    assert dJ < 1e-9 and dK < 1e-9
    assert np.abs(J - J.T).max() < 1e-12 and np.abs(K - K.T).max() < 1e-12
    assert EJ > 0 and EK < 0


MIXED = [
    dict(seed=5, natom=3, recipe=((0, 0), (0, 0), (1, 0)), skew=0.15, omega=0.35),
    dict(seed=13, natom=4, recipe=((0, 0), (1, 0)), nprim=3, a_ang=3.5, omega=0.8),
]


@pytest.mark.parametrize("case", MIXED, ids=["mixed5", "mixed13"])
def test_mixed_precision_small(lib, oracle_mod, case, monkeypatch):
    """FP32 for every quartet whose density-weighted bound is below 4e-3
    (most of them, to exercise the single-precision path) against the FP64
    oracle: stated tolerances 1e-7 for matrix elements, 1e-6 Eh/atom.  (The
    short-range Cauchy-Schwarz factors carry the erfc kernel's sqrt(1 - c),
    so 4e-3 puts about the quartets in FP32 that 1e-2 did with the Coulomb
    s-type factor.)  PBCJK_FP32_MIN_L=0 splits every class pair, so that the
    s and p FP32 kernels run too."""
    monkeypatch.setenv("PBCJK_FP32_MIN_L", "0")
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s)
    thr = Thresholds(**{**s.thr.__dict__, "fp32_below": 4e-3})
    with lib.Handle(s, thr=thr) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    dJ, dK, dEJ, dEK = _report(f"mixed {s.name} (fp32 terms {st['terms_fp32']:.0f}/{st['terms']:.0f})",
                               J, K, ref, s.natom, EJ, EK)
    assert st["terms_fp32"] > 0
    assert dJ < 1e-7 and dK < 1e-7 and dEJ < 1e-6 and dEK < 1e-6


def test_cfg3_mixed_sampled_rows(lib, oracle_mod):
    """The 64-water cell in mixed precision (FP32 below a bound of 1e-6)
    against the FP64 oracle's exact rows of three bra shells."""
    s = inputs.cfg3()
    shells = [0, 3, 7]
    ref = oracle_mod.jk(s, bra_shells=shells)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    print(f"cfg3: fp32 terms {st['terms_fp32']:.3e} of {st['terms']:.3e}; build {st['t_build_ms']:.1f} ms "
          f"(sr {st['t_sr_ms']:.1f})", flush=True)
    dJ, dK, _, _ = _report("cfg3 rows", J, K, ref, s.natom)
    assert st["terms_fp32"] > 0
    assert dJ < 1e-7 and dK < 1e-7


D_CASES = [
    dict(seed=21, natom=2, recipe=((0, 0), (1, 0), (2, 1)), lo=0.5, hi=4.0, nprim=2, a_ang=3.0),
    dict(seed=22, natom=2, recipe=((2, 0), (1, 0)), lo=0.4, hi=3.0, nprim=2, a_ang=2.8, skew=0.1),
]


@pytest.mark.parametrize("case", D_CASES, ids=["spd_spherical", "pd_cartesian_skewed"])
def test_d_shells(lib, oracle_mod, case):
    """d shells (spherical and Cartesian, skewed cell): every one of the 21
    class pairs, through both the per-lane and the cooperative kernels."""
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    dJ, dK, dEJ, dEK = _report(f"{s.name} d (terms {st['terms']:.0f})", J, K, ref, s.natom, EJ, EK)
    assert dJ < 1e-9 and dK < 1e-9 and dEJ < 1e-9 and dEK < 1e-9


@pytest.mark.parametrize("mask,key", [(1, "sr"), (2, "lr"), (4, "self")])
def test_d_parts(lib, oracle_mod, mask, key):
    s = inputs.small_cell(**D_CASES[0])
    ref = oracle_mod.jk(s, parts=key)
    with lib.Handle(s) as h:
        h.set_parts(mask)
        J, K, _, _ = h.build(s.D)
    dJ, dK, _, _ = _report(f"d part {key}", J, K, ref, s.natom)
    assert dJ < 1e-9 and dK < 1e-9


def test_d_mixed(lib, oracle_mod):
    s = inputs.small_cell(**D_CASES[0])
    ref = oracle_mod.jk(s)
    thr = Thresholds(**{**s.thr.__dict__, "fp32_below": 4e-3})
    with lib.Handle(s, thr=thr) as h:
        J, K, EJ, EK = h.build(s.D)
        st = h.stats()
    dJ, dK, dEJ, dEK = _report(f"d mixed (fp32 {st['terms_fp32']:.0f}/{st['terms']:.0f})", J, K, ref, s.natom,
                               EJ, EK)
    assert dJ < 1e-7 and dK < 1e-7 and dEJ < 1e-6 and dEK < 1e-6


def test_d_kernel_choice_over_builds(lib, oracle_mod):
    """Repeated builds of one d-shell cell: the first runs the large d class
    pairs in component slices, later ones choose per class pair from the
    previous build's shifts per quartet (this small cell has many, so the
    one-wavefront-per-group-pair kernel takes over) and fold the lattice
    sums.  Every build must match the oracle."""
    case = D_CASES[0]
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s)
    with lib.Handle(s) as h:
        for k in range(3):
            J, K, EJ, EK = h.build(s.D)
            st = h.stats()
            ratio = st["terms"] / max(1.0, st["quartets"])
            dJ, dK, dEJ, dEK = _report(f"d build {k} (shifts/quartet {ratio:.1f})", J, K, ref, s.natom, EJ, EK)
            assert dJ < 1e-9 and dK < 1e-9 and dEJ < 1e-9 and dEK < 1e-9


# ---------------------------------------------------------------- J-engine (builds without K)

J_CASES = [dict(seed=3, natom=2, recipe=((0, 0), (1, 0))),
           dict(seed=5, natom=3, recipe=((0, 0), (0, 0), (1, 0)), skew=0.15, omega=0.35),
           D_CASES[0], D_CASES[1]]


@pytest.mark.parametrize("case", J_CASES, ids=["sp", "sp_skewed", "spd_spherical", "pd_cartesian_skewed"])
def test_j_only_engine(lib, oracle_mod, case):
    """Without K the short range runs the J-engine (Hermite densities of the
    pairs, Sec. 3.2): J against the oracle's J at the FP64 bar, and the
    counters show which class pairs it ran (total angular momentum <= 5)."""
    s = inputs.small_cell(**case)
    ref = oracle_mod.jk(s)
    with lib.Handle(s) as h:
        J, K, EJ, EK = h.build(s.D, want_K=False)
        st = h.stats()
    assert K is None and EK is None
    dJ = np.abs(J - ref["J"]).max()
    dEJ = abs(EJ - ref["E_J"]) / s.natom
    print(f"J-only {s.name}: max|dJ|={dJ:.3e} dE_J/atom={dEJ:.3e} jengine mask {st['sr_jengine_mask']:#x}",
          flush=True)
    assert dJ < 1e-9 and dEJ < 1e-9
    assert st["sr_jengine_mask"] != 0


def test_j_only_cfg1_and_cfg2_rows(lib, oracle_mod):
    s1 = inputs.cfg1()
    ref1 = oracle_mod.jk(s1)
    with lib.Handle(s1) as h:
        J1, _, EJ1, _ = h.build(s1.D, want_K=False)
    d1 = np.abs(J1 - ref1["J"]).max()
    s2 = inputs.cfg2()
    shells = [0, 3, 7]
    ref2 = oracle_mod.jk(s2, bra_shells=shells)
    rows = ref2["rows"]
    with lib.Handle(s2) as h:
        J2, _, _, _ = h.build(s2.D, want_K=False)
        st = h.stats()
    d2 = np.abs(J2[rows] - ref2["J"][rows]).max()
    print(f"J-only cfg1 max|dJ|={d1:.3e} dE_J={EJ1 - ref1['E_J']:.3e}; cfg2 rows max|dJ|={d2:.3e}, "
          f"short range {st['t_sr_ms']:.1f} ms, build {st['t_build_ms']:.1f} ms", flush=True)
    assert d1 < 1e-9 and abs(EJ1 - ref1["E_J"]) < 1e-9 and d2 < 1e-9
    # every class pair of the s/p cell whose bra is not an s-s pair ran the
    # J-engine; the (ss|..) ones ran the fused kernel
    slots = [(cb, ck) for cb in range(6) for ck in range(cb, 6)]
    for k, (cb, ck) in enumerate(slots):
        if st["terms_class"][k] > 0:
            assert bool((st["sr_jengine_mask"] >> k) & 1) == (cb >= 1), k
