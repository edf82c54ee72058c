"""The allocation-free build (pbc_jk_build_device_static): its per-build work
buffers live in the library's static device array.  Through the C ABI, two
calls in a row (the second on a smaller cell, so the array is carved
differently and holds the first call's contents) must give what
pbc_jk_build_device gives on the same inputs, to the FP64 bar; a cell whose
work buffers do not fit fails with PBC_JK_ENOMEM before any work."""
import numpy as np
import pytest

from paper_2410_22278_amd import inputs

pytestmark = pytest.mark.gpu

BIG = dict(seed=41, natom=36, a_ang=7.0, recipe=((0, 0), (1, 0)), delta=1e-10, g_cut=2.0, r_cut=8.0)
SMALL = dict(seed=21, natom=2, recipe=((0, 0), (1, 0), (2, 1)), a_ang=3.2, lo=0.3, hi=4.0)


@pytest.fixture(scope="module")
def torch_lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_22278_amd import pbcjk
    pbcjk.load()
    return torch, pbcjk


def _both(torch, lib, s):
    with lib.Handle(s) as h:
        dD = torch.from_numpy(s.D).cuda()
        out = {}
        for name in ("regular", "static", "static again"):
            dJ = torch.full_like(dD, np.nan)
            dK = torch.full_like(dD, np.nan)
            fn = h.build_device if name == "regular" else h.build_device_static
            ej, ek = fn(dD, dJ, dK)
            torch.cuda.synchronize()
            out[name] = (dJ.cpu().numpy(), dK.cpu().numpy(), ej, ek, h.stats()["terms"])
    return out


def _check(tag, out, natom):
    J0, K0, ej0, ek0, t0 = out["regular"]
    for name in ("static", "static again"):
        J, K, ej, ek, t = out[name]
        dJ, dK = np.abs(J - J0).max(), np.abs(K - K0).max()
        print(f"{tag} {name}: max|dJ|={dJ:.2e} max|dK|={dK:.2e} dE_J={ej - ej0:.2e} dE_K={ek - ek0:.2e} "
              f"terms {t:.0f}/{t0:.0f}", flush=True)
        assert np.isfinite(J).all() and np.isfinite(K).all()
        assert dJ < 1e-10 and dK < 1e-10
        assert abs(ej - ej0) / natom < 1e-10 and abs(ek - ek0) / natom < 1e-10
        assert t == t0


def test_static_build_two_calls(torch_lib):
    torch, lib = torch_lib
    big = inputs.small_cell(**BIG)
    small = inputs.small_cell(**SMALL)
    assert small.nbf < big.nbf
    _check(f"nbf {big.nbf}", _both(torch, lib, big), big.natom)
    _check(f"nbf {small.nbf} after nbf {big.nbf}", _both(torch, lib, small), small.natom)


def test_static_build_rejects_oversize_cell(torch_lib):
    torch, lib = torch_lib
    s = inputs.small_cell(seed=3, natom=460, a_ang=26.0, recipe=((0, 0), (1, 0)), delta=1e-6, lo=1.0, hi=4.0)
    assert s.nbf > 1700
    with lib.Handle(s) as h:
        dD = torch.from_numpy(s.D).cuda()
        dJ = torch.empty_like(dD)
        dK = torch.empty_like(dD)
        with pytest.raises(lib.PbcJkError) as ei:
            h.build_device_static(dD, dJ, dK)
        assert ei.value.code == lib.PBC_JK_ENOMEM
        # the handle still builds normally
        h.build_device(dD, dJ, dK)
        torch.cuda.synchronize()
