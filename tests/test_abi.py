"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid inputs before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2410_22278_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pbcjk.h")).read()
    return sorted(set(re.findall(r"\b(pbc_jk_\w+)\s*\(", txt)))


def test_header_and_binding_agree():
    from paper_2410_22278_amd import pbcjk
    assert _declared() == sorted(pbcjk.EXPORTS)


def test_library_exports_every_declared_symbol():
    from paper_2410_22278_amd import pbcjk
    lib = ctypes.CDLL(pbcjk.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def _create(s, **over):
    from paper_2410_22278_amd import pbcjk
    args = dict(cell=s.cell, xyz=s.xyz, shell_atom=s.shell_atom, shell_l=s.shell_l,
                shell_pure=s.shell_pure, shell_nprim=s.shell_nprim, exps=s.exps, coefs=s.coefs,
                omega=s.omega, thr=s.thr)
    args.update(over)
    return pbcjk.pbc_jk_create(**args)


@pytest.mark.parametrize("what", ["l3", "neg_exp", "nan_xyz", "singular", "bad_atom", "zero_thr",
                                  "nan_omega", "zero_prims"])
def test_invalid_inputs_rejected(what):
    from paper_2410_22278_amd import pbcjk
    s = inputs.small_cell(3, natom=2)
    over = {}
    if what == "l3":
        l = s.shell_l.copy(); l[0] = 3; over["shell_l"] = l
    elif what == "neg_exp":
        e = s.exps.copy(); e[1] = -0.5; over["exps"] = e
    elif what == "nan_xyz":
        x = s.xyz.copy(); x[0, 1] = np.nan; over["xyz"] = x
    elif what == "singular":
        c = s.cell.copy(); c[2] = c[0] + c[1]; over["cell"] = c
    elif what == "bad_atom":
        a = s.shell_atom.copy(); a[0] = 7; over["shell_atom"] = a
    elif what == "zero_thr":
        t = inputs.Thresholds.uniform(1e-10); t.schwarz = 0.0; over["thr"] = t
    elif what == "nan_omega":
        over["omega"] = float("nan")
    elif what == "zero_prims":
        n = s.shell_nprim.copy(); n[0] = 0; over["shell_nprim"] = n
    with pytest.raises(pbcjk.PbcJkError) as ei:
        _create(s, **over)
    assert ei.value.code == pbcjk.PBC_JK_EINVAL
    assert pbcjk.pbc_jk_last_error() != ""


def test_null_handle_calls():
    from paper_2410_22278_amd import pbcjk
    lib = pbcjk.load()
    assert lib.pbc_jk_nbf(None) == pbcjk.PBC_JK_EINVAL
    assert lib.pbc_jk_set_parts(None, 1) == pbcjk.PBC_JK_EINVAL
    assert lib.pbc_jk_set_lr(None, pbcjk.LR_DENSE, 0.0) == pbcjk.PBC_JK_EINVAL
    assert lib.pbc_jk_set_sr_classes(None, 1) == pbcjk.PBC_JK_EINVAL
    lib.pbc_jk_destroy(None)   # NULL-safe
    assert lib.pbc_jk_build(None, None, None, None, None, None) == pbcjk.PBC_JK_EINVAL
