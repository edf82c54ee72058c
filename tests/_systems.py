"""Hand-built test systems (inputs only; no method arithmetic)."""
import numpy as np

from paper_2410_22278_amd.inputs import System, Thresholds


def make_system(cell, xyz, shells, omega, thr=None, D=None, pure=None, name="t"):
    """shells: list of (atom, l, exps, coefs)."""
    sa, sl, sp, sn, ex, co = [], [], [], [], [], []
    for k, (atom, l, e, c) in enumerate(shells):
        sa.append(atom); sl.append(l); sn.append(len(e))
        sp.append(int(pure[k]) if pure is not None else 0)
        ex += list(e); co += list(c)
    return System(name, np.asarray(cell, float), np.asarray(xyz, float), np.ones(len(xyz)),
                  np.array(sa, np.int32), np.array(sl, np.int32), np.array(sp, np.int32),
                  np.array(sn, np.int32), np.array(ex, float), np.array(co, float),
                  float(omega), thr if thr is not None else Thresholds.uniform(1e-14), D)


def nacl(a=10.0):
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    xyz = np.concatenate([fcc * a, (fcc + np.array([.5, 0, 0])) * a])
    q = np.array([1.0] * 4 + [-1.0] * 4)
    return xyz, q


def random_density(rng, nbf, nocc=None, psd=True):
    if psd:
        C = rng.standard_normal((nbf, nocc or nbf)) / np.sqrt(nbf)
        D = C @ C.T
    else:
        X = rng.standard_normal((nbf, nbf)) / nbf
        D = X + X.T
    return 0.5 * (D + D.T)
