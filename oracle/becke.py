"""Periodic Becke partition weights (TEST INFRASTRUCTURE).

Only the tests and the ``cpu_baseline`` leg of ``bench.py`` may use this
module.  Plain numpy in FP64, written from Sec. 2.8 ("Becke weights"):

  weight of grid point r with origin atom A      eq. becke_weight_definition:
      w(r) = P(A, r) / sum_X P(X, r)
  vicinity function                              eq. becke_vicinity_definition:
      P(X, r) = prod_{Y != X} s(X, Y, r) over the other atoms in every
      lattice image and the other images of X itself
  switching function                             eqs. becke_mu_definition,
      u = (|r - X| - |r - Y|) / |X - Y|               becke_switch_definition
      s = (1 - f(f(f(u)))) / 2,  f(x) = x (3 - x^2) / 2
  truncation: the images X, Y taken are the atom images within a sphere of
  radius rcut (17 bohr) about the origin atom A of the point; P(X, r) is zero
  as soon as one switching factor is below delta, and the weight is zero when
  P(A, r) is below delta.

Readings: the printed denominator writes a product over R3 of P(B + R3, r);
the weights of one point over all atom images then do not sum to one, and
the text that follows goes through every atom and its images within the
sphere for the denominator, so it is read as the sum over atom images B + R3
within the sphere of P(B + R3, r).
"""
from __future__ import annotations

import numpy as np


def switch(u):
    """s(u) of eq. becke_switch_definition (elementwise)."""
    f1 = 0.5 * u * (3.0 - u * u)
    f2 = 0.5 * f1 * (3.0 - f1 * f1)
    f3 = 0.5 * f2 * (3.0 - f2 * f2)
    return 0.5 * (1.0 - f3)


def atom_images(cell, xyz, a, rcut):
    """Positions of every atom image B + n0 a + n1 b + n2 c within rcut of
    atom a (its home position), the origin atom itself first."""
    cell = np.asarray(cell, float)
    xyz = np.asarray(xyz, float)
    A = xyz[a]
    inv = np.linalg.inv(cell)
    # integer range: |n_i| <= |f_i| + rcut * (column norm of the inverse)
    span = np.linalg.norm(inv, axis=0)
    out = [A.copy()]
    for b in range(len(xyz)):
        f = (xyz[b] - A) @ inv
        lo = np.floor(-f - rcut * span).astype(int)
        hi = np.ceil(-f + rcut * span).astype(int)
        for n0 in range(lo[0], hi[0] + 1):
            for n1 in range(lo[1], hi[1] + 1):
                for n2 in range(lo[2], hi[2] + 1):
                    if b == a and n0 == 0 and n1 == 0 and n2 == 0:
                        continue
                    Y = xyz[b] + n0 * cell[0] + n1 * cell[1] + n2 * cell[2]
                    if np.linalg.norm(Y - A) <= rcut:
                        out.append(Y)
    return np.array(out)


def vicinity(images, pts, delta):
    """P(X, r) for every image X (columns) and point r (rows): the product
    over the other images Y of s(X, Y, r), zero where a factor is < delta."""
    d = np.linalg.norm(pts[:, None, :] - images[None, :, :], axis=2)          # |r - X|
    D = np.linalg.norm(images[:, None, :] - images[None, :, :], axis=2)       # |X - Y|
    M = len(images)
    off = ~np.eye(M, dtype=bool)
    Dsafe = np.where(off, D, 1.0)
    u = (d[:, :, None] - d[:, None, :]) / Dsafe[None, :, :]                   # u[r, X, Y]
    s = np.where(off[None, :, :], switch(u), 1.0)
    P = np.prod(s, axis=2)
    dead = np.any(s < delta, axis=2)
    return np.where(dead, 0.0, P)


def becke_weights(cell, xyz, pts, origin, rcut=17.0, delta=1e-14, chunk=512):
    """Becke weight of each point with respect to its origin atom."""
    pts = np.asarray(pts, float)
    origin = np.asarray(origin, int)
    w = np.zeros(len(pts))
    for a in np.unique(origin):
        img = atom_images(cell, xyz, int(a), rcut)
        idx = np.nonzero(origin == a)[0]
        for c0 in range(0, len(idx), chunk):
            sel = idx[c0:c0 + chunk]
            P = vicinity(img, pts[sel], delta)
            num = P[:, 0]
            den = P.sum(axis=1)
            w[sel] = np.where(num < delta, 0.0, num / np.where(den > 0, den, 1.0))
    return w
