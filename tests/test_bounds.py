"""CPU checks of the inequalities the library's real-space neighbour lists
rely on (no GPU): the separable bound of the real-space sphere argument and
the lattice lower bound used by the single-image fast path."""
import numpy as np


def test_separable_sphere_bound():
    """C2e (1 - c) <= Z_bra Z_ket with
    C2e = Cb Ck 2 pi^{5/2}/(pq sqrt(p+q)), c = w/sqrt(rho + w^2),
    Z = sqrt2 pi^{5/4} C/(p (p + 2 a_min)^{1/4}) sqrt(1 - w/sqrt(p + w^2)),
    for exponents p, q >= 2 a_min."""
    rng = np.random.default_rng(0)
    for _ in range(20000):
        amin = rng.uniform(0.01, 2.0)
        p, q = 2 * amin + rng.exponential(5.0, 2)
        w = rng.uniform(0.05, 3.0)
        rho = p * q / (p + q)
        lhs = 2 * np.pi ** 2.5 / (p * q * np.sqrt(p + q)) * (1 - w / np.sqrt(rho + w * w))

        def z(x):
            return np.sqrt(2) * np.pi ** 1.25 / (x * (x + 2 * amin) ** 0.25) * np.sqrt(1 - w / np.sqrt(x + w * w))
        assert lhs <= z(p) * z(q) * (1 + 1e-12)


def test_lattice_lower_bound():
    """Every non-zero lattice vector is at least min_i 1/|Minv[:, i]| long."""
    rng = np.random.default_rng(1)
    for _ in range(200):
        M = np.eye(3) * rng.uniform(3, 9) + rng.uniform(-2.5, 2.5, (3, 3)) * (1 - np.eye(3))
        if abs(np.linalg.det(M)) < 1.0:
            continue
        Minv = np.linalg.inv(M)
        rmin = min(1.0 / np.linalg.norm(Minv[:, j]) for j in range(3))
        n = 6
        rr = np.arange(-n, n + 1)
        N = np.array(np.meshgrid(rr, rr, rr, indexing="ij")).reshape(3, -1).T
        N = N[np.any(N != 0, axis=1)]
        shortest = np.min(np.linalg.norm(N @ M, axis=1))
        assert rmin <= shortest * (1 + 1e-12)
