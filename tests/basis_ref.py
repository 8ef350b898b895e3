"""Test-side basis evaluation (numpy), written independently of the oracle.

Per cell K = x_K + [0,h]^3 the basis is phi_{abc}(x) = h^{-3/2} psi_a(xi_1)
psi_b(xi_2) psi_c(xi_3), xi = (x - x_K)/h, psi_m(t) = sqrt(2m+1) P_m(2t-1);
ordered by total degree, then (a,b,c) lexicographically descending.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def orders(p):
    out = []
    for d in range(p + 1):
        for a in range(d, -1, -1):
            for b in range(d - a, -1, -1):
                out.append((a, b, d - a - b))
    return out


def psi(m, t):
    c = np.zeros(m + 1)
    c[m] = 1.0
    return np.sqrt(2 * m + 1) * npleg.legval(2 * np.asarray(t) - 1, c)


def eval_cell(p, h, xi):
    """Basis values at reference points xi (n,3) in [0,1]^3 -> (n, bs)."""
    cols = [h ** -1.5 * psi(a, xi[:, 0]) * psi(b, xi[:, 1]) * psi(c, xi[:, 2]) for (a, b, c) in orders(p)]
    return np.stack(cols, axis=1)


def gauss01(q):
    x, w = npleg.leggauss(q)
    return 0.5 * (x + 1), 0.5 * w


def tensor_points(q):
    x, w = gauss01(q)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = (w[:, None, None] * w[None, :, None] * w[None, None, :]).reshape(-1)
    return np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], axis=1), W
