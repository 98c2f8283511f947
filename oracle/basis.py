"""Sufficient statistics for the oracle (test infrastructure only).

App. B writes the 35-moment statistics in an orthogonal (Hermite) form.  For
the full 3D velocity space the same idea is the orthonormal tensor Hermite
basis up to total degree 4:

    phi_(a,b,c)(u) = He_a(u_1) He_b(u_2) He_c(u_3) / sqrt(a! b! c!),  a+b+c <= 4,

which is orthonormal under N(0, I_3).  1D uses phi_k = He_k / sqrt(k!),
k = 0..4.  Ordering: by total degree, then lexicographically descending in
(a, b, c), so index 0 is the constant and indices 1, 2, 3 are u_1, u_2, u_3.

He_n is evaluated by the three-term recurrence He_{n+1} = x He_n - n He_{n-1}.
"""

import math

import numpy as np


def multi_indices(dim, degree=4):
    """Ordered list of exponent tuples with total degree <= ``degree``."""
    out = []
    for tot in range(degree + 1):
        if dim == 1:
            out.append((tot,))
            continue
        level = []
        for a in range(tot, -1, -1):
            for b in range(tot - a, -1, -1):
                c = tot - a - b
                level.append((a, b, c))
        out.extend(level)
    return out


def hermite_e(nmax, x):
    """Array He_0..He_nmax evaluated at x (shape (nmax+1,) + x.shape)."""
    x = np.asarray(x, dtype=np.float64)
    H = np.empty((nmax + 1,) + x.shape, dtype=np.float64)
    H[0] = 1.0
    if nmax >= 1:
        H[1] = x
    for n in range(1, nmax):
        H[n + 1] = x * H[n] - n * H[n - 1]
    return H


def evaluate(nodes, dim, degree=4):
    """Phi[p, i] = phi_i(nodes[p]) for the ordered basis."""
    nodes = np.asarray(nodes, dtype=np.float64).reshape(-1, dim)
    idx = multi_indices(dim, degree)
    H = [hermite_e(degree, nodes[:, d]) for d in range(dim)]
    Phi = np.empty((nodes.shape[0], len(idx)), dtype=np.float64)
    for i, e in enumerate(idx):
        v = np.ones(nodes.shape[0])
        norm = 1.0
        for d, a in enumerate(e):
            v = v * H[d][a]
            norm *= math.factorial(a)
        Phi[:, i] = v / math.sqrt(norm)
    return Phi


def index_of(dim, expo):
    """Position of an exponent tuple in the ordered basis."""
    return multi_indices(dim).index(tuple(expo))
