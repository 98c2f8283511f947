"""Oracle-side targets that need the parameter-to-moment map (test infrastructure).

The 1D perturbed-Maxwellian workload draws multipliers, not moments, so its
targets are moments of the canonical-form density (Sec. 3.1, eq. "Numerical
integration moments") evaluated with a 64-node Gauss--Hermite rule in FP64, in
the generating Maxwellian's gauge (v, sqrt(T)).

Reading (the workload statement leaves realizability open): candidates whose
64-node density puts more than 1e-10 of its mass beyond |x| > 6 are skipped,
because a 16-node rule (span +-6.63) cannot represent such a far-tail mode.
"""

import numpy as np

from . import basis as _basis
from . import maxent as _maxent
from . import quadrature as _quad


def config1_targets(cand, n_cells, n_nodes=64, tail=6.0, tail_mass=1e-10):
    """Targets M (n_cells, 5), gauge g (n_cells, 2), generating beta (n_cells, 5)."""
    x, w = _quad.gauss_hermite(n_nodes)
    nodes = x[:, None]
    logw = _quad.lebesgue_log_weights(nodes, w)
    Phi = _basis.evaluate(nodes, 1)
    P = cand["n"].shape[0]
    beta = np.zeros((P, 5))
    beta[:, 0] = cand["n"]
    beta[:, 2] = -1.0 / np.sqrt(2.0)
    beta[:, 3] = cand["c3"]
    beta[:, 4] = cand["c4"]
    sig = _maxent.sigma(beta, Phi, logw)
    far = np.sum(sig[:, np.abs(x) > tail], axis=1)
    keep = np.nonzero(far <= tail_mass)[0][:n_cells]
    if keep.size < n_cells:
        raise ValueError("candidate pool too small")
    b = beta[keep]
    M = b[:, :1] * (sig[keep] @ Phi)
    g = np.stack([cand["v"][keep], np.sqrt(cand["T"][keep])], axis=1)
    return M, g, b
