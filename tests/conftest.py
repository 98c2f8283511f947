import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running oracle cases")


@pytest.fixture(scope="session")
def rule3():
    """12^3 tensor Gauss--Hermite rule with the 35-moment basis (oracle)."""
    from oracle import basis, quadrature
    nodes, w = quadrature.tensor_rule(12, 3)
    return dict(nodes=nodes, w=w, logw=quadrature.lebesgue_log_weights(nodes, w),
                Phi=basis.evaluate(nodes, 3))


@pytest.fixture(scope="session")
def rule1():
    """16-node 1D rule with the 5-moment basis (oracle)."""
    from oracle import basis, quadrature
    x, w = quadrature.gauss_hermite(16)
    nodes = x[:, None]
    return dict(nodes=nodes, w=w, logw=quadrature.lebesgue_log_weights(nodes, w),
                Phi=basis.evaluate(nodes, 1))
