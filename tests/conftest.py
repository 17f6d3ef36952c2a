import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the C-ABI on the GPU)")
    config.addinivalue_line("markers", "slow: full-size case (tens of seconds)")


_CACHE = {}


def oracle_hmatrix(key):
    """Session cache of oracle H-matrices for the small named meshes."""
    if key in _CACHE:
        return _CACHE[key]
    import oracle
    from paper_1911_00093_amd import meshes

    if key == "sphere-L2":
        m, leaf, eps = meshes.icosphere(2), 16, 1e-6
    elif key == "sphere-L3":
        m, leaf, eps = meshes.icosphere(3), 32, 1e-6
    elif key == "sphere-L4":
        m, leaf, eps = meshes.icosphere(4), 32, 1e-6
    elif key == "plates-16":
        m, leaf, eps = meshes.parallel_plates(16, 0.1, True), 64, 1e-5
    elif key == "plates-32":
        m, leaf, eps = meshes.parallel_plates(32, 0.1, True), 64, 1e-5
    elif key == "ellipsoid-12":
        m, leaf, eps = meshes.geodesic_ellipsoid(12, axes=(1.7, 0.8, 0.6)), 32, 1e-6
    elif key == "spheres-mixed":
        m = meshes.concat([meshes.icosphere(3)] + meshes.random_small_spheres(3, seed=0, level=1))
        leaf, eps = 32, 1e-6
    else:
        raise KeyError(key)
    h = oracle.HMatrix(m.centroids, m.areas, leaf=leaf, eta=2.0, eps=eps)
    _CACHE[key] = (m, h)
    return m, h


@pytest.fixture
def rng():
    return np.random.Generator(np.random.PCG64(1234))
