"""Pins of the quasi-Helmholtz projectors (Sec. II-D)."""
import numpy as np
import pytest

from oracle.operators import Projectors, pinv_laplacian
from oracle.topology import Topology
from workloads import meshes


@pytest.fixture(params=["sphere", "torus"])
def topo(request):
    if request.param == "sphere":
        return Topology(*meshes.icosphere(1))
    return Topology(*meshes.torus(1.0, 0.4, 8, 5))


def test_pseudo_inverse_penrose(topo):
    S = topo.Sigma.toarray()
    L = S.T @ S
    X = pinv_laplacian(L)
    assert np.allclose(L @ X @ L, L, atol=1e-12)
    assert np.allclose(X @ L @ X, X, atol=1e-12)
    assert np.allclose((L @ X).T, L @ X, atol=1e-12)
    assert np.allclose((X @ L).T, X @ L, atol=1e-12)
    assert np.allclose(X, np.linalg.pinv(L), atol=1e-10)  # independent SVD route


def test_projector_identities(topo):
    p = Projectors(topo)
    I = np.eye(topo.ne)
    L, S = topo.Lambda.toarray(), topo.Sigma.toarray()
    for P in (p.PS, p.PLH, p.PPL, p.PPSH):
        assert np.abs(P @ P - P).max() < 1e-12
        assert np.abs(P - P.T).max() < 1e-12
    assert np.abs(p.PS + p.PLH - I).max() < 1e-14
    assert np.abs(p.PPL + p.PPSH - I).max() < 1e-14
    assert np.abs(p.PS @ L).max() < 1e-12  # loops are not stars
    assert np.abs(p.PPL @ S).max() < 1e-12
    assert np.abs(p.PS @ S - S).max() < 1e-12
    assert np.abs(p.PPL @ L - L).max() < 1e-12
    assert np.linalg.matrix_rank(p.PS) == topo.nc - 1
    assert np.linalg.matrix_rank(p.PPL) == topo.nv - 1
    # harmonic subspace lies in the solenoidal (loop) ranges of both
    assert np.linalg.matrix_rank(p.PLH) == topo.ne - topo.nc + 1
