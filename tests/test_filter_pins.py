"""Pins of the FP64 filter / projection oracle (oracle/filters.py) against
brute force, closed forms and finite differences (no GPU)."""
import math

import numpy as np
import pytest

from oracle import filters as OF


def _brute_filter(rho, R):
    """Eq. FilterFunction with one explicit sum per voxel over the whole box."""
    nz, ny, nx = rho.shape
    out = np.zeros_like(rho, dtype=np.float64)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                num = den = 0.0
                for kk in range(nz):
                    for jj in range(ny):
                        for ii in range(nx):
                            d = math.sqrt((i - ii) ** 2 + (j - jj) ** 2 + (k - kk) ** 2)
                            if d < R:
                                num += (R - d) * rho[kk, jj, ii]
                                den += R - d
                out[k, j, i] = num / den
    return out


@pytest.mark.parametrize("R", [1.0, 1.7, 2.5])
def test_cone_filter_matches_brute_force(R):
    rho = np.random.default_rng(3).random((4, 5, 6))
    assert np.allclose(OF.cone_filter(rho, R), _brute_filter(rho, R), rtol=0, atol=1e-14)


def test_filter_keeps_constants_and_interior_linear_fields():
    """Normalised weights: a constant stays constant everywhere; symmetric
    weights: a linear field is kept wherever the whole sphere is inside."""
    R = 2.6
    c = np.full((9, 8, 10), 0.37)
    assert np.allclose(OF.cone_filter(c, R), 0.37, rtol=0, atol=1e-15)
    k, j, i = np.meshgrid(np.arange(9), np.arange(8), np.arange(10), indexing="ij")
    lin = 0.01 * i - 0.02 * j + 0.03 * k + 0.1
    f = OF.cone_filter(lin, R)
    m = int(math.ceil(R))
    inner = (slice(m, 9 - m), slice(m, 8 - m), slice(m, 10 - m))
    assert np.allclose(f[inner], lin[inner], rtol=0, atol=1e-14)


def test_projection_closed_forms():
    beta, eta = 8.0, 0.4
    den = math.tanh(beta * eta) + math.tanh(beta * (1 - eta))
    assert OF.project(np.array([0.0]), beta, eta)[0] == pytest.approx(0.0, abs=1e-15)
    assert OF.project(np.array([1.0]), beta, eta)[0] == pytest.approx(1.0, abs=1e-15)
    assert OF.project(np.array([eta]), beta, eta)[0] == pytest.approx(math.tanh(beta * eta) / den, abs=1e-15)
    x = np.linspace(0, 1, 101)
    assert np.all(np.diff(OF.project(x, beta, eta)) > 0)
    # beta -> 0: the projection tends to the identity
    assert np.allclose(OF.project(x, 1e-6, eta), x, rtol=0, atol=1e-9)
    # derivative against central differences
    h = 1e-6
    fd = (OF.project(x + h, beta, eta) - OF.project(x - h, beta, eta)) / (2 * h)
    assert np.allclose(OF.project_derivative(x, beta, eta), fd, rtol=1e-7, atol=1e-9)


def test_filter_projection_chain_rule_matches_finite_differences():
    """Eq. GradientsFiltered against central differences of the linear
    functional F(rho) = sum c * project(filter(rho)) (smooth, so FD with
    h = 1e-6 is accurate to ~1e-9 relative)."""
    rng = np.random.default_rng(9)
    rho = rng.random((5, 6, 7))
    c = rng.standard_normal(rho.shape)
    R, beta, eta = 2.2, 5.0, 0.5

    def F(r):
        return float(np.sum(c * OF.project(OF.cone_filter(r, R), beta, eta)))

    g = OF.filter_project_grad(c, rho, R, beta, eta)
    h = 1e-6
    for idx in [(0, 0, 0), (2, 3, 4), (4, 5, 6), (1, 0, 5), (3, 2, 1)]:
        rp, rm = rho.copy(), rho.copy()
        rp[idx] += h
        rm[idx] -= h
        fd = (F(rp) - F(rm)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-7, abs=1e-10)


def test_nondiscreteness_extremes():
    assert OF.nondiscreteness(np.array([0.0, 1.0, 1.0, 0.0])) == 0.0
    assert OF.nondiscreteness(np.full(10, 0.5)) == pytest.approx(100.0)
    assert OF.nondiscreteness(np.array([0.25])) == pytest.approx(75.0)
