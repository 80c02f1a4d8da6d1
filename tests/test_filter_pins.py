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


# ------------------------------------------------ per-edge design variables
def _edge_positions(dims):
    """Physical positions (x, y, z) of every design edge, x edges first."""
    pts = []
    for c in range(3):
        sz, sy, sx = OF.edge_shape(dims, c)
        for k in range(sz):
            for j in range(sy):
                for i in range(sx):
                    p = [float(i), float(j), float(k)]
                    p[c] += 0.5
                    pts.append(p)
    return np.array(pts)


def _brute_edge_filter(flat, dims, R):
    """Eq. FilterFunction written out over the edge positions: every pair."""
    P = _edge_positions(dims)
    out = np.empty(len(P))
    for n in range(len(P)):
        d = np.sqrt(((P - P[n]) ** 2).sum(axis=1))
        w = np.where(d < R, R - d, 0.0)
        out[n] = (w * flat).sum() / w.sum()
    return out


def _flat(arrs):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in arrs])


@pytest.mark.parametrize("R", [1.0, 1.7, 2.5])
def test_edge_filter_matches_brute_force(R):
    dims = (3, 2, 4)
    rng = np.random.default_rng(5)
    rho = [rng.random(OF.edge_shape(dims, c)) for c in range(3)]
    got = _flat(OF.cone_filter_edges(rho, dims, R))
    assert np.allclose(got, _brute_edge_filter(_flat(rho), dims, R), rtol=0, atol=1e-14)


def test_edge_filter_keeps_constants_and_interior_linear_fields():
    """The per-edge filter reproduces a linear function of position wherever
    the whole sphere holds design edges: the staggered positions enter with
    their half-cell offsets (a filter that put every edge at its cell corner
    would shift the field by half a cell)."""
    dims, R = (9, 8, 10), 2.3
    c = [np.full(OF.edge_shape(dims, a), 0.42) for a in range(3)]
    assert all(np.allclose(x, 0.42, rtol=0, atol=1e-15) for x in OF.cone_filter_edges(c, dims, R))
    lin, inner = [], []
    m = int(math.ceil(R)) + 1
    for a in range(3):
        k, j, i = np.meshgrid(*[np.arange(s) for s in OF.edge_shape(dims, a)], indexing="ij")
        x, y, z = i.astype(float), j.astype(float), k.astype(float)
        (x, y, z)[a][...] += 0.5
        lin.append(0.01 * x - 0.02 * y + 0.03 * z + 0.1)
        sz, sy, sx = OF.edge_shape(dims, a)
        inner.append((slice(m, sz - m), slice(m, sy - m), slice(m, sx - m)))
    f = OF.cone_filter_edges(lin, dims, R)
    for a in range(3):
        assert np.allclose(f[a][inner[a]], lin[a][inner[a]], rtol=0, atol=1e-14)


def test_edge_filter_chain_rule_matches_finite_differences():
    rng = np.random.default_rng(7)
    dims, R, beta, eta = (4, 3, 5), 2.1, 6.0, 0.45
    rho = [rng.random(OF.edge_shape(dims, c)) for c in range(3)]
    cvec = [rng.standard_normal(OF.edge_shape(dims, c)) for c in range(3)]

    def F(r):
        rt = OF.cone_filter_edges(r, dims, R)
        return float(sum(np.sum(cvec[a] * OF.project(rt[a], beta, eta)) for a in range(3)))

    g = OF.filter_project_grad_edges(cvec, rho, dims, R, beta, eta)
    h = 1e-6
    for (a, idx) in [(0, (0, 0, 0)), (0, (5, 3, 3)), (1, (2, 1, 4)), (1, (5, 2, 0)), (2, (3, 3, 4)), (2, (1, 0, 2))]:
        rp = [x.copy() for x in rho]
        rm = [x.copy() for x in rho]
        rp[a][idx] += h
        rm[a][idx] -= h
        fd = (F(rp) - F(rm)) / (2 * h)
        assert g[a][idx] == pytest.approx(fd, rel=1e-7, abs=1e-10)
