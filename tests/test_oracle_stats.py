"""Pins of the online statistics oracle (Sec. 2.5; formulas in oracle/stats.py)."""
import numpy as np
import pytest

from oracle import stats


def _fields(rng, dims, d, n, offset=0.0):
    N = dims[0] * dims[1] * dims[2]
    return [offset + rng.standard_normal((d, N)) * (1 + 0.3 * q) for q in range(n)]


@pytest.mark.parametrize("dims,d,axis", [((5, 4, 3), 3, 1), ((6, 5, 1), 2, 1), ((4, 3, 5), 3, 0), ((4, 3, 5), 3, 2)])
def test_online_equals_definition(dims, d, axis):
    """Online merging equals the mean and population covariance of all samples of a plane
    pooled over the steps, computed cell by cell with plain loops."""
    rng = np.random.default_rng(0)
    us = _fields(rng, dims, d, 4, offset=3.0)
    st = stats.empty_state(dims[axis], d)
    for u in us:
        st = stats.accumulate(st, u, dims, axis)
    mean, cov = stats.finalize(st)
    nx, ny, nz = dims
    for p in range(dims[axis]):
        samples = []
        for u in us:
            for k in range(nz):
                for j in range(ny):
                    for i in range(nx):
                        if (i, j, k)[axis] == p:
                            samples.append(u[:, i + nx * (j + ny * k)])
        S = np.array(samples)
        mu = S.mean(axis=0)
        assert np.allclose(mean[p], mu, rtol=1e-13, atol=1e-13)
        for q, (i, j) in enumerate(stats.pairs(d)):
            ref = np.mean((S[:, i] - mu[i]) * (S[:, j] - mu[j]))
            assert abs(cov[p, q] - ref) <= 1e-12 * max(1.0, abs(ref))


def test_order_independence_and_exact_zero():
    rng = np.random.default_rng(1)
    dims, d = (6, 4, 3), 3
    us = _fields(rng, dims, d, 5)
    a = stats.empty_state(4, d)
    b = stats.empty_state(4, d)
    for u in us:
        a = stats.accumulate(a, u, dims, 1)
    for u in us[::-1]:
        b = stats.accumulate(b, u, dims, 1)
    assert np.allclose(a["mu"], b["mu"], rtol=1e-13) and np.allclose(a["C"], b["C"], rtol=1e-12)
    c = stats.empty_state(4, d)
    const = np.full((d, 72), 2.5)
    for _ in range(3):
        c = stats.accumulate(c, const, dims, 1)
    assert np.all(c["C"] == 0.0) and np.all(c["mu"] == 2.5)


def test_shift_invariance_of_covariance():
    rng = np.random.default_rng(2)
    dims, d = (5, 6, 2), 3
    us = _fields(rng, dims, d, 3)
    a = stats.empty_state(6, d)
    b = stats.empty_state(6, d)
    for u in us:
        a = stats.accumulate(a, u, dims, 1)
        b = stats.accumulate(b, u + 1e3, dims, 1)
    assert np.allclose(stats.finalize(a)[1], stats.finalize(b)[1], rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_vjp_complex_step(axis):
    rng = np.random.default_rng(3)
    dims, d = (4, 5, 3), 3
    us = _fields(rng, dims, d, 3)
    np_ = dims[axis]
    mbar = rng.standard_normal((np_, d))
    cbar = rng.standard_normal((np_, len(stats.pairs(d))))

    def loss(fields):
        st = stats.empty_state(np_, d)
        for u in fields:
            st = stats.accumulate(st, u, dims, axis)
        m, c = stats.finalize(st)
        return np.sum(mbar * m) + np.sum(cbar * c)

    st = stats.empty_state(np_, d)
    for u in us:
        st = stats.accumulate(st, u, dims, axis)
    for q in range(3):
        g = stats.stats_vjp(st, us[q], dims, axis, mbar, cbar)
        v = rng.standard_normal(us[q].shape)
        h = 1e-30
        pert = [u.astype(complex) for u in us]
        pert[q] = pert[q] + 1j * h * v
        cs = loss(pert).imag / h
        assert abs(cs - np.sum(g * v)) <= 1e-12 * max(1.0, abs(cs))
