"""Weighted reblocking (App. C) on series with known statistics."""

import numpy as np

from oracle.reblock import reblock, reblock_converged


def test_iid_series_standard_error():
    rng = np.random.default_rng(1)
    x = rng.normal(3.0, 2.0, size=20000)
    w = np.ones_like(x)
    X, S, err, nb = reblock(x, w, 1)
    assert abs(X - x.mean()) < 1e-12
    assert abs(err - 2.0 / np.sqrt(x.size)) < 0.05 * 2.0 / np.sqrt(x.size)
    m, e, L, ok = reblock_converged(x, w, discard=0)
    assert ok and abs(e - 2.0 / np.sqrt(x.size)) < 0.15 * 2.0 / np.sqrt(x.size)


def test_weighted_mean_and_variance_definition():
    # two blocks, unequal weights: X = sum w'x'/v1, S^2 = sum w'(x'-X)^2 / (v1 - v2/v1)
    x = np.array([1.0, 3.0])
    w = np.array([1.0, 3.0])
    X, S, err, nb = reblock(x, w, 1)
    assert abs(X - 2.5) < 1e-15
    v1, v2 = 4.0, 10.0
    assert abs(S ** 2 - (1 * 1.5 ** 2 + 3 * 0.5 ** 2) / (v1 - v2 / v1)) < 1e-14
    assert nb == 2 and abs(err - S) < 1e-15


def test_correlated_series_needs_blocking():
    """AR(1) with phi = 0.9: the naive error underestimates by sqrt((1+phi)/(1-phi)) ~ 4.36;
    reblocking recovers the true error of the mean."""
    rng = np.random.default_rng(2)
    n, phi = 2 ** 17, 0.9
    e = rng.normal(size=n)
    x = np.empty(n)
    x[0] = e[0]
    for i in range(1, n):
        x[i] = phi * x[i - 1] + e[i]
    w = np.ones(n)
    naive = reblock(x, w, 1)[2]
    m, err, L, ok = reblock_converged(x, w, discard=0)
    true = np.sqrt(1 / (1 - phi ** 2)) * np.sqrt((1 + phi) / (1 - phi)) / np.sqrt(n)
    assert err > 3 * naive
    assert abs(err - true) < 0.25 * true


def test_zero_variance_series_reaches_plateau():
    """A constant series has zero error at every block length: the plateau rule (error growth
    below the ratio on doubling, App. C) must accept it instead of doubling forever."""
    x = np.full(512, -12.5)
    m, err, L, ok = reblock_converged(x, np.ones(512), discard=0)
    assert ok and err == 0.0 and m == -12.5 and L == 2
    m, err, L, ok = reblock_converged(x, np.linspace(1.0, 2.0, 512), discard=0)
    assert ok and err < 1e-12 and abs(m + 12.5) < 1e-12
