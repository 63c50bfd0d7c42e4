"""The seeded input stream: Philox4x64-10 bit-exact against numpy.random.Philox, and the
Gaussian fields / comb uniforms drawn from it."""

import numpy as np

from synthetic import comb_uniform, gaussian_fields, philox_u64, u64_to_unit
from synthetic.fields import STREAM_COMB


def _numpy_philox(ctr, key):
    # numpy's generator increments the 256-bit counter before each block: start one below.
    val = sum(int(c) << (64 * i) for i, c in enumerate(ctr))
    val = (val - 1) % (1 << 256)
    cm = np.array([(val >> (64 * i)) & ((1 << 64) - 1) for i in range(4)], dtype=np.uint64)
    return np.random.Philox(key=np.asarray(key, dtype=np.uint64), counter=cm).random_raw(4)


def test_philox_matches_numpy():
    rng = np.random.default_rng(0)
    for t in range(200):
        ctr = rng.integers(0, 2 ** 64, size=4, dtype=np.uint64)
        key = rng.integers(0, 2 ** 64, size=2, dtype=np.uint64)
        if t == 0:
            ctr[:] = 0
            key[:] = 0
        assert np.array_equal(philox_u64(ctr, key), _numpy_philox(ctr, key))


def test_unit_interval_and_gaussian_moments():
    r = np.array([0, 1, 2 ** 64 - 1], dtype=np.uint64)
    u = u64_to_unit(r)
    assert np.all(u > 0) and np.all(u <= 1)
    assert u[0] == 2.0 ** -54 and u[2] == 1.0     # the sum rounds up at the very top
    x = gaussian_fields(5, 2, np.arange(2000), 11, 64)
    assert abs(x.mean()) < 0.01 and abs(x.std() - 1) < 0.01
    # kurtosis of a normal is 3
    assert abs(np.mean(x ** 4) - 3) < 0.1


def test_fields_are_a_pure_function_of_the_counter():
    a = gaussian_fields(7, 3, [5, 9], 4, 37)
    b = gaussian_fields(7, 3, [9, 5], 4, 37)
    assert np.array_equal(a[0], b[1]) and np.array_equal(a[1], b[0])
    c = gaussian_fields(7, 3, [5], 4, 40)
    assert np.array_equal(a[0], c[0, :37])          # ragged tail of the last block
    assert not np.array_equal(gaussian_fields(7, 3, [5], 5, 37), a[:1])
    # Box-Muller on the raw stream, written out
    r = philox_u64(np.array([2, 5, 4, 0], dtype=np.uint64), np.array([7, 3], dtype=np.uint64))
    u = u64_to_unit(r)
    z2 = np.sqrt(-2 * np.log(u[2])) * np.cos(2 * np.pi * u[3])
    assert a[0, 10] == z2


def test_comb_uniform_stream():
    r = philox_u64(np.array([0, 0, 12, STREAM_COMB], dtype=np.uint64), np.array([3, 1], dtype=np.uint64))
    assert comb_uniform(3, 1, 12) == u64_to_unit(r[0])
