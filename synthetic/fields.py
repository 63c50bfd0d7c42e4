"""Counter-based random stream for the auxiliary fields and population control.

The paper draws x_g ~ N(0, 1) independently for every walker, field and step
(Sec. II.B.1, eq:hs2) and leaves the generator open.  Here the stream is
Philox4x64-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written out below from that published definition and
checked bit for bit against ``numpy.random.Philox``.  A counter-based stream
lets any walker, step and field be generated independently and in any order,
so that a run on another device, in another batch, or resumed from a
checkpoint sees the same numbers.

Conventions (shared with the HIP library's own generator):

* key     = (seed, job_id)
* counter = (block, walker_id, step, stream)   -- 4 x uint64
* stream STREAM_FIELDS (0): block c yields fields x[4c .. 4c+3];
  stream STREAM_COMB (1): block 0, walker 0 yields the comb's uniform.
* uint64 r -> u = ((r >> 11) + 0.5) * 2**-53, in (0, 1] (1 only for the top 2^11 values of r, where the sum rounds up; u > 0 keeps log u finite).
* Box-Muller on (u0, u1) and (u2, u3):
  z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1), same for z2, z3.
"""

from __future__ import annotations

import numpy as np

STREAM_FIELDS = 0
STREAM_COMB = 1

_MASK32 = np.uint64(0xFFFFFFFF)
_SH32 = np.uint64(32)
# Round multipliers and Weyl key increments of Philox4x64 (SC'11, Table 2 / Sec. 4).
_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)
_W1 = np.uint64(0xBB67AE8584CAA73B)


def _mulhilo(a: np.ndarray, b: np.uint64):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a_lo = a & _MASK32
    a_hi = a >> _SH32
    b_lo = b & _MASK32
    b_hi = b >> _SH32
    p0 = a_lo * b_lo
    p1 = a_lo * b_hi
    p2 = a_hi * b_lo
    p3 = a_hi * b_hi
    mid = (p0 >> _SH32) + (p1 & _MASK32) + (p2 & _MASK32)
    hi = p3 + (p1 >> _SH32) + (p2 >> _SH32) + (mid >> _SH32)
    lo = a * b
    return hi, lo


def philox_u64(ctr, key, rounds: int = 10) -> np.ndarray:
    """Philox4x64-R of counters ``ctr`` (..., 4) under keys ``key`` (..., 2); uint64 out (..., 4)."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    shape = np.broadcast_shapes(ctr.shape[:-1], key.shape[:-1])
    x0, x1, x2, x3 = (np.broadcast_to(ctr[..., i], shape).copy() for i in range(4))
    k0 = np.broadcast_to(key[..., 0], shape).copy()
    k1 = np.broadcast_to(key[..., 1], shape).copy()
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(x0, _M0)
            hi1, lo1 = _mulhilo(x2, _M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def u64_to_unit(r: np.ndarray) -> np.ndarray:
    """uint64 -> double in (0, 1]: ((r >> 11) + 0.5) * 2^-53 (rounds to 1 only at the top of the range)."""
    r = np.asarray(r, dtype=np.uint64)
    return ((r >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def gaussian_fields(seed: int, job_id: int, walker_ids, step: int, n_chol: int) -> np.ndarray:
    """Auxiliary fields x[w, g] ~ N(0,1) for the given walkers at one step, shape (n_w, n_chol)."""
    walker_ids = np.asarray(walker_ids, dtype=np.uint64).reshape(-1)
    n_blocks = (n_chol + 3) // 4
    nw = walker_ids.size
    ctr = np.zeros((nw, n_blocks, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(n_blocks, dtype=np.uint64)[None, :]
    ctr[..., 1] = walker_ids[:, None]
    ctr[..., 2] = np.uint64(step)
    ctr[..., 3] = np.uint64(STREAM_FIELDS)
    key = np.array([seed, job_id], dtype=np.uint64)
    r = philox_u64(ctr, key)
    u = u64_to_unit(r)
    rad0 = np.sqrt(-2.0 * np.log(u[..., 0]))
    rad1 = np.sqrt(-2.0 * np.log(u[..., 2]))
    z = np.empty((nw, n_blocks, 4))
    z[..., 0] = rad0 * np.cos(2.0 * np.pi * u[..., 1])
    z[..., 1] = rad0 * np.sin(2.0 * np.pi * u[..., 1])
    z[..., 2] = rad1 * np.cos(2.0 * np.pi * u[..., 3])
    z[..., 3] = rad1 * np.sin(2.0 * np.pi * u[..., 3])
    return z.reshape(nw, 4 * n_blocks)[:, :n_chol].copy()


def comb_uniform(seed: int, job_id: int, step: int) -> float:
    """The single uniform in (0, 1] used by the population-control comb after ``step``."""
    ctr = np.array([0, 0, step, STREAM_COMB], dtype=np.uint64)
    key = np.array([seed, job_id], dtype=np.uint64)
    return float(u64_to_unit(philox_u64(ctr, key)[0]))
