"""Seeded multi-system workloads: the uneven batch and the serving trace.

Both draw molecule-shaped systems of ``gen_system`` with N = floor(M / 4) electrons per
spin and N_g = 6M Cholesky vectors; walker counts are log-uniform.

* ``batch_workload``: n systems (24 by default), M uniform on {24, ..., 160}, walkers
  round(exp(U(ln 128, ln 2048))), all drawn from ``default_rng(seed)`` in that order, per
  system; system i's Hamiltonian seed is seed + i.
* ``serving_trace``: n jobs (32 by default) arriving as a Poisson process of the given rate
  (exponential gaps), M uniform on {32, ..., 200}, walkers log-uniform on [256, 2048];
  job i's Hamiltonian seed and job id are seed + i.

Input generation only.
"""

from __future__ import annotations

import numpy as np


def _log_uniform_int(rng, lo: int, hi: int) -> int:
    return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))


def batch_workload(n: int = 24, seed: int = 4000, m_lo: int = 24, m_hi: int = 160,
                   w_lo: int = 128, w_hi: int = 2048):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        M = int(rng.integers(m_lo, m_hi + 1))
        nw = _log_uniform_int(rng, w_lo, w_hi)
        out.append(dict(M=M, N=M // 4, n_chol=6 * M, n_walkers=nw, seed=seed + i))
    return out


def serving_trace(n: int = 32, rate: float = 4.0, seed: int = 5000, m_lo: int = 32,
                  m_hi: int = 200, w_lo: int = 256, w_hi: int = 2048):
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        M = int(rng.integers(m_lo, m_hi + 1))
        nw = _log_uniform_int(rng, w_lo, w_hi)
        out.append(dict(arrival=t, M=M, N=M // 4, n_chol=6 * M, n_walkers=nw, seed=seed + i,
                        job_id=seed + i))
    return out
