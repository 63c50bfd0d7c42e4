"""Serving loop: continuous batching of AFQMC jobs on one GPU.

Jobs arrive over time.  Each job is admitted when its HBM footprint (``afqmc_footprint_bytes``:
the library's tables plus its walkers and workspace) fits the memory budget next to the jobs
already resident and a slot is free.  Admitted jobs are prepared (Hamiltonian set up, walkers
initialized, contraction tile autotuned) on a worker thread while the resident jobs keep
stepping.  Every tick advances all resident jobs by one step with one graph launch
(``Batch``); each job's mixed-estimator sums (eq:localenergy) go into a device ring buffer
(``afqmc_energy_enqueue``) that is read back every ``check_every`` ticks.  A job is retired,
and its memory freed, once the reblocked standard error of its energy (App. C) is below its
target or it reaches its step cap; its time-to-energy runs from arrival to retirement.

Jobs never share state: every job has its own system, walkers and field stream keyed by
(seed, job id), so its results do not depend on which other jobs share the GPU.
"""

from __future__ import annotations

import ctypes as C
import math
import threading
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import _lib as L
from .afqmc import Batch, System


# ---------------------------------------------------------------------------- reblocking
def blocked_error(x, w, block: int):
    """Weighted blocking (App. C) of per-step estimates x with weights w, block length ``block``:
    block weights W_b = sum of w, block means m_b = sum w x / W_b; returns (mean, S, stderr, n_b)
    with the unbiased weighted spread S of the m_b and stderr = S / sqrt(n_b - 1)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    nb = len(x) // block
    if nb < 2:
        raise ValueError("blocked_error: fewer than two blocks")
    Wb = np.add.reduceat(w[: nb * block], np.arange(0, nb * block, block))
    mb = np.add.reduceat((w * x)[: nb * block], np.arange(0, nb * block, block)) / Wb
    V1 = float(np.sum(Wb))
    V2 = float(np.sum(Wb ** 2))
    mean = float(np.sum(Wb * mb) / V1)
    spread = math.sqrt(float(np.sum(Wb * (mb - mean) ** 2)) / (V1 - V2 / V1))
    return mean, spread, spread / math.sqrt(nb - 1), nb


def energy_estimate(x, w, discard: int, min_blocks: int = 16, ratio: float = 1.1):
    """Equilibration samples dropped, the block length doubles until the standard error grows by
    less than ``ratio`` (plateau).  Returns (mean, stderr, block, plateau_reached)."""
    x = np.asarray(x, dtype=np.float64)[discard:]
    w = np.asarray(w, dtype=np.float64)[discard:]
    if len(x) < 2:
        return (float(np.average(x, weights=w)) if len(x) else math.nan), math.inf, 1, False
    block, last = 1, None
    while len(x) // block >= min_blocks:
        mean, _, err, _ = blocked_error(x, w, block)
        if last is not None and err <= ratio * last[1]:
            return mean, err, block, True
        last = (mean, err, block)
        block *= 2
    if last is None:
        mean, _, err, _ = blocked_error(x, w, 1)
        return mean, err, 1, False
    return last[0], last[1], last[2], False


# ---------------------------------------------------------------------------- jobs
@dataclass
class JobSpec:
    """One AFQMC calculation.  ``make_system`` returns the Hamiltonian and trial (an object with
    h0, h1, L, phi_up, phi_dn, M, n_up, n_dn, n_chol); it runs on the worker at admission."""
    job_id: int
    make_system: object
    M: int
    n_up: int
    n_dn: int
    n_chol: int
    n_walkers: int
    seed: int
    precision: str = "fp32"
    dtau: float = 0.005
    target_stderr: float = 1e-3
    max_steps: int = 20000
    discard: int = 200
    arrival: float = 0.0      # seconds after the server starts (trace replay)


@dataclass
class JobResult:
    job_id: int
    energy: float
    stderr: float
    plateau: bool
    steps: int
    t_arrival: float
    t_admit: float
    t_start: float
    t_done: float
    footprint: int
    energies: np.ndarray = field(repr=False, default=None)
    weights: np.ndarray = field(repr=False, default=None)

    @property
    def time_to_energy(self) -> float:
        return self.t_done - self.t_arrival


def footprint(spec: JobSpec) -> int:
    """Device bytes of the job when resident (library tables + walkers + workspace)."""
    lib = L.load()
    p = L.Params(M=spec.M, n_up=spec.n_up, n_dn=spec.n_dn, n_chol=spec.n_chol, dtau=spec.dtau,
                 e_trial=math.nan, n_taylor=6, qr_period=5, pop_period=5,
                 precision=L.PRECISIONS[spec.precision], el_cap_C=2.0, w_max=math.nan, fb_cap=1.0,
                 flags=0, n_growth=0, theta_guard=math.nan)
    sb, wb = C.c_size_t(), C.c_size_t()
    L.check(lib.afqmc_footprint_bytes(C.byref(p), 1, int(spec.n_walkers), C.byref(sb),
                                      C.byref(wb)), "afqmc_footprint_bytes")
    return int(sb.value + wb.value)


class _Run:
    """A resident job: its system, walkers and device ring of per-step estimator sums."""

    def __init__(self, spec: JobSpec, ring: int, autotune: bool):
        import torch
        s = spec.make_system()
        self.spec = spec
        self.gs = System.from_synthetic(s, dtau=spec.dtau, precision=spec.precision)
        self.wk = self.gs.walkers(spec.n_walkers)
        self.gs.init(self.wk)
        if autotune:
            self.gs.autotune(self.wk, reuse=True)
            self.gs.measure(self.wk)
        self.ring = torch.zeros((ring, 6), dtype=torch.float64, device="cuda")
        self.slot = 0
        self.x: list = []
        self.w: list = []
        torch.cuda.current_stream().synchronize()

    def record(self) -> None:
        L.check(self.gs.lib.afqmc_energy_enqueue(
            self.gs.handle, self.wk.c_ref(), C.c_void_p(int(self.ring[self.slot].data_ptr()))),
            "afqmc_energy_enqueue")
        self.slot += 1

    def drain(self) -> None:
        if self.slot == 0:
            return
        h = self.ring[: self.slot].cpu().numpy()
        self.x.extend((h[:, 0] / h[:, 2]).tolist())
        self.w.extend(h[:, 2].tolist())
        self.slot = 0

    def close(self) -> None:
        self.gs.close()


class Server:
    """Continuous batching under an HBM budget (bytes) and a slot limit."""

    def __init__(self, hbm_budget: int, max_active: int = 64, check_every: int = 50,
                 autotune: bool = True, workers: int = 1):
        self.budget = int(hbm_budget)
        self.max_active = int(max_active)
        self.check_every = int(check_every)
        self.autotune = autotune
        self.pool = ThreadPoolExecutor(max_workers=max(1, workers))
        self.waiting: deque = deque()
        self.preparing: list = []     # (spec, future, t_admit, bytes)
        self.active: list = []        # (_Run, t_arrival, t_admit, t_start, bytes)
        self.results: list = []
        self.used = 0
        self.batch = None
        self.members = None
        self.ticks = 0
        self.max_resident = 0
        self.walker_steps = 0
        self.t0 = time.perf_counter()
        self._lock = threading.Lock()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, spec: JobSpec, t_arrival: float | None = None) -> None:
        fp = footprint(spec)
        if fp > self.budget:
            raise ValueError(f"job {spec.job_id} needs {fp} bytes, above the budget {self.budget}")
        self.waiting.append((spec, self.now() if t_arrival is None else t_arrival, fp))

    # ------------------------------------------------------------------ scheduling
    def _admit(self) -> None:
        while self.waiting:
            spec, t_arr, fp = self.waiting[0]
            n_res = len(self.active) + len(self.preparing)
            if n_res >= self.max_active or self.used + fp > self.budget:
                break
            self.waiting.popleft()
            self.used += fp
            fut = self.pool.submit(_Run, spec, self.check_every, self.autotune)
            self.preparing.append((spec, fut, t_arr, self.now(), fp))

    def _join_prepared(self, wait: bool = False) -> None:
        keep = []
        for spec, fut, t_arr, t_adm, fp in self.preparing:
            if fut.done() or wait:
                run = fut.result()
                self.active.append((run, t_arr, t_adm, self.now(), fp))
            else:
                keep.append((spec, fut, t_arr, t_adm, fp))
        self.preparing = keep

    def _batch(self):
        members = [id(r[0]) for r in self.active]
        if members != self.members:
            if self.batch is not None:
                self.batch.close()
            self.batch = Batch([(r[0].gs, r[0].wk) for r in self.active]) if self.active else None
            self.members = members
        return self.batch

    def _check(self) -> None:
        import torch
        torch.cuda.synchronize()
        keep = []
        for run, t_arr, t_adm, t_start, fp in self.active:
            run.drain()
            spec = run.spec
            n = run.wk.step
            mean, err, _, plateau = energy_estimate(run.x, run.w, spec.discard)
            if (plateau and err < spec.target_stderr) or n >= spec.max_steps:
                self.results.append(JobResult(
                    spec.job_id, mean, err, plateau, n, t_arr, t_adm, t_start, self.now(), fp,
                    np.array(run.x), np.array(run.w)))
                run.close()
                self.used -= fp
            else:
                keep.append((run, t_arr, t_adm, t_start, fp))
        self.active = keep

    def tick(self) -> bool:
        """Admit what fits, step every resident job once; returns False when idle."""
        self._admit()
        self._join_prepared(wait=not self.active and bool(self.preparing))
        self.max_resident = max(self.max_resident, len(self.active))
        if not self.active:
            return False
        b = self._batch()
        b.step([r[0].spec.seed for r in self.active], [r[0].spec.job_id for r in self.active])
        for r in self.active:
            r[0].record()
            self.walker_steps += r[0].spec.n_walkers
        self.ticks += 1
        if any(r[0].slot >= self.check_every for r in self.active) or any(
                r[0].wk.step >= r[0].spec.max_steps for r in self.active):
            self._check()
        return True

    def run(self, specs, realtime: bool = True) -> list:
        """Replay arrivals (``spec.arrival`` seconds after start when ``realtime``, else all at
        once in order) and serve until every job is retired."""
        pending = deque(sorted(specs, key=lambda s: s.arrival))
        self.t0 = time.perf_counter()
        while pending or self.waiting or self.preparing or self.active:
            while pending and (not realtime or pending[0].arrival <= self.now()):
                sp = pending.popleft()
                self.submit(sp, sp.arrival if realtime else self.now())
            if not self.tick() and pending and realtime and not self.preparing:
                time.sleep(max(0.0, min(0.05, pending[0].arrival - self.now())))
        self.close()
        return sorted(self.results, key=lambda r: r.job_id)

    def close(self) -> None:
        if self.batch is not None:
            self.batch.close()
            self.batch = None
        for run, *_ in self.active:
            run.close()
        self.active = []
        self.pool.shutdown(wait=True)
