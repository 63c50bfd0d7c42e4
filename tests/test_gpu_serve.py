"""The serving loop on the GPU: a job's result is the same alone and in the mix (its own
system, walkers and field stream), admission respects the HBM budget, jobs retire at their
target standard error, and the footprint used for admission is the memory actually held."""

import math

import numpy as np
import pytest

from synthetic import gen_system
from tests.parity_helpers import log

pytestmark = pytest.mark.gpu


def _spec(job_id, M, nw, seed, **kw):
    from paper_1711_02242_amd.serve import JobSpec
    make = lambda: gen_system(M, M // 4, 6 * M, seed=seed)
    return JobSpec(job_id, make, M, M // 4, M // 4, 6 * M, nw, seed, **kw)


def _serve(specs, budget=64 << 30, check_every=20, autotune=False):
    from paper_1711_02242_amd.serve import Server
    srv = Server(budget, check_every=check_every, autotune=autotune)
    res = srv.run(specs, realtime=False)
    return srv, res


def test_alone_and_in_the_mix_agree():
    kw = dict(max_steps=60, discard=20, target_stderr=0.0)
    specs = [_spec(7, 16, 48, 101, **kw), _spec(8, 24, 32, 102, **kw), _spec(9, 40, 64, 103, **kw)]
    log("serve mix")
    srv, mix = _serve(specs)
    assert srv.max_resident == 3
    for sp, r in zip(specs, mix):
        log(f"alone {sp.job_id}")
        _, (alone,) = _serve([sp])
        assert r.steps == alone.steps == 60
        assert np.array_equal(r.energies, alone.energies), sp.job_id
        assert np.array_equal(r.weights, alone.weights)


def test_admission_respects_the_budget():
    from paper_1711_02242_amd.serve import footprint
    kw = dict(max_steps=40, discard=10, target_stderr=0.0)
    specs = [_spec(i, 32, 64, 200 + i, **kw) for i in range(3)]
    one = footprint(specs[0])
    log(f"budget for one job: {one} bytes")
    srv, res = _serve(specs, budget=int(one * 1.5))
    assert srv.max_resident == 1 and len(res) == 3
    assert all(r.steps == 40 for r in res)
    starts = sorted(r.t_start for r in res)
    dones = sorted(r.t_done for r in res)
    assert starts[1] >= dones[0] and starts[2] >= dones[1]


def test_jobs_retire_at_their_target():
    """A larger time step shortens the energy series' correlation in steps, so within the cap
    the blocked error reaches its plateau (growth below 10 % on doubling the block, App. C)
    below the target and the job retires before its cap."""
    from paper_1711_02242_amd.serve import blocked_error
    kw = dict(max_steps=20000, discard=300, target_stderr=0.05, dtau=0.05)
    srv, (r,) = _serve([_spec(3, 16, 256, 301, **kw)], check_every=200)
    log(f"retired after {r.steps} steps: {r.energy:.5f} +- {r.stderr:.5f}")
    x, w = r.energies[300:], r.weights[300:]
    log("  blocking: " + ", ".join(f"L={b}: {blocked_error(x, w, b)[2]:.5f}"
                                   for b in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512)
                                   if len(x) // b >= 16))
    assert r.plateau and r.stderr < 0.05 and r.steps < 20000 and math.isfinite(r.energy)


@pytest.mark.parametrize("M,nw,precision", [(24, 100, "fp32"), (64, 300, "bf16x3"),
                                             (136, 40, "fp32"), (40, 20, "fp64"),
                                             (150, 10, "fp64")])
def test_footprint_is_the_memory_held(M, nw, precision):
    import paper_1711_02242_amd as afq
    from paper_1711_02242_amd.serve import footprint
    sp = _spec(0, M, nw, 5, precision=precision)
    s = sp.make_system()
    gs = afq.System.from_synthetic(s, dtau=0.005, precision=precision)
    wk = gs.walkers(nw)
    held = gs.device_bytes + wk.workspace.numel() + 256 + sum(
        t.numel() * t.element_size() for t in (wk.U, wk.weight, wk.arg_ovlp, wk.log_ovlp,
                                               wk.e_loc, wk.phase, wk.walker_id))
    assert footprint(sp) == held
    gs.close()
