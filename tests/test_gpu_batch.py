"""Batches of uneven systems stepped by one graph launch per step (afqmc_batch_*): every system
must end exactly where stepping it alone with afqmc_step leaves it (same kernels, same field
stream), across the QR and comb phases, with walkers also stepped outside the batch."""

import numpy as np
import pytest

from synthetic import config_system, gen_system, noci_trial
from tests.parity_helpers import log

pytestmark = pytest.mark.gpu


def _systems():
    """(name, system kwargs builder, walkers, seed): uneven sizes, precisions and modes."""
    import paper_1711_02242_amd as afq
    tiny = config_system("tiny")
    s40 = gen_system(40, 10, 60, seed=41)
    s136 = gen_system(136, 34, 40, seed=42, n_dn=30)
    s24 = gen_system(24, 6, 36, seed=43)
    trial = noci_trial(tiny, 3, seed=44)
    return [
        ("tiny-fp64", lambda: afq.System.from_synthetic(tiny, dtau=0.01, precision="fp64"), 16, 5),
        ("m40-fp32", lambda: afq.System.from_synthetic(s40, dtau=0.005, precision="fp32"), 48, 6),
        ("m136-bf16x3-wide", lambda: afq.System.from_synthetic(s136, dtau=0.005,
                                                               precision="bf16x3"), 6, 7),
        ("m24-fp32-closed", lambda: afq.System.from_synthetic(s24, dtau=0.01, precision="fp32",
                                                              closed_shell=True), 32, 8),
        ("tiny-multidet-hybrid", lambda: afq.System.multidet(
            tiny.h0, tiny.h1, tiny.L, trial[0], np.array(trial[1]), np.array(trial[2]),
            dtau=0.01, precision="fp64", weight_mode="hybrid"), 12, 9),
    ]


def _state(wk):
    import torch
    torch.cuda.synchronize()
    return [t.cpu().numpy().copy() for t in (wk.U, wk.weight, wk.e_loc, wk.arg_ovlp,
                                             wk.walker_id)]


def _assert_same(a, b, what):
    for x, y, name in zip(a, b, ("U", "W", "E_L", "arg", "ids")):
        assert np.array_equal(x, y), f"{what}: {name} differs (max {np.abs(x - y).max()})"


def test_batch_equals_systems_stepped_alone():
    import paper_1711_02242_amd as afq
    steps = 12   # crosses two QR + comb phases (every 5 steps)
    specs = _systems()
    alone = []
    for name, make, nw, seed in specs:
        log(f"alone {name}")
        gs = make()
        wk = gs.walkers(nw)
        gs.init(wk)
        for _ in range(steps):
            gs.step(wk, seed=seed)
        alone.append(_state(wk))
        gs.close()
    log("batch")
    pairs = []
    for name, make, nw, seed in specs:
        gs = make()
        wk = gs.walkers(nw)
        gs.init(wk)
        pairs.append((gs, wk))
    b = afq.Batch(pairs)
    for _ in range(steps):
        b.step([sp[3] for sp in specs])
    for (gs, wk), ref, sp in zip(pairs, alone, specs):
        assert wk.step == steps
        _assert_same(_state(wk), ref, sp[0])
    b.close()


def test_autotuned_batch_equals_systems_alone_with_the_same_tiles():
    import paper_1711_02242_amd as afq
    steps = 6
    specs = _systems()
    pairs = []
    for name, make, nw, seed in specs:
        gs = make()
        wk = gs.walkers(nw)
        gs.init(wk)
        pairs.append((gs, wk))
    b = afq.Batch(pairs, autotune=True)
    log(f"tiles {b.tiles}")
    for _ in range(steps):
        b.step([sp[3] for sp in specs])
    for (name, make, nw, seed), tile, (gsb, wkb) in zip(specs, b.tiles, pairs):
        gs = make()
        gs.set_tile(tile)
        wk = gs.walkers(nw)
        gs.init(wk)
        for _ in range(steps):
            gs.step(wk, seed=seed)
        _assert_same(_state(wkb), _state(wk), name)
    b.close()


def test_batch_mixed_with_single_steps():
    """Steps taken outside the batch between batch steps keep the device step counter right."""
    import paper_1711_02242_amd as afq
    s = gen_system(32, 8, 48, seed=45)
    ref_gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    ref = ref_gs.walkers(24)
    ref_gs.init(ref)
    for _ in range(9):
        ref_gs.step(ref, seed=3)
    gs = afq.System.from_synthetic(s, dtau=0.005, precision="fp32")
    wk = gs.walkers(24)
    gs.init(wk)
    b = afq.Batch([(gs, wk)])
    b.step([3])
    b.step([3])
    gs.step(wk, seed=3)
    gs.step(wk, seed=3)
    for _ in range(5):
        b.step([3])
    _assert_same(_state(wk), _state(ref), "mixed")
    b.close()


def test_batch_reseed_recaptures():
    import paper_1711_02242_amd as afq
    s = config_system("tiny")
    gs = afq.System.from_synthetic(s, dtau=0.01, precision="fp64")
    wk = gs.walkers(16)
    gs.init(wk)
    b = afq.Batch([(gs, wk)])
    b.step([1])
    b.step([2])
    ref_gs = afq.System.from_synthetic(s, dtau=0.01, precision="fp64")
    ref = ref_gs.walkers(16)
    ref_gs.init(ref)
    ref_gs.step(ref, seed=1)
    ref_gs.step(ref, seed=2)
    _assert_same(_state(wk), _state(ref), "reseed")
    b.close()
