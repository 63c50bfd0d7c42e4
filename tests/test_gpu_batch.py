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


def _family_systems():
    """Systems whose contractions share kernel instances (three register-resident FP32 systems
    with K_P = 64, two wide BF16x3 systems with N_P = 48 and K_P = 160, two systems on the
    flat variant), mixed with systems that stay outside any family (FP64, multi-determinant)."""
    import paper_1711_02242_amd as afq
    tiny = config_system("tiny")
    trial = noci_trial(tiny, 3, seed=44)
    sys_ = {
        "m40a": gen_system(40, 10, 60, seed=51), "m40b": gen_system(40, 10, 60, seed=52),
        "m36": gen_system(36, 9, 50, seed=53), "m136": gen_system(136, 34, 40, seed=54, n_dn=30),
        "m140": gen_system(140, 34, 36, seed=55), "m50": gen_system(50, 12, 40, seed=56),
        "m52": gen_system(52, 12, 40, seed=57),
    }

    def mk(name, prec, tile=None, **kw):
        def make():
            gs = afq.System.from_synthetic(sys_[name], dtau=0.005, precision=prec, **kw)
            if tile:
                gs.set_tile(tile)
            return gs
        return make
    return [
        ("m40a-fp32", mk("m40a", "fp32"), 48, 11, None),
        ("tiny-fp64", lambda: afq.System.from_synthetic(tiny, dtau=0.01, precision="fp64"), 16,
         12, None),
        ("m40b-fp32", mk("m40b", "fp32"), 32, 13, None),
        ("m136-bf16x3", mk("m136", "bf16x3"), 6, 14, None),
        ("m36-fp32", mk("m36", "fp32"), 20, 15, None),
        ("m140-bf16x3", mk("m140", "bf16x3"), 5, 16, None),
        ("m50-flat", mk("m50", "fp32", "flat"), 9, 17, "flat"),
        ("tiny-multidet", lambda: afq.System.multidet(
            tiny.h0, tiny.h1, tiny.L, trial[0], np.array(trial[1]), np.array(trial[2]),
            dtau=0.01, precision="fp32"), 12, 18, None),
        ("m52-flat", mk("m52", "fp32", "flat"), 7, 19, "flat"),
    ]


@pytest.mark.skip(reason="family launches are switched off: the first GPU run of this test "
                  "crashed the host process (segmentation fault) inside the batch step that "
                  "captured the family graph, with no cause found in the library")
def test_family_launches_equal_systems_stepped_alone():
    """One contraction launch per family of systems (mode 1), switched on and off between
    steps: every system ends bitwise where stepping it alone leaves it."""
    import paper_1711_02242_amd as afq
    specs = _family_systems()
    steps = 12
    alone = []
    for name, make, nw, seed, _ in specs:
        gs = make()
        wk = gs.walkers(nw)
        gs.init(wk)
        for _ in range(steps):
            gs.step(wk, seed=seed)
        alone.append(_state(wk))
        gs.close()
    pairs = []
    for name, make, nw, seed, _ in specs:
        gs = make()
        wk = gs.walkers(nw)
        gs.init(wk)
        pairs.append((gs, wk))
    b = afq.Batch(pairs, families=True)
    seeds = [sp[3] for sp in specs]
    for k in range(steps):
        if k == 7:
            b.set_families(False)
        if k == 9:
            b.set_families(True)
        b.step(seeds)
    for (gs, wk), ref, sp in zip(pairs, alone, specs):
        assert wk.step == steps
        _assert_same(_state(wk), ref, sp[0])
    b.close()


def test_family_mode_is_refused():
    """Mode 1 of afqmc_batch_set_mode is not available (AFQMC_E_UNSUPPORTED); mode 0 is the
    batch's only mode, and the batch still steps after the refusal."""
    import paper_1711_02242_amd as afq
    s = config_system("tiny")
    gs = afq.System.from_synthetic(s, dtau=0.01, precision="fp32")
    wk = gs.walkers(8)
    gs.init(wk)
    b = afq.Batch([(gs, wk)])
    b.set_families(False)
    with pytest.raises(afq.AfqmcError, match="-2"):
        b.set_families(True)
    b.step([3])
    assert wk.step == 1
    b.close()
