"""The C-ABI library loads and exports every symbol include/afqmc.h declares, and the
ctypes structures match the C layout (no GPU needed, no compute calls)."""

import ctypes as C
import os
import re
import subprocess
import sys

import pytest

import paper_1711_02242_amd as pkg
from paper_1711_02242_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "afqmc.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"AFQMC_API\s+(?:const\s+)?\w+\*?\s+(afqmc_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(L.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = pkg.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(afqmc_\w+)", out))
    assert exported == set(declared_functions())


def test_error_strings():
    lib = pkg.load()
    assert lib.afqmc_error_string(0) == b"ok"
    assert b"argument" in lib.afqmc_error_string(-1)
    assert lib.afqmc_error_string(12345) == b"unknown error"


def test_null_arguments_are_rejected_without_device_work():
    lib = pkg.load()
    assert lib.afqmc_setup(None, 0.0, None, None, None, None, None, None) == -1
    assert lib.afqmc_destroy(None) == -1
    b = C.c_size_t()
    assert lib.afqmc_workspace_bytes(None, 4, C.byref(b)) == -1


def test_batch_argument_checks_precede_device_work():
    lib = pkg.load()
    out = C.c_void_p()
    assert lib.afqmc_batch_create(0, None, None, None, C.byref(out)) == -1
    assert lib.afqmc_batch_create(2, None, None, None, C.byref(out)) == -1
    assert lib.afqmc_batch_step(None, None) == -1
    assert lib.afqmc_batch_destroy(None) == -1


def test_multidet_argument_checks_precede_device_work():
    """n_det outside 1..1024, a missing or non-finite coefficient array are argument errors."""
    import numpy as np
    lib = pkg.load()
    M, n = 4, 1
    p = pkg._lib.Params(M=M, n_up=n, n_dn=n, n_chol=0, dtau=0.01, e_trial=float("nan"),
                        n_taylor=6, qr_period=5, pop_period=5, precision=0, el_cap_C=2.0,
                        w_max=float("nan"), fb_cap=1.0, flags=0, n_growth=0,
                        theta_guard=float("nan"))
    h1 = np.eye(M)
    phi = np.zeros((2, M, n))
    phi[:, 0, 0] = 1.0
    out = C.c_void_p()
    ok_coef = np.array([1.0, 0.0, 0.5, 0.0])
    bad_coef = np.array([1.0, 0.0, np.nan, 0.0])
    args = lambda nd, cf: (C.byref(p), 0.0, h1.ctypes.data, None, nd, cf, phi.ctypes.data,
                           phi.ctypes.data, None, C.byref(out))
    assert lib.afqmc_setup_multidet(*args(2, None)) == -1
    assert lib.afqmc_setup_multidet(*args(0, ok_coef.ctypes.data)) == -1
    assert lib.afqmc_setup_multidet(*args(1025, ok_coef.ctypes.data)) == -1
    assert lib.afqmc_setup_multidet(*args(2, bad_coef.ctypes.data)) == -1
    assert out.value is None


def test_struct_layout_matches_c(tmp_path):
    src = tmp_path / "probe.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "afqmc.h"
#define P(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
  printf("afqmc_params %zu\n", sizeof(afqmc_params));
  printf("afqmc_walkers %zu\n", sizeof(afqmc_walkers));
  printf("afqmc_fields %zu\n", sizeof(afqmc_fields));
  printf("afqmc_info %zu\n", sizeof(afqmc_info));
  P(afqmc_params, dtau) P(afqmc_params, precision) P(afqmc_params, el_cap_C) P(afqmc_params, flags)
  P(afqmc_walkers, U) P(afqmc_walkers, workspace) P(afqmc_walkers, workspace_bytes) P(afqmc_walkers, step)
  P(afqmc_fields, x) P(afqmc_fields, u_comb)
  return 0;
}
""")
    exe = tmp_path / "probe"
    r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                        str(exe)], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(r.stderr)
    vals = dict(line.rsplit(" ", 1) for line in
                subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
                if line)
    assert int(vals["afqmc_params"]) == C.sizeof(L.Params)
    assert int(vals["afqmc_walkers"]) == C.sizeof(L.WalkersC)
    assert int(vals["afqmc_fields"]) == C.sizeof(L.FieldsC)
    assert int(vals["afqmc_info"]) == C.sizeof(L.InfoC)
    for key, struct in (("afqmc_params", L.Params), ("afqmc_walkers", L.WalkersC),
                        ("afqmc_fields", L.FieldsC)):
        for k, v in vals.items():
            if k.startswith(key + "."):
                field = k.split(".", 1)[1]
                assert getattr(struct, field).offset == int(v), k


def test_header_constants_match_binding():
    text = open(HEADER).read()
    tiles = {m.group(1).lower(): int(m.group(2))
             for m in re.finditer(r"#define AFQMC_TILE_(\w+) (\d+)", text)}
    assert tiles == L.TILES
    assert int(re.search(r"#define AFQMC_MFMA_PEAK_BYTES (\d+)", text).group(1)) == \
        L.MFMA_PEAK_BYTES


def test_mfma_peak_argument_checks_precede_device_work():
    lib = pkg.load()
    t = C.c_double()
    assert lib.afqmc_mfma_peak(1, None, L.MFMA_PEAK_BYTES, None, C.byref(t)) == -1
    assert lib.afqmc_mfma_peak(1, C.c_void_p(256), L.MFMA_PEAK_BYTES - 8, None, C.byref(t)) == -1
    assert lib.afqmc_mfma_peak(1, C.c_void_p(256), L.MFMA_PEAK_BYTES, None, None) == -1
    # an unknown precision is refused before anything touches the (fake) device pointer
    unsupported = int(re.search(r"AFQMC_E_UNSUPPORTED = (-\d+)", open(HEADER).read()).group(1))
    assert lib.afqmc_mfma_peak(7, C.c_void_p(256), L.MFMA_PEAK_BYTES, None,
                               C.byref(t)) == unsupported


def test_library_binds_to_a_single_hip_runtime():
    """Loading the library first (torch not yet imported) still maps one HIP runtime: torch
    carries its own copy, and a second one would make torch's streams foreign to the library."""
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1711_02242_amd import _lib as L\n"
            "L.load()\n"
            "import torch\n"
            "maps = open('/proc/self/maps').read().splitlines()\n"
            "print(len({l.split()[-1] for l in maps if 'libamdhip64' in l}))\n") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "1"
