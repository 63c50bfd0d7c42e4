"""Python binding of the HIP AFQMC library: argument marshalling only.

Every step of the path runs in the library's kernels.  PyTorch supplies device
memory (walker arrays and workspace as CUDA/ROCm tensors) and the stream.
"""

from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


class System:
    """A Hamiltonian in Cholesky form plus a trial, resident on the GPU.

    h1 (M, M), L (n_chol, M, M), phi_up (M, n_up), phi_dn (M, n_dn): real float64 host arrays.
    With ``coeffs`` (n_det complex A_d) the trial is sum_d A_d |Psi_d> and phi_up / phi_dn are
    (n_det, M, n_up) / (n_det, M, n_dn), the leading determinant first (``System.multidet``).
    """

    def __init__(self, h0, h1, L_chol, phi_up, phi_dn, *, dtau: float, precision: str = "fp64",
                 n_taylor: int = 6, qr_period: int = 5, pop_period: int = 5, el_cap_C: float = 2.0,
                 w_max: float | None = None, fb_cap: float = 1.0, e_trial: float | None = None,
                 weight_mode: str = "phaseless", mean_field: bool = False,
                 closed_shell: bool = False, coeffs=None, n_growth: int = 200,
                 theta_guard: float | None = None, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise L.AfqmcError("no GPU visible: the AFQMC library runs on the GPU only")
        self.lib = L.load()
        h1 = np.ascontiguousarray(h1, dtype=np.float64)
        M = h1.shape[0]
        L_chol = np.ascontiguousarray(L_chol, dtype=np.float64).reshape(-1, M, M)
        if coeffs is None:
            self.n_det = 1
            phi_up = np.ascontiguousarray(phi_up, dtype=np.float64).reshape(M, -1)
            phi_dn = np.ascontiguousarray(phi_dn, dtype=np.float64).reshape(M, -1)
            n_up, n_dn = phi_up.shape[1], phi_dn.shape[1]
        else:
            cf = np.asarray(coeffs, dtype=np.complex128).reshape(-1)
            self.n_det = cf.size
            phi_up = np.ascontiguousarray(phi_up, dtype=np.float64).reshape(self.n_det, M, -1)
            phi_dn = np.ascontiguousarray(phi_dn, dtype=np.float64).reshape(self.n_det, M, -1)
            n_up, n_dn = phi_up.shape[2], phi_dn.shape[2]
            cpair = np.ascontiguousarray(np.stack([cf.real, cf.imag], axis=1))
        self.M, self.n_up, self.n_dn, self.n_chol = M, n_up, n_dn, L_chol.shape[0]
        self.closed_shell = bool(closed_shell)
        self.ntot = self.n_up if self.closed_shell else self.n_up + self.n_dn
        self.dtau = float(dtau)
        self.precision = precision
        p = L.Params(M=M, n_up=self.n_up, n_dn=self.n_dn, n_chol=self.n_chol, dtau=self.dtau,
                     e_trial=math.nan if e_trial is None else float(e_trial), n_taylor=n_taylor,
                     qr_period=qr_period, pop_period=pop_period,
                     precision=L.PRECISIONS[precision], el_cap_C=el_cap_C,
                     w_max=math.nan if w_max is None else float(w_max), fb_cap=fb_cap,
                     flags=L.WEIGHT_MODES[weight_mode]
                     | (L.FLAG_MEAN_FIELD if mean_field else 0)
                     | (L.FLAG_CLOSED_SHELL if closed_shell else 0), n_growth=int(n_growth),
                     theta_guard=math.nan if theta_guard is None else float(theta_guard))
        self.weight_mode = weight_mode
        self.params = p
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handle = C.c_void_p()
        if coeffs is None:
            rc = self.lib.afqmc_setup(C.byref(p), float(h0), h1.ctypes.data, L_chol.ctypes.data,
                                      phi_up.ctypes.data, phi_dn.ctypes.data,
                                      C.c_void_p(_stream_handle(self.stream)), C.byref(handle))
            L.check(rc, "afqmc_setup")
        else:
            rc = self.lib.afqmc_setup_multidet(C.byref(p), float(h0), h1.ctypes.data,
                                               L_chol.ctypes.data, self.n_det, cpair.ctypes.data,
                                               phi_up.ctypes.data, phi_dn.ctypes.data,
                                               C.c_void_p(_stream_handle(self.stream)),
                                               C.byref(handle))
            L.check(rc, "afqmc_setup_multidet")
        self.handle = handle
        info = L.InfoC()
        L.check(self.lib.afqmc_get_info(self.handle, C.byref(info)), "afqmc_get_info")
        self.e_trial = info.e_trial
        self.e_hf = info.e_hf
        self.device_bytes = info.device_bytes

    @classmethod
    def from_synthetic(cls, s, **kw):
        return cls(s.h0, s.h1, s.L, s.phi_up, s.phi_dn, **kw)

    @classmethod
    def multidet(cls, h0, h1, L_chol, coeffs, phis_up, phis_dn, **kw):
        """Trial sum_d coeffs[d] |Psi_d> with determinant d = (phis_up[d], phis_dn[d])."""
        return cls(h0, h1, L_chol, phis_up, phis_dn, coeffs=coeffs, **kw)

    def close(self):
        if getattr(self, "handle", None):
            L.check(self.lib.afqmc_destroy(self.handle), "afqmc_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- walkers
    def workspace_bytes(self, n_walkers: int) -> int:
        b = C.c_size_t()
        L.check(self.lib.afqmc_workspace_bytes(self.handle, int(n_walkers), C.byref(b)),
                "afqmc_workspace_bytes")
        return int(b.value)

    def walkers(self, n_walkers: int) -> "Walkers":
        return Walkers(self, n_walkers)

    def init(self, wk: "Walkers") -> None:
        L.check(self.lib.afqmc_walkers_init(self.handle, wk.c_ref()), "afqmc_walkers_init")
        wk.sync_from_c()

    def measure(self, wk: "Walkers") -> None:
        L.check(self.lib.afqmc_measure(self.handle, wk.c_ref()), "afqmc_measure")

    def _fields(self, seed, job_id, x, u_comb):
        xp = None
        if x is not None:
            xp = C.c_void_p(int(x.data_ptr()))
        return L.FieldsC(seed=int(seed), job_id=int(job_id), x=xp,
                         u_comb=math.nan if u_comb is None else float(u_comb))

    def step(self, wk: "Walkers", seed: int = 0, job_id: int = 0, x=None, u_comb=None) -> None:
        """One step of the random walk.  ``x``: optional device tensor (n_walkers, n_chol) float64."""
        if x is not None:
            torch = _torch()
            assert x.dtype == torch.float64 and x.is_cuda and x.is_contiguous()
            assert tuple(x.shape) == (wk.n, self.n_chol)
        f = self._fields(seed, job_id, x, u_comb)
        L.check(self.lib.afqmc_step(self.handle, wk.c_ref(), C.byref(f)), "afqmc_step")
        wk.sync_from_c()

    def fields_draw(self, wk: "Walkers", seed: int = 0, job_id: int = 0):
        torch = _torch()
        out = torch.empty((wk.n, self.n_chol), dtype=torch.float64, device="cuda")
        f = self._fields(seed, job_id, None, None)
        L.check(self.lib.afqmc_fields_draw(self.handle, wk.c_ref(), C.byref(f),
                                           C.c_void_p(int(out.data_ptr()))), "afqmc_fields_draw")
        return out

    def energy(self, wk: "Walkers", check: bool = True):
        """(Re sum c E, Im sum c E, Re sum c, n_alive, status) with c = W e^{i theta}
        -- synchronizes the stream.  ``energy_sums`` also returns Im sum c."""
        o = self.energy_sums(wk, check)
        return o[0], o[1], o[2], int(o[3]), int(o[4])

    def energy_sums(self, wk: "Walkers", check: bool = True):
        out = (C.c_double * 6)()
        rc = self.lib.afqmc_energy(self.handle, wk.c_ref(), out)
        if check:
            L.check(rc, "afqmc_energy")
        return tuple(out)

    def free_projection_energy(self, wk: "Walkers") -> complex:
        o = self.energy_sums(wk)
        return complex(o[0], o[1]) / complex(o[2], o[5])

    def mixed_energy(self, wk: "Walkers") -> float:
        a, _, c, _, _ = self.energy(wk)
        return a / c

    def growth(self, wk: "Walkers"):
        """(E_T, cap centre) of the population (``afqmc_get_growth``; synchronizes)."""
        out = (C.c_double * 2)()
        L.check(self.lib.afqmc_get_growth(self.handle, wk.c_ref(), out), "afqmc_get_growth")
        return out[0], out[1]

    def bound_counts(self, clear: bool = False):
        """(capped local energies, capped weights, capped force-bias components, live
        walker-steps, walker-steps redone in FP64 by the precision guard) since setup or the
        last clear (``afqmc_get_bound_counts``)."""
        out = (C.c_uint64 * 5)()
        L.check(self.lib.afqmc_get_bound_counts(self.handle, out, int(clear)),
                "afqmc_get_bound_counts")
        return tuple(int(v) for v in out)

    def status(self, clear: bool = False) -> int:
        st = C.c_uint32()
        L.check(self.lib.afqmc_get_status(self.handle, C.byref(st), int(clear)), "afqmc_get_status")
        return int(st.value)

    # ---------------------------------------------------------------- tiles
    def autotune(self, wk: "Walkers", reuse: bool = True):
        """Time the contraction variants on these walkers, keep the fastest; returns
        (tile name, ms per launch or -1 when a stored choice was reused)."""
        t = C.c_int32()
        ms = C.c_double()
        L.check(self.lib.afqmc_autotune(self.handle, wk.c_ref(), int(reuse), C.byref(t),
                                        C.byref(ms)), "afqmc_autotune")
        return {v: k for k, v in L.TILES.items()}[t.value], ms.value

    def set_tile(self, tile: str) -> None:
        L.check(self.lib.afqmc_set_tile(self.handle, L.TILES[tile]), "afqmc_set_tile")

    @property
    def tile(self) -> str:
        t = C.c_int32()
        L.check(self.lib.afqmc_get_tile(self.handle, C.byref(t)), "afqmc_get_tile")
        return {v: k for k, v in L.TILES.items()}[t.value]

    # ---------------------------------------------------------------- timing
    def kernel_timing(self, enable: bool) -> None:
        L.check(self.lib.afqmc_kernel_timing(self.handle, int(enable)), "afqmc_kernel_timing")

    def kernel_time(self, group: str | int):
        k = L.KERNEL_GROUPS.index(group) if isinstance(group, str) else int(group)
        ms = C.c_double()
        n = C.c_int64()
        L.check(self.lib.afqmc_kernel_time(self.handle, k, C.byref(ms), C.byref(n)),
                "afqmc_kernel_time")
        return ms.value, int(n.value)


class Walkers:
    """Caller-owned device arrays of a walker population (torch tensors on the GPU)."""

    def __init__(self, system: System, n_walkers: int):
        torch = _torch()
        dev = torch.device("cuda", torch.cuda.current_device())
        n = int(n_walkers)
        self.n = n
        self.system = system
        self.U = torch.zeros((n, system.ntot, system.M), dtype=torch.complex128, device=dev)
        self.weight = torch.zeros(n, dtype=torch.float64, device=dev)
        self.arg_ovlp = torch.zeros(n, dtype=torch.float64, device=dev)
        self.log_ovlp = torch.zeros(n, dtype=torch.float64, device=dev)
        self.e_loc = torch.zeros(n, dtype=torch.complex128, device=dev)
        self.phase = torch.zeros(n, dtype=torch.float64, device=dev)
        self.walker_id = torch.arange(n, dtype=torch.int64, device=dev)
        nb = system.workspace_bytes(n)
        self._ws_raw = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        off = (-int(self._ws_raw.data_ptr())) % 256
        self.workspace = self._ws_raw[off:off + nb]
        self.step = 0
        self._c = L.WalkersC()

    def c_ref(self):
        c = self._c
        c.n_walkers = self.n
        c.reserved = 0
        c.U = int(self.U.data_ptr())
        c.weight = int(self.weight.data_ptr())
        c.arg_ovlp = int(self.arg_ovlp.data_ptr())
        c.log_ovlp = int(self.log_ovlp.data_ptr())
        c.e_loc = int(self.e_loc.data_ptr())
        c.phase = int(self.phase.data_ptr())
        c.walker_id = int(self.walker_id.data_ptr())
        c.workspace = int(self.workspace.data_ptr())
        c.workspace_bytes = int(self.workspace.numel())
        c.step = int(self.step)
        return C.byref(c)

    def sync_from_c(self):
        self.step = int(self._c.step)


class Batch:
    """Systems with their walkers stepped together by one graph launch per step
    (``afqmc_batch_*``).  Keeps the systems and walkers alive while it exists."""

    def __init__(self, pairs, stream=None, autotune: bool = False, families: bool = False):
        torch = _torch()
        self.lib = L.load()
        self.pairs = list(pairs)
        n = len(self.pairs)
        self.tiles = []
        for gs, wk in self.pairs:
            if autotune:
                self.tiles.append(gs.autotune(wk)[0])
                gs.measure(wk)   # cached traces and E_L from the tile now in use
            else:
                self.tiles.append(gs.tile)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        sysv = (C.c_void_p * n)(*[gs.handle.value for gs, _ in self.pairs])
        for _, wk in self.pairs:
            wk.c_ref()
        wv = (C.POINTER(L.WalkersC) * n)(*[C.pointer(wk._c) for _, wk in self.pairs])
        self._keep = (sysv, wv)
        h = C.c_void_p()
        L.check(self.lib.afqmc_batch_create(n, sysv, wv, C.c_void_p(_stream_handle(self.stream)),
                                            C.byref(h)), "afqmc_batch_create")
        self.handle = h
        self._fields = (L.FieldsC * n)()
        if families:
            self.set_families(True)

    def set_families(self, on: bool) -> None:
        """One contraction launch per family of systems sharing a kernel instance (mode 1 of
        ``afqmc_batch_set_mode``, not available: raises) or per system (mode 0)."""
        L.check(self.lib.afqmc_batch_set_mode(self.handle, 1 if on else 0), "afqmc_batch_set_mode")

    def step(self, seeds, job_ids=None) -> None:
        """One step of every system; fields drawn on the device from (seed, job_id)."""
        n = len(self.pairs)
        for i in range(n):
            self._fields[i].seed = int(seeds[i])
            self._fields[i].job_id = 0 if job_ids is None else int(job_ids[i])
            self._fields[i].x = None
            self._fields[i].u_comb = math.nan
        L.check(self.lib.afqmc_batch_step(self.handle, self._fields), "afqmc_batch_step")
        for _, wk in self.pairs:
            wk.sync_from_c()

    def close(self):
        if getattr(self, "handle", None):
            L.check(self.lib.afqmc_batch_destroy(self.handle), "afqmc_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def modified_cholesky(eri, delta: float, max_vectors: int | None = None, stream=None):
    """Modified Cholesky decomposition of a device tensor eri[p, q, r, s] = v_pqrs (float64,
    (M, M, M, M)) on the GPU.  Returns (L, converged) with L a device tensor (n, M, M)."""
    torch = _torch()
    lib = L.load()
    assert eri.is_cuda and eri.dtype == torch.float64 and eri.is_contiguous() and eri.dim() == 4
    M = int(eri.shape[0])
    nmax = M * M if max_vectors is None else int(max_vectors)
    out = torch.empty((max(nmax, 1), M, M), dtype=torch.float64, device=eri.device)
    wb = C.c_size_t()
    L.check(lib.afqmc_mcd_workspace_bytes(M, C.byref(wb)), "afqmc_mcd_workspace_bytes")
    raw = torch.empty(wb.value + 256, dtype=torch.uint8, device=eri.device)
    off = (-int(raw.data_ptr())) % 256
    n = C.c_int32()
    conv = C.c_int32()
    L.check(lib.afqmc_modified_cholesky(C.c_void_p(int(eri.data_ptr())), M, float(delta), nmax,
                                        C.c_void_p(int(out.data_ptr())), C.byref(n), C.byref(conv),
                                        C.c_void_p(int(raw.data_ptr()) + off), wb.value,
                                        C.c_void_p(_stream_handle(stream))),
            "afqmc_modified_cholesky")
    return out[: n.value], bool(conv.value)


def mfma_peak(precision: str = "fp32", stream=None) -> float:
    """Attainable dense MFMA rate in TFLOP/s (``afqmc_mfma_peak``): fp32 -> 32x32x2 FP32,
    fp64 -> 16x16x4 FP64, bf16x3 -> 32x32x16 BF16 (one product; a BF16x3 product takes three)."""
    torch = _torch()
    lib = L.load()
    buf = torch.empty(L.MFMA_PEAK_BYTES // 8, dtype=torch.float64, device="cuda")
    out = C.c_double()
    L.check(lib.afqmc_mfma_peak(L.PRECISIONS[precision], C.c_void_p(int(buf.data_ptr())),
                                L.MFMA_PEAK_BYTES, C.c_void_p(_stream_handle(stream)),
                                C.byref(out)), "afqmc_mfma_peak")
    return out.value
