"""Python binding of libkfvm.so (include/kfvm.h): argument marshalling only.

Every step of the right-hand side runs in the library's HIP kernels; torch is
used for device memory and the current stream.  There is no fallback: if the
library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkfvm.so")

KFVM_OK, KFVM_ERR_ARG, KFVM_ERR_HIP, KFVM_ERR_NONPHYSICAL, KFVM_ERR_STATE = 0, -1, -2, -3, -4
KFVM_FP64, KFVM_SPLIT_F16, KFVM_SPLIT_BF16 = 0, 1, 2
KFVM_HLLC, KFVM_HLL = 0, 1

EXPORTED = [
    "kfvm_init", "kfvm_init_length_scale", "kfvm_rhs", "kfvm_step", "kfvm_cfl_dt", "kfvm_set_stream",
    "kfvm_set_precision",
    "kfvm_set_limiter", "kfvm_set_flattener", "kfvm_set_cfl_form", "kfvm_set_riemann", "kfvm_set_checking", "kfvm_status", "kfvm_stats",
    "kfvm_face_states", "kfvm_weights_build", "kfvm_weights_size", "kfvm_last_error", "kfvm_destroy",
    "kfvm_set_timing", "kfvm_kernel_times", "kfvm_set_flags", "kfvm_mlp_sizes", "kfvm_set_gate",
    "kfvm_get_flags", "kfvm_gate_samples", "kfvm_mlp_train_step", "kfvm_set_indicator", "kfvm_kxrcf",
    "kfvm_set_boundary", "kfvm_step_ssp432", "kfvm_cfl_dt_noalloc",
]
KERNEL_CLASSES = ("recon", "flux", "update", "indicator")
KFVM_IND_NONE, KFVM_IND_KXRCF = 0, 1
BC_KINDS = {"periodic": 0, "outflow": 1, "reflecting": 2, "inflow": 3}


class KfvmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfvm error {code}: {msg}")
        self.code = code


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3)]


class _Weights(C.Structure):
    _fields_ = [("dim", C.c_int), ("R", C.c_int), ("n0", C.c_int), ("offsets", C.POINTER(C.c_int)),
                ("n_stencils", C.c_int), ("stencil_ptr", C.POINTER(C.c_int)),
                ("members", C.POINTER(C.c_int)), ("n_pts", C.c_int), ("n_der", C.c_int),
                ("tables", C.POINTER(C.c_double)), ("gamma_lin", C.POINTER(C.c_double))]


class _Stats(C.Structure):
    _fields_ = [("limiter_cells", C.c_longlong), ("weno_cell_vars", C.c_longlong),
                ("cell_vars", C.c_longlong), ("error", C.c_int), ("min_rho", C.c_double),
                ("min_p", C.c_double)]


_lib = None


def load_library(path: str = _LIB_PATH):
    """Load libkfvm.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2401_16543_amd.build`")
    lib = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.c_int
    sig = {
        "kfvm_init": ([C.POINTER(vp), C.POINTER(_Mesh), ip, C.c_double, C.POINTER(_Weights)], ip),
        "kfvm_init_length_scale": ([C.POINTER(vp), C.POINTER(_Mesh), ip, C.c_double, C.c_double], ip),
        "kfvm_rhs": ([vp, vp, vp], ip),
        "kfvm_step": ([vp, vp, C.c_double], ip),
        "kfvm_cfl_dt": ([vp, vp, C.c_double, dp], ip),
        "kfvm_cfl_dt_noalloc": ([vp, vp, C.c_double, vp], ip),
        "kfvm_set_stream": ([vp, vp], ip),
        "kfvm_set_precision": ([vp, ip], ip),
        "kfvm_set_limiter": ([vp, ip, C.c_double], ip),
        "kfvm_set_flattener": ([vp, C.c_double], ip),
        "kfvm_set_cfl_form": ([vp, ip], ip),
        "kfvm_set_riemann": ([vp, ip], ip),
        "kfvm_set_checking": ([vp, ip], ip),
        "kfvm_status": ([vp], ip),
        "kfvm_stats": ([vp, C.POINTER(_Stats)], ip),
        "kfvm_face_states": ([vp, vp, vp], ip),
        "kfvm_weights_build": ([ip, ip, C.c_double, dp, ip], ip),
        "kfvm_weights_size": ([ip, ip], ip),
        "kfvm_last_error": ([vp], C.c_char_p),
        "kfvm_set_timing": ([vp, ip], ip),
        "kfvm_set_flags": ([vp, vp], ip),
        "kfvm_mlp_sizes": ([ip, C.POINTER(ip), C.POINTER(ip)], ip),
        "kfvm_set_gate": ([vp, vp, C.c_float], ip),
        "kfvm_get_flags": ([vp, vp], ip),
        "kfvm_gate_samples": ([vp, vp, vp, vp], ip),
        "kfvm_mlp_train_step": ([vp, vp, vp, ip, vp, vp, vp, ip, C.c_float, C.c_float, vp, vp, vp], ip),
        "kfvm_kernel_times": ([vp, dp, C.POINTER(C.c_longlong), ip], ip),
        "kfvm_set_indicator": ([vp, ip, C.c_double], ip),
        "kfvm_set_boundary": ([vp, ip, ip, ip, dp, dp], ip),
        "kfvm_step_ssp432": ([vp, vp, vp, C.c_double, C.c_double, C.c_double, dp], ip),
        "kfvm_kxrcf": ([vp, vp, C.c_double, vp, vp], ip),
        "kfvm_destroy": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes, f.restype = args, res
    _lib = lib
    return lib


def weights_build(dim: int, R: int, ell_hat: float = 5.0):
    """The library's binary128 reconstruction tables, packed as in kfvm.h (host only)."""
    import numpy as np
    lib = load_library()
    n = lib.kfvm_weights_size(dim, R)
    if n < 0:
        raise KfvmError(n, "unsupported (dim, R)")
    out = np.zeros(n)
    rc = lib.kfvm_weights_build(dim, R, ell_hat, out.ctypes.data_as(C.POINTER(C.c_double)), n)
    if rc != n:
        raise KfvmError(rc, "weight build failed")
    return out


class KFVM:
    """One context of the library for a periodic box; U tensors are float64 on the GPU,
    shaped (nvar, ny, nx) in 2D or (nvar, nz, ny, nx) in 3D."""

    def __init__(self, dim: int, n, dx=None, order: int = 5, gamma: float = 1.4, weights=None,
                 ell_hat: float | None = None):
        """weights: tables to use instead of the library's own; ell_hat: the kernel
        length scale in cells for the library's own tables (default 5)."""
        if not torch.cuda.is_available():
            raise RuntimeError("KFVM needs a ROCm GPU; none is visible")
        self.lib = load_library()
        n = list(n)
        if len(n) != dim:
            raise ValueError("len(n) must equal dim")
        dx = list(dx) if dx is not None else [1.0 / x for x in n]
        self.dim, self.n, self.dx, self.order, self.gamma = dim, n, dx, order, gamma
        self.R = 2 if order == 5 else 3
        self.nvar = dim + 2
        self.shape = (self.nvar,) + tuple(reversed(n))
        mesh = _Mesh()
        mesh.dim = dim
        mesh.n[:] = n + [1] * (3 - dim)
        mesh.dx[:] = dx + [1.0] * (3 - dim)
        wp = C.POINTER(_Weights)()
        self._keep = None
        if weights is not None:
            wp, self._keep = self._pack_weights(weights)
        h = C.c_void_p()
        if ell_hat is not None:
            if weights is not None:
                raise ValueError("pass either weights or ell_hat")
            rc = self.lib.kfvm_init_length_scale(C.byref(h), C.byref(mesh), order, gamma, float(ell_hat))
        else:
            rc = self.lib.kfvm_init(C.byref(h), C.byref(mesh), order, gamma, wp)
        if rc != KFVM_OK:
            raise KfvmError(rc, self.lib.kfvm_last_error(None).decode())
        self._h = h

    @staticmethod
    def _pack_weights(T):
        """Marshal a dict with s0, members, weights (list of [rows, N_q]), n_pts, n_der, gamma."""
        import numpy as np
        d = T["s0"].shape[1]
        off = np.ascontiguousarray(T["s0"].reshape(-1), dtype=np.int32)
        mem = np.ascontiguousarray(np.concatenate(T["members"]), dtype=np.int32)
        ptr = np.ascontiguousarray(np.concatenate([[0], np.cumsum([len(m) for m in T["members"]])]),
                                   dtype=np.int32)
        tab = np.ascontiguousarray(np.concatenate([w.reshape(-1) for w in T["weights"]]), dtype=np.float64)
        gam = np.ascontiguousarray(T["gamma"], dtype=np.float64)
        w = _Weights()
        w.dim, w.R, w.n0 = d, int(T["R"]), len(T["s0"])
        w.offsets = off.ctypes.data_as(C.POINTER(C.c_int))
        w.n_stencils = len(T["members"])
        w.stencil_ptr = ptr.ctypes.data_as(C.POINTER(C.c_int))
        w.members = mem.ctypes.data_as(C.POINTER(C.c_int))
        w.n_pts, w.n_der = int(T["n_pts"]), int(T["n_der"])
        w.tables = tab.ctypes.data_as(C.POINTER(C.c_double))
        w.gamma_lin = gam.ctypes.data_as(C.POINTER(C.c_double))
        return C.pointer(w), (off, mem, ptr, tab, gam, w)

    # -- plumbing -------------------------------------------------------------
    def _check(self, rc):
        if rc != KFVM_OK:
            raise KfvmError(rc, self.lib.kfvm_last_error(self._h).decode())

    def _stream(self):
        self._check(self.lib.kfvm_set_stream(self._h, C.c_void_p(torch.cuda.current_stream().cuda_stream)))

    def _state(self, U):
        if not (isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float64 and U.is_contiguous()):
            raise TypeError("U must be a contiguous float64 CUDA tensor")
        if tuple(U.shape) != self.shape:
            raise ValueError(f"U must have shape {self.shape}, got {tuple(U.shape)}")
        return C.c_void_p(U.data_ptr())

    def close(self):
        if getattr(self, "_h", None):
            self.lib.kfvm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ---------------------------------------------------------
    def rhs(self, U, out=None):
        if out is None:
            out = torch.empty_like(U)
        self._stream()
        self._check(self.lib.kfvm_rhs(self._h, self._state(U), self._state(out)))
        return out

    def step(self, U, dt: float):
        self._stream()
        self._check(self.lib.kfvm_step(self._h, self._state(U), float(dt)))
        return U

    def step_ssp432(self, U, U_out, dt: float, atol: float = 1e-6, rtol: float = 1e-6) -> float:
        """One SSP(4,3,2) step from U into U_out; returns the weighted RMS norm of the
        embedded error estimate (accept the step when it is at most one)."""
        self._stream()
        err = C.c_double()
        self._check(self.lib.kfvm_step_ssp432(self._h, self._state(U), self._state(U_out), float(dt), float(atol),
                                              float(rtol), C.byref(err)))
        return err.value

    def cfl_dt(self, U, cfl: float) -> float:
        self._stream()
        dt = C.c_double()
        self._check(self.lib.kfvm_cfl_dt(self._h, self._state(U), float(cfl), C.byref(dt)))
        return dt.value

    def cfl_dt_noalloc(self, U, cfl: float, out):
        """kfvm_cfl_dt_noalloc: out (float64, 3 elements, on the GPU) receives dt,
        the least density and the least pressure; asynchronous, allocates nothing."""
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != 3:
            raise ValueError("out must be a contiguous float64 CUDA tensor of 3 elements")
        self._stream()
        self._check(self.lib.kfvm_cfl_dt_noalloc(self._h, self._state(U), float(cfl), C.c_void_p(out.data_ptr())))
        return out

    def face_states(self, U):
        npts = 2 * self.dim * self.R ** (self.dim - 1)
        ncell = 1
        for x in self.n:
            ncell *= x
        out = torch.empty((ncell, npts, self.nvar), dtype=torch.float64, device=U.device)
        self._stream()
        self._check(self.lib.kfvm_face_states(self._h, self._state(U), C.c_void_p(out.data_ptr())))
        return out

    def set_limiter(self, enabled: bool, kappa: float = 0.5):
        self._check(self.lib.kfvm_set_limiter(self._h, int(enabled), float(kappa)))

    def set_flattener(self, k1: float | None):
        """The limiter's flattener eta with onset k1 (None or 0: eta = 0)."""
        self._check(self.lib.kfvm_set_flattener(self._h, float(k1) if k1 else 0.0))

    def set_cfl_form(self, form: str):
        """The formula of cfl_dt: "sum" (default) or "max_axis"."""
        self._check(self.lib.kfvm_set_cfl_form(self._h, {"sum": 0, "max_axis": 1}[form]))

    def set_riemann(self, solver: str):
        self._check(self.lib.kfvm_set_riemann(self._h, {"hllc": KFVM_HLLC, "hll": KFVM_HLL}[solver]))

    def set_precision(self, mode: str):
        self._check(self.lib.kfvm_set_precision(
            self._h, {"fp64": KFVM_FP64, "split_f16": KFVM_SPLIT_F16, "split_bf16": KFVM_SPLIT_BF16}[mode]))

    def set_checking(self, on: bool):
        self._check(self.lib.kfvm_set_checking(self._h, int(on)))

    def status(self):
        return self.lib.kfvm_status(self._h)

    def set_flags(self, flags):
        """flags: uint8 CUDA tensor [nvar, ncell] (1 = WENO-AO, 0 = linear S0) or None."""
        if flags is None:
            self._flags = None
            self._check(self.lib.kfvm_set_flags(self._h, None))
            return
        if not (flags.is_cuda and flags.dtype == torch.uint8 and flags.is_contiguous()
                and flags.numel() == self.nvar * (self.shape[1] * self.shape[2] * (self.shape[3] if self.dim == 3 else 1))):
            raise ValueError("flags must be a contiguous uint8 CUDA tensor of nvar * ncell entries")
        self._flags = flags
        self._check(self.lib.kfvm_set_flags(self._h, C.c_void_p(flags.data_ptr())))

    def set_boundary(self, axis: int, lower: str, upper: str, lower_state=None, upper_state=None):
        """Boundary conditions of one axis: "periodic" on both sides, or per side
        "outflow", "reflecting", "inflow" (with its conserved state)."""
        def arr(x):
            if x is None:
                return None
            a = (C.c_double * self.nvar)(*[float(v) for v in x])
            return C.cast(a, C.POINTER(C.c_double))
        lo, hi = arr(lower_state), arr(upper_state)
        self._check(self.lib.kfvm_set_boundary(self._h, int(axis), BC_KINDS[lower], BC_KINDS[upper], lo, hi))

    # -- KXRCF indicator -------------------------------------------------------
    def set_indicator(self, kind, m: float = 1.5):
        """kind: "kxrcf" (the two-pass reconstruction with threshold Delta^m) or None."""
        self._check(self.lib.kfvm_set_indicator(self._h, {None: KFVM_IND_NONE, "kxrcf": KFVM_IND_KXRCF}[kind],
                                                float(m)))

    def kxrcf(self, U, m: float = 1.5):
        """One pass of the indicator on U: (jumps [dim, ncell] float64 of the upper
        faces, flags [nvar, ncell] uint8, 1 = WENO-AO)."""
        ncell = U[0].numel()
        jumps = torch.empty((self.dim, ncell), dtype=torch.float64, device=U.device)
        flags = torch.empty((self.nvar, ncell), dtype=torch.uint8, device=U.device)
        self._stream()
        self._check(self.lib.kfvm_kxrcf(self._h, self._state(U), float(m), C.c_void_p(jumps.data_ptr()),
                                        C.c_void_p(flags.data_ptr())))
        return jumps, flags

    # -- learned gate ------------------------------------------------------------
    def mlp_sizes(self):
        n_in, n_p = C.c_int(), C.c_int()
        self._check(self.lib.kfvm_mlp_sizes(self.dim, C.byref(n_in), C.byref(n_p)))
        return n_in.value, n_p.value

    def set_gate(self, params, threshold: float = 0.0):
        """params: float32 CUDA tensor of the network (None disables the gate)."""
        if params is None:
            self._check(self.lib.kfvm_set_gate(self._h, None, 0.0))
            return
        self._gate_params = params.contiguous()
        self._check(self.lib.kfvm_set_gate(self._h, C.c_void_p(self._gate_params.data_ptr()), float(threshold)))

    def get_flags(self):
        ncell = 1
        for x in self.n:
            ncell *= x
        out = torch.empty((self.nvar, ncell), dtype=torch.uint8, device="cuda")
        self._stream()
        self._check(self.lib.kfvm_get_flags(self._h, C.c_void_p(out.data_ptr())))
        return out

    def gate_samples(self, U, inputs: bool = True):
        """(x [nvar, ncell, n_in] float32 or None, omega_0/gamma_0 [nvar, ncell] float32);
        inputs=False: the labels alone."""
        n_in, _ = self.mlp_sizes()
        ncell = 1
        for v in self.n:
            ncell *= v
        x = torch.empty((self.nvar, ncell, n_in), dtype=torch.float32, device=U.device) if inputs else None
        r = torch.empty((self.nvar, ncell), dtype=torch.float32, device=U.device)
        self._stream()
        self._check(self.lib.kfvm_gate_samples(self._h, self._state(U), C.c_void_p(x.data_ptr()) if inputs else None,
                                               C.c_void_p(r.data_ptr())))
        return x, r

    def mlp_train_step(self, x, y, params, m=None, v=None, t=1, lr=0.0, pos_weight=1.0, want_grad=False,
                       want_logits=False):
        """One step on a batch; returns (loss tensor, grad or None, logits or None)."""
        B = x.shape[0]
        ptr = lambda a: C.c_void_p(a.data_ptr()) if a is not None else None
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        grad = torch.empty_like(params) if want_grad else None
        logits = torch.empty(B, dtype=torch.float32, device=x.device) if want_logits else None
        self._stream()
        self._check(self.lib.kfvm_mlp_train_step(self._h, ptr(x), ptr(y), B, ptr(params), ptr(m), ptr(v), int(t),
                                                 float(lr), float(pos_weight), ptr(loss), ptr(grad), ptr(logits)))
        return loss, grad, logits

    def set_timing(self, on: bool):
        self._check(self.lib.kfvm_set_timing(self._h, int(on)))

    def kernel_times(self) -> dict:
        """{kernel class: (total ms, launches)} since the last call."""
        k = len(KERNEL_CLASSES)
        ms = (C.c_double * k)()
        n = (C.c_longlong * k)()
        self._check(self.lib.kfvm_kernel_times(self._h, ms, n, k))
        return {k: (ms[i], n[i]) for i, k in enumerate(KERNEL_CLASSES)}

    def stats(self) -> dict:
        s = _Stats()
        self._check(self.lib.kfvm_stats(self._h, C.byref(s)))
        return dict(limiter_cells=s.limiter_cells, weno_cell_vars=s.weno_cell_vars, cell_vars=s.cell_vars,
                    error=s.error, min_rho=s.min_rho, min_p=s.min_p)
