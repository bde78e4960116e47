"""Oracle: Python driver of the plain-C KFVM-WENO right-hand side (kfvm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product path never does.

`Oracle(d, R, n, dx, gamma, ...)` holds the tables of oracle.weights and exposes
rhs / step / states / rhs_cells / cfl_dt / riemann on numpy float64 arrays laid
out as U[v][z][y][x] (2D: U[v][y][x]).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import weights as _w

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kfvm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EPS_WENO = 1e-40   # epsilon of the nonlinear weights (section 3.3)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Ctx(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("R", C.c_int), ("nvar", C.c_int),
        ("n", C.c_int * 3), ("dx", C.c_double * 3), ("gamma", C.c_double),
        ("n0", C.c_int), ("s0", C.POINTER(C.c_int)), ("nst", C.c_int),
        ("mem_ptr", C.POINTER(C.c_int)), ("mem", C.POINTER(C.c_int)),
        ("w_ptr", C.POINTER(C.c_int)), ("w", C.POINTER(C.c_double)),
        ("lin_w", C.POINTER(C.c_double)), ("n_pts", C.c_int), ("n_der", C.c_int),
        ("gl_w", C.POINTER(C.c_double)), ("eps", C.c_double),
        ("limiter", C.c_int), ("kappa", C.c_double), ("riemann", C.c_int),
        ("weno", C.c_int), ("flags", C.POINTER(C.c_uint8)), ("kxrcf_m", C.c_double),
        ("bc", C.c_int * 6), ("bc_state", C.c_double * 30), ("flat_k1", C.c_double),
        ("cfl_max_axis", C.c_int),
    ]

BC_KINDS = {"periodic": 0, "outflow": 1, "reflecting": 2, "inflow": 3}


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER
        for name, args in [
            ("oracle_states", [P(_Ctx), P(C.c_double), P(C.c_double)]),
            ("oracle_rhs", [P(_Ctx), P(C.c_double), P(C.c_double)]),
            ("oracle_rhs_cells", [P(_Ctx), P(C.c_double), C.c_long, P(C.c_long), P(C.c_double)]),
            ("oracle_step", [P(_Ctx), P(C.c_double), C.c_double]),
            ("oracle_cfl_dt", [P(_Ctx), P(C.c_double), C.c_double, P(C.c_double)]),
        ]:
            f = getattr(_lib, name)
            f.argtypes, f.restype = args, C.c_int
        _lib.oracle_riemann.argtypes = [P(_Ctx), C.c_long, P(C.c_double), P(C.c_double), C.c_int,
                                        P(C.c_double)]
        _lib.oracle_riemann.restype = None
        _lib.oracle_omega_ratio.argtypes = [P(_Ctx), P(C.c_double), P(C.c_float)]
        _lib.oracle_omega_ratio.restype = C.c_int
        _lib.oracle_phi.argtypes = [P(_Ctx), P(C.c_double), P(C.c_double), P(C.c_double)]
        _lib.oracle_smoothness.argtypes = [P(_Ctx), P(C.c_double), C.c_long, P(C.c_double)]
        _lib.oracle_smoothness.restype = C.c_int
        _lib.oracle_phi.restype = None
        _lib.oracle_kxrcf.argtypes = [P(_Ctx), P(C.c_double), C.c_double, P(C.c_uint8), P(C.c_double),
                                      P(C.c_double)]
        _lib.oracle_kxrcf.restype = C.c_int
        _lib.oracle_kxrcf_cells.argtypes = [P(_Ctx), P(C.c_double), C.c_long, P(C.c_long), P(C.c_double)]
        _lib.oracle_kxrcf_cells.restype = C.c_int
        _lib.oracle_step_ssp432.argtypes = [P(_Ctx), P(C.c_double), C.c_double, C.c_double, C.c_double,
                                            P(C.c_double), P(C.c_double)]
        _lib.oracle_step_ssp432.restype = C.c_int
        _lib.oracle_flattener.argtypes = [P(_Ctx), P(C.c_double), P(C.c_double)]
        _lib.oracle_flattener.restype = C.c_int
    return _lib


def _ptr(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


class OracleError(RuntimeError):
    pass


class Oracle:
    """Plain CPU KFVM-WENO on a periodic box of n cells per axis."""

    def __init__(self, d: int, R: int, n, dx=None, gamma: float = 1.4, *, limiter: bool = True,
                 kappa: float = 0.5, riemann: str = "hllc", weno: bool = True, tables=None,
                 kxrcf_m: float | None = None, flattener: float | None = None):
        self.d, self.R = d, R
        self.nvar = d + 2
        n = list(n) + [1] * (3 - len(n))
        dx = list(dx) if dx is not None else [1.0 / n[a] for a in range(d)]
        dx = dx + [1.0] * (3 - len(dx))
        self.shape = tuple(reversed(n[:d]))        # numpy spatial shape (z, y, x)
        self.ncell = int(np.prod(n))
        T = tables if tables is not None else _w.tables(d, R)
        self.tables = T
        keep = []

        def arr(x, dt):
            a = np.ascontiguousarray(np.asarray(x, dtype=dt))
            keep.append(a)
            return a

        s0 = arr(T["s0"].reshape(-1), np.int32)
        mem = arr(np.concatenate(T["members"]), np.int32)
        mem_ptr = arr(np.concatenate([[0], np.cumsum([len(m) for m in T["members"]])]), np.int32)
        w = arr(np.concatenate([x.reshape(-1) for x in T["weights"]]), np.float64)
        w_ptr = arr(np.concatenate([[0], np.cumsum([x.size for x in T["weights"]])[:-1]]), np.int32)
        lin_w = arr(T["gamma"], np.float64)
        gl_w = arr(T["gl_weights"], np.float64)
        self._keep = keep
        ctx = _Ctx()
        ctx.dim, ctx.R, ctx.nvar = d, R, self.nvar
        ctx.n[:] = n
        ctx.dx[:] = dx
        ctx.gamma = gamma
        ctx.n0 = len(T["s0"])
        ctx.s0 = _ptr(s0, C.c_int)
        ctx.nst = len(T["members"])
        ctx.mem_ptr, ctx.mem = _ptr(mem_ptr, C.c_int), _ptr(mem, C.c_int)
        ctx.w_ptr, ctx.w = _ptr(w_ptr, C.c_int), _ptr(w)
        ctx.lin_w = _ptr(lin_w)
        ctx.n_pts, ctx.n_der = T["n_pts"], T["n_der"]
        ctx.gl_w = _ptr(gl_w)
        ctx.eps = EPS_WENO
        ctx.limiter, ctx.kappa = int(limiter), kappa
        ctx.riemann = {"hllc": 0, "hll": 1}[riemann]
        ctx.weno = int(weno)
        ctx.flags = C.POINTER(C.c_uint8)()
        ctx.kxrcf_m = float(kxrcf_m) if kxrcf_m else 0.0
        ctx.flat_k1 = float(flattener) if flattener else 0.0
        self._ctx = ctx
        self._lib = _load()

    # -- helpers ------------------------------------------------------------
    def _check_U(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        if U.shape != (self.nvar,) + self.shape:
            raise ValueError(f"U must have shape {(self.nvar,) + self.shape}, got {U.shape}")
        return U

    def _call(self, rc):
        if rc != 0:
            raise OracleError(f"oracle returned {rc}")

    def set_boundary(self, axis: int, lower: str, upper: str, lower_state=None, upper_state=None):
        """Boundary conditions of one axis (section 5.3, steps 1 and 4): "periodic"
        on both sides, or any of "outflow", "reflecting", "inflow" per side; an
        inflow side takes its conserved state (nvar values)."""
        if (lower == "periodic") != (upper == "periodic"):
            raise ValueError("periodic must be set on both sides of an axis")
        for side, (kind, state) in enumerate(((lower, lower_state), (upper, upper_state))):
            self._ctx.bc[2 * axis + side] = BC_KINDS[kind]
            if kind == "inflow":
                st = np.asarray(state, dtype=np.float64)
                if st.shape != (self.nvar,):
                    raise ValueError("an inflow side needs its conserved state")
                for v in range(self.nvar):
                    self._ctx.bc_state[(2 * axis + side) * 5 + v] = float(st[v])

    def set_flattener(self, k1):
        """The limiter's flattener eta (section 4; the compression ramp with onset
        k1, see oracle_flattener) instead of eta = 0 (None or 0: off)."""
        self._ctx.flat_k1 = float(k1) if k1 else 0.0

    def flattener(self, U):
        """eta of every cell [cells] (0 with the flattener off)."""
        U = self._check_U(U)
        eta = np.empty(self.ncell)
        self._call(self._lib.oracle_flattener(C.byref(self._ctx), _ptr(U), _ptr(eta)))
        return eta

    def set_kxrcf(self, m):
        """The KXRCF indicator (section 3.5) with threshold Delta^m picks the WENO
        cells of every right-hand side (None: off)."""
        self._ctx.kxrcf_m = float(m) if m else 0.0

    def kxrcf(self, U, m: float = 1.5):
        """KXRCF decisions of one state: (flags [nvar, cells] uint8, measure [cells]
        = max_s |q+ - q-| / <Q>, jumps [cells, 2 d] per-face maxima with the lower
        face of axis a at 2a and the upper one at 2a + 1)."""
        U = self._check_U(U)
        flags = np.empty((self.nvar, self.ncell), dtype=np.uint8)
        measure = np.empty(self.ncell)
        jumps = np.empty((self.ncell, 2 * self.d))
        self._call(self._lib.oracle_kxrcf(C.byref(self._ctx), _ptr(U), float(m), _ptr(flags, C.c_uint8),
                                          _ptr(measure), _ptr(jumps)))
        return flags, measure, jumps

    def kxrcf_cells(self, U, cells):
        """The KXRCF measure max_s |q+ - q-| / <Q> at the listed cells only."""
        U = self._check_U(U)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty(len(cells))
        self._call(self._lib.oracle_kxrcf_cells(C.byref(self._ctx), _ptr(U), len(cells), _ptr(cells, C.c_long),
                                                _ptr(out)))
        return out

    def kxrcf_threshold(self, m: float = 1.5):
        """Delta^m, Delta the largest grid spacing."""
        return max(self._ctx.dx[a] for a in range(self.d)) ** m

    def set_flags(self, flags):
        """Replay gate decisions: flags[v][cells] = 1 for WENO, 0 for the linear S0 value."""
        if flags is None:
            self._flags = None
            self._ctx.flags = C.POINTER(C.c_uint8)()
            return
        f = np.ascontiguousarray(flags, dtype=np.uint8).reshape(self.nvar, self.ncell)
        self._flags = f
        self._ctx.flags = _ptr(f, C.c_uint8)

    # -- the method ---------------------------------------------------------
    def rhs(self, U):
        U = self._check_U(U)
        out = np.empty_like(U)
        self._call(self._lib.oracle_rhs(C.byref(self._ctx), _ptr(U), _ptr(out)))
        return out

    def states(self, U):
        """Riemann states after the limiter: [cells, n_pts, nvar] (conserved variables)."""
        U = self._check_U(U)
        out = np.empty((self.ncell, self.tables["n_pts"], self.nvar))
        self._call(self._lib.oracle_states(C.byref(self._ctx), _ptr(U), _ptr(out)))
        return out

    def rhs_cells(self, U, cells):
        U = self._check_U(U)
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((len(cells), self.nvar))
        self._call(self._lib.oracle_rhs_cells(C.byref(self._ctx), _ptr(U), len(cells),
                                              _ptr(cells, C.c_long), _ptr(out)))
        return out

    def step(self, U, dt):
        U = self._check_U(U).copy()
        self._call(self._lib.oracle_step(C.byref(self._ctx), _ptr(U), float(dt)))
        return U

    def step_ssp432(self, U, dt, atol=1e-6, rtol=1e-6):
        """One SSP(4,3,2) step: (U+, weighted RMS norm of the embedded error estimate)."""
        U = self._check_U(U)
        out = np.empty_like(U)
        err = C.c_double()
        self._call(self._lib.oracle_step_ssp432(C.byref(self._ctx), _ptr(U), float(dt), float(atol), float(rtol),
                                                _ptr(out), C.byref(err)))
        return out, err.value

    def set_cfl_form(self, form: str):
        """The CFL step: "sum" (default) takes dt = cfl / max over cells of the sum
        over axes of (|u_a| + c) / dx_a, "max_axis" of its largest term."""
        self._ctx.cfl_max_axis = {"sum": 0, "max_axis": 1}[form]

    def cfl_dt(self, U, cfl):
        U = self._check_U(U)
        dt = C.c_double()
        self._call(self._lib.oracle_cfl_dt(C.byref(self._ctx), _ptr(U), float(cfl), C.byref(dt)))
        return dt.value

    def riemann(self, uL, uR, axis):
        uL = np.ascontiguousarray(uL, dtype=np.float64).reshape(-1, self.nvar)
        uR = np.ascontiguousarray(uR, dtype=np.float64).reshape(-1, self.nvar)
        F = np.empty_like(uL)
        self._lib.oracle_riemann(C.byref(self._ctx), len(uL), _ptr(uL), _ptr(uR), int(axis), _ptr(F))
        return F

    def phi(self, ref):
        """(Phi, Phi^-1) of the linearised primitive variables at a reference state."""
        ref = np.ascontiguousarray(ref, dtype=np.float64)
        A = np.empty((self.nvar, self.nvar))
        B = np.empty((self.nvar, self.nvar))
        self._lib.oracle_phi(C.byref(self._ctx), _ptr(ref), _ptr(A), _ptr(B))
        return A, B

    def smoothness(self, U, cell: int):
        """Smoothness indicators beta[variable, stencil] of one cell (eq. smoothIndic)."""
        U = self._check_U(U)
        out = np.empty((self.nvar, self._ctx.nst))
        self._call(self._lib.oracle_smoothness(C.byref(self._ctx), _ptr(U), int(cell), _ptr(out)))
        return out

    def omega_ratio(self, U):
        """omega_0 / gamma_0 of the WENO-AO weights per (variable, cell): [nvar, cells] float32."""
        U = self._check_U(U)
        out = np.empty((self.nvar, self.ncell), dtype=np.float32)
        self._call(self._lib.oracle_omega_ratio(C.byref(self._ctx), _ptr(U), _ptr(out, C.c_float)))
        return out

    def gate_inputs(self, U):
        """Gate-network inputs of every (variable, cell): [nvar, cells, n_in] float64.
        2D: the 5 x 5 window (offsets lexicographic, x slowest); 3D: the radius-2
        sphere in S0 order.  W = Phi(U_cell) U_h, increments W_h - W_c divided by the
        power of two 2^ex with max |W_h - W_c| in [2^(ex-1), 2^ex)."""
        U = self._check_U(U)
        d, nv = self.d, self.nvar
        if d == 2:
            offs = [(i - 2, j - 2) for i in range(5) for j in range(5)]
        else:
            offs = [tuple(o) for o in _w.full_stencil(3, 2)]
        n = self.shape[::-1]
        cells = np.arange(self.ncell)
        idx = [cells % n[0], (cells // n[0]) % n[1]] + ([cells // (n[0] * n[1])] if d == 3 else [])
        flat = U.reshape(nv, -1)
        out = np.empty((nv, self.ncell, len(offs)))
        Phi = np.empty((self.ncell, nv, nv))
        for c in range(self.ncell):
            Phi[c] = self.phi(flat[:, c])[0]
        Wc = np.einsum("cij,jc->ci", Phi, flat)
        for h, o in enumerate(offs):
            nb = np.zeros(self.ncell, dtype=np.int64)
            stride = 1
            for a in range(d):
                nb += ((idx[a] + o[a]) % n[a]) * stride
                stride *= n[a]
            W = np.einsum("cij,jc->ci", Phi, flat[:, nb])
            out[:, :, h] = (W - Wc).T
        amax = np.abs(out).max(axis=2, keepdims=True)
        ex = np.where(amax > 0, np.frexp(np.where(amax > 0, amax, 1.0))[1], 0)
        return np.ldexp(out, -ex)
