"""ctypes binding of the FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product library.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MB_ORACLE_LIB lets the mutation test load a deliberately broken build
LIB_PATH = os.environ.get("MB_ORACLE_LIB") or os.path.join(HERE, "libmboracle.so")

PEC, MUR1, ABSORB = 0, 1, 2
GROUND, PREPUMPED = 0, 1
NFIELDS = 24
# coefficient vector indices (mb_oracle.h)
(C_DT, C_S, C_A, C_B, C_CK, C_CF, C_BETA, C_DT32, C_DT21, C_DT10, C_DTWP, C_NA,
 C_WA, C_DWA, C_OMP2, C_COUNT) = range(16)


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("bc", C.c_int32 * 3),
        ("round_f32", C.c_int32), ("frozen_pop", C.c_int32),
        ("dx", C.c_double), ("courant", C.c_double),
        ("lambda0", C.c_double), ("dlambda", C.c_double),
        ("tau32", C.c_double), ("tau21", C.c_double), ("tau10", C.c_double),
        ("Wp", C.c_double), ("N_ref", C.c_double), ("E_ref", C.c_double),
        ("E_sp", C.c_double),
        ("seed", C.c_uint64), ("realization", C.c_uint32), ("noise", C.c_int32),
        ("absorb_cells", C.c_int32), ("absorb_order", C.c_int32), ("absorb_rate", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(Params)]
        L.orc_destroy.argtypes = [P]
        L.orc_coefficients.argtypes = [P, dp]
        L.orc_set_material.argtypes = [P, C.c_void_p, C.c_void_p]
        L.orc_set_pump.argtypes = [P, C.c_double, C.c_int]
        L.orc_set_source.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                     C.c_double, C.c_double, C.c_double]
        L.orc_source_value.restype = C.c_double
        L.orc_source_value.argtypes = [P, C.c_int64]
        L.orc_set_cw_source.argtypes = [P, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                        C.c_double, C.c_double]
        L.orc_set_plane_monitor.argtypes = [P, C.c_int]
        L.orc_read_plane_monitor.restype = C.c_int64
        L.orc_read_plane_monitor.argtypes = [P, dp]
        L.orc_set_probes.argtypes = [P, C.c_void_p, C.c_int, C.c_void_p, C.c_int]
        L.orc_set_loss_box.argtypes = [P] + [C.c_int] * 6
        L.orc_step.argtypes = [P, C.c_int64]
        L.orc_step_index.restype = C.c_int64
        L.orc_step_index.argtypes = [P]
        L.orc_get_field.argtypes = [P, C.c_int, dp]
        L.orc_set_field.argtypes = [P, C.c_int, dp]
        L.orc_read_energy.argtypes = [P, dp, dp]
        L.orc_energy_history.restype = C.c_int64
        L.orc_energy_history.argtypes = [P, dp, C.c_int64]
        L.orc_read_spectrum.argtypes = [P, dp]
        L.orc_read_loss.restype = C.c_double
        L.orc_read_loss.argtypes = [P]
        u32p = C.POINTER(C.c_uint32)
        L.orc_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.orc_normals3.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, dp]
        L.orc_p_next.restype = C.c_double
        L.orc_p_next.argtypes = [dp] + [C.c_double] * 5
        L.orc_pop_next.argtypes = [dp, dp, C.c_double, C.c_double]
        L.orc_p_series.argtypes = [dp, dp, dp, C.c_int64, dp]
        L.orc_pop_series.argtypes = [dp, dp, dp, dp, C.c_int64, dp]
        pp = C.POINTER(dp)
        L.orc_adjoint_run.argtypes = [P, C.c_int64, dp, dp, dp]
        L.orc_tangent_step.argtypes = [P, pp, pp]
        L.orc_adjoint_step.argtypes = [P, pp, pp]
        L.orc_pack_md.restype = C.c_int
        L.orc_pack_md.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_double]
        L.orc_pack_energy.argtypes = [C.c_int, dp, dp, dp, C.c_double, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def default_params(n, *, bc=(PEC, PEC, PEC), round_f32=False, frozen_pop=False,
                   noise=True, seed=0, realization=0, **kw) -> Params:
    """Parameter block with the workload defaults (dx 20 nm, Courant 0.99,
    lambda0 590 nm, 230 nm gain bandwidth, tau32 = tau10 = 100 fs,
    tau21 = 1 ns, W_p = 1e12 /s, E_ref = 1e8 V/m, N_ref = 1e24 m^-3,
    E_sp = 1e-6; lossy layer of 8 cells, quadratic grading, a_max = 0.25)."""
    if isinstance(n, int):
        n = (n, n, n)
    p = Params()
    p.nx, p.ny, p.nz = n
    for a in range(3):
        p.bc[a] = bc[a]
    p.round_f32 = int(bool(round_f32))
    p.frozen_pop = int(bool(frozen_pop))
    p.dx = kw.pop("dx", 20e-9)
    p.courant = kw.pop("courant", 0.99)
    p.lambda0 = kw.pop("lambda0", 590e-9)
    p.dlambda = kw.pop("dlambda", 230e-9)
    p.tau32 = kw.pop("tau32", 100e-15)
    p.tau21 = kw.pop("tau21", 1e-9)
    p.tau10 = kw.pop("tau10", 100e-15)
    p.Wp = kw.pop("Wp", 1e12)
    p.N_ref = kw.pop("N_ref", 1e24)
    p.E_ref = kw.pop("E_ref", 1e8)
    p.E_sp = kw.pop("E_sp", 1e-6)
    p.absorb_cells = kw.pop("absorb_cells", 8)
    p.absorb_order = kw.pop("absorb_order", 2)
    p.absorb_rate = kw.pop("absorb_rate", 0.25)
    if kw:
        raise TypeError(f"unknown parameters {sorted(kw)}")
    p.seed = seed
    p.realization = realization
    p.noise = int(bool(noise))
    return p


class Oracle:
    """One FP64 simulation on the CPU."""

    def __init__(self, params: Params):
        self.params = params
        self.n = (params.nx, params.ny, params.nz)
        self.shape = (params.nz + 1, params.ny + 1, params.nx + 1)
        self._h = lib().orc_create(C.byref(params))
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coefficients(self) -> np.ndarray:
        out = np.zeros(C_COUNT)
        lib().orc_coefficients(self._h, _dp(out))
        return out

    def set_material(self, eps: np.ndarray, gain: np.ndarray):
        eps = np.ascontiguousarray(eps, dtype=np.float32)
        gain = np.ascontiguousarray(gain, dtype=np.uint8)
        assert eps.shape == (self.n[2], self.n[1], self.n[0]) == gain.shape
        if lib().orc_set_material(self._h, eps.ctypes.data, gain.ctypes.data) != 0:
            raise ValueError("bad material")

    def set_pump(self, Na: float, init: int = PREPUMPED):
        if lib().orc_set_pump(self._h, Na, init) != 0:
            raise ValueError("bad pump")

    def set_source(self, comp, i, j, k, amp=1.0, lambda_s=532e-9, tau_p=1e-15, t0=4e-15):
        if lib().orc_set_source(self._h, comp, i, j, k, amp, lambda_s, tau_p, t0) != 0:
            raise ValueError("bad source")

    def source_value(self, n: int) -> float:
        return lib().orc_source_value(self._h, n)

    def set_cw_source(self, comp, i, j, k, amp=1.0, lambda_s=586.5e-9, t_ramp=20e-15):
        if lib().orc_set_cw_source(self._h, comp, i, j, k, amp, lambda_s, t_ramp) != 0:
            raise ValueError("bad source")

    def set_plane_monitor(self, k: int):
        if lib().orc_set_plane_monitor(self._h, int(k)) != 0:
            raise ValueError("bad plane")

    def plane_monitor(self):
        """(sums of the plane's energy density (ny, nx), steps summed)."""
        out = np.empty((self.n[1], self.n[0]))
        cnt = lib().orc_read_plane_monitor(self._h, _dp(out))
        if cnt < 0:
            raise ValueError("no plane monitor")
        return out, int(cnt)

    def set_probes(self, sites: np.ndarray, omega: np.ndarray):
        sites = np.ascontiguousarray(sites, dtype=np.int32).reshape(-1, 4)
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        self._np, self._nf = sites.shape[0], omega.shape[0]
        if lib().orc_set_probes(self._h, sites.ctypes.data, self._np, omega.ctypes.data,
                                self._nf) != 0:
            raise ValueError("bad probes")

    def set_loss_box(self, lo: Sequence[int], hi: Sequence[int]):
        if lib().orc_set_loss_box(self._h, *lo, *hi) != 0:
            raise ValueError("bad loss box")

    def step(self, n: int):
        lib().orc_step(self._h, int(n))

    @property
    def step_index(self) -> int:
        return lib().orc_step_index(self._h)

    def field(self, fid: int) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        if lib().orc_get_field(self._h, fid, _dp(out)) != 0:
            raise ValueError("bad field id")
        return out

    def set_field(self, fid: int, a: np.ndarray):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == self.shape
        if lib().orc_set_field(self._h, fid, _dp(a)) != 0:
            raise ValueError("bad field id")

    def energy(self):
        a, b = C.c_double(), C.c_double()
        lib().orc_read_energy(self._h, C.byref(a), C.byref(b))
        return a.value, b.value

    def energy_history(self) -> np.ndarray:
        n = lib().orc_energy_history(self._h, None, 0)
        out = np.empty(n)
        lib().orc_energy_history(self._h, _dp(out), n)
        return out

    def spectrum(self) -> np.ndarray:
        out = np.empty((self._np, self._nf, 2))
        lib().orc_read_spectrum(self._h, _dp(out))
        return out[..., 0] + 1j * out[..., 1]

    def loss(self) -> float:
        return lib().orc_read_loss(self._h)

    def adjoint_run(self, nsteps: int):
        """(L, dL/d eps_r per cell (nz, ny, nx), dL/dN_a) of the loss-box
        objective over nsteps from the pump; advances the run."""
        g = np.zeros((self.n[2], self.n[1], self.n[0]))
        gna, L = C.c_double(), C.c_double()
        if lib().orc_adjoint_run(self._h, int(nsteps), _dp(g), C.byref(gna), C.byref(L)) != 0:
            raise ValueError("adjoint needs a loss box, step 0 and no Mur walls")
        return L.value, g, gna.value

    def _lin(self, fn, vecs):
        vin = [np.ascontiguousarray(v, dtype=np.float64) for v in vecs]
        assert len(vin) == 24 and all(v.shape == self.shape for v in vin)
        vout = [np.empty(self.shape) for _ in range(24)]
        pin = (C.POINTER(C.c_double) * 24)(*[_dp(v) for v in vin])
        pout = (C.POINTER(C.c_double) * 24)(*[_dp(v) for v in vout])
        if fn(self._h, pin, pout) != 0:
            raise ValueError("not available with Mur walls")
        return vout

    def tangent_step(self, v):
        """J v for one step at the current state (24 field arrays in id order)."""
        return self._lin(lib().orc_tangent_step, v)

    def adjoint_step(self, w):
        """J^T w for one step at the current state."""
        return self._lin(lib().orc_adjoint_step, w)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def normals3(seed: int, cell: int, step: int, realization: int) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_normals3(seed, cell, step, realization, _dp(out))
    return out


def p_series(coef: np.ndarray, E: np.ndarray, dN: np.ndarray) -> np.ndarray:
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    dN = np.ascontiguousarray(dN, dtype=np.float64)
    out = np.empty_like(E)
    lib().orc_p_series(_dp(coef), _dp(E), _dp(dN), E.shape[0], _dp(out))
    return out


def pop_series(coef: np.ndarray, N0: np.ndarray, Ebar: np.ndarray, dP: np.ndarray) -> np.ndarray:
    coef = np.ascontiguousarray(coef, dtype=np.float64)
    N = np.ascontiguousarray(N0, dtype=np.float64).copy()
    Ebar = np.ascontiguousarray(Ebar, dtype=np.float64)
    dP = np.ascontiguousarray(dP, dtype=np.float64)
    out = np.empty((Ebar.shape[0], 4))
    lib().orc_pop_series(_dp(coef), _dp(N), _dp(Ebar), _dp(dP), Ebar.shape[0], _dp(out))
    return out


def _pack_args(box, diam, centres):
    box = np.ascontiguousarray(box, dtype=np.float64).reshape(3)
    diam = np.ascontiguousarray(diam, dtype=np.float64).reshape(-1)
    x = np.array(centres, dtype=np.float64, order="C").reshape(diam.shape[0], 3)
    return box, diam, x


def pack_md(box, diam, centres, *, s0: float = 0.5, stages: int = 50, iters: int = 20,
            final_iters: int = 500, eta: float = 0.1) -> np.ndarray:
    """Soft-sphere compression packing (pack_oracle.c): the centres after the
    schedule, as a new (n, 3) array."""
    box, diam, x = _pack_args(box, diam, centres)
    rc = lib().orc_pack_md(diam.shape[0], _dp(box), _dp(diam), _dp(x), s0, stages, iters, final_iters, eta)
    if rc != 0:
        raise ValueError("orc_pack_md: bad arguments")
    return x


def pack_energy(box, diam, centres, s: float = 1.0):
    """(U_s, largest overlap) of a configuration at scale s."""
    box, diam, x = _pack_args(box, diam, centres)
    out = np.zeros(2)
    lib().orc_pack_energy(diam.shape[0], _dp(box), _dp(diam), _dp(x), s, _dp(out))
    return float(out[0]), float(out[1])
