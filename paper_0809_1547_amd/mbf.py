"""ctypes binding of the C ABI in include/mbf.h.

Argument marshalling only: every step of the simulation runs in the HIP
library ``libmbf.so``.  Importing this module fails loudly when the library
has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# MBF_LIB selects another build of the same library (e.g. a debug build)
LIB_PATH = os.environ.get("MBF_LIB") or os.path.join(HERE, "libmbf.so")

MBF_OK, MBF_EINVAL, MBF_ECFL, MBF_ENOMEM, MBF_EHIP, MBF_ENONFINITE, MBF_ESTATE, MBF_ENODEV = \
    0, -1, -2, -3, -4, -5, -6, -7
MBF_PEC, MBF_MUR1, MBF_ABSORB = 0, 1, 2
MBF_INIT_GROUND, MBF_INIT_PREPUMPED = 0, 1
MBF_FP32, MBF_FP64 = 0, 1
MBF_MEM_HOST, MBF_MEM_DEVICE = 0, 1
MBF_FLAG_FROZEN_POP = 1
MBF_EX, MBF_EY, MBF_EZ, MBF_HX, MBF_HY, MBF_HZ = range(6)
MBF_PX, MBF_PPREVX, MBF_N1X, MBF_N2X, MBF_N3X = 6, 9, 12, 15, 18
MBF_NFIELDS = 21
(MBF_C_DT, MBF_C_S, MBF_C_A, MBF_C_B, MBF_C_CK, MBF_C_CF, MBF_C_BETA, MBF_C_DT32, MBF_C_DT21,
 MBF_C_DT10, MBF_C_DTWP, MBF_C_NA, MBF_C_COUNT) = range(13)

_ERRNAMES = {MBF_EINVAL: "MBF_EINVAL", MBF_ECFL: "MBF_ECFL", MBF_ENOMEM: "MBF_ENOMEM",
             MBF_EHIP: "MBF_EHIP", MBF_ENONFINITE: "MBF_ENONFINITE", MBF_ESTATE: "MBF_ESTATE",
             MBF_ENODEV: "MBF_ENODEV"}


class MbfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class mbf_config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("boundary", C.c_int32 * 3),
        ("precision", C.c_int32), ("noise", C.c_int32), ("flags", C.c_int32),
        ("reserved0", C.c_int32),
        ("dx", C.c_double), ("courant", C.c_double),
        ("lambda0", C.c_double), ("dlambda", C.c_double),
        ("tau32", C.c_double), ("tau21", C.c_double), ("tau10", C.c_double),
        ("Wp", C.c_double), ("N_ref", C.c_double), ("E_ref", C.c_double),
        ("E_sp", C.c_double),
        ("seed", C.c_uint64), ("realization", C.c_uint32), ("reserved1", C.c_int32),
        ("energy_history", C.c_int64),
        ("absorb_cells", C.c_int32), ("absorb_order", C.c_int32), ("absorb_rate", C.c_double),
    ]


class mbf_tuning(C.Structure):
    _fields_ = [("variant", C.c_int32), ("tile_y", C.c_int32), ("zseg", C.c_int32),
                ("xcd_remap", C.c_int32), ("group_mb", C.c_int32)]


class mbf_pack_params(C.Structure):
    _fields_ = [("s0", C.c_double), ("stages", C.c_int32), ("iters", C.c_int32),
                ("final_iters", C.c_int32), ("pad", C.c_int32), ("eta", C.c_double)]


class mbf_spec_stats(C.Structure):
    _fields_ = [("total", C.c_double), ("peak_omega", C.c_double), ("peak_value", C.c_double),
                ("mean_omega", C.c_double), ("std_omega", C.c_double), ("fit_center", C.c_double),
                ("fit_sigma", C.c_double), ("fit_amplitude", C.c_double),
                ("peak_bin", C.c_int32), ("fit_lo", C.c_int32), ("fit_hi", C.c_int32),
                ("fit_ok", C.c_int32)]


MBF_VARIANT_TWO_PASS, MBF_VARIANT_FUSED, MBF_VARIANT_TWO_PASS_SPLIT, MBF_VARIANT_FUSED_LDS = 0, 1, 2, 3
MBF_VARIANT_FUSED_PERSISTENT = 4
_VARIANTS = {"two_pass": MBF_VARIANT_TWO_PASS, "fused": MBF_VARIANT_FUSED,
             "two_pass_split": MBF_VARIANT_TWO_PASS_SPLIT, "fused_lds": MBF_VARIANT_FUSED_LDS,
             "fused_persistent": MBF_VARIANT_FUSED_PERSISTENT}


def _load():
    # torch ships its own HIP runtime under the same soname; load it first so
    # that both torch and this library bind to one runtime in the process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the library has no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    P, I, I64, D, VP = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_void_p
    dp = C.POINTER(C.c_double)
    sigs = {
        "mbf_version": (C.c_char_p, []),
        "mbf_global_error": (C.c_char_p, []),
        "mbf_last_error": (C.c_char_p, [P]),
        "mbf_config_default": (I, [C.POINTER(mbf_config), I, I, I]),
        "mbf_create": (I, [C.POINTER(mbf_config), VP, C.POINTER(P)]),
        "mbf_destroy": (None, [P]),
        "mbf_coefficients": (I, [P, dp, I]),
        "mbf_set_material": (I, [P, VP, VP, I]),
        "mbf_set_pump": (I, [P, D, I]),
        "mbf_add_point_source": (I, [P, I, I, I, I, D, D, D, D]),
        "mbf_set_probes": (I, [P, VP, I, VP, I, I]),
        "mbf_set_loss_box": (I, [P, I, I, I, I, I, I]),
        "mbf_step": (I, [P, I64]),
        "mbf_sync": (I, [P]),
        "mbf_step_index": (I, [P, C.POINTER(C.c_int64)]),
        "mbf_read_energy": (I, [P, dp, dp]),
        "mbf_read_energy_history": (I, [P, dp, I64, C.POINTER(C.c_int64)]),
        "mbf_read_spectrum": (I, [P, dp]),
        "mbf_read_loss": (I, [P, dp]),
        "mbf_read_field": (I, [P, I, VP, I]),
        "mbf_write_field": (I, [P, I, VP, I]),
        "mbf_state_size": (I, [P, C.POINTER(C.c_size_t)]),
        "mbf_save_state": (I, [P, VP, C.c_size_t]),
        "mbf_load_state": (I, [P, VP, C.c_size_t]),
        "mbf_set_tuning": (I, [P, C.POINTER(mbf_tuning)]),
        "mbf_get_tuning": (I, [P, C.POINTER(mbf_tuning)]),
        "mbf_step_timed": (I, [P, I64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "mbf_step_bytes": (I, [P, C.POINTER(C.c_double)]),
        "mbf_batch_create": (I, [C.POINTER(mbf_config), I, VP, C.POINTER(P)]),
        "mbf_batch_destroy": (None, [P]),
        "mbf_batch_last_error": (C.c_char_p, [P]),
        "mbf_batch_size": (I, [P]),
        "mbf_batch_member": (I, [P, I, C.POINTER(P)]),
        "mbf_batch_set_tuning": (I, [P, C.POINTER(mbf_tuning)]),
        "mbf_batch_get_tuning": (I, [P, C.POINTER(mbf_tuning)]),
        "mbf_batch_step": (I, [P, I64]),
        "mbf_batch_sync": (I, [P]),
        "mbf_batch_step_timed": (I, [P, I64, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
        "mbf_batch_step_bytes": (I, [P, C.POINTER(C.c_double)]),
        "mbf_autotune": (I, [P, I, C.POINTER(mbf_tuning)]),
        "mbf_adjoint_run": (I, [P, I64, I, VP, I, dp, dp]),
        "mbf_batch_autotune": (I, [P, I, C.POINTER(mbf_tuning)]),
        "mbf_spectrum_stats": (I, [P, D, C.POINTER(mbf_spec_stats)]),
        "mbf_spectral_stats": (I, [VP, I, I, VP, D, I, VP, C.POINTER(mbf_spec_stats)]),
        "mbf_spectral_stats_noalloc": (I, [VP, I, I, VP, D, VP, VP]),
        "mbf_batch_spectrum_stats": (I, [P, D, C.POINTER(mbf_spec_stats)]),
        "mbf_spectrum_peaks": (I, [P, D, I, VP, C.POINTER(C.c_int)]),
        "mbf_spectral_peaks": (I, [VP, I, I, D, I, I, VP, VP, C.POINTER(C.c_int)]),
        "mbf_add_cw_source": (I, [P, I, I, I, I, D, D, D]),
        "mbf_set_plane_monitor": (I, [P, I]),
        "mbf_reset_plane_monitor": (I, [P]),
        "mbf_read_plane_monitor": (I, [P, dp, C.POINTER(C.c_int64)]),
        "mbf_gp_solve": (I, [VP, I, I, D, I, D, I, VP, VP, VP, VP]),
        "mbf_gp_eigenvalue": (D, [D, D]),
        "mbf_gp_threshold": (D, [D]),
        "mbf_pack_md": (I, [I, dp, VP, VP, C.POINTER(mbf_pack_params), I, VP, dp, dp]),
        "mbf_kappa_fit": (I, [dp, dp, I, D, D, I, D, I, D, VP, dp, dp]),
        "mbf_growth_threshold": (I, [VP, I, I64, I64, I64, dp, I, VP, dp, dp]),
        "mbf_batch_growth_threshold": (I, [P, I64, I64, dp, dp]),
        "mbf_knee_fit": (I, [VP, VP, I, I, VP, dp]),
    }
    for name, (res, args) in sigs.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


lib = _load()
EXPORTED = [
    "mbf_version", "mbf_global_error", "mbf_last_error", "mbf_config_default", "mbf_create",
    "mbf_destroy", "mbf_coefficients", "mbf_set_material", "mbf_set_pump",
    "mbf_add_point_source", "mbf_set_probes", "mbf_set_loss_box", "mbf_step", "mbf_sync",
    "mbf_step_index", "mbf_read_energy", "mbf_read_energy_history", "mbf_read_spectrum",
    "mbf_read_loss", "mbf_read_field", "mbf_write_field", "mbf_state_size", "mbf_save_state",
    "mbf_load_state", "mbf_set_tuning", "mbf_get_tuning", "mbf_step_timed", "mbf_step_bytes",
    "mbf_batch_create", "mbf_batch_destroy", "mbf_batch_last_error", "mbf_batch_size",
    "mbf_batch_member", "mbf_batch_set_tuning", "mbf_batch_get_tuning", "mbf_batch_step",
    "mbf_batch_sync", "mbf_batch_step_timed", "mbf_batch_step_bytes", "mbf_autotune",
    "mbf_batch_autotune", "mbf_adjoint_run", "mbf_spectrum_stats", "mbf_spectral_stats",
    "mbf_batch_spectrum_stats", "mbf_spectrum_peaks", "mbf_spectral_peaks", "mbf_add_cw_source",
    "mbf_set_plane_monitor", "mbf_reset_plane_monitor", "mbf_read_plane_monitor", "mbf_gp_solve",
    "mbf_gp_eigenvalue", "mbf_gp_threshold", "mbf_pack_md", "mbf_spectral_stats_noalloc",
    "mbf_kappa_fit", "mbf_growth_threshold", "mbf_batch_growth_threshold", "mbf_knee_fit",
]


def _check(rc: int, h=None):
    if rc != MBF_OK:
        msg = (lib.mbf_last_error(h) if h else lib.mbf_global_error()) or b""
        raise MbfError(rc, msg.decode(errors="replace"))


def _bcheck(rc: int, b):
    if rc != MBF_OK:
        msg = lib.mbf_batch_last_error(b) or b""
        raise MbfError(rc, msg.decode(errors="replace"))


# ------------------------------------------------------------ raw ABI names

def mbf_version() -> str:
    return lib.mbf_version().decode()


def mbf_config_default(nx: int, ny: int, nz: int) -> mbf_config:
    cfg = mbf_config()
    _check(lib.mbf_config_default(C.byref(cfg), nx, ny, nz))
    return cfg


def mbf_create(cfg: mbf_config, stream: Optional[int] = None) -> int:
    h = C.c_void_p()
    _check(lib.mbf_create(C.byref(cfg), C.c_void_p(stream or 0), C.byref(h)))
    return h.value


def mbf_destroy(h: int) -> None:
    lib.mbf_destroy(h)


def mbf_coefficients(h: int) -> np.ndarray:
    out = np.zeros(MBF_C_COUNT)
    _check(lib.mbf_coefficients(h, out.ctypes.data_as(C.POINTER(C.c_double)), MBF_C_COUNT), h)
    return out


def _ptr_kind(a) -> Tuple[int, int, object]:
    """(address, mem_kind, keep-alive) for a numpy array or a device tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data, MBF_MEM_HOST, a
    if hasattr(a, "data_ptr") and getattr(a, "is_cuda", False):
        return a.data_ptr(), MBF_MEM_DEVICE, a
    if hasattr(a, "data_ptr"):
        return a.data_ptr(), MBF_MEM_HOST, a
    raise TypeError("expected a numpy array or a torch tensor")


def mbf_set_material(h: int, eps_r, gain) -> None:
    if isinstance(eps_r, np.ndarray):
        eps_r = np.ascontiguousarray(eps_r, dtype=np.float32)
        gain = np.ascontiguousarray(gain, dtype=np.uint8)
    pe, ke, _a = _ptr_kind(eps_r)
    pg, kg, _b = _ptr_kind(gain)
    if ke != kg:
        raise ValueError("eps_r and gain must live in the same memory")
    _check(lib.mbf_set_material(h, pe, pg, ke), h)


def mbf_set_pump(h: int, Na: float, init: int = MBF_INIT_PREPUMPED) -> None:
    _check(lib.mbf_set_pump(h, float(Na), int(init)), h)


def mbf_add_point_source(h, comp, i, j, k, amp=1.0, lambda_s=532e-9, tau_p=1e-15, t0=4e-15):
    _check(lib.mbf_add_point_source(h, comp, i, j, k, amp, lambda_s, tau_p, t0), h)


def mbf_set_probes(h: int, sites: np.ndarray, omega: np.ndarray, decim: int = 32) -> None:
    sites = np.ascontiguousarray(sites, dtype=np.int32).reshape(-1, 4)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    _check(lib.mbf_set_probes(h, sites.ctypes.data, sites.shape[0], omega.ctypes.data,
                              omega.shape[0], decim), h)


def mbf_set_loss_box(h: int, lo: Sequence[int], hi: Sequence[int]) -> None:
    _check(lib.mbf_set_loss_box(h, *lo, *hi), h)


def mbf_step(h: int, n: int) -> None:
    _check(lib.mbf_step(h, int(n)), h)


def mbf_sync(h: int) -> None:
    _check(lib.mbf_sync(h), h)


def mbf_step_index(h: int) -> int:
    v = C.c_int64()
    _check(lib.mbf_step_index(h, C.byref(v)), h)
    return v.value


def mbf_read_energy(h: int) -> Tuple[float, float]:
    a, b = C.c_double(), C.c_double()
    _check(lib.mbf_read_energy(h, C.byref(a), C.byref(b)), h)
    return a.value, b.value


def mbf_read_energy_history(h: int, cap: int) -> np.ndarray:
    out = np.zeros(max(cap, 1))
    cnt = C.c_int64()
    _check(lib.mbf_read_energy_history(h, out.ctypes.data_as(C.POINTER(C.c_double)), cap,
                                       C.byref(cnt)), h)
    return out[:min(cnt.value, cap)]


def mbf_read_spectrum(h: int, n_probes: int, n_freq: int) -> np.ndarray:
    out = np.zeros((n_probes, n_freq, 2))
    _check(lib.mbf_read_spectrum(h, out.ctypes.data_as(C.POINTER(C.c_double))), h)
    return out[..., 0] + 1j * out[..., 1]


def _stats_dict(o: mbf_spec_stats) -> dict:
    return {name: getattr(o, name) for name, _ in mbf_spec_stats._fields_}


def mbf_spectrum_stats(h: int, level: float = 0.5) -> dict:
    o = mbf_spec_stats()
    _check(lib.mbf_spectrum_stats(h, float(level), C.byref(o)), h)
    return _stats_dict(o)


def mbf_spectral_stats(spec, omega, level: float = 0.5, stream: Optional[int] = None) -> dict:
    """Statistics of caller amplitudes: spec is (n_probes, n_freq) complex128
    (numpy) or (n_probes, n_freq, 2) float64 (numpy or a device tensor, re/im
    interleaved); omega (n_freq,) float64 in the same memory."""
    if isinstance(spec, np.ndarray) and np.iscomplexobj(spec):
        spec = np.ascontiguousarray(np.stack([spec.real, spec.imag], axis=-1), dtype=np.float64)
    if isinstance(spec, np.ndarray):
        spec = np.ascontiguousarray(spec, dtype=np.float64)
        omega = np.ascontiguousarray(omega, dtype=np.float64)
    if tuple(spec.shape[-1:]) != (2,) or len(spec.shape) != 3 or omega.shape[0] != spec.shape[1]:
        raise ValueError("spec must be (n_probes, n_freq, 2) and omega (n_freq,)")
    ps, ks, _a = _ptr_kind(spec)
    pw, kw, _b = _ptr_kind(omega)
    if ks != kw:
        raise ValueError("spec and omega must live in the same memory")
    o = mbf_spec_stats()
    _check(lib.mbf_spectral_stats(ps, spec.shape[0], spec.shape[1], pw, float(level), ks,
                                  C.c_void_p(stream or 0), C.byref(o)))
    return _stats_dict(o)


def mbf_spectral_stats_noalloc(spec, omega, out, level: float = 0.5, stream: Optional[int] = None) -> None:
    """mbf_spectral_stats with nothing allocated: spec (n_probes, n_freq, 2)
    float64, omega (n_freq,) float64 and out (a device buffer of at least
    ctypes.sizeof(mbf_spec_stats) bytes) are device tensors; the work is
    queued on `stream` and out holds the statistics once the stream reaches
    it (``spec_stats_from_device`` reads them)."""
    if len(spec.shape) != 3 or spec.shape[-1] != 2 or omega.shape[0] != spec.shape[1]:
        raise ValueError("spec must be (n_probes, n_freq, 2) and omega (n_freq,)")
    if out.numel() * out.element_size() < C.sizeof(mbf_spec_stats):
        raise ValueError("out is smaller than mbf_spec_stats")
    for a in (spec, omega, out):
        if not getattr(a, "is_cuda", False) or not a.is_contiguous():
            raise ValueError("spec, omega and out must be contiguous device tensors")
    _check(lib.mbf_spectral_stats_noalloc(spec.data_ptr(), spec.shape[0], spec.shape[1], omega.data_ptr(),
                                          float(level), C.c_void_p(stream or 0), C.c_void_p(out.data_ptr())))


def spec_stats_from_device(out) -> dict:
    """The statistics held in a device buffer written by mbf_spectral_stats_noalloc."""
    raw = out.reshape(-1).view(__import__("torch").uint8)[:C.sizeof(mbf_spec_stats)].cpu().numpy().tobytes()
    return _stats_dict(mbf_spec_stats.from_buffer_copy(raw))


def mbf_spectrum_peaks(h: int, min_rel: float = 0.1, max_peaks: int = 16) -> list:
    bins = np.zeros(max_peaks, dtype=np.int32)
    cnt = C.c_int()
    _check(lib.mbf_spectrum_peaks(h, float(min_rel), int(max_peaks), bins.ctypes.data, C.byref(cnt)), h)
    return [int(b) for b in bins[:cnt.value]]


def mbf_spectral_peaks(spec, min_rel: float = 0.1, max_peaks: int = 16, stream: Optional[int] = None) -> list:
    """Peaks of caller amplitudes (layouts as mbf_spectral_stats)."""
    if isinstance(spec, np.ndarray) and np.iscomplexobj(spec):
        spec = np.ascontiguousarray(np.stack([spec.real, spec.imag], axis=-1), dtype=np.float64)
    if isinstance(spec, np.ndarray):
        spec = np.ascontiguousarray(spec, dtype=np.float64)
    if len(spec.shape) != 3 or spec.shape[-1] != 2:
        raise ValueError("spec must be (n_probes, n_freq, 2)")
    ps, ks, _a = _ptr_kind(spec)
    bins = np.zeros(max_peaks, dtype=np.int32)
    cnt = C.c_int()
    _check(lib.mbf_spectral_peaks(ps, spec.shape[0], spec.shape[1], float(min_rel), int(max_peaks), ks,
                                  C.c_void_p(stream or 0), bins.ctypes.data, C.byref(cnt)))
    return [int(b) for b in bins[:cnt.value]]


def mbf_add_cw_source(h, comp, i, j, k, amp=1.0, lambda_s=586.5e-9, t_ramp=20e-15):
    _check(lib.mbf_add_cw_source(h, comp, i, j, k, amp, lambda_s, t_ramp), h)


def mbf_set_plane_monitor(h: int, k: int) -> None:
    _check(lib.mbf_set_plane_monitor(h, int(k)), h)


def mbf_reset_plane_monitor(h: int) -> None:
    _check(lib.mbf_reset_plane_monitor(h), h)


def mbf_read_plane_monitor(h: int, nx: int, ny: int) -> Tuple[np.ndarray, int]:
    out = np.zeros((ny, nx))
    cnt = C.c_int64()
    _check(lib.mbf_read_plane_monitor(h, out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(cnt)), h)
    return out, cnt.value


GP_STATS = ("N", "w", "peak", "phi_max", "residual", "newton_steps", "converged")


def mbf_gp_solve(E, M: int = 1023, L: float = 12.0, n_nu: int = 512, dnu: float = 0.02,
                 stream: Optional[int] = None) -> dict:
    """Bound states of -phi'' + tau^2 phi + phi^3 = E phi for every E (> 1):
    {"phi": (n_E, M), "spec": (n_E, n_nu), "tau": (M,), "nu": (n_nu,), and
    one (n_E,) array per statistic of GP_STATS}."""
    E = np.ascontiguousarray(np.atleast_1d(E), dtype=np.float64)
    nE = E.shape[0]
    phi = np.zeros((nE, M))
    spec = np.zeros((nE, n_nu))
    st = np.zeros((nE, len(GP_STATS)))
    _check(lib.mbf_gp_solve(E.ctypes.data, nE, int(M), float(L), int(n_nu), float(dnu), MBF_MEM_HOST,
                            C.c_void_p(stream or 0), phi.ctypes.data, spec.ctypes.data, st.ctypes.data))
    h = 2.0 * L / (M + 1)
    out = {"phi": phi, "spec": spec, "tau": -L + h * np.arange(1, M + 1), "nu": dnu * np.arange(n_nu)}
    for q, name in enumerate(GP_STATS):
        out[name] = st[:, q]
    return out


def mbf_kappa_fit(Na, W, N_th: float, t_g: float, M: int = 1023, L: float = 14.0, n_nu: int = 512,
                  dnu: float = 0.02, stream: Optional[int] = None):
    """(kappa, model waists) of the ST-law linewidth fit to waists W (Hz) at
    pump levels Na (m^-3, above N_th)."""
    Na = np.ascontiguousarray(np.atleast_1d(Na), dtype=np.float64)
    W = np.ascontiguousarray(np.atleast_1d(W), dtype=np.float64)
    if Na.shape != W.shape:
        raise ValueError("Na and W must have the same length")
    k = C.c_double()
    Wf = np.zeros_like(W)
    _check(lib.mbf_kappa_fit(Na.ctypes.data_as(C.POINTER(C.c_double)), W.ctypes.data_as(C.POINTER(C.c_double)),
                             Na.shape[0], float(N_th), float(t_g), int(M), float(L), int(n_nu), float(dnu),
                             C.c_void_p(stream or 0), C.byref(k), Wf.ctypes.data_as(C.POINTER(C.c_double))))
    return k.value, Wf


KNEE_FIELDS = ("knee", "split", "aL", "bL", "aR", "bR", "sse")


def mbf_knee_fit(x, y, stream: Optional[int] = None) -> dict:
    """Two-line knee of y against x (numpy arrays or device tensors, float64,
    x increasing): dict of KNEE_FIELDS."""
    if isinstance(x, np.ndarray) or not getattr(x, "is_cuda", False):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(-1))
    if x.shape[0] != y.shape[0]:
        raise ValueError("x and y must have the same length")
    px, kx, _a = _ptr_kind(x)
    py, ky, _b = _ptr_kind(y)
    if kx != ky:
        raise ValueError("x and y must live in the same memory")
    out = np.zeros(7)
    _check(lib.mbf_knee_fit(px, py, int(x.shape[0]), kx, C.c_void_p(stream or 0),
                            out.ctypes.data_as(C.POINTER(C.c_double))))
    d = dict(zip(KNEE_FIELDS, (float(v) for v in out)))
    d["split"] = int(d["split"])
    return d


def mbf_growth_threshold(hist, Na, n0: int, n1: int, stream: Optional[int] = None):
    """(rates, (a, b, N_th)) of energy histories hist (n_runs, stride): numpy
    or a device tensor (float64, contiguous); Na host values (m^-3)."""
    if isinstance(hist, np.ndarray):
        hist = np.ascontiguousarray(hist, dtype=np.float64)
    if len(hist.shape) != 2:
        raise ValueError("hist must be (n_runs, stride)")
    ph, kh, _keep = _ptr_kind(hist)
    Na = np.ascontiguousarray(np.atleast_1d(Na), dtype=np.float64)
    rates = np.zeros(hist.shape[0])
    fit = np.zeros(3)
    _check(lib.mbf_growth_threshold(ph, hist.shape[0], hist.shape[1], int(n0), int(n1),
                                    Na.ctypes.data_as(C.POINTER(C.c_double)), kh, C.c_void_p(stream or 0),
                                    rates.ctypes.data_as(C.POINTER(C.c_double)),
                                    fit.ctypes.data_as(C.POINTER(C.c_double))))
    return rates, tuple(fit)


def mbf_pack_md(box, diam, centres, *, s0: float = 0.5, stages: int = 100, iters: int = 20,
                final_iters: int = 1000, eta: float = 0.15, stream: Optional[int] = None):
    """Soft-sphere compression packing of n spheres in the box.  diam (n,) and
    centres (n, 3): numpy arrays (the packed centres come back as a new array)
    or device tensors (float64, contiguous; centres are packed in place).
    Returns (centres, energy U_1, largest overlap)."""
    prm = mbf_pack_params(float(s0), int(stages), int(iters), int(final_iters), 0, float(eta))
    b = (C.c_double * 3)(*[float(v) for v in np.asarray(box, dtype=np.float64).reshape(3)])
    if isinstance(diam, np.ndarray) or not getattr(diam, "is_cuda", False):
        diam = np.ascontiguousarray(np.asarray(diam, dtype=np.float64).reshape(-1))
        centres = np.array(np.asarray(centres, dtype=np.float64).reshape(-1, 3), order="C")
        n = diam.shape[0]
        if centres.shape[0] != n:
            raise ValueError("centres must be (n, 3) for n diameters")
        pd, pc, kind = diam.ctypes.data, centres.ctypes.data, MBF_MEM_HOST
    else:
        import torch
        if diam.dtype != torch.float64 or centres.dtype != torch.float64 or not centres.is_cuda:
            raise ValueError("device diameters and centres must both be float64 device tensors")
        if not (diam.is_contiguous() and centres.is_contiguous()) or tuple(centres.shape) != (diam.shape[0], 3):
            raise ValueError("centres must be a contiguous (n, 3) tensor for n contiguous diameters")
        n = diam.shape[0]
        pd, pc, kind = diam.data_ptr(), centres.data_ptr(), MBF_MEM_DEVICE
    e, m = C.c_double(), C.c_double()
    _check(lib.mbf_pack_md(int(n), b, pd, pc, C.byref(prm), kind, C.c_void_p(stream or 0), C.byref(e), C.byref(m)))
    return centres, e.value, m.value


def mbf_gp_eigenvalue(p: float, kappa: float) -> float:
    return lib.mbf_gp_eigenvalue(float(p), float(kappa))


def mbf_gp_threshold(kappa: float) -> float:
    return lib.mbf_gp_threshold(float(kappa))


def mbf_read_loss(h: int) -> float:
    v = C.c_double()
    _check(lib.mbf_read_loss(h, C.byref(v)), h)
    return v.value


def mbf_read_field(h: int, field_id: int, dst) -> None:
    p, kind, _k = _ptr_kind(dst)
    _check(lib.mbf_read_field(h, field_id, p, kind), h)


def mbf_write_field(h: int, field_id: int, src) -> None:
    p, kind, _k = _ptr_kind(src)
    _check(lib.mbf_write_field(h, field_id, p, kind), h)


def mbf_state_size(h: int) -> int:
    v = C.c_size_t()
    _check(lib.mbf_state_size(h, C.byref(v)), h)
    return v.value


def mbf_save_state(h: int) -> bytearray:
    buf = bytearray(mbf_state_size(h))
    arr = (C.c_char * len(buf)).from_buffer(buf)
    _check(lib.mbf_save_state(h, C.addressof(arr), len(buf)), h)
    return buf


def mbf_load_state(h: int, buf: bytes) -> None:
    b = bytearray(buf)
    arr = (C.c_char * len(b)).from_buffer(b)
    _check(lib.mbf_load_state(h, C.addressof(arr), len(b)), h)


def mbf_set_tuning(h: int, variant: int = MBF_VARIANT_TWO_PASS, tile_y: int = 4, zseg: int = 0,
                   xcd_remap: int = 2, group_mb: int = 0) -> None:
    t = mbf_tuning(variant, tile_y, zseg, xcd_remap, group_mb)
    _check(lib.mbf_set_tuning(h, C.byref(t)), h)


def mbf_get_tuning(h: int) -> mbf_tuning:
    t = mbf_tuning()
    _check(lib.mbf_get_tuning(h, C.byref(t)), h)
    return t


def mbf_step_timed(h: int, n: int) -> Tuple[Tuple[float, float], int]:
    """((ms of the first field kernel, ms of the second), steps)."""
    ms = (C.c_double * 2)()
    cnt = C.c_int64()
    _check(lib.mbf_step_timed(h, int(n), ms, C.byref(cnt)), h)
    return (ms[0], ms[1]), cnt.value


def mbf_step_bytes(h: int) -> Tuple[float, float, float]:
    """Algorithmic bytes of (the step, the first field kernel, the second)."""
    b = (C.c_double * 3)()
    _check(lib.mbf_step_bytes(h, b), h)
    return b[0], b[1], b[2]


def _tuning_dict(t: mbf_tuning) -> dict:
    return dict(variant={v: k for k, v in _VARIANTS.items()}[t.variant], tile_y=t.tile_y,
                zseg=t.zseg, xcd_remap=t.xcd_remap, group_mb=t.group_mb)


def mbf_autotune(h: int, budget_ms: int = 2000) -> dict:
    t = mbf_tuning()
    _check(lib.mbf_autotune(h, int(budget_ms), C.byref(t)), h)
    return _tuning_dict(t)


def mbf_batch_autotune(b: int, budget_ms: int = 2000) -> dict:
    t = mbf_tuning()
    _bcheck(lib.mbf_batch_autotune(b, int(budget_ms), C.byref(t)), b)
    return _tuning_dict(t)


def mbf_adjoint_run(h: int, nsteps: int, K: int, grad_eps) -> Tuple[float, float]:
    """Run the loss-box adjoint over nsteps from the pump; grad_eps (caller
    owned: a float64 numpy array or device tensor of nx*ny*nz values) receives
    dL/d eps_r.  Returns (L, dL/dN_a)."""
    if isinstance(grad_eps, np.ndarray):
        assert grad_eps.dtype == np.float64 and grad_eps.flags.c_contiguous
    p, kind, _keep = _ptr_kind(grad_eps)
    gna, L = C.c_double(), C.c_double()
    _check(lib.mbf_adjoint_run(h, int(nsteps), int(K), p, kind, C.byref(gna), C.byref(L)), h)
    return L.value, gna.value


def mbf_batch_create(cfgs: Sequence[mbf_config], stream: Optional[int] = None) -> int:
    arr = (mbf_config * len(cfgs))(*cfgs)
    b = C.c_void_p()
    _check(lib.mbf_batch_create(arr, len(cfgs), C.c_void_p(stream or 0), C.byref(b)))
    return b.value


def mbf_batch_destroy(b: int) -> None:
    lib.mbf_batch_destroy(b)


def mbf_batch_size(b: int) -> int:
    return lib.mbf_batch_size(b)


def mbf_batch_member(b: int, r: int) -> int:
    h = C.c_void_p()
    _bcheck(lib.mbf_batch_member(b, r, C.byref(h)), b)
    return h.value


def mbf_batch_set_tuning(b: int, variant: int = MBF_VARIANT_TWO_PASS, tile_y: int = 4, zseg: int = 0,
                         xcd_remap: int = 2, group_mb: int = 0) -> None:
    t = mbf_tuning(variant, tile_y, zseg, xcd_remap, group_mb)
    _bcheck(lib.mbf_batch_set_tuning(b, C.byref(t)), b)


def mbf_batch_get_tuning(b: int) -> mbf_tuning:
    t = mbf_tuning()
    _bcheck(lib.mbf_batch_get_tuning(b, C.byref(t)), b)
    return t


def mbf_batch_step(b: int, n: int) -> None:
    _bcheck(lib.mbf_batch_step(b, int(n)), b)


def mbf_batch_sync(b: int) -> None:
    _bcheck(lib.mbf_batch_sync(b), b)


def mbf_batch_step_timed(b: int, n: int) -> Tuple[Tuple[float, float], int]:
    ms = (C.c_double * 2)()
    cnt = C.c_int64()
    _bcheck(lib.mbf_batch_step_timed(b, int(n), ms, C.byref(cnt)), b)
    return (ms[0], ms[1]), cnt.value


def mbf_batch_spectrum_stats(b: int, level: float = 0.5) -> list:
    R = mbf_batch_size(b)
    arr = (mbf_spec_stats * R)()
    _bcheck(lib.mbf_batch_spectrum_stats(b, float(level), arr), b)
    return [_stats_dict(o) for o in arr]


def mbf_batch_step_bytes(b: int) -> Tuple[float, float, float]:
    x = (C.c_double * 3)()
    _bcheck(lib.mbf_batch_step_bytes(b, x), b)
    return x[0], x[1], x[2]


# ------------------------------------------------------------ convenience

def make_config(n, *, boundary=("pec", "pec", "pec"), precision="fp32", noise=True,
                frozen_pop=False, seed=0, realization=0, energy_history=0, **phys) -> mbf_config:
    """An mbf_config from the workload defaults and keyword overrides."""
    if isinstance(n, int):
        n = (n, n, n)
    if isinstance(boundary, str):
        boundary = (boundary,) * 3
    cfg = mbf_config_default(*n)
    kinds = {"pec": MBF_PEC, "mur": MBF_MUR1, "absorb": MBF_ABSORB}
    for a in range(3):
        cfg.boundary[a] = kinds[boundary[a]]
    cfg.precision = MBF_FP64 if precision == "fp64" else MBF_FP32
    cfg.noise = int(bool(noise))
    cfg.flags = MBF_FLAG_FROZEN_POP if frozen_pop else 0
    cfg.seed = seed
    cfg.realization = realization
    cfg.energy_history = energy_history
    for k, v in phys.items():
        if not hasattr(cfg, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(cfg, k, v)
    return cfg


class Sim:
    """One simulation handle with numpy-friendly accessors."""

    def __init__(self, n, *, stream=None, _cfg=None, _handle=None, **kw):
        cfg = _cfg if _cfg is not None else make_config(n, **kw)
        self.cfg = cfg
        self.n = (cfg.nx, cfg.ny, cfg.nz)
        self.shape = (cfg.nz + 1, cfg.ny + 1, cfg.nx + 1)
        self.dtype = np.float64 if cfg.precision == MBF_FP64 else np.float32
        self._owned = _handle is None
        self.h = mbf_create(cfg, stream) if _handle is None else _handle
        self._np = self._nf = 0

    def close(self):
        if getattr(self, "h", None):
            if self._owned:
                mbf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coefficients(self):
        return mbf_coefficients(self.h)

    def set_material(self, eps, gain):
        mbf_set_material(self.h, eps, gain)

    def set_pump(self, Na, init="prepumped"):
        mbf_set_pump(self.h, Na, MBF_INIT_PREPUMPED if init == "prepumped" else MBF_INIT_GROUND)

    def set_source(self, comp, i, j, k, amp=1.0, lambda_s=532e-9, tau_p=1e-15, t0=4e-15):
        mbf_add_point_source(self.h, comp, i, j, k, amp, lambda_s, tau_p, t0)

    def set_probes(self, sites, omega, decim=32):
        sites = np.asarray(sites).reshape(-1, 4)
        mbf_set_probes(self.h, sites, omega, decim)
        self._np, self._nf = sites.shape[0], len(omega)

    def set_loss_box(self, lo, hi):
        mbf_set_loss_box(self.h, lo, hi)

    def step(self, n):
        mbf_step(self.h, n)

    def sync(self):
        mbf_sync(self.h)

    @property
    def step_index(self):
        return mbf_step_index(self.h)

    def field(self, fid) -> np.ndarray:
        out = np.empty(self.shape, dtype=self.dtype)
        mbf_read_field(self.h, fid, out)
        return out

    def set_field(self, fid, a):
        mbf_write_field(self.h, fid, np.ascontiguousarray(a, dtype=self.dtype))

    def energy(self):
        return mbf_read_energy(self.h)

    def energy_history(self):
        return mbf_read_energy_history(self.h, self.cfg.energy_history)

    def spectrum(self):
        return mbf_read_spectrum(self.h, self._np, self._nf)

    def loss(self):
        return mbf_read_loss(self.h)

    def spectrum_stats(self, level=0.5):
        """Peak, standard deviation and Gaussian fit of the probe-summed
        power spectrum (dict of the mbf_spec_stats fields)."""
        return mbf_spectrum_stats(self.h, level)

    def spectrum_peaks(self, min_rel=0.1, max_peaks=16):
        """Bins of the peaks of the probe-summed power spectrum, largest first."""
        return mbf_spectrum_peaks(self.h, min_rel, max_peaks)

    def set_cw_source(self, comp, i, j, k, amp=1.0, lambda_s=586.5e-9, t_ramp=20e-15):
        mbf_add_cw_source(self.h, comp, i, j, k, amp, lambda_s, t_ramp)

    def set_plane_monitor(self, k):
        mbf_set_plane_monitor(self.h, k)

    def reset_plane_monitor(self):
        mbf_reset_plane_monitor(self.h)

    def plane_monitor(self):
        """(sums of the energy density of the monitored plane (ny, nx), steps)."""
        return mbf_read_plane_monitor(self.h, self.cfg.nx, self.cfg.ny)

    def set_tuning(self, variant="two_pass", tile_y=4, zseg=0, xcd_remap=2, group_mb=0):
        mbf_set_tuning(self.h, _VARIANTS[variant], tile_y, zseg, xcd_remap, group_mb)

    def tuning(self):
        return _tuning_dict(mbf_get_tuning(self.h))

    def autotune(self, budget_ms=2000):
        return mbf_autotune(self.h, budget_ms)

    def adjoint_run(self, nsteps, K=50):
        """(L, dL/d eps_r (nz, ny, nx), dL/dN_a) of the loss-box objective over
        nsteps from the pump; leaves the run at step nsteps."""
        g = np.zeros((self.cfg.nz, self.cfg.ny, self.cfg.nx), dtype=np.float64)
        L, gna = mbf_adjoint_run(self.h, nsteps, K, g)
        return L, g, gna

    def step_timed(self, n):
        return mbf_step_timed(self.h, n)

    def step_bytes(self):
        return mbf_step_bytes(self.h)

    def save_state(self):
        return mbf_save_state(self.h)

    def load_state(self, buf):
        mbf_load_state(self.h, buf)


class Batch:
    """A batch of simulations stepped together; `members[r]` is a Sim view of
    member r (owned by the batch)."""

    def __init__(self, configs, stream=None):
        cfgs = [c if isinstance(c, mbf_config) else make_config(**c) for c in configs]
        self.b = mbf_batch_create(cfgs, stream)
        self.members = [Sim(None, _cfg=c, _handle=mbf_batch_member(self.b, r)) for r, c in enumerate(cfgs)]

    def __len__(self):
        return len(self.members)

    def __getitem__(self, r):
        return self.members[r]

    def set_tuning(self, variant="two_pass", tile_y=4, zseg=0, xcd_remap=2, group_mb=0):
        mbf_batch_set_tuning(self.b, _VARIANTS[variant], tile_y, zseg, xcd_remap, group_mb)

    def tuning(self):
        return _tuning_dict(mbf_batch_get_tuning(self.b))

    def autotune(self, budget_ms=2000):
        return mbf_batch_autotune(self.b, budget_ms)

    def step(self, n):
        mbf_batch_step(self.b, n)

    def sync(self):
        mbf_batch_sync(self.b)

    def step_timed(self, n):
        return mbf_batch_step_timed(self.b, n)

    def step_bytes(self):
        return mbf_batch_step_bytes(self.b)

    def spectrum_stats(self, level=0.5):
        """spectrum_stats of every member, in member order."""
        return mbf_batch_spectrum_stats(self.b, level)

    def growth_threshold(self, n0, n1):
        """(rates, (a, b, N_th)) over the members' energy histories."""
        rates = np.zeros(len(self.members))
        fit = np.zeros(3)
        _bcheck(lib.mbf_batch_growth_threshold(self.b, int(n0), int(n1),
                                               rates.ctypes.data_as(C.POINTER(C.c_double)),
                                               fit.ctypes.data_as(C.POINTER(C.c_double))), self.b)
        return rates, tuple(fit)

    def close(self):
        if getattr(self, "b", None):
            for m in self.members:
                m.h = None
            mbf_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
