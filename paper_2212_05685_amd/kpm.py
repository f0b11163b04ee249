"""Thin Python binding of the C ABI in include/kpm.h (argument marshalling only).

Every function here has the name of the C entry point it calls and does no
arithmetic of the method: it checks tensor dtypes/devices/shapes, passes raw
device pointers and the current HIP stream, and raises ``KpmError`` on a
nonzero status.  Tensors are torch tensors on the GPU: real arrays float64,
complex arrays complex128 (interleaved re/im, as the ABI expects).

If libkpm.so is missing, importing this module raises ImportError: there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int32, c_size_t, c_uint64, c_void_p
from dataclasses import dataclass
from typing import Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpm.so")

KPM_OK, KPM_EINVAL, KPM_ENOMEM, KPM_EDEVICE, KPM_EBOUNDS, KPM_ENOTSUP, KPM_EWORKSPACE = 0, -1, -2, -3, -4, -5, -6
KPM_ENOCONV = -7
KPM_ETOOBIG = -8
KPM_SCHED_DEFAULT, KPM_SCHED_TILE_MAJOR, KPM_SCHED_RANGES, KPM_SCHED_STRIPS, KPM_SCHED_STRIP_TILES = -1, 0, 1, 2, 3
KPM_SCHED_BALANCED = 4
KPM_NOALLOC_SCRATCH_BYTES = 64 << 20
KPM_RMFT_STATS_LEN = 520
KPM_RMFT_BISECTION, KPM_RMFT_ILLINOIS = 0, 1
KPM_RMFT_ADJOINT, KPM_RMFT_DIRECT = 0, 1
KPM_FP64, KPM_FP32 = 0, 1
KPM_PROBE_UNIT, KPM_PROBE_DENSE_Z4, KPM_PROBE_COLORED_Z4 = 0, 1, 2
NENT = 19

EXPORTS = (
    "kpm_probe_count", "kpm_build_H", "kpm_build_H_vjp", "kpm_bounds", "kpm_coefficients",
    "kpm_workspace_size", "kpm_moments", "kpm_grand_potential", "kpm_grand_potential_grad",
    "kpm_density_matrix", "kpm_status_read", "kpm_batch_create", "kpm_batch_energy_grad",
    "kpm_batch_destroy", "kpm_set_probe_block", "kpm_profile_begin", "kpm_profile_end",
    "kpm_strerror", "kpm_rmft_update", "kpm_rmft_workspace_size", "kpm_rmft_iterate",
    "kpm_density_matrix_direct", "kpm_moments_doubling", "kpm_ldos", "kpm_build_H_sdw",
    "kpm_rmft_update_sdw", "kpm_rmft_iterate_sdw", "kpm_build_H_sdw_vjp", "kpm_bloch_H", "kpm_gutzwiller_weights", "kpm_supercell_workspace_size",
    "kpm_supercell_ldos", "kpm_moments_noalloc", "kpm_set_schedule", "kpm_set_streams", "kpm_batch_tuning",
    "kpm_batch_streams", "kpm_batch_groups", "kpm_set_batch_groups",
)


class Lattice(ctypes.Structure):
    _fields_ = [("Lx", c_int32), ("Ly", c_int32), ("n_vortex", c_int32)]


class Model(ctypes.Structure):
    _fields_ = [("t", c_double), ("tp", c_double), ("J", c_double), ("mu", c_double)]


class ProbeGroup(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("count", c_int32), ("px", c_int32), ("py", c_int32),
                ("split_nambu", c_int32), ("first", c_int32), ("seed", c_uint64),
                ("weight", c_double)]


class Probes(ctypes.Structure):
    _fields_ = [("groups", POINTER(ProbeGroup)), ("ngroups", c_int32)]


class RmftParams(ctypes.Structure):
    _fields_ = [("doping", c_double), ("mix", c_double), ("tol_n", c_double), ("tol_mu", c_double),
                ("mu_step", c_double), ("tol_residual", c_double), ("max_evals", c_int32),
                ("coef_K", c_int32), ("search", c_int32), ("estimator", c_int32),
                ("anderson", c_int32), ("pad", c_int32)]


class RmftRecord(ctypes.Structure):
    _fields_ = [("mu", c_double), ("nbar", c_double), ("residual", c_double), ("omega", c_double),
                ("evals", c_int32), ("pad", c_int32)]


class KpmError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {strerror(status)} ({status})")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (build it: python paper_2212_05685_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "kpm_probe_count": (c_int32, [POINTER(Lattice), POINTER(Probes)]),
        "kpm_build_H": (c_int32, [POINTER(Lattice), POINTER(Model), P, P, P, P, P]),
        "kpm_build_H_vjp": (c_int32, [POINTER(Lattice), POINTER(Model), P, P, P, P, P, P, P, P]),
        "kpm_build_H_sdw": (c_int32, [POINTER(Lattice), POINTER(Model), P, P, P, P, P, P, P, P]),
        "kpm_bounds": (c_int32, [POINTER(Lattice), P, P, P]),
        "kpm_coefficients": (c_int32, [c_int32, c_double, P, c_int32, P, P]),
        "kpm_workspace_size": (c_size_t, [POINTER(Lattice), c_int32, c_int32, c_int32, c_int32]),
        "kpm_moments": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, c_int32, c_int32,
                                  P, P, c_size_t, P]),
        "kpm_moments_noalloc": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, c_int32, P,
                                          P]),
        "kpm_grand_potential": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, P, c_int32,
                                          c_int32, P, P, P, c_size_t, P]),
        "kpm_grand_potential_grad": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, P,
                                               c_int32, c_int32, P, P, P, c_size_t, P]),
        "kpm_density_matrix": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, P, c_int32,
                                         c_int32, P, P, P, P, P, P, P, P, P, c_size_t, P]),
        "kpm_status_read": (c_int32, [P, POINTER(c_int32), P]),
        "kpm_ldos": (c_int32, [POINTER(Lattice), P, P, c_int32, c_int32, c_int32, c_int32, P, c_int32, P,
                               P, c_size_t, P]),
        "kpm_moments_doubling": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, P, c_int32,
                                           P, P, P, c_size_t, P]),
        "kpm_density_matrix_direct": (c_int32, [POINTER(Lattice), P, P, POINTER(Probes), c_int32, P,
                                                c_int32, P, P, P, c_size_t, P]),
        "kpm_batch_create": (c_int32, [c_int32, POINTER(Lattice), POINTER(Probes), c_int32, c_int32,
                                       c_int32, POINTER(c_void_p)]),
        "kpm_batch_energy_grad": (c_int32, [P, POINTER(c_void_p), POINTER(c_void_p), POINTER(c_void_p),
                                            P, POINTER(c_void_p), c_int32, P]),
        "kpm_batch_destroy": (c_int32, [P]),
        "kpm_set_probe_block": (c_int32, [c_int32]),
        "kpm_set_schedule": (c_int32, [c_int32, c_int32]),
        "kpm_set_streams": (c_int32, [c_int32]),
        "kpm_batch_tuning": (c_int32, [P, P]),
        "kpm_batch_streams": (c_int32, [P]),
        "kpm_batch_groups": (c_int32, [P]),
        "kpm_set_batch_groups": (c_int32, [c_int32]),
        "kpm_profile_begin": (c_int32, [c_int32]),
        "kpm_profile_end": (c_int32, [POINTER(c_double), POINTER(c_int32), POINTER(c_double),
                                      POINTER(c_int32)]),
        "kpm_strerror": (ctypes.c_char_p, [c_int32]),
        "kpm_rmft_update": (c_int32, [POINTER(Lattice), P, c_double, P, P, P, P, P]),
        "kpm_rmft_workspace_size": (c_size_t, [POINTER(Lattice), c_int32, c_int32, c_int32, c_int32]),
        "kpm_rmft_iterate": (c_int32, [POINTER(Lattice), POINTER(Model), POINTER(Probes), c_int32,
                                       c_double, c_int32, c_int32, POINTER(RmftParams), c_int32, P, P,
                                       P, POINTER(c_double), POINTER(RmftRecord), POINTER(c_int32),
                                       P, c_size_t, P]),
        "kpm_rmft_update_sdw": (c_int32, [POINTER(Lattice), P, c_double, P, P, P, P, P, P, P, P]),
        "kpm_rmft_iterate_sdw": (c_int32, [POINTER(Lattice), POINTER(Model), POINTER(Probes), c_int32,
                                           c_double, c_int32, c_int32, POINTER(RmftParams), c_int32, P,
                                           P, P, P, P, P, POINTER(c_double), POINTER(RmftRecord),
                                           POINTER(c_int32), P, c_size_t, P]),
        "kpm_build_H_sdw_vjp": (c_int32, [POINTER(Lattice), POINTER(Model)] + [P] * 14),
        "kpm_bloch_H": (c_int32, [POINTER(Lattice), P, c_double, c_double, P, ctypes.c_int64, P]),
        "kpm_gutzwiller_weights": (c_int32, [POINTER(Lattice), P, P, P, P, P]),
        "kpm_supercell_workspace_size": (c_size_t, [POINTER(Lattice), c_int32]),
        "kpm_supercell_ldos": (c_int32, [POINTER(Lattice), P, c_int32, c_int32, c_int32, c_int32, c_int32,
                                         POINTER(c_int32), c_int32, P, c_int32, c_double, c_double, P, P,
                                         c_int32, P, P, P, c_size_t, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()


def strerror(status: int) -> str:
    return _lib.kpm_strerror(status).decode()


def _check(status: int, where: str) -> None:
    if status != KPM_OK:
        raise KpmError(status, where)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _ptr(t, dtype, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return c_void_p(t.data_ptr())


@dataclass(frozen=True)
class ProbeSpec:
    """One probe group (see kpm_probe_group in include/kpm.h)."""
    kind: int
    count: int
    seed: int = 0
    px: int = 1
    py: int = 1
    split_nambu: int = 0
    first: int = 0
    weight: float = 1.0


def _probes(specs: Sequence[ProbeSpec]):
    arr = (ProbeGroup * len(specs))()
    for k, s in enumerate(specs):
        arr[k] = ProbeGroup(s.kind, s.count, s.px, s.py, s.split_nambu, s.first,
                            s.seed & ((1 << 64) - 1), s.weight)
    pr = Probes(ctypes.cast(arr, POINTER(ProbeGroup)), len(specs))
    pr._keep = arr
    return pr


def lattice(Lx: int, Ly: int, n_vortex: int) -> Lattice:
    return Lattice(Lx, Ly, n_vortex)


def model(t: float, tp: float, J: float, mu: float) -> Model:
    return Model(t, tp, J, mu)


# ---------------------------------------------------------------- entry points
def kpm_probe_count(lat: Lattice, probes: Sequence[ProbeSpec]) -> int:
    r = _lib.kpm_probe_count(ctypes.byref(lat), ctypes.byref(_probes(probes)))
    if r < 0:
        raise KpmError(r, "kpm_probe_count")
    return r


def kpm_build_H(lat, mdl, n, chi, delta, h, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_build_H(ctypes.byref(lat), ctypes.byref(mdl), _ptr(n, torch.float64, N, "n"),
                            _ptr(chi, torch.complex128, 4 * N, "chi"),
                            _ptr(delta, torch.complex128, 4 * N, "delta"),
                            _ptr(h, torch.complex128, NENT * N, "h"), _stream(stream)), "kpm_build_H")


def kpm_build_H_sdw(lat, mdl, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, h, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_build_H_sdw(ctypes.byref(lat), ctypes.byref(mdl),
                                _ptr(n_up, torch.float64, N, "n_up"), _ptr(n_dn, torch.float64, N, "n_dn"),
                                _ptr(chi_up, torch.complex128, 4 * N, "chi_up"),
                                _ptr(chi_dn, torch.complex128, 4 * N, "chi_dn"),
                                _ptr(delta_up, torch.complex128, 4 * N, "delta_up"),
                                _ptr(delta_dn, torch.complex128, 4 * N, "delta_dn"),
                                _ptr(h, torch.complex128, NENT * N, "h"), _stream(stream)), "kpm_build_H_sdw")


def kpm_build_H_sdw_vjp(lat, mdl, theta, rho, grads, stream=None):
    """theta, grads: (n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn) device
    tensors (grads overwritten)."""
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_build_H_sdw_vjp(ctypes.byref(lat), ctypes.byref(mdl), *_spin_ptrs(lat, *theta),
                                    _ptr(rho, torch.complex128, NENT * N, "rho"), *_spin_ptrs(lat, *grads),
                                    _stream(stream)), "kpm_build_H_sdw_vjp")


def kpm_build_H_vjp(lat, mdl, n, chi, delta, rho, dn, dchi, ddelta, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_build_H_vjp(ctypes.byref(lat), ctypes.byref(mdl), _ptr(n, torch.float64, N, "n"),
                                _ptr(chi, torch.complex128, 4 * N, "chi"),
                                _ptr(delta, torch.complex128, 4 * N, "delta"),
                                _ptr(rho, torch.complex128, NENT * N, "rho"),
                                _ptr(dn, torch.float64, N, "dn"),
                                _ptr(dchi, torch.complex128, 4 * N, "dchi"),
                                _ptr(ddelta, torch.complex128, 4 * N, "ddelta"), _stream(stream)),
           "kpm_build_H_vjp")


def kpm_bounds(lat, h, ab, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_bounds(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                           _ptr(ab, torch.float64, 2, "ab"), _stream(stream)), "kpm_bounds")


def kpm_coefficients(M, T, ab, C, K=0, stream=None):
    _check(_lib.kpm_coefficients(M, T, _ptr(ab, torch.float64, 2, "ab"), K,
                                 _ptr(C, torch.float64, M, "C"), _stream(stream)), "kpm_coefficients")


def kpm_workspace_size(lat, R, M, ckpt_k, precision) -> int:
    n = _lib.kpm_workspace_size(ctypes.byref(lat), R, M, ckpt_k, precision)
    if n == 0:
        raise KpmError(KPM_EINVAL, "kpm_workspace_size")
    return int(n)


def kpm_moments(lat, h, ab, probes, M, precision, ckpt_k, mu, ws, stream=None):
    N = lat.Lx * lat.Ly
    R = kpm_probe_count(lat, probes)
    _check(_lib.kpm_moments(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                            _ptr(ab, torch.float64, 2, "ab"), ctypes.byref(_probes(probes)), M,
                            precision, ckpt_k, _ptr(mu, torch.float64, R * M, "mu"),
                            _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)),
           "kpm_moments")


def kpm_moments_noalloc(lat, h, ab, probes, M, precision, mu, stream=None):
    N = lat.Lx * lat.Ly
    R = kpm_probe_count(lat, probes)
    _check(_lib.kpm_moments_noalloc(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                                    _ptr(ab, torch.float64, 2, "ab"), ctypes.byref(_probes(probes)), M,
                                    precision, _ptr(mu, torch.float64, R * M, "mu"), _stream(stream)),
           "kpm_moments_noalloc")


def kpm_grand_potential(lat, h, ab, probes, M, C, precision, ckpt_k, omega, mu, ws, stream=None):
    N = lat.Lx * lat.Ly
    R = kpm_probe_count(lat, probes)
    _check(_lib.kpm_grand_potential(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                                    _ptr(ab, torch.float64, 2, "ab"), ctypes.byref(_probes(probes)),
                                    M, _ptr(C, torch.float64, M, "C"), precision, ckpt_k,
                                    _ptr(omega, torch.float64, 1, "omega"),
                                    _ptr(mu, torch.float64, R * M, "mu"),
                                    _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)),
           "kpm_grand_potential")


def kpm_grand_potential_grad(lat, h, ab, probes, M, C, precision, ckpt_k, omega_bar, rho, ws,
                             stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_grand_potential_grad(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                                         _ptr(ab, torch.float64, 2, "ab"),
                                         ctypes.byref(_probes(probes)), M,
                                         _ptr(C, torch.float64, M, "C"), precision, ckpt_k,
                                         _ptr(omega_bar, torch.float64, 1, "omega_bar"),
                                         _ptr(rho, torch.complex128, NENT * N, "rho"),
                                         _ptr(ws, torch.uint8, None, "ws"), ws.numel(),
                                         _stream(stream)), "kpm_grand_potential_grad")


def kpm_density_matrix(lat, h, ab, probes, M, C, precision, ckpt_k, omega, rho, n_up, n_dn,
                       chi_up, chi_dn, delta_up, delta_dn, ws, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_density_matrix(
        ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"), _ptr(ab, torch.float64, 2, "ab"),
        ctypes.byref(_probes(probes)), M, _ptr(C, torch.float64, M, "C"), precision, ckpt_k,
        _ptr(omega, torch.float64, 1, "omega"), _ptr(rho, torch.complex128, NENT * N, "rho"),
        _ptr(n_up, torch.float64, N, "n_up"), _ptr(n_dn, torch.float64, N, "n_dn"),
        _ptr(chi_up, torch.complex128, 4 * N, "chi_up"), _ptr(chi_dn, torch.complex128, 4 * N, "chi_dn"),
        _ptr(delta_up, torch.complex128, 4 * N, "delta_up"),
        _ptr(delta_dn, torch.complex128, 4 * N, "delta_dn"),
        _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)), "kpm_density_matrix")


def kpm_density_matrix_direct(lat, h, ab, probes, M, C, precision, omega, rho, ws, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_density_matrix_direct(
        ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"), _ptr(ab, torch.float64, 2, "ab"),
        ctypes.byref(_probes(probes)), M, _ptr(C, torch.float64, M, "C"), precision,
        _ptr(omega, torch.float64, 1, "omega"), _ptr(rho, torch.complex128, NENT * N, "rho"),
        _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)), "kpm_density_matrix_direct")


def kpm_moments_doubling(lat, h, ab, probes, M, C, precision, omega, mu, ws, stream=None):
    N = lat.Lx * lat.Ly
    R = kpm_probe_count(lat, probes)
    _check(_lib.kpm_moments_doubling(
        ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"), _ptr(ab, torch.float64, 2, "ab"),
        ctypes.byref(_probes(probes)), M, _ptr(C, torch.float64, M, "C"), precision,
        _ptr(omega, torch.float64, 1, "omega"), _ptr(mu, torch.float64, R * M, "mu"),
        _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)), "kpm_moments_doubling")


def kpm_ldos(lat, h, ab, first, count, M, precision, energies, out, ws, stream=None):
    N = lat.Lx * lat.Ly
    ne = energies.numel()
    _check(_lib.kpm_ldos(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"),
                         _ptr(ab, torch.float64, 2, "ab"), first, count, M, precision,
                         _ptr(energies, torch.float64, ne, "energies"), ne,
                         _ptr(out, torch.float64, count * ne, "out"),
                         _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)), "kpm_ldos")


def kpm_status_read(ws, stream=None) -> int:
    out = c_int32(0)
    _check(_lib.kpm_status_read(_ptr(ws, torch.uint8, None, "ws"), ctypes.byref(out), _stream(stream)),
           "kpm_status_read")
    return out.value


def kpm_set_probe_block(probes_per_thread: int) -> int:
    return int(_lib.kpm_set_probe_block(probes_per_thread))


def kpm_set_streams(n: int) -> int:
    """0 automatic, 1 one stream, 2 halves on two streams (the probes of a single
    lattice; the instances of a batch plan created while it is set); returns the
    previous value."""
    return int(_lib.kpm_set_streams(n))


def kpm_set_schedule(fwd: int, adj: int) -> None:
    _check(_lib.kpm_set_schedule(fwd, adj), "kpm_set_schedule")


def kpm_profile_begin(sample_every: int = 1) -> None:
    _check(_lib.kpm_profile_begin(sample_every), "kpm_profile_begin")


def kpm_profile_end():
    """(forward ms, forward launches, adjoint ms, adjoint launches) since begin."""
    f, a = c_double(0), c_double(0)
    nf, na = c_int32(0), c_int32(0)
    _check(_lib.kpm_profile_end(ctypes.byref(f), ctypes.byref(nf), ctypes.byref(a), ctypes.byref(na)),
           "kpm_profile_end")
    return f.value, nf.value, a.value, na.value


def kpm_strerror(status: int) -> str:
    return strerror(status)


def kpm_rmft_update(lat, rho, mix, n, chi, delta, stats, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_rmft_update(ctypes.byref(lat), _ptr(rho, torch.complex128, NENT * N, "rho"),
                                float(mix), _ptr(n, torch.float64, N, "n"),
                                _ptr(chi, torch.complex128, 4 * N, "chi"),
                                _ptr(delta, torch.complex128, 4 * N, "delta"),
                                _ptr(stats, torch.float64, KPM_RMFT_STATS_LEN, "stats"),
                                _stream(stream)), "kpm_rmft_update")


def _spin_ptrs(lat, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn):
    N = lat.Lx * lat.Ly
    return (_ptr(n_up, torch.float64, N, "n_up"), _ptr(n_dn, torch.float64, N, "n_dn"),
            _ptr(chi_up, torch.complex128, 4 * N, "chi_up"), _ptr(chi_dn, torch.complex128, 4 * N, "chi_dn"),
            _ptr(delta_up, torch.complex128, 4 * N, "delta_up"),
            _ptr(delta_dn, torch.complex128, 4 * N, "delta_dn"))


def kpm_rmft_update_sdw(lat, rho, mix, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn, stats, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_rmft_update_sdw(ctypes.byref(lat), _ptr(rho, torch.complex128, NENT * N, "rho"),
                                    float(mix), *_spin_ptrs(lat, n_up, n_dn, chi_up, chi_dn, delta_up,
                                                            delta_dn),
                                    _ptr(stats, torch.float64, KPM_RMFT_STATS_LEN, "stats"),
                                    _stream(stream)), "kpm_rmft_update_sdw")


def kpm_rmft_workspace_size(lat, R, M, ckpt_k, precision) -> int:
    n = _lib.kpm_rmft_workspace_size(ctypes.byref(lat), R, M, ckpt_k, precision)
    if n == 0:
        raise KpmError(KPM_EINVAL, "kpm_rmft_workspace_size")
    return int(n)


def rmft_params(doping, mix=0.1, tol_n=1e-6, tol_mu=1e-10, mu_step=0.004, tol_residual=0.0,
                max_evals=60, coef_K=0, search=KPM_RMFT_BISECTION,
                estimator=KPM_RMFT_ADJOINT, anderson=0) -> RmftParams:
    return RmftParams(doping, mix, tol_n, tol_mu, mu_step, tol_residual, max_evals, coef_K, search,
                      estimator, anderson, 0)


def kpm_rmft_iterate(lat, mdl, probes, M, T, precision, ckpt_k, params, n_iter, n, chi, delta, mu,
                     ws, stream=None):
    """Runs up to n_iter iterations in place on (n, chi, delta).  Returns
    (mu, history as a list of dicts, status); status is KPM_OK or KPM_ENOCONV
    (other errors raise)."""
    N = lat.Lx * lat.Ly
    mu_c = c_double(mu)
    hist = (RmftRecord * max(n_iter, 1))()
    done = c_int32(0)
    st = _lib.kpm_rmft_iterate(ctypes.byref(lat), ctypes.byref(mdl), ctypes.byref(_probes(probes)), M,
                               T, precision, ckpt_k, ctypes.byref(params), n_iter,
                               _ptr(n, torch.float64, N, "n"), _ptr(chi, torch.complex128, 4 * N, "chi"),
                               _ptr(delta, torch.complex128, 4 * N, "delta"), ctypes.byref(mu_c),
                               hist, ctypes.byref(done), _ptr(ws, torch.uint8, None, "ws"),
                               ws.numel(), _stream(stream))
    if st not in (KPM_OK, KPM_ENOCONV):
        raise KpmError(st, "kpm_rmft_iterate")
    out = [{"mu": r.mu, "nbar": r.nbar, "residual": r.residual, "omega": r.omega, "evals": r.evals}
           for r in hist[:done.value]]
    return mu_c.value, out, st


def kpm_batch_create(lats: Sequence[Lattice], probes: Sequence[Sequence[ProbeSpec]], M, precision,
                     ckpt_k) -> c_void_p:
    n = len(lats)
    L = (Lattice * n)(*lats)
    prs = [_probes(p) for p in probes]
    P = (Probes * n)(*prs)
    plan = c_void_p()
    _check(_lib.kpm_batch_create(n, L, P, M, precision, ckpt_k, ctypes.byref(plan)), "kpm_batch_create")
    return plan


def kpm_batch_energy_grad(plan, h, ab, C, omega, rho, use_graph=True, stream=None):
    n = len(h)
    arr = lambda ts, dt, nm: (c_void_p * n)(*[_ptr(t, dt, None, nm).value for t in ts])
    _check(_lib.kpm_batch_energy_grad(plan, arr(h, torch.complex128, "h"), arr(ab, torch.float64, "ab"),
                                      arr(C, torch.float64, "C"), _ptr(omega, torch.float64, n, "omega"),
                                      arr(rho, torch.complex128, "rho"), 1 if use_graph else 0,
                                      _stream(stream)), "kpm_batch_energy_grad")


def kpm_batch_destroy(plan) -> None:
    _check(_lib.kpm_batch_destroy(plan), "kpm_batch_destroy")


def kpm_batch_streams(plan) -> int:
    """2 when the plan runs as two instance halves on two streams, else 1."""
    r = _lib.kpm_batch_streams(plan)
    _check(r if r < 0 else 0, "kpm_batch_streams")
    return int(r)


def kpm_batch_groups(plan) -> int:
    """Instance groups the plan runs one after another (1: no groups)."""
    r = _lib.kpm_batch_groups(plan)
    _check(r if r < 0 else 0, "kpm_batch_groups")
    return int(r)


def kpm_set_batch_groups(groups: int) -> int:
    """0 automatic (groups sized to the Infinity Cache), else that many groups for
    batch plans created from now on; returns the previous value."""
    return int(_lib.kpm_set_batch_groups(groups))


def kpm_batch_tuning(plan) -> dict:
    """The plan's probe blocks and schedules, and where they came from."""
    out = (c_int32 * 5)()
    _check(_lib.kpm_batch_tuning(plan, out), "kpm_batch_tuning")
    src = {0: "timed", 1: "process cache", 2: "disk cache", -1: "fixed"}[out[4]]
    return {"fwd_probe_block": out[0], "fwd_schedule": out[1], "adj_probe_block": out[2],
            "adj_schedule": out[3], "source": src}


# ---------------------------------------------------------------- helpers
def workspace(lat, R, M, ckpt_k, precision, device="cuda") -> torch.Tensor:
    """A device byte tensor of kpm_workspace_size bytes, 256-byte aligned."""
    n = kpm_workspace_size(lat, R, M, ckpt_k, precision)
    ws = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + n]


def kpm_rmft_iterate_sdw(lat, mdl, probes, M, T, precision, ckpt_k, params, n_iter, n_up, n_dn, chi_up,
                         chi_dn, delta_up, delta_dn, mu, ws, stream=None):
    """kpm_rmft_iterate on a spin-polarised theta, in place.  Returns
    (mu, history, status) as kpm_rmft_iterate."""
    mu_c = c_double(mu)
    hist = (RmftRecord * max(n_iter, 1))()
    done = c_int32(0)
    st = _lib.kpm_rmft_iterate_sdw(ctypes.byref(lat), ctypes.byref(mdl), ctypes.byref(_probes(probes)),
                                   M, T, precision, ckpt_k, ctypes.byref(params), n_iter,
                                   *_spin_ptrs(lat, n_up, n_dn, chi_up, chi_dn, delta_up, delta_dn),
                                   ctypes.byref(mu_c), hist, ctypes.byref(done),
                                   _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream))
    if st not in (KPM_OK, KPM_ENOCONV):
        raise KpmError(st, "kpm_rmft_iterate_sdw")
    out = [{"mu": r.mu, "nbar": r.nbar, "residual": r.residual, "omega": r.omega, "evals": r.evals}
           for r in hist[:done.value]]
    return mu_c.value, out, st


KPM_SUPERCELL_MAX_N = 16384
KPM_SUPERCELL_MAX_K = 4096
KPM_SUPERCELL_MAX_BATCH = 16


def kpm_bloch_H(lat, h, phi_x, phi_y, Hk, ld=None, stream=None):
    """Dense Bloch matrix H(k) into Hk (complex128, column-major: a [2N, ld]
    tensor whose row q is column q of the matrix)."""
    N = lat.Lx * lat.Ly
    ld = 2 * N if ld is None else int(ld)
    _check(_lib.kpm_bloch_H(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"), float(phi_x),
                            float(phi_y), _ptr(Hk, torch.complex128, 2 * N * ld, "Hk"), ld,
                            _stream(stream)), "kpm_bloch_H")


def kpm_gutzwiller_weights(lat, n_up, n_dn, w_up, w_dn, stream=None):
    N = lat.Lx * lat.Ly
    _check(_lib.kpm_gutzwiller_weights(ctypes.byref(lat), _ptr(n_up, torch.float64, N, "n_up"),
                                       _ptr(n_dn, torch.float64, N, "n_dn"), _ptr(w_up, torch.float64, N, "w_up"),
                                       _ptr(w_dn, torch.float64, N, "w_dn"), _stream(stream)),
           "kpm_gutzwiller_weights")


def kpm_supercell_workspace_size(lat, k_batch=1) -> int:
    n = _lib.kpm_supercell_workspace_size(ctypes.byref(lat), k_batch)
    if n == 0:
        raise KpmError(KPM_EINVAL, "kpm_supercell_workspace_size")
    return int(n)


def kpm_supercell_ldos(lat, h, Mx, My, k_first, k_count, sites, omega, alpha, gamma0, w_up, w_dn,
                       accumulate, ldos, evals, ws, k_batch=1, stream=None):
    N = lat.Lx * lat.Ly
    sites = [int(i) for i in sites]
    arr = (c_int32 * max(len(sites), 1))(*sites)
    W = int(omega.numel())
    _check(_lib.kpm_supercell_ldos(ctypes.byref(lat), _ptr(h, torch.complex128, NENT * N, "h"), Mx, My,
                                   k_first, k_count, k_batch, arr, len(sites),
                                   _ptr(omega, torch.float64, W, "omega"),
                                   W, float(alpha), float(gamma0),
                                   None if w_up is None else _ptr(w_up, torch.float64, N, "w_up"),
                                   None if w_dn is None else _ptr(w_dn, torch.float64, N, "w_dn"),
                                   int(bool(accumulate)), _ptr(ldos, torch.float64, len(sites) * W, "ldos"),
                                   None if evals is None else _ptr(evals, torch.float64, k_count * 2 * N,
                                                                   "evals"),
                                   _ptr(ws, torch.uint8, None, "ws"), ws.numel(), _stream(stream)),
           "kpm_supercell_ldos")
