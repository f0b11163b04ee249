"""CPU checks of the C ABI: the library loads, exports every function that
include/kpm.h declares, the ctypes structs match the C layout, and host-side
argument validation rejects bad input before any device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "kpm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kpm_[a-z_A-Z0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2212_05685_amd import kpm

    declared = _declared()
    assert len(declared) >= 16
    for name in declared:
        assert hasattr(kpm._lib, name), name
        assert name in kpm.EXPORTS
        assert callable(getattr(kpm, name)), name


def test_struct_layouts():
    from paper_2212_05685_amd import kpm

    assert ctypes.sizeof(kpm.Lattice) == 12
    assert ctypes.sizeof(kpm.Model) == 32
    assert ctypes.sizeof(kpm.ProbeGroup) == 40
    assert kpm.ProbeGroup.seed.offset == 24 and kpm.ProbeGroup.weight.offset == 32
    assert ctypes.sizeof(kpm.Probes) == 16


def test_host_validation():
    from paper_2212_05685_amd import kpm

    lat = kpm.lattice(8, 8, 0)
    PS = kpm.ProbeSpec
    assert kpm.kpm_probe_count(lat, [PS(kpm.KPM_PROBE_UNIT, 128)]) == 128
    assert kpm.kpm_probe_count(lat, [PS(kpm.KPM_PROBE_COLORED_Z4, 2, 1, 8, 8, 1)]) == 256
    assert kpm.kpm_probe_count(lat, [PS(kpm.KPM_PROBE_COLORED_Z4, 1, 1, 4, 2, 0),
                                     PS(kpm.KPM_PROBE_DENSE_Z4, 5)]) == 13
    for bad in ([PS(kpm.KPM_PROBE_UNIT, 129)], [PS(kpm.KPM_PROBE_UNIT, 1, first=-1)],
                [PS(7, 1)], [PS(kpm.KPM_PROBE_COLORED_Z4, 1, 1, 9, 1)], [],
                [PS(kpm.KPM_PROBE_DENSE_Z4, 1)] * 5):
        with pytest.raises(kpm.KpmError):
            kpm.kpm_probe_count(lat, bad)
    for L in (kpm.lattice(2, 8, 0), kpm.lattice(8, 8, 1)):
        with pytest.raises(kpm.KpmError):
            kpm.kpm_probe_count(L, [PS(kpm.KPM_PROBE_UNIT, 1)])
        assert kpm._lib.kpm_workspace_size(ctypes.byref(L), 4, 16, 8, 0) == 0
    # workspace grows with R, M and precision; zero on invalid sizes
    s64 = kpm.kpm_workspace_size(lat, 16, 64, 8, kpm.KPM_FP64)
    s32 = kpm.kpm_workspace_size(lat, 16, 64, 8, kpm.KPM_FP32)
    assert s64 > s32 > 0
    assert kpm.kpm_workspace_size(lat, 32, 64, 8, kpm.KPM_FP64) > s64
    assert kpm._lib.kpm_workspace_size(ctypes.byref(lat), 16, 1, 8, 0) == 0
    assert kpm._lib.kpm_workspace_size(ctypes.byref(lat), 16, 64, 1, 0) == 0
    assert kpm._lib.kpm_workspace_size(ctypes.byref(lat), 16, 64, 8, 2) == 0
    # entry points reject bad arguments synchronously (nothing reaches the device)
    assert kpm._lib.kpm_build_H(ctypes.byref(kpm.lattice(2, 2, 0)), ctypes.byref(kpm.model(1, 0, 0, 0)),
                                None, None, None, None, None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_coefficients(1, 0.005, None, 0, None, None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_coefficients(64, -1.0, ctypes.c_void_p(256), 0, ctypes.c_void_p(256),
                                     None) == kpm.KPM_EINVAL
    assert kpm.strerror(kpm.KPM_EBOUNDS).startswith("spectrum")
    old = kpm.kpm_set_probe_block(4)
    assert kpm.kpm_set_probe_block(3) == 4       # invalid value leaves the setting
    assert kpm.kpm_set_probe_block(old) == 4
    # block schedules: -1 (default) .. 4 (balanced); anything else is rejected
    for bad in ((5, 0), (0, 5), (-2, 0), (0, -2)):
        assert kpm._lib.kpm_set_schedule(*bad) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_set_schedule(kpm.KPM_SCHED_STRIPS, kpm.KPM_SCHED_TILE_MAJOR) == kpm.KPM_OK
    assert kpm._lib.kpm_set_schedule(kpm.KPM_SCHED_DEFAULT, kpm.KPM_SCHED_DEFAULT) == kpm.KPM_OK
    # streams: 0 (automatic) .. 2 (probe halves); other values leave the setting
    old_streams = kpm.kpm_set_streams(2)
    assert kpm.kpm_set_streams(3) == 2 and kpm.kpm_set_streams(-1) == 2
    assert kpm.kpm_set_streams(old_streams) == 2
    out = (ctypes.c_int32 * 5)()
    assert kpm._lib.kpm_batch_tuning(None, out) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_batch_streams(None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_batch_groups(None) == kpm.KPM_EINVAL
    old_groups = kpm.kpm_set_batch_groups(3)
    assert kpm.kpm_set_batch_groups(-1) == 3 and kpm.kpm_set_batch_groups(old_groups) == 3


def test_rmft_host_validation():
    """kpm_rmft_update / kpm_rmft_iterate reject bad arguments before any
    device work (placeholder pointers are never dereferenced)."""
    from paper_2212_05685_amd import kpm

    lat = kpm.lattice(8, 8, 0)
    fake = ctypes.c_void_p(256)
    assert ctypes.sizeof(kpm.RmftParams) == 72 and kpm.RmftParams.anderson.offset == 64 and kpm.RmftParams.search.offset == 56 and kpm.RmftParams.estimator.offset == 60 and ctypes.sizeof(kpm.RmftRecord) == 40
    assert kpm.RmftRecord.evals.offset == 32
    for mix in (-0.1, 1.5, float("nan")):
        assert kpm._lib.kpm_rmft_update(ctypes.byref(lat), fake, mix, fake, fake, fake, fake,
                                        None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_rmft_update(ctypes.byref(kpm.lattice(2, 8, 0)), fake, 0.5, fake, fake, fake,
                                    fake, None) == kpm.KPM_EINVAL
    base = kpm.kpm_workspace_size(lat, 16, 64, 8, kpm.KPM_FP64)
    full = kpm.kpm_rmft_workspace_size(lat, 16, 64, 8, kpm.KPM_FP64)
    assert full > base + 2 * 19 * 64 * 16
    assert kpm._lib.kpm_rmft_workspace_size(ctypes.byref(lat), 16, 1, 8, 0) == 0

    mdl = kpm.model(1.0, -0.3, 0.3, 0.0)
    pr = kpm._probes([kpm.ProbeSpec(kpm.KPM_PROBE_UNIT, 16)])
    mu = ctypes.c_double(1.0)
    done = ctypes.c_int32(-1)

    def call(prm, ws_bytes=full, n_iter=1, T=0.005, ws=ctypes.c_void_p(1 << 20)):
        return kpm._lib.kpm_rmft_iterate(ctypes.byref(lat), ctypes.byref(mdl), ctypes.byref(pr), 64, T,
                                         kpm.KPM_FP64, 8, ctypes.byref(prm), n_iter, fake, fake, fake,
                                         ctypes.byref(mu), None, ctypes.byref(done), ws, ws_bytes, None)

    good = kpm.rmft_params(0.16)
    for bad in (kpm.rmft_params(0.0), kpm.rmft_params(1.0), kpm.rmft_params(0.16, mix=0.0),
                kpm.rmft_params(0.16, mix=1.2), kpm.rmft_params(0.16, tol_n=-1.0),
                kpm.rmft_params(0.16, mu_step=0.0), kpm.rmft_params(0.16, max_evals=0),
                kpm.rmft_params(0.16, coef_K=-1), kpm.rmft_params(0.16, search=2),
                kpm.rmft_params(0.16, estimator=2), kpm.rmft_params(0.16, anderson=-1),
                kpm.rmft_params(0.16, anderson=9)):
        assert call(bad) == kpm.KPM_EINVAL
    assert call(good, n_iter=-1) == kpm.KPM_EINVAL
    assert call(good, T=0.0) == kpm.KPM_EINVAL
    assert call(good, ws_bytes=full - 1) == kpm.KPM_EWORKSPACE
    assert call(good, ws=ctypes.c_void_p((1 << 20) + 64)) == kpm.KPM_EWORKSPACE
    assert done.value == -1                     # nothing ran
    assert kpm.strerror(kpm.KPM_ENOCONV).startswith("chemical-potential")

    mdl0 = kpm.model(1.0, -0.3, 0.3, 0.0)
    # 13 pointers (6 parameters, rho, 6 outputs) then the stream; the last output missing
    assert kpm._lib.kpm_build_H_sdw_vjp(ctypes.byref(lat), ctypes.byref(mdl0), *([fake] * 12), None,
                                        None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_build_H_sdw_vjp(ctypes.byref(kpm.lattice(2, 8, 0)), ctypes.byref(mdl0), *([fake] * 13),
                                        None) == kpm.KPM_EINVAL

    # the spin-polarised entries: same checks, plus a missing spin array
    for mix in (-0.1, 1.5, float("nan")):
        assert kpm._lib.kpm_rmft_update_sdw(ctypes.byref(lat), fake, mix, fake, fake, fake, fake, fake,
                                            fake, fake, None) == kpm.KPM_EINVAL
    assert kpm._lib.kpm_rmft_update_sdw(ctypes.byref(lat), fake, 0.5, fake, None, fake, fake, fake,
                                        fake, fake, None) == kpm.KPM_EINVAL

    def call_sdw(prm, dn=fake, ws_bytes=full):
        return kpm._lib.kpm_rmft_iterate_sdw(ctypes.byref(lat), ctypes.byref(mdl), ctypes.byref(pr), 64,
                                             0.005, kpm.KPM_FP64, 8, ctypes.byref(prm), 1, fake, dn, fake,
                                             fake, fake, fake, ctypes.byref(mu), None, ctypes.byref(done),
                                             ctypes.c_void_p(1 << 20), ws_bytes, None)

    assert call_sdw(kpm.rmft_params(0.16, anderson=9)) == kpm.KPM_EINVAL
    assert call_sdw(good, dn=None) == kpm.KPM_EINVAL
    assert call_sdw(good, ws_bytes=full - 1) == kpm.KPM_EWORKSPACE
    assert done.value == -1


def test_rmft_state_round_trip(tmp_path):
    import numpy as np
    import torch

    from paper_2212_05685_amd.solver import load_rmft_state, save_rmft_state

    rng = np.random.default_rng(5)
    n = torch.from_numpy(rng.uniform(0.7, 0.9, 12))
    chi = torch.from_numpy(rng.normal(size=(4, 12)) + 1j * rng.normal(size=(4, 12)))
    dlt = torch.from_numpy(rng.normal(size=(4, 12)) + 1j * rng.normal(size=(4, 12)))
    hist = [{"mu": 1.5, "nbar": 0.84, "residual": 0.01, "omega": -3.0, "evals": 7}]
    p = tmp_path / "state.npz"
    save_rmft_state(p, n, chi, dlt, 1.625, hist)
    n2, c2, d2, mu2, h2 = load_rmft_state(p, device="cpu")
    assert torch.equal(n, n2) and torch.equal(chi, c2) and torch.equal(dlt, d2)
    assert mu2 == 1.625 and h2 == hist


def test_supercell_host_validation():
    """kpm_bloch_H / kpm_supercell_ldos reject bad arguments before any device
    work (placeholder pointers are never dereferenced)."""
    from paper_2212_05685_amd import kpm

    lat = kpm.lattice(6, 5, 2)
    N = 30
    fake = ctypes.c_void_p(256)
    L = kpm._lib
    assert L.kpm_bloch_H(ctypes.byref(lat), fake, 0.1, 0.2, fake, 2 * N - 1, None) == kpm.KPM_EINVAL
    assert L.kpm_bloch_H(ctypes.byref(kpm.lattice(2, 5, 0)), fake, 0.0, 0.0, fake, 20, None) == kpm.KPM_EINVAL
    assert L.kpm_bloch_H(ctypes.byref(lat), fake, float("nan"), 0.0, fake, 2 * N, None) == kpm.KPM_EINVAL
    full = kpm.kpm_supercell_workspace_size(lat, 1)
    assert full >= (2 * N) ** 2 * 16
    assert kpm.kpm_supercell_workspace_size(lat, 3) >= 3 * (2 * N) ** 2 * 16
    assert L.kpm_supercell_workspace_size(ctypes.byref(kpm.lattice(130, 130, 0)), 1) == 0
    assert L.kpm_supercell_workspace_size(ctypes.byref(lat), 0) == 0
    assert L.kpm_supercell_workspace_size(ctypes.byref(lat), kpm.KPM_SUPERCELL_MAX_BATCH + 1) == 0

    def call(Mx=2, My=2, k0=0, kc=4, kb=1, sites=(0, 29), alpha=0.25, g0=3e-4, acc=0, ws_bytes=full,
             ws=ctypes.c_void_p(1 << 20)):
        arr = (ctypes.c_int32 * len(sites))(*sites)
        return L.kpm_supercell_ldos(ctypes.byref(lat), fake, Mx, My, k0, kc, kb, arr, len(sites), fake, 5,
                                    alpha, g0, None, None, acc, fake, None, ws, ws_bytes, None)

    for kw in ({"Mx": 0}, {"kc": 5}, {"k0": 3, "kc": 2}, {"kc": 0}, {"sites": (0, 30)}, {"sites": (-1,)},
               {"alpha": -0.1}, {"g0": 0.0}, {"acc": 2}, {"Mx": 4097, "My": 1}, {"kb": 0}, {"kb": 17}):
        assert call(**kw) == kpm.KPM_EINVAL, kw
    assert call(ws_bytes=full - 1) == kpm.KPM_EWORKSPACE
    assert call(kb=2) == kpm.KPM_EWORKSPACE                 # workspace sized for one matrix
    assert call(ws=ctypes.c_void_p((1 << 20) + 8)) == kpm.KPM_EWORKSPACE


def test_vortex_seed_shift():
    """workloads.Config.vortex_dx moves the seeded pairing minima along x only."""
    import numpy as np
    import workloads as wl

    Lx, Ly = 24, 16
    base = wl.Config("v", Lx, Ly, 2, 0.16, 8, (wl.ProbeSpec("unit", 1),), vortex=True)
    x, y = np.arange(Lx * Ly) % Lx, np.arange(Lx * Ly) // Lx
    for dx in (0.0, 6.0):
        _, _, dlt = wl.make_theta(wl.scaled(base, vortex_dx=dx))
        amp = np.abs(dlt[0])                      # +x bonds, midpoints (x + 1/2, y)
        for k, (X, Y) in enumerate(wl.vortex_centres(Lx, Ly, 2)):
            half = (y < Ly // 2) if k == 0 else (y >= Ly // 2)
            i = np.flatnonzero(half)[np.argmin(amp[half])]
            assert abs((x[i] + 0.5 - (X + dx) + Lx / 2) % Lx - Lx / 2) <= 1.0
            assert abs(y[i] - Y) <= 1.0


def test_core_fit_recovers_synthetic_cores():
    """rmft_run's host-side analysis: on a synthetic amplitude D0 tanh(r/xi)
    around two centres (minimum-image distances on the torus), the fit returns
    the centres, D0 and xi it was built from."""
    import numpy as np
    from paper_2212_05685_amd.rmft_run import core_fit, vortex_positions

    Lx, Ly, D0, xi = 48, 96, 0.03, 2.7
    cs = [(46.6, 28.3), (47.2, 74.4)]
    x, y = np.arange(Lx * Ly) % Lx, np.arange(Lx * Ly) // Lx
    amp = np.full(Lx * Ly, D0)
    for cx, cy in cs:
        r = np.hypot((x - cx + Lx / 2) % Lx - Lx / 2, (y - cy + Ly / 2) % Ly - Ly / 2)
        amp = amp * np.tanh(r / xi)
    pos = vortex_positions(amp, Lx, Ly, 2)
    fits = sorted(core_fit(amp, Lx, Ly, pos), key=lambda f: f["centre"][1])
    for f, (cx, cy) in zip(fits, cs):
        assert abs(f["centre"][0] - cx) < 0.05 and abs(f["centre"][1] - cy) < 0.05
        assert abs(f["xi"] - xi) < 0.05 and abs(f["D0"] - D0) < 1e-3
