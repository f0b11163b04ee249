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
