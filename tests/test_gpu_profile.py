"""The library's kernel timing (kpm_profile_begin / kpm_profile_end), which
bench.py uses for its per-launch durations: runs of consecutive launches of
one step kernel, timed by events that the dispatches record themselves."""
import pytest
import torch

import workloads as wl
from tests.gpu_helpers import problem, theta_dev

pytestmark = pytest.mark.gpu


def _cfg(M):
    return wl.Config("prof", 24, 16, 2, 0.13, M, (wl.ProbeSpec("colored_z4", 1, 5, 4, 4, 1, 0, 1.0),),
                     "fp32", vortex=True, ckpt_k=8)


@pytest.fixture(autouse=True)
def _reset():
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_probe_block(4)
    yield
    kpm.kpm_set_probe_block(0)
    kpm.kpm_set_streams(0)
    kpm.kpm_profile_end()


@pytest.mark.parametrize("streams", [1, 2])
@pytest.mark.parametrize("every", [1, 8, 32])
def test_runs_cover_whole_windows(every, streams):
    """Forward launches m = 0 .. M-2 and adjoint launches m = M-3 .. 0: a run
    of min(16, every) launches starts at every `every`-th launch of each kind
    and only complete runs count.  With probe halves on two streams only the
    caller's stream is timed, and the second stream's launches, interleaved
    with them, neither count nor break a run: the counts are those of one
    stream."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_streams(streams)
    M = 101
    cfg = _cfg(M)
    p = problem(cfg, precision="fp32")
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    p.grand_potential(h, ab, C)
    p.grand_potential_grad(h, ab, C)        # warm, and the first call's tuning is out of the way
    torch.cuda.synchronize()
    kpm.kpm_profile_begin(every)
    p.grand_potential(h, ab, C)
    p.grand_potential_grad(h, ab, C)
    torch.cuda.synchronize()
    f_ms, nf, a_ms, na = kpm.kpm_profile_end()
    w = min(16, every)
    # forward: runs start at m = 0, every, 2 every ... with m + w - 1 <= M - 2
    runs_f = len([m for m in range(0, M - 1, every) if m + w - 1 <= M - 2])
    # adjoint (flag 0 launches m = M-3 .. 0): position M-3-m multiple of every, m - w + 1 >= 0
    runs_a = len([m for m in range(M - 3, -1, -1) if (M - 3 - m) % every == 0 and m - w + 1 >= 0])
    assert nf == runs_f * w
    assert na == runs_a * w
    assert f_ms > 0.0 and a_ms > 0.0
    # per-launch averages are plausible kernel durations (above 1 us, below 10 ms)
    assert 1e-3 < f_ms / nf < 10.0 and 1e-3 < a_ms / na < 10.0


def test_nothing_counted_outside_profiling():
    from paper_2212_05685_amd import kpm
    cfg = _cfg(40)
    p = problem(cfg, precision="fp32")
    h = p.build_H(*theta_dev(cfg))
    ab = p.bounds(h)
    C = p.coefficients(ab)
    kpm.kpm_profile_begin(4)
    kpm.kpm_profile_end()
    p.grand_potential(h, ab, C)
    p.grand_potential_grad(h, ab, C)
    torch.cuda.synchronize()
    kpm.kpm_profile_begin(4)
    f_ms, nf, a_ms, na = kpm.kpm_profile_end()
    assert (nf, na) == (0, 0) and f_ms == 0.0 and a_ms == 0.0
