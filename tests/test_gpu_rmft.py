"""GPU parity of the self-consistent iteration (kpm_rmft_update,
kpm_rmft_iterate) against the oracle's loop (oracle/rmft.py), through the C ABI.

* the map + mixing kernel against ``oracle.rmft.update`` on seeded stand-in
  density matrices, element by element, at a ragged size, at the 48 x 96
  workload size and above the one-pass grid (grid-stride path): FP64 with the
  same operations, so 1e-14 absolute;
* whole iterations in FP64 with either search, either estimator of rho and
  linear or Anderson mixing (bracket decisions, evaluation counts, mu,
  mean density, residual, Omega and theta after every iteration) against the
  oracle loop on the plain KPM: evaluation counts exact, values to the FP64
  bar 1e-10 (relative for Omega and rho-derived values);
* the FP32 recursion with the chemical potential held (tol_n large, so no
  decision depends on rounding) against the same FP64 oracle: 1e-5 relative
  on rho propagates to at most ~1e-5 absolute on theta per iteration;
* the search's budget error leaves theta untouched;
* the 48 x 96 plain-vortex workload: two iterations whose accepted states meet
  the density constraint and stay physical;
* the spin-polarised loop (kpm_rmft_update_sdw, kpm_rmft_iterate_sdw): the
  per-spin map kernel against ``oracle.rmft.update`` on a six-array theta to
  1e-14, and whole FP64 iterations (linear and Anderson, both searches, both
  estimators of rho) on a staggered-moment seed against the oracle loop on
  the spin-polarised builder, to the same bars as the singlet loop.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from oracle import rmft as ormft
from tests import helpers as H
from tests.gpu_helpers import dev, host, problem, theta_dev

pytestmark = pytest.mark.gpu


def _theta_np(cfg):
    n, chi, dlt = wl.make_theta(cfg)
    return n, chi, dlt


@pytest.mark.parametrize("Lx,Ly", [(13, 7), (48, 96), (300, 300)])
@pytest.mark.parametrize("mix", [0.0, 0.3, 1.0])
def test_update_kernel_parity(Lx, Ly, mix):
    from paper_2212_05685_amd import kpm

    cfg = wl.Config("u", Lx, Ly, 2, 0.16, 8, (wl.ProbeSpec("unit", 1),), vortex=True,
                    complex_noise=0.05, seed=Lx * 1000 + Ly)
    th = _theta_np(cfg)
    rho = wl.random_stencil(cfg.N, seed=Lx + 7 * Ly)
    new_ref, nbar_ref, res_ref = ormft.update(rho, th, mix)
    n, chi, dlt = (dev(th[0]), dev(th[1]), dev(th[2]))
    stats = torch.zeros(kpm.KPM_RMFT_STATS_LEN, dtype=torch.float64, device="cuda")
    kpm.kpm_rmft_update(kpm.lattice(Lx, Ly, 2), dev(rho), mix, n, chi, dlt, stats)
    s = host(stats)
    assert abs(s[0] - nbar_ref) < 1e-14
    assert abs(s[1] - res_ref) <= 1e-15 * res_ref
    for got, ref in zip((n, chi, dlt), new_ref):
        assert np.abs(host(got) - ref).max() < 1e-14


def test_update_kernel_nan_propagates():
    from paper_2212_05685_amd import kpm

    cfg = wl.Config("u", 9, 5, 0, 0.16, 8, (wl.ProbeSpec("unit", 1),))
    th = _theta_np(cfg)
    rho = wl.random_stencil(cfg.N, seed=3)
    rho[5, 17] = np.nan
    stats = torch.zeros(kpm.KPM_RMFT_STATS_LEN, dtype=torch.float64, device="cuda")
    kpm.kpm_rmft_update(kpm.lattice(9, 5, 0), dev(rho), 0.0, dev(th[0]), dev(th[1]), dev(th[2]), stats)
    s = host(stats)
    assert np.isfinite(s[0]) and np.isnan(s[1])


def _loop_cfg(precision="fp64"):
    # field on: chi seeded at 0 (a real seed would not carry the bond phases)
    return wl.Config("r", 12, 8, 2, 0.16, 128, (wl.ProbeSpec("colored_z4", 1, 515, 4, 4, 1, 0, 1.0),),
                     precision, ckpt_k=16, vortex=True, complex_noise=0.01, seed=4242, chi0=0.0)


def _oracle_loop(cfg, prm, n_iter, mu0, estimator="adjoint"):
    R, w = H.probe_matrix(cfg)
    make = ormft.kpm_rho_fn if estimator == "adjoint" else ormft.direct_rho_fn
    fn = make(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.T, cfg.M, R, w)
    return ormft.iterate(fn, _theta_np(cfg), mu0, prm, n_iter)


def _gpu_loop(cfg, p, n_iter, mu0, precision=None, estimator="adjoint"):
    """p: oracle Params (search, anderson, tolerances) mirrored into the ABI's."""
    from paper_2212_05685_amd import kpm

    pb = problem(cfg, precision=precision)
    n, chi, dlt = theta_dev(cfg)
    search = {"bisection": kpm.KPM_RMFT_BISECTION, "illinois": kpm.KPM_RMFT_ILLINOIS}[p.search]
    est = {"adjoint": kpm.KPM_RMFT_ADJOINT, "direct": kpm.KPM_RMFT_DIRECT}[estimator]
    prm = kpm.rmft_params(p.doping, p.mix, p.tol_n, p.tol_mu, p.mu_step, p.tol_residual, p.max_evals,
                          search=search, estimator=est, anderson=p.anderson)
    mu, hist, st = pb.rmft_iterate(n, chi, dlt, mu0, prm, n_iter)
    return (host(n), host(chi), host(dlt)), mu, hist, st


@pytest.mark.parametrize("search,estimator,anderson,streams", [("bisection", "adjoint", 0, 0),
                                                               ("illinois", "adjoint", 0, 0),
                                                               ("illinois", "direct", 0, 0),
                                                               ("illinois", "adjoint", 2, 0),
                                                               ("illinois", "adjoint", 0, 2)])
def test_iterate_parity_fp64(search, estimator, anderson, streams):
    """streams 2: every density-matrix evaluation of the loop runs its probes
    as two halves on two streams (the automatic setting keeps this 12 x 8
    lattice's 32 probes on one stream)."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_streams(streams)
    try:
        _check_iterate_parity(search, estimator, anderson)
    finally:
        kpm.kpm_set_streams(0)


def _check_iterate_parity(search, estimator, anderson):
    cfg = _loop_cfg()
    prm = ormft.Params(doping=0.16, mix=0.1, tol_n=1e-5, tol_mu=1e-10, mu_step=0.004, max_evals=60,
                       search=search, anderson=anderson)
    mu0 = cfg.mu
    n_it = 4 if anderson else 3                 # Anderson: the ring wraps at the fourth iteration
    th_ref, mu_ref, hist_ref = _oracle_loop(cfg, prm, n_it, mu0, estimator)
    th, mu, hist, st = _gpu_loop(cfg, prm, n_it, mu0, estimator=estimator)
    assert st == 0 and len(hist) == len(hist_ref) == n_it
    for g, r in zip(hist, hist_ref):
        assert g["evals"] == r["evals"], (hist, hist_ref)
        assert abs(g["mu"] - r["mu"]) < 1e-12
        assert abs(g["nbar"] - r["nbar"]) < 1e-10
        assert abs(g["residual"] - r["residual"]) < 1e-10 * max(r["residual"], 1.0)
        assert abs(g["omega"] - r["omega"]) < 1e-10 * abs(r["omega"])
        assert abs(g["nbar"] - 0.84) <= 1e-5
    assert hist[0]["evals"] > 2                  # the seed's mu is off: walk + bisection ran
    assert abs(mu - mu_ref) < 1e-12
    for a, b in zip(th, th_ref):
        assert np.abs(a - b).max() < 1e-10


def test_iterate_fp32_fixed_mu():
    """FP32 recursion, mu held (every first evaluation accepted)."""
    cfg = _loop_cfg()
    prm = ormft.Params(doping=0.16, mix=0.1, tol_n=1.0, tol_mu=0.0, mu_step=0.004, max_evals=1)
    mu0 = -0.3                                   # near the density-matching mu of this seed
    th_ref, _, hist_ref = _oracle_loop(cfg, prm, 3, mu0)
    th, mu, hist, st = _gpu_loop(cfg, prm, 3, mu0, precision="fp32")
    assert st == 0 and mu == mu0
    for g, r in zip(hist, hist_ref):
        assert g["evals"] == 1
        assert abs(g["nbar"] - r["nbar"]) < 1e-5
        assert abs(g["residual"] - r["residual"]) < 3e-5
        assert abs(g["omega"] - r["omega"]) < 1e-5 * abs(r["omega"])
    for a, b in zip(th, th_ref):
        assert np.abs(a - b).max() < 3e-5


def test_iterate_budget_leaves_theta():
    from paper_2212_05685_amd import kpm

    cfg = _loop_cfg()
    th0 = _theta_np(cfg)
    prm = ormft.Params(doping=0.16, mix=0.2, tol_n=0.0, tol_mu=0.0, mu_step=0.004, max_evals=2)
    th, mu, hist, st = _gpu_loop(cfg, prm, 3, cfg.mu)
    assert st == kpm.KPM_ENOCONV and hist == [] and mu == cfg.mu
    for a, b in zip(th, th0):
        assert np.array_equal(a, b)


def test_rmft_workload_48x96():
    """Two iterations of the plain-vortex workload (FP32 recursion)."""
    cfg = wl.RMFT()
    prm = ormft.Params(doping=cfg.doping, mix=0.1, tol_n=1e-5, tol_mu=1e-9, mu_step=0.004, max_evals=60,
                       search="illinois")
    th, mu, hist, st = _gpu_loop(cfg, prm, 2, cfg.mu)
    assert st == 0 and len(hist) == 2
    for h in hist:
        assert abs(h["nbar"] - (1.0 - cfg.doping)) <= 1e-5
        assert np.isfinite(h["omega"]) and 0.0 < h["residual"] < 1.0
    n, chi, dlt = th
    assert np.all(np.isfinite(n)) and np.all((n > 0.0) & (n < 1.0))
    assert np.all(np.isfinite(chi)) and np.all(np.isfinite(dlt))
    # d-wave sign structure away from the cores: x and y bonds of opposite sign
    amp = np.abs(dlt[0])
    far = amp > 0.5 * amp.max()
    assert np.median(np.real(dlt[0][far] * np.conj(dlt[1][far]))) < 0.0


@pytest.mark.parametrize("Lx,Ly", [(13, 7), (300, 300)])
@pytest.mark.parametrize("mix", [0.0, 0.3, 1.0])
def test_update_sdw_kernel_parity(Lx, Ly, mix):
    from paper_2212_05685_amd import kpm

    cfg = wl.Config("u", Lx, Ly, 2, 0.16, 8, (wl.ProbeSpec("unit", 1),), vortex=True,
                    complex_noise=0.05, seed=Lx * 1000 + Ly + 1)
    th = wl.make_theta_sdw(cfg, m_amp=0.05, spin_noise=0.03)
    rho = wl.random_stencil(cfg.N, seed=Lx + 7 * Ly + 1)
    new_ref, nbar_ref, res_ref = ormft.update(rho, th, mix)
    d = [dev(a) for a in th]
    stats = torch.zeros(kpm.KPM_RMFT_STATS_LEN, dtype=torch.float64, device="cuda")
    kpm.kpm_rmft_update_sdw(kpm.lattice(Lx, Ly, 2), dev(rho), mix, *d, stats)
    s = host(stats)
    assert abs(s[0] - nbar_ref) < 1e-14
    assert abs(s[1] - res_ref) <= 1e-15 * res_ref
    for got, ref in zip(d, new_ref):
        assert np.abs(host(got) - ref).max() < 1e-14


def _sdw_cfg():
    # zero field, real chi seed; staggered moment m_i ~ 0.01 on top
    return wl.Config("s", 12, 8, 0, 0.16, 128, (wl.ProbeSpec("colored_z4", 1, 515, 4, 4, 1, 0, 1.0),),
                     "fp64", ckpt_k=16, vortex=False, complex_noise=0.01, seed=4242)


@pytest.mark.parametrize("search,anderson,estimator,streams", [("illinois", 0, "adjoint", 0),
                                                               ("bisection", 0, "adjoint", 0),
                                                               ("illinois", 2, "adjoint", 0),
                                                               ("illinois", 0, "direct", 0),
                                                               ("illinois", 0, "adjoint", 2)])
def test_iterate_sdw_parity_fp64(search, anderson, estimator, streams):
    """streams 2: the spin-resolved density-matrix evaluations run their probes
    as two halves on two streams."""
    from paper_2212_05685_amd import kpm
    kpm.kpm_set_streams(streams)
    try:
        _check_iterate_sdw_parity(search, anderson, estimator)
    finally:
        kpm.kpm_set_streams(0)


def _check_iterate_sdw_parity(search, anderson, estimator):
    from paper_2212_05685_amd import kpm

    cfg = _sdw_cfg()
    p = ormft.Params(doping=0.16, mix=0.1, tol_n=1e-5, tol_mu=1e-10, mu_step=0.004, max_evals=60,
                     search=search, anderson=anderson)
    n_it = 4 if anderson else 3
    th0 = wl.make_theta_sdw(cfg, m_amp=0.01)
    R, w = H.probe_matrix(cfg)
    make = ormft.sdw_kpm_rho_fn if estimator == "adjoint" else ormft.sdw_direct_rho_fn
    fn = make(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.T, cfg.M, R, w)
    th_ref, mu_ref, hist_ref = ormft.iterate(fn, th0, cfg.mu, p, n_it)

    pb = problem(cfg)
    d = [dev(a) for a in th0]
    prm = kpm.rmft_params(p.doping, p.mix, p.tol_n, p.tol_mu, p.mu_step, p.tol_residual, p.max_evals,
                          search={"bisection": kpm.KPM_RMFT_BISECTION, "illinois": kpm.KPM_RMFT_ILLINOIS}[search],
                          estimator={"adjoint": kpm.KPM_RMFT_ADJOINT, "direct": kpm.KPM_RMFT_DIRECT}[estimator],
                          anderson=anderson)
    mu, hist, st = pb.rmft_iterate_sdw(*d, cfg.mu, prm, n_it)
    assert st == 0 and len(hist) == len(hist_ref) == n_it
    for g, r in zip(hist, hist_ref):
        assert g["evals"] == r["evals"], (hist, hist_ref)
        assert abs(g["mu"] - r["mu"]) < 1e-12
        assert abs(g["nbar"] - r["nbar"]) < 1e-10
        assert abs(g["residual"] - r["residual"]) < 1e-10 * max(r["residual"], 1.0)
        assert abs(g["omega"] - r["omega"]) < 1e-10 * abs(r["omega"])
        assert abs(g["nbar"] - 0.84) <= 1e-5
    assert abs(mu - mu_ref) < 1e-12
    for a, b in zip(d, th_ref):
        assert np.abs(host(a) - b).max() < 1e-10
    m = (th_ref[0] - th_ref[1]) / 2
    assert np.abs(m).max() > 0.02                 # the staggered moment grew: not the singlet path


def test_rmft_driver_save_and_resume(tmp_path):
    """The chunked driver end to end on a small vortex lattice: a run that
    writes a restart file, then a resumed run that continues from it (the
    iteration count and mu carry over)."""
    import json
    import subprocess
    import sys

    state = tmp_path / "s.npz"
    base = [sys.executable, "-m", "paper_2212_05685_amd.rmft_run", "--lx", "16", "--ly", "16",
            "--moments", "128", "--chunk", "2"]
    env = {**__import__("os").environ, "PYTHONPATH": str(__import__("pathlib").Path(__file__).parents[1])}
    r1 = subprocess.run(base + ["--iters", "3", "--save", str(state)], capture_output=True, text=True,
                        env=env, timeout=240)
    assert r1.returncode == 0, r1.stderr[-2000:]
    s1 = json.loads(r1.stdout.strip().splitlines()[-1])
    assert s1["iterations"] == 3 and state.exists()
    r0 = subprocess.run(base + ["--iters", "0", "--resume", str(state)], capture_output=True, text=True,
                        env=env, timeout=240)
    assert r0.returncode == 0, r0.stderr[-2000:]
    s0 = json.loads(r0.stdout.strip().splitlines()[-1])
    assert s0["iterations"] == 3 and s0["mu"] == s1["mu"]          # the state carries over exactly
    r2 = subprocess.run(base + ["--iters", "2", "--resume", str(state), "--save", str(state)],
                        capture_output=True, text=True, env=env, timeout=240)
    assert r2.returncode == 0, r2.stderr[-2000:]
    s2 = json.loads(r2.stdout.strip().splitlines()[-1])
    assert s2["iterations"] == 5 and s2["status"] == 0
    assert len(s2["cores"]) == 2
