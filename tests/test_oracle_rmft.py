"""Pins of the oracle's self-consistent iteration (oracle/rmft.py) against
results fixed independently of it:

* the uniform zero-field d-wave state solved in k-space (oracle/kspace.py:
  closed-form Bloch blocks of App. A's coefficients at m = 0, exact Fermi
  occupations, its own chemical-potential bisection) must be a fixed point of
  the real-space iteration built on the autograd builder and dense
  diagonalisation, with the same chemical potential;
* the chemical-potential search must land on the k-space bisection's root;
* for a singlet state the spin-up and spin-down estimates of chi and Delta
  coincide (SU(2) symmetry of h at m_i = 0), which pins the sign conventions
  of the spin-averaged map;
* the iteration contracts towards the fixed point from a perturbed start.
"""
import numpy as np
import pytest

import workloads as wl
from oracle import kspace, mapping, rmft

L, DOP = 8, 0.16
T_, TP, J, TEMP = wl.T_HOP, wl.TP_HOP, wl.J_EX, wl.TEMP


def _kspace_fixed_point(L=L, dop=DOP):
    """Uniform d-wave solution of the same self-consistency in k-space."""
    chi = np.array([0.2, 0.2, 0.0, 0.0], dtype=complex)
    dlt = np.array([0.1, -0.1, 0.0, 0.0], dtype=complex)
    for _ in range(200):
        mu = kspace.mu_for_doping(dop, chi, dlt, T_, TP, J, TEMP, L=L, tol=1e-14)
        on, bl = kspace.uniform_blocks(dop, chi, dlt, T_, TP, J, mu)
        _, r = kspace.exact_omega_rho_site(on, bl, L, L, TEMP)
        # Nambu-spinor reading of App. B, singlet average (bond stored at its tail)
        c1 = np.array([(r[4 * d] - np.conj(r[4 * d + 3])) / 2 for d in range(4)])
        d1 = np.array([(-np.conj(r[4 * d + 1]) - r[4 * d + 2]) / 2 for d in range(4)])
        res = max(np.abs(c1 - chi).max(), np.abs(d1 - dlt).max())
        chi, dlt = c1, d1
        if res < 1e-14:
            break
    assert res < 1e-13
    return mu, chi, dlt


@pytest.fixture(scope="module")
def fixed_point():
    return _kspace_fixed_point()


def _uniform_theta(chi, dlt, N, dop=DOP):
    return (np.full(N, 1.0 - dop), np.repeat(chi[:, None], N, axis=1).astype(complex),
            np.repeat(dlt[:, None], N, axis=1).astype(complex))


def test_kspace_fixed_point_is_dwave(fixed_point):
    mu, chi, dlt = fixed_point
    assert abs(chi[0] - chi[1]) < 1e-12 and abs(dlt[0] + dlt[1]) < 1e-12
    assert abs(dlt[0]) > 0.05                      # pairing survives at this doping
    assert abs(chi[2] - chi[3]) < 1e-12 and abs(dlt[2]) < 1e-12 and abs(dlt[3]) < 1e-12


def test_kspace_solution_is_real_space_fixed_point(fixed_point):
    mu_k, chi, dlt = fixed_point
    th = _uniform_theta(chi, dlt, L * L)
    fn = rmft.exact_rho_fn(L, L, 0, T_, TP, J, TEMP)
    prm = rmft.Params(doping=DOP, mix=0.5, tol_n=1e-12, tol_mu=1e-13, mu_step=0.004, max_evals=80)
    th1, mu1, hist = rmft.iterate(fn, th, mu_k - 0.003, prm, 1)
    h = hist[0]
    assert h["evals"] > 2                         # the search had to walk and bisect
    assert abs(mu1 - mu_k) < 1e-9
    assert abs(h["nbar"] - (1.0 - DOP)) <= 1e-12
    assert h["residual"] < 1e-9
    for a, b in zip(th1, th):
        assert np.abs(a - b).max() < 1e-9


def test_mu_search_matches_kspace_bisection():
    """Seed state (not self-consistent): the root of nbar(mu) = 1 - doping."""
    chi = np.array([0.2, 0.2, 0.0, 0.0], dtype=complex)
    dlt = np.array([0.1, -0.1, 0.0, 0.0], dtype=complex)
    mu_k = kspace.mu_for_doping(DOP, chi, dlt, T_, TP, J, TEMP, L=L, tol=1e-14)
    th = _uniform_theta(chi, dlt, L * L)
    fn = rmft.exact_rho_fn(L, L, 0, T_, TP, J, TEMP)
    def e_fn(m):
        _, rho = fn(th, m)
        nbar, _ = rmft.measure(rho, th)
        return nbar - (1.0 - DOP), None

    for search in ("bisection", "illinois"):
        prm = rmft.Params(doping=DOP, tol_n=1e-12, tol_mu=1e-14, mu_step=0.05, max_evals=80,
                          search=search)
        for mu0 in (0.0, 3.0):                    # from below and from above
            mu, _, evals = rmft.solve_mu(e_fn, mu0, prm)
            assert abs(mu - mu_k) < 1e-9, (search, mu0, mu, mu_k, evals)


def test_mu_search_budget():
    prm = rmft.Params(doping=DOP, tol_n=1e-9, mu_step=0.01, max_evals=3)
    with pytest.raises(rmft.NoConvergence):
        rmft.solve_mu(lambda m: (m - 1.0, None), 0.0, prm)
    # a linear e(mu): the walk doubles its step, then bisection lands on the root
    prm = rmft.Params(doping=DOP, tol_n=0.0, tol_mu=1e-12, mu_step=0.01, max_evals=100)
    mu, _, evals = rmft.solve_mu(lambda m: (m - 1.0, None), 0.0, prm)
    assert abs(mu - 1.0) <= 1e-12 and evals > 7
    # false position is exact on a linear e(mu): one step after the bracket
    prm = rmft.Params(doping=DOP, tol_n=1e-12, tol_mu=0.0, mu_step=0.01, max_evals=100,
                      search="illinois")
    mu, _, evals_il = rmft.solve_mu(lambda m: (m - 1.0, None), 0.0, prm)
    assert abs(mu - 1.0) <= 1e-12 and evals_il == 9    # start, 7 walk steps, 1 secant step


@pytest.mark.parametrize("search", ["bisection", "illinois"])
def test_mu_search_closed_form_root(search):
    """A smooth monotone e(mu) with a known root: tanh((mu - 1)/0.3) - 0.2."""
    root = 1.0 + 0.3 * np.arctanh(0.2)
    prm = rmft.Params(doping=DOP, tol_n=1e-13, tol_mu=0.0, mu_step=0.004, max_evals=200, search=search)
    for mu0 in (-2.0, 0.9, 3.5):
        mu, _, evals = rmft.solve_mu(lambda m: (np.tanh((m - 1.0) / 0.3) - 0.2, None), mu0, prm)
        assert abs(mu - root) < 1e-12, (mu0, mu, evals)
        assert evals < (40 if search == "illinois" else 80)


def test_singlet_spin_estimates_agree():
    """m_i = 0: h is SU(2) symmetric, so chi_up = chi_dn and Delta_up = Delta_dn."""
    cfg = wl.Config("v", 6, 6, 2, 0.125, 64, (wl.ProbeSpec("unit", 72),), vortex=True,
                    complex_noise=0.02)
    th = wl.make_theta(cfg)
    _, rho = rmft.exact_rho_fn(6, 6, 2, T_, TP, J, TEMP)(th, cfg.mu)
    op = mapping.order_parameters(rho)
    assert np.abs(op["chi_up"] - op["chi_dn"]).max() < 1e-12
    assert np.abs(op["delta_up"] - op["delta_dn"]).max() < 1e-12
    assert np.abs(op["n_up"] - op["n_dn"]).max() < 1e-12
    assert np.abs(op["delta_up"][:2]).max() > 1e-3


def test_update_is_linear_mixing():
    rng = np.random.default_rng(7)
    N = 12
    rho = rng.normal(size=(19, N)) + 1j * rng.normal(size=(19, N))
    th = (rng.uniform(0.7, 0.9, N), rng.normal(size=(4, N)) + 0j, rng.normal(size=(4, N)) + 0j)
    tp = rmft.singlet_theta(rho)
    same, _, _ = rmft.update(rho, th, 0.0)
    full, nbar, res = rmft.update(rho, th, 1.0)
    half, _, _ = rmft.update(rho, th, 0.5)
    for a, b, c, d, e in zip(same, th, full, tp, half):
        assert np.array_equal(a, b)
        assert np.allclose(c, d, rtol=0, atol=1e-14)
        assert np.allclose(e, 0.5 * (b + d), rtol=0, atol=1e-14)
    assert nbar == pytest.approx(float(np.mean(tp[0])), abs=1e-15)
    assert res == max(np.abs(tp[0] - th[0]).max(), np.abs(tp[1] - th[1]).max(),
                      np.abs(tp[2] - th[2]).max())


def test_iteration_contracts_to_fixed_point(fixed_point):
    """A seeded perturbation of every parameter decays under the iteration.
    The site densities respond strongly to their own onsite energy through
    the Gutzwiller factors (a full update overshoots by an order of
    magnitude), so the mixing weight is small, as the long iteration counts
    the paper reports suggest."""
    mu_k, chi, dlt = fixed_point
    N = L * L
    n0, c0, d0 = _uniform_theta(chi, dlt, N)
    rng = np.random.default_rng(11)
    pert = 0.01
    th = (n0 + rng.uniform(-pert, pert, N),
          c0 + rng.uniform(-pert, pert, (4, N)),
          d0 + rng.uniform(-pert, pert, (4, N)) * np.array([[1], [1], [0], [0]]))
    fn = rmft.exact_rho_fn(L, L, 0, T_, TP, J, TEMP)
    prm = rmft.Params(doping=DOP, mix=0.1, tol_n=1e-6, tol_mu=1e-12, mu_step=0.004, max_evals=60)

    def dist(t):
        return max(np.abs(t[0] - n0).max(), np.abs(t[1] - c0).max(), np.abs(t[2][:2] - d0[:2]).max())

    d_start = dist(th)
    th, mu, hist = rmft.iterate(fn, th, mu_k, prm, 6)
    res = [h["residual"] for h in hist]
    assert all(b < a for a, b in zip(res, res[1:])), res
    assert res[-1] < 0.2 * res[0]
    assert dist(th) < 0.8 * d_start
    assert all(abs(h["nbar"] - (1.0 - DOP)) <= 1e-6 for h in hist)
    assert abs(mu - mu_k) < 1e-2


def test_pack_round_trip_and_layout():
    rng = np.random.default_rng(2)
    N = 7
    th = (rng.normal(size=N), rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)),
          rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)))
    x = rmft.pack(th)
    assert x.shape == (17 * N,)
    assert x[N] == th[1][0, 0].real and x[N + 1] == th[1][0, 0].imag      # interleaved re/im
    assert x[9 * N + 2] == th[2][0, 1].real
    for a, b in zip(rmft.unpack(x, N), th):
        assert np.array_equal(a, b)


def test_anderson_solves_linear_fixed_point():
    """On an affine map g(x) = A x + c (contraction), Anderson mixing with
    depth >= dim reaches the fixed point (I - A)^-1 c in dim + 2 steps."""
    rng = np.random.default_rng(4)
    d = 5
    Q = np.linalg.qr(rng.normal(size=(d, d)))[0]
    A = Q @ np.diag([0.9, -0.8, 0.5, 0.2, -0.95]) @ Q.T
    c = rng.normal(size=d)
    xs = np.linalg.solve(np.eye(d) - A, c)
    acc = rmft.Anderson(d, 0.3)
    x = np.zeros(d)
    for _ in range(d + 2):
        x = acc.step(x, A @ x + c - x)
    assert np.max(np.abs(x - xs)) < 1e-8
    # linear mixing alone is far from converged after as many steps
    y = np.zeros(d)
    for _ in range(d + 2):
        y = y + 0.3 * (A @ y + c - y)
    assert np.max(np.abs(y - xs)) > 1e-2


def test_anderson_loop_converges_faster(fixed_point):
    """The perturbed uniform state of test_iteration_contracts_to_fixed_point:
    Anderson mixing (depth 5) ends 12 iterations with a residual several times
    below linear mixing's."""
    mu_k, chi, dlt = fixed_point
    N = L * L
    n0, c0, d0 = _uniform_theta(chi, dlt, N)
    rng = np.random.default_rng(11)
    pert = 0.01
    th = (n0 + rng.uniform(-pert, pert, N), c0 + rng.uniform(-pert, pert, (4, N)),
          d0 + rng.uniform(-pert, pert, (4, N)) * np.array([[1], [1], [0], [0]]))
    fn = rmft.exact_rho_fn(L, L, 0, T_, TP, J, TEMP)
    base = dict(doping=DOP, mix=0.1, tol_n=1e-8, tol_mu=1e-12, mu_step=0.004, max_evals=60)
    _, _, h_lin = rmft.iterate(fn, th, mu_k, rmft.Params(**base), 12)
    _, _, h_and = rmft.iterate(fn, th, mu_k, rmft.Params(**base, anderson=5), 12)
    assert h_and[-1]["residual"] < 0.3 * h_lin[-1]["residual"], (h_and[-1], h_lin[-1])


def test_spin_loop_reduces_to_singlet_loop():
    """A spin-polarised theta with equal spins follows the singlet iteration:
    the per-spin map of an SU(2)-symmetric h returns equal spins, and the
    singlet average of equal spins is each of them."""
    cfg = wl.Config("v", 6, 4, 2, 0.16, 32, (wl.ProbeSpec("unit", 48),), vortex=True, complex_noise=0.01,
                    chi0=0.0)
    n, chi, dlt = wl.make_theta(cfg)
    prm = rmft.Params(doping=0.16, mix=0.3, tol_n=1e-9, tol_mu=1e-12, mu_step=0.01, max_evals=80)
    fs = rmft.exact_rho_fn(6, 4, 2, T_, TP, J, TEMP)
    fp = rmft.sdw_exact_rho_fn(6, 4, 2, T_, TP, J, TEMP)
    th_s, mu_s, h_s = rmft.iterate(fs, (n, chi, dlt), cfg.mu, prm, 2)
    th_p, mu_p, h_p = rmft.iterate(fp, (n / 2, n / 2, chi, chi, dlt, dlt), cfg.mu, prm, 2)
    assert abs(mu_s - mu_p) < 1e-9
    assert np.abs(th_p[0] + th_p[1] - th_s[0]).max() < 1e-9
    for a, b in ((th_p[2], th_s[1]), (th_p[3], th_s[1]), (th_p[4], th_s[2]), (th_p[5], th_s[2])):
        assert np.abs(a - b).max() < 1e-9
    assert [x["evals"] for x in h_s] == [x["evals"] for x in h_p]


def test_pack_six_arrays():
    rng = np.random.default_rng(3)
    N = 5
    th = (rng.normal(size=N), rng.normal(size=N)) + tuple(
        rng.normal(size=(4, N)) + 1j * rng.normal(size=(4, N)) for _ in range(4))
    x = rmft.pack(th)
    assert x.shape == (34 * N,)
    for a, b in zip(rmft.unpack(x, N, spin=True), th):
        assert np.array_equal(a, b)
