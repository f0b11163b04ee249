"""Run the self-consistent RMFT iteration (kpm_rmft_iterate) on a vortex
lattice, in chunks, writing a restart file after every chunk.

    python -m paper_2212_05685_amd.rmft_run --iters 300 --chunk 25 --save state.npz
    python -m paper_2212_05685_amd.rmft_run --resume state.npz --iters 100 --save more.npz

The default problem is the plain-vortex workload of the Results section:
48 x 96 torus, two vortices half the lattice apart in y, mean hole density
0.16, M = 1024, 128 colored probes, FP32 recursion.  The seed comes from
``workloads`` (repository root on the path).  After the run, the renormalized
pairing amplitude around each vortex is fitted to D0 tanh(r / xi) (Results:
the paper reports a core size of about three lattice constants for this
state); the fit is host-side reporting, outside the iteration.  The vortices
are free to move during the iteration (the field is uniform), so the fit
starts from the amplitude minima of the final state, not from the seed.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch


def bond_phase(x, y, d, Lx, Ly, nv):
    """Peierls phase of the bond (x, y) -> (x, y) + d, d = 0 (+x) or 1 (+y),
    in the library's gauge (kpm_build_H: Landau gauge A = B(0, x) with the
    seam twist on +x steps across the torus edge)."""
    dx, dy = (1, 0) if d == 0 else (0, 1)
    phi = -np.pi * nv * (x + 0.5 * dx) * dy / (Lx * Ly)
    seam = (x + dx) == Lx
    return phi + np.where(seam, np.pi * nv * ((y + dy) % Ly) / Ly, 0.0)


def pairing_field(n, dlt, Lx, Ly, nv):
    """Renormalized site pairing of the Results section (eq. giDelta) for a
    spin-singlet state: Delta_i = (1/4) sum over tau = +-x, +-y of
    g^t_ij (-1)^{tau_y} Delta_ij e^{-i phi_ij}, j = i + tau, phi_ij the bond's
    Peierls phase (so the factor is the paper's e^{i (pi/Phi0) int A.dr}),
    g^t_ij = g_i g_j, g_i = sqrt(2 delta_i / (1 + delta_i)); the spin sum
    gives the factor 2 over the paper's 1/8."""
    d = 1.0 - n
    g = np.sqrt(2.0 * d / (1.0 + d))
    idx = np.arange(Lx * Ly)
    x, y = idx % Lx, idx // Lx
    jx = ((x + 1) % Lx) + y * Lx
    jy = x + ((y + 1) % Ly) * Lx
    bx = g * g[jx] * dlt[0] * np.exp(-1j * bond_phase(x, y, 0, Lx, Ly, nv))     # tau = +x
    by = g * g[jy] * dlt[1] * np.exp(-1j * bond_phase(x, y, 1, Lx, Ly, nv))     # tau = +y
    mx = ((x - 1) % Lx) + y * Lx
    my = x + ((y - 1) % Ly) * Lx
    # tau = -x, -y: the bond stored at i - tau, traversed backwards (conjugate factor)
    bxm = g * g[mx] * dlt[0][mx] * np.exp(1j * bond_phase(x[mx], y[mx], 0, Lx, Ly, nv))
    bym = g * g[my] * dlt[1][my] * np.exp(1j * bond_phase(x[my], y[my], 1, Lx, Ly, nv))
    return 0.25 * (bx + bxm - by - bym)


def core_fit(amp, Lx, Ly, centres, rmax=12.0):
    """Least-squares fit of amp(r) = D0 tanh(r / xi) around each vortex, the
    centre (cx, cy) fitted too, starting from the amplitude minimum nearest
    the given point, over the sites within rmax of that minimum; r is the
    minimum-image distance."""
    from scipy.optimize import least_squares

    idx = np.arange(Lx * Ly)
    x, y = idx % Lx, idx // Lx
    out = []
    for (X, Y) in centres:
        dx0 = (x - X + Lx / 2) % Lx - Lx / 2
        dy0 = (y - Y + Ly / 2) % Ly - Ly / 2
        near = np.hypot(dx0, dy0) <= 6.0
        c = idx[near][np.argmin(amp[near])]
        sel = np.hypot((x - c % Lx + Lx / 2) % Lx - Lx / 2, (y - c // Lx + Ly / 2) % Ly - Ly / 2) <= rmax
        xs, ys, a = x[sel], y[sel], amp[sel]

        def resid(p):
            d0, xi, cx, cy = p
            r = np.hypot((xs - cx + Lx / 2) % Lx - Lx / 2, (ys - cy + Ly / 2) % Ly - Ly / 2)
            return d0 * np.tanh(r / abs(xi)) - a

        sol = least_squares(resid, [float(amp.max()), 2.0, float(c % Lx), float(c // Lx)])
        d0, xi, cx, cy = sol.x
        out.append({"centre": [float(cx % Lx), float(cy % Ly)], "D0": float(d0), "xi": float(abs(xi)),
                    "rms": float(np.sqrt(np.mean(sol.fun ** 2))), "amp_min": float(amp[c])})
    return out


def vortex_positions(amp, Lx, Ly, k):
    """The k lowest local minima of amp that are at least Ly/4 apart."""
    order = np.argsort(amp)
    picked = []
    for i in order:
        x, y = i % Lx, i // Lx
        if all(np.hypot((x - px + Lx / 2) % Lx - Lx / 2, (y - py + Ly / 2) % Ly - Ly / 2) >= Ly / 4
               for px, py in picked):
            picked.append((x, y))
        if len(picked) == k:
            break
    return picked


def main(argv=None):
    import workloads as wl
    from . import kpm
    from .solver import KPMProblem, load_rmft_state, save_rmft_state

    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--lx", type=int, default=48)
    ap.add_argument("--ly", type=int, default=96)
    ap.add_argument("--nv", type=int, default=2)
    ap.add_argument("--doping", type=float, default=0.16)
    ap.add_argument("--moments", type=int, default=1024)
    ap.add_argument("--core", type=float, default=3.0, help="tanh radius of the vortex seed")
    ap.add_argument("--vortex-dx", type=float, default=0.0,
                    help="shift of the seeded vortex centres along x (24.5 puts the 48-wide "
                         "lattice's pair on the x seam, where the gauge's torus holonomy holds them)")
    ap.add_argument("--color", type=int, default=8,
                    help="distance coloring of the probes: c x c colours, each split by Nambu component "
                         "(2 c^2 probes per draw; c must divide both sides)")
    ap.add_argument("--draws", type=int, default=1,
                    help="independent Z4 phase draws of the colored probe set, each of weight 1/draws")
    ap.add_argument("--precision", choices=("fp32", "fp64"), default="fp32")
    ap.add_argument("--mix", type=float, default=0.1)
    ap.add_argument("--tol-n", type=float, default=1e-5)
    ap.add_argument("--search", choices=("illinois", "bisection"), default="illinois")
    ap.add_argument("--estimator", choices=("adjoint", "direct"), default="adjoint")
    ap.add_argument("--anderson", type=int, default=0, help="Anderson history depth (0: linear mixing)")
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--chunk", type=int, default=25)
    ap.add_argument("--tol-residual", type=float, default=0.0)
    ap.add_argument("--resume", default="")
    ap.add_argument("--save", default="")
    args = ap.parse_args(argv)

    cfg = wl.scaled(wl.RMFT(args.precision), Lx=args.lx, Ly=args.ly, n_v=args.nv, doping=args.doping,
                    M=args.moments, core=args.core, vortex_dx=args.vortex_dx)
    if args.color != 8 or args.draws != 1:
        if args.lx % args.color or args.ly % args.color or args.draws < 1:
            ap.error("--color must divide both lattice sides and --draws must be positive")
        base = cfg.probes[0]
        cfg = wl.scaled(cfg, probes=(wl.ProbeSpec("colored_z4", args.draws, base.seed, args.color, args.color,
                                                  1, 0, 1.0 / args.draws),))
    kinds = {"unit": kpm.KPM_PROBE_UNIT, "dense_z4": kpm.KPM_PROBE_DENSE_Z4,
             "colored_z4": kpm.KPM_PROBE_COLORED_Z4}
    specs = [kpm.ProbeSpec(kinds[p.kind], p.count, p.seed, p.px, p.py, p.split_nambu, p.first, p.weight)
             for p in cfg.probes]
    prec = kpm.KPM_FP32 if args.precision == "fp32" else kpm.KPM_FP64
    prob = KPMProblem(cfg.Lx, cfg.Ly, cfg.n_v, cfg.t, cfg.tp, cfg.J, cfg.mu, cfg.T, cfg.M, specs, prec,
                      cfg.ckpt_k)
    if args.resume:
        n, chi, dlt, mu, hist = load_rmft_state(args.resume)
    else:
        n0, chi0, dlt0 = wl.make_theta(cfg)
        n, chi, dlt = (torch.from_numpy(n0).cuda(), torch.from_numpy(chi0).cuda(),
                       torch.from_numpy(dlt0).cuda())
        mu, hist = cfg.mu, []
    search = kpm.KPM_RMFT_ILLINOIS if args.search == "illinois" else kpm.KPM_RMFT_BISECTION
    est = kpm.KPM_RMFT_DIRECT if args.estimator == "direct" else kpm.KPM_RMFT_ADJOINT
    prm = kpm.rmft_params(cfg.doping, mix=args.mix, tol_n=args.tol_n, tol_mu=1e-9, mu_step=0.004,
                          tol_residual=args.tol_residual, max_evals=60, search=search, estimator=est,
                          anderson=args.anderson)
    t0 = time.perf_counter()
    done = 0
    st = kpm.KPM_OK
    while done < args.iters:
        k = min(args.chunk, args.iters - done)
        mu, h, st = prob.rmft_iterate(n, chi, dlt, mu, prm, k)
        hist += h
        done += len(h)
        if args.save:
            save_rmft_state(args.save, n, chi, dlt, mu, hist)
        last = h[-1] if h else None
        print(f"[rmft] {len(hist)} iterations, {time.perf_counter() - t0:.1f} s, mu {mu:.6f}, "
              f"residual {last['residual'] if last else float('nan'):.3e}, "
              f"evaluations {sum(x['evals'] for x in h)}", file=sys.stderr, flush=True)
        if st != kpm.KPM_OK or len(h) < k:
            break
    torch.cuda.synchronize()
    nn, dd = n.cpu().numpy(), dlt.cpu().numpy()
    amp = np.abs(pairing_field(nn, dd, cfg.Lx, cfg.Ly, cfg.n_v))
    summary = {
        "iterations": len(hist), "seconds": time.perf_counter() - t0, "mu": mu, "probes": cfg.R,
        "residual_last": hist[-1]["residual"] if hist else None, "status": st,
        "evaluations": int(sum(x["evals"] for x in hist)),
        "hole_density_min_max": [float(1 - nn.max()), float(1 - nn.min())],
        "cores": core_fit(amp, cfg.Lx, cfg.Ly, vortex_positions(amp, cfg.Lx, cfg.Ly, cfg.n_v))
        if cfg.n_v else [],
    }
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
