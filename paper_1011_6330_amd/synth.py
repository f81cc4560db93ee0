"""Seeded synthetic inputs and preset tube configurations.

This module holds no step of the method: only configuration numbers and
seeded particle loads.  The same arrays feed the GPU library and the CPU
oracle (through their ``inject`` calls), so neither side draws random numbers.

Random numbers: raw 64-bit words of NumPy's ``Philox`` bit generator (a
counter-based generator with a stable, published bit stream), mapped to
[0, 1) as ``(w >> 11) * 2**-53``.

Presets follow the paper's runs (sec. 3): c = 1, R = 1, dt = dz/2, and the
dimensionless strength a = omega_p R / c sets the charge-to-mass ratio through
omega_p^2 = 4 pi |rho_GJ| |q/m| (normalisation of sec. 3).
"""
import math

import numpy as np

RHO_UNIFORM, RHO_FRAME_DRAG, RHO_KNOTS, RHO_GR = 0, 1, 2, 3


def q_over_m_for(a, amp=1.0, radius=1.0):
    """Electron q/m giving omega_p R / c = a for a background of amplitude amp."""
    return -(a * a) / (4.0 * math.pi * amp * radius * radius)


PRESETS = {
    # flat-space SCLF, cold start (empty tube, injection from step 1)
    "c1": dict(n_cells=1024, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0,
               rho_kind=RHO_UNIFORM, rho_amp=1.0, kappa=0.0, r_star=10.0, fp_bits=32,
               sort_every=0, capacity=1 << 16, flags=0, steps=2000, warm=0),
    # same dz, a tube four times longer (the front passes 30R)
    "c1_long": dict(n_cells=4096, length=40.0, radius=1.0, dt_over_dz=0.5, q_over_m=-1.0, ppc=4.0,
                    rho_kind=RHO_UNIFORM, rho_amp=1.0, kappa=0.0, r_star=10.0, fp_bits=32,
                    sort_every=0, capacity=1 << 17, flags=0, steps=7000, warm=0),
    # frame dragging, the paper's (R, omega_p) = (6253, 1.1) pair: a = 6878, 65,536 cells,
    # about 4e7 particles warm-started with gamma up to ~6e6, cell sort every 64 steps
    "c2": dict(n_cells=65536, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=q_over_m_for(6878.0),
               ppc=610.0, rho_kind=RHO_FRAME_DRAG, rho_amp=1.0, kappa=0.15, r_star=10.0,
               fp_bits=32, sort_every=64, capacity=int(610 * 65536 * 1.05), flags=0, steps=20000,
               warm=610 * 65536),
    # the frame-dragging tube with the whole of eq. (6): redshift (r_g/R_* = 0.4) and the
    # inclination term of the paper's standard pulsar (i = 0.5 rad, theta_* = 0.67 theta_p,
    # theta_p = 0.014, varphi = 0)
    "c2gr": dict(n_cells=65536, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=q_over_m_for(6878.0),
                 ppc=610.0, rho_kind=RHO_GR, rho_amp=1.0, kappa=0.15, r_star=10.0, incl=0.5,
                 theta_star=0.67 * 0.014, cos_phi=1.0, rg_over_rstar=0.4,
                 fp_bits=32, sort_every=64, capacity=int(610 * 65536 * 1.05), flags=0, steps=20000,
                 warm=610 * 65536),
    # adjoint workload: 4096 cells, 64 knots, about 1e6 particles
    # (the macro charge is fixed at its nominal value so that it does not move with the knots)
    "c4": dict(n_cells=4096, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=q_over_m_for(430.0),
               ppc=244.0, rho_kind=RHO_KNOTS, rho_amp=1.0, kappa=0.15, r_star=10.0,
               knots=np.ones(64), fp_bits=32, sort_every=0, capacity=int(244 * 4096 * 1.3),
               flags=0, steps=1000, warm=244 * 4096, macro_charge=-(1.0 - 0.15) * (10.0 / 4096) / 244.0),
    # large tube: 2^20 cells, L = 100R, the paper's (10317, 0.66) pair: a = 6809, ~2.5e8 particles
    "c5": dict(n_cells=1 << 20, length=100.0, radius=1.0, dt_over_dz=0.5, q_over_m=q_over_m_for(6809.0),
               ppc=238.4, rho_kind=RHO_FRAME_DRAG, rho_amp=1.0, kappa=0.15, r_star=10.0,
               fp_bits=32, sort_every=16, capacity=int(250_000_000 * 1.02), flags=0, steps=5000,
               warm=250_000_000),
}


def preset(name, **over):
    """A copy of a preset with overrides; bench/test metadata keys stay in the dict."""
    c = dict(PRESETS[name])
    if c.get("knots") is not None:
        c["knots"] = np.array(c["knots"], dtype=np.float64)
    c.update(over)
    return c


def tube_params(cfg):
    """The keys the library and the oracle take (drops the metadata)."""
    return {k: v for k, v in cfg.items() if k not in ("steps", "warm")}


def uniform01(n, seed=0, stream=0):
    """n doubles in [0, 1) from the Philox stream (seed, stream)."""
    bg = np.random.Philox(key=[int(seed), int(stream)])
    w = bg.random_raw(int(n)).astype(np.uint64)
    return (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def warm_start(cfg, n_particles=None, seed=0):
    """A flowing beam already filling the tube.

    Positions are stratified in cell units, x_p = (p + U_p) N / N_p (sorted).
    Momenta follow a smooth synthetic Lorentz-factor shape of the frame-dragging
    runs (sec. 3, Fig. 5): gamma rises from 1 at the surface over one tube radius
    and saturates at the screened frame-dragging potential a^2 kappa (1 - eta^-3),
    eta = 1 + z/R_*, with a^2 = 4 pi A |q/m| R^2.  This only shapes the input;
    the step starts from it and the fields are solved from the loaded charge.
    """
    N = int(cfg["n_cells"])
    n = int(cfg["warm"] if n_particles is None else n_particles)
    if n <= 0:
        return np.zeros(0), np.zeros(0)
    L, R = float(cfg["length"]), float(cfg["radius"])
    U = uniform01(n, seed, stream=1)
    x = (np.arange(n, dtype=np.float64) + U) * (N / n)
    x = np.minimum(x, np.nextafter(float(N), 0.0))
    z = x * (L / N)
    a2 = 4.0 * math.pi * float(cfg["rho_amp"]) * abs(float(cfg["q_over_m"])) * R * R
    kappa = float(cfg.get("kappa", 0.0))
    rs = float(cfg.get("r_star", 10.0))
    eta = 1.0 + z / rs
    shape = (1.0 - eta ** -3) * (1.0 - np.exp(-z / R))
    if kappa > 0:
        g = 1.0 + a2 * kappa * shape
    else:  # flat space: the SCLF plateau sqrt(2) a reached within a few radii
        g = 1.0 + math.sqrt(2.0 * a2) * (1.0 - np.exp(-z / R))
    u = np.sqrt(g * g - 1.0)
    return x, u


def random_particles(N, n, seed=0, u_lo=-3.0, u_hi=40.0, stream=2):
    """Unsorted particles uniform in [0, N) with momenta uniform in [u_lo, u_hi)."""
    x = uniform01(n, seed, stream) * N
    x = np.minimum(x, np.nextafter(float(N), 0.0))
    u = u_lo + (u_hi - u_lo) * uniform01(n, seed, stream + 100)
    return x, u


def ensemble(n_tubes=256, seed=0, precision=1, sort_every=64, slack=1.3, dense=False):
    """Tubes of the batched workload: per tube t, four uniforms from Philox stream
    1000 + t give N_t = round(2048 * 32^U1) cells (2,048 .. 65,536), kappa_t =
    0.05 + 0.15 U2, A_t = 0.3 * 10^U3 (0.3 .. 3), N_p,t = round(1e4 * 100^U4)
    particles (1e4 .. 1e6); L = 10R, R_* = 10R and a_t = 1.05 (N_t / 10) sqrt(A_t),
    i.e. omega_p dz / c = 1.05 in every tube, as in the frame-dragging preset.
    dense: a control with the same tube count and about the same particle total,
    every tube 2,048 cells and 2.2e5 particles (about 107 per cell)."""
    out = []
    for t in range(n_tubes):
        U = uniform01(4, seed, stream=1000 + t)
        N = 2048 if dense else int(round(2048 * 32.0 ** U[0]))
        kappa = 0.05 + 0.15 * U[1]
        amp = 0.3 * 10.0 ** U[2]
        npart = 220000 if dense else int(round(1e4 * 100.0 ** U[3]))
        a = 1.05 * (N / 10.0) * math.sqrt(amp)
        out.append(dict(n_cells=N, length=10.0, radius=1.0, dt_over_dz=0.5, q_over_m=q_over_m_for(a, amp),
                        ppc=npart / N, rho_kind=RHO_FRAME_DRAG, rho_amp=amp, kappa=kappa, r_star=10.0,
                        fp_bits=32, sort_every=sort_every, capacity=int(npart * slack) + 4096, flags=0,
                        precision=precision, steps=2000, warm=npart))
    return out
