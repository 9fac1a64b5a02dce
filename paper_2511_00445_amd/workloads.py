"""Seeded synthetic workloads: parameter presets and initial conditions.

This module is shared by the tests, the benchmark and the smoke check. It holds
no arithmetic of the method itself: it only draws random numbers and lays out
the initial fields that the paper's Numerical Simulation section describes
(a homogeneous composition with small uniform noise, zero velocities), with the
nematic part drawn as a random director field at a fixed order S (Q = 2S(pp - I/2),
Model section, nematic order parameter equation).

Arrays are float64, shape [ny, nx], row-major with x fastest.

Parameter names (shared by the C header, the binding and the oracle):
  rho0            reference density of each fluid (paper: rho_1 = rho_2)
  tau_a, tau_p    BGK relaxation times of the active / passive fluid (viscosity (tau-1/2)/3)
  gamma           inter-fluid drag coefficient of F_drag
  A_ch, kappa, M  Cahn-Hilliard: mu = A_ch (phi^3 - phi) - kappa lap(phi), mobility M
  A0, gamma_ldg   Landau-de Gennes bulk energy in the (A0, gamma) form (gamma = 3: the
                  two-dimensional isotropic-nematic point)
  K               Frank elastic constant
  lam             tumbling (flow-alignment) parameter lambda
  Gamma           rotational diffusion constant of the Beris-Edwards equation
  zeta            activity (zeta > 0 extensile)
  n_sub           finite-difference sub-steps per lattice-Boltzmann step
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("nx", "ny", "rho0", "tau_a", "tau_p", "gamma", "A_ch", "kappa", "M",
               "A0", "gamma_ldg", "K", "lam", "Gamma", "zeta", "n_sub")


def base_params(nx: int, ny: int, **over) -> dict:
    """The small-grid parameter set (64x64 case) with any field overridden."""
    p = dict(nx=int(nx), ny=int(ny), rho0=1.0, tau_a=1.0, tau_p=1.0, gamma=0.01,
             A_ch=0.04, kappa=0.04, M=0.1, A0=0.1, gamma_ldg=3.0, K=0.04,
             lam=0.7, Gamma=0.34, zeta=0.005, n_sub=5)
    for k, v in over.items():
        if k not in p:
            raise KeyError(f"unknown parameter {k!r}")
        p[k] = v
    return p


# Named workloads. Each: grid, steps, parameter overrides, composition mean, seed.
WORKLOADS = {
    # 64x64, 200 steps, pointwise parity at step 100
    "small_64": dict(nx=64, ny=64, steps=200, over={}, phi_mean=0.0, seeds=(0,)),
    # 512x512 single active run, zeta = 0.01, 20,000 steps
    "active_512": dict(nx=512, ny=512, steps=20000, over=dict(zeta=0.01), phi_mean=0.0,
                       seeds=(1, 2, 3)),
    # 2048x2048 precision-study grid, 50,000 steps, zeta in {0, 0.005, 0.02}
    "large_2048": dict(nx=2048, ny=2048, steps=50000, over=dict(zeta=0.02), phi_mean=0.0,
                       seeds=(4,)),
}


def workload_params(name: str, **extra) -> dict:
    w = WORKLOADS[name]
    over = dict(w["over"])
    over.update(extra)
    return base_params(w["nx"], w["ny"], **over)


def initial_fields(nx: int, ny: int, seed: int, phi_mean: float = 0.0,
                   phi_noise: float = 0.01, S0: float = 0.1) -> dict:
    """Seeded initial condition.

    phi = phi_mean + U(-phi_noise, phi_noise); director angle theta ~ U[0, pi);
    Qxx = S0 cos(2 theta), Qxy = S0 sin(2 theta) (so Q = 2 S0 (pp - I/2));
    velocities are zero.  Draw order: phi noise, then theta.
    """
    rng = np.random.default_rng(seed)
    phi = phi_mean + rng.uniform(-phi_noise, phi_noise, size=(ny, nx))
    theta = rng.uniform(0.0, np.pi, size=(ny, nx))
    return dict(phi=phi, qxx=S0 * np.cos(2.0 * theta), qxy=S0 * np.sin(2.0 * theta))


def random_velocity(nx: int, ny: int, seed: int, amp: float = 1e-3) -> np.ndarray:
    """A seeded smooth-free random velocity plane pair [2, ny, nx] (ux, uy)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, size=(2, ny, nx))


def sweep_members(count: int = 64, seed: int = 5) -> list:
    """The batched parameter sweep: `count` members with square sizes drawn from
    {128, 256, 512} and zeta in [0, 0.02], lam in [0.3, 1.0], K in [0.01, 0.1],
    mean composition in [-0.4, 0.4] (uniform, seeded); per-member initial-condition
    seed 5000 + i.  Returns a list of dicts: params, phi_mean, seed."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice([128, 256, 512], size=count)
    zeta = rng.uniform(0.0, 0.02, size=count)
    lam = rng.uniform(0.3, 1.0, size=count)
    K = rng.uniform(0.01, 0.1, size=count)
    phibar = rng.uniform(-0.4, 0.4, size=count)
    out = []
    for i in range(count):
        n = int(sizes[i])
        out.append(dict(params=base_params(n, n, zeta=float(zeta[i]), lam=float(lam[i]), K=float(K[i])),
                        phi_mean=float(phibar[i]), seed=5000 + i))
    return out
