"""FP64 CPU oracle of the two-fluid active-nematic coupled lattice update.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import or call this module.  It shares no code with the
HIP path and the product never calls it.

What it computes (arXiv 2511.00445, "Model" and "Numerical Simulation" sections):
one coupled time step of an active nematic fluid (velocity u1 = u_a) mixed with a
passive Newtonian fluid (u2 = u_p) on a 2D periodic lattice:

  * two D2Q9 BGK lattice-Boltzmann fluids with Guo forcing (Numerical Simulation),
    coupled by the drag F_drag = gamma c1 c2 (u_p - u_a) (Model, drag force);
  * the elastic stress of the Beris-Edwards model (Model, elastic stress display),
    the active stress -zeta c1 Q (Model, active force; sign: zeta > 0 extensile)
    and the capillary force F_ch = mu grad(phi) - grad(phi mu) (Model, capillary
    force equation), discretised term by term;
  * n_sub forward-Euler finite-difference sub-steps of the Cahn-Hilliard equation
    (Model, Eqs. 1-3) and the Beris-Edwards equation (Model, Eqs. 11-12) with the
    velocities frozen at the start of the step (Numerical Simulation).

Every tensor is carried as a full 2x2 field, exactly as the paper writes the
formulas; nothing is simplified with two-dimensional identities.  Lattice units
dx = dt = 1 with finite-difference sub-step h = 1/n_sub.

Readings taken where the paper is silent or ambiguous (each also in the design notes):
  * phi is the order parameter in [-1, 1]; the fractions the paper calls phi and
    (1 - phi) are c1 = (1 + phi)/2 and c2 = (1 - phi)/2.  The chemical potential is
    mu = A_ch (phi^3 - phi) - kappa lap(phi), the paper's f'(phi) - eps^2 lap(phi)
    written for that order parameter.
  * Each lattice-Boltzmann fluid is a full-density fluid (rho0, viscosity from tau);
    the active and elastic forces act on the active fluid, the capillary force is
    shared c1 : c2, the drag is an equal and opposite exchange.
  * Stress divergence F_i = sum_j d_j sigma_ij; velocity gradient W_ij = d_j u_i.
  * Guo's half-force velocity rho u = m + F/2 is implicit through the drag; it is
    solved exactly per site as a 2x2 linear system.
  * Central differences: d_x g = (g(x+1) - g(x-1))/2, 5-point Laplacian.
  * The Beris-Edwards right-hand side is projected onto symmetric traceless
    tensors before it is applied (it acquires a trace lam*tr(W) in a weakly
    compressible flow).
  * The isotropic (pressure-like) part of the nematic stress is not added.
"""
from __future__ import annotations

import numpy as np

# D2Q9 lattice (Numerical Simulation section): velocities c_i and weights w_i.
CI = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1],
               [1, 1], [-1, 1], [-1, -1], [1, -1]], dtype=np.int64)
WI = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=np.float64)
CS2 = 1.0 / 3.0  # lattice sound speed squared

PARAM_KEYS = ("nx", "ny", "rho0", "tau_a", "tau_p", "gamma", "A_ch", "kappa", "M",
              "A0", "gamma_ldg", "K", "lam", "Gamma", "zeta", "n_sub")


# ----------------------------------------------------------------------------
# periodic finite differences (Numerical Simulation: second-order central FD,
# periodic in both directions)
# ----------------------------------------------------------------------------
def shift(g, dx, dy):
    """g evaluated at (x + dx, y + dy); the last two axes are (y, x)."""
    return np.roll(g, shift=(-dy, -dx), axis=(-2, -1))


def d_x(g):
    return 0.5 * (shift(g, 1, 0) - shift(g, -1, 0))


def d_y(g):
    return 0.5 * (shift(g, 0, 1) - shift(g, 0, -1))


def lap(g):
    return shift(g, 1, 0) + shift(g, -1, 0) + shift(g, 0, 1) + shift(g, 0, -1) - 4.0 * g


# ----------------------------------------------------------------------------
# 2x2 tensor fields: shape [2, 2, ny, nx], T[i, j] is component ij.
# ----------------------------------------------------------------------------
def eye_field(shape):
    I = np.zeros((2, 2) + shape)
    I[0, 0] = 1.0
    I[1, 1] = 1.0
    return I


def mm(A, B):
    """Matrix product of two tensor fields, (A.B)_ij = sum_k A_ik B_kj."""
    return np.einsum("ik...,kj...->ij...", A, B)


def ddot(A, B):
    """Double contraction A:B = sum_ij A_ij B_ij."""
    return np.einsum("ij...,ij...->...", A, B)


def transpose(A):
    return np.swapaxes(A, 0, 1)


def q_tensor(qxx, qxy):
    """Symmetric traceless Q from its two independent components (Model, Q = 2S(pp - I/2))."""
    return np.array([[qxx, qxy], [qxy, -qxx]])


def grad_vector(u):
    """W_ij = d_j u_i for a vector field u of shape [2, ny, nx]."""
    return np.array([[d_x(u[0]), d_y(u[0])], [d_x(u[1]), d_y(u[1])]])


# ----------------------------------------------------------------------------
# Cahn-Hilliard pieces (Model, Eqs. 1-3; reading: order parameter phi in [-1, 1])
# ----------------------------------------------------------------------------
def chemical_potential(phi, A_ch, kappa):
    """mu = f'(phi) - kappa lap(phi) with f = (A_ch/4)(phi^2 - 1)^2."""
    return A_ch * (phi ** 3 - phi) - kappa * lap(phi)


def ch_rhs(phi, uc, p):
    """Right-hand side of d_t phi = -div(phi u_c) + M lap(mu) (Model, Eq. 1)."""
    mu = chemical_potential(phi, p["A_ch"], p["kappa"])
    return -(d_x(phi * uc[0]) + d_y(phi * uc[1])) + p["M"] * lap(mu)


def capillary_force(phi, mu):
    """F_ch = mu grad(phi) - grad(phi mu) (Model, capillary force), each gradient by
    the central differences of the method, term by term as the paper writes it.
    (The continuum identity -phi grad(mu) does not hold discretely: the central
    difference of a product differs from the product rule, and the term-by-term
    form takes mu's differences across the two neighbouring faces.)"""
    return np.array([mu * d_x(phi) - d_x(phi * mu), mu * d_y(phi) - d_y(phi * mu)])


# ----------------------------------------------------------------------------
# Landau-de Gennes / Beris-Edwards pieces (Model, Eqs. 7, 8, 11, 12 and the
# elastic stress display)
# ----------------------------------------------------------------------------
def landau_coefficients(A0, gamma_ldg):
    """Bulk coefficients (A, B, C) of (A/2)TrQ^2 + (B/3)TrQ^3 + (C/4)TrQ^4 (Model, Eq. 8)
    for the workloads' (A0, gamma) parameters.  Reading: the (A0, gamma) form of the
    Landau-de Gennes energy, (A0/2)(1 - gamma/3) TrQ^2 - (A0 gamma/3) TrQ^3
    + (A0 gamma/4)(TrQ^2)^2, written in the paper's form; for a symmetric traceless
    2x2 Q, TrQ^4 = (TrQ^2)^2 / 2, so the quartic coefficient is C = 2 A0 gamma."""
    return A0 * (1.0 - gamma_ldg / 3.0), -A0 * gamma_ldg, 2.0 * A0 * gamma_ldg


def free_energy_derivative(Q, A, B, C, K):
    """dF/dQ of F = (A/2)TrQ^2 + (B/3)TrQ^3 + (C/4)TrQ^4 + (K/2)|grad Q|^2 (Model, Eq. 8)."""
    Q2 = mm(Q, Q)
    Q3 = mm(Q2, Q)
    return A * Q + B * transpose(Q2) + C * transpose(Q3) - K * lap(Q)


def molecular_field(Q, A, C, K, B=0.0):
    """H = -dF/dQ + (I/2) Tr(dF/dQ) (Model, Eq. 7)."""
    dF = free_energy_derivative(Q, A, B, C, K)
    tr = dF[0, 0] + dF[1, 1]
    return -dF + 0.5 * eye_field(Q.shape[2:]) * tr


def ericksen_stress(Q, K):
    """(grad Q) . dF/d(grad Q): entry ij is sum_kl (d_i Q_kl)(K d_j Q_kl)."""
    dQ = np.array([d_x(Q), d_y(Q)])  # dQ[i] = d_i Q, shape [2, 2, 2, ny, nx]
    return K * np.einsum("ikl...,jkl...->ij...", dQ, dQ)


def elastic_stress(Q, H, lam, K):
    """Beris-Edwards elastic stress (Model, elastic stress display), P = Q + I/2:
    -lam H.P - lam P.H + 2 lam P (Q:H) - (grad Q).dF/d(grad Q) + Q.H - H.Q."""
    P = Q + 0.5 * eye_field(Q.shape[2:])
    QH = ddot(Q, H)
    return (-lam * mm(H, P) - lam * mm(P, H) + 2.0 * lam * P * QH
            - ericksen_stress(Q, K) + mm(Q, H) - mm(H, Q))


def active_stress(Q, c1, zeta):
    """Active stress localised on the active fraction, -zeta c1 Q (Model, active force;
    zeta > 0 extensile)."""
    return -zeta * c1 * Q


def divergence(sigma):
    """F_i = sum_j d_j sigma_ij."""
    return np.array([d_x(sigma[0, 0]) + d_y(sigma[0, 1]),
                     d_x(sigma[1, 0]) + d_y(sigma[1, 1])])


def corotation(W, Q, lam):
    """S(W, Q) = (lam E + Om).P + P.(lam E - Om) - 2 lam P (Q:W) (Model, Eq. 12),
    E = (W + W^T)/2, Om = (W - W^T)/2, P = Q + I/2."""
    E = 0.5 * (W + transpose(W))
    Om = 0.5 * (W - transpose(W))
    P = Q + 0.5 * eye_field(Q.shape[2:])
    return mm(lam * E + Om, P) + mm(P, lam * E - Om) - 2.0 * lam * P * ddot(Q, W)


def be_rhs(Q, ua, W, p):
    """Full-tensor right-hand side of d_t Q = -u_a.grad Q + S(W, Q) + Gamma H (Model, Eq. 11)."""
    A, B, C = landau_coefficients(p["A0"], p["gamma_ldg"])
    H = molecular_field(Q, A, C, p["K"], B=B)
    adv = -(ua[0] * d_x(Q) + ua[1] * d_y(Q))
    return adv + corotation(W, Q, p["lam"]) + p["Gamma"] * H


def project_sym_traceless(R):
    """(Rxx - Ryy)/2 and (Rxy + Ryx)/2: the two components of the symmetric traceless part."""
    return 0.5 * (R[0, 0] - R[1, 1]), 0.5 * (R[0, 1] + R[1, 0])


# ----------------------------------------------------------------------------
# Lattice Boltzmann pieces (Numerical Simulation: D2Q9 BGK, Guo forcing)
# ----------------------------------------------------------------------------
def equilibrium(rho, u):
    """f_i^eq = w_i rho [1 + c.u/cs2 + (c.u)^2/(2 cs2^2) - u.u/(2 cs2)]."""
    cu = np.einsum("ia,a...->i...", CI.astype(np.float64), u)
    uu = u[0] ** 2 + u[1] ** 2
    return WI[:, None, None] * rho * (1.0 + cu / CS2 + 0.5 * cu ** 2 / CS2 ** 2 - 0.5 * uu / CS2)


def guo_source(u, F, tau):
    """Guo forcing term (1 - 1/(2 tau)) w_i [(c_i - u)/cs2 + (c_i.u) c_i/cs2^2] . F."""
    c = CI.astype(np.float64)
    cu = np.einsum("ia,a...->i...", c, u)
    cF = np.einsum("ia,a...->i...", c, F)
    uF = u[0] * F[0] + u[1] * F[1]
    return (1.0 - 0.5 / tau) * WI[:, None, None] * ((cF - uF) / CS2 + cu * cF / CS2 ** 2)


def moments(f):
    """rho = sum_i f_i and m = sum_i f_i c_i."""
    rho = f.sum(axis=0)
    m = np.einsum("ia,i...->a...", CI.astype(np.float64), f)
    return rho, m


def collide(f, rho, u, F, tau):
    """BGK collision with the Guo source: f* = f - (f - f^eq)/tau + S."""
    return f - (f - equilibrium(rho, u)) / tau + guo_source(u, F, tau)


def stream(fstar):
    """f_i(x + c_i) = f*_i(x) on the periodic lattice."""
    out = np.empty_like(fstar)
    for i in range(9):
        out[i] = np.roll(fstar[i], shift=(CI[i, 1], CI[i, 0]), axis=(0, 1))
    return out


def solve_velocities(rho_a, m_a, G_a, rho_p, m_p, G_p, beta):
    """Guo velocities with the drag implicit.  Unknowns u_a, u_p satisfy
    rho_a u_a = m_a + (G_a + beta (u_p - u_a))/2 and rho_p u_p = m_p + (G_p - beta (u_p - u_a))/2,
    beta = gamma c1 c2.  Solved per site and component as a 2x2 linear system."""
    g = 0.5 * beta
    mat = np.empty(rho_a.shape + (2, 2))
    mat[..., 0, 0] = rho_a + g
    mat[..., 0, 1] = -g
    mat[..., 1, 0] = -g
    mat[..., 1, 1] = rho_p + g
    rhs = np.empty(rho_a.shape + (2, 2))  # [..., fluid, component]
    rhs[..., 0, :] = np.moveaxis(m_a + 0.5 * G_a, 0, -1)
    rhs[..., 1, :] = np.moveaxis(m_p + 0.5 * G_p, 0, -1)
    sol = np.linalg.solve(mat, rhs)
    return np.moveaxis(sol[..., 0, :], -1, 0), np.moveaxis(sol[..., 1, :], -1, 0)


def guo_momenta(rho_a, u_a, G_a, rho_p, u_p, G_p, beta):
    """The momenta m_a, m_p whose Guo velocities (solve_velocities) are u_a, u_p:
    the two balance equations of solve_velocities solved for m instead of u."""
    drag = beta * (u_p - u_a)
    return rho_a * u_a - 0.5 * (G_a + drag), rho_p * u_p - 0.5 * (G_p - drag)


# ----------------------------------------------------------------------------
# The coupled step
# ----------------------------------------------------------------------------
def phi_extent(phi):
    """Largest |phi| over the sites: how far the order parameter leaves its bulk
    values +-1 (a health measure of a state, not an observable of the paper)."""
    return float(np.abs(phi).max())


class Oracle:
    """Plain FP64 solver.  State: pre-collision populations f_a, f_p [9, ny, nx]
    (the result of streaming), phi, Q components qxx, qxy [ny, nx], step counter."""

    def __init__(self, params: dict):
        p = {k: params[k] for k in PARAM_KEYS}
        p["nx"], p["ny"], p["n_sub"] = int(p["nx"]), int(p["ny"]), int(p["n_sub"])
        if p["tau_a"] <= 0.5 or p["tau_p"] <= 0.5 or p["n_sub"] < 1:
            raise ValueError("tau must exceed 1/2 and n_sub must be >= 1")
        self.p = p
        shape = (p["ny"], p["nx"])
        self.f_a = np.zeros((9,) + shape)
        self.f_p = np.zeros((9,) + shape)
        self.phi = np.zeros(shape)
        self.qxx = np.zeros(shape)
        self.qxy = np.zeros(shape)
        self.step_count = 0

    # -- state set-up ---------------------------------------------------------
    def init_fields(self, phi, qxx, qxy, u_a=None, u_p=None):
        """Fields at step 0; populations start at f^eq(rho0, u)."""
        shape = (self.p["ny"], self.p["nx"])
        self.phi = np.array(phi, dtype=np.float64).reshape(shape).copy()
        self.qxx = np.array(qxx, dtype=np.float64).reshape(shape).copy()
        self.qxy = np.array(qxy, dtype=np.float64).reshape(shape).copy()
        ua = np.zeros((2,) + shape) if u_a is None else np.array(u_a, np.float64).reshape((2,) + shape)
        up = np.zeros((2,) + shape) if u_p is None else np.array(u_p, np.float64).reshape((2,) + shape)
        rho = np.full(shape, self.p["rho0"])
        self.f_a = equilibrium(rho, ua)
        self.f_p = equilibrium(rho, up)
        self.step_count = 0

    def import_state(self, phi, qxx, qxy, u_a, u_p, rho_a, rho_p, step: int):
        """A state rebuilt from macroscopic fields (the surrogate's reconstruction, not
        a step of the paper): phi and Q as given; pre-collision populations at
        equilibrium with the given densities and with the momenta whose Guo
        velocities, under the forces of the given phi and Q, are the given ones."""
        shape = (self.p["ny"], self.p["nx"])
        self.phi = np.array(phi, np.float64).reshape(shape).copy()
        self.qxx = np.array(qxx, np.float64).reshape(shape).copy()
        self.qxy = np.array(qxy, np.float64).reshape(shape).copy()
        ua = np.array(u_a, np.float64).reshape((2,) + shape)
        up = np.array(u_p, np.float64).reshape((2,) + shape)
        ra = np.array(rho_a, np.float64).reshape(shape)
        rp = np.array(rho_p, np.float64).reshape(shape)
        fr = self.forces()
        m_a, m_p = guo_momenta(ra, ua, fr["G_a"], rp, up, fr["G_p"], self.p["gamma"] * fr["c1"] * fr["c2"])
        self.f_a = equilibrium(ra, m_a / ra)
        self.f_p = equilibrium(rp, m_p / rp)
        self.step_count = int(step)

    # -- steps 1-4: fractions, potentials, stresses, forces, velocities ---------
    def forces(self):
        """Fractions, chemical potential, Q, H, stress and the non-drag forces G_a, G_p
        of the current phi and Q."""
        p = self.p
        phi = self.phi
        c1 = 0.5 * (1.0 + phi)
        c2 = 0.5 * (1.0 - phi)
        mu = chemical_potential(phi, p["A_ch"], p["kappa"])
        Q = q_tensor(self.qxx, self.qxy)
        A, B, C = landau_coefficients(p["A0"], p["gamma_ldg"])
        H = molecular_field(Q, A, C, p["K"], B=B)
        sigma = elastic_stress(Q, H, p["lam"], p["K"]) + active_stress(Q, c1, p["zeta"])
        F_el_act = divergence(sigma)
        F_ch = capillary_force(phi, mu)
        return dict(c1=c1, c2=c2, mu=mu, Q=Q, H=H, sigma=sigma, G_a=F_el_act + c1 * F_ch, G_p=c2 * F_ch)

    def macroscopic(self):
        p = self.p
        fr = self.forces()
        c1, c2, mu, Q, H, sigma, G_a, G_p = (fr[k] for k in ("c1", "c2", "mu", "Q", "H", "sigma", "G_a", "G_p"))
        rho_a, m_a = moments(self.f_a)
        rho_p, m_p = moments(self.f_p)
        beta = p["gamma"] * c1 * c2
        u_a, u_p = solve_velocities(rho_a, m_a, G_a, rho_p, m_p, G_p, beta)
        F_drag = beta * (u_p - u_a)
        return dict(c1=c1, c2=c2, mu=mu, Q=Q, H=H, sigma=sigma, G_a=G_a, G_p=G_p,
                    rho_a=rho_a, rho_p=rho_p, m_a=m_a, m_p=m_p, u_a=u_a, u_p=u_p,
                    F_a=G_a + F_drag, F_p=G_p - F_drag, u_c=c1 * u_a + c2 * u_p)

    def step(self, n: int = 1):
        p = self.p
        h = 1.0 / p["n_sub"]
        for _ in range(int(n)):
            mac = self.macroscopic()
            # step 5: collide both fluids, then stream
            fa = collide(self.f_a, mac["rho_a"], mac["u_a"], mac["F_a"], p["tau_a"])
            fp = collide(self.f_p, mac["rho_p"], mac["u_p"], mac["F_p"], p["tau_p"])
            self.f_a = stream(fa)
            self.f_p = stream(fp)
            # step 6: n_sub finite-difference sub-steps with frozen velocities
            ua, uc = mac["u_a"], mac["u_c"]
            W = grad_vector(ua)
            phi, qxx, qxy = self.phi, self.qxx, self.qxy
            for _m in range(p["n_sub"]):
                dphi = ch_rhs(phi, uc, p)
                Rxx, Rxy = project_sym_traceless(be_rhs(q_tensor(qxx, qxy), ua, W, p))
                phi = phi + h * dphi
                qxx = qxx + h * Rxx
                qxy = qxy + h * Rxy
            self.phi, self.qxx, self.qxy = phi, qxx, qxy
            self.step_count += 1

    # -- outputs ----------------------------------------------------------------
    def get_fields(self) -> dict:
        """phi, qxx, qxy, u_a [2], u_p [2], rho_a, rho_p at the current step; u is the
        half-force-corrected velocity of the same solve the step uses."""
        mac = self.macroscopic()
        return dict(phi=self.phi.copy(), qxx=self.qxx.copy(), qxy=self.qxy.copy(),
                    u_a=mac["u_a"], u_p=mac["u_p"], rho_a=mac["rho_a"], rho_p=mac["rho_p"])

    def diagnostics(self) -> dict:
        """FP64 sums of the Results-section observables over all sites (site_observables),
        plus the count of non-finite state values."""
        p = self.p
        mac = self.macroscopic()
        obs = site_observables(self.phi, self.qxx, self.qxy, mac["rho_a"], mac["rho_p"],
                               mac["u_a"], mac["u_p"], p["K"])
        fields = [self.phi, self.qxx, self.qxy, self.f_a, self.f_p]
        nonfinite = int(sum(np.count_nonzero(~np.isfinite(a)) for a in fields))
        out = dict(step=self.step_count, nonfinite=nonfinite)
        for k in ("phi_sum", "phi_sq_sum", "mass_a", "mass_p", "ke_a", "ke_p", "ke_c", "ua_sq", "uc_sq",
                  "enstrophy_a", "enstrophy_c", "elastic"):
            out[k] = float(obs[k].sum())
        out["s_mean"] = float(obs["S"].mean())
        out["umax"] = float(obs["speed"].max())
        out["phi_absmax"] = phi_extent(self.phi)
        return out

    def free_energy(self) -> float:
        """Total free energy plus kinetic energy of both fluids (used by the passive
        energy-decay check): sum over sites of free_energy_density."""
        p = self.p
        mac = self.macroscopic()
        return float(free_energy_density(self.phi, mac["Q"], mac["rho_a"], mac["rho_p"],
                                         mac["u_a"], mac["u_p"], p).sum())


# ----------------------------------------------------------------------------
# Observables (Results section): per-site densities whose sums are the
# diagnostics, and the free-energy functional of the Model section
# ----------------------------------------------------------------------------
def vorticity(u):
    """omega = d_x u_y - d_y u_x (central differences)."""
    return d_x(u[1]) - d_y(u[0])


def kinetic_density(rho, u):
    """(1/2) rho |u|^2."""
    return 0.5 * rho * (u[0] ** 2 + u[1] ** 2)


def frank_density(Q, K):
    """(K/2) |grad Q|^2 with |grad Q|^2 = sum over k, i, j of (d_k Q_ij)^2: all four
    entries of the full tensor, so each independent component counts twice."""
    dQ = np.array([d_x(Q), d_y(Q)])
    return 0.5 * K * (dQ ** 2).sum(axis=(0, 1, 2))


def scalar_order(qxx, qxy):
    """S with Q = 2 S (pp - I/2): the eigenvalues of Q are +-S."""
    return np.sqrt(qxx ** 2 + qxy ** 2)


def site_observables(phi, qxx, qxy, rho_a, rho_p, ua, up, K):
    """Per-site densities of the diagnostic sums: phi, phi^2 (composition and its
    variance Delta), both densities, kinetic energies (1/2) rho_s |u_s|^2 of each
    fluid and (1/2)|u_c|^2 of the mixture velocity u_c = c1 u_a + c2 u_p, |u_a|^2,
    |u_c|^2, enstrophy densities omega_a^2 and omega_c^2, the Frank elastic energy
    density, the scalar order S and the larger of the two speeds."""
    c1 = 0.5 * (1.0 + phi)
    uc = c1 * ua + (1.0 - c1) * up
    return dict(phi_sum=phi, phi_sq_sum=phi ** 2, mass_a=rho_a, mass_p=rho_p,
                ke_a=kinetic_density(rho_a, ua), ke_p=kinetic_density(rho_p, up),
                ke_c=kinetic_density(1.0, uc),
                ua_sq=ua[0] ** 2 + ua[1] ** 2, uc_sq=uc[0] ** 2 + uc[1] ** 2,
                enstrophy_a=vorticity(ua) ** 2, enstrophy_c=vorticity(uc) ** 2,
                elastic=frank_density(q_tensor(qxx, qxy), K), S=scalar_order(qxx, qxy),
                speed=np.sqrt(np.maximum(ua[0] ** 2 + ua[1] ** 2, up[0] ** 2 + up[1] ** 2)))


def free_energy_density(phi, Q, rho_a, rho_p, ua, up, p):
    """Bulk and gradient Cahn-Hilliard energy (A_ch/4)(phi^2 - 1)^2 + (kappa/2)|grad phi|^2,
    Landau-de Gennes bulk (A/2)TrQ^2 + (B/3)TrQ^3 + (C/4)TrQ^4 (Model, Eq. 8), Frank
    energy (K/2)|grad Q|^2 and the kinetic energy of both fluids."""
    e_ch = 0.25 * p["A_ch"] * (phi ** 2 - 1.0) ** 2 + 0.5 * p["kappa"] * (d_x(phi) ** 2 + d_y(phi) ** 2)
    A, B, C = landau_coefficients(p["A0"], p["gamma_ldg"])
    Q2 = mm(Q, Q)
    tr = lambda T: T[0, 0] + T[1, 1]
    e_q = 0.5 * A * tr(Q2) + B / 3.0 * tr(mm(Q2, Q)) + 0.25 * C * tr(mm(Q2, Q2)) + frank_density(Q, p["K"])
    return e_ch + e_q + kinetic_density(rho_a, ua) + kinetic_density(rho_p, up)


# ----------------------------------------------------------------------------
# Host analysis of snapshots (Results: structure-factor length, energy spectrum)
# ----------------------------------------------------------------------------
def _shell_index(n):
    """Integer shell index |k| rounded, k in units of 2 pi / n (square n x n grids)."""
    k1 = np.fft.fftfreq(n) * n
    k = np.sqrt(k1[None, :] ** 2 + k1[:, None] ** 2)
    return np.floor(k + 0.5).astype(np.int64)  # unit-width shells [k-1/2, k+1/2)


def domain_length(phi) -> float:
    """Coarsening length from the structure factor (Results, L(t) equation):
    L = 2 pi sum_k Phi(k) / sum_k k Phi(k) with Phi(k) the shell sum of |phi_hat|^2,
    physical wavenumber k = 2 pi n / N, shells n >= 1 (the 1/2 cancels).  A single
    Fourier mode of index n gives L = N / n, its wavelength."""
    ny, nx = phi.shape
    if nx != ny:
        raise ValueError("analysis is defined on square grids")
    power = np.abs(np.fft.fft2(phi) / (nx * ny)) ** 2
    shell = _shell_index(nx)
    Phi = np.bincount(shell.ravel(), weights=power.ravel(), minlength=shell.max() + 1)
    k = 2.0 * np.pi * np.arange(Phi.size) / nx
    return float(2.0 * np.pi * Phi[1:].sum() / (k[1:] * Phi[1:]).sum())


def energy_spectrum(u) -> np.ndarray:
    """E(n) = 1/2 sum over shell n of |u_hat|^2, u_hat = FFT(u)/N^2, so that
    sum_n E(n) = <|u|^2>/2 (Results, kinetic energy spectrum); index n is k N / (2 pi)."""
    ny, nx = u.shape[1:]
    if nx != ny:
        raise ValueError("analysis is defined on square grids")
    power = sum(np.abs(np.fft.fft2(u[a]) / (nx * ny)) ** 2 for a in range(2))
    shell = _shell_index(nx)
    return 0.5 * np.bincount(shell.ravel(), weights=power.ravel(), minlength=shell.max() + 1)
