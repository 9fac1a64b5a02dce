"""The pins are sharp: plant a plausible mistake in the oracle, on the CPU, and the
named pin must fail.  Each entry is (mistake, oracle attribute, wrong version,
pin that catches it).  Mistakes are planted with monkeypatch, so the oracle on
disk is never touched."""
import numpy as np
import pytest

from oracle import tfan_oracle as O
import tests.test_oracle_pins as T

I2 = O.eye_field


def _P(Q):
    return Q + 0.5 * I2(Q.shape[2:])


def _H(Q, p):
    A, B, C = O.landau_coefficients(p["A0"], p["gamma_ldg"])
    return O.molecular_field(Q, A, C, p["K"], B=B)


def feq_quadratic(rho, u):                      # (c.u)^2 coefficient doubled
    cu = np.einsum("ia,a...->i...", O.CI.astype(float), u)
    uu = u[0] ** 2 + u[1] ** 2
    return O.WI[:, None, None] * rho * (1 + 3 * cu + 9 * cu ** 2 - 1.5 * uu)


def _guo(u, F, tau, drop_u=False, prefactor=True):
    c = O.CI.astype(float)
    cu = np.einsum("ia,a...->i...", c, u)
    cF = np.einsum("ia,a...->i...", c, F)
    uF = 0 if drop_u else u[0] * F[0] + u[1] * F[1]
    k = (1 - 0.5 / tau) if prefactor else 1.0
    return k * O.WI[:, None, None] * (3 * (cF - uF) + 9 * cu * cF)


MUTATIONS = [
    ("equilibrium quadratic term", "equilibrium", feq_quadratic, T.test_p1_equilibrium_moments, ()),
    ("Guo source without -u", "guo_source", lambda u, F, t: _guo(u, F, t, drop_u=True),
     T.test_p2_guo_source_moments, (1.0,)),
    ("Guo source without (1 - 1/2tau)", "guo_source", lambda u, F, t: _guo(u, F, t, prefactor=False),
     T.test_p2_guo_source_moments, (0.6,)),
    ("mu: wrong sign of kappa term", "chemical_potential",
     lambda phi, A, k: A * (phi ** 3 - phi) + k * O.lap(phi), T.test_p6_tanh_interface_chemical_potential, ()),
    ("mu: half the bulk term", "chemical_potential",
     lambda phi, A, k: 0.5 * A * (phi ** 3 - phi) - k * O.lap(phi), T.test_p6_tanh_interface_chemical_potential, ()),
    ("CH: advection sign", "ch_rhs",
     lambda phi, uc, p: (O.d_x(phi * uc[0]) + O.d_y(phi * uc[1]))
     + p["M"] * O.lap(O.chemical_potential(phi, p["A_ch"], p["kappa"])),
     T.test_p16_uniform_advection, ("phi",)),
    ("CH: mobility sign", "ch_rhs",
     lambda phi, uc, p: -(O.d_x(phi * uc[0]) + O.d_y(phi * uc[1]))
     - p["M"] * O.lap(O.chemical_potential(phi, p["A_ch"], p["kappa"])),
     T.test_p7_ch_linear_growth, (0.0, (4, 0), 0.01)),
    ("capillary force sign", "capillary_force",
     lambda phi, mu: -O.capillary_force(phi, mu), T.test_p7_ch_linear_growth, (0.3, (2, 3), 0.01)),
    ("capillary force as -phi D(mu)", "capillary_force",
     lambda phi, mu: -phi * np.array([O.d_x(mu), O.d_y(mu)]), T.test_p22_capillary_force_term_by_term, (2, 16)),
    ("H: sign of K lap Q", "molecular_field",
     lambda Q, A, C, K, B=0.0: -(A * Q + C * O.mm(O.mm(Q, Q), Q) + K * O.lap(Q)),
     T.test_p13_q_mode_relaxation, ((3, 0), 0)),
    ("H: quartic coefficient C/2", "molecular_field",
     lambda Q, A, C, K, B=0.0: -(A * Q + 0.5 * C * O.mm(O.mm(Q, Q), Q) - K * O.lap(Q)),
     T.test_p9_ldg_relaxation_recurrence, ()),
    ("Ericksen stress sign", "elastic_stress",
     lambda Q, H, lam, K: (-lam * O.mm(H, _P(Q)) - lam * O.mm(_P(Q), H) + 2 * lam * _P(Q) * O.ddot(Q, H)
                           + O.ericksen_stress(Q, K) + O.mm(Q, H) - O.mm(H, Q)),
     T.test_p18_nematic_force_of_director_pattern, (0.0, 0.0, 0.1, 3.0)),
    ("antisymmetric stress sign", "elastic_stress",
     lambda Q, H, lam, K: (-lam * O.mm(H, _P(Q)) - lam * O.mm(_P(Q), H) + 2 * lam * _P(Q) * O.ddot(Q, H)
                           - O.ericksen_stress(Q, K) - O.mm(Q, H) + O.mm(H, Q)),
     T.test_p18_nematic_force_of_director_pattern, (0.0, 0.0, 0.1, 3.0)),
    ("sign of -lam (H.P + P.H)", "elastic_stress",
     lambda Q, H, lam, K: (lam * O.mm(H, _P(Q)) + lam * O.mm(_P(Q), H) + 2 * lam * _P(Q) * O.ddot(Q, H)
                           - O.ericksen_stress(Q, K) + O.mm(Q, H) - O.mm(H, Q)),
     T.test_p18_nematic_force_of_director_pattern, (0.7, 0.0, 0.1, 6.0)),
    ("dropped 2 lam P (Q:H)", "elastic_stress",
     lambda Q, H, lam, K: (-lam * O.mm(H, _P(Q)) - lam * O.mm(_P(Q), H)
                           - O.ericksen_stress(Q, K) + O.mm(Q, H) - O.mm(H, Q)),
     T.test_p18_nematic_force_of_director_pattern, (0.7, 0.0, 0.1, 6.0)),
    ("active stress sign", "active_stress", lambda Q, c1, z: z * c1 * Q, T.test_active_stress_is_extensile, ()),
    ("active stress on the passive fraction", "active_stress", lambda Q, c1, z: -z * (1 - c1) * Q,
     T.test_p18_nematic_force_of_director_pattern, (0.7, 0.03, 0.1, 4.0)),
    ("divergence index transposed", "divergence",
     lambda s: np.array([O.d_x(s[0, 0]) + O.d_y(s[1, 0]), O.d_x(s[0, 1]) + O.d_y(s[1, 1])]),
     T.test_p18_nematic_force_of_director_pattern, (0.0, 0.0, 0.1, 3.0)),
    ("co-rotation: vorticity sign", "corotation",
     lambda W, Q, lam: O.corotation(O.transpose(W), Q, lam), T.test_p11_director_rotation_in_simple_shear,
     (0.0, 0.1)),
    ("co-rotation: dropped -2 lam P (Q:W)", "corotation",
     lambda W, Q, lam: (O.mm(lam * 0.5 * (W + O.transpose(W)) + 0.5 * (W - O.transpose(W)), _P(Q))
                        + O.mm(_P(Q), lam * 0.5 * (W + O.transpose(W)) - 0.5 * (W - O.transpose(W)))),
     T.test_p11b_extension_orders_rods, ()),
    ("velocity gradient transposed", "grad_vector",
     lambda u: np.array([[O.d_x(u[0]), O.d_x(u[1])], [O.d_y(u[0]), O.d_y(u[1])]]),
     T.test_p11c_director_turns_with_shear_wave_vorticity, ()),
    ("BE: advection sign", "be_rhs",
     lambda Q, ua, W, p: ((ua[0] * O.d_x(Q) + ua[1] * O.d_y(Q)) + O.corotation(W, Q, p["lam"])
                          + p["Gamma"] * _H(Q, p)),
     T.test_p16_uniform_advection, ("qxx",)),
    ("drag with the wrong sign", "solve_velocities",
     lambda ra, ma, Ga, rp, mp, Gp, beta: O.solve_velocities(ra, ma, Ga, rp, mp, Gp, -beta),
     T.test_p5_drag_trapezoid, (0.4, 0.5)),
    ("Guo velocity with the full force", "solve_velocities",
     lambda ra, ma, Ga, rp, mp, Gp, beta: O.solve_velocities(ra, ma + 0.5 * Ga, Ga, rp, mp + 0.5 * Gp, Gp, beta),
     T.test_p3_mass_and_momentum_balance, ()),
    ("5-point Laplacian centre weight", "lap",
     lambda g: O.shift(g, 1, 0) + O.shift(g, -1, 0) + O.shift(g, 0, 1) + O.shift(g, 0, -1) - 2.0 * g,
     T.test_p7_ch_linear_growth, (0.0, (4, 0), 0.01)),
    ("streaming against c_i", "stream",
     lambda fs: np.array([np.roll(fs[i], shift=(-O.CI[i, 1], -O.CI[i, 0]), axis=(0, 1)) for i in range(9)]),
     T.test_p19_acoustic_wave_direction_and_speed, ()),
    # diagnostics and free energy (Results-section observables)
    ("kinetic energy without 1/2", "kinetic_density", lambda rho, u: rho * (u[0] ** 2 + u[1] ** 2),
     T.test_p20_diagnostics_shear_flows, ()),
    ("Frank energy over the two stored components only", "frank_density",
     lambda Q, K: 0.5 * K * sum(d(Q[0, c]) ** 2 for c in (0, 1) for d in (O.d_x, O.d_y)),
     T.test_p20_diagnostics_frank_energy_and_order, ()),
    ("vorticity with the wrong relative sign", "vorticity", lambda u: O.d_x(u[1]) + O.d_y(u[0]),
     T.test_p20_diagnostics_cellular_flow_vorticity, ()),
    ("mixture enstrophy from u_a", "site_observables",
     lambda phi, qxx, qxy, ra, rp, ua, up, K: dict(
         O.site_observables(phi, qxx, qxy, ra, rp, ua, up, K),
         enstrophy_c=O.site_observables(phi, qxx, qxy, ra, rp, ua, ua, K)["enstrophy_c"]),
     T.test_p20_diagnostics_shear_flows, ()),
    ("mixture velocity with swapped fractions", "site_observables",
     lambda phi, qxx, qxy, ra, rp, ua, up, K: O.site_observables(-phi, qxx, qxy, ra, rp, ua, up, K),
     T.test_p20_diagnostics_cellular_flow_vorticity, ()),
    ("import momenta with the half force added", "guo_momenta",
     lambda ra, ua, Ga, rp, up, Gp, beta: (ra * ua + 0.5 * (Ga + beta * (up - ua)), rp * up + 0.5 * (Gp - beta * (up - ua))),
     T.test_p23_import_gives_back_densities_and_velocities, ()),
    ("import momenta without the drag", "guo_momenta",
     lambda ra, ua, Ga, rp, up, Gp, beta: (ra * ua - 0.5 * Ga, rp * up - 0.5 * Gp),
     T.test_p23_import_gives_back_densities_and_velocities, ()),
    ("signed maximum of phi for its extent", "phi_extent", lambda phi: float(phi.max()),
     T.test_p20_diagnostics_cellular_flow_vorticity, ()),
    ("scalar order without the square root", "scalar_order", lambda qxx, qxy: qxx ** 2 + qxy ** 2,
     T.test_p20_diagnostics_frank_energy_and_order, ()),
    ("LdG quartic coefficient A0 gamma", "landau_coefficients",
     lambda A0, g: (A0 * (1 - g / 3), -A0 * g, A0 * g), T.test_p21_free_energy_uniform_nematic, (0.2, 5.0, 0.3)),
    ("LdG quadratic coefficient without (1 - gamma/3)", "landau_coefficients",
     lambda A0, g: (A0, -A0 * g, 2 * A0 * g), T.test_p21_free_energy_uniform_nematic, (0.1, 3.0, 0.1)),
]


@pytest.mark.parametrize("name,attr,wrong,pin,args", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(monkeypatch, name, attr, wrong, pin, args):
    original = getattr(O, attr)
    pin(*args)  # the unmutated oracle passes the pin
    monkeypatch.setattr(O, attr, _bind_original(wrong, attr, original))
    with np.errstate(all="ignore"), pytest.raises((AssertionError, np.linalg.LinAlgError)):
        pin(*args)


def _bind_original(wrong, attr, original):
    """Wrong versions written in terms of the original function call it, not themselves."""
    def call(*a, **k):
        saved = getattr(O, attr)
        setattr(O, attr, original)
        try:
            return wrong(*a, **k)
        finally:
            setattr(O, attr, saved)
    return call
