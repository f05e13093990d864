"""Pins of the colour-gradient oracle (the paper's two-component model,
Appendix; case 2 of Sec. 5) against what the paper and the mathematics fix
(no GPU): the B_i table and its isotropy constraints, the perturbation's
conservation constraints and stress, the recolouring's colour flux, the
reduction to one fluid, the mean viscosity, conservation, symmetries, a
per-node twin and the Laplace law with the surface tension of Eq. sigmaA."""

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lb_cg as CG
from oracle import lb_oracle as O
from oracle import lb_single as S
from oracle import naive_cg
import synth
from test_oracle_physics import _cycle_xyz, _reflect_x, _swap_xy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "d3q19_weights.json")


def _mixed(shape, seed, amp=0.3, vel=0.03):
    """Smoothly mixed random state: rho^1 in [0.5 - amp, 0.5 + amp], rho^2 = 1 - rho^1, small velocities."""
    rng = np.random.default_rng(seed)
    r1 = 0.5 + rng.uniform(-amp, amp, shape)
    u = [rng.uniform(-vel, vel, shape) for _ in range(3)]
    return CG.init_equilibrium(r1, 1.0 - r1, u)


def _case2(shape, seed):
    """Case 2 of the paper (Sec. 5): every node pure red or pure blue at random, at rest."""
    return CG.init_equilibrium(*synth.colour_fields(shape, seed))


P = CG.Params((0.8, 1.1), 0.02, 0.7)


# --------------------------------------------------------------------------
# Coefficients and sub-steps
# --------------------------------------------------------------------------
def test_b_table_is_the_appendix_table_and_meets_its_isotropy_constraints():
    g = json.load(open(GOLDEN))
    c2 = (O.C * O.C).sum(axis=1)
    for i in range(O.Q):
        assert CG.B[i] == float(Fraction(g["B_by_c2"][str(c2[i])]))
    # the constraints the Appendix imposes on B_i, in exact rationals
    Bf = [Fraction(g["B_by_c2"][str(c2[i])]) for i in range(O.Q)]
    assert sum(Bf) == Fraction(1, 3)
    for a in range(3):
        assert sum(Bf[i] * int(O.C[i, a]) for i in range(O.Q)) == 0
        for b in range(3):
            want = Fraction(1, 3) if a == b else Fraction(0)
            assert sum(Bf[i] * int(O.C[i, a]) * int(O.C[i, b]) for i in range(O.Q)) == want


def _random_normals(n, seed):
    rng = np.random.default_rng(seed)
    g = rng.normal(size=(3, n))
    gn = np.sqrt((g * g).sum(axis=0))
    return tuple(g[a] / gn for a in range(3)), rng.uniform(0.01, 2.0, n)


def test_perturbation_meets_the_conservation_constraints():
    n, gn = _random_normals(200, 1)
    pert, _ = CG.perturbation(n, gn, 0.037)
    mass = sum(pert)
    assert np.max(np.abs(mass)) < 1e-16
    for a in range(3):
        mom = sum(O.C[i, a] * pert[i] for i in range(O.Q))
        assert np.max(np.abs(mom)) < 1e-16


def test_perturbation_stress_is_the_capillary_form_of_eq_sigmaA():
    """Summed over both components, sum_i Omega^(2)_i c_i c_i = (2/9) A |g| (n n - I)
    (from the lattice's fourth-order isotropy); with Sigma = -tau of it, the
    stress is (4/9)(A/omega)(|g|/2)(I - n n), i.e. surface tension (4/9) A / omega
    for a phase field that changes by 2 across the interface."""
    n, gn = _random_normals(100, 2)
    A = 0.05
    pert, _ = CG.perturbation(n, gn, A)
    for a in range(3):
        for b in range(3):
            got = 2.0 * sum(O.C[i, a] * O.C[i, b] * pert[i] for i in range(O.Q))
            want = (2.0 / 9.0) * A * gn * (n[a] * n[b] - (1.0 if a == b else 0.0))
            assert np.max(np.abs(got - want)) < 1e-16


def test_recolouring_keeps_totals_and_moves_colour_along_the_gradient():
    """sum_i of each component's recoloured populations is its density, the two
    add up to f*, and the colour flux is beta (rho1 rho2 / rho) ((1 + sqrt 2) / 9) n
    (sum_i w_i (c_i . n) c_i / |c_i| = (1 + sqrt 2)/9 n on D3Q19)."""
    rng = np.random.default_rng(3)
    m = 50
    n, _ = _random_normals(m, 4)
    r1 = rng.uniform(0.1, 1.0, m)
    r2 = rng.uniform(0.1, 1.0, m)
    rho = r1 + r2
    fstar = O.equilibrium(rho, *[rng.uniform(-0.05, 0.05, m) for _ in range(3)])
    cn = [CG.c_dot(i, n) for i in range(O.Q)]
    beta = 0.7
    out = CG.recolour(fstar, r1, r2, cn, beta)
    assert np.max(np.abs(out.sum(axis=1)[0] - r1)) < 1e-15
    assert np.max(np.abs(out.sum(axis=1)[1] - r2)) < 1e-15
    assert np.max(np.abs(out[0] + out[1] - fstar)) < 1e-15
    for a in range(3):
        flux = sum(O.C[i, a] * (out[0, i] - (r1 / rho) * fstar[i]) for i in range(O.Q))
        want = beta * (r1 * r2 / rho) * ((1.0 + math.sqrt(2.0)) / 9.0) * n[a]
        assert np.max(np.abs(flux - want)) < 1e-15


def test_effective_omega_is_one_over_tau_for_one_fluid_and_a_harmonic_viscosity_mean():
    r1 = np.array([1.0, 0.0, 0.3])
    r2 = np.array([0.0, 1.0, 0.7])
    p = CG.Params((0.65, 1.4))
    om = CG.effective_omega(r1, r2, p)
    assert abs(om[0] - 1.0 / 0.65) < 1e-15 and abs(om[1] - 1.0 / 1.4) < 1e-15
    nu1, nu2 = 0.15 / 3.0, 0.9 / 3.0
    nubar = 1.0 / (0.3 / nu1 + 0.7 / nu2)
    assert abs(om[2] - 1.0 / (3.0 * nubar + 0.5)) < 1e-15


# --------------------------------------------------------------------------
# Whole step
# --------------------------------------------------------------------------
def test_without_interface_terms_the_mixture_is_the_single_fluid_step():
    """sigma = beta = 0 and equal tau: the total population follows the
    single-fluid BGK step (pinned on its own), colour-blind."""
    f = _mixed((5, 6, 7), 5)
    g = CG.step(f, CG.Params((0.8, 0.8), 0.0, 0.0), n=6)
    want = S.step(f[0] + f[1], 0.8, n=6)
    assert np.max(np.abs((g[0] + g[1]) - want)) < 1e-14


@pytest.mark.parametrize("fraction", [0.5, 0.2])
def test_shear_wave_decays_with_the_harmonic_mean_viscosity(fraction):
    """Uniform composition (grad Theta = 0), nu_1 = 0.05, nu_2 = 0.3: the decay
    rate is nu_bar k^2 with 1/nu_bar = c/nu_1 + (1 - c)/nu_2 (an arithmetic
    mean of nu or of tau would be off by a factor of about two)."""
    L, U0 = 64, 1e-3
    tau = (0.65, 1.4)
    k = 2.0 * np.pi / L
    y = np.arange(L)
    ux = np.broadcast_to((U0 * np.sin(k * y))[None, :, None], (1, L, 1)).copy()
    z = np.zeros_like(ux)
    f = CG.init_equilibrium(np.full_like(ux, fraction), np.full_like(ux, 1.0 - fraction), (ux, z, z))
    p = CG.Params(tau, 0.02, 0.7)
    t_obs, amp = [], []
    for t in range(401):
        if t % 50 == 0 and t >= 100:
            _, _, u = CG.moments(f)
            amp.append(2.0 / L * np.sum(u[0][0, :, 0] * np.sin(k * y)))
            t_obs.append(t)
        f = CG.step(f, p)
    rate = -np.polyfit(t_obs, np.log(amp), 1)[0]
    nubar = 1.0 / (fraction / 0.05 + (1.0 - fraction) / 0.3)
    assert abs(rate / (nubar * k * k) - 1.0) < 0.01


def test_component_masses_and_momentum_conserved_while_demixing():
    f = _case2((12, 12, 12), 6)
    (M1, M2, *_), _ = CG.totals(f)
    r1, r2, _ = CG.moments(f)
    th0 = np.abs((r1 - r2) / (r1 + r2)).mean()
    g = CG.step(f, P, n=150)
    (N1, N2, Px, Py, Pz), nonfinite = CG.totals(g)
    assert not nonfinite
    assert abs(N1 - M1) / M1 < 1e-13 and abs(N2 - M2) / M2 < 1e-13
    assert max(abs(Px), abs(Py), abs(Pz)) / (M1 + M2) < 1e-13
    # after the first steps mix neighbours, the recolouring separates them again
    r1, r2, _ = CG.moments(g)
    th = np.abs((r1 - r2) / (r1 + r2)).mean()
    r1, r2, _ = CG.moments(CG.step(f, P, n=5))
    th5 = np.abs((r1 - r2) / (r1 + r2)).mean()
    assert th0 == 1.0 and th > th5 + 0.1


def test_uniform_mixture_at_rest_is_a_fixed_point():
    f = CG.init_equilibrium(np.full((4, 4, 4), 0.3), np.full((4, 4, 4), 0.9))
    g = CG.step(f, P, n=5)
    assert np.max(np.abs(g - f)) < 1e-16


def test_component_swap_symmetry_bitwise():
    f = _mixed((5, 5, 5), 7)
    q = CG.Params((P.tau[1], P.tau[0]), P.sigma, P.beta)
    lhs = CG.step(f[::-1].copy(), q, n=3)
    rhs = CG.step(f, P, n=3)[::-1]
    assert np.array_equal(lhs, rhs)


def test_step_commutes_with_translation_bitwise():
    f = _mixed((5, 6, 7), 8)
    sh = (2, 1, 3)
    lhs = CG.step(np.roll(f, sh, axis=(-3, -2, -1)), P, n=2)
    rhs = np.roll(CG.step(f, P, n=2), sh, axis=(-3, -2, -1))
    assert np.array_equal(lhs, rhs)


@pytest.mark.parametrize("transform", [_reflect_x, _swap_xy, _cycle_xyz])
def test_step_commutes_with_cube_symmetries(transform):
    f = _mixed((6, 6, 6), 9)
    lhs = CG.step(transform(f), P, n=2)
    rhs = transform(CG.step(f, P, n=2))
    assert O.population_error(lhs, rhs) < 1e-14


def test_per_node_twin_agrees():
    f = _mixed((4, 5, 6), 10)
    got = CG.step(f, P, n=3)
    want = naive_cg.step(f, P.tau, P.sigma, P.beta, n=3)
    assert np.max(np.abs(got - want)) / np.max(np.abs(want)) < 1e-14


def test_laplace_law_for_cylinders():
    """A cylinder of one fluid in the other (quasi-2D box, 40 x 40 x 1): at rest
    the pressure jump is sigma / R (Laplace), with sigma the input surface
    tension of Eq. sigmaA.  Measured with p = rho / 3 (the mixture's equation
    of state) inside r < R - 4 and outside r > R + 6 after 1500 steps."""
    L, sigma = 40, 0.01
    p = CG.Params((1.0, 1.0), sigma, 0.7)
    dps = {}
    for R in (8, 12):
        yy, xx = np.mgrid[0:L, 0:L]
        r = np.sqrt((xx - L / 2 + 0.5) ** 2 + (yy - L / 2 + 0.5) ** 2)
        r1 = np.where(r < R, 1.0, 0.0)[None]
        f = CG.step(CG.init_equilibrium(r1, 1.0 - r1), p, n=1500)
        pr = CG.pressure(f)[0]
        dps[R] = pr[r < R - 4].mean() - pr[r > R + 6].mean()
        assert abs(dps[R] * R / sigma - 1.0) < 0.06, (R, dps[R] * R / sigma)
    assert abs(dps[8] / dps[12] - 1.5) < 0.05
