"""Pins of the single-fluid oracle (the paper's case 1) against what the model
fixes (no GPU): the two-component step with an absent second component,
conservation, a fixed point, the viscosity of Eq. 2, and a closed-form
channel flow for the bounce-back walls."""

import numpy as np
import pytest

from oracle import lb_oracle as O
from oracle import lb_single as S
import synth


def _state(shape, seed, amp=0.05, vel=0.05, solid=None):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-amp, amp, shape)
    u = tuple(rng.uniform(-vel, vel, shape) for _ in range(3))
    return rho, u


def test_equals_two_component_step_with_an_absent_second_component():
    """With rho_B = 0 everywhere the two-component step reduces to the
    single-fluid one: psi_B = 0 removes the force on A, the common velocity
    is m_A / rho_A, and B stays empty.  Independent code paths, equal to
    rounding."""
    shape = (6, 7, 8)
    solid = synth.solid_mask(shape, np.array([[4.0, 3.0, 2.5]]), 1.6)
    rho, u = _state(shape, 3)
    f1 = S.init_equilibrium(rho, u, solid)
    f2 = O.init_equilibrium(rho, np.zeros(shape), u, solid)
    p = O.Params((0.7, 1.3), 3.5)
    g1 = S.step(f1, 0.7, solid, n=12)
    g2 = O.step(f2, p, solid, n=12)
    assert np.all(g2[1] == 0.0)
    assert np.max(np.abs(g1 - g2[0])) <= 1e-14 * np.max(np.abs(g1))


def test_mass_and_momentum_conserved_on_periodic_box():
    rho, u = _state((8, 9, 10), 4)
    f = S.init_equilibrium(rho, u)
    (M0, *P0), _ = S.totals(f)
    f = S.step(f, 0.6, n=200)
    (M, *P), nonfinite = S.totals(f)
    assert not nonfinite
    assert abs(M - M0) / M0 < 1e-13
    for a in range(3):
        assert abs(P[a] - P0[a]) / M0 < 1e-13
    # the velocity field must have relaxed for this to mean anything
    _, u1 = S.moments(f)
    assert np.max(np.abs(u1[0])) < 0.5 * np.max(np.abs(u[0]))


def test_mass_conserved_with_solids_and_walls_hold_zero():
    shape = (10, 10, 10)
    solid = synth.solid_mask(shape, np.array([[2.5, 3.0, 4.0], [7.2, 6.1, 5.5]]), 2.1)
    rho, u = _state(shape, 5)
    f = S.init_equilibrium(rho, u, solid)
    (M0, *_), _ = S.totals(f)
    f = S.step(f, 0.9, solid, n=100)
    (M, *_), _ = S.totals(f)
    assert abs(M - M0) / M0 < 1e-13
    assert np.all(f[:, solid.astype(bool)] == 0.0)


def test_uniform_flow_is_a_fixed_point():
    shape = (4, 5, 6)
    rho = np.full(shape, 1.3)
    u = tuple(np.full(shape, v) for v in (0.02, -0.01, 0.03))
    f = S.init_equilibrium(rho, u)
    g = S.step(f, 0.8, n=5)
    assert np.max(np.abs(g - f)) < 1e-15


@pytest.mark.parametrize("tau", [0.7, 1.0])
def test_shear_wave_decay_gives_eq2_viscosity(tau):
    L = 64
    y = np.arange(L)
    U0 = 1e-3
    k = 2.0 * np.pi / L
    ux = np.broadcast_to((U0 * np.sin(k * y))[None, :, None], (1, L, 1)).copy()
    z = np.zeros_like(ux)
    f = S.init_equilibrium(np.ones_like(ux), (ux, z, z))
    t_obs, amp = [], []
    for t in range(0, 601):
        if t % 50 == 0 and t >= 100:
            _, u = S.moments(f)
            amp.append(2.0 / L * np.sum(u[0][0, :, 0] * np.sin(k * y)))
            t_obs.append(t)
        f = S.step(f, tau)
    rate = -np.polyfit(t_obs, np.log(amp), 1)[0]
    nu = O.CS2 * (tau - 0.5)
    assert abs(rate / (nu * k * k) - 1.0) < 0.01


def test_channel_flow_between_bounce_back_walls_is_the_parabola():
    """Plane Poiseuille flow: walls at y = 0 and y = H + 1 (solid rows), a
    uniform body force g along x applied as a velocity shift (u = m/rho +
    tau g) in a copy of the oracle's collision, with the oracle's streaming
    and bounce-back.  The steady profile's second difference is exactly
    -g / nu (the bulk solution of the BGK step), it is symmetric, and it
    sits on the parabola u(y) = g / (2 nu) (y - 1/2)(H + 1/2 - y) of walls
    half a node outside the fluid, up to the BGK bounce-back slip, which is
    1e-3 of the peak at tau = 0.9 (it changes sign near tau = 0.93)."""
    H, tau, g = 12, 0.9, 1e-6
    shape = (1, H + 2, 1)
    solid = np.zeros(shape, dtype=np.uint8)
    solid[:, 0, :] = 1
    solid[:, H + 1, :] = 1
    f = S.init_equilibrium(np.ones(shape), None, solid)
    s = solid.astype(bool)
    for _ in range(6000):
        rho = O.density(f)
        m = O.momentum(f)
        den = np.where(s, 1.0, rho)
        ux = m[0] / den + tau * g
        feq = O.equilibrium(rho, ux, m[1] / den, m[2] / den)
        fs = (1.0 - 1.0 / tau) * f + (1.0 / tau) * feq
        fs[:, s] = 0.0
        f = O.stream(fs[None], solid)[0]
    rho = O.density(f)
    u = (O.momentum(f)[0] / np.where(s, 1.0, rho) + 0.5 * g)[0, 1:H + 1, 0]  # mid-step velocity
    y = np.arange(1, H + 1)
    nu = O.CS2 * (tau - 0.5)
    want = g / (2.0 * nu) * (y - 0.5) * (H + 0.5 - y)
    d2 = u[2:] - 2.0 * u[1:-1] + u[:-2]
    assert np.max(np.abs(d2 + g / nu)) / (g / nu) < 1e-8
    assert np.max(np.abs(u - u[::-1])) / np.max(u) < 1e-12
    assert np.max(np.abs(u - want)) / np.max(want) < 2e-3
