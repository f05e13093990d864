"""Pins of the CPU oracle's whole step against what the model fixes (no GPU).

Conservation laws, lattice symmetries, a fixed point, the viscosity of
Eq. 2 measured from a decaying shear wave, and the Laplace law for droplets
of the demixed phase.
"""

import numpy as np
import pytest

from oracle import lb_oracle as O
import synth


def _mix(shape, seed, amp=0.02):
    a, b = synth.fluid_fields(shape, amp, seed)
    return O.init_equilibrium(a, b)


# --------------------------------------------------------------------------
# Conservation
# --------------------------------------------------------------------------
def test_mass_and_momentum_conserved_on_periodic_box():
    p = O.Params((0.8, 0.8), 3.5)
    f = _mix((8, 8, 8), 1, amp=0.05)
    (MA0, MB0, *_), _ = O.totals(f)
    f = O.step(f, p, n=300)
    (MA, MB, Px, Py, Pz), nonfinite = O.totals(f)
    assert not nonfinite
    # the state must have moved far from uniform for this to mean anything
    assert np.ptp(O.density(f[0])) > 0.5
    assert abs(MA - MA0) / MA0 < 1e-13
    assert abs(MB - MB0) / MB0 < 1e-13
    assert max(abs(Px), abs(Py), abs(Pz)) / (MA0 + MB0) < 1e-13


def test_mass_conserved_with_solids():
    shape = (10, 10, 10)
    centres = np.array([[2.5, 3.0, 4.0], [7.2, 6.1, 5.5]])
    solid = synth.solid_mask(shape, centres, 2.1)
    a, b = synth.fluid_fields(shape, 0.05, 2)
    f = O.init_equilibrium(a, b, solid=solid)
    p = O.Params((1.0, 0.9), 3.5)
    (MA0, MB0, *_), _ = O.totals(f)
    f = O.step(f, p, solid, n=100)
    (MA, MB, *_), nonfinite = O.totals(f)
    assert not nonfinite
    assert abs(MA - MA0) / MA0 < 1e-13
    assert abs(MB - MB0) / MB0 < 1e-13
    assert np.all(f[:, :, solid.astype(bool)] == 0.0)


# --------------------------------------------------------------------------
# Symmetries
# --------------------------------------------------------------------------
def _perm_for(vel_map):
    """Index permutation pi with c_{pi(i)} = vel_map(c_i)."""
    out = np.empty(19, dtype=np.int64)
    for i in range(19):
        c = vel_map(O.C[i])
        out[i] = int(np.nonzero((O.C == c).all(axis=1))[0][0])
    return out


def _reflect_x(f):
    # x -> -x (mod L): field flip plus velocity cx -> -cx
    pi = _perm_for(lambda c: np.array([-c[0], c[1], c[2]]))
    g = np.roll(np.flip(f, axis=-1), 1, axis=-1)
    out = np.empty_like(g)
    out[:, pi] = g
    return out


def _swap_xy(f):
    pi = _perm_for(lambda c: np.array([c[1], c[0], c[2]]))
    g = np.swapaxes(f, -1, -2)
    out = np.empty_like(g)
    out[:, pi] = g
    return np.ascontiguousarray(out)


def _cycle_xyz(f):
    # (x, y, z) -> (y, z, x): new[z', y', x'] = old at x = z', y = x', z = y'
    pi = _perm_for(lambda c: np.array([c[2], c[0], c[1]]))
    g = np.transpose(f, (0, 1, 3, 4, 2))
    out = np.empty_like(g)
    out[:, pi] = g
    return np.ascontiguousarray(out)


@pytest.mark.parametrize("transform", [_reflect_x, _swap_xy, _cycle_xyz])
def test_step_commutes_with_cube_symmetries(transform):
    p = O.Params((0.8, 1.1), 3.5)
    a, b = synth.fluid_fields((6, 6, 6), 0.2, 4)
    rng = np.random.default_rng(4)
    u = [rng.uniform(-0.05, 0.05, (6, 6, 6)) for _ in range(3)]
    f = O.init_equilibrium(a, b, u)
    lhs = O.step(transform(f), p, n=2)
    rhs = transform(O.step(f, p, n=2))
    assert O.population_error(lhs, rhs) < 1e-14


def test_step_commutes_with_translation_bitwise():
    p = O.Params((0.8, 0.8), 3.5)
    f = _mix((5, 6, 7), 5, amp=0.2)
    sh = (1, 2, 3)
    lhs = O.step(np.roll(f, sh, axis=(-3, -2, -1)), p, n=2)
    rhs = np.roll(O.step(f, p, n=2), sh, axis=(-3, -2, -1))
    assert np.array_equal(lhs, rhs)


def test_component_swap_symmetry():
    f = _mix((5, 5, 5), 6, amp=0.2)
    p = O.Params((0.7, 1.2), 3.5)
    q = O.Params((1.2, 0.7), 3.5)
    lhs = O.step(f[::-1].copy(), q, n=2)
    rhs = O.step(f, p, n=2)[::-1]
    assert O.population_error(lhs, rhs) < 1e-14


def test_uniform_rest_state_is_a_fixed_point():
    a = np.full((4, 4, 4), 1.3)
    b = np.full((4, 4, 4), 0.4)
    f = O.init_equilibrium(a, b)
    g = O.step(f, O.Params((0.8, 1.0), 3.5), n=5)
    assert O.population_error(g, f) < 1e-14


# --------------------------------------------------------------------------
# Viscosity (Sec. 2, Eq. 2): nu = c_s^2 (tau - 1/2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau,G", [(0.8, 0.0), (1.0, 0.0), (0.8, 0.5)])
def test_shear_wave_decay_gives_eq2_viscosity(tau, G):
    L = 64
    y = np.arange(L)
    U0 = 1e-3
    k = 2.0 * np.pi / L
    ux = np.broadcast_to((U0 * np.sin(k * y))[None, :, None], (1, L, 1)).copy()
    z = np.zeros_like(ux)
    rho = np.ones_like(ux)
    f = O.init_equilibrium(rho, rho, (ux, z, z))
    p = O.Params((tau, tau), G)
    t_obs, amp = [], []
    for t in range(0, 601):
        if t % 50 == 0 and t >= 100:
            _, _, u = O.moments(f, p)
            amp.append(2.0 / L * np.sum(u[0][0, :, 0] * np.sin(k * y)))
            t_obs.append(t)
        f = O.step(f, p)
    rate = -np.polyfit(t_obs, np.log(amp), 1)[0]
    nu = O.CS2 * (tau - 0.5)
    assert abs(rate / (nu * k * k) - 1.0) < 0.01


# --------------------------------------------------------------------------
# Laplace law for demixed droplets (cylinders in a thin periodic box)
# --------------------------------------------------------------------------
@pytest.mark.slow
def test_laplace_law_for_cylindrical_droplets():
    G, L, steps = 3.5, 48, 2000
    p = O.Params((1.0, 1.0), G)
    yy, xx = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    d = np.sqrt((xx - L / 2 + 0.5) ** 2 + (yy - L / 2 + 0.5) ** 2)
    radii, dps = [], []
    for R0 in (6.0, 9.0, 12.0):
        inside = d < R0
        ra = np.where(inside, 2.3, 0.06)[None]
        rb = np.where(inside, 0.06, 2.3)[None]
        f = O.init_equilibrium(ra, rb)
        f = O.step(f, p, n=steps - 400)
        dp_hist, R_hist = [], []
        for _ in range(8):  # average over the slow residual oscillation
            f = O.step(f, p, n=50)
            a, b, _ = O.moments(f, p)
            pa, pb = O.pseudopotential(a, 1.0), O.pseudopotential(b, 1.0)
            pres = (a + b) * O.CS2 + (G * O.CS2) * pa * pb   # bulk equation of state
            c = L // 2
            dp_hist.append(pres[0, c - 1:c + 1, c - 1:c + 1].mean() - pres[0, :2, :2].mean())
            ain, aout = a[0, c, c], a[0, 0, 0]
            R_hist.append(np.sqrt(np.sum((a - aout) / (ain - aout)) / np.pi))
        radii.append(np.mean(R_hist))
        dps.append(np.mean(dp_hist))
    radii, dps = np.array(radii), np.array(dps)
    # Laplace: dp = sigma / R for a cylinder
    A = np.vstack([1.0 / radii, np.ones_like(radii)]).T
    (sigma, icpt), *_ = np.linalg.lstsq(A, dps, rcond=None)
    fit = A @ np.array([sigma, icpt])
    r2 = 1.0 - np.sum((dps - fit) ** 2) / np.sum((dps - dps.mean()) ** 2)
    assert sigma > 0
    assert r2 > 0.99
    assert abs(icpt) < 0.1 * dps.min()
    # and the drop really is demixed
    assert np.all(dps > 0)


# --------------------------------------------------------------------------
# Linear spinodal threshold: pins the pseudopotential and the velocity shift
# --------------------------------------------------------------------------
def _psi_psiprime_at_one():
    """psi(1) psi'(1) for psi = 1 - exp(-rho), written out from the closed form."""
    e = np.exp(-1.0)
    return (1.0 - e) * e


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_spinodal_threshold_matches_linear_theory(tau):
    """A symmetric mixture rho_A = rho_B = 1 demixes exactly where linear theory says.

    Linearise around rho_A = rho_B = 1 with delta = rho_A - 1 = -(rho_B - 1).
    The mass flux of component k averaged over the collision is
    j_k = rho_k v_k - (tau - 1/2) c_s^2 grad rho_k (first moment of the BGK
    non-equilibrium part), and the velocity shift puts rho_k v_k = rho_k u' +
    tau F_k.  The stencil sum is S ~ c_s^2 grad psi, so F_A = -G psi(1) S(psi_B)
    = G psi(1) psi'(1) c_s^2 grad delta.  Hence
        d delta / dt = c_s^2 [(tau - 1/2) - tau G psi(1) psi'(1)] lap delta,
    and a density-difference mode grows iff G > G_c = (tau - 1/2) / (tau psi psi').
    The threshold tests the force's coefficient tau (a shift by (tau - 1/2) F
    moves G_c to 1/(psi psi') = 4.30), the pseudopotential's value and slope
    at rho = 1 and the stencil's c_s^2 together.
    """
    L, steps, eps = 32, 600, 1e-6
    x = np.arange(L)
    mode = np.cos(2.0 * np.pi * x / L)
    Gc = (tau - 0.5) / (tau * _psi_psiprime_at_one())

    def amplitude_ratio(G):
        a = (1.0 + eps * mode).reshape(1, 1, L)
        b = (1.0 - eps * mode).reshape(1, 1, L)
        f = O.init_equilibrium(a, b)

        def amp(f):
            d = O.density(f[0]) - O.density(f[1])
            return float(np.sum(d.ravel() * mode)) * 2.0 / L

        a0 = amp(f)
        f = O.step(f, O.Params((tau, tau), G), n=steps)
        return amp(f) / a0

    below, above = amplitude_ratio(0.95 * Gc), amplitude_ratio(1.05 * Gc)
    assert below < 0.98, f"mode should decay 5% below G_c = {Gc:.4f}: ratio {below}"
    assert above > 1.02, f"mode should grow 5% above G_c = {Gc:.4f}: ratio {above}"


# --------------------------------------------------------------------------
# Output velocity of a relaxed flat interface: pins the half-force term
# --------------------------------------------------------------------------
@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_flat_interface_at_rest_has_zero_output_velocity(tau):
    """At a relaxed flat interface nothing flows, so the output velocity vanishes.

    In a steady state without flow the momentum averaged over the collision,
    (m + m*) / 2 = m + F / 2 summed over the components, is zero, while the
    pre-collision momentum sum_k m_k alone equals -sum_k F_k / 2, which is
    large where the interface force acts.  The output velocity
    (sum_k m_k + (F_A + F_B) / 2) / rho must therefore go to zero, and the bare
    sum_k m_k / rho must not.
    """
    L, steps = 32, 2000
    x = np.arange(L)
    inside = (x >= L // 4) & (x < 3 * L // 4)
    a = np.where(inside, 2.3, 0.06).reshape(1, 1, L).astype(np.float64)
    b = np.where(inside, 0.06, 2.3).reshape(1, 1, L).astype(np.float64)
    p = O.Params((tau, tau), 3.5)
    f = O.step(O.init_equilibrium(a, b), p, n=steps)
    ra, rb, u = O.moments(f, p)
    bare = (O.momentum(f[0])[0] + O.momentum(f[1])[0]) / (ra + rb)
    assert np.ptp(ra) > 2.0  # the interface is still sharp
    assert np.max(np.abs(u[0])) <= 1e-5
    assert np.max(np.abs(bare)) >= 1e-2
    assert np.max(np.abs(u[1])) <= 1e-15 and np.max(np.abs(u[2])) <= 1e-15
