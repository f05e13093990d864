"""Pins of the moving-particle oracle (the paper's particle solver: Sec. 2,
Eq. PARDYN; Appendix, Eqs. UPI, LADDFLBE, FORCEPP, FORCEPARTEQ, TORQUEPARTEQ)
against what the model and the geometry fix (no GPU)."""

import math

import numpy as np
import pytest

from oracle import lb_oracle as O
from oracle import lb_particles as PT
from oracle import lb_single as S
import synth


def _fluid(shape, seed, amp=0.01, vel=0.01):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-amp, amp, shape)
    u = [rng.uniform(-vel, vel, shape) for _ in range(3)]
    return rho, u


def _brute_owner(shape, pos, R):
    """Minimum-image distance from every node to every centre, lowest index wins."""
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    owner = np.full(shape, PT.FLUID, dtype=np.int64)
    for p in range(len(pos) - 1, -1, -1):
        d = []
        for c, r, L in ((x, pos[p][0], nx), (y, pos[p][1], ny), (z, pos[p][2], nz)):
            e = c - r
            d.append(e - L * np.round(e / L))
        inside = d[0] ** 2 + d[1] ** 2 + d[2] ** 2 <= R * R
        owner[inside] = p
    return owner


def test_owner_map_is_the_minimum_image_sphere_test():
    rng = np.random.default_rng(1)
    shape = (17, 19, 23)
    pos = [rng.uniform(0, 1, 3) * np.array([23, 19, 17]) for _ in range(4)]
    part = PT.Particles(3.3, 1.0, pos, None, None)
    assert np.array_equal(PT.owner_map(shape, part), _brute_owner(shape, pos, 3.3))


def test_box_holds_a_particles_nodes_before_and_after_a_move_under_one_node():
    rng = np.random.default_rng(2)
    for _ in range(200):
        R = rng.uniform(1.5, 6.0)
        r0 = rng.uniform(10, 20, 3)
        r1 = r0 + rng.uniform(-0.999, 0.999, 3)
        lo, S_ = PT._box(r1, R)
        for r in (r0, r1):
            for a in range(3):
                assert lo[a] <= math.ceil(r[a] - R) and math.floor(r[a] + R) <= lo[a] + S_ - 1


def test_resting_particle_is_the_fixed_solid_single_fluid_step():
    shape = (14, 15, 16)
    rho, u = _fluid(shape, 3)
    part = PT.Particles(3.5, math.inf, [[7.0, 6.5, 8.2]], None, None)
    f, owner = PT.init(rho, part, u)
    g, q, _ = PT.step(f.copy(), 0.8, part, owner, n=4)
    h = S.step(f.copy(), 0.8, (owner != PT.FLUID).astype(np.uint8), n=4)
    assert np.array_equal(g, h)
    assert np.array_equal(q.pos, part.pos)


def test_total_momentum_is_conserved_while_particles_move_and_cover_nodes():
    shape = (20, 18, 22)
    rho, u = _fluid(shape, 4)
    part = PT.Particles(3.2, 400.0, [[6.3, 5.2, 7.1], [15.4, 12.6, 13.2]],
                        [[0.08, -0.05, 0.06], [-0.07, 0.06, -0.05]], [[0.0, 0.0, 0.02], [0.02, -0.01, 0.0]])
    f, owner = PT.init(rho, part, u)
    P0 = PT.total_momentum(f, part)
    changes = 0
    for _ in range(25):
        f, part, owner_new = PT.step(f, 0.8, part, owner)
        changes += int(np.sum(owner_new != owner))
        owner = owner_new
    P1 = PT.total_momentum(f, part)
    assert changes > 20  # nodes were covered and uncovered
    assert np.max(np.abs(P1 - P0)) < 1e-13 * np.sum(rho)
    assert np.all(f[:, owner != PT.FLUID] == 0.0)


def _links(owner, p):
    """Brute-force list of links (fluid node, direction) into particle p's nodes."""
    nz, ny, nx = owner.shape
    out = []
    for z, y, x in zip(*np.nonzero(owner == p)):
        for i in range(1, O.Q):
            xf, yf, zf = (x - O.C[i, 0]) % nx, (y - O.C[i, 1]) % ny, (z - O.C[i, 2]) % nz
            if owner[zf, yf, xf] == PT.FLUID:
                out.append(i)
    return out


def test_first_step_force_on_a_translating_sphere_is_the_link_sum_closed_form():
    """Fluid at rest with density rho: f* = w_i rho, so each link hands the
    particle c_i (2 w_i rho - 6 w_i rho c_i.U) and a link set symmetric under
    c -> -c gives F = -6 rho sum_links w_i c_i (c_i . U), T = 0."""
    shape = (20, 20, 20)
    rho0 = 1.2
    U = np.array([0.01, -0.02, 0.005])
    part = PT.Particles(4.3, math.inf, [[10.0, 10.0, 10.0]], [U], None)
    f, owner = PT.init(np.full(shape, rho0), part)
    _, q, _ = PT.step(f, 0.9, part, owner)
    M = np.zeros((3, 3))
    for i in _links(owner, 0):
        M += O.W[i] * np.outer(O.C[i], O.C[i])
    want = -6.0 * rho0 * M @ U
    assert np.max(np.abs(q.force[0] - want)) < 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(q.torque[0])) < 1e-12 * np.max(np.abs(want))


def test_spinning_sphere_feels_an_opposing_torque_and_slows_down():
    """A sphere about ten times denser than the fluid, spinning in fluid at rest:
    the torque of the first step is along -omega, and the spin decays
    monotonically.  (The printed r_b x omega would make the surface drive the
    spin instead.)"""
    shape = (20, 20, 20)
    part = PT.Particles(4.3, 3000.0, [[10.0, 10.0, 10.0]], None, [[0.0, 0.0, 0.01]])
    f, owner = PT.init(np.ones(shape), part)
    spins = []
    for t in range(12):
        f, part, owner = PT.step(f, 0.9, part, owner)
        spins.append(part.omg[0, 2])
        if t == 0:
            T = part.torque[0]
            assert T[2] < 0.0 and abs(T[0]) < 1e-12 * abs(T[2]) and abs(T[1]) < 1e-12 * abs(T[2])
    assert all(b < a for a, b in zip(spins, spins[1:])) and spins[-1] > 0.0


def test_uniform_flow_moving_with_the_particle_stays_uniform():
    """A particle carried at the velocity U of the surrounding uniform flow
    (infinite mass) feels no force, and the fluid stays at f^eq(rho0, U): the
    moving-wall bounce-back returns f^eq_ibar exactly, and uncovered nodes start
    at f^eq(rho0, u_b) = f^eq(rho0, U).  It crosses about 1.5 nodes."""
    shape = (16, 18, 20)
    rho0 = 1.0
    U = np.array([0.06, 0.03, -0.04])
    part = PT.Particles(3.4, math.inf, [[9.3, 8.6, 7.8]], [U], None)
    ones = np.ones(shape)
    f, owner = PT.init(rho0 * ones, part, [U[0] * ones, U[1] * ones, U[2] * ones])
    owner0 = owner.copy()
    feq = O.equilibrium(np.float64(rho0), *[np.float64(v) for v in U])
    for _ in range(25):
        f, part, owner = PT.step(f, 0.8, part, owner, rho0=rho0)
        assert np.max(np.abs(part.force[0])) < 1e-13
    fl = owner == PT.FLUID
    assert np.max(np.abs(f[:, fl] - feq[:, None])) < 1e-14
    assert np.max(np.abs(part.pos[0] - (np.array([9.3, 8.6, 7.8]) + 25 * U))) < 1e-12
    assert np.sum(owner != owner0) > 20


def test_particle_sums_are_correctly_rounded_and_the_bound_holds():
    from fractions import Fraction
    rng = np.random.default_rng(5)
    # cancelling terms of mixed magnitude, as link terms are
    terms = rng.normal(size=(2000, 6)) * 10.0 ** rng.integers(-8, 3, size=(2000, 6))
    terms = np.concatenate([terms, -terms[:1500] * (1.0 + 1e-9)])
    got = PT.exact_sums(terms)
    bound = PT.sum_bound(terms)
    for d in range(6):
        exact = sum((Fraction(float(t)) for t in terms[:, d]), Fraction(0))
        assert got[d] == float(exact)  # Fraction -> float rounds to nearest
        # any order of n - 1 float64 additions stays within the bound
        for order in (np.arange(terms.shape[0]), np.arange(terms.shape[0])[::-1], rng.permutation(terms.shape[0])):
            s = 0.0
            for t in terms[order, d]:
                s += float(t)
            assert abs(s - got[d]) <= bound[d]
        pair = terms[:, d].copy()
        while pair.size > 1:  # pairwise tree
            if pair.size % 2:
                pair = np.append(pair, 0.0)
            pair = pair[0::2] + pair[1::2]
        assert abs(float(pair[0]) - got[d]) <= bound[d]


def test_window_step_equals_the_whole_lattice_step():
    """Locality and exact translation of the particle step: for spheres far
    from every other sphere and from the lattice's ends, one oracle step of a
    32^3 window around the sphere gives the whole-lattice step's force,
    torque, position, velocities and nearby populations bit for bit (the
    full-size GPU check relies on this).  96^3, 40 spheres of radius 5.5."""
    import particle_window as PW
    L = 96
    shape = (L, L, L)
    R = 5.5
    centres = synth.sphere_centres(shape, 40, R, 3)
    rng = np.random.default_rng(58)
    vel = rng.uniform(-0.03, 0.03, (40, 3))
    omg = rng.uniform(-0.003, 0.003, (40, 3))
    mass = synth.particle_mass(R)
    rho, _ = synth.fluid_fields(shape, 0.02, 11)
    part = PT.Particles(R, mass, centres, vel, omg)
    f, owner = PT.init(rho, part)
    f1, q, _ = PT.step(f, 1.0, part.copy(), owner, n=1)
    f1 = f1.reshape(19, -1)
    sample = PW.isolated(centres, R, shape, 8, 0)
    assert sample.size >= 3
    for p in sample:
        F, T, r1, v1, w1, fw, idx, _ = PW.step_window(rho, 1.0, R, mass, centres[p], vel[p], omg[p], shape)
        assert np.array_equal(F, q.force[p]) and np.array_equal(T, q.torque[p]), p
        assert np.array_equal(r1, q.pos[p]) and np.array_equal(v1, q.vel[p]) and np.array_equal(w1, q.omg[p]), p
        assert np.array_equal(fw, f1[:, idx]), p
