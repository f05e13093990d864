"""Pins of the CPU oracle's building blocks against closed forms (no GPU).

Each test checks the oracle against something other than itself: the paper's
weight table, exact moment identities of the equilibrium, a closed-form
response of the force stencil, exact conservation of the collision, the
streaming permutation, and an independent per-node twin.
"""

import decimal
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import lb_oracle as O
from oracle import naive as N
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Lattice (Sec. 2; Appendix weight table)
# --------------------------------------------------------------------------
def test_weights_match_paper_table():
    g = json.load(open(os.path.join(GOLDEN, "d3q19_weights.json")))
    c2 = (O.C ** 2).sum(axis=1)
    for cls, count in g["count_by_c2"].items():
        assert int(np.sum(c2 == int(cls))) == count
    for cls, w in g["w_by_c2"].items():
        sel = c2 == int(cls)
        assert np.all(O.W[sel] == float(Fraction(w)))
    assert O.CS2 == float(Fraction(g["cs2"].split()[0]))
    assert set(np.unique(c2)) == {0, 1, 2}
    assert len({tuple(c) for c in O.C}) == 19


def test_lattice_isotropy_exact():
    # Exact rational moments of the weights: sum w = 1, sum w c_a c_b = delta/3,
    # fourth moment (dd + dd + dd)/9, odd moments zero.
    w = [Fraction(1, 3)] + [Fraction(1, 18)] * 6 + [Fraction(1, 36)] * 12
    c = [tuple(int(v) for v in row) for row in O.C]
    assert sum(w) == 1
    d = lambda a, b: 1 if a == b else 0
    for a in range(3):
        assert sum(wi * ci[a] for wi, ci in zip(w, c)) == 0
        for b in range(3):
            assert sum(wi * ci[a] * ci[b] for wi, ci in zip(w, c)) == Fraction(d(a, b), 3)
            for e in range(3):
                assert sum(wi * ci[a] * ci[b] * ci[e] for wi, ci in zip(w, c)) == 0
                for g in range(3):
                    m4 = sum(wi * ci[a] * ci[b] * ci[e] * ci[g] for wi, ci in zip(w, c))
                    assert m4 == Fraction(d(a, b) * d(e, g) + d(a, e) * d(b, g) + d(a, g) * d(b, e), 9)


def test_opposite_table():
    for i in range(19):
        assert np.all(O.C[O.OPP[i]] == -O.C[i])
        assert O.OPP[O.OPP[i]] == i
        assert O.W[O.OPP[i]] == O.W[i]


# --------------------------------------------------------------------------
# Equilibrium (Appendix, Eq. LEQ)
# --------------------------------------------------------------------------
def test_equilibrium_moments():
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.1, 2.0, 500)
    v = rng.uniform(-0.2, 0.2, (3, 500))
    feq = O.equilibrium(rho, *v)
    m0 = feq.sum(axis=0)
    m1 = np.einsum("ia,in->an", O.C.astype(float), feq)
    m2 = np.einsum("ia,ib,in->abn", O.C.astype(float), O.C.astype(float), feq)
    np.testing.assert_allclose(m0, rho, rtol=1e-14)
    np.testing.assert_allclose(m1, rho * v, atol=1e-15)
    want = rho * (np.eye(3)[:, :, None] / 3.0 + v[:, None, :] * v[None, :, :])
    np.testing.assert_allclose(m2, want, atol=2e-15)


def test_equilibrium_at_rest_is_weights():
    rho = np.array([0.7, 1.0, 1.9])
    z = np.zeros(3)
    feq = O.equilibrium(rho, z, z, z)
    assert np.array_equal(feq, O.W[:, None] * rho[None, :])


# --------------------------------------------------------------------------
# exp used by the pseudopotential
# --------------------------------------------------------------------------
def test_exp_cw_against_library_and_high_precision():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-700, 700, 200000), rng.uniform(-5, 1, 200000),
                        np.array([0.0, -0.0, 1.0, -1.0, math.log(2.0), -math.log(2.0), 1e-300])])
    e = O.exp_cw(x)
    ref = np.exp(x)
    ulps = np.abs(e - ref) / np.spacing(ref)
    assert np.max(ulps) <= 1.0
    assert O.exp_cw(np.array([0.0]))[0] == 1.0
    decimal.getcontext().prec = 60
    for xv in rng.uniform(-6, 2, 300):
        exact = decimal.Decimal(float(xv)).exp()
        got = decimal.Decimal(float(O.exp_cw(np.array([xv]))[0]))
        ulp = decimal.Decimal(float(np.spacing(float(exact))))
        assert abs(got - exact) <= ulp, xv
    # The Cody-Waite split reproduces ln 2 to far below double precision.
    ln2 = decimal.Decimal(2).ln()
    assert abs(decimal.Decimal(O.LN2_HI) + decimal.Decimal(O.LN2_LO) - ln2) < decimal.Decimal("1e-25")


def test_pseudopotential_closed_form():
    rho = np.array([0.0, 1e-9, 0.5, 1.0, 2.0, 3.0])
    psi = O.pseudopotential(rho, 1.0)
    np.testing.assert_allclose(psi, 1.0 - np.exp(-rho), rtol=1e-15, atol=1e-24)
    assert psi[0] == 0.0
    r = O.psi_over_rho(rho, psi)
    assert r[0] == 1.0
    np.testing.assert_allclose(r[1:], (1.0 - np.exp(-rho[1:])) / rho[1:], rtol=1e-7)


# --------------------------------------------------------------------------
# Shan-Chen stencil: closed-form response to a sinusoid
# --------------------------------------------------------------------------
@pytest.mark.parametrize("axis", [0, 1, 2])
def test_force_stencil_sinusoid(axis):
    # For phi = a + eps sin(k x_axis): S_axis = (1/3) eps sin(k) cos(k x_axis),
    # the other two components vanish (derived from the D3Q19 weights).
    n = (6, 10, 8)  # (nz, ny, nx)
    L = n[2 - axis]
    k = 2.0 * np.pi * 3 / L
    z, y, x = np.meshgrid(*[np.arange(s) for s in n], indexing="ij")
    coord = (x, y, z)[axis]
    eps = 0.1
    phi = 0.8 + eps * np.sin(k * coord)
    S = O.sc_sum(phi)
    want = eps * np.sin(k) * np.cos(k * coord) / 3.0
    np.testing.assert_allclose(S[axis], want, atol=1e-15)
    for b in range(3):
        if b != axis:
            np.testing.assert_allclose(S[b], 0.0, atol=1e-15)


def test_force_stencil_uniform_is_exactly_zero():
    S = O.sc_sum(np.full((4, 4, 4), 0.6321))
    for a in range(3):
        assert np.all(S[a] == 0.0)


# --------------------------------------------------------------------------
# Collision invariants
# --------------------------------------------------------------------------
def _random_state(shape, seed, amp=0.2, u=0.05):
    rng = np.random.default_rng(seed)
    a, b = synth.fluid_fields(shape, amp, seed)
    vel = [rng.uniform(-u, u, shape) for _ in range(3)]
    f = O.init_equilibrium(a, b, vel)
    f = f * (1.0 + rng.uniform(-0.05, 0.05, f.shape))  # leave equilibrium
    return f


def test_collision_conserves_mass_and_adds_force():
    f = _random_state((5, 6, 7), 1)
    p = O.Params((0.7, 1.3), 3.5)
    fs, aux = O.collide(f, p)
    for k in range(2):
        np.testing.assert_allclose(O.density(fs[k]), aux["rho"][k], rtol=1e-14)
    m_after = [O.momentum(fs[k]) for k in range(2)]
    for a in range(3):
        dm = (m_after[0][a] + m_after[1][a]) - (aux["m"][0][a] + aux["m"][1][a])
        F = -p.G * aux["psi"][0] * aux["S"][0][a] - p.G * aux["psi"][1] * aux["S"][1][a]
        np.testing.assert_allclose(dm, F, atol=5e-15)


def test_collision_tau_one_no_force_gives_equilibrium_at_common_velocity():
    f = _random_state((4, 4, 5), 2)
    p = O.Params((1.0, 1.0), 0.0)
    fs, aux = O.collide(f, p)
    up = aux["u_common"]
    for k in range(2):
        np.testing.assert_allclose(fs[k], O.equilibrium(aux["rho"][k], *up), atol=1e-15)
    # with equal tau the common velocity is the barycentric one
    rho = aux["rho"][0] + aux["rho"][1]
    for a in range(3):
        np.testing.assert_allclose(up[a], (aux["m"][0][a] + aux["m"][1][a]) / rho, rtol=1e-13, atol=1e-16)


# --------------------------------------------------------------------------
# Streaming and bounce-back
# --------------------------------------------------------------------------
@pytest.mark.parametrize("i", range(19))
def test_streaming_moves_a_marked_population(i):
    shape = (4, 5, 6)
    fs = np.zeros((2,) + (19,) + shape)
    x0, y0, z0 = 5, 0, 3  # on the box edge so the wrap is exercised
    fs[1, i, z0, y0, x0] = 1.0
    out = O.stream(fs)
    cx, cy, cz = O.C[i]
    dst = ((z0 + cz) % 4, (y0 + cy) % 5, (x0 + cx) % 6)
    assert out[1, i][dst] == 1.0
    assert out.sum() == 1.0


@pytest.mark.parametrize("i", range(1, 19))
def test_bounce_back_returns_to_source(i):
    shape = (4, 5, 6)
    x0, y0, z0 = 2, 2, 1
    cx, cy, cz = O.C[i]
    solid = np.zeros(shape, np.uint8)
    solid[(z0 + cz) % 4, (y0 + cy) % 5, (x0 + cx) % 6] = 1
    fs = np.zeros((2, 19) + shape)
    fs[0, i, z0, y0, x0] = 1.0
    out = O.stream(fs, solid)
    assert out[0, O.OPP[i], z0, y0, x0] == 1.0
    assert out.sum() == 1.0


# --------------------------------------------------------------------------
# Brute-force twin
# --------------------------------------------------------------------------
@pytest.mark.parametrize("with_solid", [False, True])
def test_vectorised_oracle_matches_per_node_twin(with_solid):
    shape = (4, 5, 6)
    f = _random_state(shape, 3, amp=0.3)
    solid = None
    if with_solid:
        solid = np.zeros(shape, np.uint8)
        solid[1, 2, 3] = solid[2, 2, 3] = solid[0, 0, 0] = solid[3, 4, 5] = 1
        f[:, :, solid.astype(bool)] = 0.0
    p = O.Params((0.8, 1.3), 3.5)
    fo = O.step(f, p, solid, n=3)
    fn = N.step(f, p.tau, p.G, solid=solid, n=3)
    assert O.population_error(fn, fo) < 1e-14


def test_step_at_matches_full_step():
    shape = (6, 6, 6)
    f = _random_state(shape, 4)
    p = O.Params((0.8, 0.8), 3.5)
    full = O.step(f, p)
    sites = synth.sample_sites(shape, 12, 9)
    got = N.step_at(f, sites, p.tau, p.G)
    for s, (x, y, z) in enumerate(sites):
        np.testing.assert_allclose(got[s], full[:, :, z, y, x], rtol=1e-14, atol=1e-17)
