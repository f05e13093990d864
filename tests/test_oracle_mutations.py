"""Planted mistakes in the oracle must make a pin fail (no GPU).

Each case copies an oracle source file with one plausible error planted (a
dropped term, a flipped sign, a wrong index or weight, a shift the wrong
way), loads it in place of the real module in a fresh interpreter, and runs
the pin tests against it.  The case passes only if some pin fails.
"""

import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

FORWARD = [
    ("feq 4.5 -> 4.0", "+ 4.5 * cu * cu)", "+ 4.0 * cu * cu)"),
    ("feq drops -1.5 v.v", " - 1.5 * vv)", ")"),
    ("force sign flipped", "v = [up[a] - a_k * S[k][a] for a in range(3)]",
     "v = [up[a] + a_k * S[k][a] for a in range(3)]"),
    ("stencil uses own component", "S = [sc_sum(psi[1]), sc_sum(psi[0])]\n    den",
     "S = [sc_sum(psi[0]), sc_sum(psi[1])]\n    den"),
    ("stencil neighbour reversed", "t = W[i] * _neighbour(psi_other, C[i])", "t = W[i] * _shift(psi_other, C[i])"),
    ("common velocity not tau-weighted",
     "up = tuple((om[0] * m[0][a] + om[1] * m[1][a]) / den for a in range(3))",
     "up = tuple((m[0][a] + m[1][a]) / (rho[0] + rho[1]) for a in range(3))"),
    ("streaming the wrong way", "pulled = _shift(fs[:, i], C[i])", "pulled = _neighbour(fs[:, i], C[i])"),
    ("bounce-back keeps the index", "pulled = np.where(src_solid, fs[:, OPP[i]], pulled)",
     "pulled = np.where(src_solid, fs[:, i], pulled)"),
    ("psi = rho", "return psi_ref * (1.0 - exp_cw(-(rho / psi_ref)))", "return rho * 1.0"),
    ("exp coefficient off", "EXP_COEF = [1.0 / math.factorial(k) for k in range(EXP_DEGREE + 1)]",
     "EXP_COEF = [1.0 / math.factorial(k) for k in range(EXP_DEGREE + 1)]; EXP_COEF[5] *= 1.001"),
    ("diagonal weight 1/36 -> 1/30", "[1.0 / 36.0] * 12", "[1.0 / 30.0] * 12"),
    ("relaxation uses omega of the other component", "fs[k] = omc * f[k] + om[k] * feq",
     "fs[k] = omc * f[k] + om[1 - k] * feq"),
]

# Mistakes that the two physical pins of the readings (the linear spinodal
# threshold and the relaxed flat interface) must catch on their own: each is
# run against that pin alone, and again against all forward pins.
THRESHOLD = "test_oracle_physics.py::test_spinodal_threshold_matches_linear_theory"
FLAT = "test_oracle_physics.py::test_flat_interface_at_rest_has_zero_output_velocity"
READINGS = [
    ("velocity shift by (tau - 1/2) F", "a_k = (p.tau[k] * p.G) * psi_over_rho(rho[k], psi[k])",
     "a_k = ((p.tau[k] - 0.5) * p.G) * psi_over_rho(rho[k], psi[k])", THRESHOLD),
    ("pseudopotential with half the decay rate", "return psi_ref * (1.0 - exp_cw(-(rho / psi_ref)))",
     "return psi_ref * (1.0 - exp_cw(-(0.5 * rho / psi_ref)))", THRESHOLD),
    ("psi = rho (threshold alone)", "return psi_ref * (1.0 - exp_cw(-(rho / psi_ref)))", "return rho * 1.0",
     THRESHOLD),
    ("output velocity drops the 1/2", "ua = ((m[0][a] + m[1][a]) + 0.5 * (FA + FB)) / tot",
     "ua = ((m[0][a] + m[1][a]) + (FA + FB)) / tot", FLAT),
    ("output velocity subtracts the half force", "ua = ((m[0][a] + m[1][a]) + 0.5 * (FA + FB)) / tot",
     "ua = ((m[0][a] + m[1][a]) - 0.5 * (FA + FB)) / tot", FLAT),
    ("output velocity without the force term", "ua = ((m[0][a] + m[1][a]) + 0.5 * (FA + FB)) / tot",
     "ua = (m[0][a] + m[1][a]) / tot", FLAT),
]
FORWARD = FORWARD + [(name, old, new) for name, old, new, _ in READINGS]

ADJOINT = [
    ("drops the psi-stencil term", " - dpsi[k] * T", ""),
    ("common-velocity term sign", "- om[k] * (U * up).sum(axis=0) / D", "+ om[k] * (U * up).sum(axis=0) / D"),
    ("drops the g' term", " - VS * p.tau[k] * p.G * dg[k]", ""),
    ("stencil transpose shifted the wrong way", "O._shift(Wk[kb], C[j])", "O._neighbour(Wk[kb], C[j])"),
    ("bounce-back not transposed", "a[:, i] = np.where(dst_solid, lam_next[:, O.OPP[i]], a[:, i])", "pass"),
    ("stencil transpose uses own component", "O._shift(Wk[kb], C[j])", "O._shift(Wk[k], C[j])"),
]

SINGLE = [
    ("single: velocity not divided by rho", "u = [m[a] / den for a in range(3)]", "u = [m[a] for a in range(3)]"),
    ("single: tau in place of omega", "om = 1.0 / tau", "om = tau"),
    ("single: relaxation weights swapped", "fs = (1.0 - om) * f + om * feq", "fs = (1.0 - om) * feq + om * f"),
]

COLOUR = [
    ("cg: omega as printed, 2/(6 nu - 1)", "return 2.0 / (6.0 * nubar + 1.0)", "return 2.0 / (6.0 * nubar - 1.0)"),
    ("cg: perturbation without the 1/2", "pcoef = (0.5 * A) * gn", "pcoef = A * gn"),
    ("cg: axis B_i 1/54 -> 1/27", "[1.0 / 54.0] * 6", "[1.0 / 27.0] * 6"),
    ("cg: recolouring adds to both components", "out[1, i] = c2 * fstar[i] - t", "out[1, i] = c2 * fstar[i] + t"),
    ("cg: cos(phi) without |c_i|", "t = (r * (cn[i] / CLEN[i])) * (W[i] * rho)", "t = (r * cn[i]) * (W[i] * rho)"),
    ("cg: recolouring over rho, not rho^2", "r = (beta * (rho1 * rho2)) / (rho * rho)",
     "r = (beta * (rho1 * rho2)) / rho"),
    ("cg: gradient without 1/c_s^2", "return tuple(3.0 * S[a] for a in range(3))", "return tuple(S[a] for a in range(3))"),
    ("cg: arithmetic mean of the viscosities",
     "inv_nubar = (rho1 / rho) * inv[0] + (rho2 / rho) * inv[1]\n    nubar = 1.0 / inv_nubar",
     "nubar = (rho1 / rho) / inv[0] + (rho2 / rho) / inv[1]"),
    ("cg: phase field sign", "theta = (rho1 - rho2) / rho", "theta = (rho2 - rho1) / rho"),
    ("cg: velocity of one component", "u = tuple((m1[a] + m2[a]) / rho for a in range(3))",
     "u = tuple(m1[a] / rho for a in range(3))"),
    ("cg: no interface cut", "pos = gg > INTERFACE_G2", "pos = gg > 0.0"),
    ("cg: A without omega", "A = (2.25 * p.sigma) * omega", "A = 2.25 * p.sigma"),
]

PARTICLES = [
    ("particles: surface velocity r_b x omega as printed",
     "    ub = [v[..., 0] + (w[..., 1] * rb[2] - w[..., 2] * rb[1]),\n"
     "          v[..., 1] + (w[..., 2] * rb[0] - w[..., 0] * rb[2]),\n"
     "          v[..., 2] + (w[..., 0] * rb[1] - w[..., 1] * rb[0])]",
     "    ub = [v[..., 0] + (rb[1] * w[..., 2] - rb[2] * w[..., 1]),\n"
     "          v[..., 1] + (rb[2] * w[..., 0] - rb[0] * w[..., 2]),\n"
     "          v[..., 2] + (rb[0] * w[..., 1] - rb[1] * w[..., 0])]"),
    ("particles: moving-wall term halved", "return (6.0 * W[i]) * (rho * cub), rb", "return (3.0 * W[i]) * (rho * cub), rb"),
    ("particles: moving-wall term at unit density", "return (6.0 * W[i]) * (rho * cub), rb",
     "return (6.0 * W[i]) * cub, rb"),
    ("particles: link force counts the reflected population once", "t = (g + g) + Wi", "t = g + Wi"),
    ("particles: covered momentum not handed over", "            sign = 1.0", "            sign = 0.0"),
    ("particles: uncovered node starts at rest",
     "vals = O.equilibrium(np.float64(rho0), np.float64(ub[0]), np.float64(ub[1]), np.float64(ub[2]))",
     "vals = O.equilibrium(np.float64(rho0), np.float64(0.0), np.float64(0.0), np.float64(0.0))"),
    ("particles: torque sign", "Ti = [rb[1] * Fi[2] - rb[2] * Fi[1], rb[2] * Fi[0] - rb[0] * Fi[2], rb[0] * Fi[1] - rb[1] * Fi[0]]",
     "Ti = [rb[2] * Fi[1] - rb[1] * Fi[2], rb[0] * Fi[2] - rb[2] * Fi[0], rb[1] * Fi[0] - rb[0] * Fi[1]]"),
]

CG_PARTICLES = [
    ("cg particles: wall wetted by fluid 1", "t = W[i] * np.where(nb_solid, theta, nb)",
     "t = W[i] * np.where(nb_solid, 1.0, nb)"),
    ("cg particles: wall as a half-and-half mixture", "t = W[i] * np.where(nb_solid, theta, nb)",
     "t = W[i] * np.where(nb_solid, 0.0, nb)"),
    ("cg particles: wall term with the mixture density per component",
     "Wi, _ = PT._wall(i, x, y, z, rho[k], pidx, part, shape)",
     "Wi, _ = PT._wall(i, x, y, z, rho[0] + rho[1], pidx, part, shape)"),
    ("cg particles: covering and uncovering exchange one component only", "mom = O.momentum(vals.reshape(Q, 1))",
     "mom = O.momentum(vals.reshape(Q, 1) * (k == 0))"),
    ("cg particles: uncovered node at the other component's density",
     "vals = O.equilibrium(np.float64(rho0[k]),", "vals = O.equilibrium(np.float64(rho0[1 - k]),"),
    ("cg particles: link force counts the reflected population once", "t = (g + g) + Wi", "t = g + Wi"),
]

RUNNER = r"""
import importlib.util, sys
sys.path.insert(0, {root!r})
import oracle
spec = importlib.util.spec_from_file_location({modname!r}, {path!r})
m = importlib.util.module_from_spec(spec)
m.__package__ = "oracle"
sys.modules[{modname!r}] = m
spec.loader.exec_module(m)
setattr(oracle, {attr!r}, m)
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not slow", *{tests!r}]))
"""


def _run_mutant(src_file, modname, attr, old, new, tests):
    src = open(os.path.join(ROOT, "oracle", src_file)).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, src_file)
        with open(path, "w") as fh:
            fh.write(src.replace(old, new, 1))
        code = RUNNER.format(root=ROOT, modname=modname, path=path, attr=attr, tests=tests)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=600)
    return r.returncode


@pytest.mark.parametrize("name,old,new", FORWARD, ids=[m[0] for m in FORWARD])
def test_forward_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_units.py"), os.path.join(TESTS, "test_oracle_physics.py")]
    rc = _run_mutant("lb_oracle.py", "oracle.lb_oracle", "lb_oracle", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


@pytest.mark.parametrize("name,old,new,pin", READINGS, ids=[m[0] for m in READINGS])
def test_reading_pin_alone_catches_planted_mistake(name, old, new, pin):
    rc = _run_mutant("lb_oracle.py", "oracle.lb_oracle", "lb_oracle", old, new, [os.path.join(TESTS, pin)])
    assert rc != 0, f"{pin} did not catch the planted mistake: {name}"


@pytest.mark.parametrize("name,old,new", ADJOINT, ids=[m[0] for m in ADJOINT])
def test_adjoint_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_adjoint.py")]
    rc = _run_mutant("lb_adjoint.py", "oracle.lb_adjoint", "lb_adjoint", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


@pytest.mark.parametrize("name,old,new", SINGLE, ids=[m[0] for m in SINGLE])
def test_single_fluid_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_single.py")]
    rc = _run_mutant("lb_single.py", "oracle.lb_single", "lb_single", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


@pytest.mark.parametrize("name,old,new", COLOUR, ids=[m[0] for m in COLOUR])
def test_colour_gradient_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_cg.py")]
    rc = _run_mutant("lb_cg.py", "oracle.lb_cg", "lb_cg", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


@pytest.mark.parametrize("name,old,new", PARTICLES, ids=[m[0] for m in PARTICLES])
def test_particle_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_particles.py")]
    rc = _run_mutant("lb_particles.py", "oracle.lb_particles", "lb_particles", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


@pytest.mark.parametrize("name,old,new", CG_PARTICLES, ids=[m[0] for m in CG_PARTICLES])
def test_cg_particle_pins_catch_planted_mistake(name, old, new):
    tests = [os.path.join(TESTS, "test_oracle_cg_particles.py")]
    rc = _run_mutant("lb_cg_particles.py", "oracle.lb_cg_particles", "lb_cg_particles", old, new, tests)
    assert rc != 0, f"no pin failed for planted mistake: {name}"


def test_unmutated_oracle_passes_through_the_same_runner():
    # the runner itself must not fail on the real oracle
    tests = [os.path.join(TESTS, "test_oracle_adjoint.py")]
    rc = _run_mutant("lb_adjoint.py", "oracle.lb_adjoint", "lb_adjoint", "import numpy as np", "import numpy as np",
                     tests)
    assert rc == 0


@pytest.mark.parametrize("pin", [THRESHOLD, FLAT])
def test_reading_pins_pass_on_the_real_oracle_through_the_runner(pin):
    # a pin selected by node id must run and pass unmutated (pytest's "no
    # tests collected" would also be a non-zero exit)
    rc = _run_mutant("lb_oracle.py", "oracle.lb_oracle", "lb_oracle", "import numpy as np", "import numpy as np",
                     [os.path.join(TESTS, pin)])
    assert rc == 0


def test_unmutated_cg_particle_oracle_passes_through_the_runner():
    tests = [os.path.join(TESTS, "test_oracle_cg_particles.py")]
    rc = _run_mutant("lb_cg_particles.py", "oracle.lb_cg_particles", "lb_cg_particles", "import numpy as np",
                     "import numpy as np", tests)
    assert rc == 0
