"""FP64 CPU oracle for the two-component colour-gradient D3Q19 step, the
paper's own model for two immiscible fluids (Sec. 2; Appendix; case 2 of
Sec. 5).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library never
does, and this module imports nothing from it.

What it follows (Appendix, colour-gradient model):

* two population sets f_i^k on the D3Q19 lattice of ``lb_oracle``;
  rho^k = sum_i f_i^k, rho = rho^1 + rho^2 and the mixture momentum
  rho u = sum_k sum_i f_i^k c_i;
* the collision operator is the recolouring step applied to the sum of the
  BGK part and the perturbation part;
* BGK part: omega (f_i^{k,eq} - f_i^k) with f^{k,eq} the second-order
  equilibrium (Eq. LEQ) of rho^k at the mixture velocity u, and one
  effective omega for both components from the mean viscosity
  1/nu_bar = (rho^1/rho)/nu_1 + (rho^2/rho)/nu_2, nu_k = c_s^2 (tau_k - 1/2)
  (Eq. 2);
* perturbation part (Eq. 2coll): (A_k / 2) |grad Theta| [w_i (c_i . n)^2 - B_i]
  with n = grad Theta / |grad Theta|, the phase field
  Theta = (rho^1 - rho^2) / (rho^1 + rho^2), B_i from the Appendix table and
  A_1 = A_2 = A, where A follows from the surface tension by Eq. sigmaA,
  sigma = (4/9) A / omega, evaluated with the node's own omega;
* recolouring (Eq. 3coll, after Latva-Kokko and Rothman):
  f_i^1 = (rho^1/rho) f*_i + beta (rho^1 rho^2 / rho^2) cos(phi_i) f_i^{eq,0},
  f_i^2 = (rho^2/rho) f*_i - beta (rho^1 rho^2 / rho^2) cos(phi_i) f_i^{eq,0},
  where f*_i is the sum over both components of the post-perturbation
  populations, cos(phi_i) the cosine of the angle between c_i and
  grad Theta, and f_i^{eq,0} = w_i rho the total equilibrium at rest;
* streaming f_i^k(x + c_i, t + 1) = (post-recolouring) f_i^k(x, t) on a
  periodic box (``lb_oracle.stream``).

Readings where the paper is silent or its text is garbled:

* The printed effective relaxation rate 2/(6 nu_bar - 1) is read as
  2/(6 nu_bar + 1), the inverse of the relaxation time tau_bar that gives
  nu_bar = (tau_bar - 1/2)/3 in Eq. 2 (the printed form is negative for
  nu_bar < 1/6 and does not reduce to 1/tau for a single fluid).
* The denominator rho^2 of the recolouring coefficient is the square of the
  total density rho (its numerator is the product of the two component
  densities), so the coefficient is beta rho^1 rho^2 / rho^2 = beta c1 c2
  with c_k = rho^k / rho.
* The phase-field gradient is not given; it is the isotropic central
  difference grad Theta(x) = (1/c_s^2) sum_{i=1..18} w_i Theta(x + c_i) c_i
  with the D3Q19 weights.
* cos(phi_i) = (c_i . n) / |c_i|, and zero for the rest direction.
* The perturbation and the recolouring act only near the interface (the
  paper says so of both, Sec. 2): here, where |grad Theta|^2 > 1e-16.
  Elsewhere both are zero and n is not formed.  Without such a cut a
  uniform mixture, where grad Theta vanishes in exact arithmetic, would be
  recoloured along the direction of its rounding noise.
* The recolouring is applied to every node; f*_i in it is
  f_i^{1,*} + f_i^{2,*} with f_i^{k,*} = f_i^k + Omega^(1) + Omega^(2).
* No solid nodes: case 2 is a periodic box, and walls in this model need a
  wetting rule that the paper does not give.

Order of floating-point operations (fixed so that an implementation doing
the same IEEE operations in the same order agrees bit for bit):

* rho^k and m^k as in ``lb_oracle`` (index order); rho = rho^1 + rho^2;
  u_a = (m^1_a + m^2_a) / rho; Theta = (rho^1 - rho^2) / rho.
* S_a = sum_{i=1..18} c_ia (w_i Theta(x + c_i)) in index order
  (``lb_oracle.sc_sum``); g_a = 3 S_a.
* 1/nu_bar = (rho^1 / rho) inv_nu_1 + (rho^2 / rho) inv_nu_2 with
  inv_nu_k = 1 / ((tau_k - 0.5) / 3); nu_bar = 1 / (1/nu_bar);
  omega = 2 / (6 nu_bar + 1); A = (2.25 sigma) omega.
* gg = (g_x g_x + g_y g_y) + g_z g_z; where gg > 1e-16: |g| = sqrt(gg) and
  n_a = g_a / |g|, else |g| = n_a = 0; c.n = (c_x n_x + c_y n_y) + c_z n_z;
  P_i = ((0.5 A) |g|) (w_i (c.n c.n) - B_i).
* f^{k,eq} as ``lb_oracle.equilibrium``; f_i^{k,*} = (f_i^k + omega (f_i^{k,eq} - f_i^k)) + P_i;
  f*_i = f_i^{1,*} + f_i^{2,*}.
* r = (beta (rho^1 rho^2)) / (rho rho); cos(phi_i) = c.n / |c_i| with |c_i| = 1
  or sqrt(2) (the double nearest to it); t_i = (r cos(phi_i)) (w_i rho);
  f_i^1 = (rho^1 / rho) f*_i + t_i, f_i^2 = (rho^2 / rho) f*_i - t_i.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Tuple

import numpy as np

from . import lb_oracle as O

Q = O.Q
C = O.C
W = O.W

# B_i of the perturbation operator (Appendix table): -2/9 at rest, 1/54 on the
# axes, 1/27 on the face diagonals.
B = np.array([-2.0 / 9.0] + [1.0 / 54.0] * 6 + [1.0 / 27.0] * 12, dtype=np.float64)
# The perturbation and the recolouring act near the interface only: where
# |grad Theta| > 1e-8.  (A uniform mixture has grad Theta = 0 in exact
# arithmetic; rounding leaves |g| ~ 1e-16 there, whose direction is noise.)
INTERFACE_G2 = 1e-16
# |c_i| (0 for the rest vector is replaced by 1: c.n is 0 there anyway).
CLEN = np.array([1.0] + [1.0] * 6 + [math.sqrt(2.0)] * 12, dtype=np.float64)


@dataclasses.dataclass(frozen=True)
class Params:
    """tau of each pure component (nu_k = (tau_k - 1/2)/3), the surface tension
    sigma and the recolouring parameter beta."""

    tau: Tuple[float, float] = (1.0, 1.0)
    sigma: float = 0.0
    beta: float = 0.0

    @property
    def inv_nu(self) -> Tuple[float, float]:
        return tuple(1.0 / ((t - 0.5) / 3.0) for t in self.tau)


def phase_field(rho1: np.ndarray, rho2: np.ndarray) -> np.ndarray:
    """Theta = (rho^1 - rho^2) / (rho^1 + rho^2)."""
    return (rho1 - rho2) / (rho1 + rho2)


def gradient(theta: np.ndarray):
    """grad Theta = 3 sum_{i=1..18} w_i Theta(x + c_i) c_i (periodic)."""
    S = O.sc_sum(theta)
    return tuple(3.0 * S[a] for a in range(3))


def effective_omega(rho1, rho2, p: Params):
    """omega = 2 / (6 nu_bar + 1), 1/nu_bar = (rho^1/rho)/nu_1 + (rho^2/rho)/nu_2."""
    rho = rho1 + rho2
    inv = p.inv_nu
    inv_nubar = (rho1 / rho) * inv[0] + (rho2 / rho) * inv[1]
    nubar = 1.0 / inv_nubar
    return 2.0 / (6.0 * nubar + 1.0)


def unit_normal(g):
    """(n, |g|) at interface nodes (|g|^2 > INTERFACE_G2): n = g / |g|;
    elsewhere both are 0, which switches the perturbation and the
    recolouring off."""
    gg = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]
    pos = gg > INTERFACE_G2
    gn = np.where(pos, np.sqrt(gg), 0.0)
    safe = np.where(pos, gn, 1.0)
    n = tuple(np.where(pos, g[a] / safe, 0.0) for a in range(3))
    return n, gn


def c_dot(i: int, v) -> np.ndarray:
    return (C[i, 0] * v[0] + C[i, 1] * v[1]) + C[i, 2] * v[2]


def perturbation(n, gn, A):
    """Per-component perturbation (Eq. 2coll), [19] list of fields:
    (A / 2) |g| (w_i (c_i . n)^2 - B_i), and the list of c_i . n."""
    pcoef = (0.5 * A) * gn
    cn = [c_dot(i, n) for i in range(Q)]
    return [pcoef * (W[i] * (cn[i] * cn[i]) - B[i]) for i in range(Q)], cn


def recolour(fstar, rho1, rho2, cn, beta):
    """Split the total post-perturbation populations fstar [19][...] between
    the components (Eq. 3coll); cn[i] = c_i . n."""
    rho = rho1 + rho2
    r = (beta * (rho1 * rho2)) / (rho * rho)
    c1 = rho1 / rho
    c2 = rho2 / rho
    out = np.empty((2,) + fstar.shape, dtype=np.float64)
    for i in range(Q):
        t = (r * (cn[i] / CLEN[i])) * (W[i] * rho)
        out[0, i] = c1 * fstar[i] + t
        out[1, i] = c2 * fstar[i] - t
    return out


def collide(f: np.ndarray, p: Params):
    """Post-collision (post-recolouring) populations [2][19][nz][ny][nx]."""
    rho1 = O.density(f[0])
    rho2 = O.density(f[1])
    rho = rho1 + rho2
    m1 = O.momentum(f[0])
    m2 = O.momentum(f[1])
    u = tuple((m1[a] + m2[a]) / rho for a in range(3))
    theta = (rho1 - rho2) / rho
    n, gn = unit_normal(gradient(theta))
    omega = effective_omega(rho1, rho2, p)
    A = (2.25 * p.sigma) * omega
    pert, cn = perturbation(n, gn, A)
    feq = [O.equilibrium(rho1, *u), O.equilibrium(rho2, *u)]
    fstar = np.empty_like(f[0])
    for i in range(Q):
        fa = (f[0, i] + omega * (feq[0][i] - f[0, i])) + pert[i]
        fb = (f[1, i] + omega * (feq[1][i] - f[1, i])) + pert[i]
        fstar[i] = fa + fb
    return recolour(fstar, rho1, rho2, cn, p.beta)


def step(f: np.ndarray, p: Params, n: int = 1) -> np.ndarray:
    """Advance the pre-collision state ``f`` [2][19][nz][ny][nx] by ``n`` steps (periodic box)."""
    for _ in range(int(n)):
        f = O.stream(collide(f, p))
    return f


def init_equilibrium(rho1: np.ndarray, rho2: np.ndarray, u=None) -> np.ndarray:
    """f_i^k(x, 0) = f_i^eq(rho^k(x), u(x)); u = (ux, uy, uz) or None for rest."""
    return O.init_equilibrium(rho1, rho2, u)


def moments(f: np.ndarray):
    """(rho^1, rho^2, (ux, uy, uz)) of the pre-collision state, u = sum_k m^k / rho."""
    rho1 = O.density(f[0])
    rho2 = O.density(f[1])
    rho = rho1 + rho2
    m1 = O.momentum(f[0])
    m2 = O.momentum(f[1])
    return rho1, rho2, tuple((m1[a] + m2[a]) / rho for a in range(3))


def pressure(f: np.ndarray) -> np.ndarray:
    """p = c_s^2 rho, the mixture's equation of state."""
    return O.CS2 * (O.density(f[0]) + O.density(f[1]))


def totals(f: np.ndarray):
    """(M_1, M_2, P_x, P_y, P_z) as correctly rounded sums and a non-finite flag."""
    return O.totals(f)
