"""FP64 CPU oracle for the single-fluid D3Q19 BGK step (the paper's case 1).

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark import this module; the GPU library never
does, and this module imports nothing from it.

What it follows (the paper's single-fluid fused step, Sec. 5 case 1):

* one population set f_i on the D3Q19 lattice of ``lb_oracle`` (Sec. 2;
  weights from the Appendix table);
* rho = sum_i f_i, m = sum_i f_i c_i and the fluid velocity u = m / rho;
* BGK relaxation f* = (1 - omega) f + omega f^eq(rho, u), omega = 1/tau
  (Sec. 2, Eq. 1), with the second-order equilibrium of the Appendix
  (Eq. LEQ, c_s^2 = 1/3), so the kinematic viscosity is (tau - 1/2)/3
  (Sec. 2, Eq. 2);
* streaming f_i(x + c_i, t + 1) = f*_i(x, t) on a periodic box, and halfway
  bounce-back at solid nodes at rest (Appendix, Eq. LADDFLBE with the wall
  velocity set to zero); solid nodes do not collide and hold zeros.

Order of floating-point operations: rho and m exactly as ``lb_oracle``
forms them; u_a = m_a / rho; f^eq and f* as ``lb_oracle`` writes them.
"""

from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import lb_oracle as O


def collide(f: np.ndarray, tau: float, solid: Optional[np.ndarray] = None) -> np.ndarray:
    """Post-collision populations f* [19][nz][ny][nx]; zero at solid nodes."""
    s = O._fluid(f.shape[-3:], solid)
    rho = O.density(f)
    m = O.momentum(f)
    den = rho if s is None else np.where(s, 1.0, rho)
    u = [m[a] / den for a in range(3)]
    om = 1.0 / tau
    feq = O.equilibrium(rho, u[0], u[1], u[2])
    fs = (1.0 - om) * f + om * feq
    if s is not None:
        fs[:, s] = 0.0
    return fs


def step(f: np.ndarray, tau: float, solid: Optional[np.ndarray] = None, n: int = 1) -> np.ndarray:
    """Advance the pre-collision state ``f`` [19][nz][ny][nx] by ``n`` steps."""
    for _ in range(int(n)):
        f = O.stream(collide(f, tau, solid)[None], solid)[0]
    return f


def init_equilibrium(rho: np.ndarray, u=None, solid: Optional[np.ndarray] = None) -> np.ndarray:
    """f_i(x, 0) = f_i^eq(rho(x), u(x)); zero at solid nodes.  u = (ux, uy, uz) or None for rest."""
    rho = np.asarray(rho, dtype=np.float64)
    if u is None:
        z = np.zeros_like(rho)
        u = (z, z, z)
    f = O.equilibrium(rho, *u)
    s = O._fluid(rho.shape, solid)
    if s is not None:
        f[:, s] = 0.0
    return f


def moments(f: np.ndarray, solid: Optional[np.ndarray] = None):
    """(rho, (ux, uy, uz)) of the pre-collision state, u = m / rho; zero at solid nodes."""
    s = O._fluid(f.shape[-3:], solid)
    rho = O.density(f)
    m = O.momentum(f)
    den = rho if s is None else np.where(s, 1.0, rho)
    u = []
    for a in range(3):
        ua = m[a] / den
        if s is not None:
            ua = np.where(s, 0.0, ua)
        u.append(ua)
    if s is not None:
        rho = np.where(s, 0.0, rho)
    return rho, tuple(u)


def totals(f: np.ndarray):
    """(M, P_x, P_y, P_z) as correctly rounded sums (math.fsum) and a non-finite flag."""
    nonfinite = not bool(np.all(np.isfinite(f)))
    M = math.fsum(O.density(f).ravel())
    m = O.momentum(f)
    return (M, math.fsum(m[0].ravel()), math.fsum(m[1].ravel()), math.fsum(m[2].ravel())), nonfinite
