"""Per-node brute-force twin of the oracle step (test infrastructure only).

It computes the same step as ``lb_oracle.step`` one node at a time with
plain Python floats, explicit modulo indexing and ``math.exp``; nothing is
vectorised or shifted as a whole array.  Agreement between the two on tiny
lattices pins the vectorised oracle's neighbour indexing, wrap-around, force
stencil, collision and bounce-back bookkeeping.  ``step_at`` evaluates the
next state at chosen nodes only, so single sites of a large lattice can be
checked without running a whole oracle step.

Model (paper Sec. 2, Eq. 1; Appendix, Eq. LEQ and the weight table; halfway
bounce-back at rest, Appendix Eq. LADDFLBE) with the Shan-Chen force
F_k = -G psi_k sum_i w_i psi_kbar(x + c_i) c_i, psi = rho_0 (1 - e^{-rho/rho_0}),
applied by shifting the equilibrium velocity to u' + tau_k F_k / rho_k.
"""

from __future__ import annotations

import math

import numpy as np

# Velocity set written out independently of lb_oracle: (cx, cy, cz, w).
_VEL = [
    (0, 0, 0, 1.0 / 3.0),
    (1, 0, 0, 1.0 / 18.0), (-1, 0, 0, 1.0 / 18.0),
    (0, 1, 0, 1.0 / 18.0), (0, -1, 0, 1.0 / 18.0),
    (0, 0, 1, 1.0 / 18.0), (0, 0, -1, 1.0 / 18.0),
    (1, 1, 0, 1.0 / 36.0), (-1, -1, 0, 1.0 / 36.0),
    (1, -1, 0, 1.0 / 36.0), (-1, 1, 0, 1.0 / 36.0),
    (1, 0, 1, 1.0 / 36.0), (-1, 0, -1, 1.0 / 36.0),
    (1, 0, -1, 1.0 / 36.0), (-1, 0, 1, 1.0 / 36.0),
    (0, 1, 1, 1.0 / 36.0), (0, -1, -1, 1.0 / 36.0),
    (0, 1, -1, 1.0 / 36.0), (0, -1, 1, 1.0 / 36.0),
]


def _opposite(i: int) -> int:
    cx, cy, cz, _ = _VEL[i]
    for j, (dx, dy, dz, _) in enumerate(_VEL):
        if (dx, dy, dz) == (-cx, -cy, -cz):
            return j
    raise AssertionError


class _Lattice:
    def __init__(self, f, tau, G, psi_ref, solid):
        self.f = f
        self.nz, self.ny, self.nx = f.shape[-3:]
        self.tau = (float(tau[0]), float(tau[1]))
        self.G = float(G)
        self.psi_ref = float(psi_ref)
        self.solid = solid
        self._local = {}
        self._post = {}

    def wrap(self, x, y, z):
        return x % self.nx, y % self.ny, z % self.nz

    def is_solid(self, x, y, z):
        if self.solid is None:
            return False
        return bool(self.solid[z, y, x])

    def local(self, x, y, z):
        """(rho_k, psi_k, m_k) for k = A, B at one node; zeros at solid nodes."""
        key = (x, y, z)
        if key in self._local:
            return self._local[key]
        out = []
        for k in range(2):
            if self.is_solid(x, y, z):
                out.append((0.0, 0.0, (0.0, 0.0, 0.0)))
                continue
            vals = [float(self.f[k, i, z, y, x]) for i in range(19)]
            rho = 0.0
            for v in vals:
                rho += v
            mx = sum(v * c[0] for v, c in zip(vals, _VEL))
            my = sum(v * c[1] for v, c in zip(vals, _VEL))
            mz = sum(v * c[2] for v, c in zip(vals, _VEL))
            psi = self.psi_ref * (1.0 - math.exp(-rho / self.psi_ref))
            out.append((rho, psi, (mx, my, mz)))
        self._local[key] = out
        return out

    def post_collision(self, x, y, z):
        """The 2 x 19 post-collision populations at one fluid node."""
        key = (x, y, z)
        if key in self._post:
            return self._post[key]
        loc = self.local(x, y, z)
        S = []
        for k in range(2):
            other = 1 - k
            sx = sy = sz = 0.0
            for cx, cy, cz, w in _VEL[1:]:
                psi_n = self.local(*self.wrap(x + cx, y + cy, z + cz))[other][1]
                sx += w * psi_n * cx
                sy += w * psi_n * cy
                sz += w * psi_n * cz
            S.append((sx, sy, sz))
        om = (1.0 / self.tau[0], 1.0 / self.tau[1])
        den = om[0] * loc[0][0] + om[1] * loc[1][0]
        up = [(om[0] * loc[0][2][a] + om[1] * loc[1][2][a]) / den for a in range(3)]
        res = []
        for k in range(2):
            rho, psi, _ = loc[k]
            F = [-self.G * psi * S[k][a] for a in range(3)]
            if rho != 0.0:
                v = [up[a] + self.tau[k] * F[a] / rho for a in range(3)]
            else:
                v = [up[a] - self.tau[k] * self.G * S[k][a] for a in range(3)]
            vv = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
            row = []
            for i, (cx, cy, cz, w) in enumerate(_VEL):
                cu = cx * v[0] + cy * v[1] + cz * v[2]
                feq = w * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * vv)
                fi = float(self.f[k, i, z, y, x])
                row.append(fi + om[k] * (feq - fi))
            res.append(row)
        self._post[key] = res
        return res

    def new_value(self, k, i, x, y, z):
        """f_i^k(x, t+1) with pull streaming and halfway bounce-back."""
        if self.is_solid(x, y, z):
            return 0.0
        cx, cy, cz, _ = _VEL[i]
        src = self.wrap(x - cx, y - cy, z - cz)
        if self.is_solid(*src):
            return self.post_collision(x, y, z)[k][_opposite(i)]
        return self.post_collision(*src)[k][i]


def step(f: np.ndarray, tau, G: float, psi_ref: float = 1.0, solid=None, n: int = 1) -> np.ndarray:
    """``n`` whole-lattice steps, node by node (tiny lattices only)."""
    for _ in range(int(n)):
        lat = _Lattice(f, tau, G, psi_ref, solid)
        out = np.zeros_like(f)
        nz, ny, nx = f.shape[-3:]
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    for k in range(2):
                        for i in range(19):
                            out[k, i, z, y, x] = lat.new_value(k, i, x, y, z)
        f = out
    return f


def step_at(f: np.ndarray, sites, tau, G: float, psi_ref: float = 1.0, solid=None) -> np.ndarray:
    """f(t+1) at the nodes ``sites`` [(x, y, z), ...]; returns [len(sites), 2, 19]."""
    lat = _Lattice(f, tau, G, psi_ref, solid)
    out = np.zeros((len(sites), 2, 19), dtype=np.float64)
    for s, (x, y, z) in enumerate(sites):
        for k in range(2):
            for i in range(19):
                out[s, k, i] = lat.new_value(k, i, int(x), int(y), int(z))
    return out
