"""Per-node brute-force twin of the colour-gradient oracle step (test
infrastructure only).

The same model as ``lb_cg`` (Appendix: BGK with the mean-viscosity omega,
the perturbation of Eq. 2coll with A from Eq. sigmaA, the recolouring of
Eq. 3coll, periodic streaming), computed one node at a time with plain
Python floats, explicit modulo indexing and ``math.sqrt``.  Nothing is
shared with ``lb_cg`` or ``lb_oracle``: the velocity set, weights and B_i
are written out again, and the arithmetic is arranged the way the paper
prints it ((c_i . g)^2 / |g|^2 and (c_i . g) / (|c_i| |g|) rather than a unit
normal), so agreement to rounding pins the vectorised oracle's indexing,
wrap-around and term bookkeeping.  As there, the perturbation and the
recolouring act only where |grad Theta|^2 > 1e-16.
"""

from __future__ import annotations

import math

import numpy as np

# (cx, cy, cz, w, B)
_VEL = [(0, 0, 0, 1.0 / 3.0, -2.0 / 9.0)]
for _c in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]:
    _VEL.append(_c + (1.0 / 18.0, 1.0 / 54.0))
for _c in [(1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
           (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]:
    _VEL.append(_c + (1.0 / 36.0, 1.0 / 27.0))


def step(f: np.ndarray, tau, sigma: float, beta: float, n: int = 1) -> np.ndarray:
    """``n`` colour-gradient steps of the pre-collision state f [2][19][nz][ny][nx]."""
    f = np.array(f, dtype=np.float64)
    nz, ny, nx = f.shape[-3:]
    nu = [(float(t) - 0.5) / 3.0 for t in tau]
    for _ in range(int(n)):
        rho = np.zeros((2, nz, ny, nx))
        mom = np.zeros((3, nz, ny, nx))
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    for k in range(2):
                        s = 0.0
                        for i, (cx, cy, cz, _, _) in enumerate(_VEL):
                            v = float(f[k, i, z, y, x])
                            s += v
                            mom[0, z, y, x] += cx * v
                            mom[1, z, y, x] += cy * v
                            mom[2, z, y, x] += cz * v
                        rho[k, z, y, x] = s
        theta = (rho[0] - rho[1]) / (rho[0] + rho[1])
        out = np.zeros_like(f)
        for z in range(nz):
            for y in range(ny):
                for x in range(nx):
                    r1, r2 = float(rho[0, z, y, x]), float(rho[1, z, y, x])
                    r = r1 + r2
                    u = [float(mom[a, z, y, x]) / r for a in range(3)]
                    g = [0.0, 0.0, 0.0]
                    for cx, cy, cz, w, _ in _VEL[1:]:
                        th = float(theta[(z + cz) % nz, (y + cy) % ny, (x + cx) % nx])
                        g[0] += 3.0 * w * th * cx
                        g[1] += 3.0 * w * th * cy
                        g[2] += 3.0 * w * th * cz
                    g2 = g[0] ** 2 + g[1] ** 2 + g[2] ** 2
                    gabs = math.sqrt(g2)
                    nu_bar = 1.0 / (r1 / (r * nu[0]) + r2 / (r * nu[1]))
                    om = 1.0 / (3.0 * nu_bar + 0.5)
                    A = 9.0 * sigma * om / 4.0
                    uu = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
                    post = []
                    for i, (cx, cy, cz, w, Bi) in enumerate(_VEL):
                        cu = cx * u[0] + cy * u[1] + cz * u[2]
                        shape = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu
                        cg = cx * g[0] + cy * g[1] + cz * g[2]
                        pert = 0.0 if g2 <= 1e-16 else 0.5 * A * gabs * (w * cg * cg / g2 - Bi)
                        tot = 0.0
                        for k, rk in ((0, r1), (1, r2)):
                            fk = float(f[k, i, z, y, x])
                            tot += fk + om * (w * rk * shape - fk) + pert
                        clen = math.sqrt(cx * cx + cy * cy + cz * cz)
                        cosphi = 0.0 if (g2 <= 1e-16 or clen == 0.0) else cg / (clen * gabs)
                        t = beta * r1 * r2 / (r * r) * cosphi * w * r
                        post.append((r1 / r * tot + t, r2 / r * tot - t))
                    for i, (cx, cy, cz, _, _) in enumerate(_VEL):
                        zz, yy, xx = (z + cz) % nz, (y + cy) % ny, (x + cx) % nx
                        out[0, i, zz, yy, xx] = post[i][0]
                        out[1, i, zz, yy, xx] = post[i][1]
        f = out
    return f
