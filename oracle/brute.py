"""Naive per-node NumPy evaluation of the mimetic right-hand side, for tiny grids (<= 8^3).

TEST INFRASTRUCTURE, a second hand-written reading of the same formulas as oracle.c,
written in a different form so that a slip in one shows up against the other:
  * positions of neighbours through an explicit ghost rule (Sec. 2.5),
  * F from the three-point formulas, Delta with numpy.linalg.det,
  * B = F B0 / Delta (Sec. 2.1, eq. "B transformation"),
  * the loop circulation with edge-averaged B (Sec. 2.2, eq. "current discrete"),
  * the area vector in its second form, (dx1 x dx2 + dx2 x dx3 + dx3 x dx4 + dx4 x dx1)/4
    (Sec. 2.2, eq. "sum of triangles"),
  * J from numpy.linalg.solve of the 3x3 system (eq. "current matrix equation"),
  * u = gamma J x B, zero on line-tied faces, E_M with zeta weights (eq. "magnetic energy"),
    xi = max |J x B| / B^2 over interior nodes.
Pure Python loops: for 8^3-sized grids only.
"""
from __future__ import annotations

import numpy as np


def _pos(x, grid, idx):
    """x at integer index idx (may lie one or two nodes outside a periodic axis)."""
    n, h, bc = grid.n, grid.h, grid.bc
    q = list(idx)
    shift = np.zeros(3)
    for a in range(3):
        if bc[a] == 1:
            w, q[a] = divmod(q[a], n[a])
            shift[a] = w * n[a] * h[a]
        else:
            assert 0 <= q[a] < n[a]
    i, j, k = q
    return x[:, k, j, i] + shift, (i, j, k)


def _F(x, grid, p):
    F = np.zeros((3, 3))
    for a in range(3):
        e = np.zeros(3, dtype=int)
        e[a] = 1
        n_a = grid.n[a]
        if grid.bc[a] == 1 or 0 < p[a] < n_a - 1:
            F[:, a] = (_pos(x, grid, p + e)[0] - _pos(x, grid, p - e)[0]) / (2 * grid.h[a])
        elif p[a] == 0:
            F[:, a] = (-3 * _pos(x, grid, p)[0] + 4 * _pos(x, grid, p + e)[0]
                       - _pos(x, grid, p + 2 * e)[0]) / (2 * grid.h[a])
        else:
            F[:, a] = (3 * _pos(x, grid, p)[0] - 4 * _pos(x, grid, p - e)[0]
                       + _pos(x, grid, p - 2 * e)[0]) / (2 * grid.h[a])
    return F


def _boundary(grid, p):
    return any(grid.bc[a] == 0 and (p[a] == 0 or p[a] == grid.n[a] - 1) for a in range(3))


def rhs(grid, x, B0, gamma=1.0, tau_B2=0.0):
    """Returns dict(u, J, B, det, E_M, xi, R2, min_det)."""
    nx, ny, nz = grid.n
    B = np.zeros_like(x)
    det = np.zeros(x.shape[1:])
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                F = _F(x, grid, np.array([i, j, k]))
                D = np.linalg.det(F)
                det[k, j, i] = D
                B[:, k, j, i] = F @ B0[:, k, j, i] / D
    J = np.zeros_like(x)
    u = np.zeros_like(x)
    xi, R2, E = 0.0, 0.0, 0.0
    dV = grid.h[0] * grid.h[1] * grid.h[2]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                p = np.array([i, j, k])
                zeta = 1.0
                for a in range(3):
                    if grid.bc[a] == 0 and p[a] in (0, grid.n[a] - 1):
                        zeta *= 0.5
                Bp = B[:, k, j, i]
                E += 0.5 * zeta * (Bp @ Bp) * det[k, j, i] * dV
                if _boundary(grid, p):
                    continue
                rows, rhs_ = [], []
                # planes (a, b) with normal q: q=x -> (y, z), q=y -> (z, x), q=z -> (x, y)
                for a, b in ((1, 2), (2, 0), (0, 1)):
                    ea = np.eye(3, dtype=int)[a]
                    eb = np.eye(3, dtype=int)[b]
                    verts = [p + ea, p + eb, p - ea, p - eb]
                    X = [_pos(x, grid, v)[0] for v in verts]
                    Bv = []
                    for v in verts:
                        _, (ii, jj, kk) = _pos(x, grid, v)
                        Bv.append(B[:, kk, jj, ii])
                    dx = [X[(r + 1) % 4] - X[r] for r in range(4)]
                    circ = sum(0.5 * (Bv[r] + Bv[(r + 1) % 4]) @ dx[r] for r in range(4))
                    nA = sum(np.cross(dx[r], dx[(r + 1) % 4]) for r in range(4)) / 4.0
                    rows.append(nA)
                    rhs_.append(circ)
                Jp = np.linalg.solve(np.array(rows), np.array(rhs_))
                f = np.cross(Jp, Bp)
                J[:, k, j, i] = Jp
                u[:, k, j, i] = gamma * f
                R2 += 0.5 * det[k, j, i] * (f @ f) * dV
                B2 = Bp @ Bp
                if B2 > tau_B2:
                    xi = max(xi, np.sqrt(f @ f) / B2)
    return {"u": u, "J": J, "B": B, "det": det, "E_M": E, "xi": xi, "R2": R2, "min_det": det.min()}
