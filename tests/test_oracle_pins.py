"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a textbook or library
routine that the method reduces to in a special case, a closed form, an invariant, or a
second brute-force evaluation.  None of them re-types the oracle's own formulas.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute
import workloads as W


def nrel(a, b):
    """normwise relative error ||a-b||_inf / max(||b||_inf, tiny)"""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def interior(g):
    """slices (z, y, x) of the nodes off every line-tied face"""
    sl = []
    for a in (2, 1, 0):
        sl.append(slice(1, g.n[a] - 1) if g.bc[a] == W.LINE_TIED else slice(None))
    return tuple(sl)


def central_curl(g, B):
    """Textbook second-order central-difference curl of a nodal field (numpy.gradient for
    line-tied axes, numpy.roll for periodic ones); valid on interior nodes."""
    def D(f, a):  # derivative along grid axis a (0=x, 1=y, 2=z) of a (nz,ny,nx) array
        ax = 2 - a
        if g.bc[a] == W.PERIODIC:
            return (np.roll(f, -1, axis=ax) - np.roll(f, 1, axis=ax)) / (2 * g.h[a])
        return np.gradient(f, g.h[a], axis=ax, edge_order=2)
    Bx, By, Bz = B
    return np.stack([D(Bz, 1) - D(By, 2), D(Bx, 2) - D(Bz, 0), D(By, 0) - D(Bx, 1)])


# --------------------------------------------------------------------------------------
# T1: on the undistorted grid the mimetic current is the central-difference curl
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 0, 1), (1, 1, 1)])
def test_T1_undistorted_grid_gives_central_curl(bc):
    g = W.make_grid((9, 10, 11), [(-1.0, 1.4), (0.0, 2.25), (-2.0, 0.0)], bc)
    B0 = W.smooth_random_field(g, 1.0, seed=11, mmax=3) + np.random.default_rng(3).normal(size=g.shape) * 0.3
    f = oracle.fields(g, g.identity(), B0)
    Jc = central_curl(g, B0)
    s = (slice(None),) + interior(g)
    assert nrel(f["J"][s], Jc[s]) < 1e-13
    # B = B0 and Delta = 1 on the undistorted grid
    assert nrel(f["B"], B0) < 1e-14
    assert np.abs(f["det"] - 1).max() < 1e-13


# --------------------------------------------------------------------------------------
# T2: linear maps x = A X + b give B = A B0 / det A exactly, boundary nodes included
# --------------------------------------------------------------------------------------
def _affine(g, A, b):
    X = g.identity().reshape(3, -1)
    return (A @ X + np.asarray(b)[:, None]).reshape(g.shape)


@pytest.mark.parametrize("periodic_x", [False, True])
def test_T2_linear_map_pull_back(periodic_x):
    rng = np.random.default_rng(2)
    A = np.eye(3) + 0.3 * rng.standard_normal((3, 3))
    if periodic_x:  # x(X + P e_x) = x(X) + P e_x needs A e_x = e_x
        A[:, 0] = [1.0, 0.0, 0.0]
    assert np.linalg.det(A) > 0
    bc = (1, 0, 0) if periodic_x else (0, 0, 0)
    g = W.make_grid((8, 9, 7), [(-1.0, 1.0), (-0.5, 1.0), (0.0, 1.5)], bc)
    B0 = W.smooth_random_field(g, 1.0, seed=5)
    f = oracle.fields(g, _affine(g, A, [0.3, -0.2, 0.7]), B0)
    expect = np.einsum("ij,j...->i...", A, B0) / np.linalg.det(A)
    assert nrel(f["B"], expect) < 1e-14
    assert np.abs(f["det"] - np.linalg.det(A)).max() < 1e-13


# --------------------------------------------------------------------------------------
# T3: affine map and affine B0 -> J is the exact curl of B(x) (planar loops, linear B)
# --------------------------------------------------------------------------------------
def test_T3_affine_map_affine_field_exact_curl():
    rng = np.random.default_rng(7)
    A = np.eye(3) + 0.35 * rng.standard_normal((3, 3))
    assert np.linalg.det(A) > 0
    M0 = rng.standard_normal((3, 3))
    c0 = rng.standard_normal(3)
    g = W.make_grid((7, 8, 9), [(-1.0, 1.0), (-1.0, 0.8), (-0.6, 1.2)], (0, 0, 0))
    X = g.identity().reshape(3, -1)
    B0 = (M0 @ X + c0[:, None]).reshape(g.shape)
    f = oracle.fields(g, _affine(g, A, [0.1, 0.2, -0.3]), B0)
    G = A @ M0 @ np.linalg.inv(A) / np.linalg.det(A)  # dB_i/dx_j of B(x)
    curl = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    Ji = f["J"][(slice(None),) + interior(g)].reshape(3, -1)
    assert np.abs(Ji - curl[:, None]).max() < 1e-12 * max(1.0, np.abs(curl).max())


# --------------------------------------------------------------------------------------
# T4: flux through material faces, B . (dx/dX_a x dx/dX_b) = B0_q, with the Jacobian
# columns taken from numpy.gradient (second order, one-sided second order at the ends)
# --------------------------------------------------------------------------------------
def test_T4_material_face_flux():
    g = W.make_grid((9, 8, 10), [(-1.0, 1.0), (-1.0, 1.0), (-1.0, 1.0)], (0, 0, 0))
    x = W.distorted_grid(g, 0.08, seed=9)
    B0 = W.smooth_random_field(g, 1.0, seed=10)
    f = oracle.fields(g, x, B0)
    cols = [np.stack([np.gradient(x[c], g.h[a], axis=2 - a, edge_order=2) for c in range(3)]) for a in range(3)]
    for q, (a, b) in enumerate(((1, 2), (2, 0), (0, 1))):
        flux = (f["B"] * np.cross(cols[a], cols[b], axis=0)).sum(axis=0)
        assert np.abs(flux - B0[q]).max() < 1e-12 * np.abs(B0).max()


# --------------------------------------------------------------------------------------
# T5: ABC field on the undistorted periodic cube is a discrete fixed point
#     (central curl of a Beltrami field with wavenumber 1 = (sin h / h) B)
# --------------------------------------------------------------------------------------
def test_T5_abc_fixed_point():
    g = W.make_grid((16, 16, 16), [(0, 2 * math.pi)] * 3, (1, 1, 1))
    B0 = W.abc_field(g)
    f = oracle.fields(g, g.identity(), B0)
    h = g.h[0]
    assert nrel(f["J"], math.sin(h) / h * B0) < 1e-13
    assert np.abs(f["u"]).max() < 1e-13
    d = oracle.diagnostics(g, g.identity(), B0, tau_B2=oracle.null_threshold(B0))
    assert d["xi"] < 1e-12


# --------------------------------------------------------------------------------------
# T6: algebraic identity: mimetic J = F c / Delta with c_q = F_b . D_a B - F_a . D_b B
#     (F from numpy.gradient, D B the central difference of the oracle's B)
# --------------------------------------------------------------------------------------
def test_T6_compact_identity():
    g = W.make_grid((10, 9, 8), [(-1.0, 1.0)] * 3, (0, 0, 0))
    x = W.distorted_grid(g, 0.1, seed=13)
    B0 = W.smooth_random_field(g, 1.0, seed=14)
    f = oracle.fields(g, x, B0)
    s = interior(g)
    F = np.stack([np.stack([np.gradient(x[c], g.h[a], axis=2 - a) for a in range(3)]) for c in range(3)])  # F[c][a]
    G = [np.stack([np.gradient(f["B"][c], g.h[a], axis=2 - a) for c in range(3)]) for a in range(3)]  # G[a][c]
    c = np.zeros_like(x)
    for q, (a, b) in enumerate(((1, 2), (2, 0), (0, 1))):
        c[q] = (F[:, b] * G[a]).sum(axis=0) - (F[:, a] * G[b]).sum(axis=0)
    det = np.linalg.det(np.moveaxis(F, (0, 1), (-2, -1)))
    J = np.einsum("ca...,a...->c...", F, c) / det
    sl = (slice(None),) + s
    assert nrel(f["J"][sl], J[sl]) < 1e-12


# --------------------------------------------------------------------------------------
# T7: the magneto-frictional evolution lowers E_M monotonically (single twist, 16^3)
# --------------------------------------------------------------------------------------
def test_T7_energy_monotone_single_twist():
    w = W.single_twist_16()
    r = oracle.run(w.grid, w.x0, w.B0, 100, dt=w.dt0, tol=w.tol)
    E = r["diag"][:, 2]
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-14))
    V = np.prod(w.grid.lengths())
    Efree = E - 0.5 * V  # background e_z
    assert np.all(Efree[1:] <= Efree[:-1] + 1e-14 * E[0])
    assert E[-1] < E[0]
    # sign check the other way: reversing the force (gamma < 0) must raise the energy
    r2 = oracle.run(w.grid, w.x0, w.B0, 5, dt=1e-3, mode=oracle.MODE_FIXED, gamma=-1.0)
    assert r2["diag"][-1, 2] > r2["diag"][0, 2]


# --------------------------------------------------------------------------------------
# T8: IsoHelix: the pull-back evaluated at the closed-form relaxed map gives B -> e_z at
#     second order (Sec. 3.1, eqs. "B relaxed", "x analytical relaxed")
# --------------------------------------------------------------------------------------
@pytest.mark.slow
def test_T8_isohelix_relaxed_map_second_order():
    errs, umax = [], []
    for n in (17, 33, 65):
        g = W.make_grid((n, n, n), [(-4.0, 4.0), (-4.0, 4.0), (-10.0, 10.0)], (0, 0, 0))
        B0 = W.isohelix_field(g, phi=math.pi / 4)
        x = W.isohelix_relaxed_map(g, phi=math.pi / 4)
        f = oracle.fields(g, x, B0)
        s = (slice(None),) + interior(g)
        dB = f["B"][s] - np.array([0.0, 0.0, 1.0])[:, None, None, None]
        errs.append(float(np.sqrt((dB ** 2).sum(axis=0).mean())))
        umax.append(float(np.abs(f["u"]).max()))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.4 < r1 < 4.6 and 3.6 < r2 < 4.4, errs
    # u = J x B of the (force-free) limit also vanishes; n=17 (h_z = 1.25 vs a_z = 2) is
    # pre-asymptotic, the 33 -> 65 halving already shows close to second order
    assert umax[0] > umax[1] > umax[2] and umax[1] / umax[2] > 3.0, umax


# --------------------------------------------------------------------------------------
# T9: Cash-Karp tableau: order conditions over rooted trees (order 5 for b5, 4 for b4),
#     and the observed order of the step on the grid problem
# --------------------------------------------------------------------------------------
def _trees(max_order):
    """rooted trees as sorted tuples of children, grouped by order"""
    by = {1: [()]}
    for n in range(2, max_order + 1):
        out = set()

        def parts(rem, min_child, acc):
            if rem == 0:
                out.add(tuple(sorted(acc)))
                return
            for m in range(1, rem + 1):
                for t in by[m]:
                    key = (m, t)
                    if min_child is not None and key < min_child:
                        continue
                    parts(rem - m, key, acc + [t])
        parts(n - 1, None, [])
        by[n] = sorted(out)
    return by


def _order(t):
    return 1 + sum(_order(c) for c in t)


def _gamma(t):
    g = _order(t)
    for c in t:
        g *= _gamma(c)
    return g


def _phi(t, A):
    v = [Fraction(1)] * len(A)
    for c in t:
        pc = _phi(c, A)
        Ac = [sum(A[i][j] * pc[j] for j in range(len(A))) for i in range(len(A))]
        v = [v[i] * Ac[i] for i in range(len(A))]
    return v


def test_T9_tableau_order_conditions():
    A, b5, b4 = oracle.tableau()
    Af = [[Fraction(float(v)) for v in row] for row in A]
    b5f = [Fraction(float(v)) for v in b5]
    b4f = [Fraction(float(v)) for v in b4]
    trees = _trees(5)
    assert [len(trees[n]) for n in range(1, 6)] == [1, 1, 2, 4, 9]
    for n, ts in trees.items():
        for t in ts:
            target = Fraction(1, _gamma(t))
            ph = _phi(t, Af)
            assert abs(float(sum(b * p for b, p in zip(b5f, ph)) - target)) < 1e-15, (n, t)
            if n <= 4:
                assert abs(float(sum(b * p for b, p in zip(b4f, ph)) - target)) < 1e-15, (n, t)
    # explicit: strictly lower triangular
    assert np.all(np.triu(A) == 0)
    # the embedded pair differs at fifth order (otherwise the error estimate would vanish)
    diffs = [abs(float(sum((b - c) * p for b, c, p in zip(b5f, b4f, _phi(t, Af))))) for t in trees[5]]
    assert max(diffs) > 1e-6


def test_T9_observed_order_on_grid():
    g = W.make_grid((8, 8, 8), [(-1.0, 1.0)] * 3, (0, 0, 0))
    B0 = W.single_twist_field(g, k=0.6, a=0.6, l=0.6)
    x0 = g.identity()
    errs, lams = [], []
    for dt in (0.01, 0.005, 0.0025):
        x1, lam = oracle.ck_attempt(g, x0, B0, dt)
        ref = oracle.run(g, x0, B0, 64, dt=dt / 64, mode=oracle.MODE_FIXED)["x"]
        errs.append(np.abs(x1 - ref).max())
        lams.append(lam)
    # local error O(dt^6), embedded estimate O(dt^5)
    for i in range(2):
        assert 40 < errs[i] / errs[i + 1] < 80, errs
        assert 28 < lams[i] / lams[i + 1] < 40, lams


# --------------------------------------------------------------------------------------
# T10: step-size rule table (Sec. 2.4, eq. "time stepping")
# --------------------------------------------------------------------------------------
def test_T10_controller_rule_table():
    tol, dt = 1e-7, 0.01
    acc, d = oracle.controller(dt, 3 * tol, tol)  # reject and shrink
    assert not acc and d == pytest.approx(dt * (1 / 3) ** 0.2, rel=1e-15)
    acc, d = oracle.controller(dt, tol, tol)  # exactly at the limit: accepted, dt kept
    assert acc and d == dt
    acc, d = oracle.controller(dt, 0.7 * tol, tol)  # accept, keep
    assert acc and d == dt
    acc, d = oracle.controller(dt, 0.5 * tol, tol)  # not below tol/2: keep
    assert acc and d == dt
    acc, d = oracle.controller(dt, 0.1 * tol, tol)  # accept and grow
    assert acc and d == pytest.approx(dt * 10 ** 0.2, rel=1e-15)
    acc, d = oracle.controller(dt, 0.0, tol)  # zero error: grow 5x
    assert acc and d == 5 * dt
    # a safety factor scales the new step of the rule (reject and grow), not a kept step
    acc, d = oracle.controller(dt, 3 * tol, tol, safety=0.9)
    assert not acc and d == pytest.approx(0.9 * dt * (1 / 3) ** 0.2, rel=1e-15)
    acc, d = oracle.controller(dt, 0.1 * tol, tol, safety=0.9)
    assert acc and d == pytest.approx(0.9 * dt * 10 ** 0.2, rel=1e-15)
    acc, d = oracle.controller(dt, 0.7 * tol, tol, safety=0.9)
    assert acc and d == dt


def test_T10_safety_ends_reject_runs():
    """Near equilibrium the explicit step is stability-limited and Lambda barely depends on
    dt; with the rule as printed (safety 1) each retry then shrinks dt by (Lambda0/Lambda)^0.2
    ~ 1.  With safety 0.9 a rejected attempt's retry is at most 0.9 dt, so the number of
    rejects per accepted step stays small (IsoHelix, 17^3, steps 1000-1400)."""
    n = 17
    g = W.make_grid((n, n, n), [(-4, 4), (-4, 4), (-10, 10)], (0, 0, 0))
    B0 = W.isohelix_field(g, math.pi / 4)
    r = oracle.run(g, g.identity(), B0, 1400, dt=1e-3, tol=1e-8, safety=0.9)
    rej = r["diag"][1000:, 7]
    assert r["status"] == 0 and rej.max() <= 3 and rej.mean() < 1.5


def test_T10_run_matches_rule_applied_by_hand():
    w = W.single_twist_16()
    r = oracle.run(w.grid, w.x0, w.B0, 6, dt=w.dt0, tol=w.tol)
    x, dt = w.x0.copy(), w.dt0
    for s in range(6):
        rejects = 0
        while True:
            xn, lam = oracle.ck_attempt(w.grid, x, w.B0, dt)
            acc, dn = oracle.controller(dt, lam, w.tol)
            if acc:
                break
            rejects += 1
            dt = dn
        assert r["diag"][s, 1] == dt and r["diag"][s, 7] == rejects and r["diag"][s, 5] == lam
        x, dt = xn, dn
    assert np.array_equal(x, r["x"]) and r["dt"] == dt


# --------------------------------------------------------------------------------------
# T13: the relaxed IsoHelix field against the paper's Table 1 (mimetic, phi = pi/4, 17^3)
# --------------------------------------------------------------------------------------
def test_T13_isohelix_17_relaxed_state_matches_table1():
    """The oracle relaxes the IsoHelix field on the 17^3 grid of Table 1 (Lambda0 = 1e-8,
    safety 0.9) to the asymptotic sigma_B, sigma_x and eps* the paper prints, within 10 %."""
    from isohelix_util import PHI, grid, relaxed_state_errors, table1
    g = grid(17)
    B0 = W.isohelix_field(g, PHI)
    r = oracle.run(g, g.identity(), B0, 4000, dt=1e-3, tol=1e-8, safety=0.9)
    f = oracle.fields(g, r["x"], B0)
    sB, sx, eps = relaxed_state_errors(g, r["x"], f["B"], f["J"])
    p = table1()[17]
    assert abs(eps / p[1] - 1) < 0.1 and abs(sB / p[2] - 1) < 0.1 and abs(sx / p[3] - 1) < 0.1, (eps, sB, sx)


def test_T13_isohelix_pi_17_does_not_converge():
    """Table 1 marks the mimetic IsoHelix run with phi = pi on the 17^3 grid as not
    converging; the oracle's run breaks down (step size below dt_min) within 1000 steps."""
    import math
    from isohelix_util import grid, table1
    assert table1("pi")[17] is None
    g = grid(17)
    B0 = W.isohelix_field(g, math.pi)
    r = oracle.run(g, g.identity(), B0, 1000, dt=1e-3, tol=1e-8, safety=0.9, dt_min=1e-9, raise_on_error=False)
    assert r["status"] == oracle.E_DT and r["done"] < 1000, (r["status"], r["done"])


def test_T13_pontin09_17_relaxed_eps_star_matches_table2():
    """The oracle relaxes the Pontin09 field (phi = +-pi/2) on the 17^3 grid of Table 2 to the
    asymptotic eps* the paper prints, within 20 %."""
    from isohelix_util import epsilon_star, grid, table2
    g = grid(17)
    B0 = W.pontin09_field(g, phis=(math.pi / 2, -math.pi / 2))
    r = oracle.run(g, g.identity(), B0, 2500, dt=1e-3, tol=1e-8, safety=0.9)
    eps = epsilon_star(g, oracle.alpha_star(g, r["x"], B0))
    assert abs(eps / table2()[17][1] - 1) < 0.2, eps


# --------------------------------------------------------------------------------------
# T14: convexity (Sec. 3.2.3, eqs. "dx for convexity", "convexity")
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1), (0, 1, 0)])
def test_T14_convexity_undistorted_grid(bc):
    g = W.make_grid((7, 8, 9), [(-1.0, 1.0), (0.0, 2.0), (-3.0, 3.0)], bc)
    kappa, count = oracle.convexity(g, g.identity())
    assert count == 0 and np.all(kappa == 1)


def test_T14_convexity_affine_maps():
    """x = A X + b on a line-tied grid: every trihedron's determinant is det A times that of
    the undistorted one, so det A > 0 keeps every node convex and det A < 0 makes all concave."""
    g = W.make_grid((6, 7, 8), [(-1.0, 1.0)] * 3, (0, 0, 0))
    X = g.identity()
    A = np.array([[1.2, 0.4, -0.3], [0.1, 0.9, 0.5], [-0.2, 0.3, 1.1]])
    assert np.linalg.det(A) > 0
    x = np.einsum("ij,j...->i...", A, X) + np.array([0.3, -0.2, 0.7])[:, None, None, None]
    assert oracle.convexity(g, x)[1] == 0
    R = A @ np.diag([1.0, -1.0, 1.0])  # det < 0
    x = np.einsum("ij,j...->i...", R, X)
    kappa, count = oracle.convexity(g, x)
    assert count == g.N and np.all(kappa == -1)


def test_T14_convexity_one_folded_node():
    """Dragging one interior node past its +x neighbour reverses the edges it shares, so that
    node is concave; only trihedra that contain it change, so at most it and its 6 neighbours
    become concave."""
    g = W.make_grid((8, 8, 8), [(0.0, 1.0)] * 3, (0, 0, 0))
    x = g.identity().copy()
    i, j, k = 3, 4, 4
    x[0, k, j, i] = x[0, k, j, i + 1] + 0.5 * g.h[0]
    kappa, count = oracle.convexity(g, x)
    assert kappa[k, j, i] == -1 and 1 <= count <= 7
    bad = set(zip(*np.nonzero(kappa == -1)))
    near = {(k, j, i)} | {(k + dk, j + dj, i + di) for di, dj, dk in
                          [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]}
    assert bad <= near


# --------------------------------------------------------------------------------------
# T15: alpha* (Sec. 3.2.1)
# --------------------------------------------------------------------------------------
def _helical(g, k):
    """B0 = (sin kZ, cos kZ, 0): curl B0 = k B0, a linear force-free field with alpha = k."""
    X, Y, Z = g.coords()
    return np.stack([np.sin(k * Z), np.cos(k * Z), np.zeros_like(Z)])


@pytest.mark.parametrize("k", [1.0, -2.0])
def test_T15_alpha_star_helical_field_closed_form(k):
    """On the undistorted grid B = B0 and the mimetic current reduces to central differences,
    so J = (sin kh / h) B exactly: alpha* = sin(kh) / h at every node where loops close."""
    g = W.make_grid((5, 6, 24), [(0.0, 1.0), (0.0, 1.0), (0.0, 2 * math.pi)], (1, 1, 1))
    a = oracle.alpha_star(g, g.identity(), _helical(g, k))
    h = g.h[2]
    assert np.abs(a - math.sin(k * h) / h).max() < 1e-13


def test_T15_alpha_star_rotated_grid():
    """x = R X + b with R a rotation: B and J rotate with the grid and alpha* is unchanged
    (interior nodes sin(kh)/h as above, 0 on the line-tied faces where J vanishes)."""
    g = W.make_grid((7, 8, 13), [(-1.0, 1.0), (-1.0, 1.0), (0.0, 3.0)], (0, 0, 0))
    k = 1.3
    c, s_ = math.cos(0.7), math.sin(0.7)
    Rz = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, c, -s_], [0.0, s_, c]])
    R = Rx @ Rz
    x = np.einsum("ij,j...->i...", R, g.identity()) + np.array([0.5, -1.0, 2.0])[:, None, None, None]
    a = oracle.alpha_star(g, x, _helical(g, k))
    want = np.zeros(g.shape[1:])
    want[interior(g)] = math.sin(k * g.h[2]) / g.h[2]
    assert np.abs(a - want).max() < 1e-12


def test_T15_alpha_star_sign_scale_and_null():
    """Reversing B0 leaves alpha* unchanged (J and B both flip), and so does scaling it
    (J.B and B^2 both scale with its square); B0 = 0 gives 0, not NaN."""
    g = W.make_grid((6, 6, 10), [(0.0, 1.0), (0.0, 1.0), (0.0, 2 * math.pi)], (1, 1, 1))
    x = W.distorted_grid(g, 0.1, seed=3)
    B0 = _helical(g, 1.0)
    a = oracle.alpha_star(g, x, B0)
    assert np.array_equal(a, oracle.alpha_star(g, x, -B0))
    assert np.abs(oracle.alpha_star(g, x, 2.5 * B0) - a).max() < 1e-13 * np.abs(a).max()
    assert np.all(oracle.alpha_star(g, x, np.zeros_like(B0)) == 0.0)


# --------------------------------------------------------------------------------------
# T11: invariances: translation, cyclic permutation of the axes, periodic roll
# --------------------------------------------------------------------------------------
def test_T11_translation():
    g = W.make_grid((8, 9, 10), [(-1.0, 1.0)] * 3, (1, 0, 0))
    x = W.distorted_grid(g, 0.1, seed=21)
    B0 = W.smooth_random_field(g, 1.0, seed=22)
    a = oracle.fields(g, x, B0)
    b = oracle.fields(g, x + np.array([0.37, -1.3, 2.1])[:, None, None, None], B0)
    for k in ("u", "J", "B", "det"):
        assert nrel(b[k], a[k]) < 1e-12


def test_T11_cyclic_axis_permutation():
    g = W.make_grid((8, 9, 10), [(-1.0, 1.0), (0.0, 2.0), (-1.5, 1.5)], (1, 0, 1))
    x = W.distorted_grid(g, 0.1, seed=23)
    B0 = W.smooth_random_field(g, 1.0, seed=24)
    a = oracle.fields(g, x, B0)
    # new axes (x', y', z') = old (y, z, x)
    gp = W.Grid((g.n[1], g.n[2], g.n[0]), (g.h[1], g.h[2], g.h[0]), (g.bc[1], g.bc[2], g.bc[0]))

    def perm(v):
        return np.ascontiguousarray(np.roll(v, -1, axis=0).transpose(0, 3, 1, 2))
    b = oracle.fields(gp, perm(x), perm(B0))
    assert nrel(b["u"], perm(a["u"])) < 1e-13
    assert nrel(b["J"], perm(a["J"])) < 1e-13
    assert nrel(b["det"], a["det"].transpose(2, 0, 1)) < 1e-14


def test_T11_periodic_roll():
    g = W.make_grid((8, 9, 10), [(-1.0, 1.0)] * 3, (1, 1, 0))
    x = W.distorted_grid(g, 0.1, seed=25)
    B0 = W.smooth_random_field(g, 1.0, seed=26)
    a = oracle.fields(g, x, B0)
    xr = np.roll(x, -1, axis=3)
    xr[0, :, :, -1] += g.n[0] * g.h[0]
    b = oracle.fields(g, xr, np.roll(B0, -1, axis=3))
    assert nrel(b["u"], np.roll(a["u"], -1, axis=3)) < 1e-12
    xr = np.roll(x, 2, axis=2)
    xr[1, :, :2, :] -= g.n[1] * g.h[1]
    b = oracle.fields(g, xr, np.roll(B0, 2, axis=2))
    assert nrel(b["u"], np.roll(a["u"], 2, axis=2)) < 1e-12


# --------------------------------------------------------------------------------------
# T12: brute-force per-node NumPy evaluation on 8^3 grids
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_T12_brute_force_8cubed(bc):
    g = W.make_grid((8, 8, 8), [(-1.0, 1.0), (-1.2, 0.8), (0.0, 1.7)], bc)
    x = W.distorted_grid(g, 0.1, seed=31)
    B0 = W.smooth_random_field(g, 1.0, seed=32) + np.array([0, 0, 1.5])[:, None, None, None]
    tau = oracle.null_threshold(B0)
    o = oracle.fields(g, x, B0)
    d = oracle.diagnostics(g, x, B0, tau)
    r = brute.rhs(g, x, B0, tau_B2=tau)
    for k in ("u", "J", "B", "det"):
        assert nrel(o[k], r[k]) < 1e-13, k
    for k in ("E_M", "xi", "R2", "min_det"):
        assert abs(d[k] - r[k]) <= 1e-13 * abs(r[k]), k


# --------------------------------------------------------------------------------------
# The sampled right-hand side (spot checks of full-size grids) pulls B back at the loop
# vertices on the spot and decomposes flat node indices itself: against the brute-force
# evaluation on ragged grids small enough for it, and against the pinned full sweep on
# ragged grids (nx, ny, nz all different, so a transposed index shows) of every boundary mix
# --------------------------------------------------------------------------------------
BC_MIXES = [tuple(int(b) for b in f"{m:03b}"[::-1]) for m in range(8)]


def _ragged_case(n, bc, seed):
    g = W.make_grid(n, [(-1.0, 1.1), (-0.6, 0.9), (0.0, 1.7)], bc)
    x = W.distorted_grid(g, 0.08 * min(g.h), seed=seed)
    B0 = W.smooth_random_field(g, 1.0, seed=seed + 1) + np.array([0.3, -0.2, 1.2])[:, None, None, None]
    return g, x, B0


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 0, 1), (1, 1, 1)])
def test_rhs_sampled_matches_brute_force(bc):
    g, x, B0 = _ragged_case((7, 5, 6), bc, seed=41)
    r = brute.rhs(g, x, B0)
    nodes = np.arange(g.N)
    us = oracle.rhs_sampled(g, x, B0, nodes)
    assert nrel(us, r["u"].reshape(3, -1).T) < 1e-13


@pytest.mark.parametrize("bc", BC_MIXES, ids=["".join(map(str, b)) for b in BC_MIXES])
def test_rhs_sampled_matches_full_sweep(bc):
    g, x, B0 = _ragged_case((13, 9, 11), bc, seed=43)
    u = oracle.fields(g, x, B0, gamma=0.7)["u"].reshape(3, -1)
    rng = np.random.default_rng(44)
    corners = [((k * g.n[1]) + j) * g.n[0] + i for i in (0, 1, g.n[0] - 1) for j in (0, 1, g.n[1] - 1)
               for k in (0, 1, g.n[2] - 1)]
    nodes = np.concatenate([rng.permutation(g.N), corners])
    us = oracle.rhs_sampled(g, x, B0, nodes, gamma=0.7)
    assert np.abs(u).max() > 0.0
    assert nrel(us, u[:, nodes].T) < 1e-14


# --------------------------------------------------------------------------------------
# Diagnostics: closed forms for E_M; xi and R2 from a library curl on the undistorted grid
# --------------------------------------------------------------------------------------
@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 1, 1)])
def test_energy_uniform_field_exact(bc):
    g = W.make_grid((7, 8, 9), [(-1.0, 1.0), (0.0, 3.0), (-2.0, 2.0)], bc)
    b = np.array([0.3, -0.4, 1.2])
    d = oracle.diagnostics(g, g.identity(), W.uniform_field(g, b))
    V = np.prod(g.lengths())
    assert d["E_M"] == pytest.approx(0.5 * (b @ b) * V, rel=1e-14)


def test_energy_linear_map_exact():
    g = W.make_grid((7, 8, 9), [(-1.0, 1.0), (0.0, 3.0), (-2.0, 2.0)], (0, 0, 0))
    A = np.array([[1.1, 0.2, -0.1], [0.05, 0.9, 0.3], [-0.2, 0.1, 1.3]])
    b = np.array([0.3, -0.4, 1.2])
    d = oracle.diagnostics(g, _affine(g, A, [0.5, 0.5, 0.5]), W.uniform_field(g, b))
    V = np.prod(g.lengths())
    Ab = A @ b
    assert d["E_M"] == pytest.approx(0.5 * (Ab @ Ab) * V / np.linalg.det(A), rel=1e-13)
    assert d["min_det"] == pytest.approx(np.linalg.det(A), rel=1e-13)


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0)])
def test_xi_and_R2_on_undistorted_grid(bc):
    g = W.make_grid((9, 8, 10), [(-1.0, 1.0), (-1.0, 1.0), (-1.0, 1.0)], bc)
    B0 = W.smooth_random_field(g, 0.5, seed=41) + np.array([0, 0, 1.0])[:, None, None, None]
    d = oracle.diagnostics(g, g.identity(), B0)
    s = interior(g)
    J = central_curl(g, B0)[(slice(None),) + s]
    Bi = B0[(slice(None),) + s]
    f = np.cross(J, Bi, axis=0)
    f2 = (f ** 2).sum(axis=0)
    dV = np.prod(g.h)
    assert d["R2"] == pytest.approx(0.5 * f2.sum() * dV, rel=1e-12)
    assert d["xi"] == pytest.approx(np.sqrt(f2 / (Bi ** 2).sum(axis=0) ** 2).max(), rel=1e-12)


def test_xi_null_guard_counts_skipped_nodes():
    g = W.make_grid((8, 8, 8), [(0, 2 * math.pi)] * 3, (1, 1, 1))
    B0 = W.abc_field(g)
    # ABC has a null at X=Y=Z=3 pi / 4, which is node index 3 on an 8-point periodic axis
    assert np.abs(B0[:, 3, 3, 3]).max() < 1e-15
    d = oracle.diagnostics(g, g.identity(), B0, tau_B2=oracle.null_threshold(B0))
    assert d["skipped"] >= 1


# --------------------------------------------------------------------------------------
# Failure paths (status codes)
# --------------------------------------------------------------------------------------
def test_error_codes():
    w = W.single_twist_16()
    g = w.grid
    x = w.x0.copy()
    x[0, 8, 8, 8] -= 3 * g.h[0]  # push a node past its second neighbour -> Delta < 0 next to it
    r = oracle.run(g, x, w.B0, 3, dt=1e-3, raise_on_error=False)
    assert r["status"] == oracle.E_FOLD and r["done"] == 0
    B = w.B0.copy()
    B[1, 5, 5, 5] = np.nan
    r = oracle.run(g, w.x0, B, 3, dt=1e-3, raise_on_error=False)
    assert r["status"] == oracle.E_NAN
    r = oracle.run(g, w.x0, w.B0, 3, dt=1e-3, tol=1e-300, dt_min=1e-4, raise_on_error=False)
    assert r["status"] == oracle.E_DT
    bad = W.Grid((2, 16, 16), g.h, g.bc)
    with pytest.raises(oracle.OracleError) as e:
        oracle.fields(bad, np.zeros((3, 16, 16, 2)), np.zeros((3, 16, 16, 2)))
    assert e.value.code == oracle.E_ARG


# --------------------------------------------------------------------------------------
# Complex-step reference derivative of the fixed-dt trajectory (pins for the gradient oracle)
# --------------------------------------------------------------------------------------
def _small_case():
    g = W.make_grid((8, 8, 8), [(-1.0, 1.0)] * 3, (1, 1, 0))
    x0 = W.distorted_grid(g, 0.05, seed=51)
    B0 = W.smooth_random_field(g, 0.4, seed=52) + np.array([0, 0, 1.0])[:, None, None, None]
    return g, x0, B0


def test_complex_step_homogeneity_at_K0():
    g, x0, B0 = _small_case()
    eps = 1e-30
    E, _ = oracle.run_fixed_complex(g, x0, B0 + 1j * eps * B0, [])
    E_real = oracle.diagnostics(g, x0, B0)["E_M"]
    assert E.real == pytest.approx(E_real, rel=1e-14)
    assert E.imag / eps == pytest.approx(2 * E_real, rel=1e-13)


def test_complex_step_translation_invariance():
    g, x0, B0 = _small_case()
    eps = 1e-30
    v = np.zeros_like(x0)
    v[0] = 1.0
    v[2] = -0.5
    E, R = oracle.run_fixed_complex(g, x0 + 1j * eps * v, B0, [2e-3] * 3)
    assert abs(E.imag / eps) < 1e-12 * abs(E.real)
    assert abs(R.imag / eps) < 1e-10 * abs(R.real)


def test_complex_step_matches_central_difference():
    g, x0, B0 = _small_case()
    rng = np.random.default_rng(53)
    vx, vb = rng.standard_normal(x0.shape), rng.standard_normal(B0.shape)
    dts = [2e-3] * 3
    eps = 1e-30
    E, R = oracle.run_fixed_complex(g, x0 + 1j * eps * vx, B0 + 1j * eps * vb, dts)
    E_real = oracle.run(g, x0, B0, 3, dt=2e-3, mode=oracle.MODE_FIXED)
    h = 1e-6

    def energy(s):
        r = oracle.run(g, x0 + s * vx, B0 + s * vb, 3, dt=2e-3, mode=oracle.MODE_FIXED)
        return oracle.diagnostics(g, r["x"], B0 + s * vb)["E_M"]
    fd = (energy(h) - energy(-h)) / (2 * h)
    assert E.real == pytest.approx(oracle.diagnostics(g, E_real["x"], B0)["E_M"], rel=1e-13)
    assert E.imag / eps == pytest.approx(fd, rel=1e-7)


# --------------------------------------------------------------------------------------
# T16: the next-nearest-neighbour (octilateral) current of Sec. 2.3
# --------------------------------------------------------------------------------------
def smoothed_central_curl(g, B):
    """The curl that the octilateral loops reduce to on the undistorted grid: each derivative
    is the central difference along its axis averaged over the three lines of the loop's
    plane with weights 1/4, 1/2, 1/4 (the trapezoid rule along the edges of the 2h x 2h
    square through the eight ring neighbours).  numpy.roll throughout; valid on interior
    nodes."""
    def roll(f, a, s):
        return np.roll(f, s, axis=2 - a)

    def D(f, a, b):  # d/dX_a, smoothed along axis b
        sm = 0.25 * roll(f, b, 1) + 0.5 * f + 0.25 * roll(f, b, -1)
        return (roll(sm, a, -1) - roll(sm, a, 1)) / (2 * g.h[a])
    Bx, By, Bz = B
    return np.stack([D(Bz, 1, 2) - D(By, 2, 1), D(Bx, 2, 0) - D(Bz, 0, 2), D(By, 0, 1) - D(Bx, 1, 0)])


@pytest.mark.parametrize("bc", [(0, 0, 0), (1, 1, 0), (1, 0, 1), (1, 1, 1)])
def test_T16_octilateral_undistorted_grid_gives_smoothed_central_curl(bc):
    g = W.make_grid((9, 10, 11), [(-1.0, 1.4), (0.0, 2.25), (-2.0, 0.0)], bc)
    B0 = W.smooth_random_field(g, 1.0, seed=11, mmax=3) + np.random.default_rng(3).normal(size=g.shape) * 0.3
    with oracle.curl(oracle.CURL_NNN):
        f = oracle.fields(g, g.identity(), B0)
    s = (slice(None),) + interior(g)
    assert nrel(f["J"][s], smoothed_central_curl(g, B0)[s]) < 1e-13
    # and it is not the nearest-neighbour operator
    assert nrel(f["J"][s], central_curl(g, B0)[s]) > 1e-3


def _field_for_target(g, x, Bt):
    """B0 whose pull-back on positions x is Bt: the oracle's own F columns from three uniform
    fields (B = F e_a / det F), then B0 = det F F^-1 Bt node by node."""
    cols = []
    for a in range(3):
        e = np.zeros(g.shape)
        e[a] = 1.0
        f = oracle.fields(g, x, e)
        cols.append(f["B"] * f["det"])
    F = np.stack(cols, axis=1)  # (3 rows, 3 cols, nz, ny, nx)
    det = f["det"]
    Fm = np.moveaxis(F, (0, 1), (-2, -1))
    return np.moveaxis(np.linalg.solve(Fm, np.moveaxis(Bt, 0, -1)[..., None])[..., 0], -1, 0) * det


@pytest.mark.parametrize("curl_kind", [0, 1])
def test_T16_linear_field_on_distorted_grid_exact_curl(curl_kind):
    """A field linear in x, B = M x + c, on a non-affine, smoothly distorted grid (loops that
    are neither planar nor regular): the trapezoid circulation of a linear field along straight
    edges is exact, and Stokes holds exactly for its constant curl over any closed polygon, so J
    is the exact curl at every interior node if and only if the area vector is the loop's
    vector area.  For the octilateral that pins the circulation, the eight surface elements
    (the reading of dx_A..dx_D) and the solve; for the nearest-neighbour loops, the same."""
    rng = np.random.default_rng(31)
    M = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    g = W.make_grid((9, 8, 10), [(-1.0, 1.0), (-0.8, 0.9), (-1.2, 1.0)], (0, 0, 0))
    x = g.identity() + W.wall_sine_displacement(g, 0.06, seed=4, lo=-1.2, hi=1.2)
    Bt = np.einsum("ij,j...->i...", M, x) + c[:, None, None, None]
    B0 = _field_for_target(g, x, Bt)
    with oracle.curl(curl_kind):
        f = oracle.fields(g, x, B0)
    assert nrel(f["B"], Bt) < 1e-13
    curl = np.array([M[2, 1] - M[1, 2], M[0, 2] - M[2, 0], M[1, 0] - M[0, 1]])
    Ji = f["J"][(slice(None),) + interior(g)].reshape(3, -1)
    assert np.abs(Ji - curl[:, None]).max() < 1e-11 * np.abs(curl).max()


def test_T16_octilateral_second_order_and_close_to_nearest_neighbour():
    """On a smooth field and a smooth distortion both operators approximate the curl to second
    order: halving h cuts the octilateral's difference from the nearest-neighbour current by
    about four."""
    diffs = []
    for n in (12, 24):
        g = W.make_grid((n, n, n), [(0.0, 2 * np.pi)] * 3, (1, 1, 1))
        x0 = g.identity() + 0.05 * np.stack([np.sin(g.coords()[1]), np.sin(g.coords()[2]), np.sin(g.coords()[0])])
        B0 = W.abc_field(g)
        a = oracle.fields(g, x0, B0)["J"]
        with oracle.curl(oracle.CURL_NNN):
            b = oracle.fields(g, x0, B0)["J"]
        diffs.append(nrel(b, a))
    assert 3.0 < diffs[0] / diffs[1] < 5.0, diffs


def test_T16_octilateral_rigid_rotation_and_translation():
    """Rotating the positions and B0's image rigidly rotates J (the loops are built from
    differences of positions only)."""
    g = W.make_grid((8, 9, 7), [(-1.0, 1.0), (-1.0, 1.2), (-0.7, 0.9)], (0, 0, 0))
    x = g.identity() + W.wall_sine_displacement(g, 0.05, seed=8, lo=-1.0, hi=1.2)
    B0 = W.smooth_random_field(g, 1.0, seed=9)
    th = 0.7
    Q = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    with oracle.curl(oracle.CURL_NNN):
        f = oracle.fields(g, x, B0)
        xr = np.einsum("ij,j...->i...", Q, x) + np.array([0.3, -1.0, 2.0])[:, None, None, None]
        fr = oracle.fields(g, xr, B0)
    assert nrel(fr["J"], np.einsum("ij,j...->i...", Q, f["J"])) < 1e-12
    assert nrel(fr["B"], np.einsum("ij,j...->i...", Q, f["B"])) < 1e-13
