"""Pins of the three-dimensional FP64 oracle (D3Q19 lattice with spheres, oracle3d.c) against what
the paper and the mathematics fix (no GPU): the defining moments of the equilibrium, the
collision's conservation laws, the special cases eps = 0 and eps = 1, the paper's sub-cell solid
ratio against an independent count and the sphere volume, plane Poiseuille flow, and an exact
reduction: a lattice one cell deep in z, summed over the z-components of the velocities, evolves
as the (separately pinned) two-dimensional D2Q9 oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleConfig, OracleConfig3, OracleSim, OracleSim3
from paper_1809_07008_amd import workloads as W

E3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
W3 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
OPP3 = np.array([0] + [i + 1 if i % 2 else i - 1 for i in range(1, 19)])
CX2 = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY2 = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def rand_cell3(rng, amp=0.2):
    return W3 * (1.0 + amp * rng.uniform(-1, 1, 19))


def moments3(f):
    f = np.asarray(f)
    return f.sum(), E3.T @ f


def second3(f):
    return np.einsum("ia,ib,i->ab", E3, E3, np.asarray(f))


def relax3(f):
    """f^eq(rho, u) of the oracle without retyping Eq. (2): tau = 1, nothing else."""
    return oracle.collide_cell3(f, tau=1.0)[0]


def test_lattice_table_is_the_paper_d3q19():
    """Table 1: one rest velocity, six axis and twelve diagonal velocities; every direction has
    its opposite; the weights make the lattice isotropic to fourth order (the equilibrium's
    moments below depend on it)."""
    assert len({tuple(c) for c in E3}) == 19
    assert np.all(E3[OPP3] == -E3)
    assert abs(W3.sum() - 1) < 1e-15
    assert np.allclose(np.einsum("i,ia,ib->ab", W3, E3, E3), np.eye(3) / 3, atol=1e-16)


def test_equilibrium3_has_the_defining_moments():
    """Eq. (2): sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho (I/3 + u u) at random
    (rho, u), with rho and u taken from the input by plain sums."""
    rng = np.random.default_rng(41)
    for _ in range(100):
        f = rand_cell3(rng)
        f = f * (1.0 + 0.05 * (E3 @ rng.normal(size=3)))
        rho, m = moments3(f)
        u = m / rho
        feq = relax3(f)
        r2, m2 = moments3(feq)
        tol = 32 * np.finfo(float).eps
        assert abs(r2 - rho) <= tol
        assert np.abs(m2 - rho * u).max() <= tol
        assert np.abs(second3(feq) - rho * (np.eye(3) / 3 + np.outer(u, u))).max() <= tol
        assert np.abs(u).max() > 1e-3


def test_collision3_mass_and_momentum_balance():
    """Eqs. (12)-(16) with two spheres and a body force: mass is kept; the momentum changes by
    (1 - B_tot) rho g + sum_p B_p (rho u_s,p - m), and each sphere receives B_p (m - rho u_s,p);
    the torque is d x dF."""
    rng = np.random.default_rng(42)
    for _ in range(40):
        f = rand_cell3(rng)
        eps = rng.uniform(0.05, 0.6, 2)
        d = rng.uniform(-4, 4, (2, 3))
        v = rng.normal(0, 0.02, (2, 3))
        w = rng.normal(0, 0.004, (2, 3))
        g = rng.normal(0, 1e-4, 3)
        fo, dF, dT, Bt = oracle.collide_cell3(f, eps, d, v, w, tau=0.7, g=g)
        rho, m = moments3(f)
        r2, m2 = moments3(fo)
        assert abs(r2 - rho) <= 16 * np.finfo(float).eps
        S = eps.sum()
        expect = (1 - Bt) * rho * g
        for p in range(2):
            us = v[p] + np.cross(w[p], d[p])
            Bp = Bt * eps[p] / S
            expect = expect + Bp * (rho * us - m)
            assert np.abs(dF[p] - Bp * (m - rho * us)).max() < 1e-15
            assert np.abs(dT[p] - np.cross(d[p], dF[p])).max() < 1e-15
        assert np.abs((m2 - m) - expect).max() < 1e-15


def test_collision3_weight_at_hand_worked_points():
    """B of Eq. (14) in the 3D collision at the hand-worked interior points of
    tests/golden/weight_eq14.txt (one sphere covering the cell with eps)."""
    import os
    from fractions import Fraction
    path = os.path.join(os.path.dirname(__file__), "golden", "weight_eq14.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 6
    f = W3 * 1.01
    for e, t, num, den in rows:
        B = float(Fraction(int(num), int(den)))
        Bt = oracle.collide_cell3(f, [float(e)], [[0.1, 0.2, 0.3]], [[0, 0, 0]], [[0, 0, 0]],
                                  tau=float(t))[3]
        assert abs(Bt - B) <= 4 * np.finfo(float).eps * B


def test_collision3_eps_zero_and_eps_one():
    """eps = 0 leaves the BGK collision bit for bit; eps = 1 with a resting solid removes the
    momentum and mirrors a rest state exactly (bounce-back)."""
    rng = np.random.default_rng(43)
    f = rand_cell3(rng)
    ref = oracle.collide_cell3(f, tau=0.8, g=(1e-5, 0, -2e-6))
    got = oracle.collide_cell3(f, [0.0], [[1.0, 2.0, -0.5]], [[0.01, 0, 0]], [[0, 0.001, 0]],
                               tau=0.8, g=(1e-5, 0, -2e-6))
    assert np.array_equal(ref[0], got[0]) and np.all(got[1] == 0)
    for _ in range(10):
        f = rand_cell3(rng)
        fo, dF, dT, Bt = oracle.collide_cell3(f, [1.0], [[0.3, 0.1, -0.2]], [[0, 0, 0]],
                                              [[0, 0, 0]], tau=0.6, g=(1e-4, 0, 0))
        assert Bt == 1.0
        assert np.abs(moments3(fo)[1]).max() < 1e-16
    frest = 1.03 * W3
    fo = oracle.collide_cell3(frest, [1.0], [[0.0, 0.0, 0.0]], [[0, 0, 0]], [[0, 0, 0]], tau=0.9)[0]
    assert np.array_equal(fo, frest[OPP3])


# ---- the paper's cell-decomposition solid ratio (Sec. 2.2) in 3D

def test_subcell3_one_point_and_full_empty_cells():
    rng = np.random.default_rng(44)
    for _ in range(2000):
        r = rng.uniform(0.3, 5.0)
        d = rng.uniform(-6, 6, 3)
        assert oracle.subcell_fraction3(r, *d, 1) == (1.0 if d @ d < r * r else 0.0)
    assert oracle.subcell_fraction3(2.0, 0.0, 2.0, 0.0, 1) == 0.0  # on the surface: outside
    for _ in range(500):
        r = rng.uniform(1.0, 6.0)
        d = rng.uniform(-r - 1, r + 1, 3)
        near = np.where(d - 0.5 > 0, d - 0.5, np.where(d + 0.5 < 0, d + 0.5, 0.0))
        far = np.abs(d) + 0.5
        e = oracle.subcell_fraction3(r, *d, 5)
        if near @ near >= r * r:
            assert e == 0.0
        if far @ far < r * r:
            assert e == 1.0


@pytest.mark.parametrize("n", [2, 5, 6])
def test_subcell3_symmetries(n):
    """Sub-cell centres sit symmetrically in the cell: reflections and axis permutations of the
    cell about the sphere centre leave the count unchanged."""
    rng = np.random.default_rng(45 + n)
    cut = 0
    for _ in range(400):
        r = rng.uniform(0.7, 4.0)
        d = rng.uniform(-r - 1, r + 1, 3)
        e = oracle.subcell_fraction3(r, *d, n)
        cut += 0 < e < 1
        for dd in ((-d[0], d[1], d[2]), (d[0], -d[1], d[2]), (d[0], d[1], -d[2]),
                   (d[1], d[0], d[2]), (d[2], d[1], d[0])):
            assert oracle.subcell_fraction3(r, *dd, n) == e
    assert cut > 50


@pytest.mark.parametrize("n", [1, 3, 5])
def test_subcell3_counts_agree_with_row_interval_counts(n):
    """Independent count: in the sub-row (j, k) the inside centres are those with |x_c| < s,
    s = sqrt(r^2 - y_c^2 - z_c^2), an open interval of the progression dx - 1/2 + (i + 1/2)/n."""
    rng = np.random.default_rng(46 + n)
    for _ in range(300):
        r = rng.uniform(0.4, 4.0)
        dx, dy, dz = rng.uniform(-r - 1, r + 1, 3)
        cnt = 0
        for k in range(n):
            zc = dz - 0.5 + (k + 0.5) / n
            for j in range(n):
                yc = dy - 0.5 + (j + 0.5) / n
                q = r * r - yc * yc - zc * zc
                if q <= 0:
                    continue
                s = math.sqrt(q)
                lo = (-s - dx + 0.5) * n - 0.5
                hi = (s - dx + 0.5) * n - 0.5
                i0, i1 = max(0, math.floor(lo) + 1), min(n - 1, math.ceil(hi) - 1)
                cnt += max(0, i1 - i0 + 1)
        assert oracle.subcell_fraction3(r, dx, dy, dz, n) * n ** 3 == pytest.approx(cnt, abs=1e-9)


@pytest.mark.parametrize("n", [2, 5, 10])
def test_subcell3_total_within_lattice_point_bound(n):
    """All sub-cell centres of a sphere's cells form one cubic grid of spacing h = 1/n: the cubes
    of side h around the inside centres lie in the ball of radius r + sqrt3 h/2 and cover the
    ball of radius r - sqrt3 h/2, so |sum eps - 4/3 pi r^3| <= 4/3 pi ((r + sqrt3/(2n))^3 - r^3)."""
    rng = np.random.default_rng(47 + n)
    for _ in range(3):
        r = rng.uniform(1.5, 5.0)
        c = rng.uniform(0, 1, 3)
        R = int(r) + 2
        idx = np.arange(-R, R + 1)
        tot = sum(oracle.subcell_fraction3(r, i - c[0], j - c[1], k - c[2], n)
                  for i in idx for j in idx for k in idx)
        bound = 4 / 3 * math.pi * ((r + math.sqrt(3) / (2 * n)) ** 3 - r ** 3)
        assert abs(tot - 4 / 3 * math.pi * r ** 3) <= bound


# ---- whole steps

def d2q9_index(cx, cy):
    for i in range(9):
        if CX2[i] == cx and CY2[i] == cy:
            return i
    raise ValueError


def test_one_cell_deep_lattice_reduces_to_the_d2q9_oracle():
    """A D3Q19 lattice one cell deep in z (periodic z) with populations split symmetrically in
    +-z evolves, summed over the z-components of the velocities, exactly as the D2Q9 oracle:
    the summed weights are 4/9, 1/9, 1/36, the summed equilibrium is the D2Q9 one when u_z = 0,
    forcing and half-way bounce-back project likewise.  Pins the 3D collision, forcing,
    streaming and wall rule against the separately pinned 2D oracle (to rounding)."""
    rng = np.random.default_rng(48)
    nx, ny = 23, 14
    f2 = W.random_populations(rng, nx, ny, amplitude=0.05)
    # split every D2Q9 population over its D3Q19 preimages in proportion to their weights
    pre = [[] for _ in range(9)]
    for i in range(19):
        pre[d2q9_index(E3[i, 0], E3[i, 1])].append(i)
    f3 = np.zeros((19, 1, ny, nx))
    for j in range(9):
        ws = W3[pre[j]]
        for i, wi in zip(pre[j], ws):
            f3[i, 0] = f2[j] * (wi / ws.sum())
    for walls in (True, False):
        a = OracleSim(OracleConfig(nx=nx, ny=ny, tau0=0.73, walls=walls, gx=2e-5, gy=-1e-5))
        a.set_populations(f2)
        b = OracleSim3(OracleConfig3(nx=nx, ny=ny, nz=1, tau0=0.73, walls=walls, gx=2e-5,
                                     gy=-1e-5))
        b.set_populations(f3)
        a.step(25)
        b.step(25)
        fa, fb = a.populations(), b.populations()
        proj = np.zeros_like(fa)
        for j in range(9):
            proj[j] = fb[pre[j], 0].sum(axis=0)
        assert np.abs(proj - fa).max() < 1e-15
        _, _, uyb, uzb = b.fields()
        assert np.abs(uzb).max() < 1e-17


@pytest.mark.parametrize("ny,tau", [(8, 0.6), (9, 1.0), (16, 0.8)])
def test_plane_poiseuille3_closed_form(ny, tau):
    """Steady flow between half-way bounce-back walls driven by g along x: the same exact discrete
    profile as for D2Q9, m(y) = g/(2 nu) [(ny/2)^2 - (y - yc)^2] + g (16 L - 3)/(24 nu) - g/2,
    nu = (tau - 1/2)/3, L = (tau - 1/2)^2; uniform in x and z."""
    g = 1e-5
    s = OracleSim3(OracleConfig3(nx=2, ny=ny, nz=2, tau0=tau, gx=g))
    nu = (tau - 0.5) / 3
    L = (tau - 0.5) ** 2
    s.step(int(60 * ny * ny / (nu * math.pi ** 2)))
    rho, ux, uy, uz = s.fields()
    y = np.arange(ny)
    yc = (ny - 1) / 2
    m_th = g / (2 * nu) * ((ny / 2) ** 2 - (y - yc) ** 2) + g * (16 * L - 3) / (24 * nu) - g / 2
    assert np.abs(rho * ux - m_th[None, :, None]).max() < 1e-10 * m_th.max()
    assert np.abs(uy).max() < 1e-10 * m_th.max() and np.abs(uz).max() < 1e-10 * m_th.max()


def test_momentum_balance3_periodic_box_with_spheres():
    """Fully periodic box, body force, a fixed and a prescribed sphere: the fluid's momentum
    changes by the unsolid part of the forcing minus the forces on the spheres, every step."""
    rng = np.random.default_rng(49)
    nx, ny, nz = 20, 18, 16
    g = np.array([2e-5, -1e-5, 5e-6])
    s = OracleSim3(OracleConfig3(nx=nx, ny=ny, nz=nz, tau0=0.75, walls=False, gx=g[0], gy=g[1],
                                 gz=g[2], eps_subcells=4))
    f = W3[:, None, None, None] * (1 + 0.02 * rng.uniform(-1, 1, (19, nz, ny, nx)))
    s.set_populations(f)
    s.set_spheres([5.3, 13.7], [6.1, 11.8], [4.4, 10.2], [3.2, 2.6],
                  v=[[0, 0, 0], [0.01, -0.005, 0.002]], w=[[0, 0.002, 0], [0.001, 0, -0.003]],
                  mode=[1, 2])
    for _ in range(4):
        f0 = s.populations()
        rho0 = f0.sum(axis=0)
        eps = s.solid_field()
        B = np.minimum(eps, 1.0) * 0.25 / ((1 - np.minimum(eps, 1.0)) + 0.25)
        m0 = np.einsum("ia,izyx->a", E3, f0)
        s.step(1)
        m1 = np.einsum("ia,izyx->a", E3, s.populations())
        F, T = s.forces()
        expect = ((1 - B) * rho0).sum() * g - F.sum(axis=0)
        # the totals are sums of 19 x 5760 terms: their rounding scale
        scale = np.einsum("ia,izyx->a", np.abs(E3), f0).max()
        assert np.abs((m1 - m0) - expect).max() < 64 * np.finfo(float).eps * scale
        assert np.abs(F).max() > 1e-6


def test_co_moving_sphere_feels_no_force():
    U = np.array([0.02, -0.01, 0.015])
    s = OracleSim3(OracleConfig3(nx=24, ny=22, nz=20, tau0=0.65, walls=False))
    s.init_equilibrium(1.0, *U)
    s.set_spheres([9.3], [10.6], [8.1], [4.2], v=[U], mode=[2])
    f0 = s.populations()
    for _ in range(8):
        s.step(1)
        F, T = s.forces()
        # against the momentum a resting sphere would take per step, volume x rho |U|
        ref = 4 / 3 * math.pi * 4.2 ** 3 * np.linalg.norm(U)
        assert np.abs(F).max() < 1e-13 * ref and np.abs(T).max() < 1e-13 * 4.2 * ref
    assert np.abs(s.populations() - f0).max() < 1e-15


def test_drag_sign_and_mirror_symmetry3():
    """A fixed sphere centred between the walls and on a z-mirror plane of a periodic channel is
    pushed downstream; by symmetry it feels no lift, no side force and no torque."""
    ny, nz = 21, 20
    s = OracleSim3(OracleConfig3(nx=24, ny=ny, nz=nz, tau0=0.8, gx=1e-5))
    s.set_spheres([10.25], [(ny - 1) / 2], [(nz - 1) / 2], [4.3])
    s.step(150)
    F, T = s.forces()
    assert F[0, 0] > 0
    assert abs(F[0, 1]) < 1e-10 * F[0, 0] and abs(F[0, 2]) < 1e-10 * F[0, 0]
    assert np.abs(T[0]).max() < 1e-9 * F[0, 0]
