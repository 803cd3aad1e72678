"""Pins of the D3Q19 oracle (Sec. IV.D: the method in three dimensions).

As for the two-dimensional oracle, none of these re-types the oracle's
formulas: each compares it with a closed form, an exact invariant or a
reduction to a case whose solution is known.
"""
import numpy as np
import pytest

# The D3Q19 set written out independently here: rest, axis directions, edges.
E = np.array([(0, 0, 0)] + [(s * (d == 0), s * (d == 1), s * (d == 2)) for d in range(3) for s in (1, -1)]
             + [tuple(v) for v in ((1, 1, 0), (1, -1, 0), (-1, 1, 0), (-1, -1, 0), (1, 0, 1), (1, 0, -1),
                                   (-1, 0, 1), (-1, 0, -1), (0, 1, 1), (0, 1, -1), (0, -1, 1), (0, -1, -1))])
WT = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}  # by |e|^2


def _lookup(oracle_mod):
    """Map the oracle's velocity order onto the set above (the oracle must use
    the same nineteen vectors, in any order)."""
    order = [int(np.nonzero((E == np.array(v)).all(axis=1))[0][0]) for v in oracle_mod.E3]
    assert sorted(order) == list(range(19))
    return np.array(oracle_mod.E3), np.array([WT[int(np.dot(v, v))] for v in oracle_mod.E3])


def test_equilibrium_moments_3d(oracle_mod):
    """Eq. 8 on D3Q19: mass, momentum and the Euler stress rho/3 I + rho u u."""
    e, w = _lookup(oracle_mod)
    rng = np.random.default_rng(11)
    for _ in range(40):
        rho = rng.uniform(0.5, 1.5)
        u = rng.uniform(-0.15, 0.15, 3)
        f = oracle_mod.feq3(rho, u)
        assert abs(f.sum() - rho) <= 4e-15
        assert np.abs(e.T @ f - rho * u).max() <= 4e-15
        P = (e[:, :, None] * e[:, None, :] * f[:, None, None]).sum(0)
        assert np.abs(P - (rho / 3 * np.eye(3) + rho * np.outer(u, u))).max() <= 4e-15


def test_collision_conserves_mass_adds_momentum_3d(oracle_mod):
    """BGK + Guo: mass is conserved and the momentum gains exactly rho g."""
    e, _ = _lookup(oracle_mod)
    rng = np.random.default_rng(12)
    for tau in (0.55, 0.8, 1.7):
        f = oracle_mod.feq3(1.02, (0.03, -0.02, 0.01)) + rng.normal(0, 1e-3, 19)
        g = rng.normal(0, 1e-4, 3)
        out = oracle_mod.collide_node3(f, tau, g)
        assert abs(out.sum() - f.sum()) <= 1e-15
        assert np.abs(e.T @ out - (e.T @ f + f.sum() * g)).max() <= 1e-16


def test_link_force_closed_forms_3d(oracle_mod):
    """Eq. 9 on every D3Q19 link for a surface moving along x at U, with the
    equilibrium population a = f_eq,i(rho, v) and the bounced b: the GME
    x-force is the rest value 2 w_i rho e_ix, the CME one is (1 + 3U^2) times
    it (links with e_ix != 0); at rest both equal 2 w_i rho e_i."""
    e, w = _lookup(oracle_mod)
    rho, U = 1.03, 0.07
    for v in ((U, 0.0, 0.0), (0.0, 0.0, 0.0)):
        fe = oracle_mod.feq3(rho, v)
        for i in range(1, 19):
            a = fe[i]
            b = a - 6 * w[i] * rho * np.dot(e[i], v)
            gme = oracle_mod.link_force3(i, a, b, v, oracle_mod.GME)
            cme = oracle_mod.link_force3(i, a, b, v, oracle_mod.CME)
            if v[0] == 0.0:
                assert np.abs(gme - 2 * w[i] * rho * e[i]).max() <= 1e-16
                assert np.abs(cme - gme).max() == 0.0
            elif e[i, 0] != 0:
                assert abs(gme[0] - 2 * w[i] * rho * e[i, 0]) <= 1e-16
                assert abs(cme[0] - 2 * w[i] * rho * e[i, 0] * (1 + 3 * U * U)) <= 1e-16


@pytest.mark.parametrize("tau,steps", [(0.6, 40000), (1.0, 14000)])
def test_planes_poiseuille_exact_3d(oracle_mod, tau, steps):
    """Between the solid planes z = 0 and z = nz - 1 a y-invariant flow is the
    D2Q9 problem (summing D3Q19 over e_y gives D2Q9's weights and
    equilibrium), so the exact discrete Poiseuille solution of half-way
    bounce-back with Guo forcing holds: u(z) = g/(2nu)(Z^2 - (z - z_c)^2) + s,
    s = g [4(2tau-1)^2 - 3] / (4(2tau-1)), Z = (nz - 2)/2, z_c = (nz - 1)/2.
    The planes carry the body force, and no lateral flow appears."""
    nz, g = 14, 1e-5
    s = oracle_mod.OracleSim3D(2, 3, nz, tau, g=(g, 0.0, 0.0), duct=oracle_mod.PLANES3)
    s.step(steps)
    rho, u, own = s.fields()
    nu = (tau - 0.5) / 3
    z = np.arange(nz)
    slip = g * (4 * (2 * tau - 1) ** 2 - 3) / (4 * (2 * tau - 1))
    exact = g / (2 * nu) * (((nz - 2) / 2) ** 2 - (z - (nz - 1) / 2) ** 2) + slip
    fl = own[:, 0, 0] == 0
    assert np.abs(u[0][:, 1, 1] - exact)[fl].max() / exact.max() <= 1e-10
    assert np.abs(u[1:]).max() <= 1e-11 * exact.max()  # rounding only
    F = s.force(0, oracle_mod.CME)
    assert abs(F[0] - g * rho.sum()) <= 1e-9 * g * rho.sum()


def test_comoving_sphere_uniform_flow_3d(oracle_mod):
    """A sphere whose surface moves with the uniform flow f_eq(1, U) leaves
    the state exactly unchanged and feels no force (fixed geometry)."""
    U = np.array([0.04, -0.015, 0.02])
    sp = dict(cx=9.3, cy=8.6, cz=7.8, r=4.2, v=tuple(U))
    s = oracle_mod.OracleSim3D(20, 18, 16, 0.7, u0=tuple(U), spheres=[sp])
    fe = oracle_mod.feq3(1.0, U)
    s.step(15)
    f = s.get_f()
    _, _, own = s.fields()
    assert np.abs(f[:, own == 0] - fe[:, None]).max() <= 1e-15
    for sch in (oracle_mod.CME, oracle_mod.GME):
        assert np.abs(s.force(1, sch)[:3]).max() <= 1e-13


def _momentum(f, e):
    return np.tensordot(e.T, f, axes=(1, 0)).reshape(3, -1).sum(1)


def test_momentum_balance_3d(oracle_mod):
    """Fixed geometry: P(t+1) - P(t) = g sum(rho) - sum_s F_CME,s every step
    (every bounce-back link removes exactly the conventional exchange), with a
    tube, a translating-surface and spinning sphere and a body force; mass is
    constant."""
    e, _ = _lookup(oracle_mod)
    g = np.array([3e-5, -1e-5, 2e-5])
    sp = dict(cx=8.4, cy=7.2, cz=7.9, r=3.1, v=(0.02, 0.01, -0.005), omega=(0.003, -0.002, 0.004))
    s = oracle_mod.OracleSim3D(18, 16, 16, 0.7, g=tuple(g), duct=oracle_mod.TUBE3, R=6.8, spheres=[sp])
    s.step(10)
    f = s.get_f()
    M0 = f.sum()
    for _ in range(12):
        P0 = _momentum(f, e)
        rho, _, _ = s.fields()
        s.step(1)
        f = s.get_f()
        expect = g * rho.sum() - s.force(0, oracle_mod.CME)[:3] - s.force(1, oracle_mod.CME)[:3]
        assert np.abs(_momentum(f, e) - P0 - expect).max() <= 1e-14 * M0
        assert abs(f.sum() - M0) <= 1e-13 * M0


def test_gme_equals_cme_at_rest_and_symmetry_3d(oracle_mod):
    """A sphere at rest on the axis of a tube Poiseuille flow: with no surface
    motion GME and CME coincide bit for bit, and the mirror symmetries of the
    geometry about the axis leave no lateral force and no torque."""
    ny = nz = 15
    sp = dict(cx=9.0, cy=(ny - 1) / 2, cz=(nz - 1) / 2, r=3.0)
    s = oracle_mod.OracleSim3D(20, ny, nz, 0.8, g=(2e-5, 0.0, 0.0), duct=oracle_mod.TUBE3, R=6.5, spheres=[sp])
    s.step(300)
    for k in (0, 1):
        c, g_ = s.force(k, oracle_mod.CME), s.force(k, oracle_mod.GME)
        assert np.array_equal(c, g_)
    F = s.force(1, oracle_mod.CME)
    assert F[0] > 0
    # rounding of sums over a few hundred links of size ~rho w_i
    assert np.abs(F[1:3]).max() <= 1e-12 * F[0]
    assert np.abs(F[3:]).max() <= 1e-12 * F[0]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_spinning_sphere_torque_opposes_spin_3d(oracle_mod, axis):
    """A sphere spinning about a lattice axis in fluid at rest: the fluid
    resists, T . Omega < 0, the torque lies along the spin axis, and by the
    cubic symmetry of lattice and sphere its magnitude is the same about every
    axis; no net force."""
    om = np.zeros(3)
    om[axis] = 0.004
    sp = dict(cx=10.0, cy=10.0, cz=10.0, r=4.0, omega=tuple(om))
    s = oracle_mod.OracleSim3D(21, 21, 21, 0.8, spheres=[sp])
    s.step(40)
    ref = oracle_mod.OracleSim3D(21, 21, 21, 0.8, spheres=[dict(sp, omega=(0.0, 0.0, 0.004))])
    ref.step(40)
    for sch in (oracle_mod.CME, oracle_mod.GME):
        F = s.force(1, sch)
        assert np.dot(F[3:], om) < 0
        others = [F[3 + d] for d in range(3) if d != axis]
        assert abs(F[3 + axis]) > 1e3 * max(abs(o) for o in others)
        assert abs(F[3 + axis] - ref.force(1, sch)[5]) <= 1e-12 * abs(F[3 + axis])
        assert np.abs(F[:3]).max() <= 1e-14


# ---------------------------------------------------------------- translating spheres (Sec. IV.B in 3D)
def _poly_field(deg, rng, n=9):
    """Post-advection values f_j = polynomial of degree deg in (x, y, z)."""
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    fn = np.zeros((19, n, n, n))
    exact = np.zeros(19)
    c = n // 2
    for j in range(19):
        a = rng.normal(size=10)
        terms = [np.ones_like(x, dtype=float), x, y, z, x * x, y * y, z * z, x * y, y * z, x * z]
        p = sum(a[t] * terms[t] for t in range([1, 4, 10][deg]))
        fn[j] = p
        exact[j] = p[c, c, c]
    return fn, exact


@pytest.mark.parametrize("scheme,exact_deg,miss_deg", [(0, 2, None), (1, 1, 2), (2, 1, 2)])
def test_refill_polynomial_exactness_3d(oracle_mod, scheme, exact_deg, miss_deg):
    """A1 reproduces quadratic fields along every link and A2 linear ones; A3
    copies the first neighbour, which with all 18 directions taking part is
    exact for linear fields too (the odd terms cancel in the average); A2 and
    A3 miss quadratic fields.  With participants on one side only, A3 misses a
    linear field."""
    rng = np.random.default_rng(21)
    n = 9
    own_t = np.zeros((n, n, n), np.uint8)
    own_t[4, 4, 4] = 1
    own_n = np.zeros((n, n, n), np.uint8)
    for deg in range(3):
        fn, exact = _poly_field(deg, rng)
        out, npart = oracle_mod.refill_node3(fn, own_t, own_n, 4, 4, 4, scheme)
        assert npart == 18
        err = np.abs(out - exact).max()
        if deg <= exact_deg:
            assert err <= 1e-12 * np.abs(fn).max()
        elif deg == miss_deg:
            assert err > 1e-3
    if scheme == 2:
        one_sided = own_t.copy()
        one_sided[:, :, :4] = 1  # every node with x < 4 solid at t
        fn, exact = _poly_field(1, rng)
        out, npart = oracle_mod.refill_node3(fn, one_sided, own_n, 4, 4, 4, scheme)
        assert npart == 13  # the directions with e_x = 1 (5) and e_x = 0 (8)
        assert np.abs(out - exact).max() > 1e-3


def test_refill_participants_and_fallback_3d(oracle_mod):
    """Participants are the directions whose first neighbour is old fluid;
    where the second or third neighbour is not, A1 falls back to A2 or A3
    (a linear field is still reproduced exactly, a quadratic one is not)."""
    n = 9
    rng = np.random.default_rng(22)
    own_t = np.zeros((n, n, n), np.uint8)
    own_t[4, 4, 4] = 1
    own_t[4, 4, 5] = 1          # +x neighbour solid at t: direction +x does not take part
    own_n = np.zeros((n, n, n), np.uint8)
    own_n[4, 4, 6] = 2          # x + 2 e_x... irrelevant (+x excluded); block -x at distance 3
    own_n[4, 4, 1] = 2          # -x: x - 3 e_x covered at t+1 -> A1 falls back to A2 along -x
    fn, exact = _poly_field(1, rng)
    out, npart = oracle_mod.refill_node3(fn, own_t, own_n, 4, 4, 4, 0)
    assert npart == 17
    assert np.abs(out - exact).max() <= 1e-12 * np.abs(fn).max()
    fn2, exact2 = _poly_field(2, rng)
    out2, _ = oracle_mod.refill_node3(fn2, own_t, own_n, 4, 4, 4, 0)
    assert np.abs(out2 - exact2).max() > 1e-6  # the -x direction used A2
    own_t[4, 4, 4] = 1
    own_t[:, :, :] = 1
    own_t[4, 4, 4] = 1
    _, npart = oracle_mod.refill_node3(fn, own_t, own_n, 4, 4, 4, 0)
    assert npart == 0


@pytest.mark.parametrize("refill", [0, 1, 2])
def test_translating_sphere_comoving_flow_3d(oracle_mod, refill):
    """A sphere translating with the uniform flow f_eq(1, U) across several
    nodes (covered and newborn nodes every few steps) leaves the state exactly
    uniform, with no force, for each refill scheme."""
    U = (0.05, -0.02, 0.03)
    sp = dict(cx=9.3, cy=8.6, cz=7.8, r=3.7, v=U)
    s = oracle_mod.OracleSim3D(22, 18, 16, 0.7, u0=U, spheres=[sp])
    s.set_moving(1, True, refill)
    fe = oracle_mod.feq3(1.0, U)
    _, _, own0 = s.fields()
    for _ in range(6):
        s.step(10)
        f = s.get_f()
        _, _, own = s.fields()
        assert np.abs(f[:, own == 0] - fe[:, None]).max() <= 1e-14  # rounding of f ~ 1/3
        assert np.abs(s.force(1, oracle_mod.GME)[:3]).max() <= 1e-13
    assert s.error == 0
    # the geometry of step 60 is the sphere centred at X0 + 60 U (raster
    # written out here: minimum image, |p - X|^2 <= r^2)
    nz, ny, nx = own.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    X = [sp["cx"] + 60 * U[0], sp["cy"] + 60 * U[1], sp["cz"] + 60 * U[2]]

    def mi(d, n):
        return d - n * np.floor(d / n + 0.5)

    dx, dy, dz = mi(x - X[0], nx), mi(y - X[1], ny), mi(z - X[2], nz)
    expect = (dx * dx + dy * dy) + dz * dz <= sp["r"] ** 2
    assert np.array_equal(own == 1, expect)


def test_translating_sphere_meets_tube_3d(oracle_mod):
    """A sphere driven into the tube wall is reported."""
    sp = dict(cx=10.0, cy=10.5, cz=10.5, r=3.0, v=(0.0, 0.2, 0.0))
    s = oracle_mod.OracleSim3D(20, 22, 22, 0.7, duct=oracle_mod.TUBE3, R=9.0, spheres=[sp])
    s.set_moving(1, True, 0)
    s.step(40)
    assert s.error != 0


# ---------------------------------------------------------------- free spheres
def _fluid_momentum3(s, e):
    return _momentum(s.get_f(), e)


def test_free_sphere_at_rest_3d(oracle_mod):
    """A heavy free sphere at rest in fluid at rest without gravity stays at
    rest: every link force cancels."""
    s = oracle_mod.OracleSim3D(20, 20, 20, 0.7, spheres=[dict(cx=9.7, cy=10.2, cz=9.4, r=4.1)])
    s.set_moving(1, True, 0)
    s.set_free(1, 1.5)
    s.step(30)
    st = s.body_state(1)
    assert np.abs(st[3:]).max() <= 1e-15
    assert np.abs(st[:3] - (9.7, 10.2, 9.4)).max() <= 1e-15


def test_free_sphere_momentum_balance_3d(oracle_mod):
    """Periodic box, a free sphere (density 1.5) under gravity G with the CME
    force: P_fluid(t) + M V(t) = P_fluid(0) + M V(0) + t (M - rho0 Vol) G
    while the sphere covers the same nodes."""
    e, _ = _lookup(oracle_mod)
    r, rho_s, G = 4.3, 1.5, np.array([2e-6, -1e-6, 1.5e-6])
    s = oracle_mod.OracleSim3D(22, 20, 18, 0.7, spheres=[dict(cx=10.3, cy=9.6, cz=8.7, r=r)])
    s.set_moving(1, True, 0)
    s.set_free(1, rho_s)
    s.set_gravity(G, oracle_mod.CME)
    vol = 4 / 3 * np.pi * r ** 3
    M = rho_s * vol
    P0 = _fluid_momentum3(s, e)
    _, _, own0 = s.fields()
    for t in (40, 80, 120):
        s.step(40)
        _, _, own = s.fields()
        assert np.array_equal(own, own0)
        st = s.body_state(1)
        bal = _fluid_momentum3(s, e) + M * st[3:6] - P0 - t * (M - vol) * G
        assert np.abs(bal).max() < 1e-12
        assert np.linalg.norm(st[3:6]) > 1e-6


def test_free_sphere_spin_down_3d(oracle_mod):
    """A free sphere spinning about a lattice axis in fluid at rest slows
    down: the spin decays monotonically, stays on its axis, and the centre
    does not move."""
    s = oracle_mod.OracleSim3D(21, 21, 21, 0.8, spheres=[dict(cx=10.0, cy=10.0, cz=10.0, r=4.0)])
    s.set_moving(1, True, 0)
    s.set_free(1, 1.2, (0.0, 0.004, 0.0))
    prev = 0.004
    for _ in range(4):
        s.step(25)
        st = s.body_state(1)
        assert 0 < st[7] < prev
        prev = st[7]
        assert abs(st[6]) <= 1e-15 and abs(st[8]) <= 1e-15
        assert np.abs(st[:3] - 10.0).max() <= 1e-13


def test_free_sphere_force_average_3d(oracle_mod):
    """With the two-step force average the sphere gains sum_s (F_s + F_{s-1})/2
    (F_{-1} = F_0): fluid plus sphere momentum then balances to
    (F_0 - F_{T-1})/2 exactly; and a neutrally buoyant sphere carried by
    tube flow, which the plain explicit update throws off, moves smoothly."""
    e, _ = _lookup(oracle_mod)
    r, rho_s, G = 4.3, 1.5, np.array([2e-6, -1e-6, 1.5e-6])
    s = oracle_mod.OracleSim3D(22, 20, 18, 0.7, spheres=[dict(cx=10.3, cy=9.6, cz=8.7, r=r)])
    s.set_moving(1, True, 0)
    s.set_free(1, rho_s)
    s.set_gravity(G, oracle_mod.CME)
    s.set_force_average(True)
    vol = 4 / 3 * np.pi * r ** 3
    M = rho_s * vol
    P0 = _fluid_momentum3(s, e)
    T = 60
    s.step(T)
    F0, Fl = s.force(1, oracle_mod.CME, 0)[:3], s.force(1, oracle_mod.CME, T - 1)[:3]
    st = s.body_state(1)
    bal = _fluid_momentum3(s, e) + M * st[3:6] - P0 - T * (M - vol) * G - 0.5 * (F0 - Fl)
    assert np.abs(bal).max() < 1e-12
    n = oracle_mod.OracleSim3D(40, 24, 24, 0.6, g=(3e-5, 0, 0), duct=oracle_mod.TUBE3, R=10.3,
                               spheres=[dict(cx=10.0, cy=13.4, cz=11.5, r=3.6)])
    n.set_moving(1, True, 1)
    n.set_free(1, 1.0)
    n.set_force_average(True)
    vx = []
    for _ in range(200):
        n.step(1)
        vx.append(n.body_state(1)[3])
    vx = np.array(vx)
    assert n.error == 0
    assert 0 < vx[-1] < 0.02 and np.abs(np.diff(vx[-100:])).max() < 1e-4


def test_pressure_driven_planes_poiseuille_3d(oracle_mod):
    """Pressure inlet and outlet (non-equilibrium extrapolation) between the
    planes z = 0 and z = nz - 1: at steady state the mass flux is the same
    through every cross-section, and the profile is the exact discrete
    Poiseuille profile for the local pressure gradient (rho/3)' (up to the
    fluid's compressibility, O(drho))."""
    nx, ny, nz, tau, drho = 24, 3, 12, 1.0, 4e-4
    s = oracle_mod.OracleSim3D(nx, ny, nz, tau, duct=oracle_mod.PLANES3)
    s.set_pressure(1 + drho / 2, 1 - drho / 2)
    s.step(6000)
    rho, u, own = s.fields()
    flux = (rho * u[0])[:, 1, :].sum(0)
    assert np.ptp(flux[1:-1]) <= 1e-9 * abs(flux.mean())
    x, nu = nx // 2, (tau - 0.5) / 3
    rm = rho[1:-1, 1, :].mean(0)
    g = -(rm[x + 4] - rm[x - 4]) / 8 / 3 / rm[x]
    z = np.arange(nz)
    exact = g / (2 * nu) * (((nz - 2) / 2) ** 2 - (z - (nz - 1) / 2) ** 2) + \
        g * (4 * (2 * tau - 1) ** 2 - 3) / (4 * (2 * tau - 1))
    prof = u[0][:, 1, x]
    assert g > 0 and np.abs(prof - exact)[1:-1].max() <= 1e-4 * exact.max()
    # (the boundary planes' streamed state is replaced after each collision)
    assert np.abs(u[2][:, :, 1:-1]).max() <= 1e-5 * exact.max()  # entrance effects only
    with pytest.raises(ValueError):  # not with moving spheres
        m = oracle_mod.OracleSim3D(20, 20, 20, 0.7, spheres=[dict(cx=10.0, cy=10.0, cz=10.0, r=3.0)])
        m.set_moving(1, True, 0)
        m.set_pressure(1.001, 0.999)


def test_pressure_plane_state_3d(oracle_mod):
    """Non-equilibrium extrapolation moves the neighbour's post-collision
    state to the plane's density at the same velocity: on every plane node
    with a fluid neighbour, the post-collision density is exactly rho_b and
    the velocity that of the neighbour (the equilibrium's first two moments:
    sum w_i (1 + 3 e.u + ...) = 1, sum w_i e_i (...) = u).  A plane node
    next to a sphere keeps its own update and is skipped."""
    E3, _ = _lookup(oracle_mod)
    rin, rout = 1.0004, 0.9996
    s = oracle_mod.OracleSim3D(16, 14, 14, 0.7, duct=oracle_mod.TUBE3, R=5.6,
                               spheres=[dict(cx=1.5, cy=7.9, cz=6.2, r=2.2)])
    s.set_pressure(rin, rout)
    s.step(60)
    ft = s.get_ft()
    own = s.fields()[2]
    rho = ft.sum(0)
    j = np.einsum("id,izyx->dzyx", E3.astype(float), ft)
    kept = 0
    for xb, xf, rb in ((0, 1, rin), (15, 14, rout)):
        plane = (own[:, :, xb] == 0) & (own[:, :, xf] == 0)
        kept += int(((own[:, :, xb] == 0) & (own[:, :, xf] != 0)).sum())
        assert plane.sum() > 50
        assert np.abs(rho[:, :, xb][plane] - rb).max() <= 8e-15
        ub = j[:, :, :, xb][:, plane] / rho[:, :, xb][plane]
        uf = j[:, :, :, xf][:, plane] / rho[:, :, xf][plane]
        assert np.abs(uf).max() > 1e-6
        assert np.abs(ub - uf).max() <= 4e-15
    assert kept >= 1  # the sphere's side of the inlet


# ---------------------------------------------------------------- interpolated bounce-back in 3D
def test_ibb_sphere_link_fraction_3d(oracle_mod):
    """q of every link into a sphere is where the segment leaves the fluid,
    found here by bisection on the geometry (minimum image across x)."""
    sp = dict(cx=1.3, cy=8.6, cz=7.8, r=3.7)
    n = (16, 16, 16)
    s = oracle_mod.OracleSim3D(*n, 0.7, spheres=[sp])
    _, _, own = s.fields()
    e, _ = _lookup(oracle_mod)
    count = 0
    for z in range(n[2]):
        for y in range(n[1]):
            for x in range(n[0]):
                if own[z, y, x]:
                    continue
                for i in range(1, 19):
                    xb, yb, zb = (x + e[i, 0]) % n[0], (y + e[i, 1]) % n[1], (z + e[i, 2]) % n[2]
                    if own[zb, yb, xb] != 1:
                        continue
                    lo, hi = 0.0, 1.0
                    for _ in range(60):
                        mid = 0.5 * (lo + hi)
                        p = np.array([x, y, z]) + mid * e[i] - (sp["cx"], sp["cy"], sp["cz"])
                        p = p - np.array(n) * np.floor(p / np.array(n) + 0.5)
                        if p @ p <= sp["r"] ** 2:
                            hi = mid
                        else:
                            lo = mid
                    assert abs(s.link_q(1, x, y, z, i) - hi) <= 1e-12
                    count += 1
    assert count > 100


@pytest.mark.parametrize("moving", [False, True])
def test_ibb_comoving_uniform_flow_3d(oracle_mod, moving):
    """Uniform f_eq(1, U) around a sphere whose surface moves at U stays
    uniform under the interpolated rule for every q (translating too, with
    refill), and the sphere feels nothing."""
    U = (0.05, -0.02, 0.03)
    s = oracle_mod.OracleSim3D(22, 18, 16, 0.7, u0=U, spheres=[dict(cx=9.3, cy=8.6, cz=7.8, r=3.7, v=U)])
    if moving:
        s.set_moving(1, True, 0)
    s.set_ibb(True)
    fe = oracle_mod.feq3(1.0, U)
    for _ in range(4):
        s.step(10)
        f = s.get_f()
        _, _, own = s.fields()
        assert np.abs(f[:, own == 0] - fe[:, None]).max() <= 1e-14
        assert np.abs(s.force(1, oracle_mod.GME)[:3]).max() <= 1e-13


def test_ibb_momentum_balance_3d(oracle_mod):
    """Fixed geometry under the interpolated rule: P(t+1) - P(t) = g sum(rho)
    - sum_s F_CME,s every step, so the returning population the forces take
    is the one streamed."""
    e, _ = _lookup(oracle_mod)
    g = np.array([3e-5, -1e-5, 2e-5])
    sp = dict(cx=8.4, cy=7.2, cz=7.9, r=3.1, v=(0.02, 0.01, -0.005), omega=(0.003, -0.002, 0.004))
    s = oracle_mod.OracleSim3D(18, 16, 16, 0.7, g=tuple(g), duct=oracle_mod.TUBE3, R=6.8, spheres=[sp])
    s.set_ibb(True)
    s.step(10)
    f = s.get_f()
    M0 = f.sum()
    for _ in range(10):
        P0 = _momentum(f, e)
        rho, _, _ = s.fields()
        s.step(1)
        f = s.get_f()
        expect = g * rho.sum() - s.force(0, oracle_mod.CME)[:3] - s.force(1, oracle_mod.CME)[:3]
        assert np.abs(_momentum(f, e) - P0 - expect).max() <= 1e-14 * M0


def test_ibb_tube_link_fraction_3d(oracle_mod):
    """q of every link from the fluid to the tube wall is where the segment
    leaves the cylinder, found by bisection."""
    ny = nz = 21
    R = 8.3
    s = oracle_mod.OracleSim3D(6, ny, nz, 0.7, duct=oracle_mod.TUBE3, R=R)
    _, _, own = s.fields()
    e, _ = _lookup(oracle_mod)
    c = (ny - 1) / 2
    count = 0
    for z in range(nz):
        for y in range(ny):
            if own[z, y, 0]:
                continue
            for i in range(1, 19):
                if e[i, 1] == 0 and e[i, 2] == 0:
                    continue
                yb, zb = y + e[i, 1], z + e[i, 2]
                if own[zb, yb, 0] != 255:
                    continue
                lo, hi = 0.0, 1.0
                for _ in range(60):
                    mid = 0.5 * (lo + hi)
                    py, pz = y + mid * e[i, 1] - c, z + mid * e[i, 2] - c
                    if py * py + pz * pz > R * R:
                        hi = mid
                    else:
                        lo = mid
                assert abs(s.tube_q(y, z, i) - hi) <= 1e-12
                count += 1
    assert count > 50


def test_ibb_tube_momentum_balance_and_comoving_3d(oracle_mod):
    """Interpolated bounce-back on tube and sphere: the momentum balance holds
    every step, and a tube at rest with fluid at rest stays at rest."""
    e, _ = _lookup(oracle_mod)
    g = np.array([3e-5, -1e-5, 2e-5])
    sp = dict(cx=8.4, cy=7.2, cz=7.9, r=3.1, v=(0.02, 0.01, -0.005), omega=(0.003, -0.002, 0.004))
    s = oracle_mod.OracleSim3D(18, 16, 16, 0.7, g=tuple(g), duct=oracle_mod.TUBE3, R=6.8, spheres=[sp])
    s.set_ibb(True)
    s.step(10)
    f = s.get_f()
    M0 = f.sum()
    for _ in range(8):
        P0 = _momentum(f, e)
        rho, _, _ = s.fields()
        s.step(1)
        f = s.get_f()
        expect = g * rho.sum() - s.force(0, oracle_mod.CME)[:3] - s.force(1, oracle_mod.CME)[:3]
        assert np.abs(_momentum(f, e) - P0 - expect).max() <= 1e-14 * M0
    r = oracle_mod.OracleSim3D(10, 17, 17, 0.7, duct=oracle_mod.TUBE3, R=7.3)
    r.set_ibb(True)
    r.step(20)
    _, u, own = r.fields()
    assert np.abs(u[:, own == 0]).max() <= 1e-15


def test_ibb_surface_point_arm_and_velocity_3d(oracle_mod):
    """Under the interpolated rule a link's force acts at the point where the
    link meets the sphere: found here by bisection on the geometry, that point
    p gives (i) the torque of Eq. 7 as the sum of (p - X) x F over the link
    records, for CME and GME, and (ii) the surface velocity of the GME
    correction: F_GME - F_CME = -(a - b) v(p) is parallel to
    v(p) = V + Omega x (p - X) on every link.  The sphere spins about a tilted
    axis and translates in a driven flow, so the link forces are far from
    parallel to e_i and the point off the link midpoint changes both."""
    e, _ = _lookup(oracle_mod)
    n = (18, 16, 16)
    X = np.array([8.4, 7.2, 7.9])
    r = 3.3
    V = np.array([0.004, -0.002, 0.001])
    Om = np.array([0.004, -0.003, 0.005])
    s = oracle_mod.OracleSim3D(*n, 0.7, g=(2e-5, 1e-5, -1e-5),
                               spheres=[dict(cx=X[0], cy=X[1], cz=X[2], r=r, v=tuple(V), omega=tuple(Om))])
    s.set_ibb(True)
    s.step(30)
    s.record_links(20000)
    s.step(1)
    rec = s.links()
    rec = rec[rec[:, 4] == 1]
    assert len(rec) > 200
    T = np.zeros((2, 3))
    worst_par = 0.0
    off_mid = 0
    for x, y, z, i, _, cx, cy, cz, gx, gy, gz in rec:
        i = int(i)
        lo, hi = 0.0, 1.0
        for _ in range(60):
            mid = 0.5 * (lo + hi)
            p = np.array([x, y, z]) + mid * e[i] - X
            p = p - np.array(n) * np.floor(p / np.array(n) + 0.5)
            if p @ p <= r * r:
                hi = mid
            else:
                lo = mid
        q = hi
        off_mid += abs(q - 0.5) > 0.05
        arm = np.array([x, y, z]) + q * e[i] - X
        arm = arm - np.array(n) * np.floor(arm / np.array(n) + 0.5)
        assert abs(np.sqrt(arm @ arm) - r) <= 1e-9  # on the surface
        Fc, Fg = np.array([cx, cy, cz]), np.array([gx, gy, gz])
        T[0] += np.cross(arm, Fc)
        T[1] += np.cross(arm, Fg)
        v = V + np.cross(Om, arm)
        d = Fg - Fc
        # relative to the link's force (d is a small difference of two
        # forces, rounded at their scale)
        worst_par = max(worst_par, np.linalg.norm(np.cross(d, v)) / (np.linalg.norm(Fc) * np.linalg.norm(v)))
    assert off_mid > len(rec) // 4
    assert worst_par <= 1e-13
    for k, sch in enumerate((oracle_mod.CME, oracle_mod.GME)):
        Ts = s.force(1, sch)[3:]
        assert np.abs(Ts - T[k]).max() <= 1e-15 + 1e-12 * np.abs(T[k]).max()
