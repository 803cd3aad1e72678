"""GPU parity of the three-dimensional (D3Q19) step (Sec. IV.D) through the C
ABI against the FP64 oracle on the same inputs.

Bars as in two dimensions: FP64 storage within 1e-12 relative on fields and
1e-10 on forces (relative to each solid's largest force or torque
component); FP32 storage within 1e-5 relative on drag.
"""
import sys

import numpy as np
import pytest

from tests.helpers import plane_state

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def lbm_mod(torch_mod):
    import paper_1303_0625_amd as pkg

    pkg.lbm.load_library()
    return pkg


def _oracle(oracle_mod, c):
    return oracle_mod.OracleSim3D(c["nx"], c["ny"], c["nz"], c["tau"], g=c.get("g", (0.0, 0.0, 0.0)),
                                  u0=c.get("u0", (0.0, 0.0, 0.0)), duct=c.get("duct", 0), R=c.get("R", 0.0),
                                  spheres=c.get("spheres", ()))


def run_pair(oracle_mod, lbm_mod, c, steps, dtype="f64", chunks=2, ibb=False):
    _say(f"{c['name']} {c['nx']}x{c['ny']}x{c['nz']} steps={steps} dtype={dtype} ibb={ibb}")
    lat = lbm_mod.Lattice3D(c, dtype=dtype, history_steps=steps)
    osim = _oracle(oracle_mod, c)
    if ibb:
        lat.set_boundary(True)
        osim.set_ibb(True)
    for k, sp in enumerate(c.get("spheres", ())):
        if sp.get("moves"):
            osim.set_moving(k + 1, True, c.get("refill", 0))
    for _ in range(chunks):
        lat.step(steps // chunks)
        osim.step(steps // chunks)
    return lat, osim


def field_err(lat, osim):
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    orho, ou, oown = osim.fields()
    assert np.array_equal(own, oown)
    fl = own == 0
    er = np.abs(rho - orho)[fl].max() / orho[fl].max()
    scale = np.abs(ou[:, fl]).max()
    eu = np.abs(u[:, fl] - ou[:, fl]).max() / max(scale, 1e-300)
    _say(f"field rel err rho={er:.3e} u={eu:.3e} (max |u| {scale:.3e})")
    return er, eu


def force_err(lat, osim):
    h = lat.force_history().cpu().numpy()
    oh = np.concatenate([osim.force_history(0), osim.force_history(1)], axis=2)
    assert h.shape == oh.shape, (h.shape, oh.shape)
    worst = 0.0
    for s in range(h.shape[1]):
        for blk in (slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 12)):
            scale = np.abs(oh[:, s, blk]).max()
            if scale == 0.0:
                assert np.abs(h[:, s, blk]).max() <= 1e-14
                continue
            worst = max(worst, np.abs(h[:, s, blk] - oh[:, s, blk]).max() / scale)
    _say(f"force rel err (history max, per solid and block) = {worst:.3e}")
    return worst


def test_tube_sphere_moving_surface_f64(oracle_mod, lbm_mod):
    """Tube (R = 10.3) with a body force along it and an off-axis sphere whose
    surface translates and spins: FP64 fields and per-step CME/GME force and
    torque of tube and sphere."""
    c = dict(name="tube_sphere", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3, g=(2e-5, 0.0, 0.0),
             spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3, v=(0.01, -0.004, 0.002),
                           omega=(0.002, 0.001, -0.003))])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 600)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10


def test_two_spheres_open_box_f64(oracle_mod, lbm_mod):
    """Periodic box, oblique body force, two spheres (one across the periodic
    x boundary), initial flow."""
    c = dict(name="two_spheres", nx=36, ny=28, nz=20, tau=0.8, g=(1e-5, 5e-6, -3e-6), u0=(0.02, 0.0, 0.01),
             spheres=[dict(cx=1.2, cy=9.4, cz=10.3, r=3.6, omega=(0.0, 0.003, 0.0)),
                      dict(cx=20.7, cy=19.2, cz=8.9, r=4.1, v=(-0.01, 0.0, 0.0))])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 400)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10


def test_planes_poiseuille_gpu(lbm_mod):
    """The exact discrete Poiseuille profile between the planes z = 0 and
    z = nz - 1 (D3Q19 reduces to D2Q9 for y-invariant flow), on the GPU."""
    nz, g, tau = 14, 1e-5, 0.8
    c = dict(nx=8, ny=6, nz=nz, tau=tau, duct=2, g=(g, 0.0, 0.0))
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=16)
    lat.step(30000)
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    nu = (tau - 0.5) / 3
    z = np.arange(nz)
    slip = g * (4 * (2 * tau - 1) ** 2 - 3) / (4 * (2 * tau - 1))
    exact = g / (2 * nu) * (((nz - 2) / 2) ** 2 - (z - (nz - 1) / 2) ** 2) + slip
    fl = own[:, 0, 0] == 0
    err = np.abs(u[0][:, 2, 3] - exact)[fl].max() / exact.max()
    _say(f"planes Poiseuille rel err {err:.3e}")
    assert err <= 1e-10
    F = lat.force(0, 0)
    assert abs(F[0] - g * rho.sum()) <= 1e-9 * g * rho.sum()


def test_comoving_sphere_uniform_flow_gpu(lbm_mod):
    """Uniform f_eq(1, U) around a sphere whose surface moves at U stays
    uniform, with no force on the sphere."""
    U = (0.04, -0.015, 0.02)
    c = dict(nx=20, ny=18, nz=16, tau=0.7, u0=U, spheres=[dict(cx=9.3, cy=8.6, cz=7.8, r=4.2, v=U)])
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=32)
    lat.step(20)
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    fl = own == 0
    assert np.abs(rho[fl] - 1.0).max() <= 1e-14
    for d in range(3):
        assert np.abs(u[d][fl] - U[d]).max() <= 1e-15
    for sch in (0, 1):
        assert np.abs(np.array(lat.force(1, sch))[:3]).max() <= 1e-13


def test_tube_sphere_f32_drag(oracle_mod, lbm_mod):
    """FP32 storage (FP64 arithmetic): the sphere's drag within 1e-5 of the
    FP64 oracle over the history."""
    c = dict(name="tube_sphere_f32", nx=40, ny=24, nz=24, tau=0.6, duct=1, R=10.3, g=(2e-5, 0.0, 0.0),
             spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3)])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 1200, dtype="f32")
    h = lat.force_history().cpu().numpy()
    for sch, off in ((0, 0), (1, 6)):
        oh = osim.force_history(sch)
        rel = np.abs(h[100:, 1, off] - oh[100:, 1, 0]).max() / np.abs(oh[100:, 1, 0]).max()
        _say(f"f32 drag history rel err scheme {sch} = {rel:.3e}")
        assert rel <= 1e-5


def test_rejects_overlap_and_bad_args(lbm_mod):
    L = lbm_mod.lbm
    bad = dict(nx=20, ny=20, nz=20, tau=0.7, duct=1, R=6.0, spheres=[dict(cx=10, cy=14.0, cz=9.5, r=3.0)])
    with pytest.raises(L.LBMError):
        lbm_mod.Lattice3D(bad)
    with pytest.raises(L.LBMError):
        lbm_mod.Lattice3D(dict(nx=20, ny=20, nz=20, tau=0.5))


# --------------------------------------------------------------- translating spheres
@pytest.mark.parametrize("refill,steps", [(0, 300), (1, 200), (2, 200)])
def test_translating_sphere_f64(oracle_mod, lbm_mod, refill, steps):
    """A spinning sphere translating obliquely through a tube Poiseuille flow
    (covered and newborn nodes every few steps), refill A1/A2/A3: FP64
    fields and per-step forces and torques against the oracle."""
    c = dict(name=f"moving_sphere_refill{refill}", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3,
             g=(2e-5, 0.0, 0.0), refill=refill,
             spheres=[dict(cx=13.1, cy=13.1, cz=10.6, r=4.3, v=(0.04, 0.004, -0.003), omega=(0.0, 0.002, 0.001),
                           moves=True)])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, steps)
    assert osim.error == 0
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10


def test_translating_sphere_streamed_lattice_f64(oracle_mod, lbm_mod):
    """A lattice above the streaming threshold (2 x 19 x 903,168 FP64 nodes =
    274 MB of populations) takes the update that reads one flag byte per node
    and the owners only next to a solid, with the flags rebuilt after every
    raster of the translating sphere: FP64 fields and per-step forces against
    the oracle, as on the small lattices."""
    c = dict(name="moving_sphere_streamed", nx=128, ny=84, nz=84, tau=0.7, duct=1, R=40.0,
             g=(2e-5, 0.0, 0.0), refill=0,
             spheres=[dict(cx=30.2, cy=45.1, cz=38.3, r=6.2, v=(0.05, 0.01, -0.008), omega=(0.001, 0.002, 0.0),
                           moves=True)])
    assert 2 * 19 * c["ny"] * c["nz"] * 128 * 8 > 256 << 20
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 60, chunks=3)
    assert osim.error == 0
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10


def test_translating_sphere_comoving_gpu(lbm_mod):
    """A sphere translating with the uniform flow f_eq(1, U) across several
    nodes leaves the state uniform and feels no force."""
    U = (0.05, -0.02, 0.03)
    c = dict(nx=22, ny=18, nz=16, tau=0.7, u0=U, spheres=[dict(cx=9.3, cy=8.6, cz=7.8, r=3.7, v=U, moves=True)])
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=64)
    lat.step(60)
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    fl = own == 0
    assert np.abs(rho[fl] - 1.0).max() <= 1e-13
    for d in range(3):
        assert np.abs(u[d][fl] - U[d]).max() <= 1e-14
    assert np.abs(np.array(lat.force(1, 1))[:3]).max() <= 1e-13
    assert int((own == 1).sum()) > 0


def test_translating_sphere_path_check(lbm_mod):
    """A moving sphere that would come within 2 nodes of the tube is refused
    before any step is launched."""
    c = dict(nx=20, ny=22, nz=22, tau=0.7, duct=1, R=9.0,
             spheres=[dict(cx=10.0, cy=10.5, cz=10.5, r=3.0, v=(0.0, 0.2, 0.0), moves=True)])
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=8)
    lat.step(5)
    with pytest.raises(lbm_mod.lbm.LBMError):
        lat.step(40)
    assert lat.t == 5


# --------------------------------------------------------------- free spheres
def _free_pair(oracle_mod, lbm_mod, c, steps, free, G, scheme, average=False):
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=steps)
    osim = _oracle(oracle_mod, c)
    if average:
        lat.set_force_average(True)
        osim.set_force_average(True)
    for sid, rho_s, om in free:
        osim.set_moving(sid, True, c.get("refill", 0))
        osim.set_free(sid, rho_s, om)
        lat.set_free(sid, rho_s, om)
    osim.set_gravity(G, scheme)
    lat.set_gravity(G, scheme)
    _say(f"{c['name']} free={free} G={G} scheme={scheme} steps={steps}")
    for _ in range(2):
        lat.step(steps // 2)
        osim.step(steps // 2)
    lat.check()
    assert osim.error == 0
    return lat, osim


def _compare_bodies(lat, osim, sid, tol):
    g = np.array(lat.body_state(sid))
    o = osim.body_state(sid)
    dx = np.abs(g[:3] - o[:3]).max()
    dv = np.abs(g[3:6] - o[3:6]).max() / max(np.abs(o[3:6]).max(), 1e-12)
    dw = np.abs(g[6:] - o[6:]).max() / max(np.abs(o[6:]).max(), 1e-12)
    _say(f"sphere {sid}: X {o[:3]} |V| {np.linalg.norm(o[3:6]):.3e} |Om| {np.linalg.norm(o[6:]):.3e}; "
         f"|dX| {dx:.2e} rel dV {dv:.2e} rel dOm {dw:.2e}")
    assert dx <= tol and dv <= tol and dw <= tol


@pytest.mark.parametrize("scheme", [0, 1])
def test_free_sphere_sedimentation_f64(oracle_mod, lbm_mod, scheme):
    """A heavy sphere falling along a tube, off the axis, CME or GME driving
    it: FP64 fields, forces and the sphere's state against the oracle after it
    has moved across nodes and turned."""
    c = dict(name=f"free_sphere_s{scheme}", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3, refill=0,
             spheres=[dict(cx=12.2, cy=13.1, cz=10.6, r=4.0, moves=True)])
    lat, osim = _free_pair(oracle_mod, lbm_mod, c, 400, [(1, 1.4, (0.0, 0.0, 0.0))], (4e-4, 0.0, 0.0), scheme)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10
    _compare_bodies(lat, osim, 1, 1e-9)
    st = osim.body_state(1)
    assert st[0] - 12.2 > 1.0 and np.abs(st[6:]).max() > 0  # it has fallen and turns


def test_free_sphere_carried_by_tube_flow_f64(oracle_mod, lbm_mod):
    """A spinning sphere (density 1.5, no gravity) released off the axis of a
    tube Poiseuille flow and carried along by it: FP64 parity with the oracle,
    refill A2.  (At density 1 the explicit coupling oscillates with period 2,
    the known limit of explicit momentum exchange for neutrally buoyant
    particles.)"""
    c = dict(name="carried_sphere", nx=40, ny=24, nz=24, tau=0.6, duct=1, R=10.3, refill=1, g=(3e-5, 0.0, 0.0),
             spheres=[dict(cx=10.0, cy=13.4, cz=11.5, r=3.6, moves=True)])
    lat, osim = _free_pair(oracle_mod, lbm_mod, c, 400, [(1, 1.5, (0.0, 0.0, 0.001))], (0.0, 0.0, 0.0), 1)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10
    _compare_bodies(lat, osim, 1, 1e-9)


def test_free_sphere_api_guards(lbm_mod):
    L = lbm_mod.lbm
    c = dict(nx=24, ny=20, nz=20, tau=0.7, spheres=[dict(cx=10.0, cy=9.5, cz=9.5, r=3.0, moves=True),
                                                     dict(cx=20.0, cy=9.5, cz=9.5, r=2.0)])
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=8)
    with pytest.raises(L.LBMError):
        lat.set_free(2, 1.2)  # not created moving
    with pytest.raises(L.LBMError):
        lat.set_free(1, -1.0)
    lat.set_free(1, 1.2)
    lat.step(2)
    with pytest.raises(L.LBMError):
        lat.set_free(1, 1.3)  # after the first step
    lat.check()
    st = lat.body_state(1)
    assert abs(st[0] - 10.0) < 1e-6


def test_neutral_sphere_force_average_f64(oracle_mod, lbm_mod):
    """A neutrally buoyant sphere released off the axis of a tube Poiseuille
    flow with the two-step force average (the Sec. IV.D setting, small): FP64
    parity with the oracle while it is carried along."""
    c = dict(name="neutral_sphere_avg", nx=40, ny=24, nz=24, tau=0.6, duct=1, R=10.3, refill=0,
             g=(3e-5, 0.0, 0.0), spheres=[dict(cx=10.0, cy=13.4, cz=11.5, r=3.6, moves=True)])
    lat, osim = _free_pair(oracle_mod, lbm_mod, c, 400, [(1, 1.0, (0.0, 0.0, 0.0))], (0.0, 0.0, 0.0), 1,
                           average=True)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10
    _compare_bodies(lat, osim, 1, 1e-9)
    assert osim.body_state(1)[0] > 11.0  # carried downstream


# --------------------------------------------------------------- pressure-driven tube
def test_pressure_driven_tube_f64(oracle_mod, lbm_mod):
    """The Sec. IV.D duct driven by a pressure inlet and outlet (non-equilibrium
    extrapolation) instead of a body force, an off-axis sphere: FP64 fields on
    the interior planes, the boundary planes' extrapolated state (which
    replaces their streamed state after each collision) against the oracle's
    post-collision state there, and per-step forces."""
    c = dict(name="pressure_tube", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3,
             spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3)])
    steps = 400
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=steps)
    lat.set_pressure(1.0002, 0.9998)
    osim = _oracle(oracle_mod, c)
    osim.set_pressure(1.0002, 0.9998)
    _say(f"{c['name']} steps={steps}")
    lat.step(steps)
    osim.step(steps)
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    orho, ou, oown = osim.fields()
    assert np.array_equal(own, oown)
    fl = own == 0
    fl[:, :, 0] = False
    fl[:, :, -1] = False
    er = np.abs(rho - orho)[fl].max() / orho[fl].max()
    eu = np.abs(u[:, fl] - ou[:, fl]).max() / np.abs(ou[:, fl]).max()
    _say(f"interior field rel err rho={er:.3e} u={eu:.3e} (max |u| {np.abs(ou[:, fl]).max():.3e})")
    assert er <= 1e-12 and eu <= 1e-11
    assert force_err(lat, osim) <= 1e-10
    prho, pu, pl = plane_state(oracle_mod, osim, own)
    assert pl.sum() > 400
    epr = np.abs(rho - prho)[pl].max() / prho[pl].max()
    epu = np.abs(u[:, pl] - pu[:, pl]).max() / np.abs(ou[:, fl]).max()
    _say(f"pressure-plane rel err rho={epr:.3e} u={epu:.3e}")
    assert epr <= 1e-12 and epu <= 1e-11
    assert np.abs(rho[:, :, 0][pl[:, :, 0]] - 1.0002).max() <= 1e-13  # the inlet's density
    assert ou[0][fl].mean() > 0  # flows from the inlet to the outlet
    moving = dict(c, spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3, moves=True)])
    m = lbm_mod.Lattice3D(moving, dtype="f64", history_steps=4)
    with pytest.raises(lbm_mod.lbm.LBMError):
        m.set_pressure(1.0002, 0.9998)


@pytest.mark.parametrize("ibb", [False, True])
def test_pressure_planes_next_to_spheres_f64(oracle_mod, lbm_mod, ibb):
    """Pressure planes with a sphere against each: on lines where the node
    next to a plane is solid the plane node keeps its own update (the
    extrapolation needs a fluid neighbour), elsewhere the plane takes its
    neighbour's extrapolated state.  FP64 fields (interior and the plane nodes
    with a solid neighbour) and per-step forces and torques, half-way and
    interpolated bounce-back."""
    c = dict(name="pressure_planes_spheres", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3,
             spheres=[dict(cx=3.8, cy=13.1, cz=10.6, r=3.0), dict(cx=35.2, cy=10.4, cz=12.3, r=3.0)])
    steps = 300
    lat = lbm_mod.Lattice3D(c, dtype="f64", history_steps=steps)
    osim = _oracle(oracle_mod, c)
    if ibb:
        lat.set_boundary(True)
        osim.set_ibb(True)
    lat.set_pressure(1.0003, 0.9997)
    osim.set_pressure(1.0003, 0.9997)
    _say(f"{c['name']} steps={steps} ibb={ibb}")
    lat.step(steps)
    osim.step(steps)
    rho, u, own = (a.cpu().numpy() for a in lat.fields())
    orho, ou, oown = osim.fields()
    assert np.array_equal(own, oown)
    kept_in = (own[:, :, 0] == 0) & (own[:, :, 1] != 0)
    kept_out = (own[:, :, -1] == 0) & (own[:, :, -2] != 0)
    assert kept_in.sum() >= 3 and kept_out.sum() >= 3  # the case this test is for
    fl = own == 0
    fl[:, :, 0] = kept_in
    fl[:, :, -1] = kept_out
    er = np.abs(rho - orho)[fl].max() / orho[fl].max()
    eu = np.abs(u[:, fl] - ou[:, fl]).max() / np.abs(ou[:, fl]).max()
    _say(f"field rel err rho={er:.3e} u={eu:.3e}")
    assert er <= 1e-12 and eu <= 1e-11
    assert force_err(lat, osim) <= 1e-10


# --------------------------------------------------------------- interpolated bounce-back in 3D
def test_ibb_tube_sphere_f64(oracle_mod, lbm_mod):
    """Interpolated bounce-back on a spinning, off-axis sphere in a tube flow
    (the duct half-way): FP64 fields and per-step forces and torques."""
    c = dict(name="ibb_tube_sphere", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3, g=(2e-5, 0.0, 0.0),
             spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3, v=(0.01, -0.004, 0.002), omega=(0.002, 0.001, -0.003))])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 400, ibb=True)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10
    hw = _oracle(oracle_mod, c)
    hw.step(400)
    assert np.abs(hw.fields()[1] - osim.fields()[1]).max() > 1e-7  # the rule is on


@pytest.mark.parametrize("refill", [0, 2])
def test_ibb_translating_sphere_f64(oracle_mod, lbm_mod, refill):
    """A translating, spinning sphere under the interpolated rule: the refill
    stencil streams with the same rule."""
    c = dict(name=f"ibb_moving_sphere_refill{refill}", nx=40, ny=24, nz=24, tau=0.7, duct=1, R=10.3,
             g=(2e-5, 0.0, 0.0), refill=refill,
             spheres=[dict(cx=13.1, cy=13.1, cz=10.6, r=4.3, v=(0.04, 0.004, -0.003), omega=(0.0, 0.002, 0.001),
                           moves=True)])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 240, ibb=True)
    er, eu = field_err(lat, osim)
    assert er <= 1e-12 and eu <= 1e-12
    assert force_err(lat, osim) <= 1e-10


def test_ibb_tube_sphere_f32_drag(oracle_mod, lbm_mod):
    """FP32 storage with the interpolated rule: drag within 1e-5 of the FP64
    oracle."""
    c = dict(name="ibb_tube_sphere_f32", nx=40, ny=24, nz=24, tau=0.6, duct=1, R=10.3, g=(2e-5, 0.0, 0.0),
             spheres=[dict(cx=17.4, cy=13.1, cz=10.6, r=4.3)])
    lat, osim = run_pair(oracle_mod, lbm_mod, c, 1000, dtype="f32", ibb=True)
    h = lat.force_history().cpu().numpy()
    for sch, off in ((0, 0), (1, 6)):
        oh = osim.force_history(sch)
        rel = np.abs(h[100:, 1, off] - oh[100:, 1, 0]).max() / np.abs(oh[100:, 1, 0]).max()
        _say(f"ibb f32 drag history rel err scheme {sch} = {rel:.3e}")
        assert rel <= 1e-5
