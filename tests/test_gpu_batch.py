"""Batched steady-state solver through the C ABI (lbm_batch_*).

* a case advanced in a batch of uneven cases matches the same case advanced
  alone (lbm_step) bit for bit, fields and forces, for every tiling;
* FP64 batch against the FP64 oracle (1e-12 on fields, 1e-10 on forces);
* the device residual equals r = ||u_t - u_{t-k}|| / (k ||u_t||) computed on
  the host from the fields;
* run to steady state: cases retire at different steps, a retired case is
  frozen at the state a lone run reaches in the same number of steps, graph
  replay and plain launches agree bit for bit, and at convergence the total
  CME x-force on all solids balances the driving g_x * sum(rho) (momentum
  balance of a steady state);
* the autotuner leaves the initial state untouched and caches its choice.
"""
import os
import sys

import numpy as np
import pytest

import lbm_cases as lc
from tests.helpers import field_errors, force_errors, link_load, oracle_sim

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
    from paper_1303_0625_amd import lbm

    lbm.load_library()
    return lbm


def uneven_cases():
    """Three fixed-geometry cases of uneven size: a walled channel with a
    disc (ragged row length 130), a small channel without bodies and a
    periodic box with a square obstacle."""
    a = lc.make_case(130, 66, 0.8, walls_y=True, gx=2e-6,
                     bodies=[lc.disc(40.3, 32.7, 7.2)], name="chan_disc_130x66")
    b = lc.make_case(64, 16, 1.0, walls_y=True, gx=1e-5, name="chan_empty_64x16")
    c = lc.make_case(96, 80, 0.7, walls_y=False, gx=1e-6, gy=-4e-7,
                     bodies=[lc.box(30.0, 41.0, 6.0, 9.5), lc.disc(70.5, 20.0, 6.0)], name="periodic_box_96x80")
    return [a, b, c]


def _np(t):
    return t.detach().cpu().numpy()


def lone_state(lbm_mod, case, dtype, steps, n_force=1):
    """Fields after `steps` steps and the forces of steps [steps, steps +
    n_force) of a lone run ([n_force][n_solids+1][6]; the first record alone
    when n_force is 1)."""
    lat = lbm_mod.Lattice(case, dtype=dtype, history_steps=steps + n_force + 1)
    lat.step(steps)
    rho, ux, uy, _ = lat.fields("f64")
    fields = (_np(rho), _np(ux), _np(uy))
    lat.step(n_force)
    h = _np(lat.force_history(steps, n_force))
    return fields, (h[0] if n_force == 1 else h)


def batch_forces(batch, k, nb, lbm_mod):
    """[nb+1][6] forces of case k at the last monitor."""
    return np.array([batch.force(k, s, lbm_mod.LBM_CME) + batch.force(k, s, lbm_mod.LBM_GME)
                     for s in range(nb + 1)])


# With 16-bit storage the batch and the lone kernel are two separately compiled
# kernels whose FP32 arithmetic may fuse multiply-adds differently: a one-ulp
# difference at a node kept in FP32 can flip a 16-bit rounding elsewhere, so
# there the states agree to about one 16-bit unit (BF16: 2^-8 of the value)
# instead of bit for bit: velocities and forces within one unit relative to
# their largest magnitude (a one-unit flip at one node moves its velocity by
# ~1e-3 of the field's largest), densities within 1e-5.
SIXTEEN_BIT_UNIT = 2.0 ** -8
SIXTEEN_BIT_RHO = 1e-5


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_batch_matches_lone_runs_bitwise(lbm_mod, dtype):
    cases = uneven_cases()
    steps = 37
    lone = [lone_state(lbm_mod, case, dtype, steps) for case in cases]
    for waves in (1, 2, 4, 8):
        for nt in (False, True):
            _say(f"batch vs lone {dtype} waves={waves} nontemporal={nt}")
            batch = lbm_mod.LatticeBatch(cases, dtype=dtype)
            batch.set_tiling(waves, nt)
            assert batch.tiling() == (waves, int(nt))
            batch.step(steps)
            batch.monitor()
            for k, case in enumerate(cases):
                (rho, ux, uy), h = lone[k]
                brho, bux, buy = (_np(a) for a in batch.fields(k, "f64"))
                bf = batch_forces(batch, k, len(case["bodies"]), lbm_mod)
                if dtype == "bf16":
                    assert np.abs(brho - rho).max() <= SIXTEEN_BIT_RHO, (case["name"], waves, nt)
                    umax = max(np.abs(ux).max(), np.abs(uy).max())
                    du = max(np.abs(bux - ux).max(), np.abs(buy - uy).max())
                    _say(f"  {case['name']}: max |du| / max |u| = {du / umax:.2e}")
                    assert du <= SIXTEEN_BIT_UNIT * umax, (case["name"], waves, nt)
                    assert np.abs(bf - h).max() <= SIXTEEN_BIT_UNIT * max(np.abs(h).max(), 1e-12), case["name"]
                    continue
                assert np.array_equal(brho, rho), (case["name"], waves, nt)
                assert np.array_equal(bux, ux), (case["name"], waves, nt)
                assert np.array_equal(buy, uy), (case["name"], waves, nt)
                assert np.array_equal(bf, h), case["name"]
            del batch


def test_batch_f64_oracle_parity(lbm_mod, oracle_mod):
    # flows with speeds of a few 1e-2 (the oracle keeps absolute populations,
    # whose rounding is ~1e-16 of f ~ 0.1-0.4: relative to a slow start-up
    # flow of |u| ~ 1e-4 that alone is ~1e-12)
    periodic = dict(uneven_cases()[2], u0=(0.03, -0.01), name="periodic_box_96x80_u0")
    cases = [lc.channel_cylinder("moving"), periodic]
    steps = 300
    _say(f"batch f64 vs oracle, {steps} steps")
    batch = lbm_mod.LatticeBatch(cases, dtype="f64")
    batch.step(steps)
    batch.monitor()
    for k, case in enumerate(cases):
        nb = len(case["bodies"])
        osim = oracle_sim(oracle_mod, case)
        osim.step(steps)
        of = osim.fields()
        rho, ux, uy = (_np(a) for a in batch.fields(k, "f64"))
        assert np.array_equal(rho == 0, of[3] != 0)  # solids carry rho = 0
        e = field_errors((rho, ux, uy, of[3]), of)
        _say(f"{case['name']} field err rho={e[0]:.3e} u={e[1]:.3e}")
        assert max(e) <= 1e-12
        # forces of step `steps`: the oracle evaluates them in its next step
        osim.step(1)
        oh = np.array([np.concatenate([osim.force(s, 0, steps), osim.force(s, 1, steps)])
                       for s in range(nb + 1)])
        h = batch_forces(batch, k, nb, lbm_mod)
        worst, rel, where = force_errors(h[None], oh[None], case, 1e-10, link_load(osim, nb))
        _say(f"{case['name']} force err {rel:.3e} (normalised {worst:.3f} at {where})")
        assert worst <= 1.0


def test_batch_residual_matches_host(lbm_mod):
    cases = uneven_cases()
    batch = lbm_mod.LatticeBatch(cases, dtype="f32")
    batch.step(50)
    batch.monitor()
    conv, steps, res, _ = batch.status()
    assert all(r == -1.0 for r in res)
    before = [tuple(_np(a) for a in batch.fields(k, "f64")) for k in range(len(cases))]
    k_int = 30
    batch.step(k_int)
    batch.monitor()
    conv, steps, res, _ = batch.status()
    assert steps == [80] * len(cases) and conv == [0] * len(cases)
    for k in range(len(cases)):
        rho, ux, uy = (_np(a) for a in batch.fields(k, "f64"))
        m = rho != 0
        d2 = ((ux - before[k][1]) ** 2 + (uy - before[k][2]) ** 2)[m].sum()
        u2 = (ux ** 2 + uy ** 2)[m].sum()
        r = np.sqrt(d2) / (k_int * np.sqrt(u2))
        _say(f"case {k}: device r={res[k]:.6e} host r={r:.6e}")
        assert abs(res[k] - r) <= 1e-12 * r


def steady_cases():
    a = lc.make_case(64, 16, 1.0, walls_y=True, gx=1e-5, name="fast_64x16")
    b = lc.make_case(96, 34, 0.9, walls_y=True, gx=4e-6, bodies=[lc.disc(30.2, 16.8, 4.5)], name="disc_96x34")
    c = lc.make_case(70, 40, 0.8, walls_y=True, gx=3e-6, bodies=[lc.box(35.0, 19.5, 4.0, 6.0)], name="box_70x40")
    return [a, b, c]


def test_batch_run_retires_and_balances(lbm_mod):
    cases = steady_cases()
    tol = 1e-11
    _say("batch run to steady state (graph) and without graph")
    runs = []
    for use_graph in (True, False):
        batch = lbm_mod.LatticeBatch(cases, dtype="f64")
        batch.set_graph(use_graph)
        done = batch.run(200000, tol, 100)
        runs.append((batch, done))
    (bg, dg), (bp, dp) = runs
    assert dg == dp
    sg, sp = bg.status(), bp.status()
    _say(f"steps={sg[1]} residual={sg[2]}")
    assert sg == sp
    conv, steps, res, drag = sg
    assert all(conv), res
    assert len(set(steps)) > 1  # uneven convergence
    assert all(0 <= r < tol for r in res)
    for k, case in enumerate(cases):
        fg = [_np(a) for a in bg.fields(k, "f64")]
        fp = [_np(a) for a in bp.fields(k, "f64")]
        for x, y in zip(fg, fp):
            assert np.array_equal(x, y)
        # frozen at retirement: the lone run reaches the same state in as many steps
        nb = len(case["bodies"])
        lone, h = lone_state(lbm_mod, case, "f64", steps[k], n_force=2)
        for x, y in zip(fg, lone):
            assert np.array_equal(x, y), case["name"]
        assert np.array_equal(batch_forces(bg, k, nb, lbm_mod), h[0])
        # steady momentum balance: P(t+1) - P(t) = g_x sum(rho) - sum_s F_x,s
        # (CME).  The staggered momentum sum_x (-1)^x j_x changes sign every
        # step and is not damped (LBGK has the eigenvalue -1 at wavevector
        # (pi, 0) for any tau, and half-way bounce-back keeps it), so near a
        # body the force alternates with period 2 and an even check interval
        # does not see it: the balance holds for the mean over two steps.
        rho = fg[0]
        drive = case["gx"] * rho[rho != 0].sum()
        f2 = h[:, :, 0].sum(axis=1)
        _say(f"{case['name']}: F_x(t)={f2[0]:.12e} F_x(t+1)={f2[1]:.12e} g*sum(rho)={drive:.12e} "
             f"steps={steps[k]}")
        assert abs(0.5 * (f2[0] + f2[1]) - drive) <= 1e-7 * abs(drive)
        if case["bodies"]:
            bsum = sum(bg.force(k, s, lbm_mod.LBM_CME)[0] for s in range(1, len(case["bodies"]) + 1))
            assert drag[k][0] == bsum


def test_batch_autotune_keeps_state_and_caches(lbm_mod, tmp_path):
    cases = uneven_cases()
    cache = str(tmp_path / "tune.txt")
    fresh = lbm_mod.LatticeBatch(cases, dtype="f32")
    ref = [tuple(_np(a) for a in fresh.fields(k, "f64")) for k in range(len(cases))]
    tuned = lbm_mod.LatticeBatch(cases, dtype="f32")
    tuned.autotune(cache)
    assert tuned.t == 0
    w, nt = tuned.tiling()
    _say(f"autotune chose waves={w} nontemporal={nt}")
    assert w in (1, 2, 4, 8)
    for k in range(len(cases)):
        got = [_np(a) for a in tuned.fields(k, "f64")]
        for x, y in zip(got, ref[k]):
            assert np.array_equal(x, y)
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].count("|") == 3
    again = lbm_mod.LatticeBatch(cases, dtype="f32")
    again.autotune(cache)
    assert again.tiling() == (w, nt)
    assert len(open(cache).read().splitlines()) == 1
    tuned.step(5)
    with pytest.raises(lbm_mod.LBMError):
        tuned.autotune(cache)


def test_batch_rejects_bad_input(lbm_mod):
    moving = lc.make_case(64, 32, 0.8, walls_y=True, bodies=[lc.disc(20.0, 15.5, 4.0, vx=0.01, moves=True)])
    with pytest.raises(lbm_mod.LBMError):
        lbm_mod.LatticeBatch([uneven_cases()[0], moving], dtype="f32")
    batch = lbm_mod.LatticeBatch(uneven_cases()[:1], dtype="f32")
    with pytest.raises(lbm_mod.LBMError):
        batch.set_tiling(3)
    with pytest.raises(lbm_mod.LBMError):
        batch.run(100, 1e-8, 1)
    with pytest.raises(lbm_mod.LBMError):
        batch.force(0, 5, 0)


def test_poiseuille_start(lbm_mod):
    """The exact plane-Poiseuille start of an empty walled channel (FP64):
    the fields equal the closed form at once; the populations start at
    equilibrium (no shear part), so the flow relaxes briefly and returns to the
    closed form, its steady state; in a batch that case retires long before the
    same channel started cold."""
    case = lc.make_case(64, 24, 0.8, walls_y=True, gx=5e-6, name="poiseuille_64x24")
    nu, g, ny, tau = 0.1, 5e-6, 24, 0.8
    y = np.arange(ny)
    slip = g * (4 * (2 * tau - 1) ** 2 - 3) / (4 * (2 * tau - 1))
    exact = g / (2 * nu) * ((ny / 2) ** 2 - (y - (ny - 1) / 2) ** 2) + slip
    lat = lbm_mod.Lattice(case, dtype="f64", history_steps=4)
    lat.init_poiseuille()
    rho, ux, uy, _ = (_np(a) for a in lat.fields("f64"))
    assert np.abs(ux - exact[:, None]).max() <= 1e-15 * exact.max() * 10
    assert np.abs(uy).max() <= 1e-15 * exact.max() and np.abs(rho - 1).max() <= 1e-15
    lat.step(40000)
    rho, ux, uy, _ = (_np(a) for a in lat.fields("f64"))
    assert np.abs(ux - exact[:, None]).max() <= 1e-10 * exact.max()
    batch = lbm_mod.LatticeBatch([case, case], dtype="f64")
    batch.init_poiseuille(0)
    batch.run(200000, 1e-10, 100)
    conv, steps, res, _ = batch.status()
    _say(f"steps to r < 1e-10: Poiseuille start {steps[0]}, cold {steps[1]}")
    assert conv == [1, 1] and steps[0] < 0.7 * steps[1]
    # at retirement the distance left to steady state is ~ r / lambda, with
    # lambda = pi^2 nu / ny^2 the slowest decay rate: 1e-10 / 1.7e-3 here
    lam = np.pi ** 2 * nu / ny ** 2
    assert np.abs(_np(batch.fields(0, "f64")[1]) - exact[:, None]).max() <= 10 * 1e-10 / lam * exact.max()


def test_set_active_retires_and_resumes_across_parity(lbm_mod):
    case = uneven_cases()[0]
    batch = lbm_mod.LatticeBatch([case, case], dtype="f64")
    batch.step(10)
    batch.set_active(1, False)
    batch.step(7)  # odd: the retired case's state now sits in the other buffer
    batch.set_active(1, True)
    batch.step(5)
    for k, steps in ((0, 22), (1, 15)):
        (rho, ux, uy), _ = lone_state(lbm_mod, case, "f64", steps)
        got = [_np(a) for a in batch.fields(k, "f64")]
        assert np.array_equal(got[0], rho) and np.array_equal(got[1], ux) and np.array_equal(got[2], uy), k
