"""Pins of the network oracle (oracle/cnn_oracle.py), CPU only.

Each check compares against something other than the oracle's own formulas:
brute-force loops on tiny inputs, adjoint identities (the backward of a linear
map is its transpose), symmetries (x-periodicity, equivariance of the whole
network under shifts by a multiple of 8 nodes), central finite differences of
the loss, and the closed form of Adam's first steps.
"""
import numpy as np
import pytest

from oracle import cnn_oracle as co

RNG = np.random.default_rng(1234)


def brute_conv(x, W, b):
    Bn, H, Wd, C = x.shape
    O = W.shape[0]
    y = np.zeros((Bn, H, Wd, O))
    for n in range(Bn):
        for yy in range(H):
            for xx in range(Wd):
                for o in range(O):
                    acc = b[o]
                    for ky in range(3):
                        sy = yy + ky - 1
                        if sy < 0 or sy >= H:
                            continue
                        for kx in range(3):
                            sx = (xx + kx - 1) % Wd
                            for c in range(C):
                                acc += W[o, ky, kx, c] * x[n, sy, sx, c]
                    y[n, yy, xx, o] = acc
    return y


def test_conv_matches_brute_force():
    x = RNG.normal(size=(2, 4, 6, 3))
    W = RNG.normal(size=(5, 3, 3, 3))
    b = RNG.normal(size=5)
    assert np.abs(co.conv(x, W, b) - brute_conv(x, W, b)).max() <= 1e-13


def test_conv_backward_is_adjoint():
    x = RNG.normal(size=(2, 6, 8, 4))
    W = RNG.normal(size=(3, 3, 3, 4))
    g = RNG.normal(size=(2, 6, 8, 3))
    zero = np.zeros(3)
    dx, dW, db = co.conv_backward(x, W, g)
    lhs = (g * co.conv(x, W, zero)).sum()
    # bilinear in (x, W): <g, conv(x, W)> = <dx, x> = <dW, W>
    assert abs(lhs - (dx * x).sum()) <= 1e-12 * abs(lhs) + 1e-12
    assert abs(lhs - (dW * W).sum()) <= 1e-12 * abs(lhs) + 1e-12
    assert np.abs(db - g.sum(axis=(0, 1, 2))).max() <= 1e-12


def test_pool_and_upsample_adjoints():
    x = RNG.normal(size=(2, 8, 12, 3))
    g = RNG.normal(size=(2, 4, 6, 3))
    assert abs((co.pool(x) * g).sum() - (x * co.pool_backward(g)).sum()) <= 1e-12
    xs = RNG.normal(size=(2, 4, 6, 3))
    gs = RNG.normal(size=(2, 8, 12, 3))
    assert abs((co.upsample(xs) * gs).sum() - (xs * co.upsample_backward(gs)).sum()) <= 1e-12
    # pool of an upsampled field returns it (mean of four equal values)
    assert np.abs(co.pool(co.upsample(xs)) - xs).max() <= 1e-15


def test_conv_periodic_in_x_and_walls_in_y():
    x = RNG.normal(size=(1, 5, 7, 2))
    W = RNG.normal(size=(2, 3, 3, 2))
    b = RNG.normal(size=2)
    y = co.conv(x, W, b)
    assert np.abs(co.conv(np.roll(x, 3, axis=2), W, b) - np.roll(y, 3, axis=2)).max() <= 1e-13
    # an all-ones input with all-ones weights counts the taps inside the walls
    ones = np.ones((1, 5, 7, 1))
    cnt = co.conv(ones, np.ones((1, 3, 3, 1)), np.zeros(1))[0, :, :, 0]
    assert (cnt[0] == 6).all() and (cnt[-1] == 6).all() and (cnt[1:-1] == 9).all()


def _small_net():
    ch = (2, 3, 4, 5)
    p = RNG.normal(size=co.param_count(ch)) * 0.4
    return ch, p


def test_global_context_sees_the_whole_channel():
    """A change of the input ~120 nodes away (both ways round the periodic x,
    beyond the receptive field of the convolutions) changes the output through
    the bottleneck mean; with the global-context weights zeroed it does not."""
    ch, p = _small_net()
    x = RNG.normal(size=(1, 8, 256, 2))
    x2 = x.copy()
    x2[0, :, 124:132, :] += 1.0
    y, _ = co.forward(p, x, ch)
    y2, _ = co.forward(p, x2, ch)
    assert np.abs(y2 - y)[0, :, 0:8].max() > 1e-6
    layers = co.unpack(p, ch)
    W8, b8 = layers[8]
    W8 = W8.copy()
    W8[..., ch[3] + ch[2]:] = 0.0  # the broadcast-mean input channels of the first decoder conv
    layers[8] = (W8, b8)
    p0 = co.pack(layers)
    y, _ = co.forward(p0, x, ch)
    y2, _ = co.forward(p0, x2, ch)
    assert np.abs(y2 - y)[0, :, 0:8].max() == 0.0


def test_network_shift_equivariance():
    """Three 2x2 poolings: shifting the input by 8 nodes along x shifts the
    output by 8 (x is periodic); a shift of 1 in general does not."""
    ch, p = _small_net()
    x = RNG.normal(size=(1, 16, 32, 2))
    y, _ = co.forward(p, x, ch)
    y8, _ = co.forward(p, np.roll(x, 8, axis=2), ch)
    assert np.abs(y8 - np.roll(y, 8, axis=2)).max() <= 1e-12
    y1, _ = co.forward(p, np.roll(x, 1, axis=2), ch)
    assert np.abs(y1 - np.roll(y, 1, axis=2)).max() > 1e-6


def test_network_gradient_finite_differences():
    ch, p = _small_net()
    x = RNG.normal(size=(2, 8, 16, 2))
    t = RNG.normal(size=(2, 8, 16, 3))
    fluid = RNG.random(size=(2, 8, 16)) > 0.2

    def loss(q):
        y, _ = co.forward(q, x, ch)
        return co.masked_mse(y, t, fluid)[0]

    y, tape = co.forward(p, x, ch)
    _, gy = co.masked_mse(y, t, fluid)
    g = co.backward(p, tape, gy, ch)
    idx = RNG.choice(len(p), size=60, replace=False)
    # every layer's bias and a weight of every layer are among the probes
    starts = np.cumsum([0] + [o * 9 * i + o for i, o, _ in co.layer_shapes(ch)])
    idx = np.unique(np.concatenate([idx, starts[:-1], starts[1:] - 1]))
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3 * np.abs(g).max()), (k, fd, g[k])


def test_adam_first_steps_closed_form():
    p0 = RNG.normal(size=10)
    g = RNG.normal(size=10)
    m = np.zeros(10)
    v = np.zeros(10)
    lr, eps = 1e-3, 1e-8
    p1, m, v = co.adam(p0, g, m, v, 1, lr, eps=eps)
    # bias-corrected moments equal g and g^2 for a constant gradient
    assert np.abs(p1 - (p0 - lr * g / (np.abs(g) + eps))).max() <= 1e-15
    p2, m, v = co.adam(p1, g, m, v, 2, lr, eps=eps)
    assert np.abs(p2 - (p1 - lr * g / (np.abs(g) + eps))).max() <= 1e-15


def test_normalisation_round_trip():
    solid = RNG.random(size=(2, 8, 16)) > 0.8
    rho = 1.0 + 1e-3 * RNG.normal(size=solid.shape)
    ux = 0.02 * RNG.normal(size=solid.shape)
    uy = 0.01 * RNG.normal(size=solid.shape)
    uc = np.array([0.03, 0.011])
    t = co.make_target(rho, ux, uy, uc, 0.5)
    r2, x2, y2 = co.fields_from_output(t, solid, uc, 0.5)
    fl = ~solid
    for a, b in ((r2, rho), (x2, ux), (y2, uy)):
        assert np.abs(a[fl] - b[fl]).max() <= 1e-15
        assert (a[solid] == 0).all()
    x = co.make_input(solid, [10.0, 55.0])
    assert (x[..., 0] == solid).all() and (x[1, ..., 1] == 0.55).all()
    # plane-Poiseuille centre-line speed: u_c = g H^2 / (8 nu)
    assert co.u_scale(1e-5, 0.8, 64) == pytest.approx(1e-5 * 64 * 64 / (8 * 0.1), rel=1e-15)


def test_param_count_of_the_warm_start_network():
    # 15 convolutions 3x3 with biases, channels (32, 64, 128, 256); the first
    # decoder convolution also reads the 256 global-context channels
    n = co.param_count()
    expect = sum(o * 9 * i + o for i, o in [(2, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128),
                                            (128, 256), (256, 256), (640, 128), (128, 128), (192, 64),
                                            (64, 64), (96, 32), (32, 32), (32, 3)])
    assert n == expect == 2_242_339


def test_bf16_rounding():
    # 7 stored fraction bits: ulp(1) = 2^-7; halfway cases go to the even neighbour
    cases = {1.0: 1.0, 1 + 2 ** -8: 1.0, 1 + 3 * 2 ** -8: 1 + 2 ** -6, 1 + 2 ** -8 + 2 ** -20: 1 + 2 ** -7,
             -3.0: -3.0, 0.0: 0.0, 2.0 ** -130: 2.0 ** -130}
    for x, want in cases.items():
        assert co.bf16(np.array([x]))[0] == want, x
    torch = pytest.importorskip("torch")
    v = RNG.normal(size=10000) * 10.0 ** RNG.integers(-8, 8, size=10000)
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(co.bf16(v), ref)


def test_storage_rounding_hook():
    """q = identity reproduces the plain network; q = bf16 keeps every stored
    tensor on the bfloat16 grid and moves the output by ~1e-2 at most."""
    ch, p = _small_net()
    x = RNG.normal(size=(1, 8, 16, 2))
    y0, _ = co.forward(p, x, ch)
    y1, t1 = co.forward(p, x, ch, q=lambda a: a)
    assert np.array_equal(y0, y1)
    yb, tb = co.forward(p, x, ch, q=co.bf16)
    for k, inp, _ in tb:
        assert np.array_equal(inp, co.bf16(inp)), k
    assert 0 < np.abs(yb - y0).max() <= 5e-2 * np.abs(y0).max()


def test_warm_project_invariants():
    solid = np.zeros((16, 32), np.uint8)
    yy, xx = np.mgrid[0:16, 0:32]
    solid[(xx - 10.3) ** 2 + (yy - 7.6) ** 2 <= 9] = 1
    rho = 1 + 1e-3 * RNG.normal(size=solid.shape)
    ux = 0.02 + 0.01 * RNG.normal(size=solid.shape)
    uy = 0.01 * RNG.normal(size=solid.shape)
    r, u, v = co.warm_project(solid, rho, ux, uy, 1.0)
    fl = solid == 0
    assert abs(r[fl].mean() - 1.0) <= 1e-15
    J = (r * u).sum(axis=0)
    assert np.abs(J - J.mean()).max() <= 1e-15 * np.abs(J).max() * 10
    assert np.abs((r * v).sum(axis=1)).max() <= 1e-16
    assert abs(((-1.0) ** np.arange(32) * J).sum()) <= 1e-14
    assert (r[~fl] == 0).all() and (u[~fl] == 0).all() and (v[~fl] == 0).all()
    r2, u2, v2 = co.warm_project(solid, r, u, v, 1.0)  # a projection
    assert np.abs(u2 - u).max() <= 1e-16 and np.abs(v2 - v).max() <= 1e-17 and np.abs(r2 - r).max() <= 1e-15


def test_warm_project_removes_the_period_two_force(oracle_mod):
    """A channel with a disc started at equilibrium from the plane-Poiseuille
    profile carries staggered momentum: the drag alternates from step to step
    for good.  Started from the projected profile the alternation decays
    below that of a cold start."""
    nx, ny, tau, g = 64, 32, 0.8, 2e-6
    case = dict(nx=nx, ny=ny, tau=tau, walls_y=True, gx=g, bodies=[{"kind": "disc", "cx": 20.3, "cy": 15.7, "r": 5.2}])
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    slip = g * (4 * (2 * tau - 1) ** 2 - 3) / (4 * (2 * tau - 1))
    prof = g / (2 * nu) * ((ny / 2) ** 2 - (y - (ny - 1) / 2) ** 2) + slip
    swing = {}
    for project in (False, True):
        s = oracle_mod.OracleSim(nx, ny, tau, walls_y=True, gx=g, bodies=case["bodies"])
        solid = s.fields()[3] != 0
        rho = np.where(solid, 0.0, 1.0)
        ux = np.where(solid, 0.0, prof[:, None] * np.ones((1, nx)))
        uy = np.zeros((ny, nx))
        if project:
            rho, ux, uy = co.warm_project(solid, rho, ux, uy, 1.0)
        s.init_fields(rho, ux, uy)
        s.step(10000)
        f = [s.force(1, oracle_mod.CME, st)[0] for st in range(9990, 10000)]
        swing[project] = max(abs(f[k + 1] - f[k]) for k in range(9)) / abs(np.mean(f))
    # measured: 2.8e-3 unprojected (constant from 3000 steps on), 1.9e-7
    # projected; a cold start keeps 1.1e-6 (its amplitude g S / 2)
    assert swing[False] > 1e-3 and swing[True] < 1e-6, swing
