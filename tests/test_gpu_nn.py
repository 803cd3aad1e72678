"""Warm-start network on the GPU (lbm_nn_*) against the FP64 network oracle.

Real channel widths (32, 64, 128, 256) on a 32 x 64 lattice (levels down to
4 x 8, pixel counts that leave ragged workgroups), batch 2 of a maximum 3.
Bars: FP32 mode within 1e-5 of the oracle per tensor, relative to its largest
magnitude; BF16 mode within 2e-2 per tensor in relative L2 norm (forward
output, the gradient of every layer's weights and biases); Adam against the
oracle's Adam; training reduces the loss; repeated calls are bit-identical.
In BF16 mode the oracle rounds every stored tensor to bfloat16 where the
kernels store one, so both sides take the ReLU decisions on the same values
(its arithmetic stays FP64).
"""
import sys

import numpy as np
import pytest

from oracle import cnn_oracle as co

pytestmark = pytest.mark.gpu

H, W, B, MAXB = 32, 64, 2, 3
CH = (32, 64, 128, 256)


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


def he_params(seed):
    """He-normal weights (fan-in 9 c_in), small random biases."""
    rng = np.random.default_rng(seed)
    layers = []
    for ci, o, _ in co.layer_shapes(CH):
        Wt = rng.normal(size=(o, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
        b = rng.normal(size=o) * 0.05
        layers.append((Wt, b))
    return co.pack(layers)


def inputs(seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((B, H, W, 2))
    yy, xx = np.mgrid[0:H, 0:W]
    for b in range(B):
        cx, cy, r = rng.uniform(10, W - 10), rng.uniform(8, H - 8), rng.uniform(3, 7)
        x[b, :, :, 0] = ((xx - cx) ** 2 + (yy - cy) ** 2 <= r * r)
        x[b, :, :, 1] = rng.uniform(0.01, 1.0)
    return x


def layer_slices():
    out, k = [], 0
    for ci, o, _ in co.layer_shapes(CH):
        nw = o * 9 * ci
        out.append((slice(k, k + nw), slice(k + nw, k + nw + o)))
        k += nw + o
    return out


def rel_max(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-5), ("bf16", 2e-2)])
def test_forward_backward_parity(torch_mod, lbm_mod, dtype, tol):
    """FP32: max-norm error per tensor, output gradient random noise.  BF16:
    relative L2 error per tensor against the oracle with the same bfloat16
    storage, output gradient of the masked squared-error loss of a smooth
    target.  (A bfloat16 network amplifies single rounding flips: exact ties
    of 2x2 means of bfloat16 values cascade through the levels, so a max-norm
    or a noise gradient measures that chaos, not the kernels.)"""
    torch = torch_mod
    p = he_params(7)
    x = inputs(8)
    if dtype == "f32":
        gy = np.random.default_rng(9).normal(size=(B, H, W, 3))
        q, metric = (lambda a: a), rel_max
    else:
        y64, _ = co.forward(p, x, CH)
        _, gy = co.masked_mse(y64, 0.5 * np.tanh(y64) + 0.1, x[..., 0] == 0)
        q, metric = co.bf16, rel_l2
    _say(f"network {dtype}: oracle forward/backward")
    y_ref, tape = co.forward(p, x, CH, q=q)
    g_ref = co.backward(p, tape, gy, CH, q=q)
    _say(f"network {dtype}: GPU")
    net = lbm_mod.WarmStartNet(H, W, MAXB, dtype=dtype, ch=CH)
    assert net.n_params == co.param_count(CH)
    net.set_params(torch.from_numpy(p))
    y = net.forward(torch.from_numpy(x)).cpu().numpy()
    e_y = metric(y, y_ref)
    net.backward(torch.from_numpy(gy))
    g = net.grads().cpu().numpy()
    worst = (0.0, None)
    for k, (sw, sb) in enumerate(layer_slices()):
        for name, s in (("w", sw), ("b", sb)):
            e = metric(g[s], g_ref[s])
            if e > worst[0]:
                worst = (e, (k, name))
    _say(f"{dtype}: output rel err {e_y:.3e}; worst gradient rel err {worst[0]:.3e} at layer {worst[1]}")
    assert e_y <= tol
    assert worst[0] <= tol
    # bit-identical on a repeat
    y2 = net.forward(torch.from_numpy(x)).cpu().numpy()
    net.backward(torch.from_numpy(gy))
    assert np.array_equal(y, y2)
    assert np.array_equal(g, net.grads().cpu().numpy())


def test_adam_matches_oracle(torch_mod, lbm_mod):
    torch = torch_mod
    p = he_params(11)
    x = inputs(12)
    gy = np.random.default_rng(13).normal(size=(B, H, W, 3))
    net = lbm_mod.WarmStartNet(H, W, MAXB, dtype="f32", ch=CH)
    net.set_params(torch.from_numpy(p))
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    q = p.copy()
    for t in (1, 2, 3):
        net.forward(torch.from_numpy(x))
        net.backward(torch.from_numpy(gy))
        g = net.grads().cpu().numpy().astype(np.float64)
        q, m, v = co.adam(np.float32(q).astype(np.float64), g, m, v, t, 1e-3)
        net.adam(1e-3)
        got = net.params().cpu().numpy()
        # FP32 master: one rounding of the update per step
        assert np.abs(got - q).max() <= 1e-6 * max(np.abs(q).max(), 1.0), t


def synthetic_set(torch, n, seed):
    """Channel-like samples: a disc in a walled channel, a plane-Poiseuille
    flow with a smooth wake (a fixed analytic map of (mask, Re)), so the
    network has something learnable."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    solid = np.zeros((n, H, W), np.uint8)
    rho = np.zeros((n, H, W), np.float32)
    ux = np.zeros((n, H, W), np.float32)
    uy = np.zeros((n, H, W), np.float32)
    re = rng.uniform(1, 100, size=n)
    tau = rng.uniform(0.55, 1.2, size=n)
    gx = rng.uniform(1e-6, 1e-5, size=n)
    for k in range(n):
        cx, cy, r = rng.uniform(12, W - 12), rng.uniform(10, H - 10), rng.uniform(3, 6)
        d2 = (xx - cx) ** 2 + (yy - cy) ** 2
        solid[k] = d2 <= r * r
        uc = co.u_scale(gx[k], tau[k], H)
        prof = 4 * (yy + 0.5) * (H - 0.5 - yy) / (H * H)
        wake = np.exp(-d2 / (4 * r * r) * (1 + re[k] / 100))
        ux[k] = np.where(solid[k], 0, uc * prof * (1 - wake))
        uy[k] = np.where(solid[k], 0, uc * 0.1 * (yy - cy) / r * wake)
        rho[k] = np.where(solid[k], 0, 1 + 0.01 * uc * (xx - cx) / W)
    dev = "cuda"
    return {"solid": torch.from_numpy(solid).to(dev), "rho": torch.from_numpy(rho).to(dev),
            "ux": torch.from_numpy(ux).to(dev), "uy": torch.from_numpy(uy).to(dev),
            "re": torch.from_numpy(re).to(dev), "gx": torch.from_numpy(gx).to(dev),
            "tau": torch.from_numpy(tau).to(dev)}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_training_reduces_loss_and_infer_matches_oracle(torch_mod, lbm_mod, dtype):
    torch = torch_mod
    data = synthetic_set(torch, 12, 21)
    net = lbm_mod.WarmStartNet(H, W, MAXB, dtype=dtype, ch=CH, rho_scale=0.05)
    net.set_params(torch.from_numpy(he_params(22)))
    all_idx = torch.arange(MAXB, dtype=torch.int32, device="cuda")
    loss0 = net.eval(data, all_idx)
    rng = np.random.default_rng(23)
    for it in range(150):
        idx = torch.from_numpy(rng.choice(12, size=MAXB, replace=False).astype(np.int32)).to("cuda")
        net.train_step(data, idx, 1e-3)
    loss1 = net.eval(data, all_idx)
    _say(f"{dtype}: loss {loss0:.4e} -> {loss1:.4e} after 150 steps")
    assert loss1 < 0.2 * loss0
    # the loss the library reports equals the oracle's on its own output
    p = net.params().cpu().numpy().astype(np.float64)
    solid = data["solid"][:MAXB].cpu().numpy()
    x = co.make_input(solid, data["re"][:MAXB].cpu().numpy())
    uc = co.u_scale(data["gx"][:MAXB].cpu().numpy(), data["tau"][:MAXB].cpu().numpy(), H)
    t = co.make_target(data["rho"][:MAXB].cpu().numpy(), data["ux"][:MAXB].cpu().numpy(),
                       data["uy"][:MAXB].cpu().numpy(), uc, 0.05)
    y_ref, _ = co.forward(p, x, CH, q=co.bf16 if dtype == "bf16" else (lambda a: a))
    l_ref = co.masked_mse(y_ref, t, solid == 0)[0]
    tol = 1e-5 if dtype == "f32" else 2e-2
    # an output error dy moves the loss by at most 2 sqrt(loss) rms(dy) + rms(dy)^2
    fl3 = np.broadcast_to((solid == 0)[..., None], y_ref.shape)
    dy = tol * (np.abs(y_ref).max() if dtype == "f32" else np.sqrt(np.mean(y_ref[fl3] ** 2)))
    _say(f"{dtype}: loss {loss1:.6e}, oracle {l_ref:.6e}")
    assert abs(loss1 - l_ref) <= 2.0 * np.sqrt(l_ref) * dy + dy * dy
    rho, ux, uy = net.infer(data["solid"][:MAXB].contiguous(), data["re"][:MAXB].contiguous(),
                            data["gx"][:MAXB].contiguous(), data["tau"][:MAXB].contiguous())
    r_ref, x_ref, v_ref = co.fields_from_output(y_ref, solid, uc, 0.05)
    fl = solid == 0
    rho_g, ux_g, uy_g = rho.cpu().numpy(), ux.cpu().numpy(), uy.cpu().numpy()
    if dtype == "f32":
        # each field against its own largest magnitude; rho is written in FP32
        # next to 1, so one unit in the last place on top
        assert rel_max(np.stack([ux_g, uy_g]), np.stack([x_ref, v_ref])) <= tol
        assert np.abs(rho_g[fl] - r_ref[fl]).max() <= tol * np.abs(r_ref[fl] - 1.0).max() + 1.2e-7
    else:
        # the fields back in network units, against the whole output (relative L2)
        ucb = np.broadcast_to(uc[:, None, None], solid.shape)
        back = np.stack([(rho_g - 1.0) / (ucb * 0.05), ux_g / ucb, uy_g / ucb], axis=-1)[fl]
        e = rel_l2(back, y_ref[fl])
        _say(f"bf16: inferred fields vs oracle output, relative L2 {e:.3e}")
        assert e <= tol
    assert (rho.cpu().numpy()[~fl] == 0).all()


def test_augmentation_codes(torch_mod, lbm_mod):
    """A drawn sample shifted in x (bits 0..15) or mirrored about the centre
    line (bit 16, u_y negated) gives the loss of the same sample transformed
    on the host and stored; equal up to the order of the loss sum."""
    torch = torch_mod
    base = synthetic_set(torch, 1, 31)
    s0 = {k: v.cpu().numpy() for k, v in base.items()}

    def mirror(a):
        return a[:, ::-1, :].copy()

    def roll(a):
        return np.roll(a, 5, axis=2)

    data = {"solid": np.concatenate([s0["solid"], mirror(s0["solid"]), roll(s0["solid"])]),
            "rho": np.concatenate([s0["rho"], mirror(s0["rho"]), roll(s0["rho"])]),
            "ux": np.concatenate([s0["ux"], mirror(s0["ux"]), roll(s0["ux"])]),
            "uy": np.concatenate([s0["uy"], -mirror(s0["uy"]), roll(s0["uy"])])}
    for k in ("re", "gx", "tau"):
        data[k] = np.repeat(s0[k], 3)
    data = {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for k, v in data.items()}
    net = lbm_mod.WarmStartNet(H, W, 1, dtype="f32", ch=CH, rho_scale=0.05)
    p = torch.from_numpy(he_params(32))

    def loss(sample, code):
        net.set_params(p)
        idx = torch.tensor([sample], dtype=torch.int32, device="cuda")
        aug = torch.tensor([code], dtype=torch.int32, device="cuda") if code is not None else None
        return net.train_step(data, idx, 1e-9, want_loss=True, aug=aug)

    assert loss(0, None) == loss(0, 0)
    assert abs(loss(0, 1 << 16) - loss(1, None)) <= 1e-6 * loss(1, None)
    assert abs(loss(0, 5) - loss(2, None)) <= 1e-6 * loss(2, None)
    assert abs(loss(0, 5) - loss(0, None)) > 1e-4 * loss(0, None)  # the network is not shift-invariant by 5


def test_warm_project_matches_oracle(torch_mod, lbm_mod):
    torch = torch_mod
    rng = np.random.default_rng(41)
    n, ny, nx = 3, 32, 64
    yy, xx = np.mgrid[0:ny, 0:nx]
    solid = np.zeros((n, ny, nx), np.uint8)
    for k in range(n):
        solid[k][(xx - rng.uniform(10, 50)) ** 2 + (yy - rng.uniform(8, 24)) ** 2 <= rng.uniform(9, 36)] = 1
    rho = (1 + 1e-3 * rng.normal(size=solid.shape)).astype(np.float32)
    ux = (0.02 + 0.005 * rng.normal(size=solid.shape)).astype(np.float32)
    uy = (0.003 * rng.normal(size=solid.shape)).astype(np.float32)
    # a second field set is averaged in first
    rho2 = (rho + 1e-4).astype(np.float32)
    ux2 = (ux * 0.9).astype(np.float32)
    uy2 = (-uy).astype(np.float32)
    tens = [torch.from_numpy(a).to("cuda") for a in (solid, rho, ux, uy)]
    second = tuple(torch.from_numpy(a).to("cuda") for a in (rho2, ux2, uy2))
    lbm_mod.warm_project(*tens, rho0=1.0, second=second)
    torch.cuda.synchronize()
    for k in range(n):
        r, u, v = co.warm_project(solid[k], 0.5 * (rho[k] + rho2[k]), 0.5 * (ux[k] + ux2[k]), 0.5 * (uy[k] + uy2[k]), 1.0)
        fl = solid[k] == 0
        g = [t[k].cpu().numpy().astype(np.float64) for t in tens[1:]]
        assert np.abs(g[0][fl] - r[fl]).max() <= 2e-7
        assert np.abs(g[1][fl] - u[fl]).max() <= 1e-6 * np.abs(u).max()
        assert np.abs(g[2][fl] - v[fl]).max() <= 1e-6 * np.abs(uy[k]).max() + 1e-9
        # the staggered column flux of the projected field vanishes
        J = (g[0] * g[1] * fl).sum(axis=0)
        assert abs(((-1.0) ** np.arange(nx) * J).sum()) <= 1e-5 * np.abs(J).max()


def _layer_wgrad_case(torch, lbm, h, w, ch, batch, dtype, seed):
    """Every layer's weight and bias gradient through lbm_nn_layer_wgrad on
    random tensors of the compute type (padding channels filled with noise
    that must not leak), against the oracle's conv_backward on the same
    values in FP64.  The products of two stored values are exact in FP32, so
    the only difference is the FP32 accumulation order: max-norm 2e-5."""
    net = lbm.WarmStartNet(h, w, batch, dtype=dtype, ch=ch)
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    rng = np.random.default_rng(seed)
    worst = 0.0
    for k, (cout, cin) in enumerate(net.layer_shapes()):
        lv = net.LAYER_LEVELS[k]
        hl, wl = h >> lv, w >> lv
        x_cs = max(16, cin)
        g_cs = (cout + 31) // 32 * 32
        xt = torch.tensor(rng.normal(size=(batch, hl, wl, x_cs)), dtype=tdt, device="cuda")
        gt = torch.tensor(rng.normal(size=(batch, hl, wl, g_cs)), dtype=tdt, device="cuda")
        got = net.layer_wgrad(k, xt, gt).cpu().numpy().astype(np.float64)
        x64 = xt.float().cpu().numpy().astype(np.float64)[..., :cin]
        g64 = gt.float().cpu().numpy().astype(np.float64)[..., :cout]
        _, dW, db = co.conv_backward(x64, np.zeros((cout, 3, 3, cin)), g64)
        ref = np.concatenate([dW.reshape(-1), db])
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        _say(f"layer_wgrad {dtype} {h}x{w} batch {batch} layer {k} ({cout}x{cin}, level {lv}): {err:.2e}")
        assert err < 2e-5, (k, err)
        worst = max(worst, err)
    return worst


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_layer_wgrad_exact_small(torch_mod, lbm_mod, dtype):
    """32 x 64 lattice: levels 2 and 3 (rows of 16 and 8) take the per-tap
    kernel, levels 0 and 1 the nine-tap kernel in BF16."""
    _layer_wgrad_case(torch_mod, lbm_mod, H, W, CH, 3, dtype, 71)


def test_layer_wgrad_exact_full(torch_mod, lbm_mod):
    """The 256 x 128 training lattice at batch 3 (every level nine-tap in
    BF16; split counts from the planner, ragged last splits)."""
    _layer_wgrad_case(torch_mod, lbm_mod, 128, 256, CH, 3, "bf16", 72)


def _layer_forward_case(torch, lbm, h, w, batch, seed):
    """Layers 1..13 through lbm_nn_layer_forward on random BF16 inputs, against
    ReLU(conv + b) of the oracle in FP64 on the same inputs and the weights
    rounded to bfloat16.  The kernels add exact products in FP32 and round
    the sum to bfloat16 once: |y - ref| <= 2^-8 |ref| + 1e-5 max |ref|."""
    net = lbm.WarmStartNet(h, w, batch, dtype="bf16", ch=CH)
    params = he_params(seed)
    net.set_params(params)
    layers = co.unpack(params, CH)
    rng = np.random.default_rng(seed + 1)
    for k in range(1, 14):
        cout, cin = net.layer_shapes()[k]
        lv = net.LAYER_LEVELS[k]
        hl, wl = h >> lv, w >> lv
        xt = torch.tensor(rng.normal(size=(batch, hl, wl, cin)), dtype=torch.bfloat16, device="cuda")
        y = net.layer_forward(k, xt).float().cpu().numpy().astype(np.float64)
        x64 = xt.float().cpu().numpy().astype(np.float64)
        Wk, bk = layers[k]
        ref = np.maximum(co.conv(x64, co.bf16(Wk), bk), 0.0)
        excess = (np.abs(y - ref) - 2.0 ** -8 * np.abs(ref)).max() / np.abs(ref).max()
        _say(f"layer_forward {h}x{w} batch {batch} layer {k} ({cout}x{cin}, level {lv}): excess {excess:.2e}")
        assert excess <= 1e-5, (k, excess)


def test_layer_forward_exact_full(torch_mod, lbm_mod):
    """The 256 x 128 training lattice at batch 3 (levels 0-2 on the kernel that
    holds the input tile across the taps, level 3 on the LDS-tiled GEMM)."""
    _layer_forward_case(torch_mod, lbm_mod, 128, 256, 3, 81)


def test_layer_forward_exact_small(torch_mod, lbm_mod):
    """32 x 64 lattice: too few tiles for the tap-holding kernel, every layer
    on the LDS-tiled GEMM."""
    _layer_forward_case(torch_mod, lbm_mod, H, W, 2, 82)
