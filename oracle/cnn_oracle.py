"""FP64 CPU oracle of the warm-start network (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU leg may import
this module; it shares no code with the GPU path.  Everything is plain numpy
in float64: one 3x3 convolution is nine shifted matrix products, written from
the definition, and every backward is the adjoint of its forward written out.
The paper has no network (it is this project's learned warm start); the oracle
is pinned by brute-force loops, adjoint identities, symmetries, finite
differences and Adam's closed form (tests/test_cnn_oracle_pins.py).

Network (the layout of the warm-start network of this project):
  input  [B][H][W][2]  : solid mask (1 solid, 0 fluid), Re / 100
  output [B][H][W][3]  : (rho - 1) / (U_c s_rho), u_x / U_c, u_y / U_c
  encoder level l = 0..2 : conv(c_l) ReLU conv(c_l) ReLU  -> skip_l, 2x2 mean pool
  bottleneck             : conv(c_3) ReLU conv(c_3) ReLU -> b, and its mean
                           over the sample's nodes m [c_3] (global context)
  decoder level l = 2..0 : nearest 2x upsample, concat [up, skip_l] (level 2
                           also [.., m broadcast to every node]),
                           conv(c_l) ReLU conv(c_l) ReLU
  head                   : conv(3), no activation
Every conv is 3x3 with a bias; x is periodic (the channel is periodic in x),
y is zero-padded (walls).  Arrays are NHWC.

Parameter vector (flat, float64): for each of the 15 convolutions in the order
enc0a enc0b enc1a enc1b enc2a enc2b bota botb dec2a dec2b dec1a dec1b dec0a
dec0b head: the weights W[c_out][ky][kx][c_in] (ky, kx = 0..2 for offsets
-1..1), then the bias [c_out].
"""
from __future__ import annotations

import numpy as np

IN_CH, OUT_CH = 2, 3


def layer_shapes(ch=(32, 64, 128, 256)):
    """(c_in, c_out, relu) of the 15 convolutions in parameter order."""
    c0, c1, c2, c3 = ch
    return [
        (IN_CH, c0, True), (c0, c0, True),
        (c0, c1, True), (c1, c1, True),
        (c1, c2, True), (c2, c2, True),
        (c2, c3, True), (c3, c3, True),
        (c3 + c2 + c3, c2, True), (c2, c2, True),
        (c2 + c1, c1, True), (c1, c1, True),
        (c1 + c0, c0, True), (c0, c0, True),
        (c0, OUT_CH, False),
    ]


def param_count(ch=(32, 64, 128, 256)) -> int:
    return sum(co * 9 * ci + co for ci, co, _ in layer_shapes(ch))


def unpack(params, ch=(32, 64, 128, 256)):
    """Flat vector -> list of (W [co][3][3][ci], b [co])."""
    out, k = [], 0
    for ci, co, _ in layer_shapes(ch):
        n = co * 9 * ci
        W = np.asarray(params[k:k + n], dtype=np.float64).reshape(co, 3, 3, ci)
        k += n
        b = np.asarray(params[k:k + co], dtype=np.float64)
        k += co
        out.append((W, b))
    assert k == len(params)
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# ----------------------------------------------------------------- primitives
def shift(x, dy, dx):
    """s[b, y, x, c] = x[b, y + dy, (x + dx) mod W, c], zero where y + dy is
    outside [0, H)."""
    H = x.shape[1]
    s = np.roll(x, -dx, axis=2)
    out = np.zeros_like(s)
    if dy == 0:
        out[:] = s
    elif dy > 0:
        out[:, :H - dy] = s[:, dy:]
    else:
        out[:, -dy:] = s[:, :H + dy]
    return out


def conv(x, W, b):
    """y[b,y,x,o] = b[o] + sum over ky, kx, c of W[o,ky,kx,c] x[b, y+ky-1, x+kx-1, c]."""
    Bn, H, Wd, C = x.shape
    co = W.shape[0]
    y = np.zeros((Bn, H, Wd, co)) + b
    for ky in range(3):
        for kx in range(3):
            s = shift(x, ky - 1, kx - 1).reshape(-1, C)
            y += (s @ W[:, ky, kx, :].T).reshape(Bn, H, Wd, co)
    return y


def conv_backward(x, W, g):
    """Gradients of sum(g * conv(x, W, b)) with respect to x, W and b."""
    Bn, H, Wd, C = x.shape
    co = W.shape[0]
    gf = g.reshape(-1, co)
    dW = np.zeros_like(W)
    dx = np.zeros_like(x)
    for ky in range(3):
        for kx in range(3):
            dy_, dx_ = ky - 1, kx - 1
            s = shift(x, dy_, dx_).reshape(-1, C)
            dW[:, ky, kx, :] = gf.T @ s
            # adjoint of the shift: the input node (y + dy, x + dx) received
            # g[y, x] W, i.e. shift g by (-dy, -dx)
            dx += shift((gf @ W[:, ky, kx, :]).reshape(Bn, H, Wd, C), -dy_, -dx_)
    db = gf.sum(axis=0)
    return dx, dW, db


def pool(x):
    """2x2 mean."""
    Bn, H, Wd, C = x.shape
    return x.reshape(Bn, H // 2, 2, Wd // 2, 2, C).mean(axis=(2, 4))


def pool_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) / 4.0


def upsample(x):
    """Nearest neighbour, 2x in both directions."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample_backward(g):
    Bn, H, Wd, C = g.shape
    return g.reshape(Bn, H // 2, 2, Wd // 2, 2, C).sum(axis=(2, 4))


# ----------------------------------------------------------------- storage
def bf16(x):
    """Round to the nearest bfloat16 (ties to even) through float32, as a
    float32 value is stored in 16 bits: keep the top 16 bits after adding
    0x7fff plus the lowest kept bit."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _ident(x):
    return x


# ----------------------------------------------------------------- network
# `q` is the storage rounding of every tensor that is kept between layers
# (network input, weights, activations, pooled maps, and in backward the
# activation gradients); the identity by default.  With q = bf16 the ReLU
# decisions and stored values are those of a BF16-storage implementation while
# the arithmetic stays in float64.
def forward(params, x, ch=(32, 64, 128, 256), q=_ident):
    """Returns (output, tape) where tape holds what backward needs."""
    L = [(q(W), b) for W, b in unpack(params, ch)]
    shapes = layer_shapes(ch)
    tape = []

    def layer(k, inp):
        W, b = L[k]
        pre = conv(inp, W, b)
        out = q(np.maximum(pre, 0.0)) if shapes[k][2] else pre
        tape.append((k, inp, pre))
        return out

    skips = []
    h = q(x)
    for lev in range(3):
        h = layer(2 * lev, h)
        h = layer(2 * lev + 1, h)
        skips.append(h)
        h = q(pool(h))
    h = layer(6, h)
    h = layer(7, h)
    m = q(h.mean(axis=(1, 2)))  # [B][c3]
    for j, lev in enumerate((2, 1, 0)):
        parts = [upsample(h), skips[lev]]
        if lev == 2:
            Bn, H2, W2, _ = skips[2].shape
            parts.append(np.broadcast_to(m[:, None, None, :], (Bn, H2, W2, m.shape[1])))
        h = np.concatenate(parts, axis=3)
        h = layer(8 + 2 * j, h)
        h = layer(9 + 2 * j, h)
    y = layer(14, h)
    return y, tape


def backward(params, tape, gy, ch=(32, 64, 128, 256), q=_ident):
    """Gradient of sum(gy * forward(params, x)) with respect to the parameter
    vector (same layout); q as in forward (the tape must come from a forward
    with the same q)."""
    L = [(q(W), b) for W, b in unpack(params, ch)]
    shapes = layer_shapes(ch)
    grads = [None] * len(L)
    by_k = {k: (inp, pre) for k, inp, pre in tape}
    c = list(ch)

    def layer_back(k, g_out):
        inp, pre = by_k[k]
        g_pre = g_out * (pre > 0) if shapes[k][2] else g_out
        gx, dW, db = conv_backward(inp, L[k][0], g_pre)
        grads[k] = (dW, db)
        return q(gx)

    g = layer_back(14, q(gy))
    g_skip = [None, None, None]
    # decoder in reverse order: level 0 (layers 12, 13) was applied last
    for j, lev in ((2, 0), (1, 1), (0, 2)):
        g = layer_back(9 + 2 * j, g)
        g = layer_back(8 + 2 * j, g)
        c_up = c[lev + 1]
        g_skip[lev] = g[..., c_up:c_up + c[lev]]
        up = upsample_backward(g[..., :c_up])
        if lev == 2:
            # the mean's adjoint: the summed gradient of the broadcast
            # channels, spread evenly over the bottleneck's nodes
            gm = g[..., c_up + c[lev]:].sum(axis=(1, 2))
            up = up + gm[:, None, None, :] / (up.shape[1] * up.shape[2])
        g = q(up)
    g = layer_back(7, g)
    g = layer_back(6, g)
    for lev in (2, 1, 0):
        g = q(pool_backward(g) + g_skip[lev])
        g = layer_back(2 * lev + 1, g)
        g = layer_back(2 * lev, g)
    return pack(grads)


# ----------------------------------------------------------------- loss, data
def masked_mse(y, t, fluid):
    """Mean over fluid nodes and the three output channels of (y - t)^2;
    returns (loss, dloss/dy)."""
    m = fluid[..., None].astype(np.float64)
    n = 3.0 * m.sum()
    d = (y - t) * m
    return float((d * d).sum() / n), 2.0 * d / n


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba): returns (p, m, v); t counts from 1."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def u_scale(gx, tau, ny):
    """Centre-line speed of the unobstructed channel, g H^2 / (8 nu)."""
    nu = (tau - 0.5) / 3.0
    return gx * ny * ny / (8.0 * nu)


def make_input(solid, re):
    """solid [B][H][W] (nonzero = solid), re [B] -> network input [B][H][W][2]."""
    s = (np.asarray(solid) != 0).astype(np.float64)
    r = np.broadcast_to(np.asarray(re, dtype=np.float64)[:, None, None] / 100.0, s.shape)
    return np.stack([s, r], axis=3)


def make_target(rho, ux, uy, uc, rho_scale):
    """Fields [B][H][W] and U_c [B] -> normalised target [B][H][W][3]."""
    uc = np.asarray(uc, dtype=np.float64)[:, None, None]
    return np.stack([(np.asarray(rho) - 1.0) / (uc * rho_scale), np.asarray(ux) / uc,
                     np.asarray(uy) / uc], axis=3)


def fields_from_output(y, solid, uc, rho_scale):
    """Network output -> (rho, ux, uy) [B][H][W]; zero at solid nodes."""
    uc = np.asarray(uc, dtype=np.float64)[:, None, None]
    fl = (np.asarray(solid) == 0)
    rho = np.where(fl, 1.0 + y[..., 0] * uc * rho_scale, 0.0)
    ux = np.where(fl, y[..., 1] * uc, 0.0)
    uy = np.where(fl, y[..., 2] * uc, 0.0)
    return rho, ux, uy


def warm_project(solid, rho, ux, uy, rho0=1.0):
    """Warm-start projection of fields [ny][nx] (fluid nodes only): rho
    shifted to mean rho0; u_x of every column scaled so that its flux
    sum_y rho u_x equals the mean column flux; u_y of every row shifted so that
    its flux sum_x rho u_y is zero.  Returns new arrays."""
    fl = np.asarray(solid) == 0
    rho = np.where(fl, np.asarray(rho, dtype=np.float64), 0.0)
    rho = np.where(fl, rho + (rho0 - rho[fl].mean()), 0.0)
    ux = np.where(fl, np.asarray(ux, dtype=np.float64), 0.0)
    uy = np.where(fl, np.asarray(uy, dtype=np.float64), 0.0)
    J = (rho * ux).sum(axis=0)
    scale = np.where(J != 0.0, J.mean() / np.where(J != 0.0, J, 1.0), 1.0)
    ux = ux * scale[None, :]
    K = (rho * uy).sum(axis=1)
    R = rho.sum(axis=1)
    uy = np.where(fl, uy - np.where(R > 0, K / np.where(R > 0, R, 1.0), 0.0)[:, None], 0.0)
    return rho, ux, uy
