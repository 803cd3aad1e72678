"""Learned warm start: training data from the batched solver, training of the
U-Net through lbm_nn_*, and the comparison of cold, exact-Poiseuille and
learned starts on held-out channels.

Every arithmetic step runs in the library's HIP kernels (solver, network,
normalisation, initialisation); this module orders the calls, draws the
seeded parameter initialisation and minibatch order, and keeps the tallies.

Command line (one GPU):
    python -m paper_1303_0625_amd.warmstart train --train 2000 --epochs 300 --out DIR
        solves 2000 channels (seed 5005) to steady state, trains, and writes
        DIR/warmstart_weights.npz (parameters, rho_scale, channels, grid) and
        DIR/warmstart_train.json;
    python -m paper_1303_0625_amd.warmstart eval --weights W --held 200 --out DIR
        starts 200 held-out channels (seed 5006) cold, from the Poiseuille flow
        and from the network, solves them, writes DIR/warmstart_eval.json.
Both print progress lines as they go.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

from . import lbm

CH = (32, 64, 128, 256)


def _log(msg):
    print(f"[warmstart] {msg}", flush=True)


# --------------------------------------------------------------------- solving
def solve(batch, tol, check, cap, chunk=20000, log=_log, record=False, t0=None, step0=0):
    """Advance a LatticeBatch until every case retires (r < tol) or `cap`
    steps.  With record, one check interval per call and after each check the
    drag and residual of every case: returns (history
    [(wall_s, step0 + step, drags, residuals)], wall seconds)."""
    t0 = time.perf_counter() if t0 is None else t0
    hist = []
    last = time.perf_counter()
    while batch.t < cap:
        if record:
            done = batch.run(check, tol, check)
            conv, _, res, drag = batch.status()
            hist.append((time.perf_counter() - t0, step0 + batch.t, [d[0] for d in drag], list(res)))
        else:
            done = batch.run(min(chunk, cap - batch.t), tol, check)
            conv, _, res, _ = batch.status()
        # a start that diverged (its residual is no longer finite) falls back
        # to the cold start
        for k, r in enumerate(res):
            if not conv[k] and not math.isfinite(r):
                batch.init_cold(k)
                getattr(batch, "fallback", set()).add(k)
                log(f"  case {k}: residual not finite at step {batch.t}, restarted cold")
        if all(conv) or done == 0:
            break
        if time.perf_counter() - last > 20.0:
            last = time.perf_counter()
            log(f"  step {batch.t}: {sum(conv)}/{len(conv)} converged")
    return hist, time.perf_counter() - t0


# --------------------------------------------------------------------- data
def generate(cases, tol=1e-8, check=100, cap=2_000_000, log=_log):
    """Solve every case to steady state (FP32, cold start) and gather the
    training set on the device: solid u8, rho/ux/uy f32 [N][ny][nx], re/gx/tau
    f64 [N]; plus per-case converged flags and steps."""
    import torch

    t0 = time.perf_counter()
    batch = lbm.LatticeBatch(cases, dtype="f32")
    batch.autotune(None)
    solve(batch, tol, check, cap, log=log)
    conv, steps, res, drag = batch.status()
    n = len(cases)
    ny, nx = cases[0]["ny"], cases[0]["nx"]
    dev = batch.workspace.device
    data = {"solid": torch.empty((n, ny, nx), dtype=torch.uint8, device=dev),
            "rho": torch.empty((n, ny, nx), dtype=torch.float32, device=dev),
            "ux": torch.empty((n, ny, nx), dtype=torch.float32, device=dev),
            "uy": torch.empty((n, ny, nx), dtype=torch.float32, device=dev)}
    for k in range(n):
        rho, ux, uy, own = batch.fields(k, "f32", owner=True)
        data["rho"][k], data["ux"][k], data["uy"][k] = rho, ux, uy
        data["solid"][k] = own != 0
    for key, vals in (("re", [c["Re"] for c in cases]), ("gx", [c["gx"] for c in cases]),
                      ("tau", [c["tau"] for c in cases])):
        data[key] = torch.tensor(vals, dtype=torch.float64, device=dev)
    wall = time.perf_counter() - t0
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    log(f"generated {n} cases in {wall:.1f} s: {sum(conv)} converged, steps max {max(steps)}, "
        f"{nodes * float(np.mean(steps)) / 1e9:.2f} G node-steps")
    del batch
    torch.cuda.empty_cache()
    return data, {"converged": conv, "steps": steps, "residual": res, "drag": drag, "wall_s": wall}


def rho_scale_of(data):
    """Root-mean-square of (rho - 1) / U_c over fluid nodes (the density
    output's scale), U_c = g_x ny^2 / (8 nu)."""
    import torch

    nu = (data["tau"] - 0.5) / 3.0
    ny = data["rho"].shape[1]
    uc = (data["gx"] * ny * ny / (8.0 * nu)).to(torch.float64)[:, None, None]
    fl = data["solid"] == 0
    d = (data["rho"].double() - 1.0) / uc
    return float(torch.sqrt((d[fl] ** 2).mean()).item())


# --------------------------------------------------------------------- network
def init_params(seed, ch=CH):
    """He-normal weights (fan-in 9 c_in), zero biases, head scaled by 0.1."""
    rng = np.random.default_rng(seed)
    c0, c1, c2, c3 = ch
    shapes = [(2, c0), (c0, c0), (c0, c1), (c1, c1), (c1, c2), (c2, c2), (c2, c3), (c3, c3),
              (2 * c3 + c2, c2), (c2, c2), (c2 + c1, c1), (c1, c1), (c1 + c0, c0), (c0, c0), (c0, 3)]
    out = []
    for k, (ci, co) in enumerate(shapes):
        w = rng.normal(size=co * 9 * ci) * np.sqrt(2.0 / (9 * ci))
        if k == len(shapes) - 1:
            w *= 0.1
        out += [w, np.zeros(co)]
    return np.concatenate(out).astype(np.float32)


def train(data, train_idx, val_idx, epochs=60, batch=8, lr=1e-3, lr_min=1e-5, seed=0, dtype="bf16",
          rho_scale=1.0, augment=True, log=_log):
    """Adam with a cosine learning-rate decay, each drawn sample shifted in x
    and mirrored in y at random (augment); returns (net, history)."""
    import torch

    ny, nx = data["rho"].shape[1:]
    net = lbm.WarmStartNet(ny, nx, batch, dtype=dtype, ch=CH, rho_scale=rho_scale)
    net.set_params(torch.from_numpy(init_params(seed)))
    rng = np.random.default_rng(seed + 1)
    dev = data["rho"].device
    steps_per_epoch = max(1, len(train_idx) // batch)
    total = epochs * steps_per_epoch
    hist = []
    t0 = time.perf_counter()
    it = 0

    def eval_set(idx):
        if len(idx) == 0:
            return float("nan")
        s = 0.0
        for k in range(0, len(idx), batch):
            part = torch.tensor(idx[k:k + batch], dtype=torch.int32, device=dev)
            s += net.eval(data, part) * len(part)
        return s / len(idx)

    for ep in range(epochs):
        order = rng.permutation(train_idx)
        for k in range(steps_per_epoch):
            frac = it / max(total - 1, 1)
            cur = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * frac))
            part = torch.tensor(order[k * batch:(k + 1) * batch], dtype=torch.int32, device=dev)
            # exact symmetries of the periodic walled channel: x shift, mirror in y
            codes = rng.integers(0, nx, size=len(part)) | (rng.integers(0, 2, size=len(part)) << 16)
            aug = torch.tensor(codes.astype(np.int32), device=dev) if augment else None
            net.train_step(data, part, float(cur), aug=aug)
            it += 1
        if ep % max(1, epochs // 10) == 0 or ep == epochs - 1:
            tr, va = eval_set(train_idx[:64]), eval_set(val_idx)
            hist.append({"epoch": ep, "train_loss": tr, "val_loss": va, "wall_s": time.perf_counter() - t0})
            log(f"epoch {ep}: train loss {tr:.4e}, held-out loss {va:.4e} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return net, {"history": hist, "wall_s": time.perf_counter() - t0, "steps": it, "batch": batch}


def save_weights(path, net, rho_scale):
    np.savez(path, params=net.params().cpu().numpy(), rho_scale=np.float64(rho_scale),
             ch=np.asarray(CH, dtype=np.int32), h=np.int32(net.h), w=np.int32(net.w))


def load_weights(path):
    """(params float32, rho_scale, ch, h, w) from a weights file (no pickles)."""
    with np.load(path, allow_pickle=False) as z:
        return (z["params"].astype(np.float32), float(z["rho_scale"]), tuple(int(c) for c in z["ch"]),
                int(z["h"]), int(z["w"]))


# --------------------------------------------------------------------- evaluation
DESTAGGER_STEPS = 100


def start_batch(cases, kind, net=None, dtype="f32", project=True, fields=None, destagger=DESTAGGER_STEPS):
    """A LatticeBatch of the cases started cold, from the exact Poiseuille
    flow ("poiseuille"), from the network ("learned"), or from given fields
    (rho, ux, uy [n][ny][nx] float32, "fields").  Warm-start fields are
    projected (lbm_warm_project: the cold start's mass, equal column fluxes,
    zero row fluxes) unless project=False, so that they excite no undamped
    staggered momentum.  With destagger = N > 0 the started batch runs N
    steps, and is started again from the projected mean of its fields at
    steps N and N + 1: a warm field meeting a body at rest excites staggered
    modes (sign change every step, decay as slow as the slowest shear mode),
    which that mean removes.  The batch's step counter then stands at N + 1."""
    import torch

    b = lbm.LatticeBatch(cases, dtype=dtype)
    b.fallback = set()  # cases started cold instead (warm fields failed the start check)
    if kind == "cold":
        return b
    _init_warm(b, cases, kind, net, project, fields)
    if destagger > 0:
        b.step(destagger)
        f1 = all_fields(b, len(cases))
        b.step(1)
        f2 = all_fields(b, len(cases))
        own = torch.stack([b.fields(k, "f32", owner=True)[3] for k in range(len(cases))]).contiguous()
        rho0 = float(cases[0].get("rho0", 1.0))
        lbm.warm_project(own, *f1, rho0=rho0, second=f2)
        ok = lbm.warm_check(own, *f1, rho0=rho0).cpu()
        for k in range(len(cases)):
            if k in b.fallback:
                continue  # a cold start needs no de-staggering
            if ok[k]:
                b.init_fields(k, f1[0][k].contiguous(), f1[1][k].contiguous(), f1[2][k].contiguous())
            else:
                b.init_cold(k)
                b.fallback.add(k)
    torch.cuda.synchronize()
    return b


def _init_warm(b, cases, kind, net, project, fields):
    import torch

    dev = b.workspace.device
    step = net.max_batch if net is not None else 16
    for k0 in range(0, len(cases), step):
        part = cases[k0:k0 + step]
        own = torch.stack([b.fields(k0 + j, "f32", owner=True)[3] for j in range(len(part))]).contiguous()
        if kind == "poiseuille":
            fl = []
            for j in range(len(part)):
                b.init_poiseuille(k0 + j)
                fl.append(b.fields(k0 + j, "f32"))
            rho, ux, uy = (torch.stack([f[i] for f in fl]).contiguous() for i in range(3))
        elif kind == "fields":
            rho, ux, uy = (f[k0:k0 + len(part)].clone().contiguous() for f in fields)
        else:
            re = torch.tensor([c["Re"] for c in part], dtype=torch.float64, device=dev)
            gx = torch.tensor([c["gx"] for c in part], dtype=torch.float64, device=dev)
            tau = torch.tensor([c["tau"] for c in part], dtype=torch.float64, device=dev)
            rho, ux, uy = net.infer((own != 0).to(torch.uint8).contiguous(), re, gx, tau)
        rho0 = float(part[0].get("rho0", 1.0))
        if project:
            lbm.warm_project(own, rho, ux, uy, rho0=rho0)
        # the cold start is the fallback of fields that are not safe to start from
        ok = lbm.warm_check(own, rho, ux, uy, rho0=rho0).cpu()
        for j in range(len(part)):
            if ok[j]:
                b.init_fields(k0 + j, rho[j].contiguous(), ux[j].contiguous(), uy[j].contiguous())
            else:
                b.init_cold(k0 + j)
                b.fallback.add(k0 + j)


def all_fields(b, n):
    """rho, ux, uy [n][ny][nx] float32 of a batch's cases (at retirement)."""
    import torch

    fl = [b.fields(k, "f32") for k in range(n)]
    return [torch.stack([f[i] for f in fl]).contiguous() for i in range(3)]


def _step_of(step, k):
    return step[k] if isinstance(step, (list, tuple)) else step


def first_below(hist, k, tol):
    """(step, wall) of the first check at which case k's residual is below
    tol (a record's step is the batch step or a per-case list)."""
    for wall, step, _, res in hist:
        if 0 <= res[k] < tol:
            return _step_of(step, k), wall
    return None


def steady_time(hist, d_inf, rel=1e-4):
    """Per case, the first (step, wall) after which |D - D_inf| <= rel |D_inf|
    at every later check; None if never."""
    out = [None] * len(d_inf)
    for k in range(len(d_inf)):
        ok_from = None
        for rec in hist:
            wall, step, drags = rec[0], rec[1], rec[2]
            good = abs(drags[k] - d_inf[k]) <= rel * abs(d_inf[k])
            if good and ok_from is None:
                ok_from = (_step_of(step, k), wall)
            elif not good:
                ok_from = None
        out[k] = ok_from
    return out


def run_mixed(cases, net, tol_stop, check, cap, switch_tol=1e-5, switch_frac=0.9, max_f16=None, log=_log):
    """Learned start with FP16-offset storage (half the bytes per step) until
    switch_frac of the cases have r < switch_tol (or max_f16 steps), then every
    case in FP32 storage, restarted from its FP16 fields through the same
    de-staggering restart as a warm start.  Per-case step counts add the FP16
    steps a case took (a case retired early waits, uncounted) and the FP32
    steps.  Returns (history [(wall, per-case steps, drags, residuals)],
    per-case converged, per-case steps, wall seconds, FP32 start step)."""
    import torch

    n = len(cases)
    max_f16 = max_f16 if max_f16 is not None else cap // 5
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b16 = start_batch(cases, "learned", net, dtype="f16")
    steps = [b16.t] * n
    hist = []
    while b16.t < max_f16:
        b16.run(check, switch_tol, check)
        conv, steps, res, drag = b16.status()  # steps: at retirement, or the current step
        hist.append((time.perf_counter() - t0, list(steps), [d[0] for d in drag], list(res)))
        if sum(conv) >= switch_frac * n:
            break
    fields = all_fields(b16, n)
    del b16
    b = start_batch(cases, "fields", fields=fields)  # de-staggering restart in FP32
    base = list(steps)
    h2, _ = solve(b, tol_stop, check, cap - max(steps), log=log, record=True, t0=t0)
    for wall, t, drags, res in h2:
        hist.append((wall, [base[k] + t for k in range(n)], drags, res))
    conv, st, _, _ = b.status()
    del b
    return hist, conv, [base[k] + st[k] for k in range(n)], time.perf_counter() - t0, list(base)


def run_start(cases, kind, net, tol_stop, check, cap, log=_log):
    """One start (cold, poiseuille, learned: FP32 storage) solved to tol_stop
    with per-check records [(wall, step, drags, residuals)]; the step is the
    batch step (every active case advances together)."""
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = start_batch(cases, kind, net)
    hist, _ = solve(b, tol_stop, check, cap, log=log, record=True, t0=t0)
    st = b.status()
    del b
    return hist, st, time.perf_counter() - t0


def reference_drag(cases, tol_ref, check, cap, log=_log):
    """Steady drag of every case from a cold start in FP64 storage solved to
    r < tol_ref (a case retired at r still differs from its steady state by
    ~ r / lambda, lambda the slowest decay rate: r < 1e-11 puts D_inf within
    ~1e-5 for the slowest channels here).  Returns (D_inf, reached)."""
    import torch

    b = lbm.LatticeBatch(cases, dtype="f64")
    solve(b, tol_ref, check, cap, log=log)
    conv, _, _, drag = b.status()
    del b
    torch.cuda.empty_cache()
    return [d[0] for d in drag], conv


def evaluate(cases, net, tol=1e-8, tol_stop=1e-9, tol_ref=1e-11, check=100, cap=3_000_000,
             kinds=("cold", "poiseuille", "learned", "learned_f16"), log=_log):
    """Solve the held-out cases from each start (FP32 storage unless named)
    to r < tol_stop with per-check records.  D_inf comes from an FP64 cold
    run to r < tol_ref.  Per start: the step (and wall time) of r < tol, and
    the step and wall time after which the drag stays within 1e-4 of D_inf;
    per batch, the wall time until every case with a reference is steady."""
    import torch

    t0 = time.perf_counter()
    d_inf, ref_ok = reference_drag(cases, tol_ref, check, cap, log=log)
    steady = [k for k, c in enumerate(ref_ok) if c]
    out = {"steady_cases": steady, "d_inf": d_inf, "reference_wall_s": time.perf_counter() - t0}
    log(f"reference: {len(steady)}/{len(cases)} cases below {tol_ref:g} (FP64)")
    for kind in kinds:
        if kind == "learned_f16":
            hist, conv, steps, wall, switch = run_mixed(cases, net, tol_stop, check, cap, log=log)
            r = {"converged_stop": conv, "steps_stop": steps, "drag": hist[-1][2], "wall_s": wall,
                 "switch_step": switch}
        else:
            hist, st, wall = run_start(cases, kind, net, tol_stop, check, cap, log=log)
            conv, steps, res, drag = st
            r = {"converged_stop": conv, "steps_stop": steps, "drag": [d[0] for d in drag], "wall_s": wall}
        fb = [first_below(hist, k, tol) for k in range(len(cases))]
        r["steps_tol"] = [f[0] if f else None for f in fb]
        r["wall_tol"] = [f[1] if f else None for f in fb]
        r["min_residual"] = [min((h[3][k] for h in hist if h[3][k] >= 0), default=None) for k in range(len(cases))]
        sd = steady_time(hist, d_inf)
        r["drag_steady_step"] = [sd[k][0] if sd[k] else None for k in steady]
        r["drag_steady_wall"] = [sd[k][1] if sd[k] else None for k in steady]
        ok = [sd[k][1] for k in steady if sd[k]]
        r["batch_drag_steady_wall_s"] = max(ok) if ok and len(ok) == len(steady) else None
        r["drag_rel_err_end"] = [abs(r["drag"][k] - d_inf[k]) / abs(d_inf[k]) for k in steady]
        out[kind] = r
        log(f"{kind}: {sum(conv)}/{len(conv)} below {tol_stop:g}, wall {wall:.1f} s")
        torch.cuda.empty_cache()
    return out


# --------------------------------------------------------------------- throughput
def network_flops(h, w, ch=CH):
    """Algorithmic FLOPs of one sample through the network: forward (every 3x3
    convolution at its level, real channel counts) and a training step
    (forward, input gradients of layers 1..14, weight gradients)."""
    c0, c1, c2, c3 = ch
    layers = [(2, c0, 0), (c0, c0, 0), (c0, c1, 1), (c1, c1, 1), (c1, c2, 2), (c2, c2, 2), (c2, c3, 3),
              (c3, c3, 3), (2 * c3 + c2, c2, 2), (c2, c2, 2), (c2 + c1, c1, 1), (c1, c1, 1), (c1 + c0, c0, 0),
              (c0, c0, 0), (c0, 3, 0)]
    fwd = [2 * 9 * ci * co * (h >> l) * (w >> l) for ci, co, l in layers]
    return sum(fwd), sum(fwd) + sum(fwd[1:]) + sum(fwd)


def network_throughput(h=128, w=256, batch=8, steps=40, dtype="bf16", seed=0):
    """Training steps per second of the network on synthetic fields (the
    arithmetic does not depend on the values), and inference time per batch.
    Returns a dict with algorithmic TFLOP/s."""
    import torch

    dev = "cuda"
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = 4 * batch
    data = {"solid": (torch.rand((n, h, w), generator=g) < 0.05).to(torch.uint8).to(dev),
            "rho": (1 + 1e-3 * torch.randn((n, h, w), generator=g)).float().to(dev),
            "ux": (0.02 * torch.rand((n, h, w), generator=g)).float().to(dev),
            "uy": (0.002 * torch.randn((n, h, w), generator=g)).float().to(dev),
            "re": (1 + 99 * torch.rand(n, generator=g)).double().to(dev),
            "gx": torch.full((n,), 2e-6, dtype=torch.float64, device=dev),
            "tau": torch.full((n,), 0.6, dtype=torch.float64, device=dev)}
    net = lbm.WarmStartNet(h, w, batch, dtype=dtype, ch=CH, rho_scale=0.01)
    net.set_params(torch.from_numpy(init_params(seed)))
    idx = [torch.arange(k * batch, (k + 1) * batch, dtype=torch.int32, device=dev) for k in range(4)]
    for k in range(3):
        net.train_step(data, idx[k % 4], 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        net.train_step(data, idx[k % 4], 1e-4)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    solid, re, gx, tau = data["solid"][:batch].contiguous(), data["re"][:batch], data["gx"][:batch], data["tau"][:batch]
    net.infer(solid, re, gx, tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        net.infer(solid, re, gx, tau)
    torch.cuda.synchronize()
    di = (time.perf_counter() - t0) / steps
    f_fwd, f_train = network_flops(h, w)
    return {"batch": batch, "dtype": dtype, "train_step_ms": dt * 1e3, "infer_ms": di * 1e3,
            "train_tflops": batch * f_train / dt / 1e12, "infer_tflops": batch * f_fwd / di / 1e12,
            "gflop_per_sample_forward": f_fwd / 1e9, "gflop_per_sample_train": f_train / 1e9}


# --------------------------------------------------------------------- command line
def load_net(path, max_batch=8, dtype="bf16"):
    """A WarmStartNet with the weights of a weights file."""
    import torch

    params, rs, ch, h, w = load_weights(path)
    net = lbm.WarmStartNet(h, w, max_batch, dtype=dtype, ch=ch, rho_scale=rs)
    net.set_params(torch.from_numpy(params))
    return net


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train", help="generate steady fields with the solver, train, save the weights")
    t.add_argument("--train", type=int, default=2000)
    t.add_argument("--tol", type=float, default=1e-8)
    t.add_argument("--cap", type=int, default=2_000_000)
    t.add_argument("--epochs", type=int, default=300)
    t.add_argument("--batch", type=int, default=8)
    t.add_argument("--lr", type=float, default=5e-4)
    t.add_argument("--dtype", default="bf16")
    t.add_argument("--out", required=True)
    e = sub.add_parser("eval", help="cold, Poiseuille and learned starts on held-out channels")
    e.add_argument("--weights", required=True)
    e.add_argument("--held", type=int, default=200)
    e.add_argument("--tol", type=float, default=1e-8)
    e.add_argument("--tol-stop", type=float, default=1e-9)
    e.add_argument("--tol-ref", type=float, default=1e-11)
    e.add_argument("--cap", type=int, default=3_000_000)
    e.add_argument("--kinds", default="cold,poiseuille,learned,learned_f16")
    e.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    import torch

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import lbm_cases as lc

    lbm.load_library()
    torch.cuda.set_device(0)
    os.makedirs(a.out, exist_ok=True)
    if a.cmd == "train":
        cases = lc.warmstart_channels(seed=5005, n_cases=a.train)
        _log(f"training set: {a.train} channels (seed 5005)")
        data, gen = generate(cases, a.tol, 100, a.cap)
        keep = [k for k in range(a.train) if gen["converged"][k]]
        _log(f"{len(keep)} of {a.train} training cases converged (the rest are dropped)")
        sub_data = {k: (v[keep] if v.shape[0] == a.train else v) for k, v in data.items()}
        # density errors relax on the fast acoustic time scale, velocity
        # errors (the flow rate above all) on the slow diffusive one: the
        # density output is normalised by 3x its rms, i.e. 1/9 of the weight
        rs = 3.0 * rho_scale_of(sub_data)
        _log(f"rho_scale {rs:.4e}")
        n_val = max(1, len(keep) // 16)
        val_idx, train_idx = np.array(keep[:n_val]), np.array(keep[n_val:])
        net, tr = train(data, train_idx, val_idx, a.epochs, a.batch, a.lr, dtype=a.dtype, rho_scale=rs)
        save_weights(os.path.join(a.out, "warmstart_weights.npz"), net, rs)
        res = {"train_cases": a.train, "tol": a.tol, "cap": a.cap, "rho_scale": rs,
               "generation": {k: gen[k] for k in ("converged", "steps", "wall_s")},
               "re": [c["Re"] for c in cases], "training": tr}
        with open(os.path.join(a.out, "warmstart_train.json"), "w") as fh:
            json.dump(res, fh)
        return 0
    held = lc.warmstart_channels(seed=5006, n_cases=a.held)
    _log(f"held-out set: {a.held} channels (seed 5006)")
    net = load_net(a.weights)
    kinds = tuple(a.kinds.split(","))
    ev = evaluate(held, net, a.tol, a.tol_stop, a.tol_ref, 100, a.cap, kinds=kinds)
    ev["re"] = [c["Re"] for c in held]
    with open(os.path.join(a.out, "warmstart_eval.json"), "w") as fh:
        json.dump(ev, fh)
    steady = ev["steady_cases"]
    _log(f"{len(steady)} of {a.held} held-out cases reach r < {a.tol_ref:g} from an FP64 cold start")
    for kind in kinds:
        r = ev[kind]
        st = [x for x in r["drag_steady_step"] if x]
        line = f"{kind}: steady drag (1e-4) for {len(st)}/{len(steady)} cases, median steps {np.median(st):.0f}"
        if "cold" in ev:
            ratio = [x / y for x, y in zip(r["drag_steady_step"], ev["cold"]["drag_steady_step"]) if x and y]
            line += f", median ratio to cold {np.median(ratio):.3f}"
        _log(f"{line}; batch steady at {r['batch_drag_steady_wall_s']} s (total {r['wall_s']:.1f} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main())
