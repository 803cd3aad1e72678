#!/usr/bin/env python3
"""Benchmark of the D2Q9 momentum-exchange hot path on one MI355X.

Headline workload: the 4096 x 4096 periodic lattice with 64 seeded fixed
cylinders (radii U(8, 16), seed 3003), tau = 0.6, body force 1e-5, plain FP32
storage, CME and GME force and torque of every cylinder every step.  Its two
population buffers (1.2 GB) are 4.7x the 256 MB Infinity Cache, so the step
streams from HBM.  A "step" is one full time step of the hot path (forces and
the fused advection + bounce-back + collision, one launch).

Prints one JSON line: MLUPS over all nodes (events around the timed steps),
the roofline of the one-per-step launch whose update role moves 18
populations per fluid node (timed with HIP events attached to each dispatch on
the library's stream), and in "extra": the same lattice with FP16 and BF16
offset storage, the 2048 x 1024 channel with 32 cylinders (16 translating;
Infinity-Cache resident) with BGK, MRT and interpolated bounce-back, free-disc
sedimentation, the three-dimensional tube, the batched solver on 256 uneven
channel/cylinder cases, the learned warm start (network throughput and time
to steady drag against a plain cold start on held-out channels); and the FP64
CPU oracle timed on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "MLUPS and % HBM roofline; time-to-steady drag at 1e-4 (learned+mixed vs plain)"
BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}


def stored_traffic(workload: str, kernel: str = "k_fused", family: str = "lbm"):
    """HBM bytes per launch of a time-step kernel from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size);
    None when absent or taken on other kernel sources."""
    from paper_1303_0625_amd.build import source_hash

    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != source_hash(family):
        return None
    return round(rec.get("hbm_bytes_per_launch"))


def _note(msg: str) -> None:
    """A progress line on stderr (stdout carries the one JSON line)."""
    print(f"# {time.strftime('%H:%M:%S')} {msg}", file=sys.stderr, flush=True)


def run_copy(torch, mib, repeats=3):
    """A plain device copy of `mib` MiB (torch's copy kernel), timed with HIP
    events: the read-plus-write bandwidth a streaming kernel reaches on this
    device, the practical reference next to the 8 TB/s peak."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(repeats):
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_mib": mib, "repeats": repeats, "ms": [round(m, 4) for m in ms],
            "read_plus_write_GBs": round(2 * n * 4 / (min(ms) * 1e-3) / 1e9, 1)}


def run_gpu(case, dtype, steps, warmup, torch, pkg, mrt=None, ibb=False):
    """Warm up, then time `steps` steps with HIP events around the whole timed
    region, on the lattice's stream.  Whole blocks of 32 steps replay one HIP
    graph, so the step kernels run back to back and the time per step is the
    step kernel's duration plus a gap well under 1 us (the rocprofv3 trace of
    the same command reproduces it; an event pair around each single launch
    would add ~4 us to every launch).  The graph of a start parity is
    instantiated on the first block of 32 steps that starts there: with a
    warm-up of at least 32 steps and an even count it exists before the timed
    region (a shorter or odd warm-up leaves that one-time cost in the timed
    region; fewer than 32 timed steps launch one by one).  A short pass with
    events on each launch then counts the launches per step.  Returns
    (lattice, total_ms, warm-up steps, launches per step, fluid nodes)."""
    warm = warmup
    lat = pkg.Lattice(case, dtype=dtype, history_steps=steps + warm + 9, mrt=mrt)
    if ibb:
        lat.set_boundary(True)
    stream = lat.stream
    lat.step(warm)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    lat.profile(True)
    lat.step(8)
    _, n_launch = lat.profile_read()
    lat.profile(False)
    lat.check()
    _, _, _, own = lat.fields("f32")
    n_fluid = int((own == 0).sum().item())
    return lat, total_ms, warm, n_launch / 8.0, n_fluid


def run_batch(lc, pkg, torch, steps):
    """The 256 uneven channel/cylinder cases (nx = 2 round(U(64, 512)),
    ny = nx/2, seed 4004) advanced together in FP32: autotuned tiling, then
    `steps` steps as graph-captured intervals of 100 steps, each followed by
    the residual/force monitor (tolerance 1e-8).  Throughput counts every node
    of every case; bytes are 72 per fluid node and step."""
    cases = lc.uneven_channels()
    nodes = sum(c["nx"] * c["ny"] for c in cases)
    b = pkg.LatticeBatch(cases, dtype="f32")
    b.autotune(None)
    waves, nt = b.tiling()
    n_fluid = 0
    for k in range(len(cases)):
        rho, _, _ = b.fields(k, "f32")
        n_fluid += int((rho != 0).sum().item())
    b.run(200, 1e-8, 100)  # warm-up: first snapshot, graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = b.run(steps, 1e-8, 100)
    dt = time.perf_counter() - t0
    conv, _, res, _ = b.status()
    gbs = 72 * n_fluid * done / dt / 1e9
    traffic = stored_traffic("batched_uneven_256", "k_batch_step")
    del b
    return {"mlups": round(nodes * done / dt / 1e6, 1), "ms_per_step": round(dt / done * 1e3, 4),
            "steps": done, "cases": len(cases), "nodes": nodes, "fluid_nodes": n_fluid,
            "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "tiling": {"waves_per_workgroup": waves, "nontemporal": bool(nt)},
            "traffic_per_step": traffic, "alg_bytes_per_step": 72 * n_fluid,
            "check_every": 100, "converged": int(sum(conv)), "max_residual": max(res),
            "timing": "wall clock around graph replays, monitor included"}


def run_batch_converge(lc, pkg, torch, cap, start="cold", wall_cap=0.0, chunk=50_000):
    """The 256 uneven cases, FP32, from a cold start or from the exact
    Poiseuille channel flow, to r < 1e-8 (checks every 100 steps,
    graph-replayed intervals, autotuned tiling), at most `cap` steps (and at
    most `wall_cap` seconds when > 0, checked between chunks): converged
    fraction, steps at retirement per case, wall time.  A progress line per
    chunk of steps."""
    cases = lc.uneven_channels()
    b = pkg.LatticeBatch(cases, dtype="f32")
    b.autotune(None)
    if start == "poiseuille":
        for k in range(len(cases)):
            b.init_poiseuille(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while b.t < cap:
        done = b.run(min(chunk, cap - b.t), 1e-8, 100)
        conv = b.status()[0]
        print(f"# step {b.t}: {sum(conv)}/{len(conv)} converged, {time.perf_counter() - t0:.0f} s", flush=True)
        if all(conv) or done == 0 or (wall_cap > 0 and time.perf_counter() - t0 > wall_cap):
            break
    wall = time.perf_counter() - t0
    conv, steps, res, _ = b.status()
    re = [c["Re"] for c in cases]
    nodes = [c["nx"] * c["ny"] for c in cases]
    return {"cases": len(cases), "start": start, "cap": cap, "steps_run": int(b.t), "converged": int(sum(conv)),
            "converged_fraction": round(sum(conv) / len(conv), 4), "wall_s": round(wall, 1),
            "steps": [int(s) if c else None for s, c in zip(steps, conv)],
            "residual_at_end": [float(r) for r in res], "Re": re, "nodes": nodes,
            "criterion": "r = ||u_t - u_{t-100}|| / (100 ||u_t||) < 1e-8 over fluid nodes"}


def run_sedimentation(lc, pkg, torch, steps):
    """Sec. IV.A in lattice units: a channel 120 wide (walls at y) and 1200
    long (periodic in x), a free disc of diameter 30 (0.1 cm in a 0.4 cm
    channel) and density 1.03, released 22.8 nodes (0.076 cm) from a wall,
    tau = 0.6 (nu = 0.01 cm^2/s), gravity 980 cm/s^2 along the channel
    = 4.03e-4 in lattice units.  Timed with GME driving the disc; then the
    paper's frame test: fluid, disc and walls given an extra V = 0.01 along
    the channel, and the trajectory relative to the channel (x - V t, y,
    Omega) compared with the V = 0 run, for GME and for CME, with half-way
    and with interpolated bounce-back (the rule the paper runs with)."""
    nx, ny, r, rho_s, G = 1200, 120, 15.0, 1.03, 4.03e-4

    def case(V):
        body = lc.disc(100.0, 22.3, r, vx=V, moves=True)
        return lc.make_case(nx, ny, 0.6, walls_y=True, u0=(V, 0.0), wall_v=(V, 0.0), bodies=[body],
                            name=f"sediment_V{V}")

    def run(V, scheme, ibb=False):
        lat = pkg.Lattice(case(V), dtype="f64", history_steps=steps + 1)
        if ibb:
            lat.set_boundary(True)
        lat.set_free(1, rho_s)
        lat.set_gravity((G, 0.0), scheme)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat.step(steps)
        lat.check()
        dt = time.perf_counter() - t0
        st = lat.body_state(1)
        return st, dt

    out = {"nx": nx, "ny": ny, "d": 2 * r, "rho_s": rho_s, "G": G, "tau": 0.6, "steps": steps, "dtype": "f64"}
    for ibb in (False, True):
        dst = out
        if ibb:
            dst = out["interpolated_bounce_back"] = {}
        for name, scheme in (("gme", 1), ("cme", 0)):
            s0, dt0 = run(0.0, scheme, ibb)
            s1, _ = run(0.01, scheme, ibb)
            rel = [s1[0] - 0.01 * steps - s0[0], s1[1] - s0[1], s1[4] - s0[4]]
            dst[name] = {"state_V0": [round(v, 9) for v in s0],
                         "frame_V0.01_minus_V0": {"x": rel[0], "y": rel[1], "omega": rel[2]}}
            if scheme == 1:
                dst["ms_per_step"] = round(dt0 / steps * 1e3, 4)
                dst["mlups"] = round(nx * ny * steps / dt0 / 1e6, 1)
    return out


def run_3d(pkg, torch, steps):
    """Sec. IV.D in lattice units: a tube of radius 0.2/0.061 x 5.9 = 19.34
    nodes and length 150, a sphere of radius 5.9 at r*/R = 0.21 (at rest,
    interpolated bounce-back), the pressure drop 1.825e-5 between a pressure
    inlet and outlet (densities 1 +- 3 x 1.825e-5 / 2), tau = 0.6, FP32
    storage.  Then a larger periodic
    tube (768 x 192 x 192, R = 94, the same sphere scaled by 16) driven by the
    equivalent body force 1.825e-5/150, for the kernel's bandwidth: 19
    populations read and written per fluid node, 152 B in FP32."""
    out = {}
    for name, nx, n, R, r in (("tube_150x42x42", 150, 42, 19.34, 5.9), ("tube_768x192x192", 768, 192, 94.0, 28.7)):
        cy = (n - 1) / 2
        small = nx == 150
        case = dict(nx=nx, ny=n, nz=n, tau=0.6, duct=pkg.lbm.LBM3D_TUBE, R=R,
                    g=(0.0, 0.0, 0.0) if small else (1.825e-5 / 150, 0.0, 0.0),
                    spheres=[dict(cx=nx / 4, cy=cy + 0.21 * R, cz=cy, r=r)])
        k = steps if small else max(20, steps // 10)
        lat = pkg.Lattice3D(case, dtype="f32", history_steps=2 * k + 21)
        if small:
            lat.set_pressure(1 + 1.5 * 1.825e-5, 1 - 1.5 * 1.825e-5)
            lat.set_boundary(True)  # the paper's interpolated rule on the sphere
        lat.step(20)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(lat.stream)
        lat.step(k)
        e1.record(lat.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        lat.profile(True)
        lat.step(k)
        kms, kn = lat.profile_read()
        lat.profile(False)
        _, _, own = lat.fields()
        nf = int((own == 0).sum().item())
        nodes = nx * n * n
        kus = kms / max(kn, 1) * 1e3
        out[name] = {"mlups": round(nodes * k / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms / k, 5),
                     "kernel_us": round(kus, 2), "fluid_nodes": nf, "links": lat.link_count(),
                     "achieved_GBs": round(152 * nf / (kus * 1e-6) / 1e9, 1),
                     "frac": round(152 * nf / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "drag_gme": lat.force(1, 1)[0], "drive": "pressure" if small else "body force",
                     "sphere_boundary": "interpolated" if small else "half-way",
                     "alg_bytes_per_launch": 152 * nf,
                     "traffic": None if small else stored_traffic(name, "k3_step", "lbm3d")}
        del lat
        torch.cuda.empty_cache()
    return out


MFMA_BF16_PEAK_TFLOPS = 2500.0


def run_network(pkg):
    """Training and inference throughput of the warm-start network (BF16
    matrix-core convolutions) at 256 x 128, batch 8, in algorithmic FLOPs."""
    from paper_1303_0625_amd import warmstart as ws

    r = ws.network_throughput(batch=8, steps=40)
    r["train_frac_of_bf16_peak"] = round(r["train_tflops"] / MFMA_BF16_PEAK_TFLOPS, 4)
    out = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
    # the deep levels give too few output tiles at batch 8 to fill the
    # device: the same kernels at larger batches
    sweep = {}
    for b in (32, 64):
        q = ws.network_throughput(batch=b, steps=20)
        sweep[str(b)] = {"train_step_ms": round(q["train_step_ms"], 4), "train_tflops": round(q["train_tflops"], 1),
                         "train_frac_of_bf16_peak": round(q["train_tflops"] / MFMA_BF16_PEAK_TFLOPS, 4),
                         "infer_ms": round(q["infer_ms"], 4), "infer_tflops": round(q["infer_tflops"], 1)}
    out["batch_sweep"] = sweep
    return out


def run_warm_start(lc, pkg, n_cases):
    """Time to steady drag (within 1e-4 of an FP64 cold run solved to
    r < 1e-11) of the first n_cases held-out channels (seed 5006): plain FP32
    cold start vs the learned start with FP16 storage switching to FP32."""
    import numpy as np

    from paper_1303_0625_amd import warmstart as ws

    held = lc.warmstart_channels(seed=5006, n_cases=n_cases)
    net = ws.load_net(os.path.join(ROOT, "paper_1303_0625_amd", "weights", "warmstart_256x128.npz"))
    ev = ws.evaluate(held, net, tol=1e-8, tol_stop=1e-9, tol_ref=1e-11, check=100, cap=3_000_000,
                     kinds=("cold", "learned_f16"), log=lambda m: None)
    cold, warm = ev["cold"], ev["learned_f16"]
    ratio = [a / b for a, b in zip(warm["drag_steady_step"], cold["drag_steady_step"]) if a and b]
    tc, tw = cold["batch_drag_steady_wall_s"], warm["batch_drag_steady_wall_s"]
    return {"cases": n_cases, "cases_with_reference": len(ev["steady_cases"]),
            "plain_fp32_cold_s": round(tc, 3) if tc else None,
            "learned_fp16_mixed_s": round(tw, 3) if tw else None,
            "speedup": round(tc / tw, 3) if tc and tw else None,
            "median_step_ratio": round(float(np.median(ratio)), 3) if ratio else None,
            "criterion": "drag within 1e-4 of an FP64 cold run at r < 1e-11, at every later check"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_cpu_baseline(case, steps):
    """The FP64 oracle on a bounded sample of the headline workload: `steps`
    steps of the same lattice, on all host cores (its OpenMP build: the
    per-node collision and advection split over OMP_NUM_THREADS threads, the
    force sum serial), and for reference on one core."""
    import oracle

    def timed(omp):
        o = oracle.OracleSim(case["nx"], case["ny"], case["tau"], gx=case["gx"], bodies=case["bodies"],
                             omp=omp)
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        return time.perf_counter() - t0

    nodes = case["nx"] * case["ny"]
    dt_all = timed(True)
    dt_one = timed(False)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nodes * steps / dt_all / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{steps} steps of the same 4096x4096 workload, FP64 ({dt_all:.1f} s on {threads} threads)",
            "single_thread_mlups": round(nodes * steps / dt_one / 1e6, 3), "cpu_model": cpu_model()}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--dtype", default="f32", choices=list(BYTES))
    ap.add_argument("--cpu-sample-steps", type=int, default=6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reduced-case", action="store_true")
    ap.add_argument("--no-channel-case", action="store_true")
    ap.add_argument("--no-batch-case", action="store_true")
    ap.add_argument("--no-mrt-case", action="store_true")
    ap.add_argument("--no-free-case", action="store_true")
    ap.add_argument("--no-ibb-case", action="store_true")
    ap.add_argument("--no-3d-case", action="store_true")
    ap.add_argument("--free-steps", type=int, default=4000)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-warm-start", action="store_true")
    ap.add_argument("--warm-cases", type=int, default=16)
    ap.add_argument("--only-hbm-case", action="store_true",
                    help="run only the 4096 x 4096 measurement (profiling)")
    ap.add_argument("--only-network", action="store_true",
                    help="run only the warm-start network throughput (profiling)")
    ap.add_argument("--only-c4", type=int, default=0, metavar="CAP",
                    help="run only the 256 uneven channel/cylinder cases (FP32, cold start) to r < 1e-8, "
                         "at most CAP steps; prints progress and the converged fraction and steps per case")
    ap.add_argument("--c4-start", choices=("cold", "poiseuille"), default="cold")
    ap.add_argument("--c4-wall", type=float, default=0.0, metavar="S",
                    help="stop the --only-c4 run after S seconds (checked between chunks of steps)")
    ap.add_argument("--only-copy", type=int, default=0, metavar="MIB",
                    help="run only a plain device copy of MIB MiB, three times (the known-size "
                         "reference that scales the HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the library has no "
              "multi-GPU path.", file=sys.stderr)
        return 2

    import torch

    import lbm_cases as lc
    import paper_1303_0625_amd as pkg

    pkg.lbm.load_library()
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)

    if args.only_copy:
        # a plain device copy of known size: the reference that scales the
        # traffic counters, and the bandwidth a streaming kernel reaches here
        print(json.dumps(run_copy(torch, args.only_copy)), flush=True)
        return 0
    if args.only_network:
        print(json.dumps(run_network(pkg)), flush=True)
        return 0
    if args.only_c4:
        print(json.dumps(run_batch_converge(lc, pkg, torch, args.only_c4, args.c4_start, args.c4_wall)), flush=True)
        return 0
    big = lc.periodic_cylinders()
    if args.only_hbm_case:
        lat2, tms2, w2, lps2, nf2 = run_gpu(big, args.dtype, args.steps, args.warmup, torch, pkg)
        avg2 = tms2 / args.steps * 1e-3
        print(json.dumps({"periodic_4096x4096_kernel_us": round(avg2 * 1e6, 2),
                          "ms_per_step": round(tms2 / args.steps, 5), "launches_per_step": lps2,
                          "warmup": w2, "alg_bytes_per_launch": 18 * BYTES[args.dtype] * nf2,
                          "achieved_GBs": round(18 * BYTES[args.dtype] * nf2 / avg2 / 1e9, 1)}), flush=True)
        return 0

    # headline: the HBM-resident 4096 x 4096 lattice, plain FP32 storage
    nx, ny = big["nx"], big["ny"]
    lat, total_ms, warm, lps, n_fluid = run_gpu(big, args.dtype, args.steps, args.warmup, torch, pkg)
    ms_per_step = total_ms / args.steps
    mlups = nx * ny * args.steps / (total_ms * 1e-3) / 1e6
    # one launch per step (checked): the step kernel's duration is the time
    # per step of the graph-replayed region, back-to-back launches
    assert lps == 1.0, lps
    upd_avg_s = ms_per_step * 1e-3
    alg_bytes = 18 * BYTES[args.dtype] * n_fluid
    achieved = alg_bytes / upd_avg_s / 1e9
    wl = "periodic_4096x4096"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": stored_traffic(wl) if args.dtype == "f32" else None,
                "kernel": "k_fused (one launch per step: force and fused-update roles)",
                "kernel_us": round(upd_avg_s * 1e6, 3), "alg_bytes_per_launch": alg_bytes,
                "timing": "HIP events around the graph-replayed timed region, per step",
                "alg_bytes_per_fluid_node": 18 * BYTES[args.dtype]}
    del lat
    torch.cuda.empty_cache()
    # the same fraction against what a plain device copy reaches here (after
    # the timed region, so that it does not warm the device for it)
    cp = run_copy(torch, 1024)
    roofline["copy_GBs"] = cp["read_plus_write_GBs"]
    roofline["frac_of_copy"] = round(achieved / cp["read_plus_write_GBs"], 4)

    _note(f"headline {wl} done: {ms_per_step * 1e3:.2f} us per step")
    extra = {}
    if not args.no_reduced_case:
        # the same lattice with 16-bit offset storage (FP32 collision, nodes
        # next to a cylinder kept in FP32)
        for dt in ("f16", "bf16"):
            r_steps = min(args.steps, 1000)
            latr, tmsr, _, _, nfr = run_gpu(big, dt, r_steps, min(args.warmup, 64), torch, pkg)
            avgr = tmsr / r_steps * 1e-3
            abr = 18 * BYTES[dt] * nfr
            extra[f"{wl}_{dt}"] = {
                "mlups": round(nx * ny * r_steps / (tmsr * 1e-3) / 1e6, 1),
                "ms_per_step": round(tmsr / r_steps, 5),
                "achieved_GBs": round(abr / avgr / 1e9, 1), "frac": round(abr / avgr / 1e9 / HBM_PEAK_GBS, 4),
                "alg_bytes_per_fluid_node": 18 * BYTES[dt],
                # the 16-bit update issues ~40% more VALU work per node than
                # the FP32 one (decode, segment reference, encode): it is bound
                # by instruction issue and load latency, not by HBM
                "bound": "instruction issue"}
            del latr
            torch.cuda.empty_cache()
    _note("16-bit legs done")
    case = lc.moving_cylinders()
    cwl = "moving_cylinders_2048x1024"
    cnx, cny = case["nx"], case["ny"]
    if not args.no_channel_case:
        # 2048 x 1024 channel, 32 cylinders (16 translating with refill): its
        # FP32 A/B buffers (151 MB) stay in the 256 MB Infinity Cache, so this
        # is not an HBM figure
        c_steps = min(args.steps, 2000)
        latc, tmsc, _, _, nfc = run_gpu(case, "f32", c_steps, args.warmup, torch, pkg)
        avgc = tmsc / c_steps * 1e-3
        abc = 72 * nfc
        extra[cwl] = {"mlups": round(cnx * cny * c_steps / (tmsc * 1e-3) / 1e6, 1),
                      "ms_per_step": round(tmsc / c_steps, 5),
                      "achieved_GBs": round(abc / avgc / 1e9, 1), "frac": round(abc / avgc / 1e9 / HBM_PEAK_GBS, 4),
                      "traffic": stored_traffic(cwl), "residency": "Infinity Cache (151 MB A/B working set)"}
        del latc
        torch.cuda.empty_cache()
    if not args.no_mrt_case:
        # the channel workload with the MRT operator of Sec. IV (paper's rates)
        mrt = pkg.lbm.PAPER_MRT_RATES
        m_steps = min(args.steps, 2000)
        lat3, tms3, _, _, nf3 = run_gpu(case, "f32", m_steps, args.warmup, torch, pkg, mrt=mrt)
        avg3 = tms3 / m_steps * 1e-3
        ab3 = 72 * nf3
        extra["mrt_" + cwl] = {
            "rates_e_eps_q": list(mrt),
            "mlups": round(cnx * cny * m_steps / (tms3 * 1e-3) / 1e6, 1),
            "ms_per_step": round(tms3 / m_steps, 5),
            "achieved_GBs": round(ab3 / avg3 / 1e9, 1),
            "frac": round(ab3 / avg3 / 1e9 / HBM_PEAK_GBS, 4)}
        del lat3
        torch.cuda.empty_cache()
    if not args.no_ibb_case:
        # the channel workload with interpolated bounce-back on the cylinders
        i_steps = min(args.steps, 2000)
        lat4, tms4, _, _, nf4 = run_gpu(case, "f32", i_steps, args.warmup, torch, pkg, ibb=True)
        avg4 = tms4 / i_steps * 1e-3
        ab4 = 72 * nf4
        extra["ibb_" + cwl] = {
            "mlups": round(cnx * cny * i_steps / (tms4 * 1e-3) / 1e6, 1),
            "ms_per_step": round(tms4 / i_steps, 5),
            "achieved_GBs": round(ab4 / avg4 / 1e9, 1),
            "frac": round(ab4 / avg4 / 1e9 / HBM_PEAK_GBS, 4)}
        del lat4
        torch.cuda.empty_cache()
    _note("channel, MRT and interpolated legs done")
    if not args.no_free_case:
        extra["free_sedimentation_1200x120"] = run_sedimentation(lc, pkg, torch, args.free_steps)
        torch.cuda.empty_cache()
    _note("free-body leg done")
    if not args.no_3d_case:
        extra["three_d"] = run_3d(pkg, torch, 2000)

    _note("3D legs done")
    if not args.no_batch_case:
        extra["batched_uneven_256"] = run_batch(lc, pkg, torch, args.batch_steps)
        torch.cuda.empty_cache()

    _note("batch leg done")
    if not args.no_warm_start:
        extra["warm_start_network"] = run_network(pkg)
        extra["warm_start_time_to_steady"] = run_warm_start(lc, pkg, args.warm_cases)
        torch.cuda.empty_cache()

    _note("warm-start legs done")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = run_cpu_baseline(big, args.cpu_sample_steps)

    extra["headline_fluid_node_mlups"] = round(n_fluid * args.steps / (total_ms * 1e-3) / 1e6, 1)
    out = {
        "metric": METRIC, "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{wl}: periodic lattice, 64 fixed cylinders r~U(8,16) seed 3003, "
                               "tau 0.6, body force 1e-5, CME+GME force/torque of every cylinder every step",
                   "nx": nx, "ny": ny, "fluid_nodes": n_fluid},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
