"""Learned warm start on held-out channels (GPU): with the committed weights
(trained by `python -m paper_1303_0625_amd.warmstart train --train 2000
--epochs 300` on the channels of seed 5005), the held-out channels of seed 5006 with Re < 16 reach a steady drag
(within 1e-4 of an FP64 cold run solved to r < 1e-11) in fewer steps from the
learned start than from rest and than from the exact Poiseuille flow; every
start reaches the same steady drag."""
import os
import sys

import numpy as np
import pytest

import lbm_cases as lc

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1303_0625_amd",
                       "weights", "warmstart_256x128.npz")


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_learned_start_reaches_steady_drag_sooner(torch_mod):
    from paper_1303_0625_amd import lbm, warmstart as ws

    lbm.load_library()
    held = [c for c in lc.warmstart_channels(seed=5006, n_cases=64) if c["Re"] < 16.0]
    _say(f"{len(held)} held-out channels with Re < 16")
    net = ws.load_net(WEIGHTS)
    ev = ws.evaluate(held, net, tol=1e-8, tol_stop=1e-9, tol_ref=1e-11, check=100, cap=1_000_000,
                     kinds=("cold", "poiseuille", "learned"), log=_say)
    steady = ev["steady_cases"]
    assert len(steady) == len(held)
    med = {}
    for kind in ("cold", "poiseuille", "learned"):
        st = ev[kind]["drag_steady_step"]
        assert all(s is not None for s in st), kind  # every start reaches the steady drag
        med[kind] = float(np.median(st))
        _say(f"{kind}: median steps to steady drag {med[kind]:.0f}, batch {ev[kind]['batch_drag_steady_wall_s']:.2f} s")
    assert med["learned"] < 0.8 * med["cold"]
    assert med["learned"] < med["poiseuille"]


def test_bad_learned_fields_fall_back_to_cold_start(torch_mod):
    """Warm fields that are not safe to start from (a NaN density in one
    channel, an unphysical speed in another) fail the device start check, and
    those channels start cold instead: their state is the cold start's bit for
    bit, and the batch still solves them; the good channel keeps its warm
    start.  A NaN put into a running case (a diverged start) is restarted cold
    by the solver loop."""
    import torch

    from paper_1303_0625_amd import lbm, warmstart as ws

    lbm.load_library()
    cases = lc.warmstart_channels(seed=5006, n_cases=3)
    ny, nx = cases[0]["ny"], cases[0]["nx"]
    cold = lbm.LatticeBatch(cases, dtype="f32")
    f_cold = ws.all_fields(cold, 3)
    own = torch.stack([cold.fields(k, "f32", owner=True)[3] for k in range(3)]).contiguous()
    rho = torch.ones((3, ny, nx), dtype=torch.float32, device="cuda")
    ux = torch.full((3, ny, nx), 0.01, dtype=torch.float32, device="cuda")
    uy = torch.zeros((3, ny, nx), dtype=torch.float32, device="cuda")
    rho[1, ny // 2, nx // 3] = float("nan")
    ux[2, 5, 7] = 0.9
    fl = (own == 0)
    ok = lbm.warm_check(own, rho, ux, uy).cpu().tolist()
    _say(f"start check {ok}")
    assert ok == [1, 0, 0]
    b = ws.start_batch(cases, "fields", fields=(rho, ux, uy), project=False, destagger=0)
    assert b.fallback == {1, 2}
    f_b = ws.all_fields(b, 3)
    for k in (1, 2):
        for q in range(3):
            assert bool(torch.equal(f_b[q][k], f_cold[q][k])), (k, q)
    assert not bool(torch.equal(f_b[1][0][fl[0]], f_cold[1][0][fl[0]]))
    # a case whose state goes non-finite while running is restarted cold
    bad = rho.clone()
    bad[0, ny // 2, nx // 3] = float("nan")
    b.init_fields(0, bad[0].contiguous(), ux[0].contiguous(), uy[0].contiguous())
    b.fallback.clear()
    ws.solve(b, 1e-8, 100, 400, chunk=200, log=_say)
    assert 0 in b.fallback
    res = b.status()[2]
    assert all(np.isfinite(r) for r in res)
