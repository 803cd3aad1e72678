"""lbm_create_static (the context in the library's static scratch, for callers
that cannot allocate device memory) against lbm_create with a caller
workspace: the same steps give the same populations, fields and force
history bit for bit, on two contexts in a row (the second smaller, so that
it runs over what the first left in the scratch), in FP64 and FP16 storage;
a second static context on the device and a configuration larger than the
scratch are refused."""
import sys

import numpy as np
import pytest

import lbm_cases as lc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lbm_mod():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1303_0625_amd import lbm

    lbm.load_library()
    return lbm


def _run(lbm_mod, case, dtype, steps, static):
    import torch

    lat = lbm_mod.Lattice(case, dtype=dtype, history_steps=steps, static=static)
    lat.step(steps)
    torch.cuda.synchronize()
    out = (lat.populations().cpu().numpy(), [a.cpu().numpy() for a in lat.fields("f64")],
           lat.force_history().cpu().numpy())
    return lat, out


@pytest.mark.parametrize("dtype", ["f64", "f16"])
def test_static_scratch_matches_workspace(lbm_mod, dtype):
    big = lc.make_case(256, 128, 0.7, walls_y=True, gx=2e-6, name="static_big",
                       bodies=[lc.disc(60.3, 60.2, 9.1, vx=0.03, moves=True), lc.disc(180.2, 64.5, 8.3)])
    small = lc.make_case(96, 48, 0.8, walls_y=True, gx=5e-6, name="static_small",
                         bodies=[lc.disc(40.4, 23.7, 6.2)])
    for case, steps in ((big, 150), (small, 70)):
        _say(f"{case['name']} {dtype}: static scratch vs workspace, {steps} steps")
        ref, ro = _run(lbm_mod, case, dtype, steps, static=False)
        lat, so = _run(lbm_mod, case, dtype, steps, static=True)
        assert np.array_equal(so[0], ro[0])
        for a, b in zip(so[1], ro[1]):
            assert np.array_equal(a, b)
        assert np.array_equal(so[2], ro[2])
        # one static context per device at a time
        with pytest.raises(lbm_mod.LBMError) as e:
            lbm_mod.Lattice(small, dtype=dtype, history_steps=4, static=True)
        assert e.value.status == lbm_mod.LBM_ESTATE
        del lat, ref


def test_static_scratch_refuses_large(lbm_mod):
    c = lc.make_case(2048, 1024, 0.7, walls_y=True, name="static_large")
    with pytest.raises(lbm_mod.LBMError) as e:
        lbm_mod.Lattice(c, dtype="f64", history_steps=4, static=True)
    assert e.value.status == lbm_mod.LBM_ESIZE
    assert "static scratch" in str(e.value)
