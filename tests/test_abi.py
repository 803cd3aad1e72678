"""The C ABI library loads and exports every symbol include/lbm.h declares, and
argument validation rejects bad input before any device work (CPU only)."""
import ctypes
import os
import re

import pytest

import lbm_cases as lc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_1303_0625_amd import lbm

    if not os.path.exists(lbm.LIB_PATH):
        from paper_1303_0625_amd.build import build_library

        build_library()
    lbm.load_library()
    return lbm


def header_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm(?:3d)?_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 52
    lib = ctypes.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.exported_symbols())
    assert L.lbm_abi_version() == 1


def _create(L, case, tau=0.8, ws=None, nbytes=1 << 30, dtype="f64"):
    g = L.make_grid(case, dtype)
    arr, n = L._solid_array(case["bodies"])
    ctx = ctypes.c_void_p()
    st = L.load_library().lbm_create(ctypes.byref(g), tau, arr, n, 16, ws, nbytes, None,
                                     ctypes.byref(ctx))
    return st, ctx


def test_validation_errors(L):
    c = lc.channel_cylinder("rest")
    assert _create(L, c, tau=0.5)[0] == L.LBM_EINVAL
    assert "tau" in L.lbm_last_error()
    assert _create(L, c, ws=None)[0] == L.LBM_EINVAL
    assert _create(L, c, ws=256 * 7 + 1)[0] == L.LBM_EINVAL  # misaligned
    assert _create(L, c, ws=1 << 20, nbytes=64)[0] == L.LBM_ESIZE
    fast = dict(c, bodies=[lc.disc(63.5, 31.5, 5.0, vx=0.31)])
    assert _create(L, fast)[0] == L.LBM_EINVAL
    both = dict(c, bodies=[lc.disc(40.0, 31.5, 5.0), lc.disc(50.5, 31.5, 5.0)])
    assert _create(L, both)[0] == L.LBM_EGEOM
    wall = dict(c, bodies=[lc.disc(63.5, 6.0, 5.0)])
    assert _create(L, wall)[0] == L.LBM_EGEOM
    bad = dict(c, nx=2)
    assert _create(L, bad)[0] == L.LBM_EINVAL
    g = L.make_grid(c, "f64")
    g.dtype = 9
    out = ctypes.c_size_t()
    arr, n = L._solid_array(c["bodies"])
    assert L.load_library().lbm_workspace_bytes(ctypes.byref(g), arr, n, 16, ctypes.byref(out)) == L.LBM_EINVAL


def test_workspace_scales_with_dtype(L):
    c = lc.channel_cylinder("rest")
    sizes = {d: L.lbm_workspace_bytes(L.make_grid(c, d), c["bodies"], 16) for d in ("f64", "f32", "f16", "bf16")}
    assert sizes["f64"] > sizes["f32"] and sizes["f16"] == sizes["bf16"]
    # two population buffers dominate: 2 * 9 * ny * pitch * bytes
    assert sizes["f32"] >= 2 * 9 * 64 * 128 * 4
    # 16-bit storage: two buffers, each with an FP32 array for the nodes next
    # to a solid, the buffers one such array apart
    assert sizes["f16"] >= 2 * 9 * 64 * 128 * (2 + 4)


def test_batch_workspace_validation(L):
    a = lc.make_case(130, 66, 0.8, walls_y=True, gx=2e-6, bodies=[lc.disc(40.3, 32.7, 7.2)])
    b = lc.make_case(64, 16, 1.0, walls_y=True, gx=1e-5)
    grids = [L.make_grid(a, "f32"), L.make_grid(b, "f32")]
    solids = [a["bodies"], b["bodies"]]
    nbytes = L.lbm_batch_workspace_bytes(grids, [0.8, 1.0], solids)
    # both cases' two population buffers (rows padded to 64 nodes)
    assert nbytes >= 2 * 9 * 4 * (66 * 192 + 16 * 64)
    with pytest.raises(L.LBMError) as e:
        L.lbm_batch_workspace_bytes(grids, [0.8, 0.5], solids)
    assert "case 1" in str(e.value) and "tau" in str(e.value)
    moving = [[lc.disc(40.3, 32.7, 7.2, vx=0.01, moves=True)], []]
    with pytest.raises(L.LBMError) as e:
        L.lbm_batch_workspace_bytes(grids, [0.8, 1.0], moving)
    assert "moves" in str(e.value)
    mixed = [L.make_grid(a, "f32"), L.make_grid(b, "f16")]
    with pytest.raises(L.LBMError) as e:
        L.lbm_batch_workspace_bytes(mixed, [0.8, 1.0], solids)
    assert "dtype" in str(e.value)
    with pytest.raises(L.LBMError):
        L.lbm_batch_workspace_bytes([], [], [])


def test_3d_workspace_holds_maps(L):
    """The 3D workspace holds the two population buffers (the second 1 MiB
    past the end of the first) and, per step parity, an owner map and a
    node-flag map of one byte per node of the padded lattice: the FP64 and
    FP32 workspaces differ by the populations alone, and what is not
    populations holds at least the four maps."""
    case = dict(nx=24, ny=20, nz=20, tau=0.7, duct=L.LBM3D_TUBE, R=8.0)
    nodes = 20 * 20 * 64  # lines x pitch
    n64, n32 = (L.lbm3d_workspace_bytes(L.make_grid3(case, d), (), 16) for d in ("f64", "f32"))
    assert n64 - n32 == 2 * 19 * nodes * 4
    assert n32 - (2 * 19 * nodes * 4 + (1 << 20)) >= 4 * nodes


def test_3d_validation(L):
    """lbm3d_workspace_bytes validates on the host (no device needed)."""
    tube = dict(nx=24, ny=20, nz=20, tau=0.7, duct=L.LBM3D_TUBE, R=8.0,
                spheres=[dict(cx=10.0, cy=9.5, cz=9.5, r=3.0)])

    def bytes_for(case, dtype="f64", hist=16):
        return L.lbm3d_workspace_bytes(L.make_grid3(case, dtype), case.get("spheres", ()), hist)

    n16 = bytes_for(tube)
    assert n16 > 2 * 19 * 20 * 20 * 64 * 8
    assert bytes_for(tube, hist=1000) > n16
    assert bytes_for(tube, "f32") < n16
    E = L.LBMError
    with pytest.raises(E):
        bytes_for(dict(tube, tau=0.5))
    g = L.make_grid3(tube)
    g.dtype = L.LBM_F16
    with pytest.raises(E):
        L.lbm3d_workspace_bytes(g, tube["spheres"], 16)
    with pytest.raises(E):  # the sphere reaches the tube wall
        bytes_for(dict(tube, spheres=[dict(cx=10.0, cy=15.5, cz=9.5, r=3.0)]))
    assert "sphere" in L.load_library().lbm3d_last_error(None).decode()
    with pytest.raises(E):  # two spheres overlap
        bytes_for(dict(tube, spheres=[dict(cx=10.0, cy=9.5, cz=9.5, r=2.5), dict(cx=13.0, cy=9.5, cz=9.5, r=2.5)]))
    with pytest.raises(E):  # link codes hold 2^27 nodes
        bytes_for(dict(nx=1024, ny=512, nz=256, tau=0.7))
    with pytest.raises(E):  # surface speed
        bytes_for(dict(tube, spheres=[dict(cx=10.0, cy=9.5, cz=9.5, r=3.0, v=(0.3, 0.0, 0.0))]))
    with pytest.raises(E):
        bytes_for(dict(tube, R=1.0))
