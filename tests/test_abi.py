"""Host-side checks of the C ABI: the library loads, exports every symbol include/lbpf.h
declares, and validates parameters before any device work (no GPU calls here)."""
import ctypes
import os
import re

import pytest

from paper_1902_08933_amd import lbpf, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbpf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbpf[0-9a-z]*_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbpf.LIB_PATH):
        from paper_1902_08933_amd import build
        build.build()
    return lbpf.library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 19
    for name in names:
        assert hasattr(lib, name), name
    # and the binding knows the signature of each
    assert set(names) == set(lbpf.SIGNATURES)


def test_params_struct_layout_matches_header():
    # 8 int32 fields then 11 doubles, no padding
    assert ctypes.sizeof(lbpf.Params) == 8 * 4 + 11 * 8
    assert ctypes.sizeof(lbpf.Diag) == 3 * 8 + 2 * 8


def test_workspace_size_scales_with_grid(lib):
    cfg, _ = workloads.static_droplet(n=64)
    a = lbpf.workspace_size(cfg)
    b = lbpf.workspace_size(dict(cfg, nx=128, ny=128))
    # two population copies of 21 planes (f_1..8, h hi/lo pair and h_1..8, p, phi u), rows of
    # planes 64 + 32 floats apart (short rows), and the FP64 scratch of ny * pitch doubles; the
    # layout pad and the reduction area do not depend on the grid size
    def grid_floats(n):
        return 2 * 21 * n * (n + 32) + 2 * n * n
    assert b - a == 4 * (grid_floats(128) - grid_floats(64))


@pytest.mark.parametrize("bad,why", [
    (dict(nx=2), "nx and ny"),
    (dict(ny=1), "nx and ny"),
    (dict(tau_h=0.5), "tau_h"),
    (dict(nu_A=0.0), "nu_A"),
    (dict(rho_B=-1.0), "rho_A and rho_B"),
    (dict(W=0.0), "W must"),
    (dict(sigma=-0.1), "sigma"),
    (dict(variant="qim", force_x=float("nan")), "finite"),
    # in-plane offsets are 32-bit byte offsets and row offsets use a 24-bit multiply
    (dict(nx=1 << 24, ny=3), "below 2^24"),
    (dict(nx=32768, ny=32768), "2^30"),
])
def test_invalid_parameters_rejected(lib, bad, why):
    cfg, _ = workloads.static_droplet(n=16, R=4)
    cfg = dict(cfg, **bad)
    with pytest.raises(lbpf.LbpfError) as ei:
        lbpf.workspace_size(cfg)
    assert ei.value.status == -1
    assert why in str(ei.value)


def test_largest_plane_accepted(lib):
    # 32768 x 32704 nodes (plus the layout pad) stays below 2^30 floats per plane; planes of a
    # grid this large are stored separately (interleaved, a copy would exceed 2^30 floats)
    cfg, _ = workloads.static_droplet(n=16, R=4)
    assert lbpf.workspace_size(dict(cfg, nx=32768, ny=32704)) > 44 * 4 * 32768 * 32704


def test_planar_layout_size(lib, monkeypatch):
    # separate planes carry one layout pad per plane; interleaved copies one per copy, and their
    # short rows 32 floats more per plane
    cfg, _ = workloads.static_droplet(n=64)
    inter = lbpf.workspace_size(cfg)
    monkeypatch.setenv("LBPF_STATE_LAYOUT", "planar")
    planar = lbpf.workspace_size(cfg)
    assert planar - inter == (2 * 20 * 4160 - 2 * 21 * 64 * 32) * 4


def test_status_strings(lib):
    for s in (0, -1, -2, -3, -4, -5):
        assert lib.lbpf_status_string(s)
    assert lib.lbpf_destroy(None) == 0
    assert lib.lbpf_step_count(None) == -1


def test_create_rejects_null_workspace(lib):
    cfg, _ = workloads.static_droplet(n=16, R=4)
    h = ctypes.c_void_p()
    st = lib.lbpf_create(ctypes.byref(lbpf.make_params(cfg)), None, 0, None, ctypes.byref(h))
    assert st == -1 and not h.value
    assert b"workspace" in lib.lbpf_create_error()


def test_tile_shapes_listed(lib):
    shapes = lbpf.tile_shapes()
    assert len(shapes) >= 4
    for tx, rows, nt in shapes:
        assert nt % tx == 0 and nt // tx >= 2 and rows % (nt // tx) == 0


def test_params3d_struct_layout_matches_header():
    # 10 int32 fields then 12 doubles, no padding
    assert ctypes.sizeof(lbpf.Params3D) == 10 * 4 + 12 * 8


def _cfg3d(**kw):
    c = dict(nx=64, ny=48, nz=40, rho_A=3, rho_B=1, nu_A=0.01, nu_B=0.1, sigma=0.03, W=4,
             M_phi=0.01, tau_h=1)
    c.update(kw)
    return c


def test_workspace3d_size(lib):
    n = ctypes.c_size_t()
    p = lbpf.make_params3d(_cfg3d())
    assert lib.lbpf3d_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    # two population copies of 34 planes (g_1..14, h hi/lo pair and h_1..14, p, phi u), planes
    # interleaved by row 64 + 32 floats apart, one layout pad per copy, then the reduction area
    copy = 34 * 40 * 48 * (64 + 32) + 4160
    assert 2 * copy * 4 <= n.value < 2 * copy * 4 + 256 + 8 * (2048 * 4 + 64)


@pytest.mark.parametrize("bad", [dict(nz=2), dict(nx=1 << 24), dict(tau_h=0.5), dict(nu_A=0.0),
                                 dict(bc=2), dict(nx=1024, ny=1024, nz=1024), dict(W=0.0)])
def test_invalid_3d_parameters_rejected(lib, bad):
    cfg = _cfg3d(**{k: v for k, v in bad.items() if k != "bc"})
    p = lbpf.make_params3d(cfg)
    if "bc" in bad:
        p.bc = bad["bc"]
    n = ctypes.c_size_t()
    assert lib.lbpf3d_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1
    assert lib.lbpf3d_last_error(None)
    h = ctypes.c_void_p()
    assert lib.lbpf3d_create(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_size_t(1 << 40), None,
                             ctypes.byref(h)) == -1
    assert not h.value


def test_create3d_rejects_small_or_null_workspace(lib):
    p = lbpf.make_params3d(_cfg3d())
    h = ctypes.c_void_p()
    assert lib.lbpf3d_create(ctypes.byref(p), None, ctypes.c_size_t(1 << 40), None, ctypes.byref(h)) == -1
    assert lib.lbpf3d_create(ctypes.byref(p), ctypes.c_void_p(256), ctypes.c_size_t(1024), None,
                             ctypes.byref(h)) == -3
    assert not h.value


def test_shapes3d_listed(lib):
    shapes = lbpf.shapes3d()
    assert len(shapes) >= 4 and all(tx * ty in (256, 512) for tx, ty, _ in shapes)
    assert lib.lbpf3d_shape_info(len(shapes), None, None, None) == -1


def test_long_rows_fall_back_to_separate_planes(lib):
    # Row offsets y * pitch use the 24-bit multiplier. At nx = 800000 an interleaved copy would
    # have a row stride of 21 * 800000 = 16.8 M floats >= 2^24 (but only 52.9 M floats per copy,
    # well below 2^30), so the layout must be separate planes, whose row stride is 800000.
    cfg, _ = workloads.static_droplet(n=16, R=4)
    nx, ny = 800000, 63
    got = lbpf.workspace_size(dict(cfg, nx=nx, ny=ny))
    red = 8 * (4096 * 8 + 64)
    planar = (2 * 21 * (ny * nx + 4160) + 2 * ny * nx) * 4 + red
    interleaved = (2 * (21 * ny * nx + 4160) + 2 * ny * nx) * 4 + red
    assert got == planar != interleaved
    # the largest row stride an interleaved copy may have: 21 * 798912 < 2^24 <= 21 * 798976
    for nx, inter in ((798912, True), (798976, False)):
        got = lbpf.workspace_size(dict(cfg, nx=nx, ny=ny))
        expect = ((2 * (21 * ny * nx + 4160) if inter else 2 * 21 * (ny * nx + 4160))
                  + 2 * ny * nx) * 4 + red
        assert got == expect, nx


def test_row_pitch_of_2_pow_24_rejected(lib):
    # nx = 2^24 - 10 rounds up to a pitch of 2^24, whose low 24 bits are 0
    cfg, _ = workloads.static_droplet(n=16, R=4)
    with pytest.raises(lbpf.LbpfError) as ei:
        lbpf.workspace_size(dict(cfg, nx=(1 << 24) - 10, ny=3))
    assert ei.value.status == -1 and "2^24" in str(ei.value)
    p = lbpf.make_params3d(_cfg3d(nx=(1 << 24) - 10, ny=3, nz=3))
    n = ctypes.c_size_t()
    assert lib.lbpf3d_workspace_size(ctypes.byref(p), ctypes.byref(n)) == -1


def test_long_rows_3d_fall_back_to_separate_planes(lib):
    # D3Q15 copies interleave 34 planes per row, (pitch + 32) floats apart: 34 * (493440 + 32)
    # = 16.78 M floats >= 2^24, so a 493440-wide grid is stored as separate planes
    def size(nx):
        n = ctypes.c_size_t()
        p = lbpf.make_params3d(_cfg3d(nx=nx, ny=3, nz=3))
        assert lib.lbpf3d_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
        return n.value
    for nx, inter in ((493376, True), (493440, False)):
        rows = 9
        copy = 34 * rows * (nx + 32) + 4160 if inter else 34 * (rows * nx + 4160)
        assert 2 * copy * 4 <= size(nx) < 2 * copy * 4 + 256 + 8 * (2048 * 4 + 64), nx
