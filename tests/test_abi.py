"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every symbol include/sgs.h declares, its struct sizes match the binding, and
the host helpers (CoordEngine, layout, sizes, argument checks) behave."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import sgs_synth as S
from oracle import sgs_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2605_18334_amd import _abi
    return _abi, _abi.load()


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "sgs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgs_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    _abi, lib = _lib()
    names = _declared_symbols()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
        assert n in _abi.SIGNATURES, f"binding lacks {n}"


def test_struct_sizes_match_binding():
    _abi, lib = _lib()
    for i, s in enumerate(_abi.STRUCTS):
        assert lib.sgs_struct_size(i) == C.sizeof(s), s.__name__
    assert lib.sgs_struct_size(99) == 0


def test_default_options_and_status_strings():
    _abi, lib = _lib()
    o = _abi.default_options()
    assert (o.tile_w, o.tile_h, o.blend_batch, o.sort_mode, o.compensate) == (16, 16, 0, -1, 1)
    assert o.split_tiles == -1 and o.depth_digit_bits == 0 and o.blend_lists == 0
    assert o.alpha_min == pytest.approx(1 / 255) and o.alpha_max == pytest.approx(0.99)
    assert o.t_min == pytest.approx(1e-4) and o.filter_s == pytest.approx(0.3)
    assert lib.sgs_status_string(0) == b"ok"
    assert lib.sgs_status_string(1) == b"invalid argument"


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_camera_from_gl_matches_oracle_coord_engine(seed):
    """The library's CoordEngine/K (float32 out) equals the oracle's FP64
    M_cv = M_gl T_align, w2c = M_cv^-1, K."""
    from paper_2605_18334_amd.raster import CameraBatch
    rng = np.random.default_rng(seed)
    pose = S.random_request_pose(rng)
    cam = CameraBatch.camera_from_pose(pose)
    ref = O.camera_from_pose(pose)
    w2c = np.array(list(cam.w2c)).reshape(3, 4)
    np.testing.assert_allclose(w2c, ref.w2c[:3], rtol=0, atol=2e-6 * max(1.0, np.abs(ref.w2c).max()))
    np.testing.assert_allclose([cam.fx, cam.fy, cam.cx, cam.cy],
                               [ref.K[0, 0], ref.K[1, 1], ref.K[0, 2], ref.K[1, 2]], rtol=1e-6)
    np.testing.assert_allclose(list(cam.campos), ref.position, atol=1e-5)
    assert (cam.width, cam.height) == (pose.width, pose.height)


def test_camera_from_gl_rejects_bad_input():
    _abi, lib = _lib()
    cam = _abi.Camera()
    m = (C.c_double * 16)(*np.eye(4).reshape(-1))
    assert lib.sgs_camera_from_gl(m, 0, 10, 1.0, 0.0, 0.2, None, C.byref(cam)) == 1
    assert lib.sgs_camera_from_gl(m, 10, 10, 0.0, 0.0, 0.2, None, C.byref(cam)) == 1
    bad = (C.c_double * 16)(*([float("nan")] + [0.0] * 15))
    assert lib.sgs_camera_from_gl(bad, 10, 10, 1.0, 0.0, 0.2, None, C.byref(cam)) == 1
    sing = (C.c_double * 16)(*np.zeros(16))
    assert lib.sgs_camera_from_gl(sing, 10, 10, 1.0, 0.0, 0.2, None, C.byref(cam)) == 1


def test_camera_layout_tiles_and_pixels():
    _abi, lib = _lib()
    from paper_2605_18334_amd.raster import CameraBatch
    poses = S.spline_poses(5, 4)
    cams = [CameraBatch.camera_from_pose(p) for p in poses]
    arr = (_abi.Camera * 4)(*cams)
    for tw, th in [(16, 16), (16, 8), (8, 8)]:
        o = _abi.default_options(tile_w=tw, tile_h=th)
        tt, tp = C.c_int64(), C.c_int64()
        assert lib.sgs_camera_layout(arr, 4, C.byref(o), C.byref(tt), C.byref(tp)) == 0
        exp_t = sum(-(-p.width // tw) * -(-p.height // th) for p in poses)
        assert tt.value == exp_t and tp.value == sum(p.width * p.height for p in poses)
        base = 0
        for v in range(4):
            assert arr[v].tile_base == base
            base += arr[v].tiles_x * arr[v].tiles_y
    o = _abi.default_options(tile_w=12)
    assert lib.sgs_camera_layout(arr, 4, C.byref(o), None, None) == 1


def test_size_helpers():
    _abi, lib = _lib()
    assert lib.sgs_geom_rec_floats(10, 0) == 160 and lib.sgs_geom_rec_floats(10, 1) == 160   # 64 B per record
    assert lib.sgs_geom_block_entries(300, 2) == 2 * 2 + 1
    o = _abi.default_options()
    a = lib.sgs_bin_sort_scratch_bytes(1000, 5000, 64, C.byref(o))
    b = lib.sgs_bin_sort_scratch_bytes(1000, 50000, 64, C.byref(o))
    assert 0 < a < b


def test_entry_points_reject_null_arguments_without_gpu():
    """Argument checks happen before any HIP call."""
    _abi, lib = _lib()
    o = _abi.default_options()
    g = _abi.Geom()
    p = _abi.Params()
    p.n = -1
    assert lib.sgs_preprocess(C.byref(p), None, None, 1, C.byref(o), C.byref(g), None) == 1
    assert lib.sgs_bin_sort(None, 0, None, None, 1, C.byref(o), 0, None, None, None, None, None, None, 0,
                            None) == 1
    assert lib.sgs_render_fwd(None, 0, None, 0, None, None, None, None, 1, 0, C.byref(o), None, None, None,
                              None, None, 0, None) == 1
    assert lib.sgs_render_bwd(None, None, 0, None, 0, None, None, None, None, 1, C.byref(o), None, None, None,
                              0, None, None, None) == 1


def test_options_are_validated_on_the_host():
    """sgs_camera_layout checks the options (no GPU needed): unsupported tile
    shapes, LDS batches, sort modes and split counts are rejected."""
    _abi, lib = _lib()
    cams = (_abi.Camera * 1)()
    cams[0].width, cams[0].height = 64, 48
    tt, tp = C.c_int64(), C.c_int64()
    ok = _abi.default_options()
    assert lib.sgs_camera_layout(cams, 1, C.byref(ok), C.byref(tt), C.byref(tp)) == 0
    assert (tt.value, tp.value) == (4 * 3, 64 * 48)
    for bad in (dict(tile_w=32), dict(blend_batch=100), dict(sort_mode=3), dict(sort_mode=-2), dict(split_tiles=-2),
                dict(alpha_min=0.0), dict(t_min=1.0), dict(depth_digit_bits=11), dict(blend_lists=2)):
        o = _abi.default_options(**bad)
        assert lib.sgs_camera_layout(cams, 1, C.byref(o), C.byref(tt), C.byref(tp)) == 1, bad


def test_missing_library_fails_loudly():
    """No fallback: in a fresh interpreter, loading a library that is not
    there raises instead of handing back a substitute."""
    import subprocess
    import sys
    code = ("from paper_2605_18334_amd import _abi\n"
            "try:\n"
            "    _abi.load('/nonexistent/libsgs.so')\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    raise SystemExit('no error for a missing library')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "raised:" in r.stdout and "missing" in r.stdout


def test_package_never_reaches_the_oracle():
    """The product path has no route into the CPU oracle: no source file of
    the package imports, loads or names it."""
    pkg = os.path.join(ROOT, "paper_2605_18334_amd")
    found = []
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp", ".c")):
                text = open(os.path.join(dirpath, f), errors="replace").read()
                if re.search(r"\boracle\b", text):
                    found.append(os.path.relpath(os.path.join(dirpath, f), ROOT))
    assert not found, found


def test_bin_sort_mode_choice_on_the_host():
    """sgs_bin_sort_mode (no GPU): auto picks row binning from 3 * 2^17 instances
    of capacity, the tile-key sort below; row binning needs the row counts,
    at most 256 tiles per row and 1024 tile rows, else the tile-key sort
    runs; explicit modes are kept; bad arguments give -1."""
    _abi, lib = _lib()
    o = _abi.default_options()
    cams = (_abi.Camera * 2)()
    for k in range(2):
        cams[k].width, cams[k].height, cams[k].fx, cams[k].fy = 1600, 1064, 900.0, 900.0
    tt, tp = C.c_int64(), C.c_int64()
    assert lib.sgs_camera_layout(cams, 2, C.byref(o), C.byref(tt), C.byref(tp)) == 0
    big, small = 3 << 17, (3 << 17) - 1
    assert lib.sgs_bin_sort_mode(C.byref(o), big, cams, 2, 1) == 2
    assert lib.sgs_bin_sort_mode(C.byref(o), small, cams, 2, 1) == 1
    assert lib.sgs_bin_sort_mode(C.byref(o), big, cams, 2, 0) == 1          # no row counts
    for mode in (0, 1, 2):
        assert lib.sgs_bin_sort_mode(C.byref(_abi.default_options(sort_mode=mode)), 1000, cams, 2, 1) == mode
    wide = (_abi.Camera * 1)()
    wide[0].width, wide[0].height, wide[0].fx, wide[0].fy = 4112, 64, 900.0, 900.0   # 257 tiles per row
    assert lib.sgs_camera_layout(wide, 1, C.byref(o), C.byref(tt), C.byref(tp)) == 0
    assert lib.sgs_bin_sort_mode(C.byref(o), big, wide, 1, 1) == 1
    tall = (_abi.Camera * 1)()
    tall[0].width, tall[0].height, tall[0].fx, tall[0].fy = 64, 16400, 900.0, 900.0  # 1025 tile rows
    assert lib.sgs_camera_layout(tall, 1, C.byref(o), C.byref(tt), C.byref(tp)) == 0
    assert lib.sgs_bin_sort_mode(C.byref(o), big, tall, 1, 1) == 1
    assert lib.sgs_bin_sort_mode(C.byref(_abi.default_options(sort_mode=5)), big, cams, 2, 1) == -1
    assert lib.sgs_bin_sort_mode(C.byref(o), -1, cams, 2, 1) == -1
