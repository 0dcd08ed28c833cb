"""sgs_bin_sort_noalloc (fixed per-device scratch, no allocation) against
sgs_bin_sort (caller's scratch), through the C ABI: instance count, sorted
keys and values, tile ranges and tile order bit-identical, on two calls in a
row (the second with a smaller input, so that whatever the first left in the
shared array must not leak into it), in both sort modes."""
import ctypes as C

import numpy as np
import pytest
import torch

import sgs_synth as S

pytestmark = pytest.mark.gpu


def _inputs(case):
    if case == "multiview":     # 2 views of 40k Gaussians: ~2.5M instances, ~35 MiB of scratch
        return S.blobs_scene(21, 40_000, 0), S.spline_poses(3, 3)[1:]
    if case == "tiny":
        sc, pose = S.tiny_config()
        return sc, [pose]
    sc = S.blobs_scene(5, 500, 1)  # smaller still, ragged image
    return sc, [S.Pose(S.look_at_gl((0.3, 0.2, 7.0), up=(0, 1, 0)), 97, 45)]


def _sort_both(case, mode):
    from paper_2605_18334_amd import _abi
    from paper_2605_18334_amd import raster as R
    lib = _abi.load()
    sc, poses = _inputs(case)
    opt = _abi.default_options(sort_mode=mode)
    gs = R.GaussianSet.from_scene(sc)
    cams = R.CameraBatch.from_poses(poses, opt)
    m = gs.n * cams.n_views
    geom, bufs = R.preprocess(gs, cams, opt)
    cap = int(bufs["block_off"][-1].item()) + 777          # exact count plus an unused tail
    need = int(lib.sgs_bin_sort_scratch_bytes(m, cap, cams.total_tiles, C.byref(opt)))
    print(f"case {case} mode {mode}: {m} records, capacity {cap}, scratch {need / 2**20:.1f} MiB", flush=True)
    assert need <= _abi.NOALLOC_SCRATCH_BYTES, "test case larger than the fixed scratch"
    outs = []
    for noalloc in (False, True):
        dev = bufs["depth"].device
        o = {"keys": torch.full((cap,), -1, dtype=torch.int64, device=dev),
             "vals": torch.full((cap,), -1, dtype=torch.int32, device=dev),
             "ranges": torch.full((2 * cams.total_tiles,), -1, dtype=torch.int32, device=dev),
             "n_inst": torch.full((1,), -1, dtype=torch.int32, device=dev),
             "order": torch.full((cams.total_tiles,), -1, dtype=torch.int32, device=dev)}
        sched = _abi.Schedule(o["order"].data_ptr(), None)
        args = (C.byref(geom), m, cams.host, cams.dev.data_ptr(), cams.n_views, C.byref(opt), cap,
                o["keys"].data_ptr(), o["vals"].data_ptr(), o["ranges"].data_ptr(), o["n_inst"].data_ptr(),
                C.byref(sched))
        stream = torch.cuda.current_stream().cuda_stream
        if noalloc:
            st = lib.sgs_bin_sort_noalloc(*args, stream)
        else:
            sb = int(lib.sgs_bin_sort_scratch_bytes(m, cap, cams.total_tiles, C.byref(opt)))
            o["scratch"] = torch.empty(sb, dtype=torch.uint8, device=dev)
            st = lib.sgs_bin_sort(*args, o["scratch"].data_ptr(), sb, stream)
        assert st == 0, _abi.STATUS.get(st, st)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in o.items() if k != "scratch"})
    a, b = outs
    n = int(a["n_inst"][0])
    assert 0 < n < cap and int(b["n_inst"][0]) == n
    np.testing.assert_array_equal(a["vals"][:n], b["vals"][:n])
    np.testing.assert_array_equal(a["keys"][:n], b["keys"][:n])
    np.testing.assert_array_equal(a["ranges"], b["ranges"])
    # the tile order is a permutation by list-length bucket; inside a bucket
    # the order is whatever the atomics gave, so compare the buckets' sets
    rg = a["ranges"].reshape(-1, 2).astype(np.int64)
    length = np.maximum(rg[:, 1] - rg[:, 0], 0)
    buckets = []
    for order in (a["order"], b["order"]):
        assert sorted(order.tolist()) == list(range(cams.total_tiles))
        buckets.append(_bucket(length[order]))
        assert (np.diff(buckets[-1]) <= 0).all()     # longest lists first
    np.testing.assert_array_equal(buckets[0], buckets[1])
    return n


def _bucket(length):
    """Quarter-octave length class: 0 for empty lists, else 1 + 4 floor(log2 len)
    + the two bits after the leading one."""
    out = np.zeros(len(length), np.int64)
    for i, x in enumerate(length.tolist()):
        if x:
            lg = x.bit_length() - 1
            frac = (x >> (lg - 2)) & 3 if lg >= 2 else (x << (2 - lg)) & 3
            out[i] = min(127, 1 + 4 * lg + frac)
    return out


@pytest.mark.parametrize("mode", [1, 0])
def test_noalloc_bin_sort_equals_bin_sort_on_consecutive_calls(mode):
    n_big = _sort_both("multiview", mode)
    n_small = _sort_both("tiny", mode)
    n_smaller = _sort_both("ragged", mode)
    assert n_big > 1_000_000 and n_big > n_small > n_smaller


def test_noalloc_rejects_sizes_beyond_its_array():
    """ECAPACITY before any work is enqueued when the scratch the sizes need
    exceeds the fixed array."""
    from paper_2605_18334_amd import _abi
    from paper_2605_18334_amd import raster as R
    lib = _abi.load()
    sc, pose = S.tiny_config()
    opt = _abi.default_options()
    gs = R.GaussianSet.from_scene(sc)
    cams = R.CameraBatch.from_poses([pose], opt)
    geom, bufs = R.preprocess(gs, cams, opt)
    cap = 200_000_000
    assert lib.sgs_bin_sort_scratch_bytes(gs.n, cap, cams.total_tiles, C.byref(opt)) > _abi.NOALLOC_SCRATCH_BYTES
    dummy = torch.zeros(16, dtype=torch.int32, device="cuda")
    st = lib.sgs_bin_sort_noalloc(C.byref(geom), gs.n, cams.host, cams.dev.data_ptr(), 1, C.byref(opt), cap,
                                  None, dummy.data_ptr(), dummy.data_ptr(), dummy.data_ptr(), None,
                                  torch.cuda.current_stream().cuda_stream)
    assert st == 2
    torch.cuda.synchronize()
