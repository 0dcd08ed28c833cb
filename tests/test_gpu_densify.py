"""Densification step on the GPU (sgs_densify) against the oracle: decisions
bit-exact (both sides decide in float32), the new set's size and parent
indices exact, copied attributes bit-identical, split children within
float32 rounding of the FP64 oracle.  Statistics are seeded inputs (with
values placed on and around the thresholds), fed to both sides."""
import numpy as np
import pytest
import torch

import sgs_synth as S
from oracle import sgs_oracle as O

pytestmark = pytest.mark.gpu


def _stats(rng, n):
    cnt = rng.integers(0, 4, n).astype(np.uint32)
    uv = (np.float32(0.001) * cnt * rng.uniform(0.5, 1.6, n)).astype(np.float32)
    uv[::17] = np.float32(0.001) * cnt[::17]           # exactly on the threshold (float32)
    z = rng.uniform(0.0, 0.0016, n).astype(np.float32)
    z[::13] = np.float32(0.001)
    return uv, cnt, z


@pytest.mark.parametrize("case", ["skew_sh2", "symmetric_enhanced"])
def test_densify_matches_oracle(case):
    import paper_2605_18334_amd as P
    rng = np.random.default_rng(31)
    if case == "skew_sh2":
        sc = S.blobs_scene(8, 5000, 2)
    else:
        sc = S.blobs_scene(9, 3000, 1, enhanced=True)
        sc = S.Scene(sc.mean, sc.log_scale, sc.quat, None, sc.opa_logit, sc.sh, sc.sh_degree,
                     sc.opa2_logit, sc.opa_dir)
    # largest scale below 0.01 for about half (cloned when selected), above for the rest (split)
    sc.log_scale[:] = np.log(rng.uniform(0.001, 0.012, sc.log_scale.shape)).astype(np.float32)
    sc.log_scale[0, ::11] = np.float32(np.log(0.01))     # largest scale exactly at the split bound
    uv, cnt, z = _stats(rng, sc.n)
    gs = P.GaussianSet.from_scene(sc)
    st = {"uv": torch.from_numpy(uv).cuda(), "count": torch.from_numpy(cnt.view(np.int32)).cuda(),
          "z": torch.from_numpy(z).cuda()}
    new, dec, parent = P.densify(gs, st)
    torch.cuda.synchronize()
    ref_d = O.densify_decisions(sc.log_scale, uv, cnt, z)
    got_d = dec.cpu().numpy().astype(np.int8)
    np.testing.assert_array_equal(got_d, ref_d)
    assert (ref_d == 1).sum() > 100 and (ref_d == 2).sum() > 100 and (ref_d == 0).sum() > 100
    ref = O.densify(sc, ref_d)
    np.testing.assert_array_equal(parent.cpu().numpy(), ref["parent"])
    assert new.n == len(ref["parent"]) == sc.n + int((ref_d > 0).sum())
    split = np.repeat(ref_d, np.where(ref_d > 0, 2, 1)) == 2
    for f in ("mean", "log_scale"):
        g = getattr(new, f).cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(g[:, ~split], ref[f][:, ~split].astype(np.float32))
        np.testing.assert_allclose(g[:, split], ref[f][:, split], rtol=1e-5, atol=2e-6, err_msg=f)
    for f in ("quat", "skew", "opa_logit", "opa2_logit", "opa_dir", "sh"):
        if ref[f] is None:
            assert getattr(new, f) is None
            continue
        np.testing.assert_array_equal(getattr(new, f).cpu().numpy(), ref[f].astype(np.float32), err_msg=f)


def test_densify_without_statistics_keeps_everything_and_fits_capacity():
    import paper_2605_18334_amd as P
    sc = S.blobs_scene(4, 700, 0)
    gs = P.GaussianSet.from_scene(sc)
    new, dec, parent = P.densify(gs, None)
    torch.cuda.synchronize()
    assert (dec.cpu().numpy() == 0).all() and new.n == sc.n
    np.testing.assert_array_equal(new.mean.cpu().numpy(), sc.mean)
    # a capacity smaller than the output drops the tail, never writes past it
    rng = np.random.default_rng(2)
    uv, cnt, z = _stats(rng, sc.n)
    st = {"uv": torch.from_numpy(uv).cuda(), "count": torch.from_numpy(cnt.view(np.int32)).cuda(),
          "z": torch.from_numpy(z).cuda()}
    full, _, _ = P.densify(gs, st)
    part, _, pp = P.densify(gs, st, capacity=sc.n // 2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(part.mean.cpu().numpy(), full.mean[:, :sc.n // 2].cpu().numpy())
