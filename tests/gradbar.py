"""The gradient bar of the parity tests (a helper module, not a test file)."""
import numpy as np


def compare_grads(got: dict, ref: dict, rtol=1e-2, floor=1e-3, maxes=None, norms=None, label=""):
    """The gradient bar: per tensor, relative L2 error <= rtol; per element,
    relative error <= rtol wherever |g| > floor * max |g| of that tensor
    (maxes / norms: the tensor's max and L2 norm over all Gaussians, when
    got / ref hold a sample of them)."""
    res = {}
    for k, rv in ref.items():
        gv = np.asarray(got[k], np.float64).reshape(rv.shape)
        rel = np.linalg.norm(gv - rv) / max(np.linalg.norm(rv), 1e-30)
        gmax = np.abs(rv).max() if maxes is None else maxes[k]
        big = np.abs(rv) > floor * gmax
        e = np.abs(gv - rv)[big] / np.abs(rv)[big] if big.any() else np.zeros(1)
        res[k] = (rel, float(e.max()))
        print(f"{label} {k}: rel L2 {rel:.2e}, {int(big.sum())} elements above {floor:g} x max, "
              f"worst element {e.max():.2e}", flush=True)
        assert rel <= rtol, (k, rel)
        assert e.max() <= rtol, (k, e.max())
    return res
