"""The image bar of the parity tests (a helper module, not a test file)."""
import numpy as np

IMG_TOL = 1e-4

AMB_TOL = 2e-2   # pixels with an uncertain decision and no enumerated outcomes


def check_image_values(got, gT, ref, tol=IMG_TOL, max_amb=0.01, extra=None):
    """got [P,3], gT [P] at ref.pixels against the oracle: unambiguous pixels
    within tol; an ambiguous pixel within tol of one of the oracle's outcomes
    of its uncertain decisions (each taken either way), or within AMB_TOL
    when the oracle listed none.  extra: optional per-pixel (bound_C [P,3],
    bound_T [P]) added to tol."""
    amb = ref.ambiguous
    ok = ~amb
    err = np.abs(got - ref.color)
    terr = np.abs(gT - ref.T)
    if extra is not None:
        err = err - extra[0]
        terr = terr - extra[1]
    err = np.maximum(err.max(1), terr)
    alt_err = np.full(len(err), np.inf)
    for q in np.nonzero(amb)[0]:
        rows = ref.alt_rows[ref.alt_start[q]:ref.alt_start[q + 1]] if ref.alt_start is not None else []
        if len(rows):
            e = np.maximum(np.abs(rows[:, :3] - got[q]).max(1), np.abs(rows[:, 3] - gT[q]))
            if extra is not None:
                e = e - max(extra[0][q].max(), extra[1][q])
            alt_err[q] = e.min()
    listed = amb & np.isfinite(alt_err)
    loose = amb & ~listed
    print(f"image check: {len(err)} pixels, {amb.mean():.5f} ambiguous ({int(amb.sum())}: {int(listed.sum())} "
          f"against their outcomes, {int(loose.sum())} loosely), max err {err[ok].max(initial=0):.2e}"
          f"{'' if not listed.any() else f', ambiguous max err {alt_err[listed].max():.2e}'}", flush=True)
    assert amb.mean() <= max_amb, f"{amb.mean():.4f} of pixels ambiguous"
    worst = int(np.argmax(np.where(ok, err, 0)))
    assert err[ok].max(initial=0) <= tol, (
        f"max err {err[ok].max():.3e} at pixel {ref.pixels[worst]} got {got[worst]} ref {ref.color[worst]}")
    assert alt_err[listed].max(initial=0) <= tol, alt_err[listed].max()
    assert np.abs(got - ref.color).max(1)[loose].max(initial=0) <= AMB_TOL
    return err
