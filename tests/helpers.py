"""Shared test helpers: run the GPU path through the C ABI and the oracle on the same inputs."""
from __future__ import annotations

import numpy as np

# Parity bars: max |RGBA_gpu - RGBA_oracle| over non-fragile pixels for float32 storage (and
# for 16-bit storage against the oracle on the dequantised cube), and for 16-bit storage
# against the oracle on the original float32 cube.
TOL32 = 1e-5
TOL16 = 2e-3


AMP_MAX = 6.0
# Ill-conditioned pixels (amplification above AMP_MAX) still carry only rounding-level
# errors; this bound catches a wrong colour or weight on them.
COND_TOL = 1e-3


def margins(lo, hi, params=None, **kw):
    """Decision margins sized to the float32 path's errors (sample values within about
    1.2e-6 of the value range on average, up to ~1e-5 at steep gradients far from the
    origin): thresholds dv, ties ds, termination da.  The conditioning
    probe moves every sample by pv = 1e-7 of the range and flags pixels whose RGBA moves by
    more than AMP_MAX times the resulting change of s (a direct map through a table moves
    by its slope, <= 3); s moves by pv/(hi - lo), or pv/(max_t - min_t) under domain
    scaling.  Sample errors of the float32 path reach ~1.3e-6 in s, so amplification 6
    keeps robust pixels under the 1e-5 tolerance."""
    pv = 1e-7 * (hi - lo)
    slope = 1.0 / (hi - lo)
    if params and params.get("filter") == "scale":
        slope = 1.0 / (params["max_t"] - params["min_t"])
    m = dict(dv=1e-5 * (hi - lo), ds=1e-5, da=2e-6, pv=pv, pt=AMP_MAX * pv * slope)
    m.update(kw)
    return m


F32_KEYS = ("k", "min_val", "ert", "dt", "min_t", "max_t", "min_t2", "max_t2", "ratio_lo",
            "ratio_hi")


def f32(x):
    return float(np.float32(x))


def rounded(params):
    """Parameters as the GPU sees them (float32), for the oracle."""
    q = dict(params)
    for k in F32_KEYS:
        if k in q:
            q[k] = f32(q[k])
    if q.get("star"):
        c0, pairs = q["star"]
        q["star"] = (f32(c0), [(f32(o), f32(w)) for o, w in pairs])
    return q


def to_cuda(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_render(svr, vol, cam, lut_t, params, lo, hi, vol2=None):
    """Render through svr_render; returns (rgba[npix, 4] float64, samples[npix])."""
    q = dict(params)
    img, ns = svr.svr_render(vol, cam, lut_t, q, clim_lo=f32(lo), clim_hi=f32(hi), vol2=vol2,
                             samples=True)
    svr.svr_sync()
    return (img.cpu().numpy().reshape(-1, 4).astype(np.float64), ns.cpu().numpy().ravel())


def oracle_render(oracle, cube, cam, lut, params, lo, hi, cube2=None, pixels=None,
                  margins=None, forced_n=None, bits=False):
    q = rounded(params)
    q["lo"], q["hi"] = f32(lo), f32(hi)
    return oracle.render(cube, cam, lut, q, cube2=cube2, pixels=pixels, margins=margins,
                         forced_n=forced_n, bits=bits)


def compare_render(oracle, got, ns, cube, cam, lut, params, lo, hi, cube2=None, pixels=None,
                   margins=None, cond_tol=None):
    """Compare a GPU render with the oracle.

    Robust pixels must match.  A pixel whose only fragility is a near-threshold AVIP
    termination is re-rendered by the oracle with the GPU's stop index (the other valid
    reading of that decision) and must then match.  Pixels flagged only by the conditioning
    probe (continuous outputs, amplified sample errors) must stay within cond_tol when it is
    given.  Returns (max error, fragile mask after
    the re-check, number of near-threshold pixels re-checked)."""
    ref, bits, rns = oracle_render(oracle, cube, cam, lut, params, lo, hi, cube2, pixels,
                                   margins, bits=True)
    ert = (bits == oracle.FRAG_ERT)
    frag = bits != 0
    if ert.any():
        sel = np.nonzero(ert)[0]
        pix = sel if pixels is None else np.asarray(pixels)[sel]
        assert np.all(np.abs(ns[sel] - rns[sel]) <= 1)
        r2, b2, n2 = oracle_render(oracle, cube, cam, lut, params, lo, hi, cube2, pix,
                                   margins, forced_n=ns[sel], bits=True)
        assert np.array_equal(n2, ns[sel])
        ok = (b2 & ~np.uint8(oracle.FRAG_ERT)) == 0
        ref = ref.copy()
        ref[sel[ok]] = r2[ok]
        frag = frag.copy()
        frag[sel[ok]] = False
    assert_counts(ns, rns, frag | ert)
    if cond_tol is not None:
        cond = bits == oracle.FRAG_COND
        if cond.any():
            ec = float(np.abs(got[cond] - ref[cond]).max())
            print(f"  {int(cond.sum())} ill-conditioned pixels: max err {ec:.3e}", flush=True)
            assert ec <= cond_tol
    err = max_err(got, ref, frag)
    if err > 1e-5:
        ok = np.nonzero(~frag)[0]
        i = ok[np.argmax(np.abs(got[ok] - ref[ok]).max(axis=1))]
        pid = i if pixels is None else np.asarray(pixels)[i]
        print(f"  worst pixel {pid}: gpu {got[i]} oracle {ref[i]} samples {ns[i]}/{rns[i]} "
              f"bits {bits[i]}", flush=True)
    return err, frag, int(ert.sum())


def max_err(got, ref, fragile):
    ok = ~fragile
    if not ok.any():
        return 0.0
    return float(np.abs(got[ok] - ref[ok]).max())


def assert_counts(ns, rns, fragile):
    """Per-pixel sample counts agree exactly wherever no discrete decision is near a flip."""
    bad = (np.asarray(ns) != np.asarray(rns)) & ~np.asarray(fragile)
    assert not bad.any(), f"{bad.sum()} non-fragile pixels with different sample counts"
