"""Shared test helpers: run the GPU path through the C ABI and the oracle on the same inputs."""
from __future__ import annotations

import json
import os

import numpy as np

# Parity bars: max |RGBA_gpu - RGBA_oracle| over non-fragile pixels for float32 storage (and
# for 16-bit storage against the oracle on the dequantised cube), and for 16-bit storage
# against the oracle on the original float32 cube.
TOL32 = 1e-5
TOL16 = 2e-3


# Ill-conditioned pixels (see margins) still carry only rounding-level errors; this bound
# catches a wrong colour or weight on them.
COND_TOL = 1e-3


def margins(lo, hi, params=None, **kw):
    """Decision margins sized to the float32 path's errors.  Sample positions are formed in
    float64, so a sample value carries only the float32 trilinear blend's rounding: three
    lerps of exactly stored corners with fractions rounded once, at most about four ulp of
    the largest stored magnitude, ev = 4 * 2^-24 * max(|lo|, |hi|).  Thresholds: dv = 2e-6
    of the range (more than ten times ev on the test cubes); ties ds = 1e-5 in s;
    termination da = 2e-6 in alpha.  The conditioning probe moves every sample by
    pv = 1e-7 of the range in four patterns (all up, random signs, a ramp along the ray,
    opposite on the two cubes of a ratio); its largest RGBA change times ev/pv predicts the
    error that rounding of that size could cause, and a pixel is flagged (and then held to
    COND_TOL instead of the tolerance) when that prediction exceeds half the tolerance:
    pt = TOL32 pv / (2 ev)."""
    pv = 1e-7 * (hi - lo)
    ev = 4.0 * 2.0 ** -24 * max(abs(lo), abs(hi))
    m = dict(dv=2e-6 * (hi - lo), ds=1e-5, da=2e-6, pv=pv, pt=0.5 * TOL32 * pv / ev)
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
    reading of that decision) and must then match.  A MIP1 / MIP_RGB pixel whose only
    fragility is a near tie of the maximum must match the oracle's colour at one of the
    samples within the tie margin of the maximum (each a valid arg-max).  Pixels flagged
    only by the conditioning probe (continuous outputs, amplified sample errors) must stay
    within cond_tol when it is given.  Returns (max error, fragile mask after the
    re-checks, number of near-threshold pixels re-checked)."""
    ref, bits, rns = oracle_render(oracle, cube, cam, lut, params, lo, hi, cube2, pixels,
                                   margins, bits=True)
    ert = (bits == oracle.FRAG_ERT)
    frag = bits != 0
    ties = (bits == oracle.FRAG_ARGMAX) & (ns == rns)
    if params.get("mode") in ("mip1", "miprgb") and not params.get("ratio") and ties.any():
        ref, frag = recheck_ties(oracle, got, np.nonzero(ties)[0], rns, ref, frag, cube, cam,
                                 lut, params, lo, hi, pixels, margins)
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


def recheck_ties(oracle, got, sel, rns, ref, frag, cube, cam, lut, params, lo, hi, pixels,
                 margins):
    """Near ties of the MIP maximum: the oracle colours each pixel in `sel` once per sample
    taken as the arg-max; the GPU's colour must equal one whose sample lies within the tie
    margin of the maximum.  That candidate becomes the reference (still checked against
    the tolerance with every other pixel)."""
    ref, frag = ref.copy(), frag.copy()
    m = dict(margins or {}, pv=0.0, pp=0.0)
    matched = 0
    for i in sel:
        pid = int(i if pixels is None else np.asarray(pixels)[i])
        n = int(rns[i])
        cand, cb, _ = oracle_render(oracle, cube, cam, lut, params, lo, hi,
                                    pixels=np.full(n, pid), margins=m,
                                    forced_n=np.arange(n), bits=True)
        valid = (cb & np.uint8(oracle.NOT_CANDIDATE)) == 0
        assert valid.any()
        cand = cand[valid]
        d = np.abs(cand - got[i]).max(axis=1)
        j = int(np.argmin(d))
        ref[i] = cand[j]
        frag[i] = False
        matched += int(d[j] <= TOL32)
    print(f"  {len(sel)} near-tie pixels checked against every valid arg-max: {matched} "
          f"match one", flush=True)
    return ref, frag


def max_err(got, ref, fragile):
    ok = ~fragile
    if not ok.any():
        return 0.0
    return float(np.abs(got[ok] - ref[ok]).max())


def assert_counts(ns, rns, fragile):
    """Per-pixel sample counts agree exactly wherever no discrete decision is near a flip."""
    bad = (np.asarray(ns) != np.asarray(rns)) & ~np.asarray(fragile)
    assert not bad.any(), f"{bad.sum()} non-fragile pixels with different sample counts"


def report(kind, **record):
    """Append one JSON record to $SVR_REPORT_DIR/<kind>.jsonl when that variable is set (the
    per-configuration error tables are read from these records)."""
    d = os.environ.get("SVR_REPORT_DIR")
    if not d:
        return
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, f"{kind}.jsonl"), "a") as f:
        f.write(json.dumps(record) + "\n")
