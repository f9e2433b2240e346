"""Pins of the FP64 oracle against facts the paper and the mathematics fix (CPU only).

Each test names the passage it pins.  None of them re-types the oracle's own recurrence:
they use closed forms, library routines (scipy's trilinear interpolation and 1D
correlation, numpy's binary16 cast, torch's bfloat16 cast), invariants and brute force.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth
from oracle import taps, quant

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def scipy_trilinear(cube, pts):
    """Library trilinear interpolation, clamp-to-edge, at points (N, 3) given as (x, y, z)."""
    coords = np.stack([pts[:, 2], pts[:, 1], pts[:, 0]])  # order [z][y][x]
    return ndimage.map_coordinates(np.asarray(cube, np.float64), coords, order=1,
                                   mode="nearest")


def norm01(v, lo, hi):
    return np.clip((v - lo) / (hi - lo), 0.0, 1.0)


def ortho_z_samples(n, width, height, dt=0.5):
    """Sample positions of an axis-aligned parallel projection along +z through an n^3
    cube whose image spans one face (closed form: z = -0.5 + k dt, k < n/dt)."""
    px, py = np.meshgrid(np.arange(width), np.arange(height), indexing="xy")
    x = (n - 1) / 2.0 + (2.0 * (px + 0.5) / width - 1.0) * n / 2.0
    y = (n - 1) / 2.0 + (2.0 * (py + 0.5) / height - 1.0) * n / 2.0
    zs = -0.5 + dt * np.arange(int(round(n / dt)))
    return x.ravel(), y.ravel(), zs


# ------------------------------------------------------------------ trilinear, ray/box
def test_trilinear_matches_library_interpolation():
    """The fetch cube[loc] (Alg. 1) is trilinear with clamp-to-edge: equal to scipy's
    order-1 map_coordinates with mode 'nearest' at random points, in and outside."""
    rng = np.random.default_rng(3)
    cube = rng.standard_normal((7, 9, 11))
    pts = rng.uniform(-2.0, 13.0, size=(500, 3))
    ref = scipy_trilinear(cube, pts)
    got = np.array([oracle.trilinear(cube, p) for p in pts])
    assert np.max(np.abs(got - ref)) < 1e-12


def test_ray_box_entry_on_surface_and_chord_by_bruteforce():
    """Appendix A rays against the cell-centred box [-0.5, n-0.5]^3: the entry point lies
    on the box surface and the chord length agrees with dense brute-force sampling."""
    rng = np.random.default_rng(5)
    n = (6, 9, 13)  # (nz, ny, nx)
    hi = np.array([n[2], n[1], n[0]]) - 0.5
    hits = 0
    for _ in range(200):
        o = rng.uniform(-15, 25, 3)
        target = rng.uniform(-1.0, 1.0, 3) * (hi + 1.0)
        d = (target - o) if rng.random() < 0.75 else rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = oracle.ray_box(n, o, d)
        ts = np.linspace(0, 60, 600001)
        pts = o[None] + ts[:, None] * d[None]
        inside = np.all((pts >= -0.5) & (pts <= hi[None]), axis=1)
        if r is None:
            assert inside.sum() <= 1
            continue
        hits += 1
        t0, t1 = r
        assert abs((t1 - t0) - inside.sum() * 1e-4) < 3e-4
        p0 = o + t0 * d
        if t0 > 0:
            on_face = np.isclose(p0, -0.5, atol=1e-9) | np.isclose(p0, hi, atol=1e-9)
            assert on_face.any()
    assert hits > 40


# ------------------------------------------------------------------ MIP pins (P2-P4)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mip0_axis_aligned_is_column_max(seed):
    """Eq. MIP along z with one ray per voxel column (64x64 image on a 64^3 cube): the
    result is colourMap(max_z V) exactly (trilinear weights are 0/1 or clamp)."""
    cube = synth.blob_cube_64(seed)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.ortho_axis(64, 64, 64, 64, 64, "+z")
    lut = synth.lut_heat(256)
    rgba, frag, ns = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi))
    assert (ns == 128).all() and not frag.any()
    s = norm01(cube.astype(np.float64).max(axis=0).ravel(), lo, hi)
    for ch in range(4):
        ref = np.interp(s, np.arange(256) / 255.0, lut[:, ch].astype(np.float64))
        assert np.max(np.abs(rgba[:, ch] - ref)) < 1e-12


def test_mip0_oversampled_matches_library_trilinear_max():
    """256x256 rays over a 64^3 cube: MIP0 equals the max over library-interpolated samples
    at the closed-form sample positions z = -0.5 + 0.5 k, k = 0..127."""
    cube = synth.blob_cube_64(0)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.ortho_axis(64, 64, 64, 256, 256, "+z")
    lut = synth.lut_ramp(256)
    x, y, zs = ortho_z_samples(64, 256, 256)
    pix = np.random.default_rng(0).choice(256 * 256, 400, replace=False)
    rgba, _, ns = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi), pixels=pix)
    assert (ns == 128).all()
    for i, p in enumerate(pix):
        pts = np.stack([np.full_like(zs, x[p]), np.full_like(zs, y[p]), zs], 1)
        s = norm01(scipy_trilinear(cube, pts).max(), lo, hi)
        ref = np.interp(s, np.arange(256) / 255.0, lut[:, 0].astype(np.float64))
        assert abs(rgba[i, 0] - ref) < 1e-12


def test_mip1_and_rgb_use_last_argmax_and_loc():
    """Alg. MIP1 / MIP_RGB: the colour comes from the location of the maximum, the later
    sample winning ties ('>='); loc = (p + 0.5)/n.  Built with planted exact ties."""
    rng = np.random.default_rng(11)
    n = 16
    cube = rng.uniform(0, 1, (n, n, n)).astype(np.float32)
    # plant an exact tie of the column maximum at two depths in every column
    cube[3] = 2.0
    cube[9] = 2.0
    lut = synth.lut_heat(64)
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    p = dict(lo=0.0, hi=2.0)
    m1, f1, _ = oracle.render(cube, cam, lut, dict(p, mode="mip1"))
    rgb, f2, _ = oracle.render(cube, cam, lut, dict(p, mode="miprgb"))
    # samples at z = 8.5 and 9.0 both read 2.0?  No: 8.5 interpolates planes 8 and 9.
    zstar = 9.0  # last sample reaching the maximum is the one at z = 9
    locz = (zstar + 0.5) / n
    refc = [np.interp(locz, np.arange(64) / 63.0, lut[:, ch].astype(np.float64)) for ch in range(3)]
    assert np.allclose(m1[:, :3], np.array(refc)[None], atol=1e-12)
    assert np.allclose(m1[:, 3], 1.0)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    assert np.allclose(rgb[:, 0], locz)
    assert np.allclose(rgb[:, 1], ((yy + 0.5) / n).ravel())
    assert np.allclose(rgb[:, 2], ((xx + 0.5) / n).ravel())
    assert np.allclose(rgb[:, 3], 1.0)


def test_mirror_views_give_mirrored_mip0():
    """Parallel views along +z and -z see the same maxima: the images are mirror images."""
    cube = synth.blob_cube_64(1)
    lo, hi = quant.finite_minmax(cube)
    lut = synth.lut_ramp(256)
    a = synth.ortho_axis(64, 64, 64, 128, 128, "+z")
    b = synth.ortho_axis(64, 64, 64, 128, 128, "-z")
    ra, _, _ = oracle.render(cube, a, lut, dict(mode="mip0", lo=lo, hi=hi))
    rb, _, _ = oracle.render(cube, b, lut, dict(mode="mip0", lo=lo, hi=hi))
    # both cameras use U = +x, V = +y: identical pixel grids, same maxima
    assert np.max(np.abs(ra - rb)) < 1e-12


def test_axis_transpose_invariance_perspective():
    """Swapping the cube's x and y axes and the camera's x and y components (and U with V
    on a square image) transposes the perspective MIP0 image: pins the per-axis handling of
    oblique rays in ray generation, box entry and interpolation."""
    cube = synth.blob_cube(24, 3, seed=4)
    lo, hi = quant.finite_minmax(cube)
    lut = synth.lut_heat(256)
    cam = synth.perspective_lookat(24, 24, 24, 35.0, 25.0, 60.0, 40.0, 48, 48)
    sw = lambda v: (v[1], v[0], v[2])  # noqa: E731
    cam_t = synth.Camera(1, sw(cam.eye), sw(cam.V), sw(cam.U), sw(cam.W), 48, 48)
    cube_t = np.ascontiguousarray(np.swapaxes(cube, 1, 2))
    a, _, na = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi))
    b, _, nb = oracle.render(cube_t, cam_t, lut, dict(mode="mip0", lo=lo, hi=hi))
    a = a.reshape(48, 48, 4)
    b = b.reshape(48, 48, 4)
    assert np.max(np.abs(a - np.transpose(b, (1, 0, 2)))) < 1e-9
    assert (na.reshape(48, 48) == nb.reshape(48, 48).T).all()
    assert (na > 0).sum() > 1000


def test_perspective_samples_match_library_trilinear():
    """Perspective MIP0 at random pixels equals the maximum of library-interpolated samples
    along the same ray (points o + (t0 + k dt) d, N = ceil((t1 - t0)/dt))."""
    cube = synth.blob_cube(20, 2, seed=7)
    lo, hi = quant.finite_minmax(cube)
    lut = synth.lut_ramp(256)
    cam = synth.perspective_lookat(20, 20, 20, 50.0, -30.0, 45.0, 50.0, 40, 30)
    pix = np.arange(40 * 30)
    rgba, _, ns = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi, dt=0.37),
                                pixels=pix)
    checked = 0
    for i in pix:
        o, d = oracle.pixel_ray(cam, int(i % 40), int(i // 40))
        r = oracle.ray_box(cube.shape, o, d)
        if r is None:
            assert ns[i] == 0 and np.all(rgba[i] == 0)
            continue
        t0, t1 = r
        N = int(math.ceil((t1 - t0) / 0.37))
        assert ns[i] == N
        ts = t0 + 0.37 * np.arange(N)
        vals = scipy_trilinear(cube, o[None] + ts[:, None] * d[None])
        s = norm01(vals.max(), lo, hi)
        assert abs(rgba[i, 0] - s) < 1e-7  # ramp table stored in float32
        checked += 1
    assert checked > 300


# ------------------------------------------------------------------ AVIP pins (P1, P5, P13)
def test_avip_uniform_cube_closed_form():
    """Alg. AVIP0 on a uniform cube with a = k s constant: alpha_n = 1 - (1 - a)^n and the
    colour is the table colour exactly.  a = 0.01 over 128 samples gives 0.7237483323."""
    n = 64
    cube = np.full((n, n, n), 0.5, np.float32)
    cam = synth.ortho_axis(n, n, n, 8, 8, "+z")
    lut = synth.lut_heat(256)
    rgba, frag, ns = oracle.render(cube, cam, lut, dict(mode="avip0", lo=0.0, hi=1.0, k=0.02))
    assert (ns == 128).all()
    alpha = 1.0 - (1.0 - 0.01) ** 128
    assert abs(alpha - 0.7237483323) < 1e-10
    assert np.max(np.abs(rgba[:, 3] - alpha)) < 1e-12
    c = [np.interp(0.5, np.arange(256) / 255.0, lut[:, ch].astype(np.float64)) for ch in range(3)]
    assert np.max(np.abs(rgba[:, :3] - np.array(c)[None])) < 1e-12


def test_avip_early_termination_index():
    """Alg. AVIP0 stops after the first sample whose alpha exceeds 0.99: with a = 0.1,
    alpha_43 = 0.98922 and alpha_44 = 0.99030, so exactly 44 samples are composited."""
    n = 64
    cube = np.full((n, n, n), 0.5, np.float32)
    cam = synth.ortho_axis(n, n, n, 4, 4, "+z")
    lut = synth.lut_ramp(256)
    rgba, frag, ns = oracle.render(cube, cam, lut, dict(mode="avip0", lo=0.0, hi=1.0, k=0.2))
    assert abs((1 - 0.9 ** 43) - 0.98922) < 1e-5 and abs((1 - 0.9 ** 44) - 0.99030) < 1e-5
    assert (ns == 44).all()
    assert np.max(np.abs(rgba[:, 3] - (1 - 0.9 ** 44))) < 1e-12


@pytest.mark.parametrize("mode", ["avip0", "avip1", "aviprgb"])
def test_avip_equals_premultiplied_emission_absorption(mode):
    """With the minVal clamp inactive, the paper's normalised recurrence equals the textbook
    front-to-back emission-absorption sum C' = C + c a (1 - A), A' = A + a (1 - A), with the
    output colour C/A.  Samples come from library interpolation at closed-form positions."""
    n = 24
    cube = synth.blob_cube(n, 3, seed=2)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    lut = synth.lut_heat(128)
    k = 0.31
    rgba, _, ns = oracle.render(cube, cam, lut, dict(mode=mode, lo=lo, hi=hi, k=k, ert=0.99))
    x, y, zs = ortho_z_samples(n, n, n)
    grid = np.arange(128) / 127.0
    tab = lambda s, ch: np.interp(s, grid, lut[:, ch].astype(np.float64))  # noqa: E731
    for p in range(0, n * n, 7):
        pts = np.stack([np.full_like(zs, x[p]), np.full_like(zs, y[p]), zs], 1)
        s = norm01(scipy_trilinear(cube, pts), lo, hi)
        Cp = np.zeros(3)
        A = 0.0
        cnt = 0
        for kk in range(len(zs)):
            if mode == "avip0":
                col = np.array([tab(s[kk], ch) for ch in range(3)])
            else:
                loc = np.clip((pts[kk] + 0.5) / n, 0, 1)
                col = (np.array([tab(loc[2], ch) for ch in range(3)]) if mode == "avip1"
                       else np.array([loc[2], loc[1], loc[0]]))
            a = k * s[kk]
            Cp += col * a * (1 - A)
            A += a * (1 - A)
            cnt += 1
            if A > 0.99:
                break
        assert ns[p] == cnt
        assert abs(rgba[p, 3] - A) < 1e-12
        assert np.max(np.abs(rgba[p, :3] - Cp / A)) < 1e-10


def test_avip_gradient_closed_form_uniform():
    """d alpha_n / d a = n (1 - a)^(n-1) for the uniform cube (Eq. AVIP unrolled), pushed to
    the transfer function's alpha control points through a = k * tf(s).a."""
    n = 32
    cube = np.full((n, n, n), 0.5, np.float32)
    cam = synth.ortho_axis(n, n, n, 2, 2, "+z")
    M = 5
    tf = np.full((M, 4), 0.3)
    k = 0.1
    a = k * 0.3
    g = np.zeros((4, 4))
    g[:, 3] = 1.0
    rgba, gtf, gvox = oracle.render_grad(cube, cam, tf, dict(lo=0.0, hi=1.0, k=k, ert=2.0), g)
    N = 64
    assert np.allclose(rgba[:, 3], 1 - (1 - a) ** N)
    dA_da = N * (1 - a) ** (N - 1)
    # s = 0.5 -> x = 2.0 -> interval j0 = 2, f = 0: all weight on control point 2
    assert abs(gtf[2, 3] - 4 * dA_da * k) < 1e-10
    assert np.allclose(np.delete(gtf[:, 3], 2), 0.0)


def test_avip_gradient_matches_central_differences():
    """The oracle's reverse pass agrees with central finite differences of its own forward
    pass (h = 1e-6) for transfer-function control points and voxel values."""
    cube = synth.gradcheck_cube(0, n=12).astype(np.float64)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.perspective_lookat(12, 12, 12, 30.0, 20.0, 30.0, 40.0, 6, 6)
    M = 8
    tf = synth.tf_bumps(M, seed=1).astype(np.float64) * 0.9 + 0.05
    params = dict(lo=lo, hi=hi, k=0.4, ert=0.99, dt=0.5)
    rng = np.random.default_rng(0)
    grad = rng.standard_normal((36, 4))
    rgba, gtf, gvox = oracle.render_grad(cube, cam, tf, params, grad)

    def loss(tf_, cube_):
        p = dict(params, mode="avip0", opacity_from_lut=1)
        r, frag, _ = oracle.render(cube_, cam, tf_, p, margins=dict(da=1e-4))
        return float((r * grad).sum()), frag

    _, frag = loss(tf, cube)
    h = 1e-6
    for (j, ch) in [(1, 0), (3, 3), (5, 1), (6, 2), (2, 3)]:
        tp, tm = tf.copy(), tf.copy()
        tp[j, ch] += h
        tm[j, ch] -= h
        fd = (loss(tp, cube)[0] - loss(tm, cube)[0]) / (2 * h)
        assert abs(fd - gtf[j, ch]) <= 1e-6 * max(1.0, abs(fd))
    idx = np.argsort(-np.abs(gvox).ravel())[:6]
    for i in idx:
        cp, cm = cube.copy().ravel(), cube.copy().ravel()
        cp[i] += h
        cm[i] -= h
        fd = (loss(tf, cp.reshape(cube.shape))[0] - loss(tf, cm.reshape(cube.shape))[0]) / (2 * h)
        assert abs(fd - gvox.ravel()[i]) <= 1e-6 * max(1.0, abs(fd))


# ------------------------------------------------------------------ filters (P10)
def test_filters_reduce_to_identity_when_inactive():
    """Clipping with minT below and maxT above the data, domain scaling over [lo, hi],
    and box smoothing of a constant cube all leave the render unchanged."""
    cube = synth.blob_cube_64(2)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.perspective_lookat(64, 64, 64, 20.0, 10.0, 120.0, 40.0, 48, 32)
    lut = synth.lut_heat(256)
    for mode in ("mip0", "mip1", "avip0", "aviprgb"):
        base, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=lo, hi=hi))
        clip, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=lo, hi=hi, filter="clip",
                                                         min_t=lo - 1, max_t=hi + 1))
        scale, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=lo, hi=hi,
                                                          filter="scale", min_t=lo, max_t=hi))
        assert np.max(np.abs(base - clip)) == 0.0
        assert np.max(np.abs(base - scale)) < 1e-12
    const = np.full((16, 16, 16), 0.37, np.float32)
    cam2 = synth.perspective_lookat(16, 16, 16, 40.0, 30.0, 40.0, 40.0, 16, 16)
    for mode in ("mip1", "avip0"):
        a, _, _ = oracle.render(const, cam2, lut, dict(mode=mode, lo=0, hi=1))
        b, _, _ = oracle.render(const, cam2, lut, dict(mode=mode, lo=0, hi=1, box_arm=3))
        assert np.max(np.abs(a - b)) < 1e-12


def test_clip_and_scale_follow_the_algorithms():
    """Alg. intensity clipping: a fetched value below minT or above maxT becomes DATAMIN
    (s = 0).  Alg. domain scaling: out of [minT, maxT] -> DATAMIN, inside
    (v - minT)/(maxT - minT).  Both act on the interpolated sample (Alg. 1 filter())."""
    n = 8
    rng = np.random.default_rng(1)
    cube = rng.uniform(0, 10, (n, n, n)).astype(np.float32)
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    lut = synth.lut_ramp(256)
    lo, hi = quant.finite_minmax(cube)
    x, y, zs = ortho_z_samples(n, n, n)
    rc, _, _ = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi, filter="clip",
                                                  min_t=3.0, max_t=7.0))
    rs, _, _ = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi, filter="scale",
                                                  min_t=3.0, max_t=7.0))
    for p in range(n * n):
        pts = np.stack([np.full_like(zs, x[p]), np.full_like(zs, y[p]), zs], 1)
        v = scipy_trilinear(cube, pts)
        out = (v < 3.0) | (v > 7.0)
        kept = np.where(out, lo, v).max()
        assert abs(rc[p, 0] - norm01(kept, lo, hi)) < 1e-7
        sc = np.where(out, 0.0, (v - 3.0) / 4.0).max()
        assert abs(rs[p, 0] - sc) < 1e-7


def test_box_smoothing_is_mean_along_the_ray():
    """Section 4.1: with filterArm a the value at sample k is the mean of the samples at
    k-a..k+a along the ray; axis-aligned, that is a running mean of library samples."""
    n = 12
    cube = synth.blob_cube(n, 2, seed=9)
    lo, hi = quant.finite_minmax(cube)
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    lut = synth.lut_ramp(256)
    a = 2
    r, _, ns = oracle.render(cube, cam, lut, dict(mode="mip0", lo=lo, hi=hi, box_arm=a))
    x, y, zs = ortho_z_samples(n, n, n)
    zext = -0.5 + 0.5 * np.arange(-a, len(zs) + a)
    for p in range(0, n * n, 5):
        pts = np.stack([np.full_like(zext, x[p]), np.full_like(zext, y[p]), zext], 1)
        v = scipy_trilinear(cube, pts)
        mean = np.convolve(v, np.ones(2 * a + 1) / (2 * a + 1), mode="valid")
        assert abs(r[p, 0] - norm01(mean.max(), lo, hi)) < 1e-7


# ------------------------------------------------------------------ misses (P14)
def test_missing_rays_and_backward_camera_give_zero():
    cube = synth.blob_cube_64(0)
    lut = synth.lut_ramp(256)
    away = synth.Camera(1, (31.5, 31.5, -50.0), (0.2, 0, 0), (0, 0.2, 0), (0, 0, -1.0), 8, 8)
    r, _, ns = oracle.render(cube, away, lut, dict(mode="avip0", lo=-5, hi=20))
    assert np.all(r == 0) and np.all(ns == 0)
    side = synth.Camera(0, (100.0, 31.5, 31.5), (0, 5, 0), (0, 0, 5), (1.0, 0, 0), 8, 8)
    r, _, ns = oracle.render(cube, side, lut, dict(mode="mip0", lo=-5, hi=20))
    assert np.all(r == 0) and np.all(ns == 0)


def test_eye_inside_volume_starts_at_eye():
    cube = synth.blob_cube_64(0)
    lut = synth.lut_ramp(256)
    cam = synth.Camera(1, (31.5, 31.5, 31.5), (0.3, 0, 0), (0, 0.3, 0), (0, 0, 1.0), 2, 2)
    _, _, ns = oracle.render(cube, cam, lut, dict(mode="mip0", lo=-5, hi=20, dt=0.5))
    o, d = oracle.pixel_ray(cam, 0, 0)
    t0, t1 = oracle.ray_box(cube.shape, o, d)
    assert t0 == 0.0
    assert ns[0] == math.ceil(t1 / 0.5)


# ------------------------------------------------------------------ line ratio (P8, P9)
def test_line_ratio_of_gaussian_lines_closed_form():
    """Section 4.5 method 2 per voxel: two Gaussian lines A1 g(z; c, s1), A2 g(z; c, s2) have
    ratio (A2/A1) exp(-(z - c)^2 (1/s2^2 - 1/s1^2)/2); equal widths give a constant A2/A1."""
    n, nz = 20, 40
    l1, l2 = synth.two_line_pair(n, nz, ratio=0.4, sig1=3.0, sig2=2.0)
    cube = np.concatenate([l1, l2], axis=0)
    R = oracle.line_ratio(cube, 0, nz, nz, datamin=-1.0)
    z = np.arange(nz)[:, None, None]
    c = nz / 2.0
    ref = 0.4 * np.exp(-((z - c) ** 2) * (1 / 2.0 ** 2 - 1 / 3.0 ** 2) / 2.0)
    ok = l1 > 1e-200
    assert np.max(np.abs(R - np.broadcast_to(ref, R.shape))[ok] / ref.max()) < 1e-10


def test_ratio_render_methods_on_proportional_lines():
    """Method 1 (ratio of maxima, strict '>') and method 2 (MIP of per-sample ratios) both
    return A2/A1 when the two lines have equal widths, at any viewing angle."""
    n, nz = 16, 24
    l1, l2 = synth.two_line_pair(n, nz, ratio=0.45, sig1=2.5, sig2=2.5, amp=2.0)
    l1 = l1 + 0.05  # keep cube 1 positive everywhere so every sample is defined
    l2 = l2 + 0.45 * 0.05
    lut = synth.lut_ramp(256)
    cam = synth.perspective_lookat(n, n, nz, 25.0, 15.0, 50.0, 40.0, 20, 20)
    for method in (1, 2):
        r, frag, ns = oracle.render(l1, cam, lut, dict(mode="mip0", ratio=method, lo=0.0, hi=1.0,
                                                       ratio_lo=0.0, ratio_hi=1.0), cube2=l2)
        hit = ns > 0
        assert hit.sum() > 100
        assert np.max(np.abs(r[hit, 0] - 0.45)) < 1e-7


def test_ratio_of_a_cube_with_itself_is_one():
    cube = synth.blob_cube_64(0)
    R = oracle.line_ratio(cube, 10, 10, 20, datamin=-99.0)
    pos = cube[10:30] > 0
    assert np.all(R[pos] == 1.0)
    assert np.all(R[~pos] == -99.0)


# ------------------------------------------------------------------ smoothing (P6, P7)
def test_binomial_taps_are_pascal_rows():
    """Section 4.2: b_n = [1, 1]^{*n} is the binomial series (Pascal's triangle)."""
    for T in (3, 5, 9, 13):
        n = T - 1
        ref = np.array([math.comb(n, j) for j in range(T)], dtype=np.float64) / 2.0 ** n
        assert np.array_equal(taps.binomial(T), ref)


def test_paper9_printed_constants_are_trimmed_b12():
    """The printed 9-tap weights/offsets (Section 4.2, golden fixture) are the linear-sampling
    form of b_12 with its two outermost taps per side dropped and renormalised:
    [66, 220, 495, 792, 924, 792, 495, 220, 66] / 4070."""
    g = json.load(open(os.path.join(GOLDEN, "paper9_taps.json")))
    assert taps.PAPER9_CENTRE_WEIGHT == g["coeff0"]
    assert taps.PAPER9_PAIRS == ((g["off1"], g["coeff1"]), (g["off2"], g["coeff2"]))
    ref = np.array([66, 220, 495, 792, 924, 792, 495, 220, 66], dtype=np.float64) / 4070.0
    b12 = np.array([math.comb(12, j) for j in range(13)], dtype=np.float64)[2:11]
    assert np.allclose(b12 / b12.sum(), ref, atol=0)
    assert np.max(np.abs(taps.paper9() - ref)) < 5e-10  # printed to 10 digits
    f = json.load(open(os.path.join(GOLDEN, "fetch_counts.json")))
    per_axis = 1 + 2 * len(taps.PAPER9_PAIRS)
    assert 3 * (per_axis - 1) + 1 == f["gauss"]["9"]


def test_paper9_linear_sampling_equals_direct_sum_on_a_row():
    """Applying the shader's 5 linear-sampled fetches to a random row equals the 9-tap
    discrete sum with the expanded taps (interpolation by numpy.interp)."""
    rng = np.random.default_rng(0)
    row = rng.standard_normal(64)
    xs = np.arange(64)
    t = taps.paper9()
    for c in range(10, 54):
        shader = g0 = taps.PAPER9_CENTRE_WEIGHT * row[c]
        for off, w in taps.PAPER9_PAIRS:
            shader += w * (np.interp(c + off, xs, row) + np.interp(c - off, xs, row))
        direct = float(np.dot(t, row[c - 4:c + 5]))
        assert abs(shader - direct) < 1e-12 + 0 * g0


def test_gaussian_taps_and_fwhm():
    """Eq. Gaussian (isotropic) and Eq. FWHM: the sampled kernel is symmetric with unit sum
    and variance close to sigma^2; the continuous profile is half maximum at FWHM/2."""
    for sigma in (1.0, 2.0, 3.0):
        g = taps.gauss(sigma)
        r = len(g) // 2
        assert len(g) == 2 * math.ceil(3 * sigma) + 1
        assert np.allclose(g, g[::-1]) and abs(g.sum() - 1) < 1e-15
        a = np.arange(-r, r + 1)
        var = float((g * a * a).sum())
        assert abs(var - sigma ** 2) / sigma ** 2 < 0.03
        h = taps.fwhm(sigma) / 2.0
        assert abs(math.exp(-h * h / (2 * sigma * sigma)) - 0.5) < 1e-15


def test_smooth_separable_equals_library_and_triple_sum():
    """Section 4.2 successive 1D convolution per axis with clamp-to-edge equals scipy's 1D
    correlation along each axis (mode 'nearest') and the direct triple sum; a constant
    cube is unchanged and a centred delta returns the kernel g x g x g."""
    rng = np.random.default_rng(2)
    cube = rng.standard_normal((11, 13, 16))
    for g in (taps.binomial(5), taps.gauss(1.0), taps.paper9()):
        out = oracle.smooth(cube, g)
        ref = cube
        for ax in (2, 1, 0):
            ref = ndimage.correlate1d(ref, g, axis=ax, mode="nearest")
        assert np.max(np.abs(out - ref)) < 1e-13
        idx = rng.choice(cube.size, 50, replace=False)
        assert np.max(np.abs(oracle.smooth_at(cube, g, idx) - out.ravel()[idx])) < 1e-13
    const = np.full((9, 9, 9), 3.25)
    assert np.max(np.abs(oracle.smooth(const, taps.gauss(2.0)) - 3.25)) < 1e-14
    g = taps.gauss(1.0)
    r = len(g) // 2
    delta = np.zeros((15, 15, 15))
    delta[7, 7, 7] = 1.0
    out = oracle.smooth(delta, g)
    kern = np.einsum("i,j,k->ijk", g, g, g)
    assert np.max(np.abs(out[7 - r:8 + r, 7 - r:8 + r, 7 - r:8 + r] - kern)) < 1e-16


# ------------------------------------------------------------------ storage (N1)
def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.standard_normal(10000).astype(np.float32) * 100,
                        np.array([0.0, -0.0, 1e-40, np.inf, -np.inf, 3.0e38], np.float32)])
    ours = quant.to_bf16_as_f32(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(quant.to_bf16_as_f32(np.array([np.nan], np.float32))).all()


def test_finite_minmax_ignores_nan():
    cube = synth.nan_mosaic_cube(32, 32, 8)
    lo, hi = quant.finite_minmax(cube)
    f = cube[np.isfinite(cube)]
    assert lo == f.min() and hi == f.max() and np.isnan(cube).any()


# ------------------------------------------------------------------ moment maps (Section 2.2)
def _gauss_line_cube(nx, ny, nz, seed):
    """Each spectrum one Gaussian line A exp(-(z - mu)^2 / 2 s^2), s = 3 channels, with mu at
    least 10 s from both ends: the channel sums equal the integrals up to terms below 1e-20
    (Poisson summation), so M0 = dv A s sqrt(2 pi) and M1 = mu."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 4.0, (ny, nx))
    mu = rng.uniform(31.0, nz - 31.0, (ny, nx))
    z = np.arange(nz, dtype=np.float64)[:, None, None]
    s = 3.0
    return amp * np.exp(-(z - mu[None]) ** 2 / (2 * s * s)), amp, mu, s


def test_moments_gaussian_line_closed_form():
    V, amp, mu, s = _gauss_line_cube(7, 5, 96, 0)
    dv = 2.5
    m0, m1, am = oracle.moments(V, dv=dv)
    assert np.max(np.abs(m0 / (dv * amp * s * math.sqrt(2 * math.pi)) - 1.0)) < 1e-12
    assert np.max(np.abs(m1 - mu)) < 1e-10
    # the peak channel is the channel nearest to mu (mu is never within 1e-3 of a half-integer
    # for this seed, checked here)
    assert np.min(np.abs(mu - np.floor(mu) - 0.5)) > 1e-3
    assert np.array_equal(am, np.rint(mu).astype(np.int32))


def test_moments_window_uses_absolute_channel():
    """A window holding the whole line gives the same moments as the full spectrum; M1 is a
    channel index of the cube, not of the window."""
    V, amp, mu, s = _gauss_line_cube(4, 3, 128, 1)
    mu_lo, mu_hi = int(mu.min()), int(mu.max())
    z0 = max(0, mu_lo - 40)
    nzw = min(128, mu_hi + 40) - z0
    full = oracle.moments(V)
    win = oracle.moments(V, z0=z0, nzw=nzw)
    assert np.max(np.abs(win[0] - full[0])) < 1e-12 * np.max(np.abs(full[0]))
    assert np.max(np.abs(win[1] - full[1])) < 1e-10
    assert np.array_equal(win[2], full[2])


def test_moments_ties_symmetry_and_exclusions():
    # plateau maximum: the later channel (MIP's >= rule); symmetric spectrum: M1 at the centre
    V = np.zeros((6, 1, 1))
    V[:, 0, 0] = [0.0, 1.0, 3.0, 3.0, 1.0, 0.0]
    m0, m1, am = oracle.moments(V)
    assert m0[0, 0] == 8.0 and m1[0, 0] == 2.5 and am[0, 0] == 3
    # non-finite channels and channels outside [min_t, max_t] do not count
    V = np.zeros((6, 1, 1))
    V[:, 0, 0] = [1.0, 2.0, np.nan, 5.0, 100.0, -np.inf]
    m0, m1, am = oracle.moments(V, dv=0.5, min_t=-1.0, max_t=10.0)
    assert m0[0, 0] == 0.5 * 8.0
    assert abs(m1[0, 0] - (0 * 1 + 1 * 2 + 3 * 5) / 8.0) < 1e-15
    assert am[0, 0] == 3
    # nothing counts: M0 = 0, M1 undefined, no argmax; a zero sum leaves M1 undefined too
    V = np.full((4, 1, 2), np.nan)
    V[:, 0, 1] = [1.0, -1.0, 2.0, -2.0]
    m0, m1, am = oracle.moments(V)
    assert m0[0, 0] == 0.0 and np.isnan(m1[0, 0]) and am[0, 0] == -1
    assert m0[0, 1] == 0.0 and np.isnan(m1[0, 1]) and am[0, 1] == 2


def test_moments_linearity():
    """M0 scales with the data, M1 and the argmax do not; both are independent per spectrum."""
    rng = np.random.default_rng(3)
    V = rng.uniform(0.1, 1.0, (20, 3, 4))
    a = oracle.moments(V, dv=1.5)
    b = oracle.moments(3.0 * V, dv=1.5)
    assert np.max(np.abs(b[0] - 3.0 * a[0])) < 1e-12 * np.max(b[0])
    assert np.max(np.abs(b[1] - a[1])) < 1e-12 * np.max(a[1])
    assert np.array_equal(a[2], b[2])


# ------------------------------------------------------------------ in-ray Gaussian (Section 4.2)
# The paper's 9-tap stencil: centre weight and (offset, weight) pairs (golden constants).
STAR9 = (taps.PAPER9_CENTRE_WEIGHT, taps.PAPER9_PAIRS)


def _axis_view_red(cube, axis, star):
    """MIP0 through the two-entry grey table [0, 1], parallel rays along `axis` through voxel
    centres:
    every sample of a ray shares the two other coordinates, and on a cube that varies only
    across the ray the rendered value is the smoothed value itself."""
    nz, ny, nx = cube.shape
    n = {"x": nx, "y": ny, "z": nz}
    others = [a for a in "xyz" if a != axis]
    cam = synth.ortho_axis(nx, ny, nz, n[others[0]], n[others[1]], "+" + axis)
    lo, hi = float(cube.min()), float(cube.max())
    p = dict(mode="mip0", lo=lo - 1.0, hi=hi + 1.0, dt=0.5, star=star)
    ramp = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 1.0, 1.0, 1.0]])  # red = s exactly
    rgba, frag, ns = oracle.render(cube, cam, ramp, p)
    s = rgba[:, 0].reshape(n[others[1]], n[others[0]])
    return s * (p["hi"] - p["lo"]) + p["lo"]


def _interp_clamped(f, t):
    return np.interp(t, np.arange(f.size, dtype=np.float64), f)


def _one_axis(f, t, c0, pairs):
    """c0 f(t) + sum_k w_k (f(t + o_k) + f(t - o_k)) on the clamped linear interpolant of f."""
    out = c0 * _interp_clamped(f, t)
    for o, w in pairs:
        out = out + w * (_interp_clamped(f, t + o) + _interp_clamped(f, t - o))
    return out


def test_star_weights_sum_to_one_and_constant_cube():
    c0, pairs = STAR9
    assert abs(c0 + 2 * sum(w for _, w in pairs) - 1.0) < 1e-9
    cube = np.full((12, 10, 9), 3.25)
    v = _axis_view_red(cube, "z", STAR9)
    assert np.max(np.abs(v - 3.25)) < 1e-8


def test_star_reduces_to_one_axis_filter():
    """On a cube that varies along one axis only, the stencils of the other two axes see a
    constant and the result has a closed form: along z (the last axis) the 1D stencil itself;
    along y, c0 F + (1 - c0) f; along x, c0^2 F + (1 - c0^2) f (F the 1D stencil, f the
    value), since each later axis takes the earlier result as its centre and fetches the raw
    cube around it."""
    c0, pairs = STAR9
    rng = np.random.default_rng(5)
    f = rng.standard_normal(17)
    t = np.arange(17, dtype=np.float64)
    F = _one_axis(f, t, c0, pairs)
    # varies along z, rays along x: image rows are z
    cube = np.broadcast_to(f[:, None, None], (17, 6, 5)).copy()
    v = _axis_view_red(cube, "x", STAR9)
    assert np.max(np.abs(v - F[:, None])) < 1e-9
    # varies along y, rays along z: image rows are y
    cube = np.broadcast_to(f[None, :, None], (6, 17, 5)).copy()
    v = _axis_view_red(cube, "z", STAR9)
    assert np.max(np.abs(v - (c0 * F + (1 - c0) * f)[:, None])) < 1e-9
    # varies along x, rays along z: image columns are x
    cube = np.broadcast_to(f[None, None, :], (6, 5, 17)).copy()
    v = _axis_view_red(cube, "z", STAR9)
    assert np.max(np.abs(v - (c0 * c0 * F + (1 - c0 * c0) * f)[None, :])) < 1e-9


def test_star_linear_sampling_at_voxel_centres():
    """At voxel centres the 9-tap stencil of fractional offsets equals the discrete 9-tap
    filter of the paper's taps (the linear-sampling identity of the printed constants)."""
    g = taps.paper9()
    assert g.size == 9
    rng = np.random.default_rng(6)
    f = rng.standard_normal(30)
    c0, pairs = STAR9
    t = np.arange(4, 26, dtype=np.float64)
    F = _one_axis(f, t, c0, pairs)
    direct = np.array([sum(g[j] * f[int(ti) + j - 4] for j in range(9)) for ti in t])
    assert np.max(np.abs(F - direct)) < 1e-9


# ------------------------------------------------------------------ branches pinned by closed forms
def _pinhole_pixel(cam, point):
    """Continuous pixel coordinates of a world point under a pinhole camera whose axes
    U, V are orthogonal to the unit viewing direction W: the point's offset from the eye,
    divided by its depth along W, has components u |U| and v |V| across the image, and
    pixel centres sit at u = 2 (px + 0.5)/width - 1 (inverted here)."""
    r = np.asarray(point, np.float64) - np.asarray(cam.eye, np.float64)
    U, V, W = (np.asarray(a, np.float64) for a in (cam.U, cam.V, cam.W))
    depth = float(r @ W)
    u = float(r @ U) / float(U @ U) / depth
    v = float(r @ V) / float(V @ V) / depth
    return (u + 1.0) * cam.width / 2.0 - 0.5, (v + 1.0) * cam.height / 2.0 - 0.5


@pytest.mark.parametrize("az,el", [(0.0, 0.0), (40.0, 20.0), (130.0, -35.0), (220.0, 60.0),
                                   (300.0, 10.0)])
def test_perspective_bright_voxel_lands_on_pinhole_pixel(az, el):
    """Appendix A perspective projection, orientation: a single bright voxel off the
    viewing axis lights the pixel the pinhole model predicts for the look-at camera (u to
    the camera's right along U, v along V; a mirrored, rotated or u/v-swapped image moves
    the brightest pixel far from the prediction).  MIP0 of a zero cube with one voxel at 1:
    the brightest ray is the one passing nearest the voxel centre."""
    nx, ny, nz = 24, 20, 28
    W, H = 64, 48
    lut = synth.lut_ramp(256)
    cam = synth.perspective_lookat(nx, ny, nz, az, el, 48.0, 30.0, W, H)
    checked = 0
    for vox in [(18, 5, 9), (4, 15, 20), (15, 13, 3)]:
        cube = np.zeros((nz, ny, nx), np.float32)
        cube[vox[2], vox[1], vox[0]] = 1.0
        rgba, _, _ = oracle.render(cube, cam, lut, dict(mode="mip0", lo=0.0, hi=1.0, dt=0.05))
        img = rgba[:, 0].reshape(H, W)
        py, px = np.unravel_index(int(np.argmax(img)), img.shape)
        ex, ey = _pinhole_pixel(cam, vox)
        # the voxel must project well away from the image centre for this to pin orientation
        assert abs(ex - (W - 1) / 2) + abs(ey - (H - 1) / 2) > 6
        assert abs(px - ex) <= 1.0 and abs(py - ey) <= 1.0, (vox, (px, py), (ex, ey))
        assert img.max() > 0.5  # a ray passes within half a pixel (~0.2 voxel) of the centre
        checked += 1
    assert checked == 3


def test_perspective_centre_ray_and_field_of_view():
    """Appendix A perspective rays: on an image of odd size the centre pixel's ray runs
    along W through the look-at point (the cube centre), and the rays through the outer
    pixel centres of the middle column (row) subtend 2 atan(tan(fov/2) (1 - 1/H)) (and
    2 atan(tan(fov/2) (W/H) (1 - 1/W)) across), the field of view of the look-at camera
    less half a pixel at each edge."""
    nx, ny, nz = 30, 22, 40
    W, H, fov = 65, 33, 36.0
    cam = synth.perspective_lookat(nx, ny, nz, 25.0, 15.0, 70.0, fov, W, H)
    centre = np.array([(nx - 1) / 2, (ny - 1) / 2, (nz - 1) / 2])
    o, d = oracle.pixel_ray(cam, W // 2, H // 2)
    assert np.allclose(o, cam.eye)
    # distance from the cube centre to the centre ray
    w = centre - o
    assert np.linalg.norm(w - (w @ d) * d) < 1e-9
    assert abs(np.linalg.norm(d) - 1.0) < 1e-14

    def angle(a, b):
        return math.acos(max(-1.0, min(1.0, float(a @ b))))
    t = math.tan(math.radians(fov) / 2)
    _, d_lo = oracle.pixel_ray(cam, W // 2, 0)
    _, d_hi = oracle.pixel_ray(cam, W // 2, H - 1)
    assert abs(angle(d_lo, d_hi) - 2 * math.atan(t * (1 - 1 / H))) < 1e-12
    _, d_l = oracle.pixel_ray(cam, 0, H // 2)
    _, d_r = oracle.pixel_ray(cam, W - 1, H // 2)
    assert abs(angle(d_l, d_r) - 2 * math.atan(t * (W / H) * (1 - 1 / W))) < 1e-12
    # rows and columns move along V and U respectively (not swapped, not mirrored)
    U, V = np.asarray(cam.U), np.asarray(cam.V)
    assert (d_hi - d_lo) @ V > 0 and abs((d_hi - d_lo) @ U) < 1e-12
    assert (d_r - d_l) @ U > 0 and abs((d_r - d_l) @ V) < 1e-12


def test_avip_all_transparent_ray_ends_at_min_val():
    """Alg. AVIP0's minVal: a ray whose samples are all at DATAMIN (s = 0, no opacity) has
    alpha1 + alpha2 = 0 at every sample, so alpha is held at minVal and the colour stays 0:
    the fragment is (0, 0, 0, minVal) for any minVal, in every AVIP colouring."""
    n = 16
    cube = np.full((n, n, n), 2.0, np.float32)
    cam = synth.ortho_axis(n, n, n, 8, 8, "+z")
    lut = synth.lut_heat(256)
    for mode in ("avip0", "avip1", "aviprgb"):
        for mv in (1e-6, 0.3):
            rgba, _, ns = oracle.render(cube, cam, lut, dict(mode=mode, lo=2.0, hi=3.0,
                                                             k=0.5, min_val=mv))
            assert (ns == 2 * n).all()
            assert np.all(rgba[:, :3] == 0.0)
            assert np.all(rgba[:, 3] == mv)


def test_avip_min_val_clamp_closed_form():
    """Alg. AVIP0's minVal clamp when the first sample's opacity a = k s is below minVal:
    alpha_1 = max(a, minVal) = minVal and the first colour weight is a/minVal; afterwards
    1 - alpha_n = (1 - minVal)(1 - a)^(n-1), and the premultiplied colour grows by
    c a (1 - alpha_{n-1}) per sample, so rgb_n = c (a + alpha_n - minVal)/alpha_n."""
    n = 64
    cube = np.full((n, n, n), 0.5, np.float32)
    cam = synth.ortho_axis(n, n, n, 4, 4, "+z")
    lut = synth.lut_heat(256)
    mv, k = 0.05, 0.01
    a = k * 0.5
    rgba, frag, ns = oracle.render(cube, cam, lut, dict(mode="avip0", lo=0.0, hi=1.0, k=k,
                                                        min_val=mv))
    N = 128
    assert (ns == N).all()
    alpha = 1.0 - (1.0 - mv) * (1.0 - a) ** (N - 1)
    c = np.array([np.interp(0.5, np.arange(256) / 255.0, lut[:, ch].astype(np.float64))
                  for ch in range(3)])
    assert np.max(np.abs(rgba[:, 3] - alpha)) < 1e-12
    assert np.max(np.abs(rgba[:, :3] - c[None] * (a + alpha - mv) / alpha)) < 1e-12
    # the clamp really changed the result: without it the colour would be c exactly
    assert np.min(np.abs(rgba[:, 0] - c[0])) > 1e-3


@pytest.mark.parametrize("mode", ["mip0", "mip1", "miprgb"])
def test_mip_alpha_workaround_closed_form(mode):
    """The Discussion's transparency workaround (mip_alpha = 2): a fragment is opaque where
    the ray's maximum exceeds minThreshold, and keeps the plain MIP alpha (s_max for MIP1
    and MIP_RGB, the table's alpha at s_max for MIP0) where it does not.  Axis-aligned rays
    through voxel centres see s_max = (max_z V - lo)/(hi - lo) exactly."""
    n = 16
    rng = np.random.default_rng(21)
    cube = rng.uniform(0.0, 0.7, (n, n, n)).astype(np.float32)
    hot = rng.random((n, n)) < 0.5
    zi = rng.integers(0, n, (n, n))
    yy, xx = np.nonzero(hot)
    cube[zi[yy, xx], yy, xx] = rng.uniform(0.805, 1.0, yy.size).astype(np.float32)
    min_t = float(np.float32(0.8))
    # maxima just below the threshold, and exactly at it (not above: stays transparent)
    cube[3, 0, :6] = np.linspace(0.77, 0.795, 6).astype(np.float32)
    cube[5, 1, :4] = np.float32(min_t)
    cube[:, 0, :6] = np.minimum(cube[:, 0, :6], cube[3, 0, :6][None])
    cube[:, 1, :4] = np.minimum(cube[:, 1, :4], np.float32(min_t))
    lut = synth.lut_heat(256)
    lut[:, 3] = np.sqrt(np.arange(256) / 255.0)  # table alpha distinct from s
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    rgba, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=0.0, hi=1.0, mip_alpha=2,
                                                    min_t=min_t))
    smax = cube.astype(np.float64).max(axis=0).ravel()
    above = smax > min_t
    assert above.any() and (~above).any()
    assert (smax == min_t).sum() == 4 and ((smax > 0.765) & (smax < 0.8)).sum() == 6
    if mode == "mip0":
        plain = np.interp(smax, np.arange(256) / 255.0, lut[:, 3].astype(np.float64))
    else:
        plain = smax
    expect = np.where(above, 1.0, plain)
    assert np.max(np.abs(rgba[:, 3] - expect)) < 1e-12
    # the other settings: plain alpha (0) and always opaque (1)
    r0, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=0.0, hi=1.0, mip_alpha=0))
    r1, _, _ = oracle.render(cube, cam, lut, dict(mode=mode, lo=0.0, hi=1.0, mip_alpha=1))
    assert np.max(np.abs(r0[:, 3] - plain)) < 1e-12
    assert np.all(r1[:, 3] == 1.0)


def test_ratio_method1_nonpositive_denominator_gives_zero():
    """Alg. line ratio, method 1: the fragment is colourMap(max2/max1) only where the first
    cube's maximum along the ray is positive; a ray whose max1 is 0 or negative gives
    (0, 0, 0, 0) whatever the second cube holds.  Axis-aligned rays through voxel centres
    see max_i = max_z V_i exactly."""
    n = 12
    rng = np.random.default_rng(5)
    v1 = rng.uniform(0.2, 1.0, (n, n, n))
    v2 = rng.uniform(0.1, 0.9, (n, n, n))
    v1[:, :4, :] = -rng.uniform(0.1, 1.0, (n, 4, n))     # max1 < 0
    v1[:, 4:6, :] = 0.0                                  # max1 = 0
    v1[:, 4:6, :3] = -0.5                                # still max1 = 0 for x >= 3
    v1, v2 = v1.astype(np.float32), v2.astype(np.float32)
    cam = synth.ortho_axis(n, n, n, n, n, "+z")
    lut = synth.lut_heat(64)
    rgba, _, _ = oracle.render(v1, cam, lut, dict(mode="mip0", ratio=1, ratio_lo=0.0,
                                                  ratio_hi=2.0, lo=-1.0, hi=1.0), cube2=v2)
    m1 = v1.astype(np.float64).max(axis=0).ravel()
    m2 = v2.astype(np.float64).max(axis=0).ravel()
    pos = m1 > 0
    assert (~pos).sum() == n * 6 and pos.sum() == n * (n - 6)
    assert np.all(rgba[~pos] == 0.0)
    s = np.clip((m2[pos] / m1[pos] - 0.0) / 2.0, 0.0, 1.0)
    for ch in range(4):
        ref = np.interp(s, np.arange(64) / 63.0, lut[:, ch].astype(np.float64))
        assert np.max(np.abs(rgba[pos, ch] - ref)) < 1e-12
