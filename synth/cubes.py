"""Seeded synthetic spectral cubes, stored C-order as [z][y][x] (x = RA, y = Dec, z = velocity).

All generators use ``numpy.random.default_rng(seed)``; values are built in float64 and
cast to float32 at the end unless a dtype is requested.  Nothing here renders or filters.
"""
from __future__ import annotations

import math

import numpy as np


def _noise(rng, shape, sigma=1.0, dtype=np.float32):
    # float32 draws keep the 1 GiB cube cheap to build; the draw is still seeded and exact.
    if dtype == np.float64:
        return rng.standard_normal(shape) * sigma
    out = rng.standard_normal(shape, dtype=np.float32)
    if sigma != 1.0:
        out *= np.float32(sigma)
    return out


def blob_cube(n=64, nblobs=3, seed=0, noise=1.0):
    """n^3 cube: N(0, noise^2) plus ``nblobs`` Gaussian emission blobs.

    Each blob has amplitude U(5, 20) (in units of the noise sigma), centre U(12, 52)^3 for
    n = 64 (scaled with n), spatial sigma U(2, 5), spectral sigma U(1.5, 4) channels and a
    centroid velocity that shifts linearly with x: z_c(x) = z_j + g_j (x - x_j),
    g_j ~ U(-0.5, 0.5).
    """
    rng = np.random.default_rng(seed)
    cube = rng.standard_normal((n, n, n)) * noise
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    lo, hi = 12.0 * n / 64.0, 52.0 * n / 64.0
    for _ in range(nblobs):
        amp = rng.uniform(5.0, 20.0)
        xc, yc, zc = rng.uniform(lo, hi, size=3)
        ss = rng.uniform(2.0, 5.0)
        sz = rng.uniform(1.5, 4.0)
        g = rng.uniform(-0.5, 0.5)
        zcx = zc + g * (x - xc)
        cube += amp * np.exp(-((x - xc) ** 2 + (y - yc) ** 2) / (2 * ss * ss)) \
            * np.exp(-((z - zcx) ** 2) / (2 * sz * sz))
    return cube.astype(np.float32)


def add_disc(cube, xc, yc, zsys, vflat, cosi, pa, rd, snr, dv_chan, sigma_kms=10.0,
             trunc=4.0):
    """Add one inclined, thin, rotating exponential disc to ``cube`` in place.

    Rotation curve V(R) = vflat * (2/pi) * atan(R / (0.2 rd)); surface profile
    exp(-R / rd) truncated at ``trunc`` * rd; Gaussian line of width ``sigma_kms``;
    peak amplitude ``snr`` (noise sigma = 1); ``dv_chan`` km/s per channel.
    """
    nz, ny, nx = cube.shape
    sini = math.sqrt(max(0.0, 1.0 - cosi * cosi))
    rmax = trunc * rd
    x0, x1 = max(0, int(math.floor(xc - rmax))), min(nx, int(math.ceil(xc + rmax)) + 1)
    y0, y1 = max(0, int(math.floor(yc - rmax))), min(ny, int(math.ceil(yc + rmax)) + 1)
    if x0 >= x1 or y0 >= y1:
        return cube
    sig_ch = sigma_kms / dv_chan
    vspan = vflat * sini / dv_chan + 5.0 * sig_ch
    z0, z1 = max(0, int(math.floor(zsys - vspan))), min(nz, int(math.ceil(zsys + vspan)) + 1)
    if z0 >= z1:
        return cube
    yy, xx = np.meshgrid(np.arange(y0, y1, dtype=np.float64),
                         np.arange(x0, x1, dtype=np.float64), indexing="ij")
    dx, dy = xx - xc, yy - yc
    xp = dx * math.cos(pa) + dy * math.sin(pa)
    yp = (-dx * math.sin(pa) + dy * math.cos(pa)) / max(cosi, 1e-6)
    r = np.hypot(xp, yp)
    costh = np.where(r > 0, xp / np.where(r > 0, r, 1.0), 0.0)
    vrot = vflat * (2.0 / math.pi) * np.arctan(r / (0.2 * rd))
    vchan = zsys + vrot * sini * costh / dv_chan
    surf = np.where(r <= rmax, np.exp(-r / rd), 0.0)
    zz = np.arange(z0, z1, dtype=np.float64)[:, None, None]
    line = np.exp(-((zz - vchan[None]) ** 2) / (2 * sig_ch * sig_ch))
    block = (snr * surf[None] * line).astype(cube.dtype)
    cube[z0:z1, y0:y1, x0:x1] += block
    return cube


def disc_cube(nx, ny, nz, ndiscs, seed, dv_chan=4.0, centre_margin=40.0, rd_range=(3.0, 10.0),
              zsys_margin=100.0, dtype=np.float32):
    """HI-like cube: N(0,1) noise plus ``ndiscs`` rotating discs (flat curve 100-300 km/s,
    cos i ~ U(cos 80deg, cos 20deg), PA ~ U(0, 2pi), exponential profile, line width
    10 km/s, peak SNR log-uniform in [3, 30])."""
    rng = np.random.default_rng(seed)
    cube = _noise(rng, (nz, ny, nx), dtype=dtype)
    for _ in range(ndiscs):
        xc = rng.uniform(centre_margin, nx - centre_margin)
        yc = rng.uniform(centre_margin, ny - centre_margin)
        zsys = rng.uniform(zsys_margin, nz - zsys_margin)
        vflat = rng.uniform(100.0, 300.0)
        cosi = rng.uniform(math.cos(math.radians(80.0)), math.cos(math.radians(20.0)))
        pa = rng.uniform(0.0, 2 * math.pi)
        rd = rng.uniform(*rd_range)
        snr = math.exp(rng.uniform(math.log(3.0), math.log(30.0)))
        add_disc(cube, xc, yc, zsys, vflat, cosi, pa, rd, snr, dv_chan)
    return cube


def blob_cube_64(seed=0):
    """64^3 float32: noise sigma 1 + 3 blobs whose centroid velocity shifts with x."""
    return blob_cube(64, 3, seed)


def hi_cube_512x512x1024(seed=0, nx=512, ny=512, nz=1024):
    """512 x 512 x 1024 float32 HI-like cube with 50 discs (4 km/s channels)."""
    return disc_cube(nx, ny, nz, 50, seed)


def disc_cube_256(seed=0, n=256, ndiscs=10):
    """256^3 float32: noise + 10 discs (the 512x512x1024 recipe scaled by 1/2 in space,
    8 km/s channels)."""
    s = n / 256.0
    return disc_cube(n, n, n, ndiscs, seed, dv_chan=8.0, centre_margin=24.0 * s,
                     rd_range=(2.0 * s, 6.0 * s), zsys_margin=48.0 * s)


def gradcheck_cube(seed=0, n=32):
    """32^3 float64-built cube (noise + 2 discs) for gradient checks."""
    s = n / 32.0
    return disc_cube(n, n, n, 2, seed, dv_chan=16.0, centre_margin=8.0 * s,
                     rd_range=(1.0 * s, 2.5 * s), zsys_margin=8.0 * s)


def smooth_analytic_cube(nx, ny, nz):
    """Deterministic smooth float32 cube sin(0.07 x) cos(0.05 y) + 0.5 sin(0.03 z + 0.01 x)
    (x fastest), cheap to build at sizes of several GiB."""
    x = np.arange(nx, dtype=np.float32)
    y = np.arange(ny, dtype=np.float32)
    z = np.arange(nz, dtype=np.float32)
    cube = np.empty((nz, ny, nx), dtype=np.float32)
    plane = np.sin(0.07 * x)[None, :] * np.cos(0.05 * y)[:, None]
    for k in range(nz):
        cube[k] = plane + 0.5 * np.sin(0.03 * z[k] + 0.01 * x)[None, :]
    return cube


def uniform_cube(n, seed=0):
    """Uniform [0, 1) float32 cube as in the paper's benchmark (Appendix B)."""
    rng = np.random.default_rng(seed)
    return rng.random((n, n, n), dtype=np.float32)


def nan_mosaic_cube(nx=96, ny=96, nz=24, seed=0, noise=1e-2, angle_deg=20.0):
    """Antennae-like mosaic stand-in: noise + emission, NaN outside a tilted rectangle."""
    rng = np.random.default_rng(seed)
    cube = _noise(rng, (nz, ny, nx), sigma=noise).astype(np.float32)
    add_disc(cube, nx * 0.5, ny * 0.5, nz * 0.5, 150.0, 0.6, 0.3, nx / 10.0, 0.6, 20.0)
    yy, xx = np.meshgrid(np.arange(ny) - ny / 2.0, np.arange(nx) - nx / 2.0, indexing="ij")
    a = math.radians(angle_deg)
    u = xx * math.cos(a) + yy * math.sin(a)
    v = -xx * math.sin(a) + yy * math.cos(a)
    outside = (np.abs(u) > 0.38 * nx) | (np.abs(v) > 0.3 * ny)
    cube[:, outside] = np.nan
    return cube


def two_line_pair(n=50, nz=37, seed=0, ratio=0.4, sig1=2.0, sig2=2.0, amp=1.0, noise=0.0):
    """GAMA-like pair of line cubes on one grid: line 1 (strong, e.g. H-alpha) and line 2
    (faint, e.g. [NII]) with the same centroid per spaxel, Gaussian spectral profiles of
    widths ``sig1``/``sig2`` channels and amplitude ratio ``ratio``."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(n), np.arange(n), indexing="ij")
    c = nz / 2.0
    sky = amp * np.exp(-((x - n / 2.0) ** 2 + (y - n / 2.0) ** 2) / (2 * (n / 5.0) ** 2))
    l1 = sky * np.exp(-((z - c) ** 2) / (2 * sig1 ** 2))
    l2 = ratio * sky * np.exp(-((z - c) ** 2) / (2 * sig2 ** 2))
    if noise > 0:
        l1 = l1 + rng.standard_normal(l1.shape) * noise
        l2 = l2 + rng.standard_normal(l2.shape) * noise
    return l1, l2


def two_line_pair_512x512x32(seed=0):
    """Full-size line pair on the grid of two 32-channel windows of the 512 x 512 x 1024
    cube: an extended source (Gaussian sky profile of width 102 px, peak SNR 20 over unit
    noise) seen in a strong line (width 2.5 channels) and a line 0.4 times fainter
    (width 1.8 channels), float32."""
    l1, l2 = two_line_pair(n=512, nz=32, seed=seed, ratio=0.4, sig1=2.5, sig2=1.8, amp=20.0,
                           noise=1.0)
    return l1.astype(np.float32), l2.astype(np.float32)


def subcube_batch_specs(count=512, seed=0):
    """Per-sub-cube size and disc parameters for the batched workload: nx, ny log-uniform
    in [32, 256], nz log-uniform in [64, 512]; one disc centred within +-10 %, rd =
    min(nx, ny)/10, flat velocity U(100, 300) and a channel width chosen so that
    2 vflat sin i spans nz/2 channels."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(count):
        nx = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
        ny = int(round(math.exp(rng.uniform(math.log(32), math.log(256)))))
        nz = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        vflat = rng.uniform(100.0, 300.0)
        cosi = rng.uniform(math.cos(math.radians(80.0)), math.cos(math.radians(20.0)))
        sini = math.sqrt(1 - cosi * cosi)
        specs.append(dict(
            nx=nx, ny=ny, nz=nz,
            xc=nx * (0.5 + rng.uniform(-0.1, 0.1)), yc=ny * (0.5 + rng.uniform(-0.1, 0.1)),
            zsys=nz * (0.5 + rng.uniform(-0.1, 0.1)), vflat=vflat, cosi=cosi,
            pa=rng.uniform(0, 2 * math.pi), rd=min(nx, ny) / 10.0,
            snr=math.exp(rng.uniform(math.log(3.0), math.log(30.0))),
            dv_chan=2.0 * vflat * sini / (nz / 2.0),
            noise_seed=int(rng.integers(0, 2 ** 31 - 1)),
            view=rng.standard_normal(3),
        ))
    return specs


def subcube(spec, dtype=np.float16):
    """Materialise one sub-cube of the batched workload (noise + one disc)."""
    rng = np.random.default_rng(spec["noise_seed"])
    cube = _noise(rng, (spec["nz"], spec["ny"], spec["nx"]))
    add_disc(cube, spec["xc"], spec["yc"], spec["zsys"], spec["vflat"], spec["cosi"],
             spec["pa"], spec["rd"], spec["snr"], spec["dv_chan"])
    return cube.astype(dtype)
