"""GPU parity of the moment maps (Section 2.2, Eq. mom0 / Eq. mom1 and the argmax variant)
against the FP64 oracle.

Both sides sum in float64, channel by channel in increasing channel order with every operation
rounded separately, so the float32-rounded M0 and M1 and the argmax must be identical: the bar
is bit-exact (NaN where M1 is undefined on both sides).  The oracle itself is pinned to closed
forms in test_oracle_pins.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import quant
from helpers import f32, to_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def svr():
    import paper_1707_00442_amd as m
    m.lib()
    return m


def _check(svr, cube_np, gpu_cube=None, ref_cube=None, **kw):
    """Run svr_moments and the oracle with the same (float32-exact) arguments; compare."""
    q = {k: (f32(v) if k in ("dv", "min_t", "max_t") else v) for k, v in kw.items()}
    t = to_cuda(cube_np) if gpu_cube is None else gpu_cube
    m0, m1, am = svr.svr_moments(t, **q)
    svr.svr_sync()
    ref = oracle.moments(cube_np if ref_cube is None else ref_cube,
                         **{("nzw" if k == "nz_w" else k): v for k, v in q.items()})
    r0 = ref[0].astype(np.float32)
    r1 = ref[1].astype(np.float32)
    g0, g1, ga = m0.cpu().numpy(), m1.cpu().numpy(), am.cpu().numpy()
    assert np.array_equal(g0.view(np.uint32), r0.view(np.uint32)), np.abs(g0 - r0).max()
    assert np.array_equal(np.isnan(g1), np.isnan(r1))
    ok = ~np.isnan(r1)
    assert np.array_equal(g1[ok].view(np.uint32), r1[ok].view(np.uint32)), \
        np.abs(g1[ok] - r1[ok]).max()
    assert np.array_equal(ga, ref[2])
    return g0, g1, ga


def test_moments_ragged_cube(svr):
    """Dims that fill no wave or workgroup evenly; a channel count that is not a multiple of
    the 16 reads in flight (ragged tail)."""
    cube = synth.disc_cube(45, 37, 70, 3, seed=5, dv_chan=8.0, centre_margin=10.0,
                           rd_range=(2.0, 5.0), zsys_margin=15.0)
    _check(svr, cube)
    _check(svr, cube, dv=2.5)


@pytest.mark.parametrize("z0,nzw", [(0, 1), (3, 17), (11, 48), (69, 1)])
def test_moments_windows_and_clip(svr, z0, nzw):
    cube = synth.disc_cube(45, 37, 70, 3, seed=6, dv_chan=8.0, centre_margin=10.0,
                           rd_range=(2.0, 5.0), zsys_margin=15.0)
    _check(svr, cube, z0=z0, nz_w=nzw)
    _check(svr, cube, z0=z0, nz_w=nzw, dv=0.75, min_t=0.5, max_t=6.0)


def test_moments_nan_and_empty_spectra(svr):
    """Blanked (NaN) regions: spectra with no counted channel give M0 = 0, M1 = NaN and
    argmax -1; a clip window that admits nothing does the same everywhere."""
    cube = synth.nan_mosaic_cube(53, 41, 19)
    assert np.isnan(cube).any()
    _, g1, ga = _check(svr, cube)
    assert (ga == -1).any() and np.isnan(g1).any()
    _, g1, ga = _check(svr, cube, min_t=1e30, max_t=2e30)
    assert (ga == -1).all() and np.isnan(g1).all()


@pytest.mark.parametrize("storage", ["f16", "bf16"])
def test_moments_half_storage(svr, storage):
    """16-bit cubes: the oracle sums the same dequantised values."""
    import torch
    cube = synth.disc_cube(40, 33, 64, 3, seed=7, dv_chan=8.0, centre_margin=10.0,
                           rd_range=(2.0, 5.0), zsys_margin=15.0)
    deq = quant.dequantize(cube, storage)
    t = to_cuda(cube).to(torch.float16 if storage == "f16" else torch.bfloat16)
    _check(svr, cube, gpu_cube=t, ref_cube=deq)


def test_moments_strided_view(svr):
    """A non-contiguous view (every second x column of a larger cube)."""
    cube = synth.disc_cube(64, 30, 40, 2, seed=8, dv_chan=8.0, centre_margin=10.0,
                           rd_range=(2.0, 5.0), zsys_margin=10.0)
    t = to_cuda(cube)[:, :, ::2]
    assert not t.is_contiguous()
    _check(svr, np.ascontiguousarray(cube[:, :, ::2]), gpu_cube=t)


def test_moments_full_size_sampled_spectra(svr):
    """512x512x1024 cube (the main workload), whole spectral axis, at the launch the
    benchmark times; 4000 spectra checked against the oracle one by one."""
    cube = synth.hi_cube_512x512x1024(0)
    m0, m1, am = svr.svr_moments(to_cuda(cube))
    svr.svr_sync()
    rng = np.random.default_rng(11)
    ys = rng.integers(0, 512, 4000)
    xs = rng.integers(0, 512, 4000)
    sub = np.ascontiguousarray(cube[:, ys, xs][:, None, :])
    r0, r1, ra = oracle.moments(sub)
    g0 = m0.cpu().numpy()[ys, xs]
    g1 = m1.cpu().numpy()[ys, xs]
    ga = am.cpu().numpy()[ys, xs]
    assert np.array_equal(g0.view(np.uint32), r0[0].astype(np.float32).view(np.uint32))
    assert np.array_equal(g1.view(np.uint32), r1[0].astype(np.float32).view(np.uint32))
    assert np.array_equal(ga, ra[0])


def test_moments_argmax_matches_mip1_location(svr):
    """Axis-aligned parallel MIP1 colours each pixel by the location of its ray's maximum.
    With one ray per voxel column and a step of half a channel every channel value is sampled
    exactly (the samples between lie between their neighbours), so the render's location is
    the moment map's argmax: loc.z = (argmax + 0.5) / nz (the argmax variant behaves like MIP,
    Section 2.2).  Columns whose two largest values normalise to within 1e-5 are skipped (the
    render compares normalised samples)."""
    cube = synth.blob_cube(24, 3, seed=4)
    nz, ny, nx = cube.shape
    _, _, am = svr.svr_moments(to_cuda(cube))
    vol = svr.svr_volume_create(to_cuda(cube))
    cam = synth.ortho_axis(nx, ny, nz, nx, ny, "+z").as_f32()
    lo, hi = quant.finite_minmax(cube)
    lut = np.zeros((nz, 4), np.float32)
    lut[:, 0] = np.arange(nz, dtype=np.float32) / (nz - 1)  # red = normalised location
    img = svr.svr_render(vol, cam, to_cuda(lut), mode="mip1", dt=0.5, clim_lo=lo, clim_hi=hi)
    svr.svr_sync()
    red = img.cpu().numpy()[..., 0]
    amax = am.cpu().numpy()
    srt = np.sort(cube, axis=0)
    robust = (srt[-1] - srt[-2]) > 1e-5 * (hi - lo)
    assert robust.mean() > 0.9
    ref = (amax + 0.5) / nz
    assert np.max(np.abs(red - ref)[robust]) < 1e-5


def test_moments_degenerate_shapes(svr):
    """One voxel; one spectrum; one channel over a row wider than a workgroup."""
    rng = np.random.default_rng(12)
    for shape in ((1, 1, 1), (37, 1, 1), (1, 3, 300), (40, 2, 257)):
        cube = rng.standard_normal(shape).astype(np.float32)
        _check(svr, cube)
        _check(svr, cube, dv=0.5, min_t=-0.5)
