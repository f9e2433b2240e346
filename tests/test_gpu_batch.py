"""Batched persistent rendering (one hipGraph-captured launch over many sub-cubes)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import quant
from helpers import compare_render, f32, to_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def svr():
    import paper_1707_00442_amd as m
    m.lib()
    return m


def _subcubes(count, seed, scale=0.25):
    """Uneven sub-cubes (sizes log-uniform as in the batched workload, scaled down)."""
    specs = synth.subcube_batch_specs(count, seed)
    out = []
    for sp in specs:
        sp = dict(sp)
        for k in ("nx", "ny", "nz"):
            sp[k] = max(3, int(round(sp[k] * scale)))
        sp["xc"] *= scale
        sp["yc"] *= scale
        sp["zsys"] *= scale
        sp["rd"] = max(1.0, sp["rd"] * scale)
        sp["dv_chan"] /= scale
        cube = synth.subcube(sp, dtype=np.float16).astype(np.float32)
        v = sp["view"] / np.linalg.norm(sp["view"])
        radius = 0.5 * np.sqrt(sp["nx"] ** 2 + sp["ny"] ** 2 + sp["nz"] ** 2)
        centre = ((sp["nx"] - 1) / 2, (sp["ny"] - 1) / 2, (sp["nz"] - 1) / 2)
        cam = synth.perspective_direction(centre, v, 2 * radius, 30.0, 48, 40).as_f32()
        out.append((cube, cam))
    return out


@pytest.mark.parametrize("mode", ["mip0", "mip1", "miprgb", "avip0", "avip1", "aviprgb"])
@pytest.mark.parametrize("tune", [False, True])
def test_batched_equals_single_renders(svr, mode, tune):
    import torch
    items = _subcubes(24, seed=3)
    lut = to_cuda(synth.lut_heat(256))
    vols = [svr.svr_volume_create(to_cuda(c), storage="f16") for c, _ in items]
    cams = [cam for _, cam in items]
    p = dict(mode=mode, k=0.22)
    b = svr.svr_batch_create(vols, cams, lut, p, tune=2 if tune else 0)
    assert b.items == sum(((c.width + 15) // 16) * ((c.height + 15) // 16) for c in cams) or tune
    if tune:
        print(f"  tuned: {b.stats}", flush=True)
    for rep in range(3):
        for o in b.outs:
            o.fill_(-1.0)
        b.launch()
        svr.svr_sync()
        for v, cam, o in zip(vols, cams, b.outs):
            ref = svr.svr_render(v, cam, lut, p)
            assert torch.equal(o, ref), f"replay {rep}"
        # eager work between graph replays
        _ = torch.ones(1000, device="cuda").sum().item()
    b.close()


def test_batched_parity_with_oracle(svr):
    items = _subcubes(6, seed=5)
    lut_np = synth.lut_heat(256)
    lut = to_cuda(lut_np)
    vols = [svr.svr_volume_create(to_cuda(c), storage="f16") for c, _ in items]
    p = dict(mode="avip0", k=0.3)
    b = svr.svr_batch_create(vols, [c for _, c in items], lut, p)
    b.launch()
    svr.svr_sync()
    for (cube, cam), v, o in zip(items, vols, b.outs):
        lo, hi = svr.svr_volume_clim(v)
        deq = quant.dequantize(cube, "f16")
        got = o.cpu().numpy().reshape(-1, 4).astype(np.float64)
        _, ns = svr.svr_render(v, cam, lut, p, samples=True)
        err, frag, _ = compare_render(oracle, got, ns.cpu().numpy().ravel(), deq, cam, lut_np,
                                      p, lo, hi, margins=dict(dv=2e-6 * (hi - lo), da=2e-6))
        assert err <= 1e-5
    b.close()


def test_batch_argument_checks(svr):
    c = synth.blob_cube(16, 1, seed=0)
    a = svr.svr_volume_create(to_cuda(c), storage="f16")
    b = svr.svr_volume_create(to_cuda(c), storage="f32")
    cam = synth.perspective_lookat(16, 16, 16, 10.0, 10.0, 40.0, 40.0, 16, 16)
    lut = to_cuda(synth.lut_ramp(16))
    with pytest.raises(svr.SvrError):
        svr.svr_batch_create([a, b], [cam, cam], lut, dict(mode="mip0"))
    with pytest.raises(svr.SvrError):
        svr.svr_batch_create([a], [cam], lut, dict(mode="mip0", ratio=1))


def test_autotune_cache_reuse_and_rebricked_copies(svr, tmp_path):
    """The autotuner (brick edge x tile x grid, median of three launches) stores its choice
    for the batch's size class in the cache file; a second batch of the same class takes
    it from there without timing.  A cached choice of the other brick edge makes the batch
    render from re-bricked copies: images still equal svr_render of the caller's volumes."""
    import torch
    cache = tmp_path / "tune.txt"
    svr.svr_set_tune_cache(str(cache))
    try:
        items = _subcubes(16, seed=7)
        lut = to_cuda(synth.lut_heat(256))
        vols = [svr.svr_volume_create(to_cuda(c), storage="f16") for c, _ in items]
        cams = [cam for _, cam in items]
        p = dict(mode="mip1", k=0.22)
        b1 = svr.svr_batch_create(vols, cams, lut, p, tune=2)
        s1 = b1.stats
        print(f"  searched: {s1}", flush=True)
        assert s1["from_cache"] == 0 and s1["brick"] in (8, 16)
        assert 0.0 < s1["tuned_ms"] <= s1["default_ms"]
        lines = cache.read_text().split()
        assert len(lines) == 4 and int(lines[1]) == s1["brick"]
        b2 = svr.svr_batch_create(vols, cams, lut, p, tune=1)
        s2 = b2.stats
        assert s2["from_cache"] == 1
        assert (s2["brick"], s2["tile_waves_x"], s2["grid"]) == \
            (s1["brick"], s1["tile_waves_x"], s1["grid"])
        b1.close()
        b2.close()
        # force the brick edge the caller's volumes do not have (16) through the cache
        key = lines[0]
        cache.write_text(f"{key} 16 4 2\n")
        b3 = svr.svr_batch_create(vols, cams, lut, p, tune=1)
        s3 = b3.stats
        assert s3["from_cache"] == 1 and s3["brick"] == 16 and s3["tile_waves_x"] == 4
        for rep in range(2):
            for o in b3.outs:
                o.fill_(-1.0)
            b3.launch()
            svr.svr_sync()
            for v, cam, o in zip(vols, cams, b3.outs):
                assert torch.equal(o, svr.svr_render(v, cam, lut, p)), f"replay {rep}"
        b3.close()
        # a different size class (other transfer function) is not taken from the cache
        b4 = svr.svr_batch_create(vols, cams, lut, dict(p, mode="avip0"), tune=1)
        assert b4.stats["from_cache"] == 0
        b4.close()
        assert len(cache.read_text().splitlines()) == 2
    finally:
        svr.svr_set_tune_cache(None)


def test_batch_tune_argument_checked(svr):
    c = synth.blob_cube(16, 1, seed=0)
    a = svr.svr_volume_create(to_cuda(c), storage="f16")
    cam = synth.perspective_lookat(16, 16, 16, 10.0, 10.0, 40.0, 40.0, 16, 16)
    lut = to_cuda(synth.lut_ramp(16))
    with pytest.raises(svr.SvrError):
        svr.svr_batch_create([a], [cam], lut, dict(mode="mip0"), tune=3)
