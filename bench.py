#!/usr/bin/env python
"""Benchmark of the ray-cast colouring/filtering hot path on one MI355X.

Workload (one step): the 512 x 512 x 1024 float32 HI-like cube (noise + 50 rotating discs,
seed 0) seen by a perspective camera at 1920 x 1080 from the next view of a full rotation
(azimuth step 10 deg, elevation 20 deg, distance twice the half-diagonal, vertical field of
view 40 deg), dt = 0.5 voxel:
  * separable 3D Gaussian smoothing with sigma = 1, 2, 3 voxels (three passes each);
  * upload of the cube into the bricked float32 volume (finite min/max, NaN fill, apron);
  * the six transfer functions (MIP0, MIP1, MIP_RGB, AVIP0, AVIP1, AVIP_RGB; k = 0.22,
    clipping at minT = 3 sigma);
  * the voxel-wise line ratio of the spectral windows [400, 432) and [600, 632), and the
    two in-ray line-ratio methods over a 512 x 512 x 32 two-line pair (the windows' grid:
    an extended source in a strong and a 0.4 times fainter line, unit noise, both clipped at
    3 sigma).
value = ray samples processed per second over the whole step (samples counted per pixel
by the renderer itself, verified against the oracle in the tests).

Further forms are timed after the main loop (reported, not part of `value`): float16 and
bfloat16 storage, the differentiable forward + adjoint, and the batched persistent launch
of 512 sub-cubes.  The oracle (FP64, C, OpenMP) is timed on a bounded sample of pixels of
the same workload on this machine's host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("ray samples/sec and frames/sec @1920x1080 (fwd, fwd+bwd) vs FP32 plain; "
          "HBM GB/s")
PEAK_HBM = 8.0e12            # bytes/s
PEAK_ALU = 256 * 64 * 2.4e9  # VALU lane operations/s (256 CUs x 4 SIMD x 16 lanes x 2.4 GHz)

# Algorithmic VALU operations per sample (the arithmetic the method itself needs; address
# generation, loads and loop control are not counted).  Shared by every transfer function:
# position 3 (p0 + k step), clamp 3, cell 3 (floor), fraction 3, trilinear 14 (7 lerps of
# sub + fma) = 26; clipping filter 3 (two compares, one select) + normalise 1 (fma with
# clamp) = 4.  MIP0 adds 1 (max), MIP1/MIP_RGB 3 (compare + 2 selects).  AVIP adds the
# compositing step 14 (alpha2 2, alpha 2, rcp 1, weights 2, colour 6, termination 1) and
# its opacity 1, plus the colour: table lookup 11 (scale, floor, fraction, 4 lerps) for
# AVIP0 and AVIP1 (AVIP1 also 2 for loc.z), 3 for AVIP_RGB (loc).
OPS_PER_SAMPLE = {"mip0": 31, "mip1": 33, "miprgb": 33, "avip0": 56, "avip1": 58,
                  "aviprgb": 48, "ratio1": 26 * 2 + 6 + 2, "ratio2": 26 * 2 + 6 + 4}
MODES = ("mip0", "mip1", "miprgb", "avip0", "avip1", "aviprgb")
# sources of each kernel family (recorded counters are void once any of them changes)
KERNEL_SOURCES = {
    "render": ("common.h", "sampler.h", "march.h", "render.hip"),
    "smooth": ("common.h", "smooth.hip"),
    "line_ratio": ("common.h", "smooth.hip"),
    "upload": ("common.h", "volume.hip"),
    "train": ("common.h", "sampler.h", "train.hip"),
    "moments": ("common.h", "moments.hip"),
    "copy": (),
}


def kernel_family(kernel):
    for fam in ("render", "smooth", "line_ratio", "upload", "train", "moments", "copy"):
        if kernel.startswith(fam):
            return fam
    raise KeyError(kernel)


def _code_only(text):
    """C++ source without comments and blank space: edits to comments leave it unchanged.
    (String and character literals in these sources hold no comment markers.)"""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def source_hash(kernel):
    """Hash of the code (comments stripped) of the sources a kernel family is built from."""
    h = hashlib.sha256()
    for n in KERNEL_SOURCES[kernel_family(kernel)]:
        with open(os.path.join(ROOT, "paper_1707_00442_amd", "csrc", n)) as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-forms", action="store_true", help="skip the extra forms")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--protocol", action="store_true",
                    help="instead of the step: the paper's frame-rate protocol (uniform [0,1] "
                         "cubes 128^3..1024^3, raw and box 3..11, MIP0 and AVIP0, median fps "
                         "over a full rotation x3 at 1000x1000, and the canvas sweep)")
    ap.add_argument("--summarize", default=None, metavar="DIR",
                    help="summarise rocprofv3 output written under DIR (trace/ from a "
                         "--kernel-trace --stats run of the step, pmc_<kernel>_<COUNTER>/ from "
                         "--pmc runs of --profile <kernel>, and sq_/ta_/tcp_<kernel>/ from the "
                         "three render counter passes) into markdown on stdout and "
                         "profiles/traffic.json; no GPU needed")
    ap.add_argument("--profile", default=None,
                    help="run only this kernel on the main workload, --steps times (for "
                         "rocprofv3): render_<mode>, render_sparse, smooth_sigma<s>, upload, "
                         "line_ratio, moments, train_fwd, train_bwd, copy (a 1 GiB device copy used to "
                         "scale the counters)")
    return ap.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every svr call is enqueued on)."""

    def __init__(self, torch):
        self.torch = torch
        self.spans = {}

    def span(self, name):
        t = self.torch
        e0, e1 = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        outer = self

        class _S:
            def __enter__(self):
                e0.record()

            def __exit__(self, *a):
                e1.record()
                outer.spans.setdefault(name, []).append((e0, e1))
        return _S()

    def ms(self, name):
        return [a.elapsed_time(b) for a, b in self.spans.get(name, [])]


def roofline_entry(bound, achieved, peak, unit, traffic=None):
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": traffic}


def load_traffic(kernel):
    """HBM bytes per launch of `kernel` measured with rocprofv3 counters (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy kernel of known size), if recorded for the current source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(kernel)
        if e and e.get("source_hash") == source_hash(kernel):
            return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


# kernels each --profile mode launches per call (rocprofv3 kernel-name prefixes)
PROFILE_KERNELS = {
    "render": ("svr::render_kernel<", "svr::split_clear_kernel", "svr::render_split_kernel<",
               "svr::split_finalize_kernel<"),
    "smooth": ("svr::smooth_fused_kernel<",),
    "upload": ("svr::upload_init", "svr::brick_group_kernel<", "svr::upload_final<",
               "svr::upload_fill<"),
    "moments": ("svr::moments_kernel<",),
    "line_ratio": ("svr::line_ratio_kernel<", "svr::line_ratio_vec4_kernel<"),
    "copy": ("__amd_rocclr_copyBuffer",),
}


def _kernel_name(name):
    """A rocprofv3 kernel name without 'void ' and its argument list."""
    name = name[5:] if name.startswith("void ") else name
    depth = 0
    for i, ch in enumerate(name):
        depth += ch == "<"
        depth -= ch == ">"
        if ch == "(" and depth == 0:
            return name[:i]
    return name


def _per_call(path, kernel, calls):
    """Counter value per call of `kernel` (KiB): the last `calls` dispatches of each of the
    kernels that call launches, summed over those kernels, averaged over the calls.  Kernels
    of the family that the call does not launch (the split MIP kernels of a one-pass render)
    have no dispatches and are skipped."""
    import csv
    rows = list(csv.DictReader(open(path)))
    total = 0.0
    found = 0
    for prefix in PROFILE_KERNELS[kernel_family(kernel)]:
        vals = [float(r["Counter_Value"]) for r in rows
                if _kernel_name(r["Kernel_Name"]).startswith(prefix)]
        if not vals:
            continue
        if len(vals) < calls:
            raise SystemExit(f"{path}: {len(vals)} dispatches of {prefix}, expected {calls}")
        total += sum(vals[-calls:])
        found += 1
    if not found:
        raise SystemExit(f"{path}: no dispatches of the {kernel} kernels")
    return total / calls


def summarize(d, calls=20):
    """Markdown tables from rocprofv3 output under d, and profiles/traffic.json: HBM bytes per
    launch = FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what the same
    counter reads for a 1 GiB device copy (bytes read and written are known)."""
    import csv
    import glob
    out = []
    stats = glob.glob(os.path.join(d, "trace", "*_kernel_stats.csv"))
    if stats:
        rows = list(csv.DictReader(open(stats[0])))
        out.append("| kernel | calls | average (ms) | min (ms) | max (ms) | share |")
        out.append("|---|---|---|---|---|---|")
        for r in rows:
            if not r["Name"].startswith("void svr::") and "svr::" not in r["Name"]:
                continue
            out.append(f"| `{_kernel_name(r['Name'])}` | {r['Calls']} | "
                       f"{float(r['AverageNs']) / 1e6:.4f} | {float(r['MinNs']) / 1e6:.4f} | "
                       f"{float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f}% |")
        out.append("")
    pmc = {}
    for path in glob.glob(os.path.join(d, "pmc_*_*_SIZE", "*counter_collection.csv")):
        tag = os.path.basename(os.path.dirname(path))[4:]
        kernel, counter = tag.rsplit("_", 2)[0], "_".join(tag.rsplit("_", 2)[1:])
        pmc.setdefault(kernel, {})[counter] = _per_call(path, kernel, calls)
    if pmc:
        copy = pmc.pop("copy")
        f_fetch = 2.0 ** 30 / (copy["FETCH_SIZE"] * 1024.0)
        f_write = 2.0 ** 30 / (copy["WRITE_SIZE"] * 1024.0)
        out.append(f"Calibration: a 1 GiB device copy reads {copy['FETCH_SIZE'] / 2 ** 20:.4f} "
                   f"GiB by FETCH_SIZE and writes {copy['WRITE_SIZE'] / 2 ** 20:.4f} GiB by "
                   f"WRITE_SIZE: FETCH_SIZE x {f_fetch:.3f}, WRITE_SIZE x {f_write:.3f}.")
        out.append("")
        out.append("| kernel | fetched (GB) | written (GB) | total (GB) | calls |")
        out.append("|---|---|---|---|---|")
        traffic = {}
        for k in sorted(pmc):
            fb = pmc[k]["FETCH_SIZE"] * 1024.0 * f_fetch
            wb = pmc[k]["WRITE_SIZE"] * 1024.0 * f_write
            out.append(f"| {k} | {fb / 1e9:.3f} | {wb / 1e9:.4f} | {(fb + wb) / 1e9:.3f} | "
                       f"{calls} |")
            traffic[k] = dict(bytes_per_launch=fb + wb, fetched=fb, written=wb,
                              source_hash=source_hash(k))
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as f:
            json.dump(traffic, f, indent=1)
    out += _counter_tables(d, calls)
    print("\n".join(out))


def _counter_tables(d, calls):
    """Render counter passes (sq_<kernel>/, ta_<kernel>/, tcp_<kernel>/ under d): means per
    call summed over the kernels one call launches, and the derived shares (VALU issue =
    SQ_INSTS_VALU x 4 / (1024 SIMDs x C), C = GRBM_GUI_ACTIVE / 8 cycles per launch)."""
    import csv
    import glob
    from collections import defaultdict
    kernels = sorted({os.path.basename(p).split("_", 1)[1]
                      for p in glob.glob(os.path.join(d, "sq_*")) if os.path.isdir(p)})
    if not kernels:
        return []
    res = {}
    for k in kernels:
        vals, ms = defaultdict(float), 0.0
        for grp in ("sq", "ta", "tcp"):
            path = glob.glob(os.path.join(d, f"{grp}_{k}", "*counter_collection.csv"))[0]
            rows = list(csv.DictReader(open(path)))
            for prefix in PROFILE_KERNELS[kernel_family(k)]:
                by = defaultdict(dict)
                for r in rows:
                    if _kernel_name(r["Kernel_Name"]).startswith(prefix):
                        by[int(r["Dispatch_Id"])][r["Counter_Name"]] = (
                            float(r["Counter_Value"]),
                            int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
                ids = sorted(by)[-calls:]
                for i in ids:
                    for c, (v, _) in by[i].items():
                        vals[c] += v / calls
                if grp == "ta" and ids:
                    ms += sum(next(iter(by[i].values()))[1] for i in ids) / calls / 1e6
        res[k] = (vals, ms)
    out = ["", "| kernel | ms | clock (GHz) | waves | VALU instr / wave | loads / wave | "
           "VALU issue | TA busy | waiting | L1 lookups / load | to L2 | L1 pending stall | "
           "TD stall on L2 |", "|" + "---|" * 13]
    for k, (v, ms) in res.items():
        c = v["GRBM_GUI_ACTIVE"] / 8
        w = v["SQ_WAVES"]
        out.append(
            f"| {k} | {ms:.3f} | {c / (ms * 1e-3) / 1e9:.2f} | {w:.0f} | "
            f"{v['SQ_INSTS_VALU'] / w:.0f} | {v['SQ_INSTS_VMEM_RD'] / w:.0f} | "
            f"{v['SQ_INSTS_VALU'] * 4 / (1024 * c):.0%} | {v['TA_BUSY_avr'] / c:.0%} | "
            f"{v['SQ_WAIT_INST_ANY'] / v['SQ_WAVE_CYCLES']:.0%} | "
            f"{v['TCP_TOTAL_CACHE_ACCESSES_sum'] / v['SQ_INSTS_VMEM_RD']:.1f} | "
            f"{v['TCP_TCC_READ_REQ_sum'] / v['TCP_TOTAL_CACHE_ACCESSES_sum']:.1%} | "
            f"{v['TCP_PENDING_STALL_CYCLES_sum'] / (256 * c):.0%} | "
            f"{v['TD_TC_STALL_sum'] / (256 * c):.0%} |")
    keys = sorted(set().union(*[set(v) for v, _ in res.values()]))
    out += ["", "| kernel | " + " | ".join(keys) + " |", "|---|" + "---|" * len(keys)]
    for k, (v, _) in res.items():
        out.append(f"| {k} | " + " | ".join(f"{v[c]:.4g}" for c in keys) + " |")
    return out


def main():
    args = parse()
    if args.summarize:
        return summarize(args.summarize, calls=args.steps)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the split over several GPUs is a design, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1707_00442_amd as svr
    import synth
    from paper_1707_00442_amd import taps as tapgen

    torch.cuda.set_device(0)
    svr.lib()
    if args.protocol:
        return run_protocol(torch, svr, synth)
    t_setup = time.time()
    nx, ny, nz = 512, 512, 1024
    W, H = 1920, 1080
    log("building the 512x512x1024 cube")
    cube_np = synth.hi_cube_512x512x1024(0)
    cube = torch.from_numpy(cube_np).cuda()
    lo, hi = svr.svr_minmax(cube)
    views = [v.as_f32() for v in synth.rotation_views(nx, ny, nz, W, H)]
    lut = torch.from_numpy(synth.lut_heat(256)).cuda()
    vol = svr.svr_volume_create(cube, storage="f32")
    # in-ray line ratios: a two-line pair on the grid of two 32-channel windows (an extended
    # source in a strong and a 0.4 times fainter line); the voxel-wise pass runs on the
    # windows [400, 432) and [600, 632) of the cube itself
    pair_a, pair_b = synth.two_line_pair_512x512x32(0)
    vol_a = svr.svr_volume_create(torch.from_numpy(pair_a).cuda())
    vol_b = svr.svr_volume_create(torch.from_numpy(pair_b).cuda())
    del pair_a, pair_b
    ratio_views = [v.as_f32() for v in synth.rotation_views(nx, ny, 32, W, H)]
    taps = {s: tapgen.gauss(float(s)).astype(np.float32) for s in (1, 2, 3)}
    smooth_out = torch.empty_like(cube)
    ws = None  # the fused 7/13/19-tap passes need no workspace
    assert all(svr.svr_smooth_workspace(cube, len(taps[s])) == 0 for s in taps)
    ratio_out = torch.empty((32, ny, nx), dtype=torch.float32, device="cuda")
    imgs = {m: torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for m in MODES}
    rimg = {r: torch.empty((H, W, 4), dtype=torch.float32, device="cuda") for r in (1, 2)}
    params = {m: dict(mode=m, k=0.22, filter="clip", min_t=3.0, clim_lo=lo, clim_hi=hi)
              for m in MODES}
    rlo, rhi = svr.svr_volume_clim(vol_a)
    rparams = {r: dict(mode="mip0", ratio=r, filter="clip", min_t=3.0, min_t2=3.0,
                       clim_lo=rlo, clim_hi=rhi, ratio_lo=0.0, ratio_hi=1.0) for r in (1, 2)}

    K, Wu = args.steps, args.warmup
    if args.profile:
        return profile_one(args, torch, svr, synth, cube, vol, views, lut, params, taps,
                           smooth_out, ws, ratio_out, lo)
    # per-pixel sample counts of every render the timed steps will run (untimed)
    log("counting samples per view")
    samples = {}
    for i in range(Wu, Wu + K):
        cam = views[i % len(views)]
        for m in MODES:
            _, ns = svr.svr_render(vol, cam, lut, params[m], samples=True)
            samples[(i, m)] = int(ns.sum().item())
        rc = ratio_views[i % len(ratio_views)]
        for r in (1, 2):
            _, ns = svr.svr_render(vol_a, rc, lut, rparams[r], vol2=vol_b, samples=True)
            samples[(i, f"ratio{r}")] = int(ns.sum().item())
    torch.cuda.synchronize()

    timer = Timer(torch)

    def step(i, timed):
        cam = views[i % len(views)]
        tm = timer if timed else None

        def span(name):
            return tm.span(name) if tm else _Null()
        for s in (1, 2, 3):
            with span(f"smooth_sigma{s}"):
                svr.svr_smooth(cube, taps[s], out=smooth_out, workspace=ws)
        with span("upload"):
            svr.svr_volume_upload(vol, cube)
        for m in MODES:
            with span(f"render_{m}"):
                svr.svr_render(vol, cam, lut, params[m], out=imgs[m])
        with span("line_ratio"):
            svr.svr_line_ratio(cube, 400, 600, 32, datamin=lo, out=ratio_out)
        rc = ratio_views[i % len(ratio_views)]
        for r in (1, 2):
            with span(f"render_ratio{r}"):
                svr.svr_render(vol_a, rc, lut, rparams[r], vol2=vol_b, out=rimg[r])

    log(f"warmup {Wu} steps")
    for i in range(Wu):
        step(i, False)
    torch.cuda.synchronize()
    log(f"timing {K} steps")
    t0 = time.perf_counter()
    for i in range(Wu, Wu + K):
        step(i, True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / K
    total_samples = sum(samples.values())
    value = total_samples / elapsed
    render_samples = sum(v for (i, m), v in samples.items() if m in MODES)
    frames = K * len(MODES)

    # per-kernel figures from the HIP events
    nvox = nx * ny * nz
    kernels = {}
    for m in MODES + ("ratio1", "ratio2"):
        ms = timer.ms(f"render_{m}")
        ns = [samples[(i, m)] for i in range(Wu, Wu + K)]
        ops = np.array(ns, dtype=np.float64) * OPS_PER_SAMPLE[m]
        kernels[f"render_{m}"] = dict(
            ms_mean=float(np.mean(ms)), samples_per_s=float(np.sum(ns) / (np.sum(ms) * 1e-3)),
            fps=float(1e3 / np.mean(ms)),
            alu_ops_per_s=float(np.sum(ops) / (np.sum(ms) * 1e-3)))
    for s in (1, 2, 3):
        # the operation reads the cube once and writes it once (the implementation's two
        # passes move 16 B per voxel: see profiles/)
        ms = timer.ms(f"smooth_sigma{s}")
        kernels[f"smooth_sigma{s}"] = dict(ms_mean=float(np.mean(ms)),
                                           hbm_bytes_algorithmic=8 * nvox,
                                           gbps=8 * nvox / (np.mean(ms) * 1e-3) / 1e9)
    ms = timer.ms("upload")
    kernels["upload"] = dict(ms_mean=float(np.mean(ms)), hbm_bytes_algorithmic=8 * nvox,
                             gbps=8 * nvox / (np.mean(ms) * 1e-3) / 1e9)
    ms = timer.ms("line_ratio")
    nr = 32 * nx * ny
    kernels["line_ratio"] = dict(ms_mean=float(np.mean(ms)), hbm_bytes_algorithmic=12 * nr,
                                 gbps=12 * nr / (np.mean(ms) * 1e-3) / 1e9)
    # dominant kernel: the largest share of the step
    share = {k: v["ms_mean"] for k, v in kernels.items()}
    dominant = max(share, key=share.get)
    if dominant.startswith("render_"):
        m = dominant[len("render_"):]
        ach = kernels[dominant]["alu_ops_per_s"] / 1e12
        roof = roofline_entry("alu", ach, PEAK_ALU / 1e12, "Tops/s",
                              load_traffic(dominant))
        roof["kernel"] = dominant
        roof["ops_per_sample"] = OPS_PER_SAMPLE[m]
    else:
        ach = kernels[dominant]["gbps"]
        roof = roofline_entry("hbm", ach, PEAK_HBM / 1e9, "GB/s", load_traffic(dominant))
        roof["kernel"] = dominant

    out = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1, "steps": K,
        "warmup": Wu, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "HI-like cube 512x512x1024 float32 (noise + 50 discs, seed 0); "
                               "perspective 1920x1080 rotation views, dt 0.5; per step: "
                               "smooth sigma 1,2,3 + upload + 6 transfer functions (clip "
                               "minT 3) + voxel-wise line ratio of windows [400,432)/"
                               "[600,632) + the two in-ray ratio methods on a 512x512x32 "
                               "two-line pair (clip 3 sigma)",
                   "image": [W, H], "cube": [nx, ny, nz], "dt": 0.5},
        "fps_render": frames / (sum(sum(timer.ms(f"render_{m}")) for m in MODES) * 1e-3),
        "render_samples_per_s": render_samples / (sum(sum(timer.ms(f"render_{m}"))
                                                       for m in MODES) * 1e-3),
        "roofline": roof,
        "kernels": kernels,
    }
    # pixels the in-ray ratio methods coloured in the last timed step (rays through the
    # source of the line pair), and voxels of the ratio pass that carry a ratio
    out["ratio_coloured_pixels"] = {f"method{r}": int((rimg[r].abs().sum(dim=2) > 0).sum())
                                    for r in (1, 2)}
    out["line_ratio_voxels_with_ratio"] = int((ratio_out != lo).sum().item())
    log(f"main: {value:.4g} samples/s, {ms_per_step:.2f} ms/step, dominant {dominant}")

    if not args.no_forms:
        out["forms"] = run_forms(torch, svr, synth, cube, lo, hi, views, lut, params,
                                 kernels, args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cube_np, views[Wu], synth, lo, hi, args)
    log(f"total {time.time() - t_setup:.1f}s")
    print(json.dumps(out), flush=True)


def run_protocol(torch, svr, synth, sizes=(128, 256, 512, 1024), canvas=1000, reps=3):
    """The paper's frame-rate benchmark (Section 6, Appendix B) on this GPU: uniform [0, 1)
    float32 cubes, one sample per voxel (dt = 1), the rotation views (10 degree steps), each
    frame timed on its own; fps = 1000 / median frame time over `reps` full rotations.
    Kernels: raw, box smoothing of 3..11 samples (filterArm 1..5) and the in-ray N-tap
    Gaussians (N = 5, 9, 13); MIP0, and AVIP0 with k = 0.22 and clipping at minThreshold = 0.9
    (the paper's settings).  Canvas sweep: MIP0 raw at 500^2 .. 2000^2."""
    from paper_1707_00442_amd import taps as tapgen
    lut = torch.from_numpy(synth.lut_heat(256)).cuda()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def median_fps(vol, views, p, out):
        ms = []
        for _ in range(reps):
            for cam in views:
                e0.record()
                svr.svr_render(vol, cam, lut, p, out=out)
                e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
        return 1e3 / float(np.median(ms))

    res = {"fps": {}, "canvas": {}}
    for n in sizes:
        log(f"protocol: {n}^3 uniform cube")
        cube = torch.from_numpy(synth.uniform_cube(n, seed=0)).cuda()
        lo, hi = svr.svr_minmax(cube)
        vol = svr.svr_volume_create(cube)
        del cube
        views = [v.as_f32() for v in synth.rotation_views(n, n, n, canvas, canvas)]
        out = torch.empty((canvas, canvas, 4), dtype=torch.float32, device="cuda")
        kernels = [("raw", {})] + [(f"box{2 * a + 1}", dict(box_arm=a)) for a in range(1, 6)]
        kernels += [(f"gauss{N}", dict(star=tapgen.star(N))) for N in (5, 9, 13)]
        for mode in ("mip0", "avip0"):
            for name, extra in kernels:
                p = dict(mode=mode, k=0.22, dt=1.0, clim_lo=lo, clim_hi=hi, **extra)
                if mode == "avip0":
                    p.update(filter="clip", min_t=0.9)
                svr.svr_render(vol, views[0], lut, p, out=out)
                res["fps"][f"{n}^3 {mode} {name}"] = round(median_fps(vol, views, p, out), 1)
                log(f"protocol: {n}^3 {mode} {name}: {res['fps'][f'{n}^3 {mode} {name}']} fps")
        for cv in (500, 1000, 1500, 2000):
            cviews = [v.as_f32() for v in synth.rotation_views(n, n, n, cv, cv)]
            cout = torch.empty((cv, cv, 4), dtype=torch.float32, device="cuda")
            p = dict(mode="mip0", dt=1.0, clim_lo=lo, clim_hi=hi)
            svr.svr_render(vol, cviews[0], lut, p, out=cout)
            res["canvas"][f"{n}^3 {cv}x{cv}"] = round(median_fps(vol, cviews, p, cout), 1)
        vol.close()
        log(f"protocol: {n}^3 done")
    print(json.dumps({"protocol": "paper frame-rate benchmark (uniform cubes, dt = 1, "
                                  "rotation median x3)", "canvas_px": canvas, **res}),
          flush=True)


def sparse_camera(synth):
    """Parallel view along +z, 256x256 over the 512x512 face, dt = 1: 0.25 samples per
    voxel, every voxel touched once (the HBM-bound corner of the ray-march)."""
    return synth.ortho_axis(512, 512, 1024, 256, 256, "+z").as_f32()


def profile_one(args, torch, svr, synth, cube, vol, views, lut, params, taps, smooth_out, ws,
                ratio_out, lo):
    """Run one kernel --steps times on the views the timed loop renders (after --warmup),
    so per-launch counters compare with the timed per-launch figures."""
    name = args.profile
    cams = [views[(args.warmup + i) % len(views)] for i in range(args.steps)]
    it = iter(range(args.steps))
    if name == "copy":
        a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        fn = lambda: b.copy_(a)  # noqa: E731
    elif name == "render_sparse":
        c = sparse_camera(synth)
        p = dict(params["mip0"], dt=1.0)
        fn = lambda: svr.svr_render(vol, c, lut, p)  # noqa: E731
    elif name.startswith("render_"):
        m = name[len("render_"):]
        fn = lambda: svr.svr_render(vol, cams[next(it)], lut, params[m])  # noqa: E731
    elif name.startswith("smooth_sigma"):
        s = int(name[-1])
        fn = lambda: svr.svr_smooth(cube, taps[s], out=smooth_out, workspace=ws)  # noqa: E731
    elif name == "upload":
        fn = lambda: svr.svr_volume_upload(vol, cube)  # noqa: E731
    elif name == "line_ratio":
        fn = lambda: svr.svr_line_ratio(cube, 400, 600, 32, datamin=lo, out=ratio_out)  # noqa: E731
    elif name == "moments":
        mom = svr.svr_moments(cube)
        fn = lambda: svr.svr_moments(cube, out=mom)  # noqa: E731
    elif name in ("train_fwd", "train_bwd"):
        # the differentiable form: 256^3 cube, 1024x1024, 64-point transfer function
        c4 = torch.from_numpy(synth.disc_cube_256(0)).cuda()
        l4, h4 = svr.svr_minmax(c4)
        v4 = svr.svr_volume_create(c4)
        tf = torch.from_numpy(synth.tf_ramp(64)).cuda()
        p4 = dict(mode="avip0", opacity_from_lut=1, k=0.22, clim_lo=l4, clim_hi=h4)
        cam4 = synth.perspective_lookat(256, 256, 256, 30.0, 20.0, 256 * 3 ** 0.5, 40.0,
                                        1024, 1024).as_f32()
        img, wsp = svr.svr_render_train(v4, cam4, tf, p4)
        g = torch.randn(1024, 1024, 4, device="cuda")
        gtf, gvox = torch.zeros_like(tf), torch.zeros_like(c4)
        if name == "train_fwd":
            fn = lambda: svr.svr_render_train(v4, cam4, tf, p4, out=img, workspace=wsp)  # noqa: E731,E501
        else:
            fn = lambda: svr.svr_render_backward(v4, cam4, tf, p4, wsp, g, grad_tf=gtf,  # noqa: E731
                                                 grad_vox=gvox)
    else:
        raise SystemExit(f"unknown kernel {name}")
    for i in range(args.steps):
        fn()
        torch.cuda.synchronize()
        log(f"profile {name}: call {i + 1}/{args.steps} done")
    print(json.dumps({"profiled": name, "calls": args.steps, "source_hash": source_hash(name)}))


class _Null:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def _time(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def run_forms(torch, svr, synth, cube, lo, hi, views, lut, params, kernels, args):
    forms = {}
    cam = views[0]
    plain = {}
    vol32 = _vol32(svr, cube)
    for m in ("mip0", "avip0"):
        _, ns = svr.svr_render(vol32, cam, lut, params[m], samples=True)
        n = int(ns.sum().item())
        ms = _time(torch, lambda: svr.svr_render(vol32, cam, lut, params[m]), 5)
        plain[m] = dict(ms=ms, samples_per_s=n / (ms * 1e-3), fps=1e3 / ms)
    forms["fp32_plain"] = plain
    # the paper's Section 6 protocol on this workload: every frame of the full rotation (36
    # views, 10 degree steps) timed on its own, fps = 1000 / median frame time
    log("form: rotation median")
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    img = torch.empty((cam.height, cam.width, 4), dtype=torch.float32, device="cuda")
    rot = {}
    for m in MODES:
        ms = []
        for v in views:
            ev0.record()
            svr.svr_render(vol32, v, lut, params[m], out=img)
            ev1.record()
            ev1.synchronize()
            ms.append(ev0.elapsed_time(ev1))
        rot[m] = dict(fps_median=1e3 / float(np.median(ms)), ms_min=float(np.min(ms)),
                      ms_max=float(np.max(ms)), views=len(ms))
    forms["rotation_36_views"] = rot
    # the voxel-wise line-ratio pass: one 32-channel window pair is ~12 us of HBM time, so
    # it is also timed over the 32 window offsets back to back and on 256-channel windows
    nx_, ny_ = cube.shape[2], cube.shape[1]
    rout = torch.empty((256, ny_, nx_), dtype=torch.float32, device="cuda")

    def offsets():
        for j in range(32):
            svr.svr_line_ratio(cube, 400 + j, 600 + j, 32, datamin=lo, out=rout[:32])
    ms32 = _time(torch, offsets, 5) / 32
    ms256 = _time(torch, lambda: svr.svr_line_ratio(cube, 0, 512, 256, datamin=lo, out=rout), 5)
    b32, b256 = 12 * 32 * nx_ * ny_, 12 * 256 * nx_ * ny_
    forms["line_ratio_pass"] = dict(
        offsets32_ms_per_launch=ms32, offsets32_gbps=b32 / (ms32 * 1e-3) / 1e9,
        window256_ms=ms256, window256_gbps=b256 / (ms256 * 1e-3) / 1e9,
        window256_hbm_frac=b256 / (ms256 * 1e-3) / PEAK_HBM)
    del rout
    # low sample density: HBM-bound ray-march
    c = sparse_camera(synth)
    p = dict(params["mip0"], dt=1.0)
    _, ns = svr.svr_render(vol32, c, lut, p, samples=True)
    n = int(ns.sum().item())
    ms = _time(torch, lambda: svr.svr_render(vol32, c, lut, p), 10)
    nbytes = 4 * cube.numel()
    forms["sparse_mip0"] = dict(ms=ms, samples=n, samples_per_voxel=n / cube.numel(),
                                samples_per_s=n / (ms * 1e-3),
                                hbm_bytes_algorithmic=nbytes,
                                gbps=nbytes / (ms * 1e-3) / 1e9,
                                hbm_frac=nbytes / (ms * 1e-3) / PEAK_HBM,
                                stored_bytes=vol32.nbytes)
    # the same view from 16-voxel bricks (smaller apron) and from 16-bit storage: the
    # algorithmic bytes are the voxels' (4 or 2 B each); stored_bytes is what the layout holds
    for st, br in (("f32", 16), ("f16", 8), ("bf16", 8)):
        v = svr.svr_volume_create(cube, storage=st, brick=br)
        ms = _time(torch, lambda: svr.svr_render(v, c, lut, p), 10)
        nb = (4 if st == "f32" else 2) * cube.numel()
        forms[f"sparse_mip0_{st}_brick{br}"] = dict(
            ms=ms, samples_per_s=n / (ms * 1e-3), hbm_bytes_algorithmic=nb,
            gbps=nb / (ms * 1e-3) / 1e9, hbm_frac=nb / (ms * 1e-3) / PEAK_HBM,
            stored_bytes=v.nbytes, stored_gbps=v.nbytes / (ms * 1e-3) / 1e9)
        v.close()
    # split MIP rays: an oblique view with few rays (256 x 256, rotation view 3, dt 0.5), each ray
    # rendered in segments on several workgroups; the batched kernel renders the same view in
    # one pass (its own tuning: context, not an A/B of the split alone)
    cs = synth.rotation_views(512, 512, 1024, 256, 256)[3].as_f32()
    r = {}
    for m in ("mip0", "mip1"):
        pm = params[m]
        _, ns = svr.svr_render(vol32, cs, lut, pm, samples=True)
        n = int(ns.sum().item())
        ms = _time(torch, lambda: svr.svr_render(vol32, cs, lut, pm), 10)
        b = svr.svr_batch_create([vol32], [cs], lut, pm, tune=0)
        ms_b = _time(torch, b.launch, 10)
        b.close()
        r[m] = dict(ms=ms, segments=svr.svr_render_segments(vol32, cs, pm),
                    samples_per_s=n / (ms * 1e-3), batched_one_pass_ms=ms_b)
    forms["small_oblique_view_split"] = r
    # the paper's in-ray 9-tap Gaussian (13 trilinear fetches per sample), view 0
    star9 = (0.2270270270, [(1.3846153846, 0.3162162162), (3.2307692308, 0.0702702703)])
    r = {}
    for m in ("mip0", "avip0"):
        ps = dict(params[m], star=star9)
        _, ns = svr.svr_render(vol32, cam, lut, ps, samples=True)
        n = int(ns.sum().item())
        ms = _time(torch, lambda: svr.svr_render(vol32, cam, lut, ps), 3)
        r[m] = dict(ms=ms, samples_per_s=n / (ms * 1e-3), fetches_per_s=13 * n / (ms * 1e-3),
                    fps=1e3 / ms)
    forms["star9_in_ray_gaussian"] = r
    # the 64^3 blob cube (noise + 3 blobs), parallel view along +z at 256 x 256, dt = 0.5 (128
    # samples per ray), ramp table: float32, float16 and bfloat16 storage
    log("form: 64^3 blob cube")
    c0 = torch.from_numpy(synth.blob_cube_64(0)).cuda()
    l0, h0 = svr.svr_minmax(c0)
    cam0 = synth.ortho_axis(64, 64, 64, 256, 256, "+z").as_f32()
    ramp = torch.from_numpy(synth.lut_ramp(256)).cuda()
    r0 = {}
    for st in ("f32", "f16", "bf16"):
        v = svr.svr_volume_create(c0, storage=st)
        for m in ("mip0", "avip0"):
            p0 = dict(mode=m, k=0.22, clim_lo=l0, clim_hi=h0)
            _, ns = svr.svr_render(v, cam0, ramp, p0, samples=True)
            n0 = int(ns.sum().item())
            ms = _time(torch, lambda: svr.svr_render(v, cam0, ramp, p0), 50)
            r0[f"{st}_{m}"] = dict(ms=ms, samples_per_s=n0 / (ms * 1e-3), fps=1e3 / ms)
        v.close()
    forms["blob64_256x256"] = r0
    # moment maps M0 / M1 / argmax over the whole spectral axis: one streaming read of the cube
    log("form: moment maps")
    mom = svr.svr_moments(cube)
    ms = _time(torch, lambda: svr.svr_moments(cube, out=mom), 10)
    nbytes = 4 * cube.numel() + 12 * cube.shape[1] * cube.shape[2]
    forms["moments"] = dict(ms=ms, hbm_bytes_algorithmic=nbytes,
                            gbps=nbytes / (ms * 1e-3) / 1e9,
                            hbm_frac=nbytes / (ms * 1e-3) / PEAK_HBM)
    # float16 / bfloat16 storage (FP32 arithmetic)
    for st in ("f16", "bf16"):
        log(f"form: {st} storage")
        v = svr.svr_volume_create(cube, storage=st)
        r = {}
        for m in ("mip0", "avip0"):
            i16, ns = svr.svr_render(v, cam, lut, params[m], samples=True)
            n = int(ns.sum().item())
            ms = _time(torch, lambda: svr.svr_render(v, cam, lut, params[m]), 5)
            # the image against the float32-storage image of the same view (the storage
            # rounding carried through the transfer function; the error against the FP64
            # oracle is measured in the tests)
            # (max over the image is set by samples within the storage rounding of the
            # clipping threshold, which flip between clipped and kept: the tests exclude
            # such pixels; the 99.99th percentile and the count above 2e-3 show the rest)
            i32 = svr.svr_render(vol32, cam, lut, params[m])
            d = (i16 - i32).abs().amax(dim=2).flatten()
            r[m] = dict(ms=ms, samples_per_s=n / (ms * 1e-3), fps=1e3 / ms,
                        speedup_vs_fp32=plain[m]["ms"] / ms,
                        max_abs_vs_fp32_storage=float(d.max()),
                        p9999_abs_vs_fp32_storage=float(torch.quantile(d[::4].float(), 0.9999)),
                        pixels_above_2e3=int((d > 2e-3).sum()),
                        mean_abs_vs_fp32_storage=float(d.mean()))
        forms[f"{st}_storage"] = r
        v.close()
    vol32.close()
    # differentiable forward + adjoint: 256^3 cube, 64-point transfer function
    log("form: forward + adjoint")
    c4 = torch.from_numpy(synth.disc_cube_256(0)).cuda()
    l4, h4 = svr.svr_minmax(c4)
    v4 = svr.svr_volume_create(c4)
    tf = torch.from_numpy(synth.tf_ramp(64)).cuda()
    p4 = dict(mode="avip0", opacity_from_lut=1, k=0.22, clim_lo=l4, clim_hi=h4)
    fb = {}
    for (w, h) in ((1024, 1024), (1920, 1080)):
        cam4 = synth.perspective_lookat(256, 256, 256, 30.0, 20.0, 256 * 3 ** 0.5, 40.0,
                                        w, h).as_f32()
        img, wsp = svr.svr_render_train(v4, cam4, tf, p4)
        _, ns = svr.svr_render(v4, cam4, tf, p4, samples=True)
        n = int(ns.sum().item())
        g = torch.randn(h, w, 4, device="cuda")
        gtf = torch.zeros_like(tf)
        gvox = torch.zeros_like(c4)
        ms_f = _time(torch, lambda: svr.svr_render(v4, cam4, tf, p4), 5)
        ms_t = _time(torch, lambda: svr.svr_render_train(v4, cam4, tf, p4, out=img,
                                                          workspace=wsp), 5)
        ms_b = _time(torch, lambda: svr.svr_render_backward(v4, cam4, tf, p4, wsp, g,
                                                             grad_tf=gtf, grad_vox=gvox), 3)
        fb[f"{w}x{h}"] = dict(samples=n, fwd_ms=ms_f, train_fwd_ms=ms_t, bwd_ms=ms_b,
                              fwd_fps=1e3 / ms_f, fwd_bwd_fps=1e3 / (ms_t + ms_b),
                              fwd_samples_per_s=n / (ms_f * 1e-3),
                              fwd_bwd_samples_per_s=n / ((ms_t + ms_b) * 1e-3),
                              fwd_bwd_vs_fwd=(ms_t + ms_b) / ms_f)
    forms["fwd_bwd"] = fb
    v4.close()
    # batched: 512 float16 sub-cubes, 512x512 each, one persistent graph launch
    log("form: batched sub-cubes")
    forms["batched"] = run_batched(torch, svr, synth, lut)
    return forms


def _vol32(svr, cube):
    return svr.svr_volume_create(cube, storage="f32")


def _make_sub(spec):
    import synth
    return synth.subcube(spec)


def _subcube_camera(synth, sp):
    """The sub-cube's own perspective camera: along its random view direction, at twice its
    bounding radius, 30 degree field of view, 512 x 512."""
    v = sp["view"] / np.linalg.norm(sp["view"])
    radius = 0.5 * math.sqrt(sp["nx"] ** 2 + sp["ny"] ** 2 + sp["nz"] ** 2)
    centre = ((sp["nx"] - 1) / 2, (sp["ny"] - 1) / 2, (sp["nz"] - 1) / 2)
    return synth.perspective_direction(centre, v, 2 * radius, 30.0, 512, 512).as_f32()


def run_batched(torch, svr, synth, lut):
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    specs = synth.subcube_batch_specs(512, 0)
    t = time.time()
    # fresh worker processes (numpy only): no fork of this GPU-initialised process
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(max_workers=min(16, os.cpu_count() or 4), mp_context=ctx) as ex:
        cubes = list(ex.map(_make_sub, specs, chunksize=8))
    log(f"  generated 512 sub-cubes in {time.time() - t:.1f}s")
    vols, cams = [], []
    for sp, c in zip(specs, cubes):
        tc = torch.from_numpy(c).cuda()
        vols.append(svr.svr_volume_create(tc, storage="f16"))
        cams.append(_subcube_camera(synth, sp))
    del cubes
    res = {}
    for m in ("mip0", "avip0"):
        p = dict(mode=m, k=0.22)
        # the autotuner's search (brick edge x tile x grid, median of three launches each)
        t = time.perf_counter()
        b = svr.svr_batch_create(vols, cams, lut, p, tune=2)
        tune_s = time.perf_counter() - t
        d = svr.svr_batch_create(vols, cams, lut, p, tune=0, outs=b.outs)
        n = 0
        for v, c in zip(vols, cams):
            _, ns = svr.svr_render(v, c, lut, p, samples=True)
            n += int(ns.sum().item())
        ms_b = _time(torch, lambda: b.launch(), 5)
        ms_d = _time(torch, lambda: d.launch(), 5)
        outs = b.outs

        def per_cube():
            for v, c, o in zip(vols, cams, outs):
                svr.svr_render(v, c, lut, p, out=o)
        ms_p = _time(torch, per_cube, 3)
        st = b.stats
        res[m] = dict(samples=n, batched_ms=ms_b, default_shape_ms=ms_d,
                      tuned_vs_default=ms_d / ms_b, per_cube_launches_ms=ms_p,
                      speedup=ms_p / ms_b, samples_per_s=n / (ms_b * 1e-3),
                      items=st["items"], grid=st["grid"], tile_waves_x=st["tile_waves_x"],
                      brick=st["brick"], search_default_ms=st["default_ms"],
                      search_tuned_ms=st["tuned_ms"], search_s=tune_s)
        b.close()
        d.close()
    for v in vols:
        v.close()
    return res


def _oracle_rate(oracle, cube64, cam, lut, p, budget, rng, threads, npx=256):
    """Oracle samples/s on random pixels of one frame, the pixel count grown until the
    render takes about `budget` seconds."""
    total = cam.width * cam.height
    while True:
        pix = rng.choice(total, min(npx, total), replace=False)
        t = time.perf_counter()
        _, _, ns = oracle.render(cube64, cam, lut, p, pixels=pix, nthreads=threads)
        dt = time.perf_counter() - t
        if dt > 0.5 * budget or npx >= total:
            return int(ns.sum()), dt, len(pix)
        npx = int(min(total, npx * max(2.0, 0.8 * budget / max(dt, 1e-3))))


def cpu_baseline(cube_np, cam, synth, lo, hi, args):
    """The FP64 oracle (test infrastructure, timed here as the CPU baseline) on bounded
    samples: random pixels of the benchmark frame (MIP0 and AVIP0) on all host cores and on
    one core, and short timings of the other workloads (64^3 frames, the differentiable
    256^3 form with its FP64 adjoint, sampled pixels of sub-cubes of the batched form)."""
    import oracle
    log("CPU baseline: oracle on sampled pixels")
    cube64 = cube_np.astype(np.float64)
    lut = synth.lut_heat(256)
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(0)
    budget = args.cpu_seconds
    total_s, total_n, total_px = 0.0, 0, 0
    one_s, one_n = 0.0, 0
    for m in ("mip0", "avip0"):
        p = dict(mode=m, k=0.22, filter="clip", min_t=3.0, lo=lo, hi=hi)
        n, dt, npx = _oracle_rate(oracle, cube64, cam, lut, p, 0.5 * budget, rng, threads)
        total_s, total_n, total_px = total_s + dt, total_n + n, total_px + npx
        n, dt, _ = _oracle_rate(oracle, cube64, cam, lut, p, 0.1 * budget, rng, 1, npx=16)
        one_s, one_n = one_s + dt, one_n + n
    del cube64
    out = {"value": total_n / total_s, "unit": "samples/s", "cores": threads, "kind": "oracle",
           "sample": f"{total_px} random pixels of the 1920x1080 frame (MIP0 and AVIP0, clip "
                     f"minT 3) on the 512x512x1024 cube, {total_n} samples in {total_s:.1f}s",
           "one_core": {"value": one_n / one_s, "unit": "samples/s", "cores": 1,
                        "sample": f"{one_n} samples of the same frame in {one_s:.1f}s"}}
    log("CPU baseline: other workloads")
    cfg = {}
    # 64^3 blob cube, full 256x256 frames
    c0 = synth.blob_cube_64(0).astype(np.float64)
    l0, h0 = float(c0.min()), float(c0.max())
    cam0 = synth.ortho_axis(64, 64, 64, 256, 256, "+z").as_f32()
    for m in ("mip0", "avip0"):
        t = time.perf_counter()
        _, _, ns = oracle.render(c0, cam0, synth.lut_ramp(256), dict(mode=m, k=0.22, lo=l0, hi=h0),
                                 nthreads=threads)
        dt = time.perf_counter() - t
        cfg[f"blob64_{m}_256x256"] = dict(s_per_frame=dt, samples_per_s=int(ns.sum()) / dt)
    # 256^3 differentiable form at 1024x1024: forward on all cores, FP64 adjoint on one core
    c4 = synth.disc_cube_256(0).astype(np.float64)
    l4, h4 = float(c4.min()), float(c4.max())
    cam4 = synth.perspective_lookat(256, 256, 256, 30.0, 20.0, 256 * 3 ** 0.5, 40.0,
                                    1024, 1024).as_f32()
    tf = synth.tf_ramp(64)
    p4 = dict(mode="avip0", opacity_from_lut=1, k=0.22, lo=l4, hi=h4)
    n, dt, npx = _oracle_rate(oracle, c4, cam4, tf, p4, 2.0, rng, threads)
    cfg["disc256_avip0_1024x1024_forward"] = dict(samples_per_s=n / dt, sample=f"{npx} pixels")
    pix = rng.choice(1024 * 1024, 400, replace=False)
    t = time.perf_counter()
    oracle.render_grad(c4, cam4, tf, p4, np.ones((400, 4)), pixels=pix)
    dt = time.perf_counter() - t
    _, _, ns = oracle.render(c4, cam4, tf, p4, pixels=pix, nthreads=threads)
    cfg["disc256_avip0_1024x1024_forward_adjoint_1core"] = dict(
        samples_per_s=int(ns.sum()) / dt, sample="400 pixels, forward + FP64 adjoint")
    del c4
    # sub-cubes of the batched form (float16 values), sampled pixels of 8 of them
    specs = synth.subcube_batch_specs(512, 0)[:8]
    n_all, s_all = 0, 0.0
    for sp in specs:
        c = synth.subcube(sp).astype(np.float64)
        camc = _subcube_camera(synth, sp)
        pix = rng.choice(512 * 512, 2000, replace=False)
        t = time.perf_counter()
        _, _, ns = oracle.render(c, camc, lut, dict(mode="mip0", lo=float(c.min()),
                                                    hi=float(c.max())),
                                 pixels=pix, nthreads=threads)
        s_all += time.perf_counter() - t
        n_all += int(ns.sum())
    cfg["subcubes_mip0_512x512"] = dict(samples_per_s=n_all / s_all,
                                        sample="2000 pixels of each of 8 sub-cubes")
    out["configs"] = cfg
    return out


if __name__ == "__main__":
    main()
