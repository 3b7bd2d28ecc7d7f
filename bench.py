#!/usr/bin/env python3
"""Throughput of the cached FastNeRF render on one MI355X.

Workload (the paper-scale configuration): a k=768 position cache (D=8 radiance
components, about 8% of voxels occupied by 28 ellipsoids and 12 thin shells),
an l=384 direction cache, a 40-view orbit at radius 4 rendered at 800x800 with
N=192 samples inside the box, eps=1e-4, nearest position lookup, bilinear
direction lookup, 8^3 occupancy bricks, FP32 cache. One step renders the whole
orbit, one persistent launch per view. Inputs are synthetic (seeded) and
resident in HBM before timing starts.

The JSON line also carries: per-frame p50/p99 latency, the same orbit with FP16
and FP8 caches, the roofline of the render kernel (algorithmic bytes per launch
over its measured duration) and the FP64 CPU oracle timed on a bounded sample
of the same workload (which also gives the algorithmic byte count and a sampled
parity check).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "k_render_f32_paper_scale_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2103_10380_amd", "csrc", f)
                  for f in ("fastnerf_kernels.hip", "fastnerf_device.h")]


def kernel_digest():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_caches(spec, storages, want_sparse, device):
    """Generates the scene slab by slab on the GPU and uploads it to one cache
    per storage format; optionally keeps a brick-sparse host copy."""
    import paper_2103_10380_amd as fn
    import synth
    p = synth.draw(spec)
    beta = synth.beta_table(p)
    caches = {}
    for st in storages:
        desc = fn.make_desc(spec.k, spec.D, spec.l, storage=st, brick=8,
                            sample_mode=fn.IN_BOX)
        caches[st] = fn.Cache.create_empty(desc, beta)
    k, sb = spec.k, 8
    if "fp8" in caches:  # per-channel scales need the whole cache first
        for z0 in range(0, k, sb):
            if z0 % (16 * sb) == 0:
                log(f"scan slab z0={z0}/{k}")
            sig = synth.density(p, z0, sb, device)
            u = synth.radiance(p, z0, sb, device)
            caches["fp8"].scan_slab(z0, sig, u)
    nb = k // sb
    slot = np.full(nb ** 3, -1, np.int32) if want_sparse else None
    ss, su, n, occ_vox = [], [], 0, 0
    for z0 in range(0, k, sb):
        if z0 % (16 * sb) == 0:
            log(f"upload slab z0={z0}/{k}")
        sig = synth.density(p, z0, sb, device)
        u = synth.radiance(p, z0, sb, device)
        occ_vox += int((sig > 0).sum())
        for c in caches.values():
            c.upload_slab(z0, sig, u)
        if want_sparse:
            idx, s1, u1 = synth.brick_sparse_slab(sig, u, sb)
            slot[(z0 // sb) * nb * nb + idx] = np.arange(n, n + len(idx), dtype=np.int32)
            n += len(idx)
            ss.append(s1)
            su.append(u1)
    for c in caches.values():
        c.finalize()
    sparse = None
    if want_sparse:
        sparse = (sb, slot, np.concatenate(ss), np.concatenate(su))
    return p, beta, caches, sparse, occ_vox / k ** 3


def time_orbit(fn, cache, views, N, eps, steps, warmup):
    import torch
    outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
    for _ in range(warmup):
        for v, o in zip(views, outs):
            fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, out=o)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps * len(views))]
    t0 = time.perf_counter()
    q = 0
    for _ in range(steps):
        for v, o in zip(views, outs):
            evs[q][0].record()
            fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, out=o)
            evs[q][1].record()
            q += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    frame_ms = np.array([a.elapsed_time(b) for a, b in evs])
    return wall, frame_ms, outs


def oracle_sample(beta, sparse, spec, views, N, eps, pix_per_view, seconds, outs, seed=11):
    """The FP64 oracle, single-threaded, on random pixels of every view (stops
    at the time budget after completing a whole view). Each view's oracle
    result is compared at once with the GPU renders in ``outs`` (storage ->
    list of [H,W,4] device tensors) and only the summary is kept."""
    import oracle
    import torch
    sb, slot, ss, su = sparse
    sc = oracle.Scene(beta, k=spec.k, sparse=(sb, slot, ss, su), in_box=True, occ_brick=8)
    rng = np.random.default_rng(seed)
    rays, t_cpu, nviews = 0, 0.0, 0
    totals = dict(hit=0, occ_samples=0, rays=0, pixels=0)
    f32 = dict(worst=0.0, fails=0, checked=0)
    other = {st: dict(worst=0.0, se=0.0, n=0) for st in outs if st != "f32"}
    for vi, v in enumerate(views):
        pix = np.sort(rng.choice(v.H * v.W, pix_per_view, replace=False))
        t0 = time.perf_counter()
        r = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, pix=pix,
                          tol=oracle.DEFAULT_TOL)
        t_cpu += time.perf_counter() - t0
        rays += len(pix)
        nviews += 1
        for key in ("hit", "occ_samples", "rays"):
            totals[key] += r["counts"][key]
        totals["pixels"] += v.H * v.W
        idx = torch.as_tensor(pix, device=outs["f32"][vi].device)
        g = outs["f32"][vi].reshape(-1, 4)[idx].cpu().numpy().astype(np.float64)
        err, ok = oracle.matches(g, r, 1e-4)
        unchecked = (r["flags"] & oracle.UNCHECKED) != 0
        f32["fails"] += int((~ok & ~unchecked).sum())
        f32["checked"] += int((~unchecked).sum())
        if (~unchecked).any():
            f32["worst"] = max(f32["worst"], float(err[~unchecked].max()))
        for st, acc in other.items():
            g = outs[st][vi].reshape(-1, 4)[idx].cpu().numpy().astype(np.float64)
            err, _ = oracle.matches(g, r, 1.0)
            acc["worst"] = max(acc["worst"], float(err.max()))
            acc["se"] += float(np.sum((g[:, :3] - r["rgba"][:, :3]) ** 2))
            acc["n"] += g.shape[0] * 3
        del r
        if t_cpu >= seconds:
            break
    return rays, t_cpu, nviews, totals, f32, other


def summarize_profile(paths, match=("k_render", "neg_kernel")):
    """Compact text summary of rocprofv3 CSV output (kernel stats and counter
    collections): per-kernel calls and durations, per-dispatch counter means."""
    import csv
    import glob
    lines = []
    for root in paths:
        for f in sorted(glob.glob(os.path.join(root, "**", "*kernel_stats.csv"), recursive=True)):
            lines.append(f"# kernel stats ({os.path.basename(root)})")
            lines.append("name | calls | avg_us | min_us | max_us | total_%")
            for r in csv.DictReader(open(f)):
                if any(m in r["Name"] for m in match):
                    lines.append(f"{r['Name'][:90]} | {r['Calls']} | "
                                 f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                                 f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}")
        for f in sorted(glob.glob(os.path.join(root, "**", "*counter_collection.csv"),
                               recursive=True)):
            acc = {}
            for r in csv.DictReader(open(f)):
                name = r.get("Kernel_Name", "")
                if not any(m in name for m in match):
                    continue
                key = (name[:90], r["Counter_Name"])
                a = acc.setdefault(key, [0.0, set()])
                a[0] += float(r["Counter_Value"])
                a[1].add(r.get("Dispatch_Id", r.get("Correlation_Id")))
            lines.append(f"# counters ({os.path.basename(root)}): mean per dispatch")
            lines.append("kernel | counter | dispatches | mean")
            for (name, cn), (tot, ids) in sorted(acc.items()):
                lines.append(f"{name} | {cn} | {len(ids)} | {tot / max(1, len(ids)):.6g}")
    return "\n".join(lines)


def counter_means(root, counter):
    """Mean per dispatch of one rocprofv3 counter, per kernel name."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(root, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            a = acc.setdefault(r.get("Kernel_Name", ""), [0.0, set()])
            a[0] += float(r["Counter_Value"])
            a[1].add(r.get("Dispatch_Id", r.get("Correlation_Id")))
    return {name: tot / max(1, len(ids)) for name, (tot, ids) in acc.items()}


def pmc_traffic(fetch_dir, write_dir, kernel="k_render<0, 8, false>", calib="neg_kernel"):
    """HBM bytes per launch of the render kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    calibration kernel (torch.neg over 2^28 floats: 1 GiB read, 1 GiB written)."""
    out = {}
    for key, root, cn in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        m = counter_means(root, cn)
        kr = [v for n, v in m.items() if kernel in n]
        kc = [v for n, v in m.items() if calib in n]
        if len(kr) != 1 or len(kc) != 1:
            raise SystemExit(f"{cn}: expected one render and one calibration kernel, got "
                             f"{len(kr)} and {len(kc)}")
        factor = (1 << 30) / (kc[0] * 1024.0)
        out[key] = dict(kib_per_dispatch=kr[0], calib_kib_per_dispatch=kc[0],
                        calib_factor=factor, bytes=kr[0] * 1024.0 * factor)
    return {"kernel": kernel, "kernel_digest": kernel_digest(),
            "hbm_bytes_per_launch": round(out["fetch"]["bytes"] + out["write"]["bytes"]),
            "fetch": out["fetch"], "write": out["write"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--views", type=int, default=40)
    ap.add_argument("--k", type=int, default=768)
    ap.add_argument("--no-variants", action="store_true", help="FP32 cache only")
    ap.add_argument("--storages", default="f32,f16,fp8",
                    help="comma-separated cache formats to time (f32 is always included)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-pixels", type=int, default=65536, help="oracle pixels per view")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for profiler byte counters)")
    ap.add_argument("--summarize-profile", nargs="+", metavar="DIR",
                    help="print a summary of rocprofv3 CSV output directories and exit")
    ap.add_argument("--pmc-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the render kernel's calibrated HBM bytes per launch (JSON) "
                         "from FETCH_SIZE and WRITE_SIZE runs made with --calibrate-copy")
    args = ap.parse_args()
    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile))
        return
    if args.pmc_traffic:
        print(json.dumps(pmc_traffic(*args.pmc_traffic), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (this build "
              "renders on a single MI355X; multi-GPU sharding is a design note only)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2103_10380_amd as fn
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fn.lib()

    N, eps = 192, 1e-4
    spec = synth.paper_scene_spec(k=args.k)
    views = synth.paper_orbit(args.views)
    storages = ["f32"] + [st for st in args.storages.split(",") if st and st != "f32"]
    if args.no_variants:
        storages = ["f32"]
    t0 = time.perf_counter()
    p, beta, caches, sparse, occ = build_caches(spec, storages, not args.no_cpu, "cuda")
    torch.cuda.synchronize()
    log(f"scene k={spec.k} occupancy {occ:.4f}, caches {storages} built in "
        f"{time.perf_counter() - t0:.1f}s; resident "
        f"{sum(c.resident_bytes for c in caches.values()) / 2**30:.1f} GiB")

    results = {}
    outs_f32 = None
    for st in storages:
        wall, frame_ms, outs = time_orbit(fn, caches[st], views, N, eps, args.steps,
                                          args.warmup)
        rays = args.steps * sum(v.H * v.W for v in views)
        results[st] = dict(wall=wall, frame_ms=frame_ms, mrays=rays / wall / 1e6)
        if st == "f32":
            outs_f32 = outs
        else:
            results[st]["outs"] = outs
        log(f"{st}: {results[st]['mrays']:.1f} Mrays/s, frame p50 "
            f"{np.percentile(frame_ms, 50):.3f} ms p99 {np.percentile(frame_ms, 99):.3f} ms")

    if args.calibrate_copy:
        # a plain streaming kernel of known size: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        log("calibration: 3 x neg over 1 GiB (1 GiB read + 1 GiB written each)")

    r32 = results["f32"]
    frame_ms = r32["frame_ms"]
    line = {
        "metric": "Mrays/s at 800x800, cached render (paper-scale cache, FP32)",
        "value": round(r32["mrays"], 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["wall"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"paper-scale cached render: k={spec.k}^3 position cache, D=8, "
                         f"l=384 direction cache, {occ * 100:.1f}% voxels occupied "
                         "(28 ellipsoids + 12 shells, seed 1), "
                         f"{args.views}-view orbit r=4 el=0.5 at 800x800, N=192 samples in "
                         "the box, eps=1e-4, nearest position / bilinear direction lookup, "
                         "8^3 occupancy bricks, FP32 cache"),
            "views_per_step": args.views, "width": 800, "height": 800, "N": N,
        },
        "fps": round(1e3 / float(np.mean(frame_ms)), 1),
        "frame_ms_p50": round(float(np.percentile(frame_ms, 50)), 4),
        "frame_ms_p99": round(float(np.percentile(frame_ms, 99)), 4),
    }

    # ---------------------------------------------------------------- oracle leg
    units = None
    psnr_in = {}
    if not args.no_cpu:
        outs_all = {"f32": outs_f32}
        outs_all.update({st: results[st]["outs"] for st in storages if st != "f32"})
        rays, t_cpu, nv, totals, f32, other = oracle_sample(
            beta, sparse, spec, views, N, eps, args.cpu_pixels, args.cpu_seconds, outs_all)
        line["cpu_baseline"] = {
            "value": round(rays / t_cpu / 1e6, 5), "unit": "Mrays/s", "cores": 1,
            "kind": "oracle",
            "sample": (f"{rays} random pixels ({args.cpu_pixels} per view over the first "
                       f"{nv} views) of the same workload, FP64 single-threaded, "
                       f"{t_cpu:.1f} s"),
        }
        # algorithmic bytes per launch: records of samples in occupied bricks,
        # the four direction cells per hit ray, the RGBA write (sampled counts
        # scaled to whole views)
        scale = totals["pixels"] / totals["rays"] / nv
        units = dict(occ_samples=totals["occ_samples"] * scale, hit_rays=totals["hit"] * scale,
                     rays=totals["pixels"] / nv)
        line["parity"] = {"pixels": f32["checked"], "max_abs_err": f32["worst"],
                          "failing": f32["fails"], "tol": 1e-4,
                          "reference": "FP64 oracle, FP32 cache"}
        for st, acc in other.items():
            m = acc["se"] / max(1, acc["n"])
            psnr_in[st] = dict(max_abs_err=acc["worst"],
                               psnr_db=(float("inf") if m == 0 else 10 * np.log10(1 / m)))
    # ---------------------------------------------------------------- roofline
    if units is not None:
        stride, payload = caches["f32"].record_bytes
        D = spec.D
        alg_bytes = units["occ_samples"] * payload + units["hit_rays"] * 4 * D * 4 + \
            units["rays"] * 16
        avg_s = float(np.mean(frame_ms)) / 1e3
        achieved = alg_bytes / avg_s / 1e9
        traffic = None
        if os.path.exists(PMC_SUMMARY):
            pmc = json.load(open(PMC_SUMMARY))
            if pmc.get("kernel_digest") == kernel_digest():
                traffic = pmc.get("hbm_bytes_per_launch")
        line["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1),
                            "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                            "kernel": "k_render<FP32, D<=8, nearest>",
                            "algorithmic_bytes_per_launch": round(alg_bytes),
                            "occupied_samples_per_launch": round(units["occ_samples"]),
                            "record_payload_bytes": payload, "record_stride_bytes": stride}
    variants = {}
    for st in storages:
        r = results[st]
        variants[st] = {"mrays_per_s": round(r["mrays"], 2),
                        "fps": round(1e3 / float(np.mean(r["frame_ms"])), 1),
                        "frame_ms_p50": round(float(np.percentile(r["frame_ms"], 50)), 4),
                        "frame_ms_p99": round(float(np.percentile(r["frame_ms"], 99)), 4),
                        "speedup_vs_f32": round(r["mrays"] / r32["mrays"], 3)}
        if not args.no_cpu and st != "f32":
            variants[st].update({k2: round(v2, 6) for k2, v2 in psnr_in[st].items()})
    line["variants"] = variants
    line["kernel_digest"] = kernel_digest()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
