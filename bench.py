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


def bake_digest():
    h = hashlib.sha256(open(os.path.join(ROOT, "paper_2103_10380_amd", "csrc",
                                         "fastnerf_bake.hip"), "rb").read())
    return h.hexdigest()[:16]


def kernel_digest():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def storage_of(name):
    """Cache format and brick-sparsity of a storage name: "fp8" is a dense FP8
    cache, "fp8s" the brick-sparse one."""
    return (name[:-1], True) if name.endswith("s") else (name, False)


def build_caches(spec, storages, want_sparse, device, brick=8):
    """Generates the scene slab by slab on the GPU and uploads it to one cache
    per storage format; optionally keeps a brick-sparse host copy. `brick` is
    the occupancy brick edge of the dense caches (brick-sparse ones use 8)."""
    import paper_2103_10380_amd as fn
    import synth
    p = synth.draw(spec)
    beta = synth.beta_table(p)
    caches = {}
    for st in storages:
        base, is_sparse = storage_of(st)
        desc = fn.make_desc(spec.k, spec.D, spec.l, storage=base,
                            brick=8 if is_sparse else brick, sample_mode=fn.IN_BOX,
                            sparse=is_sparse)
        caches[st] = fn.Cache.create_empty(desc, beta)
    k, sb = spec.k, 8
    # FP8 scales and the stored bricks of sparse caches need the whole cache first
    scanned = [st for st in storages if storage_of(st)[0] == "fp8" or storage_of(st)[1]]
    if scanned:
        for z0 in range(0, k, sb):
            if z0 % (16 * sb) == 0:
                log(f"scan slab z0={z0}/{k}")
            sig = synth.density(p, z0, sb, device)
            u = synth.radiance(p, z0, sb, device)
            for st in scanned:
                caches[st].scan_slab(z0, sig, u)
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


def time_single(fn, cache, views, N, eps, steps, warmup):
    """Per-frame latency: every view in a launch of its own, HIP events around
    each launch on the launch stream."""
    import torch
    outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
    for _ in range(warmup):
        for v, o in zip(views, outs):
            fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, out=o)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps * len(views))]
    q = 0
    for _ in range(steps):
        for v, o in zip(views, outs):
            evs[q][0].record()
            fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, out=o)
            evs[q][1].record()
            q += 1
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


def time_batched(fn, cache, views, N, eps, steps, warmup):
    """Throughput: one step renders every view of the orbit in one persistent
    launch; the wall clock brackets exactly `steps` steps, with a device
    synchronisation on both sides, and HIP events time every launch."""
    import torch
    outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
    for _ in range(warmup):
        fn.render_batch(cache, views, N, eps, outs=outs)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn.render_batch(cache, views, N, eps, outs=outs)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([a.elapsed_time(b) for a, b in evs]), outs


def host_cpu():
    """CPU model name and logical CPU counts of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return dict(cpu_model=model, nproc=os.cpu_count(), usable_cpus=usable)


def oracle_threads():
    """Threads of the all-core oracle leg: the CPUs this process may use,
    capped by OMP_NUM_THREADS when it is set (the host's share of CPUs)."""
    n = host_cpu()["usable_cpus"] or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def oracle_sample(beta, sparse, spec, views, N, eps, pix_per_view, seconds, outs, seed=11,
                  threads=1, brick=8):
    """The FP64 oracle on random pixels of every view, single-threaded (stops
    at the time budget after completing a whole view) and, on the same pixels,
    split into row bands over `threads` threads (bitwise the same results,
    checked). Each view's oracle result is compared at once with the GPU
    renders in ``outs`` (storage -> list of [H,W,4] device tensors) and only
    the summary is kept."""
    import oracle
    import torch
    sb, slot, ss, su = sparse
    sc = oracle.Scene(beta, k=spec.k, sparse=(sb, slot, ss, su), in_box=True, occ_brick=brick)
    rng = np.random.default_rng(seed)
    rays, t_cpu, t_mt, nviews = 0, 0.0, 0.0, 0
    totals = dict(hit=0, occ_samples=0, rays=0, pixels=0)
    f32 = dict(worst=0.0, fails=0, checked=0, unchecked=0)
    other = {st: dict(worst=0.0, se=0.0, n=0) for st in outs if st != "f32"}
    for vi, v in enumerate(views):
        pix = np.sort(rng.choice(v.H * v.W, pix_per_view, replace=False))
        t0 = time.perf_counter()
        r = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, pix=pix,
                          tol=oracle.DEFAULT_TOL)
        t_cpu += time.perf_counter() - t0
        if threads > 1:
            t0 = time.perf_counter()
            rm = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, pix=pix,
                               tol=oracle.DEFAULT_TOL, threads=threads)
            t_mt += time.perf_counter() - t0
            if not (np.array_equal(rm["rgba"], r["rgba"]) and rm["counts"] == r["counts"]):
                raise RuntimeError("threaded oracle differs from the single-threaded one")
            del rm
        rays += len(pix)
        nviews += 1
        for key in ("hit", "occ_samples", "rays"):
            totals[key] += r["counts"][key]
        totals["pixels"] += v.H * v.W
        idx = torch.as_tensor(pix, device=outs["f32"][vi].device)
        g = outs["f32"][vi].reshape(-1, 4)[idx].cpu().numpy().astype(np.float64)
        # a pixel with too many ambiguous lookups to enumerate is checked
        # against the oracle's interval bounds of all its admissible results
        err, ok = oracle.matches(g, r, 1e-4)
        unchecked = (r["flags"] & oracle.UNCHECKED) != 0
        f32["fails"] += int((~ok).sum())
        f32["checked"] += int((~unchecked).sum())
        f32["unchecked"] += int(unchecked.sum())
        if (~unchecked).any():
            f32["worst"] = max(f32["worst"], float(err[~unchecked].max()))
        if unchecked.any():
            wdt = (r["env"][unchecked, 1] - r["env"][unchecked, 0]).max(axis=1)
            f32["bound_width_max"] = max(f32.get("bound_width_max", 0.0), float(wdt.max()))
        # the other formats over the same checked pixels (an unchecked pixel
        # has no admissible oracle result to compare with)
        chk = ~unchecked
        for st, acc in other.items():
            g = outs[st][vi].reshape(-1, 4)[idx].cpu().numpy().astype(np.float64)[chk]
            if not len(g):
                continue
            rc = {key: r[key][chk] for key in ("cand", "ncand")}
            err, _ = oracle.matches(g, rc, 1.0)
            acc["worst"] = max(acc["worst"], float(err.max()))
            acc["se"] += float(np.sum((g[:, :3] - oracle.matched(g, rc)[:, :3]) ** 2))
            acc["n"] += g.shape[0] * 3
        del r
        if t_cpu >= seconds:
            break
    return dict(rays=rays, t_cpu=t_cpu, t_mt=t_mt, threads=threads, nviews=nviews,
                totals=totals, f32=f32, other=other)


def launch_units(totals, views):
    """Per-launch counts behind the algorithmic bytes: the oracle's per-ray
    averages over its sampled pixels times the rays of the whole launch."""
    rays = float(sum(v.H * v.W for v in views))
    per_ray = rays / totals["rays"]
    return dict(rays=rays, occ_samples=totals["occ_samples"] * per_ray,
                hit_rays=totals["hit"] * per_ray)


def alg_bytes(units, payload, D):
    """Algorithmic bytes of a launch: the record payload of every sample in an
    occupied brick, the four direction cells (D floats each) per hit ray, the
    16-byte RGBA write per pixel."""
    rec = units["occ_samples"] * payload
    beta = units["hit_rays"] * 4 * D * 4
    wr = units["rays"] * 16
    return dict(records=rec, beta=beta, writes=wr, total=rec + beta + wr)


def time_launches(fn_launch, reps, warmup):
    """Mean and per-launch durations (ms) of fn_launch() with events on the
    current stream, after warmup launches."""
    import torch
    for _ in range(warmup):
        fn_launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn_launch()
        b.record()
    torch.cuda.synchronize()
    return np.array([a.elapsed_time(b) for a, b in evs])


def precision_sweep(fn, reps=20):
    """The plain scene (k=128, D=8, l=64, 6 ellipsoids, seed 0) on an 8-view
    orbit at r=3, el=0.4 (200x200, samples in [2, 4], N=128, eps=1e-4), with the
    position cache stored FP32 / FP16 / BF16 / FP8-E4M3, accumulation in FP32:
    error against the FP64 oracle on the FP32 inputs, Mrays/s and the
    algorithmic GB/s (this cache fits the last-level cache, so the rate is not
    an HBM rate)."""
    import oracle
    import synth
    sig, u, beta, _ = synth.scene_arrays(synth.plain_scene_spec())
    views = [synth.orbit_view(3.0, 2 * np.pi * v / 8 + 0.7, 0.4, 200, 200, 2.0, 4.0)
             for v in range(8)]
    N, eps = 128, 1e-4
    sc = oracle.Scene(beta, sig, u, occ_brick=8)
    ref, totals = [], dict(hit=0, occ_samples=0, rays=0)
    for v in views:
        r = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps,
                          tol=oracle.DEFAULT_TOL)
        ref.append(r)
        for key in totals:
            totals[key] += r["counts"][key]
    out = {}
    for st in ("f32", "f16", "bf16", "fp8"):
        cache = fn.Cache.create(fn.make_desc(128, 8, 64, storage=st, brick=8), sig, u, beta)
        stride, payload = cache.record_bytes
        import torch
        outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]

        def orbit():
            for v, o in zip(views, outs):
                fn.render(cache, v.K, v.c2w, v.H, v.W, v.near, v.far, N, eps, out=o)
        ms = time_launches(orbit, reps, 3)
        errs, se, n, se_hit, n_hit, se_p = [], 0.0, 0, 0.0, 0, 0.0
        for o, res in zip(outs, ref):
            g = o.reshape(-1, 4).cpu().numpy().astype(np.float64)
            # max-abs and PSNR against the nearest admissible oracle result
            # (voxel-face and stop-point ties); PSNR against the oracle's
            # primary result beside it
            err, _ = oracle.matches(g, res, 1.0)
            errs.append(float(err.max()))
            r = oracle.matched(g, res)
            d2 = (g[:, :3] - r[:, :3]) ** 2
            se += d2.sum()
            n += d2.size
            se_p += float(((g[:, :3] - res["rgba"][:, :3]) ** 2).sum())
            hit = r[:, 3] > 0.01
            se_hit += d2[hit].sum()
            n_hit += d2[hit].size
        rays = sum(v.H * v.W for v in views)
        alg = totals["occ_samples"] * payload + totals["hit"] * 4 * 8 * 4 + rays * 16
        psnr = lambda e, m: float("inf") if e == 0 else 10 * np.log10(m / e)
        out[st] = {"max_abs_err": float(max(errs)), "psnr_db": round(psnr(se, n), 3),
                   "psnr_hit_db": round(psnr(se_hit, n_hit), 3),
                   "psnr_vs_primary_db": round(psnr(se_p, n), 3),
                   "mrays_per_s": round(rays / (float(np.mean(ms)) / 1e3) / 1e6, 1),
                   "alg_gb_per_s": round(alg / (float(np.mean(ms)) / 1e3) / 1e9, 1)}
        cache.destroy()
    return out


def batched_uneven(fn, reps=10):
    """64 views of the plain scene in one launch: resolutions drawn from
    {256^2, 512^2, 800^2, 1024^2, 1280x720}, radii U[3,5], elevations U[-1,1]
    (seed 2); trilinear position lookup, FP16 cache, samples in the box,
    N=128, eps=1e-4."""
    import torch
    import synth
    sig, u, beta, _ = synth.scene_arrays(synth.plain_scene_spec())
    cache = fn.Cache.create(fn.make_desc(128, 8, 64, storage="f16", pos_interp=fn.LINEAR,
                                         brick=8, sample_mode=fn.IN_BOX), sig, u, beta)
    views = synth.random_views(64, 2, [(256, 256), (512, 512), (800, 800), (1024, 1024),
                                       (1280, 720)], (3.0, 5.0), (-1.0, 1.0), 0.0, 100.0)
    outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
    ms = time_launches(lambda: fn.render_batch(cache, views, 128, 1e-4, outs=outs), reps, 2)
    rays = sum(v.H * v.W for v in views)
    cache.destroy()
    return {"views": 64, "rays_per_launch": rays, "launch_ms_mean": round(float(np.mean(ms)), 4),
            "launch_ms_p50": round(float(np.percentile(ms, 50)), 4),
            "mrays_per_s": round(rays / (float(np.mean(ms)) / 1e3) / 1e6, 1)}


MFMA_F16_PEAK_TFLOPS = 2500.0  # MI355X dense binary16 matrix peak


def bake_measure(fn, k=768, l=384, slab=64, sample=3000, cpu_points=1 << 18, with_cpu=True):
    """Cache bake of the paper's networks (Sec. 4: 8 x 384 position MLP, skip
    input at layer 5, L = 10; 4 x 128 direction MLP, L = 4; D = 8; random
    binary16 weights, seed 7): the whole k^3 position grid in launches of
    `slab` layers and the l x l direction grid, HIP events per launch.
    Sampled parity against the oracle and the oracle's own rate on a bounded
    sample belong to the CPU leg."""
    import torch
    import synth
    spec = synth.MlpSpec()
    w = synth.mlp_weights(spec)
    net = fn.Mlp(spec, w)
    pos_shapes, dir_shapes = synth.mlp_shapes(spec)
    flop_pt = 2 * sum(a * b for a, b in pos_shapes)
    box = ((-1.0, -1.0, -1.0), (1.0, 1.0, 1.0))
    sig = torch.empty((slab, k, k), dtype=torch.float32, device="cuda")
    u = torch.empty((slab, k, k, spec.D, 3), dtype=torch.float32, device="cuda")
    net.bake_position(k, *box, 0, slab, sig, u)  # warm-up
    torch.cuda.synchronize()
    evs = []
    t0 = time.perf_counter()
    for z0 in range(0, k, slab):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        net.bake_position(k, *box, z0, min(slab, k - z0), sig, u)
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in evs])
    pts = k ** 3
    launch_pts = slab * k * k
    achieved = flop_pt * launch_pts / (ms.mean() / 1e3) / 1e12
    beta = net.bake_direction(l)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    net.bake_direction(l, beta)
    b.record()
    torch.cuda.synchronize()
    out = {
        "workload": (f"F_pos (8 x 384, skip at layer 5, L=10, D=8) at the {k}^3 voxel centres "
                     f"in {len(evs)} launches of {slab} layers; F_dir (4 x 128, L=4) on the "
                     f"{l}^2 direction grid; random binary16 weights (seed 7)"),
        "position_mpoints_per_s": round(pts / wall / 1e6, 1),
        "position_grid_s": round(wall, 3),
        "launch_ms_mean": round(float(ms.mean()), 3),
        "direction_grid_ms": round(a.elapsed_time(b), 4),
        "flop_per_point": flop_pt,
        "roofline": {"bound": "mfma", "achieved": round(achieved, 1),
                     "peak": MFMA_F16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / MFMA_F16_PEAK_TFLOPS, 4),
                     "kernel": "k_bake<position>, binary16 products, FP32 accumulation",
                     "algorithmic_flop_per_launch": flop_pt * launch_pts},
        "uncached_frame_ms_est": round(800 * 800 * 192 / (pts / wall) * 1e3, 1),
    }
    if with_cpu:
        from oracle import mlp as omlp
        rng = np.random.default_rng(5)
        z0 = k - slab  # the last launch's layers are still in sig / u
        idx = np.stack([rng.integers(0, k, sample), rng.integers(0, k, sample),
                        rng.integers(z0, k, sample)], axis=1)
        rows = (idx[:, 2] - z0) * k * k + idx[:, 1] * k + idx[:, 0]
        s_ref, u_ref = omlp.bake_position(w, spec, k, *box, idx)
        s_g = sig.reshape(-1)[torch.as_tensor(rows, device="cuda")].cpu().numpy()
        u_g = u.reshape(-1, spec.D, 3)[torch.as_tensor(rows, device="cuda")].cpu().numpy()
        cells = omlp.grid_indices(l)[rng.choice(l * l, sample, replace=False)]
        b_ref = omlp.bake_direction(w, spec, l, cells)
        b_g = beta.reshape(-1, spec.D).cpu().numpy()[cells[:, 0] * l + cells[:, 1]]
        out["parity"] = {"points": sample, "sigma_max_abs_err": float(np.abs(s_g - s_ref).max()),
                         "u_max_abs_err": float(np.abs(u_g - u_ref).max()),
                         "beta_max_abs_err": float(np.abs(b_g - b_ref).max()),
                         "reference": "FP64 oracle (oracle/mlp.py)"}
        t_cpu = 0.0
        for c0 in range(0, cpu_points, 16384):  # bounded memory per call
            cidx = np.stack([rng.integers(0, k, 16384) for _ in range(3)], axis=1)
            t1 = time.perf_counter()
            omlp.bake_position(w, spec, k, *box, cidx)
            t_cpu += time.perf_counter() - t1
        try:
            from threadpoolctl import threadpool_info
            cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
        except Exception:
            cores = None
        out["cpu_baseline"] = {"value": round(cpu_points / t_cpu / 1e6, 5), "unit": "Mpoints/s",
                               "cores": cores, "kind": "oracle",
                               "sample": f"{cpu_points} voxel centres, FP64 numpy, {t_cpu:.2f} s"}
    net.destroy()
    return out


def voxel_sweep(fn, main=None, ks=(256, 384, 512, 768, 1024), nviews=8, reps=3, pix=200,
                sparse_from=1024):
    """The per-voxel integration (N = 0: every voxel a ray crosses) against N=192
    samples in the box, on the paper-scale generator at several k (seed 1,
    FP32 caches; brick-sparse from k = sparse_from on, so that k = 1024 fits
    beside the caches already resident), the first nviews views of the
    800x800 orbit in one launch each; sampled pixels of one view against the
    oracle's traversal. main = (k, FP32 cache, brick-sparse copy or None, beta)
    of the scene already built, reused at its k."""
    import oracle
    import synth
    import torch
    out = {}
    views = synth.paper_orbit(40)[:nviews]
    rays = sum(v.H * v.W for v in views)
    for k in ks:
        spec = synth.paper_scene_spec(k=k)
        if main is not None and main[0] == k and main[1] is not None:
            _, cache, sparse, beta = main
            own = False
        else:
            st = "f32s" if k >= sparse_from else "f32"
            p_, beta, cs, sparse, _ = build_caches(spec, [st], True, "cuda")
            cache, own = cs[st], True
        row = {"cache": "brick-sparse FP32" if own and k >= sparse_from else "dense FP32"}
        for name, N in (("voxels", 0), ("n192", 192)):
            outs = [torch.empty((v.H, v.W, 4), dtype=torch.float32, device="cuda") for v in views]
            ms = time_launches(lambda: fn.render_batch(cache, views, N, 1e-4, outs=outs), reps, 1)
            row[name] = {"ms_per_view": round(float(np.mean(ms)) / nviews, 4),
                         "mrays_per_s": round(rays / (float(np.mean(ms)) / 1e3) / 1e6, 1)}
            if N == 0 and sparse is not None:
                v = views[1]
                rng = np.random.default_rng(k)
                px = np.sort(rng.choice(v.H * v.W, pix, replace=False))
                g = outs[1].reshape(-1, 4)[torch.as_tensor(px, device="cuda")].cpu().numpy()
                sc = oracle.Scene(beta, k=k, sparse=sparse, in_box=True, occ_brick=8)
                r = oracle.render(sc, v.K, v.c2w, v.H, v.W, v.near, v.far, 0, 1e-4, pix=px,
                                  tol=oracle.DEFAULT_TOL)
                err, ok = oracle.matches(g.astype(np.float64), r, 1e-4)
                row["voxels"]["parity_max_abs_err"] = float(err.max())
                row["voxels"]["parity_failing"] = int((~ok).sum())
                row["voxels"]["occupied_pieces_per_hit_ray"] = round(
                    r["counts"]["occ_samples"] / max(1, r["counts"]["hit"]), 2)
        out[str(k)] = row
        log(f"voxel traversal k={k}: {row}")
        if own:
            cache.destroy()
    return out


SERVE_RES = [(400, 400), (800, 800), (1280, 720), (1920, 1080)]


def serve_offline(fn, caches, n_req, n_warm, seed=3, N=192, eps=1e-4, chunk=32):
    """The measured requests of serve_poisson (the same draws) rendered without
    the server: per scene, in submission order, batched launches of up to
    `chunk` views (the server's max_inflight), back to back on one stream. The
    rate the server's steps are compared with."""
    import torch
    import synth
    rng = np.random.default_rng(seed)
    per_scene = [[] for _ in caches]
    for i in range(n_warm + n_req):
        rng.exponential(1.0)
        W, H = SERVE_RES[rng.integers(len(SERVE_RES))]
        v = synth.orbit_view(rng.uniform(3.0, 5.0), rng.uniform(0, 2 * np.pi),
                             rng.uniform(-1.0, 1.0), W, H, 0.0, 100.0)
        scene = int(rng.integers(len(caches)))
        if i >= n_warm:
            per_scene[scene].append(v)
    batches = [(c, vs[j:j + chunk]) for c, vs in zip(caches, per_scene)
               for j in range(0, len(vs), chunk)]
    flat = torch.empty(chunk * max(w * h for w, h in SERVE_RES) * 4, dtype=torch.float32,
                       device="cuda")

    def outs_for(vs):
        out, off = [], 0
        for v in vs:
            out.append(flat.narrow(0, off, v.H * v.W * 4).view(v.H, v.W, 4))
            off += v.H * v.W * 4
        return out
    outs = [outs_for(vs) for _, vs in batches]

    def run():
        for (c, vs), o in zip(batches, outs):
            fn.render_batch(c, vs, N, eps, outs=o)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rays = sum(v.H * v.W for _, vs in batches for v in vs)
    return {"requests": n_req, "launches": len(batches), "views_per_launch_max": chunk,
            "frames_per_s": round(n_req / el, 1), "mrays_per_s": round(rays / el / 1e6, 1)}


def serve_poisson(fn, caches, lam, n_req, n_warm, seed=3, N=192, eps=1e-4, arena_bytes=0):
    """Poisson arrivals at lam requests/s over the resident caches: each request
    draws a scene, a resolution from SERVE_RES and a pose (r U[3,5], az U[0,2pi),
    el U[-1,1]); a waiter thread collects results in submission order.
    Latency is the server's (submission to completion). arena_bytes = 0: the
    server admits requests against a quarter of the free device memory."""
    import threading
    import queue
    import synth
    rng = np.random.default_rng(seed)
    srv = fn.Server(caches, arena_bytes=arena_bytes, max_inflight=32)
    q = queue.Queue()
    lat, rays_done, done_t = [], [0], [0.0]

    def waiter():
        while True:
            item = q.get()
            if item is None:
                return
            tk, nr, measured = item
            _, ms = srv.wait(tk)
            srv.release(tk)
            if measured:
                lat.append(ms)
                rays_done[0] += nr
                done_t[0] = time.perf_counter()
    th = threading.Thread(target=waiter)
    th.start()
    rejected = 0
    t_next = time.perf_counter()
    t_first = None
    for i in range(n_warm + n_req):
        t_next += rng.exponential(1.0 / lam)
        W, H = SERVE_RES[rng.integers(len(SERVE_RES))]
        v = synth.orbit_view(rng.uniform(3.0, 5.0), rng.uniform(0, 2 * np.pi),
                             rng.uniform(-1.0, 1.0), W, H, 0.0, 100.0)
        scene = int(rng.integers(len(caches)))
        while time.perf_counter() < t_next:
            time.sleep(max(0.0, min(0.0005, t_next - time.perf_counter())))
        if i == n_warm:
            t_first = time.perf_counter()
        try:
            tk = srv.submit(scene, v.K, v.c2w, H, W, v.near, v.far, N, eps)
        except fn.FastNeRFError:
            rejected += 1
            continue
        q.put((tk, W * H, i >= n_warm))
    q.put(None)
    th.join()
    st = srv.stats()
    srv.destroy()
    el = done_t[0] - t_first
    lat = np.array(lat)
    return {"lambda_req_per_s": lam, "requests": int(len(lat)), "rejected": rejected,
            "latency_ms_p50": round(float(np.percentile(lat, 50)), 3),
            "latency_ms_p99": round(float(np.percentile(lat, 99)), 3),
            "frames_per_s": round(len(lat) / el, 1),
            "mrays_per_s": round(rays_done[0] / el / 1e6, 1),
            "server_steps": st["steps"], "max_requests_per_step": st["max_batch"]}


def serving_scenes(fn):
    """The four resident serving scenes: k=512 FP16 (seed 10), k=512 FP8 (11),
    k=768 FP16 (12), k=768 FP8 (13); paper-scale generator, D=8, l=384."""
    import synth
    caches = []
    for k, st, seed in ((512, "f16", 10), (512, "fp8", 11), (768, "f16", 12), (768, "fp8", 13)):
        spec = synth.paper_scene_spec(k=k, seed=seed)
        _, _, cs, _, occ = build_caches(spec, [st], False, "cuda")
        log(f"serving scene k={k} {st} seed {seed}: occupancy {occ:.4f}")
        caches.append(cs[st])
    return caches


def step_gaps(path, match="k_render_step", skip=0.2):
    """Busy fraction and gaps of the serving step kernels in a rocprofv3 kernel
    trace (CSV): the first `skip` of the launches (warm-up, ramp) is left out;
    a gap is the idle time before a launch after every earlier one ended."""
    import csv
    import glob
    f = sorted(glob.glob(os.path.join(path, "**", "*kernel_trace.csv"), recursive=True))[0]
    rows = [r for r in csv.DictReader(open(f)) if match in r["Kernel_Name"]]
    st = np.array([int(r["Start_Timestamp"]) for r in rows], np.int64)
    en = np.array([int(r["End_Timestamp"]) for r in rows], np.int64)
    o = np.argsort(st)
    st, en = st[o], en[o]
    a = int(len(st) * skip)
    st, en = st[a:], en[a:]
    dur = (en - st) / 1e3
    span = (en.max() - st[0]) / 1e3
    ends = np.maximum.accumulate(en)
    gaps = np.maximum(st[1:] - ends[:-1], 0) / 1e3
    lines = [f"# {match}: {len(rows)} launches, the last {len(st)} analysed",
             f"window {span / 1e3:.1f} ms, busy {1 - gaps.sum() / span:.3f} of it"]
    for q in (10, 50, 90, 99):
        lines.append(f"duration p{q}: {np.percentile(dur, q):.1f} us; "
                     f"gap p{q}: {np.percentile(gaps, q):.1f} us")
    lines.append(f"mean duration {dur.mean():.1f} us, mean gap {gaps.mean():.1f} us, "
                 f"total gap {gaps.sum() / 1e3:.1f} ms")
    return "\n".join(lines)


def summarize_profile(paths, match=("k_render", "k_bake", "neg_kernel", "k_line_gather")):
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


def line_ceiling(gib=32, regions_kib=(64, 2048, 65536), blocks=16384, iters=32, modes=(0, 1, 2)):
    """Sustained rate of random 128-byte line reads on this GPU (liblinebench.so):
    each wave reads random lines inside a random region per round, lanes reading
    whole lines, 32-byte pieces, or one line per 8 lanes. The render's record
    gathers reach HBM as such lines, so this is the achievable rate they are
    measured against (the HBM peak assumes streaming). A buffer of a few MiB
    stays in the L2 and one of some hundred MiB in the memory-side cache, so
    small sizes give the rates of those levels; regions larger than the buffer
    are skipped."""
    import ctypes
    import torch
    lb = ctypes.CDLL(os.path.join(ROOT, "paper_2103_10380_amd", "liblinebench.so"))
    fnl = lb.fnr_line_gather
    fnl.restype = ctypes.c_int
    fnl.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                    ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p]
    nbytes = int(gib * (1 << 30)) // 128 * 128
    if nbytes < 128:
        raise ValueError("line buffer below one line")
    buf = torch.zeros(nbytes // 4, dtype=torch.float32, device="cuda")
    sink = torch.zeros(4, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    lines = blocks * 256 * iters
    rates = {}
    for mode, name in ((0, "line_per_lane"), (1, "32B_per_lane"), (2, "line_per_8_lanes")):
        if mode not in modes:
            continue
        for rk in regions_kib:
            if (rk << 10) > nbytes:
                continue

            def go(seed):
                rc = fnl(buf.data_ptr(), nbytes, rk << 10, mode, blocks, iters, seed,
                         sink.data_ptr(), st.cuda_stream)
                if rc != 0:
                    raise RuntimeError(f"fnr_line_gather failed ({rc})")
            go(1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for r in range(3):
                go(2 + r)
            e1.record(st)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / 3
            rates[f"{name}_region_{rk}KiB"] = round(lines / ms / 1e6, 2)
    del buf
    torch.cuda.empty_cache()
    best = max(rates.values())
    return {"unit": "G lines/s", "buffer_gib": gib, "lines_per_launch": lines, "rates": rates,
            "max_glines_per_s": best, "max_tb_per_s_of_lines": round(best * 128 / 1e3, 3)}


def pmc_traffic(fetch_dir, write_dir, tcc_dir=None, kernel="k_render_locc<0, 8, false>",
                calib="neg_kernel"):
    """HBM bytes per launch of the render kernel from FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by what the same counter reads for the
    calibration kernel (torch.neg over 2^28 floats: 1 GiB read, 1 GiB written);
    with a TCC_HIT_sum / TCC_MISS_sum run, also the kernel's L2 hit rate."""
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
    res = {"kernel": kernel, "kernel_digest": kernel_digest(),
           "hbm_bytes_per_launch": round(out["fetch"]["bytes"] + out["write"]["bytes"]),
           "fetch": out["fetch"], "write": out["write"]}
    if tcc_dir:
        hit = [v for n, v in counter_means(tcc_dir, "TCC_HIT_sum").items() if kernel in n]
        miss = [v for n, v in counter_means(tcc_dir, "TCC_MISS_sum").items() if kernel in n]
        if len(hit) == 1 and len(miss) == 1:
            res["tcc_hit"], res["tcc_miss"] = hit[0], miss[0]
            res["l2_hit_rate"] = round(hit[0] / (hit[0] + miss[0]), 4)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--views", type=int, default=40)
    ap.add_argument("--k", type=int, default=768)
    ap.add_argument("--no-variants", action="store_true", help="FP32 cache only")
    ap.add_argument("--storages", default="f32,f16,fp8,f32s,fp8s",
                    help="comma-separated cache formats to time (f32 is always included; "
                         "a trailing s selects the brick-sparse cache of that format)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-pixels", type=int, default=65536, help="oracle pixels per view")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for profiler byte counters)")
    ap.add_argument("--summarize-profile", nargs="+", metavar="DIR",
                    help="print a summary of rocprofv3 CSV output directories and exit")
    ap.add_argument("--serving", action="store_true",
                    help="only the serving workload: four resident scenes, Poisson arrivals "
                         "at 50/100/200/400/1600/6400/12800 requests/s (one JSON line)")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-rates", default="50,100,200,400,1600,6400,12800",
                    help="Poisson arrival rates (requests/s) of --serving")
    ap.add_argument("--bake", action="store_true",
                    help="only the cache bake of the paper's networks (one JSON line)")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-view latency launches (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision sweep, the batched launch and the serving sample")
    ap.add_argument("--step-gaps", metavar="DIR",
                    help="busy fraction and gaps of the serving step kernels in a kernel trace")
    ap.add_argument("--pmc-traffic", nargs="+", metavar="DIR",
                    help="print the render kernel's calibrated HBM bytes per launch (JSON) "
                         "from FETCH_SIZE and WRITE_SIZE runs made with --calibrate-copy "
                         "(FETCH_DIR WRITE_DIR [TCC_DIR]; the third adds the L2 hit rate)")
    ap.add_argument("--brick", type=int, default=8,
                    help="occupancy brick edge of the dense caches (the workload's 8: a 96^3 "
                         "bitgrid at k=768)")
    ap.add_argument("--schedule", default="auto",
                    choices=["auto", "tiles", "refill", "wide", "split"],
                    help="schedule of the render launches (fastnerf_set_schedule)")
    ap.add_argument("--line-ceiling", action="store_true",
                    help="only measure the random 128-byte line read rate (liblinebench.so)")
    ap.add_argument("--line-regions", default="64,2048,65536",
                    help="--line-ceiling: region sizes in KiB, comma-separated")
    ap.add_argument("--line-modes", default="0,1,2",
                    help="--line-ceiling: 0 line per lane, 1 32 B per lane, 2 line per 8 lanes")
    ap.add_argument("--line-gib", type=float, default=32,
                    help="--line-ceiling: buffer size in GiB (fractions allowed, e.g. 0.002 for 2 MiB)")
    ap.add_argument("--pmc-kernel", default="k_render_locc<0, 8, false>",
                    help="kernel name (substring) that --pmc-traffic reports")
    args = ap.parse_args()
    if args.summarize_profile:
        print(summarize_profile(args.summarize_profile))
        return
    if args.line_ceiling:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(line_ceiling(
            gib=args.line_gib, regions_kib=tuple(int(x) for x in args.line_regions.split(",")),
            modes=tuple(int(x) for x in args.line_modes.split(",")))), flush=True)
        return
    if args.step_gaps:
        print(step_gaps(args.step_gaps))
        return
    if args.pmc_traffic:
        if len(args.pmc_traffic) not in (2, 3):
            raise SystemExit("--pmc-traffic takes FETCH_DIR WRITE_DIR [TCC_DIR]")
        print(json.dumps(pmc_traffic(*args.pmc_traffic, kernel=args.pmc_kernel), indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the renderer "
              "runs on a single MI355X; sharding across GPUs is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2103_10380_amd as fn
    import synth
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fn.lib()
    fn.set_schedule(args.schedule)

    if args.serving:
        t0 = time.perf_counter()
        caches = serving_scenes(fn)
        log(f"serving scenes built in {time.perf_counter() - t0:.1f}s")
        rows = []
        for lam in [int(x) for x in args.serve_rates.split(",")]:
            r = serve_poisson(fn, caches, lam, args.serve_requests, 100)
            log(f"lambda {lam}: p50 {r['latency_ms_p50']} ms p99 {r['latency_ms_p99']} ms, "
                f"{r['frames_per_s']} frames/s")
            rows.append(r)
        off = serve_offline(fn, caches, args.serve_requests, 100)
        log(f"same requests without the server: {off['frames_per_s']} frames/s, "
            f"{off['mrays_per_s']} Mrays/s")
        print(json.dumps({
            "metric": "serving latency (p50/p99) under Poisson arrivals", "unit": "ms",
            "n_gpus": 1, "data": "synthetic",
            "config": {"workload": "4 resident scenes (k=512 FP16 seed 10, k=512 FP8 seed 11, "
                                   "k=768 FP16 seed 12, k=768 FP8 seed 13; D=8, l=384), "
                                   "requests of 400^2/800^2/1280x720/1920x1080 at random "
                                   "poses, N=192 in the box, eps=1e-4, seed 3",
                       "warmup_requests": 100, "requests_per_rate": args.serve_requests},
            "rates": rows, "offline_same_mix": off, "kernel_digest": kernel_digest()}),
              flush=True)
        return

    if args.bake:
        r = bake_measure(fn, with_cpu=not args.no_cpu)
        print(json.dumps({"metric": "cache bake throughput (position network)",
                          "value": r["position_mpoints_per_s"], "unit": "Mpoints/s",
                          "n_gpus": 1, "dtype": "f16", "data": "synthetic", **r,
                          "bake_digest": bake_digest()}), flush=True)
        return

    N, eps = 192, 1e-4
    spec = synth.paper_scene_spec(k=args.k)
    views = synth.paper_orbit(args.views)
    storages = ["f32"] + [st for st in args.storages.split(",") if st and st != "f32"]
    if args.no_variants:
        storages = ["f32"]
    t0 = time.perf_counter()
    p, beta, caches, sparse, occ = build_caches(spec, storages, not args.no_cpu, "cuda",
                                                brick=args.brick)
    torch.cuda.synchronize()
    log(f"scene k={spec.k} occupancy {occ:.4f}, caches {storages} built in "
        f"{time.perf_counter() - t0:.1f}s; resident "
        f"{sum(c.resident_bytes for c in caches.values()) / 2**30:.1f} GiB")

    results = {}
    outs_f32 = None
    for st in storages:
        wall, step_ms, outs = time_batched(fn, caches[st], views, N, eps, args.steps,
                                           args.warmup)
        frame_ms = (np.array([0.0]) if args.no_single else
                    time_single(fn, caches[st], views, N, eps, args.steps, args.warmup))
        rays = args.steps * sum(v.H * v.W for v in views)
        results[st] = dict(wall=wall, step_ms=step_ms, frame_ms=frame_ms,
                           mrays=rays / wall / 1e6, resident=caches[st].resident_bytes)
        if st == "f32":
            outs_f32 = outs
        else:
            results[st]["outs"] = outs
        log(f"{st}: {results[st]['mrays']:.1f} Mrays/s ({len(views)} views per launch, "
            f"{np.mean(step_ms):.3f} ms per launch); single-view frame p50 "
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
    nv = len(views)
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
                         f"{args.brick}^3 occupancy bricks, FP32 cache; one step = the whole orbit in one "
                         "persistent launch"),
            "views_per_step": args.views, "width": 800, "height": 800, "N": N,
        },
        "fps": round(nv * args.steps / r32["wall"], 1),
        "launch_ms_mean": round(float(np.mean(r32["step_ms"])), 4),
        "single_view": None if args.no_single else {
            "fps": round(1e3 / float(np.mean(frame_ms)), 1),
            "frame_ms_p50": round(float(np.percentile(frame_ms, 50)), 4),
            "frame_ms_p99": round(float(np.percentile(frame_ms, 99)), 4),
            "note": "each view in a launch of its own; HIP events per launch"},
    }

    # ---------------------------------------------------------------- oracle leg
    units = None
    psnr_in = {}
    if not args.no_cpu:
        outs_all = {"f32": outs_f32}
        outs_all.update({st: results[st]["outs"] for st in storages if st != "f32"})
        threads = oracle_threads()
        o = oracle_sample(beta, sparse, spec, views, N, eps, args.cpu_pixels, args.cpu_seconds,
                          outs_all, threads=threads, brick=args.brick)
        host = host_cpu()
        sample = (f"{o['rays']} random pixels ({args.cpu_pixels} per view over the first "
                  f"{o['nviews']} of the {nv} views) of the same workload, FP64")
        one = dict(value=round(o["rays"] / o["t_cpu"] / 1e6, 5), unit="Mrays/s", cores=1,
                   seconds=round(o["t_cpu"], 2))
        if threads > 1:
            line["cpu_baseline"] = {
                "value": round(o["rays"] / o["t_mt"] / 1e6, 5), "unit": "Mrays/s",
                "cores": threads, "kind": "oracle",
                "sample": sample + f", split into row bands over {threads} threads "
                                   f"({o['t_mt']:.1f} s; bitwise equal to the 1-thread run)",
                "single_core": one, **host}
        else:
            line["cpu_baseline"] = {**one, "kind": "oracle", "sample": sample + ", 1 thread",
                                    **host}
        units = launch_units(o["totals"], views)
        f32 = o["f32"]
        line["parity"] = {"pixels": f32["checked"], "max_abs_err": f32["worst"],
                          "failing": f32["fails"], "bounded": f32["unchecked"],
                          "bounded_width_max": f32.get("bound_width_max"), "tol": 1e-4,
                          "reference": "FP64 oracle, FP32 cache; pixels with more than 3 "
                                       "ambiguous lookups checked against interval bounds of "
                                       "all their admissible results"}
        for st, acc in o["other"].items():
            m = acc["se"] / max(1, acc["n"])
            psnr_in[st] = dict(max_abs_err=acc["worst"],
                               psnr_db=(float("inf") if m == 0 else 10 * np.log10(1 / m)))
    # ---------------------------------------------------------------- roofline
    if units is not None:
        stride, payload = caches["f32"].record_bytes
        ab = alg_bytes(units, payload, spec.D)
        avg_s = float(np.mean(r32["step_ms"])) / 1e3
        achieved = ab["total"] / avg_s / 1e9
        pmc = None
        if os.path.exists(PMC_SUMMARY):
            pmc = json.load(open(PMC_SUMMARY))
            if pmc.get("kernel_digest") != kernel_digest():
                pmc = None
        traffic = pmc.get("hbm_bytes_per_launch") if pmc else None
        line["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": (f"k_render_locc<FP32, D<=8, nearest> (tile kernel, bitgrid in LDS), "
                       f"{nv} views per launch"),
            "algorithmic_bytes_per_launch": round(ab["total"]),
            "bytes_per_launch": {key: round(ab[key]) for key in ("records", "beta", "writes")},
            "frac_records_and_writes": round((ab["records"] + ab["writes"]) / avg_s / 1e9 /
                                             HBM_PEAK_GBS, 4),
            "occupied_samples_per_launch": round(units["occ_samples"]),
            "hit_rays_per_launch": round(units["hit_rays"]),
            "rays_per_launch": round(units["rays"]),
            "record_payload_bytes": payload, "record_stride_bytes": stride,
            "launch_ms_mean": round(avg_s * 1e3, 4),
            "l2_hit_rate": pmc.get("l2_hit_rate") if pmc else None,
            "useful_bytes_fraction": (round(ab["total"] / traffic, 4) if traffic else None),
            "note": ("achieved = algorithmic bytes per launch / mean launch time (HIP events on "
                     "the launch stream); traffic, L2 hit rate from rocprofv3 counters of the "
                     "same kernel source (null when the source changed since)")}
    variants = {}
    for st in storages:
        r = results[st]
        variants[st] = {"mrays_per_s": round(r["mrays"], 2),
                        "fps": round(nv * args.steps / r["wall"], 1),
                        "launch_ms_mean": round(float(np.mean(r["step_ms"])), 4),
                        "single_view_frame_ms_p50": None if args.no_single else
                        round(float(np.percentile(r["frame_ms"], 50)), 4),
                        "single_view_frame_ms_p99": None if args.no_single else
                        round(float(np.percentile(r["frame_ms"], 99)), 4),
                        "speedup_vs_f32": round(r["mrays"] / r32["mrays"], 3),
                        "resident_gib": round(r["resident"] / 2**30, 3),
                        "brick_sparse": storage_of(st)[1]}
        if not args.no_cpu and st != "f32":
            variants[st].update({k2: round(v2, 6) for k2, v2 in psnr_in[st].items()})
        if units is not None and st in caches:
            # the FP32 cache's sample counts with this format's record payload
            # over this format's launch time
            _, pl = caches[st].record_bytes
            vb = alg_bytes(units, pl, spec.D)
            sec = float(np.mean(r["step_ms"])) / 1e3
            gbs = vb["total"] / sec / 1e9
            variants[st].update({"record_payload_bytes": pl, "alg_gb_per_s": round(gbs, 1),
                                 "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                                 "hbm_frac_records_and_writes": round(
                                     (vb["records"] + vb["writes"]) / sec / 1e9 /
                                     HBM_PEAK_GBS, 4)})
    line["variants"] = variants
    if not args.no_extras and not args.no_single:
        # the a9 schedules: the same FP32 launches (the 40-view batch, and the
        # views one launch each) under each schedule
        per = {}
        for sch in ("tiles", "wide", "split", "refill"):
            fn.set_schedule(sch)
            wall_t, step_t, _ = time_batched(fn, caches["f32"], views, N, eps, args.steps,
                                             args.warmup)
            frame_t = time_single(fn, caches["f32"], views, N, eps, 2, 1)
            per[sch] = {"launch_ms_mean": round(float(np.mean(step_t)), 4),
                        "single_view_frame_ms_p50": round(float(np.percentile(frame_t, 50)), 4),
                        "single_view_frame_ms_p99": round(float(np.percentile(frame_t, 99)), 4)}
        fn.set_schedule(args.schedule)
        line["schedule_compare"] = {
            "note": ("FP32 cache. tiles = one 8x8 tile per wave until its slowest ray stops "
                     "(bitgrid in LDS); wide = tiles with more records in flight per lane; "
                     "split = 4x4 tiles, four lanes per ray (single views; batches run wide); "
                     "refill = wave-level ray queue (ballot, LDS pool, refill). auto = split "
                     "(or wide) up to 20,000 8x8 tiles, tiles above"),
            "schedule": args.schedule,
            "default": {
                "launch_ms_mean": round(float(np.mean(r32["step_ms"])), 4),
                "single_view_frame_ms_p50": round(float(np.percentile(frame_ms, 50)), 4),
                "single_view_frame_ms_p99": round(float(np.percentile(frame_ms, 99)), 4)},
            **per}
        log(f"schedules: {line['schedule_compare']}")
    if not args.no_extras:
        # the served path per storage format on one resident copy of the same
        # scene: latency at 200 requests/s and throughput when saturated
        by_fmt = {}
        for st in ("f32", "f16", "fp8"):
            if st not in caches:
                continue
            lo = serve_poisson(fn, [caches[st]], 200, 300, 30)
            hi = serve_poisson(fn, [caches[st]], 12800, 800, 80)
            by_fmt[st] = {"p50_ms_at_200": lo["latency_ms_p50"],
                          "p99_ms_at_200": lo["latency_ms_p99"],
                          "saturated_frames_per_s": hi["frames_per_s"],
                          "saturated_mrays_per_s": hi["mrays_per_s"],
                          "psnr_db_vs_fp64_oracle": (None if st == "f32" or st not in psnr_in
                                                     else round(psnr_in[st]["psnr_db"], 2))}
        if "f32" in by_fmt:
            for st, r in by_fmt.items():
                r["saturated_speedup_vs_f32"] = round(
                    r["saturated_frames_per_s"] / by_fmt["f32"]["saturated_frames_per_s"], 3)
        line["serving_by_format"] = by_fmt
        log(f"serving by format: {by_fmt}")
        if "f16" in caches and "fp8" in caches:
            # continuous batching over the two reduced-precision caches already resident
            r = serve_poisson(fn, [caches["f16"], caches["fp8"]], 200, 300, 30)
            r["scenes"] = "paper-scale k=768 FP16 and FP8 caches of this run"
            line["serving_sample"] = r
            log(f"serving sample: p50 {r['latency_ms_p50']} ms p99 {r['latency_ms_p99']} ms")
            # the same scenes with arrivals faster than the GPU can serve them,
            # beside the same requests rendered without the server
            pair = [caches["f16"], caches["fp8"]]
            r = serve_poisson(fn, pair, 12800, 1000, 100)
            r["scenes"] = "paper-scale k=768 FP16 and FP8 caches of this run"
            r["offline_same_mix"] = serve_offline(fn, pair, 1000, 100)
            line["serving_saturated"] = r
            log(f"serving at 12800 req/s: {r['frames_per_s']} frames/s, offline "
                f"{r['offline_same_mix']['frames_per_s']} frames/s")
        line["voxel_traversal"] = voxel_sweep(fn, (spec.k, caches.get("f32"), sparse, beta))
        # level of detail: the level the library picks for the orbit's camera
        # among the swept resolutions, and its cost from the sweep
        ks = sorted(int(k) for k in line["voxel_traversal"])
        pick = ks[fn.lod_select(ks, (-1.0,) * 3, (1.0,) * 3, views[0].K, views[0].c2w, 1.0)]
        line["lod"] = {"levels": ks, "ratio": 1.0, "picked_k": pick,
                       "n192_ms_per_view": line["voxel_traversal"][str(pick)]["n192"]["ms_per_view"],
                       "rule": "coarsest k whose voxel edge <= ratio x pixel footprint at the "
                               "box centre"}
        for c in caches.values():
            c.destroy()
        caches = {}
        line["batched_uneven"] = batched_uneven(fn)
        log(f"batched uneven: {line['batched_uneven']}")
        line["precision_sweep"] = precision_sweep(fn)
        log(f"precision sweep: {line['precision_sweep']}")
        line["bake"] = bake_measure(fn, with_cpu=not args.no_cpu)
        log(f"bake: {line['bake']}")
        lc = line_ceiling()
        line["line_ceiling"] = lc
        log(f"line ceiling: {lc}")
        rl = line.get("roofline")
        if rl is not None:
            # lines the FP32 launch fetched (L2 misses, from the counters of this
            # kernel source) per second, against the ceiling just measured
            miss = None
            if os.path.exists(PMC_SUMMARY):
                pmc = json.load(open(PMC_SUMMARY))
                if pmc.get("kernel_digest") == kernel_digest():
                    miss = pmc.get("tcc_miss")
            if miss:
                rate = miss / (rl["launch_ms_mean"] / 1e3) / 1e9
                rl["line_rate_glines_per_s"] = round(rate, 2)
                rl["frac_of_line_ceiling"] = round(rate / lc["max_glines_per_s"], 4)
    line["kernel_digest"] = kernel_digest()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
