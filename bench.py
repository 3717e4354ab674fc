#!/usr/bin/env python3
"""Throughput of the fused CT augmentation path on one MI355X.

Headline workload (one step = one training batch through the whole forward
path): 16 int16 CT-like phantoms with per-axis sizes U{96..256}, each with
its own random affine (rotation, scale, centre displacement, crop shift) and
photometrics (gain, offset, Gaussian noise sigma = 10 HU, window, gamma),
warped to a common 120x120x160 float32 crop plus nearest-neighbour int8
labels.  A step uploads the batch's 16 job descriptors and runs one
persistent launch, both replayed from a HIP graph.  Three input batches
(about 1.3 GB in total, over 5x the 256 MB Infinity Cache) rotate so that no
step finds its inputs cache-resident, and each batch cycles through four
parameter draws.

Also reported in the same JSON line: the kernel-only roofline of the fused
batched kernel (timed over the same input sets and parameter draws as the
steps): algorithmic bytes per launch over its duration against the 8 TB/s
HBM peak, with the rocprofv3-measured traffic and the VALU issue fraction
beside it; the CPU oracle timed on this host; and secondary workloads
(full-resolution 512x512x320 volume; forward and forward+backward of the
differentiable warp on 8 x 128^3; the nonrigid B-spline warp on 4 x 256^3;
the warp alone; the host-to-device FIFO).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-secondary]
       [--no-cpu] [--profile]
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published
C3_OUT = (120, 120, 160)
# The batch plans take their launch shape (tile, workgroups per CU, LDS cells,
# LDS cell format) from the library's autotune cache, loaded from this file;
# `--autotune` re-runs the sweep on this workload and rewrites the file.
TUNING_CACHE = os.path.join(ROOT, "paper_1811_11226_amd", "autotune_cache.txt")
C3_CANDIDATES = [(tile, 0, lds, fmt) for tile in [(8, 16, 16), (16, 16, 16), (16, 16, 32)]
                 for lds in (0, 8176, 10208, 12272) for fmt in (0, 1)]

# VALU roofline.  Peak: 256 CUs x 64 lanes x 2.4 GHz non-packed lane-ops
# (one FP32/INT32 op per lane per cycle; transcendentals and 32x32->64-bit
# multiplies issue at quarter rate and are counted as 4).
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# Lane-ops the method's arithmetic needs (not the kernel's instruction count):
#  sampled voxel: coordinate 3 FMA; trilinear 3 floor + 3 fraction + 7 lerps x 2;
#    base-cell index 3 conversions + 2 multiply-adds + 1 add; label 3 add + 3
#    floor + 3 conversions + 3 index; one int16 conversion            = 42
#  every voxel, photometrics: gain/offset FMA, noise FMA, window 4
#    (sub, mul, max, min), gamma log2 + mul + exp2 (4 + 1 + 4)         = 15
#  every voxel, noise: Philox4x32-10 per 4 voxels, 10 rounds of 2 64-bit
#    products (4 each) + 2 three-input XOR = 100 / 4 = 25; Box-Muller per
#    pair 2 x (shift, convert, fma) + log2 4 + mul + sqrt 4 + sin 4 + cos 4
#    + 2 mul = 25 / 2 = 12.5                                            = 37.5
OPS_SAMPLED = 42.0
OPS_PHOTO = 15.0
OPS_NOISE = 37.5


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash():
    """Hash of the sources the batched forward kernel is compiled from."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1811_11226_amd", "csrc")
    for name in ("device_common.h", "bspline_eval.h", "tile_geom.h", "warp_fwd.hip"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()


def stored_traffic(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters for the current
    kernel sources, or None if absent or taken on different sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# ---------------------------------------------------------------------------
# Algorithmic bytes: every output written once, every distinct input voxel
# the method needs read once (corners with nonzero trilinear weight, nearest
# label voxels), nothing else.
# ---------------------------------------------------------------------------

def touched_counts(in_dim, out_dim, M, dev):
    import torch
    A = torch.tensor(M, dtype=torch.float64, device=dev).reshape(3, 4)
    n = torch.tensor(in_dim, dtype=torch.float64, device=dev)
    img_mark = torch.zeros(int(in_dim[0] * in_dim[1] * in_dim[2]), dtype=torch.bool, device=dev)
    lbl_mark = torch.zeros_like(img_mark)
    sampled = 0
    X, Y, Z = out_dim
    ys, zs = torch.meshgrid(torch.arange(Y, device=dev, dtype=torch.float64),
                            torch.arange(Z, device=dev, dtype=torch.float64), indexing="ij")
    ys, zs = ys.reshape(-1), zs.reshape(-1)
    strides = torch.tensor([in_dim[1] * in_dim[2], in_dim[2], 1], dtype=torch.int64, device=dev)
    for x0 in range(0, X, 16):
        xs = torch.arange(x0, min(X, x0 + 16), device=dev, dtype=torch.float64)
        P = torch.stack([xs[:, None].expand(-1, ys.numel()).reshape(-1),
                         ys.repeat(xs.numel()), zs.repeat(xs.numel())])
        q = A[:, :3] @ P + A[:, 3:4]
        guard = ((q > -1) & (q < n[:, None])).all(0)
        sampled += int(guard.sum().item())
        q = q[:, guard]
        f = torch.floor(q)
        t = q - f
        fi = f.to(torch.int64)
        for corner in range(8):
            off = ((corner >> 2) & 1, (corner >> 1) & 1, corner & 1)
            c = fi + torch.tensor(off, device=dev)[:, None]
            w_nz = torch.ones(c.shape[1], dtype=torch.bool, device=dev)
            for i in range(3):
                # the weight of the upper corner is t, of the lower corner 1 - t
                w_nz &= (t[i] != 0) if off[i] else (t[i] != 1)
            ok = w_nz & ((c >= 0) & (c < n.to(torch.int64)[:, None])).all(0)
            img_mark[(c[:, ok] * strides[:, None]).sum(0)] = True
        j = torch.floor(q + 0.5).to(torch.int64)
        ok = ((j >= 0) & (j < n.to(torch.int64)[:, None])).all(0)
        lbl_mark[(j[:, ok] * strides[:, None]).sum(0)] = True
    return int(img_mark.sum().item()), int(lbl_mark.sum().item()), sampled


# ---------------------------------------------------------------------------
# Headline: batched fused forward (c3)
# ---------------------------------------------------------------------------

class C3Set:
    """One 16-volume input batch resident in HBM with its outputs, a batch
    plan, and a pool of parameter draws."""

    def __init__(self, batch, n_pool, dev):
        import numpy as np
        import torch

        import paper_1811_11226_amd as ctaug
        from synth import AugmentRanges, configs, draw_affine_params, draw_photo
        self.jobs = configs.c3(batch=batch)
        self.imgs = [torch.from_numpy(j.img).to(dev) for j in self.jobs]
        self.lbls = [torch.from_numpy(j.lbl).to(dev) for j in self.jobs]
        self.outs = [torch.empty(C3_OUT, dtype=torch.float32, device=dev) for _ in self.jobs]
        self.louts = [torch.empty(C3_OUT, dtype=torch.int8, device=dev) for _ in self.jobs]
        self.pool = []          # list of (list of (M, photo))
        for p in range(n_pool):
            entry = []
            for k, j in enumerate(self.jobs):
                if p == 0:
                    prm, ph = j.prm, j.photo
                else:
                    rng = np.random.Generator(np.random.PCG64(
                        configs.seeds(3, j.volume_id)[1] + 1000 * p))
                    prm = draw_affine_params(rng, AugmentRanges(), j.in_dim, C3_OUT)
                    ph = draw_photo(rng, AugmentRanges(), seed=configs.seeds(3, j.volume_id)[2] + p,
                                    volume_id=j.volume_id)
                _, M = ctaug.affine_matrix(prm, j.in_dim, C3_OUT)
                entry.append((M, ph))
            self.pool.append(entry)
        self.job_arrays = []
        for entry in self.pool:
            cj = [ctaug.make_job(self.imgs[k], M, self.outs[k], self.lbls[k], self.louts[k],
                                 fill=j.fill, label_fill=j.label_fill, photo=ph)
                  for k, (j, (M, ph)) in enumerate(zip(self.jobs, entry))]
            self.job_arrays.append(cj)
        self.plan = ctaug.BatchPlan(self.job_arrays[0])      # launch shape from the cache

    def voxels(self):
        return len(self.jobs) * C3_OUT[0] * C3_OUT[1] * C3_OUT[2]


def run_c3(args, dev):
    import numpy as np
    import torch

    import paper_1811_11226_amd as ctaug
    n_sets, n_pool = 3, 4
    if os.path.exists(TUNING_CACHE) and not args.autotune:
        n = ctaug.autotune_cache_load(TUNING_CACHE)
        log(f"c3: autotune cache {os.path.relpath(TUNING_CACHE, ROOT)} ({n} entries)")
    log("c3: generating 3 x 16 phantoms")
    t0 = time.time()
    sets = [C3Set(b, n_pool, dev) for b in range(n_sets)]
    log(f"c3: inputs resident ({time.time() - t0:.1f} s)")
    stream = torch.cuda.Stream()

    times = None
    cached = ctaug.autotune_cache_lookup(sets[0].job_arrays[0]) is not None
    if args.autotune:
        # sweep launch shapes on batch 0 (the winner enters the library's
        # cache), save the cache, and rebuild every plan from it
        with torch.cuda.stream(stream):
            best, times = sets[0].plan.autotune(C3_CANDIDATES, reps=3)
        order = sorted(range(len(C3_CANDIDATES)), key=lambda i: times[i])
        log(f"c3: autotune best {best} ({min(times):.3f} ms); top 5 "
            f"{[(C3_CANDIDATES[i], round(times[i], 3)) for i in order[:5]]}")
        ctaug.autotune_cache_save(TUNING_CACHE)
        cached = True
        for s in sets:
            s.plan.close()
            s.plan = ctaug.BatchPlan(s.job_arrays[0])
    best = sets[0].plan.tuning()
    log(f"c3: launch shape {best} ({'autotune cache' if cached else 'library default'})")
    with torch.cuda.stream(stream):
        for s in sets:
            s.plan.launch()
            s.plan.capture()
    torch.cuda.synchronize()

    # descriptors validated and built once per (input set, parameter draw);
    # a step installs one prepared set (one copy into pinned staging) and
    # replays the graph (descriptor upload + launch)
    prepared = [[s.plan.prepare(cj) for cj in s.job_arrays] for s in sets]

    def step(i):
        s = sets[i % n_sets]
        s.plan.update_prepared(prepared[i % n_sets][(i // n_sets) % n_pool])
        s.plan.replay()

    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            step(i)
    torch.cuda.synchronize()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        start.record(stream)
        h0 = time.perf_counter()
        for i in range(args.steps):
            step(args.warmup + i)
        host_ms = (time.perf_counter() - h0) * 1e3 / args.steps
        end.record(stream)
    torch.cuda.synchronize()
    step_ms = start.elapsed_time(end) / args.steps
    # host cost of a step without the wait for the plan's previous replay: the
    # same calls with the GPU idle before each
    nowait = []
    with torch.cuda.stream(stream):
        for i in range(min(args.steps, 30)):
            torch.cuda.synchronize()
            h0 = time.perf_counter()
            step(i)
            nowait.append((time.perf_counter() - h0) * 1e3)
    torch.cuda.synchronize()
    host_nowait_ms = float(np.median(nowait))
    log(f"c3: {step_ms:.4f} ms per step (graph replay incl. descriptor upload); host enqueue "
        f"{host_ms:.4f} ms per step in the timed loop, {host_nowait_ms:.4f} ms with nothing "
        f"to wait for")

    # kernel-only duration of the fused batched kernel, per launch, same stream,
    # over the same (input set, parameter draw) sequence as the steps: one plan
    # per pair, its table uploaded beforehand, so that only kernels are timed
    pairs = [(i % n_sets, (i // n_sets) % n_pool) for i in range(args.steps)]
    kplans = {}
    with torch.cuda.stream(stream):
        for (si, d) in sorted(set(pairs)):
            kplans[(si, d)] = ctaug.BatchPlan(sets[si].job_arrays[d])
            assert kplans[(si, d)].tuning() == best
            kplans[(si, d)].launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    with torch.cuda.stream(stream):
        for pair, (a, b) in zip(pairs, evs):
            a.record(stream)
            kplans[pair].run()
            b.record(stream)
    torch.cuda.synchronize()
    kts = np.array([a.elapsed_time(b) for a, b in evs])
    kern_ms = float(np.mean(kts))
    kern_pct = [float(np.percentile(kts, q)) for q in (10, 50, 90)]
    log(f"c3: fused batched kernel {kern_ms:.4f} ms per launch (p10/p50/p90 "
        f"{kern_pct[0]:.4f}/{kern_pct[1]:.4f}/{kern_pct[2]:.4f})")

    # correctness spot check of the last kernel-only launch against single calls
    si, d = pairs[-1]
    s = sets[si]
    for k in (0, 7, 15):
        j = s.jobs[k]
        M, ph = s.pool[d][k]
        o, lo = ctaug.warp_affine(s.imgs[k], M, lbl=s.lbls[k], fill=j.fill, photo=ph,
                                  out_dim=C3_OUT)
        torch.cuda.synchronize()
        if not (torch.equal(o, s.outs[k]) and torch.equal(lo, s.louts[k])):
            raise SystemExit("bench: batched output differs from the single-volume call")
    for kp in kplans.values():
        kp.close()
    for row in prepared:
        for pj in row:
            pj.close()

    # algorithmic bytes and lane-ops of the timed kernel-only launches, averaged
    # over the same sequence of (set, draw) pairs
    t0 = time.time()
    per_pair = {}
    touched = []
    nv = C3_OUT[0] * C3_OUT[1] * C3_OUT[2]
    for (si, d) in sorted(set(pairs)):
        s = sets[si]
        b = ops = 0
        for k, j in enumerate(s.jobs):
            ti, tl, ns = touched_counts(j.in_dim, C3_OUT, s.pool[d][k][0], dev)
            touched.append(ti / nv)
            b += nv * (4 + 1) + ti * 2 + tl * 1
            ops += ns * OPS_SAMPLED + nv * (OPS_PHOTO + OPS_NOISE)
        per_pair[(si, d)] = (b, ops)
    alg_bytes = float(np.mean([per_pair[p][0] for p in pairs]))
    alg_ops = float(np.mean([per_pair[p][1] for p in pairs]))
    log(f"c3: algorithmic bytes per launch {alg_bytes / 1e6:.1f} MB "
        f"(mean touched fraction f = {np.mean(touched):.3f}; {time.time() - t0:.1f} s)")
    log(f"c3: algorithmic lane-ops per launch {alg_ops / 1e9:.3f} G")
    return dict(sets=sets, step_ms=step_ms, kern_ms=kern_ms, kern_pct=kern_pct,
                alg_bytes=alg_bytes, alg_ops=alg_ops, host_ms=host_ms,
                host_nowait_ms=host_nowait_ms, cached=cached,
                tuning=best, tune_ms=times, voxels=sets[0].voxels(), stream=stream)


# ---------------------------------------------------------------------------
# Secondary workloads
# ---------------------------------------------------------------------------

def time_loop(fn, reps, stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        fn()
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def time_split(fns, reps, stream):
    """Mean ms of each of fns run in sequence, reps times, with events between
    them on the stream: every part timed in the cache state the sequence
    leaves for it (a part repeated alone can find its working set in the
    Infinity Cache)."""
    import torch
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(fns) + 1)]
          for _ in range(reps)]
    with torch.cuda.stream(stream):
        for fn in fns:
            fn()
        torch.cuda.synchronize()
        for r in range(reps):
            ev[r][0].record(stream)
            for i, fn in enumerate(fns):
                fn()
                ev[r][i + 1].record(stream)
    torch.cuda.synchronize()
    return [sum(ev[r][i].elapsed_time(ev[r][i + 1]) for r in range(reps)) / reps
            for i in range(len(fns))]


class SideStreams:
    """Independent per-volume calls spread over side streams (default
    priority) that fork from the current stream and join back into it, so
    that one call's ramp and tail overlap another's work; each side stream
    needs its own workspace."""

    def __init__(self, n):
        import torch
        self.streams = [torch.cuda.Stream() for _ in range(n)]

    def __len__(self):
        return len(self.streams)

    def fork(self):
        import torch
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        for s in self.streams:
            s.wait_event(ev)

    def handle(self, i):
        return ctypes.c_void_p(self.streams[i].cuda_stream)

    def join(self):
        import torch
        cur = torch.cuda.current_stream()
        for s in self.streams:
            ev = torch.cuda.Event()
            ev.record(s)
            cur.wait_event(ev)


def run_c2(dev, stream, reps):
    import torch

    import paper_1811_11226_amd as ctaug
    from synth import configs
    j = configs.c2()[0]
    img, lbl = torch.from_numpy(j.img).to(dev), torch.from_numpy(j.lbl).to(dev)
    _, M = ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)
    out = torch.empty(j.out_dim, dtype=torch.float32, device=dev)
    lout = torch.empty(j.out_dim, dtype=torch.int8, device=dev)
    ms = time_loop(lambda: ctaug.warp_affine(img, M, lbl=lbl, fill=j.fill, photo=j.photo, out=out,
                                             lbl_out=lout), reps, stream)
    ti, tl, _ = touched_counts(j.in_dim, j.out_dim, M, dev)
    nv = out.numel()
    alg = nv * 5 + ti * 2 + tl
    return {"workload": "512x512x320 int16 + int8 labels -> f32 + int8, full photometrics",
            "ms": round(ms, 4), "gvoxel_s": round(nv / ms / 1e6, 2),
            "alg_GBs": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}


def run_labels_back(dev, stream, reps):
    """Nearest-neighbour resampling of a predicted label map back to the
    original grid (labels only, no image): 160x160x100 int8 -> 512x512x320."""
    import numpy as np
    import torch

    import paper_1811_11226_amd as ctaug
    from synth import phantom_pair
    pred_dim, orig_dim = (160, 160, 100), (512, 512, 320)
    _, lbl = phantom_pair(pred_dim, seed=20181129)
    lin = torch.from_numpy(lbl).to(dev)
    M = np.zeros(12, np.float32)
    for i in range(3):                  # voxel p of the original grid reads (p + 1/2) r - 1/2
        r = pred_dim[i] / orig_dim[i]
        M[4 * i + i] = r
        M[4 * i + 3] = 0.5 * r - 0.5
    lout = torch.empty(orig_dim, dtype=torch.int8, device=dev)
    ms = time_loop(lambda: ctaug.warp_labels(lin, M, label_fill=0, lbl_out=lout), reps, stream)
    nv = lout.numel()
    alg = nv + lin.numel()              # every output byte written, every input byte read
    return {"workload": "labels only: 160x160x100 int8 prediction resampled back to "
                        "512x512x320 by nearest neighbour",
            "ms": round(ms, 4), "gvoxel_s": round(nv / ms / 1e6, 2),
            "alg_GBs": round(alg / ms / 1e6, 1), "hbm_frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)}


def run_c4(dev, stream, reps):
    import torch

    import paper_1811_11226_amd as ctaug
    from synth import configs
    jobs, grads = configs.c4()
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    gs = [torch.from_numpy(g).to(dev) for g in grads]
    Ms = [ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)[1] for j in jobs]
    outs = [torch.empty(j.out_dim, dtype=torch.float32, device=dev) for j in jobs]
    plan = ctaug.BatchPlan([ctaug.make_job(imgs[k], Ms[k], outs[k], fill=jobs[k].fill)
                            for k in range(len(jobs))])
    # the image gradients of the batch live in one buffer, cleared by one fill
    g_all = torch.empty((len(jobs),) + tuple(imgs[0].shape), dtype=torch.float32, device=dev)
    g_imgs = [g_all[k] for k in range(len(jobs))]
    g_M = torch.empty((len(jobs), 12), dtype=torch.float64, device=dev)
    side = SideStreams(2)
    ws_bytes = ctaug.ops.warp_backward_workspace(jobs[0].out_dim)
    ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=dev) for _ in range(len(side))]
    L = ctaug._lib.load()
    Mc = [ctaug.ops._M32(M) for M in Ms]
    vi = [ctaug.ops.vol(i) for i in imgs]
    vg = [ctaug.ops.vol(g) for g in gs]
    vgi = [ctaug.ops.vol(g) for g in g_imgs]

    def fwd():
        plan.launch()

    def bwd():
        g_all.zero_()
        side.fork()
        for k in range(len(jobs)):
            i = k % len(side)
            r = L.ctaug_warp_affine_backward(ctypes.byref(vi[k]), Mc[k], jobs[k].fill, None,
                                             ctypes.byref(vg[k]), ctypes.byref(vgi[k]),
                                             ctypes.c_void_p(g_M[k].data_ptr()),
                                             ctypes.c_void_p(ws[i].data_ptr()), ws_bytes,
                                             side.handle(i))
            assert r == 0
        side.join()

    # the batched adjoint: one launch over the 8 volumes, one reduction
    bjobs = (ctaug._lib.BwdJob * len(jobs))(*[
        ctaug.ops.make_bwd_job(imgs[k], Ms[k], gs[k], grad_img=g_imgs[k], grad_M=g_M[k],
                               fill=jobs[k].fill) for k in range(len(jobs))])
    bws = torch.empty(ctaug.ops.warp_affine_backward_batch_workspace(len(jobs)), dtype=torch.uint8,
                      device=dev)

    def bwd_batch():
        g_all.zero_()
        ctaug.ops.warp_affine_backward_batch(bjobs, bws)

    f_ms = time_loop(fwd, reps, stream)
    fb_ms = time_loop(lambda: (fwd(), bwd_batch()), reps, stream)
    fb_vol_ms = time_loop(lambda: (fwd(), bwd()), reps, stream)
    sf_ms, sb_ms = time_split([fwd, bwd_batch], reps, stream)
    nv = sum(o.numel() for o in outs)
    plan.close()
    return {"workload": "8 x 128^3 f32 affine warp; backward to image (tile sums in fixed point, "
                        "incl. zeroing) and to the 12 affine params (FP64 reduction) in one "
                        "batched launch",
            "fwd_ms": round(f_ms, 4), "fwd_bwd_ms": round(fb_ms, 4),
            "fwd_gvoxel_s": round(nv / f_ms / 1e6, 2), "fwd_bwd_gvoxel_s": round(nv / fb_ms / 1e6, 2),
            "fwd_bwd_over_fwd": round(fb_ms / f_ms, 3),
            "per_volume_calls_fwd_bwd_ms": round(fb_vol_ms, 4),
            "per_volume_calls_note": "8 backward calls alternating over 2 streams",
            "in_sequence_fwd_ms": round(sf_ms, 4), "in_sequence_bwd_ms": round(sb_ms, 4),
            "in_sequence_fwd_bwd_over_fwd": round((sf_ms + sb_ms) / sf_ms, 3),
            "in_sequence_note": "forward and backward each timed with events inside the "
                                "forward-then-backward sequence; fwd_ms repeats the forward "
                                "alone, whose 134 MB stay in the 256 MB Infinity Cache"}


def run_c5(dev, stream, reps):
    """Nonrigid workload: forward with the B-spline field evaluated inside the
    warp, and the adjoint with the control-grid gradient fused in (through the
    C ABI, buffers allocated once); the unfused route (dense field through
    memory) timed beside it."""
    import torch

    import paper_1811_11226_amd as ctaug
    from synth import configs
    jobs, ctrls, grads = configs.c5()
    imgs = [torch.from_numpy(j.img).to(dev) for j in jobs]
    cs = [torch.from_numpy(c).to(dev) for c in ctrls]
    gs = [torch.from_numpy(g).to(dev) for g in grads]
    Ms = [ctaug.affine_matrix(j.prm, j.in_dim, j.out_dim)[1] for j in jobs]
    us = [torch.empty((3,) + j.out_dim, dtype=torch.float32, device=dev) for j in jobs]
    outs = [torch.empty(j.out_dim, dtype=torch.float32, device=dev) for j in jobs]
    L = ctaug._lib.load()
    P = ctypes.c_void_p
    od = (ctypes.c_int64 * 3)(*jobs[0].out_dim)
    G = (ctypes.c_int64 * 3)(*ctrls[0].shape[1:])
    side = SideStreams(len(jobs))        # one stream per volume's backward
    ws_bytes = int(L.ctaug_warp_bspline_backward_workspace(od, G))
    ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=dev) for _ in range(len(side))]
    g_all = torch.empty((len(jobs),) + tuple(imgs[0].shape), dtype=torch.float32, device=dev)
    g_imgs = [g_all[k] for k in range(len(jobs))]
    g_Ms = [torch.empty(12, dtype=torch.float64, device=dev) for _ in jobs]
    g_cs = [torch.empty_like(c) for c in cs]
    vi = [ctaug.ops.vol(i) for i in imgs]
    vg = [ctaug.ops.vol(g) for g in gs]
    vgi = [ctaug.ops.vol(g) for g in g_imgs]
    Mc = [ctaug.ops._M32(M) for M in Ms]

    def fwd():
        for k, j in enumerate(jobs):
            ctaug.warp_bspline(imgs[k], Ms[k], cs[k], fill=j.fill, photo=j.photo, out=outs[k])

    def bwd():
        g_all.zero_()
        side.fork()
        for k, j in enumerate(jobs):
            i = k % len(side)
            r = L.ctaug_warp_bspline_backward(ctypes.byref(vi[k]), Mc[k], P(cs[k].data_ptr()), G,
                                              j.fill, None, ctypes.byref(vg[k]),
                                              ctypes.byref(vgi[k]),
                                              P(g_Ms[k].data_ptr()), P(g_cs[k].data_ptr()),
                                              P(ws[i].data_ptr()), ws_bytes, side.handle(i))
            assert r == 0
        side.join()

    def fwd_dense():
        for k, j in enumerate(jobs):
            ctaug.bspline_upsample(cs[k], j.out_dim, out=us[k])
            ctaug.warp_displacement(imgs[k], Ms[k], us[k], fill=j.fill, photo=j.photo, out=outs[k])

    def bwd_dense():
        for k, j in enumerate(jobs):
            _, _, g_u = ctaug.warp_displacement_backward(imgs[k], Ms[k], us[k], gs[k], fill=j.fill)
            ctaug.bspline_upsample_adjoint(g_u, ctrls[k].shape[1:])

    f_ms = time_loop(fwd, reps, stream)
    fb_ms = time_loop(lambda: (fwd(), bwd()), reps, stream)
    sf_ms, sb_ms = time_split([fwd, bwd], reps, stream)
    fd_ms = time_loop(fwd_dense, reps, stream)
    fbd_ms = time_loop(lambda: (fwd_dense(), bwd_dense()), reps, stream)
    nv = sum(o.numel() for o in outs)
    return {"workload": "4 x 256^3 f32, affine + cubic B-spline displacement (8^3 control grid) "
                        "evaluated in the warp, noise; backward to image, params and control grid "
                        "(fused); each volume's backward call on a stream of its own",
            "fwd_ms": round(f_ms, 4), "fwd_bwd_ms": round(fb_ms, 4),
            "fwd_gvoxel_s": round(nv / f_ms / 1e6, 2), "fwd_bwd_gvoxel_s": round(nv / fb_ms / 1e6, 2),
            "fwd_bwd_over_fwd": round(fb_ms / f_ms, 3),
            "in_sequence_fwd_ms": round(sf_ms, 4), "in_sequence_bwd_ms": round(sb_ms, 4),
            "in_sequence_fwd_bwd_over_fwd": round((sf_ms + sb_ms) / sf_ms, 3),
            "dense_field_fwd_ms": round(fd_ms, 4), "dense_field_fwd_bwd_ms": round(fbd_ms, 4)}


def run_warp_only(sets, dev, stream, tuning, reps=30):
    """The 16-volume batches with the photometric chain and the labels off: the
    pure trilinear gather, whose bound is HBM (algorithmic bytes: 4 per output
    voxel written, 2 per touched int16 input voxel read).  The three input sets
    rotate, as in the headline measurement."""
    import numpy as np
    import torch

    import paper_1811_11226_amd as ctaug
    plans, nbytes = [], []
    nv = C3_OUT[0] * C3_OUT[1] * C3_OUT[2]
    for cs in sets:
        jobs = [ctaug.make_job(cs.imgs[k], cs.pool[0][k][0], cs.outs[k], fill=j.fill)
                for k, j in enumerate(cs.jobs)]
        plans.append(ctaug.BatchPlan(jobs, tile=tuning[0], wg_per_cu=tuning[1],
                                     lds_cells=tuning[2], lds_format=tuning[3]))
        b = 0
        for k, j in enumerate(cs.jobs):
            ti, _, _ = touched_counts(j.in_dim, C3_OUT, cs.pool[0][k][0], dev)
            b += nv * 4 + ti * 2
        nbytes.append(b)
    with torch.cuda.stream(stream):
        for p in plans:
            p.launch()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    with torch.cuda.stream(stream):
        for i, (a, b) in enumerate(evs):
            a.record(stream)
            plans[i % len(plans)].run()
            b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    for p in plans:
        p.close()
    b = float(np.mean(nbytes))
    gbs = b / ms / 1e6
    return {"workload": "the 16-volume batches, trilinear warp only (no labels, no photometrics)",
            "kernel_ms": round(ms, 4), "gvoxel_s": round(sets[0].voxels() / ms / 1e6, 2),
            "alg_bytes": int(b), "alg_GBs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}


def run_fifo(cset, dev, reps=6):
    """The 16-volume batch streamed from pinned host memory through the
    host-to-device FIFO (one slot per volume, each filled once beforehand):
    PCIe-inclusive throughput with transfers overlapping the warps, beside
    the same submissions with a full synchronisation after each volume and
    beside the bare transfers of the same bytes (pinned host to device, one
    stream, no warps), which bound the FIFO from below.  The three legs
    alternate and each reports the median of its repeats."""
    import numpy as np
    import torch

    import paper_1811_11226_amd as ctaug
    jobs = cset.jobs
    slot = max(ctaug.Pipeline.slot_bytes_for(j.img.shape, j.img.dtype) for j in jobs)
    outs, louts = cset.outs, cset.louts
    pipe = ctaug.Pipeline(len(jobs), slot)
    addrs = []
    for k, j in enumerate(jobs):                # fill every slot once (producer side)
        a = pipe.acquire()
        ctypes.memmove(a, j.img.ctypes.data, j.img.nbytes)
        la = a + (j.img.nbytes + 255) // 256 * 256
        ctypes.memmove(la, j.lbl.ctypes.data, j.lbl.nbytes)
        addrs.append((a, la))
        M, ph = cset.pool[0][k]
        pipe.submit(a, j.img, M, la, j.lbl, fill=j.fill, photo=ph, out=outs[k], lbl_out=louts[k])
    pipe.sync()
    hosts = [torch.from_numpy(a).pin_memory() for j in jobs for a in (j.img, j.lbl)]
    devs = [torch.empty_like(h, device=dev) for h in hosts]
    copy_stream = torch.cuda.Stream()

    def one_pass(serial):
        for k, j in enumerate(jobs):
            a, la = addrs[k]
            assert pipe.acquire() == a
            M, ph = cset.pool[0][k]
            pipe.submit(a, j.img, M, la, j.lbl, fill=j.fill, photo=ph, out=outs[k],
                        lbl_out=louts[k])
            if serial:
                pipe.sync()
        pipe.sync()

    def copy_only():
        with torch.cuda.stream(copy_stream):
            for h, d in zip(hosts, devs):
                d.copy_(h, non_blocking=True)
        torch.cuda.synchronize()

    legs = {"pipelined": lambda: one_pass(False), "serial": lambda: one_pass(True),
            "copy_only": copy_only}
    times = {k: [] for k in legs}
    for f in legs.values():
        f()
    for _ in range(reps):
        for k, f in legs.items():
            t0 = time.perf_counter()
            f()
            times[k].append((time.perf_counter() - t0) * 1e3)
    ms = {k: float(np.median(v)) for k, v in times.items()}
    pipe.close()
    in_bytes = sum(j.img.nbytes + j.lbl.nbytes for j in jobs)
    nv = cset.voxels()
    return {"workload": "the 16-volume batch (int16 + int8 labels) streamed from pinned host "
                        "memory: per volume H2D copy then fused warp, copies on their own stream",
            "pipelined_ms": round(ms["pipelined"], 3), "serial_ms": round(ms["serial"], 3),
            "copy_only_ms": round(ms["copy_only"], 3),
            "pipelined_gvoxel_s": round(nv / ms["pipelined"] / 1e6, 2),
            "serial_gvoxel_s": round(nv / ms["serial"] / 1e6, 2),
            "h2d_GBs_pipelined": round(in_bytes / ms["pipelined"] / 1e6, 1),
            "h2d_GBs_copy_only": round(in_bytes / ms["copy_only"] / 1e6, 1),
            "overlap_speedup": round(ms["serial"] / ms["pipelined"], 3),
            "copy_only_over_pipelined": round(ms["copy_only"] / ms["pipelined"], 3)}


def copy_bandwidth(dev, stream, nbytes=1 << 30, reps=10):
    import torch

    import paper_1811_11226_amd as ctaug
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    ms = time_loop(lambda: ctaug.ops.copy(src, dst), reps, stream)
    return 2 * nbytes / ms / 1e6


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, as it stands, on this host's cores
# ---------------------------------------------------------------------------

def cpu_baseline(sets, min_seconds=10.0):
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    s = sets[0]
    nv = 0
    passes = 0
    t0 = time.perf_counter()
    while passes == 0 or time.perf_counter() - t0 < min_seconds:
        for k, j in enumerate(s.jobs):
            M, ph = s.pool[0][k]
            oracle.warp(j.img, M, C3_OUT, lbl=j.lbl, fill=j.fill, label_fill=j.label_fill,
                        photo=ph)
            nv += C3_OUT[0] * C3_OUT[1] * C3_OUT[2]
        passes += 1
    dt = time.perf_counter() - t0
    return {"value": round(nv / dt / 1e9, 5), "unit": "Gvoxel/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the 16-volume batch {passes}x ({nv / 1e6:.1f} Mvoxel out), {dt:.2f} s "
                      f"wall, oracle in parity mode (FP32-pinned coordinates, FP64 "
                      f"interpolation), OpenMP over x-slabs"}


def write_traffic(fetch_csv, write_csv, copy_bytes=1 << 30):
    """Summarise two rocprofv3 --pmc runs of `bench.py --profile` (FETCH_SIZE,
    then WRITE_SIZE) into profiles/warp_batch_c3_traffic.txt: per-dispatch KiB of
    the batched kernel, scaled by what the same counter reads for the copy
    kernel moving copy_bytes each way."""
    import csv

    def per_kernel(path, counter):
        vals = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name = r["Kernel_Name"]
                key = "batch" if "k_warp_batch" in name else "copy" if "k_copy16" in name else None
                if key:
                    vals.setdefault(key, []).append(float(r["Counter_Value"]))
        return vals

    fv, wv = per_kernel(fetch_csv, "FETCH_SIZE"), per_kernel(write_csv, "WRITE_SIZE")
    mean = lambda v: sum(v) / len(v)
    f_scale = mean(fv["copy"]) * 1024.0 / copy_bytes
    w_scale = mean(wv["copy"]) * 1024.0 / copy_bytes
    fetch = mean(fv["batch"]) * 1024.0 / f_scale
    write = mean(wv["batch"]) * 1024.0 / w_scale
    path = os.path.join(ROOT, "profiles", "warp_batch_c3_traffic.txt")
    with open(path, "w") as f:
        f.write("# HBM-side traffic of k_warp_batch on the 16-volume 120x120x160 batch\n")
        f.write("# (cd /tmp && export TMPDIR=/tmp)\n")
        for c in ("FETCH_SIZE", "WRITE_SIZE TCC_HIT_sum TCC_MISS_sum"):
            f.write(f"# timeout -s KILL 240 rocprofv3 --pmc {c} --kernel-include-regex "
                    f"'k_warp_batch|k_copy16' --output-format csv -d <dir> -o run -- "
                    f"python3 bench.py --profile --steps 20 --warmup 2\n")
        f.write("# python3 bench.py --traffic <FETCH_SIZE dir>/run_counter_collection.csv "
                "<WRITE_SIZE dir>/run_counter_collection.csv\n")
        f.write("# KiB per dispatch (mean over the batched kernel's dispatches) scaled by\n")
        f.write("# what the same counter reads for the copy kernel moving 1 GiB each way\n")
        f.write(f"batch_dispatches = {len(fv['batch'])}\n")
        f.write(f"fetch_kib_raw = {mean(fv['batch']):.1f}\n")
        f.write(f"write_kib_raw = {mean(wv['batch']):.1f}\n")
        f.write(f"copy_fetch_scale = {f_scale:.4f}\n")
        f.write(f"copy_write_scale = {w_scale:.4f}\n")
        f.write(f"fetch_bytes_per_launch = {fetch:.0f}\n")
        f.write(f"write_bytes_per_launch = {write:.0f}\n")
        f.write(f"hbm_bytes_per_launch = {fetch + write:.0f}\n")
        f.write(f"source_sha256 = {source_hash()}\n")
    print(path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="short run for rocprofv3: headline workload + copy reference only")
    ap.add_argument("--profile-adjoint", action="store_true",
                    help="short run for rocprofv3: the 8 x 128^3 and 4 x 256^3 forward + "
                         "adjoint workloads and the copy reference only")
    ap.add_argument("--autotune", action="store_true",
                    help="sweep launch shapes on the headline workload and rewrite the "
                         "autotune cache file the plans read")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/warp_batch_c3_traffic.txt from two rocprofv3 --pmc "
                         "counter_collection.csv files and exit (no GPU needed)")
    args = ap.parse_args()
    if args.traffic:
        write_traffic(*args.traffic)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (each volume of a batch is "
              "independent; a multi-GPU run would shard volumes across GPUs with no exchange)",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        args.no_secondary = args.no_cpu = True

    import torch

    from paper_1811_11226_amd import _lib
    _lib.load()                           # fails loudly if the HIP library is missing
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(0)
    log(f"device {props.name} {getattr(props, 'gcnArchName', '')} CUs={props.multi_processor_count}")

    if args.profile_adjoint:
        stream = torch.cuda.Stream()
        copy_bandwidth(dev, stream, reps=3)
        out = {"diff_affine_8x128": run_c4(dev, stream, reps=3),
               "nonrigid_4x256": run_c5(dev, stream, reps=2)}
        print(json.dumps(out), flush=True)
        return

    r = run_c3(args, dev)
    stream = r["stream"]
    copy_gbs = copy_bandwidth(dev, stream)
    log(f"copy reference kernel: {copy_gbs:.0f} GB/s")
    value = r["voxels"] / (r["step_ms"] * 1e-3) / 1e9
    hbm_gbs = r["alg_bytes"] / (r["kern_ms"] * 1e-3) / 1e9
    achieved = r["alg_ops"] / (r["kern_ms"] * 1e-3) / 1e12
    traffic = stored_traffic("warp_batch_c3")
    result = {
        "metric": "augmented Gvoxel/s + % HBM peak (fwd, fwd+bwd) at 1 GPU vs CPU oracle",
        "value": round(value, 3),
        "unit": "Gvoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r["step_ms"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched fused forward: 16 int16 CT phantoms, per-axis sizes U{96..256}, "
                        "each with its own affine (rot U(+-30 deg), scale U(0.8,1.2), shift "
                        "U(+-10), crop) and photometrics (gain, offset, noise sigma 10 HU, "
                        "window [-1000,1000], gamma) -> 120x120x160 f32 + int8 NN labels; one "
                        + ("launch per batch with one workgroup per output tile"
                           if r["tuning"][1] == 0 else
                           f"persistent launch per batch ({r['tuning'][1]} workgroups per CU)")
                        + ", descriptor upload and launch replayed from a hipGraph",
            "global_batch": 16,
            "out_dim": list(C3_OUT),
            "tile": list(r["tuning"][0]),
            "wg_per_cu": r["tuning"][1],
            "lds_cells": r["tuning"][2],
            "lds_format": "int16" if r["tuning"][3] == 1 else "f32",
            "launch_shape_from": "autotune cache" if r["cached"] else "library default",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(hbm_gbs, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(hbm_gbs / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else int(traffic),
            "kernel": "k_warp_batch",
            "kernel_ms": round(r["kern_ms"], 5),
            "algorithmic_bytes_per_launch": int(r["alg_bytes"]),
            "traffic_over_algorithmic": None if traffic is None else
            round(traffic / r["alg_bytes"], 3),
            "copy_kernel_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(hbm_gbs / copy_gbs, 4),
            "kernel_ms_p10_p50_p90": [round(v, 5) for v in r["kern_pct"]],
            "valu": {"achieved_TOPs": round(achieved, 3), "peak_TOPs": round(ALU_PEAK_TOPS, 2),
                     "frac": round(achieved / ALU_PEAK_TOPS, 4),
                     "algorithmic_lane_ops_per_launch": int(r["alg_ops"])},
        },
        "host_enqueue_ms_per_step": {"timed_loop": round(r["host_ms"], 4),
                                     "without_wait": round(r["host_nowait_ms"], 4)},
        "device": {"name": props.name, "arch": getattr(props, "gcnArchName", ""),
                   "cus": props.multi_processor_count, "hip": torch.version.hip},
    }
    if not args.no_cpu:
        log("cpu baseline: oracle on the batch")
        result["cpu_baseline"] = cpu_baseline(r["sets"])
    if not args.no_secondary:
        sec = {}
        log("secondary: 512x512x320")
        sec["full_res_512x512x320"] = run_c2(dev, stream, reps=10)
        log("secondary: labels resampled back")
        sec["labels_back_512x512x320"] = run_labels_back(dev, stream, reps=20)
        log("secondary: 8 x 128^3 fwd / fwd+bwd")
        sec["diff_affine_8x128"] = run_c4(dev, stream, reps=10)
        log("secondary: 4 x 256^3 nonrigid fwd / fwd+bwd")
        sec["nonrigid_4x256"] = run_c5(dev, stream, reps=5)
        log("secondary: warp only")
        sec["warp_only_c3"] = run_warp_only(r["sets"], dev, stream, r["tuning"])
        log("secondary: host-to-device FIFO")
        sec["host_fifo_c3"] = run_fifo(r["sets"][0], dev)
        result["secondary"] = sec
    for s in r["sets"]:
        s.plan.close()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
