#!/usr/bin/env python
"""Benchmark: differentiable Gaussian-splat render forward + backward on one GPU.

Workload (tracking/mapping-shaped): 200k Gaussians in a 6 x 3 x 4 m room-shaped
box, 1200 x 680 pinhole (f = 600), L1 RGB + depth loss against a render at a
pose perturbed by 2 deg / 3 cm.  One step = one optimisation iteration:
project -> tile binning -> composite forward -> L1 loss -> composite backward
-> projection backward -> Adam on every Gaussian parameter and on the camera
pose.  Inputs are resident in HBM before timing; no host sync inside a step.
Every call of the step is timed with HIP events on the launch stream, which
gives each kernel group's HBM fraction from its algorithmic bytes.

The same loop is then timed with the full mapping loss (L1 + SSIM colour
term, depth term, isotropic scale regulariser), followed by the opacity
pruning of the submap, the map adjustment after pose-graph optimisation (64
resident submaps of 200k Gaussians) and the geometric overlap ratio of the
registration pair's submaps.

Then the registration workloads (keyframe localisation with the paper's
colour + depth L1, 200 Adam iterations per view; the masked tracking loss as
a labelled variant):
  - one pair of 150k + 120k Gaussians with 8 + 8 keyframes at 640x480, with
    all views and with the paper's k = 2 views per direction;
  - a set of 32 pairs (Gaussians per submap log-uniform in [20k, 300k],
    4..12 keyframes each at 640x480, each with its own ground truth), run
    one pair at a time through ls_register_pair ("plain") and all submitted
    at once to the continuous-batching server ("batched");
  - the same sizes with the x-split layout (a stress set whose uneven pairs
    see content only one submap holds);
  - a serving stream of Poisson arrivals (20 requests/s, submap sizes
    lognormal with median 100k, 640x480 or 1200x680): the plain path as a
    FIFO queue against the server with and without an active-pixel cap.

Synthetic inputs are generated, and the FP64 CPU oracle is timed on a
bounded sample of the render workload (single process, then one process per
host core), before the GPU is touched.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work of the compositing kernels per evaluated fragment (a
# (pixel, list entry) pair up to and including the one that stops the pixel),
# as counted for the hot-path scope: forward ~20 ops (1 exponential + ~18
# FP32 ops), backward ~45.  The count derived from this build's instruction
# mix (per evaluated entry + per composited entry) is reported beside it.
FWD_OPS_PER_FRAG, BWD_OPS_PER_FRAG = 20, 45
FWD_EVAL, FWD_COMP = 14, 11
BWD_EVAL, BWD_COMP = 14, 53
# mapping-loss kernel, algorithmic work per pixel: HBM bytes (rendered and
# target colour 24, rendered and target depth 8, colour and depth gradients
# 16) and FP32 operations (separable 11-tap filtering of five moments and of
# three derivative maps, the index and its derivatives: ~390 per channel).
MAP_BYTES_PX = 48
MAP_FLOPS_PX = 3 * 390
PEAK_FP32_TFLOPS = 157.3   # MI355X published FP32 vector peak (FMA = 2, packed)
PEAK_LANE_OPS_T = 39.3     # unpacked issue rate: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
PEAK_HBM_GBS = 8000.0


def algorithmic_bytes(n: int, inst: int, px: int, tiles: int) -> dict:
    """HBM bytes of one render-loop step per kernel group, each array read or
    written once: per Gaussian, per tile instance, per pixel and per tile."""
    return {
        "project": 88 * n,                                # parameters 56 in, record 32 out
        "bin_sort": 28 * n + 44 * inst + 8 * tiles,       # scan 8 + emit read 20; emit 12, sort 24, ranges 8
        "fwd": 44 * inst + 28 * px,                       # record gather, image out
        # the L1 gradient is formed inside the backward, which also writes each tile's loss
        # partial; "loss" is the per-render sum of those partials
        "loss": 8 * tiles,
        "bwd": 44 * inst + 60 * px + 40 * n + 8 * tiles,  # records, image state + images + targets, 2D grads
        # projection backward with the Adam steps of the Gaussians and the pose fused: 2D gradients
        # 40, parameters 56 in and out, moments 112 in and out (the gradients never go to memory)
        "bwd_project_adam": 376 * n,
    }


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None if the kernel source changed since the counters were taken."""
    import hashlib

    src = b"".join(open(os.path.join(ROOT, "paper_2408_10154_amd", "csrc", f), "rb").read()
                   for f in ("composite.hip", "common.h"))
    digest = hashlib.sha256(src).hexdigest()[:16]
    path = os.path.join(ROOT, "profiles", "render_loop_200k_1200x680_hbm_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        f = line.split()
        if len(f) == 5 and f[0] == "traffic" and f[1] == kernel and f[3] == "source":
            return int(f[2]) if f[4] == digest else None
    return None


def measured_valu_busy(kernel: str):
    """VALU-busy share of `kernel` on the render loop from the committed SQ
    counter summary (None when absent)."""
    path = os.path.join(ROOT, "profiles", "compositing_200k_1200x680_and_registration_pair_valu_counters.md")
    if not os.path.exists(path):
        return None
    for line in open(path):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) >= 6 and cells[0] == f"ls::k_{kernel}" and cells[4].endswith("%"):
            return float(cells[4][:-1]) / 100.0
    return None


def log(msg: str):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--kernel-steps", type=int, default=10,
                    help="steps after the timed region with HIP events around every call (per-kernel table)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-tiles", type=int, default=1600, help="tiles in the oracle's timed sample")
    ap.add_argument("--cpu-workers", type=int, default=0, help="oracle processes (0: host cores, at most 16)")
    ap.add_argument("--gaussians", type=int, default=200_000)
    ap.add_argument("--pairs", type=int, default=32, help="pairs in the batched-vs-plain registration set")
    ap.add_argument("--reg-iters", type=int, default=200)
    ap.add_argument("--no-registration", action="store_true")
    ap.add_argument("--no-stress", action="store_true", help="skip the x-split stress set")
    ap.add_argument("--stream-requests", type=int, default=24, help="requests of the serving stream (0: skip)")
    ap.add_argument("--stream-rate", type=float, default=20.0, help="stream arrivals per second")
    ap.add_argument("--mapping-steps", type=int, default=20,
                    help="timed iterations of the same loop with the full mapping loss (0: skip)")
    ap.add_argument("--no-overlap", action="store_true", help="skip the overlap-ratio timing")
    ap.add_argument("--no-prune", action="store_true", help="skip the opacity-pruning timing")
    ap.add_argument("--adjust-submaps", type=int, default=64,
                    help="submaps of 200k Gaussians in the timed map adjustment (0: skip)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device once (a known-size kernel that "
                         "calibrates HBM byte counters in a profiler run)")
    return ap.parse_args()


# ---------------------------------------------------------------- CPU phase

def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _oracle_tiles(scene, tiles):
    """One process's share of the oracle's sample: projection and binning of
    all Gaussians, then forward + L1 loss + backward on `tiles` (one torch
    thread).  Returns (seconds for project+bin, seconds for the tiles, pixels)."""
    import numpy as np
    import torch

    from oracle import raster as R

    torch.set_num_threads(1)
    cam = R.Camera(**scene["cam"])
    w2c = torch.as_tensor(np.asarray(scene["w2c"], np.float64))
    g = R.to_f64(scene["gauss"], requires_grad=True)
    pose = R.identity_pose().requires_grad_(True)
    t0 = time.perf_counter()
    pr = R.project(g["mean"], g["log_scale"], g["quat"], cam, w2c, pose)
    _, gid, ranges = R.bin_sort(pr["u32"], pr["v32"], pr["z32"], pr["radius"], cam)
    t1 = time.perf_counter()
    out = R.composite(pr["u"], pr["v"], pr["conic"], torch.sigmoid(g["opacity_logit"]), g["rgb"], pr["depth"], gid,
                      ranges, cam, tiles_subset=np.asarray(tiles), with_margins=False)
    loss = R.loss_l1(out["rgb"], out["depth"], out["rgb"].detach() * 0.9, out["depth"].detach() * 1.01 + 0.01)
    loss.backward()
    t2 = time.perf_counter()
    px = 0
    for t in tiles:
        ty, tx = divmod(int(t), cam.tiles_x)
        px += min(16, cam.height - ty * 16) * min(16, cam.width - tx * 16)
    return t1 - t0, t2 - t1, px


def cpu_baseline(scene, sample_tiles: int, workers: int):
    """The FP64 oracle on a bounded sample of the render workload: projection
    and binning of all Gaussians, then forward + L1 + backward on
    `sample_tiles` evenly spaced tiles, first in one process with one thread,
    then split over `workers` forked processes with one thread each (every
    process projects all Gaussians itself).  Per-image times are
    extrapolated by tile count: one process t_bin + tiles * t_tile; N
    processes max t_bin + (tiles / N) * max per-tile time.  Every run is a
    forked child process."""
    import multiprocessing as mp

    import numpy as np

    cam = scene["cam"]
    ntiles = ((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16)
    subset = np.linspace(0, ntiles - 1, sample_tiles).round().astype(int)
    pixels = cam["width"] * cam["height"]
    # every oracle run is a forked child: autograd threads started in this
    # process would make later forks unusable
    with mp.get_context("fork").Pool(1) as pool:
        tb, tt, px = pool.starmap(_oracle_tiles, [(scene, subset)])[0]
    t1 = tb + ntiles * tt / len(subset)
    single = dict(value=pixels / t1 / 1e6, cores=1, seconds_per_image=round(t1, 2),
                  sample=f"{len(subset)} of {ntiles} tiles ({px} px): project+bin {tb:.1f} s, tiles {tt:.1f} s")
    out = dict(unit="Mpixels/s", kind="oracle", cpu_model=_cpu_model(), host_cores=_host_cores(),
               single_process=single)
    if workers > 1:
        parts = [subset[i::workers] for i in range(workers)]
        with mp.get_context("fork").Pool(workers) as pool:
            t0 = time.perf_counter()
            res = pool.starmap(_oracle_tiles, [(scene, p) for p in parts])
            wall = time.perf_counter() - t0
        tbm = max(r[0] for r in res)
        per_tile = max(r[1] / len(p) for r, p in zip(res, parts))
        tn = tbm + (ntiles / workers) * per_tile
        out.update(value=pixels / tn / 1e6, cores=workers,
                   sample=(f"FP64 oracle, one fwd+L1+bwd of the 200k-Gaussian 1200x680 render: {len(subset)} of "
                           f"{ntiles} tiles over {workers} processes x 1 thread ({wall:.1f} s wall; each process "
                           f"projects and bins all Gaussians in {tbm:.1f} s); per-image time {tn:.1f} s extrapolated "
                           "by tile count"))
    else:
        out.update(value=single["value"], cores=1, sample="single process: " + single["sample"])
    return out


# ---------------------------------------------------------------- GPU parts

def _events(stream, fn):
    import torch

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    return e0, e1


def map_adjust(n_sub: int, n: int = 200_000, poses: int = 100, reps: int = 20):
    """Globally consistent map adjustment after pose-graph optimisation:
    n_sub resident submaps of n Gaussians and `poses` keyframes each, every
    one moved by its own rigid correction (means, quaternions, poses in
    place), timed with HIP events on the launch stream."""
    import types

    import numpy as np
    import torch

    from paper_2408_10154_amd.render import adjust_submaps

    rng = np.random.default_rng(5)
    mean = torch.rand(n_sub, 3, n, device="cuda") * 4.0 - 2.0
    quat = torch.randn(n_sub, 4, n, device="cuda")
    c2w = torch.zeros(n_sub, poses, 12, device="cuda")
    c2w[:, :, 0] = c2w[:, :, 5] = c2w[:, :, 10] = 1.0
    subs = []
    for k in range(n_sub):
        ang = rng.normal(size=3) * 0.01
        c, s_ = math.cos(ang[2]), math.sin(ang[2])
        T = np.array([[c, -s_, 0.0, ang[0]], [s_, c, 0.0, ang[1]], [0.0, 0.0, 1.0, 0.0]])
        subs.append((types.SimpleNamespace(n=n, mean=mean[k], quat=quat[k]), c2w[k], T))
    stream = torch.cuda.current_stream()
    adjust_submaps(subs)
    torch.cuda.synchronize()
    evs = [_events(stream, lambda: adjust_submaps(subs)) for _ in range(reps)]
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in evs)[reps // 2]
    algo = 56 * n * n_sub + 96 * poses * n_sub  # mean 12 + quat 16 read and written; poses 48 + 48
    # practical roof: a device-to-device copy moving the same bytes (half read, half written)
    src = torch.empty(algo // 8, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    cev = [_events(stream, lambda: dst.copy_(src)) for _ in range(reps)]
    torch.cuda.synchronize()
    cms = sorted(a.elapsed_time(b) for a, b in cev)[reps // 2]
    del src, dst
    return {"submaps": n_sub, "gaussians": n * n_sub, "keyframes": poses * n_sub, "ms": round(ms, 4),
            "achieved_gbs": round(algo / (ms * 1e-3) / 1e9, 1), "bound": "hbm",
            "frac": round(algo / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "same_bytes_copy_gbs": round(algo / (cms * 1e-3) / 1e9, 1)}


def prune_timing(reps: int = 20):
    """Opacity pruning after mapping (o_thre 0.5, the real-data setting) of
    one 200k-Gaussian submap and of 12.8 M Gaussians in one call, with the
    five parameter arrays and two Adam moments per parameter compacted:
    median call time (HIP events around ls_prune_gaussians, no host read-back
    inside) and HBM fraction of the algorithmic bytes: every array read once
    (the logit and 14 floats x 3 arrays per Gaussian: with half of the
    Gaussians kept at random every cache line of the inputs is needed) and
    the kept Gaussians' 42 floats and index written once."""
    import numpy as np
    import torch

    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd import synth
    from paper_2408_10154_amd.render import GaussianSet

    out = {}
    stream = torch.cuda.current_stream()
    sp = L.C.c_void_p(stream.cuda_stream)
    for n in (200_000, 12_800_000):
        rng = np.random.default_rng(n)
        g = synth.gaussians_in_box(rng, n, (-3, -1.5, 0.5), (3, 1.5, 4.5))
        gs = GaussianSet.from_numpy(g)
        srcs = [getattr(gs, k) for k in GaussianSet.FIELDS]
        srcs += [torch.zeros_like(t) for t in srcs for _ in range(2)]
        dsts = [torch.empty_like(t) for t in srcs]
        arr = (L.ls_prune_array * len(srcs))(*[L.ls_prune_array(a.data_ptr(), d.data_ptr(),
                                                                 1 if a.dim() == 1 else a.shape[0], 0)
                                               for a, d in zip(srcs, dsts)])
        kept = torch.empty(n, dtype=torch.int32, device="cuda")
        count = torch.empty(1, dtype=torch.int32, device="cuda")
        work = torch.empty(L.ls_prune_workspace_size(n), dtype=torch.uint8, device="cuda")

        def call():
            L.ls_prune_gaussians(gs.opacity_logit.data_ptr(), n, 0.5, arr, len(srcs), kept.data_ptr(),
                                 count.data_ptr(), work.data_ptr(), work.numel(), sp)

        call()
        evs = [_events(stream, call) for _ in range(reps)]
        torch.cuda.synchronize()
        k = int(count.item())
        ms = sorted(a.elapsed_time(c) for a, c in evs)[reps // 2]
        algo = 4 * n + n * 4 * 14 * 3 + k * (4 * 14 * 3 + 4)
        out[str(n)] = {"kept": k, "ms": round(ms, 4), "achieved_gbs": round(algo / (ms * 1e-3) / 1e9, 1),
                       "frac": round(algo / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        del gs, srcs, dsts, kept, work
        torch.cuda.empty_cache()
    out["note"] = "o_thre 0.5 on opacity logits N(0, 1); 5 parameter arrays and 2 moments each compacted"
    return out


def overlap(reps: int = 10):
    """Geometric overlap ratio (reciprocal nearest neighbours, tau = 0.2 m)
    of the single-pair registration workload's submaps (150k + 120k
    Gaussians) under the ground truth and under the identity, timed with HIP
    events on the launch stream (inputs resident)."""
    import numpy as np
    import torch

    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd import synth
    from paper_2408_10154_amd.render import overlap_ratio

    d = synth.registration_pair(2, 150_000, 120_000, views_p=1, views_q=1, layout="views")
    p = torch.as_tensor(np.asarray(d["P"]["mean"], np.float32), device="cuda").contiguous()
    q = torch.as_tensor(np.asarray(d["Q"]["mean"], np.float32), device="cuda").contiguous()
    work = torch.empty(L.ls_overlap_workspace_size(p.shape[1], q.shape[1]), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    out = {}
    for name, T in (("ground_truth", d["T_gt"]), ("identity", np.eye(4))):
        r, pairs, inl, _, _ = overlap_ratio(p, q, T, 0.2, work=work)
        evs = [_events(stream, lambda: overlap_ratio(p, q, T, 0.2, work=work)) for _ in range(reps)]
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in evs)[reps // 2]
        out[name] = {"ratio": round(r, 4), "pairs": pairs, "within_tau": inl, "ms": round(ms, 4)}
    out["points"] = [int(p.shape[1]), int(q.shape[1])]
    return out


def _rnd(d):
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}


def registration(host, iters: int):
    """Single-pair time and accuracy (all views and k = 2), then the pair
    set plain vs batched with both losses, the stress set and the serving
    stream.  Results of the plain and batched paths are compared bit for bit."""
    import numpy as np
    import torch

    from paper_2408_10154_amd import regbench as RB
    from paper_2408_10154_amd import register as REG

    def errs(res, p):
        return dict(rot_deg=round(REG.rotation_error_deg(res["T"], p["T_gt"]), 4),
                    trans_cm=round(REG.translation_error_cm(res["T"], p["T_gt"]), 4))

    spec1, d1 = host["single"]
    one = [RB.upload_pair(d1, spec1)]
    RB.run_plain(one, iters=10)                                  # warm-up
    single = dict(workload="150k + 120k Gaussians (60 % shared), 8 + 8 keyframes at 640x480, f = 500", iters=iters)
    for label, kw in (("l1", dict(loss="l1")), ("tracking_variant", dict(loss="tracking")),
                      ("l1_top2", dict(loss="l1", top_k=2))):
        res, rs = RB.run_plain(one, iters=iters, **kw)
        single[label] = dict(seconds=round(res["seconds"], 4),
                             mpix_per_s=round(one[0]["pixels"] * iters / res["seconds"] / 1e6, 2)
                             if label != "l1_top2" else None,
                             **errs(rs[0], one[0]))
    single["l1_top2"]["views"] = "2 + 2 of 8 + 8, ranked by rendered co-visibility"
    p0 = one[0]
    args = list(p0["args"])
    args[7] = (1.15 * args[7] + 0.03).contiguous()  # rgbQ under another exposure
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rx = REG.register_pair(*args, params=REG.default_params(iters, exposure=True))
    single["exposure_changed_q"] = dict(seconds=round(time.perf_counter() - t0, 4), **errs(rx, p0),
                                        q_exposure_median=[round(float(v), 4) for v in
                                                           np.median(rx["exposure"][8:], axis=0)])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rj = REG.register_pair(*p0["args"], params=REG.default_params(iters, joint=True))
    single["joint_transform"] = dict(seconds=round(time.perf_counter() - t0, 4), **errs(rj, p0))
    del one, args, rx, rj
    torch.cuda.empty_cache()

    log("registration: pair set")
    specs, ds = host["set"]
    pairs = [RB.upload_pair(d, sp) for d, sp in zip(ds, specs)]
    RB.run_batched(pairs[:2], iters=10)                          # warm-up (server thread, graph path)
    out_set = dict(workload=(f"{len(pairs)} pairs, Gaussians per submap log-uniform [20k, 300k], 4..12 keyframes "
                             "each at 640x480, own ground truth (<= 10 deg, <= 0.3 m); every keyframe sees only "
                             "Gaussians both submaps hold"),
                   iters=iters, pixels=int(sum(p["pixels"] for p in pairs)))
    for loss in ("l1", "tracking"):
        plain, rp = RB.run_plain(pairs, iters=iters, loss=loss)
        batched, rb = RB.run_batched(pairs, iters=iters, loss=loss)
        log(f"registration: pair set {loss}: plain {plain['pairs_per_s']:.2f}, batched {batched['pairs_per_s']:.2f} "
            f"pairs/s, success {plain['success']:.3f} / {batched['success']:.3f}")
        same = [bool(np.array_equal(a["T"], b["T"])) for a, b in zip(rp, rb)]
        out_set[loss if loss == "l1" else "tracking_variant"] = dict(
            plain=_rnd(plain), batched=_rnd(batched), speedup=round(batched["pairs_per_s"] / plain["pairs_per_s"], 3),
            identical_results=float(np.mean(same)))
    top2, _ = RB.run_plain(pairs, iters=iters, loss="l1", top_k=2)
    out_set["l1_top2_plain"] = _rnd(top2)
    del pairs, rp, rb
    torch.cuda.empty_cache()

    out = dict(single_pair=single, pair_set=out_set)
    if host.get("stress"):
        log("registration: stress set")
        specs, ds = host["stress"]
        pairs = [RB.upload_pair(d, sp) for d, sp in zip(ds, specs)]
        res, _ = RB.run_plain(pairs, iters=iters, loss="l1")
        out["stress_set_x_split"] = dict(workload="the pair set's sizes with the x-split layout (uneven pairs see "
                                                  "content one submap lacks)", plain=_rnd(res))
        del pairs
        torch.cuda.empty_cache()
    if host.get("stream"):
        log("registration: serving stream")
        specs, ds = host["stream"]
        built = [RB.upload_pair(d, sp) for d, sp in zip(ds, specs)]
        rate = host["stream_rate"]
        st = dict(workload=(f"{len(built)} requests, Poisson arrivals at {rate}/s, Gaussians per submap lognormal "
                            "(median 100k, sigma 0.8, clipped to [5k, 500k]), 4..12 keyframes each at 640x480 or "
                            "1200x680, budget 200 GB"), iters=iters)
        res, _ = RB.run_stream_plain(specs, built, iters=iters)
        st["plain_fifo"] = _rnd(res)
        for label, cap in (("server_no_cap", 0), ("server_cap_2_5mpx", 2_500_000)):
            res, _ = RB.run_stream(specs, built, iters=iters, max_active_pixels=cap)
            st[label] = _rnd(res)
        out["serving_stream"] = st
        del built
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent registration pairs and image-tile bands would shard across GPUs)", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    from paper_2408_10154_amd import regbench as RB
    from paper_2408_10154_amd import synth

    # ---- CPU phase: inputs and the oracle baseline, before any device call
    log("generating inputs")
    scene = synth.scene_room_volume(seed=1, n=args.gaussians)
    workers = args.cpu_workers or min(16, _host_cores())
    host = {}
    if not args.no_registration:
        single_spec = RB.single_pair_spec()
        host["single"] = (single_spec, RB.gen_pair(single_spec))
        specs = synth.pair_set(3, args.pairs)
        host["set"] = (specs, RB.gen_pairs(specs, workers))
        if not args.no_stress:
            specs = synth.pair_set(3, args.pairs, layout="x_split")
            host["stress"] = (specs, RB.gen_pairs(specs, workers))
        if args.stream_requests > 0:
            specs = synth.request_stream(100, args.stream_requests, args.stream_rate)
            host["stream"] = (specs, RB.gen_pairs(specs, workers))
            host["stream_rate"] = args.stream_rate
    log("inputs ready; timing the CPU oracle" if not args.no_cpu_baseline else "inputs ready")
    cpu = None if args.no_cpu_baseline else cpu_baseline(scene, args.cpu_tiles, workers)
    log("render loop")

    # ---- GPU phase
    import torch

    from paper_2408_10154_amd import lib as L
    from paper_2408_10154_amd.render import GaussianSet, RenderBatch, adam

    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    cam = scene["cam"]
    gs = GaussianSet.from_numpy(scene["gauss"])
    b = RenderBatch([(gs, cam, scene["w2c"])], auto_grow=True)

    # target: the scene rendered at the perturbed pose (fixed for the run)
    tpose = torch.as_tensor(scene["target_pose"][None], device="cuda")
    b.project(tpose)
    b.bin_sort()
    b.render_fwd()
    tgt_rgb, tgt_depth = b.rgb.clone(), b.depth.clone()
    b._alloc_bins(int(b.instances() * 1.5) + 4096)  # headroom: no host sync inside a step
    b.auto_grow = False

    pose = torch.as_tensor(synth.identity_pose()[None], device="cuda").contiguous()
    grads = gs.zeros_like()
    pose_grad = torch.zeros_like(pose)
    lr = dict(mean=1e-3, log_scale=5e-3, quat=1e-3, opacity_logit=5e-2, rgb=2.5e-3)
    # render loop: the Adam steps of the Gaussians and the pose fused into the projection backward
    mom = {name: (torch.zeros_like(getattr(gs, name)), torch.zeros_like(getattr(gs, name)), lr[name])
           for name in GaussianSet.FIELDS}
    pm, pv = torch.zeros_like(pose), torch.zeros_like(pose)
    pose_groups = [(pose[0, :4], pose_grad[0, :4], pm[0, :4], pv[0, :4], 2e-3),   # tracking rotation lr
                   (pose[0, 4:], pose_grad[0, 4:], pm[0, 4:], pv[0, 4:], 1e-2)]   # tracking translation lr
    # mapping loop (its regulariser adds to the log-scale gradient): gradient arrays and one ls_adam
    groups = []
    for name in GaussianSet.FIELDS:
        p = getattr(gs, name)
        groups.append((p, getattr(grads, name), torch.zeros_like(p), torch.zeros_like(p), lr[name]))
    groups += pose_groups
    loss = torch.zeros(1, device="cuda")
    g_rgb = torch.zeros_like(b.rgb)
    g_depth = torch.zeros_like(b.depth)
    g_scale = torch.zeros(1, device="cuda")
    stream = torch.cuda.current_stream()
    # 1 / |Omega| of the fixed targets, once (ls_loss_l1's grad_scale)
    b.loss_l1(tgt_rgb, tgt_depth, loss, g_rgb, g_depth, g_scale)
    kinds = ("project", "bin_sort", "fwd", "bwd", "loss", "bwd_project_adam")
    ev = {k: [] for k in kinds}
    step_no = [0]
    sp = L.C.c_void_p(stream.cuda_stream)

    def step(timed: str):
        """timed: "" (warm-up), "dominant" (events around the backward only:
        the timed steps) or "all" (events around every call: the per-kernel
        pass after the timed region)."""
        def run(kind, fn):
            if timed == "all" or (timed == "dominant" and kind == "bwd"):
                ev[kind].append(_events(stream, fn))
            else:
                fn()

        run("project", lambda: b.project(pose))
        run("bin_sort", lambda: L.ls_bin_sort(b.h, b.proj, b.bins, sp))
        run("fwd", lambda: b.render_fwd())
        run("bwd", lambda: b.render_bwd_tiles_l1(tgt_rgb, tgt_depth, g_scale))
        run("loss", lambda: b.loss_l1_tiles(loss))
        step_no[0] += 1
        run("bwd_project_adam", lambda: b.render_bwd_project_adam([mom], step_no[0], pose=pose, pose_grad=pose_grad,
                                                                  pose_adam=(pm, pv, 2e-3, 1e-2)))

    for _ in range(args.warmup):
        step("")
    torch.cuda.synchronize()
    loss0 = float(loss.item())
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step("dominant")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if int(b.count[1].item()) != 0:
        raise RuntimeError("tile-instance capacity overflowed during the timed steps")
    loss1 = float(loss.item())
    dt = (t1 - t0) / args.steps
    pixels = cam["width"] * cam["height"]
    value = pixels / dt / 1e6
    bwd_timed = sum(a.elapsed_time(c) for a, c in ev["bwd"]) / len(ev["bwd"])
    # per-kernel pass (outside the timed region): events around every call
    for k in kinds:
        ev[k] = []
    for _ in range(args.kernel_steps):
        step("all")
    torch.cuda.synchronize()
    kms = {k: sum(a.elapsed_time(c) for a, c in v) / len(v) for k, v in ev.items()}
    kms["bwd"] = bwd_timed
    evaluated, composited = b.render_stats()
    instances = b.instances()
    ntiles = ((cam["width"] + 15) // 16) * ((cam["height"] + 15) // 16)
    algo = algorithmic_bytes(args.gaussians, instances, pixels, ntiles)
    per_kernel = {k: {"ms": round(kms[k], 4), "algorithmic_mb": round(algo[k] / 1e6, 2),
                      "hbm_frac": round(algo[k] / (kms[k] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)} for k in kinds}
    path_bytes = sum(algo.values())
    ops = {"fwd": FWD_OPS_PER_FRAG * evaluated, "bwd": BWD_OPS_PER_FRAG * evaluated}
    dom = "bwd"
    achieved = ops[dom] / (kms[dom] * 1e-3) / 1e12
    build_count = {"fwd": FWD_EVAL * evaluated + FWD_COMP * composited,
                   "bwd": BWD_EVAL * evaluated + BWD_COMP * composited}
    for k in ("fwd", "bwd"):
        per_kernel[k]["alu_t_ops"] = round(ops[k] / (kms[k] * 1e-3) / 1e12, 3)
        per_kernel[k]["alu_frac"] = round(ops[k] / (kms[k] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)
        per_kernel[k]["alu_frac_unpacked_issue"] = round(ops[k] / (kms[k] * 1e-3) / 1e12 / PEAK_LANE_OPS_T, 4)
        per_kernel[k]["valu_busy_profiled"] = measured_valu_busy("composite_" + ("fwd_band" if k == "fwd" else k))

    log(f"render loop: {dt * 1e3:.3f} ms per step")
    mapping = None
    if args.mapping_steps > 0:
        # the same loop with the submap-update loss: L1 + SSIM colour term,
        # depth term, isotropic scale regulariser (all weights 1, SSIM 0.2)
        from paper_2408_10154_amd.render import loss_isotropic

        reg_loss = torch.zeros(1, device="cuda")
        work = torch.empty(L.LS_ISOTROPIC_WORK_FLOATS, device="cuda")
        mev = []

        def map_step(timed: bool):
            b.project(pose)
            L.ls_bin_sort(b.h, b.proj, b.bins, sp)
            b.render_fwd()
            fn = lambda: b.loss_mapping(tgt_rgb, tgt_depth, 0.2, 1.0, 1.0, loss, g_rgb, g_depth, g_scale)  # noqa
            if timed:
                mev.append(_events(stream, fn))
            else:
                fn()
            b.render_bwd_tiles(up_rgb=g_rgb, up_depth=g_depth, scale=g_scale)
            b.render_bwd_project(grads=[grads], pose=pose, pose_grad=pose_grad)
            loss_isotropic(gs.log_scale, 1.0, loss=reg_loss, grad=grads.log_scale, work=work)
            step_no[0] += 1
            adam(groups, step_no[0])

        for _ in range(3):
            map_step(False)
        torch.cuda.synchronize()
        m0 = time.perf_counter()
        for _ in range(args.mapping_steps):
            map_step(True)
        torch.cuda.synchronize()
        mdt = (time.perf_counter() - m0) / args.mapping_steps
        if int(b.count[1].item()) != 0:
            raise RuntimeError("tile-instance capacity overflowed during the mapping steps")
        lms = sum(a.elapsed_time(c) for a, c in mev) / len(mev)
        mapping = {
            "loss": "lambda_color (0.8 L1 + 0.2 (1 - SSIM)) + lambda_depth L1 + lambda_reg isotropic, weights 1",
            "ms_per_step": round(mdt * 1e3, 4), "mpix_s": round(pixels / mdt / 1e6, 3),
            "loss_ms": round(lms, 4),
            "loss_roofline": {"hbm_frac": round(MAP_BYTES_PX * pixels / (lms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                              "alu_frac": round(MAP_FLOPS_PX * pixels / (lms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS, 4)},
            "last_loss": round(float(loss.item()) + float(reg_loss.item()), 5),
        }

    if args.calib_copy_mb > 0:
        n = args.calib_copy_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    del b, gs, grads, groups, mom
    torch.cuda.empty_cache()
    log("pruning, map adjustment, overlap ratio")
    prune = None if args.no_prune else prune_timing()
    torch.cuda.empty_cache()
    adjust = map_adjust(args.adjust_submaps) if args.adjust_submaps > 0 else None
    torch.cuda.empty_cache()
    ovl = None if args.no_overlap else overlap()
    reg = None
    if not args.no_registration:
        torch.cuda.empty_cache()
        log("registration")
        reg = registration(host, args.reg_iters)

    out = {
        "metric": "fwd+bwd Mpixels/s; batched pair registrations/s + p50/p99 vs plain",
        "value": round(value, 3),
        "unit": "Mpixels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "tracking/mapping render loop: 200k Gaussians (6x3x4 m box), 1200x680 f=600, "
                               "fwd+bwd+Adam on Gaussians and camera pose",
                   "gaussians": args.gaussians, "width": cam["width"], "height": cam["height"],
                   "instances": instances, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "composite_bwd", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                     "traffic": measured_traffic("composite_bwd"),
                     "ops_per_fragment": BWD_OPS_PER_FRAG, "fragments_evaluated": evaluated,
                     "frac_unpacked_issue": round(achieved / PEAK_LANE_OPS_T, 4),
                     "valu_busy_profiled": measured_valu_busy("composite_bwd"),
                     "build_count": {"ops": build_count[dom], "per_eval": BWD_EVAL, "per_composited": BWD_COMP,
                                     "frac": round(build_count[dom] / (kms[dom] * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                                                   4)}},
        "kernels": per_kernel,
        "whole_path": {"algorithmic_mb": round(path_bytes / 1e6, 1),
                       "gbs": round(path_bytes / dt / 1e9, 1),
                       "hbm_frac": round(path_bytes / dt / 1e9 / PEAK_HBM_GBS, 4)},
        "fragments": {"evaluated": evaluated, "composited": composited},
        "loss": {"first_timed": round(loss0, 5), "last": round(loss1, 5)},
        "mapping": mapping,
        "prune": prune,
        "map_adjust": adjust,
        "overlap": ovl,
        "registration": reg,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
