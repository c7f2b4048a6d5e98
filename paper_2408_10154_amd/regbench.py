"""Registration throughput and latency: the plain per-pair path
(ls_register_pair, one pair at a time) against the serving loop (all pairs
admitted together or as they arrive, continuously batched)."""

from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import register as REG
from . import synth
from .render import GaussianSet


def gen_pair(spec: dict, width=640, height=480, f=500.0) -> dict:
    """Host arrays of a pair spec of synth.pair_set / synth.request_stream
    (NumPy only, no device work), built by synth.registration_pair."""
    return synth.registration_pair(spec["seed"], spec["n_p"], spec["n_q"], views_p=spec["views_p"],
                                   views_q=spec["views_q"], width=spec.get("width", width),
                                   height=spec.get("height", height), f=spec.get("f", f),
                                   layout=spec.get("layout", "views"))


def gen_pairs(specs, workers: int = 1) -> list:
    """gen_pair over many specs, in `workers` forked processes when > 1 (call
    it before the process touches the GPU)."""
    if workers <= 1 or len(specs) <= 1:
        return [gen_pair(sp) for sp in specs]
    import multiprocessing as mp

    with mp.get_context("fork").Pool(min(workers, len(specs))) as pool:
        return pool.map(gen_pair, specs)


def upload_pair(d: dict, spec: dict) -> dict:
    """Device-resident pair (Gaussians and keyframe targets rendered by the
    rasterizer) from gen_pair's host arrays."""
    P, Q = GaussianSet.from_numpy(d["P"]), GaussianSet.from_numpy(d["Q"])
    rgbP, depP = REG.keyframe_targets(P, d["cam"], d["kf_p"])
    rgbQ, depQ = REG.keyframe_targets(Q, d["cam"], d["kf_q"])
    return dict(T_gt=d["T_gt"], args=(P, Q, d["cam"], d["kf_p"], d["kf_q"], rgbP, depP, rgbQ, depQ),
                pixels=(spec["views_p"] + spec["views_q"]) * d["cam"]["width"] * d["cam"]["height"],
                n_p=d["P"]["mean"].shape[1], n_q=d["Q"]["mean"].shape[1], shared=d["shared"])


def build_pair(spec: dict, width=640, height=480, f=500.0):
    """Device-resident pair (Gaussians and keyframe targets) for a spec of
    synth.pair_set / synth.request_stream, built by synth.registration_pair."""
    return upload_pair(gen_pair(spec, width, height, f), spec)


def _errors(results, pairs):
    rot = [REG.rotation_error_deg(r["T"], p["T_gt"]) for r, p in zip(results, pairs)]
    tr = [REG.translation_error_cm(r["T"], p["T_gt"]) for r, p in zip(results, pairs)]
    ok = [a < 0.5 and b < 1.0 for a, b in zip(rot, tr)]
    return dict(success=float(np.mean(ok)), rot_deg_median=float(np.median(rot)), trans_cm_median=float(np.median(tr)),
                rot_deg_max=float(np.max(rot)), trans_cm_max=float(np.max(tr)))


def _pct(x, q):
    return float(np.percentile(np.asarray(x, np.float64), q))


def run_plain(pairs, iters=200, loss="l1", exit_rel_tol=0.0, exit_patience=0, top_k=0, exit_mode="loss"):
    """One pair at a time through ls_register_pair; latency of pair k counts
    from the start of the run (all requests present at t = 0)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, done = [], []
    for p in pairs:
        results.append(REG.register_pair(*p["args"], params=REG.default_params(
            iters, loss=loss, exit_rel_tol=exit_rel_tol, exit_patience=exit_patience, top_k=top_k,
            exit_mode=exit_mode)))
        done.append(time.perf_counter() - t0)
    total = time.perf_counter() - t0
    return dict(seconds=total, pairs_per_s=len(pairs) / total, p50_s=_pct(done, 50), p99_s=_pct(done, 99),
                mean_iters=float(np.mean([r["iters"] for r in results])), **_errors(results, pairs)), results


def run_batched(pairs, iters=200, loss="l1", chunk_iters=16, use_graphs=True, max_slots=64, budget=200 << 30,
                exit_rel_tol=0.0, exit_patience=0, exit_mode="loss"):
    """Every pair submitted at t = 0 to one server."""
    from .serve import Server

    with Server(budget_bytes=budget, max_slots=max_slots, chunk_iters=chunk_iters, use_graphs=use_graphs) as sv:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prm = REG.default_params(iters, loss=loss, exit_rel_tol=exit_rel_tol, exit_patience=exit_patience,
                                 exit_mode=exit_mode)
        tickets = [sv.submit(*p["args"], params=prm) for p in pairs]
        results = [sv.wait(t) for t in tickets]
        total = time.perf_counter() - t0
        st = sv.stats()
    lat = [r["times"]["total"] for r in results]
    return dict(seconds=total, pairs_per_s=len(pairs) / total, p50_s=_pct(lat, 50), p99_s=_pct(lat, 99),
                epochs=st["epochs"], graph_replays=st["graph_replays"],
                mean_iters=float(np.mean([r["iters"] for r in results])), **_errors(results, pairs)), results


def run_stream(stream, built, iters=200, loss="l1", chunk_iters=16, budget=200 << 30, max_slots=64,
               max_active_pixels=0):
    """Requests submitted at their arrival times (a host thread paces them)."""
    from .serve import Server

    with Server(budget_bytes=budget, max_slots=max_slots, chunk_iters=chunk_iters,
                max_active_pixels=max_active_pixels) as sv:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = []
        for spec, p in zip(stream, built):
            delay = spec["arrival"] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets.append(sv.submit(*p["args"], params=REG.default_params(iters, loss=loss)))
        results = [sv.wait(t) for t in tickets]
        total = time.perf_counter() - t0
        st = sv.stats()
    lat = [r["times"]["total"] for r in results]
    return dict(seconds=total, pairs_per_s=len(built) / total, p50_s=_pct(lat, 50), p99_s=_pct(lat, 99),
                max_active_bytes=st["peak_bytes"], peak_active=st["peak_active"], epochs=st["epochs"],
                **_errors(results, built)), results


def run_stream_plain(stream, built, iters=200, loss="l1"):
    """The plain path under the same arrivals: a FIFO queue served one pair at
    a time by ls_register_pair; latency counts from each request's arrival."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results, lat = [], []
    for spec, p in zip(stream, built):
        delay = spec["arrival"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        results.append(REG.register_pair(*p["args"], params=REG.default_params(iters, loss=loss)))
        lat.append(time.perf_counter() - t0 - spec["arrival"])
    total = time.perf_counter() - t0
    return dict(seconds=total, pairs_per_s=len(built) / total, p50_s=_pct(lat, 50), p99_s=_pct(lat, 99),
                **_errors(results, built)), results


def single_pair_spec(seed=2):
    """The single-pair workload: 150k + 120k Gaussians (60 % shared), 8 + 8
    keyframes at 640x480, f = 500."""
    return dict(seed=seed, n_p=150_000, n_q=120_000, views_p=8, views_q=8, layout="views")


def _exit_rule(text):
    """'off' -> ("loss", 0, 0); 'loss:TOL:PATIENCE' / 'step:RATIO:PATIENCE'."""
    if text == "off":
        return "loss", 0.0, 0
    kind, tol, patience = text.split(":")
    if kind not in ("loss", "step"):
        raise ValueError(f"unknown early exit rule {text!r}")
    return kind, float(tol), int(patience)


def main(argv=None):
    """Command-line runs of the registration workloads (one JSON line each),
    e.g. under a kernel-trace profiler:
      python -m paper_2408_10154_amd.regbench --workload single --iters 50
      python -m paper_2408_10154_amd.regbench --workload set --pairs 8 --mode both
      python -m paper_2408_10154_amd.regbench --workload stream --requests 40 --rate 2 --mode both"""
    import argparse
    import json

    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", choices=["single", "set", "stream"], default="single")
    ap.add_argument("--requests", type=int, default=40, help="requests of the stream (seed 100)")
    ap.add_argument("--rate", type=float, default=2.0, help="stream arrivals per second")
    ap.add_argument("--max-active-pixels", type=int, nargs="+", default=[0],
                    help="server admission caps to try (0: none)")
    ap.add_argument("--pairs", type=int, default=8, help="pairs of the pair set (seed 3)")
    ap.add_argument("--iters", type=int, default=200)
    ap.add_argument("--mode", choices=["plain", "batched", "both"], default="plain")
    ap.add_argument("--loss", choices=["tracking", "l1"], default="l1")
    ap.add_argument("--layout", choices=["views", "x_split"], default="views",
                    help="submap split of the synthetic pairs (see synth.registration_pair)")
    ap.add_argument("--exit", nargs="+", default=["off"],
                    help="per-view early exit rules to run in turn: 'off', 'loss:REL_TOL:PATIENCE' or "
                         "'step:RATIO:PATIENCE' (set and single workloads)")
    a = ap.parse_args(argv)
    torch.cuda.set_device(0)
    if a.workload == "single":
        specs = [single_pair_spec()]
    elif a.workload == "set":
        specs = synth.pair_set(3, a.pairs)
    else:
        specs = synth.request_stream(100, a.requests, a.rate)
    for sp in specs:
        sp["layout"] = a.layout
    pairs = [build_pair(sp) for sp in specs]
    print(json.dumps(dict(event="built", pairs=len(pairs))), flush=True)
    for mode in (["plain", "batched"] if a.mode == "both" else [a.mode]):
        caps = a.max_active_pixels if (mode == "batched" and a.workload == "stream") else [0]
        for cap in caps:
            if a.workload == "stream":
                if mode == "plain":
                    res, _ = run_stream_plain(specs, pairs, iters=a.iters, loss=a.loss)
                else:
                    res, _ = run_stream(specs, pairs, iters=a.iters, loss=a.loss, max_active_pixels=cap)
                extra = dict(rate=a.rate, requests=a.requests)
                if mode == "batched":
                    extra["max_active_pixels"] = cap
                print(json.dumps(dict(workload=a.workload, mode=mode, iters=a.iters, **extra,
                                      **{k: round(v, 4) if isinstance(v, float) else v for k, v in res.items()})),
                      flush=True)
                continue
            run = run_plain if mode == "plain" else run_batched
            for rule in a.exit:
                kind, tol, patience = _exit_rule(rule)
                res, _ = run(pairs, iters=a.iters, loss=a.loss, exit_rel_tol=tol, exit_patience=patience,
                             exit_mode=kind)
                print(json.dumps(dict(workload=a.workload, mode=mode, iters=a.iters, exit=rule,
                                      **{k: round(v, 4) if isinstance(v, float) else v for k, v in res.items()})),
                      flush=True)


if __name__ == "__main__":
    main()
