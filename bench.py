"""Benchmark of the coding loop on one MI355X.

Workload (default): the Sentinel-2-like cloud-gapped cube, 500 frames x
128 x 128 x 6 bands float32 with ~10% NaN, converted to 12 bits and coded at
QP {17, 22, 27, 32, 37} x block {8, 16, 32} (15 runs), search range 16,
closed GOPs of 16.  One step = encode + decode + PSNR/bpppb of all 15 runs.
The cube is generated on the GPU and resident in HBM before timing starts.

Two forms are timed back to back on the same inputs:
  plain    one cube-run at a time (xv_encode_cube / xv_decode_cube)
  batched  all 15 runs per call (xv_encode_batch / xv_decode_batch: one launch
           per frame step and block-size class)
Both produce bit-identical outputs (checked), hence identical PSNR and bpppb.

Prints ONE JSON line.  `value` is the batched throughput in Mpx*band/s of
encode + decode (px*band = T*H*W*bands per run, summed over runs).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mpx·band/s encode+decode at fixed PSNR, batched/served vs plain; p50/p99 ms"

# MI355X peaks used for the roofline fractions
HBM_PEAK_GBS = 8000.0
# v_sad_u16: 2 SAD terms per lane-op; 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz
SAD_PEAK_TTERMS = 256 * 64 * 2.4e9 * 2 / 1e12

# Measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a 1 GiB
# copy), with the sha256 of the kernel sources they were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "s2cloud_sweep_hbm_traffic.json")


def _measured_traffic():
    """Per-kernel HBM bytes per launch from the committed counter summary, or
    None when any listed kernel source has changed since it was taken."""
    import hashlib
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        for rel, digest in t["sources_sha256"].items():
            with open(os.path.join(ROOT, rel), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != digest:
                    return None
    except (OSError, KeyError, ValueError):
        return None
    out = {}
    for k, v in t["per_launch_bytes"].items():
        name = k.split("<")[0]
        # the two motion-search window layouts are one kernel class
        out.setdefault("me" if name in ("me_kernel", "me_rp_kernel") else name, []).append(float(v))
    # each kernel launches equally often per block size in the sweep step
    return {k: sum(v) / len(v) for k, v in out.items()}


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def cpu_baseline(cube_host, wl, seconds_hint=""):
    """The oracle as it stands, on the host cores: encode + decode + metrics of
    all 15 runs over the full cube (the same work as one GPU step)."""
    from oracle import oracle as O
    O.lib()
    runs = [(qp, N) for N in wl.blocks for qp in wl.qps]
    t0 = time.perf_counter()
    for qp, N in runs:
        p = O.CodingParams(bit_depth=wl.bit_depth, qp=qp, block=N, search_range=wl.search_range,
                           gop=wl.gop, pad_mode=wl.pad_mode, fill_mode=wl.fill_mode)
        enc = O.encode_cube(cube_host, p)
        rec = O.decode_cube(p, cube_host.shape, enc["levels"], enc["mvs"])
        O.denormalize_cube(rec, cube_host.shape, N, wl.bit_depth, enc["mn"], enc["mx"],
                           O.F32 if cube_host.dtype.name == "float32" else O.U16)
        O.metrics(cube_host, enc, p)
    dt = time.perf_counter() - t0
    pxb = wl.px_band * len(runs)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": pxb / dt / 1e6, "unit": "Mpx·band/s", "cores": cores, "kind": "oracle",
            "sample": f"one full step: all {len(runs)} runs on the {wl.T}x{wl.H}x{wl.W}x"
                      f"{wl.bands} cube, encode+decode+metrics, {dt:.1f} s wall"}


def quality_bench(xv, torch, cube, params, runs, steps):
    """SSIM of the coded planes (xv_ssim) and spectral angle of the decoded
    cube (xv_spectral_angle) for every run of the sweep: the values, and the
    kernel time per step of all runs from HIP events."""
    encs = xv.encode_batch([cube] * len(params), params)
    outs = [torch.empty_like(cube) for _ in params]
    xv.decode_batch(encs, outs)
    torch.cuda.synchronize()
    vals = [(xv.ssim(e), xv.spectral_angle(cube, o)) for e, o in zip(encs, outs)]  # warm-up
    xv.profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        vals = [(xv.ssim(e), xv.spectral_angle(cube, o)) for e, o in zip(encs, outs)]
    dt = time.perf_counter() - t0
    prof = xv.profile_read()["quality"]
    xv.profile_enable(False)
    for e in encs:
        e.free()
    pxb = cube.numel() * len(params)
    out = {"ssim_mean_per_run": [round(sum(s) / len(s), 6) for s, _ in vals],
           "spectral_angle_rad_per_run": [round(a, 8) for _, (a, _) in vals],
           "runs": [f"QP{qp}/N{N}" for qp, N in runs],
           "ms_per_step": round(dt / steps * 1e3, 3),
           "Mpx_band_s": round(pxb * steps / dt / 1e6, 1)}
    if prof["launches"]:
        ms = prof["ms"] / steps
        out["kernel_ms_per_step"] = round(ms, 3)
        out["kernel_input_GBs"] = round(prof["work"] / steps / (ms * 1e-3) / 1e9, 1)
    return out


def bits_bench(xv, torch, cube, params, pxb_step, steps):
    """Serialise the sweep's 15 encoded runs (xv_pack) and parse them back
    (xv_unpack), timed per call on the host (each call synchronises once) and
    per kernel with HIP events; checks that the parsed levels equal the
    encoded ones."""
    import numpy as np
    encs = xv.encode_batch([cube] * len(params), params)
    torch.cuda.synchronize()
    packed = [xv.pack(e) for e in encs]  # warm-up
    for u in [xv.unpack(p.tensor()) for p in packed]:
        u.free()
    for p in packed:
        p.free()
    xv.profile_enable(True)
    t_pack = t_unpack = 0.0
    payload = 0
    for _ in range(steps):
        t0 = time.perf_counter()
        packed = [xv.pack(e) for e in encs]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        unpacked = [xv.unpack(p.tensor()) for p in packed]
        t2 = time.perf_counter()
        t_pack += t1 - t0
        t_unpack += t2 - t1
        payload = sum(p.view()["payload_bits"] for p in packed)
        for u in unpacked:
            u.free()
        for p in packed:
            p.free()
    prof = xv.profile_read()
    xv.profile_enable(False)
    same = all(np.array_equal(a.export()["levels"].cpu().numpy(),
                              b.export()["levels"].cpu().numpy())
               for a, b in [(encs[0], xv.unpack(xv.pack(encs[0]).tensor()))])
    wr, pa = prof["bits_write"], prof["bits_parse"]
    coded = sum(e.export()["levels"].numel() for e in encs)  # coded samples (levels read)
    out = {"runs": len(encs), "payload_MB_per_step": round(payload / 8 / 1e6, 3),
           "pack_ms_per_step": round(t_pack / steps * 1e3, 3),
           "unpack_ms_per_step": round(t_unpack / steps * 1e3, 3),
           "pack_Mpx_band_s": round(pxb_step * steps / t_pack / 1e6, 1),
           "unpack_Mpx_band_s": round(pxb_step * steps / t_unpack / 1e6, 1),
           "parsed_equals_encoded": bool(same)}
    if wr["launches"]:
        ms = wr["ms"] / steps
        out["write_kernel_ms_per_step"] = round(ms, 3)
        out["write_kernel_levels_GBs"] = round(coded * 2 / (ms * 1e-3) / 1e9, 1)
    if pa["launches"]:
        ms = pa["ms"] / steps
        out["parse_kernel_ms_per_step"] = round(ms, 3)
        out["parse_kernel_payload_GBs"] = round(payload / 8 / (ms * 1e-3) / 1e9, 2)
    for e in encs:
        e.free()
    return out


def serve_bench(xv, synth, torch, n=160, seed=4, loads=(0.5, 0.9, 1.2, 2.0)):
    """Serving mix: requests with the mix's recipe (encode or decode with
    p = 1/2, log-uniform sizes, bands {3, 4, 6}, QP 17..37, N = 16, R = 16)
    at sizes capped to T <= 96 and side <= 256 so the run takes seconds.
    Offered loads are fractions of the plain path's measured capacity; the
    plain baseline serves the same arrivals one request at a time."""
    import numpy as np
    dev = torch.device("cuda:0")
    reqs = synth.request_trace(n, rate_per_s=1.0, seed=seed, t_range=(16, 96), s_range=(64, 256))
    items = []
    for r in reqs:
        cube = synth.tiny_cube(seed=r.seed, T=r.T, H=r.S, W=r.S, bands=r.bands, device=dev)
        prm = xv.Params(bit_depth=10, qp=r.qp, block=16, search_range=16, gop=16,
                        flags=xv.FLAG_DROP_WORK)
        pxb = r.T * r.S * r.S * r.bands
        if r.op == "decode":
            items.append(("decode", xv.encode_cube(cube, prm), torch.empty_like(cube), pxb))
        else:
            items.append(("encode", cube, prm, pxb))
    torch.cuda.synchronize()
    total_pxb = sum(it[3] for it in items)

    def run_plain_one(it):
        if it[0] == "encode":
            e = xv.encode_cube(it[1], it[2])
            torch.cuda.synchronize()
            e.free()
        else:
            xv.decode_cube(it[1], it[2])
            torch.cuda.synchronize()

    for it in items[:8]:
        run_plain_one(it)  # warm-up
    t0 = time.perf_counter()
    for it in items:
        run_plain_one(it)
    cap_s = time.perf_counter() - t0
    mean_service = cap_s / len(items)
    out = {"requests": len(items), "px_band_total": total_pxb,
           "trace": "Poisson arrivals; encode/decode p=1/2; T log-uniform 16..96, side "
                    "log-uniform 64..256 (multiple of 32), bands {3,4,6}, QP 17..37, N=16, R=16",
           "plain_capacity_mpxb_s": round(total_pxb / cap_s / 1e6, 3), "loads": []}
    rng = np.random.default_rng(seed + 1)
    gaps_unit = rng.exponential(1.0, len(items))
    for rho in loads:
        gaps = gaps_unit * mean_service / rho
        arrive = np.cumsum(gaps) - gaps[0]
        # plain FIFO at the same arrivals
        lat = []
        base = time.perf_counter()
        for it, a in zip(items, arrive):
            now = time.perf_counter() - base
            if now < a:
                time.sleep(a - now)
            run_plain_one(it)
            lat.append((time.perf_counter() - base - a) * 1e3)
        plain_span = time.perf_counter() - base
        # served
        sv = xv.Server(max_slots=64)
        tickets = []
        base = time.perf_counter()
        for it, a in zip(items, arrive):
            now = time.perf_counter() - base
            if now < a:
                time.sleep(a - now)
            if it[0] == "encode":
                tickets.append(sv.submit_encode(it[1], it[2]))
            else:
                tickets.append(sv.submit_decode(it[1], it[2]))
        res = [sv.wait(t) for t in tickets]
        served_span = time.perf_counter() - base
        st = sv.stats()
        sv.close()
        if any(r["status"] != xv.OK for r in res):
            raise SystemExit("served request failed")
        slat = [r["done_ms"] - r["submit_ms"] for r in res]
        out["loads"].append({
            "rho": rho, "offered_req_per_s": round(1.0 / (mean_service / rho), 2),
            "served": {"value": round(total_pxb / served_span / 1e6, 3),
                       "p50_ms": round(_percentile(slat, 0.5), 3),
                       "p99_ms": round(_percentile(slat, 0.99), 3),
                       "peak_active": st["peak_active"], "iterations": st["iterations"]},
            "plain": {"value": round(total_pxb / plain_span / 1e6, 3),
                      "p50_ms": round(_percentile(lat, 0.5), 3),
                      "p99_ms": round(_percentile(lat, 0.99), 3)}})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mode", choices=["both", "batched", "plain"], default="both")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-mix section")
    ap.add_argument("--no-bits", action="store_true", help="skip the bitstream section")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the SSIM / spectral-angle section")
    ap.add_argument("--counters", action="store_true",
                    help="workload for hardware-counter runs only: one 1 GiB device copy (the "
                         "calibration of FETCH_SIZE / WRITE_SIZE), then one batched sweep step "
                         "with the geometry file's geometry; prints no result line")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the motion-search geometry tuner (model defaults)")
    ap.add_argument("--geometry-file", default=None,
                    help="load tuned motion-search geometries from this JSON file if it "
                         "exists, else tune and write them there")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(one GPU's share of the work is what it measures)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2506_19656_amd import synth
    from paper_2506_19656_amd import xv

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.WORKLOADS["s2cloud"]
    print(f"[bench] generating {wl.name} cube on {dev}", file=sys.stderr, flush=True)
    cube = synth.s2cloud_cube(device=dev)
    torch.cuda.synchronize()
    runs = [(qp, N) for N in wl.blocks for qp in wl.qps]
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=N, search_range=wl.search_range,
                        gop=wl.gop, pad_mode=wl.pad_mode, fill_mode=wl.fill_mode)
              for qp, N in runs]
    outs = [torch.empty_like(cube) for _ in runs]
    pxb_step = wl.px_band * len(runs)

    if args.counters:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # launch-geometry tuning (outside the timed region; outputs never depend on it)
    tuning = {}
    cached = None
    if args.geometry_file and os.path.exists(args.geometry_file):
        with open(args.geometry_file) as f:
            cached = json.load(f)
    for N in wl.blocks:
        if cached is not None and f"N{N}" in cached:
            g = cached[f"N{N}"]
            xv.set_me_geometry(N, wl.search_range, g["blocks_per_wg"], g["cands_per_lane"],
                               g["threads"], g.get("rows_per_lane", 0), g.get("layout", 1))
            tuning[f"N{N}"] = dict(g, tuned=True, from_file=True)
        elif not args.no_tune:
            print(f"[bench] tuning motion search N={N}", file=sys.stderr, flush=True)
            # tuned on the first P step of exactly the batch the timed steps launch
            pn = [p for p in params if p.block == N]
            t = xv.autotune_me_batch([cube] * len(pn), pn)
            tuning[f"N{N}"] = dict(t, tuned=True)
        else:
            tuning[f"N{N}"] = dict(xv.get_me_geometry(N, wl.search_range, -(-wl.W // N)),
                                   tuned=False)
    if args.geometry_file and cached is None:
        with open(args.geometry_file, "w") as f:
            json.dump(tuning, f)

    if args.counters:
        if cached is None:
            raise SystemExit("--counters needs an existing --geometry-file")
        encs = xv.encode_batch([cube] * len(params), params)
        xv.decode_batch(encs, outs)
        torch.cuda.synchronize()
        for e in encs:
            e.free()
        print("[bench] counter workload done", file=sys.stderr, flush=True)
        return

    def step_plain(lat=None):
        ms = []
        for p, out in zip(params, outs):
            t0 = time.perf_counter()
            enc = xv.encode_cube(cube, p)
            xv.decode_cube(enc, out)
            ms.append(xv.psnr_bpppb(cube, enc))  # synchronises
            enc.free()
            if lat is not None:
                lat.append((time.perf_counter() - t0) * 1e3)
        return ms

    def step_batched(lat=None):
        t0 = time.perf_counter()
        encs = xv.encode_batch([cube] * len(params), params)
        xv.decode_batch(encs, outs)
        ms = xv.psnr_bpppb_batch([cube] * len(encs), encs)
        for e in encs:
            e.free()
        if lat is not None:
            lat.append((time.perf_counter() - t0) * 1e3)
        return ms

    def timed(fn, profile):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        lat = []
        if profile:
            # only the dominant kernel (motion search) is event-timed inside
            # the timed region: every event pair costs queue time
            xv.profile_select([xv.K_ME])
            xv.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ms = fn(lat)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = xv.profile_read() if profile else None
        if profile:
            xv.profile_enable(False)
        return dt, lat, ms, prof

    res = {}
    prof_all = None
    if args.mode in ("both", "plain"):
        print("[bench] plain path", file=sys.stderr, flush=True)
        dt, lat, ms_plain, _ = timed(step_plain, profile=False)
        res["plain"] = dict(value=pxb_step * args.steps / dt / 1e6, ms_per_step=dt / args.steps * 1e3,
                            p50_ms=_percentile(lat, 0.5), p99_ms=_percentile(lat, 0.99),
                            latency_unit="one run: encode+decode+metrics")
    if args.mode in ("both", "batched"):
        print("[bench] batched path", file=sys.stderr, flush=True)
        dt, lat, ms_batch, prof = timed(step_batched, profile=True)
        # every kernel class, timed on one more step outside the timed region
        xv.profile_select(None)
        xv.profile_enable(True)
        step_batched()
        prof_all = xv.profile_read()
        xv.profile_enable(False)
        res["batched"] = dict(value=pxb_step * args.steps / dt / 1e6, ms_per_step=dt / args.steps * 1e3,
                              p50_ms=_percentile(lat, 0.5), p99_ms=_percentile(lat, 0.99),
                              latency_unit="one step: all 15 runs")
    if "plain" in res and "batched" in res:
        same = all(a["psnr"] == b["psnr"] and a["bpppb"] == b["bpppb"]
                   for a, b in zip(ms_plain, ms_batch))
        if not same:
            raise SystemExit("batched and plain paths disagree")
    ms = ms_batch if "batched" in res else ms_plain
    main_form = "batched" if "batched" in res else "plain"

    line = {
        "metric": METRIC,
        "value": round(res[main_form]["value"], 3),
        "unit": "Mpx·band/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res[main_form]["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.T}x{wl.H}x{wl.W}x{wl.bands} f32 cube with ~10% "
                               f"NaN cloud gaps, B={wl.bit_depth}, QP{list(wl.qps)} x "
                               f"N{list(wl.blocks)} (15 runs), R={wl.search_range}, "
                               f"GOP {wl.gop}", "form": main_form,
                   "px_band_per_step": pxb_step},
        "me_geometry": tuning,
        "p50_ms": round(res[main_form]["p50_ms"], 3),
        "p99_ms": round(res[main_form]["p99_ms"], 3),
        "forms": {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                  for k, v in res.items()},
        "quality": {"psnr_db_mean_per_run": [round(float(np.mean(m["psnr"])), 4) for m in ms],
                    "psnr_phys_db_mean_per_run": [round(float(np.mean(m["psnr_phys"])), 4)
                                                  for m in ms],
                    "bpppb_per_run": [round(m["bpppb"], 5) for m in ms],
                    "runs": [f"QP{qp}/N{N}" for qp, N in runs]},
    }
    if "plain" in res and "batched" in res:
        line["speedup_batched_vs_plain"] = round(res["batched"]["value"] / res["plain"]["value"], 3)
    if prof is not None:
        traffic = _measured_traffic() or {}
        me = prof["me"]                  # timed region (motion search only)
        enc = prof_all["encode"]         # one extra step, every class timed
        dec = prof_all["decode"]
        me_avg_ms = me["ms"] / max(1, me["launches"])
        me_terms = me["work"] / max(1, me["launches"])
        achieved = me_terms / (me_avg_ms * 1e-3) / 1e12
        line["roofline"] = {"kernel": "motion search (me_rp_kernel / me_kernel)", "bound": "alu",
                            "achieved": round(achieved, 3), "peak": round(SAD_PEAK_TTERMS, 2),
                            "unit": "T SAD-terms/s", "frac": round(achieved / SAD_PEAK_TTERMS, 4),
                            "traffic": round(traffic["me"]) if "me" in traffic else None,
                            "traffic_unit": "bytes per launch",
                            "avg_launch_ms": round(me_avg_ms, 4),
                            "launches": me["launches"], "terms_per_launch": me_terms,
                            "timed": "HIP events around every motion-search launch of the timed "
                                     "steps (no other class timed there)"}
        for name, d in (("encode_kernel (fused transform coding)", enc),
                        ("decode_kernel", dec)):
            if d["launches"]:
                avg = d["ms"] / d["launches"]
                gbs = d["work"] / d["launches"] / (avg * 1e-3) / 1e9
                kname = name.split(" ")[0]
                key = "roofline_encode" if name.startswith("encode") else "roofline_decode"
                line[key] = {"kernel": name, "bound": "hbm", "achieved": round(gbs, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "traffic": (round(traffic[kname]) if kname in traffic else None),
                             "traffic_unit": "bytes per launch",
                             "algorithmic_bytes_per_launch": round(d["work"] / d["launches"]),
                             "avg_launch_ms": round(avg, 4), "launches": d["launches"],
                             "timed": "one batched step after the timed region, every class timed"}
        line["kernel_ms_per_step"] = {k: round(v["ms"], 3) for k, v in prof_all.items()
                                      if v["launches"]}
    if not args.no_quality:
        print("[bench] quality metrics", file=sys.stderr, flush=True)
        line["quality_metrics"] = quality_bench(xv, torch, cube, params, runs, args.steps)
    if not args.no_bits:
        print("[bench] bitstream", file=sys.stderr, flush=True)
        line["bitstream"] = bits_bench(xv, torch, cube, params, pxb_step, args.steps)
    if not args.no_serve:
        print("[bench] serving mix", file=sys.stderr, flush=True)
        line["served"] = serve_bench(xv, synth, torch)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(cube.cpu().numpy(), wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
