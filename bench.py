"""Benchmark of the coding loop on one MI355X.

Headline workload: the Planet-like cube (stand-in for DynamicEarthNet),
730 daily frames x 1024 x 1024 x 4 bands u16 (RGB + NIR; the second band
group carries NIR and two zero channels), converted to 10 bits and coded at
QP 22 and QP 32 with 16 x 16 blocks, search range 32, closed GOPs of 16.
One step = encode + decode + PSNR/bpppb of both QP runs over the whole cube.
The cube is generated on the GPU and resident in HBM before timing starts.

Two forms are timed back to back on the same inputs:
  plain    one run at a time (xv_encode_cube / xv_decode_cube / xv_psnr_bpppb)
  batched  both runs per call (xv_encode_batch / xv_decode_batch /
           xv_psnr_bpppb_batch: one launch per frame step covering both runs)
Both produce bit-identical outputs (checked), hence identical PSNR and bpppb.

Secondary sections (not the headline): the cloud-gapped Sentinel-2-like sweep
(500 x 128 x 128 x 6 f32, 15 QP x N runs), the reanalysis-like cube
(744 x 721 x 1440 x 3 f32, QP 17 and 27, N = 32, R = 8), the sweep again with
quarter-sample motion against integer vectors, the headline cube coded as its
first three principal components, SSIM / spectral angle and the bitstream on
the headline runs, a small serving mix, and the oracle on the
host cores on sampled GOP units of the headline cube.

Prints ONE JSON line.  `value` is the batched throughput in Mpx*band/s of
encode + decode (px*band = T*H*W*bands per run, summed over runs).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
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

HEADLINE = "planet"


def traffic_file(workload: str) -> str:
    """Measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated on a
    1 GiB copy) of one workload, with the sha256 of the kernel sources they
    were taken on."""
    stem = {"s2cloud": "s2cloud_sweep"}.get(workload, workload)
    return os.path.join(ROOT, "profiles", f"{stem}_hbm_traffic.json")


def _measured_traffic(workload: str):
    """Per-kernel-class HBM bytes per launch from the committed counter
    summary, or None when any listed kernel source has changed since."""
    import hashlib
    try:
        with open(traffic_file(workload)) as f:
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
        # the motion-search window layouts are one kernel class
        out.setdefault("me" if name in ("me_kernel", "me_rp_kernel") else name, []).append(float(v))
    return {k: sum(v) / len(v) for k, v in out.items()}


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload_params(xv, wl):
    runs = [(qp, N) for N in wl.blocks for qp in wl.qps]
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=N, search_range=wl.search_range,
                        gop=wl.gop, pad_mode=wl.pad_mode, fill_mode=wl.fill_mode)
              for qp, N in runs]
    return runs, params


def describe(wl) -> str:
    kind = {"planet": "u16 Voronoi land-cover patches (stand-in for DynamicEarthNet), RGB+NIR, "
                      "second band group NIR + 2 zero channels",
            "s2cloud": "f32 with ~10% NaN cloud gaps (stand-in for DeepExtremeCubes)",
            "era5": "f32 reanalysis-like variables (stand-in for ERA5), rows edge-padded to 736",
            "drift": "u16 1/f^3 texture drifting by (0.37, -0.23) samples per frame"}
    return (f"{wl.name}: {wl.T}x{wl.H}x{wl.W}x{wl.bands} {kind.get(wl.name, wl.dtype)}, "
            f"B={wl.bit_depth}, QP{list(wl.qps)} x N{list(wl.blocks)} "
            f"({len(wl.qps) * len(wl.blocks)} runs per step), R={wl.search_range}, "
            f"GOP {wl.gop}, pad {'zero' if wl.pad_mode == 0 else 'repeat'}")


def tune(xv, wl, cube, params, cached, no_tune, split=False):
    """Motion-search launch geometry per block size, tuned on the first P step
    of exactly the batch the timed steps launch (outputs never depend on it).
    split: the adaptive block size's search (params carry FLAG_SPLIT)."""
    tuning = {}
    R = wl.search_range
    setter = xv.set_me_split_geometry if split else xv.set_me_geometry
    getter = xv.get_me_split_geometry if split else xv.get_me_geometry
    for N in wl.blocks:
        key = f"N{N}R{R}" + ("split" if split else "")
        if cached is not None and key in cached:
            g = cached[key]
            setter(N, R, g["blocks_per_wg"], g["cands_per_lane"], g["threads"],
                   g.get("rows_per_lane", 0), g.get("layout", 1))
            tuning[key] = dict(g, tuned=True, from_file=True)
        elif not no_tune:
            _log(f"tuning motion search {wl.name} N={N} R={R}" + (" (split)" if split else ""))
            pn = [p for p in params if p.block == N]
            tuning[key] = dict(xv.autotune_me_batch([cube] * len(pn), pn), tuned=True)
        else:
            tuning[key] = dict(getter(N, R, -(-wl.W // N)), tuned=False)
    return tuning


def run_workload(xv, torch, wl, cube, params, steps, warmup, mode="both", profile_me=True,
                 graphs=True):
    """Times the plain and batched forms; returns their throughput, the
    metrics of the runs, and the kernel profile of the timed steps (motion
    search only) and of one extra step (every class)."""
    outs = [torch.empty_like(cube) for _ in params]
    pxb_step = wl.px_band * len(params)

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
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        lat = []
        if profile:
            # only the dominant kernel (motion search) is event-timed inside
            # the timed region: every event pair costs queue time
            xv.profile_select([xv.K_ME])
            xv.profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            ms = fn(lat)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = xv.profile_read() if profile else None
        if profile:
            xv.profile_enable(False)
        return dt, lat, ms, prof

    res, prof, prof_all = {}, None, None
    ms_plain = ms_batch = None
    if mode in ("both", "plain"):
        _log(f"{wl.name}: plain path")
        dt, lat, ms_plain, _ = timed(step_plain, profile=False)
        res["plain"] = dict(value=pxb_step * steps / dt / 1e6, ms_per_step=dt / steps * 1e3,
                            p50_ms=_percentile(lat, 0.5), p99_ms=_percentile(lat, 0.99),
                            latency_unit="one run: encode+decode+metrics")
    if mode in ("both", "batched"):
        _log(f"{wl.name}: batched path")
        dt, lat, ms_batch, prof = timed(step_batched, profile=profile_me)
        # every kernel class, timed on one more step outside the timed region
        xv.profile_select(None)
        xv.profile_enable(True)
        step_batched()
        prof_all = xv.profile_read()
        xv.profile_enable(False)
        res["batched"] = dict(value=pxb_step * steps / dt / 1e6, ms_per_step=dt / steps * 1e3,
                              p50_ms=_percentile(lat, 0.5), p99_ms=_percentile(lat, 0.99),
                              latency_unit=f"one step: all {len(params)} runs")
        if graphs:
            # the same batched steps with the frame-step launches replayed
            # from captured graphs (no event timing inside)
            _log(f"{wl.name}: batched path, graph replay")
            xv.set_graph_mode(True)
            try:
                dt, lat, ms_graph, _ = timed(step_batched, profile=False)
            finally:
                xv.set_graph_mode(False)
            if any(a["psnr"] != b["psnr"] or a["bpppb"] != b["bpppb"]
                   for a, b in zip(ms_graph, ms_batch)):
                raise SystemExit(f"{wl.name}: graph replay and eager launches disagree")
            res["batched_graph"] = dict(value=pxb_step * steps / dt / 1e6,
                                        ms_per_step=dt / steps * 1e3,
                                        p50_ms=_percentile(lat, 0.5),
                                        p99_ms=_percentile(lat, 0.99),
                                        latency_unit=f"one step: all {len(params)} runs")
    if ms_plain is not None and ms_batch is not None:
        same = all(a["psnr"] == b["psnr"] and a["bpppb"] == b["bpppb"]
                   and a["coef_bits"] == b["coef_bits"] and a["mv_bits"] == b["mv_bits"]
                   for a, b in zip(ms_plain, ms_batch))
        if not same:
            raise SystemExit(f"{wl.name}: batched and plain paths disagree")
    del outs
    return dict(res=res, ms=ms_batch if ms_batch is not None else ms_plain, prof=prof,
                prof_all=prof_all, pxb_step=pxb_step)


def rooflines(r, traffic):
    """Roofline objects: motion search from the timed steps, the transform and
    decode kernels from the extra fully profiled step."""
    out = {}
    prof, prof_all = r["prof"], r["prof_all"]
    traffic = traffic or {}
    if prof is not None and prof["me"]["launches"]:
        me = prof["me"]
        avg_ms = me["ms"] / me["launches"]
        terms = me["work"] / me["launches"]
        achieved = terms / (avg_ms * 1e-3) / 1e12
        out["roofline"] = {"kernel": "motion search (me_rp_kernel / me_kernel)", "bound": "alu",
                           "achieved": round(achieved, 3), "peak": round(SAD_PEAK_TTERMS, 2),
                           "unit": "T SAD-terms/s", "frac": round(achieved / SAD_PEAK_TTERMS, 4),
                           "traffic": round(traffic["me"]) if "me" in traffic else None,
                           "traffic_unit": "bytes per launch",
                           "avg_launch_ms": round(avg_ms, 4), "launches": me["launches"],
                           "terms_per_launch": terms,
                           "timed": "HIP events around every motion-search launch of the timed "
                                    "steps (no other class timed there)"}
    if prof_all is not None:
        for key, kname, label in (("roofline_encode", "encode_kernel",
                                   "encode_kernel (fused transform coding)"),
                                  ("roofline_decode", "decode_kernel", "decode_kernel")):
            d = prof_all[kname.split("_")[0]]
            if not d["launches"]:
                continue
            avg = d["ms"] / d["launches"]
            gbs = d["work"] / d["launches"] / (avg * 1e-3) / 1e9
            out[key] = {"kernel": label, "bound": "hbm", "achieved": round(gbs, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                        "traffic": round(traffic[kname]) if kname in traffic else None,
                        "traffic_unit": "bytes per launch",
                        "algorithmic_bytes_per_launch": round(d["work"] / d["launches"]),
                        "avg_launch_ms": round(avg, 4), "launches": d["launches"],
                        "timed": "one batched step after the timed region, every class timed"}
        out["kernel_ms_per_step"] = {k: round(v["ms"], 3) for k, v in prof_all.items()
                                     if v["launches"]}
    return out


def forms_summary(res):
    return {k: {kk: (round(vv, 3) if isinstance(vv, float) else vv) for kk, vv in v.items()}
            for k, v in res.items()}


def cpu_baseline(cube_host, wl, units_per_qp=8, frames_per_unit=4, cores=None):
    """The oracle as it stands, on the host cores, on a bounded sample of the
    headline step: for each QP, `units_per_qp` (group, GOP) units spread over
    both groups and the cube's length, the first `frames_per_unit` pictures of
    each (the I picture and P pictures with the full search), encoded and then
    decoded, one unit per host thread.  The oracle's band statistics run over
    the whole cube; their time is prorated to the sample's share of the step."""
    import numpy as np
    from oracle import oracle as O
    O.lib()
    if cores is None:
        cores = max(1, min(int(os.environ.get("OMP_NUM_THREADS", "16")), os.cpu_count() or 1))
    T, H, W, Bn = cube_host.shape
    G = (Bn + 2) // 3
    ngop = -(-T // wl.gop)
    t0 = time.perf_counter()
    mn, mx, _ = O.stats(cube_host)
    t_stats = time.perf_counter() - t0
    gops = np.linspace(0, ngop - 1, units_per_qp // G).round().astype(int)
    units = [(qp, g, int(k) * wl.gop, min(frames_per_unit, T - int(k) * wl.gop))
             for qp in wl.qps for g in range(G) for k in gops]

    def one(u):
        qp, g, t0_, n = u
        p = O.CodingParams(bit_depth=wl.bit_depth, qp=qp, block=wl.blocks[0],
                           search_range=wl.search_range, gop=wl.gop, pad_mode=wl.pad_mode,
                           fill_mode=wl.fill_mode)
        o = O.encode_gop(cube_host, mn, mx, p, g, t0_, n)
        O.decode_gop(p, H, W, o["levels"], o["mvs"])
        return min(3, Bn - 3 * g) * n * H * W

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=cores) as ex:
        pxb = sum(ex.map(one, units))
    t_units = time.perf_counter() - t0
    step_pxb = wl.px_band * len(wl.qps) * len(wl.blocks)
    t = t_units + t_stats * pxb / step_pxb
    return {"value": pxb / t / 1e6, "unit": "Mpx·band/s", "cores": min(cores, len(units)),
            "kind": "oracle",
            "sample": f"{len(units)} (QP, group, GOP) units of the {wl.T}x{wl.H}x{wl.W}x{wl.bands} "
                      f"cube (QP {list(wl.qps)} x groups 0..{G - 1} x GOPs {gops.tolist()}), the "
                      f"first {frames_per_unit} pictures of each (I + {frames_per_unit - 1} P, "
                      f"full search R={wl.search_range}), encode + decode, one unit per host "
                      f"thread: {pxb / 1e6:.1f} Mpx·band in {t_units:.1f} s wall, plus the "
                      f"whole-cube band statistics ({t_stats:.1f} s) prorated to the sample "
                      f"({pxb / step_pxb:.4f} of a step). A whole unit has 15 P pictures per I, "
                      f"so the sample slightly favours the oracle."}


def quality_bench(xv, torch, cube, params, runs, steps):
    """SSIM of the coded planes (xv_ssim) and spectral angle of the decoded
    cube (xv_spectral_angle) for every run: the values, and the kernel time
    per step of all runs from HIP events."""
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
    del outs
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
    """Serialise the encoded runs (xv_pack) and parse them back (xv_unpack),
    timed per call on the host (each call synchronises once) and per kernel
    with HIP events; checks that the parsed levels equal the encoded ones."""
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
    pk = xv.pack(encs[0])
    up = xv.unpack(pk.tensor())
    same = bool(torch.equal(up.export()["levels"], encs[0].export()["levels"]))
    up.free()
    pk.free()
    wr, pa = prof["bits_write"], prof["bits_parse"]
    coded = sum(e.export()["levels"].numel() for e in encs)  # coded samples (levels read)
    out = {"runs": len(encs), "payload_MB_per_step": round(payload / 8 / 1e6, 3),
           "pack_ms_per_step": round(t_pack / steps * 1e3, 3),
           "unpack_ms_per_step": round(t_unpack / steps * 1e3, 3),
           "pack_Mpx_band_s": round(pxb_step * steps / t_pack / 1e6, 1),
           "unpack_Mpx_band_s": round(pxb_step * steps / t_unpack / 1e6, 1),
           "parsed_equals_encoded": same}
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


def serve_bench(xv, synth, torch, n=160, seed=4, loads=(0.5, 0.9, 1.2, 2.0),
                t_range=(16, 96), s_range=(64, 256)):
    """Serving mix: requests with the mix's recipe (encode or decode with
    p = 1/2, log-uniform sizes, bands {3, 4, 6}, QP 17..37, N = 16, R = 16)
    at sizes capped to t_range and s_range.  Offered loads are fractions of
    the plain path's measured capacity; the plain baseline serves the same
    arrivals one request at a time."""
    import numpy as np
    dev = torch.device("cuda:0")
    reqs = synth.request_trace(n, rate_per_s=1.0, seed=seed, t_range=t_range, s_range=s_range)
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
           "trace": f"Poisson arrivals; encode/decode p=1/2; T log-uniform {t_range[0]}.."
                    f"{t_range[1]}, side log-uniform {s_range[0]}..{s_range[1]} (multiple of "
                    f"32), bands {{3,4,6}}, QP 17..37, N=16, R=16",
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
    for it in items:
        if it[0] == "decode":
            it[1].free()
    return out


def serve_at_size(xv, synth, torch, n, loads=(0.5, 0.9, 1.2), seed=4):
    """The serving mix at its stated sizes: n requests (encode or decode with
    p = 1/2), T log-uniform in 16..730 and side log-uniform in 64..1024 (the
    tiny recipe's fields up to the Planet-like cube's shape), bands {3, 4, 6},
    QP 17..37, N = 16, R = 16, GOP 16, Poisson arrivals at the offered loads
    rho x the plain path's measured capacity.  Inputs are made at arrival time
    from per-band-count pools of 32 generated 1024 x 1024 frames (frame t of a
    request is pool frame t mod 32, cropped), so only the requests in flight
    occupy memory; decode requests decode one of 8 cubes encoded beforehand.
    Plain = one request at a time in arrival order; served = the continuous-
    batching server.  Latency = completion - arrival."""
    import numpy as np
    dev = torch.device("cuda:0")
    reqs = synth.request_trace(n, rate_per_s=1.0, seed=seed, t_range=(16, 730),
                               s_range=(64, 1024))
    # pools held as int16 views of the u16 samples (gathers support that type)
    pools = {b: synth.tiny_cube(seed=90 + b, T=32, H=1024, W=1024, bands=b,
                                device=dev).view(torch.int16) for b in (3, 4, 6)}
    frame_idx = torch.arange(730, device=dev) % 32

    def make(T, S, b):
        return pools[b].index_select(0, frame_idx[:T])[:, :S, :S, :].contiguous().view(
            torch.uint16)

    def params(qp):
        return xv.Params(bit_depth=10, qp=qp, block=16, search_range=16, gop=16,
                         flags=xv.FLAG_DROP_WORK)

    dec_src = [r for r in reqs if r.op == "decode"][:8]
    pool_enc = []
    for r in dec_src:
        c = make(r.T, r.S, r.bands)
        pool_enc.append((xv.encode_cube(c, params(r.qp)), (r.T, r.S, r.S, r.bands)))
        del c
    torch.cuda.synchronize()
    items = []
    k = 0
    for r in reqs:
        if r.op == "decode":
            e, shape = pool_enc[k % len(pool_enc)]
            k += 1
            items.append(("decode", e, shape, shape[0] * shape[1] * shape[2] * shape[3]))
        else:
            items.append(("encode", (r.T, r.S, r.bands), params(r.qp),
                          r.T * r.S * r.S * r.bands))
    total_pxb = sum(it[3] for it in items)

    def run_plain(it):
        if it[0] == "encode":
            c = make(*it[1])
            e = xv.encode_cube(c, it[2])
            torch.cuda.synchronize()
            e.free()
        else:
            out = torch.empty(it[2], dtype=torch.uint16, device=dev)
            xv.decode_cube(it[1], out)
            torch.cuda.synchronize()

    for it in items[:4]:
        run_plain(it)
    _log(f"serving at size: plain capacity over {n} requests")
    t0 = time.perf_counter()
    for it in items:
        run_plain(it)
    cap_s = time.perf_counter() - t0
    mean_service = cap_s / len(items)
    out = {"requests": len(items), "px_band_total": total_pxb,
           "trace": "Poisson arrivals; encode/decode p=1/2; T log-uniform 16..730, side "
                    "log-uniform 64..1024 (multiple of 32), bands {3,4,6}, QP 17..37, N=16, "
                    "R=16, GOP 16; decode requests decode one of 8 pre-encoded cubes",
           "plain_capacity_mpxb_s": round(total_pxb / cap_s / 1e6, 3),
           "mean_service_ms": round(mean_service * 1e3, 3), "loads": []}
    rng = np.random.default_rng(seed + 1)
    gaps_unit = rng.exponential(1.0, len(items))
    for rho in loads:
        gaps = gaps_unit * mean_service / rho
        arrive = np.cumsum(gaps) - gaps[0]
        _log(f"serving at size: rho {rho} plain")
        lat = []
        base = time.perf_counter()
        for it, a in zip(items, arrive):
            now = time.perf_counter() - base
            if now < a:
                time.sleep(a - now)
            run_plain(it)
            lat.append((time.perf_counter() - base - a) * 1e3)
        plain_span = time.perf_counter() - base
        _log(f"serving at size: rho {rho} served")
        sv = xv.Server(max_slots=64, hbm_budget=96 << 30)
        pending = {}
        slat = []
        st_fail = 0

        def reap(block=False):
            nonlocal st_fail
            for t in list(pending):
                r = sv.wait(t) if block else sv.poll(t)
                if r is None:
                    continue
                delay_ms, _ = pending.pop(t)
                if r["status"] != xv.OK:
                    st_fail += 1
                # arrival -> submit (input made on arrival) + submit -> done
                slat.append(delay_ms + r["done_ms"] - r["submit_ms"])
                if r["enc"] is not None:
                    r["enc"].free()

        base = time.perf_counter()
        for i, (it, a) in enumerate(zip(items, arrive)):
            now = time.perf_counter() - base
            if now < a:
                time.sleep(a - now)
            if it[0] == "encode":
                c = make(*it[1])
                torch.cuda.synchronize()  # the server's stream reads it
                t = sv.submit_encode(c, it[2])
                buf = c
            else:
                buf = torch.empty(it[2], dtype=torch.uint16, device=dev)
                torch.cuda.synchronize()
                t = sv.submit_decode(it[1], buf)
            pending[t] = ((time.perf_counter() - base - a) * 1e3, buf)
            if i % 8 == 0:
                reap()
        reap(block=True)
        served_span = time.perf_counter() - base
        st = sv.stats()
        sv.close()
        if st_fail:
            raise SystemExit("served request failed")
        out["loads"].append({
            "rho": rho,
            "served": {"value": round(total_pxb / served_span / 1e6, 3),
                       "p50_ms": round(_percentile(slat, 0.5), 3),
                       "p99_ms": round(_percentile(slat, 0.99), 3),
                       "peak_active": st["peak_active"], "peak_GB": round(st["peak_bytes"] / 1e9, 1),
                       "iterations": st["iterations"]},
            "plain": {"value": round(total_pxb / plain_span / 1e6, 3),
                      "p50_ms": round(_percentile(lat, 0.5), 3),
                      "p99_ms": round(_percentile(lat, 0.99), 3)}})
    for e, _ in pool_enc:
        e.free()
    return out


def secondary(xv, torch, synth, name, steps, warmup, cached, no_tune):
    """A secondary workload: plain and batched throughput and the rooflines."""
    wl = synth.WORKLOADS[name]
    _log(f"generating {name} cube")
    cube = synth.make_cube(name, device="cuda")
    torch.cuda.synchronize()
    runs, params = workload_params(xv, wl)
    tuning = tune(xv, wl, cube, params, cached, no_tune)
    r = run_workload(xv, torch, wl, cube, params, steps, warmup)
    out = {"workload": describe(wl), "px_band_per_step": r["pxb_step"],
           "forms": forms_summary(r["res"]), "me_geometry": tuning,
           "psnr_db_mean_per_run": [round(sum(m["psnr"]) / len(m["psnr"]), 4) for m in r["ms"]],
           "bpppb_per_run": [round(m["bpppb"], 5) for m in r["ms"]],
           "runs": [f"QP{qp}/N{N}" for qp, N in runs]}
    if "plain" in r["res"] and "batched" in r["res"]:
        out["speedup_batched_vs_plain"] = round(r["res"]["batched"]["value"] /
                                                r["res"]["plain"]["value"], 3)
    out.update(rooflines(r, _measured_traffic(name)))
    del cube
    return out, tuning


def qpel_bench(xv, torch, synth, steps, warmup, cached, no_tune):
    """Quarter-sample motion (XV_FLAG_QPEL) on the drift cube, whose texture
    moves by fractions of a sample per frame: its runs coded with the
    refinement, batched, against the same runs with integer vectors:
    throughput, the refinement kernel's share of the step, and PSNR / bpppb
    of both."""
    wl = synth.WORKLOADS["drift"]
    cube = synth.make_cube("drift", device="cuda")
    torch.cuda.synchronize()
    runs, params = workload_params(xv, wl)
    tune(xv, wl, cube, params, cached, no_tune)
    qparams = [xv.Params(bit_depth=p.bit_depth, qp=p.qp, block=p.block,
                         search_range=p.search_range, gop=p.gop, pad_mode=p.pad_mode,
                         fill_mode=p.fill_mode, flags=xv.FLAG_QPEL) for p in params]
    outs = [torch.empty_like(cube) for _ in params]

    def step(ps):
        encs = xv.encode_batch([cube] * len(ps), ps)
        xv.decode_batch(encs, outs)
        ms = xv.psnr_bpppb_batch([cube] * len(encs), encs)
        for e in encs:
            e.free()
        return ms

    out = {"workload": describe(wl) + "; every run coded twice: integer and quarter-sample "
                                      "vectors", "runs": [f"QP{qp}/N{N}" for qp, N in runs]}
    for name, ps in (("integer", params), ("quarter_sample", qparams)):
        for _ in range(warmup):
            step(ps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ms = step(ps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xv.profile_select(None)
        xv.profile_enable(True)
        step(ps)
        prof = xv.profile_read()
        xv.profile_enable(False)
        out[name] = {"value": round(wl.px_band * len(ps) * steps / dt / 1e6, 3),
                     "ms_per_step": round(dt / steps * 1e3, 3),
                     "psnr_db_mean_per_run": [round(sum(m["psnr"]) / len(m["psnr"]), 4) for m in ms],
                     "bpppb_per_run": [round(m["bpppb"], 5) for m in ms],
                     "kernel_ms_per_step": {k: round(v["ms"], 3) for k, v in prof.items()
                                            if v["launches"]}}
        if prof["subpel"]["launches"]:
            sp = prof["subpel"]
            out[name]["subpel_candidate_samples_per_s"] = sp["work"] / (sp["ms"] * 1e-3)
    del outs, cube
    return out


def split_bench(xv, torch, wl, cube, params, runs, steps, cached, no_tune, warmup=1):
    """Adaptive block size (XV_FLAG_SPLIT) on the headline cube: the same
    runs, batched, with every P block coded whole or as four N/2 blocks by
    SAD + lambda * bits: throughput (one search serves the blocks and their
    cells, with four partial sums per candidate; its geometry tuned like the
    plain search's), the share of split blocks, and PSNR / bpppb.  Returns
    (section, tuning)."""
    sparams = [xv.Params(bit_depth=p.bit_depth, qp=p.qp, block=p.block,
                         search_range=p.search_range, gop=p.gop, pad_mode=p.pad_mode,
                         fill_mode=p.fill_mode, flags=xv.FLAG_SPLIT) for p in params]
    tuning = tune(xv, wl, cube, sparams, cached, no_tune, split=True)
    outs = [torch.empty_like(cube) for _ in sparams]
    frac = []

    def step(count=False):
        encs = xv.encode_batch([cube] * len(sparams), sparams)
        xv.decode_batch(encs, outs)
        ms = xv.psnr_bpppb_batch([cube] * len(encs), encs)
        if count:
            for e in encs:
                sp = e.export()["splits"]
                frac.append(float(sp.to(torch.int32).sum().item()) / sp.numel())
        for e in encs:
            e.free()
        return ms

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ms = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xv.profile_select(None)
    xv.profile_enable(True)
    step(count=True)
    prof = xv.profile_read()
    xv.profile_enable(False)
    del outs
    px_band = wl.px_band * len(sparams)
    n_i = -(-wl.T // params[0].gop)  # I pictures per stream group
    return {"workload": describe(wl) + "; P blocks whole or split into four N/2 blocks",
            "me_geometry": tuning,
            "runs": [f"QP{qp}/N{N}" for qp, N in runs],
            "value": round(px_band * steps / dt / 1e6, 3),
            "ms_per_step": round(dt / steps * 1e3, 3),
            "psnr_db_mean_per_run": [round(sum(m["psnr"]) / len(m["psnr"]), 4) for m in ms],
            "bpppb_per_run": [round(m["bpppb"], 5) for m in ms],
            # over all blocks, I pictures (never split) included
            "split_block_fraction_per_run": [round(f, 4) for f in frac],
            "split_block_fraction_of_P_blocks": [round(f * wl.T / (wl.T - n_i), 4) for f in frac],
            "kernel_ms_per_step": {k: round(v["ms"], 3) for k, v in prof.items() if v["launches"]},
            # the combined search over the whole blocks' in-picture SAD terms
            # (each term serves a block and one of its cells)
            "me_Tterms_per_s": round(prof["me"]["work"] / (prof["me"]["ms"] * 1e-3) / 1e12, 3),
            "me_frac_sad_peak": round(prof["me"]["work"] / (prof["me"]["ms"] * 1e-3) / 1e12
                                      / SAD_PEAK_TTERMS, 4)}, tuning


def intra_bench(xv, torch, wl, cube, params, runs, steps, warmup=1):
    """Intra-predicted I pictures (XV_FLAG_INTRA) on the headline cube: the
    same runs, batched, with every I block predicted by planar or DC from its
    reconstructed neighbours (the I step coded in wavefronts) instead of the
    constant mid-level: throughput, the wavefront kernel's share of the step
    and its bandwidth, and PSNR / bpppb."""
    iparams = [xv.Params(bit_depth=p.bit_depth, qp=p.qp, block=p.block,
                         search_range=p.search_range, gop=p.gop, pad_mode=p.pad_mode,
                         fill_mode=p.fill_mode, flags=xv.FLAG_INTRA) for p in params]
    outs = [torch.empty_like(cube) for _ in iparams]

    def step():
        encs = xv.encode_batch([cube] * len(iparams), iparams)
        xv.decode_batch(encs, outs)
        ms = xv.psnr_bpppb_batch([cube] * len(encs), encs)
        for e in encs:
            e.free()
        return ms

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ms = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xv.profile_select(None)
    xv.profile_enable(True)
    step()
    prof = xv.profile_read()
    xv.profile_enable(False)
    del outs
    px_band = wl.px_band * len(iparams)
    out = {"workload": describe(wl) + "; I pictures intra-predicted (planar / DC)",
           "runs": [f"QP{qp}/N{N}" for qp, N in runs],
           "value": round(px_band * steps / dt / 1e6, 3),
           "ms_per_step": round(dt / steps * 1e3, 3),
           "psnr_db_mean_per_run": [round(sum(m["psnr"]) / len(m["psnr"]), 4) for m in ms],
           "bpppb_per_run": [round(m["bpppb"], 5) for m in ms],
           "kernel_ms_per_step": {k: round(v["ms"], 3) for k, v in prof.items() if v["launches"]}}
    ip = prof["intra"]
    if ip["launches"]:
        out["intra_launches_per_step"] = int(ip["launches"])
        out["intra_GBps"] = round(ip["work"] / (ip["ms"] * 1e-3) / 1e9, 1)
        # latency-bound small launches: their algorithmic bytes against HBM
        out["intra_frac_hbm"] = round(ip["work"] / (ip["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def pca_bench(xv, torch, wl, cube, steps, warmup, k=3):
    """Sec. II-A's example on the headline cube: R, G, B, NIR coded as their
    first k = 3 principal components in one band group instead of two.  One
    step = PCA fit (moments of the whole cube) + projection + encode of both
    QP runs of the PC cube + decode + inverse to the four u16 bands.  Quality
    is the physical-domain PSNR of the inverse against the original (peak =
    band maximum, Sec. II-C), computed for the report only."""
    T, H, W, Bn = cube.shape
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=wl.blocks[0],
                        search_range=wl.search_range, gop=wl.gop) for qp in wl.qps]
    pcs = torch.empty((T, H, W, k), dtype=torch.float32, device=cube.device)
    dec = [torch.empty_like(pcs) for _ in params]
    back = [torch.empty_like(cube) for _ in params]

    def step():
        pca = xv.Pca(cube)  # synchronises (host eigen-decomposition)
        pca.project(cube, 0, k, pcs)
        encs = xv.encode_batch([pcs] * len(params), params)
        xv.decode_batch(encs, dec)
        ms = xv.psnr_bpppb_batch([pcs] * len(encs), encs)
        for d, b in zip(dec, back):
            pca.inverse(d, b)
        torch.cuda.synchronize()
        for e in encs:
            e.free()
        ev = pca.view()["eigval"]
        pca.free()
        return ms, ev

    for _ in range(warmup):
        step()
    t0 = time.perf_counter()
    for _ in range(steps):
        ms, ev = step()
    dt = time.perf_counter() - t0
    xv.profile_select(None)
    xv.profile_enable(True)
    step()
    prof = xv.profile_read()
    xv.profile_enable(False)
    pxb = T * H * W * Bn * len(params)
    out = {"workload": f"{wl.name} cube, bands coded as their first {k} principal components "
                       f"(one band group), QP {list(wl.qps)}, N={wl.blocks[0]}, "
                       f"R={wl.search_range}; one step = fit + project + encode + decode + "
                       f"inverse of both runs",
           "value": round(pxb * steps / dt / 1e6, 3), "unit": "Mpx·band/s (original bands)",
           "ms_per_step": round(dt / steps * 1e3, 3),
           "explained_variance": [round(float(v / ev.sum()), 6) for v in ev],
           "kernel_ms_per_step": {kk: round(v["ms"], 3) for kk, v in prof.items() if v["launches"]}}
    if prof["pca"]["launches"]:
        d = prof["pca"]
        out["pca_kernels_GBs"] = round(d["work"] / (d["ms"] * 1e-3) / 1e9, 1)
        out["pca_kernels_frac_hbm"] = round(d["work"] / (d["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    mx = torch.zeros(Bn, dtype=torch.float64, device=cube.device)
    for t0 in range(0, T, 32):  # band maxima, in slabs
        mx = torch.maximum(mx, cube[t0:t0 + 32].to(torch.int32).reshape(-1, Bn).amax(0).double())
    psnr, bpppb = [], []
    for b_, m in zip(back, ms):
        sse = torch.zeros(Bn, dtype=torch.float64, device=cube.device)
        for t0 in range(0, T, 32):  # in slabs: a float64 copy of the cube is 24 GB
            diff = (b_[t0:t0 + 32].to(torch.int32).double() -
                    cube[t0:t0 + 32].to(torch.int32).double()).reshape(-1, Bn)
            sse += (diff * diff).sum(0)
        mse = sse / (T * H * W)
        psnr.append([round(float(10 * torch.log10(mx[i] ** 2 / mse[i])), 4) for i in range(Bn)])
        bpppb.append(round((m["coef_bits"] + m["mv_bits"]) / (T * H * W * Bn), 5))
    out["psnr_phys_db_per_run_band"] = psnr
    out["bpppb_per_run"] = bpppb
    del pcs, dec, back
    return out


def free_device(xv, torch):
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    xv.cache_release()


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
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the cloud-gapped sweep and the reanalysis-like cube")
    ap.add_argument("--no-qpel", action="store_true",
                    help="skip the quarter-sample motion section")
    ap.add_argument("--no-intra", action="store_true",
                    help="skip the intra-predicted I pictures section")
    ap.add_argument("--no-split", action="store_true",
                    help="skip the adaptive block size section")
    ap.add_argument("--no-pca", action="store_true",
                    help="skip the principal-components section")
    ap.add_argument("--serve-size", type=int, default=0,
                    help="run only the serving mix at its stated sizes with this many "
                         "requests and print its JSON object")
    ap.add_argument("--counters", action="store_true",
                    help="workload for hardware-counter runs only: one 1 GiB device copy (the "
                         "calibration of FETCH_SIZE / WRITE_SIZE), then one batched step of the "
                         "--workload with the geometry file's geometry; prints no result line")
    ap.add_argument("--workload", default=HEADLINE, choices=["planet", "s2cloud", "era5"],
                    help="workload of the --counters run")
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
    cached = None
    if args.geometry_file and os.path.exists(args.geometry_file):
        with open(args.geometry_file) as f:
            cached = json.load(f)
    all_tuning = {}

    if args.serve_size > 0:
        print(json.dumps({"serving_mix_at_size": serve_at_size(xv, synth, torch,
                                                               args.serve_size)}), flush=True)
        return

    if args.counters:
        if cached is None:
            raise SystemExit("--counters needs an existing --geometry-file")
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        wl = synth.WORKLOADS[args.workload]
        cube = synth.make_cube(args.workload, device=dev)
        runs, params = workload_params(xv, wl)
        tune(xv, wl, cube, params, cached, True)
        outs = [torch.empty_like(cube) for _ in params]
        encs = xv.encode_batch([cube] * len(params), params)
        xv.decode_batch(encs, outs)
        torch.cuda.synchronize()
        for e in encs:
            e.free()
        _log("counter workload done")
        return

    wl = synth.WORKLOADS[HEADLINE]
    _log(f"generating {wl.name} cube on {dev}")
    cube = synth.make_cube(HEADLINE, device=dev)
    torch.cuda.synchronize()
    runs, params = workload_params(xv, wl)
    tuning = tune(xv, wl, cube, params, cached, args.no_tune)
    all_tuning.update(tuning)
    r = run_workload(xv, torch, wl, cube, params, args.steps, args.warmup, args.mode)
    res, ms = r["res"], r["ms"]
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
        "config": {"workload": describe(wl), "form": main_form,
                   "px_band_per_step": r["pxb_step"]},
        "me_geometry": tuning,
        "p50_ms": round(res[main_form]["p50_ms"], 3),
        "p99_ms": round(res[main_form]["p99_ms"], 3),
        "forms": forms_summary(res),
        "quality": {"psnr_db_mean_per_run": [round(float(np.mean(m["psnr"])), 4) for m in ms],
                    "psnr_phys_db_mean_per_run": [round(float(np.mean(m["psnr_phys"])), 4)
                                                  for m in ms],
                    "bpppb_per_run": [round(m["bpppb"], 5) for m in ms],
                    "runs": [f"QP{qp}/N{N}" for qp, N in runs]},
    }
    if "plain" in res and "batched" in res:
        line["speedup_batched_vs_plain"] = round(res["batched"]["value"] / res["plain"]["value"], 3)
    line.update(rooflines(r, _measured_traffic(HEADLINE)))
    qsteps = max(1, min(args.steps, 5))
    if not args.no_quality:
        _log("quality metrics")
        line["quality_metrics"] = quality_bench(xv, torch, cube, params, runs, qsteps)
    if not args.no_bits:
        _log("bitstream")
        line["bitstream"] = bits_bench(xv, torch, cube, params, r["pxb_step"], qsteps)
    if not args.no_intra:
        _log("intra-predicted I pictures")
        line["intra"] = intra_bench(xv, torch, wl, cube, params, runs, qsteps)
    if not args.no_split:
        _log("adaptive block size")
        line["split"], t = split_bench(xv, torch, wl, cube, params, runs, max(1, min(args.steps, 3)),
                                       cached, args.no_tune)
        all_tuning.update(t)
    if not args.no_pca:
        _log("principal components")
        line["pca"] = pca_bench(xv, torch, wl, cube, max(1, min(args.steps, 3)), 1)
    host = None
    if not args.no_cpu_baseline:
        host = cube.cpu().numpy()
    del cube, r
    free_device(xv, torch)
    if not args.no_secondary:
        sec = {}
        for name in ("s2cloud", "era5"):
            sec[name], t = secondary(xv, torch, synth, name, max(1, min(args.steps, 10)),
                                     max(1, min(args.warmup, 2)), cached, args.no_tune)
            all_tuning.update(t)
            free_device(xv, torch)
        line["secondary"] = sec
    if not args.no_qpel:
        _log("quarter-sample motion")
        line["quarter_sample"] = qpel_bench(xv, torch, synth, max(1, min(args.steps, 10)),
                                            max(1, min(args.warmup, 2)), cached, args.no_tune)
        free_device(xv, torch)
    if not args.no_serve:
        _log("serving mix")
        line["served"] = serve_bench(xv, synth, torch)
        free_device(xv, torch)
    # write the geometry file when it was missing, or add the keys tuned now
    fresh = {k: {f: v[f] for f in v if f != "from_file"}
             for k, v in all_tuning.items() if not v.get("from_file") and v.get("tuned")}
    if args.geometry_file and (cached is None or fresh):
        merged = dict(cached or {})
        merged.update(fresh if cached is not None else all_tuning)
        with open(args.geometry_file, "w") as f:
            json.dump(merged, f, indent=1)
    if host is not None:
        _log("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(host, wl)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
