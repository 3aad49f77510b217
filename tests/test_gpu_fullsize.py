"""Parity at the full workload sizes, in the launch configuration the
benchmark times (tuned motion-search geometry, batched multi-run encode).

The oracle cannot code a 6-9 GB cube in test time, so it computes sampled
outputs one by one: whole GOP units (every picture: converted frames, vectors,
levels, reconstructions and bit counts) of the cloud-gapped sweep, of the
Planet-like cube and of the reanalysis-like cube, including each cube's
shorter last GOP, from band statistics it computes itself over the whole
cube, and the decoded samples of those units on whole frames.  Properties
that hold at any size are checked on everything: two encodes are identical,
and the batched path equals the plain one."""
import concurrent.futures as cf
import hashlib

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

KEYS = ("frames", "levels", "mvs", "recon", "coef_bits", "mv_bits")


def _op(p: xv.Params) -> O.CodingParams:
    return O.CodingParams(bit_depth=p.bit_depth, qp=p.qp, block=p.block,
                          search_range=p.search_range, gop=p.gop, pad_mode=p.pad_mode,
                          fill_mode=p.fill_mode, qpel=int(bool(p.flags & xv.FLAG_QPEL)),
                          intra=int(bool(p.flags & xv.FLAG_INTRA)),
                          split=int(bool(p.flags & xv.FLAG_SPLIT)))


def _gpu_unit(enc: xv.Encoded, g: int, t0: int, n: int) -> dict:
    """Host copies of frames t0..t0+n-1 of group g."""
    ex = enc.export()
    types = {"frames": np.uint16, "recon": np.uint16, "levels": np.int16, "mvs": np.int8,
             "coef_bits": np.uint32, "mv_bits": np.uint32}
    out = {k: ex[k][g, t0:t0 + n].cpu().numpy().view(ty) for k, ty in types.items()}
    if ex["splits"] is not None:
        # a split block's slot: its four N/2 blocks in z-order, each
        # column-major; presented like the oracle's, each as [l][k]
        sp = ex["splits"][g, t0:t0 + n].cpu().numpy().view(np.uint8)
        raw = ex["levels_raw"][g, t0:t0 + n].cpu().numpy().view(np.int16)
        N = raw.shape[-1]
        cells = raw.reshape(*raw.shape[:-2], 4, N // 2, N // 2).swapaxes(-1, -2).reshape(raw.shape)
        out["levels"] = np.where(sp.astype(bool)[:, None, :, :, None, None], cells, out["levels"])
        out["splits"] = sp
    return out


def _oracle_units(cube_host, mn, mx, p: xv.Params, units):
    """units: list of (g, t0, len); run in parallel host threads."""
    op = _op(p)

    def one(u):
        g, t0, n = u
        return O.encode_gop(cube_host, mn, mx, op, g, t0, n)

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(one, units))


def _compare(name, got, ref):
    for k in KEYS:
        a, b = got[k], ref[k]
        if not np.array_equal(a, b):
            d = np.argwhere(a != b)
            raise AssertionError(f"{name}: {k} differs in {len(d)} elements, first {d[0].tolist()}")


def _digest(enc: xv.Encoded) -> str:
    ex = enc.export()
    h = hashlib.sha256()
    for k in ("levels", "mvs", "recon", "coef_bits", "mv_bits"):
        h.update(ex[k].cpu().numpy().tobytes())
    return h.hexdigest()


@pytest.mark.timeout(900)
def test_s2cloud_full_sweep_sampled_units():
    wl = synth.WORKLOADS["s2cloud"]
    print(f"[case] s2cloud full {wl.T}x{wl.H}x{wl.W}x{wl.bands}", flush=True)
    cube = synth.s2cloud_cube(device="cuda")
    host = cube.cpu().numpy()
    runs = [(qp, N) for N in wl.blocks for qp in wl.qps]
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=N, search_range=wl.search_range,
                        gop=wl.gop, pad_mode=wl.pad_mode, fill_mode=wl.fill_mode)
              for qp, N in runs]
    for N in wl.blocks:  # tuned as the benchmark tunes: on each block size's batch
        pn = [p for p in params if p.block == N]
        xv.autotune_me_batch([cube] * len(pn), pn)
    encs = xv.encode_batch([cube] * len(params), params)
    mn, mx, nv = O.stats(host)
    ngop = -(-wl.T // wl.gop)
    rng = np.random.default_rng(123)
    for i, (p, e) in enumerate(zip(params, encs)):
        got_all = e.host()
        assert np.array_equal(got_all["band_min"], mn) and np.array_equal(got_all["band_max"], mx)
        assert [int(v) for v in got_all["n_valid"]] == [int(v) for v in nv]
        units = [(int(rng.integers(0, 2)), int(k) * wl.gop) for k in rng.choice(ngop, 2, replace=False)]
        units = [(g, t0, min(wl.gop, wl.T - t0)) for g, t0 in units] + [(1, (ngop - 1) * wl.gop,
                                                                          wl.T - (ngop - 1) * wl.gop)]
        refs = _oracle_units(host, mn, mx, p, units)
        for (g, t0, n), ref in zip(units, refs):
            got = {k: got_all[k][g, t0:t0 + n] for k in KEYS}
            _compare(f"s2cloud {runs[i]} unit g{g} t{t0}+{n}", got, ref)
    # plain path equals batched path (two runs) and repeat encodes are identical
    for i in (0, len(params) - 1):
        plain = xv.encode_cube(cube, params[i])
        assert _digest(plain) == _digest(encs[i])
    again = xv.encode_batch([cube] * 2, params[:2])
    assert _digest(again[0]) == _digest(encs[0]) and _digest(again[1]) == _digest(encs[1])


def _unit_decode_reference(cube_host, mn, mx, p: xv.Params, g: int, recon_unit):
    """The oracle's decoded samples of one unit: its reconstruction of group g
    mapped back to the input dtype (other groups left out)."""
    n = recon_unit.shape[0]
    T, H, W, Bn = cube_host.shape
    G = (Bn + 2) // 3
    full = np.zeros((G,) + recon_unit.shape, np.uint16)
    full[g] = recon_unit
    dt = O.U16 if cube_host.dtype == np.uint16 else O.F32
    return O.denormalize_cube(full, (n, H, W, Bn), p.block, p.bit_depth, mn, mx, dt)


def _whole_unit_parity(name, cube, params, gops, groups=None):
    """Both runs of the workload encoded together as the benchmark encodes
    them; for every run, band group and sampled GOP, the whole unit (all of
    its pictures) compared with the oracle, and the decoded cube's samples of
    that unit compared with the oracle's decode."""
    host = cube.cpu().numpy()
    T, H, W, Bn = host.shape
    G = (Bn + 2) // 3
    print(f"[case] {name}: oracle stats over {host.size} samples", flush=True)
    mn, mx, nv = O.stats(host)
    # each search tuned on its own runs (plain, adaptive block size)
    for split in (False, True):
        ps = [p for p in params if bool(p.flags & xv.FLAG_SPLIT) == split]
        if ps:
            xv.autotune_me_batch([cube] * len(ps), ps)
    encs = xv.encode_batch([cube] * len(params), params)
    outs = [torch.empty_like(cube) for _ in params]
    xv.decode_batch(encs, outs)
    ms = xv.psnr_bpppb_batch([cube] * len(encs), encs)
    for e in encs:
        ex = e.export()
        assert np.array_equal(ex["band_min"].cpu().numpy(), mn)
        assert np.array_equal(ex["band_max"].cpu().numpy(), mx)
        assert [int(v) for v in ex["n_valid"].cpu().numpy()] == [int(v) for v in nv]
    jobs = []
    for i, p in enumerate(params):
        for g in (range(G) if groups is None else groups):
            for k in gops:
                t0 = k * p.gop
                jobs.append((i, g, t0, min(p.gop, T - t0)))
    print(f"[case] {name}: oracle on whole units (run, group, t0, len) {jobs}", flush=True)
    op = {i: _op(p) for i, p in enumerate(params)}
    with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        refs = list(ex.map(lambda j: O.encode_gop(host, mn, mx, op[j[0]], j[1], j[2], j[3]), jobs))
    for (i, g, t0, n), ref in zip(jobs, refs):
        tag = f"{name} QP{params[i].qp} unit g{g} t{t0}+{n}"
        got = _gpu_unit(encs[i], g, t0, n)
        _compare(tag, got, ref)
        if "splits" in got:
            assert np.array_equal(got["splits"], ref["splits"]), tag
        # the decoded cube on the samples of this unit, whole frames
        dref = _unit_decode_reference(host, mn, mx, params[i], g, ref["recon"])
        b0, b1 = 3 * g, min(Bn, 3 * g + 3)
        got = outs[i][t0:t0 + n, :, :, b0:b1].cpu().numpy()
        exp = dref[:, :, :, b0:b1]
        if not np.array_equal(got, exp):
            d = np.argwhere(got != exp)
            raise AssertionError(f"{tag}: decoded samples differ in {len(d)} places, "
                                 f"first {d[0].tolist()}")
        print(f"[case] {tag}: ok", flush=True)
    assert all(np.isfinite(m["psnr"]).all() and m["bpppb"] > 0 for m in ms)
    # the plain path gives the batched path's outputs
    plain = xv.encode_cube(cube, params[-1])
    assert _digest(plain) == _digest(encs[-1])
    plain.free()
    for e in encs:
        e.free()


@pytest.mark.timeout(900)
def test_planet_full_size_coding_tools():
    # intra-predicted I pictures and the adaptive block size on the
    # benchmark cube, batched as the bench runs them: the last (short) GOP of
    # band group 1 (NIR and two zero channels) whole, for each tool
    wl = synth.WORKLOADS["planet"]
    print(f"[case] planet full {wl.T}x{wl.H}x{wl.W}x{wl.bands}: intra, split", flush=True)
    cube = synth.planet_cube(device="cuda")
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=16, search_range=wl.search_range,
                        gop=wl.gop, pad_mode=wl.pad_mode, flags=f)
              for qp, f in ((22, xv.FLAG_INTRA), (32, xv.FLAG_SPLIT))]
    _whole_unit_parity("planet tools", cube, params, gops=[45], groups=[1])


@pytest.mark.timeout(1100)
def test_planet_full_size_whole_units():
    wl = synth.WORKLOADS["planet"]
    print(f"[case] planet full {wl.T}x{wl.H}x{wl.W}x{wl.bands}", flush=True)
    cube = synth.planet_cube(device="cuda")
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=16, search_range=wl.search_range,
                        gop=wl.gop, pad_mode=wl.pad_mode) for qp in wl.qps]
    # GOP 45 is the last one: frames 720..729, shorter than the others
    _whole_unit_parity("planet", cube, params, gops=[17, 45])


@pytest.mark.timeout(900)
def test_era5_full_size_whole_units():
    wl = synth.WORKLOADS["era5"]
    print(f"[case] era5 full {wl.T}x{wl.H}x{wl.W}x{wl.bands}", flush=True)
    cube = synth.era5_cube(device="cuda")
    params = [xv.Params(bit_depth=wl.bit_depth, qp=qp, block=32, search_range=wl.search_range,
                        gop=wl.gop) for qp in wl.qps]
    # GOP 46 is the last one: frames 736..743
    _whole_unit_parity("era5", cube, params, gops=[0, 23, 46])
