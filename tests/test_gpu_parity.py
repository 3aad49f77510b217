"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.  Integer outputs (converted frames,
levels, vectors, reconstructions, bit counts, squared errors) must be
bit-exact; PSNR within 1e-9 dB."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv

pytestmark = pytest.mark.gpu

PSNR_TOL_DB = 1e-9
INT_KEYS = ("frames", "levels", "mvs", "recon", "coef_bits", "mv_bits")


def _oparams(p: xv.Params) -> O.CodingParams:
    return O.CodingParams(bit_depth=p.bit_depth, qp=p.qp, block=p.block,
                          search_range=p.search_range, gop=p.gop, pad_mode=p.pad_mode,
                          fill_mode=p.fill_mode, qpel=1 if p.flags & xv.FLAG_QPEL else 0,
                          intra=1 if p.flags & xv.FLAG_INTRA else 0,
                          split=1 if p.flags & xv.FLAG_SPLIT else 0)


def _to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _psnr_close(a, b):
    if math.isinf(a) or math.isinf(b) or math.isnan(a) or math.isnan(b):
        return (math.isinf(a) and math.isinf(b)) or (math.isnan(a) and math.isnan(b))
    return abs(a - b) <= PSNR_TOL_DB


def check_cube(name: str, host: np.ndarray, p: xv.Params, decode_dtypes=("same",)):
    print(f"[case] {name} shape={host.shape} dtype={host.dtype} {p}", flush=True)
    cube = _to_dev(host)
    enc = xv.encode_cube(cube, p)
    m = xv.psnr_bpppb(cube, enc)
    got = enc.host()
    op = _oparams(p)
    ref = O.encode_cube(host, op)
    for k in INT_KEYS:
        if not np.array_equal(got[k], ref[k]):
            diff = np.argwhere(got[k] != ref[k])
            raise AssertionError(f"{name}: {k} differs in {len(diff)} elements, first at "
                                 f"{diff[0].tolist()}: gpu={got[k][tuple(diff[0])]} "
                                 f"oracle={ref[k][tuple(diff[0])]}")
    if op.split:
        assert np.array_equal(got["splits"], ref["splits"]), f"{name}: split flags differ"
    assert np.array_equal(got["band_min"], ref["mn"]) and np.array_equal(got["band_max"], ref["mx"])
    Bn = host.shape[3]
    sse_gpu = [int(got["sse"][3 * (b // 3) + b % 3]) for b in range(Bn)]
    assert sse_gpu == [int(v) for v in ref["sse"]], (sse_gpu, ref["sse"])
    assert [int(v) for v in got["n_valid"]] == [int(v) for v in ref["nvalid"]]
    om = O.metrics(host, ref, op)
    for b in range(Bn):
        assert _psnr_close(m["psnr"][b], om["psnr"][b]), (b, m["psnr"][b], om["psnr"][b])
        assert _psnr_close(m["psnr_phys"][b], om["psnr_phys"][b]), \
            (b, m["psnr_phys"][b], om["psnr_phys"][b])
    assert m["coef_bits"] == om["coef_bits"] and m["mv_bits"] == om["mv_bits"]
    assert abs(m["bpppb"] - om["bpppb"]) <= 1e-12 * max(1.0, om["bpppb"])
    # decode: closed loop and the caller's dtype
    dec_q = O.decode_cube(op, host.shape, ref["levels"], ref["mvs"],
                          ref["splits"] if op.split else None)
    assert np.array_equal(dec_q, ref["recon"])
    for dt in decode_dtypes:
        tdt = cube.dtype if dt == "same" else dt
        out = torch.empty(host.shape, dtype=tdt, device="cuda")
        xv.decode_cube(enc, out)
        code = O.U16 if tdt == torch.uint16 else O.F32
        expect = O.denormalize_cube(dec_q, host.shape, p.block, p.bit_depth, ref["mn"], ref["mx"],
                                    code)
        got_out = out.cpu().numpy()
        assert np.array_equal(got_out, expect), f"{name}: decoded cube differs ({tdt})"
    enc.free()
    return m


def test_tiny_workload_bit_exact():
    host = synth.tiny_cube(seed=0).numpy()
    check_cube("tiny", host, xv.Params(bit_depth=10, qp=27, block=8, search_range=8, gop=16),
               decode_dtypes=("same", torch.float32))


def _textured(T, H, W, Bn, seed, dtype=np.uint16, nan_frac=0.0, hi=9000):
    """Moving texture with noise: P pictures find non-zero vectors."""
    rng = np.random.default_rng(seed)
    base = rng.integers(0, hi, (H + 16, W + 16, Bn)).astype(np.float64)
    # smooth it a little so that motion is identifiable
    base = (base + np.roll(base, 1, 0) + np.roll(base, 1, 1) + np.roll(base, (1, 1), (0, 1))) / 4
    frames = []
    for t in range(T):
        sy, sx = (t * 2) % 7 - 3, (t * 3) % 5 - 2
        f = np.roll(base, (sy, sx), (0, 1))[:H, :W] + rng.normal(0, 30, (H, W, Bn))
        frames.append(f)
    cube = np.clip(np.stack(frames), 0, 65535)
    if dtype == np.uint16:
        cube = np.round(cube).astype(np.uint16)
    else:
        cube = cube.astype(np.float32)
        if nan_frac > 0:
            cube[rng.random(cube.shape[:3]) < nan_frac] = np.nan
    return cube


@pytest.mark.parametrize("N", [4, 8, 16, 32])
@pytest.mark.parametrize("B", [8, 10, 12])
def test_block_sizes_and_bit_depths_ragged(N, B):
    # H, W not multiples of N (ragged tail), several tiles, 2 band groups
    host = _textured(5, 45, 70 + N, 4, seed=N * 10 + B)
    for qp in (-6 * (B - 8), 22, 51):
        for pad in (xv.PAD_ZERO, xv.PAD_REPEAT):
            p = xv.Params(bit_depth=B, qp=qp, block=N, search_range=5, gop=3, pad_mode=pad)
            check_cube(f"N{N}_B{B}_qp{qp}_pad{pad}", host, p)


@pytest.mark.parametrize("R", [0, 1, 4, 9, 16, 33])
def test_search_ranges(R):
    host = _textured(4, 48, 64, 3, seed=100 + R)
    for N in (8, 16):
        check_cube(f"R{R}_N{N}", host, xv.Params(bit_depth=10, qp=27, block=N, search_range=R,
                                                 gop=4))


@pytest.mark.parametrize("fill", [xv.FILL_NEAREST, xv.FILL_FORWARD])
@pytest.mark.parametrize("bands", [1, 2, 5, 7])
def test_float_input_with_gaps(fill, bands):
    host = _textured(9, 37, 50, bands, seed=7 + bands, dtype=np.float32, nan_frac=0.15)
    host[:, 0, 0, 0] = np.nan  # a pixel series with no valid sample
    p = xv.Params(bit_depth=12, qp=17, block=8, search_range=6, gop=4, fill_mode=fill,
                  pad_mode=xv.PAD_REPEAT)
    check_cube(f"f32_gaps_fill{fill}_bands{bands}", host, p,
               decode_dtypes=("same", torch.uint16))


def test_u16_output_at_rounding_boundaries():
    # float bands from 0.5 to 1023.5 at B = 10 (L = 1023, range R = 1023):
    # band 0 decodes every sample to mn + q R / L = q + 1/2, so its u16
    # output rounds exactly at half-integers, where the product with 1/L
    # defers to the exact quotient; bands 1 and 2 are shifted by +2^-12 and
    # -2^-12 (exact in binary32 at this magnitude), just above and just
    # below those boundaries
    rng = np.random.default_rng(31)
    host = (rng.integers(0, 1024, (5, 24, 40, 3)) + 0.5).astype(np.float64)
    host[0, 0, 0, :] = 0.5
    host[0, 0, 1, :] = 1023.5
    host[..., 1] += 2.0 ** -12
    host[..., 2] -= 2.0 ** -12
    assert np.array_equal(host.astype(np.float32).astype(np.float64), host)  # exact in binary32
    host = host.astype(np.float32)
    for qp in (-12, 27):
        check_cube(f"u16_boundary_qp{qp}", host,
                   xv.Params(bit_depth=10, qp=qp, block=8, search_range=2, gop=5),
                   decode_dtypes=(torch.uint16,))


def test_float_input_without_gaps_and_constant_band():
    host = _textured(6, 33, 41, 3, seed=3, dtype=np.float32)
    host[..., 1] = 273.15  # constant band: q = 0, decodes exactly, PSNR infinite
    m = check_cube("f32_dense_constant", host,
                   xv.Params(bit_depth=12, qp=27, block=16, search_range=4, gop=6))
    assert math.isinf(m["psnr_phys"][1])


@pytest.mark.parametrize("T,H,W,N", [(15, 204, 144, 4), (41, 256, 256, 8)])
def test_group_totals_over_several_ragged_chunks(T, H, W, N):
    # the per-group totals add the per-tile sums in chunks of at most 2048
    # tiles (at most 256 chunks per group): these shapes give 2295 and 5248
    # tiles per group, two and three chunks with a short last one, in two
    # band groups
    Hb, Wb = -(-H // N), -(-W // N)
    n = T * Hb * -(-Wb // (64 // N))
    chunks = min(256, -(-n // 2048))
    assert chunks >= 2 and -(-n // chunks) * chunks != n
    host = _textured(T, H, W, 4, seed=31 + N)
    check_cube(f"totals_{chunks}_chunks_N{N}", host,
               xv.Params(bit_depth=10, qp=27, block=N, search_range=4, gop=8))


def test_edge_shapes():
    # frame smaller than the search window; single frame; all-intra; gop > T
    check_cube("tiny_frame_big_R", _textured(4, 8, 8, 3, seed=1),
               xv.Params(bit_depth=10, qp=27, block=8, search_range=16, gop=4))
    check_cube("single_frame", _textured(1, 20, 30, 3, seed=2),
               xv.Params(bit_depth=10, qp=30, block=4, search_range=2, gop=16))
    check_cube("all_intra", _textured(5, 24, 24, 2, seed=3),
               xv.Params(bit_depth=10, qp=30, block=8, search_range=2, gop=1))
    check_cube("gop_longer_than_T", _textured(7, 24, 40, 3, seed=4),
               xv.Params(bit_depth=10, qp=12, block=8, search_range=3, gop=64))
    check_cube("one_pixel_wide", _textured(3, 5, 1, 1, seed=5),
               xv.Params(bit_depth=8, qp=0, block=4, search_range=2, gop=3))


@pytest.mark.parametrize("layout,nb,kx,threads,rows", [
    (xv.ME_COLUMN_PAIRS, 2, 2, 256, 3), (xv.ME_ROW_PAIRS, 2, 5, 256, 1),
    (xv.ME_ROW_PAIRS_BY_CHANNEL, 1, 5, 512, 1)])
def test_edge_shapes_every_layout(layout, nb, kx, threads, rows):
    # pictures smaller than the window, one block wide, one band (a single
    # real channel), odd window origins (odd R)
    cases = [("tiny_frame_big_R", _textured(4, 8, 8, 3, seed=1), 10, 8, 16),
             ("one_pixel_wide", _textured(3, 5, 1, 1, seed=5), 8, 4, 2),
             ("one_band_odd_R", _textured(4, 20, 44, 1, seed=6), 10, 4, 5),
             ("two_bands_R7", _textured(4, 40, 24, 2, seed=7), 12, 8, 7)]
    for name, host, B, N, R in cases:
        try:
            xv.set_me_geometry(N, R, nb, kx, threads, rows, layout)
            check_cube(f"{name}_layout{layout}", host,
                       xv.Params(bit_depth=B, qp=27, block=N, search_range=R, gop=4))
        finally:
            xv.set_me_geometry(N, R)


def test_row_pair_layouts_at_extreme_search_ranges():
    # R = 0 (one candidate: every other column of a group lies past the
    # range), R = 1, and R = 64 (a window of 2R + N - 1 pair rows that only
    # the channel-by-channel staging fits in LDS)
    host = _textured(4, 48, 64, 3, seed=61)
    cases = [(8, 0, 1, 2, xv.ME_ROW_PAIRS), (16, 0, 2, 11, xv.ME_ROW_PAIRS_BY_CHANNEL),
             (8, 1, 3, 3, xv.ME_ROW_PAIRS), (4, 1, 2, 5, xv.ME_ROW_PAIRS_BY_CHANNEL),
             (4, 64, 1, 13, xv.ME_ROW_PAIRS_BY_CHANNEL), (8, 64, 1, 13, xv.ME_ROW_PAIRS_BY_CHANNEL),
             (16, 64, 1, 13, xv.ME_ROW_PAIRS_BY_CHANNEL)]
    for N, R, nb, kx, lay in cases:
        try:
            xv.set_me_geometry(N, R, nb, kx, 512, 1, lay)
            check_cube(f"N{N}_R{R}_layout{lay}_kx{kx}", host,
                       xv.Params(bit_depth=10, qp=27, block=N, search_range=R, gop=4))
        finally:
            xv.set_me_geometry(N, R)
    with pytest.raises(xv.XvError):  # all three channels of R = 64 exceed the LDS
        xv.set_me_geometry(16, 64, 1, 13, 512, 1, xv.ME_ROW_PAIRS)


def test_s2cloud_reduced_sweep():
    host = synth.s2cloud_cube(T=40).numpy()
    for N in (8, 16, 32):
        for qp in (17, 37):
            check_cube(f"s2cloud40_N{N}_qp{qp}", host,
                       xv.Params(bit_depth=12, qp=qp, block=N, search_range=16, gop=16))


def test_batch_equals_plain_and_is_deterministic():
    cubes = [_textured(6, 40, 56, 4, seed=11), _textured(9, 32, 32, 3, seed=12),
             _textured(5, 64, 48, 6, seed=13, dtype=np.float32, nan_frac=0.05)]
    params = [xv.Params(bit_depth=10, qp=27, block=8, search_range=8, gop=4),
              xv.Params(bit_depth=12, qp=22, block=16, search_range=4, gop=8),
              xv.Params(bit_depth=10, qp=32, block=8, search_range=8, gop=3)]
    dev = [_to_dev(c) for c in cubes]
    plain = [xv.encode_cube(c, p).host() for c, p in zip(dev, params)]
    again = [xv.encode_cube(c, p).host() for c, p in zip(dev, params)]
    batch = [e.host() for e in xv.encode_batch(dev, params)]
    for i in range(3):
        for k in INT_KEYS:
            assert np.array_equal(plain[i][k], again[i][k]), (i, k, "repeat")
            assert np.array_equal(plain[i][k], batch[i][k]), (i, k, "batch")
    encs = xv.encode_batch(dev, params)
    outs = [torch.empty_like(c) for c in dev]
    xv.decode_batch(encs, outs)
    for i in range(3):
        single = torch.empty_like(dev[i])
        xv.decode_cube(encs[i], single)
        assert torch.equal(outs[i], single)


def _same_metrics(a, b):
    assert a.keys() == b.keys()
    for k in a:
        x, y = np.asarray(a[k], dtype=np.float64), np.asarray(b[k], dtype=np.float64)
        assert np.array_equal(x, y, equal_nan=True), (k, a[k], b[k])


def test_batched_metrics_equal_single_calls():
    cubes = [_to_dev(_textured(4, 40, 56, 5, seed=51)),
             torch.from_numpy(synth.s2cloud_cube(seed=3, T=4, H=32, W=40, bands=4).numpy()).cuda(),
             _to_dev(_textured(3, 24, 24, 2, seed=52))]
    params = [xv.Params(bit_depth=10, qp=27, block=8, search_range=4, gop=4),
              xv.Params(bit_depth=12, qp=22, block=16, search_range=3, gop=2),
              xv.Params(bit_depth=8, qp=32, block=4, search_range=2, gop=3)]
    encs = [xv.encode_cube(c, p) for c, p in zip(cubes, params)]
    single = [xv.psnr_bpppb(c, e) for c, e in zip(cubes, encs)]
    batch = xv.psnr_bpppb_batch(cubes, encs)
    for a, b in zip(single, batch):
        _same_metrics(a, b)
    single = [xv.psnr_bpppb(None, e) for e in encs]
    for a, b in zip(single, xv.psnr_bpppb_batch(None, encs)):
        _same_metrics(a, b)
    with pytest.raises(xv.XvError):  # a cube that differs from its encode
        xv.psnr_bpppb_batch([cubes[1], cubes[0], cubes[2]], encs)
    for e in encs:
        e.free()


def test_motion_geometry_never_changes_outputs():
    host = _textured(4, 64, 96, 3, seed=21)
    cube = _to_dev(host)
    p = xv.Params(bit_depth=10, qp=27, block=8, search_range=9, gop=4)
    base = xv.encode_cube(cube, p).host()
    try:
        for nb, kx, th, rows in [(1, 2, 64, 1), (2, 18, 128, 1), (5, 8, 256, 1), (3, 6, 512, 1),
                                 (7, 10, 192, 1), (1, 2, 64, 2), (2, 18, 128, 2), (5, 8, 256, 2),
                                 (3, 6, 512, 2), (12, 12, 320, 2), (1, 2, 64, 3), (4, 6, 192, 3),
                                 (7, 12, 448, 3), (1, 2, 64, 5), (6, 4, 256, 5), (2, 2, 128, 5)]:
            xv.set_me_geometry(8, 9, nb, kx, th, rows, xv.ME_COLUMN_PAIRS)
            got = xv.encode_cube(cube, p).host()
            assert np.array_equal(got["mvs"], base["mvs"]), (nb, kx, th, rows)
            assert np.array_equal(got["recon"], base["recon"]), (nb, kx, th, rows)
        # row-pair layout: every instance, odd and even candidate counts
        for nb, kx, th in [(1, 2, 64), (2, 13, 128), (5, 3, 256), (3, 11, 512), (7, 5, 192),
                           (4, 7, 448), (12, 9, 320), (2, 4, 64), (3, 6, 128), (1, 8, 64)]:
            xv.set_me_geometry(8, 9, nb, kx, th, 1, xv.ME_ROW_PAIRS)
            got = xv.encode_cube(cube, p).host()
            assert np.array_equal(got["mvs"], base["mvs"]), ("rows", nb, kx, th)
            assert np.array_equal(got["recon"], base["recon"]), ("rows", nb, kx, th)
        # row pairs staged channel by channel: items of a workgroup within
        # three rounds of its threads (span 19 here)
        for nb, kx, th in [(1, 2, 64), (2, 13, 128), (5, 3, 256), (3, 11, 512), (7, 5, 192),
                           (4, 7, 448), (12, 9, 320), (2, 4, 64), (3, 6, 128), (1, 8, 64)]:
            xv.set_me_geometry(8, 9, nb, kx, th, 1, xv.ME_ROW_PAIRS_BY_CHANNEL)
            got = xv.encode_cube(cube, p).host()
            assert np.array_equal(got["mvs"], base["mvs"]), ("by channel", nb, kx, th)
            assert np.array_equal(got["recon"], base["recon"]), ("by channel", nb, kx, th)
        with pytest.raises(xv.XvError):  # 16 x 19 x 10 items > 3 x 64
            xv.set_me_geometry(8, 9, 16, 2, 64, 1, xv.ME_ROW_PAIRS_BY_CHANNEL)
    finally:
        xv.set_me_geometry(8, 9)
    # every kernel form against the oracle at every block size, odd and even R
    for N, R in ((4, 3), (16, 8), (32, 5)):
        q = xv.Params(bit_depth=10, qp=22, block=N, search_range=R, gop=4)
        try:
            for kx, rows, lay in ((2, 1, 1), (6, 2, 1), (4, 3, 1), (2, 5, 1), (4, 5, 1),
                                  (3, 1, 2), (11, 1, 2), (2, 1, 2)):
                xv.set_me_geometry(N, R, 2, kx, 256, rows, lay)
                check_cube(f"layout{lay}_rows{rows}_kx{kx}_N{N}_R{R}", host, q)
            for kx in (3, 11, 2):
                xv.set_me_geometry(N, R, 1, kx, 512, 1, xv.ME_ROW_PAIRS_BY_CHANNEL)
                check_cube(f"layout3_kx{kx}_N{N}_R{R}", host, q)
        finally:
            xv.set_me_geometry(N, R)
    # small blocks select with one packed 32-bit key up to R = 32, with the
    # general key beyond
    for R in (32, 33):
        q = xv.Params(bit_depth=12, qp=22, block=8, search_range=R, gop=4)
        try:
            for nb, kx, lay in ((2, 3, xv.ME_ROW_PAIRS), (1, 11, xv.ME_ROW_PAIRS),
                                (1, 13, xv.ME_ROW_PAIRS_BY_CHANNEL)):
                xv.set_me_geometry(8, R, nb, kx, 512, 1, lay)
                check_cube(f"layout{lay}_kx{kx}_N8_R{R}", host, q)
        finally:
            xv.set_me_geometry(8, R)


def test_batch_tuner_installs_a_geometry_that_keeps_outputs():
    cubes = [_to_dev(_textured(5, 48, 80, 4, seed=31 + i)) for i in range(3)]
    params = [xv.Params(bit_depth=10, qp=qp, block=16, search_range=6, gop=4) for qp in (22, 27, 32)]
    before = [xv.encode_cube(c, p).host() for c, p in zip(cubes, params)]
    try:
        g = xv.autotune_me_batch(cubes, params, max_candidates=6)
        assert g["rows_per_lane"] in (1, 2, 3, 5) and g["kernel_ms"] > 0
        assert g["layout"] in (xv.ME_COLUMN_PAIRS, xv.ME_ROW_PAIRS, xv.ME_ROW_PAIRS_BY_CHANNEL)
        assert xv.get_me_geometry(16, 6)["threads"] == g["threads"]
        after = [e.host() for e in xv.encode_batch(cubes, params)]
        for a, b in zip(before, after):
            for k in INT_KEYS:
                assert np.array_equal(a[k], b[k]), k
    finally:
        xv.set_me_geometry(16, 6)


def test_large_sad_blocks_rank_correctly():
    # 12-bit white noise at N = 32: block SADs of several million, far above
    # 16 bits, with many near-ties between candidates
    rng = np.random.default_rng(77)
    host = rng.integers(0, 60000, (4, 64, 96, 3)).astype(np.uint16)
    for N in (16, 32):
        check_cube(f"noise12_N{N}", host, xv.Params(bit_depth=12, qp=17, block=N,
                                                    search_range=4, gop=4))
