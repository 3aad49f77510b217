"""GPU parity of the adaptive block size (XV_FLAG_SPLIT) against the oracle:
split flags, cell-grid vectors, levels (whole blocks and the z-ordered cells
of split ones), reconstructions and bit counts bit-exact, PSNR within 1e-9
dB, decode equal to the oracle's.  Covers N = 8, 16, 32 at every bit depth
on ragged frames, 1..3 real channels per group, the search-range limits,
f32 input with gaps, the batched, graph-replayed and served forms mixed
with cubes without the flag, and the bitstream round trip."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv
from test_gpu_bitstream import _sections
from test_gpu_parity import _textured, check_cube

pytestmark = pytest.mark.gpu


def _mixed_motion(T, H, W, Bn, seed):
    """A moving texture whose N/2 cells move by different vectors, so that
    both choices occur."""
    rng = np.random.default_rng(seed)
    tex = rng.integers(0, 6000, (H + 24, W + 24, Bn)).astype(np.float64)
    tex = (tex + np.roll(tex, 1, 0) + np.roll(tex, 1, 1)) / 3
    frames = []
    for t in range(T):
        f = np.roll(tex, ((t * 2) % 5 - 2, (t * 3) % 7 - 3), (0, 1))[:H, :W].copy()
        for _ in range(max(1, H * W // 400)):
            y, x = rng.integers(0, H - 8), rng.integers(0, W - 8)
            sy, sx = rng.integers(-3, 4, 2)
            f[y:y + 8, x:x + 8] = np.roll(tex, (int(sy), int(sx)), (0, 1))[y:y + 8, x:x + 8]
        frames.append(f + rng.normal(0, 12, (H, W, Bn)))
    return np.clip(np.round(np.stack(frames)), 0, 65535).astype(np.uint16)


@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("B", [8, 10, 12])
def test_split_block_sizes_and_bit_depths(N, B):
    host = _mixed_motion(5, 45 + N, 70 + 2 * N, 4, seed=N * 10 + B)
    seen = set()
    for qp in (-6 * (B - 8), 22, 37):
        p = xv.Params(bit_depth=B, qp=qp, block=N, search_range=4, gop=4, flags=xv.FLAG_SPLIT)
        check_cube(f"split N{N} B{B} QP{qp}", host, p)
        e = xv.encode_cube(torch.from_numpy(host).cuda(), p)
        seen |= set(np.unique(e.host()["splits"]).tolist())
    assert seen == {0, 1}


def test_split_search_ranges_padding_and_channels():
    host = _mixed_motion(4, 40, 56, 5, seed=3)
    for R in (0, 1, 9):
        for pad in (xv.PAD_ZERO, xv.PAD_REPEAT):
            p = xv.Params(bit_depth=10, qp=22, block=16, search_range=R, gop=4, pad_mode=pad,
                          flags=xv.FLAG_SPLIT)
            check_cube(f"split R{R} pad{pad}", host, p)
    cube = torch.from_numpy(host).cuda()
    for flags in (xv.FLAG_SPLIT | xv.FLAG_QPEL, xv.FLAG_SPLIT | xv.FLAG_INTRA):
        with pytest.raises(xv.XvError) as ei:
            xv.encode_cube(cube, xv.Params(bit_depth=10, qp=22, block=8, search_range=4, gop=4,
                                           flags=flags))
        assert ei.value.code == xv.EINVAL
    with pytest.raises(xv.XvError):
        xv.encode_cube(cube, xv.Params(bit_depth=10, qp=22, block=4, search_range=4, gop=4,
                                       flags=xv.FLAG_SPLIT))


def test_split_float_gaps_and_tiny_workload():
    host = _textured(6, 37, 50, 6, seed=5, dtype=np.float32, nan_frac=0.05)
    p = xv.Params(bit_depth=12, qp=27, block=16, search_range=6, gop=6, flags=xv.FLAG_SPLIT)
    check_cube("split f32 gaps", host, p, decode_dtypes=("same", torch.uint16))
    host = synth.tiny_cube(seed=0).numpy()
    p = xv.Params(bit_depth=10, qp=27, block=8, search_range=8, gop=16, flags=xv.FLAG_SPLIT)
    check_cube("split tiny", host, p)


def _digest(enc):
    h = enc.host()
    return [h[k].tobytes() for k in ("levels", "mvs", "recon", "coef_bits", "mv_bits", "splits")
            if h.get(k) is not None]


def test_batched_graph_and_served_forms_mix_split_and_plain_cubes():
    hosts = [_mixed_motion(7, 48, 64, 3, seed=11), _mixed_motion(9, 40, 40, 4, seed=12),
             _mixed_motion(5, 64, 48, 6, seed=13)]
    cubes = [torch.from_numpy(h).cuda() for h in hosts]
    params = [xv.Params(bit_depth=10, qp=22, block=16, search_range=4, gop=4, flags=xv.FLAG_SPLIT),
              xv.Params(bit_depth=10, qp=27, block=16, search_range=4, gop=4),
              xv.Params(bit_depth=12, qp=30, block=16, search_range=4, gop=3, flags=xv.FLAG_SPLIT)]
    print("[case] split batched + graph + served mix", flush=True)
    plain = [xv.encode_cube(c, p) for c, p in zip(cubes, params)]
    batch = xv.encode_batch(cubes, params)
    for a, b in zip(plain, batch):
        assert _digest(a) == _digest(b)
    outs_p = [torch.empty_like(c) for c in cubes]
    outs_b = [torch.empty_like(c) for c in cubes]
    for e, o in zip(plain, outs_p):
        xv.decode_cube(e, o)
    xv.decode_batch(batch, outs_b)
    for a, b in zip(outs_p, outs_b):
        assert torch.equal(a, b)
    xv.set_graph_mode(True)
    try:
        for rep in range(3):
            g = xv.encode_batch(cubes, params)
            outs_g = [torch.empty_like(c) for c in cubes]
            xv.decode_batch(g, outs_g)
            torch.cuda.synchronize()
            for a, b in zip(plain, g):
                assert _digest(a) == _digest(b), rep
            for a, b in zip(outs_p, outs_g):
                assert torch.equal(a, b), rep
            for e in g:
                e.free()
    finally:
        xv.set_graph_mode(False)
    sv = xv.Server(max_slots=8)
    tickets = [sv.submit_encode(c, p) for c, p in zip(cubes, params)]
    outs_s = [torch.empty_like(c) for c in cubes]
    tickets += [sv.submit_decode(e, o) for e, o in zip(plain, outs_s)]
    res = [sv.wait(t) for t in tickets]
    assert all(r["status"] == xv.OK for r in res)
    for r, a in zip(res[:3], plain):
        assert _digest(r["enc"]) == _digest(a)
    for a, b in zip(outs_s, outs_p):
        assert torch.equal(a, b)
    sv.close()


def test_split_bitstream_round_trip():
    host = _mixed_motion(6, 40, 48, 4, seed=21)
    cube = torch.from_numpy(host).cuda()
    p = xv.Params(bit_depth=10, qp=25, block=16, search_range=6, gop=3, flags=xv.FLAG_SPLIT)
    enc = xv.encode_cube(cube, p)
    h = enc.host()
    op = O.CodingParams(bit_depth=10, qp=25, block=16, search_range=6, gop=3, split=1)
    ref = O.encode_cube(host, op)
    assert ref["splits"].any()
    # coefficient units of coded flags 0 only, whole (1 bit) and split (4 bits):
    # the writer emits those without reading the levels
    sp = np.broadcast_to(ref["splits"].astype(bool)[:, :, None], ref["coef_bits"].shape)
    assert ((ref["coef_bits"] == 4) & sp).any() and ((ref["coef_bits"] == 1) & ~sp).any()
    # payload bytes and index are the oracle writer's on the oracle's own encode
    ref_bits = O.write_bitstream(ref["levels"], ref["mvs"], 3, splits=ref["splits"])
    pk = xv.pack(enc)
    assert pk.view()["payload_bits"] == ref_bits["bits"]
    sec = _sections(pk.tensor().cpu().numpy())
    assert np.array_equal(sec["payload"], ref_bits["payload"])
    assert np.array_equal(sec["index"], ref_bits["index"])
    assert not sec["tail"].any()
    un = xv.unpack(pk.tensor())
    g = un.host()
    for k in ("levels", "mvs", "coef_bits", "mv_bits", "splits"):
        assert np.array_equal(g[k], h[k]), k
    a, b = torch.empty_like(cube), torch.empty_like(cube)
    xv.decode_cube(enc, a)
    xv.decode_cube(un, b)
    assert torch.equal(a, b)
    dq = O.decode_cube(op, host.shape, ref["levels"], ref["mvs"], ref["splits"])
    assert np.array_equal(b.cpu().numpy(), O.denormalize_cube(dq, host.shape, 16, 10, ref["mn"],
                                                              ref["mx"], O.U16))


def test_split_at_a_large_picture():
    # a 1024 x 1024 picture pair at N = 16, R = 8 against the oracle
    host = _mixed_motion(2, 1024, 1024, 3, seed=77)
    p = xv.Params(bit_depth=10, qp=27, block=16, search_range=8, gop=16, flags=xv.FLAG_SPLIT)
    print("[case] split 1024x1024 N16", flush=True)
    check_cube("split 1024^2", host, p)


def test_split_search_geometry_never_changes_outputs():
    # every combined-search instance (both row-pair layouts, 5, 7, 11 and 13
    # candidates per lane) at several workgroup shapes, on ragged frames whose
    # edge cells reach candidates their blocks cannot; one geometry against
    # the oracle, the others against it
    for N, R in ((8, 9), (16, 5), (32, 4)):
        host = _mixed_motion(4, 45 + N, 70 + 2 * N, 4, seed=N + R)
        cube = torch.from_numpy(host).cuda()
        p = xv.Params(bit_depth=10, qp=25, block=N, search_range=R, gop=4, flags=xv.FLAG_SPLIT)
        span = 2 * R + 1
        ref = None
        try:
            for lay in (xv.ME_ROW_PAIRS, xv.ME_ROW_PAIRS_BY_CHANNEL):
                for kx in (5, 7, 11, 13):
                    rounds = 1 if kx >= 11 else 2
                    for nb, th in ((1, 64), (3, 192), (2, 512)):
                        items = nb * span * (-(-span // kx))
                        if lay == xv.ME_ROW_PAIRS_BY_CHANNEL and items > rounds * th:
                            continue
                        xv.set_me_split_geometry(N, R, nb, kx, th, 1, lay)
                        print(f"[case] split geometry N{N} R{R} layout{lay} kx{kx} nb{nb} th{th}",
                              flush=True)
                        if ref is None:
                            check_cube(f"split geometry N{N}", host, p)
                            ref = _digest(xv.encode_cube(cube, p))
                        else:
                            assert _digest(xv.encode_cube(cube, p)) == ref, (lay, kx, nb, th)
            # the tuner on split params installs the combined search's geometry
            g = xv.autotune_me_batch([cube], [p], max_candidates=6)
            assert xv.get_me_split_geometry(N, R) == {k: g[k] for k in (
                "blocks_per_wg", "cands_per_lane", "threads", "rows_per_lane", "layout")}
            assert _digest(xv.encode_cube(cube, p)) == ref
        finally:
            xv.set_me_split_geometry(N, R)
