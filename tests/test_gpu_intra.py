"""GPU parity of intra-predicted I pictures (XV_FLAG_INTRA) against the
oracle: modes, levels, reconstructions and bit counts bit-exact, PSNR within
1e-9 dB, decode equal to the oracle's.  Covers every block size and bit
depth on ragged frames (border blocks without top-right or left neighbours),
pictures one block wide or tall, zero and repeated padding channels, f32
input with gaps, quarter-sample P pictures after intra I pictures, the
batched, graph-replayed and served forms mixed with cubes without the flag,
and the bitstream round trip of the modes."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv
from test_gpu_parity import _textured, check_cube
from test_gpu_qpel import _smooth_motion

pytestmark = pytest.mark.gpu


def _smooth(T, H, W, Bn, seed, noise=10.0):
    """Smooth gradients with edges: both modes win somewhere."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    out = np.empty((T, H, W, Bn))
    for b in range(Bn):
        base = (1500 + 900 * np.sin(xx / (6.0 + b)) + 700 * np.cos(yy / 9.0) + 11 * xx
                + 600 * ((xx + 2 * yy) % 37 < 9))
        for t in range(T):
            out[t, :, :, b] = base + 13 * t + rng.normal(0, noise, (H, W))
    return np.clip(np.round(out), 0, 65535).astype(np.uint16)


def _modes(enc, gop):
    mv = enc.host()["mvs"]
    return mv[:, ::gop, :, :, 0]


@pytest.mark.parametrize("N", [4, 8, 16, 32])
@pytest.mark.parametrize("B", [8, 10, 12])
def test_intra_block_sizes_and_bit_depths(N, B):
    # ragged H and W, two band groups (3 + 1 real channels), several wavefronts
    host = _smooth(5, 45 + N, 70 + 2 * N, 4, seed=N * 10 + B)
    for qp in (-6 * (B - 8), 30):
        p = xv.Params(bit_depth=B, qp=qp, block=N, search_range=4, gop=4, flags=xv.FLAG_INTRA)
        check_cube(f"intra N{N} B{B} QP{qp}", host, p)
    cube = torch.from_numpy(host).cuda()
    e = xv.encode_cube(cube, xv.Params(bit_depth=B, qp=30, block=N, search_range=4, gop=4,
                                       flags=xv.FLAG_INTRA))
    modes = _modes(e, 4)
    assert set(np.unique(modes)) <= {0, 1}
    if N <= 16:
        assert (modes == 0).any() and (modes == 1).any()


def test_intra_thin_pictures_and_padding_modes():
    for (H, W) in ((8, 200), (200, 8), (8, 8), (33, 17)):
        host = _smooth(3, H, W, 5, seed=H * W)
        for pad in (xv.PAD_ZERO, xv.PAD_REPEAT):
            p = xv.Params(bit_depth=10, qp=25, block=8, search_range=3, gop=2, pad_mode=pad,
                          flags=xv.FLAG_INTRA)
            check_cube(f"intra {H}x{W} pad{pad}", host, p)


def test_intra_float_gaps_and_gop_one():
    host = _textured(6, 37, 50, 6, seed=5, dtype=np.float32, nan_frac=0.05)
    p = xv.Params(bit_depth=12, qp=27, block=16, search_range=6, gop=6, flags=xv.FLAG_INTRA)
    check_cube("intra f32 gaps", host, p, decode_dtypes=("same", torch.uint16))
    host = _smooth(4, 40, 48, 3, seed=8)
    p = xv.Params(bit_depth=10, qp=22, block=8, search_range=4, gop=1, flags=xv.FLAG_INTRA)
    check_cube("intra all-I", host, p)


def test_intra_with_quarter_sample_motion():
    host = _smooth_motion(6, 45, 70, 4, seed=31)
    p = xv.Params(bit_depth=10, qp=27, block=8, search_range=5, gop=3,
                  flags=xv.FLAG_INTRA | xv.FLAG_QPEL)
    check_cube("intra + qpel", host, p)


def test_intra_tiny_workload():
    host = synth.tiny_cube(seed=0).numpy()
    p = xv.Params(bit_depth=10, qp=27, block=8, search_range=8, gop=16, flags=xv.FLAG_INTRA)
    check_cube("intra tiny", host, p)


def _digest(enc):
    h = enc.host()
    return [h[k].tobytes() for k in ("levels", "mvs", "recon", "coef_bits", "mv_bits")]


def test_batched_graph_and_served_forms_mix_intra_and_plain_cubes():
    hosts = [_smooth(7, 48, 64, 3, seed=11), _smooth(9, 40, 40, 4, seed=12),
             _smooth(5, 64, 48, 6, seed=13), _smooth(6, 40, 56, 3, seed=14)]
    cubes = [torch.from_numpy(h).cuda() for h in hosts]
    params = [xv.Params(bit_depth=10, qp=22, block=8, search_range=4, gop=4, flags=xv.FLAG_INTRA),
              xv.Params(bit_depth=10, qp=27, block=8, search_range=4, gop=4),
              xv.Params(bit_depth=12, qp=30, block=8, search_range=7, gop=3,
                        flags=xv.FLAG_INTRA | xv.FLAG_QPEL),
              xv.Params(bit_depth=10, qp=32, block=16, search_range=4, gop=5,
                        flags=xv.FLAG_INTRA)]
    print("[case] intra batched + graph + served mix", flush=True)
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
    # graph replay: capture on the first batch, replay on later ones
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
    for r, a in zip(res[:4], plain):
        assert _digest(r["enc"]) == _digest(a)
    for a, b in zip(outs_s, outs_p):
        assert torch.equal(a, b)
    sv.close()


def test_intra_bitstream_round_trip():
    host = _smooth(6, 40, 48, 4, seed=21)
    cube = torch.from_numpy(host).cuda()
    p = xv.Params(bit_depth=10, qp=25, block=8, search_range=6, gop=3, flags=xv.FLAG_INTRA)
    enc = xv.encode_cube(cube, p)
    h = enc.host()
    op = O.CodingParams(bit_depth=10, qp=25, block=8, search_range=6, gop=3, intra=1)
    ref = O.encode_cube(host, op)
    # the payload length and bytes are the oracle writer's on the oracle's own encode
    ref_bits = O.write_bitstream(ref["levels"], ref["mvs"], 3, imodes=1)
    pk = xv.pack(enc)
    v = pk.view()
    assert v["payload_bits"] == ref_bits["bits"]
    un = xv.unpack(pk.tensor())
    g = un.host()
    for k in ("levels", "mvs", "coef_bits", "mv_bits"):
        assert np.array_equal(g[k], h[k]), k
    a, b = torch.empty_like(cube), torch.empty_like(cube)
    xv.decode_cube(enc, a)
    xv.decode_cube(un, b)
    assert torch.equal(a, b)
    dq = O.decode_cube(op, host.shape, ref["levels"], ref["mvs"])
    assert np.array_equal(b.cpu().numpy(), O.denormalize_cube(dq, host.shape, 8, 10, ref["mn"],
                                                              ref["mx"], O.U16))


def test_intra_at_a_large_picture_sampled():
    # a 1024 x 1024 picture pair at N = 16 (the benchmark's block size and
    # shape): every block of the intra I picture and of the P picture after
    # it against the oracle's encode of that one GOP
    H = W = 1024
    host = _smooth(2, H, W, 3, seed=77, noise=20.0)
    p = xv.Params(bit_depth=10, qp=22, block=16, search_range=4, gop=16, flags=xv.FLAG_INTRA)
    print("[case] intra 1024x1024 N16", flush=True)
    check_cube("intra 1024^2", host, p)
