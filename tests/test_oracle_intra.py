"""CPU pins of the oracle's intra prediction of I pictures (planar and DC,
ITU-T H.265 8.4.4.2), and of the coding loop with it.

What pins it, none of it derived from the oracle itself:
- hand-worked planar and DC predictions with the intermediate values written
  out (tests/golden/hevc_intra.txt): no smoothing at N = 4, [1 2 1] smoothing
  at N = 8 and 16, strong smoothing at N = 32 on and off across its
  threshold, the DC edge filter below N = 32 only;
- closed forms: constant references predict the constant (both modes, all N);
  DC of a constant left column and top row;
- structure of planar: transposing the references transposes the prediction;
  an impulse on p[-1][y0] at N = 4 reaches row y0 only, decreasing to the
  right; the top-right sample shapes every row alike;
- the reference-sample process written independently here (per-sample
  availability in raster block order, then the substitution scan), compared
  on every block of random planes for every N;
- brute force over the two modes: the chosen mode has the smaller SAD over
  the real channels (planar on ties) against the reconstruction the oracle
  made, and its levels are the transform and quantiser of the residual
  against that prediction;
- the coding loop: decode reproduces the encoder's reconstruction; each I
  block costs one mode bit; the bitstream round trip keeps the modes; the
  first block of a picture has no neighbours, so its levels equal those of
  the constant mid-level prediction.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hevc_intra.txt")


def _list(tok, n):
    """'k*v' repeats, 'base v set i:w ...' or n plain values."""
    if tok[0] == "base":
        v = [int(tok[1])] * n
        if len(tok) > 2:
            assert tok[2] == "set"
            for s in tok[3:]:
                i, w = s.split(":")
                v[int(i)] = int(w)
        return v
    out = []
    for t in tok:
        if "*" in t:
            k, v = t.split("*")
            out += [int(v)] * int(k)
        else:
            out.append(int(t))
    assert len(out) == n, (tok, n)
    return out


def _scan_refs(N, corner, left, top):
    """The 4N + 1 references in substitution-scan order."""
    return np.array(list(reversed(left)) + [corner] + list(top), np.int32)


def _golden():
    refs, cases = {}, []
    for line in open(GOLD):
        line = line.split("#")[0].split()
        if not line:
            continue
        if line[0] == "refs":
            name, N = line[1], int(line[2])
            i_l, i_t = line.index("left"), line.index("top")
            corner = int(line[line.index("corner") + 1])
            left = _list(line[i_l + 1:i_t], 2 * N)
            top = _list(line[i_t + 1:], 2 * N)
            refs[name] = (N, _scan_refs(N, corner, left, top))
        elif line[0] == "expect":
            cases.append((line[1], int(line[2]), int(line[3]), int(line[4]), int(line[5]),
                          int(line[6])))
        elif line[0] == "allequal":
            cases.append((line[1], int(line[2]), int(line[3]), None, None, int(line[4])))
    return refs, cases


def test_golden_worked_examples():
    refs, cases = _golden()
    assert len(cases) >= 40
    for name, B, mode, y, x, v in cases:
        N, r = refs[name]
        pred = O.intra_predict(r, N, mode, B)
        if y is None:
            assert (pred == v).all(), (name, mode, np.unique(pred))
        else:
            assert pred[y, x] == v, (name, mode, y, x, pred[y, x], v)


@pytest.mark.parametrize("N", [4, 8, 16, 32])
@pytest.mark.parametrize("B", [8, 10, 12])
def test_constant_references_predict_the_constant(N, B):
    for v in (0, 1, 77, (1 << B) - 1):
        r = np.full(4 * N + 1, v, np.int32)
        for mode in (0, 1):
            assert (O.intra_predict(r, N, mode, B) == v).all()


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_dc_of_two_constant_edges(N):
    # left a, top b: dcVal = floor((a + b + 1) / 2); edge filter below N = 32
    for a, b in ((100, 300), (7, 8), (1000, 3)):
        r = _scan_refs(N, 0, [a] * (2 * N), [b] * (2 * N))
        p = O.intra_predict(r, N, 1, 10)
        dc = (a + b + 1) // 2
        if N == 32:
            assert (p == dc).all()
            continue
        assert p[0, 0] == (a + 2 * dc + b + 2) // 4
        assert (p[0, 1:] == (b + 3 * dc + 2) // 4).all()
        assert (p[1:, 0] == (a + 3 * dc + 2) // 4).all()
        assert (p[1:, 1:] == dc).all()


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_planar_transposes_with_its_references(N):
    rng = np.random.default_rng(N)
    for _ in range(20):
        left = rng.integers(0, 1024, 2 * N)
        top = rng.integers(0, 1024, 2 * N)
        c = int(rng.integers(0, 1024))
        for mode in (0, 1):
            a = O.intra_predict(_scan_refs(N, c, left, top), N, mode, 10)
            b = O.intra_predict(_scan_refs(N, c, top, left), N, mode, 10)
            assert (a == b.T).all()


def test_planar_impulse_responses_at_n4():
    # no smoothing at N = 4: an impulse on p[-1][y0] reaches row y0 only and
    # falls off to the right; the top-right sample weighs every row alike,
    # growing to the right; the bottom-left one every column alike
    N, K = 4, 1000
    for y0 in range(N):
        left = [0] * 8
        left[y0] = K
        p = O.intra_predict(_scan_refs(N, 0, left, [0] * 8), N, 0, 10)
        assert (np.delete(p, y0, axis=0) == 0).all()
        assert (np.diff(p[y0]) < 0).all() and p[y0, 0] > 0
    top = [0] * 8
    top[N] = K
    p = O.intra_predict(_scan_refs(N, 0, [0] * 8, top), N, 0, 10)
    assert (p == p[0]).all() and (np.diff(p[0]) > 0).all()
    left = [0] * 8
    left[N] = K
    p = O.intra_predict(_scan_refs(N, 0, left, [0] * 8), N, 0, 10)
    assert (p.T == p[:, 0]).all() and (np.diff(p[:, 0]) > 0).all()
    # rounding: a single unit on p[-1][N] gives ((y + 1) + 4) >> 3
    left = [0] * 8
    left[N] = 1
    p = O.intra_predict(_scan_refs(N, 0, left, [0] * 8), N, 0, 8)
    assert list(p[:, 0]) == [0, 0, 0, 1]


def _refs_brute(plane, N, B, bx, by):
    """H.265 8.4.4.2.2 written out here: availability of each neighbour
    sample (inside the picture and in a block coded earlier in raster order),
    then the substitution scan from p[-1][2N-1] up and along the top."""
    Hp, Wp = plane.shape
    Wb = Wp // N
    x0, y0 = bx * N, by * N
    pos = [(x0 - 1, y0 + 2 * N - 1 - i) for i in range(2 * N)]
    pos += [(x0 - 1, y0 - 1)]
    pos += [(x0 + i, y0 - 1) for i in range(2 * N)]
    vals = []
    for (x, y) in pos:
        ok = 0 <= x < Wp and 0 <= y < Hp and (y // N) * Wb + (x // N) < by * Wb + bx
        vals.append(int(plane[y, x]) if ok else None)
    if all(v is None for v in vals):
        return np.full(len(vals), 1 << (B - 1), np.int32)
    if vals[0] is None:
        vals[0] = next(v for v in vals if v is not None)
    for i in range(1, len(vals)):
        if vals[i] is None:
            vals[i] = vals[i - 1]
    return np.array(vals, np.int32)


@pytest.mark.parametrize("N", [4, 8, 16, 32])
def test_reference_samples_against_the_process(N):
    rng = np.random.default_rng(100 + N)
    for Hb, Wb in ((3, 4), (1, 3), (4, 1), (2, 2)):
        plane = rng.integers(0, 4096, (Hb * N, Wb * N)).astype(np.uint16)
        for by in range(Hb):
            for bx in range(Wb):
                got = O.intra_refs(plane, N, 12, bx, by)
                exp = _refs_brute(plane, N, 12, bx, by)
                assert (got == exp).all(), (N, Hb, Wb, bx, by)


def test_reference_samples_special_cases():
    N, B = 4, 10
    plane = (np.arange(12 * 16).reshape(12, 16) + 5).astype(np.uint16)
    # first block: nothing available -> 2^(B-1)
    assert (O.intra_refs(plane, N, B, 0, 0) == 512).all()
    # top row, bx > 0: the left column; the bottom-left part repeats
    # p[-1][N-1]; the corner and the whole top repeat p[-1][0]
    r = O.intra_refs(plane, N, B, 2, 0)
    left = [int(plane[y, 7]) for y in range(N)]
    assert list(r[N:2 * N]) == left[::-1]
    assert (r[:N] == left[N - 1]).all()
    assert (r[2 * N:] == left[0]).all()
    # left column, by > 0: everything before the top row repeats p[0][-1]
    r = O.intra_refs(plane, N, B, 0, 1)
    assert (r[:2 * N + 1] == plane[3, 0]).all()
    assert list(r[2 * N + 1:]) == [int(plane[3, x]) for x in range(2 * N)]
    # last column: no top-right; it repeats p[N-1][-1]
    r = O.intra_refs(plane, N, B, 3, 1)
    assert list(r[2 * N + 1:3 * N + 1]) == [int(plane[3, 12 + x]) for x in range(N)]
    assert (r[3 * N + 1:] == plane[3, 15]).all()
    assert r[2 * N] == plane[3, 11]


def _cube(T=5, H=40, W=56, bands=3, seed=0, dtype=np.uint16):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    c = np.empty((T, H, W, bands), np.float64)
    for b in range(bands):
        base = 400 + 300 * np.sin(xx / (5 + b)) + 200 * np.cos(yy / 7) + 3 * xx
        for t in range(T):
            c[t, :, :, b] = base + 20 * t + rng.normal(0, 15, (H, W))
    return np.clip(np.round(c), 0, 4000).astype(dtype)


def _params(**kw):
    d = dict(bit_depth=12, qp=22, block=8, search_range=4, gop=3, intra=1)
    d.update(kw)
    return O.CodingParams(**d)


@pytest.mark.parametrize("N,bands,pad", [(4, 3, 0), (8, 4, 0), (16, 3, 0), (32, 2, 0),
                                         (8, 4, 1), (16, 5, 1)])
def test_mode_choice_by_brute_force(N, bands, pad):
    # with PAD_REPEAT the padding channels copy a real band: they must not
    # count twice in the choice
    cube = _cube(T=4, H=70, W=90, bands=bands, seed=N)
    p = _params(block=N, pad_mode=pad)
    enc = O.encode_cube(cube, p)
    G = enc["frames"].shape[0]
    Hb, Wb = enc["mvs"].shape[2:4]
    B = p.bit_depth
    seen = set()
    for g in range(G):
        nch = min(3, bands - 3 * g)
        for t in range(0, cube.shape[0], p.gop):
            cur = enc["frames"][g, t].astype(np.int64)
            rec = enc["recon"][g, t]
            for by in range(Hb):
                for bx in range(Wb):
                    preds = [[O.intra_predict(_refs_brute(rec[c], N, B, bx, by), N, m, B)
                              for c in range(3)] for m in (0, 1)]
                    ys, xs = slice(by * N, by * N + N), slice(bx * N, bx * N + N)
                    cost = [sum(int(np.abs(cur[c, ys, xs] - preds[m][c]).sum())
                                for c in range(nch)) for m in (0, 1)]
                    mode = 1 if cost[1] < cost[0] else 0
                    assert enc["mvs"][g, t, by, bx, 0] == mode, (g, t, bx, by, cost)
                    assert enc["mvs"][g, t, by, bx, 1] == 0
                    assert enc["mv_bits"][g, t, by, bx] == 1
                    seen.add(mode)
                    c = (bx + by) % 3
                    r = (cur[c, ys, xs] - preds[mode][c]).astype(np.int32)
                    lev = O.quantize(O.forward_transform(r, B), B, p.qp, True)
                    assert (enc["levels"][g, t, c, by, bx] == lev).all(), (g, t, c, bx, by)
    assert seen == {0, 1}


@pytest.mark.parametrize("N", [4, 8, 16, 32])
@pytest.mark.parametrize("B", [8, 10, 12])
def test_decode_reproduces_the_reconstruction(N, B):
    cube = _cube(T=7, H=45, W=70, bands=4, seed=B)
    cube = np.minimum(cube, (1 << B) - 1).astype(np.uint16)
    for qpel in (0, 1):
        p = _params(block=N, bit_depth=B, qpel=qpel)
        enc = O.encode_cube(cube, p)
        rec = O.decode_cube(p, cube.shape, enc["levels"], enc["mvs"])
        assert (rec == enc["recon"]).all()


def test_first_block_matches_the_mid_level_prediction():
    cube = _cube(T=3, H=32, W=32, seed=4)
    for N in (4, 8, 16, 32):
        a = O.encode_cube(cube, _params(block=N, intra=1))
        b = O.encode_cube(cube, _params(block=N, intra=0))
        assert (a["levels"][:, 0, :, 0, 0] == b["levels"][:, 0, :, 0, 0]).all()
        assert (a["mvs"][:, 0, 0, 0] == 0).all()
        # P pictures after it see a different reference: no equality asked
        assert (b["mv_bits"][:, 0] == 0).all() and (a["mv_bits"][:, 0] == 1).all()


def test_intra_prediction_lowers_the_bits_of_smooth_pictures():
    # a smooth, noise-free picture at small N: predicting each block from its
    # neighbours costs clearly fewer bits than coding it against the constant
    # mid-level (the mode is chosen by SAD, not by bits, so no such bound is
    # asked at large N or for the squared error)
    H = W = 64
    yy, xx = np.mgrid[0:H, 0:W]
    c = np.stack([600 + 400 * np.sin(xx / 9.0) + 300 * np.cos(yy / 11.0) + 4 * xx + 2 * yy
                  + 50 * b for b in range(3)], -1)[None]
    cube = np.round(c).astype(np.uint16)
    for N in (4, 8):
        for qp in (22, 32):
            a = O.encode_cube(cube, _params(block=N, intra=1, gop=1, qp=qp))
            b = O.encode_cube(cube, _params(block=N, intra=0, gop=1, qp=qp))
            bits_a = int(a["coef_bits"].sum() + a["mv_bits"].sum())
            assert bits_a < 0.85 * int(b["coef_bits"].sum()), (N, qp)


def test_bitstream_carries_the_modes():
    cube = _cube(T=5, H=40, W=48, bands=4, seed=6)
    p = _params(block=8, gop=2)
    enc = O.encode_cube(cube, p)
    w = O.write_bitstream(enc["levels"], enc["mvs"], p.gop, imodes=1)
    assert w["bits"] == int(enc["coef_bits"].sum() + enc["mv_bits"].sum())
    r = O.read_bitstream(w["payload"], w["bits"], enc["levels"].shape, p.gop, imodes=1)
    assert (r["levels"] == enc["levels"]).all()
    assert (r["mvs"] == enc["mvs"]).all()
    assert (r["index"] == w["index"]).all()
    # without the mode bits the stream is shorter by one bit per I block
    w0 = O.write_bitstream(enc["levels"], enc["mvs"], p.gop, imodes=0)
    G, T, Hb, Wb = enc["mvs"].shape[:4]
    n_i = G * len(range(0, T, p.gop)) * Hb * Wb
    assert w["bits"] - w0["bits"] == n_i


def test_intra_flag_is_checked():
    with pytest.raises(ValueError):
        O.encode_cube(_cube(T=2, H=16, W=16), _params(intra=2))
