"""CPU pins of the oracle's adaptive block size of P pictures (a block of
size N coded whole or as four N/2 blocks, chosen by SAD + lambda * bits).

What pins it, none of it derived from the oracle's split code:
- the cost multiplier against hand-worked values (tests/golden/
  split_lambda.txt) and its doubling every 6 QP steps;
- the choice recomputed here for every block of small cubes: candidate
  vectors from the full search (itself pinned by brute force elsewhere), the
  costs J = 16 SAD + lambda16 (bits of each vector against zero), a tie kept
  whole; the vector field on the N/2 grid; the vector bits of each block
  (split flag + each coded vector against the cell to its left); the levels
  of each coded block as the transform and quantiser of its residual against
  the displaced previous reconstruction;
- planted motion: four cells of a block moving apart are split with their
  own vectors at low QP; a static picture stays whole;
- the coding loop: decode reproduces the reconstruction; the bitstream round
  trip restores levels, vectors and split flags, and its length is the sum of
  the bit counts;
- the tool is refused at N = 4, with quarter-sample vectors and with intra
  modes.
"""
import os

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "split_lambda.txt")


def test_lambda_worked_values():
    n = 0
    for line in open(GOLD):
        t = line.split("#")[0].split()
        if t and t[0] == "lambda":
            qp, B, v = int(t[1]), int(t[2]), int(t[3])
            assert O.split_lambda(qp, B) == v, (qp, B)
            n += 1
    assert n == 8
    for qP in range(0, 70):
        a = O.split_lambda(qP, 8)
        b = O.split_lambda(qP + 6, 8)
        assert abs(b - 2 * a) <= 1 and O.split_lambda(qP + 1, 8) >= a


def test_choice_on_crafted_costs():
    zero = [(0, 0)] * 4
    # J = 16 SAD + lambda16 * bits, every vector against (0, 0): (0,0) costs
    # 2 bits, (1,0) and (0,-1) 4, (2,-1) 5 + 3 = 8
    # whole 16*100 + 2 lam; split 16*94 + 8 lam: equal at lam = 16 -> whole
    assert O.split_choose(100, (0, 0), [20, 20, 20, 34], zero, 16) == 0
    assert O.split_choose(100, (0, 0), [20, 20, 20, 34], zero, 15) == 1
    # the whole vector costs 4 bits: 1600 + 4 lam vs 1504 + 8 lam, equal at 24
    assert O.split_choose(100, (1, 0), [20, 20, 20, 34], zero, 24) == 0
    assert O.split_choose(100, (1, 0), [20, 20, 20, 34], zero, 23) == 1
    # split vectors' bits: (2,-1) 8 bits, (0,-1) 4: 16*90 + (8 + 4 + 2 + 2) lam
    # = 1440 + 16 lam vs 1600 + 2 lam: split iff 14 lam < 160, lam <= 11
    cells = [(2, -1), (0, -1), (0, 0), (0, 0)]
    assert O.split_choose(100, (0, 0), [20, 20, 20, 30], cells, 11) == 1
    assert O.split_choose(100, (0, 0), [20, 20, 20, 30], cells, 12) == 0


def _cube(T, H, W, Bn, seed, motion=True):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 3000, (H + 24, W + 24, Bn)).astype(np.float64)
    base = (base + np.roll(base, 1, 0) + np.roll(base, 1, 1)) / 3
    frames = []
    for t in range(T):
        sy, sx = ((t * 2) % 5 - 2, (t * 3) % 7 - 3) if motion else (0, 0)
        frames.append(np.roll(base, (sy, sx), (0, 1))[:H, :W] + rng.normal(0, 20, (H, W, Bn)))
    return np.clip(np.round(np.stack(frames)), 0, 65535).astype(np.uint16)


def _params(**kw):
    d = dict(bit_depth=10, qp=22, block=8, search_range=3, gop=4, split=1)
    d.update(kw)
    return O.CodingParams(**d)


def _recompute_gop_frame(enc, p, g, t, nch):
    """The choice, vectors, vector bits and levels of P frame t recomputed."""
    N, h, R, B = p.block, p.block // 2, p.search_range, p.bit_depth
    cur = enc["frames"][g, t]
    ref = enc["recon"][g, t - 1]
    _, Hp, Wp = cur.shape
    Hb, Wb = Hp // N, Wp // N
    lam = O.split_lambda(p.qp, B)
    mvu = np.zeros((2 * Hb, 2 * Wb, 2), np.int64)
    splits = np.zeros((Hb, Wb), np.uint8)
    choice = {}
    for by in range(Hb):
        for bx in range(Wb):
            vx, vy, sad = O.motion_search(cur, ref, N, R, bx, by, nch)
            jw = 16 * sad + lam * O.mv_bits(vx, vy, 0, 0)
            cells = [O.motion_search(cur, ref, h, R, 2 * bx + (i & 1), 2 * by + (i >> 1), nch)
                     for i in range(4)]
            js = sum(16 * c[2] + lam * O.mv_bits(c[0], c[1], 0, 0) for c in cells)
            sp = js < jw
            splits[by, bx] = sp
            for i in range(4):
                v = cells[i][:2] if sp else (vx, vy)
                mvu[2 * by + (i >> 1), 2 * bx + (i & 1)] = v
            choice[(bx, by)] = (sp, (vx, vy), [c[:2] for c in cells])
    mbits = np.zeros((Hb, Wb), np.int64)
    for by in range(Hb):
        for bx in range(Wb):
            sp = splits[by, bx]
            b = 1
            for i in range(4 if sp else 1):
                xu, yu = 2 * bx + (i & 1), 2 * by + (i >> 1)
                pm = mvu[yu, xu - 1] if xu > 0 else (0, 0)
                b += O.mv_bits(int(mvu[yu, xu, 0]), int(mvu[yu, xu, 1]), int(pm[0]), int(pm[1]))
            mbits[by, bx] = b
    return splits, mvu, mbits, choice


@pytest.mark.parametrize("N,bands,qp", [(8, 3, 22), (16, 4, 30), (32, 2, 17), (8, 5, 37)])
def test_choice_vectors_bits_and_levels_recomputed(N, bands, qp):
    cube = _cube(5, 2 * N + 9, 3 * N + 5, bands, seed=N + qp)
    p = _params(block=N, qp=qp, search_range=3)
    enc = O.encode_cube(cube, p)
    G = enc["frames"].shape[0]
    h, B = N // 2, p.bit_depth
    seen = set()
    for g in range(G):
        nch = min(3, bands - 3 * g)
        for t in range(cube.shape[0]):
            if t % p.gop == 0:
                assert (enc["splits"][g, t] == 0).all() and (enc["mvs"][g, t] == 0).all()
                assert (enc["mv_bits"][g, t] == 0).all()
                continue
            splits, mvu, mbits, choice = _recompute_gop_frame(enc, p, g, t, nch)
            assert (enc["splits"][g, t] == splits).all(), (g, t)
            assert (enc["mvs"][g, t] == mvu).all(), (g, t)
            assert (enc["mv_bits"][g, t] == mbits).all(), (g, t)
            seen |= set(splits.ravel().tolist())
            cur = enc["frames"][g, t].astype(np.int64)
            ref = enc["recon"][g, t - 1].astype(np.int64)
            Hb, Wb = splits.shape
            for by in range(Hb):
                for bx in range(Wb):
                    c = (bx + 2 * by) % 3
                    lev = enc["levels"][g, t, c, by, bx].reshape(-1)
                    blocks = ([(bx * N, by * N, N, mvu[2 * by, 2 * bx])] if not splits[by, bx]
                              else [(bx * N + (i & 1) * h, by * N + (i >> 1) * h, h,
                                     mvu[2 * by + (i >> 1), 2 * bx + (i & 1)]) for i in range(4)])
                    off = 0
                    bits = 0
                    for x0, y0, n, v in blocks:
                        r = cur[c, y0:y0 + n, x0:x0 + n] - \
                            ref[c, y0 + v[1]:y0 + v[1] + n, x0 + v[0]:x0 + v[0] + n]
                        want = O.quantize(O.forward_transform(r.astype(np.int32), B), B, qp, False)
                        assert (lev[off:off + n * n].reshape(n, n) == want).all(), (g, t, bx, by)
                        bits += O.coef_bits(want)
                        off += n * n
                    assert enc["coef_bits"][g, t, c, by, bx] == bits
    assert seen == {0, 1}, seen


def test_planted_cell_motion_splits_and_static_stays_whole():
    N, h = 16, 8
    rng = np.random.default_rng(9)
    H = W = 48
    tex = rng.integers(0, 4000, (H + 16, W + 16, 3)).astype(np.float64)
    f0 = tex[8:8 + H, 8:8 + W]
    f1 = f0.copy()
    # block (1, 1): its four cells move by different vectors
    offs = [(2, 1), (-2, 0), (1, -2), (-1, 2)]
    for i, (dx, dy) in enumerate(offs):
        y0, x0 = N + (i >> 1) * h, N + (i & 1) * h
        f1[y0:y0 + h, x0:x0 + h] = tex[8 + y0 + dy:8 + y0 + dy + h, 8 + x0 + dx:8 + x0 + dx + h]
    cube = np.round(np.stack([f0, f1])).astype(np.uint16)
    enc = O.encode_cube(cube, _params(block=N, qp=-12, search_range=3, gop=2, bit_depth=10))
    assert enc["splits"][0, 1, 1, 1] == 1
    for i, (dx, dy) in enumerate(offs):
        assert tuple(enc["mvs"][0, 1, 2 + (i >> 1), 2 + (i & 1)]) == (dx, dy)
    # a static picture: every vector zero, nothing split
    still = np.round(np.stack([f0, f0, f0])).astype(np.uint16)
    enc = O.encode_cube(still, _params(block=N, qp=22, search_range=3, gop=3))
    assert (enc["splits"] == 0).all() and (enc["mvs"] == 0).all()


@pytest.mark.parametrize("N", [8, 16, 32])
def test_decode_and_bitstream_round_trip(N):
    cube = _cube(7, 45, 70, 4, seed=N)
    p = _params(block=N, gop=3, search_range=4)
    enc = O.encode_cube(cube, p)
    rec = O.decode_cube(p, cube.shape, enc["levels"], enc["mvs"], enc["splits"])
    assert (rec == enc["recon"]).all()
    w = O.write_bitstream(enc["levels"], enc["mvs"], p.gop, splits=enc["splits"])
    assert w["bits"] == int(enc["coef_bits"].sum() + enc["mv_bits"].sum())
    r = O.read_bitstream(w["payload"], w["bits"], enc["levels"].shape, p.gop, split=1)
    for k in ("levels", "mvs", "splits"):
        assert (r[k] == enc[k]).all(), k
    assert (r["index"] == w["index"]).all()


def test_split_lowers_the_cost_of_mixed_motion():
    # cells moving apart: the adaptive size codes the P pictures in fewer bits
    cube = _cube(6, 64, 64, 3, seed=3)
    rng = np.random.default_rng(4)
    for t in range(1, 6):
        for _ in range(12):
            y, x = rng.integers(0, 56, 2)
            cube[t, y:y + 8, x:x + 8] = np.roll(cube[t], (int(rng.integers(-2, 3)), 1),
                                               (0, 1))[y:y + 8, x:x + 8]
    a = O.encode_cube(cube, _params(block=16, split=1, gop=6, search_range=4))
    b = O.encode_cube(cube, _params(block=16, split=0, gop=6, search_range=4))
    bits = lambda e: int(e["coef_bits"][:, 1:].sum() + e["mv_bits"][:, 1:].sum())
    assert bits(a) < bits(b)
    assert a["splits"].any()


def test_split_is_refused_where_undefined():
    cube = _cube(2, 16, 16, 3, seed=1)
    for kw in (dict(block=4), dict(qpel=1), dict(intra=1), dict(split=2)):
        with pytest.raises(ValueError):
            O.encode_cube(cube, _params(**kw))
