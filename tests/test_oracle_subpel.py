"""CPU pins of the oracle's quarter-sample motion (interpolation, refinement,
and the coding loop with quarter-sample vectors).

What pins it, none of it derived from the oracle itself:
- the H.265 luma filter table typed from the standard (tests/golden/
  hevc_luma_interp.txt), and properties of a filter table: each row sums to
  64, the half-sample row is symmetric, the quarter rows mirror each other,
  the first moments are 15, 32 and 49;
- hand-worked predicted samples with their intermediate values written out
  (ramps, an impulse, a negative lobe, the final clip), same file;
- closed forms: a constant plane predicts the constant at every phase and bit
  depth; integer positions reproduce the reference sample;
- the clamp to the picture: predictions near the border equal predictions at
  the same phase inside a plane padded by edge replication (numpy);
- an independent vectorised separable filter (numpy), all 16 phases, random
  planes, interior positions;
- brute force over the refinement's candidate sets with the lexicographic key,
  and a planted quarter-sample displacement found with zero SAD;
- the coding loop: decode reproduces the encoder's reconstruction, vector bits
  are the Exp-Golomb lengths of the quarter-sample differences, R > 31 is
  refused.
"""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "hevc_luma_interp.txt")


def _golden():
    filt, cases = {}, []
    for line in open(GOLD):
        line = line.split("#")[0].strip()
        if not line:
            continue
        tok = line.split()
        if tok[0] == "filter":
            filt[int(tok[1])] = [int(v) for v in tok[2:]]
        elif tok[0] == "case":
            cases.append((tok[1], int(tok[2]), tok[3], int(tok[4]), int(tok[5]), int(tok[6])))
    return filt, cases


def _plane(spec, B, size=48):
    L = (1 << B) - 1
    m = re.match(r"(\w+)\(([-\d,]+)\)", spec)
    kind, args = m.group(1), [int(v) for v in m.group(2).split(",")]
    y, x = np.mgrid[0:size, 0:size]
    if kind == "ramp":
        a, b, c = args
        p = a + b * x + c * y
    else:
        bg, peak, x0, y0 = args
        p = np.full((size, size), bg)
        p[y0, x0] = peak
    return np.clip(p, 0, L).astype(np.uint16)


def test_filter_table_is_the_standards():
    filt, _ = _golden()
    for p in (1, 2, 3):
        assert [O.luma_filter(p, i) for i in range(8)] == filt[p]
    assert [O.luma_filter(0, i) for i in range(8)] == [0, 0, 0, 64, 0, 0, 0, 0]
    # properties of the typed table itself
    for p in (1, 2, 3):
        assert sum(filt[p]) == 64
    assert filt[2] == filt[2][::-1]
    assert filt[3] == filt[1][::-1]
    assert [sum(f * (i - 3) for i, f in enumerate(filt[p])) for p in (1, 2, 3)] == [15, 32, 49]


@pytest.mark.parametrize("case", _golden()[1], ids=lambda c: c[0])
def test_hand_worked_predicted_samples(case):
    name, B, spec, xq, yq, expect = case
    assert O.interp_sample(_plane(spec, B), B, xq, yq) == expect


@pytest.mark.parametrize("B", [8, 10, 12])
def test_constant_plane_and_integer_positions(B):
    rng = np.random.default_rng(B)
    L = (1 << B) - 1
    for v in (0, 1, L // 3, L):
        plane = np.full((20, 24), v, np.uint16)
        for xq in range(-9, 4 * 24 + 9, 3):
            for yq in range(-9, 4 * 20 + 9, 5):
                assert O.interp_sample(plane, B, xq, yq) == v
    plane = rng.integers(0, L + 1, (20, 24)).astype(np.uint16)
    for x in range(24):
        for y in range(20):
            assert O.interp_sample(plane, B, 4 * x, 4 * y) == plane[y, x]


def _numpy_interp(plane, B, fx, fy):
    """Independent vectorised form: the separable filter over a plane padded
    by edge replication; returns the predicted sample at (4x + fx, 4y + fy)
    for every (y, x) of the plane."""
    filt, _ = _golden()
    filt[0] = [0, 0, 0, 64, 0, 0, 0, 0]
    H, W = plane.shape
    P = np.pad(plane.astype(np.int64), 4, mode="edge")  # P[y + 4, x + 4] = plane[y, x] clamped
    s1, s3 = B - 8, 14 - B

    def hpass(rows):  # rows: slice of P rows; horizontal taps at x + i - 3
        return sum(filt[fx][i] * rows[:, 1 + i: 1 + i + W] for i in range(8))

    if fx == 0 and fy == 0:
        pred = P[4:4 + H, 4:4 + W] << s3
    elif fy == 0:
        pred = hpass(P[4:4 + H]) >> s1
    elif fx == 0:
        pred = sum(filt[fy][i] * P[1 + i: 1 + i + H, 4:4 + W] for i in range(8)) >> s1
    else:
        tmp = hpass(P) >> s1  # all padded rows
        pred = sum(filt[fy][i] * tmp[1 + i: 1 + i + H] for i in range(8)) >> 6
    w = 14 - B
    return np.clip((pred + (1 << (w - 1))) >> w, 0, (1 << B) - 1)


@pytest.mark.parametrize("B", [8, 10, 12])
def test_against_an_independent_separable_filter(B):
    rng = np.random.default_rng(100 + B)
    plane = rng.integers(0, 1 << B, (13, 17)).astype(np.uint16)
    for fy in range(4):
        for fx in range(4):
            ref = _numpy_interp(plane, B, fx, fy)
            got = np.array([[O.interp_sample(plane, B, 4 * x + fx, 4 * y + fy) for x in range(17)]
                            for y in range(13)])
            assert np.array_equal(got, ref), (fx, fy)


def test_border_clamp_equals_edge_replication():
    """Positions outside the picture read the nearest edge sample: the same
    prediction as inside a plane explicitly padded by replication."""
    B = 10
    rng = np.random.default_rng(7)
    plane = rng.integers(0, 1024, (12, 16)).astype(np.uint16)
    pad = 9
    big = np.pad(plane, pad, mode="edge")
    for yq in range(-4 * 6, 4 * 18, 3):
        for xq in range(-4 * 6, 4 * 22, 5):
            a = O.interp_sample(plane, B, xq, yq)
            b = O.interp_sample(big, B, xq + 4 * pad, yq + 4 * pad)
            assert a == b, (xq, yq)


def _brute_refine(cur, ref, N, B, bx, by, dx, dy, nch):
    """Both refinement stages by enumeration: every candidate of a stage, the
    minimum of (SAD, |mx| + |my|, my, mx) taken by sorting."""
    x0, y0 = bx * N, by * N

    def sad(mx, my):
        s = 0
        for c in range(nch):
            for i in range(N):
                for j in range(N):
                    p = O.interp_sample(ref[c], B, 4 * (x0 + j) + mx, 4 * (y0 + i) + my)
                    s += abs(int(cur[c, y0 + i, x0 + j]) - p)
        return s

    cx, cy = 4 * dx, 4 * dy
    for step in (2, 1):
        keys = sorted((sad(cx + ox, cy + oy), abs(cx + ox) + abs(cy + oy), cy + oy, cx + ox)
                      for oy in (-step, 0, step) for ox in (-step, 0, step))
        best = keys[0]
        cx, cy = best[3], best[2]
    return cx, cy, best[0]


@pytest.mark.parametrize("N,B,nch", [(4, 8, 3), (4, 10, 1), (8, 12, 2)])
def test_refinement_is_the_minimum_of_each_stage(N, B, nch):
    rng = np.random.default_rng(N * 10 + B)
    H = W = 4 * N
    # smooth content so that sub-sample positions matter, plus noise for ties
    yy, xx = np.mgrid[0:H, 0:W]
    base = (0.4 * (1 << B)) * (1 + np.sin(xx / 3.1 + yy / 4.3)) / 2
    ref = np.stack([np.clip(base + rng.normal(0, 3, (H, W)) + 40 * c, 0, (1 << B) - 1)
                    for c in range(3)]).astype(np.uint16)
    cur = np.stack([np.clip(np.roll(ref[c].astype(float), (1, 2), (0, 1)) * 0.5 +
                            0.5 * np.roll(ref[c].astype(float), (1, 1), (0, 1)), 0, (1 << B) - 1)
                    for c in range(3)]).astype(np.uint16)
    for bx in range(W // N):
        for by in range(H // N):
            for dx, dy in ((0, 0), (1, -1), (-2, 1)):
                got = O.subpel_refine(cur, ref, N, B, bx, by, dx, dy, nch)
                assert got == _brute_refine(cur, ref, N, B, bx, by, dx, dy, nch), (bx, by, dx, dy)


def test_flat_reference_keeps_the_integer_vector():
    """All candidates tie on a flat picture; the key's L1 term keeps the
    centre when it is (0, 0), else moves towards (0, 0)."""
    B, N = 10, 8
    ref = np.full((3, 16, 16), 300, np.uint16)
    cur = np.full((3, 16, 16), 310, np.uint16)
    assert O.subpel_refine(cur, ref, N, B, 0, 0, 0, 0) == (0, 0, 3 * 64 * 10)
    # from (1, 0): half stage reaches (2, 0) (L1 2), quarter stage (1, 0) (L1 1)
    assert O.subpel_refine(cur, ref, N, B, 0, 0, 1, 0)[:2] == (1, 0)


def test_planted_quarter_sample_displacement_is_found():
    """A current block made of the prediction at a known quarter-sample
    vector is found with SAD 0 by the integer search plus refinement."""
    B, N, R = 10, 8, 4
    rng = np.random.default_rng(3)
    H = W = 32
    ref = rng.integers(0, 1024, (3, H, W)).astype(np.uint16)
    for (mx, my) in ((5, -3), (-6, 7), (2, 2), (-1, -9)):
        cur = ref.copy()
        bx, by = 1, 2
        for c in range(3):
            for i in range(N):
                for j in range(N):
                    cur[c, by * N + i, bx * N + j] = O.interp_sample(
                        ref[c], B, 4 * (bx * N + j) + mx, 4 * (by * N + i) + my)
        dx, dy, _ = O.motion_search(cur, ref, N, R, bx, by)
        got = O.subpel_refine(cur, ref, N, B, bx, by, dx, dy)
        # random texture: the integer search lands next to the true vector
        if abs(4 * dx - mx) <= 2 and abs(4 * dy - my) <= 2:
            assert got == (mx, my, 0), (mx, my, dx, dy, got)


def _tiny_cube(seed, T=6, H=24, W=40, Bn=4):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    frames = []
    for t in range(T):
        f = [2000 + 900 * np.sin((xx + 0.7 * t) / 4.0 + b) * np.cos((yy - 0.4 * t) / 5.0)
             + rng.normal(0, 20, (H, W)) for b in range(Bn)]
        frames.append(np.stack(f, -1))
    return np.clip(np.stack(frames), 0, 65535).round().astype(np.uint16)


@pytest.mark.parametrize("N,B,R", [(4, 10, 3), (8, 8, 5), (16, 12, 2)])
def test_coding_loop_with_quarter_sample_vectors(N, B, R):
    cube = _tiny_cube(N + B)
    p = O.CodingParams(bit_depth=B, qp=22, block=N, search_range=R, gop=4, qpel=1)
    enc = O.encode_cube(cube, p)
    mvs = enc["mvs"].astype(int)
    assert np.abs(mvs).max() <= 4 * R + 3
    # some vectors are not whole samples
    assert (mvs % 4 != 0).any()
    rec = O.decode_cube(p, cube.shape, enc["levels"], enc["mvs"])
    assert np.array_equal(rec, enc["recon"])
    # vector bits: se lengths of the differences to the left neighbour, quarter samples
    G, T, Hb, Wb, _ = mvs.shape
    for g in range(G):
        for t in range(T):
            if t % p.gop == 0:
                assert not enc["mv_bits"][g, t].any()
                continue
            for by in range(Hb):
                pmx = pmy = 0
                for bx in range(Wb):
                    mx, my = mvs[g, t, by, bx]
                    want = O.se_len(mx - pmx) + O.se_len(my - pmy)
                    assert enc["mv_bits"][g, t, by, bx] == want
                    pmx, pmy = mx, my
    # integer-sample coding of the same cube differs (the tool changes the output)
    q = O.CodingParams(bit_depth=B, qp=22, block=N, search_range=R, gop=4, qpel=0)
    assert not np.array_equal(O.encode_cube(cube, q)["mvs"], enc["mvs"])


def test_quarter_sample_needs_search_range_at_most_31():
    cube = _tiny_cube(1, T=2, H=16, W=16, Bn=3)
    with pytest.raises(ValueError):
        O.encode_cube(cube, O.CodingParams(bit_depth=10, qp=22, block=8, search_range=32,
                                           gop=2, qpel=1))
    O.encode_cube(cube, O.CodingParams(bit_depth=10, qp=22, block=8, search_range=31,
                                       gop=2, qpel=1))


def test_equal_sad_and_l1_break_ties_on_my_then_mx():
    """On a picture that is a function of x + y, the half-sample candidates
    (2, 0) and (0, 2) predict the same samples; with the block equal to that
    prediction both have SAD 0 and L1 2, and the key prefers the smaller my."""
    B, N = 10, 8
    rng = np.random.default_rng(11)
    H = W = 24
    g = rng.integers(100, 900, H + W)
    yy, xx = np.mgrid[0:H, 0:W]
    ref = np.stack([g[xx + yy] + 10 * c for c in range(3)]).astype(np.uint16)
    bx, by = 1, 1
    for planted in ((2, 0), (-2, 0)):
        cur = ref.copy()
        for c in range(3):
            for i in range(N):
                for j in range(N):
                    cur[c, by * N + i, bx * N + j] = O.interp_sample(
                        ref[c], B, 4 * (bx * N + j) + planted[0], 4 * (by * N + i) + planted[1])
        swapped = (planted[1], planted[0])
        assert O.subpel_refine(cur, ref, N, B, bx, by, 0, 0)[2] == 0
        # (0, 2) / (0, -2) predict the same block
        assert O.subpel_refine(cur, ref, N, B, bx, by, 0, 0)[:2] == min(planted, swapped,
                                                                         key=lambda v: (v[1], v[0]))
