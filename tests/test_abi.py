"""The C-ABI library loads and exports every symbol include/xv.h declares;
argument validation is host-only and is checked here without a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "xv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xv_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def xvmod():
    from paper_2506_19656_amd import xv
    if not os.path.exists(xv.LIB_PATH):
        from paper_2506_19656_amd import build
        build.build(verbose=False)
    xv.lib()
    return xv


def test_every_declared_symbol_is_exported(xvmod):
    names = _declared()
    assert len(names) >= 14
    lib = C.CDLL(xvmod.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(xvmod.EXPORTED) <= set(names)


def test_abi_version_and_status_strings(xvmod):
    L = xvmod.lib()
    assert L.xv_abi_version() == 8
    assert L.xv_status_str(0) == b"ok"
    assert L.xv_status_str(-1) == b"invalid argument"


def _cube(xv, data=1 << 20, dtype=0, T=4, H=16, W=16, Bn=3):
    return xv.Cube(C.c_void_p(data), dtype, 0, T, H, W, Bn)


@pytest.mark.parametrize("field,value", [("bit_depth", 7), ("bit_depth", 13), ("block", 12),
                                         ("block", 64), ("qp", 52), ("qp", -13),
                                         ("search_range", 65), ("search_range", -1),
                                         ("gop", 0), ("pad_mode", 2), ("fill_mode", 5),
                                         ("flags", 16)])
def test_invalid_params_are_rejected_before_any_device_work(xvmod, field, value):
    p = xvmod.Params(bit_depth=10, qp=27, block=8, search_range=8, gop=16)
    setattr(p, field, value)
    pc = p.c()
    cb = _cube(xvmod)
    h = C.c_void_p(123)
    rc = xvmod.lib().xv_encode_cube(C.byref(cb), C.byref(pc), None, C.byref(h))
    assert rc == xvmod.EINVAL
    assert h.value is None  # *out is NULL on error
    assert xvmod.lib().xv_last_error()


@pytest.mark.parametrize("kw", [dict(data=0), dict(dtype=7), dict(T=0), dict(H=-1),
                                dict(Bn=65), dict(data=(1 << 20) + 1)])
def test_invalid_cubes_are_rejected(xvmod, kw):
    p = xvmod.Params().c()
    cb = _cube(xvmod, **kw)
    h = C.c_void_p()
    rc = xvmod.lib().xv_encode_cube(C.byref(cb), C.byref(p), None, C.byref(h))
    assert rc == xvmod.EINVAL


def test_null_handles(xvmod):
    L = xvmod.lib()
    assert L.xv_encode_cube(None, None, None, None) == xvmod.EINVAL
    assert L.xv_decode_cube(None, None, None) == xvmod.EINVAL
    m = xvmod.MetricsC()
    assert L.xv_psnr_bpppb(None, None, C.byref(m), None) == xvmod.EINVAL
    ms = (xvmod.MetricsC * 2)()
    assert L.xv_psnr_bpppb_batch(0, None, None, ms, None) == xvmod.EINVAL
    assert L.xv_psnr_bpppb_batch(2, None, None, ms, None) == xvmod.EINVAL
    hs = (C.c_void_p * 2)(None, None)
    assert L.xv_psnr_bpppb_batch(2, None, hs, ms, None) == xvmod.EINVAL
    L.xv_encoded_free(None)  # no-op


def test_me_geometry_validation(xvmod):
    col, row = xvmod.ME_COLUMN_PAIRS, xvmod.ME_ROW_PAIRS
    bad = [dict(cands_per_lane=3, rows_per_lane=1, layout=col),   # column pairs: even counts
           dict(cands_per_lane=2, rows_per_lane=4, layout=col),   # no 4-row instance
           dict(cands_per_lane=6, rows_per_lane=5, layout=col),   # 5 rows: 2 or 4 columns
           dict(cands_per_lane=10, rows_per_lane=1, layout=row),  # row pairs: 2..9, 11, 13
           dict(cands_per_lane=3, rows_per_lane=2, layout=row),   # row pairs: one row
           dict(cands_per_lane=3, rows_per_lane=1, layout=4),     # no such layout
           dict(blocks_per_wg=16, cands_per_lane=2, threads=64, rows_per_lane=1,
                layout=xvmod.ME_ROW_PAIRS_BY_CHANNEL),            # items > 3 rounds
           dict(threads=1024), dict(threads=96), dict(blocks_per_wg=65)]
    for kw in bad:
        with pytest.raises(xvmod.XvError):
            xvmod.set_me_geometry(8, 8, **kw)
    with pytest.raises(xvmod.XvError):
        xvmod.set_me_geometry(12, 8)
    try:
        xvmod.set_me_geometry(8, 8, 3, 11, 192, 1, row)
        assert xvmod.get_me_geometry(8, 8) == dict(blocks_per_wg=3, cands_per_lane=11, threads=192,
                                                  rows_per_lane=1, layout=row)
        xvmod.set_me_geometry(8, 8, 2, 6, 256, 3, col)
        assert xvmod.get_me_geometry(8, 8)["layout"] == col
    finally:
        xvmod.set_me_geometry(8, 8)
    for N in (4, 8, 16, 32):
        g = xvmod.get_me_geometry(N, 16)
        assert g["threads"] % 64 == 0 and g["blocks_per_wg"] >= 1
        if g["layout"] == col:
            assert g["cands_per_lane"] % 2 == 0 and g["rows_per_lane"] in (1, 2, 3, 5)
        else:
            assert g["layout"] in (row, xvmod.ME_ROW_PAIRS_BY_CHANNEL) and g["rows_per_lane"] == 1
            assert g["cands_per_lane"] in (2, 3, 4, 5, 6, 7, 8, 9, 11, 13)


def test_me_split_geometry_validation(xvmod):
    col, row, byc = xvmod.ME_COLUMN_PAIRS, xvmod.ME_ROW_PAIRS, xvmod.ME_ROW_PAIRS_BY_CHANNEL
    bad = [dict(cands_per_lane=6, rows_per_lane=1, layout=col),   # row-pair layouts only
           dict(cands_per_lane=9, rows_per_lane=1, layout=row),   # 5, 7, 11 or 13 candidates
           dict(cands_per_lane=5, rows_per_lane=2, layout=row),   # one row
           # by channel, 13 candidates: 65 x 5 = 325 items per block, one round
           dict(blocks_per_wg=1, cands_per_lane=13, threads=256, rows_per_lane=1, layout=byc),
           # 5 candidates: 65 x 13 = 845 items per block, two rounds
           dict(blocks_per_wg=1, cands_per_lane=5, threads=384, rows_per_lane=1, layout=byc),
           dict(threads=1024), dict(blocks_per_wg=65)]
    for kw in bad:
        with pytest.raises(xvmod.XvError):
            xvmod.set_me_split_geometry(16, 32, **kw)
    for N in (4, 12):  # the adaptive block size needs N >= 8
        with pytest.raises(xvmod.XvError):
            xvmod.set_me_split_geometry(N, 16)
    try:
        xvmod.set_me_split_geometry(16, 32, 1, 13, 384, 1, byc)
        assert xvmod.get_me_split_geometry(16, 32) == dict(
            blocks_per_wg=1, cands_per_lane=13, threads=384, rows_per_lane=1, layout=byc)
        xvmod.set_me_split_geometry(16, 32, 1, 5, 448, 1, byc)  # 845 <= 2 x 448
        xvmod.set_me_split_geometry(16, 32, 2, 7, 256, 1, row)
        assert xvmod.get_me_split_geometry(16, 32)["layout"] == row
        # the plain search's table is a different one
        assert xvmod.get_me_geometry(16, 32, 64)["cands_per_lane"] != 7 or \
            xvmod.get_me_geometry(16, 32, 64)["layout"] != row
    finally:
        xvmod.set_me_split_geometry(16, 32)
    for N in (8, 16, 32):
        for R in (8, 16, 32):
            g = xvmod.get_me_split_geometry(N, R, 1024 // N)
            assert g["layout"] in (row, byc) and g["rows_per_lane"] == 1
            assert g["cands_per_lane"] in (5, 7, 11, 13) and g["threads"] % 64 == 0
            # the default is one the setter accepts
            xvmod.set_me_split_geometry(N, R, g["blocks_per_wg"], g["cands_per_lane"],
                                        g["threads"], 1, g["layout"])
            xvmod.set_me_split_geometry(N, R)


def test_tuner_refuses_mixed_batches_before_any_device_work(xvmod):
    # the tuner times one search: a batch mixing the adaptive block size with
    # fixed blocks (or block sizes) is refused after validation alone
    L = xvmod.lib()
    cbs = (xvmod.Cube * 2)(_cube(xvmod), _cube(xvmod))
    for flags1, block1 in ((xvmod.FLAG_SPLIT, 16), (0, 8)):
        ps = (xvmod.ParamsC * 2)(xvmod.Params(bit_depth=10, qp=27, block=16, search_range=8,
                                              gop=16).c(),
                                 xvmod.Params(bit_depth=10, qp=27, block=block1, search_range=8,
                                              gop=16, flags=flags1).c())
        g = xvmod.MeGeometryC()
        ms = C.c_double()
        assert L.xv_autotune_me_batch(2, cbs, ps, None, 0, C.byref(g), C.byref(ms)) == xvmod.EINVAL
        assert L.xv_last_error()


def test_memory_record_and_release_without_device_work(xvmod):
    m = xvmod.memory_read()
    assert set(m) == {"live_bytes", "cached_bytes", "peak_bytes"}
    assert m["live_bytes"] <= m["peak_bytes"]
    L = xvmod.lib()
    assert L.xv_memory_read(None) == xvmod.EINVAL


def test_bitstream_entry_points_reject_bad_arguments(xvmod):
    L = xvmod.lib()
    h = C.c_void_p()
    assert L.xv_pack(None, None, C.byref(h)) == xvmod.EINVAL
    assert L.xv_pack(None, None, None) == xvmod.EINVAL
    assert L.xv_unpack(None, 0, None, C.byref(h)) == xvmod.EINVAL
    assert L.xv_unpack(C.c_void_p(16), 100, None, C.byref(h)) == xvmod.EINVAL  # < header
    assert L.xv_packed_view(None, None, None, None) == xvmod.EINVAL
    L.xv_packed_free(None)  # no-op


def test_profile_classes_match_the_header():
    import re
    from paper_2506_19656_amd import xv
    hdr = open(os.path.join(ROOT, "include", "xv.h")).read()
    n = int(re.search(r"#define XV_K_COUNT (\d+)", hdr).group(1))
    assert len(xv.K_NAMES) == n
    p = xv.ProfileC()
    assert len(p.ms) == n and len(p.launches) == n and len(p.work) == n


def test_default_geometries_are_admissible(xvmod):
    # the model's default for every block size over the search-range range is
    # a geometry the setter accepts (LDS, instances, rounds of items)
    try:
        for N in (4, 8, 16, 32):
            for R in (0, 1, 2, 5, 8, 16, 23, 32, 33, 48, 64):
                for wb in (1, 3, 16, 45):
                    g = xvmod.get_me_geometry(N, R, wb)
                    xvmod.set_me_geometry(N, R, g["blocks_per_wg"], g["cands_per_lane"],
                                          g["threads"], g["rows_per_lane"], g["layout"])
                    assert xvmod.get_me_geometry(N, R, wb) == g, (N, R, wb, g)
                    xvmod.set_me_geometry(N, R)
    finally:
        for N in (4, 8, 16, 32):
            for R in (0, 1, 2, 5, 8, 16, 23, 32, 33, 48, 64):
                xvmod.set_me_geometry(N, R)
