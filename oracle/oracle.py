"""Python access to the CPU oracle (test infrastructure only).

The oracle is the plain C implementation in ``xv_oracle.c``; this module only
marshals numpy arrays into it.  It is used by the tests, by the smoke check and
by the CPU-baseline leg of the benchmark -- never by the product library, which
shares no code with it.  Each wrapper names the C function it calls; the C
source cites the passage of the paper (or the stated reading of it) that the
step follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xv_oracle.c")
LIB = os.path.join(HERE, "libxv_oracle.so")

U16, F32 = 0, 1
PAD_ZERO, PAD_REPEAT = 0, 1
FILL_NEAREST, FILL_FORWARD = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FP contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-shared", "-fPIC", SRC, "-o", LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Params(C.Structure):
    _fields_ = [("bit_depth", C.c_int32), ("qp", C.c_int32), ("block", C.c_int32),
                ("search_range", C.c_int32), ("gop", C.c_int32),
                ("pad_mode", C.c_int32), ("fill_mode", C.c_int32), ("qpel", C.c_int32),
                ("intra", C.c_int32), ("split", C.c_int32)]


@dataclass
class CodingParams:
    bit_depth: int = 10
    qp: int = 27
    block: int = 8
    search_range: int = 8
    gop: int = 16
    pad_mode: int = PAD_ZERO
    fill_mode: int = FILL_NEAREST
    qpel: int = 0
    intra: int = 0
    split: int = 0

    def c(self) -> Params:
        return Params(self.bit_depth, self.qp, self.block, self.search_range,
                      self.gop, self.pad_mode, self.fill_mode, self.qpel, self.intra,
                      self.split)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        L = C.CDLL(LIB)
        p = C.c_void_p
        i64 = C.c_int64
        L.xvo_selfcheck.restype = C.c_int
        L.xvo_check_params.argtypes = [C.POINTER(Params)]
        L.xvo_stats.argtypes = [p, C.c_int, i64, i64, i64, i64, p, p, p]
        L.xvo_filled_value.argtypes = [p, C.c_int, i64, i64, i64, i64, i64, i64, i64,
                                       i64, C.c_int, C.c_double, C.POINTER(C.c_int)]
        L.xvo_filled_value.restype = C.c_double
        L.xvo_normalize.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
        L.xvo_normalize.restype = C.c_int32
        L.xvo_denormalize.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int]
        L.xvo_denormalize.restype = C.c_double
        L.xvo_cast_output.argtypes = [C.c_double, C.c_int]
        L.xvo_cast_output.restype = C.c_double
        L.xvo_source_band.argtypes = [i64, C.c_int, i64, C.c_int]
        L.xvo_source_band.restype = i64
        L.xvo_make_frame.argtypes = [p, C.c_int, i64, i64, i64, i64, p, p,
                                     C.POINTER(Params), i64, i64, i64, i64, p, p]
        L.xvo_dct_matrix.argtypes = [C.c_int, p]
        L.xvo_forward_transform.argtypes = [C.c_int, C.c_int, p, p]
        L.xvo_iq_scale.argtypes = [C.c_int]
        L.xvo_iq_scale.restype = C.c_int32
        L.xvo_q_scale.argtypes = [C.c_int]
        L.xvo_q_scale.restype = C.c_int32
        L.xvo_quantize.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, p, p]
        L.xvo_dequantize.argtypes = [C.c_int, C.c_int, C.c_int, p, p]
        L.xvo_inverse_transform.argtypes = [C.c_int, C.c_int, p, p]
        L.xvo_ue_len.argtypes = [C.c_uint32]
        L.xvo_se_len.argtypes = [C.c_int32]
        L.xvo_scan_order.argtypes = [C.c_int, p]
        L.xvo_coef_bits.argtypes = [C.c_int, p]
        L.xvo_coef_bits.restype = C.c_uint32
        L.xvo_mv_bits.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.xvo_mv_bits.restype = C.c_uint32
        L.xvo_motion_search.argtypes = [p, p, i64, i64, C.c_int, C.c_int, C.c_int, i64,
                                        i64, p, p, p]
        L.xvo_luma_filter.argtypes = [C.c_int, C.c_int]
        L.xvo_interp_sample.argtypes = [p, i64, i64, C.c_int, i64, i64]
        L.xvo_interp_sample.restype = C.c_int32
        L.xvo_subpel_refine.argtypes = [p, p, i64, i64, C.c_int, C.c_int, C.c_int, i64, i64,
                                        C.c_int, C.c_int, p, p, p]
        L.xvo_intra_refs.argtypes = [p, i64, i64, C.c_int, C.c_int, i64, i64, p]
        L.xvo_intra_predict.argtypes = [p, C.c_int, C.c_int, C.c_int, p]
        L.xvo_pca_moments.argtypes = [p, i64, i64, p, p]
        L.xvo_pca_eigen.argtypes = [p, i64, p, p]
        L.xvo_pca_project.argtypes = [p, i64, i64, p, p, i64, i64, p]
        L.xvo_pca_inverse.argtypes = [p, i64, i64, i64, p, p, C.c_int, p]
        L.xvo_split_lambda.argtypes = [C.c_int, C.c_int]
        L.xvo_split_lambda.restype = C.c_int32
        L.xvo_split_choose.argtypes = [C.c_uint32, C.c_int, C.c_int, p, p, p, C.c_int32]
        L.xvo_encode_gop.argtypes = [p, C.c_int, i64, i64, i64, i64, p, p,
                                     C.POINTER(Params), i64, i64, i64,
                                     p, p, p, p, p, p, p, p, p]
        L.xvo_decode_gop.argtypes = [C.POINTER(Params), i64, i64, i64, p, p, p, p]
        L.xvo_encode_cube.argtypes = [p, C.c_int, i64, i64, i64, i64, C.POINTER(Params),
                                      p, p, p, p, p, p, p, p, p, p, p]
        L.xvo_decode_cube.argtypes = [C.POINTER(Params), i64, i64, i64, i64, p, p, p, p]
        L.xvo_denormalize_cube.argtypes = [p, i64, i64, i64, i64, C.c_int, C.c_int,
                                           p, p, C.c_int, p]
        L.xvo_psnr.argtypes = [C.c_double, C.c_double, C.c_double]
        L.xvo_psnr.restype = C.c_double
        L.xvo_psnr_int.argtypes = [C.c_int, C.c_uint64, C.c_uint64]
        L.xvo_psnr_int.restype = C.c_double
        L.xvo_bpppb.argtypes = [C.c_uint64, i64, i64, i64, i64]
        L.xvo_bpppb.restype = C.c_double
        L.xvo_phys_sse.argtypes = [p, C.c_int, i64, i64, i64, i64, p, C.c_int, C.c_int,
                                   p, p, p]
        L.xvo_bitstream_bits.argtypes = [C.c_int, i64, i64, C.c_int, i64, i64, C.c_int, p, p,
                                         p]
        L.xvo_bitstream_bits.restype = C.c_uint64
        L.xvo_write_bitstream.argtypes = [C.c_int, i64, i64, C.c_int, i64, i64, C.c_int, p, p,
                                          p, p, C.c_uint64, p]
        L.xvo_read_bitstream.argtypes = [C.c_int, i64, i64, C.c_int, i64, i64, C.c_int, p, p,
                                         C.c_uint64, p, p, p]
        L.xvo_ssim_window.argtypes = [p]
        L.xvo_ssim_plane.argtypes = [p, p, i64, i64, i64, C.c_int]
        L.xvo_ssim_plane.restype = C.c_double
        L.xvo_ssim_bands.argtypes = [p, p, i64, i64, i64, i64, C.c_int, C.c_int, p]
        L.xvo_spectral_angle.argtypes = [p, C.c_int, p, C.c_int, i64, i64, i64, i64,
                                         C.POINTER(C.c_uint64)]
        L.xvo_spectral_angle.restype = C.c_double
        if L.xvo_selfcheck() != 0:
            raise RuntimeError("oracle requires arithmetic right shifts")
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _dtype_code(cube: np.ndarray) -> int:
    if cube.dtype == np.uint16:
        return U16
    if cube.dtype == np.float32:
        return F32
    raise TypeError(f"unsupported cube dtype {cube.dtype}")


def padded(n: int, N: int) -> int:
    return (n + N - 1) // N * N


# -- steps -----------------------------------------------------------------

def stats(cube: np.ndarray):
    """xvo_stats: per-band NaN-aware min, max and valid count."""
    T, H, W, Bn = cube.shape
    mn = np.zeros(Bn, np.float64)
    mx = np.zeros(Bn, np.float64)
    nv = np.zeros(Bn, np.int64)
    lib().xvo_stats(_ptr(cube), _dtype_code(cube), T, H, W, Bn, _ptr(mn), _ptr(mx), _ptr(nv))
    return mn, mx, nv


def filled_value(cube, t, y, x, b, fill_mode, mn_b):
    T, H, W, Bn = cube.shape
    ok = C.c_int(0)
    v = lib().xvo_filled_value(_ptr(cube), _dtype_code(cube), T, H, W, Bn, t, y, x, b,
                               fill_mode, mn_b, C.byref(ok))
    return v, bool(ok.value)


def normalize(x: float, mn: float, mx: float, B: int) -> int:
    return lib().xvo_normalize(float(x), float(mn), float(mx), B)


def denormalize(q: int, mn: float, mx: float, B: int) -> float:
    return lib().xvo_denormalize(int(q), float(mn), float(mx), B)


def cast_output(v: float, dtype_code: int) -> float:
    return lib().xvo_cast_output(float(v), dtype_code)


def source_band(g, c, Bn, pad_mode):
    return lib().xvo_source_band(g, c, Bn, pad_mode)


def make_frame(cube, mn, mx, params: CodingParams, g, t):
    T, H, W, Bn = cube.shape
    N = params.block
    Hp, Wp = padded(H, N), padded(W, N)
    fr = np.zeros((3, Hp, Wp), np.uint16)
    va = np.zeros((3, Hp, Wp), np.uint8)
    pc = params.c()
    lib().xvo_make_frame(_ptr(cube), _dtype_code(cube), T, H, W, Bn, _ptr(mn), _ptr(mx),
                         C.byref(pc), g, t, Hp, Wp, _ptr(fr), _ptr(va))
    return fr, va


def dct_matrix(N: int) -> np.ndarray:
    M = np.zeros((N, N), np.int32)
    lib().xvo_dct_matrix(N, _ptr(M))
    return M


def forward_transform(r: np.ndarray, B: int) -> np.ndarray:
    r = np.ascontiguousarray(r, np.int32)
    N = r.shape[0]
    out = np.zeros((N, N), np.int32)
    lib().xvo_forward_transform(N, B, _ptr(r), _ptr(out))
    return out


def iq_scale(k: int) -> int:
    return lib().xvo_iq_scale(k)


def q_scale(k: int) -> int:
    return lib().xvo_q_scale(k)


def quantize(Cc: np.ndarray, B: int, qp: int, intra: bool) -> np.ndarray:
    Cc = np.ascontiguousarray(Cc, np.int32)
    N = Cc.shape[0]
    out = np.zeros((N, N), np.int16)
    lib().xvo_quantize(N, B, qp, int(intra), _ptr(Cc), _ptr(out))
    return out


def dequantize(lev: np.ndarray, B: int, qp: int) -> np.ndarray:
    lev = np.ascontiguousarray(lev, np.int16)
    N = lev.shape[0]
    out = np.zeros((N, N), np.int32)
    lib().xvo_dequantize(N, B, qp, _ptr(lev), _ptr(out))
    return out


def inverse_transform(d: np.ndarray, B: int) -> np.ndarray:
    d = np.ascontiguousarray(d, np.int32)
    N = d.shape[0]
    out = np.zeros((N, N), np.int32)
    lib().xvo_inverse_transform(N, B, _ptr(d), _ptr(out))
    return out


def ue_len(k: int) -> int:
    return lib().xvo_ue_len(k)


def se_len(v: int) -> int:
    return lib().xvo_se_len(v)


def scan_order(N: int) -> np.ndarray:
    o = np.zeros(N * N, np.int32)
    lib().xvo_scan_order(N, _ptr(o))
    return o


def coef_bits(lev: np.ndarray) -> int:
    lev = np.ascontiguousarray(lev, np.int16)
    return lib().xvo_coef_bits(lev.shape[0], _ptr(lev))


def mv_bits(mvx, mvy, pmx, pmy) -> int:
    return lib().xvo_mv_bits(mvx, mvy, pmx, pmy)


def motion_search(cur: np.ndarray, ref: np.ndarray, N: int, R: int, bx: int, by: int,
                  nch: int = 3):
    cur = np.ascontiguousarray(cur, np.uint16)
    ref = np.ascontiguousarray(ref, np.uint16)
    _, Hp, Wp = cur.shape
    dx, dy, sad = C.c_int32(), C.c_int32(), C.c_uint32()
    lib().xvo_motion_search(_ptr(cur), _ptr(ref), Hp, Wp, N, R, nch, bx, by,
                            C.byref(dx), C.byref(dy), C.byref(sad))
    return dx.value, dy.value, sad.value


def luma_filter(frac: int, tap: int) -> int:
    """xvo_luma_filter: H.265 luma interpolation coefficient fL[frac][tap]."""
    return lib().xvo_luma_filter(frac, tap)


def interp_sample(plane: np.ndarray, B: int, xq: int, yq: int) -> int:
    """xvo_interp_sample: predicted sample at quarter-sample position (xq, yq)."""
    plane = np.ascontiguousarray(plane, np.uint16)
    Hp, Wp = plane.shape
    return lib().xvo_interp_sample(_ptr(plane), Hp, Wp, B, xq, yq)


def subpel_refine(cur: np.ndarray, ref: np.ndarray, N: int, B: int, bx: int, by: int,
                  dx: int, dy: int, nch: int = 3):
    """xvo_subpel_refine: half- then quarter-sample refinement of (dx, dy);
    returns (mvx, mvy, sad) with the vector in quarter samples."""
    cur = np.ascontiguousarray(cur, np.uint16)
    ref = np.ascontiguousarray(ref, np.uint16)
    _, Hp, Wp = cur.shape
    mx, my, sad = C.c_int32(), C.c_int32(), C.c_uint32()
    lib().xvo_subpel_refine(_ptr(cur), _ptr(ref), Hp, Wp, N, B, nch, bx, by, dx, dy,
                            C.byref(mx), C.byref(my), C.byref(sad))
    return mx.value, my.value, sad.value


def intra_refs(rec_plane: np.ndarray, N: int, B: int, bx: int, by: int) -> np.ndarray:
    """xvo_intra_refs: the 4N + 1 reference samples of block (bx, by) of a
    [Hp][Wp] plane, in substitution-scan order (H.265 8.4.4.2.2)."""
    plane = np.ascontiguousarray(rec_plane, np.uint16)
    Hp, Wp = plane.shape
    refs = np.zeros(4 * N + 1, np.int32)
    lib().xvo_intra_refs(_ptr(plane), Hp, Wp, N, B, bx, by, _ptr(refs))
    return refs


def intra_predict(refs: np.ndarray, N: int, mode: int, B: int) -> np.ndarray:
    """xvo_intra_predict: N x N prediction [y][x] of mode 0 (planar) or 1 (DC)."""
    r = np.ascontiguousarray(refs, np.int32)
    assert r.size == 4 * N + 1
    pred = np.zeros((N, N), np.int32)
    lib().xvo_intra_predict(_ptr(r), N, mode, B, _ptr(pred))
    return pred


def pca_moments(cube: np.ndarray):
    """xvo_pca_moments: band means and covariance of a u16 cube [..][Bn]."""
    cube = np.ascontiguousarray(cube, np.uint16)
    Bn = cube.shape[-1]
    npix = cube.size // Bn
    mean = np.zeros(Bn, np.float64)
    cov = np.zeros((Bn, Bn), np.float64)
    if lib().xvo_pca_moments(_ptr(cube), npix, Bn, _ptr(mean), _ptr(cov)) != 0:
        raise ValueError("xvo_pca_moments failed")
    return mean, cov


def pca_eigen(cov: np.ndarray):
    """xvo_pca_eigen: eigenvalues (decreasing) and basis [b][j] (column j = PC j)."""
    cov = np.ascontiguousarray(cov, np.float64)
    Bn = cov.shape[0]
    ev = np.zeros(Bn, np.float64)
    basis = np.zeros((Bn, Bn), np.float64)
    if lib().xvo_pca_eigen(_ptr(cov), Bn, _ptr(ev), _ptr(basis)) != 0:
        raise ValueError("xvo_pca_eigen failed")
    return ev, basis


def pca_project(cube: np.ndarray, mean, basis, j0: int, j1: int) -> np.ndarray:
    """xvo_pca_project: PCs j0..j1-1 of every sample, f32 [..][j1-j0]."""
    cube = np.ascontiguousarray(cube, np.uint16)
    Bn = cube.shape[-1]
    npix = cube.size // Bn
    out = np.zeros(cube.shape[:-1] + (j1 - j0,), np.float32)
    lib().xvo_pca_project(_ptr(cube), npix, Bn, _ptr(np.ascontiguousarray(mean)),
                          _ptr(np.ascontiguousarray(basis)), j0, j1, _ptr(out))
    return out


def pca_inverse(pcs: np.ndarray, mean, basis, out_dtype: int) -> np.ndarray:
    """xvo_pca_inverse: bands from the first k PCs (pcs f32 [..][k])."""
    pcs = np.ascontiguousarray(pcs, np.float32)
    k = pcs.shape[-1]
    Bn = basis.shape[0]
    npix = pcs.size // k
    out = np.zeros(pcs.shape[:-1] + (Bn,), np.uint16 if out_dtype == U16 else np.float32)
    lib().xvo_pca_inverse(_ptr(pcs), npix, Bn, k, _ptr(np.ascontiguousarray(mean)),
                          _ptr(np.ascontiguousarray(basis)), out_dtype, _ptr(out))
    return out


# -- whole-GOP and whole-cube drivers ----------------------------------------

def _gop_arrays(len_, Hp, Wp, N, split=0):
    Hb, Wb = Hp // N, Wp // N
    m = 2 if split else 1  # vectors on the N/2 grid with the adaptive block size
    return dict(
        frames=np.zeros((len_, 3, Hp, Wp), np.uint16),
        levels=np.zeros((len_, 3, Hb, Wb, N, N), np.int16),
        mvs=np.zeros((len_, m * Hb, m * Wb, 2), np.int8),
        recon=np.zeros((len_, 3, Hp, Wp), np.uint16),
        coef_bits=np.zeros((len_, 3, Hb, Wb), np.uint32),
        mv_bits=np.zeros((len_, Hb, Wb), np.uint32),
        splits=np.zeros((len_, Hb, Wb), np.uint8),
    )


def split_choose(sad_whole: int, v, sads, cells, lam16: int) -> int:
    """xvo_split_choose: 1 when the four cells cost less than the whole block."""
    sa = np.array(sads, np.uint32)
    ux = np.array([c[0] for c in cells], np.int32)
    uy = np.array([c[1] for c in cells], np.int32)
    return int(lib().xvo_split_choose(sad_whole, v[0], v[1], _ptr(sa), _ptr(ux), _ptr(uy),
                                      lam16))


def split_lambda(qp: int, B: int) -> int:
    """xvo_split_lambda: the whole/split cost multiplier in 1/16 SAD units."""
    return int(lib().xvo_split_lambda(qp, B))


def encode_gop(cube, mn, mx, params: CodingParams, g: int, t0: int, len_: int):
    """xvo_encode_gop: one closed GOP of one band group (all outputs)."""
    T, H, W, Bn = cube.shape
    N = params.block
    Hp, Wp = padded(H, N), padded(W, N)
    o = _gop_arrays(len_, Hp, Wp, N, params.split)
    sse = np.zeros(3, np.uint64)
    nv = np.zeros(3, np.uint64)
    pc = params.c()
    rc = lib().xvo_encode_gop(_ptr(cube), _dtype_code(cube), T, H, W, Bn, _ptr(mn), _ptr(mx),
                              C.byref(pc), g, t0, len_, _ptr(o["frames"]), _ptr(o["levels"]),
                              _ptr(o["mvs"]), _ptr(o["recon"]), _ptr(o["coef_bits"]),
                              _ptr(o["mv_bits"]), _ptr(o["splits"]), _ptr(sse), _ptr(nv))
    if rc != 0:
        raise ValueError(f"xvo_encode_gop failed ({rc})")
    o["sse"], o["nvalid"] = sse, nv
    return o


def decode_gop(params: CodingParams, H: int, W: int, levels, mvs, splits=None):
    N = params.block
    len_ = levels.shape[0]
    Hp, Wp = padded(H, N), padded(W, N)
    rec = np.zeros((len_, 3, Hp, Wp), np.uint16)
    pc = params.c()
    sp = _ptr(np.ascontiguousarray(splits, np.uint8)) if splits is not None else None
    rc = lib().xvo_decode_gop(C.byref(pc), H, W, len_, _ptr(np.ascontiguousarray(levels)),
                              _ptr(np.ascontiguousarray(mvs)), sp, _ptr(rec))
    if rc != 0:
        raise ValueError(f"xvo_decode_gop failed ({rc})")
    return rec


def encode_cube(cube: np.ndarray, params: CodingParams) -> dict:
    """xvo_encode_cube: every (group, GOP) unit; layouts [G][T][...]."""
    T, H, W, Bn = cube.shape
    N = params.block
    G = (Bn + 2) // 3
    Hp, Wp = padded(H, N), padded(W, N)
    Hb, Wb = Hp // N, Wp // N
    m = 2 if params.split else 1  # vectors on the N/2 grid with the adaptive block size
    o = dict(
        frames=np.zeros((G, T, 3, Hp, Wp), np.uint16),
        levels=np.zeros((G, T, 3, Hb, Wb, N, N), np.int16),
        mvs=np.zeros((G, T, m * Hb, m * Wb, 2), np.int8),
        recon=np.zeros((G, T, 3, Hp, Wp), np.uint16),
        coef_bits=np.zeros((G, T, 3, Hb, Wb), np.uint32),
        mv_bits=np.zeros((G, T, Hb, Wb), np.uint32),
        splits=np.zeros((G, T, Hb, Wb), np.uint8),
    )
    mn = np.zeros(Bn, np.float64)
    mx = np.zeros(Bn, np.float64)
    sse = np.zeros(Bn, np.uint64)
    nv = np.zeros(Bn, np.uint64)
    pc = params.c()
    cube = np.ascontiguousarray(cube)
    rc = lib().xvo_encode_cube(_ptr(cube), _dtype_code(cube), T, H, W, Bn, C.byref(pc),
                               _ptr(mn), _ptr(mx), _ptr(o["frames"]), _ptr(o["levels"]),
                               _ptr(o["mvs"]), _ptr(o["recon"]), _ptr(o["coef_bits"]),
                               _ptr(o["mv_bits"]), _ptr(o["splits"]), _ptr(sse), _ptr(nv))
    if rc != 0:
        raise ValueError(f"xvo_encode_cube failed ({rc})")
    o.update(mn=mn, mx=mx, sse=sse, nvalid=nv)
    return o


def write_bitstream(levels: np.ndarray, mvs: np.ndarray, gop: int, imodes: int = 0,
                    splits=None) -> dict:
    """xvo_write_bitstream: levels [G][T][3][Hb][Wb][N][N] i16 and vectors
    [G][T][Hb][Wb][2] i8 -> payload bytes, its length in bits and the bit
    offset of every segment (4 * Hb per frame).  imodes: I blocks carry
    their intra mode bit; splits ([G][T][Hb][Wb], adaptive block size: the
    vectors are then on the N/2 grid)."""
    G, T, _, Hb, Wb, N, _ = levels.shape
    levels = np.ascontiguousarray(levels, np.int16)
    mvs = np.ascontiguousarray(mvs, np.int8)
    sp = None
    if splits is not None:
        splits = np.ascontiguousarray(splits, np.uint8)
        sp = _ptr(splits)
    bits = int(lib().xvo_bitstream_bits(N, G, T, gop, Hb, Wb, imodes, sp, _ptr(levels),
                                        _ptr(mvs)))
    nbytes = (bits + 7) // 8
    out = np.zeros(max(1, nbytes), np.uint8)
    index = np.zeros(G * T * 4 * Hb, np.uint64)
    rc = lib().xvo_write_bitstream(N, G, T, gop, Hb, Wb, imodes, sp, _ptr(levels), _ptr(mvs),
                                   _ptr(out), out.size, _ptr(index))
    if rc != 0:
        raise ValueError(f"xvo_write_bitstream failed ({rc})")
    return dict(payload=out[:nbytes], bits=bits, index=index)


def read_bitstream(payload: np.ndarray, bits: int, shape_lev, gop: int, imodes: int = 0,
                   split: int = 0) -> dict:
    """xvo_read_bitstream: sequential parse back to levels and vectors (and
    split flags with the adaptive block size); also returns the segment
    offsets met."""
    G, T, _, Hb, Wb, N, _ = shape_lev
    m = 2 if split else 1
    levels = np.zeros(shape_lev, np.int16)
    mvs = np.zeros((G, T, m * Hb, m * Wb, 2), np.int8)
    splits = np.zeros((G, T, Hb, Wb), np.uint8)
    index = np.zeros(G * T * 4 * Hb, np.uint64)
    buf = np.ascontiguousarray(payload, np.uint8)
    if buf.size == 0:
        buf = np.zeros(1, np.uint8)
    rc = lib().xvo_read_bitstream(N, G, T, gop, Hb, Wb, imodes,
                                  _ptr(splits) if split else None, _ptr(buf), bits,
                                  _ptr(levels), _ptr(mvs), _ptr(index))
    if rc != 0:
        raise ValueError(f"xvo_read_bitstream failed ({rc})")
    out = dict(levels=levels, mvs=mvs, index=index)
    if split:
        out["splits"] = splits
    return out


def decode_cube(params: CodingParams, shape, levels, mvs, splits=None) -> np.ndarray:
    T, H, W, Bn = shape
    N = params.block
    G = (Bn + 2) // 3
    rec = np.zeros((G, T, 3, padded(H, N), padded(W, N)), np.uint16)
    pc = params.c()
    if params.split and splits is None:
        raise ValueError("the adaptive block size needs the split flags")
    sp = _ptr(np.ascontiguousarray(splits, np.uint8)) if params.split else None
    rc = lib().xvo_decode_cube(C.byref(pc), T, H, W, Bn, _ptr(np.ascontiguousarray(levels)),
                               _ptr(np.ascontiguousarray(mvs)), sp, _ptr(rec))
    if rc != 0:
        raise ValueError(f"xvo_decode_cube failed ({rc})")
    return rec


def denormalize_cube(recon, shape, N, B, mn, mx, out_dtype) -> np.ndarray:
    T, H, W, Bn = shape
    out = np.zeros(shape, np.uint16 if out_dtype == U16 else np.float32)
    lib().xvo_denormalize_cube(_ptr(np.ascontiguousarray(recon)), T, H, W, Bn, N, B,
                               _ptr(mn), _ptr(mx), out_dtype, _ptr(out))
    return out


def psnr(peak: float, sse: float, n: float) -> float:
    return lib().xvo_psnr(float(peak), float(sse), float(n))


def psnr_int(B: int, sse: int, n: int) -> float:
    return lib().xvo_psnr_int(B, int(sse), int(n))


def bpppb(bits: int, T, H, W, Bn) -> float:
    return lib().xvo_bpppb(int(bits), T, H, W, Bn)


def phys_sse(cube, recon, N, B, mn, mx) -> np.ndarray:
    T, H, W, Bn = cube.shape
    out = np.zeros(Bn, np.float64)
    lib().xvo_phys_sse(_ptr(cube), _dtype_code(cube), T, H, W, Bn,
                       _ptr(np.ascontiguousarray(recon)), N, B, _ptr(mn), _ptr(mx), _ptr(out))
    return out


def metrics(cube: np.ndarray, enc: dict, params: CodingParams) -> dict:
    """Per-band PSNR (integer and physical domain) and bpppb of an encode."""
    T, H, W, Bn = cube.shape
    G = (Bn + 2) // 3
    B = params.bit_depth
    coef = int(enc["coef_bits"].astype(np.uint64).sum())
    mvb = int(enc["mv_bits"].astype(np.uint64).sum())
    psnr_i = [psnr_int(B, int(enc["sse"][b]), int(enc["nvalid"][b])) for b in range(Bn)]
    sse_p = phys_sse(cube, enc["recon"], params.block, B, enc["mn"], enc["mx"])
    psnr_p = [psnr(enc["mx"][b], sse_p[b], int(enc["nvalid"][b])) if enc["mx"][b] > 0
              else float("nan") for b in range(Bn)]
    per_group = []
    for g in range(G):
        nb = min(3, Bn - 3 * g)
        bits_g = int(enc["coef_bits"][g].astype(np.uint64).sum()) + \
            int(enc["mv_bits"][g].astype(np.uint64).sum())
        per_group.append(bpppb(bits_g, T, H, W, nb))
    return dict(psnr=psnr_i, psnr_phys=psnr_p, sse_phys=sse_p, coef_bits=coef, mv_bits=mvb,
                bpppb=bpppb(coef + mvb, T, H, W, Bn), bpppb_group=per_group)


def ssim_window() -> np.ndarray:
    """xvo_ssim_window: the normalised 11-tap Gaussian (sigma 1.5)."""
    w = np.zeros(11, np.float64)
    lib().xvo_ssim_window(_ptr(w))
    return w


def ssim_plane(a: np.ndarray, b: np.ndarray, B: int) -> float:
    """xvo_ssim_plane: mean SSIM of two u16 planes (coded domain, L = 2^B - 1)."""
    a = np.ascontiguousarray(a, np.uint16)
    b = np.ascontiguousarray(b, np.uint16)
    H, W = a.shape
    return lib().xvo_ssim_plane(_ptr(a), _ptr(b), W, H, W, B)


def ssim_bands(frames, recon, shape, N: int, B: int) -> np.ndarray:
    """xvo_ssim_bands: per-band mean SSIM of an encode's frames and recon."""
    T, H, W, Bn = shape
    out = np.zeros(Bn, np.float64)
    lib().xvo_ssim_bands(_ptr(np.ascontiguousarray(frames)), _ptr(np.ascontiguousarray(recon)),
                         T, H, W, Bn, N, B, _ptr(out))
    return out


def spectral_angle(orig: np.ndarray, dec: np.ndarray):
    """xvo_spectral_angle: mean angle (radians) and the number of pixels used."""
    T, H, W, Bn = orig.shape
    assert dec.shape == orig.shape
    n = C.c_uint64(0)
    orig = np.ascontiguousarray(orig)
    dec = np.ascontiguousarray(dec)
    v = lib().xvo_spectral_angle(_ptr(orig), _dtype_code(orig), _ptr(dec), _dtype_code(dec),
                                 T, H, W, Bn, C.byref(n))
    return v, int(n.value)
