"""Python binding of libxv (argument marshalling only).

Every function here forwards to the C ABI declared in include/xv.h; all
compute runs in the library's HIP kernels.  PyTorch supplies device memory
(tensors) and the HIP stream (torch.cuda.current_stream()).  There is no
fallback: if libxv.so is missing or fails to load, the import of the library
raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libxv.so")

OK, EINVAL, ENOMEM, EHIP, EBUSY, ECANCELED, EPENDING = 0, -1, -2, -3, -4, -5, -6
U16, F32 = 0, 1
PAD_ZERO, PAD_REPEAT = 0, 1
FILL_NEAREST, FILL_FORWARD = 0, 1
FLAG_DROP_WORK = 1
FLAG_QPEL = 2
FLAG_INTRA = 4
FLAG_SPLIT = 8
ME_COLUMN_PAIRS, ME_ROW_PAIRS, ME_ROW_PAIRS_BY_CHANNEL = 1, 2, 3
MAX_BANDS, MAX_GROUPS = 64, 22
K_STATS, K_PACK, K_ME, K_ENCODE, K_DECODE, K_DENORM, K_METRICS, K_BITS_WRITE, K_BITS_PARSE, \
    K_QUALITY, K_SUBPEL, K_PCA, K_INTRA = range(13)
K_NAMES = ["stats", "pack", "me", "encode", "decode", "denorm", "metrics", "bits_write",
           "bits_parse", "quality", "subpel", "pca", "intra"]


class XvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


class Cube(C.Structure):
    _fields_ = [("data", C.c_void_p), ("dtype", C.c_int32), ("reserved", C.c_int32),
                ("T", C.c_int64), ("H", C.c_int64), ("W", C.c_int64), ("bands", C.c_int64)]


class ParamsC(C.Structure):
    _fields_ = [("bit_depth", C.c_int32), ("qp", C.c_int32), ("block", C.c_int32),
                ("search_range", C.c_int32), ("gop", C.c_int32), ("pad_mode", C.c_int32),
                ("fill_mode", C.c_int32), ("flags", C.c_uint32)]


class MetricsC(C.Structure):
    _fields_ = [("bands", C.c_int32), ("groups", C.c_int32),
                ("psnr", C.c_double * MAX_BANDS), ("psnr_phys", C.c_double * MAX_BANDS),
                ("sse_phys", C.c_double * MAX_BANDS), ("sse", C.c_uint64 * MAX_BANDS),
                ("n_valid", C.c_uint64 * MAX_BANDS), ("band_min", C.c_double * MAX_BANDS),
                ("band_max", C.c_double * MAX_BANDS), ("coef_bits", C.c_uint64),
                ("mv_bits", C.c_uint64), ("header_bits", C.c_uint64), ("bpppb", C.c_double),
                ("bpppb_group", C.c_double * MAX_GROUPS)]


class ExportC(C.Structure):
    _fields_ = [("T", C.c_int64), ("H", C.c_int64), ("W", C.c_int64), ("bands", C.c_int64),
                ("groups", C.c_int64), ("Hp", C.c_int64), ("Wp", C.c_int64), ("Hb", C.c_int64),
                ("Wb", C.c_int64), ("params", ParamsC), ("src_dtype", C.c_int32),
                ("reserved", C.c_int32), ("frames", C.c_void_p), ("recon", C.c_void_p),
                ("levels", C.c_void_p), ("mvs", C.c_void_p), ("coef_bits", C.c_void_p),
                ("mv_bits", C.c_void_p), ("band_min", C.c_void_p), ("band_max", C.c_void_p),
                ("sse", C.c_void_p), ("n_valid", C.c_void_p), ("splits", C.c_void_p)]


class MeGeometryC(C.Structure):
    _fields_ = [("blocks_per_wg", C.c_int32), ("cands_per_lane", C.c_int32),
                ("threads", C.c_int32), ("rows_per_lane", C.c_int32), ("layout", C.c_int32)]


class ProfileC(C.Structure):
    _fields_ = [("ms", C.c_double * 13), ("launches", C.c_uint64 * 13), ("work", C.c_double * 13)]


class MemoryC(C.Structure):
    _fields_ = [("live_bytes", C.c_uint64), ("cached_bytes", C.c_uint64),
                ("peak_bytes", C.c_uint64)]


class ServerCfgC(C.Structure):
    _fields_ = [("hbm_budget", C.c_uint64), ("max_slots", C.c_int32), ("max_queue", C.c_int32),
                ("stream", C.c_void_p)]


class RequestC(C.Structure):
    _fields_ = [("op", C.c_int32), ("reserved", C.c_int32), ("cube", Cube), ("params", ParamsC),
                ("enc", C.c_void_p)]


class ResultC(C.Structure):
    _fields_ = [("status", C.c_int32), ("op", C.c_int32), ("enc", C.c_void_p),
                ("submit_ms", C.c_double), ("admit_ms", C.c_double), ("done_ms", C.c_double)]


class ServerStatsC(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("cancelled", C.c_uint64),
                ("failed", C.c_uint64), ("iterations", C.c_uint64), ("launches", C.c_uint64),
                ("peak_bytes", C.c_uint64), ("peak_active", C.c_int32), ("reserved", C.c_int32)]


OP_ENCODE, OP_DECODE = 0, 1

EXPORTED = ["xv_abi_version", "xv_status_str", "xv_last_error", "xv_encode_cube",
            "xv_decode_cube", "xv_psnr_bpppb", "xv_psnr_bpppb_batch", "xv_encoded_export",
            "xv_encoded_free",
            "xv_encode_batch", "xv_decode_batch", "xv_set_me_geometry", "xv_get_me_geometry",
            "xv_set_me_split_geometry", "xv_get_me_split_geometry", "xv_autotune_me", "xv_autotune_me_batch", "xv_profile_enable", "xv_profile_select", "xv_profile_read", "xv_server_create",
            "xv_server_submit", "xv_server_poll", "xv_server_wait", "xv_server_cancel",
            "xv_server_stats_read", "xv_server_destroy", "xv_memory_read", "xv_cache_release", "xv_pack", "xv_packed_view",
            "xv_packed_free", "xv_unpack", "xv_ssim", "xv_spectral_angle",
            "xv_spectral_angle_noalloc", "xv_pca_fit", "xv_pca_view", "xv_pca_project",
            "xv_pca_inverse", "xv_pca_free", "xv_set_graph_mode", "xv_get_graph_mode"]

_lib = None


def lib():
    """Load libxv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.xv_abi_version.restype = C.c_int
        L.xv_status_str.argtypes = [C.c_int]
        L.xv_status_str.restype = C.c_char_p
        L.xv_last_error.restype = C.c_char_p
        L.xv_encode_cube.argtypes = [C.POINTER(Cube), C.POINTER(ParamsC), vp, C.POINTER(vp)]
        L.xv_decode_cube.argtypes = [vp, C.POINTER(Cube), vp]
        L.xv_psnr_bpppb.argtypes = [C.POINTER(Cube), vp, C.POINTER(MetricsC), vp]
        L.xv_psnr_bpppb_batch.argtypes = [C.c_int, C.POINTER(Cube), C.POINTER(vp),
                                          C.POINTER(MetricsC), vp]
        L.xv_ssim.argtypes = [vp, C.POINTER(C.c_double), vp]
        L.xv_spectral_angle.argtypes = [C.POINTER(Cube), C.POINTER(Cube), C.POINTER(C.c_double),
                                        C.POINTER(C.c_uint64), vp]
        L.xv_spectral_angle_noalloc.argtypes = [C.POINTER(Cube), C.POINTER(Cube),
                                                C.POINTER(C.c_double), C.POINTER(C.c_uint64), vp]
        L.xv_pca_fit.argtypes = [C.POINTER(Cube), vp, C.POINTER(vp)]
        L.xv_pca_view.argtypes = [vp, C.POINTER(C.c_int32), vp, vp, vp, vp]
        L.xv_pca_project.argtypes = [vp, C.POINTER(Cube), C.c_int32, C.c_int32, C.POINTER(Cube),
                                     vp]
        L.xv_pca_inverse.argtypes = [vp, C.POINTER(Cube), C.POINTER(Cube), vp]
        L.xv_pca_free.argtypes = [vp]
        L.xv_pca_free.restype = None
        L.xv_set_graph_mode.argtypes = [C.c_int]
        L.xv_get_graph_mode.argtypes = []
        L.xv_encoded_export.argtypes = [vp, C.POINTER(ExportC)]
        L.xv_encoded_free.argtypes = [vp]
        L.xv_encoded_free.restype = None
        L.xv_encode_batch.argtypes = [C.c_int, C.POINTER(Cube), C.POINTER(ParamsC), vp,
                                      C.POINTER(vp)]
        L.xv_decode_batch.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(Cube), vp]
        L.xv_set_me_geometry.argtypes = [C.c_int, C.c_int, C.POINTER(MeGeometryC)]
        L.xv_get_me_geometry.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(MeGeometryC)]
        L.xv_set_me_split_geometry.argtypes = [C.c_int, C.c_int, C.POINTER(MeGeometryC)]
        L.xv_get_me_split_geometry.argtypes = [C.c_int, C.c_int, C.c_int,
                                               C.POINTER(MeGeometryC)]
        L.xv_autotune_me.argtypes = [C.POINTER(Cube), C.POINTER(ParamsC), vp, C.c_int,
                                     C.POINTER(MeGeometryC), C.POINTER(C.c_double)]
        L.xv_autotune_me_batch.argtypes = [C.c_int, C.POINTER(Cube), C.POINTER(ParamsC), vp,
                                           C.c_int, C.POINTER(MeGeometryC),
                                           C.POINTER(C.c_double)]
        L.xv_pack.argtypes = [vp, vp, C.POINTER(vp)]
        L.xv_packed_view.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_uint64),
                                     C.POINTER(C.c_uint64)]
        L.xv_packed_free.argtypes = [vp]
        L.xv_packed_free.restype = None
        L.xv_unpack.argtypes = [vp, C.c_uint64, vp, C.POINTER(vp)]
        L.xv_memory_read.argtypes = [C.POINTER(MemoryC)]
        L.xv_cache_release.argtypes = [C.POINTER(C.c_uint64)]
        L.xv_server_create.argtypes = [C.POINTER(ServerCfgC), C.POINTER(vp)]
        L.xv_server_submit.argtypes = [vp, C.POINTER(RequestC), C.POINTER(C.c_uint64)]
        L.xv_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(ResultC)]
        L.xv_server_wait.argtypes = [vp, C.c_uint64, C.POINTER(ResultC)]
        L.xv_server_cancel.argtypes = [vp, C.c_uint64]
        L.xv_server_stats_read.argtypes = [vp, C.POINTER(ServerStatsC)]
        L.xv_server_destroy.argtypes = [vp]
        L.xv_profile_enable.argtypes = [C.c_int]
        L.xv_profile_select.argtypes = [C.c_uint32]
        L.xv_profile_read.argtypes = [C.POINTER(ProfileC)]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise XvError(rc, lib().xv_last_error().decode(errors="replace"))


@dataclass
class Params:
    bit_depth: int = 10
    qp: int = 27
    block: int = 8
    search_range: int = 8
    gop: int = 16
    pad_mode: int = PAD_ZERO
    fill_mode: int = FILL_NEAREST
    flags: int = 0

    def c(self) -> ParamsC:
        return ParamsC(self.bit_depth, self.qp, self.block, self.search_range, self.gop,
                       self.pad_mode, self.fill_mode, self.flags)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _cube(t) -> Cube:
    import torch
    if not t.is_cuda:
        raise ValueError("cube must be a device tensor")
    if t.dim() != 4:
        raise ValueError("cube must be [T, H, W, bands]")
    if not t.is_contiguous():
        raise ValueError("cube must be contiguous")
    if t.dtype == torch.uint16:
        dt = U16
    elif t.dtype == torch.float32:
        dt = F32
    else:
        raise ValueError(f"unsupported dtype {t.dtype}")
    T, H, W, Bn = t.shape
    return Cube(C.c_void_p(t.data_ptr()), dt, 0, T, H, W, Bn)


class _DevArray:
    """__cuda_array_interface__ view of library-owned device memory."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(int(s) for s in shape),
                                         "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}


@dataclass
class Encoded:
    handle: C.c_void_p
    shape: tuple
    params: Params
    _freed: bool = field(default=False)

    def export(self) -> dict:
        """Device views (torch tensors) of the encoded buffers; signed element
        types are used for unsigned buffers (reinterpret with numpy .view)."""
        import torch
        v = ExportC()
        _check(lib().xv_encoded_export(self.handle, C.byref(v)))
        G, T, Hp, Wp, Hb, Wb = v.groups, v.T, v.Hp, v.Wp, v.Hb, v.Wb
        N = v.params.block
        Bn = v.bands
        out = {"dims": dict(T=T, H=v.H, W=v.W, bands=Bn, groups=G, Hp=Hp, Wp=Wp, Hb=Hb, Wb=Wb)}

        def view(ptr, shape, ts):
            if not ptr:
                return None
            return torch.as_tensor(_DevArray(ptr, shape, ts), device="cuda")

        out["frames"] = view(v.frames, (G, T, 3, Hp, Wp), "<i2")
        out["recon"] = view(v.recon, (G, T, 3, Hp, Wp), "<i2")
        # stored column-major inside a block ([k][l]); presented as [l][k]
        lev = view(v.levels, (G, T, 3, Hb, Wb, N, N), "<i2")
        out["levels"] = None if lev is None else lev.transpose(-1, -2)
        out["levels_raw"] = lev
        # adaptive block size: split flags, vectors on the N/2 cell grid
        out["splits"] = view(v.splits, (G, T, Hb, Wb), "|i1")
        m = 2 if v.splits else 1
        out["mvs"] = view(v.mvs, (G, T, m * Hb, m * Wb, 2), "|i1")
        out["coef_bits"] = view(v.coef_bits, (G, T, 3, Hb, Wb), "<i4")
        out["mv_bits"] = view(v.mv_bits, (G, T, Hb, Wb), "<i4")
        out["band_min"] = view(v.band_min, (Bn,), "<f8")
        out["band_max"] = view(v.band_max, (Bn,), "<f8")
        out["sse"] = view(v.sse, (3 * G,), "<i8")
        out["n_valid"] = view(v.n_valid, (Bn,), "<i8")
        return out

    def host(self) -> dict:
        """Synchronous host copies with the library's element types."""
        import torch
        torch.cuda.synchronize()
        ex = self.export()
        types = {"frames": np.uint16, "recon": np.uint16, "levels": np.int16, "mvs": np.int8,
                 "coef_bits": np.uint32, "mv_bits": np.uint32, "band_min": np.float64,
                 "band_max": np.float64, "sse": np.uint64, "n_valid": np.uint64}
        out = {"dims": ex["dims"]}
        for k, ty in types.items():
            t = ex[k]
            out[k] = None if t is None else t.cpu().numpy().view(ty)
        if ex["splits"] is not None:
            # a split block's slot holds its four N/2 blocks (z-order), each
            # column-major: present each as [l][k], one after another
            sp = ex["splits"].cpu().numpy().view(np.uint8)
            out["splits"] = sp
            raw = ex["levels_raw"].cpu().numpy().view(np.int16)
            N = raw.shape[-1]
            h = N // 2
            flat = raw.reshape(*raw.shape[:-2], 4, h, h).swapaxes(-1, -2).reshape(raw.shape)
            mask = sp.astype(bool)[:, :, None, :, :, None, None]
            out["levels"] = np.where(mask, flat, out["levels"])
        return out

    def free(self):
        if not self._freed:
            lib().xv_encoded_free(self.handle)
            self._freed = True

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def encode_cube(cube, params: Params, stream=None) -> Encoded:
    """xv_encode_cube on a device tensor [T, H, W, bands] (uint16 or float32)."""
    cb = _cube(cube)
    pc = params.c()
    h = C.c_void_p()
    _check(lib().xv_encode_cube(C.byref(cb), C.byref(pc), _stream_handle(stream), C.byref(h)))
    return Encoded(h, tuple(cube.shape), params)


def encode_batch(cubes, params, stream=None) -> list:
    """xv_encode_batch: several cubes, one launch per frame step and class."""
    n = len(cubes)
    cbs = (Cube * n)(*[_cube(c) for c in cubes])
    pcs = (ParamsC * n)(*[p.c() for p in params])
    hs = (C.c_void_p * n)()
    _check(lib().xv_encode_batch(n, cbs, pcs, _stream_handle(stream), hs))
    return [Encoded(C.c_void_p(hs[i]), tuple(cubes[i].shape), params[i]) for i in range(n)]


def decode_cube(enc: Encoded, out, stream=None):
    """xv_decode_cube into a device tensor of the encoded cube's shape."""
    cb = _cube(out)
    _check(lib().xv_decode_cube(enc.handle, C.byref(cb), _stream_handle(stream)))
    return out


def decode_batch(encs, outs, stream=None):
    n = len(encs)
    hs = (C.c_void_p * n)(*[e.handle.value for e in encs])
    cbs = (Cube * n)(*[_cube(o) for o in outs])
    _check(lib().xv_decode_batch(n, hs, cbs, _stream_handle(stream)))
    return outs


def psnr_bpppb(orig, enc: Encoded, stream=None) -> dict:
    """xv_psnr_bpppb; orig may be None (no physical-domain PSNR)."""
    m = MetricsC()
    cp = C.byref(_cube(orig)) if orig is not None else None
    _check(lib().xv_psnr_bpppb(cp, enc.handle, C.byref(m), _stream_handle(stream)))
    return _metrics_dict(m)


def psnr_bpppb_batch(origs, encs, stream=None) -> list:
    """xv_psnr_bpppb_batch: metrics of several encodes, one synchronisation;
    origs may be None (no physical-domain PSNR)."""
    n = len(encs)
    ms = (MetricsC * n)()
    hs = (C.c_void_p * n)(*[e.handle for e in encs])
    cbs = (Cube * n)(*[_cube(c) for c in origs]) if origs is not None else None
    _check(lib().xv_psnr_bpppb_batch(n, cbs, hs, ms, _stream_handle(stream)))
    return [_metrics_dict(m) for m in ms]


def _metrics_dict(m) -> dict:
    Bn, G = m.bands, m.groups
    return dict(psnr=list(m.psnr[:Bn]), psnr_phys=list(m.psnr_phys[:Bn]),
                sse_phys=list(m.sse_phys[:Bn]), sse=list(m.sse[:Bn]),
                n_valid=list(m.n_valid[:Bn]), band_min=list(m.band_min[:Bn]),
                band_max=list(m.band_max[:Bn]), coef_bits=m.coef_bits, mv_bits=m.mv_bits,
                header_bits=m.header_bits, bpppb=m.bpppb,
                bpppb_group=list(m.bpppb_group[:G]))


def ssim(enc: Encoded, stream=None) -> list:
    """xv_ssim: per-band mean SSIM of the coded planes (NaN below 11 x 11)."""
    out = (C.c_double * MAX_BANDS)()
    _check(lib().xv_ssim(enc.handle, out, _stream_handle(stream)))
    return list(out[:enc.shape[-1]])


def spectral_angle(orig, decoded, stream=None):
    """xv_spectral_angle: (mean angle in radians, pixels used)."""
    v = C.c_double()
    n = C.c_uint64()
    _check(lib().xv_spectral_angle(C.byref(_cube(orig)), C.byref(_cube(decoded)), C.byref(v),
                                   C.byref(n), _stream_handle(stream)))
    return v.value, int(n.value)


def spectral_angle_noalloc(orig, decoded, stream=None):
    """xv_spectral_angle_noalloc: as spectral_angle, with the library's static
    scratch array instead of any allocation."""
    v = C.c_double()
    n = C.c_uint64()
    _check(lib().xv_spectral_angle_noalloc(C.byref(_cube(orig)), C.byref(_cube(decoded)),
                                           C.byref(v), C.byref(n), _stream_handle(stream)))
    return v.value, int(n.value)


def set_graph_mode(on: bool):
    """xv_set_graph_mode: replay captured graphs of the batched step loops."""
    _check(lib().xv_set_graph_mode(1 if on else 0))


def get_graph_mode() -> bool:
    return bool(lib().xv_get_graph_mode())


class Pca:
    """xv_pca_*: principal components of a u16 device cube's bands."""

    def __init__(self, cube, stream=None):
        self._h = C.c_void_p()
        _check(lib().xv_pca_fit(C.byref(_cube(cube)), _stream_handle(stream), C.byref(self._h)))
        b = C.c_int32()
        _check(lib().xv_pca_view(self._h, C.byref(b), None, None, None, None))
        self.bands = b.value

    def view(self) -> dict:
        """Host copies: mean [bands], cov [bands][bands], eigval [bands] and
        basis [bands][bands] (column j = PC j)."""
        n = self.bands
        mean = np.zeros(n, np.float64)
        cov = np.zeros((n, n), np.float64)
        ev = np.zeros(n, np.float64)
        basis = np.zeros((n, n), np.float64)
        _check(lib().xv_pca_view(self._h, None, mean.ctypes.data_as(C.c_void_p),
                                 cov.ctypes.data_as(C.c_void_p), ev.ctypes.data_as(C.c_void_p),
                                 basis.ctypes.data_as(C.c_void_p)))
        return dict(mean=mean, cov=cov, eigval=ev, basis=basis)

    def project(self, cube, j0, j1, out, stream=None):
        _check(lib().xv_pca_project(self._h, C.byref(_cube(cube)), j0, j1, C.byref(_cube(out)),
                                    _stream_handle(stream)))

    def inverse(self, pcs, out, stream=None):
        _check(lib().xv_pca_inverse(self._h, C.byref(_cube(pcs)), C.byref(_cube(out)),
                                    _stream_handle(stream)))

    def free(self):
        if self._h:
            lib().xv_pca_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def set_me_geometry(block: int, search_range: int, blocks_per_wg=0, cands_per_lane=0,
                    threads=0, rows_per_lane=0, layout=0):
    """xv_set_me_geometry; layout is ME_COLUMN_PAIRS, ME_ROW_PAIRS or
    ME_ROW_PAIRS_BY_CHANNEL (0: default)."""
    g = MeGeometryC(blocks_per_wg, cands_per_lane, threads, rows_per_lane, layout)
    _check(lib().xv_set_me_geometry(block, search_range, C.byref(g)))


def get_me_geometry(block: int, search_range: int, width_blocks: int = 0) -> dict:
    g = MeGeometryC()
    _check(lib().xv_get_me_geometry(block, search_range, width_blocks, C.byref(g)))
    return dict(blocks_per_wg=g.blocks_per_wg, cands_per_lane=g.cands_per_lane,
                threads=g.threads, rows_per_lane=g.rows_per_lane, layout=g.layout)


def set_me_split_geometry(block: int, search_range: int, blocks_per_wg=0, cands_per_lane=0,
                          threads=0, rows_per_lane=0, layout=0):
    """xv_set_me_split_geometry: the adaptive block size's search (row-pair
    layouts, 5, 7, 11 or 13 candidates per lane; all zero: default)."""
    g = MeGeometryC(blocks_per_wg, cands_per_lane, threads, rows_per_lane, layout)
    _check(lib().xv_set_me_split_geometry(block, search_range, C.byref(g)))


def get_me_split_geometry(block: int, search_range: int, width_blocks: int = 0) -> dict:
    g = MeGeometryC()
    _check(lib().xv_get_me_split_geometry(block, search_range, width_blocks, C.byref(g)))
    return dict(blocks_per_wg=g.blocks_per_wg, cands_per_lane=g.cands_per_lane,
                threads=g.threads, rows_per_lane=g.rows_per_lane, layout=g.layout)


def autotune_me(cube, params: Params, stream=None, max_candidates: int = 0) -> dict:
    """xv_autotune_me: time candidate motion-search geometries on the cube's
    first P step and install the fastest for (block, search_range)."""
    cb = _cube(cube)
    pc = params.c()
    g = MeGeometryC()
    ms = C.c_double()
    _check(lib().xv_autotune_me(C.byref(cb), C.byref(pc), _stream_handle(stream), max_candidates,
                                C.byref(g), C.byref(ms)))
    return dict(blocks_per_wg=g.blocks_per_wg, cands_per_lane=g.cands_per_lane,
                threads=g.threads, rows_per_lane=g.rows_per_lane, layout=g.layout,
                kernel_ms=ms.value)


def autotune_me_batch(cubes, params, stream=None, max_candidates: int = 0) -> dict:
    """xv_autotune_me_batch: tune on the first P step of the batch as
    encode_batch would launch it (cubes share block and search_range)."""
    n = len(cubes)
    cbs = (Cube * n)(*[_cube(c) for c in cubes])
    pcs = (ParamsC * n)(*[p.c() for p in params])
    g = MeGeometryC()
    ms = C.c_double()
    _check(lib().xv_autotune_me_batch(n, cbs, pcs, _stream_handle(stream), max_candidates,
                                      C.byref(g), C.byref(ms)))
    return dict(blocks_per_wg=g.blocks_per_wg, cands_per_lane=g.cands_per_lane,
                threads=g.threads, rows_per_lane=g.rows_per_lane, layout=g.layout,
                kernel_ms=ms.value)


def profile_enable(on: bool = True):
    _check(lib().xv_profile_enable(1 if on else 0))


def profile_select(classes=None):
    """xv_profile_select: time only the given kernel classes (K_* indices);
    None times all of them."""
    mask = 0 if not classes else sum(1 << k for k in classes)
    _check(lib().xv_profile_select(mask))


def profile_read() -> dict:
    p = ProfileC()
    _check(lib().xv_profile_read(C.byref(p)))
    return {K_NAMES[i]: dict(ms=p.ms[i], launches=p.launches[i], work=p.work[i])
            for i in range(len(K_NAMES))}


class Packed:
    """A serialised encoded cube (xv_pack): one device buffer."""

    def __init__(self, handle, shape, params):
        self.handle = handle
        self.shape = shape
        self.params = params
        self._freed = False

    def view(self) -> dict:
        d = C.c_void_p()
        n = C.c_uint64()
        bits = C.c_uint64()
        _check(lib().xv_packed_view(self.handle, C.byref(d), C.byref(n), C.byref(bits)))
        return dict(ptr=d.value, bytes=n.value, payload_bits=bits.value)

    def tensor(self):
        """The buffer as a uint8 device tensor (a view; valid while self lives)."""
        import torch
        v = self.view()

        class _CAI:
            __cuda_array_interface__ = dict(shape=(v["bytes"],), typestr="|u1",
                                            data=(v["ptr"], False), version=3)
        return torch.as_tensor(_CAI(), device="cuda")

    def free(self):
        if not self._freed:
            lib().xv_packed_free(self.handle)
            self._freed = True

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pack(enc: "Encoded", stream=None) -> Packed:
    """xv_pack: serialise an encoded cube (header, metric span, segment index,
    Exp-Golomb payload)."""
    h = C.c_void_p()
    _check(lib().xv_pack(enc.handle, _stream_handle(stream), C.byref(h)))
    return Packed(h, enc.shape, enc.params)


def unpack(buf, stream=None, shape=None, params=None) -> "Encoded":
    """xv_unpack: parse a serialised cube held in a uint8 device tensor."""
    h = C.c_void_p()
    _check(lib().xv_unpack(C.c_void_p(buf.data_ptr()), buf.numel(), _stream_handle(stream),
                           C.byref(h)))
    return Encoded(h, shape, params)


def memory_read() -> dict:
    """xv_memory_read: bytes held by live objects, cached for reuse, and the peak."""
    m = MemoryC()
    _check(lib().xv_memory_read(C.byref(m)))
    return dict(live_bytes=m.live_bytes, cached_bytes=m.cached_bytes, peak_bytes=m.peak_bytes)


def cache_release() -> int:
    """xv_cache_release: return every cached device block to the runtime."""
    n = C.c_uint64(0)
    _check(lib().xv_cache_release(C.byref(n)))
    return n.value


class Server:
    """Continuous-batching encode/decode server (xv_server_*)."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 0, max_queue: int = 0, stream=None):
        cfg = ServerCfgC(hbm_budget, max_slots, max_queue,
                         None if stream is None else _stream_handle(stream))
        h = C.c_void_p()
        _check(lib().xv_server_create(C.byref(cfg), C.byref(h)))
        self.handle = h
        self._keep = {}  # device buffers referenced by in-flight requests

    def submit_encode(self, cube, params: Params) -> int:
        rq = RequestC(OP_ENCODE, 0, _cube(cube), params.c(), None)
        t = C.c_uint64()
        _check(lib().xv_server_submit(self.handle, C.byref(rq), C.byref(t)))
        self._keep[t.value] = (cube, params)
        return t.value

    def submit_decode(self, enc: "Encoded", out) -> int:
        rq = RequestC(OP_DECODE, 0, _cube(out), ParamsC(), enc.handle)
        t = C.c_uint64()
        _check(lib().xv_server_submit(self.handle, C.byref(rq), C.byref(t)))
        self._keep[t.value] = (enc, out)
        return t.value

    def _result(self, ticket, r: ResultC):
        kept = self._keep.pop(ticket, None)
        enc = None
        if r.enc:
            cube, params = kept
            enc = Encoded(C.c_void_p(r.enc), tuple(cube.shape), params)
        return dict(status=r.status, op=r.op, enc=enc, submit_ms=r.submit_ms,
                    admit_ms=r.admit_ms, done_ms=r.done_ms)

    def poll(self, ticket: int):
        r = ResultC()
        rc = lib().xv_server_poll(self.handle, ticket, C.byref(r))
        if rc == EPENDING:
            return None
        _check(rc)
        return self._result(ticket, r)

    def wait(self, ticket: int) -> dict:
        r = ResultC()
        _check(lib().xv_server_wait(self.handle, ticket, C.byref(r)))
        return self._result(ticket, r)

    def cancel(self, ticket: int):
        _check(lib().xv_server_cancel(self.handle, ticket))

    def stats(self) -> dict:
        st = ServerStatsC()
        _check(lib().xv_server_stats_read(self.handle, C.byref(st)))
        return {k: getattr(st, k) for k, _ in ServerStatsC._fields_ if k != "reserved"}

    def close(self):
        if self.handle:
            lib().xv_server_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
