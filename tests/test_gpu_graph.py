"""Graph replay of the batched step loops (xv_set_graph_mode): every replay
equals the eager launches bit for bit, with the program's own eager work and
synchronisations between replays; a batch of the same shape but other data
replays the same graph on its own buffers; other shapes capture their own
graphs; timing falls back to eager launches."""
import numpy as np
import pytest
import torch

from paper_2506_19656_amd import xv
from test_gpu_parity import _textured

pytestmark = pytest.mark.gpu


def _digest(enc):
    h = enc.host()
    return [h[k].tobytes() for k in ("levels", "mvs", "recon", "coef_bits", "mv_bits", "sse")]


def _batch(seed):
    hosts = [_textured(7, 40, 56, 4, seed=seed), _textured(5, 48, 40, 3, seed=seed + 1),
             _textured(9, 33, 70, 6, seed=seed + 2, dtype=np.float32, nan_frac=0.03)]
    cubes = [torch.from_numpy(h).cuda() for h in hosts]
    params = [xv.Params(bit_depth=10, qp=22, block=8, search_range=4, gop=4),
              xv.Params(bit_depth=10, qp=30, block=8, search_range=4, gop=3,
                        flags=xv.FLAG_QPEL),
              xv.Params(bit_depth=12, qp=27, block=16, search_range=6, gop=4)]
    return cubes, params


def _eager(cubes, params):
    xv.set_graph_mode(False)
    encs = xv.encode_batch(cubes, params)
    outs = [torch.empty_like(c) for c in cubes]
    xv.decode_batch(encs, outs)
    torch.cuda.synchronize()
    return [_digest(e) for e in encs], outs


def test_replays_equal_eager_launches():
    cubes, params = _batch(100)
    ref, ref_out = _eager(cubes, params)
    other_cubes, _ = _batch(200)  # same shapes, other data
    other_ref, other_out = _eager(other_cubes, params)
    xv.set_graph_mode(True)
    try:
        for rep in range(4):
            print(f"[case] graph replay {rep}", flush=True)
            cs = cubes if rep % 2 == 0 else other_cubes
            want, want_out = (ref, ref_out) if rep % 2 == 0 else (other_ref, other_out)
            encs = xv.encode_batch(cs, params)
            outs = [torch.empty_like(c) for c in cs]
            xv.decode_batch(encs, outs)
            # eager work of the program between replays
            plain = xv.encode_cube(cs[0], params[0])
            _ = (cs[1].float() * 2).sum().item()
            torch.cuda.synchronize()
            assert [_digest(e) for e in encs] == want, rep
            for a, b in zip(outs, want_out):
                assert torch.equal(a, b), rep
            assert _digest(plain) == want[0]
            for e in encs:
                e.free()
            plain.free()
        # another shape captures its own graph
        small = [c[:3].contiguous() for c in cubes]
        xv.set_graph_mode(False)
        e_ref = [_digest(e) for e in xv.encode_batch(small, params)]
        xv.set_graph_mode(True)
        assert [_digest(e) for e in xv.encode_batch(small, params)] == e_ref
        # timing on: eager launches, every class timed
        xv.profile_enable(True)
        encs = xv.encode_batch(cubes, params)
        torch.cuda.synchronize()
        prof = xv.profile_read()
        xv.profile_enable(False)
        assert prof["me"]["launches"] > 0 and prof["encode"]["launches"] > 0
        assert [_digest(e) for e in encs] == ref
    finally:
        xv.set_graph_mode(False)
        xv.cache_release()
