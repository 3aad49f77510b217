"""The continuous-batching server: every result is the same alone and in the
mix, admission respects the memory budget, cancellation and shutdown with
work in flight behave."""
import hashlib
import time

import numpy as np
import pytest
import torch

from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv

pytestmark = pytest.mark.gpu


def _digest(enc: xv.Encoded) -> str:
    ex = enc.export()
    h = hashlib.sha256()
    for k in ("levels", "mvs", "coef_bits", "mv_bits", "sse"):
        t = ex[k]
        if t is not None:
            h.update(t.cpu().numpy().tobytes())
    return h.hexdigest()


def _mix(n, seed=7):
    """Mixed-size request cubes (sizes, bands, QPs, block sizes) on the GPU."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        T = int(rng.integers(3, 20))
        S = int(rng.choice([32, 48, 64, 96]))
        Bn = int(rng.choice([3, 4, 6]))
        cube = synth.tiny_cube(seed=1000 + i, T=T, H=S, W=S + 16, bands=Bn, device="cuda")
        p = xv.Params(bit_depth=10, qp=int(rng.integers(17, 38)), block=int(rng.choice([8, 16])),
                      search_range=int(rng.choice([4, 8])), gop=int(rng.choice([4, 8, 16])),
                      flags=xv.FLAG_DROP_WORK)
        out.append((cube, p))
    return out


def test_each_result_is_the_same_alone_and_in_the_mix():
    mix = _mix(24)
    alone = [_digest(xv.encode_cube(c, p)) for c, p in mix]
    sv = xv.Server(max_slots=8)
    tickets = []
    for i, (c, p) in enumerate(mix):
        tickets.append(sv.submit_encode(c, p))
        if i % 5 == 4:
            time.sleep(0.002)  # arrivals while others are on the GPU
    results = [sv.wait(t) for t in tickets]
    st = sv.stats()
    for (r, a) in zip(results, alone):
        assert r["status"] == xv.OK
        assert _digest(r["enc"]) == a
        assert r["submit_ms"] <= r["admit_ms"] <= r["done_ms"]
    assert st["completed"] == len(mix) and st["failed"] == 0
    assert st["peak_active"] > 1  # requests overlapped on the device
    # iterations launch the next step of every resident request together
    total_steps = sum(min(p.gop, c.shape[0]) for c, p in mix)
    assert st["iterations"] < total_steps
    # decode requests, mixed with encodes
    encs = [r["enc"] for r in results[:8]]
    outs = [torch.empty_like(c) for c, _ in mix[:8]]
    ref = []
    for e, (c, _) in zip(encs, mix[:8]):
        o = torch.empty_like(c)
        xv.decode_cube(e, o)
        ref.append(o)
    tk = [sv.submit_decode(e, o) for e, o in zip(encs, outs)]
    tk2 = [sv.submit_encode(c, p) for c, p in mix[8:12]]
    for t in tk:
        assert sv.wait(t)["status"] == xv.OK
    for t, a in zip(tk2, alone[8:12]):
        assert _digest(sv.wait(t)["enc"]) == a
    torch.cuda.synchronize()
    for o, r in zip(outs, ref):
        assert torch.equal(o, r)
    sv.close()


def test_budget_admission_and_oversized_request():
    mix = _mix(10, seed=9)
    sizes = []
    for c, p in mix:
        T, H, W, Bn = c.shape
        G = (Bn + 2) // 3
        Hp, Wp = -(-H // p.block) * p.block, -(-W // p.block) * p.block
        sizes.append(G * T * 3 * Hp * Wp * 2 * 3)  # levels + frames + recon, lower bound
    budget = int(max(sizes) * 1.6)
    sv = xv.Server(hbm_budget=budget, max_slots=16)
    tickets = [sv.submit_encode(c, p) for c, p in mix]
    big = synth.tiny_cube(seed=5, T=40, H=256, W=256, bands=6, device="cuda")
    tb = sv.submit_encode(big, xv.Params(block=8, search_range=4, gop=8))
    for t in tickets:
        assert sv.wait(t)["status"] == xv.OK
    assert sv.wait(tb)["status"] == xv.ENOMEM
    st = sv.stats()
    assert st["peak_bytes"] <= budget
    assert st["failed"] == 1
    sv.close()


def test_cancel_queued_requests_and_destroy_with_work_in_flight():
    mix = _mix(12, seed=11)
    sv = xv.Server(max_slots=1)
    tickets = [sv.submit_encode(c, p) for c, p in mix]
    for t in tickets[4:]:
        sv.cancel(t)
    statuses = [sv.wait(t)["status"] for t in tickets]
    assert all(s == xv.OK for s in statuses[:1])
    assert sum(s == xv.ECANCELED for s in statuses) >= len(tickets) - 5
    with pytest.raises(xv.XvError):
        sv.poll(tickets[0])  # retired ticket
    # submit more and destroy while they run: the server drains
    more = [sv.submit_encode(c, p) for c, p in mix[:6]]
    assert len(more) == 6
    sv.close()
    torch.cuda.synchronize()
