"""GPU parity of the principal components of the bands (xv_pca_*) against
the oracle: the moments, covariance, eigenvalues and basis bit-exact (exact
integer sums on the GPU, the same binary64 chain on the host), the PC cube
bit-exact, the coding of a PC cube through the ordinary path bit-exact, and
the inverse of the decoded PCs bit-exact; band counts 1 to 30 (one to
several sums per thread), cubes spanning many blocks, and the error paths."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv
from test_gpu_parity import check_cube

pytestmark = pytest.mark.gpu


def _bands_cube(T, H, W, Bn, seed):
    """Correlated u16 bands: a few smooth latent fields mixed into Bn bands."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    lat = []
    for k in range(3):
        ph = rng.uniform(0, 6.28, 2)
        lat.append(np.stack([np.sin(xx / (5.0 + 2 * k) + ph[0] + 0.2 * t) *
                             np.cos(yy / (7.0 + k) + ph[1]) for t in range(T)]))
    mix = rng.uniform(-1, 1, (3, Bn))
    x = sum(lat[k][..., None] * mix[k] for k in range(3)) * 1500 + 4000
    x = x + rng.normal(0, 40, x.shape)
    return np.clip(x, 0, 65535).round().astype(np.uint16)


def _fit_parity(host):
    cube = torch.from_numpy(host).cuda()
    pca = xv.Pca(cube)
    v = pca.view()
    mean, cov = O.pca_moments(host)
    ev, basis = O.pca_eigen(cov)
    assert np.array_equal(v["mean"], mean)
    assert np.array_equal(v["cov"], cov)
    assert np.array_equal(v["eigval"], ev)
    assert np.array_equal(v["basis"], basis)
    return cube, pca, mean, basis


@pytest.mark.parametrize("Bn", [1, 2, 4, 10, 13, 30])
def test_fit_and_projection_bit_exact(Bn):
    host = _bands_cube(5, 33, 47, Bn, seed=Bn)
    print(f"[case] pca fit {host.shape}", flush=True)
    cube, pca, mean, basis = _fit_parity(host)
    for j0, j1 in ((0, Bn), (0, min(3, Bn)), (Bn - 1, Bn)):
        out = torch.empty(host.shape[:3] + (j1 - j0,), dtype=torch.float32, device="cuda")
        pca.project(cube, j0, j1, out)
        ref = O.pca_project(host, mean, basis, j0, j1)
        assert np.array_equal(out.cpu().numpy(), ref), (j0, j1)
    # every PC back to the integers, and a truncated inverse in both dtypes
    pcs = torch.empty(host.shape[:3] + (Bn,), dtype=torch.float32, device="cuda")
    pca.project(cube, 0, Bn, pcs)
    back = torch.empty_like(cube)
    pca.inverse(pcs, back)
    assert np.array_equal(back.cpu().numpy(), host)
    k = max(1, Bn - 1)
    for dt, code in ((torch.uint16, O.U16), (torch.float32, O.F32)):
        o = torch.empty(host.shape, dtype=dt, device="cuda")
        pca.inverse(pcs[..., :k].contiguous(), o)
        ref = O.pca_inverse(pcs[..., :k].cpu().numpy(), mean, basis, code)
        assert np.array_equal(o.cpu().numpy(), ref), dt
    pca.free()


def test_moments_over_many_blocks():
    # 2.6 M pixels: the moments kernel runs its full grid of 1024 blocks
    host = _bands_cube(40, 256, 256, 4, seed=77)
    print("[case] pca fit 40x256x256x4", flush=True)
    _fit_parity(host)[1].free()


def test_coding_the_pcs_and_inverting_the_decode():
    """Sec. II-A's example: R, G, B, NIR coded as their first 3 PCs in one
    video.  The PC cube goes through the ordinary coding path; its decode
    goes back to four bands."""
    host = _bands_cube(9, 40, 56, 4, seed=5)
    cube, pca, mean, basis = _fit_parity(host)
    pcs = torch.empty(host.shape[:3] + (3,), dtype=torch.float32, device="cuda")
    pca.project(cube, 0, 3, pcs)
    pcs_ref = O.pca_project(host, mean, basis, 0, 3)
    assert np.array_equal(pcs.cpu().numpy(), pcs_ref)
    p = xv.Params(bit_depth=12, qp=22, block=8, search_range=6, gop=4)
    check_cube("pca 3 PCs of 4 bands", pcs_ref, p)
    enc = xv.encode_cube(pcs, p)
    dec = torch.empty_like(pcs)
    xv.decode_cube(enc, dec)
    op = O.CodingParams(bit_depth=12, qp=22, block=8, search_range=6, gop=4)
    ref = O.encode_cube(pcs_ref, op)
    dq = O.decode_cube(op, pcs_ref.shape, ref["levels"], ref["mvs"])
    dec_ref = O.denormalize_cube(dq, pcs_ref.shape, 8, 12, ref["mn"], ref["mx"], O.F32)
    assert np.array_equal(dec.cpu().numpy(), dec_ref)
    back = torch.empty_like(cube)
    pca.inverse(dec, back)
    assert np.array_equal(back.cpu().numpy(), O.pca_inverse(dec_ref, mean, basis, O.U16))
    # the two dropped-band groups: 3 coded channels instead of 6
    assert enc.export()["levels"].shape[0] == 1
    pca.free()


def test_pca_error_paths():
    host = _bands_cube(2, 16, 16, 4, seed=1)
    cube = torch.from_numpy(host).cuda()
    with pytest.raises(xv.XvError) as ei:
        xv.Pca(cube.to(torch.float32))
    assert ei.value.code == xv.EINVAL
    pca = xv.Pca(cube)
    out = torch.empty((2, 16, 16, 2), dtype=torch.float32, device="cuda")
    for j0, j1 in ((0, 3), (3, 5), (2, 2)):
        with pytest.raises(xv.XvError):
            pca.project(cube, j0, j1, out)
    with pytest.raises(xv.XvError):  # output dtype must be f32
        pca.project(cube, 0, 2, out.to(torch.int32).to(torch.uint16))
    with pytest.raises(xv.XvError):  # more PCs than bands
        pca.inverse(torch.zeros((2, 16, 16, 5), dtype=torch.float32, device="cuda"), cube)
    pca.free()
