"""The allocation-free spectral angle through the C ABI
(xv_spectral_angle_noalloc): the same result as xv_spectral_angle, bit for
bit, on two calls in a row -- the first on a cube whose grid fills the whole
static scratch array, the second on a smaller one -- and on float cubes with
missing samples; the library's device allocator is not touched."""
import numpy as np
import pytest
import torch

from paper_2506_19656_amd import synth
from paper_2506_19656_amd import xv

pytestmark = pytest.mark.gpu


def _decoded(cube, seed):
    """A second cube of the same shape: the first plus small seeded noise."""
    g = torch.Generator(device=cube.device).manual_seed(seed)
    noise = torch.randint(-40, 41, cube.shape, generator=g, device=cube.device)
    if cube.dtype == torch.uint16:
        return (cube.to(torch.int32) + noise).clamp(0, 65535).to(torch.uint16)
    return cube + noise.to(cube.dtype)


def _both(orig, dec):
    ref = xv.spectral_angle(orig, dec)
    torch.cuda.synchronize()
    before = xv.memory_read()
    got = xv.spectral_angle_noalloc(orig, dec)
    torch.cuda.synchronize()
    after = xv.memory_read()
    assert after == before, (before, after)
    return ref, got


def test_noalloc_equals_the_allocating_entry_point_on_two_calls():
    dev = torch.device("cuda:0")
    # 40 x 200 x 300 pixels: the per-block pass runs its largest grid (4096 blocks)
    big = synth.tiny_cube(seed=5, T=40, H=200, W=300, bands=5, device=dev)
    small = synth.tiny_cube(seed=6, T=4, H=30, W=50, bands=3, device=dev)
    print("[case] noalloc spectral angle 40x200x300x5 then 4x30x50x3 u16", flush=True)
    for cube, seed in ((big, 1), (small, 2)):
        dec = _decoded(cube, seed)
        (ref, nref), (got, ngot) = _both(cube, dec)
        assert nref == ngot == cube.shape[0] * cube.shape[1] * cube.shape[2]
        assert np.float64(got).tobytes() == np.float64(ref).tobytes(), (got, ref)
        assert 0.0 < got < 0.1


def test_noalloc_float_cubes_with_missing_samples_and_mixed_dtypes():
    dev = torch.device("cuda:0")
    host = synth.s2cloud_cube(T=8, H=64, W=64, device="cpu")
    cube = host.to(dev)
    dec = torch.nan_to_num(_decoded(cube, 3), nan=100.0)
    print("[case] noalloc spectral angle 8x64x64x6 f32 with gaps", flush=True)
    (ref, nref), (got, ngot) = _both(cube, dec)
    valid = int((~torch.isnan(host).any(dim=3)).sum())
    assert nref == ngot == valid
    assert np.float64(got).tobytes() == np.float64(ref).tobytes()
    # u16 original against a float decode, then the smaller call again
    u = synth.tiny_cube(seed=7, T=6, H=40, W=40, bands=4, device=dev)
    (ref, nref), (got, ngot) = _both(u, _decoded(u.to(torch.float32), 4))
    assert nref == ngot and np.float64(got).tobytes() == np.float64(ref).tobytes()


def test_noalloc_rejects_mismatched_shapes():
    dev = torch.device("cuda:0")
    a = synth.tiny_cube(seed=8, T=2, H=16, W=16, bands=3, device=dev)
    b = synth.tiny_cube(seed=8, T=2, H=16, W=17, bands=3, device=dev)
    with pytest.raises(xv.XvError) as ei:
        xv.spectral_angle_noalloc(a, b)
    assert ei.value.code == xv.EINVAL
