"""Seeded synthetic cubes standing in for the paper's datasets.

The paper benchmarks on DynamicEarthNet, DeepExtremeCubes and ERA5 (Sec. II-B),
none of which is available here.  These generators produce cubes of the same
shapes, dtypes and value structure: smooth spatial fields with a power-law
spectrum, temporal drift or seasonality, cloud gaps (NaN) for the
Sentinel-2-like cube, piecewise-constant land-cover patches for the
Planet-like cube, and a diurnal cycle with a latitude gradient for the
reanalysis-like cube.  They hold none of the coding arithmetic; the tests feed
the same cube to the GPU path and to the oracle.

Every generator is a pure function of its seed and of the torch device it runs
on (torch's CPU and GPU random streams differ, so a cube is regenerated on the
device where it is used and copied to the host for the oracle).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch


def grf(shape_hw, beta: float, n: int, gen: torch.Generator, device) -> torch.Tensor:
    """n independent standardised 2-D Gaussian random fields with power
    spectrum |f|^-beta (zero mean), float32 [n, H, W]."""
    H, W = shape_hw
    fy = torch.fft.fftfreq(H, device=device).view(H, 1)
    fx = torch.fft.rfftfreq(W, device=device).view(1, W // 2 + 1)
    f = torch.sqrt(fx * fx + fy * fy)
    amp = torch.where(f > 0, f.clamp_min(1e-12) ** (-beta / 2.0), torch.zeros_like(f))
    re = torch.randn((n, H, W // 2 + 1), generator=gen, device=device)
    im = torch.randn((n, H, W // 2 + 1), generator=gen, device=device)
    spec = torch.complex(re, im) * amp
    field = torch.fft.irfft2(spec, s=(H, W))
    field = field - field.mean(dim=(1, 2), keepdim=True)
    std = field.std(dim=(1, 2), keepdim=True).clamp_min(1e-12)
    return (field / std).float()


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


# ---------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    T: int
    H: int
    W: int
    bands: int
    dtype: str  # "u16" or "f32"
    bit_depth: int
    qps: tuple
    blocks: tuple
    search_range: int
    gop: int = 16
    pad_mode: int = 0   # 0 zero channel, 1 repeat last band
    fill_mode: int = 0  # 0 nearest valid time, 1 forward

    @property
    def px_band(self) -> int:
        return self.T * self.H * self.W * self.bands


WORKLOADS = {
    # 16 x 64x64 x 3, AR(1) fields, 10-bit, N=8, R=8, QP 27
    "tiny": Workload("tiny", 16, 64, 64, 3, "u16", 10, (27,), (8,), 8),
    # 500 x 128x128 x 6 f32 with cloud gaps, 12-bit, QP x N sweep, R=16
    "s2cloud": Workload("s2cloud", 500, 128, 128, 6, "f32", 12, (17, 22, 27, 32, 37),
                        (8, 16, 32), 16),
    # 730 x 1024x1024 x 4 u16 land-cover patches, 10-bit, N=16, R=32, zero pad
    "planet": Workload("planet", 730, 1024, 1024, 4, "u16", 10, (22, 32), (16,), 32),
    # 744 x 721x1440 x 3 f32 reanalysis-like, 12-bit, N=32, R=8
    "era5": Workload("era5", 744, 721, 1440, 3, "f32", 12, (17, 27), (32,), 8),
    # 128 x 256x256 x 3 u16 texture drifting by fractions of a sample per
    # frame, 10-bit, N=16, R=16 (the content sub-sample motion is for)
    "drift": Workload("drift", 128, 256, 256, 3, "u16", 10, (22, 27, 32, 37), (16,), 16),
}


# ---------------------------------------------------------------------------
# Generators
# ---------------------------------------------------------------------------

def tiny_cube(seed: int = 0, T: int = 16, H: int = 64, W: int = 64, bands: int = 3,
              device="cpu") -> torch.Tensor:
    """Per band an AR(1) sequence of 1/f^2 fields (rho = 0.95); the whole cube
    min-max mapped to [0, 10000] and rounded to uint16.  [T, H, W, bands]."""
    gen = _gen(seed, device)
    rho = 0.95
    z = grf((H, W), 2.0, bands, gen, device)
    frames = []
    for _ in range(T):
        frames.append(z)
        z = rho * z + math.sqrt(1 - rho * rho) * grf((H, W), 2.0, bands, gen, device)
    cube = torch.stack(frames, 0).permute(0, 2, 3, 1).contiguous()  # T H W B
    lo, hi = cube.min(), cube.max()
    cube = torch.round((cube - lo) / (hi - lo) * 10000.0)
    return cube.to(torch.int32).to(torch.uint16)


def _to_u16(x: torch.Tensor) -> torch.Tensor:
    return x.clamp(0, 65535).round().to(torch.int32).to(torch.uint16)


def s2cloud_cube(seed: int = 1, T: int = 500, H: int = 128, W: int = 128, bands: int = 6,
                 cloud_frac: float = 0.10, device="cpu") -> torch.Tensor:
    """Sentinel-2-like reflectance cube, float32 [T, H, W, bands] holding integers
    0..10000 and NaN under clouds.  Per band: a static 1/f^2 field, a seasonal
    sinusoid (5-day cadence) whose phase varies smoothly in space, and per-pixel
    AR(1) noise (rho = 0.95).  Clouds: per frame, discs of radius 4..20 px at
    uniform centres are added until at least cloud_frac of the frame is
    covered; the mask is shared by all bands."""
    gen = _gen(seed, device)
    base = 3000.0 + 1200.0 * grf((H, W), 2.0, bands, gen, device)          # B H W
    phase = 0.6 * grf((H, W), 3.0, 1, gen, device)[0]                       # H W
    amp = 400.0 + 400.0 * torch.rand((bands, 1, 1), generator=gen, device=device)
    rho = 0.95
    noise = 150.0 * torch.randn((bands, H, W), generator=gen, device=device)
    yy = torch.arange(H, device=device).view(H, 1).float()
    xx = torch.arange(W, device=device).view(1, W).float()
    out = torch.empty((T, H, W, bands), dtype=torch.float32, device=device)
    for t in range(T):
        season = torch.sin(2 * math.pi * 5.0 * t / 365.25 + phase)          # H W
        frame = base + amp * season + noise                                   # B H W
        frame = frame.clamp(0, 10000).round()
        mask = torch.zeros((H, W), dtype=torch.bool, device=device)
        while mask.float().mean().item() < cloud_frac:
            r = int(torch.randint(4, 21, (1,), generator=gen, device=device).item())
            cy = float(torch.rand((1,), generator=gen, device=device).item() * H)
            cx = float(torch.rand((1,), generator=gen, device=device).item() * W)
            mask |= (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
        frame = torch.where(mask.unsqueeze(0), torch.full_like(frame, float("nan")), frame)
        out[t] = frame.permute(1, 2, 0)
        noise = rho * noise + math.sqrt(1 - rho * rho) * 150.0 * torch.randn(
            (bands, H, W), generator=gen, device=device)
    return out


def planet_cube(seed: int = 2, T: int = 730, H: int = 1024, W: int = 1024, bands: int = 4,
                cells: int = 256, classes: int = 64, device="cpu",
                t_begin: int = 0, t_end: int | None = None) -> torch.Tensor:
    """Planet-like uint16 cube [T, H, W, bands]: Voronoi land-cover patches
    (uniform seeds, one of `classes` classes each with per-band means
    U(500, 9000)), a static 1/f^2 texture (sigma 300), a per-patch linear trend
    N(0, 1) per day, a fresh weak 1/f^2 field per frame (sigma 60) and a
    per-frame integer registration jitter of up to 2 px, clipped to
    [0, 10000].  Frames t_begin..t_end-1 can be generated alone (the same
    values as inside the full cube)."""
    t_end = T if t_end is None else t_end
    gen = _gen(seed, device)
    sy = torch.rand((cells,), generator=gen, device=device) * H
    sx = torch.rand((cells,), generator=gen, device=device) * W
    cls = torch.randint(0, classes, (cells,), generator=gen, device=device)
    means = 500.0 + 8500.0 * torch.rand((classes, bands), generator=gen, device=device)
    trend = torch.randn((cells, bands), generator=gen, device=device)
    tex = 300.0 * grf((H, W), 2.0, bands, gen, device).permute(1, 2, 0)      # H W B
    jit = torch.randint(-2, 3, (T, 2), generator=gen, device=device)
    # nearest seed per pixel, in row chunks
    cell = torch.empty((H, W), dtype=torch.long, device=device)
    xx = torch.arange(W, device=device).float().view(1, W, 1)
    for y0 in range(0, H, 64):
        yy = torch.arange(y0, min(H, y0 + 64), device=device).float().view(-1, 1, 1)
        d = (yy - sy.view(1, 1, -1)) ** 2 + (xx - sx.view(1, 1, -1)) ** 2
        cell[y0:y0 + yy.shape[0]] = d.argmin(dim=2)
    static = means[cls[cell]] + tex                                          # H W B
    tr = trend[cell]                                                          # H W B
    out = torch.empty((t_end - t_begin, H, W, bands), dtype=torch.uint16, device=device)
    for t in range(T):
        # the per-frame field is drawn for every t so that a slab matches the
        # full cube exactly
        weak = 60.0 * grf((H, W), 2.0, bands, gen, device).permute(1, 2, 0)
        if t < t_begin or t >= t_end:
            continue
        f = static + tr * float(t) + weak
        f = torch.roll(f, shifts=(int(jit[t, 0]), int(jit[t, 1])), dims=(0, 1))
        out[t - t_begin] = _to_u16(f.clamp(0, 10000))
    return out


def era5_cube(seed: int = 3, T: int = 744, H: int = 721, W: int = 1440, bands: int = 3,
              device="cpu", t_begin: int = 0, t_end: int | None = None) -> torch.Tensor:
    """Reanalysis-like float32 cube [T, H, W, bands], hourly: per variable an
    offset, a cos(latitude) gradient, a 24-h diurnal cycle whose phase follows
    longitude, and an AR(1)-evolving 1/f^3 field.  Variables are
    temperature-like (200..320 K), humidity-like (0..100) and wind-like
    (0..40, positive)."""
    t_end = T if t_end is None else t_end
    gen = _gen(seed, device)
    lat = torch.linspace(90.0, -90.0, H, device=device).view(H, 1) * math.pi / 180.0
    lon = torch.linspace(0.0, 360.0, W + 1, device=device)[:W].view(1, W) * math.pi / 180.0
    spec = [  # offset, gradient, diurnal, field sigma, lo, hi
        (220.0, 75.0, 3.0, 6.0, 200.0, 320.0),
        (35.0, 30.0, 8.0, 14.0, 0.0, 100.0),
        (12.0, -6.0, 2.0, 5.0, 0.0, 40.0),
    ]
    rho = 0.98
    z = grf((H, W), 3.0, bands, gen, device)
    out = torch.empty((t_end - t_begin, H, W, bands), dtype=torch.float32, device=device)
    for t in range(T):
        if t >= t_begin and t < t_end:
            chans = []
            for b in range(bands):
                off, grad, di, sig, lo, hi = spec[b % 3]
                v = off + grad * torch.cos(lat) + di * torch.cos(2 * math.pi * t / 24.0 + lon) \
                    + sig * z[b]
                if b % 3 == 2:
                    v = v.abs()
                chans.append(v.clamp(lo, hi))
            out[t - t_begin] = torch.stack(chans, -1)
        z = rho * z + math.sqrt(1 - rho * rho) * grf((H, W), 3.0, bands, gen, device)
        if t + 1 >= t_end:
            break
    return out


def drift_cube(seed: int = 5, T: int = 128, H: int = 256, W: int = 256, bands: int = 3,
               velocity=(0.37, -0.23), device="cpu") -> torch.Tensor:
    """uint16 cube [T, H, W, bands] of a periodic 1/f^3 texture per band
    translated by t * velocity samples (x, y) in frame t -- an exact
    sub-sample shift, applied as a phase ramp on the texture's spectrum --
    scaled to a peak excursion of 4800 about 5000, plus white noise (sigma
    8), clipped to [0, 10000] and rounded: the motion of a registration
    drift or an advected field, which integer vectors only approximate."""
    gen = _gen(seed, device)
    fy = torch.fft.fftfreq(H, device=device).view(H, 1)
    fx = torch.fft.rfftfreq(W, device=device).view(1, W // 2 + 1)
    f = torch.sqrt(fx * fx + fy * fy)
    amp = torch.where(f > 0, f.clamp_min(1e-12) ** -1.5, torch.zeros_like(f))
    spec = torch.complex(torch.randn((bands, H, W // 2 + 1), generator=gen, device=device),
                         torch.randn((bands, H, W // 2 + 1), generator=gen, device=device)) * amp
    base = torch.fft.irfft2(spec, s=(H, W))
    scale = 4800.0 / base.abs().amax(dim=(1, 2), keepdim=True).clamp_min(1e-12)
    vx, vy = velocity
    out = torch.empty((T, H, W, bands), dtype=torch.uint16, device=device)
    for t in range(T):
        ph = torch.exp(torch.complex(torch.zeros_like(f), -2 * math.pi * (fx * vx * t + fy * vy * t)))
        frame = torch.fft.irfft2(spec * ph, s=(H, W)) * scale + 5000.0
        frame = frame + 8.0 * torch.randn((bands, H, W), generator=gen, device=device)
        out[t] = _to_u16(frame.clamp(0, 10000)).permute(1, 2, 0)
    return out


def make_cube(name: str, device="cpu", **kw) -> torch.Tensor:
    if name == "tiny":
        return tiny_cube(device=device, **kw)
    if name == "s2cloud":
        return s2cloud_cube(device=device, **kw)
    if name == "planet":
        return planet_cube(device=device, **kw)
    if name == "era5":
        return era5_cube(device=device, **kw)
    if name == "drift":
        return drift_cube(device=device, **kw)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Serving mix: request trace
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Request:
    idx: int
    op: str          # "encode" or "decode"
    T: int
    S: int           # H = W = S
    bands: int
    qp: int
    seed: int
    arrival_s: float


def request_trace(n: int = 4096, rate_per_s: float = 100.0, seed: int = 4,
                  t_range=(16, 730), s_range=(64, 1024)) -> list:
    """n requests with Poisson arrivals at rate_per_s: encode or decode with
    p = 1/2; T log-uniform in t_range, side S log-uniform in s_range rounded
    to a multiple of 32; bands from {3, 4, 6}; QP uniform in 17..37."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n)
    at = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(n):
        T = int(round(math.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1])))))
        S = int(round(math.exp(rng.uniform(math.log(s_range[0]), math.log(s_range[1]))) / 32)) * 32
        S = max(32, S)
        reqs.append(Request(i, "encode" if rng.random() < 0.5 else "decode", T, S,
                            int(rng.choice([3, 4, 6])), int(rng.integers(17, 38)),
                            4_000_000 + i, float(at[i])))
    return reqs
