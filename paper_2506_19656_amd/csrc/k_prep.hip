// k_prep.hip -- HBM-bound kernels around the coding loop:
//   stats      per-band NaN-aware min/max (bit-depth conversion, paper Sec. II-A;
//              per-channel PSNR peak, Sec. II-C)
//   pack       conversion to B-bit integers, grouping of bands into 3-channel
//              frames with repeat or zero padding (Sec. II-A), edge padding to a
//              multiple of the block size, and the time fill of missing
//              samples (Sec. III-B; nearest-time or forward)
//   denorm     decoded frames back to the caller's dtype
//   phys_sse   physical-domain squared error per band (Sec. II-C PSNR)
// All floating point is IEEE binary64 with contraction disabled at build time,
// so the conversion is the same chain of correctly rounded operations as its
// mathematical definition.
#include "xv_internal.h"

namespace xv {

namespace {

constexpr int kThreads = 256;

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, unsigned long long v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Order-preserving 32-bit key of a non-NaN float (unsigned order == float order).
__device__ inline uint32_t f32_key(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float key_f32(uint32_t k) {
  uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(u);
}

// Each thread owns one band: element e = gtid + j*stride with stride a
// multiple of the band count, so consecutive lanes read consecutive memory.
__global__ void __launch_bounds__(kThreads) stats_kernel(StatsArgs a) {
  __shared__ uint32_t smin[XV_MAX_BANDS], smax[XV_MAX_BANDS], snan[XV_MAX_BANDS];
  const int bands = a.bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
    snan[i] = 0u;
  }
  __syncthreads();
  const int64_t total = a.npix * bands;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  const int64_t stride = (nthr / bands) * bands;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t lo = 0xffffffffu, hi = 0u, nn = 0u;
  if (gtid < stride) {
    if (a.dtype == XV_U16) {
      const uint16_t* d = (const uint16_t*)a.data;
      for (int64_t e = gtid; e < total; e += stride) {
        uint32_t k = d[e];
        lo = min(lo, k);
        hi = max(hi, k);
      }
    } else {
      const float* d = (const float*)a.data;
      for (int64_t e = gtid; e < total; e += stride) {
        float f = d[e];
        if (f != f) {
          nn++;
          continue;
        }
        uint32_t k = f32_key(f);
        lo = min(lo, k);
        hi = max(hi, k);
      }
    }
    const int b = (int)(gtid % bands);
    atomicMin(&smin[b], lo);
    atomicMax(&smax[b], hi);
    if (nn) atomicAdd(&snan[b], nn);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    if (smin[i] != 0xffffffffu) atomicMin(&a.minkey[i], smin[i]);
    if (smax[i] != 0u) atomicMax(&a.maxkey[i], smax[i]);
    if (snan[i]) {
      atomicAdd(&a.nan_count[i], snan[i]);
      atomicAdd(a.nan_total, snan[i]);
    }
  }
}

// Keys -> binary64 statistics.  A band without a valid sample gets 0, 0.
__global__ void stats_finalize_kernel(StatsArgs a) {
  int b = threadIdx.x;
  if (b >= a.bands) return;
  uint32_t nn = a.nan_count[b];
  bool any = (uint64_t)nn < (uint64_t)a.npix;
  double lo = 0.0, hi = 0.0;
  if (any) {
    if (a.dtype == XV_U16) {
      lo = (double)a.minkey[b];
      hi = (double)a.maxkey[b];
    } else {
      lo = (double)key_f32(a.minkey[b]);
      hi = (double)key_f32(a.maxkey[b]);
    }
  }
  a.mn[b] = lo;
  a.mx[b] = hi;
  a.n_valid[b] = (unsigned long long)(a.npix - (int64_t)nn);
}

// q = floor((x - mn) * L / (mx - mn) + 1/2) clamped to [0, L]; constant band -> 0.
__device__ inline uint16_t convert(double x, double mn, double range, double L) {
  if (range == 0.0) return 0;
  double d = x - mn;
  double num = d * L;
  double v = num / range;
  double q = floor(v + 0.5);
  q = q < 0.0 ? 0.0 : q;
  q = q > L ? L : q;
  return (uint16_t)q;
}

__device__ inline double load_sample(const void* data, int dtype, int64_t i) {
  return dtype == XV_U16 ? (double)((const uint16_t*)data)[i] : (double)((const float*)data)[i];
}

// Gap-free path: one thread per padded pixel (t, y, x); reads the pixel's
// bands (contiguous) and writes one sample to each of the 3G channel planes.
__global__ void __launch_bounds__(kThreads) pack_dense_kernel(PackArgs a) {
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  if (a.dtype == XV_F32 && *a.nan_total != 0u) return;  // gap-filling path runs
  for (int i = threadIdx.x; i < a.bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
  }
  __syncthreads();
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const int64_t total = a.T * plane;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int64_t t = idx / plane;
  const int64_t o = idx - t * plane;
  const int y = (int)(o / a.Wp), x = (int)(o - (int64_t)(o / a.Wp) * a.Wp);
  const int64_t ys = y < a.H ? y : a.H - 1, xs = x < a.W ? x : a.W - 1;
  const int64_t src = ((t * a.H + ys) * a.W + xs) * a.bands;
  const double L = (double)((1 << a.bit_depth) - 1);
  uint16_t last = 0;
  for (int b = 0; b < a.bands; b++) {
    uint16_t q = convert(load_sample(a.data, a.dtype, src + b), smn[b], srg[b], L);
    const int g = b / 3, c = b - 3 * (b / 3);
    a.frames[((int64_t)(g * a.T + t) * 3 + c) * plane + o] = q;
    last = q;
  }
  const int g = a.groups - 1;
  for (int c = a.bands - 3 * g; c < 3; c++)
    a.frames[((int64_t)(g * a.T + t) * 3 + c) * plane + o] =
        a.pad_mode == XV_PAD_REPEAT ? last : (uint16_t)0;
}

// Gap-filling path (float input holding NaN): one thread per (padded pixel,
// band) walks the time series once; each gap is resolved when its end is
// found, choosing the nearest valid time (ties to the earlier one) or the
// last valid value (forward fill; leading gaps take the first valid value).
// A series without any valid sample takes the band minimum.  Also writes the
// validity bytes (real pixel of a real band that was not missing).
__global__ void __launch_bounds__(kThreads) pack_fill_kernel(PackArgs a) {
  if (*a.nan_total == 0u) return;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= plane * a.bands) return;
  const int b = (int)(idx % a.bands);
  const int64_t o = idx / a.bands;
  const int y = (int)(o / a.Wp), x = (int)(o - (int64_t)(o / a.Wp) * a.Wp);
  const int64_t ys = y < a.H ? y : a.H - 1, xs = x < a.W ? x : a.W - 1;
  const bool real = y < a.H && x < a.W;
  const float* d = (const float*)a.data;
  const int64_t fstride = a.H * a.W * a.bands;
  const int64_t src = (ys * a.W + xs) * a.bands + b;
  const double mn = a.mn[b], range = a.mx[b] - a.mn[b];
  const double L = (double)((1 << a.bit_depth) - 1);
  const int g = b / 3, c = b - 3 * g;
  const bool last_band = (b == a.bands - 1);
  const int nch_last = a.bands - 3 * (a.groups - 1);

  auto emit = [&](int64_t t, double v, bool valid) {
    uint16_t q = convert(v, mn, range, L);
    int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
    a.frames[off] = q;
    a.vmask[off] = (uint8_t)(valid && real);
    if (last_band) {
      for (int cc = nch_last; cc < 3; cc++) {
        int64_t po = ((int64_t)(g * a.T + t) * 3 + cc) * plane + o;
        a.frames[po] = a.pad_mode == XV_PAD_REPEAT ? q : (uint16_t)0;
        a.vmask[po] = 0;
      }
    }
  };

  int64_t prevT = -1;
  double prevV = 0.0;
  int64_t t = 0;
  while (t < a.T) {
    float f = d[t * fstride + src];
    if (f == f) {
      emit(t, (double)f, true);
      prevT = t;
      prevV = (double)f;
      t++;
      continue;
    }
    int64_t u = t + 1;
    float fu = 0.f;
    while (u < a.T) {
      fu = d[u * fstride + src];
      if (fu == fu) break;
      u++;
    }
    const bool has_next = u < a.T;
    const double nextV = (double)fu;
    for (int64_t s = t; s < u; s++) {
      double v;
      if (a.fill_mode == XV_FILL_FORWARD) {
        v = prevT >= 0 ? prevV : (has_next ? nextV : mn);
      } else if (prevT >= 0 && has_next) {
        v = (s - prevT <= u - s) ? prevV : nextV;
      } else {
        v = prevT >= 0 ? prevV : (has_next ? nextV : mn);
      }
      emit(s, v, false);
    }
    t = u;
  }
}

__global__ void __launch_bounds__(kThreads) denorm_kernel(DenormArgs a) {
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  for (int i = threadIdx.x; i < a.bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
  }
  __syncthreads();
  const int64_t npix = a.T * a.H * a.W;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= npix) return;
  const int64_t t = p / (a.H * a.W);
  const int64_t r = p - t * (a.H * a.W);
  const int64_t y = r / a.W, x = r - (r / a.W) * a.W;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const double L = (double)((1 << a.bit_depth) - 1);
  for (int b = 0; b < a.bands; b++) {
    const int g = b / 3, c = b - 3 * g;
    uint16_t q = a.recon[((int64_t)(g * a.T + t) * 3 + c) * plane + y * a.Wp + x];
    double num = (double)q * srg[b];
    double v = smn[b] + num / L;
    if (a.out_dtype == XV_U16) {
      double rr = floor(v + 0.5);
      rr = rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
      ((uint16_t*)a.out)[p * a.bands + b] = (uint16_t)rr;
    } else {
      ((float*)a.out)[p * a.bands + b] = (float)v;
    }
  }
}

// Physical squared error: element mapping as in stats (one band per thread);
// per-block partial sums are reduced in a fixed order, so the result is
// deterministic.
__global__ void __launch_bounds__(kThreads) phys_sse_kernel(PhysArgs a) {
  __shared__ double sacc[kThreads];
  const int bands = a.bands;
  const int64_t npix = a.T * a.H * a.W;
  const int64_t total = npix * bands;
  const int64_t nthr = (int64_t)gridDim.x * blockDim.x;
  const int64_t stride = (nthr / bands) * bands;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const double L = (double)((1 << a.bit_depth) - 1);
  double acc = 0.0;
  if (gtid < stride) {
    const int b = (int)(gtid % bands);
    const int g = b / 3, c = b - 3 * g;
    const double mn = a.mn[b], range = a.mx[b] - a.mn[b];
    for (int64_t e = gtid; e < total; e += stride) {
      double xv = load_sample(a.orig, a.dtype, e);
      if (xv != xv) continue;
      const int64_t p = e / bands;
      const int64_t t = p / (a.H * a.W);
      const int64_t r = p - t * (a.H * a.W);
      const int64_t y = r / a.W, x = r - (r / a.W) * a.W;
      uint16_t q = a.recon[((int64_t)(g * a.T + t) * 3 + c) * plane + y * a.Wp + x];
      double num = (double)q * range;
      double v = mn + num / L;
      double xh;
      if (a.dtype == XV_U16) {
        double rr = floor(v + 0.5);
        xh = rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
      } else {
        xh = (double)(float)v;
      }
      double e2 = (xv - xh) * (xv - xh);
      acc = acc + e2;
    }
  }
  sacc[threadIdx.x] = acc;
  __syncthreads();
  // band of local thread i is (blockIdx.x*blockDim.x + i) % bands
  if ((int)threadIdx.x < bands) {
    const int64_t base = (int64_t)blockIdx.x * blockDim.x;
    const int b = (int)threadIdx.x;
    double s = 0.0;
    for (int i = 0; i < (int)blockDim.x; i++) {
      int64_t g = base + i;
      if (g < stride && (int)(g % bands) == b) s = s + sacc[i];
    }
    a.partial[(int64_t)blockIdx.x * bands + b] = s;
  }
}

__global__ void phys_reduce_kernel(PhysArgs a) {
  int b = threadIdx.x;
  if (b >= a.bands) return;
  double s = 0.0;
  for (int k = 0; k < a.nblocks; k++) s = s + a.partial[(int64_t)k * a.bands + b];
  a.out[b] = s;
}

// Job table of one cube, step-major: entry (s, g * nk + k) describes frame
// t = k * gop + s of band group g (nk = GOPs that have a frame at step s).
__global__ void plan_kernel(CubePlan p) {
  const int64_t total = plan_step_offset(p.T, p.G, p.gop, p.nsteps);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int s = 0;
  int64_t base = 0;
  for (;;) {
    const int64_t n = (int64_t)p.G * ((p.T - s + p.gop - 1) / p.gop);
    if (i < base + n) break;
    base += n;
    s++;
  }
  const int nk = (p.T - s + p.gop - 1) / p.gop;
  const int j = (int)(i - base);
  const int g = j / nk, k = j - (j / nk) * nk;
  const int t = k * p.gop + s;
  const int64_t f = (int64_t)g * p.T + t;
  const int64_t plane = (int64_t)p.Hp * p.Wp;
  const int Hb = p.Hp / p.N, Wb = p.Wp / p.N;
  FrameJob jb;
  jb.cur = p.frames ? p.frames + f * 3 * plane : nullptr;
  jb.ref = s > 0 ? p.recon + (f - 1) * 3 * plane : nullptr;
  jb.rec = p.recon + f * 3 * plane;
  jb.lev = p.lev + f * 3 * (int64_t)Hb * Wb * p.N * p.N;
  jb.mv = p.mv + f * (int64_t)Hb * Wb * 2;
  jb.cbits = p.cbits ? p.cbits + f * 3 * (int64_t)Hb * Wb : nullptr;
  jb.mbits = p.mbits ? p.mbits + f * (int64_t)Hb * Wb : nullptr;
  jb.vmask = p.vmask ? p.vmask + f * 3 * plane : nullptr;
  jb.nan_total = p.nan_total;
  jb.sse = p.sse ? p.sse + 3 * g : nullptr;
  jb.bits = p.bits ? p.bits + 2 * g : nullptr;
  jb.Hp = p.Hp;
  jb.Wp = p.Wp;
  jb.H = p.H;
  jb.W = p.W;
  jb.nch = min(3, p.bands - 3 * g);
  jb.intra = s == 0;
  jb.bit_depth = p.bit_depth;
  jb.qp = p.qp;
  p.jobs[i] = jb;
}

inline int grid_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

hipError_t launch_plan(const CubePlan& p, hipStream_t s) {
  const int64_t total = plan_step_offset(p.T, p.G, p.gop, p.nsteps);
  if (total <= 0) return hipSuccess;
  plan_kernel<<<grid_for(total, 128), 128, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u32_kernel<<<grid_for(n, kThreads), kThreads, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  fill_u64_kernel<<<grid_for(n, kThreads), kThreads, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t launch_stats(const StatsArgs& a, hipStream_t s) {
  hipError_t e;
  if ((e = launch_fill_u32(a.minkey, 0xffffffffu, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.maxkey, 0u, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.nan_count, 0u, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.nan_total, 0u, 1, s)) != hipSuccess) return e;
  int64_t total = a.npix * a.bands;
  int blocks = grid_for(total, kThreads * 16);
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  if ((int64_t)blocks * kThreads < a.bands) blocks = grid_for(a.bands, kThreads);
  stats_kernel<<<blocks, kThreads, 0, s>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  stats_finalize_kernel<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  pack_dense_kernel<<<grid_for(a.T * plane, kThreads), kThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.dtype != XV_F32) return e;
  pack_fill_kernel<<<grid_for(plane * a.bands, kThreads), kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_denorm(const DenormArgs& a, hipStream_t s) {
  denorm_kernel<<<grid_for(a.T * a.H * a.W, kThreads), kThreads, 0, s>>>(a);
  return hipGetLastError();
}

int phys_blocks(int64_t npix) {
  int64_t b = (npix + kThreads * 8 - 1) / (kThreads * 8);
  return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

hipError_t launch_phys_sse(const PhysArgs& a, hipStream_t s) {
  phys_sse_kernel<<<a.nblocks, kThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  phys_reduce_kernel<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace xv
