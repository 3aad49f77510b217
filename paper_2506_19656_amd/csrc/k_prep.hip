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

// Pixel-major scan: thread i handles pixels i, i + stride, ... and keeps
// per-band keys for a chunk of up to 8 bands in registers; blocks merge them
// in LDS, then with one global atomic per band (min/max/count are order
// independent, so the result is deterministic).
template <typename Tv>
__device__ inline void stats_chunk(const Tv* d, int64_t npix, int bands, int b0, int nb,
                                   uint32_t* smin, uint32_t* smax, uint32_t* snan) {
  uint32_t lo[8], hi[8], nn[8];
#pragma unroll
  for (int j = 0; j < 8; j++) {
    lo[j] = 0xffffffffu;
    hi[j] = 0u;
    nn[j] = 0u;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += stride) {
    const Tv* px = d + p * bands + b0;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (j >= nb) break;
      uint32_t k;
      if constexpr (sizeof(Tv) == 2) {
        k = (uint32_t)px[j];
      } else {
        const float f = px[j];
        if (f != f) {
          nn[j]++;
          continue;
        }
        k = f32_key(f);
      }
      lo[j] = min(lo[j], k);
      hi[j] = max(hi[j], k);
    }
  }
#pragma unroll
  for (int j = 0; j < 8; j++) {
    if (j >= nb) break;
    if (lo[j] != 0xffffffffu) atomicMin(&smin[b0 + j], lo[j]);
    if (hi[j] != 0u) atomicMax(&smax[b0 + j], hi[j]);
    if (nn[j]) atomicAdd(&snan[b0 + j], nn[j]);
  }
}

__global__ void __launch_bounds__(kThreads) stats_kernel(StatsArgs a) {
  __shared__ uint32_t smin[XV_MAX_BANDS], smax[XV_MAX_BANDS], snan[XV_MAX_BANDS];
  const int bands = a.bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
    snan[i] = 0u;
  }
  __syncthreads();
  for (int b0 = 0; b0 < bands; b0 += 8) {
    const int nb = min(8, bands - b0);
    if (a.dtype == XV_U16)
      stats_chunk<uint16_t>((const uint16_t*)a.data, a.npix, bands, b0, nb, smin, smax, snan);
    else
      stats_chunk<float>((const float*)a.data, a.npix, bands, b0, nb, smin, smax, snan);
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

// Missing-sample fill along time at one (pixel, band) series; `src` indexes
// the sample of frame 0, `fstride` is the frame size in elements.  NEAREST:
// the valid sample at the smallest |t - t'|, ties to the earlier t'.
// FORWARD: the last valid value before t, else the first one after it.  A
// series without a valid sample gives the band minimum.
__device__ inline double fill_missing(const float* d, int64_t src, int64_t fstride, int64_t t,
                                      int64_t T, int fill_mode, double mn) {
  if (fill_mode == XV_FILL_FORWARD) {
    for (int64_t u = t - 1; u >= 0; u--) {
      const float f = d[u * fstride + src];
      if (f == f) return (double)f;
    }
    for (int64_t u = t + 1; u < T; u++) {
      const float f = d[u * fstride + src];
      if (f == f) return (double)f;
    }
    return mn;
  }
  for (int64_t dd = 1; dd < T; dd++) {
    if (t - dd < 0 && t + dd >= T) break;
    if (t - dd >= 0) {
      const float f = d[(t - dd) * fstride + src];
      if (f == f) return (double)f;
    }
    if (t + dd < T) {
      const float f = d[(t + dd) * fstride + src];
      if (f == f) return (double)f;
    }
  }
  return mn;
}

// Conversion and packing: one thread per padded pixel (t, y, x) reads the
// pixel's bands (contiguous), fills missing samples, converts, and writes
// one sample to each of the 3G channel planes (edge pixels replicate the
// last real row/column; padding channels are zero or repeat the last band).
// Validity bytes are written only when the cube has missing samples.
__global__ void __launch_bounds__(kThreads) pack_kernel(PackArgs a) {
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  __shared__ int sall[XV_MAX_BANDS];
  const bool gaps = a.dtype == XV_F32 && *a.nan_total != 0u;
  for (int i = threadIdx.x; i < a.bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
    sall[i] = gaps && (int64_t)a.nan_count[i] == a.T * a.H * a.W;
  }
  __syncthreads();
  // workgroup -> (frame row, 256-pixel chunk); one uniform division
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const int xch = (a.Wp + kThreads - 1) / kThreads;
  const int64_t rowid = blockIdx.x / xch;
  const int x = (int)(blockIdx.x - rowid * xch) * kThreads + threadIdx.x;
  if (x >= a.Wp) return;
  const int64_t t = rowid / a.Hp;
  const int y = (int)(rowid - t * a.Hp);
  const int64_t o = (int64_t)y * a.Wp + x;
  const int64_t ys = y < a.H ? y : a.H - 1, xs = x < a.W ? x : a.W - 1;
  const bool real = y < a.H && x < a.W;
  const int64_t fstride = a.H * a.W * a.bands;
  const int64_t pix = (ys * a.W + xs) * a.bands;
  const double L = (double)((1 << a.bit_depth) - 1);
  uint16_t last = 0;
  for (int b = 0; b < a.bands; b++) {
    double v;
    bool valid = true;
    if (a.dtype == XV_U16) {
      v = (double)((const uint16_t*)a.data)[t * fstride + pix + b];
    } else {
      const float* d = (const float*)a.data;
      const float f = d[t * fstride + pix + b];
      if (f == f) {
        v = (double)f;
      } else {
        valid = false;
        v = sall[b] ? smn[b] : fill_missing(d, pix + b, fstride, t, a.T, a.fill_mode, smn[b]);
      }
    }
    const uint16_t q = convert(v, smn[b], srg[b], L);
    const int g = b / 3, c = b - 3 * (b / 3);
    const int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
    a.frames[off] = q;
    if (gaps) a.vmask[off] = (uint8_t)(valid && real);
    last = q;
  }
  const int g = a.groups - 1;
  for (int c = a.bands - 3 * g; c < 3; c++) {
    const int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
    a.frames[off] = a.pad_mode == XV_PAD_REPEAT ? last : (uint16_t)0;
    if (gaps) a.vmask[off] = 0;
  }
}

__global__ void __launch_bounds__(kThreads) denorm_kernel(DenormArgs a) {
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  for (int i = threadIdx.x; i < a.bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
  }
  __syncthreads();
  const int xch = (int)((a.W + kThreads - 1) / kThreads);
  const int64_t rowid = blockIdx.x / xch;
  const int64_t x = (int64_t)(blockIdx.x - rowid * xch) * kThreads + threadIdx.x;
  if (x >= a.W) return;
  const int64_t t = rowid / a.H;
  const int64_t y = rowid - t * a.H;
  const int64_t p = (t * a.H + y) * a.W + x;
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

// Physical squared error: thread per pixel x of a frame row, rows taken
// grid-stride by workgroup; per-band sums for a chunk of up to 8 bands live in
// registers.  Each block reduces its sums with a fixed LDS tree into
// partial[block][band]; the final sum over blocks has a fixed order too, so
// the result is deterministic.
__global__ void __launch_bounds__(kThreads) phys_sse_kernel(PhysArgs a) {
  __shared__ double sred[kThreads];
  const int bands = a.bands;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const double L = (double)((1 << a.bit_depth) - 1);
  const int xch = (int)((a.W + kThreads - 1) / kThreads);
  const int64_t nrows = a.T * a.H * xch;
  for (int b0 = 0; b0 < bands; b0 += 8) {
    const int nb = min(8, bands - b0);
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) acc[j] = 0.0;
    for (int64_t rid = blockIdx.x; rid < nrows; rid += gridDim.x) {
      const int64_t row = rid / xch;
      const int64_t x = (rid - row * xch) * kThreads + threadIdx.x;
      if (x >= a.W) continue;
      const int64_t t = row / a.H, y = row - (row / a.H) * a.H;
      const int64_t e0 = ((t * a.H + y) * a.W + x) * bands + b0;
#pragma unroll
      for (int j = 0; j < 8; j++) {
        if (j >= nb) break;
        const int b = b0 + j;
        const double xv = load_sample(a.orig, a.dtype, e0 + j);
        if (xv != xv) continue;
        const int g = b / 3, c = b - 3 * g;
        const uint16_t q = a.recon[((int64_t)(g * a.T + t) * 3 + c) * plane + y * a.Wp + x];
        const double num = (double)q * (a.mx[b] - a.mn[b]);
        const double v = a.mn[b] + num / L;
        double xh;
        if (a.dtype == XV_U16) {
          const double rr = floor(v + 0.5);
          xh = rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
        } else {
          xh = (double)(float)v;
        }
        acc[j] = acc[j] + (xv - xh) * (xv - xh);
      }
    }
    for (int j = 0; j < nb; j++) {
      sred[threadIdx.x] = acc[j];
      __syncthreads();
      for (int w = kThreads / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sred[threadIdx.x] = sred[threadIdx.x] + sred[threadIdx.x + w];
        __syncthreads();
      }
      if (threadIdx.x == 0) a.partial[(int64_t)blockIdx.x * bands + b0 + j] = sred[0];
      __syncthreads();
    }
  }
}

// Deterministic final sum: block b sums partial[*][b] with a fixed
// assignment of partials to threads and a fixed tree.
__global__ void __launch_bounds__(kThreads) phys_reduce_kernel(PhysArgs a) {
  __shared__ double sred[kThreads];
  const int b = blockIdx.x;
  double v = 0.0;
  for (int k = threadIdx.x; k < a.nblocks; k += blockDim.x) v = v + a.partial[(int64_t)k * a.bands + b];
  sred[threadIdx.x] = v;
  __syncthreads();
  for (int w = kThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sred[threadIdx.x] = sred[threadIdx.x] + sred[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.out[b] = sred[0];
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
  // grid: enough blocks to fill the GPU several times over, each looping
  hipError_t e;
  if ((e = launch_fill_u32(a.minkey, 0xffffffffu, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.maxkey, 0u, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.nan_count, 0u, a.bands, s)) != hipSuccess) return e;
  if ((e = launch_fill_u32(a.nan_total, 0u, 1, s)) != hipSuccess) return e;
  int blocks = grid_for(a.npix, kThreads * 4);
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  stats_kernel<<<blocks, kThreads, 0, s>>>(a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  stats_finalize_kernel<<<1, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  const int64_t blocks = a.T * a.Hp * (int64_t)((a.Wp + kThreads - 1) / kThreads);
  pack_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_denorm(const DenormArgs& a, hipStream_t s) {
  const int64_t blocks = a.T * a.H * ((a.W + kThreads - 1) / kThreads);
  denorm_kernel<<<(unsigned)blocks, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

int phys_blocks(int64_t npix) {
  int64_t b = (npix + kThreads * 4 - 1) / (kThreads * 4);
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

hipError_t launch_phys_sse(const PhysArgs& a, hipStream_t s) {
  phys_sse_kernel<<<a.nblocks, kThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  phys_reduce_kernel<<<a.bands, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace xv
