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

// ---------------------------------------------------------------------------
// Row-chunk staging through LDS.  The pixel-major cube ([T][H][W][bands]) is
// read and written in contiguous runs of chunk * bands elements with 16-byte
// accesses; the kernels then address single samples in LDS.  Element i of a
// run starting at global address g lives at lds[mis + i], mis being the
// element offset of g past the previous 16-byte boundary, so every whole
// 16-byte granule of the run maps onto one aligned LDS vector; the elements
// of granules cut by either end of the run are copied one by one.
// ---------------------------------------------------------------------------
constexpr int kStage = 4096;  // elements of one staged run at most

// The staged run lives in dynamic LDS sized to the launch's chunk (see
// stage_bytes), so small chunks keep occupancy high.
extern __shared__ uint4 xv_stage_lds[];

inline size_t stage_bytes(int chunk_px, int bands, int elem) {
  return ((size_t)chunk_px * bands * elem + 16 + 15) / 16 * 16;
}

template <typename T>
__device__ inline int stage_mis(const T* g) {
  return (int)(((uintptr_t)g & 15) / sizeof(T));
}

template <typename T>
__device__ inline int stage_in(const T* __restrict__ g, T* lds, int n) {
  constexpr int V = 16 / sizeof(T);
  const int mis = stage_mis(g);
  const int body0 = mis ? V - mis : 0;  // first element of the first whole granule
  const int nfull = n > body0 ? (n - body0) / V : 0;
  const int body1 = body0 + nfull * V;
  const uint4* gv = (const uint4*)(g + body0);
  uint4* lv = (uint4*)(lds + mis + body0);
  for (int k = threadIdx.x; k < nfull; k += blockDim.x) lv[k] = gv[k];
  const int head = n < body0 ? n : body0;
  for (int e = threadIdx.x; e < head; e += blockDim.x) lds[mis + e] = g[e];
  for (int e = body1 + threadIdx.x; e < n; e += blockDim.x) lds[mis + e] = g[e];
  return mis;
}

template <typename T>
__device__ inline void stage_out(const T* lds, T* __restrict__ g, int n, int mis) {
  constexpr int V = 16 / sizeof(T);
  const int body0 = mis ? V - mis : 0;
  const int nfull = n > body0 ? (n - body0) / V : 0;
  const int body1 = body0 + nfull * V;
  uint4* gv = (uint4*)(g + body0);
  const uint4* lv = (const uint4*)(lds + mis + body0);
  for (int k = threadIdx.x; k < nfull; k += blockDim.x) gv[k] = lv[k];
  const int head = n < body0 ? n : body0;
  for (int e = threadIdx.x; e < head; e += blockDim.x) g[e] = lds[mis + e];
  for (int e = body1 + threadIdx.x; e < n; e += blockDim.x) g[e] = lds[mis + e];
}

// ---------------------------------------------------------------------------
// Statistics.  The cube is read as one flat array with coalesced loads of V
// consecutive elements (16 bytes when the data is 16-byte aligned, else one
// element).  The grid stride in elements is a multiple of the band count, so
// slot j of every load a thread makes holds the same band, (tid * V + j) %
// bands, and the per-band keys stay in V registers per kind.  Blocks merge in
// LDS and write one partial per band; min, max and counts are order
// independent, so the result is deterministic.
// ---------------------------------------------------------------------------
template <typename Tv>
__device__ inline void stats_acc(Tv x, uint32_t& lo, uint32_t& hi, uint32_t& nn) {
  if constexpr (sizeof(Tv) == 2) {
    const uint32_t k = x;
    lo = min(lo, k);
    hi = max(hi, k);
  } else {
    const bool nan = x != x;
    const uint32_t k = f32_key(x);
    lo = nan ? lo : min(lo, k);
    hi = nan ? hi : max(hi, k);
    nn += nan ? 1u : 0u;
  }
}

template <typename Tv, int V>
__device__ inline void load_run(const Tv* __restrict__ d, int64_t v, Tv (&x)[V]) {
  if constexpr (V == 1) {
    x[0] = d[v];
  } else if constexpr (sizeof(Tv) == 4) {
    const float4 f = ((const float4*)d)[v];
    x[0] = f.x;
    x[1] = f.y;
    x[2] = f.z;
    x[3] = f.w;
  } else {
    const uint4 u = ((const uint4*)d)[v];
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int j = 0; j < 4; j++) {
      x[2 * j] = (Tv)(w[j] & 0xffffu);
      x[2 * j + 1] = (Tv)(w[j] >> 16);
    }
  }
}

template <typename Tv, int V>
__global__ void __launch_bounds__(kThreads) stats_kernel(StatsArgs a) {
  __shared__ uint32_t smin[XV_MAX_BANDS], smax[XV_MAX_BANDS], snan[XV_MAX_BANDS];
  const int bands = a.bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smin[i] = 0xffffffffu;
    smax[i] = 0u;
    snan[i] = 0u;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.nan_total = 0u;  // summed by the finalize kernel
  __syncthreads();
  const Tv* d = (const Tv*)a.data;
  const int64_t n = a.npix * bands;
  const int64_t nvec = n / V;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t lo[V], hi[V], nn[V];
#pragma unroll
  for (int j = 0; j < V; j++) {
    lo[j] = 0xffffffffu;
    hi[j] = 0u;
    nn[j] = 0u;
  }
  int64_t v = tid;
  for (; v + 3 * nth < nvec; v += 4 * nth) {
    Tv x[4][V];
#pragma unroll
    for (int u = 0; u < 4; u++) load_run<Tv, V>(d, v + u * nth, x[u]);
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int j = 0; j < V; j++) stats_acc(x[u][j], lo[j], hi[j], nn[j]);
  }
  for (; v < nvec; v += nth) {
    Tv x[V];
    load_run<Tv, V>(d, v, x);
#pragma unroll
    for (int j = 0; j < V; j++) stats_acc(x[j], lo[j], hi[j], nn[j]);
  }
  const int bt = (int)((tid * V) % bands);
#pragma unroll
  for (int j = 0; j < V; j++) {
    const int b = (bt + j) % bands;
    atomicMin(&smin[b], lo[j]);
    atomicMax(&smax[b], hi[j]);
    if (nn[j]) atomicAdd(&snan[b], nn[j]);
  }
  // the last n % V elements
  const int64_t e = nvec * V + tid;
  if (e < n) {
    uint32_t l = 0xffffffffu, h = 0u, c = 0u;
    stats_acc(d[e], l, h, c);
    const int b = (int)(e % bands);
    atomicMin(&smin[b], l);
    atomicMax(&smax[b], h);
    if (c) atomicAdd(&snan[b], c);
  }
  __syncthreads();
  uint32_t* out = a.part + (int64_t)blockIdx.x * 3 * bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    out[i] = smin[i];
    out[bands + i] = smax[i];
    out[2 * bands + i] = snan[i];
  }
}

// One workgroup per band merges the block partials (fixed tree; min, max and
// counts are order independent anyway); keys -> binary64 statistics.  A band
// without a valid sample gets 0, 0.
constexpr int kFinThreads = 1024;

__global__ void __launch_bounds__(kFinThreads) stats_finalize_kernel(StatsArgs a) {
  __shared__ uint32_t rlo[kFinThreads / 64], rhi[kFinThreads / 64], rnn[kFinThreads / 64];
  const int b = blockIdx.x;
  const int bands = a.bands;
  uint32_t lo = 0xffffffffu, hi = 0u, nn = 0u;
  for (int k = threadIdx.x; k < a.nblocks; k += kFinThreads) {
    const uint32_t* p = a.part + (int64_t)k * 3 * bands;
    lo = min(lo, p[b]);
    hi = max(hi, p[bands + b]);
    nn += p[2 * bands + b];
  }
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    lo = min(lo, (uint32_t)__shfl_xor((int)lo, w, 64));
    hi = max(hi, (uint32_t)__shfl_xor((int)hi, w, 64));
    nn += (uint32_t)__shfl_xor((int)nn, w, 64);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rlo[wv] = lo;
    rhi[wv] = hi;
    rnn[wv] = nn;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 1; i < kFinThreads / 64; i++) {
    lo = min(lo, rlo[i]);
    hi = max(hi, rhi[i]);
    nn += rnn[i];
  }
  const bool any = (uint64_t)nn < (uint64_t)a.npix;
  double l = 0.0, h = 0.0;
  if (any) {
    if (a.dtype == XV_U16) {
      l = (double)lo;
      h = (double)hi;
    } else {
      l = (double)key_f32(lo);
      h = (double)key_f32(hi);
    }
  }
  a.mn[b] = l;
  a.mx[b] = h;
  a.n_valid[b] = (unsigned long long)(a.npix - (int64_t)nn);
  a.nan_count[b] = nn;
  if (nn) atomicAdd(a.nan_total, nn);
}

// q = floor((x - mn) * L / (mx - mn) + 1/2) clamped to [0, L]; constant band -> 0.
// The quotient is formed as a product with the band's reciprocal; the two
// differ by at most a few ulp (below 3e-12, as the quotient is at most L <
// 2^12), which changes floor(v + 1/2) only when v + 1/2 lies that close to an
// integer, so within 1e-9 of one the exact IEEE quotient is taken instead and
// the result is always that of the division.
__device__ inline uint16_t convert(double x, double mn, double range, double inv, double L) {
  if (range == 0.0) return 0;
  const double num = (x - mn) * L;
  double w = num * inv + 0.5;
  double fw = floor(w);
  const double fr = w - fw;
  if (fr < 1e-9 || fr > 1.0 - 1e-9) {
    w = num / range + 0.5;
    fw = floor(w);
  }
  double q = fw < 0.0 ? 0.0 : fw;
  q = q > L ? L : q;
  return (uint16_t)q;
}

// Missing-sample fill along time for up to 8 bands of one pixel at once;
// `src` indexes the first of them in frame 0, `fstride` is the frame size in
// elements, bit j of `miss` marks band j as missing at time t.  NEAREST: the
// valid sample at the smallest |t - t'|, ties to the earlier t', searched
// from distance dd0 on (the caller has resolved the nearer ones).  FORWARD:
// the last valid value before t, else the first one after it.  Each probe
// of a time reads all the pixel's bands together; bands left without a
// valid sample in the whole series keep their preset value (the band
// minimum).
template <class V>
__device__ inline void fill_missing(const float* __restrict__ d, int64_t src, int nb,
                                    int64_t fstride, int64_t t, int64_t T, int fill_mode,
                                    uint32_t miss, V (&v)[8], int64_t dd0 = 1) {
  auto probe = [&](int64_t u) {
    float f[8];
#pragma unroll
    for (int j = 0; j < 8; j++) f[j] = d[u * fstride + src + min(j, nb - 1)];
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (((miss >> j) & 1u) && f[j] == f[j]) {
        v[j] = (V)f[j];
        miss &= ~(1u << j);
      }
    }
  };
  if (fill_mode == XV_FILL_FORWARD) {
    for (int64_t u = t - 1; u >= 0 && miss; u--) probe(u);
    for (int64_t u = t + 1; u < T && miss; u++) probe(u);
    return;
  }
  for (int64_t dd = dd0; miss && (t - dd >= 0 || t + dd < T); dd++) {
    if (t - dd >= 0) probe(t - dd);
    if (miss && t + dd < T) probe(t + dd);
  }
}

// Conversion and packing.  A workgroup takes one padded row chunk (t, y,
// x0 .. x0 + chunk - 1): it stages the real pixels of the source row (rows
// past H replicate row H - 1) and each thread then converts one pixel's bands
// and writes one sample to each of the 3G channel planes (columns past W
// replicate column W - 1; padding channels are zero or repeat the last
// band).  Missing samples are filled along time from global memory.
// Validity bytes are written only when the cube has missing samples.  The
// chunk is a multiple of the block size, so every chunk holds a real column.
template <typename Tv>
__global__ void __launch_bounds__(kThreads) pack_kernel(PackArgs a) {
  Tv* stage = (Tv*)xv_stage_lds;
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS], sinv[XV_MAX_BANDS];
  __shared__ int sall[XV_MAX_BANDS];
  const int bands = a.bands;
  const bool gaps = sizeof(Tv) == 4 && *a.nan_total != 0u;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
    sinv[i] = srg[i] != 0.0 ? 1.0 / srg[i] : 0.0;
    sall[i] = gaps && (int64_t)a.nan_count[i] == a.T * a.H * a.W;
  }
  const int P = a.chunk_px;
  const int xch = (a.Wp + P - 1) / P;
  const int64_t rowid = blockIdx.x / xch;
  const int x0 = (int)(blockIdx.x - rowid * xch) * P;
  const int64_t t = rowid / a.Hp;
  const int y = (int)(rowid - t * a.Hp);
  const int64_t ys = y < a.H ? y : a.H - 1;
  const int nreal = min(P, (int)a.W - x0);
  const Tv* d = (const Tv*)a.data;
  const int64_t fstride = a.H * a.W * bands;
  const int mis = stage_in(d + t * fstride + (ys * a.W + x0) * bands, stage, nreal * bands);
  __syncthreads();
  const int xi = threadIdx.x;
  const int x = x0 + xi;
  if (xi >= P || x >= a.Wp) return;
  const int xr = min(xi, nreal - 1);
  const bool real = y < a.H && x < a.W;
  const Tv* px = stage + mis + xr * bands;
  const int64_t pix = (ys * a.W + x0 + xr) * bands;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const int64_t o = (int64_t)y * a.Wp + x;
  const double L = (double)((1 << a.bit_depth) - 1);
  uint16_t last = 0;
  for (int b0 = 0; b0 < bands; b0 += 8) {
    const int nb = min(8, bands - b0);
    double v[8];
    uint32_t miss = 0u;
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (j >= nb) break;
      const int b = b0 + j;
      if constexpr (sizeof(Tv) == 2) {
        v[j] = (double)px[b];
      } else {
        const float f = px[b];
        const bool nan = f != f;
        v[j] = nan ? smn[b] : (double)f;
        // a band missing in every frame keeps its minimum without a search
        miss |= (nan && !sall[b]) ? (1u << j) : 0u;
      }
    }
    uint32_t invalid = miss;
    if constexpr (sizeof(Tv) == 4) {
#pragma unroll
      for (int j = 0; j < 8; j++)
        if (j < nb && px[b0 + j] != px[b0 + j]) invalid |= 1u << j;
      if (miss) fill_missing(d, pix + b0, nb, fstride, t, a.T, a.fill_mode, miss, v);
    }
#pragma unroll
    for (int j = 0; j < 8; j++) {
      if (j >= nb) break;
      const int b = b0 + j;
      const uint16_t q = convert(v[j], smn[b], srg[b], sinv[b], L);
      const int g = b / 3, c = b - 3 * g;
      const int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
      a.frames[off] = q;
      if (gaps) a.vmask[off] = (uint8_t)(!((invalid >> j) & 1u) && real);
      last = q;
    }
  }
  const int g = a.groups - 1;
  for (int c = bands - 3 * g; c < 3; c++) {
    const int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
    a.frames[off] = a.pad_mode == XV_PAD_REPEAT ? last : (uint16_t)0;
    if (gaps) a.vmask[off] = 0;
  }
}

// Decoded frames back to the caller's dtype: x = mn + q * (mx - mn) / L in
// binary64 (u16: rounded half up and clamped; f32: rounded to nearest).  A
// workgroup takes one row chunk, reads each band's plane row coalesced,
// assembles the pixel-major run in LDS and writes it with 16-byte stores.
template <typename To>
__global__ void __launch_bounds__(kThreads) denorm_kernel(DenormArgs a) {
  To* stage = (To*)xv_stage_lds;
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  const int bands = a.bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
  }
  __syncthreads();
  const int P = a.chunk_px;
  const int xch = (int)((a.W + P - 1) / P);
  const int64_t rowid = blockIdx.x / xch;
  const int x0 = (int)(blockIdx.x - rowid * xch) * P;
  const int64_t t = rowid / a.H;
  const int64_t y = rowid - t * a.H;
  const int nreal = min(P, (int)a.W - x0);
  To* dst = (To*)a.out + ((t * a.H + y) * a.W + x0) * bands;
  const int mis = stage_mis(dst);
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const double L = (double)((1 << a.bit_depth) - 1);
  const int xi = threadIdx.x;
  if (xi < nreal) {
    const uint16_t* rrow = a.recon + y * a.Wp + x0 + xi;
    for (int b0 = 0; b0 < bands; b0 += 8) {
      uint16_t q[8];
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int b = min(b0 + j, bands - 1);  // in-bounds loads, issued together
        const int g = b / 3, c = b - 3 * g;
        q[j] = rrow[((int64_t)(g * a.T + t) * 3 + c) * plane];
      }
#pragma unroll
      for (int j = 0; j < 8; j++) {
        const int b = b0 + j;
        if (b >= bands) break;
        const double num = (double)q[j] * srg[b];
        const double v = smn[b] + num / L;
        To o;
        if constexpr (sizeof(To) == 2) {
          double rr = floor(v + 0.5);
          rr = rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
          o = (To)rr;
        } else {
          o = (To)v;
        }
        stage[mis + xi * bands + b] = o;
      }
    }
  }
  __syncthreads();
  stage_out(stage, dst, nreal * bands, mis);
}

// Physical squared error.  Workgroups take row chunks grid-stride, stage the
// original samples, and each thread accumulates per-band sums of its pixel
// in registers (8 bands per pass).  Each block reduces with a fixed LDS tree
// into partial[block][band]; the final sum over blocks has a fixed order
// too, so the result is deterministic.
template <typename Tv>
__global__ void __launch_bounds__(kThreads) phys_sse_kernel(PhysArgs a) {
  Tv* stage = (Tv*)xv_stage_lds;
  __shared__ double sred[kThreads];
  __shared__ double smn[XV_MAX_BANDS], srg[XV_MAX_BANDS];
  const int bands = a.bands;
  for (int i = threadIdx.x; i < bands; i += blockDim.x) {
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
  }
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const double L = (double)((1 << a.bit_depth) - 1);
  const int P = a.chunk_px;
  const int xch = (int)((a.W + P - 1) / P);
  const int64_t units = a.T * a.H * xch;
  const Tv* orig = (const Tv*)a.orig;
  const int xi = threadIdx.x;
  for (int b0 = 0; b0 < bands; b0 += 8) {
    const int nb = min(8, bands - b0);
    double acc[8];
#pragma unroll
    for (int j = 0; j < 8; j++) acc[j] = 0.0;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
      const int64_t row = u / xch;
      const int x0 = (int)(u - row * xch) * P;
      const int64_t t = row / a.H, y = row - t * a.H;
      const int nreal = min(P, (int)a.W - x0);
      __syncthreads();  // the previous chunk has been read
      const int mis = stage_in(orig + (row * a.W + x0) * bands, stage, nreal * bands);
      __syncthreads();
      if (xi < nreal) {
        const uint16_t* rrow = a.recon + y * a.Wp + x0 + xi;
        uint16_t q[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int b = min(b0 + j, bands - 1);
          const int g = b / 3, c = b - 3 * g;
          q[j] = rrow[((int64_t)(g * a.T + t) * 3 + c) * plane];
        }
        const Tv* px = stage + mis + xi * bands;
#pragma unroll
        for (int j = 0; j < 8; j++) {
          const int b = b0 + j;
          if (b >= bands) break;
          const double xv = (double)px[b];
          const double num = (double)q[j] * srg[b];
          const double v = smn[b] + num / L;
          double xh;
          if constexpr (sizeof(Tv) == 2) {
            const double rr = floor(v + 0.5);
            xh = rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
          } else {
            xh = (double)(float)v;
          }
          const double e = xv - xh;
          acc[j] = (xv == xv) ? acc[j] + e * e : acc[j];
        }
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

// ---------------------------------------------------------------------------
// Pixel-group kernels for up to 8 bands.  A thread owns g consecutive pixels
// of a row, g the smallest count whose bands fill whole 16-byte granules
// (6 float bands: 2 pixels, 48 bytes), so the pixel-major side is read or
// written with aligned 16-byte accesses straight into registers, and each
// channel plane sees g consecutive samples per thread.  Used when the data
// pointer is 16-byte aligned and the row width is a multiple of g; the
// row-staged kernels above cover every other case.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int gcd_c(int x, int y) { return y == 0 ? x : gcd_c(y, x % y); }

template <typename T, int BANDS>
struct PixGroup {
  static constexpr int bpp = BANDS * (int)sizeof(T);  // bytes per pixel
  static constexpr int g = 16 / gcd_c(16, bpp);      // pixels per group
  static constexpr int nv = g * bpp / 16;            // 16-byte granules per group
  static constexpr int ne = g * BANDS;               // elements per group
};

template <typename T, int NE>
__device__ inline void load_granules(const T* __restrict__ p, T (&v)[NE]) {
  constexpr int nv = NE * (int)sizeof(T) / 16;
  uint4 w[nv];
#pragma unroll
  for (int i = 0; i < nv; i++) w[i] = ((const uint4*)p)[i];
  __builtin_memcpy(v, w, sizeof w);
}

template <typename T, int NE>
__device__ inline void store_granules(T* __restrict__ p, const T (&v)[NE]) {
  constexpr int nv = NE * (int)sizeof(T) / 16;
  uint4 w[nv];
  __builtin_memcpy(w, v, sizeof w);
#pragma unroll
  for (int i = 0; i < nv; i++) ((uint4*)p)[i] = w[i];
}

// g consecutive u16 samples (or bytes) of a plane, one access when aligned.
template <int G, typename T>
__device__ inline void load_run_g(const T* __restrict__ p, T (&q)[G], bool aligned) {
  if (aligned && G * sizeof(T) >= 2 && G * sizeof(T) <= 16) {
    if constexpr (G * sizeof(T) == 16) {
      const uint4 w = *(const uint4*)p;
      __builtin_memcpy(q, &w, 16);
      return;
    } else if constexpr (G * sizeof(T) == 8) {
      const uint2 w = *(const uint2*)p;
      __builtin_memcpy(q, &w, 8);
      return;
    } else if constexpr (G * sizeof(T) == 4) {
      const uint32_t w = *(const uint32_t*)p;
      __builtin_memcpy(q, &w, 4);
      return;
    } else if constexpr (G * sizeof(T) == 2) {
      const uint16_t w = *(const uint16_t*)p;
      __builtin_memcpy(q, &w, 2);
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < G; i++) q[i] = p[i];
}

template <int G, typename T>
__device__ inline void store_run_g(T* __restrict__ p, const T (&q)[G], bool aligned, int n) {
  if (aligned && n == G) {
    if constexpr (G * sizeof(T) == 16) {
      uint4 w;
      __builtin_memcpy(&w, q, 16);
      *(uint4*)p = w;
      return;
    } else if constexpr (G * sizeof(T) == 8) {
      uint2 w;
      __builtin_memcpy(&w, q, 8);
      *(uint2*)p = w;
      return;
    } else if constexpr (G * sizeof(T) == 4) {
      uint32_t w;
      __builtin_memcpy(&w, q, 4);
      *(uint32_t*)p = w;
      return;
    } else if constexpr (G * sizeof(T) == 2) {
      uint16_t w;
      __builtin_memcpy(&w, q, 2);
      *(uint16_t*)p = w;
      return;
    }
  }
#pragma unroll
  for (int i = 0; i < G; i++)
    if (i < n) p[i] = q[i];
}

// Pixel groups a thread of the vectorised u16 kernels takes (groups of ne
// elements): their loads are issued together, so that enough bytes are in
// flight to keep HBM busy -- about 32 elements per thread, at most 4
// groups.  The f32 kernels, whose conversions take a binary64 division per
// sample, keep one group (more measured slower).
__host__ __device__ constexpr int vec_unroll(int elem, int ne) {
  return elem != 2 ? 1 : ne >= 32 ? 1 : (32 / ne > 4 ? 4 : 32 / ne);
}

// Conversion and packing over the padded frame (rows past H replicate row
// H - 1, columns past W column W - 1): vec_unroll pixel groups per thread,
// blockDim.x groups apart, their input loads issued together.
template <typename Tv, int BANDS>
__global__ void __launch_bounds__(kThreads) pack_vec_kernel(PackArgs a) {
  using PG = PixGroup<Tv, BANDS>;
  constexpr int G = PG::g;
  constexpr int kVecUnroll = vec_unroll((int)sizeof(Tv), PG::ne);
  __shared__ double smn[BANDS], srg[BANDS], sinv[BANDS];
  __shared__ int sall[BANDS];
  const bool gaps = sizeof(Tv) == 4 && *a.nan_total != 0u;
  if (threadIdx.x < BANDS) {
    const int i = threadIdx.x;
    smn[i] = a.mn[i];
    srg[i] = a.mx[i] - a.mn[i];
    sinv[i] = srg[i] != 0.0 ? 1.0 / srg[i] : 0.0;
    sall[i] = gaps && (int64_t)a.nan_count[i] == a.T * a.H * a.W;
  }
  __syncthreads();
  const int gpr = (a.Wp + G - 1) / G;
  const int64_t total = a.T * a.Hp * gpr;
  const int64_t gid0 = (int64_t)blockIdx.x * blockDim.x * kVecUnroll + threadIdx.x;
  const Tv* d = (const Tv*)a.data;
  const int64_t fstride = a.H * a.W * BANDS;
  Tv vs[kVecUnroll][PG::ne];
  int64_t ts[kVecUnroll];
  int x0s[kVecUnroll], y_s[kVecUnroll];
#pragma unroll
  for (int u = 0; u < kVecUnroll; u++) {
    const int64_t gid = gid0 + (int64_t)u * blockDim.x;
    if (gid >= total) break;
    const int64_t row = gid / gpr;
    const int x0 = (int)(gid - row * gpr) * G;
    const int64_t t = row / a.Hp;
    const int y = (int)(row - t * a.Hp);
    ts[u] = t;
    x0s[u] = x0;
    y_s[u] = y;
    const int64_t ys = y < a.H ? y : a.H - 1;
    const Tv* src = d + t * fstride + ys * a.W * BANDS;
    if (x0 + G <= a.W) {
      load_granules<Tv, PG::ne>(src + (int64_t)x0 * BANDS, vs[u]);
    } else {
#pragma unroll
      for (int p = 0; p < G; p++) {
        const int xs = min(x0 + p, (int)a.W - 1);
#pragma unroll
        for (int b = 0; b < BANDS; b++) vs[u][p * BANDS + b] = src[(int64_t)xs * BANDS + b];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kVecUnroll; u++) {
    if (gid0 + (int64_t)u * blockDim.x >= total) break;
    const int64_t t = ts[u];
    const int x0 = x0s[u];
    const int y = y_s[u];
    const int64_t ys = y < a.H ? y : a.H - 1;
    const Tv(&v)[PG::ne] = vs[u];
    const double L = (double)((1 << a.bit_depth) - 1);
    uint16_t q[BANDS][G];
    uint8_t ok[BANDS][G];
    // samples as float: u16 values and the minimum of a float band are exact
    // there, and a filled sample is an input float
    float dv[G][8];
    uint32_t miss[G];
#pragma unroll
    for (int p = 0; p < G; p++) {
      miss[p] = 0u;
#pragma unroll
      for (int b = 0; b < BANDS; b++) {
        if constexpr (sizeof(Tv) == 2) {
          dv[p][b] = (float)v[p * BANDS + b];
        } else {
          const float f = v[p * BANDS + b];
          const bool nan = f != f;
          dv[p][b] = nan ? (float)smn[b] : f;
          miss[p] |= (nan && !sall[b]) ? (1u << b) : 0u;
        }
      }
    }
    if constexpr (sizeof(Tv) == 4) {
      uint32_t any = 0u;
#pragma unroll
      for (int p = 0; p < G; p++) any |= miss[p];
      if (any) {
        int64_t dd0 = 1;
        if (a.fill_mode == XV_FILL_NEAREST) {
          // the usual case resolves at distance 1: load times t - 1 and t + 1
          // of the group's pixels together, take t - 1 where valid, else
          // t + 1, and search further only for what is still missing
          const float* df = (const float*)d;
          float fm[PG::ne], fp[PG::ne];
          const bool hm = t >= 1, hp = t + 1 < a.T;
#pragma unroll
          for (int p = 0; p < G; p++) {
            const int64_t px = (ys * a.W + min(x0 + p, (int)a.W - 1)) * BANDS;
#pragma unroll
            for (int b = 0; b < BANDS; b++) {
              fm[p * BANDS + b] = hm ? df[(t - 1) * fstride + px + b] : __builtin_nanf("");
              fp[p * BANDS + b] = hp ? df[(t + 1) * fstride + px + b] : __builtin_nanf("");
            }
          }
#pragma unroll
          for (int p = 0; p < G; p++)
#pragma unroll
            for (int b = 0; b < BANDS; b++) {
              const float m = fm[p * BANDS + b], n = fp[p * BANDS + b];
              if ((miss[p] >> b) & 1u) {
                if (m == m) {
                  dv[p][b] = m;
                  miss[p] &= ~(1u << b);
                } else if (n == n) {
                  dv[p][b] = n;
                  miss[p] &= ~(1u << b);
                }
              }
            }
          dd0 = 2;
        }
#pragma unroll
        for (int p = 0; p < G; p++)
          if (miss[p]) {
            const int xs = min(x0 + p, (int)a.W - 1);
            fill_missing((const float*)d, (ys * a.W + xs) * BANDS, BANDS, fstride, t, a.T, a.fill_mode,
                         miss[p], dv[p], dd0);
          }
      }
    }
#pragma unroll
    for (int p = 0; p < G; p++) {
      const bool real = y < a.H && x0 + p < a.W;
#pragma unroll
      for (int b = 0; b < BANDS; b++) {
        q[b][p] = convert((double)dv[p][b], smn[b], srg[b], sinv[b], L);
        bool valid = true;
        if constexpr (sizeof(Tv) == 4) {
          const float f = v[p * BANDS + b];
          valid = f == f;
        }
        ok[b][p] = (uint8_t)(valid && real);
      }
    }
    const int64_t plane = (int64_t)a.Hp * a.Wp;
    const int64_t o = (int64_t)y * a.Wp + x0;
    const bool al = (a.Wp % G) == 0;
    const int n = min(G, a.Wp - x0);
#pragma unroll
    for (int b = 0; b < BANDS; b++) {
      const int g = b / 3, c = b - 3 * g;
      const int64_t off = ((int64_t)(g * a.T + t) * 3 + c) * plane + o;
      store_run_g<G>(a.frames + off, q[b], al, n);
      if (gaps) store_run_g<G>(a.vmask + off, ok[b], al, n);
    }
    constexpr int GL = (BANDS - 1) / 3;  // last group
    uint16_t z[G];
    uint8_t zm[G];
#pragma unroll
    for (int p = 0; p < G; p++) {
      z[p] = a.pad_mode == XV_PAD_REPEAT ? q[BANDS - 1][p] : (uint16_t)0;
      zm[p] = 0;
    }
#pragma unroll
    for (int c = BANDS - 3 * GL; c < 3; c++) {
      const int64_t off = ((int64_t)(GL * a.T + t) * 3 + c) * plane + o;
      store_run_g<G>(a.frames + off, z, al, n);
      if (gaps) store_run_g<G>(a.vmask + off, zm, al, n);
    }
  }
}


// A decoded sample back to u16: floor(mn + q R / L + 1/2) clamped to
// [0, 65535], each operation rounded as written.  For a band range below
// 2^16 the quotient is taken as a product with 1/L: it then differs from
// the IEEE quotient by under 2^-35, and so does the sum for every x that
// does not clamp (|x| < 2^17), which changes the floor only when x + 1/2
// lies within 2^-20 of an integer; there the exact division is taken.
__device__ inline double to_u16_sample(uint32_t q, double mn, double range, double L, double invL) {
  const double num = (double)q * range;  // q < 2^12, range < 2^16 when it matters: exact
  if (range < 65536.0) {
    const double w = (mn + num * invL) + 0.5;
    const double f = floor(w);
    const double fr = w - f;
    if (fr >= 0x1p-20 && fr <= 1.0 - 0x1p-20) return f < 0.0 ? 0.0 : (f > 65535.0 ? 65535.0 : f);
  }
  const double rr = floor((mn + num / L) + 0.5);
  return rr < 0.0 ? 0.0 : (rr > 65535.0 ? 65535.0 : rr);
}

// Decoded frames back to the caller's dtype, vec_unroll pixel groups per
// thread (groups blockDim.x apart, so that each load instruction of a wave
// stays contiguous).
template <typename To, int BANDS>
__global__ void __launch_bounds__(kThreads) denorm_vec_kernel(DenormArgs a) {
  using PG = PixGroup<To, BANDS>;
  constexpr int G = PG::g;
  constexpr int kVecUnroll = vec_unroll((int)sizeof(To), PG::ne);
  __shared__ double smn[BANDS], srg[BANDS];
  if (threadIdx.x < BANDS) {
    smn[threadIdx.x] = a.mn[threadIdx.x];
    srg[threadIdx.x] = a.mx[threadIdx.x] - a.mn[threadIdx.x];
  }
  __syncthreads();
  const int gpr = (int)(a.W / G);
  const int64_t total = a.T * a.H * gpr;
  const int64_t gid0 = (int64_t)blockIdx.x * blockDim.x * kVecUnroll + threadIdx.x;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const bool al = (a.Wp % G) == 0;
  const double L = (double)((1 << a.bit_depth) - 1);
  const double invL = 1.0 / L;
  uint16_t q[kVecUnroll][BANDS][G];
  int64_t rows[kVecUnroll];
  int xs[kVecUnroll];
#pragma unroll
  for (int u = 0; u < kVecUnroll; u++) {
    const int64_t gid = gid0 + (int64_t)u * blockDim.x;
    if (gid >= total) break;
    const int64_t row = gid / gpr;
    const int x0 = (int)(gid - row * gpr) * G;
    const int64_t t = row / a.H;
    const int64_t y = row - t * a.H;
    rows[u] = row;
    xs[u] = x0;
#pragma unroll
    for (int b = 0; b < BANDS; b++) {
      const int g = b / 3, c = b - 3 * g;
      load_run_g<G>(a.recon + ((int64_t)(g * a.T + t) * 3 + c) * plane + y * a.Wp + x0, q[u][b], al);
    }
  }
#pragma unroll
  for (int u = 0; u < kVecUnroll; u++) {
    if (gid0 + (int64_t)u * blockDim.x >= total) break;
    To v[PG::ne];
#pragma unroll
    for (int p = 0; p < G; p++) {
#pragma unroll
      for (int b = 0; b < BANDS; b++) {
        if constexpr (sizeof(To) == 2) {
          v[p * BANDS + b] = (To)to_u16_sample(q[u][b][p], smn[b], srg[b], L, invL);
        } else {
          const double num = (double)q[u][b][p] * srg[b];
          v[p * BANDS + b] = (To)(smn[b] + num / L);
        }
      }
    }
    store_granules<To, PG::ne>((To*)a.out + (rows[u] * a.W + xs[u]) * BANDS, v);
  }
}

// Physical squared error, vec_unroll pixel groups per thread and step of a
// grid-stride loop (their loads issued together); per-band sums in
// registers, fixed LDS tree per block.
template <typename Tv, int BANDS>
__global__ void __launch_bounds__(kThreads) phys_vec_kernel(PhysArgs a) {
  using PG = PixGroup<Tv, BANDS>;
  constexpr int G = PG::g;
  constexpr int kVecUnroll = vec_unroll((int)sizeof(Tv), PG::ne);
  __shared__ double sred[kThreads];
  __shared__ double smn[BANDS], srg[BANDS];
  if (threadIdx.x < BANDS) {
    smn[threadIdx.x] = a.mn[threadIdx.x];
    srg[threadIdx.x] = a.mx[threadIdx.x] - a.mn[threadIdx.x];
  }
  __syncthreads();
  const int gpr = (int)(a.W / G);
  const int64_t total = a.T * a.H * gpr;
  const int64_t plane = (int64_t)a.Hp * a.Wp;
  const bool al = (a.Wp % G) == 0;
  const double L = (double)((1 << a.bit_depth) - 1);
  const double invL = 1.0 / L;
  const Tv* orig = (const Tv*)a.orig;
  double acc[BANDS];
#pragma unroll
  for (int b = 0; b < BANDS; b++) acc[b] = 0.0;
  for (int64_t gid0 = (int64_t)blockIdx.x * blockDim.x * kVecUnroll + threadIdx.x; gid0 < total;
       gid0 += (int64_t)gridDim.x * blockDim.x * kVecUnroll) {
    Tv v[kVecUnroll][PG::ne];
    uint16_t q[kVecUnroll][BANDS][G];
#pragma unroll
    for (int u = 0; u < kVecUnroll; u++) {
      const int64_t gid = gid0 + (int64_t)u * blockDim.x;
      if (gid >= total) break;
      const int64_t row = gid / gpr;
      const int x0 = (int)(gid - row * gpr) * G;
      const int64_t t = row / a.H;
      const int64_t y = row - t * a.H;
      load_granules<Tv, PG::ne>(orig + (row * a.W + x0) * BANDS, v[u]);
#pragma unroll
      for (int b = 0; b < BANDS; b++) {
        const int g = b / 3, c = b - 3 * g;
        load_run_g<G>(a.recon + ((int64_t)(g * a.T + t) * 3 + c) * plane + y * a.Wp + x0, q[u][b], al);
      }
    }
#pragma unroll
    for (int u = 0; u < kVecUnroll; u++) {
      if (gid0 + (int64_t)u * blockDim.x >= total) break;
#pragma unroll
      for (int p = 0; p < G; p++) {
#pragma unroll
        for (int b = 0; b < BANDS; b++) {
          const double xv = (double)v[u][p * BANDS + b];
          double xh;
          if constexpr (sizeof(Tv) == 2) {
            xh = to_u16_sample(q[u][b][p], smn[b], srg[b], L, invL);
          } else {
            const double num = (double)q[u][b][p] * srg[b];
            xh = (double)(float)(smn[b] + num / L);
          }
          const double e = xv - xh;
          acc[b] = (xv == xv) ? acc[b] + e * e : acc[b];
        }
      }
    }
  }
#pragma unroll
  for (int b = 0; b < BANDS; b++) {
    sred[threadIdx.x] = acc[b];
    __syncthreads();
    for (int w = kThreads / 2; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) sred[threadIdx.x] = sred[threadIdx.x] + sred[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[(int64_t)blockIdx.x * BANDS + b] = sred[0];
    __syncthreads();
  }
}

// Per-group totals of the transform kernel's per-tile sums, in two passes
// with a fixed assignment of tiles to threads and a fixed order of addition.
// Pass 1: block (c, g) reads whole tile records (kTileSums words each,
// adjacent threads on adjacent records) of chunk c of group g and writes
// five chunk sums (squared error of channels 0..2, coefficient bits of the
// three channels, vector bits).  Pass 2 adds the chunk sums of each (g,
// quantity); integer sums do not depend on the order.
constexpr int kTotThreads = 256;

__global__ void __launch_bounds__(kTotThreads) tile_totals_kernel(
    const unsigned long long* part, int64_t n, int chunks, unsigned long long* chunk_sum) {
  const int c = blockIdx.x, g = blockIdx.y;
  const int64_t per = (n + chunks - 1) / chunks;
  const int64_t j0 = (int64_t)c * per, j1 = j0 + per < n ? j0 + per : n;
  const unsigned long long* pg = part + (int64_t)g * n * kTileSums;
  unsigned long long v[5] = {0, 0, 0, 0, 0};
  int64_t j = j0 + threadIdx.x;
  for (; j + kTotThreads < j1; j += 2 * kTotThreads) {  // two records in flight
    unsigned long long r[2][kTileSums];
#pragma unroll
    for (int u = 0; u < 2; u++)
#pragma unroll
      for (int k = 0; k < kTileSums; k++) r[u][k] = pg[(j + u * kTotThreads) * kTileSums + k];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      v[0] += r[u][0];
      v[1] += r[u][1];
      v[2] += r[u][2];
      v[3] += r[u][3] + r[u][4] + r[u][5];
      v[4] += r[u][6];
    }
  }
  if (j < j1) {
    const unsigned long long* r = pg + j * kTileSums;
    v[0] += r[0];
    v[1] += r[1];
    v[2] += r[2];
    v[3] += r[3] + r[4] + r[5];
    v[4] += r[6];
  }
  __shared__ unsigned long long red[5][kTotThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 5; k++) {
    for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o);
    if (lane == 0) red[k][wv] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    unsigned long long t = 0;
    for (int w = 0; w < kTotThreads / 64; w++) t += red[threadIdx.x][w];
    chunk_sum[((int64_t)g * chunks + c) * 5 + threadIdx.x] = t;
  }
}

// One wave per (group, quantity): lane l adds chunks l, l + 64, ..., then a
// butterfly over the wave.
__global__ void __launch_bounds__(64) totals_finish_kernel(const unsigned long long* chunk_sum,
                                                          int chunks, unsigned long long* sse,
                                                          unsigned long long* bits) {
  const int g = blockIdx.x / 5, k = blockIdx.x - g * 5;
  unsigned long long t = 0;
  for (int c = threadIdx.x; c < chunks; c += 64) t += chunk_sum[((int64_t)g * chunks + c) * 5 + k];
  for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
  if (threadIdx.x == 0) {
    if (k < 3) sse[3 * g + k] = t;
    else bits[2 * g + k - 3] = t;
  }
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
  // vectors per frame: one per block, or one per N/2 cell with split flags
  const int64_t mvf = (p.split ? 4 : 1) * (int64_t)Hb * Wb;
  jb.mv = p.mv + f * mvf * 2;
  jb.split = p.split ? p.split + f * (int64_t)Hb * Wb : nullptr;
  jb.sad = p.sad_cell ? p.sad_cell + f * mvf : nullptr;
  jb.mv_whole = p.mv_whole ? p.mv_whole + f * (int64_t)Hb * Wb * 2 : nullptr;
  jb.sad_whole = p.sad_whole ? p.sad_whole + f * (int64_t)Hb * Wb : nullptr;
  jb.lambda16 = p.lambda16;
  jb.cbits = p.cbits ? p.cbits + f * 3 * (int64_t)Hb * Wb : nullptr;
  jb.mbits = p.mbits ? p.mbits + f * (int64_t)Hb * Wb : nullptr;
  jb.vmask = p.vmask ? p.vmask + f * 3 * plane : nullptr;
  jb.nan_total = p.nan_total;
  jb.part = p.part ? p.part + f * p.tpf * kTileSums : nullptr;
  // one prediction plane per stream (g, k), reused by the stream's steps
  const int ngop = (p.T + p.gop - 1) / p.gop;
  jb.pred = (p.pred && (s > 0 ? p.qpel : p.imode)) ? p.pred + ((int64_t)g * ngop + k) * 3 * plane
                                                    : nullptr;
  jb.Hp = p.Hp;
  jb.Wp = p.Wp;
  jb.H = p.H;
  jb.W = p.W;
  jb.nch = min(3, p.bands - 3 * g);
  jb.intra = s == 0;
  jb.imode = s == 0 && p.imode;
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

int encode_totals_chunks(int64_t tiles) {
  const int64_t c = (tiles + 8 * kTotThreads - 1) / (8 * kTotThreads);
  return (int)std::min<int64_t>(kTotMaxChunks, std::max<int64_t>(1, c));
}

hipError_t launch_encode_totals(const unsigned long long* part, int G, int T, int tpf,
                                unsigned long long* chunk_sum, unsigned long long* sse,
                                unsigned long long* bits, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  const int64_t n = (int64_t)T * tpf;
  const int chunks = encode_totals_chunks(n);
  tile_totals_kernel<<<dim3(chunks, G), kTotThreads, 0, s>>>(part, n, chunks, chunk_sum);
  totals_finish_kernel<<<5 * G, 64, 0, s>>>(chunk_sum, chunks, sse, bits);
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

int chunk_px_for(int64_t width, int bands) {
  int p = 64;
  while (p < kThreads && p < width) p <<= 1;
  while (p > 64 && p * bands > kStage) p >>= 1;
  return p;
}

namespace {
int gcd_int(int x, int y) {
  while (y) {
    const int r = x % y;
    x = y;
    y = r;
  }
  return x;
}
}  // namespace

int stats_blocks(const StatsArgs& a) {
  const int V = a.vec ? (a.dtype == XV_U16 ? 8 : 4) : 1;
  const int64_t nvec = a.npix * a.bands / V;
  int64_t b = (nvec + kThreads * 8 - 1) / (kThreads * 8);  // about 8 loads per thread
  b = b < 1 ? 1 : (b > kStatsMaxBlocks ? kStatsMaxBlocks : b);
  // the grid stride in elements must be a multiple of the band count
  const int m = a.bands / gcd_int(a.bands, kThreads * V);
  b = b / m * m;
  if (b < m) b = m;
  return (int)b;
}

hipError_t launch_stats(const StatsArgs& in, hipStream_t s) {
  StatsArgs a = in;
  a.nblocks = stats_blocks(a);
  if (a.dtype == XV_U16) {
    if (a.vec)
      stats_kernel<uint16_t, 8><<<a.nblocks, kThreads, 0, s>>>(a);
    else
      stats_kernel<uint16_t, 1><<<a.nblocks, kThreads, 0, s>>>(a);
  } else {
    if (a.vec)
      stats_kernel<float, 4><<<a.nblocks, kThreads, 0, s>>>(a);
    else
      stats_kernel<float, 1><<<a.nblocks, kThreads, 0, s>>>(a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  stats_finalize_kernel<<<a.bands, kFinThreads, 0, s>>>(a);
  return hipGetLastError();
}

// Pixels per group of the pixel-group kernels for (element size, bands).
int group_px(int elem, int bands) { return 16 / gcd_int(16, bands * elem); }

#define XV_BANDS_SWITCH(bands, CALL) \
  switch (bands) {                   \
    case 1: CALL(1); break;          \
    case 2: CALL(2); break;          \
    case 3: CALL(3); break;          \
    case 4: CALL(4); break;          \
    case 5: CALL(5); break;          \
    case 6: CALL(6); break;          \
    case 7: CALL(7); break;          \
    default: CALL(8); break;         \
  }

hipError_t launch_pack(const PackArgs& a, hipStream_t s) {
  const int elem = a.dtype == XV_U16 ? 2 : 4;
  const int g = group_px(elem, a.bands);
  if (a.bands <= 8 && ((uintptr_t)a.data & 15) == 0 && a.W % g == 0) {
    const int64_t n = a.T * a.Hp * (int64_t)((a.Wp + g - 1) / g);
    const int per = kThreads * vec_unroll(elem, g * a.bands);
    const unsigned grid = (unsigned)((n + per - 1) / per);
    if (a.dtype == XV_U16) {
#define XV_CALL(B) pack_vec_kernel<uint16_t, B><<<grid, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    } else {
#define XV_CALL(B) pack_vec_kernel<float, B><<<grid, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    }
    return hipGetLastError();
  }
  const int P = a.chunk_px;
  const int64_t blocks = a.T * a.Hp * (int64_t)((a.Wp + P - 1) / P);
  if (a.dtype == XV_U16)
    pack_kernel<uint16_t><<<(unsigned)blocks, P, stage_bytes(P, a.bands, 2), s>>>(a);
  else
    pack_kernel<float><<<(unsigned)blocks, P, stage_bytes(P, a.bands, 4), s>>>(a);
  return hipGetLastError();
}

hipError_t launch_denorm(const DenormArgs& a, hipStream_t s) {
  const int elem = a.out_dtype == XV_U16 ? 2 : 4;
  const int g = group_px(elem, a.bands);
  if (a.bands <= 8 && ((uintptr_t)a.out & 15) == 0 && a.W % g == 0) {
    const int64_t n = a.T * a.H * (a.W / g);
    const int per = kThreads * vec_unroll(elem, g * a.bands);
    const unsigned grid = (unsigned)((n + per - 1) / per);
    if (a.out_dtype == XV_U16) {
#define XV_CALL(B) denorm_vec_kernel<uint16_t, B><<<grid, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    } else {
#define XV_CALL(B) denorm_vec_kernel<float, B><<<grid, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    }
    return hipGetLastError();
  }
  const int P = a.chunk_px;
  const int64_t blocks = a.T * a.H * ((a.W + P - 1) / P);
  if (a.out_dtype == XV_U16)
    denorm_kernel<uint16_t><<<(unsigned)blocks, P, stage_bytes(P, a.bands, 2), s>>>(a);
  else
    denorm_kernel<float><<<(unsigned)blocks, P, stage_bytes(P, a.bands, 4), s>>>(a);
  return hipGetLastError();
}

// Blocks of the physical-error kernels (a grid-stride loop of equal work per
// block): up to 8192, several times what the chip holds at once, so that
// the last partial round of blocks is a small share of the launch.
int phys_blocks(int64_t npix) {
  int64_t b = (npix + kThreads * 16 - 1) / (kThreads * 16);
  return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

hipError_t launch_phys_sse(const PhysArgs& a, hipStream_t s) {
  const int elem = a.dtype == XV_U16 ? 2 : 4;
  const int g = group_px(elem, a.bands);
  if (a.bands <= 8 && ((uintptr_t)a.orig & 15) == 0 && a.W % g == 0) {
    if (a.dtype == XV_U16) {
#define XV_CALL(B) phys_vec_kernel<uint16_t, B><<<a.nblocks, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    } else {
#define XV_CALL(B) phys_vec_kernel<float, B><<<a.nblocks, kThreads, 0, s>>>(a)
      XV_BANDS_SWITCH(a.bands, XV_CALL)
#undef XV_CALL
    }
  } else if (a.dtype == XV_U16) {
    phys_sse_kernel<uint16_t><<<a.nblocks, kThreads, stage_bytes(a.chunk_px, a.bands, 2), s>>>(a);
  } else {
    phys_sse_kernel<float><<<a.nblocks, kThreads, stage_bytes(a.chunk_px, a.bands, 4), s>>>(a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  phys_reduce_kernel<<<a.bands, kThreads, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace xv
