// k_quality.hip -- the two quality metrics the paper reports beside PSNR
// (Sec. II-C): structural similarity and spectral angle.
//
// SSIM (Wang et al., 2004), coded domain: for every real channel of every
// frame, the converted frame q against its reconstruction, dynamic range
// L = 2^B - 1, an 11 x 11 Gaussian window of standard deviation 1.5 with unit
// sum, K1 = 0.01, K2 = 0.03, over every window position inside the real
// H x W picture.  A band scores the mean over its frames of the per-plane
// mean.  The window is separable, so a workgroup filters a tile of window
// positions in two passes through LDS: rows (11 taps, moment sums in
// binary64), then columns, then the SSIM of each position.  The variances
// enter SSIM only as their sum, so four moments suffice: the two means,
// E[a^2 + b^2] and E[ab].  Per-tile sums go to a partial array that one
// workgroup per band reduces in a fixed order.
//
// Spectral angle (Kruse et al., 1993): per pixel, arccos of the normalised
// dot product of the original and decoded band vectors, in binary64, pixels
// with a NaN or a zero-norm vector skipped; the mean over pixels.  A
// grid-stride kernel with a fixed grid writes per-block sums and counts that
// one workgroup reduces, so the result does not depend on scheduling.
#include "xv_internal.h"

namespace xv {

namespace {

constexpr int kTileX = 32;               // window positions per tile along x
constexpr int kTileY = 16;               // and along y
constexpr int kInX = kTileX + 10;        // input columns of a tile
constexpr int kInY = kTileY + 10;        // input rows of a tile
constexpr int kSsimThreads = 256;

struct alignas(16) SsimLds {
  double h[4][kInY][kTileX];             // row-filtered a, b, aa + bb, ab
  float a[kInY][kInX];                   // the tile's samples (exact in binary32)
  float b[kInY][kInX];
  double red[kSsimThreads / 64];
};

__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += red[i];
  return t;  // valid in thread 0
}

__global__ void __launch_bounds__(kSsimThreads) ssim_kernel(const SsimArgs a) {
  __shared__ SsimLds s;
  const int tiles = a.tiles_x * a.tiles_y;
  const int blk = blockIdx.x;
  const int tile = blk % tiles;
  const int plane = blk / tiles;             // band * T + t
  const int band = plane / a.T, t = plane - band * a.T;
  const int g = band / 3, c = band - 3 * g;
  const int ty = tile / a.tiles_x, tx = tile - ty * a.tiles_x;
  const int x0 = tx * kTileX, y0 = ty * kTileY;
  const size_t off = (((size_t)g * a.T + t) * 3 + c) * (size_t)a.Hp * a.Wp;
  const uint16_t* pa = a.frames + off;
  const uint16_t* pb = a.recon + off;

  for (int i = threadIdx.x; i < kInY * kInX; i += kSsimThreads) {
    const int r = i / kInX, q = i - r * kInX;
    const int y = y0 + r, x = x0 + q;
    const bool in = y < a.H && x < a.W;  // outside samples only feed skipped positions
    s.a[r][q] = in ? (float)pa[(size_t)y * a.Wp + x] : 0.0f;
    s.b[r][q] = in ? (float)pb[(size_t)y * a.Wp + x] : 0.0f;
  }
  __syncthreads();

  // Row pass: a thread filters 4 adjacent positions of one input row from 14
  // samples held in registers.
  constexpr int kHx = 4;
  for (int i = threadIdx.x; i < kInY * (kTileX / kHx); i += kSsimThreads) {
    const int r = i / (kTileX / kHx), j0 = (i - r * (kTileX / kHx)) * kHx;
    double u[kHx + 10], v[kHx + 10];
#pragma unroll
    for (int q = 0; q < kHx + 10; q++) {
      u[q] = (double)s.a[r][j0 + q];
      v[q] = (double)s.b[r][j0 + q];
    }
#pragma unroll
    for (int jj = 0; jj < kHx; jj++) {
      double sa = 0.0, sb = 0.0, ss = 0.0, sab = 0.0;
#pragma unroll
      for (int k = 0; k < 11; k++) {
        const double wu = a.w[k] * u[jj + k], wv = a.w[k] * v[jj + k];
        sa += wu;
        sb += wv;
        ss = fma(wv, v[jj + k], fma(wu, u[jj + k], ss));
        sab = fma(wu, v[jj + k], sab);
      }
      s.h[0][r][j0 + jj] = sa;
      s.h[1][r][j0 + jj] = sb;
      s.h[2][r][j0 + jj] = ss;
      s.h[3][r][j0 + jj] = sab;
    }
  }
  __syncthreads();

  // Column pass: a thread takes 2 vertically adjacent window positions, which
  // share 10 of their 11 filtered rows.
  double acc = 0.0;
  for (int i = threadIdx.x; i < (kTileY / 2) * kTileX; i += kSsimThreads) {
    const int r0 = (i / kTileX) * 2, j = i - (i / kTileX) * kTileX;
    double m0[4] = {0.0, 0.0, 0.0, 0.0}, m1[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 12; k++) {
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const double h = s.h[q][r0 + k][j];
        if (k < 11) m0[q] = fma(a.w[k], h, m0[q]);
        if (k > 0) m1[q] = fma(a.w[k - 1], h, m1[q]);
      }
    }
#pragma unroll
    for (int d = 0; d < 2; d++) {
      const double* m = d == 0 ? m0 : m1;
      if (y0 + r0 + d + 11 > a.H || x0 + j + 11 > a.W) continue;
      // sum of the variances, covariance
      const double mm = m[0] * m[0] + m[1] * m[1];
      const double vs = m[2] - mm;
      const double cab = m[3] - m[0] * m[1];
      acc += ((2.0 * m[0] * m[1] + a.C1) * (2.0 * cab + a.C2)) / ((mm + a.C1) * (vs + a.C2));
    }
  }
  const double tot = block_sum(acc, s.red);
  if (threadIdx.x == 0) a.part[blk] = tot;
}

// out[band] = sum of the band's tile sums / (windows per plane * T).
__global__ void __launch_bounds__(kSsimThreads) ssim_reduce_kernel(const SsimArgs a, double* out) {
  __shared__ double red[kSsimThreads / 64];
  const int band = blockIdx.x;
  const int64_t n = (int64_t)a.T * a.tiles_x * a.tiles_y;
  const double* p = a.part + (size_t)band * n;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kSsimThreads) v += p[i];
  const double tot = block_sum(v, red);
  if (threadIdx.x == 0) {
    const double nwin = (double)(a.H - 10) * (double)(a.W - 10);
    out[band] = tot / (nwin * (double)a.T);
  }
}

template <class T>
__device__ inline double sample(const T* p, int64_t i) {
  return (double)p[i];
}

template <class To, class Td>
__global__ void __launch_bounds__(kSaThreads) sa_kernel(const SaArgs a) {
  __shared__ double red[kSaThreads / 64];
  __shared__ unsigned long long redn[kSaThreads / 64];
  const To* o = (const To*)a.orig;
  const Td* d = (const Td*)a.dec;
  double acc = 0.0;
  unsigned long long cnt = 0;
  for (int64_t p = (int64_t)blockIdx.x * kSaThreads + threadIdx.x; p < a.npix;
       p += (int64_t)gridDim.x * kSaThreads) {
    double dot = 0.0, n1 = 0.0, n2 = 0.0;
    bool bad = false;
    for (int b = 0; b < a.bands; b++) {
      const double u = sample(o, p * a.bands + b), v = sample(d, p * a.bands + b);
      bad |= (u != u) || (v != v);
      dot += u * v;
      n1 += u * u;
      n2 += v * v;
    }
    if (bad || n1 == 0.0 || n2 == 0.0) continue;
    const double r = fmin(fmax(dot / (sqrt(n1) * sqrt(n2)), -1.0), 1.0);
    acc += acos(r);
    cnt++;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc += __shfl_down(acc, off);
    cnt += __shfl_down(cnt, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = acc;
    redn[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    unsigned long long n = 0;
    for (int i = 0; i < kSaThreads / 64; i++) {
      t += red[i];
      n += redn[i];
    }
    a.part_sum[blockIdx.x] = t;
    a.part_n[blockIdx.x] = n;
  }
}

// The same with both cubes of one dtype T and BANDS bands, 16-byte aligned,
// read as whole 16-byte granules: a group of g pixels is ne = g BANDS
// elements, and a thread loads U groups of each cube before any arithmetic
// (about 32 elements per cube), so that enough bytes are in flight.  Each
// pixel's sums run over its bands in the same order as above.
__host__ __device__ constexpr int sa_gcd(int x, int y) { return y == 0 ? x : sa_gcd(y, x % y); }
template <typename T, int BANDS>
struct SaGroup {
  static constexpr int g = 16 / sa_gcd(16, BANDS * (int)sizeof(T));  // pixels per group
  static constexpr int ne = g * BANDS;
  static constexpr int nv = ne * (int)sizeof(T) / 16;  // granules per group
  static constexpr int U = ne >= 32 ? 1 : (32 / ne > 4 ? 4 : 32 / ne);
};

template <typename T, int BANDS>
__global__ void __launch_bounds__(kSaThreads) sa_vec_kernel(const SaArgs a) {
  using SG = SaGroup<T, BANDS>;
  constexpr int U = SG::U;
  __shared__ double red[kSaThreads / 64];
  __shared__ unsigned long long redn[kSaThreads / 64];
  const T* o = (const T*)a.orig;
  const T* d = (const T*)a.dec;
  const int64_t ngroups = a.npix / SG::g;
  double acc = 0.0;
  unsigned long long cnt = 0;
  for (int64_t q0 = (int64_t)blockIdx.x * kSaThreads * U + threadIdx.x; q0 < ngroups;
       q0 += (int64_t)gridDim.x * kSaThreads * U) {
    T ov[U][SG::ne], dv[U][SG::ne];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t q = q0 + (int64_t)u * kSaThreads;
      if (q >= ngroups) break;
      uint4 wo[SG::nv], wd[SG::nv];
#pragma unroll
      for (int i = 0; i < SG::nv; i++) {
        wo[i] = ((const uint4*)(o + q * SG::ne))[i];
        wd[i] = ((const uint4*)(d + q * SG::ne))[i];
      }
      __builtin_memcpy(ov[u], wo, sizeof wo);
      __builtin_memcpy(dv[u], wd, sizeof wd);
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (q0 + (int64_t)u * kSaThreads >= ngroups) break;
#pragma unroll
      for (int p = 0; p < SG::g; p++) {
        double dot = 0.0, n1 = 0.0, n2 = 0.0;
        bool bad = false;
#pragma unroll
        for (int b = 0; b < BANDS; b++) {
          const double x = (double)ov[u][p * BANDS + b], y = (double)dv[u][p * BANDS + b];
          bad |= (x != x) || (y != y);
          dot += x * y;
          n1 += x * x;
          n2 += y * y;
        }
        if (bad || n1 == 0.0 || n2 == 0.0) continue;
        const double r = fmin(fmax(dot / (sqrt(n1) * sqrt(n2)), -1.0), 1.0);
        acc += acos(r);
        cnt++;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc += __shfl_down(acc, off);
    cnt += __shfl_down(cnt, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = acc;
    redn[w] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    unsigned long long n = 0;
    for (int i = 0; i < kSaThreads / 64; i++) {
      t += red[i];
      n += redn[i];
    }
    a.part_sum[blockIdx.x] = t;
    a.part_n[blockIdx.x] = n;
  }
}

__global__ void __launch_bounds__(kSaThreads) sa_reduce_kernel(const SaArgs a, int nblocks) {
  __shared__ double red[kSaThreads / 64];
  __shared__ unsigned long long redn[kSaThreads / 64];
  double v = 0.0;
  unsigned long long n = 0;
  for (int i = threadIdx.x; i < nblocks; i += kSaThreads) {
    v += a.part_sum[i];
    n += a.part_n[i];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_down(v, off);
    n += __shfl_down(n, off);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[w] = v;
    redn[w] = n;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    unsigned long long m = 0;
    for (int i = 0; i < kSaThreads / 64; i++) {
      t += red[i];
      m += redn[i];
    }
    a.out[0] = t;  // sum of angles; the host divides by the count
    ((unsigned long long*)a.out)[1] = m;
  }
}

}  // namespace

void ssim_tiles(int H, int W, int* tiles_x, int* tiles_y) {
  *tiles_x = (W - 10 + kTileX - 1) / kTileX;
  *tiles_y = (H - 10 + kTileY - 1) / kTileY;
}

hipError_t launch_ssim(const SsimArgs& a, double* out, hipStream_t s) {
  const int64_t blocks = (int64_t)a.bands * a.T * a.tiles_x * a.tiles_y;
  if (blocks <= 0 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  ssim_kernel<<<(unsigned)blocks, kSsimThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  ssim_reduce_kernel<<<a.bands, kSsimThreads, 0, s>>>(a, out);
  return hipGetLastError();
}

namespace {

// The granule kernel for both cubes of dtype T, if the shape and alignment
// allow it.
template <typename T>
bool launch_sa_vec(const SaArgs& a, int nblocks, hipStream_t s) {
  const int g = 16 / sa_gcd(16, a.bands * (int)sizeof(T));
  if (a.bands > 8 || a.npix % g != 0 || ((uintptr_t)a.orig & 15) || ((uintptr_t)a.dec & 15))
    return false;
  switch (a.bands) {
#define XV_SA(B) \
  case B:        \
    sa_vec_kernel<T, B><<<nblocks, kSaThreads, 0, s>>>(a); \
    return true;
    XV_SA(1) XV_SA(2) XV_SA(3) XV_SA(4) XV_SA(5) XV_SA(6) XV_SA(7) XV_SA(8)
#undef XV_SA
    default: return false;
  }
}

}  // namespace

hipError_t launch_spectral_angle(const SaArgs& a, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipErrorInvalidValue;
  if (a.dtype_orig == a.dtype_dec &&
      (a.dtype_orig == XV_U16 ? launch_sa_vec<uint16_t>(a, nblocks, s)
                              : launch_sa_vec<float>(a, nblocks, s))) {
  } else if (a.dtype_orig == XV_U16 && a.dtype_dec == XV_U16)
    sa_kernel<uint16_t, uint16_t><<<nblocks, kSaThreads, 0, s>>>(a);
  else if (a.dtype_orig == XV_U16)
    sa_kernel<uint16_t, float><<<nblocks, kSaThreads, 0, s>>>(a);
  else if (a.dtype_dec == XV_U16)
    sa_kernel<float, uint16_t><<<nblocks, kSaThreads, 0, s>>>(a);
  else
    sa_kernel<float, float><<<nblocks, kSaThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  sa_reduce_kernel<<<1, kSaThreads, 0, s>>>(a, nblocks);
  return hipGetLastError();
}

}  // namespace xv
