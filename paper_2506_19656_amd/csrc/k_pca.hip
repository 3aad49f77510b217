// k_pca.hip -- principal components of the bands: the moments of the band
// vectors, the projection onto the principal axes and its inverse.
//
// The paper's library can replace the bands by their first k principal
// components before packing them into videos (Sec. II-A, the number of PCs
// in a mapping rule; Sec. III-C, the SimpleS2 runs).  It names no algorithm;
// the stated reading: every (t, y, x) of a u16 cube is one sample of the band
// vector; the mean and population covariance come from the exact integer
// sums S_b = sum x_b and Q_bc = sum x_b x_c (so the result does not depend on
// the order of summation); the eigen-decomposition of the small Bn x Bn
// matrix runs on the host; PC j of a sample is
// y_j = sum_b V[b][j] (x_b - m_b) in binary64, b increasing, rounded to
// binary32; the inverse from k PCs is x_b = m_b + sum_{j<k} V[b][j] y_j.
//
// Mapping: the moments kernel stages chunks of 256 pixels x Bn bands of its
// pixel range in LDS with coalesced loads; each thread owns one of the
// P = Bn (Bn + 3) / 2 sums (the upper triangle of Q and the S_b), or one of
// several copies of it that take every R-th pixel when P is small; its 64-bit
// partial cannot overflow (a block covers at most 2^32 / 1024 pixels).  A
// second kernel adds the per-block partials into 128-bit totals.  The
// projection and inverse are one thread per pixel, HBM-bound (2 B per band in,
// 4 B per PC out, and the reverse).
#include "xv_internal.h"

#include <algorithm>

namespace xv {

namespace {

constexpr int kMomThreads = 256;
constexpr int kMomChunk = 256;  // pixels staged per round

__host__ __device__ inline int pca_pairs(int Bn) { return Bn * (Bn + 1) / 2 + Bn; }

// Pair q < Bn (Bn + 1) / 2: (b, c) with b <= c in row-major order of the
// upper triangle; q >= that: S_{q - Bn (Bn + 1) / 2} (c = -1).
__device__ inline void pair_of(int q, int Bn, int& b, int& c) {
  const int tri = Bn * (Bn + 1) / 2;
  if (q >= tri) {
    b = q - tri;
    c = -1;
    return;
  }
  int row = 0, start = 0;
  while (q >= start + (Bn - row)) {
    start += Bn - row;
    row++;
  }
  b = row;
  c = row + (q - start);
}

constexpr int kMaxPer = 9;  // sums per thread when P > threads: 9 * 256 >= 64 * 67 / 2

__global__ void __launch_bounds__(kMomThreads) pca_moments_kernel(const PcaMomArgs a) {
  extern __shared__ uint16_t chunk[];  // [kMomChunk][Bn]
  __shared__ unsigned long long red[kMomThreads];
  const int Bn = a.bands;
  const int P = pca_pairs(Bn);
  const int R = P >= kMomThreads ? 1 : kMomThreads / P;  // copies of each sum
  const int per = (P + kMomThreads - 1) / kMomThreads;    // sums per thread (1 if R > 1)
  const int64_t p0 = a.npix * blockIdx.x / gridDim.x;
  const int64_t p1 = a.npix * (blockIdx.x + 1) / gridDim.x;
  const int t = (int)threadIdx.x;
  // R > 1: thread t = r P + q keeps copy r of sum q over pixels r, r + R, ...
  // R = 1: thread t keeps sums t, t + 256, ... over every pixel
  const int rep = R > 1 ? t / P : 0;
  const bool active = t < R * P || R == 1;
  unsigned long long acc[kMaxPer];
  int qb[kMaxPer], qc[kMaxPer];
#pragma unroll
  for (int u = 0; u < kMaxPer; u++) {
    acc[u] = 0;
    const int q = (R > 1 ? t % P : t) + u * kMomThreads;
    if (u < per && q < P && active) pair_of(q, Bn, qb[u], qc[u]);
    else qb[u] = qc[u] = -2;
  }
  const __attribute__((address_space(1))) uint16_t* src =
      (const __attribute__((address_space(1))) uint16_t*)a.data;
  for (int64_t c0 = p0; c0 < p1; c0 += kMomChunk) {
    const int n = (int)min<int64_t>(kMomChunk, p1 - c0);
    __syncthreads();
    for (int i = t; i < n * Bn; i += kMomThreads) chunk[i] = src[c0 * Bn + i];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kMaxPer; u++) {
      const int b = qb[u], c = qc[u];
      if (b < 0) continue;
      unsigned long long sum = 0;
      if (c < 0) {
        for (int p = rep; p < n; p += R) sum += chunk[p * Bn + b];
      } else {
        for (int p = rep; p < n; p += R)
          sum += (unsigned long long)((uint32_t)chunk[p * Bn + b] * (uint32_t)chunk[p * Bn + c]);
      }
      acc[u] += sum;
    }
  }
  if (R > 1) {
    // the copies of sum q sit at red[r P + q], r < R: fold them in a fixed order
    __syncthreads();
    red[t] = active ? acc[0] : 0ull;
    __syncthreads();
    if (t < P) {
      unsigned long long v = 0;
      for (int r = 0; r < R; r++) v += red[r * P + t];
      a.part[(int64_t)blockIdx.x * P + t] = v;
    }
  } else {
#pragma unroll
    for (int u = 0; u < kMaxPer; u++) {
      const int q = t + u * kMomThreads;
      if (u < per && q < P) a.part[(int64_t)blockIdx.x * P + q] = acc[u];
    }
  }
}

// 128-bit totals of the per-block partials: one thread per sum.
__global__ void pca_total_kernel(const PcaMomArgs a, int nblocks) {
  const int P = pca_pairs(a.bands);
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= P) return;
  unsigned long long lo = 0, hi = 0;
  for (int k = 0; k < nblocks; k++) {
    const unsigned long long v = a.part[(int64_t)k * P + q];
    lo += v;
    hi += lo < v ? 1ull : 0ull;
  }
  a.total[2 * q] = lo;
  a.total[2 * q + 1] = hi;
}

// BM bounds the band count at compile time so that the per-pixel vectors
// stay in registers for the common small counts.
template <int BM>
__global__ void __launch_bounds__(256) pca_project_kernel(const PcaProjArgs a) {
  __shared__ double mean[64];
  __shared__ double basis[64 * 64];
  const int Bn = a.bands;
  for (int i = threadIdx.x; i < Bn; i += blockDim.x) mean[i] = a.mean[i];
  for (int i = threadIdx.x; i < Bn * Bn; i += blockDim.x) basis[i] = a.basis[i];
  __syncthreads();
  const int k = a.j1 - a.j0;
  const __attribute__((address_space(1))) uint16_t* src =
      (const __attribute__((address_space(1))) uint16_t*)a.data;
  __attribute__((address_space(1))) float* dst = (__attribute__((address_space(1))) float*)a.out;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npix;
       p += (int64_t)gridDim.x * blockDim.x) {
    double d[BM];
#pragma unroll
    for (int b = 0; b < BM; b++) d[b] = b < Bn ? (double)src[p * Bn + b] - mean[b] : 0.0;
    for (int j = a.j0; j < a.j1; j++) {
      double y = 0.0;
#pragma unroll
      for (int b = 0; b < BM; b++)
        if (b < Bn) y = y + basis[b * Bn + j] * d[b];
      dst[p * k + (j - a.j0)] = (float)y;
    }
  }
}

template <int BM>
__global__ void __launch_bounds__(256) pca_inverse_kernel(const PcaInvArgs a) {
  __shared__ double mean[64];
  __shared__ double basis[64 * 64];
  const int Bn = a.bands;
  for (int i = threadIdx.x; i < Bn; i += blockDim.x) mean[i] = a.mean[i];
  for (int i = threadIdx.x; i < Bn * Bn; i += blockDim.x) basis[i] = a.basis[i];
  __syncthreads();
  const int k = a.k;
  const __attribute__((address_space(1))) float* src =
      (const __attribute__((address_space(1))) float*)a.pcs;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < a.npix;
       p += (int64_t)gridDim.x * blockDim.x) {
    double y[BM];
#pragma unroll
    for (int j = 0; j < BM; j++) y[j] = j < k ? (double)src[p * k + j] : 0.0;
    for (int b = 0; b < Bn; b++) {
      double x = mean[b];
#pragma unroll
      for (int j = 0; j < BM; j++)
        if (j < k) x = x + basis[b * Bn + j] * y[j];
      if (a.out_dtype == XV_U16) {
        // nearest integer, halves up, clamped to the u16 range
        double r = floor(x + 0.5);
        r = r < 0.0 ? 0.0 : (r > 65535.0 ? 65535.0 : r);
        ((__attribute__((address_space(1))) uint16_t*)a.out)[p * Bn + b] = (uint16_t)r;
      } else {
        ((__attribute__((address_space(1))) float*)a.out)[p * Bn + b] = (float)x;
      }
    }
  }
}

inline int grid_for_px(int64_t npix) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((npix + 255) / 256, 8192));
}

}  // namespace

int pca_moment_blocks(int64_t npix) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((npix + kMomChunk - 1) / kMomChunk, 1024));
}

int pca_sum_count(int bands) { return pca_pairs(bands); }

hipError_t launch_pca_moments(const PcaMomArgs& a, int nblocks, hipStream_t s) {
  if (a.bands < 1 || a.bands > 64) return hipErrorInvalidValue;
  if (pca_pairs(a.bands) > kMaxPer * kMomThreads) return hipErrorInvalidValue;
  const size_t lds = (size_t)kMomChunk * a.bands * sizeof(uint16_t);
  pca_moments_kernel<<<nblocks, kMomThreads, lds, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int P = pca_pairs(a.bands);
  pca_total_kernel<<<(P + 127) / 128, 128, 0, s>>>(a, nblocks);
  return hipGetLastError();
}

hipError_t launch_pca_project(const PcaProjArgs& a, hipStream_t s) {
  if (a.npix <= 0) return hipSuccess;
  if (a.bands < 1 || a.bands > 64 || a.j0 < 0 || a.j1 <= a.j0 || a.j1 > a.bands)
    return hipErrorInvalidValue;
  const int g = grid_for_px(a.npix);
  if (a.bands <= 4) pca_project_kernel<4><<<g, 256, 0, s>>>(a);
  else if (a.bands <= 8) pca_project_kernel<8><<<g, 256, 0, s>>>(a);
  else if (a.bands <= 16) pca_project_kernel<16><<<g, 256, 0, s>>>(a);
  else pca_project_kernel<64><<<g, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_pca_inverse(const PcaInvArgs& a, hipStream_t s) {
  if (a.npix <= 0) return hipSuccess;
  if (a.bands < 1 || a.bands > 64 || a.k < 1 || a.k > a.bands) return hipErrorInvalidValue;
  const int g = grid_for_px(a.npix);
  if (a.k <= 4) pca_inverse_kernel<4><<<g, 256, 0, s>>>(a);
  else if (a.k <= 8) pca_inverse_kernel<8><<<g, 256, 0, s>>>(a);
  else if (a.k <= 16) pca_inverse_kernel<16><<<g, 256, 0, s>>>(a);
  else pca_inverse_kernel<64><<<g, 256, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace xv
