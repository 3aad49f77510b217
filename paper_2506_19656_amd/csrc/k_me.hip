// k_me.hip -- full-search integer-pel block motion estimation for P pictures.
//
// For every N x N block of a P picture the vector (dx, dy) in [-R, R]^2 that
// keeps the displaced block inside the padded reference picture and minimises
// (SAD, |dx|+|dy|, dy, dx) lexicographically is chosen; SAD is summed over
// the channels of the band group that carry a real band.  The reference is
// the reconstruction of the previous picture (closed loop).  The paper's
// encoder (x265 behind ffmpeg) is a black box; this search is the stated
// reading of its motion-compensated prediction.
//
// Mapping onto gfx950:
//  * a workgroup owns a horizontal run of `nb` blocks; the union of their
//    search windows, (N + 2R) rows x (nb N + G KX) columns per channel, is
//    staged in LDS as packed u16 pairs with an odd dword pitch, so lanes that
//    differ in dy hit different banks;
//  * a lane evaluates KX consecutive candidates dx at one dy ("item") and
//    reuses every reference dword it loads for all KX of them;
//  * v_sad_u16 adds |a.lo-b.lo| + |a.hi-b.hi| in one instruction (two SAD
//    terms per lane-op); odd candidate offsets use pairs realigned with
//    alignbit;
//  * the argmin is one 64-bit key (SAD << 21 | L1 << 13 | raster index for
//    R <= 32; 23/15 for larger R) reduced with an LDS atomic min.
#include "xv_internal.h"

namespace xv {

namespace {

struct MeShape {
  int R, G, span, ipb;  // span = 2R+1, ipb = items per block
  int wc, pitch;        // window columns (u16) and pitch (dwords)
  int rows;             // N + 2R
};

__host__ __device__ inline MeShape me_shape(int N, int R, int kx, int nb) {
  MeShape s;
  s.R = R;
  s.span = 2 * R + 1;
  s.G = (s.span + kx - 1) / kx;
  s.ipb = s.span * s.G;
  s.wc = nb * N + s.G * kx;
  s.pitch = s.wc / 2;
  if ((s.pitch & 1) == 0) s.pitch += 1;
  s.rows = N + 2 * R;
  return s;
}

__host__ __device__ inline size_t me_lds_bytes(int N, const MeShape& s, int nb) {
  size_t win = (size_t)3 * s.rows * s.pitch * 4;
  size_t cur = (size_t)3 * N * (nb * N / 2) * 4;
  return win + cur + (size_t)nb * 8;
}

template <int N, int KX>
__global__ void __launch_bounds__(512) me_kernel(const LaunchDesc jd, int R, int nb) {
  extern __shared__ __align__(16) uint32_t lds[];
  int tl;
  const FrameJob& job = *desc_job(jd, blockIdx.x, tl);
  const int Hp = job.Hp, Wp = job.Wp;
  const int Hb = Hp / N, Wb = Wp / N;
  const int runs = (Wb + nb - 1) / nb;
  if (tl >= Hb * runs) return;
  const int by = tl / runs;
  const int bx0 = (tl - by * runs) * nb;
  const int nbv = min(nb, Wb - bx0);
  const int nch = job.nch;
  const MeShape s = me_shape(N, R, KX, nb);

  uint32_t* win = lds;
  uint32_t* curt = lds + 3 * s.rows * s.pitch;
  unsigned long long* best = (unsigned long long*)(curt + 3 * N * (nb * N / 2));
  const int cpitch = nb * N / 2;

  // Stage reference windows (zero outside the picture) and current blocks.
  const int gy0 = by * N - R, gx0 = bx0 * N - R;
  const int wpairs = s.wc / 2;
  const int nwin = nch * s.rows * wpairs;
  const size_t plane = (size_t)Hp * Wp;
  for (int e = threadIdx.x; e < nwin; e += blockDim.x) {
    const int ch = e / (s.rows * wpairs);
    const int rem = e - ch * s.rows * wpairs;
    const int row = rem / wpairs, m = rem - (rem / wpairs) * wpairs;
    const int gy = gy0 + row, gx = gx0 + 2 * m;
    uint32_t v0 = 0, v1 = 0;
    if (gy >= 0 && gy < Hp) {
      const uint16_t* rp = job.ref + ch * plane + (size_t)gy * Wp;
      if (gx >= 0 && gx < Wp) v0 = rp[gx];
      if (gx + 1 >= 0 && gx + 1 < Wp) v1 = rp[gx + 1];
    }
    win[(ch * s.rows + row) * s.pitch + m] = v0 | (v1 << 16);
  }
  const int ncur = nch * N * (nbv * N / 2);
  for (int e = threadIdx.x; e < ncur; e += blockDim.x) {
    const int per = N * (nbv * N / 2);
    const int ch = e / per;
    const int rem = e - ch * per;
    const int row = rem / (nbv * N / 2), m = rem - (rem / (nbv * N / 2)) * (nbv * N / 2);
    const uint32_t* cp = (const uint32_t*)(job.cur + ch * plane + (size_t)(by * N + row) * Wp +
                                           bx0 * N);
    curt[(ch * N + row) * cpitch + m] = cp[m];
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) best[b] = ~0ull;
  __syncthreads();

  constexpr int ND = (KX + N) / 2;  // reference dwords per row and item
  const int items = nbv * s.ipb;
  const int keyshift_sad = R <= 32 ? 21 : 23;
  const int keyshift_l1 = R <= 32 ? 13 : 15;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    const int b = it / s.ipb;
    const int rem = it - b * s.ipb;
    const int gxi = rem / s.span;
    const int dy = rem - gxi * s.span;
    uint32_t acc[KX];
#pragma unroll
    for (int k = 0; k < KX; k++) acc[k] = 0;
    for (int ch = 0; ch < nch; ch++) {
      const uint32_t* wbase = win + (ch * s.rows + dy) * s.pitch + (b * N + gxi * KX) / 2;
      const uint32_t* cbase = curt + ch * N * cpitch + b * (N / 2);
      // v_sad_u16 keeps its sum in 16 bits, so at most 8 of them (16 terms
      // of at most 4095) are chained into a partial before it is added to the
      // 32-bit SAD: RPP rows per partial for N < 16, two partials per row
      // for N = 32.
      constexpr int RPP = N >= 16 ? 1 : 16 / N;
      for (int i0 = 0; i0 < N; i0 += RPP) {
        uint32_t part[KX];
#pragma unroll
        for (int k = 0; k < KX; k++) part[k] = 0;
#pragma unroll
        for (int rr = 0; rr < RPP; rr++) {
          uint32_t D[ND], O[ND - 1], C[N / 2];
          const uint32_t* wr = wbase + (i0 + rr) * s.pitch;
#pragma unroll
          for (int q = 0; q < ND; q++) D[q] = wr[q];
#pragma unroll
          for (int q = 0; q < ND - 1; q++) O[q] = __builtin_amdgcn_alignbit(D[q + 1], D[q], 16);
#pragma unroll
          for (int m = 0; m < N / 2; m++) C[m] = cbase[(i0 + rr) * cpitch + m];
#pragma unroll
          for (int k = 0; k < KX; k++) {
#pragma unroll
            for (int m = 0; m < N / 2; m++) {
              const uint32_t pr = (k & 1) ? O[(k >> 1) + m] : D[(k >> 1) + m];
              part[k] = __builtin_amdgcn_sad_u16(pr, C[m], part[k]);
              if (N == 32 && m == 7) {
                acc[k] += part[k];
                part[k] = 0;
              }
            }
          }
        }
#pragma unroll
        for (int k = 0; k < KX; k++) acc[k] += part[k];
      }
    }
    const int x0 = (bx0 + b) * N, y0 = by * N;
    const int dyv = dy - R;
    unsigned long long kbest = ~0ull;
    const bool yok = (y0 + dyv >= 0) && (y0 + dyv + N <= Hp);
#pragma unroll
    for (int k = 0; k < KX; k++) {
      const int cx = gxi * KX + k;
      const int dxv = cx - R;
      const bool ok = yok && cx < s.span && (x0 + dxv >= 0) && (x0 + dxv + N <= Wp);
      const unsigned long long l1 = (unsigned long long)(abs(dxv) + abs(dyv));
      const unsigned long long key = ((unsigned long long)acc[k] << keyshift_sad) |
                                     (l1 << keyshift_l1) |
                                     (unsigned long long)(dy * s.span + cx);
      kbest = ok && key < kbest ? key : kbest;
    }
    if (kbest != ~0ull) atomicMin(&best[b], kbest);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbv; b += blockDim.x) {
    const unsigned long long key = best[b];
    const int idx = (int)(key & ((1ull << keyshift_l1) - 1));
    const int dy = idx / s.span - R, dx = idx - (idx / s.span) * s.span - R;
    int8_t* mv = job.mv + ((size_t)by * Wb + bx0 + b) * 2;
    mv[0] = (int8_t)dx;
    mv[1] = (int8_t)dy;
  }
}

template <int N, int KX>
hipError_t launch_me_t(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  const MeShape sh = me_shape(N, R, KX, g.nb);
  const size_t lds = me_lds_bytes(N, sh, g.nb);
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)me_kernel<N, KX>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  me_kernel<N, KX><<<r.tiles, g.threads, lds, s>>>(r, R, g.nb);
  return hipGetLastError();
}

template <int N>
hipError_t launch_me_n(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  switch (g.kx) {
    case 2: return launch_me_t<N, 2>(R, g, r, s);
    case 4: return launch_me_t<N, 4>(R, g, r, s);
    case 6: return launch_me_t<N, 6>(R, g, r, s);
    case 8: return launch_me_t<N, 8>(R, g, r, s);
    case 10: return launch_me_t<N, 10>(R, g, r, s);
    case 12: return launch_me_t<N, 12>(R, g, r, s);
    case 14: return launch_me_t<N, 14>(R, g, r, s);
    case 16: return launch_me_t<N, 16>(R, g, r, s);
    case 18: return launch_me_t<N, 18>(R, g, r, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

size_t me_lds_bytes_for(int N, int R, const MeGeom& g) {
  return me_lds_bytes(N, me_shape(N, R, g.kx, g.nb), g.nb);
}

MeGeom me_default_geometry(int N, int R) {
  const int span = 2 * R + 1;
  // candidates per lane: least wasted candidates, then the widest
  int kx = 2, waste = 1 << 30;
  for (int k = 2; k <= 18; k += 2) {
    int w = ((span + k - 1) / k) * k - span;
    if (w < waste || (w == waste && k > kx)) { waste = w; kx = k; }
  }
  // blocks per workgroup: best lane occupancy of the final round, LDS <= 64 KB
  const int threads = 256;
  int nb = 1;
  double bestf = -1.0;
  for (int c = 1; c <= 16; c++) {
    MeShape sh = me_shape(N, R, kx, c);
    if (me_lds_bytes(N, sh, c) > 64 * 1024 && c > 1) break;
    int items = c * sh.ipb;
    int rounds = (items + threads - 1) / threads;
    double f = (double)items / (double)(rounds * threads);
    if (f > bestf + 1e-9) { bestf = f; nb = c; }
  }
  return MeGeom{nb, kx, threads};
}

int me_tiles_per_job(int Hb, int Wb, const MeGeom& g) {
  return Hb * ((Wb + g.nb - 1) / g.nb);
}

hipError_t launch_me(int N, int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  if (g.threads <= 0 || g.threads > 512 || (g.threads & 63) || g.nb < 1) return hipErrorInvalidValue;
  if (me_lds_bytes_for(N, R, g) > 160 * 1024) return hipErrorInvalidValue;
  switch (N) {
    case 4: return launch_me_n<4>(R, g, r, s);
    case 8: return launch_me_n<8>(R, g, r, s);
    case 16: return launch_me_n<16>(R, g, r, s);
    case 32: return launch_me_n<32>(R, g, r, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xv
