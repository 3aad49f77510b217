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
//    search windows is staged in LDS with an odd dword pitch, so lanes that
//    read different window rows hit different banks;
//  * v_sad_u16 adds |a.lo-b.lo| + |a.hi-b.hi| in one instruction (two SAD
//    terms per lane-op).  Two window layouts pair the samples differently:
//    column pairs (two horizontally adjacent samples per dword; odd
//    candidate offsets realigned with alignbit; a lane takes KX candidate
//    columns on ROWS candidate rows and reuses every loaded dword for all of
//    them) and row pairs (two vertically adjacent samples per dword, so any
//    column offset reads whole dwords; a lane takes KX candidate columns of
//    one candidate row), the latter optionally staged channel by channel;
//  * the argmin is one 64-bit key (SAD << 21 | L1 << 13 | raster index for
//    R <= 32; 23/15 for larger R) reduced with an LDS atomic min.
#include "xv_internal.h"

#include <algorithm>

#ifndef XV_INLINE
#define XV_INLINE __attribute__((always_inline))
#endif
#include <vector>

namespace xv {

namespace {

// An item is (block, group of KX candidate columns, ROWS consecutive
// candidate rows dy0 .. dy0 + ROWS - 1).  A lane sums all ROWS rows' SADs
// from one pass over the N + ROWS - 1 window rows they share.
struct MeShape {
  int R, G, span, dyp, ipb;  // span = 2R+1; dyp = row groups; ipb = items per block
  int wc, pitch;             // window columns (u16) and pitch (dwords)
  int rows;                  // staged rows ROWS * dyp + N - 1 (rows past N + 2R only
                             // serve candidate rows outside the range)
};

__host__ __device__ inline MeShape me_shape(int N, int R, int kx, int nb, int nrow) {
  MeShape s;
  s.R = R;
  s.span = 2 * R + 1;
  s.G = (s.span + kx - 1) / kx;
  s.dyp = (s.span + nrow - 1) / nrow;
  s.ipb = s.dyp * s.G;
  s.wc = nb * N + s.G * kx;
  s.pitch = s.wc / 2;
  if ((s.pitch & 1) == 0) s.pitch += 1;
  s.rows = nrow * s.dyp + N - 1;
  return s;
}

// LDS layout of a workgroup, in dwords: the windows [3][rows][pitch], the
// current blocks [3][N][nb N / 2] from a 16-byte boundary, then the nb 64-bit
// argmin keys from an 8-byte boundary (rows * pitch may be odd).
struct MeLds {
  size_t cur, best, bytes;
};

__host__ __device__ inline MeLds me_lds_layout(int N, const MeShape& s, int nb) {
  MeLds l;
  const size_t win = (size_t)3 * s.rows * s.pitch;
  l.cur = (win + 3) & ~(size_t)3;
  l.best = (l.cur + (size_t)3 * N * (nb * N / 2) + 1) & ~(size_t)1;
  l.bytes = l.best * 4 + (size_t)nb * 8;
  return l;
}

__host__ __device__ inline size_t me_lds_bytes(int N, const MeShape& s, int nb) {
  return me_lds_layout(N, s, nb).bytes;
}

// Global-memory views of the job's pointers (they are stored as generic
// pointers in the job table; these casts let the loads be global loads that
// only count against the vector-memory counter).
typedef const __attribute__((address_space(1))) uint16_t gu16;
typedef const __attribute__((address_space(1))) uint32_t gu32;

constexpr int kBatch = 8;  // staging loads in flight per thread

// Stages the reference windows of one workgroup: per channel, s.rows rows of
// wpairs u16 pairs starting at column gx0, zero outside the picture.
// Thread t covers pair column t % wpairs of rows t / wpairs + k * rpp; loads
// are issued kBatch at a time from clamped (always in-bounds) addresses and
// masked afterwards.  With an even gx0 a pair is wholly inside or wholly
// outside the picture (Wp is even), so one dword load serves it.  Offsets
// are 32-bit byte offsets from the channel plane (a padded frame stays below
// 2^31 bytes, which the host checks).
typedef const __attribute__((address_space(1))) char gchar;
typedef uint32_t u32x4_l __attribute__((ext_vector_type(4)));

template <bool kEven>
__device__ inline void stage_window(uint32_t* win, const uint16_t* ref, const MeShape& s, int nch,
                                    int wpairs, int gx0, int gy0, int Hp, int Wp) {
  const uint32_t plane_bytes = 2u * (uint32_t)Hp * (uint32_t)Wp;
  const int rpp = max(1, (int)blockDim.x / wpairs);  // rows per pass
  const int r0 = threadIdx.x / wpairs;
  if (r0 >= rpp) return;
  for (int m = threadIdx.x - r0 * wpairs; m < wpairs; m += (int)blockDim.x) {
    const int gx = gx0 + 2 * m;
    const bool in0 = gx >= 0 && gx < Wp, in1 = gx + 1 >= 0 && gx + 1 < Wp;
    const uint32_t bx0 = 2u * (uint32_t)min(max(gx, 0), Wp - 1);
    const uint32_t bx1 = 2u * (uint32_t)min(max(gx + 1, 0), Wp - 1);
    const uint32_t bxe = 2u * (uint32_t)min(max(gx, 0), Wp - 2);
    for (int ch = 0; ch < nch; ch++) {
      gchar* base = (gchar*)ref + (size_t)ch * plane_bytes;
      uint32_t* wch = win + ch * s.rows * s.pitch + m;
      for (int rb = r0; rb < s.rows; rb += kBatch * rpp) {
        uint32_t v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
          const int gy = gy0 + min(rb + u * rpp, s.rows - 1);
          const bool yin = (unsigned)gy < (unsigned)Hp;
          // row * Wp < 2^31 / 6, so the 24-bit multiply is exact
          const uint32_t row = 2u * __umul24((uint32_t)min(max(gy, 0), Hp - 1), (uint32_t)Wp);
          if constexpr (kEven) {
            const uint32_t off = row + bxe;
            const uint32_t w = *(const __attribute__((address_space(1))) uint32_t*)(base + off);
            v[u] = (yin && in0) ? w : 0u;
          } else {
            const uint32_t o0 = row + bx0, o1 = row + bx1;
            const uint32_t lo = *(const __attribute__((address_space(1))) uint16_t*)(base + o0);
            const uint32_t hi = *(const __attribute__((address_space(1))) uint16_t*)(base + o1);
            v[u] = ((yin && in0) ? lo : 0u) | (((yin && in1) ? hi : 0u) << 16);
          }
        }
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
          const int rr = rb + u * rpp;
          if (rr < s.rows) wch[rr * s.pitch] = v[u];
        }
      }
    }
  }
}

template <int N, int KX, int ROWS>
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
  const MeShape s = me_shape(N, R, KX, nb, ROWS);

  const MeLds ll = me_lds_layout(N, s, nb);
  uint32_t* win = lds;
  uint32_t* curt = lds + ll.cur;
  unsigned long long* best = (unsigned long long*)(lds + ll.best);
  const int cpitch = nb * N / 2;

  // Stage the reference windows and the current blocks, kBatch loads in
  // flight per thread.
  const int gy0 = by * N - R, gx0 = bx0 * N - R;
  const int wpairs = s.wc / 2;
  if ((gx0 & 1) == 0)
    stage_window<true>(win, job.ref, s, nch, wpairs, gx0, gy0, Hp, Wp);
  else
    stage_window<false>(win, job.ref, s, nch, wpairs, gx0, gy0, Hp, Wp);
  {
    const int cw = nbv * N / 2;  // dwords per current row
    const int rpp = max(1, (int)blockDim.x / cw);
    const int r0 = threadIdx.x / cw;
    const int crows = nch * N;
    for (int m = threadIdx.x - r0 * cw; m < cw; m += (int)blockDim.x) {
      if (r0 >= rpp) break;
      for (int rb = r0; rb < crows; rb += kBatch * rpp) {
        uint32_t v[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
          const int rr = min(rb + u * rpp, crows - 1);
          const int ch = rr / N, row = rr - (rr / N) * N;  // N is a power of two
          const uint32_t off =
              4u * (uint32_t)m + 2u * __umul24((uint32_t)(ch * Hp + by * N + row), (uint32_t)Wp) +
              2u * (uint32_t)(bx0 * N);
          v[u] = *(const __attribute__((address_space(1))) uint32_t*)((gchar*)job.cur + off);
        }
#pragma unroll
        for (int u = 0; u < kBatch; u++) {
          const int rr = rb + u * rpp;
          if (rr < crows) curt[rr * cpitch + m] = v[u];
        }
      }
    }
  }
  for (int b = threadIdx.x; b < nb; b += blockDim.x) best[b] = ~0ull;
  __syncthreads();

  constexpr int ND = (KX + N) / 2;  // reference dwords per row and item
  constexpr int NC = N / 2;         // current dwords per row
  // Only items holding a candidate that keeps the displaced block inside the
  // padded picture are evaluated: candidate rows dy + R in [rlo, rhi] (the
  // same for every block of the run) and, per block, candidate columns
  // dx + R in [max(0, R - x0), min(2R, Wp - N - x0 + R)].  Consecutive items
  // of a block differ in their row group, so neighbouring lanes read window
  // rows a pitch apart.
  const int y0b = by * N;
  const int glo_r = max(0, R - y0b) / ROWS;
  const int ndy = min(s.span - 1, Hp - N - y0b + R) / ROWS - glo_r + 1;
  int items = 0;
  for (int b = 0; b < nbv; b++) {
    const int x0 = (bx0 + b) * N;
    items += ndy * (min(s.span - 1, Wp - N - x0 + R) / KX - max(0, R - x0) / KX + 1);
  }
  const int keyshift_sad = R <= 32 ? 21 : 23;
  const int keyshift_l1 = R <= 32 ? 13 : 15;
  const float inv_ndy = 1.0f / (float)ndy;
  for (int it = threadIdx.x; it < items; it += blockDim.x) {
    int b = 0, rem = it, glo_c = 0;
    for (;; b++) {
      const int x0 = (bx0 + b) * N;
      glo_c = max(0, R - x0) / KX;
      const int n = ndy * (min(s.span - 1, Wp - N - x0 + R) / KX - glo_c + 1);
      if (rem < n || b + 1 >= nbv) break;
      rem -= n;
    }
    // rem / ndy in binary32 (exact: quotient below 2R + 2, distance from an
    // integer at least 1/(2 ndy))
    const int gq = (int)(((float)rem + 0.5f) * inv_ndy);
    const int gxi = glo_c + gq;
    const int dy0 = ROWS * (glo_r + rem - gq * ndy);
    uint32_t acc[ROWS][KX];
#pragma unroll
    for (int h = 0; h < ROWS; h++)
#pragma unroll
      for (int k = 0; k < KX; k++) acc[h][k] = 0;
    for (int ch = 0; ch < nch; ch++) {
      const uint32_t* wbase = win + (ch * s.rows + dy0) * s.pitch + (b * N + gxi * KX) / 2;
      const uint32_t* cbase = curt + ch * N * cpitch + b * NC;
      uint32_t D[ND], O[ND - 1], CA[NC], CB[NC];
      // window row w serves candidate row dy0 + h with current row w - h
      auto load_win = [&](int w) {
        const uint32_t* wr = wbase + w * s.pitch;
#pragma unroll
        for (int q = 0; q < ND; q++) D[q] = wr[q];
#pragma unroll
        for (int q = 0; q < ND - 1; q++) O[q] = __builtin_amdgcn_alignbit(D[q + 1], D[q], 16);
      };
      auto load_cur = [&](int w, uint32_t(&C)[NC]) {
#pragma unroll
        for (int m = 0; m < NC; m++) C[m] = cbase[w * cpitch + m];
      };
      auto sad = [&](uint32_t(&acc)[KX], const uint32_t(&C)[NC]) {
#pragma unroll
        for (int k = 0; k < KX; k++) {
#pragma unroll
          for (int m = 0; m < NC; m++) {
            const uint32_t pr = (k & 1) ? O[(k >> 1) + m] : D[(k >> 1) + m];
            acc[k] = __builtin_amdgcn_sad_u16(pr, C[m], acc[k]);
          }
        }
      };
      if constexpr (ROWS == 1) {
#pragma unroll 2
        for (int w = 0; w < N; w++) {
          load_win(w);
          load_cur(w, CA);
          sad(acc[0], CA);
        }
      } else if constexpr (ROWS == 2) {
        load_win(0);
        load_cur(0, CA);
        sad(acc[0], CA);
        for (int w = 1; w + 1 < N; w += 2) {
          load_win(w);
          load_cur(w, CB);
          sad(acc[0], CB);
          sad(acc[1], CA);
          load_win(w + 1);
          load_cur(w + 1, CA);
          sad(acc[0], CA);
          sad(acc[1], CB);
        }
        load_win(N - 1);
        load_cur(N - 1, CB);
        sad(acc[0], CB);
        sad(acc[1], CA);
        load_win(N);
        sad(acc[1], CB);
      } else {
        // ring of the last ROWS current rows: current row r lives in slot
        // r % ROWS; the loop is unrolled by ROWS so every slot index is a
        // compile-time constant
        uint32_t ring[ROWS][NC];
        constexpr int NW = N + ROWS - 1;  // window rows of the item
        for (int w0 = 0; w0 < NW; w0 += ROWS) {
#pragma unroll
          for (int j = 0; j < ROWS; j++) {
            const int w = w0 + j;
            if (w < NW) {
              load_win(w);
              if (w < N) load_cur(w, ring[j]);
#pragma unroll
              for (int h = 0; h < ROWS; h++)
                if (w - h >= 0 && w - h < N) sad(acc[h], ring[(j - h + ROWS) % ROWS]);
            }
          }
        }
      }
    }
    // Best candidate of the item.  SAD < 2^24 and L1 <= 128, so (SAD, L1)
    // fits one 32-bit key; candidates are visited in increasing raster
    // index (dy, then dx), so a strict < keeps the smallest index among
    // equal keys and the item's winner is its lexicographic minimum of
    // (SAD, L1, dy, dx).  Only that one gets the full 64-bit key.
    const int x0 = (bx0 + b) * N, y0 = by * N;
    const int c0 = gxi * KX;
    const int klo = max(0, R - x0) - c0;                        // displaced block inside
    const int khi = min(s.span - 1, Wp - N - x0 + R) - c0;      // the padded picture
    uint32_t kb32 = 0xffffffffu;
    int bsel = -1;
    const uint32_t cx = (uint32_t)(c0 + KX);  // below 2^16, as is R + KX - k
#pragma unroll
    for (int h = 0; h < ROWS; h++) {
      const int dyv = dy0 + h - R;
      const bool yok = dy0 + h < s.span && (y0 + dyv >= 0) && (y0 + dyv + N <= Hp);
      const uint32_t ly = (uint32_t)abs(dyv);
#pragma unroll
      for (int k = 0; k < KX; k++) {
        // L1 = |c0 + k - R| + |dy|, the first term as a 16-bit absolute difference
        const uint32_t l1 = __builtin_amdgcn_sad_u16(cx, (uint32_t)(R + KX - k), ly);
        const uint32_t key = (acc[h][k] << 8) | l1;
        const bool take = yok && k >= klo && k <= khi && key < kb32;
        kb32 = take ? key : kb32;
        bsel = take ? h * KX + k : bsel;
      }
    }
    if (bsel >= 0) {
      const int h = bsel / KX, k = bsel - h * KX;
      const unsigned long long idx = (unsigned long long)((dy0 + h) * s.span + c0 + k);
      const unsigned long long key = ((unsigned long long)(kb32 >> 8) << keyshift_sad) |
                                     ((unsigned long long)(kb32 & 0xffu) << keyshift_l1) | idx;
      atomicMin(&best[b], key);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbv; b += blockDim.x) {
    const unsigned long long key = best[b];
    const int idx = (int)(key & ((1ull << keyshift_l1) - 1));
    const int dy = idx / s.span - R, dx = idx - (idx / s.span) * s.span - R;
    int8_t* mv = job.mv + ((size_t)by * Wb + bx0 + b) * 2;
    mv[0] = (int8_t)dx;
    mv[1] = (int8_t)dy;
    if (job.sad) job.sad[(size_t)by * Wb + bx0 + b] = (uint32_t)(key >> keyshift_sad);
  }
}

// ---- Row-pair layout --------------------------------------------------
//
// The second layout stores, for every window row r and column c, the dword
// (w[r][c], w[r+1][c]): two vertically adjacent samples.  A candidate at any
// column offset then reads whole dwords (no realignment), and candidate row r
// pairs its window rows r + 2j, r + 2j + 1 with current rows 2j, 2j + 1,
// stored paired the same way.  A lane evaluates KX consecutive candidate
// columns of one candidate row; KX need not be even, so a group size that
// divides the span 2R+1 (3 or 11 for R = 16) leaves no column unused.  The
// window is twice the bytes of the column-pair one.
struct RpShape {
  int span, xr, wc, pitch;  // xr pair rows; wc staged columns (even); pitch odd, dwords
};

__host__ __device__ inline RpShape rp_shape(int N, int R, int kx, int nb) {
  RpShape s;
  s.span = 2 * R + 1;
  s.xr = 2 * R + N - 1;
  s.wc = nb * N + 2 * R + kx - 1;
  s.wc += s.wc & 1;
  s.pitch = s.wc + 1;
  return s;
}

// LDS of a workgroup, in dwords: pair rows [C][xr][pitch], paired current
// blocks [C][nb][N/2][N] from a 16-byte boundary, nb 64-bit keys; C = 3
// channels resident at once, or 1 when they are staged one after another.
__host__ __device__ inline MeLds rp_lds_layout(int N, const RpShape& s, int nb, int chans,
                                               int keys = 1) {
  MeLds l;
  const size_t x = (size_t)chans * s.xr * s.pitch;
  l.cur = (x + 3) & ~(size_t)3;
  l.best = l.cur + (size_t)chans * nb * (N / 2) * N;  // a multiple of 4 past cur
  l.bytes = l.best * 4 + (size_t)nb * keys * 8;
  return l;
}

// Items per thread held across the channels when they are staged one after
// another.
constexpr int kRpRounds = 3;

// Stages the pair rows of the window.  A thread owns column pair m (window
// columns 2m, 2m+1 at picture columns gx0 + 2m, gx0 + 2m + 1) and walks the
// (channel, chunk of kRc pair rows) tasks q0, q0 + qstep, ...; a task loads
// kRc + 1 window rows (zero outside the picture) and writes 2 kRc pair
// dwords.  Offsets are 32-bit byte offsets from the uniform frame base (a
// padded frame of three channels stays below 2^31 bytes).
template <bool kEven>
__device__ inline void stage_row_pairs(uint32_t* X, const uint16_t* ref, const RpShape& s,
                                       int nch, int gx0, int gy0, int Hp, int Wp) {
  constexpr int kRc = 8;
  typedef const __attribute__((address_space(1))) uint32_t gu32_t;
  typedef const __attribute__((address_space(1))) uint16_t gu16_t;
  const uint32_t plane_bytes = 2u * (uint32_t)Hp * (uint32_t)Wp;
  const uint32_t step = 2u * (uint32_t)Wp;
  gchar* base = (gchar*)ref;
  const int mp = s.wc / 2;
  const int nk = (s.xr + kRc - 1) / kRc;
  const int qstep = max(1, (int)blockDim.x / mp);
  const int q0 = (int)threadIdx.x / mp;
  if (q0 >= qstep) return;
  for (int m = (int)threadIdx.x - q0 * mp; m < mp; m += (int)blockDim.x) {
    const int gx = gx0 + 2 * m;
    const bool in0 = gx >= 0 && gx < Wp, in1 = gx + 1 >= 0 && gx + 1 < Wp;
    const uint32_t bx0 = 2u * (uint32_t)min(max(gx, 0), Wp - 1);
    const uint32_t bx1 = 2u * (uint32_t)min(max(gx + 1, 0), Wp - 1);
    const uint32_t bxe = 2u * (uint32_t)min(max(gx, 0), Wp - 2);
    int ch = q0 / nk, k = q0 - (q0 / nk) * nk;
    for (; ch < nch;) {
      const uint32_t cho = (uint32_t)ch * plane_bytes;
      const int r0 = k * kRc;
      uint32_t v[kRc + 1];
      if (gy0 + r0 >= 0 && gy0 + r0 + kRc < Hp) {
        // all rows inside the picture: one row offset, stepped
        uint32_t row = cho + 2u * __umul24((uint32_t)(gy0 + r0), (uint32_t)Wp);
        if constexpr (kEven) {
          // an even column pair lies wholly inside or wholly outside
          if (in0) {
#pragma unroll
            for (int u = 0; u <= kRc; u++, row += step) v[u] = *(gu32_t*)(base + (row + bxe));
          } else {
#pragma unroll
            for (int u = 0; u <= kRc; u++) v[u] = 0u;
          }
        } else {
#pragma unroll
          for (int u = 0; u <= kRc; u++, row += step) {
            const uint32_t lo = *(gu16_t*)(base + (row + bx0));
            const uint32_t hi = *(gu16_t*)(base + (row + bx1));
            v[u] = (in0 ? lo : 0u) | ((in1 ? hi : 0u) << 16);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u <= kRc; u++) {
          const int gy = gy0 + r0 + u;
          const bool yin = (unsigned)gy < (unsigned)Hp;
          const uint32_t row = cho + 2u * __umul24((uint32_t)min(max(gy, 0), Hp - 1), (uint32_t)Wp);
          if constexpr (kEven) {
            const uint32_t w = *(gu32_t*)(base + (row + bxe));
            v[u] = (yin && in0) ? w : 0u;
          } else {
            const uint32_t lo = *(gu16_t*)(base + (row + bx0));
            const uint32_t hi = *(gu16_t*)(base + (row + bx1));
            v[u] = ((yin && in0) ? lo : 0u) | (((yin && in1) ? hi : 0u) << 16);
          }
        }
      }
      uint32_t* xo = X + (ch * s.xr + r0) * s.pitch + 2 * m;
      if (r0 + kRc <= s.xr) {
#pragma unroll
        for (int u = 0; u < kRc; u++) {
          xo[u * s.pitch] = (v[u] & 0xffffu) | (v[u + 1] << 16);
          xo[u * s.pitch + 1] = (v[u] >> 16) | (v[u + 1] & 0xffff0000u);
        }
      } else {
#pragma unroll
        for (int u = 0; u < kRc; u++) {
          if (r0 + u < s.xr) {
            xo[u * s.pitch] = (v[u] & 0xffffu) | (v[u + 1] << 16);
            xo[u * s.pitch + 1] = (v[u] >> 16) | (v[u + 1] & 0xffff0000u);
          }
        }
      }
      k += qstep;
      while (k >= nk) {
        k -= nk;
        ch++;
      }
    }
  }
}

// pair rows unrolled per channel: all of them up to N = 16, two for N = 32
template <int N>
constexpr int kRpUnroll = N <= 16 ? N / 2 : 2;
// the same over half a block's pair rows (the combined search's halves)
template <int N>
constexpr int kRpUnrollHalf = N <= 16 ? N / 4 : 2;

// Row-pair motion search.  RND = 0: the three channels' windows are
// resident together and a thread takes its items one at a time.  RND > 0:
// the channels are staged one after another into a third of the LDS, and a
// thread keeps the sums of its (at most RND) items across them.
//
// SP = 1: the search of the adaptive block size, whole blocks and their four
// N/2 cells in one pass.  A candidate's SAD over a block is the sum of its
// SADs over the four cells, so the sums are kept per cell (top/bottom half of
// the pair rows, left/right half of the columns) and each of the five
// targets (the block, its cells in z-order) takes its own lexicographic
// minimum over the candidates that keep that target inside the picture.  The
// candidate set is the union of the targets' (a cell near the picture's
// left or top edge reaches further than its block); the staged window
// covers every candidate in [-R, R]^2 with zeros outside the picture, which
// only candidates invalid for a target read, for that target.  Outputs: the
// block's vector and SAD to mv_whole / sad_whole, the cells' to the cell
// grid (mv / sad), exactly what the separate searches at N and N/2 give.
// Waves per SIMD the register allocator is asked to leave room for: 4 for
// the plain search (the widest instances otherwise take 3, and every
// instance reaches 4 without spilling); the launch bound's 2 for the
// combined search (5 for the instances that reach it, with chunks of one
// cell column to save registers, measured slower).  Resident waves still
// depend on LDS and workgroup size.
template <int SP>
constexpr int kRpWaves = SP ? 2 : 4;

template <int N, int KX, int RND, int SP = 0>
__global__ void __launch_bounds__(512)
    __attribute__((amdgpu_waves_per_eu(kRpWaves<SP>)))
    me_rp_kernel(const LaunchDesc jd, int R, int nb) {
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
  const RpShape s = rp_shape(N, R, KX, nb);
  constexpr int KEYS = SP ? 5 : 1;  // targets per block
  const MeLds ll = rp_lds_layout(N, s, nb, RND == 0 ? 3 : 1, KEYS);
  uint32_t* X = lds;
  uint32_t* curx = lds + ll.cur;
  unsigned long long* best = (unsigned long long*)(lds + ll.best);
  const int gy0 = by * N - R, gx0 = bx0 * N - R;
  const uint32_t plane_bytes = 2u * (uint32_t)Hp * (uint32_t)Wp;

  // Stages channels c0 .. c0 + cn - 1 into LDS slots 0 .. cn - 1: the pair
  // rows of the window and the current blocks, dword (c[2j][x], c[2j+1][x])
  // at [slot][b][j][x].
  auto stage = [&](int c0, int cn) XV_INLINE {
    const uint16_t* ref = (const uint16_t*)((gchar*)job.ref + (size_t)c0 * plane_bytes);
    if ((gx0 & 1) == 0)
      stage_row_pairs<true>(X, ref, s, cn, gx0, gy0, Hp, Wp);
    else
      stage_row_pairs<false>(X, ref, s, cn, gx0, gy0, Hp, Wp);
    constexpr int CM = N / 2;  // column pairs of a block row
    const int tasks = nbv * (N / 2) * CM;
    for (int ch = 0; ch < cn; ch++)
      for (int t = threadIdx.x; t < tasks; t += blockDim.x) {
        const int m = t % CM, q = t / CM;
        const int j = q % (N / 2), b = q / (N / 2);
        const uint32_t off =
            2u * __umul24((uint32_t)((c0 + ch) * Hp + by * N + 2 * j), (uint32_t)Wp) +
            2u * (uint32_t)((bx0 + b) * N + 2 * m);
        const uint32_t a0 = *(const __attribute__((address_space(1))) uint32_t*)((gchar*)job.cur + off);
        const uint32_t a1 = *(const __attribute__((address_space(1))) uint32_t*)(
            (gchar*)job.cur + (off + 2u * (uint32_t)Wp));
        uint32_t* co = curx + ((ch * nb + b) * (N / 2) + j) * N + 2 * m;
        co[0] = (a0 & 0xffffu) | (a1 << 16);
        co[1] = (a0 >> 16) | (a1 & 0xffff0000u);
      }
  };

  // Items: (block b, group g of KX candidate columns from the block's first
  // in-picture column, candidate row r), r fastest so that neighbouring
  // lanes read pair rows a pitch apart and share the current block.
  // SP: the candidates of the union of the block's and its cells' ranges
  constexpr int ext = SP ? N / 2 : 0;
  const int y0b = by * N;
  const int rlo = max(0, R - y0b - ext);
  const int nr = min(s.span - 1, Hp - N + ext - y0b + R) - rlo + 1;
  int items = 0;
  for (int b = 0; b < nbv; b++) {
    const int x0 = (bx0 + b) * N;
    const int clo = max(0, R - x0 - ext), chi = min(s.span - 1, Wp - N + ext - x0 + R);
    items += nr * ((chi - clo + KX) / KX);
  }
  const int keyshift_sad = R <= 32 ? 21 : 23;
  const int keyshift_l1 = R <= 32 ? 13 : 15;
  const float inv_nr = 1.0f / (float)nr;

  // (b, r, c0, chi) of item it.  The items of a wave are consecutive: the
  // block of its first item is found with wave-uniform (scalar) arithmetic,
  // then each lane steps on from there, rarely more than once.
  auto decode = [&](int it, int& b, int& r, int& c0, int& chi) XV_INLINE {
    const int it0 = __builtin_amdgcn_readfirstlane(it);
    int start = 0, clo, n;
    b = 0;
    for (;; b++) {
      const int x0 = (bx0 + b) * N;
      clo = max(0, R - x0 - ext);
      chi = min(s.span - 1, Wp - N + ext - x0 + R);
      n = nr * ((chi - clo + KX) / KX);
      if (it0 < start + n || b + 1 >= nbv) break;
      start += n;
    }
    int rem = it - start;
    while (rem >= n && b + 1 < nbv) {
      rem -= n;
      b++;
      const int x0 = (bx0 + b) * N;
      clo = max(0, R - x0 - ext);
      chi = min(s.span - 1, Wp - N + ext - x0 + R);
      n = nr * ((chi - clo + KX) / KX);
    }
    // rem / nr in binary32: rem + 1/2 and nr are exact, the quotient is
    // below 2R + 2 <= 130 with a relative error of a few 2^-24, and its
    // distance from an integer is at least 1/(2 nr) >= 1/258
    const int g = (int)(((float)rem + 0.5f) * inv_nr);
    r = rlo + rem - g * nr;
    c0 = clo + g * KX;
  };

  // acc[k] += SAD of candidate (r, c0 + k) of block b over the channel in
  // LDS slot sl.  A pair row is taken in chunks of CW columns, which bounds
  // the registers of N = 32.
  auto accumulate = [&](int sl, int b, int r, int c0, uint32_t(&acc)[KX]) XV_INLINE {
    constexpr int CW = N < 16 ? N : 16;  // columns per chunk
    constexpr int NQ = KX + CW - 1;      // window dwords per chunk
    const int xbase = (sl * s.xr + r) * s.pitch + b * N + c0;
    const u32x4_l* cp = (const u32x4_l*)(curx + (sl * nb + b) * (N / 2) * N);
#pragma unroll kRpUnroll<N>
    for (int j = 0; j < N / 2; j++) {
#pragma unroll
      for (int cc = 0; cc < N / CW; cc++) {
        uint32_t P[NQ], C[CW];
        // One base per pair row and immediate offsets for its dwords; the
        // empty asm keeps the compiler from strength-reducing every load
        // address into an induction variable of its own.
        int xo = xbase + 2 * j * s.pitch;
        asm volatile("" : "+v"(xo));
#pragma unroll
        for (int q = 0; q < NQ; q++) P[q] = X[xo + cc * CW + q];
#pragma unroll
        for (int q = 0; q < CW / 4; q++) {
          const u32x4_l c4 = cp[j * (N / 4) + cc * (CW / 4) + q];
          C[4 * q] = c4.x;
          C[4 * q + 1] = c4.y;
          C[4 * q + 2] = c4.z;
          C[4 * q + 3] = c4.w;
        }
#pragma unroll
        for (int k = 0; k < KX; k++)
#pragma unroll
          for (int x = 0; x < CW; x++) acc[k] = __builtin_amdgcn_sad_u16(P[k + x], C[x], acc[k]);
        // keep the next chunk's loads after these sums: hoisting them costs
        // registers, hence waves, and other waves hide the LDS latency
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };

  // The item's candidates share row r and are visited in increasing dx, so
  // a strict < over (SAD << 8 | L1) keeps the lexicographic minimum of
  // (SAD, L1, dy, dx) among them; its full key goes to the block's LDS min.
  auto select = [&](int b, int r, int c0, int chi, const uint32_t(&acc)[KX]) XV_INLINE {
    const int khi = chi - c0;
    if constexpr (N <= 8) {
      if (R <= 32) {
        // One 32-bit key SAD << 11 | L1 << 4 | k holds the whole order
        // (SAD < 3 N^2 2^12 <= 2^20, L1 <= 64, k < 16), so a plain min picks
        // the candidate; 16 L1 + k comes from one 16-bit SAD of operands
        // scaled by 16.
        const uint32_t cx16 = 16u * (uint32_t)(c0 + KX);
        const uint32_t ly16 = 16u * (uint32_t)abs(r - R);
        uint32_t kb = 0xffffffffu;
#pragma unroll
        for (int k = 0; k < KX; k++) {
          const uint32_t lk = __builtin_amdgcn_sad_u16(cx16, 16u * (uint32_t)(R + KX - k), ly16 + k);
          const uint32_t key = (acc[k] << 11) | lk;
          kb = k <= khi ? min(kb, key) : kb;
        }
        if (kb != 0xffffffffu) {
          const int k = (int)(kb & 15u);
          const unsigned long long idx = (unsigned long long)(r * s.span + c0 + k);
          const unsigned long long key = ((unsigned long long)(kb >> 11) << keyshift_sad) |
                                         ((unsigned long long)((kb >> 4) & 127u) << keyshift_l1) | idx;
          atomicMin(&best[b], key);
        }
        return;
      }
    }
    const uint32_t ly = (uint32_t)abs(r - R);
    uint32_t kb32 = 0xffffffffu;
    int bsel = -1;
    const uint32_t cx = (uint32_t)(c0 + KX);  // below 2^16, as is R + KX - k
#pragma unroll
    for (int k = 0; k < KX; k++) {
      // L1 = |c0 + k - R| + |r - R|, the first term as the 16-bit absolute
      // difference of c0 + KX and R + KX - k
      const uint32_t l1 = __builtin_amdgcn_sad_u16(cx, (uint32_t)(R + KX - k), ly);
      const uint32_t key = (acc[k] << 8) | l1;
      const bool take = k <= khi && key < kb32;
      kb32 = take ? key : kb32;
      bsel = take ? k : bsel;
    }
    if (bsel >= 0) {
      const unsigned long long idx = (unsigned long long)(r * s.span + c0 + bsel);
      const unsigned long long key = ((unsigned long long)(kb32 >> 8) << keyshift_sad) |
                                     ((unsigned long long)(kb32 & 0xffu) << keyshift_l1) | idx;
      atomicMin(&best[b], key);
    }
  };

  // SP: acc[q][k] += SAD of candidate (r, c0 + k) over cell q (2 * (lower
  // half) + right half) of block b, channel in LDS slot sl.
  auto accumulate4 = [&](int sl, int b, int r, int c0, uint32_t(&acc)[4][KX]) XV_INLINE {
    constexpr int CW = N < 16 ? N : 16;  // columns per chunk
    constexpr int NQ = KX + CW - 1;      // window dwords per chunk
    const int xbase = (sl * s.xr + r) * s.pitch + b * N + c0;
    const u32x4_l* cp = (const u32x4_l*)(curx + (sl * nb + b) * (N / 2) * N);
#pragma unroll
    for (int hy = 0; hy < 2; hy++) {
#pragma unroll kRpUnrollHalf<N>
      for (int jj = 0; jj < N / 4; jj++) {
        const int j = hy * (N / 4) + jj;
#pragma unroll
        for (int cc = 0; cc < N / CW; cc++) {
          uint32_t P[NQ], C[CW];
          int xo = xbase + 2 * j * s.pitch;
          asm volatile("" : "+v"(xo));
#pragma unroll
          for (int q = 0; q < NQ; q++) P[q] = X[xo + cc * CW + q];
#pragma unroll
          for (int q = 0; q < CW / 4; q++) {
            const u32x4_l c4 = cp[j * (N / 4) + cc * (CW / 4) + q];
            C[4 * q] = c4.x;
            C[4 * q + 1] = c4.y;
            C[4 * q + 2] = c4.z;
            C[4 * q + 3] = c4.w;
          }
#pragma unroll
          for (int k = 0; k < KX; k++)
#pragma unroll
            for (int x = 0; x < CW; x++) {
              const int qd = 2 * hy + ((cc * CW + x) >= N / 2 ? 1 : 0);
              acc[qd][k] = __builtin_amdgcn_sad_u16(P[k + x], C[x], acc[qd][k]);
            }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
  };

  // SP: the five targets' minima over the item's candidates.  Target t = 0
  // is the block (the sum of the four cells), t = 1 + q cell q; a candidate
  // counts for a target only if it keeps the target inside the picture.
  auto select5 = [&](int b, int r, int c0, const uint32_t(&acc)[4][KX]) XV_INLINE {
    constexpr int h = N / 2;
    const int x0 = (bx0 + b) * N;
    const uint32_t ly = (uint32_t)abs(r - R);
    const uint32_t cx = (uint32_t)(c0 + KX);
    int clo[5], chi[5];
    bool rok[5];
#pragma unroll
    for (int t = 0; t < 5; t++) {
      const int n = t == 0 ? N : h;
      const int xs = x0 + (t == 0 ? 0 : ((t - 1) & 1) * h);
      const int ys = y0b + (t == 0 ? 0 : ((t - 1) >> 1) * h);
      clo[t] = max(0, R - xs) - c0;
      chi[t] = min(s.span - 1, Wp - n - xs + R) - c0;
      rok[t] = r >= R - ys && r <= Hp - n - ys + R;
    }
    uint32_t kb[5];
    int bsel[5];
#pragma unroll
    for (int t = 0; t < 5; t++) {
      kb[t] = 0xffffffffu;
      bsel[t] = -1;
    }
#pragma unroll
    for (int k = 0; k < KX; k++) {
      const uint32_t l1 = __builtin_amdgcn_sad_u16(cx, (uint32_t)(R + KX - k), ly);
#pragma unroll
      for (int t = 0; t < 5; t++) {
        const uint32_t sad = t == 0 ? acc[0][k] + acc[1][k] + acc[2][k] + acc[3][k] : acc[t - 1][k];
        const uint32_t key = (sad << 8) | l1;
        const bool take = rok[t] && k >= clo[t] && k <= chi[t] && key < kb[t];
        kb[t] = take ? key : kb[t];
        bsel[t] = take ? k : bsel[t];
      }
    }
#pragma unroll
    for (int t = 0; t < 5; t++)
      if (bsel[t] >= 0) {
        const unsigned long long idx = (unsigned long long)(r * s.span + c0 + bsel[t]);
        const unsigned long long key = ((unsigned long long)(kb[t] >> 8) << keyshift_sad) |
                                       ((unsigned long long)(kb[t] & 0xffu) << keyshift_l1) | idx;
        atomicMin(&best[b * 5 + t], key);
      }
  };

  for (int b = threadIdx.x; b < nb * KEYS; b += blockDim.x) best[b] = ~0ull;
  if constexpr (SP) {
    if constexpr (RND == 0) {
      stage(0, nch);
      __syncthreads();
      for (int it = threadIdx.x; it < items; it += blockDim.x) {
        int b, r, c0, chi;
        decode(it, b, r, c0, chi);
        uint32_t acc[4][KX];
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
          for (int k = 0; k < KX; k++) acc[q][k] = 0;
        for (int ch = 0; ch < nch; ch++) accumulate4(ch, b, r, c0, acc);
        select5(b, r, c0, acc);
      }
    } else {
      int ib[RND], ir[RND], ic[RND], ih[RND];
      uint32_t acc[RND][4][KX];
#pragma unroll
      for (int u = 0; u < RND; u++) {
        const int it = threadIdx.x + u * blockDim.x;
        if (it < items) decode(it, ib[u], ir[u], ic[u], ih[u]);
#pragma unroll
        for (int q = 0; q < 4; q++)
#pragma unroll
          for (int k = 0; k < KX; k++) acc[u][q][k] = 0;
      }
      for (int ch = 0; ch < nch; ch++) {
        if (ch > 0) __syncthreads();  // every read of the previous channel done
        stage(ch, 1);
        __syncthreads();
#pragma unroll
        for (int u = 0; u < RND; u++)
          if (threadIdx.x + u * blockDim.x < items) accumulate4(0, ib[u], ir[u], ic[u], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < RND; u++)
        if (threadIdx.x + u * blockDim.x < items) select5(ib[u], ir[u], ic[u], acc[u]);
    }
    __syncthreads();
    const int Wu = 2 * Wb;
    for (int i = threadIdx.x; i < nbv * 5; i += blockDim.x) {
      const int b = i / 5, t = i - (i / 5) * 5;
      const unsigned long long key = best[i];
      const int idx = (int)(key & ((1ull << keyshift_l1) - 1));
      const int dy = idx / s.span - R, dx = idx - (idx / s.span) * s.span - R;
      const uint32_t sad = (uint32_t)(key >> keyshift_sad);
      if (t == 0) {
        const size_t ci = (size_t)by * Wb + bx0 + b;
        job.mv_whole[2 * ci] = (int8_t)dx;
        job.mv_whole[2 * ci + 1] = (int8_t)dy;
        job.sad_whole[ci] = sad;
      } else {
        const int sx = (t - 1) & 1, sy = (t - 1) >> 1;
        const size_t u = (size_t)(2 * by + sy) * Wu + 2 * (bx0 + b) + sx;
        job.mv[2 * u] = (int8_t)dx;
        job.mv[2 * u + 1] = (int8_t)dy;
        job.sad[u] = sad;
      }
    }
    return;
  }
  if constexpr (RND == 0) {
    stage(0, nch);
    __syncthreads();
    for (int it = threadIdx.x; it < items; it += blockDim.x) {
      int b, r, c0, chi;
      decode(it, b, r, c0, chi);
      uint32_t acc[KX];
#pragma unroll
      for (int k = 0; k < KX; k++) acc[k] = 0;
      for (int ch = 0; ch < nch; ch++) accumulate(ch, b, r, c0, acc);
      select(b, r, c0, chi, acc);
    }
  } else {
    // the host admits a geometry only if every workgroup's items fit in RND
    // rounds of its threads
    int ib[RND], ir[RND], ic[RND], ih[RND];
    uint32_t acc[RND][KX];
#pragma unroll
    for (int u = 0; u < RND; u++) {
      const int it = threadIdx.x + u * blockDim.x;
      if (it < items) decode(it, ib[u], ir[u], ic[u], ih[u]);
#pragma unroll
      for (int k = 0; k < KX; k++) acc[u][k] = 0;
    }
    for (int ch = 0; ch < nch; ch++) {
      if (ch > 0) __syncthreads();  // every read of the previous channel done
      stage(ch, 1);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < RND; u++)
        if (threadIdx.x + u * blockDim.x < items) accumulate(0, ib[u], ir[u], ic[u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < RND; u++)
      if (threadIdx.x + u * blockDim.x < items) select(ib[u], ir[u], ic[u], ih[u], acc[u]);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbv; b += blockDim.x) {
    const unsigned long long key = best[b];
    const int idx = (int)(key & ((1ull << keyshift_l1) - 1));
    const int dy = idx / s.span - R, dx = idx - (idx / s.span) * s.span - R;
    int8_t* mv = job.mv + ((size_t)by * Wb + bx0 + b) * 2;
    mv[0] = (int8_t)dx;
    mv[1] = (int8_t)dy;
    if (job.sad) job.sad[(size_t)by * Wb + bx0 + b] = (uint32_t)(key >> keyshift_sad);
  }
}

template <int N, int KX, int ROWS>
hipError_t launch_me_t(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  const MeShape sh = me_shape(N, R, KX, g.nb, ROWS);
  const size_t lds = me_lds_bytes(N, sh, g.nb);
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)me_kernel<N, KX, ROWS>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  me_kernel<N, KX, ROWS><<<r.tiles, g.threads, lds, s>>>(r, R, g.nb);
  return hipGetLastError();
}

// Calls f.template operator()<KX, ROWS>() for the geometry's instance.
// Rows 1..3 exist for every even KX in 2..18; 5 rows (which divide the
// span 2R+1 = 65 of R = 32) for KX = 2 and 4.
template <class F>
auto me_dispatch(const MeGeom& g, F&& f) -> decltype(f.template operator()<2, 1>()) {
  using Ret = decltype(f.template operator()<2, 1>());
#define XV_ME_KX(kx)                                                               \
  case kx:                                                                         \
    return g.rows == 3   ? f.template operator()<kx, 3>()                          \
           : g.rows == 2 ? f.template operator()<kx, 2>()                          \
                         : f.template operator()<kx, 1>();
  if (g.rows == 5) {
    if (g.kx == 2) return f.template operator()<2, 5>();
    if (g.kx == 4) return f.template operator()<4, 5>();
    return (Ret)hipErrorInvalidValue;
  }
  switch (g.kx) {
    XV_ME_KX(2)
    XV_ME_KX(4)
    XV_ME_KX(6)
    XV_ME_KX(8)
    XV_ME_KX(10)
    XV_ME_KX(12)
    XV_ME_KX(14)
    XV_ME_KX(16)
    XV_ME_KX(18)
    default: return (Ret)hipErrorInvalidValue;
  }
#undef XV_ME_KX
}

template <int N, int KX, int RND>
hipError_t launch_me_rp_t(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  const size_t lds = rp_lds_layout(N, rp_shape(N, R, KX, g.nb), g.nb, RND == 0 ? 3 : 1).bytes;
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)me_rp_kernel<N, KX, RND>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  me_rp_kernel<N, KX, RND><<<r.tiles, g.threads, lds, s>>>(r, R, g.nb);
  return hipGetLastError();
}

// The combined whole-and-cells search (SP = 1) exists for KX = 5, 7, 11 and
// 13 in both row-pair layouts; staged by channel, a thread keeps
// kSplitRounds(KX) items (four sums per candidate each).
constexpr int kSplitRounds(int kx) { return kx >= 11 ? 1 : 2; }

template <int N, int KX, int RND>
hipError_t launch_me_rp_split_t(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  const size_t lds = rp_lds_layout(N, rp_shape(N, R, KX, g.nb), g.nb, RND == 0 ? 3 : 1, 5).bytes;
  static bool attr_set = false;
  if (!attr_set && lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)me_rp_kernel<N, KX, RND, 1>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  me_rp_kernel<N, KX, RND, 1><<<r.tiles, g.threads, lds, s>>>(r, R, g.nb);
  return hipGetLastError();
}

// Calls f.template operator()<KX, RND>() for the combined search's instance
// of g.
template <class F>
auto split_dispatch(const MeGeom& g, F&& f) -> decltype(f.template operator()<5, 0>()) {
  using Ret = decltype(f.template operator()<5, 0>());
  const bool byc = g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL;
  switch (g.kx) {
#define XV_SPLIT_KX(kx) \
  case kx:              \
    return byc ? f.template operator()<kx, kSplitRounds(kx)>() : f.template operator()<kx, 0>();
    XV_SPLIT_KX(5)
    XV_SPLIT_KX(7)
    XV_SPLIT_KX(11)
    XV_SPLIT_KX(13)
#undef XV_SPLIT_KX
    default: return (Ret)hipErrorInvalidValue;
  }
}

template <int N>
int me_split_vgprs_n(const MeGeom& g) {
  hipFuncAttributes a{};
  const hipError_t e = split_dispatch(g, [&]<int KX, int RND>() {
    return hipFuncGetAttributes(&a, (const void*)me_rp_kernel<N, KX, RND, 1>);
  });
  return (e == hipSuccess && a.numRegs > 0) ? a.numRegs : 128;
}

// Calls f.template operator()<KX>() for the row-pair instance of g.kx.
template <class F>
auto rp_dispatch(const MeGeom& g, F&& f) -> decltype(f.template operator()<2>()) {
  using Ret = decltype(f.template operator()<2>());
  switch (g.kx) {
    case 2: return f.template operator()<2>();
    case 3: return f.template operator()<3>();
    case 4: return f.template operator()<4>();
    case 5: return f.template operator()<5>();
    case 6: return f.template operator()<6>();
    case 7: return f.template operator()<7>();
    case 8: return f.template operator()<8>();
    case 9: return f.template operator()<9>();
    case 11: return f.template operator()<11>();
    case 13: return f.template operator()<13>();
    default: return (Ret)hipErrorInvalidValue;
  }
}

template <int N>
hipError_t launch_me_n(int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  if (g.layout == XV_ME_ROW_PAIRS)
    return rp_dispatch(g, [&]<int KX>() { return launch_me_rp_t<N, KX, 0>(R, g, r, s); });
  if (g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL)
    return rp_dispatch(g, [&]<int KX>() { return launch_me_rp_t<N, KX, kRpRounds>(R, g, r, s); });
  if (g.kx < 2 || g.kx > 18 || (g.kx & 1)) return hipErrorInvalidValue;
  return me_dispatch(g, [&]<int KX, int ROWS>() { return launch_me_t<N, KX, ROWS>(R, g, r, s); });
}

// VGPRs per lane of the motion-search kernel instance for (N, KX, rows).
template <int N>
int me_vgprs_n(const MeGeom& g) {
  hipFuncAttributes a{};
  const hipError_t e =
      g.layout == XV_ME_ROW_PAIRS
          ? rp_dispatch(g, [&]<int KX>() {
              return hipFuncGetAttributes(&a, (const void*)me_rp_kernel<N, KX, 0>);
            })
      : g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL
          ? rp_dispatch(g, [&]<int KX>() {
              return hipFuncGetAttributes(&a, (const void*)me_rp_kernel<N, KX, kRpRounds>);
            })
          : me_dispatch(g, [&]<int KX, int ROWS>() {
              return hipFuncGetAttributes(&a, (const void*)me_kernel<N, KX, ROWS>);
            });
  return (e == hipSuccess && a.numRegs > 0) ? a.numRegs : 128;
}

int me_vgprs(int N, const MeGeom& g) {
  switch (N) {
    case 4: return me_vgprs_n<4>(g);
    case 8: return me_vgprs_n<8>(g);
    case 16: return me_vgprs_n<16>(g);
    default: return me_vgprs_n<32>(g);
  }
}

}  // namespace

// Whether a kernel instance exists for the geometry's layout, KX and rows.
bool me_instance_exists(const MeGeom& g) {
  if (g.layout == XV_ME_ROW_PAIRS || g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL)
    return g.rows == 1 && ((g.kx >= 2 && g.kx <= 9) || g.kx == 11 || g.kx == 13);
  if (g.layout != XV_ME_COLUMN_PAIRS) return false;
  if (g.kx < 2 || g.kx > 18 || (g.kx & 1)) return false;
  if (g.rows >= 1 && g.rows <= 3) return true;
  return g.rows == 5 && (g.kx == 2 || g.kx == 4);
}

size_t me_lds_bytes_for(int N, int R, const MeGeom& g) {
  if (g.layout == XV_ME_ROW_PAIRS)
    return rp_lds_layout(N, rp_shape(N, R, g.kx, g.nb), g.nb, 3).bytes;
  if (g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL)
    return rp_lds_layout(N, rp_shape(N, R, g.kx, g.nb), g.nb, 1).bytes;
  return me_lds_bytes(N, me_shape(N, R, g.kx, g.nb, g.rows), g.nb);
}

// Whether the geometry can run (N, R): its LDS fits a CU, and with the
// channels staged one after another every workgroup's items (at most nb
// blocks x 2R+1 rows x ceil((2R+1)/KX) column groups) fit in the rounds a
// thread holds.
bool me_geometry_fits(int N, int R, const MeGeom& g) {
  if (me_lds_bytes_for(N, R, g) > 160 * 1024) return false;
  if (g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL) {
    const long span = 2L * R + 1, groups = (span + g.kx - 1) / g.kx;
    if ((long)g.nb * span * groups > (long)kRpRounds * g.threads) return false;
  }
  return true;
}

// Model of a CU (160 KB LDS, 4 SIMDs with 512 VGPRs per lane, at most 8
// waves each) used to rank geometries.  Score = share of SAD instructions in
// a lane's VALU work x share of useful candidates x lane occupancy of the
// waves that hold items x resident waves per SIMD (saturating at 3).  Per item
// and channel, column pairs: rows N KX N/2 SADs against N + rows - 1 window
// rows of (KX+N)/2 - 1 realignments; row pairs: N/2 KX N SADs and N/2
// address updates.  Per item, about 40 + 6 x candidates instructions select
// the best candidate.  Useful candidates: 2R+1 of G KX columns, and for
// column pairs 2R+1 of rows * ceil((2R+1)/rows) rows.
namespace {

// The model for an instance with vgpr registers per lane, lds bytes per
// workgroup and sel instructions of selection per item and channel.
double model_score(int N, int R, const MeGeom& g, int width_blocks, int vgpr, size_t lds,
                   double sel) {
  const int span = 2 * R + 1;
  const int kx = g.kx, th = g.threads;
  const int G = (span + kx - 1) / kx;
  const bool rp = g.layout == XV_ME_ROW_PAIRS || g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL;
  double eff;
  int ipb;
  if (rp) {
    const double sad = (double)(N / 2) * kx * N;
    eff = sad / (sad + N / 2 + sel) * (double)span / (double)(G * kx);
    ipb = span * G;
  } else {
    const double sad = (double)g.rows * N * kx * N / 2;
    const double perm = (double)(N + g.rows - 1) * ((kx + N) / 2 - 1);
    const int dyp = (span + g.rows - 1) / g.rows;
    eff = sad / (sad + perm + sel) * (double)span / (double)(G * kx) * (double)span /
          (double)(g.rows * dyp);
    ipb = dyp * G;
  }
  // lane occupancy over the runs of a block row (full runs of nb blocks and
  // a last run of the remaining ones): a wave with no item left exits, so
  // only the idle lanes of the last busy wave of a run are lost
  const int wbk = std::max(1, width_blocks);
  const int runs = (wbk + g.nb - 1) / g.nb;
  double busy = 0.0, slots = 0.0;
  for (int r = 0; r < runs; r++) {
    const int items = std::min(g.nb, wbk - r * g.nb) * ipb;
    busy += items;
    slots += (double)((items + 63) / 64) * 64;
  }
  const double lane = busy / slots;
  const int wpg = th / 64;
  const int waves_by_vgpr = std::max(1, std::min(8, 512 / std::max(1, vgpr)));
  const int wg_lds = (int)((160 * 1024) / std::max<size_t>(1, lds));
  const int wg_waves = (4 * waves_by_vgpr) / wpg;
  const int wg = std::max(0, std::min(wg_lds, wg_waves));
  if (wg == 0) return -1.0;
  const double occ = std::min(3.0, (double)(wg * wpg) / 4.0);
  return eff * lane * occ;
}

}  // namespace

double me_model_score(int N, int R, const MeGeom& g, int width_blocks) {
  if (!me_geometry_fits(N, R, g)) return -1.0;
  return model_score(N, R, g, width_blocks, me_vgprs(N, g), me_lds_bytes_for(N, R, g),
                     (40.0 + 6.0 * g.kx * g.rows) / 3.0);  // per channel of a 3-channel group
}

std::vector<MeGeom> me_candidates(int N, int R, int width_blocks) {
  std::vector<MeGeom> v;
  const int cmax = std::max(1, std::min(16, width_blocks));
  auto add = [&](const MeGeom& g) {
    if (me_instance_exists(g) && me_geometry_fits(N, R, g) && me_lds_bytes_for(N, R, g) <= 96 * 1024)
      v.push_back(g);
  };
  for (int rows : {1, 2, 3, 5})
    for (int kx = 2; kx <= 18; kx += 2)
      for (int c = 1; c <= cmax; c++)
        for (int th = 64; th <= 512; th += 64) add(MeGeom{c, kx, th, rows, XV_ME_COLUMN_PAIRS});
  for (int lay : {XV_ME_ROW_PAIRS, XV_ME_ROW_PAIRS_BY_CHANNEL})
    for (int kx : {2, 3, 4, 5, 6, 7, 8, 9, 11, 13})
      for (int c = 1; c <= cmax; c++)
        for (int th = 64; th <= 512; th += 64) add(MeGeom{c, kx, th, 1, lay});
  return v;
}

// Default geometry: the best model score (ties: more blocks per workgroup).
MeGeom me_default_geometry(int N, int R, int max_nb) {
  MeGeom best{1, 2, 256, 1, XV_ME_COLUMN_PAIRS};
  double bs = -2.0;
  for (const MeGeom& g : me_candidates(N, R, max_nb)) {
    const double sc = me_model_score(N, R, g, max_nb);
    if (sc > bs + 1e-9 || (sc > bs - 1e-9 && g.nb > best.nb)) {
      bs = sc;
      best = g;
    }
  }
  return best;
}

// ---- adaptive block size: whole or split ---------------------------------
// One thread per block of a P step: J = 16 SAD + lambda16 bits for the whole
// block (size-N search) and summed over its four N/2 cells (size-N/2
// search, z-order), bits = Exp-Golomb lengths of each vector against zero;
// split iff the cells cost less.  Whole blocks repeat their vector over
// their cells, so the cell grid then holds every block's final vectors.
namespace {

constexpr int kDecideThreads = 256;

__device__ inline uint32_t se_len(int v) {
  return v ? 65u - 2u * (uint32_t)__builtin_clz((uint32_t)abs(v)) : 1u;
}

__global__ void __launch_bounds__(kDecideThreads) split_decide_kernel(const LaunchDesc d, int N) {
  int tl;
  const FrameJob* jp = desc_job(d, (int)blockIdx.x, tl);
  const int Hb = jp->Hp / N, Wb = jp->Wp / N;
  const int ci = tl * kDecideThreads + (int)threadIdx.x;
  if (ci >= Hb * Wb) return;
  const int by = ci / Wb, bx = ci - by * Wb;
  const int Wu = 2 * Wb;
  int8_t* mv = jp->mv;
  const uint64_t lam = (uint32_t)jp->lambda16;
  const int vx = jp->mv_whole[2 * ci], vy = jp->mv_whole[2 * ci + 1];
  const uint64_t jw = 16ull * jp->sad_whole[ci] + lam * (se_len(vx) + se_len(vy));
  uint64_t js = 0;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int u = (2 * by + (i >> 1)) * Wu + 2 * bx + (i & 1);
    js += 16ull * jp->sad[u] + lam * (se_len(mv[2 * u]) + se_len(mv[2 * u + 1]));
  }
  const bool split = js < jw;
  jp->split[ci] = split ? 1 : 0;
  if (!split) {
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int u = (2 * by + (i >> 1)) * Wu + 2 * bx + (i & 1);
      mv[2 * u] = (int8_t)vx;
      mv[2 * u + 1] = (int8_t)vy;
    }
  }
}

}  // namespace

int split_tiles_per_job(int Hb, int Wb) { return (Hb * Wb + kDecideThreads - 1) / kDecideThreads; }

hipError_t launch_split_decide(int N, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  split_decide_kernel<<<r.tiles, kDecideThreads, 0, s>>>(r, N);
  return hipGetLastError();
}

// ---- the combined search's geometry ------------------------------------------
bool me_split_instance_exists(int N, const MeGeom& g) {
  return (N == 8 || N == 16 || N == 32) && g.rows == 1 &&
         (g.layout == XV_ME_ROW_PAIRS || g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL) &&
         (g.kx == 5 || g.kx == 7 || g.kx == 11 || g.kx == 13);
}

size_t me_split_lds_bytes(int N, int R, const MeGeom& g) {
  return rp_lds_layout(N, rp_shape(N, R, g.kx, g.nb), g.nb,
                       g.layout == XV_ME_ROW_PAIRS ? 3 : 1, 5).bytes;
}

int me_split_rounds(const MeGeom& g) {
  return g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL ? kSplitRounds(g.kx) : 0;
}

bool me_split_fits(int N, int R, const MeGeom& g) {
  if (!me_split_instance_exists(N, g) || g.nb < 1 || g.threads < 64 || g.threads > 512 ||
      (g.threads & 63))
    return false;
  if (me_split_lds_bytes(N, R, g) > 160 * 1024) return false;
  if (g.layout == XV_ME_ROW_PAIRS_BY_CHANNEL) {
    const long span = 2L * R + 1, groups = (span + g.kx - 1) / g.kx;
    if ((long)g.nb * span * groups > (long)me_split_rounds(g) * g.threads) return false;
  }
  return true;
}

// Model score of a combined-search geometry: the plain search's model with
// this instance's registers and LDS and a selection over five targets.
double me_split_model_score(int N, int R, const MeGeom& g, int width_blocks) {
  if (!me_split_fits(N, R, g)) return -1.0;
  int vgpr = 128;
  switch (N) {
    case 8: vgpr = me_split_vgprs_n<8>(g); break;
    case 16: vgpr = me_split_vgprs_n<16>(g); break;
    default: vgpr = me_split_vgprs_n<32>(g); break;
  }
  return model_score(N, R, g, width_blocks, vgpr, me_split_lds_bytes(N, R, g),
                     (40.0 + 5 * 6.0 * g.kx) / 3.0);
}

std::vector<MeGeom> me_split_candidates(int N, int R, int width_blocks) {
  std::vector<MeGeom> v;
  const int cmax = std::max(1, std::min(16, width_blocks));
  for (int lay : {XV_ME_ROW_PAIRS, XV_ME_ROW_PAIRS_BY_CHANNEL})
    for (int kx : {5, 7, 11, 13})
      for (int c = 1; c <= cmax; c++)
        for (int th = 64; th <= 512; th += 64) {
          const MeGeom g{c, kx, th, 1, lay};
          if (me_split_fits(N, R, g) && me_split_lds_bytes(N, R, g) <= 96 * 1024) v.push_back(g);
        }
  return v;
}

MeGeom me_split_default_geometry(int N, int R, int width_blocks) {
  MeGeom best{1, 13, 384, 1, XV_ME_ROW_PAIRS_BY_CHANNEL};
  double bs = -2.0;
  for (const MeGeom& g : me_split_candidates(N, R, width_blocks)) {
    const double sc = me_split_model_score(N, R, g, width_blocks);
    if (sc > bs + 1e-9 || (sc > bs - 1e-9 && g.nb > best.nb)) {
      bs = sc;
      best = g;
    }
  }
  return best;
}

hipError_t launch_me_split(int N, int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  if (!me_split_fits(N, R, g)) return hipErrorInvalidValue;
  auto go = [&]<int NN>() {
    return split_dispatch(
        g, [&]<int KX, int RND>() { return launch_me_rp_split_t<NN, KX, RND>(R, g, r, s); });
  };
  switch (N) {
    case 8: return go.template operator()<8>();
    case 16: return go.template operator()<16>();
    case 32: return go.template operator()<32>();
    default: return hipErrorInvalidValue;
  }
}

int me_tiles_per_job(int Hb, int Wb, const MeGeom& g) {
  return Hb * ((Wb + g.nb - 1) / g.nb);
}

hipError_t launch_me(int N, int R, const MeGeom& g, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  if (g.threads <= 0 || g.threads > 512 || (g.threads & 63) || g.nb < 1 || !me_instance_exists(g))
    return hipErrorInvalidValue;
  if (!me_geometry_fits(N, R, g)) return hipErrorInvalidValue;
  switch (N) {
    case 4: return launch_me_n<4>(R, g, r, s);
    case 8: return launch_me_n<8>(R, g, r, s);
    case 16: return launch_me_n<16>(R, g, r, s);
    case 32: return launch_me_n<32>(R, g, r, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xv
