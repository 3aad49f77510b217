// k_xform.hip -- fused transform coding of one picture step (encode) and its
// reconstruction from stored levels (decode).
//
// Encode, per N x N block of each of the 3 channels of a band group:
//   prediction (I: the constant 2^(B-1); P: the reference reconstruction
//   displaced by the block's vector) -> residual -> forward H.265 integer
//   DCT (rows, shift log2N + B - 9; columns, shift log2N + 6) -> dead-zone
//   quantisation -> Exp-Golomb rate proxy of the levels in up-right diagonal
//   scan order -> dequantisation -> inverse DCT (columns, clip to 16 bits,
//   shift 7; rows, shift 20 - B) -> reconstruction clipped to [0, 2^B-1] ->
//   squared error over valid real samples.  The vector bits of each block
//   (signed Exp-Golomb of the difference to the left neighbour's vector) are
//   counted in the same pass.  The paper leaves the codec internals to x265;
//   these steps are the stated H.265-style reading of them.
//
// Mapping: a workgroup of 192 threads (3 waves) owns a 64-pixel-wide run of
// blocks (NBW = 64 / N blocks) in one block row and all 3 channels; wave c
// handles channel c.  Row stages give one thread one block row, column stages
// one block column; intermediate tiles stay in LDS, so HBM sees each sample
// read and written once: cur + prediction in, levels + reconstruction out.
//
// Arithmetic: every product is a v_dot2 of two 16-bit pairs with the matrix
// entries as instruction literals.  The forward row stage and both inverse
// stages use the even/odd (butterfly) factorisation of the H.265 matrices;
// the forward column stage, whose inputs may need the full 16 bits, stays a
// plain matrix product.  All sums are exact integers, so the factorised
// forms give the same results as the matrix products they replace.
#include <algorithm>
#include <utility>

#include "xv_internal.h"

namespace xv {

namespace {

// ---------------------------------------------------------------------------
// Compile-time loops: f(Ic<0>{}), ..., f(Ic<n-1>{}), so that loop indices are
// constant expressions (matrix entries become instruction literals).
// ---------------------------------------------------------------------------
template <int I>
using Ic = std::integral_constant<int, I>;

#define XV_INLINE __attribute__((always_inline))

template <class F, int... I>
__device__ inline XV_INLINE void unroll_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(Ic<I>{}), ...);
}
template <int n, class F>
__device__ inline XV_INLINE void unroll(F&& f) {
  unroll_impl(f, std::make_integer_sequence<int, n>{});
}

// Packed 16-bit pairs (lo = element 2j, hi = element 2j + 1).
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline s16x2 as_v(uint32_t x) { return __builtin_bit_cast(s16x2, x); }
__device__ inline uint32_t as_u(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ inline uint32_t swap_halves(uint32_t x) { return (x >> 16) | (x << 16); }
__device__ inline uint32_t padd(uint32_t a, uint32_t b) { return as_u(as_v(a) + as_v(b)); }
__device__ inline uint32_t psub(uint32_t a, uint32_t b) { return as_u(as_v(a) - as_v(b)); }
// Two int32 -> one pair, each saturated to [-32768, 32767].
__device__ inline uint32_t pack_sat(int lo, int hi) {
  return as_u(__builtin_amdgcn_cvt_pk_i16(lo, hi));
}

__host__ __device__ constexpr uint32_t cpair(int lo, int hi) {
  return ((uint32_t)lo & 0xffffu) | (((uint32_t)hi & 0xffffu) << 16);
}

// Coefficient pair (M_n[k0][m0], M_n[k1][m1]), formed at compile time.
template <int n, int k0, int m0, int k1, int m1>
constexpr uint32_t kPair = cpair(dct_coef(n, k0, m0), dct_coef(n, k1, m1));

// acc + lo(c) lo(x) + hi(c) hi(x), signed 16-bit halves, exact in int32.
__device__ inline int dot2(uint32_t c, uint32_t x, int acc) {
  return __builtin_amdgcn_sdot2(as_v(c), as_v(x), acc, false);
}

// The first product of a sum: the same operation in its three-operand form
// with the constant pair in a scalar register and the start value in a
// vector register (or zero), so that no vector move initialises the
// accumulator (the two-operand form accumulates into its destination).
template <uint32_t C>
__device__ inline int dot2_first(uint32_t x, int acc) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(r) : "s"(C), "v"(x), "v"(acc));
  return r;
}
template <uint32_t C>
__device__ inline int dot2_first0(uint32_t x) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "s"(C), "v"(x));
  return r;
}

template <int N>
struct Tile {
  static constexpr int NBW = 64 / N;    // blocks per workgroup along x
  static constexpr int P = N + 2;       // LDS pitch (int16) of a tile row (odd dword count)
  static constexpr int L2N = ilog2c(N);
  // register target of the encode kernel: 8 waves per SIMD where the
  // compiler fits that without spilling (N = 8, 16); N = 4 and 32 keep their
  // natural allocation
  static constexpr int kEncWaves = (N == 8 || N == 16) ? 8 : 1;
};

// ---------------------------------------------------------------------------
// Forward n-point transform of x (n/2 packed pairs): out[S k] = sum_m M_n[k][m]
// x[m] + rnd.  Odd outputs come from o[m] = x[m] - x[n-1-m] (M_n[k][n-1-m] =
// -M_n[k][m] for odd k), even ones are the n/2-point transform of e[m] = x[m]
// + x[n-1-m] (M_n[2k][m] = M_{n/2}[k][m]).  The pre-adds run on packed 16-bit
// pairs: for residuals |x| <= 4095 the sums stay within 8190, 16380 and
// 32760 after one, two and three levels, and the 4-point base takes a plain
// product, so no level overflows 16 bits for n <= 32.
// ---------------------------------------------------------------------------
template <int n, int S, class Out>
__device__ inline void fwd_part(const uint32_t (&xp)[n / 2], Out& out, int rnd) {
  if constexpr (n == 4) {
    unroll<4>([&](auto kk) XV_INLINE {
      constexpr int k = kk;
      int a = dot2_first<kPair<4, k, 0, k, 1>>(xp[0], rnd);
      a = dot2(kPair<4, k, 2, k, 3>, xp[1], a);
      out[S * k] = a;
    });
  } else {
    uint32_t ep[n / 4], op[n / 4];
    unroll<n / 4>([&](auto jj) XV_INLINE {
      constexpr int j = jj;
      // (x[n-1-2j], x[n-2-2j]) against (x[2j], x[2j+1])
      const uint32_t m = swap_halves(xp[n / 2 - 1 - j]);
      ep[j] = padd(xp[j], m);
      op[j] = psub(xp[j], m);
    });
    unroll<n / 2>([&](auto kk) XV_INLINE {
      constexpr int k = 2 * kk + 1;
      int a = dot2_first<kPair<n, k, 0, k, 1>>(op[0], rnd);
      unroll<n / 4 - 1>([&](auto jj) XV_INLINE {
        constexpr int j = jj + 1;
        a = dot2(kPair<n, k, 2 * j, k, 2 * j + 1>, op[j], a);
      });
      out[S * k] = a;
    });
    fwd_part<n / 2, 2 * S>(ep, out, rnd);
  }
}

// ---------------------------------------------------------------------------
// Inverse n-point transform: out[m] = sum_k M_n[k][m] y[k] + rnd, m < n, with
// y given as packed pairs in "inverse order": the odd entries (y1, y3), (y5,
// y7), ... first, then the even entries y0, y2, ... in the same order
// recursively, down to a 4-point part in natural order.  out[m] = E[m] +
// O[m] and out[n-1-m] = E[m] - O[m], E the inverse n/2-point transform of
// the even entries, O the odd entries against the odd rows.
// ---------------------------------------------------------------------------
template <int n>
__device__ inline void inv_part(const uint32_t* ip, int (&out)[n], int rnd) {
  if constexpr (n == 4) {
    unroll<4>([&](auto mm) XV_INLINE {
      constexpr int m = mm;
      int a = dot2_first<kPair<4, 0, m, 1, m>>(ip[0], rnd);
      a = dot2(kPair<4, 2, m, 3, m>, ip[1], a);
      out[m] = a;
    });
  } else {
    int E[n / 2];
    inv_part<n / 2>(ip + n / 4, E, rnd);
    unroll<n / 2>([&](auto mm) XV_INLINE {
      constexpr int m = mm;
      int o = dot2_first0<kPair<n, 1, m, 3, m>>(ip[0]);
      unroll<n / 4 - 1>([&](auto jj) XV_INLINE {
        constexpr int j = jj + 1;
        o = dot2(kPair<n, 4 * j + 1, m, 4 * j + 3, m>, ip[j], o);
      });
      out[m] = E[m] + o;
      out[n - 1 - m] = E[m] - o;
    });
  }
}

// Element of y held in slot s of the inverse order, and the slot of element k.
__host__ __device__ constexpr int inv_elem(int n, int s) {
  if (n == 4) return s;
  if (s < n / 2) return 2 * s + 1;
  return 2 * inv_elem(n / 2, s - n / 2);
}
template <int N>
__device__ inline int inv_slot(int k) {
  int slot = 0, kk = k;
#pragma unroll
  for (int n = N; n > 4; n >>= 1) {
    if (kk & 1) return slot + (kk >> 1);
    slot += n / 2;
    kk >>= 1;
  }
  return slot + kk;
}

// y[0..N-1] (int32, saturated to 16 bits) as pairs in inverse order.
template <int N>
__device__ inline void to_inverse_order(const int (&y)[N], uint32_t (&ip)[N / 2]) {
  unroll<N / 2>([&](auto ss) XV_INLINE {
    constexpr int s = ss;
    constexpr int e0 = inv_elem(N, 2 * s), e1 = inv_elem(N, 2 * s + 1);
    ip[s] = pack_sat(y[e0], y[e1]);
  });
}

// Forward column stage: out[l] = sum_y M[l][y] T[y] + rnd, T as N/2 pairs.
// Row-stage outputs may use all 16 bits, which the butterfly's packed
// pre-adds cannot take in general; but when every |T| of the wave's columns is
// at most 32767 >> (log2 N - 2), the sums of all its pre-add levels stay in
// 16 bits and the even/odd form gives the same sums with fewer products.  The
// choice is one vote per wave, so lanes never diverge on it.
// Column-stage accumulators as one vector value: the two forms of the stage
// then update it by element insertion, which stays in registers.
template <int N>
using ivec = int __attribute__((ext_vector_type(N)));

template <int N>
__device__ inline void fwd_product(const uint32_t (&t)[N / 2], ivec<N>& out, int rnd) {
  unroll<N>([&](auto ll) XV_INLINE {
    constexpr int l = ll;
    int a = dot2_first<kPair<N, l, 0, l, 1>>(t[0], rnd);
    unroll<N / 2 - 1>([&](auto jj) XV_INLINE {
      constexpr int j = jj + 1;
      a = dot2(kPair<N, l, 2 * j, l, 2 * j + 1>, t[j], a);
    });
    out[l] = a;
  });
}

template <int N>
__device__ inline void fwd_column(const uint32_t* tp, ivec<N>& out, int rnd) {
  uint32_t t[N / 2];
#pragma unroll
  for (int j = 0; j < N / 2; j++) t[j] = tp[j];
  bool fast = false;
  if constexpr (N >= 16) {
    constexpr short kLim = (short)(32767 >> (ilog2c(N) - 2));
    s16x2 mx = as_v(t[0]), mn = as_v(t[0]);
#pragma unroll
    for (int j = 1; j < N / 2; j++) {
      mx = __builtin_elementwise_max(mx, as_v(t[j]));
      mn = __builtin_elementwise_min(mn, as_v(t[j]));
    }
    fast = __all(max(mx.x, mx.y) <= kLim && min(mn.x, mn.y) >= -kLim);
  }
  if (fast)
    fwd_part<N, 1>(t, out, rnd);
  else
    fwd_product<N>(t, out, rnd);
}

// Ordering of the LDS accesses of one wave: every lane's earlier reads and
// writes happen before any lane's later ones.  The waves of a transform
// workgroup share no LDS data (each has its channel's tiles, sums and run
// table), so this is all the synchronisation they need.
// The scheduler keeps each stage's instructions on its side, as a workgroup
// barrier would (otherwise hoisted work raises the register count).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  __builtin_amdgcn_sched_barrier(0);
}

// LDS layout per workgroup, encode (int16):
//   TD [3][NBW][N][P]  forward row-stage output transposed ([k][y]); each
//                      column thread then overwrites its own row k with the
//                      column's levels ([k][l])
//   E  [3][NBW][N][P]  inverse column-stage output, row y, entries in
//                      inverse order
//   sums               per-workgroup squared error per channel, bits
template <int N>
struct alignas(16) LdsEnc {
  int16_t TD[3][Tile<N>::NBW][N][Tile<N>::P];
  int16_t E[3][Tile<N>::NBW][N][Tile<N>::P];
  unsigned long long sse[3];
  uint32_t cbits[3][Tile<N>::NBW];
  uint32_t mvbits;
  uint8_t runs[3][256];  // kRunTab, one copy per wave, for the rate proxy
};

// Decode works one channel per workgroup (the channels of a frame are
// independent there): the inverse column-stage output of that channel.
template <int N>
struct alignas(16) LdsDec {
  int16_t E[Tile<N>::NBW][N][Tile<N>::P];
};

// Up-right diagonal scan of an N x N block (ITU-T H.265 6.5.3): anti-
// diagonals d = x + y in order, each from its bottom-left end upwards.  The
// table maps scan position to the byte offset 2 (x * P + y) of the level in
// the transposed LDS tile.
template <int N>
struct alignas(16) ScanTab {
  uint32_t v[N * N];
};
template <int N>
constexpr ScanTab<N> make_scan_tab() {
  ScanTab<N> t{};
  for (int i = 0; i < N * N; i++) {
    const int y = i / N, x = i % N;
    const int d = x + y;
    const int before = d < N ? d * (d + 1) / 2 : N * N - (2 * N - 1 - d) * (2 * N - d) / 2;
    const int first_x = d < N ? 0 : d - N + 1;
    t.v[before + x - first_x] = (uint32_t)(2 * (x * Tile<N>::P + y));
  }
  return t;
}
template <int N>
constexpr ScanTab<N> kScanTab = make_scan_tab<N>();

// Run table of the rate proxy: for an 8-bit mask c of nonzero positions,
// the sum over its set bits b of floor(log2(b - a)), a the previous set bit
// (-1 for the first).
struct alignas(16) RunTab {
  uint8_t v[256];
};
constexpr RunTab make_run_tab() {
  RunTab t{};
  for (int c = 0; c < 256; c++) {
    int prev = -1, sum = 0;
    for (int b = 0; b < 8; b++)
      if ((c >> b) & 1) {
        int g = b - prev, l = 0;
        while (g >>= 1) l++;
        sum += l;
        prev = b;
      }
    t.v[c] = (uint8_t)sum;
  }
  return t;
}
constexpr RunTab kRunTab = make_run_tab();

struct TileCoord {
  const FrameJob* job;
  int tl, by, bx0, Hb, Wb;
};

template <int N>
__device__ inline bool locate_at(const LaunchDesc& jd, int tile, TileCoord& tc) {
  int tl;
  tc.job = desc_job(jd, tile, tl);
  tc.tl = tl;
  const FrameJob& job = *tc.job;
  tc.Hb = job.Hp / N;
  tc.Wb = job.Wp / N;
  const int runs = (tc.Wb + Tile<N>::NBW - 1) / Tile<N>::NBW;
  if (tl >= tc.Hb * runs) return false;
  tc.by = tl / runs;
  tc.bx0 = (tl - tc.by * runs) * Tile<N>::NBW;
  return true;
}

// XCD-aware order: workgroup IDs are dealt round-robin to the 8 XCDs, each
// with its own L2.  Mapping the IDs an XCD receives to one contiguous range
// of tiles keeps vertically and horizontally neighbouring tiles -- which read
// overlapping rows of the motion-compensated reference -- in the same L2.
__device__ inline int xcd_tile(int id, int n) {
  constexpr int kXcd = 8;
  const int x = id % kXcd, i = id / kXcd;
  const int per = n / kXcd, rem = n % kXcd;
  return x * per + min(x, rem) + i;
}

template <int N>
__device__ inline bool locate(const LaunchDesc& jd, TileCoord& tc) {
  return locate_at<N>(jd, xcd_tile((int)blockIdx.x, (int)gridDim.x), tc);
}

// Global memory through address space 1 at a 32-bit byte offset from a base
// pointer (global loads and stores with a scalar base; a padded frame stays
// below 2^31 bytes, which the host checks).
#define XV_G __attribute__((address_space(1)))
template <class T>
__device__ inline T gld(const void* base, uint32_t off) {
  return *(const XV_G T*)((const XV_G char*)base + off);
}
template <class T>
__device__ inline void gst(void* base, uint32_t off, T v) {
  *(XV_G T*)((XV_G char*)base + off) = v;
}

// N packed u16 (or i16) samples at base + off (16-byte aligned for N >= 8).
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

template <int N>
__device__ inline void load_row_packed(const void* base, uint32_t off, uint32_t (&v)[N / 2]) {
  if constexpr (N >= 8) {
#pragma unroll
    for (int q = 0; q < N / 8; q++) {
      const u32x4 w = gld<u32x4>(base, off + 16 * q);
      v[4 * q + 0] = w.x;
      v[4 * q + 1] = w.y;
      v[4 * q + 2] = w.z;
      v[4 * q + 3] = w.w;
    }
  } else {
    const u32x2 w = gld<u32x2>(base, off);
    v[0] = w.x;
    v[1] = w.y;
  }
}

template <int N>
__device__ inline void store_row_packed(void* base, uint32_t off, const uint32_t (&v)[N / 2]) {
  if constexpr (N >= 8) {
#pragma unroll
    for (int q = 0; q < N / 8; q++) {
      const u32x4 w = {v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
      gst<u32x4>(base, off + 16 * q, w);
    }
  } else {
    const u32x2 w = {v[0], v[1]};
    gst<u32x2>(base, off, w);
  }
}

// Prediction row as packed pairs: the step's prediction plane where it has
// one (quarter-sample P steps, intra-predicted I steps); else I -> 2^(B-1)
// and P -> the reference displaced by (dx, dy).  A coded vector keeps the
// displaced block inside the padded picture; the clamp only guarantees
// in-bounds reads for a corrupt vector.  The row is read as aligned dwords
// and shifted by one sample when the displaced column is odd; the extra
// dword is then in bounds (rx + N is odd and Wp even, so rx + N < Wp).
template <int N>
__device__ inline void pred_row(const FrameJob& job, int c, int r, int y, int x0, int dx, int dy,
                                uint32_t (&pp)[N / 2]) {
  if (job.intra && !job.pred) {
    const uint32_t h = 1u << (job.bit_depth - 1);
#pragma unroll
    for (int j = 0; j < N / 2; j++) pp[j] = h | (h << 16);
  } else {
    // a prediction plane is read at displacement zero
    const uint16_t* src = job.pred ? job.pred : job.ref;
    if (job.pred) dx = dy = 0;
    const int ry = min(max(y - r + dy, 0), job.Hp - N) + r;
    const int rx = min(max(x0 + dx, 0), job.Wp - N);
    const uint32_t off = 2u * ((uint32_t)(c * job.Hp + ry) * (uint32_t)job.Wp + (uint32_t)(rx & ~1));
    // one row pointer with constant offsets, so that the loads merge
    const XV_G uint32_t* rw = (const XV_G uint32_t*)((const XV_G char*)src + off);
    uint32_t w[N / 2 + 1];
#pragma unroll
    for (int j = 0; j < N / 2; j++) w[j] = rw[j];
    const int odd = rx & 1;
    w[N / 2] = odd ? rw[N / 2] : 0u;
    const uint32_t sh = (uint32_t)odd << 4;
#pragma unroll
    for (int j = 0; j < N / 2; j++) pp[j] = __builtin_amdgcn_alignbit(w[j + 1], w[j], sh);
  }
}

// The block's vector (dx, dy), two int8 at byte offset off of mv.
__device__ inline void load_mv(const int8_t* mv, uint32_t off, int& dx, int& dy) {
  const uint32_t v = gld<uint16_t>(mv, off);
  dx = (int)(int8_t)(v & 0xffu);
  dy = (int)(int8_t)(v >> 8);
}

// Dequantisation d = clip16((level * IQ[qP%6] * 16 * 2^(qP/6) + 2^(bd-1)) >> bd),
// evaluated exactly in 32 bits: with X = level * IQ * 16 (|X| < 2^26) and
// sh = bd - qP/6, the power of two factors out of the rounding shift, so
// d = clip16((X + 2^(sh-1)) >> sh) for sh > 0 and clip16(X << -sh) for
// sh <= 0, where clamping X to +-2^15 first changes no result.  The final
// clip16 is the saturation of the pair packing.
struct Dequant {
  int m;   // IQ[qP%6] * 16
  int sh;  // bd - qP/6
};

__device__ inline Dequant dequant_params(int qP, int bd) { return Dequant{kIQ[qP % 6] * 16, bd - qP / 6}; }

template <int N>
__device__ inline void dequant_pairs(const int (&lv)[N], const Dequant& q, uint32_t (&ip)[N / 2]) {
  int d[N];
  if (q.sh > 0) {
    const int rnd = 1 << (q.sh - 1);
#pragma unroll
    for (int l = 0; l < N; l++) d[l] = (__mul24(lv[l], q.m) + rnd) >> q.sh;
  } else {
#pragma unroll
    for (int l = 0; l < N; l++) d[l] = min(max(__mul24(lv[l], q.m), -32768), 32768) << (-q.sh);
  }
  to_inverse_order<N>(d, ip);
}

// Inverse column stage of block column k from its dequantised column (pairs
// in inverse order): E[y][slot(k)] = clip16((sum_l M[l][y] d[l] + 64) >> 7).
template <int N>
__device__ inline void inverse_column(const uint32_t (&dq)[N / 2], int16_t (*E)[Tile<N>::P],
                                      int slot) {
  int acc[N];
  inv_part<N>(dq, acc, 64);
#pragma unroll
  for (int y = 0; y < N; y += 2) {
    const uint32_t e = pack_sat(acc[y] >> 7, acc[y + 1] >> 7);
    E[y][slot] = (int16_t)(e & 0xffffu);
    E[y + 1][slot] = (int16_t)(e >> 16);
  }
}

// Inverse row stage and reconstruction of block row r into packed pairs:
// rec = clip(pred + ((sum_k M[k][x] E[k] + 2^(19-B)) >> (20-B)), 0, 2^B-1).
// The residual is saturated to 16 bits and added with 16-bit saturation; as
// 0 <= pred < 2^12, neither saturation can change the clipped result.
template <int N>
__device__ inline void inverse_row(const int16_t* Erow, const uint32_t (&pp)[N / 2], int B,
                                   uint32_t (&rp)[N / 2]) {
  const int sh = 20 - B;
  uint32_t ein[N / 2];
#pragma unroll
  for (int j = 0; j < N / 2; j++) ein[j] = ((const uint32_t*)Erow)[j];
  int acc[N];
  inv_part<N>(ein, acc, 1 << (19 - B));
  const s16x2 zero = {0, 0};
  const s16x2 top = {(short)((1 << B) - 1), (short)((1 << B) - 1)};
#pragma unroll
  for (int j = 0; j < N / 2; j++) {
    const s16x2 res = as_v(pack_sat(acc[2 * j] >> sh, acc[2 * j + 1] >> sh));
    s16x2 v = __builtin_elementwise_add_sat(as_v(pp[j]), res);
    v = __builtin_elementwise_min(__builtin_elementwise_max(v, zero), top);
    rp[j] = as_u(v);
  }
}

// Rate proxy of every coded block of channel c in the tile (one wave per
// channel; bit b of `coded` set for block b).
// The tile holds w = 2|level| + 1.  Lane (b, j) takes scan positions jN ..
// jN+N-1 of block b.  Each nonzero level at position p with previous nonzero
// q (-1 if none) costs ue(p-q-1) + se(level) = 128 - 2 (clz(p - q) +
// clz(|level|)) bits, and clz(|level|) = clz(w) + 1.  The lane's terms, with
// its own segment start as q of its first nonzero, are accumulated as
// 2^17 * count + sum of the clz terms; that term is replaced once the last
// nonzero of the earlier segments is known.  Adds the block's total to
// s.cbits[c][b].
//
// The lane reads each w once and keeps two things: S = sum of clz(w) over
// all N positions (a zero level gives clz(1) = 31) and the mask m of its
// nonzero positions, built as the sum of min(w, 2) << i less the sum of
// 1 << i.  Then, with R = sum over m's set bits of floor(log2 gap) (gaps as
// above, from the 8-bit run table and one correction per further byte of
// m), the accumulated sum is count (2^17 + 63) - R + S - 31 N: each nonzero
// contributes 2^17 + 1 + (31 - floor(log2 gap)) + clz(w), and the zero
// levels' 31 each leave S.
template <int N>
__device__ inline void block_bits(LdsEnc<N>& s, uint32_t coded, int c) {
  const int lane = threadIdx.x & 63;
  const int b = lane / N, j = lane - b * N;
  const bool vb = (coded >> b) & 1u;
  const char* tile = (const char*)&s.TD[c][b][0][0];
  uint32_t acc = 0;
  int prev = -1, first = N;
  if (vb) {
    const uint32_t* tab = kScanTab<N>.v + j * N;
    uint32_t S = 0, ml = 0, mh = 0;
    // groups of at most eight positions (their table offsets and levels in
    // flight together): registers, hence waves
    constexpr int GP = N < 8 ? N : 8;
#pragma unroll
    for (int g0 = 0; g0 < N; g0 += GP) {
      uint32_t sc[GP];
#pragma unroll
      for (int q = 0; q < GP / 4; q++) {
        const u32x4 w = gld<u32x4>(tab, 4 * g0 + 16 * q);
        sc[4 * q] = w.x;
        sc[4 * q + 1] = w.y;
        sc[4 * q + 2] = w.z;
        sc[4 * q + 3] = w.w;
      }
#pragma unroll
      for (int u = 0; u < GP; u++) {
        const int i = g0 + u;
        const uint32_t w = *(const uint16_t*)(tile + sc[u]);  // >= 1
        S += (uint32_t)__builtin_clz(w);
        const uint32_t v = min(w, 2u);
        if (i < 16)
          ml += v << i;
        else
          mh += v << (i - 16);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    uint32_t m = ml - (N >= 16 ? 0xffffu : (1u << N) - 1u);
    if constexpr (N > 16) m |= (mh - 0xffffu) << 16;
    if (m) {
      int r = 0;
#pragma unroll
      for (int k = 0; k < (N + 7) / 8; k++) {
        const uint32_t ck = (m >> (8 * k)) & 0xffu;
        r += s.runs[c][ck];
        if (k > 0 && ck) {
          // the byte's first gap runs from the last set bit below it
          const uint32_t lo = m & ((1u << (8 * k)) - 1u);
          const int last = lo ? 31 - __builtin_clz(lo) : -1;
          const int f = __builtin_ctz(ck);
          r += (31 - __builtin_clz((uint32_t)(8 * k + f - last))) -
               (31 - __builtin_clz((uint32_t)(f + 1)));
        }
      }
      acc = (uint32_t)__builtin_popcount(m) * ((1u << 17) + 63u) - (uint32_t)r + S - 31u * N;
      first = __builtin_ctz(m);
      prev = 31 - __builtin_clz(m);
    }
  }
  // last nonzero of the nearest earlier segment of the same block
  const bool has = first < N;
  const unsigned long long m = __ballot(has);
  const unsigned long long below = m & ((1ull << lane) - 1) & ~((1ull << (b * N)) - 1);
  const int src = below ? 63 - __clzll((long long)below) : lane;
  const int src_last = __shfl(prev + j * N, src);  // block-relative position
  if (has) {
    const int pf = j * N + first;
    const int q = below ? src_last : -1;
    acc += (uint32_t)__builtin_clz((uint32_t)(pf - q)) - (uint32_t)__builtin_clz((uint32_t)(first + 1));
  }
  if (vb && acc) atomicAdd(&s.cbits[c][b], acc);
}

// Squared error of one reconstructed row against the current row over the
// valid samples: x < W and, with kMask, a nonzero validity byte.
template <int N, bool kMask>
__device__ inline uint32_t row_sse(const uint32_t (&cp)[N / 2], const uint32_t (&rp)[N / 2],
                                   const uint8_t* vmask, uint32_t voff, int x0, int W) {
  uint32_t pm[N / 2];
#pragma unroll
  for (int j = 0; j < N / 2; j++) pm[j] = 0xffffffffu;
  if constexpr (kMask) {
    uint32_t w[N / 4 > 0 ? N / 4 : 1];
    if constexpr (N >= 16) {
#pragma unroll
      for (int q = 0; q < N / 16; q++) {
        const u32x4 v = gld<u32x4>(vmask, voff + 16 * q);
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
      }
    } else if constexpr (N == 8) {
      const u32x2 v = gld<u32x2>(vmask, voff);
      w[0] = v.x;
      w[1] = v.y;
    } else {
      w[0] = gld<uint32_t>(vmask, voff);
    }
#pragma unroll
    for (int j = 0; j < N / 2; j++) {
      const uint32_t h = w[j >> 1] >> (16 * (j & 1));  // bytes 2j, 2j+1: 0 or 1
      const uint32_t t = (h & 0xffu) | ((h & 0xff00u) << 8);
      pm[j] = __umul24(t, 0xffffu);
    }
  }
  int sse = 0;  // at most 32 * 4095^2 < 2^31
  if (!kMask && x0 + N <= W) {
    // every sample valid: no mask
#pragma unroll
    for (int j = 0; j < N / 2; j++) {
      const uint32_t d = psub(cp[j], rp[j]);
      sse = dot2(d, d, sse);
    }
    return (uint32_t)sse;
  }
  if (x0 + N > W) {
#pragma unroll
    for (int j = 0; j < N / 2; j++)
      pm[j] &= (x0 + 2 * j < W ? 0xffffu : 0u) | (x0 + 2 * j + 1 < W ? 0xffff0000u : 0u);
  }
#pragma unroll
  for (int j = 0; j < N / 2; j++) {
    const uint32_t d = psub(cp[j], rp[j]) & pm[j];
    sse = dot2(d, d, sse);
  }
  return (uint32_t)sse;
}

// Adaptive block size roles (kRole): 0 -- no split flags; 1 -- size-N
// kernel, codes the whole blocks (all blocks of an I step), writes every
// block's vector bits and zero coefficient bits for split blocks; 2 --
// size-N/2 kernel over the cell grid, codes the cells of split blocks into
// their block's level slot (z-order) and adds their coefficient bits to
// their block's.
template <int kRole>
__device__ inline bool split_codes(const FrameJob& job, int by, int bx, int Wb) {
  if constexpr (kRole == 1) return job.intra || !job.split[by * Wb + bx];
  if constexpr (kRole == 2) return !job.intra && job.split[(by >> 1) * (Wb >> 1) + (bx >> 1)];
  return true;
}

// Level offset (elements) of column k of block (by, bx), channel c: blocks
// are [3][Hb][Wb][N*N]; a cell of a split block sits at z-position
// 2 (by & 1) + (bx & 1) inside its block's (2N)^2 slot.
template <int N, int kRole>
__device__ inline uint32_t level_offset(int c, int by, int bx, int Hb, int Wb, int k) {
  if constexpr (kRole == 2) {
    const uint32_t blk2 = (uint32_t)((by >> 1) * (Wb >> 1) + (bx >> 1));
    const uint32_t z = (uint32_t)(((by & 1) << 1) | (bx & 1));
    return ((uint32_t)c * (uint32_t)(Hb >> 1) * (uint32_t)(Wb >> 1) + blk2) * (4 * N * N) + z * (N * N) +
           (uint32_t)(k * N);
  }
  return ((uint32_t)c * (uint32_t)Hb * (uint32_t)Wb + (uint32_t)(by * Wb + bx)) * (N * N) +
         (uint32_t)(k * N);
}

// Vector entry of block (by, bx): the block's own, or with split flags
// (role 1) its top-left cell on the cell grid.
template <int kRole>
__device__ inline uint32_t vector_index(int by, int bx, int Wb) {
  if constexpr (kRole == 1) return (uint32_t)(2 * by * 2 * Wb + 2 * bx);
  return (uint32_t)(by * Wb + bx);
}

template <int N, int kRole>
__global__ void __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(Tile<N>::kEncWaves)))
encode_kernel(const LaunchDesc jr) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int L2N = Tile<N>::L2N;
  __shared__ LdsEnc<N> s;
  TileCoord tc;
  if (!locate<N>(jr, tc)) return;
  const FrameJob job = *tc.job;
  // read before any store of the kernel, so that it stays a scalar load
  const bool usemask = job.vmask != nullptr && gld<uint32_t>(job.nan_total, 0) != 0u;

  const int t = threadIdx.x;
  const int c = t >> 6;
  const int rem = t & 63;
  const int r = rem / NBW;      // block row (row stages) / column (column stages)
  const int b = rem - r * NBW;
  const int bx = tc.bx0 + b;
  const bool vb = bx < tc.Wb;                                   // the block exists
  const bool code = vb && split_codes<kRole>(job, tc.by, bx, tc.Wb);  // this kernel codes it
  const int B = job.bit_depth;
  const int x0 = bx * N;
  const int y = tc.by * N + r;
  const uint32_t blk = (uint32_t)(tc.by * tc.Wb + bx);                  // block index in a plane
  // byte offset of the thread's row; opaque to the compiler, so that the
  // sample offset is not kept beside it (the kernel is at its register limit)
  uint32_t row_b = 2u * ((uint32_t)(c * job.Hp + y) * (uint32_t)job.Wp + (uint32_t)x0);
  asm volatile("" : "+v"(row_b));
  // each wave sets up its own channel's sums and run table
  if (rem == 0) s.sse[c] = 0ull;
  if (rem < NBW) s.cbits[c][rem] = 0u;
  ((uint32_t*)s.runs[c])[rem] = gld<uint32_t>(kRunTab.v, 4u * (uint32_t)rem);
  if (t == 0) s.mvbits = 0u;
  // coded blocks of the tile, bit b (lanes 0 .. NBW-1 are r = 0)
  const uint32_t coded = (uint32_t)__ballot(code) & ((1u << NBW) - 1u);

  int dx = 0, dy = 0;
  if (code && !job.intra) load_mv(job.mv, 2u * vector_index<kRole>(tc.by, bx, tc.Wb), dx, dy);

  // Forward row stage of row r: T[y][k] = (sum_x M[k][x] res[x] + 2^(s1-1)) >> s1,
  // stored transposed.
  uint32_t cp[N / 2], pp[N / 2];
  if (code) {
    load_row_packed<N>(job.cur, row_b, cp);
    pred_row<N>(job, c, r, y, x0, dx, dy, pp);
    uint32_t er[N / 2];
#pragma unroll
    for (int m = 0; m < N / 2; m++) er[m] = psub(cp[m], pp[m]);  // |res| <= 4095
    const int s1 = L2N + B - 9;
    int acc[N];
    fwd_part<N, 1>(er, acc, 1 << (s1 - 1));
#pragma unroll
    for (int k = 0; k < N; k++) s.TD[c][b][k][r] = (int16_t)(acc[k] >> s1);
  }
  wave_sync();

  // Column stage of column k: forward transform, quantise (levels out to
  // global memory, column-major inside the block, and into the thread's own
  // TD row), dequantise and inverse column transform.
  const int k = r;
  const int qP = job.qp + 6 * (B - 8);
  const Dequant dqp = dequant_params(qP, B + L2N - 5);
  int lv[N];
  bool lane_nz = false;
  if (code) {
    const int qbits = 29 + qP / 6 - B - L2N;
    const int off = (job.intra ? 171 : 85) << (qbits - 9);
    const int offn = (1 << qbits) - 1 - off;
    const int qf = kQf[qP % 6];
    uint32_t* row = (uint32_t*)s.TD[c][b][k];
    ivec<N> acc;
    fwd_column<N>(row, acc, 1 << (L2N + 5));
    // level = sgn(C) min(32767, (|C| Qf + off) >> qbits) in signed form:
    // C >= 0: (C Qf + off) >> qbits; C < 0: (C Qf + 2^qbits - 1 - off) >> qbits
    // (|C Qf| < 2^30, so nothing overflows).  |C| <= 2^15 (the DC row's 64 N
    // is the largest absolute row sum of M, and |T| <= 2^15), so with
    // qbits >= 15 every |level| is at most 2^15 Qf / 2^15 + 1 <= 26215 and
    // the clamp cannot act: a wave-uniform branch leaves it out.
    if (qbits >= 15) {
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int C = acc[l] >> (L2N + 6);
        lv[l] = (__mul24(C, qf) + (C >= 0 ? off : offn)) >> qbits;
      }
    } else {
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int C = acc[l] >> (L2N + 6);
        const int v = (__mul24(C, qf) + (C >= 0 ? off : offn)) >> qbits;
        lv[l] = min(max(v, -32767), 32767);
      }
    }
    // levels out; the tile row gets 2|level| + 1 (never zero) for the rate proxy
    uint32_t lpair[N / 2];
#pragma unroll
    for (int m = 0; m < N / 2; m++) {
      lpair[m] = pack_sat(lv[2 * m], lv[2 * m + 1]);
      const s16x2 v = as_v(lpair[m]);
      const u16x2 a = __builtin_bit_cast(u16x2, __builtin_elementwise_max(v, -v));
      row[m] = __builtin_bit_cast(uint32_t, (u16x2)(a + a + (u16x2){1, 1}));
    }
    store_row_packed<N>(job.lev, 2u * level_offset<N, kRole>(c, tc.by, bx, tc.Hb, tc.Wb, k), lpair);
    uint32_t any = 0;
#pragma unroll
    for (int m = 0; m < N / 2; m++) any |= lpair[m];
    lane_nz = any != 0u;
  }
  // A wave (one channel of the tile) whose levels are all zero -- padding
  // channels, and flat content at high QP -- skips the inverse stages and the
  // rate scan: zero levels dequantise and inverse-transform to an exactly
  // zero residual, so the reconstruction is the prediction, and every block
  // costs its coded-flag bit only.
  const bool wave_nz = __any(lane_nz);
  if (code && wave_nz) {
    uint32_t dq[N / 2];
    dequant_pairs<N>(lv, dqp, dq);
    inverse_column<N>(dq, s.E[c][b], inv_slot<N>(k));
  }
  wave_sync();

  // Rate proxy per block and channel (levels in TD).
  if (wave_nz) block_bits<N>(s, coded, c);

  // Inverse row stage, reconstruction, squared error.
  if (code) {
    uint32_t rp[N / 2];
    if (wave_nz) {
      inverse_row<N>(s.E[c][b][r], pp, B, rp);
    } else {
#pragma unroll
      for (int j = 0; j < N / 2; j++) rp[j] = pp[j];
    }
    store_row_packed<N>(job.rec, row_b, rp);
    // the row index afresh from the lane (mbcnt), not kept from the start
    if (c < job.nch && tc.by * N + (int)__lane_id() / NBW < job.H) {
      const uint32_t sse = usemask ? row_sse<N, true>(cp, rp, job.vmask, row_b >> 1, x0, job.W)
                                   : row_sse<N, false>(cp, rp, nullptr, 0, x0, job.W);
      if (sse) atomicAdd(&s.sse[c], (unsigned long long)sse);
    }
  }

  // se(v) costs 2 floor(log2 |v|) + 3 bits, 1 for v = 0
  auto se_len = [](int v) { return v ? 65u - 2u * (uint32_t)__builtin_clz((uint32_t)abs(v)) : 1u; };
  if constexpr (kRole == 0) {
    if (c == 0 && r == 0 && vb) {
      uint32_t bits = 0;
      if (job.intra) {
        // an intra mode (written by the wavefront kernel) costs one bit
        if (job.imode)
          bits = 1u;
        else
          gst<uint16_t>(job.mv, 2u * blk, (uint16_t)0);
      } else {
        int pmx = 0, pmy = 0;
        if (bx > 0) load_mv(job.mv, 2u * (blk - 1), pmx, pmy);
        bits = se_len(dx - pmx) + se_len(dy - pmy);
      }
      gst<uint32_t>(job.mbits, 4u * blk, bits);
      if (bits) atomicAdd(&s.mvbits, bits);
    }
  } else if constexpr (kRole == 1) {
    // every block's vector unit: I -- nothing (flags and cells zeroed);
    // P -- the split flag, then per coded vector (one, or four in z-order) se
    // of its difference to the vector of the cell left of its top-left cell
    if (c == 0 && r == 0 && vb) {
      const uint32_t Wu = 2u * (uint32_t)tc.Wb;
      const uint32_t u0 = vector_index<1>(tc.by, bx, tc.Wb);
      uint32_t bits = 0;
      if (job.intra) {
        job.split[blk] = 0;
        gst<uint16_t>(job.mv, 2u * u0, (uint16_t)0);
        gst<uint16_t>(job.mv, 2u * (u0 + 1), (uint16_t)0);
        gst<uint16_t>(job.mv, 2u * (u0 + Wu), (uint16_t)0);
        gst<uint16_t>(job.mv, 2u * (u0 + Wu + 1), (uint16_t)0);
      } else {
        const bool sp = job.split[blk] != 0;
        bits = 1u;
        for (int i = 0; i < (sp ? 4 : 1); i++) {
          const uint32_t u = u0 + (uint32_t)(i >> 1) * Wu + (uint32_t)(i & 1);
          const bool first_col = bx == 0 && (i & 1) == 0;
          int mx, my, pmx = 0, pmy = 0;
          load_mv(job.mv, 2u * u, mx, my);
          if (!first_col) load_mv(job.mv, 2u * (u - 1), pmx, pmy);
          bits += se_len(mx - pmx) + se_len(my - pmy);
        }
      }
      gst<uint32_t>(job.mbits, 4u * blk, bits);
      if (bits) atomicAdd(&s.mvbits, bits);
    }
  }
  wave_sync();
  // coefficient bits of the wave's channel c per block (lanes 0 .. NBW-1):
  // bits = 1 (coded flag) + [nnz > 0] (ue(nnz - 1) + 128 nnz - 2 sum clz).
  // The lane index is taken afresh (mbcnt), not kept from the start.
  const int ln = (int)__lane_id();
  uint32_t cb = 0;
  if (ln < NBW && tc.bx0 + ln < tc.Wb) {
    const int bxx = tc.bx0 + ln;
    const uint32_t v = s.cbits[c][ln];
    const uint32_t nnz = v >> 17, sum = v & 0x1ffffu;
    const bool cbk = (coded >> ln) & 1u;
    cb = cbk ? 1u + (nnz > 0 ? 63u - 2u * (uint32_t)__builtin_clz(nnz) + 128u * nnz - 2u * sum : 0u)
             : 0u;
    if constexpr (kRole == 2) {
      // a cell adds to its block's count (zeroed by the size-N kernel)
      if (cbk) {
        const uint32_t Wb2 = (uint32_t)tc.Wb >> 1;
        atomicAdd(job.cbits + ((uint32_t)c * ((uint32_t)tc.Hb >> 1) + (uint32_t)(tc.by >> 1)) * Wb2 +
                      (uint32_t)(bxx >> 1),
                  cb);
      }
    } else {
      gst<uint32_t>(job.cbits, 4u * (((uint32_t)c * tc.Hb + tc.by) * tc.Wb + bxx), cb);
    }
  }
  // the channel's total over the tile (3 * 64 * N coefficients of < 64 bits
  // in all: no overflow)
#pragma unroll
  for (int o = NBW / 2; o >= 1; o >>= 1) cb += __shfl_xor(cb, o);
  // this tile's sums, each wave its channel's; the per-group totals are
  // formed after the last step (the size-N/2 kernel's tiles follow the
  // size-N kernel's)
  uint32_t tile = (uint32_t)tc.tl;
  if constexpr (kRole == 2) {
    constexpr int NBW2 = Tile<2 * N>::NBW;
    tile += (uint32_t)((tc.Hb >> 1) * (((tc.Wb >> 1) + NBW2 - 1) / NBW2));
  }
  const uint32_t part = 8u * kTileSums * tile;
  if (ln == 0) {
    gst<unsigned long long>(job.part, part + 8u * (uint32_t)c, s.sse[c]);
    gst<unsigned long long>(job.part, part + 8u * (3u + (uint32_t)c), (unsigned long long)cb);
    if (c == 0) gst<unsigned long long>(job.part, part + 48u, (unsigned long long)s.mvbits);
  }
}

// One wave per (tile, channel): workgroup 3 w + c decodes channel c of tile w.
// kRole as for the transform kernel: 1 decodes whole blocks, 2 the cells of
// split blocks.
template <int N, int kRole>
__global__ void __launch_bounds__(64) decode_kernel(const LaunchDesc jr) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int L2N = Tile<N>::L2N;
  __shared__ LdsDec<N> s;
  TileCoord tc;
  const int id = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int c = id % 3;
  if (!locate_at<N>(jr, id / 3, tc)) return;
  const FrameJob job = *tc.job;
  const int rem = threadIdx.x;
  const int r = rem / NBW;
  const int b = rem - r * NBW;
  const int bx = tc.bx0 + b;
  const bool vb = bx < tc.Wb && split_codes<kRole>(job, tc.by, bx, tc.Wb);
  const int B = job.bit_depth;
  const int x0 = bx * N;
  const int y = tc.by * N + r;
  const uint32_t row_off = ((uint32_t)(c * job.Hp + y) * (uint32_t)job.Wp + (uint32_t)x0);

  uint32_t pp[N / 2];
  uint32_t lp[N / 2];
  const int k = r;  // column k = r of the block: its N levels are contiguous
  bool lane_nz = false;
  if (vb) {
    load_row_packed<N>(job.lev, 2u * level_offset<N, kRole>(c, tc.by, bx, tc.Hb, tc.Wb, k), lp);
    int dx = 0, dy = 0;
    if (!job.intra) load_mv(job.mv, 2u * vector_index<kRole>(tc.by, bx, tc.Wb), dx, dy);
    pred_row<N>(job, c, r, y, x0, dx, dy, pp);
    uint32_t any = 0;
#pragma unroll
    for (int m = 0; m < N / 2; m++) any |= lp[m];
    lane_nz = any != 0u;
  }
  // all-zero levels in the wave: the residual is exactly zero (as in encode)
  const bool wave_nz = __any(lane_nz);
  if (vb && wave_nz) {
    const int qP = job.qp + 6 * (B - 8);
    const Dequant dqp = dequant_params(qP, B + L2N - 5);
    int lv[N];
#pragma unroll
    for (int m = 0; m < N / 2; m++) {
      lv[2 * m] = (int)(int16_t)(lp[m] & 0xffffu);
      lv[2 * m + 1] = (int)(int16_t)(lp[m] >> 16);
    }
    uint32_t dq[N / 2];
    dequant_pairs<N>(lv, dqp, dq);
    inverse_column<N>(dq, s.E[b], inv_slot<N>(k));
  }
  __syncthreads();
  if (vb) {
    uint32_t rp[N / 2];
    if (wave_nz) {
      inverse_row<N>(s.E[b][r], pp, B, rp);
    } else {
#pragma unroll
      for (int j = 0; j < N / 2; j++) rp[j] = pp[j];
    }
    store_row_packed<N>(job.rec, 2u * row_off, rp);
  }
}

// ---------------------------------------------------------------------------
// Intra-predicted I steps, one wavefront per launch.  In raster order a
// block predicts from its left, top-left, top and top-right neighbours, all
// in earlier wavefronts w = bx + 2 by, so the blocks of one wavefront are
// independent.  A workgroup takes NBW blocks of the wavefront (consecutive
// by) with their 3 channels, in the thread layout of the transform kernel
// (wave c = channel; lane = block row r of block b).
//
// References (ITU-T H.265 8.4.4.2.2) in substitution-scan order: entry i <
// 2N holds p[-1][2N-1-i], entry 2N the corner, entry 2N+1+x holds p[x][-1].
// With equal blocks in raster order the left block is available iff bx > 0,
// the top one iff by > 0, the top-left iff both, the top-right iff by > 0
// and bx + 1 < Wb, the bottom-left never.  The substitution scan then
// reduces to reading every entry from one fixed sample: left entries from
// the left column (its lower half repeating p[-1][N-1]) or, without a left
// block, p[0][-1]; the corner from itself, else p[-1][0], else p[0][-1];
// top entries from the top row (past p[N-1][-1] repeating it without a
// top-right block) or, without a top block, p[-1][0]; nothing available:
// 2^(B-1).
// ---------------------------------------------------------------------------
template <int N>
struct alignas(16) LdsIntra {
  int16_t TD[3][Tile<N>::NBW][N][Tile<N>::P];
  int16_t E[3][Tile<N>::NBW][N][Tile<N>::P];
  uint16_t ref[3][Tile<N>::NBW][4 * N + 2];  // substituted references
  uint16_t flt[3][Tile<N>::NBW][4 * N + 2];  // smoothed for planar (N >= 8)
  uint32_t sad[Tile<N>::NBW][2];             // per block: planar, DC
};

template <int N>
__device__ inline int intra_ref(const FrameJob& job, int c, int x0, int y0, bool aL, bool aT,
                                bool aTR, int i) {
  if (!aL && !aT) return 1 << (job.bit_depth - 1);
  int x, y;
  if (i < 2 * N) {
    x = aL ? x0 - 1 : x0;
    y = aL ? y0 + min(2 * N - 1 - i, N - 1) : y0 - 1;
  } else if (i == 2 * N) {
    x = aL ? x0 - 1 : x0;
    y = aT ? y0 - 1 : y0;
  } else {
    x = aT ? x0 + min(i - 2 * N - 1, aTR ? 2 * N - 1 : N - 1) : x0 - 1;
    y = aT ? y0 - 1 : y0;
  }
  return gld<uint16_t>(job.rec, 2u * ((uint32_t)(c * job.Hp + y) * (uint32_t)job.Wp + (uint32_t)x));
}

template <int N>
__global__ void __launch_bounds__(192) intra_kernel(const LaunchDesc jr, int wave, int decode) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int L2N = Tile<N>::L2N;
  constexpr int NR = 4 * N + 1;
  __shared__ LdsIntra<N> s;
  int tl;
  const FrameJob job = *desc_job(jr, (int)blockIdx.x, tl);
  const int Hb = job.Hp / N, Wb = job.Wp / N;
  // the wavefront's blocks: by in [by_lo, by_hi], bx = wave - 2 by
  const int lo = wave - (Wb - 1);
  const int by_lo = lo > 0 ? (lo + 1) / 2 : 0;
  const int by_hi = min(Hb - 1, wave / 2);
  const int by0 = by_lo + tl * NBW;
  if (by0 > by_hi) return;  // the whole workgroup

  const int t = threadIdx.x;
  const int c = t >> 6;
  const int rem = t & 63;
  const int r = rem / NBW;
  const int b = rem - r * NBW;
  const int by = by0 + b;
  const bool vb = by <= by_hi;  // then 0 <= bx < Wb
  const int bx = wave - 2 * by;
  const int B = job.bit_depth;
  const int x0 = bx * N, y0 = by * N;
  const uint32_t blk = (uint32_t)(by * Wb + bx);
  const uint32_t row_off = (uint32_t)(c * job.Hp + y0 + r) * (uint32_t)job.Wp + (uint32_t)x0;
  if (t < 2 * NBW) s.sad[t >> 1][t & 1] = 0u;

  if (vb) {
    const bool aL = bx > 0, aT = by > 0, aTR = aT && bx + 1 < Wb;
    for (int i = r; i < NR; i += N) s.ref[c][b][i] = (uint16_t)intra_ref<N>(job, c, x0, y0, aL, aT, aTR, i);
  }
  __syncthreads();

  // planar's references: [1 2 1] along the scan (ends kept), or at N = 32 the
  // strong bilinear smoothing when both edges are near-linear (8.4.4.2.3)
  if constexpr (N >= 8) {
    if (vb) {
      const uint16_t* rf = s.ref[c][b];
      const int corner = rf[2 * N], endL = rf[0], midL = rf[N], endT = rf[4 * N], midT = rf[3 * N];
      const int thr = 1 << (B - 5);
      const bool strong = N == 32 && abs(corner + endT - 2 * midT) < thr &&
                          abs(corner + endL - 2 * midL) < thr;
      for (int i = r; i < NR; i += N) {
        int v;
        if (i == 0 || i == 4 * N) {
          v = rf[i];
        } else if (strong) {
          if (i < 2 * N) {
            const int yy = 2 * N - 1 - i;
            v = ((63 - yy) * corner + (yy + 1) * endL + 32) >> 6;
          } else if (i == 2 * N) {
            v = corner;
          } else {
            const int xx = i - 2 * N - 1;
            v = ((63 - xx) * corner + (xx + 1) * endT + 32) >> 6;
          }
        } else {
          v = (rf[i - 1] + 2 * rf[i] + rf[i + 1] + 2) >> 2;
        }
        s.flt[c][b][i] = (uint16_t)v;
      }
    }
    __syncthreads();
  }

  // planar (8.4.4.2.5) and DC (8.4.4.2.6, edges filtered below N = 32) at
  // (x, r) of block b, channel c
  const uint16_t* rf = s.ref[c][b];
  const uint16_t* pf = N >= 8 ? s.flt[c][b] : s.ref[c][b];
  int dc = 0;
  if (vb) {
    int sum = N;
    for (int i = 0; i < N; i++) sum += rf[2 * N + 1 + i] + rf[2 * N - 1 - i];
    dc = sum >> (L2N + 1);
  }
  auto planar = [&](int x) {
    return ((N - 1 - x) * pf[2 * N - 1 - r] + (x + 1) * pf[3 * N + 1] +
            (N - 1 - r) * pf[2 * N + 1 + x] + (r + 1) * pf[N - 1] + N) >>
           (L2N + 1);
  };
  auto dcv = [&](int x) {
    if (N < 32 && r == 0 && x == 0) return (rf[2 * N - 1] + 2 * dc + rf[2 * N + 1] + 2) >> 2;
    if (N < 32 && r == 0) return (rf[2 * N + 1 + x] + 3 * dc + 2) >> 2;
    if (N < 32 && x == 0) return (rf[2 * N - 1 - r] + 3 * dc + 2) >> 2;
    return dc;
  };

  uint32_t cp[N / 2];
  int mode = 0;
  if (!decode) {
    // mode: the smaller SAD over the real channels, planar on a tie
    if (vb) {
      load_row_packed<N>(job.cur, 2u * row_off, cp);
      if (c < job.nch) {
        uint32_t s0 = 0, s1 = 0;
#pragma unroll
        for (int x = 0; x < N; x++) {
          const int v = (int)((cp[x >> 1] >> (16 * (x & 1))) & 0xffffu);
          s0 += (uint32_t)abs(v - planar(x));
          s1 += (uint32_t)abs(v - dcv(x));
        }
        atomicAdd(&s.sad[b][0], s0);
        atomicAdd(&s.sad[b][1], s1);
      }
    }
    __syncthreads();
    mode = s.sad[b][1] < s.sad[b][0] ? 1 : 0;
  } else if (vb) {
    mode = (gld<uint16_t>(job.mv, 2u * blk) & 0xffu) != 0u ? 1 : 0;
  }

  uint32_t pp[N / 2];
  if (vb) {
#pragma unroll
    for (int j = 0; j < N / 2; j++) {
      const int a0 = mode ? dcv(2 * j) : planar(2 * j);
      const int a1 = mode ? dcv(2 * j + 1) : planar(2 * j + 1);
      pp[j] = (uint32_t)a0 | ((uint32_t)a1 << 16);
    }
  }

  const int qP = job.qp + 6 * (B - 8);
  const Dequant dqp = dequant_params(qP, B + L2N - 5);
  const int k = r;  // column stages: block column k
  if (!decode) {
    // residual, forward rows (as the transform kernel)
    if (vb) {
      uint32_t er[N / 2];
#pragma unroll
      for (int m = 0; m < N / 2; m++) er[m] = psub(cp[m], pp[m]);
      const int s1 = L2N + B - 9;
      int acc[N];
      fwd_part<N, 1>(er, acc, 1 << (s1 - 1));
#pragma unroll
      for (int kk = 0; kk < N; kk++) s.TD[c][b][kk][r] = (int16_t)(acc[kk] >> s1);
    }
    __syncthreads();
    // forward column, intra dead-zone quantisation, dequantisation, inverse
    // column; the levels themselves are written by the transform kernel's
    // pass over the step
    if (vb) {
      const int qbits = 29 + qP / 6 - B - L2N;
      const int off = 171 << (qbits - 9);
      const int offn = (1 << qbits) - 1 - off;
      const int qf = kQf[qP % 6];
      ivec<N> acc;
      fwd_column<N>((const uint32_t*)s.TD[c][b][k], acc, 1 << (L2N + 5));
      int lv[N];
#pragma unroll
      for (int l = 0; l < N; l++) {
        const int C = acc[l] >> (L2N + 6);
        const int v = (__mul24(C, qf) + (C >= 0 ? off : offn)) >> qbits;
        lv[l] = min(max(v, -32767), 32767);
      }
      uint32_t dq[N / 2];
      dequant_pairs<N>(lv, dqp, dq);
      inverse_column<N>(dq, s.E[c][b], inv_slot<N>(k));
    }
  } else if (vb) {
    uint32_t lp[N / 2];
    load_row_packed<N>(job.lev, 2u * (((uint32_t)c * Hb * Wb + blk) * (N * N) + k * N), lp);
    int lv[N];
#pragma unroll
    for (int m = 0; m < N / 2; m++) {
      lv[2 * m] = (int)(int16_t)(lp[m] & 0xffffu);
      lv[2 * m + 1] = (int)(int16_t)(lp[m] >> 16);
    }
    uint32_t dq[N / 2];
    dequant_pairs<N>(lv, dqp, dq);
    inverse_column<N>(dq, s.E[c][b], inv_slot<N>(k));
  }
  __syncthreads();

  // inverse rows and reconstruction; encode also keeps the prediction and
  // the mode
  if (vb) {
    uint32_t rp[N / 2];
    inverse_row<N>(s.E[c][b][r], pp, B, rp);
    store_row_packed<N>(job.rec, 2u * row_off, rp);
    if (!decode) {
      store_row_packed<N>(job.pred, 2u * row_off, pp);
      if (c == 0 && r == 0) gst<uint16_t>(job.mv, 2u * blk, (uint16_t)mode);
    }
  }
}

template <int N>
hipError_t launch_intra_t(const LaunchDesc& d, int wave, int decode, hipStream_t s) {
  intra_kernel<N><<<d.tiles, 192, 0, s>>>(d, wave, decode);
  return hipGetLastError();
}

template <int N, int kRole = 0>
hipError_t launch_encode_t(const LaunchDesc& d, hipStream_t s) {
  encode_kernel<N, kRole><<<d.tiles, 192, 0, s>>>(d);
  return hipGetLastError();
}
template <int N, int kRole = 0>
hipError_t launch_decode_t(const LaunchDesc& d, hipStream_t s) {
  decode_kernel<N, kRole><<<3u * (unsigned)d.tiles, 64, 0, s>>>(d);
  return hipGetLastError();
}

}  // namespace

int xf_tiles_per_job(int N, int Hb, int Wb) {
  const int nbw = 64 / N;
  return Hb * ((Wb + nbw - 1) / nbw);
}

hipError_t launch_encode(int N, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  switch (N) {
    case 4: return launch_encode_t<4>(r, s);
    case 8: return launch_encode_t<8>(r, s);
    case 16: return launch_encode_t<16>(r, s);
    case 32: return launch_encode_t<32>(r, s);
    default: return hipErrorInvalidValue;
  }
}

int intra_tiles_per_job(int N, int Hb, int Wb) {
  // a wavefront holds at most min(Hb, ceil(Wb / 2)) blocks
  const int nbw = 64 / N;
  const int most = std::min(Hb, (Wb + 1) / 2);
  return (most + nbw - 1) / nbw;
}

hipError_t launch_intra(int N, const LaunchDesc& r, int wave, int decode, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  switch (N) {
    case 4: return launch_intra_t<4>(r, wave, decode, s);
    case 8: return launch_intra_t<8>(r, wave, decode, s);
    case 16: return launch_intra_t<16>(r, wave, decode, s);
    case 32: return launch_intra_t<32>(r, wave, decode, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_encode_split(int N, int role, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  if (role == 1) {
    switch (N) {
      case 8: return launch_encode_t<8, 1>(r, s);
      case 16: return launch_encode_t<16, 1>(r, s);
      case 32: return launch_encode_t<32, 1>(r, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (role == 2) {
    switch (N) {
      case 4: return launch_encode_t<4, 2>(r, s);
      case 8: return launch_encode_t<8, 2>(r, s);
      case 16: return launch_encode_t<16, 2>(r, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_decode_split(int N, int role, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  if (role == 1) {
    switch (N) {
      case 8: return launch_decode_t<8, 1>(r, s);
      case 16: return launch_decode_t<16, 1>(r, s);
      case 32: return launch_decode_t<32, 1>(r, s);
      default: return hipErrorInvalidValue;
    }
  }
  if (role == 2) {
    switch (N) {
      case 4: return launch_decode_t<4, 2>(r, s);
      case 8: return launch_decode_t<8, 2>(r, s);
      case 16: return launch_decode_t<16, 2>(r, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

hipError_t launch_decode(int N, const LaunchDesc& r, hipStream_t s) {
  if (r.nseg <= 0 || r.tiles <= 0) return hipSuccess;
  switch (N) {
    case 4: return launch_decode_t<4>(r, s);
    case 8: return launch_decode_t<8>(r, s);
    case 16: return launch_decode_t<16>(r, s);
    case 32: return launch_decode_t<32>(r, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xv
