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
#include "xv_internal.h"

namespace xv {

namespace {

__device__ inline int ue_len(uint32_t k) { return 2 * (31 - __clz((int)(k + 1))) + 1; }
__device__ inline int se_len(int v) {
  return ue_len(v > 0 ? (uint32_t)(2 * v - 1) : (uint32_t)(-2 * v));
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

// LDS layout per workgroup, encode (int16):
//   TD [3][NBW][N][P]  forward row-stage output transposed ([k][y]); each
//                      column thread then overwrites its own row k with the
//                      column's levels ([k][l])
//   E  [3][NBW][N][P]  inverse column-stage output ([y][k])
//   scan [N*N]         scan position -> offset (k * P + l) of the level in a
//                      block's TD tile
//   sums               per-workgroup squared error per channel, bits
// Residual rows and dequantised columns stay in registers.
template <int N>
struct alignas(16) LdsEnc {
  int16_t TD[3][Tile<N>::NBW][N][Tile<N>::P];
  int16_t E[3][Tile<N>::NBW][N][Tile<N>::P];
  uint16_t scan[N * N];
  unsigned long long sse[3];
  uint32_t cbits[3][Tile<N>::NBW];
  uint32_t nnz[3][Tile<N>::NBW];
  uint32_t mvbits;
};

// Decode: the levels as stored (raster [l][k] per block) and the inverse
// column-stage output.
template <int N>
struct alignas(16) LdsDec {
  int16_t L[3][Tile<N>::NBW][N * N];
  int16_t E[3][Tile<N>::NBW][N][Tile<N>::P];
};

// Up-right diagonal scan of an N x N block (ITU-T H.265 6.5.3): anti-
// diagonals d = x + y in order, each from its bottom-left end upwards.  The
// table maps scan position to the level's offset in the transposed tile.
template <int N>
__device__ inline void build_scan(uint16_t* scan) {
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
    const int y = i / N, x = i - (i / N) * N;
    const int d = x + y;
    const int before = d < N ? d * (d + 1) / 2 : N * N - (2 * N - 1 - d) * (2 * N - d) / 2;
    const int first_x = d < N ? 0 : d - N + 1;
    scan[before + x - first_x] = (uint16_t)(x * Tile<N>::P + y);
  }
}

struct TileCoord {
  const FrameJob* job;
  int tl, by, bx0, Hb, Wb;
};

template <int N>
__device__ inline bool locate(const LaunchDesc& jd, TileCoord& tc) {
  int tl;
  tc.job = desc_job(jd, blockIdx.x, tl);
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

// ---------------------------------------------------------------------------
// Matrix products on v_dot2c_i32_i16: two 16x16-bit products per lane-op.
// Every stage is an outer-product loop over input pairs m: all N outputs
// accumulate acc[k] += M[k][2m] x[2m] + M[k][2m+1] x[2m+1], the coefficient
// pairs coming through scalar loads (SGPR operands) from tables passed by
// pointer, the input pair from LDS.  Inputs are 16-bit by construction:
// residuals (|r| <= 4095), row-stage outputs (|T| < 2^15), dequantised levels
// and the inverse column-stage output (both clipped to 16 bits).
// Table layout per N: fwd[m][k] = (M[k][2m], M[k][2m+1]) (y = M x), then
// inv[m][n] = (M[2m][n], M[2m+1][n]) (x = M^T y); tables for N = 4, 8, 16,
// 32 follow each other.
// ---------------------------------------------------------------------------
typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ inline int dot2(uint32_t coef_pair, uint32_t x_pair, int acc) {
  return __builtin_amdgcn_sdot2(__builtin_bit_cast(s16x2, coef_pair),
                                __builtin_bit_cast(s16x2, x_pair), acc, false);
}

__host__ __device__ constexpr uint32_t cpair(int lo, int hi) {
  return ((uint32_t)lo & 0xffffu) | (((uint32_t)hi & 0xffffu) << 16);
}

__host__ __device__ constexpr int coef_offset(int N) {
  return N == 4 ? 0 : (N == 8 ? 2 * 4 * 2 : (N == 16 ? 2 * 4 * 2 + 2 * 8 * 4 : 2 * 4 * 2 + 2 * 8 * 4 + 2 * 16 * 8));
}
constexpr int kCoefWords = coef_offset(32) + 2 * 32 * 16;

struct CoefTables {
  uint32_t w[kCoefWords];
};

constexpr CoefTables make_coef_tables() {
  CoefTables t{};
  for (int N = 4; N <= 32; N *= 2) {
    uint32_t* f = t.w + coef_offset(N);
    uint32_t* v = f + (N / 2) * N;
    for (int m = 0; m < N / 2; m++)
      for (int k = 0; k < N; k++) {
        f[m * N + k] = cpair(dct_coef(N, k, 2 * m), dct_coef(N, k, 2 * m + 1));
        v[m * N + k] = cpair(dct_coef(N, 2 * m, k), dct_coef(N, 2 * m + 1, k));
      }
  }
  return t;
}

__constant__ CoefTables kCoef = make_coef_tables();

// acc[k] = sum_m dot2(table[m][k], src[m]); src: N/2 packed pairs in LDS.
template <int N>
__device__ inline void mat_pairs(const uint32_t* __restrict__ tb, const uint32_t* src, int (&acc)[N]) {
#pragma unroll
  for (int k = 0; k < N; k++) acc[k] = 0;
  constexpr int kUnrollM = N <= 8 ? N / 2 : 4;
#pragma unroll kUnrollM
  for (int m = 0; m < N / 2; m++) {
    const uint32_t x = src[m];
#pragma unroll
    for (int k = 0; k < N; k++) acc[k] = dot2(tb[m * N + k], x, acc[k]);
  }
}

// The same with the input pairs in registers.
template <int N>
__device__ inline void mat_pairs_r(const uint32_t* __restrict__ tb, const uint32_t (&src)[N / 2],
                                   int (&acc)[N]) {
#pragma unroll
  for (int k = 0; k < N; k++) acc[k] = 0;
#pragma unroll
  for (int m = 0; m < N / 2; m++) {
#pragma unroll
    for (int k = 0; k < N; k++) acc[k] = dot2(tb[m * N + k], src[m], acc[k]);
  }
}

// Packed 16-bit residual pair: (cur - pred) per half.
__device__ inline uint32_t sub_pairs(uint32_t a, uint32_t b) {
  const int lo = (int)(a & 0xffffu) - (int)(b & 0xffffu);
  const int hi = (int)(a >> 16) - (int)(b >> 16);
  return ((uint32_t)lo & 0xffffu) | ((uint32_t)hi << 16);
}

// Packed u16 row (N samples) from global memory.
template <int N>
__device__ inline void load_row_packed(const uint16_t* p, uint32_t (&v)[N / 2]) {
  if constexpr (N >= 8) {
#pragma unroll
    for (int q = 0; q < N / 8; q++) {
      const uint4 w = ((const uint4*)p)[q];
      v[4 * q + 0] = w.x;
      v[4 * q + 1] = w.y;
      v[4 * q + 2] = w.z;
      v[4 * q + 3] = w.w;
    }
  } else {
    const uint2 w = *(const uint2*)p;
    v[0] = w.x;
    v[1] = w.y;
  }
}

template <int N>
__device__ inline void store_row_packed(uint16_t* p, const uint32_t (&v)[N / 2]) {
  if constexpr (N >= 8) {
#pragma unroll
    for (int q = 0; q < N / 8; q++)
      ((uint4*)p)[q] = make_uint4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
    *(uint2*)p = make_uint2(v[0], v[1]);
  }
}

// Prediction row as packed pairs: I -> 2^(B-1); P -> the reference displaced
// by (dx, dy).  A coded vector keeps the displaced block inside the padded
// picture; the clamp only guarantees in-bounds reads for a corrupt vector.
template <int N>
__device__ inline void pred_row(const FrameJob& job, int c, int y, int x0, int dx, int dy,
                                uint32_t (&pp)[N / 2]) {
  if (job.intra) {
    const uint32_t h = 1u << (job.bit_depth - 1);
#pragma unroll
    for (int j = 0; j < N / 2; j++) pp[j] = h | (h << 16);
  } else {
    const int yb = y - (y % N);
    const int ry = min(max(yb + dy, 0), job.Hp - N) + (y - yb);
    const int rx = min(max(x0 + dx, 0), job.Wp - N);
    const uint16_t* rp = job.ref + (size_t)c * job.Hp * job.Wp + (size_t)ry * job.Wp + rx;
    if ((rx & 1) == 0) {
      const uint32_t* r32 = (const uint32_t*)rp;
#pragma unroll
      for (int j = 0; j < N / 2; j++) pp[j] = r32[j];
    } else {
#pragma unroll
      for (int j = 0; j < N / 2; j++) pp[j] = (uint32_t)rp[2 * j] | ((uint32_t)rp[2 * j + 1] << 16);
    }
  }
}

// Dequantisation d = clip16((level * IQ[qP%6] * 16 * 2^(qP/6) + 2^(bd-1)) >> bd),
// evaluated exactly in 32 bits: with X = level * IQ * 16 (|X| < 2^26) and
// sh = bd - qP/6, the power of two factors out of the rounding shift, so
// d = clip16((X + 2^(sh-1)) >> sh) for sh > 0 and clip16(X << -sh) for
// sh <= 0, where clamping X to +-2^15 first changes no result.
struct Dequant {
  int m;   // IQ[qP%6] * 16
  int sh;  // bd - qP/6
};

__device__ inline Dequant dequant_params(int qP, int bd) { return Dequant{kIQ[qP % 6] * 16, bd - qP / 6}; }

__device__ inline int clamp16(int v) { return min(max(v, -32768), 32767); }

__device__ inline int dequant(int lv, const Dequant& q) {
  const int X = lv * q.m;
  if (q.sh > 0) return clamp16((X + (1 << (q.sh - 1))) >> q.sh);
  return clamp16(min(max(X, -32768), 32768) << (-q.sh));
}

// Inverse column stage of block column k from its dequantised column (pairs
// in registers): E[y][k] = clip16((sum_l M[l][y] d[l] + 64) >> 7).
template <int N>
__device__ inline void inverse_column(const uint32_t* inv, const uint32_t (&dpair)[N / 2],
                                      int16_t (*E)[Tile<N>::P], int k) {
  int acc[N];
  mat_pairs_r<N>(inv, dpair, acc);
#pragma unroll
  for (int y = 0; y < N; y++) E[y][k] = (int16_t)clamp16((acc[y] + 64) >> 7);
}

// Inverse row stage and reconstruction of block row r into packed pairs.
template <int N>
__device__ inline void inverse_row(const uint32_t* inv, const int16_t* Erow,
                                   const uint32_t (&pp)[N / 2], int B, uint32_t (&rp)[N / 2]) {
  const int sh = 20 - B;
  const int rnd = 1 << (19 - B);
  const int Lmax = (1 << B) - 1;
  int acc[N];
  mat_pairs<N>(inv, (const uint32_t*)Erow, acc);
#pragma unroll
  for (int j = 0; j < N / 2; j++) {
    int v0 = (int)(pp[j] & 0xffffu) + ((acc[2 * j] + rnd) >> sh);
    int v1 = (int)(pp[j] >> 16) + ((acc[2 * j + 1] + rnd) >> sh);
    v0 = v0 < 0 ? 0 : (v0 > Lmax ? Lmax : v0);
    v1 = v1 < 0 ? 0 : (v1 > Lmax ? Lmax : v1);
    rp[j] = (uint32_t)v0 | ((uint32_t)v1 << 16);
  }
}

// Rate proxy of every block of channel c in the tile (one wave per channel):
// each nonzero level adds ue(run) + se(level) to its block's LDS counter.
template <int N>
__device__ inline void block_bits(LdsEnc<N>& s, const TileCoord& tc, int c) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int S = N * N < 64 ? N * N : 64;  // lanes per block segment
  constexpr int BPC = 64 / S;                  // blocks per pass
  constexpr int CPB = (N * N) / S;             // chunks per block
  const int lane = threadIdx.x & 63;
  const int seg = lane / S, pin = lane - seg * S;
  for (int bb = 0; bb < NBW; bb += BPC) {
    const int b = bb + seg;
    const bool vb = (tc.bx0 + b) < tc.Wb;
    int last = -1;
    uint32_t acc = 0;
#pragma unroll
    for (int ci = 0; ci < CPB; ci++) {
      const int p = ci * S + pin;
      const int lv = vb ? (int)(&s.TD[c][b][0][0])[s.scan[p]] : 0;
      const unsigned long long m = __ballot(lv != 0);
      const unsigned long long segm = (S == 64) ? m : ((m >> (seg * S)) & ((1ull << S) - 1));
      const unsigned long long below = segm & ((1ull << pin) - 1);
      const int prev = below ? ci * S + 63 - __clzll((long long)below) : last;
      if (lv != 0) acc += (uint32_t)(ue_len((uint32_t)(p - prev - 1)) + se_len(lv));
      if (segm) last = ci * S + 63 - __clzll((long long)segm);
      if (pin == 0 && segm) atomicAdd(&s.nnz[c][b], (uint32_t)__popcll(segm));
    }
    if (acc) atomicAdd(&s.cbits[c][b], acc);
  }
}

template <int N>
__global__ void __launch_bounds__(192) __attribute__((amdgpu_waves_per_eu(Tile<N>::kEncWaves)))
encode_kernel(const LaunchDesc jr) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int L2N = Tile<N>::L2N;
  __shared__ LdsEnc<N> s;
  TileCoord tc;
  if (!locate<N>(jr, tc)) return;
  const FrameJob& job = *tc.job;
  const uint32_t* __restrict__ fwd = jr.coef + coef_offset(N);
  const uint32_t* __restrict__ inv = fwd + (N / 2) * N;
  build_scan<N>(s.scan);

  const int t = threadIdx.x;
  const int c = t >> 6;
  const int rem = t & 63;
  const int r = rem / NBW;      // block row (row stages) / column (column stages)
  const int b = rem - r * NBW;
  const int bx = tc.bx0 + b;
  const bool vb = bx < tc.Wb;
  const int B = job.bit_depth;
  const size_t plane = (size_t)job.Hp * job.Wp;
  const int x0 = bx * N;
  const int y = tc.by * N + r;
  if (t < 3) s.sse[t] = 0ull;
  if (t < 3 * NBW) {
    s.cbits[t / NBW][t % NBW] = 0u;
    s.nnz[t / NBW][t % NBW] = 0u;
  }
  if (t == 0) s.mvbits = 0u;

  int dx = 0, dy = 0;
  if (vb && !job.intra) {
    const int8_t* mv = job.mv + ((size_t)tc.by * tc.Wb + bx) * 2;
    dx = mv[0];
    dy = mv[1];
  }

  // Forward row stage of row r: T[y][k] = (sum_x M[k][x] res[x] + 2^(s1-1)) >> s1,
  // stored transposed.
  uint32_t cp[N / 2], pp[N / 2];
  if (vb) {
    load_row_packed<N>(job.cur + c * plane + (size_t)y * job.Wp + x0, cp);
    pred_row<N>(job, c, y, x0, dx, dy, pp);
    uint32_t er[N / 2];
#pragma unroll
    for (int m = 0; m < N / 2; m++) er[m] = sub_pairs(cp[m], pp[m]);
    int acc[N];
    mat_pairs_r<N>(fwd, er, acc);
    const int s1 = L2N + B - 9;
    const int rnd1 = 1 << (s1 - 1);
#pragma unroll
    for (int k = 0; k < N; k++) s.TD[c][b][k][r] = (int16_t)((acc[k] + rnd1) >> s1);
  }
  __syncthreads();

  // Column stage of column k: forward transform, quantise (levels into the
  // thread's own TD row, transposed), dequantise and inverse column
  // transform from registers.
  if (vb) {
    const int k = r;
    const int qP = job.qp + 6 * (B - 8);
    const int qbits = 29 + qP / 6 - B - L2N;
    const uint32_t off = (uint32_t)(job.intra ? 171 : 85) << (qbits - 9);
    const uint32_t qf = (uint32_t)kQf[qP % 6];
    const Dequant dqp = dequant_params(qP, B + L2N - 5);
    // the row is only accessed as packed 32-bit pairs (no mixed-width aliasing)
    uint32_t* row = (uint32_t*)s.TD[c][b][k];
    int acc[N];
    mat_pairs<N>(fwd, row, acc);
    uint32_t lpair[N / 2], dpair[N / 2];
#pragma unroll
    for (int l = 0; l < N; l += 2) {
      int lv[2], dq[2];
#pragma unroll
      for (int h = 0; h < 2; h++) {
        const int C = (acc[l + h] + (1 << (L2N + 5))) >> (L2N + 6);
        const uint32_t a = (uint32_t)(C < 0 ? -C : C);
        uint32_t mq = (a * qf + off) >> qbits;
        mq = mq > 32767u ? 32767u : mq;
        lv[h] = C < 0 ? -(int)mq : (int)mq;
        dq[h] = dequant(lv[h], dqp);
      }
      lpair[l / 2] = ((uint32_t)lv[0] & 0xffffu) | ((uint32_t)lv[1] << 16);
      dpair[l / 2] = ((uint32_t)dq[0] & 0xffffu) | ((uint32_t)dq[1] << 16);
    }
#pragma unroll
    for (int m = 0; m < N / 2; m++) row[m] = lpair[m];
    inverse_column<N>(inv, dpair, s.E[c][b], k);
  }
  __syncthreads();

  // Levels out (block-major, raster [l][k] inside a block) in 16-byte
  // chunks gathered from the transposed tiles.
  {
    constexpr int CH = (N * N) / 8;  // uint4 chunks per block
    for (int e = t; e < 3 * NBW * CH; e += blockDim.x) {
      const int cb = e / CH, q = e - cb * CH;
      const int cc = cb / NBW, bb = cb - cc * NBW;
      if (tc.bx0 + bb >= tc.Wb) continue;
      const int16_t* tile = &s.TD[cc][bb][0][0];
      uint32_t w[4];
#pragma unroll
      for (int j = 0; j < 4; j++) {
        const int i0 = q * 8 + 2 * j, i1 = i0 + 1;
        const int v0 = tile[(i0 % N) * Tile<N>::P + i0 / N];
        const int v1 = tile[(i1 % N) * Tile<N>::P + i1 / N];
        w[j] = ((uint32_t)v0 & 0xffffu) | ((uint32_t)v1 << 16);
      }
      int16_t* dst = job.lev + (((size_t)cc * tc.Hb + tc.by) * tc.Wb + tc.bx0 + bb) * (N * N);
      ((uint4*)dst)[q] = make_uint4(w[0], w[1], w[2], w[3]);
    }
  }

  // Inverse row stage, reconstruction, squared error.
  if (vb) {
    uint32_t rp[N / 2];
    inverse_row<N>(inv, s.E[c][b][r], pp, B, rp);
    store_row_packed<N>(job.rec + c * plane + (size_t)y * job.Wp + x0, rp);
    if (c < job.nch && y < job.H) {
      const bool usemask = job.vmask != nullptr && *job.nan_total != 0u;
      const uint8_t* vm = usemask ? job.vmask + c * plane + (size_t)y * job.Wp + x0 : nullptr;
      uint32_t sse = 0;  // at most 32 * 4095^2 < 2^32
#pragma unroll
      for (int j = 0; j < N; j++) {
        const int cv = (int)((cp[j >> 1] >> (16 * (j & 1))) & 0xffffu);
        const int rv = (int)((rp[j >> 1] >> (16 * (j & 1))) & 0xffffu);
        const bool ok = (x0 + j < job.W) && (!usemask || vm[j]);
        const int e = cv - rv;
        sse += ok ? (uint32_t)(e * e) : 0u;
      }
      if (sse) atomicAdd(&s.sse[c], (unsigned long long)sse);
    }
  }

  // Rate proxy per block and channel; vector bits.
  block_bits<N>(s, tc, c);
  if (c == 0 && r == 0 && vb) {
    int8_t* mv = job.mv + ((size_t)tc.by * tc.Wb + bx) * 2;
    uint32_t bits = 0;
    if (job.intra) {
      mv[0] = 0;
      mv[1] = 0;
    } else {
      int pmx = 0, pmy = 0;
      if (bx > 0) {
        pmx = mv[-2];
        pmy = mv[-1];
      }
      bits = (uint32_t)(se_len(dx - pmx) + se_len(dy - pmy));
    }
    job.mbits[(size_t)tc.by * tc.Wb + bx] = bits;
    if (bits) atomicAdd(&s.mvbits, bits);
  }
  __syncthreads();
  if (t < 3 * NBW) {
    const int cc = t / NBW, bb = t - cc * NBW;
    if (tc.bx0 + bb < tc.Wb) {
      const uint32_t nnz = s.nnz[cc][bb];
      const uint32_t bits = 1u + (nnz > 0 ? (uint32_t)ue_len(nnz - 1) + s.cbits[cc][bb] : 0u);
      job.cbits[((size_t)cc * tc.Hb + tc.by) * tc.Wb + tc.bx0 + bb] = bits;
      s.cbits[cc][bb] = bits;  // per-block total, summed below by thread 0
    }
  }
  __syncthreads();
  // this tile's sums; the per-group totals are formed after the last step
  unsigned long long* part = job.part + (size_t)tc.tl * 5;
  if (t == 0) {
    unsigned long long cb = 0;
    for (int i = 0; i < 3 * NBW; i++)
      if (tc.bx0 + (i % NBW) < tc.Wb) cb += s.cbits[i / NBW][i % NBW];
    part[3] = cb;
    part[4] = s.mvbits;
  }
  if (t < 3) part[t] = s.sse[t];
}

template <int N>
__global__ void __launch_bounds__(192) decode_kernel(const LaunchDesc jr) {
  constexpr int NBW = Tile<N>::NBW;
  constexpr int L2N = Tile<N>::L2N;
  __shared__ LdsDec<N> s;
  TileCoord tc;
  if (!locate<N>(jr, tc)) return;
  const FrameJob& job = *tc.job;
  const uint32_t* __restrict__ inv = jr.coef + coef_offset(N) + (N / 2) * N;
  const int t = threadIdx.x;
  const int c = t >> 6;
  const int rem = t & 63;
  const int r = rem / NBW;
  const int b = rem - r * NBW;
  const int bx = tc.bx0 + b;
  const bool vb = bx < tc.Wb;
  const int B = job.bit_depth;
  const size_t plane = (size_t)job.Hp * job.Wp;
  const int x0 = bx * N;
  const int y = tc.by * N + r;

  {
    constexpr int CH = (N * N) / 8;
    for (int e = t; e < 3 * NBW * CH; e += blockDim.x) {
      const int cb = e / CH, q = e - cb * CH;
      const int cc = cb / NBW, bb = cb - cc * NBW;
      if (tc.bx0 + bb >= tc.Wb) continue;
      const int16_t* src =
          job.lev + (((size_t)cc * tc.Hb + tc.by) * tc.Wb + tc.bx0 + bb) * (N * N);
      ((uint4*)s.L[cc][bb])[q] = ((const uint4*)src)[q];
    }
  }
  uint32_t pp[N / 2];
  if (vb) {
    int dx = 0, dy = 0;
    if (!job.intra) {
      const int8_t* mv = job.mv + ((size_t)tc.by * tc.Wb + bx) * 2;
      dx = mv[0];
      dy = mv[1];
    }
    pred_row<N>(job, c, y, x0, dx, dy, pp);
  }
  __syncthreads();
  if (vb) {
    const int k = r;
    const int qP = job.qp + 6 * (B - 8);
    const Dequant dqp = dequant_params(qP, B + L2N - 5);
    uint32_t dpair[N / 2];
#pragma unroll
    for (int m = 0; m < N / 2; m++) {
      const int d0 = dequant(s.L[c][b][(2 * m) * N + k], dqp);
      const int d1 = dequant(s.L[c][b][(2 * m + 1) * N + k], dqp);
      dpair[m] = ((uint32_t)d0 & 0xffffu) | ((uint32_t)d1 << 16);
    }
    inverse_column<N>(inv, dpair, s.E[c][b], k);
  }
  __syncthreads();
  if (vb) {
    uint32_t rp[N / 2];
    inverse_row<N>(inv, s.E[c][b][r], pp, B, rp);
    store_row_packed<N>(job.rec + c * plane + (size_t)y * job.Wp + x0, rp);
  }
}

const uint32_t* coef_tables() {
  static const uint32_t* ptr = nullptr;
  if (!ptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(kCoef)) == hipSuccess) ptr = (const uint32_t*)p;
  }
  return ptr;
}

template <int N>
hipError_t launch_encode_t(const LaunchDesc& r, hipStream_t s) {
  LaunchDesc d = r;
  d.coef = coef_tables();
  if (!d.coef) return hipErrorInvalidSymbol;
  encode_kernel<N><<<d.tiles, 192, 0, s>>>(d);
  return hipGetLastError();
}
template <int N>
hipError_t launch_decode_t(const LaunchDesc& r, hipStream_t s) {
  LaunchDesc d = r;
  d.coef = coef_tables();
  if (!d.coef) return hipErrorInvalidSymbol;
  decode_kernel<N><<<d.tiles, 192, 0, s>>>(d);
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
