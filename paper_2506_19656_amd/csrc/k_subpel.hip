// k_subpel.hip -- quarter-sample motion: refinement of the integer search's
// vectors (encode) and motion-compensated prediction from quarter-sample
// vectors (decode).
//
// The paper's x265 presets use sub-sample motion (Appendix, codec
// configurations) without describing it; this is the stated reading, the
// H.265 tool itself: vectors in quarter samples, the prediction at a
// fractional position given by the luma fractional sample interpolation of
// ITU-T H.265 (8-tap filters, intermediate shifts B - 8 and 6, reference
// coordinates clamped to the picture) and the default weighted prediction of
// one reference (round, shift by 14 - B, clip to [0, 2^B - 1]), every plane
// of a band group treated alike (4:4:4, independent bands).  The refinement
// takes the best of the integer vector and its 8 half-sample neighbours,
// then of that one and its 8 quarter-sample neighbours, by the lexicographic
// minimum of (SAD over the real channels, |mx| + |my|, my, mx).
//
// Mapping: one workgroup per block.  The reference samples the refinement
// can reach -- (N + 8)^2 per channel around the integer vector, clamped to
// the picture -- and the current block are staged in LDS once.  Per stage,
// the horizontal filter of each of the stage's three candidate columns is
// evaluated once into LDS (16-bit), then every thread sums the nine
// candidates' absolute differences over its samples from the vertical filter
// of those rows.  The winner's prediction of all three channels is written
// to the step's prediction plane, which the transform kernel reads at
// displacement zero; the vector goes back to the vector array in quarter
// samples.
#include "xv_internal.h"

namespace xv {

namespace {

// fL[frac][tap] of H.265; tap i weighs the sample at integer offset i - 3.
// Taps are below 64 in magnitude and the samples they weigh (u16 samples of
// at most 12 bits, 16-bit filter outputs) fit 24 bits, so every product is a
// full-rate 24-bit multiply (__mul24) and exact.
__constant__ int kLuma[4][8] = {{0, 0, 0, 64, 0, 0, 0, 0},
                                {-1, 4, -10, 58, 17, -5, 1, 0},
                                {-1, 4, -11, 40, 40, -11, 4, -1},
                                {0, 1, -5, 17, 58, -10, 4, -1}};

template <int N>
struct SpLds {
  static constexpr int WN = N + 8;  // staged window side
  uint16_t win[3][WN][WN];          // reference at (y0 + by - 4 + r, x0 + bx - 4 + q), clamped
  uint16_t cur[3][N][N];
  int16_t hb[3][3][WN][N];          // horizontal filter, per candidate column slot
  uint32_t red[4][9];               // per-wave partial SADs
  int32_t best[2];                  // chosen vector of a stage (quarter samples)
};

template <int N>
constexpr int sp_threads() {
  return N >= 16 ? 256 : 64;
}

typedef const __attribute__((address_space(1))) uint16_t gu16s;

// Stage the clamped reference window around integer position (bx, by) of the
// block and (optionally) the current block.
template <int N>
__device__ inline void stage(SpLds<N>& s, const FrameJob& job, int x0, int y0, int bx, int by,
                             bool with_cur) {
  constexpr int T = sp_threads<N>();
  constexpr int WN = SpLds<N>::WN;
  const int plane = job.Hp * job.Wp;
  const gu16s* ref = (const gu16s*)job.ref;
  for (int idx = threadIdx.x; idx < 3 * WN * WN; idx += T) {
    const int c = idx / (WN * WN);
    const int rem = idx - c * WN * WN;
    const int r = rem / WN, q = rem - (rem / WN) * WN;
    const int y = min(max(y0 + by - 4 + r, 0), job.Hp - 1);
    const int x = min(max(x0 + bx - 4 + q, 0), job.Wp - 1);
    s.win[c][r][q] = ref[(uint32_t)c * plane + (uint32_t)y * job.Wp + (uint32_t)x];
  }
  if (with_cur) {
    const gu16s* cur = (const gu16s*)job.cur;
    for (int idx = threadIdx.x; idx < 3 * N * N; idx += T) {
      const int c = idx / (N * N);
      const int rem = idx - c * N * N;
      const int i = rem / N, j = rem - (rem / N) * N;
      s.cur[c][i][j] = cur[(uint32_t)c * plane + (uint32_t)(y0 + i) * job.Wp + (uint32_t)(x0 + j)];
    }
  }
}

// Horizontal filter of candidate column slot xs: integer offset xo (-1 or 0
// from the window's centre column) and fraction fx != 0, for every window row.
template <int N>
__device__ inline void hpass(SpLds<N>& s, int xs, int xo, int fx, int shift1) {
  constexpr int T = sp_threads<N>();
  constexpr int WN = SpLds<N>::WN;
  int f[8];
#pragma unroll
  for (int i = 0; i < 8; i++) f[i] = kLuma[fx][i];
  for (int idx = threadIdx.x; idx < 3 * WN * N; idx += T) {
    const int c = idx / (WN * N);
    const int rem = idx - c * WN * N;
    const int r = rem / N, j = rem - (rem / N) * N;
    int acc = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) acc += __mul24(f[i], (int)s.win[c][r][j + xo + 1 + i]);
    s.hb[xs][c][r][j] = (int16_t)(acc >> shift1);
  }
}

// Predicted sample (i, j) of channel c at the candidate whose column slot xs
// has integer offset xo and fraction fx and whose row has integer offset yo
// and fraction fy (offsets relative to the window's centre).
template <int N>
__device__ inline int vsample(const SpLds<N>& s, int c, int i, int j, int xs, int xo, int fx,
                              int yo, int fy, int B) {
  int pred;
  if (fy == 0) {
    const int r = i + yo + 4;
    pred = fx ? (int)s.hb[xs][c][r][j] : (int)s.win[c][r][j + xo + 4] << (14 - B);
  } else {
    int acc = 0;
    if (fx) {
#pragma unroll
      for (int t = 0; t < 8; t++) acc += __mul24(kLuma[fy][t], (int)s.hb[xs][c][i + yo + 1 + t][j]);
      pred = acc >> 6;
    } else {
#pragma unroll
      for (int t = 0; t < 8; t++)
        acc += __mul24(kLuma[fy][t], (int)s.win[c][i + yo + 1 + t][j + xo + 4]);
      pred = acc >> (B - 8);
    }
  }
  const int shw = 14 - B;
  const int v = (pred + (1 << (shw - 1))) >> shw;
  return min(max(v, 0), (1 << B) - 1);
}

// Lexicographic order of (SAD, |mx| + |my|, my, mx).
__device__ inline bool key_less(uint32_t sa, int mxa, int mya, uint32_t sb, int mxb, int myb) {
  if (sa != sb) return sa < sb;
  const int la = abs(mxa) + abs(mya), lb = abs(mxb) + abs(myb);
  if (la != lb) return la < lb;
  if (mya != myb) return mya < myb;
  return mxa < mxb;
}

template <int N>
__device__ inline void write_pred(const SpLds<N>& s, const FrameJob& job, int x0, int y0, int xs,
                                  int xo, int fx, int yo, int fy) {
  constexpr int T = sp_threads<N>();
  const int plane = job.Hp * job.Wp;
  __attribute__((address_space(1))) uint16_t* out =
      (__attribute__((address_space(1))) uint16_t*)job.pred;
  for (int idx = threadIdx.x; idx < 3 * N * N; idx += T) {
    const int c = idx / (N * N);
    const int rem = idx - c * N * N;
    const int i = rem / N, j = rem - (rem / N) * N;
    out[(uint32_t)c * plane + (uint32_t)(y0 + i) * job.Wp + (uint32_t)(x0 + j)] =
        (uint16_t)vsample<N>(s, c, i, j, xs, xo, fx, yo, fy, job.bit_depth);
  }
}

template <int N>
__global__ void __launch_bounds__(sp_threads<N>()) subpel_kernel(const LaunchDesc d) {
  constexpr int T = sp_threads<N>();
  __shared__ SpLds<N> s;
  int local = 0;
  const FrameJob* jp = desc_job(d, (int)blockIdx.x, local);
  const FrameJob job = *jp;
  const int Wb = job.Wp / N;
  const int bxi = local % Wb, byi = local / Wb;
  const int x0 = bxi * N, y0 = byi * N;
  const int B = job.bit_depth;
  const uint32_t blk = (uint32_t)local;
  const uint16_t mvw = *(const __attribute__((address_space(1))) uint16_t*)(
      (const __attribute__((address_space(1))) char*)job.mv + 2u * blk);
  const int dx = (int)(int8_t)(mvw & 0xffu), dy = (int)(int8_t)(mvw >> 8);
  stage<N>(s, job, x0, y0, dx, dy, true);
  __syncthreads();

  int cx = 4 * dx, cy = 4 * dy;
  int xo_x[3], fx_x[3], yo_y[3], fy_y[3];
  for (int st = 0; st < 2; st++) {
    const int step = st == 0 ? 2 : 1;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int mx = cx + (k - 1) * step, my = cy + (k - 1) * step;
      xo_x[k] = (mx >> 2) - dx;
      fx_x[k] = mx & 3;
      yo_y[k] = (my >> 2) - dy;
      fy_y[k] = my & 3;
    }
#pragma unroll
    for (int k = 0; k < 3; k++)
      if (fx_x[k]) hpass<N>(s, k, xo_x[k], fx_x[k], B - 8);
    __syncthreads();
    uint32_t sad[9];
#pragma unroll
    for (int q = 0; q < 9; q++) sad[q] = 0;
    for (int idx = threadIdx.x; idx < job.nch * N * N; idx += T) {
      const int c = idx / (N * N);
      const int rem = idx - c * N * N;
      const int i = rem / N, j = rem - (rem / N) * N;
      const int a = s.cur[c][i][j];
#pragma unroll
      for (int ky = 0; ky < 3; ky++)
#pragma unroll
        for (int kx = 0; kx < 3; kx++)
          sad[ky * 3 + kx] += (uint32_t)abs(
              a - vsample<N>(s, c, i, j, kx, xo_x[kx], fx_x[kx], yo_y[ky], fy_y[ky], B));
    }
#pragma unroll
    for (int q = 0; q < 9; q++) {
      uint32_t v = sad[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
      sad[q] = v;
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
      for (int q = 0; q < 9; q++) s.red[w][q] = sad[q];
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t bs = 0;
      int bmx = 0, bmy = 0;
      for (int q = 0; q < 9; q++) {
        uint32_t v = 0;
        for (int ww = 0; ww < T / 64; ww++) v += s.red[ww][q];
        const int mx = cx + (q % 3 - 1) * step, my = cy + (q / 3 - 1) * step;
        if (q == 0 || key_less(v, mx, my, bs, bmx, bmy)) {
          bs = v;
          bmx = mx;
          bmy = my;
        }
      }
      s.best[0] = bmx;
      s.best[1] = bmy;
    }
    __syncthreads();
    // the same for every lane: keep it (and the filter choices) scalar
    cx = __builtin_amdgcn_readfirstlane(s.best[0]);
    cy = __builtin_amdgcn_readfirstlane(s.best[1]);
    if (st == 0) __syncthreads();  // the next stage overwrites hb and best
  }
  // the winner is one of the last stage's three columns and three rows; the
  // slots of that stage hold distinct vectors, so exactly one of each matches
  int kx = 1, ky = 1;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    if ((cx >> 2) - dx == xo_x[k] && (cx & 3) == fx_x[k]) kx = k;
    if ((cy >> 2) - dy == yo_y[k] && (cy & 3) == fy_y[k]) ky = k;
  }
  write_pred<N>(s, job, x0, y0, kx, xo_x[kx], fx_x[kx], yo_y[ky], fy_y[ky]);
  if (threadIdx.x == 0) {
    const uint16_t v = (uint16_t)((uint8_t)(int8_t)cx | ((uint16_t)(uint8_t)(int8_t)cy << 8));
    *(__attribute__((address_space(1))) uint16_t*)(
        (__attribute__((address_space(1))) char*)job.mv + 2u * blk) = v;
  }
}

// Decode: the prediction plane of a P step from the stored quarter-sample
// vectors.
template <int N>
__global__ void __launch_bounds__(sp_threads<N>()) mc_kernel(const LaunchDesc d) {
  __shared__ SpLds<N> s;
  int local = 0;
  const FrameJob* jp = desc_job(d, (int)blockIdx.x, local);
  const FrameJob job = *jp;
  const int Wb = job.Wp / N;
  const int bxi = local % Wb, byi = local / Wb;
  const int x0 = bxi * N, y0 = byi * N;
  const uint16_t mvw = *(const __attribute__((address_space(1))) uint16_t*)(
      (const __attribute__((address_space(1))) char*)job.mv + 2u * (uint32_t)local);
  const int mx = (int)(int8_t)(mvw & 0xffu), my = (int)(int8_t)(mvw >> 8);
  // window centred on the vector's integer part: offsets are then zero
  stage<N>(s, job, x0, y0, mx >> 2, my >> 2, false);
  __syncthreads();
  if (mx & 3) hpass<N>(s, 0, 0, mx & 3, job.bit_depth - 8);
  __syncthreads();
  write_pred<N>(s, job, x0, y0, 0, 0, mx & 3, 0, my & 3);
}

template <int N>
hipError_t launch_subpel_t(const LaunchDesc& d, hipStream_t st) {
  subpel_kernel<N><<<d.tiles, sp_threads<N>(), 0, st>>>(d);
  return hipGetLastError();
}

template <int N>
hipError_t launch_mc_t(const LaunchDesc& d, hipStream_t st) {
  mc_kernel<N><<<d.tiles, sp_threads<N>(), 0, st>>>(d);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_subpel(int N, const LaunchDesc& d, hipStream_t s) {
  if (d.tiles <= 0) return hipSuccess;
  switch (N) {
    case 4: return launch_subpel_t<4>(d, s);
    case 8: return launch_subpel_t<8>(d, s);
    case 16: return launch_subpel_t<16>(d, s);
    case 32: return launch_subpel_t<32>(d, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mc(int N, const LaunchDesc& d, hipStream_t s) {
  if (d.tiles <= 0) return hipSuccess;
  switch (N) {
    case 4: return launch_mc_t<4>(d, s);
    case 8: return launch_mc_t<8>(d, s);
    case 16: return launch_mc_t<16>(d, s);
    case 32: return launch_mc_t<32>(d, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace xv
