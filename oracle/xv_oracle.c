/*
 * xv_oracle.c -- CPU oracle for the band-packed transform-coding loop.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU path is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product
 * library never does.  It shares no source with the GPU path.
 *
 * What is computed, and where it comes from (paper: "Video Compression for
 * Spatiotemporal Earth System Data", arXiv 2506.19656):
 *   - bit-depth conversion of every band to B-bit integers   (Sec. II-A)
 *   - grouping of the bands, in input order, into 3-channel frames, with the
 *     remainder group padded by repeating its last band      (Sec. II-A, Listing 1 text)
 *   - forward fill of missing (NaN) data                      (Sec. III-B)
 *   - bits per pixel per band and per-channel PSNR whose peak is the maximum
 *     of the original channel                                  (Sec. II-C)
 * The paper hands frames to an HEVC encoder and describes none of its
 * internals.  Below the frame level this oracle therefore follows a stated
 * reading built on the public ITU-T H.265 conventions (integer DCT-II,
 * QP-driven scalar quantiser, Exp-Golomb codes); each such step is marked
 * "paper silent; reading".  The readings are listed in the design notes.
 *
 * Conventions: all arithmetic on coded values is integer; ">>" of a negative
 * value must be an arithmetic (flooring) shift, which xvo_selfcheck() asserts.
 * Floating point is IEEE binary64 with no contraction (build with
 * -ffp-contract=off, no fast-math).
 */
#include "xv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Basic helpers                                                              */
/* ------------------------------------------------------------------------- */

static int ilog2(int n) {
  int k = 0;
  while ((1 << k) < n) k++;
  return k;
}

int xvo_selfcheck(void) {
  volatile int32_t a = -7;
  volatile int64_t b = -7;
  if ((a >> 1) != -4) return -1;
  if ((b >> 2) != -2) return -1;
  return 0;
}

static double read_sample(const void* data, int dtype, int64_t idx) {
  if (dtype == XVO_U16) return (double)((const uint16_t*)data)[idx];
  return (double)((const float*)data)[idx];
}

/* ------------------------------------------------------------------------- */
/* Step 1: per-band statistics (bit-depth conversion, Sec. II-A; per-channel  */
/* peak, Sec. II-C).  Paper silent on the conversion; reading: min-max over   */
/* the whole cube per band, NaN excluded.  All-NaN band -> mn = mx = 0.       */
/* ------------------------------------------------------------------------- */
void xvo_stats(const void* data, int dtype, int64_t T, int64_t H, int64_t W,
               int64_t Bn, double* mn, double* mx, int64_t* n_valid) {
  for (int64_t b = 0; b < Bn; b++) {
    double lo = INFINITY, hi = -INFINITY;
    int64_t cnt = 0;
    for (int64_t p = 0; p < T * H * W; p++) {
      double v = read_sample(data, dtype, p * Bn + b);
      if (isnan(v)) continue;
      if (v < lo) lo = v;
      if (v > hi) hi = v;
      cnt++;
    }
    if (cnt == 0) { lo = 0.0; hi = 0.0; }
    mn[b] = lo;
    mx[b] = hi;
    if (n_valid) n_valid[b] = cnt;
  }
}

/* ------------------------------------------------------------------------- */
/* Step 2: missing-data fill (Sec. III-B: forward fill).                      */
/* FILL_FORWARD: the last valid value before t; leading gaps take the first   */
/* valid value after t.  FILL_NEAREST (reading used for cloud-gapped cubes):  */
/* the valid sample at the smallest |t - t'|, ties to the earlier t'.  A      */
/* series with no valid sample takes mn_b.                                    */
/* ------------------------------------------------------------------------- */
double xvo_filled_value(const void* data, int dtype, int64_t T, int64_t H,
                        int64_t W, int64_t Bn, int64_t t, int64_t y, int64_t x,
                        int64_t b, int fill_mode, double mn_b, int* is_valid) {
  int64_t pix = (y * W + x) * Bn + b;
  int64_t frame = H * W * Bn;
  double v = read_sample(data, dtype, t * frame + pix);
  if (!isnan(v)) {
    if (is_valid) *is_valid = 1;
    return v;
  }
  if (is_valid) *is_valid = 0;
  if (fill_mode == XVO_FILL_FORWARD) {
    for (int64_t u = t - 1; u >= 0; u--) {
      double w = read_sample(data, dtype, u * frame + pix);
      if (!isnan(w)) return w;
    }
    for (int64_t u = t + 1; u < T; u++) {
      double w = read_sample(data, dtype, u * frame + pix);
      if (!isnan(w)) return w;
    }
    return mn_b;
  }
  for (int64_t d = 1; d < T; d++) {
    if (t - d >= 0) {
      double w = read_sample(data, dtype, (t - d) * frame + pix);
      if (!isnan(w)) return w;
    }
    if (t + d < T) {
      double w = read_sample(data, dtype, (t + d) * frame + pix);
      if (!isnan(w)) return w;
    }
  }
  return mn_b;
}

/* ------------------------------------------------------------------------- */
/* Step 3: normalisation to B bits (Sec. II-A bit-depth conversion; formula   */
/* paper silent, reading: per-band min-max, round half up).                   */
/* q = floor((x - mn) * L / (mx - mn) + 1/2) clamped to [0, L], L = 2^B - 1,  */
/* evaluated as exactly this chain of IEEE binary64 operations; a constant    */
/* band (mx == mn) maps to 0.                                                 */
/* ------------------------------------------------------------------------- */
int32_t xvo_normalize(double x, double mn, double mx, int B) {
  double L = (double)((1 << B) - 1);
  double range = mx - mn;
  if (range == 0.0) return 0;
  double d = x - mn;
  double num = d * L;
  double v = num / range;
  double q = floor(v + 0.5);
  if (q < 0.0) q = 0.0;
  if (q > L) q = L;
  return (int32_t)q;
}

/* Inverse of the conversion, used by decode and the physical-domain PSNR:
 * x_hat = mn + (q * (mx - mn)) / L in binary64, then cast to the output type
 * (u16: floor(x_hat + 1/2) clamped to [0, 65535]; f32: round to nearest). */
double xvo_denormalize(int32_t q, double mn, double mx, int B) {
  double L = (double)((1 << B) - 1);
  double range = mx - mn;
  double num = (double)q * range;
  return mn + num / L;
}

double xvo_cast_output(double v, int dtype) {
  if (dtype == XVO_U16) {
    double r = floor(v + 0.5);
    if (r < 0.0) r = 0.0;
    if (r > 65535.0) r = 65535.0;
    return r;
  }
  return (double)(float)v;
}

/* ------------------------------------------------------------------------- */
/* Steps 4-5: packing into 3-channel frames (Sec. II-A: bands split in input  */
/* order into groups of three; the remainder group repeats its last band) and */
/* spatial edge padding to a multiple of the block size (paper silent;        */
/* reading: replicate the last real row/column).                              */
/* frame: [3][Hp][Wp] u16; valid: [3][Hp][Wp] u8 (1 = real pixel of a real    */
/* band that was not missing).                                                */
/* ------------------------------------------------------------------------- */
int64_t xvo_source_band(int64_t g, int c, int64_t Bn, int pad_mode) {
  int64_t b = 3 * g + c;
  if (b < Bn) return b;
  if (pad_mode == XVO_PAD_REPEAT) return Bn - 1;
  return -1; /* zero channel */
}

void xvo_make_frame(const void* data, int dtype, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, const double* mn, const double* mx,
                    const xvo_params* p, int64_t g, int64_t t, int64_t Hp,
                    int64_t Wp, uint16_t* frame, uint8_t* valid) {
  for (int c = 0; c < 3; c++) {
    int64_t b = xvo_source_band(g, c, Bn, p->pad_mode);
    int real_band = (3 * g + c) < Bn;
    for (int64_t y = 0; y < Hp; y++) {
      for (int64_t x = 0; x < Wp; x++) {
        int64_t o = ((int64_t)c * Hp + y) * Wp + x;
        if (b < 0) {
          frame[o] = 0;
          if (valid) valid[o] = 0;
          continue;
        }
        int64_t ys = y < H ? y : H - 1;
        int64_t xs = x < W ? x : W - 1;
        int ok = 0;
        double v = xvo_filled_value(data, dtype, T, H, W, Bn, t, ys, xs, b,
                                    p->fill_mode, mn[b], &ok);
        frame[o] = (uint16_t)xvo_normalize(v, mn[b], mx[b], p->bit_depth);
        if (valid) valid[o] = (uint8_t)(real_band && ok && y < H && x < W);
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Integer DCT-II matrix of ITU-T H.265 (paper silent on codec internals;     */
/* reading: the standard's transform).  For k > 0 the 32-point entry is the   */
/* standard's integer approximation of 64*sqrt(2)*cos(pi*m/64) with           */
/* m = (2n+1)k mod 128; the row k = 0 is 64.  Magnitudes for m = 1..31 are    */
/* the normative values; the sign and quadrant follow the cosine.  The        */
/* N-point matrix takes rows k*32/N of the 32-point one, first N columns.     */
/* ------------------------------------------------------------------------- */
static const int kCosMag[32] = {
    0,  90, 90, 90, 89, 88, 87, 85, 83, 82, 80, 78, 75, 73, 70, 67,
    64, 61, 57, 54, 50, 46, 43, 38, 36, 31, 25, 22, 18, 13, 9,  4};

static int dct32_entry(int k, int n) {
  if (k == 0) return 64;
  int m = ((2 * n + 1) * k) % 128;
  if (m < 32) return kCosMag[m];
  if (m < 64) return -kCosMag[64 - m];
  if (m < 96) return -kCosMag[m - 64];
  return kCosMag[128 - m];
}

void xvo_dct_matrix(int N, int32_t* M) {
  for (int k = 0; k < N; k++)
    for (int n = 0; n < N; n++) M[k * N + n] = dct32_entry(k * (32 / N), n);
}

/* ------------------------------------------------------------------------- */
/* Forward 2-D transform (paper silent; reading: H.265 forward core           */
/* transform).  Stage 1 over each row y: T[y][k] = (sum_x M[k][x] r[y][x] +   */
/* 2^(s1-1)) >> s1, s1 = log2N + B - 9.  Stage 2 over each column k:          */
/* C[l][k] = (sum_y M[l][y] T[y][k] + 2^(s2-1)) >> s2, s2 = log2N + 6.        */
/* r and C are N*N row-major ([y][x] and [l][k], l vertical frequency).       */
/* ------------------------------------------------------------------------- */
void xvo_forward_transform(int N, int B, const int32_t* r, int32_t* C) {
  int32_t M[32 * 32];
  int32_t Tm[32 * 32];
  xvo_dct_matrix(N, M);
  int s1 = ilog2(N) + B - 9;
  int s2 = ilog2(N) + 6;
  for (int y = 0; y < N; y++)
    for (int k = 0; k < N; k++) {
      int64_t acc = 0;
      for (int x = 0; x < N; x++) acc += (int64_t)M[k * N + x] * r[y * N + x];
      Tm[y * N + k] = (int32_t)((acc + ((int64_t)1 << (s1 - 1))) >> s1);
    }
  for (int l = 0; l < N; l++)
    for (int k = 0; k < N; k++) {
      int64_t acc = 0;
      for (int y = 0; y < N; y++) acc += (int64_t)M[l * N + y] * Tm[y * N + k];
      C[l * N + k] = (int32_t)((acc + ((int64_t)1 << (s2 - 1))) >> s2);
    }
}

/* ------------------------------------------------------------------------- */
/* Quantiser scales (paper silent; reading: H.265 scalar quantiser).          */
/* IQ[k] = round(64 * 2^((k-4)/6)), Qf[k] = round(2^20 / IQ[k]), k = 0..5,    */
/* evaluated here from their closed forms.                                    */
/* ------------------------------------------------------------------------- */
int32_t xvo_iq_scale(int k) { return (int32_t)floor(64.0 * pow(2.0, (k - 4) / 6.0) + 0.5); }
int32_t xvo_q_scale(int k) {
  return (int32_t)floor(1048576.0 / (double)xvo_iq_scale(k) + 0.5);
}

/* Dead-zone quantisation.  qP = QP + 6(B-8); qbits = 29 + floor(qP/6) - B -
 * log2N; rounding offset 171/512 (intra) or 85/512 (inter) of a step;
 * level = sign(C) * min(32767, (|C| * Qf[qP%6] + off) >> qbits). */
void xvo_quantize(int N, int B, int qp, int intra, const int32_t* C,
                  int16_t* lev) {
  int qP = qp + 6 * (B - 8);
  int qbits = 29 + qP / 6 - B - ilog2(N);
  int64_t off = (int64_t)(intra ? 171 : 85) << (qbits - 9);
  int64_t qf = xvo_q_scale(qP % 6);
  for (int i = 0; i < N * N; i++) {
    int64_t a = C[i] < 0 ? -(int64_t)C[i] : (int64_t)C[i];
    int64_t m = (a * qf + off) >> qbits;
    if (m > 32767) m = 32767;
    lev[i] = (int16_t)(C[i] < 0 ? -m : m);
  }
}

/* Dequantisation.  bd = B + log2N - 5;
 * d = clip16((level * IQ[qP%6] * 16 * 2^floor(qP/6) + 2^(bd-1)) >> bd). */
void xvo_dequantize(int N, int B, int qp, const int16_t* lev, int32_t* d) {
  int qP = qp + 6 * (B - 8);
  int bd = B + ilog2(N) - 5;
  int64_t scale = (int64_t)xvo_iq_scale(qP % 6) * 16 * ((int64_t)1 << (qP / 6));
  for (int i = 0; i < N * N; i++) {
    int64_t v = ((int64_t)lev[i] * scale + ((int64_t)1 << (bd - 1))) >> bd;
    if (v < -32768) v = -32768;
    if (v > 32767) v = 32767;
    d[i] = (int32_t)v;
  }
}

/* Inverse 2-D transform (paper silent; reading: H.265 inverse transform,
 * vertical first).  E[y][k] = clip16((sum_l M[l][y] d[l][k] + 64) >> 7);
 * r[y][x] = (sum_k M[k][x] E[y][k] + 2^(19-B)) >> (20 - B). */
void xvo_inverse_transform(int N, int B, const int32_t* d, int32_t* r) {
  int32_t M[32 * 32];
  int32_t E[32 * 32];
  xvo_dct_matrix(N, M);
  int s2 = 20 - B;
  for (int y = 0; y < N; y++)
    for (int k = 0; k < N; k++) {
      int64_t acc = 0;
      for (int l = 0; l < N; l++) acc += (int64_t)M[l * N + y] * d[l * N + k];
      int64_t v = (acc + 64) >> 7;
      if (v < -32768) v = -32768;
      if (v > 32767) v = 32767;
      E[y * N + k] = (int32_t)v;
    }
  for (int y = 0; y < N; y++)
    for (int x = 0; x < N; x++) {
      int64_t acc = 0;
      for (int k = 0; k < N; k++) acc += (int64_t)M[k * N + x] * E[y * N + k];
      r[y * N + x] = (int32_t)((acc + ((int64_t)1 << (s2 - 1))) >> s2);
    }
}

/* ------------------------------------------------------------------------- */
/* Rate proxy (Exp-Golomb code lengths; paper silent on the entropy coder,    */
/* reading: order-0 Exp-Golomb lengths in place of CABAC).                    */
/* ------------------------------------------------------------------------- */
int xvo_ue_len(uint32_t k) {
  uint64_t v = (uint64_t)k + 1;
  int nb = 0;
  while ((v >> nb) > 1) nb++;
  return 2 * nb + 1;
}

int xvo_se_len(int32_t v) {
  uint32_t k = v > 0 ? (uint32_t)(2 * (int64_t)v - 1) : (uint32_t)(-2 * (int64_t)v);
  return xvo_ue_len(k);
}

/* Up-right diagonal scan over the whole N x N block: positions ordered by
 * anti-diagonal x + y ascending, then by x ascending (x = column).
 * order[i] = y * N + x of the i-th scanned position. */
void xvo_scan_order(int N, int32_t* order) {
  int i = 0;
  for (int s = 0; s <= 2 * (N - 1); s++)
    for (int x = 0; x < N; x++) {
      int y = s - x;
      if (y < 0 || y >= N) continue;
      order[i++] = y * N + x;
    }
}

/* bits = 1 (coded flag) + [nnz > 0] * (ue(nnz - 1) + sum over nonzero levels in
 * scan order of (ue(run) + se(level))), run = zeros since the previous
 * nonzero (or since the scan start). */
uint32_t xvo_coef_bits(int N, const int16_t* lev) {
  int32_t order[32 * 32];
  xvo_scan_order(N, order);
  int nnz = 0;
  for (int i = 0; i < N * N; i++) nnz += lev[i] != 0;
  uint32_t bits = 1;
  if (nnz == 0) return bits;
  bits += (uint32_t)xvo_ue_len((uint32_t)(nnz - 1));
  int run = 0;
  for (int i = 0; i < N * N; i++) {
    int16_t v = lev[order[i]];
    if (v == 0) {
      run++;
      continue;
    }
    bits += (uint32_t)(xvo_ue_len((uint32_t)run) + xvo_se_len(v));
    run = 0;
  }
  return bits;
}

/* Motion-vector bits: se(mvx - pmx) + se(mvy - pmy), predictor = the left
 * neighbour's vector in the same block row, (0,0) in the first column. */
uint32_t xvo_mv_bits(int mvx, int mvy, int pmx, int pmy) {
  return (uint32_t)(xvo_se_len(mvx - pmx) + xvo_se_len(mvy - pmy));
}

/* ------------------------------------------------------------------------- */
/* Bitstream.  The codes the rate proxy counts, written out MSB-first:        */
/* ue(k) = floor(log2(k+1)) zero bits followed by k+1 in binary; se(v) maps   */
/* v > 0 to 2v - 1 and v <= 0 to -2v (the Exp-Golomb codes of ITU-T H.265    */
/* clause 9.2, which the rate proxy's lengths are the lengths of).            */
/* Order, frame by frame (f = g * T + t):                                     */
/*   the Hb block rows of vectors: per block, se(dx - pdx) then se(dy - pdy), */
/*   pdx/pdy the left neighbour's vector, (0,0) in column 0; nothing for an   */
/*   I frame;                                                                 */
/*   for channel c = 0, 1, 2 the Hb block rows of coefficients: per block the */
/*   coded flag (1 bit, set when a level is nonzero), then ue(nnz - 1) and,   */
/*   per nonzero level in up-right diagonal scan order, ue(run) and          */
/*   se(level).                                                               */
/* Each block row is a segment; the bit offset of every segment is recorded  */
/* so that rows can be parsed independently.  The code lengths are exactly   */
/* the rate proxy's, so the payload holds coef_bits + mv_bits bits.          */
/* ------------------------------------------------------------------------- */
typedef struct {
  uint8_t* buf;
  uint64_t cap_bits;
  uint64_t pos;
  int overflow;
} bit_writer;

static void put_bit(bit_writer* w, int b) {
  if (w->pos >= w->cap_bits) {
    w->overflow = 1;
    return;
  }
  if (b) w->buf[w->pos >> 3] |= (uint8_t)(0x80u >> (w->pos & 7));
  w->pos++;
}

static void put_ue(bit_writer* w, uint32_t k) {
  uint64_t v = (uint64_t)k + 1;
  int m = 0;
  while ((v >> m) > 1) m++;
  for (int i = 0; i < m; i++) put_bit(w, 0);
  for (int i = m; i >= 0; i--) put_bit(w, (int)((v >> i) & 1));
}

static void put_se(bit_writer* w, int32_t v) {
  put_ue(w, v > 0 ? (uint32_t)(2 * (int64_t)v - 1) : (uint32_t)(-2 * (int64_t)v));
}

typedef struct {
  const uint8_t* buf;
  uint64_t bits;
  uint64_t pos;
  int overrun;
} bit_reader;

static int get_bit(bit_reader* r) {
  if (r->pos >= r->bits) {
    r->overrun = 1;
    return 0;
  }
  int b = (r->buf[r->pos >> 3] >> (7 - (r->pos & 7))) & 1;
  r->pos++;
  return b;
}

static uint32_t get_ue(bit_reader* r) {
  int m = 0;
  while (!r->overrun && get_bit(r) == 0) {
    m++;
    if (m > 32) {
      r->overrun = 1;
      return 0;
    }
  }
  uint64_t v = 1;
  for (int i = 0; i < m; i++) v = (v << 1) | (uint64_t)get_bit(r);
  return (uint32_t)(v - 1);
}

static int32_t get_se(bit_reader* r) {
  uint32_t k = get_ue(r);
  return (k & 1) ? (int32_t)((k + 1) / 2) : -(int32_t)(k / 2);
}

/* Stream structure shared by the three functions below.  Per frame: the
 * vector units of the blocks in raster order, then for channel c = 0, 1, 2
 * the coefficient units of the blocks in raster order; a row of units is a
 * segment.  A P block's vector unit holds se(dx - pdx), se(dy - pdy) with
 * the left block's vector as predictor ((0,0) in column 0).  An I block's
 * vector unit is empty, or one intra-mode bit with imodes.  With the
 * adaptive block size (splits non-NULL) a P block's vector unit is its split
 * flag and then its one or four vectors (the vector and predictor rule of
 * the split reading), and its coefficient unit holds one N x N or four
 * N/2 x N/2 block codes in z-order.  A block code: the coded flag, then
 * ue(nnz - 1) and per nonzero level in up-right diagonal scan order ue(run),
 * se(level). */
typedef struct {
  int N;
  int64_t G, T, Hb, Wb;
  int gop, imodes;
  int32_t order[32 * 32], order_h[16 * 16];
} stream_shape;

static void shape_init(stream_shape* sh, int N, int64_t G, int64_t T, int gop, int64_t Hb,
                       int64_t Wb, int imodes) {
  sh->N = N;
  sh->G = G;
  sh->T = T;
  sh->gop = gop;
  sh->Hb = Hb;
  sh->Wb = Wb;
  sh->imodes = imodes;
  xvo_scan_order(N, sh->order);
  if (N >= 8) xvo_scan_order(N / 2, sh->order_h);
}

/* vectors of frame f: [Hb][Wb][2], or [2 Hb][2 Wb][2] with splits */
static const int8_t* frame_mvs(const stream_shape* sh, const int8_t* mvs, int64_t f, int split) {
  return mvs + f * (split ? 4 : 1) * sh->Hb * sh->Wb * 2;
}

/* Vector-unit codes of block (bx, by) of a P frame with splits: the flag,
 * then each coded vector against the cell to its left; calls put_se for
 * each difference (w NULL: only counts).  Returns the unit's length. */
static uint32_t split_vector_unit(const stream_shape* sh, const int8_t* mvu, int split,
                                  int64_t bx, int64_t by, bit_writer* w) {
  int64_t Wu = 2 * sh->Wb;
  uint32_t bits = 1;
  if (w) put_bit(w, split);
  for (int i = 0; i < (split ? 4 : 1); i++) {
    int64_t xu = 2 * bx + (i & 1), yu = 2 * by + (i >> 1);
    int pmx = xu > 0 ? mvu[2 * (yu * Wu + xu - 1)] : 0;
    int pmy = xu > 0 ? mvu[2 * (yu * Wu + xu - 1) + 1] : 0;
    int mx = mvu[2 * (yu * Wu + xu)], my = mvu[2 * (yu * Wu + xu) + 1];
    bits += xvo_mv_bits(mx, my, pmx, pmy);
    if (w) {
      put_se(w, mx - pmx);
      put_se(w, my - pmy);
    }
  }
  return bits;
}

static void put_block(bit_writer* w, int n, const int32_t* order, const int16_t* lev) {
  int nnz = 0;
  for (int i = 0; i < n * n; i++) nnz += lev[i] != 0;
  put_bit(w, nnz > 0);
  if (nnz == 0) return;
  put_ue(w, (uint32_t)(nnz - 1));
  int run = 0;
  for (int i = 0; i < n * n; i++) {
    int16_t v = lev[order[i]];
    if (v == 0) {
      run++;
      continue;
    }
    put_ue(w, (uint32_t)run);
    put_se(w, v);
    run = 0;
  }
}

static void get_block(bit_reader* r, int n, const int32_t* order, int16_t* lev) {
  if (!get_bit(r)) return;
  int nnz = (int)get_ue(r) + 1;
  int p = -1;
  for (int k = 0; k < nnz && !r->overrun; k++) {
    p += (int)get_ue(r) + 1;
    int32_t v = get_se(r);
    if (p >= n * n) {
      r->overrun = 1;
      break;
    }
    lev[order[p]] = (int16_t)v;
  }
}

uint64_t xvo_bitstream_bits(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                            int64_t Wb, int imodes, const uint8_t* splits,
                            const int16_t* levels, const int8_t* mvs) {
  stream_shape sh;
  shape_init(&sh, N, G, T, gop, Hb, Wb, imodes);
  int h = N / 2;
  uint64_t bits = 0;
  for (int64_t f = 0; f < G * T; f++) {
    int intra = (f % T) % gop == 0;
    const int8_t* fm = frame_mvs(&sh, mvs, f, splits != NULL);
    const uint8_t* fs = splits ? splits + f * Hb * Wb : NULL;
    for (int64_t by = 0; by < Hb; by++) {
      int pmx = 0, pmy = 0;
      for (int64_t bx = 0; bx < Wb; bx++) {
        if (intra) {
          bits += imodes ? 1 : 0;
        } else if (fs) {
          bits += split_vector_unit(&sh, fm, fs[by * Wb + bx], bx, by, NULL);
        } else {
          const int8_t* mv = fm + (by * Wb + bx) * 2;
          bits += xvo_mv_bits(mv[0], mv[1], pmx, pmy);
          pmx = mv[0];
          pmy = mv[1];
        }
      }
    }
    for (int64_t i = 0; i < 3 * Hb * Wb; i++) {
      const int16_t* lev = levels + (f * 3 * Hb * Wb + i) * N * N;
      if (fs && !intra && fs[i % (Hb * Wb)]) {
        for (int q = 0; q < 4; q++) bits += xvo_coef_bits(h, lev + q * h * h);
      } else {
        bits += xvo_coef_bits(N, lev);
      }
    }
  }
  return bits;
}

int xvo_write_bitstream(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                        int64_t Wb, int imodes, const uint8_t* splits,
                        const int16_t* levels, const int8_t* mvs, uint8_t* out,
                        uint64_t out_bytes, uint64_t* index) {
  stream_shape sh;
  shape_init(&sh, N, G, T, gop, Hb, Wb, imodes);
  int h = N / 2;
  memset(out, 0, out_bytes);
  bit_writer w = {out, out_bytes * 8, 0, 0};
  int64_t seg = 0;
  for (int64_t f = 0; f < G * T; f++) {
    int intra = (f % T) % gop == 0;
    const int8_t* fm = frame_mvs(&sh, mvs, f, splits != NULL);
    const uint8_t* fs = splits ? splits + f * Hb * Wb : NULL;
    for (int64_t by = 0; by < Hb; by++) {
      index[seg++] = w.pos;
      int pmx = 0, pmy = 0;
      for (int64_t bx = 0; bx < Wb; bx++) {
        if (intra) {
          /* the mode is the vector's first byte */
          if (imodes) put_bit(&w, fm[(by * Wb + bx) * 2] != 0);
        } else if (fs) {
          split_vector_unit(&sh, fm, fs[by * Wb + bx], bx, by, &w);
        } else {
          const int8_t* mv = fm + (by * Wb + bx) * 2;
          put_se(&w, mv[0] - pmx);
          put_se(&w, mv[1] - pmy);
          pmx = mv[0];
          pmy = mv[1];
        }
      }
    }
    for (int c = 0; c < 3; c++)
      for (int64_t by = 0; by < Hb; by++) {
        index[seg++] = w.pos;
        for (int64_t bx = 0; bx < Wb; bx++) {
          const int16_t* lev = levels + ((f * 3 + c) * Hb * Wb + by * Wb + bx) * N * N;
          if (fs && !intra && fs[by * Wb + bx]) {
            for (int q = 0; q < 4; q++) put_block(&w, h, sh.order_h, lev + q * h * h);
          } else {
            put_block(&w, N, sh.order, lev);
          }
        }
      }
  }
  return w.overflow ? -1 : 0;
}

/* Sequential parse of the whole stream; index (may be NULL) receives the
 * segment offsets met on the way.  Levels not listed are zero; I frames get
 * the vector (0,0), or (mode, 0) with imodes; with splits, the split flags
 * of P blocks are read into splits (I blocks: 0) and whole blocks repeat
 * their vector over their four cells. */
int xvo_read_bitstream(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                       int64_t Wb, int imodes, uint8_t* splits, const uint8_t* in,
                       uint64_t bits, int16_t* levels, int8_t* mvs, uint64_t* index) {
  stream_shape sh;
  shape_init(&sh, N, G, T, gop, Hb, Wb, imodes);
  int h = N / 2;
  int64_t Wu = 2 * Wb;
  bit_reader r = {in, bits, 0, 0};
  int64_t seg = 0;
  memset(levels, 0, (size_t)(G * T * 3 * Hb * Wb * N * N) * sizeof(int16_t));
  for (int64_t f = 0; f < G * T; f++) {
    int intra = (f % T) % gop == 0;
    int8_t* fm = (int8_t*)frame_mvs(&sh, mvs, f, splits != NULL);
    uint8_t* fs = splits ? splits + f * Hb * Wb : NULL;
    for (int64_t by = 0; by < Hb; by++) {
      if (index) index[seg] = r.pos;
      seg++;
      int pmx = 0, pmy = 0;
      for (int64_t bx = 0; bx < Wb; bx++) {
        if (fs) {
          int split = intra ? 0 : get_bit(&r);
          fs[by * Wb + bx] = (uint8_t)split;
          for (int i = 0; i < 4; i++) {
            int64_t u = (2 * by + (i >> 1)) * Wu + 2 * bx + (i & 1);
            int mx = 0, my = 0;
            if (!intra && (split || i == 0)) {
              int64_t xu = 2 * bx + (i & 1), yu = 2 * by + (i >> 1);
              int qx = xu > 0 ? fm[2 * (yu * Wu + xu - 1)] : 0;
              int qy = xu > 0 ? fm[2 * (yu * Wu + xu - 1) + 1] : 0;
              mx = qx + get_se(&r);
              my = qy + get_se(&r);
            } else if (!intra) {
              mx = fm[2 * ((2 * by) * Wu + 2 * bx)];
              my = fm[2 * ((2 * by) * Wu + 2 * bx) + 1];
            }
            fm[2 * u] = (int8_t)mx;
            fm[2 * u + 1] = (int8_t)my;
          }
          continue;
        }
        int8_t* mv = fm + (by * Wb + bx) * 2;
        int dx = 0, dy = 0;
        if (!intra) {
          dx = pmx + get_se(&r);
          dy = pmy + get_se(&r);
        } else if (imodes) {
          dx = get_bit(&r);
        }
        mv[0] = (int8_t)dx;
        mv[1] = (int8_t)dy;
        pmx = dx;
        pmy = dy;
      }
    }
    for (int c = 0; c < 3; c++)
      for (int64_t by = 0; by < Hb; by++) {
        if (index) index[seg] = r.pos;
        seg++;
        for (int64_t bx = 0; bx < Wb; bx++) {
          int16_t* lev = levels + ((f * 3 + c) * Hb * Wb + by * Wb + bx) * N * N;
          if (fs && fs[by * Wb + bx]) {
            for (int q = 0; q < 4; q++) get_block(&r, h, sh.order_h, lev + q * h * h);
          } else {
            get_block(&r, N, sh.order, lev);
          }
        }
      }
  }
  if (r.overrun) return -1;
  return r.pos == bits ? 0 : -2;
}

/* ------------------------------------------------------------------------- */
/* Full-search integer-pel motion estimation (paper silent; reading: one      */
/* vector per N x N block shared by the group's 3 channels, SAD summed over   */
/* the group's channels that carry a real band (c < nch; padding channels do  */
/* not steer the search), candidates (dx,dy) in [-R,R]^2 with the displaced block      */
/* fully inside the padded frame, lexicographic minimum of                   */
/* (SAD, |dx|+|dy|, dy, dx)).  cur and ref are [3][Hp][Wp].                   */
/* ------------------------------------------------------------------------- */
void xvo_motion_search(const uint16_t* cur, const uint16_t* ref, int64_t Hp,
                       int64_t Wp, int N, int R, int nch, int64_t bx, int64_t by,
                       int32_t* best_dx, int32_t* best_dy, uint32_t* best_sad) {
  int64_t x0 = bx * N, y0 = by * N;
  uint32_t bs = UINT32_MAX;
  int bl1 = 0, bdx = 0, bdy = 0;
  for (int dy = -R; dy <= R; dy++) {
    for (int dx = -R; dx <= R; dx++) {
      if (x0 + dx < 0 || x0 + dx + N > Wp || y0 + dy < 0 || y0 + dy + N > Hp)
        continue;
      uint32_t sad = 0;
      for (int c = 0; c < nch; c++)
        for (int i = 0; i < N; i++)
          for (int j = 0; j < N; j++) {
            int a = cur[(c * Hp + y0 + i) * Wp + x0 + j];
            int b = ref[(c * Hp + y0 + dy + i) * Wp + x0 + dx + j];
            sad += (uint32_t)(a > b ? a - b : b - a);
          }
      int l1 = abs(dx) + abs(dy);
      /* raster order (dy, then dx) makes the first strict improvement the
       * lexicographic minimum of (SAD, L1, dy, dx) */
      if (sad < bs || (sad == bs && l1 < bl1)) {
        bs = sad;
        bl1 = l1;
        bdx = dx;
        bdy = dy;
      }
    }
  }
  *best_dx = bdx;
  *best_dy = bdy;
  *best_sad = bs;
}

/* ------------------------------------------------------------------------- */
/* Quarter-sample motion (one of the HEVC coding tools the paper's x265      */
/* presets use, Appendix table of codec configurations; the paper describes  */
/* none of its internals).  Reading: vectors in quarter samples; the         */
/* prediction at a fractional position is the ITU-T H.265 luma fractional    */
/* sample interpolation (clause 8.5.3.3.3.1: 8-tap filters, intermediate     */
/* shifts shift1 = B - 8, shift2 = 6, shift3 = 14 - B, reference coordinates */
/* clamped to the picture) followed by the default weighted sample           */
/* prediction of a single reference (clause 8.5.3.3.4.2: round and shift by  */
/* 14 - B, clip to [0, 2^B - 1]).  The three planes of a frame are           */
/* independent bands (4:4:4, no colour transform), so every plane uses the   */
/* luma filters.                                                             */
/* ------------------------------------------------------------------------- */

/* Filter coefficient fL[frac][tap] of H.265 (frac in quarter samples 0..3;  */
/* tap 0..7 weighs the reference sample at integer offset tap - 3).          */
int xvo_luma_filter(int frac, int tap) {
  static const int f[4][8] = {{0, 0, 0, 64, 0, 0, 0, 0},
                              {-1, 4, -10, 58, 17, -5, 1, 0},
                              {-1, 4, -11, 40, 40, -11, 4, -1},
                              {0, 1, -5, 17, 58, -10, 4, -1}};
  return f[frac][tap];
}

static int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : v > hi ? hi : v; }

static int32_t ref_at(const uint16_t* plane, int64_t Hp, int64_t Wp, int64_t x, int64_t y) {
  return plane[clamp64(y, 0, Hp - 1) * Wp + clamp64(x, 0, Wp - 1)];
}

/* Predicted sample at the quarter-sample position (xq, yq) of a plane. */
int32_t xvo_interp_sample(const uint16_t* plane, int64_t Hp, int64_t Wp, int B,
                          int64_t xq, int64_t yq) {
  const int64_t xi = xq >> 2, yi = yq >> 2; /* floor: arithmetic shifts */
  const int fx = (int)(xq & 3), fy = (int)(yq & 3);
  const int shift1 = B - 8, shift2 = 6, shift3 = 14 - B;
  int32_t pred;
  if (fx == 0 && fy == 0) {
    pred = ref_at(plane, Hp, Wp, xi, yi) << shift3;
  } else if (fy == 0) {
    int32_t acc = 0;
    for (int i = 0; i < 8; i++) acc += xvo_luma_filter(fx, i) * ref_at(plane, Hp, Wp, xi + i - 3, yi);
    pred = acc >> shift1;
  } else if (fx == 0) {
    int32_t acc = 0;
    for (int i = 0; i < 8; i++) acc += xvo_luma_filter(fy, i) * ref_at(plane, Hp, Wp, xi, yi + i - 3);
    pred = acc >> shift1;
  } else {
    int32_t tmp[8];
    for (int n = 0; n < 8; n++) {
      int32_t acc = 0;
      for (int i = 0; i < 8; i++)
        acc += xvo_luma_filter(fx, i) * ref_at(plane, Hp, Wp, xi + i - 3, yi + n - 3);
      tmp[n] = acc >> shift1;
    }
    int32_t acc = 0;
    for (int i = 0; i < 8; i++) acc += xvo_luma_filter(fy, i) * tmp[i];
    pred = acc >> shift2;
  }
  /* default weighted sample prediction, one reference */
  const int shw = 14 - B;
  int32_t v = (pred + (1 << (shw - 1))) >> shw;
  const int32_t L = (1 << B) - 1;
  return v < 0 ? 0 : v > L ? L : v;
}

/* SAD of the block (bx, by) against the prediction at vector (mx, my), in   */
/* quarter samples, over the group's real channels.                          */
static uint32_t subpel_sad(const uint16_t* cur, const uint16_t* ref, int64_t Hp, int64_t Wp,
                           int N, int B, int nch, int64_t bx, int64_t by, int mx, int my) {
  const int64_t x0 = bx * N, y0 = by * N;
  uint32_t sad = 0;
  for (int c = 0; c < nch; c++)
    for (int i = 0; i < N; i++)
      for (int j = 0; j < N; j++) {
        int a = cur[(c * Hp + y0 + i) * Wp + x0 + j];
        int b = xvo_interp_sample(ref + c * Hp * Wp, Hp, Wp, B, 4 * (x0 + j) + mx,
                                  4 * (y0 + i) + my);
        sad += (uint32_t)(a > b ? a - b : b - a);
      }
  return sad;
}

/* Refinement of an integer vector (dx, dy) (reading, as HEVC encoders do):  */
/* the best of the centre and its 8 half-sample neighbours, then the best of */
/* that and its 8 quarter-sample neighbours, each by the lexicographic       */
/* minimum of (SAD, |mx| + |my|, my, mx) with the vector in quarter samples. */
void xvo_subpel_refine(const uint16_t* cur, const uint16_t* ref, int64_t Hp,
                       int64_t Wp, int N, int B, int nch, int64_t bx, int64_t by,
                       int dx, int dy, int32_t* mvx, int32_t* mvy,
                       uint32_t* best_sad) {
  int cx = 4 * dx, cy = 4 * dy;
  uint32_t bs = 0;
  for (int step = 2; step >= 1; step--) {
    int bx_ = cx, by_ = cy;
    bs = UINT32_MAX;
    int bl1 = 0;
    for (int oy = -step; oy <= step; oy += step)
      for (int ox = -step; ox <= step; ox += step) {
        const int mx = cx + ox, my = cy + oy;
        const uint32_t sad = subpel_sad(cur, ref, Hp, Wp, N, B, nch, bx, by, mx, my);
        const int l1 = abs(mx) + abs(my);
        int better = sad < bs;
        if (sad == bs) {
          if (l1 != bl1) better = l1 < bl1;
          else if (my != by_) better = my < by_;
          else better = mx < bx_;
        }
        if (better) {
          bs = sad;
          bl1 = l1;
          bx_ = mx;
          by_ = my;
        }
      }
    cx = bx_;
    cy = by_;
  }
  *mvx = cx;
  *mvy = cy;
  *best_sad = bs;
}

/* ------------------------------------------------------------------------- */
/* Coding of one closed group of pictures of one band group (paper silent on */
/* codec internals; reading: an I picture predicted from the constant         */
/* 2^(B-1), then P pictures predicted from the reconstruction of the picture  */
/* just before, closed loop).                                                 */
/* Layouts (len frames of this GOP, local index f):                           */
/*   frames, recon : [len][3][Hp][Wp] u16                                     */
/*   levels        : [len][3][Hb][Wb][N][N] i16                               */
/*   mvs           : [len][Hb][Wb][2] i8 (dx, dy); zero for the I picture     */
/*   coef_bits     : [len][3][Hb][Wb] u32                                     */
/*   mv_bits       : [len][Hb][Wb] u32                                        */
/*   sse, nvalid   : [3] u64, over valid pixels of the coded GOP              */
/* ------------------------------------------------------------------------- */
/* Intra prediction of I pictures (ITU-T H.265 8.4.4.2).  The paper names    */
/* no intra modes; the reading is: the two non-directional H.265 modes,      */
/* planar (0) and DC (1); blocks coded in raster order at the fixed size N,  */
/* so a sample is available when it lies in the padded picture and in a      */
/* block before the current one in raster order; every channel treated as   */
/* H.265 luma (DC edge filter for N < 32); strong smoothing of 32 x 32       */
/* references on, as in x265's default; one mode per block for the group's   */
/* three channels, the one with the smaller SAD against the source over the  */
/* real channels, planar on a tie.                                           */
/*                                                                           */
/* refs holds the 4N + 1 reference samples in the order of the substitution  */
/* scan (H.265 8.4.4.2.2): refs[i] = p[-1][2N-1-i] for i < 2N, refs[2N] =    */
/* p[-1][-1], refs[2N+1+x] = p[x][-1].                                       */
/* ------------------------------------------------------------------------- */
void xvo_intra_refs(const uint16_t* rec_plane, int64_t Hp, int64_t Wp, int N, int B,
                    int64_t bx, int64_t by, int32_t* refs) {
  int64_t Wb = Wp / N, cur = by * Wb + bx;
  int64_t x0 = bx * N, y0 = by * N;
  int avail[4 * 32 + 1];
  int n = 4 * N + 1, any = 0;
  for (int i = 0; i < n; i++) {
    int64_t x, y;
    if (i < 2 * N) {
      x = x0 - 1;
      y = y0 + (2 * N - 1 - i);
    } else if (i == 2 * N) {
      x = x0 - 1;
      y = y0 - 1;
    } else {
      x = x0 + (i - 2 * N - 1);
      y = y0 - 1;
    }
    int in = x >= 0 && y >= 0 && x < Wp && y < Hp;
    avail[i] = in && (y / N) * Wb + x / N < cur;
    refs[i] = avail[i] ? rec_plane[y * Wp + x] : 0;
    any |= avail[i];
  }
  if (!any) {
    for (int i = 0; i < n; i++) refs[i] = 1 << (B - 1);
    return;
  }
  /* the first entry takes the first available sample of the scan; every
   * other unavailable entry takes the entry before it */
  if (!avail[0]) {
    int k = 1;
    while (!avail[k]) k++;
    refs[0] = refs[k];
  }
  for (int i = 1; i < n; i++)
    if (!avail[i]) refs[i] = refs[i - 1];
}

/* p[-1][y] and p[x][-1] of a reference array in scan order */
#define XVO_LEFT(a, y) ((a)[2 * N - 1 - (y)])
#define XVO_TOP(a, x) ((a)[2 * N + 1 + (x)])

void xvo_intra_predict(const int32_t* refs, int N, int mode, int B, int32_t* pred) {
  int k = ilog2(N);
  if (mode == 0) {
    /* planar: references smoothed first for N >= 8 (H.265 8.4.4.2.3) */
    int32_t f[4 * 32 + 1];
    int n = 4 * N + 1;
    for (int i = 0; i < n; i++) f[i] = refs[i];
    if (N >= 8) {
      int thr = 1 << (B - 5);
      int corner = XVO_LEFT(refs, -1);
      int strong = N == 32 &&
                   abs(corner + XVO_TOP(refs, 2 * N - 1) - 2 * XVO_TOP(refs, N - 1)) < thr &&
                   abs(corner + XVO_LEFT(refs, 2 * N - 1) - 2 * XVO_LEFT(refs, N - 1)) < thr;
      if (strong) {
        /* bilinear between the corner and the far ends of each edge */
        for (int y = 0; y < 2 * N - 1; y++)
          XVO_LEFT(f, y) = ((63 - y) * corner + (y + 1) * XVO_LEFT(refs, 2 * N - 1) + 32) >> 6;
        for (int x = 0; x < 2 * N - 1; x++)
          XVO_TOP(f, x) = ((63 - x) * corner + (x + 1) * XVO_TOP(refs, 2 * N - 1) + 32) >> 6;
      } else {
        /* [1 2 1] along the scan; both ends kept */
        for (int i = 1; i < n - 1; i++) f[i] = (refs[i - 1] + 2 * refs[i] + refs[i + 1] + 2) >> 2;
      }
    }
    for (int y = 0; y < N; y++)
      for (int x = 0; x < N; x++)
        pred[y * N + x] = ((N - 1 - x) * XVO_LEFT(f, y) + (x + 1) * XVO_TOP(f, N) +
                           (N - 1 - y) * XVO_TOP(f, x) + (y + 1) * XVO_LEFT(f, N) + N) >>
                          (k + 1);
  } else {
    /* DC from the unsmoothed references, edges filtered for N < 32 */
    int sum = N;
    for (int i = 0; i < N; i++) sum += XVO_TOP(refs, i) + XVO_LEFT(refs, i);
    int dc = sum >> (k + 1);
    for (int i = 0; i < N * N; i++) pred[i] = dc;
    if (N < 32) {
      pred[0] = (XVO_LEFT(refs, 0) + 2 * dc + XVO_TOP(refs, 0) + 2) >> 2;
      for (int x = 1; x < N; x++) pred[x] = (XVO_TOP(refs, x) + 3 * dc + 2) >> 2;
      for (int y = 1; y < N; y++) pred[y * N] = (XVO_LEFT(refs, y) + 3 * dc + 2) >> 2;
    }
  }
}

#undef XVO_LEFT
#undef XVO_TOP

/* Mode of an I block (reading above) from the current frame and the        */
/* partly reconstructed one; preds receives the chosen mode's prediction of  */
/* each channel, [3][N][N].                                                  */
static int intra_choose(const uint16_t* cur, const uint16_t* rec, int64_t Hp, int64_t Wp,
                        int N, int B, int nch, int64_t bx, int64_t by, int32_t* preds) {
  int64_t plane = Hp * Wp;
  int32_t refs[4 * 32 + 1], cand[2][3][32 * 32];
  uint64_t cost[2] = {0, 0};
  for (int c = 0; c < 3; c++) {
    xvo_intra_refs(rec + c * plane, Hp, Wp, N, B, bx, by, refs);
    for (int m = 0; m < 2; m++) {
      xvo_intra_predict(refs, N, m, B, cand[m][c]);
      if (c >= nch) continue;
      for (int y = 0; y < N; y++)
        for (int x = 0; x < N; x++) {
          int d = (int)cur[c * plane + (by * N + y) * Wp + bx * N + x] - cand[m][c][y * N + x];
          cost[m] += (uint64_t)(d < 0 ? -d : d);
        }
    }
  }
  int mode = cost[1] < cost[0] ? 1 : 0;
  for (int c = 0; c < 3; c++) memcpy(preds + c * N * N, cand[mode][c], sizeof(int32_t) * N * N);
  return mode;
}

/* Prediction of sample (x, y) of a P block from the reference plane: the    */
/* displaced sample for integer vectors, the interpolated one for quarter-    */
/* sample vectors.                                                            */
static int predict_sample(const xvo_params* p, const uint16_t* ref_plane, int64_t Hp,
                          int64_t Wp, int64_t x, int64_t y, int dx, int dy) {
  if (p->qpel)
    return xvo_interp_sample(ref_plane, Hp, Wp, p->bit_depth, 4 * x + dx, 4 * y + dy);
  return ref_plane[(y + dy) * Wp + x + dx];
}

static void code_block(const xvo_params* p, int N, int intra, const int32_t* ipred,
                       const uint16_t* cur, const uint16_t* pred_plane, int64_t Hp,
                       int64_t Wp, int64_t x0, int64_t y0, int dx, int dy, int16_t* lev_out,
                       uint16_t* rec_plane, uint32_t* bits_out) {
  int B = p->bit_depth;
  int L = (1 << B) - 1;
  int32_t r[32 * 32] = {0}, C[32 * 32], d[32 * 32], rr[32 * 32], pred[32 * 32];
  for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
      int pv = ipred   ? ipred[i * N + j]
               : intra ? (1 << (B - 1))
                       : predict_sample(p, pred_plane, Hp, Wp, x0 + j, y0 + i, dx, dy);
      pred[i * N + j] = pv;
      r[i * N + j] = (int32_t)cur[(y0 + i) * Wp + x0 + j] - pv;
    }
  xvo_forward_transform(N, B, r, C);
  xvo_quantize(N, B, p->qp, intra, C, lev_out);
  *bits_out = xvo_coef_bits(N, lev_out);
  xvo_dequantize(N, B, p->qp, lev_out, d);
  xvo_inverse_transform(N, B, d, rr);
  for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
      int v = pred[i * N + j] + rr[i * N + j];
      if (v < 0) v = 0;
      if (v > L) v = L;
      rec_plane[(y0 + i) * Wp + x0 + j] = (uint16_t)v;
    }
}

/* Adaptive block size of P pictures (XVO split).  The paper's x265 presets  */
/* choose block sizes per coding tree; its text gives no rule.  Reading: a   */
/* block of the configured size N (the tree's root) is either coded whole    */
/* or split once into four N/2 blocks in z-order, each with its own vector   */
/* and transform, whichever has the smaller cost J = 16 SAD + lambda16 bits, */
/* where SAD is each block's full-search SAD (the integer search above) and  */
/* bits the Exp-Golomb length of its vector against the zero vector (the     */
/* coded predictors depend on the choices to the left, so the choice does    */
/* not); a tie keeps the block whole.  lambda = sqrt(0.57 2^((qP-12)/3)),    */
/* the motion-cost multiplier of the H.265 reference encoder, in 1/16 SAD    */
/* units.  I pictures are never split.  Vectors live on the N/2 grid (a      */
/* whole block repeats its vector over its four cells); a block's vector     */
/* bits are one split flag plus, per coded vector in z-order, se of the      */
/* difference to the vector of the N/2 cell to the left of its top-left      */
/* cell ((0,0) in cell column 0).  A split block's levels are its four N/2   */
/* blocks' levels one after another in z-order.                              */
int32_t xvo_split_lambda(int qp, int B) {
  int qP = qp + 6 * (B - 8);
  return (int32_t)floor(16.0 * sqrt(0.57 * pow(2.0, (qP - 12) / 3.0)) + 0.5);
}

int xvo_split_choose(uint32_t sad_whole, int vx, int vy, const uint32_t* sads,
                     const int32_t* ux, const int32_t* uy, int32_t lam16) {
  uint64_t lam = (uint64_t)lam16;
  uint64_t j_whole = 16 * (uint64_t)sad_whole + lam * (uint64_t)xvo_mv_bits(vx, vy, 0, 0);
  uint64_t j_split = 0;
  for (int i = 0; i < 4; i++)
    j_split += 16 * (uint64_t)sads[i] + lam * (uint64_t)xvo_mv_bits(ux[i], uy[i], 0, 0);
  return j_split < j_whole;
}

static void encode_p_split(const xvo_params* p, const uint16_t* cur, const uint16_t* ref,
                           int64_t Hp, int64_t Wp, int nch, int16_t* levels, int8_t* mvu,
                           uint8_t* splits, uint32_t* coef_bits, uint32_t* mv_bits,
                           uint16_t* rec) {
  int N = p->block, h = N / 2, R = p->search_range;
  int64_t Hb = Hp / N, Wb = Wp / N, Wu = 2 * Wb, plane = Hp * Wp;
  int32_t lam = xvo_split_lambda(p->qp, p->bit_depth);
  for (int64_t by = 0; by < Hb; by++)
    for (int64_t bx = 0; bx < Wb; bx++) {
      int64_t ci = by * Wb + bx;
      int32_t vx, vy, ux[4], uy[4];
      uint32_t sad, usad[4];
      xvo_motion_search(cur, ref, Hp, Wp, N, R, nch, bx, by, &vx, &vy, &sad);
      for (int i = 0; i < 4; i++)
        xvo_motion_search(cur, ref, Hp, Wp, h, R, nch, 2 * bx + (i & 1), 2 * by + (i >> 1),
                          &ux[i], &uy[i], &usad[i]);
      int split = xvo_split_choose(sad, vx, vy, usad, ux, uy, lam);
      splits[ci] = (uint8_t)split;
      for (int i = 0; i < 4; i++) {
        int64_t u = (2 * by + (i >> 1)) * Wu + 2 * bx + (i & 1);
        mvu[2 * u] = (int8_t)(split ? ux[i] : vx);
        mvu[2 * u + 1] = (int8_t)(split ? uy[i] : vy);
      }
      uint32_t mb = 1; /* the split flag */
      for (int i = 0; i < (split ? 4 : 1); i++) {
        int64_t xu = 2 * bx + (i & 1), yu = 2 * by + (i >> 1);
        int pmx = 0, pmy = 0;
        if (xu > 0) {
          pmx = mvu[2 * (yu * Wu + xu - 1)];
          pmy = mvu[2 * (yu * Wu + xu - 1) + 1];
        }
        mb += xvo_mv_bits(mvu[2 * (yu * Wu + xu)], mvu[2 * (yu * Wu + xu) + 1], pmx, pmy);
      }
      mv_bits[ci] = mb;
      for (int c = 0; c < 3; c++) {
        int16_t* lev = levels + (c * Hb * Wb + ci) * N * N;
        uint32_t* cb = &coef_bits[c * Hb * Wb + ci];
        if (!split) {
          code_block(p, N, 0, NULL, cur + c * plane, ref + c * plane, Hp, Wp, bx * N, by * N,
                     vx, vy, lev, rec + c * plane, cb);
          continue;
        }
        *cb = 0;
        for (int i = 0; i < 4; i++) {
          uint32_t b;
          code_block(p, h, 0, NULL, cur + c * plane, ref + c * plane, Hp, Wp,
                     bx * N + (i & 1) * h, by * N + (i >> 1) * h, ux[i], uy[i], lev + i * h * h,
                     rec + c * plane, &b);
          *cb += b;
        }
      }
    }
}

int xvo_encode_gop(const void* data, int dtype, int64_t T, int64_t H,
                   int64_t W, int64_t Bn, const double* mn, const double* mx,
                   const xvo_params* p, int64_t g, int64_t t0, int64_t len,
                   uint16_t* frames, int16_t* levels, int8_t* mvs,
                   uint16_t* recon, uint32_t* coef_bits, uint32_t* mv_bits,
                   uint8_t* splits, uint64_t* sse, uint64_t* nvalid) {
  if (xvo_check_params(p) != 0) return -1;
  int N = p->block;
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  int64_t Hb = Hp / N, Wb = Wp / N;
  int64_t plane = Hp * Wp, fsz = 3 * plane;
  int64_t mvf = (p->split ? 4 : 1) * Hb * Wb; /* vectors per frame */
  int nch = (int)(Bn - 3 * g < 3 ? Bn - 3 * g : 3);
  uint8_t* valid = (uint8_t*)malloc((size_t)fsz);
  if (!valid) return -2;
  for (int c = 0; c < 3; c++) { sse[c] = 0; nvalid[c] = 0; }
  for (int64_t f = 0; f < len; f++) {
    int64_t t = t0 + f;
    uint16_t* cur = frames + f * fsz;
    uint16_t* rec = recon + f * fsz;
    const uint16_t* ref = f > 0 ? recon + (f - 1) * fsz : NULL;
    int intra = (f == 0);
    xvo_make_frame(data, dtype, T, H, W, Bn, mn, mx, p, g, t, Hp, Wp, cur, valid);
    if (p->split) {
      memset(mvs + f * mvf * 2, 0, (size_t)mvf * 2);
      memset(splits + f * Hb * Wb, 0, (size_t)(Hb * Wb));
    }
    if (!intra && p->split) {
      encode_p_split(p, cur, ref, Hp, Wp, nch, levels + f * fsz, mvs + f * mvf * 2,
                     splits + f * Hb * Wb, coef_bits + f * 3 * Hb * Wb, mv_bits + f * Hb * Wb,
                     rec);
    } else
    for (int64_t by = 0; by < Hb; by++) {
      int pmx = 0, pmy = 0;
      for (int64_t bx = 0; bx < Wb; bx++) {
        int32_t dx = 0, dy = 0;
        uint32_t sad = 0;
        int64_t bi = by * Wb + bx;
        int32_t ipred[3 * 32 * 32];
        int use_ipred = intra && p->intra;
        if (use_ipred) /* the mode travels in the vector's first byte */
          dx = intra_choose(cur, rec, Hp, Wp, N, p->bit_depth, nch, bx, by, ipred);
        if (!intra) {
          xvo_motion_search(cur, ref, Hp, Wp, N, p->search_range, nch, bx, by, &dx,
                            &dy, &sad);
          if (p->qpel) {
            int32_t qx, qy;
            xvo_subpel_refine(cur, ref, Hp, Wp, N, p->bit_depth, nch, bx, by, dx, dy,
                              &qx, &qy, &sad);
            dx = qx;
            dy = qy;
          }
        }
        if (!p->split) { /* (split: I cells stay zero) */
          mvs[(f * Hb * Wb + bi) * 2 + 0] = (int8_t)dx;
          mvs[(f * Hb * Wb + bi) * 2 + 1] = (int8_t)dy;
        }
        mv_bits[f * Hb * Wb + bi] =
            intra ? (uint32_t)p->intra /* one mode bit */ : xvo_mv_bits(dx, dy, pmx, pmy);
        pmx = intra ? 0 : dx;
        pmy = intra ? 0 : dy;
        for (int c = 0; c < 3; c++) {
          int16_t* lev = levels + ((f * 3 + c) * Hb * Wb + bi) * N * N;
          code_block(p, N, intra, use_ipred ? ipred + c * N * N : NULL, cur + c * plane,
                     ref ? ref + c * plane : NULL,
                     Hp, Wp, bx * N, by * N, dx, dy, lev, rec + c * plane,
                     &coef_bits[(f * 3 + c) * Hb * Wb + bi]);
        }
      }
    }
    for (int c = 0; c < 3; c++)
      for (int64_t o = 0; o < plane; o++) {
        if (!valid[c * plane + o]) continue;
        int64_t e = (int64_t)cur[c * plane + o] - (int64_t)rec[c * plane + o];
        sse[c] += (uint64_t)(e * e);
        nvalid[c] += 1;
      }
  }
  free(valid);
  return 0;
}

/* Decoding of one GOP from its levels and vectors: the same prediction,
 * dequantisation and inverse transform as the encoder's reconstruction. */
/* Reconstruction of one N x N P block at (x0, y0) from its levels. */
static void decode_block(const xvo_params* p, int N, const int16_t* lev,
                         const uint16_t* ref_plane, int64_t Hp, int64_t Wp, int64_t x0,
                         int64_t y0, int dx, int dy, uint16_t* rec_plane) {
  int B = p->bit_depth, L = (1 << B) - 1;
  int32_t d[32 * 32], rr[32 * 32];
  xvo_dequantize(N, B, p->qp, lev, d);
  xvo_inverse_transform(N, B, d, rr);
  for (int i = 0; i < N; i++)
    for (int j = 0; j < N; j++) {
      int v = predict_sample(p, ref_plane, Hp, Wp, x0 + j, y0 + i, dx, dy) + rr[i * N + j];
      if (v < 0) v = 0;
      if (v > L) v = L;
      rec_plane[(y0 + i) * Wp + x0 + j] = (uint16_t)v;
    }
}

int xvo_decode_gop(const xvo_params* p, int64_t H, int64_t W, int64_t len,
                   const int16_t* levels, const int8_t* mvs, const uint8_t* splits,
                   uint16_t* recon) {
  if (xvo_check_params(p) != 0) return -1;
  int N = p->block, B = p->bit_depth, L = (1 << B) - 1;
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  int64_t Hb = Hp / N, Wb = Wp / N, plane = Hp * Wp, fsz = 3 * plane;
  int32_t d[32 * 32], rr[32 * 32];
  for (int64_t f = 0; f < len; f++) {
    uint16_t* rec = recon + f * fsz;
    const uint16_t* ref = f > 0 ? recon + (f - 1) * fsz : NULL;
    if (f > 0 && p->split) {
      /* whole blocks take the vector of their top-left cell */
      int h = N / 2;
      int64_t Wu = 2 * Wb;
      const int8_t* mvu = mvs + f * 4 * Hb * Wb * 2;
      for (int64_t by = 0; by < Hb; by++)
        for (int64_t bx = 0; bx < Wb; bx++) {
          int64_t ci = by * Wb + bx;
          int split = splits[f * Hb * Wb + ci] != 0;
          for (int c = 0; c < 3; c++) {
            const int16_t* lev = levels + ((f * 3 + c) * Hb * Wb + ci) * N * N;
            for (int i = 0; i < (split ? 4 : 1); i++) {
              int64_t u = (2 * by + (i >> 1)) * Wu + 2 * bx + (i & 1);
              decode_block(p, split ? h : N, lev + i * h * h, ref + c * plane, Hp, Wp,
                           bx * N + (i & 1) * h, by * N + (i >> 1) * h, mvu[2 * u],
                           mvu[2 * u + 1], rec + c * plane);
            }
          }
        }
      continue;
    }
    for (int64_t by = 0; by < Hb; by++)
      for (int64_t bx = 0; bx < Wb; bx++) {
        int64_t bi = by * Wb + bx;
        int dx = p->split ? 0 : mvs[(f * Hb * Wb + bi) * 2 + 0];
        int dy = p->split ? 0 : mvs[(f * Hb * Wb + bi) * 2 + 1];
        for (int c = 0; c < 3; c++) {
          const int16_t* lev = levels + ((f * 3 + c) * Hb * Wb + bi) * N * N;
          int32_t ipred[32 * 32], refs[4 * 32 + 1];
          if (f == 0 && p->intra) {  /* mode in the vector's first byte */
            xvo_intra_refs(rec + c * plane, Hp, Wp, N, B, bx, by, refs);
            xvo_intra_predict(refs, N, dx, B, ipred);
          }
          xvo_dequantize(N, B, p->qp, lev, d);
          xvo_inverse_transform(N, B, d, rr);
          for (int i = 0; i < N; i++)
            for (int j = 0; j < N; j++) {
              int64_t y = by * N + i, x = bx * N + j;
              int pv = f == 0 ? (p->intra ? ipred[i * N + j] : (1 << (B - 1)))
                              : predict_sample(p, ref + c * plane, Hp, Wp, x, y, dx, dy);
              int v = pv + rr[i * N + j];
              if (v < 0) v = 0;
              if (v > L) v = L;
              rec[(c * Hp + y) * Wp + x] = (uint16_t)v;
            }
        }
      }
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Whole-cube drivers: every (group, GOP) unit is independent (closed GOPs),  */
/* so units run in parallel.  Full-cube layouts prepend [G][T] to the GOP     */
/* layouts above; sse and nvalid are per real band.                           */
/* ------------------------------------------------------------------------- */
int xvo_check_params(const xvo_params* p) {
  int N = p->block, B = p->bit_depth;
  if (!(N == 4 || N == 8 || N == 16 || N == 32)) return -1;
  if (B < 8 || B > 12) return -1;
  if (p->qp < -6 * (B - 8) || p->qp > 51) return -1;
  if (p->search_range < 0 || p->search_range > 64) return -1;
  if (p->qpel != 0 && p->qpel != 1) return -1;
  if (p->intra != 0 && p->intra != 1) return -1;
  if (p->split != 0 && p->split != 1) return -1;
  /* adaptive block size: N/2 >= 4, integer vectors, constant I prediction */
  if (p->split && (N < 8 || p->qpel || p->intra)) return -1;
  /* quarter-sample vectors reach 4R + 3, which must fit int8 */
  if (p->qpel && p->search_range > 31) return -1;
  if (p->gop < 1) return -1;
  if (p->pad_mode != XVO_PAD_ZERO && p->pad_mode != XVO_PAD_REPEAT) return -1;
  if (p->fill_mode != XVO_FILL_NEAREST && p->fill_mode != XVO_FILL_FORWARD) return -1;
  return 0;
}

int xvo_encode_cube(const void* data, int dtype, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, const xvo_params* p, double* mn,
                    double* mx, uint16_t* frames, int16_t* levels, int8_t* mvs,
                    uint16_t* recon, uint32_t* coef_bits, uint32_t* mv_bits,
                    uint8_t* splits, uint64_t* sse, uint64_t* nvalid) {
  if (xvo_check_params(p) != 0) return -1;
  int N = p->block;
  int64_t G = (Bn + 2) / 3;
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  int64_t Hb = Hp / N, Wb = Wp / N, fsz = 3 * Hp * Wp;
  int64_t mvf = (p->split ? 4 : 1) * Hb * Wb;
  int64_t ngop = (T + p->gop - 1) / p->gop;
  xvo_stats(data, dtype, T, H, W, Bn, mn, mx, NULL);
  uint64_t* part = (uint64_t*)calloc((size_t)(G * ngop * 6), sizeof(uint64_t));
  if (!part) return -2;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t u = 0; u < G * ngop; u++) {
    int64_t g = u / ngop, k = u % ngop;
    int64_t t0 = k * p->gop;
    int64_t len = T - t0 < p->gop ? T - t0 : p->gop;
    int64_t ft = g * T + t0;
    err |= xvo_encode_gop(data, dtype, T, H, W, Bn, mn, mx, p, g, t0, len,
                          frames + ft * fsz, levels + ft * fsz, mvs + ft * mvf * 2,
                          recon + ft * fsz, coef_bits + ft * 3 * Hb * Wb,
                          mv_bits + ft * Hb * Wb, splits ? splits + ft * Hb * Wb : NULL,
                          part + u * 6, part + u * 6 + 3);
  }
  for (int64_t b = 0; b < Bn; b++) { sse[b] = 0; nvalid[b] = 0; }
  for (int64_t u = 0; u < G * ngop; u++) {
    int64_t g = u / ngop;
    for (int c = 0; c < 3; c++) {
      int64_t b = 3 * g + c;
      if (b >= Bn) continue;
      sse[b] += part[u * 6 + c];
      nvalid[b] += part[u * 6 + 3 + c];
    }
  }
  free(part);
  return err ? -1 : 0;
}

int xvo_decode_cube(const xvo_params* p, int64_t T, int64_t H, int64_t W,
                    int64_t Bn, const int16_t* levels, const int8_t* mvs,
                    const uint8_t* splits, uint16_t* recon) {
  if (xvo_check_params(p) != 0) return -1;
  int N = p->block;
  int64_t G = (Bn + 2) / 3;
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  int64_t Hb = Hp / N, Wb = Wp / N, fsz = 3 * Hp * Wp;
  int64_t mvf = (p->split ? 4 : 1) * Hb * Wb;
  int64_t ngop = (T + p->gop - 1) / p->gop;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
  for (int64_t u = 0; u < G * ngop; u++) {
    int64_t g = u / ngop, k = u % ngop;
    int64_t t0 = k * p->gop;
    int64_t len = T - t0 < p->gop ? T - t0 : p->gop;
    int64_t ft = g * T + t0;
    err |= xvo_decode_gop(p, H, W, len, levels + ft * fsz, mvs + ft * mvf * 2,
                          splits ? splits + ft * Hb * Wb : NULL, recon + ft * fsz);
  }
  return err ? -1 : 0;
}

/* Decoded cube in the caller's dtype, [T][H][W][Bn] (inverse conversion of
 * Sec. II-A; output rounding paper silent, reading in xvo_cast_output). */
void xvo_denormalize_cube(const uint16_t* recon, int64_t T, int64_t H,
                          int64_t W, int64_t Bn, int N, int B, const double* mn,
                          const double* mx, int out_dtype, void* out) {
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  for (int64_t t = 0; t < T; t++)
    for (int64_t y = 0; y < H; y++)
      for (int64_t x = 0; x < W; x++)
        for (int64_t b = 0; b < Bn; b++) {
          int64_t g = b / 3, c = b % 3;
          int32_t q = recon[(((g * T + t) * 3 + c) * Hp + y) * Wp + x];
          double v = xvo_cast_output(xvo_denormalize(q, mn[b], mx[b], B), out_dtype);
          int64_t o = ((t * H + y) * W + x) * Bn + b;
          if (out_dtype == XVO_U16)
            ((uint16_t*)out)[o] = (uint16_t)v;
          else
            ((float*)out)[o] = (float)v;
        }
}

/* ------------------------------------------------------------------------- */
/* Principal components of the bands before coding (Sec. II-A: the third     */
/* entry of a mapping rule sets how many PCs are kept; Sec. III-C: PCA over  */
/* the ten SimpleS2 bands, the least important PC dropped or coded at lower  */
/* quality).  The paper names no algorithm; reading:                         */
/*  - every (t, y, x) is one sample of the band vector x in R^Bn (u16 cubes, */
/*    the integer data the paper applies PCA to);                            */
/*  - mean m_b = S_b / n and covariance                                      */
/*    C_bc = (n Q_bc - S_b S_c) / n^2 (population form), from the exact      */
/*    integer sums S_b = sum x_b and Q_bc = sum x_b x_c, evaluated as the    */
/*    binary64 chain ((double) num / n) / n;                                 */
/*  - eigenvectors by the cyclic Jacobi method (Golub and Van Loan,          */
/*    "Matrix Computations", the symmetric Schur 2x2 rotation applied in     */
/*    row-cyclic order), sweeps until the off-diagonal sum of squares is at  */
/*    most 1e-30 of the diagonal's or 60 sweeps; eigenvalues in decreasing   */
/*    order (ties: original index), each eigenvector's component of largest  */
/*    magnitude (first such) made positive;                                  */
/*  - PC j of a sample: y_j = sum_b V[b][j] (x_b - m_b) in binary64, b in    */
/*    increasing order, rounded to binary32;                                 */
/*  - inverse from k PCs: x_b = m_b + sum_{j<k} V[b][j] y_j in binary64, j   */
/*    in increasing order, then cast to the output type as the decode does.  */
/* ------------------------------------------------------------------------- */
int xvo_pca_moments(const uint16_t* data, int64_t npix, int64_t Bn, double* mean,
                    double* cov) {
  if (npix <= 0 || Bn <= 0 || Bn > 64) return -1;
  uint64_t S[64] = {0};
  unsigned __int128* Q = (unsigned __int128*)calloc((size_t)(Bn * Bn), sizeof(unsigned __int128));
  if (!Q) return -2;
  for (int64_t i = 0; i < npix; i++) {
    const uint16_t* x = data + i * Bn;
    for (int64_t b = 0; b < Bn; b++) {
      S[b] += x[b];
      for (int64_t c = 0; c < Bn; c++) Q[b * Bn + c] += (unsigned __int128)((uint64_t)x[b] * x[c]);
    }
  }
  const double n = (double)npix;
  for (int64_t b = 0; b < Bn; b++) mean[b] = (double)S[b] / n;
  for (int64_t b = 0; b < Bn; b++)
    for (int64_t c = 0; c < Bn; c++) {
      __int128 num = (__int128)((unsigned __int128)npix * Q[b * Bn + c]) -
                     (__int128)((unsigned __int128)S[b] * S[c]);
      cov[b * Bn + c] = ((double)num / n) / n;
    }
  free(Q);
  return 0;
}

int xvo_pca_eigen(const double* cov, int64_t Bn, double* eigval, double* basis) {
  if (Bn <= 0 || Bn > 64) return -1;
  double A[64][64], V[64][64];
  for (int64_t i = 0; i < Bn; i++)
    for (int64_t j = 0; j < Bn; j++) {
      A[i][j] = cov[i * Bn + j];
      V[i][j] = i == j ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0.0, dia = 0.0;
    for (int64_t p = 0; p < Bn; p++) {
      dia += A[p][p] * A[p][p];
      for (int64_t q = p + 1; q < Bn; q++) off += A[p][q] * A[p][q];
    }
    if (off <= 1e-30 * dia) break;
    for (int64_t p = 0; p < Bn - 1; p++)
      for (int64_t q = p + 1; q < Bn; q++) {
        if (A[p][q] == 0.0) continue;
        /* rotation (c, s) that zeroes A[p][q]: the smaller root t of
         * t^2 + 2 tau t - 1 = 0, tau = (A[q][q] - A[p][p]) / (2 A[p][q]) */
        const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        for (int64_t k = 0; k < Bn; k++) { /* A <- A J */
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int64_t k = 0; k < Bn; k++) { /* A <- J^T A */
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int64_t k = 0; k < Bn; k++) { /* V <- V J */
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  /* decreasing eigenvalues, ties by index (selection of the largest left) */
  int64_t order[64];
  int used[64] = {0};
  for (int64_t j = 0; j < Bn; j++) {
    int64_t best = -1;
    for (int64_t i = 0; i < Bn; i++)
      if (!used[i] && (best < 0 || A[i][i] > A[best][best])) best = i;
    used[best] = 1;
    order[j] = best;
  }
  for (int64_t j = 0; j < Bn; j++) {
    const int64_t src = order[j];
    eigval[j] = A[src][src];
    int64_t arg = 0;
    for (int64_t b = 1; b < Bn; b++)
      if (fabs(V[b][src]) > fabs(V[arg][src])) arg = b;
    const double sg = V[arg][src] < 0.0 ? -1.0 : 1.0;
    for (int64_t b = 0; b < Bn; b++) basis[b * Bn + j] = sg * V[b][src];
  }
  return 0;
}

void xvo_pca_project(const uint16_t* data, int64_t npix, int64_t Bn, const double* mean,
                     const double* basis, int64_t j0, int64_t j1, float* out) {
  for (int64_t i = 0; i < npix; i++)
    for (int64_t j = j0; j < j1; j++) {
      double y = 0.0;
      for (int64_t b = 0; b < Bn; b++) {
        const double d = (double)data[i * Bn + b] - mean[b];
        y = y + basis[b * Bn + j] * d;
      }
      out[i * (j1 - j0) + (j - j0)] = (float)y;
    }
}

void xvo_pca_inverse(const float* pcs, int64_t npix, int64_t Bn, int64_t k,
                     const double* mean, const double* basis, int out_dtype, void* out) {
  for (int64_t i = 0; i < npix; i++)
    for (int64_t b = 0; b < Bn; b++) {
      double x = mean[b];
      for (int64_t j = 0; j < k; j++) x = x + basis[b * Bn + j] * (double)pcs[i * k + j];
      const double v = xvo_cast_output(x, out_dtype);
      if (out_dtype == XVO_U16)
        ((uint16_t*)out)[i * Bn + b] = (uint16_t)v;
      else
        ((float*)out)[i * Bn + b] = (float)v;
    }
}

/* ------------------------------------------------------------------------- */
/* Metrics (Sec. II-C).                                                       */
/* PSNR with a given peak: 10 log10(peak^2 / MSE); MSE = 0 gives +inf.        */
/* ------------------------------------------------------------------------- */
double xvo_psnr(double peak, double sse, double n) {
  if (n <= 0.0) return NAN;
  double mse = sse / n;
  if (mse == 0.0) return INFINITY;
  return 10.0 * log10(peak * peak / mse);
}

/* Integer-domain PSNR of band b: peak L = 2^B - 1 (the maximum of the
 * converted band whenever it is not constant). */
double xvo_psnr_int(int B, uint64_t sse, uint64_t n) {
  return xvo_psnr((double)((1 << B) - 1), (double)sse, (double)n);
}

/* bpppb = stored bits / (pixels x bands) (Sec. II-C), real pixels and bands. */
double xvo_bpppb(uint64_t bits, int64_t T, int64_t H, int64_t W, int64_t Bn) {
  return (double)bits / ((double)T * (double)H * (double)W * (double)Bn);
}

/* Physical-domain squared error of band b over valid samples, decoded in the
 * original dtype; Neumaier-compensated summation. */
void xvo_phys_sse(const void* data, int dtype, int64_t T, int64_t H, int64_t W,
                  int64_t Bn, const uint16_t* recon, int N, int B,
                  const double* mn, const double* mx, double* sse_out) {
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  for (int64_t b = 0; b < Bn; b++) {
    int64_t g = b / 3, c = b % 3;
    double s = 0.0, comp = 0.0;
    for (int64_t t = 0; t < T; t++)
      for (int64_t y = 0; y < H; y++)
        for (int64_t x = 0; x < W; x++) {
          double v = read_sample(data, dtype, ((t * H + y) * W + x) * Bn + b);
          if (isnan(v)) continue;
          int32_t q = recon[(((g * T + t) * 3 + c) * Hp + y) * Wp + x];
          double xh = xvo_cast_output(xvo_denormalize(q, mn[b], mx[b], B), dtype);
          double e = (v - xh) * (v - xh);
          double tt = s + e;
          if (fabs(s) >= fabs(e))
            comp += (s - tt) + e;
          else
            comp += (e - tt) + s;
          s = tt;
        }
    sse_out[b] = s + comp;
  }
}

/* ---- Quality metrics reported beside PSNR (Sec. II-C) ----------------------
 * The paper names SSIM (Wang et al., 2004) and the spectral angle (Kruse et
 * al., 1993) without parameters or domain; paper silent; reading:
 *   SSIM: per coded plane (one real channel of one frame) in the coded integer
 *   domain -- converted frame q against its reconstruction, dynamic range
 *   L = 2^B - 1 -- with the 11 x 11 circularly symmetric Gaussian window of
 *   standard deviation 1.5 normalised to unit sum, K1 = 0.01, K2 = 0.03, at
 *   every window position that lies entirely inside the real H x W picture.
 *   Local statistics are the weighted mean, the weighted variance about it
 *   and the weighted covariance.  A plane scores the mean over its window
 *   positions, a band the mean over its frames; NaN when no window fits.
 *   Spectral angle: per pixel, the angle in radians between the original and
 *   the decoded band vectors, arccos(<s, d> / (|s| |d|)) with the ratio
 *   clamped to [-1, 1]; pixels with a NaN in either vector or a zero-norm
 *   vector are skipped; the cube scores the mean over the remaining pixels
 *   (NaN if none). */

/* Normalised 1-D Gaussian, sigma 1.5, 11 taps; the 2-D window is the outer
 * product of two of them, which is the normalised 2-D Gaussian. */
void xvo_ssim_window(double w[11]) {
  double s = 0.0;
  for (int i = 0; i < 11; i++) {
    double d = (double)(i - 5);
    w[i] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    s += w[i];
  }
  for (int i = 0; i < 11; i++) w[i] /= s;
}

/* Mean SSIM of one plane pair (row stride `stride` samples). */
double xvo_ssim_plane(const uint16_t* a, const uint16_t* b, int64_t stride, int64_t H,
                      int64_t W, int B) {
  if (H < 11 || W < 11) return NAN;
  double w[11];
  xvo_ssim_window(w);
  double L = (double)((1 << B) - 1);
  double C1 = (0.01 * L) * (0.01 * L), C2 = (0.03 * L) * (0.03 * L);
  double sum = 0.0;
  int64_t n = 0;
  for (int64_t y0 = 0; y0 + 11 <= H; y0++)
    for (int64_t x0 = 0; x0 + 11 <= W; x0++) {
      double ma = 0.0, mb = 0.0;
      for (int i = 0; i < 11; i++)
        for (int j = 0; j < 11; j++) {
          double wt = w[i] * w[j];
          ma += wt * a[(y0 + i) * stride + x0 + j];
          mb += wt * b[(y0 + i) * stride + x0 + j];
        }
      double va = 0.0, vb = 0.0, cab = 0.0;
      for (int i = 0; i < 11; i++)
        for (int j = 0; j < 11; j++) {
          double wt = w[i] * w[j];
          double da = a[(y0 + i) * stride + x0 + j] - ma;
          double db = b[(y0 + i) * stride + x0 + j] - mb;
          va += wt * da * da;
          vb += wt * db * db;
          cab += wt * da * db;
        }
      sum += ((2.0 * ma * mb + C1) * (2.0 * cab + C2)) /
             ((ma * ma + mb * mb + C1) * (va + vb + C2));
      n++;
    }
  return sum / (double)n;
}

/* Per-band mean SSIM of an encode: frames and recon are [G][T][3][Hp][Wp]. */
void xvo_ssim_bands(const uint16_t* frames, const uint16_t* recon, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, int N, int B, double* out) {
  int64_t Hp = (H + N - 1) / N * N, Wp = (W + N - 1) / N * N;
  for (int64_t band = 0; band < Bn; band++) {
    int64_t g = band / 3, c = band % 3;
    double s = 0.0;
    for (int64_t t = 0; t < T; t++) {
      int64_t off = ((g * T + t) * 3 + c) * Hp * Wp;
      s += xvo_ssim_plane(frames + off, recon + off, Wp, H, W, B);
    }
    out[band] = s / (double)T;
  }
}

/* Mean spectral angle (radians) between two [T][H][W][Bn] cubes. */
double xvo_spectral_angle(const void* orig, int dtype_o, const void* dec, int dtype_d,
                          int64_t T, int64_t H, int64_t W, int64_t Bn, uint64_t* n_out) {
  double s = 0.0, comp = 0.0;
  uint64_t n = 0;
  for (int64_t p = 0; p < T * H * W; p++) {
    double dot = 0.0, n1 = 0.0, n2 = 0.0;
    int bad = 0;
    for (int64_t b = 0; b < Bn; b++) {
      double u = read_sample(orig, dtype_o, p * Bn + b);
      double v = read_sample(dec, dtype_d, p * Bn + b);
      if (isnan(u) || isnan(v)) bad = 1;
      dot += u * v;
      n1 += u * u;
      n2 += v * v;
    }
    if (bad || n1 == 0.0 || n2 == 0.0) continue;
    double r = dot / (sqrt(n1) * sqrt(n2));
    if (r > 1.0) r = 1.0;
    if (r < -1.0) r = -1.0;
    double e = acos(r);
    double tt = s + e;
    if (fabs(s) >= fabs(e))
      comp += (s - tt) + e;
    else
      comp += (e - tt) + s;
    s = tt;
    n++;
  }
  if (n_out) *n_out = n;
  return n ? (s + comp) / (double)n : NAN;
}
