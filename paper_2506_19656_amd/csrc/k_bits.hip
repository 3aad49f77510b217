// k_bits.hip -- the Exp-Golomb bitstream of an encoded cube: the codes the
// rate proxy counts, written out, and parsed back.
//
// Code of a value: ue(k) is floor(log2(k+1)) zero bits followed by k+1 in
// binary, se(v) is ue(2v - 1) for v > 0 and ue(-2v) otherwise (the
// Exp-Golomb codes of ITU-T H.265 clause 9.2).  Bits are MSB-first in
// bytes.  Stream order, frame by frame (f = g * T + t): the vector units of
// the frame's blocks in raster order (se(dx - pdx), se(dy - pdy), the left
// neighbour's vector as predictor, (0,0) in column 0; I frames have empty
// vector units, or one bit holding the block's intra mode when I blocks are
// intra-predicted; with the adaptive block size a P block's unit is its
// split flag and then its one or four vectors, each against the vector of
// the cell left of its top-left cell), then for channel c = 0, 1, 2 the coefficient units of the
// blocks in raster order (coded flag, then ue(nnz - 1) and per nonzero level
// in up-right diagonal scan order ue(run), se(level); a split block: its four
// N/2 blocks' codes in z-order).  A frame therefore
// has 4 Hb Wb units; a row of Wb units is a segment, whose bit offset is
// stored so that segments parse independently.
//
// Packing: the unit lengths are the per-block bit counts the transform
// kernel already produced; an exclusive scan over them gives every unit its
// offset and one thread per unit emits its codes.  Words a unit owns
// completely are stored; the words it shares with its neighbours at either
// end are OR-ed in atomically (the payload starts zeroed).
// Parsing: one thread per segment.
#include "xv_internal.h"

namespace xv {

namespace {

constexpr int kBitsThreads = 256;

// Length of unit u (stream order) from the per-block bit counts.
__device__ inline uint32_t unit_len(const BitsArgs& a, int64_t u) {
  const int64_t hw = (int64_t)a.Hb * a.Wb;
  const int64_t f = u / (4 * hw);
  const int64_t r = u - f * 4 * hw;
  if (r < hw) return a.mbits[f * hw + r];
  return a.cbits[f * 3 * hw + (r - hw)];
}

__device__ inline uint64_t block_sum_u64(uint64_t v, uint64_t* red) {
  // fixed-order tree over the block
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBitsThreads / 2; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const uint64_t s = red[0];
  __syncthreads();
  return s;
}

// Exclusive prefix sum over the block (Hillis-Steele in LDS).
__device__ inline uint64_t block_exclusive_u64(uint64_t v, uint64_t* buf) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int d = 1; d < kBitsThreads; d <<= 1) {
    const uint64_t add = (int)threadIdx.x >= d ? buf[threadIdx.x - d] : 0ull;
    __syncthreads();
    buf[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t incl = buf[threadIdx.x];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kBitsThreads) unit_block_sums_kernel(BitsArgs a) {
  __shared__ uint64_t red[kBitsThreads];
  const int64_t u = (int64_t)blockIdx.x * kBitsThreads + threadIdx.x;
  const uint64_t len = u < a.nunits ? unit_len(a, u) : 0u;
  const uint64_t s = block_sum_u64(len, red);
  if (threadIdx.x == 0) a.block_off[blockIdx.x] = s;
}

// One workgroup turns the block sums into exclusive block offsets (in
// place) and writes the total.
__global__ void __launch_bounds__(1024) scan_block_sums_kernel(uint64_t* v, int64_t n,
                                                               uint64_t* total) {
  __shared__ uint64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b0 = t * per, b1 = min(n, b0 + per);
  uint64_t s = 0;
  for (int64_t i = b0; i < b1; i++) s += v[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    const uint64_t add = t >= d ? part[t - d] : 0ull;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  uint64_t run = part[t] - s;
  for (int64_t i = b0; i < b1; i++) {
    const uint64_t x = v[i];
    v[i] = run;
    run += x;
  }
  if (t == 1023) *total = part[1023];
}

// Bit sink of one unit: pending bits in the low n bits of acc (earliest
// first); complete words leave in stream order, byte-swapped so that memory
// holds the stream's bytes in order.
struct BitSink {
  uint32_t* words;
  uint64_t w;       // index of the word being filled
  uint64_t acc;
  int n;
  bool first;       // the word being filled is shared with the previous unit

  __device__ void emit(uint32_t word, bool shared) {
    const uint32_t m = __builtin_bswap32(word);
    if (shared)
      atomicOr(&words[w], m);
    else
      words[w] = m;
    w++;
  }
  __device__ void put(uint32_t v, int len) {  // len <= 32
    acc = (acc << len) | v;
    n += len;
    if (n >= 32) {
      emit((uint32_t)(acc >> (n - 32)), first);
      first = false;
      n -= 32;
      acc &= (n ? ((1ull << n) - 1) : 0ull);
    }
  }
  __device__ void ue(uint32_t k) {
    const uint32_t v = k + 1;
    const int m = 31 - __clz((int)v);
    put(v, 2 * m + 1);
  }
  __device__ void se(int v) { ue(v > 0 ? (uint32_t)(2 * v - 1) : (uint32_t)(-2 * v)); }
  __device__ void flush() {
    if (n > 0) emit((uint32_t)(acc << (32 - n)), true);
  }
};

__device__ inline void build_scan_table(uint16_t* scan, int N) {
  for (int i = threadIdx.x; i < N * N; i += blockDim.x) {
    const int y = i / N, x = i - (i / N) * N;
    const int d = x + y;
    const int before = d < N ? d * (d + 1) / 2 : N * N - (2 * N - 1 - d) * (2 * N - d) / 2;
    const int first_x = d < N ? 0 : d - N + 1;
    scan[before + x - first_x] = (uint16_t)(x * N + y);  // levels are column-major
  }
}

// Codes of one block's levels (n x n, column-major) in scan order.
__device__ inline void put_block(BitSink& bs, const int16_t* lev, int n, const uint16_t* scan) {
  int nnz = 0;
  for (int i = 0; i < n * n; i += 8) {
    const uint4 w = *(const uint4*)(lev + i);
    const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int j = 0; j < 4; j++) nnz += ((q[j] & 0xffffu) != 0) + ((q[j] >> 16) != 0);
  }
  bs.put(nnz > 0 ? 1u : 0u, 1);
  if (nnz > 0) {
    bs.ue((uint32_t)(nnz - 1));
    // eight scan positions per batch, their loads issued together (n * n is
    // a multiple of 8); zeros after the last nonzero only lengthen a run that
    // is never written
    int run = 0, seen = 0;
    for (int p0 = 0; p0 < n * n && seen < nnz; p0 += 8) {
      int v[8];
#pragma unroll
      for (int j = 0; j < 8; j++) v[j] = lev[scan[p0 + j]];
#pragma unroll
      for (int j = 0; j < 8; j++) {
        if (v[j] == 0) {
          run++;
          continue;
        }
        bs.ue((uint32_t)run);
        bs.se(v[j]);
        run = 0;
        seen++;
      }
    }
  }
}

__global__ void __launch_bounds__(kBitsThreads) write_units_kernel(BitsArgs a) {
  __shared__ uint64_t buf[kBitsThreads];
  __shared__ uint16_t scan[32 * 32];
  __shared__ uint16_t scan_h[16 * 16];
  const int N = a.N;
  build_scan_table(scan, N);
  if (a.splits) build_scan_table(scan_h, N / 2);
  const int64_t u = (int64_t)blockIdx.x * kBitsThreads + threadIdx.x;
  const uint64_t len = u < a.nunits ? unit_len(a, u) : 0u;
  const uint64_t off = a.block_off[blockIdx.x] + block_exclusive_u64(len, buf);  // syncs
  if (u >= a.nunits) return;
  if (u % a.Wb == 0) a.index[u / a.Wb] = off;
  if (len == 0) return;
  BitSink bs{a.words, off >> 5, 0ull, (int)(off & 31), (off & 31) != 0};
  const int64_t hw = (int64_t)a.Hb * a.Wb;
  const int64_t f = u / (4 * hw);
  const int64_t r = u - f * 4 * hw;
  const bool intra = (f % a.T) % a.gop == 0;
  if (r < hw) {
    if (a.splits) {  // a P block's split flag and vectors (I units are empty)
      const int8_t* mvu = a.mvs + f * 4 * hw * 2;
      const int by = (int)(r / a.Wb), bx = (int)(r - (int64_t)by * a.Wb);
      const int64_t Wu = 2 * (int64_t)a.Wb;
      const bool sp = a.splits[f * hw + r] != 0;
      bs.put(sp ? 1u : 0u, 1);
      for (int i = 0; i < (sp ? 4 : 1); i++) {
        const int64_t xu = 2 * bx + (i & 1), yu = 2 * by + (i >> 1);
        const int8_t* v = mvu + (yu * Wu + xu) * 2;
        const int pmx = xu > 0 ? v[-2] : 0, pmy = xu > 0 ? v[-1] : 0;
        bs.se(v[0] - pmx);
        bs.se(v[1] - pmy);
      }
    } else {
      const int8_t* mv = a.mvs + (f * hw + r) * 2;
      if (intra) {  // an intra mode (I units are empty otherwise)
        bs.put(mv[0] != 0 ? 1u : 0u, 1);
        bs.flush();
        return;
      }
      int pmx = 0, pmy = 0;
      if (r % a.Wb != 0) {
        pmx = mv[-2];
        pmy = mv[-1];
      }
      bs.se(mv[0] - pmx);
      bs.se(mv[1] - pmy);
    }
  } else {
    const int16_t* lev = a.levels + (f * 3 * hw + (r - hw)) * N * N;
    const bool sp = a.splits && !intra && a.splits[f * hw + (r - hw) % hw];
    if (len == (sp ? 4u : 1u)) {
      // one bit per block is a coded flag of 0 alone (a block with a nonzero
      // level takes at least 6 bits): the levels need not be read
      bs.put(0u, sp ? 4 : 1);
    } else if (sp) {
      const int h = N / 2;
      for (int q = 0; q < 4; q++) put_block(bs, lev + q * h * h, h, scan_h);
    } else {
      put_block(bs, lev, N, scan);
    }
  }
  bs.flush();
}

// Bit reader over the payload words (byte-swapped back to stream order).
// The next bits of the stream are held MSB-first in a 128-bit register pair
// with at least 65 of them valid (the longest code the writer emits has 33),
// so a code is read from the upper register alone and two new words are
// fetched only once 64 bits have been consumed.  Word reads are clamped to
// the buffer.
struct BitSource {
  const uint32_t* words;
  int64_t nwords;
  uint64_t pos;    // bits consumed, from the start of the payload
  uint64_t hi, lo;  // the next bits, MSB first (hi before lo); bits past nbits are zero
  int nbits;       // valid bits in hi:lo, at least 65 between codes
  int64_t next;    // next word to load

  __device__ uint32_t word(int64_t w) const {
    return __builtin_bswap32(words[min(w, nwords - 1)]);
  }
  __device__ uint64_t pair(int64_t w) const { return ((uint64_t)word(w) << 32) | word(w + 1); }
  // Appends the next 64 payload bits once no more than 64 are left: one wait
  // for memory per 64 bits parsed (the level stores in flight count in it).
  __device__ void refill() {
    if (nbits > 64) return;
    const uint64_t c = pair(next);
    next += 2;
    if (nbits == 64) {
      lo = c;
    } else {
      hi |= c >> nbits;
      lo = c << (64 - nbits);
    }
    nbits += 64;
  }
  __device__ void start(const uint32_t* w, int64_t nw, uint64_t at) {
    words = w;
    nwords = nw;
    pos = at;
    const int64_t w0 = (int64_t)(at >> 5);
    const int sh = (int)(at & 31);
    hi = pair(w0);
    lo = pair(w0 + 2);
    next = w0 + 4;
    if (sh) {
      hi = (hi << sh) | (lo >> (64 - sh));
      lo <<= sh;
    }
    nbits = 128 - sh;
  }
  // n in 1..33
  __device__ void skip(int n) {
    hi = (hi << n) | (lo >> (64 - n));
    lo <<= n;
    nbits -= n;
    pos += (uint64_t)n;
    refill();
  }
  __device__ int bit() {
    const int b = (int)(hi >> 63);
    skip(1);
    return b;
  }
  // ue(k): m leading zeros, then m + 1 bits holding k + 1; false on a code
  // longer than any the writer emits.
  __device__ bool ue(uint32_t& k) {
    if (hi == 0) return false;
    const int m = __clzll((long long)hi);
    if (m > 16) return false;
    const int len = 2 * m + 1;
    k = (uint32_t)(hi >> (64 - len)) - 1u;
    skip(len);
    return true;
  }
  __device__ bool se(int& v) {
    uint32_t k;
    if (!ue(k)) return false;
    v = (k & 1) ? (int)((k + 1) / 2) : -(int)(k / 2);
    return true;
  }
  // ue(run) then se(v): one shift when the two codes together take at most
  // 33 bits (both then lie in the upper register), else the two reads.
  __device__ bool run_level(uint32_t& run, int& v) {
    if (hi == 0) return false;
    const int m1 = __clzll((long long)hi);
    if (m1 > 16) return false;
    const int l1 = 2 * m1 + 1;
    const uint64_t x = hi << l1;
    if (x != 0) {
      const int l2 = 2 * __clzll((long long)x) + 1;
      if (l1 + l2 <= 33) {
        run = (uint32_t)(hi >> (64 - l1)) - 1u;
        const uint32_t k = (uint32_t)(x >> (64 - l2)) - 1u;
        v = (k & 1) ? (int)((k + 1) / 2) : -(int)(k / 2);
        skip(l1 + l2);
        return true;
      }
    }
    return ue(run) && se(v);
  }
};

// One thread per segment (a row of Wb units).  Levels must be zero on entry.
// Any inconsistency (a code no writer emits, a position past the block, a
// vector out of range, a segment not ending where the next begins) sets
// *err and stops that segment.
// Levels of one n x n block (column-major, zero on entry) from its codes.
__device__ inline bool get_block(BitSource& src, int16_t* lev, int n, const uint16_t* scan) {
  if (!src.bit()) return true;
  uint32_t k;
  if (!src.ue(k) || k >= (uint32_t)(n * n)) return false;
  // a fixed nnz iterations without an early exit; a bad code sets `bad`
  // (the caller then rejects the whole buffer) and every store stays inside
  // the block
  bool bad = false;
  int p = -1;
  for (int i = 0; i <= (int)k; i++) {
    uint32_t run = 0;
    int v = 0;
    bad |= !src.run_level(run, v);
    p = min(p + (int)run + 1, n * n);
    bad |= v == 0 || v < -32767 || v > 32767 || p == n * n;
    lev[scan[min(p, n * n - 1)]] = (int16_t)v;
  }
  return !bad;
}

__global__ void __launch_bounds__(kBitsThreads) parse_segments_kernel(BitsArgs a) {
  __shared__ uint16_t scan[32 * 32];
  __shared__ uint16_t scan_h[16 * 16];
  const int N = a.N;
  build_scan_table(scan, N);
  if (a.splits_out) build_scan_table(scan_h, N / 2);
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * kBitsThreads + threadIdx.x;
  const int64_t nseg = a.nunits / a.Wb;
  if (s >= nseg) return;
  const int64_t hw = (int64_t)a.Hb * a.Wb;
  const int64_t spf = 4 * (int64_t)a.Hb;  // segments per frame
  const int64_t f = s / spf;
  const int64_t r = s - f * spf;
  const uint64_t end = s + 1 < nseg ? a.index[s + 1] : a.total_bits;
  BitSource src;
  src.start(a.words, a.nwords, a.index[s]);
  const int t = (int)(f % a.T);
  const bool intra = t % a.gop == 0;
  bool ok = true;
  // with split flags the vector rows parse first (phase 0), then the
  // coefficient rows, which need the flags (phase 1)
  if (a.phase >= 0 && (r < a.Hb) != (a.phase == 0)) return;
  if (r < a.Hb && a.splits_out) {
    const int64_t row = r;
    const int64_t Wu = 2 * (int64_t)a.Wb;
    int8_t* mvu = a.mvs_out + f * 4 * hw * 2;
    for (int bx = 0; bx < a.Wb && ok; bx++) {
      const int64_t blk = f * hw + row * a.Wb + bx;
      const uint64_t p0 = src.pos;
      const bool sp = !intra && src.bit();
      a.splits_out[blk] = sp ? 1 : 0;
      for (int i = 0; i < 4; i++) {
        const int64_t xu = 2 * bx + (i & 1), yu = 2 * row + (i >> 1);
        int8_t* v = mvu + (yu * Wu + xu) * 2;
        int mx = 0, my = 0;
        if (!intra && (sp || i == 0)) {
          int ddx = 0, ddy = 0;
          ok = ok && src.se(ddx) && src.se(ddy);
          mx = (xu > 0 ? v[-2] : 0) + ddx;
          my = (xu > 0 ? v[-1] : 0) + ddy;
          ok = ok && mx >= -128 && mx <= 127 && my >= -128 && my <= 127;
        } else if (!intra) {  // a whole block repeats its vector
          mx = mvu[(2 * row * Wu + 2 * bx) * 2];
          my = mvu[(2 * row * Wu + 2 * bx) * 2 + 1];
        }
        v[0] = (int8_t)mx;
        v[1] = (int8_t)my;
      }
      a.mbits_out[blk] = (uint32_t)(src.pos - p0);
    }
  } else if (r < a.Hb) {
    const int64_t row = r;
    int pmx = 0, pmy = 0;
    for (int bx = 0; bx < a.Wb && ok; bx++) {
      const int64_t blk = f * hw + row * a.Wb + bx;
      int dx = 0, dy = 0;
      const uint64_t p0 = src.pos;
      if (!intra) {
        int ddx = 0, ddy = 0;
        ok = src.se(ddx) && src.se(ddy);
        dx = pmx + ddx;
        dy = pmy + ddy;
        ok = ok && dx >= -128 && dx <= 127 && dy >= -128 && dy <= 127;
      } else if (a.imodes) {
        dx = src.bit();
      }
      a.mvs_out[blk * 2] = (int8_t)dx;
      a.mvs_out[blk * 2 + 1] = (int8_t)dy;
      a.mbits_out[blk] = (uint32_t)(src.pos - p0);
      pmx = dx;
      pmy = dy;
    }
  } else {
    const int c = (int)((r - a.Hb) / a.Hb);
    const int64_t row = (r - a.Hb) - (int64_t)c * a.Hb;
    for (int bx = 0; bx < a.Wb && ok; bx++) {
      const int64_t blk = (f * 3 + c) * hw + row * a.Wb + bx;
      int16_t* lev = a.levels_out + blk * N * N;
      const uint64_t p0 = src.pos;
      if (a.splits_out && a.splits_out[f * hw + row * a.Wb + bx]) {
        const int h = N / 2;
        for (int q = 0; q < 4 && ok; q++) ok = get_block(src, lev + q * h * h, h, scan_h);
      } else {
        ok = get_block(src, lev, N, scan);
      }
      a.cbits_out[blk] = (uint32_t)(src.pos - p0);
    }
  }
  if (!ok || src.pos != end) atomicOr(a.err, 1u);
}

__global__ void write_header_kernel(PackHeader h, PackHeader* dst) { *dst = h; }

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

int64_t bits_scan_blocks(int64_t nunits) { return (nunits + kBitsThreads - 1) / kBitsThreads; }

hipError_t launch_bits_scan(const BitsArgs& a, hipStream_t s) {
  const int64_t nb = bits_scan_blocks(a.nunits);
  if (nb <= 0) return hipSuccess;
  unit_block_sums_kernel<<<(unsigned)nb, kBitsThreads, 0, s>>>(a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  scan_block_sums_kernel<<<1, 1024, 0, s>>>(a.block_off, nb, a.total);
  return hipGetLastError();
}

hipError_t launch_bits_write(const BitsArgs& a, hipStream_t s) {
  const int64_t nb = bits_scan_blocks(a.nunits);
  if (nb <= 0) return hipSuccess;
  write_units_kernel<<<(unsigned)nb, kBitsThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_bits_parse(const BitsArgs& a, hipStream_t s) {
  const int64_t nseg = a.nunits / a.Wb;
  if (nseg <= 0) return hipSuccess;
  if (!a.splits_out) {
    BitsArgs b = a;
    b.phase = -1;
    parse_segments_kernel<<<blocks_for(nseg, kBitsThreads), kBitsThreads, 0, s>>>(b);
    return hipGetLastError();
  }
  for (int ph = 0; ph < 2; ph++) {
    BitsArgs b = a;
    b.phase = ph;
    parse_segments_kernel<<<blocks_for(nseg, kBitsThreads), kBitsThreads, 0, s>>>(b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_write_header(const PackHeader& h, void* dst, hipStream_t s) {
  write_header_kernel<<<1, 1, 0, s>>>(h, (PackHeader*)dst);
  return hipGetLastError();
}

}  // namespace xv
