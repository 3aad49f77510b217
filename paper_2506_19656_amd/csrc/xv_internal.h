// xv_internal.h -- shared declarations of the HIP kernels and the host
// runtime of libxv (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "xv.h"

namespace xv {

// ---------------------------------------------------------------------------
// Work descriptors.  A "stream" is one closed GOP of one band group of one
// cube; frame step s codes frame s of every stream.  One FrameJob describes
// one frame of one stream at one step.  The jobs of one cube are stored
// step-major ([step][group][gop]) by the plan kernel; a launch covers up to
// kMaxSeg segments (contiguous job ranges, e.g. one per cube) that share the
// block size N and, for motion search, the range R.
// ---------------------------------------------------------------------------
// Per-tile sums of the transform kernel: squared error of channels 0..2,
// coefficient bits of channels 0..2, vector bits (each wave of a tile
// writes its channel's slots).
constexpr int kTileSums = 7;

struct FrameJob {
  const uint16_t* cur;         // [3][Hp][Wp] converted frame (encode)
  const uint16_t* ref;         // [3][Hp][Wp] reconstruction of frame t-1 (P)
  uint16_t* rec;               // [3][Hp][Wp] reconstruction of this frame
  int16_t* lev;                // [3][Hb][Wb][N][N], column-major in a block
  int8_t* mv;                  // [Hb][Wb][2]
  uint32_t* cbits;             // [3][Hb][Wb]
  uint32_t* mbits;             // [Hb][Wb]
  const uint8_t* vmask;        // [3][Hp][Wp] validity bytes, or null
  const uint32_t* nan_total;   // device flag: non-zero -> vmask is meaningful
  unsigned long long* part;    // [tiles of the frame][kTileSums] per-tile sums: squared
                               // error and coefficient bits of channels 0..2, vector bits
  uint16_t* pred;              // [3][Hp][Wp] prediction plane read at displacement
                               // zero: the motion-compensated prediction of a P step
                               // with quarter-sample vectors, or the intra prediction
                               // of an I step with intra modes; null: the prediction
                               // is ref displaced (P) or 2^(B-1) (I)
  uint8_t* split;              // adaptive block size: [Hb][Wb] split flags, else null;
                               // mv is then the [2 Hb][2 Wb] grid of N/2 cells
  uint32_t* sad;               // SAD of each searched block's vector, or null
  int8_t* mv_whole;            // adaptive block size, P steps: the whole blocks'
  uint32_t* sad_whole;         // vectors [Hb][Wb][2] and SADs [Hb][Wb]
  int32_t Hp, Wp, H, W;
  int32_t nch;                 // channels carrying a real band (1..3)
  int32_t intra;               // I picture
  int32_t imode;               // I picture whose blocks are intra-predicted; the mode
                               // is the first byte of the block's vector entry
  int32_t bit_depth, qp;
  int32_t lambda16;            // adaptive block size: whole/split cost multiplier
};

constexpr int kMaxSeg = 32;
struct Seg {
  const FrameJob* jobs;  // first job of the segment (device)
  int32_t count;         // jobs in the segment
  int32_t tpj;           // workgroups (tiles) per job
  int32_t tile0;         // first tile of the segment in the launch
  int32_t pad_;
};
struct LaunchDesc {
  int32_t nseg;
  int32_t tiles;
  Seg seg[kMaxSeg];
};

// Locate the job and the job-local tile of workgroup `tile`.
__device__ inline const FrameJob* desc_job(const LaunchDesc& d, int tile, int& local) {
  int i = 0;
  for (int k = 1; k < d.nseg; k++)
    if (d.seg[k].tile0 <= tile) i = k;
  const int rel = tile - d.seg[i].tile0;
  const int j = rel / d.seg[i].tpj;
  local = rel - j * d.seg[i].tpj;
  return d.seg[i].jobs + j;
}

// By-value description of one cube for the plan kernel.
struct CubePlan {
  const uint16_t* frames;      // [G][T][3][Hp][Wp] (null for decode)
  uint16_t* recon;             // [G][T][3][Hp][Wp] written by the coding loop
  int16_t* lev;
  int8_t* mv;
  uint32_t* cbits;
  uint32_t* mbits;
  const uint8_t* vmask;
  const uint32_t* nan_total;
  unsigned long long* part;    // [G][T][tpf][kTileSums] per-tile sums (null for decode)
  uint16_t* pred;              // [G][GOPs][3][Hp][Wp] prediction planes, one per stream,
                               // or null
  FrameJob* jobs;              // [sum over steps of jobs]
  int32_t T, G, gop, nsteps, Hp, Wp, H, W, bands, N, bit_depth, qp;
  int32_t tpf;                 // transform tiles per frame
  int32_t qpel;                // P steps read their prediction from pred
  int32_t imode;               // I blocks intra-predicted; with pred, the I step's
                               // prediction goes to pred too (encode)
  // adaptive block size (null / 0 without): split flags [G][T][Hb][Wb], the
  // whole blocks' vectors and SADs [G][T][Hb][Wb] and the cells' SADs
  // [G][T][2 Hb][2 Wb]
  uint8_t* split;
  int8_t* mv_whole;
  uint32_t* sad_whole;
  uint32_t* sad_cell;
  int32_t lambda16;
};

// Per-group totals of the per-tile sums, in a fixed order: sse [3G] and
// bits [2G] (coefficient, vector) of one encoded cube.  chunk_sum holds
// [G][kTotMaxChunks][5] intermediate sums.
constexpr int kTotMaxChunks = 256;
int encode_totals_chunks(int64_t tiles);
hipError_t launch_encode_totals(const unsigned long long* part, int G, int T, int tpf,
                                unsigned long long* chunk_sum, unsigned long long* sse,
                                unsigned long long* bits, hipStream_t s);

// Jobs at step s: G * ceil((T - s) / gop); offset of step s in the table.
inline int plan_jobs_at(int T, int G, int gop, int s) { return G * ((T - s + gop - 1) / gop); }
__host__ __device__ inline int64_t plan_step_offset(int T, int G, int gop, int s) {
  int64_t o = 0;
  for (int q = 0; q < s; q++) o += (int64_t)G * ((T - q + gop - 1) / gop);
  return o;
}

// ---------------------------------------------------------------------------
// Integer DCT-II of ITU-T H.265.  The 32-point odd rows below are the
// standard's coefficients for rows 1, 3, ..., 31 and columns 0..15; rows of a
// smaller transform are rows k*32/N of the 32-point matrix.  Entry (k, n) of
// the N-point matrix follows from the even/odd symmetry
//   M[k][N-1-n] = (-1)^k M[k][n]
// and the recursion "even rows of the N-point matrix are the N/2-point
// matrix" down to the 2-point DC row (64).
// ---------------------------------------------------------------------------
constexpr int kOdd32[16][16] = {
    {90, 90, 88, 85, 82, 78, 73, 67, 61, 54, 46, 38, 31, 22, 13, 4},
    {90, 82, 67, 46, 22, -4, -31, -54, -73, -85, -90, -88, -78, -61, -38, -13},
    {88, 67, 31, -13, -54, -82, -90, -78, -46, -4, 38, 73, 90, 85, 61, 22},
    {85, 46, -13, -67, -90, -73, -22, 38, 82, 88, 54, -4, -61, -90, -78, -31},
    {82, 22, -54, -90, -61, 13, 78, 85, 31, -46, -90, -67, 4, 73, 88, 38},
    {78, -4, -82, -73, 13, 85, 67, -22, -88, -61, 31, 90, 54, -38, -90, -46},
    {73, -31, -90, -22, 78, 67, -38, -90, -13, 82, 61, -46, -88, -4, 85, 54},
    {67, -54, -78, 38, 85, -22, -90, 4, 90, 13, -88, -31, 82, 46, -73, -61},
    {61, -73, -46, 82, 31, -88, -13, 90, -4, -90, 22, 85, -38, -78, 54, 67},
    {54, -85, -4, 88, -46, -61, 82, 13, -90, 38, 67, -78, -22, 90, -31, -73},
    {46, -90, 38, 54, -90, 31, 61, -88, 22, 67, -85, 13, 73, -82, 4, 78},
    {38, -88, 73, -4, -67, 90, -46, -31, 85, -78, 13, 61, -90, 54, 22, -82},
    {31, -78, 90, -61, 4, 54, -88, 82, -38, -22, 73, -90, 67, -13, -46, 85},
    {22, -61, 85, -90, 73, -38, -4, 46, -78, 90, -82, 54, -13, -31, 67, -88},
    {13, -38, 61, -78, 88, -90, 85, -73, 54, -31, 4, 22, -46, 67, -82, 90},
    {4, -13, 22, -31, 38, -46, 54, -61, 67, -73, 78, -82, 85, -88, 90, -90},
};
constexpr int kOdd16[8][8] = {
    {90, 87, 80, 70, 57, 43, 25, 9},   {87, 57, 9, -43, -80, -90, -70, -25},
    {80, 9, -70, -87, -25, 57, 90, 43}, {70, -43, -87, 9, 90, 25, -80, -57},
    {57, -80, -25, 90, -9, -87, 43, 70}, {43, -90, 57, 25, -87, 70, 9, -80},
    {25, -70, 90, -80, 43, 9, -57, 87}, {9, -25, 43, -57, 70, -80, 87, -90},
};
constexpr int kOdd8[4][4] = {
    {89, 75, 50, 18}, {75, -18, -89, -50}, {50, -89, 18, 75}, {18, -50, 75, -89}};
constexpr int kOdd4[2][2] = {{83, 36}, {36, -83}};

// Entry (k, n) of the n-point matrix (n = 4, 8, 16, 32).
__host__ __device__ constexpr int dct_coef(int N, int k, int n) {
  if (n >= N / 2) return (k & 1) ? -dct_coef(N, k, N - 1 - n) : dct_coef(N, k, N - 1 - n);
  if (k == 0) return 64;
  if (N == 2) return 64;  // k == 1 of the 2-point matrix: 64, -64 by symmetry
  if (k & 1) {
    if (N == 32) return kOdd32[k >> 1][n];
    if (N == 16) return kOdd16[k >> 1][n];
    if (N == 8) return kOdd8[k >> 1][n];
    return kOdd4[k >> 1][n];
  }
  return dct_coef(N / 2, k >> 1, n);
}

__host__ __device__ constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

// Quantiser scales: IQ[k] = round(64 * 2^((k-4)/6)), Qf[k] = round(2^20/IQ[k]).
constexpr int kIQ[6] = {40, 45, 51, 57, 64, 72};
constexpr int kQf[6] = {26214, 23302, 20560, 18396, 16384, 14564};

// Quality metrics beside PSNR: SSIM of the coded planes and the spectral angle.
struct SsimArgs {
  const uint16_t* frames;      // [G][T][3][Hp][Wp] converted frames
  const uint16_t* recon;       // [G][T][3][Hp][Wp] reconstruction
  double* part;                // [bands][T][tiles] per-tile SSIM sums
  double w[11];                // normalised Gaussian taps (sigma 1.5)
  double C1, C2;               // (0.01 L)^2, (0.03 L)^2
  int32_t T, Hp, Wp, H, W, bands;
  int32_t tiles_x, tiles_y;
};
constexpr int kSaThreads = 256;
struct SaArgs {
  const void* orig;            // [T][H][W][bands]
  const void* dec;             // [T][H][W][bands]
  int32_t dtype_orig, dtype_dec;
  int32_t bands;
  int64_t npix;                // T * H * W
  double* part_sum;            // [blocks]
  unsigned long long* part_n;  // [blocks]
  double* out;                 // [2]: sum of angles, pixel count (u64 bits)
};
void ssim_tiles(int H, int W, int* tiles_x, int* tiles_y);
hipError_t launch_ssim(const SsimArgs& a, double* out, hipStream_t s);
hipError_t launch_spectral_angle(const SaArgs& a, int nblocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Kernel launchers (each returns hipGetLastError of its launch).
// ---------------------------------------------------------------------------
struct StatsArgs {
  const void* data;
  int32_t dtype;
  int32_t vec;         // 1: 16-byte loads (data 16-byte aligned); 0: element loads
  int64_t npix;        // T*H*W
  int32_t bands;
  int32_t nblocks;     // grid; nblocks * threads * (elements per load) % bands == 0
  uint32_t* part;      // [nblocks][3][bands] min key, max key, missing count
  uint32_t* nan_count; // [bands]
  uint32_t* nan_total; // [1]
  double* mn;          // [bands]
  double* mx;          // [bands]
  unsigned long long* n_valid;  // [bands]
};
constexpr int kStatsMaxBlocks = 2048;
int stats_blocks(const StatsArgs& a);

struct PackArgs {
  const void* data;
  int32_t dtype;
  int64_t T, H, W;
  int32_t bands, groups;
  int32_t Hp, Wp;
  int32_t bit_depth;
  int32_t pad_mode, fill_mode;
  const double* mn;
  const double* mx;
  const uint32_t* nan_total;
  const uint32_t* nan_count;  // [bands]
  uint16_t* frames;    // [G][T][3][Hp][Wp]
  uint8_t* vmask;      // [G][T][3][Hp][Wp] or null
  int32_t chunk_px;    // pixels of one row chunk (chunk_px_for)
};
// Pixels per row chunk of the row-staged kernels: a power of two in 64..256,
// at least the row width when that is below 256, with chunk * bands <= 4096.
int chunk_px_for(int64_t width, int bands);

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n,
                           hipStream_t s);
hipError_t launch_stats(const StatsArgs& a, hipStream_t s);
hipError_t launch_pack(const PackArgs& a, hipStream_t s);

struct MeGeom {
  int nb;       // blocks per workgroup along x
  int kx;       // candidates per lane along x
  int threads;  // workgroup size
  int rows;     // candidate rows per lane
  int layout;   // XV_ME_COLUMN_PAIRS, XV_ME_ROW_PAIRS or XV_ME_ROW_PAIRS_BY_CHANNEL
};
MeGeom me_default_geometry(int N, int R, int max_nb = 16);
double me_model_score(int N, int R, const MeGeom& g, int width_blocks);
std::vector<MeGeom> me_candidates(int N, int R, int width_blocks);
size_t me_lds_bytes_for(int N, int R, const MeGeom& g);
bool me_geometry_fits(int N, int R, const MeGeom& g);
bool me_instance_exists(const MeGeom& g);
int me_tiles_per_job(int Hb, int Wb, const MeGeom& g);
hipError_t launch_me(int N, int R, const MeGeom& g, const LaunchDesc& d, hipStream_t s);
// Adaptive block size: one search for whole blocks and their N/2 cells
// (k_me.hip; row-pair layouts, KX 5, 7, 11 or 13, N 8..32): the block's
// vector and SAD to mv_whole / sad_whole, the cells' to the cell grid
// (mv / sad).  Its geometries, model and candidates mirror the plain
// search's; by channel, a thread keeps me_split_rounds(g) items.
bool me_split_instance_exists(int N, const MeGeom& g);
size_t me_split_lds_bytes(int N, int R, const MeGeom& g);
int me_split_rounds(const MeGeom& g);
bool me_split_fits(int N, int R, const MeGeom& g);
double me_split_model_score(int N, int R, const MeGeom& g, int width_blocks);
std::vector<MeGeom> me_split_candidates(int N, int R, int width_blocks);
MeGeom me_split_default_geometry(int N, int R, int width_blocks);
hipError_t launch_me_split(int N, int R, const MeGeom& g, const LaunchDesc& d, hipStream_t s);

int xf_tiles_per_job(int N, int Hb, int Wb);
hipError_t launch_encode(int N, const LaunchDesc& d, hipStream_t s);
// Adaptive block size (k_xform.hip).  role 1: the size-N kernel over a
// step's blocks: codes the whole blocks, writes every block's vector bits
// (split flag and coded vectors) and zero coefficient bits for split blocks;
// role 2: the size-N/2 kernel over the N/2 grid (N here is N/2): codes the
// cells of split blocks, adds their coefficient bits to their block's and
// writes its tile sums after the size-N kernel's.  Role 1 runs first.
hipError_t launch_encode_split(int N, int role, const LaunchDesc& d, hipStream_t s);
hipError_t launch_decode_split(int N, int role, const LaunchDesc& d, hipStream_t s);
// Whole-or-split choice of every block of a P step (k_me.hip), after the
// combined search (whole blocks: mv_whole, sad_whole; cells: mv, sad on the
// cell grid): writes split flags and the final cell vectors.
int split_tiles_per_job(int Hb, int Wb);
hipError_t launch_split_decide(int N, const LaunchDesc& d, hipStream_t s);
// Quarter-sample motion (k_subpel.hip): one workgroup per block of a P step.
// launch_subpel refines the integer vectors in jobs' mv (quarter samples
// back into mv) and writes the prediction planes; launch_mc writes the
// prediction planes from stored quarter-sample vectors (decode).
hipError_t launch_subpel(int N, const LaunchDesc& d, hipStream_t s);
hipError_t launch_mc(int N, const LaunchDesc& d, hipStream_t s);
hipError_t launch_decode(int N, const LaunchDesc& d, hipStream_t s);
// Intra-predicted I steps (k_xform.hip): blocks in raster order depend on
// their left, top-left, top and top-right neighbours, so block (bx, by) runs
// in wavefront w = bx + 2 by, one launch per wavefront over every job of d.
// Encode chooses the mode, codes the block and writes its reconstruction,
// its prediction (job pred plane) and its mode (job mv); the transform
// kernel then recodes the step from the prediction plane for levels, bit
// counts and sums.  Decode reconstructs from the stored levels and modes.
int intra_tiles_per_job(int N, int Hb, int Wb);
inline int intra_waves(int Hb, int Wb) { return Wb + 2 * Hb - 2; }
hipError_t launch_intra(int N, const LaunchDesc& d, int wave, int decode, hipStream_t s);
hipError_t launch_plan(const CubePlan& p, hipStream_t s);

struct DenormArgs {
  const uint16_t* recon;   // [G][T][3][Hp][Wp]
  int64_t T, H, W;
  int32_t bands, Hp, Wp, bit_depth;
  const double* mn;
  const double* mx;
  int32_t out_dtype;
  void* out;               // [T][H][W][bands]
  int32_t chunk_px;
};
hipError_t launch_denorm(const DenormArgs& a, hipStream_t s);

struct PhysArgs {
  const void* orig;        // [T][H][W][bands]
  int32_t dtype;
  const uint16_t* recon;   // [G][T][3][Hp][Wp]
  int64_t T, H, W;
  int32_t bands, Hp, Wp, bit_depth;
  const double* mn;
  const double* mx;
  double* partial;         // [nblocks][bands]
  double* out;             // [bands]
  int32_t nblocks;
  int32_t chunk_px;
};
int phys_blocks(int64_t npix);
hipError_t launch_phys_sse(const PhysArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Bitstream (k_bits.hip).  Units in stream order: per frame the Hb*Wb vector
// units, then the 3*Hb*Wb coefficient units; a row of Wb units is a segment.
// ---------------------------------------------------------------------------
struct BitsArgs {
  int32_t N, Hb, Wb, T, gop;
  int32_t imodes;              // I blocks carry their intra mode as one bit
  int64_t nunits;              // G * T * 4 * Hb * Wb
  const uint32_t* cbits;       // [G][T][3][Hb][Wb] unit lengths (pack)
  const uint32_t* mbits;       // [G][T][Hb][Wb]
  const int16_t* levels;       // [G][T][3][Hb][Wb][N*N] (pack)
  const int8_t* mvs;           // [G][T][Hb][Wb][2] (pack)
  uint64_t* block_off;         // [bits_scan_blocks] scratch: block sums -> offsets
  uint64_t* total;             // [1] payload bits
  uint64_t* index;             // [nunits / Wb] segment bit offsets
  uint32_t* words;             // payload, byte order = stream order
  int64_t nwords;              // payload words incl. 2 words of padding (parse)
  uint64_t total_bits;         // (parse)
  int16_t* levels_out;         // (parse) zero on entry
  int8_t* mvs_out;
  uint32_t* cbits_out;
  uint32_t* mbits_out;
  uint32_t* err;               // (parse) set on an inconsistent stream
  // adaptive block size: split flags [G][T][Hb][Wb] (pack) / out (parse), else
  // null; vectors are then on the [2 Hb][2 Wb] cell grid
  const uint8_t* splits;
  uint8_t* splits_out;
  int32_t phase;               // (parse) -1 all segments, 0 vector, 1 coefficient rows
};
int64_t bits_scan_blocks(int64_t nunits);
hipError_t launch_bits_scan(const BitsArgs& a, hipStream_t s);
hipError_t launch_bits_write(const BitsArgs& a, hipStream_t s);
hipError_t launch_bits_parse(const BitsArgs& a, hipStream_t s);

// Header of a serialised cube (first 256 bytes of the buffer).
struct PackHeader {
  char magic[8];               // "XVPACK01"
  uint32_t version, header_bytes;
  int64_t T, H, W, bands;
  int32_t src_dtype, G, N, Hp, Wp, Hb, Wb, reserved;
  xv_params params;
  uint64_t nseg, payload_bits, nwords;
  uint64_t off_span, span_bytes, off_index, off_payload, total_bytes;
  uint8_t pad[256 - 176];
};
static_assert(sizeof(PackHeader) == 256, "pack header size");
hipError_t launch_write_header(const PackHeader& h, void* dst, hipStream_t s);

// ---------------------------------------------------------------------------
// Principal components of the bands (k_pca.hip).
// ---------------------------------------------------------------------------
struct PcaMomArgs {
  const void* data;               // u16 [npix][bands]
  int64_t npix;
  int32_t bands;
  unsigned long long* part;       // [nblocks][P] per-block sums
  unsigned long long* total;      // [P][2] 128-bit totals (low, high)
};
// P = bands (bands + 1) / 2 + bands sums: the upper triangle of Q (row-major,
// b <= c), then S_0 .. S_{bands-1}.
int pca_sum_count(int bands);
int pca_moment_blocks(int64_t npix);
hipError_t launch_pca_moments(const PcaMomArgs& a, int nblocks, hipStream_t s);

struct PcaProjArgs {
  const void* data;               // u16 [npix][bands]
  int64_t npix;
  int32_t bands, j0, j1;          // PCs j0 .. j1-1
  const double* mean;             // [bands]
  const double* basis;            // [bands][bands], column j = PC j
  void* out;                      // f32 [npix][j1 - j0]
};
hipError_t launch_pca_project(const PcaProjArgs& a, hipStream_t s);

struct PcaInvArgs {
  const void* pcs;                // f32 [npix][k]
  int64_t npix;
  int32_t bands, k;
  const double* mean;
  const double* basis;
  int32_t out_dtype;              // XV_U16 or XV_F32
  void* out;                      // [npix][bands]
};
hipError_t launch_pca_inverse(const PcaInvArgs& a, hipStream_t s);

// ---------------------------------------------------------------------------
// Caching device allocator (xv_alloc.cpp).  dev_free keeps the block for
// reuse: at once on the same stream, on another stream once the work queued
// before the free has completed.
// ---------------------------------------------------------------------------
hipError_t dev_alloc(void** out, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);
void dev_stream_retired(hipStream_t s);  // before a stream is destroyed
size_t dev_cache_release();              // waits for and frees every cached block
void dev_cache_stats(size_t* live, size_t* cached, size_t* peak);

}  // namespace xv
