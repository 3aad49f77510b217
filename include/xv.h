/*
 * xv.h -- C ABI of the MI355X transform-coding library (libxv.so).
 *
 * The library compresses a multichannel spatiotemporal cube (time x y x x x
 * bands) the way the paper "Video Compression for Spatiotemporal Earth System
 * Data" (arXiv 2506.19656) does: every band is converted to B-bit integers
 * (Sec. II-A, bit-depth conversion), bands are packed in input order into
 * 3-channel frames (Sec. II-A), missing samples are filled along time
 * (Sec. III-B), and the frames are coded by a hybrid video coder.  The coder
 * is the lossy loop of an HEVC-style encoder: integer-pel block motion search
 * for P pictures, motion-compensated residuals, the H.265 integer DCT-II
 * (N = 4, 8, 16, 32), a QP-driven dead-zone quantiser, dequantisation and
 * inverse transform to the reconstruction.  Its rate is measured by
 * Exp-Golomb code lengths of coefficients and motion vectors (no arithmetic
 * coder); quality by per-band PSNR whose peak is the band's maximum
 * (Sec. II-C) and by bits per pixel per band (Sec. II-C).
 *
 * All compute runs in HIP kernels on the GPU; the caller hands in device
 * pointers and a HIP stream (hipStream_t passed as void*, NULL = the null
 * stream).  Every call is asynchronous on that stream unless stated.
 *
 * Status codes: every int-returning call returns XV_OK (0) or a negative
 * XV_E* code; xv_last_error() returns a thread-local message for the last
 * failure of the calling thread.  No C++ exception crosses this ABI.
 *
 * Data layouts (all C-contiguous, row-major):
 *   input / output cube   [T][H][W][bands]     (the paper's time, y, x,
 *                                               channel order, Listing 1)
 *   converted frames      [G][T][3][Hp][Wp] u16   G = ceil(bands / 3)
 *   reconstruction        [G][T][3][Hp][Wp] u16   Hp, Wp = H, W rounded up
 *                                                 to a multiple of N
 *   levels                [G][T][3][Hb][Wb][N][N] i16 (block-major; inside a
 *                          block column-major: the level of vertical
 *                          frequency l, horizontal frequency k at k * N + l)
 *   motion vectors        [G][T][Hb][Wb][2] i8 (dx, dy); zero in I pictures
 *                          ((mode, 0) under XV_FLAG_INTRA: 0 planar, 1 DC);
 *                          in quarter samples under XV_FLAG_QPEL
 *   coefficient bits      [G][T][3][Hb][Wb] u32
 *   motion-vector bits    [G][T][Hb][Wb] u32
 */
#ifndef XV_H
#define XV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XV_ABI_VERSION 8

/* status codes */
#define XV_OK 0
#define XV_EINVAL (-1)    /* null pointer, bad shape, dtype or parameter     */
#define XV_ENOMEM (-2)    /* device allocation failed or over budget         */
#define XV_EHIP (-3)      /* HIP runtime error (text in xv_last_error)       */
#define XV_EBUSY (-4)     /* server queue full                               */
#define XV_ECANCELED (-5) /* server request cancelled                        */
#define XV_EPENDING (-6)  /* server request not finished yet                 */

/* element types of a cube */
#define XV_U16 0
#define XV_F32 1

/* padding of the last band group when bands % 3 != 0 */
#define XV_PAD_ZERO 0   /* missing channels are zero                          */
#define XV_PAD_REPEAT 1 /* missing channels repeat the last band (Sec. II-A)  */

/* missing-data (NaN) fill along time, float input only */
#define XV_FILL_NEAREST 0 /* value at the nearest valid time, ties earlier   */
#define XV_FILL_FORWARD 1 /* last valid value (Sec. III-B); leading gaps take
                             the first valid value                          */

/* xv_params.flags */
#define XV_FLAG_DROP_WORK 1u /* free converted frames and reconstruction when
                                the encode completes (physical PSNR and the
                                export of those buffers become unavailable) */
#define XV_FLAG_QPEL 2u      /* quarter-sample motion: the integer search's
                                vector of each block refined to half and then
                                quarter samples with the H.265 luma
                                interpolation filters; vectors are stored in
                                quarter samples (needs search_range <= 31) */
#define XV_FLAG_INTRA 4u     /* intra prediction of I pictures: each block
                                predicted from its reconstructed neighbours
                                by planar or DC (ITU-T H.265 8.4.4.2), the
                                mode with the smaller SAD over the real
                                channels (planar on a tie), one mode per
                                block for the group; blocks coded in raster
                                order, so a picture is coded in wavefronts.
                                The mode is stored as the first byte of the
                                block's vector entry and costs one vector
                                bit. */
#define XV_FLAG_SPLIT 8u     /* adaptive block size of P pictures: each
                                block (block >= 8) coded whole or as four
                                block/2 blocks in z-order, each with its own
                                vector and transform, whichever has the
                                smaller 16 SAD + lambda16 bits (bits of the
                                vectors against zero; lambda16 =
                                floor(16 sqrt(0.57 2^((qP-12)/3)) + 1/2),
                                qP = qp + 6 (bit_depth - 8); a tie keeps it
                                whole).  Vectors are then stored on the
                                block/2 grid ([G][T][2Hb][2Wb][2], a whole
                                block's vector repeated over its four cells)
                                and a split block's levels are its four
                                blocks' levels in z-order inside its slot.
                                A block's vector bits: one split flag plus
                                se of each coded vector's difference to the
                                vector of the cell left of its top-left cell.
                                Not with XV_FLAG_QPEL or XV_FLAG_INTRA. */

#define XV_MAX_BANDS 64
#define XV_MAX_GROUPS 22

/* A cube in device memory: data points to T*H*W*bands elements of dtype. */
typedef struct {
  void* data;
  int32_t dtype; /* XV_U16 or XV_F32 */
  int32_t reserved;
  int64_t T, H, W, bands; /* each >= 1; bands <= XV_MAX_BANDS; H, W <= 65536,
                             T*H*W < 2^32 and (H+31)*(W+31) < 2^31 / 6 */
} xv_cube;

/* Coding parameters of one encode. */
typedef struct {
  int32_t bit_depth;    /* B in 8..12: samples are converted to [0, 2^B-1]  */
  int32_t qp;           /* -6(B-8)..51; qP = QP + 6(B-8) drives the step    */
  int32_t block;        /* N in {4, 8, 16, 32}: prediction and transform    */
  int32_t search_range; /* R in 0..64 (0..31 with XV_FLAG_QPEL): motion
                           search over [-R, R]^2                            */
  int32_t gop;          /* closed GOP length >= 1: one I then gop-1 P       */
  int32_t pad_mode;     /* XV_PAD_*                                          */
  int32_t fill_mode;    /* XV_FILL_*                                         */
  uint32_t flags;       /* XV_FLAG_*                                         */
} xv_params;

/* Opaque encoded cube: levels, motion vectors, bit counts, band statistics
 * and (unless XV_FLAG_DROP_WORK) the converted frames and reconstruction,
 * all in device memory owned by the library. */
typedef struct xv_encoded xv_encoded;

/* Quality and rate of an encode (Sec. II-C). */
typedef struct {
  int32_t bands, groups;
  double psnr[XV_MAX_BANDS];      /* integer domain, peak 2^B-1            */
  double psnr_phys[XV_MAX_BANDS]; /* physical domain, peak = band maximum;
                                     NaN if no original was given or the
                                     peak is <= 0                          */
  double sse_phys[XV_MAX_BANDS];
  uint64_t sse[XV_MAX_BANDS];     /* integer-domain squared error          */
  uint64_t n_valid[XV_MAX_BANDS]; /* non-missing real samples              */
  double band_min[XV_MAX_BANDS], band_max[XV_MAX_BANDS];
  uint64_t coef_bits, mv_bits;    /* rate proxy totals                     */
  uint64_t header_bits;           /* 128 per band + 256, not in bpppb      */
  double bpppb;                   /* (coef + mv bits) / (T H W bands)      */
  double bpppb_group[XV_MAX_GROUPS];
} xv_metrics;

/* Read-only view of an encoded cube (device pointers owned by the encoded
 * object, valid until xv_encoded_free; NULL where dropped). */
typedef struct {
  int64_t T, H, W, bands, groups, Hp, Wp, Hb, Wb;
  xv_params params;
  int32_t src_dtype;
  int32_t reserved;
  const uint16_t* frames;
  const uint16_t* recon;
  const int16_t* levels;
  const int8_t* mvs;
  const uint32_t* coef_bits;
  const uint32_t* mv_bits;
  const double* band_min; /* [bands] */
  const double* band_max; /* [bands] */
  const uint64_t* sse;    /* [3*groups]: per coded channel; entry 3g+c is band 3g+c */
  const uint64_t* n_valid;/* [bands] */
  const uint8_t* splits;  /* [groups][T][Hb][Wb] split flags (XV_FLAG_SPLIT), else NULL */
} xv_export;

int xv_abi_version(void);
const char* xv_status_str(int status);
const char* xv_last_error(void);

/* Encode a device-resident cube (Sec. II-A conversion and packing, then the
 * coding loop).  The caller keeps in->data alive and unchanged until the
 * stream has passed the call.  On success *out receives a new encoded cube
 * owned by the caller, to be released with xv_encoded_free.  On error *out
 * is NULL.  Errors: XV_EINVAL, XV_ENOMEM, XV_EHIP. */
int xv_encode_cube(const xv_cube* in, const xv_params* p, void* hip_stream,
                   xv_encoded** out);

/* Decode an encoded cube into out: the reverse of the encode, the library's
 * video-to-cube step (Sec. II-A, `video2xarray`): prediction from the stored
 * vectors, dequantisation and inverse transform to the reconstruction, then
 * the B-bit samples mapped back through the stored band minima and maxima.
 * out is device memory owned by the caller, with the same T, H, W, bands as
 * the encoded cube and dtype XV_U16 or XV_F32.  Output
 * samples are min + q (max - min) / (2^B - 1) rounded half up and clamped
 * (u16) or rounded to the nearest float (f32).  Missing samples of the
 * original decode to their filled values.  Errors: XV_EINVAL (shape or dtype
 * mismatch), XV_ENOMEM, XV_EHIP. */
int xv_decode_cube(const xv_encoded* e, const xv_cube* out, void* hip_stream);

/* Metrics of an encode (Sec. II-C).  orig may be NULL; otherwise it is the
 * cube that was encoded and the physical-domain PSNR is computed from it.
 * Synchronises hip_stream.  m is caller memory.  Errors: XV_EINVAL, XV_EHIP. */
int xv_psnr_bpppb(const xv_cube* orig, const xv_encoded* e, xv_metrics* m,
                  void* hip_stream);
/* The metrics of n encodes with one synchronisation of hip_stream: ms[i] as
 * xv_psnr_bpppb(origs ? &origs[i] : NULL, encs[i], &ms[i]) would give them.
 * origs (n cubes) may be NULL; ms is caller memory for n results.  The
 * metric spans are gathered in a device buffer the call allocates and
 * frees.  Errors: XV_EINVAL (n < 1, a NULL pointer, a cube that differs
 * from its encode), XV_ENOMEM, XV_EHIP. */
int xv_psnr_bpppb_batch(int n, const xv_cube* origs, const xv_encoded* const* encs,
                        xv_metrics* ms, void* hip_stream);

/* Structural similarity per band (Sec. II-C names SSIM, Wang et al. 2004,
 * without parameters; this is the stated reading): in the coded domain, each
 * real channel of each frame -- the converted frame against its
 * reconstruction, dynamic range L = 2^B - 1 -- with an 11 x 11 Gaussian
 * window of standard deviation 1.5 (unit sum), K1 = 0.01, K2 = 0.03, at every
 * window position inside the real H x W picture; a plane scores the mean over
 * its positions, a band the mean over its frames.  ssim[b] for b < bands
 * (caller memory); NaN when H or W is below 11.  Needs the encode's converted
 * frames and reconstruction: XV_EINVAL after XV_FLAG_DROP_WORK or for a cube
 * read from a bitstream.  Synchronises hip_stream.  Errors: XV_EINVAL,
 * XV_ENOMEM, XV_EHIP. */
int xv_ssim(const xv_encoded* e, double* ssim, void* hip_stream);

/* Mean spectral angle in radians between two device cubes of equal shape
 * (Sec. II-C names it, Kruse et al. 1993): per pixel arccos(<s, d> / (|s|
 * |d|)) over the band vectors, in binary64, the ratio clamped to [-1, 1];
 * pixels with a NaN in either vector or a zero-norm vector are skipped.
 * *mean_rad is NaN when every pixel is skipped; *n_pixels (may be NULL)
 * receives the number used.  Either cube may be XV_U16 or XV_F32.
 * Synchronises hip_stream.  Errors: XV_EINVAL (shape mismatch), XV_ENOMEM,
 * XV_EHIP. */
int xv_spectral_angle(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                      uint64_t* n_pixels, void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as xv_spectral_angle, bit for bit, with no allocation of any kind.
 * Its kernels keep their scratch (per-block partial sums and counts, 65,552
 * bytes at most) in one static device array per GPU, held until the process
 * ends; every call on a GPU shares that GPU's array, so calls that overlap
 * on one GPU (on different streams or threads) race and must be serialised
 * by the caller.  The caller passes both cubes (device memory) and the host
 * outputs, as for xv_spectral_angle.  Synchronises hip_stream.  Errors:
 * XV_EINVAL (shape mismatch, or a grid needing more scratch than the array
 * holds, which no valid cube does), XV_EHIP. */
int xv_spectral_angle_noalloc(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                              uint64_t* n_pixels, void* hip_stream);

/* Fill a read-only view of the encoded cube's device buffers. */
int xv_encoded_export(const xv_encoded* e, xv_export* v);

/* Release an encoded cube (stream-ordered on the stream of its encode).
 * NULL is a no-op. */
void xv_encoded_free(xv_encoded* e);

/* ---- Batched path: several cubes, one launch per frame step ------------ */

/* Encode n cubes of possibly different shapes and parameters.  Every frame
 * step launches one kernel per (block size, search range) class covering all
 * cubes (motion search, then transform coding), launched eagerly on
 * hip_stream.  Outputs are identical to n calls of xv_encode_cube.  outs[i]
 * receive the encoded cubes (all NULL on error). */
int xv_encode_batch(int n, const xv_cube* cubes, const xv_params* params,
                    void* hip_stream, xv_encoded** outs);

/* Decode n encoded cubes into outs[i] (as xv_decode_cube, batched). */
int xv_decode_batch(int n, xv_encoded* const* encs, const xv_cube* outs,
                    void* hip_stream);

/* Graph replay of the batched paths (process-wide, off by default).  With it
 * on and per-launch timing off, xv_encode_batch and xv_decode_batch capture
 * the frame-step launches of each (block size, search range) class as a HIP
 * graph the first time a batch of that shape runs on a stream, and replay
 * it for later batches of the same shape (frame count, groups, GOP, padded
 * size, block size, search range, quarter-sample flag, motion-search
 * geometry, stream): each call writes its job tables as usual and copies
 * them into the graph's own tables before the replay, so outputs are those
 * of the eager launches.  Up to 32 graphs are kept (least recently used
 * dropped); xv_cache_release drops them all.  A stream a graph was replayed
 * on must stay alive until then. */
int xv_set_graph_mode(int on);
int xv_get_graph_mode(void);

/* ---- Serving loop: continuous batching of encode / decode requests ---- */

/* A server owns one scheduler thread and one HIP stream.  Requests are
 * admitted in arrival order while a slot is free and their device footprint
 * fits the memory budget; every scheduler iteration then launches the next
 * frame step of all resident requests together (one launch per block-size
 * class, whatever step each request is at), so requests that arrive while
 * others are on the GPU join the running batch.  A request's outputs are
 * identical to those of xv_encode_cube / xv_decode_cube. */
#define XV_OP_ENCODE 0
#define XV_OP_DECODE 1

typedef struct {
  uint64_t hbm_budget; /* bytes for in-flight requests (0: 64 GiB)            */
  int32_t max_slots;   /* resident requests at once (<= 0: 64)                */
  int32_t max_queue;   /* queued requests before submit fails (<= 0: 65536)   */
  void* stream;        /* HIP stream to launch on (NULL: the server makes one) */
} xv_server_cfg;

typedef struct xv_server xv_server;

typedef struct {
  int32_t op;            /* XV_OP_ENCODE or XV_OP_DECODE                       */
  int32_t reserved;
  xv_cube cube;          /* encode: input; decode: output buffer (device)      */
  xv_params params;      /* encode only                                        */
  const xv_encoded* enc; /* decode only: the encoded cube (must outlive it)    */
} xv_request;

typedef struct {
  int32_t status;  /* XV_OK, XV_ECANCELED or the request's error              */
  int32_t op;
  xv_encoded* enc; /* encode result; the caller owns it once returned         */
  double submit_ms, admit_ms, done_ms; /* steady host clock, milliseconds     */
} xv_result;

typedef struct {
  uint64_t submitted, completed, cancelled, failed;
  uint64_t iterations, launches;
  uint64_t peak_bytes;
  int32_t peak_active;
  int32_t reserved;
} xv_server_stats;

/* Create a server.  Errors: XV_EINVAL, XV_EHIP. */
int xv_server_create(const xv_server_cfg* cfg, xv_server** out);
/* Queue a request (non-blocking); *ticket identifies it.  The caller keeps
 * the request's device buffers alive until its result is returned.  Errors:
 * XV_EINVAL (bad request), XV_EBUSY (queue full). */
int xv_server_submit(xv_server* sv, const xv_request* rq, uint64_t* ticket);
/* XV_EPENDING while the request runs; XV_OK once *res holds its result (the
 * ticket is then retired).  XV_EINVAL for an unknown ticket. */
int xv_server_poll(xv_server* sv, uint64_t ticket, xv_result* res);
/* As xv_server_poll, but blocks until the request completes. */
int xv_server_wait(xv_server* sv, uint64_t ticket, xv_result* res);
/* Cancel: a queued request never runs; a running one finishes on the GPU
 * and its result is discarded.  Its status becomes XV_ECANCELED. */
int xv_server_cancel(xv_server* sv, uint64_t ticket);
int xv_server_stats_read(xv_server* sv, xv_server_stats* st);
/* Drain queued and running requests, release unretrieved results, stop the
 * scheduler and free the server.  NULL is a no-op. */
int xv_server_destroy(xv_server* sv);

/* ---- Launch geometry (never changes coded outputs) -------------------- */

/* Window layouts of the motion-search kernel in LDS.  Column pairs: a
 * dword holds two horizontally adjacent samples; a lane takes an even
 * number of candidate columns (2..18) on 1, 2, 3 or (for 2 or 4 columns) 5
 * candidate rows.  Row pairs: a dword holds two vertically adjacent
 * samples (twice the LDS); a lane takes 2..9, 11 or 13 candidate columns on
 * one candidate row.  Row pairs by channel: the same with the three
 * channels staged one after another (a third of the LDS); a workgroup's
 * items, blocks_per_wg x (2R+1) x ceil((2R+1)/cands_per_lane), must not
 * exceed 3 x threads. */
#define XV_ME_COLUMN_PAIRS 1
#define XV_ME_ROW_PAIRS 2
#define XV_ME_ROW_PAIRS_BY_CHANNEL 3

/* Geometry of the motion-search kernel for one (N, R): blocks per
 * workgroup along x, candidates per lane along x, threads per workgroup
 * (multiple of 64, <= 512), candidate rows per lane, window layout (above).
 * Zero fields take the default; NULL or all fields zero restores the
 * default for (block, search_range). */
typedef struct {
  int32_t blocks_per_wg;
  int32_t cands_per_lane;
  int32_t threads;
  int32_t rows_per_lane;
  int32_t layout;
} xv_me_geometry;

/* Installs g for (block, search_range) in this process.  A layout other
 * than the default's with rows_per_lane zero takes one candidate row per
 * lane.  Errors: XV_EINVAL for a bad block or search range, an unknown
 * layout, a count of candidates or rows the layout has no kernel for,
 * threads outside 64..512 or not a multiple of 64, blocks_per_wg outside
 * 1..64, more than 160 KB of LDS, or (row pairs by channel) more items per
 * workgroup than three rounds of its threads. */
int xv_set_me_geometry(int block, int search_range, const xv_me_geometry* g);
/* Geometry used for (block, search_range) on frames width_blocks blocks wide
 * (width_blocks <= 0: 16): the one set or tuned, else the model default. */
int xv_get_me_geometry(int block, int search_range, int width_blocks, xv_me_geometry* g);

/* The same pair for the search of the adaptive block size (XV_FLAG_SPLIT),
 * which finds the vectors of every block and of its four N/2 cells in one
 * pass (block 8, 16 or 32): row-pair layouts only, 5, 7, 11 or 13
 * candidates per lane, one row; staged by channel, a workgroup's items
 * must not exceed 2 rounds of its threads for 5 or 7 candidates, 1 round
 * for 11 or 13.  Same errors as above. */
int xv_set_me_split_geometry(int block, int search_range, const xv_me_geometry* g);
int xv_get_me_split_geometry(int block, int search_range, int width_blocks, xv_me_geometry* g);

/* Empirical tuner: times the motion-search kernel on the first P-picture
 * step of the cube `in` (device memory) coded with p, for the geometries the
 * model ranks highest (max_candidates of them, <= 0: 512, shared equally
 * among the window layouts), times the six fastest again in nine
 * interleaved rounds, and installs the one with the lowest median for
 * (p->block, p->search_range) as xv_set_me_geometry would.
 * Coded outputs never depend on the geometry.  Synchronises hip_stream; out
 * (optional) receives the chosen geometry and *best_ms (optional) its
 * median kernel time.  Errors: XV_EINVAL (also for a cube with T < 2), XV_ENOMEM,
 * XV_EHIP. */
int xv_autotune_me(const xv_cube* in, const xv_params* p, void* hip_stream, int max_candidates,
                   xv_me_geometry* out, double* best_ms);
/* The same over the first P-picture step of a batch coded together, as
 * xv_encode_batch would launch it: n cubes with their params, which must
 * all share block and search_range.  Tuning on the batch that will run
 * accounts for its grid size, which changes the best geometry.  With
 * XV_FLAG_SPLIT in every params entry (in none or all), both tuners time
 * and install the adaptive block size's search instead, as
 * xv_set_me_split_geometry would. */
int xv_autotune_me_batch(int n, const xv_cube* cubes, const xv_params* params, void* hip_stream,
                         int max_candidates, xv_me_geometry* out, double* best_ms);

/* ---- Kernel timing (HIP events on the launch stream) ------------------ */

#define XV_K_STATS 0
#define XV_K_PACK 1
#define XV_K_ME 2
#define XV_K_ENCODE 3
#define XV_K_DECODE 4
#define XV_K_DENORM 5
#define XV_K_METRICS 6
#define XV_K_BITS_WRITE 7
#define XV_K_BITS_PARSE 8
#define XV_K_QUALITY 9
#define XV_K_SUBPEL 10 /* quarter-sample refinement and motion compensation */
#define XV_K_PCA 11    /* principal components: moments, projection, inverse */
#define XV_K_INTRA 12  /* intra-predicted I pictures, one launch per wavefront */
#define XV_K_COUNT 13

typedef struct {
  double ms[XV_K_COUNT];       /* summed kernel time per kernel class     */
  uint64_t launches[XV_K_COUNT];
  double work[XV_K_COUNT];     /* algorithmic units processed: bytes for
                                  HBM-bound kernels, SAD terms for motion
                                  search                                 */
} xv_profile;

/* Enable (1) or disable (0) per-launch event timing; enabling clears the
 * counters.  Timing adds an event pair around every timed launch. */
int xv_profile_enable(int on);
/* Restrict timing to the kernel classes whose bits (1 << XV_K_*) are set in
 * class_mask; 0 times every class (the default).  Fewer timed launches cost
 * less: each event pair adds a few microseconds of queue time. */
int xv_profile_select(uint32_t class_mask);
/* Synchronises the streams that were timed and returns the totals. */
int xv_profile_read(xv_profile* out);

/* ---- bitstream -------------------------------------------------------------
 * The codes the rate proxy counts, written out: a serialised encoded cube.
 * Codes are the Exp-Golomb ue/se codes of ITU-T H.265 clause 9.2, MSB-first.
 * Payload order, frame by frame (f = g*T + t): the vectors of the frame's
 * blocks in raster order (se(dx - pdx), se(dy - pdy) with the left
 * neighbour's vector as predictor, (0,0) in column 0; nothing for I frames,
 * or one mode bit per block under XV_FLAG_INTRA; under XV_FLAG_SPLIT a P
 * block's split flag and then its one or four vectors),
 * then for channel c = 0, 1, 2 the blocks' coefficients in raster order (a
 * coded-flag bit, then ue(nnz-1) and per nonzero level in up-right diagonal
 * scan order ue(run), se(level); a split block: its four blocks' codes in
 * z-order).  The payload has exactly coef_bits +
 * mv_bits bits.  Every block row of vectors or of one channel's
 * coefficients is a segment whose bit offset is stored, so rows parse in
 * parallel.  Buffer layout (little-endian): a 256-byte header (magic
 * "XVPACK01", dims, dtype, params, offsets), the metric span (band min/max,
 * squared errors, valid counts, bit totals), the segment index (u64 bit
 * offsets, 4*Hb per frame) and the payload bytes. */
typedef struct xv_packed xv_packed;

/* Serialise an encoded cube into one device buffer on hip_stream.
 * Synchronises the stream once (the payload size comes from a device-side
 * scan of the per-block bit counts).  *out is owned by the caller
 * (xv_packed_free); e may be freed afterwards.  Errors: XV_EINVAL,
 * XV_ENOMEM, XV_EHIP. */
int xv_pack(const xv_encoded* e, void* hip_stream, xv_packed** out);
/* Device pointer and size of the serialised buffer, and the payload length
 * in bits (all outputs optional).  The buffer is valid until xv_packed_free
 * and complete once the stream passed the xv_pack call. */
int xv_packed_view(const xv_packed* p, const void** data, uint64_t* bytes,
                   uint64_t* payload_bits);
void xv_packed_free(xv_packed* p);
/* Parse a serialised cube (device memory holding what xv_pack wrote, of
 * `bytes` bytes; the caller keeps it alive during the call) into a new
 * encoded cube: levels, vectors, per-block bit counts and the metric span,
 * which xv_decode_cube and xv_psnr_bpppb accept (physical PSNR needs the
 * encoder's reconstruction and is NaN here).  Synchronises hip_stream.
 * Errors: XV_EINVAL for a header that does not describe a valid cube or a
 * payload that does not parse as the codes above (nothing is written to
 * *out then), XV_ENOMEM, XV_EHIP. */
int xv_unpack(const void* data, uint64_t bytes, void* hip_stream, xv_encoded** out);

/* ---- principal components of the bands ------------------------------------
 * Sec. II-A: a mapping rule's third entry sets how many principal components
 * (PCs) of its bands are kept, and those PCs are coded instead of the bands
 * (e.g. the first 3 PCs of R, G, B, NIR in one video); Sec. III-C codes the
 * ten SimpleS2 bands as 9 PCs, or as all 10 with the less important ones at
 * lower quality.  The paper names no algorithm; this is the stated reading,
 * for u16 cubes: every (t, y, x) is one sample of the band vector; the mean
 * m and population covariance C come from exact integer sums of the samples
 * and their pairwise products (independent of summation order), with
 * m_b = S_b / n and C_bc = ((n Q_bc - S_b S_c) / n) / n in binary64; the
 * eigenvectors come from the cyclic Jacobi method, eigenvalues decreasing,
 * each eigenvector's largest component positive.  PC j of a sample is
 * y_j = sum_b V[b][j] (x_b - m_b) in binary64 (b increasing), stored as
 * binary32; the inverse from the first k PCs is
 * x_b = m_b + sum_{j<k} V[b][j] y_j (j increasing), rounded like a decode.
 * A PC cube is an ordinary XV_F32 cube: encode it with xv_encode_cube (or
 * several PC ranges with different QPs with xv_encode_batch), decode it to
 * XV_F32, then xv_pca_inverse. */
typedef struct xv_pca xv_pca;

/* Fit the PCs of a u16 device cube (1 to 64 bands).  Synchronises
 * hip_stream.  *out is owned by the caller (xv_pca_free).  Errors:
 * XV_EINVAL (null or bad cube, dtype other than XV_U16), XV_ENOMEM, XV_EHIP. */
int xv_pca_fit(const xv_cube* in, void* hip_stream, xv_pca** out);
/* Host copies of the fit (each output optional; caller memory of bands,
 * bands^2, bands and bands^2 doubles; basis[b * bands + j] is component b of
 * PC j). */
int xv_pca_view(const xv_pca* p, int32_t* bands, double* mean, double* cov, double* eigval,
                double* basis);
/* PCs j0..j1-1 of every sample of `in` (u16, the fitted band count) into pcs
 * (XV_F32, same T, H, W, j1 - j0 bands).  Asynchronous.  Errors: XV_EINVAL,
 * XV_EHIP. */
int xv_pca_project(const xv_pca* p, const xv_cube* in, int32_t j0, int32_t j1,
                   const xv_cube* pcs, void* hip_stream);
/* Bands from the first k = pcs->bands PCs (XV_F32) into out (XV_U16:
 * nearest integer, halves up, clamped; XV_F32: nearest float; the fitted
 * band count).  Asynchronous.  Errors: XV_EINVAL, XV_EHIP. */
int xv_pca_inverse(const xv_pca* p, const xv_cube* pcs, const xv_cube* out, void* hip_stream);
void xv_pca_free(xv_pca* p);

/* ---- device memory ---------------------------------------------------------
 * Every device buffer of the library comes from one caching allocator per
 * process.  A freed buffer (xv_encoded_free, the end of a decode, a dropped
 * work buffer) is kept for reuse instead of being returned to the runtime:
 * immediately by later work on the stream it was freed on, and by work on
 * any other stream once everything queued on that stream before the free has
 * completed.  A stream handed to the library must therefore stay alive until
 * the objects used on it are freed and that work has completed.  Memory goes
 * back to the runtime only when an allocation fails for lack of it (cached
 * blocks are released and the allocation retried) or on xv_cache_release. */
typedef struct xv_memory {
  uint64_t live_bytes;    /* held by live objects and in-flight calls */
  uint64_t cached_bytes;  /* freed, kept for reuse */
  uint64_t peak_bytes;    /* maximum of live_bytes since the library loaded */
} xv_memory;

int xv_memory_read(xv_memory* out);
/* Waits for the last use of every cached block and returns it to the
 * runtime; *released_bytes (may be NULL) receives the total. */
int xv_cache_release(uint64_t* released_bytes);

#ifdef __cplusplus
}
#endif
#endif
