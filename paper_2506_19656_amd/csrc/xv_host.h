// xv_host.h -- declarations shared by the host-side translation units of
// libxv (not part of the public ABI): the encoded-cube object, error
// reporting, launch timing, the motion-search geometry table, and the
// encode / decode sequencing that the plain, batched, tuning and serving
// entry points are built from.
#pragma once

#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "xv_internal.h"

struct xv_encoded {
  int64_t T, H, W, bands;
  int G, N, Hp, Wp, Hb, Wb, nsteps;
  int64_t njobs;
  xv_params p;
  int src_dtype;
  hipStream_t stream;
  void* keep;  // levels, vectors, bit counts, statistics, job table
  void* work;  // converted frames, reconstruction, validity bytes, per-tile sums
  unsigned long long* tile_part;  // [G][T][tpf][kTileSums] per-tile sums of the transform kernel
  int tpf;                        // transform tiles per frame
  unsigned long long* tot_chunk;  // [G][kTotMaxChunks][5] chunk sums of the totals, in work
  uint16_t* frames;
  uint16_t* recon;
  uint8_t* vmask;
  uint16_t* pred;  // prediction planes, one per stream (XV_FLAG_QPEL or XV_FLAG_INTRA), in work
  int16_t* levels;
  int8_t* mvs;
  uint32_t* cbits;
  uint32_t* mbits;
  uint32_t* stats_part;  // [kStatsMaxBlocks][3][bands] per-block statistics
  uint32_t* nan_count;
  uint32_t* nan_total;
  // metric span, contiguous (one copy to the host): mn, mx, phys [bands]
  // doubles; nvalid [bands], sse [3G], bits [2G] u64
  void* span;
  size_t span_bytes;
  double* mn;
  double* mx;
  double* phys;
  unsigned long long* nvalid;
  unsigned long long* sse;   // [3G]
  unsigned long long* bits;  // [2G]
  double* phys_partial;      // [phys_blocks][bands]
  int phys_nb;
  xv::FrameJob* jobs;
  // adaptive block size (XV_FLAG_SPLIT), else null: split flags [G][T][Hb][Wb]
  // (keep); the whole blocks' vectors and SADs and the cells' SADs (work)
  uint8_t* splits;
  int8_t* mv_whole;
  uint32_t* sad_whole;
  uint32_t* sad_cell;
};

namespace xv {
namespace host {

// ---- errors: the thread-local text behind xv_last_error --------------------
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
const char* last_error();

#define XV_HIP(call, what)                           \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return ::xv::host::hip_fail(e_, what); \
  } while (0)

struct Carve {
  size_t off = 0;
  template <class T>
  size_t take(size_t count) {
    size_t o = (off + 255) & ~(size_t)255;
    off = o + count * sizeof(T);
    return o;
  }
};

// ---- per-launch event timing (xv_profile_*) ---------------------------------
// Records an event pair around the launches issued during its lifetime when
// timing is enabled for class c; `work` is the launch's algorithmic work.
struct ProfScope {
  int cls;
  hipStream_t s;
  double work;
  hipEvent_t a = nullptr, b = nullptr;
  bool on;
  ProfScope(int c, hipStream_t st, double w);
  ~ProfScope();
};

// True while per-launch event timing is enabled (xv_profile_enable).
bool profiling_enabled();

// ---- motion-search geometry table --------------------------------------------
// Explicit geometries (xv_set_me_geometry, the tuner) per (N, R); otherwise
// the model default for the class's widest frame in blocks.
MeGeom geometry_for(int N, int R, int Wb = 16);
void geometry_install(int N, int R, const MeGeom& g);
// The same for the adaptive block size's combined search
// (xv_set_me_split_geometry, the tuner on XV_FLAG_SPLIT params).
MeGeom split_geometry_for(int N, int R, int Wb = 16);
void split_geometry_install(int N, int R, const MeGeom& g);

// ---- validation ----------------------------------------------------------------
int check_cube(const xv_cube* c, const char* name);
int check_params(const xv_params* p);

// ---- encode ----------------------------------------------------------------------
void dims_of(xv_encoded* e, const xv_cube* in, const xv_params* p);

// Device layout of an encoded cube: "keep" (levels, vectors, bit counts,
// statistics, metric span, job table) and "work" (converted frames,
// reconstruction, validity bytes).  Offsets in bytes.
struct EncLayout {
  size_t o_lev, o_mv, o_cb, o_mb, o_keys, o_span, o_pp, o_jobs, o_split, keep;
  size_t o_fr, o_rc, o_vm, o_part, o_tot, o_pred, o_mvw, o_sadw, o_sadc, work;
  size_t span_words;
  int phys_nb;
};
EncLayout enc_layout(const xv_encoded* e);
// Transform tiles per frame: the size-N kernel's, plus with the adaptive
// block size the size-N/2 kernel's (its tile sums follow).
int tiles_per_frame(const xv_encoded* e);
// The whole/split cost multiplier in 1/16 SAD units.
int32_t split_lambda16(int qp, int bit_depth);
size_t decode_bytes(const xv_encoded* e);
void bind_keep(xv_encoded* e, const EncLayout& lay);
int encode_prepare(const xv_cube* in, const xv_params* p, hipStream_t s, xv_encoded** out);
// SAD terms of motion-search step s at block size n (0: the cube's N).
double me_work(const xv_encoded* e, int s, int n = 0);
double xf_frames(const xv_encoded* e, int s);

struct SegSrc {
  xv_encoded* e;
  int step;
};

struct DecSrc {
  const xv_encoded* e;
  xv::FrameJob* jobs;
  int step;
};

// One launch per chunk of up to kMaxSeg segments.
template <class F>
int launch_segments(const std::vector<SegSrc>& src, int tpj_kind, const MeGeom& geom, F launch) {
  size_t i = 0;
  while (i < src.size()) {
    LaunchDesc d;
    memset(&d, 0, sizeof d);
    int tiles = 0;
    double work = 0;
    for (; i < src.size() && d.nseg < kMaxSeg; i++) {
      xv_encoded* e = src[i].e;
      const int s = src[i].step;
      const int n = plan_jobs_at((int)e->T, e->G, e->p.gop, s);
      int tpj = tpj_kind == 0 ? xf_tiles_per_job(e->N, e->Hb, e->Wb)
                              : me_tiles_per_job(e->Hb, e->Wb, geom);
      Seg& g = d.seg[d.nseg++];
      g.jobs = e->jobs + plan_step_offset((int)e->T, e->G, e->p.gop, s);
      g.count = n;
      g.tpj = tpj;
      g.tile0 = tiles;
      tiles += n * tpj;
      // transform: algorithmic bytes (cur + pred in, level + recon out, 8 B per
      // sample; an I step without intra modes has a constant prediction, 6 B);
      // search: SAD terms
      const bool const_pred = s == 0 && !(e->p.flags & XV_FLAG_INTRA);
      work += tpj_kind == 0 ? xf_frames(e, s) * 3.0 * e->Hp * e->Wp * (const_pred ? 6.0 : 8.0)
                            : me_work(e, s);
    }
    d.tiles = tiles;
    int rc = launch(d, work);
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

// One launch per chunk of up to kMaxSeg sources, with each source's job
// table (of step 0), tiles per job and work given by the caller.
template <class Src, class Jobs, class Tpj, class Work, class F>
int launch_chunks(const std::vector<Src>& src, Jobs jobs_of, Tpj tpj_of, Work work_of, F launch) {
  size_t i = 0;
  while (i < src.size()) {
    LaunchDesc d;
    memset(&d, 0, sizeof d);
    int tiles = 0;
    double work = 0;
    for (; i < src.size() && d.nseg < kMaxSeg; i++) {
      const xv_encoded* e = src[i].e;
      const int st = src[i].step;
      Seg& g = d.seg[d.nseg++];
      g.jobs = jobs_of(src[i]) + plan_step_offset((int)e->T, e->G, e->p.gop, st);
      g.count = plan_jobs_at((int)e->T, e->G, e->p.gop, st);
      g.tpj = tpj_of(e);
      g.tile0 = tiles;
      tiles += g.count * g.tpj;
      work += work_of(src[i]);
    }
    d.tiles = tiles;
    int rc = launch(d, work);
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

// Adaptive block size (sources with XV_FLAG_SPLIT, one class): the P step's
// searches at N and N/2 and the whole-or-split choice; the step's transform
// coding (size-N kernel, then size-N/2 kernel); the decode of a step.
int launch_split_search(const std::vector<SegSrc>& src, hipStream_t s);
int launch_split_transform(const std::vector<SegSrc>& src, hipStream_t s);
int launch_split_decode(const std::vector<DecSrc>& src, hipStream_t s);

int encode_steps(std::vector<xv_encoded*>& es, hipStream_t s);
int finish_encode(xv_encoded* e);

// ---- decode ----------------------------------------------------------------------
int check_decode_out(const xv_encoded* e, const xv_cube* out);

struct DecodeBuf {
  void* mem = nullptr;
  uint16_t* recon = nullptr;
  uint16_t* pred = nullptr;  // prediction planes (quarter-sample vectors only)
  FrameJob* jobs = nullptr;
};
int decode_prepare(const xv_encoded* e, hipStream_t s, DecodeBuf& db);

int decode_launch(const std::vector<DecSrc>& src, hipStream_t s);
// Quarter-sample motion of one frame step: refinement of the integer vectors
// (encode) or the prediction planes from stored vectors (decode), over the
// sources coded with XV_FLAG_QPEL (step > 0); *launches counts launches.
int launch_subpel_step(const std::vector<SegSrc>& src, hipStream_t s, uint64_t* launches);
int launch_mc_step(const std::vector<DecSrc>& src, hipStream_t s, uint64_t* launches);
// Intra-predicted I steps (XV_FLAG_INTRA), one launch per wavefront, over
// the sources at step 0 that carry the flag: encode (mode choice, coding,
// reconstruction and prediction plane; the transform launch of the step
// follows) and decode (reconstruction; decode_launch skips these steps).
int launch_intra_step(const std::vector<SegSrc>& src, hipStream_t s, uint64_t* launches);
int launch_intra_decode_step(const std::vector<DecSrc>& src, hipStream_t s, uint64_t* launches);
// Bytes of the prediction planes: one [3][Hp][Wp] plane per stream.
size_t pred_plane_bytes(const xv_encoded* e);
int decode_steps(std::vector<DecSrc> base, hipStream_t s);
int decode_finish(const xv_encoded* e, const xv_cube* out, DecodeBuf& db, hipStream_t s);

// ---- graph replay of the step loops (xv_graph.cpp) ----------------------------
// With graph mode on (xv_set_graph_mode) and timing off, the batched paths
// replay a captured graph of the step loop instead of launching it.
bool graphs_enabled();
int encode_steps_graph(std::vector<xv_encoded*>& es, hipStream_t s);
int decode_steps_graph(const std::vector<DecSrc>& base, hipStream_t s);
size_t graph_cache_release();

}  // namespace host
}  // namespace xv
