// xv_api.cpp -- host runtime behind the C ABI of include/xv.h.
//
// Responsibilities: argument validation, device allocation (stream-ordered,
// from the device's default memory pool), launch sequencing of the coding
// loop (stats -> pack -> plan -> for every frame step: motion search (P) and
// fused transform coding), decode, metrics, the batched multi-cube path,
// per-launch event timing and the motion-search launch geometry table.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>
#include <cstdarg>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "xv_internal.h"

using namespace xv;

struct xv_encoded {
  int64_t T, H, W, bands;
  int G, N, Hp, Wp, Hb, Wb, nsteps;
  int64_t njobs;
  xv_params p;
  int src_dtype;
  hipStream_t stream;
  void* keep;  // levels, vectors, bit counts, statistics, job table
  void* work;  // converted frames, reconstruction, validity bytes, per-tile sums
  unsigned long long* tile_part;  // [G][T][tpf][5] per-tile sums of the transform kernel
  int tpf;                        // transform tiles per frame
  uint16_t* frames;
  uint16_t* recon;
  uint8_t* vmask;
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
  FrameJob* jobs;
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(XV_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(XV_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define XV_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
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

// ---- profiling ----------------------------------------------------------------
struct ProfRec {
  int cls;
  hipEvent_t a, b;
  double work;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
uint32_t g_prof_mask = ~0u;           // classes timed while enabled
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_events;  // idle events, reused across launches
xv_profile g_prof_tot;

hipEvent_t prof_event_locked() {
  if (!g_prof_events.empty()) {
    hipEvent_t e = g_prof_events.back();
    g_prof_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct ProfScope {
  int cls;
  hipStream_t s;
  double work;
  hipEvent_t a = nullptr, b = nullptr;
  bool on;
  ProfScope(int c, hipStream_t st, double w) : cls(c), s(st), work(w) {
    on = g_prof_on && ((g_prof_mask >> c) & 1u);
    if (on) {
      {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        a = prof_event_locked();
        b = prof_event_locked();
      }
      (void)hipEventRecord(a, s);
    }
  }
  ~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back(ProfRec{cls, a, b, work});
  }
};

// ---- motion-search geometry table -----------------------------------------
// Explicit geometries (xv_set_me_geometry) per (N, R); otherwise the model
// default for the class's widest frame in blocks, cached per (N, R, Wb).
std::mutex g_geom_mu;
std::map<std::pair<int, int>, MeGeom> g_geom;
std::map<std::tuple<int, int, int>, MeGeom> g_geom_default;

MeGeom geometry_for(int N, int R, int Wb = 16) {
  std::lock_guard<std::mutex> lk(g_geom_mu);
  auto it = g_geom.find({N, R});
  if (it != g_geom.end()) return it->second;
  const int wb = std::max(1, std::min(16, Wb));
  auto d = g_geom_default.find({N, R, wb});
  if (d != g_geom_default.end()) return d->second;
  MeGeom g = me_default_geometry(N, R, wb);
  g_geom_default[{N, R, wb}] = g;
  return g;
}

// ---- validation -----------------------------------------------------------
int check_cube(const xv_cube* c, const char* name) {
  if (!c) return fail(XV_EINVAL, "%s: null cube", name);
  if (!c->data) return fail(XV_EINVAL, "%s: null data pointer", name);
  if (c->dtype != XV_U16 && c->dtype != XV_F32) return fail(XV_EINVAL, "%s: bad dtype %d", name, c->dtype);
  if (c->T < 1 || c->H < 1 || c->W < 1 || c->bands < 1)
    return fail(XV_EINVAL, "%s: shape must be positive", name);
  if (c->bands > XV_MAX_BANDS) return fail(XV_EINVAL, "%s: more than %d bands", name, XV_MAX_BANDS);
  if (c->H > 65536 || c->W > 65536 || c->T > (1 << 24) ||
      (double)c->T * (double)c->H * (double)c->W >= 4294967296.0)
    return fail(XV_EINVAL, "%s: dimension too large (T*H*W must be below 2^32)", name);
  // a padded 3-channel u16 frame must stay addressable with 32-bit byte offsets
  if ((double)(c->H + 31) * (double)(c->W + 31) * 6.0 >= 2147483648.0)
    return fail(XV_EINVAL, "%s: frame too large ((H+31)*(W+31) must be below 2^31/6)", name);
  const size_t el = c->dtype == XV_U16 ? 2 : 4;
  if (((uintptr_t)c->data) % el) return fail(XV_EINVAL, "%s: misaligned data pointer", name);
  return XV_OK;
}

int check_params(const xv_params* p) {
  if (!p) return fail(XV_EINVAL, "null params");
  const int B = p->bit_depth, N = p->block;
  if (B < 8 || B > 12) return fail(XV_EINVAL, "bit_depth %d not in 8..12", B);
  if (!(N == 4 || N == 8 || N == 16 || N == 32)) return fail(XV_EINVAL, "block %d not in {4,8,16,32}", N);
  if (p->qp < -6 * (B - 8) || p->qp > 51) return fail(XV_EINVAL, "qp %d outside %d..51", p->qp, -6 * (B - 8));
  if (p->search_range < 0 || p->search_range > 64) return fail(XV_EINVAL, "search_range %d not in 0..64", p->search_range);
  if (p->gop < 1) return fail(XV_EINVAL, "gop must be >= 1");
  if (p->pad_mode != XV_PAD_ZERO && p->pad_mode != XV_PAD_REPEAT) return fail(XV_EINVAL, "bad pad_mode");
  if (p->fill_mode != XV_FILL_NEAREST && p->fill_mode != XV_FILL_FORWARD) return fail(XV_EINVAL, "bad fill_mode");
  if (p->flags & ~XV_FLAG_DROP_WORK) return fail(XV_EINVAL, "unknown flags");
  return XV_OK;
}

// ---- encode -----------------------------------------------------------------
void dims_of(xv_encoded* e, const xv_cube* in, const xv_params* p) {
  e->T = in->T;
  e->H = in->H;
  e->W = in->W;
  e->bands = in->bands;
  e->G = (int)((in->bands + 2) / 3);
  e->N = p->block;
  e->Hp = (int)((in->H + p->block - 1) / p->block * p->block);
  e->Wp = (int)((in->W + p->block - 1) / p->block * p->block);
  e->Hb = e->Hp / e->N;
  e->Wb = e->Wp / e->N;
  e->nsteps = (int)std::min<int64_t>(p->gop, in->T);
  e->njobs = plan_step_offset((int)e->T, e->G, p->gop, e->nsteps);
  e->p = *p;
  e->src_dtype = in->dtype;
}

// Device layout of an encoded cube: "keep" (levels, vectors, bit counts,
// statistics, metric span, job table) and "work" (converted frames,
// reconstruction, validity bytes).  Offsets in bytes.
struct EncLayout {
  size_t o_lev, o_mv, o_cb, o_mb, o_keys, o_span, o_pp, o_jobs, keep;
  size_t o_fr, o_rc, o_vm, o_part, work;
  size_t span_words;
  int phys_nb;
};

EncLayout enc_layout(const xv_encoded* e) {
  EncLayout L{};
  const int64_t G = e->G, T = e->T;
  const int64_t plane = (int64_t)e->Hp * e->Wp;
  const int64_t nframes = G * T;
  const int64_t nblk = nframes * e->Hb * e->Wb;
  const int64_t bands = e->bands;
  Carve k;
  L.o_lev = k.take<int16_t>((size_t)nframes * 3 * plane);
  L.o_mv = k.take<int8_t>((size_t)nblk * 2);
  L.o_cb = k.take<uint32_t>((size_t)nblk * 3);
  L.o_mb = k.take<uint32_t>((size_t)nblk);
  L.o_keys = k.take<uint32_t>((size_t)bands + 1 + (size_t)kStatsMaxBlocks * 3 * bands);
  L.span_words = (size_t)3 * bands + bands + 3 * G + 2 * G;
  L.o_span = k.take<uint64_t>(L.span_words);
  L.phys_nb = phys_blocks(T * e->H * e->W * bands);
  L.o_pp = k.take<double>((size_t)L.phys_nb * bands);
  L.o_jobs = k.take<FrameJob>((size_t)e->njobs);
  L.keep = k.off;
  Carve w;
  L.o_fr = w.take<uint16_t>((size_t)nframes * 3 * plane);
  L.o_rc = w.take<uint16_t>((size_t)nframes * 3 * plane);
  L.o_vm = e->src_dtype == XV_F32 ? w.take<uint8_t>((size_t)nframes * 3 * plane) : 0;
  L.o_part = w.take<uint64_t>((size_t)nframes * xf_tiles_per_job(e->N, e->Hb, e->Wb) * 5);
  L.work = w.off;
  return L;
}

[[maybe_unused]] size_t decode_bytes(const xv_encoded* e) {
  Carve c;
  c.take<uint16_t>((size_t)e->G * e->T * 3 * (size_t)e->Hp * e->Wp);
  c.take<FrameJob>((size_t)e->njobs);
  return c.off;
}

// Pointers into the keep buffer (levels, vectors, bit counts, statistics,
// metric span, job table).
void bind_keep(xv_encoded* e, const EncLayout& lay) {
  const int64_t bands = e->bands, G = e->G;
  char* kb = (char*)e->keep;
  e->levels = (int16_t*)(kb + lay.o_lev);
  e->mvs = (int8_t*)(kb + lay.o_mv);
  e->cbits = (uint32_t*)(kb + lay.o_cb);
  e->mbits = (uint32_t*)(kb + lay.o_mb);
  e->nan_count = (uint32_t*)(kb + lay.o_keys);
  e->nan_total = e->nan_count + bands;
  e->stats_part = e->nan_total + 1;
  e->span = kb + lay.o_span;
  e->span_bytes = lay.span_words * 8;
  e->mn = (double*)e->span;
  e->mx = e->mn + bands;
  e->phys = e->mx + bands;
  e->nvalid = (unsigned long long*)(e->phys + bands);
  e->sse = e->nvalid + bands;
  e->bits = e->sse + 3 * G;
  e->phys_partial = (double*)(kb + lay.o_pp);
  e->jobs = (FrameJob*)(kb + lay.o_jobs);
}

// Allocates the encoded object and launches stats, pack and plan.
int encode_prepare(const xv_cube* in, const xv_params* p, hipStream_t s, xv_encoded** out) {
  xv_encoded* e = new (std::nothrow) xv_encoded();
  if (!e) return fail(XV_ENOMEM, "host allocation failed");
  memset(e, 0, sizeof *e);
  dims_of(e, in, p);
  e->stream = s;
  const int64_t G = e->G, T = e->T;
  const int64_t plane = (int64_t)e->Hp * e->Wp;
  const int64_t nframes = G * T;
  const int64_t bands = e->bands;
  const EncLayout lay = enc_layout(e);
  struct {
    size_t off;
  } k{lay.keep}, w{lay.work};
  const size_t o_fr = lay.o_fr, o_rc = lay.o_rc, o_vm = lay.o_vm, o_part = lay.o_part;
  e->phys_nb = lay.phys_nb;

  hipError_t he = dev_alloc(&e->keep, k.off, s);
  if (he != hipSuccess) {
    delete e;
    return hip_fail(he, "device allocation of the encoded cube");
  }
  he = dev_alloc(&e->work, w.off, s);
  if (he != hipSuccess) {
    dev_free(e->keep, s);
    delete e;
    return hip_fail(he, "device allocation of the coding work buffers");
  }
  bind_keep(e, lay);
  char* wb = (char*)e->work;
  e->frames = (uint16_t*)(wb + o_fr);
  e->recon = (uint16_t*)(wb + o_rc);
  e->vmask = in->dtype == XV_F32 ? (uint8_t*)(wb + o_vm) : nullptr;
  e->tile_part = (unsigned long long*)(wb + o_part);
  e->tpf = xf_tiles_per_job(e->N, e->Hb, e->Wb);
  *out = e;

  const double elb = in->dtype == XV_U16 ? 2.0 : 4.0;
  const double in_bytes = (double)T * e->H * e->W * bands * elb;
  {
    StatsArgs a{in->data, in->dtype, ((uintptr_t)in->data & 15) == 0, T * e->H * e->W,
                (int32_t)bands, 0, e->stats_part, e->nan_count, e->nan_total, e->mn, e->mx,
                e->nvalid};
    ProfScope ps(XV_K_STATS, s, in_bytes);
    XV_HIP(launch_stats(a, s), "stats kernel");
  }
  {
    PackArgs a{in->data, in->dtype, T, e->H, e->W, (int32_t)bands, e->G, e->Hp, e->Wp,
               p->bit_depth, p->pad_mode, p->fill_mode, e->mn, e->mx, e->nan_total,
               e->nan_count, e->frames, e->vmask, chunk_px_for(e->Wp, (int)bands)};
    ProfScope ps(XV_K_PACK, s, in_bytes + (double)nframes * 3 * plane * 2.0);
    XV_HIP(launch_pack(a, s), "pack kernel");
  }
  {
    CubePlan pl{e->frames, e->recon, e->levels, e->mvs, e->cbits, e->mbits, e->vmask,
                e->nan_total, e->tile_part, e->jobs, (int32_t)T, e->G, p->gop, e->nsteps,
                e->Hp, e->Wp, (int32_t)e->H, (int32_t)e->W, (int32_t)bands, e->N,
                p->bit_depth, p->qp, e->tpf};
    XV_HIP(launch_plan(pl, s), "plan kernel");
  }
  return XV_OK;
}

// SAD terms of a motion-search launch: (2R+1)^2 per real-channel sample.
// SAD terms of one motion-search step: every candidate that keeps the
// displaced block inside the padded picture, N^2 terms per real channel.
double me_work(const xv_encoded* e, int s) {
  const int R = e->p.search_range, N = e->N;
  auto axis = [&](int P) {  // sum over block positions of the admissible displacements
    double tot = 0;
    for (int x0 = 0; x0 + N <= P; x0 += N) tot += std::min(R, P - N - x0) - std::max(-R, -x0) + 1;
    return tot;
  };
  const int nk = (int)((e->T - s + e->p.gop - 1) / e->p.gop);
  double ch = 0;
  for (int g = 0; g < e->G; g++) ch += std::min<int64_t>(3, e->bands - 3 * g);
  return axis(e->Hp) * axis(e->Wp) * (double)N * N * ch * nk;
}

double xf_frames(const xv_encoded* e, int s) {
  const int nk = (int)((e->T - s + e->p.gop - 1) / e->p.gop);
  return (double)e->G * nk;
}

struct SegSrc {
  xv_encoded* e;
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
      // sample; an I step has a constant prediction, 6 B); search: SAD terms
      work += tpj_kind == 0 ? xf_frames(e, s) * 3.0 * e->Hp * e->Wp * (s == 0 ? 6.0 : 8.0)
                            : me_work(e, s);
    }
    d.tiles = tiles;
    int rc = launch(d, work);
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

// Frame-step loop over a set of encodes that share N and R.
int encode_steps(std::vector<xv_encoded*>& es, hipStream_t s) {
  if (es.empty()) return XV_OK;
  const int N = es[0]->N, R = es[0]->p.search_range;
  int max_wb = 1;
  for (auto* e : es) max_wb = std::max(max_wb, e->Wb);
  const MeGeom geom = geometry_for(N, R, max_wb);
  int maxsteps = 0;
  for (auto* e : es) maxsteps = std::max(maxsteps, e->nsteps);
  for (int st = 0; st < maxsteps; st++) {
    std::vector<SegSrc> src;
    for (auto* e : es)
      if (st < e->nsteps) src.push_back(SegSrc{e, st});
    if (st > 0) {
      int rc = launch_segments(src, 1, geom, [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ME, s, work);
        XV_HIP(launch_me(N, R, geom, d, s), "motion search kernel");
        return XV_OK;
      });
      if (rc != XV_OK) return rc;
    }
    int rc = launch_segments(src, 0, geom, [&](const LaunchDesc& d, double work) {
      ProfScope ps(XV_K_ENCODE, s, work);
      XV_HIP(launch_encode(N, d, s), "transform kernel");
      return XV_OK;
    });
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

// After the last step: per-group totals from the per-tile sums, then the
// work buffers go if the caller asked for that.
int finish_encode(xv_encoded* e) {
  XV_HIP(launch_encode_totals(e->tile_part, e->G, (int)e->T, e->tpf, e->sse, e->bits, e->stream),
         "encode totals kernel");
  if (e->p.flags & XV_FLAG_DROP_WORK) {
    dev_free(e->work, e->stream);
    e->work = nullptr;
    e->tile_part = nullptr;
    e->frames = nullptr;
    e->recon = nullptr;
    e->vmask = nullptr;
  }
  return XV_OK;
}

// ---- decode -----------------------------------------------------------------
int check_decode_out(const xv_encoded* e, const xv_cube* out) {
  int rc = check_cube(out, "decode output");
  if (rc != XV_OK) return rc;
  if (out->T != e->T || out->H != e->H || out->W != e->W || out->bands != e->bands)
    return fail(XV_EINVAL, "decode output shape differs from the encoded cube");
  return XV_OK;
}

struct DecodeBuf {
  void* mem = nullptr;
  uint16_t* recon = nullptr;
  FrameJob* jobs = nullptr;
};

int decode_prepare(const xv_encoded* e, hipStream_t s, DecodeBuf& db) {
  Carve c;
  const int64_t plane = (int64_t)e->Hp * e->Wp;
  size_t o_rc = c.take<uint16_t>((size_t)e->G * e->T * 3 * plane);
  size_t o_jb = c.take<FrameJob>((size_t)e->njobs);
  db.mem = nullptr;
  XV_HIP(dev_alloc(&db.mem, c.off, s), "device allocation of the decode buffers");
  db.recon = (uint16_t*)((char*)db.mem + o_rc);
  db.jobs = (FrameJob*)((char*)db.mem + o_jb);
  CubePlan pl{nullptr, db.recon, e->levels, e->mvs, nullptr, nullptr, nullptr, nullptr,
              nullptr, db.jobs, (int32_t)e->T, e->G, e->p.gop, e->nsteps,
              e->Hp, e->Wp, (int32_t)e->H, (int32_t)e->W, (int32_t)e->bands, e->N,
              e->p.bit_depth, e->p.qp, 0};
  XV_HIP(launch_plan(pl, s), "plan kernel");
  return XV_OK;
}

struct DecSrc {
  const xv_encoded* e;
  FrameJob* jobs;
  int step;
};

// One launch per chunk of segments; each source brings its own step.
int decode_launch(const std::vector<DecSrc>& src, hipStream_t s) {
  if (src.empty()) return XV_OK;
  const int N = src[0].e->N;
  size_t i = 0;
  while (i < src.size()) {
    LaunchDesc d;
    memset(&d, 0, sizeof d);
    int tiles = 0;
    double work = 0;
    for (; i < src.size() && d.nseg < kMaxSeg; i++) {
      const xv_encoded* e = src[i].e;
      const int st = src[i].step;
      const int n = plan_jobs_at((int)e->T, e->G, e->p.gop, st);
      const int tpj = xf_tiles_per_job(e->N, e->Hb, e->Wb);
      Seg& g = d.seg[d.nseg++];
      g.jobs = src[i].jobs + plan_step_offset((int)e->T, e->G, e->p.gop, st);
      g.count = n;
      g.tpj = tpj;
      g.tile0 = tiles;
      tiles += n * tpj;
      // level + pred in, recon out: 6 B per sample (an I step has no pred read)
      work += (double)n * 3.0 * e->Hp * e->Wp * (st == 0 ? 4.0 : 6.0);
    }
    d.tiles = tiles;
    ProfScope ps(XV_K_DECODE, s, work);
    XV_HIP(launch_decode(N, d, s), "decode kernel");
  }
  return XV_OK;
}

int decode_steps(std::vector<DecSrc> base, hipStream_t s) {
  if (base.empty()) return XV_OK;
  int maxsteps = 0;
  for (auto& b : base) maxsteps = std::max(maxsteps, b.e->nsteps);
  for (int st = 0; st < maxsteps; st++) {
    std::vector<DecSrc> src;
    for (auto& b : base)
      if (st < b.e->nsteps) src.push_back(DecSrc{b.e, b.jobs, st});
    int rc = decode_launch(src, s);
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

int decode_finish(const xv_encoded* e, const xv_cube* out, DecodeBuf& db, hipStream_t s) {
  DenormArgs a{db.recon, e->T, e->H, e->W, (int32_t)e->bands, e->Hp, e->Wp, e->p.bit_depth,
               e->mn, e->mx, out->dtype, out->data, chunk_px_for(e->W, (int)e->bands)};
  const double ob = out->dtype == XV_U16 ? 2.0 : 4.0;
  {
    ProfScope ps(XV_K_DENORM, s, (double)e->T * e->H * e->W * e->bands * (2.0 + ob));
    XV_HIP(launch_denorm(a, s), "denormalise kernel");
  }
  dev_free(db.mem, s);
  db.mem = nullptr;
  return XV_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

int xv_abi_version(void) { return XV_ABI_VERSION; }

const char* xv_status_str(int st) {
  switch (st) {
    case XV_OK: return "ok";
    case XV_EINVAL: return "invalid argument";
    case XV_ENOMEM: return "out of device memory";
    case XV_EHIP: return "HIP runtime error";
    case XV_EBUSY: return "busy";
    case XV_ECANCELED: return "cancelled";
    case XV_EPENDING: return "pending";
    default: return "unknown status";
  }
}

const char* xv_last_error(void) { return g_err.c_str(); }

int xv_encode_cube(const xv_cube* in, const xv_params* p, void* hip_stream, xv_encoded** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  int rc = check_cube(in, "input");
  if (rc != XV_OK) return rc;
  if ((rc = check_params(p)) != XV_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  xv_encoded* e = nullptr;
  if ((rc = encode_prepare(in, p, s, &e)) != XV_OK) {
    if (e) xv_encoded_free(e);
    return rc;
  }
  std::vector<xv_encoded*> es{e};
  if ((rc = encode_steps(es, s)) != XV_OK) {
    xv_encoded_free(e);
    return rc;
  }
  if ((rc = finish_encode(e)) != XV_OK) {
    xv_encoded_free(e);
    return rc;
  }
  *out = e;
  return XV_OK;
}

int xv_encode_batch(int n, const xv_cube* cubes, const xv_params* params, void* hip_stream,
                    xv_encoded** outs) {
  if (n < 0 || (n > 0 && (!cubes || !params || !outs))) return fail(XV_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; i++) outs[i] = nullptr;
  for (int i = 0; i < n; i++) {
    int rc = check_cube(&cubes[i], "batch input");
    if (rc != XV_OK) return rc;
    if ((rc = check_params(&params[i])) != XV_OK) return rc;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<xv_encoded*> all(n, nullptr);
  auto cleanup = [&](int rc) {
    for (auto* e : all)
      if (e) xv_encoded_free(e);
    return rc;
  };
  for (int i = 0; i < n; i++) {
    int rc = encode_prepare(&cubes[i], &params[i], s, &all[i]);
    if (rc != XV_OK) return cleanup(rc);
  }
  // one step loop per (N, R) class; classes are independent
  std::map<std::pair<int, int>, std::vector<xv_encoded*>> cls;
  for (auto* e : all) cls[{e->N, e->p.search_range}].push_back(e);
  for (auto& kv : cls) {
    int rc = encode_steps(kv.second, s);
    if (rc != XV_OK) return cleanup(rc);
  }
  for (int i = 0; i < n; i++) {
    int rc = finish_encode(all[i]);
    if (rc != XV_OK) return cleanup(rc);
  }
  for (int i = 0; i < n; i++) outs[i] = all[i];
  return XV_OK;
}

int xv_decode_cube(const xv_encoded* e, const xv_cube* out, void* hip_stream) {
  if (!e) return fail(XV_EINVAL, "null encoded cube");
  int rc = check_decode_out(e, out);
  if (rc != XV_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  DecodeBuf db;
  if ((rc = decode_prepare(e, s, db)) != XV_OK) return rc;
  std::vector<DecSrc> src{DecSrc{e, db.jobs, 0}};
  if ((rc = decode_steps(src, s)) != XV_OK) {
    dev_free(db.mem, s);
    return rc;
  }
  return decode_finish(e, out, db, s);
}

int xv_decode_batch(int n, xv_encoded* const* encs, const xv_cube* outs, void* hip_stream) {
  if (n < 0 || (n > 0 && (!encs || !outs))) return fail(XV_EINVAL, "bad batch arguments");
  for (int i = 0; i < n; i++) {
    if (!encs[i]) return fail(XV_EINVAL, "null encoded cube in batch");
    int rc = check_decode_out(encs[i], &outs[i]);
    if (rc != XV_OK) return rc;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<DecodeBuf> bufs(n);
  auto cleanup = [&](int rc) {
    for (auto& b : bufs)
      if (b.mem) dev_free(b.mem, s);
    return rc;
  };
  for (int i = 0; i < n; i++) {
    int rc = decode_prepare(encs[i], s, bufs[i]);
    if (rc != XV_OK) return cleanup(rc);
  }
  std::map<int, std::vector<DecSrc>> cls;
  for (int i = 0; i < n; i++) cls[encs[i]->N].push_back(DecSrc{encs[i], bufs[i].jobs, 0});
  for (auto& kv : cls) {
    int rc = decode_steps(kv.second, s);
    if (rc != XV_OK) return cleanup(rc);
  }
  for (int i = 0; i < n; i++) {
    int rc = decode_finish(encs[i], &outs[i], bufs[i], s);
    if (rc != XV_OK) return cleanup(rc);
  }
  return XV_OK;
}

int xv_ssim(const xv_encoded* e, double* ssim, void* hip_stream) {
  if (!e || !ssim) return fail(XV_EINVAL, "null encoded cube or output");
  if (!e->frames || !e->recon)
    return fail(XV_EINVAL, "SSIM needs the converted frames and the reconstruction "
                           "(dropped by XV_FLAG_DROP_WORK; absent for a cube read from a bitstream)");
  const int bands = (int)e->bands;
  if (e->H < 11 || e->W < 11) {
    for (int b = 0; b < bands; b++) ssim[b] = NAN;
    return XV_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  SsimArgs a;
  memset(&a, 0, sizeof a);
  a.frames = e->frames;
  a.recon = e->recon;
  double ws = 0.0;
  for (int i = 0; i < 11; i++) {
    const double d = (double)(i - 5);
    a.w[i] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    ws += a.w[i];
  }
  for (int i = 0; i < 11; i++) a.w[i] /= ws;
  const double L = (double)((1 << e->p.bit_depth) - 1);
  a.C1 = (0.01 * L) * (0.01 * L);
  a.C2 = (0.03 * L) * (0.03 * L);
  a.T = (int)e->T;
  a.Hp = e->Hp;
  a.Wp = e->Wp;
  a.H = (int)e->H;
  a.W = (int)e->W;
  a.bands = bands;
  ssim_tiles(a.H, a.W, &a.tiles_x, &a.tiles_y);
  const size_t nparts = (size_t)bands * a.T * a.tiles_x * a.tiles_y;
  void* mem = nullptr;
  hipError_t he = dev_alloc(&mem, (nparts + bands) * sizeof(double), s);
  if (he != hipSuccess) return fail(XV_ENOMEM, "SSIM scratch: %s", hipGetErrorString(he));
  a.part = (double*)mem;
  double* out = a.part + nparts;
  {
    ProfScope ps(XV_K_QUALITY, s, (double)e->T * e->H * e->W * bands * 4.0);
    he = launch_ssim(a, out, s);
  }
  if (he == hipSuccess) he = hipMemcpyAsync(ssim, out, bands * sizeof(double), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(mem, s);
  if (he != hipSuccess) return fail(XV_EHIP, "SSIM: %s", hipGetErrorString(he));
  return XV_OK;
}

int xv_spectral_angle(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                      uint64_t* n_pixels, void* hip_stream) {
  if (!mean_rad) return fail(XV_EINVAL, "null output");
  int rc = check_cube(orig, "original");
  if (rc != XV_OK) return rc;
  if ((rc = check_cube(decoded, "decoded")) != XV_OK) return rc;
  if (orig->T != decoded->T || orig->H != decoded->H || orig->W != decoded->W ||
      orig->bands != decoded->bands)
    return fail(XV_EINVAL, "spectral angle: cubes differ in shape");
  hipStream_t s = (hipStream_t)hip_stream;
  SaArgs a;
  memset(&a, 0, sizeof a);
  a.orig = orig->data;
  a.dec = decoded->data;
  a.dtype_orig = orig->dtype;
  a.dtype_dec = decoded->dtype;
  a.bands = (int)orig->bands;
  a.npix = orig->T * orig->H * orig->W;
  const int64_t want = (a.npix + kSaThreads - 1) / kSaThreads;
  const int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  void* mem = nullptr;
  hipError_t he = dev_alloc(&mem, (size_t)nblocks * 16 + 16, s);
  if (he != hipSuccess) return fail(XV_ENOMEM, "spectral angle scratch: %s", hipGetErrorString(he));
  a.part_sum = (double*)mem;
  a.part_n = (unsigned long long*)(a.part_sum + nblocks);
  a.out = (double*)(a.part_n + nblocks);
  {
    const double ib = (orig->dtype == XV_U16 ? 2.0 : 4.0) + (decoded->dtype == XV_U16 ? 2.0 : 4.0);
    ProfScope ps(XV_K_QUALITY, s, (double)a.npix * a.bands * ib);
    he = launch_spectral_angle(a, nblocks, s);
  }
  uint64_t host[2] = {0, 0};
  if (he == hipSuccess) he = hipMemcpyAsync(host, a.out, 16, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(mem, s);
  if (he != hipSuccess) return fail(XV_EHIP, "spectral angle: %s", hipGetErrorString(he));
  double sum;
  memcpy(&sum, &host[0], 8);
  const uint64_t n = host[1];
  *mean_rad = n ? sum / (double)n : NAN;
  if (n_pixels) *n_pixels = n;
  return XV_OK;
}

namespace {

// Checks orig against e and launches the physical-domain error kernels when
// both the original and the reconstruction are there; *have_phys tells.
int launch_metrics(const xv_cube* orig, const xv_encoded* e, hipStream_t s, bool* have_phys) {
  *have_phys = false;
  if (!orig) return XV_OK;
  int rc = check_cube(orig, "original");
  if (rc != XV_OK) return rc;
  if (orig->T != e->T || orig->H != e->H || orig->W != e->W || orig->bands != e->bands ||
      orig->dtype != e->src_dtype)
    return fail(XV_EINVAL, "original cube differs from the encoded one");
  if (e->recon) {
    PhysArgs a{orig->data, orig->dtype, e->recon, e->T, e->H, e->W, (int)e->bands, e->Hp,
               e->Wp, e->p.bit_depth, e->mn, e->mx, e->phys_partial, e->phys, e->phys_nb,
               chunk_px_for(e->W, (int)e->bands)};
    const double ib = orig->dtype == XV_U16 ? 2.0 : 4.0;
    ProfScope ps(XV_K_METRICS, s, (double)e->T * e->H * e->W * e->bands * (ib + 2.0));
    XV_HIP(launch_phys_sse(a, s), "physical error kernel");
    *have_phys = true;
  }
  return XV_OK;
}

// Fills m from a host copy of e's metric span (band min and max, physical
// squared errors, valid counts, coded squared errors, bit totals).
void fill_metrics(const xv_encoded* e, const uint64_t* span, bool dphys, xv_metrics* m) {
  const int bands = (int)e->bands, G = e->G;
  const double* mn = (const double*)span;
  const double* mx = mn + bands;
  const double* phys = mx + bands;
  const unsigned long long* nv = (const unsigned long long*)(phys + bands);
  const unsigned long long* sse = nv + bands;
  const unsigned long long* bits = sse + 3 * G;

  memset(m, 0, sizeof *m);
  m->bands = bands;
  m->groups = G;
  const double L = (double)((1 << e->p.bit_depth) - 1);
  for (int b = 0; b < bands; b++) {
    const unsigned long long se = sse[3 * (b / 3) + b % 3];
    m->sse[b] = se;
    m->n_valid[b] = nv[b];
    m->band_min[b] = mn[b];
    m->band_max[b] = mx[b];
    if (nv[b] == 0) {
      m->psnr[b] = NAN;
    } else if (se == 0) {
      m->psnr[b] = INFINITY;
    } else {
      const double mse = (double)se / (double)nv[b];
      m->psnr[b] = 10.0 * log10(L * L / mse);
    }
    m->sse_phys[b] = dphys ? phys[b] : NAN;
    if (!dphys || nv[b] == 0 || !(mx[b] > 0.0)) {
      m->psnr_phys[b] = NAN;
    } else if (phys[b] == 0.0) {
      m->psnr_phys[b] = INFINITY;
    } else {
      const double mse = phys[b] / (double)nv[b];
      m->psnr_phys[b] = 10.0 * log10(mx[b] * mx[b] / mse);
    }
  }
  unsigned long long cb = 0, mb = 0;
  const double pix = (double)e->T * (double)e->H * (double)e->W;
  for (int g = 0; g < G; g++) {
    cb += bits[2 * g];
    mb += bits[2 * g + 1];
    const int nb = (int)std::min<int64_t>(3, e->bands - 3 * g);
    if (g < XV_MAX_GROUPS) m->bpppb_group[g] = (double)(bits[2 * g] + bits[2 * g + 1]) / (pix * nb);
  }
  m->coef_bits = cb;
  m->mv_bits = mb;
  m->header_bits = 128ull * bands + 256ull;
  m->bpppb = (double)(cb + mb) / (pix * (double)bands);
}

}  // namespace

int xv_psnr_bpppb(const xv_cube* orig, const xv_encoded* e, xv_metrics* m, void* hip_stream) {
  if (!e || !m) return fail(XV_EINVAL, "null encoded cube or metrics");
  hipStream_t s = (hipStream_t)hip_stream;
  bool have_phys = false;
  int rc = launch_metrics(orig, e, s, &have_phys);
  if (rc != XV_OK) return rc;
  std::vector<uint64_t> host(e->span_bytes / 8);
  XV_HIP(hipMemcpyAsync(host.data(), e->span, e->span_bytes, hipMemcpyDeviceToHost, s), "copy metrics");
  XV_HIP(hipStreamSynchronize(s), "synchronise metrics");
  fill_metrics(e, host.data(), have_phys, m);
  return XV_OK;
}

int xv_psnr_bpppb_batch(int n, const xv_cube* origs, const xv_encoded* const* encs, xv_metrics* ms,
                        void* hip_stream) {
  if (n < 1 || !encs || !ms) return fail(XV_EINVAL, "bad metrics batch");
  for (int i = 0; i < n; i++)
    if (!encs[i]) return fail(XV_EINVAL, "null encoded cube %d in the metrics batch", i);
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<char> phys(n, 0);
  size_t total = 0;
  for (int i = 0; i < n; i++) {
    bool hp = false;
    const int rc = launch_metrics(origs ? &origs[i] : nullptr, encs[i], s, &hp);
    if (rc != XV_OK) return rc;
    phys[i] = hp;
    total += encs[i]->span_bytes;
  }
  // the spans gathered in one device buffer, one copy to the host, one wait
  void* gather = nullptr;
  XV_HIP(dev_alloc(&gather, total, s), "device allocation of the metrics gather");
  size_t off = 0;
  hipError_t he = hipSuccess;
  for (int i = 0; i < n && he == hipSuccess; i++) {
    he = hipMemcpyAsync((char*)gather + off, encs[i]->span, encs[i]->span_bytes,
                        hipMemcpyDeviceToDevice, s);
    off += encs[i]->span_bytes;
  }
  std::vector<uint64_t> host(total / 8);
  if (he == hipSuccess)
    he = hipMemcpyAsync(host.data(), gather, total, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(gather, s);
  XV_HIP(he, "gather metrics");
  off = 0;
  for (int i = 0; i < n; i++) {
    fill_metrics(encs[i], host.data() + off / 8, phys[i], &ms[i]);
    off += encs[i]->span_bytes;
  }
  return XV_OK;
}

int xv_encoded_export(const xv_encoded* e, xv_export* v) {
  if (!e || !v) return fail(XV_EINVAL, "null argument");
  memset(v, 0, sizeof *v);
  v->T = e->T;
  v->H = e->H;
  v->W = e->W;
  v->bands = e->bands;
  v->groups = e->G;
  v->Hp = e->Hp;
  v->Wp = e->Wp;
  v->Hb = e->Hb;
  v->Wb = e->Wb;
  v->params = e->p;
  v->src_dtype = e->src_dtype;
  v->frames = e->frames;
  v->recon = e->recon;
  v->levels = e->levels;
  v->mvs = e->mvs;
  v->coef_bits = e->cbits;
  v->mv_bits = e->mbits;
  v->band_min = e->mn;
  v->band_max = e->mx;
  v->sse = (const uint64_t*)e->sse;
  v->n_valid = (const uint64_t*)e->nvalid;
  return XV_OK;
}

void xv_encoded_free(xv_encoded* e) {
  if (!e) return;
  if (e->work) dev_free(e->work, e->stream);
  if (e->keep) dev_free(e->keep, e->stream);
  delete e;
}

int xv_set_me_geometry(int block, int search_range, const xv_me_geometry* g) {
  if (!(block == 4 || block == 8 || block == 16 || block == 32) || search_range < 0 ||
      search_range > 64)
    return fail(XV_EINVAL, "bad block or search range");
  if (!g || (g->blocks_per_wg == 0 && g->cands_per_lane == 0 && g->threads == 0 &&
             g->rows_per_lane == 0 && g->layout == 0)) {
    std::lock_guard<std::mutex> lk(g_geom_mu);
    g_geom.erase({block, search_range});  // back to the model default
    return XV_OK;
  }
  MeGeom m = me_default_geometry(block, search_range);
  if (g) {
    if (g->blocks_per_wg) m.nb = g->blocks_per_wg;
    if (g->cands_per_lane) m.kx = g->cands_per_lane;
    if (g->threads) m.threads = g->threads;
    if (g->layout) {
      if (g->layout != m.layout && !g->rows_per_lane) m.rows = 1;
      m.layout = g->layout;
    }
    if (g->rows_per_lane) m.rows = g->rows_per_lane;
  }
  if (m.layout != XV_ME_COLUMN_PAIRS && m.layout != XV_ME_ROW_PAIRS &&
      m.layout != XV_ME_ROW_PAIRS_BY_CHANNEL)
    return fail(XV_EINVAL, "unknown window layout %d", m.layout);
  if (m.nb < 1 || m.nb > 64) return fail(XV_EINVAL, "blocks_per_wg out of range");
  if (m.threads < 64 || m.threads > 512 || (m.threads & 63))
    return fail(XV_EINVAL, "threads must be a multiple of 64 in 64..512");
  if (!me_instance_exists(m))
    return fail(XV_EINVAL,
                m.layout != XV_ME_COLUMN_PAIRS
                    ? "no row-pair kernel for %d candidates x %d rows per lane (one row; 2..9, "
                      "11 or 13 candidates)"
                    : "no column-pair kernel for %d candidates x %d rows per lane (rows 1..3 for "
                      "any even count 2..18; 5 rows for 2 or 4 candidates)",
                m.kx, m.rows);
  if (me_lds_bytes_for(block, search_range, m) > 160 * 1024)
    return fail(XV_EINVAL, "geometry needs more than 160 KB of LDS");
  if (!me_geometry_fits(block, search_range, m))
    return fail(XV_EINVAL, "a workgroup's items exceed 3 rounds of its threads");
  std::lock_guard<std::mutex> lk(g_geom_mu);
  g_geom[{block, search_range}] = m;
  return XV_OK;
}

int xv_get_me_geometry(int block, int search_range, int width_blocks, xv_me_geometry* g) {
  if (!g) return fail(XV_EINVAL, "null geometry");
  if (!(block == 4 || block == 8 || block == 16 || block == 32) || search_range < 0 ||
      search_range > 64)
    return fail(XV_EINVAL, "bad block or search range");
  MeGeom m = geometry_for(block, search_range, width_blocks > 0 ? width_blocks : 16);
  g->blocks_per_wg = m.nb;
  g->cands_per_lane = m.kx;
  g->threads = m.threads;
  g->rows_per_lane = m.rows;
  g->layout = m.layout;
  return XV_OK;
}

int xv_autotune_me(const xv_cube* in, const xv_params* p, void* hip_stream, int max_candidates,
                   xv_me_geometry* out, double* best_ms) {
  if (!in || !p) return fail(XV_EINVAL, "null tuning input");
  return xv_autotune_me_batch(1, in, p, hip_stream, max_candidates, out, best_ms);
}

int xv_autotune_me_batch(int n, const xv_cube* cubes, const xv_params* params, void* hip_stream,
                         int max_candidates, xv_me_geometry* out, double* best_ms) {
  if (n < 1 || n > kMaxSeg || !cubes || !params)
    return fail(XV_EINVAL, "tuning needs 1..%d cubes", kMaxSeg);
  int rc = XV_OK;
  for (int i = 0; i < n; i++) {
    if ((rc = check_cube(&cubes[i], "tuning input")) != XV_OK) return rc;
    if ((rc = check_params(&params[i])) != XV_OK) return rc;
    if (cubes[i].T < 2 || params[i].gop < 2)
      return fail(XV_EINVAL, "tuning needs a P picture (T >= 2, gop >= 2)");
    if (params[i].block != params[0].block || params[i].search_range != params[0].search_range)
      return fail(XV_EINVAL, "tuning batch mixes block sizes or search ranges");
  }
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<xv_encoded*> encs(n, nullptr);
  auto cleanup = [&](int r) {
    for (auto* e : encs)
      if (e) xv_encoded_free(e);
    return r;
  };
  for (int i = 0; i < n; i++) {
    xv_params q = params[i];
    q.flags = 0;
    if ((rc = encode_prepare(&cubes[i], &q, s, &encs[i])) != XV_OK) return cleanup(rc);
  }
  const int N = encs[0]->N, R = params[0].search_range;
  int wb = 1;
  for (auto* e : encs) wb = std::max(wb, e->Wb);
  // step 0 (I pictures) provides the references of step 1
  {
    std::vector<SegSrc> src;
    for (auto* e : encs) src.push_back(SegSrc{e, 0});
    const MeGeom g0 = geometry_for(N, R, wb);
    rc = launch_segments(src, 0, g0, [&](const LaunchDesc& d, double) {
      XV_HIP(launch_encode(N, d, s), "transform kernel");
      return XV_OK;
    });
    if (rc != XV_OK) return cleanup(rc);
  }
  // the model's best of each window layout, an equal share of the timed set
  // each (the model's scores are not comparable enough across layouts to
  // rank them against each other); a share a layout cannot fill goes to the
  // others
  constexpr int kLayouts = 3;  // XV_ME_COLUMN_PAIRS .. XV_ME_ROW_PAIRS_BY_CHANNEL
  std::vector<std::pair<double, MeGeom>> scored[kLayouts];
  for (const MeGeom& g : me_candidates(N, R, wb))
    scored[g.layout - 1].push_back({me_model_score(N, R, g, wb), g});
  const size_t keep = (size_t)(max_candidates > 0 ? max_candidates : 512);
  size_t share[kLayouts] = {0, 0, 0};
  for (size_t left = keep, open = kLayouts; left > 0 && open > 0;) {
    open = 0;
    for (int l = 0; l < kLayouts && left > 0; l++)
      if (share[l] < scored[l].size()) {
        share[l]++;
        left--;
        open++;
      }
  }
  std::vector<MeGeom> cand;
  for (int l = 0; l < kLayouts; l++) {
    std::stable_sort(scored[l].begin(), scored[l].end(),
                     [](const auto& a, const auto& b) { return a.first > b.first; });
    for (size_t i = 0; i < share[l]; i++) cand.push_back(scored[l][i].second);
  }
  const MeGeom def = geometry_for(N, R, wb);
  if (std::find_if(cand.begin(), cand.end(), [&](const MeGeom& g) {
        return g.nb == def.nb && g.kx == def.kx && g.threads == def.threads &&
               g.rows == def.rows && g.layout == def.layout;
      }) == cand.end())
    cand.push_back(def);
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  (void)hipEventCreate(&ev0);
  (void)hipEventCreate(&ev1);
  MeGeom best = def;
  float best_t = 1e30f;
  std::vector<SegSrc> src;
  for (auto* e : encs) src.push_back(SegSrc{e, 1});
  auto time_once = [&](const MeGeom& g, float* ms) {
    (void)hipEventRecord(ev0, s);
    int r = launch_segments(src, 1, g, [&](const LaunchDesc& d, double) {
      XV_HIP(launch_me(N, R, g, d, s), "motion search kernel");
      return XV_OK;
    });
    (void)hipEventRecord(ev1, s);
    if (r != XV_OK) return r;
    if (hipEventSynchronize(ev1) != hipSuccess) return fail(XV_EHIP, "tuning event");
    *ms = 0.f;
    (void)hipEventElapsedTime(ms, ev0, ev1);
    return XV_OK;
  };
  // every candidate: the best of three runs after one that warms caches
  std::vector<std::pair<float, MeGeom>> timed;
  for (const MeGeom& g : cand) {
    float tmin = 1e30f, ms = 0.f;
    for (int rep = 0; rep < 4 && rc == XV_OK; rep++) {
      rc = time_once(g, &ms);
      if (rc == XV_OK && rep > 0) tmin = std::min(tmin, ms);
    }
    if (rc != XV_OK) break;
    timed.push_back({tmin, g});
  }
  // the closest few again, in interleaved rounds so that drift of the clock
  // affects them alike, ranked by their median
  if (rc == XV_OK && !timed.empty()) {
    std::stable_sort(timed.begin(), timed.end(),
                     [](const auto& a, const auto& b) { return a.first < b.first; });
    const size_t top = std::min<size_t>(6, timed.size());
    constexpr int kRounds = 9;
    std::vector<std::vector<float>> runs(top);
    for (int rep = 0; rep < kRounds && rc == XV_OK; rep++)
      for (size_t i = 0; i < top && rc == XV_OK; i++) {
        float ms = 0.f;
        rc = time_once(timed[i].second, &ms);
        runs[i].push_back(ms);
      }
    if (rc == XV_OK)
      for (size_t i = 0; i < top; i++) {
        std::sort(runs[i].begin(), runs[i].end());
        const float med = runs[i][runs[i].size() / 2];
        if (med < best_t) {
          best_t = med;
          best = timed[i].second;
        }
      }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  cleanup(XV_OK);
  if (rc != XV_OK) return rc;
  XV_HIP(hipStreamSynchronize(s), "synchronise tuning");
  {
    std::lock_guard<std::mutex> lk(g_geom_mu);
    g_geom[{N, R}] = best;
  }
  if (out) {
    out->blocks_per_wg = best.nb;
    out->cands_per_lane = best.kx;
    out->threads = best.threads;
    out->rows_per_lane = best.rows;
    out->layout = best.layout;
  }
  if (best_ms) *best_ms = best_t;
  return XV_OK;
}

int xv_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_pending) {
    (void)hipEventSynchronize(r.b);
    g_prof_events.push_back(r.a);
    g_prof_events.push_back(r.b);
  }
  g_prof_pending.clear();
  memset(&g_prof_tot, 0, sizeof g_prof_tot);
  g_prof_on = on != 0;
  return XV_OK;
}

int xv_profile_select(uint32_t class_mask) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_mask = class_mask ? class_mask : ~0u;
  return XV_OK;
}

// ---- bitstream ---------------------------------------------------------------

}  // extern "C"

struct xv_packed {
  void* mem;
  uint64_t bytes;
  uint64_t payload_bits;
  hipStream_t stream;
};

namespace {

constexpr char kPackMagic[8] = {'X', 'V', 'P', 'A', 'C', 'K', '0', '1'};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

BitsArgs bits_args_of(const xv_encoded* e) {
  BitsArgs a{};
  a.N = e->N;
  a.Hb = e->Hb;
  a.Wb = e->Wb;
  a.T = (int32_t)e->T;
  a.gop = e->p.gop;
  a.nunits = (int64_t)e->G * e->T * 4 * e->Hb * e->Wb;
  return a;
}

}  // namespace

extern "C" {

int xv_pack(const xv_encoded* e, void* hip_stream, xv_packed** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  if (!e) return fail(XV_EINVAL, "null encoded cube");
  hipStream_t s = (hipStream_t)hip_stream;
  BitsArgs a = bits_args_of(e);
  a.cbits = e->cbits;
  a.mbits = e->mbits;
  a.levels = e->levels;
  a.mvs = e->mvs;
  const int64_t nb = bits_scan_blocks(a.nunits);
  void* scratch = nullptr;
  XV_HIP(dev_alloc(&scratch, (size_t)(nb + 1) * 8, s), "device allocation of the scan buffer");
  a.block_off = (uint64_t*)scratch;
  a.total = a.block_off + nb;
  uint64_t total = 0;
  hipError_t he = launch_bits_scan(a, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&total, a.total, 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    dev_free(scratch, s);
    return hip_fail(he, "bitstream scan");
  }
  const uint64_t nseg = (uint64_t)(a.nunits / a.Wb);
  const uint64_t nwords = (total + 31) / 32 + 2;  // two words of padding for readers
  PackHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kPackMagic, 8);
  h.version = 1;
  h.header_bytes = sizeof(PackHeader);
  h.T = e->T;
  h.H = e->H;
  h.W = e->W;
  h.bands = e->bands;
  h.src_dtype = e->src_dtype;
  h.G = e->G;
  h.N = e->N;
  h.Hp = e->Hp;
  h.Wp = e->Wp;
  h.Hb = e->Hb;
  h.Wb = e->Wb;
  h.params = e->p;
  h.nseg = nseg;
  h.payload_bits = total;
  h.nwords = nwords;
  h.off_span = align256(sizeof(PackHeader));
  h.span_bytes = e->span_bytes;
  h.off_index = align256(h.off_span + h.span_bytes);
  h.off_payload = align256(h.off_index + nseg * 8);
  h.total_bytes = h.off_payload + nwords * 4;
  xv_packed* pk = new (std::nothrow) xv_packed();
  if (!pk) {
    dev_free(scratch, s);
    return fail(XV_ENOMEM, "host allocation failed");
  }
  pk->bytes = h.total_bytes;
  pk->payload_bits = total;
  pk->stream = s;
  he = dev_alloc(&pk->mem, h.total_bytes, s);
  if (he != hipSuccess) {
    delete pk;
    dev_free(scratch, s);
    return hip_fail(he, "device allocation of the serialised cube");
  }
  char* m = (char*)pk->mem;
  a.index = (uint64_t*)(m + h.off_index);
  a.words = (uint32_t*)(m + h.off_payload);
  he = launch_write_header(h, m, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(m + h.off_span, e->span, e->span_bytes, hipMemcpyDeviceToDevice, s);
  if (he == hipSuccess) he = launch_fill_u32(a.words, 0u, (int64_t)nwords, s);
  if (he == hipSuccess) {
    ProfScope ps(XV_K_BITS_WRITE, s, (double)total / 8.0);
    he = launch_bits_write(a, s);
  }
  dev_free(scratch, s);
  if (he != hipSuccess) {
    dev_free(pk->mem, s);
    delete pk;
    return hip_fail(he, "bitstream write");
  }
  *out = pk;
  return XV_OK;
}

int xv_packed_view(const xv_packed* p, const void** data, uint64_t* bytes, uint64_t* payload_bits) {
  if (!p) return fail(XV_EINVAL, "null packed cube");
  if (data) *data = p->mem;
  if (bytes) *bytes = p->bytes;
  if (payload_bits) *payload_bits = p->payload_bits;
  return XV_OK;
}

void xv_packed_free(xv_packed* p) {
  if (!p) return;
  if (p->mem) dev_free(p->mem, p->stream);
  delete p;
}

int xv_unpack(const void* data, uint64_t bytes, void* hip_stream, xv_encoded** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  if (!data || bytes < sizeof(PackHeader)) return fail(XV_EINVAL, "buffer too small for a header");
  hipStream_t s = (hipStream_t)hip_stream;
  PackHeader h;
  XV_HIP(hipMemcpyAsync(&h, data, sizeof h, hipMemcpyDeviceToHost, s), "copy header");
  XV_HIP(hipStreamSynchronize(s), "synchronise header copy");
  if (memcmp(h.magic, kPackMagic, 8) != 0 || h.version != 1 || h.header_bytes != sizeof h)
    return fail(XV_EINVAL, "not a serialised cube (bad magic or version)");
  xv_cube cube{(void*)data, h.src_dtype, 0, h.T, h.H, h.W, h.bands};
  int rc = check_cube(&cube, "serialised cube");
  if (rc != XV_OK) return rc;
  if ((rc = check_params(&h.params)) != XV_OK) return rc;
  xv_encoded* e = new (std::nothrow) xv_encoded();
  if (!e) return fail(XV_ENOMEM, "host allocation failed");
  memset(e, 0, sizeof *e);
  dims_of(e, &cube, &h.params);
  e->stream = s;
  BitsArgs a = bits_args_of(e);
  const uint64_t nseg = (uint64_t)(a.nunits / a.Wb);
  const EncLayout lay = enc_layout(e);
  if (e->G != h.G || e->N != h.N || e->Hp != h.Hp || e->Wp != h.Wp || e->Hb != h.Hb ||
      e->Wb != h.Wb || h.nseg != nseg || h.span_bytes != lay.span_words * 8 ||
      h.nwords != (h.payload_bits + 31) / 32 + 2 || h.off_span < sizeof h ||
      h.off_index < h.off_span + h.span_bytes || h.off_payload < h.off_index + nseg * 8 ||
      h.total_bytes != h.off_payload + h.nwords * 4 || h.total_bytes > bytes) {
    delete e;
    return fail(XV_EINVAL, "serialised cube header is inconsistent");
  }
  e->phys_nb = lay.phys_nb;
  hipError_t he = dev_alloc(&e->keep, lay.keep, s);
  if (he != hipSuccess) {
    delete e;
    return hip_fail(he, "device allocation of the encoded cube");
  }
  bind_keep(e, lay);
  void* err = nullptr;
  he = dev_alloc(&err, 256, s);
  if (he != hipSuccess) {
    xv_encoded_free(e);
    return hip_fail(he, "device allocation");
  }
  const char* m = (const char*)data;
  a.index = (uint64_t*)(m + h.off_index);
  a.words = (uint32_t*)(m + h.off_payload);
  a.nwords = (int64_t)h.nwords;
  a.total_bits = h.payload_bits;
  a.levels_out = e->levels;
  a.mvs_out = e->mvs;
  a.cbits_out = e->cbits;
  a.mbits_out = e->mbits;
  a.err = (uint32_t*)err;
  const int64_t lev_words = (int64_t)e->G * e->T * 3 * e->Hp * e->Wp / 2;
  uint32_t herr = 0;
  he = hipMemcpyAsync(e->span, m + h.off_span, h.span_bytes, hipMemcpyDeviceToDevice, s);
  if (he == hipSuccess) he = launch_fill_u32((uint32_t*)e->levels, 0u, lev_words, s);
  if (he == hipSuccess) he = launch_fill_u32(a.err, 0u, 1, s);
  if (he == hipSuccess) {
    ProfScope ps(XV_K_BITS_PARSE, s, (double)h.payload_bits / 8.0);
    he = launch_bits_parse(a, s);
  }
  if (he == hipSuccess) he = hipMemcpyAsync(&herr, a.err, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(err, s);
  if (he != hipSuccess) {
    xv_encoded_free(e);
    return hip_fail(he, "bitstream parse");
  }
  if (herr) {
    xv_encoded_free(e);
    return fail(XV_EINVAL, "payload does not parse as the stored codes");
  }
  *out = e;
  return XV_OK;
}

int xv_memory_read(xv_memory* out) {
  if (!out) return fail(XV_EINVAL, "null memory record");
  size_t live = 0, cached = 0, peak = 0;
  dev_cache_stats(&live, &cached, &peak);
  out->live_bytes = live;
  out->cached_bytes = cached;
  out->peak_bytes = peak;
  return XV_OK;
}

int xv_cache_release(uint64_t* released_bytes) {
  const size_t n = dev_cache_release();
  if (released_bytes) *released_bytes = n;
  return XV_OK;
}

int xv_profile_read(xv_profile* out) {
  if (!out) return fail(XV_EINVAL, "null profile");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_pending) {
    hipError_t he = hipEventSynchronize(r.b);
    if (he != hipSuccess) return hip_fail(he, "profile event");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, r.a, r.b);
    g_prof_tot.ms[r.cls] += ms;
    g_prof_tot.launches[r.cls] += 1;
    g_prof_tot.work[r.cls] += r.work;
    g_prof_events.push_back(r.a);
    g_prof_events.push_back(r.b);
  }
  g_prof_pending.clear();
  *out = g_prof_tot;
  return XV_OK;
}

}  // extern "C"

// ===========================================================================
// Serving loop
// ===========================================================================
namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct SReq {
  uint64_t ticket = 0;
  int op = XV_OP_ENCODE;
  xv_cube cube{};
  xv_params params{};
  const xv_encoded* src = nullptr;
  enum State { QUEUED, ACTIVE, DONE } state = QUEUED;
  int status = XV_EPENDING;
  bool cancel = false;
  xv_encoded* enc = nullptr;  // encode: the cube being built
  DecodeBuf db;               // decode: buffers
  int step = 0, nsteps = 0;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;
  bool ev_recorded = false;
  double t_submit = 0, t_admit = 0, t_done = 0;
  int N = 0, R = 0;
};

}  // namespace

struct xv_server {
  xv_server_cfg cfg{};
  hipStream_t s = nullptr;
  bool own_stream = false;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<SReq*> queue;
  std::vector<SReq*> active;
  std::unordered_map<uint64_t, SReq*> reqs;
  uint64_t next = 1;
  size_t used = 0;
  bool stop = false;
  xv_server_stats st{};
  std::deque<hipEvent_t> inflight;  // iteration events, oldest first
  std::thread th;
};

namespace {

// Device bytes a request holds while resident.
size_t request_bytes(const SReq* r) {
  if (r->op == XV_OP_ENCODE) {
    xv_encoded tmp;
    memset(&tmp, 0, sizeof tmp);
    dims_of(&tmp, &r->cube, &r->params);
    const EncLayout L = enc_layout(&tmp);
    return L.keep + L.work;
  }
  return decode_bytes(r->src);
}

void finish(xv_server* sv, SReq* r, int status) {
  if (r->ev) {
    (void)hipEventDestroy(r->ev);
    r->ev = nullptr;
  }
  if (r->state == SReq::ACTIVE) sv->used -= r->bytes;
  r->state = SReq::DONE;
  r->t_done = now_ms();
  r->status = r->cancel ? XV_ECANCELED : status;
  if (r->status != XV_OK && r->enc) {
    xv_encoded_free(r->enc);
    r->enc = nullptr;
  }
  if (r->status == XV_OK) sv->st.completed++;
  else if (r->status == XV_ECANCELED) sv->st.cancelled++;
  else sv->st.failed++;
  sv->cv_done.notify_all();
}

int admit(xv_server* sv, SReq* r) {
  if (r->op == XV_OP_ENCODE) {
    int rc = encode_prepare(&r->cube, &r->params, sv->s, &r->enc);
    if (rc != XV_OK) {
      if (r->enc) xv_encoded_free(r->enc);
      r->enc = nullptr;
      return rc;
    }
    r->nsteps = r->enc->nsteps;
    r->N = r->enc->N;
    r->R = r->params.search_range;
  } else {
    int rc = decode_prepare(r->src, sv->s, r->db);
    if (rc != XV_OK) return rc;
    r->nsteps = r->src->nsteps;
    r->N = r->src->N;
  }
  r->step = 0;
  r->state = SReq::ACTIVE;
  r->t_admit = now_ms();
  return XV_OK;
}

// Launch the next frame step of every resident request that has one.
int iterate(xv_server* sv) {
  std::map<std::pair<int, int>, std::vector<SegSrc>> enc_cls;  // (N, R)
  std::map<int, std::vector<DecSrc>> dec_cls;
  std::vector<SReq*> stepped;
  for (SReq* r : sv->active) {
    if (r->step >= r->nsteps) continue;
    if (r->op == XV_OP_ENCODE) enc_cls[{r->N, r->R}].push_back(SegSrc{r->enc, r->step});
    else dec_cls[r->N].push_back(DecSrc{r->src, r->db.jobs, r->step});
    stepped.push_back(r);
  }
  if (stepped.empty()) return XV_OK;
  for (auto& kv : enc_cls) {
    const int N = kv.first.first, R = kv.first.second;
    int max_wb = 1;
    for (auto& sg : kv.second) max_wb = std::max(max_wb, sg.e->Wb);
    const MeGeom geom = geometry_for(N, R, max_wb);
    std::vector<SegSrc> p;
    for (auto& sg : kv.second)
      if (sg.step > 0) p.push_back(sg);
    if (!p.empty()) {
      int rc = launch_segments(p, 1, geom, [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ME, sv->s, work);
        XV_HIP(launch_me(N, R, geom, d, sv->s), "motion search kernel");
        sv->st.launches++;
        return XV_OK;
      });
      if (rc != XV_OK) return rc;
    }
    int rc = launch_segments(kv.second, 0, geom, [&](const LaunchDesc& d, double work) {
      ProfScope ps(XV_K_ENCODE, sv->s, work);
      XV_HIP(launch_encode(N, d, sv->s), "transform kernel");
      sv->st.launches++;
      return XV_OK;
    });
    if (rc != XV_OK) return rc;
  }
  for (auto& kv : dec_cls) {
    int rc = decode_launch(kv.second, sv->s);
    if (rc != XV_OK) return rc;
    sv->st.launches++;
  }
  for (SReq* r : stepped) {
    r->step++;
    if (r->step == r->nsteps) {
      if (r->op == XV_OP_DECODE) {
        int rc = decode_finish(r->src, &r->cube, r->db, sv->s);
        if (rc != XV_OK) return rc;
      } else {
        int rc = finish_encode(r->enc);
        if (rc != XV_OK) return rc;
      }
      XV_HIP(hipEventRecord(r->ev, sv->s), "request event");
      r->ev_recorded = true;
    }
  }
  sv->st.iterations++;
  return XV_OK;
}

void scheduler(xv_server* sv) {
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    sv->cv_work.wait(lk, [&] { return sv->stop || !sv->queue.empty() || !sv->active.empty(); });
    if (sv->stop && sv->queue.empty() && sv->active.empty()) break;
    // retire completed requests
    for (size_t i = 0; i < sv->active.size();) {
      SReq* r = sv->active[i];
      if (r->ev_recorded && hipEventQuery(r->ev) == hipSuccess) {
        finish(sv, r, XV_OK);
        sv->active.erase(sv->active.begin() + i);
      } else {
        i++;
      }
    }
    // admit in arrival order while a slot and memory are free
    while (!sv->queue.empty() && (int)sv->active.size() < sv->cfg.max_slots) {
      SReq* r = sv->queue.front();
      if (r->cancel) {
        sv->queue.pop_front();
        finish(sv, r, XV_ECANCELED);
        continue;
      }
      if (r->bytes > sv->cfg.hbm_budget) {
        sv->queue.pop_front();
        finish(sv, r, fail(XV_ENOMEM, "request needs %zu bytes, budget is %llu", r->bytes,
                           (unsigned long long)sv->cfg.hbm_budget));
        continue;
      }
      if (sv->used + r->bytes > sv->cfg.hbm_budget) break;  // wait for memory
      sv->queue.pop_front();
      const int rc = admit(sv, r);
      if (rc != XV_OK) {
        finish(sv, r, rc);
        continue;
      }
      sv->used += r->bytes;
      sv->active.push_back(r);
      sv->st.peak_bytes = std::max<uint64_t>(sv->st.peak_bytes, sv->used);
      sv->st.peak_active = std::max<int32_t>(sv->st.peak_active, (int32_t)sv->active.size());
    }
    // keep at most two iterations queued ahead of the GPU
    while (sv->inflight.size() >= 2) {
      hipEvent_t ev = sv->inflight.front();
      sv->inflight.pop_front();
      lk.unlock();
      (void)hipEventSynchronize(ev);
      (void)hipEventDestroy(ev);
      lk.lock();
    }
    bool any_steps = false;
    for (SReq* r : sv->active) any_steps |= r->step < r->nsteps;
    if (any_steps) {
      const int rc = iterate(sv);
      if (rc != XV_OK) {
        // a launch failed: fail every resident request
        for (SReq* r : sv->active) finish(sv, r, rc);
        sv->active.clear();
      } else {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
          (void)hipEventRecord(ev, sv->s);
          sv->inflight.push_back(ev);
        }
      }
    } else if (!sv->active.empty()) {
      // everything resident is waiting for the GPU: wait for the oldest
      SReq* r = sv->active.front();
      hipEvent_t ev = r->ev;
      lk.unlock();
      if (ev) (void)hipEventSynchronize(ev);
      lk.lock();
    }
  }
  for (hipEvent_t ev : sv->inflight) {
    (void)hipEventSynchronize(ev);
    (void)hipEventDestroy(ev);
  }
  sv->inflight.clear();
}

int take_result(xv_server* sv, SReq* r, xv_result* res) {
  // a returned encode has completed on the GPU: later frees need not be
  // ordered on the server's stream, which may be gone by then
  if (r->enc && sv->own_stream) r->enc->stream = nullptr;
  if (res) {
    res->status = r->status;
    res->op = r->op;
    res->enc = r->enc;
    res->submit_ms = r->t_submit;
    res->admit_ms = r->t_admit;
    res->done_ms = r->t_done;
  } else if (r->enc) {
    xv_encoded_free(r->enc);
  }
  sv->reqs.erase(r->ticket);
  delete r;
  return XV_OK;
}

}  // namespace

extern "C" {

int xv_server_create(const xv_server_cfg* cfg, xv_server** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  xv_server* sv = new (std::nothrow) xv_server();
  if (!sv) return fail(XV_ENOMEM, "host allocation failed");
  if (cfg) sv->cfg = *cfg;
  if (sv->cfg.hbm_budget == 0) sv->cfg.hbm_budget = 64ull << 30;
  if (sv->cfg.max_slots <= 0) sv->cfg.max_slots = 64;
  if (sv->cfg.max_queue <= 0) sv->cfg.max_queue = 65536;
  if (sv->cfg.stream) {
    sv->s = (hipStream_t)sv->cfg.stream;
  } else {
    hipError_t e = hipStreamCreateWithFlags(&sv->s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete sv;
      return hip_fail(e, "server stream");
    }
    sv->own_stream = true;
  }
  sv->th = std::thread(scheduler, sv);
  *out = sv;
  return XV_OK;
}

int xv_server_submit(xv_server* sv, const xv_request* rq, uint64_t* ticket) {
  if (!sv || !rq || !ticket) return fail(XV_EINVAL, "null argument");
  int rc;
  if (rq->op == XV_OP_ENCODE) {
    if ((rc = check_cube(&rq->cube, "request input")) != XV_OK) return rc;
    if ((rc = check_params(&rq->params)) != XV_OK) return rc;
  } else if (rq->op == XV_OP_DECODE) {
    if (!rq->enc) return fail(XV_EINVAL, "decode request without an encoded cube");
    if ((rc = check_decode_out(rq->enc, &rq->cube)) != XV_OK) return rc;
  } else {
    return fail(XV_EINVAL, "unknown request op %d", rq->op);
  }
  SReq* r = new (std::nothrow) SReq();
  if (!r) return fail(XV_ENOMEM, "host allocation failed");
  r->op = rq->op;
  r->cube = rq->cube;
  r->params = rq->params;
  r->src = rq->enc;
  r->bytes = request_bytes(r);
  if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
    delete r;
    return fail(XV_EHIP, "request event");
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  if ((int)sv->queue.size() >= sv->cfg.max_queue) {
    (void)hipEventDestroy(r->ev);
    delete r;
    return fail(XV_EBUSY, "server queue is full");
  }
  r->ticket = sv->next++;
  r->t_submit = now_ms();
  sv->reqs[r->ticket] = r;
  sv->queue.push_back(r);
  sv->st.submitted++;
  *ticket = r->ticket;
  sv->cv_work.notify_one();
  return XV_OK;
}

int xv_server_poll(xv_server* sv, uint64_t ticket, xv_result* res) {
  if (!sv) return fail(XV_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(XV_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  if (it->second->state != SReq::DONE) {
    if (res) res->status = XV_EPENDING;
    return XV_EPENDING;
  }
  return take_result(sv, it->second, res);
}

int xv_server_wait(xv_server* sv, uint64_t ticket, xv_result* res) {
  if (!sv) return fail(XV_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(XV_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  SReq* r = it->second;
  sv->cv_done.wait(lk, [&] { return r->state == SReq::DONE; });
  return take_result(sv, r, res);
}

int xv_server_cancel(xv_server* sv, uint64_t ticket) {
  if (!sv) return fail(XV_EINVAL, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(XV_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
  SReq* r = it->second;
  if (r->state == SReq::DONE) return XV_OK;
  r->cancel = true;
  if (r->state == SReq::QUEUED) {
    for (auto q = sv->queue.begin(); q != sv->queue.end(); ++q)
      if (*q == r) {
        sv->queue.erase(q);
        break;
      }
    finish(sv, r, XV_ECANCELED);
  }
  sv->cv_work.notify_one();
  return XV_OK;
}

int xv_server_stats_read(xv_server* sv, xv_server_stats* st) {
  if (!sv || !st) return fail(XV_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  *st = sv->st;
  return XV_OK;
}

int xv_server_destroy(xv_server* sv) {
  if (!sv) return XV_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
    sv->cv_work.notify_all();
  }
  if (sv->th.joinable()) sv->th.join();
  (void)hipStreamSynchronize(sv->s);
  for (auto& kv : sv->reqs) {
    SReq* r = kv.second;
    if (r->enc) xv_encoded_free(r->enc);
    if (r->ev) (void)hipEventDestroy(r->ev);
    delete r;
  }
  sv->reqs.clear();
  if (sv->own_stream) {
    dev_stream_retired(sv->s);
    (void)hipStreamDestroy(sv->s);
  }
  delete sv;
  return XV_OK;
}

}  // extern "C"
