// xv_api.cpp -- the coding loop behind the C ABI of include/xv.h: argument
// validation, device buffers of an encoded cube, launch sequencing (stats ->
// pack -> plan -> for every frame step: motion search (P) and fused transform
// coding), decode, metrics, the batched multi-cube path and the export view.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <vector>

#include "xv_host.h"

using namespace xv;

namespace xv {
namespace host {

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
  if (p->flags & ~(XV_FLAG_DROP_WORK | XV_FLAG_QPEL | XV_FLAG_INTRA | XV_FLAG_SPLIT))
    return fail(XV_EINVAL, "unknown flags");
  if ((p->flags & XV_FLAG_QPEL) && p->search_range > 31)
    return fail(XV_EINVAL, "quarter-sample motion needs search_range <= 31 (int8 vectors)");
  if ((p->flags & XV_FLAG_SPLIT) && (N < 8 || (p->flags & (XV_FLAG_QPEL | XV_FLAG_INTRA))))
    return fail(XV_EINVAL, "the adaptive block size needs block >= 8, integer vectors and no intra modes");
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

int tiles_per_frame(const xv_encoded* e) {
  int t = xf_tiles_per_job(e->N, e->Hb, e->Wb);
  if (e->p.flags & XV_FLAG_SPLIT) t += xf_tiles_per_job(e->N / 2, 2 * e->Hb, 2 * e->Wb);
  return t;
}

int32_t split_lambda16(int qp, int bit_depth) {
  const int qP = qp + 6 * (bit_depth - 8);
  return (int32_t)floor(16.0 * sqrt(0.57 * pow(2.0, (qP - 12) / 3.0)) + 0.5);
}

EncLayout enc_layout(const xv_encoded* e) {
  EncLayout L{};
  const int64_t G = e->G, T = e->T;
  const int64_t plane = (int64_t)e->Hp * e->Wp;
  const int64_t nframes = G * T;
  const int64_t nblk = nframes * e->Hb * e->Wb;
  const int64_t bands = e->bands;
  const bool split = (e->p.flags & XV_FLAG_SPLIT) != 0;
  Carve k;
  L.o_lev = k.take<int16_t>((size_t)nframes * 3 * plane);
  L.o_mv = k.take<int8_t>((size_t)nblk * 2 * (split ? 4 : 1));
  L.o_cb = k.take<uint32_t>((size_t)nblk * 3);
  L.o_mb = k.take<uint32_t>((size_t)nblk);
  L.o_keys = k.take<uint32_t>((size_t)bands + 1 + (size_t)kStatsMaxBlocks * 3 * bands);
  L.span_words = (size_t)3 * bands + bands + 3 * G + 2 * G;
  L.o_span = k.take<uint64_t>(L.span_words);
  L.phys_nb = phys_blocks(T * e->H * e->W * bands);
  L.o_pp = k.take<double>((size_t)L.phys_nb * bands);
  L.o_jobs = k.take<FrameJob>((size_t)e->njobs);
  L.o_split = split ? k.take<uint8_t>((size_t)nblk) : 0;
  L.keep = k.off;
  Carve w;
  L.o_fr = w.take<uint16_t>((size_t)nframes * 3 * plane);
  L.o_rc = w.take<uint16_t>((size_t)nframes * 3 * plane);
  L.o_vm = e->src_dtype == XV_F32 ? w.take<uint8_t>((size_t)nframes * 3 * plane) : 0;
  L.o_part = w.take<uint64_t>((size_t)nframes * tiles_per_frame(e) * kTileSums);
  L.o_tot = w.take<uint64_t>((size_t)G * kTotMaxChunks * 5);
  L.o_pred = (e->p.flags & (XV_FLAG_QPEL | XV_FLAG_INTRA)) ? w.take<uint8_t>(pred_plane_bytes(e))
                                                           : 0;
  L.o_mvw = split ? w.take<int8_t>((size_t)nblk * 2) : 0;
  L.o_sadw = split ? w.take<uint32_t>((size_t)nblk) : 0;
  L.o_sadc = split ? w.take<uint32_t>((size_t)nblk * 4) : 0;
  L.work = w.off;
  return L;
}

size_t pred_plane_bytes(const xv_encoded* e) {
  const int64_t ngop = (e->T + e->p.gop - 1) / e->p.gop;
  return (size_t)e->G * ngop * 3 * (size_t)e->Hp * e->Wp * sizeof(uint16_t);
}

size_t decode_bytes(const xv_encoded* e) {
  Carve c;
  c.take<uint16_t>((size_t)e->G * e->T * 3 * (size_t)e->Hp * e->Wp);
  c.take<FrameJob>((size_t)e->njobs);
  if (e->p.flags & XV_FLAG_QPEL) c.take<uint8_t>(pred_plane_bytes(e));
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
  const bool split = (e->p.flags & XV_FLAG_SPLIT) != 0;
  e->splits = split ? (uint8_t*)(kb + lay.o_split) : nullptr;
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
  e->tot_chunk = (unsigned long long*)(wb + lay.o_tot);
  e->pred = (p->flags & (XV_FLAG_QPEL | XV_FLAG_INTRA)) ? (uint16_t*)(wb + lay.o_pred) : nullptr;
  const bool split = (p->flags & XV_FLAG_SPLIT) != 0;
  e->mv_whole = split ? (int8_t*)(wb + lay.o_mvw) : nullptr;
  e->sad_whole = split ? (uint32_t*)(wb + lay.o_sadw) : nullptr;
  e->sad_cell = split ? (uint32_t*)(wb + lay.o_sadc) : nullptr;
  e->tpf = tiles_per_frame(e);
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
                e->nan_total, e->tile_part, e->pred, e->jobs, (int32_t)T, e->G, p->gop, e->nsteps,
                e->Hp, e->Wp, (int32_t)e->H, (int32_t)e->W, (int32_t)bands, e->N,
                p->bit_depth, p->qp, e->tpf, (p->flags & XV_FLAG_QPEL) != 0,
                (p->flags & XV_FLAG_INTRA) != 0, e->splits, e->mv_whole, e->sad_whole,
                e->sad_cell, split ? split_lambda16(p->qp, p->bit_depth) : 0};
    XV_HIP(launch_plan(pl, s), "plan kernel");
  }
  return XV_OK;
}

// SAD terms of a motion-search launch: (2R+1)^2 per real-channel sample.
// SAD terms of one motion-search step: every candidate that keeps the
// displaced block inside the padded picture, N^2 terms per real channel.
double me_work(const xv_encoded* e, int s, int n) {
  const int R = e->p.search_range, N = n > 0 ? n : e->N;
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
    // sources with the adaptive block size take their own launches
    std::vector<SegSrc> src, split;
    for (auto* e : es)
      if (st < e->nsteps) ((e->p.flags & XV_FLAG_SPLIT) ? split : src).push_back(SegSrc{e, st});
    if (st > 0) {
      if (!src.empty()) {
        int rc = launch_segments(src, 1, geom, [&](const LaunchDesc& d, double work) {
          ProfScope ps(XV_K_ME, s, work);
          XV_HIP(launch_me(N, R, geom, d, s), "motion search kernel");
          return XV_OK;
        });
        if (rc != XV_OK) return rc;
        uint64_t nl = 0;
        if ((rc = launch_subpel_step(src, s, &nl)) != XV_OK) return rc;
      }
      if (int rc = launch_split_search(split, s); rc != XV_OK) return rc;
    } else {
      uint64_t nl = 0;
      int rc = launch_intra_step(src, s, &nl);
      if (rc != XV_OK) return rc;
    }
    if (!src.empty()) {
      int rc = launch_segments(src, 0, geom, [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ENCODE, s, work);
        XV_HIP(launch_encode(N, d, s), "transform kernel");
        return XV_OK;
      });
      if (rc != XV_OK) return rc;
    }
    if (int rc = launch_split_transform(split, s); rc != XV_OK) return rc;
  }
  return XV_OK;
}

int launch_split_search(const std::vector<SegSrc>& src, hipStream_t s) {
  if (src.empty()) return XV_OK;
  const int N = src[0].e->N, R = src[0].e->p.search_range;
  int max_wb = 1;
  for (auto& x : src) max_wb = std::max(max_wb, x.e->Wb);
  const MeGeom g = split_geometry_for(N, R, max_wb);
  // one search for the whole blocks and their cells; the SAD terms counted
  // are the whole blocks' (each term serves the block and one cell)
  int rc = launch_chunks(
      src, [](const SegSrc& x) { return x.e->jobs; },
      [&](const xv_encoded* e) { return me_tiles_per_job(e->Hb, e->Wb, g); },
      [](const SegSrc& x) { return me_work(x.e, x.step); },
      [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ME, s, work);
        XV_HIP(launch_me_split(N, R, g, d, s), "motion search kernel (whole blocks and cells)");
        return XV_OK;
      });
  if (rc != XV_OK) return rc;
  return launch_chunks(
      src, [](const SegSrc& x) { return x.e->jobs; },
      [](const xv_encoded* e) { return split_tiles_per_job(e->Hb, e->Wb); },
      [](const SegSrc&) { return 0.0; },
      [&](const LaunchDesc& d, double) {
        XV_HIP(launch_split_decide(N, d, s), "whole-or-split choice kernel");
        return XV_OK;
      });
}

int launch_split_transform(const std::vector<SegSrc>& src, hipStream_t s) {
  if (src.empty()) return XV_OK;
  const int N = src[0].e->N;
  // the step's algorithmic bytes go with the size-N launch
  int rc = launch_chunks(
      src, [](const SegSrc& x) { return x.e->jobs; },
      [&](const xv_encoded* e) { return xf_tiles_per_job(N, e->Hb, e->Wb); },
      [](const SegSrc& x) {
        return xf_frames(x.e, x.step) * 3.0 * x.e->Hp * x.e->Wp * (x.step == 0 ? 6.0 : 8.0);
      },
      [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ENCODE, s, work);
        XV_HIP(launch_encode_split(N, 1, d, s), "transform kernel (whole blocks)");
        return XV_OK;
      });
  if (rc != XV_OK) return rc;
  return launch_chunks(
      src, [](const SegSrc& x) { return x.e->jobs; },
      [&](const xv_encoded* e) { return xf_tiles_per_job(N / 2, 2 * e->Hb, 2 * e->Wb); },
      [](const SegSrc&) { return 0.0; },
      [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ENCODE, s, work);
        XV_HIP(launch_encode_split(N / 2, 2, d, s), "transform kernel (cells)");
        return XV_OK;
      });
}

int launch_split_decode(const std::vector<DecSrc>& src, hipStream_t s) {
  if (src.empty()) return XV_OK;
  const int N = src[0].e->N;
  int rc = launch_chunks(
      src, [](const DecSrc& x) { return x.jobs; },
      [&](const xv_encoded* e) { return xf_tiles_per_job(N, e->Hb, e->Wb); },
      [](const DecSrc& x) {
        return xf_frames(x.e, x.step) * 3.0 * x.e->Hp * x.e->Wp * (x.step == 0 ? 4.0 : 6.0);
      },
      [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_DECODE, s, work);
        XV_HIP(launch_decode_split(N, 1, d, s), "decode kernel (whole blocks)");
        return XV_OK;
      });
  if (rc != XV_OK) return rc;
  return launch_chunks(
      src, [](const DecSrc& x) { return x.jobs; },
      [&](const xv_encoded* e) { return xf_tiles_per_job(N / 2, 2 * e->Hb, 2 * e->Wb); },
      [](const DecSrc&) { return 0.0; },
      [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_DECODE, s, work);
        XV_HIP(launch_decode_split(N / 2, 2, d, s), "decode kernel (cells)");
        return XV_OK;
      });
}

// After the last step: per-group totals from the per-tile sums, then the
// work buffers go if the caller asked for that.
int finish_encode(xv_encoded* e) {
  XV_HIP(launch_encode_totals(e->tile_part, e->G, (int)e->T, e->tpf, e->tot_chunk, e->sse,
                              e->bits, e->stream),
         "encode totals kernel");
  if (e->p.flags & XV_FLAG_DROP_WORK) {
    dev_free(e->work, e->stream);
    e->work = nullptr;
    e->tile_part = nullptr;
    e->tot_chunk = nullptr;
    e->pred = nullptr;
    e->mv_whole = nullptr;
    e->sad_whole = nullptr;
    e->sad_cell = nullptr;
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


int decode_prepare(const xv_encoded* e, hipStream_t s, DecodeBuf& db) {
  Carve c;
  const int64_t plane = (int64_t)e->Hp * e->Wp;
  size_t o_rc = c.take<uint16_t>((size_t)e->G * e->T * 3 * plane);
  size_t o_jb = c.take<FrameJob>((size_t)e->njobs);
  const bool qpel = (e->p.flags & XV_FLAG_QPEL) != 0;
  size_t o_pr = qpel ? c.take<uint8_t>(pred_plane_bytes(e)) : 0;
  db.mem = nullptr;
  XV_HIP(dev_alloc(&db.mem, c.off, s), "device allocation of the decode buffers");
  db.recon = (uint16_t*)((char*)db.mem + o_rc);
  db.jobs = (FrameJob*)((char*)db.mem + o_jb);
  db.pred = qpel ? (uint16_t*)((char*)db.mem + o_pr) : nullptr;
  CubePlan pl{nullptr, db.recon, e->levels, e->mvs, nullptr, nullptr, nullptr, nullptr,
              nullptr, db.pred, db.jobs, (int32_t)e->T, e->G, e->p.gop, e->nsteps,
              e->Hp, e->Wp, (int32_t)e->H, (int32_t)e->W, (int32_t)e->bands, e->N,
              e->p.bit_depth, e->p.qp, 0, qpel, (e->p.flags & XV_FLAG_INTRA) != 0,
              e->splits, nullptr, nullptr, nullptr, 0};
  XV_HIP(launch_plan(pl, s), "plan kernel");
  return XV_OK;
}


// One launch per chunk of segments; each source brings its own step.
// Sources with the adaptive block size take their own launches.
int decode_launch(const std::vector<DecSrc>& all, hipStream_t s) {
  if (all.empty()) return XV_OK;
  std::vector<DecSrc> src, split;
  for (auto& x : all) ((x.e->p.flags & XV_FLAG_SPLIT) ? split : src).push_back(x);
  if (int rc = launch_split_decode(split, s); rc != XV_OK) return rc;
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
      if (st == 0 && (e->p.flags & XV_FLAG_INTRA)) continue;  // wavefront kernel's
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
    if (d.nseg == 0) continue;
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
    uint64_t nl = 0;
    int rc = launch_mc_step(src, s, &nl);
    if (rc != XV_OK) return rc;
    if ((rc = launch_intra_decode_step(src, s, &nl)) != XV_OK) return rc;
    rc = decode_launch(src, s);
    if (rc != XV_OK) return rc;
  }
  return XV_OK;
}

namespace {

// One workgroup per block; segments of the quarter-sample sources of a step.
// work: predicted samples the launch evaluates (per block, the refinement's
// 2 x 9 candidates over the real channels plus the 3-channel prediction it
// writes; motion compensation writes the 3-channel prediction only).
template <class Src, class JobsOf, class L>
int launch_blockwise(const std::vector<Src>& src, JobsOf jobs_of, bool refine, L launch,
                     uint64_t* launches) {
  size_t i = 0;
  while (i < src.size()) {
    LaunchDesc d;
    memset(&d, 0, sizeof d);
    int tiles = 0;
    double work = 0;
    int N = 0;
    for (; i < src.size() && d.nseg < kMaxSeg; i++) {
      const xv_encoded* e = src[i].e;
      const int st = src[i].step;
      if (st == 0 || !(e->p.flags & XV_FLAG_QPEL)) continue;
      N = e->N;
      const int n = plan_jobs_at((int)e->T, e->G, e->p.gop, st);
      const int tpj = e->Hb * e->Wb;
      Seg& g = d.seg[d.nseg++];
      g.jobs = jobs_of(src[i]) + plan_step_offset((int)e->T, e->G, e->p.gop, st);
      g.count = n;
      g.tpj = tpj;
      g.tile0 = tiles;
      tiles += n * tpj;
      double ch = 0;
      for (int gg = 0; gg < e->G; gg++) ch += std::min<int64_t>(3, e->bands - 3 * gg);
      const double per_group = refine ? 18.0 * ch / e->G + 3.0 : 3.0;
      work += (double)n * tpj * (double)e->N * e->N * per_group;
    }
    if (d.nseg == 0) continue;
    d.tiles = tiles;
    int rc = launch(N, d, work);
    if (rc != XV_OK) return rc;
    ++*launches;
  }
  return XV_OK;
}

}  // namespace

int launch_subpel_step(const std::vector<SegSrc>& src, hipStream_t s, uint64_t* launches) {
  return launch_blockwise(
      src, [](const SegSrc& x) { return x.e->jobs; }, true,
      [&](int N, const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_SUBPEL, s, work);
        XV_HIP(launch_subpel(N, d, s), "quarter-sample refinement kernel");
        return XV_OK;
      },
      launches);
}

int launch_mc_step(const std::vector<DecSrc>& src, hipStream_t s, uint64_t* launches) {
  return launch_blockwise(
      src, [](const DecSrc& x) { return x.jobs; }, false,
      [&](int N, const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_SUBPEL, s, work);
        XV_HIP(launch_mc(N, d, s), "motion compensation kernel");
        return XV_OK;
      },
      launches);
}

namespace {

// One launch per wavefront for each chunk of up to kMaxSeg intra sources
// at step 0 (one class: one N).  work per launch: the algorithmic bytes of
// the wavefront's blocks (encode: current, reconstruction and prediction,
// 6 B per sample; decode: level and reconstruction, 4 B).
template <class Src, class JobsOf>
int launch_intra_waves(const std::vector<Src>& src, JobsOf jobs_of, int decode, hipStream_t s,
                       uint64_t* launches) {
  size_t i = 0;
  while (i < src.size()) {
    LaunchDesc d;
    memset(&d, 0, sizeof d);
    int tiles = 0, N = 0, waves = 0;
    std::vector<std::pair<const xv_encoded*, int>> chunk;
    for (; i < src.size() && d.nseg < kMaxSeg; i++) {
      const xv_encoded* e = src[i].e;
      if (src[i].step != 0 || !(e->p.flags & XV_FLAG_INTRA)) continue;
      N = e->N;
      const int n = plan_jobs_at((int)e->T, e->G, e->p.gop, 0);
      const int tpj = intra_tiles_per_job(e->N, e->Hb, e->Wb);
      Seg& g = d.seg[d.nseg++];
      g.jobs = jobs_of(src[i]);
      g.count = n;
      g.tpj = tpj;
      g.tile0 = tiles;
      tiles += n * tpj;
      waves = std::max(waves, intra_waves(e->Hb, e->Wb));
      chunk.push_back({e, n});
    }
    if (d.nseg == 0) continue;
    d.tiles = tiles;
    for (int w = 0; w < waves; w++) {
      double work = 0;
      for (auto& ce : chunk) {
        const int Hb = ce.first->Hb, Wb = ce.first->Wb;
        const int lo = w - (Wb - 1) > 0 ? (w - (Wb - 1) + 1) / 2 : 0;
        const int hi = std::min(Hb - 1, w / 2);
        if (hi >= lo)
          work += (double)ce.second * (hi - lo + 1) * 3.0 * N * N * (decode ? 4.0 : 6.0);
      }
      ProfScope ps(XV_K_INTRA, s, work);
      XV_HIP(launch_intra(N, d, w, decode, s), "intra wavefront kernel");
      ++*launches;
    }
  }
  return XV_OK;
}

}  // namespace

int launch_intra_step(const std::vector<SegSrc>& src, hipStream_t s, uint64_t* launches) {
  return launch_intra_waves(
      src, [](const SegSrc& x) { return x.e->jobs; }, 0, s, launches);
}

int launch_intra_decode_step(const std::vector<DecSrc>& src, hipStream_t s, uint64_t* launches) {
  return launch_intra_waves(
      src, [](const DecSrc& x) { return x.jobs; }, 1, s, launches);
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


}  // namespace host
}  // namespace xv

using namespace xv::host;

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

extern "C" {

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
  const bool graph = graphs_enabled() && !profiling_enabled();
  for (auto& kv : cls) {
    int rc = graph ? encode_steps_graph(kv.second, s) : encode_steps(kv.second, s);
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
  const bool graph = graphs_enabled() && !profiling_enabled();
  for (auto& kv : cls) {
    int rc = graph ? decode_steps_graph(kv.second, s) : decode_steps(kv.second, s);
    if (rc != XV_OK) return cleanup(rc);
  }
  for (int i = 0; i < n; i++) {
    int rc = decode_finish(encs[i], &outs[i], bufs[i], s);
    if (rc != XV_OK) return cleanup(rc);
  }
  return XV_OK;
}


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
  v->splits = e->splits;
  return XV_OK;
}

void xv_encoded_free(xv_encoded* e) {
  if (!e) return;
  if (e->work) dev_free(e->work, e->stream);
  if (e->keep) dev_free(e->keep, e->stream);
  delete e;
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
  graph_cache_release();  // their job tables go back to the cache first
  const size_t n = dev_cache_release();
  if (released_bytes) *released_bytes = n;
  return XV_OK;
}

}  // extern "C"
