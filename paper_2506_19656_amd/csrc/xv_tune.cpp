// xv_tune.cpp -- the empirical motion-search geometry tuner
// (xv_autotune_me, xv_autotune_me_batch): candidates ranked by the CU model,
// timed on the first P-picture step of the batch that will run.  Params with
// XV_FLAG_SPLIT tune the adaptive block size's combined search instead.
#include <algorithm>
#include <vector>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

extern "C" {

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
    if ((params[i].flags ^ params[0].flags) & XV_FLAG_SPLIT)
      return fail(XV_EINVAL, "tuning batch mixes the adaptive block size with fixed blocks");
  }
  const bool split = (params[0].flags & XV_FLAG_SPLIT) != 0;
  hipStream_t s = (hipStream_t)hip_stream;
  std::vector<xv_encoded*> encs(n, nullptr);
  auto cleanup = [&](int r) {
    for (auto* e : encs)
      if (e) xv_encoded_free(e);
    return r;
  };
  for (int i = 0; i < n; i++) {
    xv_params q = params[i];
    q.flags = split ? XV_FLAG_SPLIT : 0;
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
    rc = split ? launch_split_transform(src, s)
               : launch_segments(src, 0, g0, [&](const LaunchDesc& d, double) {
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
  if (split) {
    for (const MeGeom& g : me_split_candidates(N, R, wb))
      scored[g.layout - 1].push_back({me_split_model_score(N, R, g, wb), g});
  } else {
    for (const MeGeom& g : me_candidates(N, R, wb))
      scored[g.layout - 1].push_back({me_model_score(N, R, g, wb), g});
  }
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
  const MeGeom def = split ? split_geometry_for(N, R, wb) : geometry_for(N, R, wb);
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
      XV_HIP(split ? launch_me_split(N, R, g, d, s) : launch_me(N, R, g, d, s),
             "motion search kernel");
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
  if (split)
    split_geometry_install(N, R, best);
  else
    geometry_install(N, R, best);
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

}  // extern "C"
