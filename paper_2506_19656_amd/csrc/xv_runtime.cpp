// xv_runtime.cpp -- process-wide state of libxv: error text, per-launch
// event timing (xv_profile_*), the motion-search geometry table
// (xv_set_me_geometry / xv_get_me_geometry), status strings and the
// device-memory cache queries.
#include <stdarg.h>
#include <stdio.h>

#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "xv_host.h"

using namespace xv;

namespace xv {
namespace host {

namespace {
thread_local std::string g_err;
}  // namespace

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

const char* last_error() { return g_err.c_str(); }

namespace {
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

std::mutex g_geom_mu;
std::map<std::pair<int, int>, MeGeom> g_geom;
std::map<std::tuple<int, int, int>, MeGeom> g_geom_default;
std::map<std::pair<int, int>, MeGeom> g_split_geom;
std::map<std::tuple<int, int, int>, MeGeom> g_split_geom_default;
}  // namespace

ProfScope::ProfScope(int c, hipStream_t st, double w) : cls(c), s(st), work(w) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  on = g_prof_on && ((g_prof_mask >> c) & 1u);
  if (on) {
    a = prof_event_locked();
    b = prof_event_locked();
    (void)hipEventRecord(a, s);
  }
}

ProfScope::~ProfScope() {
  if (!on) return;
  (void)hipEventRecord(b, s);
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back(ProfRec{cls, a, b, work});
}

bool profiling_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

MeGeom geometry_for(int N, int R, int Wb) {
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

void geometry_install(int N, int R, const MeGeom& g) {
  std::lock_guard<std::mutex> lk(g_geom_mu);
  g_geom[{N, R}] = g;
}

void geometry_reset(int N, int R) {
  std::lock_guard<std::mutex> lk(g_geom_mu);
  g_geom.erase({N, R});
}

MeGeom split_geometry_for(int N, int R, int Wb) {
  std::lock_guard<std::mutex> lk(g_geom_mu);
  auto it = g_split_geom.find({N, R});
  if (it != g_split_geom.end()) return it->second;
  const int wb = std::max(1, std::min(16, Wb));
  auto d = g_split_geom_default.find({N, R, wb});
  if (d != g_split_geom_default.end()) return d->second;
  MeGeom g = me_split_default_geometry(N, R, wb);
  g_split_geom_default[{N, R, wb}] = g;
  return g;
}

void split_geometry_install(int N, int R, const MeGeom& g) {
  std::lock_guard<std::mutex> lk(g_geom_mu);
  g_split_geom[{N, R}] = g;
}

}  // namespace host
}  // namespace xv

using namespace xv::host;

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

const char* xv_last_error(void) { return last_error(); }

int xv_set_me_geometry(int block, int search_range, const xv_me_geometry* g) {
  if (!(block == 4 || block == 8 || block == 16 || block == 32) || search_range < 0 ||
      search_range > 64)
    return fail(XV_EINVAL, "bad block or search range");
  if (!g || (g->blocks_per_wg == 0 && g->cands_per_lane == 0 && g->threads == 0 &&
             g->rows_per_lane == 0 && g->layout == 0)) {
    geometry_reset(block, search_range);  // back to the model default
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
  geometry_install(block, search_range, m);
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

int xv_set_me_split_geometry(int block, int search_range, const xv_me_geometry* g) {
  if (!(block == 8 || block == 16 || block == 32) || search_range < 0 || search_range > 64)
    return fail(XV_EINVAL, "bad block or search range for the adaptive block size");
  if (!g || (g->blocks_per_wg == 0 && g->cands_per_lane == 0 && g->threads == 0 &&
             g->rows_per_lane == 0 && g->layout == 0)) {
    std::lock_guard<std::mutex> lk(g_geom_mu);
    g_split_geom.erase({block, search_range});  // back to the model default
    return XV_OK;
  }
  MeGeom m = me_split_default_geometry(block, search_range, 16);
  if (g->blocks_per_wg) m.nb = g->blocks_per_wg;
  if (g->cands_per_lane) m.kx = g->cands_per_lane;
  if (g->threads) m.threads = g->threads;
  if (g->layout) m.layout = g->layout;
  if (g->rows_per_lane) m.rows = g->rows_per_lane;
  if (m.layout != XV_ME_ROW_PAIRS && m.layout != XV_ME_ROW_PAIRS_BY_CHANNEL)
    return fail(XV_EINVAL, "the combined search has row-pair layouts only (got %d)", m.layout);
  if (m.nb < 1 || m.nb > 64) return fail(XV_EINVAL, "blocks_per_wg out of range");
  if (m.threads < 64 || m.threads > 512 || (m.threads & 63))
    return fail(XV_EINVAL, "threads must be a multiple of 64 in 64..512");
  if (!me_split_instance_exists(block, m))
    return fail(XV_EINVAL,
                "no combined-search kernel for %d candidates x %d rows per lane (one row; 5, 7, "
                "11 or 13 candidates)",
                m.kx, m.rows);
  if (me_split_lds_bytes(block, search_range, m) > 160 * 1024)
    return fail(XV_EINVAL, "geometry needs more than 160 KB of LDS");
  if (!me_split_fits(block, search_range, m))
    return fail(XV_EINVAL, "a workgroup's items exceed %d round(s) of its threads",
                me_split_rounds(m));
  split_geometry_install(block, search_range, m);
  return XV_OK;
}

int xv_get_me_split_geometry(int block, int search_range, int width_blocks, xv_me_geometry* g) {
  if (!g) return fail(XV_EINVAL, "null geometry");
  if (!(block == 8 || block == 16 || block == 32) || search_range < 0 || search_range > 64)
    return fail(XV_EINVAL, "bad block or search range for the adaptive block size");
  MeGeom m = split_geometry_for(block, search_range, width_blocks > 0 ? width_blocks : 16);
  g->blocks_per_wg = m.nb;
  g->cands_per_lane = m.kx;
  g->threads = m.threads;
  g->rows_per_lane = m.rows;
  g->layout = m.layout;
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
