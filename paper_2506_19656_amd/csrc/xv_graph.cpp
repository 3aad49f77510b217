// xv_graph.cpp -- the frame-step launches of a batched encode or decode
// captured once as a HIP graph and replayed for later batches of the same
// shape (xv_set_graph_mode).
//
// A captured launch carries its arguments by value, and the arguments of the
// step kernels are job-table addresses.  So a graph is built against job
// tables at fixed addresses owned by its cache entry: each call writes its
// own job tables as usual (plan kernel), copies them into the entry's tables
// (one device-to-device copy per cube, outside the graph), and replays the
// graph, whose kernels then reach this call's frames, levels and
// reconstructions through them.  The key is everything the launches depend
// on: per cube the frame count, group count, GOP, padded size, block size,
// search range and the quarter-sample, intra and adaptive-block-size flags; the
// motion-search geometries of the class (plain, and combined for the adaptive
// block size); and the stream.  Graphs hold kernel nodes only (no memset or copy
// nodes).  Capture runs on a stream of the library's own, so the caller's
// stream may be the null stream; nothing captured executes during capture.
#include <string.h>

#include <list>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

namespace {

std::mutex g_graph_mu;
bool g_graph_on = false;
hipStream_t g_capture_stream = nullptr;

struct GraphKey {
  int kind;  // 0 encode steps, 1 decode steps
  hipStream_t stream;
  MeGeom geom, sgeom;  // sgeom: the combined search's (zero without split cubes)
  std::vector<int64_t> dims;
  bool operator<(const GraphKey& o) const {
    return std::tie(kind, stream, geom.nb, geom.kx, geom.threads, geom.rows, geom.layout,
                    sgeom.nb, sgeom.kx, sgeom.threads, sgeom.rows, sgeom.layout, dims) <
           std::tie(o.kind, o.stream, o.geom.nb, o.geom.kx, o.geom.threads, o.geom.rows,
                    o.geom.layout, o.sgeom.nb, o.sgeom.kx, o.sgeom.threads, o.sgeom.rows,
                    o.sgeom.layout, o.dims);
  }
};

struct GraphEntry {
  hipGraphExec_t exec = nullptr;
  void* tables = nullptr;          // job tables of every cube, back to back
  std::vector<size_t> offsets;     // byte offset of cube i's table
  hipStream_t stream = nullptr;
  uint64_t last_use = 0;
};

std::map<GraphKey, GraphEntry> g_graphs;
uint64_t g_graph_clock = 0;
constexpr size_t kMaxGraphs = 32;

void destroy_entry(GraphEntry& g) {
  // a replay may still run on the entry's stream: let it finish first
  if (g.exec && g.stream) (void)hipStreamSynchronize(g.stream);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.tables) dev_free(g.tables, g.stream);
  g.exec = nullptr;
  g.tables = nullptr;
}

std::vector<int64_t> dims_key(const std::vector<const xv_encoded*>& es) {
  std::vector<int64_t> d;
  for (const xv_encoded* e : es) {
    const int64_t v[] = {e->T, e->G, e->p.gop, e->Hp, e->Wp, e->N, e->p.search_range,
                         (int64_t)(e->p.flags & (XV_FLAG_QPEL | XV_FLAG_INTRA | XV_FLAG_SPLIT)),
                         e->nsteps, e->njobs};
    d.insert(d.end(), v, v + 10);
  }
  return d;
}

// Captures `launch` (the class's step loop, launching with job tables at the
// entry's addresses) into a new graph.
template <class F>
int capture(GraphEntry& g, F launch) {
  if (!g_capture_stream) {
    XV_HIP(hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking), "capture stream");
  }
  XV_HIP(hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  int rc = launch(g_capture_stream);
  hipGraph_t graph = nullptr;
  hipError_t he = hipStreamEndCapture(g_capture_stream, &graph);
  if (rc != XV_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  XV_HIP(he, "end capture");
  he = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  XV_HIP(he, "instantiate graph");
  return XV_OK;
}

// The cache entry for `key` (captured on first use), its tables refreshed
// from each cube's own job table; then one replay on s.
template <class Tables, class Launch>
int replay(const GraphKey& key, const std::vector<size_t>& bytes, Tables tables_of,
           Launch launch, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  auto it = g_graphs.find(key);
  if (it == g_graphs.end()) {
    if (g_graphs.size() >= kMaxGraphs) {  // evict the least recently used
      auto old = g_graphs.begin();
      for (auto i = g_graphs.begin(); i != g_graphs.end(); ++i)
        if (i->second.last_use < old->second.last_use) old = i;
      destroy_entry(old->second);
      g_graphs.erase(old);
    }
    GraphEntry g;
    g.stream = s;
    size_t total = 0;
    for (size_t b : bytes) {
      g.offsets.push_back(total);
      total += (b + 255) & ~(size_t)255;
    }
    XV_HIP(dev_alloc(&g.tables, total, s), "graph job tables");
    std::vector<FrameJob*> fixed;
    for (size_t o : g.offsets) fixed.push_back((FrameJob*)((char*)g.tables + o));
    int rc = capture(g, [&](hipStream_t cs) { return launch(fixed, cs); });
    if (rc != XV_OK) {
      destroy_entry(g);
      return rc;
    }
    it = g_graphs.emplace(key, g).first;
  }
  GraphEntry& g = it->second;
  g.last_use = ++g_graph_clock;
  for (size_t i = 0; i < bytes.size(); i++)
    XV_HIP(hipMemcpyAsync((char*)g.tables + g.offsets[i], tables_of(i), bytes[i],
                          hipMemcpyDeviceToDevice, s),
           "refresh graph job tables");
  XV_HIP(hipGraphLaunch(g.exec, s), "graph launch");
  return XV_OK;
}

}  // namespace

namespace xv {
namespace host {

bool graphs_enabled() {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  return g_graph_on;
}

int encode_steps_graph(std::vector<xv_encoded*>& es, hipStream_t s) {
  // the widest frame, of all cubes and of those with the adaptive block size
  int max_wb = 1, max_wb_split = 0;
  for (auto* e : es) {
    max_wb = std::max(max_wb, e->Wb);
    if (e->p.flags & XV_FLAG_SPLIT) max_wb_split = std::max(max_wb_split, e->Wb);
  }
  const int N = es[0]->N, R = es[0]->p.search_range;
  GraphKey key{0, s, geometry_for(N, R, max_wb),
               max_wb_split ? split_geometry_for(N, R, max_wb_split) : MeGeom{},
               dims_key(std::vector<const xv_encoded*>(es.begin(), es.end()))};
  std::vector<size_t> bytes;
  for (auto* e : es) bytes.push_back((size_t)e->njobs * sizeof(FrameJob));
  return replay(
      key, bytes, [&](size_t i) { return (const void*)es[i]->jobs; },
      [&](const std::vector<FrameJob*>& fixed, hipStream_t cs) {
        // the step loop with every cube's job table at its fixed address
        std::vector<FrameJob*> own;
        for (size_t i = 0; i < es.size(); i++) {
          own.push_back(es[i]->jobs);
          es[i]->jobs = fixed[i];
        }
        const int rc = encode_steps(es, cs);
        for (size_t i = 0; i < es.size(); i++) es[i]->jobs = own[i];
        return rc;
      },
      s);
}

int decode_steps_graph(const std::vector<DecSrc>& base, hipStream_t s) {
  std::vector<const xv_encoded*> es;
  for (auto& b : base) es.push_back(b.e);
  GraphKey key{1, s, MeGeom{}, MeGeom{}, dims_key(es)};
  std::vector<size_t> bytes;
  for (auto& b : base) bytes.push_back((size_t)b.e->njobs * sizeof(FrameJob));
  return replay(
      key, bytes, [&](size_t i) { return (const void*)base[i].jobs; },
      [&](const std::vector<FrameJob*>& fixed, hipStream_t cs) {
        std::vector<DecSrc> moved(base);
        for (size_t i = 0; i < moved.size(); i++) moved[i].jobs = fixed[i];
        return decode_steps(moved, cs);
      },
      s);
}

size_t graph_cache_release() {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  const size_t n = g_graphs.size();
  for (auto& kv : g_graphs) destroy_entry(kv.second);
  g_graphs.clear();
  return n;
}

}  // namespace host
}  // namespace xv

extern "C" {

int xv_set_graph_mode(int on) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  g_graph_on = on != 0;
  return XV_OK;
}

int xv_get_graph_mode(void) {
  std::lock_guard<std::mutex> lk(g_graph_mu);
  return g_graph_on ? 1 : 0;
}

}  // extern "C"
