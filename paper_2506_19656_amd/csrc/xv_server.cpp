// xv_server.cpp -- the continuous-batching server (xv_server_*): admission
// by device-memory budget, one launch per frame step and class across all
// resident requests, a scheduler thread per server.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

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
  // QUEUED: waiting in the queue; ADMITTING: taken from the queue, its
  // buffers and first launches being set up by the scheduler without the
  // server lock; ACTIVE: resident; DONE: result ready
  enum State { QUEUED, ADMITTING, ACTIVE, DONE } state = QUEUED;
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
  // a decode that did not reach its last step still holds its buffers
  if (r->db.mem) {
    dev_free(r->db.mem, sv->s);
    r->db.mem = nullptr;
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
    if (rc != XV_OK) {
      if (r->db.mem) dev_free(r->db.mem, sv->s);
      r->db.mem = nullptr;
      return rc;
    }
    r->nsteps = r->src->nsteps;
    r->N = r->src->N;
  }
  r->step = 0;
  return XV_OK;
}

// Launch the next frame step of every request of `run` that has one.  Runs
// on the scheduler thread without the server lock: only that thread changes
// a resident request's step and buffers.  *launches counts the launches.
int iterate(xv_server* sv, const std::vector<SReq*>& run, uint64_t* launches) {
  std::map<std::pair<int, int>, std::vector<SegSrc>> enc_cls;  // (N, R)
  std::map<int, std::vector<DecSrc>> dec_cls;
  std::vector<SReq*> stepped;
  for (SReq* r : run) {
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
    // requests with the adaptive block size take their own launches
    std::vector<SegSrc> p, all, split, split_p;
    for (auto& sg : kv.second) {
      const bool sp = (sg.e->p.flags & XV_FLAG_SPLIT) != 0;
      (sp ? split : all).push_back(sg);
      if (sg.step > 0) (sp ? split_p : p).push_back(sg);
    }
    if (!split_p.empty()) {
      if (int rc = launch_split_search(split_p, sv->s); rc != XV_OK) return rc;
      *launches += 3;
    }
    if (!split.empty()) {
      if (int rc = launch_split_transform(split, sv->s); rc != XV_OK) return rc;
      *launches += 2;
    }
    if (all.empty()) continue;
    if (!p.empty()) {
      int rc = launch_segments(p, 1, geom, [&](const LaunchDesc& d, double work) {
        ProfScope ps(XV_K_ME, sv->s, work);
        XV_HIP(launch_me(N, R, geom, d, sv->s), "motion search kernel");
        ++*launches;
        return XV_OK;
      });
      if (rc != XV_OK) return rc;
      if ((rc = launch_subpel_step(p, sv->s, launches)) != XV_OK) return rc;
    }
    if (int rc = launch_intra_step(all, sv->s, launches); rc != XV_OK) return rc;
    int rc = launch_segments(all, 0, geom, [&](const LaunchDesc& d, double work) {
      ProfScope ps(XV_K_ENCODE, sv->s, work);
      XV_HIP(launch_encode(N, d, sv->s), "transform kernel");
      ++*launches;
      return XV_OK;
    });
    if (rc != XV_OK) return rc;
  }
  for (auto& kv : dec_cls) {
    int rc = launch_mc_step(kv.second, sv->s, launches);
    if (rc != XV_OK) return rc;
    if ((rc = launch_intra_decode_step(kv.second, sv->s, launches)) != XV_OK) return rc;
    rc = decode_launch(kv.second, sv->s);
    if (rc != XV_OK) return rc;
    ++*launches;
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
    // take requests in arrival order while a slot and memory are free; their
    // memory is reserved now, their buffers are set up below without the lock
    std::vector<SReq*> admitting;
    while (!sv->queue.empty() &&
           (int)(sv->active.size() + admitting.size()) < sv->cfg.max_slots) {
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
      sv->used += r->bytes;
      r->state = SReq::ADMITTING;
      admitting.push_back(r);
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
    std::vector<SReq*> run = sv->active;
    // allocations and launches without the lock: submit, poll and cancel
    // proceed meanwhile (they touch the queue, the ticket map and the
    // cancel flag, never a resident request's buffers)
    lk.unlock();
    std::vector<int> arc(admitting.size(), XV_OK);
    std::vector<std::string> aerr(admitting.size());
    for (size_t i = 0; i < admitting.size(); i++) {
      arc[i] = admit(sv, admitting[i]);
      if (arc[i] == XV_OK) run.push_back(admitting[i]);
      else aerr[i] = last_error();
    }
    bool any_steps = false;
    for (SReq* r : run) any_steps |= r->step < r->nsteps;
    int rc = XV_OK;
    uint64_t launches = 0;
    if (any_steps) {
      rc = iterate(sv, run, &launches);
      if (rc == XV_OK) {
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
          (void)hipEventRecord(ev, sv->s);
          lk.lock();
          sv->inflight.push_back(ev);
          lk.unlock();
        }
      }
    }
    lk.lock();
    for (size_t i = 0; i < admitting.size(); i++) {
      SReq* r = admitting[i];
      if (arc[i] != XV_OK) {
        sv->used -= r->bytes;  // never became resident
        fail(arc[i], "%s", aerr[i].c_str());
        finish(sv, r, arc[i]);
        continue;
      }
      r->state = SReq::ACTIVE;
      r->t_admit = now_ms();
      sv->active.push_back(r);
      sv->st.peak_bytes = std::max<uint64_t>(sv->st.peak_bytes, sv->used);
      sv->st.peak_active = std::max<int32_t>(sv->st.peak_active, (int32_t)sv->active.size());
    }
    sv->st.launches += launches;
    if (any_steps && rc == XV_OK) sv->st.iterations++;
    if (rc != XV_OK) {
      // a launch failed: fail every resident request
      for (SReq* r : sv->active) finish(sv, r, rc);
      sv->active.clear();
    } else if (!any_steps && !sv->active.empty()) {
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
