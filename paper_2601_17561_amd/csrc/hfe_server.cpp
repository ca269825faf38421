// Continuous-batching server: a worker thread admits queued requests into steps (batched int8
// CCMM + per-request decryption) on a ring of preallocated slots, each with its own stream,
// workspace (an hfe_plan) and decryption scratch.  Completion is signalled by a host function
// enqueued behind each step, which timestamps the requests and frees the slot.
//
// Host state stays bounded for a server that runs indefinitely: finished request records are
// kept for the last kRetainFinished finished tickets only, and latency samples for the last
// kLatWindow completions (percentiles are taken over that window, the mean over every completion
// since the last reset).  Each step is bracketed by timing events on its slot's stream; when a
// slot is reused (or the statistics are read) the step's device interval is compared with the
// intervals of the other slots' steps, which counts the pairs of steps that ran on the device at
// the same time.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hfe_internal.h"

namespace hfe {
namespace {
double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Request {
  const hfe_qct* q = nullptr;
  int32_t* ip_out = nullptr;   // decrypted inner products, or
  hfe_rct* ct_out = nullptr;   // the encrypted result (copied from the step's workspace)
  int64_t d3 = 0;
  int level = 0;
  int state = 0;  // 0 queued, 1 running, 2 done, < 0 rejected
  double t_submit = 0, t_admit = 0, t_done = 0;
};

struct Slot;
struct StepDone {
  hfe_server* srv;
  int slot;
  std::vector<uint64_t> tickets;
};

struct Slot {
  hfe_plan* plan = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_begin = nullptr, ev_end = nullptr;  // device interval of the slot's last step
  bool timed = false;                               // both events recorded, interval not yet read
  DevBuf y;
  bool busy = false;
  StepDone done;
};

constexpr size_t kRetainFinished = 1024;  // finished request records kept for poll / wait
constexpr size_t kLatWindow = 65536;      // latency samples kept for the percentiles
constexpr size_t kIntervals = 64;         // device intervals of recent steps kept for overlap

// Fixed-capacity ring of the most recent samples.
struct Window {
  std::vector<double> v;
  size_t next = 0;
  void push(double x) {
    if (v.size() < kLatWindow) {
      v.push_back(x);
    } else {
      v[next] = x;
      next = (next + 1) % kLatWindow;
    }
  }
  void clear() {
    v.clear();
    next = 0;
  }
};

struct Interval {
  int slot;
  float t0, t1;  // ms after the server's reference event
};

double pct(std::vector<double> v, double p) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const size_t i = std::min(v.size() - 1, (size_t)(p * (v.size() - 1) + 0.5));
  return v[i];
}
}  // namespace
}  // namespace hfe

struct hfe_server : hfe::HandleBase {
  const hfe_db* db = nullptr;
  int device = 0;
  int64_t max_cols = 0;
  int max_items = 0, max_level = 0;
  std::vector<std::unique_ptr<hfe::Slot>> slots;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, hfe::Request> reqs;
  std::deque<uint64_t> finished;  // tickets in the order they finished (done or failed)
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  hipEvent_t ev_ref = nullptr;  // recorded once at creation: origin of the device intervals
  std::deque<hfe::Interval> intervals;
  // statistics since creation / reset
  hfe::Window lat, svc;
  double lat_sum = 0;
  int64_t submitted = 0, completed = 0, rejected = 0, steps = 0, max_queue = 0, cols_steps = 0;
  int64_t busy_now = 0, max_busy = 0, overlap_pairs = 0;
  double t_first = -1, t_last = 0, cmp = 0;

  void finish_step(int si);
  void retire(uint64_t tk);       // caller holds mu
  void read_interval(int si);     // caller holds mu
  void run();
};

using namespace hfe;

static void on_step_done(void* p) {
  StepDone* d = static_cast<StepDone*>(p);
  d->srv->finish_step(d->slot);
}

void hfe_server::retire(uint64_t tk) {
  finished.push_back(tk);
  while (finished.size() > kRetainFinished) {
    auto it = reqs.find(finished.front());
    if (it != reqs.end() && (it->second.state == 2 || it->second.state < 0)) reqs.erase(it);
    finished.pop_front();
  }
}

void hfe_server::read_interval(int si) {
  Slot& sl = *slots[si];
  if (!sl.timed || sl.busy) return;
  sl.timed = false;
  float t0 = 0, t1 = 0;
  if (hipEventElapsedTime(&t0, ev_ref, sl.ev_begin) != hipSuccess ||
      hipEventElapsedTime(&t1, ev_ref, sl.ev_end) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  for (const Interval& o : intervals)
    if (o.slot != si && o.t0 < t1 && t0 < o.t1) ++overlap_pairs;
  intervals.push_back({si, t0, t1});
  if (intervals.size() > kIntervals) intervals.pop_front();
}

void hfe_server::finish_step(int si) {
  std::lock_guard<std::mutex> l(mu);
  Slot& sl = *slots[si];
  const double t = now_s();
  for (uint64_t tk : sl.done.tickets) {
    auto it = reqs.find(tk);
    if (it == reqs.end()) continue;
    Request& r = it->second;
    r.state = 2;
    r.t_done = t;
    const double ms = (t - r.t_submit) * 1e3;
    lat.push(ms);
    lat_sum += ms;
    svc.push((t - r.t_admit) * 1e3);
    ++completed;
    cmp += (double)r.d3 * db->d1;
    t_last = t;
    retire(tk);
  }
  sl.busy = false;
  --busy_now;
  cv.notify_all();
}

void hfe_server::run() {
  (void)hipSetDevice(device);
  const int64_t d1 = db->d1;
  for (;;) {
    int si = -1;
    std::vector<hfe_batch_item> items;
    std::vector<uint64_t> tickets;
    {
      std::unique_lock<std::mutex> l(mu);
      cv.wait(l, [&] {
        if (stop) return true;
        if (queue.empty()) return false;
        for (auto& s : slots)
          if (!s->busy) return true;
        return false;
      });
      if (stop) {
        cv.wait(l, [&] {
          for (auto& s : slots)
            if (s->busy) return false;
          return true;
        });
        for (uint64_t tk : queue) {
          reqs[tk].state = HFE_EBUSY;
          retire(tk);
        }
        queue.clear();
        return;
      }
      for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i]->busy) {
          si = (int)i;
          break;
        }
      // admission in arrival order: columns, request count and workspace of one step
      int64_t cols = 0;
      const double t = now_s();
      while (!queue.empty() && (int)items.size() < max_items) {
        Request& r = reqs[queue.front()];
        if (r.d3 > max_cols) {
          r.state = HFE_EBUSY;
          r.t_done = t;
          ++rejected;
          retire(queue.front());
          queue.pop_front();
          continue;
        }
        if (cols + r.d3 > max_cols) break;
        cols += r.d3;
        r.state = 1;
        r.t_admit = t;
        items.push_back({r.q, 0, d1});
        tickets.push_back(queue.front());
        queue.pop_front();
      }
      if (items.empty()) continue;
      read_interval(si);
      slots[si]->busy = true;
      max_busy = std::max(max_busy, ++busy_now);
      ++steps;
      cols_steps += cols;
    }
    Slot& sl = *slots[si];
    const bool timed = hipEventRecord(sl.ev_begin, sl.stream) == hipSuccess;
    hfe_status st = hfe_plan_run(sl.plan, items.data(), (int32_t)items.size(), 1, sl.stream);
    size_t off = 0;
    for (size_t i = 0; st == HFE_OK && i < items.size(); ++i) {
      const hfe_rct* view = nullptr;
      st = hfe_plan_result(sl.plan, (int32_t)i, &view);
      int32_t* ip_out = nullptr;
      hfe_rct* ct_out = nullptr;
      {
        std::lock_guard<std::mutex> l(mu);
        ip_out = reqs[tickets[i]].ip_out;
        ct_out = reqs[tickets[i]].ct_out;
      }
      if (st != HFE_OK) break;
      if (ct_out) {
        const size_t bytes = sizeof(uint64_t) * (size_t)view->level * view->d3 * view->R_out;
        if (hipMemcpyAsync(ct_out->outp, view->outp, bytes, hipMemcpyDeviceToDevice, sl.stream) != hipSuccess)
          st = fail(HFE_EDEVICE, "copy of an encrypted result failed");
      } else {
        st = decrypt_impl(db->keys, view, nullptr, ip_out, sl.y.as<uint64_t>() + off, sl.stream);
      }
      off += (size_t)view->level * view->d3 * view->rows;
    }
    sl.done.srv = this;
    sl.done.slot = si;
    sl.done.tickets = tickets;
    if (st == HFE_OK && timed && hipEventRecord(sl.ev_end, sl.stream) == hipSuccess) {
      std::lock_guard<std::mutex> l(mu);
      sl.timed = true;  // read once the step is done and the slot is free
    }
    hipError_t e = hipSuccess;
    if (st == HFE_OK) e = hipLaunchHostFunc(sl.stream, on_step_done, &sl.done);
    if (st != HFE_OK || e != hipSuccess) {
      std::lock_guard<std::mutex> l(mu);
      for (uint64_t tk : tickets) {
        reqs[tk].state = st != HFE_OK ? st : HFE_EDEVICE;
        retire(tk);
      }
      sl.timed = false;
      sl.busy = false;
      --busy_now;
      cv.notify_all();
    }
  }
}

namespace hfe {
void destroy_server(void* handle) {
  hfe_server* S = static_cast<hfe_server*>(handle);
  {
    std::lock_guard<std::mutex> l(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->worker.joinable()) S->worker.join();
  for (auto& sl : S->slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    hfe_free(sl->plan);
    sl->y.reset();
    if (sl->ev_begin) (void)hipEventDestroy(sl->ev_begin);
    if (sl->ev_end) (void)hipEventDestroy(sl->ev_end);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
  }
  if (S->ev_ref) (void)hipEventDestroy(S->ev_ref);
  S->kind = 0;
  delete S;
}
}  // namespace hfe

extern "C" {

hfe_status hfe_server_create(const hfe_db* db, size_t mem_budget, int64_t max_cols_per_step, int32_t max_items_per_step,
                             int32_t n_slots, uint32_t max_level, int32_t form, hfe_server** out) {
  if (!out) return fail(HFE_EINVAL, "out is NULL");
  *out = nullptr;
  const HandleBase* hb = static_cast<const HandleBase*>(static_cast<const void*>(db));
  if (!db || hb->kind != kDb) return fail(HFE_EINVAL, "invalid database handle");
  if (db->keys->family) return fail(HFE_EINVAL, "the server does not run the n^2 modulus chain");
  if (form != HFE_FORM_I8_MFMA && form != HFE_FORM_RNS_I8 && form != HFE_FORM_P2_I8)
    return fail(HFE_EINVAL, "the server runs an int8 form");
  if (!(db->forms & (uint32_t)form)) return fail(HFE_EINVAL, "database not prepared for this form");
  if (n_slots < 1 || n_slots > 8 || max_items_per_step < 1 || max_items_per_step > kMaxBatch ||
      max_cols_per_step < 1 || max_level < 1 || (int)max_level > db->keys->L)
    return fail(HFE_EINVAL, "bad server configuration");
  // workspace per query column of one step: query planes, small-modulus residues, contraction
  // output, result, decryption scratch (plus the column padding of each request)
  const FormShape fs = form_shape(db, form);
  const int planes = fs.planes;
  const int64_t qpad = fs.qpad;
  const int res_planes = fs.p2 ? db->n_p2 : fs.rns ? db->n_rns : 0;
  const int64_t ndb = 1ll << db->keys->P.log_n_db, R_max = ndb + db->d1;
  const size_t per_col = (size_t)(max_level + 1) * planes * db->KB * kKB +
                         (size_t)(max_level + 1) * res_planes * R_max * fs.res_bytes +
                         (size_t)(max_level + 1) * R_max * 8 + (size_t)max_level * R_max * 8 +
                         (size_t)max_level * db->d1 * 8;
  const size_t pad = (size_t)max_items_per_step * (qpad - 1) * (max_level + 1) * planes * db->KB * kKB;
  const size_t per_slot = mem_budget / (size_t)n_slots;
  if (per_slot <= pad + per_col) return fail(HFE_ENOMEM, "memory budget below one column per slot");
  const int64_t cols = std::min<int64_t>(max_cols_per_step, (int64_t)((per_slot - pad) / per_col));
  hfe_server* S = new (std::nothrow) hfe_server();
  if (!S) return fail(HFE_ENOMEM, "host allocation failed");
  S->kind = kServer;
  S->stream = nullptr;
  S->db = db;
  S->max_cols = cols;
  S->max_items = max_items_per_step;
  S->max_level = (int)max_level;
  (void)hipGetDevice(&S->device);
  for (int i = 0; i < n_slots; ++i) {
    auto sl = std::make_unique<Slot>();
    hfe_status st = hfe_plan_create(db, max_items_per_step, cols, max_level, form, &sl->plan);
    if (st == HFE_OK) st = sl->y.alloc(sizeof(uint64_t) * (size_t)max_level * cols * db->d1, nullptr);
    if (st == HFE_OK && hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking) != hipSuccess)
      st = fail(HFE_EDEVICE, "stream creation failed");
    if (st == HFE_OK && (hipEventCreate(&sl->ev_begin) != hipSuccess || hipEventCreate(&sl->ev_end) != hipSuccess))
      st = fail(HFE_EDEVICE, "event creation failed");
    S->slots.push_back(std::move(sl));
    if (st != HFE_OK) {
      destroy_server(S);
      return st;
    }
  }
  if (hipEventCreate(&S->ev_ref) != hipSuccess || hipEventRecord(S->ev_ref, S->slots[0]->stream) != hipSuccess ||
      hipEventSynchronize(S->ev_ref) != hipSuccess) {
    destroy_server(S);
    return fail(HFE_EDEVICE, "reference event failed");
  }
  S->worker = std::thread([S] { S->run(); });
  *out = S;
  return HFE_OK;
}

static hfe_server* as_server(hfe_server* s) {
  return (s && static_cast<HandleBase*>(static_cast<void*>(s))->kind == kServer) ? s : nullptr;
}

hfe_status hfe_server_submit(hfe_server* srv, const hfe_qct* q, int32_t* ip_out, uint64_t* ticket) {
  hfe_server* S = as_server(srv);
  const HandleBase* qb = static_cast<const HandleBase*>(static_cast<const void*>(q));
  if (!S || !q || qb->kind != kQct || !ip_out || !ticket) return fail(HFE_EINVAL, "invalid server, query, output or ticket");
  if (q->keys != S->db->keys) return fail(HFE_EINVAL, "query encrypted under other keys");
  if (q->K != S->db->K) return fail(HFE_ESHAPE, "query and database code lengths differ");
  if (q->level > S->max_level) return fail(HFE_ELEVEL, "query level above the server's maximum");
  std::lock_guard<std::mutex> l(S->mu);
  const uint64_t tk = S->next_ticket++;
  Request& r = S->reqs[tk];
  r.q = q;
  r.ip_out = ip_out;
  r.d3 = q->d3;
  r.level = q->level;
  r.t_submit = now_s();
  if (S->t_first < 0) S->t_first = r.t_submit;
  S->queue.push_back(tk);
  ++S->submitted;
  S->max_queue = std::max<int64_t>(S->max_queue, (int64_t)S->queue.size());
  S->cv.notify_all();
  *ticket = tk;
  return HFE_OK;
}

hfe_status hfe_server_submit_encrypted(hfe_server* srv, const hfe_qct* q, hfe_rct* result, uint64_t* ticket) {
  hfe_server* S = as_server(srv);
  const HandleBase* qb = static_cast<const HandleBase*>(static_cast<const void*>(q));
  const HandleBase* rb = static_cast<const HandleBase*>(static_cast<const void*>(result));
  if (!S || !q || qb->kind != kQct || !result || rb->kind != kRct || !ticket)
    return fail(HFE_EINVAL, "invalid server, query, result or ticket");
  if (q->keys != S->db->keys || result->keys != S->db->keys) return fail(HFE_EINVAL, "handles under other keys");
  if (q->K != S->db->K) return fail(HFE_ESHAPE, "query and database code lengths differ");
  if (q->level > S->max_level) return fail(HFE_ELEVEL, "query level above the server's maximum");
  const int64_t ndb = 1ll << S->db->keys->P.log_n_db;
  if (result->is_view || !result->outp || result->level != q->level || result->d3 != q->d3 || result->row0 != 0 ||
      result->rows != S->db->d1 || result->R_out != ndb + S->db->d1)
    return fail(HFE_ESHAPE, "result handle not shaped for this query (use hfe_result_create)");
  std::lock_guard<std::mutex> l(S->mu);
  const uint64_t tk = S->next_ticket++;
  Request& r = S->reqs[tk];
  r.q = q;
  r.ct_out = result;
  r.d3 = q->d3;
  r.level = q->level;
  r.t_submit = now_s();
  if (S->t_first < 0) S->t_first = r.t_submit;
  S->queue.push_back(tk);
  ++S->submitted;
  S->max_queue = std::max<int64_t>(S->max_queue, (int64_t)S->queue.size());
  S->cv.notify_all();
  *ticket = tk;
  return HFE_OK;
}

hfe_status hfe_server_poll(hfe_server* srv, uint64_t ticket, int32_t* state) {
  hfe_server* S = as_server(srv);
  if (!S || !state) return fail(HFE_EINVAL, "invalid server or state");
  std::lock_guard<std::mutex> l(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(HFE_EINVAL, "unknown ticket");
  *state = it->second.state;
  return HFE_OK;
}

hfe_status hfe_server_wait(hfe_server* srv, uint64_t ticket, int64_t timeout_ms) {
  hfe_server* S = as_server(srv);
  if (!S) return fail(HFE_EINVAL, "invalid server");
  std::unique_lock<std::mutex> l(S->mu);
  if (S->reqs.find(ticket) == S->reqs.end()) return fail(HFE_EINVAL, "unknown ticket");
  // looked up afresh on every wake-up: submissions may rehash the table while this thread waits,
  // and hfe_server_reset_stats may drop finished requests
  int state = 0;
  auto ready = [&] {
    auto it = S->reqs.find(ticket);
    state = it == S->reqs.end() ? 2 : it->second.state;
    return state == 2 || state < 0;
  };
  if (timeout_ms < 0)
    S->cv.wait(l, ready);
  else if (!S->cv.wait_for(l, std::chrono::milliseconds(timeout_ms), ready))
    return fail(HFE_EBUSY, "timed out");
  if (state == HFE_EBUSY) return fail(HFE_EBUSY, "request rejected: larger than one step, or the server stopped");
  if (state < 0) return fail(state, "the request's step failed");
  return HFE_OK;
}

hfe_status hfe_server_drain(hfe_server* srv, int64_t timeout_ms) {
  hfe_server* S = as_server(srv);
  if (!S) return fail(HFE_EINVAL, "invalid server");
  std::unique_lock<std::mutex> l(S->mu);
  auto idle = [&] {
    if (!S->queue.empty()) return false;
    for (auto& s : S->slots)
      if (s->busy) return false;
    return true;
  };
  if (timeout_ms < 0)
    S->cv.wait(l, idle);
  else if (!S->cv.wait_for(l, std::chrono::milliseconds(timeout_ms), idle))
    return fail(HFE_EBUSY, "timed out");
  return HFE_OK;
}

hfe_status hfe_server_stats(hfe_server* srv, hfe_server_report* out) {
  hfe_server* S = as_server(srv);
  if (!S || !out) return fail(HFE_EINVAL, "invalid server or out");
  std::memset(out, 0, sizeof(*out));
  std::vector<double> lat, svc;
  {
    // copies under the lock, sorting outside it: the completion callbacks take the same lock
    std::lock_guard<std::mutex> l(S->mu);
    for (size_t i = 0; i < S->slots.size(); ++i) S->read_interval((int)i);
    lat = S->lat.v;
    svc = S->svc.v;
    out->submitted = S->submitted;
    out->completed = S->completed;
    out->rejected = S->rejected;
    out->steps = S->steps;
    out->max_queue = S->max_queue;
    out->mean_ms = S->completed ? S->lat_sum / S->completed : 0.0;
    out->elapsed_s = S->t_first < 0 ? 0.0 : S->t_last - S->t_first;
    out->req_per_s = out->elapsed_s > 0 ? S->completed / out->elapsed_s : 0.0;
    out->cmp_per_s = out->elapsed_s > 0 ? S->cmp / out->elapsed_s : 0.0;
    out->mean_cols_per_step = S->steps ? (double)S->cols_steps / S->steps : 0.0;
    out->retained = (int64_t)S->reqs.size();
    out->max_busy_slots = S->max_busy;
    out->overlap_pairs = S->overlap_pairs;
  }
  out->p50_ms = pct(lat, 0.50);
  out->p99_ms = pct(lat, 0.99);
  out->service_p50_ms = pct(svc, 0.50);
  out->service_p99_ms = pct(std::move(svc), 0.99);
  return HFE_OK;
}

hfe_status hfe_server_reset_stats(hfe_server* srv) {
  hfe_server* S = as_server(srv);
  if (!S) return fail(HFE_EINVAL, "invalid server");
  std::lock_guard<std::mutex> l(S->mu);
  S->lat.clear();
  S->svc.clear();
  S->lat_sum = 0;
  S->submitted = S->completed = S->rejected = S->steps = S->max_queue = S->cols_steps = 0;
  S->max_busy = S->busy_now;
  S->overlap_pairs = 0;
  S->intervals.clear();
  S->t_first = -1;
  S->t_last = 0;
  S->cmp = 0;
  for (auto it = S->reqs.begin(); it != S->reqs.end();) {
    if (it->second.state == 2 || it->second.state < 0)
      it = S->reqs.erase(it);
    else
      ++it;
  }
  S->finished.clear();
  return HFE_OK;
}

}  // extern "C"
