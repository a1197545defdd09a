// Serving loop: continuous batching of arriving invocations onto the GPU.
//
// The Manager spawns invocations as their inputs resolve and the Configurator
// decides each one (Sec. 3.3, Sec. 4); the paper bounds each backend's commit
// queue to what saturates it (Sec. 4.3).  Here:
//   * requests live in a ring of slots in pinned host memory that the
//     decision kernels read and write directly (no copies per batch);
//   * admission takes a request when a slot is free and the memory budget
//     (bytes per request x requests admitted and not yet collected) allows;
//   * a worker thread forms a batch from every admitted request not yet on
//     the GPU (up to max_batch, contiguous in the ring), launches it on one of
//     max_inflight streams while earlier batches still run, and retires
//     batches in order, stamping each request's decision time;
//   * the caller collects decisions in admission order, which frees slots.
// Each decision depends only on its own invocation, so it is the same alone
// as in any batch.
#include <hip/hip_runtime_api.h>

#include <time.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

using llama::fail;
using llama::enter;

namespace {

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

template <typename T>
T* pinned(size_t n) {
  void* p = nullptr;
  if (hipHostMalloc(&p, sizeof(T) * (n ? n : 1), hipHostMallocMapped) != hipSuccess) return nullptr;
  return static_cast<T*>(p);
}

}  // namespace

struct llama_server {
  llama_ctx* ctx = nullptr;
  llama_serve_config cfg{};
  int64_t bpr = 0;  // bytes charged per admitted request
  // ring (pinned host memory, visible to the GPU)
  int32_t *op = nullptr, *el = nullptr, *slo = nullptr, *choice = nullptr;
  uint8_t* flag = nullptr;
  uint16_t* feat = nullptr;
  std::vector<int64_t> t_arrival, t_done;
  std::vector<uint8_t> done;
  // sequence numbers: [tail, dispatched) on the GPU or done, [dispatched, head) admitted and waiting
  int64_t head = 0, dispatched = 0, tail = 0;
  struct Inflight {
    int64_t first, count;
    int stream;
  };
  std::deque<Inflight> inflight;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  std::vector<int> free_streams;
  std::mutex mu;
  std::condition_variable cv;
  std::thread worker;
  bool stop = false;
  hipError_t error = hipSuccess;
  llama_serve_stats st{};

  int64_t slot(int64_t seq) const { return seq % cfg.n_slots; }

  hipError_t launch(int64_t first, int64_t count, int s) {
    const int64_t o = slot(first);
    llama::Batch b{};
    b.n = count;
    b.op = op + o;
    b.elapsed = el + o;
    b.slo = slo + o;
    b.cfg = choice + o;
    b.flag = flag + o;
    b.mode = cfg.slack_mode;
    hipStream_t stream = streams[s];
    const llama::DevTables t = ctx->tables();
    if (cfg.learned) {
      llama::LearnedArgs a{};
      const llama::Surrogate& su = ctx->surr;
      const int64_t nE = su.n_rows * llama::SURR_EMB;
      const int64_t ob1 = nE + (int64_t)llama::SURR_HID * llama::SURR_IN;
      const int64_t ob2 = ob1 + llama::SURR_HID + (int64_t)llama::SURR_HID * llama::SURR_HID;
      const int64_t ob3 = ob2 + llama::SURR_HID + 2 * llama::SURR_HID;
      a.feat = feat + o * llama::SURR_FEAT;
      a.E16 = su.E16.p;
      a.W1_16 = su.W1_16.p;
      a.W2p16 = su.W2p16.p;
      a.W3_16 = su.W3_16.p;
      a.b1 = su.master.as<float>() + ob1;
      a.b2 = su.master.as<float>() + ob2;
      a.b3 = su.master.as<float>() + ob3;
      a.spread_max = cfg.spread_max;
      return llama::launch_decide_learned(t, b, a, stream);
    }
    return llama::launch_decide_indexed(t, b, stream);
  }

  // after the last activity the worker polls for SPIN_NS before sleeping, so
  // that a request arriving shortly after another is not delayed by a wake-up
  static constexpr int64_t SPIN_NS = 200000;

  void run() {
    (void)hipSetDevice(ctx->device);
    int64_t idle_since = mono_ns();
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool progress = false;
      // retire finished batches, oldest first
      while (!inflight.empty()) {
        const Inflight& f = inflight.front();
        const hipError_t q = hipEventQuery(events[f.stream]);
        if (q == hipErrorNotReady) break;
        if (q != hipSuccess && error == hipSuccess) error = q;
        const int64_t now = mono_ns();
        for (int64_t k = f.first; k < f.first + f.count; ++k) {
          t_done[slot(k)] = now;
          done[slot(k)] = 1;
        }
        st.decided += f.count;
        free_streams.push_back(f.stream);
        inflight.pop_front();
        progress = true;
      }
      // launch every admitted request that is not on the GPU yet
      while (dispatched < head && !free_streams.empty() && error == hipSuccess) {
        const int64_t first = dispatched;
        int64_t count = std::min<int64_t>(head - first, cfg.max_batch);
        count = std::min<int64_t>(count, cfg.n_slots - slot(first));  // contiguous in the ring
        const int s = free_streams.back();
        free_streams.pop_back();
        hipError_t e = launch(first, count, s);
        if (e == hipSuccess) e = hipEventRecord(events[s], streams[s]);
        if (e != hipSuccess) {
          error = e;
          free_streams.push_back(s);
          break;
        }
        inflight.push_back({first, count, s});
        dispatched += count;
        st.batches += 1;
        st.max_batch_seen = std::max<int64_t>(st.max_batch_seen, count);
        progress = true;
      }
      if (stop && inflight.empty() && (dispatched == head || error != hipSuccess)) break;
      if (progress) cv.notify_all();
      if (progress) idle_since = mono_ns();
      if (inflight.empty() && dispatched == head && !stop && mono_ns() - idle_since > SPIN_NS) {
        cv.wait(lk);  // idle for a while: sleep until a submit
      } else if (!progress) {
        lk.unlock();
        std::this_thread::yield();  // batches are running: poll their events
        lk.lock();
      }
    }
    cv.notify_all();
  }
};

extern "C" {

int64_t llama_serve_bytes_per_request(int32_t learned) {
  // op, elapsed, slo (12 B) + choice and flag (5 B) + arrival and decision
  // times (16 B) + slot state, rounded to 64 B; + 32 B of BF16 features
  return learned ? 96 : 64;
}

int llama_serve_open(llama_ctx* c, const llama_serve_config* cfg, llama_server** out) {
  int rc = enter(c);
  if (rc) return rc;
  if (!cfg || !out) return fail(c, LLAMA_E_ARG, "serve_open: null pointer");
  *out = nullptr;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "serve_open: call llama_set_profiles first");
  if (cfg->n_slots < 1 || cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 16)
    return fail(c, LLAMA_E_ARG, "serve_open: need n_slots >= 1, max_batch >= 1, 1 <= max_inflight <= 16");
  if (cfg->slack_mode != LLAMA_SLACK_PAPER && cfg->slack_mode != LLAMA_SLACK_PROB)
    return fail(c, LLAMA_E_ARG, "serve_open: bad slack_mode");
  if (!cfg->learned && !llama::records_current(c, cfg->slack_mode))
    return fail(c, LLAMA_E_STATE, "serve_open: the last relaxation left out the records of slack mode %d", cfg->slack_mode);
  if (cfg->learned && (!c->surr.ready || c->surr.n_rows != c->n_cfg))
    return fail(c, LLAMA_E_STATE, "serve_open: learned mode needs a surrogate");
  if (cfg->learned && !(cfg->spread_max >= 0.0f)) return fail(c, LLAMA_E_ARG, "serve_open: spread_max < 0");
  const int64_t bpr = llama_serve_bytes_per_request(cfg->learned);
  if (cfg->mem_budget_bytes < bpr) return fail(c, LLAMA_E_ARG, "serve_open: memory budget below one request");
  llama_server* s = new (std::nothrow) llama_server();
  if (!s) return LLAMA_E_NOMEM;
  s->ctx = c;
  s->cfg = *cfg;
  s->bpr = bpr;
  const size_t n = (size_t)cfg->n_slots;
  s->op = pinned<int32_t>(n);
  s->el = pinned<int32_t>(n);
  s->slo = pinned<int32_t>(n);
  s->choice = pinned<int32_t>(n);
  s->flag = pinned<uint8_t>(n);
  s->feat = cfg->learned ? pinned<uint16_t>(n * llama::SURR_FEAT) : nullptr;
  s->t_arrival.assign(n, 0);
  s->t_done.assign(n, 0);
  s->done.assign(n, 0);
  bool ok = s->op && s->el && s->slo && s->choice && s->flag && (!cfg->learned || s->feat);
  for (int k = 0; ok && k < cfg->max_inflight; ++k) {
    hipStream_t st = nullptr;
    hipEvent_t ev = nullptr;
    ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    if (st) s->streams.push_back(st);
    if (ev) s->events.push_back(ev);
    s->free_streams.push_back(k);
  }
  if (!ok) {
    llama_serve_close(s);
    return fail(c, LLAMA_E_NOMEM, "serve_open: pinned memory or streams");
  }
  s->worker = std::thread([s] { s->run(); });
  *out = s;
  return LLAMA_OK;
}

int llama_serve_submit(llama_server* s, int32_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                       const uint16_t* feat, const int64_t* arrival_ns, int64_t* tickets, int32_t* n_admitted) {
  if (!s || !n_admitted || n < 0) return LLAMA_E_ARG;
  *n_admitted = 0;
  if (n > 0 && (!op || !elapsed || !slo)) return LLAMA_E_ARG;
  if (s->cfg.learned && n > 0 && !feat) return LLAMA_E_ARG;
  const int64_t now = mono_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->error != hipSuccess) return LLAMA_E_DEVICE;
  s->st.submitted += n;
  const int64_t in_use = s->head - s->tail;
  const int64_t by_slots = s->cfg.n_slots - in_use;
  const int64_t by_memory = s->cfg.mem_budget_bytes / s->bpr - in_use;
  const int32_t k = (int32_t)std::max<int64_t>(0, std::min<int64_t>({(int64_t)n, by_slots, by_memory}));
  for (int32_t j = 0; j < k; ++j) {
    const int64_t seq = s->head + j;
    const int64_t o = s->slot(seq);
    s->op[o] = op[j];
    s->el[o] = elapsed[j];
    s->slo[o] = slo[j];
    if (s->cfg.learned) std::memcpy(s->feat + o * llama::SURR_FEAT, feat + (int64_t)j * llama::SURR_FEAT, 2 * llama::SURR_FEAT);
    s->t_arrival[o] = arrival_ns ? arrival_ns[j] : now;
    s->done[o] = 0;
    if (tickets) tickets[j] = seq;
  }
  s->head += k;
  s->st.admitted += k;
  s->st.rejected += n - k;
  s->st.bytes_in_use = (s->head - s->tail) * s->bpr;
  s->st.peak_bytes_in_use = std::max(s->st.peak_bytes_in_use, s->st.bytes_in_use);
  *n_admitted = k;
  if (k) s->cv.notify_all();
  return LLAMA_OK;
}

int llama_serve_poll(llama_server* s, int32_t max, int64_t* tickets, int32_t* choice, uint8_t* flag,
                     int64_t* latency_ns, int32_t* n_out, int32_t wait_ms) {
  if (!s || !n_out || max < 0) return LLAMA_E_ARG;
  *n_out = 0;
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [s] { return (s->tail < s->head && s->done[s->slot(s->tail)]) || s->error != hipSuccess; };
  if (wait_ms > 0 && !ready()) s->cv.wait_for(lk, std::chrono::milliseconds(wait_ms), ready);
  if (s->error != hipSuccess) return LLAMA_E_DEVICE;
  int32_t k = 0;
  while (k < max && s->tail < s->head && s->done[s->slot(s->tail)]) {
    const int64_t o = s->slot(s->tail);
    if (tickets) tickets[k] = s->tail;
    if (choice) choice[k] = s->choice[o];
    if (flag) flag[k] = s->flag[o];
    if (latency_ns) latency_ns[k] = s->t_done[o] - s->t_arrival[o];
    s->done[o] = 0;
    ++s->tail;
    ++k;
  }
  s->st.collected += k;
  s->st.bytes_in_use = (s->head - s->tail) * s->bpr;
  *n_out = k;
  return LLAMA_OK;
}

int llama_serve_stats_get(llama_server* s, llama_serve_stats* out) {
  if (!s || !out) return LLAMA_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->in_flight_batches = (int64_t)s->inflight.size();
  return s->error == hipSuccess ? LLAMA_OK : LLAMA_E_DEVICE;
}

int llama_serve_close(llama_server* s) {
  if (!s) return LLAMA_OK;
  int rc = LLAMA_OK;
  if (s->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv.notify_all();
    s->worker.join();
  }
  if (s->error != hipSuccess) rc = LLAMA_E_DEVICE;
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
  for (void* p : {(void*)s->op, (void*)s->el, (void*)s->slo, (void*)s->choice, (void*)s->flag, (void*)s->feat})
    if (p) (void)hipHostFree(p);
  delete s;
  return rc;
}

}  // extern "C"
