// Serving loop: continuous batching of arriving invocations by a persistent
// decision kernel.
//
// The Manager spawns invocations as their inputs resolve and the Configurator
// decides each one (Sec. 3.3, Sec. 4); the paper bounds each backend's commit
// queue to what saturates it (Sec. 4.3).  Here:
//   * a request holds one slot of a ring in pinned host memory mapped into the
//     device (16 bytes of request, 8 of result, 8 of device time, plus 32 of
//     BF16 features in the learned form) from admission until its decision is
//     collected; the ring is allocated with min(n_slots, memory budget /
//     bytes per request) slots, so the smaller of the two bounds how many
//     requests are admitted at once;
//   * submit writes the admitted requests into their slots and publishes them
//     by advancing a head word (release order);
//   * a persistent kernel, captured once per record set as a HIP graph and
//     replayed whenever it has exited with requests outstanding, claims
//     published requests as they appear (up to max_batch per wavefront in the
//     plain form, one per wavefront in the learned form), decides them and
//     writes each result word, tagged with its sequence number, after the
//     device clock at which it was written; it exits on the host's stop word,
//     once no wavefront has claimed work for IDLE_US, or after LIFE_US;
//   * poll collects decisions in admission order as their tags appear and
//     converts device times to host time: a clock handshake at open anchors
//     the mapping, and every REANCHOR_NS while the kernel runs one of its
//     wavefronts answers another handshake, which re-anchors it and refits
//     the device clock's rate against CLOCK_MONOTONIC (the two drift apart
//     by parts in 10^4, tens of microseconds a second, which would otherwise
//     add up in the reported latencies);
//   * the host tells whether the kernel is still running from an exit word
//     its last wavefront sets, and asks the runtime (the launch's event) only
//     once that word is set.
// There is no host worker thread and no launch per batch: batches form on the
// device from whatever has been published when a wavefront looks.  Each
// decision depends only on its own invocation, so it is the same alone as in
// any mix.
#include <hip/hip_runtime_api.h>

#include <time.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

using llama::enter;
using llama::fail;

namespace {

constexpr int64_t IDLE_US = 20000;   // the kernel exits once no wavefront has claimed work for this long
constexpr int64_t LIFE_US = 250000;  // and any wavefront after this long (the host relaunches)
constexpr int CLOCK_ROUNDS = 24;
constexpr int64_t REANCHOR_NS = 10000000;  // re-anchor the clock mapping this often while serving
constexpr int64_t PROBE_WAIT_NS = 50000;   // longest wait for a running kernel's answer
constexpr double FIT_NS = 50e6;            // shortest baseline for refitting the clock rate

int64_t mono_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (int64_t)ts.tv_sec * 1000000000ll + ts.tv_nsec;
}

template <typename T>
T* pinned(size_t n) {
  void* p = nullptr;
  if (hipHostMalloc(&p, sizeof(T) * (n ? n : 1), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
    return nullptr;
  std::memset(p, 0, sizeof(T) * (n ? n : 1));
  return static_cast<T*>(p);
}

}  // namespace

struct llama_server {
  llama_ctx* ctx = nullptr;
  llama_serve_config cfg{};
  int64_t bpr = 0;  // ring bytes per slot
  int64_t cap = 0;  // slots
  // ring and control words (pinned host memory, device-mapped): the words
  // the host writes in one 64-byte line, those the device writes in the next
  int4* req = nullptr;
  uint16_t* feat = nullptr;
  unsigned long long* res = nullptr;
  unsigned long long* ts = nullptr;
  long long* ctl = nullptr;
  long long* head_w = nullptr;
  int* stop_w = nullptr;
  int* probe_w = nullptr;
  int* ack_w = nullptr;
  unsigned long long* stamp_w = nullptr;
  int* exited_w = nullptr;
  unsigned long long* d_ctr = nullptr;  // device: next seq to claim, claims, largest claim, wavefronts alive,
                                        // clock of the latest claim
  std::vector<int64_t> t_arrival;
  // [tail, head) admitted and not collected; [tail, seen) decided (tags seen)
  int64_t head = 0, tail = 0, seen = 0;
  hipStream_t stream = nullptr, aux = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};  // per record set
  hipEvent_t done = nullptr;
  bool running = false;
  // host time of device tick k: t_anchor + (k - k_anchor) * ns_per_tick
  double ns_per_tick = 10.0, nominal_ns_per_tick = 10.0;
  double t_anchor = 0.0, t_first = 0.0;
  unsigned long long k_anchor = 0, k_first = 0;
  int probe_seq = 0;
  int64_t last_probe_ns = 0, last_query_ns = 0, anchors = 0, probes = 0, probe_timeouts = 0;
  double probe_rtt_min = 1e30, probe_rtt_last = 0.0;
  uint64_t tick_hz = 100000000ull;
  hipError_t error = hipSuccess;
  int64_t launches = 0;
  double clock_rtt_ns = 0.0;
  llama_serve_stats st{};
  std::mutex mu;

  int64_t slot(int64_t seq) const { return seq % cap; }

  bool decided(int64_t seq) const {
    const unsigned long long v = __atomic_load_n(res + slot(seq), __ATOMIC_ACQUIRE);
    return (uint32_t)(v >> 32) == (uint32_t)(seq + 1);
  }

  void advance_seen() {
    while (seen < head && decided(seen)) ++seen;
  }

  llama::ServeRing ring() const {
    llama::ServeRing r{};
    r.req = req;
    r.feat = feat;
    r.res = res;
    r.ts = ts;
    r.head = head_w;
    r.stop = stop_w;
    r.probe = probe_w;
    r.ack = ack_w;
    r.stamp = stamp_w;
    r.exited = exited_w;
    r.ctr = d_ctr;
    r.cap = cap;
    r.mode = cfg.slack_mode;
    r.chunk = cfg.learned ? 1 : std::max(1, std::min(64, cfg.max_batch));
    r.idle_ticks = (uint64_t)((double)tick_hz * IDLE_US * 1e-6);
    r.life_ticks = (uint64_t)((double)tick_hz * LIFE_US * 1e-6);
    return r;
  }

  hipError_t launch_kernel(int set) {
    const llama::DevTables t = ctx->tables_for(set);
    if (cfg.learned) {
      llama::LearnedArgs a{};
      const llama::Surrogate& su = ctx->surr;
      const int64_t nE = su.n_rows * llama::SURR_EMB;
      const int64_t ob1 = nE + (int64_t)llama::SURR_HID * llama::SURR_IN;
      const int64_t ob2 = ob1 + llama::SURR_HID + (int64_t)llama::SURR_HID * llama::SURR_HID;
      const int64_t ob3 = ob2 + llama::SURR_HID + 2 * llama::SURR_HID;
      a.feat = feat;
      a.E16 = su.E16.p;
      a.W1_16 = su.W1_16.p;
      a.W2p16 = su.W2p16.p;
      a.W3_16 = su.W3_16.p;
      a.b1 = su.master.as<float>() + ob1;
      a.b2 = su.master.as<float>() + ob2;
      a.b3 = su.master.as<float>() + ob3;
      a.spread_max = cfg.spread_max;
      return llama::launch_serve_learned(t, ring(), a, cfg.max_inflight, stream);
    }
    return llama::launch_serve_plain(t, ring(), cfg.max_inflight, stream);
  }

  // Replay the persistent kernel's graph for the current record set
  // (captured on first use).
  hipError_t relaunch() {
    const int set = ctx->rec_cur;
    if (!exec[set]) {
      hipGraph_t g = nullptr;
      if (cfg.learned) {
        const hipError_t pe = llama::prepare_serve_learned(ctx->tables_for(set));
        if (pe != hipSuccess) return pe;
      }
      hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return e;
      const hipError_t le = launch_kernel(set);
      e = hipStreamEndCapture(stream, &g);
      if (le != hipSuccess) e = le;
      if (e == hipSuccess) e = hipGraphInstantiate(&exec[set], g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) return e;
    }
    __atomic_store_n(exited_w, 0, __ATOMIC_RELEASE);
    hipError_t e = hipGraphLaunch(exec[set], stream);
    if (e == hipSuccess) e = hipEventRecord(done, stream);
    if (e == hipSuccess) {
      running = true;
      ++launches;
    }
    return e;
  }

  // Keep a kernel running while published requests are undecided.
  void ensure_running() {
    if (error != hipSuccess) return;
    if (running) {
      // a wavefront is alive: ask the runtime only every REANCHOR_NS (for errors)
      if (__atomic_load_n(exited_w, __ATOMIC_ACQUIRE) == 0) {
        const int64_t now = mono_ns();
        if (now - last_query_ns < REANCHOR_NS) return;
        last_query_ns = now;
      }
      const hipError_t q = hipEventQuery(done);
      if (q == hipErrorNotReady) return;
      if (q != hipSuccess) {
        error = q;
        return;
      }
      running = false;
    }
    advance_seen();
    if (seen < head) {
      const hipError_t e = relaunch();
      if (e != hipSuccess) error = e;
    }
  }

  double to_host_ns(unsigned long long tick) const {
    return t_anchor + (double)(long long)(tick - k_anchor) * ns_per_tick;
  }

  // Re-anchor the clock mapping from a handshake with the running kernel
  // (at most every REANCHOR_NS): write a new probe number, wait for its
  // acknowledgement, and keep the answer if its round trip is within 2 us
  // (or twice) of the shortest one seen so far; the rate is refitted over
  // the baseline from the first anchor once that spans FIT_NS.
  void reanchor() {
    const int64_t t0 = mono_ns();
    if (!running || t0 - last_probe_ns < REANCHOR_NS) return;
    last_probe_ns = t0;
    ++probes;
    const int k = ++probe_seq;
    __atomic_store_n(probe_w, k, __ATOMIC_RELEASE);
    int64_t t1 = t0;
    while (__atomic_load_n(ack_w, __ATOMIC_ACQUIRE) != k) {
      t1 = mono_ns();
      if (t1 - t0 > PROBE_WAIT_NS) {  // busy or exiting: try again later
        ++probe_timeouts;
        return;
      }
    }
    t1 = mono_ns();
    const double rtt = (double)(t1 - t0);
    probe_rtt_last = rtt;
    probe_rtt_min = std::min(probe_rtt_min, rtt);
    if (rtt > std::max(2.0 * probe_rtt_min, probe_rtt_min + 2000.0)) return;
    const unsigned long long tick = __atomic_load_n(stamp_w, __ATOMIC_RELAXED);
    const double mid = 0.5 * (double)(t0 + t1);
    if (mid - t_first >= FIT_NS && tick > k_first) ns_per_tick = (mid - t_first) / (double)(tick - k_first);
    t_anchor = mid;
    k_anchor = tick;
    ++anchors;
  }

  // Host/device clock anchor: the kernel stamps its clock when it sees each
  // round's flag; the round with the shortest host round trip fixes the
  // mapping to within half of it.
  hipError_t calibrate() {
    int khz = 0;
    hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device);
    if (e != hipSuccess) return e;
    if (khz <= 0) return hipErrorInvalidValue;
    tick_hz = (uint64_t)khz * 1000ull;
    ns_per_tick = nominal_ns_per_tick = 1e6 / (double)khz;
    int* flag = pinned<int>(2);
    unsigned long long* stamp = pinned<unsigned long long>(CLOCK_ROUNDS);
    if (!flag || !stamp) {
      if (flag) (void)hipHostFree(flag);
      if (stamp) (void)hipHostFree(stamp);
      return hipErrorOutOfMemory;
    }
    int* ack = flag + 1;
    e = llama::launch_clock_probe(flag, ack, stamp, CLOCK_ROUNDS, tick_hz, stream);  // gives up after 1 s
    double best = 1e30;
    int rounds = 0;
    for (int k = 0; k < CLOCK_ROUNDS && e == hipSuccess; ++k) {
      const int64_t t0 = mono_ns();
      __atomic_store_n(flag, k + 1, __ATOMIC_RELEASE);
      int64_t t1 = t0;
      while (__atomic_load_n(ack, __ATOMIC_ACQUIRE) != k + 1) {
        t1 = mono_ns();
        if (t1 - t0 > 200000000ll) break;  // 200 ms
      }
      if (__atomic_load_n(ack, __ATOMIC_ACQUIRE) != k + 1) break;
      t1 = mono_ns();
      const double rtt = (double)(t1 - t0);
      if (rtt < best) {
        best = rtt;
        t_anchor = t_first = 0.5 * (double)(t0 + t1);
        k_anchor = k_first = stamp[k];
      }
      ++rounds;
    }
    const hipError_t se = hipStreamSynchronize(stream);
    if (e == hipSuccess) e = se;
    (void)hipHostFree(flag);
    (void)hipHostFree(stamp);
    if (e == hipSuccess && rounds == 0) e = hipErrorNotReady;
    clock_rtt_ns = best;
    last_probe_ns = mono_ns();
    return e;
  }
};

extern "C" {

int64_t llama_serve_bytes_per_request(int32_t learned) {
  // request {op, elapsed, slo, 0} (16 B) + tagged result (8 B) + device time
  // (8 B), + 32 B of BF16 features in the learned form
  return learned ? 64 : 32;
}

int llama_serve_open(llama_ctx* c, const llama_serve_config* cfg, llama_server** out) {
  int rc = enter(c);
  if (rc) return rc;
  if (!cfg || !out) return fail(c, LLAMA_E_ARG, "serve_open: null pointer");
  *out = nullptr;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "serve_open: call llama_set_profiles first");
  if (cfg->n_slots < 1 || cfg->max_batch < 1 || cfg->max_inflight < 1 || cfg->max_inflight > 256)
    return fail(c, LLAMA_E_ARG, "serve_open: need n_slots >= 1, max_batch >= 1, 1 <= max_inflight <= 256");
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
  s->cap = std::min<int64_t>(cfg->n_slots, cfg->mem_budget_bytes / bpr);
  const size_t n = (size_t)s->cap;
  s->req = pinned<int4>(n);
  s->res = pinned<unsigned long long>(n);
  s->ts = pinned<unsigned long long>(n);
  s->feat = cfg->learned ? pinned<uint16_t>(n * llama::SURR_FEAT) : nullptr;
  s->ctl = pinned<long long>(16);
  if (s->ctl) {
    s->head_w = s->ctl;
    s->stop_w = reinterpret_cast<int*>(s->ctl + 1);
    s->probe_w = reinterpret_cast<int*>(s->ctl + 2);
    s->ack_w = reinterpret_cast<int*>(s->ctl + 8);
    s->stamp_w = reinterpret_cast<unsigned long long*>(s->ctl + 9);
    s->exited_w = reinterpret_cast<int*>(s->ctl + 10);
  }
  s->t_arrival.assign(n, 0);
  bool ok = s->req && s->res && s->ts && s->ctl && (!cfg->learned || s->feat);
  ok = ok && hipMalloc(&s->d_ctr, 5 * sizeof(unsigned long long)) == hipSuccess &&
       hipMemset(s->d_ctr, 0, 5 * sizeof(unsigned long long)) == hipSuccess &&
       hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
       hipStreamCreateWithFlags(&s->aux, hipStreamNonBlocking) == hipSuccess &&
       hipEventCreateWithFlags(&s->done, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    llama_serve_close(s);
    return fail(c, LLAMA_E_NOMEM, "serve_open: pinned ring, counters or streams");
  }
  const hipError_t e = s->calibrate();
  if (e != hipSuccess) {
    llama_serve_close(s);
    return llama::hip_fail(c, e, "serve_open: device clock calibration");
  }
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
  const int32_t k = (int32_t)std::max<int64_t>(0, std::min<int64_t>((int64_t)n, s->cap - (s->head - s->tail)));
  for (int32_t j = 0; j < k; ++j) {
    const int64_t seq = s->head + j;
    const int64_t o = s->slot(seq);
    s->req[o] = make_int4(op[j], elapsed[j], slo[j], 0);
    if (s->cfg.learned)
      std::memcpy(s->feat + o * llama::SURR_FEAT, feat + (int64_t)j * llama::SURR_FEAT, 2 * llama::SURR_FEAT);
    s->t_arrival[o] = arrival_ns ? arrival_ns[j] : now;
    if (tickets) tickets[j] = seq;
  }
  s->head += k;
  __atomic_store_n(s->head_w, (long long)s->head, __ATOMIC_RELEASE);  // publish
  s->st.admitted += k;
  s->st.rejected += n - k;
  s->st.bytes_in_use = (s->head - s->tail) * s->bpr;
  s->st.peak_bytes_in_use = std::max(s->st.peak_bytes_in_use, s->st.bytes_in_use);
  if (k) s->ensure_running();
  *n_admitted = k;
  return s->error == hipSuccess ? LLAMA_OK : LLAMA_E_DEVICE;
}

int llama_serve_poll(llama_server* s, int32_t max, int64_t* tickets, int32_t* choice, uint8_t* flag,
                     int64_t* latency_ns, int32_t* n_out, int32_t wait_ms) {
  if (!s || !n_out || max < 0) return LLAMA_E_ARG;
  *n_out = 0;
  const int64_t deadline = mono_ns() + (int64_t)std::max(0, wait_ms) * 1000000ll;
  std::unique_lock<std::mutex> lk(s->mu);
  int32_t k = 0;
  s->reanchor();
  for (;;) {
    s->ensure_running();
    if (s->error != hipSuccess) return LLAMA_E_DEVICE;
    while (k < max && s->tail < s->head && s->decided(s->tail)) {
      const int64_t o = s->slot(s->tail);
      const unsigned long long v = __atomic_load_n(s->res + o, __ATOMIC_ACQUIRE);
      if (tickets) tickets[k] = s->tail;
      if (choice) choice[k] = (int32_t)(v & 0x7FFFFFFFull) - 1;
      if (flag) flag[k] = (uint8_t)((v >> 31) & 1u);
      if (latency_ns) {
        latency_ns[k] = (int64_t)(s->to_host_ns(s->ts[o]) - (double)s->t_arrival[o]);
      }
      ++s->tail;
      ++k;
    }
    if (s->seen < s->tail) s->seen = s->tail;
    if (k > 0 || max == 0 || s->tail == s->head || mono_ns() >= deadline) break;
    lk.unlock();
    std::this_thread::yield();
    lk.lock();
  }
  s->st.collected += k;
  s->st.bytes_in_use = (s->head - s->tail) * s->bpr;
  *n_out = k;
  return LLAMA_OK;
}

int llama_serve_stats_get(llama_server* s, llama_serve_stats* out) {
  if (!s || !out) return LLAMA_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  s->advance_seen();
  unsigned long long ctr[5] = {0, 0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(ctr, s->d_ctr, sizeof(ctr), hipMemcpyDeviceToHost, s->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(s->aux);
  *out = s->st;
  out->decided = s->seen;
  out->batches = (int64_t)ctr[1];
  out->max_batch_seen = (int64_t)ctr[2];
  out->in_flight_batches = s->running && hipEventQuery(s->done) == hipErrorNotReady ? 1 : 0;
  out->capacity = s->cap;
  out->kernel_launches = s->launches;
  out->clock_rtt_ns = (int64_t)s->clock_rtt_ns;
  out->clock_anchors = s->anchors;
  out->clock_probes = s->probes;
  out->clock_probe_timeouts = s->probe_timeouts;
  out->clock_probe_rtt_min_ns = s->probes > s->probe_timeouts ? (int64_t)s->probe_rtt_min : 0;
  out->clock_probe_rtt_last_ns = (int64_t)s->probe_rtt_last;
  out->clock_rate_ppb = (int64_t)((s->ns_per_tick / s->nominal_ns_per_tick - 1.0) * 1e9);
  return e == hipSuccess && s->error == hipSuccess ? LLAMA_OK : LLAMA_E_DEVICE;
}

int llama_serve_close(llama_server* s) {
  if (!s) return LLAMA_OK;
  int rc = LLAMA_OK;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // decide what was admitted (bounded wait), then stop the kernel
    if (s->done && s->head_w) {
      const int64_t deadline = mono_ns() + 10000000000ll;
      for (;;) {
        s->ensure_running();
        s->advance_seen();
        if (s->seen >= s->head || s->error != hipSuccess || mono_ns() >= deadline) break;
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      }
    }
    if (s->stop_w) __atomic_store_n(s->stop_w, 1, __ATOMIC_RELEASE);
    if (s->running && hipEventSynchronize(s->done) != hipSuccess) s->error = hipErrorUnknown;
    s->running = false;
    if (s->error != hipSuccess) rc = LLAMA_E_DEVICE;
  }
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  for (hipGraphExec_t& x : s->exec)
    if (x) (void)hipGraphExecDestroy(x);
  if (s->done) (void)hipEventDestroy(s->done);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->aux) (void)hipStreamDestroy(s->aux);
  if (s->d_ctr) (void)hipFree(s->d_ctr);
  for (void* p : {(void*)s->req, (void*)s->res, (void*)s->ts, (void*)s->feat, (void*)s->ctl})
    if (p) (void)hipHostFree(p);
  delete s;
  return rc;
}

}  // extern "C"
