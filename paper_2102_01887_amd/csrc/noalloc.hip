// llama_decide_full_noalloc: the full-scan decision (every configuration of
// each invocation's op, Eq. 1 after Alg. 1) without any device allocation.
//
// llama_decide's FULL mode buckets invocations by op in scratch that the
// context grows with hipMalloc.  This entry point takes the same scratch
// (bucket counts, starts and cursors per op, the permutation of invocations,
// per-chunk histograms) from one file-scope device array instead, so it can
// be called where allocating is not allowed.  The array's device address is
// resolved once per device, when a context is created on it, and only that
// address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

namespace {

constexpr int64_t NOALLOC_WORDS = LLAMA_NOALLOC_SCRATCH_BYTES / 4;
static_assert(LLAMA_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size must keep 256-byte alignment");

// One copy per device; every call on a device shares it.
static __device__ __align__(256) int32_t scratch[NOALLOC_WORDS];

constexpr int MAX_DEVICES = 256;
std::mutex g_mu;
int32_t* g_ptr[MAX_DEVICES] = {};  // device address of `scratch` per device, null until resolved

// Words of scratch one call needs, each part starting on a 64-word (256-byte) boundary.
int64_t round64(int64_t w) { return (w + 63) & ~(int64_t)63; }

struct Layout {
  int64_t cnt, start, cursor, perm, hist, total;
};

Layout layout(int64_t n_inv, int32_t n_ops) {
  Layout l{};
  l.cnt = 0;
  l.start = l.cnt + round64((int64_t)n_ops + 1);
  l.cursor = l.start + round64((int64_t)n_ops + 1);
  l.perm = l.cursor + round64(n_ops);
  l.hist = l.perm + round64(n_inv);
  l.total = l.hist + round64(llama::full_scan_hist_words(n_inv, n_ops));
  return l;
}

}  // namespace

namespace llama {

// Called with `device` current (context creation).  Resolves the device
// address of the scratch array once per device.
hipError_t noalloc_attach(int device) {
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_ptr[device] = static_cast<int32_t*>(p);
  return hipSuccess;
}

}  // namespace llama

extern "C" {

int64_t llama_decide_full_noalloc_words(int64_t n_inv, int32_t n_ops) {
  if (n_inv < 0 || n_ops < 0) return -1;
  return layout(n_inv, n_ops).total;
}

int llama_decide_full_noalloc(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed,
                              const int32_t* slo, const int64_t* queue, int32_t mode, int32_t* cfg,
                              uint8_t* flag, void* stream) {
  int rc = llama::enter(c);
  if (rc) return rc;
  if (!c->has_prof) return llama::fail(c, LLAMA_E_STATE, "decide_full_noalloc: call llama_set_dag and llama_set_profiles first");
  if (n < 0) return llama::fail(c, LLAMA_E_ARG, "decide_full_noalloc: n_inv < 0");
  if (n > 0 && (!op || !elapsed || !slo || !cfg)) return llama::fail(c, LLAMA_E_ARG, "decide_full_noalloc: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB)
    return llama::fail(c, LLAMA_E_ARG, "decide_full_noalloc: bad slack_mode %d", mode);
  if (n > INT32_MAX) return llama::fail(c, LLAMA_E_RANGE, "decide_full_noalloc: more than 2^31-1 invocations");
  const Layout l = layout(n, c->n_ops);
  if (l.total > NOALLOC_WORDS)
    return llama::fail(c, LLAMA_E_RANGE,
                       "decide_full_noalloc: %lld invocations over %d ops need %lld bytes of scratch, above the %lld-byte limit",
                       (long long)n, c->n_ops, (long long)(4 * l.total), (long long)LLAMA_NOALLOC_SCRATCH_BYTES);
  int32_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (c->device >= 0 && c->device < MAX_DEVICES) base = g_ptr[c->device];
  }
  if (!base) return llama::fail(c, LLAMA_E_STATE, "decide_full_noalloc: scratch address not resolved on device %d", c->device);
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.cfg = cfg; b.flag = flag; b.mode = mode;
  const llama::FullScratch w{base + l.cnt, base + l.start, base + l.cursor, base + l.perm, base + l.hist};
  const hipError_t e = llama::launch_decide_full(c->tables(), b, w, (hipStream_t)stream);
  if (e != hipSuccess) return llama::hip_fail(c, e, "decide_full_noalloc launch");
  return LLAMA_OK;
}

}  // extern "C"
