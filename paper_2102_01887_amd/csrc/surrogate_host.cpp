// Host side of the learned latency surrogate: parameter state (FP32 master,
// AdamW moments, BF16 shadows), training workspace, checkpoints, and the
// launches of its kernels.  Implements the llama_surrogate_* and
// llama_decide_learned entry points of include/llama.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "llama.h"
#include "llama_ctx.h"
#include "llama_internal.h"

using llama::fail;
using llama::hip_fail;
using llama::upload;
using llama::enter;
using llama::sync_ctx;

namespace {

constexpr int HID = llama::SURR_HID, IN = llama::SURR_IN, EMB = llama::SURR_EMB;
constexpr char MAGIC[8] = {'L', 'L', 'S', 'U', 'R', 'R', '0', '1'};

struct Layout {
  int64_t nE, oW1, ob1, oW2, ob2, oW3, ob3, n;
  explicit Layout(int64_t n_rows) {
    nE = n_rows * EMB;
    oW1 = nE;
    ob1 = oW1 + (int64_t)HID * IN;
    oW2 = ob1 + HID;
    ob2 = oW2 + (int64_t)HID * HID;
    oW3 = ob2 + HID;
    ob3 = oW3 + 2 * HID;
    n = ob3 + 2;
  }
};

llama::SurrogateBufs bufs(const llama_ctx* c) {
  const llama::Surrogate& s = c->surr;
  const Layout lay(s.n_rows);
  llama::SurrogateBufs w{};
  w.n_params = lay.n;
  w.nE = lay.nE;
  w.oW1 = lay.oW1;
  w.ob1 = lay.ob1;
  w.oW2 = lay.oW2;
  w.ob2 = lay.ob2;
  w.oW3 = lay.oW3;
  w.ob3 = lay.ob3;
  w.master = s.master.as<float>();
  w.adam_m = s.adam_m.as<float>();
  w.adam_v = s.adam_v.as<float>();
  w.grad = s.grad.as<float>();
  w.b1 = w.master + lay.ob1;
  w.b2 = w.master + lay.ob2;
  w.b3 = w.master + lay.ob3;
  w.E16 = s.E16.p;
  w.W1_16 = s.W1_16.p;
  w.W2_16 = s.W2_16.p;
  w.W2p16 = s.W2p16.p;
  w.W3_16 = s.W3_16.p;
  w.W1T16 = s.W1T16.p;
  w.W2T16 = s.W2T16.p;
  w.dE = s.dE.as<unsigned long long>();
  w.part = s.part.as<float>();
  w.X16 = s.X16.p;
  w.h1 = s.h1.p;
  w.h2 = s.h2.p;
  w.z1 = s.z1.as<float>();
  w.z2 = s.z2.as<float>();
  w.out = s.out.as<float>();
  return w;
}

int check_ready(llama_ctx* c, const char* fn) {
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "%s: call llama_set_profiles first", fn);
  if (!c->surr.ready || c->surr.n_rows != c->n_cfg)
    return fail(c, LLAMA_E_STATE, "%s: no surrogate for the current profiles (llama_surrogate_init/set/load)", fn);
  return LLAMA_OK;
}

// (Re)allocate parameter state for n_rows embedding rows and upload `params`.
int install(llama_ctx* c, const float* params, const float* m, const float* v, int64_t step) {
  llama::Surrogate& s = c->surr;
  s.ready = false;
  s.n_rows = c->n_cfg;
  const Layout lay(s.n_rows);
  s.n_params = lay.n;
  const size_t pb = sizeof(float) * (size_t)lay.n;
  int rc;
  if ((rc = upload(c, s.master, params, pb, "surrogate parameters")) ||
      (rc = upload(c, s.adam_m, m, pb, "AdamW first moment")) ||
      (rc = upload(c, s.adam_v, v, pb, "AdamW second moment")) ||
      (rc = upload(c, s.grad, nullptr, pb, "surrogate gradients")) ||
      (rc = upload(c, s.E16, nullptr, 2 * (size_t)lay.nE, "embedding (bf16)")) ||
      (rc = upload(c, s.W1_16, nullptr, 2 * (size_t)HID * IN, "W1 (bf16)")) ||
      (rc = upload(c, s.W2_16, nullptr, 2 * (size_t)HID * HID, "W2 (bf16)")) ||
      (rc = upload(c, s.W2p16, nullptr, 2 * (size_t)HID * HID, "W2 permuted (bf16)")) ||
      (rc = upload(c, s.W3_16, nullptr, 2 * (size_t)2 * HID, "W3 (bf16)")) ||
      (rc = upload(c, s.W1T16, nullptr, 2 * (size_t)HID * IN, "W1 transposed (bf16)")) ||
      (rc = upload(c, s.W2T16, nullptr, 2 * (size_t)HID * HID, "W2 transposed (bf16)")) ||
      (rc = upload(c, s.dE, nullptr, sizeof(uint64_t) * (size_t)(lay.nE ? lay.nE : 1), "embedding gradient")))
    return rc;
  if (hipMemsetAsync(s.dE.p, 0, s.dE.bytes, c->stream) != hipSuccess) return fail(c, LLAMA_E_DEVICE, "memset");
  if (!m && hipMemsetAsync(s.adam_m.p, 0, pb, c->stream) != hipSuccess) return fail(c, LLAMA_E_DEVICE, "memset");
  if (!v && hipMemsetAsync(s.adam_v.p, 0, pb, c->stream) != hipSuccess) return fail(c, LLAMA_E_DEVICE, "memset");
  hipError_t e = llama::launch_shadows(bufs(c), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate shadows");
  if ((rc = sync_ctx(c, "surrogate install"))) return rc;
  s.step = step;
  s.ready = true;
  return LLAMA_OK;
}

// Partial-gradient buffer for training batches of B rows (at most
// TRAIN_MAX_CHUNKS chunks per pass; larger batches run several passes).
int reserve_part(llama_ctx* c, int64_t B, hipStream_t stream) {
  llama::Surrogate& s = c->surr;
  const int64_t chunks = std::min<int64_t>((B + llama::TRAIN_ROWS - 1) / llama::TRAIN_ROWS, llama::TRAIN_MAX_CHUNKS);
  if (chunks <= s.part_chunks) return LLAMA_OK;
  if (stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
      return fail(c, LLAMA_E_STATE, "surrogate: training workspace for %lld rows must be reserved before graph capture", (long long)B);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "surrogate reserve sync");
  s.part_chunks = 0;
  const int64_t P = s.n_params - Layout(s.n_rows).nE;
  int rc = upload(c, s.part, nullptr, sizeof(float) * (size_t)chunks * (size_t)P, "partial gradients");
  if (rc) return rc;
  s.part_chunks = chunks;
  return LLAMA_OK;
}

// One training step on B rows: fused forward + backward per 64-row chunk,
// then the chunk sums, AdamW and the shadows (update), in passes of at most
// TRAIN_MAX_CHUNKS chunks.
hipError_t train_step(llama_ctx* c, int64_t B, const int32_t* rows, const uint16_t* feat, const float* y, float lr,
                      float wd, bool update, float* loss_sum, hipStream_t s) {
  const llama::SurrogateBufs w = bufs(c);
  const int64_t per = (int64_t)llama::TRAIN_ROWS * llama::TRAIN_MAX_CHUNKS;
  hipError_t e = hipSuccess;
  for (int64_t off = 0; off < B && e == hipSuccess; off += per) {
    const int64_t n = std::min(per, B - off);
    const bool last = off + per >= B;
    llama::TrainArgs a;
    a.n = n;
    a.rows = rows + off;
    a.feat = feat + off * llama::SURR_FEAT;
    a.y = y + off;
    a.inv_B = 1.0f / (float)B;
    a.loss_sum = loss_sum;
    e = llama::launch_train_chunks(w, a, s);
    if (e != hipSuccess) break;
    if (update && last) c->surr.step += 1;
    e = llama::launch_train_reduce(w, (int)((n + llama::TRAIN_ROWS - 1) / llama::TRAIN_ROWS), off == 0,
                                   update && last, lr, wd, c->surr.step, s);
  }
  return e;
}

int reserve_ws(llama_ctx* c, int64_t B, hipStream_t stream) {
  llama::Surrogate& s = c->surr;
  if (B <= s.ws_batch) return LLAMA_OK;
  if (stream) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &st) == hipSuccess && st != hipStreamCaptureStatusNone)
      return fail(c, LLAMA_E_STATE, "surrogate: workspace for %lld rows must be reserved before graph capture", (long long)B);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(c, e, "surrogate reserve sync");
  s.ws_batch = 0;
  const size_t b = (size_t)B;
  int rc;
  if ((rc = upload(c, s.X16, nullptr, 2 * b * IN, "X")) || (rc = upload(c, s.z1, nullptr, 4 * b * HID, "z1")) ||
      (rc = upload(c, s.h1, nullptr, 2 * b * HID, "h1")) || (rc = upload(c, s.z2, nullptr, 4 * b * HID, "z2")) ||
      (rc = upload(c, s.h2, nullptr, 2 * b * HID, "h2")) || (rc = upload(c, s.out, nullptr, 4 * b * 2, "out")))
    return rc;
  s.ws_batch = B;
  return LLAMA_OK;
}

// SplitMix64 (Steele, Lea, Flood 2014) and Box-Muller normals for the
// deterministic initial parameters.
struct SplitMix {
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() {
    const double u = uniform(), v = uniform();
    return std::sqrt(-2.0 * std::log(u)) * std::cos(6.283185307179586 * v);
  }
};

}  // namespace

extern "C" {

int64_t llama_surrogate_param_count(int64_t n_rows) { return n_rows < 0 ? -1 : Layout(n_rows).n; }

int llama_surrogate_init(llama_ctx* c, uint64_t seed, float mean_log_latency) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "surrogate_init: call llama_set_profiles first");
  if (!std::isfinite(mean_log_latency)) return fail(c, LLAMA_E_ARG, "surrogate_init: mean_log_latency not finite");
  const Layout lay(c->n_cfg);
  std::vector<float> p(lay.n, 0.0f);
  SplitMix rng{seed};
  for (int64_t i = 0; i < lay.nE; ++i) p[i] = (float)rng.normal();
  for (int64_t i = 0; i < (int64_t)HID * IN; ++i) p[lay.oW1 + i] = (float)(rng.normal() * std::sqrt(2.0 / IN));
  for (int64_t i = 0; i < (int64_t)HID * HID; ++i) p[lay.oW2 + i] = (float)(rng.normal() * std::sqrt(2.0 / HID));
  for (int64_t i = 0; i < 2 * HID; ++i) p[lay.oW3 + i] = (float)(rng.normal() * std::sqrt(1.0 / HID));
  p[lay.ob3] = mean_log_latency;
  p[lay.ob3 + 1] = mean_log_latency + 0.5f;
  return install(c, p.data(), nullptr, nullptr, 0);
}

int llama_surrogate_set(llama_ctx* c, const float* params, int64_t n) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "surrogate_set: call llama_set_profiles first");
  if (!params) return fail(c, LLAMA_E_ARG, "surrogate_set: null pointer");
  if (n != Layout(c->n_cfg).n) return fail(c, LLAMA_E_ARG, "surrogate_set: %lld parameters, need %lld", (long long)n, (long long)Layout(c->n_cfg).n);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(params[i])) return fail(c, LLAMA_E_RANGE, "surrogate_set: parameter %lld not finite", (long long)i);
  return install(c, params, nullptr, nullptr, 0);
}

int llama_surrogate_get(llama_ctx* c, float* params, int64_t n) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_get"))) return rc;
  if (!params || n != c->surr.n_params) return fail(c, LLAMA_E_ARG, "surrogate_get: need %lld floats", (long long)c->surr.n_params);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(params, c->surr.master.p, sizeof(float) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_get");
  return LLAMA_OK;
}

int llama_surrogate_grads(llama_ctx* c, float* grads, int64_t n) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_grads"))) return rc;
  if (!grads || n != c->surr.n_params) return fail(c, LLAMA_E_ARG, "surrogate_grads: need %lld floats", (long long)c->surr.n_params);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(grads, c->surr.grad.p, sizeof(float) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_grads");
  return LLAMA_OK;
}

int llama_surrogate_reserve(llama_ctx* c, int64_t max_batch) {
  int rc = enter(c);
  if (rc) return rc;
  if (max_batch < 0 || max_batch > INT32_MAX) return fail(c, LLAMA_E_ARG, "surrogate_reserve: bad size");
  return reserve_ws(c, max_batch, nullptr);
}

int llama_surrogate_forward(llama_ctx* c, int64_t n, const int32_t* d_rows, const uint16_t* d_feat, float* d_out,
                            void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_forward"))) return rc;
  if (n < 0 || n > INT32_MAX) return fail(c, LLAMA_E_ARG, "surrogate_forward: bad n");
  if (n == 0) return LLAMA_OK;
  if (!d_rows || !d_feat || !d_out) return fail(c, LLAMA_E_ARG, "surrogate_forward: null pointer");
  if ((rc = reserve_ws(c, n, (hipStream_t)stream))) return rc;
  llama::SurrogateBufs w = bufs(c);
  w.out = d_out;
  hipError_t e = llama::launch_surrogate_forward(w, n, d_rows, d_feat, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_forward launch");
  return LLAMA_OK;
}

int llama_surrogate_train_step(llama_ctx* c, int64_t batch, const int32_t* d_rows, const uint16_t* d_feat,
                               const float* d_y, float lr, float weight_decay, int32_t update, float* d_loss_sum,
                               void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_train_step"))) return rc;
  if (batch < 1 || batch > INT32_MAX) return fail(c, LLAMA_E_ARG, "surrogate_train_step: batch must be >= 1");
  if (!d_rows || !d_feat || !d_y) return fail(c, LLAMA_E_ARG, "surrogate_train_step: null pointer");
  if (!(lr >= 0.0f) || !(weight_decay >= 0.0f)) return fail(c, LLAMA_E_ARG, "surrogate_train_step: bad lr or weight decay");
  if ((rc = reserve_part(c, batch, (hipStream_t)stream))) return rc;
  hipError_t e = train_step(c, batch, d_rows, d_feat, d_y, lr, weight_decay, update != 0, d_loss_sum,
                            (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_train_step launch");
  return LLAMA_OK;
}

int llama_surrogate_fit(llama_ctx* c, int64_t n, const int32_t* d_rows, const uint16_t* d_feat, const float* d_y,
                        int32_t epochs, int64_t batch, float lr_max, float weight_decay, float* d_loss_sum,
                        void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_fit"))) return rc;
  if (batch < 1 || batch > INT32_MAX || n < batch || epochs < 1)
    return fail(c, LLAMA_E_ARG, "surrogate_fit: need epochs >= 1 and n >= batch >= 1");
  if (!d_rows || !d_feat || !d_y) return fail(c, LLAMA_E_ARG, "surrogate_fit: null pointer");
  if (!(lr_max >= 0.0f) || !(weight_decay >= 0.0f)) return fail(c, LLAMA_E_ARG, "surrogate_fit: bad lr or weight decay");
  if ((rc = reserve_part(c, batch, (hipStream_t)stream))) return rc;
  const int64_t per_epoch = n / batch, steps = per_epoch * epochs;
  hipStream_t s = (hipStream_t)stream;
  for (int64_t k = 0; k < steps; ++k) {
    const int64_t off = (k % per_epoch) * batch;
    const float lr = (float)(0.5 * lr_max * (1.0 + std::cos(3.141592653589793 * (double)k / (double)steps)));
    // the loss of the last tenth of the final epoch
    float* loss = (d_loss_sum && k >= steps - (per_epoch + 9) / 10) ? d_loss_sum : nullptr;
    const hipError_t e = train_step(c, batch, d_rows + off, d_feat + off * llama::SURR_FEAT, d_y + off, lr,
                                    weight_decay, true, loss, s);
    if (e != hipSuccess) return hip_fail(c, e, "surrogate_fit launch");
  }
  return LLAMA_OK;
}

int llama_surrogate_save(llama_ctx* c, const char* path) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "surrogate_save"))) return rc;
  if (!path) return fail(c, LLAMA_E_ARG, "surrogate_save: null path");
  const int64_t n = c->surr.n_params;
  std::vector<float> buf(3 * (size_t)n);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(buf.data(), c->surr.master.p, 4 * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + n, c->surr.adam_m.p, 4 * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * n, c->surr.adam_v.p, 4 * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "surrogate_save copy");
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, LLAMA_E_ARG, "surrogate_save: cannot open %s", path);
  const uint32_t version = 1;
  const int64_t hdr[3] = {c->surr.n_rows, n, c->surr.step};
  bool ok = std::fwrite(MAGIC, 1, 8, f) == 8 && std::fwrite(&version, 4, 1, f) == 1 &&
            std::fwrite(hdr, 8, 3, f) == 3 && std::fwrite(buf.data(), 4, buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, LLAMA_E_ARG, "surrogate_save: write to %s failed", path);
  return LLAMA_OK;
}

int llama_surrogate_load(llama_ctx* c, const char* path) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "surrogate_load: call llama_set_profiles first");
  if (!path) return fail(c, LLAMA_E_ARG, "surrogate_load: null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, LLAMA_E_ARG, "surrogate_load: cannot open %s", path);
  char magic[8];
  uint32_t version = 0;
  int64_t hdr[3];
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, MAGIC, 8) == 0 &&
            std::fread(&version, 4, 1, f) == 1 && version == 1 && std::fread(hdr, 8, 3, f) == 3;
  if (!ok || hdr[0] != c->n_cfg || hdr[1] != Layout(c->n_cfg).n || hdr[2] < 0) {
    std::fclose(f);
    return fail(c, LLAMA_E_STATE, "surrogate_load: %s is not a checkpoint for %lld profile rows", path, (long long)c->n_cfg);
  }
  const int64_t n = hdr[1];
  std::vector<float> buf(3 * (size_t)n);
  ok = std::fread(buf.data(), 4, buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) return fail(c, LLAMA_E_STATE, "surrogate_load: %s is truncated", path);
  return install(c, buf.data(), buf.data() + n, buf.data() + 2 * n, hdr[2]);
}

int llama_set_simulator(llama_ctx* c, const double* a_coef, const double* b_coef, double sigma) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_prof) return fail(c, LLAMA_E_STATE, "set_simulator: call llama_set_profiles first");
  if (!a_coef || !b_coef) return fail(c, LLAMA_E_ARG, "set_simulator: null pointer");
  if (!(sigma >= 0.0) || !std::isfinite(sigma)) return fail(c, LLAMA_E_ARG, "set_simulator: sigma must be finite and >= 0");
  const int64_t na = (int64_t)c->n_ops * c->n_hw;
  for (int64_t i = 0; i < na; ++i)
    if (!std::isfinite(a_coef[i])) return fail(c, LLAMA_E_RANGE, "set_simulator: a_coef[%lld] not finite", (long long)i);
  for (int v = 0; v < c->n_ops; ++v)
    if (!std::isfinite(b_coef[v])) return fail(c, LLAMA_E_RANGE, "set_simulator: b_coef[%d] not finite", v);
  std::vector<int32_t> row_op(c->n_cfg);
  for (int v = 0; v < c->n_ops; ++v)
    for (int64_t x = c->cfg_off[v]; x < c->cfg_off[v + 1]; ++x) row_op[x] = v;
  c->has_sim = false;
  if ((rc = upload(c, c->d_sim_a, a_coef, sizeof(double) * (size_t)na, "simulator coefficients")) ||
      (rc = upload(c, c->d_sim_b, b_coef, sizeof(double) * (size_t)c->n_ops, "simulator coefficients")) ||
      (rc = upload(c, c->d_sim_row_op, row_op.data(), sizeof(int32_t) * row_op.size(), "simulator row ops")) ||
      (rc = sync_ctx(c, "set_simulator")))
    return rc;
  c->sim_sigma = sigma;
  c->has_sim = true;
  return LLAMA_OK;
}

int llama_simulate(llama_ctx* c, int64_t n, uint64_t seed, int64_t first, int32_t* d_rows, uint16_t* d_feat,
                   float* d_y, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if (!c->has_sim) return fail(c, LLAMA_E_STATE, "simulate: call llama_set_simulator first");
  if (n < 0 || first < 0 || first > ((int64_t)1 << 32) - n)
    return fail(c, LLAMA_E_ARG, "simulate: need n >= 0, first >= 0 and first + n <= 2^32");
  if (n == 0) return LLAMA_OK;
  if (!d_rows || !d_feat || !d_y) return fail(c, LLAMA_E_ARG, "simulate: null pointer");
  llama::SimArgs a{};
  a.n = n;
  a.first = first;
  a.seed = seed;
  a.n_rows = c->n_cfg;
  a.n_hw = c->n_hw;
  a.row_op = c->d_sim_row_op.as<int32_t>();
  a.cfg_hw = c->d_cfg_hw.as<int32_t>();
  a.cfg_lat = c->d_cfg_lat.as<int32_t>();
  a.a_coef = c->d_sim_a.as<double>();
  a.b_coef = c->d_sim_b.as<double>();
  a.sigma = c->sim_sigma;
  a.rows = d_rows;
  a.feat = d_feat;
  a.y = d_y;
  hipError_t e = llama::launch_simulate(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "simulate launch");
  return LLAMA_OK;
}

int llama_decide_learned(llama_ctx* c, int64_t n, const int32_t* op, const int32_t* elapsed, const int32_t* slo,
                         const int64_t* queue, int32_t mode, const uint16_t* d_feat, float spread_max, int32_t* cfg,
                         uint8_t* flag, int32_t* d_lat_out, int64_t lat_stride, void* stream) {
  int rc = enter(c);
  if (rc) return rc;
  if ((rc = check_ready(c, "decide_learned"))) return rc;
  if (n < 0) return fail(c, LLAMA_E_ARG, "decide_learned: n_inv < 0");
  if (n > 0 && (!op || !elapsed || !slo || !cfg || !d_feat)) return fail(c, LLAMA_E_ARG, "decide_learned: null pointer");
  if (mode != LLAMA_SLACK_PAPER && mode != LLAMA_SLACK_PROB) return fail(c, LLAMA_E_ARG, "decide_learned: bad slack_mode %d", mode);
  if (!(spread_max >= 0.0f)) return fail(c, LLAMA_E_ARG, "decide_learned: spread_max must be >= 0");
  if (d_lat_out) {
    int64_t mx = 0;
    for (int v = 0; v < c->n_ops; ++v) mx = std::max<int64_t>(mx, c->cfg_off[v + 1] - c->cfg_off[v]);
    if (lat_stride < mx) return fail(c, LLAMA_E_ARG, "decide_learned: lat_stride %lld < %lld configurations", (long long)lat_stride, (long long)mx);
  }
  llama::Batch b{};
  b.n = n; b.op = op; b.elapsed = elapsed; b.slo = slo; b.queue = queue; b.cfg = cfg; b.flag = flag; b.mode = mode;
  const llama::SurrogateBufs w = bufs(c);
  llama::LearnedArgs a{};
  a.feat = d_feat;
  a.E16 = w.E16;
  a.W1_16 = w.W1_16;
  a.W2p16 = w.W2p16;
  a.W3_16 = w.W3_16;
  a.b1 = w.b1;
  a.b2 = w.b2;
  a.b3 = w.b3;
  a.spread_max = spread_max;
  a.lat_out = d_lat_out;
  a.lat_stride = lat_stride;
  hipError_t e = llama::launch_decide_learned(c->tables(), b, a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "decide_learned launch");
  return LLAMA_OK;
}

}  // extern "C"
