// Pipeline simulator on the GPU: the executions the learned latency
// surrogate is trained on, drawn where it trains.
//
// The paper's latencies depend on the content an invocation processes
// (Sec. 2, Fig. 3: object counts change detection and recognition time by up
// to 17x on CPU and 4x on GPU), which a static profile cannot see.  The
// simulator gives every execution a configuration row (uniform over the
// profile rows), content (object counts, resolution, motion, blur,
// brightness, branch hit rate, frame phase) and an observed ln latency: the
// row's profiled ln latency, plus a content term with per-(op, backend) and
// per-op coefficients, plus Gaussian noise.
//
// One thread per sample.  Random numbers: Philox4x32-10 (Salmon, Moraes,
// Dror, Shaw, SC 2011) under key (seed low, seed high) at counters
// (sample, k, 0, 0), k = 0..5; the 24 words are used in a fixed order (see
// llama_simulate in include/llama.h), so a sample does not depend on how
// the samples are split between calls.  All arithmetic is FP64; features are
// rounded to FP32 and then to BF16, y to FP32.
#include <hip/hip_runtime.h>

#include "llama_internal.h"

namespace llama {
namespace {

constexpr uint32_t PHILOX_M0 = 0xD2511F53u, PHILOX_M1 = 0xCD9E8D57u;
constexpr uint32_t PHILOX_W0 = 0x9E3779B9u, PHILOX_W1 = 0xBB67AE85u;

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = PHILOX_M0 * c.x, hi0 = __umulhi(PHILOX_M0, c.x);
    const uint32_t lo1 = PHILOX_M1 * c.z, hi1 = __umulhi(PHILOX_M1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  return c;
}

__device__ __forceinline__ double unit(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

// Smallest k <= cap with u < P(X <= k), X ~ Poisson(rate) (pmf recurrence).
__device__ __forceinline__ int poisson_inv(double u, double rate, int cap) {
  double p = exp(-rate), cdf = p;
  int k = 0;
  while (!(u < cdf) && k < cap) {
    ++k;
    p = p * rate / (double)k;
    cdf += p;
  }
  return k;
}

// Smallest k <= m with u < P(X <= k), X ~ Binomial(m, p).
__device__ __forceinline__ int binomial_inv(double u, int m, double p) {
  const double q = 1.0 - p;
  double pk = pow(q, (double)m), cdf = pk;
  int k = 0;
  while (!(u < cdf) && k < m) {
    ++k;
    pk = pk * (double)(m - k + 1) / (double)k * (p / q);
    cdf += pk;
  }
  return k;
}

__global__ __launch_bounds__(256) void simulate_kernel(SimArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n) return;
  const int64_t i = a.first + s;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
  uint32_t w[24];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const uint4 q = philox4x32_10(make_uint4((uint32_t)i, (uint32_t)k, 0u, 0u), k0, k1);
    w[4 * k] = q.x;
    w[4 * k + 1] = q.y;
    w[4 * k + 2] = q.z;
    w[4 * k + 3] = q.w;
  }
  const int row = (int)(((uint64_t)w[0] * (uint64_t)a.n_rows) >> 32);
  const double two_pi = 6.283185307179586;
  const double r1 = sqrt(-2.0 * log(unit(w[1])));
  const double z_people = r1 * cos(two_pi * unit(w[2]));
  const double z_cars = r1 * sin(two_pi * unit(w[2]));
  const double r2 = sqrt(-2.0 * log(unit(w[3])));
  const double z_noise = r2 * cos(two_pi * unit(w[4]));
  const double ln2 = 0.6931471805599453;
  const int people = poisson_inv(unit(w[5]), exp(ln2 + z_people), 60);
  const int cars = poisson_inv(unit(w[6]), exp(ln2 + z_cars), 60 - people);
  const int faces = binomial_inv(unit(w[7]), people, 0.6);
  const int res = (int)(((uint64_t)w[8] * 3ull) >> 32);
  const int wd = res == 0 ? 854 : res == 1 ? 1280 : 1920;
  const int ht = res == 0 ? 480 : res == 1 ? 720 : 1080;
  const double px = (double)wd * (double)ht;
  const double g3 = -log(unit(w[12]) * unit(w[13]) * unit(w[14]));
  const double g7 = -log(unit(w[15]) * unit(w[16]) * unit(w[17]) * unit(w[18]) * unit(w[19]) * unit(w[20]) *
                         unit(w[21]));
  const double phase = two_pi * unit(w[22]);
  const int n_obj = people + cars;
  double f[16];
  f[0] = people / 60.0;
  f[1] = cars / 60.0;
  f[2] = faces / 60.0;
  f[3] = log1p((double)n_obj) / log(61.0);
  f[4] = wd / 1920.0;
  f[5] = ht / 1080.0;
  f[6] = px / (1920.0 * 1080.0);
  f[7] = unit(w[9]);
  f[8] = unit(w[10]);
  f[9] = unit(w[11]);
  f[10] = g3 / (g3 + g7);
  f[11] = sin(phase);
  f[12] = cos(phase);
  f[13] = f[14] = f[15] = 0.0;
  const int op = a.row_op[row];
  const int h = a.cfg_hw[row];
  const double mu = log((double)a.cfg_lat[row]) + a.a_coef[(int64_t)op * a.n_hw + h] * log1p((double)n_obj) +
                    a.b_coef[op] * log(px / (1280.0 * 720.0));
  a.rows[s] = row;
  a.y[s] = (float)(mu + a.sigma * z_noise);
  __bf16* out = reinterpret_cast<__bf16*>(a.feat) + s * 16;
#pragma unroll
  for (int j = 0; j < 16; ++j) out[j] = (__bf16)(float)f[j];
}

}  // namespace

hipError_t launch_simulate(const SimArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(simulate_kernel, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace llama
