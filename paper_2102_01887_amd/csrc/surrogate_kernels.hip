// HIP kernels (gfx950) of the learned latency surrogate.
//
// The network, per (invocation, configuration) row:
//   x = [E[row] (16), f (16)] (BF16)
//   h1 = GELU(W1 x + b1), h2 = GELU(W2 h1 + b2) (256 each, rounded to BF16)
//   (mu, q) = W3 h2 + b3 : mean and 95th percentile of ln(latency in us)
// GELU is the tanh form (Hendrycks & Gimpel 2016), written here as
// x * sigmoid(2u), u = sqrt(2/pi) (x + 0.044715 x^3), which is the same
// function.
//
// Training: train_chunk_kernel runs the forward and backward passes of 64
// rows per workgroup with v_mfma_f32_16x16x32_bf16 (FP32 accumulation) and
// every activation in LDS and registers, writing per-chunk partial
// gradients; train_reduce_kernel sums them, applies AdamW to the FP32 master
// weights and writes the BF16 shadows.  gemm_bf16_kernel (LDS tiles) serves
// the stand-alone training-path forward.
//
// Inference: decide_learned_kernel, persistent, two wavefronts per
// invocation, each taking 32 of every 64 configuration rows.  W1 and
// K-permuted copies of W2 and W3 sit in LDS (about 156 KB, rows padded
// against bank conflicts); hidden activations never leave registers: the
// output fragment of each lane in layers 1 and 2 is, up to a fixed
// permutation of the contraction index, exactly its input fragment of the
// next layer.  Each row's p95 latency feeds
// the Eq. 1 scan of the plain path, reduced across the wavefront.
#include <hip/hip_runtime.h>

#include "llama_internal.h"
#include "serve_device.h"

namespace llama {
namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float GELU_C = 0.7978845608028654f;
constexpr float GELU_A = 0.044715f;
constexpr float TAU = 0.95f;
constexpr int HID = 256, IN = 32, EMB = 16;

// x * sigmoid(2u) with the hardware reciprocal (about one ulp) instead of an
// IEEE division: the result is rounded to BF16, and the fused inference
// evaluates 512 of these per row, which made the division its largest VALU
// cost.  Large negative x: the exponential overflows to infinity and the
// reciprocal to 0, giving -0.
// The exponent -2u log2(e) = x (k1 + k2 x^2) goes to exp2 directly, with
// k1 = -2 log2(e) sqrt(2/pi) and k2 = k1 * 0.044715 folded at compile time.
constexpr float GELU_K1 = -2.0f * 1.4426950408889634f * GELU_C;
constexpr float GELU_K2 = GELU_K1 * GELU_A;
__device__ __forceinline__ float gelu(float x) {
  const float t = x * fmaf(GELU_K2, x * x, GELU_K1);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

// GELU and its derivative from one sigmoid: with s = sigmoid(2u) (the
// forward's exp2 and reciprocal), GELU(x) = x s and GELU'(x) = s + 2 sqrt(2/pi)
// x s (1 - s) (1 + 3 * 0.044715 x^2), the derivative of the tanh form written
// with tanh(u) = 2s - 1.  h is bit-identical to gelu(x).
constexpr float GELU_D1 = 2.0f * GELU_C, GELU_D2 = 3.0f * GELU_A;
__device__ __forceinline__ void gelu_and_grad(float x, float* h, float* gp) {
  const float x2 = x * x;
  const float t = x * fmaf(GELU_K2, x2, GELU_K1);
  const float sg = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
  *h = x * sg;
  const float q = fmaf(-sg, sg, sg);  // s (1 - s)
  *gp = fmaf(GELU_D1 * x * q, fmaf(GELU_D2, x2, 1.0f), sg);
}

__device__ __forceinline__ floatx4 mfma16x16x32(const bf16x8& a, const bf16x8& b, const floatx4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// C[m][n] (+)= sum_k A(m,k) B(k,n) (+ bias[n]), BF16 inputs with arbitrary
// element strides, FP32 output.  64x64 tile per 256-lane workgroup, each
// wavefront a 32x32 quarter (2x2 MFMA blocks), K in steps of 32 through LDS.
// Tiles are loaded along whichever index has unit stride, so both plain and
// transposed operands read coalesced.  Used by the training-path forward
// (llama_surrogate_forward); training steps run the fused kernels below.
// ---------------------------------------------------------------------------
// One thread's share of a 64 x 32 operand tile: 8 consecutive elements along
// the operand's contiguous dimension (the row dimension when `along_row`, else
// k), with one 16-byte load when the 8 lie inside the matrix and are aligned,
// else 8 bounds-checked loads.
struct TileVec {
  bf16x8 v;
};
__device__ __forceinline__ TileVec load_tile_vec(const bf16* __restrict__ p, int64_t s_row, int64_t s_k, bool along_row,
                                                 bool vec_ok, int row0, int rows, int k0, int kend, int tid) {
  TileVec t;
  const int rr = along_row ? (tid & 7) * 8 : tid >> 2;   // first row of the vector
  const int kk = along_row ? tid >> 3 : (tid & 3) * 8;   // first k of the vector
  const int gr = row0 + rr, gk = k0 + kk;
  const bool inside = along_row ? (gr + 8 <= rows && gk < kend) : (gr < rows && gk + 8 <= kend);
  if (vec_ok && inside) {
    t.v = *reinterpret_cast<const bf16x8*>(p + (int64_t)gr * s_row + (int64_t)gk * s_k);
  } else {
    const bf16 zero = (bf16)0.0f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int r = along_row ? gr + j : gr, k = along_row ? gk : gk + j;
      t.v[j] = (r < rows && k < kend) ? p[(int64_t)r * s_row + (int64_t)k * s_k] : zero;
    }
  }
  return t;
}

__device__ __forceinline__ void store_tile_vec(bf16 (*sT)[40], const TileVec& t, bool along_row, int tid) {
  if (along_row) {
    const int rr = (tid & 7) * 8, kk = tid >> 3;
#pragma unroll
    for (int j = 0; j < 8; ++j) sT[rr + j][kk] = t.v[j];
  } else {
    *reinterpret_cast<bf16x8*>(&sT[tid >> 2][(tid & 3) * 8]) = t.v;
  }
}

__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const bf16* __restrict__ a,
                                                        int64_t sam, int64_t sak, const bf16* __restrict__ b,
                                                        int64_t sbk, int64_t sbn, float* __restrict__ c,
                                                        int64_t ldc, const float* __restrict__ bias,
                                                        int accumulate) {
  __shared__ __attribute__((aligned(16))) bf16 sA[64][40];  // [m][k], 8 pad columns
  __shared__ __attribute__((aligned(16))) bf16 sB[64][40];  // [n][k]
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb0 = 0, kb1 = K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int g = lane >> 4, r = lane & 15;
  // each operand is staged along its contiguous dimension; 16-byte loads need
  // a unit stride there, the other stride a multiple of 8 and an aligned base
  const bool a_along_m = sam == 1 && sak != 1;
  const bool b_along_n = sbn == 1 && sbk != 1;
  const bool a_vec = (a_along_m ? (sak % 8 == 0) : (sak == 1 && sam % 8 == 0)) &&
                     (reinterpret_cast<uintptr_t>(a) & 15) == 0;
  const bool b_vec = (b_along_n ? (sbk % 8 == 0) : (sbk == 1 && sbn % 8 == 0)) &&
                     (reinterpret_cast<uintptr_t>(b) & 15) == 0;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
  // the next tile is loaded into registers while the current one is multiplied
  TileVec ta = load_tile_vec(a, sam, sak, a_along_m, a_vec, m0, M, kb0, kb1, tid);
  TileVec tb = load_tile_vec(b, sbn, sbk, b_along_n, b_vec, n0, N, kb0, kb1, tid);
  for (int k0 = kb0; k0 < kb1; k0 += 32) {
    store_tile_vec(sA, ta, a_along_m, tid);
    store_tile_vec(sB, tb, b_along_n, tid);
    __syncthreads();
    if (k0 + 32 < kb1) {
      ta = load_tile_vec(a, sam, sak, a_along_m, a_vec, m0, M, k0 + 32, kb1, tid);
      tb = load_tile_vec(b, sbn, sbk, b_along_n, b_vec, n0, N, k0 + 32, kb1, tid);
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
      const bf16x8 af = *reinterpret_cast<const bf16x8*>(&sA[wm + mb * 16 + r][8 * g]);
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const bf16x8 bfr = *reinterpret_cast<const bf16x8*>(&sB[wn + nb * 16 + r][8 * g]);
        acc[mb][nb] = mfma16x16x32(af, bfr, acc[mb][nb]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = m0 + wm + mb * 16 + 4 * g + i;
        const int col = n0 + wn + nb * 16 + r;
        if (row < M && col < N) {
          float x = acc[mb][nb][i] + (bias ? bias[col] : 0.0f);
          if (accumulate) x += c[row * ldc + col];
          c[row * ldc + col] = x;
        }
      }
}

// X[m] = [E16[rows[m]], feat[m]]
__global__ __launch_bounds__(256) void gather_x_kernel(int64_t B, const int32_t* rows, const bf16* feat,
                                                       const bf16* E16, bf16* X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * IN) return;
  const int64_t m = e / IN;
  const int j = (int)(e % IN);
  X[e] = j < EMB ? E16[(int64_t)rows[m] * EMB + j] : feat[m * EMB + (j - EMB)];
}

__global__ __launch_bounds__(256) void gelu_round_kernel(int64_t n, const float* z, bf16* h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) h[i] = (bf16)gelu(z[i]);
}

// BF16 shadows of one master parameter: E, W1 (and W1T[k][o]), W2 (and
// W2T[k][o] and the K-permuted W2p used by the fused inference kernel:
// W2p[o][32 kb + 8 g + j] = W2[o][32 kb + (j < 4 ? 4g + j : 12 + 4g + j)]),
// W3; the biases have none.
struct Shadows {
  bf16 *E16, *W1_16, *W1T16, *W2_16, *W2T16, *W2p16, *W3_16;
  int64_t nE;
};

__device__ __forceinline__ int w2p_column(int c) {
  const int kb = c >> 5, ci = c & 31;
  const int g = ci < 16 ? ci >> 2 : (ci - 16) >> 2;
  const int j = ci < 16 ? ci & 3 : 4 + ((ci - 16) & 3);
  return 32 * kb + 8 * g + j;
}

__device__ __forceinline__ void write_shadow(const Shadows& sh, int64_t i, float x) {
  const bf16 h = (bf16)x;
  if (i < sh.nE) {
    sh.E16[i] = h;
    return;
  }
  int64_t j = i - sh.nE;
  if (j < HID * IN) {
    sh.W1_16[j] = h;
    sh.W1T16[(j % IN) * HID + j / IN] = h;
    return;
  }
  j -= HID * IN + HID;
  if (j < 0) return;  // b1
  if (j < HID * HID) {
    const int o = (int)(j / HID), c = (int)(j % HID);
    sh.W2_16[j] = h;
    sh.W2T16[(int64_t)c * HID + o] = h;
    sh.W2p16[(int64_t)o * HID + w2p_column(c)] = h;
    return;
  }
  j -= HID * HID + HID;
  if (j >= 0 && j < 2 * HID) sh.W3_16[j] = h;  // else b2 or b3
}

__global__ __launch_bounds__(256) void shadows_kernel(const float* master, int64_t n, Shadows sh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) write_shadow(sh, i, master[i]);
}

// ---------------------------------------------------------------------------
// Fused training step (launch_train_chunks / launch_train_reduce).
//
// A workgroup of eight wavefronts (two per SIMD) takes TRAIN_ROWS rows and
// runs, with
// the same rounding points as the product-by-product form (BF16 operands,
// FP32 accumulation, activations and their gradients rounded to BF16):
//   X = [E[row], f]               LDS, row-major and transposed
//   z1 = X W1^T + b1              MFMA, K = 32; wavefront w: columns 32w..32w+31
//   h1 = GELU(z1)                 LDS, row-major and transposed; GELU'(z1) kept in
//                                 registers (one sigmoid gives both)
//   z2 = h1 W2^T + b2             MFMA, K = 256, all of the wavefront's W2 fragments
//                                 loaded from L2 before the first product
//   h2 = GELU(z2)                 LDS; GELU'(z2) kept in registers
//   (mu, q) = h2 W3^T + b3        VALU, TR_LPR lanes per row, W3 staged in LDS
//   dout = loss gradient          LDS; rows past the batch get 0
//   dW3 = dout^T h2, db3          VALU, a lane per column
//   dz2 = (dout W3) GELU'(z2)     in registers, then LDS (both layouts); db2
//   dz1 = (dz2 W2) GELU'(z1)      MFMA with the transposed W2 shadow, then LDS; db1
//   dW1 = dz1^T X                 MFMA over the rows
//   dE[row] += (dz1 W1)[:, :16]   MFMA with the transposed W1 shadow, 64-bit
//                                 fixed-point integer atomics
//   dW2 = dz2^T h1                MFMA over the rows, four passes of 64 columns,
//                                 last, so that its stores delay no load
// Partial gradients go to part[chunk] in the parameter order after E; the
// reduce kernel sums them in chunk order, so the sum does not depend on
// timing.  dE is summed in fixed point (units of 2^-40, each term clamped
// to |t| <= 2^8): integer addition is associative, so its atomics give the
// same sum in any order and a training run is repeatable bit for bit.  At
// most 256 chunks x 64 rows add into one element per launch, so the sum
// stays below 2^(8 + 40 + 14) = 2^62.
// ---------------------------------------------------------------------------
constexpr float DE_SCALE = 1099511627776.0f;  // 2^40
constexpr double DE_UNIT = 1.0 / 1099511627776.0;
constexpr float DE_CLAMP = 256.0f;
constexpr int TR_LDX = IN + 8;          // bf16 stride of X rows
constexpr int TR_LDT = TRAIN_ROWS + 8;  // bf16 stride of transposed rows
constexpr int TR_LDA = HID + 8;         // bf16 stride of activation rows
constexpr size_t TR_OFF_XT = sizeof(bf16) * TRAIN_ROWS * TR_LDX;
constexpr size_t TR_OFF_A = TR_OFF_XT + sizeof(bf16) * IN * TR_LDT;
constexpr size_t TR_OFF_AT = TR_OFF_A + sizeof(bf16) * TRAIN_ROWS * TR_LDA;
constexpr size_t TR_OFF_B = TR_OFF_AT + sizeof(bf16) * HID * TR_LDT;
constexpr size_t TR_OFF_BT = TR_OFF_B + sizeof(bf16) * TRAIN_ROWS * TR_LDA;
constexpr size_t TR_OFF_D = TR_OFF_BT + sizeof(bf16) * HID * TR_LDT;
constexpr size_t TR_OFF_ROW = TR_OFF_D + sizeof(float) * TRAIN_ROWS * 2;
constexpr size_t TR_OFF_RED = TR_OFF_ROW + sizeof(int32_t) * TRAIN_ROWS;
constexpr size_t TR_OFF_W3 = TR_OFF_RED + sizeof(float) * 16;  // one loss partial per wavefront (at most 16)
constexpr size_t TRAIN_LDS = TR_OFF_W3 + sizeof(bf16) * 2 * HID;

struct TrainKArgs {
  TrainArgs a;
  const bf16 *E16, *W1_16, *W1T16, *W2_16, *W2T16, *W3_16;
  const float *b1, *b2, *b3;
  float* part;
  int64_t P;  // partial-gradient floats per chunk
  unsigned long long* dE;  // fixed point, units of DE_UNIT
  int64_t n_rows;  // embedding rows: a row id outside [0, n_rows) trains as a zero row
};

// partial-gradient offsets (parameter order after E)
constexpr int64_t PG_W1 = 0, PG_B1 = HID * IN, PG_W2 = PG_B1 + HID, PG_B2 = PG_W2 + HID * HID,
                  PG_W3 = PG_B2 + HID, PG_B3 = PG_W3 + 2 * HID;

__device__ __forceinline__ bf16x8 lds_frag(const bf16* base, int stride, int row, int col) {
  return *reinterpret_cast<const bf16x8*>(base + row * stride + col);
}

__device__ __forceinline__ bf16x8 global_frag(const bf16* base, int64_t stride, int row, int col) {
  return *reinterpret_cast<const bf16x8*>(base + (int64_t)row * stride + col);
}

// Store a 16 x 16 FP32 tile fragment (rows 4g..4g+3 of column r, offset by
// row0/col0) rounded to BF16: row-major into A (stride lda) and, when AT is
// given, transposed into AT (stride ldt), 4 consecutive rows in one 8-byte store.
__device__ __forceinline__ void store_frag_bf16(bf16* A, int lda, bf16* AT, int ldt, int row0, int col0, int g, int r,
                                                const float (&v)[4]) {
  bf16 h[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    h[i] = (bf16)v[i];
    A[(row0 + 4 * g + i) * lda + col0 + r] = h[i];
  }
  if (AT) {
    typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
    bf16x4 q = {h[0], h[1], h[2], h[3]};
    *reinterpret_cast<bf16x4*>(AT + (col0 + r) * ldt + row0 + 4 * g) = q;
  }
}

// Column sums over the rows of a wavefront's MB x NB tiles (values already
// rounded to BF16), reduced across the four row groups; lanes 0..15 return
// the sums of columns 16 nb + lane.
template <int MB, int NB>
__device__ __forceinline__ void column_sums(const float (&v)[MB][NB][4], float (&out)[NB]) {
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    float t = 0.0f;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int i = 0; i < 4; ++i) t += v[mb][nb][i];
    t += __shfl_xor(t, 16, 64);
    t += __shfl_xor(t, 32, 64);
    out[nb] = t;
  }
}

// Workgroup barrier for LDS data only: waits for this wavefront's LDS
// accesses, not its global loads and stores, so weight fragments loaded
// before a barrier stay in flight across it and partial-gradient stores
// drain behind later work.  (The kernel reads no global memory that other
// wavefronts of the workgroup write.)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

constexpr int TR_WAVES = 8;                 // wavefronts per workgroup, two per SIMD
constexpr int TR_THREADS = 64 * TR_WAVES;
constexpr int TR_COLS = HID / TR_WAVES;     // hidden units per wavefront
constexpr int TR_NB = TR_COLS / 16;         // 16-column tiles per wavefront
constexpr int TR_KS = HID / 32;             // K steps of a 256-long contraction
constexpr int TR_MB = TRAIN_ROWS / 16;      // 16-row tiles of a chunk
constexpr int TR_LPR = TR_THREADS / TRAIN_ROWS;  // lanes per row in the output layer
static_assert(TRAIN_ROWS % 32 == 0 && TRAIN_ROWS * 4 <= 256 && TR_LPR <= 64, "chunk shape");
static_assert(TR_WAVES <= 16 && HID % (16 * TR_WAVES) == 0 && TR_THREADS >= 256 + HID,
              "one loss partial per wavefront, whole column tiles, threads for the X and W3 staging");

__global__ __launch_bounds__(TR_THREADS) void train_chunk_kernel(TrainKArgs k) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  bf16* sX = reinterpret_cast<bf16*>(lds);
  bf16* sXT = reinterpret_cast<bf16*>(lds + TR_OFF_XT);
  bf16* sA = reinterpret_cast<bf16*>(lds + TR_OFF_A);
  bf16* sAT = reinterpret_cast<bf16*>(lds + TR_OFF_AT);
  bf16* sB = reinterpret_cast<bf16*>(lds + TR_OFF_B);
  bf16* sBT = reinterpret_cast<bf16*>(lds + TR_OFF_BT);
  float* sD = reinterpret_cast<float*>(lds + TR_OFF_D);
  int32_t* sRow = reinterpret_cast<int32_t*>(lds + TR_OFF_ROW);
  float* sRed = reinterpret_cast<float*>(lds + TR_OFF_RED);
  bf16* sW3 = reinterpret_cast<bf16*>(lds + TR_OFF_W3);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int c0 = TR_COLS * w;  // this wavefront's hidden units
  const int64_t base = (int64_t)blockIdx.x * TRAIN_ROWS;
  const int nrow = k.a.n - base < TRAIN_ROWS ? (int)(k.a.n - base) : TRAIN_ROWS;
  float* part = k.part + (int64_t)blockIdx.x * k.P;
  // Loads in the order their values are needed: a wavefront's loads complete
  // in order, so a value loaded after a prefetch would make its first use
  // wait for the prefetch.  Small operands and the gathered X first, then
  // the W1 and W2 fragments, then the LDS stores of X.
  float b1v[TR_NB], b2v[TR_NB];
#pragma unroll
  for (int nb = 0; nb < TR_NB; ++nb) {
    b1v[nb] = k.b1[c0 + 16 * nb + r];
    b2v[nb] = k.b2[c0 + 16 * nb + r];
  }
  const float b3a = k.b3[0], b3b = k.b3[1];
  const float yv = tid < nrow ? k.a.y[base + tid] : 0.0f;
  // X = [E[row], f]: threads 0 .. 4 TRAIN_ROWS - 1 take 8 columns of row t / 4;
  // threads 256 .. 256 + HID - 1 stage W3
  const int xrow = tid >> 2, xq = tid & 3;
  bf16x8 xv;
  int xid = -1;
  bf16 w3v[2];
  if (tid < 4 * TRAIN_ROWS) {
    xid = xrow < nrow ? k.a.rows[base + xrow] : -1;
    if (xid >= k.n_rows) xid = -1;
    if (xid >= 0) {
      if (xq < 2) {
        xv = *reinterpret_cast<const bf16x8*>(k.E16 + (int64_t)xid * EMB + 8 * xq);
      } else {
        const uint16_t* f = reinterpret_cast<const uint16_t*>(k.a.feat) + (base + xrow) * EMB + 8 * (xq - 2);
#pragma unroll
        for (int j = 0; j < 8; ++j) xv[j] = __builtin_bit_cast(bf16, f[j]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) xv[j] = (bf16)0.0f;
    }
  } else if (tid >= 256 && tid < 256 + HID) {  // two W3 values per thread
    w3v[0] = k.W3_16[2 * (tid - 256)];
    w3v[1] = k.W3_16[2 * (tid - 256) + 1];
  }
  bf16x8 bw1[TR_NB];        // W1 fragments of z1
  bf16x8 bw[TR_KS][TR_NB];  // W2 fragments of z2, then W2T of dh1
#pragma unroll
  for (int nb = 0; nb < TR_NB; ++nb) bw1[nb] = global_frag(k.W1_16, IN, c0 + 16 * nb + r, 8 * g);
#pragma unroll
  for (int ks = 0; ks < TR_KS; ++ks)
#pragma unroll
    for (int nb = 0; nb < TR_NB; ++nb) bw[ks][nb] = global_frag(k.W2_16, HID, c0 + 16 * nb + r, 32 * ks + 8 * g);
  float* sY = sD;  // targets of the chunk's rows, until dout replaces them
  if (tid < TRAIN_ROWS) sY[tid] = yv;
  if (tid < 4 * TRAIN_ROWS) {
    if (xq == 0) sRow[xrow] = xid;
    *reinterpret_cast<bf16x8*>(sX + xrow * TR_LDX + 8 * xq) = xv;
#pragma unroll
    for (int j = 0; j < 8; ++j) sXT[(8 * xq + j) * TR_LDT + xrow] = xv[j];
  } else if (tid >= 256 && tid < 256 + HID) {
    sW3[2 * (tid - 256)] = w3v[0];
    sW3[2 * (tid - 256) + 1] = w3v[1];
  }
  lds_barrier();

  // ---- z1, h1; GELU'(z1) kept in registers ----
  float gp1[TR_MB][TR_NB][4];
  {
    floatx4 c[TR_MB][TR_NB];
#pragma unroll
    for (int mb = 0; mb < TR_MB; ++mb) {
      const bf16x8 ax = lds_frag(sX, TR_LDX, 16 * mb + r, 8 * g);
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) c[mb][nb] = mfma16x16x32(ax, bw1[nb], floatx4{0.f, 0.f, 0.f, 0.f});
    }
#pragma unroll
    for (int nb = 0; nb < TR_NB; ++nb) {
      const float bias = b1v[nb];
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb) {
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) gelu_and_grad(c[mb][nb][i] + bias, &h[i], &gp1[mb][nb][i]);
        store_frag_bf16(sA, TR_LDA, sAT, TR_LDT, 16 * mb, c0 + 16 * nb, g, r, h);
      }
    }
  }
  lds_barrier();

  // ---- z2, h2; GELU'(z2) kept in registers ----
  float gp2[TR_MB][TR_NB][4];
  {
    floatx4 acc[TR_MB][TR_NB];
#pragma unroll
    for (int mb = 0; mb < TR_MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < TR_KS; ++ks) {
      bf16x8 ah[TR_MB];
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb) ah[mb] = lds_frag(sA, TR_LDA, 16 * mb + r, 32 * ks + 8 * g);
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < TR_NB; ++nb) acc[mb][nb] = mfma16x16x32(ah[mb], bw[ks][nb], acc[mb][nb]);
    }
    // the transposed W2 fragments of dh1 load while the output layer runs
#pragma unroll
    for (int ks = 0; ks < TR_KS; ++ks)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) bw[ks][nb] = global_frag(k.W2T16, HID, c0 + 16 * nb + r, 32 * ks + 8 * g);
#pragma unroll
    for (int nb = 0; nb < TR_NB; ++nb) {
      const float bias = b2v[nb];
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb) {
        float h[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) gelu_and_grad(acc[mb][nb][i] + bias, &h[i], &gp2[mb][nb][i]);
        store_frag_bf16(sB, TR_LDA, nullptr, 0, 16 * mb, c0 + 16 * nb, g, r, h);
      }
    }
  }
  lds_barrier();

  // ---- (mu, q), loss, dout: TR_LPR lanes per row ----
  {
    constexpr int KPL = HID / TR_LPR;
    const int row = tid / TR_LPR, q = tid % TR_LPR;
    float s0 = 0.0f, s1 = 0.0f;
    const bf16* h2 = sB + row * TR_LDA + KPL * q;
    const bf16* w0 = sW3 + KPL * q;
    const bf16* w1 = sW3 + HID + KPL * q;
#pragma unroll 8
    for (int j = 0; j < KPL; ++j) {
      const float h = (float)h2[j];
      s0 = fmaf(h, (float)w0[j], s0);
      s1 = fmaf(h, (float)w1[j], s1);
    }
#pragma unroll
    for (int o = 1; o < TR_LPR; o <<= 1) {
      s0 += __shfl_xor(s0, o, 64);
      s1 += __shfl_xor(s1, o, 64);
    }
    float loss = 0.0f;
    const float t = sY[row];
    lds_barrier();  // every target is read before dout overwrites them
    if (q == 0) {
      float d0 = 0.0f, d1 = 0.0f;
      if (row < nrow) {
        const float mu = s0 + b3a, qv = s1 + b3b;
        const bool below = t < qv;
        d0 = (float)(bf16)(2.0f * (mu - t) * k.a.inv_B);
        d1 = (float)(bf16)(((below ? 1.0f : 0.0f) - TAU) * k.a.inv_B);
        const float u = t - qv;
        loss = (mu - t) * (mu - t) + u * (TAU - (below ? 1.0f : 0.0f));
      }
      sD[2 * row] = d0;
      sD[2 * row + 1] = d1;
    }
    if (k.a.loss_sum) {
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) loss += __shfl_xor(loss, o, 64);
      if (lane == 0) sRed[w] = loss;
    }
  }
  lds_barrier();
  if (k.a.loss_sum && tid == 0) {
    float t = 0.0f;
    for (int i = 0; i < TR_WAVES; ++i) t += sRed[i];
    atomicAdd(k.a.loss_sum, t);
  }

  // ---- dW3, db3 (a lane per column of h2) ----
  if (tid < HID) {
    float a0 = 0.0f, a1 = 0.0f;
#pragma unroll 8
    for (int row = 0; row < TRAIN_ROWS; ++row) {
      const float h = (float)sB[row * TR_LDA + tid];
      a0 = fmaf(sD[2 * row], h, a0);
      a1 = fmaf(sD[2 * row + 1], h, a1);
    }
    part[PG_W3 + tid] = a0;
    part[PG_W3 + HID + tid] = a1;
    if (tid < 2) {
      float t = 0.0f;
      for (int row = 0; row < TRAIN_ROWS; ++row) t += sD[2 * row + tid];
      part[PG_B3 + tid] = t;
    }
  }
  lds_barrier();  // h2 is read above; dz2 overwrites it below

  // ---- dz2 = (dout W3) GELU'(z2), db2 ----
  {
    float w3a[TR_NB], w3b[TR_NB];
#pragma unroll
    for (int nb = 0; nb < TR_NB; ++nb) {
      w3a[nb] = (float)sW3[c0 + 16 * nb + r];
      w3b[nb] = (float)sW3[HID + c0 + 16 * nb + r];
    }
#pragma unroll
    for (int mb = 0; mb < TR_MB; ++mb) {
      float d0[4], d1[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        d0[i] = sD[2 * (16 * mb + 4 * g + i)];
        d1[i] = sD[2 * (16 * mb + 4 * g + i) + 1];
      }
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) {
        float v[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float dh = fmaf(d1[i], w3b[nb], d0[i] * w3a[nb]);
          v[i] = (float)(bf16)(dh * gp2[mb][nb][i]);
          gp2[mb][nb][i] = v[i];  // GELU'(z2) is dead from here: keep dz2
        }
        store_frag_bf16(sB, TR_LDA, sBT, TR_LDT, 16 * mb, c0 + 16 * nb, g, r, v);
      }
    }
    float cs[TR_NB];
    column_sums<TR_MB, TR_NB>(gp2, cs);
    if (g == 0)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) part[PG_B2 + c0 + 16 * nb + r] = cs[nb];
  }
  lds_barrier();

  // ---- dz1 = (dz2 W2) GELU'(z1), db1; dz1 goes to the row-major buffer of h1 ----
  {
    floatx4 acc[TR_MB][TR_NB];
#pragma unroll
    for (int mb = 0; mb < TR_MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < TR_KS; ++ks) {
      bf16x8 ad[TR_MB];
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb) ad[mb] = lds_frag(sB, TR_LDA, 16 * mb + r, 32 * ks + 8 * g);
#pragma unroll
      for (int mb = 0; mb < TR_MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < TR_NB; ++nb) acc[mb][nb] = mfma16x16x32(ad[mb], bw[ks][nb], acc[mb][nb]);
    }
#pragma unroll
    for (int mb = 0; mb < TR_MB; ++mb)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) gp1[mb][nb][i] = (float)(bf16)(acc[mb][nb][i] * gp1[mb][nb][i]);
        store_frag_bf16(sA, TR_LDA, nullptr, 0, 16 * mb, c0 + 16 * nb, g, r, gp1[mb][nb]);
      }
    float cs[TR_NB];
    column_sums<TR_MB, TR_NB>(gp1, cs);
    if (g == 0)
#pragma unroll
      for (int nb = 0; nb < TR_NB; ++nb) part[PG_B1 + c0 + 16 * nb + r] = cs[nb];
  }
  bf16x8 bt[TR_KS];  // W1T fragments of the embedding gradient
  if (w < TRAIN_ROWS / 16)
#pragma unroll
    for (int ks = 0; ks < TR_KS; ++ks) bt[ks] = global_frag(k.W1T16, HID, r, 32 * ks + 8 * g);
  lds_barrier();

  // ---- dW1 = dz1^T X: wavefront w takes outputs c0 .. c0 + TR_COLS - 1 (dz1
  // read down its columns: 8 two-byte LDS reads per fragment) ----
  {
    floatx4 acc[TR_NB][2];
#pragma unroll
    for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < TRAIN_ROWS / 32; ++ks) {
      bf16x8 a[TR_NB], b[2];
#pragma unroll
      for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
        for (int j = 0; j < 8; ++j) a[mb][j] = sA[(32 * ks + 8 * g + j) * TR_LDA + c0 + 16 * mb + r];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) b[nb] = lds_frag(sXT, TR_LDT, 16 * nb + r, 32 * ks + 8 * g);
#pragma unroll
      for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) acc[mb][nb] = mfma16x16x32(a[mb], b[nb], acc[mb][nb]);
    }
#pragma unroll
    for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 2; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          part[PG_W1 + (c0 + 16 * mb + 4 * g + i) * IN + 16 * nb + r] = acc[mb][nb][i];
  }

  // ---- embedding gradient: wavefronts 0..3 take rows 16w..16w+15 of dz1 W1[:, :16] ----
  if (w < TRAIN_ROWS / 16) {
    floatx4 acc = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < TR_KS; ++ks) acc = mfma16x16x32(lds_frag(sA, TR_LDA, 16 * w + r, 32 * ks + 8 * g), bt[ks], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = 16 * w + 4 * g + i;
      if (row < nrow && sRow[row] >= 0) {
        const float t = fminf(fmaxf(acc[i], -DE_CLAMP), DE_CLAMP) * DE_SCALE;
        atomicAdd(k.dE + (int64_t)sRow[row] * EMB + r, (unsigned long long)__float2ll_rn(t));
      }
    }
  }

  // ---- dW2 = dz2^T h1, last: its 256 KB of partial stores then hold up no
  // later load.  Wavefront w takes outputs c0 .. c0 + TR_COLS - 1, four
  // passes of 64 inputs ----
#pragma unroll 1
  for (int pass = 0; pass < 4; ++pass) {
    floatx4 acc[TR_NB][4];
#pragma unroll
    for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < TRAIN_ROWS / 32; ++ks) {
      bf16x8 a[TR_NB], b[4];
#pragma unroll
      for (int mb = 0; mb < TR_NB; ++mb) a[mb] = lds_frag(sBT, TR_LDT, c0 + 16 * mb + r, 32 * ks + 8 * g);
#pragma unroll
      for (int nb = 0; nb < 4; ++nb) b[nb] = lds_frag(sAT, TR_LDT, 64 * pass + 16 * nb + r, 32 * ks + 8 * g);
#pragma unroll
      for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) acc[mb][nb] = mfma16x16x32(a[mb], b[nb], acc[mb][nb]);
    }
#pragma unroll
    for (int mb = 0; mb < TR_NB; ++mb)
#pragma unroll
      for (int nb = 0; nb < 4; ++nb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          part[PG_W2 + (int64_t)(c0 + 16 * mb + 4 * g + i) * HID + 64 * pass + 16 * nb + r] = acc[mb][nb][i];
  }
}

// Sum of the chunks' partials (chunk order) or the embedding accumulator;
// then AdamW as adamw_kernel and the new value's shadows.
__global__ __launch_bounds__(256) void train_reduce_kernel(int64_t n, int64_t nE, const float* part, int n_chunks,
                                                           unsigned long long* dE, float* grad, int first, int update, float* p,
                                                           float* m, float* v, float lr, float wd, float c1,
                                                           float c2, int64_t d0, int64_t d1a, int64_t d1b,
                                                           int64_t d2a, int64_t d2b, Shadows sh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi;
  if (i < nE) {
    gi = (float)((double)(long long)dE[i] * DE_UNIT);
    dE[i] = 0ull;
  } else {
    // 32 loads in flight, added in chunk order
    const int64_t P = n - nE;
    const float* q = part + (i - nE);
    gi = 0.0f;
    int c = 0;
    for (; c + 32 <= n_chunks; c += 32) {
      float t[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) t[j] = q[(int64_t)(c + j) * P];
#pragma unroll
      for (int j = 0; j < 32; ++j) gi += t[j];
    }
    for (; c < n_chunks; ++c) gi += q[(int64_t)c * P];
  }
  if (!first) gi += grad[i];
  grad[i] = gi;
  if (!update) return;
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  float wv = p[i];
  const bool decay = i < d0 || (i >= d1a && i < d1b) || (i >= d2a && i < d2b);
  if (decay) wv *= 1.0f - lr * wd;
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  wv = wv - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = wv;
  write_shadow(sh, i, wv);
}

// ---------------------------------------------------------------------------
// Fused inference + Eq. 1 scan (see file comment).
// ---------------------------------------------------------------------------
constexpr int LEARNED_WAVES = 4;  // wavefronts per workgroup (one per SIMD: 512 registers each)
// LDS row strides of the staged weight matrices, padded by 16 bytes: the 16
// lanes that read one A fragment take 16 consecutive rows at one column, and
// unpadded 512- and 64-byte strides put those rows in the same banks.
constexpr int W2_LD = HID + 8, W1_LD = IN + 8;
constexpr size_t LEARNED_LDS = sizeof(bf16) * (HID * W2_LD + HID * W1_LD + 3 * HID) + sizeof(float) * (HID * 2);
static_assert(LEARNED_LDS <= 160 * 1024, "fused inference LDS");

__device__ __forceinline__ int64_t remaining(int64_t r0, int64_t queue) {
  int64_t r = r0 - queue;
  r = r < 0 ? 0 : r;
  return r > 0x7FFFFFFFll ? 0x7FFFFFFFll : r;
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = (int64_t)((double)a / (double)b);
  const int64_t rem = a - q * b;
  if (rem < 0) q -= 1; else if (rem >= b) q += 1;
  return q;
}

// Weights of the fused inference staged in LDS by a whole workgroup.
struct LearnedStage {
  const bf16* sW2;   // [256][W2_LD] K-permuted
  const bf16* sW1;   // [256][W1_LD]
  const float* sB1;  // [256]
  const float* sB2;  // [256]
  const bf16* sW3;   // [3][256] K-permuted: W3's two rows, then zeros
  float b3_0, b3_1;
};

// Every thread of the workgroup copies its share; the caller synchronizes.
__device__ __forceinline__ LearnedStage learned_stage(const LearnedArgs& s, unsigned char* lds) {
  bf16* sW2 = reinterpret_cast<bf16*>(lds);
  bf16* sW1 = sW2 + HID * W2_LD;
  float* sB1 = reinterpret_cast<float*>(sW1 + HID * W1_LD);
  float* sB2 = sB1 + HID;
  bf16* sW3 = reinterpret_cast<bf16*>(sB2 + HID);
  const int tid = threadIdx.x;
  const bf16* W3_16 = reinterpret_cast<const bf16*>(s.W3_16);
  const uint4* src = reinterpret_cast<const uint4*>(s.W2p16);  // 16 bytes = 8 BF16
  uint4* dst = reinterpret_cast<uint4*>(sW2);
  for (int i = tid; i < HID * HID / 8; i += blockDim.x) dst[(i / (HID / 8)) * (W2_LD / 8) + i % (HID / 8)] = src[i];
  const uint4* src1 = reinterpret_cast<const uint4*>(s.W1_16);
  uint4* dst1 = reinterpret_cast<uint4*>(sW1);
  for (int i = tid; i < HID * IN / 8; i += blockDim.x) dst1[(i / (IN / 8)) * (W1_LD / 8) + i % (IN / 8)] = src1[i];
  for (int i = tid; i < HID; i += blockDim.x) {
    sB1[i] = s.b1[i];
    sB2[i] = s.b2[i];
    sW3[w2p_column(i)] = W3_16[i];
    sW3[HID + w2p_column(i)] = W3_16[HID + i];
    sW3[2 * HID + i] = (bf16)0.0f;
  }
  return LearnedStage{sW2, sW1, sB1, sB2, sW3, s.b3[0], s.b3[1]};
}

// One valid invocation (op v, elapsed e, SLO sl, features feat_i) evaluated
// by a wavefront over row blocks nb0 .. nb0 + NB - 1 (16 rows each) of every
// 64-row chunk of its op's configurations: targets, each row's predicted p95
// latency (profile fallback), and the wavefront's minima of Eq. 1's keys:
// *best the cheapest feasible key, *fast the fastest (L << 16 | k), in every
// lane.  lat_row, when given, receives each row's latency.
template <int NHW, int NB>
__device__ __forceinline__ void learned_scan_rows(const DevTables& t, int mode, const int64_t* queue,
                                                  const LearnedArgs& s, const LearnedStage& st, int v, int e,
                                                  int sl, const bf16* feat_i, int32_t* lat_row, int nb0,
                                                  uint32_t* best_out, uint64_t* fast_out) {
  const bf16* sW2 = st.sW2;
  const bf16* sW1 = st.sW1;
  const float* sB1 = st.sB1;
  const float* sB2 = st.sB2;
  const float b3_0 = st.b3_0, b3_1 = st.b3_1;
  const bf16* E16 = reinterpret_cast<const bf16*>(s.E16);
  const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
  // layer 3 as a product whose 16 A rows repeat (W3 row 0, W3 row 1, 0, 0):
  // every lane group then holds mu and q of its row in accumulator slots 0, 1
  const bf16* w3row = st.sW3 + (int64_t)((lane & 3) < 2 ? (lane & 3) : 2) * HID;
  const int64_t r0 = (int64_t)sl - e;
  const int64_t ref = t.ref[v];
  const int64_t W = t.W[(int64_t)mode * t.n_ops + v];
  int32_t tgt[NHW];
#pragma unroll
  for (int h = 0; h < NHW; ++h) {
    const int64_t R = remaining(r0, queue ? queue[h] : 0);
    tgt[h] = R == 0 ? 0 : (int32_t)floor_div(ref * R, W);
  }
  const int a0 = t.cfg_off[v], n_c = t.cfg_off[v + 1] - a0;
  // feature half of the layer-1 input fragment (lane groups 2 and 3)
  bf16x8 ffrag;
  if (g >= 2) ffrag = *reinterpret_cast<const bf16x8*>(feat_i + 8 * (g - 2));
  uint32_t best = KEY_NONE;
  uint64_t fast = ~0ull;
  for (int c0 = 0; c0 < n_c; c0 += 64) {
    // ---- layer 1: z1^T[unit][row] = W1 . x^T, 16 unit blocks x 4 row blocks
    bf16x8 xfrag[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = c0 + (nb0 + nb) * 16 + r;
      const int row = a0 + (k < n_c ? k : 0);
      xfrag[nb] = g < 2 ? *reinterpret_cast<const bf16x8*>(E16 + (int64_t)row * EMB + 8 * g) : ffrag;
    }
    // hf[kb][nb] is the layer-2 input fragment of row 16nb + r for K block
    // kb: units 32kb + 4g + q (slots 0..3) and 32kb + 16 + 4g + q (slots
    // 4..7), exactly the layer-1 outputs of unit blocks 2kb and 2kb + 1.
    bf16x8 hf[8][NB];
    // an offset the compiler cannot see through keeps the layer-1 weight
    // reads inside the chunk loop: hoisted, their 128 registers stay live
    // through layers 2 and 3 and serialise the GELU chains there
    int wofs = 0;
    asm volatile("" : "+v"(wofs));
#pragma unroll
    for (int mb = 0; mb < 16; ++mb) {
      const bf16x8 w1 = *reinterpret_cast<const bf16x8*>(sW1 + wofs + (16 * mb + r) * W1_LD + 8 * g);
      // the accumulator starts at the bias of this lane's four units
      const floatx4 b1 = *reinterpret_cast<const floatx4*>(sB1 + wofs + 16 * mb + 4 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const floatx4 z = mfma16x16x32(w1, xfrag[nb], b1);
#pragma unroll
        for (int q = 0; q < 4; ++q) hf[mb >> 1][nb][4 * (mb & 1) + q] = (bf16)gelu(z[q]);
      }
    }
    // ---- layers 2 and 3: unit blocks 2kb and 2kb + 1 of layer 2 make the
    // layer-3 input fragment of K block kb (the layer-1 -> 2 arrangement)
    floatx4 o3[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) o3[nb] = floatx4{b3_0, b3_1, 0.0f, 0.0f};
#pragma unroll 1
    for (int kb3 = 0; kb3 < 8; ++kb3) {
      bf16x8 h2f[NB];
#pragma unroll
      for (int hb = 0; hb < 2; ++hb) {
        const int mb2 = 2 * kb3 + hb;
        floatx4 acc[NB];
        const floatx4 b2 = *reinterpret_cast<const floatx4*>(sB2 + 16 * mb2 + 4 * g);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[nb] = b2;
#pragma unroll
        for (int kb = 0; kb < 8; ++kb) {
          const bf16x8 w2 = *reinterpret_cast<const bf16x8*>(sW2 + (16 * mb2 + r) * W2_LD + 32 * kb + 8 * g);
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) acc[nb] = mfma16x16x32(w2, hf[kb][nb], acc[nb]);
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
#pragma unroll
          for (int q = 0; q < 4; ++q) h2f[nb][4 * hb + q] = (bf16)gelu(acc[nb][q]);
      }
      const bf16x8 w3 = *reinterpret_cast<const bf16x8*>(w3row + 32 * kb3 + 8 * g);
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) o3[nb] = mfma16x16x32(w3, h2f[nb], o3[nb]);
    }
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int k = c0 + (nb0 + nb) * 16 + r;
      if (k >= n_c) continue;
      const int x = a0 + k;
      const float mu = o3[nb][0], q95 = o3[nb][1];
      const float spread = q95 - mu;
      int32_t L;
      // predicted p95 when the spread is finite and in [0, spread_max], else the profile
      if (spread >= 0.0f && spread <= s.spread_max && mu == mu && q95 == q95) {
        const float ex = ceilf(expf(q95));
        L = ex >= 2147483647.0f ? 0x7FFFFFFF : (int32_t)ex;
      } else {
        L = t.cfg_lat[x];
      }
      if (lat_row && g == 0) lat_row[k] = L;
      const int h = t.cfg_hw[x];
      int32_t tg = tgt[0];
#pragma unroll
      for (int hh = 1; hh < NHW; ++hh) tg = h == hh ? tgt[hh] : tg;
      const uint32_t key = t.cfg_key[x];
      if (L < tg) best = key < best ? key : best;
      const uint64_t fk = ((uint64_t)(uint32_t)L << 16) | (uint64_t)k;
      fast = fk < fast ? fk : fast;
    }
  }
  // minimum over the wavefront (every lane group holds the same rows)
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t ob = __shfl_xor(best, d, 64);
    best = ob < best ? ob : best;
    const uint64_t of = __shfl_xor(fast, d, 64);
    fast = of < fast ? of : fast;
  }
  *best_out = best;
  *fast_out = fast;
}

// The choice and flag from the minima: the cheapest feasible configuration,
// else the fastest.
__device__ __forceinline__ void learned_choice(uint32_t best, uint64_t fast, int32_t* cfg_out, uint8_t* flag_out) {
  *flag_out = best != KEY_NONE ? 1 : 0;
  *cfg_out = best != KEY_NONE ? (int32_t)(best & 0xFFFFu) : (int32_t)(fast & 0xFFFFu);
}


// Batch of invocations: a workgroup of twelve wavefronts (three per SIMD, at
// most 168 registers each) takes six invocations at a time; the two
// wavefronts of an invocation each evaluate two of the four 16-row blocks of
// its 64-row chunks (each A fragment read from LDS feeds two products), so
// that one wavefront's GELU work overlaps another's matrix products on their
// SIMD, and their minima meet in LDS.  Measured on C4 (1 M invocations x 64
// configurations): 13.5 ms; one block per wavefront and sixteen wavefronts
// 14.4 ms, four blocks and eight wavefronts 13.9 ms.
constexpr int LEARNED_BATCH_WAVES = 12;
constexpr int LEARNED_WAVE_BLOCKS = 2;
constexpr int LEARNED_WPI = 4 / LEARNED_WAVE_BLOCKS;  // wavefronts per invocation
static_assert(4 % LEARNED_WAVE_BLOCKS == 0 && LEARNED_BATCH_WAVES % LEARNED_WPI == 0 && LEARNED_BATCH_WAVES <= 16,
              "batch workgroup shape");
template <int NHW>
__global__ __launch_bounds__(64 * LEARNED_BATCH_WAVES) void decide_learned_kernel(DevTables t, Batch b,
                                                                                  LearnedArgs s) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const LearnedStage st = learned_stage(s, lds);
  __shared__ uint32_t sBest[LEARNED_BATCH_WAVES];
  __shared__ unsigned long long sFast[LEARNED_BATCH_WAVES];
  __syncthreads();
  const bf16* feat = reinterpret_cast<const bf16*>(s.feat);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, part = w % LEARNED_WPI;
  constexpr int PER = LEARNED_BATCH_WAVES / LEARNED_WPI;  // invocations per workgroup at a time
  for (int64_t i0 = (int64_t)blockIdx.x * PER; i0 < b.n; i0 += (int64_t)gridDim.x * PER) {
    const int64_t i = i0 + w / LEARNED_WPI;
    bool valid = false;
    uint32_t best = KEY_NONE;
    uint64_t fast = ~0ull;
    if (i < b.n) {
      const int v = b.op[i], e = b.elapsed[i], sl = b.slo[i];
      valid = (unsigned)v < (unsigned)t.n_ops && (e | sl) >= 0;
      if (valid) {
        learned_scan_rows<NHW, LEARNED_WAVE_BLOCKS>(t, b.mode, b.queue, s, st, v, e, sl, feat + i * EMB,
                                                    s.lat_out ? s.lat_out + i * s.lat_stride : nullptr,
                                                    LEARNED_WAVE_BLOCKS * part, &best, &fast);
      } else if (part == 0 && lane == 0) {
        b.cfg[i] = -1;
        if (b.flag) b.flag[i] = 0;
        atomicOr(t.err, 1u);
      }
    }
    if (lane == 0) {
      sBest[w] = best;
      sFast[w] = fast;
    }
    __syncthreads();
    if (valid && part == 0 && lane == 0) {
#pragma unroll
      for (int o = 1; o < LEARNED_WPI; ++o) {
        const uint32_t ob = sBest[w + o];
        const unsigned long long of = sFast[w + o];
        best = ob < best ? ob : best;
        fast = of < fast ? of : fast;
      }
      int32_t cfg;
      uint8_t f;
      learned_choice(best, fast, &cfg, &f);
      b.cfg[i] = cfg;
      if (b.flag) b.flag[i] = f;
    }
    __syncthreads();  // sBest and sFast are rewritten next time round
  }
}

// Persistent learned decisions for the serving ring: the weights are staged
// once per workgroup, then the workgroup takes one published request at a
// time (wavefront 0 claims it), its four wavefronts each evaluate one
// 16-row block of the op's configurations, and the minima meet in LDS, so a
// request's latency is a quarter of one wavefront's work (exit rules as
// serve_plain_kernel, decided by wavefront 0).
template <int NHW>
__global__ __launch_bounds__(256) void serve_learned_kernel(DevTables t, ServeRing r, LearnedArgs s) {
  extern __shared__ __attribute__((aligned(16))) unsigned char lds[];
  const LearnedStage st = learned_stage(s, lds);
  __shared__ long long sClaim[2];  // first claimed sequence, claimed count (-1: exit)
  __shared__ uint32_t sBest[LEARNED_WAVES];
  __shared__ unsigned long long sFast[LEARNED_WAVES];
  __syncthreads();
  const bf16* feat = reinterpret_cast<const bf16*>(r.feat);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int answered = 0;
  int* clock = blockIdx.x == 0 ? &answered : nullptr;
  serve_enter(r, lane);  // every wavefront counts itself in; wavefront 0 claims for the workgroup
  const unsigned long long start = (unsigned long long)wall_clock64();
  unsigned long long last = start;
  for (;;) {
    // wavefront 0 claims one request for the workgroup and tells the others
    if (w == 0) {
      const unsigned long long now = (unsigned long long)wall_clock64();
      long long first = 0, count = -1;
      if (now - start <= r.life_ticks) {
        for (;;) {
          const unsigned long long t_now = (unsigned long long)wall_clock64();
          const ServeClaim c = serve_claim(r, lane, 1, clock);
          if (c.stop) break;
          if (c.count > 0) {
            first = c.first;
            count = c.count;
            last = t_now;
            break;
          }
          if (serve_idle(r, t_now, last) || t_now - start > r.life_ticks) break;
          __builtin_amdgcn_s_sleep(8);
        }
      }
      if (lane == 0) {
        sClaim[0] = first;
        sClaim[1] = count;
      }
    }
    __syncthreads();
    const long long seq = sClaim[0], count = sClaim[1];
    if (count < 0) break;
    const long long slot = seq % r.cap;
    const int4 q = r.req[slot];
    const bool valid = (unsigned)q.x < (unsigned)t.n_ops && (q.y | q.z) >= 0;
    // each wavefront takes one 16-row block of the op's 64-row chunks
    uint32_t best = KEY_NONE;
    uint64_t fast = ~0ull;
    if (valid)
      learned_scan_rows<NHW, 1>(t, r.mode, nullptr, s, st, q.x, q.y, q.z, feat + slot * EMB, nullptr, w, &best,
                                &fast);
    if (lane == 0) {
      sBest[w] = best;
      sFast[w] = fast;
    }
    __syncthreads();
    if (w == 0) {
      int32_t cfg = -1;
      uint8_t f = 0;
      if (!valid) {
        if (lane == 0) atomicOr(t.err, 1u);
      } else {
#pragma unroll
        for (int u = 1; u < LEARNED_WAVES; ++u) {
          best = sBest[u] < best ? sBest[u] : best;
          fast = sFast[u] < fast ? sFast[u] : fast;
        }
        learned_choice(best, fast, &cfg, &f);
      }
      if (lane == 0) serve_write(r, seq, slot, cfg, f);
    }
  }
  serve_leave(r, lane);
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_gemm_bf16(int M, int N, int K, const void* a, int64_t sam, int64_t sak, const void* bm,
                            int64_t sbk, int64_t sbn, float* c, int64_t ldc, const float* bias, bool accumulate,
                            hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3(grid1(N, 64), grid1(M, 64)), dim3(256), 0, s, M, N, K, (const bf16*)a,
                     sam, sak, (const bf16*)bm, sbk, sbn, c, ldc, bias, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_surrogate_forward(const SurrogateBufs& w, int64_t B, const int32_t* rows, const void* feat,
                                    hipStream_t s) {
  hipLaunchKernelGGL(gather_x_kernel, dim3(grid1(B * IN, 256)), dim3(256), 0, s, B, rows, (const bf16*)feat,
                     (const bf16*)w.E16, (bf16*)w.X16);
  hipError_t e;
  if ((e = launch_gemm_bf16((int)B, HID, IN, w.X16, IN, 1, w.W1_16, 1, IN, w.z1, HID, w.b1, false, s))) return e;
  hipLaunchKernelGGL(gelu_round_kernel, dim3(grid1(B * HID, 256)), dim3(256), 0, s, B * HID, w.z1, (bf16*)w.h1);
  if ((e = launch_gemm_bf16((int)B, HID, HID, w.h1, HID, 1, w.W2_16, 1, HID, w.z2, HID, w.b2, false, s))) return e;
  hipLaunchKernelGGL(gelu_round_kernel, dim3(grid1(B * HID, 256)), dim3(256), 0, s, B * HID, w.z2, (bf16*)w.h2);
  return launch_gemm_bf16((int)B, 2, HID, w.h2, HID, 1, w.W3_16, 1, HID, w.out, 2, w.b3, false, s);
}

namespace {
Shadows shadows_of(const SurrogateBufs& w) {
  Shadows sh;
  sh.E16 = (bf16*)w.E16;
  sh.W1_16 = (bf16*)w.W1_16;
  sh.W1T16 = (bf16*)w.W1T16;
  sh.W2_16 = (bf16*)w.W2_16;
  sh.W2T16 = (bf16*)w.W2T16;
  sh.W2p16 = (bf16*)w.W2p16;
  sh.W3_16 = (bf16*)w.W3_16;
  sh.nE = w.nE;
  return sh;
}
}  // namespace

hipError_t launch_shadows(const SurrogateBufs& w, hipStream_t s) {
  hipLaunchKernelGGL(shadows_kernel, dim3(grid1(w.n_params, 256)), dim3(256), 0, s, w.master, w.n_params,
                     shadows_of(w));
  return hipGetLastError();
}

hipError_t launch_train_chunks(const SurrogateBufs& w, const TrainArgs& a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int64_t chunks = (a.n + TRAIN_ROWS - 1) / TRAIN_ROWS;
  if (chunks > TRAIN_MAX_CHUNKS) return hipErrorInvalidValue;
  TrainKArgs k;
  k.a = a;
  k.E16 = (const bf16*)w.E16;
  k.W1_16 = (const bf16*)w.W1_16;
  k.W1T16 = (const bf16*)w.W1T16;
  k.W2_16 = (const bf16*)w.W2_16;
  k.W2T16 = (const bf16*)w.W2T16;
  k.W3_16 = (const bf16*)w.W3_16;
  k.b1 = w.b1;
  k.b2 = w.b2;
  k.b3 = w.b3;
  k.part = w.part;
  k.P = w.n_params - w.nE;
  k.dE = w.dE;
  k.n_rows = w.nE / EMB;
  hipError_t e = hipFuncSetAttribute((const void*)train_chunk_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)TRAIN_LDS);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(train_chunk_kernel, dim3((unsigned)chunks), dim3(TR_THREADS), TRAIN_LDS, s, k);
  return hipGetLastError();
}

hipError_t launch_train_reduce(const SurrogateBufs& w, int n_chunks, bool first, bool update, float lr, float wd,
                               int64_t step, hipStream_t s) {
  const float beta1 = 0.9f, beta2 = 0.999f;
  const float c1 = update ? 1.0f - powf(beta1, (float)step) : 1.0f;
  const float c2 = update ? 1.0f - powf(beta2, (float)step) : 1.0f;
  hipLaunchKernelGGL(train_reduce_kernel, dim3(grid1(w.n_params, 256)), dim3(256), 0, s, w.n_params, w.nE, w.part,
                     n_chunks, w.dE, w.grad, first ? 1 : 0, update ? 1 : 0, w.master, w.adam_m, w.adam_v, lr, wd, c1,
                     c2, w.ob1, w.oW2, w.ob2, w.oW3, w.ob3, shadows_of(w));
  return hipGetLastError();
}

hipError_t launch_decide_learned(const DevTables& t, const Batch& b, const LearnedArgs& a, hipStream_t s) {
  if (b.n == 0) return hipSuccess;
  const int blocks = 256;  // persistent: one workgroup per CU (LDS-bound), grid-stride over invocations
  constexpr int per = LEARNED_BATCH_WAVES / LEARNED_WPI;
  const unsigned grid = (unsigned)(b.n < (int64_t)blocks * per ? (b.n + per - 1) / per : blocks);
#define LLAMA_LEARNED_CASE(N)                                                                          \
  case N:                                                                                              \
    {                                                                                                  \
      hipError_t e = hipFuncSetAttribute((const void*)decide_learned_kernel<N>,                        \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)LEARNED_LDS); \
      if (e != hipSuccess) return e;                                                                   \
    }                                                                                                  \
    hipLaunchKernelGGL(decide_learned_kernel<N>, dim3(grid), dim3(64 * LEARNED_BATCH_WAVES), LEARNED_LDS, s, t, b, a); \
    break;
  switch (t.n_hw) {
    LLAMA_LEARNED_CASE(1)
    LLAMA_LEARNED_CASE(2)
    LLAMA_LEARNED_CASE(3)
    LLAMA_LEARNED_CASE(4)
    LLAMA_LEARNED_CASE(5)
    LLAMA_LEARNED_CASE(6)
    LLAMA_LEARNED_CASE(7)
    LLAMA_LEARNED_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef LLAMA_LEARNED_CASE
  return hipGetLastError();
}

hipError_t prepare_serve_learned(const DevTables& t) {
  switch (t.n_hw) {
#define LLAMA_SERVE_PREP_CASE(N)                                                                      \
  case N:                                                                                             \
    return hipFuncSetAttribute((const void*)serve_learned_kernel<N>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                               (int)LEARNED_LDS);
    LLAMA_SERVE_PREP_CASE(1)
    LLAMA_SERVE_PREP_CASE(2)
    LLAMA_SERVE_PREP_CASE(3)
    LLAMA_SERVE_PREP_CASE(4)
    LLAMA_SERVE_PREP_CASE(5)
    LLAMA_SERVE_PREP_CASE(6)
    LLAMA_SERVE_PREP_CASE(7)
    LLAMA_SERVE_PREP_CASE(8)
#undef LLAMA_SERVE_PREP_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_serve_learned(const DevTables& t, const ServeRing& r, const LearnedArgs& a, int workgroups,
                                hipStream_t s) {
  if (workgroups < 1 || r.cap < 1 || !r.feat) return hipErrorInvalidValue;
#define LLAMA_SERVE_LEARNED_CASE(N)                                                                   \
  case N:                                                                                             \
    hipLaunchKernelGGL(serve_learned_kernel<N>, dim3(workgroups), dim3(64 * LEARNED_WAVES), LEARNED_LDS, s, t, r, a); \
    break;
  switch (t.n_hw) {
    LLAMA_SERVE_LEARNED_CASE(1)
    LLAMA_SERVE_LEARNED_CASE(2)
    LLAMA_SERVE_LEARNED_CASE(3)
    LLAMA_SERVE_LEARNED_CASE(4)
    LLAMA_SERVE_LEARNED_CASE(5)
    LLAMA_SERVE_LEARNED_CASE(6)
    LLAMA_SERVE_LEARNED_CASE(7)
    LLAMA_SERVE_LEARNED_CASE(8)
    default:
      return hipErrorInvalidValue;
  }
#undef LLAMA_SERVE_LEARNED_CASE
  return hipGetLastError();
}

}  // namespace llama
