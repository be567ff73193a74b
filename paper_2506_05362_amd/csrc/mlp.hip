// Surrogate network on gfx950: BF16 matrix-core GEMMs with FP32 accumulation,
// fused bias / GELU / GELU' epilogues, MSE loss and FP32 Adam.  C ABI in
// include/pd_mlp.h.
//
// Every layer product is one kernel k_gemm: a 256-thread workgroup computes a
// 64 x 64 tile of C = A B with gfx950's v_mfma_f32_16x16x32_bf16 (each
// wavefront owns a 32 x 32 quarter as 2 x 2 matrix-core blocks); A and B are
// read from FP32 arrays through arbitrary strides (so the transposed operands
// of the backward pass need no copies), rounded to BF16 and staged in LDS 32
// columns of K at a time.

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "pd_mlp.h"

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;
constexpr int kK = 32;
constexpr int kKRow = kK + 8;  // LDS row of a staged tile (bf16): 16-byte aligned, banks staggered

// C += A B on the matrix cores, 16 x 16 x 32 in BF16 with FP32 accumulation.
// Lane l holds 8 consecutive k of row l % 16 of A (group l / 16) and the same
// 8 k of column l % 16 of B, so A and B pair each k alike; the result C[4
// (l / 16) + e][l % 16] lands in element e.
__device__ __forceinline__ v4f mfma_16x16x32(const v8s& a, const v8s& b, const v4f& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ short to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct Gemm {
  const float* A;
  int64_t sam, sak;  // A(m, k) = A[m * sam + k * sak]
  const float* B;
  int64_t sbk, sbn;  // B(k, n) = B[k * sbk + n * sbn]
  int64_t M, N, K;
  float* C;
  int64_t ldc;         // C(m, n) = C[m * ldc + n]
  const float* bias;   // [N]
  float* Zout;         // pre-activation store (ldc), may be null
  const float* Zin;    // pre-activation for GELU' (ldc)
};

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

// Eight consecutive k of one row (or column) of an operand, rounded to BF16:
// X(k) = p[k * sk] for k0 <= k < k0 + 8, zero past K or where ok is false.
// A contiguous, 16-byte aligned run inside K is read as two float4.
__device__ __forceinline__ v8s load8_bf16(const float* p, int64_t sk, int64_t k0, int64_t K, bool ok) {
  v8s r;
  if (ok && sk == 1 && k0 + 8 <= K && ((reinterpret_cast<uintptr_t>(p + k0) & 15u) == 0)) {
    const float4 x = *reinterpret_cast<const float4*>(p + k0);
    const float4 y = *reinterpret_cast<const float4*>(p + k0 + 4);
    r = v8s{to_bf16(x.x), to_bf16(x.y), to_bf16(x.z), to_bf16(x.w), to_bf16(y.x), to_bf16(y.y), to_bf16(y.z),
            to_bf16(y.w)};
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = k0 + e;
      r[e] = to_bf16((ok && k < K) ? p[k * sk] : 0.0f);
    }
  }
  return r;
}

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm(Gemm g) {
  __shared__ __align__(16) short As[kTile][kKRow];  // As[m][k]
  __shared__ __align__(16) short Bs[kTile][kKRow];  // Bs[n][k] (B transposed)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
  const int wm = (wv >> 1) * 32, wn = (wv & 1) * 32;
  v4f acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  const int lr = tid >> 2, lk = (tid & 3) * 8;  // staging: row / column of the tile, 8 k each
  for (int64_t k0 = 0; k0 < g.K; k0 += kK) {
    {
      // one 16-byte LDS store per operand and thread
      const int64_t m = m0 + lr, n = n0 + lr;
      *reinterpret_cast<v8s*>(&As[lr][lk]) = load8_bf16(g.A + (m < g.M ? m * g.sam : 0), g.sak, k0 + lk, g.K, m < g.M);
      *reinterpret_cast<v8s*>(&Bs[lr][lk]) = load8_bf16(g.B + (n < g.N ? n * g.sbn : 0), g.sbk, k0 + lk, g.K, n < g.N);
    }
    __syncthreads();
    v8s a[2], b[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const v8s*>(&As[wm + i * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const v8s*>(&Bs[wn + j * 16 + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma_16x16x32(a[i], b[j], acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t m = m0 + wm + i * 16 + 4 * (lane >> 4) + e;
        const int64_t n = n0 + wn + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const float v = acc[i][j][e];
        const int64_t o = m * g.ldc + n;
        if (EPI == EPI_STORE) {
          g.C[o] = v;
        } else if (EPI == EPI_BIAS) {
          g.C[o] = v + g.bias[n];
        } else if (EPI == EPI_BIAS_GELU) {
          const float z = v + g.bias[n];
          if (g.Zout) g.Zout[o] = z;
          g.C[o] = gelu(z);
        } else {
          g.C[o] = v * gelu_grad(g.Zin[o]);
        }
      }
}

// residual, loss partial sums and dY = 2 (Y_hat - Y) / (B * d)
__global__ __launch_bounds__(256) void k_loss(const float* yh, const float* y, float* dy, int64_t n,
                                               float scale, double* partial) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256) {
    const float r = yh[i] - y[i];
    dy[i] = scale * r;
    s += (double)r * (double)r;
  }
  red[tid] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) red[tid] += red[tid + o];
    __syncthreads();
  }
  if (tid == 0) partial[blockIdx.x] = red[0];
}

// db[n] = sum_m dZ[m][n]
__global__ void k_colsum(const float* dz, int64_t M, int64_t N, float* db) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  for (int64_t m = 0; m < M; ++m) s += dz[m * N + n];
  db[n] = s;
}

// Adam with decoupled weight decay: p -= lr (m_hat / (sqrt(v_hat) + eps) + wd p)
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float wd, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i];
  p[i] = pi - lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * pi);
}

// ---------------------------------------------------------------------------
// Fused inference for din <= 16 -> 256 -> 256 -> 256 -> dout <= 16.
// Phase A: layer 1 on the vector units (its 6-wide products are too small for
// the matrix cores), its GELU outputs become the BF16 A operand of layer 2
// directly in registers; layer 2 on the matrix cores with W2 resident in LDS;
// GELU; BF16 H2 to HBM.  Phase B: layer 3 from H2 with W3 in LDS; each 16 x 16
// output tile is GELU'd and turned into the A operand of layer 4 through a
// small per-wavefront LDS tile, so layer 4 runs on the matrix cores as it goes.
// Operands are rounded to BF16 exactly where the layer-by-layer path rounds
// them (x, W1, activations, W2..W4); accumulation is FP32.
// Each workgroup keeps a weight matrix in LDS and walks tiles of 16 rows per
// wavefront.  The weights fill most of a CU's LDS, so one workgroup runs per
// CU: eight wavefronts (two per SIMD) let one hide the latency of the other's
// vector work (the exact-erf GELUs) and matrix-core chains.
// ---------------------------------------------------------------------------

constexpr int kH = 256;          // hidden width of the fused path
constexpr int kWRow = kH + 8;    // LDS row of a transposed weight matrix (bf16), padded, 16-byte aligned
constexpr int kTRow = 32 + 8;    // per-wavefront transpose tile row (bf16)
constexpr int kIW = 8;           // wavefronts per workgroup
constexpr int kIRows = 16 * kIW;  // batch rows per tile

// Order the LDS accesses of one wavefront's lanes (all of them converged here):
// writes before the call are seen by reads after it in every lane.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float bf16_to_f(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

struct Infer {
  const float* x;
  int64_t M;
  int din, dout;
  const float* W1;   // [din][kH] fp32 (rounded to bf16 on use)
  const float* b1;
  const short* W2t;  // [kH][kH] bf16, transposed (n-major)
  const float* b2;
  const short* W3t;
  const float* b3;
  const short* W4t;  // [16][kH] bf16, rows >= dout zero
  const float* b4;
  short* H2;         // [M][kH] bf16
  float* y;          // [M][dout]
};

// out[n][k] = bf16(W[k][n]) for n < N, zero rows for N <= n < rows_out
__global__ void k_pack_t(const float* W, int K, int N, int rows_out, short* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)rows_out * K) return;
  const int n = (int)(i / K), k = (int)(i % K);
  out[i] = n < N ? to_bf16(W[(int64_t)k * N + n]) : (short)0;
}

__device__ __forceinline__ void stage_weights_t(const short* src, int rows, short* dst) {
  // rows x kH bf16 (16-byte pieces) into LDS rows of kWRow
  for (int i = threadIdx.x; i < rows * (kH / 8); i += blockDim.x) {
    const int r = i / (kH / 8), c = (i % (kH / 8)) * 8;
    *reinterpret_cast<v8s*>(dst + r * kWRow + c) = *reinterpret_cast<const v8s*>(src + (int64_t)r * kH + c);
  }
}

template <int DINP>
__global__ __launch_bounds__(64 * kIW) void k_infer_a(Infer a) {
  extern __shared__ __align__(16) char smem[];
  short* sW = reinterpret_cast<short*>(smem);                                   // [kH][kWRow]
  float* sW1 = reinterpret_cast<float*>(smem + sizeof(short) * kH * kWRow);     // [DINP][kH]
  float* sb1 = sW1 + DINP * kH;
  float* sb2 = sb1 + kH;
  short* sT = reinterpret_cast<short*>(sb2 + kH);                               // [kIW][16][kTRow]
  const int tid = threadIdx.x;
  stage_weights_t(a.W2t, kH, sW);
  for (int i = tid; i < DINP * kH; i += blockDim.x) sW1[i] = i < a.din * kH ? bf16_to_f(to_bf16(a.W1[i])) : 0.0f;
  for (int i = tid; i < kH; i += blockDim.x) {
    sb1[i] = a.b1[i];
    sb2[i] = a.b2[i];
  }
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  short* T = sT + wv * 16 * kTRow;
  const int64_t ntiles = (a.M + kIRows - 1) / kIRows;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * kIRows + wv * 16;
    const int64_t row = r0 + lr;
    float xv[DINP];
#pragma unroll
    for (int i = 0; i < DINP; ++i) xv[i] = (i < a.din && row < a.M) ? bf16_to_f(to_bf16(a.x[row * a.din + i])) : 0.0f;
    // k-step outer: the layer-1 output for this k-step is the A operand of all
    // 16 output tiles of layer 2, each with its own accumulator
    v4f acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kk = 0; kk < kH / 32; ++kk) {
      v8s A;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int k = kk * 32 + 8 * lg + j;
        float z = 0.0f;
#pragma unroll
        for (int i = 0; i < DINP; ++i) z = fmaf(xv[i], sW1[i * kH + k], z);
        A[j] = to_bf16(gelu(z + sb1[k]));
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const v8s b = *reinterpret_cast<const v8s*>(sW + (q * 16 + lr) * kWRow + kk * 32 + 8 * lg);
        acc[q] = mfma_16x16x32(A, b, acc[q]);
      }
    }
    // GELU of each pair of 16 x 16 tiles through this wavefront's LDS tile,
    // so that every lane stores 16 contiguous bytes of one row of H2
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * q2 + h, col = q * 16 + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) T[(4 * lg + e) * kTRow + 16 * h + lr] = to_bf16(gelu(acc[q][e] + sb2[col]));
      }
      wave_sync();
      const v8s hv = *reinterpret_cast<const v8s*>(T + lr * kTRow + 8 * lg);
      if (row < a.M) *reinterpret_cast<v8s*>(a.H2 + row * kH + q2 * 32 + 8 * lg) = hv;
      wave_sync();
    }
  }
}

__global__ __launch_bounds__(64 * kIW) void k_infer_b(Infer a) {
  extern __shared__ __align__(16) char smem[];
  short* sW = reinterpret_cast<short*>(smem);                  // [kH][kWRow]
  short* sW4 = sW + kH * kWRow;                                // [16][kWRow]
  short* sT = sW4 + 16 * kWRow;                                // [kIW][16][kTRow]
  static_assert((kWRow * 2) % 16 == 0 && (kTRow * 2) % 16 == 0, "16-byte LDS rows");
  float* sb3 = reinterpret_cast<float*>(sT + kIW * 16 * kTRow);  // [kH]
  float* sb4 = sb3 + kH;                                       // [16]
  const int tid = threadIdx.x;
  stage_weights_t(a.W3t, kH, sW);
  stage_weights_t(a.W4t, 16, sW4);
  for (int i = tid; i < kH; i += blockDim.x) sb3[i] = a.b3[i];
  if (tid < 16) sb4[tid] = tid < a.dout ? a.b4[tid] : 0.0f;
  __syncthreads();
  const int wv = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  short* T = sT + wv * 16 * kTRow;
  const int64_t ntiles = (a.M + kIRows - 1) / kIRows;
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * kIRows + wv * 16;
    const int64_t row = r0 + lr;
    v4f acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
    for (int kk = 0; kk < kH / 32; ++kk) {
      const v8s A = row < a.M ? *reinterpret_cast<const v8s*>(a.H2 + row * kH + kk * 32 + 8 * lg)
                              : v8s{0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const v8s b = *reinterpret_cast<const v8s*>(sW + (q * 16 + lr) * kWRow + kk * 32 + 8 * lg);
        acc[q] = mfma_16x16x32(A, b, acc[q]);
      }
    }
    // each pair of 16 x 16 tiles of layer 3: GELU, then transposed into the
    // 16 x 32 A operand of layer 4
    v4f acc4 = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q2 = 0; q2 < 8; ++q2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q = 2 * q2 + h, col = q * 16 + lr;
#pragma unroll
        for (int e = 0; e < 4; ++e) T[(4 * lg + e) * kTRow + 16 * h + lr] = to_bf16(gelu(acc[q][e] + sb3[col]));
      }
      wave_sync();  // T is this wavefront's own tile: no wait for the others
      const v8s a4 = *reinterpret_cast<const v8s*>(T + lr * kTRow + 8 * lg);
      const v8s b4 = *reinterpret_cast<const v8s*>(sW4 + lr * kWRow + q2 * 32 + 8 * lg);
      acc4 = mfma_16x16x32(a4, b4, acc4);
      wave_sync();
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t rr = r0 + 4 * lg + e;
      if (rr < a.M && lr < a.dout) a.y[rr * a.dout + lr] = acc4[e] + sb4[lr];
    }
  }
}

template <int DINP>
constexpr size_t lds_a() {
  return sizeof(short) * (kH * kWRow + kIW * 16 * kTRow) + sizeof(float) * (DINP * kH + 2 * kH);
}
constexpr size_t kLdsB = sizeof(short) * (kH * kWRow + 16 * kWRow + kIW * 16 * kTRow) + sizeof(float) * (kH + 16);

}  // namespace

struct pdm_net {
  std::vector<int32_t> dims;
  int64_t max_batch = 0, n_params = 0;
  hipStream_t stream = nullptr;
  int own_stream = 0;
  std::string err;
  float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  std::vector<float*> Z, Aout, dZ;  // per layer, [max_batch][dims[l+1]]
  float* yhat = nullptr;            // [max_batch][d_out]
  double* partial = nullptr;
  int nloss_blocks = 0;
  std::vector<int64_t> woff, boff;  // offsets of W_l, b_l in the parameter vector
  float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f, weight_decay = 0.0f;
  // fused inference path (din <= 16 -> 256 -> 256 -> 256 -> dout <= 16)
  int fused_ok = 0, use_fused = 0, cus = 0;
  short *W2t = nullptr, *W3t = nullptr, *W4t = nullptr, *H2 = nullptr;
  int64_t t = 0;
  std::vector<void*> owned;
  pd_alloc_fn alloc = nullptr;  // caller's device allocator (hipMalloc when none)
  pd_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
};

namespace {

pd_status fail(pdm_net* n, pd_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (n) n->err = buf;
  return st;
}

#define HIPCHK(net, call)                                                                    \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail((net), PD_ERR_HIP, "%s failed: %s", #call, hipGetErrorName(e_));           \
  } while (0)

template <typename T>
pd_status alloc(pdm_net* n, T** p, int64_t count) {
  void* q = nullptr;
  const size_t bytes = (sizeof(T) * (size_t)(count > 0 ? count : 1) + 255) & ~size_t(255);
  if (n->alloc) q = n->alloc(bytes, n->alloc_user);
  else if (hipMalloc(&q, bytes) != hipSuccess) q = nullptr;
  if (!q) return fail(n, PD_ERR_OOM, "device allocation of %lld elements failed", (long long)count);
  n->owned.push_back(q);
  *p = static_cast<T*>(q);
  return PD_OK;
}

#define TRY(e)                        \
  do {                                \
    pd_status s_ = (e);               \
    if (s_ != PD_OK) return s_;       \
  } while (0)

template <int EPI>
hipError_t gemm(const Gemm& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.N + kTile - 1) / kTile), (unsigned)((g.M + kTile - 1) / kTile));
  hipLaunchKernelGGL(k_gemm<EPI>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

int n_layers(const pdm_net* n) { return (int)n->dims.size() - 1; }

// forward of `batch` rows (<= max_batch) from x into y (device pointers)
pd_status forward_chunk(pdm_net* n, const float* x, int64_t batch, float* y, bool keep_z) {
  const int L = n_layers(n);
  const float* A = x;
  for (int l = 0; l < L; ++l) {
    const int64_t din = n->dims[l], dout = n->dims[l + 1];
    Gemm g{};
    g.A = A;
    g.sam = din;
    g.sak = 1;
    g.B = n->params + n->woff[l];
    g.sbk = dout;
    g.sbn = 1;
    g.M = batch;
    g.N = dout;
    g.K = din;
    g.bias = n->params + n->boff[l];
    g.ldc = dout;
    if (l < L - 1) {
      g.C = n->Aout[l];
      g.Zout = keep_z ? n->Z[l] : nullptr;
      HIPCHK(n, gemm<EPI_BIAS_GELU>(g, n->stream));
      A = n->Aout[l];
    } else {
      g.C = y;
      HIPCHK(n, gemm<EPI_BIAS>(g, n->stream));
    }
  }
  return PD_OK;
}

// loss and gradient into n->grad for one batch
pd_status loss_and_grad(pdm_net* n, const float* x, const float* y, int64_t batch, float* loss) {
  const int L = n_layers(n);
  const int64_t dout = n->dims[L];
  TRY(forward_chunk(n, x, batch, n->yhat, true));
  const int64_t cnt = batch * dout;
  hipLaunchKernelGGL(k_loss, dim3(n->nloss_blocks), dim3(256), 0, n->stream, n->yhat, y, n->dZ[L - 1],
                     cnt, 2.0f / (float)cnt, n->partial);
  HIPCHK(n, hipGetLastError());
  for (int l = L - 1; l >= 0; --l) {
    const int64_t din = n->dims[l], dl = n->dims[l + 1];
    const float* Ain = l == 0 ? x : n->Aout[l - 1];
    // dW_l = A_in^T dZ_l
    Gemm gw{};
    gw.A = Ain;
    gw.sam = 1;
    gw.sak = din;
    gw.B = n->dZ[l];
    gw.sbk = dl;
    gw.sbn = 1;
    gw.M = din;
    gw.N = dl;
    gw.K = batch;
    gw.C = n->grad + n->woff[l];
    gw.ldc = dl;
    HIPCHK(n, gemm<EPI_STORE>(gw, n->stream));
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((dl + 255) / 256)), dim3(256), 0, n->stream, n->dZ[l],
                       batch, dl, n->grad + n->boff[l]);
    HIPCHK(n, hipGetLastError());
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l^T) * GELU'(Z_{l-1})
      Gemm gx{};
      gx.A = n->dZ[l];
      gx.sam = dl;
      gx.sak = 1;
      gx.B = n->params + n->woff[l];
      gx.sbk = 1;
      gx.sbn = dl;
      gx.M = batch;
      gx.N = din;
      gx.K = dl;
      gx.C = n->dZ[l - 1];
      gx.ldc = din;
      gx.Zin = n->Z[l - 1];
      HIPCHK(n, gemm<EPI_GELU_GRAD>(gx, n->stream));
    }
  }
  if (loss) {
    std::vector<double> part((size_t)n->nloss_blocks);
    HIPCHK(n, hipMemcpyAsync(part.data(), n->partial, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                             n->stream));
    HIPCHK(n, hipStreamSynchronize(n->stream));
    double s = 0.0;
    for (double p : part) s += p;
    *loss = (float)(s / (double)cnt);
  }
  return PD_OK;
}

}  // namespace

extern "C" {

pd_status pdm_create(pdm_net** out, const int32_t* dims, int32_t n_dims, int64_t max_batch, pd_alloc_fn alloc_fn,
                     pd_free_fn free_fn, void* alloc_user, void* stream) {
  if (!out) return PD_ERR_INVALID;
  *out = nullptr;
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return PD_ERR_INVALID;
  pdm_net* n = new (std::nothrow) pdm_net();
  if (!n) return PD_ERR_OOM;
  *out = n;
  n->alloc = alloc_fn;
  n->free_fn = free_fn;
  n->alloc_user = alloc_user;
  if (!dims || n_dims < 2) return fail(n, PD_ERR_INVALID, "need at least two layer widths");
  for (int k = 0; k < n_dims; ++k)
    if (dims[k] < 1 || dims[k] > 1024) return fail(n, PD_ERR_INVALID, "layer width %d out of [1, 1024]", dims[k]);
  if (max_batch < 1 || max_batch > (1 << 24)) return fail(n, PD_ERR_INVALID, "max_batch out of range");
  n->dims.assign(dims, dims + n_dims);
  n->max_batch = max_batch;
  n->stream = static_cast<hipStream_t>(stream);
  if (!n->stream) {
    if (hipStreamCreate(&n->stream) != hipSuccess) return fail(n, PD_ERR_HIP, "hipStreamCreate failed");
    n->own_stream = 1;
  }
  const int L = n_dims - 1;
  int64_t o = 0;
  for (int l = 0; l < L; ++l) {
    n->woff.push_back(o);
    o += (int64_t)dims[l] * dims[l + 1];
    n->boff.push_back(o);
    o += dims[l + 1];
  }
  n->n_params = o;
  TRY(alloc(n, &n->params, o));
  TRY(alloc(n, &n->grad, o));
  TRY(alloc(n, &n->m, o));
  TRY(alloc(n, &n->v, o));
  n->Z.resize(L);
  n->Aout.resize(L);
  n->dZ.resize(L);
  for (int l = 0; l < L; ++l) {
    TRY(alloc(n, &n->Z[l], max_batch * dims[l + 1]));
    TRY(alloc(n, &n->Aout[l], max_batch * dims[l + 1]));
    TRY(alloc(n, &n->dZ[l], max_batch * dims[l + 1]));
  }
  TRY(alloc(n, &n->yhat, max_batch * dims[L]));
  if (n_dims == 5 && dims[1] == kH && dims[2] == kH && dims[3] == kH && dims[0] <= 16 && dims[4] <= 16) {
    int dev = 0, lds = 0;
    const size_t need_a = dims[0] <= 8 ? lds_a<8>() : lds_a<16>();
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        hipDeviceGetAttribute(&n->cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        (size_t)lds >= need_a && (size_t)lds >= kLdsB &&
        hipFuncSetAttribute(dims[0] <= 8 ? reinterpret_cast<const void*>(&k_infer_a<8>)
                                         : reinterpret_cast<const void*>(&k_infer_a<16>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)need_a) == hipSuccess &&
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_infer_b),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsB) == hipSuccess) {
      TRY(alloc(n, &n->W2t, (int64_t)kH * kH));
      TRY(alloc(n, &n->W3t, (int64_t)kH * kH));
      TRY(alloc(n, &n->W4t, (int64_t)16 * kH));
      TRY(alloc(n, &n->H2, max_batch * kH));
      n->fused_ok = n->use_fused = 1;
    }
    (void)hipGetLastError();
  }
  n->nloss_blocks = 256;
  TRY(alloc(n, &n->partial, n->nloss_blocks));
  HIPCHK(n, hipMemsetAsync(n->params, 0, sizeof(float) * o, n->stream));
  HIPCHK(n, hipMemsetAsync(n->m, 0, sizeof(float) * o, n->stream));
  HIPCHK(n, hipMemsetAsync(n->v, 0, sizeof(float) * o, n->stream));
  HIPCHK(n, hipStreamSynchronize(n->stream));
  return PD_OK;
}

int64_t pdm_param_count(const pdm_net* n) { return n ? n->n_params : 0; }

pd_status pdm_set_params(pdm_net* n, const float* p, int64_t cnt) {
  if (!n || !p) return PD_ERR_INVALID;
  if (cnt != n->n_params) return fail(n, PD_ERR_INVALID, "expected %lld parameters", (long long)n->n_params);
  HIPCHK(n, hipMemcpyAsync(n->params, p, sizeof(float) * cnt, hipMemcpyHostToDevice, n->stream));
  HIPCHK(n, hipMemsetAsync(n->m, 0, sizeof(float) * cnt, n->stream));
  HIPCHK(n, hipMemsetAsync(n->v, 0, sizeof(float) * cnt, n->stream));
  HIPCHK(n, hipStreamSynchronize(n->stream));
  n->t = 0;
  return PD_OK;
}

pd_status pdm_get_params(pdm_net* n, float* p, int64_t cnt) {
  if (!n || !p) return PD_ERR_INVALID;
  if (cnt < n->n_params) return fail(n, PD_ERR_INVALID, "expected room for %lld parameters", (long long)n->n_params);
  HIPCHK(n, hipMemcpyAsync(p, n->params, sizeof(float) * n->n_params, hipMemcpyDeviceToHost, n->stream));
  HIPCHK(n, hipStreamSynchronize(n->stream));
  return PD_OK;
}

pd_status pdm_set_adam(pdm_net* n, float b1, float b2, float eps, float weight_decay) {
  if (!n) return PD_ERR_INVALID;
  if (!(b1 >= 0 && b1 < 1 && b2 >= 0 && b2 < 1 && eps > 0 && weight_decay >= 0))
    return fail(n, PD_ERR_INVALID, "bad Adam parameters");
  n->weight_decay = weight_decay;
  n->beta1 = b1;
  n->beta2 = b2;
  n->eps = eps;
  return PD_OK;
}

pd_status pdm_set_inference(pdm_net* n, int32_t fused) {
  if (!n) return PD_ERR_INVALID;
  if (fused && !n->fused_ok)
    return fail(n, PD_ERR_UNSUPPORTED, "the fused inference path needs dims din<=16,256,256,256,dout<=16 "
                                       "and enough LDS per workgroup");
  n->use_fused = fused ? 1 : 0;
  return PD_OK;
}

pd_status pdm_forward(pdm_net* n, const float* x, int64_t batch, float* y) {
  if (!n || (!x && batch > 0) || (!y && batch > 0) || batch < 0) return PD_ERR_INVALID;
  const int64_t din = n->dims.front(), dout = n->dims.back();
  if (n->use_fused && batch > 0) {
    // BF16 transposed copies of W2, W3, W4 (parameters may have changed since the last call)
    const int64_t e = (int64_t)kH * kH;
    hipLaunchKernelGGL(k_pack_t, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, n->stream,
                       n->params + n->woff[1], kH, kH, kH, n->W2t);
    hipLaunchKernelGGL(k_pack_t, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, n->stream,
                       n->params + n->woff[2], kH, kH, kH, n->W3t);
    hipLaunchKernelGGL(k_pack_t, dim3((unsigned)((16 * kH + 255) / 256)), dim3(256), 0, n->stream,
                       n->params + n->woff[3], kH, (int)dout, 16, n->W4t);
    HIPCHK(n, hipGetLastError());
    for (int64_t b0 = 0; b0 < batch; b0 += n->max_batch) {
      const int64_t cb = batch - b0 < n->max_batch ? batch - b0 : n->max_batch;
      Infer a{};
      a.x = x + b0 * din;
      a.M = cb;
      a.din = (int)din;
      a.dout = (int)dout;
      a.W1 = n->params + n->woff[0];
      a.b1 = n->params + n->boff[0];
      a.W2t = n->W2t;
      a.b2 = n->params + n->boff[1];
      a.W3t = n->W3t;
      a.b3 = n->params + n->boff[2];
      a.W4t = n->W4t;
      a.b4 = n->params + n->boff[3];
      a.H2 = n->H2;
      a.y = y + b0 * dout;
      const int64_t tiles = (cb + kIRows - 1) / kIRows;
      const unsigned grid = (unsigned)std::min<int64_t>(tiles, std::max(n->cus, 1));
      if (din <= 8) hipLaunchKernelGGL(k_infer_a<8>, dim3(grid), dim3(64 * kIW), lds_a<8>(), n->stream, a);
      else hipLaunchKernelGGL(k_infer_a<16>, dim3(grid), dim3(64 * kIW), lds_a<16>(), n->stream, a);
      hipLaunchKernelGGL(k_infer_b, dim3(grid), dim3(64 * kIW), kLdsB, n->stream, a);
      HIPCHK(n, hipGetLastError());
    }
  } else {
    for (int64_t b0 = 0; b0 < batch; b0 += n->max_batch) {
      const int64_t cb = batch - b0 < n->max_batch ? batch - b0 : n->max_batch;
      TRY(forward_chunk(n, x + b0 * din, cb, y + b0 * dout, false));
    }
  }
  HIPCHK(n, hipStreamSynchronize(n->stream));
  return PD_OK;
}

pd_status pdm_gradients(pdm_net* n, const float* x, const float* y, int64_t batch, float* loss, float* grad) {
  if (!n || !x || !y || !grad) return PD_ERR_INVALID;
  if (batch < 1 || batch > n->max_batch) return fail(n, PD_ERR_INVALID, "batch must be in [1, max_batch]");
  TRY(loss_and_grad(n, x, y, batch, loss));
  HIPCHK(n, hipMemcpyAsync(grad, n->grad, sizeof(float) * n->n_params, hipMemcpyDeviceToHost, n->stream));
  HIPCHK(n, hipStreamSynchronize(n->stream));
  return PD_OK;
}

pd_status pdm_train_step(pdm_net* n, const float* x, const float* y, int64_t batch, float lr, float* loss) {
  if (!n || !x || !y) return PD_ERR_INVALID;
  if (batch < 1 || batch > n->max_batch) return fail(n, PD_ERR_INVALID, "batch must be in [1, max_batch]");
  if (!(lr > 0)) return fail(n, PD_ERR_INVALID, "learning rate must be > 0");
  TRY(loss_and_grad(n, x, y, batch, loss));
  n->t += 1;
  const float c1 = 1.0f - powf(n->beta1, (float)n->t), c2 = 1.0f - powf(n->beta2, (float)n->t);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n->n_params + 255) / 256)), dim3(256), 0, n->stream, n->params,
                     n->grad, n->m, n->v, n->n_params, lr, n->beta1, n->beta2, n->eps, n->weight_decay, c1, c2);
  HIPCHK(n, hipGetLastError());
  if (!loss) HIPCHK(n, hipStreamSynchronize(n->stream));
  return PD_OK;
}

void pdm_destroy(pdm_net* n) {
  if (!n) return;
  (void)hipStreamSynchronize(n->stream);
  for (void* p : n->owned) {
    if (n->free_fn) n->free_fn(p, n->alloc_user);
    else (void)hipFree(p);
  }
  if (n->own_stream) (void)hipStreamDestroy(n->stream);
  delete n;
}

const char* pdm_last_error(const pdm_net* n) { return n ? n->err.c_str() : "null network"; }

}  // extern "C"
