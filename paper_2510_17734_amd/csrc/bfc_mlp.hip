// Dense layers of the warm-start network: forward, backward and ADAM for
// FP32 training, a BF16-input forward for inference.  Every product is one
// LDS-tiled MFMA kernel with a 64 x 64 output tile per 256-thread workgroup,
// each wavefront a 32 x 32 quarter as 2 x 2 MFMA blocks, bias and activation
// fused into the store: FP32 MFMA 16x16x4 on k-slabs of 16 for training
// (loaded along whichever operand dimension is contiguous), BF16 MFMA
// 16x16x32 with FP32 accumulation on k-slabs of 32 for inference.  The ReLU derivative of the backward pass
// is applied while the gradient operand is loaded, so dZ = dY * (Y > 0) is
// never stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>

#include "bfc_common.h"
#include "bfc_device.h"
#include "../../include/bfc_mlp.h"

namespace bfc {
namespace {

constexpr int kTile = 64, kSlab = 16, kPad = 4;

__device__ inline float load_as_float(const float* p, int64_t i) { return p[i]; }

// round to nearest even (finite inputs)
__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

struct Operand {
  const void* p;
  int64_t s_outer, s_k;  // element (outer, k) at p[outer * s_outer + k * s_k]
  const float* mask;     // optional: the element counts only where mask > 0
};

// C[i][j] = act(sum_k A(i, k) B(j, k) + bias[j]); A is M x K, B is N x K as
// (outer, k) operands.  Split over k (gridDim.z > 1): block z sums k in
// [z kc, (z+1) kc) and stores its plain partial tile at C + z M N (ldc = N).
template <typename TI>
__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, int64_t kc,
                                                   Operand A, Operand B, const float* bias,
                                                   int act, float* C, uint16_t* Ch,
                                                   int64_t ldc) {
  __shared__ float As[kSlab][kTile + kPad];
  __shared__ float Bs[kSlab][kTile + kPad];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;  // this wavefront's 32 x 32 quarter
  const int64_t i0 = (int64_t)blockIdx.y * kTile, j0 = (int64_t)blockIdx.x * kTile;
  const TI* ap = (const TI*)A.p;
  const TI* bp = (const TI*)B.p;
  const bool a_outer_fast = A.s_outer == 1, b_outer_fast = B.s_outer == 1;
  floatx4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int64_t kb = (int64_t)blockIdx.z * kc;
  const int64_t ke = kb + kc < K ? kb + kc : K;
  if (gridDim.z > 1) C += (int64_t)blockIdx.z * M * N;
  for (int64_t k0 = kb; k0 < ke; k0 += kSlab) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      // the contiguous dimension varies fastest across threads
      const int o = a_outer_fast ? (e & (kTile - 1)) : (e >> 4);
      const int kk = a_outer_fast ? (e >> 6) : (e & (kSlab - 1));
      const int64_t gi = i0 + o, gk = k0 + kk;
      float v = 0.f;
      if (gi < M && gk < ke) {
        const int64_t idx = gi * A.s_outer + gk * A.s_k;
        v = load_as_float(ap, idx);
        if (A.mask && !(A.mask[idx] > 0.f)) v = 0.f;
      }
      As[kk][o] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      const int o = b_outer_fast ? (e & (kTile - 1)) : (e >> 4);
      const int kk = b_outer_fast ? (e >> 6) : (e & (kSlab - 1));
      const int64_t gj = j0 + o, gk = k0 + kk;
      float v = 0.f;
      if (gj < N && gk < ke) {
        const int64_t idx = gj * B.s_outer + gk * B.s_k;
        v = load_as_float(bp, idx);
        if (B.mask && !(B.mask[idx] > 0.f)) v = 0.f;
      }
      Bs[kk][o] = v;
    }
    __syncthreads();
    // MFMA 16x16x4: lane supplies A[i = lane % 16][k = lane / 16] and
    // B[k = lane / 16][j = lane % 16] of its block
#pragma unroll
    for (int ks = 0; ks < kSlab; ks += 4) {
      const int g = ks + (lane >> 4), col = lane & 15;
      float xa[2], yb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) xa[x] = As[g][wr * 32 + x * 16 + col];
#pragma unroll
      for (int y = 0; y < 2; ++y) yb[y] = Bs[g][wc * 32 + y * 16 + col];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = Mfma<float>::step(xa[x], yb[y], acc[x][y]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + wr * 32 + x * 16 + Mfma<float>::out_row(lane, v);
        const int64_t gj = j0 + wc * 32 + y * 16 + (lane & 15);
        if (gi >= M || gj >= N) continue;
        float o = acc[x][y][v] + (bias ? bias[gj] : 0.f);
        if (act == 1) o = o > 0.f ? o : 0.f;
        if (C) C[gi * ldc + gj] = o;
        if (Ch) Ch[gi * ldc + gj] = to_bf16(o);
      }
}

// Inference product on the BF16 matrix cores: C = act(Xh Wh + bias) with Xh
// (M x K, row-major) and Wh (K x N, row-major) in BF16, FP32 accumulation.
// A 64 x 64 output tile per 256-thread workgroup, k-slabs of 32 (the depth
// of the 16x16x32 BF16 instruction) staged in LDS with k contiguous for both
// operands (Wh is transposed on the way in), so each lane reads its eight
// consecutive k values of a row or column as one 16-byte vector: lane l
// supplies A[l%16][8(l/16)..8(l/16)+7] and B[8(l/16)..8(l/16)+7][l%16].  Each
// wavefront computes a 32 x 32 quarter as 2 x 2 blocks; the output layout is
// the FP32 16x16x4 instruction's.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
constexpr int kSlabH = 32, kLdH = kSlabH + 8;  // padded row of a staged slab (80 bytes)

__global__ __launch_bounds__(256) void gemm_bf16_kernel(int64_t M, int64_t N, int64_t K,
                                                        const uint16_t* X, const uint16_t* W,
                                                        const float* bias, int act, float* C,
                                                        uint16_t* Ch, int64_t ldc) {
  __shared__ __attribute__((aligned(16))) uint16_t As[kTile * kLdH];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile * kLdH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int64_t i0 = (int64_t)blockIdx.y * kTile, j0 = (int64_t)blockIdx.x * kTile;
  floatx4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};
  for (int64_t k0 = 0; k0 < K; k0 += kSlabH) {
    {  // A: thread -> row tid / 4, eight k values from (tid % 4) * 8
      const int o = tid >> 2, kk = (tid & 3) * 8;
      const int64_t gi = i0 + o;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t gk = k0 + kk + t;
        As[o * kLdH + kk + t] = (gi < M && gk < K) ? X[gi * K + gk] : (uint16_t)0;
      }
    }
    {  // B: thread -> k row tid / 8, eight consecutive columns from (tid % 8) * 8
      const int kk = tid >> 3, o = (tid & 7) * 8;
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int64_t gj = j0 + o + t;
        Bs[(o + t) * kLdH + kk] = (gj < N && gk < K) ? W[gk * N + gj] : (uint16_t)0;
      }
    }
    __syncthreads();
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    bf16x8_t xa[2], yb[2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
      xa[x] = *(const bf16x8_t*)(As + (wr * 32 + x * 16 + r16) * kLdH + kq);
#pragma unroll
    for (int y = 0; y < 2; ++y)
      yb[y] = *(const bf16x8_t*)(Bs + (wc * 32 + y * 16 + r16) * kLdH + kq);
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[x], yb[y], acc[x][y], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + wr * 32 + x * 16 + Mfma<float>::out_row(lane, v);
        const int64_t gj = j0 + wc * 32 + y * 16 + (lane & 15);
        if (gi >= M || gj >= N) continue;
        float o = acc[x][y][v] + (bias ? bias[gj] : 0.f);
        if (act == 1) o = o > 0.f ? o : 0.f;
        if (C) C[gi * ldc + gj] = o;
        if (Ch) Ch[gi * ldc + gj] = to_bf16(o);
      }
}

// The split products' partial tiles summed in chunk order, then bias and
// activation, as the unsplit store does.
__global__ void splitk_reduce_kernel(int64_t M, int64_t N, int S, const float* ws,
                                     const float* bias, int act, float* C, uint16_t* Ch,
                                     int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t i = e / N, j = e % N;
  float o = 0.f;
  for (int z = 0; z < S; ++z) o += ws[(int64_t)z * M * N + e];
  o += bias ? bias[j] : 0.f;
  if (act == 1) o = o > 0.f ? o : 0.f;
  if (C) C[i * ldc + j] = o;
  if (Ch) Ch[i * ldc + j] = to_bf16(o);
}

// db[j] = sum_i dY[i][j] (* (Y[i][j] > 0) for ReLU), rows summed in order
__global__ void colsum_kernel(int64_t m, int64_t n, const float* dY, const float* Y, float* db) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float s = 0.f;
  for (int64_t i = 0; i < m; ++i) {
    const float g = dY[i * n + j];
    if (!Y || Y[i * n + j] > 0.f) s += g;
  }
  db[j] = s;
}

__global__ void adam_kernel(int64_t count, float* p, const float* g, float* m, float* v,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.f - b1) * gk;
  const float vk = b2 * v[k] + (1.f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

__global__ void to_bf16_kernel(int64_t count, const float* src, uint16_t* dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) dst[k] = to_bf16(src[k]);
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Workgroups a product should fill before its reduction is split, and the
// shortest chunk of the reduction one split block takes.
constexpr int64_t kSplitTarget = 1024, kMinChunk = 1024;

// The split products' partial tiles: one workspace per GPU, grown on demand
// and kept until the process ends.  Work on one stream is ordered; calls that
// overlap on different streams of one GPU would share it.
bfc_status splitk_workspace(size_t floats, float** out) {
  static std::mutex mu;
  static void* buf[64] = {};
  static size_t cap[64] = {};
  int dev = 0;
  BFC_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) {
    set_error("bfc_mlp: device index out of range");
    return BFC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (cap[dev] < floats) {
    void* fresh = nullptr;
    BFC_HIP_TRY(lib_malloc(&fresh, floats * sizeof(float)));
    if (buf[dev]) {
      // work queued on the old buffer finishes before it goes
      BFC_HIP_TRY(hipDeviceSynchronize());
      (void)hipFree(buf[dev]);
    }
    buf[dev] = fresh;
    cap[dev] = floats;
  }
  *out = (float*)buf[dev];
  return BFC_OK;
}

template <typename TI>
bfc_status gemm(int64_t M, int64_t N, int64_t K, Operand A, Operand B, const float* bias,
                int act, float* C, uint16_t* Ch, int64_t ldc, hipStream_t st) {
  if (M == 0 || N == 0) return BFC_OK;
  const int64_t gx = (N + kTile - 1) / kTile, gy = (M + kTile - 1) / kTile;
  if (gx > 0x7FFFFFFF || gy > 65535) {
    set_error("bfc_mlp: matrix too large for one launch");
    return BFC_EINVAL;
  }
  // few output tiles over a long reduction: split k so the launch fills the
  // GPU, chunks a multiple of the slab, partial tiles summed in order
  int64_t split = 1;
  if (gx * gy < kSplitTarget && K >= 2 * kMinChunk)
    split = std::min((kSplitTarget + gx * gy - 1) / (gx * gy), K / kMinChunk);
  if (split > 1) {
    int64_t kc = (K + split - 1) / split;
    kc = (kc + kSlab - 1) / kSlab * kSlab;
    split = (K + kc - 1) / kc;
    float* ws = nullptr;
    BFC_TRY(splitk_workspace((size_t)(split * M * N), &ws));
    gemm_kernel<TI><<<dim3((unsigned)gx, (unsigned)gy, (unsigned)split), 256, 0, st>>>(
        M, N, K, kc, A, B, nullptr, 0, ws, nullptr, N);
    BFC_HIP_TRY(hipGetLastError());
    splitk_reduce_kernel<<<blocks_for(M * N, 256), 256, 0, st>>>(M, N, (int)split, ws, bias, act,
                                                                 C, Ch, ldc);
    BFC_HIP_TRY(hipGetLastError());
    return BFC_OK;
  }
  gemm_kernel<TI><<<dim3((unsigned)gx, (unsigned)gy), 256, 0, st>>>(M, N, K, K, A, B, bias, act,
                                                                     C, Ch, ldc);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

bool bad_sizes(int64_t m, int64_t k, int64_t n) { return m < 0 || k < 0 || n < 0; }

}  // namespace
}  // namespace bfc

using namespace bfc;

extern "C" {

bfc_status bfc_mlp_forward(int64_t m, int64_t k, int64_t n, const float* X, const float* W,
                           const float* b, int32_t act, float* Y, void* hip_stream) {
  if (bad_sizes(m, k, n) || (act != 0 && act != 1) || (m * n > 0 && !Y) ||
      (m * k > 0 && !X) || (k * n > 0 && !W)) {
    set_error("bad bfc_mlp_forward arguments");
    return BFC_EINVAL;
  }
  // A(i, kk) = X[i][kk]; B(j, kk) = W[kk][j]
  return gemm<float>(m, n, k, Operand{X, k, 1, nullptr}, Operand{W, 1, n, nullptr}, b, act, Y,
                     nullptr, n, (hipStream_t)hip_stream);
}

bfc_status bfc_mlp_backward(int64_t m, int64_t k, int64_t n, const float* X, const float* W,
                            const float* Y, const float* dY, int32_t act, float* dX, float* dW,
                            float* db, void* hip_stream) {
  const bool mn = m * n > 0;
  if (bad_sizes(m, k, n) || (act != 0 && act != 1) || (act == 1 && mn && !Y) || (mn && !dY) ||
      (dW && m * k > 0 && !X) || (dX && k * n > 0 && !W)) {
    set_error("bad bfc_mlp_backward arguments");
    return BFC_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  const float* mask = act == 1 ? Y : nullptr;
  // dW[kk][j] = sum_i X[i][kk] dZ[i][j]: A(kk, i) = X[i][kk], B(j, i) = dZ[i][j]
  if (dW)
    BFC_TRY(gemm<float>(k, n, m, Operand{X, 1, k, nullptr}, Operand{dY, 1, n, mask}, nullptr, 0,
                        dW, nullptr, n, st));
  // dX[i][kk] = sum_j dZ[i][j] W[kk][j]: A(i, j) = dZ[i][j], B(kk, j) = W[kk][j]
  if (dX)
    BFC_TRY(gemm<float>(m, k, n, Operand{dY, n, 1, mask}, Operand{W, n, 1, nullptr}, nullptr, 0,
                        dX, nullptr, k, st));
  if (db && n > 0) {
    colsum_kernel<<<blocks_for(n, 256), 256, 0, st>>>(m, n, dY, mask, db);
    BFC_HIP_TRY(hipGetLastError());
  }
  return BFC_OK;
}

bfc_status bfc_mlp_forward_bf16(int64_t m, int64_t k, int64_t n, const uint16_t* Xh,
                                const uint16_t* Wh, const float* b, int32_t act, float* Y,
                                uint16_t* Yh, void* hip_stream) {
  if (bad_sizes(m, k, n) || (act != 0 && act != 1) || (m * n > 0 && !Y && !Yh) ||
      (m * k > 0 && !Xh) || (k * n > 0 && !Wh)) {
    set_error("bad bfc_mlp_forward_bf16 arguments");
    return BFC_EINVAL;
  }
  if (m == 0 || n == 0) return BFC_OK;
  const int64_t gx = (n + kTile - 1) / kTile, gy = (m + kTile - 1) / kTile;
  if (gx > 0x7FFFFFFF || gy > 65535) {
    set_error("bfc_mlp: matrix too large for one launch");
    return BFC_EINVAL;
  }
  gemm_bf16_kernel<<<dim3((unsigned)gx, (unsigned)gy), 256, 0, (hipStream_t)hip_stream>>>(
      m, n, k, Xh, Wh, b, act, Y, Yh, n);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

bfc_status bfc_mlp_to_bf16(int64_t count, const float* src, uint16_t* dst, void* hip_stream) {
  if (count < 0 || (count > 0 && (!src || !dst))) {
    set_error("bad bfc_mlp_to_bf16 arguments");
    return BFC_EINVAL;
  }
  if (count == 0) return BFC_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  to_bf16_kernel<<<blocks_for(count, 256), 256, 0, st>>>(count, src, dst);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

bfc_status bfc_mlp_adam(int64_t count, float* params, const float* grads, float* m, float* v,
                        int32_t t, float lr, float beta1, float beta2, float eps,
                        void* hip_stream) {
  if (count < 0 || t < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) ||
      !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f) ||
      (count > 0 && (!params || !grads || !m || !v))) {
    set_error("bad bfc_mlp_adam arguments");
    return BFC_EINVAL;
  }
  if (count == 0) return BFC_OK;
  const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
  hipStream_t st = (hipStream_t)hip_stream;
  adam_kernel<<<blocks_for(count, 256), 256, 0, st>>>(count, params, grads, m, v, lr, beta1,
                                                      beta2, eps, c1, c2);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

}  // extern "C"
