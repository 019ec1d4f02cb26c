// Randomized low-rank to butterfly conversion (Sec. 5.2, Alg.
// Randomized_LR_to_Butterfly): the paper's initial guess for the sweeps turns
// the result X = A B^T of low-rank completion (the sweep with L = 0) into
// butterfly cores.
//
// Rows go from the leaves up to the middle level and columns likewise.  A
// leaf block's basis is the first r columns of the column-pivoted QR of its
// Gaussian sketch; at an inner level the two child blocks' projected factors
// (2r x R) are stacked, sketched with the other side's factor restricted to
// the current block and a Gaussian matrix, and the first r columns of the
// pivoted QR give the two children's r x r slices and the parent's projected
// factor Q^H F.  The middle core absorbs V W^T.  Everything is complex FP64;
// the conversion costs O(n r R log n) and runs once per completion.
//
// Layout: one wavefront per block, lane i holding row i of the block's
// sketch (at most 64 rows: c <= 64 at the leaves, 2r at inner levels) and
// its r + p columns in registers; column norms and inner products are
// wavefront butterfly sums, identical in every lane.
#include <mutex>
#include <string>
#include <utility>

#include "bfc_common.h"
#include "bfc_device.h"

namespace bfc {
namespace {

constexpr int kLrCols = 32;  // r + p
constexpr int kLrR = 16;     // rank R of the low-rank input
constexpr int kLrRank = 8;   // butterfly rank r

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline double2 wave_sum(double2 v) { return make_double2(wave_sum(v.x), wave_sum(v.y)); }
__device__ inline double2 cfma2(double2 acc, double2 a, double2 b) {  // acc + a b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
  return acc;
}
__device__ inline double2 conj_mul(double2 a, double2 b) {  // conj(a) b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// c ? a : b per component (a select of whole structs is lowered through
// scratch memory)
__device__ inline double2 sel(bool c, double2 a, double2 b) {
  return make_double2(c ? a.x : b.x, c ? a.y : b.y);
}

// First k columns of the Q factor of a column-pivoted Householder QR of the
// nrows x ncol matrix whose row `lane` is m (rows >= nrows are zero).  Each
// step pivots the remaining column of largest norm (first on ties) and
// reflects it onto beta e_j, beta = -exp(i arg x_j) ||x||; Q is the product
// of the reflectors applied to the first k unit vectors.  Lane i receives
// row i of Q.
__device__ __attribute__((always_inline)) inline void wave_qrcp(double2 (&m)[kLrCols], int ncol,
                                                                int nrows, int k,
                                                                double2 (&Q)[kLrRank], int lane) {
  const bool row = lane < nrows;
  double2 U[kLrRank];
#pragma unroll
  for (int j = 0; j < kLrRank; ++j) {
    U[j] = make_double2(0.0, 0.0);
    if (j >= k) continue;
    double best = -1.0;
    int t = j;
#pragma unroll
    for (int col = j; col < kLrCols; ++col) {
      if (col >= ncol) continue;
      const double a = (row && lane >= j) ? m[col].x * m[col].x + m[col].y * m[col].y : 0.0;
      const double s = wave_sum(a);
      if (s > best) {
        best = s;
        t = col;
      }
    }
    {
      const double2 mj = m[j];
      double2 nj = mj;
#pragma unroll
      for (int col = j + 1; col < kLrCols; ++col) {
        const bool sw = col == t;
        nj = sel(sw, m[col], nj);
        m[col] = sel(sw, mj, m[col]);
      }
      m[j] = nj;
    }
    const double nx = sqrt(best);
    if (!(nx > 0.0)) continue;  // a zero column: the reflector is the identity
    const double2 x = sel(row && lane >= j, m[j], make_double2(0.0, 0.0));
    const double2 alpha = make_double2(__shfl(x.x, j), __shfl(x.y, j));
    const double aa = sqrt(alpha.x * alpha.x + alpha.y * alpha.y);
    const double2 phase =
        sel(aa > 0.0, make_double2(alpha.x / aa, alpha.y / aa), make_double2(1.0, 0.0));
    const double2 v =
        sel(lane == j, make_double2(alpha.x + phase.x * nx, alpha.y + phase.y * nx), x);
    const double vn = sqrt(wave_sum(v.x * v.x + v.y * v.y));
    const double2 u = make_double2(v.x / vn, v.y / vn);
    U[j] = u;
#pragma unroll
    for (int col = j + 1; col < kLrCols; ++col) {
      if (col >= ncol) continue;
      const double2 w = wave_sum(conj_mul(u, m[col]));
      m[col].x -= 2.0 * (u.x * w.x - u.y * w.y);
      m[col].y -= 2.0 * (u.x * w.y + u.y * w.x);
    }
  }
#pragma unroll
  for (int a = 0; a < kLrRank; ++a) Q[a] = make_double2(lane == a && a < k ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int j = kLrRank - 1; j >= 0; --j) {
    if (j >= k) continue;
#pragma unroll
    for (int a = 0; a < kLrRank; ++a) {
      if (a >= k) continue;
      const double2 w = wave_sum(conj_mul(U[j], Q[a]));
      Q[a].x -= 2.0 * (U[j].x * w.x - U[j].y * w.y);
      Q[a].y -= 2.0 * (U[j].x * w.y + U[j].y * w.x);
    }
  }
}

// S[b][z][q] = sum_t F[b len + t][z] O[t][q]: the sketch of every block of one
// level, F the other side's factor (B for rows, A for columns).  One
// workgroup per (block, z, q): a strided sum and a fixed-order tree.
__global__ __launch_bounds__(256) void lr_sketch_kernel(const double2* F, int R, const double2* O,
                                                        int ncol, int64_t len, double2* S) {
  const int q = blockIdx.x % ncol;
  const int z = (blockIdx.x / ncol) % R;
  const int64_t b = blockIdx.x / ((int64_t)ncol * R);
  double2 acc = make_double2(0.0, 0.0);
  for (int64_t t = threadIdx.x; t < len; t += 256)
    acc = cfma2(acc, F[(b * len + t) * R + z], O[t * ncol + q]);
  __shared__ double2 red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[threadIdx.x].x += red[threadIdx.x + s].x;
      red[threadIdx.x].y += red[threadIdx.x + s].y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) S[(b * R + z) * ncol + q] = red[0];
}

// Projected factor Vout[blk][k][z] = sum_i conj(Q_i[k]) f_i[z] over the lanes.
__device__ __attribute__((always_inline)) inline void project(const double2 (&Q)[kLrRank],
                                                              const double2 (&f)[kLrR], int r, int R,
                                                              double2* out, int lane) {
#pragma unroll
  for (int k = 0; k < kLrRank; ++k) {
    if (k >= r) continue;
#pragma unroll
    for (int z = 0; z < kLrR; ++z) {
      if (z >= R) continue;
      const double2 s = wave_sum(conj_mul(Q[k], f[z]));
      if (lane == 0) out[k * R + z] = s;
    }
  }
}

// One wavefront per leaf block of c rows: M = F_block S, Q its basis (the
// block's rows of Z^1 or Z^(L+2)), V = Q^H F_block.
__global__ __launch_bounds__(64) void lr_leaf_kernel(const double2* F, int R, const double2* S,
                                                     int ncol, int c, int r, double2* core,
                                                     double2* Vout) {
  const int b = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < c;
  const int64_t g = (int64_t)b * c + (row ? lane : 0);
  double2 f[kLrR];
#pragma unroll
  for (int z = 0; z < kLrR; ++z)
    f[z] = sel(row && z < R, F[g * R + (z < R ? z : 0)], make_double2(0.0, 0.0));
  double2 m[kLrCols];
#pragma unroll
  for (int q = 0; q < kLrCols; ++q) {
    m[q] = make_double2(0.0, 0.0);
    if (q >= ncol) continue;
#pragma unroll
    for (int z = 0; z < kLrR; ++z)
      if (z < R) m[q] = cfma2(m[q], f[z], S[z * ncol + q]);
  }
  double2 Q[kLrRank];
  wave_qrcp(m, ncol, c, r, Q, lane);
  if (row) {
#pragma unroll
    for (int k = 0; k < kLrRank; ++k)
      if (k < r) core[g * r + k] = Q[k];
  }
  project(Q, f, r, R, Vout + (int64_t)b * r * R, lane);
}

// One wavefront per (parent, other-side block) of inner level l.  Row side:
// block index (u << l) | w, children ((2u+beta) << (l-1)) | (w >> 1) of the
// previous level, sketch block w, slices ((2u+beta) << l) | w of core l with
// row k of the slice = row beta r + k of Q.  Column side: block index
// (x << (L-l)) | v, children ((x >> 1) << (L-l+1)) | (2v+beta), sketch block
// x, slices (x << m) | (2v+beta) of core m = L+1-l, the slice being the
// transpose of Q's half.
__global__ __launch_bounds__(64) void lr_inner_kernel(const double2* Vin, int R, const double2* S,
                                                      int ncol, int r, int L, int l, int colside,
                                                      double2* core, double2* Vout) {
  const int idx = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < 2 * r;
  const int beta = row ? lane / r : 0, k = row ? lane % r : 0;
  int child, sblk;
  int64_t key;
  if (!colside) {
    const int u = idx >> l, w = idx & ((1 << l) - 1);
    child = ((2 * u + beta) << (l - 1)) | (w >> 1);
    sblk = w;
    key = ((int64_t)(2 * u + beta) << l) | w;
  } else {
    const int x = idx >> (L - l), v = idx & ((1 << (L - l)) - 1);
    child = ((x >> 1) << (L - l + 1)) | (2 * v + beta);
    sblk = x;
    key = ((int64_t)x << (L + 1 - l)) | (2 * v + beta);
  }
  double2 f[kLrR];
#pragma unroll
  for (int z = 0; z < kLrR; ++z)
    f[z] = sel(row && z < R, Vin[((int64_t)child * r + k) * R + (z < R ? z : 0)],
               make_double2(0.0, 0.0));
  const double2* Sb = S + (int64_t)sblk * R * ncol;
  double2 m[kLrCols];
#pragma unroll
  for (int q = 0; q < kLrCols; ++q) {
    m[q] = make_double2(0.0, 0.0);
    if (q >= ncol) continue;
#pragma unroll
    for (int z = 0; z < kLrR; ++z)
      if (z < R) m[q] = cfma2(m[q], f[z], Sb[z * ncol + q]);
  }
  double2 Q[kLrRank];
  wave_qrcp(m, ncol, 2 * r, r, Q, lane);
  if (row) {
    double2* slice = core + key * r * r;
#pragma unroll
    for (int a = 0; a < kLrRank; ++a) {
      if (a >= r) continue;
      if (!colside)
        slice[k * r + a] = Q[a];
      else
        slice[a * r + k] = Q[a];
    }
  }
  project(Q, f, r, R, Vout + (int64_t)idx * r * R, lane);
}

// Middle core (the last row-side one, core lr): slice key absorbs V W^T of
// block ((key >> lr) >> 1, key & (2^lr - 1)).  One thread per slice row.
__global__ __launch_bounds__(256) void lr_middle_kernel(double2* core, const double2* V,
                                                        const double2* W, int r, int R, int lr,
                                                        int64_t nrows) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= nrows) return;
  const int64_t key = t / r;
  const int a = (int)(t % r);
  const int64_t u = (key >> lr) >> 1, w = key & ((1 << lr) - 1);
  const int64_t blk = (u << lr) | w;
  const double2* Vb = V + blk * r * R;
  const double2* Wb = W + blk * r * R;
  double2* zrow = core + key * r * r + (int64_t)a * r;
  double2 z[kLrRank], o[kLrRank];
#pragma unroll
  for (int q = 0; q < kLrRank; ++q) {
    z[q] = sel(q < r, zrow[q < r ? q : 0], make_double2(0.0, 0.0));
    o[q] = make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int b = 0; b < kLrRank; ++b) {
    if (b >= r) continue;
#pragma unroll
    for (int q = 0; q < kLrRank; ++q) {
      if (q >= r) continue;
      double2 tqb = make_double2(0.0, 0.0);  // (V W^T)[q][b]
      for (int zz = 0; zz < R; ++zz) tqb = cfma2(tqb, Vb[q * R + zz], Wb[b * R + zz]);
      o[b] = cfma2(o[b], z[q], tqb);
    }
  }
#pragma unroll
  for (int b = 0; b < kLrRank; ++b)
    if (b < r) zrow[b] = o[b];
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Arguments shared by both entry points, checked; sets the error message.
bfc_status lr2bf_check(int64_t n, int32_t L, int32_t r, int32_t R, int32_t p, const void* d_A,
                       const void* d_B, const void* d_sketches, const void* d_cores_out,
                       const char* who) {
  if (!d_A || !d_B || !d_sketches || !d_cores_out) {
    set_error(std::string(who) + ": null pointer");
    return BFC_EINVAL;
  }
  if (L < 1 || L > 24 || n <= 0 || (n >> L) << L != n) {
    set_error(std::string(who) + ": need L >= 1 and n = c 2^L");
    return BFC_EINVAL;
  }
  const int64_t c = n >> L;
  if (r < 1 || r > kLrRank || c < r || c > 64 || R < 1 || R > kLrR || p < 0 ||
      r + p > kLrCols) {
    set_error(std::string(who) + ": need 1 <= r <= 8, r <= c <= 64, 1 <= R <= 16, "
              "0 <= p, r + p <= 32");
    return BFC_EINVAL;
  }
  return BFC_OK;
}

// Scratch values (complex128) the conversion needs: the projected factors of
// two levels for each side and the sketches of one level.
int64_t lr2bf_scratch_elems(int32_t L, int32_t r, int32_t R, int32_t p) {
  const int64_t nb = (int64_t)1 << L;
  return 4 * nb * r * R + nb * R * (r + p);
}

// Enqueues the whole conversion on st with buf as its scratch (every value of
// it is written before it is read, so its contents on entry do not matter).
// Allocates nothing.
bfc_status lr2bf_enqueue(int64_t n, int32_t L, int32_t r, int32_t R, int32_t p, const double2* A,
                         const double2* B, const double2* sk, double2* cores, double2* buf,
                         hipStream_t st) {
  const int64_t c = n >> L;
  const int ncol = r + p;
  const int lr = (L + 1) / 2, lc = L / 2;
  const double2* orow[13];  // L <= 24: at most 13 levels per side
  const double2* ocol[13];
  int64_t off = 0;
  for (int l = 0; l <= lr; ++l) {
    orow[l] = sk + off;
    off += (n >> l) * ncol;
  }
  for (int l = 0; l <= lc; ++l) {
    ocol[l] = sk + off;
    off += (n >> l) * ncol;
  }
  const int64_t nb = (int64_t)1 << L;
  const int64_t fac = nb * r * R;  // projected factors of one level
  double2 *V0 = buf, *V1 = buf + fac, *W0 = buf + 2 * fac, *W1 = buf + 3 * fac, *S = buf + 4 * fac;
  auto inner_core = [&](int m) { return cores + n * r + (int64_t)(m - 1) * (nb * 2) * r * r; };
  double2* last = cores + n * r + (int64_t)L * (nb * 2) * r * r;
  // row leaves, sketched through B^T O
  lr_sketch_kernel<<<(unsigned)(R * ncol), 256, 0, st>>>(B, R, orow[0], ncol, n, S);
  lr_leaf_kernel<<<(unsigned)nb, 64, 0, st>>>(A, R, S, ncol, (int)c, r, cores, V0);
  // column leaves, sketched through A^T O
  lr_sketch_kernel<<<(unsigned)(R * ncol), 256, 0, st>>>(A, R, ocol[0], ncol, n, S);
  lr_leaf_kernel<<<(unsigned)nb, 64, 0, st>>>(B, R, S, ncol, (int)c, r, last, W0);
  if (hipGetLastError() != hipSuccess) return BFC_EHIP;
  for (int l = 1; l <= lr; ++l) {
    lr_sketch_kernel<<<(unsigned)(((int64_t)1 << l) * R * ncol), 256, 0, st>>>(
        B, R, orow[l], ncol, n >> l, S);
    lr_inner_kernel<<<(unsigned)nb, 64, 0, st>>>(V0, R, S, ncol, r, L, l, 0, inner_core(l), V1);
    std::swap(V0, V1);
  }
  for (int l = 1; l <= lc; ++l) {
    lr_sketch_kernel<<<(unsigned)(((int64_t)1 << l) * R * ncol), 256, 0, st>>>(
        A, R, ocol[l], ncol, n >> l, S);
    lr_inner_kernel<<<(unsigned)nb, 64, 0, st>>>(W0, R, S, ncol, r, L, l, 1,
                                                 inner_core(L + 1 - l), W1);
    std::swap(W0, W1);
  }
  const int64_t rows = nb * 2 * r;
  lr_middle_kernel<<<blocks_for(rows, 256), 256, 0, st>>>(inner_core(lr), V0, W0, r, R, lr, rows);
  if (hipGetLastError() != hipSuccess) return BFC_EHIP;
  return BFC_OK;
}

// Scratch of bfc_lowrank_to_butterfly_noalloc: kLrScratchBytes of device
// memory per GPU the library runs on, held until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is a
// stand-in, not a device address): its device address is looked up once per
// device with hipGetSymbolAddress, on that device's first call, and kept.
constexpr int64_t kLrScratchBytes = int64_t(16) << 20;
static __device__ __align__(256) double scratch[kLrScratchBytes / sizeof(double)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

bfc_status scratch_of_current_device(double2** out) {
  int dev = -1;
  BFC_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("bfc_lowrank_to_butterfly_noalloc: device index out of range");
    return BFC_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("bfc_lowrank_to_butterfly_noalloc: hipGetSymbolAddress: ") +
                hipGetErrorString(e));
      return BFC_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = (double2*)g_scratch_ptr[dev];
  return BFC_OK;
}

}  // namespace
}  // namespace bfc

using namespace bfc;

extern "C" bfc_status bfc_lowrank_to_butterfly(int64_t n, int32_t L, int32_t r, int32_t R,
                                               int32_t p, const void* d_A, const void* d_B,
                                               const void* d_sketches, void* d_cores_out,
                                               void* hip_stream) {
  set_error("");
  BFC_TRY(lr2bf_check(n, L, r, R, p, d_A, d_B, d_sketches, d_cores_out,
                      "bfc_lowrank_to_butterfly"));
  hipStream_t st = (hipStream_t)hip_stream;
  double2* buf = nullptr;
  BFC_HIP_TRY(lib_malloc((void**)&buf, sizeof(double2) * lr2bf_scratch_elems(L, r, R, p)));
  const bfc_status status =
      lr2bf_enqueue(n, L, r, R, p, (const double2*)d_A, (const double2*)d_B,
                    (const double2*)d_sketches, (double2*)d_cores_out, buf, st);
  const hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(buf);
  if (status != BFC_OK || e != hipSuccess) {
    set_error("bfc_lowrank_to_butterfly: a kernel launch failed");
    return BFC_EHIP;
  }
  return BFC_OK;
}

extern "C" bfc_status bfc_lowrank_to_butterfly_noalloc(int64_t n, int32_t L, int32_t r, int32_t R,
                                                       int32_t p, const void* d_A, const void* d_B,
                                                       const void* d_sketches, void* d_cores_out,
                                                       void* hip_stream) {
  set_error("");
  BFC_TRY(lr2bf_check(n, L, r, R, p, d_A, d_B, d_sketches, d_cores_out,
                      "bfc_lowrank_to_butterfly_noalloc"));
  const int64_t need = lr2bf_scratch_elems(L, r, R, p) * (int64_t)sizeof(double2);
  if (need > kLrScratchBytes) {
    set_error("bfc_lowrank_to_butterfly_noalloc: needs " + std::to_string(need) +
              " bytes of scratch, above the " + std::to_string(kLrScratchBytes) +
              "-byte maximum (2^L (4 r R + R (r + p)) complex128 values); use "
              "bfc_lowrank_to_butterfly");
    return BFC_EINVAL;
  }
  double2* buf = nullptr;
  BFC_TRY(scratch_of_current_device(&buf));
  if (lr2bf_enqueue(n, L, r, R, p, (const double2*)d_A, (const double2*)d_B,
                    (const double2*)d_sketches, (double2*)d_cores_out, buf,
                    (hipStream_t)hip_stream) != BFC_OK) {
    set_error("bfc_lowrank_to_butterfly_noalloc: a kernel launch failed");
    return BFC_EHIP;
  }
  return BFC_OK;
}
