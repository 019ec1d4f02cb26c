// ALS sweep kernels for the tensorized butterfly (Alg. "ALS for Butterfly
// Completion", Sec. 5.1.1), entry reconstruction (eq. (BF_tensor_rep)) and the
// residual norms of eq. (BF_convergence).
//
// Outer cores (Z^1 fibers = rows, Z^(L+2) fibers = columns): one wavefront per
// fiber.  Each lane builds the local least-squares row a_e of its entries (the
// full right or left chain of r x r products), accumulates the real
// coordinates of conj(a) a^T and conj(a) t, the wavefront reduces them, and
// the same wavefront solves the r x r system in FP64.
//
// Inner cores: the Gram matrix of slice k is K = sum_e (conj(l) l^T) kron
// (conj(rho) rho^T) over its entries (l: left environment, rho: right).  In
// real coordinates (r^2 reals per Hermitian factor) this is the real matrix
// product S = A^T B over subgroups of entries that share one environment
// (same row or same column of the slice's tile): A holds the shared side,
// B the sum over the subgroup of the other side.  The right-hand side rides
// along as 2r extra columns, so one MFMA product per wavefront gives both.
// Work items (runs of subgroups of one slice) write partial products; a
// second kernel sums them per slice in a fixed order, forms the Hermitian
// system in FP64 and solves it with one wavefront.
#include "bfc_device.h"

namespace bfc {

namespace {

inline unsigned grid_for(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// reconstruction and residual
// ---------------------------------------------------------------------------
template <typename T, int R>
__device__ inline cx<T> entry_value(const cx<T>* cores, int64_t n, int L, int c, int i, int j) {
  if (i < 0 || j < 0 || i >= n || j >= n) {  // never read outside the cores
    const T nan = __builtin_nan("");
    return {nan, nan};
  }
  const uint32_t ib = (uint32_t)i / (uint32_t)c, jb = (uint32_t)j / (uint32_t)c;
  cx<T> v[R];
  left_chain<T, R>(cores, n, L, L + 1, i, ib, jb, v);
  const cx<T>* z = cores + last_off(n, L, R) + (int64_t)j * R;
  cx<T> x = {T(0), T(0)};
#pragma unroll
  for (int a = 0; a < R; ++a) cfma(x, v[a], z[a]);
  return x;
}

template <typename T, int R>
__global__ __launch_bounds__(256) void predict_kernel(const cx<T>* cores, int64_t n, int L, int c,
                                                      const int32_t* rows, const int32_t* cols,
                                                      int64_t m, double2* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m) return;
  const cx<T> x = entry_value<T, R>(cores, n, L, c, rows[e], cols[e]);
  out[e] = make_double2((double)x.x, (double)x.y);
}

constexpr int kResThreads = 256;

template <typename T, int R>
__global__ __launch_bounds__(kResThreads) void residual_kernel(
    const cx<T>* cores, int64_t n, int L, int c, const int32_t* rows, const int32_t* cols,
    const double2* vals, int64_t m, int64_t per_block, double* partial) {
  __shared__ double s0[kResThreads], s1[kResThreads];
  double a0 = 0.0, a1 = 0.0;
  const int64_t beg = (int64_t)blockIdx.x * per_block;
  const int64_t end = beg + per_block < m ? beg + per_block : m;
  for (int64_t e = beg + threadIdx.x; e < end; e += kResThreads) {
    const cx<T> x = entry_value<T, R>(cores, n, L, c, rows[e], cols[e]);
    const double2 t = vals[e];
    const double dx = t.x - (double)x.x, dy = t.y - (double)x.y;
    a0 += dx * dx + dy * dy;
    a1 += t.x * t.x + t.y * t.y;
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int off = kResThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s0[0];
    partial[2 * blockIdx.x + 1] = s1[0];
  }
}

__global__ __launch_bounds__(kResThreads) void residual_final_kernel(const double* partial,
                                                                     int nblk, double* out) {
  __shared__ double s0[kResThreads], s1[kResThreads];
  double a0 = 0.0, a1 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += kResThreads) {
    a0 += partial[2 * b];
    a1 += partial[2 * b + 1];
  }
  s0[threadIdx.x] = a0;
  s1[threadIdx.x] = a1;
  __syncthreads();
  for (int off = kResThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s0[0];
    out[1] = s1[0];
  }
}

// ---------------------------------------------------------------------------
// Hermitian system assembly from real coordinates
// ---------------------------------------------------------------------------

// K[(a,b),(a2,b2)] of an inner slice from S (row-major, width W):
// K = sum (Hl[a][a2] * Hr[b][b2]) with Hl, Hr given by their real coordinates.
template <int R>
__device__ inline double2 inner_K(const double* S, int W, int row, int col) {
  const int a = row / R, b = row % R, a2 = col / R, b2 = col % R;
  int reA, imA, sA, reB, imB, sB;
  herm_coord(a, a2, R, reA, imA, sA);
  herm_coord(b, b2, R, reB, imB, sB);
  double re = S[reA * W + reB];
  double im = 0.0;
  if (imA >= 0 && imB >= 0) re -= (double)(sA * sB) * S[imA * W + imB];
  if (imB >= 0) im += (double)sB * S[reA * W + imB];
  if (imA >= 0) im += (double)sA * S[imA * W + reB];
  return make_double2(re, im);
}

// right-hand side h[(a,b)] from the 2r x 2r corner of S
template <int R>
__device__ inline double2 inner_h(const double* S, int W, int row) {
  const int a = row / R, b = row % R;
  const int D = R * R;
  const int Are = D + a, Aim = D + R + a, Bre = D + b, Bim = D + R + b;
  return make_double2(S[Are * W + Bre] + S[Aim * W + Bim], S[Are * W + Bim] - S[Aim * W + Bre]);
}

// ---------------------------------------------------------------------------
// outer cores: one wavefront (workgroup of 64) per fiber, fused solve
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(64) void outer_update_kernel(
    cx<T>* cores, int64_t n, int L, int c, int last, const int32_t* rows, const int32_t* cols,
    const cx<T>* vals, const int32_t* blk_off, int nblocks, double reg_rel, double reg_floor,
    int prox, int32_t* flags) {
  constexpr int D = R * R;
  __shared__ double2 M[R * R];
  __shared__ double2 rhs[R];
  __shared__ double2 sol[R];
  __shared__ double Ssh[D + 2 * R];
  const int lane = threadIdx.x;
  const int b = blockIdx.x;
  const int e0 = blk_off[b], e1 = blk_off[b + 1];
  if (e0 == e1) return;  // no observed entry: keep the fiber
  T acc[D];
  T hx[R], hy[R];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = T(0);
#pragma unroll
  for (int k = 0; k < R; ++k) hx[k] = hy[k] = T(0);
  for (int e = e0 + lane; e < e1; e += 64) {
    const int i = rows[e], j = cols[e];
    const uint32_t ib = (uint32_t)i / (uint32_t)c, jb = (uint32_t)j / (uint32_t)c;
    const cx<T> t = vals[e];
    cx<T> a[R];
    if (last)
      left_chain<T, R>(cores, n, L, L + 1, i, ib, jb, a);
    else
      right_chain<T, R>(cores, n, L, 0, j, ib, jb, a);
    herm_acc<T, R>(acc, a);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      cx<T> h = {hx[k], hy[k]};
      cfma_conj(h, a[k], t);
      hx[k] = h.x;
      hy[k] = h.y;
    }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = wave_sum(acc[k]);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    hx[k] = wave_sum(hx[k]);
    hy[k] = wave_sum(hy[k]);
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < D; ++k) Ssh[k] = (double)acc[k];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      Ssh[D + k] = (double)hx[k];
      Ssh[D + R + k] = (double)hy[k];
    }
  }
  __syncthreads();
  // K[a][a2] from the real coordinates; trace; regularization ladder
  double tr = 0.0;
#pragma unroll
  for (int a = 0; a < R; ++a) tr += Ssh[a * R + a];
  const double tau = tr / R;
  const double unit = fmax(reg_floor, 0x1p-53);
  double lam = fmax(reg_rel, R * reg_floor) * tau;
  cx<T>* fiber = cores + (last ? last_off(n, L, R) : 0) + (int64_t)b * R;
  bool ok = false;
  int attempt = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, R * unit * tau);
    }
    __syncthreads();
    if (lane < R * R) {
      const int a = lane / R, a2 = lane % R;
      int re, im, sg;
      herm_coord(a, a2, R, re, im, sg);
      double2 v = make_double2(Ssh[re], im >= 0 ? sg * Ssh[im] : 0.0);
      if (a == a2) v.x += lam;
      M[lane] = v;
    }
    if (lane < R) {
      const cx<T> old = fiber[lane];
      double2 h = make_double2(Ssh[D + lane], Ssh[D + R + lane]);
      if (prox) {
        h.x += lam * (double)old.x;
        h.y += lam * (double)old.y;
      }
      rhs[lane] = h;
      sol[lane] = h;
    }
    __syncthreads();
    ok = wave_cholesky(M, R, lane);
    if (ok) break;
  }
  if (!ok) {
    if (lane == 0) atomicAdd(flags, 1);
    return;
  }
  if (attempt > 0 && lane == 0) atomicAdd(flags + 1, 1);
  wave_chol_solve(M, sol, R, lane);
  // one refinement step against the assembled FP64 system
  if (lane < R) {
    double2 res = rhs[lane];
    for (int k = 0; k < R; ++k) {
      int re, im, sg;
      herm_coord(lane, k, R, re, im, sg);
      double2 m = make_double2(Ssh[re], im >= 0 ? sg * Ssh[im] : 0.0);
      if (k == lane) m.x += lam;
      const double2 s = sol[k];
      res.x -= m.x * s.x - m.y * s.y;
      res.y -= m.x * s.y + m.y * s.x;
    }
    rhs[lane] = res;
  }
  __syncthreads();
  wave_chol_solve(M, rhs, R, lane);
  if (lane < R) {
    const double2 s = sol[lane], d = rhs[lane];
    fiber[lane] = {T(s.x + d.x), T(s.y + d.y)};
  }
}

// ---------------------------------------------------------------------------
// inner cores: Gram/RHS partial products per work item (one wavefront)
// ---------------------------------------------------------------------------
template <int R>
struct InnerGeom {
  static constexpr int D = R * R;
  static constexpr int W = D + 2 * R;
  static constexpr int WP = (W + 15) / 16 * 16;
  static constexpr int NB = WP / 16;
  static constexpr int LDW = WP + 1;  // padded LDS row
};

template <typename T, int R, int BYROW>
__global__ __launch_bounds__(64) void inner_gram_kernel(
    const cx<T>* cores, int64_t n, int L, int c, int p, const int32_t* rows, const int32_t* cols,
    const cx<T>* vals, const int32_t* sub_off, const WorkItem* items, T* partials) {
  typedef InnerGeom<R> G;
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T As[64 * G::LDW];
  __shared__ T Bs[64 * G::LDW];
  const int lane = threadIdx.x;
  const WorkItem it = items[blockIdx.x];
  acc_t acc[G::NB][G::NB];
#pragma unroll
  for (int x = 0; x < G::NB; ++x)
#pragma unroll
    for (int y = 0; y < G::NB; ++y) acc[x][y] = acc_t{T(0), T(0), T(0), T(0)};

  for (int base = it.sub0; base < it.sub1; base += 64) {
    const int s = base + lane;
    T* arow = As + lane * G::LDW;
    T* brow = Bs + lane * G::LDW;
#pragma unroll
    for (int k = 0; k < G::WP; ++k) {
      arow[k] = T(0);
      brow[k] = T(0);
    }
    if (s < it.sub1) {
      const int e0 = sub_off[s], e1 = sub_off[s + 1];
      const int i0 = rows[e0], j0 = cols[e0];
      const uint32_t ib0 = (uint32_t)i0 / (uint32_t)c, jb0 = (uint32_t)j0 / (uint32_t)c;
      T sum[G::D];
      T yx[R], yy[R];
#pragma unroll
      for (int k = 0; k < G::D; ++k) sum[k] = T(0);
#pragma unroll
      for (int k = 0; k < R; ++k) yx[k] = yy[k] = T(0);
      cx<T> shared_env[R];
      if (BYROW) {
        // one row: left environment shared, right environment per entry
        left_chain<T, R>(cores, n, L, p, i0, ib0, jb0, shared_env);
        for (int e = e0; e < e1; ++e) {
          const int j = cols[e];
          const uint32_t jb = (uint32_t)j / (uint32_t)c;
          const cx<T> t = vals[e];
          cx<T> rho[R];
          right_chain<T, R>(cores, n, L, p, j, ib0, jb, rho);
          herm_acc<T, R>(sum, rho);
#pragma unroll
          for (int k = 0; k < R; ++k) {
            cx<T> h = {yx[k], yy[k]};
            cfma_conj(h, rho[k], t);
            yx[k] = h.x;
            yy[k] = h.y;
          }
        }
        T tmp[G::D];
#pragma unroll
        for (int k = 0; k < G::D; ++k) tmp[k] = T(0);
        herm_acc<T, R>(tmp, shared_env);
#pragma unroll
        for (int k = 0; k < G::D; ++k) {
          arow[k] = tmp[k];
          brow[k] = sum[k];
        }
#pragma unroll
        for (int k = 0; k < R; ++k) {
          arow[G::D + k] = shared_env[k].x;
          arow[G::D + R + k] = shared_env[k].y;
          brow[G::D + k] = yx[k];
          brow[G::D + R + k] = yy[k];
        }
      } else {
        // one column: right environment shared, left environment per entry
        right_chain<T, R>(cores, n, L, p, j0, ib0, jb0, shared_env);
        for (int e = e0; e < e1; ++e) {
          const int i = rows[e];
          const uint32_t ib = (uint32_t)i / (uint32_t)c;
          const cx<T> t = vals[e];
          cx<T> lft[R];
          left_chain<T, R>(cores, n, L, p, i, ib, jb0, lft);
          herm_acc<T, R>(sum, lft);
#pragma unroll
          for (int k = 0; k < R; ++k) {
            cx<T> h = {yx[k], yy[k]};
            cfma_conj(h, lft[k], t);
            yx[k] = h.x;
            yy[k] = h.y;
          }
        }
        T tmp[G::D];
#pragma unroll
        for (int k = 0; k < G::D; ++k) tmp[k] = T(0);
        herm_acc<T, R>(tmp, shared_env);
#pragma unroll
        for (int k = 0; k < G::D; ++k) {
          arow[k] = sum[k];
          brow[k] = tmp[k];
        }
        // w = sum conj(l) t on the A side, rho on the B side, imaginary parts
        // negated so that the right-hand side reads like the row case
#pragma unroll
        for (int k = 0; k < R; ++k) {
          arow[G::D + k] = yx[k];
          arow[G::D + R + k] = -yy[k];
          brow[G::D + k] = shared_env[k].x;
          brow[G::D + R + k] = -shared_env[k].y;
        }
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 64; kk += 4) {
      const int g = kk + (lane >> 4);
      const int col = lane & 15;
      T xa[G::NB], yb[G::NB];
#pragma unroll
      for (int x = 0; x < G::NB; ++x) xa[x] = As[g * G::LDW + x * 16 + col];
#pragma unroll
      for (int y = 0; y < G::NB; ++y) yb[y] = Bs[g * G::LDW + y * 16 + col];
#pragma unroll
      for (int x = 0; x < G::NB; ++x)
#pragma unroll
        for (int y = 0; y < G::NB; ++y) acc[x][y] = Mfma<T>::step(xa[x], yb[y], acc[x][y]);
    }
    __syncthreads();
  }
  T* out = partials + (int64_t)blockIdx.x * G::WP * G::WP;
#pragma unroll
  for (int x = 0; x < G::NB; ++x)
#pragma unroll
    for (int y = 0; y < G::NB; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = x * 16 + Mfma<T>::out_row(lane, v);
        const int col = y * 16 + (lane & 15);
        out[row * G::WP + col] = acc[x][y][v];
      }
}

// ---------------------------------------------------------------------------
// inner cores: per-slice sum of partials, FP64 Hermitian solve (one wavefront)
// ---------------------------------------------------------------------------
template <typename T, int R>
__global__ __launch_bounds__(64) void inner_solve_kernel(cx<T>* slices, const T* partials,
                                                         const int32_t* tile_items,
                                                         double reg_rel, double reg_floor,
                                                         int prox, int32_t* flags) {
  typedef InnerGeom<R> G;
  constexpr int D = G::D;
  constexpr int WP = G::WP;
  __shared__ double S[WP * WP];
  __shared__ double2 M[D * D];
  __shared__ double2 rhs[D];
  __shared__ double2 sol[D];
  const int lane = threadIdx.x;
  const int tile = blockIdx.x;
  const int it0 = tile_items[tile], it1 = tile_items[tile + 1];
  if (it0 == it1) return;  // no observed entry in this slice: keep it
  for (int k = lane; k < WP * WP; k += 64) {
    double s = 0.0;
    for (int it = it0; it < it1; ++it) s += (double)partials[(int64_t)it * WP * WP + k];
    S[k] = s;
  }
  __syncthreads();
  double trl = 0.0;
  for (int k = lane; k < D; k += 64) trl += inner_K<R>(S, WP, k, k).x;
  const double tau = wave_sum(trl) / D;
  const double unit = fmax(reg_floor, 0x1p-53);
  double lam = fmax(reg_rel, D * reg_floor) * tau;
  cx<T>* slice = slices + (int64_t)tile * D;
  bool ok = false;
  int attempt = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, D * unit * tau);
    }
    __syncthreads();
    for (int k = lane; k < D * D; k += 64) {
      double2 v = inner_K<R>(S, WP, k / D, k % D);
      if (k / D == k % D) v.x += lam;
      M[k] = v;
    }
    for (int k = lane; k < D; k += 64) {
      double2 h = inner_h<R>(S, WP, k);
      if (prox) {
        const cx<T> old = slice[k];
        h.x += lam * (double)old.x;
        h.y += lam * (double)old.y;
      }
      rhs[k] = h;
      sol[k] = h;
    }
    __syncthreads();
    ok = wave_cholesky(M, D, lane);
    if (ok) break;
  }
  if (!ok) {
    if (lane == 0) atomicAdd(flags, 1);
    return;
  }
  if (attempt > 0 && lane == 0) atomicAdd(flags + 1, 1);
  wave_chol_solve(M, sol, D, lane);
  // one step of iterative refinement against the FP64 system rebuilt from S
  if (lane < D) {
    double2 res = rhs[lane];
    for (int k = 0; k < D; ++k) {
      double2 m = inner_K<R>(S, WP, lane, k);
      if (k == lane) m.x += lam;
      const double2 s = sol[k];
      res.x -= m.x * s.x - m.y * s.y;
      res.y -= m.x * s.y + m.y * s.x;
    }
    rhs[lane] = res;
  }
  __syncthreads();
  wave_chol_solve(M, rhs, D, lane);
  if (lane < D) {
    const double2 s = sol[lane], d = rhs[lane];
    slice[lane] = {T(s.x + d.x), T(s.y + d.y)};
  }
}

// ---------------------------------------------------------------------------
// cores: conversion and counter-based random start
// ---------------------------------------------------------------------------
template <typename T>
__global__ void cores_from_c128_kernel(const double2* src, cx<T>* dst, int64_t m) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[k] = {T(src[k].x), T(src[k].y)};
}
template <typename T>
__global__ void cores_to_c128_kernel(const cx<T>* src, double2* dst, int64_t m) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[k] = make_double2((double)src[k].x, (double)src[k].y);
}

// SplitMix64 output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ inline uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Value k: u1, u2 from splitmix64(seed ^ splitmix64(2k)), splitmix64(seed ^
// splitmix64(2k+1)) (53-bit uniforms in (0, 1]), Box-Muller pair scaled to
// CN(0, 1/r).
template <typename T>
__global__ void random_cores_kernel(cx<T>* dst, int64_t m, uint64_t seed, double sd) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const uint64_t h1 = splitmix64(seed ^ splitmix64(2 * (uint64_t)k));
  const uint64_t h2 = splitmix64(seed ^ splitmix64(2 * (uint64_t)k + 1));
  const double u1 = ((h1 >> 11) + 1) * (1.0 / 9007199254740992.0);
  const double u2 = (h2 >> 11) * (1.0 / 9007199254740992.0);
  const double rad = sqrt(-2.0 * log(u1)) * sd;
  const double ang = 6.283185307179586 * u2;
  dst[k] = {T(rad * cos(ang)), T(rad * sin(ang))};
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename T, int R>
bfc_status sweep_core_t(Problem* P, int p, hipStream_t st) {
  cx<T>* cores = (cx<T>*)P->cores;
  const CoreLayout& C = P->lay[p];
  const double reg = P->cfg.reg_rel;
  // Gram accumulated in FP32: keep lam above its rounding level
  const double floor_ = P->prec == BFC_C128 ? 0.0 : 0x1p-24;
  const int prox = P->cfg.reg_mode == BFC_REG_PROXIMAL ? 1 : 0;
  const int L = P->L;
  if (p == 0 || p == L + 1) {
    {
      ProfScope ps(&P->prof, KIND_OUTER, st);
      outer_update_kernel<T, R><<<C.nblocks, 64, 0, st>>>(
          cores, P->n, L, P->c, p == L + 1 ? 1 : 0, C.rows, C.cols, (const cx<T>*)C.vals,
          C.blk_off, C.nblocks, reg, floor_, prox, P->flags);
    }
    BFC_HIP_TRY(hipGetLastError());
    return BFC_OK;
  }
  if (C.nitems > 0) {
    ProfScope ps(&P->prof, KIND_INNER_GRAM, st);
    if (C.group_by_row)
      inner_gram_kernel<T, R, 1><<<C.nitems, 64, 0, st>>>(cores, P->n, L, P->c, p, C.rows, C.cols,
                                                          (const cx<T>*)C.vals, C.sub_off, C.items,
                                                          (T*)P->partials);
    else
      inner_gram_kernel<T, R, 0><<<C.nitems, 64, 0, st>>>(cores, P->n, L, P->c, p, C.rows, C.cols,
                                                          (const cx<T>*)C.vals, C.sub_off, C.items,
                                                          (T*)P->partials);
    BFC_HIP_TRY(hipGetLastError());
  }
  cx<T>* slices = cores + inner_off(P->n, L, R, p);
  {
    ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
    inner_solve_kernel<T, R><<<C.nblocks, 64, 0, st>>>(slices, (const T*)P->partials,
                                                       C.tile_items, reg, floor_, prox,
                                                       P->flags);
  }
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <typename T, int R>
bfc_status predict_t(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                     void* out, hipStream_t st) {
  {
    ProfScope ps(&P->prof, KIND_PREDICT, st);
    predict_kernel<T, R><<<grid_for(m), 256, 0, st>>>((const cx<T>*)P->cores, P->n, P->L, P->c,
                                                      rows, cols, m, (double2*)out);
  }
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <typename T, int R>
bfc_status residual_t(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                      const void* vals, double* out2, hipStream_t st) {
  const int64_t nblk_max = (int64_t)(P->red_len / 2);
  int64_t per = (m + nblk_max - 1) / nblk_max;
  per = ((per + kResThreads - 1) / kResThreads) * kResThreads;
  if (per < kResThreads) per = kResThreads;
  const int64_t nblk = (m + per - 1) / per;
  ProfScope ps(&P->prof, KIND_RESIDUAL, st);
  residual_kernel<T, R><<<(unsigned)nblk, kResThreads, 0, st>>>(
      (const cx<T>*)P->cores, P->n, P->L, P->c, rows, cols, (const double2*)vals, m, per, P->red);
  BFC_HIP_TRY(hipGetLastError());
  residual_final_kernel<<<1, kResThreads, 0, st>>>(P->red, (int)nblk, out2);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <template <typename, int> class F, typename... Args>
bfc_status dispatch(int prec, int r, Args... args) {
#define BFC_CASE(RR)                                                     \
  case RR:                                                               \
    return prec == BFC_C128 ? F<double, RR>::run(args...) : F<float, RR>::run(args...);
  switch (r) {
    BFC_CASE(1)
    BFC_CASE(2)
    BFC_CASE(3)
    BFC_CASE(4)
    BFC_CASE(5)
    BFC_CASE(6)
    BFC_CASE(7)
    BFC_CASE(8)
    default:
      set_error("rank out of range");
      return BFC_EINVAL;
  }
#undef BFC_CASE
}

template <typename T, int R>
struct SweepF {
  static bfc_status run(Problem* P, int p, hipStream_t st) { return sweep_core_t<T, R>(P, p, st); }
};
template <typename T, int R>
struct PredictF {
  static bfc_status run(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                        void* out, hipStream_t st) {
    return predict_t<T, R>(P, m, rows, cols, out, st);
  }
};
template <typename T, int R>
struct ResidualF {
  static bfc_status run(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                        const void* vals, double* out2, hipStream_t st) {
    return residual_t<T, R>(P, m, rows, cols, vals, out2, st);
  }
};

}  // namespace

size_t inner_partial_bytes(int prec, int r) {
  const int W = r * r + 2 * r;
  const int WP = (W + 15) / 16 * 16;
  return (size_t)WP * WP * (prec == BFC_C128 ? 8 : 4);
}

bfc_status launch_sweep_core(Problem* P, int core, hipStream_t st) {
  return dispatch<SweepF>(P->prec, P->r, P, core, st);
}

bfc_status launch_predict(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                          void* out, hipStream_t st) {
  if (m == 0) return BFC_OK;
  return dispatch<PredictF>(P->prec, P->r, P, m, rows, cols, out, st);
}

bfc_status launch_residual(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                           const void* vals, double* out2, hipStream_t st) {
  return dispatch<ResidualF>(P->prec, P->r, P, m, rows, cols, vals, out2, st);
}

bfc_status launch_convert_cores(Problem* P, const void* src, void* dst, bool to_internal,
                                hipStream_t st) {
  const int64_t m = P->nparams;
  if (to_internal) {
    if (P->prec == BFC_C128)
      cores_from_c128_kernel<double><<<grid_for(m), 256, 0, st>>>((const double2*)src,
                                                                  (cx<double>*)P->cores, m);
    else
      cores_from_c128_kernel<float><<<grid_for(m), 256, 0, st>>>((const double2*)src,
                                                                 (cx<float>*)P->cores, m);
  } else {
    if (P->prec == BFC_C128)
      cores_to_c128_kernel<double><<<grid_for(m), 256, 0, st>>>((const cx<double>*)P->cores,
                                                                (double2*)dst, m);
    else
      cores_to_c128_kernel<float><<<grid_for(m), 256, 0, st>>>((const cx<float>*)P->cores,
                                                               (double2*)dst, m);
  }
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

bfc_status launch_random_cores(Problem* P, uint64_t seed, hipStream_t st) {
  const int64_t m = P->nparams;
  const double sd = sqrt(0.5 / P->r);
  if (P->prec == BFC_C128)
    random_cores_kernel<double><<<grid_for(m), 256, 0, st>>>((cx<double>*)P->cores, m, seed, sd);
  else
    random_cores_kernel<float><<<grid_for(m), 256, 0, st>>>((cx<float>*)P->cores, m, seed, sd);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

}  // namespace bfc
