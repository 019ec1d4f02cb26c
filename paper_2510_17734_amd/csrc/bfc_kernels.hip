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
#include <cmath>
#include <type_traits>

#include "bfc_device.h"
#include "bfc_wide.h"

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

// One block per task: the per-block partial norms of one problem summed in
// the same order as residual_final_kernel.
struct ResFinalArgs {
  const double* partial;
  int nblk;
  double* out;
};
__global__ __launch_bounds__(kResThreads) void residual_final_batched(const ResFinalArgs* tasks) {
  const ResFinalArgs a = tasks[blockIdx.x];
  __shared__ double s0[kResThreads], s1[kResThreads];
  double a0 = 0.0, a1 = 0.0;
  for (int b = threadIdx.x; b < a.nblk; b += kResThreads) {
    a0 += a.partial[2 * b];
    a1 += a.partial[2 * b + 1];
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
    a.out[0] = s0[0];
    a.out[1] = s1[0];
  }
}

// ---------------------------------------------------------------------------
// Hermitian system assembly from real coordinates
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// outer cores: 16 lanes (one DPP row) per fiber, fused serial solve
// ---------------------------------------------------------------------------
constexpr int kOuterThreads = 256;
// blocks of an outer-core launch: 16 lanes per fiber
inline int outer_grid(const CoreLayout& C) {
  return (int)(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
}

// Regularized r x r solve of one fiber from its real-coordinate Gram (acc)
// and right-hand side (hx, hy); writes the fiber, or keeps it and counts a
// failure when no rung of the regularization ladder is positive definite.
template <typename T, int R>
__device__ __attribute__((always_inline)) inline void outer_fiber_solve(
    const T (&acc)[R * R], const T (&hx)[R], const T (&hy)[R], double reg_rel, double reg_floor,
    int prox, int32_t* flags, cx<T>* fiber) {
  // K[a][a2] from the real coordinates; trace; regularization ladder
  double tr = 0.0;
#pragma unroll
  for (int a = 0; a < R; ++a) tr += (double)acc[a * R + a];
  const double tau = tr / R;
  const double unit = fmax(reg_floor, 0x1p-53);
  double lam = fmax(reg_rel, R * reg_floor) * tau;
  double2 M[R][R];
  bool ok = false;
  int attempt = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, R * unit * tau);
    }
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        int re, im, sg;
        herm_coord(i, j, R, re, im, sg);
        M[i][j] = make_double2((double)acc[re], im >= 0 ? sg * (double)acc[im] : 0.0);
        if (i == j) M[i][j].x += lam;
      }
    ok = serial_cholesky<R>(M);
    if (ok) break;
  }
  if (!ok) {
    atomicAdd(flags, 1);
    return;
  }
  if (attempt > 0) atomicAdd(flags + 1, 1);
  double2 sol[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    sol[k] = make_double2((double)hx[k], (double)hy[k]);
    if (prox) {
      sol[k].x += lam * (double)fiber[k].x;
      sol[k].y += lam * (double)fiber[k].y;
    }
  }
  serial_chol_solve<R>(M, sol);
#pragma unroll
  for (int k = 0; k < R; ++k) fiber[k] = {T(sol[k].x), T(sol[k].y)};
}

template <typename T>
struct OuterArgs {
  cx<T>* fibers;
  const cx<T>* env;
  const int32_t* env_idx;
  const cx<T>* vals;
  const int32_t* blk_off;
  int nblocks;
  double reg_rel;
  double reg_floor;
  int prox;
  int32_t* flags;
  double* res_partial;  // per block: residual norms after the update, or null
  // UP > 0 (see outer_update_body): the adjacent inner core, L and c
  const cx<T>* zsl;
  int L, c;
};

// UP = 0: env holds every entry's environment vector (trie level 0 for core
// 0, level L+1 for core L+1) and env_idx names it.  UP = 1 (core 0) or 2
// (core L+1): env is the level above (right level 1, left level L) and
// env_idx holds 2 x node + bit (CoreLayout::up_node); the entry's vector is
// that node times one of the fiber's two slices of the adjacent core (Z^2
// on the left for UP = 1, Z^(L+1) on the right for UP = 2), the product
// that would have built the outermost level, with the same arithmetic, so
// that level is never stored.
template <typename T, int R, int UP = 0>
__device__ __attribute__((always_inline)) inline void outer_update_body(const OuterArgs<T>& A, int blk) {
  cx<T>* fibers = A.fibers;
  const cx<T>* env = A.env;
  const int32_t* env_idx = A.env_idx;
  const cx<T>* vals = A.vals;
  const int32_t* blk_off = A.blk_off;
  int nblocks = A.nblocks;
  double reg_rel = A.reg_rel;
  double reg_floor = A.reg_floor;
  int prox = A.prox;
  int32_t* flags = A.flags;

  constexpr int D = R * R;
  const int sub = threadIdx.x & 15;
  const int b = (blk * kOuterThreads + threadIdx.x) >> 4;
  int e0 = 0, e1 = 0;
  if (b < nblocks) {
    e0 = blk_off[b];
    e1 = blk_off[b + 1];
  }
  T acc[D];
  T hx[R], hy[R];
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = T(0);
#pragma unroll
  for (int k = 0; k < R; ++k) hx[k] = hy[k] = T(0);
  // UP > 0: the fiber's two slices of the adjacent core, staged by its 16
  // lanes (one wavefront) in LDS; the slice key is that of the outermost
  // trie level: (ib << 1) | top bit of jb for core 0 (fiber = row i, ib =
  // i / c), (top bit of ib << L) | jb for core L+1 (fiber = column j)
  __shared__ cx<T> zs[UP ? kOuterThreads / 16 : 1][2][R * R];
  const int fslot = UP ? (int)(threadIdx.x >> 4) : 0;
  if constexpr (UP > 0) {
    if (b < nblocks) {
      const int64_t blk_idx = b / A.c;
      const int64_t k0 = UP == 1 ? (blk_idx << 1) : blk_idx;
      const int64_t k1 = UP == 1 ? (blk_idx << 1) | 1 : ((int64_t)1 << A.L) | blk_idx;
      const cx<T>* s0 = A.zsl + k0 * (R * R);
      const cx<T>* s1 = A.zsl + k1 * (R * R);
      for (int e = sub; e < R * R; e += 16) {
        zs[fslot][0][e] = s0[e];
        zs[fslot][1][e] = s1[e];
      }
    }
    wave_sync();
  }
  // entry q's vector from its loaded node (UP > 0), in place
  auto lift = [&](cx<T> (&v)[R], int half) {
    if constexpr (UP == 1) mat_vec<T, R>(zs[fslot][half], v);
    if constexpr (UP == 2) vec_mat<T, R>(v, zs[fslot][half]);
  };
  // four entries per lane and step, their loads issued as one group
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4], half[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
      half[q] = 0;
      if (UP && id[q] >= 0) {
        half[q] = id[q] & 1;
        id[q] >>= 1;
      }
    }
    cx<T> v[4][R], t[4];
    gather_group<T, R, 4, true>(env, vals, id, ent, v, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      lift(v[q], half[q]);
      herm_acc<T, R>(acc, v[q]);
#pragma unroll
      for (int k = 0; k < R; ++k) {
        cx<T> h = {hx[k], hy[k]};
        cfma_conj(h, v[q][k], t[q]);
        hx[k] = h.x;
        hy[k] = h.y;
      }
    }
  }
  // every lane of the wavefront takes part in the row reductions
#pragma unroll
  for (int k = 0; k < D; ++k) acc[k] = row16_sum(acc[k]);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    hx[k] = row16_sum(hx[k]);
    hy[k] = row16_sum(hy[k]);
  }
  // the solve, by lane 0 of the fiber's row; z ends as the fiber's value
  cx<T> z[R];
#pragma unroll
  for (int k = 0; k < R; ++k) z[k] = cx<T>{T(0), T(0)};
  if (sub == 0 && b < nblocks) {
    cx<T>* fiber = fibers + (int64_t)b * R;
    if (e0 != e1)  // empty fiber: keep it
      outer_fiber_solve<T, R>(acc, hx, hy, reg_rel, reg_floor, prox, flags, fiber);
#pragma unroll
    for (int k = 0; k < R; ++k) z[k] = fiber[k];
  }
  if (!A.res_partial) return;  // the same for the whole launch
  // residual norms of the updated fiber over its entries: x_e = a_e . z
  const int src = (int)(threadIdx.x & 63) & ~15;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    z[k].x = __shfl(z[k].x, src);
    z[k].y = __shfl(z[k].y, src);
  }
  double r0 = 0.0, r1 = 0.0;
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4], half[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
      half[q] = 0;
      if (UP && id[q] >= 0) {
        half[q] = id[q] & 1;
        id[q] >>= 1;
      }
    }
    cx<T> vv[4][R], tt[4];
    gather_group<T, R, 4, true>(env, vals, id, ent, vv, tt);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      lift(vv[q], half[q]);
      const cx<T> t = tt[q];
      const cx<T>(&v)[R] = vv[q];
      cx<T> x = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < R; ++k) cfma(x, v[k], z[k]);
      const double dx = (double)t.x - (double)x.x, dy = (double)t.y - (double)x.y;
      r0 += dx * dx + dy * dy;
      r1 += (double)t.x * (double)t.x + (double)t.y * (double)t.y;
    }
  }
  r0 = row16_sum(r0);
  r1 = row16_sum(r1);
  // the block's 16 fibers summed in a fixed order: one pair per block
  __shared__ double fr[2 * (kOuterThreads / 16)];
  if (sub == 0) {
    fr[2 * (threadIdx.x >> 4)] = r0;
    fr[2 * (threadIdx.x >> 4) + 1] = r1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int f = 0; f < kOuterThreads / 16; ++f) {
      s0 += fr[2 * f];
      s1 += fr[2 * f + 1];
    }
    A.res_partial[2 * blk] = s0;
    A.res_partial[2 * blk + 1] = s1;
  }
}

template <typename T, int R, int UP>
__global__ __launch_bounds__(kOuterThreads) void outer_update_kernel(OuterArgs<T> A) {
  outer_update_body<T, R, UP>(A, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <typename T, int R, int UP>
__global__ __launch_bounds__(kOuterThreads) void outer_update_kernel_batched(const OuterArgs<T>* tasks, const int32_t* block_off,
    int ntasks) {
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int t = find_task(block_off, ntasks, b);
  outer_update_body<T, R, UP>(tasks[t], b - block_off[t]);
}


// ---------------------------------------------------------------------------
// inner cores: Gram/RHS partial products per work item (one wavefront)
// ---------------------------------------------------------------------------
// entries of a subgroup whose environment loads are in flight together
constexpr int kGatherGroup = 4;
// Entries whose loads a lane issues together while it forms a subgroup's Gram
// rows: four, or all eight of a subgroup at r = 8 in FP32, where the rows and
// the MFMA accumulators allow one wavefront per SIMD anyway and the loads in
// flight per wavefront are what hides the gather latency.
constexpr int gram_gather_group(int r, int bytes) { return (r == 8 && bytes == 4) ? 8 : 4; }

template <int R>
struct InnerGeom {
  static constexpr int D = R * R;
  static constexpr int W = D + 2 * R;
  static constexpr int WP = (W + 15) / 16 * 16;
  static constexpr int NB = WP / 16;
  static constexpr int LDW = WP + 1;  // padded LDS row
};

// The A and B rows of one subgroup (entries e0..e1 of one slice sharing a row
// when BYROW, else a column), in the Hermitian real coordinates described
// above; live = false gives zero rows.  Row case: A = [Rl | Re l | Im l],
// B = [sum Rrho | Re y | Im y], y = sum conj(rho) t.  Column case:
// A = [sum Rl | Re w | -Im w], B = [Rrho | Re rho | -Im rho], w = sum conj(l) t:
// the imaginary parts are negated so that the right-hand side reads the same
// way as in the row case.
// The same from indices already in registers: `shared` is the node of the
// environment the subgroup's entries share (left when BYROW), id[q] the node
// of the other environment of entry e0 + q (-1 from e1 on).
template <typename T, int R, int BYROW>
__device__ __attribute__((always_inline)) inline void subgroup_rows_ids(
    bool live, int e0, int e1, int shared, const int (&id)[kSubgroup], const cx<T>* lenv,
    const cx<T>* renv, const cx<T>* vals, T (&arow)[InnerGeom<R>::W],
    T (&brow)[InnerGeom<R>::W]) {
  constexpr int D = R * R;
  constexpr int GG = gram_gather_group(R, sizeof(T));
  T sum[D];
  T yx[R], yy[R];
  cx<T> shared_env[R];
#pragma unroll
  for (int k = 0; k < D; ++k) sum[k] = T(0);
#pragma unroll
  for (int k = 0; k < R; ++k) {
    yx[k] = yy[k] = T(0);
    shared_env[k] = cx<T>{T(0), T(0)};
  }
  if (live) load_env<T, R>(BYROW ? lenv : renv, shared, shared_env);
  {
    const cx<T>* esrc = BYROW ? renv : lenv;
    // entries in groups of G whose vector loads are issued together; a group
    // that no lane of the wavefront needs is skipped
#pragma unroll
    for (int g0 = 0; g0 < kSubgroup; g0 += GG) {
      if (__ballot(e0 + g0 < e1) == 0) break;
      int gid[GG], ent[GG];
#pragma unroll
      for (int g = 0; g < GG; ++g) {
        gid[g] = id[g0 + g];
        ent[g] = e0 + g0 + g;
      }
      cx<T> v[GG][R], t[GG];
      gather_group<T, R, GG>(esrc, vals, gid, ent, v, t);
#pragma unroll
      for (int g = 0; g < GG; ++g) {
        if (gid[g] < 0) continue;
        herm_acc<T, R>(sum, v[g]);
#pragma unroll
        for (int k = 0; k < R; ++k) {
          cx<T> h = {yx[k], yy[k]};
          cfma_conj(h, v[g][k], t[g]);
          yx[k] = h.x;
          yy[k] = h.y;
        }
      }
    }
  }
  T tmp[D];
#pragma unroll
  for (int k = 0; k < D; ++k) tmp[k] = T(0);
  herm_acc<T, R>(tmp, shared_env);
#pragma unroll
  for (int k = 0; k < D; ++k) {
    arow[k] = BYROW ? tmp[k] : sum[k];
    brow[k] = BYROW ? sum[k] : tmp[k];
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (BYROW) {
      arow[D + k] = shared_env[k].x;
      arow[D + R + k] = shared_env[k].y;
      brow[D + k] = yx[k];
      brow[D + R + k] = yy[k];
    } else {
      arow[D + k] = yx[k];
      arow[D + R + k] = -yy[k];
      brow[D + k] = shared_env[k].x;
      brow[D + R + k] = -shared_env[k].y;
    }
  }
}

// The A and B rows of one subgroup from the per-entry index arrays (lidx and
// ridx name each sorted entry's left and right environment source).
template <typename T, int R, int BYROW>
__device__ __attribute__((always_inline)) inline void subgroup_rows(
    bool live, int e0, int e1, const cx<T>* lenv, const int32_t* lidx, const cx<T>* renv,
    const int32_t* ridx, const cx<T>* vals, T (&arow)[InnerGeom<R>::W],
    T (&brow)[InnerGeom<R>::W]) {
  // a subgroup holds at most kSubgroup entries: every index load first
  const int32_t* eidx = BYROW ? ridx : lidx;
  int shared = 0;
  if (live) shared = BYROW ? lidx[e0] : ridx[e0];
  int id[kSubgroup];
#pragma unroll
  for (int q = 0; q < kSubgroup; ++q) id[q] = (e0 + q < e1) ? eidx[e0 + q] : -1;
  subgroup_rows_ids<T, R, BYROW>(live, e0, e1, shared, id, lenv, renv, vals, arow, brow);
}

template <typename T>
struct GramArgs {
  const cx<T>* lenv;
  const cx<T>* renv;
  const cx<T>* vals;
  const int4* sub_rec;  // kSubRec / 4 int4 per subgroup (CoreLayout::sub_rec)
  const WorkItem* items;
  T* partials;
};

template <typename T, int R, int BYROW>
__device__ __attribute__((always_inline)) inline void inner_gram_body(const GramArgs<T>& A, int blk) {
  const cx<T>* lenv = A.lenv;
  const cx<T>* renv = A.renv;
  const cx<T>* vals = A.vals;
  const int4* sub_rec = A.sub_rec;
  const WorkItem* items = A.items;
  T* partials = A.partials;

  typedef InnerGeom<R> G;
  typedef typename Mfma<T>::acc_t acc_t;
  // A batch of 64 subgroups (one per lane) is staged through LDS in PH
  // phases of 64/PH rows: at r <= 6 two phases halve the LDS a wavefront
  // holds, so twice as many wavefronts fit on a CU
  constexpr int PH = (R <= 6 && sizeof(T) == 4) ? 2 : 1, RP = 64 / PH;
  __shared__ T As[RP * G::LDW];
  __shared__ T Bs[RP * G::LDW];
  const int lane = threadIdx.x;
  const int item = blk;
  const WorkItem it = items[item];
  acc_t acc[G::NB][G::NB];
#pragma unroll
  for (int x = 0; x < G::NB; ++x)
#pragma unroll
    for (int y = 0; y < G::NB; ++y) acc[x][y] = acc_t{T(0), T(0), T(0), T(0)};

  for (int base = it.sub0; base < it.sub1; base += 64) {
    const int s = base + lane;
    const bool live = s < it.sub1;
    // the subgroup's whole record in one round of loads (no offset first)
    int e0 = 0, cnt = 0, shared = 0;
    int id[kSubgroup];
#pragma unroll
    for (int q = 0; q < kSubgroup; ++q) id[q] = -1;
    if (live) {
      static_assert(kSubRec == 12 && kSubgroup == 8, "record layout");
      const int4* rp = sub_rec + (int64_t)s * (kSubRec / 4);
      const int4 h = rp[0], i0 = rp[1], i1 = rp[2];
      e0 = h.x;
      cnt = h.y;
      shared = h.z;
      id[0] = i0.x; id[1] = i0.y; id[2] = i0.z; id[3] = i0.w;
      id[4] = i1.x; id[5] = i1.y; id[6] = i1.z; id[7] = i1.w;
    }
    T a[G::W], b[G::W];
    subgroup_rows_ids<T, R, BYROW>(live, e0, e0 + cnt, shared, id, lenv, renv, vals, a, b);
#pragma unroll
    for (int ph = 0; ph < PH; ++ph) {
      if (lane / RP == ph) {
        T* arow = As + (lane % RP) * G::LDW;
        T* brow = Bs + (lane % RP) * G::LDW;
#pragma unroll
        for (int k = 0; k < G::W; ++k) {
          arow[k] = a[k];
          brow[k] = b[k];
        }
#pragma unroll
        for (int k = G::W; k < G::WP; ++k) {
          arow[k] = T(0);
          brow[k] = T(0);
        }
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < RP; kk += 4) {
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
  }
  T* out = partials + (int64_t)item * G::WP * G::WP;
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

template <typename T, int R, int BYROW>
__global__ __launch_bounds__(64) void inner_gram_kernel(GramArgs<T> A) {
  inner_gram_body<T, R, BYROW>(A, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <typename T, int R, int BYROW>
__global__ __launch_bounds__(64) void inner_gram_kernel_batched(const GramArgs<T>* tasks, const int32_t* block_off,
    int ntasks) {
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int t = find_task(block_off, ntasks, b);
  inner_gram_body<T, R, BYROW>(tasks[t], b - block_off[t]);
}


// BF16-input variant (precision BFC_C64_BF16GRAM): the same A/B rows as the
// FP32 kernel, multiplied on the BF16 matrix cores (16x16x32, FP32
// accumulation).  Each FP32 value x is split into three bf16 parts
// h = bf16(x), m = bf16(x - h), l = bf16(x - h - m) (round to nearest even;
// both differences are exact in FP32), so x = h + m + l to about 2^-27 of |x|,
// and the six products h h' + h m' + m h' + h l' + m m' + l h' give x x' to
// about 2^-26 relative (the dropped m l', l m', l l' are smaller): each
// product of two bf16 values is exact in FP32, so the Gram carries the
// rounding of its FP32 accumulation, as in the FP32 kernel, and takes the same
// regularization floor.  Rows are staged as FP32 values, coordinate-major, in
// two phases of 32 subgroups (one 32-deep k block of the instruction each):
// lane l reads the eight consecutive subgroups 8(l/16)..8(l/16)+7 of
// coordinate l%16 of a tile as two 16-byte loads and splits them in
// registers.  The output layout equals the FP32 instruction's, so the partial
// products keep their format.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
// Regularization floor of the FP32-accumulated Grams: the FP32 unit roundoff
// 2^-24 times the sqrt(256) growth of the sums that form them (at most 8
// entries per subgroup, then up to 128 subgroups per MFMA chain and per
// outer-fiber lane).  At 2^-24 itself the long-run sweeps drift along
// directions the data leave undetermined until the cores overflow (about 40
// sweeps on the Green's-function workloads); at 2^-20 they stay bounded.
constexpr double kF32RegFloor = 0x1p-20;
constexpr int kBf16IrSteps = 1;
constexpr int kBfLdk = 32 + 4;  // subgroups per staged coordinate row (one phase), padded

// Rounding level u of a problem's regularization floor: that of its Gram
// accumulation, raised to the configured lower bound.
inline double reg_floor_of(const Problem* P) {
  // the wide-rank kernels accumulate every Gram in FP64
  const double uk = (P->prec == BFC_C128 || P->r > kNarrowRank) ? 0.0 : kF32RegFloor;
  return uk > P->cfg.reg_floor ? uk : P->cfg.reg_floor;
}

// x = h + m + l, each part bf16 rounded to nearest even (see above).
__device__ __attribute__((always_inline)) inline void split_bf16x3(const floatx4& x0,
                                                                   const floatx4& x1,
                                                                   bf16x8& h, bf16x8& m,
                                                                   bf16x8& l) {
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const float x = t < 4 ? x0[t] : x1[t - 4];
    const __bf16 hh = (__bf16)x;
    const float r1 = x - (float)hh;
    const __bf16 mm = (__bf16)r1;
    const float r2 = r1 - (float)mm;
    h[t] = hh;
    m[t] = mm;
    l[t] = (__bf16)r2;
  }
}

template <int R, int BYROW>
__global__ __launch_bounds__(64) void inner_gram_bf16_kernel(
    const cx<float>* lenv, const int32_t* lidx, const cx<float>* renv, const int32_t* ridx,
    const cx<float>* vals, const int32_t* sub_off, const WorkItem* items, float* partials) {
  typedef InnerGeom<R> G;
  typedef Mfma<float>::acc_t acc_t;
  __shared__ __attribute__((aligned(16))) float At[G::WP * kBfLdk];
  __shared__ __attribute__((aligned(16))) float Bt[G::WP * kBfLdk];
  const int lane = threadIdx.x;
  const int item = xcd_swizzle(blockIdx.x, gridDim.x);
  const WorkItem it = items[item];
  acc_t acc[G::NB][G::NB];
#pragma unroll
  for (int x = 0; x < G::NB; ++x)
#pragma unroll
    for (int y = 0; y < G::NB; ++y) acc[x][y] = acc_t{0.f, 0.f, 0.f, 0.f};

  for (int base = it.sub0; base < it.sub1; base += 64) {
    const int s = base + lane;
    const bool live = s < it.sub1;
    int e0 = 0, e1 = 0;
    if (live) {
      e0 = sub_off[s];
      e1 = sub_off[s + 1];
    }
    float a[G::W], b[G::W];
    subgroup_rows<float, R, BYROW>(live, e0, e1, lenv, lidx, renv, ridx, vals, a, b);
#pragma unroll
    for (int ph = 0; ph < 2; ++ph) {
      if ((lane >> 5) == ph) {
        const int col = lane & 31;
#pragma unroll
        for (int k = 0; k < G::W; ++k) {
          At[k * kBfLdk + col] = a[k];
          Bt[k * kBfLdk + col] = b[k];
        }
#pragma unroll
        for (int k = G::W; k < G::WP; ++k) {
          At[k * kBfLdk + col] = 0.f;
          Bt[k * kBfLdk + col] = 0.f;
        }
      }
      __syncthreads();
      const int off = (lane & 15) * kBfLdk + 8 * (lane >> 4);
      bf16x8 yh[G::NB], ym[G::NB], yl[G::NB];
#pragma unroll
      for (int y = 0; y < G::NB; ++y) {
        const float* src = Bt + y * 16 * kBfLdk + off;
        split_bf16x3(*(const floatx4*)src, *(const floatx4*)(src + 4), yh[y], ym[y], yl[y]);
      }
#pragma unroll
      for (int x = 0; x < G::NB; ++x) {
        const float* src = At + x * 16 * kBfLdk + off;
        bf16x8 xh, xm, xl;
        split_bf16x3(*(const floatx4*)src, *(const floatx4*)(src + 4), xh, xm, xl);
#pragma unroll
        for (int y = 0; y < G::NB; ++y) {
          // the small products first
          acc_t c = acc[x][y];
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, ym[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xm, yh[y], c, 0, 0, 0);
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, ym[y], c, 0, 0, 0);
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh[y], c, 0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  float* out = partials + (int64_t)item * G::WP * G::WP;
#pragma unroll
  for (int x = 0; x < G::NB; ++x)
#pragma unroll
    for (int y = 0; y < G::NB; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = x * 16 + Mfma<float>::out_row(lane, v);
        const int col = y * 16 + (lane & 15);
        out[row * G::WP + col] = acc[x][y][v];
      }
}

// Residual vector of an inner core's slices at their current values,
// recomputed from the entries in the compute precision T (FP32 for the
// refinement of the BF16-Gram solves, T for the ADAM gradients, which are its
// negation): per work item, g = sum_e conj(a_e) (t_e - a_e . s0) over its
// subgroups, with s0 the slice just solved for (a_e = l (x) rho, so a_e . s0 =
// l^T S0 rho).  Row groups share l: v = l^T S0 once, then per entry
// res = t - v . rho and w += conj(rho) res, and g += conj(l) (x) w.  Column
// groups share rho: u = S0 rho, res = t - l . u, w += conj(l) res,
// g += w (x) conj(rho).  Output: ir_part[item][2 d] (re, im interleaved),
// the wavefront's lanes summed in a fixed order.  ZT: the targets are taken
// as zero, which gives -sum conj(a_e) (a_e . s0) (the Gram applied to s0).
template <typename T, int R, int BYROW, bool ZT = false>
__global__ __launch_bounds__(64) void inner_ir_kernel(
    const cx<T>* lenv, const int32_t* lidx, const cx<T>* renv, const int32_t* ridx,
    const cx<T>* vals, const int32_t* sub_off, const WorkItem* items, const cx<T>* slices,
    T* ir_part) {
  constexpr int D = R * R, LDR = 2 * D + 1;
  __shared__ T red[64 * LDR];
  __shared__ cx<T> S0[D];
  const int lane = threadIdx.x;
  const int item = xcd_swizzle(blockIdx.x, gridDim.x);
  const WorkItem it = items[item];
  for (int k = lane; k < D; k += 64) S0[k] = slices[(int64_t)it.tile * D + k];
  __syncthreads();
  T gx[D], gy[D];
#pragma unroll
  for (int k = 0; k < D; ++k) gx[k] = gy[k] = T(0);
  for (int base = it.sub0; base < it.sub1; base += 64) {
    const int s = base + lane;
    if (s >= it.sub1) continue;
    const int e0 = sub_off[s], e1 = sub_off[s + 1];
    cx<T> sh[R], m[R], w[R];
    if (BYROW)
      load_env<T, R>(lenv, lidx[e0], sh);
    else
      load_env<T, R>(renv, ridx[e0], sh);
#pragma unroll
    for (int k = 0; k < R; ++k) {
      m[k] = cx<T>{T(0), T(0)};
      w[k] = cx<T>{T(0), T(0)};
    }
    // BYROW: m_b = sum_a l_a S0[a][b]; else m_a = sum_b S0[a][b] rho_b
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) {
        if (BYROW)
          cfma(m[b], sh[a], S0[a * R + b]);
        else
          cfma(m[a], S0[a * R + b], sh[b]);
      }
    const int32_t* eidx = BYROW ? ridx : lidx;
    const cx<T>* esrc = BYROW ? renv : lenv;
    int id[kSubgroup];
#pragma unroll
    for (int q = 0; q < kSubgroup; ++q) id[q] = (e0 + q < e1) ? eidx[e0 + q] : -1;
#pragma unroll
    for (int g0 = 0; g0 < kSubgroup; g0 += kGatherGroup) {
      if (__ballot(e0 + g0 < e1) == 0) break;
      int gid[kGatherGroup], ent[kGatherGroup];
#pragma unroll
      for (int g = 0; g < kGatherGroup; ++g) {
        gid[g] = id[g0 + g];
        ent[g] = e0 + g0 + g;
      }
      cx<T> vv[kGatherGroup][R], tt[kGatherGroup];
      gather_group<T, R, kGatherGroup>(esrc, vals, gid, ent, vv, tt);
#pragma unroll
      for (int g = 0; g < kGatherGroup; ++g) {
        if (gid[g] < 0) continue;
        cx<T> x = {T(0), T(0)};
#pragma unroll
        for (int k = 0; k < R; ++k) cfma(x, m[k], vv[g][k]);
        const cx<T> res = ZT ? cx<T>{-x.x, -x.y} : cx<T>{tt[g].x - x.x, tt[g].y - x.y};
#pragma unroll
        for (int k = 0; k < R; ++k) cfma_conj(w[k], vv[g][k], res);  // w += conj(v) res
      }
    }
    // g[a*R+b] += conj(l_a) w_b (row groups) or w_a conj(rho_b) (column groups)
#pragma unroll
    for (int a = 0; a < R; ++a)
#pragma unroll
      for (int b = 0; b < R; ++b) {
        const cx<T> p = BYROW ? sh[a] : sh[b];
        const cx<T> q = BYROW ? w[b] : w[a];
        gx[a * R + b] += p.x * q.x + p.y * q.y;  // conj(p) q
        gy[a * R + b] += p.x * q.y - p.y * q.x;
      }
  }
#pragma unroll
  for (int k = 0; k < D; ++k) {
    red[lane * LDR + 2 * k] = gx[k];
    red[lane * LDR + 2 * k + 1] = gy[k];
  }
  __syncthreads();
  for (int k = lane; k < 2 * D; k += 64) {
    T acc = T(0);
    for (int l = 0; l < 64; ++l) acc += red[l * LDR + k];
    ir_part[(int64_t)item * 2 * D + k] = acc;
  }
}

// ---------------------------------------------------------------------------
// inner cores: per-slice sum of partials, FP64 Hermitian solve (one workgroup)
// ---------------------------------------------------------------------------
// The work items' partial products are summed in a fixed order, so results do
// not depend on scheduling.  K and the factor are row-major with an odd
// leading dimension.  LDS: the real partial sum S is only needed to assemble
// K and h, so the factor M reuses its space; K passes through registers (a
// retry of the regularization ladder sums the partial products again), so a
// slice holds one D x D complex array in LDS, not two.
template <int R>
struct SolveGeom {
  static constexpr int D = R * R;
  static constexpr int WP = InnerGeom<R>::WP;
  static constexpr int LD = (D % 2) ? D : D + 1;
  static constexpr int S_BYTES = WP * WP * 8;
  static constexpr int F_BYTES = (D + 1) * LD * 16;  // factor and its border row
  static constexpr int M_BYTES = (F_BYTES > S_BYTES ? F_BYTES : S_BYTES);
  static constexpr int NP = (D + kNb - 1) / kNb;  // diagonal blocks
};
constexpr int kSolveThreads = 256;

// One workgroup per slice: sum the slice's partial products (S), assemble the
// Hermitian system (K, h), factor K + lam I bordered by the right-hand side
// h + lam s_old (regularization ladder), back-substitute, write the slice.
// pass 0: the one solve of the FP64 / FP32-Gram modes.  pass 1: the first
// solve of the BF16-Gram mode, which also keeps the slice's regularization
// (ir_lam, negative when the slice is kept), its old values (ir_old) and the
// factor of K + lam I with its diagonal-block inverses (ir_fac).  pass 2: the
// refinement, (K + lam I) delta = g + lam (s_old - s0) (ridge: g - lam s0)
// with g the entries' residual vector (ir_part, per work item), solved with
// the kept factor by one forward and one back substitution (no partial sums,
// no factorization); the slice becomes s0 + delta.
template <typename T>
struct SolveArgs {
  cx<T>* slices;
  const T* partials;
  const int32_t* tile_items;
  double reg_rel;
  double reg_floor;
  int prox;
  int32_t* flags;
  int pass;
  double* ir_lam;
  cx<T>* ir_old;
  const float* ir_part;
  double2* ir_fac;  // per slice: the factor's D x LD rows, then the diagonal-block inverses
};

template <int R>
constexpr int solve_factor_elems() {
  return SolveGeom<R>::D * SolveGeom<R>::LD + SolveGeom<R>::NP * kNb * kNb;
}

template <typename T, int R>
__device__ __attribute__((always_inline)) inline void inner_solve_body(const SolveArgs<T>& A, int blk) {
  cx<T>* slices = A.slices;
  const T* partials = A.partials;
  const int32_t* tile_items = A.tile_items;
  double reg_rel = A.reg_rel;
  double reg_floor = A.reg_floor;
  int prox = A.prox;
  int32_t* flags = A.flags;
  int pass = A.pass;
  double* ir_lam = A.ir_lam;
  cx<T>* ir_old = A.ir_old;
  const float* ir_part = A.ir_part;

  typedef SolveGeom<R> G;
  constexpr int D = G::D, WP = G::WP, LD = G::LD, NT = kSolveThreads;
  __shared__ __attribute__((aligned(16))) unsigned char mbuf[G::M_BYTES];
  __shared__ double2 panel[(D + 1) * kPanelLd];
  __shared__ double2 dinv[G::NP * kNb * kNb];
  double* S = (double*)mbuf;
  double2* M = (double2*)mbuf;
  const int tid = threadIdx.x, lane = tid & 63;
  // same XCD-contiguous mapping as the Gram items, so the slice's partial
  // products are read from the L2 that holds them
  const int tile = blk;
  const int it0 = tile_items[tile], it1 = tile_items[tile + 1];
  if (it0 == it1) return;  // no observed entry in this slice: keep it
  // S (in mbuf) = the sum of the slice's partial products; run again by a
  // retry of the regularization ladder, since the factor overwrites S
  auto sum_partials = [&]() {
    // items outer, 16-byte vectors inner, two items in flight per pass
    typedef typename std::conditional<sizeof(T) == 4, float4, double2>::type V;
    constexpr int VE = 16 / sizeof(T);
    constexpr int NV = WP * WP / VE;  // WP is a multiple of 16
    constexpr int PV = (NV + NT - 1) / NT;
    double acc[PV][VE];
#pragma unroll
    for (int q = 0; q < PV; ++q)
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[q][e] = 0.0;
    auto add = [&](const V& v, int q) {
      const T* t = (const T*)&v;
#pragma unroll
      for (int e = 0; e < VE; ++e) acc[q][e] += (double)t[e];
    };
    int it = it0;
    for (; it + 1 < it1; it += 2) {
      const V* s0 = (const V*)(partials + (int64_t)it * WP * WP);
      const V* s1 = s0 + NV;
      V v0[PV], v1[PV];
#pragma unroll
      for (int q = 0; q < PV; ++q) {
        const int k = tid + NT * q;
        if (k < NV) {
          v0[q] = s0[k];
          v1[q] = s1[k];
        }
      }
#pragma unroll
      for (int q = 0; q < PV; ++q)
        if (tid + NT * q < NV) {
          add(v0[q], q);
          add(v1[q], q);
        }
    }
    if (it < it1) {
      const V* s0 = (const V*)(partials + (int64_t)it * WP * WP);
#pragma unroll
      for (int q = 0; q < PV; ++q)
        if (tid + NT * q < NV) add(s0[tid + NT * q], q);
    }
#pragma unroll
    for (int q = 0; q < PV; ++q) {
      const int k = tid + NT * q;
      if (k < NV)
#pragma unroll
        for (int e = 0; e < VE; ++e) S[k * VE + e] = acc[q][e];
    }
  };
  sum_partials();
  __syncthreads();
  double2 h = make_double2(0.0, 0.0);
  if (tid < D) h = inner_h<R>(S, WP, tid);
  double tr = 0.0;
  for (int i = 0; i < D; ++i) tr += inner_K<R>(S, WP, i, i).x;  // same order in every thread
  const double tau = tr / D;
  const double unit = fmax(reg_floor, 0x1p-53);
  double lam = fmax(reg_rel, D * reg_floor) * tau;
  cx<T>* slice = slices + (int64_t)tile * D;
  double2 old = make_double2(0.0, 0.0);
  if (prox && tid < D) old = make_double2((double)slice[tid].x, (double)slice[tid].y);
  double2 rhs = h;  // right-hand side of the bordered factorization
  if (pass == 1 && tid < D) ir_old[(int64_t)tile * D + tid] = slice[tid];
  // K = inner_K(S) is assembled into registers (entry k = tid + NT q of the
  // D x LD layout) and written, regularized, over S as the factor M
  constexpr int PK = (D * LD + NT - 1) / NT;
  bool ok = false;
  int attempt = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, D * unit * tau);
      __syncthreads();  // the failed factor is dead
      sum_partials();
      __syncthreads();
    }
    double2 kreg[PK];
#pragma unroll
    for (int q = 0; q < PK; ++q) {
      const int k = tid + NT * q;
      kreg[q] = make_double2(0.0, 0.0);
      if (k < D * LD && k % LD < D) kreg[q] = inner_K<R>(S, WP, k / LD, k % LD);
    }
    __syncthreads();  // S is dead from here on; M takes its place
#pragma unroll
    for (int q = 0; q < PK; ++q) {
      const int k = tid + NT * q;
      if (k < D * LD) {
        double2 v = kreg[q];
        if (k % LD == k / LD) v.x += lam;
        M[k] = v;
      }
    }
    if (tid < D) {  // border row: conj(right-hand side)
      double2 b = rhs;
      if (prox) {
        b.x += lam * old.x;
        b.y += lam * old.y;
      }
      M[D * LD + tid] = make_double2(b.x, -b.y);
    }
    __syncthreads();
    ok = wg_cholesky<NT>(M, D, LD, panel, dinv, tid);
    if (ok) break;
  }
  if (!ok) {
    if (tid == 0) {
      atomicAdd(flags, 1);
      if (pass == 1) ir_lam[tile] = -1.0;
    }
    return;
  }
  if (tid == 0) {
    if (attempt > 0) atomicAdd(flags + 1, 1);
    if (pass == 1) ir_lam[tile] = lam;
  }
  if (pass == 1) {  // keep the factor for the refinement pass
    double2* F = A.ir_fac + (int64_t)tile * solve_factor_elems<R>();
    for (int k = tid; k < D * LD; k += NT) F[k] = M[k];
    for (int k = tid; k < G::NP * kNb * kNb; k += NT) F[D * LD + k] = dinv[k];
  }
  if (tid >= 64) return;  // one wavefront solves; no barriers below
  double2 y = make_double2(0.0, 0.0);
  if (lane < D) {
    const double2 t = M[D * LD + lane];
    y = make_double2(t.x, -t.y);
  }
  wave_back_solve(M, dinv, D, LD, y, lane);
  if (lane < D) slice[lane] = {T(y.x), T(y.y)};
}

// Refinement of the BF16-Gram mode (the second pass): (K + lam I) delta =
// g + lam (s_old - s0) (ridge: g - lam s0), g the entries' residual vector
// (ir_part, per work item, summed in a fixed order), solved with the factor
// the first pass kept (ir_fac) by one forward and one back substitution; the
// slice becomes s0 + delta.  A slice the first pass kept (ir_lam < 0) or
// without entries is left alone.
template <typename T, int R>
__global__ __launch_bounds__(kSolveThreads) void inner_refine_kernel(SolveArgs<T> A) {
  typedef SolveGeom<R> G;
  constexpr int D = G::D, LD = G::LD, NT = kSolveThreads;
  __shared__ double2 Mf[D * LD];
  __shared__ double2 dinv[G::NP * kNb * kNb];
  const int tid = threadIdx.x, lane = tid & 63;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int it0 = A.tile_items[tile], it1 = A.tile_items[tile + 1];
  if (it0 == it1) return;
  const double lam = A.ir_lam[tile];
  if (!(lam >= 0.0)) return;
  const double2* F = A.ir_fac + (int64_t)tile * solve_factor_elems<R>();
  for (int k = tid; k < D * LD; k += NT) Mf[k] = F[k];
  for (int k = tid; k < G::NP * kNb * kNb; k += NT) dinv[k] = F[D * LD + k];
  cx<T>* slice = A.slices + (int64_t)tile * D;
  double2 s0 = make_double2(0.0, 0.0), rhs = make_double2(0.0, 0.0);
  if (tid < D) {
    s0 = make_double2((double)slice[tid].x, (double)slice[tid].y);
    double gx = 0.0, gy = 0.0;
    for (int it = it0; it < it1; ++it) {
      gx += (double)A.ir_part[(int64_t)it * 2 * D + 2 * tid];
      gy += (double)A.ir_part[(int64_t)it * 2 * D + 2 * tid + 1];
    }
    const cx<T> so = A.ir_old[(int64_t)tile * D + tid];
    const double ox = A.prox ? (double)so.x : 0.0, oy = A.prox ? (double)so.y : 0.0;
    rhs = make_double2(gx + lam * (ox - s0.x), gy + lam * (oy - s0.y));
  }
  __syncthreads();
  if (tid >= 64) return;  // one wavefront solves; no barriers below
  wave_fwd_solve(Mf, dinv, D, LD, rhs, lane);
  wave_back_solve(Mf, dinv, D, LD, rhs, lane);
  if (lane < D) slice[lane] = {T(s0.x + rhs.x), T(s0.y + rhs.y)};
}

template <typename T, int R>
__global__ __launch_bounds__(kSolveThreads) __attribute__((amdgpu_waves_per_eu(2))) void inner_solve_kernel(SolveArgs<T> A) {
  inner_solve_body<T, R>(A, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <typename T, int R>
__global__ __launch_bounds__(kSolveThreads) __attribute__((amdgpu_waves_per_eu(2))) void inner_solve_kernel_batched(const SolveArgs<T>* tasks, const int32_t* block_off,
    int ntasks) {
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int t = find_task(block_off, ntasks, b);
  inner_solve_body<T, R>(tasks[t], b - block_off[t]);
}


// ---------------------------------------------------------------------------
// environment-trie levels
// ---------------------------------------------------------------------------

// Right level p (0 <= p < L): node (u, j) = Z^(p+2)[k] * parent, where
// k = ((ib >> p) << (p+1)) | (jb >> (L-p-1)) with ib >> p = u, and the parent
// is node (u >> 1, j) of level p+1 (a row of Z^(L+2) when p = L-1).
// Left level p (2 <= p <= L+1): node (w, i) = parent * Z^p[k], where
// k = ((ib >> (p-2)) << (p-1)) | (jb >> (L-p+1)) with jb >> (L-p+1) = w, and
// the parent is node (w >> 1, i) of level p-1 (a row of Z^1 when p = 2).
template <typename T>
struct EnvArgs {
  const cx<T>* cores;
  int64_t n;
  int L, c, p, count;
  const int32_t* node_a;  // u (right) or w (left)
  const int32_t* node_b;  // column j (right) or row i (left)
  const int32_t* parent;
  const cx<T>* parent_vec;
  cx<T>* out;
};

// Nodes are sorted so that neighbours mostly multiply the same core slice.
// When every node of a wavefront does, the wavefront stages that slice in LDS
// once (36 or 64 values) instead of each lane streaming it through L1.
template <typename T, int R, int RIGHT>
__device__ __attribute__((always_inline)) inline void env_level_body(const EnvArgs<T>& a,
                                                                     int blk) {
  __shared__ cx<T> zs[4][R * R];  // one slice per wavefront of the 256-thread block
  const int k = blk * 256 + (int)threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool live = k < a.count;
  // lane 0 holds the wavefront's first node: no live lane without it
  if (__builtin_amdgcn_readfirstlane(live ? 1 : 0) == 0) return;
  const int L = a.L, p = a.p;
  uint32_t key = 0, na = 0, nb = 0;
  cx<T> v[R];
  if (live) {
    na = (uint32_t)a.node_a[k];
    nb = (uint32_t)a.node_b[k];
    key = RIGHT ? (na << (p + 1)) | ((nb / (uint32_t)a.c) >> (L - p - 1))
                : (((nb / (uint32_t)a.c) >> (p - 2)) << (p - 1)) | na;
    load_env<T, R>(a.parent_vec, a.parent[k], v);
  }
  const cx<T>* Zcore = a.cores + inner_off(a.n, L, R, RIGHT ? p + 1 : p - 1);
  const uint32_t k0 = __builtin_amdgcn_readfirstlane(key);
  const bool uniform = __ballot(live && key != k0) == 0;
  if (uniform) {
    const cx<T>* src = Zcore + (int64_t)k0 * R * R;
    for (int e = lane; e < R * R; e += 64) zs[wave][e] = src[e];
    wave_sync();
    if (RIGHT)
      mat_vec<T, R>(zs[wave], v);
    else
      vec_mat<T, R>(v, zs[wave]);
  } else {
    const cx<T>* Z = Zcore + (int64_t)key * R * R;
    if (RIGHT)
      mat_vec<T, R>(Z, v);
    else
      vec_mat<T, R>(v, Z);
  }
  if (!live) return;
  cx<T>* o = a.out + (int64_t)k * R;
#pragma unroll
  for (int q = 0; q < R; ++q) o[q] = v[q];
}

template <typename T, int R, int RIGHT>
__global__ __launch_bounds__(256) void env_level_kernel(EnvArgs<T> a) {
  env_level_body<T, R, RIGHT>(a, xcd_swizzle(blockIdx.x, gridDim.x));
}

template <typename T, int R, int RIGHT>
__global__ __launch_bounds__(256) void env_level_batched(const EnvArgs<T>* tasks,
                                                         const int32_t* block_off, int ntasks) {
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  const int t = find_task(block_off, ntasks, b);
  env_level_body<T, R, RIGHT>(tasks[t], b - block_off[t]);
}

// The top right levels hold few nodes, and one launch per level costs more
// than the arithmetic.  Each of their nodes is computed here from scratch,
// as the chain Z^(p+2)[k] ... Z^(L+1)[k] Z^(L+2)[j] (the right environment of
// Section 5.1.1), all levels in one launch.  The products are taken in the
// same order as level by level, so the vectors are bit-identical.  Every
// level starts at a multiple of 64 threads, so a wavefront walks one chain
// length, and a slice that all its nodes use is staged in LDS once.
constexpr int kDirectLevels = 4;
template <typename T>
struct DirectEnvArgs {
  const cx<T>* cores;
  int64_t n;
  int L, c, nlev;
  int p[kDirectLevels];
  int count[kDirectLevels];
  int off[kDirectLevels + 1];  // first thread of each level, multiples of 64
  const int32_t* node_a[kDirectLevels];
  const int32_t* node_b[kDirectLevels];
  cx<T>* out[kDirectLevels];
};

template <typename T, int R>
__global__ __launch_bounds__(256) void env_right_direct_kernel(DirectEnvArgs<T> a) {
  __shared__ cx<T> zs[4][R * R];
  const int k = (int)(blockIdx.x * 256 + threadIdx.x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (__builtin_amdgcn_readfirstlane(k) >= a.off[a.nlev]) return;  // the whole wavefront
  int l = 0;
  while (l + 1 < a.nlev && k >= a.off[l + 1]) ++l;
  l = __builtin_amdgcn_readfirstlane(l);
  const int i = k - a.off[l];
  const bool live = i < a.count[l];
  const int p = a.p[l], L = a.L;
  uint32_t u = 0, j = 0;
  if (live) {
    u = (uint32_t)a.node_a[l][i];
    j = (uint32_t)a.node_b[l][i];
  }
  const uint32_t ib = u << p, jb = j / (uint32_t)a.c;  // the chain reads ib only as ib >> p
  cx<T> w[R];
  load_env<T, R>(a.cores + last_off(a.n, L, R), (int)j, w);
  for (int m = L; m > p; --m) {
    const cx<T>* Zc = a.cores + inner_off(a.n, L, R, m);
    const uint32_t key = slice_key(ib, jb, L, m);
    const uint32_t kf = __builtin_amdgcn_readfirstlane(key);
    if (__ballot(live && key != kf) == 0) {
      const cx<T>* src = Zc + (int64_t)kf * R * R;
      for (int e = lane; e < R * R; e += 64) zs[wave][e] = src[e];
      wave_sync();
      mat_vec<T, R>(zs[wave], w);
      wave_sync();  // every lane has read the slice before the next one lands
    } else {
      mat_vec<T, R>(Zc + (int64_t)key * R * R, w);
    }
  }
  if (!live) return;
  cx<T>* o = a.out[l] + (int64_t)i * R;
#pragma unroll
  for (int q = 0; q < R; ++q) o[q] = w[q];
}

// Residual on the observed set from the cached left environments of the last
// core: x = l_(L+1) . Z^(L+2)[j].  Entries in the last core's order.
template <typename T>
struct ResObsArgs {
  const cx<T>* lenv;
  const int32_t* lidx;
  const cx<T>* zlast;
  const int32_t* cols;
  const cx<T>* vals;
  int64_t m;
  int64_t per_block;
  double* partial;
};

template <typename T, int R>
__device__ __attribute__((always_inline)) inline void residual_observed_body(const ResObsArgs<T>& A, int blk) {
  const cx<T>* lenv = A.lenv;
  const int32_t* lidx = A.lidx;
  const cx<T>* zlast = A.zlast;
  const int32_t* cols = A.cols;
  const cx<T>* vals = A.vals;
  int64_t m = A.m;
  int64_t per_block = A.per_block;
  double* partial = A.partial;

  __shared__ double s0[kResThreads], s1[kResThreads];
  double a0 = 0.0, a1 = 0.0;
  const int64_t beg = (int64_t)blk * per_block;
  const int64_t end = beg + per_block < m ? beg + per_block : m;
  for (int64_t e = beg + threadIdx.x; e < end; e += kResThreads) {
    cx<T> v[R], z[R];
    load_env<T, R>(lenv, lidx[e], v);
    load_env<T, R>(zlast, cols[e], z);
    cx<T> x = {T(0), T(0)};
#pragma unroll
    for (int a = 0; a < R; ++a) cfma(x, v[a], z[a]);
    const cx<T> t = vals[e];
    const double dx = (double)t.x - (double)x.x, dy = (double)t.y - (double)x.y;
    a0 += dx * dx + dy * dy;
    a1 += (double)t.x * (double)t.x + (double)t.y * (double)t.y;
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
    partial[2 * blk] = s0[0];
    partial[2 * blk + 1] = s1[0];
  }
}

template <typename T, int R>
__global__ __launch_bounds__(kResThreads) void residual_observed_kernel(ResObsArgs<T> A) {
  residual_observed_body<T, R>(A, (int)blockIdx.x);
}

template <typename T, int R>
__global__ __launch_bounds__(kResThreads) void residual_observed_kernel_batched(const ResObsArgs<T>* tasks, const int32_t* block_off,
    int ntasks) {
  const int b = (int)blockIdx.x;
  const int t = find_task(block_off, ntasks, b);
  residual_observed_body<T, R>(tasks[t], b - block_off[t]);
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
// Right level p depends on cores p+1..L+1, left level p on cores 0..p-1.
// Arguments of the launch computing right (right = 1) or left level q.
template <typename T, int R>
EnvArgs<T> env_args(const Problem* P, int q, int right) {
  const int L = P->L;
  const cx<T>* cores = (const cx<T>*)P->cores;
  const EnvLevel& E = right ? P->rlev[q] : P->llev[q];
  EnvArgs<T> a;
  a.cores = cores;
  a.n = P->n;
  a.L = L;
  a.c = P->c;
  a.p = q;
  a.count = E.count;
  a.node_a = E.node_a;
  a.node_b = E.node_b;
  a.parent = E.parent;
  if (right)
    a.parent_vec = (q == L - 1) ? cores + last_off(P->n, L, R) : (const cx<T>*)P->rlev[q + 1].vec;
  else
    a.parent_vec = (q == 2) ? cores : (const cx<T>*)P->llev[q - 1].vec;
  a.out = (cx<T>*)E.vec;
  return a;
}

template <typename T, int R>
bfc_status ensure_right(Problem* P, int p, hipStream_t st) {
  const int L = P->L;
  if (p >= L) return BFC_OK;  // the right environment of core L is Z^(L+2) itself
  int top = -1;
  for (int q = L - 1; q >= p; --q)
    if (!P->rlev[q].valid) {
      top = q;
      break;
    }
  if (top < 0) return BFC_OK;
  // levels L-1 .. L-kDirectLevels from scratch in one launch, the rest level
  // by level from their parents
  int q = top;
  {
    DirectEnvArgs<T> d;
    d.cores = (const cx<T>*)P->cores;
    d.n = P->n;
    d.L = L;
    d.c = P->c;
    d.nlev = 0;
    d.off[0] = 0;
    for (; q >= p && q >= L - kDirectLevels; --q) {
      EnvLevel& E = P->rlev[q];
      E.valid = true;
      if (E.count <= 0) continue;
      d.p[d.nlev] = q;
      d.count[d.nlev] = E.count;
      d.node_a[d.nlev] = E.node_a;
      d.node_b[d.nlev] = E.node_b;
      d.out[d.nlev] = (cx<T>*)E.vec;
      d.off[d.nlev + 1] = d.off[d.nlev] + (E.count + 63) / 64 * 64;
      ++d.nlev;
    }
    if (d.nlev > 0) {
      env_right_direct_kernel<T, R><<<grid_for(d.off[d.nlev]), 256, 0, st>>>(d);
      BFC_HIP_TRY(hipGetLastError());
    }
  }
  for (; q >= p; --q) {
    EnvLevel& E = P->rlev[q];
    if (E.count > 0)
      env_level_kernel<T, R, 1><<<grid_for(E.count), 256, 0, st>>>(env_args<T, R>(P, q, 1));
    BFC_HIP_TRY(hipGetLastError());
    E.valid = true;
  }
  return BFC_OK;
}

template <typename T, int R>
bfc_status ensure_left(Problem* P, int p, hipStream_t st) {
  const int L = P->L;
  if (p <= 1) return BFC_OK;  // the left environment of core 1 is Z^1 itself
  int low = -1;
  for (int q = 2; q <= p; ++q)
    if (!P->llev[q].valid) {
      low = q;
      break;
    }
  if (low < 0) return BFC_OK;
  for (int q = low; q <= p; ++q) {
    EnvLevel& E = P->llev[q];
    if (E.count > 0)
      env_level_kernel<T, R, 0><<<grid_for(E.count), 256, 0, st>>>(env_args<T, R>(P, q, 0));
    BFC_HIP_TRY(hipGetLastError());
    E.valid = true;
  }
  return BFC_OK;
}

template <typename T, int R>
bfc_status sweep_core_wide(Problem* P, int p, hipStream_t st) {
  cx<T>* cores = (cx<T>*)P->cores;
  const CoreLayout& C = P->lay[p];
  const int L = P->L;
  const double reg = P->cfg.reg_rel;
  const double floor_ = reg_floor_of(P);
  const int prox = P->cfg.reg_mode == BFC_REG_PROXIMAL ? 1 : 0;
  {
    ProfScope ps(&P->prof, KIND_ENV, st);
    BFC_TRY(ensure_right<T, R>(P, p, st));
    BFC_TRY(ensure_left<T, R>(P, p, st));
  }
  const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R)
                               : (p <= L - 1 ? (const cx<T>*)P->rlev[p].vec : nullptr);
  const int32_t* ridx = (p == L) ? C.cols : C.rnode;
  const cx<T>* lenv = (p == 1) ? cores : (p >= 2 ? (const cx<T>*)P->llev[p].vec : nullptr);
  const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
  if (p == 0 || p == L + 1) {
    cx<T>* fibers = cores + (p == 0 ? 0 : last_off(P->n, L, R));
    ProfScope ps(&P->prof, KIND_OUTER, st);
    BFC_TRY(launch_outer_wide<T, R>(
        WideOuterArgs<T>{fibers, p == 0 ? renv : lenv, p == 0 ? ridx : lidx,
                         (const cx<T>*)C.vals, C.blk_off, C.nblocks, reg, floor_, prox, P->flags},
        st));
  } else if (C.nitems > 0) {
    ProfScope ps(&P->prof, KIND_INNER_GRAM, st);
    const WideArgs<T> a{cores + inner_off(P->n, L, R, p), lenv, lidx, renv, ridx,
                        (const cx<T>*)C.vals, C.sub_off, C.items, C.tile_items,
                        (unsigned char*)P->partials, reg, floor_, prox, P->flags};
    BFC_TRY(launch_inner_wide<T, R>(a, C.nblocks, C.group_by_row, st));
  }
  P->fused_res_valid = false;
  for (int q = 0; q < p && q < L; ++q) P->rlev[q].valid = false;
  for (int q = p + 1; q <= L + 1; ++q)
    if (q >= 2) P->llev[q].valid = false;
  return BFC_OK;
}

template <typename T, int R>
bfc_status sweep_core_t(Problem* P, int p, hipStream_t st) {
  cx<T>* cores = (cx<T>*)P->cores;
  const CoreLayout& C = P->lay[p];
  const double reg = P->cfg.reg_rel;
  // keep lam above the rounding level of the Gram: none for FP64, the unit
  // roundoff of FP32 accumulation, or that of the bf16 inputs
  const int L = P->L;
  const double floor_ = reg_floor_of(P);
  const int prox = P->cfg.reg_mode == BFC_REG_PROXIMAL ? 1 : 0;
  // the outer cores take their environments from the level above the
  // outermost one when they can (up_node), which is then never built
  const bool up = (p == 0 || p == L + 1) && C.up_node != nullptr;
  {
    ProfScope ps(&P->prof, KIND_ENV, st);
    BFC_TRY(ensure_right<T, R>(P, up && p == 0 ? 1 : p, st));
    BFC_TRY(ensure_left<T, R>(P, up && p == L + 1 ? L : p, st));
  }
  // environment sources of core p: cached level, or a row of Z^1 / Z^(L+2)
  const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R)
                               : (p <= L - 1 ? (const cx<T>*)P->rlev[p].vec : nullptr);
  const int32_t* ridx = (p == L) ? C.cols : C.rnode;
  const cx<T>* lenv = (p == 1) ? cores : (p >= 2 ? (const cx<T>*)P->llev[p].vec : nullptr);
  const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
  if (p == 0 || p == L + 1) {
    cx<T>* fibers = cores + (p == 0 ? 0 : last_off(P->n, L, R));
    const cx<T>* env = p == 0 ? renv : lenv;
    const int32_t* idx = p == 0 ? ridx : lidx;
    {
      ProfScope ps(&P->prof, KIND_OUTER, st);
      const unsigned grid = (unsigned)(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
      // the last core's update also leaves the train residual's per-fiber norms
      OuterArgs<T> oa{fibers, env, idx, (const cx<T>*)C.vals, C.blk_off, C.nblocks, reg, floor_,
                      prox, P->flags, p == L + 1 ? P->fused_res : nullptr, nullptr, L, P->c};
      if (!up) {
        outer_update_kernel<T, R, 0><<<grid, kOuterThreads, 0, st>>>(oa);
      } else if (p == 0) {
        oa.env = (const cx<T>*)P->rlev[1].vec;
        oa.env_idx = C.up_node;
        oa.zsl = cores + inner_off(P->n, L, R, 1);
        outer_update_kernel<T, R, 1><<<grid, kOuterThreads, 0, st>>>(oa);
      } else {
        oa.env = (const cx<T>*)P->llev[L].vec;
        oa.env_idx = C.up_node;
        oa.zsl = cores + inner_off(P->n, L, R, L);
        outer_update_kernel<T, R, 2><<<grid, kOuterThreads, 0, st>>>(oa);
      }
    }
    BFC_HIP_TRY(hipGetLastError());
  } else {
    const bool bf16 = P->prec == BFC_C64_BF16GRAM;
    if (C.nitems > 0) {
      ProfScope ps(&P->prof, KIND_INNER_GRAM, st);
      if constexpr (std::is_same<T, float>::value) {
        if (bf16) {
          if (C.group_by_row)
            inner_gram_bf16_kernel<R, 1><<<C.nitems, 64, 0, st>>>(
                lenv, lidx, renv, ridx, (const cx<float>*)C.vals, C.sub_off, C.items,
                (float*)P->partials);
          else
            inner_gram_bf16_kernel<R, 0><<<C.nitems, 64, 0, st>>>(
                lenv, lidx, renv, ridx, (const cx<float>*)C.vals, C.sub_off, C.items,
                (float*)P->partials);
        }
      }
      if (!bf16) {
        if (C.group_by_row)
          inner_gram_kernel<T, R, 1><<<C.nitems, 64, 0, st>>>(GramArgs<T>{
              lenv, renv, (const cx<T>*)C.vals, (const int4*)C.sub_rec, C.items, (T*)P->partials});
        else
          inner_gram_kernel<T, R, 0><<<C.nitems, 64, 0, st>>>(GramArgs<T>{
              lenv, renv, (const cx<T>*)C.vals, (const int4*)C.sub_rec, C.items, (T*)P->partials});
      }
      BFC_HIP_TRY(hipGetLastError());
    }
    cx<T>* slices = cores + inner_off(P->n, L, R, p);
    {
      ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
      inner_solve_kernel<T, R><<<C.nblocks, kSolveThreads, 0, st>>>(SolveArgs<T>{
          slices, (const T*)P->partials, C.tile_items, reg, floor_, prox, P->flags, bf16 ? 1 : 0,
          P->ir_lam, (cx<T>*)P->ir_old, (const float*)P->ir_part, (double2*)P->ir_fac});
    }
    BFC_HIP_TRY(hipGetLastError());
    if constexpr (std::is_same<T, float>::value) {
      for (int step = 0; bf16 && C.nitems > 0 && step < kBf16IrSteps; ++step) {
        {
          ProfScope ps(&P->prof, KIND_INNER_IR, st);
          if (C.group_by_row)
            inner_ir_kernel<float, R, 1><<<C.nitems, 64, 0, st>>>(
                lenv, lidx, renv, ridx, (const cx<float>*)C.vals, C.sub_off, C.items, slices,
                (float*)P->ir_part);
          else
            inner_ir_kernel<float, R, 0><<<C.nitems, 64, 0, st>>>(
                lenv, lidx, renv, ridx, (const cx<float>*)C.vals, C.sub_off, C.items, slices,
                (float*)P->ir_part);
        }
        BFC_HIP_TRY(hipGetLastError());
        {
          ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
          inner_refine_kernel<T, R><<<C.nblocks, kSolveThreads, 0, st>>>(SolveArgs<T>{
              slices, (const T*)P->partials, C.tile_items, reg, floor_, prox, P->flags, 2,
              P->ir_lam, (cx<T>*)P->ir_old, (const float*)P->ir_part, (double2*)P->ir_fac});
        }
        BFC_HIP_TRY(hipGetLastError());
      }
    }
  }
  P->fused_res_valid = (p == L + 1);
  // core p changed: right levels below it and left levels above it are stale
  for (int q = 0; q < p && q < L; ++q) P->rlev[q].valid = false;
  for (int q = p + 1; q <= L + 1; ++q)
    if (q >= 2) P->llev[q].valid = false;
  return BFC_OK;
}

// ---------------------------------------------------------------------------
// ADAM for butterfly completion (Sec. 5.1.2, Alg. "ADAM for Butterfly
// Completion" and Alg. "ADAM_Update"): per core, the gradient
// g = sum_e conj(a_e) (x_e - t_e) of phi at the current cores (the Wirtinger
// gradient; the printed (x - t) v is its real-data form) from the same
// environments as the ALS update, then one ADAM step on every parameter of
// the core: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) |g|^2,
// s <- s - alpha m_hat / (sqrt(v_hat) + sigma).  The step itself is FP64.
// ---------------------------------------------------------------------------
struct AdamArgs {
  double alpha, b1, b2, sigma;
  double c1, c2;  // 1 - b1^t, 1 - b2^t
};

template <typename T>
__device__ inline void adam_step(cx<T>& s, cx<T>& m, T& v, double gx, double gy,
                                 const AdamArgs& a) {
  const double mx = a.b1 * (double)m.x + (1.0 - a.b1) * gx;
  const double my = a.b1 * (double)m.y + (1.0 - a.b1) * gy;
  const double vv = a.b2 * (double)v + (1.0 - a.b2) * (gx * gx + gy * gy);
  const double den = sqrt(vv / a.c2) + a.sigma;
  const double step = a.alpha / (a.c1 * den);
  s = cx<T>{T((double)s.x - step * mx), T((double)s.y - step * my)};
  m = cx<T>{T(mx), T(my)};
  v = T(vv);
}

// Outer core: 16 lanes per fiber sum conj(a_e) (x_e - t_e) over the fiber's
// entries (x_e = z . a_e with z the fiber's current value), reduce over the
// row of 16 lanes, and lane k < R steps element k.
template <typename T, int R>
__global__ __launch_bounds__(kOuterThreads) void outer_adam_kernel(
    cx<T>* fibers, const cx<T>* env, const int32_t* env_idx, const cx<T>* vals,
    const int32_t* blk_off, int nblocks, cx<T>* mom, T* vel, AdamArgs a) {
  const int sub = threadIdx.x & 15;
  const int b = (int)((blockIdx.x * kOuterThreads + threadIdx.x) >> 4);
  int e0 = 0, e1 = 0;
  if (b < nblocks) {
    e0 = blk_off[b];
    e1 = blk_off[b + 1];
  }
  cx<T> z[R];
#pragma unroll
  for (int k = 0; k < R; ++k)
    z[k] = b < nblocks ? fibers[(int64_t)b * R + k] : cx<T>{T(0), T(0)};
  T gx[R], gy[R];
#pragma unroll
  for (int k = 0; k < R; ++k) gx[k] = gy[k] = T(0);
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
    }
    cx<T> v[4][R], t[4];
    gather_group<T, R, 4>(env, vals, id, ent, v, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      cx<T> x = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < R; ++k) cfma(x, z[k], v[q][k]);
      const cx<T> res = {x.x - t[q].x, x.y - t[q].y};
#pragma unroll
      for (int k = 0; k < R; ++k) {  // g += conj(a) res
        cx<T> h = {gx[k], gy[k]};
        cfma_conj(h, v[q][k], res);
        gx[k] = h.x;
        gy[k] = h.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    gx[k] = row16_sum(gx[k]);
    gy[k] = row16_sum(gy[k]);
  }
  if (b >= nblocks || sub >= R) return;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k == sub) {
      sx = (double)gx[k];
      sy = (double)gy[k];
    }
  const int64_t o = (int64_t)b * R + sub;
  cx<T> sv = fibers[o], mv = mom[o];
  T vv = vel[o];
  adam_step(sv, mv, vv, sx, sy, a);
  fibers[o] = sv;
  mom[o] = mv;
  vel[o] = vv;
}

// Inner core: the slice's work items' residual vectors (sum conj(a)(t - x),
// the negated gradient) summed in a fixed order, then one ADAM step per
// element (thread k of the slice's wavefront).
template <typename T, int R>
__global__ __launch_bounds__(64) void inner_adam_kernel(cx<T>* slices, const T* part,
                                                        const int32_t* tile_items, cx<T>* mom,
                                                        T* vel, AdamArgs a) {
  constexpr int D = R * R;
  const int tile = blockIdx.x, k = threadIdx.x;
  if (k >= D) return;
  const int it0 = tile_items[tile], it1 = tile_items[tile + 1];
  double gx = 0.0, gy = 0.0;
  for (int it = it0; it < it1; ++it) {
    gx -= (double)part[(int64_t)it * 2 * D + 2 * k];
    gy -= (double)part[(int64_t)it * 2 * D + 2 * k + 1];
  }
  const int64_t o = (int64_t)tile * D + k;
  cx<T> sv = slices[o], mv = mom[o];
  T vv = vel[o];
  adam_step(sv, mv, vv, gx, gy, a);
  slices[o] = sv;
  mom[o] = mv;
  vel[o] = vv;
}

template <typename T, int R>
bfc_status adam_core_t(Problem* P, int p, const AdamArgs& a, hipStream_t st) {
  cx<T>* cores = (cx<T>*)P->cores;
  const CoreLayout& C = P->lay[p];
  const int L = P->L;
  {
    ProfScope ps(&P->prof, KIND_ENV, st);
    BFC_TRY(ensure_right<T, R>(P, p, st));
    BFC_TRY(ensure_left<T, R>(P, p, st));
  }
  const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R)
                               : (p <= L - 1 ? (const cx<T>*)P->rlev[p].vec : nullptr);
  const int32_t* ridx = (p == L) ? C.cols : C.rnode;
  const cx<T>* lenv = (p == 1) ? cores : (p >= 2 ? (const cx<T>*)P->llev[p].vec : nullptr);
  const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
  const int64_t off = p == 0 ? 0 : (p == L + 1 ? last_off(P->n, L, R) : inner_off(P->n, L, R, p));
  cx<T>* mom = (cx<T>*)P->adam_m + off;
  T* vel = (T*)P->adam_v + off;
  if (p == 0 || p == L + 1) {
    cx<T>* fibers = cores + off;
    const unsigned grid =
        (unsigned)(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
    ProfScope ps(&P->prof, KIND_OUTER, st);
    outer_adam_kernel<T, R><<<grid, kOuterThreads, 0, st>>>(
        fibers, p == 0 ? renv : lenv, p == 0 ? ridx : lidx, (const cx<T>*)C.vals, C.blk_off,
        C.nblocks, mom, vel, a);
    BFC_HIP_TRY(hipGetLastError());
  } else {
    cx<T>* slices = cores + off;
    if (C.nitems > 0) {
      ProfScope ps(&P->prof, KIND_INNER_IR, st);
      if (C.group_by_row)
        inner_ir_kernel<T, R, 1><<<C.nitems, 64, 0, st>>>(lenv, lidx, renv, ridx,
                                                          (const cx<T>*)C.vals, C.sub_off,
                                                          C.items, slices, (T*)P->adam_part);
      else
        inner_ir_kernel<T, R, 0><<<C.nitems, 64, 0, st>>>(lenv, lidx, renv, ridx,
                                                          (const cx<T>*)C.vals, C.sub_off,
                                                          C.items, slices, (T*)P->adam_part);
      BFC_HIP_TRY(hipGetLastError());
    }
    ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
    inner_adam_kernel<T, R><<<C.nblocks, 64, 0, st>>>(slices, (const T*)P->adam_part,
                                                      C.tile_items, mom, vel, a);
    BFC_HIP_TRY(hipGetLastError());
  }
  P->fused_res_valid = false;
  for (int q = 0; q < p && q < L; ++q) P->rlev[q].valid = false;
  for (int q = p + 1; q <= L + 1; ++q)
    if (q >= 2) P->llev[q].valid = false;
  return BFC_OK;
}

// ---------------------------------------------------------------------------
// ADF for butterfly completion (Sec. 5.1.3, Alg. "ADF for Butterfly
// Completion") with the orthogonalization sweeps of App. A.3.  QR factors are
// taken in FP64 by one wavefront per block or slice pair (row i of the
// factored matrix in lane i, at most 64 rows: leaf blocks of c <= 64 rows,
// slice pairs of 2r rows).
// ---------------------------------------------------------------------------
constexpr int kQrCols = 8;  // the largest rank

// Sum over the 64 lanes, the same value and order in every lane: DPP sums
// within each row of 16 lanes, then the four row sums read as scalars (no
// LDS round trips, which dominate the serial QR steps otherwise).
__device__ inline double wsum(double v) {
  v = row16_sum(v);
  return (bcast_d(v, 0) + bcast_d(v, 16)) + (bcast_d(v, 32) + bcast_d(v, 48));
}

// Reduced Householder QR of the nrows x r matrix whose row `lane` is a (rows
// >= nrows zero; reflector beta = -exp(i arg x_j) ||x||).  On return lane i
// holds row i of Q in q and, for i < r, row i of R in a (columns >= i).
__device__ __attribute__((always_inline)) inline void wave_qr(double2 (&a)[kQrCols], int nrows,
                                                              int r, double2 (&q)[kQrCols],
                                                              int lane) {
  const bool row = lane < nrows;
  double2 U[kQrCols];
#pragma unroll
  for (int j = 0; j < kQrCols; ++j) {
    U[j] = make_double2(0.0, 0.0);
    if (j >= r) continue;
    const bool below = row && lane >= j;
    const double2 x = make_double2(below ? a[j].x : 0.0, below ? a[j].y : 0.0);
    const double nx = sqrt(wsum(x.x * x.x + x.y * x.y));
    if (!(nx > 0.0)) continue;
    const double2 al = make_double2(bcast_d(x.x, j), bcast_d(x.y, j));
    const double aa = sqrt(al.x * al.x + al.y * al.y);
    const double px = aa > 0.0 ? al.x / aa : 1.0, py = aa > 0.0 ? al.y / aa : 0.0;
    const double2 v = make_double2(lane == j ? al.x + px * nx : x.x, lane == j ? al.y + py * nx : x.y);
    const double vn = sqrt(wsum(v.x * v.x + v.y * v.y));
    const double2 u = make_double2(v.x / vn, v.y / vn);
    U[j] = u;
#pragma unroll
    for (int col = j + 1; col < kQrCols; ++col) {
      if (col >= r) continue;
      const double2 w = make_double2(wsum(u.x * a[col].x + u.y * a[col].y),
                                     wsum(u.x * a[col].y - u.y * a[col].x));
      a[col].x -= 2.0 * (u.x * w.x - u.y * w.y);
      a[col].y -= 2.0 * (u.x * w.y + u.y * w.x);
    }
    // column j becomes beta e_j
    a[j] = make_double2(lane == j ? -px * nx : (lane < j ? a[j].x : 0.0),
                        lane == j ? -py * nx : (lane < j ? a[j].y : 0.0));
  }
#pragma unroll
  for (int c = 0; c < kQrCols; ++c) q[c] = make_double2(lane == c && c < r ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int j = kQrCols - 1; j >= 0; --j) {
    if (j >= r) continue;
#pragma unroll
    for (int c = 0; c < kQrCols; ++c) {
      if (c >= r) continue;
      const double2 w = make_double2(wsum(U[j].x * q[c].x + U[j].y * q[c].y),
                                     wsum(U[j].x * q[c].y - U[j].y * q[c].x));
      q[c].x -= 2.0 * (U[j].x * w.x - U[j].y * w.y);
      q[c].y -= 2.0 * (U[j].x * w.y + U[j].y * w.x);
    }
  }
}

// Row `lane` (< nrows) of a block stored row-major with r columns: x <- x F,
// F (r x r) given by rows held in lanes 0..r-1 (trans: x <- x F^T).
template <typename T>
__device__ __attribute__((always_inline)) inline void rows_times(cx<T>* blk, int nrows, int r,
                                                                 const double2 (&f)[kQrCols],
                                                                 bool trans, int lane) {
  double2 x[kQrCols], y[kQrCols];
  const bool row = lane < nrows;
#pragma unroll
  for (int k = 0; k < kQrCols; ++k) {
    const cx<T> v = (row && k < r) ? blk[(int64_t)lane * r + k] : cx<T>{T(0), T(0)};
    x[k] = make_double2((double)v.x, (double)v.y);
    y[k] = make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int i = 0; i < kQrCols; ++i) {
    if (i >= r) continue;
#pragma unroll
    for (int k = 0; k < kQrCols; ++k) {
      if (k >= r) continue;
      // F[i][k] from lane i
      const double2 fik = make_double2(bcast_d(f[k].x, i), bcast_d(f[k].y, i));
      // trans: y[i] += x[k] F[i][k]; else y[k] += x[i] F[i][k]
      if (trans) {
        y[i].x += x[k].x * fik.x - x[k].y * fik.y;
        y[i].y += x[k].x * fik.y + x[k].y * fik.x;
      } else {
        y[k].x += x[i].x * fik.x - x[i].y * fik.y;
        y[k].y += x[i].x * fik.y + x[i].y * fik.x;
      }
    }
  }
  if (!row) return;
#pragma unroll
  for (int k = 0; k < kQrCols; ++k)
    if (k < r) blk[(int64_t)lane * r + k] = cx<T>{T(y[k].x), T(y[k].y)};
}

// Left-to-right: QR of leaf block ib of Z^1 (c rows), R absorbed from the
// left into the slices (ib << 1) | b of core 1 (L >= 1) or, for L = 0, from
// the right (transposed) into the rows of Z^2.
template <typename T, int R>
__global__ __launch_bounds__(64) void orth_z1_left_kernel(cx<T>* z1, cx<T>* next, int c, int L) {
  const int ib = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < c;
  cx<T>* blk = z1 + (int64_t)ib * c * R;
  double2 a[kQrCols], q[kQrCols];
#pragma unroll
  for (int k = 0; k < kQrCols; ++k) {
    const cx<T> v = (row && k < R) ? blk[(int64_t)lane * R + k] : cx<T>{T(0), T(0)};
    a[k] = make_double2((double)v.x, (double)v.y);
  }
  wave_qr(a, c, R, q, lane);
  if (row) {
#pragma unroll
    for (int k = 0; k < R; ++k) blk[(int64_t)lane * R + k] = cx<T>{T(q[k].x), T(q[k].y)};
  }
  if (L == 0) {
    rows_times<T>(next + (int64_t)ib * c * R, c, R, a, true, lane);
    return;
  }
  // slices of core 1: new row i = sum_k R[i][k] slice row k, i.e. the slice's
  // transpose times R^T: treat the slice's columns as rows
  for (int b = 0; b < 2; ++b) {
    cx<T>* sl = next + (int64_t)((ib << 1) | b) * R * R;
    double2 col[kQrCols], out[kQrCols];
    // lane i < R gathers column i of the slice: col[k] = slice[k][i]
#pragma unroll
    for (int k = 0; k < kQrCols; ++k) {
      const cx<T> v = (lane < R && k < R) ? sl[k * R + lane] : cx<T>{T(0), T(0)};
      col[k] = make_double2((double)v.x, (double)v.y);
      out[k] = make_double2(0.0, 0.0);
    }
    // out (column lane of R S) [i] = sum_k R[i][k] S[k][lane]
#pragma unroll
    for (int i = 0; i < kQrCols; ++i) {
      if (i >= R) continue;
#pragma unroll
      for (int k = 0; k < kQrCols; ++k) {
        if (k >= R) continue;
        const double2 rik = make_double2(bcast_d(a[k].x, i), bcast_d(a[k].y, i));
        out[i].x += rik.x * col[k].x - rik.y * col[k].y;
        out[i].y += rik.x * col[k].y + rik.y * col[k].x;
      }
    }
    if (lane < R) {
#pragma unroll
      for (int i = 0; i < kQrCols; ++i)
        if (i < R) sl[i * R + lane] = cx<T>{T(out[i].x), T(out[i].y)};
    }
  }
}

// Left-to-right for inner core m: pair pi of slices (k0, k1 = k0 | 2^m),
// stacked along the left rank (lane beta r + i holds row i of slice k_beta);
// R absorbed from the left into the slices (pi << 1) | b of core m+1, or for
// m = L from the right (transposed) into the rows of Z^(L+2) block pi.
template <typename T, int R>
__global__ __launch_bounds__(64) void orth_inner_left_kernel(cx<T>* core, cx<T>* next, int m,
                                                             int L, int c) {
  const int pi = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < 2 * R;
  const int beta = row ? lane / R : 0, i = row ? lane % R : 0;
  const int64_t k0 = ((int64_t)(pi >> m) << (m + 1)) | (pi & ((1 << m) - 1));
  cx<T>* sl = core + (k0 | ((int64_t)beta << m)) * R * R;
  double2 a[kQrCols], q[kQrCols];
#pragma unroll
  for (int k = 0; k < kQrCols; ++k) {
    const cx<T> v = (row && k < R) ? sl[i * R + k] : cx<T>{T(0), T(0)};
    a[k] = make_double2((double)v.x, (double)v.y);
  }
  wave_qr(a, 2 * R, R, q, lane);
  if (row) {
#pragma unroll
    for (int k = 0; k < R; ++k) sl[i * R + k] = cx<T>{T(q[k].x), T(q[k].y)};
  }
  if (m == L) {
    rows_times<T>(next + (int64_t)pi * c * R, c, R, a, true, lane);
    return;
  }
  for (int b = 0; b < 2; ++b) {
    cx<T>* s2 = next + (int64_t)((pi << 1) | b) * R * R;
    double2 col[kQrCols], out[kQrCols];
#pragma unroll
    for (int k = 0; k < kQrCols; ++k) {
      const cx<T> v = (lane < R && k < R) ? s2[k * R + lane] : cx<T>{T(0), T(0)};
      col[k] = make_double2((double)v.x, (double)v.y);
      out[k] = make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int ii = 0; ii < kQrCols; ++ii) {
      if (ii >= R) continue;
#pragma unroll
      for (int k = 0; k < kQrCols; ++k) {
        if (k >= R) continue;
        const double2 rik = make_double2(bcast_d(a[k].x, ii), bcast_d(a[k].y, ii));
        out[ii].x += rik.x * col[k].x - rik.y * col[k].y;
        out[ii].y += rik.x * col[k].y + rik.y * col[k].x;
      }
    }
    if (lane < R) {
#pragma unroll
      for (int ii = 0; ii < kQrCols; ++ii)
        if (ii < R) s2[ii * R + lane] = cx<T>{T(out[ii].x), T(out[ii].y)};
    }
  }
}

// Right-to-left: QR of leaf block jb of Z^(L+2) (stored c x r), R^T absorbed
// from the right into the slices (b << L) | jb of core L, or for L = 0 into
// the rows of Z^1.
template <typename T, int R>
__global__ __launch_bounds__(64) void orth_zlast_right_kernel(cx<T>* zl, cx<T>* prev, cx<T>* z1,
                                                              int c, int L) {
  const int jb = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < c;
  cx<T>* blk = zl + (int64_t)jb * c * R;
  double2 a[kQrCols], q[kQrCols];
#pragma unroll
  for (int k = 0; k < kQrCols; ++k) {
    const cx<T> v = (row && k < R) ? blk[(int64_t)lane * R + k] : cx<T>{T(0), T(0)};
    a[k] = make_double2((double)v.x, (double)v.y);
  }
  wave_qr(a, c, R, q, lane);
  if (row) {
#pragma unroll
    for (int k = 0; k < R; ++k) blk[(int64_t)lane * R + k] = cx<T>{T(q[k].x), T(q[k].y)};
  }
  if (L == 0) {
    rows_times<T>(z1 + (int64_t)jb * c * R, c, R, a, true, lane);
    return;
  }
  for (int b = 0; b < 2; ++b)
    rows_times<T>(prev + ((int64_t)b << L | jb) * R * R, R, R, a, true, lane);
}

// Right-to-left for inner core m: pair pi of slices (2 pi, 2 pi + 1) side by
// side along the right rank; lane beta r + j holds column j of slice
// k_beta (the transposed pair is factored by QR, an LQ of the pair); the L
// factor (R^T) is absorbed from the right into the slices of core m-1 that
// differ in bit m-1, or for m = 1 into the rows of Z^1 block pi.
template <typename T, int R>
__global__ __launch_bounds__(64) void orth_inner_right_kernel(cx<T>* core, cx<T>* prev, int m,
                                                              int c) {
  const int pi = blockIdx.x, lane = threadIdx.x;
  const bool row = lane < 2 * R;
  const int beta = row ? lane / R : 0, j = row ? lane % R : 0;
  cx<T>* sl = core + ((int64_t)2 * pi + beta) * R * R;
  double2 a[kQrCols], q[kQrCols];
#pragma unroll
  for (int k = 0; k < kQrCols; ++k) {
    const cx<T> v = (row && k < R) ? sl[k * R + j] : cx<T>{T(0), T(0)};
    a[k] = make_double2((double)v.x, (double)v.y);
  }
  wave_qr(a, 2 * R, R, q, lane);
  if (row) {
#pragma unroll
    for (int k = 0; k < R; ++k) sl[k * R + j] = cx<T>{T(q[k].x), T(q[k].y)};
  }
  if (m == 1) {
    rows_times<T>(prev + (int64_t)pi * c * R, c, R, a, true, lane);
    return;
  }
  const int hi = pi >> (m - 1), lo = pi & ((1 << (m - 1)) - 1);
  for (int b = 0; b < 2; ++b) {
    const int64_t kp = ((int64_t)((hi << 1) | b) << (m - 1)) | lo;
    rows_times<T>(prev + kp * R * R, R, R, a, true, lane);
  }
}

// ADF step of an outer core: 16 lanes per fiber; pass 1 forms the direction
// N = sum conj(a_e) (t_e - z . a_e), pass 2 the norm ||A N||^2 over the
// fiber's entries, and lane k < R moves element k by alpha N_k with
// alpha = ||N||^2 / ||A N||^2 (the fiber keeps its values when A N = 0).
template <typename T, int R>
__global__ __launch_bounds__(kOuterThreads) void outer_adf_kernel(
    cx<T>* fibers, const cx<T>* env, const int32_t* env_idx, const cx<T>* vals,
    const int32_t* blk_off, int nblocks) {
  const int sub = threadIdx.x & 15;
  const int b = (int)((blockIdx.x * kOuterThreads + threadIdx.x) >> 4);
  int e0 = 0, e1 = 0;
  if (b < nblocks) {
    e0 = blk_off[b];
    e1 = blk_off[b + 1];
  }
  cx<T> z[R];
#pragma unroll
  for (int k = 0; k < R; ++k)
    z[k] = b < nblocks ? fibers[(int64_t)b * R + k] : cx<T>{T(0), T(0)};
  T nx[R], ny[R];
#pragma unroll
  for (int k = 0; k < R; ++k) nx[k] = ny[k] = T(0);
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
    }
    cx<T> v[4][R], t[4];
    gather_group<T, R, 4>(env, vals, id, ent, v, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      cx<T> x = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < R; ++k) cfma(x, z[k], v[q][k]);
      const cx<T> res = {t[q].x - x.x, t[q].y - x.y};
#pragma unroll
      for (int k = 0; k < R; ++k) {
        cx<T> h = {nx[k], ny[k]};
        cfma_conj(h, v[q][k], res);
        nx[k] = h.x;
        ny[k] = h.y;
      }
    }
  }
  cx<T> N[R];
#pragma unroll
  for (int k = 0; k < R; ++k) N[k] = cx<T>{row16_sum(nx[k]), row16_sum(ny[k])};
  double zz = 0.0;
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
    }
    cx<T> v[4][R], t[4];
    gather_group<T, R, 4>(env, vals, id, ent, v, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      cx<T> x = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < R; ++k) cfma(x, N[k], v[q][k]);
      zz += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
    }
  }
  zz = row16_sum(zz);
  if (b >= nblocks || sub >= R || !(zz > 0.0)) return;
  double nn = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k) nn += (double)N[k].x * (double)N[k].x + (double)N[k].y * (double)N[k].y;
  const double alpha = nn / zz;
  double sx = 0.0, sy = 0.0;
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k == sub) {
      sx = (double)N[k].x;
      sy = (double)N[k].y;
    }
  const int64_t o = (int64_t)b * R + sub;
  const cx<T> s = fibers[o];
  fibers[o] = cx<T>{T((double)s.x + alpha * sx), T((double)s.y + alpha * sy)};
}

// ADF on an inner core, per slice: stage 1 sums the work items' vectors
// sum conj(a)(t - x) into the direction N (dir); stage 2 sums the items'
// -sum conj(a)(a . N), so ||A N||^2 = -Re <N, that>, and moves the slice by
// alpha N, alpha = ||N||^2 / ||A N||^2 (kept when A N = 0).  One wavefront
// per slice, thread k < D for element k; the norms are wavefront sums.
template <typename T, int R>
__global__ __launch_bounds__(64) void inner_adf_kernel(cx<T>* slices, cx<T>* dir, const T* part,
                                                       const int32_t* tile_items, int stage) {
  constexpr int D = R * R;
  const int tile = blockIdx.x, k = threadIdx.x;
  const int it0 = tile_items[tile], it1 = tile_items[tile + 1];
  double gx = 0.0, gy = 0.0;
  if (k < D)
    for (int it = it0; it < it1; ++it) {
      gx += (double)part[(int64_t)it * 2 * D + 2 * k];
      gy += (double)part[(int64_t)it * 2 * D + 2 * k + 1];
    }
  const int64_t o = (int64_t)tile * D + k;
  if (stage == 1) {
    if (k < D) dir[o] = cx<T>{T(gx), T(gy)};
    return;
  }
  cx<T> nv = k < D ? dir[o] : cx<T>{T(0), T(0)};
  const double nn = wsum((double)nv.x * (double)nv.x + (double)nv.y * (double)nv.y);
  const double zz = -wsum((double)nv.x * gx + (double)nv.y * gy);
  if (k >= D || !(zz > 0.0)) return;
  const double alpha = nn / zz;
  const cx<T> s = slices[o];
  slices[o] = cx<T>{T((double)s.x + alpha * (double)nv.x), T((double)s.y + alpha * (double)nv.y)};
}

template <typename T, int R>
bfc_status adf_sweep_t(Problem* P, hipStream_t st) {
  cx<T>* cores = (cx<T>*)P->cores;
  const int L = P->L;
  const int c = P->c;
  const int64_t nb = (int64_t)1 << L;
  auto off = [&](int p) -> int64_t {
    return p == 0 ? 0 : (p == L + 1 ? last_off(P->n, L, R) : inner_off(P->n, L, R, p));
  };
  // right-to-left orthogonalization: cores L+1 .. 1
  {
    ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
    orth_zlast_right_kernel<T, R><<<(unsigned)nb, 64, 0, st>>>(
        cores + off(L + 1), L >= 1 ? cores + off(L) : nullptr, cores, c, L);
    for (int m = L; m >= 1; --m)
      orth_inner_right_kernel<T, R><<<(unsigned)nb, 64, 0, st>>>(cores + off(m),
                                                                 cores + off(m - 1), m, c);
    BFC_HIP_TRY(hipGetLastError());
  }
  invalidate_envs(P);
  for (int p = 0; p <= L + 1; ++p) {
    const CoreLayout& C = P->lay[p];
    {
      ProfScope ps(&P->prof, KIND_ENV, st);
      BFC_TRY(ensure_right<T, R>(P, p, st));
      BFC_TRY(ensure_left<T, R>(P, p, st));
    }
    const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R)
                                 : (p <= L - 1 ? (const cx<T>*)P->rlev[p].vec : nullptr);
    const int32_t* ridx = (p == L) ? C.cols : C.rnode;
    const cx<T>* lenv = (p == 1) ? cores : (p >= 2 ? (const cx<T>*)P->llev[p].vec : nullptr);
    const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
    if (p == 0 || p == L + 1) {
      const unsigned grid =
          (unsigned)(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
      ProfScope ps(&P->prof, KIND_OUTER, st);
      outer_adf_kernel<T, R><<<grid, kOuterThreads, 0, st>>>(
          cores + off(p), p == 0 ? renv : lenv, p == 0 ? ridx : lidx, (const cx<T>*)C.vals,
          C.blk_off, C.nblocks);
    } else {
      cx<T>* slices = cores + off(p);
      cx<T>* dir = (cx<T>*)P->adf_dir;
      T* part = (T*)P->adam_part;
      ProfScope ps(&P->prof, KIND_INNER_IR, st);
      for (int stage = 1; stage <= 2; ++stage) {
        if (C.nitems > 0) {
          const cx<T>* s0 = stage == 1 ? slices : dir;
          if (C.group_by_row) {
            if (stage == 1)
              inner_ir_kernel<T, R, 1, false><<<C.nitems, 64, 0, st>>>(
                  lenv, lidx, renv, ridx, (const cx<T>*)C.vals, C.sub_off, C.items, s0, part);
            else
              inner_ir_kernel<T, R, 1, true><<<C.nitems, 64, 0, st>>>(
                  lenv, lidx, renv, ridx, (const cx<T>*)C.vals, C.sub_off, C.items, s0, part);
          } else {
            if (stage == 1)
              inner_ir_kernel<T, R, 0, false><<<C.nitems, 64, 0, st>>>(
                  lenv, lidx, renv, ridx, (const cx<T>*)C.vals, C.sub_off, C.items, s0, part);
            else
              inner_ir_kernel<T, R, 0, true><<<C.nitems, 64, 0, st>>>(
                  lenv, lidx, renv, ridx, (const cx<T>*)C.vals, C.sub_off, C.items, s0, part);
          }
        }
        inner_adf_kernel<T, R><<<C.nblocks, 64, 0, st>>>(slices, dir, part, C.tile_items, stage);
      }
    }
    BFC_HIP_TRY(hipGetLastError());
    if (p <= L) {
      ProfScope ps(&P->prof, KIND_INNER_SOLVE, st);
      if (p == 0)
        orth_z1_left_kernel<T, R><<<(unsigned)nb, 64, 0, st>>>(cores, cores + off(1), c, L);
      else
        orth_inner_left_kernel<T, R><<<(unsigned)nb, 64, 0, st>>>(cores + off(p),
                                                                  cores + off(p + 1), p, L, c);
      BFC_HIP_TRY(hipGetLastError());
    }
    // cores p and p+1 changed: right levels below p+1 and left levels above p
    for (int q = 0; q <= p && q < L; ++q) P->rlev[q].valid = false;
    for (int q = p + 1; q <= L + 1; ++q)
      if (q >= 2) P->llev[q].valid = false;
  }
  P->fused_res_valid = false;
  return BFC_OK;
}

template <typename T, int R>
struct AdfF {
  static bfc_status run(Problem* P, hipStream_t st) { return adf_sweep_t<T, R>(P, st); }
};

// Entries per block and block count of a residual over m entries (the block
// partials fit the problem's reduction scratch).
inline void residual_split(const Problem* P, int64_t m, int64_t& per, int64_t& nblk) {
  const int64_t nblk_max = (int64_t)(P->red_len / 2);
  per = (m + nblk_max - 1) / nblk_max;
  per = ((per + kResThreads - 1) / kResThreads) * kResThreads;
  if (per < kResThreads) per = kResThreads;
  nblk = (m + per - 1) / per;
}

template <typename T, int R>
bfc_status residual_observed_t(Problem* P, double* out2, hipStream_t st) {
  const int L = P->L;
  if (P->fused_res_valid) {
    // the last core's update left per-fiber norms for exactly these cores
    ProfScope ps(&P->prof, KIND_RESIDUAL, st);
    residual_final_kernel<<<1, kResThreads, 0, st>>>(P->fused_res, outer_grid(P->lay[L + 1]),
                                                      out2);
    BFC_HIP_TRY(hipGetLastError());
    return BFC_OK;
  }
  BFC_TRY(ensure_left<T, R>(P, L + 1, st));
  cx<T>* cores = (cx<T>*)P->cores;
  const CoreLayout& C = P->lay[L + 1];
  const cx<T>* lenv = (L + 1 == 1) ? cores : (const cx<T>*)P->llev[L + 1].vec;
  const int32_t* lidx = (L + 1 == 1) ? C.rows : C.lnode;
  const int64_t m = P->nnz;
  int64_t per, nblk;
  residual_split(P, m, per, nblk);
  ProfScope ps(&P->prof, KIND_RESIDUAL, st);
  residual_observed_kernel<T, R><<<(unsigned)nblk, kResThreads, 0, st>>>(ResObsArgs<T>{
      lenv, lidx, cores + last_off(P->n, L, R), C.cols, (const cx<T>*)C.vals, m, per, P->red});
  BFC_HIP_TRY(hipGetLastError());
  residual_final_kernel<<<1, kResThreads, 0, st>>>(P->red, (int)nblk, out2);
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

#define BFC_CASE(RR)                                                     \
  case RR:                                                               \
    return prec == BFC_C128 ? F<double, RR>::run(args...) : F<float, RR>::run(args...);

// Calls that exist at ranks 1 .. kNarrowRank only (ADAM, ADF, the loss
// gradient): instantiated for those ranks.
template <template <typename, int> class F, typename... Args>
bfc_status dispatch(int prec, int r, Args... args) {
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
      set_error("this call supports ranks 1 .. 8");
      return BFC_EINVAL;
  }
}

// The ALS sweep, reconstruction and residuals: every rank up to BFC_MAX_RANK.
template <template <typename, int> class F, typename... Args>
bfc_status dispatch_any(int prec, int r, Args... args) {
  switch (r) {
    BFC_CASE(1)
    BFC_CASE(2)
    BFC_CASE(3)
    BFC_CASE(4)
    BFC_CASE(5)
    BFC_CASE(6)
    BFC_CASE(7)
    BFC_CASE(8)
    BFC_CASE(9)
    BFC_CASE(10)
    BFC_CASE(11)
    BFC_CASE(12)
    default:
      set_error("rank out of range");
      return BFC_EINVAL;
  }
}
#undef BFC_CASE

template <typename T, int R>
struct SweepF {
  static bfc_status run(Problem* P, int p, hipStream_t st) {
    if constexpr (R > kNarrowRank)
      return sweep_core_wide<T, R>(P, p, st);
    else
      return sweep_core_t<T, R>(P, p, st);
  }
};
template <typename T, int R>
struct AdamF {
  static bfc_status run(Problem* P, int p, const AdamArgs* a, hipStream_t st) {
    return adam_core_t<T, R>(P, p, *a, st);
  }
};
template <typename T, int R>
struct PredictF {
  static bfc_status run(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                        void* out, hipStream_t st) {
    return predict_t<T, R>(P, m, rows, cols, out, st);
  }
};
template <typename T, int R>
struct ResidualObservedF {
  static bfc_status run(Problem* P, double* out2, hipStream_t st) {
    return residual_observed_t<T, R>(P, out2, st);
  }
};
template <typename T, int R>
struct ResidualF {
  static bfc_status run(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                        const void* vals, double* out2, hipStream_t st) {
    return residual_t<T, R>(P, m, rows, cols, vals, out2, st);
  }
};

// ---------------------------------------------------------------------------
// batched sweeps of independent problems
// ---------------------------------------------------------------------------
// The launch list of one sweep of every problem, in dependency order (a
// problem's own order is exactly that of a single sweep, so results are
// bit-identical to sweeping the problems one by one):
//   right levels from the top (depth t computes level L-1-t of each problem),
//   core 0 of every problem,
//   then per step s = 1 .. max L + 1: left level s (problems with
//   2 <= s <= L+1), the inner Gram and solve of core s (s <= L), the outer
//   update of core s (s = L+1).
// Each entry is one launch per rank present at that step.

template <typename T, typename A>
bfc_status upload_tasks(Batch* B, int kind, int r, const std::vector<A>& args,
                        const std::vector<int64_t>& blocks) {
  if (args.empty()) return BFC_OK;
  BatchLaunch bl;
  bl.kind = kind;
  bl.r = r;
  bl.ntasks = (int)args.size();
  std::vector<int32_t> off(args.size() + 1, 0);
  for (size_t k = 0; k < args.size(); ++k) {
    const int64_t next = off[k] + blocks[k];
    if (next > 0x7FFFFFFF) {
      set_error("batched launch too large");
      return BFC_EINVAL;
    }
    off[k + 1] = (int32_t)next;
  }
  bl.blocks = off.back();
  if (bl.blocks == 0) return BFC_OK;
  BFC_HIP_TRY(lib_malloc(&bl.tasks, sizeof(A) * args.size()));
  B->allocs.push_back(bl.tasks);
  BFC_HIP_TRY(lib_malloc((void**)&bl.block_off, sizeof(int32_t) * off.size()));
  B->allocs.push_back(bl.block_off);
  BFC_HIP_TRY(hipMemcpy(bl.tasks, args.data(), sizeof(A) * args.size(), hipMemcpyHostToDevice));
  BFC_HIP_TRY(hipMemcpy(bl.block_off, off.data(), sizeof(int32_t) * off.size(),
                        hipMemcpyHostToDevice));
  (kind == BK_RES || kind == BK_RES_FINAL   ? B->resid
   : kind == BK_RES_FUSED                   ? B->resid_fused
                                            : B->sweep)
      .push_back(bl);
  return BFC_OK;
}

template <typename T, int R>
struct BatchStep {
  // arguments of every kernel of problem P at step s of the sweep
  static void env(const Problem* P, int q, int right, std::vector<EnvArgs<T>>& a,
                  std::vector<int64_t>& b) {
    const EnvLevel& E = right ? P->rlev[q] : P->llev[q];
    if (E.count <= 0) return;
    // formed by the outer update next to it instead (up_node)
    if (right ? (q == 0 && P->lay[0].up_node) : (q == P->L + 1 && P->lay[P->L + 1].up_node))
      return;
    a.push_back(env_args<T, R>(P, q, right));
    b.push_back(grid_for(E.count));
  }
  // the outer update of core p; with up_node it forms the outermost level's
  // products itself (a BK_OUTER_UP1 / UP2 task), else it reads that level
  static void outer(const Problem* P, int p, std::vector<OuterArgs<T>>& a,
                    std::vector<int64_t>& b) {
    const int L = P->L;
    const CoreLayout& C = P->lay[p];
    cx<T>* cores = (cx<T>*)P->cores;
    cx<T>* fibers = cores + (p == 0 ? 0 : last_off(P->n, L, R));
    const cx<T>* env;
    const int32_t* idx;
    const cx<T>* zsl = nullptr;
    if (C.up_node) {
      env = p == 0 ? (const cx<T>*)P->rlev[1].vec : (const cx<T>*)P->llev[L].vec;
      idx = C.up_node;
      zsl = cores + inner_off(P->n, L, R, p == 0 ? 1 : L);
    } else if (p == 0) {
      env = (L == 0) ? cores + last_off(P->n, L, R) : (const cx<T>*)P->rlev[0].vec;
      idx = (L == 0) ? C.cols : C.rnode;
    } else {
      env = (p == 1) ? cores : (const cx<T>*)P->llev[p].vec;
      idx = (p == 1) ? C.rows : C.lnode;
    }
    a.push_back(OuterArgs<T>{fibers, env, idx, (const cx<T>*)C.vals, C.blk_off, C.nblocks,
                             P->cfg.reg_rel, reg_floor_of(P),
                             P->cfg.reg_mode == BFC_REG_PROXIMAL ? 1 : 0, P->flags,
                             p == L + 1 ? P->fused_res : nullptr, zsl, L, P->c});
    b.push_back(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
  }
  static void inner(const Problem* P, int p, std::vector<GramArgs<T>>& grow,
                    std::vector<int64_t>& brow, std::vector<GramArgs<T>>& gcol,
                    std::vector<int64_t>& bcol, std::vector<SolveArgs<T>>& sv,
                    std::vector<int64_t>& bs) {
    const int L = P->L;
    const CoreLayout& C = P->lay[p];
    cx<T>* cores = (cx<T>*)P->cores;
    const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R) : (const cx<T>*)P->rlev[p].vec;
    const cx<T>* lenv = (p == 1) ? cores : (const cx<T>*)P->llev[p].vec;
    if (C.nitems > 0) {
      GramArgs<T> g{lenv, renv, (const cx<T>*)C.vals, (const int4*)C.sub_rec, C.items,
                    (T*)P->partials};
      if (C.group_by_row) {
        grow.push_back(g);
        brow.push_back(C.nitems);
      } else {
        gcol.push_back(g);
        bcol.push_back(C.nitems);
      }
    }
    sv.push_back(SolveArgs<T>{cores + inner_off(P->n, L, R, p), (const T*)P->partials,
                              C.tile_items, P->cfg.reg_rel, reg_floor_of(P),
                              P->cfg.reg_mode == BFC_REG_PROXIMAL ? 1 : 0, P->flags, 0,
                              nullptr, nullptr, nullptr, nullptr});
    bs.push_back(C.nblocks);
  }
  static void resid(Problem* P, double* out, std::vector<ResObsArgs<T>>& a,
                    std::vector<int64_t>& b, std::vector<ResFinalArgs>& f) {
    const int L = P->L;
    const CoreLayout& C = P->lay[L + 1];
    cx<T>* cores = (cx<T>*)P->cores;
    const cx<T>* lenv = (L + 1 == 1) ? cores : (const cx<T>*)P->llev[L + 1].vec;
    const int32_t* lidx = (L + 1 == 1) ? C.rows : C.lnode;
    int64_t per, nblk;
    residual_split(P, P->nnz, per, nblk);
    a.push_back(ResObsArgs<T>{lenv, lidx, cores + last_off(P->n, L, R), C.cols,
                              (const cx<T>*)C.vals, P->nnz, per, P->red});
    b.push_back(nblk);
    f.push_back(ResFinalArgs{P->red, (int)nblk, out});
  }
};

// All problems of one rank R: append their launches for one phase.
template <typename T, int R>
struct BatchPlanR {
  static bfc_status run(Batch* B, const std::vector<Problem*>& ps, int phase, int step) {
    typedef BatchStep<T, R> S;
    if (phase == 0) {  // right level at depth `step` from the top
      std::vector<EnvArgs<T>> a;
      std::vector<int64_t> b;
      for (Problem* P : ps)
        if (step < P->L) S::env(P, P->L - 1 - step, 1, a, b);
      return upload_tasks<T>(B, BK_ENV_RIGHT, R, a, b);
    }
    if (phase == 1) {  // left level `step`
      std::vector<EnvArgs<T>> a;
      std::vector<int64_t> b;
      for (Problem* P : ps)
        if (step >= 2 && step <= P->L + 1) S::env(P, step, 0, a, b);
      return upload_tasks<T>(B, BK_ENV_LEFT, R, a, b);
    }
    if (phase == 2) {  // inner core `step`
      std::vector<GramArgs<T>> gr, gc;
      std::vector<SolveArgs<T>> sv;
      std::vector<int64_t> br, bc, bs;
      for (Problem* P : ps)
        if (step >= 1 && step <= P->L) S::inner(P, step, gr, br, gc, bc, sv, bs);
      BFC_TRY(upload_tasks<T>(B, BK_GRAM_ROW, R, gr, br));
      BFC_TRY(upload_tasks<T>(B, BK_GRAM_COL, R, gc, bc));
      return upload_tasks<T>(B, BK_SOLVE, R, sv, bs);
    }
    if (phase == 3) {  // outer core 0 (step 0) or L+1 (step = L+1)
      std::vector<OuterArgs<T>> a, au;
      std::vector<int64_t> b, bu;
      for (Problem* P : ps) {
        const int p = step == 0 ? 0 : step;
        if (step != 0 && step != P->L + 1) continue;
        if (P->lay[p].up_node)
          S::outer(P, p, au, bu);
        else
          S::outer(P, p, a, b);
      }
      BFC_TRY(upload_tasks<T>(B, BK_OUTER, R, a, b));
      return upload_tasks<T>(B, step == 0 ? BK_OUTER_UP1 : BK_OUTER_UP2, R, au, bu);
    }
    // phase 4: residual norms
    std::vector<ResObsArgs<T>> a;
    std::vector<int64_t> b;
    std::vector<ResFinalArgs> f;
    std::vector<int64_t> one;
    for (Problem* P : ps) {
      size_t k = 0;
      while (B->probs[k] != P) ++k;
      S::resid(P, B->res + 2 * k, a, b, f);
      one.push_back(1);
    }
    BFC_TRY(upload_tasks<T>(B, BK_RES, R, a, b));
    BFC_TRY(upload_tasks<T>(B, BK_RES_FINAL, R, f, one));
    // the same norms from the per-fiber sums the last core's update leaves
    std::vector<ResFinalArgs> fz;
    for (Problem* P : ps) {
      size_t k = 0;
      while (B->probs[k] != P) ++k;
      fz.push_back(ResFinalArgs{P->fused_res, outer_grid(P->lay[P->L + 1]), B->res + 2 * k});
    }
    return upload_tasks<T>(B, BK_RES_FUSED, R, fz, one);
  }
};

template <typename T>
bfc_status batch_plan_phase(Batch* B, int phase, int step) {
  for (int r = 1; r <= BFC_MAX_RANK; ++r) {
    std::vector<Problem*> ps;
    for (Problem* P : B->probs)
      if (P->r == r) ps.push_back(P);
    if (ps.empty()) continue;
    bfc_status s = BFC_OK;
    switch (r) {
#define BFC_PLAN(RR) \
  case RR:           \
    s = BatchPlanR<T, RR>::run(B, ps, phase, step); \
    break;
      BFC_PLAN(1) BFC_PLAN(2) BFC_PLAN(3) BFC_PLAN(4) BFC_PLAN(5) BFC_PLAN(6) BFC_PLAN(7)
      BFC_PLAN(8)
#undef BFC_PLAN
    }
    BFC_TRY(s);
  }
  return BFC_OK;
}

template <typename T>
bfc_status build_batch_plan_t(Batch* B) {
  int maxL = 0;
  for (Problem* P : B->probs) maxL = P->L > maxL ? P->L : maxL;
  for (int t = 0; t < maxL; ++t) BFC_TRY(batch_plan_phase<T>(B, 0, t));
  BFC_TRY(batch_plan_phase<T>(B, 3, 0));
  for (int s = 1; s <= maxL + 1; ++s) {
    BFC_TRY(batch_plan_phase<T>(B, 1, s));
    BFC_TRY(batch_plan_phase<T>(B, 2, s));
    BFC_TRY(batch_plan_phase<T>(B, 3, s));
  }
  return batch_plan_phase<T>(B, 4, 0);
}

template <typename T, int R>
bfc_status launch_batched_r(const BatchLaunch& bl, hipStream_t st) {
  const unsigned g = (unsigned)bl.blocks;
  switch (bl.kind) {
    case BK_ENV_RIGHT:
      env_level_batched<T, R, 1><<<g, 256, 0, st>>>((const EnvArgs<T>*)bl.tasks, bl.block_off,
                                                     bl.ntasks);
      break;
    case BK_ENV_LEFT:
      env_level_batched<T, R, 0><<<g, 256, 0, st>>>((const EnvArgs<T>*)bl.tasks, bl.block_off,
                                                     bl.ntasks);
      break;
    case BK_OUTER:
      outer_update_kernel_batched<T, R, 0><<<g, kOuterThreads, 0, st>>>(
          (const OuterArgs<T>*)bl.tasks, bl.block_off, bl.ntasks);
      break;
    case BK_OUTER_UP1:
      outer_update_kernel_batched<T, R, 1><<<g, kOuterThreads, 0, st>>>(
          (const OuterArgs<T>*)bl.tasks, bl.block_off, bl.ntasks);
      break;
    case BK_OUTER_UP2:
      outer_update_kernel_batched<T, R, 2><<<g, kOuterThreads, 0, st>>>(
          (const OuterArgs<T>*)bl.tasks, bl.block_off, bl.ntasks);
      break;
    case BK_GRAM_ROW:
      inner_gram_kernel_batched<T, R, 1><<<g, 64, 0, st>>>((const GramArgs<T>*)bl.tasks,
                                                           bl.block_off, bl.ntasks);
      break;
    case BK_GRAM_COL:
      inner_gram_kernel_batched<T, R, 0><<<g, 64, 0, st>>>((const GramArgs<T>*)bl.tasks,
                                                           bl.block_off, bl.ntasks);
      break;
    case BK_SOLVE:
      inner_solve_kernel_batched<T, R><<<g, kSolveThreads, 0, st>>>(
          (const SolveArgs<T>*)bl.tasks, bl.block_off, bl.ntasks);
      break;
    case BK_RES:
      residual_observed_kernel_batched<T, R><<<g, kResThreads, 0, st>>>(
          (const ResObsArgs<T>*)bl.tasks, bl.block_off, bl.ntasks);
      break;
    case BK_RES_FINAL:
    case BK_RES_FUSED:
      residual_final_batched<<<bl.ntasks, kResThreads, 0, st>>>((const ResFinalArgs*)bl.tasks);
      break;
  }
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <typename T>
bfc_status launch_batched(const BatchLaunch& bl, hipStream_t st) {
  switch (bl.r) {
#define BFC_LB(RR) \
  case RR:         \
    return launch_batched_r<T, RR>(bl, st);
    BFC_LB(1) BFC_LB(2) BFC_LB(3) BFC_LB(4) BFC_LB(5) BFC_LB(6) BFC_LB(7) BFC_LB(8)
#undef BFC_LB
  }
  set_error("rank out of range");
  return BFC_EINVAL;
}

}  // namespace

bfc_status build_batch_plan(Batch* B) {
  return B->prec == BFC_C128 ? build_batch_plan_t<double>(B) : build_batch_plan_t<float>(B);
}

bfc_status launch_batch(const std::vector<BatchLaunch>& plan, int prec, hipStream_t st) {
  for (const BatchLaunch& bl : plan)
    BFC_TRY(prec == BFC_C128 ? launch_batched<double>(bl, st) : launch_batched<float>(bl, st));
  return BFC_OK;
}

size_t inner_factor_bytes(int r) {
  switch (r) {
    case 1: return solve_factor_elems<1>() * 16;
    case 2: return solve_factor_elems<2>() * 16;
    case 3: return solve_factor_elems<3>() * 16;
    case 4: return solve_factor_elems<4>() * 16;
    case 5: return solve_factor_elems<5>() * 16;
    case 6: return solve_factor_elems<6>() * 16;
    case 7: return solve_factor_elems<7>() * 16;
    default: return solve_factor_elems<8>() * 16;
  }
}

size_t inner_partial_bytes(int prec, int r) {
  if (r > kNarrowRank) return wide_region_bytes(r);  // the fused kernels' per-slice region
  const int W = r * r + 2 * r;
  const int WP = (W + 15) / 16 * 16;
  return (size_t)WP * WP * (prec == BFC_C128 ? 8 : 4);
}

bfc_status launch_sweep_core(Problem* P, int core, hipStream_t st) {
  return dispatch_any<SweepF>(P->prec, P->r, P, core, st);
}

bfc_status launch_adam_core(Problem* P, int core, int t, double alpha, double beta1,
                            double beta2, double sigma, hipStream_t st) {
  const AdamArgs a{alpha, beta1, beta2, sigma, 1.0 - std::pow(beta1, (double)t),
                   1.0 - std::pow(beta2, (double)t)};
  return dispatch<AdamF>(P->prec, P->r, P, core, &a, st);
}

bfc_status launch_adf_sweep(Problem* P, hipStream_t st) {
  return dispatch<AdfF>(P->prec, P->r, P, st);
}

bfc_status launch_predict(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                          void* out, hipStream_t st) {
  if (m == 0) return BFC_OK;
  return dispatch_any<PredictF>(P->prec, P->r, P, m, rows, cols, out, st);
}

bfc_status launch_residual(const Problem* P, int64_t m, const int32_t* rows, const int32_t* cols,
                           const void* vals, double* out2, hipStream_t st) {
  return dispatch_any<ResidualF>(P->prec, P->r, P, m, rows, cols, vals, out2, st);
}

bfc_status launch_residual_observed(Problem* P, double* out2, hipStream_t st) {
  return dispatch_any<ResidualObservedF>(P->prec, P->r, P, out2, st);
}

void invalidate_envs(Problem* P) {
  for (auto& E : P->rlev) E.valid = false;
  for (auto& E : P->llev) E.valid = false;
  P->fused_res_valid = false;
}

bfc_status launch_convert_cores(Problem* P, const void* src, void* dst, bool to_internal,
                                hipStream_t st) {
  const int64_t m = P->nparams;
  if (to_internal) {
    invalidate_envs(P);
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

template <typename T>
__global__ void values_to_layout_kernel(const int32_t* perm, const double2* src, cx<T>* dst,
                                        int64_t nnz, int32_t* bad) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nnz) return;
  const double2 v = src[perm[k]];
  if (!isfinite(v.x) || !isfinite(v.y)) atomicOr(bad, 1);
  dst[k] = cx<T>{T(v.x), T(v.y)};
}

// Values into every core's sorted layout; non-finite values set *bad_flag
// (which the caller clears beforehand).  Asynchronous.
bfc_status enqueue_set_values(Problem* P, const void* d_vals, hipStream_t st) {
  const int64_t nnz = P->nnz;
  if (nnz == 0) return BFC_OK;
  for (int p = 0; p <= P->L + 1; ++p) {
    const CoreLayout& C = P->lay[p];
    if (P->prec == BFC_C128)
      values_to_layout_kernel<double><<<grid_for(nnz), 256, 0, st>>>(
          C.perm, (const double2*)d_vals, (cx<double>*)C.vals, nnz, P->bad_flag);
    else
      values_to_layout_kernel<float><<<grid_for(nnz), 256, 0, st>>>(
          C.perm, (const double2*)d_vals, (cx<float>*)C.vals, nnz, P->bad_flag);
    BFC_HIP_TRY(hipGetLastError());
  }
  P->fused_res_valid = false;
  return BFC_OK;
}

bfc_status launch_set_values(Problem* P, const void* d_vals, hipStream_t st) {
  if (P->nnz == 0) return BFC_OK;
  BFC_HIP_TRY(hipMemsetAsync(P->bad_flag, 0, 4, st));
  BFC_TRY(enqueue_set_values(P, d_vals, st));
  int32_t bad = 0;
  BFC_HIP_TRY(hipMemcpyAsync(&bad, P->bad_flag, 4, hipMemcpyDeviceToHost, st));
  BFC_HIP_TRY(hipStreamSynchronize(st));
  if (bad) {
    set_error("bfc_set_values: a value is NaN or Inf (the layout now holds it)");
    return BFC_ENONFINITE;
  }
  return BFC_OK;
}

template <typename T>
__global__ void cores_from_f32_kernel(const float2* src, cx<T>* dst, int64_t m) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) dst[k] = {T(src[k].x), T(src[k].y)};
}

bfc_status launch_cores_from_f32(Problem* P, const float* src, hipStream_t st) {
  const int64_t m = P->nparams;
  invalidate_envs(P);
  if (P->prec == BFC_C128)
    cores_from_f32_kernel<double><<<grid_for(m), 256, 0, st>>>((const float2*)src,
                                                               (cx<double>*)P->cores, m);
  else
    cores_from_f32_kernel<float><<<grid_for(m), 256, 0, st>>>((const float2*)src,
                                                              (cx<float>*)P->cores, m);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

// Gradient of an outer core: 16 lanes per fiber sum conj(a_e)(x_e - t_e);
// lane k < R writes element k.
template <typename T, int R>
__global__ __launch_bounds__(kOuterThreads) void outer_grad_kernel(
    const cx<T>* fibers, const cx<T>* env, const int32_t* env_idx, const cx<T>* vals,
    const int32_t* blk_off, int nblocks, cx<T>* grad) {
  const int sub = threadIdx.x & 15;
  const int b = (int)((blockIdx.x * kOuterThreads + threadIdx.x) >> 4);
  int e0 = 0, e1 = 0;
  if (b < nblocks) {
    e0 = blk_off[b];
    e1 = blk_off[b + 1];
  }
  cx<T> z[R];
#pragma unroll
  for (int k = 0; k < R; ++k)
    z[k] = b < nblocks ? fibers[(int64_t)b * R + k] : cx<T>{T(0), T(0)};
  T gx[R], gy[R];
#pragma unroll
  for (int k = 0; k < R; ++k) gx[k] = gy[k] = T(0);
  for (int base = e0 + sub; base < e1; base += 16 * 4) {
    int id[4], ent[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ent[q] = base + 16 * q;
      id[q] = (ent[q] < e1) ? env_idx[ent[q]] : -1;
    }
    cx<T> v[4][R], t[4];
    gather_group<T, R, 4>(env, vals, id, ent, v, t);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (id[q] < 0) continue;
      cx<T> x = {T(0), T(0)};
#pragma unroll
      for (int k = 0; k < R; ++k) cfma(x, z[k], v[q][k]);
      const cx<T> res = {x.x - t[q].x, x.y - t[q].y};
#pragma unroll
      for (int k = 0; k < R; ++k) {
        cx<T> h = {gx[k], gy[k]};
        cfma_conj(h, v[q][k], res);
        gx[k] = h.x;
        gy[k] = h.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < R; ++k) {
    gx[k] = row16_sum(gx[k]);
    gy[k] = row16_sum(gy[k]);
  }
  if (b >= nblocks || sub >= R) return;
  cx<T> g = {T(0), T(0)};
#pragma unroll
  for (int k = 0; k < R; ++k)
    if (k == sub) g = cx<T>{gx[k], gy[k]};
  grad[(int64_t)b * R + sub] = g;
}

// Gradient of an inner slice: minus the sum of its work items' vectors
// sum conj(a)(t - x), in a fixed order (thread k for element k).
template <typename T, int R>
__global__ __launch_bounds__(64) void inner_grad_kernel(const T* part, const int32_t* tile_items,
                                                        cx<T>* grad) {
  constexpr int D = R * R;
  const int tile = blockIdx.x, k = threadIdx.x;
  if (k >= D) return;
  const int it0 = tile_items[tile], it1 = tile_items[tile + 1];
  double gx = 0.0, gy = 0.0;
  for (int it = it0; it < it1; ++it) {
    gx -= (double)part[(int64_t)it * 2 * D + 2 * k];
    gy -= (double)part[(int64_t)it * 2 * D + 2 * k + 1];
  }
  grad[(int64_t)tile * D + k] = cx<T>{T(gx), T(gy)};
}

template <typename T, typename O>
__global__ void grad_out_kernel(const cx<T>* g, O* out, int64_t m, float scale) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  out[2 * k] = O((double)scale * (double)g[k].x);
  out[2 * k + 1] = O((double)scale * (double)g[k].y);
}

template <typename T, int R>
bfc_status loss_gradient_t(Problem* P, float scale, void* out, int out_fp64, hipStream_t st) {
  const cx<T>* cores = (const cx<T>*)P->cores;
  cx<T>* grad = (cx<T>*)P->grad;
  const int L = P->L;
  auto off = [&](int p) -> int64_t {
    return p == 0 ? 0 : (p == L + 1 ? last_off(P->n, L, R) : inner_off(P->n, L, R, p));
  };
  for (int p = 0; p <= L + 1; ++p) {
    const CoreLayout& C = P->lay[p];
    {
      ProfScope ps(&P->prof, KIND_ENV, st);
      BFC_TRY(ensure_right<T, R>(P, p, st));
      BFC_TRY(ensure_left<T, R>(P, p, st));
    }
    const cx<T>* renv = (p == L) ? cores + last_off(P->n, L, R)
                                 : (p <= L - 1 ? (const cx<T>*)P->rlev[p].vec : nullptr);
    const int32_t* ridx = (p == L) ? C.cols : C.rnode;
    const cx<T>* lenv = (p == 1) ? cores : (p >= 2 ? (const cx<T>*)P->llev[p].vec : nullptr);
    const int32_t* lidx = (p == 1) ? C.rows : C.lnode;
    if (p == 0 || p == L + 1) {
      const unsigned grid =
          (unsigned)(((int64_t)C.nblocks * 16 + kOuterThreads - 1) / kOuterThreads);
      ProfScope ps(&P->prof, KIND_OUTER, st);
      outer_grad_kernel<T, R><<<grid, kOuterThreads, 0, st>>>(
          cores + off(p), p == 0 ? renv : lenv, p == 0 ? ridx : lidx, (const cx<T>*)C.vals,
          C.blk_off, C.nblocks, grad + off(p));
    } else {
      ProfScope ps(&P->prof, KIND_INNER_IR, st);
      T* part = (T*)P->adam_part;
      if (C.nitems > 0) {
        if (C.group_by_row)
          inner_ir_kernel<T, R, 1><<<C.nitems, 64, 0, st>>>(lenv, lidx, renv, ridx,
                                                            (const cx<T>*)C.vals, C.sub_off,
                                                            C.items, cores + off(p), part);
        else
          inner_ir_kernel<T, R, 0><<<C.nitems, 64, 0, st>>>(lenv, lidx, renv, ridx,
                                                            (const cx<T>*)C.vals, C.sub_off,
                                                            C.items, cores + off(p), part);
      }
      inner_grad_kernel<T, R><<<C.nblocks, 64, 0, st>>>(part, C.tile_items, grad + off(p));
    }
    BFC_HIP_TRY(hipGetLastError());
  }
  const int64_t m = P->nparams;
  if (out_fp64)
    grad_out_kernel<T, double><<<grid_for(m), 256, 0, st>>>(grad, (double*)out, m, scale);
  else
    grad_out_kernel<T, float><<<grid_for(m), 256, 0, st>>>(grad, (float*)out, m, scale);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <typename T, int R>
struct LossGradF {
  static bfc_status run(Problem* P, float scale, void* out, int out_fp64, hipStream_t st) {
    return loss_gradient_t<T, R>(P, scale, out, out_fp64, st);
  }
};

bfc_status launch_loss_gradient(Problem* P, float scale, void* out, int out_fp64,
                                hipStream_t st) {
  return dispatch<LossGradF>(P->prec, P->r, P, scale, out, out_fp64, st);
}

bfc_status launch_random_cores(Problem* P, uint64_t seed, hipStream_t st) {
  const int64_t m = P->nparams;
  invalidate_envs(P);
  const double sd = sqrt(0.5 / P->r);
  if (P->prec == BFC_C128)
    random_cores_kernel<double><<<grid_for(m), 256, 0, st>>>((cx<double>*)P->cores, m, seed, sd);
  else
    random_cores_kernel<float><<<grid_for(m), 256, 0, st>>>((cx<float>*)P->cores, m, seed, sd);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

}  // namespace bfc
