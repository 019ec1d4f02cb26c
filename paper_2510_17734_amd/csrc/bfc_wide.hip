// ALS core updates at the wide ranks (Alg. "ALS for Butterfly Completion",
// Sec. 5.1.1): the same normal equations, regularization and ladder as the
// one-wavefront kernels, laid out for r^2 = 81 .. 144 unknowns per slice.
// Both precisions form the Gram matrices in FP64 (products of the stored
// complex64 or complex128 values, FP64 MFMA): these kernels are bound by
// gathers and synchronization rather than by matrix throughput, and an
// FP64 Gram needs no rounding floor in the regularization, which at
// d = r^2 = 144 unknowns would be large (d times the floor).
#include "bfc_device.h"
#include "bfc_wide.h"

namespace bfc {

namespace {

// ---------------------------------------------------------------------------
// Ranks 9 .. 12 (the ranks the paper runs for its c = 4 Green's-function grids
// and the Radon transform, Sec. 6.1 and 6.3).  There the one-wavefront kernels
// above run out of registers (the inner Gram's r^2 + 2r wide rows) and LDS
// (the d = r^2 system), so both ALS updates have kernels of their own:
//
// * outer cores: one wavefront per fiber.  Chunks of 64 entries are staged in
//   LDS; each lane accumulates its share of the r(r+1)/2 entries of the lower
//   triangle of K = sum conj(a_e) a_e^T and of h = sum conj(a_e) t_e; the
//   regularized system is factored column by column in LDS by the wavefront.
// * inner cores: one workgroup per slice, Gram and solve fused.  With
//   1024 threads per slice: batches of 16 subgroups are gathered by one
//   wavefront each, which also forms the subgroup's real-coordinate rows (as
//   in the one-wavefront kernel); the 16 wavefronts take the MFMA tiles of
//   S = A^T B in turn, and only the tiles the system reads are computed (the
//   K block and the right-hand-side corner).  S goes to the slice's region
//   of device memory (it does not fit in LDS at r = 12); the bordered system
//   is assembled from it into registers over a thread grid and factored
//   there (reg_cholesky): at r <= 11 by a launch of its own over a 16 x 16
//   grid, at r = 12 by the same workgroup over a 32 x 32 grid (WideGeom).
//   The factor's rows replace S in the region, and a last launch
//   back-substitutes with one wavefront per slice.
// ---------------------------------------------------------------------------
constexpr int kWideSub = 16;       // subgroups per batch of the fused inner kernel
constexpr int kWideThreads = 1024;  // threads of the fused inner kernel

template <typename T>
__device__ __attribute__((always_inline)) inline cx<double> widen(cx<T> v) {
  return {(double)v.x, (double)v.y};
}

template <int R>
struct WideGeom {
  static constexpr int D = R * R;
  static constexpr int W = D + 2 * R;
  static constexpr int WP = (W + 15) / 16 * 16;
  static constexpr int NB = WP / 16;
  static constexpr int LDW = WP + 1;          // padded LDS row
  // The factorization runs in a launch of its own over a 16 x 16 thread grid
  // (four wavefronts, one per SIMD, up to 512 registers a lane) where that
  // leaves two workgroups per CU (r <= 11: at most 230 registers); at r = 12
  // it needs 316, one workgroup per CU, and runs faster inside the Gram's
  // 1024-thread workgroup over a 32 x 32 grid.
  static constexpr bool SPLIT = R <= 11;
  static constexpr int G = SPLIT ? 16 : 32;   // factorization grid: G x G threads
  static constexpr int NS = RegGrid<D, G>::NS;
  static constexpr size_t S_BYTES = (size_t)WP * WP * 8;
  static constexpr size_t F_BYTES = (size_t)D * (D + 1) / 2 * 16;
  // after the factorization: the factor's rows, then w = L^-1 (h + lam s_old)
  // and a status value (1: factored, 0: no rung of the ladder was)
  static constexpr size_t FW_BYTES = F_BYTES + (size_t)(D + 1) * 16;
  static constexpr size_t REGION = S_BYTES > FW_BYTES ? S_BYTES : FW_BYTES;
};

// MFMA tile (x, y) of S is read by the system: the K block (coordinates
// below D on both sides) or the right-hand-side corner (at or above D).
template <int R>
__device__ __host__ constexpr bool wide_tile_needed(int x, int y) {
  return (x * 16 < R * R && y * 16 < R * R) || ((x + 1) * 16 > R * R && (y + 1) * 16 > R * R);
}

template <int R>
constexpr int wide_tiles() {
  int n = 0;
  for (int x = 0; x < WideGeom<R>::NB; ++x)
    for (int y = 0; y < WideGeom<R>::NB; ++y) n += wide_tile_needed<R>(x, y) ? 1 : 0;
  return n;
}

// One real coordinate (index k = p R + q) of conj(v) v^T, as in herm_acc,
// in FP64 (exact for complex64 inputs up to the one final rounding).
template <typename T>
__device__ __attribute__((always_inline)) inline double herm_value(const cx<T>* v, int p, int q) {
  const double px = v[p].x, py = v[p].y, qx = v[q].x, qy = v[q].y;
  if (p == q) return px * px + py * py;
  if (p < q) return px * qx + py * qy;
  return qx * py - qy * px;
}

// Wavefront Cholesky of the leading d x d block of M (row-major, leading
// dimension ld, lower triangle read and written) in LDS; every lane returns
// the same value (false at the first pivot that is not positive).
__device__ inline bool wave_cholesky_lds(double2* M, int ld, int d, int lane) {
  for (int k = 0; k < d; ++k) {
    const double p = M[k * ld + k].x;
    if (!(p > 0.0)) return false;
    const double sq = sqrt(p), rs = 1.0 / sq;
    wave_sync();  // every lane has read the pivot
    const int i = k + 1 + lane;
    if (i < d) {
      M[i * ld + k].x *= rs;
      M[i * ld + k].y *= rs;
    }
    if (lane == 0) M[k * ld + k] = make_double2(sq, 0.0);
    wave_sync();
    const int m = d - k - 1;
    for (int t = lane; t < m * m; t += 64) {
      const int ii = k + 1 + t / m, jj = k + 1 + t % m;
      if (jj <= ii) {  // a_ij -= l_ik conj(l_jk)
        const double2 a = M[ii * ld + k], b = M[jj * ld + k];
        M[ii * ld + jj].x -= a.x * b.x + a.y * b.y;
        M[ii * ld + jj].y -= a.y * b.x - a.x * b.y;
      }
    }
    wave_sync();
  }
  return true;
}

// Outer core update at ranks above the one-wavefront kernels' range: one
// wavefront per fiber (the fiber's r unknowns, its entries blk_off[b] ..
// blk_off[b+1]).  The Gram is accumulated in FP64 from the stored values in
// both precisions, and the regularized solve is FP64.
template <typename T, int R>
__global__ __launch_bounds__(64) void outer_wide_kernel(WideOuterArgs<T> A) {
  constexpr int NP = R * (R + 1) / 2;  // lower-triangle entries of K
  constexpr int NJ = NP + R;           // and the right-hand side
  constexpr int JL = (NJ + 63) / 64;   // per lane
  constexpr int LD = R + 1;
  __shared__ cx<T> vs[64][R];
  __shared__ cx<T> ts[64];
  __shared__ double2 M[R * LD];
  __shared__ double2 hv[R];
  __shared__ double2 yv[R];
  const int lane = threadIdx.x;
  const int b = xcd_swizzle(blockIdx.x, gridDim.x);
  if (b >= A.nblocks) return;
  const int e0 = A.blk_off[b], e1 = A.blk_off[b + 1];
  if (e0 == e1) return;  // no observed entry: keep the fiber
  // the lane's jobs: lower-triangle pairs (i, j) in packed order, then h
  int ji[JL], jj[JL];
#pragma unroll
  for (int q = 0; q < JL; ++q) {
    const int job = lane + 64 * q;
    int i = 0;
    while (i < R && (i + 1) * (i + 2) / 2 <= job) ++i;
    ji[q] = job < NP ? i : (job < NJ ? job - NP : -1);
    jj[q] = job < NP ? job - i * (i + 1) / 2 : -1;
  }
  cx<double> acc[JL];  // FP64 accumulation in both precisions
#pragma unroll
  for (int q = 0; q < JL; ++q) acc[q] = cx<double>{0.0, 0.0};
  for (int base = e0; base < e1; base += 64) {
    const int e = base + lane;
    if (e < e1) {
      const cx<T>* v = A.env + (int64_t)A.env_idx[e] * R;
#pragma unroll
      for (int k = 0; k < R; ++k) vs[lane][k] = v[k];
      ts[lane] = A.vals[e];
    }
    wave_sync();
    const int cnt = e1 - base < 64 ? e1 - base : 64;
    for (int u = 0; u < cnt; ++u) {
#pragma unroll
      for (int q = 0; q < JL; ++q) {
        const int job = lane + 64 * q;
        if (job < NP)
          cfma_conj(acc[q], widen(vs[u][ji[q]]), widen(vs[u][jj[q]]));
        else if (job < NJ)
          cfma_conj(acc[q], widen(vs[u][ji[q]]), widen(ts[u]));
      }
    }
    wave_sync();
  }
  // K = sum conj(v_i) v_j (i >= j) into M's lower triangle, h into hv
  double kd[JL][2];
#pragma unroll
  for (int q = 0; q < JL; ++q) {
    const int job = lane + 64 * q;
    kd[q][0] = acc[q].x;
    kd[q][1] = acc[q].y;
    if (job >= NP && job < NJ) hv[ji[q]] = make_double2(kd[q][0], kd[q][1]);
    if (job < NP && ji[q] == jj[q]) M[ji[q] * LD + ji[q]] = make_double2(kd[q][0], 0.0);
  }
  wave_sync();
  double tr = 0.0;
  for (int i = 0; i < R; ++i) tr += M[i * LD + i].x;  // the same order in every lane
  const double tau = tr / R;
  const double unit = fmax(A.reg_floor, 0x1p-53);
  double lam = fmax(A.reg_rel, R * A.reg_floor) * tau;
  cx<T>* fiber = A.fibers + (int64_t)b * R;
  bool ok = false;
  int attempt = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, R * unit * tau);
    }
    wave_sync();  // every lane is done with the previous attempt's M
#pragma unroll
    for (int q = 0; q < JL; ++q) {
      const int job = lane + 64 * q;
      if (job < NP)
        M[ji[q] * LD + jj[q]] =
            make_double2(kd[q][0] + (ji[q] == jj[q] ? lam : 0.0), ji[q] == jj[q] ? 0.0 : kd[q][1]);
    }
    wave_sync();
    ok = wave_cholesky_lds(M, LD, R, lane);
    if (ok) break;
  }
  if (!ok) {
    if (lane == 0) atomicAdd(A.flags, 1);
    return;
  }
  if (lane == 0 && attempt > 0) atomicAdd(A.flags + 1, 1);
  // L y = h + lam z_old, then L^H z = y (column by column)
  if (lane < R) {
    double2 h = hv[lane];
    if (A.prox) {
      h.x += lam * (double)fiber[lane].x;
      h.y += lam * (double)fiber[lane].y;
    }
    yv[lane] = h;
  }
  wave_sync();
  for (int k = 0; k < R; ++k) {
    const double inv = 1.0 / M[k * LD + k].x;
    const double2 yk = make_double2(yv[k].x * inv, yv[k].y * inv);
    wave_sync();
    if (lane == k) yv[k] = yk;
    if (lane > k && lane < R) {  // y_i -= l_ik y_k
      const double2 l = M[lane * LD + k];
      yv[lane].x -= l.x * yk.x - l.y * yk.y;
      yv[lane].y -= l.x * yk.y + l.y * yk.x;
    }
    wave_sync();
  }
  for (int k = R - 1; k >= 0; --k) {
    const double inv = 1.0 / M[k * LD + k].x;
    const double2 zk = make_double2(yv[k].x * inv, yv[k].y * inv);
    wave_sync();
    if (lane == k) yv[k] = zk;
    if (lane < k) {  // y_i -= conj(l_ki) z_k
      const double2 l = M[k * LD + lane];
      yv[lane].x -= l.x * zk.x + l.y * zk.y;
      yv[lane].y -= l.x * zk.y - l.y * zk.x;
    }
    wave_sync();
  }
  if (lane < R) fiber[lane] = cx<T>{T(yv[lane].x), T(yv[lane].y)};
}


// Fused Gram and solve of one inner slice (blockIdx -> slice), ranks 9..12.
// The slice's subgroups are those of its work items (one item per slice at
// these ranks), summed in subgroup order, so results do not depend on
// scheduling.
template <typename T, int R>
__device__ void factor_slice(const WideArgs<T>& A, int tile, double* S);

template <typename T, int R, int BYROW>
__global__ __launch_bounds__(kWideThreads) void inner_wide_kernel(WideArgs<T> A) {
  typedef WideGeom<R> G;
  constexpr int D = G::D, W = G::W, WP = G::WP, NB = G::NB, LDW = G::LDW;
  constexpr int NT = kWideThreads, NW = NT / 64;
  constexpr int NTILE = wide_tiles<R>(), TPW = (NTILE + NW - 1) / NW;
  static_assert(kWideSub == NW, "one wavefront per subgroup of a batch");
  typedef Mfma<double>::acc_t acc_t;  // the Gram in FP64 in both precisions
  __shared__ cx<T> us[kWideSub][R];              // each subgroup's shared environment
  __shared__ cx<T> vs[kWideSub][kSubgroup][R];   // its entries' other environment
  __shared__ cx<T> ts[kWideSub][kSubgroup];      // its entries' values
  __shared__ double As[kWideSub * LDW];
  __shared__ double Bs[kWideSub * LDW];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int it0 = A.tile_items[tile], it1 = A.tile_items[tile + 1];
  if (it0 == it1) return;  // no observed entry in this slice: keep it
  const int s_beg = A.items[it0].sub0, s_end = A.items[it1 - 1].sub1;
  // the wavefront's MFMA tiles: needed tiles wave, wave + NW, ... in row order
  int tx[TPW], ty[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) {
    const int want = wave + NW * q;
    tx[q] = -1;
    ty[q] = 0;
    int cnt = 0;
    for (int x = 0; x < NB; ++x)
      for (int y = 0; y < NB; ++y)
        if (wide_tile_needed<R>(x, y)) {
          if (cnt == want) {
            tx[q] = x;
            ty[q] = y;
          }
          ++cnt;
        }
  }
  acc_t acc[TPW];
#pragma unroll
  for (int q = 0; q < TPW; ++q) acc[q] = acc_t{0.0, 0.0, 0.0, 0.0};
  const cx<T> zero = {T(0), T(0)};
  for (int base = s_beg; base < s_end; base += kWideSub) {
    {  // gather: wavefront `wave` takes subgroup base + wave
      const int s = base + wave;
      const bool live = s < s_end;
      int e0 = 0, e1 = 0;
      if (live) {
        e0 = A.sub_off[s];
        e1 = A.sub_off[s + 1];
      }
      const int32_t* sidx = BYROW ? A.lidx : A.ridx;
      const cx<T>* ssrc = BYROW ? A.lenv : A.renv;
      const int32_t* eidx = BYROW ? A.ridx : A.lidx;
      const cx<T>* esrc = BYROW ? A.renv : A.lenv;
      if (lane < R) us[wave][lane] = live ? ssrc[(int64_t)sidx[e0] * R + lane] : zero;
      for (int j = lane; j < kSubgroup * R; j += 64) {
        const int q = j / R, k = j - q * R;
        vs[wave][q][k] = (e0 + q < e1) ? esrc[(int64_t)eidx[e0 + q] * R + k] : zero;
      }
      if (lane < kSubgroup) ts[wave][lane] = (e0 + lane < e1) ? A.vals[e0 + lane] : zero;
    }
    wave_sync();
    {  // the subgroup's rows: A = shared side, B = the sum over its entries
       // (row case; the column case swaps them and conjugates the RHS parts)
      double* arow = As + wave * LDW;
      double* brow = Bs + wave * LDW;
      for (int k = lane; k < WP; k += 64) {
        double a = 0.0, bv = 0.0;
        if (k < D) {
          const int p = k / R, q = k - p * R;
          const double hs = herm_value<T>(us[wave], p, q);
          double he = 0.0;
#pragma unroll
          for (int e = 0; e < kSubgroup; ++e) he += herm_value<T>(vs[wave][e], p, q);
          a = BYROW ? hs : he;
          bv = BYROW ? he : hs;
        } else if (k < W) {
          const int c = (k - D) % R;
          const bool im = k - D >= R;
          cx<double> y = {0.0, 0.0};  // sum conj(v_e) t_e at coordinate c
#pragma unroll
          for (int e = 0; e < kSubgroup; ++e) cfma_conj(y, widen(vs[wave][e][c]), widen(ts[wave][e]));
          const cx<double> u = widen(us[wave][c]);
          if (BYROW) {
            a = im ? u.y : u.x;
            bv = im ? y.y : y.x;
          } else {
            a = im ? -y.y : y.x;
            bv = im ? -u.y : u.x;
          }
        }
        arow[k] = a;
        brow[k] = bv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kWideSub; kk += 4) {
      const int g = kk + (lane >> 4), c16 = lane & 15;
#pragma unroll
      for (int q = 0; q < TPW; ++q)
        if (tx[q] >= 0) {
          const double xa = As[g * LDW + tx[q] * 16 + c16];
          const double yb = Bs[g * LDW + ty[q] * 16 + c16];
          acc[q] = Mfma<double>::step(xa, yb, acc[q]);
        }
    }
    // the next batch writes us/vs/ts first; its rows only after the barrier
    // above has been passed by every wavefront, i.e. after these reads
    __syncthreads();
  }
  double* S = (double*)(A.region + (size_t)it0 * G::REGION);
#pragma unroll
  for (int q = 0; q < TPW; ++q)
    if (tx[q] >= 0)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = tx[q] * 16 + Mfma<double>::out_row(lane, v);
        const int cl = ty[q] * 16 + (lane & 15);
        S[row * WP + cl] = acc[q][v];
      }
  if constexpr (!G::SPLIT) {
    static_assert(G::G * G::G == NT, "the fused factorization's grid is the workgroup");
    // S passes between the workgroup's threads through device memory; the
    // workgroup barrier orders it (one CU, one L1 and L2: no device-scope
    // fence, which on this chip writes back and invalidates the XCD's L2)
    __syncthreads();
    factor_slice<T, R>(A, tile, S);
  }
}

// The bordered system of one slice (blockIdx -> slice) assembled from its
// Gram S in the slice's region into registers over a 16 x 16 thread grid
// and factored there (reg_cholesky, one column per barrier of the grid's
// four wavefronts, one per SIMD); the regularization ladder re-reads S.
// The bordered system of a slice assembled from its Gram S (in the slice's
// region) into registers over the G x G grid of the calling threads and
// factored there (reg_cholesky, one column per barrier); the
// regularization ladder re-reads S.  Leaves the factor's rows, w and the
// status over S for the back substitution.  Every thread of the workgroup
// calls it (the grid is the whole workgroup).
template <typename T, int R>
__device__ void factor_slice(const WideArgs<T>& A, int tile, double* S) {
  typedef WideGeom<R> G;
  constexpr int D = G::D, WP = G::WP, GG = G::G, NS = G::NS, NT = GG * GG;
  __shared__ double2 col[2 * (D + 1)];
  __shared__ double2 hb[D];
  __shared__ double2 ob[D];
  __shared__ double dg[D];
  const int tid = threadIdx.x;
  cx<T>* slice = A.slices + (int64_t)tile * D;
  for (int i = tid; i < D; i += NT) {
    dg[i] = inner_K<R>(S, WP, i, i).x;
    hb[i] = inner_h<R>(S, WP, i);
    const cx<T> o = slice[i];
    ob[i] = A.prox ? make_double2((double)o.x, (double)o.y) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  double tr = 0.0;
  for (int i = 0; i < D; ++i) tr += dg[i];  // the same order in every thread
  const double tau = tr / D;
  const double unit = fmax(A.reg_floor, 0x1p-53);
  double lam = fmax(A.reg_rel, D * A.reg_floor) * tau;
  const int ga = tid / GG, gc = tid % GG;
  double mr[NS][NS], mi[NS][NS];
  bool ok = false;
  int attempt = 0;
  int opaque = 0;
  for (; attempt < 4; ++attempt) {
    if (attempt > 0) {
      if (!(lam > 0.0)) break;
      lam = fmax(100.0 * lam, D * unit * tau);
    }
    // S is re-read on every attempt: an offset the compiler cannot see
    // through keeps the slots' index arithmetic, addresses and loads inside
    // the loop (hoisted, they would hold more registers than the grid's
    // threads have)
    asm volatile("" : "+s"(opaque));
    const double* Sa = S + opaque;
    const int ga_ = ga + opaque, gc_ = gc + opaque;
#pragma unroll
    for (int ia = 0; ia < NS; ++ia)
#pragma unroll
      for (int jc = 0; jc <= ia; ++jc) {
        const int i = ga_ + GG * ia, j = gc_ + GG * jc;
        double2 v = make_double2(0.0, 0.0);
        if (i < D && j <= i) {
          v = inner_K<R>(Sa, WP, i, j);
          if (i == j) v.x += lam;
        } else if (i == D && j < D) {  // border row: conj(h_j + lam s_old_j)
          const double2 h = hb[j], o = ob[j];
          v = make_double2(h.x + lam * o.x, -(h.y + lam * o.y));
        }
        mr[ia][jc] = v.x;
        mi[ia][jc] = v.y;
      }
    ok = reg_cholesky<D, GG, NS>(mr, mi, ga, gc, col);
    if (ok) break;
    __syncthreads();  // every thread is done with the failed attempt's column buffers
  }
  // every thread finished reading S before the factorization's first
  // barrier: the factor's rows (packed, L_ij at i (i + 1) / 2 + j), w (from
  // the border row, conj(w)) and the status go over it
  double2* F = (double2*)S;
  double2* Wv = F + D * (D + 1) / 2;
  if (!ok) {
    if (tid == 0) {
      atomicAdd(A.flags, 1);
      Wv[D] = make_double2(0.0, 0.0);
    }
    return;
  }
  if (tid == 0) {
    if (attempt > 0) atomicAdd(A.flags + 1, 1);
    Wv[D] = make_double2(1.0, 0.0);
  }
#pragma unroll
  for (int ia = 0; ia < NS; ++ia)
#pragma unroll
    for (int jc = 0; jc <= ia; ++jc) {
      const int i = ga + GG * ia, j = gc + GG * jc;
      if (i < D && j <= i) F[i * (i + 1) / 2 + j] = make_double2(mr[ia][jc], mi[ia][jc]);
      if (i == D && j < D) Wv[j] = make_double2(mr[ia][jc], -mi[ia][jc]);
    }
}

// The factorization as a launch of its own (ranks with G::SPLIT).
template <typename T, int R>
__global__ __launch_bounds__(WideGeom<R>::G * WideGeom<R>::G) void wide_factor_kernel(
    WideArgs<T> A) {
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int it0 = A.tile_items[tile], it1 = A.tile_items[tile + 1];
  if (it0 == it1) return;  // no observed entry in this slice: keep it
  factor_slice<T, R>(A, tile, (double*)(A.region + (size_t)it0 * WideGeom<R>::REGION));
}

// Back substitution L^H s = w of every factored slice, one wavefront per
// slice (a launch after the fused kernel, so that many slices overlap the
// latency of their factor rows).  Rows k0 .. k0+3 per step: every lane
// solves the 4 x 4 diagonal block itself and updates its entries j < k0;
// the next step's rows are loaded while the current one is used.
template <typename T, int R>
__global__ __launch_bounds__(64) void wide_backsub_kernel(WideArgs<T> A) {
  typedef WideGeom<R> G;
  constexpr int D = G::D, TB = 4, JP = (D + 63) / 64;
  __shared__ double2 ys[D];
  const int lane = threadIdx.x;
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x);
  const int it0 = A.tile_items[tile], it1 = A.tile_items[tile + 1];
  if (it0 == it1) return;
  const double2* F = (const double2*)(A.region + (size_t)it0 * G::REGION);
  const double2* Wv = F + D * (D + 1) / 2;
  if (!(Wv[D].x > 0.0)) return;  // not factored: the slice keeps its values
  for (int j = lane; j < D; j += 64) ys[j] = Wv[j];
  wave_sync();
  // the factor values one step uses: the diagonal block and rows k0+q at
  // the lane's entries j = lane + 64 p < k0
  double2 dd[TB][TB], lr[TB][JP];
  auto fetch = [&](int k0, double2 (&d)[TB][TB], double2 (&l)[TB][JP]) {
    const int nb = D - k0 < TB ? D - k0 : TB;
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const int r0 = (k0 + q) * (k0 + q + 1) / 2;
#pragma unroll
      for (int t = 0; t < TB; ++t)
        d[q][t] = (q < nb && t <= q) ? F[r0 + k0 + t] : make_double2(t == q ? 1.0 : 0.0, 0.0);
#pragma unroll
      for (int p = 0; p < JP; ++p) {
        const int j = lane + 64 * p;
        l[q][p] = (q < nb && j < k0) ? F[r0 + j] : make_double2(0.0, 0.0);
      }
    }
  };
  int k0 = ((D - 1) / TB) * TB;
  fetch(k0, dd, lr);
#pragma unroll 1
  for (; k0 >= 0; k0 -= TB) {
    double2 dn[TB][TB], ln[TB][JP];
    if (k0 >= TB) fetch(k0 - TB, dn, ln);
    const int nb = D - k0 < TB ? D - k0 : TB;
    double2 yb[TB], sb[TB];
#pragma unroll
    for (int q = 0; q < TB; ++q) yb[q] = q < nb ? ys[k0 + q] : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = TB - 1; q >= 0; --q) {  // s_q = (y_q - sum_{t>q} conj(L_tq) s_t) / L_qq
      double2 v = yb[q];
#pragma unroll
      for (int t = q + 1; t < TB; ++t) {
        v.x -= dd[t][q].x * sb[t].x + dd[t][q].y * sb[t].y;
        v.y -= dd[t][q].x * sb[t].y - dd[t][q].y * sb[t].x;
      }
      const double rr = 1.0 / dd[q][q].x;
      sb[q] = make_double2(v.x * rr, v.y * rr);
    }
    wave_sync();  // every lane has read the block's y
#pragma unroll
    for (int p = 0; p < JP; ++p) {  // y_j -= sum_q conj(L_(k0+q) j) s_q
      const int j = lane + 64 * p;
      if (j < k0) {
        double2 y = ys[j];
#pragma unroll
        for (int q = 0; q < TB; ++q) {
          y.x -= lr[q][p].x * sb[q].x + lr[q][p].y * sb[q].y;
          y.y -= lr[q][p].x * sb[q].y - lr[q][p].y * sb[q].x;
        }
        ys[j] = y;
      }
    }
#pragma unroll
    for (int q = 0; q < TB; ++q)
      if (lane == q && q < nb) ys[k0 + q] = sb[q];
    wave_sync();
    if (k0 >= TB) {
#pragma unroll
      for (int q = 0; q < TB; ++q) {
#pragma unroll
        for (int t = 0; t < TB; ++t) dd[q][t] = dn[q][t];
#pragma unroll
        for (int p = 0; p < JP; ++p) lr[q][p] = ln[q][p];
      }
    }
  }
  cx<T>* slice = A.slices + (int64_t)tile * D;
  for (int j = lane; j < D; j += 64) slice[j] = cx<T>{T(ys[j].x), T(ys[j].y)};
}

}  // namespace

template <typename T, int R>
bfc_status launch_outer_wide(const WideOuterArgs<T>& a, hipStream_t st) {
  if (a.nblocks > 0) outer_wide_kernel<T, R><<<a.nblocks, 64, 0, st>>>(a);
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

template <typename T, int R>
bfc_status launch_inner_wide(const WideArgs<T>& a, int nslices, int by_row, hipStream_t st) {
  if (nslices > 0) {
    if (by_row)
      inner_wide_kernel<T, R, 1><<<nslices, kWideThreads, 0, st>>>(a);
    else
      inner_wide_kernel<T, R, 0><<<nslices, kWideThreads, 0, st>>>(a);
    BFC_HIP_TRY(hipGetLastError());
    if constexpr (WideGeom<R>::SPLIT) {
      wide_factor_kernel<T, R><<<nslices, WideGeom<R>::G * WideGeom<R>::G, 0, st>>>(a);
      BFC_HIP_TRY(hipGetLastError());
    }
    wide_backsub_kernel<T, R><<<nslices, 64, 0, st>>>(a);
  }
  BFC_HIP_TRY(hipGetLastError());
  return BFC_OK;
}

size_t wide_region_bytes(int r) {
  switch (r) {
    case 9: return WideGeom<9>::REGION;
    case 10: return WideGeom<10>::REGION;
    case 11: return WideGeom<11>::REGION;
    case 12: return WideGeom<12>::REGION;
    default: return 0;
  }
}

#define BFC_WIDE_INST(T, R)                                                                     \
  template bfc_status launch_outer_wide<T, R>(const WideOuterArgs<T>&, hipStream_t);          \
  template bfc_status launch_inner_wide<T, R>(const WideArgs<T>&, int, int, hipStream_t);
BFC_WIDE_INST(double, 9)
BFC_WIDE_INST(double, 10)
BFC_WIDE_INST(double, 11)
BFC_WIDE_INST(double, 12)
BFC_WIDE_INST(float, 9)
BFC_WIDE_INST(float, 10)
BFC_WIDE_INST(float, 11)
BFC_WIDE_INST(float, 12)
#undef BFC_WIDE_INST

}  // namespace bfc
