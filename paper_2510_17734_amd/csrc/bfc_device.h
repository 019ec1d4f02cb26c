// Device-side building blocks of the butterfly ALS kernels.
#pragma once

#include "bfc_common.h"

namespace bfc {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// Core storage: Z^1 (n x R) at 0, inner core q (q = 1..L, the paper's
// Z^(q+1)) at n*R + (q-1) * 2^(L+1) * R*R, Z^(L+2) (n x R) after them.
__host__ __device__ inline int64_t inner_off(int64_t n, int L, int R, int q) {
  return n * R + (int64_t)(q - 1) * ((int64_t)1 << (L + 1)) * R * R;
}
__host__ __device__ inline int64_t last_off(int64_t n, int L, int R) {
  return n * R + (int64_t)L * ((int64_t)1 << (L + 1)) * R * R;
}

// Slice index of inner core q for leaf blocks (ib, jb): psi^{-1} of
// (i_0..i_(L-q), j_0..j_(q-1)), i.e. the top L-q+1 bits of ib followed by the
// top q bits of jb (App. A.2, eq. (reshaped_tensors)).
__host__ __device__ inline uint32_t slice_key(uint32_t ib, uint32_t jb, int L, int q) {
  return ((ib >> (q - 1)) << q) | (jb >> (L - q));
}

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2.  xcd_swizzle maps the hardware block index so that each
// XCD receives a contiguous range of logical blocks (blocks that share data
// then share an L2).  A bijection on [0, nblocks).
__device__ inline int xcd_swizzle(int bid, int nblocks) {
  constexpr int kXcd = 8;
  const int per = nblocks / kXcd, rem = nblocks % kXcd;
  const int x = bid % kXcd, q = bid / kXcd;
  // XCD x owns logical blocks [start_x, start_x + per + (x < rem))
  const int start = x * per + (x < rem ? x : rem);
  return start + q;
}

// Work of one launch split into tasks (one per instance of a batch): a
// batched kernel reads its task's arguments from `tasks` and its block index
// within the task from the prefix table `block_off` (ntasks + 1 entries).
__device__ __attribute__((always_inline)) inline int find_task(const int32_t* block_off,
                                                               int ntasks, int b) {
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {  // last task with block_off[t] <= b
    const int mid = (lo + hi + 1) >> 1;
    if (block_off[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// v <- the R-vector at src + idx * R.  WIDE: two complex64 values per
// 16-byte load where R is even (the vectors then start on 16-byte
// boundaries); it costs registers, so only kernels with room use it.
template <typename T, int R, bool WIDE = false>
__device__ inline void load_env(const cx<T>* __restrict__ src, int idx, cx<T> (&v)[R]) {
  const cx<T>* p = src + (int64_t)idx * R;
  if constexpr (WIDE && sizeof(T) == 4 && R % 2 == 0) {
    const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int k = 0; k < R / 2; ++k) {
      const float4 t = q[k];
      v[2 * k] = cx<T>{t.x, t.y};
      v[2 * k + 1] = cx<T>{t.z, t.w};
    }
  } else {
#pragma unroll
    for (int a = 0; a < R; ++a) v[a] = p[a];
  }
}

// Marks a loaded value as used here.  Placed after a group of loads, it keeps
// the compiler from moving any of them into the conditional code that
// consumes it: every load of the group is in flight before the first wait,
// so the group costs one memory latency instead of one per load.
template <typename T>
__device__ __attribute__((always_inline)) inline void pin(cx<T>& v) {
  asm volatile("" : "+v"(v.x), "+v"(v.y));
}

// Environment vectors and values of G entries, loaded as one group.  An absent
// entry (id < 0) reads vector 0 and value 0 (both exist whenever the kernel
// runs) and must be skipped by the caller.
template <typename T, int R, int G, bool WIDE = false>
__device__ __attribute__((always_inline)) inline void gather_group(
    const cx<T>* __restrict__ src, const cx<T>* __restrict__ vals, const int (&id)[G],
    const int (&ent)[G], cx<T> (&v)[G][R], cx<T> (&t)[G]) {
#pragma unroll
  for (int g = 0; g < G; ++g) {
    load_env<T, R, WIDE>(src, id[g] >= 0 ? id[g] : 0, v[g]);
    t[g] = vals[id[g] >= 0 ? ent[g] : 0];
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
#pragma unroll
    for (int a = 0; a < R; ++a) pin(v[g][a]);
    pin(t[g]);
  }
}

// v <- v * Z   (row vector times an R x R slice)
template <typename T, int R>
__device__ inline void vec_mat(cx<T> (&v)[R], const cx<T>* __restrict__ Z) {
  cx<T> o[R];
#pragma unroll
  for (int b = 0; b < R; ++b) o[b] = {T(0), T(0)};
#pragma unroll
  for (int a = 0; a < R; ++a) {
#pragma unroll
    for (int b = 0; b < R; ++b) cfma(o[b], v[a], Z[a * R + b]);
  }
#pragma unroll
  for (int b = 0; b < R; ++b) v[b] = o[b];
}

// w <- Z * w   (R x R slice times a column vector)
template <typename T, int R>
__device__ inline void mat_vec(const cx<T>* __restrict__ Z, cx<T> (&w)[R]) {
  cx<T> o[R];
#pragma unroll
  for (int a = 0; a < R; ++a) {
    o[a] = {T(0), T(0)};
#pragma unroll
    for (int b = 0; b < R; ++b) cfma(o[a], Z[a * R + b], w[b]);
  }
#pragma unroll
  for (int a = 0; a < R; ++a) w[a] = o[a];
}

// Left environment of core p (1 <= p <= L+1): Z^1[i] Z^2[k] ... Z^p[k]
// (cores 0..p-1 in the 0-based numbering).
template <typename T, int R>
__device__ inline void left_chain(const cx<T>* __restrict__ cores, int64_t n, int L, int p,
                                  int i, uint32_t ib, uint32_t jb, cx<T> (&v)[R]) {
  const cx<T>* z = cores + (int64_t)i * R;
#pragma unroll
  for (int a = 0; a < R; ++a) v[a] = z[a];
  for (int q = 1; q < p; ++q) {
    const cx<T>* Z = cores + inner_off(n, L, R, q) + (int64_t)slice_key(ib, jb, L, q) * R * R;
    vec_mat<T, R>(v, Z);
  }
}

// Right environment of core p (0 <= p <= L): Z^(p+2)[k] ... Z^(L+1)[k] Z^(L+2)[j]^T
// (cores p+1..L+1 in the 0-based numbering).
template <typename T, int R>
__device__ inline void right_chain(const cx<T>* __restrict__ cores, int64_t n, int L, int p,
                                   int j, uint32_t ib, uint32_t jb, cx<T> (&w)[R]) {
  const cx<T>* z = cores + last_off(n, L, R) + (int64_t)j * R;
#pragma unroll
  for (int a = 0; a < R; ++a) w[a] = z[a];
  for (int q = L; q > p; --q) {
    const cx<T>* Z = cores + inner_off(n, L, R, q) + (int64_t)slice_key(ib, jb, L, q) * R * R;
    mat_vec<T, R>(Z, w);
  }
}

// Real coordinates of the Hermitian outer product H = conj(v) v^T (R*R reals):
//   Rv[a*R+a] = |v_a|^2,  Rv[a*R+b] = Re(conj(v_a) v_b),  Rv[b*R+a] = Im(conj(v_a) v_b)
// for a < b.  acc += Rv.
template <typename T, int R>
__device__ inline void herm_acc(T* acc, const cx<T> (&v)[R]) {
#pragma unroll
  for (int a = 0; a < R; ++a) {
    acc[a * R + a] = fma(v[a].x, v[a].x, fma(v[a].y, v[a].y, acc[a * R + a]));
#pragma unroll
    for (int b = a + 1; b < R; ++b) {
      acc[a * R + b] = fma(v[a].x, v[b].x, fma(v[a].y, v[b].y, acc[a * R + b]));
      acc[b * R + a] = fma(v[a].x, v[b].y, fma(-v[a].y, v[b].x, acc[b * R + a]));
    }
  }
}

// Hermitian matrix entry H[a][b] from its real coordinates Rv (see herm_acc):
// returns (index of the real part, index of the imaginary part or -1, sign).
__host__ __device__ inline void herm_coord(int a, int b, int R, int& re, int& im, int& sg) {
  if (a == b) {
    re = a * R + a; im = -1; sg = 0;
  } else if (a < b) {
    re = a * R + b; im = b * R + a; sg = 1;
  } else {
    re = b * R + a; im = a * R + b; sg = -1;
  }
}

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

// MFMA wrappers: D(16x16) += X(16x4) Y(4x16); lane l supplies X[l%16][l/16]
// and Y[l/16][l%16].  Element v of the accumulator holds D[out_row][l%16];
// the row mapping differs between the FP32 and the FP64 instruction (both
// measured on gfx950 with one-hot inputs).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ inline acc_t step(float x, float y, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};
template <>
struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ inline acc_t step(double x, double y, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  static __device__ inline int out_row(int lane, int v) { return 4 * v + (lane >> 4); }
};

// ---------------------------------------------------------------------------
// Hermitian positive definite solve by one workgroup, d <= 64 unknowns.
// M is row-major with an odd leading dimension ld (element (i, j) at
// i*ld + j), so a row walk across lanes (stride ld) and a column walk
// (consecutive j) both touch distinct LDS banks.
//
// Right-looking blocked Cholesky, panel width kNb.  Per panel every thread
// factors the kNb x kNb diagonal block in registers and inverts the factor
// (Di = L_BB^-1); the rows below then need no substitution chain
// (L_i = a_i Di^H), and the trailing lower triangle is split evenly over the
// workgroup's threads.  The triangular solves reuse the Di blocks, so a panel
// of a solve is one broadcast and two short matrix-vector products.
// ---------------------------------------------------------------------------

// Uniform-lane broadcast of a double (lane index in a scalar register).
__device__ inline double bcast_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

constexpr int kNb = 4;
constexpr int kPanelLd = kNb + 1;  // odd count of 16-byte values per panel row

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cmul_conj(double2 a, double2 b) {  // a * conj(b)
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}

// 1/sqrt(x) for x > 0: hardware estimate and two Newton steps
// y <- y (3 - x y^2) / 2, each of which doubles the correct bits.
__device__ __attribute__((always_inline)) inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
#pragma unroll
  for (int k = 0; k < 2; ++k) y = y * fma(-hx * y, y, 1.5);
  return y;
}

// Factor the nb x nb lower diagonal block at (k0, k0) of M and return the
// inverse of its factor: dg receives the (real) diagonal of L_BB^-1 and
// Di[i][j], i > j, its strictly lower part (rows and columns >= nb are the
// identity).  The diagonal of a Hermitian matrix and of its Cholesky factor
// is real, so only the real parts of pivots are formed and products with
// diagonal entries are real scalings.  False if a pivot is not positive;
// every thread reads the same values and reaches the same answer.
__device__ __attribute__((always_inline)) inline bool diag_block_inverse(
    const double2* M, int ld, int k0, int nb, double (&dg)[kNb], double2 (&Di)[kNb][kNb]) {
  double2 D[kNb][kNb];
  double dd[kNb];
#pragma unroll
  for (int a = 0; a < kNb; ++a) {
    dd[a] = (a < nb) ? M[(k0 + a) * ld + k0 + a].x : 1.0;
#pragma unroll
    for (int b = 0; b < a; ++b)
      D[a][b] = (a < nb) ? M[(k0 + a) * ld + k0 + b] : make_double2(0.0, 0.0);
  }
#pragma unroll
  for (int k = 0; k < kNb; ++k) {
    if (!(dd[k] > 0.0)) return false;
    dg[k] = rsqrt_nr(dd[k]);  // 1 / L[k][k]
#pragma unroll
    for (int i = k + 1; i < kNb; ++i) {
      D[i][k].x *= dg[k];
      D[i][k].y *= dg[k];
    }
#pragma unroll
    for (int j = k + 1; j < kNb; ++j) {
      dd[j] = fma(-D[j][k].x, D[j][k].x, fma(-D[j][k].y, D[j][k].y, dd[j]));
#pragma unroll
      for (int i = j + 1; i < kNb; ++i) {
        const double2 t = cmul_conj(D[i][k], D[j][k]);
        D[i][j].x -= t.x;
        D[i][j].y -= t.y;
      }
    }
  }
  // Di[i][j] = -dg[i] * (L[i][j] dg[j] + sum_{k=j+1}^{i-1} L[i][k] Di[k][j])
#pragma unroll
  for (int j = 0; j < kNb; ++j)
#pragma unroll
    for (int i = j + 1; i < kNb; ++i) {
      double2 s = make_double2(D[i][j].x * dg[j], D[i][j].y * dg[j]);
#pragma unroll
      for (int k = j + 1; k < i; ++k) {
        const double2 t = cmul(D[i][k], Di[k][j]);
        s.x += t.x;
        s.y += t.y;
      }
      Di[i][j] = make_double2(-dg[i] * s.x, -dg[i] * s.y);
    }
  return true;
}

// Row a and column b (b <= a) of entry e of a packed lower triangle.
__device__ __attribute__((always_inline)) inline void tri_coords(int e, int& a, int& b) {
  int t = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  if ((t + 1) * (t + 2) / 2 <= e) ++t;
  if (t * (t + 1) / 2 > e) --t;
  a = t;
  b = e - t * (t + 1) / 2;
}

// In-place blocked lower Cholesky factor of the d x d matrix M by NT threads
// (the whole workgroup; tid = threadIdx.x), with row d of M bordering it:
// the factor of [[K, b], [b^H, *]] has y^H = (L^-1 b)^H in its last row, so
// holding conj(b) in row d on entry gives conj(L^-1 b) there on exit (the
// forward substitution rides along with the factorization).  Below the
// diagonal blocks M receives L; the diagonal blocks of M are left as partial
// updates, and dinv[(k0 / kNb) * kNb * kNb + a * kNb + b] receives
// L_BB^-1[a][b] instead.  panel is (d + 1) * kPanelLd values of scratch.
// Returns false (in every thread) if a pivot is not positive.
template <int NT>
__device__ __attribute__((always_inline)) inline bool wg_cholesky(double2* M, int d, int ld,
                                                                  double2* panel, double2* dinv,
                                                                  int tid) {
#pragma unroll 1
  for (int k0 = 0; k0 < d; k0 += kNb) {
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    double dg[kNb];
    double2 Di[kNb][kNb];
    if (!diag_block_inverse(M, ld, k0, nb, dg, Di)) return false;
    const int r0 = k0 + nb, m = d + 1 - r0;  // rows below the block, border included
    for (int t = tid; t < m; t += NT) {
      double2* row = M + (r0 + t) * ld + k0;
      double2 a[kNb];
#pragma unroll
      for (int q = 0; q < kNb; ++q) a[q] = q < nb ? row[q] : make_double2(0.0, 0.0);
#pragma unroll
      for (int q = 0; q < kNb; ++q) {  // L_i[q] = a[q] dg[q] + sum_{p<q} a[p] conj(Di[q][p])
        double2 l = make_double2(a[q].x * dg[q], a[q].y * dg[q]);
#pragma unroll
        for (int p = 0; p < q; ++p) {
          const double2 s = cmul_conj(a[p], Di[q][p]);
          l.x += s.x;
          l.y += s.y;
        }
        if (q < nb) row[q] = l;
        panel[(r0 + t) * kPanelLd + q] = l;
      }
    }
    if (tid == 0) {  // the full block L_BB^-1 for the triangular solves
#pragma unroll
      for (int a = 0; a < kNb; ++a)
#pragma unroll
        for (int b = 0; b < kNb; ++b)
          dinv[k0 * kNb + a * kNb + b] = a == b  ? make_double2(dg[a], 0.0)
                                         : a > b ? Di[a][b]
                                                 : make_double2(0.0, 0.0);
    }
    __syncthreads();
    // lower triangle of the trailing rows; the border's own diagonal entry
    // (the last one) is never used and is skipped
    const int ne = m * (m + 1) / 2 - 1;
    for (int e = tid; e < ne; e += NT) {
      int a, b;
      tri_coords(e, a, b);
      const double2* pi = panel + (r0 + a) * kPanelLd;
      const double2* pj = panel + (r0 + b) * kPanelLd;
      double2* mij = M + (r0 + a) * ld + r0 + b;
      double2 v = *mij;
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        const double2 s = cmul_conj(pi[q], pj[q]);
        v.x -= s.x;
        v.y -= s.y;
      }
      *mij = v;
    }
    __syncthreads();
  }
  return true;
}

// Solve L^H s = y with the factor of wg_cholesky, by one wavefront: lane i
// holds y_i in a register and ends with s_i (lanes >= d carry nothing of
// use).  Per diagonal block: broadcast the block's running values, multiply
// by L_BB^-H, and subtract the block's contribution from the rows above.
// Reads only LDS (no writes, no barriers).
__device__ __attribute__((always_inline)) inline void wave_back_solve(const double2* M,
                                                                      const double2* dinv, int d,
                                                                      int ld, double2& b,
                                                                      int lane) {
  const int li = lane < d ? lane : 0;
  const int last = ((d - 1) / kNb) * kNb;
  for (int k0 = last; k0 >= 0; k0 -= kNb) {
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    const double2* Di = dinv + k0 * kNb;
    double2 l[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) l[q] = q < nb ? M[(k0 + q) * ld + li] : make_double2(0.0, 0.0);
    double2 bb[kNb], s[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q)
      bb[q] = q < nb ? make_double2(bcast_d(b.x, k0 + q), bcast_d(b.y, k0 + q))
                     : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kNb; ++q) {  // s[q] = sum_{p>=q} conj(Di[p][q]) bb[p], Di[q][q] real
      const double dq = Di[q * kNb + q].x;
      s[q] = make_double2(bb[q].x * dq, bb[q].y * dq);
#pragma unroll
      for (int p = q + 1; p < kNb; ++p) {
        const double2 t = cmul_conj(bb[p], Di[p * kNb + q]);
        s[q].x += t.x;
        s[q].y += t.y;
      }
      if (lane == k0 + q) b = s[q];
    }
    if (lane < k0) {  // b_i -= conj(L[k0+q][i]) s_q
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        const double2 t = cmul_conj(s[q], l[q]);
        b.x -= t.x;
        b.y -= t.y;
      }
    }
  }
}

// Orders LDS writes of one wavefront before its later LDS reads by other
// lanes of the same wavefront.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Sums over one DPP row (16 lanes): butterfly with quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror and row_mirror.  Every lane of the row
// ends with the same, identically ordered sum.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ inline float dpp_f(float v) {
  return __int_as_float(
      __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline float row16_sum(float v) {
  v += dpp_f<0xB1>(v);
  v += dpp_f<0x4E>(v);
  v += dpp_f<0x141>(v);
  v += dpp_f<0x140>(v);
  return v;
}
__device__ inline double row16_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return v;
}

// ---------------------------------------------------------------------------
// Serial Hermitian solve in registers (one lane), small R.
// ---------------------------------------------------------------------------
template <int R>
__device__ __attribute__((always_inline)) inline bool serial_cholesky(double2 (&M)[R][R]) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double piv = M[k][k].x;
    if (!(piv > 0.0)) return false;
    const double lkk = sqrt(piv), inv = 1.0 / lkk;
    M[k][k] = make_double2(lkk, 0.0);
#pragma unroll
    for (int i = k + 1; i < R; ++i) {
      M[i][k].x *= inv;
      M[i][k].y *= inv;
    }
#pragma unroll
    for (int j = k + 1; j < R; ++j)
#pragma unroll
      for (int i = j; i < R; ++i) {
        M[i][j].x -= M[i][k].x * M[j][k].x + M[i][k].y * M[j][k].y;
        M[i][j].y -= M[i][k].y * M[j][k].x - M[i][k].x * M[j][k].y;
      }
  }
  return true;
}

template <int R>
__device__ __attribute__((always_inline)) inline void serial_chol_solve(const double2 (&M)[R][R],
                                                                        double2 (&b)[R]) {
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const double inv = 1.0 / M[k][k].x;
    b[k].x *= inv;
    b[k].y *= inv;
#pragma unroll
    for (int i = k + 1; i < R; ++i) {
      b[i].x -= M[i][k].x * b[k].x - M[i][k].y * b[k].y;
      b[i].y -= M[i][k].x * b[k].y + M[i][k].y * b[k].x;
    }
  }
#pragma unroll
  for (int k = R - 1; k >= 0; --k) {
    const double inv = 1.0 / M[k][k].x;
    b[k].x *= inv;
    b[k].y *= inv;
#pragma unroll
    for (int i = 0; i < k; ++i) {  // b_i -= conj(L[k][i]) s_k
      b[i].x -= M[k][i].x * b[k].x + M[k][i].y * b[k].y;
      b[i].y -= M[k][i].x * b[k].y - M[k][i].y * b[k].x;
    }
  }
}

// Solve L y = b with the factor of wg_cholesky, by one wavefront: lane i
// holds b_i in a register and ends with y_i.  Per diagonal block: broadcast
// the block's running values, multiply by L_BB^-1, and subtract the block's
// contribution from the rows below.  Reads only LDS (no writes, no barriers).
__device__ __attribute__((always_inline)) inline void wave_fwd_solve(const double2* M,
                                                                     const double2* dinv, int d,
                                                                     int ld, double2& b,
                                                                     int lane) {
  const int li = lane < d ? lane : 0;
#pragma unroll 1
  for (int k0 = 0; k0 < d; k0 += kNb) {
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    const double2* Di = dinv + k0 * kNb;
    double2 bb[kNb], s[kNb], l[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q)
      bb[q] = q < nb ? make_double2(bcast_d(b.x, k0 + q), bcast_d(b.y, k0 + q))
                     : make_double2(0.0, 0.0);
#pragma unroll
    for (int q = 0; q < kNb; ++q) {  // s[q] = sum_{p<=q} Di[q][p] bb[p], Di[q][q] real
      const double dq = Di[q * kNb + q].x;
      s[q] = make_double2(bb[q].x * dq, bb[q].y * dq);
#pragma unroll
      for (int p = 0; p < q; ++p) {
        const double2 t = cmul(Di[q * kNb + p], bb[p]);
        s[q].x += t.x;
        s[q].y += t.y;
      }
      if (lane == k0 + q && q < nb) b = s[q];
    }
    // rows below the block: b_i -= sum_q L[i][k0+q] s_q (row li of the factor)
#pragma unroll
    for (int q = 0; q < kNb; ++q) l[q] = q < nb ? M[li * ld + k0 + q] : make_double2(0.0, 0.0);
    if (lane >= k0 + nb && lane < d) {
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        const double2 t = cmul(l[q], s[q]);
        b.x -= t.x;
        b.y -= t.y;
      }
    }
  }
}

// Deterministic sum over the 64 lanes of a wavefront (every lane gets the
// same value, summed in the same order).
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Hermitian positive definite solve with the matrix in registers.
//
// The (D+1) x (D+1) bordered matrix [[K, .], [conj(b)^T, .]] (K Hermitian,
// D x D; only entries on or below the diagonal are held, the last row being
// the conjugated right-hand side) is distributed 2D block-cyclically over a
// G x G grid of threads: thread (a, c) holds entry (i, j) = (a + G ia,
// c + G jc) in (mr, mi)[ia][jc] (ia >= jc; slots with i < j are carried but
// never read).  The Cholesky factorization [[K, b], [b^H, *]] = [[L, 0], [w^H, *]]
// [[L^H, w], [0, *]] leaves L in place of K and conj(w) = conj(L^-1 b) in
// the last row, so the forward substitution rides along.
// ---------------------------------------------------------------------------
template <int D, int G>
struct RegGrid {
  static constexpr int D1 = D + 1;                 // rows, the border included
  static constexpr int NS = (D1 + G - 1) / G;      // slot rows (and columns) per thread
};

// Orders the LDS traffic of the threads of one grid: a wavefront fence when
// the grid is one wavefront, a workgroup barrier otherwise.
template <int G>
__device__ __attribute__((always_inline)) inline void grid_sync() {
  if constexpr (G * G <= 64) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// Right-looking factorization, one column at a time, one sync per column.
// The owners of column k publish it (unscaled) to col (two buffers of D+1
// values, used alternately) and every thread reads it back with the pivot
// p = a_kk; every thread then updates its trailing entries
// a_ij -= a_ik conj(a_jk) / p (i, j > k), and the owners of column k scale
// it (l_kk = sqrt(p), l_ik = a_ik / sqrt(p)).  The pivot is read by every
// thread from the same LDS value, so a pivot that is not positive makes
// every thread return false at the same column.
// Columns KB*G .. KB*G+G-1 (slot column KB of every thread); a template per
// slot column, so every slot index is a constant and the slots stay in
// registers (real and imaginary parts in plain double arrays: a struct array
// with union members is not split into registers).  The row factor a_ik / p
// is read per slot row inside the update, so only the column factors of the
// thread's slot columns are held.
template <int D, int G, int NS, int KB>
__device__ __attribute__((always_inline)) inline bool reg_cholesky_cols(double (&mr)[NS][NS],
                                                                        double (&mi)[NS][NS],
                                                                        int a, int c,
                                                                        double2* col) {
  if constexpr (KB >= NS) {
    return true;
  } else {
    constexpr int D1 = D + 1;
#pragma unroll 1
    for (int kk = 0; kk < G; ++kk) {
      const int k = KB * G + kk;
      if (k >= D) break;
      double2* buf = col + (k & 1) * D1;
      if (c == kk) {
#pragma unroll
        for (int ia = KB; ia < NS; ++ia) {
          const int i = a + G * ia;
          if (i >= k && i <= D) buf[i] = make_double2(mr[ia][KB], mi[ia][KB]);
        }
      }
      grid_sync<G>();
      const double p = buf[k].x;
      if (!(p > 0.0)) return false;
      const double rs = rsqrt_nr(p), inv = rs * rs;
      double cjr[NS], cji[NS];
#pragma unroll
      for (int q = KB; q < NS; ++q) {
        const int j = c + G * q;
        const double2 v = (j > k && j < D) ? buf[j] : make_double2(0.0, 0.0);
        cjr[q] = v.x;
        cji[q] = v.y;
      }
#pragma unroll
      for (int ia = KB; ia < NS; ++ia) {
        const int i = a + G * ia;
        const double2 u = (i > k && i <= D) ? buf[i] : make_double2(0.0, 0.0);
        const double cr = u.x * inv, ci = u.y * inv;
#pragma unroll
        for (int jc = KB; jc <= ia; ++jc) {
          mr[ia][jc] -= cr * cjr[jc] + ci * cji[jc];
          mi[ia][jc] -= ci * cjr[jc] - cr * cji[jc];
        }
      }
      if (c == kk) {
#pragma unroll
        for (int ia = KB; ia < NS; ++ia) {
          const int i = a + G * ia;
          if (i == k) {
            mr[ia][KB] = p * rs;
            mi[ia][KB] = 0.0;
          } else if (i > k && i <= D) {
            mr[ia][KB] *= rs;
            mi[ia][KB] *= rs;
          }
        }
      }
    }
    return reg_cholesky_cols<D, G, NS, KB + 1>(mr, mi, a, c, col);
  }
}

template <int D, int G, int NS>
__device__ __attribute__((always_inline)) inline bool reg_cholesky(double (&mr)[NS][NS],
                                                                   double (&mi)[NS][NS], int a,
                                                                   int c, double2* col) {
  static_assert(NS == RegGrid<D, G>::NS, "slot count of the grid");
  return reg_cholesky_cols<D, G, NS, 0>(mr, mi, a, c, col);
}

}  // namespace bfc
