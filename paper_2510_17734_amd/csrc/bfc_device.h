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

// v <- the R-vector at src + idx * R
template <typename T, int R>
__device__ inline void load_env(const cx<T>* __restrict__ src, int idx, cx<T> (&v)[R]) {
  const cx<T>* p = src + (int64_t)idx * R;
#pragma unroll
  for (int a = 0; a < R; ++a) v[a] = p[a];
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
// Hermitian positive definite solve by one wavefront (a workgroup of exactly
// 64 threads, so __syncthreads is a wavefront barrier), d <= 64 unknowns.
// M is row-major with an odd leading dimension ld (element (i, j) at
// i*ld + j): a row walk across lanes (stride ld) and a column walk
// (consecutive j) both touch distinct LDS banks.  Lane i owns row i.
// ---------------------------------------------------------------------------

// Uniform-lane broadcast of a double (lane index in a scalar register).
__device__ inline double bcast_d(double x, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
  return __hiloint2double(hi, lo);
}

// Blocked factorization, panel width kNb: per panel the kNb x kNb diagonal
// block is factored redundantly in every lane's registers, the rows below
// solve for their panel entries, and the trailing update subtracts a rank-kNb
// product.  panel (d x kNb values of LDS) holds the panel for the trailing
// reads, an array the row updates never write.
constexpr int kNb = 4;

// Factor the nb x nb lower block at (k0, k0) of M into D (registers).
__device__ __attribute__((always_inline)) inline bool diag_block_factor(const double2* M, int ld,
                                                                         int k0, int nb,
                                                                         double2 (&D)[kNb][kNb]) {
#pragma unroll
  for (int a = 0; a < kNb; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b)
      D[a][b] = (a < nb) ? M[(k0 + a) * ld + k0 + b] : make_double2(a == b ? 1.0 : 0.0, 0.0);
#pragma unroll
  for (int k = 0; k < kNb; ++k) {
    const double piv = D[k][k].x;
    if (!(piv > 0.0)) return false;
    const double lkk = sqrt(piv), inv = 1.0 / lkk;
    D[k][k] = make_double2(lkk, 0.0);
#pragma unroll
    for (int i = k + 1; i < kNb; ++i) {
      D[i][k].x *= inv;
      D[i][k].y *= inv;
    }
#pragma unroll
    for (int j = k + 1; j < kNb; ++j)
#pragma unroll
      for (int i = j; i < kNb; ++i) {
        D[i][j].x -= D[i][k].x * D[j][k].x + D[i][k].y * D[j][k].y;
        D[i][j].y -= D[i][k].y * D[j][k].x - D[i][k].x * D[j][k].y;
      }
  }
  return true;
}

// In-place lower Cholesky factor of the d x d matrix M.  Returns false if a
// pivot is not positive (the result is the same in every lane).
__device__ inline bool lds_cholesky(double2* M, int d, int ld, double2* panel, int lane) {
  for (int k0 = 0; k0 < d; k0 += kNb) {
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    double2 D[kNb][kNb];
    if (!diag_block_factor(M, ld, k0, nb, D)) return false;
    double rinv[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) rinv[q] = 1.0 / D[q][q].x;
    double2 Li[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) Li[q] = make_double2(0.0, 0.0);
    if (lane >= k0 + nb && lane < d) {
      // L_i L_D^H = a_i, solved by forward substitution over the panel
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        if (q >= nb) break;
        double2 v = M[lane * ld + k0 + q];
#pragma unroll
        for (int p = 0; p < q; ++p) {  // v -= L_i[p] conj(L_D[q][p])
          v.x -= Li[p].x * D[q][p].x + Li[p].y * D[q][p].y;
          v.y -= Li[p].y * D[q][p].x - Li[p].x * D[q][p].y;
        }
        const double inv = rinv[q];
        Li[q] = make_double2(v.x * inv, v.y * inv);
        M[lane * ld + k0 + q] = Li[q];
        panel[lane * kNb + q] = Li[q];
      }
    } else if (lane >= k0 && lane < k0 + nb) {
      const int a = lane - k0;
#pragma unroll
      for (int q = 0; q < kNb; ++q)
#pragma unroll
        for (int r = 0; r < kNb; ++r)
          if (r == a && q <= r) M[lane * ld + k0 + q] = D[r][q];
    }
    __syncthreads();
    if (lane >= k0 + nb && lane < d) {
      double2* row = M + lane * ld;
      for (int j = k0 + nb; j <= lane; ++j) {
        const double2* pj = panel + j * kNb;  // same address in every lane
        double2 m = row[j];
#pragma unroll
        for (int q = 0; q < kNb; ++q) {
          const double2 c = pj[q];
          m.x -= Li[q].x * c.x + Li[q].y * c.y;  // m -= L_i[q] conj(L_j[q])
          m.y -= Li[q].y * c.x - Li[q].x * c.y;
        }
        row[j] = m;
      }
    }
    __syncthreads();
  }
  return true;
}

// Solve L L^H s = b with the factor of lds_cholesky and rdiag[k] =
// 1 / L[k][k].  Lane i holds b_i in a register and ends with s_i; lanes >= d
// carry nothing of use.  Blocked by
// kNb columns; no LDS writes and no barriers: the block's running values are
// broadcast with readlane and its triangle is read by every lane.
__device__ inline void lds_chol_solve(const double2* M, const double* rdiag, int d, int ld,
                                      double2& b, int lane) {
  const int li = lane < d ? lane : 0;
  for (int k0 = 0; k0 < d; k0 += kNb) {  // L y = b
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    double2 y[kNb];
#pragma unroll
    for (int q = 0; q < kNb; ++q) {
      y[q] = make_double2(0.0, 0.0);
      if (q >= nb) continue;
      double2 v = make_double2(bcast_d(b.x, k0 + q), bcast_d(b.y, k0 + q));
#pragma unroll
      for (int p = 0; p < q; ++p) {
        const double2 l = M[(k0 + q) * ld + k0 + p];
        v.x -= l.x * y[p].x - l.y * y[p].y;
        v.y -= l.x * y[p].y + l.y * y[p].x;
      }
      const double inv = rdiag[k0 + q];
      y[q] = make_double2(v.x * inv, v.y * inv);
      if (lane == k0 + q) b = y[q];
    }
    if (lane >= k0 + nb && lane < d) {
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        if (q >= nb) break;
        const double2 l = M[li * ld + k0 + q];
        b.x -= l.x * y[q].x - l.y * y[q].y;
        b.y -= l.x * y[q].y + l.y * y[q].x;
      }
    }
  }
  const int last = ((d - 1) / kNb) * kNb;
  for (int k0 = last; k0 >= 0; k0 -= kNb) {  // L^H s = y
    const int nb = d - k0 < kNb ? d - k0 : kNb;
    double2 x[kNb];
#pragma unroll
    for (int q = kNb - 1; q >= 0; --q) {
      x[q] = make_double2(0.0, 0.0);
      if (q >= nb) continue;
      double2 v = make_double2(bcast_d(b.x, k0 + q), bcast_d(b.y, k0 + q));
#pragma unroll
      for (int p = q + 1; p < kNb; ++p) {  // v -= conj(L[k0+p][k0+q]) s_p
        if (p >= nb) break;
        const double2 l = M[(k0 + p) * ld + k0 + q];
        v.x -= l.x * x[p].x + l.y * x[p].y;
        v.y -= l.x * x[p].y - l.y * x[p].x;
      }
      const double inv = rdiag[k0 + q];
      x[q] = make_double2(v.x * inv, v.y * inv);
      if (lane == k0 + q) b = x[q];
    }
    if (lane < k0) {
#pragma unroll
      for (int q = 0; q < kNb; ++q) {
        if (q >= nb) break;
        const double2 l = M[(k0 + q) * ld + li];  // conj(L[k0+q][lane]) s_q
        b.x -= l.x * x[q].x + l.y * x[q].y;
        b.y -= l.x * x[q].y - l.y * x[q].x;
      }
    }
  }
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

// Deterministic sum over the 64 lanes of a wavefront (every lane gets the
// same value, summed in the same order).
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace bfc
