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

// Hermitian positive definite solve by one wavefront (workgroup of exactly
// 64 threads, so __syncthreads is a wavefront barrier).  M (d x d, row-major,
// d <= 64) is overwritten by its lower Cholesky factor.  Returns false if a
// pivot is not positive (M is then partly overwritten).
__device__ inline bool wave_cholesky(double2* M, int d, int lane) {
  for (int k = 0; k < d; ++k) {
    const double piv = M[k * d + k].x;
    if (!(piv > 0.0)) return false;
    const double lkk = sqrt(piv);
    const double inv = 1.0 / lkk;
    __syncthreads();
    if (lane > k && lane < d) {
      double2 v = M[lane * d + k];
      M[lane * d + k] = make_double2(v.x * inv, v.y * inv);
    }
    if (lane == k) M[k * d + k] = make_double2(lkk, 0.0);
    __syncthreads();
    if (lane > k && lane < d) {
      const double2 lik = M[lane * d + k];
      for (int j = k + 1; j <= lane; ++j) {
        const double2 ljk = M[j * d + k];
        double2 m = M[lane * d + j];
        // m -= lik * conj(ljk)
        m.x -= lik.x * ljk.x + lik.y * ljk.y;
        m.y -= lik.y * ljk.x - lik.x * ljk.y;
        M[lane * d + j] = m;
      }
    }
    __syncthreads();
  }
  return true;
}

// Solve (L L^H) s = b with the factor from wave_cholesky; b (LDS, length d)
// is overwritten by s.
__device__ inline void wave_chol_solve(const double2* M, double2* b, int d, int lane) {
  for (int k = 0; k < d; ++k) {
    __syncthreads();
    const double inv = 1.0 / M[k * d + k].x;
    const double2 yk = make_double2(b[k].x * inv, b[k].y * inv);
    __syncthreads();
    if (lane == k) b[k] = yk;
    if (lane > k && lane < d) {
      const double2 lik = M[lane * d + k];
      double2 v = b[lane];
      v.x -= lik.x * yk.x - lik.y * yk.y;
      v.y -= lik.x * yk.y + lik.y * yk.x;
      b[lane] = v;
    }
  }
  for (int k = d - 1; k >= 0; --k) {
    __syncthreads();
    const double inv = 1.0 / M[k * d + k].x;
    const double2 sk = make_double2(b[k].x * inv, b[k].y * inv);
    __syncthreads();
    if (lane == k) b[k] = sk;
    if (lane < k) {
      const double2 lki = M[k * d + lane];  // (L^H)[lane][k] = conj(L[k][lane])
      double2 v = b[lane];
      v.x -= lki.x * sk.x + lki.y * sk.y;
      v.y -= lki.x * sk.y - lki.y * sk.x;
      b[lane] = v;
    }
  }
  __syncthreads();
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
