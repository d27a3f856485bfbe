// B-orthonormal basis of the filtered subspace for the Rayleigh-Ritz step (gfx950).
//
// The reduced problem Aq W = Bq W Lambda (FEAST Hermitian RCI, Table tab-rci1) is
// solved in an explicitly B-orthonormal basis of span(Q), built in two passes:
//   pass 1  Cholesky of the equilibrated overlap S' = D Q^H B Q D with column
//           dropping: a column whose Schur-complement pivot is below tau is
//           (numerically) in the span of the earlier ones and is left out, so the
//           subspace dimension M0 shrinks to the kept count.  G1 = D L^-H on the
//           kept columns gives Q1 = Q G1, B-orthonormal up to eps / min pivot.
//   pass 2  S1 = Q1^H B Q1 = I + F is formed again from the n x k blocks; its
//           inverse square root (coupled Newton-Schulz iteration, GEMMs only)
//           restores orthonormality to working precision.
// Every dense step is an MFMA product except the CH_NB x CH_NB diagonal blocks of
// the Cholesky, which one workgroup factors (and inverts) in LDS.
#include "kernels.hpp"

namespace mf {

constexpr int CH_NB = 32;  // Cholesky / triangular-inverse block width

// ---------------------------------------------------------------------------
// Diagonal block jb of the right-looking Cholesky (row-major m x m matrix A, lower
// part used).  Factors the (already updated) CH_NB x CH_NB block in LDS, dropping
// columns whose pivot is <= tau.  Writes L_jj (lower, upper zeroed) into A, its
// pseudo-inverse into Linv (same position), and keep[j] in {0,1}.
template <typename T>
__global__ __launch_bounds__(256) void k_chol_diag(int m, int jb, T* A, T* Linv, int* keep, double tau) {
  __shared__ T a[CH_NB][CH_NB + 1];
  __shared__ T x[CH_NB][CH_NB + 1];
  __shared__ int s_keep[CH_NB];
  const int tid = threadIdx.x;
  const int bc = min(CH_NB, m - jb);
  for (int e = tid; e < CH_NB * CH_NB; e += 256) {
    const int i = e / CH_NB, j = e % CH_NB;
    a[i][j] = (i < bc && j < bc && j <= i) ? A[(int64_t)(jb + i) * m + jb + j] : T(0.0);
  }
  __syncthreads();
  for (int j = 0; j < bc; ++j) {
    // every thread takes the pivot itself (no broadcast round); a[j][j] is overwritten only
    // in the trailing-update phase below, which does not read it
    const double d = real_part(a[j][j]);
    const int kj = (d > tau) ? 1 : 0;
    const double ljj = kj ? sqrt(d) : 0.0;
    if (tid == 0) s_keep[j] = kj;
    // column j below the diagonal
    if (tid > j && tid < bc) a[tid][j] = (ljj > 0.0) ? (1.0 / ljj) * a[tid][j] : T(0.0);
    __syncthreads();
    if (tid == 0) a[j][j] = T(ljj);
    // trailing update of the block's lower triangle
    for (int e = tid; e < CH_NB * CH_NB; e += 256) {
      const int i = e / CH_NB, k = e % CH_NB;
      if (i < bc && k > j && k <= i) a[i][k] = a[i][k] - a[i][j] * conj(a[k][j]);
    }
    __syncthreads();
  }
  // pseudo-inverse of the lower-triangular block: column c by forward substitution (the
  // column in registers; same order of the terms), rows and columns of dropped indices
  // are zero
  if (tid < CH_NB) {
    const int c = tid;
    T xr[CH_NB];
    double rd[CH_NB];
#pragma unroll
    for (int i = 0; i < CH_NB; ++i) rd[i] = 1.0 / real_part(a[i][i]);
    // the terms of rows k < c and of dropped rows are exact zeros (xr[k] = 0 there), so
    // every term is taken without a branch and the LDS reads are not serialized
#pragma unroll
    for (int i = 0; i < CH_NB; ++i) {
      T v = (i == c) ? T(1.0) : T(0.0);
#pragma unroll
      for (int k = 0; k < i; ++k) v = v - a[i][k] * xr[k];
      const bool ok = i < bc && c < bc && i >= c && s_keep[i] != 0 && s_keep[c] != 0;
      xr[i] = ok ? rd[i] * v : T(0.0);
    }
#pragma unroll
    for (int i = 0; i < CH_NB; ++i) x[i][c] = xr[i];
  }
  __syncthreads();
  for (int e = tid; e < CH_NB * CH_NB; e += 256) {
    const int i = e / CH_NB, j = e % CH_NB;
    if (i < bc && j < bc) {
      // rows of dropped indices are cleared by the final fix-up
      A[(int64_t)(jb + i) * m + jb + j] = (j <= i && s_keep[j]) ? a[i][j] : T(0.0);
      Linv[(int64_t)(jb + i) * m + jb + j] = x[i][j];
    }
  }
  if (tid < bc) keep[jb + tid] = s_keep[tid];
}

// zero the strictly upper triangle and the rows of dropped indices of L
template <typename T>
__global__ void k_chol_fix(int m, T* A, const int* __restrict__ keep) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m) return;
  if (j > i || !keep[i] || !keep[j]) A[(int64_t)i * m + j] = T(0.0);
}

template <typename T>
__global__ void k_fill(int64_t count, T* p, T v) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename T>
static int gemmT(hipStream_t s, GemmOp oa, GemmOp ob, int M, int N, int K, const T* A, int64_t lda, const T* B,
                 int64_t ldb, T* C, int64_t ldc, double alpha, double beta) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda;
  g.B = B; g.ldb = ldb;
  g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  return gemm_op<double, is_cplx<T>::value>(s, oa, ob, g, 1);
}

// L (in place of A, lower) and Linv = pseudo-inverse of L; keep[j] = column kept.
// work: at least m * CH_NB entries of T.
template <typename T>
int chol_drop(hipStream_t s, int m, T* A, T* Linv, int* keep, double tau, T* work) {
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL((k_fill<T>), dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, s, mm, Linv, T(0.0));
  for (int jb = 0; jb < m; jb += CH_NB) {
    const int bc = std::min(CH_NB, m - jb);
    hipLaunchKernelGGL((k_chol_diag<T>), dim3(1), dim3(256), 0, s, m, jb, A, Linv, keep, tau);
    const int rest = m - jb - bc;
    if (rest > 0) {
      // panel: L[below, j] = A[below, j] * Linv_jj^H   (in place, one column tile)
      if (gemmT<T>(s, OP_N, OP_C, rest, bc, bc, A + (int64_t)(jb + bc) * m + jb, m, Linv + (int64_t)jb * m + jb, m,
                   A + (int64_t)(jb + bc) * m + jb, m, 1.0, 0.0))
        return -2;
      // trailing: A[below, below] -= L_p L_p^H
      if (gemmT<T>(s, OP_N, OP_C, rest, rest, bc, A + (int64_t)(jb + bc) * m + jb, m, A + (int64_t)(jb + bc) * m + jb,
                   m, A + (int64_t)(jb + bc) * m + jb + bc, m, -1.0, 1.0))
        return -2;
    }
  }
  hipLaunchKernelGGL((k_chol_fix<T>), dim3((m + 255) / 256, m), dim3(256), 0, s, m, A, keep);
  // blocked inverse, last block first: Linv[r, j] = -(Linv[r, r] L[r, j]) Linv_jj, r = rows below block j
  const int nblk = (m + CH_NB - 1) / CH_NB;
  for (int b = nblk - 1; b >= 0; --b) {
    const int jb = b * CH_NB;
    const int bc = std::min(CH_NB, m - jb);
    const int rest = m - jb - bc;
    if (rest <= 0) continue;
    if (gemmT<T>(s, OP_N, OP_N, rest, bc, rest, Linv + (int64_t)(jb + bc) * m + jb + bc, m,
                 A + (int64_t)(jb + bc) * m + jb, m, work, bc, 1.0, 0.0))
      return -2;
    if (gemmT<T>(s, OP_N, OP_N, rest, bc, bc, work, bc, Linv + (int64_t)jb * m + jb, m,
                 Linv + (int64_t)(jb + bc) * m + jb, m, -1.0, 0.0))
      return -2;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// H1 (m x k, row-major) = D Linv^H restricted to the kept columns idx[0..k)
template <typename T>
__global__ void k_build_h1(int m, int k, const T* __restrict__ Linv, const double* __restrict__ d,
                           const int* __restrict__ idx, T* __restrict__ H1) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (t >= k) return;
  H1[(int64_t)i * k + t] = d[i] * conj(Linv[(int64_t)idx[t] * m + i]);
}

template <typename T>
int build_h1(hipStream_t s, int m, int k, const T* Linv, const double* d, const int* idx, T* H1) {
  hipLaunchKernelGGL((k_build_h1<T>), dim3((k + 255) / 256, m), dim3(256), 0, s, m, k, Linv, d, idx, H1);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// ||S - I||_F (partial sums per row, then a single-block sum)
template <typename T>
__global__ void k_dev_from_identity(int k, const T* __restrict__ S, double* part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  double acc = 0.0;
  for (int j = 0; j < k; ++j) {
    T v = S[(int64_t)i * k + j];
    if (i == j) v = v - T(1.0);
    acc += norm2(v);
  }
  part[i] = acc;
}

__global__ void k_sum(int k, const double* __restrict__ part, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

template <typename T>
int dev_from_identity(hipStream_t s, int k, const T* S, double* part, double* out) {
  hipLaunchKernelGGL((k_dev_from_identity<T>), dim3((k + 255) / 256), dim3(256), 0, s, k, S, part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, k, part, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// P = (3 I - P) / 2 in place
template <typename T>
__global__ void k_ns_step(int k, T* P) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= k) return;
  const int64_t e = (int64_t)i * k + j;
  T v = (-0.5) * P[e];
  if (i == j) v = v + T(1.5);
  P[e] = v;
}

// Z = S^{-1/2} by the coupled Newton-Schulz iteration
//   Y0 = S, Z0 = I;  P = (3I - Z Y)/2;  Y <- Y P;  Z <- P Z
// valid for ||I - S|| < 1; `iters` steps.  work: 3 k x k matrices.
template <typename T>
int ns_invsqrt(hipStream_t s, int k, const T* S, T* Z, int iters, T* work) {
  const int64_t kk = (int64_t)k * k;
  const size_t bytes = kk * sizeof(T);
  T* Y = work;
  T* P = work + kk;
  T* W = work + 2 * kk;
  MF_HIP_CHECK(hipMemcpyAsync(Y, S, bytes, hipMemcpyDeviceToDevice, s));
  for (int it = 0; it < iters; ++it) {
    if (it == 0) {
      MF_HIP_CHECK(hipMemcpyAsync(P, Y, bytes, hipMemcpyDeviceToDevice, s));  // Z0 Y0 = S
    } else if (gemmT<T>(s, OP_N, OP_N, k, k, k, Z, k, Y, k, P, k, 1.0, 0.0)) {
      return -2;
    }
    hipLaunchKernelGGL((k_ns_step<T>), dim3((k + 255) / 256, k), dim3(256), 0, s, k, P);
    if (gemmT<T>(s, OP_N, OP_N, k, k, k, Y, k, P, k, W, k, 1.0, 0.0)) return -2;  // W = Y P (new Y)
    if (it == 0) {
      MF_HIP_CHECK(hipMemcpyAsync(Z, P, bytes, hipMemcpyDeviceToDevice, s));  // Z1 = P I
    } else {
      if (gemmT<T>(s, OP_N, OP_N, k, k, k, P, k, Z, k, Y, k, 1.0, 0.0)) return -2;  // old Y is free
      MF_HIP_CHECK(hipMemcpyAsync(Z, Y, bytes, hipMemcpyDeviceToDevice, s));
    }
    MF_HIP_CHECK(hipMemcpyAsync(Y, W, bytes, hipMemcpyDeviceToDevice, s));
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define MF_ORTH_INST(T)                                                                       \
  template int chol_drop<T>(hipStream_t, int, T*, T*, int*, double, T*);                       \
  template int build_h1<T>(hipStream_t, int, int, const T*, const double*, const int*, T*);   \
  template int dev_from_identity<T>(hipStream_t, int, const T*, double*, double*);            \
  template int ns_invsqrt<T>(hipStream_t, int, const T*, T*, int, T*);

MF_ORTH_INST(double)
MF_ORTH_INST(c64)

}  // namespace mf
