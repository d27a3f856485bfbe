// Contour solves and the weighted quadrature sum (gfx950).
//
// For every node z_j the M0 right-hand sides are solved with the stored LU factors
// (FEAST Hermitian RCI case 11); for complex Hermitian problems the conjugate node
// conj(z_j) is served by a solve with (z_j B - A)^H reusing the same factors (cases
// 20/21).  Every triangular block step is two MFMA products: the inverted diagonal
// block applied in place, then the update of the remaining rows.  The quadrature
// sum then forms the new subspace in FP64 (see k_accumulate).
#include "kernels.hpp"

namespace mf {

// ---------------------------------------------------------------------------
template <typename T, typename C>
__global__ void k_rhs_prepare(int64_t n, int m, const T* __restrict__ rhs, int64_t ld,
                              const double* __restrict__ cs, int ne, const int* __restrict__ perm,
                              C* __restrict__ Wf, C* __restrict__ Wc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= m) return;
  const double sc = cs[c];
  const int64_t blk = n * (int64_t)m;
  if (Wc != nullptr) {
    const T v = rhs[i * ld + c];
    const C cv = convert<C, c64>(convert<c64, T>(v) * c64(sc, 0.0));
    for (int j = 0; j < ne; ++j) Wc[j * blk + i * m + c] = cv;
  }
  for (int j = 0; j < ne; ++j) {
    const int64_t src = perm[(int64_t)j * n + i];
    const T v = rhs[src * ld + c];
    Wf[j * blk + i * m + c] = convert<C, c64>(convert<c64, T>(v) * c64(sc, 0.0));
  }
}

template <typename T, typename C>
int rhs_prepare(hipStream_t s, int64_t n, int m, const T* rhs, int64_t ld, const double* colscale,
                int ne, const int* perm, C* Wf, C* Wc) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_rhs_prepare<T, C>), grid, dim3(256), 0, s, n, m, rhs, ld, colscale, ne, perm, Wf, Wc);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Blocked triangular solves.  Block kb covers rows [k, k + nbc), k = kb * LU_NB.
template <typename C>
int lu_solve(hipStream_t s, int64_t n, int m, int ne, const C* LU, const C* Dinv, C* Wf, C* Wc) {
  using R = typename real_of<C>::type;
  const int64_t nblk = (n + LU_NB - 1) / LU_NB;
  const int64_t dstride = nblk * 2 * LU_NB * LU_NB;  // Dinv entries per node
  const int64_t wstride = n * (int64_t)m;
  const int64_t lstride = n * n;
  auto diag = [&](C* W, int64_t kb, bool upper, bool herm) -> int {
    const int64_t k = kb * LU_NB;
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    GemmArgs g{};
    g.M = nbc; g.N = m; g.K = nbc;
    g.A = Dinv + kb * 2 * LU_NB * LU_NB + (upper ? LU_NB * LU_NB : 0);
    g.lda = LU_NB; g.a_bs = dstride;
    g.B = W + k * m; g.ldb = m; g.b_bs = wstride;
    g.C = W + k * m; g.ldc = m; g.c_bs = wstride;
    g.alpha = 1.0; g.beta = 0.0;
    // herm: apply the conjugate transpose of the stored inverse (M-contiguous + conj)
    return gemm<R, true>(s, herm, herm, g, ne);
  };
  // algorithmic work of one direction: 8 n^2 m flops per node (L and U sweeps)
  const double dir_flops = 8.0 * (double)n * n * m * ne;
  const double dir_bytes = (double)sizeof(C) * ne * ((double)n * n + 2.0 * n * m);
  // forward direction:  L then U
  int tok = prof_begin(s);
  for (int64_t kb = 0; kb < nblk; ++kb) {
    const int64_t k = kb * LU_NB;
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    if (diag(Wf, kb, false, false)) return -2;
    const int64_t rest = n - k - nbc;
    if (rest > 0) {
      GemmArgs g{};
      g.M = (int)rest; g.N = m; g.K = nbc;
      g.A = LU + (k + nbc) * n + k; g.lda = n; g.a_bs = lstride;
      g.B = Wf + k * m; g.ldb = m; g.b_bs = wstride;
      g.C = Wf + (k + nbc) * m; g.ldc = m; g.c_bs = wstride;
      g.alpha = -1.0; g.beta = 1.0;
      if (gemm<R, true>(s, false, false, g, ne)) return -2;
    }
  }
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t k = kb * LU_NB;
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    if (diag(Wf, kb, true, false)) return -2;
    if (k > 0) {
      GemmArgs g{};
      g.M = (int)k; g.N = m; g.K = nbc;
      g.A = LU + k; g.lda = n; g.a_bs = lstride;  // rows [0,k), columns [k, k+nbc)
      g.B = Wf + k * m; g.ldb = m; g.b_bs = wstride;
      g.C = Wf; g.ldc = m; g.c_bs = wstride;
      g.alpha = -1.0; g.beta = 1.0;
      if (gemm<R, true>(s, false, false, g, ne)) return -2;
    }
  }
  prof_end(tok, s, K_SOLVE_GEMM, dir_flops, dir_bytes);
  if (Wc == nullptr) return 0;
  // conjugate-transpose direction: U^H (lower) then L^H (unit upper)
  tok = prof_begin(s);
  for (int64_t kb = 0; kb < nblk; ++kb) {
    const int64_t k = kb * LU_NB;
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    if (diag(Wc, kb, true, true)) return -2;
    const int64_t rest = n - k - nbc;
    if (rest > 0) {
      GemmArgs g{};
      g.M = (int)rest; g.N = m; g.K = nbc;
      // op(A)(i, kk) = conj(U[k + kk][k + nbc + i])  -> M-contiguous view of the U block row
      g.A = LU + k * n + k + nbc; g.lda = n; g.a_bs = lstride;
      g.B = Wc + k * m; g.ldb = m; g.b_bs = wstride;
      g.C = Wc + (k + nbc) * m; g.ldc = m; g.c_bs = wstride;
      g.alpha = -1.0; g.beta = 1.0;
      if (gemm<R, true>(s, true, true, g, ne)) return -2;
    }
  }
  for (int64_t kb = nblk - 1; kb >= 0; --kb) {
    const int64_t k = kb * LU_NB;
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    if (diag(Wc, kb, false, true)) return -2;
    if (k > 0) {
      GemmArgs g{};
      g.M = (int)k; g.N = m; g.K = nbc;
      // op(A)(i, kk) = conj(L[k + kk][i]), i < k
      g.A = LU + k * n; g.lda = n; g.a_bs = lstride;
      g.B = Wc + k * m; g.ldb = m; g.b_bs = wstride;
      g.C = Wc; g.ldc = m; g.c_bs = wstride;
      g.alpha = -1.0; g.beta = 1.0;
      if (gemm<R, true>(s, true, true, g, ne)) return -2;
    }
  }
  prof_end(tok, s, K_SOLVE_GEMM, dir_flops, dir_bytes);
  return 0;
}

// ---------------------------------------------------------------------------
// Quadrature sum in FP64.  With d_j the forward solutions and e_j the conjugate-node
// solutions (already mapped back through perm_inv), for column c:
//   real symmetric:   Q = rho_c X + unscale_c * sum_j 2 Re(cf_j[c] d_j)
//   complex Hermitian: Q = rho_c X + unscale_c * sum_j (cf_j[c] d_j + cc_j[c] e_j)
// Residual form: cf_j[c] = w_j / (z_j - lambda_c), cc_j[c] = conj(w_j) / (conj(z_j) - lambda_c),
// rho_c = rho(lambda_c).  Classic form (first contour): cf = w_j, cc = conj(w_j), no X term.
// Nodes are summed in order j = 0..ne-1.
template <typename T, typename C>
__global__ void k_accumulate(int64_t n, int m, int ne, const C* __restrict__ Wf, const C* __restrict__ Wc,
                             const int* __restrict__ perm_inv, const c64* __restrict__ cf,
                             const c64* __restrict__ cc, const double* __restrict__ rho,
                             const double* __restrict__ unscale, const T* __restrict__ X,
                             T* __restrict__ Q, int resid) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= m) return;
  const int64_t blk = n * (int64_t)m;
  if constexpr (is_cplx<T>::value) {
    c64 acc(0.0, 0.0);
    for (int j = 0; j < ne; ++j) {
      const c64 d = convert<c64, C>(Wf[j * blk + r * m + c]);
      const int64_t rr = perm_inv[(int64_t)j * n + r];
      const c64 e = convert<c64, C>(Wc[j * blk + rr * m + c]);
      acc = acc + cf[(int64_t)j * m + c] * d + cc[(int64_t)j * m + c] * e;
    }
    acc = unscale[c] * acc;
    if (resid) acc = acc + rho[c] * X[r * m + c];
    Q[r * m + c] = acc;
  } else {
    double acc = 0.0;
    for (int j = 0; j < ne; ++j) {
      const c64 d = convert<c64, C>(Wf[j * blk + r * m + c]);
      const c64 p = cf[(int64_t)j * m + c] * d;
      acc += 2.0 * p.re;
    }
    acc *= unscale[c];
    if (resid) acc += rho[c] * X[r * m + c];
    Q[r * m + c] = acc;
  }
}

template <typename T, typename C>
int accumulate(hipStream_t s, int64_t n, int m, int ne, const C* Wf, const C* Wc, const int* perm_inv,
               const c64* coef_f, const c64* coef_c, const double* rho, const double* unscale,
               const T* X, T* Q, int resid) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_accumulate<T, C>), grid, dim3(256), 0, s, n, m, ne, Wf, Wc, perm_inv, coef_f,
                     coef_c, rho, unscale, X, Q, resid);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int rhs_prepare<double, c32>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, c32*, c32*);
template int rhs_prepare<double, c64>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, c64*, c64*);
template int rhs_prepare<c64, c32>(hipStream_t, int64_t, int, const c64*, int64_t, const double*, int, const int*, c32*, c32*);
template int rhs_prepare<c64, c64>(hipStream_t, int64_t, int, const c64*, int64_t, const double*, int, const int*, c64*, c64*);
template int lu_solve<c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, c32*, c32*);
template int lu_solve<c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, c64*, c64*);
template int accumulate<double, c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, const int*, const c64*, const c64*, const double*, const double*, const double*, double*, int);
template int accumulate<double, c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, const int*, const c64*, const c64*, const double*, const double*, const double*, double*, int);
template int accumulate<c64, c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, const int*, const c64*, const c64*, const double*, const double*, const c64*, c64*, int);
template int accumulate<c64, c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, const int*, const c64*, const c64*, const double*, const double*, const c64*, c64*, int);

}  // namespace mf
