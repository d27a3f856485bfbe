// Gradient of a loss on the eigenpairs in the search interval with respect to A
// (real symmetric A, B = I), the backward pass of the FEAST eigensolver.
//
// For the pairs (lambda_i, x_i), i in S, with loss gradients g_i = dL/dlambda_i and
// G_i = dL/dx_i, and a loss invariant under rotations inside span(X_S), first-order
// perturbation of the symmetric eigenproblem gives
//   dL/dA = X diag(g) X^T + (X Y^T + Y X^T) / 2,
// where column y_i is the component of the eigenvector response outside span(X_S):
// the unique solution orthogonal to X_S of the deflated shifted system
//   (lambda_i I - A + sigma X X^T) y_i = (I - X X^T) G_i,
// nonsingular for sigma != lambda_j - lambda_i (j in S); sigma = 1 + 2 (max - min) of the
// given eigenvalues.  The M shifted matrices are real; they are factored together by the
// batched LU of the contour solves (nodes z_i = lambda_i) in real arithmetic, FP64
// (precision 0) or FP32 (precision 1); each solve is refined with FP64 residuals of the
// deflated system.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/mfeast.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace mf;

namespace {

// Y[r][i] (+)= Re(W_i[r][i]) * us[i]: column i of node i's solution (W row-major n x M per node)
template <typename C>
__global__ void k_adj_extract(int64_t n, int M, const C* __restrict__ W, const double* __restrict__ us,
                              double* __restrict__ Y, int add) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * (int64_t)M) return;
  const int64_t r = e / M;
  const int i = (int)(e % M);
  const double v = (double)real_part(W[((int64_t)i * n + r) * M + i]) * us[i];
  Y[e] = add ? Y[e] + v : v;
}

// Rc = R - lambda_i Y + (Ad Y): residual of (lambda_i I - Ad) Y_i = R_i, Ad = A - sigma X X^T
__global__ void k_adj_resid(int64_t n, int M, const double* __restrict__ R, const double* __restrict__ lam,
                            const double* __restrict__ Y, const double* __restrict__ AdY, double* __restrict__ Rc) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * (int64_t)M) return;
  const int i = (int)(e % M);
  Rc[e] = R[e] - lam[i] * Y[e] + AdY[e];
}

// gdiag[r] = sum_i g_i X[r][i]^2 + X[r][i] Y[r][i];  W1[r][i] = g_i X[r][i] + Y[r][i] / 2
__global__ void k_adj_diag(int64_t n, int M, const double* __restrict__ X, const double* __restrict__ g,
                           const double* __restrict__ Y, double* __restrict__ gdiag, double* __restrict__ W1) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i < M; ++i) {
    const double x = X[r * M + i], y = Y[r * M + i];
    acc += g[i] * x * x + x * y;
    if (W1 != nullptr) W1[r * M + i] = g[i] * x + 0.5 * y;
  }
  if (gdiag != nullptr) gdiag[r] = acc;
}

unsigned blocks_for(int64_t count) { return (unsigned)((count + 255) / 256); }

template <typename C>
int adjoint_run(mfeast_ctx* h, int64_t n, const double* A, int64_t lda, int M, const double* E, const double* X,
                int64_t ldx, const double* gE, const double* gX, int64_t ldgx, double* gA, int64_t ldga,
                double* gdiag, int refine) {
  Timer total, ph;
  total.start();
  hipStream_t s = h->stream;
  const int64_t nm = n * (int64_t)M;
  // eigenvalues and loss gradients of S on the host (M values) for the shifts and sigma
  std::vector<double> e(M), g(M, 0.0);
  MF_HIP_CHECK(hipMemcpyAsync(e.data(), E, M * sizeof(double), hipMemcpyDeviceToHost, s));
  if (gE) MF_HIP_CHECK(hipMemcpyAsync(g.data(), gE, M * sizeof(double), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < M; ++i)
    if (!std::isfinite(e[i]) || !std::isfinite(g[i])) return -2;
  const double lo = *std::min_element(e.begin(), e.end()), hi = *std::max_element(e.begin(), e.end());
  const double sigma = 1.0 + 2.0 * (hi - lo);

  double* Xr = (double*)h->ws(S_ADJ_XR, 2 * nm * sizeof(double));  // Xr, W1
  double* Rb = (double*)h->ws(S_ADJ_R, 3 * nm * sizeof(double));   // G, R, Rc
  double* Yb = (double*)h->ws(S_ADJ_Y, 3 * nm * sizeof(double));   // Y, Ad Y, Y column-major
  double* small = (double*)h->ws(S_ADJ_SMALL, ((size_t)M * M + 6 * (size_t)M + 64) * sizeof(double));
  char* hp = h->host((4 * (size_t)M + 64) * sizeof(double));
  if (!Xr || !Rb || !Yb || !small || !hp) return -2;
  double* W1 = Xr + nm;
  double* Gr = Rb;
  double* R = Rb + nm;
  double* Rc = Rb + 2 * nm;
  double* Y = Yb;
  double* AdY = Yb + nm;
  double* Ycm = Yb + 2 * nm;
  double* P = small;
  double* d_lam = small + (size_t)M * M;
  double* d_g = d_lam + M;
  double* d_absmax = d_g + M;
  double* d_cs = d_absmax + M;
  double* d_us = d_cs + M;
  double* h_absmax = (double*)hp;
  double* h_cs = h_absmax + M;
  double* h_us = h_cs + M;
  MF_HIP_CHECK(hipMemcpyAsync(d_lam, e.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  MF_HIP_CHECK(hipMemcpyAsync(d_g, g.data(), M * sizeof(double), hipMemcpyHostToDevice, s));
  MF_TRY(copy_cm_to_rm<double>(s, n, M, X, ldx, Xr, M));

  double t_fact = 0.0, t_solve = 0.0;
  if (gX != nullptr) {
    // R = (I - X X^T) G
    MF_TRY(copy_cm_to_rm<double>(s, n, M, gX, ldgx, Gr, M));
    MF_TRY(rm_gemm<double>(s, M, M, (int)n, Xr, M, true, false, Gr, M, P, M));
    MF_HIP_CHECK(hipMemcpyAsync(R, Gr, nm * sizeof(double), hipMemcpyDeviceToDevice, s));
    MF_TRY(rm_gemm<double>(s, (int)n, M, M, Xr, M, false, false, P, M, R, M, -1.0, 1.0));
    // Ad = A - sigma X X^T (symmetric: row-major and column-major views coincide)
    double* Ad = (double*)h->ws(S_ADJ_AD, (size_t)n * n * sizeof(double));
    if (!Ad) return -2;
    MF_HIP_CHECK(hipMemcpy2DAsync(Ad, n * sizeof(double), A, lda * sizeof(double), n * sizeof(double), n,
                                  hipMemcpyDeviceToDevice, s));
    MF_TRY(rm_gemm<double>(s, (int)n, (int)n, M, Xr, M, false, false, X, ldx, Ad, n, -sigma, 1.0));
    // factor lambda_i I - Ad for every i, batched like the contour nodes
    ph.start();
    const int64_t nblk = (n + LU_NB - 1) / LU_NB;
    C* LU = (C*)h->ws(S_LU, (size_t)M * n * lu_ld(n) * sizeof(C));
    C* Dinv = (C*)h->ws(S_DINV, (size_t)M * nblk * 2 * LU_NB * LU_NB * sizeof(C));
    int* ipiv = (int*)h->ws(S_IPIV, (size_t)M * n * 4);
    int* perm = (int*)h->ws(S_PERM, (size_t)M * n * 4);
    int* pinv = (int*)h->ws(S_PINV, (size_t)M * n * 4);
    int* linfo = (int*)h->ws(S_INFO, (size_t)M * 4 + 64);
    c64* zdev = (c64*)h->ws(S_Z, (size_t)M * sizeof(c64));
    C* Wf = (C*)h->ws(S_WF, (size_t)M * nm * sizeof(C));
    C* Wy = (C*)h->ws(S_WY, (size_t)M * nm * sizeof(C));
    C* Pinv = (C*)h->ws(S_PANINV, (size_t)M * panel_inverse_entries(n) * sizeof(C));
    if (!LU || !Dinv || !ipiv || !perm || !pinv || !linfo || !zdev || !Wf || !Wy || !Pinv) return -2;
    std::vector<c64> z(M);
    for (int i = 0; i < M; ++i) z[i] = c64(e[i], 0.0);
    MF_HIP_CHECK(hipMemcpyAsync(zdev, z.data(), M * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemsetAsync(linfo, 0, M * 4, s));
    MF_TRY(shift_form<double, C>(s, n, Ad, n, nullptr, 0, zdev, M, LU, perm));
    MF_TRY(lu_factor<C>(s, n, M, LU, ipiv, perm, pinv, linfo, Dinv));
    MF_TRY(panel_inverses<C>(s, n, M, LU, Dinv, Pinv));
    std::vector<int> hinfo(M);
    MF_HIP_CHECK(hipMemcpyAsync(hinfo.data(), linfo, M * 4, hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_fact = ph.stop();
    for (int i = 0; i < M; ++i)
      if (hinfo[i] != 0) return -2;
    // solve and refine with FP64 residuals of the deflated systems
    ph.start();
    const double* rhs = R;
    for (int step = 0; step <= refine; ++step) {
      MF_TRY(col_absmax<double>(s, n, M, rhs, M, d_absmax));
      MF_HIP_CHECK(hipMemcpyAsync(h_absmax, d_absmax, M * sizeof(double), hipMemcpyDeviceToHost, s));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      bool all_zero = true;
      for (int i = 0; i < M; ++i) {
        const double a = h_absmax[i];
        if (!std::isfinite(a)) return -2;
        all_zero = all_zero && !(a > 0.0);
        h_cs[i] = a > 0.0 ? 1.0 / a : 1.0;
        h_us[i] = a > 0.0 ? a : 0.0;
      }
      if (all_zero && step > 0) break;
      MF_HIP_CHECK(hipMemcpyAsync(d_cs, h_cs, M * sizeof(double), hipMemcpyHostToDevice, s));
      MF_HIP_CHECK(hipMemcpyAsync(d_us, h_us, M * sizeof(double), hipMemcpyHostToDevice, s));
      MF_TRY(rhs_prepare<double, C>(s, n, M, rhs, M, d_cs, M, perm, Wf, (C*)nullptr));
      MF_TRY(lu_solve<C>(s, n, M, M, LU, Pinv, Wf, (C*)nullptr, Wy));
      hipLaunchKernelGGL((k_adj_extract<C>), dim3(blocks_for(nm)), dim3(256), 0, s, n, M, (const C*)Wf,
                         (const double*)d_us, Y, step > 0 ? 1 : 0);
      if (step < refine) {
        MF_TRY(rm_gemm<double>(s, (int)n, M, (int)n, Ad, n, false, false, Y, M, AdY, M));
        hipLaunchKernelGGL(k_adj_resid, dim3(blocks_for(nm)), dim3(256), 0, s, n, M, (const double*)R,
                           (const double*)d_lam, (const double*)Y, (const double*)AdY, Rc);
        rhs = Rc;
      }
    }
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_solve = ph.stop();
  } else {
    MF_HIP_CHECK(hipMemsetAsync(Y, 0, nm * sizeof(double), s));
  }
  // outputs
  hipLaunchKernelGGL(k_adj_diag, dim3(blocks_for(n)), dim3(256), 0, s, n, M, (const double*)Xr,
                     (const double*)d_g, (const double*)Y, gdiag, gA ? W1 : nullptr);
  if (gA != nullptr) {
    // gA = W1 X^T + (X Y^T) / 2 with W1 = X diag(g) + Y / 2 (symmetric result)
    MF_TRY(rm_gemm<double>(s, (int)n, (int)n, M, W1, M, false, false, X, ldx, gA, ldga, 1.0, 0.0));
    MF_TRY(copy_rm_to_cm<double>(s, n, M, Y, M, Ycm, n));
    MF_TRY(rm_gemm<double>(s, (int)n, (int)n, M, Xr, M, false, false, Ycm, n, gA, ldga, 0.5, 1.0));
  }
  MF_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < 8; ++i) h->timing[i] = 0.0;
  h->timing[0] = t_fact;
  h->timing[1] = t_solve;
  h->timing[5] = total.stop();
  h->timing[4] = h->timing[5] - t_fact - t_solve;
  return 0;
}

}  // namespace

extern "C" int mfeast_dsy_adjoint(mfeast_handle h, int64_t n, const double* A, int64_t lda, int32_t M,
                                  const double* E, const double* X, int64_t ldx, const double* gE,
                                  const double* gX, int64_t ldgx, int32_t precision, double* gA, int64_t ldga,
                                  double* gdiag) {
  if (n < 1) return 202;
  if (M < 1 || M > n) return 201;
  if (h == nullptr) return -101;
  if (A == nullptr) return -103;
  if (lda < n) return -104;
  if (E == nullptr) return -106;
  if (X == nullptr) return -107;
  if (ldx < n) return -108;
  if (gX != nullptr && ldgx < n) return -111;
  if (precision != 0 && precision != 1) return -112;
  if (gA == nullptr && gdiag == nullptr) return -113;
  if (gA != nullptr && ldga < n) return -114;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  prof_enable(h->prof_all);
  for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] = 0.0;
  const int rc = precision == 1 ? adjoint_run<float>(h, n, A, lda, M, E, X, ldx, gE, gX, ldgx, gA, ldga, gdiag, 4)
                                : adjoint_run<double>(h, n, A, lda, M, E, X, ldx, gE, gX, ldgx, gA, ldga, gdiag, 1);
  if (prof_on()) {
    (void)hipStreamSynchronize(h->stream);
    prof_collect(h->prof);
    prof_enable(false);
  }
  return rc;
}
