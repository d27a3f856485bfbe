// Launch wrappers of the HIP kernels behind the C interface (internal header).
//
// Conventions shared by every kernel:
//  * the user's A, B, X are column-major with a leading dimension (LAPACK);
//  * every internal n x m block (Q, X, R, A*Q, B*Q, right-hand sides) is
//    row-major, so a row permutation moves contiguous rows;
//  * the shifted matrices z_j B - A and their LU factors are row-major, one
//    n x n matrix per quadrature node, stored back to back;
//  * complex values are interleaved (re, im).
#pragma once

#include <vector>

#include "common.hpp"
#include "prof.hpp"

namespace mf {

// ------------------------------------------------------------------ GEMM
struct GemmArgs {
  int M, N, K;
  const void* A;
  int64_t lda, a_bs;  // element (i,k) of op(A): A[i*lda+k] (K-contiguous) or A[i+k*lda] (M-contiguous)
  const void* B;
  int64_t ldb, b_bs;  // element (k,j) of B: B[k*ldb+j]
  void* C;
  int64_t ldc, c_bs;  // element (i,j) of C: C[i*ldc+j]
  double alpha, beta;
  int tag;  // 1: LU trailing update, 2: contour-solve update (distinct kernel names), else 0
};
// operand forms: OP_N as stored (A K-contiguous, B N-contiguous), OP_T transposed view,
// OP_C conjugate-transposed view
enum GemmOp { OP_N = 0, OP_T = 1, OP_C = 2 };
template <typename R, bool CPLX>
int gemm_op(hipStream_t s, GemmOp opa, GemmOp opb, const GemmArgs& g, int batch);
template <typename R, bool CPLX>
int gemm(hipStream_t s, bool a_mcontig, bool conj_a, const GemmArgs& g, int batch);
// Device scratch for the split-K partial sums of the calling host thread: fn(owner, bytes)
// returns a buffer of at least `bytes` (or nullptr: the product then runs unsplit).
using ScratchFn = void* (*)(void* owner, size_t bytes);
void set_gemm_scratch(ScratchFn fn, void* owner);
// complex FP32 products of the calling host thread use Gauss's three-product scheme
// (default on; fpm(53) = 1 selects the four-product scheme for a call)
void set_gemm_3m(bool on);
bool gemm_3m();
// Tile autotuner for the LU trailing updates (products with tag 1): while tuning is on
// for the calling host thread, the first product of each size class (element type,
// scheme, log2 buckets of M, N, K and batch) times the 64x64, 32x64, 64x32 and 32x32
// tiles on a scratch output (synchronizing the stream) and keeps the fastest for the
// process; later products of the class use it, tuning on or off.  The tile does not
// change the order of the K sums, so every choice gives the same results.
void set_gemm_tuning(bool on);
// number of size classes tuned so far, and the tile index chosen for the last one tuned
int gemm_tuned_classes();

// ------------------------------------------------------------------ LU
constexpr int LU_NB = 64;  // outer panel width of the blocked LU and of the blocked solves

// Row stride of the stored shifted matrices and LU factors: n rounded up to an odd
// multiple of 32 elements.  With a power-of-two stride every row of a column panel
// starts at the same offset modulo the memory-channel interleave, and the panel's
// accesses pile onto a few channels.
__host__ __device__ inline int64_t lu_ld(int64_t n) {
  int64_t b = (n + 31) / 32;
  if ((b & 1) == 0) ++b;
  return b * 32;
}

// Full Hermitian/symmetric copy (ld = n, column-major) from the triangle named by uplo.
template <typename T>
int expand_full(hipStream_t s, char uplo, int64_t n, const T* src, int64_t lds, T* dst);

// LU_j = z_j * B - A, row-major with row stride lu_ld(n) (n x lu_ld(n) entries per
// node), for j = 0..ne-1 (B == nullptr means identity); with b_node, matrix ne is B
// itself (factored beside the shifted matrices for B^-1 products); also sets perm_j =
// identity for every matrix written.  A, B: full storage column-major (ld).
template <typename T, typename C>
int shift_form(hipStream_t s, int64_t n, const T* A, int64_t lda, const T* B, int64_t ldb,
               const c64* z_dev, int ne, C* LU, int* perm, bool b_node = false);

// Blocked right-looking LU with partial pivoting of all ne matrices (P A = L U).
// ipiv (n per node, global row indices), perm (n per node: (PA)[i] = A[perm[i]]),
// perm_inv, a per-node info flag (>0: first zero pivot + 1), and Dinv: per node and per
// diagonal block, the inverses of the unit-lower and of the upper LU_NB x LU_NB blocks
// (row-major, 2 * LU_NB^2 entries per block, ceil(n / LU_NB) blocks per node).
template <typename C>
int lu_factor(hipStream_t s, int64_t n, int ne, C* LU, int* ipiv, int* perm, int* perm_inv, int* info,
              C* Dinv);

// ------------------------------------------------------------------ solves
// Build per-node right-hand sides W_j (row-major n x m, type C) from an FP64 block RHS
// (row-major, ld), each column multiplied by colscale[c]; forward blocks are gathered
// with perm_j (W_j[i] = RHS[perm_j[i]]), conjugate-transpose blocks are not permuted.
// With nreal < n the factors are those of a matrix padded with an identity block: RHS
// has nreal rows and the rows beyond are zero.
template <typename T, typename C>
int rhs_prepare(hipStream_t s, int64_t n, int m, const T* rhs, int64_t ld, const double* colscale,
                int ne, const int* perm, C* Wf, C* Wc, int64_t nreal = -1);

// Inverses of the diagonal blocks of L and U over panels of 4 LU_NB rows, formed once
// per factorization from LU and Dinv; panel_inverse_entries(n) entries of C per node.
size_t panel_inverse_entries(int64_t n);
template <typename C>
int panel_inverses(hipStream_t s, int64_t n, int ne, const C* LU, const C* Dinv, C* Pinv);

// Solve LU_j x = W_j (forward direction; Wf already permuted) and, if Wc != nullptr,
// (LU_j)^H y = W_j for the conjugate direction (unpermuted on output; perm_inv is
// applied by the accumulation).  Results overwrite Wf / Wc; Y (n x m per node) is
// scratch.  All nodes batched.
// The conjugate-transpose direction on a second stream (s2, with its own ping-pong
// buffer Y2 of n x m per node) next to the forward one on s; s waits for it.
template <typename C>
struct SolveSide {
  hipStream_t s2;
  hipEvent_t fork, join;
  C* Y2;
};
template <typename C>
int lu_solve(hipStream_t s, int64_t n, int m, int ne, const C* LU, const C* Pinv, C* Wf, C* Wc, C* Y,
             const SolveSide<C>* side = nullptr, int cls = K_SOLVE_GEMM);

// Refinement of the FP32 contour solves (fpm(50)): dst = (add ? dst : 0) + widen(src);
// row gather dst_j[r] = src_j[perm_inv_j[r]]; residual of node j's system (z_j B - A) x
// = rhs diag(cs) (conj(z_j) for the conjugate node) from FP64 products AX, BX, written
// (row-permuted by perm when given) in FP32.
template <typename C>
int widen(hipStream_t s, int64_t count, const C* src, c64* dst, bool add);
int gather_rows_c64(hipStream_t s, int64_t n, int m, int ne, const c64* src, const int* perm_inv, c64* dst);
template <typename T, typename C>
int ir_residual(hipStream_t s, int64_t n, int m, int ne, const T* rhs, int64_t ld, const double* cs, const c64* z,
                bool conj_z, const int* perm, const c64* AX, const c64* BX, C* out);

// out[c] = Re(sum_r conj(R[r][c]) X[r][c]) / cs[c] for row-major n x m blocks R (FP64)
// and X (solve precision), both with leading dimension m; partial: ceil(n / 256) * m
// doubles.  With X = B^-1 R diag(cs) this is r_c^H B^-1 r_c.
template <typename T, typename C>
int col_dots_mixed(hipStream_t s, int64_t n, int m, const T* R, const C* X, const double* cs, double* out,
                   double* partial);

// Q = (resid ? X*diag(rho) : 0) + diag-scaled sum over nodes (see accumulate in solve.hip).
// With nreal < n (padded factors, see rhs_prepare) only the first nreal rows of Q are formed.
template <typename T, typename C>
int accumulate(hipStream_t s, int64_t n, int m, int ne, const C* Wf, const C* Wc, const int* perm_inv,
               const c64* coef_f, const c64* coef_c, const double* rho, const double* unscale,
               const T* X, T* Q, int resid, int64_t nreal = -1);

// ------------------------------------------------------------------ Rayleigh-Ritz helpers
template <typename T>
int col_absmax(hipStream_t s, int64_t n, int m, const T* X, int64_t ld, double* out);  // out[c] = max_r |X[r][c]|
template <typename T>
int gram_equilibrate(hipStream_t s, int m, T* S, T* Tm, double* d, int* flag);
// Hermitian eigensolver of the m x m row-major H (destroyed): V eigenvectors (columns),
// evals unsorted.  m <= 64: one cooperative scalar Jacobi launch; larger m: block
// Jacobi.  work: jacobi_work_bytes(m, sizeof(T)) bytes.
// big_rel: a block-Jacobi sweep in which no rotation exceeds big_rel * max|diag(H)| is
// the last one (1e-10 for results that are returned; the off-diagonal left behind is of
// the order of big_rel^2 max|diag(H)|).
template <typename T>
int jacobi_eigh(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps_out, double* work,
                double big_rel = 1.0e-10);
// Hermitian eigensolver by Householder reduction to real tridiagonal form, multisection
// bisection, inverse iteration and a blocked back-transformation (tri.hip); m <= 1024.
// H (m x m row-major, full storage) is destroyed; V gets the eigenvectors (columns),
// evals the eigenvalues in ascending order.  A group of more than 64 eigenvalues within
// 1e-10 of the spectral radius of each other is handed to jacobi_eigh (fell_back = 1,
// big_rel passed on).  Synchronizes the stream once.  work: tri_work_bytes(m, sizeof(T)).
template <typename T>
int tri_eigh(hipStream_t s, int m, T* H, T* V, double* evals, char* work, int* fell_back, int* sweeps_out,
             double big_rel);
size_t tri_work_bytes(int m, size_t elem);
template <typename T>
int block_jacobi(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps_out, T* ubuf, int* counter,
                 int max_sweeps, double big_rel);
size_t block_jacobi_work_bytes(int m, size_t elem);
inline size_t jacobi_work_bytes(int m, size_t elem) {
  const size_t a = (size_t)m * m * elem, b = block_jacobi_work_bytes(m, elem);
  return a > b ? a : b;
}
template <typename T>
int gather_scale_cols(hipStream_t s, int rows, int k, const T* V, int ldv, const int* idx,
                      const double* scale, T* G, int ldg);
template <typename T>
int scale_rows_permute_cols(hipStream_t s, int rows, int k, const T* GZ, int ldgz, const double* d,
                            const int* perm, T* W, int ldw);
template <typename T>
int copy_block(hipStream_t s, int rows, int cols, const T* src, int64_t lds, T* dst, int64_t ldd, bool conj_t);
// dst[i][j] = src[p[i]][p[j]] (m x m)
template <typename T>
int sym_permute(hipStream_t s, int m, const T* src, const int* p, T* dst);
// dst[p[r]][:] = src[r][:] (rows x cols, leading dimension cols)
template <typename T>
int scatter_rows(hipStream_t s, int rows, int cols, const T* src, const int* p, T* dst);
template <typename T>
int residual_norms(hipStream_t s, int64_t n, int m, const T* AX, const T* BX, const double* lam, T* R,
                   double* rnorm2, double* bnorm2, double* partial);
template <typename T>
int copy_rm_to_cm(hipStream_t s, int64_t n, int m, const T* src, int64_t lds, T* dst, int64_t ldd,
                  const int* colmap = nullptr);
template <typename T>
int copy_cm_to_rm(hipStream_t s, int64_t n, int m, const T* src, int64_t lds, T* dst, int64_t ldd);
template <typename T>
int random_block(hipStream_t s, int64_t n, int m, uint64_t seed, T* Y, int64_t ld);
// n x m row-major block of +-1 (stochastic count probes; SplitMix64 top bit, counter i + j n)
template <typename T>
int rademacher_block(hipStream_t s, int64_t n, int m, uint64_t seed, T* Y, int64_t ld);
// out[c] = Re(sum_r conj(Y[r][c]) Q[r][c]), row-major n x m blocks with leading dimension m;
// partial: ceil(n / 256) * m doubles
template <typename T>
int col_dots(hipStream_t s, int64_t n, int m, const T* Y, const T* Q, double* out, double* partial);

// ------------------------------------------------------------------ B-orthonormalization (orth.hip)
// Cholesky with column dropping of a Hermitian m x m row-major A (lower part): L in place,
// Linv = pseudo-inverse of L, keep[j] = 1 for kept columns.  work >= 32 m entries.
template <typename T>
int chol_drop(hipStream_t s, int m, T* A, T* Linv, int* keep, double tau, T* work);
// H1 (m x k) = D Linv^H on the kept columns idx
template <typename T>
int build_h1(hipStream_t s, int m, int k, const T* Linv, const double* d, const int* idx, T* H1);
// out = ||S - I||_F (S k x k row-major); part >= k doubles
template <typename T>
int dev_from_identity(hipStream_t s, int k, const T* S, double* part, double* out);
// Z = S^-1/2 (Newton-Schulz, `iters` steps); work >= 3 k^2 entries
template <typename T>
int ns_invsqrt(hipStream_t s, int k, const T* S, T* Z, int iters, T* work);
template <typename T>
int hermitian_part(hipStream_t s, int m, T* H);

// ------------------------------------------------------------------ sparse path (sparse.hip)
// Workspace of one CSR conversion (grown on demand, freed by release()).
struct CsrWork {
  static constexpr int NBUF = 9;
  void* buf[NBUF] = {};
  size_t cap[NBUF] = {};
  void* get(int k, size_t bytes);
  void release();
};
// 0-based full-storage CSR, columns sorted within each row; values in FP64 (vd) and in
// the BiCGSTAB precision R (vr).  Arrays live in the CsrWork it was built in.
template <typename R>
struct CsrMat {
  int64_t n = 0, nnz = 0;
  int32_t* rp = nullptr;
  int32_t* ci = nullptr;
  double* vd = nullptr;
  R* vr = nullptr;
};
// From the caller's CSR (base 0 or 1; uplo 'F', or 'L'/'U' for one triangle of a symmetric
// matrix).  *err: 0 ok, 1 bad row pointers, 2 column index out of range, 3 too many entries.
template <typename R>
int csr_full(hipStream_t s, int64_t n, const double* a, const int32_t* ia, const int32_t* ja, int base, char uplo,
             CsrWork& w, CsrMat<R>& out, int* err);
// Y = M X, X and Y row-major n x m FP64 blocks
int spmm_rm(hipStream_t s, const CsrMat<float>& M, int m, const double* X, int64_t ldx, double* Y, int64_t ldy);
int spmm_rm(hipStream_t s, const CsrMat<double>& M, int m, const double* X, int64_t ldx, double* Y, int64_t ldy);

// per-column BiCGSTAB scalars (FP64)
struct BiCol {
  c64 rho, alpha, omega, beta;
  double bn2;
  int state, its;
};
// One batch of shifted systems (z_j B - A) x = b: columns c = j * m0 + q, node j's shift
// zn[j], right-hand side column q of bh (n x m0 row-major).  Vectors are tile-major:
// element (i, c) at ((c / 64) * n + i) * 64 + c % 64, n x ceil(ncol / 64) * 64 entries.
template <typename C>
struct BiSys {
  using R = typename real_of<C>::type;
  int64_t n = 0;
  int ncol = 0, m0 = 0;
  const CsrMat<R>* A = nullptr;
  const CsrMat<R>* B = nullptr;  // nullptr: identity
  const c64* zn = nullptr;
  const R* bh = nullptr;
  C *x = nullptr, *r = nullptr, *p = nullptr, *v = nullptr, *t = nullptr;
  BiCol* col = nullptr;   // ncol
  int* tiles = nullptr;   // ceil(ncol / 64)
  double* part = nullptr; // 8 * (ceil(n / 256) + 32) * ceil(ncol / 64) * 64
};
// BiCGSTAB on every column to ||r|| <= tol ||b|| or maxit iterations; its[c] = iterations
// of column c.  d_buf, h_buf (pinned): ncol + 64 ints of scratch each.
template <typename C>
int bicgstab_batched(hipStream_t s, const BiSys<C>& sys, int maxit, double tol, std::vector<int>& its, int* d_buf,
                     int* h_buf);
// bh = rhs .* colscale (row-major n x m0), in the BiCGSTAB precision
template <typename R>
int bi_rhs(hipStream_t s, int64_t n, int m0, const double* rhs, const double* cs, R* bh);
// out[c] = sign * Re(sum_i R[i][c] x(i, c)) / cs[c]; R row-major n x m FP64, x tile-major
// (m columns of one node); partial: ceil(n / 256) * m doubles
template <typename C>
int bi_coldots(hipStream_t s, int64_t n, int m, const double* R, const C* x, const double* cs, double sign,
               double* out, double* partial);
// quadrature sum of the sparse path, see sparse.hip (mode 0: set, 1: set + rho X, 2: add)
template <typename C>
int bi_accumulate(hipStream_t s, int64_t n, int m0, int nj, int j0, const C* x, const c64* cf, const double* rho,
                  const double* us, const double* X, double* Q, int mode);

}  // namespace mf
