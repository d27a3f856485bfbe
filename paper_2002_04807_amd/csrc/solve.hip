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
                              C* __restrict__ Wf, C* __restrict__ Wc, int64_t nreal) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= m) return;
  const double sc = cs[c];
  const int64_t blk = n * (int64_t)m;
  if (Wc != nullptr) {
    const c64 v = i < nreal ? convert<c64, T>(rhs[i * ld + c]) : c64(0.0, 0.0);
    const C cv = convert<C, c64>(v * c64(sc, 0.0));
    for (int j = 0; j < ne; ++j) Wc[j * blk + i * m + c] = cv;
  }
  for (int j = 0; j < ne; ++j) {
    const int64_t src = perm[(int64_t)j * n + i];
    const c64 v = src < nreal ? convert<c64, T>(rhs[src * ld + c]) : c64(0.0, 0.0);
    Wf[j * blk + i * m + c] = convert<C, c64>(v * c64(sc, 0.0));
  }
}

template <typename T, typename C>
int rhs_prepare(hipStream_t s, int64_t n, int m, const T* rhs, int64_t ld, const double* colscale,
                int ne, const int* perm, C* Wf, C* Wc, int64_t nreal) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_rhs_prepare<T, C>), grid, dim3(256), 0, s, n, m, rhs, ld, colscale, ne, perm, Wf, Wc,
                     nreal < 0 ? n : nreal);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Column dot products of an FP64 block with a block in the solve precision, in
// 256-row chunks (one partial per chunk and column), then one ordered sum per column.
constexpr int DOT_ROWS = 256;

template <typename T, typename C>
__global__ void k_coldot_mixed_partial(int64_t n, int m, const T* __restrict__ R, const C* __restrict__ X,
                                       double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  double acc = 0.0;
  const int64_t r1 = ((chunk + 1) * DOT_ROWS < n) ? (chunk + 1) * DOT_ROWS : n;
  for (int64_t r = chunk * DOT_ROWS; r < r1; ++r) {
    const c64 a = convert<c64, T>(R[r * m + c]);
    const c64 x = convert<c64, C>(X[r * m + c]);
    acc += a.re * x.re + a.im * x.im;
  }
  part[chunk * m + c] = acc;
}

__global__ void k_coldot_mixed_final(int m, int nchunk, const double* __restrict__ part,
                                     const double* __restrict__ cs, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double acc = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) acc += part[(int64_t)ch * m + c];
  out[c] = acc / cs[c];
}

template <typename T, typename C>
int col_dots_mixed(hipStream_t s, int64_t n, int m, const T* R, const C* X, const double* cs, double* out,
                   double* partial) {
  const int nchunk = (int)((n + DOT_ROWS - 1) / DOT_ROWS);
  hipLaunchKernelGGL((k_coldot_mixed_partial<T, C>), dim3((m + 255) / 256, nchunk), dim3(256), 0, s, n, m, R, X,
                     partial);
  hipLaunchKernelGGL(k_coldot_mixed_final, dim3((m + 255) / 256), dim3(256), 0, s, m, nchunk, partial, cs, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Blocked triangular solves, two levels.  The rows are cut into panels of TRSM_PH =
// TRSM_SUB * LU_NB rows.  Once per factorization the inverse of every panel's
// diagonal block of L and of U is formed (panel_inverses); a solve then takes two
// MFMA products per panel: the panel's rows times the inverse, written to the other
// buffer of a ping-pong pair, and the update of every row beyond the panel, with K =
// the panel height.
//
// The four sweeps differ in direction and in how a coupling block is read:
//   L  (forward, unit lower)      ascending,  A(i, k) = LU[r_i][c_k]
//   U  (forward, upper)           descending, A(i, k) = LU[r_i][c_k]
//   U^H (conjugate node, lower)   ascending,  A(i, k) = conj(LU[c_k][r_i])
//   L^H (conjugate node, upper)   descending, A(i, k) = conj(LU[c_k][r_i])
// with r_i the row being updated and c_k a row of the block just solved; the
// diagonal block uses the upper inverse when DESC != HERM, conjugate-transposed
// when HERM.
constexpr int TRSM_SUB = 4;
constexpr int TRSM_PH = TRSM_SUB * LU_NB;

int64_t panel_count(int64_t n) { return (n + TRSM_PH - 1) / TRSM_PH; }
size_t panel_inverse_entries(int64_t n) { return (size_t)panel_count(n) * 2 * TRSM_PH * TRSM_PH; }

// right-hand-side columns per workgroup: 16 keeps the LDS tiles of complex FP32 at 65 KB, two
// workgroups per compute unit (32 columns: 97 KB, one; the batched factorizations' panel
// inverses took 14 ms more per call)
template <typename C> struct trsm_cols { static constexpr int value = 16; };

// In-LDS block solve of one panel, used to form the panel inverses from the
// identity.  Workgroup (x, y, z): CW right-hand-side columns x, panel pan0 + y, node
// z.  The panel's rows live at W + z * w_node + y * w_panel (+ p0 * ldw when
// rows_global), one row every ldw entries; rows past n are treated as zero.
template <typename C, bool DESC, bool HERM>
__global__ __launch_bounds__(256) void k_trsm_panel(int64_t n, int ncols, int64_t pan0, const C* __restrict__ LUall,
                                                    const C* __restrict__ Dinv, int64_t dstride, C* __restrict__ Wall,
                                                    int64_t ldw, int64_t w_node, int64_t w_panel, int rows_global) {
  constexpr int CW = trsm_cols<C>::value;
  constexpr int RR = 4;        // rows per thread: 16 row groups x 4 = LU_NB
  constexpr int RC = CW / 16;  // columns per thread: 16 column groups
  __shared__ C Ws[TRSM_PH][CW];
  __shared__ C As[LU_NB][LU_NB + 1];
  const int tid = threadIdx.x;
  const int node = blockIdx.z;
  const int c0 = blockIdx.x * CW;
  const int64_t p0 = (pan0 + blockIdx.y) * TRSM_PH;
  const int nsb = (int)((min<int64_t>(TRSM_PH, n - p0) + LU_NB - 1) / LU_NB);
  const int64_t ld = lu_ld(n);
  const C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  const C* __restrict__ D = Dinv + (int64_t)node * dstride;
  C* __restrict__ W = Wall + (int64_t)node * w_node + (int64_t)blockIdx.y * w_panel + (rows_global ? p0 * ldw : 0);
  const int rows = nsb * LU_NB;
  for (int e = tid; e < rows * CW; e += 256) {
    const int r = e / CW, c = e % CW;
    Ws[r][c] = (p0 + r < n && c0 + c < ncols) ? W[(int64_t)r * ldw + c0 + c] : C(0);
  }
  const int tr = (tid >> 4) * RR, tc = (tid & 15) * RC;
  for (int step = 0; step < nsb; ++step) {
    const int b = DESC ? nsb - 1 - step : step;
    const int64_t rb = p0 + (int64_t)b * LU_NB;
    const C* __restrict__ Di = D + (rb / LU_NB) * 2 * LU_NB * LU_NB + ((DESC != HERM) ? LU_NB * LU_NB : 0);
    __syncthreads();
    for (int e = tid; e < LU_NB * LU_NB; e += 256) {
      const int a = e / LU_NB, c = e % LU_NB;
      if (HERM) As[c][a] = conj(Di[e]);  // Di[a][c] is op(D)(c, a)
      else As[a][c] = Di[e];
    }
    __syncthreads();
    C acc[RR][RC];
    for (int i = 0; i < RR; ++i)
      for (int j = 0; j < RC; ++j) acc[i][j] = C(0);
    for (int k = 0; k < LU_NB; ++k) {
      C a[RR], x[RC];
      for (int i = 0; i < RR; ++i) a[i] = As[tr + i][k];
      for (int j = 0; j < RC; ++j) x[j] = Ws[b * LU_NB + k][tc + j];
      for (int i = 0; i < RR; ++i)
        for (int j = 0; j < RC; ++j) acc[i][j] = acc[i][j] + a[i] * x[j];
    }
    __syncthreads();
    for (int i = 0; i < RR; ++i)
      for (int j = 0; j < RC; ++j) Ws[b * LU_NB + tr + i][tc + j] = acc[i][j];
    for (int s2 = step + 1; s2 < nsb; ++s2) {
      const int b2 = DESC ? nsb - 1 - s2 : s2;
      const int64_t rb2 = p0 + (int64_t)b2 * LU_NB;
      __syncthreads();
      for (int e = tid; e < LU_NB * LU_NB; e += 256) {
        const int a = e / LU_NB, c = e % LU_NB;  // c runs along memory
        if (HERM) {
          // As[i][k] = conj(LU[rb + k][rb2 + i]) with k = a, i = c
          As[c][a] = (rb + a < n && rb2 + c < n) ? conj(LU[(rb + a) * ld + rb2 + c]) : C(0);
        } else {
          As[a][c] = (rb2 + a < n && rb + c < n) ? LU[(rb2 + a) * ld + rb + c] : C(0);
        }
      }
      __syncthreads();
      for (int i = 0; i < RR; ++i)
        for (int j = 0; j < RC; ++j) acc[i][j] = C(0);
      for (int k = 0; k < LU_NB; ++k) {
        C a[RR], x[RC];
        for (int i = 0; i < RR; ++i) a[i] = As[tr + i][k];
        for (int j = 0; j < RC; ++j) x[j] = Ws[b * LU_NB + k][tc + j];
        for (int i = 0; i < RR; ++i)
          for (int j = 0; j < RC; ++j) acc[i][j] = acc[i][j] + a[i] * x[j];
      }
      for (int i = 0; i < RR; ++i)
        for (int j = 0; j < RC; ++j) Ws[b2 * LU_NB + tr + i][tc + j] = Ws[b2 * LU_NB + tr + i][tc + j] - acc[i][j];
    }
  }
  __syncthreads();
  for (int e = tid; e < rows * CW; e += 256) {
    const int r = e / CW, c = e % CW;
    if (p0 + r < n && c0 + c < ncols) W[(int64_t)r * ldw + c0 + c] = Ws[r][c];
  }
}

template <typename C>
__global__ void k_identity_panels(int64_t count, C* P) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const int64_t w = e % ((int64_t)TRSM_PH * TRSM_PH);
  P[e] = (w / TRSM_PH == w % TRSM_PH) ? C(1) : C(0);
}

// Pinv, per node: panel_count(n) x {L_PP^-1, U_PP^-1}, each TRSM_PH x TRSM_PH
// row-major (a narrower last panel uses the leading block).
template <typename C>
int panel_inverses(hipStream_t s, int64_t n, int ne, const C* LU, const C* Dinv, C* Pinv) {
  constexpr int CW = trsm_cols<C>::value;
  const int64_t npan = panel_count(n);
  const int64_t nblk = (n + LU_NB - 1) / LU_NB;
  const int64_t dstride = nblk * 2 * LU_NB * LU_NB;
  const int64_t per_node = (int64_t)panel_inverse_entries(n);
  const int64_t count = per_node * ne;
  hipLaunchKernelGGL((k_identity_panels<C>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, Pinv);
  const dim3 grid(TRSM_PH / CW, (unsigned)npan, (unsigned)ne);
  const int64_t sq = (int64_t)TRSM_PH * TRSM_PH;
  hipLaunchKernelGGL((k_trsm_panel<C, false, false>), grid, dim3(256), 0, s, n, TRSM_PH, (int64_t)0, LU, Dinv,
                     dstride, Pinv, (int64_t)TRSM_PH, per_node, 2 * sq, 0);
  hipLaunchKernelGGL((k_trsm_panel<C, true, false>), grid, dim3(256), 0, s, n, TRSM_PH, (int64_t)0, LU, Dinv,
                     dstride, Pinv + sq, (int64_t)TRSM_PH, per_node, 2 * sq, 0);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename C>
int lu_solve(hipStream_t s, int64_t n, int m, int ne, const C* LU, const C* Pinv, C* Wf, C* Wc, C* Y,
             const SolveSide<C>* side, int cls) {
  using R = typename real_of<C>::type;
  const int64_t wstride = n * (int64_t)m;
  const int64_t ld = lu_ld(n);
  const int64_t lstride = n * ld;
  const int64_t npan = panel_count(n);
  const int64_t sq = (int64_t)TRSM_PH * TRSM_PH;
  const int64_t pstride = (int64_t)panel_inverse_entries(n);
  // one sweep: rows of the right-hand sides in `in`, solution to `out` (in is consumed)
  auto sweep = [&](hipStream_t st, const C* in0, C* out, bool desc, bool herm) -> int {
    C* in = const_cast<C*>(in0);
    for (int64_t q = 0; q < npan; ++q) {
      const int64_t p = desc ? npan - 1 - q : q;
      const int64_t p0 = p * TRSM_PH;
      const int64_t ph = std::min<int64_t>(TRSM_PH, n - p0);
      // out_P = op(inverse of the diagonal block) in_P
      GemmArgs d{};
      d.M = (int)ph; d.N = m; d.K = (int)ph;
      d.A = Pinv + p * 2 * sq + ((desc != herm) ? sq : 0); d.lda = TRSM_PH; d.a_bs = pstride;
      d.B = in + p0 * m; d.ldb = m; d.b_bs = wstride;
      d.C = out + p0 * m; d.ldc = m; d.c_bs = wstride;
      d.alpha = 1.0; d.beta = 0.0;
      if (gemm<R, is_cplx<C>::value>(st, herm, herm, d, ne)) return -2;
      // rows beyond the panel: in_rest -= A out_P
      GemmArgs g{};
      g.N = m; g.K = (int)ph;
      g.B = out + p0 * m; g.ldb = m; g.b_bs = wstride;
      g.lda = ld; g.a_bs = lstride;
      g.c_bs = wstride; g.ldc = m;
      g.alpha = -1.0; g.beta = 1.0;
      if (!desc) {
        const int64_t rest = n - p0 - ph;
        if (rest <= 0) continue;
        g.M = (int)rest;
        g.C = in + (p0 + ph) * m;
        // L: rows below the panel, its columns; U^H: M-contiguous view of the panel's U rows
        g.A = herm ? LU + p0 * ld + p0 + ph : LU + (p0 + ph) * ld + p0;
      } else {
        if (p0 <= 0) continue;
        g.M = (int)p0;
        g.C = in;
        // U: rows above the panel, its columns; L^H: M-contiguous view of the panel's L rows
        g.A = herm ? LU + p0 * ld : LU + p0;
      }
      if (gemm<R, is_cplx<C>::value>(st, herm, herm, g, ne)) return -2;
    }
    return 0;
  };
  // algorithmic work of one direction: 8 n^2 m flops per node (L and U sweeps)
  const double dir_flops = 8.0 * (double)n * n * m * ne;
  const double dir_bytes = (double)sizeof(C) * ne * ((double)n * n + 2.0 * n * m);
  if (Wf != nullptr && Wc != nullptr && side != nullptr) {
    // both directions at once: they share only the factors, which they read; the
    // conjugate-transpose one runs on side->s2 with its own ping-pong buffer
    const int tok = prof_begin(s);
    if (hipEventRecord(side->fork, s) != hipSuccess) return -2;
    if (hipStreamWaitEvent(side->s2, side->fork, 0) != hipSuccess) return -2;
    if (sweep(side->s2, Wc, side->Y2, false, true) || sweep(side->s2, side->Y2, Wc, true, true)) return -2;
    if (hipEventRecord(side->join, side->s2) != hipSuccess) return -2;
    if (sweep(s, Wf, Y, false, false) || sweep(s, Y, Wf, true, false)) return -2;
    if (hipStreamWaitEvent(s, side->join, 0) != hipSuccess) return -2;
    prof_end(tok, s, cls, 2.0 * dir_flops, 2.0 * dir_bytes);
    return 0;
  }
  // forward direction: L (W -> Y) then U (Y -> W); skipped when Wf is null
  int tok;
  if (Wf != nullptr) {
    tok = prof_begin(s);
    if (sweep(s, Wf, Y, false, false) || sweep(s, Y, Wf, true, false)) return -2;
    prof_end(tok, s, cls, dir_flops, dir_bytes);
  }
  if (Wc == nullptr) return 0;
  // conjugate-transpose direction: U^H (lower) then L^H (unit upper)
  tok = prof_begin(s);
  if (sweep(s, Wc, Y, false, true) || sweep(s, Y, Wc, true, true)) return -2;
  prof_end(tok, s, cls, dir_flops, dir_bytes);
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
               const T* X, T* Q, int resid, int64_t nreal) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)(nreal < 0 ? n : nreal));
  hipLaunchKernelGGL((k_accumulate<T, C>), grid, dim3(256), 0, s, n, m, ne, Wf, Wc, perm_inv, coef_f,
                     coef_c, rho, unscale, X, Q, resid);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Extra iterative refinement of the FP32 contour solves (fpm(50) steps): the
// solutions are kept in FP64, their residuals against the FP64 operator are formed
// with FP64 products, solved again with the FP32 factors and added.

// dst = (add ? dst : 0) + widen(src), count elements
template <typename C>
__global__ void k_widen(int64_t count, const C* __restrict__ src, c64* __restrict__ dst, int add) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  const c64 v = convert<c64, C>(src[e]);
  dst[e] = add ? dst[e] + v : v;
}

template <typename C>
int widen(hipStream_t s, int64_t count, const C* src, c64* dst, bool add) {
  hipLaunchKernelGGL((k_widen<C>), dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src, dst,
                     add ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// dst_j[r][:] = src_j[perm_inv_j[r]][:]  (n x m per node)
__global__ void k_gather_rows_c64(int64_t n, int m, const c64* __restrict__ src, const int* __restrict__ perm_inv,
                                  c64* __restrict__ dst) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  const int64_t j = blockIdx.z;
  if (c >= m) return;
  const int64_t blk = n * (int64_t)m;
  dst[j * blk + r * m + c] = src[j * blk + (int64_t)perm_inv[j * n + r] * m + c];
}

int gather_rows_c64(hipStream_t s, int64_t n, int m, int ne, const c64* src, const int* perm_inv, c64* dst) {
  hipLaunchKernelGGL(k_gather_rows_c64, dim3((unsigned)((m + 255) / 256), (unsigned)n, (unsigned)ne), dim3(256), 0, s,
                     n, m, src, perm_inv, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Residual of node j's system (z_j B - A) x = b with b = rhs * diag(cs) (or the
// conjugate node conj(z_j) for the conjugate-transpose solve of a Hermitian pencil):
// r = b - z BX + AX, rounded to C.  out_j[i] = r[perm_j[i]] (forward solves take
// permuted right-hand sides) or r[i] when perm is null.
template <typename T, typename C>
__global__ void k_ir_residual(int64_t n, int m, const T* __restrict__ rhs, int64_t ld, const double* __restrict__ cs,
                              const c64* __restrict__ z, int conj_z, const int* __restrict__ perm,
                              const c64* __restrict__ AX, const c64* __restrict__ BX, C* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  const int64_t j = blockIdx.z;
  if (c >= m) return;
  const int64_t blk = n * (int64_t)m;
  const int64_t src = perm ? (int64_t)perm[j * n + i] : i;
  const c64 zj = conj_z ? c64(z[j].re, -z[j].im) : z[j];
  const c64 b = convert<c64, T>(rhs[src * ld + c]) * c64(cs[c], 0.0);
  const c64 r = b - zj * BX[j * blk + src * m + c] + AX[j * blk + src * m + c];
  out[j * blk + i * m + c] = convert<C, c64>(r);
}

template <typename T, typename C>
int ir_residual(hipStream_t s, int64_t n, int m, int ne, const T* rhs, int64_t ld, const double* cs, const c64* z,
                bool conj_z, const int* perm, const c64* AX, const c64* BX, C* out) {
  hipLaunchKernelGGL((k_ir_residual<T, C>), dim3((unsigned)((m + 255) / 256), (unsigned)n, (unsigned)ne), dim3(256), 0,
                     s, n, m, rhs, ld, cs, z, conj_z ? 1 : 0, perm, AX, BX, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int widen<c32>(hipStream_t, int64_t, const c32*, c64*, bool);
template int ir_residual<double, c32>(hipStream_t, int64_t, int, int, const double*, int64_t, const double*,
                                      const c64*, bool, const int*, const c64*, const c64*, c32*);
template int ir_residual<c64, c32>(hipStream_t, int64_t, int, int, const c64*, int64_t, const double*, const c64*,
                                   bool, const int*, const c64*, const c64*, c32*);

template int rhs_prepare<double, c32>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, c32*, c32*, int64_t);
template int rhs_prepare<double, c64>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, c64*, c64*, int64_t);
template int rhs_prepare<c64, c32>(hipStream_t, int64_t, int, const c64*, int64_t, const double*, int, const int*, c32*, c32*, int64_t);
template int rhs_prepare<c64, c64>(hipStream_t, int64_t, int, const c64*, int64_t, const double*, int, const int*, c64*, c64*, int64_t);
template int lu_solve<c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, c32*, c32*, c32*,
                          const SolveSide<c32>*, int);
template int lu_solve<c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, c64*, c64*, c64*,
                          const SolveSide<c64>*, int);
template int panel_inverses<c32>(hipStream_t, int64_t, int, const c32*, const c32*, c32*);
template int panel_inverses<c64>(hipStream_t, int64_t, int, const c64*, const c64*, c64*);
template int rhs_prepare<double, float>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, float*, float*, int64_t);
template int rhs_prepare<double, double>(hipStream_t, int64_t, int, const double*, int64_t, const double*, int, const int*, double*, double*, int64_t);
template int lu_solve<float>(hipStream_t, int64_t, int, int, const float*, const float*, float*, float*, float*,
                             const SolveSide<float>*, int);
template int lu_solve<double>(hipStream_t, int64_t, int, int, const double*, const double*, double*, double*, double*,
                              const SolveSide<double>*, int);
template int panel_inverses<float>(hipStream_t, int64_t, int, const float*, const float*, float*);
template int panel_inverses<double>(hipStream_t, int64_t, int, const double*, const double*, double*);
template int accumulate<double, c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, const int*, const c64*, const c64*, const double*, const double*, const double*, double*, int, int64_t);
template int accumulate<double, c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, const int*, const c64*, const c64*, const double*, const double*, const double*, double*, int, int64_t);
template int accumulate<c64, c32>(hipStream_t, int64_t, int, int, const c32*, const c32*, const int*, const c64*, const c64*, const double*, const double*, const c64*, c64*, int, int64_t);
template int accumulate<c64, c64>(hipStream_t, int64_t, int, int, const c64*, const c64*, const int*, const c64*, const c64*, const double*, const double*, const c64*, c64*, int, int64_t);

template int col_dots_mixed<double, c32>(hipStream_t, int64_t, int, const double*, const c32*, const double*,
                                         double*, double*);
template int col_dots_mixed<double, c64>(hipStream_t, int64_t, int, const double*, const c64*, const double*,
                                         double*, double*);
template int col_dots_mixed<c64, c32>(hipStream_t, int64_t, int, const c64*, const c32*, const double*, double*,
                                      double*);
template int col_dots_mixed<c64, c64>(hipStream_t, int64_t, int, const c64*, const c64*, const double*, double*,
                                      double*);

}  // namespace mf
