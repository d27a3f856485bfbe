// Shifted matrices and their blocked LU factorization with partial pivoting (gfx950).
//
// One factorization per quadrature node z_j of Az_j = z_j B - A (FEAST Hermitian RCI
// case 10; the factorizations are kept for every later solve, fpm(10)=1).  All nodes
// are factored together: every launch covers the ne independent matrices.
//
// Right-looking blocked LU, panel width LU_NB:
//   panel     a cooperative launch of ceil((n-k)/RPW) workgroups per node holds the
//             (n-k) x LU_NB panel in registers and exchanges one pivot candidate per
//             workgroup and column (k_panel_coop).  When the grid cannot be resident
//             at once, one 1024-thread workgroup per node factors the panel instead,
//             in register-resident sub-panels of IB columns: the
//             pivot of each column is the row of largest |re|+|im| (lowest index on
//             ties), found with a wavefront shuffle reduction and an LDS reduction
//             across the 16 wavefronts; the rows are exchanged through LDS, the column
//             is scaled and the sub-panel updated in registers.  The rest of the panel
//             is swapped, solved and updated from the sub-panel.
//   invert    the unit-lower and the upper LU_NB x LU_NB diagonal blocks are inverted
//             in LDS and stored beside the factors, so that every triangular block
//             solve (here and in the contour solves) is an MFMA product.
//   laswp     the panel's interchanges applied to all columns outside the panel
//             (rows are contiguous because the matrices are row-major).
//   U12       U12 = L11^-1 A12 (MFMA product, in place).
//   trailing  A22 -= L21 U12 (MFMA complex GEMM, the dense contraction of the LU).
#include <climits>

#include "kernels.hpp"

namespace mf {

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_expand_full(int64_t n, char uplo, const T* __restrict__ src, int64_t lds, T* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // row
  const int64_t j = blockIdx.y;                                       // column
  if (i >= n) return;
  // column-major: element (i, j) at src[i + j*lds]
  T v;
  const bool lower = (uplo == 'L' || uplo == 'l');
  if (i == j) {
    v = T(real_part(src[i + j * lds]));
  } else if ((i > j) == lower) {
    v = src[i + j * lds];
  } else {
    v = conj(src[j + i * lds]);
  }
  dst[i + j * n] = v;
}

template <typename T>
int expand_full(hipStream_t s, char uplo, int64_t n, const T* src, int64_t lds, T* dst) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_expand_full<T>), grid, dim3(256), 0, s, n, uplo, src, lds, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
template <typename T, typename C>
__global__ void k_shift_form(int64_t n, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                             int64_t ldb, const c64* __restrict__ z, int ne, C* __restrict__ LU,
                             int* __restrict__ perm) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= n) return;
  // For a Hermitian matrix stored column-major, buf[i*ld + c] is element (c, i), the
  // conjugate of element (i, c): reading it keeps the row-major writes coalesced.
  const c64 a = convert<c64, T>(conj(A[i * lda + c]));
  c64 b;
  if (B != nullptr) b = convert<c64, T>(conj(B[i * ldb + c]));
  else b = c64(i == c ? 1.0 : 0.0, 0.0);
  for (int j = 0; j < ne; ++j) {
    const c64 v = z[j] * b - a;
    LU[(int64_t)j * n * n + i * n + c] = convert<C, c64>(v);
  }
  if (i == 0)
    for (int j = 0; j < ne; ++j) perm[(int64_t)j * n + c] = (int)c;
}

template <typename T, typename C>
int shift_form(hipStream_t s, int64_t n, const T* A, int64_t lda, const T* B, int64_t ldb,
               const c64* z_dev, int ne, C* LU, int* perm) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_shift_form<T, C>), grid, dim3(256), 0, s, n, A, lda, B, ldb, z_dev, ne, LU, perm);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// panel factorization
constexpr int PANEL_THREADS = 1024;
constexpr int MAX_N = 16384;

template <typename R>
__device__ inline void argmax_merge(R& v, int& i, R ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}

template <typename C, int IB, int RMAX>
__global__ __launch_bounds__(PANEL_THREADS) void k_panel(int64_t n, int k, int nbc, C* __restrict__ LUall,
                                                           int* __restrict__ ipiv_all, int* __restrict__ perm_all,
                                                           int* __restrict__ info_all) {
  using R = typename real_of<C>::type;
  const int node = blockIdx.x;
  C* __restrict__ LU = LUall + (int64_t)node * n * n;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  __shared__ int s_perm[MAX_N];
  __shared__ int s_ipiv[LU_NB];
  __shared__ C prow[IB], crow[IB];
  __shared__ C Lsub[IB][IB];
  __shared__ C Ublk[IB][LU_NB];
  __shared__ R red_v[PANEL_THREADS / 64];
  __shared__ int red_i[PANEL_THREADS / 64];
  __shared__ int s_p;
  __shared__ int s_zero;

  const int rows_k = (int)(n - k);
  for (int r = tid; r < rows_k; r += PANEL_THREADS) s_perm[r] = perm_all[(int64_t)node * n + k + r];
  if (tid == 0) s_zero = 0;
  __syncthreads();

  for (int jb = 0; jb < nbc; jb += IB) {
    const int ibc = min(IB, nbc - jb);
    const int64_t row0 = k + jb;
    const int mr = (int)(n - row0);
    C v[RMAX][IB];
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
      const int r = tid + t * PANEL_THREADS;
#pragma unroll
      for (int c = 0; c < IB; ++c)
        v[t][c] = (r < mr && c < ibc) ? LU[(row0 + r) * n + row0 + c] : C(0);
    }

    for (int j = 0; j < ibc; ++j) {
      // ---- pivot search over local rows r >= j of sub-panel column j
      R best = R(-1);
      int bi = INT_MAX;
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int r = tid + t * PANEL_THREADS;
        R a = R(-1);
#pragma unroll
        for (int c = 0; c < IB; ++c)
          if (c == j) a = abs1(v[t][c]);
        if (r >= j && r < mr && a > best) {
          best = a;
          bi = r;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const R ov = __shfl_xor(best, off);
        const int oi = __shfl_xor(bi, off);
        argmax_merge(best, bi, ov, oi);
      }
      if (lane == 0) {
        red_v[wave] = best;
        red_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        R bv = red_v[0];
        int bx = red_i[0];
        for (int w = 1; w < PANEL_THREADS / 64; ++w) argmax_merge(bv, bx, red_v[w], red_i[w]);
        if (bx == INT_MAX || !(bv > R(0))) {
          // zero (or non-finite) column: keep the diagonal row, flag the breakdown
          if (s_zero == 0) s_zero = (int)(row0 + j) + 1;
          bx = j;
        }
        s_p = bx;
        s_ipiv[jb + j] = (int)row0 + bx;
      }
      __syncthreads();
      const int p = s_p;
      // ---- exchange local rows j and p through LDS
      if (tid == (p & (PANEL_THREADS - 1))) {
#pragma unroll
        for (int t = 0; t < RMAX; ++t)
          if (t == (p >> 10))
#pragma unroll
            for (int c = 0; c < IB; ++c) prow[c] = v[t][c];
      }
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < IB; ++c) crow[c] = v[0][c];
      }
      __syncthreads();
      if (tid == j) {
#pragma unroll
        for (int c = 0; c < IB; ++c) v[0][c] = prow[c];
      }
      if (p != j && tid == (p & (PANEL_THREADS - 1))) {
#pragma unroll
        for (int t = 0; t < RMAX; ++t)
          if (t == (p >> 10))
#pragma unroll
            for (int c = 0; c < IB; ++c) v[t][c] = crow[c];
      }
      // ---- scale column j below the diagonal and update the sub-panel
      C piv = C(0);
#pragma unroll
      for (int c = 0; c < IB; ++c)
        if (c == j) piv = prow[c];
      const bool ok = abs1(piv) > R(0);
      const C inv = ok ? cdiv(C(1), piv) : C(0);
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int r = tid + t * PANEL_THREADS;
        if (r > j && r < mr && ok) {
          C l = C(0);
#pragma unroll
          for (int c = 0; c < IB; ++c)
            if (c == j) l = v[t][c] * inv;
#pragma unroll
          for (int c = 0; c < IB; ++c) {
            if (c == j) v[t][c] = l;
            else if (c > j) v[t][c] = v[t][c] - l * prow[c];
          }
        }
      }
      __syncthreads();
    }

    // ---- write the factored sub-panel back; keep its unit-lower top block in LDS
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
      const int r = tid + t * PANEL_THREADS;
#pragma unroll
      for (int c = 0; c < IB; ++c)
        if (r < mr && c < ibc) LU[(row0 + r) * n + row0 + c] = v[t][c];
    }
    if (tid < ibc) {
#pragma unroll
      for (int c = 0; c < IB; ++c) Lsub[tid][c] = v[0][c];
    }
    __syncthreads();

    // ---- interchanges of this sub-panel applied to the other panel columns, and to perm
    const int ocols = nbc - ibc;
    for (int cc = tid; cc < ocols; cc += PANEL_THREADS) {
      const int64_t col = (cc < jb) ? (k + cc) : (k + cc + ibc);
      for (int j = 0; j < ibc; ++j) {
        const int64_t a = row0 + j, b = s_ipiv[jb + j];
        if (a != b) {
          const C t0 = LU[a * n + col];
          LU[a * n + col] = LU[b * n + col];
          LU[b * n + col] = t0;
        }
      }
    }
    if (tid == 0) {
      for (int j = 0; j < ibc; ++j) {
        const int a = jb + j, b = s_ipiv[jb + j] - k;
        const int t0 = s_perm[a];
        s_perm[a] = s_perm[b];
        s_perm[b] = t0;
      }
    }
    __syncthreads();

    // ---- U rows of the sub-panel for the remaining panel columns
    const int ucols = (int)((k + nbc) - (row0 + ibc));
    for (int cc = tid; cc < ucols; cc += PANEL_THREADS) {
      const int64_t col = row0 + ibc + cc;
      C x[IB];
#pragma unroll
      for (int j = 0; j < IB; ++j) {
        if (j < ibc) {
          C s = LU[(row0 + j) * n + col];
#pragma unroll
          for (int i = 0; i < IB; ++i)
            if (i < j) s = s - Lsub[j][i] * x[i];
          x[j] = s;
          LU[(row0 + j) * n + col] = s;
          Ublk[j][cc] = s;
        }
      }
    }
    __syncthreads();

    // ---- update of the remaining panel columns below the sub-panel
    if (ucols > 0) {
#pragma unroll
      for (int t = 0; t < RMAX; ++t) {
        const int r = tid + t * PANEL_THREADS;
        if (r >= ibc && r < mr) {
          for (int cc = 0; cc < ucols; ++cc) {
            const int64_t idx = (row0 + r) * n + row0 + ibc + cc;
            C s = LU[idx];
#pragma unroll
            for (int i = 0; i < IB; ++i)
              if (i < ibc) s = s - v[t][i] * Ublk[i][cc];
            LU[idx] = s;
          }
        }
      }
    }
    __syncthreads();
  }

  for (int r = tid; r < rows_k; r += PANEL_THREADS) perm_all[(int64_t)node * n + k + r] = s_perm[r];
  if (tid < nbc) ipiv_all[(int64_t)node * n + k + tid] = s_ipiv[tid];
  if (tid == 0 && s_zero != 0 && info_all[node] == 0) info_all[node] = s_zero;
}

// ---------------------------------------------------------------------------
// inverses of the diagonal blocks: Linv (unit lower) and Uinv (upper), row-major
// LU_NB x LU_NB per block, zero-padded when the last block is narrower.
template <typename C>
__global__ __launch_bounds__(256) void k_invert_diag(int64_t n, int kfirst, int nblocks, const C* __restrict__ LUall,
                                                      C* __restrict__ Dinv) {
  const int node = blockIdx.y;
  const int blk = kfirst / LU_NB + blockIdx.x;
  const int64_t k = (int64_t)blk * LU_NB;
  const int nbc = (int)min<int64_t>(LU_NB, n - k);
  const C* __restrict__ LU = LUall + (int64_t)node * n * n;
  const int nblk_total = (int)((n + LU_NB - 1) / LU_NB);
  C* __restrict__ Li = Dinv + ((int64_t)node * nblk_total + blk) * 2 * LU_NB * LU_NB;
  C* __restrict__ Ui = Li + LU_NB * LU_NB;
  __shared__ C Ls[LU_NB][LU_NB + 1];
  __shared__ C X[LU_NB][LU_NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < LU_NB * LU_NB; e += 256) {
    const int i = e / LU_NB, j = e % LU_NB;
    Ls[i][j] = (i < nbc && j < nbc) ? LU[(k + i) * n + k + j] : C(0);
  }
  __syncthreads();
  // unit lower inverse: column c solved by thread c
  if (tid < LU_NB) {
    const int c = tid;
    for (int i = 0; i < LU_NB; ++i) {
      C s = (i == c) ? C(1) : C(0);
      if (i > c && i < nbc) {
        for (int j = c; j < i; ++j) s = s - Ls[i][j] * X[j][c];
      }
      if (i >= nbc || c >= nbc) s = C(0);
      X[i][c] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < LU_NB * LU_NB; e += 256) Li[e] = X[e / LU_NB][e % LU_NB];
  __syncthreads();
  // upper inverse: column c by back substitution
  if (tid < LU_NB) {
    const int c = tid;
    for (int i = LU_NB - 1; i >= 0; --i) {
      C s = C(0);
      if (c < nbc && i <= c) {
        s = (i == c) ? C(1) : C(0);
        for (int j = i + 1; j <= c; ++j) s = s - Ls[i][j] * X[j][c];
        const C d = Ls[i][i];
        s = (abs1(d) > 0) ? cdiv(s, d) : C(0);
      }
      X[i][c] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < LU_NB * LU_NB; e += 256) Ui[e] = X[e / LU_NB][e % LU_NB];
}

// ---------------------------------------------------------------------------
template <typename C>
__global__ void k_laswp(int64_t n, int k, int nbc, C* __restrict__ LUall, const int* __restrict__ ipiv_all) {
  __shared__ int sp[LU_NB];
  const int node = blockIdx.y;
  if (threadIdx.x < nbc) sp[threadIdx.x] = ipiv_all[(int64_t)node * n + k + threadIdx.x];
  __syncthreads();
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n || (c >= k && c < k + nbc)) return;
  C* __restrict__ LU = LUall + (int64_t)node * n * n;
  for (int j = 0; j < nbc; ++j) {
    const int64_t a = k + j, b = sp[j];
    if (a != b) {
      const C t0 = LU[a * n + c];
      LU[a * n + c] = LU[b * n + c];
      LU[b * n + c] = t0;
    }
  }
}

__global__ void k_perm_inverse(int64_t n, int ne, const int* __restrict__ perm, int* __restrict__ perm_inv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int node = blockIdx.y;
  if (i >= n) return;
  perm_inv[(int64_t)node * n + perm[(int64_t)node * n + i]] = (int)i;
}

// ---------------------------------------------------------------------------
// Cooperative panel factorization: G workgroups per node, all resident at once
// (cooperative launch).  Workgroup g holds panel rows [g*RPW, (g+1)*RPW) in registers,
// QPR threads per row, CPT = 64/QPR columns per thread.  For every column j:
//   1. each workgroup finds its candidate (largest |re|+|im| among its rows not yet
//      chosen, lowest global row on ties) and publishes value, row and the whole row;
//   2. one arrive/wait barrier across the node's workgroups (device-scope atomics);
//   3. every workgroup picks the same pivot from the G candidates and reads its row;
//   4. rows not yet chosen are scaled and updated in registers; the pivot's owner
//      retires it (it is row j of U).
// Rows are not moved while the panel is factored: at the end, the LAPACK sequence of
// interchanges (k + j <-> current position of pivot j) is replayed on a short list
// of moved rows, every row is written once to its final position, and ipiv, perm
// are updated.  Same pivots as row-by-row partial pivoting with that tie rule.
constexpr int COOP_THREADS = 256;

template <typename C>
struct PanelWork {
  using R = typename real_of<C>::type;
  R* cv;    // [2][gmax] candidate values (double-buffered by column parity)
  int* ci;  // [2][gmax] candidate global rows
  C* cr;    // [2][gmax][LU_NB] candidate rows
};

template <typename C>
__host__ __device__ inline PanelWork<C> panel_work(char* base, int node, int gmax) {
  using R = typename real_of<C>::type;
  const size_t per_node = (size_t)2 * gmax * (sizeof(R) + sizeof(int) + LU_NB * sizeof(C)) + 256;
  char* p = base + per_node * node;
  PanelWork<C> w;
  w.cr = reinterpret_cast<C*>(p);
  w.cv = reinterpret_cast<R*>(p + (size_t)2 * gmax * LU_NB * sizeof(C));
  w.ci = reinterpret_cast<int*>(p + (size_t)2 * gmax * (LU_NB * sizeof(C) + sizeof(R)));
  return w;
}

template <typename C>
size_t panel_work_bytes(int64_t n, int ne, int rpw) {
  using R = typename real_of<C>::type;
  const int gmax = (int)((n + rpw - 1) / rpw);
  return ((size_t)2 * gmax * (sizeof(R) + sizeof(int) + LU_NB * sizeof(C)) + 256) * ne;
}

template <typename C, int QPR>
__global__ __launch_bounds__(COOP_THREADS) void k_panel_coop(int64_t n, int k, int nbc, int ne, int G, int gmax,
                                                              C* __restrict__ LUall, int* __restrict__ ipiv_all,
                                                              int* __restrict__ perm_all, int* __restrict__ info_all,
                                                              int* __restrict__ bar, char* __restrict__ work) {
  using R = typename real_of<C>::type;
  constexpr int CPT = LU_NB / QPR;
  constexpr int RPW = COOP_THREADS / QPR;
  const int node = blockIdx.x % ne;
  const int g = blockIdx.x / ne;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = tid / QPR, h = tid % QPR;
  const int64_t m = n - k;
  const int64_t rloc = (int64_t)g * RPW + lr;
  const bool valid = rloc < m;
  const int64_t grow = k + rloc;  // position of this row when the panel starts
  C* __restrict__ LU = LUall + (int64_t)node * n * n;
  const PanelWork<C> pw = panel_work<C>(work, node, gmax);

  __shared__ R s_wv[COOP_THREADS / 64];
  __shared__ int s_wi[COOP_THREADS / 64];
  __shared__ R s_cv;
  __shared__ int s_ci;
  __shared__ R s_pv;
  __shared__ int s_pi, s_pw;
  __shared__ C prow[LU_NB];
  __shared__ int s_piv[LU_NB];
  __shared__ int s_zero;
  __shared__ int s_timeout;
  __shared__ int mv_row[2 * LU_NB], mv_pos[2 * LU_NB], s_nmv;
  __shared__ int s_ipiv[LU_NB];
  __shared__ int s_permv[2 * LU_NB];

  C v[CPT];
#pragma unroll
  for (int c = 0; c < CPT; ++c) {
    const int col = h * CPT + c;
    v[c] = (valid && col < nbc) ? LU[grow * n + k + col] : C(R(0), R(0));
  }
  bool active = valid;
  if (tid == 0) {
    s_zero = 0;
    s_timeout = 0;
  }

  for (int j = 0; j < nbc; ++j) {
    const int par = j & 1;
    const int hj = j / CPT, jj = j % CPT;
    // ---- 1. candidate of this workgroup
    R a = R(-1);
    int ai = INT_MAX;
    if (active && h == hj) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (c == jj) a = abs1(v[c]);
      if (!(a >= R(0))) a = R(0);  // a non-finite entry is caught by the pivot test
      ai = (int)grow;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const R ov = __shfl_xor(a, off);
      const int oi = __shfl_xor(ai, off);
      argmax_merge(a, ai, ov, oi);
    }
    if (lane == 0) {
      s_wv[wave] = a;
      s_wi[wave] = ai;
    }
    __syncthreads();
    if (tid == 0) {
      R bv = s_wv[0];
      int bi = s_wi[0];
      for (int w = 1; w < COOP_THREADS / 64; ++w) argmax_merge(bv, bi, s_wv[w], s_wi[w]);
      s_cv = bv;
      s_ci = bi;
      pw.cv[par * gmax + g] = bv;
      pw.ci[par * gmax + g] = bi;
    }
    __syncthreads();
    if (valid && (int)grow == s_ci) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) pw.cr[((int64_t)par * gmax + g) * LU_NB + h * CPT + c] = v[c];
      __threadfence();
    }
    __syncthreads();
    // ---- 2. barrier across the node's workgroups
    if (tid == 0) {
      __threadfence();
      atomicAdd(&bar[node], 1);
      const int target = (j + 1) * G;
      int spin = 0;
      // bounded wait (a few ms): a workgroup that never arrives ends the panel with an
      // error instead of a hang; after one timeout no later column waits
      while (!s_timeout &&
             __hip_atomic_load(&bar[node], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spin > (1 << 18)) s_timeout = 1;
      }
      __threadfence();
    }
    __syncthreads();
    // ---- 3. the node's pivot
    if (wave == 0) {
      R bv = R(-1);
      int bi = INT_MAX, bw = -1;
      for (int t = lane; t < G; t += 64) {
        const R cv = __hip_atomic_load(&pw.cv[par * gmax + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int cix = __hip_atomic_load(&pw.ci[par * gmax + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (cv > bv || (cv == bv && cix < bi)) {
          bv = cv;
          bi = cix;
          bw = t;
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const R ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        const int ow = __shfl_xor(bw, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
          bw = ow;
        }
      }
      if (lane == 0) {
        s_pv = bv;
        s_pi = bi;
        s_pw = bw < 0 ? 0 : bw;
      }
    }
    __syncthreads();
    if (tid < LU_NB) prow[tid] = pw.cr[((int64_t)par * gmax + s_pw) * LU_NB + tid];
    if (tid == 0) s_piv[j] = s_pi;
    __syncthreads();
    // ---- 4. scale and update
    const C piv = prow[j];
    const bool ok = s_pv > R(0) && abs1(piv) > R(0) && isfinite(piv.re) && isfinite(piv.im);
    if (tid == 0 && !ok && s_zero == 0) s_zero = k + j + 1;
    const C inv = ok ? cdiv(C(R(1), R(0)), piv) : C(R(0), R(0));
    const bool is_piv = active && (int)grow == s_pi;
    if (is_piv) active = false;
    C lj(R(0), R(0));
    if (active && h == hj) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        if (c == jj) lj = v[c] * inv;
    }
    // every lane of the row takes the multiplier from the lane that owns column j
    const int src = (lane & ~(QPR - 1)) | hj;
    lj.re = __shfl(lj.re, src);
    lj.im = __shfl(lj.im, src);
    if (active) {
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int col = h * CPT + c;
        if (col == j) v[c] = lj;
        else if (col > j && col < nbc) v[c] = v[c] - lj * prow[col];
      }
    }
  }

  // ---- replay the interchanges on the list of moved rows (wave 0, lane-parallel)
  if (wave == 0) {
    int er0 = -1, ep0 = -1, er1 = -1, ep1 = -1;  // entries lane and lane + 64: (row, position)
    int cnt = 0;
    auto find = [&](const int* key0, const int* key1, int want, int& slot) -> bool {
      const unsigned long long b0 = __ballot(*key0 == want);
      const unsigned long long b1 = __ballot(*key1 == want);
      if (b0) {
        slot = __ffsll((long long)b0) - 1;
        return true;
      }
      if (b1) {
        slot = 64 + __ffsll((long long)b1) - 1;
        return true;
      }
      return false;
    };
    auto read = [&](int slot, bool pos) -> int {
      const int l = slot & 63;
      const int v0 = __shfl(pos ? ep0 : er0, l), v1 = __shfl(pos ? ep1 : er1, l);
      return slot < 64 ? v0 : v1;
    };
    auto write = [&](int slot, int row, int pos) {
      if (lane == (slot & 63)) {
        if (slot < 64) {
          er0 = row;
          ep0 = pos;
        } else {
          er1 = row;
          ep1 = pos;
        }
      }
    };
    for (int j = 0; j < nbc; ++j) {
      const int target = k + j;
      int p = s_piv[j];
      if (p < k || (int64_t)p >= n) p = target;  // only after a failed barrier (info is set)
      int sp, st;
      const bool hp = find(&er0, &er1, p, sp);   // p's current position
      const int pos_p = hp ? read(sp, true) : p;
      const bool ht = find(&ep0, &ep1, target, st);  // row now at position target
      const int row_t = ht ? read(st, false) : target;
      if (lane == 0) s_ipiv[j] = pos_p;
      if (pos_p != target) {
        if (hp) write(sp, p, target);
        else {
          write(cnt, p, target);
          ++cnt;
        }
        if (ht) write(st, row_t, pos_p);
        else {
          write(cnt, row_t, pos_p);
          ++cnt;
        }
      }
    }
    if (lane < cnt) {
      mv_row[lane] = er0;
      mv_pos[lane] = ep0;
    }
    if (lane + 64 < cnt) {
      mv_row[lane + 64] = er1;
      mv_pos[lane + 64] = ep1;
    }
    if (lane == 0) s_nmv = cnt;
  }
  __syncthreads();
  // ---- every row to its final position (the rows were all read before the first barrier)
  if (valid) {
    int64_t fp = grow;
    for (int e = 0; e < s_nmv; ++e)
      if (mv_row[e] == (int)grow) fp = mv_pos[e];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int col = h * CPT + c;
      if (col < nbc) LU[fp * n + k + col] = v[c];
    }
  }
  if (g == 0) {
    int* perm = perm_all + (int64_t)node * n;
    const int nm = s_nmv;
    if (tid < nm) s_permv[tid] = perm[mv_row[tid]];
    __syncthreads();
    if (tid < nm) perm[mv_pos[tid]] = s_permv[tid];
    if (tid < nbc) ipiv_all[(int64_t)node * n + k + tid] = s_ipiv[tid];
    if (tid == 0) {
      const int z = s_timeout ? (k + 1) : s_zero;
      if (z != 0 && info_all[node] == 0) info_all[node] = z;
    }
  } else if (tid == 0 && s_timeout && info_all[node] == 0) {
    info_all[node] = k + 1;
  }
}

template <typename C, int QPR>
static bool launch_panel_coop(hipStream_t s, int64_t n, int k, int nbc, int ne, C* LU, int* ipiv, int* perm,
                              int* info, int* bar, char* work) {
  constexpr int RPW = COOP_THREADS / QPR;
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return false;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_panel_coop<C, QPR>, COOP_THREADS, 0) != hipSuccess)
    return false;
  int G = (int)((n - k + RPW - 1) / RPW);
  const int gmax = (int)((n + RPW - 1) / RPW);
  if ((int64_t)G * ne > (int64_t)ncu * per_cu) return false;
  int64_t n_ = n;
  int k_ = k, nbc_ = nbc, ne_ = ne, G_ = G, gmax_ = gmax;
  void* args[] = {&n_, &k_, &nbc_, &ne_, &G_, &gmax_, &LU, &ipiv, &perm, &info, &bar, &work};
  return hipLaunchCooperativeKernel((const void*)k_panel_coop<C, QPR>, dim3(G * ne), dim3(COOP_THREADS), args, 0,
                                    s) == hipSuccess;
}

template <typename C>
static int launch_panel(hipStream_t s, int64_t n, int k, int nbc, int ne, C* LU, int* ipiv, int* perm, int* info) {
  const int64_t rows = n;
  constexpr bool dbl = sizeof(C) == 16;
  dim3 grid(ne), block(PANEL_THREADS);
  if (rows <= 1024) {
    if (dbl) hipLaunchKernelGGL((k_panel<C, 4, 1>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
    else hipLaunchKernelGGL((k_panel<C, 8, 1>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
  } else if (rows <= 2048) {
    if (dbl) hipLaunchKernelGGL((k_panel<C, 4, 2>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
    else hipLaunchKernelGGL((k_panel<C, 8, 2>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
  } else if (rows <= 4096) {
    if (dbl) hipLaunchKernelGGL((k_panel<C, 4, 4>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
    else hipLaunchKernelGGL((k_panel<C, 8, 4>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
  } else if (rows <= 8192) {
    if (dbl) hipLaunchKernelGGL((k_panel<C, 2, 8>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
    else hipLaunchKernelGGL((k_panel<C, 4, 8>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
  } else {
    if (dbl) hipLaunchKernelGGL((k_panel<C, 1, 16>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
    else hipLaunchKernelGGL((k_panel<C, 2, 16>), grid, block, 0, s, n, k, nbc, LU, ipiv, perm, info);
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename C>
constexpr int panel_qpr() {
  return sizeof(C) == 16 ? 4 : 2;
}

__global__ void k_zero_ints(int count, int* __restrict__ p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

template <typename C>
size_t lu_work_bytes(int64_t n, int ne) {
  const int npanel = (int)((n + LU_NB - 1) / LU_NB);
  return panel_work_bytes<C>(n, ne, COOP_THREADS / panel_qpr<C>()) + (size_t)npanel * ne * sizeof(int) + 256;
}

template <typename C>
int lu_factor(hipStream_t s, int64_t n, int ne, C* LU, int* ipiv, int* perm, int* perm_inv, int* info,
              C* Dinv, void* work) {
  if (n > MAX_N) return -2;
  using R = typename real_of<C>::type;
  constexpr int QPR = panel_qpr<C>();
  const int npanel = (int)((n + LU_NB - 1) / LU_NB);
  // barrier counters (one per panel and node), then the candidate exchange areas
  int* bars = reinterpret_cast<int*>(work);
  char* pwork = reinterpret_cast<char*>(work) + (((size_t)npanel * ne * sizeof(int) + 255) / 256) * 256;
  hipLaunchKernelGGL(k_zero_ints, dim3((npanel * ne + 255) / 256), dim3(256), 0, s, npanel * ne, bars);
  for (int64_t k = 0; k < n; k += LU_NB) {
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    int tok = prof_begin(s);
    const bool coop = coop_allowed() && launch_panel_coop<C, QPR>(s, n, (int)k, nbc, ne, LU, ipiv, perm, info,
                                                                 bars + (k / LU_NB) * ne, pwork);
    if (!coop && launch_panel<C>(s, n, (int)k, nbc, ne, LU, ipiv, perm, info)) return -2;
    // panel flops: (n-k) nbc^2 / 2 complex multiply-adds per node
    prof_end(tok, s, K_LU_PANEL, 8.0 * 0.5 * (double)(n - k) * nbc * nbc * ne, 2.0 * sizeof(C) * (n - k) * nbc * ne);
    hipLaunchKernelGGL((k_invert_diag<C>), dim3(1, ne), dim3(256), 0, s, n, (int)k, 1, LU, Dinv);
    hipLaunchKernelGGL((k_laswp<C>), dim3((unsigned)((n + 255) / 256), ne), dim3(256), 0, s, n, (int)k, nbc, LU, ipiv);
    const int64_t rest = n - k - nbc;
    if (rest > 0) {
      const int64_t nblk_total = (n + LU_NB - 1) / LU_NB;
      // U12 = L11^-1 A12 in place (one tile row: every workgroup owns whole columns)
      GemmArgs g{};
      g.M = nbc; g.N = (int)rest; g.K = nbc;
      g.A = Dinv + (k / LU_NB) * 2 * LU_NB * LU_NB; g.lda = LU_NB; g.a_bs = nblk_total * 2 * LU_NB * LU_NB;
      g.B = LU + k * n + k + nbc; g.ldb = n; g.b_bs = n * n;
      g.C = LU + k * n + k + nbc; g.ldc = n; g.c_bs = n * n;
      g.alpha = 1.0; g.beta = 0.0;
      if (gemm<R, true>(s, false, false, g, ne)) return -2;
      // A22 -= L21 U12
      GemmArgs t{};
      t.M = (int)rest; t.N = (int)rest; t.K = nbc;
      t.A = LU + (k + nbc) * n + k; t.lda = n; t.a_bs = n * n;
      t.B = LU + k * n + k + nbc; t.ldb = n; t.b_bs = n * n;
      t.C = LU + (k + nbc) * n + k + nbc; t.ldc = n; t.c_bs = n * n;
      t.alpha = -1.0; t.beta = 1.0;
      t.tag = 1;
      tok = prof_begin(s);
      if (gemm<R, true>(s, false, false, t, ne)) return -2;
      prof_end(tok, s, K_LU_GEMM, 8.0 * (double)rest * rest * nbc * ne,
               (double)sizeof(C) * ne * (2.0 * rest * rest + 2.0 * rest * nbc));
    }
  }
  hipLaunchKernelGGL(k_perm_inverse, dim3((unsigned)((n + 255) / 256), ne), dim3(256), 0, s, n, ne, perm, perm_inv);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int expand_full<double>(hipStream_t, char, int64_t, const double*, int64_t, double*);
template int expand_full<c64>(hipStream_t, char, int64_t, const c64*, int64_t, c64*);
template int shift_form<double, c32>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, c32*, int*);
template int shift_form<double, c64>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, c64*, int*);
template int shift_form<c64, c32>(hipStream_t, int64_t, const c64*, int64_t, const c64*, int64_t, const c64*, int, c32*, int*);
template int shift_form<c64, c64>(hipStream_t, int64_t, const c64*, int64_t, const c64*, int64_t, const c64*, int, c64*, int*);
template int lu_factor<c32>(hipStream_t, int64_t, int, c32*, int*, int*, int*, int*, c32*, void*);
template int lu_factor<c64>(hipStream_t, int64_t, int, c64*, int*, int*, int*, int*, c64*, void*);
template size_t lu_work_bytes<c32>(int64_t, int);
template size_t lu_work_bytes<c64>(int64_t, int);

}  // namespace mf
