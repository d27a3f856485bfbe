// Sparse (CSR) kernels of the FEAST path without factorization (IFEAST).
//
//  * csr_full: the caller's CSR (0- or 1-based, full storage or one triangle of a
//    symmetric matrix) becomes a 0-based full-storage CSR with sorted columns, values
//    in FP64 (outer products A Q, B Q) and in the BiCGSTAB precision.
//  * spmm_rm: Y = M X for a row-major FP64 block X (the FP64 side of the iteration).
//  * bicgstab_batched: BiCGSTAB (van der Vorst 1992) on all shifted systems
//    (z_j B - A) x = b at once: one column per (node j, right-hand side q).  Every
//    node shares the same right-hand side block b (n x m0, real), so the shadow residual
//    r_hat = r_0 = b is stored once.  Columns c = j * m0 + q (ncol = nodes * m0) are
//    grouped in tiles of 64; a vector is stored tile-major, element (i, c) at
//    ((c / 64) * n + i) * 64 + c % 64, so one tile is a contiguous n x 64 block
//    (a wave reads 512 contiguous bytes per row, consecutive rows are adjacent, and
//    the few tiles still active late in the solve spread over every memory channel).
//    Per-column inner products are reduced in FP64, deterministically: one partial
//    per column and 256-row block, then a fixed-order sum by one workgroup per tile.
//    Converged columns stop: a device-side list of the tiles that still hold an
//    active column drives every kernel.
#include <algorithm>
#include <vector>

#include "kernels.hpp"

namespace mf {

// ===========================================================================
// CSR to full, 0-based, sorted
// ===========================================================================
namespace {

constexpr int SCAN_B = 1024;

// mode 0: full storage; 1: lower triangle given; 2: upper triangle given
__device__ inline bool csr_keep(int mode, int64_t i, int64_t j) {
  return mode == 0 || (mode == 1 && j <= i) || (mode == 2 && j >= i);
}

__global__ void k_csr_count(int64_t n, const int32_t* __restrict__ ia, const int32_t* __restrict__ ja, int base,
                            int mode, int64_t nnz_in, int* __restrict__ cnt, int* __restrict__ flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = (int64_t)ia[i] - base, e = (int64_t)ia[i + 1] - base;
  if (b < 0 || e < b || e > nnz_in) {
    atomicOr(flag, 1);
    return;
  }
  for (int64_t k = b; k < e; ++k) {
    const int64_t j = (int64_t)ja[k] - base;
    if (j < 0 || j >= n) {
      atomicOr(flag, 2);
      continue;
    }
    if (!csr_keep(mode, i, j)) continue;
    atomicAdd(&cnt[i], 1);
    if (mode != 0 && j != i) atomicAdd(&cnt[j], 1);
  }
}

__global__ void k_scan_local(int64_t n, const int* __restrict__ cnt, int64_t* __restrict__ bsum) {
  __shared__ int64_t red[SCAN_B];
  const int64_t i = blockIdx.x * (int64_t)SCAN_B + threadIdx.x;
  red[threadIdx.x] = (i < n) ? cnt[i] : 0;
  __syncthreads();
  for (int off = SCAN_B / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// one workgroup: exclusive scan of nb block sums in place
__global__ void k_scan_top(int64_t nb, int64_t* __restrict__ bsum) {
  __shared__ int64_t part[SCAN_B];
  const int64_t per = (nb + SCAN_B - 1) / SCAN_B;
  const int64_t b0 = threadIdx.x * per, b1 = (b0 + per < nb) ? b0 + per : nb;
  int64_t s = 0;
  for (int64_t b = b0; b < b1; ++b) s += bsum[b];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < SCAN_B; ++t) {
      const int64_t v = part[t];
      part[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = part[threadIdx.x];
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t v = bsum[b];
    bsum[b] = run;
    run += v;
  }
}

// rp[i + 1] = inclusive prefix of cnt; cursor[i] = rp[i]
__global__ void k_scan_final(int64_t n, const int* __restrict__ cnt, const int64_t* __restrict__ boff,
                             int64_t* __restrict__ rp, int64_t* __restrict__ cursor) {
  __shared__ int64_t buf[2][SCAN_B];
  const int64_t i = blockIdx.x * (int64_t)SCAN_B + threadIdx.x;
  const int64_t v = (i < n) ? cnt[i] : 0;
  buf[0][threadIdx.x] = v;
  __syncthreads();
  int src = 0;
  for (int off = 1; off < SCAN_B; off <<= 1) {
    const int64_t a = buf[src][threadIdx.x];
    const int64_t b = ((int)threadIdx.x >= off) ? buf[src][threadIdx.x - off] : 0;
    buf[src ^ 1][threadIdx.x] = a + b;
    src ^= 1;
    __syncthreads();
  }
  const int64_t incl = boff[blockIdx.x] + buf[src][threadIdx.x];
  if (i < n) {
    rp[i + 1] = incl;
    cursor[i] = incl - v;
  }
  if (i == 0) rp[0] = 0;
}

__global__ void k_csr_fill(int64_t n, const int32_t* __restrict__ ia, const int32_t* __restrict__ ja,
                           const double* __restrict__ a, int base, int mode, int64_t* __restrict__ cursor,
                           int32_t* __restrict__ ci, double* __restrict__ vd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = (int64_t)ia[i] - base, e = (int64_t)ia[i + 1] - base;
  for (int64_t k = b; k < e; ++k) {
    const int64_t j = (int64_t)ja[k] - base;
    if (!csr_keep(mode, i, j)) continue;
    const double v = a[k];
    int64_t pos = atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[i]), 1ull);
    ci[pos] = (int32_t)j;
    vd[pos] = v;
    if (mode != 0 && j != i) {
      pos = atomicAdd(reinterpret_cast<unsigned long long*>(&cursor[j]), 1ull);
      ci[pos] = (int32_t)i;
      vd[pos] = v;
    }
  }
}

// insertion sort of each row by (column, value bits): a fixed order of the row's
// products whatever order the atomics above placed them in
template <typename R>
__global__ void k_csr_sort(int64_t n, const int64_t* __restrict__ rp, int32_t* __restrict__ ci,
                           double* __restrict__ vd, R* __restrict__ vr, int32_t* __restrict__ rp32) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i > n) return;
  rp32[i] = (int32_t)rp[i];
  if (i == n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  for (int64_t k = b + 1; k < e; ++k) {
    const int32_t c = ci[k];
    const double v = vd[k];
    int64_t q = k - 1;
    while (q >= b && (ci[q] > c || (ci[q] == c && __double_as_longlong(vd[q]) > __double_as_longlong(v)))) {
      ci[q + 1] = ci[q];
      vd[q + 1] = vd[q];
      --q;
    }
    ci[q + 1] = c;
    vd[q + 1] = v;
  }
  for (int64_t k = b; k < e; ++k) vr[k] = (R)vd[k];
}

}  // namespace

void* CsrWork::get(int k, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (cap[k] < bytes) {
    if (buf[k]) (void)hipFree(buf[k]);
    buf[k] = nullptr;
    cap[k] = 0;
    if (hipMalloc(&buf[k], bytes) != hipSuccess) return nullptr;
    cap[k] = bytes;
  }
  return buf[k];
}

void CsrWork::release() {
  for (int k = 0; k < NBUF; ++k) {
    if (buf[k]) (void)hipFree(buf[k]);
    buf[k] = nullptr;
    cap[k] = 0;
  }
}

template <typename R>
int csr_full(hipStream_t s, int64_t n, const double* a, const int32_t* ia, const int32_t* ja, int base, char uplo,
             CsrWork& w, CsrMat<R>& out, int* err) {
  *err = 0;
  const int mode = (uplo == 'L' || uplo == 'l') ? 1 : (uplo == 'U' || uplo == 'u') ? 2 : 0;
  int32_t ends[2] = {0, 0};
  MF_HIP_CHECK(hipMemcpyAsync(&ends[0], ia, 4, hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipMemcpyAsync(&ends[1], ia + n, 4, hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  if (ends[0] != base) {
    *err = 1;
    return 0;
  }
  const int64_t nnz_in = (int64_t)ends[1] - base;
  if (nnz_in < 0) {
    *err = 1;
    return 0;
  }
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  int* cnt = (int*)w.get(0, (size_t)n * 4);
  int64_t* bsum = (int64_t*)w.get(1, (size_t)nb * 8 + 64);
  int64_t* rp = (int64_t*)w.get(2, (size_t)(n + 1) * 8);
  int64_t* cursor = (int64_t*)w.get(3, (size_t)n * 8);
  int* flag = (int*)w.get(4, 64);
  if (!cnt || !bsum || !rp || !cursor || !flag) return -2;
  MF_HIP_CHECK(hipMemsetAsync(cnt, 0, (size_t)n * 4, s));
  MF_HIP_CHECK(hipMemsetAsync(flag, 0, 4, s));
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_csr_count, dim3(g), dim3(256), 0, s, n, ia, ja, base, mode, nnz_in, cnt, flag);
  int hflag = 0;
  MF_HIP_CHECK(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  if (hflag != 0) {
    *err = (hflag & 1) ? 1 : 2;
    return 0;
  }
  hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(SCAN_B), 0, s, n, cnt, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(SCAN_B), 0, s, nb, bsum);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(SCAN_B), 0, s, n, cnt, bsum, rp, cursor);
  int64_t nnz = 0;
  MF_HIP_CHECK(hipMemcpyAsync(&nnz, rp + n, 8, hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  if (nnz > (int64_t)INT32_MAX) {
    *err = 3;
    return 0;
  }
  out.n = n;
  out.nnz = nnz;
  out.rp = (int32_t*)w.get(5, (size_t)(n + 1) * 4);
  out.ci = (int32_t*)w.get(6, (size_t)nnz * 4 + 16);
  out.vd = (double*)w.get(7, (size_t)nnz * 8 + 16);
  out.vr = (R*)w.get(8, (size_t)nnz * sizeof(R) + 16);
  if (!out.rp || !out.ci || !out.vd || !out.vr) return -2;
  hipLaunchKernelGGL(k_csr_fill, dim3(g), dim3(256), 0, s, n, ia, ja, a, base, mode, cursor, out.ci, out.vd);
  hipLaunchKernelGGL((k_csr_sort<R>), dim3((unsigned)((n + 256) / 256)), dim3(256), 0, s, n, rp, out.ci, out.vd,
                     out.vr, out.rp);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ===========================================================================
// FP64 sparse times row-major block: Y = M X  (n x m, leading dimensions ldx, ldy)
// ===========================================================================
namespace {
__global__ void k_spmm_rm(int64_t n, int m, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                          const double* __restrict__ val, const double* __restrict__ X, int64_t ldx,
                          double* __restrict__ Y, int64_t ldy) {
  // 64 columns x 4 rows per workgroup; rows on grid x
  const int c = blockIdx.y * 64 + (threadIdx.x & 63);
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n || c >= m) return;
  double acc = 0.0;
  const int kb = rp[i], ke = rp[i + 1];
  for (int k = kb; k < ke; ++k) acc += val[k] * X[(int64_t)ci[k] * ldx + c];
  Y[i * ldy + c] = acc;
}
}  // namespace

int spmm_rm(hipStream_t s, const CsrMat<float>& M, int m, const double* X, int64_t ldx, double* Y, int64_t ldy) {
  dim3 grid((unsigned)((M.n + 3) / 4), (unsigned)((m + 63) / 64));
  hipLaunchKernelGGL(k_spmm_rm, grid, dim3(256), 0, s, M.n, m, M.rp, M.ci, M.vd, X, ldx, Y, ldy);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}
int spmm_rm(hipStream_t s, const CsrMat<double>& M, int m, const double* X, int64_t ldx, double* Y, int64_t ldy) {
  dim3 grid((unsigned)((M.n + 3) / 4), (unsigned)((m + 63) / 64));
  hipLaunchKernelGGL(k_spmm_rm, grid, dim3(256), 0, s, M.n, m, M.rp, M.ci, M.vd, X, ldx, Y, ldy);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ===========================================================================
// Batched BiCGSTAB
// ===========================================================================
// One iteration is three sweeps over the vectors plus three per-column scalar steps:
//   A  v = (z B - A) p,                       partial r_hat^H v
//      alpha = rho / r_hat^H v
//   B  t = (z B - A) s with s = r - alpha v formed on the fly (s is never stored),
//      partials r_hat^H s, r_hat^H t, t^H s, t^H t, s^H s
//      half-step test on ||s||; omega = t^H s / t^H t;
//      rho' = r_hat^H r' = r_hat^H s - omega r_hat^H t, beta = (rho' / rho)(alpha / omega)
//   C  x += alpha p + omega s, r' = s - omega t, p' = r' + beta (p - omega v),  ||r'||^2
//      final test on ||r'||
// rho' is the textbook r_hat^H r' written through the two inner products of B (the
// same quantity; it only lets the p update join the x and r updates in one sweep).
// Every sweep reads its own rows plus, in A and B, the sparse neighbours (through the
// caches); the per-iteration HBM traffic is 13 vector passes (A 2, B 3, C 8).
namespace {

constexpr int BI_TILE = 64;                // columns per tile: one lane per column
constexpr int BI_WAVES = 4;                // waves per workgroup, each on its own rows
constexpr int BI_RB = 256;                 // rows per workgroup
constexpr int BI_RW = BI_RB / BI_WAVES;    // rows per wave
constexpr int BI_NQ = 8;                   // partial sums per column (largest sweep)
constexpr int BI_NSPLIT = 32;              // first-stage groups of row blocks

enum { ST_ACTIVE = 0, ST_HALF = 1, ST_DONE = 2, ST_LAST = 3 };

template <typename C>
struct BiK {
  using R = typename real_of<C>::type;
  int64_t n;
  int ncol, m0, nrb;
  const int32_t *rp, *ci;
  const R* va;
  const int32_t *rpb, *cib;  // B (rpb == nullptr: identity)
  const R* vb;
  const c64* zn;  // shift of each node in this batch
  const R* bh;    // right-hand side b = shadow residual, n x m0 real
  C *x, *r, *p, *v, *t;  // tile-major
  BiCol* col;
  const int* tiles;
  const int* ntile;  // number of valid entries of tiles (device)
  double* part;      // [quantity][row block][column], ncol rounded up to whole tiles
  double* part2;     // [quantity][split][column]: sums over groups of row blocks
  int ldp;           // that rounded column count
  int nsplit;        // number of row-block groups
};

// sum the per-lane partials of the 4 waves and store them as one partial per column
template <int NQ>
__device__ inline void bi_store_partials(const double (&acc)[NQ], double* part, int nrb, int ncol, int c) {
  __shared__ double red[NQ][BI_WAVES][BI_TILE];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][w][lane] = acc[q];
  __syncthreads();
  if (w == 0 && c >= 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double v = red[q][0][lane] + red[q][1][lane] + red[q][2][lane] + red[q][3][lane];
      part[((int64_t)q * nrb + blockIdx.x) * ncol + c] = v;
    }
  }
}

// the same, reusing a caller's LDS block (at least NQ * 2 KB) that other code of the
// kernel used before: the leading barrier ends those uses
template <int NQ>
__device__ inline void bi_store_partials_in(const double (&acc)[NQ], double* part, int nrb, int ncol, int c,
                                            double* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[(q * BI_WAVES + w) * BI_TILE + lane] = acc[q];
  __syncthreads();
  if (w == 0 && c >= 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double v = red[(q * BI_WAVES + 0) * BI_TILE + lane] + red[(q * BI_WAVES + 1) * BI_TILE + lane] +
                       red[(q * BI_WAVES + 2) * BI_TILE + lane] + red[(q * BI_WAVES + 3) * BI_TILE + lane];
      part[((int64_t)q * nrb + blockIdx.x) * ncol + c] = v;
    }
  }
}

// rows of this wave
struct RowRange {
  int64_t r0, r1;
};
__device__ inline RowRange bi_rows(int64_t n) {
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
  return {r0, (r0 + BI_RW < n) ? r0 + BI_RW : n};
}

// A's rows of one wave staged in LDS (row pointers relative to the first entry, column
// indices, values), so that a row's gathers wait only for LDS and not for the chain of
// global loads rp -> ci -> operand.  Waves whose rows hold more than BI_CAP entries read
// A from global memory as before.
constexpr int BI_CAP = 512;
template <typename R>
struct BiStage {
  int rp[BI_RW + 1];
  int ci[BI_CAP];
  R va[BI_CAP];
};
template <typename R, int NQ>
constexpr size_t bi_lds_bytes() {
  return (BI_WAVES * sizeof(BiStage<R>) > (size_t)NQ * BI_WAVES * BI_TILE * sizeof(double))
             ? BI_WAVES * sizeof(BiStage<R>)
             : (size_t)NQ * BI_WAVES * BI_TILE * sizeof(double);
}
template <typename R>
__device__ inline bool bi_stage_rows(BiStage<R>& S, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                                     const R* __restrict__ va, int64_t r0, int64_t r1, int lane) {
  if (r1 <= r0) return false;
  const int kb0 = rp[r0], ke1 = rp[r1];
  if (ke1 - kb0 > BI_CAP) return false;
  const int nr = (int)(r1 - r0);
  for (int l = lane; l <= nr; l += 64) S.rp[l] = rp[r0 + l] - kb0;
  for (int k = lane; k < ke1 - kb0; k += 64) {
    S.ci[k] = ci[kb0 + k];
    S.va[k] = va[kb0 + k];
  }
  return true;
}

// sum_k M(i, k) in(k) over one sparse row, eight entries in flight at a time; `get`
// returns the operand of column c at row k
template <typename C, typename R, typename Get>
__device__ inline C bi_row_dot(const int32_t* __restrict__ ci, const R* __restrict__ va, int kb, int ke, Get get) {
  C acc(R(0), R(0));
  for (int k0 = kb; k0 < ke; k0 += 8) {
    C xv[8];
    R av[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (k0 + u < ke) {
        av[u] = va[k0 + u];
        xv[u] = get((int64_t)ci[k0 + u]);
      } else {
        av[u] = R(0);
        xv[u] = C(R(0), R(0));
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc.re += av[u] * xv[u].re;
      acc.im += av[u] * xv[u].im;
    }
  }
  return acc;
}

// x = 0, r = p = b; partial b^T b
template <typename C>
__global__ __launch_bounds__(256) void k_bi_init(BiK<C> a) {
  using R = typename real_of<C>::type;
  const int lane = threadIdx.x & 63;
  const int tile = a.tiles[blockIdx.y];
  const int c = tile * BI_TILE + lane;
  const bool in = c < a.ncol;
  const int q = in ? c % a.m0 : 0;
  double acc[1] = {0.0};
  const RowRange rr = bi_rows(a.n);
  const int64_t tb = (int64_t)tile * a.n * BI_TILE + lane;
  if (in) {
    for (int64_t i = rr.r0; i < rr.r1; ++i) {
      const R b = a.bh[i * a.m0 + q];
      const int64_t o = tb + i * BI_TILE;
      a.r[o] = C(b, R(0));
      a.p[o] = C(b, R(0));
      a.x[o] = C(R(0), R(0));
      acc[0] += (double)b * (double)b;
    }
  }
  bi_store_partials<1>(acc, a.part, a.nrb, a.ldp, in ? c : -1);
}

// sweep A: v = z_j (B p) - A p; partial r_hat^H v
template <typename C>
__global__ __launch_bounds__(256) void k_bi_sweep_a(BiK<C> a) {
  using R = typename real_of<C>::type;
  if ((int)blockIdx.y >= *a.ntile) return;
  const int lane = threadIdx.x & 63;
  const int tile = a.tiles[blockIdx.y];
  const int c = tile * BI_TILE + lane;
  const bool act = c < a.ncol && a.col[c].state == ST_ACTIVE;
  C z(R(0), R(0));
  int q = 0;
  if (act) {
    z = convert<C, c64>(a.zn[c / a.m0]);
    q = c % a.m0;
  }
  double acc[2] = {0.0, 0.0};
  const RowRange rr = bi_rows(a.n);
  const int64_t tb = (int64_t)tile * a.n * BI_TILE + lane;
  const C* __restrict__ p = a.p + tb;
  C* __restrict__ v = a.v + tb;
  auto get = [&](int64_t k) { return p[k * BI_TILE]; };
  __shared__ __align__(16) char lds[bi_lds_bytes<R, 2>()];
  BiStage<R>& S = reinterpret_cast<BiStage<R>*>(lds)[threadIdx.x >> 6];
  const bool staged = bi_stage_rows<R>(S, a.rp, a.ci, a.va, rr.r0, rr.r1, lane);
  __syncthreads();
  auto row = [&](int64_t i, const C& sa) {
    const C sb = (a.rpb == nullptr) ? get(i) : bi_row_dot<C, R>(a.cib, a.vb, a.rpb[i], a.rpb[i + 1], get);
    const C o = z * sb - sa;
    v[i * BI_TILE] = o;
    const double h = (double)a.bh[i * a.m0 + q];
    acc[0] += h * (double)o.re;
    acc[1] += h * (double)o.im;
  };
  if (staged) {
    for (int64_t i = rr.r0; i < rr.r1; ++i) {
      const int kb = S.rp[i - rr.r0], ke = S.rp[i - rr.r0 + 1];
      if (!act) continue;
      row(i, bi_row_dot<C, R>(S.ci, S.va, kb, ke, get));
    }
  } else {
    for (int64_t i = rr.r0; i < rr.r1; ++i) {
      const int kb = a.rp[i], ke = a.rp[i + 1];
      if (!act) continue;
      row(i, bi_row_dot<C, R>(a.ci, a.va, kb, ke, get));
    }
  }
  bi_store_partials_in<2>(acc, a.part, a.nrb, a.ldp, act ? c : -1, reinterpret_cast<double*>(lds));
}

// sweep B: s = r - alpha v (not stored), t = z_j (B s) - A s;
// partials r_hat^H s (2), r_hat^H t (2), t^H s (2), t^H t, s^H s
template <typename C>
__global__ __launch_bounds__(256) void k_bi_sweep_b(BiK<C> a) {
  using R = typename real_of<C>::type;
  if ((int)blockIdx.y >= *a.ntile) return;
  const int lane = threadIdx.x & 63;
  const int tile = a.tiles[blockIdx.y];
  const int c = tile * BI_TILE + lane;
  const bool act = c < a.ncol && a.col[c].state == ST_ACTIVE;
  C z(R(0), R(0)), al(R(0), R(0));
  int q = 0;
  if (act) {
    z = convert<C, c64>(a.zn[c / a.m0]);
    al = convert<C, c64>(a.col[c].alpha);
    q = c % a.m0;
  }
  double acc[BI_NQ];
#pragma unroll
  for (int k = 0; k < BI_NQ; ++k) acc[k] = 0.0;
  const RowRange rr = bi_rows(a.n);
  const int64_t tb = (int64_t)tile * a.n * BI_TILE + lane;
  const C* __restrict__ r = a.r + tb;
  const C* __restrict__ v = a.v + tb;
  C* __restrict__ t = a.t + tb;
  auto get = [&](int64_t k) { return r[k * BI_TILE] - al * v[k * BI_TILE]; };
  __shared__ __align__(16) char lds[bi_lds_bytes<R, BI_NQ>()];
  BiStage<R>& S = reinterpret_cast<BiStage<R>*>(lds)[threadIdx.x >> 6];
  const bool staged = bi_stage_rows<R>(S, a.rp, a.ci, a.va, rr.r0, rr.r1, lane);
  __syncthreads();
  auto row = [&](int64_t i, const C& sa) {
    const C si = get(i);
    const C sb = (a.rpb == nullptr) ? si : bi_row_dot<C, R>(a.cib, a.vb, a.rpb[i], a.rpb[i + 1], get);
    const C o = z * sb - sa;
    t[i * BI_TILE] = o;
    const double h = (double)a.bh[i * a.m0 + q];
    const double sre = si.re, sim = si.im, tre = o.re, tim = o.im;
    acc[0] += h * sre;
    acc[1] += h * sim;
    acc[2] += h * tre;
    acc[3] += h * tim;
    acc[4] += tre * sre + tim * sim;  // conj(t) s
    acc[5] += tre * sim - tim * sre;
    acc[6] += tre * tre + tim * tim;
    acc[7] += sre * sre + sim * sim;
  };
  if (staged) {
    for (int64_t i = rr.r0; i < rr.r1; ++i) {
      const int kb = S.rp[i - rr.r0], ke = S.rp[i - rr.r0 + 1];
      if (!act) continue;
      row(i, bi_row_dot<C, R>(S.ci, S.va, kb, ke, get));
    }
  } else {
    for (int64_t i = rr.r0; i < rr.r1; ++i) {
      const int kb = a.rp[i], ke = a.rp[i + 1];
      if (!act) continue;
      row(i, bi_row_dot<C, R>(a.ci, a.va, kb, ke, get));
    }
  }
  bi_store_partials_in<BI_NQ>(acc, a.part, a.nrb, a.ldp, act ? c : -1, reinterpret_cast<double*>(lds));
}

// sweep C: x += alpha p + omega s, r' = s - omega t, p' = r' + beta (p - omega v);
// x += alpha p only for a column that converged at the half step; partial ||r'||^2
template <typename C>
__global__ __launch_bounds__(256) void k_bi_sweep_c(BiK<C> a) {
  if ((int)blockIdx.y >= *a.ntile) return;
  const int lane = threadIdx.x & 63;
  const int tile = a.tiles[blockIdx.y];
  const int c = tile * BI_TILE + lane;
  const int st = (c < a.ncol) ? a.col[c].state : ST_DONE;
  double acc[1] = {0.0};
  if (st != ST_DONE) {
    const C al = convert<C, c64>(a.col[c].alpha), om = convert<C, c64>(a.col[c].omega),
            be = convert<C, c64>(a.col[c].beta);
    const RowRange rr = bi_rows(a.n);
    const int64_t tb = (int64_t)tile * a.n * BI_TILE + lane;
    if (st == ST_HALF) {
      for (int64_t i = rr.r0; i < rr.r1; ++i) {
        const int64_t o = tb + i * BI_TILE;
        a.x[o] = a.x[o] + al * a.p[o];
      }
    } else {
#pragma unroll 2
      for (int64_t i = rr.r0; i < rr.r1; ++i) {
        const int64_t o = tb + i * BI_TILE;
        const C pv = a.p[o], vv = a.v[o], sv = a.r[o] - al * vv, tv = a.t[o];
        a.x[o] = a.x[o] + al * pv + om * sv;
        const C rv = sv - om * tv;
        a.r[o] = rv;
        a.p[o] = rv + be * (pv - om * vv);
        acc[0] += (double)rv.re * rv.re + (double)rv.im * rv.im;
      }
    }
  }
  bi_store_partials<1>(acc, a.part, a.nrb, a.ldp, (st == ST_ACTIVE || st == ST_LAST) ? c : -1);
}

// First stage of the column sums: workgroup (tile, split) adds the partials of row
// blocks split, split + nsplit, ... (lane = column, the 4 waves interleaved), in a
// fixed order.
template <int NQ>
__global__ __launch_bounds__(256) void k_bi_reduce(const int* __restrict__ tiles, const int* __restrict__ ntile,
                                                   const double* __restrict__ part, double* __restrict__ part2,
                                                   int nrb, int ldp, int nsplit) {
  __shared__ double red[NQ][BI_WAVES][BI_TILE];
  if ((int)blockIdx.x >= *ntile) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int c = tiles[blockIdx.x] * BI_TILE + lane;
  const int sp = blockIdx.y;
  double sum[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
#pragma unroll 4
  for (int b = sp + w * nsplit; b < nrb; b += BI_WAVES * nsplit) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) sum[q] += part[((int64_t)q * nrb + b) * ldp + c];
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) red[q][w][lane] = sum[q];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      part2[((int64_t)q * nsplit + sp) * ldp + c] = red[q][0][lane] + red[q][1][lane] + red[q][2][lane] + red[q][3][lane];
  }
}

// per-column scalar step after each sweep: one wave per listed tile adds the nsplit
// first-stage sums in a fixed order and updates its columns.
// MODE 0: init, 1: alpha, 2: half-step test, omega, rho', beta, 3: final test
template <typename C, int MODE>
__global__ __launch_bounds__(64) void k_bi_scalar(BiK<C> a, int it, int maxit, double tol2) {
  constexpr int NQ = MODE == 0 ? 1 : MODE == 1 ? 2 : MODE == 2 ? BI_NQ : 1;
  if ((int)blockIdx.x >= *a.ntile) return;
  const int c = a.tiles[blockIdx.x] * BI_TILE + (int)threadIdx.x;
  if (c >= a.ncol) return;
  double sum[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
#pragma unroll 8
  for (int sp = 0; sp < a.nsplit; ++sp) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) sum[q] += a.part2[((int64_t)q * a.nsplit + sp) * a.ldp + c];
  }
  BiCol& cs = a.col[c];
  if constexpr (MODE == 0) {
    cs.bn2 = sum[0];
    cs.rho = c64(sum[0], 0.0);
    cs.alpha = c64(1.0, 0.0);
    cs.omega = c64(1.0, 0.0);
    cs.beta = c64(0.0, 0.0);
    cs.its = 0;
    cs.state = sum[0] > 0.0 ? ST_ACTIVE : ST_DONE;
  } else if constexpr (MODE == 1) {
    if (cs.state != ST_ACTIVE) return;
    const c64 den(sum[0], sum[1]);
    if (den.re == 0.0 && den.im == 0.0) {
      cs.state = ST_DONE;  // breakdown: x stays as it is
      cs.its = it;
    } else {
      cs.alpha = cdiv(cs.rho, den);
    }
  } else if constexpr (MODE == 2) {
    if (cs.state != ST_ACTIVE) return;
    if (sum[7] <= tol2 * cs.bn2) {
      cs.state = ST_HALF;
      return;
    }
    const c64 om = sum[6] != 0.0 ? c64(sum[4] / sum[6], sum[5] / sum[6]) : c64(0.0, 0.0);
    const c64 rho_new = c64(sum[0], sum[1]) - om * c64(sum[2], sum[3]);
    cs.omega = om;
    if ((om.re == 0.0 && om.im == 0.0) || (rho_new.re == 0.0 && rho_new.im == 0.0)) {
      cs.state = ST_LAST;  // breakdown at the next step: finish this update, then stop
      cs.beta = c64(0.0, 0.0);
    } else {
      cs.beta = cdiv(rho_new, cs.rho) * cdiv(cs.alpha, om);
    }
    cs.rho = rho_new;
  } else {
    if (cs.state == ST_DONE) return;
    cs.its = it;
    if (cs.state == ST_HALF || cs.state == ST_LAST || sum[0] <= tol2 * cs.bn2 || it >= maxit) cs.state = ST_DONE;
  }
}

// list of 64-column tiles that still hold an active column (one workgroup)
__global__ void k_bi_compact(int ncol, const BiCol* __restrict__ col, int* __restrict__ tiles,
                             int* __restrict__ ntile) {
  __shared__ int scan[256];
  __shared__ int base;
  if (threadIdx.x == 0) base = 0;
  __syncthreads();
  const int nt = (ncol + BI_TILE - 1) / BI_TILE;
  for (int t0 = 0; t0 < nt; t0 += 256) {
    const int t = t0 + (int)threadIdx.x;
    int flag = 0;
    if (t < nt) {
      const int c1 = (t + 1) * BI_TILE < ncol ? (t + 1) * BI_TILE : ncol;
      for (int c = t * BI_TILE; c < c1 && !flag; ++c) flag = col[c].state == ST_ACTIVE;
    }
    scan[threadIdx.x] = flag;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const int add = (int)threadIdx.x >= off ? scan[threadIdx.x - off] : 0;
      __syncthreads();
      scan[threadIdx.x] += add;
      __syncthreads();
    }
    if (flag) tiles[base + scan[threadIdx.x] - 1] = t;
    __syncthreads();
    if (threadIdx.x == 255) base += scan[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) *ntile = base;
}

// iteration counts of every column, packed
__global__ void k_bi_its(int ncol, const BiCol* __restrict__ col, int* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncol) out[c] = col[c].its;
}

}  // namespace

template <typename C>
int bicgstab_batched(hipStream_t s, const BiSys<C>& sys, int maxit, double tol, std::vector<int>& its,
                     int* d_buf, int* h_buf) {
  BiK<C> a{};
  a.n = sys.n;
  a.ncol = sys.ncol;
  a.m0 = sys.m0;
  a.nrb = (int)((sys.n + BI_RB - 1) / BI_RB);
  a.rp = sys.A->rp;
  a.ci = sys.A->ci;
  a.va = sys.A->vr;
  a.rpb = sys.B ? sys.B->rp : nullptr;
  a.cib = sys.B ? sys.B->ci : nullptr;
  a.vb = sys.B ? sys.B->vr : nullptr;
  a.zn = sys.zn;
  a.bh = sys.bh;
  a.x = sys.x;
  a.r = sys.r;
  a.p = sys.p;
  a.v = sys.v;
  a.t = sys.t;
  a.col = sys.col;
  a.tiles = sys.tiles;
  a.ntile = d_buf;  // d_buf[0]: tile count; d_buf + 64: iteration counts
  a.part = sys.part;
  const int ntile_all = (sys.ncol + BI_TILE - 1) / BI_TILE;
  a.ldp = ntile_all * BI_TILE;
  a.nsplit = std::min(a.nrb, BI_NSPLIT);
  a.part2 = sys.part + (size_t)BI_NQ * a.nrb * a.ldp;
  std::vector<int> tl(ntile_all);
  for (int i = 0; i < ntile_all; ++i) tl[i] = i;
  MF_HIP_CHECK(hipMemcpyAsync(sys.tiles, tl.data(), ntile_all * sizeof(int), hipMemcpyHostToDevice, s));
  h_buf[0] = ntile_all;
  MF_HIP_CHECK(hipMemcpyAsync(d_buf, h_buf, sizeof(int), hipMemcpyHostToDevice, s));
  const unsigned gs = (unsigned)((sys.ncol + 255) / 256);
  const dim3 sb(64);
  // column sums of NQ quantities over the listed tiles (first stage)
  auto reduce = [&](int nq, int nt) {
    const dim3 g(nt, a.nsplit);
    if (nq == 1)
      hipLaunchKernelGGL(k_bi_reduce<1>, g, dim3(256), 0, s, a.tiles, a.ntile, a.part, a.part2, a.nrb, a.ldp,
                         a.nsplit);
    else if (nq == 2)
      hipLaunchKernelGGL(k_bi_reduce<2>, g, dim3(256), 0, s, a.tiles, a.ntile, a.part, a.part2, a.nrb, a.ldp,
                         a.nsplit);
    else
      hipLaunchKernelGGL(k_bi_reduce<BI_NQ>, g, dim3(256), 0, s, a.tiles, a.ntile, a.part, a.part2, a.nrb, a.ldp,
                         a.nsplit);
  };
  const double tol2 = tol * tol;
  const double nb = (double)sys.n * sizeof(C);
  const double nnzA = (double)sys.A->nnz, nnzB = sys.B ? (double)sys.B->nnz : 0.0;
  {
    const int tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_init<C>), dim3(a.nrb, ntile_all), dim3(256), 0, s, a);
    reduce(1, ntile_all);
    hipLaunchKernelGGL((k_bi_scalar<C, 0>), dim3(ntile_all), sb, 0, s, a, 0, maxit, tol2);
    prof_end(tok, s, K_BICG, 0.0, (double)sys.ncol * nb * 3.0);
  }
  // the launch grid follows the tile count read back every CHECK iterations; in
  // between, workgroups beyond the device-side count exit at once
  constexpr int CHECK = 4;
  int ntile = ntile_all;
  for (int it = 1; it <= maxit && ntile > 0; ++it) {
    const double cols = (double)ntile * BI_TILE;  // upper bound of the active columns
    int tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_sweep_a<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    prof_end(tok, s, K_SPMV, cols * 8.0 * (nnzA + nnzB + sys.n), cols * nb * 2.0);
    tok = prof_begin(s);
    reduce(2, ntile);
    hipLaunchKernelGGL((k_bi_scalar<C, 1>), dim3(ntile), sb, 0, s, a, it, maxit, tol2);
    prof_end(tok, s, K_BICG, 0.0, 0.0);
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_sweep_b<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    prof_end(tok, s, K_SPMV, cols * 8.0 * (nnzA + nnzB + sys.n), cols * nb * 3.0);
    tok = prof_begin(s);
    reduce(BI_NQ, ntile);
    hipLaunchKernelGGL((k_bi_scalar<C, 2>), dim3(ntile), sb, 0, s, a, it, maxit, tol2);
    hipLaunchKernelGGL((k_bi_sweep_c<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    reduce(1, ntile);
    hipLaunchKernelGGL((k_bi_scalar<C, 3>), dim3(ntile), sb, 0, s, a, it, maxit, tol2);
    hipLaunchKernelGGL(k_bi_compact, dim3(1), dim3(256), 0, s, sys.ncol, (const BiCol*)sys.col, sys.tiles, d_buf);
    prof_end(tok, s, K_BICG, 0.0, cols * nb * 8.0);
    if (hipGetLastError() != hipSuccess) return -2;
    if (it % CHECK == 0 || it == maxit) {
      MF_HIP_CHECK(hipMemcpyAsync(h_buf, d_buf, sizeof(int), hipMemcpyDeviceToHost, s));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      ntile = h_buf[0];
    }
  }
  its.assign(sys.ncol, 0);
  hipLaunchKernelGGL(k_bi_its, dim3(gs), dim3(256), 0, s, sys.ncol, (const BiCol*)sys.col, d_buf + 64);
  MF_HIP_CHECK(hipMemcpyAsync(h_buf + 64, d_buf + 64, sys.ncol * sizeof(int), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  for (int c = 0; c < sys.ncol; ++c) its[c] = h_buf[64 + c];
  return 0;
}

// ===========================================================================
// right-hand side and quadrature sum of the sparse path
// ===========================================================================
namespace {
template <typename R>
__global__ void k_bi_rhs(int64_t total, int m0, const double* __restrict__ rhs, const double* __restrict__ cs,
                         R* __restrict__ bh) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  bh[e] = (R)(rhs[e] * cs[e % m0]);
}

// Q[i][q] (+)= [resid: rho_q X[i][q]] + us_q * sum_j 2 Re(cf[j][q] x(i, j m0 + q)) over the
// nodes j0 .. j0 + nj - 1 held in the batch (x tile-major, columns start at node j0)
template <typename C>
__global__ void k_bi_accumulate(int64_t total, int64_t n, int m0, int nj, int j0, const C* __restrict__ x,
                                const c64* __restrict__ cf, const double* __restrict__ rho,
                                const double* __restrict__ us, const double* __restrict__ X,
                                double* __restrict__ Q, int mode) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t i = e / m0;
  const int q = (int)(e % m0);
  double acc = 0.0;
  for (int j = 0; j < nj; ++j) {
    const int64_t c = (int64_t)j * m0 + q;
    const c64 d = convert<c64, C>(x[((c >> 6) * n + i) * 64 + (c & 63)]);
    const c64 p = cf[(int64_t)(j0 + j) * m0 + q] * d;
    acc += 2.0 * p.re;
  }
  acc *= us[q];
  if (mode == 1) acc += rho[q] * X[e];
  if (mode == 2) acc += Q[e];
  Q[e] = acc;
}
}  // namespace

template <typename R>
int bi_rhs(hipStream_t s, int64_t n, int m0, const double* rhs, const double* cs, R* bh) {
  const int64_t total = n * (int64_t)m0;
  hipLaunchKernelGGL((k_bi_rhs<R>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, m0, rhs, cs, bh);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename C>
int bi_accumulate(hipStream_t s, int64_t n, int m0, int nj, int j0, const C* x, const c64* cf, const double* rho,
                  const double* us, const double* X, double* Q, int mode) {
  const int64_t total = n * (int64_t)m0;
  hipLaunchKernelGGL((k_bi_accumulate<C>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, n, m0,
                     nj, j0, x, cf, rho, us, X, Q, mode);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int csr_full<float>(hipStream_t, int64_t, const double*, const int32_t*, const int32_t*, int, char,
                             CsrWork&, CsrMat<float>&, int*);
template int csr_full<double>(hipStream_t, int64_t, const double*, const int32_t*, const int32_t*, int, char,
                              CsrWork&, CsrMat<double>&, int*);
// out[c] = sign * Re(sum_i R[i][c] x(i, c)) / cs[c]: R row-major n x m FP64 (ld m), x
// tile-major (one node of m columns); 256-row partials, then one ordered sum per column
template <typename C>
__global__ void k_bi_coldot_partial(int64_t n, int m, const double* __restrict__ R, const C* __restrict__ x,
                                    double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  double acc = 0.0;
  const int64_t r1 = ((chunk + 1) * 256 < n) ? (chunk + 1) * 256 : n;
  for (int64_t i = chunk * 256; i < r1; ++i) {
    const c64 d = convert<c64, C>(x[(((int64_t)c >> 6) * n + i) * 64 + (c & 63)]);
    acc += R[i * m + c] * d.re;
  }
  part[chunk * m + c] = acc;
}

__global__ void k_bi_coldot_final(int m, int nchunk, const double* __restrict__ part, const double* __restrict__ cs,
                                  double sign, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double acc = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) acc += part[(int64_t)ch * m + c];
  out[c] = sign * acc / cs[c];
}

template <typename C>
int bi_coldots(hipStream_t s, int64_t n, int m, const double* R, const C* x, const double* cs, double sign,
               double* out, double* partial) {
  const int nchunk = (int)((n + 255) / 256);
  hipLaunchKernelGGL((k_bi_coldot_partial<C>), dim3((m + 255) / 256, nchunk), dim3(256), 0, s, n, m, R, x, partial);
  hipLaunchKernelGGL(k_bi_coldot_final, dim3((m + 255) / 256), dim3(256), 0, s, m, nchunk, partial, cs, sign, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int bi_coldots<c32>(hipStream_t, int64_t, int, const double*, const c32*, const double*, double, double*,
                             double*);
template int bi_coldots<c64>(hipStream_t, int64_t, int, const double*, const c64*, const double*, double, double*,
                             double*);
template int bicgstab_batched<c32>(hipStream_t, const BiSys<c32>&, int, double, std::vector<int>&, int*, int*);
template int bicgstab_batched<c64>(hipStream_t, const BiSys<c64>&, int, double, std::vector<int>&, int*, int*);
template int bi_rhs<float>(hipStream_t, int64_t, int, const double*, const double*, float*);
template int bi_rhs<double>(hipStream_t, int64_t, int, const double*, const double*, double*);
template int bi_accumulate<c32>(hipStream_t, int64_t, int, int, int, const c32*, const c64*, const double*,
                                const double*, const double*, double*, int);
template int bi_accumulate<c64>(hipStream_t, int64_t, int, int, int, const c64*, const c64*, const double*,
                                const double*, const double*, double*, int);

}  // namespace mf
