// Sparse (CSR) kernels of the FEAST path without factorization (IFEAST).
//
//  * csr_full: the caller's CSR (0- or 1-based, full storage or one triangle of a
//    symmetric matrix) becomes a 0-based full-storage CSR with sorted columns, values
//    in FP64 (outer products A Q, B Q) and in the BiCGSTAB precision.
//  * spmm_rm: Y = M X for a row-major FP64 block X (the FP64 side of the iteration).
//  * bicgstab_batched: BiCGSTAB (van der Vorst 1992) on all shifted systems
//    (z_j B - A) x = b at once: one column per (node j, right-hand side q).  Every
//    node shares the same right-hand side block b (n x m0, real), so the shadow residual
//    r_hat = r_0 = b is stored once.  Vectors are row-major n x ncol blocks
//    (ncol = nodes * m0, column c = j * m0 + q) so that a sparse row touches
//    contiguous memory across all columns; per-column inner products are reduced in
//    FP64, deterministically (per-workgroup partials, then a fixed-order sum).
//    Converged columns stop: the host rebuilds the list of 64-column tiles that
//    still hold an active column after every iteration and launches only those.
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
namespace {

constexpr int BI_TILE = 64;                // columns per tile: one lane per column
constexpr int BI_WAVES = 4;                // waves per workgroup, each on its own rows
constexpr int BI_RB = 256;                 // rows per workgroup
constexpr int BI_RW = BI_RB / BI_WAVES;    // rows per wave

enum { ST_ACTIVE = 0, ST_HALF = 1, ST_DONE = 2 };

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
  C *x, *r, *p, *v, *s, *t;
  BiCol* col;
  const int* tiles;
  double* part;  // [quantity][row block][column]
};

// sum the per-lane partials of the 4 waves and store them as one partial per column
template <int NQ>
__device__ inline void bi_store_partials(double (&acc)[NQ], double* part, int nrb, int ncol, int c) {
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

// x = 0, r = b; partial b^T b
template <typename C>
__global__ __launch_bounds__(256) void k_bi_init(BiK<C> a) {
  using R = typename real_of<C>::type;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.tiles[blockIdx.y] * BI_TILE + lane;
  const bool in = c < a.ncol;
  const int q = in ? c % a.m0 : 0;
  double acc[1] = {0.0};
  const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
  const int64_t r1 = (r0 + BI_RW < a.n) ? r0 + BI_RW : a.n;
  if (in) {
    for (int64_t i = r0; i < r1; ++i) {
      const R b = a.bh[i * a.m0 + q];
      a.r[i * a.ncol + c] = C(b, R(0));
      a.x[i * a.ncol + c] = C(R(0), R(0));
      acc[0] += (double)b * (double)b;
    }
  }
  bi_store_partials<1>(acc, a.part, a.nrb, a.ncol, in ? c : -1);
}

// p = r (first iteration) or p = r + beta (p - omega v)
template <typename C>
__global__ __launch_bounds__(256) void k_bi_p(BiK<C> a, int first) {
  using R = typename real_of<C>::type;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.tiles[blockIdx.y] * BI_TILE + lane;
  if (c >= a.ncol || a.col[c].state != ST_ACTIVE) return;
  const C be = convert<C, c64>(a.col[c].beta), om = convert<C, c64>(a.col[c].omega);
  const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
  const int64_t r1 = (r0 + BI_RW < a.n) ? r0 + BI_RW : a.n;
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t o = i * a.ncol + c;
    const C rv = a.r[o];
    if (first) {
      a.p[o] = rv;
    } else {
      a.p[o] = rv + be * (a.p[o] - om * a.v[o]);
    }
  }
}

// out = z_j (B in) - A in for the active columns, with per-column partial sums:
// MODE 0: r_hat^H out (2 values); MODE 1: out^H in (2), ||out||^2, ||in||^2
template <typename C, int MODE>
__global__ __launch_bounds__(256) void k_bi_spmv(BiK<C> a, const C* __restrict__ in, C* __restrict__ out) {
  using R = typename real_of<C>::type;
  constexpr int NQ = MODE == 0 ? 2 : 4;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.tiles[blockIdx.y] * BI_TILE + lane;
  const bool act = c < a.ncol && a.col[c].state == ST_ACTIVE;
  C z(R(0), R(0));
  int q = 0;
  if (act) {
    z = convert<C, c64>(a.zn[c / a.m0]);
    q = c % a.m0;
  }
  double acc[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) acc[k] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
  const int64_t r1 = (r0 + BI_RW < a.n) ? r0 + BI_RW : a.n;
  const int64_t ld = a.ncol;
  for (int64_t i = r0; i < r1; ++i) {
    const int kb = a.rp[i], ke = a.rp[i + 1];
    if (!act) continue;
    C sa(R(0), R(0));
    for (int k = kb; k < ke; ++k) {
      const R av = a.va[k];
      const C xv = in[(int64_t)a.ci[k] * ld + c];
      sa.re += av * xv.re;
      sa.im += av * xv.im;
    }
    const C xi = in[i * ld + c];
    C sb = xi;
    if (a.rpb != nullptr) {
      sb = C(R(0), R(0));
      const int bb = a.rpb[i], be = a.rpb[i + 1];
      for (int k = bb; k < be; ++k) {
        const R bv = a.vb[k];
        const C xv = in[(int64_t)a.cib[k] * ld + c];
        sb.re += bv * xv.re;
        sb.im += bv * xv.im;
      }
    }
    const C o = z * sb - sa;
    out[i * ld + c] = o;
    if constexpr (MODE == 0) {
      const double h = (double)a.bh[i * a.m0 + q];
      acc[0] += h * (double)o.re;
      acc[1] += h * (double)o.im;
    } else {
      const double ore = o.re, oim = o.im, sre = xi.re, sim = xi.im;
      acc[0] += ore * sre + oim * sim;  // conj(t) s
      acc[1] += ore * sim - oim * sre;
      acc[2] += ore * ore + oim * oim;
      acc[3] += sre * sre + sim * sim;
    }
  }
  bi_store_partials<NQ>(acc, a.part, a.nrb, a.ncol, act ? c : -1);
}

// s = r - alpha v
template <typename C>
__global__ __launch_bounds__(256) void k_bi_s(BiK<C> a) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.tiles[blockIdx.y] * BI_TILE + lane;
  if (c >= a.ncol || a.col[c].state != ST_ACTIVE) return;
  const C al = convert<C, c64>(a.col[c].alpha);
  const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
  const int64_t r1 = (r0 + BI_RW < a.n) ? r0 + BI_RW : a.n;
  for (int64_t i = r0; i < r1; ++i) {
    const int64_t o = i * a.ncol + c;
    a.s[o] = a.r[o] - al * a.v[o];
  }
}

// x += alpha p + omega s, r = s - omega t (active); x += alpha p (converged at the half
// step); partial r_hat^H r (2), ||r||^2
template <typename C>
__global__ __launch_bounds__(256) void k_bi_update(BiK<C> a) {
  using R = typename real_of<C>::type;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int c = a.tiles[blockIdx.y] * BI_TILE + lane;
  const int st = (c < a.ncol) ? a.col[c].state : ST_DONE;
  double acc[3] = {0.0, 0.0, 0.0};
  if (st != ST_DONE) {
    const C al = convert<C, c64>(a.col[c].alpha), om = convert<C, c64>(a.col[c].omega);
    const int q = c % a.m0;
    const int64_t r0 = (int64_t)blockIdx.x * BI_RB + (int64_t)w * BI_RW;
    const int64_t r1 = (r0 + BI_RW < a.n) ? r0 + BI_RW : a.n;
    for (int64_t i = r0; i < r1; ++i) {
      const int64_t o = i * a.ncol + c;
      if (st == ST_HALF) {
        a.x[o] = a.x[o] + al * a.p[o];
      } else {
        const C sv = a.s[o];
        a.x[o] = a.x[o] + al * a.p[o] + om * sv;
        const C rv = sv - om * a.t[o];
        a.r[o] = rv;
        const double h = (double)a.bh[i * a.m0 + q];
        acc[0] += h * (double)rv.re;
        acc[1] += h * (double)rv.im;
        acc[2] += (double)rv.re * rv.re + (double)rv.im * rv.im;
      }
    }
  }
  bi_store_partials<3>(acc, a.part, a.nrb, a.ncol, (st == ST_ACTIVE) ? c : -1);
}

// per-column scalar step after each reduction (one thread per column, fixed-order sums)
// MODE 0: init, 1: alpha, 2: omega and the half-step test, 3: rho, beta and the final test
template <typename C, int MODE>
__global__ void k_bi_scalar(BiK<C> a, int it, int maxit, double tol2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= a.ncol) return;
  BiCol& cs = a.col[c];
  constexpr int NQ = MODE == 0 ? 1 : MODE == 1 ? 2 : MODE == 2 ? 4 : 3;
  if constexpr (MODE != 0) {
    if (MODE == 3 ? cs.state == ST_DONE : cs.state != ST_ACTIVE) return;
  }
  double sum[NQ];
  for (int q = 0; q < NQ; ++q) sum[q] = 0.0;
  if (MODE != 3 || cs.state == ST_ACTIVE) {
    for (int b = 0; b < a.nrb; ++b)
      for (int q = 0; q < NQ; ++q) sum[q] += a.part[((int64_t)q * a.nrb + b) * a.ncol + c];
  }
  if constexpr (MODE == 0) {
    cs.bn2 = sum[0];
    cs.rho = c64(sum[0], 0.0);
    cs.alpha = c64(1.0, 0.0);
    cs.omega = c64(1.0, 0.0);
    cs.beta = c64(0.0, 0.0);
    cs.its = 0;
    cs.state = sum[0] > 0.0 ? ST_ACTIVE : ST_DONE;
  } else if constexpr (MODE == 1) {
    const c64 den(sum[0], sum[1]);
    if (den.re == 0.0 && den.im == 0.0) {
      cs.state = ST_DONE;
      cs.its = it;
    } else {
      cs.alpha = cdiv(cs.rho, den);
    }
  } else if constexpr (MODE == 2) {
    if (sum[3] <= tol2 * cs.bn2) {
      cs.state = ST_HALF;
    } else {
      cs.omega = sum[2] != 0.0 ? c64(sum[0] / sum[2], sum[1] / sum[2]) : c64(0.0, 0.0);
    }
  } else {
    cs.its = it;
    if (cs.state == ST_HALF) {
      cs.state = ST_DONE;
      return;
    }
    const c64 rho_new(sum[0], sum[1]);
    if (sum[2] <= tol2 * cs.bn2 || (rho_new.re == 0.0 && rho_new.im == 0.0) ||
        (cs.omega.re == 0.0 && cs.omega.im == 0.0) || it >= maxit) {
      cs.state = ST_DONE;
      return;
    }
    cs.beta = cdiv(rho_new, cs.rho) * cdiv(cs.alpha, cs.omega);
    cs.rho = rho_new;
  }
}

}  // namespace

namespace {
// states (which = 0) or iteration counts (which = 1) of every column, packed
__global__ void k_bi_gather(int ncol, const BiCol* __restrict__ col, int which, int* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncol) out[c] = which == 0 ? col[c].state : col[c].its;
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
  a.s = sys.s;
  a.t = sys.t;
  a.col = sys.col;
  a.tiles = sys.tiles;
  a.part = sys.part;
  const int ntile_all = (sys.ncol + BI_TILE - 1) / BI_TILE;
  std::vector<int> tl(ntile_all);
  for (int i = 0; i < ntile_all; ++i) tl[i] = i;
  int* d_tiles = sys.tiles;
  MF_HIP_CHECK(hipMemcpyAsync(d_tiles, tl.data(), ntile_all * sizeof(int), hipMemcpyHostToDevice, s));
  int ntile = ntile_all;
  const unsigned gs = (unsigned)((sys.ncol + 255) / 256);
  const double tol2 = tol * tol;
  const double nb = (double)sys.n * sizeof(C);
  {
    const int tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_init<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_bi_scalar<C, 0>), dim3(gs), dim3(256), 0, s, a, 0, maxit, tol2);
    prof_end(tok, s, K_BICG, 0.0, (double)sys.ncol * nb * 2.0);
  }
  std::vector<int> st(sys.ncol);
  for (int it = 1; it <= maxit && ntile > 0; ++it) {
    const double cols = (double)ntile * BI_TILE;
    const double nnzA = (double)sys.A->nnz, nnzB = sys.B ? (double)sys.B->nnz : 0.0;
    int tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_p<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a, it == 1 ? 1 : 0);
    prof_end(tok, s, K_BICG, 0.0, cols * nb * (it == 1 ? 2.0 : 4.0));
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_spmv<C, 0>), dim3(a.nrb, ntile), dim3(256), 0, s, a, (const C*)a.p, a.v);
    prof_end(tok, s, K_SPMV, cols * 8.0 * (nnzA + nnzB + sys.n), cols * nb * 2.0);
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_scalar<C, 1>), dim3(gs), dim3(256), 0, s, a, it, maxit, tol2);
    hipLaunchKernelGGL((k_bi_s<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    prof_end(tok, s, K_BICG, 0.0, cols * nb * 3.0);
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_spmv<C, 1>), dim3(a.nrb, ntile), dim3(256), 0, s, a, (const C*)a.s, a.t);
    prof_end(tok, s, K_SPMV, cols * 8.0 * (nnzA + nnzB + sys.n), cols * nb * 2.0);
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_bi_scalar<C, 2>), dim3(gs), dim3(256), 0, s, a, it, maxit, tol2);
    hipLaunchKernelGGL((k_bi_update<C>), dim3(a.nrb, ntile), dim3(256), 0, s, a);
    hipLaunchKernelGGL((k_bi_scalar<C, 3>), dim3(gs), dim3(256), 0, s, a, it, maxit, tol2);
    prof_end(tok, s, K_BICG, 0.0, cols * nb * 6.0);
    if (hipGetLastError() != hipSuccess) return -2;
    // rebuild the tile list from the column states
    hipLaunchKernelGGL(k_bi_gather, dim3(gs), dim3(256), 0, s, sys.ncol, (const BiCol*)sys.col, 0, d_buf);
    MF_HIP_CHECK(hipMemcpyAsync(h_buf, d_buf, sys.ncol * sizeof(int), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    ntile = 0;
    for (int tix = 0; tix < ntile_all; ++tix) {
      bool any = false;
      for (int c = tix * BI_TILE; c < std::min(sys.ncol, (tix + 1) * BI_TILE); ++c)
        any = any || h_buf[c] == ST_ACTIVE;
      if (any) tl[ntile++] = tix;
    }
    if (ntile > 0)
      MF_HIP_CHECK(hipMemcpyAsync(d_tiles, tl.data(), ntile * sizeof(int), hipMemcpyHostToDevice, s));
  }
  its.assign(sys.ncol, 0);
  hipLaunchKernelGGL(k_bi_gather, dim3(gs), dim3(256), 0, s, sys.ncol, (const BiCol*)sys.col, 1, d_buf);
  MF_HIP_CHECK(hipMemcpyAsync(h_buf, d_buf, sys.ncol * sizeof(int), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  for (int c = 0; c < sys.ncol; ++c) its[c] = h_buf[c];
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

// Q[i][q] (+)= [resid: rho_q X[i][q]] + us_q * sum_j 2 Re(cf[j][q] x[i][j m0 + q]) over the
// nodes j0 .. j0 + nj - 1 held in the batch (x columns start at node j0)
template <typename C>
__global__ void k_bi_accumulate(int64_t total, int m0, int nj, int j0, const C* __restrict__ x, int ncol,
                                const c64* __restrict__ cf, const double* __restrict__ rho,
                                const double* __restrict__ us, const double* __restrict__ X,
                                double* __restrict__ Q, int mode) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int64_t i = e / m0;
  const int q = (int)(e % m0);
  double acc = 0.0;
  for (int j = 0; j < nj; ++j) {
    const c64 d = convert<c64, C>(x[i * ncol + (int64_t)j * m0 + q]);
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
int bi_accumulate(hipStream_t s, int64_t n, int m0, int nj, int j0, const C* x, int ncol, const c64* cf,
                  const double* rho, const double* us, const double* X, double* Q, int mode) {
  const int64_t total = n * (int64_t)m0;
  hipLaunchKernelGGL((k_bi_accumulate<C>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, total, m0, nj,
                     j0, x, ncol, cf, rho, us, X, Q, mode);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int csr_full<float>(hipStream_t, int64_t, const double*, const int32_t*, const int32_t*, int, char,
                             CsrWork&, CsrMat<float>&, int*);
template int csr_full<double>(hipStream_t, int64_t, const double*, const int32_t*, const int32_t*, int, char,
                              CsrWork&, CsrMat<double>&, int*);
template int bicgstab_batched<c32>(hipStream_t, const BiSys<c32>&, int, double, std::vector<int>&, int*, int*);
template int bicgstab_batched<c64>(hipStream_t, const BiSys<c64>&, int, double, std::vector<int>&, int*, int*);
template int bi_rhs<float>(hipStream_t, int64_t, int, const double*, const double*, float*);
template int bi_rhs<double>(hipStream_t, int64_t, int, const double*, const double*, double*);
template int bi_accumulate<c32>(hipStream_t, int64_t, int, int, int, const c32*, int, const c64*, const double*,
                                const double*, const double*, double*, int);
template int bi_accumulate<c64>(hipStream_t, int64_t, int, int, int, const c64*, int, const c64*, const double*,
                                const double*, const double*, double*, int);

}  // namespace mf
