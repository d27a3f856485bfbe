// Rayleigh-Ritz helpers in FP64 (gfx950): column reductions, equilibration of the
// reduced overlap, the reduced Hermitian eigensolver, residuals and layout copies.
//
// The reduced problem Aq W = Bq W Lambda (Aq = Q^H A Q, Bq = Q^H B Q; FEAST Hermitian
// RCI, Table tab-rci1) is solved by two Hermitian eigendecompositions: of the
// equilibrated overlap (rank-revealing, so a subspace that lost rank shrinks M0)
// and of the projected Aq.  The eigensolver is a two-sided cyclic Jacobi method
// with round-robin (circle) ordering: every round rotates M/2 disjoint index pairs
// at once, which makes each 2x2 block update of the round independent.
#include <hip/hip_cooperative_groups.h>

#include "kernels.hpp"

namespace cg = cooperative_groups;

namespace mf {

__device__ inline double absval(double a) { return fabs(a); }
__device__ inline double absval(c64 a) { return sqrt(a.re * a.re + a.im * a.im); }

// ---------------------------------------------------------------------------
__global__ void k_fill_double(int count, double* p, double v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <typename T>
__global__ void k_col_absmax(int64_t n, int m, const T* __restrict__ X, int64_t ld, double* out) {
  // block: 64 columns x 4 row lanes; each block covers 256 rows
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t r0 = (int64_t)blockIdx.y * 256 + (threadIdx.x >> 6);
  if (c >= m) return;
  double mx = 0.0;
  const int64_t rend = ((int64_t)blockIdx.y * 256 + 256 < n) ? (int64_t)blockIdx.y * 256 + 256 : n;
  for (int64_t r = r0; r < rend; r += 4) mx = fmax(mx, absval(X[r * ld + c]));
  // non-negative doubles order like their bit patterns
  atomicMax(reinterpret_cast<unsigned long long*>(out + c), (unsigned long long)__double_as_longlong(mx));
}

template <typename T>
int col_absmax(hipStream_t s, int64_t n, int m, const T* X, int64_t ld, double* out) {
  hipLaunchKernelGGL(k_fill_double, dim3((m + 255) / 256), dim3(256), 0, s, m, out, 0.0);
  dim3 grid((unsigned)((m + 63) / 64), (unsigned)((n + 255) / 256));
  hipLaunchKernelGGL((k_col_absmax<T>), grid, dim3(256), 0, s, n, m, X, ld, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// d_i = 1 / sqrt(Re S_ii); S <- D (S + S^H)/2 D, Tm <- D (Tm + Tm^H)/2 D, in place.
__global__ void k_diag_scale(int m, const void* Sv, int cplx, double* d, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double sii = cplx ? static_cast<const c64*>(Sv)[(int64_t)i * m + i].re
                          : static_cast<const double*>(Sv)[(int64_t)i * m + i];
  if (!(sii > 0.0)) {
    atomicOr(flag, 1);
    d[i] = 0.0;
  } else {
    d[i] = 1.0 / sqrt(sii);
  }
}

template <typename T>
__global__ void k_sym_scale(int m, T* S, T* Tm, const double* __restrict__ d) {
  // one thread per (i, j) with i <= j; writes both (i, j) and (j, i)
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m || j < i) return;
  const double f = d[i] * d[j];
  const int64_t a = (int64_t)i * m + j, b = (int64_t)j * m + i;
  T s = 0.5 * (S[a] + conj(S[b]));
  T t = 0.5 * (Tm[a] + conj(Tm[b]));
  s = f * s;
  t = f * t;
  if (i == j) {
    s = T(real_part(s));
    t = T(real_part(t));
  }
  S[a] = s;
  S[b] = conj(s);
  Tm[a] = t;
  Tm[b] = conj(t);
}

template <typename T>
__global__ void k_herm_part(int m, T* H) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m || j < i) return;
  const int64_t a = (int64_t)i * m + j, b = (int64_t)j * m + i;
  T v = 0.5 * (H[a] + conj(H[b]));
  if (i == j) v = T(real_part(v));
  H[a] = v;
  H[b] = conj(v);
}

template <typename T>
int hermitian_part(hipStream_t s, int m, T* H) {
  hipLaunchKernelGGL((k_herm_part<T>), dim3((m + 255) / 256, m), dim3(256), 0, s, m, H);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int gram_equilibrate(hipStream_t s, int m, T* S, T* Tm, double* d, int* flag) {
  hipLaunchKernelGGL(k_diag_scale, dim3((m + 255) / 256), dim3(256), 0, s, m, (const void*)S,
                     (int)is_cplx<T>::value, d, flag);
  hipLaunchKernelGGL((k_sym_scale<T>), dim3((m + 255) / 256, m), dim3(256), 0, s, m, S, Tm, d);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Cyclic Jacobi, round-robin ordering, cooperative launch.  H (m x m, row-major,
// Hermitian) is read from one buffer and written to the other every round so that
// the rotation parameters (computed redundantly by every workgroup from the 2x2
// diagonal blocks) never race with the updates.  Every workgroup sees the same
// rotations and therefore takes the same decisions, so no grid-wide vote is needed
// to stop: the sweep loop ends after a sweep in which no pair was rotated.
constexpr int JAC_MAXPAIR = 512;  // m <= 1024

template <typename T>
__device__ inline T rot_sigma(double s, T ph);
template <> __device__ inline double rot_sigma<double>(double s, double ph) { return s * ph; }
template <> __device__ inline c64 rot_sigma<c64>(double s, c64 ph) { return c64(s * ph.re, s * ph.im); }

template <typename T>
__device__ inline T phase_of(T b, double ab);
template <> __device__ inline double phase_of<double>(double b, double ab) { return b >= 0 ? 1.0 : -1.0; }
template <> __device__ inline c64 phase_of<c64>(c64 b, double ab) { return c64(b.re / ab, b.im / ab); }

template <typename T>
__global__ __launch_bounds__(256) void k_jacobi(int m, T* Ha, T* Hb, T* V, double* evals, int max_sweeps,
                                                 double tol, int* sweeps_out) {
  cg::grid_group grid = cg::this_grid();
  const int mp = m + (m & 1);
  const int npair = mp / 2;
  __shared__ double s_c[JAC_MAXPAIR];
  __shared__ T s_sg[JAC_MAXPAIR];
  __shared__ int s_p[JAC_MAXPAIR], s_q[JAC_MAXPAIR];
  __shared__ int s_cnt;
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
  const int64_t mm = (int64_t)m * m;

  for (int64_t e = gtid; e < mm; e += gsz) V[e] = (e / m == e % m) ? T(1.0) : T(0.0);
  T* src = Ha;
  T* dst = Hb;
  // absolute floor for rotations: off-diagonal entries below 2 eps max|h_ii| carry
  // no information beyond rounding
  double dmax = 0.0;
  for (int i = 0; i < m; ++i) dmax = fmax(dmax, fabs(real_part(Ha[(int64_t)i * m + i])));
  const double abs_floor = 4.440892098500626e-16 * dmax + 1e-300;
  grid.sync();

  int sweep = 0;
  for (; sweep < max_sweeps; ++sweep) {
    int total = 0;
    for (int round = 0; round < mp - 1; ++round) {
      if (threadIdx.x == 0) s_cnt = 0;
      __syncthreads();
      for (int i = threadIdx.x; i < npair; i += blockDim.x) {
        const int a = (i == 0) ? 0 : 1 + (i - 1 + round) % (mp - 1);
        const int b = 1 + (mp - 2 - i + round) % (mp - 1);
        const int p = min(a, b), q = max(a, b);
        double c = 1.0;
        T sg = T(0.0);
        if (q < m) {
          const double app = real_part(src[(int64_t)p * m + p]);
          const double aqq = real_part(src[(int64_t)q * m + q]);
          const T apq = src[(int64_t)p * m + q];
          const double ab = absval(apq);
          if (ab > tol * sqrt(fabs(app * aqq)) && ab > abs_floor) {
            const T ph = phase_of<T>(apq, ab);
            const double tau = (aqq - app) / (2.0 * ab);
            double t;
            if (fabs(tau) > 1e150) t = 0.5 / tau;
            else t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sg = rot_sigma<T>(t * c, ph);
            atomicAdd(&s_cnt, 1);
          }
        }
        s_c[i] = c;
        s_sg[i] = sg;
        s_p[i] = p;
        s_q[i] = q;
      }
      __syncthreads();
      const int cnt = s_cnt;
      __syncthreads();  // every thread has read the count before it is reset next round
      total += cnt;
      if (cnt == 0) continue;  // uniform across the grid: nothing to apply this round
      // H' = J^H H J blockwise, J_P = [[c, sg], [-conj(sg), c]] on (p, q)
      const int64_t nblk = (int64_t)npair * npair;
      for (int64_t e = gtid; e < nblk; e += gsz) {
        const int P = (int)(e / npair), Qb = (int)(e % npair);
        const int p1 = s_p[P], q1 = s_q[P], p2 = s_p[Qb], q2 = s_q[Qb];
        const double cP = s_c[P], cQ = s_c[Qb];
        const T sP = s_sg[P], sQ = s_sg[Qb];
        const bool v1 = q1 < m, v2 = q2 < m;  // phantom index m when m is odd
        const T h11 = src[(int64_t)p1 * m + p2];
        const T h12 = v2 ? src[(int64_t)p1 * m + q2] : T(0.0);
        const T h21 = v1 ? src[(int64_t)q1 * m + p2] : T(0.0);
        const T h22 = (v1 && v2) ? src[(int64_t)q1 * m + q2] : T(0.0);
        // t = h J_Q
        const T t11 = cQ * h11 - h12 * conj(sQ);
        const T t12 = h11 * sQ + cQ * h12;
        const T t21 = cQ * h21 - h22 * conj(sQ);
        const T t22 = h21 * sQ + cQ * h22;
        // J_P^H t
        const T r11 = cP * t11 - sP * t21;
        const T r12 = cP * t12 - sP * t22;
        const T r21 = conj(sP) * t11 + cP * t21;
        const T r22 = conj(sP) * t12 + cP * t22;
        dst[(int64_t)p1 * m + p2] = r11;
        if (v2) dst[(int64_t)p1 * m + q2] = r12;
        if (v1) dst[(int64_t)q1 * m + p2] = r21;
        if (v1 && v2) dst[(int64_t)q1 * m + q2] = r22;
      }
      // V' = V J
      const int64_t nv = (int64_t)m * npair;
      for (int64_t e = gtid; e < nv; e += gsz) {
        const int x = (int)(e / npair), Qb = (int)(e % npair);
        const int p2 = s_p[Qb], q2 = s_q[Qb];
        if (q2 >= m) continue;
        const double cQ = s_c[Qb];
        const T sQ = s_sg[Qb];
        const T a = V[(int64_t)x * m + p2];
        const T b = V[(int64_t)x * m + q2];
        V[(int64_t)x * m + p2] = cQ * a - b * conj(sQ);
        V[(int64_t)x * m + q2] = a * sQ + cQ * b;
      }
      T* tmp = src;
      src = dst;
      dst = tmp;
      grid.sync();
    }
    if (total == 0) break;
  }
  for (int64_t i = gtid; i < m; i += gsz) evals[i] = real_part(src[i * m + i]);
  if (gtid == 0) *sweeps_out = sweep;
}

template <typename T>
int jacobi_eigh(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps_out, double* work, double big_rel) {
  if (m > 2 * JAC_MAXPAIR) return -2;
  if (m > 64 || !coop_allowed()) {
    // block Jacobi (eig.hip); work holds the round's unitaries, then a counter
    T* ubuf = reinterpret_cast<T*>(work);
    int* counter = reinterpret_cast<int*>(reinterpret_cast<char*>(work) + block_jacobi_work_bytes(m, sizeof(T)) - 64);
    return block_jacobi<T>(s, m, H, V, evals, sweeps_out, ubuf, counter, 40, big_rel);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -2;
  int ncu = 0, per_cu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -2;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_jacobi<T>, 256, 0) != hipSuccess) return -2;
  const int npair = (m + 1) / 2;
  const int64_t work_items = (int64_t)npair * npair;
  int nblocks = (int)std::min<int64_t>((work_items + 255) / 256, (int64_t)ncu * std::max(1, per_cu));
  nblocks = std::max(1, std::min(nblocks, 2 * ncu));
  T* Hb = reinterpret_cast<T*>(work);
  int max_sweeps = 40;
  double tol = 1.0e-15;
  void* args[] = {&m, &H, &Hb, &V, &evals, &max_sweeps, &tol, &sweeps_out};
  hipError_t e = hipLaunchCooperativeKernel((const void*)k_jacobi<T>, dim3(nblocks), dim3(256), args, 0, s);
  return e == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_gather_scale_cols(int rows, int k, const T* __restrict__ V, int ldv, const int* __restrict__ idx,
                                    const double* __restrict__ scale, T* __restrict__ G, int ldg) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (t >= k) return;
  G[(int64_t)i * ldg + t] = scale[t] * V[(int64_t)i * ldv + idx[t]];
}

template <typename T>
int gather_scale_cols(hipStream_t s, int rows, int k, const T* V, int ldv, const int* idx, const double* scale,
                      T* G, int ldg) {
  hipLaunchKernelGGL((k_gather_scale_cols<T>), dim3((k + 255) / 256, rows), dim3(256), 0, s, rows, k, V, ldv, idx,
                     scale, G, ldg);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
__global__ void k_scale_rows_permute_cols(int rows, int k, const T* __restrict__ GZ, int ldgz,
                                          const double* __restrict__ d, const int* __restrict__ perm,
                                          T* __restrict__ W, int ldw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (t >= k) return;
  W[(int64_t)i * ldw + t] = d[i] * GZ[(int64_t)i * ldgz + perm[t]];
}

template <typename T>
int scale_rows_permute_cols(hipStream_t s, int rows, int k, const T* GZ, int ldgz, const double* d, const int* perm,
                            T* W, int ldw) {
  hipLaunchKernelGGL((k_scale_rows_permute_cols<T>), dim3((k + 255) / 256, rows), dim3(256), 0, s, rows, k, GZ,
                     ldgz, d, perm, W, ldw);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// R = AX - BX diag(lam); column sums of |R|^2 and |BX|^2 (two deterministic passes)
constexpr int RES_ROWS = 256;

template <typename T>
__global__ void k_residual_partial(int64_t n, int m, const T* __restrict__ AX, const T* __restrict__ BX,
                                   const double* __restrict__ lam, T* __restrict__ R, double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  double sr = 0.0, sb = 0.0;
  const int64_t r1 = ((chunk + 1) * RES_ROWS < n) ? (chunk + 1) * RES_ROWS : n;
  for (int64_t r = chunk * RES_ROWS; r < r1; ++r) {
    const T bx = BX[r * m + c];
    const T rv = AX[r * m + c] - lam[c] * bx;
    R[r * m + c] = rv;
    sr += norm2(rv);
    sb += norm2(bx);
  }
  part[(chunk * m + c) * 2] = sr;
  part[(chunk * m + c) * 2 + 1] = sb;
}

__global__ void k_residual_final(int m, int nchunk, const double* __restrict__ part, double* rn, double* bn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double sr = 0.0, sb = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    sr += part[((int64_t)ch * m + c) * 2];
    sb += part[((int64_t)ch * m + c) * 2 + 1];
  }
  rn[c] = sr;
  bn[c] = sb;
}

template <typename T>
int residual_norms(hipStream_t s, int64_t n, int m, const T* AX, const T* BX, const double* lam, T* R, double* rnorm2,
                   double* bnorm2, double* partial) {
  const int nchunk = (int)((n + RES_ROWS - 1) / RES_ROWS);
  hipLaunchKernelGGL((k_residual_partial<T>), dim3((m + 255) / 256, nchunk), dim3(256), 0, s, n, m, AX, BX, lam, R,
                     partial);
  hipLaunchKernelGGL(k_residual_final, dim3((m + 255) / 256), dim3(256), 0, s, m, nchunk, partial, rnorm2, bnorm2);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_transpose_copy(int64_t rows, int64_t cols, const T* __restrict__ src, int64_t lds,
                                 T* __restrict__ dst, int64_t ldd, const int* __restrict__ colmap) {
  // dst[j*ldd + i] = src[i*lds + colmap[j]] (colmap null: identity), tiled through LDS
  __shared__ T tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32, j0 = (int64_t)blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t i = i0 + yy, j = j0 + tx;
    if (i < rows && j < cols) tile[yy][tx] = src[i * lds + (colmap ? (int64_t)colmap[j] : j)];
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t j = j0 + yy, i = i0 + tx;
    if (i < rows && j < cols) dst[j * ldd + i] = tile[tx][yy];
  }
}

template <typename T>
int copy_rm_to_cm(hipStream_t s, int64_t n, int m, const T* src, int64_t lds, T* dst, int64_t ldd,
                  const int* colmap) {
  // src row-major n x m  ->  dst column-major n x m, column j taken from src column colmap[j]
  dim3 grid((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32));
  hipLaunchKernelGGL((k_transpose_copy<T>), grid, dim3(256), 0, s, n, (int64_t)m, src, lds, dst, ldd, colmap);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T>
int copy_cm_to_rm(hipStream_t s, int64_t n, int m, const T* src, int64_t lds, T* dst, int64_t ldd) {
  // src column-major n x m (viewed as row-major m x n) -> dst row-major n x m
  dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
  hipLaunchKernelGGL((k_transpose_copy<T>), grid, dim3(256), 0, s, (int64_t)m, n, src, lds, dst, ldd,
                     (const int*)nullptr);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Starting block from SplitMix64 (Steele, Lea, Flood 2014): entry counter t maps to
// state seed + (t+1) * 0x9E3779B97F4A7C15, the published finaliser, then 2*(z>>11)*2^-53 - 1.
// Counter of entry (i, j) of the n x m block: t = i + j*n (real), 2(i + j*n) + {0,1} (complex).
__device__ inline uint64_t splitmix_raw(uint64_t seed, uint64_t t) {
  uint64_t z = seed + (t + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double splitmix_uniform(uint64_t seed, uint64_t t) {
  return 2.0 * ((double)(splitmix_raw(seed, t) >> 11) * 0x1.0p-53) - 1.0;
}

template <typename T>
__global__ void k_random_block(int64_t n, int m, uint64_t seed, T* __restrict__ Y, int64_t ld) {
  // rows on grid x (no 16-bit limit for tall blocks), 256-column chunks on grid y
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.x;
  if (j >= m) return;
  const uint64_t t = (uint64_t)i + (uint64_t)j * (uint64_t)n;
  if constexpr (is_cplx<T>::value) {
    Y[i * ld + j] = T(splitmix_uniform(seed, 2 * t), splitmix_uniform(seed, 2 * t + 1));
  } else {
    Y[i * ld + j] = splitmix_uniform(seed, t);
  }
}

template <typename T>
int random_block(hipStream_t s, int64_t n, int m, uint64_t seed, T* Y, int64_t ld) {
  hipLaunchKernelGGL((k_random_block<T>), dim3((unsigned)n, (m + 255) / 256), dim3(256), 0, s, n, m, seed, Y, ld);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Probe block of the stochastic eigenvalue count: real Rademacher entries, -1 where the
// top bit of SplitMix64 output t = i + j*n is set, else +1 (imaginary parts zero).
template <typename T>
__global__ void k_rademacher_block(int64_t n, int m, uint64_t seed, T* __restrict__ Y, int64_t ld) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.x;
  if (j >= m) return;
  const uint64_t t = (uint64_t)i + (uint64_t)j * (uint64_t)n;
  Y[i * ld + j] = T((splitmix_raw(seed, t) >> 63) ? -1.0 : 1.0);
}

template <typename T>
int rademacher_block(hipStream_t s, int64_t n, int m, uint64_t seed, T* Y, int64_t ld) {
  hipLaunchKernelGGL((k_rademacher_block<T>), dim3((unsigned)n, (m + 255) / 256), dim3(256), 0, s, n, m, seed, Y,
                     ld);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// out[c] = Re(sum_r conj(Y[r][c]) Q[r][c]) for row-major n x m blocks (leading dimension
// m): per-chunk partial sums of RES_ROWS rows, then one sum over the chunks per column
// (deterministic order)
template <typename T>
__global__ void k_coldot_partial(int64_t n, int m, const T* __restrict__ Y, const T* __restrict__ Q,
                                 double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  double acc = 0.0;
  const int64_t r1 = ((chunk + 1) * RES_ROWS < n) ? (chunk + 1) * RES_ROWS : n;
  for (int64_t r = chunk * RES_ROWS; r < r1; ++r) {
    const T y = Y[r * m + c], q = Q[r * m + c];
    if constexpr (is_cplx<T>::value) acc += y.re * q.re + y.im * q.im;
    else acc += y * q;
  }
  part[chunk * m + c] = acc;
}

__global__ void k_coldot_final(int m, int nchunk, const double* __restrict__ part, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double acc = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) acc += part[(int64_t)ch * m + c];
  out[c] = acc;
}

template <typename T>
int col_dots(hipStream_t s, int64_t n, int m, const T* Y, const T* Q, double* out, double* partial) {
  const int nchunk = (int)((n + RES_ROWS - 1) / RES_ROWS);
  hipLaunchKernelGGL((k_coldot_partial<T>), dim3((m + 255) / 256, nchunk), dim3(256), 0, s, n, m, Y, Q, partial);
  hipLaunchKernelGGL(k_coldot_final, dim3((m + 255) / 256), dim3(256), 0, s, m, nchunk, partial, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
// Block copies for the deflated reduced eigensolve.  dst (rows x cols) = src, or with
// conj_t, dst (cols x rows) = src^H.
template <typename T>
__global__ void k_copy_block(int rows, int cols, const T* __restrict__ src, int64_t lds, T* __restrict__ dst,
                             int64_t ldd, int conj_t) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= cols) return;
  const T v = src[(int64_t)r * lds + c];
  if (conj_t) dst[(int64_t)c * ldd + r] = conj(v);
  else dst[(int64_t)r * ldd + c] = v;
}

template <typename T>
int copy_block(hipStream_t s, int rows, int cols, const T* src, int64_t lds, T* dst, int64_t ldd, bool conj_t) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL((k_copy_block<T>), dim3((cols + 255) / 256, rows), dim3(256), 0, s, rows, cols, src, lds, dst,
                     ldd, conj_t ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// dst[i][j] = src[p[i]][p[j]] (m x m, both with leading dimension m)
template <typename T>
__global__ void k_sym_permute(int m, const T* __restrict__ src, const int* __restrict__ p, T* __restrict__ dst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m) return;
  dst[(int64_t)i * m + j] = src[(int64_t)p[i] * m + p[j]];
}

template <typename T>
int sym_permute(hipStream_t s, int m, const T* src, const int* p, T* dst) {
  if (m <= 0) return 0;
  hipLaunchKernelGGL((k_sym_permute<T>), dim3((m + 255) / 256, m), dim3(256), 0, s, m, src, p, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// dst[p[r]][:] = src[r][:] (rows x cols, leading dimension cols)
template <typename T>
__global__ void k_scatter_rows(int rows, int cols, const T* __restrict__ src, const int* __restrict__ p,
                               T* __restrict__ dst) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (c >= cols) return;
  dst[(int64_t)p[r] * cols + c] = src[(int64_t)r * cols + c];
}

template <typename T>
int scatter_rows(hipStream_t s, int rows, int cols, const T* src, const int* p, T* dst) {
  if (rows <= 0 || cols <= 0) return 0;
  hipLaunchKernelGGL((k_scatter_rows<T>), dim3((cols + 255) / 256, rows), dim3(256), 0, s, rows, cols, src, p, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

#define MF_RR_INST(T)                                                                                          \
  template int col_absmax<T>(hipStream_t, int64_t, int, const T*, int64_t, double*);                           \
  template int gram_equilibrate<T>(hipStream_t, int, T*, T*, double*, int*);                                   \
  template int jacobi_eigh<T>(hipStream_t, int, T*, T*, double*, int*, double*, double);                               \
  template int gather_scale_cols<T>(hipStream_t, int, int, const T*, int, const int*, const double*, T*, int); \
  template int scale_rows_permute_cols<T>(hipStream_t, int, int, const T*, int, const double*, const int*, T*, \
                                          int);                                                                \
  template int residual_norms<T>(hipStream_t, int64_t, int, const T*, const T*, const double*, T*, double*,    \
                                 double*, double*);                                                            \
  template int copy_rm_to_cm<T>(hipStream_t, int64_t, int, const T*, int64_t, T*, int64_t, const int*);        \
  template int copy_cm_to_rm<T>(hipStream_t, int64_t, int, const T*, int64_t, T*, int64_t);                    \
  template int random_block<T>(hipStream_t, int64_t, int, uint64_t, T*, int64_t);                            \
  template int rademacher_block<T>(hipStream_t, int64_t, int, uint64_t, T*, int64_t);                        \
  template int col_dots<T>(hipStream_t, int64_t, int, const T*, const T*, double*, double*);                  \
  template int hermitian_part<T>(hipStream_t, int, T*);                                                     \
  template int copy_block<T>(hipStream_t, int, int, const T*, int64_t, T*, int64_t, bool);                     \
  template int sym_permute<T>(hipStream_t, int, const T*, const int*, T*);                                    \
  template int scatter_rows<T>(hipStream_t, int, int, const T*, const int*, T*);

MF_RR_INST(double)
MF_RR_INST(c64)

}  // namespace mf
