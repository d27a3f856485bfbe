// Non-Hermitian FEAST for dense complex general pencils (the guide's Section 3.3).
//
// Eigenpairs of A x = lambda B x (A, B complex general, B = I allowed) with lambda inside a
// full contour: an ellipse centred at Emid with horizontal radius r, axis ratio
// fpm(18)/100 and rotation fpm(19) degrees, sampled at fpm(8) nodes (trapezoidal, the
// non-Hermitian default fpm(16) = 1, or Gauss fpm(16) = 0).  One call runs:
//   factor    F_j = (z_j B - A)^H for every node, blocked LU (the Hermitian kernels read a
//             column-major matrix as its conjugate transpose, so F_j is formed with the
//             conjugate nodes and coalesced loads); right solves M_j x = b use the
//             conjugate-transpose sweeps of F_j, left solves M_j^H y = b its forward sweeps
//             (RCI cases 10/11/20/21 with one factorization per node)
//   contour   iteration 0: Q = sum_j w_j M_j^-1 B Y, Q~ = sum_j conj(w_j) M_j^-H B^H Y~;
//             iteration k > 0: the residual form with R = A X - B X Lambda and
//             R~ = A^H Y - B^H Y conj(Lambda): Q = X rho(Lambda) + sum_j w_j M_j^-1 R
//             (z_j - Lambda)^-1, and the conjugate form for Q~
//   RR        equilibrated, rank-truncated orthonormal bases of Q and Q~ (Cholesky of the
//             Gram matrix with column drops, then Newton-Schulz), the reduced pencil
//             Aq = Q~^H A Q, Bq = Q~^H B Q (two-sided, fpm(15) = 0; Q~ = Q one-sided,
//             fpm(15) = 1), its eigenvalues and right and left eigenvectors on the device
//             (nh_eigensolve: Newton-Schulz inverse of Bq and GEMMs, Householder Hessenberg
//             form and windowed shifted QR in one workgroup, triangular eigenvectors one
//             workgroup per eigenvalue), X = Q W (unit columns), Y = Q~ W~ (y_i^H B x_i = 1)
//   stop      M = #lambda inside the ellipse; residuals ||A x - lambda B x|| / ||alpha B x||
//             and ||A^H y - conj(lambda) B^H y|| / ||alpha B^H y||, alpha = |Emid| + r;
//             epsout = |trace_k - trace_{k-1}| / alpha (Table tab-common2).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <limits>
#include <vector>

#include "../../include/mfeast.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace mf;

namespace {

constexpr int NH_MAX_M0 = 512;  // the Schur form of the reduced problem runs in one workgroup
constexpr int NH_THREADS = 256;
constexpr double NH_SPURIOUS_RES = 1.0e-1;
// nominal work of the Schur form and the eigenvectors of the triangular factor of an
// order-m matrix, in flops per m^3 (a complex nonsymmetric eigensolve with vectors: four
// times the usual 25 m^3 real count); the GEMMs around it count their own flops
constexpr double NH_SCHUR_FLOPS = 100.0;

// ---------------------------------------------------------------------------
// full contour: z(theta) = emid + e^{i phi} (r cos theta + i e r sin theta), theta in
// [0, 2 pi); (1/2 pi i) z' dtheta = (1/2 pi) e^{i phi} (e r cos theta + i r sin theta) dtheta
void gauss_legendre_nodes(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      pp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    pp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

bool gauss_full_allowed(int ne) { return (ne >= 2 && ne <= 40) || ne == 48 || ne == 64 || ne == 80 || ne == 96 || ne == 112; }

void full_contour(std::complex<double> emid, double r, int ne, int rule, int ratio_pct, int angle_deg,
                  std::vector<std::complex<double>>& z, std::vector<std::complex<double>>& w) {
  const double e = ratio_pct / 100.0;
  const std::complex<double> rot = std::polar(1.0, angle_deg * M_PI / 180.0);
  std::vector<double> x, om;
  if (rule == 0) gauss_legendre_nodes(ne, x, om);
  z.resize(ne);
  w.resize(ne);
  for (int j = 0; j < ne; ++j) {
    double th, sc;
    if (rule == 0) {
      th = M_PI * (1.0 + x[j]);
      sc = om[j] / 2.0;
    } else {
      th = 2.0 * M_PI * (j + 0.5) / ne;
      sc = 1.0 / ne;
    }
    z[j] = emid + rot * std::complex<double>(r * std::cos(th), e * r * std::sin(th));
    w[j] = sc * rot * std::complex<double>(e * r * std::cos(th), r * std::sin(th));
  }
}

bool inside_ellipse(std::complex<double> l, std::complex<double> emid, double r, int ratio_pct, int angle_deg) {
  const std::complex<double> u = std::polar(1.0, -angle_deg * M_PI / 180.0) * (l - emid);
  const double e = ratio_pct / 100.0;
  const double a = u.real() / r, b = u.imag() / (e * r);
  return a * a + b * b <= 1.0;
}

// ---------------------------------------------------------------------------
// right-hand sides of both directions: Wc_j (right, conjugate-transpose sweeps of F_j,
// unpermuted) from rhsR, Wf_j (left, forward sweeps, rows gathered with perm_j) from rhsL
template <typename C>
__global__ void k_rhs_two(int64_t n, int m, const c64* __restrict__ rhsR, const c64* __restrict__ rhsL,
                          const double* __restrict__ csR, const double* __restrict__ csL, int ne,
                          const int* __restrict__ perm, C* __restrict__ Wf, C* __restrict__ Wc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= m) return;
  const int64_t blk = n * (int64_t)m;
  const C vr = convert<C, c64>(csR[c] * rhsR[i * m + c]);
  for (int j = 0; j < ne; ++j) Wc[j * blk + i * m + c] = vr;
  if (Wf != nullptr)
    for (int j = 0; j < ne; ++j) {
      const int64_t src = perm[(int64_t)j * n + i];
      Wf[j * blk + i * m + c] = convert<C, c64>(csL[c] * rhsL[src * m + c]);
    }
}

// Q[r][c] = [resid: rho_c X[r][c]] + usR_c sum_j cR[j][c] Wc_j[perm_inv_j[r]][c];
// QL[r][c] = [resid: conj(rho_c) XL[r][c]] + usL_c sum_j cL[j][c] Wf_j[r][c]
template <typename C>
__global__ void k_accumulate_two(int64_t n, int m, int ne, const C* __restrict__ Wf, const C* __restrict__ Wc,
                                 const int* __restrict__ perm_inv, const c64* __restrict__ cR,
                                 const c64* __restrict__ cL, const c64* __restrict__ rho,
                                 const double* __restrict__ usR, const double* __restrict__ usL,
                                 const c64* __restrict__ X, const c64* __restrict__ XL, c64* __restrict__ Q,
                                 c64* __restrict__ QL, int resid) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = blockIdx.y;
  if (c >= m) return;
  const int64_t blk = n * (int64_t)m;
  c64 a(0.0, 0.0), b(0.0, 0.0);
  for (int j = 0; j < ne; ++j) {
    const int64_t rr = perm_inv[(int64_t)j * n + r];
    a = a + cR[(int64_t)j * m + c] * convert<c64, C>(Wc[j * blk + rr * m + c]);
    if (Wf != nullptr) b = b + cL[(int64_t)j * m + c] * convert<c64, C>(Wf[j * blk + r * m + c]);
  }
  a = usR[c] * a;
  if (resid) a = a + rho[c] * X[r * m + c];
  Q[r * m + c] = a;
  if (Wf != nullptr) {
    b = usL[c] * b;
    if (resid) b = b + conj(rho[c]) * XL[r * m + c];
    QL[r * m + c] = b;
  }
}

// R = AX - BX diag(lam) (conj(lam) with conj_lam), column sums of |R|^2 and |BX|^2 in
// 256-row chunks, then one ordered sum per column
constexpr int NH_ROWS = 256;
__global__ void k_nh_resid_partial(int64_t n, int m, const c64* __restrict__ AX, const c64* __restrict__ BX,
                                   const c64* __restrict__ lam, int conj_lam, c64* __restrict__ R,
                                   double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  const c64 l = conj_lam ? conj(lam[c]) : lam[c];
  double sr = 0.0, sb = 0.0;
  const int64_t r1 = ((chunk + 1) * NH_ROWS < n) ? (chunk + 1) * NH_ROWS : n;
  for (int64_t r = chunk * NH_ROWS; r < r1; ++r) {
    const c64 bx = BX[r * m + c];
    const c64 v = AX[r * m + c] - l * bx;
    R[r * m + c] = v;
    sr += norm2(v);
    sb += norm2(bx);
  }
  const int64_t nchunk = gridDim.y;
  part[chunk * m + c] = sr;
  part[(nchunk + chunk) * m + c] = sb;
}

__global__ void k_nh_resid_final(int m, int nchunk, const double* __restrict__ part, double* __restrict__ rn2,
                                 double* __restrict__ bn2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double a = 0.0, b = 0.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    a += part[(int64_t)ch * m + c];
    b += part[(int64_t)(nchunk + ch) * m + c];
  }
  rn2[c] = a;
  bn2[c] = b;
}

int nh_resid(hipStream_t s, int64_t n, int m, const c64* AX, const c64* BX, const c64* lam, bool conj_lam, c64* R,
             double* rn2, double* bn2, double* part) {
  const int nchunk = (int)((n + NH_ROWS - 1) / NH_ROWS);
  hipLaunchKernelGGL(k_nh_resid_partial, dim3((m + 255) / 256, nchunk), dim3(256), 0, s, n, m, AX, BX, lam,
                     conj_lam ? 1 : 0, R, part);
  hipLaunchKernelGGL(k_nh_resid_final, dim3((m + 255) / 256), dim3(256), 0, s, m, nchunk, part, rn2, bn2);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// dst = conj(src), count elements
__global__ void k_conj(int64_t count, const c64* __restrict__ src, c64* __restrict__ dst) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < count) dst[e] = conj(src[e]);
}

// dst (rows x k) = src[:, 0:k] with the leading dimension changed
__global__ void k_take_cols(int rows, int k, const c64* __restrict__ src, int lds, c64* __restrict__ dst) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (c >= k) return;
  dst[(int64_t)i * k + c] = src[(int64_t)i * lds + c];
}

// ---------------------------------------------------------------------------
// The reduced non-Hermitian pencil (Aq, Bq), order m <= NH_MAX_M0, in four stages:
//   1. Binv = Bq^-1 by the Newton-Schulz iteration X <- X (2I - Bq X) from
//      X0 = Bq^H / (||Bq||_1 ||Bq||_inf) (FP64 GEMMs), then C = Binv Aq
//   2. Householder reduction of C to Hessenberg form (Z accumulated; three launches per
//      column: the reflector, the update from the left over column blocks, the update
//      from the right over row blocks of H and Z), then, in one workgroup, shifted QR
//      with Wilkinson shifts to the Schur form T = Z^H C Z: each sweep chases its bulge
//      through windows of QW rotations held in LDS by one wavefront, and the rest of H
//      and Z receives each window's rotations from all threads afterwards
//   3. eigenvectors of the triangular T (one workgroup per eigenvalue): right V (upper),
//      left U (lower, u^H T = lambda u^H)
//   4. W = Z V (unit columns); left: WL = Binv^H Z U scaled so that wl^H Bq w = 1
__device__ inline double cabs(c64 a) { return hypot(a.re, a.im); }

__device__ inline c64 csqrt(c64 z) {
  const double r = cabs(z);
  if (r == 0.0) return c64(0.0, 0.0);
  if (z.re >= 0.0) {
    const double t = sqrt(0.5 * (r + z.re));
    return c64(t, z.im / (2.0 * t));
  }
  const double t = sqrt(0.5 * (r - z.re));
  return c64(fabs(z.im) / (2.0 * t), copysign(t, z.im));
}

template <int NT>
__device__ inline double block_sum(double v, double* red_v) {
  const int tid = threadIdx.x;
  red_v[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red_v[tid] += red_v[tid + s];
    __syncthreads();
  }
  const double r = red_v[0];
  __syncthreads();
  return r;
}

template <int NT>
__device__ inline int block_max_int(int v, int* red_i) {
  const int tid = threadIdx.x;
  red_i[tid] = v;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) red_i[tid] = max(red_i[tid], red_i[tid + s]);
    __syncthreads();
  }
  const int r = red_i[0];
  __syncthreads();
  return r;
}

// ---- stage 1: Newton-Schulz inverse
// X0 = Bq^H / (max column sum * max row sum of |Bq|) (one workgroup)
__global__ __launch_bounds__(NH_THREADS) void k_ns_init(int m, const c64* __restrict__ B, c64* __restrict__ X) {
  __shared__ double red_v[NH_THREADS];
  __shared__ double s_alpha;
  const int tid = threadIdx.x;
  double cmax = 0.0, rmax = 0.0;
  for (int j = tid; j < m; j += NH_THREADS) {
    double cs = 0.0, rs = 0.0;
    for (int i = 0; i < m; ++i) {
      cs += cabs(B[(int64_t)i * m + j]);
      rs += cabs(B[(int64_t)j * m + i]);
    }
    cmax = fmax(cmax, cs);
    rmax = fmax(rmax, rs);
  }
  red_v[tid] = cmax;
  __syncthreads();
  for (int s = NH_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red_v[tid] = fmax(red_v[tid], red_v[tid + s]);
    __syncthreads();
  }
  const double c1 = red_v[0];
  __syncthreads();
  red_v[tid] = rmax;
  __syncthreads();
  for (int s = NH_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red_v[tid] = fmax(red_v[tid], red_v[tid + s]);
    __syncthreads();
  }
  if (tid == 0) s_alpha = (c1 > 0.0 && red_v[0] > 0.0) ? 1.0 / (c1 * red_v[0]) : 0.0;
  __syncthreads();
  const double al = s_alpha;
  for (int64_t e = tid; e < (int64_t)m * m; e += NH_THREADS) {
    const int i = (int)(e / m), j = (int)(e % m);
    X[e] = al * conj(B[(int64_t)j * m + i]);
  }
}

// T <- 2I - T in place, and per-workgroup partial sums of ||I - T||_F^2 (T = Bq X on entry)
constexpr int NS_BLOCKS = 64;
__global__ void k_ns_step(int m, c64* __restrict__ T, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t mm = (int64_t)m * m;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < mm; e += (int64_t)gridDim.x * 256) {
    const int i = (int)(e / m), j = (int)(e % m);
    const c64 t = T[e];
    const c64 r = c64((i == j ? 1.0 : 0.0) - t.re, -t.im);
    acc += norm2(r);
    T[e] = c64((i == j ? 2.0 : 0.0) - t.re, -t.im);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// ---- stage 2: Hessenberg form and windowed shifted QR (one workgroup)
constexpr int QW = 20;       // rotations per window
constexpr int QR_THREADS = 512;
constexpr int QS = QW + 3;   // window order: the bulge column, QW rotation pairs, one more row

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// ---- Householder reduction to upper Hessenberg form, column k
// the reflector I - beta v v^H mapping H[k+1.., k] to alpha e_1: v (entries k+1..m-1) and beta
// to vb (vb[m] holds beta in its real part); column k of H set to its final value
__global__ __launch_bounds__(256) void k_hess_vec(int m, int k, c64* __restrict__ H, c64* __restrict__ vb) {
  __shared__ double red_v[256];
  const int tid = threadIdx.x;
  const c64 x0 = H[(int64_t)(k + 1) * m + k];
  double part = 0.0;
  for (int i = k + 1 + tid; i < m; i += 256) part += norm2(H[(int64_t)i * m + k]);
  const double xn2 = block_sum<256>(part, red_v);
  if (xn2 == 0.0) {
    for (int i = k + 1 + tid; i < m; i += 256) vb[i] = c64(0.0, 0.0);
    if (tid == 0) vb[m] = c64(0.0, 0.0);
    return;
  }
  const double ax0 = cabs(x0), xn = sqrt(xn2);
  const c64 ph = ax0 > 0.0 ? c64(x0.re / ax0, x0.im / ax0) : c64(1.0, 0.0);
  const c64 alpha = c64(-xn * ph.re, -xn * ph.im);
  const double vn2 = xn2 - ax0 * ax0 + norm2(x0 - alpha);
  for (int i = k + 1 + tid; i < m; i += 256) {
    vb[i] = (i == k + 1) ? x0 - alpha : H[(int64_t)i * m + k];
    H[(int64_t)i * m + k] = (i == k + 1) ? alpha : c64(0.0, 0.0);
  }
  if (tid == 0) vb[m] = c64(vn2 > 0.0 ? 2.0 / vn2 : 0.0, 0.0);
}

// from the left: columns k+1..m-1 (16 per workgroup), rows k+1..m-1
__global__ __launch_bounds__(256) void k_hess_left(int m, int k, c64* __restrict__ H, const c64* __restrict__ vb) {
  __shared__ c64 red[256];
  const double beta = vb[m].re;
  if (beta == 0.0) return;
  const int tc = threadIdx.x % 16, tr = threadIdx.x / 16;
  const int c = k + 1 + blockIdx.x * 16 + tc;
  c64 acc(0.0, 0.0);
  if (c < m)
    for (int i = k + 1 + tr; i < m; i += 16) acc = acc + conj(vb[i]) * H[(int64_t)i * m + c];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st >= 16; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + st];
    __syncthreads();
  }
  const c64 w = beta * red[tc];
  if (c < m)
    for (int i = k + 1 + tr; i < m; i += 16) H[(int64_t)i * m + c] = H[(int64_t)i * m + c] - vb[i] * w;
}

// from the right: rows of H (0..m-1) and of Z (m..2m-1), 16 per workgroup, columns k+1..m-1
__global__ __launch_bounds__(256) void k_hess_right(int m, int k, c64* __restrict__ H, c64* __restrict__ Z,
                                                    const c64* __restrict__ vb) {
  const double beta = vb[m].re;
  if (beta == 0.0) return;
  const int tc = threadIdx.x % 16, tr = threadIdx.x / 16;
  const int r = blockIdx.x * 16 + tr;
  if (r >= 2 * m) return;
  c64* row = (r < m ? H + (int64_t)r * m : Z + (int64_t)(r - m) * m);
  c64 acc(0.0, 0.0);
  for (int c = k + 1 + tc; c < m; c += 16) acc = acc + row[c] * vb[c];
  for (int o = 8; o > 0; o >>= 1) {
    acc.re += __shfl_xor(acc.re, o, 16);
    acc.im += __shfl_xor(acc.im, o, 16);
  }
  const c64 t = beta * acc;
  for (int c = k + 1 + tc; c < m; c += 16) row[c] = row[c] - t * conj(vb[c]);
}

__global__ void k_eye(int m, c64* __restrict__ Z) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= (int64_t)m * m) return;
  Z[e] = c64(e / m == e % m ? 1.0 : 0.0, 0.0);
}

// A window's rotations applied to one segment v[0..nrot] (loaded by the caller): rotation r
// acts as [c s; -conj(s) c] on (v_r, v_r+1), with s replaced by conj(s) for a column segment
// (rotations applied from the right)
__device__ inline void qr_rotate_segment(c64 (&v)[QW + 1], int nrot, bool cols, const double* __restrict__ rc,
                                         const c64* __restrict__ rs) {
#pragma unroll
  for (int r = 0; r < QW; ++r) {
    // the rotations' LDS reads are issued four at a time (hoisting all of them would hold
    // 6 QW registers and spill)
    if ((r & 3) == 0) __asm__ volatile("" ::: "memory");
    if (r < nrot) {
      const double cc = rc[r];
      const c64 ss = cols ? conj(rs[r]) : rs[r];
      const c64 xa = v[r], yb = v[r + 1];
      v[r] = cc * xa + ss * yb;
      v[r + 1] = cc * yb - conj(ss) * xa;
    }
  }
}

// shifted QR: H (in: upper Hessenberg; out: the Schur form T, upper triangular), Z (in:
// the Hessenberg transform; out: C = Z T Z^H), both m x m row-major; tnorm: max |T_ij| over
// the upper triangle; flag 2 when the iteration does not converge within 40 m sweeps
__global__ __launch_bounds__(QR_THREADS) void k_nh_qr(int m, c64* __restrict__ H, c64* __restrict__ Z,
                                                      double* __restrict__ tnorm, int* __restrict__ flag) {
  __shared__ double red_v[QR_THREADS];
  __shared__ int red_i[QR_THREADS];
  __shared__ c64 sH[2][QS * QS];
  __shared__ c64 sF[2][QS * QS];  // next block's entries from H, staged by wavefronts 1..7
  __shared__ double s_rc[2][QW];
  __shared__ c64 s_rs[2][QW];
  __shared__ c64 s_mu;
  const int tid = threadIdx.x;
  const double eps = 2.220446049250313e-16;
  if (tid == 0) *flag = 0;
  // ---- shifted QR on the active block [lo, hi]
  int hi = m - 1, its = 0, total = 0;
  while (hi >= 1) {
    // lo: the largest l <= hi with a negligible subdiagonal entry H[l][l-1] (0 if none)
    int cand = 0;
    for (int l = 1 + tid; l <= hi; l += QR_THREADS) {
      const double sub = cabs(H[(int64_t)l * m + l - 1]);
      const double dsum = cabs(H[(int64_t)l * m + l]) + cabs(H[(int64_t)(l - 1) * m + l - 1]);
      if (sub <= eps * dsum || sub < 1e-300) cand = l;
    }
    const int lo = block_max_int<QR_THREADS>(cand, red_i);
    if (lo >= 1 && tid == 0) H[(int64_t)lo * m + lo - 1] = c64(0.0, 0.0);
    if (lo == hi) {
      __syncthreads();
      --hi;
      its = 0;
      continue;
    }
    if (++total > 40 * m) {
      if (tid == 0) *flag = 2;
      return;
    }
    ++its;
    if (tid == 0) {
      c64 mu;
      const c64 a = H[(int64_t)(hi - 1) * m + hi - 1], b = H[(int64_t)(hi - 1) * m + hi];
      const c64 c = H[(int64_t)hi * m + hi - 1], d = H[(int64_t)hi * m + hi];
      if (its % 11 == 10) {
        // exceptional shift after a run of slow iterations
        mu = d + c64(0.75 * cabs(c), 0.0);
      } else {
        const c64 half(0.5 * (a.re - d.re), 0.5 * (a.im - d.im));
        const c64 disc = csqrt(half * half + b * c);
        const c64 m1 = c64(0.5 * (a.re + d.re), 0.5 * (a.im + d.im)) + disc;
        const c64 m2 = c64(0.5 * (a.re + d.re), 0.5 * (a.im + d.im)) - disc;
        mu = cabs(m1 - d) <= cabs(m2 - d) ? m1 : m2;
      }
      s_mu = mu;
    }
    __syncthreads();
    const c64 mu = s_mu;
    // The sweep in windows of QW rotations.  Phase p: wavefront 0 chases window p inside
    // its LDS block while the other wavefronts apply window p - 1's rotations to the rest of
    // H and Z; one barrier per phase.  Window p's block needs window p - 1's row rotations
    // on the columns it adds to the right (rows k0_{p-1}..k0_p of columns e_{p-1}+1..e_p):
    // wavefront 0 applies those itself first, and the other wavefronts leave them out.
    const int nwin = (hi - lo + QW - 1) / QW;
    constexpr int NQ = (QS * QS + 63) / 64;  // block entries per lane
    for (int p = 0; p <= nwin; ++p) {
      const int buf = p & 1;
      if (tid < 64) {
        if (p < nwin) {
          const int lane = tid;
          const int k0 = lo + p * QW;
          const int kend = min(k0 + QW, hi);
          const int nrot = kend - k0;
          const int a = (p == 0) ? lo : k0 - 1;
          const int e = min(hi, k0 + QW + 1);
          const int sz = e - a + 1;
          c64* __restrict__ S = sH[buf];
          if (p == 0) {
            c64 g[NQ];
#pragma unroll
            for (int t = 0; t < NQ; ++t) {
              const int q = lane + 64 * t;
              const int i = q / QS, j = q % QS;
              g[t] = (q < QS * QS && i < sz && j < sz) ? H[(int64_t)(a + i) * m + a + j] : c64(0.0, 0.0);
            }
#pragma unroll
            for (int t = 0; t < NQ; ++t)
              if (lane + 64 * t < QS * QS) S[lane + 64 * t] = g[t];
          } else {
            // the previous window is a full one: rows pk0..k0 rotated, block [pa, pe].  The new
            // block takes its top-left 3 x 3 from the previous block, rows k0-1 and k0 of the
            // columns right of pe from the catch-up (those columns' rows pk0..k0 receive the
            // previous window's row rotations here: the other wavefronts leave them out), and
            // the rest from H (staged in LDS by the other wavefronts in the previous phase).
            const int pk0 = k0 - QW, pe = k0 + 1;
            const int pa = (p == 1) ? lo : pk0 - 1;
            const c64* __restrict__ P = sH[buf ^ 1];
            const int ncu = e - pe;  // catch-up columns pe+1..e (at most QW), one per lane
#pragma unroll
            for (int t = 0; t < NQ; ++t) {
              const int q = lane + 64 * t;
              const int i = q / QS, j = q % QS;
              const int gi = a + i, gj = a + j;
              if (q < QS * QS) {
                if (!(i < sz && j < sz)) S[q] = c64(0.0, 0.0);
                else if (gi <= pe && gj <= pe) S[q] = P[(gi - pa) * QS + (gj - pa)];
                else if (!(gj > pe && gi <= k0)) S[q] = sF[buf][q];
              }
            }
            const int col = pe + 1 + lane;
            c64 v[QW + 1];
            if (lane < ncu) {
#pragma unroll
              for (int q = 0; q <= QW; ++q) v[q] = H[(int64_t)(pk0 + q) * m + col];
            }
            if (lane < ncu) {
              qr_rotate_segment(v, QW, false, s_rc[buf ^ 1], s_rs[buf ^ 1]);
              // rows pk0..k0-2 are done for this window; rows a = k0-1 and k0 go into the
              // block (written back with it)
#pragma unroll
              for (int q = 0; q < QW - 1; ++q) H[(int64_t)(pk0 + q) * m + col] = v[q];
              S[col - a] = v[QW - 1];
              S[QS + col - a] = v[QW];
            }
          }
          wave_sync();
          // the chase inside the window: per rotation one round of LDS reads, the rotation
          // (computed by every lane), one pair update per lane and one round of writes.
          // Lanes 0-31 update rows kl, kl+1 at column c0l + lane (the row rotation; columns kl
          // and kl+1 excluded), lanes 32-63 columns kl, kl+1 at row lane - 32 (the column
          // rotation, rows i <= k+2; rows kl and kl+1 start from the row-rotated 2 x 2 block).
          const bool rowl = lane < 32;
          const int hl = lane & 31;
          for (int r = 0; r < nrot; ++r) {
            const int k = k0 + r, kl = k - a;
            const int c0l = (k == lo) ? kl : kl - 1;
            const int rmax = min(k + 2, hi) - a;
            const int j = c0l + hl;  // row lanes: column
            const int i = hl;        // column lanes: row
            const c64 x = (k == lo) ? S[kl * QS + kl] - mu : S[kl * QS + kl - 1];
            const c64 y = (k == lo) ? S[(kl + 1) * QS + kl] : S[(kl + 1) * QS + kl - 1];
            const c64 b00 = S[kl * QS + kl], b01 = S[kl * QS + kl + 1];
            const c64 b10 = S[(kl + 1) * QS + kl], b11 = S[(kl + 1) * QS + kl + 1];
            const int jc = min(j, QS - 1), ic = min(i, QS - 1);
            const int ua = rowl ? kl * QS + jc : ic * QS + kl;
            const int wa = rowl ? (kl + 1) * QS + jc : ic * QS + kl + 1;
            c64 u = S[ua], w = S[wa];
            // G = [c s; -conj(s) c] with G [x; y] = [r; 0], c real
            const double ax2 = norm2(x), ay2 = norm2(y);
            double cc;
            c64 ss;
            if (ay2 == 0.0) {
              cc = 1.0;
              ss = c64(0.0, 0.0);
            } else if (ax2 == 0.0) {
              const double iy = 1.0 / sqrt(ay2);
              cc = 0.0;
              ss = c64(y.re * iy, -y.im * iy);
            } else {
              // c = |x| / r, s = x conj(y) / (|x| r), r = sqrt(|x|^2 + |y|^2): the two square
              // roots side by side, then one division
              const double ax = sqrt(ax2);
              const double rr = sqrt(ax2 + ay2);
              const double f = 1.0 / (ax * rr);
              cc = ax2 * f;
              ss = c64(f * (x.re * y.re + x.im * y.im), f * (x.im * y.re - x.re * y.im));
            }
            if (lane == 0) {
              s_rc[buf][r] = cc;
              s_rs[buf][r] = ss;
            }
            // column lanes of rows kl, kl+1: the row-rotated block, row kl = (c b00 + s b10,
            // c b01 + s b11), row kl+1 = (c b10 - conj(s) b00, c b11 - conj(s) b01)
            const bool top = (i == kl);
            const c64 tm = top ? ss : c64(-ss.re, ss.im);  // s, or -conj(s)
            const c64 p1 = top ? b00 : b10, q1 = top ? b10 : b00;
            const c64 p2 = top ? b01 : b11, q2 = top ? b11 : b01;
            if (!rowl && (i == kl || i == kl + 1)) {
              u = cc * p1 + tm * q1;
              w = cc * p2 + tm * q2;
            }
            // row lanes rotate by [c s; -conj(s) c], column lanes by [c conj(s); -s c]
            const c64 t = rowl ? ss : conj(ss);
            const c64 un = cc * u + t * w;
            const c64 wn = cc * w - conj(t) * u;
            const bool act = rowl ? (j < sz && j != kl && j != kl + 1) : (i <= rmax);
            if (act) {
              S[ua] = un;
              S[wa] = wn;
            }
            wave_sync();
          }
          // the block back to H
          for (int q = lane; q < sz * sz; q += 64) {
            const int i = q / sz, j = q % sz;
            H[(int64_t)(a + i) * m + a + j] = S[i * QS + j];
          }
        }
      } else {
        if (p + 1 < nwin) {
          // the entries of window p+1's block that come from H (rows k0n+1 and below, past the
          // columns its top-left 3 x 3 and its catch-up cover; none of them changes before that
          // block is formed), staged in LDS for wavefront 0
          const int k0n = lo + (p + 1) * QW, an = k0n - 1, pen = k0n + 1;
          const int szn = min(hi, k0n + QW + 1) - an + 1;
          for (int q = tid - 64; q < QS * QS; q += QR_THREADS - 64) {
            const int i = q / QS, j = q % QS;
            const int gi = an + i, gj = an + j;
            if (i < szn && j < szn && !(gi <= pen && gj <= pen) && !(gj > pen && gi <= k0n))
              sF[buf ^ 1][q] = H[(int64_t)gi * m + gj];
          }
        }
      }
      if (tid >= 64 && p >= 1) {
        // window p - 1's rotations on the rest (entries k0..kend of each segment): rows of the
        // columns right of its block (past the next block's columns), the rows above its block,
        // and every row of Z
        const int k0 = lo + (p - 1) * QW;
        const int kend = min(k0 + QW, hi);
        const int nrot = kend - k0;
        const int a = (p == 1) ? lo : k0 - 1;
        const int e = min(hi, k0 + QW + 1);
        const int cfirst = (p < nwin) ? min(hi, kend + QW + 1) + 1 : e + 1;
        const int ncol = m - cfirst, nabove = a;
        const int items = ncol + nabove + m;
        const int rb = buf ^ 1;
        for (int it = tid - 64; it < items; it += QR_THREADS - 64) {
          c64* M = H;
          int64_t base, stride;
          bool cols;
          if (it < ncol) {
            base = (int64_t)k0 * m + cfirst + it;
            stride = m;
            cols = false;
          } else {
            const bool isz = it >= ncol + nabove;
            const int i = isz ? it - ncol - nabove : it - ncol;
            if (isz) M = Z;
            base = (int64_t)i * m + k0;
            stride = 1;
            cols = true;
          }
          // unconditional loads of entries k0..k0+QW (clamped to kend), issued together
          c64 v[QW + 1];
#pragma unroll
          for (int q = 0; q <= QW; ++q) v[q] = M[base + (int64_t)min(q, nrot) * stride];
          qr_rotate_segment(v, nrot, cols, s_rc[rb], s_rs[rb]);
#pragma unroll
          for (int q = 0; q <= QW; ++q)
            if (q <= nrot) M[base + (int64_t)q * stride] = v[q];
        }
      }
      __syncthreads();
    }
  }
  double tn = 0.0;
  for (int64_t e = tid; e < (int64_t)m * m; e += QR_THREADS) {
    const int i = (int)(e / m), c = (int)(e % m);
    if (c >= i) tn = fmax(tn, cabs(H[e]));
  }
  red_v[tid] = tn;
  __syncthreads();
  for (int s = QR_THREADS / 2; s > 0; s >>= 1) {
    if (tid < s) red_v[tid] = fmax(red_v[tid], red_v[tid + s]);
    __syncthreads();
  }
  if (tid == 0) *tnorm = red_v[0];
}

// ---- stage 3: eigenvectors of the triangular T, one workgroup (one wavefront) per eigenvalue i:
// right V[:, i] (V[k][i] = 0 for k > i, V[i][i] = 1, back substitution upwards) and, with
// two, left U[:, i] (u^H (T - lambda_i I) = 0: u_k = 0 for k < i, u_i = 1, forward)
__global__ __launch_bounds__(64) void k_nh_trivec(int m, const c64* __restrict__ T, const double* __restrict__ tnorm,
                                                  int two, c64* __restrict__ lam, c64* __restrict__ V,
                                                  c64* __restrict__ U) {
  __shared__ c64 col[NH_MAX_M0];
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  const double small = fmax(2.220446049250313e-16 * (*tnorm), 1e-300);
  const c64 li = T[(int64_t)i * m + i];
  if (lane == 0) lam[i] = li;
  for (int k = lane; k < m; k += 64) col[k] = c64(k == i ? 1.0 : 0.0, 0.0);
  __syncthreads();
  for (int k = i - 1; k >= 0; --k) {
    c64 acc(0.0, 0.0);
    for (int l = k + 1 + lane; l <= i; l += 64) acc = acc + T[(int64_t)k * m + l] * col[l];
    for (int o = 32; o > 0; o >>= 1) {
      acc.re += __shfl_xor(acc.re, o);
      acc.im += __shfl_xor(acc.im, o);
    }
    c64 d = T[(int64_t)k * m + k] - li;
    if (cabs(d) < small) d = c64(small, 0.0);
    const c64 q = cdiv(acc, d);
    if (lane == 0) col[k] = c64(-q.re, -q.im);
    __syncthreads();
  }
  for (int k = lane; k < m; k += 64) V[(int64_t)k * m + i] = col[k];
  if (!two) return;
  __syncthreads();
  for (int k = lane; k < m; k += 64) col[k] = c64(k == i ? 1.0 : 0.0, 0.0);
  __syncthreads();
  // conj(u_k) = -sum_{l=i..k-1} conj(u_l) T[l][k] / (T[k][k] - lambda_i)
  for (int k = i + 1; k < m; ++k) {
    c64 acc(0.0, 0.0);
    for (int l = i + lane; l < k; l += 64) acc = acc + conj(col[l]) * T[(int64_t)l * m + k];
    for (int o = 32; o > 0; o >>= 1) {
      acc.re += __shfl_xor(acc.re, o);
      acc.im += __shfl_xor(acc.im, o);
    }
    c64 d = T[(int64_t)k * m + k] - li;
    if (cabs(d) < small) d = c64(small, 0.0);
    const c64 q = cdiv(acc, d);
    if (lane == 0) col[k] = conj(c64(-q.re, -q.im));
    __syncthreads();
  }
  for (int k = lane; k < m; k += 64) U[(int64_t)k * m + i] = col[k];
}

// ---- stage 4: unit columns of W; with two, WL[:, j] scaled so that wl_j^H (Bq w_j) = 1
// (BW = Bq W before the scaling of W)
__global__ void k_nh_normalize(int m, c64* __restrict__ W, const c64* __restrict__ BW, c64* __restrict__ WL, int two) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double nn = 0.0;
  for (int i = 0; i < m; ++i) nn += norm2(W[(int64_t)i * m + j]);
  const double f = nn > 0.0 ? 1.0 / sqrt(nn) : 1.0;
  for (int i = 0; i < m; ++i) W[(int64_t)i * m + j] = f * W[(int64_t)i * m + j];
  if (!two) return;
  c64 d(0.0, 0.0);
  for (int i = 0; i < m; ++i) d = d + conj(WL[(int64_t)i * m + j]) * BW[(int64_t)i * m + j];
  d = f * d;
  const c64 g = cabs(d) > 0.0 ? cdiv(c64(1.0, 0.0), conj(d)) : c64(1.0, 0.0);
  for (int i = 0; i < m; ++i) WL[(int64_t)i * m + j] = WL[(int64_t)i * m + j] * g;
}

// Reduced eigensolver workspace: Binv, X2, T (m x m each; T also holds U Z products), H,
// Z, V, U (m x m), part (>= NS_BLOCKS + 2 doubles, device), flag (device int).
struct NhEig {
  c64 *binv, *x2, *t, *h, *z, *v, *u;
  double* part;
  int* flag;
};

// eigenvalues lam (device, m), right eigenvectors W (unit columns) and, with two, left
// eigenvectors WL (wl_j^H Bq w_j = 1) of the pencil (Aq, Bq), all m x m row-major on the
// device; h_flag (host): 0, 1 (Bq numerically singular), 2 (QR did not converge).
// Host-synchronizing (the Newton-Schulz stop test).
int nh_eigensolve(hipStream_t s, int m, const c64* Aq, const c64* Bq, bool two, NhEig& w, c64* lam, c64* W,
                         c64* WL, int* h_flag) {
  *h_flag = 0;
  // ---- Bq^-1 by Newton-Schulz: stop when ||I - Bq X||_F has reached rounding level
  int tok0 = prof_begin(s);
  hipLaunchKernelGGL(k_ns_init, dim3(1), dim3(NH_THREADS), 0, s, m, Bq, w.binv);
  MF_HIP_CHECK(hipGetLastError());
  prof_end(tok0, s, K_EIG, 0.0, 0.0);
  const int nb = std::min(NS_BLOCKS, (int)(((int64_t)m * m + 255) / 256));
  std::vector<double> hp(nb);
  double prev = std::numeric_limits<double>::infinity();
  bool ok = false;
  for (int it = 0; it < 100; ++it) {
    MF_TRY(rm_gemm<c64>(s, m, m, m, Bq, m, false, false, w.binv, m, w.t, m, 1.0, 0.0, K_EIG));
    const int tk = prof_begin(s);
    hipLaunchKernelGGL(k_ns_step, dim3(nb), dim3(256), 0, s, m, w.t, w.part);
    MF_HIP_CHECK(hipGetLastError());
    prof_end(tk, s, K_EIG, 0.0, 0.0);
    MF_TRY(rm_gemm<c64>(s, m, m, m, w.binv, m, false, false, w.t, m, w.x2, m, 1.0, 0.0, K_EIG));
    std::swap(w.binv, w.x2);
    MF_HIP_CHECK(hipMemcpyAsync(hp.data(), w.part, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    double r2 = 0.0;
    for (int b = 0; b < nb; ++b) r2 += hp[b];
    const double r = std::sqrt(r2);
    if (!std::isfinite(r)) break;
    // the residual of the previous iterate; the new one is at least as good once it is small
    if (r < 64.0 * m * 2.220446049250313e-16 || (r < 1e-6 && r > 0.25 * prev)) {
      ok = true;
      break;
    }
    prev = r;
  }
  if (!ok) {
    *h_flag = 1;
    return 0;
  }
  // ---- C = Binv Aq, then the Schur form
  MF_TRY(rm_gemm<c64>(s, m, m, m, w.binv, m, false, false, Aq, m, w.h, m, 1.0, 0.0, K_EIG));
  int tok = prof_begin(s);
  hipLaunchKernelGGL(k_eye, dim3((unsigned)(((int64_t)m * m + 255) / 256)), dim3(256), 0, s, m, w.z);
  for (int k = 0; k + 2 < m; ++k) {
    hipLaunchKernelGGL(k_hess_vec, dim3(1), dim3(256), 0, s, m, k, w.h, w.x2);
    hipLaunchKernelGGL(k_hess_left, dim3((m - k - 1 + 15) / 16), dim3(256), 0, s, m, k, w.h, (const c64*)w.x2);
    hipLaunchKernelGGL(k_hess_right, dim3((2 * m + 15) / 16), dim3(256), 0, s, m, k, w.h, w.z, (const c64*)w.x2);
  }
  MF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_nh_qr, dim3(1), dim3(QR_THREADS), 0, s, m, w.h, w.z, w.part, w.flag);
  MF_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_nh_trivec, dim3(m), dim3(64), 0, s, m, w.h, w.part, two ? 1 : 0, lam, w.v, w.u);
  MF_HIP_CHECK(hipGetLastError());
  prof_end(tok, s, K_EIG, NH_SCHUR_FLOPS * (double)m * m * m, 0.0);
  // ---- W = Z V; left: WL = Binv^H (Z U); BW = Bq W
  MF_TRY(rm_gemm<c64>(s, m, m, m, w.z, m, false, false, w.v, m, W, m, 1.0, 0.0, K_EIG));
  if (two) {
    MF_TRY(rm_gemm<c64>(s, m, m, m, w.z, m, false, false, w.u, m, w.t, m, 1.0, 0.0, K_EIG));
    MF_TRY(rm_gemm<c64>(s, m, m, m, w.binv, m, true, true, w.t, m, WL, m, 1.0, 0.0, K_EIG));
    MF_TRY(rm_gemm<c64>(s, m, m, m, Bq, m, false, false, W, m, w.t, m, 1.0, 0.0, K_EIG));
  }
  tok = prof_begin(s);
  hipLaunchKernelGGL(k_nh_normalize, dim3((m + 63) / 64), dim3(64), 0, s, m, W, w.t, WL, two ? 1 : 0);
  MF_HIP_CHECK(hipGetLastError());
  prof_end(tok, s, K_EIG, 0.0, 0.0);
  MF_HIP_CHECK(hipMemcpyAsync(h_flag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  return 0;
}

// ---------------------------------------------------------------------------
// Orthonormal basis of the range of the n x m block Q (row-major): equilibrated Gram
// matrix, Cholesky with column drops, then one Newton-Schulz pass; returns the kept count
// and the m x kept transform T (Q T orthonormal).  Host-synchronizing (reads the drops).
struct Orth {
  c64 *S, *S2, *Linv, *H1, *V, *TG, *Tr;
  double* d;
  int* keep;
  int* flag;
  int* idx;
  double* part;
  double* bn;
};

int orthonormalize(hipStream_t s, int64_t n, int m, const c64* Q, Orth& o, int* h_keep, int* h_idx, double* h_scal,
                   int& kept) {
  MF_TRY(rm_gemm<c64>(s, m, m, (int)n, Q, m, true, true, Q, m, o.S, m));
  MF_HIP_CHECK(hipMemsetAsync(o.flag, 0, 16, s));
  const int tok = prof_begin(s);
  MF_TRY(gram_equilibrate<c64>(s, m, o.S, o.S2, o.d, o.flag));
  const double tau = 32.0 * m * 2.220446049250313e-16;
  MF_TRY(chol_drop<c64>(s, m, o.S, o.Linv, o.keep, tau, o.TG));
  prof_end(tok, s, K_ORTH, 0.0, 0.0);
  MF_HIP_CHECK(hipMemcpyAsync(h_keep, o.keep, m * sizeof(int), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipMemcpyAsync(h_scal, o.flag, sizeof(int), hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  int k = 0;
  for (int i = 0; i < m; ++i)
    if (h_keep[i]) h_idx[k++] = i;
  kept = k;
  if (k == 0) return 0;
  MF_HIP_CHECK(hipMemcpyAsync(o.idx, h_idx, k * sizeof(int), hipMemcpyHostToDevice, s));
  MF_TRY(build_h1<c64>(s, m, k, o.Linv, o.d, o.idx, o.H1));
  // second pass: S1 = (Q H1)^H (Q H1) = H1^H (Q^H Q) H1, from the Gram matrix of Q
  MF_TRY(rm_gemm<c64>(s, m, m, (int)n, Q, m, true, true, Q, m, o.S, m));
  MF_TRY(rm_gemm<c64>(s, m, k, m, o.S, m, false, false, o.H1, k, o.TG, k));
  MF_TRY(rm_gemm<c64>(s, k, k, m, o.H1, k, true, true, o.TG, k, o.S2, k));
  MF_TRY(hermitian_part<c64>(s, k, o.S2));
  MF_TRY(ns_invsqrt<c64>(s, k, o.S2, o.V, 3, o.TG));
  MF_TRY(hermitian_part<c64>(s, k, o.V));
  MF_TRY(rm_gemm<c64>(s, m, k, k, o.H1, k, false, false, o.V, k, o.Tr, k));
  return 0;
}

// ---------------------------------------------------------------------------
// Polynomial FEAST (Section 3.4): kernels of its driver
//
// F_j = P(z_j)^H = sum_k conj(z_j)^k A_k^H (Horner), row-major with row stride ld; the
// coefficient matrices are column-major, A_k at As + k lda n, read as their conjugate
// transposes (coalesced, as the shift-form kernel); zc holds the conjugate nodes
template <typename C>
__global__ void k_poly_form(int64_t n, int64_t ld, const c64* __restrict__ As, int64_t lda, int p,
                            const c64* __restrict__ zc, int ne, C* __restrict__ LU, int* __restrict__ perm) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= n) return;
  const int64_t mstride = lda * n;
  for (int j = 0; j < ne; ++j) {
    c64 acc = conj(As[(int64_t)p * mstride + i * lda + c]);
    for (int k = p - 1; k >= 0; --k) acc = acc * zc[j] + conj(As[(int64_t)k * mstride + i * lda + c]);
    LU[(int64_t)j * n * ld + i * ld + c] = convert<C, c64>(acc);
  }
  if (i == 0)
    for (int j = 0; j < ne; ++j) perm[(int64_t)j * n + c] = (int)c;
}

// companion linearization of sum_k lambda^k Aq_k (each m x m, row-major, Aq_k at Aq + k m m):
// L0 = [[0, I, ...], ..., [-Aq_0, ..., -Aq_(p-1)]], L1 = diag(I, ..., I, Aq_p), size p m
__global__ void k_companion(int m, int p, const c64* __restrict__ Aq, c64* __restrict__ L0, c64* __restrict__ L1) {
  const int pm = p * m;
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  const int row = blockIdx.y;
  if (col >= pm) return;
  const int bi = row / m, ri = row % m, bj = col / m, cj = col % m;
  c64 l0(0.0, 0.0), l1(0.0, 0.0);
  if (bi < p - 1) {
    if (bj == bi + 1 && ri == cj) l0 = c64(1.0, 0.0);
    if (bj == bi && ri == cj) l1 = c64(1.0, 0.0);
  } else {
    const c64 a = Aq[((int64_t)bj * m + ri) * m + cj];
    l0 = c64(-a.re, -a.im);
    if (bj == p - 1) l1 = Aq[((int64_t)p * m + ri) * m + cj];
  }
  L0[(int64_t)row * pm + col] = l0;
  L1[(int64_t)row * pm + col] = l1;
}

// Wsel (m x m) = first block rows of the selected eigenvector columns, unit columns
__global__ void k_first_block(int m, int pm, const c64* __restrict__ Wz, const int* __restrict__ sel,
                              c64* __restrict__ Wsel) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int s = sel[j];
  double nn = 0.0;
  for (int i = 0; i < m; ++i) nn += norm2(Wz[(int64_t)i * pm + s]);
  const double f = nn > 0.0 ? 1.0 / sqrt(nn) : 1.0;
  for (int i = 0; i < m; ++i) Wsel[(int64_t)i * m + j] = f * Wz[(int64_t)i * pm + s];
}

// R = sum_k lam^k AkX_k (AkX_k at AkX + k n m), column sums of |R|^2 and of |AkX_k|^2 per k,
// in 256-row chunks: part[(q nchunk + chunk) m + c], q = 0 for R, 1 + k for AkX_k
__global__ void k_poly_resid_partial(int64_t n, int m, int p, const c64* __restrict__ AkX, const c64* __restrict__ lam,
                                     c64* __restrict__ R, double* __restrict__ part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t chunk = blockIdx.y;
  if (c >= m) return;
  const int64_t nchunk = gridDim.y;
  const int64_t blk = n * (int64_t)m;
  const c64 l = lam[c];
  double sr = 0.0;
  double sk[9];
  for (int k = 0; k <= p; ++k) sk[k] = 0.0;
  const int64_t r1 = ((chunk + 1) * NH_ROWS < n) ? (chunk + 1) * NH_ROWS : n;
  for (int64_t r = chunk * NH_ROWS; r < r1; ++r) {
    c64 acc(0.0, 0.0), pw(1.0, 0.0);
    for (int k = 0; k <= p; ++k) {
      const c64 a = AkX[k * blk + r * m + c];
      sk[k] += norm2(a);
      acc = acc + pw * a;
      pw = pw * l;
    }
    R[r * m + c] = acc;
    sr += norm2(acc);
  }
  part[chunk * m + c] = sr;
  for (int k = 0; k <= p; ++k) part[((int64_t)(1 + k) * nchunk + chunk) * m + c] = sk[k];
}

__global__ void k_poly_resid_final(int m, int p, int nchunk, const double* __restrict__ part, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  for (int q = 0; q <= p + 1; ++q) {
    double a = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) a += part[((int64_t)q * nchunk + ch) * m + c];
    out[(int64_t)q * m + c] = a;
  }
}

constexpr int POLY_MAX_P = 8;

}  // namespace

// ---------------------------------------------------------------------------
template <typename C>
static int nh_run(mfeast_ctx* h, int64_t n, const c64* A, int64_t lda, const c64* B, int64_t ldb, int32_t* fpm,
                  double* epsout, int32_t* loop, std::complex<double> emid, double r, int32_t* m0p, double* E,
                  c64* Xu, int64_t ldx, int32_t* Mout, double* res_out, const std::vector<std::complex<double>>& z,
                  const std::vector<std::complex<double>>& w) {
  auto f = [&](int i) { return fpm[i - 1]; };
  hipStream_t s = h->stream;
  const int ne = (int)z.size();
  const int m0in = *m0p;
  int m0 = m0in;
  const bool two = f(15) == 0;
  const bool hasB = B != nullptr;
  const double alpha = std::abs(emid) + r;
  const double eps = std::pow(10.0, -f(3));
  const int64_t ld = lu_ld(n);
  const size_t szC = sizeof(C);
  const size_t blk = (size_t)n * m0 * sizeof(c64);
  const size_t sq = (size_t)m0 * m0 * sizeof(c64);
  Timer total_t, ph;
  total_t.start();
  double t_fact = 0, t_solve = 0, t_ax = 0, t_bx = 0, t_eig = 0;

  // ---- workspace
  C* LU = (C*)h->ws(S_LU, (size_t)ne * n * ld * szC);
  C* Dinv = (C*)h->ws(S_DINV, (size_t)ne * ((n + LU_NB - 1) / LU_NB) * 2 * LU_NB * LU_NB * szC);
  C* Pinv = (C*)h->ws(S_PANINV, (size_t)ne * panel_inverse_entries(n) * szC);
  int* ipiv = (int*)h->ws(S_IPIV, (size_t)ne * n * 4);
  int* perm = (int*)h->ws(S_PERM, (size_t)ne * n * 4);
  int* pinv = (int*)h->ws(S_PINV, (size_t)ne * n * 4);
  int* linfo = (int*)h->ws(S_INFO, (size_t)ne * 4 + 64);
  c64* zdev = (c64*)h->ws(S_Z, (size_t)ne * sizeof(c64));
  C* Wf = two ? (C*)h->ws(S_WF, (size_t)ne * n * m0 * szC) : nullptr;
  C* Wc = (C*)h->ws(S_WC, (size_t)ne * n * m0 * szC);
  C* Wy = (C*)h->ws(S_WY, (size_t)ne * n * m0 * szC);
  SolveSide<C> side{};
  bool two_streams = false;
  if (two && h->ensure_aux()) {
    C* Wy2 = (C*)h->ws(S_WY2, (size_t)ne * n * m0 * szC);
    if (!Wy2) return -2;
    side = SolveSide<C>{h->aux, h->ev_fork, h->ev_join, Wy2};
    two_streams = true;
  }
  c64* X = (c64*)h->ws(S_X, blk);
  c64* XL = (c64*)h->ws(S_NH_XL, blk);
  c64* Q = (c64*)h->ws(S_Q, blk);
  c64* QL = (c64*)h->ws(S_NH_QL, blk);
  c64* R = (c64*)h->ws(S_R, blk);
  c64* RL = (c64*)h->ws(S_NH_RL, blk);
  c64* AQ = (c64*)h->ws(S_AQ, blk);
  c64* BQ = hasB ? (c64*)h->ws(S_BQ, blk) : nullptr;
  c64* AhQ = two ? (c64*)h->ws(S_NH_AHQ, blk) : nullptr;
  c64* BhQ = (two && hasB) ? (c64*)h->ws(S_NH_BHQ, blk) : nullptr;
  c64* Qo = (c64*)h->ws(S_AX, blk);
  c64* QLo = two ? (c64*)h->ws(S_NH_QLO, blk) : nullptr;
  c64* AQo = (c64*)h->ws(S_BX, blk);
  c64* BQo = hasB ? (c64*)h->ws(S_NH_BQO, blk) : nullptr;
  c64* AhQo = two ? (c64*)h->ws(S_NH_AHQO, blk) : nullptr;
  c64* BhQo = (two && hasB) ? (c64*)h->ws(S_NH_BHQO, blk) : nullptr;
  c64* T3 = (c64*)h->ws(S_NH_T3, blk);  // A X, then A^H Y
  c64* T4 = (c64*)h->ws(S_NH_T4, blk);  // B X, then B^H Y
  c64* Aq = (c64*)h->ws(S_S, sq);
  c64* Bq = (c64*)h->ws(S_T, sq);
  c64* Wr = (c64*)h->ws(S_W, sq);
  c64* Wl = (c64*)h->ws(S_NH_WL, sq);
  c64* Gw = (c64*)h->ws(S_HW, 3 * sq);
  c64* Hw = (c64*)h->ws(S_V, sq);
  c64* Zw = (c64*)h->ws(S_G, sq);
  c64* Vw = (c64*)h->ws(S_C, sq);
  c64* Uw = (c64*)h->ws(S_Z2, sq);
  Orth orr{}, orl{};
  orr.S = (c64*)h->ws(S_NH_O1, sq);
  orr.S2 = (c64*)h->ws(S_NH_O2, sq);
  orr.Linv = (c64*)h->ws(S_NH_O3, sq);
  orr.H1 = (c64*)h->ws(S_NH_O4, sq);
  orr.V = (c64*)h->ws(S_NH_O5, sq);
  orr.TG = (c64*)h->ws(S_TG, std::max(3 * sq, (size_t)m0 * 32 * sizeof(c64)));
  orr.Tr = (c64*)h->ws(S_NH_TR, sq);
  orl = orr;
  orl.Tr = (c64*)h->ws(S_NH_TL, sq);
  const size_t nsmall = (size_t)m0 * 24 + (size_t)ne * m0 * 8 + 256;
  double* small = (double*)h->ws(S_SMALL, nsmall * sizeof(double));
  const int nchunk = (int)((n + 255) / 256);
  double* part = (double*)h->ws(S_PART, (size_t)nchunk * m0 * 2 * sizeof(double) + 64);
  char* hp = h->host(nsmall * sizeof(double) + 4096);
  if (!LU || !Dinv || !Pinv || !ipiv || !perm || !pinv || !linfo || !zdev || (two && !Wf) || !Wc || !Wy || !X ||
      !XL || !Q || !QL || !R || !RL || !AQ || (hasB && !BQ) || (two && !AhQ) || (two && hasB && !BhQ) || !Qo ||
      (two && !QLo) || !AQo || (hasB && !BQo) || (two && !AhQo) || (two && hasB && !BhQo) || !T3 || !T4 || !Aq ||
      !Bq || !Wr || !Wl || !Gw || !Hw || !Zw || !Vw || !Uw || !orr.S || !orr.S2 || !orr.Linv || !orr.H1 ||
      !orr.V || !orr.TG || !orr.Tr || !orl.Tr || !small || !part || !hp)
    return -2;
  // small device arrays and their pinned host mirrors (same offsets)
  auto dsl = [&](size_t off) { return small + off; };
  auto hsl = [&](size_t off) { return reinterpret_cast<double*>(hp) + off; };
  const size_t o_cs = 0, o_csl = m0, o_us = 2 * m0, o_usl = 3 * m0, o_rn = 4 * m0, o_bn = 5 * m0, o_rnl = 6 * m0,
               o_bnl = 7 * m0, o_lam = 8 * m0 /* 2 m0 */, o_rho = 10 * m0 /* 2 m0 */, o_keep = 12 * m0,
               o_idx = 13 * m0, o_keepl = 14 * m0, o_idxl = 15 * m0, o_d = 16 * m0, o_dl = 17 * m0,
               o_flag = 18 * m0, o_perm = 19 * m0, o_cR = 24 * (size_t)m0 /* 2 ne m0 */,
               o_cL = 24 * (size_t)m0 + 2 * (size_t)ne * m0 /* 2 ne m0 */;
  orr.d = dsl(o_d);
  orl.d = dsl(o_dl);
  orr.keep = (int*)dsl(o_keep);
  orl.keep = (int*)dsl(o_keepl);
  orr.idx = (int*)dsl(o_idx);
  orl.idx = (int*)dsl(o_idxl);
  orr.flag = orl.flag = (int*)dsl(o_flag);
  orr.part = orl.part = part;
  c64* d_lam = reinterpret_cast<c64*>(dsl(o_lam));
  c64* h_lam = reinterpret_cast<c64*>(hsl(o_lam));
  c64* d_rho = reinterpret_cast<c64*>(dsl(o_rho));
  c64* h_rho = reinterpret_cast<c64*>(hsl(o_rho));
  c64* d_cR = reinterpret_cast<c64*>(dsl(o_cR));
  c64* h_cR = reinterpret_cast<c64*>(hsl(o_cR));
  c64* d_cL = reinterpret_cast<c64*>(dsl(o_cL));
  c64* h_cL = reinterpret_cast<c64*>(hsl(o_cL));
  int* d_flag = (int*)dsl(o_flag);
  int* h_flag = (int*)hsl(o_flag);

  // ---- factorizations F_j = (z_j B - A)^H: the shift-form kernel reads a column-major
  //      matrix as its conjugate transpose, so it is given the conjugate nodes
  ph.start();
  {
    std::vector<c64> zc(ne);
    for (int j = 0; j < ne; ++j) zc[j] = c64(z[j].real(), -z[j].imag());
    MF_HIP_CHECK(hipMemcpyAsync(zdev, zc.data(), ne * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemsetAsync(linfo, 0, ne * 4, s));
    int tok = prof_begin(s);
    MF_TRY(shift_form<c64, C>(s, n, A, lda, B, ldb, zdev, ne, LU, perm));
    prof_end(tok, s, K_OTHER, 0.0, (double)n * n * ((hasB ? 2.0 : 1.0) * sizeof(c64) + ne * szC));
    MF_TRY(lu_factor<C>(s, n, ne, LU, ipiv, perm, pinv, linfo, Dinv));
    tok = prof_begin(s);
    MF_TRY(panel_inverses<C>(s, n, ne, LU, Dinv, Pinv));
    prof_end(tok, s, K_LU_ROWS, 0.0, 0.0);
    std::vector<int> hi(ne);
    MF_HIP_CHECK(hipMemcpyAsync(hi.data(), linfo, ne * 4, hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < ne; ++j)
      if (hi[j] != 0) return -2;
  }
  t_fact += ph.stop();

  // ---- starting blocks (row-major n x m0)
  if (f(5) == 1) {
    MF_TRY(copy_cm_to_rm<c64>(s, n, m0, Xu, ldx, X, m0));
    if (two) MF_TRY(copy_cm_to_rm<c64>(s, n, m0, Xu + (int64_t)m0in * ldx, ldx, XL, m0));
  } else {
    MF_TRY(random_block<c64>(s, n, m0, (uint64_t)(uint32_t)f(51), X, m0));
    if (two) MF_TRY(random_block<c64>(s, n, m0, (uint64_t)(uint32_t)(f(51) + 1), XL, m0));
  }

  auto prod = [&](const c64* Mat, int64_t ldm, bool herm, int m, const c64* Xi, c64* Yo) -> int {
    // Yo = op(Mat) Xi with Mat column-major (element (i, k) at Mat[i + k ldm]): for op = N
    // the rows of Mat are read M-contiguous; Mat^H Xi = conj(Mat^T conj(Xi)), with Mat^T the
    // row-major view as stored (T3 holds conj(Xi))
    if (!herm) return rm_gemm<c64>(s, (int)n, m, (int)n, Mat, ldm, true, false, Xi, m, Yo, m);
    const int64_t cnt = n * (int64_t)m;
    hipLaunchKernelGGL(k_conj, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, Xi, T3);
    MF_TRY(rm_gemm<c64>(s, (int)n, m, (int)n, Mat, ldm, false, false, T3, m, Yo, m));
    hipLaunchKernelGGL(k_conj, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, Yo, Yo);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  };

  std::vector<std::complex<double>> lam;
  std::vector<double> resR, resL;
  std::vector<int> order;
  double trace_prev_re = 0.0, trace_prev_im = 0.0;
  int info = 0, M = 0, k = 0;
  for (;;) {
    const bool resid = k > 0;
    // ---- right-hand sides: B Y, B^H Y~ (first contour) or the residuals R, R~
    const c64* rhsR = R;
    const c64* rhsL = RL;
    if (!resid) {
      ph.start();
      if (hasB) {
        MF_TRY(prod(B, ldb, false, m0, X, R));
        if (two) MF_TRY(prod(B, ldb, true, m0, XL, RL));
      } else {
        rhsR = X;
        rhsL = XL;
      }
      MF_HIP_CHECK(hipStreamSynchronize(s));
      t_bx += ph.stop();
    }
    ph.start();
    MF_TRY(col_absmax<c64>(s, n, m0, rhsR, m0, dsl(o_rn)));
    if (two) MF_TRY(col_absmax<c64>(s, n, m0, rhsL, m0, dsl(o_rnl)));
    MF_HIP_CHECK(hipMemcpyAsync(hsl(o_rn), dsl(o_rn), m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipMemcpyAsync(hsl(o_rnl), dsl(o_rnl), m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < m0; ++c) {
      const double a = hsl(o_rn)[c], b = two ? hsl(o_rnl)[c] : 1.0;
      if (!std::isfinite(a) || !std::isfinite(b)) return -2;
      hsl(o_cs)[c] = a > 0.0 ? 1.0 / a : 1.0;
      hsl(o_us)[c] = a > 0.0 ? a : 1.0;
      hsl(o_csl)[c] = b > 0.0 ? 1.0 / b : 1.0;
      hsl(o_usl)[c] = b > 0.0 ? b : 1.0;
      std::complex<double> rho(0.0, 0.0);
      for (int j = 0; j < ne; ++j) {
        std::complex<double> cr = w[j];
        if (resid) cr = w[j] / (z[j] - lam[c]);
        rho += cr;
        const std::complex<double> cl = std::conj(cr);
        h_cR[(size_t)j * m0 + c] = c64(cr.real(), cr.imag());
        h_cL[(size_t)j * m0 + c] = c64(cl.real(), cl.imag());
      }
      h_rho[c] = c64(rho.real(), rho.imag());
    }
    MF_HIP_CHECK(hipMemcpyAsync(dsl(o_cs), hsl(o_cs), 4 * (size_t)m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_rho, h_rho, m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_cR, h_cR, (size_t)ne * m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_cL, h_cL, (size_t)ne * m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    {
      int tok = prof_begin(s);
      dim3 grid((unsigned)((m0 + 255) / 256), (unsigned)n);
      hipLaunchKernelGGL((k_rhs_two<C>), grid, dim3(256), 0, s, n, m0, rhsR, rhsL, dsl(o_cs), dsl(o_csl), ne, perm,
                         two ? Wf : (C*)nullptr, Wc);
      MF_HIP_CHECK(hipGetLastError());
      prof_end(tok, s, K_OTHER, 0.0, (double)n * m0 * (two ? 2.0 : 1.0) * (16.0 + ne * szC));
      // right: conjugate-transpose sweeps of F_j (Wc); left: forward sweeps (Wf)
      MF_TRY(lu_solve<C>(s, n, m0, ne, LU, Pinv, two ? Wf : (C*)nullptr, Wc, Wy, two_streams ? &side : nullptr));
      tok = prof_begin(s);
      hipLaunchKernelGGL((k_accumulate_two<C>), grid, dim3(256), 0, s, n, m0, ne, two ? Wf : (C*)nullptr, Wc, pinv,
                         d_cR, d_cL, d_rho, dsl(o_us), dsl(o_usl), X, XL, Q, QL, resid ? 1 : 0);
      MF_HIP_CHECK(hipGetLastError());
      prof_end(tok, s, K_OTHER, 0.0, (double)n * m0 * (two ? 2.0 : 1.0) * (ne * szC + 32.0));
    }
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_solve += ph.stop();

    // ---- Rayleigh-Ritz: products with A, B (and A^H, B^H) on the raw blocks
    ph.start();
    MF_TRY(prod(A, lda, false, m0, Q, AQ));
    if (two) MF_TRY(prod(A, lda, true, m0, QL, AhQ));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_ax += ph.stop();
    if (hasB) {
      ph.start();
      MF_TRY(prod(B, ldb, false, m0, Q, BQ));
      if (two) MF_TRY(prod(B, ldb, true, m0, QL, BhQ));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      t_bx += ph.stop();
    }
    ph.start();
    int kr = 0, kl = 0;
    MF_TRY(orthonormalize(s, n, m0, Q, orr, (int*)hsl(o_keep), (int*)hsl(o_idx), hsl(o_flag), kr));
    if (h_flag[0] != 0 || kr == 0) { info = -3; break; }
    if (two) {
      MF_TRY(orthonormalize(s, n, m0, QL, orl, (int*)hsl(o_keepl), (int*)hsl(o_idxl), hsl(o_flag), kl));
      if (h_flag[0] != 0 || kl == 0) { info = -3; break; }
    } else {
      kl = kr;
    }
    const int kk = std::min(kr, kl);
    // transforms restricted to the first kk kept columns (m0 x kk)
    c64* Tr = orr.Tr;
    c64* Tl = two ? orl.Tr : orr.Tr;
    if (kk < kr) {
      hipLaunchKernelGGL(k_take_cols, dim3((kk + 255) / 256, m0), dim3(256), 0, s, m0, kk, orr.Tr, kr, orr.S2);
      Tr = orr.S2;
    }
    if (two && kk < kl) {
      hipLaunchKernelGGL(k_take_cols, dim3((kk + 255) / 256, m0), dim3(256), 0, s, m0, kk, orl.Tr, kl, orl.H1);
      Tl = orl.H1;
    }
    const int krs = (kk < kr) ? kk : kr, kls = (two && kk < kl) ? kk : kl;
    (void)krs;
    (void)kls;
    // Qo = Q Tr, A Qo, B Qo; QLo = QL Tl, A^H QLo, B^H QLo  (n x kk, leading dimension kk)
    MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, Q, m0, false, false, Tr, kk, Qo, kk));
    MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, AQ, m0, false, false, Tr, kk, AQo, kk));
    if (hasB) MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, BQ, m0, false, false, Tr, kk, BQo, kk));
    const c64* QLx = Qo;
    if (two) {
      MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, QL, m0, false, false, Tl, kk, QLo, kk));
      MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, AhQ, m0, false, false, Tl, kk, AhQo, kk));
      if (hasB) MF_TRY(rm_gemm<c64>(s, (int)n, kk, m0, BhQ, m0, false, false, Tl, kk, BhQo, kk));
      QLx = QLo;
    }
    // reduced pencil Aq = QLo^H A Qo, Bq = QLo^H B Qo
    MF_TRY(rm_gemm<c64>(s, kk, kk, (int)n, QLx, kk, true, true, AQo, kk, Aq, kk));
    MF_TRY(rm_gemm<c64>(s, kk, kk, (int)n, QLx, kk, true, true, hasB ? BQo : Qo, kk, Bq, kk));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_eig += ph.stop();
    ph.start();
    {
      NhEig ew{Gw, Gw + (size_t)kk * kk, Gw + 2 * (size_t)kk * kk, Hw, Zw, Vw, Uw, part, d_flag};
      MF_TRY(nh_eigensolve(s, kk, Aq, Bq, two, ew, d_lam, Wr, Wl, h_flag));
    }
    MF_HIP_CHECK(hipMemcpyAsync(h_lam, d_lam, kk * sizeof(c64), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_eig += ph.stop();
    if (h_flag[0] != 0) { info = -3; break; }
    m0 = kk;
    lam.resize(m0);
    bool finite = true;
    for (int c = 0; c < m0; ++c) {
      lam[c] = std::complex<double>(h_lam[c].re, h_lam[c].im);
      if (!std::isfinite(lam[c].real()) || !std::isfinite(lam[c].imag())) finite = false;
    }
    if (!finite) { info = -3; break; }
    // ---- Ritz vectors and residuals
    ph.start();
    MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, Qo, m0, false, false, Wr, m0, X, m0));
    MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, AQo, m0, false, false, Wr, m0, T3, m0));
    const c64* BX = X;
    if (hasB) {
      MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, BQo, m0, false, false, Wr, m0, T4, m0));
      BX = T4;
    }
    {
      const int tok = prof_begin(s);
      MF_TRY(nh_resid(s, n, m0, T3, BX, d_lam, false, R, dsl(o_rn), dsl(o_bn), part));
      prof_end(tok, s, K_RESID, 0.0, (double)n * m0 * 48.0);
    }
    if (two) {
      MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, QLo, m0, false, false, Wl, m0, XL, m0));
      MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, AhQo, m0, false, false, Wl, m0, T3, m0));
      const c64* BhY = XL;
      if (hasB) {
        MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, BhQo, m0, false, false, Wl, m0, T4, m0));
        BhY = T4;
      }
      const int tok = prof_begin(s);
      MF_TRY(nh_resid(s, n, m0, T3, BhY, d_lam, true, RL, dsl(o_rnl), dsl(o_bnl), part));
      prof_end(tok, s, K_RESID, 0.0, (double)n * m0 * 48.0);
    }
    MF_HIP_CHECK(hipMemcpyAsync(hsl(o_rn), dsl(o_rn), 4 * (size_t)m0in * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_eig += ph.stop();
    resR.assign(m0, 0.0);
    resL.assign(m0, 0.0);
    bool fin = true;
    for (int c = 0; c < m0; ++c) {
      resR[c] = std::sqrt(hsl(o_rn)[c]) / (alpha * std::sqrt(hsl(o_bn)[c]));
      if (two) resL[c] = std::sqrt(hsl(o_rnl)[c]) / (alpha * std::sqrt(hsl(o_bnl)[c]));
      if (!std::isfinite(resR[c]) || !std::isfinite(resL[c])) fin = false;
    }
    if (!fin) { info = -2; break; }
    // ---- count, order (inside first, each by real then imaginary part), trace, stop
    // found: inside the contour with residuals below NH_SPURIOUS_RES (spurious Ritz values
    // of the projected non-normal problem may fall inside with residuals of order one)
    std::vector<char> in(m0);
    M = 0;
    int n_inside = 0;
    for (int c = 0; c < m0; ++c) {
      const bool geo = inside_ellipse(lam[c], emid, r, f(18), f(19));
      const bool ok = resR[c] < NH_SPURIOUS_RES && (!two || resL[c] < NH_SPURIOUS_RES);
      n_inside += geo ? 1 : 0;
      in[c] = (geo && ok) ? 1 : 0;
      M += in[c];
    }
    order.resize(m0);
    for (int c = 0; c < m0; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (in[a] != in[b]) return in[a] > in[b];
      if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
      return lam[a].imag() < lam[b].imag();
    });
    double tr_re = 0.0, tr_im = 0.0, maxres = 0.0;
    for (int q = 0; q < M; ++q) {
      const int c = order[q];
      tr_re += lam[c].real();
      tr_im += lam[c].imag();
      maxres = std::max(maxres, resR[c]);
      if (two) maxres = std::max(maxres, resL[c]);
    }
    const double eo = (k == 0) ? 1.0 : std::hypot(tr_re - trace_prev_re, tr_im - trace_prev_im) / alpha;
    trace_prev_re = tr_re;
    trace_prev_im = tr_im;
    *epsout = eo;
    *loop = k;
    *Mout = M;
    if (f(1) != 0)
      fprintf(stderr, "%3d %6d  %24.16E %24.16E  %24.16E  %24.16E  m0=%d\n", k, M, tr_re, tr_im, eo, maxres, m0);
    if (n_inside == 0) { info = 1; break; }
    if (n_inside >= m0) { info = 3; break; }
    if (M > 0 && ((f(6) == 1) ? (maxres < eps) : (eo < eps))) { info = 0; break; }
    if (k >= f(4)) { info = 2; break; }
    ++k;
  }
  if (info == 0 || info == 1 || info == 2 || info == 3) {
    // eigenpairs to the caller's layout in the reported order: E complex (m0 values), X
    // right vectors in columns 0..m0-1 and left vectors in columns m0in.., res right
    // then left (at m0in)
    std::vector<int> hperm(order.begin(), order.end());
    int* d_perm = (int*)dsl(o_perm);
    MF_HIP_CHECK(hipMemcpyAsync(d_perm, hperm.data(), m0 * sizeof(int), hipMemcpyHostToDevice, s));
    MF_TRY(copy_rm_to_cm<c64>(s, n, m0, X, m0, Xu, ldx, d_perm));
    if (two) MF_TRY(copy_rm_to_cm<c64>(s, n, m0, XL, m0, Xu + (int64_t)m0in * ldx, ldx, d_perm));
    std::vector<double> e_out(2 * (size_t)m0), r_out(two ? 2 * (size_t)m0in : (size_t)m0, 0.0);
    for (int q = 0; q < m0; ++q) {
      e_out[2 * q] = lam[order[q]].real();
      e_out[2 * q + 1] = lam[order[q]].imag();
      r_out[q] = resR[order[q]];
      if (two) r_out[m0in + q] = resL[order[q]];
    }
    MF_HIP_CHECK(hipMemcpyAsync(E, e_out.data(), e_out.size() * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(res_out, r_out.data(), r_out.size() * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    *m0p = m0;
  }
  h->timing[0] = t_fact;
  h->timing[1] = t_solve;
  h->timing[2] = t_ax;
  h->timing[3] = t_bx;
  h->timing[5] = total_t.stop();
  h->timing[4] = h->timing[5] - t_fact - t_solve - t_ax - t_bx;
  h->timing[6] = (double)(*loop + 1);
  h->timing[7] = t_eig;
  return info;
}

// ---------------------------------------------------------------------------
// Polynomial FEAST driver (right eigenvectors; the readings of the polynomial oracle)
template <typename C>
static int poly_run(mfeast_ctx* h, int p, int64_t n, const c64* As, int64_t lda, int32_t* fpm, double* epsout,
                    int32_t* loop, std::complex<double> emid, double r, int32_t* m0p, double* E, c64* Xu,
                    int64_t ldx, int32_t* Mout, double* res_out, const std::vector<std::complex<double>>& z,
                    const std::vector<std::complex<double>>& w) {
  auto f = [&](int i) { return fpm[i - 1]; };
  hipStream_t s = h->stream;
  const int ne = (int)z.size();
  const int m0in = *m0p;
  int m0 = m0in;
  const double alpha = std::abs(emid) + r;
  const double eps = std::pow(10.0, -f(3));
  const int64_t ld = lu_ld(n);
  const size_t szC = sizeof(C);
  const size_t blk = (size_t)n * m0 * sizeof(c64);
  const size_t sq = (size_t)m0 * m0 * sizeof(c64);
  const int pmax = p * m0;
  const size_t psq = (size_t)pmax * pmax * sizeof(c64);
  const int64_t mstride = lda * n;
  Timer total_t, ph;
  total_t.start();
  double t_fact = 0, t_solve = 0, t_ax = 0, t_eig = 0;

  C* LU = (C*)h->ws(S_LU, (size_t)ne * n * ld * szC);
  C* Dinv = (C*)h->ws(S_DINV, (size_t)ne * ((n + LU_NB - 1) / LU_NB) * 2 * LU_NB * LU_NB * szC);
  C* Pinv = (C*)h->ws(S_PANINV, (size_t)ne * panel_inverse_entries(n) * szC);
  int* ipiv = (int*)h->ws(S_IPIV, (size_t)ne * n * 4);
  int* perm = (int*)h->ws(S_PERM, (size_t)ne * n * 4);
  int* pinv = (int*)h->ws(S_PINV, (size_t)ne * n * 4);
  int* linfo = (int*)h->ws(S_INFO, (size_t)ne * 4 + 64);
  c64* zdev = (c64*)h->ws(S_Z, (size_t)ne * sizeof(c64));
  C* Wc = (C*)h->ws(S_WC, (size_t)ne * n * m0 * szC);
  C* Wy = (C*)h->ws(S_WY, (size_t)ne * n * m0 * szC);
  c64* X = (c64*)h->ws(S_X, blk);
  c64* Q = (c64*)h->ws(S_Q, blk);
  c64* R = (c64*)h->ws(S_R, blk);
  c64* Qo = (c64*)h->ws(S_AX, blk);
  c64* T3 = (c64*)h->ws(S_NH_T3, blk);
  c64* AkQ = (c64*)h->ws(S_PL_AKQ, (size_t)(p + 1) * blk);
  c64* AkQo = (c64*)h->ws(S_PL_AKQO, (size_t)(p + 1) * blk);
  c64* AkX = (c64*)h->ws(S_PL_AKX, (size_t)(p + 1) * blk);
  c64* Aq = (c64*)h->ws(S_PL_AQ, (size_t)(p + 1) * sq);
  c64* L0 = (c64*)h->ws(S_PL_L0, psq);
  c64* L1 = (c64*)h->ws(S_PL_L1, psq);
  c64* Wz = (c64*)h->ws(S_PL_WZ, psq);
  c64* Wsel = (c64*)h->ws(S_W, sq);
  c64* Gw = (c64*)h->ws(S_PL_G, 3 * psq);
  c64* Hw = (c64*)h->ws(S_PL_H, psq);
  c64* Zw = (c64*)h->ws(S_PL_Z, psq);
  c64* Vw = (c64*)h->ws(S_PL_V, psq);
  Orth orr{};
  orr.S = (c64*)h->ws(S_NH_O1, sq);
  orr.S2 = (c64*)h->ws(S_NH_O2, sq);
  orr.Linv = (c64*)h->ws(S_NH_O3, sq);
  orr.H1 = (c64*)h->ws(S_NH_O4, sq);
  orr.V = (c64*)h->ws(S_NH_O5, sq);
  orr.TG = (c64*)h->ws(S_TG, std::max(3 * sq, (size_t)m0 * 32 * sizeof(c64)));
  orr.Tr = (c64*)h->ws(S_NH_TR, sq);
  const size_t nsmall = (size_t)m0 * 24 + (size_t)pmax * 4 + (size_t)(p + 2) * m0 + (size_t)ne * m0 * 4 + 256;
  double* small = (double*)h->ws(S_SMALL, nsmall * sizeof(double));
  const int nchunk = (int)((n + 255) / 256);
  double* part = (double*)h->ws(S_PART, (size_t)nchunk * m0 * (p + 2) * sizeof(double) + 64);
  char* hp = h->host(nsmall * sizeof(double) + 4096);
  if (!LU || !Dinv || !Pinv || !ipiv || !perm || !pinv || !linfo || !zdev || !Wc || !Wy || !X || !Q || !R || !Qo ||
      !T3 || !AkQ || !AkQo || !AkX || !Aq || !L0 || !L1 || !Wz || !Wsel || !Gw || !Hw || !Zw || !Vw || !orr.S ||
      !orr.S2 || !orr.Linv || !orr.H1 || !orr.V || !orr.TG || !orr.Tr || !small || !part || !hp)
    return -2;
  auto dsl = [&](size_t off) { return small + off; };
  auto hsl = [&](size_t off) { return reinterpret_cast<double*>(hp) + off; };
  const size_t o_cs = 0, o_us = m0, o_keep = 2 * m0, o_idx = 3 * m0, o_d = 4 * m0, o_flag = 5 * m0,
               o_perm = 6 * m0, o_sel = 7 * m0, o_rho = 8 * m0 /* 2 m0 */, o_lam = 10 * m0 /* 2 m0 */,
               o_nrm = 24 * (size_t)m0 /* (p + 2) m0 */, o_mu = o_nrm + (size_t)(p + 2) * m0 /* 2 pmax */,
               o_cR = o_mu + 2 * (size_t)pmax /* 2 ne m0 */;
  orr.d = dsl(o_d);
  orr.keep = (int*)dsl(o_keep);
  orr.idx = (int*)dsl(o_idx);
  orr.flag = (int*)dsl(o_flag);
  orr.part = part;
  int* d_flag = (int*)dsl(o_flag);
  int* h_flag = (int*)hsl(o_flag);
  c64* d_mu = reinterpret_cast<c64*>(dsl(o_mu));
  c64* h_mu = reinterpret_cast<c64*>(hsl(o_mu));
  c64* d_lam = reinterpret_cast<c64*>(dsl(o_lam));
  c64* h_lam = reinterpret_cast<c64*>(hsl(o_lam));
  c64* d_rho = reinterpret_cast<c64*>(dsl(o_rho));
  c64* h_rho = reinterpret_cast<c64*>(hsl(o_rho));
  c64* d_cR = reinterpret_cast<c64*>(dsl(o_cR));
  c64* h_cR = reinterpret_cast<c64*>(hsl(o_cR));

  // ---- F_j = P(z_j)^H for every node (right solves by its conjugate-transpose sweeps)
  ph.start();
  {
    std::vector<c64> zc(ne);
    for (int j = 0; j < ne; ++j) zc[j] = c64(z[j].real(), -z[j].imag());
    MF_HIP_CHECK(hipMemcpyAsync(zdev, zc.data(), ne * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemsetAsync(linfo, 0, ne * 4, s));
    int tok = prof_begin(s);
    hipLaunchKernelGGL((k_poly_form<C>), dim3((unsigned)((n + 255) / 256), (unsigned)n), dim3(256), 0, s, n, ld, As,
                       lda, p, zdev, ne, LU, perm);
    MF_HIP_CHECK(hipGetLastError());
    prof_end(tok, s, K_OTHER, 0.0, (double)n * n * ((p + 1.0) * sizeof(c64) + ne * szC));
    MF_TRY(lu_factor<C>(s, n, ne, LU, ipiv, perm, pinv, linfo, Dinv));
    tok = prof_begin(s);
    MF_TRY(panel_inverses<C>(s, n, ne, LU, Dinv, Pinv));
    prof_end(tok, s, K_LU_ROWS, 0.0, 0.0);
    std::vector<int> hi(ne);
    MF_HIP_CHECK(hipMemcpyAsync(hi.data(), linfo, ne * 4, hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < ne; ++j)
      if (hi[j] != 0) return -2;
  }
  t_fact += ph.stop();
  if (f(5) == 1) MF_TRY(copy_cm_to_rm<c64>(s, n, m0, Xu, ldx, X, m0));
  else MF_TRY(random_block<c64>(s, n, m0, (uint64_t)(uint32_t)f(51), X, m0));

  std::vector<std::complex<double>> lam;
  std::vector<double> res;
  std::vector<int> order;
  double tpr = 0.0, tpi = 0.0;
  int info = 0, M = 0, k = 0;
  for (;;) {
    const bool resid = k > 0;
    const c64* rhs = resid ? R : X;
    ph.start();
    MF_TRY(col_absmax<c64>(s, n, m0, rhs, m0, dsl(o_cs)));
    MF_HIP_CHECK(hipMemcpyAsync(hsl(o_cs), dsl(o_cs), m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < m0; ++c) {
      const double a = hsl(o_cs)[c];
      if (!std::isfinite(a)) return -2;
      hsl(o_cs)[c] = a > 0.0 ? 1.0 / a : 1.0;
      hsl(o_us)[c] = a > 0.0 ? a : 1.0;
      std::complex<double> rho(0.0, 0.0);
      for (int j = 0; j < ne; ++j) {
        std::complex<double> cr = w[j];
        if (resid) {
          const std::complex<double> q = w[j] / (z[j] - lam[c]);
          rho += q;
          cr = -q;
        }
        h_cR[(size_t)j * m0 + c] = c64(cr.real(), cr.imag());
      }
      h_rho[c] = c64(rho.real(), rho.imag());
    }
    MF_HIP_CHECK(hipMemcpyAsync(dsl(o_cs), hsl(o_cs), 2 * (size_t)m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_rho, h_rho, m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_cR, h_cR, (size_t)ne * m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    {
      int tok = prof_begin(s);
      dim3 grid((unsigned)((m0 + 255) / 256), (unsigned)n);
      hipLaunchKernelGGL((k_rhs_two<C>), grid, dim3(256), 0, s, n, m0, rhs, (const c64*)nullptr, dsl(o_cs),
                         dsl(o_cs), ne, perm, (C*)nullptr, Wc);
      MF_HIP_CHECK(hipGetLastError());
      prof_end(tok, s, K_OTHER, 0.0, (double)n * m0 * (16.0 + ne * szC));
      MF_TRY(lu_solve<C>(s, n, m0, ne, LU, Pinv, (C*)nullptr, Wc, Wy, nullptr));
      tok = prof_begin(s);
      hipLaunchKernelGGL((k_accumulate_two<C>), grid, dim3(256), 0, s, n, m0, ne, (const C*)nullptr, Wc, pinv, d_cR,
                         d_cR, d_rho, dsl(o_us), dsl(o_us), X, X, Q, Q, resid ? 1 : 0);
      MF_HIP_CHECK(hipGetLastError());
      prof_end(tok, s, K_OTHER, 0.0, (double)n * m0 * (ne * szC + 32.0));
    }
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_solve += ph.stop();

    // ---- Rayleigh-Ritz: A_k Q, orthonormal basis, reduced coefficients, companion form
    ph.start();
    for (int kk = 0; kk <= p; ++kk)
      MF_TRY(rm_gemm<c64>(s, (int)n, m0, (int)n, As + kk * mstride, lda, true, false, Q, m0, AkQ + (size_t)kk * n * m0,
                          m0));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_ax += ph.stop();
    ph.start();
    int kr = 0;
    MF_TRY(orthonormalize(s, n, m0, Q, orr, (int*)hsl(o_keep), (int*)hsl(o_idx), hsl(o_flag), kr));
    if (h_flag[0] != 0 || kr == 0) { info = -3; break; }
    if (p * kr > NH_MAX_M0) { info = -3; break; }
    MF_TRY(rm_gemm<c64>(s, (int)n, kr, m0, Q, m0, false, false, orr.Tr, kr, Qo, kr));
    for (int kk = 0; kk <= p; ++kk) {
      MF_TRY(rm_gemm<c64>(s, (int)n, kr, m0, AkQ + (size_t)kk * n * m0, m0, false, false, orr.Tr, kr,
                          AkQo + (size_t)kk * n * kr, kr));
      MF_TRY(rm_gemm<c64>(s, kr, kr, (int)n, Qo, kr, true, true, AkQo + (size_t)kk * n * kr, kr,
                          Aq + (size_t)kk * kr * kr, kr));
    }
    const int pm = p * kr;
    hipLaunchKernelGGL(k_companion, dim3((pm + 255) / 256, pm), dim3(256), 0, s, kr, p, Aq, L0, L1);
    MF_HIP_CHECK(hipGetLastError());
    {
      NhEig ew{Gw, Gw + (size_t)pm * pm, Gw + 2 * (size_t)pm * pm, Hw, Zw, Vw, Vw, part, d_flag};
      MF_TRY(nh_eigensolve(s, pm, L0, L1, false, ew, d_mu, Wz, Wz, h_flag));
    }
    MF_HIP_CHECK(hipMemcpyAsync(h_mu, d_mu, pm * sizeof(c64), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_eig += ph.stop();
    if (h_flag[0] != 0) { info = -3; break; }
    // the kr values of the companion pencil nearest the contour's centre (ellipse metric)
    std::vector<int> sel(pm);
    std::vector<double> metric(pm);
    const std::complex<double> rot = std::polar(1.0, -f(19) * M_PI / 180.0);
    for (int q = 0; q < pm; ++q) {
      const std::complex<double> mu(h_mu[q].re, h_mu[q].im);
      const std::complex<double> u = rot * (mu - emid);
      const double e = f(18) / 100.0;
      const double mt = (u.real() / r) * (u.real() / r) + (u.imag() / (e * r)) * (u.imag() / (e * r));
      metric[q] = std::isfinite(mt) ? mt : std::numeric_limits<double>::infinity();
      sel[q] = q;
    }
    std::stable_sort(sel.begin(), sel.end(), [&](int a, int b) { return metric[a] < metric[b]; });
    m0 = kr;
    lam.resize(m0);
    bool fin = true;
    int* hsel = (int*)hsl(o_sel);
    for (int q = 0; q < m0; ++q) {
      hsel[q] = sel[q];
      lam[q] = std::complex<double>(h_mu[sel[q]].re, h_mu[sel[q]].im);
      h_lam[q] = h_mu[sel[q]];
      if (!std::isfinite(metric[sel[q]])) fin = false;
    }
    if (!fin) { info = -3; break; }
    ph.start();
    MF_HIP_CHECK(hipMemcpyAsync(dsl(o_sel), hsel, m0 * sizeof(int), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_lam, h_lam, m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_first_block, dim3((m0 + 255) / 256), dim3(256), 0, s, m0, pm, Wz, (const int*)dsl(o_sel),
                       Wsel);
    MF_HIP_CHECK(hipGetLastError());
    // Ritz vectors, A_k X, residuals
    MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, Qo, m0, false, false, Wsel, m0, X, m0));
    for (int kk = 0; kk <= p; ++kk)
      MF_TRY(rm_gemm<c64>(s, (int)n, m0, m0, AkQo + (size_t)kk * n * m0, m0, false, false, Wsel, m0,
                          AkX + (size_t)kk * n * m0, m0));
    {
      const int tok = prof_begin(s);
      hipLaunchKernelGGL(k_poly_resid_partial, dim3((m0 + 255) / 256, nchunk), dim3(256), 0, s, n, m0, p, AkX, d_lam,
                         R, part);
      hipLaunchKernelGGL(k_poly_resid_final, dim3((m0 + 255) / 256), dim3(256), 0, s, m0, p, nchunk, part,
                         dsl(o_nrm));
      MF_HIP_CHECK(hipGetLastError());
      prof_end(tok, s, K_RESID, 0.0, (double)n * m0 * (p + 2.0) * 16.0);
    }
    MF_HIP_CHECK(hipMemcpyAsync(hsl(o_nrm), dsl(o_nrm), (size_t)(p + 2) * m0 * sizeof(double), hipMemcpyDeviceToHost,
                                s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_eig += ph.stop();
    res.assign(m0, 0.0);
    for (int c = 0; c < m0; ++c) {
      double den = 0.0, pw = 1.0;
      for (int kk = 0; kk <= p; ++kk) {
        den += pw * std::sqrt(hsl(o_nrm)[(size_t)(1 + kk) * m0 + c]);
        pw *= std::abs(lam[c]);
      }
      res[c] = std::sqrt(hsl(o_nrm)[c]) / den;
      if (!std::isfinite(res[c])) fin = false;
    }
    if (!fin) { info = -2; break; }
    // found: inside the contour with a residual below min(0.1, 10^(-fpm(3)/2)); values of the
    // linearization that belong to no eigenpair keep residuals of 1e-2 to 1e-1
    const double ftol = std::min(NH_SPURIOUS_RES, std::pow(10.0, -0.5 * f(3)));
    std::vector<char> in(m0);
    M = 0;
    int n_inside = 0;
    for (int c = 0; c < m0; ++c) {
      const bool geo = inside_ellipse(lam[c], emid, r, f(18), f(19));
      n_inside += geo ? 1 : 0;
      in[c] = (geo && res[c] < ftol) ? 1 : 0;
      M += in[c];
    }
    order.resize(m0);
    for (int c = 0; c < m0; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      if (in[a] != in[b]) return in[a] > in[b];
      if (lam[a].real() != lam[b].real()) return lam[a].real() < lam[b].real();
      return lam[a].imag() < lam[b].imag();
    });
    double tr_re = 0.0, tr_im = 0.0, maxres = 0.0;
    for (int q = 0; q < M; ++q) {
      tr_re += lam[order[q]].real();
      tr_im += lam[order[q]].imag();
      maxres = std::max(maxres, res[order[q]]);
    }
    const double eo = (k == 0) ? 1.0 : std::hypot(tr_re - tpr, tr_im - tpi) / alpha;
    tpr = tr_re;
    tpi = tr_im;
    *epsout = eo;
    *loop = k;
    *Mout = M;
    if (f(1) != 0) fprintf(stderr, "%3d %6d  %24.16E  %24.16E  m0=%d\n", k, M, eo, maxres, m0);
    if (n_inside == 0) { info = 1; break; }
    if (n_inside >= m0) { info = 3; break; }
    if (M > 0 && ((f(6) == 1) ? (maxres < eps) : (eo < eps))) { info = 0; break; }
    if (k >= f(4)) { info = 2; break; }
    ++k;
  }
  if (info == 0 || info == 1 || info == 2 || info == 3) {
    std::vector<int> hperm(order.begin(), order.end());
    int* d_perm = (int*)dsl(o_perm);
    MF_HIP_CHECK(hipMemcpyAsync(d_perm, hperm.data(), m0 * sizeof(int), hipMemcpyHostToDevice, s));
    MF_TRY(copy_rm_to_cm<c64>(s, n, m0, X, m0, Xu, ldx, d_perm));
    std::vector<double> e_out(2 * (size_t)m0), r_out((size_t)m0);
    for (int q = 0; q < m0; ++q) {
      e_out[2 * q] = lam[order[q]].real();
      e_out[2 * q + 1] = lam[order[q]].imag();
      r_out[q] = res[order[q]];
    }
    MF_HIP_CHECK(hipMemcpyAsync(E, e_out.data(), e_out.size() * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(res_out, r_out.data(), r_out.size() * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    *m0p = m0;
  }
  h->timing[0] = t_fact;
  h->timing[1] = t_solve;
  h->timing[2] = t_ax;
  h->timing[3] = 0.0;
  h->timing[5] = total_t.stop();
  h->timing[4] = h->timing[5] - t_fact - t_solve - t_ax;
  h->timing[6] = (double)(*loop + 1);
  h->timing[7] = t_eig;
  return info;
}

static int check_general_fpm(const int32_t* fpm, bool expert) {
  auto f = [&](int i) { return fpm[i - 1]; };
  if (!expert) {
    if (f(16) != 0 && f(16) != 1) return 116;
    if (f(16) == 0 && !gauss_full_allowed(f(8))) return 108;
    if (f(16) == 1 && f(8) < 2) return 108;
    if (f(18) <= 0) return 118;
    if (f(19) < -180 || f(19) > 180) return 119;
  } else if (f(8) < 1) {
    return 108;
  }
  if (f(3) < 0 || f(3) > 16) return 103;
  if (f(4) < 0) return 104;
  if (f(5) != 0 && f(5) != 1) return 105;
  if (f(6) != 0 && f(6) != 1) return 106;
  if (f(14) != 0) return 114;
  if (f(15) != 0 && f(15) != 1) return 115;
  if (f(42) != 0 && f(42) != 1) return 142;
  if (f(53) != 0 && f(53) != 1) return 153;
  return 0;
}

extern "C" {

void mfeast_init_general(int32_t* fpm) {
  if (fpm == nullptr) return;
  mfeast_init(fpm);
  fpm[14] = 0;    // fpm(15) two-sided: right and left eigenvectors
  fpm[15] = 1;    // fpm(16) trapezoidal
  fpm[17] = 100;  // fpm(18) circle
}

int mfeast_gcontour(double emid_re, double emid_im, double r, int32_t ne, int32_t rule, int32_t ratio_pct,
                    int32_t angle_deg, double* zne, double* wne) {
  if (!(r > 0.0)) return 200;
  if (rule != 0 && rule != 1) return 116;
  if ((rule == 0 && !gauss_full_allowed(ne)) || (rule == 1 && ne < 2)) return 108;
  if (ratio_pct <= 0) return 118;
  if (angle_deg < -180 || angle_deg > 180) return 119;
  if (zne == nullptr) return -108;
  if (wne == nullptr) return -109;
  std::vector<std::complex<double>> z, w;
  full_contour(std::complex<double>(emid_re, emid_im), r, ne, rule, ratio_pct, angle_deg, z, w);
  for (int j = 0; j < ne; ++j) {
    zne[2 * j] = z[j].real();
    zne[2 * j + 1] = z[j].imag();
    wne[2 * j] = w[j].real();
    wne[2 * j + 1] = w[j].imag();
  }
  return 0;
}

int mfeast_zgegv(mfeast_handle h, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                 int32_t* fpm, double* epsout, int32_t* loop, const double* emid, double r, int32_t* m0, double* E,
                 double* X, int64_t ldx, int32_t* M, double* res, const double* zne, const double* wne) {
  // argument positions: h 1, n 2, A 3, lda 4, B 5, ldb 6, fpm 7, epsout 8, loop 9, emid 10,
  // r 11, m0 12, E 13, X 14, ldx 15, M 16, res 17, zne 18, wne 19
  if (n < 1 || n > 16384) return 202;
  if (m0 == nullptr) return -112;
  if (*m0 < 1 || *m0 > n || *m0 > NH_MAX_M0) return 201;
  if (emid == nullptr) return -110;
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(emid[0]) || !std::isfinite(emid[1])) return 200;
  if (fpm == nullptr) return -107;
  if ((zne == nullptr) != (wne == nullptr)) return zne == nullptr ? -118 : -119;
  const int fi = check_general_fpm(fpm, zne != nullptr);
  if (fi) return fi;
  if (h == nullptr) return -101;
  if (A == nullptr) return -103;
  if (lda < n) return -104;
  if (B != nullptr && ldb < n) return -106;
  if (epsout == nullptr) return -108;
  if (loop == nullptr) return -109;
  if (E == nullptr) return -113;
  if (X == nullptr) return -114;
  if (ldx < n) return -115;
  if (M == nullptr) return -116;
  if (res == nullptr) return -117;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  const std::complex<double> em(emid[0], emid[1]);
  std::vector<std::complex<double>> z, w;
  const int ne = fpm[7];
  if (zne != nullptr) {
    z.resize(ne);
    w.resize(ne);
    for (int j = 0; j < ne; ++j) {
      z[j] = std::complex<double>(zne[2 * j], zne[2 * j + 1]);
      w[j] = std::complex<double>(wne[2 * j], wne[2 * j + 1]);
    }
  } else {
    full_contour(em, r, ne, fpm[15], fpm[17], fpm[18], z, w);
  }
  set_gemm_3m(fpm[52] == 0);
  prof_enable(fpm[51] == 1 || h->prof_all);
  for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] = 0.0;
  const c64* Ac = reinterpret_cast<const c64*>(A);
  const c64* Bc = reinterpret_cast<const c64*>(B);
  c64* Xc = reinterpret_cast<c64*>(X);
  int info;
  if (fpm[41] == 1)
    info = nh_run<c32>(h, n, Ac, lda, Bc, ldb, fpm, epsout, loop, em, r, m0, E, Xc, ldx, M, res, z, w);
  else
    info = nh_run<c64>(h, n, Ac, lda, Bc, ldb, fpm, epsout, loop, em, r, m0, E, Xc, ldx, M, res, z, w);
  if (prof_on()) {
    (void)hipStreamSynchronize(h->stream);
    prof_collect(h->prof);
    prof_enable(false);
  }
  return info;
}

void mfeast_init_polynomial(int32_t* fpm) {
  if (fpm == nullptr) return;
  mfeast_init_general(fpm);
  fpm[14] = 1;  // fpm(15) right eigenvectors
}

int mfeast_zgepev(mfeast_handle h, int32_t p, int64_t n, const double* A, int64_t lda, int32_t* fpm, double* epsout,
                  int32_t* loop, const double* emid, double r, int32_t* m0, double* E, double* X, int64_t ldx,
                  int32_t* M, double* res, const double* zne, const double* wne) {
  // argument positions: h 1, p 2, n 3, A 4, lda 5, fpm 6, epsout 7, loop 8, emid 9, r 10,
  // m0 11, E 12, X 13, ldx 14, M 15, res 16, zne 17, wne 18
  if (p < 1 || p > POLY_MAX_P) return -102;
  if (n < 1 || n > 16384) return 202;
  if (m0 == nullptr) return -111;
  if (*m0 < 1 || *m0 > n || (int64_t)p * *m0 > NH_MAX_M0) return 201;
  if (emid == nullptr) return -109;
  if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(emid[0]) || !std::isfinite(emid[1])) return 200;
  if (fpm == nullptr) return -106;
  if ((zne == nullptr) != (wne == nullptr)) return zne == nullptr ? -117 : -118;
  const int fi = check_general_fpm(fpm, zne != nullptr);
  if (fi) return fi;
  if (fpm[14] != 1) return 115;
  if (h == nullptr) return -101;
  if (A == nullptr) return -104;
  if (lda < n) return -105;
  if (epsout == nullptr) return -107;
  if (loop == nullptr) return -108;
  if (E == nullptr) return -112;
  if (X == nullptr) return -113;
  if (ldx < n) return -114;
  if (M == nullptr) return -115;
  if (res == nullptr) return -116;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  const std::complex<double> em(emid[0], emid[1]);
  std::vector<std::complex<double>> z, w;
  const int ne = fpm[7];
  if (zne != nullptr) {
    z.resize(ne);
    w.resize(ne);
    for (int j = 0; j < ne; ++j) {
      z[j] = std::complex<double>(zne[2 * j], zne[2 * j + 1]);
      w[j] = std::complex<double>(wne[2 * j], wne[2 * j + 1]);
    }
  } else {
    full_contour(em, r, ne, fpm[15], fpm[17], fpm[18], z, w);
  }
  set_gemm_3m(fpm[52] == 0);
  prof_enable(fpm[51] == 1 || h->prof_all);
  for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] = 0.0;
  const c64* Ac = reinterpret_cast<const c64*>(A);
  c64* Xc = reinterpret_cast<c64*>(X);
  int info;
  if (fpm[41] == 1)
    info = poly_run<c32>(h, p, n, Ac, lda, fpm, epsout, loop, em, r, m0, E, Xc, ldx, M, res, z, w);
  else
    info = poly_run<c64>(h, p, n, Ac, lda, fpm, epsout, loop, em, r, m0, E, Xc, ldx, M, res, z, w);
  if (prof_on()) {
    (void)hipStreamSynchronize(h->stream);
    prof_collect(h->prof);
    prof_enable(false);
  }
  return info;
}

}  // extern "C"
