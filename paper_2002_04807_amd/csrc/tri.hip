// Hermitian eigensolver by reduction to real tridiagonal form (gfx950), used for the large
// reduced problems of the Rayleigh-Ritz step whose eigenvectors only seed later work (the
// first subspace iteration, and the block of the pairs not yet found before the deflated
// sweeps).  Every stage is either one launch over many workgroups or one independent task
// per eigenvalue, so the solve is not a long chain of dependent rotation rounds.
//
//   reduce      one launch per column k (k_trd_step): every workgroup applies the rank-2
//               update of reflector k-1 to its rows of the trailing block while forming
//               p_k = tau_k A^(k) v_k for them; reflector k itself (chosen so that the
//               off-diagonal entry beta_k is real) is recomputed by every workgroup from
//               row k, so no launch waits for another workgroup of the same launch.
//   eigenvalues multisection bisection on the Sturm counts of T - x I: one wavefront per
//               eigenvalue, its 64 lanes counting at 64 interior points of the bracket.
//   eigenvectors inverse iteration on T - lambda I (tridiagonal LU with row interchanges,
//               three solves from a counter-hashed start), one workgroup per group of
//               eigenvalues closer than 1e-10 of the spectral radius; inside a group the
//               vectors are orthogonalized against the earlier ones (twice per solve).
//   back-transform  X = Q Z with Q = H_0 ... H_{m-2} applied in blocks of 32 reflectors
//               through their compact WY form I - V T V^H (three MFMA products per block).
// A group of more than TRD_CLMAX eigenvalues that close sets a flag, and the caller then
// uses the Jacobi solver on a copy of the input.
#include <algorithm>
#include <cfloat>

#include "ctx.hpp"

namespace mf {

constexpr int TRD_CPL = 16;                 // trailing columns per lane in the reduction
constexpr int TRD_MAXM = 64 * TRD_CPL;      // largest order (1024)
constexpr int TRD_NB = 32;                  // reflectors per block of the back-transform
constexpr int TRD_CLMAX = 64;               // largest group of close eigenvalues

template <typename T> __device__ inline double imag_part(T) { return 0.0; }
template <> __device__ inline double imag_part<c64>(c64 a) { return a.im; }

// sum over a wavefront in a fixed order (down-sweep, then lane 0 broadcast): every lane
// and every workgroup that sums the same values gets the same bits
__device__ inline double wave_sum_fixed(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off);
  return __shfl(x, 0);
}
__device__ inline c64 wave_sum_fixed(c64 x) { return c64(wave_sum_fixed(x.re), wave_sum_fixed(x.im)); }

// 256-thread sum in a fixed order; s_red holds 4 entries; ends with a barrier
template <typename T>
__device__ inline T block_sum_fixed(T x, T* s_red) {
  x = wave_sum_fixed(x);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = x;
  __syncthreads();
  const T r = ((s_red[0] + s_red[1]) + s_red[2]) + s_red[3];
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Reduction step k (k = 0 .. m-1).  A (m x m row-major, full Hermitian storage) holds
// A^(k-1) on rows and columns >= k on entry and A^(k) on rows and columns >= k+1 on exit
// (rows of the trailing block are updated by the workgroup that owns them).
//   w_{k-1} = p_{k-1} + alpha v_{k-1},  alpha = -Re(conj(tau_{k-1}) v_{k-1}^H p_{k-1}) / 2
//   A^(k) = A^(k-1) - v_{k-1} w_{k-1}^H - w_{k-1} v_{k-1}^H
//   H_k = I - tau_k v_k v_k^H with H_k^H x = (beta_k, 0, ..)^T for x = A^(k)[k+1:, k]
//   p_k = tau_k A^(k) v_k on the trailing rows; d_k = A^(k)[k][k], e_k = beta_k.
// Launch k = m-1 only forms d_{m-1}.  P and vb are double-buffered by the parity of k.
template <typename T>
__global__ __launch_bounds__(256) void k_trd_step(int m, int k, T* __restrict__ A, T* __restrict__ Vh,
                                                  T* __restrict__ P, T* __restrict__ vb, T* __restrict__ tau,
                                                  double* __restrict__ d, double* __restrict__ e) {
  __shared__ T s_vo[TRD_MAXM];
  __shared__ T s_wo[TRD_MAXM];
  __shared__ T s_v[TRD_MAXM];
  __shared__ T s_red[4];
  __shared__ double s_redr[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool prev = k >= 1;
  const int r = k + 1 + (int)blockIdx.x * 4 + wave;
  const bool has_row = k <= m - 2 && r < m;

  // this wavefront's row of the trailing block and this thread's entries of row k, loaded
  // before anything waits on them
  T a[TRD_CPL];
#pragma unroll
  for (int t = 0; t < TRD_CPL; ++t) {
    const int c = k + 1 + lane + 64 * t;
    a[t] = (has_row && c < m) ? A[(int64_t)r * m + c] : T(0);
  }
  T xr[TRD_MAXM / 256];
#pragma unroll
  for (int t = 0; t < TRD_MAXM / 256; ++t) {
    const int c = k + tid + 256 * t;
    xr[t] = c < m ? A[(int64_t)k * m + c] : T(0);
  }

  // ---- w_{k-1}
  if (prev) {
    const T* vo = vb + (int64_t)((k - 1) & 1) * m;
    const T* po = P + (int64_t)((k - 1) & 1) * m;
    T part = T(0);
    for (int i = k + tid; i < m; i += 256) {
      const T v = vo[i], p = po[i];
      s_vo[i] = v;
      s_wo[i] = p;
      part = part + conj(v) * p;
    }
    const T c = block_sum_fixed(part, s_red);
    const double alpha = -0.5 * real_part(conj(tau[k - 1]) * c);
    for (int i = k + tid; i < m; i += 256) s_wo[i] = s_wo[i] + alpha * s_vo[i];
    __syncthreads();
  }

  // ---- row k of A^(k): d_k, and the reflector of column k (its conjugate below the diagonal)
  double xn2 = 0.0;
#pragma unroll
  for (int t = 0; t < TRD_MAXM / 256; ++t) {
    const int c = k + tid + 256 * t;
    T val = xr[t];
    if (c < m && prev) val = val - s_vo[k] * conj(s_wo[c]) - s_wo[k] * conj(s_vo[c]);
    xr[t] = conj(val);
    if (c >= k + 2 && c < m) xn2 += norm2(val);
  }
  if (tid == 0 && blockIdx.x == 0) d[k] = real_part(xr[0]);
  if (k == m - 1) return;
  xn2 = block_sum_fixed(xn2, s_redr);
  // alpha of the reflector: entry k+1 (thread 1 holds it in xr[0]); broadcast through LDS
  if (tid == 1) s_red[0] = xr[0];
  __syncthreads();
  const T al = s_red[0];
  double beta;
  T tk, scale;
  if (xn2 == 0.0 && imag_part(al) == 0.0) {
    beta = real_part(al);
    tk = T(0);
    scale = T(0);
  } else {
    beta = -copysign(sqrt(norm2(al) + xn2), real_part(al));
    tk = cdiv(T(beta) - al, T(beta));
    scale = cdiv(T(1), al - T(beta));
  }
#pragma unroll
  for (int t = 0; t < TRD_MAXM / 256; ++t) {
    const int c = k + tid + 256 * t;
    if (c < m) {
      const T v = (c <= k) ? T(0) : (c == k + 1 ? T(1) : xr[t] * scale);
      if (c > k) s_v[c] = v;
      if (blockIdx.x == 0) {
        vb[(int64_t)(k & 1) * m + c] = v;
        Vh[(int64_t)c * m + k] = v;
      }
    }
  }
  if (blockIdx.x == 0) {
    for (int c = tid; c < k; c += 256) {
      vb[(int64_t)(k & 1) * m + c] = T(0);
      Vh[(int64_t)c * m + k] = T(0);
    }
    if (tid == 0) {
      tau[k] = tk;
      e[k] = beta;
    }
  }
  __syncthreads();

  // ---- rank-2 update of this row and its part of p_k
  if (!has_row) return;
  T acc = T(0);
  const T vr = prev ? s_vo[r] : T(0), wr = prev ? s_wo[r] : T(0);
#pragma unroll
  for (int t = 0; t < TRD_CPL; ++t) {
    const int c = k + 1 + lane + 64 * t;
    if (c < m) {
      T x = a[t];
      if (prev) x = x - vr * conj(s_wo[c]) - wr * conj(s_vo[c]);
      A[(int64_t)r * m + c] = x;
      acc = acc + x * s_v[c];
    }
  }
  acc = wave_sum_fixed(acc);
  if (lane == 0) P[(int64_t)(k & 1) * m + r] = tk * acc;
}

// ---------------------------------------------------------------------------
// Gershgorin bounds of T, the pivot floor of the Sturm counts, and e^2, into LDS.
struct TrdBounds {
  double gl, gu, tnorm, pivmin;
};

__device__ inline TrdBounds trd_bounds(int m, const double* __restrict__ d, const double* __restrict__ e,
                                       double* s_d, double* s_e2, double* s_red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
  for (int j = tid; j < m; j += nt) {
    const double dj = d[j];
    const double ej = j < m - 1 ? e[j] : 0.0, ep = j > 0 ? e[j - 1] : 0.0;
    s_d[j] = dj;
    s_e2[j] = ej * ej;
    const double rad = fabs(ej) + fabs(ep);
    lo = fmin(lo, dj - rad);
    hi = fmax(hi, dj + rad);
    emax = fmax(emax, ej * ej);
  }
  // min / max over the block (exact operations: the order does not matter)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    emax = fmax(emax, __shfl_xor(emax, off));
  }
  const int nw = (nt + 63) / 64;
  if ((tid & 63) == 0) {
    s_red[3 * (tid >> 6)] = lo;
    s_red[3 * (tid >> 6) + 1] = hi;
    s_red[3 * (tid >> 6) + 2] = emax;
  }
  __syncthreads();
  TrdBounds b;
  b.gl = s_red[0];
  b.gu = s_red[1];
  emax = s_red[2];
  for (int w = 1; w < nw; ++w) {
    b.gl = fmin(b.gl, s_red[3 * w]);
    b.gu = fmax(b.gu, s_red[3 * w + 1]);
    emax = fmax(emax, s_red[3 * w + 2]);
  }
  b.tnorm = fmax(fabs(b.gl), fabs(b.gu));
  b.pivmin = DBL_MIN * fmax(1.0, emax);
  const double pad = 2.0 * b.tnorm * DBL_EPSILON * m + 2.0 * b.pivmin;
  b.gl -= pad;
  b.gu += pad;
  return b;
}

// number of eigenvalues of T below x (signs of the pivots of the LDL^T of T - x I)
__device__ inline int sturm_count(int m, const double* s_d, const double* s_e2, double x, double pivmin) {
  double q = s_d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
#pragma unroll 8
  for (int j = 1; j < m; ++j) {
    // e2 / q by the hardware reciprocal and one Newton step (the count only needs the signs
    // of a backward-stable recurrence)
    double rq = __builtin_amdgcn_rcp(q);
    rq = fma(fma(-q, rq, 1.0), rq, rq);
    q = (s_d[j] - x) - s_e2[j - 1] * rq;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// eigenvalue i (ascending) by multisection: lane l counts at lo + (hi - lo)(l + 1)/65
__global__ __launch_bounds__(256) void k_trd_bisect(int m, const double* __restrict__ d, const double* __restrict__ e,
                                                    double* __restrict__ lam) {
  __shared__ double s_d[TRD_MAXM], s_e2[TRD_MAXM], s_red[12];
  const TrdBounds b = trd_bounds(m, d, e, s_d, s_e2, s_red);
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int i = (int)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const double tol = 4.0 * DBL_EPSILON * b.tnorm;
  double lo = b.gl, hi = b.gu;
  for (int round = 0; round < 16 && hi - lo > tol; ++round) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count(m, s_d, s_e2, x, b.pivmin);
    const unsigned long long hit = __ballot(cnt >= i + 1);
    const int l = hit ? __ffsll((long long)hit) - 1 : 64;
    const double nlo = l == 0 ? lo : lo + (hi - lo) * (double)l / 65.0;
    const double nhi = l == 64 ? hi : lo + (hi - lo) * (double)(l + 1) / 65.0;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// counter-hashed start vector entry in (-1, 1)
__device__ inline double trd_start(int i, int r) {
  unsigned long long z = ((unsigned long long)(unsigned)i << 32) ^ (unsigned)r;
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Eigenvectors by inverse iteration; workgroup i handles the group of close eigenvalues
// that starts at i (other workgroups return).  Zt row i = eigenvector i of T.
__global__ __launch_bounds__(64) void k_trd_invit(int m, const double* __restrict__ d, const double* __restrict__ e,
                                                  const double* __restrict__ lam, double* __restrict__ Zt,
                                                  int* __restrict__ flag) {
  __shared__ double s_d[TRD_MAXM], s_e[TRD_MAXM], s_l[TRD_MAXM], s_u0[TRD_MAXM], s_u1[TRD_MAXM],
      s_u2[TRD_MAXM], s_x[TRD_MAXM];
  __shared__ unsigned char s_pv[TRD_MAXM];
  const int i = blockIdx.x, lane = threadIdx.x;
  const double lmax = fmax(fabs(lam[0]), fabs(lam[m - 1]));
  const double thr = 1.0e-10 * lmax;
  if (i > 0 && lam[i] - lam[i - 1] <= thr) return;
  int j1 = i + 1;
  while (j1 < m && lam[j1] - lam[j1 - 1] <= thr) ++j1;
  if (j1 - i > TRD_CLMAX) {
    if (lane == 0) flag[0] = 1;
    return;
  }
  for (int j = lane; j < m; j += 64) {
    s_d[j] = d[j];
    s_e[j] = j < m - 1 ? e[j] : 0.0;
  }
  __syncthreads();
  const double pivtol = lmax > 0.0 ? DBL_EPSILON * lmax : DBL_MIN;
  for (int mb = i; mb < j1; ++mb) {
    const double lm = lam[mb];
    if (lane == 0) {
      // T - lm I = P L U with row interchanges; U has two superdiagonals
      double alpha = s_d[0] - lm, beta = s_e[0];
      // unrolled so that the independent LDS reads of later steps are issued early
#pragma unroll 8
      for (int j = 0; j < m - 1; ++j) {
        const double c = s_e[j], an = s_d[j + 1] - lm, bn = s_e[j + 1];
        if (fabs(alpha) >= fabs(c)) {
          const double l = alpha != 0.0 ? c / alpha : 0.0;
          s_u0[j] = alpha;
          s_u1[j] = beta;
          s_u2[j] = 0.0;
          s_pv[j] = 0;
          s_l[j] = l;
          alpha = an - l * beta;
          beta = bn;
        } else {
          const double l = alpha / c;
          s_u0[j] = c;
          s_u1[j] = an;
          s_u2[j] = bn;
          s_pv[j] = 1;
          s_l[j] = l;
          alpha = beta - l * an;
          beta = -l * bn;
        }
      }
      s_u0[m - 1] = alpha;
#pragma unroll 8
      for (int j = 0; j < m; ++j) {
        const double u = s_u0[j];
        s_u0[j] = 1.0 / (fabs(u) < pivtol ? (u >= 0.0 ? pivtol : -pivtol) : u);
      }
    }
    for (int r = lane; r < m; r += 64) s_x[r] = trd_start(mb, r);
    __syncthreads();
    for (int it = 0; it < 3; ++it) {
      if (lane == 0) {
        // the running entry stays in a register (no LDS store is read back in the chain)
        double cur = s_x[0];
#pragma unroll 8
        for (int j = 0; j < m - 1; ++j) {
          double nxt = s_x[j + 1];
          if (s_pv[j]) {
            const double t = cur;
            cur = nxt;
            nxt = t;
          }
          s_x[j] = cur;
          cur = nxt - s_l[j] * cur;
        }
        s_x[m - 1] = cur;
        double x2 = s_x[m - 1] * s_u0[m - 1];
        s_x[m - 1] = x2;
        double x1 = x2;
        if (m > 1) {
          x1 = (s_x[m - 2] - s_u1[m - 2] * x2) * s_u0[m - 2];
          s_x[m - 2] = x1;
        }
#pragma unroll 8
        for (int j = m - 3; j >= 0; --j) {
          const double x0 = (s_x[j] - s_u1[j] * x1 - s_u2[j] * x2) * s_u0[j];
          s_x[j] = x0;
          x2 = x1;
          x1 = x0;
        }
      }
      __syncthreads();
      // against the earlier vectors of the group, twice
      for (int pass = 0; pass < 2; ++pass)
        for (int q = i; q < mb; ++q) {
          double part = 0.0;
          for (int r = lane; r < m; r += 64) part += Zt[(int64_t)q * m + r] * s_x[r];
          const double dq = wave_sum_fixed(part);
          for (int r = lane; r < m; r += 64) s_x[r] -= dq * Zt[(int64_t)q * m + r];
        }
      double part = 0.0;
      for (int r = lane; r < m; r += 64) part += s_x[r] * s_x[r];
      const double nrm = sqrt(wave_sum_fixed(part));
      const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
      for (int r = lane; r < m; r += 64) s_x[r] *= inv;
      __syncthreads();
    }
    for (int r = lane; r < m; r += 64) Zt[(int64_t)mb * m + r] = s_x[r];
    __syncthreads();
  }
}

// V[r][i] = Zt[i][r] (as T), and evals[i] = lam[i]
template <typename T>
__global__ __launch_bounds__(256) void k_trd_expand(int m, const double* __restrict__ Zt, const double* __restrict__ lam,
                                                    T* __restrict__ V, double* __restrict__ evals) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int i = by + j, r = bx + tx;
    tile[j][tx] = (i < m && r < m) ? Zt[(int64_t)i * m + r] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = bx + j, i = by + tx;
    if (r < m && i < m) V[(int64_t)r * m + i] = T(tile[tx][j]);
  }
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < m; i += 256) evals[i] = lam[i];
}

// compact WY factor of each block of TRD_NB reflectors from its Gram G = V_b^H V_b:
// T[c][c] = tau_c,  T[0:c, c] = -tau_c T[0:c, 0:c] G[0:c, c]
template <typename T>
__global__ __launch_bounds__(64) void k_trd_larft(int nref, const T* __restrict__ tau, const T* __restrict__ G,
                                                  T* __restrict__ Tf) {
  __shared__ T s_t[TRD_NB][TRD_NB + 1];
  const int b = blockIdx.x, k0 = b * TRD_NB, kb = min(TRD_NB, nref - k0);
  const T* g = G + (int64_t)b * TRD_NB * TRD_NB;
  const int j = threadIdx.x;
  if (j < TRD_NB)
    for (int c = 0; c < TRD_NB; ++c) s_t[j][c] = T(0);
  __syncthreads();
  for (int c = 0; c < kb; ++c) {
    const T tc = tau[k0 + c];
    if (j < c) {
      T sacc = T(0);
      for (int l = j; l < c; ++l) sacc = sacc + s_t[j][l] * g[l * TRD_NB + c];
      s_t[j][c] = T(0) - tc * sacc;
    }
    if (j == c) s_t[c][c] = tc;
    __syncthreads();
  }
  if (j < TRD_NB)
    for (int c = 0; c < TRD_NB; ++c) Tf[(int64_t)b * TRD_NB * TRD_NB + j * TRD_NB + c] = s_t[j][c];
}

// ---------------------------------------------------------------------------
static inline size_t trd_align(size_t x) { return (x + 255) & ~(size_t)255; }

struct TrdLayout {
  size_t vh, hc, zt, p, vb, tau, d, e, lam, tf, g, y1, y2, flag, total;
};

static TrdLayout trd_layout(int m, size_t elem) {
  const int nblk = (m - 1 + TRD_NB - 1) / TRD_NB;
  TrdLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o += trd_align(bytes);
    return at;
  };
  L.vh = take(((size_t)m * m + TRD_NB) * elem);  // the last block's Gram reads past column m-1
  L.hc = take((size_t)m * m * elem);
  L.zt = take((size_t)m * m * sizeof(double));
  L.p = take((size_t)2 * m * elem);
  L.vb = take((size_t)2 * m * elem);
  L.tau = take((size_t)m * elem);
  L.d = take((size_t)m * sizeof(double));
  L.e = take((size_t)m * sizeof(double));
  L.lam = take((size_t)m * sizeof(double));
  L.tf = take((size_t)std::max(nblk, 1) * TRD_NB * TRD_NB * elem);
  L.g = take((size_t)std::max(nblk, 1) * TRD_NB * TRD_NB * elem);
  L.y1 = take((size_t)TRD_NB * m * elem);
  L.y2 = take((size_t)TRD_NB * m * elem);
  L.flag = take(256);
  L.total = o;
  return L;
}

size_t tri_work_bytes(int m, size_t elem) { return trd_layout(m, elem).total; }

// row-major C = alpha op(A) B + beta C (as rm_gemm, without a timing region of its own)
template <typename T>
static int trd_gemm(hipStream_t s, int M, int N, int K, const T* A, int64_t lda, bool a_mcontig, const T* B,
                    int64_t ldb, T* C, int64_t ldc, double alpha, double beta) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.a_bs = 0;
  g.B = B; g.ldb = ldb; g.b_bs = 0;
  g.C = C; g.ldc = ldc; g.c_bs = 0;
  g.alpha = alpha; g.beta = beta;
  return gemm<double, is_cplx<T>::value>(s, a_mcontig, a_mcontig, g, 1);
}

template <typename T>
int tri_eigh(hipStream_t s, int m, T* H, T* V, double* evals, char* work, int* fell_back, int* sweeps_out,
             double big_rel) {
  *fell_back = 0;
  if (m < 2 || m > TRD_MAXM) return -2;
  const TrdLayout L = trd_layout(m, sizeof(T));
  T* Vh = reinterpret_cast<T*>(work + L.vh);
  T* Hc = reinterpret_cast<T*>(work + L.hc);
  double* Zt = reinterpret_cast<double*>(work + L.zt);
  T* P = reinterpret_cast<T*>(work + L.p);
  T* vbuf = reinterpret_cast<T*>(work + L.vb);
  T* tau = reinterpret_cast<T*>(work + L.tau);
  double* d = reinterpret_cast<double*>(work + L.d);
  double* e = reinterpret_cast<double*>(work + L.e);
  double* lam = reinterpret_cast<double*>(work + L.lam);
  T* Tf = reinterpret_cast<T*>(work + L.tf);
  T* G = reinterpret_cast<T*>(work + L.g);
  T* Y1 = reinterpret_cast<T*>(work + L.y1);
  T* Y2 = reinterpret_cast<T*>(work + L.y2);
  int* flag = reinterpret_cast<int*>(work + L.flag);
  const size_t mat = (size_t)m * m * sizeof(T);
  MF_HIP_CHECK(hipMemcpyAsync(Hc, H, mat, hipMemcpyDeviceToDevice, s));
  MF_HIP_CHECK(hipMemsetAsync(flag, 0, 4, s));
  MF_HIP_CHECK(hipMemsetAsync(Vh, 0, mat + TRD_NB * sizeof(T), s));  // column m-1 is no reflector
  for (int k = 0; k < m; ++k) {
    const unsigned g = k <= m - 2 ? (unsigned)((m - k - 1 + 3) / 4) : 1u;
    hipLaunchKernelGGL((k_trd_step<T>), dim3(g), dim3(256), 0, s, m, k, H, Vh, P, vbuf, tau, d, e);
  }
  hipLaunchKernelGGL(k_trd_bisect, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, m, d, e, lam);
  hipLaunchKernelGGL(k_trd_invit, dim3((unsigned)m), dim3(64), 0, s, m, d, e, lam, Zt, flag);
  if (hipGetLastError() != hipSuccess) return -2;
  int hflag = 0;
  MF_HIP_CHECK(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
  MF_HIP_CHECK(hipStreamSynchronize(s));
  if (hflag != 0) {
    // a group of nearly equal eigenvalues too large for one workgroup: Jacobi on the copy
    *fell_back = 1;
    MF_HIP_CHECK(hipMemcpyAsync(H, Hc, mat, hipMemcpyDeviceToDevice, s));
    return jacobi_eigh<T>(s, m, H, V, evals, sweeps_out, reinterpret_cast<double*>(work), big_rel);
  }
  MF_HIP_CHECK(hipMemsetAsync(sweeps_out, 0, sizeof(int), s));
  const unsigned nt = (unsigned)((m + 31) / 32);
  hipLaunchKernelGGL((k_trd_expand<T>), dim3(nt, nt), dim3(256), 0, s, m, Zt, lam, V, evals);
  // back-transform X = Q Z: blocks of TRD_NB reflectors, last block first
  const int nref = m - 1;
  const int nblk = (nref + TRD_NB - 1) / TRD_NB;
  {
    // Grams of every block at once (rows of a block above its first reflector are zero)
    GemmArgs g{};
    g.M = TRD_NB; g.N = TRD_NB; g.K = m;
    g.A = Vh; g.lda = m; g.a_bs = TRD_NB;
    g.B = Vh; g.ldb = m; g.b_bs = TRD_NB;
    g.C = G; g.ldc = TRD_NB; g.c_bs = (int64_t)TRD_NB * TRD_NB;
    g.alpha = 1.0; g.beta = 0.0;
    if (gemm<double, is_cplx<T>::value>(s, true, true, g, nblk)) return -2;
  }
  hipLaunchKernelGGL((k_trd_larft<T>), dim3((unsigned)nblk), dim3(64), 0, s, nref, tau, G, Tf);
  for (int b = nblk - 1; b >= 0; --b) {
    const int k0 = b * TRD_NB, kb = std::min(TRD_NB, nref - k0);
    const int rows = m - k0 - 1;
    const T* Vb = Vh + (int64_t)(k0 + 1) * m + k0;
    T* Vr = V + (int64_t)(k0 + 1) * m;
    MF_TRY(trd_gemm<T>(s, kb, m, rows, Vb, m, true, Vr, m, Y1, m, 1.0, 0.0));  // V_b^H X
    MF_TRY(trd_gemm<T>(s, kb, m, kb, Tf + (int64_t)b * TRD_NB * TRD_NB, TRD_NB, false, Y1, m, Y2, m, 1.0, 0.0));
    MF_TRY(trd_gemm<T>(s, rows, m, kb, Vb, m, false, Y2, m, Vr, m, -1.0, 1.0));  // X -= V_b T V_b^H X
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int tri_eigh<double>(hipStream_t, int, double*, double*, double*, char*, int*, int*, double);
template int tri_eigh<c64>(hipStream_t, int, c64*, c64*, double*, char*, int*, int*, double);

}  // namespace mf
