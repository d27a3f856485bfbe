// Block two-sided Jacobi eigensolver for the reduced Hermitian problem (gfx950).
//
// The m x m matrix (m up to 1024) is split into blocks of JB indices (8 by default,
// 16 selectable).  Every round pairs the blocks with the round-robin (circle)
// ordering; each pair (P, Q) forms a 2JB x 2JB Hermitian subproblem
// [H_PP H_PQ; H_QP H_QQ] on which one workgroup runs one cyclic Jacobi sweep in LDS
// (its own round-robin ordering of the 2JB local indices), giving a unitary
// U_PQ.  The round's U's are then applied: every super-block H[I_i, I_j] becomes
// U_i^H H[I_i, I_j] U_j (the pairs of a round are disjoint, so the super-blocks update
// independently) and V[:, I_j] becomes V[:, I_j] U_j.  Only the 2 npr super-blocks that
// the next round's subproblems read get a launch of their own between the rounds; the
// other super-blocks and V are updated by spare workgroups of the next round's
// subproblem launch (which never touches them).  A sweep covers every block pair once;
// sweeps stop when no subproblem needed a rotation.
#include <cstdlib>

#include "kernels.hpp"

namespace mf {

constexpr int JT = 256;      // threads per workgroup

template <typename T> __device__ inline double absv(T a);
template <> __device__ inline double absv<double>(double a) { return fabs(a); }
template <> __device__ inline double absv<c64>(c64 a) { return sqrt(a.re * a.re + a.im * a.im); }

template <typename T>
__device__ inline T sgn_phase(T b, double ab);
template <> __device__ inline double sgn_phase<double>(double b, double ab) { return b >= 0 ? 1.0 : -1.0; }
template <> __device__ inline c64 sgn_phase<c64>(c64 b, double ab) { return c64(b.re / ab, b.im / ab); }

// 1/sqrt(x) and 1/x for x > 0 from the hardware approximations plus three Newton steps
// (each step squares the relative error, so full FP64 accuracy from any start within
// about 1e-3)
__device__ inline double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
#pragma unroll
  for (int k = 0; k < 3; ++k) y = y * fma(-0.5 * x * y, y, 1.5);
  return y;
}
__device__ inline double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int k = 0; k < 3; ++k) y = y * fma(-x, y, 2.0);
  return y;
}

// block pair of round r, circle method over nbp (even) block indices
__device__ inline void block_pair(int i, int r, int nbp, int& P, int& Q) {
  const int a = (i == 0) ? 0 : 1 + (i - 1 + r) % (nbp - 1);
  const int b = 1 + (nbp - 2 - i + r) % (nbp - 1);
  P = min(a, b);
  Q = max(a, b);
}

// global index of local index l (0..2 JB - 1) of the subproblem of blocks (P, Q)
template <int JB>
__device__ inline int gidx(int l, int P, int Q) { return l < JB ? P * JB + l : Q * JB + (l - JB); }

// ---------------------------------------------------------------------------
// rotation of local pair (p, q) from the 2 x 2 diagonal block of S: c real, s complex
template <typename T>
__device__ inline int jrot(double app, double aqq, T apq, double tol, double abs_floor, double big_floor, double& c,
                           T& sg) {
  double ab2;
  if constexpr (is_cplx<T>::value) ab2 = apq.re * apq.re + apq.im * apq.im;
  else ab2 = apq * apq;
  c = 1.0;
  sg = T(0.0);
  if (!(ab2 > tol * tol * fabs(app * aqq) && ab2 > abs_floor * abs_floor)) return 0;
  const double inv_ab = rsqrt_nr(ab2);
  const T ph = inv_ab * apq;
  const double tau = (aqq - app) * 0.5 * inv_ab;
  double t;
  if (fabs(tau) > 1e150) {
    t = 0.5 * rcp_nr(tau);
  } else {
    const double u = fma(tau, tau, 1.0);
    const double h = u * rsqrt_nr(u);
    t = (tau >= 0 ? 1.0 : -1.0) * rcp_nr(fabs(tau) + h);
  }
  c = rsqrt_nr(fma(t, t, 1.0));
  sg = (t * c) * ph;
  return (ab2 > big_floor * big_floor) ? 2 : 1;
}

// local pair i of round r (circle method over JS indices)
template <int JS>
__device__ inline void local_pair(int i, int r, int& p, int& q) {
  const int a = (i == 0) ? 0 : 1 + (i - 1 + r) % (JS - 1);
  const int b = 1 + (JS - 2 - i + r) % (JS - 1);
  p = min(a, b);
  q = max(a, b);
}

// V[:, I_j] <- V[:, I_j] U_j for the pairs j of round `round`: item bid covers row block
// bid / npr (JS rows) and pair bid % npr; X and Um are LDS tiles of the caller.
template <typename T, int JB>
__device__ inline void bj_v_update(int m, int nbp, int round, int bid, T* __restrict__ V, const T* __restrict__ Ubuf,
                                   T (*X)[2 * JB + 1], T (*Um)[2 * JB + 1]) {
  constexpr int JS = 2 * JB;
  constexpr int RW = JS / 16;
  const int tid = threadIdx.x;
  const int npr = nbp / 2;
  const int r0 = (tid >> 4) * RW, c0 = (tid & 15) * RW;
  T acc[RW][RW];
  {
    const int j = bid % npr;
    const int xb = bid / npr;  // row block of JS rows of V
    int Pj, Qj;
    block_pair(j, round, nbp, Pj, Qj);
    const T* Uj = Ubuf + (int64_t)j * JS * JS;
    for (int e = tid; e < JS * JS; e += JT) {
      const int a = e / JS, c = e % JS;
      const int ga = xb * JS + a, gc = gidx<JB>(c, Pj, Qj);
      X[a][c] = (ga < m && gc < m) ? V[(int64_t)ga * m + gc] : T(0.0);
      Um[a][c] = Uj[e];
    }
    __syncthreads();
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) acc[a][c] = T(0.0);
    for (int k = 0; k < JS; ++k) {
      T xa[RW], ub[RW];
      for (int a = 0; a < RW; ++a) xa[a] = X[r0 + a][k];
      for (int c = 0; c < RW; ++c) ub[c] = Um[k][c0 + c];
      for (int a = 0; a < RW; ++a)
        for (int c = 0; c < RW; ++c) acc[a][c] = acc[a][c] + xa[a] * ub[c];
    }
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) {
        const int ga = xb * JS + r0 + a, gc = gidx<JB>(c0 + c, Pj, Qj);
        if (ga < m && gc < m) V[(int64_t)ga * m + gc] = acc[a][c];
      }
  }
}

// H[I_i, I_j] <- U_i^H H[I_i, I_j] U_j for the pairs i <= j of round `round` (the (j, i)
// block is written as the conjugate transpose); X, Um and Ui_s are LDS tiles of the caller
// (the block and both unitaries are loaded together, one global round trip).
template <typename T, int JB>
__device__ inline void bj_h_update(int m, int nbp, int round, int i, int j, T* __restrict__ H,
                                   const T* __restrict__ Ubuf, T (*X)[2 * JB + 1], T (*Um)[2 * JB + 1],
                                   T (*Ui_s)[2 * JB + 1]) {
  constexpr int JS = 2 * JB;
  constexpr int RW = JS / 16;  // rows (and columns) of the result per thread: 16 x 16 threads
  const int tid = threadIdx.x;
  // each thread owns an RW x RW tile of the JS x JS result
  const int r0 = (tid >> 4) * RW, c0 = (tid & 15) * RW;
  T acc[RW][RW];
  {
    int Pi, Qi, Pj, Qj;
    block_pair(i, round, nbp, Pi, Qi);
    block_pair(j, round, nbp, Pj, Qj);
    const T* Ui = Ubuf + (int64_t)i * JS * JS;
    const T* Uj = Ubuf + (int64_t)j * JS * JS;
    for (int e = tid; e < JS * JS; e += JT) {
      const int a = e / JS, c = e % JS;
      const int ga = gidx<JB>(a, Pi, Qi), gc = gidx<JB>(c, Pj, Qj);
      X[a][c] = (ga < m && gc < m) ? H[(int64_t)ga * m + gc] : T(0.0);
      Um[a][c] = Uj[e];
      Ui_s[a][c] = Ui[e];
    }
    __syncthreads();
    // T = X Uj
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) acc[a][c] = T(0.0);
    for (int k = 0; k < JS; ++k) {
      T xa[RW], ub[RW];
      for (int a = 0; a < RW; ++a) xa[a] = X[r0 + a][k];
      for (int c = 0; c < RW; ++c) ub[c] = Um[k][c0 + c];
      for (int a = 0; a < RW; ++a)
        for (int c = 0; c < RW; ++c) acc[a][c] = acc[a][c] + xa[a] * ub[c];
    }
    __syncthreads();
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) X[r0 + a][c0 + c] = acc[a][c];
    __syncthreads();
    // out = Ui^H T
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) acc[a][c] = T(0.0);
    for (int k = 0; k < JS; ++k) {
      T ua[RW], xb[RW];
      for (int a = 0; a < RW; ++a) ua[a] = conj(Ui_s[k][r0 + a]);
      for (int c = 0; c < RW; ++c) xb[c] = X[k][c0 + c];
      for (int a = 0; a < RW; ++a)
        for (int c = 0; c < RW; ++c) acc[a][c] = acc[a][c] + ua[a] * xb[c];
    }
    for (int a = 0; a < RW; ++a)
      for (int c = 0; c < RW; ++c) {
        const int ga = gidx<JB>(r0 + a, Pi, Qi), gc = gidx<JB>(c0 + c, Pj, Qj);
        if (ga < m && gc < m) {
          H[(int64_t)ga * m + gc] = acc[a][c];
          if (i != j) H[(int64_t)gc * m + ga] = conj(acc[a][c]);
        }
      }
  }
}

// Pair of round r that holds block x (inverse of block_pair: the circle keeps block 0
// in pair 0 and rotates the others through R = nbp - 1 positions).
__device__ inline int bj_pair_of(int x, int r, int nbp) {
  if (x == 0) return 0;
  const int R = nbp - 1, npr = nbp / 2;
  const int d = ((x - 1 - r) % R + R) % R;
  return d <= npr - 2 ? d + 1 : R - 1 - d;
}

// Super-block (i, j), i <= j, of round r is read by the subproblems of the next round rn
// (before which it must be updated) if i == j or some pair of round rn joins a block of
// pair i with one of pair j.  The others can be updated beside those subproblems.
__device__ inline bool bj_sb_critical(int i, int j, int r, int rn, int nbp) {
  if (i == j) return true;
  int ai, bi, aj, bj, pa, qa, pb, qb;
  block_pair(i, r, nbp, ai, bi);
  block_pair(j, r, nbp, aj, bj);
  block_pair(bj_pair_of(ai, rn, nbp), rn, nbp, pa, qa);
  block_pair(bj_pair_of(bi, rn, nbp), rn, nbp, pb, qb);
  const int na = pa == ai ? qa : pa, nb = pb == bi ? qb : pb;  // next-round partners
  return na == aj || na == bj || nb == aj || nb == bj;
}

// (i, j), i <= j, from the linear index of the npr (npr + 1) / 2 super-blocks
__device__ inline void bj_sb_index(int bid, int npr, int& i, int& j) {
  i = 0;
  while (bid >= npr - i) {
    bid -= npr - i;
    ++i;
  }
  j = i + bid;
}

// One cyclic sweep of the 2JB x 2JB subproblem.  S is double-buffered so that a round
// needs one barrier: every thread computes the one or two rotations its own items need
// from the current buffer (redundantly with other threads) and writes the rotated
// values to the other buffer.  Items: the (JS/2)^2 2 x 2 blocks of S and the JS x JS/2
// column pairs of U.
// Workgroups [0, nsub) run the subproblems of round `round`; the ones after them finish
// the previous round `vround` with its unitaries Uv: first V (read by no subproblem),
// then the super-blocks of H that no subproblem of `round` reads (the others were
// updated before this launch), so that only the latter lie on the path between rounds.
template <typename T, int JB>
__global__ __launch_bounds__(256) void k_bj_sub(int m, int nbp, int round, int nsub, T* __restrict__ H,
                                                T* __restrict__ Ubuf, int* __restrict__ rotcount, double tol,
                                                double big_rel, int vround, T* __restrict__ V,
                                                const T* __restrict__ Uv) {
  constexpr int JS = 2 * JB;
  constexpr int NSI = (JS / 2) * (JS / 2), NUI = JS * (JS / 2);
  __shared__ T S[2][JS][JS + 1];
  __shared__ T U[JS][JS + 1];
  __shared__ int s_total;
  __shared__ double s_dmax;
  if ((int)blockIdx.x >= nsub) {
    const int npr = nbp / 2;
    const int nvi = ((m + JS - 1) / JS) * npr;
    const int b = (int)blockIdx.x - nsub;
    if (b < nvi) {
      bj_v_update<T, JB>(m, nbp, vround, b, V, Uv, S[0], S[1]);
    } else {
      int i, j;
      bj_sb_index(b - nvi, npr, i, j);
      if (!bj_sb_critical(i, j, vround, (vround + 1) % (nbp - 1), nbp))
        bj_h_update<T, JB>(m, nbp, vround, i, j, H, Uv, S[0], S[1], U);
    }
    return;
  }
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  int P, Q;
  block_pair(blockIdx.x, round, nbp, P, Q);
  for (int e = tid; e < JS * JS; e += nt) {
    const int a = e / JS, c = e % JS;
    const int ga = gidx<JB>(a, P, Q), gc = gidx<JB>(c, P, Q);
    S[0][a][c] = (ga < m && gc < m) ? H[(int64_t)ga * m + gc] : T(0.0);
    U[a][c] = (a == c) ? T(1.0) : T(0.0);
  }
  if (tid == 0) s_total = 0;
  __syncthreads();
  if (tid < 64) {
    double d = tid < JS ? fabs(real_part(S[0][tid][tid])) : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d = fmax(d, __shfl_xor(d, off));
    if (tid == 0) s_dmax = d;
  }
  __syncthreads();
  const double abs_floor = 4.440892098500626e-16 * s_dmax + 1e-300;
  const double big_floor = big_rel * s_dmax;
  int my_big = 0;
  int cur = 0;
  for (int r = 0; r < JS - 1; ++r) {
    for (int e = tid; e < NSI + NUI; e += nt) {
      if (e < NSI) {
        const int Pi = e / (JS / 2), Qi = e % (JS / 2);
        int p1, q1, p2, q2;
        local_pair<JS>(Pi, r, p1, q1);
        local_pair<JS>(Qi, r, p2, q2);
        double cP, cQ;
        T sP, sQ;
        const int fP = jrot<T>(real_part(S[cur][p1][p1]), real_part(S[cur][q1][q1]), S[cur][p1][q1], tol, abs_floor,
                               big_floor, cP, sP);
        const int fQ = (Qi == Pi) ? fP
                                  : jrot<T>(real_part(S[cur][p2][p2]), real_part(S[cur][q2][q2]), S[cur][p2][q2],
                                            tol, abs_floor, big_floor, cQ, sQ);
        if (Qi == Pi) {
          cQ = cP;
          sQ = sP;
          my_big += (fP == 2) ? 1 : 0;
        }
        const T h11 = S[cur][p1][p2], h12 = S[cur][p1][q2], h21 = S[cur][q1][p2], h22 = S[cur][q1][q2];
        T o11 = h11, o12 = h12, o21 = h21, o22 = h22;
        if (fP || fQ) {
          const T t11 = cQ * h11 - h12 * conj(sQ);
          const T t12 = h11 * sQ + cQ * h12;
          const T t21 = cQ * h21 - h22 * conj(sQ);
          const T t22 = h21 * sQ + cQ * h22;
          o11 = cP * t11 - sP * t21;
          o12 = cP * t12 - sP * t22;
          o21 = conj(sP) * t11 + cP * t21;
          o22 = conj(sP) * t12 + cP * t22;
        }
        S[cur ^ 1][p1][p2] = o11;
        S[cur ^ 1][p1][q2] = o12;
        S[cur ^ 1][q1][p2] = o21;
        S[cur ^ 1][q1][q2] = o22;
      } else {
        const int u = e - NSI;
        const int x = u / (JS / 2), Qi = u % (JS / 2);
        int p2, q2;
        local_pair<JS>(Qi, r, p2, q2);
        double cQ;
        T sQ;
        if (jrot<T>(real_part(S[cur][p2][p2]), real_part(S[cur][q2][q2]), S[cur][p2][q2], tol, abs_floor, big_floor,
                    cQ, sQ)) {
          const T a = U[x][p2], b = U[x][q2];
          U[x][p2] = cQ * a - b * conj(sQ);
          U[x][q2] = a * sQ + cQ * b;
        }
      }
    }
    cur ^= 1;
    __syncthreads();
  }
  if (my_big) atomicAdd(&s_total, my_big);
  __syncthreads();
  T* Uo = Ubuf + (int64_t)blockIdx.x * JS * JS;
  for (int e = tid; e < JS * JS; e += nt) Uo[e] = U[e / JS][e % JS];
  if (tid == 0 && s_total > 0) atomicAdd(rotcount, s_total);
}

// ---------------------------------------------------------------------------
// The super-blocks of round `round` that the next round's subproblems read: 2 npr
// workgroups, (b, b) for b < npr, then per next-round pair the super-block that couples
// its two blocks (none when both lie in one pair, which only happens for a single pair).
template <typename T, int JB>
__global__ __launch_bounds__(JT) void k_bj_upd(int m, int nbp, int round, int rn, T* __restrict__ H,
                                               const T* __restrict__ Ubuf) {
  constexpr int JS = 2 * JB;
  __shared__ T X[JS][JS + 1];
  __shared__ T Um[JS][JS + 1];
  __shared__ T Ui_s[JS][JS + 1];
  const int npr = nbp / 2;
  const int b = blockIdx.x;
  if (b < npr) {
    bj_h_update<T, JB>(m, nbp, round, b, b, H, Ubuf, X, Um, Ui_s);
    return;
  }
  int P, Q;
  block_pair(b - npr, rn, nbp, P, Q);
  const int i = bj_pair_of(P, round, nbp), j = bj_pair_of(Q, round, nbp);
  if (i == j) return;
  // two next-round pairs can couple the same two pairs of this round (with four blocks both
  // do): only the first of them updates that super-block, or two workgroups would rotate
  // the same entries at once
  for (int t = 0; t < b - npr; ++t) {
    int Pt, Qt;
    block_pair(t, rn, nbp, Pt, Qt);
    const int it = bj_pair_of(Pt, round, nbp), jt = bj_pair_of(Qt, round, nbp);
    if (min(it, jt) == min(i, j) && max(it, jt) == max(i, j)) return;
  }
  bj_h_update<T, JB>(m, nbp, round, min(i, j), max(i, j), H, Ubuf, X, Um, Ui_s);
}

template <typename T>
__global__ void k_identity(int m, T* V) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j < m) V[(int64_t)i * m + j] = (i == j) ? T(1.0) : T(0.0);
}

template <typename T>
__global__ void k_diag_out(int m, const T* __restrict__ H, double* evals, int* counter) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) evals[i] = real_part(H[(int64_t)i * m + i]);
  if (i == 0) counter[0] = 0;
}

__global__ void k_zero_int(int* p) { *p = 0; }

// H (m x m) destroyed; V receives the eigenvectors (columns), evals the eigenvalues
// (unsorted).  ubuf: 2 (2 JB)^2 (nbp/2) entries of T for two rounds' unitaries; counter:
// 2 ints.
template <typename T, int JB>
static int block_jacobi_jb(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps_out, T* ubuf, int* counter,
                           int max_sweeps, double big_rel) {
  constexpr int JS = 2 * JB;
  const int nb = (m + JB - 1) / JB;
  const int nbp = nb + (nb & 1);
  const int npr = nbp / 2;
  const int nh = npr * (npr + 1) / 2;
  const int nvrow = (m + JS - 1) / JS;
  const int nvi = nvrow * npr;  // V items of one round
  // the unitaries alternate between two buffers: round g's subproblems write Ub[g % 2]
  // while the V items of round g - 1 in the same launch read Ub[(g - 1) % 2]
  T* Ub[2] = {ubuf, ubuf + (size_t)JS * JS * npr};
  hipLaunchKernelGGL((k_identity<T>), dim3((m + 255) / 256, m), dim3(256), 0, s, m, V);
  int sweep = 0;
  int hcount = 1;
  int g = 0;
  int vpend = -1;  // round whose V items are still to run (the last round of the last sweep)
  for (; sweep < max_sweeps; ++sweep) {
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, counter);
    const int nr = nbp - 1;
    hipLaunchKernelGGL((k_bj_sub<T, JB>), dim3(npr + (vpend >= 0 ? nvi + nh : 0)), dim3(JT), 0, s, m, nbp, 0, npr,
                       H, Ub[g & 1], counter, 1.0e-15, big_rel, vpend, V, Ub[(g + 1) & 1]);
    for (int r = 0; r < nr; ++r, ++g) {
      hipLaunchKernelGGL((k_bj_upd<T, JB>), dim3(2 * npr), dim3(JT), 0, s, m, nbp, r, (r + 1) % nr, H, Ub[g & 1]);
      if (r + 1 < nr) {
        hipLaunchKernelGGL((k_bj_sub<T, JB>), dim3(npr + nvi + nh), dim3(JT), 0, s, m, nbp, r + 1, npr, H,
                           Ub[(g + 1) & 1], counter, 1.0e-15, big_rel, r, V, Ub[g & 1]);
      } else {
        vpend = r;
      }
    }
    if (hipMemcpyAsync(&hcount, counter, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
    if (hipStreamSynchronize(s) != hipSuccess) return -2;
    if (hcount == 0) break;
  }
  if (vpend >= 0)
    hipLaunchKernelGGL((k_bj_sub<T, JB>), dim3(nvi + nh), dim3(JT), 0, s, m, nbp, 0, 0, H, Ub[g & 1], counter,
                       1.0e-15, big_rel, vpend, V, Ub[(g + 1) & 1]);
  hipLaunchKernelGGL((k_diag_out<T>), dim3((m + 255) / 256), dim3(256), 0, s, m, H, evals, counter + 1);
  int sw = sweep + 1;
  if (hipMemcpyAsync(sweeps_out, &sw, sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) return -2;
  if (hipStreamSynchronize(s) != hipSuccess) return -2;
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

static int bj_width() {
  // 8-wide blocks measured fastest at M0 = 600: a 16 x 16 subproblem needs 15 inner
  // rounds instead of 31, which outweighs the doubled number of outer rounds
  static const int w = getenv("MFEAST_BJ_WIDTH") ? atoi(getenv("MFEAST_BJ_WIDTH")) : 8;
  return w == 16 ? 16 : 8;
}

template <typename T>
int block_jacobi(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps_out, T* ubuf, int* counter,
                 int max_sweeps, double big_rel) {
  if (bj_width() == 8)
    return block_jacobi_jb<T, 8>(s, m, H, V, evals, sweeps_out, ubuf, counter, max_sweeps, big_rel);
  return block_jacobi_jb<T, 16>(s, m, H, V, evals, sweeps_out, ubuf, counter, max_sweeps, big_rel);
}

size_t block_jacobi_work_bytes(int m, size_t elem) {
  // two sets of round unitaries for either block width, then the counters
  const int nb8 = (m + 7) / 8, nb16 = (m + 15) / 16;
  const size_t u8 = (size_t)256 * ((nb8 + (nb8 & 1)) / 2), u16 = (size_t)1024 * ((nb16 + (nb16 & 1)) / 2);
  return 2 * (u8 > u16 ? u8 : u16) * elem + 64;
}

template int block_jacobi<double>(hipStream_t, int, double*, double*, double*, int*, double*, int*, int, double);
template int block_jacobi<c64>(hipStream_t, int, c64*, c64*, double*, int*, c64*, int*, int, double);

}  // namespace mf
