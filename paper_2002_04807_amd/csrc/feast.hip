// Host side of the Hermitian FEAST contour-integration subspace iteration (C interface).
//
// One call runs the whole method of the FEAST v4.0 guide for a Hermitian (real
// symmetric) pencil, every numerical step in the HIP kernels of this library.  The
// subspace loop (feast_loop) is shared by two matrix formats, each an Operator:
//   dense     Az_j = z_j B - A for every node, blocked LU with partial pivoting,
//             factors kept for all iterations (RCI case 10, fpm(10)=1); solves by
//             blocked triangular products (cases 11 and 21)
//   CSR       no factorization (IFEAST, Section 3.5): every shifted system solved
//             inexactly by BiCGSTAB, all nodes and right-hand sides batched
// The loop:
//   contour   iteration 0: solve Az_j Q_j = B Y for the starting block Y (case 11,
//             and case 21 with Az_j^H for complex Hermitian problems);
//             iteration k > 0: residual inverse iteration (v4.0, Section 1.2 and the
//             Tips of Section 3.1): only R = A X - B X Lambda (FP64) is solved and
//             Q = X diag(rho(Lambda)) + sum_j [w_j d_j diag(1/(z_j - lambda)) + ...],
//             so that FP32 solves (fpm(42)=1) keep FP64 accuracy
//   RR        A Q, B Q (cases 30/40), Aq = Q^H A Q, Bq = Q^H B Q, reduced eigenproblem,
//             X = Q W, residuals res_i = ||A x_i - lambda_i B x_i|| / ||alpha B x_i||
//   stop      M = #lambda in [Emin, Emax]; converged when max_{i<=M} res_i < 10^-fpm(3)
//             (fpm(6)=1) or epsout < 10^-fpm(3) (fpm(6)=0); fpm(4) bounds the loops.
// The host only sequences launches and reads back O(M0) scalars per iteration.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdlib>
#include <thread>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/mfeast.h"
#include "ctx.hpp"
#include "kernels.hpp"

using namespace mf;

namespace {

constexpr double RANK_TOL = 1.0e-13;  // kept directions of the equilibrated overlap: s > RANK_TOL * max s
// Ritz values inside the interval with a relative residual at or above this bound, or
// above the Kato-Temple bound of the interval (see the found-pair test), are spurious
// (mixtures of weakly filtered eigenvectors from both sides of the interval) and are not
// counted among the M eigenvalues found.
constexpr double SPURIOUS_RES = 1.0e-1;
// Sizes the kernels support: the dense LU up to n = 16384 rows, the reduced eigensolver up
// to M0 = 1024 (larger values are reported as invalid N / M0, Table tab_info 202 / 201)
constexpr int64_t MAX_DENSE_N = 16384;
constexpr int MAX_M0 = 1024;

}  // namespace

// ---------------------------------------------------------------------------
// contour (host, FP64): Gauss-Legendre nodes by Newton iteration on P_n
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    // initial guess for the i-th largest root, refined by Newton's method
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = (n == 1) ? 1.0 : n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[n - 1 - i] = z;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

static bool gauss_allowed(int ne) {
  return (ne >= 1 && ne <= 20) || ne == 24 || ne == 32 || ne == 40 || ne == 48 || ne == 56;
}

// nodes z_j and half-contour weights w_j on the ellipse through emin, emax (see mfeast.h)
static void make_contour(double emin, double emax, int ne, int rule, int ratio_pct, std::vector<c64>& z,
                         std::vector<c64>& w) {
  const double c = 0.5 * (emin + emax), r = 0.5 * (emax - emin), e = ratio_pct / 100.0;
  z.resize(ne);
  w.resize(ne);
  std::vector<double> x, om;
  if (rule == 0) gauss_legendre(ne, x, om);
  for (int j = 0; j < ne; ++j) {
    double th, sc;
    if (rule == 0) {
      th = 0.5 * M_PI * (1.0 - x[j]);
      sc = om[j] / 4.0;
    } else {
      th = M_PI * (ne - (j + 1) + 0.5) / ne;
      sc = 1.0 / (2.0 * ne);
    }
    z[j] = c64(c + r * std::cos(th), e * r * std::sin(th));
    w[j] = c64(sc * e * r * std::cos(th), sc * r * std::sin(th));
  }
}

// ---------------------------------------------------------------------------
// Zolotarev rule (fpm(16) = 2; the guide cites Guettel, Polizzi, Tang and Viaud 2015 and
// prints no construction).  Zolotarev's best approximation of sign(x) on [-1,-l] u [l,1]
// of odd type (2m-1, 2m),
//   Z(x) = C x prod_{q<m} (x^2 + c_{2q}) / prod_{q<=m} (x^2 + c_{2q-1}),
//   c_i = l^2 sn^2(i K'/(2m); l') / cn^2(i K'/(2m); l'),   l' = sqrt(1 - l^2),
// equioscillates on [l, 1] at x_k = l / dn(k K'/(2m); l'); the filter of the interval
// is f(t) = (1 + Z(kappa (1 + t)/(1 - t)))/2 in t = (lambda - c)/r, with kappa =
// (1 - a)/(1 + a), l = kappa^2 and a = fpm(54)/100 the half-width (relative) inside
// which f stays within delta/2 of 1 (and beyond 1/a within delta/2 of 0).  Its m poles
// in the upper half plane lie on the unit circle; partial fractions give the nodes, the
// half-contour weights and the constant term f(inf) = (1 + Z(-kappa))/2.

// Jacobi elliptic functions of modulus k = sqrt(1 - kp^2), given by its complementary
// modulus kp (0 < kp <= 1, exact for moduli near 1), by the arithmetic-geometric mean
// (descending Landen) method; also K(k) = pi / (2 a_N).
static void jacobi_agm(double u, double kp, double& sn, double& cn, double& dn, double* Kout) {
  double a[64], c[64];
  a[0] = 1.0;
  double b = kp;
  c[0] = std::sqrt((1.0 - kp) * (1.0 + kp));
  int N = 0;
  while (N < 62 && std::fabs(c[N]) > 1e-17 * a[N]) {
    a[N + 1] = 0.5 * (a[N] + b);
    c[N + 1] = 0.5 * (a[N] - b);
    b = std::sqrt(a[N] * b);
    ++N;
  }
  if (Kout) *Kout = M_PI / (2.0 * a[N]);
  double phi = std::ldexp(a[N] * u, N), phi1 = phi;
  for (int n = N; n >= 1; --n) {
    phi1 = phi;
    phi = 0.5 * (phi + std::asin(c[n] * std::sin(phi) / a[n]));
  }
  sn = std::sin(phi);
  cn = std::cos(phi);
  dn = (N >= 1) ? cn / std::cos(phi1 - phi) : 1.0;
}

// x prod_{q<m} (x^2 + c_{2q}) / prod_{q<=m} (x^2 + c_{2q-1}) as a product of ratios
// (cs[i] = c_{i+1})
static std::complex<double> zolo_product(std::complex<double> x, const std::vector<double>& cs, int m) {
  std::complex<double> out = x / (x * x + cs[2 * m - 2]);
  for (int q = 1; q < m; ++q) out *= (x * x + cs[2 * q - 1]) / (x * x + cs[2 * q - 2]);
  return out;
}

static void zolotarev_contour(double emin, double emax, int m, int band_pct, std::vector<c64>& z,
                              std::vector<c64>& w, double& c_inf) {
  const double a = band_pct / 100.0;
  const double kappa = (1.0 - a) / (1.0 + a);
  const double l = kappa * kappa;  // the modulus of the functions is l', its complement l
  double sn, cn, dn, Kp;
  jacobi_agm(0.0, l, sn, cn, dn, &Kp);
  // c_i for i <= m from the functions; c_{2m-i} = l^2 / c_i (quarter-period reflection),
  // which keeps the large coefficients accurate
  std::vector<double> cs(2 * m - 1);
  for (int i = 1; i <= m && i <= 2 * m - 1; ++i) {
    jacobi_agm(i * Kp / (2.0 * m), l, sn, cn, dn, nullptr);
    cs[i - 1] = l * l * sn * sn / (cn * cn);
  }
  for (int i = m + 1; i <= 2 * m - 1; ++i) cs[i - 1] = l * l / cs[2 * m - i - 1];
  // normalization from the first two alternation points x_0 = l, x_1 = l / dn(K'/(2m))
  jacobi_agm(Kp / (2.0 * m), l, sn, cn, dn, nullptr);
  const double z0 = zolo_product(l, cs, m).real(), z1 = zolo_product(l / dn, cs, m).real();
  const double C = 2.0 / (z0 + z1);
  const double cen = 0.5 * (emin + emax), r = 0.5 * (emax - emin);
  std::vector<std::pair<double, std::pair<c64, c64>>> nodes;
  for (int q = 0; q < m; ++q) {
    const double p = cs[2 * q];  // c_{2q+1}: the squared modulus of this pole pair
    // residue of Z at i sqrt(p): C N(-p) / (2 D'(-p)), as a product of ratios
    double ratio = 1.0;
    int e = 0;
    for (int o = 0; o < m; ++o) {
      if (o == q) continue;
      ratio *= (cs[2 * e + 1] - p) / (cs[2 * o] - p);
      ++e;
    }
    const double res_x = C * ratio / 2.0;
    const double y = std::sqrt(p) / kappa;
    const std::complex<double> tq((y * y - 1.0) / (y * y + 1.0), 2.0 * y / (y * y + 1.0));
    const std::complex<double> res_t = 0.5 * res_x * (1.0 - tq) * (1.0 - tq) / (2.0 * kappa);
    const std::complex<double> zq = cen + r * tq, wq = -r * res_t;
    nodes.push_back({tq.real(), {c64(zq.real(), zq.imag()), c64(wq.real(), wq.imag())}});
  }
  std::stable_sort(nodes.begin(), nodes.end(),
                   [](const std::pair<double, std::pair<c64, c64>>& A, const std::pair<double, std::pair<c64, c64>>& B) {
                     return A.first < B.first;
                   });
  z.resize(m);
  w.resize(m);
  for (int q = 0; q < m; ++q) {
    z[q] = nodes[q].second.first;
    w[q] = nodes[q].second.second;
  }
  c_inf = 0.5 * (1.0 + C * zolo_product(-kappa, cs, m).real());
}

// ---------------------------------------------------------------------------
// argument checks shared by the dense drivers (Table tab_info order)
static int check_fpm(const int32_t* fpm, bool expert) {
  auto f = [&](int i) { return fpm[i - 1]; };
  if (!expert) {
    if (f(16) < 0 || f(16) > 2) return 116;
    if ((f(16) == 0 || f(16) == 2) && !gauss_allowed(f(2))) return 102;
    if (f(16) == 1 && f(2) < 1) return 102;
    if (f(18) <= 0) return 118;
    if (f(16) == 2 && (f(54) < 1 || f(54) > 99)) return 154;
  } else if (f(2) < 1) {
    return 102;
  }
  if (f(3) < 0 || f(3) > 16) return 103;
  if (f(4) < 0) return 104;
  if (f(5) != 0 && f(5) != 1) return 105;
  if (f(6) != 0 && f(6) != 1) return 106;
  if (f(14) < 0 || f(14) > 2) return 114;
  if (f(42) != 0 && f(42) != 1) return 142;
  if (f(50) < 0 || f(50) > 8) return 150;
  if (f(53) != 0 && f(53) != 1) return 153;
  return 0;
}

// reduced eigensolver call, timed as its own class.  Algorithmic work of a two-sided
// Jacobi sweep: m(m-1)/2 rotations, each updating two rows and two columns of H and
// two columns of V, about 6 m^3 multiply-adds (48 m^3 flops complex, 12 m^3 real).
// Solves whose eigenvectors only seed later work (seed_only) use the tridiagonal solver
// from order TRI_MIN on (reduction 4/3 m^3 and back-transformation 2 m^3 multiply-adds);
// MFEAST_TRIDIAG=0 keeps the Jacobi solver for them.
constexpr int TRI_MIN = 128;

static bool tri_enabled() {
  static const int mode = getenv("MFEAST_TRIDIAG") ? atoi(getenv("MFEAST_TRIDIAG")) : 1;
  return mode != 0;
}

template <typename T>
static int eig_timed(hipStream_t s, int m, T* H, T* V, double* evals, int* sweeps, double* work,
                     double big_rel = 1.0e-10, bool seed_only = false, bool* used_tri = nullptr) {
  const bool tri = seed_only && tri_enabled() && m >= TRI_MIN;
  if (used_tri) *used_tri = tri;
  const int tok = prof_begin(s);
  int fell_back = 0;
  const int rc = tri ? tri_eigh<T>(s, m, H, V, evals, reinterpret_cast<char*>(work), &fell_back, sweeps, big_rel)
                     : jacobi_eigh<T>(s, m, H, V, evals, sweeps, work, big_rel);
  double flops = 0.0;
  if (prof_on() && rc == 0) {
    if (tri && !fell_back) {
      flops = (is_cplx<T>::value ? 8.0 : 2.0) * (4.0 / 3.0 + 2.0) * (double)m * m * m;
    } else {
      int sw = 0;
      if (hipMemcpyAsync(&sw, sweeps, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) return -2;
      if (hipStreamSynchronize(s) != hipSuccess) return -2;
      flops = (is_cplx<T>::value ? 48.0 : 12.0) * (double)m * m * m * sw;
    }
  }
  prof_end(tok, s, K_EIG, flops, 0.0);
  return rc;
}


// ---------------------------------------------------------------------------
// What the subspace loop needs from a matrix format.  All blocks are row-major
// n x m FP64 (T) with leading dimension m.
struct Coef {
  const double* cs;  // column scales applied to the right-hand side before the solves
  const double* us;  // their inverses, applied to the quadrature sum
  const double* rho; // rational filter at the current Ritz values (residual form)
  const c64* cf;     // per node and column: w_j / (z_j - lambda_c) (residual) or w_j (classic)
  const c64* cc;     // the same for the conjugate node (complex Hermitian)
};

template <typename T>
struct Operator {
  bool hasB = false;
  virtual ~Operator() = default;
  // once per call, before the loop (factorization / format conversion); returns info
  virtual int prepare(hipStream_t s) = 0;
  virtual int apply_A(hipStream_t s, int m, const T* X, T* Y) = 0;
  virtual int apply_B(hipStream_t s, int m, const T* X, T* Y) = 0;
  // Q = [resid: X diag(rho)] + sum over the nodes of the weighted solves with rhs
  virtual int contour(hipStream_t s, int m, const T* rhs, const Coef& k, const T* X, T* Q, bool resid) = 0;
  // out[c] = r_c^H B^-1 r_c for the columns of the row-major n x m block R (only called
  // when hasB); cs[c] > 0 scales column c before the solve; partial: ceil(n/256) * m doubles
  virtual int binv_dots(hipStream_t s, int m, const T* R, const double* cs, double* out, double* partial) = 0;
  // FP32 solves near their accuracy limit: later contours add one FP64 refinement step per
  // solve (as fpm(50) = 1).  Returns whether the operator changed.
  virtual bool raise_precision(hipStream_t) { return false; }
  // the seeding eigensolves (first iteration, not-found block) may use the tridiagonal
  // solver; off where an iteration costs seconds and the eigensolve does not matter
  bool tri_seed = true;
};

// dense storage: LU of every shifted matrix, blocked triangular solves
template <typename T, typename C>
struct DenseOp : Operator<T> {
  mfeast_ctx* h;
  char uplo;
  int64_t n;
  const T *A, *B;
  int64_t lda, ldb;
  const std::vector<c64>& z;
  int ne, m0max;
  int nf;  // matrices factored: the ne shifted ones, and B itself when B is given (B^-1 products)
  const T* Af = nullptr;
  const T* Bf = nullptr;
  int64_t ldaf = 0, ldbf = 0;
  C *LU = nullptr, *Dinv = nullptr, *Wf = nullptr, *Wc = nullptr, *Wy = nullptr, *Wy2 = nullptr, *Pinv = nullptr;
  SolveSide<C> side{};
  bool two_streams = false;  // the conjugate-transpose solves on the handle's second stream
  int *ipiv = nullptr, *perm = nullptr, *pinv = nullptr, *linfo = nullptr;
  c64* zdev = nullptr;
  // fpm(50): extra refinement steps of the FP32 solves (FP64 solutions and residuals)
  int ir_steps = 0;
  c64 *irXf = nullptr, *irYc = nullptr, *irT = nullptr, *irAX = nullptr, *irBX = nullptr;
  // factors supplied by the caller (LU, Pinv, perm, pinv set before prepare): those of the
  // nf matrices padded to order nw >= n with an identity block; the solves run at order nw
  // on right-hand sides whose rows beyond n are zero
  bool ext = false;
  int64_t nw = 0;

  DenseOp(mfeast_ctx* h_, char uplo_, int64_t n_, const T* A_, int64_t lda_, const T* B_, int64_t ldb_,
          const std::vector<c64>& z_, int m0_)
      : h(h_), uplo(uplo_), n(n_), A(A_), B(B_), lda(lda_), ldb(ldb_), z(z_), ne((int)z_.size()), m0max(m0_) {
    this->hasB = B_ != nullptr;
    nf = ne + (B_ != nullptr ? 1 : 0);
    nw = n_;
  }

  // FP64 blocks of the refinement steps
  bool ir_buffers() {
    constexpr bool CPLX = is_cplx<T>::value;
    const size_t blk64 = (size_t)ne * n * m0max * sizeof(c64);
    irXf = (c64*)h->ws(S_IR_XF, blk64);
    irYc = CPLX ? (c64*)h->ws(S_IR_YC, blk64) : nullptr;
    irT = CPLX ? (c64*)h->ws(S_IR_T, blk64) : nullptr;
    irAX = (c64*)h->ws(S_IR_AX, blk64);
    irBX = B ? (c64*)h->ws(S_IR_BX, blk64) : nullptr;
    const bool ok = irXf && (!CPLX || (irYc && irT)) && irAX && (!B || irBX);
    if (!ok) irXf = nullptr;
    return ok;
  }

  // not for caller-supplied (padded) factors, and not inside the no-allocation entry point,
  // whose fixed array is sized for the call as requested
  bool raise_precision(hipStream_t) override {
    if (sizeof(C) != sizeof(c32) || ext || ir_steps != 0 || h->arena != nullptr) return false;
    if (!ir_buffers()) return false;
    ir_steps = 1;
    return true;
  }

  int prepare(hipStream_t s) override {
    constexpr bool CPLX = is_cplx<T>::value;
    if (ext) {
      const size_t szC = sizeof(C);
      Wf = (C*)h->ws(S_WF, (size_t)ne * nw * m0max * szC);
      Wc = CPLX ? (C*)h->ws(S_WC, (size_t)ne * nw * m0max * szC) : nullptr;
      Wy = (C*)h->ws(S_WY, (size_t)ne * nw * m0max * szC);
      if (!Wf || (CPLX && !Wc) || !Wy || !LU || !Pinv || !perm || !pinv || ir_steps != 0 || uplo != 'F') return -2;
      Af = A;
      ldaf = lda;
      Bf = B;
      ldbf = ldb;
      return 0;
    }
    const int64_t nblk = (n + LU_NB - 1) / LU_NB;
    const size_t szT = sizeof(T), szC = sizeof(C);
    LU = (C*)h->ws(S_LU, (size_t)nf * n * lu_ld(n) * szC);
    Dinv = (C*)h->ws(S_DINV, (size_t)nf * nblk * 2 * LU_NB * LU_NB * szC);
    ipiv = (int*)h->ws(S_IPIV, (size_t)nf * n * 4);
    perm = (int*)h->ws(S_PERM, (size_t)nf * n * 4);
    pinv = (int*)h->ws(S_PINV, (size_t)nf * n * 4);
    linfo = (int*)h->ws(S_INFO, (size_t)nf * 4 + 64);
    zdev = (c64*)h->ws(S_Z, (size_t)ne * sizeof(c64));
    Wf = (C*)h->ws(S_WF, (size_t)ne * n * m0max * szC);
    Wc = CPLX ? (C*)h->ws(S_WC, (size_t)ne * n * m0max * szC) : nullptr;
    Wy = (C*)h->ws(S_WY, (size_t)ne * n * m0max * szC);
    if (CPLX && h->ensure_aux()) {
      Wy2 = (C*)h->ws(S_WY2, (size_t)ne * n * m0max * szC);
      if (!Wy2) return -2;
      side = SolveSide<C>{h->aux, h->ev_fork, h->ev_join, Wy2};
      two_streams = true;
    }
    Pinv = (C*)h->ws(S_PANINV, (size_t)nf * panel_inverse_entries(n) * szC);
    if (!LU || !Dinv || !ipiv || !perm || !pinv || !linfo || !zdev || !Wf || (CPLX && !Wc) || !Wy || !Pinv) return -2;
    if (ir_steps > 0 && sizeof(C) == sizeof(c32) && !ir_buffers()) return -2;
    // full storage if a triangle was given
    Af = A;
    ldaf = lda;
    Bf = B;
    ldbf = ldb;
    if (uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u') {
      T* a2 = (T*)h->ws(S_AF, (size_t)n * n * szT);
      if (!a2) return -2;
      MF_TRY(expand_full<T>(s, uplo, n, A, lda, a2));
      Af = a2;
      ldaf = n;
      if (B) {
        T* b2 = (T*)h->ws(S_BF, (size_t)n * n * szT);
        if (!b2) return -2;
        MF_TRY(expand_full<T>(s, uplo, n, B, ldb, b2));
        Bf = b2;
        ldbf = n;
      }
    }
    // nodes up and factorization flags down through the handle's pinned area (nodes first,
    // flags after them)
    char* hx = h->host_aux((size_t)nf * (sizeof(c64) + 4) + 64);
    if (!hx) return -2;
    c64* hz = reinterpret_cast<c64*>(hx);
    int* hinfo = reinterpret_cast<int*>(hx + (size_t)ne * sizeof(c64));
    for (int j = 0; j < ne; ++j) hz[j] = z[j];
    MF_HIP_CHECK(hipMemcpyAsync(zdev, hz, ne * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemsetAsync(linfo, 0, nf * 4, s));
    {
      const int tok = prof_begin(s);
      MF_TRY(shift_form<T, C>(s, n, Af, ldaf, Bf, ldbf, zdev, ne, LU, perm, nf > ne));
      prof_end(tok, s, K_OTHER, 0.0, (double)n * n * ((B ? 2.0 : 1.0) * sizeof(T) + nf * sizeof(C)));
    }
    MF_TRY(lu_factor<C>(s, n, nf, LU, ipiv, perm, pinv, linfo, Dinv));
    {
      const int tok = prof_begin(s);
      MF_TRY(panel_inverses<C>(s, n, nf, LU, Dinv, Pinv));
      prof_end(tok, s, K_LU_ROWS, 0.0, 0.0);
    }
    MF_HIP_CHECK(hipMemcpyAsync(hinfo, linfo, nf * 4, hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int j = 0; j < ne; ++j)
      if (hinfo[j] != 0) return -2;
    // a singular B (zero pivot) is not positive definite (Table tab_info -3)
    if (nf > ne && hinfo[ne] != 0) return -3;
    return 0;
  }

  // B^-1 R diag(cs) with the stored factors of B (matrix ne), then the column dots
  int binv_dots(hipStream_t s, int m, const T* R, const double* cs, double* out, double* partial) override {
    if (nf == ne) return -2;
    const int64_t ld = lu_ld(nw);
    int tok = prof_begin(s);
    MF_TRY(rhs_prepare<T, C>(s, nw, m, R, m, cs, 1, perm + (int64_t)ne * nw, Wf, nullptr, n));
    prof_end(tok, s, K_RESID, 0.0, (double)n * m * (sizeof(T) + sizeof(C)));
    MF_TRY(lu_solve<C>(s, nw, m, 1, LU + (int64_t)ne * nw * ld, Pinv + (size_t)ne * panel_inverse_entries(nw), Wf,
                       nullptr, Wy, nullptr, K_RESID));
    tok = prof_begin(s);
    MF_TRY(col_dots_mixed<T, C>(s, n, m, R, Wf, cs, out, partial));
    prof_end(tok, s, K_RESID, 0.0, (double)n * m * (sizeof(T) + sizeof(C)));
    return 0;
  }

  int apply_A(hipStream_t s, int m, const T* X, T* Y) override {
    return rm_gemm<T>(s, (int)n, m, (int)n, Af, ldaf, true, false, X, m, Y, m);
  }
  int apply_B(hipStream_t s, int m, const T* X, T* Y) override {
    return rm_gemm<T>(s, (int)n, m, (int)n, Bf, ldbf, true, false, X, m, Y, m);
  }

  int contour(hipStream_t s, int m, const T* rhs, const Coef& k, const T* X, T* Q, bool resid) override {
    constexpr bool CPLX = is_cplx<T>::value;
    const double nb = (double)n * m;
    const int dirs = CPLX ? 2 : 1;
    int tok = prof_begin(s);
    MF_TRY(rhs_prepare<T, C>(s, nw, m, rhs, m, k.cs, ne, perm, Wf, Wc, n));
    prof_end(tok, s, K_OTHER, 0.0, nb * (sizeof(T) + (double)dirs * ne * sizeof(C)));
    MF_TRY(lu_solve<C>(s, nw, m, ne, LU, Pinv, Wf, Wc, Wy, two_streams ? &side : nullptr));
    if (sizeof(C) == sizeof(c32) && irXf != nullptr) {
      if constexpr (sizeof(C) == sizeof(c32)) MF_TRY(refine(s, m, rhs, k));
      tok = prof_begin(s);
      MF_TRY(accumulate<T, c64>(s, n, m, ne, irXf, irYc, pinv, k.cf, k.cc, k.rho, k.us, X, Q, resid ? 1 : 0));
      prof_end(tok, s, K_OTHER, 0.0, nb * ((double)dirs * ne * sizeof(c64) + (resid ? 2.0 : 1.0) * sizeof(T)));
      return 0;
    }
    tok = prof_begin(s);
    MF_TRY(accumulate<T, C>(s, nw, m, ne, Wf, Wc, pinv, k.cf, k.cc, k.rho, k.us, X, Q, resid ? 1 : 0, n));
    prof_end(tok, s, K_OTHER, 0.0, nb * ((double)dirs * ne * sizeof(C) + (resid ? 2.0 : 1.0) * sizeof(T)));
    return 0;
  }

  // Y_j = Mat X_j for every node (Mat: this operator's full FP64 A or B, column-major,
  // shared by the nodes); complex X with a real Mat is read as 2m real columns
  int apply_nodes(hipStream_t s, const T* Mat, int64_t ldm, int m, const c64* X, c64* Y) {
    constexpr bool CPLX = is_cplx<T>::value;
    GemmArgs g{};
    g.M = (int)n; g.K = (int)n;
    g.A = Mat; g.lda = ldm; g.a_bs = 0;
    g.alpha = 1.0; g.beta = 0.0;
    const int cols = CPLX ? m : 2 * m;
    g.N = cols;
    g.B = X; g.ldb = cols; g.b_bs = n * (int64_t)cols;
    g.C = Y; g.ldc = cols; g.c_bs = n * (int64_t)cols;
    const int tok = prof_begin(s);
    const int rc = gemm<double, CPLX>(s, true, false, g, ne);
    prof_end(tok, s, K_RR_GEMM, 8.0 * (double)n * n * m * ne, 0.0);
    return rc;
  }

  // fpm(50) refinement steps: the FP32 solutions in Wf / Wc are widened to FP64; each
  // step forms the FP64 residual of every node's system, solves it with the FP32
  // factors and adds the correction.  The conjugate-node solutions stay in the row
  // order of the factors (the accumulation applies perm_inv), so their residual is
  // formed on a gathered copy.
  int refine(hipStream_t s, int m, const T* rhs, const Coef& k) {
    constexpr bool CPLX = is_cplx<T>::value;
    const int64_t cnt = (int64_t)ne * n * m;
    MF_TRY(widen<C>(s, cnt, Wf, irXf, false));
    if (CPLX) MF_TRY(widen<C>(s, cnt, Wc, irYc, false));
    for (int step = 0; step < ir_steps; ++step) {
      MF_TRY(apply_nodes(s, Af, ldaf, m, irXf, irAX));
      const c64* BXf = irXf;
      if (Bf) {
        MF_TRY(apply_nodes(s, Bf, ldbf, m, irXf, irBX));
        BXf = irBX;
      }
      MF_TRY(ir_residual<T, C>(s, n, m, ne, rhs, m, k.cs, zdev, false, perm, irAX, BXf, Wf));
      if (CPLX) {
        MF_TRY(gather_rows_c64(s, n, m, ne, irYc, pinv, irT));
        MF_TRY(apply_nodes(s, Af, ldaf, m, irT, irAX));
        const c64* BXc = irT;
        if (Bf) {
          MF_TRY(apply_nodes(s, Bf, ldbf, m, irT, irBX));
          BXc = irBX;
        }
        MF_TRY(ir_residual<T, C>(s, n, m, ne, rhs, m, k.cs, zdev, true, nullptr, irAX, BXc, Wc));
      }
      MF_TRY(lu_solve<C>(s, n, m, ne, LU, Pinv, Wf, Wc, Wy, two_streams ? &side : nullptr));
      MF_TRY(widen<C>(s, cnt, Wf, irXf, true));
      if (CPLX) MF_TRY(widen<C>(s, cnt, Wc, irYc, true));
    }
    return 0;
  }
};

// CSR storage, real symmetric: BiCGSTAB on every shifted system (IFEAST)
template <typename C>
struct CsrOp : Operator<double> {
  using R = typename real_of<C>::type;
  mfeast_ctx* h;
  char uplo;
  int64_t n;
  const double *a, *b;
  const int32_t *ia, *ja, *ib, *jb;
  int base;
  const std::vector<c64>& z;
  int ne, m0max, maxit;
  double tol;
  CsrMat<R> MA, MB;
  int group = 0;  // nodes per BiCGSTAB batch (bounded by device memory)
  c64* zdev = nullptr;
  R* bh = nullptr;
  C* vec = nullptr;
  BiCol* col = nullptr;
  int* tiles = nullptr;
  double* part = nullptr;
  int* dbuf = nullptr;
  int* hbuf = nullptr;
  int64_t iterations = 0;  // fpm(60): sum over solves of the largest column count per node
  std::vector<c64> zhost;

  CsrOp(mfeast_ctx* h_, char uplo_, int64_t n_, const double* a_, const int32_t* ia_, const int32_t* ja_,
        int base_, const double* b_, const int32_t* ib_, const int32_t* jb_, const std::vector<c64>& z_, int m0_,
        int maxit_, double tol_)
      : h(h_), uplo(uplo_), n(n_), a(a_), b(b_), ia(ia_), ja(ja_), ib(ib_), jb(jb_), base(base_), z(z_),
        ne((int)z_.size()), m0max(m0_), maxit(maxit_), tol(tol_) {
    this->hasB = b_ != nullptr;
    // BiCGSTAB takes seconds per iteration here; with the tridiagonal first eigensolve the
    // 64^3 Laplacian needed one iteration more (27.2 against 21.7 s), so Jacobi stays
    this->tri_seed = false;
  }

  int prepare(hipStream_t s) override {
    int err = 0;
    MF_TRY(csr_full<R>(s, n, a, ia, ja, base, uplo, h->csrA, MA, &err));
    if (err) {
      return err == 1 ? -105 : err == 2 ? -106 : -104;
    }
    if (b) {
      MF_TRY(csr_full<R>(s, n, b, ib, jb, base, uplo, h->csrB, MB, &err));
      if (err) {
        return err == 1 ? -109 : err == 2 ? -110 : -108;
      }
    }
    // nodes per batch: five n x (nodes * m0) vectors must fit in device memory
    const int64_t nrb = (n + 255) / 256;
    const double per_node =
        5.0 * (double)n * m0max * sizeof(C) + 8.0 * (nrb + 32.0) * m0max * 8.0 + m0max * sizeof(BiCol);
    size_t fr = 0, tot = 0;
    MF_HIP_CHECK(hipMemGetInfo(&fr, &tot));
    const double avail = 0.85 * ((double)fr + (double)h->cap[S_BI_VEC] + (double)h->cap[S_BI_PART]);
    group = (int)std::min<double>(ne, std::floor(avail / per_node));
    group = std::min(group, (int)(65535LL * 64 / std::max(1, m0max)));
    if (group < 1) return -2;
    const size_t ncolmax = ((size_t)group * m0max + 63) / 64 * 64;  // whole 64-column tiles
    const size_t blk = (size_t)n * ncolmax;
    zdev = (c64*)h->ws(S_Z, (size_t)(ne + 1) * sizeof(c64));
    bh = (R*)h->ws(S_BI_BH, (size_t)n * m0max * sizeof(R));
    vec = (C*)h->ws(S_BI_VEC, 5 * blk * sizeof(C));
    col = (BiCol*)h->ws(S_BI_COL, ncolmax * sizeof(BiCol));
    tiles = (int*)h->ws(S_BI_TILES, ((ncolmax + 63) / 64) * sizeof(int));
    part = (double*)h->ws(S_BI_PART, 8 * ((size_t)nrb + 32) * ncolmax * sizeof(double));
    dbuf = (int*)h->ws(S_BI_BUF, (ncolmax + 64) * sizeof(int));
    hbuf = h->host_ints(ncolmax + 64);
    if (!zdev || !bh || !vec || !col || !tiles || !part || !dbuf || !hbuf) return -2;
    // the shifts, then 0: with A's place taken by B, node ne solves (0 B' - B) x = b,
    // i.e. x = -B^-1 b (B^-1 products of the found-pair test)
    zhost.assign(z.begin(), z.end());
    zhost.push_back(c64(0.0, 0.0));
    MF_HIP_CHECK(hipMemcpyAsync(zdev, zhost.data(), (ne + 1) * sizeof(c64), hipMemcpyHostToDevice, s));
    return 0;
  }

  // r^H B^-1 r by BiCGSTAB on B alone (FP64 right-hand sides scaled by cs, rounded to the
  // solve precision), to 1e-6 relative in FP32 and 1e-12 in FP64; not counted in fpm(60)
  int binv_dots(hipStream_t s, int m, const double* Rb, const double* cs, double* out, double* partial) override {
    if (!b) return -2;
    MF_TRY(bi_rhs<R>(s, n, m, Rb, cs, bh));
    const size_t blk = (size_t)n * (((size_t)group * m0max + 63) / 64 * 64);
    BiSys<C> sys;
    sys.n = n;
    sys.ncol = m;
    sys.m0 = m;
    sys.A = &MB;
    sys.B = nullptr;
    sys.zn = zdev + ne;
    sys.bh = bh;
    sys.x = vec;
    sys.r = vec + blk;
    sys.p = vec + 2 * blk;
    sys.v = vec + 3 * blk;
    sys.t = vec + 4 * blk;
    sys.col = col;
    sys.tiles = tiles;
    sys.part = part;
    std::vector<int> its;
    const double btol = sizeof(R) == sizeof(float) ? 1.0e-6 : 1.0e-12;
    MF_TRY(bicgstab_batched<C>(s, sys, 1000, btol, its, dbuf, hbuf));
    MF_TRY(bi_coldots<C>(s, n, m, Rb, vec, cs, -1.0, out, partial));
    return 0;
  }

  int apply_A(hipStream_t s, int m, const double* X, double* Y) override {
    const int tok = prof_begin(s);
    MF_TRY(spmm_rm(s, MA, m, X, m, Y, m));
    prof_end(tok, s, K_OTHER, 2.0 * MA.nnz * m, (double)m * n * 16.0 + MA.nnz * 12.0);
    return 0;
  }
  int apply_B(hipStream_t s, int m, const double* X, double* Y) override {
    const int tok = prof_begin(s);
    MF_TRY(spmm_rm(s, MB, m, X, m, Y, m));
    prof_end(tok, s, K_OTHER, 2.0 * MB.nnz * m, (double)m * n * 16.0 + MB.nnz * 12.0);
    return 0;
  }

  int contour(hipStream_t s, int m, const double* rhs, const Coef& k, const double* X, double* Q,
              bool resid) override {
    MF_TRY(bi_rhs<R>(s, n, m, rhs, k.cs, bh));
    const size_t blk = (size_t)n * (((size_t)group * m0max + 63) / 64 * 64);
    std::vector<int> its;
    for (int j0 = 0; j0 < ne; j0 += group) {
      const int nj = std::min(group, ne - j0);
      BiSys<C> sys;
      sys.n = n;
      sys.ncol = nj * m;
      sys.m0 = m;
      sys.A = &MA;
      sys.B = b ? &MB : nullptr;
      sys.zn = zdev + j0;
      sys.bh = bh;
      sys.x = vec;
      sys.r = vec + blk;
      sys.p = vec + 2 * blk;
      sys.v = vec + 3 * blk;
      sys.t = vec + 4 * blk;
      sys.col = col;
      sys.tiles = tiles;
      sys.part = part;
      MF_TRY(bicgstab_batched<C>(s, sys, maxit, tol, its, dbuf, hbuf));
      for (int j = 0; j < nj; ++j) {
        int mx = 0;
        for (int q = 0; q < m; ++q) mx = std::max(mx, its[(size_t)j * m + q]);
        iterations += mx;
      }
      const int tok = prof_begin(s);
      MF_TRY(bi_accumulate<C>(s, n, m, nj, j0, sys.x, k.cf, k.rho, k.us, X, Q, j0 == 0 ? (resid ? 1 : 0) : 2));
      prof_end(tok, s, K_OTHER, 0.0, (double)n * m * (nj * sizeof(C) + (resid ? 2.0 : 1.0) * 8.0));
    }
    return 0;
  }
};

// ---------------------------------------------------------------------------
// The subspace iteration, shared by every storage format.
template <typename T>
static int feast_loop(mfeast_ctx* h, Operator<T>& op, int64_t n, int32_t* fpm, double emin, double emax,
                      int32_t* m0p, double* E, T* Xu, int64_t ldx, int32_t* Mout, double* res_out,
                      double* epsout, int32_t* loop, const std::vector<c64>& z, const std::vector<c64>& w,
                      double c_inf) {
  constexpr bool CPLX = is_cplx<T>::value;
  Timer total_t, ph;
  total_t.start();
  double t_fact = 0, t_solve = 0, t_prod = 0, t_eig = 0, t_ax = 0, t_bx = 0;
  hipStream_t s = h->stream;
  auto f = [&](int i) { return fpm[i - 1]; };
  const int ne = (int)z.size();
  int m0 = *m0p;
  const double alpha = std::max(std::fabs(emin), std::fabs(emax));
  const double eps = std::pow(10.0, -f(3));
  const bool hasB = op.hasB;

  // ---------------- workspace of the loop
  const size_t szT = sizeof(T);
  const size_t blk = (size_t)n * m0 * szT;
  T* Xw = (T*)h->ws(S_X, blk);
  T* Q = (T*)h->ws(S_Q, blk);
  T* R = (T*)h->ws(S_R, blk);
  T* AQ = (T*)h->ws(S_AQ, blk);
  T* BQ = hasB ? (T*)h->ws(S_BQ, blk) : Q;
  T* AX = (T*)h->ws(S_AX, blk);
  T* BX = hasB ? (T*)h->ws(S_BX, blk) : Xw;
  const size_t sq = (size_t)m0 * m0 * szT;
  T* Sm = (T*)h->ws(S_S, sq);
  T* Tm = (T*)h->ws(S_T, sq);
  T* Hw = (T*)h->ws(S_HW, std::max({sq, jacobi_work_bytes(m0, szT),
                                     m0 >= TRI_MIN ? tri_work_bytes(m0, szT) : (size_t)0}));
  T* V = (T*)h->ws(S_V, sq);
  T* G = (T*)h->ws(S_G, sq);
  T* TG = (T*)h->ws(S_TG, std::max(3 * sq, (size_t)m0 * 32 * szT));  // also Cholesky / Newton-Schulz work
  T* Cm = (T*)h->ws(S_C, sq);
  T* Zm = (T*)h->ws(S_Z2, sq);
  T* GZ = (T*)h->ws(S_GZ, sq);
  T* W = (T*)h->ws(S_W, sq);
  // small device arrays, packed
  const size_t nsmall = (size_t)m0 * 15 + (size_t)ne * m0 * 4 + 64;
  double* small = (double*)h->ws(S_SMALL, nsmall * sizeof(double));
  const int nchunk = (int)((n + 255) / 256);
  double* part = (double*)h->ws(S_PART, (size_t)nchunk * m0 * 2 * sizeof(double));
  int* dflag = (int*)h->ws(S_FLAG, 256);
  char* hp = h->host(nsmall * sizeof(double) + 4096);
  if (!Xw || !Q || !R || !AQ || !BQ || !AX || !BX || !Sm || !Tm || !Hw || !V || !G || !TG || !Cm || !Zm || !GZ ||
      !W || !small || !part || !dflag || !hp)
    return -2;
  double* d_absmax = small;             // m0
  double* d_cs = small + m0;            // m0
  double* d_us = small + 2 * m0;        // m0
  double* d_rho = small + 3 * m0;       // m0
  double* d_dscale = small + 4 * m0;    // m0
  double* d_evals = small + 5 * m0;     // m0
  double* d_lam = small + 6 * m0;       // m0
  double* d_rn = small + 7 * m0;        // m0
  double* d_bn = small + 8 * m0;        // m0
  double* d_gs = small + 9 * m0;        // m0
  int* d_idx = (int*)(small + 10 * m0); // m0 ints (fits in m0 doubles)
  int* d_perm = (int*)(small + 11 * m0);
  c64* d_cf = (c64*)(small + 12 * m0);               // ne*m0
  c64* d_cc = d_cf + (size_t)ne * m0;                // ne*m0
  int* d_sweeps = (int*)(small + 12 * m0 + 4 * (size_t)ne * m0);
  int* d_pi = (int*)(small + 12 * m0 + 4 * (size_t)ne * m0 + 64);  // m0 ints
  double* d_kt = small + 13 * m0 + 4 * (size_t)ne * m0 + 64;        // m0: r^H B^-1 r
  double* d_kcs = small + 14 * m0 + 4 * (size_t)ne * m0 + 64;       // m0: its column scales
  // pinned host staging (same packing)
  double* h_absmax = (double*)hp;
  double* h_cs = h_absmax + m0;
  double* h_us = h_absmax + 2 * m0;
  double* h_rho = h_absmax + 3 * m0;
  double* h_evals = h_absmax + 5 * m0;
  double* h_lam = h_absmax + 6 * m0;
  double* h_rn = h_absmax + 7 * m0;
  double* h_bn = h_absmax + 8 * m0;
  double* h_gs = h_absmax + 9 * m0;
  int* h_idx = (int*)(h_absmax + 10 * m0);
  int* h_perm = (int*)(h_absmax + 11 * m0);
  c64* h_cf = (c64*)(h_absmax + 12 * m0);
  c64* h_cc = h_cf + (size_t)ne * m0;
  int* h_flag = (int*)(h_absmax + 12 * m0 + 4 * (size_t)ne * m0);
  int* h_pi = (int*)(h_absmax + 12 * m0 + 4 * (size_t)ne * m0 + 64);
  double* h_kt = h_absmax + 13 * m0 + 4 * (size_t)ne * m0 + 64;
  double* h_kcs = h_absmax + 14 * m0 + 4 * (size_t)ne * m0 + 64;

  // ---------------- factor (dense) or convert (sparse)
  ph.start();
  {
    const int rc = op.prepare(s);
    if (rc != 0) return rc;
  }
  MF_HIP_CHECK(hipStreamSynchronize(s));
  t_fact += ph.stop();

  // ---------------- starting block
  // (the stochastic count probes with its own +-1 block whatever fpm(5) says)
  if (f(14) == 2) MF_TRY(rademacher_block<T>(s, n, m0, (uint64_t)(uint32_t)f(51), Xw, m0));
  else if (f(5) == 1) MF_TRY(copy_cm_to_rm<T>(s, n, m0, Xu, ldx, Xw, m0));
  else MF_TRY(random_block<T>(s, n, m0, (uint64_t)(uint32_t)f(51), Xw, m0));

  std::vector<double> lam_cur;
  std::vector<int> order;
  int last_sweeps = 0, last_osweeps = 0, last_mi = 0;
  double last_dev = 0.0;
  // found flags of the current Ritz pairs (eigensolver order), for the deflation above
  std::vector<char> found_prev;
  static const int deflate_mode = getenv("MFEAST_DEFLATE") ? atoi(getenv("MFEAST_DEFLATE")) : 1;
  const bool deflate = deflate_mode != 0;
  double trace_prev = 0.0;
  double maxres_prev = 1.0e300;
  int info = 0;
  int M = 0;
  int k = 0;
  std::vector<double> res_h;
  for (;;) {
    // ---- right-hand side block: B*Y (first contour) or the FP64 residual R
    const bool resid = (k > 0);
    const T* rhs;
    if (!resid) {
      if (hasB) {
        ph.start();
        MF_TRY(op.apply_B(s, m0, Xw, R));
        MF_HIP_CHECK(hipStreamSynchronize(s));
        t_bx += ph.stop();
        rhs = R;
      } else {
        rhs = Xw;
      }
    } else {
      rhs = R;
    }
    ph.start();
    MF_TRY(col_absmax<T>(s, n, m0, rhs, m0, d_absmax));
    MF_HIP_CHECK(hipMemcpyAsync(h_absmax, d_absmax, m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    for (int c = 0; c < m0; ++c) {
      const double a = h_absmax[c];
      const bool ok = a > 0.0 && std::isfinite(a);
      if (!std::isfinite(a)) return -2;
      h_cs[c] = ok ? 1.0 / a : 1.0;
      h_us[c] = ok ? a : 1.0;
    }
    for (int j = 0; j < ne; ++j) {
      for (int c = 0; c < m0; ++c) {
        if (resid) {
          const std::complex<double> zj(z[j].re, z[j].im), wj(w[j].re, w[j].im);
          const std::complex<double> a = wj / (zj - lam_cur[c]);
          const std::complex<double> b = std::conj(wj) / (std::conj(zj) - lam_cur[c]);
          h_cf[(size_t)j * m0 + c] = c64(a.real(), a.imag());
          h_cc[(size_t)j * m0 + c] = c64(b.real(), b.imag());
        } else {
          h_cf[(size_t)j * m0 + c] = w[j];
          h_cc[(size_t)j * m0 + c] = c64(w[j].re, -w[j].im);
        }
      }
    }
    // the filter at the Ritz values (residual form); its constant term (Zolotarev rule)
    // acts on the block itself, also in the first contour (classic form: Q = c_inf Y + ...)
    for (int c = 0; c < m0; ++c) {
      double rho = c_inf;
      if (resid) {
        for (int j = 0; j < ne; ++j) {
          const std::complex<double> zj(z[j].re, z[j].im), wj(w[j].re, w[j].im);
          rho += 2.0 * (wj / (zj - lam_cur[c])).real();
        }
      }
      h_rho[c] = rho;
    }
    // slots are laid out for the initial M0; m0 may have shrunk since, so copy each array
    MF_HIP_CHECK(hipMemcpyAsync(d_cs, h_cs, m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_us, h_us, m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_rho, h_rho, m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_cf, h_cf, (size_t)ne * m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(d_cc, h_cc, (size_t)ne * m0 * sizeof(c64), hipMemcpyHostToDevice, s));
    {
      const Coef kc{d_cs, d_us, d_rho, d_cf, d_cc};
      MF_TRY(op.contour(s, m0, rhs, kc, Xw, Q, resid || c_inf != 0.0));
    }
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_solve += ph.stop();

    if (f(14) == 2) {
      // stochastic count: Q is the filter applied to the +-1 probes Y, and
      // Re(trace(Y^H Q)) / m0 estimates the sum of the filter over the spectrum, i.e.
      // the number of eigenvalues inside (Hutchinson's estimator on the quadrature filter)
      double* d_dots = d_absmax;
      MF_TRY(col_dots<T>(s, n, m0, Xw, Q, d_dots, part));
      MF_HIP_CHECK(hipMemcpyAsync(h_absmax, d_dots, m0 * sizeof(double), hipMemcpyDeviceToHost, s));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      double est = 0.0;
      for (int c = 0; c < m0; ++c) est += h_absmax[c];
      est /= m0;
      if (!std::isfinite(est)) return -2;
      MF_HIP_CHECK(hipMemcpyAsync(E, &est, sizeof(double), hipMemcpyHostToDevice, s));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      *m0p = m0;
      *Mout = est > 0.0 ? (int32_t)std::floor(est + 0.5) : 0;
      *loop = 0;
      *epsout = 1.0;
      info = 5;
      break;
    }
    if (f(14) == 1) {
      MF_TRY(copy_rm_to_cm<T>(s, n, m0, Q, m0, Xu, ldx));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      *m0p = m0;
      *Mout = 0;
      *loop = 0;
      *epsout = 1.0;
      info = 4;
      break;
    }

    // ---- Rayleigh-Ritz on span(Q) in an explicitly B-orthonormal basis (two passes)
    ph.start();
    MF_TRY(op.apply_A(s, m0, Q, AQ));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_ax += ph.stop();
    T* BQp = Q;
    if (hasB) {
      ph.start();
      MF_TRY(op.apply_B(s, m0, Q, BQ));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      t_bx += ph.stop();
      BQp = BQ;
    }
    ph.start();
    MF_TRY(rm_gemm<T>(s, m0, m0, (int)n, Q, m0, true, true, BQp, m0, Sm, m0));
    // Order of pass 1: the columns of the pairs found last iteration first.  Those columns
    // are B-orthogonal to all others up to their residual, while the filtered columns of
    // the far outside pairs carry components along them that are large after scaling;
    // with the found columns first, Cholesky removes those components from the others
    // and never mixes the others into the found ones.
    int nfound = 0;
    const bool permuted = deflate && resid && (int)found_prev.size() == m0;
    if (permuted) {
      for (int i = 0; i < m0; ++i)
        if (found_prev[i]) h_pi[nfound++] = i;
      int a = nfound;
      for (int i = 0; i < m0; ++i)
        if (!found_prev[i]) h_pi[a++] = i;
      MF_HIP_CHECK(hipMemcpyAsync(d_pi, h_pi, m0 * sizeof(int), hipMemcpyHostToDevice, s));
      MF_TRY(sym_permute<T>(s, m0, Sm, d_pi, Cm));
      MF_TRY(copy_block<T>(s, m0, m0, Cm, m0, Sm, m0, false));
    }
    MF_HIP_CHECK(hipMemsetAsync(dflag, 0, 16, s));
    int otok = prof_begin(s);
    MF_TRY(gram_equilibrate<T>(s, m0, Sm, Tm, d_dscale, dflag));
    // pass 1: Cholesky of the equilibrated overlap with column dropping (d_perm = keep mask)
    const double tau = 32.0 * m0 * 2.220446049250313e-16;
    MF_TRY(chol_drop<T>(s, m0, Sm, Hw, d_perm, tau, TG));
    prof_end(otok, s, K_ORTH, 0.0, 0.0);
    MF_HIP_CHECK(hipMemcpyAsync(h_perm, d_perm, m0 * sizeof(int), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipMemcpyAsync(h_flag, dflag, 4, hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    if (h_flag[0] != 0) { info = -3; break; }
    int kk = 0;
    for (int i = 0; i < m0; ++i)
      if (h_perm[i]) h_idx[kk++] = i;
    if (kk == 0) { info = -3; break; }
    MF_HIP_CHECK(hipMemcpyAsync(d_idx, h_idx, kk * sizeof(int), hipMemcpyHostToDevice, s));
    MF_TRY(build_h1<T>(s, m0, kk, Hw, d_dscale, d_idx, G));
    // H1 is in the permuted row order: its row i belongs to column h_pi[i] of Q
    T* H1 = G;
    if (permuted) {
      MF_TRY(scatter_rows<T>(s, m0, kk, G, d_pi, Cm));
      H1 = Cm;
    }
    // Q1 = Q H1, A Q1 = (A Q) H1, B Q1 = (B Q) H1  (no new product with A or B)
    T* Q1 = R;
    T* AQ1 = AX;
    T* BQ1 = hasB ? BX : Q1;
    MF_TRY(rm_gemm<T>(s, (int)n, kk, m0, Q, m0, false, false, H1, kk, Q1, kk));
    MF_TRY(rm_gemm<T>(s, (int)n, kk, m0, AQ, m0, false, false, H1, kk, AQ1, kk));
    if (hasB) MF_TRY(rm_gemm<T>(s, (int)n, kk, m0, BQp, m0, false, false, H1, kk, BQ1, kk));
    // pass 2: S1 = Q1^H B Q1 = I + F, T1 = Q1^H A Q1
    MF_TRY(rm_gemm<T>(s, kk, kk, (int)n, Q1, kk, true, true, BQ1, kk, Sm, kk));
    MF_TRY(rm_gemm<T>(s, kk, kk, (int)n, Q1, kk, true, true, AQ1, kk, Tm, kk));
    MF_TRY(hermitian_part<T>(s, kk, Sm));
    MF_TRY(hermitian_part<T>(s, kk, Tm));
    otok = prof_begin(s);
    MF_TRY(dev_from_identity<T>(s, kk, Sm, part, d_bn));
    prof_end(otok, s, K_ORTH, 0.0, 0.0);
    double dev_f = 0.0;
    MF_HIP_CHECK(hipMemcpyAsync(&h_bn[0], d_bn, sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    dev_f = h_bn[0];
    if (!std::isfinite(dev_f)) { info = -2; break; }
    t_prod += ph.stop();
    ph.start();
    int kk2 = kk;
    T* G2 = V;
    if (dev_f < 0.5) {
      int iters = 1;
      for (double e = dev_f; e > 1e-18 && iters < 12; ++iters) e = 0.75 * e * e + 1e-300;
      otok = prof_begin(s);
      MF_TRY(ns_invsqrt<T>(s, kk, Sm, V, iters, TG));
      MF_TRY(hermitian_part<T>(s, kk, V));
      prof_end(otok, s, K_ORTH, 8.0 * (is_cplx<T>::value ? 4.0 : 1.0) * 3.0 * iters * (double)kk * kk * kk / 4.0,
               0.0);
    } else {
      // far from orthonormal: eigen-decompose S1 and drop its weak directions
      MF_TRY(eig_timed<T>(s, kk, Sm, Zm, d_evals, d_sweeps, (double*)Hw));
      MF_HIP_CHECK(hipMemcpyAsync(h_evals, d_evals, kk * sizeof(double), hipMemcpyDeviceToHost, s));
      MF_HIP_CHECK(hipStreamSynchronize(s));
      double smax = 0.0;
      for (int i = 0; i < kk; ++i) smax = std::max(smax, h_evals[i]);
      kk2 = 0;
      for (int i = 0; i < kk; ++i)
        if (smax > 0.0 && h_evals[i] > RANK_TOL * smax) {
          h_idx[kk2] = i;
          h_gs[kk2] = 1.0 / std::sqrt(h_evals[i]);
          ++kk2;
        }
      if (kk2 == 0) { info = -3; break; }
      MF_HIP_CHECK(hipMemcpyAsync(d_idx, h_idx, kk2 * sizeof(int), hipMemcpyHostToDevice, s));
      MF_HIP_CHECK(hipMemcpyAsync(d_gs, h_gs, kk2 * sizeof(double), hipMemcpyHostToDevice, s));
      MF_TRY(gather_scale_cols<T>(s, kk, kk2, Zm, kk, d_idx, d_gs, V, kk2));
    }
    // Deflation of the pairs found last iteration: with them first in pass 1 (above) and
    // Newton-Schulz leaving G2 close to I, the leading block of C belongs to them, is
    // diagonal up to their residuals and is coupled to the rest only to the same order;
    // only the trailing block of the others needs the full eigensolver.
    int mi = 0;
    if (permuted && dev_f < 0.5 && deflate_mode == 1) {
      while (mi < kk && h_idx[mi] < nfound) ++mi;
      if (mi < 1 || kk2 - mi < 2) mi = 0;
    }
    // C = G2^H T1 G2, eigenpairs of C
    MF_TRY(rm_gemm<T>(s, kk, kk2, kk, Tm, kk, false, false, G2, kk2, TG, kk2));
    MF_TRY(rm_gemm<T>(s, kk2, kk2, kk, G2, kk2, true, true, TG, kk2, Cm, kk2));
    MF_TRY(hermitian_part<T>(s, kk2, Cm));
    int osweeps = 0;
    if (mi > 0) {
      // C = [C_II C_IO; C_OI C_OO]: V_OO diagonalizes C_OO; C <- diag(I, V_OO)^H C diag(I, V_OO);
      // the full eigensolver on that matrix then only removes the small coupling, and the
      // eigenvectors of the original C are diag(I, V_OO) times its.
      const int mo = kk2 - mi;
      T* Coo = Sm;
      T* Voo = Tm;
      double* ev_oo = d_gs;  // unused eigenvalues of C_OO
      T* Coo_o = Cm + (int64_t)mi * kk2 + mi;  // C_OO in place, leading dimension kk2
      MF_TRY(copy_block<T>(s, mo, mo, Coo_o, kk2, Coo, mo, false));
      // (V_OO only prepares the full sweeps below, whose 1e-10 test decides the accuracy,
      // so its own sweeps stop at rotations below 1e-4 max|diag|)
      bool oo_tri = false;
      MF_TRY(eig_timed<T>(s, mo, Coo, Voo, ev_oo, d_sweeps + 1, (double*)Hw, 1.0e-4, op.tri_seed, &oo_tri));
      if (oo_tri) {
        // inverse-iteration vectors are orthogonal to about eps over the relative gap: V_OO
        // is replaced by its polar factor V_OO (V_OO^H V_OO)^-1/2 (Newton-Schulz), so that
        // the blocks formed with it below are similar to those of C
        MF_TRY(rm_gemm<T>(s, mo, mo, mo, Voo, mo, true, true, Voo, mo, Coo, mo));
        MF_TRY(ns_invsqrt<T>(s, mo, Coo, Hw, 4, TG));
        MF_TRY(rm_gemm<T>(s, mo, mo, mo, Voo, mo, false, false, Hw, mo, Coo, mo));
        MF_TRY(copy_block<T>(s, mo, mo, Coo, mo, Voo, mo, false));
      }
      // the rotated blocks are formed from the original C (V_OO^H C_OO V_OO keeps what the
      // eigensolver left off the diagonal, which the full sweeps below then remove)
      T* IOr = TG;                        // mi x mo
      T* OOr = TG + (size_t)mi * mo;      // mo x mo
      MF_TRY(rm_gemm<T>(s, mi, mo, mo, Cm + mi, kk2, false, false, Voo, mo, IOr, mo));
      MF_TRY(rm_gemm<T>(s, mo, mo, mo, Coo_o, kk2, false, false, Voo, mo, Coo, mo));
      MF_TRY(rm_gemm<T>(s, mo, mo, mo, Voo, mo, true, true, Coo, mo, OOr, mo));
      MF_TRY(copy_block<T>(s, mi, mo, IOr, mo, Cm + mi, kk2, false));
      MF_TRY(copy_block<T>(s, mi, mo, IOr, mo, Cm + (int64_t)mi * kk2, kk2, true));
      MF_TRY(copy_block<T>(s, mo, mo, OOr, mo, Coo_o, kk2, false));
      MF_TRY(hermitian_part<T>(s, kk2, Cm));
      MF_TRY(eig_timed<T>(s, kk2, Cm, Zm, d_evals, d_sweeps, (double*)Hw));
      MF_TRY(rm_gemm<T>(s, mo, kk2, mo, Voo, mo, false, false, Zm + (int64_t)mi * kk2, kk2, TG, kk2));
      MF_TRY(copy_block<T>(s, mo, kk2, TG, kk2, Zm + (int64_t)mi * kk2, kk2, false));
      MF_HIP_CHECK(hipMemcpyAsync(&osweeps, d_sweeps + 1, sizeof(int), hipMemcpyDeviceToHost, s));
    } else {
      // the first iteration's Ritz pairs only seed the next contour (its subspace does not
      // depend on the basis chosen inside span(Q), and their residuals are far above the
      // threshold), so its sweeps stop at rotations below 1e-4 max|diag|, which still leaves
      // off-diagonal entries of the order of 1e-8 max|diag|
      MF_TRY(eig_timed<T>(s, kk2, Cm, Zm, d_evals, d_sweeps, (double*)Hw, k == 0 ? 1.0e-4 : 1.0e-10,
                          k == 0 && op.tri_seed));
    }
    int sweeps = 0;
    MF_HIP_CHECK(hipMemcpyAsync(h_evals, d_evals, kk2 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipMemcpyAsync(&sweeps, d_sweeps, sizeof(int), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    last_sweeps = sweeps;
    last_osweeps = osweeps;
    last_mi = mi;
    last_dev = dev_f;
    t_eig += ph.stop();
    ph.start();
    // Ritz pairs keep the eigensolver's order internally; the reported order (found
    // pairs ascending, then the others ascending) is applied when copying out.
    lam_cur.assign(h_evals, h_evals + kk2);
    for (int i = 0; i < kk2; ++i) h_lam[i] = lam_cur[i];
    MF_HIP_CHECK(hipMemcpyAsync(d_lam, h_lam, kk2 * sizeof(double), hipMemcpyHostToDevice, s));
    // W = G2 U;  X = Q1 W, AX = (A Q1) W, BX = (B Q1) W  (n x kk2, leading dimension kk2)
    MF_TRY(rm_gemm<T>(s, kk, kk2, kk2, G2, kk2, false, false, Zm, kk2, W, kk2));
    T* AXn = AQ;
    T* BXn = hasB ? BQ : Xw;
    MF_TRY(rm_gemm<T>(s, (int)n, kk2, kk, Q1, kk, false, false, W, kk2, Xw, kk2));
    MF_TRY(rm_gemm<T>(s, (int)n, kk2, kk, AQ1, kk, false, false, W, kk2, AXn, kk2));
    if (hasB) MF_TRY(rm_gemm<T>(s, (int)n, kk2, kk, BQ1, kk, false, false, W, kk2, BXn, kk2));
    m0 = kk2;
    {
      const int rtok = prof_begin(s);
      MF_TRY(residual_norms<T>(s, n, m0, AXn, BXn, d_lam, R, d_rn, d_bn, part));
      prof_end(rtok, s, K_RESID, 0.0, (double)n * m0 * 3.0 * sizeof(T));
    }
    MF_HIP_CHECK(hipMemcpyAsync(h_rn, d_rn, m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipMemcpyAsync(h_bn, d_bn, m0 * sizeof(double), hipMemcpyDeviceToHost, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    t_prod += ph.stop();
    res_h.assign(m0, 0.0);
    bool finite = true;
    for (int i = 0; i < m0; ++i) {
      res_h[i] = std::sqrt(h_rn[i]) / (alpha * std::sqrt(h_bn[i]));
      if (!std::isfinite(res_h[i])) finite = false;
    }
    if (!finite) { info = -2; break; }
    // Kato-Temple terms of the found-pair test: r^H B^-1 r (||r||^2 for B = I), needed only
    // for the candidates (inside the interval, relative residual below SPURIOUS_RES); their
    // residual columns are gathered into Q (free at this point), scaled by 1/||r||
    if (hasB) {
      ph.start();
      int kc = 0;
      for (int c = 0; c < m0; ++c) {
        h_kt[c] = 0.0;
        const double l = lam_cur[c];
        if (l >= emin && l <= emax && res_h[c] < SPURIOUS_RES) {
          h_idx[kc] = c;
          h_kcs[kc] = h_rn[c] > 0.0 ? 1.0 / std::sqrt(h_rn[c]) : 1.0;
          ++kc;
        }
      }
      if (kc > 0) {
        for (int q = 0; q < kc; ++q) h_gs[q] = 1.0;
        MF_HIP_CHECK(hipMemcpyAsync(d_idx, h_idx, kc * sizeof(int), hipMemcpyHostToDevice, s));
        MF_HIP_CHECK(hipMemcpyAsync(d_kcs, h_kcs, kc * sizeof(double), hipMemcpyHostToDevice, s));
        MF_HIP_CHECK(hipMemcpyAsync(d_gs, h_gs, kc * sizeof(double), hipMemcpyHostToDevice, s));
        MF_TRY(gather_scale_cols<T>(s, (int)n, kc, R, m0, d_idx, d_kcs, Q, kc));
        MF_TRY(op.binv_dots(s, kc, Q, d_gs, d_kt, part));
        MF_HIP_CHECK(hipMemcpyAsync(h_gs, d_kt, kc * sizeof(double), hipMemcpyDeviceToHost, s));
        MF_HIP_CHECK(hipStreamSynchronize(s));
        for (int q = 0; q < kc; ++q) h_kt[h_idx[q]] = h_gs[q] / (h_kcs[q] * h_kcs[q]);
      }
      t_bx += ph.stop();
    } else {
      for (int c = 0; c < m0; ++c) h_kt[c] = h_rn[c];
    }
    // found pairs: inside the interval with a residual below the spurious threshold
    int n_inside = 0;
    M = 0;
    double maxres = 0.0, trace = 0.0;
    // found: inside, relative residual below SPURIOUS_RES, and r^H B^-1 r < (emax - l)(l - emin)
    // (Kato-Temple for B^-1 A, self-adjoint in the B inner product: a B-unit vector
    // B-orthogonal to the eigenvectors in the interval has r^H B^-1 r >= (emax - l)(l - emin),
    // so a pair below the bound is no mixture of outside ones; the test does not change
    // when A and B are scaled together)
    auto found = [&](int i) {
      const double l = lam_cur[i];
      return l >= emin && l <= emax && res_h[i] < SPURIOUS_RES && h_kt[i] < (emax - l) * (l - emin);
    };
    found_prev.assign(m0, 0);
    for (int i = 0; i < m0; ++i) {
      const bool in = lam_cur[i] >= emin && lam_cur[i] <= emax;
      n_inside += in ? 1 : 0;
      if (found(i)) {
        found_prev[i] = 1;
        ++M;
        maxres = std::max(maxres, res_h[i]);
        trace += lam_cur[i];
      }
    }
    order.resize(m0);
    for (int i = 0; i < m0; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      const bool fa = found(a), fb = found(b);
      if (fa != fb) return fa;
      return lam_cur[a] < lam_cur[b];
    });
    const double eo = (k == 0) ? 1.0 : std::fabs(trace - trace_prev) / alpha;
    trace_prev = trace;
    *epsout = eo;
    *loop = k;
    *Mout = M;
    if (n_inside == 0) { info = 1; break; }
    if (n_inside >= m0) { info = 3; break; }
    if (f(1) != 0) {
      // runtime comments (fpm(1)): iteration, #eigenvalues, trace, relative trace change,
      // largest residual of the found pairs, subspace size, spurious count
      fprintf(stderr, "%3d %6d  %24.16E  %24.16E  %24.16E  m0=%d spurious=%d |S1-I|=%.1e sweeps=%d",
              k, M, trace, eo, maxres, m0, n_inside - M, last_dev, last_sweeps);
      if (last_mi > 0) fprintf(stderr, " (deflated %d, %d sweeps on the other %d)", last_mi, last_osweeps, m0 - last_mi);
      fprintf(stderr, "\n");
    }
    const bool conv = M > 0 && ((f(6) == 1) ? (maxres < eps) : (eo < eps));
    if (conv) { info = 0; break; }
    if (k >= f(4)) { info = 2; break; }
    // FP32 solves leave a residual floor of about 1e-11 (it varies with rounding up to about
    // 6e-11): for a tolerance below 1e-10, once the found pairs are within reach of that floor
    // (largest residual below 1e-9), and for any tolerance once their residual falls by less
    // than ten times in an iteration, the later contours refine every solve once in FP64
    const bool near_floor = eps < 1.0e-10 && maxres < 1.0e-9;
    const bool stalled = maxres > 0.1 * maxres_prev;
    if (k >= 2 && M > 0 && maxres >= eps && (near_floor || stalled) && op.raise_precision(s) && f(1) != 0)
      fprintf(stderr, "    FP32 solves refined once in FP64 from the next contour on\n");
    maxres_prev = M > 0 ? maxres : maxres_prev;
    ++k;
  }

  if (info != 4 && info != 5 && info != -3 && info != -2) {
    // copy eigenpairs to the caller's layout in the reported order (values through the
    // handle's pinned area)
    double* e_out = reinterpret_cast<double*>(h->host_aux(2 * (size_t)m0 * sizeof(double) + 64));
    if (!e_out) return -2;
    double* r_out = e_out + m0;
    for (int i = 0; i < m0; ++i) {
      h_perm[i] = order[i];
      e_out[i] = lam_cur[order[i]];
      r_out[i] = res_h[order[i]];
    }
    MF_HIP_CHECK(hipMemcpyAsync(d_perm, h_perm, m0 * sizeof(int), hipMemcpyHostToDevice, s));
    MF_TRY(copy_rm_to_cm<T>(s, n, m0, Xw, m0, Xu, ldx, d_perm));
    MF_HIP_CHECK(hipMemcpyAsync(E, e_out, m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipMemcpyAsync(res_out, r_out, m0 * sizeof(double), hipMemcpyHostToDevice, s));
    MF_HIP_CHECK(hipStreamSynchronize(s));
    *m0p = m0;
  }
  // the guide's FEAST-RCI timing split: Fact., Solve, A*x, B*x, Misc., Total; then the
  // iteration count and the reduced eigensolver's share of Misc.
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
// nodes from fpm(2), fpm(16), fpm(18) (fpm(54) for the Zolotarev rule, whose constant
// term is returned in c_inf), or the caller's expert contour (no constant term)
static void nodes_for(const int32_t* fpm, double emin, double emax, const double* zne, const double* wne,
                      std::vector<c64>& z, std::vector<c64>& w, double& c_inf) {
  const int ne = fpm[1];
  c_inf = 0.0;
  if (zne != nullptr) {
    z.resize(ne);
    w.resize(ne);
    for (int j = 0; j < ne; ++j) {
      z[j] = c64(zne[2 * j], zne[2 * j + 1]);
      w[j] = c64(wne[2 * j], wne[2 * j + 1]);
    }
  } else if (fpm[15] == 2) {
    zolotarev_contour(emin, emax, ne, fpm[53], z, w, c_inf);
  } else {
    make_contour(emin, emax, ne, fpm[15], fpm[17], z, w);
  }
}

// per-call set-up around the loop: device, optional kernel timing
template <typename T>
static int run_loop(mfeast_ctx* h, Operator<T>& op, int64_t n, int32_t* fpm, double emin, double emax,
                    int32_t* m0, double* E, T* X, int64_t ldx, int32_t* M, double* res, double* epsout,
                    int32_t* loop, const std::vector<c64>& z, const std::vector<c64>& w, double c_inf) {
  prof_enable(fpm[51] == 1 || h->prof_all);
  for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] = 0.0;
  const int info = feast_loop<T>(h, op, n, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, z, w, c_inf);
  if (prof_on()) {
    (void)hipStreamSynchronize(h->stream);
    prof_collect(h->prof);
    prof_enable(false);
  }
  return info;
}

// argument checks of the dense drivers, in Table tab_info order: N, M0, interval, fpm,
// then argument positions
static int dense_check(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda, const double* B,
                       int64_t ldb, const int32_t* fpm, double emin, double emax, const int32_t* m0, const double* E,
                       const double* X, int64_t ldx, const int32_t* M, const double* res, const double* epsout,
                       const int32_t* loop, const double* zne, const double* wne) {
  if (n < 1 || n > MAX_DENSE_N) return 202;
  if (m0 == nullptr) return -111;
  if (*m0 < 1 || *m0 > n || *m0 > MAX_M0) return 201;
  if (!(emin < emax)) return 200;
  if (fpm == nullptr) return -108;
  if ((zne == nullptr) != (wne == nullptr)) return zne == nullptr ? -119 : -120;
  const int fi = check_fpm(fpm, zne != nullptr);
  if (fi) return fi;
  if (h == nullptr) return -101;
  if (!(uplo == 'F' || uplo == 'f' || uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) return -102;
  if (A == nullptr) return -104;
  if (lda < n) return -105;
  if (B != nullptr && ldb < n) return -107;
  if (E == nullptr) return -112;
  if (X == nullptr) return -113;
  if (ldx < n) return -114;
  if (M == nullptr) return -115;
  if (res == nullptr) return -116;
  if (epsout == nullptr) return -117;
  if (loop == nullptr) return -118;
  return 0;
}

template <typename T>
static int dense_entry(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda, const double* B,
                       int64_t ldb, int32_t* fpm, double emin, double emax, int32_t* m0, double* E, double* X,
                       int64_t ldx, int32_t* M, double* res, double* epsout, int32_t* loop, const double* zne,
                       const double* wne) {
  const int chk = dense_check(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop,
                              zne, wne);
  if (chk) return chk;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  const T* At = reinterpret_cast<const T*>(A);
  const T* Bt = reinterpret_cast<const T*>(B);
  T* Xt = reinterpret_cast<T*>(X);
  std::vector<c64> z, w;
  double c_inf = 0.0;
  nodes_for(fpm, emin, emax, zne, wne, z, w, c_inf);
  set_gemm_3m(fpm[52] == 0);
  if (fpm[41] == 1) {
    DenseOp<T, c32> op(h, uplo, n, At, lda, Bt, ldb, z, *m0);
    op.ir_steps = fpm[49];
    return run_loop<T>(h, op, n, fpm, emin, emax, m0, E, Xt, ldx, M, res, epsout, loop, z, w, c_inf);
  }
  DenseOp<T, c64> op(h, uplo, n, At, lda, Bt, ldb, z, *m0);
  return run_loop<T>(h, op, n, fpm, emin, emax, m0, E, Xt, ldx, M, res, epsout, loop, z, w, c_inf);
}

// ---------------------------------------------------------------------------
// Batched problems (the first level of parallelism of Section 1.1, independent problems):
// the factorizations of every (problem, node) item as one captured launch sequence.  The
// items are grouped into size classes (order rounded up to a multiple of 256); each matrix
// is padded to its class order with an identity block, so that the factors of the padded
// matrix are those of the problem's matrix in the leading block, and every class is a
// uniform batch for the blocked LU.  The classes run as parallel branches of one HIP graph,
// captured once per set of sizes and buffers (after an ordinary run of the same launches
// with the GEMM tile autotuner on) and replayed by later calls.  The subspace iterations
// of each problem then solve with its stored factors at the class order.
struct BtItem {
  const double* A;
  const double* B;
  int64_t lda, ldb, n;
  double zre, zim;
  int kind;  // 0: z B - A (B = I when null), 1: B itself
  int pad_;
};

template <typename C>
__global__ void k_bt_shift_form(int64_t nw, int64_t ld, const BtItem* __restrict__ items, C* __restrict__ LU,
                                int* __restrict__ perm, int* __restrict__ info) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  const int q = blockIdx.z;
  if (c >= nw) return;
  const BtItem it = items[q];
  c64 v(i == c ? 1.0 : 0.0, 0.0);
  if (i < it.n && c < it.n) {
    // real symmetric, column-major: element (i, c) read as A[i lda + c] (coalesced)
    const double a = it.A[i * it.lda + c];
    const double b = it.B != nullptr ? it.B[i * it.ldb + c] : (i == c ? 1.0 : 0.0);
    v = it.kind ? c64(b, 0.0) : c64(it.zre * b - a, it.zim * b);
  }
  LU[(int64_t)q * nw * ld + i * ld + c] = convert<C, c64>(v);
  if (i == 0) {
    perm[(int64_t)q * nw + c] = (int)c;
    if (c == 0) info[q] = 0;
  }
}

constexpr int64_t BT_CLASS = 256;

template <typename C>
struct BtFactors {
  int64_t nw = 0;
  C* LU = nullptr;
  C* Pinv = nullptr;
  int* perm = nullptr;
  int* pinv = nullptr;
};

struct BtClass {
  int64_t nw;
  int items, item0;
  size_t lu, dinv, pinv, ints;
};

template <typename C>
static int bt_class_launches(hipStream_t s, const BtClass& k, C* LU, C* Dinv, C* Pinv, int* ipiv, int* perm,
                             int* pinv, int* info, const BtItem* items) {
  const int64_t ld = lu_ld(k.nw);
  hipLaunchKernelGGL((k_bt_shift_form<C>), dim3((unsigned)((k.nw + 255) / 256), (unsigned)k.nw, (unsigned)k.items),
                     dim3(256), 0, s, k.nw, ld, items + k.item0, LU + k.lu, perm + k.ints, info + k.item0);
  MF_HIP_CHECK(hipGetLastError());
  MF_TRY(lu_factor<C>(s, k.nw, k.items, LU + k.lu, ipiv + k.ints, perm + k.ints, pinv + k.ints, info + k.item0,
                      Dinv + k.dinv));
  MF_TRY(panel_inverses<C>(s, k.nw, k.items, LU + k.lu, Dinv + k.dinv, Pinv + k.pinv));
  return 0;
}

// state[p]: 0 = not factored here (the problem runs the ordinary path), 1 = factored
// (fac[p] holds its factors), 2 = finished with info[p] (a singular shifted matrix or B)
template <typename C>
static int bt_factor(mfeast_handle h, int32_t nprob, const int64_t* n, const double* const* A, const int64_t* lda,
                     const double* const* B, const int64_t* ldb, const int32_t* fpm, const double* emin,
                     const double* emax, int32_t* m0, double* const* E, double* const* X, const int64_t* ldx,
                     int32_t* M, double* const* res, double* epsout, int32_t* loop, int32_t* info,
                     std::vector<int>& state, std::vector<BtFactors<C>>& fac, double& t_fact) {
  state.assign(nprob, 0);
  fac.assign(nprob, BtFactors<C>());
  t_fact = 0.0;
  if (fpm[49] != 0) return 0;  // fpm(50) refinement re-forms the shifted matrices per problem
  const int ne = fpm[1];
  std::vector<int> nf(nprob, 0);
  std::map<int64_t, std::vector<int>> byclass;
  for (int p = 0; p < nprob; ++p) {
    const double* Bp = B ? B[p] : nullptr;
    const int64_t ldbp = B ? ldb[p] : n[p];
    if (dense_check(h, 'F', n[p], A[p], lda[p], Bp, ldbp, fpm, emin[p], emax[p], &m0[p], E[p], X[p], ldx[p], &M[p],
                    res[p], &epsout[p], &loop[p], nullptr, nullptr) != 0)
      continue;
    nf[p] = ne + (Bp != nullptr ? 1 : 0);
    byclass[(n[p] + BT_CLASS - 1) / BT_CLASS * BT_CLASS].push_back(p);
  }
  if (byclass.empty()) return 0;
  // classes, largest first; item tables and buffer offsets
  std::vector<BtClass> cls;
  std::vector<BtItem> items;
  std::vector<int> first(nprob, -1);
  size_t lu = 0, dinv = 0, pinvs = 0, ints = 0;
  for (auto it = byclass.rbegin(); it != byclass.rend(); ++it) {
    BtClass k{it->first, 0, (int)items.size(), lu, dinv, pinvs, ints};
    for (int p : it->second) {
      std::vector<c64> z, w;
      double c_inf = 0.0;
      nodes_for(fpm, emin[p], emax[p], nullptr, nullptr, z, w, c_inf);
      first[p] = (int)items.size();
      const double* Bp = B ? B[p] : nullptr;
      const int64_t ldbp = B ? ldb[p] : n[p];
      for (int j = 0; j < ne; ++j) items.push_back(BtItem{A[p], Bp, lda[p], ldbp, n[p], z[j].re, z[j].im, 0, 0});
      if (Bp != nullptr) items.push_back(BtItem{A[p], Bp, lda[p], ldbp, n[p], 0.0, 0.0, 1, 0});
      k.items += nf[p];
    }
    const int64_t nblk = (k.nw + LU_NB - 1) / LU_NB;
    lu += (size_t)k.items * k.nw * lu_ld(k.nw);
    dinv += (size_t)k.items * nblk * 2 * LU_NB * LU_NB;
    pinvs += (size_t)k.items * panel_inverse_entries(k.nw);
    ints += (size_t)k.items * k.nw;
    cls.push_back(k);
  }
  const int nitems = (int)items.size();
  C* LU = (C*)h->ws(S_BT_LU, lu * sizeof(C));
  C* Dinv = (C*)h->ws(S_BT_DINV, dinv * sizeof(C));
  C* Pinv = (C*)h->ws(S_BT_PANINV, pinvs * sizeof(C));
  int* ipiv = (int*)h->ws(S_BT_IPIV, ints * 4);
  int* perm = (int*)h->ws(S_BT_PERM, ints * 4);
  int* pinv = (int*)h->ws(S_BT_PINV, ints * 4);
  int* dinfo = (int*)h->ws(S_BT_INFO, (size_t)nitems * 4);
  BtItem* ditems = (BtItem*)h->ws(S_BT_ITEMS, (size_t)nitems * sizeof(BtItem));
  if (!LU || !Dinv || !Pinv || !ipiv || !perm || !pinv || !dinfo || !ditems) return -2;
  hipStream_t s = h->stream;
  MF_HIP_CHECK(hipMemcpyAsync(ditems, items.data(), (size_t)nitems * sizeof(BtItem), hipMemcpyHostToDevice, s));
  // the graph depends on the sizes, the counts, the buffers and the product scheme
  std::vector<int64_t> key = {(int64_t)sizeof(C), (int64_t)gemm_3m(), (int64_t)(intptr_t)LU, (int64_t)(intptr_t)Dinv,
                              (int64_t)(intptr_t)Pinv, (int64_t)(intptr_t)ipiv, (int64_t)(intptr_t)perm,
                              (int64_t)(intptr_t)pinv, (int64_t)(intptr_t)dinfo, (int64_t)(intptr_t)ditems};
  for (const BtClass& k : cls) {
    key.push_back(k.nw);
    key.push_back(k.items);
  }
  GemmScratchScope scratch_scope(h);
  const bool prof_was = prof_on();
  prof_enable(false);
  // streams: [0] the origin of the graph (owned, so that capture never touches the
  // caller's stream), [1..] one per class; events: [0] fork, [1..] class joins, then the
  // hand-over from the caller's stream and back
  const size_t nc = cls.size();
  int rc = 0;
  while (rc == 0 && h->bt_streams.size() < nc + 1) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      rc = -2;
      break;
    }
    h->bt_streams.push_back(st);
  }
  while (rc == 0 && h->bt_events.size() < nc + 3) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      rc = -2;
      break;
    }
    h->bt_events.push_back(e);
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (rc == 0 && (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)) rc = -2;
  hipStream_t o = rc == 0 ? h->bt_streams[0] : nullptr;
  hipEvent_t ev_in = rc == 0 ? h->bt_events[nc + 1] : nullptr, ev_out = rc == 0 ? h->bt_events[nc + 2] : nullptr;
  if (rc == 0 && (hipEventRecord(ev_in, s) != hipSuccess || hipStreamWaitEvent(o, ev_in, 0) != hipSuccess ||
                  hipEventRecord(t0, o) != hipSuccess))
    rc = -2;
  if (rc == 0 && h->bt_exec != nullptr && h->bt_key == key) {
    if (hipGraphLaunch(h->bt_exec, o) != hipSuccess) rc = -2;
    if (rc == 0 && hipEventRecord(t1, o) != hipSuccess) rc = -2;
  } else if (rc == 0) {
    if (h->bt_exec != nullptr) (void)hipGraphExecDestroy(h->bt_exec);
    h->bt_exec = nullptr;
    h->bt_key.clear();
    // this call's factorization, with the tile autotuner on (it synchronizes per new class)
    set_gemm_tuning(true);
    for (const BtClass& k : cls)
      if (rc == 0) rc = bt_class_launches<C>(o, k, LU, Dinv, Pinv, ipiv, perm, pinv, dinfo, ditems);
    set_gemm_tuning(false);
    if (rc == 0 && hipEventRecord(t1, o) != hipSuccess) rc = -2;
    // the same launches captured for later calls: one branch per class
    if (rc == 0 && hipStreamBeginCapture(o, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      int crc = hipEventRecord(h->bt_events[0], o) == hipSuccess ? 0 : -2;
      for (size_t c = 0; c < nc && crc == 0; ++c) {
        hipStream_t st = h->bt_streams[c + 1];
        if (hipStreamWaitEvent(st, h->bt_events[0], 0) != hipSuccess) crc = -2;
        if (crc == 0) crc = bt_class_launches<C>(st, cls[c], LU, Dinv, Pinv, ipiv, perm, pinv, dinfo, ditems);
        if (crc == 0 && hipEventRecord(h->bt_events[c + 1], st) != hipSuccess) crc = -2;
        if (crc == 0 && hipStreamWaitEvent(o, h->bt_events[c + 1], 0) != hipSuccess) crc = -2;
      }
      hipGraph_t graph = nullptr;
      const bool ended = hipStreamEndCapture(o, &graph) == hipSuccess;
      if (crc == 0 && ended && graph != nullptr &&
          hipGraphInstantiate(&h->bt_exec, graph, nullptr, nullptr, 0) == hipSuccess)
        h->bt_key = key;
      else
        h->bt_exec = nullptr;
      if (graph != nullptr) (void)hipGraphDestroy(graph);
    }
  }
  if (o != nullptr && (hipEventRecord(ev_out, o) != hipSuccess || hipStreamWaitEvent(s, ev_out, 0) != hipSuccess))
    rc = -2;
  std::vector<int> hinfo(nitems);
  if (rc == 0 && hipMemcpyAsync(hinfo.data(), dinfo, (size_t)nitems * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
    rc = -2;
  if (hipStreamSynchronize(s) != hipSuccess) rc = -2;
  float ms = 0.0f;
  if (rc == 0) (void)hipEventElapsedTime(&ms, t0, t1);
  if (t0) (void)hipEventDestroy(t0);
  if (t1) (void)hipEventDestroy(t1);
  prof_enable(prof_was);
  t_fact = ms * 1e-3;
  if (rc != 0) return rc;
  for (const BtClass& k : cls) {
    const int64_t ld = lu_ld(k.nw);
    int q = 0;
    for (int p : byclass[k.nw]) {
      bool shift_ok = true, b_ok = true;
      for (int j = 0; j < nf[p]; ++j) {
        if (hinfo[first[p] + j] != 0) (j < ne ? shift_ok : b_ok) = false;
      }
      if (!shift_ok || !b_ok) {
        info[p] = !shift_ok ? -2 : -3;
        state[p] = 2;
      } else {
        state[p] = 1;
        BtFactors<C>& f = fac[p];
        f.nw = k.nw;
        f.LU = LU + k.lu + (size_t)q * k.nw * ld;
        f.Pinv = Pinv + k.pinv + (size_t)q * panel_inverse_entries(k.nw);
        f.perm = perm + k.ints + (size_t)q * k.nw;
        f.pinv = pinv + k.ints + (size_t)q * k.nw;
      }
      q += nf[p];
    }
  }
  return 0;
}

// one batched problem with its stored factors
template <typename C>
static int dense_entry_ext(mfeast_handle h, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                           int32_t* fpm, double emin, double emax, int32_t* m0, double* E, double* X, int64_t ldx,
                           int32_t* M, double* res, double* epsout, int32_t* loop, const BtFactors<C>& f) {
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  std::vector<c64> z, w;
  double c_inf = 0.0;
  nodes_for(fpm, emin, emax, nullptr, nullptr, z, w, c_inf);
  set_gemm_3m(fpm[52] == 0);
  DenseOp<double, C> op(h, 'F', n, A, lda, B, ldb, z, *m0);
  op.ext = true;
  op.nw = f.nw;
  op.LU = f.LU;
  op.Pinv = f.Pinv;
  op.perm = f.perm;
  op.pinv = f.pinv;
  return run_loop<double>(h, op, n, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, z, w, c_inf);
}

static int csr_entry(mfeast_handle h, char uplo, int64_t n, const double* a, const int32_t* ia, const int32_t* ja,
                     int32_t base, const double* b, const int32_t* ib, const int32_t* jb, int32_t* fpm, double emin,
                     double emax, int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M, double* res,
                     double* epsout, int32_t* loop, const double* zne, const double* wne) {
  if (n < 1) return 202;
  if (m0 == nullptr) return -114;
  if (*m0 < 1 || *m0 > n || *m0 > MAX_M0) return 201;
  if (!(emin < emax)) return 200;
  if (fpm == nullptr) return -111;
  if ((zne == nullptr) != (wne == nullptr)) return zne == nullptr ? -122 : -123;
  const int fi = check_fpm(fpm, zne != nullptr);
  if (fi) return fi;
  if (fpm[44] < 0 || fpm[44] > 16) return 145;
  if (fpm[45] < 1) return 146;
  if (h == nullptr) return -101;
  if (!(uplo == 'F' || uplo == 'f' || uplo == 'L' || uplo == 'l' || uplo == 'U' || uplo == 'u')) return -102;
  if (n > (int64_t)INT32_MAX - 1) return -103;
  if (a == nullptr) return -104;
  if (ia == nullptr) return -105;
  if (ja == nullptr) return -106;
  if (base != 0 && base != 1) return -107;
  if (b != nullptr && ib == nullptr) return -109;
  if (b != nullptr && jb == nullptr) return -110;
  if (E == nullptr) return -115;
  if (X == nullptr) return -116;
  if (ldx < n) return -117;
  if (M == nullptr) return -118;
  if (res == nullptr) return -119;
  if (epsout == nullptr) return -120;
  if (loop == nullptr) return -121;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  GemmScratchScope scratch_scope(h);
  std::vector<c64> z, w;
  double c_inf = 0.0;
  nodes_for(fpm, emin, emax, zne, wne, z, w, c_inf);
  set_gemm_3m(fpm[52] == 0);
  const double tol = std::pow(10.0, -fpm[44]);
  fpm[59] = 0;
  int info;
  int64_t its;
  if (fpm[41] == 1) {
    CsrOp<c32> op(h, uplo, n, a, ia, ja, base, b, ib, jb, z, *m0, fpm[45], tol);
    info = run_loop<double>(h, op, n, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, z, w, c_inf);
    its = op.iterations;
  } else {
    CsrOp<c64> op(h, uplo, n, a, ia, ja, base, b, ib, jb, z, *m0, fpm[45], tol);
    info = run_loop<double>(h, op, n, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, z, w, c_inf);
    its = op.iterations;
  }
  fpm[59] = (int32_t)std::min<int64_t>(its, INT32_MAX);
  return info;
}

// ---------------------------------------------------------------------------
// The allocation-free entry point's workspace: one static device array per GPU (each
// device holds its own copy at its own address until the process ends).  Host code
// never passes the array's name to a kernel: its device address is looked up once per
// device, with that device current, and kept.
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64] = {};

// device address of `scratch` on the current device `device` (nullptr on failure)
static void* noalloc_scratch(int device) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return nullptr;
    g_scratch_ptr[device] = p;
  }
  return g_scratch_ptr[device];
}

extern "C" {

int mfeast_create(mfeast_handle* h, int device, void* hip_stream) {
  if (h == nullptr) return -101;
  *h = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count <= 0 || device < 0 || device >= count) return -900;
  if (hipSetDevice(device) != hipSuccess) return -900;
  mfeast_ctx* c = new mfeast_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  *h = c;
  return 0;
}

int mfeast_destroy(mfeast_handle h) {
  if (h == nullptr) return -101;
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  for (mfeast_ctx* w : h->workers) {
    if (w->owns_stream && w->stream) (void)hipStreamDestroy(w->stream);
    w->stream = nullptr;
    (void)mfeast_destroy(w);
  }
  h->workers.clear();
  if (h->bt_exec) (void)hipGraphExecDestroy(h->bt_exec);
  for (hipEvent_t e : h->bt_events) (void)hipEventDestroy(e);
  for (hipStream_t st : h->bt_streams) (void)hipStreamDestroy(st);
  for (int i = 0; i < S_NSLOTS; ++i)
    if (h->buf[i]) (void)hipFree(h->buf[i]);
  h->csrA.release();
  h->csrB.release();
  h->release_aux();
  if (h->pinned) (void)hipHostFree(h->pinned);
  if (h->pinned_i) (void)hipHostFree(h->pinned_i);
  if (h->pinned_aux) (void)hipHostFree(h->pinned_aux);
  delete h;
  return 0;
}

int mfeast_set_stream(mfeast_handle h, void* hip_stream) {
  if (h == nullptr) return -101;
  h->stream = static_cast<hipStream_t>(hip_stream);
  return 0;
}

void mfeast_init(int32_t* fpm) {
  if (fpm == nullptr) return;
  for (int i = 0; i < 64; ++i) fpm[i] = 0;
  fpm[0] = 0;    // fpm(1)  no runtime comments
  fpm[1] = 8;    // fpm(2)  half-contour nodes
  fpm[2] = 12;   // fpm(3)  eps = 1e-12
  fpm[3] = 20;   // fpm(4)  refinement loops
  fpm[4] = 0;    // fpm(5)  no initial guess
  fpm[5] = 1;    // fpm(6)  residual criterion
  fpm[7] = 16;   // fpm(8)  full-contour nodes (non-Hermitian, unused)
  fpm[9] = 1;    // fpm(10) factorizations stored
  fpm[13] = 0;   // fpm(14) normal run
  fpm[14] = 2;   // fpm(15) left = right* (Hermitian)
  fpm[15] = 0;   // fpm(16) Gauss-Legendre
  fpm[17] = 30;  // fpm(18) ellipse ratio 0.30
  fpm[40] = 1;   // fpm(41) matrix scaling (sparse drivers)
  fpm[41] = 1;   // fpm(42) single-precision solves
  fpm[44] = 1;   // fpm(45) BiCGStab accuracy 1e-1
  fpm[45] = 40;  // fpm(46) BiCGStab iterations
  fpm[49] = 0;   // fpm(50) extra refinement steps of the FP32 solves (dense)
  fpm[50] = 0;   // fpm(51) seed of the random starting block
  fpm[51] = 0;   // fpm(52) per-class kernel timing (mfeast_get_profile) off
  fpm[52] = 0;   // fpm(53) complex FP32 products: 0 three-product scheme, 1 four-product
  fpm[53] = 90;  // fpm(54) Zolotarev rule: flat band, percent of the half-width
}

int mfeast_contour(double emin, double emax, int32_t ne, int32_t rule, int32_t ratio_pct, double* zne, double* wne) {
  if (!(emin < emax)) return 200;
  if (rule < 0 || rule > 2) return 116;
  if (((rule == 0 || rule == 2) && !gauss_allowed(ne)) || ne < 1) return 102;
  if (ratio_pct <= 0) return 118;
  if (rule == 2 && ratio_pct > 99) return 154;
  if (zne == nullptr) return -106;
  if (wne == nullptr) return -107;
  std::vector<c64> z, w;
  if (rule == 2) {
    double c_inf = 0.0;
    zolotarev_contour(emin, emax, ne, ratio_pct, z, w, c_inf);
  } else {
    make_contour(emin, emax, ne, rule, ratio_pct, z, w);
  }
  for (int j = 0; j < ne; ++j) {
    zne[2 * j] = z[j].re;
    zne[2 * j + 1] = z[j].im;
    wne[2 * j] = w[j].re;
    wne[2 * j + 1] = w[j].im;
  }
  return 0;
}

int mfeast_zolotarev(double emin, double emax, int32_t ne, int32_t band_pct, double* zne, double* wne,
                     double* c_inf) {
  if (!(emin < emax)) return 200;
  if (!gauss_allowed(ne)) return 102;
  if (band_pct < 1 || band_pct > 99) return 154;
  if (zne == nullptr) return -105;
  if (wne == nullptr) return -106;
  if (c_inf == nullptr) return -107;
  std::vector<c64> z, w;
  zolotarev_contour(emin, emax, ne, band_pct, z, w, *c_inf);
  for (int j = 0; j < ne; ++j) {
    zne[2 * j] = z[j].re;
    zne[2 * j + 1] = z[j].im;
    wne[2 * j] = w[j].re;
    wne[2 * j + 1] = w[j].im;
  }
  return 0;
}

int mfeast_dsygv(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                 int32_t* fpm, double emin, double emax, int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M,
                 double* res, double* epsout, int32_t* loop, const double* zne, const double* wne) {
  return dense_entry<double>(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, zne,
                             wne);
}

int mfeast_dsygv_noalloc(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda, const double* B,
                         int64_t ldb, int32_t* fpm, double emin, double emax, int32_t* m0, double* E, double* X,
                         int64_t ldx, int32_t* M, double* res, double* epsout, int32_t* loop, const double* zne,
                         const double* wne) {
  if (h == nullptr || fpm == nullptr) {
    // argument errors only: the checks of mfeast_dsygv, in the table's order
    return dense_entry<double>(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop,
                               zne, wne);
  }
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  void* arena = noalloc_scratch(h->device);
  if (arena == nullptr) return -900;
  // a call-local context: same device and stream, workspace carved from the array, no
  // per-class timing (its events would be created on first use)
  int32_t f[64];
  for (int i = 0; i < 64; ++i) f[i] = fpm[i];
  f[51] = 0;
  mfeast_ctx tmp;
  tmp.device = h->device;
  tmp.stream = h->stream;
  tmp.arena = static_cast<char*>(arena);
  tmp.arena_cap = NOALLOC_BYTES;
  int info = dense_entry<double>(&tmp, uplo, n, A, lda, B, ldb, f, emin, emax, m0, E, X, ldx, M, res, epsout, loop,
                                 zne, wne);
  if (tmp.arena_overflow) info = -901;
  for (int i = 0; i < 8; ++i) h->timing[i] = tmp.timing[i];
  return info;
}

int mfeast_zhegv(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                 int32_t* fpm, double emin, double emax, int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M,
                 double* res, double* epsout, int32_t* loop, const double* zne, const double* wne) {
  return dense_entry<c64>(h, uplo, n, A, lda, B, ldb, fpm, emin, emax, m0, E, X, ldx, M, res, epsout, loop, zne,
                          wne);
}

int mfeast_dcsrgv(mfeast_handle h, char uplo, int64_t n, const double* a, const int32_t* ia, const int32_t* ja,
                  int32_t index_base, const double* b, const int32_t* ib, const int32_t* jb, int32_t* fpm,
                  double emin, double emax, int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M,
                  double* res, double* epsout, int32_t* loop, const double* zne, const double* wne) {
  return csr_entry(h, uplo, n, a, ia, ja, index_base, b, ib, jb, fpm, emin, emax, m0, E, X, ldx, M, res, epsout,
                   loop, zne, wne);
}

int mfeast_dsygv_batched(mfeast_handle h, int32_t nprob, const int64_t* n, const double* const* A,
                         const int64_t* lda, const double* const* B, const int64_t* ldb, const int32_t* fpm,
                         const double* emin, const double* emax, int32_t* m0, double* const* E, double* const* X,
                         const int64_t* ldx, int32_t* M, double* const* res, double* epsout, int32_t* loop,
                         int32_t* info) {
  if (h == nullptr) return -101;
  if (nprob < 1) return -102;
  if (n == nullptr) return -103;
  if (A == nullptr) return -104;
  if (lda == nullptr) return -105;
  if (B != nullptr && ldb == nullptr) return -107;
  if (fpm == nullptr) return -108;
  if (emin == nullptr) return -109;
  if (emax == nullptr) return -110;
  if (m0 == nullptr) return -111;
  if (E == nullptr) return -112;
  if (X == nullptr) return -113;
  if (ldx == nullptr) return -114;
  if (M == nullptr) return -115;
  if (res == nullptr) return -116;
  if (epsout == nullptr) return -117;
  if (loop == nullptr) return -118;
  if (info == nullptr) return -119;
  if (hipSetDevice(h->device) != hipSuccess) return -900;
  Timer total;
  total.start();
  // inputs may still be in flight on the caller's stream
  MF_HIP_CHECK(hipStreamSynchronize(h->stream));
  static const int env_streams = getenv("MFEAST_BATCH_STREAMS") ? atoi(getenv("MFEAST_BATCH_STREAMS")) : 8;
  const int nw = std::max(1, std::min<int>(nprob, env_streams));
  while ((int)h->workers.size() < nw) {
    mfeast_ctx* w = new mfeast_ctx();
    w->device = h->device;
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess) {
      delete w;
      return -2;
    }
    w->owns_stream = true;
    h->workers.push_back(w);
  }
  // the factorizations of every problem and node first, in padded size classes (one graph)
  int32_t fb[64];
  for (int i = 0; i < 64; ++i) fb[i] = fpm[i];
  const bool fp32 = fpm[41] == 1;
  const bool prof_req = fpm[51] == 1 || h->prof_all;
  std::vector<int> state;
  std::vector<BtFactors<c32>> fac32;
  std::vector<BtFactors<c64>> fac64;
  double t_fact = 0.0;
  set_gemm_3m(fpm[52] == 0);
  const int brc = fp32 ? bt_factor<c32>(h, nprob, n, A, lda, B, ldb, fb, emin, emax, m0, E, X, ldx, M, res, epsout,
                                        loop, info, state, fac32, t_fact)
                       : bt_factor<c64>(h, nprob, n, A, lda, B, ldb, fb, emin, emax, m0, E, X, ldx, M, res, epsout,
                                        loop, info, state, fac64, t_fact);
  if (brc != 0) state.assign(nprob, 0);
  double fact_flops = 0.0;
  for (int p = 0; p < nprob; ++p)
    if (state[p] != 0) fact_flops += (fpm[1] + (B && B[p] ? 1 : 0)) * (8.0 / 3.0) * (double)n[p] * n[p] * n[p];
  // largest problems first
  std::vector<int> order(nprob);
  for (int p = 0; p < nprob; ++p) order[p] = p;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return n[a] > n[b]; });
  std::atomic<int> next(0);
  for (mfeast_ctx* w : h->workers)
    for (int i = 0; i < K_NCLASS * 4; ++i) w->prof_sum[i] = 0.0;
  auto work = [&](mfeast_ctx* w) {
    (void)hipSetDevice(w->device);
    set_coop_allowed(false);
    for (;;) {
      const int t = next.fetch_add(1);
      if (t >= nprob) break;
      const int p = order[t];
      int32_t f[64];
      for (int i = 0; i < 64; ++i) f[i] = fpm[i];
      f[51] = (fpm[51] == 1 || h->prof_all) ? 1 : 0;
      const double* Bp = B ? B[p] : nullptr;
      const int64_t ldbp = B ? ldb[p] : n[p];
      if (state[p] == 2) continue;
      if (state[p] == 1)
        info[p] = fp32 ? dense_entry_ext<c32>(w, n[p], A[p], lda[p], Bp, ldbp, f, emin[p], emax[p], &m0[p], E[p],
                                              X[p], ldx[p], &M[p], res[p], &epsout[p], &loop[p], fac32[p])
                       : dense_entry_ext<c64>(w, n[p], A[p], lda[p], Bp, ldbp, f, emin[p], emax[p], &m0[p], E[p],
                                              X[p], ldx[p], &M[p], res[p], &epsout[p], &loop[p], fac64[p]);
      else
        info[p] = dense_entry<double>(w, 'F', n[p], A[p], lda[p], Bp, ldbp, f, emin[p], emax[p], &m0[p], E[p], X[p],
                                      ldx[p], &M[p], res[p], &epsout[p], &loop[p], nullptr, nullptr);
      for (int i = 0; i < K_NCLASS * 4; ++i) w->prof_sum[i] += w->prof[i];
    }
    (void)hipStreamSynchronize(w->stream);
    set_coop_allowed(true);
  };
  std::vector<std::thread> threads;
  for (int i = 1; i < nw; ++i) threads.emplace_back(work, h->workers[i]);
  work(h->workers[0]);
  for (std::thread& t : threads) t.join();
  // per-class timings: the sum over the workers' last calls is not meaningful, so each
  // worker keeps a running sum of its calls' classes (see work above) and they are added
  for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] = 0.0;
  for (int wi = 0; wi < nw; ++wi)
    for (int i = 0; i < K_NCLASS * 4; ++i) h->prof[i] += h->workers[wi]->prof_sum[i];
  if (prof_req && fact_flops > 0.0) {
    h->prof[K_BT_FACT * 4 + 0] = 1.0;
    h->prof[K_BT_FACT * 4 + 1] = t_fact * 1e3;
    h->prof[K_BT_FACT * 4 + 2] = fact_flops;
  }
  int worst = 0;
  for (int p = 0; p < nprob; ++p)
    if (info[p] < 0 && (worst >= 0 || info[p] < worst)) worst = info[p];
  if (worst == 0)
    for (int p = 0; p < nprob; ++p) worst = std::max(worst, (int)info[p]);
  for (int i = 0; i < 8; ++i) h->timing[i] = 0.0;
  h->timing[0] = t_fact;
  h->timing[5] = total.stop();
  h->timing[6] = (double)nprob;
  return worst;
}

void mfeast_init_ifeast(int32_t* fpm) {
  if (fpm == nullptr) return;
  mfeast_init(fpm);
  fpm[1] = 4;     // fpm(2)  half-contour nodes
  fpm[3] = 50;    // fpm(4)  refinement loops
  fpm[15] = 1;    // fpm(16) trapezoidal rule
  fpm[17] = 100;  // fpm(18) circle
}

void mfeast_init_stochastic(int32_t* fpm) {
  if (fpm == nullptr) return;
  mfeast_init(fpm);
  fpm[1] = 3;    // fpm(2)  half-contour nodes
  fpm[7] = 6;    // fpm(8)  full-contour nodes (non-Hermitian, unused)
  fpm[13] = 2;   // fpm(14) stochastic estimate of the count
  fpm[14] = 1;   // fpm(15) one-sided contour
}

int mfeast_set_profiling(mfeast_handle h, int32_t on) {
  if (h == nullptr) return -101;
  if (on != 0 && on != 1) return -102;
  h->prof_all = on == 1;
  return 0;
}

int mfeast_get_profile(mfeast_handle h, double* out, int32_t count) {
  if (h == nullptr) return -101;
  if (out == nullptr) return -102;
  for (int i = 0; i < count && i < K_NCLASS * 4; ++i) out[i] = h->prof[i];
  return 0;
}

int mfeast_get_timing(mfeast_handle h, double* out) {
  if (h == nullptr) return -101;
  if (out == nullptr) return -102;
  for (int i = 0; i < 8; ++i) out[i] = h->timing[i];
  return 0;
}

}  // extern "C"
