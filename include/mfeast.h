/*
 * mfeast: Hermitian FEAST contour-integration eigensolver for AMD MI355X (gfx950).
 *
 * C interface of libmfeast.so.  The problem statement follows the FEAST v4.0 User
 * Guide (arXiv:2002.04807): find the eigenpairs (lambda, x) of A x = lambda B x,
 * A Hermitian (real symmetric), B Hermitian positive definite (or B = I), with
 * lambda in the closed interval [Emin, Emax], using a search subspace of size M0
 * (Section 3.2 "FEAST Hermitian", Table tab-common1 for the common arguments,
 * Table tab-spec1 for the dense storage arguments).  Algorithm options travel in the
 * integer array fpm[64] (Table tab_fpm; C index = Fortran index - 1), results and
 * errors use the guide's info codes (Table tab_info).
 *
 * Conventions for every entry point:
 *  - Matrix and vector arguments named "device" are HIP device pointers (for example
 *    the data pointers of PyTorch tensors on the GPU); everything else is host memory.
 *  - Dense matrices are column-major with a leading dimension (LAPACK), as in the
 *    guide; complex numbers are interleaved (re, im) doubles.
 *  - The caller owns every buffer passed in; the library never frees them.  A handle
 *    owns its workspace (including the stored LU factors of all contour nodes), which
 *    grows on demand, is reused by later calls and is released by mfeast_destroy.
 *  - Every call returns info.  Argument checks run on the host before any device
 *    work, in the order of Table tab_info: 202 (N), 201 (M0), 200 (Emin/Emax),
 *    100+i (fpm(i), Fortran numbering), then -(100+i) for an invalid i-th argument of
 *    the call (1-based position in the C prototype).  Warnings: 1 no eigenvalue in the
 *    interval, 2 no convergence within fpm(4) loops, 3 M0 too small (M >= M0),
 *    4 subspace returned after one contour (fpm(14)=1), 5 only the stochastic estimate
 *    of the eigenvalue count returned (fpm(14)=2).  Errors: -2 device or
 *    factorization failure (zero pivot, non-finite value, HIP error), -3 the reduced
 *    problem is not positive definite (B may not be positive definite).
 *    -900 no usable HIP device for the handle (a code outside the guide's ranges).
 *  - Calls are synchronous with respect to the host: the results are complete on the
 *    device when the call returns (the subspace iteration needs host-visible scalars
 *    after every Rayleigh-Ritz step).  A handle may be used by one thread at a time.
 */
#ifndef MFEAST_H
#define MFEAST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfeast_ctx* mfeast_handle;

/* Create a handle bound to HIP device `device`; work is issued on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  For complex Hermitian problems the
 * handle also creates, on first use, a non-blocking stream of its own and two events:
 * the conjugate-transpose block solves run there next to the forward ones and are
 * joined back to `hip_stream` before the contour sum.  Returns 0, -101 (h NULL) or
 * -900. */
int mfeast_create(mfeast_handle* h, int device, void* hip_stream);

/* Release the handle, its workspace and its internal stream.  Returns 0 or -101. */
int mfeast_destroy(mfeast_handle h);

/* Change the stream later calls of this handle issue work on. */
int mfeast_set_stream(mfeast_handle h, void* hip_stream);

/* Default parameters (feastinit; Table tab_fpm).  fpm: 64 int32 (host).
 * Project slots (reserved in the guide): fpm(50) = 0..8 extra refinement steps of the
 * FP32 contour solves of the dense drivers (default 0; each step forms the FP64
 * residual of every node's system and solves it again with the FP32 factors),
 * fpm(51) seed of the random starting block, fpm(52) = 1 records per-class kernel
 * timings for mfeast_get_profile, fpm(53) = 1 forms complex products with four real
 * products instead of Gauss's three (default 0: three; FP32 products everywhere, FP64
 * products outside the LU trailing updates, which always take four), fpm(54) = 1..99 the flat
 * band of the Zolotarev rule in percent of the half-width (default 90; see
 * mfeast_zolotarev).  Return 154 from the drivers: fpm(16)=2 with fpm(54) outside 1..99. */
void mfeast_init(int32_t* fpm);

/* Half-contour nodes and weights (zfeast_contour; Section 4.2 "Search contour",
 * Table tab_contour).  Ellipse through Emin and Emax centred on the real axis with
 * axis ratio ratio_pct/100; rule 0 Gauss-Legendre (ne in 1..20, 24, 32, 40, 48, 56),
 * 1 trapezoidal (ne >= 1), 2 Zolotarev (fpm(16)=2; ne as for Gauss; ratio_pct is then
 * the flat band fpm(54) in 1..99, and the rule's constant term is returned by
 * mfeast_zolotarev).  zne, wne: host arrays of 2*ne doubles (re, im) receiving
 * the upper-half nodes z_j (j = 1 nearest Emin) and weights w_j such that the spectral
 * projector is approximated by sum_j [w_j f(z_j) + conj(w_j) f(conj z_j)].
 * Returns 0, 200, 102, 116, 118, 154 or -(100+i) for a NULL array. */
int mfeast_contour(double emin, double emax, int32_t ne, int32_t rule, int32_t ratio_pct,
                   double* zne, double* wne);

/* Zolotarev rule (fpm(16)=2, Table tab_fpm: Hermitian problems only; the guide cites
 * Guettel, Polizzi, Tang and Viaud 2015 for it).  Zolotarev's best uniform approximation
 * Z of sign(x) on [-1,-l] u [l,1] by an odd rational function of type (2ne-1, 2ne),
 * composed with the map x = kappa (1 + t)/(1 - t), t = (lambda - c)/r, gives the filter
 * f(lambda) = (1 + Z)/2 of the interval [emin, emax] (centre c, half-width r): within
 * delta/2 of 1 for |t| <= a and of 0 for |t| >= 1/a, exactly 1/2 at emin and emax, with
 * a = band_pct/100, kappa = (1 - a)/(1 + a), l = kappa^2 and delta Zolotarev's error.
 * Its ne poles in the upper half plane lie on the circle through emin and emax.  In
 * partial fractions f(lambda) = c_inf + sum_j 2 Re(w_j / (z_j - lambda)).
 *  zne, wne  host, 2*ne doubles each: nodes z_j (ascending real part) and weights w_j
 *  c_inf     host, 1 double: the constant term f(infinity) (of size delta/2); the
 *            drivers apply it to the block itself (c_inf Y in the first contour, and
 *            inside the filter of the residual form)
 * Returns 0, 200 (emin >= emax), 102 (ne not a permitted Gauss count), 154 (band_pct
 * outside 1..99), or -(100+i) for a NULL array argument i. */
int mfeast_zolotarev(double emin, double emax, int32_t ne, int32_t band_pct, double* zne, double* wne,
                     double* c_inf);

/* Dense real symmetric problem (dfeast_sygv / dfeast_syev and their {x} forms).
 *  h       handle
 *  uplo    'F', 'L' or 'U': which part of A (and B) is referenced (Table tab-spec1)
 *  n       order of the system (1 <= n <= 16384: the dense LU kernels' limit; else 202)
 *  A       device, n x n column-major, leading dimension lda >= n
 *  B       device, n x n column-major (ldb >= n), or NULL for B = I (standard problem)
 *  fpm     host, 64 int32 (in/out; fpm(60) unused here)
 *  emin, emax  search interval (closed)
 *  m0      host, in: subspace size M0 (1 <= M0 <= min(n, 1024): the reduced eigensolver's
 *          limit; else 201); out: possibly reduced M0
 *  E       device, m0 doubles: eigenvalues, inside pairs first (ascending), then outside
 *          (in: initial guess when fpm(5)=1)
 *  X       device, n x m0 column-major (ldx >= n): eigenvectors following E, or the
 *          subspace Q after one contour when fpm(14)=1 (in: initial subspace when fpm(5)=1)
 *  M       host: number of eigenvalues found in [emin, emax] (the estimate rounded to the
 *          nearest integer when fpm(14)=2)
 *  res     device, m0 doubles: ||A x_i - lambda_i B x_i|| / ||alpha B x_i||,
 *          alpha = max(|emin|, |emax|)
 *  epsout  host: relative trace change |trace_k - trace_{k-1}| / alpha
 *  loop    host: index of the last subspace iteration (0 = first contour)
 *  zne,wne host, 2*fpm(2) doubles each, or both NULL: custom nodes and half-contour
 *          weights (expert mode, no constant term); NULL = generated from fpm(2),
 *          fpm(16), fpm(18), and fpm(54) for the Zolotarev rule (fpm(16)=2)
 * fpm(42)=1 (default) factors and solves the shifted systems in complex FP32 with the
 * FP64 residual form of the iteration (plus fpm(50) refinement steps of each solve);
 * fpm(42)=0 uses complex FP64 throughout.  FP32 solves reach a residual floor near 1e-11:
 * with fpm(50)=0, once the found pairs' largest residual is above the tolerance and
 * either below 1e-9 with a tolerance below 1e-10, or has fallen by less than ten times in
 * an iteration, the later contours add one refinement step per solve (not in
 * mfeast_dsygv_noalloc, and not for the batched driver's padded factors).  Return 150:
 * fpm(50) outside 0..8; 153: fpm(53) not 0 or 1. */
int mfeast_dsygv(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda,
                 const double* B, int64_t ldb, int32_t* fpm, double emin, double emax,
                 int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M, double* res,
                 double* epsout, int32_t* loop, const double* zne, const double* wne);

/* Allocation-free variant of mfeast_dsygv, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, semantics and results as mfeast_dsygv; every workspace
 * buffer of the call (stored LU factors, solve blocks, Rayleigh-Ritz blocks, reduction
 * partials, split-K partials) is carved from one static device array of 64 MiB per GPU
 * (held by each GPU the library runs on until the process ends), host staging uses
 * ordinary host memory, and the call makes no hipMalloc, hipHostMalloc, hipFree,
 * stream or event creation.  The handle supplies the device and stream only; its own
 * workspace is neither used nor grown.  fpm(52) is ignored (no per-class timing).
 * The array is shared by every call on a GPU and keeps the last call's contents (the
 * call clears what it needs): calls that overlap on one GPU, from any thread or handle,
 * race and must be serialized by the caller.
 * Returns the codes of mfeast_dsygv, and -901 when the call's workspace does not fit the
 * array (detected before any kernel runs; about n <= 256 with m0 <= 96 fit in FP64
 * with B, larger n with FP32 solves, B = NULL or a smaller m0). */
int mfeast_dsygv_noalloc(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda,
                         const double* B, int64_t ldb, int32_t* fpm, double emin, double emax,
                         int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M, double* res,
                         double* epsout, int32_t* loop, const double* zne, const double* wne);

/* Dense complex Hermitian problem (zfeast_hegv / zfeast_heev).  Same arguments as
 * mfeast_dsygv with A, B, X complex (interleaved doubles).  The conjugate contour node
 * is handled by a solve with (z B - A)^H that reuses the factorization of z B - A
 * (Hermitian RCI cases 20/21). */
int mfeast_zhegv(mfeast_handle h, char uplo, int64_t n, const double* A, int64_t lda,
                 const double* B, int64_t ldb, int32_t* fpm, double emin, double emax,
                 int32_t* m0, double* E, double* X, int64_t ldx, int32_t* M, double* res,
                 double* epsout, int32_t* loop, const double* zne, const double* wne);

/* Non-Hermitian FEAST (Section 3.3 "FEAST Non-Hermitian"; Tables tab-common2, tab-rci2)
 * ---------------------------------------------------------------------------------------
 * mfeast_init_general: mfeast_init, then the non-Hermitian defaults of Table tab_fpm:
 * fpm(15)=0 (two-sided: right and left eigenvectors), fpm(16)=1 (trapezoidal),
 * fpm(18)=100 (circle); fpm(8)=16 full-contour nodes is common. */
void mfeast_init_general(int32_t* fpm);

/* Full-contour nodes and weights (zfeast_gcontour; Section 4.2 "Search contour"): the
 * ellipse z(t) = Emid + e^{i phi} (r cos t + i e r sin t), t in [0, 2 pi), with e =
 * ratio_pct/100 and phi = angle_deg degrees (counter-clockwise; 0 keeps the axes on the
 * real and imaginary directions), ne nodes: rule 1 trapezoidal (t_j = 2 pi (j - 1/2)/ne,
 * ne >= 2), rule 0 Gauss-Legendre in t (ne in 2..40, 48, 64, 80, 96, 112).  The filter
 * of an eigenvalue lambda is sum_j w_j / (z_j - lambda).  zne, wne: host, 2*ne doubles.
 * Returns 0, 200 (r <= 0), 108, 116, 118, 119 (angle outside -180..180), -108, -109. */
int mfeast_gcontour(double emid_re, double emid_im, double r, int32_t ne, int32_t rule, int32_t ratio_pct,
                    int32_t angle_deg, double* zne, double* wne);

/* Dense complex general problem A x = lambda B x (zfeast_gegv / zfeast_geev and their {x}
 * forms; real general matrices are passed as complex): the eigenvalues inside the full
 * contour of Emid, r, fpm(18), fpm(19) with fpm(8) nodes (or the expert nodes zne,
 * weights wne: host, 2*fpm(8) doubles each), their right eigenvectors and, with
 * fpm(15)=0, their left eigenvectors (y^H A = lambda y^H B).  Each node's z_j B - A is
 * factored once; right solves use (z_j B - A)^-1 and left solves (z_j B - A)^-H with the
 * same factors (RCI cases 10/11/20/21).  fpm(42)=1 factors and solves in complex FP32
 * with the FP64 residual form, fpm(42)=0 in complex FP64.
 *  A, B    device, n x n complex column-major (lda, ldb >= n); B NULL for B = I
 *  fpm     host, 64 int32 (fpm(14) must be 0)
 *  epsout  host: |trace_k - trace_{k-1}| / alpha, alpha = |Emid| + r
 *  loop    host: index of the last iteration
 *  emid    host, 2 doubles (re, im): centre of the ellipse; r > 0 its horizontal radius
 *  m0      host, in: subspace size (1 <= M0 <= min(n, 512)); out: possibly reduced
 *  E       device, 2*m0 doubles: complex eigenvalues, the M inside the contour first, then
 *          the others (each group by real part, then imaginary part)
 *  X       device, complex column-major (ldx >= n): right eigenvectors (unit 2-norm) in
 *          columns 0..m0-1 following E; with fpm(15)=0 left eigenvectors, scaled so that
 *          y_i^H B x_i = 1, in columns M0..M0+m0-1 (M0 the value on entry), so X holds
 *          2*M0 columns.  With fpm(5)=1 the same columns hold the starting blocks.
 *  M       host: number of eigenvalues inside the contour
 *  res     device: ||A x_i - lambda_i B x_i|| / ||alpha B x_i|| in res[0..m0-1]; with
 *          fpm(15)=0 ||A^H y_i - conj(lambda_i) B^H y_i|| / ||alpha B^H y_i|| in
 *          res[M0..M0+m0-1] (2*M0 doubles)
 * The reduced pencil (Q~^H A Q, Q~^H B Q on orthonormal, rank-truncated bases of the two
 * subspaces) is solved on the device in one workgroup.  Returns Table tab_info codes:
 * 202 (n), 201 (M0), 200 (r or Emid), 1xx (fpm(i)), -(100+i) for argument i, 1 (no
 * eigenvalue inside), 2 (no convergence), 3 (M0 too small), -2, -3 (reduced pencil
 * singular or its eigensolver did not converge), -900. */
int mfeast_zgegv(mfeast_handle h, int64_t n, const double* A, int64_t lda, const double* B, int64_t ldb,
                 int32_t* fpm, double* epsout, int32_t* loop, const double* emid, double r, int32_t* m0,
                 double* E, double* X, int64_t ldx, int32_t* M, double* res, const double* zne,
                 const double* wne);

/* Defaults of the polynomial driver: mfeast_init_general, then fpm(15)=1 (right
 * eigenvectors only, the one mode of Section 3.4's drivers). */
void mfeast_init_polynomial(int32_t* fpm);

/* Dense complex polynomial eigenvalue problem sum_{k=0..p} lambda^k A_k x = 0 (Section
 * 3.4, zfeast_gepev / zfeast_sypev forms; real or symmetric coefficients are passed as
 * general complex ones): the eigenvalues inside the full contour of Emid, r, fpm(18),
 * fpm(19) with fpm(8) nodes (or the expert nodes zne, weights wne) and their right
 * eigenvectors.  P(z_j) = sum_k z_j^k A_k is formed and factored once per node (RCI
 * cases 10/11); the first iteration applies sum_j w_j P(z_j)^-1 to the starting block,
 * later ones the residual form rho(lambda_i) x_i - sum_j w_j/(z_j - lambda_i)
 * P(z_j)^-1 P(lambda_i) x_i.  Rayleigh-Ritz projects every A_k on an orthonormal,
 * rank-truncated basis of the subspace and solves the companion linearization of the
 * projected polynomial (size p m <= 512) on the device in one workgroup; of its p m
 * eigenvalues the m nearest the contour's centre in the ellipse's own metric are kept.
 * A pair is counted in M when its value lies inside the contour and its residual is
 * below min(0.1, 10^(-fpm(3)/2)); info 3 when all m kept values lie inside (the p m values
 * of the linearization crowd the subspace: about 1.5 times the count inside is enough
 * for M0).  fpm(42)=1 factors and solves in complex FP32, fpm(42)=0 in FP64.
 *  p       degree, 1 <= p <= 8
 *  A       device, the p+1 complex column-major n x n matrices A_0..A_p, element (i, j)
 *          of A_k at A[2*(i + j*lda + k*lda*n)] (re, im) (Table tab-spec3's A(LDA,N,p+1))
 *  fpm     host, 64 int32 (fpm(15) must be 1)
 *  m0      host, in: 1 <= M0 <= n with p*M0 <= 512; out: possibly reduced
 *  E, X, M, epsout, loop, emid, r, zne, wne as for mfeast_zgegv (right eigenvectors only)
 *  res     device, m0 doubles: ||P(lambda_i) x_i|| / sum_k |lambda_i|^k ||A_k x_i||
 * Returns Table tab_info codes: 202 (n), 201 (M0), 200 (r or Emid), 115 (fpm(15) != 1),
 * other 1xx (fpm(i)), -102 (p), -(100+i) for argument i, 1, 2, 3, -2, -3 (singular
 * projected leading coefficient or the reduced eigensolver did not converge), -900. */
int mfeast_zgepev(mfeast_handle h, int32_t p, int64_t n, const double* A, int64_t lda, int32_t* fpm,
                  double* epsout, int32_t* loop, const double* emid, double r, int32_t* m0, double* E, double* X,
                  int64_t ldx, int32_t* M, double* res, const double* zne, const double* wne);

/* Many independent dense real symmetric problems in one call (the first of the three
 * levels of parallelism of Section 1.1, independent search intervals or problems): the
 * arguments of mfeast_dsygv as arrays over nprob problems.  n, lda, ldb, ldx, emin, emax,
 * m0 (in/out), M, epsout, loop, info are host arrays of nprob entries; A, B, E, X, res are
 * host arrays of nprob device pointers (B may be NULL for B = I everywhere, or hold NULL
 * entries); fpm (64 entries) is shared.  First the shifted matrices of every problem and
 * node (and B) are formed and factored together: grouped in size classes (the order
 * rounded up to a multiple of 256, padded with an identity block), each class one batched
 * blocked LU, all classes as parallel branches of one HIP graph that the handle captures at
 * the first call with a given set of sizes and keeps for later calls with the same sizes
 * (the first call also tunes the GEMM tiles of the LU updates; the handle's device memory
 * holds all factors at once).  Then the problems iterate, largest first, on concurrent
 * streams of the handle's device (one host worker thread each, 8 by default,
 * MFEAST_BATCH_STREAMS in the environment overrides), solving with the stored factors;
 * cooperative kernels are not used in this mode.  With fpm(50) > 0 every problem factors
 * its own matrices instead.  info[p] is problem p's code; the return value is the most
 * negative code, else the largest positive one, else 0, or -(100+i) for an invalid
 * argument i.  mfeast_get_timing: [0] the factorization of all problems, [5] the call,
 * [6] nprob. */
int mfeast_dsygv_batched(mfeast_handle h, int32_t nprob, const int64_t* n, const double* const* A,
                         const int64_t* lda, const double* const* B, const int64_t* ldb,
                         const int32_t* fpm, const double* emin, const double* emax, int32_t* m0,
                         double* const* E, double* const* X, const int64_t* ldx, int32_t* M,
                         double* const* res, double* epsout, int32_t* loop, int32_t* info);

/* Stochastic estimate of the eigenvalue count (fpm(14)=2; Table tab_fpm, Table tab_info
 * code 5; the method cited in the guide's references, Di Napoli, Polizzi, Saad 2016):
 * the first contour is applied to m0 probe vectors Y with entries +1 or -1 (SplitMix64,
 * seed fpm(51): -1 where the top bit of output i + j*n is set), giving Q; the estimate
 * is Re(trace(Y^H Q)) / m0, which approximates the sum of the quadrature filter over the
 * spectrum, i.e. the number of eigenvalues inside up to the filter's smearing at the
 * interval ends.  On return (info 5): M = the estimate rounded to the nearest integer
 * (at least 0), E[0] (device) = the unrounded estimate, loop = 0, epsout = 1; X, res and
 * E[1..] are not written.  fpm(5) is ignored in this mode.  Every dense, batched and
 * sparse entry point accepts it (the sparse ones with their inexact BiCGSTAB solves).
 * mfeast_init_stochastic sets the guide's defaults for the mode: mfeast_init, then
 * fpm(2)=3 half-contour nodes, fpm(8)=6, fpm(14)=2, fpm(15)=1. */
void mfeast_init_stochastic(int32_t* fpm);

/* IFEAST defaults (Section 3.5, Table tab_fpm "using IFEAST"): mfeast_init, then
 * fpm(2)=4 nodes, fpm(4)=50 loops, fpm(16)=1 trapezoidal rule, fpm(18)=100 (circle).
 * BiCGSTAB accuracy fpm(45)=1 (10^-1) and fpm(46)=40 iterations are the common defaults. */
void mfeast_init_ifeast(int32_t* fpm);

/* Sparse real symmetric problem in CSR storage, solved without factorization
 * (difeast_scsrgv / difeast_scsrev; Section 3.5 "IFEAST"; CSR arguments as in
 * Table tab-spec1 for sparse storage).  Every shifted system z_j B - A is solved
 * inexactly by BiCGSTAB, to ||r|| <= 10^-fpm(45) ||b|| or fpm(46) iterations per
 * column; all quadrature nodes and right-hand sides run as one batch (split into node
 * groups only when device memory is short).  The subspace iteration, Rayleigh-Ritz,
 * residuals, outputs and info codes are those of mfeast_dsygv.
 *  uplo        'F': full storage; 'L' / 'U': only the lower / upper triangle is stored
 *              (entries of the other triangle are ignored)
 *  n           order (n < 2^31 - 1)
 *  a, ia, ja   device: values (double), row pointers (n+1 int32), column indices (int32)
 *              of A; after expansion of a triangle at most 2^31 - 1 entries
 *  index_base  0 or 1: base of ia and ja (the guide's examples are 1-based)
 *  b, ib, jb   device: CSR of B with the same base and uplo, or b = NULL for B = I
 *  other arguments as for mfeast_dsygv (argument positions shift accordingly)
 * fpm(42)=1 (default) runs BiCGSTAB in complex FP32 (values of A and B rounded to FP32);
 * fpm(42)=0 in complex FP64.  The outer products A Q, B Q and the residuals are FP64.
 * On return fpm(60) holds the total number of BiCGSTAB iterations: for every contour
 * and node, the largest iteration count among the node's columns, summed.
 * Errors: -105 (row pointers not monotone, ia(1) != base, or ia(n+1) - base < 0),
 * -106 (column index outside 1..n), -104 (more than 2^31 - 1 stored entries after
 * expansion), -109 / -110 / -108 the same for B; 145 fpm(45) outside 0..16,
 * 146 fpm(46) < 1.  The CSR arrays are checked on the device before any iteration. */
int mfeast_dcsrgv(mfeast_handle h, char uplo, int64_t n, const double* a, const int32_t* ia,
                  const int32_t* ja, int32_t index_base, const double* b, const int32_t* ib,
                  const int32_t* jb, int32_t* fpm, double emin, double emax, int32_t* m0,
                  double* E, double* X, int64_t ldx, int32_t* M, double* res, double* epsout,
                  int32_t* loop, const double* zne, const double* wne);

/* Gradient of a loss on the eigenpairs found in the interval with respect to A, for a real
 * symmetric standard problem (B = I): the backward pass of mfeast_dsygv.  For the M pairs
 * (E_i, x_i) and loss gradients gE_i = dL/dE_i, gX_i = dL/dx_i, with a loss invariant
 * under rotations inside span(X) (e.g. sum E_i + sum_i x_i^T C x_i, C symmetric),
 * first-order perturbation of the eigenproblem (Section 1.1's eigenpairs as functions of
 * A) gives dL/dA = X diag(gE) X^T + (X Y^T + Y X^T)/2, where y_i solves the deflated
 * shifted system (E_i I - A + sigma X X^T) y_i = (I - X X^T) gX_i (sigma = 1 + 2 spread
 * of E).  The M shifted matrices are factored by the batched LU of the contour solves
 * and every solve is refined with FP64 residuals.
 *  A          device, n x n column-major (lda >= n), full storage
 *  M          number of pairs (1 <= M <= n)
 *  E          device, M doubles; X device n x M column-major (ldx >= n), orthonormal
 *  gE         device, M doubles, or NULL (zero); gX device n x M (ldgx >= n) or NULL (zero)
 *  precision  0: real FP64 factorization, one refinement step;
 *             1: real FP32 factorization, up to four FP64 refinement steps
 *  gA         device, n x n column-major (ldga >= n), or NULL
 *  gdiag      device, n doubles: the diagonal of dL/dA (dL/dv for A + diag(v)), or NULL
 * At least one of gA, gdiag.  Returns 0, 202 (n), 201 (M), -(100+i) for argument i,
 * -2 (zero pivot, non-finite value, HIP error), -900. */
int mfeast_dsy_adjoint(mfeast_handle h, int64_t n, const double* A, int64_t lda, int32_t M,
                       const double* E, const double* X, int64_t ldx, const double* gE,
                       const double* gX, int64_t ldgx, int32_t precision, double* gA,
                       int64_t ldga, double* gdiag);

/* Timing of the last call in seconds, host clock around synchronized phases, split as
 * the guide's "FEAST-RCI timing" table (Section 2.4): out[0] Fact. (shift-form and LU of
 * every node), [1] Solve (contour solves with their right-hand-side preparation and the
 * quadrature sum), [2] A*x (the products A Q), [3] B*x (B Y, B Q, and the B^-1 products
 * of the found-pair test; 0 for B = I), [4] Misc. (Gram products, B-orthonormalization,
 * reduced eigensolver, residuals and the host's decisions), [5] total, [6] number of
 * subspace iterations (loop + 1), [7] the reduced eigensolver's part of [4].
 * out: host, 8 doubles.  The batched entry point reports only [5] and [6] (problems). */
int mfeast_get_timing(mfeast_handle h, double* out);

/* Device timing by kernel class of the last call, recorded with HIP events on the
 * handle's streams when fpm(52)=1 was set for that call (project slot, reserved in the
 * guide) or mfeast_set_profiling(h, 1) is in effect (the only switch for
 * mfeast_dsy_adjoint).  For class c: out[4c+0] launches (or launch groups), [4c+1]
 * milliseconds, [4c+2] algorithmic flops (8 per complex multiply-add), [4c+3]
 * algorithmic bytes.  Classes: 0 LU trailing update, 1 LU panel (leaves and their
 * updates), 2 contour solves (per direction), 3 FP64 Rayleigh-Ritz products, 4 reduced
 * eigensolver, 5 other kernels (shift-form, right-hand sides, quadrature sum, small
 * copies), 6 sparse shifted products inside
 * BiCGSTAB, 7 BiCGSTAB vector updates and reductions, 8 B-orthonormalization
 * (equilibration, Cholesky with column drops, Newton-Schulz), 9 LU row interchanges,
 * U12 substitution and the inverses of the diagonal blocks and panels, 10 residual
 * norms and the B^-1 products of the found-pair test, 11 the factorization graph of the
 * batched entry point (every problem and node, one replay; flops of the unpadded
 * matrices).  For the batched entry point the other classes are summed over all
 * problems (their streams run concurrently, so the times may add up to more than the
 * call's wall time).  out: host, `count` doubles (48 cover all classes). */
int mfeast_get_profile(mfeast_handle h, double* out, int32_t count);

/* Per-class timing (see mfeast_get_profile) for every later call on the handle:
 * on = 1 enables, 0 disables (then fpm(52) decides per call).  Returns 0, -101, -102. */
int mfeast_set_profiling(mfeast_handle h, int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* MFEAST_H */
