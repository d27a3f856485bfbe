// Optional per-class kernel timing with HIP events (enabled per call by the caller).
//
// Each instrumented launch records an event pair on the stream it is issued on and
// the algorithmic work it performs (flops counted as 8 per complex multiply-add,
// bytes as the compulsory HBM traffic).  Elapsed times are read after the call has
// synchronized, so the timing does not add host synchronizations.
#pragma once

#include <hip/hip_runtime.h>

namespace mf {

enum KClass {
  K_LU_GEMM = 0,   // trailing update A22 -= L21 U12 of the blocked LU
  K_LU_PANEL = 1,  // panel factorization
  K_SOLVE_GEMM = 2,  // block updates of the contour solves
  K_RR_GEMM = 3,   // FP64 Rayleigh-Ritz products
  K_EIG = 4,       // reduced eigensolver
  K_OTHER = 5,     // shift-form, right-hand sides, quadrature sum, small kernels
  K_SPMV = 6,      // sparse shifted products inside BiCGSTAB
  K_BICG = 7,      // BiCGSTAB vector updates and reductions
  K_ORTH = 8,      // B-orthonormalization: equilibration, Cholesky with drops, Newton-Schulz
  K_LU_ROWS = 9,   // LU row interchanges, U12 substitution, diagonal-block and panel inverses
  K_RESID = 10,    // residual norms and the B^-1 products of the found-pair test
  K_BT_FACT = 11,  // batched problems: the factorization graph of every (problem, node) item
  K_NCLASS = 12
};

bool prof_on();
// cooperative (grid-resident) kernels may be used by this host thread; off while several
// streams of one process run FEAST calls concurrently, where two partly resident grids
// could wait on each other
bool coop_allowed();
void set_coop_allowed(bool on);
void prof_enable(bool on);
// begin/end around one or more launches on stream s
int prof_begin(hipStream_t s);
void prof_end(int token, hipStream_t s, int cls, double flops, double bytes);
// after the stream has synchronized: out[c*4 + {0,1,2,3}] += launches, ms, flops, bytes
void prof_collect(double* out);

}  // namespace mf
