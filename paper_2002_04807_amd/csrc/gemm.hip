// Batched MFMA GEMM for the contour solves and the Rayleigh-Ritz products (gfx950).
//
//   C[b] = alpha * op(A[b]) * B[b] + beta * C[b]      (b = blockIdx.z)
//
// op(A) is M x K and is read either K-contiguous (row-major, element (i,k) at
// A[i*lda + k]) or M-contiguous (column-major / a transposed view, element (i,k)
// at A[i + k*lda]), optionally conjugated.  op(B) (K x N) is read N-contiguous
// (element (k,j) at B[k*ldb + j]) or K-contiguous (B[k + j*ldb]), optionally
// conjugated.  C (M x N) is row-major.
// Complex operands are interleaved (re, im) in memory and planar in LDS; a
// complex product is four real MFMAs (re*re - im*im, re*im + im*re), so the
// flop count is 8 per complex multiply-add as in the algorithmic count.
// FP32 tiles use v_mfma_f32_16x16x4f32, FP64 tiles v_mfma_f64_16x16x4f64; the
// output lane layouts of the two differ and were checked on the device.
#include "kernels.hpp"

namespace mf {

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef double d4_t __attribute__((ext_vector_type(4)));

template <typename R> struct mfma_op;
template <> struct mfma_op<float> {
  using acc_t = f4_t;
  __device__ static inline acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator register r of lane l holds C[row][l % 16]
  __device__ static inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct mfma_op<double> {
  using acc_t = d4_t;
  __device__ static inline acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <typename R, bool CPLX, bool A_MCONTIG, bool CONJ_A, bool B_KCONTIG, bool CONJ_B, int BM, int BN, int BK,
          int TAG>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  using M_ = mfma_op<R>;
  using acc_t = typename M_::acc_t;
  constexpr int NT = 256;
  constexpr int PAD = (sizeof(R) == 4) ? 4 : 2;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int ES = CPLX ? 2 : 1;  // reals per element in global memory

  __shared__ R As[ES][BK][BM + PAD];
  __shared__ R Bs[ES][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave & 1) * WM;
  const int wn0 = (wave >> 1) * WN;
  const int m0 = blockIdx.y * BM;
  const int n0 = blockIdx.x * BN;
  const int64_t bz = blockIdx.z;
  const R* A = static_cast<const R*>(g.A) + bz * g.a_bs * ES;
  const R* B = static_cast<const R*>(g.B) + bz * g.b_bs * ES;
  R* C = static_cast<R*>(g.C) + bz * g.c_bs * ES;
  const int M = g.M, N = g.N, K = g.K;

  acc_t acc[ES][FM][FN];
#pragma unroll
  for (int e = 0; e < ES; ++e)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
        for (int r = 0; r < 4; ++r) acc[e][i][j][r] = R(0);

  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    // ---- A tile -> LDS [k][m]
    if constexpr (A_MCONTIG) {
      constexpr int KS = NT / BM;
#pragma unroll
      for (int kk = tid / BM; kk < BK; kk += KS) {
        const int i = tid % BM;
        const int gi = m0 + i, gk = k0 + kk;
        R re = R(0), im = R(0);
        if (gi < M && gk < K) {
          const int64_t off = ((int64_t)gi + (int64_t)gk * g.lda) * ES;
          re = A[off];
          if constexpr (CPLX) im = A[off + 1];
        }
        As[0][kk][i] = re;
        if constexpr (CPLX) As[1][kk][i] = CONJ_A ? -im : im;
      }
    } else {
      constexpr int IS = NT / BK;
#pragma unroll
      for (int i = tid / BK; i < BM; i += IS) {
        const int kk = tid % BK;
        const int gi = m0 + i, gk = k0 + kk;
        R re = R(0), im = R(0);
        if (gi < M && gk < K) {
          const int64_t off = ((int64_t)gi * g.lda + gk) * ES;
          re = A[off];
          if constexpr (CPLX) im = A[off + 1];
        }
        As[0][kk][i] = re;
        if constexpr (CPLX) As[1][kk][i] = CONJ_A ? -im : im;
      }
    }
    // ---- B tile -> LDS [k][n]
    if constexpr (!B_KCONTIG) {
      constexpr int KS = NT / BN;
#pragma unroll
      for (int kk = tid / BN; kk < BK; kk += KS) {
        const int j = tid % BN;
        const int gj = n0 + j, gk = k0 + kk;
        R re = R(0), im = R(0);
        if (gj < N && gk < K) {
          const int64_t off = ((int64_t)gk * g.ldb + gj) * ES;
          re = B[off];
          if constexpr (CPLX) im = B[off + 1];
        }
        Bs[0][kk][j] = re;
        if constexpr (CPLX) Bs[1][kk][j] = CONJ_B ? -im : im;
      }
    } else {
      constexpr int JS = NT / BK;
#pragma unroll
      for (int j = tid / BK; j < BN; j += JS) {
        const int kk = tid % BK;
        const int gj = n0 + j, gk = k0 + kk;
        R re = R(0), im = R(0);
        if (gj < N && gk < K) {
          const int64_t off = ((int64_t)gk + (int64_t)gj * g.ldb) * ES;
          re = B[off];
          if constexpr (CPLX) im = B[off + 1];
        }
        Bs[0][kk][j] = re;
        if constexpr (CPLX) Bs[1][kk][j] = CONJ_B ? -im : im;
      }
    }
    __syncthreads();
    // ---- MFMA over the BK slab, 4 at a time
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int cl = lane & 15;
      R ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kr][wm0 + i * 16 + cl];
        if constexpr (CPLX) ai[i] = As[1][kr][wm0 + i * 16 + cl];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kr][wn0 + j * 16 + cl];
        if constexpr (CPLX) bi[j] = Bs[1][kr][wn0 + j * 16 + cl];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc[0][i][j] = M_::run(ar[i], br[j], acc[0][i][j]);
          if constexpr (CPLX) {
            acc[0][i][j] = M_::run(-ai[i], bi[j], acc[0][i][j]);
            acc[1][i][j] = M_::run(ar[i], bi[j], acc[1][i][j]);
            acc[1][i][j] = M_::run(ai[i], br[j], acc[1][i][j]);
          }
        }
    }
  }

  // ---- epilogue: C = alpha * acc + beta * C
  const R alpha = (R)g.alpha, beta = (R)g.beta;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gi = m0 + wm0 + i * 16 + M_::row(lane, r);
        const int gj = n0 + wn0 + j * 16 + (lane & 15);
        if (gi < M && gj < N) {
          const int64_t off = ((int64_t)gi * g.ldc + gj) * ES;
          R vr = alpha * acc[0][i][j][r];
          R vi = CPLX ? alpha * acc[ES - 1][i][j][r] : R(0);
          if (g.beta != 0.0) {
            vr += beta * C[off];
            if constexpr (CPLX) vi += beta * C[off + 1];
          }
          C[off] = vr;
          if constexpr (CPLX) C[off + 1] = vi;
        }
      }
}

template <typename R, bool CPLX, bool AM, bool CJ, bool BK_, bool CJB>
static void launch(const GemmArgs& g, int batch, hipStream_t s) {
  constexpr int BM = 64, BN = 64, BK = 16;
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, batch);
  if constexpr (CPLX && !AM && !CJ && !BK_ && !CJB) {
    if (g.tag == 1) {
      hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 1>), grid, dim3(256), 0, s, g);
      return;
    }
    if (g.tag == 2) {
      hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 2>), grid, dim3(256), 0, s, g);
      return;
    }
  }
  hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 0>), grid, dim3(256), 0, s, g);
}

template <typename R, bool CPLX, bool AM, bool CJ>
static void launch_b(GemmOp opb, const GemmArgs& g, int batch, hipStream_t s) {
  if (opb == OP_N) launch<R, CPLX, AM, CJ, false, false>(g, batch, s);
  else if (opb == OP_T || !CPLX) launch<R, CPLX, AM, CJ, true, false>(g, batch, s);
  else launch<R, CPLX, AM, CJ, true, CPLX>(g, batch, s);
}

template <typename R, bool CPLX>
int gemm_op(hipStream_t s, GemmOp opa, GemmOp opb, const GemmArgs& g, int batch) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return 0;
  if (opa == OP_N) launch_b<R, CPLX, false, false>(opb, g, batch, s);
  else if (opa == OP_T || !CPLX) launch_b<R, CPLX, true, false>(opb, g, batch, s);
  else launch_b<R, CPLX, true, CPLX>(opb, g, batch, s);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename R, bool CPLX>
int gemm(hipStream_t s, bool a_mcontig, bool conj_a, const GemmArgs& g, int batch) {
  const GemmOp opa = !a_mcontig ? OP_N : (conj_a ? OP_C : OP_T);
  return gemm_op<R, CPLX>(s, opa, OP_N, g, batch);
}

template int gemm_op<float, true>(hipStream_t, GemmOp, GemmOp, const GemmArgs&, int);
template int gemm_op<double, true>(hipStream_t, GemmOp, GemmOp, const GemmArgs&, int);
template int gemm_op<double, false>(hipStream_t, GemmOp, GemmOp, const GemmArgs&, int);
template int gemm<float, true>(hipStream_t, bool, bool, const GemmArgs&, int);
template int gemm<double, true>(hipStream_t, bool, bool, const GemmArgs&, int);
template int gemm<double, false>(hipStream_t, bool, bool, const GemmArgs&, int);

}  // namespace mf
