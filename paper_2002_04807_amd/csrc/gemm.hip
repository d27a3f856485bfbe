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
// Products with few output tiles and a long K (the Gram matrices Q^H B Q, n x M0 by
// n x M0) split K over several workgroups per tile: each writes its partial tile to a
// scratch buffer and a second kernel adds the partials in split order (deterministic).
#include <algorithm>
#include <map>
#include <mutex>

#include "kernels.hpp"

#ifndef GEMM_XCD_REMAP
#define GEMM_XCD_REMAP 1
#endif

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

template <typename R> struct vec2;
template <> struct vec2<float> { using t = float2; };
template <> struct vec2<double> { using t = double2; };

// One workgroup computes a BM x BN tile of C with four waves in a 2 x 2 grid (each a
// BM/2 x BN/2 block of 16 x 16 MFMA tiles; 64 x 64 measured best: larger tiles drop
// occupancy to one wave per SIMD).  K advances in slabs of BK: the next
// slab's operands are loaded from global memory into registers while the current slab
// is multiplied out of LDS, so the load latency hides behind the MFMAs.  LDS rows are
// padded to 16 mod 64 words, which puts the four k rows an MFMA operand read touches
// on disjoint banks.
// Workgroups of 4 waves per compute unit the register allocation has to leave room for:
// 3 for complex FP64 (the accumulators move from AGPRs into VGPRs; 12-15% faster on the
// LU and solve shapes than at 2), 5 for FP32 (1-8% faster than at 4).
template <typename R, bool CPLX, bool G3M>
constexpr int gemm_min_blocks() {
  return (sizeof(R) == 8 && CPLX) ? (G3M ? 2 : 3) : (sizeof(R) == 4 ? 5 : 1);
}

template <typename R, bool CPLX, bool A_MCONTIG, bool CONJ_A, bool B_KCONTIG, bool CONJ_B, int BM, int BN, int BK,
          int TAG, bool SPLIT = false, bool G3M = false>
__global__ __launch_bounds__(256, (gemm_min_blocks<R, CPLX, G3M>())) void k_gemm(GemmArgs g, int nsplit, int kchunk, R* __restrict__ part) {
  using M_ = mfma_op<R>;
  using acc_t = typename M_::acc_t;
  using V2 = typename vec2<R>::t;
  constexpr int NT = 256;
  constexpr int PAD = 16;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int ES = CPLX ? 2 : 1;  // reals per element in global memory
  constexpr int NA = BM * BK / NT, NB = BN * BK / NT;
  static_assert(NA * NT == BM * BK && NB * NT == BN * BK, "tile");

  __shared__ R As[ES][BK][BM + PAD];
  __shared__ R Bs[ES][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave & 1) * WM;
  const int wn0 = (wave >> 1) * WN;
  // Workgroups are handed to the 8 XCDs round-robin by linear id, and each XCD has its
  // own L2.  The linear id is remapped so that every XCD works through one contiguous
  // range of tiles (N fastest, then M, then the batch): the tiles resident on an XCD
  // at one time share their A row-tiles and the B panel in that XCD's L2.
  unsigned bxu = blockIdx.x, byu = blockIdx.y, bzu = blockIdx.z;
#if GEMM_XCD_REMAP
  {
    constexpr unsigned NX = 8;
    const unsigned gx = gridDim.x, gy = gridDim.y;
    const unsigned G = gx * gy * gridDim.z;
    const unsigned w = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    const unsigned per = (G + NX - 1) / NX;  // tiles of the larger XCD ranges
    const unsigned tall = G % NX == 0 ? NX : G % NX;
    const unsigned x = w % NX, local = w / NX;
    const unsigned t = x < tall ? x * per + local : tall * per + (x - tall) * (per - 1) + local;
    bxu = t % gx;
    byu = (t / gx) % gy;
    bzu = t / (gx * gy);
  }
#endif
  const int m0 = byu * BM;
  const int n0 = bxu * BN;
  const int64_t bz = SPLIT ? bzu / nsplit : bzu;
  const int sp = SPLIT ? (int)(bzu % nsplit) : 0;
  const R* A = static_cast<const R*>(g.A) + bz * g.a_bs * ES;
  const R* B = static_cast<const R*>(g.B) + bz * g.b_bs * ES;
  R* C = static_cast<R*>(g.C) + bz * g.c_bs * ES;
  const int M = g.M, N = g.N;
  const int kfirst = SPLIT ? sp * kchunk : 0;
  const int K = SPLIT ? min(g.K, kfirst + kchunk) : g.K;

  // complex products: four real passes (P_re += Ar Br - Ai Bi, P_im += Ar Bi + Ai Br), or
  // with G3M the three of Gauss's scheme: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi),
  // re = P1 - P2, im = P3 - P1 - P2
  constexpr int NACC = !CPLX ? 1 : (G3M ? 3 : 2);
  acc_t acc[NACC][FM][FN];
#pragma unroll
  for (int e = 0; e < NACC; ++e)
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[e][i][j][r] = R(0);

  // element q of this thread's share of a slab: (row, k) of op(A), (k, col) of B
  auto a_pos = [&](int q, int& i, int& kk) {
    const int e = tid + NT * q;
    if constexpr (A_MCONTIG) { i = e % BM; kk = e / BM; }
    else { i = e / BK; kk = e % BK; }
  };
  auto b_pos = [&](int q, int& kk, int& j) {
    const int e = tid + NT * q;
    if constexpr (B_KCONTIG) { kk = e % BK; j = e / BK; }
    else { j = e % BN; kk = e / BN; }
  };
  R ra[NA][ES], rb[NB][ES];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int i, kk;
      a_pos(q, i, kk);
      const int gi = m0 + i, gk = k0 + kk;
      ra[q][0] = R(0);
      if constexpr (CPLX) ra[q][1] = R(0);
      if (gi < M && gk < K) {
        const int64_t off = A_MCONTIG ? ((int64_t)gi + (int64_t)gk * g.lda) : ((int64_t)gi * g.lda + gk);
        if constexpr (CPLX) {
          const V2 v = *reinterpret_cast<const V2*>(A + off * 2);
          ra[q][0] = v.x;
          ra[q][1] = CONJ_A ? -v.y : v.y;
        } else {
          ra[q][0] = A[off];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int kk, j;
      b_pos(q, kk, j);
      const int gj = n0 + j, gk = k0 + kk;
      rb[q][0] = R(0);
      if constexpr (CPLX) rb[q][1] = R(0);
      if (gj < N && gk < K) {
        const int64_t off = B_KCONTIG ? ((int64_t)gk + (int64_t)gj * g.ldb) : ((int64_t)gk * g.ldb + gj);
        if constexpr (CPLX) {
          const V2 v = *reinterpret_cast<const V2*>(B + off * 2);
          rb[q][0] = v.x;
          rb[q][1] = CONJ_B ? -v.y : v.y;
        } else {
          rb[q][0] = B[off];
        }
      }
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int i, kk;
      a_pos(q, i, kk);
#pragma unroll
      for (int e = 0; e < ES; ++e) As[e][kk][i] = ra[q][e];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int kk, j;
      b_pos(q, kk, j);
#pragma unroll
      for (int e = 0; e < ES; ++e) Bs[e][kk][j] = rb[q][e];
    }
  };

  if (kfirst < K) load(kfirst);
  for (int k0 = kfirst; k0 < K; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < K) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      const int cl = lane & 15;
      R ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kr][wm0 + i * 16 + cl];
        if constexpr (CPLX) ai[i] = As[ES - 1][kr][wm0 + i * 16 + cl];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kr][wn0 + j * 16 + cl];
        if constexpr (CPLX) bi[j] = Bs[ES - 1][kr][wn0 + j * 16 + cl];
      }
      // one pass per real product, so consecutive MFMAs write different accumulators
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[0][i][j] = M_::run(ar[i], br[j], acc[0][i][j]);
      if constexpr (CPLX && G3M) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[1][i][j] = M_::run(ai[i], bi[j], acc[1][i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i) ai[i] = ar[i] + ai[i];
#pragma unroll
        for (int j = 0; j < FN; ++j) bi[j] = br[j] + bi[j];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[2][i][j] = M_::run(ai[i], bi[j], acc[2][i][j]);
      } else if constexpr (CPLX) {
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[1][i][j] = M_::run(ar[i], bi[j], acc[1][i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[1][i][j] = M_::run(ai[i], br[j], acc[1][i][j]);
#pragma unroll
        for (int i = 0; i < FM; ++i) ai[i] = -ai[i];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) acc[0][i][j] = M_::run(ai[i], bi[j], acc[0][i][j]);
      }
    }
  }

  // real and imaginary parts of the product tile
  auto re_of = [&](int i, int j, int r) -> R {
    if constexpr (CPLX && G3M) return acc[0][i][j][r] - acc[1][i][j][r];
    else return acc[0][i][j][r];
  };
  auto im_of = [&](int i, int j, int r) -> R {
    if constexpr (CPLX && G3M) return acc[2][i][j][r] - acc[0][i][j][r] - acc[1][i][j][r];
    else return acc[NACC - 1][i][j][r];
  };

  if constexpr (SPLIT) {
    // partial tile of split sp: part[(bz * nsplit + sp)][M][N] (interleaved complex)
    R* P = part + (bz * nsplit + sp) * (int64_t)M * N * ES;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = m0 + wm0 + i * 16 + M_::row(lane, r);
          const int gj = n0 + wn0 + j * 16 + (lane & 15);
          if (gi < M && gj < N) {
            const int64_t off = ((int64_t)gi * N + gj) * ES;
            P[off] = re_of(i, j, r);
            if constexpr (CPLX) P[off + 1] = im_of(i, j, r);
          }
        }
    return;
  }
  // ---- epilogue: C = alpha * acc + beta * C
  const R alpha = (R)g.alpha, beta = (R)g.beta;
  const bool use_c = g.beta != 0.0;
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
          R vr = alpha * re_of(i, j, r);
          if constexpr (CPLX) {
            R vi = alpha * im_of(i, j, r);
            if (use_c) {
              const V2 c = *reinterpret_cast<const V2*>(C + off);
              vr += beta * c.x;
              vi += beta * c.y;
            }
            V2 o;
            o.x = vr;
            o.y = vi;
            *reinterpret_cast<V2*>(C + off) = o;
          } else {
            if (use_c) vr += beta * C[off];
            C[off] = vr;
          }
        }
      }
}

// C = alpha * sum of the partial tiles (in split order) + beta * C
template <typename R, bool CPLX>
__global__ void k_gemm_splitk_sum(GemmArgs g, int nsplit, const R* __restrict__ part) {
  constexpr int ES = CPLX ? 2 : 1;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t bz = blockIdx.y;
  if (e >= mn) return;
  const int gi = (int)(e / g.N), gj = (int)(e % g.N);
  R sr = R(0), si = R(0);
  for (int sp = 0; sp < nsplit; ++sp) {
    const R* P = part + (bz * nsplit + sp) * mn * ES;
    sr += P[e * ES];
    if constexpr (CPLX) si += P[e * ES + 1];
  }
  R* C = static_cast<R*>(g.C) + bz * g.c_bs * ES;
  const int64_t off = ((int64_t)gi * g.ldc + gj) * ES;
  R vr = (R)g.alpha * sr, vi = (R)g.alpha * si;
  if (g.beta != 0.0) {
    vr += (R)g.beta * C[off];
    if constexpr (CPLX) vi += (R)g.beta * C[off + 1];
  }
  C[off] = vr;
  if constexpr (CPLX) C[off + 1] = vi;
}

// scratch for split-K partials, supplied by the handle the calling thread works for
// (bound by the entry points; without one the products run without splitting K)
namespace {
thread_local ScratchFn g_scratch_fn = nullptr;
thread_local void* g_scratch_owner = nullptr;
}  // namespace

void set_gemm_scratch(ScratchFn fn, void* owner) {
  g_scratch_fn = fn;
  g_scratch_owner = owner;
}

static void* splitk_scratch(size_t bytes) {
  return g_scratch_fn != nullptr ? g_scratch_fn(g_scratch_owner, bytes) : nullptr;
}

template <typename R, bool CPLX, bool AM, bool CJ, bool BK_, bool CJB, int BM, int BN, int BK, bool G3M>
static void launch_tile(const GemmArgs& g, int batch, hipStream_t s) {
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, batch);
  if constexpr (CPLX && !AM && !CJ && !BK_ && !CJB) {
    if (g.tag == 1) {
      hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 1, false, G3M>), grid, dim3(256), 0, s, g, 1, 0,
                         (R*)nullptr);
      return;
    }
    if (g.tag == 2) {
      hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 2, false, G3M>), grid, dim3(256), 0, s, g, 1, 0,
                         (R*)nullptr);
      return;
    }
  }
  hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 0, false, G3M>), grid, dim3(256), 0, s, g, 1, 0,
                     (R*)nullptr);
}

// Gauss's three-product complex scheme for FP32 products (measured 10-25% faster there;
// with FP64 the third accumulator set lowers occupancy and it is slower)
static thread_local bool g_3m = true;
void set_gemm_3m(bool on) { g_3m = on; }
bool gemm_3m() { return g_3m; }

// ---------------------------------------------------------------------------
// tile autotuner (see kernels.hpp)
namespace {
std::mutex g_tune_mu;
std::map<uint64_t, int> g_tune;  // size class -> tile index
thread_local bool g_tune_on = false;

int bucket(int64_t v) {
  int b = 0;
  while (b < 31 && (int64_t(1) << b) < v) ++b;
  return b;
}

uint64_t tune_key(int rbytes, bool cplx, bool g3m, const GemmArgs& g, int batch) {
  return (uint64_t)rbytes | ((uint64_t)cplx << 4) | ((uint64_t)g3m << 5) | ((uint64_t)bucket(g.M) << 8) |
         ((uint64_t)bucket(g.N) << 16) | ((uint64_t)bucket(g.K) << 24) | ((uint64_t)bucket(batch) << 32);
}
}  // namespace

void set_gemm_tuning(bool on) { g_tune_on = on; }
int gemm_tuned_classes() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  return (int)g_tune.size();
}

template <typename R, bool CPLX, bool AM, bool CJ, bool BK_, bool CJB, int TBK, bool G3M>
static void launch_tile_choice(int tile, const GemmArgs& g, int batch, hipStream_t s) {
  switch (tile) {
    case 1: launch_tile<R, CPLX, AM, CJ, BK_, CJB, 32, 64, TBK, G3M>(g, batch, s); return;
    case 2: launch_tile<R, CPLX, AM, CJ, BK_, CJB, 64, 32, TBK, G3M>(g, batch, s); return;
    case 3: launch_tile<R, CPLX, AM, CJ, BK_, CJB, 32, 32, TBK, G3M>(g, batch, s); return;
    default: launch_tile<R, CPLX, AM, CJ, BK_, CJB, 64, 64, TBK, G3M>(g, batch, s); return;
  }
}

// tile for an LU trailing update: the cached choice of its class; on a miss with tuning on,
// each candidate runs twice on a scratch output (at most 8 batch entries) and the second
// run is timed
template <typename R, bool CPLX, bool TBK_, int TBK, bool G3M>
static int tuned_tile(const GemmArgs& g, int batch, hipStream_t s) {
  const uint64_t key = tune_key((int)sizeof(R), CPLX, G3M, g, batch);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) return it->second;
  }
  if (!g_tune_on) return 0;
  constexpr int ES = CPLX ? 2 : 1;
  const int bt = std::min(batch, 8);
  R* out = static_cast<R*>(splitk_scratch((size_t)bt * g.M * g.N * ES * sizeof(R)));
  if (out == nullptr) return 0;
  GemmArgs t = g;
  t.C = out;
  t.ldc = g.N;
  t.c_bs = (int64_t)g.M * g.N;
  t.beta = 0.0;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return 0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return 0;
  }
  int best = 0;
  float best_ms = 0.0f;
  for (int tile = 0; tile < 4; ++tile) {
    launch_tile_choice<R, CPLX, false, false, false, false, TBK, G3M>(tile, t, bt, s);
    (void)hipEventRecord(e0, s);
    launch_tile_choice<R, CPLX, false, false, false, false, TBK, G3M>(tile, t, bt, s);
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (tile == 0 || ms < best_ms) {
      best = tile;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = best;
  return best;
}

template <typename R, bool CPLX, bool AM, bool CJ, bool BK_, bool CJB>
static void launch(const GemmArgs& g, int batch, hipStream_t s) {
  constexpr int BK = 16;
  const int tiles = ((g.N + 63) / 64) * ((g.M + 63) / 64) * batch;
  // Few output tiles and a long K: split K so that about 512 workgroups run.  FP64
  // tile counts between 128 and 768 (the 4096 x 600 products of the Rayleigh-Ritz
  // step: 640 tiles) leave a second, mostly idle round of the 512 resident
  // workgroups; two K halves (measured 17-24% faster there) even it out.
  int nsplit = 0;
  if (tiles < 128 && g.K >= 1024) nsplit = std::min(std::min(std::max(2, 512 / tiles), g.K / 256), 64);
  else if (sizeof(R) == 8 && tiles < 768 && g.K >= 512) nsplit = 2;
  if (nsplit > 1) {
    constexpr int BM = 64, BN = 64;
    const int kchunk = ((g.K + nsplit - 1) / nsplit + BK - 1) / BK * BK;
    nsplit = (g.K + kchunk - 1) / kchunk;
    constexpr int ES = CPLX ? 2 : 1;
    R* part = static_cast<R*>(splitk_scratch((size_t)nsplit * batch * g.M * g.N * ES * sizeof(R)));
    if (part != nullptr && nsplit > 1) {
      dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, batch * nsplit);
      constexpr bool F64C = CPLX && sizeof(R) == 8;  // complex FP64: three products unless fpm(53) = 1
      if (F64C && g_3m)
        hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 0, true, F64C>), grid, dim3(256), 0, s, g,
                           nsplit, kchunk, part);
      else
        hipLaunchKernelGGL((k_gemm<R, CPLX, AM, CJ, BK_, CJB, BM, BN, BK, 0, true>), grid, dim3(256), 0, s, g, nsplit,
                           kchunk, part);
      const int64_t mn = (int64_t)g.M * g.N;
      hipLaunchKernelGGL((k_gemm_splitk_sum<R, CPLX>), dim3((unsigned)((mn + 255) / 256), batch), dim3(256), 0, s, g,
                         nsplit, (const R*)part);
      return;
    }
  }
  // 8-deep K slabs for FP32 (measured 3-7% faster there), 16-deep for FP64
  constexpr int TBK = sizeof(R) == 4 ? 8 : 16;
  // LU trailing updates: the autotuned tile of their size class
  if constexpr (CPLX && !AM && !CJ && !BK_ && !CJB) {
    if (g.tag == 1) {
      if constexpr (sizeof(R) == 4) {
        if (g_3m) {
          const int tile = tuned_tile<R, CPLX, false, TBK, true>(g, batch, s);
          launch_tile_choice<R, CPLX, AM, CJ, BK_, CJB, TBK, true>(tile, g, batch, s);
          return;
        }
      }
      const int tile = tuned_tile<R, CPLX, false, TBK, false>(g, batch, s);
      launch_tile_choice<R, CPLX, AM, CJ, BK_, CJB, TBK, false>(tile, g, batch, s);
      return;
    }
  }
  // Fewer than two 64 x 64 tiles per compute unit (the 256-row panel-inverse products of the
  // block solves: 320 for 8 nodes and 600 columns, 28 for one matrix; the M0 x M0 products of
  // the Rayleigh-Ritz step: 100): 32 x 32 tiles, four times as many workgroups.  The tile
  // does not change the order of any K sum.
  const bool few = tiles < 512;
  if constexpr (CPLX) {
    if (g_3m) {
      if (few) launch_tile<R, CPLX, AM, CJ, BK_, CJB, 32, 32, TBK, true>(g, batch, s);
      else launch_tile<R, CPLX, AM, CJ, BK_, CJB, 64, 64, TBK, true>(g, batch, s);
      return;
    }
  }
  if (few) launch_tile<R, CPLX, AM, CJ, BK_, CJB, 32, 32, TBK, false>(g, batch, s);
  else launch_tile<R, CPLX, AM, CJ, BK_, CJB, 64, 64, TBK, false>(g, batch, s);
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
template int gemm_op<float, false>(hipStream_t, GemmOp, GemmOp, const GemmArgs&, int);
template int gemm<float, false>(hipStream_t, bool, bool, const GemmArgs&, int);

}  // namespace mf
