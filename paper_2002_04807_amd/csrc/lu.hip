// Shifted matrices and their blocked LU factorization with partial pivoting (gfx950).
//
// One factorization per quadrature node z_j of Az_j = z_j B - A (FEAST Hermitian RCI
// case 10; the factorizations are kept for every later solve, fpm(10)=1).  All nodes
// are factored together: every launch covers the ne independent matrices.
//
// Right-looking blocked LU, panel width LU_NB:
//   panel     recursive, in leaves of IB columns: one 1024-thread workgroup per node
//             factors the (n-k) x IB leaf in registers (k_leaf): the pivot of each
//             column is the row of largest |re|+|im| (lowest index on ties), found
//             with a wavefront shuffle reduction and an LDS reduction across the 16
//             wavefronts; rows are exchanged through LDS, the column is scaled and the
//             leaf updated in registers.  The same launch applies the leaf's
//             interchanges to the other panel columns and forms its rows of U; the
//             panel columns right of the leaf are then updated by many workgroups
//             (k_leaf_update).
//   laswp     the panel's interchanges applied to all columns outside the panel
//             (rows are contiguous because the matrices are row-major).
//   U12       U12 = L11^-1 A12 by forward substitution in LDS and registers.
//   invert    after the last block, the unit-lower and the upper LU_NB x LU_NB
//             diagonal blocks of every block row are inverted (one launch) and
//             stored beside the factors for the contour solves.
//   trailing  A22 -= L21 U12 (MFMA complex GEMM, the dense contraction of the LU).
#include <climits>

#include "kernels.hpp"

namespace mf {

// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_expand_full(int64_t n, char uplo, const T* __restrict__ src, int64_t lds, T* __restrict__ dst) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;  // row
  const int64_t j = blockIdx.y;                                       // column
  if (i >= n) return;
  // column-major: element (i, j) at src[i + j*lds]
  T v;
  const bool lower = (uplo == 'L' || uplo == 'l');
  if (i == j) {
    v = T(real_part(src[i + j * lds]));
  } else if ((i > j) == lower) {
    v = src[i + j * lds];
  } else {
    v = conj(src[j + i * lds]);
  }
  dst[i + j * n] = v;
}

template <typename T>
int expand_full(hipStream_t s, char uplo, int64_t n, const T* src, int64_t lds, T* dst) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_expand_full<T>), grid, dim3(256), 0, s, n, uplo, src, lds, dst);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
template <typename T, typename C>
__global__ void k_shift_form(int64_t n, int64_t ld, const T* __restrict__ A, int64_t lda, const T* __restrict__ B,
                             int64_t ldb, const c64* __restrict__ z, int ne, int bnode, C* __restrict__ LU,
                             int* __restrict__ perm) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (c >= n) return;
  // For a Hermitian matrix stored column-major, buf[i*ld + c] is element (c, i), the
  // conjugate of element (i, c): reading it keeps the row-major writes coalesced.
  const c64 a = convert<c64, T>(conj(A[i * lda + c]));
  c64 b;
  if (B != nullptr) b = convert<c64, T>(conj(B[i * ldb + c]));
  else b = c64(i == c ? 1.0 : 0.0, 0.0);
  for (int j = 0; j < ne; ++j) {
    const c64 v = z[j] * b - a;
    LU[(int64_t)j * n * ld + i * ld + c] = convert<C, c64>(v);
  }
  if (bnode) LU[(int64_t)ne * n * ld + i * ld + c] = convert<C, c64>(b);
  if (i == 0)
    for (int j = 0; j < ne + bnode; ++j) perm[(int64_t)j * n + c] = (int)c;
}

template <typename T, typename C>
int shift_form(hipStream_t s, int64_t n, const T* A, int64_t lda, const T* B, int64_t ldb,
               const c64* z_dev, int ne, C* LU, int* perm, bool b_node) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL((k_shift_form<T, C>), grid, dim3(256), 0, s, n, lu_ld(n), A, lda, B, ldb, z_dev, ne,
                     b_node ? 1 : 0, LU, perm);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ---------------------------------------------------------------------------
constexpr int MAX_N = 16384;

// ---------------------------------------------------------------------------
// Recursive panel: the LU_NB-wide panel is factored in leaves of IB columns.  For each
// leaf, one 1024-thread workgroup per node factors the (n - row0) x IB leaf with
// partial pivoting in registers (k_leaf); the same launch applies the leaf's
// interchanges to the other panel columns and forms the leaf's rows of U for the
// panel columns to its right.  k_leaf_update then subtracts L_leaf U_leaf from the
// panel columns to the right over many workgroups.  No grid-wide synchronization.
constexpr int LEAF_THREADS = 1024;

// Wavefront-wide max / min of a 32-bit unsigned value with DPP: two quad
// permutations and two rotations inside each row of 16 lanes, then the row-15 and
// row-31 broadcasts; lane 63 ends with the result, which every lane then reads.
template <bool MAX>
__device__ inline unsigned wave_reduce_u32(unsigned x) {
  auto op = [](unsigned a, unsigned b) { return MAX ? max(a, b) : min(a, b); };
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0xB1, 0xF, 0xF, false));   // quad_perm 1,0,3,2
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x4E, 0xF, 0xF, false));   // quad_perm 2,3,0,1
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x124, 0xF, 0xF, false));  // row_ror 4
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x128, 0xF, 0xF, false));  // row_ror 8
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x142, 0xA, 0xF, false));  // row_bcast 15
  x = op(x, (unsigned)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x143, 0xC, 0xF, false));  // row_bcast 31
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}

// Pivot keys: an eligible magnitude a >= 0 maps to its bit pattern plus one (which
// orders like a), an ineligible row or a NaN to 0.  The key is 32 bits for float and
// 64 bits for double magnitudes.
template <typename R> struct pivot_key;
template <> struct pivot_key<float> {
  using K = unsigned;
  __device__ static K of(float a, bool ok) { return (ok && a >= 0.0f) ? __float_as_uint(a) + 1u : 0u; }
  __device__ static K wave_max(K x) { return wave_reduce_u32<true>(x); }
};
template <> struct pivot_key<double> {
  using K = unsigned long long;
  __device__ static K of(double a, bool ok) {
    return (ok && a >= 0.0) ? (K)__double_as_longlong(a) + 1ull : 0ull;
  }
  __device__ static K wave_max(K x) {
    const unsigned hi = wave_reduce_u32<true>((unsigned)(x >> 32));
    const unsigned lo = wave_reduce_u32<true>((unsigned)(x >> 32) == hi ? (unsigned)x : 0u);
    return ((K)hi << 32) | lo;
  }
};

// a row segment of N consecutive elements as 16-byte loads and stores (16-byte aligned
// when its size is a multiple of 16 bytes; element by element otherwise)
template <typename C, int N>
__device__ inline void load_row(const C* p, C (&out)[N]) {
  if constexpr ((N * sizeof(C)) % 16 == 0) {
    union { uint4 q[N * sizeof(C) / 16]; C e[N]; } u;
#pragma unroll
    for (int i = 0; i < (int)(N * sizeof(C) / 16); ++i) u.q[i] = reinterpret_cast<const uint4*>(p)[i];
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = u.e[i];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = p[i];
  }
}
template <typename C, int N>
__device__ inline void store_row(C* p, const C (&in)[N]) {
  if constexpr ((N * sizeof(C)) % 16 == 0) {
    union { uint4 q[N * sizeof(C) / 16]; C e[N]; } u;
#pragma unroll
    for (int i = 0; i < N; ++i) u.e[i] = in[i];
#pragma unroll
    for (int i = 0; i < (int)(N * sizeof(C) / 16); ++i) reinterpret_cast<uint4*>(p)[i] = u.q[i];
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) p[i] = in[i];
  }
}

template <typename C, int IB, int RMAX, int NT = LEAF_THREADS>
__global__ __launch_bounds__(NT) void k_leaf(int64_t n, int64_t ld, int k, int jb, int nbc, C* __restrict__ LUall,
                                                         int* __restrict__ ipiv_all, int* __restrict__ perm_all,
                                                         int* __restrict__ info_all) {
  using R = typename real_of<C>::type;
  const int node = blockIdx.x;
  C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int ibc = min(IB, nbc - jb);
  const int64_t row0 = k + jb;
  const int mr = (int)(n - row0);

  __shared__ int s_ipiv[IB];
  __shared__ C prow[IB], crow[IB];
  __shared__ C Lsub[IB][IB];
  using PK = pivot_key<R>;
  __shared__ typename PK::K red_k[NT / 64];
  __shared__ unsigned red_i[NT / 64];
  __shared__ int s_zero;
  // rows touched by the interchanges: the leaf's top rows and the pivot rows
  __shared__ int s_rows[2 * IB];
  __shared__ int s_nrows;
  __shared__ int s_swa[IB], s_swb[IB];  // per interchange: indices into s_rows
  __shared__ C oval[2 * IB][LU_NB];      // touched rows of the other panel columns
  __shared__ int opv[2 * IB];            // and of perm

  if (tid == 0) s_zero = 0;
  // rows of the leaf are 16-byte aligned (ld and row0 are multiples of IB); a narrower
  // last leaf reads its padding columns and zeroes them
  C v[RMAX][IB];
#pragma unroll
  for (int t = 0; t < RMAX; ++t) {
    const int r = tid + t * NT;
    if (r < mr) load_row<C, IB>(LU + (row0 + r) * ld + row0, v[t]);
#pragma unroll
    for (int c = 0; c < IB; ++c)
      if (!(r < mr && c < ibc)) v[t][c] = C(0);
  }
  __syncthreads();

  // the column loop is unrolled so that every register index below is a constant
#pragma unroll
  for (int j = 0; j < IB; ++j) {
    if (j >= ibc) break;
    // ---- pivot: largest |re|+|im| among local rows r >= j of column j, lowest index on ties
    typename PK::K best = 0;
    unsigned bi = 0xFFFFFFFFu;
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
      const int r = tid + t * NT;
      const typename PK::K key = PK::of(abs1(v[t][j]), r >= j && r < mr);
      if (key > best) {
        best = key;
        bi = (unsigned)r;
      }
    }
    const typename PK::K wbest = PK::wave_max(best);
    const unsigned wbi = wave_reduce_u32<false>(best == wbest ? bi : 0xFFFFFFFFu);
    if (lane == 0) {
      red_k[wave] = wbest;
      red_i[wave] = wbi;
    }
    __syncthreads();
    // every thread merges the per-wavefront candidates itself (no broadcast round)
    typename PK::K bk = red_k[0];
    unsigned bu = red_i[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) {
      const typename PK::K ok = red_k[w];
      const unsigned oi = red_i[w];
      if (ok > bk || (ok == bk && oi < bu)) {
        bk = ok;
        bu = oi;
      }
    }
    int bx = (int)bu;
    // a zero (or non-finite) column: keep the diagonal row, flag the breakdown
    if (bk <= 1) {
      if (tid == 0 && s_zero == 0) s_zero = (int)(row0 + j) + 1;
      bx = j;
    }
    const int p = bx;
    if (tid == 0) s_ipiv[j] = p;
    // ---- exchange local rows j and p through LDS
    if (tid == (p & (NT - 1))) {
#pragma unroll
      for (int t = 0; t < RMAX; ++t)
        if (t == (p / NT))
#pragma unroll
          for (int c = 0; c < IB; ++c) prow[c] = v[t][c];
    }
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < IB; ++c) crow[c] = v[0][c];
    }
    __syncthreads();
    if (tid == j) {
#pragma unroll
      for (int c = 0; c < IB; ++c) v[0][c] = prow[c];
    }
    if (p != j && tid == (p & (NT - 1))) {
#pragma unroll
      for (int t = 0; t < RMAX; ++t)
        if (t == (p / NT))
#pragma unroll
          for (int c = 0; c < IB; ++c) v[t][c] = crow[c];
    }
    // ---- scale column j below the diagonal and update the leaf.  No barrier follows:
    //      red_k / red_i were last read before the barrier above, and prow / crow are
    //      rewritten only after the next column's first barrier.
    C piv = C(0);
#pragma unroll
    for (int c = 0; c < IB; ++c)
      if (c == j) piv = prow[c];
    const bool ok = abs1(piv) > R(0);
    const C inv = ok ? cdiv(C(1), piv) : C(0);
#pragma unroll
    for (int t = 0; t < RMAX; ++t) {
      const int r = tid + t * NT;
      if (r > j && r < mr && ok) {
        C l = C(0);
#pragma unroll
        for (int c = 0; c < IB; ++c)
          if (c == j) l = v[t][c] * inv;
#pragma unroll
        for (int c = 0; c < IB; ++c) {
          if (c == j) v[t][c] = l;
          else if (c > j) v[t][c] = v[t][c] - l * prow[c];
        }
      }
    }
  }
  __syncthreads();

  // ---- the factored leaf back to memory; its unit-lower top block to LDS
  // (columns past ibc are padding of the last block and receive zeros)
#pragma unroll
  for (int t = 0; t < RMAX; ++t) {
    const int r = tid + t * NT;
    if (r < mr) store_row<C, IB>(LU + (row0 + r) * ld + row0, v[t]);
  }
  if (tid < ibc) {
#pragma unroll
    for (int c = 0; c < IB; ++c) Lsub[tid][c] = v[0][c];
  }
  // ---- list of the rows the interchanges touch (local indices) in order of first
  //      appearance in the sequence j, ipiv[j], j+1, ipiv[j+1], ...; and the swap
  //      sequence as slots of that list.  One wavefront: lane e holds the e-th row of the
  //      sequence, finds its first occurrence, and counts the distinct rows before it.
  if (tid < 64) {
    const int e = tid;
    const bool live = e < 2 * ibc;
    const int r = !live ? -1 : ((e & 1) ? s_ipiv[e >> 1] : (e >> 1));
    int first = e;  // lowest lane holding the same row
#pragma unroll
    for (int f = 0; f < 2 * IB; ++f) {
      const int rf = __shfl(r, f);
      if (f < first && rf == r) first = f;
    }
    const bool is_first = live && first == e;
    const unsigned long long firsts = __ballot(is_first);
    const int my_slot = __popcll(firsts & ((1ull << e) - 1ull));  // valid on first lanes
    const int slot = __shfl(my_slot, first);
    if (is_first) s_rows[my_slot] = r;
    if (live) {
      if (e & 1) s_swb[e >> 1] = slot;
      else s_swa[e >> 1] = slot;
    }
    if (e == 0) s_nrows = __popcll(firsts);
  }
  __syncthreads();
  const int nr = s_nrows;
  int* perm = perm_all + (int64_t)node * n;
  // ---- interchanges on the other panel columns (one thread per column);
  //      thread LU_NB applies them to perm.  Then U rows of the leaf for the columns right
  //      of it: U = Lsub^-1 (swapped top rows).
  const int ocols = nbc - ibc;
  if (tid < ocols || tid == LU_NB) {
    // each thread owns one column (or perm) and keeps the touched rows in its own LDS
    // column, where the swap sequence and the U solve index freely
    const bool is_perm = (tid == LU_NB);
    const int cc = tid;
    const int64_t col = is_perm ? 0 : ((cc < jb) ? (k + cc) : (k + cc + ibc));
    // all the gathers are issued before the first one is used; every slot loads (slots
    // past nr repeat the first touched row, nr >= 1) so that the staging arrays stay in
    // registers, and only the nr real ones are kept
    if (is_perm) {
      int gp[2 * IB];
#pragma unroll
      for (int e = 0; e < 2 * IB; ++e) gp[e] = perm[row0 + s_rows[e < nr ? e : 0]];
#pragma unroll
      for (int e = 0; e < 2 * IB; ++e)
        if (e < nr) opv[e] = gp[e];
    } else {
      C gv[2 * IB];
#pragma unroll
      for (int e = 0; e < 2 * IB; ++e) gv[e] = LU[(row0 + s_rows[e < nr ? e : 0]) * ld + col];
#pragma unroll
      for (int e = 0; e < 2 * IB; ++e)
        if (e < nr) oval[e][cc] = gv[e];
    }
    for (int j = 0; j < ibc; ++j) {
      const int a = s_swa[j], b = s_swb[j];
      if (a == b) continue;
      if (is_perm) {
        const int t0 = opv[a];
        opv[a] = opv[b];
        opv[b] = t0;
      } else {
        const C t0 = oval[a][cc];
        oval[a][cc] = oval[b][cc];
        oval[b][cc] = t0;
      }
    }
    // U rows of the leaf (columns right of the leaf): local row j sits in slot s_swa[j]
    if (!is_perm && cc >= jb) {
      for (int j = 0; j < ibc; ++j) {
        C x = oval[s_swa[j]][cc];
        for (int i = 0; i < j; ++i) x = x - Lsub[j][i] * oval[s_swa[i]][cc];
        oval[s_swa[j]][cc] = x;
      }
    }
    for (int e = 0; e < nr; ++e) {
      const int64_t row = row0 + s_rows[e];
      if (is_perm) perm[row] = opv[e];
      else LU[row * ld + col] = oval[e][cc];
    }
  }
  if (tid < ibc) ipiv_all[(int64_t)node * n + row0 + tid] = (int)row0 + s_ipiv[tid];
  if (tid == 0 && s_zero != 0 && info_all[node] == 0) info_all[node] = s_zero;
}

// A[row0+IB.., cols right of the leaf within the panel] -= L_leaf * U_leaf
constexpr int LU_ROWS = 64;  // rows per workgroup of the update

template <typename C, int IB>
__global__ __launch_bounds__(256) void k_leaf_update(int64_t n, int64_t ld, int k, int jb, int nbc, C* __restrict__ LUall) {
  const int node = blockIdx.y;
  C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  const int ibc = min(IB, nbc - jb);
  const int64_t row0 = k + jb;
  const int64_t c0 = row0 + ibc;             // first column right of the leaf
  const int ucols = (int)(k + nbc - c0);      // columns to update
  const int64_t rbeg = row0 + ibc + (int64_t)blockIdx.x * LU_ROWS;
  const int64_t rend = min<int64_t>(rbeg + LU_ROWS, n);
  if (ucols <= 0 || rbeg >= n) return;
  __shared__ C Us[IB][LU_NB];
  __shared__ C Ls[LU_ROWS][IB];
  const int tid = threadIdx.x;
  for (int e = tid; e < IB * LU_NB; e += 256) {
    const int i = e / LU_NB, c = e % LU_NB;
    Us[i][c] = (i < ibc && c < ucols) ? LU[(row0 + i) * ld + c0 + c] : C(0);
  }
  for (int e = tid; e < LU_ROWS * IB; e += 256) {
    const int r = e / IB, i = e % IB;
    const int64_t row = rbeg + r;
    Ls[r][i] = (row < rend && i < ibc) ? LU[row * ld + row0 + i] : C(0);
  }
  __syncthreads();
  for (int e = tid; e < LU_ROWS * ucols; e += 256) {
    const int r = e / ucols, c = e % ucols;
    const int64_t row = rbeg + r;
    if (row >= rend) continue;
    C s = LU[row * ld + c0 + c];
#pragma unroll
    for (int i = 0; i < IB; ++i) s = s - Ls[r][i] * Us[i][c];
    LU[row * ld + c0 + c] = s;
  }
}

template <typename C, int IB, int RMAX, int NT = LEAF_THREADS>
static int run_leaves(hipStream_t s, int64_t n, int k, int nbc, int ne, C* LU, int* ipiv, int* perm, int* info) {
  for (int jb = 0; jb < nbc; jb += IB) {
    hipLaunchKernelGGL((k_leaf<C, IB, RMAX, NT>), dim3(ne), dim3(NT), 0, s, n, lu_ld(n), k, jb, nbc, LU, ipiv,
                       perm, info);
    const int ibc = std::min(IB, nbc - jb);
    if (jb + ibc < nbc) {
      const int64_t rows = n - (k + jb + ibc);
      hipLaunchKernelGGL((k_leaf_update<C, IB>), dim3((unsigned)((rows + LU_ROWS - 1) / LU_ROWS), ne), dim3(256), 0, s,
                         n, lu_ld(n), k, jb, nbc, LU);
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename C>
static int launch_leaves(hipStream_t s, int64_t n, int k, int nbc, int ne, C* LU, int* ipiv, int* perm, int* info) {
  constexpr bool dbl = sizeof(C) == 16;
  const int64_t rows = n - k;
  // short panels: fewer waves, several rows each (cheaper barriers and candidate merges)
  if (rows <= 1024) return dbl ? run_leaves<C, 4, 4, 256>(s, n, k, nbc, ne, LU, ipiv, perm, info)
                               : run_leaves<C, 8, 4, 256>(s, n, k, nbc, ne, LU, ipiv, perm, info);
  if (rows <= 2048) return dbl ? run_leaves<C, 4, 8, 256>(s, n, k, nbc, ne, LU, ipiv, perm, info)
                               : run_leaves<C, 8, 8, 256>(s, n, k, nbc, ne, LU, ipiv, perm, info);
  if (rows <= 4096) return dbl ? run_leaves<C, 4, 8, 512>(s, n, k, nbc, ne, LU, ipiv, perm, info)
                               : run_leaves<C, 8, 8, 512>(s, n, k, nbc, ne, LU, ipiv, perm, info);
  if (rows <= 8192) return dbl ? run_leaves<C, 2, 8>(s, n, k, nbc, ne, LU, ipiv, perm, info)
                               : run_leaves<C, 4, 8>(s, n, k, nbc, ne, LU, ipiv, perm, info);
  return dbl ? run_leaves<C, 1, 16>(s, n, k, nbc, ne, LU, ipiv, perm, info)
             : run_leaves<C, 2, 16>(s, n, k, nbc, ne, LU, ipiv, perm, info);
}

// ---------------------------------------------------------------------------
// inverses of the diagonal blocks: Linv (unit lower) and Uinv (upper), row-major
// LU_NB x LU_NB per block, zero-padded when the last block is narrower.
template <typename C>
__global__ __launch_bounds__(256) void k_invert_diag(int64_t n, int64_t ld, int kfirst, int nblocks, const C* __restrict__ LUall,
                                                      C* __restrict__ Dinv) {
  const int node = blockIdx.y;
  const int blk = kfirst / LU_NB + blockIdx.x;
  const int64_t k = (int64_t)blk * LU_NB;
  const int nbc = (int)min<int64_t>(LU_NB, n - k);
  const C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  const int nblk_total = (int)((n + LU_NB - 1) / LU_NB);
  C* __restrict__ Li = Dinv + ((int64_t)node * nblk_total + blk) * 2 * LU_NB * LU_NB;
  C* __restrict__ Ui = Li + LU_NB * LU_NB;
  __shared__ C Ls[LU_NB][LU_NB + 1];
  __shared__ C X[LU_NB][LU_NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < LU_NB * LU_NB; e += 256) {
    const int i = e / LU_NB, j = e % LU_NB;
    Ls[i][j] = (i < nbc && j < nbc) ? LU[(k + i) * ld + k + j] : C(0);
  }
  __syncthreads();
  // unit lower inverse: column c solved by thread c
  if (tid < LU_NB) {
    const int c = tid;
    for (int i = 0; i < LU_NB; ++i) {
      C s = (i == c) ? C(1) : C(0);
      if (i > c && i < nbc) {
        for (int j = c; j < i; ++j) s = s - Ls[i][j] * X[j][c];
      }
      if (i >= nbc || c >= nbc) s = C(0);
      X[i][c] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < LU_NB * LU_NB; e += 256) Li[e] = X[e / LU_NB][e % LU_NB];
  __syncthreads();
  // upper inverse: column c by back substitution
  if (tid < LU_NB) {
    const int c = tid;
    for (int i = LU_NB - 1; i >= 0; --i) {
      C s = C(0);
      if (c < nbc && i <= c) {
        s = (i == c) ? C(1) : C(0);
        for (int j = i + 1; j <= c; ++j) s = s - Ls[i][j] * X[j][c];
        const C d = Ls[i][i];
        s = (abs1(d) > 0) ? cdiv(s, d) : C(0);
      }
      X[i][c] = s;
    }
  }
  __syncthreads();
  for (int e = tid; e < LU_NB * LU_NB; e += 256) Ui[e] = X[e / LU_NB][e % LU_NB];
}

// ---------------------------------------------------------------------------
// U12 = L11^-1 A12 for the LU_NB rows of block k (A12 already interchanged): forward
// substitution in LDS and registers.  Workgroup x owns CW columns of A12; thread
// (wave w, lane c) keeps rows w, w + 4, ... of its column in registers; at step i
// the owner of row i publishes it through LDS and every row below subtracts
// L[r][i] times it.
template <typename C>
struct u12_cols { static constexpr int value = sizeof(C) == 8 ? 64 : 32; };

template <typename C>
__global__ __launch_bounds__(256) void k_trsm_u12(int64_t n, int64_t ld, int k, int rest, C* __restrict__ LUall) {
  constexpr int CW = u12_cols<C>::value;
  constexpr int RG = 256 / CW;       // row groups
  constexpr int RPT = LU_NB / RG;    // rows per thread
  const int node = blockIdx.y;
  C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  const int tid = threadIdx.x;
  const int c = tid % CW, w = tid / CW;
  const int64_t col = (int64_t)k + LU_NB + (int64_t)blockIdx.x * CW + c;
  const bool live = blockIdx.x * CW + c < rest;
  __shared__ C Ls[LU_NB][LU_NB + 1];
  __shared__ C rowbuf[2][RPT][CW];
  for (int e = tid; e < LU_NB * LU_NB; e += 256) {
    const int i = e / LU_NB, j = e % LU_NB;
    Ls[i][j] = LU[((int64_t)k + i) * ld + k + j];
  }
  // row group w holds the RPT consecutive rows w*RPT .. w*RPT + RPT - 1 of its column
  C v[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) v[q] = live ? LU[((int64_t)k + w * RPT + q) * ld + col] : C(0);
  __syncthreads();
  // block b: its owner finishes the substitution inside the block in registers and
  // publishes the block's rows; the groups below apply them.  Every row receives the
  // terms of the rows above it in increasing order, as in a row-by-row substitution.
  for (int b = 0; b < RG; ++b) {
    if (w == b) {
#pragma unroll
      for (int qs = 0; qs < RPT; ++qs) {
        const C x = v[qs];
#pragma unroll
        for (int q = qs + 1; q < RPT; ++q) v[q] = v[q] - Ls[b * RPT + q][b * RPT + qs] * x;
        rowbuf[b & 1][qs][c] = x;
      }
    }
    __syncthreads();
    if (w > b) {
#pragma unroll
      for (int qs = 0; qs < RPT; ++qs) {
        const C x = rowbuf[b & 1][qs][c];
#pragma unroll
        for (int q = 0; q < RPT; ++q) v[q] = v[q] - Ls[w * RPT + q][b * RPT + qs] * x;
      }
    }
  }
  if (live) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) LU[((int64_t)k + w * RPT + q) * ld + col] = v[q];
  }
}

// ---------------------------------------------------------------------------
// Row interchanges of a panel (rows k + j <-> ipiv[k + j], j = 0 .. nbc - 1, in order) on the
// columns outside the panel.  The net effect on the touched rows is a permutation: each
// workgroup builds it once (slots 0 .. nbc - 1 are rows k .. k + nbc - 1, then the
// distinct pivot rows below the panel; the swap sequence is replayed on slot labels),
// then gathers the touched rows of its LSW_COLS columns into LDS and writes them back
// permuted, instead of a chain of nbc dependent swaps per column.
constexpr int LSW_COLS = 64;

template <typename C>
__global__ __launch_bounds__(256) void k_laswp(int64_t n, int64_t ld, int k, int nbc, C* __restrict__ LUall,
                                               const int* __restrict__ ipiv_all) {
  __shared__ C buf[2 * LU_NB][LSW_COLS];
  __shared__ int s_row[2 * LU_NB];    // row of each slot
  __shared__ int s_lab[2 * LU_NB];    // slot whose original content ends in each slot
  __shared__ int s_sb[LU_NB];         // slot of the pivot row of interchange j
  __shared__ int s_nslot;
  const int node = blockIdx.y;
  const int tid = threadIdx.x;
  if (tid < 64) {
    // lane j: interchange j; pivot rows below the panel get slots nbc, nbc + 1, ... in
    // order of first appearance
    const int j = tid;
    const int b = j < nbc ? ipiv_all[(int64_t)node * n + k + j] : -1;
    const bool below = j < nbc && b >= k + nbc;
    int first = j;
#pragma unroll 8
    for (int f = 0; f < LU_NB; ++f) {
      const int bf = __shfl(b, f);
      if (f < first && below && bf == b) first = f;
    }
    const bool is_first = below && first == j;
    const unsigned long long firsts = __ballot(is_first);
    const int my_slot = nbc + __popcll(firsts & ((1ull << j) - 1ull));
    const int slot_first = __shfl(my_slot, first);
    if (j < nbc) {
      s_row[j] = k + j;
      s_sb[j] = below ? slot_first : b - k;
    }
    if (is_first) s_row[my_slot] = b;
    if (j == 0) s_nslot = nbc + __popcll(firsts);
  }
  __syncthreads();
  const int ns = s_nslot;
  if (tid == 0) {
    for (int q = 0; q < ns; ++q) s_lab[q] = q;
    for (int j = 0; j < nbc; ++j) {
      const int a = j, bb = s_sb[j];
      const int t0 = s_lab[a];
      s_lab[a] = s_lab[bb];
      s_lab[bb] = t0;
    }
  }
  __syncthreads();
  const int cl = tid % LSW_COLS, g = tid / LSW_COLS;  // column in the workgroup, row group
  const int64_t c = (int64_t)blockIdx.x * LSW_COLS + cl;
  const bool live = c < n && !(c >= k && c < k + nbc);
  C* __restrict__ LU = LUall + (int64_t)node * n * ld;
  if (live)
    for (int q = g; q < ns; q += 256 / LSW_COLS) buf[q][cl] = LU[(int64_t)s_row[q] * ld + c];
  __syncthreads();
  if (live)
    for (int q = g; q < ns; q += 256 / LSW_COLS) {
      const int from = s_lab[q];
      if (from != q) LU[(int64_t)s_row[q] * ld + c] = buf[from][cl];
    }
}

__global__ void k_perm_inverse(int64_t n, int ne, const int* __restrict__ perm, int* __restrict__ perm_inv) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int node = blockIdx.y;
  if (i >= n) return;
  perm_inv[(int64_t)node * n + perm[(int64_t)node * n + i]] = (int)i;
}

template <typename C>
int lu_factor(hipStream_t s, int64_t n, int ne, C* LU, int* ipiv, int* perm, int* perm_inv, int* info,
              C* Dinv) {
  if (n > MAX_N) return -2;
  using R = typename real_of<C>::type;
  const int64_t ld = lu_ld(n);
  for (int64_t k = 0; k < n; k += LU_NB) {
    const int nbc = (int)std::min<int64_t>(LU_NB, n - k);
    int tok = prof_begin(s);
    if (launch_leaves<C>(s, n, (int)k, nbc, ne, LU, ipiv, perm, info)) return -2;
    // panel flops: (n-k) nbc^2 / 2 complex multiply-adds per node
    prof_end(tok, s, K_LU_PANEL, 8.0 * 0.5 * (double)(n - k) * nbc * nbc * ne, 2.0 * sizeof(C) * (n - k) * nbc * ne);
    // row interchanges outside the panel and U12 = L11^-1 A12
    tok = prof_begin(s);
    hipLaunchKernelGGL((k_laswp<C>), dim3((unsigned)((n + LSW_COLS - 1) / LSW_COLS), ne), dim3(256), 0, s, n, ld, (int)k,
                       nbc, LU, ipiv);
    const int64_t rest = n - k - nbc;
    if (rest > 0) {
      // U12 = L11^-1 A12 in place (nbc == LU_NB whenever columns remain to the right)
      constexpr int CW = u12_cols<C>::value;
      hipLaunchKernelGGL((k_trsm_u12<C>), dim3((unsigned)((rest + CW - 1) / CW), ne), dim3(256), 0, s, n, ld, (int)k,
                         (int)rest, LU);
    }
    prof_end(tok, s, K_LU_ROWS, 8.0 * 0.5 * (double)nbc * nbc * (rest > 0 ? rest : 0) * ne,
             2.0 * sizeof(C) * (double)ne * nbc * n);
    if (rest > 0) {
      // A22 -= L21 U12
      GemmArgs t{};
      t.M = (int)rest; t.N = (int)rest; t.K = nbc;
      t.A = LU + (k + nbc) * ld + k; t.lda = ld; t.a_bs = n * ld;
      t.B = LU + k * ld + k + nbc; t.ldb = ld; t.b_bs = n * ld;
      t.C = LU + (k + nbc) * ld + k + nbc; t.ldc = ld; t.c_bs = n * ld;
      t.alpha = -1.0; t.beta = 1.0;
      t.tag = 1;
      tok = prof_begin(s);
      if (gemm<R, is_cplx<C>::value>(s, false, false, t, ne)) return -2;
      prof_end(tok, s, K_LU_GEMM, 8.0 * (double)rest * rest * nbc * ne,
               (double)sizeof(C) * ne * (2.0 * rest * rest + 2.0 * rest * nbc));
    }
  }
  // inverses of every diagonal block, for the solves
  const int64_t nblk = (n + LU_NB - 1) / LU_NB;
  const int tok = prof_begin(s);
  hipLaunchKernelGGL((k_invert_diag<C>), dim3((unsigned)nblk, ne), dim3(256), 0, s, n, ld, 0, (int)nblk, LU, Dinv);
  hipLaunchKernelGGL(k_perm_inverse, dim3((unsigned)((n + 255) / 256), ne), dim3(256), 0, s, n, ne, perm, perm_inv);
  prof_end(tok, s, K_LU_ROWS, 0.0, 0.0);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template int expand_full<double>(hipStream_t, char, int64_t, const double*, int64_t, double*);
template int expand_full<c64>(hipStream_t, char, int64_t, const c64*, int64_t, c64*);
template int shift_form<double, c32>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, c32*, int*, bool);
template int shift_form<double, c64>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, c64*, int*, bool);
template int shift_form<c64, c32>(hipStream_t, int64_t, const c64*, int64_t, const c64*, int64_t, const c64*, int, c32*, int*, bool);
template int shift_form<c64, c64>(hipStream_t, int64_t, const c64*, int64_t, const c64*, int64_t, const c64*, int, c64*, int*, bool);
template int lu_factor<c32>(hipStream_t, int64_t, int, c32*, int*, int*, int*, int*, c32*);
template int lu_factor<c64>(hipStream_t, int64_t, int, c64*, int*, int*, int*, int*, c64*);
template int shift_form<double, float>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, float*, int*, bool);
template int shift_form<double, double>(hipStream_t, int64_t, const double*, int64_t, const double*, int64_t, const c64*, int, double*, int*, bool);
template int lu_factor<float>(hipStream_t, int64_t, int, float*, int*, int*, int*, int*, float*);
template int lu_factor<double>(hipStream_t, int64_t, int, double*, int*, int*, int*, int*, double*);

}  // namespace mf
