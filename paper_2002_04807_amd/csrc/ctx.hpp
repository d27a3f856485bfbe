// Handle of the C interface: device, stream and the workspace that grows on demand
// and is reused by later calls (internal header shared by the entry points).
#pragma once

#include <chrono>
#include <cstddef>
#include <vector>

#include "kernels.hpp"

namespace mf {

enum Slot {
  S_LU, S_DINV, S_PANINV, S_WY, S_WY2, S_IPIV, S_PERM, S_PINV, S_INFO, S_Z, S_WF, S_WC,
  S_X, S_Q, S_R, S_AQ, S_BQ, S_AX, S_BX, S_AF, S_BF,
  S_S, S_T, S_HW, S_V, S_G, S_TG, S_C, S_Z2, S_GZ, S_W,
  S_SMALL, S_PART, S_FLAG,
  S_BI_VEC, S_BI_BH, S_BI_COL, S_BI_TILES, S_BI_PART, S_BI_BUF,
  S_ADJ_AD, S_ADJ_XR, S_ADJ_R, S_ADJ_Y, S_ADJ_T, S_ADJ_SMALL,
  S_IR_XF, S_IR_YC, S_IR_T, S_IR_AX, S_IR_BX,
  S_SPLITK,
  // non-Hermitian driver: left blocks, products with A^H and B^H, bases, reduced factors
  S_NH_XL, S_NH_QL, S_NH_RL, S_NH_AHQ, S_NH_BHQ, S_NH_QLO, S_NH_BQO, S_NH_AHQO, S_NH_BHQO, S_NH_T3, S_NH_T4,
  S_NH_WL, S_NH_O1, S_NH_O2, S_NH_O3, S_NH_O4, S_NH_O5, S_NH_TR, S_NH_TL,
  // polynomial driver: products with every coefficient, reduced coefficients, companion form
  S_PL_AKQ, S_PL_AKQO, S_PL_AKX, S_PL_AQ, S_PL_L0, S_PL_L1, S_PL_WZ, S_PL_G, S_PL_H, S_PL_Z, S_PL_V,
  // batched problems: factors of every (problem, node) item, grouped in padded size classes
  S_BT_LU, S_BT_DINV, S_BT_PANINV, S_BT_IPIV, S_BT_PERM, S_BT_PINV, S_BT_INFO, S_BT_ITEMS,
  S_NSLOTS
};

#define MF_TRY(...)                      \
  do {                                   \
    if ((__VA_ARGS__) != 0) return -2;   \
  } while (0)

template <typename T> inline int gemmT(hipStream_t s, bool am, bool cj, const GemmArgs& g) {
  return gemm<double, is_cplx<T>::value>(s, am, cj, g, 1);
}

// row-major product C(MxN) = op(A) * B, helper for the internal blocks
template <typename T>
inline int rm_gemm(hipStream_t s, int M, int N, int K, const T* A, int64_t lda, bool a_mcontig, bool conj_a,
                   const T* B, int64_t ldb, T* C, int64_t ldc, double alpha = 1.0, double beta = 0.0,
                   int cls = K_RR_GEMM) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.a_bs = 0;
  g.B = B; g.ldb = ldb; g.b_bs = 0;
  g.C = C; g.ldc = ldc; g.c_bs = 0;
  g.alpha = alpha; g.beta = beta;
  const int tok = prof_begin(s);
  const int rc = gemmT<T>(s, a_mcontig, conj_a, g);
  const double fl = (is_cplx<T>::value ? 8.0 : 2.0) * (double)M * N * K;
  prof_end(tok, s, cls, fl, (double)sizeof(T) * ((double)M * K + (double)K * N + 2.0 * M * N));
  return rc;
}

struct Timer {
  std::chrono::steady_clock::time_point t0;
  void start() { t0 = std::chrono::steady_clock::now(); }
  double stop() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

}  // namespace mf

struct mfeast_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void* buf[mf::S_NSLOTS] = {};
  size_t cap[mf::S_NSLOTS] = {};
  char* pinned = nullptr;
  size_t pinned_cap = 0;
  int* pinned_i = nullptr;  // column states of the batched BiCGSTAB
  size_t pinned_i_cap = 0;
  char* pinned_aux = nullptr;  // small transfers of a call: contour nodes, LU flags, outputs
  size_t pinned_aux_cap = 0;
  mf::CsrWork csrA, csrB;
  std::vector<mfeast_ctx*> workers;  // batched calls: one handle and stream per worker thread
  bool owns_stream = false;
  // second stream and two events: the conjugate-transpose solves of the complex
  // Hermitian drivers run there next to the forward ones
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  double timing[8] = {};
  double prof[mf::K_NCLASS * 4] = {};
  bool prof_all = false;  // per-class timing of every later call (mfeast_set_profiling)
  double prof_sum[mf::K_NCLASS * 4] = {};  // batched workers: classes summed over their calls
  // batched problems: the captured factorization of all size classes (a HIP graph), the
  // key it was captured for (sizes, counts, buffers), one stream and event per class
  hipGraphExec_t bt_exec = nullptr;
  std::vector<int64_t> bt_key;
  std::vector<hipStream_t> bt_streams;
  std::vector<hipEvent_t> bt_events;
  // Allocation-free mode (mfeast_dsygv_noalloc): every workspace slot is carved from a
  // caller-supplied device region (a static device array), host staging uses ordinary
  // host memory, and nothing is ever freed.  A request that does not fit sets
  // arena_overflow and returns nullptr.
  char* arena = nullptr;
  size_t arena_cap = 0, arena_off = 0;
  bool arena_overflow = false;
  std::vector<char> arena_host[3];

  void* ws(mf::Slot s, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (arena != nullptr) {
      if (cap[s] >= bytes) return buf[s];
      const size_t off = (arena_off + 255) / 256 * 256;
      if (off > arena_cap || bytes > arena_cap - off) {
        arena_overflow = true;
        return nullptr;
      }
      buf[s] = arena + off;
      cap[s] = bytes;
      arena_off = off + bytes;
      return buf[s];
    }
    if (cap[s] < bytes) {
      if (buf[s]) (void)hipFree(buf[s]);
      buf[s] = nullptr;
      cap[s] = 0;
      if (hipMalloc(&buf[s], bytes) != hipSuccess) return nullptr;
      cap[s] = bytes;
    }
    return buf[s];
  }
  bool ensure_aux() {
    if (arena != nullptr) return false;  // no stream creation in the allocation-free mode
    if (aux != nullptr) return true;
    if (hipStreamCreateWithFlags(&aux, hipStreamNonBlocking) != hipSuccess) {
      aux = nullptr;
      return false;
    }
    if (hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_join, hipEventDisableTiming) != hipSuccess) {
      release_aux();
      return false;
    }
    return true;
  }
  void release_aux() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (aux) (void)hipStreamDestroy(aux);
    ev_fork = ev_join = nullptr;
    aux = nullptr;
  }
  char* host(size_t bytes) {
    if (arena != nullptr) {
      if (arena_host[0].size() < bytes) arena_host[0].resize(bytes);
      return arena_host[0].data();
    }
    if (pinned_cap < bytes) {
      if (pinned) (void)hipHostFree(pinned);
      pinned = nullptr;
      pinned_cap = 0;
      if (hipHostMalloc((void**)&pinned, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
      pinned_cap = bytes;
    }
    return pinned;
  }
  char* host_aux(size_t bytes) {
    if (arena != nullptr) {
      if (arena_host[1].size() < bytes) arena_host[1].resize(bytes);
      return arena_host[1].data();
    }
    if (pinned_aux_cap < bytes) {
      if (pinned_aux) (void)hipHostFree(pinned_aux);
      pinned_aux = nullptr;
      pinned_aux_cap = 0;
      if (hipHostMalloc((void**)&pinned_aux, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
      pinned_aux_cap = bytes;
    }
    return pinned_aux;
  }
  int* host_ints(size_t count) {
    const size_t bytes = count * sizeof(int) + 64;
    if (arena != nullptr) {
      if (arena_host[2].size() < bytes) arena_host[2].resize(bytes);
      return reinterpret_cast<int*>(arena_host[2].data());
    }
    if (pinned_i_cap < bytes) {
      if (pinned_i) (void)hipHostFree(pinned_i);
      pinned_i = nullptr;
      pinned_i_cap = 0;
      if (hipHostMalloc((void**)&pinned_i, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
      pinned_i_cap = bytes;
    }
    return pinned_i;
  }
};

// split-K scratch of a handle's GEMMs: its own slot, grown after the device is idle (earlier
// launches may still read the old buffer)
inline void* ctx_splitk_scratch(void* owner, size_t bytes) {
  mfeast_ctx* c = static_cast<mfeast_ctx*>(owner);
  if (c->arena != nullptr) {
    // allocation-free mode: carve it if it fits (a miss runs the product unsplit and is
    // not an error)
    const bool before = c->arena_overflow;
    void* p = c->ws(mf::S_SPLITK, bytes);
    if (p == nullptr) c->arena_overflow = before;
    return p;
  }
  if (c->cap[mf::S_SPLITK] < bytes && c->buf[mf::S_SPLITK] != nullptr) (void)hipDeviceSynchronize();
  return c->ws(mf::S_SPLITK, bytes);
}

// binds a handle's split-K scratch to the calling thread for the duration of an entry point
struct GemmScratchScope {
  explicit GemmScratchScope(mfeast_ctx* c) { mf::set_gemm_scratch(&ctx_splitk_scratch, c); }
  ~GemmScratchScope() { mf::set_gemm_scratch(nullptr, nullptr); }
  GemmScratchScope(const GemmScratchScope&) = delete;
  GemmScratchScope& operator=(const GemmScratchScope&) = delete;
};
