// Drivers for the loop-based LU variants and the C ABI (include/mlu.h).
//
// Each variant is the paper's loop over an evolving 2x2 / 3x3 partition
// (FLAME notation); a partition is never copied: every block is a pointer and
// the leading dimension of the row-major matrix.  For iteration k with j
// columns done and block size b:
//   A11 = A + j*lda + j (b x b), A21 = A + (j+b)*lda + j, A12 = A + j*lda + j+b,
//   A22 = A + (j+b)*lda + j+b.
//
//  RL  (Fig. "LU", right)      RL1 panel -> interchanges -> RL2 trsm -> RL3 gemm
//  LA  (Fig. "LU_la_blk")      interchanges of the pending panel, then
//                              T_PF {PF1, PF2, PF3} on a second stream while
//                              T_RU {RU1, RU2} runs on the caller's stream
//  LL  (Section 4.2)           lazy interchanges of the panel columns, LL1 trsm
//                              and LL2 gemm block by block, LL3 panel,
//                              interchanges of the left columns
//  LA with early termination   LA whose PF3 is a left-looking inner LU that
//  (Section 4.2, Fig.          stops when RU2 signals; the width it reached
//  "LU_LA_ET")                 is the next block size
//
// The panel [A11; A21] is itself factored by the blocked RL or LL algorithm
// with the inner block size b_i <= 32 (the paper's outer / inner LU, Section
// 4.2), each b_i-wide block by the register-resident kernel (a block wider
// than its 16 register columns in two passes).
#include "mlu_internal.h"
#include "../../include/mlu.h"

#include <mutex>
#include <vector>

// The no-allocation entry point's scratch array (see init_static_scratch).
constexpr size_t kScratchBytes = (sizeof(mlu::Workspace) + 4095) / 4096 * 4096;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace mlu {
namespace {

__global__ void k_zero(unsigned* p, size_t nwords) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

// RU2 of outer iteration k is complete (stream order): publish k + 1 to the
// panel's stream with an agent-scope release.
__global__ void k_et_signal(unsigned* ru_done, unsigned k1) {
  if (threadIdx.x == 0) __hip_atomic_store(ru_done, k1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// End of one inner iteration of the look-ahead panel (Section 4.2, early
// termination): unless the panel has already stopped, it now covers `cols`
// columns; it stops once RU2 of the current outer iteration has signalled.
// The flag is read once per inner iteration, so every later launch of the
// panel sees one stable value.  A panel narrower than min_cols does not stop
// (0: any width, the rule of the method).
__global__ void k_et_check(const unsigned* ru_done, unsigned k1, int32_t* stop, int32_t* width, int cols,
                           int min_cols) {
  if (threadIdx.x == 0 && *stop == 0) {
    *width = cols;
    if (cols >= min_cols && __hip_atomic_load(ru_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= k1)
      *stop = 1;
  }
}

__global__ void k_et_reset(int32_t* stop, int32_t* width) {
  if (threadIdx.x == 0) {
    *stop = 0;
    *width = 0;
  }
}

// one library-owned stream and four events per device for the look-ahead fork;
// early termination adds one event and a pinned word for the panel width.
// `run` is held while one call enqueues its fork / join sequence, so that two
// host threads factoring on one device do not interleave their event records.
struct AuxStreams {
  bool ready = false;
  hipStream_t s1 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, ru1 = nullptr, pf2 = nullptr, width_ev = nullptr;
  int32_t* h_width = nullptr;
  std::mutex run;
};

// Look-ahead overlap: RU2 leaves the CUs with id < kLaReserve (mod 8) in every
// shader engine (4 per XCD per unit, 32 per unit on the chip) to the panel
// factorization, whose register-resident kernel needs whole CUs; once PF3 is
// done, kLaHelpers workgroups on the panel's stream join RU2's tile queue.
#ifndef MLU_LA_RESERVE
#define MLU_LA_RESERVE 1
#endif
constexpr int kLaReserve = MLU_LA_RESERVE;
constexpr int kLaHelpers = 64 * kLaReserve;
std::mutex g_aux_mu;
AuxStreams g_aux[64];

hipError_t get_aux(AuxStreams** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  AuxStreams& a = g_aux[dev];
  if (!a.ready) {
    if ((e = hipStreamCreateWithFlags(&a.s1, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.fork, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.join, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.ru1, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.pf2, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&a.width_ev, hipEventDisableTiming)) != hipSuccess) return e;
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&a.h_width), sizeof(int32_t), hipHostMallocDefault)) !=
        hipSuccess)
      return e;
    a.ready = true;
  }
  *out = &a;
  return hipSuccess;
}

#define MLU_TRY(x)                      \
  do {                                  \
    hipError_t e__ = (x);               \
    if (e__ != hipSuccess) return e__;  \
  } while (0)

struct Ctx {
  double* A;
  int lda, m, n;
  int32_t* ipiv;
  int32_t* info;
  int bi;
  PanelWork* work;
  QueueWork* queue;
  int prec;          // product precision of the outer trailing updates
  unsigned* epoch;   // panel launch counter of this call (panels run one at a time)
  int inner;         // algorithm of the panel factorization: MLU_RL or MLU_LL
  bool sharing = true;   // look-ahead: the panel's workgroups join RU2 after PF3
  double* at(int i, int j) const { return A + (size_t)i * lda + j; }
};

// LU_unb of the bw-column diagonal block at (jj, jj), bw <= 32 (Fig. "LU",
// left), inside a panel with cl columns to the block's left and cr to its
// right: the block's interchanges are applied to all of them, and the block's
// rows of the first ns right columns are solved with its unit lower triangle
// (the inner RL2).  The register-resident kernel holds up to 16 columns at any
// height and up to 32 in panels of at most kPanelWideRows rows; a wider block
// in a taller panel is eliminated in two register passes, right-looking over
// its columns: the first 16 columns (their rows of the other half solved), a
// rank-16 update of the other half, then that half; the second pass solves
// the right columns with the whole 32 x 32 triangle.
hipError_t factor_block(hipStream_t s, const Ctx& c, int jj, int bw, int cl, int cr, int ns,
                        const int32_t* skip = nullptr) {
  if (bw <= kPanelRegCols || c.m - jj <= kPanelWideRows)
    return panel_factor(s, c.at(jj, jj), c.lda, c.m - jj, bw, jj, c.ipiv, c.info, c.work, ++*c.epoch, cl, cr, skip,
                        ns);
  const int h1 = kPanelRegCols, h2 = bw - kPanelRegCols;
  MLU_TRY(panel_factor(s, c.at(jj, jj), c.lda, c.m - jj, h1, jj, c.ipiv, c.info, c.work, ++*c.epoch, cl, h2 + cr,
                       skip, h2));
  const int j2 = jj + h1;
  if (j2 < c.m)
    MLU_TRY(gemm_update(s, c.m - j2, h2, h1, c.at(j2, jj), c.lda, c.at(jj, j2), c.lda, c.at(j2, j2), c.lda, false,
                        kPrecF64, false, skip));
  return panel_factor(s, c.at(j2, j2), c.lda, c.m - j2, h2, j2, c.ipiv, c.info, c.work, ++*c.epoch, cl + h1, cr,
                      skip, ns, ns > 0 ? h1 : 0);
}

hipError_t factor_panel_ll(hipStream_t s, const Ctx& c, int j, int b, EtWork* et, unsigned k1, int min_cols);

// RL1 / PF3 / LL3: factor the panel rows j..m-1, columns j..j+b-1 by the
// inner variant with b_i-wide register-resident blocks; its interchanges are
// applied to the panel's own columns only.
hipError_t factor_panel(hipStream_t s, const Ctx& c, int j, int b) {
  if (c.inner == MLU_LL) return factor_panel_ll(s, c, j, b, nullptr, 0, 0);
  for (int jj = j; jj < j + b; jj += c.bi) {
    const int bw = (j + b - jj) < c.bi ? (j + b - jj) : c.bi;
    // the register-resident kernel also applies the block's interchanges to
    // the panel's other columns and solves the block's rows of the columns to
    // its right (the inner RL2); the inner RL3 follows
    const int rest = j + b - jj - bw;
    MLU_TRY(factor_block(s, c, jj, bw, jj - j, rest, rest));
    if (rest > 0 && jj + bw < c.m)
      MLU_TRY(gemm_update(s, c.m - jj - bw, rest, bw, c.at(jj + bw, jj), c.lda, c.at(jj, jj + bw), c.lda,
                          c.at(jj + bw, jj + bw), c.lda));
  }
  return hipSuccess;
}

// RL2 + RL3 (also RU1 + RU2 / PF1 + PF2) on columns [c0, c1) for the panel at j (size b)
hipError_t update_cols(hipStream_t s, const Ctx& c, int j, int b, int c0, int c1, bool traced = true) {
  if (c1 <= c0) return hipSuccess;
  MLU_TRY(trsm_left(s, true, true, b, c1 - c0, c.at(j, j), c.lda, c.at(j, c0), c.lda));
  if (j + b < c.m)
    MLU_TRY(gemm_update(s, c.m - j - b, c1 - c0, b, c.at(j + b, j), c.lda, c.at(j, c0), c.lda, c.at(j + b, c0),
                        c.lda, /*trailing=*/true, c.prec, traced));
  return hipSuccess;
}

hipError_t run_rl(hipStream_t s, const Ctx& c, const std::vector<int>& sched, int limit) {
  int j = 0;
  for (size_t it = 0; it < sched.size(); ++it) {
    if (limit >= 0 && (int)it >= limit) break;
    const int b = sched[it];
    MLU_TRY(factor_panel(s, c, j, b));                                           // RL1
    MLU_TRY(laswp(s, c.A, c.lda, c.m, j, j + b, c.ipiv, 0, j, j + b, c.n, c.info));
    MLU_TRY(update_cols(s, c, j, b, j + b, c.n));                                // RL2, RL3
    j += b;
  }
  return hipSuccess;
}

hipError_t run_la(hipStream_t s0, const Ctx& c, const std::vector<int>& sched, int limit) {
  AuxStreams* aux = nullptr;
  MLU_TRY(get_aux(&aux));
  std::lock_guard<std::mutex> lk(aux->run);
  hipStream_t s1 = aux->s1;
  if (sched.empty()) return hipSuccess;
  int b = sched[0];
  MLU_TRY(factor_panel(s0, c, 0, b));                                            // initial A_BR^P
  int j = 0;
  const int mn = c.m < c.n ? c.m : c.n;
  for (size_t k = 0; j < mn; ++k) {
    if (limit >= 0 && (int)k >= limit) break;
    // interchanges of the panel factored last, outside it
    MLU_TRY(laswp(s0, c.A, c.lda, c.m, j, j + b, c.ipiv, 0, j, j + b, c.n, c.info));
    const int jn = j + b;
    const int bp = (k + 1 < sched.size()) ? sched[k + 1] : 0;
    if (bp > 0) {
      MLU_TRY(hipEventRecord(aux->fork, s0));
      // T_RU: RU1, then RU2 as a persistent tile queue that leaves CUs to T_PF.
      // RU2 starts once PF2 is done: PF2's tiles would otherwise take CUs that
      // the persistent RU2 workgroups cannot get back until they finish,
      // which costs RU2 more than the wait (measured at n = 16384; starting
      // RU2 first only in the iterations where it is the longer chain was
      // measured too and is slower)
      const int c0 = jn + bp;
      const int mr = c.m - jn, nr = c.n - c0;
      unsigned* q = c.queue->ctr[k % kQueueSlots];
      unsigned* next = c.queue->ctr[(k + 2) % kQueueSlots];
      if (c0 < c.n) MLU_TRY(trsm_left(s0, true, true, b, c.n - c0, c.at(j, j), c.lda, c.at(j, c0), c.lda));
      MLU_TRY(hipEventRecord(aux->ru1, s0));
      // T_PF: PF1, PF2, PF3, then (worker sharing) it joins RU2's queue once RU1 is done
      MLU_TRY(hipStreamWaitEvent(s1, aux->fork, 0));
      MLU_TRY(update_cols(s1, c, j, b, jn, jn + bp, /*traced=*/false));         // PF1, PF2
      MLU_TRY(hipEventRecord(aux->pf2, s1));
      MLU_TRY(hipStreamWaitEvent(s0, aux->pf2, 0));
      int tid = -1;
      MLU_TRY(gemm_queue(s0, mr, nr, b, c.at(jn, j), c.lda, c.at(j, c0), c.lda, c.at(jn, c0), c.lda, q, next,
                         kLaReserve, 0, true, c.prec, &tid));
      MLU_TRY(factor_panel(s1, c, jn, bp));                                      // PF3
      if (c.sharing) {
        MLU_TRY(hipStreamWaitEvent(s1, aux->ru1, 0));
        MLU_TRY(gemm_queue(s1, mr, nr, b, c.at(jn, j), c.lda, c.at(j, c0), c.lda, c.at(jn, c0), c.lda, q,
                           nullptr, 0, kLaHelpers, false, c.prec, nullptr, tid, /*edges=*/false));
      }
      MLU_TRY(hipEventRecord(aux->join, s1));
      MLU_TRY(hipStreamWaitEvent(s0, aux->join, 0));
    } else {
      MLU_TRY(update_cols(s0, c, j, b, jn, c.n));                                // RU1, RU2
    }
    j = jn;
    b = bp;
  }
  return hipSuccess;
}

hipError_t run_ll(hipStream_t s, const Ctx& c, const std::vector<int>& sched, int limit) {
  int j = 0;
  bool completed = true;
  for (size_t it = 0; it < sched.size(); ++it) {
    if (limit >= 0 && (int)it >= limit) {
      completed = false;
      break;
    }
    const int b = sched[it];
    // the panel's columns receive every earlier interchange (lazy)
    MLU_TRY(laswp(s, c.A, c.lda, c.m, 0, j, c.ipiv, j, j + b, 0, 0, c.info));
    // LL1 and LL2, one earlier panel at a time: X_l := trilu(L_ll)^{-1} B_l,
    // then every row below panel l (A01 rows and [A11; A21]) -= L_{.,l} X_l
    int jl = 0;
    for (size_t l = 0; l < it; ++l) {
      const int bl = sched[l];
      MLU_TRY(trsm_left(s, true, true, bl, b, c.at(jl, jl), c.lda, c.at(jl, j), c.lda));
      MLU_TRY(gemm_update(s, c.m - jl - bl, b, bl, c.at(jl + bl, jl), c.lda, c.at(jl, j), c.lda,
                          c.at(jl + bl, j), c.lda, /*trailing=*/true, c.prec));
      jl += bl;
    }
    MLU_TRY(factor_panel(s, c, j, b));                                           // LL3
    MLU_TRY(laswp(s, c.A, c.lda, c.m, j, j + b, c.ipiv, 0, j, 0, 0, c.info));    // left columns
    j += b;
  }
  const int mn = c.m < c.n ? c.m : c.n;
  if (completed && c.n > mn) {
    MLU_TRY(laswp(s, c.A, c.lda, c.m, 0, mn, c.ipiv, mn, c.n, 0, 0, c.info));
    MLU_TRY(trsm_left(s, true, true, mn, c.n - mn, c.A, c.lda, c.at(0, mn), c.lda));
  }
  return hipSuccess;
}

// PF3 / the initial panel of the early-termination variant: the panel rows
// j..m-1, columns j..j+b-1, factored by the blocked left-looking algorithm
// with b_i-wide blocks (Section 4.2): before block [jj, jj+bw) it receives the
// panel's earlier interchanges (lazy), LL1 solves its rows j..jj-1 with the
// panel's unit lower triangle, LL2 updates its rows jj.. with the panel's
// columns to its left, LL3 factors it (interchanges applied to the panel's
// columns to its left only).  Nothing right of the block is touched, so the
// panel can stop after any block.  With `et`, every block after the first
// takes the stop flag and a check follows each block.
hipError_t factor_panel_ll(hipStream_t s, const Ctx& c, int j, int b, EtWork* et, unsigned k1, int min_cols) {
  for (int jj = j; jj < j + b; jj += c.bi) {
    const int bw = (j + b - jj) < c.bi ? (j + b - jj) : c.bi;
    const int32_t* skip = (et != nullptr && jj > j) ? &et->stop : nullptr;
    if (jj > j) {
      MLU_TRY(laswp(s, c.A, c.lda, c.m, j, jj, c.ipiv, jj, jj + bw, 0, 0, c.info, skip));
      MLU_TRY(trsm_left(s, true, true, jj - j, bw, c.at(j, j), c.lda, c.at(j, jj), c.lda, skip));     // LL1
      if (jj < c.m)
        MLU_TRY(gemm_update(s, c.m - jj, bw, jj - j, c.at(jj, j), c.lda, c.at(j, jj), c.lda, c.at(jj, jj),
                            c.lda, false, kPrecF64, false, skip));                                        // LL2
    }
    MLU_TRY(factor_block(s, c, jj, bw, jj - j, 0, 0, skip));                                             // LL3
    if (et != nullptr) {
      hipLaunchKernelGGL(k_et_check, dim3(1), dim3(64), 0, s, &et->ru_done, k1, &et->stop, &et->width,
                         jj + bw - j, min_cols);
      MLU_TRY(hipGetLastError());
    }
  }
  return hipSuccess;
}

// Look-ahead with early termination of the panel factorization (Section 4.2,
// Fig. "LU_LA_ET"): as run_la, with PF3 the left-looking inner LU above and
// a signal after RU2.  The host waits once per outer iteration for the width
// the panel reached (the next iteration's b); `force` = 1 stops every
// look-ahead panel after its first block, 2 never stops it.
hipError_t run_la_et(hipStream_t s0, const Ctx& c, int nb, EtWork* et, int force, int min_cols,
                     std::vector<int>* widths) {
  AuxStreams* aux = nullptr;
  MLU_TRY(get_aux(&aux));
  std::lock_guard<std::mutex> lk(aux->run);
  hipStream_t s1 = aux->s1;
  const int mn = c.m < c.n ? c.m : c.n;
  int b = nb < mn ? nb : mn;
  MLU_TRY(factor_panel_ll(s0, c, 0, b, nullptr, 0, 0));                          // initial A_BR^P
  widths->push_back(b);
  int j = 0;
  for (unsigned k = 0; j < mn; ++k) {
    MLU_TRY(laswp(s0, c.A, c.lda, c.m, j, j + b, c.ipiv, 0, j, j + b, c.n, c.info));
    const int jn = j + b;
    const int bp = (mn - jn) < nb ? (mn - jn) : nb;
    int bnext = 0;
    if (bp > 0) {
      const unsigned k1 = k + 1;
      MLU_TRY(hipEventRecord(aux->fork, s0));
      const int c0 = jn + bp;
      unsigned* q = c.queue->ctr[k % kQueueSlots];
      unsigned* next = c.queue->ctr[(k + 2) % kQueueSlots];
      if (c0 < c.n) MLU_TRY(trsm_left(s0, true, true, b, c.n - c0, c.at(j, j), c.lda, c.at(j, c0), c.lda));
      MLU_TRY(hipEventRecord(aux->ru1, s0));
      MLU_TRY(hipStreamWaitEvent(s1, aux->fork, 0));
      MLU_TRY(update_cols(s1, c, j, b, jn, jn + bp, /*traced=*/false));          // PF1, PF2
      hipLaunchKernelGGL(k_et_reset, dim3(1), dim3(64), 0, s1, &et->stop, &et->width);
      MLU_TRY(hipGetLastError());
      MLU_TRY(hipEventRecord(aux->pf2, s1));
      // RU2 once PF2 is done (as in run_la), then its completion signal
      const int mr = c.m - jn, nr = c.n - c0;
      MLU_TRY(hipStreamWaitEvent(s0, aux->pf2, 0));
      int tid = -1;
      MLU_TRY(gemm_queue(s0, mr, nr, b, c.at(jn, j), c.lda, c.at(j, c0), c.lda, c.at(jn, c0), c.lda, q, next,
                         kLaReserve, 0, true, c.prec, &tid));
      if (force != 2) {   // RU2 done: tell the panel
        hipLaunchKernelGGL(k_et_signal, dim3(1), dim3(64), 0, s0, &et->ru_done, k1);
        MLU_TRY(hipGetLastError());
      }
      if (force == 1) {   // as if RU2 had finished before the panel started
        hipLaunchKernelGGL(k_et_signal, dim3(1), dim3(64), 0, s1, &et->ru_done, k1);
        MLU_TRY(hipGetLastError());
      }
      MLU_TRY(factor_panel_ll(s1, c, jn, bp, et, k1, force == 1 ? 0 : min_cols));  // PF3, may stop early
      MLU_TRY(hipMemcpyAsync(aux->h_width, &et->width, sizeof(int32_t), hipMemcpyDeviceToHost, s1));
      MLU_TRY(hipEventRecord(aux->width_ev, s1));
      MLU_TRY(hipStreamWaitEvent(s1, aux->ru1, 0));
      MLU_TRY(gemm_queue(s1, mr, nr, b, c.at(jn, j), c.lda, c.at(j, c0), c.lda, c.at(jn, c0), c.lda, q, nullptr,
                         0, kLaHelpers, false, c.prec, nullptr, tid, /*edges=*/false));
      MLU_TRY(hipEventRecord(aux->join, s1));
      MLU_TRY(hipStreamWaitEvent(s0, aux->join, 0));
      MLU_TRY(hipEventSynchronize(aux->width_ev));
      bnext = *aux->h_width;
      if (bnext < 1 || bnext > bp) return hipErrorUnknown;
      widths->push_back(bnext);
    } else {
      MLU_TRY(update_cols(s0, c, j, b, jn, c.n));                                // RU1, RU2
    }
    j = jn;
    b = bnext;
  }
  return hipSuccess;
}

// Scratch of mlu_dgetrf_noalloc: one factorization workspace per device in a
// file-scope device array (each device holds its own copy until the process
// ends).  Host code never passes the array's name to a kernel: on the host it
// is a stand-in, not a device address.  init_static_scratch resolves the
// array's address on the current device once, and every use goes through it.
std::mutex g_scratch_mu;
void* g_scratch[64];

// The current device's scratch address, or null before mlu_init ran on it.
void* static_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[dev];
}

// Whether mlu_init has created the library stream of the current device.
bool aux_ready() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return false;
  std::lock_guard<std::mutex> lk(g_aux_mu);
  return g_aux[dev].ready;
}

}  // namespace

// Resolve the scratch array's address on the current device (once per device).
hipError_t init_static_scratch() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] != nullptr) return hipSuccess;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
  if (e != hipSuccess) return e;
  if (ptr == nullptr) return hipErrorInvalidSymbol;
  g_scratch[dev] = ptr;
  return hipSuccess;
}

hipError_t zero_bytes(hipStream_t s, void* p, size_t bytes) {
  const size_t nw = bytes / 4;
  if (nw == 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((nw + 255) / 256)), dim3(256), 0, s, (unsigned*)p, nw);
  return hipGetLastError();
}

}  // namespace mlu

using namespace mlu;

extern "C" {

int mlu_version(void) { return 200; }

int mlu_init(void) {
  AuxStreams* aux = nullptr;
  if (get_aux(&aux) != hipSuccess) return MLU_ERR_HIP;
  return init_static_scratch() == hipSuccess ? 0 : MLU_ERR_HIP;
}

int mlu_dgetrf_workspace(int m, int n, int variant, int nb, int nb_inner, size_t* bytes) {
  if (m < 0) return -1;
  if (n < 0) return -2;
  if (!valid_variant(variant)) return -3;
  if (nb < 1) return -4;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -5;
  if (!bytes) return -6;
  *bytes = workspace_bytes();
  // the library's per-device stream and events, created here (outside any
  // stream capture the caller may start afterwards); without a device this
  // does nothing, and a factorization call reports the failure
  (void)mlu_init();
  return 0;
}

}  // extern "C"

namespace mlu {

// mlu_dgetrf and mlu_dsgetrf; `sh` = 1 when called through mlu_dsgetrf, whose
// arguments after `precision` (argument 12) are numbered one higher.
int getrf_entry(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
                int nb, int nb_inner, int inner, int precision, const int32_t* h_schedule, int n_schedule,
                int iters_limit, void* d_work, size_t work_bytes, int sh) {
  const int mn = m < n ? m : n;
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (mn > 0 && !dA) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (mn > 0 && !d_ipiv) return -6;
  if (!d_info) return -7;
  if (!valid_variant(variant)) return -8;
  if (nb < 1) return -9;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -10;
  if (inner != MLU_RL && inner != MLU_LL) return -11;
  if (precision != MLU_PREC_FP64 && precision != MLU_PREC_FP32 && precision != MLU_PREC_BF16) return -12;
  if (h_schedule) {
    if (n_schedule < 1) return -13 - sh;
    for (int i = 0; i < n_schedule; ++i)
      if (h_schedule[i] < 1) return -12 - sh;
  }
  if (iters_limit < -1) return -14 - sh;
  if (!d_work) return -15 - sh;
  if (work_bytes < workspace_bytes()) return -16 - sh;
  if (m > kPanelMaxRows) return -2;
  return getrf_run(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, precision, h_schedule,
                   n_schedule, iters_limit, d_work);
}

// The factorization of a checked call; `d_work` holds a Workspace.
int getrf_run(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
              int nb, int nb_inner, int inner, int precision, const int32_t* h_schedule, int n_schedule,
              int iters_limit, void* d_work) {
  const int mn = m < n ? m : n;

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (zero_bytes(s, d_info, sizeof(int32_t)) != hipSuccess) return MLU_ERR_HIP;
  if (mn == 0) return 0;
  if (zero_bytes(s, d_work, sizeof(Workspace)) != hipSuccess) return MLU_ERR_HIP;

  std::vector<int> sched;
  int j = 0;
  for (int i = 0; h_schedule && i < n_schedule && j < mn; ++i) {
    const int b = h_schedule[i] < mn - j ? h_schedule[i] : mn - j;
    sched.push_back(b);
    j += b;
  }
  while (j < mn) {
    const int b = nb < mn - j ? nb : mn - j;
    sched.push_back(b);
    j += b;
  }
  unsigned epoch = 0;
  Workspace* ws = reinterpret_cast<Workspace*>(d_work);
  Ctx c{dA, lda, m, n, d_ipiv, d_info, 0, &ws->panel, &ws->queue,
        precision == MLU_PREC_FP32 ? kPrecF32 : (precision == MLU_PREC_BF16 ? kPrecBF16 : kPrecF64), &epoch, inner};
  c.bi = nb_inner > 0 ? nb_inner : (nb < kPanelRegCols ? nb : kPanelRegCols);
  c.sharing = variant != MLU_LA_NOWS;

  hipError_t e;
  if (variant == MLU_RL) e = run_rl(s, c, sched, iters_limit);
  else if (variant == MLU_LA || variant == MLU_LA_NOWS) e = run_la(s, c, sched, iters_limit);
  else e = run_ll(s, c, sched, iters_limit);
  return e == hipSuccess ? 0 : MLU_ERR_HIP;
}

}  // namespace mlu

extern "C" {

int mlu_dgetrf(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
               int nb, int nb_inner, int inner, const int32_t* h_schedule, int n_schedule, int iters_limit,
               void* d_work, size_t work_bytes) {
  const int rc = getrf_entry(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, MLU_PREC_FP64,
                             h_schedule, n_schedule, iters_limit, d_work, work_bytes, 0);
  return rc;
}

int mlu_dgetrf_noalloc(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info,
                       int variant, int nb, int nb_inner, int inner, const int32_t* h_schedule, int n_schedule,
                       int iters_limit) {
  const int mn = m < n ? m : n;
  if (m < 0 || m > kPanelMaxRows) return -2;
  if (n < 0) return -3;
  if (mn > 0 && !dA) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (mn > 0 && !d_ipiv) return -6;
  if (!d_info) return -7;
  if (!valid_variant(variant)) return -8;
  if (nb < 1) return -9;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -10;
  if (inner != MLU_RL && inner != MLU_LL) return -11;
  if (h_schedule) {
    if (n_schedule < 1) return -13;
    for (int i = 0; i < n_schedule; ++i)
      if (h_schedule[i] < 1) return -12;
  }
  if (iters_limit < -1) return -14;
  // the device's scratch array (and, for the look-ahead variant, the library
  // stream) must have been set up by mlu_init: nothing is created here
  void* ws = static_scratch();
  if (ws == nullptr || !aux_ready()) return MLU_ERR_NOINIT;
  static_assert(sizeof(Workspace) <= kScratchBytes, "the scratch array holds one workspace");
  return getrf_run(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, MLU_PREC_FP64, h_schedule,
                   n_schedule, iters_limit, ws);
}

int mlu_dsgetrf(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
                int nb, int nb_inner, int inner, int precision, const int32_t* h_schedule, int n_schedule,
                int iters_limit, void* d_work, size_t work_bytes) {
  return getrf_entry(stream, m, n, dA, lda, d_ipiv, d_info, variant, nb, nb_inner, inner, precision, h_schedule,
                     n_schedule, iters_limit, d_work, work_bytes, 1);
}

int mlu_dgetrf_et(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int nb,
                  int nb_inner, int force, int min_width, int32_t* h_widths, int max_widths, int* n_widths,
                  void* d_work, size_t work_bytes) {
  const int mn = m < n ? m : n;
  if (m < 0 || m > kPanelMaxRows) return -2;
  if (n < 0) return -3;
  if (mn > 0 && !dA) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (mn > 0 && !d_ipiv) return -6;
  if (!d_info) return -7;
  if (nb < 1) return -8;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -9;
  if (force < 0 || force > 2) return -10;
  if (min_width < 0) return -11;
  if (max_widths > 0 && !h_widths) return -12;
  if (max_widths < 0) return -13;
  if (!n_widths) return -14;
  if (!d_work) return -15;
  if (work_bytes < workspace_bytes()) return -16;
  *n_widths = 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (zero_bytes(s, d_info, sizeof(int32_t)) != hipSuccess) return MLU_ERR_HIP;
  if (mn == 0) return 0;
  if (zero_bytes(s, d_work, sizeof(Workspace)) != hipSuccess) return MLU_ERR_HIP;
  unsigned epoch = 0;
  Workspace* ws = reinterpret_cast<Workspace*>(d_work);
  Ctx c{dA, lda, m, n, d_ipiv, d_info, 0, &ws->panel, &ws->queue, kPrecF64, &epoch, MLU_LL};
  c.bi = nb_inner > 0 ? nb_inner : (nb < kPanelRegCols ? nb : kPanelRegCols);
  std::vector<int> widths;
  if (run_la_et(s, c, nb, &ws->et, force, min_width, &widths) != hipSuccess) return MLU_ERR_HIP;
  *n_widths = (int)widths.size();
  for (int i = 0; i < (int)widths.size() && i < max_widths; ++i) h_widths[i] = widths[i];
  return 0;
}

int mlu_dtrsm(void* stream, char uplo, char diag, int m, int nrhs, const double* dT, int ldt, double* dB,
              int ldb) {
  const bool lower = uplo == 'L' || uplo == 'l';
  const bool upper = uplo == 'U' || uplo == 'u';
  const bool unit = diag == 'U' || diag == 'u';
  const bool nonunit = diag == 'N' || diag == 'n';
  if (!lower && !upper) return -2;
  if (!unit && !nonunit) return -3;
  if (m < 0) return -4;
  if (nrhs < 0) return -5;
  if (m > 0 && !dT) return -6;
  if (ldt < (m > 1 ? m : 1)) return -7;
  if (m > 0 && nrhs > 0 && !dB) return -8;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -9;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return trsm_left(s, lower, unit, m, nrhs, dT, ldt, dB, ldb) == hipSuccess ? 0 : MLU_ERR_HIP;
}

int mlu_dgetrs(void* stream, int n, int nrhs, const double* dLU, int lda, const int32_t* d_ipiv, double* dB,
               int ldb) {
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (n > 0 && !dLU) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && !d_ipiv) return -6;
  if (n > 0 && nrhs > 0 && !dB) return -7;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -8;
  if (n == 0 || nrhs == 0) return 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (laswp(s, dB, ldb, n, 0, n, d_ipiv, 0, nrhs, 0, 0, nullptr) != hipSuccess) return MLU_ERR_HIP;
  if (trsm_left(s, true, true, n, nrhs, dLU, lda, dB, ldb) != hipSuccess) return MLU_ERR_HIP;
  if (trsm_left(s, false, false, n, nrhs, dLU, lda, dB, ldb) != hipSuccess) return MLU_ERR_HIP;
  return 0;
}

int mlu_dgemm_update(void* stream, int m, int n, int k, const double* dA, int lda, const double* dB, int ldb,
                     double* dC, int ldc) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (k < 0) return -4;
  if (m > 0 && k > 0 && !dA) return -5;
  if (lda < (k > 1 ? k : 1)) return -6;
  if (k > 0 && n > 0 && !dB) return -7;
  if (ldb < (n > 1 ? n : 1)) return -8;
  if (m > 0 && n > 0 && !dC) return -9;
  if (ldc < (n > 1 ? n : 1)) return -10;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return gemm_update(s, m, n, k, dA, lda, dB, ldb, dC, ldc) == hipSuccess ? 0 : MLU_ERR_HIP;
}

int mlu_dlaswp(void* stream, int m, int ncols, double* dA, int lda, int k1, int k2, const int32_t* d_ipiv,
               int32_t* d_info) {
  if (m < 0) return -2;
  if (ncols < 0) return -3;
  if (m > 0 && ncols > 0 && !dA) return -4;
  if (lda < (ncols > 1 ? ncols : 1)) return -5;
  if (k1 < 0 || k1 > m) return -6;
  if (k2 < k1 || k2 > m) return -7;
  if (k2 > k1 && !d_ipiv) return -8;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return laswp(s, dA, lda, m, k1, k2, d_ipiv, 0, ncols, 0, 0, d_info) == hipSuccess ? 0 : MLU_ERR_HIP;
}

int mlu_dgetf2_block(void* stream, int m, int bw, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info,
                     void* d_work, size_t work_bytes) {
  if (m < 0 || m > kPanelMaxRows) return -2;
  if (bw < 0 || bw > kPanelWideCols || bw > m) return -3;
  if (bw > kPanelRegCols && m > kPanelWideRows) return -2;
  if (bw > 0 && !dA) return -4;
  if (lda < (bw > 1 ? bw : 1)) return -5;
  if (bw > 0 && !d_ipiv) return -6;
  if (!d_info) return -7;
  if (!d_work) return -8;
  if (work_bytes < workspace_bytes()) return -9;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (zero_bytes(s, d_info, sizeof(int32_t)) != hipSuccess) return MLU_ERR_HIP;
  if (bw == 0) return 0;
  if (zero_bytes(s, d_work, sizeof(Workspace)) != hipSuccess) return MLU_ERR_HIP;
  return panel_factor(s, dA, lda, m, bw, 0, d_ipiv, d_info, &reinterpret_cast<Workspace*>(d_work)->panel, 1u) == hipSuccess
             ? 0
             : MLU_ERR_HIP;
}

int mlu_trace_begin(int capacity) {
  if (capacity < 1 || capacity > (1 << 20)) return -1;
  return trace_begin(capacity) == hipSuccess ? 0 : MLU_ERR_HIP;
}

int mlu_trace_end(int* launches, double* total_ms, double* flops, double* bytes) {
  if (!launches) return -1;
  if (!total_ms) return -2;
  if (!flops) return -3;
  if (!bytes) return -4;
  return trace_end(launches, total_ms, flops, bytes) == hipSuccess ? 0 : MLU_ERR_HIP;
}

}  // extern "C"
