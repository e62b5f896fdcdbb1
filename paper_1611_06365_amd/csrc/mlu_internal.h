// Internal declarations shared by the HIP sources of libmlu (not part of the ABI).
#pragma once
#include "../../include/mlu.h"
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace mlu {

// mlu_dgetrf's variant argument: one of the enum's values
inline bool valid_variant(int v) { return v == MLU_RL || v == MLU_LL || v == MLU_LA || v == MLU_LA_NOWS; }

typedef double v4d __attribute__((ext_vector_type(4)));
// Two consecutive doubles read from global memory with one 16-byte load at
// any 8-byte aligned address (loads of several dwords need only dword
// alignment on this hardware), so that rows of an odd leading dimension keep
// the wide loads.
typedef double dbl2_g __attribute__((ext_vector_type(2), aligned(8)));

constexpr int kWave = 64;

// Workgroup barrier that orders LDS only.  __syncthreads() also waits for the
// wave's outstanding global loads and stores (the vector memory counter counts
// both), which defeats loads issued ahead of a barrier for later use and, in
// the panel kernel, device-coherent stores (about a microsecond per column).
// For kernels whose waves exchange nothing through global memory inside the
// workgroup.
__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------- panel kernel
// Widest register-resident panel block, the largest number of cooperating
// workgroups of one panel launch and the tallest panel they hold (the leader
// holds 512 rows, every other workgroup 1024).
constexpr int kPanelMaxCols = 32;   // exchange-area width
constexpr int kPanelRegCols = 16;   // block width of the kernel at any height
constexpr int kPanelMaxWG = 33;
constexpr int kPanelMaxRows = 512 + (kPanelMaxWG - 1) * 1024;
// The kernel also holds blocks of up to kPanelWideCols columns in registers,
// one row per thread, in panels of at most kPanelWideRows rows (16 workgroups
// of 512 rows).
constexpr int kPanelWideCols = 32;
constexpr int kPanelWideWG = 16;
constexpr int kPanelWideRows = kPanelWideWG * 512;

// One published value: {value, aux, tag}, written and read as one 16-byte
// device-coherent access so that the tag and the value arrive together.
struct alignas(16) Chunk {
  double v;
  unsigned aux;
  unsigned tag;
};

// Cross-workgroup exchange area of the panel kernel.  Exact mode: per
// workgroup a header {|candidate|, row} and the candidate row, plus the
// diagonal row from workgroup 0, double-buffered by column parity.
// Speculative mode: the leader's pivot row of every column, and each
// workgroup's check result.  spec_off turns speculation off for the rest of a
// call once it has failed.
struct PanelWork {
  Chunk hdr[2][kPanelMaxWG];
  Chunk cand[2][kPanelMaxWG][kPanelMaxCols];
  Chunk diag[2][kPanelMaxCols];
  Chunk spec[kPanelMaxCols][kPanelMaxCols];
  Chunk verify[kPanelMaxWG];
  alignas(64) unsigned spec_off;
};

// Tile queues of the persistent trailing update (one per XCD, each counter on
// its own 128-byte line), in a ring of slots: the update of look-ahead
// iteration i takes slot i mod kQueueSlots and clears slot (i + 2) mod
// kQueueSlots, whose last users finished before it started.
constexpr int kXcd = 8;
constexpr int kQueueStride = 32;   // unsigned words between counters
constexpr int kQueueSlots = 4;
struct QueueWork {
  alignas(128) unsigned ctr[kQueueSlots][kXcd * kQueueStride];
};

// Early termination of the look-ahead panel: RU2 of outer iteration k stores
// k + 1 into ru_done; after each inner block of the panel a check raises stop
// once that is seen, and width records the panel columns factored so far.
struct EtWork {
  alignas(128) unsigned ru_done;
  int32_t stop;
  int32_t width;
};

struct Workspace {
  PanelWork panel;
  QueueWork queue;
  EtWork et;
};

size_t workspace_bytes();

// ---------------------------------------------------------------- launchers
// All take row-major operands; element (i, j) of X is X[i*ldx + j].

// C := C - A B   (A m x k, B k x n, C m x n).  `trailing` marks the outer
// trailing updates (RL3, PF2, RU2, LL2): same kernel body, own kernel name.
// Precision of the product in the outer trailing updates (the mixed-precision
// factorization): the operands are rounded to it, the product accumulated in
// it, and C stays FP64.
constexpr int kPrecF64 = 0;
constexpr int kPrecF32 = 1;
constexpr int kPrecBF16 = 2;   // BF16 operands, FP32 accumulation

// `trailing` selects the trailing-update kernel (and allows prec = kPrecF32 or
// kPrecBF16);
// `traced` lets a trailing launch record events while a trace is active.
// `skip` (device flag, may be null; generic kernel only): when it reads
// nonzero the launch does nothing.
hipError_t gemm_update(hipStream_t s, int m, int n, int k, const double* A, int lda,
                       const double* B, int ldb, double* C, int ldc, bool trailing = false,
                       int prec = kPrecF64, bool traced = true, const int32_t* skip = nullptr);
// The same update as a persistent kernel fed by the tile queues of one slot
// (`q`: kXcd counters kQueueStride words apart, zero before the first launch
// that uses them).  Each workgroup takes tiles from the queue of its own XCD,
// then from the others.  `reserve` > 0 makes workgroups that start on a CU
// whose id within its shader engine is < reserve (mod 8) leave at once, so those
// CUs stay free for the panel factorization running beside it; only valid when
// another launch on the same queue without reserve follows (it finishes the
// tiles).  `clear` (may be null): kXcd counters that workgroup 0 zeroes first.
// `grid` 0 = two workgroups per CU.  `trace_id` (may be null) receives the
// trace slot of a traced launch (-1 if none); `tail_of` >= 0 marks a helper
// launch joining the queue of that traced launch, whose duration then extends
// to the helpers' end if they joined before it ended.  In FP64 with k a
// multiple of 16 the queue holds the whole 128 x 128 tiles only, and the
// partial last tile row and column are updated after them by the tile
// kernels when `edges` is set: the launch that owns the update sets it, its
// helpers (same m, n, k, hence the same queue) do not.
hipError_t gemm_queue(hipStream_t s, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                      double* C, int ldc, unsigned* q, unsigned* clear, int reserve, int grid, bool traced,
                      int prec = kPrecF64, int* trace_id = nullptr, int tail_of = -1, bool edges = true);
hipError_t trace_begin(int capacity);
hipError_t trace_end(int* launches, double* ms, double* flops, double* bytes);

// Factor the m x bw block whose top-left entry is global diagonal entry
// (row0, row0): partial pivoting over its rows, interchanges applied inside the
// block only; ipiv[row0 + c] = row0 + p + 1 (1-based); a zero pivot sets
// *info = row0 + c + 1 if *info was 0.
// `epoch` must differ between the launches of one call (the exchange area is
// cleared at the start of the call).  When the block lies inside a wider panel
// (cl columns of it to the block's left, cr to its right, same rows), the
// block's interchanges are also applied to those columns and the top rows of
// the first ns (-1: all cr) right columns are solved with a unit lower
// triangle: the block's own, or with lb = 16 (the second register pass of a
// 32-column diagonal block) the 32 x 32 triangle made of the 16 rows above the
// block and the block's rows, over the 16 columns to its left and its own.
// A nonzero *skip (a device flag written before the launch in stream order)
// makes every workgroup return at once.
hipError_t panel_factor(hipStream_t s, double* A, int lda, int m, int bw, int row0,
                        int32_t* ipiv, int32_t* info, PanelWork* work, unsigned epoch, int cl = 0,
                        int cr = 0, const int32_t* skip = nullptr, int ns = -1, int lb = 0);

// Apply interchanges ipiv[k1 .. k2) (1-based values, each >= its own index and
// < m) to columns [ca0, ca1) and [cb0, cb1) of the m-row matrix A.
hipError_t laswp(hipStream_t s, double* A, int lda, int m, int k1, int k2,
                 const int32_t* ipiv, int ca0, int ca1, int cb0, int cb1, int32_t* info,
                 const int32_t* skip = nullptr);

// B := T^{-1} B with T (nr x nr) lower/upper, unit/non-unit, B nr x ncols.
hipError_t trsm_left(hipStream_t s, bool lower, bool unit, int nr, int ncols,
                     const double* T, int ldt, double* B, int ldb, const int32_t* skip = nullptr);

// Inverses of the ib x ib diagonal blocks of the triangle of T (n x n): Inv
// holds ceil(n/ib) blocks of ib x ib (leading dimension ib), which must hold
// identities (the leading nr x nr of each) on entry.  The refinement applies
// the factors as GEMVs with these inverses (each block's solve) and with the
// off-diagonal blocks (the updates between them), 4 launches per block row
// and per pair of factors.  ib = 256 takes one batched triangular-solve
// launch per triangle; larger blocks solve each block on its own (ib^2 / 3
// flops per row, far more time) and save launches in every later
// application.  Plain refinement applies the factors a few times and uses
// 256; GMRES-IR applies them once per Krylov step and uses 1024 (256 when it
// makes plain corrections only, as mlu_dsgesv_ir).
constexpr int kIrInvBlock = 256;
constexpr int kGmresInvBlock = 1024;
hipError_t invert_diag_blocks(hipStream_t s, bool lower, bool unit, int n, const double* T, int ldt, double* Inv,
                              int ib);

hipError_t zero_bytes(hipStream_t s, void* p, size_t bytes);

// batched LU: workspace (queue counter and the size-sorted order) and the
// one-time raise of the kernels' LDS limit
size_t batched_workspace_bytes(int batch);
hipError_t batched_set_lds_limits();

// Argument checks and the whole factorization of mlu_dgetrf / mlu_dsgetrf
// (C-ABI return codes; `sh` shifts the numbers of arguments after
// `precision`), and the factorization alone for checked arguments (d_work
// holds a Workspace).
int getrf_entry(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
                int nb, int nb_inner, int inner, int precision, const int32_t* h_schedule, int n_schedule,
                int iters_limit, void* d_work, size_t work_bytes, int sh);
int getrf_run(void* stream, int m, int n, double* dA, int lda, int32_t* d_ipiv, int32_t* d_info, int variant,
              int nb, int nb_inner, int inner, int precision, const int32_t* h_schedule, int n_schedule,
              int iters_limit, void* d_work);
hipError_t init_static_scratch();

}  // namespace mlu
