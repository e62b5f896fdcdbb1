// Triangular solves B := T^{-1} B (left side, no transpose), row-major.
//
// RL2 / PF1 / RU1 / LL1 use the unit lower triangle trilu(A11) (Fig. "LU");
// the solve entry point also takes the upper / non-unit forms used by the
// back substitution of a linear solve.
//
// One kernel solves a triangle of up to 256 rows.  Each workgroup owns a block
// of 32 columns of B (16 when B has at most 256 columns, so that a narrow
// solve spreads over twice the workgroups), which it keeps in LDS for the
// whole solve (read once, written once), and runs blocked substitution on it
// with 16-row diagonal blocks and one barrier per block: while waves 1..3
// update the rows of the later blocks by the block just solved, with
// v_mfma_f64_16x16x4f64 (A = -T from global memory, B = the solved rows, C =
// the LDS rows), wave 0 updates the next block's rows first and solves them
// (one column per lane, T's diagonal block staged in LDS a step ahead).  A
// wave owns whole 16-row blocks of the update, so the -T entries of a row are
// fetched once per step (two 16-byte loads per lane on aligned rows) and feed
// every 16-column part.  Every row block receives the same updates, in the
// same order and by the same operations, as in plain blocked substitution.
// Taller triangles are processed in 256-row blocks: solve a block, then update
// the rows still to be solved with the matrix-core GEMM.
#include "mlu_internal.h"

namespace mlu {
namespace {

constexpr int kRows = 256;     // rows per kernel
constexpr int kCols = 32;      // columns of B per workgroup (16 for narrow right-hand sides)
constexpr int kDiag = 16;      // diagonal block

// Batched form (gridDim.y > 1, n_total > 0): triangle y is the diagonal block
// of rows/columns [y kRows, min((y+1) kRows, n_total)) of T, solved against its
// own square B block at B + y b_stride (the inverses of the diagonal blocks
// when B holds identities).
template <bool LOWER, bool UNIT, int KC>
__global__ __launch_bounds__(256, 2) void k_trsm_lds(int nr, int ncols, const double* __restrict__ T, int ldt,
                                                  double* __restrict__ B, int ldb,
                                                  const int32_t* __restrict__ skip, int n_total,
                                                  long long b_stride) {
  if (skip != nullptr && *skip != 0) return;   // a flag the caller raised on the device
  if (n_total > 0) {
    const int y = blockIdx.y;
    nr = min(kRows, n_total - y * kRows);
    ncols = nr;
    T += (size_t)y * kRows * ((size_t)ldt + 1);
    B += (size_t)y * (size_t)b_stride;
  }
  constexpr int kPitch = KC + 4;
  __shared__ __attribute__((aligned(16))) double X[kRows * kPitch];
  __shared__ double Td[2][kDiag][kDiag + 1];   // diagonal blocks, by step parity
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int c0 = blockIdx.x * KC;

  // B block -> LDS (rows >= nr and columns >= ncols are zero and never
  // stored): all of this thread's loads are issued first, unconditionally
  // from clamped addresses, then masked into LDS
  {
    constexpr int kPer = kRows * KC / 256;
    double bv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + 256 * i, r = e / KC, c = e % KC;
      bv[i] = B[(size_t)min(r, nr - 1) * ldb + min(c0 + c, ncols - 1)];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + 256 * i, r = e / KC, c = e % KC;
      X[r * kPitch + c] = (r < nr && c0 + c < ncols) ? bv[i] : 0.0;
    }
  }

  const int nblk = (nr + kDiag - 1) / kDiag;
  const bool t_vec = (reinterpret_cast<uintptr_t>(T) & 7) == 0;
  const int dr = tid / kDiag, dc = tid % kDiag;
  auto blk_of = [&](int step) { return LOWER ? step : nblk - 1 - step; };
  // this thread's entry of the diagonal block of a step, and its staging into
  // the LDS buffer of the step's parity (zero outside the block)
  auto diag_entry = [&](int step) {
    const int blk = blk_of(step);
    const int bsz = min(kDiag, nr - blk * kDiag);
    return T[(size_t)(blk * kDiag + min(dr, bsz - 1)) * ldt + blk * kDiag + min(dc, bsz - 1)];
  };
  auto stage_diag = [&](int step, double tdv) {
    const int bs = min(kDiag, nr - blk_of(step) * kDiag);
    Td[step & 1][dr][dc] = (dr < bs && dc < bs) ? tdv : 0.0;
  };
  // The block of a step solved in place, one column per lane (lanes
  // 0..KC-1 of the calling wave).  No branch on the block size: rows past
  // bs are rows past nr, zero in LDS, and T is zero there, so they only ever
  // subtract exact zeros (and are divided only when r < bs).  Lower: column
  // by column, each row receives its terms in the order of substitution (q
  // ascending), so the result is the row-by-row one, while the rows of one
  // column update independently.
  auto solve = [&](int step) {
    const int ib = blk_of(step) * kDiag;
    const int bs = min(kDiag, nr - ib);
    const double(*D)[kDiag + 1] = Td[step & 1];
    if (lane < KC) {
      double x[kDiag];
#pragma unroll
      for (int r = 0; r < kDiag; ++r) x[r] = X[(ib + r) * kPitch + lane];
      if (LOWER) {
#pragma unroll
        for (int q = 0; q < kDiag; ++q) {
          if (!UNIT) x[q] = q < bs ? x[q] / D[q][q] : x[q];
#pragma unroll
          for (int r = q + 1; r < kDiag; ++r) x[r] = x[r] - D[r][q] * x[q];
        }
      } else {
#pragma unroll
        for (int r = kDiag - 1; r >= 0; --r) {
          double v = x[r];
#pragma unroll
          for (int q = r + 1; q < kDiag; ++q) v = v - D[r][q] * x[q];
          if (!UNIT) v = r < bs ? v / D[r][r] : v;
          x[r] = v;
        }
      }
#pragma unroll
      for (int r = 0; r < kDiag; ++r) X[(ib + r) * kPitch + lane] = x[r];
    }
  };
  // -T entries of the 16 rows at R0 against the block of a step: MFMA step
  // st feeds lane group lq with k = 4 lq + st, so a lane's four entries are
  // contiguous and a full block takes them in two 16-byte loads.  The loads
  // are unconditional, from addresses clamped into the triangle, and masked
  // where they are used: a select at issue would make every load wait for
  // its own result.
  auto load_ta = [&](int step, int R0, double (&ta)[4]) {
    const int ib = blk_of(step) * kDiag;
    const int bs = min(kDiag, nr - ib);
    const int tr = min(R0 + li, nr - 1);
    if (t_vec && bs == kDiag) {
      const dbl2_g* pt = reinterpret_cast<const dbl2_g*>(T + (size_t)tr * ldt + ib + 4 * lq);
      const dbl2_g u0 = pt[0], u1 = pt[1];
      ta[0] = u0.x;
      ta[1] = u0.y;
      ta[2] = u1.x;
      ta[3] = u1.y;
    } else {
#pragma unroll
      for (int st = 0; st < 4; ++st) ta[st] = T[(size_t)tr * ldt + ib + min(4 * lq + st, bs - 1)];
    }
  };
  // The 16 rows at R0 (each 16-column part) minus T[R0.., block] times the
  // solved rows of the block of a step: one MFMA chain per part, sharing the
  // -T operands.
  auto update = [&](int step, int R0, const double (&ta)[4]) {
    const int ib = blk_of(step) * kDiag;
    const int bs = min(kDiag, nr - ib);
    const bool row_ok = R0 + li < nr;
    v4d acc[KC / 16];
#pragma unroll
    for (int h = 0; h < KC / 16; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[h][r] = X[(R0 + lq + 4 * r) * kPitch + 16 * h + li];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const double a = (row_ok && 4 * lq + st < bs) ? -ta[st] : 0.0;
#pragma unroll
      for (int h = 0; h < KC / 16; ++h)
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, X[(ib + 4 * lq + st) * kPitch + 16 * h + li], acc[h], 0, 0,
                                                      0);
    }
#pragma unroll
    for (int h = 0; h < KC / 16; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) X[(R0 + lq + 4 * r) * kPitch + 16 * h + li] = acc[h][r];
  };

  // Blocked substitution with one barrier per diagonal block.  While the
  // rows of the other blocks receive the update by the block just solved
  // (waves 1..3), wave 0 updates the rows of the next block first and solves
  // them, so the next step starts with its block solved.  Every row block
  // receives the same updates, in the same order and with the same
  // operations, as in plain blocked substitution.
  stage_diag(0, diag_entry(0));
  double tdv = nblk > 1 ? diag_entry(1) : 0.0;
  lds_sync();
  if (wave == 0) solve(0);
  if (nblk > 1) stage_diag(1, tdv);
  lds_sync();
  constexpr int kRB = (kRows / 16 - 2 + 2) / 3;   // blocks other than the next one, per wave 1..3
  for (int step = 0; step + 1 < nblk; ++step) {
    // rows still to be solved: below the block (lower) or above it (upper),
    // 16-row blocks rb = 0..nrb-1 from rlo; the next step's block is one of them
    const int ib = blk_of(step) * kDiag;
    const int rlo = LOWER ? ib + kDiag : 0;
    const int rhi = LOWER ? nr : ib;
    const int nrb = (rhi - rlo + 15) / 16;
    const int next_rb = LOWER ? 0 : nrb - 1;
    if (step + 2 < nblk) tdv = diag_entry(step + 2);
    if (wave == 0) {
      double ta[4];
      load_ta(step, rlo + 16 * next_rb, ta);
      update(step, rlo + 16 * next_rb, ta);
      // the wave's own LDS writes, in order, before its lanes read the rows back
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
      solve(step + 1);
    } else {
      double ta[kRB][4];
#pragma unroll
      for (int i = 0; i < kRB; ++i) {
        const int k = (wave - 1) + 3 * i;
        if (k < nrb - 1) load_ta(step, rlo + 16 * (LOWER ? 1 + k : k), ta[i]);
      }
#pragma unroll
      for (int i = 0; i < kRB; ++i) {
        const int k = (wave - 1) + 3 * i;
        if (k < nrb - 1) update(step, rlo + 16 * (LOWER ? 1 + k : k), ta[i]);
      }
    }
    if (step + 2 < nblk) stage_diag(step + 2, tdv);
    lds_sync();
  }

  for (int e = tid; e < kRows * KC; e += 256) {
    const int r = e / KC, c = e % KC;
    if (r < nr && c0 + c < ncols) B[(size_t)r * ldb + c0 + c] = X[r * kPitch + c];
  }
}

template <int KC>
void launch_trsm(hipStream_t s, bool lower, bool unit, dim3 grid, int nr, int ncols, const double* T, int ldt,
                 double* B, int ldb, const int32_t* skip, int n_total, long long b_stride) {
  const dim3 block(256);
  if (lower && unit)
    hipLaunchKernelGGL((k_trsm_lds<true, true, KC>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, n_total,
                       b_stride);
  else if (lower)
    hipLaunchKernelGGL((k_trsm_lds<true, false, KC>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, n_total,
                       b_stride);
  else if (unit)
    hipLaunchKernelGGL((k_trsm_lds<false, true, KC>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, n_total,
                       b_stride);
  else
    hipLaunchKernelGGL((k_trsm_lds<false, false, KC>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, n_total,
                       b_stride);
}

// Right-hand sides of at most this many columns go to workgroups of 16
// columns (twice the workgroups, half the update work on each one's chain).
constexpr int kNarrowCols = 256;

hipError_t solve_block(hipStream_t s, bool lower, bool unit, int nr, int ncols, const double* T, int ldt,
                       double* B, int ldb, const int32_t* skip) {
  if (ncols <= kNarrowCols)
    launch_trsm<16>(s, lower, unit, dim3((ncols + 15) / 16), nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
  else
    launch_trsm<kCols>(s, lower, unit, dim3((ncols + kCols - 1) / kCols), nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
  return hipGetLastError();
}

}  // namespace

hipError_t invert_diag_blocks(hipStream_t s, bool lower, bool unit, int n, const double* T, int ldt, double* Inv,
                              int ib) {
  if (n <= 0) return hipSuccess;
  if (ib < 1) return hipErrorInvalidValue;
  if (ib != kRows) {   // each block's inverse solves T_kk X = I by the blocked solve
    for (int r0 = 0; r0 < n; r0 += ib) {
      const int nb = n - r0 < ib ? n - r0 : ib;
      const hipError_t e = trsm_left(s, lower, unit, nb, nb, T + (size_t)r0 * ldt + r0, ldt,
                                     Inv + (size_t)(r0 / ib) * ib * ib, ib);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int nblk = (n + kRows - 1) / kRows;
  launch_trsm<kCols>(s, lower, unit, dim3(kRows / kCols, nblk), 0, 0, T, ldt, Inv, kRows, nullptr, n,
                     (long long)kRows * kRows);
  return hipGetLastError();
}

hipError_t trsm_left(hipStream_t s, bool lower, bool unit, int nr, int ncols, const double* T, int ldt,
                     double* B, int ldb, const int32_t* skip) {
  if (nr <= 0 || ncols <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (lower) {
    for (int r0 = 0; r0 < nr; r0 += kRows) {
      const int rb = nr - r0 < kRows ? nr - r0 : kRows;
      e = solve_block(s, true, unit, rb, ncols, T + (size_t)r0 * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb, skip);
      if (e != hipSuccess) return e;
      const int rest = nr - r0 - rb;
      if (rest > 0) {
        e = gemm_update(s, rest, ncols, rb, T + (size_t)(r0 + rb) * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb,
                        B + (size_t)(r0 + rb) * ldb, ldb, false, kPrecF64, true, skip);
        if (e != hipSuccess) return e;
      }
    }
  } else {
    for (int r1 = nr; r1 > 0; r1 -= kRows) {
      const int r0 = r1 - kRows > 0 ? r1 - kRows : 0;
      e = solve_block(s, false, unit, r1 - r0, ncols, T + (size_t)r0 * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb,
                      skip);
      if (e != hipSuccess) return e;
      if (r0 > 0) {
        e = gemm_update(s, r0, ncols, r1 - r0, T + r0, ldt, B + (size_t)r0 * ldb, ldb, B, ldb, false, kPrecF64, true,
                        skip);
        if (e != hipSuccess) return e;
      }
    }
  }
  return e;
}

}  // namespace mlu
