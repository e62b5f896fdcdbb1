// Triangular solves B := T^{-1} B (left side, no transpose), row-major.
//
// RL2 / PF1 / RU1 / LL1 use the unit lower triangle trilu(A11) (Fig. "LU");
// the solve entry point also takes the upper / non-unit forms used by the
// back substitution of a linear solve.
//
// One kernel solves a triangle of up to 256 rows.  Each workgroup owns a block
// of 32 columns of B, which it keeps in LDS for the whole solve (read once,
// written once), and runs blocked substitution on it: for each 16-row diagonal
// block, 32 threads solve the block's rows (column by column, T's diagonal
// block staged in LDS), then the four waves update the rows still to be solved
// with v_mfma_f64_16x16x4f64 (A = -T from global memory, B = the solved rows,
// C = the LDS rows).  A wave owns whole 16-row blocks of the update, so the
// -T entries of a row are fetched once per step (two 16-byte loads per lane
// on aligned rows) and feed both 16-column halves; they are requested before
// the block solve, from clamped addresses with no condition, so they arrive
// while it runs.  Taller triangles are processed in 256-row blocks: solve a
// block, then update the rows still to be solved with the matrix-core GEMM.
#include "mlu_internal.h"

namespace mlu {
namespace {

constexpr int kRows = 256;     // rows per kernel
constexpr int kCols = 32;      // columns of B per workgroup
constexpr int kPitch = kCols + 4;
constexpr int kDiag = 16;      // diagonal block

// Batched form (gridDim.y > 1, n_total > 0): triangle y is the diagonal block
// of rows/columns [y kRows, min((y+1) kRows, n_total)) of T, solved against its
// own square B block at B + y b_stride (the inverses of the diagonal blocks
// when B holds identities).
template <bool LOWER, bool UNIT>
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
  __shared__ __attribute__((aligned(16))) double X[kRows * kPitch];
  __shared__ double Td[kDiag][kDiag + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lq = lane >> 4;
  const int c0 = blockIdx.x * kCols;

  // B block -> LDS (rows >= nr and columns >= ncols are zero and never
  // stored): all of this thread's loads are issued first, unconditionally
  // from clamped addresses, then masked into LDS
  {
    constexpr int kPer = kRows * kCols / 256;
    double bv[kPer];
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + 256 * i, r = e / kCols, c = e % kCols;
      bv[i] = B[(size_t)min(r, nr - 1) * ldb + min(c0 + c, ncols - 1)];
    }
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + 256 * i, r = e / kCols, c = e % kCols;
      X[r * kPitch + c] = (r < nr && c0 + c < ncols) ? bv[i] : 0.0;
    }
  }

  const int nblk = (nr + kDiag - 1) / kDiag;
  constexpr int kRB = (kRows / 16) / 4;   // 16-row blocks of the update per wave, at most
  const bool t_vec = (reinterpret_cast<uintptr_t>(T) & 7) == 0;
  // this thread's entry of T's diagonal block, loaded one step ahead
  const int dr = tid / kDiag, dc = tid % kDiag;
  auto diag_entry = [&](int step) {
    const int blk = LOWER ? step : nblk - 1 - step;
    const int bsz = min(kDiag, nr - blk * kDiag);
    return T[(size_t)(blk * kDiag + min(dr, bsz - 1)) * ldt + blk * kDiag + min(dc, bsz - 1)];
  };
  double tdv = diag_entry(0);
  // The loads are unconditional, from addresses clamped into the triangle
  // (rows < nr, columns ib..ib+bs-1), and masked where they are used: a
  // select at issue would make every load wait for its own result.  A lane's
  // four entries of an item are contiguous (k = 4 lq .. 4 lq + 3), so a full
  // block takes them in two 16-byte loads.
  auto load_ta = [&](int step, double (&ta)[kRB][4]) {
    const int blk = LOWER ? step : nblk - 1 - step;
    const int ib = blk * kDiag;
    const int bs = min(kDiag, nr - ib);
    const int rlo = LOWER ? ib + kDiag : 0;
    if (t_vec && bs == kDiag) {
#pragma unroll
      for (int i = 0; i < kRB; ++i) {
        const int tr = min(rlo + (wave + 4 * i) * 16 + li, nr - 1);
        const dbl2_g* pt = reinterpret_cast<const dbl2_g*>(T + (size_t)tr * ldt + ib + 4 * lq);
        const dbl2_g u0 = pt[0], u1 = pt[1];
        ta[i][0] = u0.x;
        ta[i][1] = u0.y;
        ta[i][2] = u1.x;
        ta[i][3] = u1.y;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kRB; ++i) {
        const int tr = min(rlo + (wave + 4 * i) * 16 + li, nr - 1);
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int k = min(4 * lq + st, bs - 1);   // MFMA step st feeds lane group lq with k = 4 lq + st
          ta[i][st] = T[(size_t)tr * ldt + ib + k];
        }
      }
    }
  };
  double ta[kRB][4];
  for (int step = 0; step < nblk; ++step) {
    const int blk = LOWER ? step : nblk - 1 - step;
    const int ib = blk * kDiag;
    const int bs = min(kDiag, nr - ib);
    // rows still to be solved: below the block (lower) or above it (upper);
    // this wave's 16-row blocks' -T entries are requested now, so the loads
    // overlap the block solve
    const int rlo = LOWER ? ib + kDiag : 0;
    const int rhi = LOWER ? nr : ib;
    const int nrb = rhi > rlo ? (rhi - rlo + 15) / 16 : 0;
    load_ta(step, ta);
    // T's diagonal block -> LDS (zero outside the block), then the next
    // step's entry is requested
    Td[dr][dc] = (dr < bs && dc < bs) ? tdv : 0.0;
    if (step + 1 < nblk) tdv = diag_entry(step + 1);
    lds_sync();
    // solve the block's rows, one column per thread.  No branch on the block
    // size: rows past bs are rows past nr, zero in LDS, and T is zero there,
    // so they only ever subtract exact zeros (and are divided only when
    // r < bs).  Lower: column by column, each row receives its terms in the
    // order of substitution (q ascending), so the result is the row-by-row
    // one, while the rows of one column update independently.
    if (tid < kCols) {
      double x[kDiag];
#pragma unroll
      for (int r = 0; r < kDiag; ++r) x[r] = X[(ib + r) * kPitch + tid];
      if (LOWER) {
#pragma unroll
        for (int q = 0; q < kDiag; ++q) {
          if (!UNIT) x[q] = q < bs ? x[q] / Td[q][q] : x[q];
#pragma unroll
          for (int r = q + 1; r < kDiag; ++r) x[r] = x[r] - Td[r][q] * x[q];
        }
      } else {
#pragma unroll
        for (int r = kDiag - 1; r >= 0; --r) {
          double v = x[r];
#pragma unroll
          for (int q = r + 1; q < kDiag; ++q) v = v - Td[r][q] * x[q];
          if (!UNIT) v = r < bs ? v / Td[r][r] : v;
          x[r] = v;
        }
      }
#pragma unroll
      for (int r = 0; r < kDiag; ++r) X[(ib + r) * kPitch + tid] = x[r];
    }
    lds_sync();
    // each wave updates whole 16-row blocks (wave, wave + 4, ...): both
    // 16-column halves of a block share its -T operands, as two MFMA chains
#pragma unroll
    for (int i = 0; i < kRB; ++i) {
      const int rb = wave + 4 * i;
      if (rb < nrb) {
        const int R0 = rlo + rb * 16;
        const bool row_ok = R0 + li < nr;
        v4d acc0, acc1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          acc0[r] = X[(R0 + lq + 4 * r) * kPitch + li];
          acc1[r] = X[(R0 + lq + 4 * r) * kPitch + 16 + li];
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const double b0 = X[(ib + 4 * lq + st) * kPitch + li];
          const double b1 = X[(ib + 4 * lq + st) * kPitch + 16 + li];
          const double a = (row_ok && 4 * lq + st < bs) ? -ta[i][st] : 0.0;
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc1, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          X[(R0 + lq + 4 * r) * kPitch + li] = acc0[r];
          X[(R0 + lq + 4 * r) * kPitch + 16 + li] = acc1[r];
        }
      }
    }
    lds_sync();
  }

  for (int e = tid; e < kRows * kCols; e += 256) {
    const int r = e / kCols, c = e % kCols;
    if (r < nr && c0 + c < ncols) B[(size_t)r * ldb + c0 + c] = X[r * kPitch + c];
  }
}

hipError_t solve_block(hipStream_t s, bool lower, bool unit, int nr, int ncols, const double* T, int ldt,
                       double* B, int ldb, const int32_t* skip) {
  const dim3 grid((ncols + kCols - 1) / kCols), block(256);
  if (lower && unit) hipLaunchKernelGGL((k_trsm_lds<true, true>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
  else if (lower) hipLaunchKernelGGL((k_trsm_lds<true, false>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
  else if (unit) hipLaunchKernelGGL((k_trsm_lds<false, true>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
  else hipLaunchKernelGGL((k_trsm_lds<false, false>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb, skip, 0, 0LL);
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
  const dim3 grid(kRows / kCols, nblk), block(256);
  const long long stride = (long long)kRows * kRows;
  if (lower && unit)
    hipLaunchKernelGGL((k_trsm_lds<true, true>), grid, block, 0, s, 0, 0, T, ldt, Inv, kRows, nullptr, n, stride);
  else if (lower)
    hipLaunchKernelGGL((k_trsm_lds<true, false>), grid, block, 0, s, 0, 0, T, ldt, Inv, kRows, nullptr, n, stride);
  else if (unit)
    hipLaunchKernelGGL((k_trsm_lds<false, true>), grid, block, 0, s, 0, 0, T, ldt, Inv, kRows, nullptr, n, stride);
  else
    hipLaunchKernelGGL((k_trsm_lds<false, false>), grid, block, 0, s, 0, 0, T, ldt, Inv, kRows, nullptr, n, stride);
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
