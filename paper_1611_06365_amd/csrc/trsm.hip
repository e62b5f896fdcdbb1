// Triangular solves B := T^{-1} B (left side, no transpose), row-major.
//
// RL2 / PF1 / RU1 / LL1 use the unit lower triangle trilu(A11) (Fig. "LU");
// the solve entry point also takes the upper / non-unit forms used by the
// back substitution of a linear solve.
//
// A block of at most 32 rows is solved by one kernel in which each thread owns
// one column of B in registers and reads T through uniform (scalar) loads.
// Taller triangles are processed in 32-row blocks: solve a block, then update
// the rows still to be solved with the matrix-core GEMM (C := C - A B).
#include "mlu_internal.h"

namespace mlu {
namespace {

constexpr int kRows = 32;

template <bool LOWER, bool UNIT>
__global__ __launch_bounds__(256) void k_trsm_block(int nr, int ncols, const double* __restrict__ T, int ldt,
                                                    double* __restrict__ B, int ldb) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double x[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) x[r] = (r < nr) ? B[(size_t)r * ldb + col] : 0.0;
  if (LOWER) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (r < nr) {
        double s = x[r];
#pragma unroll
        for (int c = 0; c < r; ++c) s = s - T[(size_t)r * ldt + c] * x[c];
        if (!UNIT) s = s / T[(size_t)r * ldt + r];
        x[r] = s;
      }
    }
  } else {
#pragma unroll
    for (int r = kRows - 1; r >= 0; --r) {
      if (r < nr) {
        double s = x[r];
#pragma unroll
        for (int c = r + 1; c < kRows; ++c)
          if (c < nr) s = s - T[(size_t)r * ldt + c] * x[c];
        if (!UNIT) s = s / T[(size_t)r * ldt + r];
        x[r] = s;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < kRows; ++r)
    if (r < nr) B[(size_t)r * ldb + col] = x[r];
}

hipError_t solve_block(hipStream_t s, bool lower, bool unit, int nr, int ncols, const double* T, int ldt,
                       double* B, int ldb) {
  const dim3 grid((ncols + 255) / 256), block(256);
  if (lower && unit) hipLaunchKernelGGL((k_trsm_block<true, true>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb);
  else if (lower) hipLaunchKernelGGL((k_trsm_block<true, false>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb);
  else if (unit) hipLaunchKernelGGL((k_trsm_block<false, true>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb);
  else hipLaunchKernelGGL((k_trsm_block<false, false>), grid, block, 0, s, nr, ncols, T, ldt, B, ldb);
  return hipGetLastError();
}

}  // namespace

hipError_t trsm_left(hipStream_t s, bool lower, bool unit, int nr, int ncols, const double* T, int ldt,
                     double* B, int ldb) {
  if (nr <= 0 || ncols <= 0) return hipSuccess;
  hipError_t e = hipSuccess;
  if (lower) {
    for (int r0 = 0; r0 < nr; r0 += kRows) {
      const int rb = nr - r0 < kRows ? nr - r0 : kRows;
      e = solve_block(s, true, unit, rb, ncols, T + (size_t)r0 * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb);
      if (e != hipSuccess) return e;
      const int rest = nr - r0 - rb;
      if (rest > 0) {
        e = gemm_update(s, rest, ncols, rb, T + (size_t)(r0 + rb) * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb,
                        B + (size_t)(r0 + rb) * ldb, ldb);
        if (e != hipSuccess) return e;
      }
    }
  } else {
    for (int r1 = nr; r1 > 0; r1 -= kRows) {
      const int r0 = r1 - kRows > 0 ? r1 - kRows : 0;
      e = solve_block(s, false, unit, r1 - r0, ncols, T + (size_t)r0 * ldt + r0, ldt, B + (size_t)r0 * ldb, ldb);
      if (e != hipSuccess) return e;
      if (r0 > 0) {
        e = gemm_update(s, r0, ncols, r1 - r0, T + r0, ldt, B + (size_t)r0 * ldb, ldb, B, ldb);
        if (e != hipSuccess) return e;
      }
    }
  }
  return e;
}

}  // namespace mlu
