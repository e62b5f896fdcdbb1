// Internal declarations shared by the HIP sources of libmlu (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace mlu {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kWave = 64;

// ---------------------------------------------------------------- panel kernel
// Widest register-resident panel block and the largest number of cooperating
// workgroups of one panel launch.
constexpr int kPanelMaxCols = 32;
constexpr int kPanelThreads = 256;
constexpr int kPanelMaxWG = 128;

// Cross-workgroup barrier state (device memory, zero at the start of a call).
struct alignas(64) GridBar {
  unsigned count;
  unsigned gen;
  unsigned err;
  unsigned pad[13];
};

// One candidate published by a workgroup for the pivot of a column:
// |value|, the relative row, the origin label of the row's contents and the
// row's values in the block's columns.
struct PanelSlot {
  double absval;
  long long row;
  long long pad;
  double vals[kPanelMaxCols];
};

struct PanelWork {
  GridBar bar;
  PanelSlot slot[2][kPanelMaxWG];
  PanelSlot diag[2];
};

size_t workspace_bytes();

// ---------------------------------------------------------------- launchers
// All take row-major operands; element (i, j) of X is X[i*ldx + j].

// C := C - A B   (A m x k, B k x n, C m x n)
hipError_t gemm_update(hipStream_t s, int m, int n, int k, const double* A, int lda,
                       const double* B, int ldb, double* C, int ldc);

// Factor the m x bw block whose top-left entry is global diagonal entry
// (row0, row0): partial pivoting over its rows, interchanges applied inside the
// block only; ipiv[row0 + c] = row0 + p + 1 (1-based); a zero pivot sets
// *info = row0 + c + 1 if *info was 0.
hipError_t panel_factor(hipStream_t s, double* A, int lda, int m, int bw, int row0,
                        int32_t* ipiv, int32_t* info, PanelWork* work);

// Apply interchanges ipiv[k1 .. k2) (1-based values, each >= its own index and
// < m) to columns [ca0, ca1) and [cb0, cb1) of the m-row matrix A.
hipError_t laswp(hipStream_t s, double* A, int lda, int m, int k1, int k2,
                 const int32_t* ipiv, int ca0, int ca1, int cb0, int cb1, int32_t* info);

// B := T^{-1} B with T (nr x nr) lower/upper, unit/non-unit, B nr x ncols.
hipError_t trsm_left(hipStream_t s, bool lower, bool unit, int nr, int ncols,
                     const double* T, int ldt, double* B, int ldb);

hipError_t zero_bytes(hipStream_t s, void* p, size_t bytes);

}  // namespace mlu
