// Row interchanges (the "row permutations" applied after each panel
// factorization, Section 3.1 trace discussion; LAPACK's laswp).
//
// Storage is row-major, so interchanging two rows moves contiguous runs of
// memory.  The interchanges ipiv[k1..k2) are sequential: step c swaps rows c
// and ipiv[c]-1.  Instead of replaying them one by one per column, every
// workgroup first composes them (in LDS) into one permutation of the rows they
// touch -- the block rows k1..k2-1 and the distinct "far" pivot rows -- and then
// moves each displaced row segment exactly once: all sources of its column
// chunk are read into LDS, then written to their destinations.
#include "mlu_internal.h"

namespace mlu {
namespace {

constexpr int kMaxSteps = 256;   // interchanges per launch
constexpr int kCols = 16;        // columns per workgroup
constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void k_laswp(double* __restrict__ A, int lda, int m, int k1, int k2,
                                                    const int32_t* __restrict__ ipiv, int ca0, int ca1,
                                                    int cb0, int cb1, int32_t* __restrict__ info, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;   // a flag the caller raised on the device
  __shared__ int s_piv[kMaxSteps];
  __shared__ int s_slot[kMaxSteps];
  __shared__ int s_label[2 * kMaxSteps];
  __shared__ int s_row[2 * kMaxSteps];
  __shared__ double s_buf[2 * kMaxSteps][kCols];
  __shared__ int s_any;

  const int tid = threadIdx.x;
  const int nst = k2 - k1;
  if (tid == 0) s_any = 0;
  for (int c = tid; c < nst; c += kThreads) {
    int p = ipiv[k1 + c] - 1;
    if (p < k1 + c || p >= m) {  // not a valid partial-pivoting interchange
      if (info) atomicExch(info, -998);
      p = k1 + c;
    }
    s_piv[c] = p;
  }
  for (int s = tid; s < 2 * nst; s += kThreads) {
    s_label[s] = s;
    s_row[s] = s < nst ? k1 + s : -1;
  }
  __syncthreads();
  // slot of each step's partner row: a block row is its own slot; a far row gets
  // the slot of the first step that names it
  for (int c = tid; c < nst; c += kThreads) {
    const int p = s_piv[c];
    int slot;
    if (p < k2) {
      slot = p - k1;
    } else {
      int first = c;
      for (int q = 0; q < c; ++q)
        if (s_piv[q] == p) {
          first = q;
          break;
        }
      slot = nst + first;
      if (first == c) s_row[nst + c] = p;
    }
    s_slot[c] = slot;
    if (p != k1 + c) s_any = 1;
  }
  __syncthreads();
  if (!s_any) return;  // every interchange is the identity
  if (tid == 0) {
    for (int c = 0; c < nst; ++c) {
      const int t = s_label[c];
      s_label[c] = s_label[s_slot[c]];
      s_label[s_slot[c]] = t;
    }
  }
  __syncthreads();

  // this workgroup's columns
  const int na = ca1 - ca0, ntot = na + (cb1 - cb0);
  const int g = blockIdx.x * kCols + (tid % kCols);
  const bool colok = g < ntot;
  const int col = g < na ? ca0 + g : cb0 + (g - na);
  const int e0 = tid / kCols, estep = kThreads / kCols;

  // every slot is read, from a clamped row and column (an unused slot's LDS
  // entry is never written back), all of this thread's loads first, so they
  // do not wait for one another
  const int colc = colok ? col : (na > 0 ? ca0 : cb0);
  constexpr int kPer = 2 * kMaxSteps / (kThreads / kCols);   // slots per thread, at most
  double v[kPer];
#pragma unroll
  for (int t = 0; t < kPer; ++t) {
    const int sl = min(e0 + t * estep, 2 * nst - 1);
    v[t] = A[(size_t)max(s_row[s_label[sl]], 0) * lda + colc];
  }
#pragma unroll
  for (int t = 0; t < kPer; ++t)
    if (e0 + t * estep < 2 * nst) s_buf[e0 + t * estep][tid % kCols] = v[t];
  __syncthreads();
  for (int s = e0; s < 2 * nst; s += estep) {
    const int src = s_label[s];
    if (s_row[s] >= 0 && src != s && colok) A[(size_t)s_row[s] * lda + col] = s_buf[s][tid % kCols];
  }
}

}  // namespace

hipError_t laswp(hipStream_t s, double* A, int lda, int m, int k1, int k2, const int32_t* ipiv, int ca0,
                 int ca1, int cb0, int cb1, int32_t* info, const int32_t* skip) {
  if (ca1 < ca0) ca1 = ca0;
  if (cb1 < cb0) cb1 = cb0;
  const int ntot = (ca1 - ca0) + (cb1 - cb0);
  if (ntot <= 0 || k2 <= k1) return hipSuccess;
  const unsigned grid = (unsigned)((ntot + kCols - 1) / kCols);
  for (int a = k1; a < k2; a += kMaxSteps) {
    const int b = (k2 - a) < kMaxSteps ? k2 : a + kMaxSteps;
    hipLaunchKernelGGL(k_laswp, dim3(grid), dim3(kThreads), 0, s, A, lda, m, a, b, ipiv, ca0, ca1, cb0, cb1,
                       info, skip);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mlu
