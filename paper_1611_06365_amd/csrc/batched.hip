// Batched LU with partial pivoting of many independent matrices of different
// orders in one persistent launch (the method of Section 3 applied to each
// operand: blocked right-looking, Fig. "LU", with the panel factored
// unblocked, Fig. "LU" left).
//
// A device counting sort orders the matrices by decreasing order (the largest
// first, so that the launch's tail holds small ones); a persistent grid of
// 256-thread workgroups takes matrices from an atomic queue in that order.
// One workgroup factors one matrix at a time, kNB columns per step:
//   1. the (n - j) x kNB panel is loaded into LDS and factored there with
//      partial pivoting (argmax by wave reduction, first row on ties; the
//      swap, the scaling and the rank-1 update in LDS);
//   2. each thread owns columns outside the panel and applies the panel's
//      interchanges to them in order (no barrier needed);
//   3. A12 is staged into LDS 64 columns at a time, solved there with the
//      panel's unit lower triangle (A12 := trilu(A11)^-1 A12, one column per
//      thread), written back as U12, and the trailing matrix is updated with
//      the chunk, A22 -= A21 U12, 4 x 4 register tiles of FMAs with A21 read
//      from the LDS panel.  (FP64 vector and matrix peaks are equal on this part; the
//      operands are small and irregular, so the update stays on the VALU.)
// Matrices are row-major (element (i, j) at A[i*lda + j]), in place.
#include "mlu_internal.h"
#include "../../include/mlu.h"

#include <climits>
#include <mutex>

namespace mlu {
namespace {

constexpr int kBT = 256;           // threads per workgroup
constexpr int kNB = 32;            // panel width
constexpr int kNBp = kNB + 1;      // LDS pitch of the panel
constexpr int kUC = 64;            // A12 columns staged per chunk
constexpr int kMaxN = MLU_BATCH_MAX_N;

template <typename T>
struct BatchLds {
  T P[kMaxN * kNBp];       // the panel, rows 0 .. n-j-1
  T U[kNB * kUC];          // A12 chunk
  T wv[kBT / kWave];
  int wr[kBT / kWave];
  int piv[kNB];
  int p;
  int item;
};

template <typename T>
__device__ __forceinline__ void wave_argmax_t(T& v, int& r) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(v, off);
    const int orr = __shfl_xor(r, off);
    if (ov > v || (ov == v && orr < r)) {
      v = ov;
      r = orr;
    }
  }
}

template <typename T>
__device__ void factor_one(int n, T* __restrict__ A, int lda, int32_t* __restrict__ ipiv, int32_t* __restrict__ info,
                           BatchLds<T>& L) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int zero_col = INT_MAX;
  for (int j = 0; j < n; j += kNB) {
    const int nb = min(kNB, n - j), rows = n - j;
    // 1. panel -> LDS
    for (int e = tid; e < rows * kNB; e += kBT) {
      const int r = e / kNB, c = e % kNB;
      L.P[r * kNBp + c] = c < nb ? A[(size_t)(j + r) * lda + j + c] : T(0);
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      T bv = T(-1);
      int br = INT_MAX;
      for (int r = c + tid; r < rows; r += kBT) {
        const T a = fabs(L.P[r * kNBp + c]);
        if (a > bv) {   // rows visited in increasing order: the first maximum stays
          bv = a;
          br = r;
        }
      }
      wave_argmax_t(bv, br);
      if (lane == 0) {
        L.wv[wave] = bv;
        L.wr[wave] = br;
      }
      __syncthreads();
      if (tid == 0) {
        T v = L.wv[0];
        int r = L.wr[0];
        for (int w = 1; w < kBT / kWave; ++w)
          if (L.wv[w] > v || (L.wv[w] == v && L.wr[w] < r)) {
            v = L.wv[w];
            r = L.wr[w];
          }
        L.p = r;
        L.piv[c] = r;
      }
      __syncthreads();
      const int p = L.p;
      if (p != c && tid < nb) {
        const T t = L.P[c * kNBp + tid];
        L.P[c * kNBp + tid] = L.P[p * kNBp + tid];
        L.P[p * kNBp + tid] = t;
      }
      __syncthreads();
      const T pv = L.P[c * kNBp + c];
      if (pv == T(0)) {
        if (j + c < zero_col) zero_col = j + c;   // same value in every thread
      } else {
        for (int r = c + 1 + tid; r < rows; r += kBT) {
          const T l = L.P[r * kNBp + c] / pv;
          L.P[r * kNBp + c] = l;
          for (int cc = c + 1; cc < nb; ++cc) L.P[r * kNBp + cc] -= l * L.P[c * kNBp + cc];
        }
      }
      __syncthreads();
    }
    // panel -> global, interchanges recorded
    for (int e = tid; e < rows * kNB; e += kBT) {
      const int r = e / kNB, c = e % kNB;
      if (c < nb) A[(size_t)(j + r) * lda + j + c] = L.P[r * kNBp + c];
    }
    if (tid < nb) ipiv[j + tid] = j + L.piv[tid] + 1;
    // 2. columns outside the panel: the panel's interchanges, in order (a
    //    thread owns its columns, so no barrier between the swaps)
    for (int col = tid; col < n - nb; col += kBT) {
      const int g = col < j ? col : col + nb;
      for (int c = 0; c < nb; ++c) {
        const int p = L.piv[c];
        if (p != c) {
          T* a = A + (size_t)(j + c) * lda + g;
          T* b = A + (size_t)(j + p) * lda + g;
          const T t = *a;
          *a = *b;
          *b = t;
        }
      }
    }
    __syncthreads();   // global writes visible inside the workgroup
    // 3. per chunk of kUC right columns: A12 -> LDS, A12 := trilu(A11)^-1 A12
    //    (one column per thread, in LDS), back to global as U12, then
    //    A22 -= A21 U12 with the chunk
    const int R = rows - nb;
    for (int c0 = 0; c0 < R; c0 += kUC) {
      const int cw = min(kUC, R - c0);
      for (int e = tid; e < kNB * kUC; e += kBT) {
        const int k = e / kUC, c = e % kUC;
        L.U[e] = (k < nb && c < cw) ? A[(size_t)(j + k) * lda + j + nb + c0 + c] : T(0);
      }
      __syncthreads();
      if (tid < cw) {
        for (int r = 1; r < nb; ++r) {
          T v = L.U[r * kUC + tid];
          for (int q = 0; q < r; ++q) v -= L.P[r * kNBp + q] * L.U[q * kUC + tid];
          L.U[r * kUC + tid] = v;
        }
        for (int r = 1; r < nb; ++r) A[(size_t)(j + r) * lda + j + nb + c0 + tid] = L.U[r * kUC + tid];
      }
      __syncthreads();
      const int tr = (R + 3) / 4, tc = (cw + 3) / 4;
      for (int t = tid; t < tr * tc; t += kBT) {
        const int r0 = (t / tc) * 4, cc0 = (t % tc) * 4;
        T acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q) acc[i][q] = T(0);
        for (int k = 0; k < nb; ++k) {
          T a[4], b[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = (r0 + i < R) ? L.P[(nb + r0 + i) * kNBp + k] : T(0);
#pragma unroll
          for (int q = 0; q < 4; ++q) b[q] = L.U[k * kUC + cc0 + q];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[i][q] += a[i] * b[q];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (r0 + i < R && cc0 + q < cw) {
              T* cp = A + (size_t)(j + nb + r0 + i) * lda + j + nb + c0 + cc0 + q;
              *cp -= acc[i][q];
            }
      }
      __syncthreads();
    }
  }
  if (tid == 0) *info = zero_col == INT_MAX ? 0 : zero_col + 1;
}

// order[] := matrix indices by decreasing order n (counting sort, one
// workgroup); entries with an invalid order are placed last.
__global__ __launch_bounds__(1024) void k_batch_order(int batch, const int32_t* __restrict__ d_n, int max_n,
                                                      int32_t* __restrict__ order, unsigned* __restrict__ queue) {
  __shared__ int cnt[kMaxN + 2];
  const int tid = threadIdx.x;
  for (int b = tid; b < kMaxN + 2; b += blockDim.x) cnt[b] = 0;
  if (tid == 0) *queue = 0u;
  __syncthreads();
  auto bucket = [&](int i) {
    const int n = d_n[i];
    return (n < 0 || n > max_n) ? kMaxN + 1 : kMaxN - n;   // larger n -> smaller bucket
  };
  for (int i = tid; i < batch; i += blockDim.x) atomicAdd(&cnt[bucket(i)], 1);
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int b = 0; b < kMaxN + 2; ++b) {
      const int c = cnt[b];
      cnt[b] = s;
      s += c;
    }
  }
  __syncthreads();
  for (int i = tid; i < batch; i += blockDim.x) order[atomicAdd(&cnt[bucket(i)], 1)] = i;
}

template <typename T>
__global__ __launch_bounds__(kBT) void k_getrf_batched(int batch, const int32_t* __restrict__ d_n, T* const* d_A,
                                                       const int32_t* __restrict__ d_lda, int32_t* const* d_ipiv,
                                                       int32_t* __restrict__ d_info, int max_n,
                                                       const int32_t* __restrict__ order, unsigned* queue) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  BatchLds<T>& L = *reinterpret_cast<BatchLds<T>*>(smem);
  while (true) {
    if (threadIdx.x == 0) {
      const unsigned t = atomicAdd(queue, 1u);
      L.item = t < (unsigned)batch ? order[t] : -1;
    }
    __syncthreads();
    // the item and the matrix's order are the same in every thread: make them
    // scalar, so that the compiler sees every branch below as uniform (all
    // paths then reach the same barriers, and the next fetch)
    const int i = __builtin_amdgcn_readfirstlane(L.item);
    __syncthreads();
    if (i < 0) break;
    const int n = __builtin_amdgcn_readfirstlane(d_n[i]);
    const int lda = __builtin_amdgcn_readfirstlane(d_lda[i]);
    const bool bad = n < 0 || n > max_n || lda < (n > 1 ? n : 1);
    if (bad || n == 0) {
      if (threadIdx.x == 0) d_info[i] = bad ? -1 : 0;
    } else {
      factor_one<T>(n, d_A[i], lda, d_ipiv[i], &d_info[i], L);
    }
    __syncthreads();
  }
}

template <typename T>
int launch_batched(void* stream, int batch, const int32_t* d_n, T* const* d_A, const int32_t* d_lda,
                   int32_t* const* d_ipiv, int32_t* d_info, int max_n, void* d_work, size_t work_bytes) {
  if (batch < 0) return -2;
  if (batch > 0 && !d_n) return -3;
  if (batch > 0 && !d_A) return -4;
  if (batch > 0 && !d_lda) return -5;
  if (batch > 0 && !d_ipiv) return -6;
  if (batch > 0 && !d_info) return -7;
  if (max_n < 0 || max_n > kMaxN) return -8;
  if (!d_work) return -9;
  if (work_bytes < batched_workspace_bytes(batch)) return -10;
  if (batch == 0) return 0;
  if (batched_set_lds_limits() != hipSuccess) return MLU_ERR_HIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  unsigned* queue = reinterpret_cast<unsigned*>(d_work);
  int32_t* order = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_work) + 256);
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, batch, d_n, max_n, order, queue);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MLU_ERR_HIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return MLU_ERR_HIP;
  const size_t lds = sizeof(BatchLds<T>);
  const int per_cu = (int)((160u * 1024u) / lds) >= 2 ? 2 : 1;
  const int grid = cus * per_cu < batch ? cus * per_cu : batch;
  hipLaunchKernelGGL((k_getrf_batched<T>), dim3(grid), dim3(kBT), lds, s, batch, d_n, d_A, d_lda, d_ipiv, d_info,
                     max_n, order, queue);
  return hipGetLastError() == hipSuccess ? 0 : MLU_ERR_HIP;
}

}  // namespace

size_t batched_workspace_bytes(int batch) { return 256 + (size_t)(batch > 0 ? batch : 0) * sizeof(int32_t); }

// Raises the kernels' dynamic-LDS limit above the default once per process
// (the device's own limit is 160 KB per workgroup), so that a later call can
// be captured in a stream graph without any non-stream API in between.
hipError_t batched_set_lds_limits() {
  static std::mutex mu;
  static bool done = false;
  std::lock_guard<std::mutex> lk(mu);
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrf_batched<double>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(BatchLds<double>));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_getrf_batched<float>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(BatchLds<float>));
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace mlu

using namespace mlu;

extern "C" {

int mlu_getrf_batched_workspace(int batch, size_t* bytes) {
  if (batch < 0) return -1;
  if (!bytes) return -2;
  *bytes = batched_workspace_bytes(batch);
  return 0;
}

int mlu_dgetrf_batched(void* stream, int batch, const int32_t* d_n, double* const* d_A, const int32_t* d_lda,
                       int32_t* const* d_ipiv, int32_t* d_info, int max_n, void* d_work, size_t work_bytes) {
  return launch_batched<double>(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, d_work, work_bytes);
}

int mlu_sgetrf_batched(void* stream, int batch, const int32_t* d_n, float* const* d_A, const int32_t* d_lda,
                       int32_t* const* d_ipiv, int32_t* d_info, int max_n, void* d_work, size_t work_bytes) {
  return launch_batched<float>(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, d_work, work_bytes);
}

}  // extern "C"
