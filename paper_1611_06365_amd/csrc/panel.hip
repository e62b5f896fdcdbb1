// Panel factorization with partial pivoting (LU_unb of Fig. "LU", left, applied
// to a block of at most 32 columns: the diagonal-block step RL1 / PF3 / LL3).
//
// The m x bw block is held in registers across nwg cooperating workgroups of
// 512 threads; thread t of workgroup w owns rows w*1024 + t + 512*k (k < R).
// Per column c:
//   1. each thread finds its best candidate |a(r, c)|, r >= c (first row on
//      ties); a wave64 shuffle reduction and an LDS pass give the workgroup's;
//   2. with nwg > 1, every workgroup publishes its candidate (value, row and the
//      row's bw values) and workgroup 0 also publishes row c; one grid barrier;
//      every wave then reduces the published candidates itself;
//   3. rows c and p are exchanged (inside the block only), a21 := a21 / alpha11
//      (a true division, zero pivots skipped and reported), and the rank-1
//      update a22 := a22 - a21 a12^T runs on the owned rows.
// One grid barrier per column is the whole cross-workgroup cost; the barrier is
// a generation counter in device memory with agent-scope acquire/release and a
// bounded wait (a timeout flags the call instead of hanging).
#include "mlu_internal.h"

#include <climits>
#include <type_traits>
#include <utility>

namespace mlu {
namespace {

constexpr int PT = 1024;  // rows per workgroup at R = 2
constexpr int NT = 512;   // threads per workgroup
constexpr int NWAVE = NT / kWave;
constexpr long long kSpinLimit = 1LL << 22;  // ~0.1 s of s_sleep(1) polls

__device__ __forceinline__ void st_relaxed(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p), (unsigned long long)__double_as_longlong(v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_relaxed(const double* p) {
  unsigned long long x = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)x);
}
__device__ __forceinline__ void st_relaxed_i(long long* p, long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_relaxed_i(const long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier over the nwg co-resident workgroups of this launch.
__device__ void grid_barrier(GridBar* bar, unsigned nwg, int32_t* info) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned g = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nwg - 1) {
      __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&bar->gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kSpinLimit) {
          __hip_atomic_store(&bar->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicExch(info, -999);
          break;
        }
      }
    }
  }
  __syncthreads();
}

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ bool better(double av, long long ar, double bv, long long br) {
  return av > bv || (av == bv && ar < br);
}

template <int BW, int R>
__global__ __launch_bounds__(NT) void k_panel(double* __restrict__ A, int lda, int m, int bw, int row0,
                                              int32_t* __restrict__ ipiv, int32_t* __restrict__ info,
                                              PanelWork* __restrict__ work, int nwg) {
  __shared__ double s_val[NWAVE];
  __shared__ long long s_row[NWAVE];
  __shared__ double s_prow[BW];
  __shared__ double s_drow[BW];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wg = blockIdx.x;
  const int base = wg * NT * R;

  double v[R][BW];
  int rows[R];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    rows[k] = base + tid + k * NT;
    const bool ok = rows[k] < m;
    const double* src = A + (size_t)(ok ? rows[k] : 0) * lda;
#pragma unroll
    for (int c = 0; c < BW; ++c) v[k][c] = (ok && c < bw) ? src[c] : 0.0;
  }

  // Columns are visited through a compile-time index so that v[k][c] stays in
  // registers (a runtime column index would send the array to scratch).
  static_for<BW>([&](auto cidx) {
    constexpr int c = decltype(cidx)::value;
    if (c < bw) {
    // 1. candidate of this thread, wave and workgroup
    double bv = -1.0;
    long long br = LLONG_MAX;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int r = rows[k];
      if (r < m && r >= c) {
        const double a = fabs(v[k][c]);
        if (a > bv) {
          bv = a;
          br = r;
        }
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ov = __shfl_xor(bv, off);
      const long long orr = __shfl_xor(br, off);
      if (better(ov, orr, bv, br)) {
        bv = ov;
        br = orr;
      }
    }
    if (lane == 0) {
      s_val[wave] = bv;
      s_row[wave] = br;
    }
    __syncthreads();
    bv = s_val[0];
    br = s_row[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w)
      if (better(s_val[w], s_row[w], bv, br)) {
        bv = s_val[w];
        br = s_row[w];
      }

    long long p;
    if (nwg > 1) {
      PanelSlot* mine = &work->slot[c & 1][wg];
      bool owner = false;
#pragma unroll
      for (int k = 0; k < R; ++k)
        if ((long long)rows[k] == br) {
          owner = true;
#pragma unroll
          for (int cc = 0; cc < BW; ++cc) st_relaxed(&mine->vals[cc], v[k][cc]);
        }
      if (owner || (br == LLONG_MAX && tid == 0)) {
        st_relaxed(&mine->absval, bv);
        st_relaxed_i(&mine->row, br);
        __threadfence();
      }
#pragma unroll
      for (int k = 0; k < R; ++k)
        if (rows[k] == c) {
#pragma unroll
          for (int cc = 0; cc < BW; ++cc) st_relaxed(&work->diag[c & 1].vals[cc], v[k][cc]);
          __threadfence();
        }
      grid_barrier(&work->bar, (unsigned)nwg, info);
      // every wave reduces the published candidates on its own
      double gv = -1.0;
      long long gr = LLONG_MAX;
      int gw = 0;
      for (int w = lane; w < nwg; w += kWave) {
        const PanelSlot* sl = &work->slot[c & 1][w];
        const double sv = ld_relaxed(&sl->absval);
        const long long sr = ld_relaxed_i(&sl->row);
        if (better(sv, sr, gv, gr)) {
          gv = sv;
          gr = sr;
          gw = w;
        }
      }
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(gv, off);
        const long long orr = __shfl_xor(gr, off);
        const int ow = __shfl_xor(gw, off);
        if (better(ov, orr, gv, gr)) {
          gv = ov;
          gr = orr;
          gw = ow;
        }
      }
      p = gr;
      if (tid < BW) {
        s_prow[tid] = ld_relaxed(&work->slot[c & 1][gw].vals[tid]);
        s_drow[tid] = ld_relaxed(&work->diag[c & 1].vals[tid]);
      }
    } else {
      p = br;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        if ((long long)rows[k] == p) {
#pragma unroll
          for (int cc = 0; cc < BW; ++cc) s_prow[cc] = v[k][cc];
        }
        if (rows[k] == c) {
#pragma unroll
          for (int cc = 0; cc < BW; ++cc) s_drow[cc] = v[k][cc];
        }
      }
    }
    __syncthreads();

    // 3. interchange rows c and p, scale, rank-1 update
    const double piv = s_prow[c];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int r = rows[k];
      if (r == c) {
#pragma unroll
        for (int cc = 0; cc < BW; ++cc) v[k][cc] = s_prow[cc];
      } else if ((long long)r == p) {
#pragma unroll
        for (int cc = 0; cc < BW; ++cc) v[k][cc] = s_drow[cc];
      }
      if (r > c && r < m) {
        double l = v[k][c];
        if (piv != 0.0) {
          l = l / piv;
          v[k][c] = l;
        }
#pragma unroll
        for (int cc = c + 1; cc < BW; ++cc)
          if (cc < bw) v[k][cc] = v[k][cc] - l * s_prow[cc];
      }
    }
    if (wg == 0 && tid == 0) {
      ipiv[c] = row0 + (int)p + 1;
      if (piv == 0.0) atomicCAS(info, 0, row0 + c + 1);
    }
    }  // c < bw
  });

#pragma unroll
  for (int k = 0; k < R; ++k) {
    if (rows[k] < m) {
      double* dst = A + (size_t)rows[k] * lda;
#pragma unroll
      for (int c = 0; c < BW; ++c)
        if (c < bw) dst[c] = v[k][c];
    }
  }
}

template <int BW>
hipError_t launch_panel(hipStream_t s, double* A, int lda, int m, int bw, int row0, int32_t* ipiv,
                        int32_t* info, PanelWork* work) {
  if (m <= NT) {
    hipLaunchKernelGGL((k_panel<BW, 1>), dim3(1), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv, info, work, 1);
  } else {
    const int nwg = (m + PT - 1) / PT;
    if (nwg > kPanelMaxWG) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_panel<BW, 2>), dim3(nwg), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv, info, work,
                       nwg);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t panel_factor(hipStream_t s, double* A, int lda, int m, int bw, int row0, int32_t* ipiv,
                        int32_t* info, PanelWork* work) {
  if (m <= 0 || bw <= 0) return hipSuccess;
  if (bw > kPanelMaxCols || bw > m) return hipErrorInvalidValue;
  ipiv += row0;
  if (bw <= 8) return launch_panel<8>(s, A, lda, m, bw, row0, ipiv, info, work);
  if (bw <= 16) return launch_panel<16>(s, A, lda, m, bw, row0, ipiv, info, work);
  return launch_panel<32>(s, A, lda, m, bw, row0, ipiv, info, work);
}

size_t workspace_bytes() { return (sizeof(PanelWork) + 4095) / 4096 * 4096; }

}  // namespace mlu
