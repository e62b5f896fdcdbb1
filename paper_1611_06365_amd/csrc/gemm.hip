// Trailing update C := C - A B on FP64 matrix cores (gfx950).
//
// This is the GEMM-shaped step of every variant: RL3 / PF2 / RU2 of the
// right-looking algorithms and LL2 of the left-looking one (Fig. "LU",
// Fig. "LU_la_blk", Section 4.2); it carries nearly all of the 2n^3/3 flops.
//
// Design (row-major operands, element (i, j) of X at X[i*ldx + j]):
//  * 128 x 128 C tile per 256-thread workgroup; four wave64s in a 2 x 2 grid,
//    each owning 64 x 64 of C as 4 x 4 blocks of v_mfma_f64_16x16x4_f64.
//  * K advances in stages of 16 through double-buffered LDS: the A tile is
//    kept [i][k] and the B tile [k][j], both straight copies of the row-major
//    source so global loads stay contiguous 64-byte runs per thread.
//  * Inside a stage, MFMA step s (0..3) feeds lane group q = lane/16 with
//    k = 4q + s.  A and B use the same k mapping, so every k is summed exactly
//    once.  Each step's eight fragments are read from LDS one step ahead
//    (two register sets), which keeps the kernel at 2 waves/SIMD unspilled.
//  * The accumulators start as the C tile and B is negated as it is staged
//    into LDS, so the MFMAs accumulate C - A B directly and the epilogue is a
//    plain store: C is read once, ahead of the main loop, instead of after it.
//  * Next stage's global loads are issued before the current stage's MFMAs.
//  * Workgroup -> tile mapping is XCD-aware: hardware deals workgroups to the
//    eight XCDs round-robin, so consecutive logical tiles are given to one XCD,
//    and logical tiles walk 8-tile-row groups so an XCD's L2 sees few A and B
//    panels at a time.
#include "mlu_internal.h"

#include <hip/hip_bf16.h>

#include <mutex>
#include <vector>

namespace mlu {
namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int LDS_A = BK + 2;    // 144-byte row pitch: 16-byte reads of 8 lanes hit distinct banks
constexpr int LDS_B = BN + 4;    // row pitch offset so lane groups q, q+1 use different banks
constexpr int GROUP_M = 8;

// Logical tile t -> (tile row, tile column): tiles walk groups of GROUP_M tile
// rows column by column, so neighbouring t share A rows and B columns.
__device__ __forceinline__ void group_coords(int t, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int per_group = GROUP_M * tiles_n;
  const int group = t / per_group;
  const int first_m = group * GROUP_M;
  const int gsz = min(tiles_m - first_m, GROUP_M);
  const int within = t - group * per_group;
  tm = first_m + within % gsz;
  tn = within / gsz;
}

// Workgroup -> tile for one-tile-per-workgroup launches: workgroups are dealt
// to the XCDs round-robin, so XCD x (= wg mod 8) gets the contiguous logical
// range starting at x * T/8.
__device__ __forceinline__ void tile_coords(int wg, int tiles_m, int tiles_n, int& tm, int& tn) {
  const int T = tiles_m * tiles_n;
  const int nfull = (T / 8) * 8;
  int t = wg;
  if (wg < nfull) t = (wg & 7) * (nfull >> 3) + (wg >> 3);
  group_coords(t, tiles_m, tiles_n, tm, tn);
}

__device__ __forceinline__ unsigned hw_xcc_id() { return __builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & 7u; }
__device__ __forceinline__ unsigned hw_cu_id() { return (__builtin_amdgcn_s_getreg(4 | (0 << 6) | (31 << 11)) >> 8) & 15u; }

// The tile's LDS stages; a kernel that runs several tile loops gives them the
// same one.
struct TileLds {
  double As[2][BM * LDS_A];
  double Bs[2][BK * LDS_B];
};

// One 128 x 128 tile of C := C - A B.  Ends with a workgroup barrier, so the
// caller may start another tile at once.
// CLAMP selects the edge-tile form: unconditional loads from clamped addresses
// (the inner dimension masked as the stage goes to LDS; a C element outside
// the matrix is loaded from a clamped address and never stored), so edge
// loads stay in flight together; without it, edge loads are conditional, which
// keeps the registers of the general persistent kernel (k_gemm_queue) as they
// are.
template <bool VEC, bool CLAMP = false>
__device__ __forceinline__ void gemm_tile_in(TileLds& L, int tm, int tn, int m, int n, int k,
                                             const double* __restrict__ A, int lda, const double* __restrict__ B,
                                             int ldb, double* __restrict__ C, int ldc) {
  auto& As = L.As;
  auto& Bs = L.Bs;
  const int row0 = tm * BM, col0 = tn * BN;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lq = lane >> 4;

  // global -> register staging: A tile row ar, 8 k's from ac; B tile row br, 8 j's from bc
  const int ar = tid >> 1, ac = (tid & 1) * 8;
  const int br = tid >> 4, bc = (tid & 15) * 8;
  const bool interior_mn = (row0 + BM <= m) && (col0 + BN <= n);

  double ra[8], rb[8];
  auto gload = [&](int k0) {
    const bool full = VEC && interior_mn && (k0 + BK <= k);
    if (full) {
      const dbl2_g* pa = reinterpret_cast<const dbl2_g*>(A + (size_t)(row0 + ar) * lda + k0 + ac);
      const dbl2_g* pb = reinterpret_cast<const dbl2_g*>(B + (size_t)(k0 + br) * ldb + col0 + bc);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        dbl2_g x = pa[e];
        ra[2 * e] = x.x;
        ra[2 * e + 1] = x.y;
        dbl2_g y = pb[e];
        rb[2 * e] = -y.x;
        rb[2 * e + 1] = -y.y;
      }
    } else if constexpr (CLAMP) {
      const int gr = min(row0 + ar, m - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = A[(size_t)gr * lda + min(k0 + ac + e, k - 1)];
      const int gk = min(k0 + br, k - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = -B[(size_t)gk * ldb + min(col0 + bc + e, n - 1)];
    } else {
      const int gr = row0 + ar;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gk = k0 + ac + e;
        ra[e] = (gr < m && gk < k) ? A[(size_t)gr * lda + gk] : 0.0;
      }
      const int gk = k0 + br;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int gc = col0 + bc + e;
        rb[e] = (gk < k && gc < n) ? -B[(size_t)gk * ldb + gc] : 0.0;
      }
    }
  };
  auto sstore = [&](int buf, int k0) {
    if constexpr (CLAMP) {
      if (!(VEC && interior_mn && k0 + BK <= k)) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (k0 + ac + e >= k) ra[e] = 0.0;
          if (k0 + br >= k) rb[e] = 0.0;
        }
      }
    }
    double* pa = &As[buf][ar * LDS_A + ac];
    double* pb = &Bs[buf][br * LDS_B + bc];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      *reinterpret_cast<double2*>(pa + e) = make_double2(ra[e], ra[e + 1]);
      *reinterpret_cast<double2*>(pb + e) = make_double2(rb[e], rb[e + 1]);
    }
  };

  // Accumulator layout of the 16x16 f64 block (measured on gfx950): lane
  // (li, lq) holds rows lq + 4*r (r = 0..3) of column li.
  v4d acc[4][4];
  double* const cbase = C + (size_t)(row0 + wm * 64 + lq) * ldc + col0 + wn * 64 + li;
  if (interior_mn) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = cbase[(size_t)(i * 16 + 4 * r) * ldc + j * 16];
  } else if constexpr (CLAMP) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(row0 + wm * 64 + i * 16 + lq + 4 * r, m - 1);
          const int col = min(col0 + wn * 64 + j * 16 + li, n - 1);
          acc[i][j][r] = C[(size_t)row * ldc + col];
        }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + wm * 64 + i * 16 + lq + 4 * r;
          const int col = col0 + wn * 64 + j * 16 + li;
          acc[i][j][r] = (row < m && col < n) ? cbase[(size_t)(i * 16 + 4 * r) * ldc + j * 16] : 0.0;
        }
  }

  const int nk = (k + BK - 1) / BK;
  gload(0);
  sstore(0, 0);
  __syncthreads();

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);

    double a[2][4], b[2][4];
    auto frag = [&](int st, int q) {
#pragma unroll
      for (int blk = 0; blk < 4; ++blk) {
        a[q][blk] = As[buf][(wm * 64 + blk * 16 + li) * LDS_A + 4 * lq + st];
        b[q][blk] = Bs[buf][(4 * lq + st) * LDS_B + wn * 64 + blk * 16 + li];
      }
    };
    frag(0, 0);
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      if (st + 1 < 4) frag(st + 1, (st + 1) & 1);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st & 1][i], b[st & 1][j], acc[i][j], 0, 0, 0);
    }

    if (kt + 1 < nk) sstore(buf ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  if (interior_mn) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) cbase[(size_t)(i * 16 + 4 * r) * ldc + j * 16] = acc[i][j][r];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + wm * 64 + i * 16 + lq + 4 * r;
          const int col = col0 + wn * 64 + j * 16 + li;
          if (row < m && col < n) cbase[(size_t)(i * 16 + 4 * r) * ldc + j * 16] = acc[i][j][r];
        }
  }
}

template <bool VEC, bool CLAMP = false>
__device__ __forceinline__ void gemm_tile(int tm, int tn, int m, int n, int k, const double* __restrict__ A,
                                          int lda, const double* __restrict__ B, int ldb,
                                          double* __restrict__ C, int ldc) {
  __shared__ TileLds L;
  gemm_tile_in<VEC, CLAMP>(L, tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
}

// The same 128 x 128 tile with the product in FP32: A and B are rounded to
// FP32 as they are staged into LDS, v_mfma_f32_16x16x4f32 accumulates in FP32
// over the whole inner dimension, and the epilogue subtracts the product from
// the FP64 C.  Used for the outer trailing updates of the mixed-precision
// factorization (the panel and its inner updates stay FP64).  Accumulator
// layout of the 16 x 16 f32 block (measured on gfx950): lane (li, lq) holds
// rows 4 lq + r (r = 0..3) of column li.
typedef float v4f __attribute__((ext_vector_type(4)));

// C -= acc for a 128 x 128 tile whose FP32 accumulators hold, in each 16 x 16
// block, rows rb + 16 i + r (r = 0..3) of column cb + 16 j: the C values of
// two 16-row blocks at a time (32 per lane) are loaded, from addresses clamped
// into C, before the first is used, so those loads are in flight together;
// out-of-range elements are not stored.  NT marks C's loads and stores
// non-temporal; the persistent queue (RU2) sets it: there C is read and
// written once per launch, and unmarked it streamed through the L2 and
// evicted the A and B panels that other tiles read again (LA at n = 16384:
// 2% faster with FP32 products, 4% with BF16).  The plain launches (RL3, PF2)
// leave it off: PF2's output is the next panel, read right after.
template <bool NT = false>
__device__ __forceinline__ void sub_acc_f32(const v4f (&acc)[4][4], double* __restrict__ C, int ldc, int m, int n,
                                            int rb, int cb) {
#pragma unroll
  for (int i0 = 0; i0 < 4; i0 += 2) {
    double cv[2][4][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if constexpr (NT) cv[i][j][r] = __builtin_nontemporal_load(&C[(size_t)min(rb + (i0 + i) * 16 + r, m - 1) * ldc + min(cb + j * 16, n - 1)]);
          else cv[i][j][r] = C[(size_t)min(rb + (i0 + i) * 16 + r, m - 1) * ldc + min(cb + j * 16, n - 1)];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb + (i0 + i) * 16 + r, col = cb + j * 16;
          if (row < m && col < n) {
            if constexpr (NT) __builtin_nontemporal_store(cv[i][j][r] - (double)acc[i0 + i][j][r], &C[(size_t)row * ldc + col]);
            else C[(size_t)row * ldc + col] = cv[i][j][r] - (double)acc[i0 + i][j][r];
          }
        }
  }
}
constexpr int LDSF_A = BK + 4;   // floats per A row in LDS
constexpr int LDSF_B = BN + 4;

template <bool VEC, bool NT = false>
__device__ __forceinline__ void gemm_tile_f32(int tm, int tn, int m, int n, int k, const double* __restrict__ A,
                                              int lda, const double* __restrict__ B, int ldb,
                                              double* __restrict__ C, int ldc) {
  __shared__ __attribute__((aligned(16))) float Asf[2][BM * LDSF_A];
  __shared__ __attribute__((aligned(16))) float Bsf[2][BK * LDSF_B];

  const int row0 = tm * BM, col0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int ar = tid >> 1, ac = (tid & 1) * 8;
  const int br = tid >> 4, bc = (tid & 15) * 8;
  const bool interior_mn = (row0 + BM <= m) && (col0 + BN <= n);

  double ra[8], rb[8];
  auto gload = [&](int k0) {
    const bool full = VEC && interior_mn && (k0 + BK <= k);
    if (full) {
      const dbl2_g* pa = reinterpret_cast<const dbl2_g*>(A + (size_t)(row0 + ar) * lda + k0 + ac);
      const dbl2_g* pb = reinterpret_cast<const dbl2_g*>(B + (size_t)(k0 + br) * ldb + col0 + bc);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        dbl2_g x = pa[e];
        ra[2 * e] = x.x;
        ra[2 * e + 1] = x.y;
        dbl2_g y = pb[e];
        rb[2 * e] = y.x;
        rb[2 * e + 1] = y.y;
      }
    } else {   // unconditional loads from clamped addresses; sstore masks the inner dimension
      const int gr = min(row0 + ar, m - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = A[(size_t)gr * lda + min(k0 + ac + e, k - 1)];
      const int gk = min(k0 + br, k - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = B[(size_t)gk * ldb + min(col0 + bc + e, n - 1)];
    }
  };
  auto kmask = [&](int k0) {
    if (!(VEC && interior_mn && k0 + BK <= k)) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (k0 + ac + e >= k) ra[e] = 0.0;
        if (k0 + br >= k) rb[e] = 0.0;
      }
    }
  };
  auto sstore = [&](int buf, int k0) {
    kmask(k0);
    float* pa = &Asf[buf][ar * LDSF_A + ac];
    float* pb = &Bsf[buf][br * LDSF_B + bc];
#pragma unroll
    for (int e = 0; e < 8; e += 4) {
      *reinterpret_cast<float4*>(pa + e) =
          make_float4((float)ra[e], (float)ra[e + 1], (float)ra[e + 2], (float)ra[e + 3]);
      *reinterpret_cast<float4*>(pb + e) =
          make_float4((float)rb[e], (float)rb[e + 1], (float)rb[e + 2], (float)rb[e + 3]);
    }
  };

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (k + BK - 1) / BK;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    float a[4][4], b[4][4];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const float4 a4 = *reinterpret_cast<const float4*>(&Asf[buf][(wm * 64 + blk * 16 + li) * LDSF_A + 4 * lq]);
      a[blk][0] = a4.x;
      a[blk][1] = a4.y;
      a[blk][2] = a4.z;
      a[blk][3] = a4.w;
      const float* pb = &Bsf[buf][(4 * lq) * LDSF_B + wn * 64 + blk * 16 + li];
#pragma unroll
      for (int st = 0; st < 4; ++st) b[blk][st] = pb[st * LDSF_B];
    }
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][st], b[j][st], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) sstore(buf ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  sub_acc_f32<NT>(acc, C, ldc, m, n, row0 + wm * 64 + 4 * lq, col0 + wn * 64 + li);
}

// A 64 x 64 tile of C := C - A B in FP64, for launches with too few 128 x 128
// tiles to fill the chip (the small trailing matrices at the end of a
// factorization, the panel's inner updates): four waves in a 2 x 2 grid, each
// owning 32 x 32 of C as 2 x 2 MFMA blocks; the K stages, the LDS double
// buffer, the negated B and the C-preloaded accumulators are as in gemm_tile.
constexpr int SBM = 64, SBN = 64;
constexpr int LDS_SB = SBN + 4;

template <bool VEC>
__device__ __forceinline__ void gemm_tile_small(int tm, int tn, int m, int n, int k, const double* __restrict__ A,
                                                int lda, const double* __restrict__ B, int ldb,
                                                double* __restrict__ C, int ldc) {
  __shared__ double As[2][SBM * LDS_A];
  __shared__ double Bs[2][BK * LDS_SB];

  const int row0 = tm * SBM, col0 = tn * SBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lq = lane >> 4;
  // global -> register staging: A row ar, 4 k's from ac; B row br, 4 j's from bc
  const int ar = tid >> 2, ac = (tid & 3) * 4;
  const int br = tid >> 4, bc = (tid & 15) * 4;
  const bool interior_mn = (row0 + SBM <= m) && (col0 + SBN <= n);

  double ra[4], rb[4];
  auto gload = [&](int k0) {
    const bool full = VEC && interior_mn && (k0 + BK <= k);
    if (full) {
      const dbl2_g* pa = reinterpret_cast<const dbl2_g*>(A + (size_t)(row0 + ar) * lda + k0 + ac);
      const dbl2_g* pb = reinterpret_cast<const dbl2_g*>(B + (size_t)(k0 + br) * ldb + col0 + bc);
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        const dbl2_g x = pa[e];
        ra[2 * e] = x.x;
        ra[2 * e + 1] = x.y;
        const dbl2_g y = pb[e];
        rb[2 * e] = -y.x;
        rb[2 * e + 1] = -y.y;
      }
    } else {   // unconditional loads from clamped addresses; sstore masks the inner dimension
      const int gr = min(row0 + ar, m - 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) ra[e] = A[(size_t)gr * lda + min(k0 + ac + e, k - 1)];
      const int gk = min(k0 + br, k - 1);
#pragma unroll
      for (int e = 0; e < 4; ++e) rb[e] = -B[(size_t)gk * ldb + min(col0 + bc + e, n - 1)];
    }
  };
  auto sstore = [&](int buf, int k0) {
    if (!(VEC && interior_mn && k0 + BK <= k)) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (k0 + ac + e >= k) ra[e] = 0.0;
        if (k0 + br >= k) rb[e] = 0.0;
      }
    }
    double* pa = &As[buf][ar * LDS_A + ac];
    double* pb = &Bs[buf][br * LDS_SB + bc];
#pragma unroll
    for (int e = 0; e < 4; e += 2) {
      *reinterpret_cast<double2*>(pa + e) = make_double2(ra[e], ra[e + 1]);
      *reinterpret_cast<double2*>(pb + e) = make_double2(rb[e], rb[e + 1]);
    }
  };

  // lane (li, lq) of a 16 x 16 f64 block holds rows lq + 4 r of column li
  v4d acc[2][2];
  double* const cbase = C + (size_t)(row0 + wm * 32 + lq) * ldc + col0 + wn * 32 + li;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {   // clamped: an accumulator outside C is never stored
        const int row = min(row0 + wm * 32 + i * 16 + lq + 4 * r, m - 1);
        const int col = min(col0 + wn * 32 + j * 16 + li, n - 1);
        acc[i][j][r] = C[(size_t)row * ldc + col];
      }

  const int nk = (k + BK - 1) / BK;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      double a[2], b[2];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        a[blk] = As[buf][(wm * 32 + blk * 16 + li) * LDS_A + 4 * lq + st];
        b[blk] = Bs[buf][(4 * lq + st) * LDS_SB + wn * 32 + blk * 16 + li];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(buf ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row0 + wm * 32 + i * 16 + lq + 4 * r;
        const int col = col0 + wn * 32 + j * 16 + li;
        if (interior_mn || (row < m && col < n)) cbase[(size_t)(i * 16 + 4 * r) * ldc + j * 16] = acc[i][j][r];
      }
}

// The same 128 x 128 tile with BF16 operands and FP32 accumulation: A and B
// are rounded to BF16 as they are staged into LDS (through FP32, round to
// nearest even), v_mfma_f32_16x16x16bf16_1k takes one 16-deep K stage per
// MFMA, and the epilogue subtracts the FP32 product from the FP64 C.  B is kept
// transposed in LDS so that each lane's four K values are contiguous.  Lane
// layout (checked on gfx950): A element (i, k) from lane i + 16 q, slot s with
// k = 4 q + s; B element (k, j) from lane j + 16 q, slot s; D rows 4 q + r of
// column j in lane j + 16 q.
typedef short v4bf __attribute__((ext_vector_type(4)));
constexpr int LDSH_A = BK + 8;   // bf16 per A row in LDS (48 bytes)
constexpr int LDSH_B = BK + 8;   // bf16 per transposed-B row in LDS

__device__ __forceinline__ unsigned short to_bf16(double x) {
  const __hip_bfloat16 h = __float2bfloat16((float)x);
  return *reinterpret_cast<const unsigned short*>(&h);
}

template <bool VEC, bool NT = false>
__device__ __forceinline__ void gemm_tile_bf16(int tm, int tn, int m, int n, int k, const double* __restrict__ A,
                                               int lda, const double* __restrict__ B, int ldb,
                                               double* __restrict__ C, int ldc) {
  __shared__ __attribute__((aligned(16))) unsigned short Ash[2][BM * LDSH_A];
  __shared__ __attribute__((aligned(16))) unsigned short Bth[2][BN * LDSH_B];

  const int row0 = tm * BM, col0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int ar = tid >> 1, ac = (tid & 1) * 8;
  const int br = tid >> 4, bc = (tid & 15) * 8;
  const bool interior_mn = (row0 + BM <= m) && (col0 + BN <= n);

  double ra[8], rb[8];
  auto gload = [&](int k0) {
    const bool full = VEC && interior_mn && (k0 + BK <= k);
    if (full) {
      const dbl2_g* pa = reinterpret_cast<const dbl2_g*>(A + (size_t)(row0 + ar) * lda + k0 + ac);
      const dbl2_g* pb = reinterpret_cast<const dbl2_g*>(B + (size_t)(k0 + br) * ldb + col0 + bc);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const dbl2_g x = pa[e];
        ra[2 * e] = x.x;
        ra[2 * e + 1] = x.y;
        const dbl2_g y = pb[e];
        rb[2 * e] = y.x;
        rb[2 * e + 1] = y.y;
      }
    } else {   // unconditional loads from clamped addresses; sstore masks the inner dimension
      const int gr = min(row0 + ar, m - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) ra[e] = A[(size_t)gr * lda + min(k0 + ac + e, k - 1)];
      const int gk = min(k0 + br, k - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) rb[e] = B[(size_t)gk * ldb + min(col0 + bc + e, n - 1)];
    }
  };
  auto kmask = [&](int k0) {
    if (!(VEC && interior_mn && k0 + BK <= k)) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        if (k0 + ac + e >= k) ra[e] = 0.0;
        if (k0 + br >= k) rb[e] = 0.0;
      }
    }
  };
  auto sstore = [&](int buf, int k0) {
    kmask(k0);
    unsigned short ha[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) ha[e] = to_bf16(ra[e]);
    uint4 pk;
    pk.x = ha[0] | ((unsigned)ha[1] << 16);
    pk.y = ha[2] | ((unsigned)ha[3] << 16);
    pk.z = ha[4] | ((unsigned)ha[5] << 16);
    pk.w = ha[6] | ((unsigned)ha[7] << 16);
    *reinterpret_cast<uint4*>(&Ash[buf][ar * LDSH_A + ac]) = pk;
#pragma unroll
    for (int e = 0; e < 8; ++e) Bth[buf][(bc + e) * LDSH_B + br] = to_bf16(rb[e]);
  };

  v4f acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = (k + BK - 1) / BK;
  gload(0);
  sstore(0, 0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
    v4bf a[4], b[4];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      a[blk] = *reinterpret_cast<const v4bf*>(&Ash[buf][(wm * 64 + blk * 16 + li) * LDSH_A + 4 * lq]);
      b[blk] = *reinterpret_cast<const v4bf*>(&Bth[buf][(wn * 64 + blk * 16 + li) * LDSH_B + 4 * lq]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    if (kt + 1 < nk) sstore(buf ^ 1, (kt + 1) * BK);
    __syncthreads();
  }

  sub_acc_f32<NT>(acc, C, ldc, m, n, row0 + wm * 64 + 4 * lq, col0 + wn * 64 + li);
}

// one tile in the requested product precision
template <bool VEC, int PREC, bool CLAMP = false, bool NT = false>
__device__ __forceinline__ void tile_any(int tm, int tn, int m, int n, int k, const double* __restrict__ A,
                                         int lda, const double* __restrict__ B, int ldb, double* __restrict__ C,
                                         int ldc) {
  if constexpr (PREC == kPrecF32) gemm_tile_f32<VEC, NT>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
  else if constexpr (PREC == kPrecBF16) gemm_tile_bf16<VEC, NT>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
  else gemm_tile<VEC, CLAMP>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
}

// Generic launches (inner panel updates, blocked triangular solves) and the
// outer trailing updates (RL3, PF2, RU2) run the same body under two kernel
// names, so that a kernel trace separates the dominant launches.
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_update(int m, int n, int k, const double* __restrict__ A,
                                                        int lda, const double* __restrict__ B, int ldb,
                                                        double* __restrict__ C, int ldc, int tiles_m,
                                                        int tiles_n, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;   // a flag the caller raised on the device
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  gemm_tile<VEC, true>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
}
template <bool VEC, int PREC>
__global__ __launch_bounds__(256, 2) void k_gemm_trailing(int m, int n, int k, const double* __restrict__ A,
                                                          int lda, const double* __restrict__ B, int ldb,
                                                          double* __restrict__ C, int ldc, int tiles_m,
                                                          int tiles_n) {
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  tile_any<VEC, PREC, true>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
}

// The 64 x 64 tile form of both (FP64 only), chosen by the host for launches
// with fewer than kSmallTiles 128 x 128 tiles.
constexpr int kSmallTiles = 128;   // half the CUs of the device
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_small(int m, int n, int k, const double* __restrict__ A, int lda,
                                                       const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                       int ldc, int tiles_m, int tiles_n,
                                                       const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;   // a flag the caller raised on the device
  int tm, tn;
  tile_coords(blockIdx.x, tiles_m, tiles_n, tm, tn);
  gemm_tile_small<VEC>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
}

// The FP64 persistent tile loop, pipelined across tiles, over the whole tiles
// of a launch whose K stages are all whole (k a multiple of 16; the host
// updates a partial last tile row and column with the tile kernels): the
// ticket of the
// next tile is taken while the current tile's first K stage runs (issued
// before its products, resolved after them), the next tile's first K stage is
// loaded while the current tile's last stage runs, and the epilogue stores each
// accumulator of the current tile and loads the same element of the next
// tile's C in its place, so the stores drain while the next loads are in
// flight.  Each tile's arithmetic is that of gemm_tile (the same K stages, the
// same MFMA order), so results do not depend on which workgroup took a tile.
// `x` is the queue the workgroup draws from; only thread 0 uses it.
template <bool VEC>
__device__ __forceinline__ void queue_loop_f64_whole(TileLds& L, int k, const double* __restrict__ A, int lda,
                                                     const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                     int ldc, int tiles_m, int tiles_n, unsigned* __restrict__ q,
                                                     int x) {
  auto& As = L.As;
  auto& Bs = L.Bs;
  __shared__ int s_next;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lq = lane >> 4;
  const int ar = tid >> 1, ac = (tid & 1) * 8;
  const int br = tid >> 4, bc = (tid & 15) * 8;
  const long long T = (long long)tiles_m * tiles_n;
  // thread 0, holding a ticket of queue x: its tile, or the next queue's
  // ticket while this one is exhausted; -1 once every queue is
  auto walk = [&](unsigned ticket) -> int {
    for (int tries = 0;; ++tries) {
      const long long lo = T * x / kXcd, hi = T * (x + 1) / kXcd;
      if (lo + (long long)ticket < hi) return (int)(lo + ticket);
      if (tries + 1 >= kXcd) return -1;
      x = (x + 1) & (kXcd - 1);
      ticket = atomicAdd(&q[x * kQueueStride], 1u);
    }
  };
  double ra[8], rb[8];
  // stage k0 of the tile at (r0, c0) into registers, B negated (k is a
  // multiple of 16: every stage is whole); 16-byte loads when the operands
  // are 8-byte aligned, 8-byte ones otherwise
  auto gload = [&](int r0, int c0, int k0) {
    const double* qa = A + (size_t)(r0 + ar) * lda + k0 + ac;
    const double* qb = B + (size_t)(k0 + br) * ldb + c0 + bc;
    if constexpr (VEC) {
      const dbl2_g* pa = reinterpret_cast<const dbl2_g*>(qa);
      const dbl2_g* pb = reinterpret_cast<const dbl2_g*>(qb);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const dbl2_g xa = pa[e];
        ra[2 * e] = xa.x;
        ra[2 * e + 1] = xa.y;
        const dbl2_g yb = pb[e];
        rb[2 * e] = -yb.x;
        rb[2 * e + 1] = -yb.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        ra[e] = qa[e];
        rb[e] = -qb[e];
      }
    }
  };
  auto sstore = [&](int buf) {
    double* pa = &As[buf][ar * LDS_A + ac];
    double* pb = &Bs[buf][br * LDS_B + bc];
#pragma unroll
    for (int e = 0; e < 8; e += 2) {
      *reinterpret_cast<double2*>(pa + e) = make_double2(ra[e], ra[e + 1]);
      *reinterpret_cast<double2*>(pb + e) = make_double2(rb[e], rb[e + 1]);
    }
  };
  // lane (li, lq) of a 16 x 16 f64 accumulator block holds rows lq + 4 r of column li
  auto cptr = [&](int r0, int c0) { return C + (size_t)(r0 + wm * 64 + lq) * ldc + c0 + wn * 64 + li; };

  if (tid == 0) s_next = walk(atomicAdd(&q[x * kQueueStride], 1u));
  __syncthreads();
  const int t = __builtin_amdgcn_readfirstlane(s_next);
  if (t < 0) return;
  int tm, tn;
  group_coords(t, tiles_m, tiles_n, tm, tn);
  int row0 = tm * BM, col0 = tn * BN;
  v4d acc[4][4];
  {
    const double* cb = cptr(row0, col0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[i][j][r] = cb[(size_t)(i * 16 + 4 * r) * ldc + j * 16];
  }
  gload(row0, col0, 0);
  sstore(0);
  __syncthreads();   // also: every thread has read s_next before it is written again
  int buf = 0;
  const int nk = (k + BK - 1) / BK;
  while (true) {
    unsigned tk = 0;
    if (tid == 0) tk = atomicAdd(&q[x * kQueueStride], 1u);   // resolved after stage 0's products
    int next = -1, nrow0 = 0, ncol0 = 0;
    for (int kt = 0; kt < nk; ++kt) {
      const bool last = kt + 1 == nk;
      if (!last) gload(row0, col0, (kt + 1) * BK);
      else if (next >= 0) gload(nrow0, ncol0, 0);
      double a[2][4], b[2][4];
      auto frag = [&](int st, int qq) {
#pragma unroll
        for (int blk = 0; blk < 4; ++blk) {
          a[qq][blk] = As[buf][(wm * 64 + blk * 16 + li) * LDS_A + 4 * lq + st];
          b[qq][blk] = Bs[buf][(4 * lq + st) * LDS_B + wn * 64 + blk * 16 + li];
        }
      };
      frag(0, 0);
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (st + 1 < 4) frag(st + 1, (st + 1) & 1);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[st & 1][i], b[st & 1][j], acc[i][j], 0, 0, 0);
      }
      if (kt == 0 && tid == 0) s_next = walk(tk);
      if (!last || next >= 0) sstore(buf ^ 1);
      __syncthreads();
      if (kt == 0) {   // the next tile is known once stage 0's barrier has passed
        next = __builtin_amdgcn_readfirstlane(s_next);
        if (next >= 0) {
          int ntm, ntn;
          group_coords(next, tiles_m, tiles_n, ntm, ntn);
          nrow0 = ntm * BM;
          ncol0 = ntn * BN;
        }
      }
      buf ^= 1;
    }
    // epilogue: store this tile, loading the next tile's C into the same
    // registers.  C is read and written once per launch, so both accesses are
    // marked non-temporal: they need not stay in the L2, which then keeps
    // more of the A and B panels that the XCD's other tiles read again (LA at
    // n = 16384: 1.4% faster on B B^T + n I, 1.8% on U(0, 1); the same marks
    // on the first tile's C load and in the plain tile kernels were slower)
    double* cb = cptr(row0, col0);
    if (next >= 0) {
      const double* nb = cptr(nrow0, ncol0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            __builtin_nontemporal_store((double)acc[i][j][r], &cb[(size_t)(i * 16 + 4 * r) * ldc + j * 16]);
            acc[i][j][r] = __builtin_nontemporal_load(&nb[(size_t)(i * 16 + 4 * r) * ldc + j * 16]);
          }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            __builtin_nontemporal_store((double)acc[i][j][r], &cb[(size_t)(i * 16 + 4 * r) * ldc + j * 16]);
      break;
    }
    if (nk == 1) {   // with one stage the next tile was known too late to load it during this one
      gload(nrow0, ncol0, 0);
      sstore(buf);
      __syncthreads();
    }
    row0 = nrow0;
    col0 = ncol0;
  }
}

// The persistent FP64 update over the whole tiles of a launch with whole K
// stages (the host hands the partial last tile row and column to the tile
// kernels): the pipelined tile loop above, under its own kernel name so that
// a kernel trace tells the two forms apart.
template <bool VEC>
__global__ __launch_bounds__(256, 2) void k_gemm_queue_whole(int k, const double* __restrict__ A, int lda,
                                                             const double* __restrict__ B, int ldb,
                                                             double* __restrict__ C, int ldc, int tiles_m,
                                                             int tiles_n, unsigned* __restrict__ q,
                                                             unsigned* __restrict__ clear, int reserve) {
  __shared__ TileLds L;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && clear != nullptr && tid < kXcd) clear[tid * kQueueStride] = 0u;
  if (reserve > 0 && (int)(hw_cu_id() & 7u) < reserve) return;   // uniform over the workgroup
  queue_loop_f64_whole<VEC>(L, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, q, (int)hw_xcc_id());
}

// Persistent form for the look-ahead variant's RU2: queue x holds the logical
// tiles [x T / 8, (x + 1) T / 8); a workgroup takes tickets from the queue of
// the XCD it runs on, then from the other queues in turn, and leaves when all
// are exhausted.  Tickets past a queue's end are harmless (the counters are
// cleared before the slot is used again).  No workgroup waits for another, so
// the launch drains whatever runs beside it.
template <bool VEC, int PREC>
__global__ __launch_bounds__(256, 2) void k_gemm_queue(int m, int n, int k, const double* __restrict__ A,
                                                       int lda, const double* __restrict__ B, int ldb,
                                                       double* __restrict__ C, int ldc, int tiles_m,
                                                       int tiles_n, unsigned* __restrict__ q,
                                                       unsigned* __restrict__ clear, int reserve) {
  __shared__ int s_t;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0 && clear != nullptr && tid < kXcd) clear[tid * kQueueStride] = 0u;
  if (reserve > 0 && (int)(hw_cu_id() & 7u) < reserve) return;   // uniform over the workgroup
  const long long T = (long long)tiles_m * tiles_n;
  int x = (int)hw_xcc_id();
  int empty = 0;
  while (empty < kXcd) {
    if (tid == 0) {
      const long long lo = T * x / kXcd, hi = T * (x + 1) / kXcd;
      const unsigned ticket = atomicAdd(&q[x * kQueueStride], 1u);
      s_t = (lo + (long long)ticket < hi) ? (int)(lo + ticket) : -1;
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_t);
    __syncthreads();
    if (t < 0) {
      ++empty;
      x = (x + 1) & (kXcd - 1);
      continue;
    }
    empty = 0;
    int tm, tn;
    group_coords(t, tiles_m, tiles_n, tm, tn);
    tile_any<VEC, PREC, false, PREC != kPrecF64>(tm, tn, m, n, k, A, lda, B, ldb, C, ldc);
  }
}

// Event timing of the outer trailing-update launches (see mlu_trace_begin).
// Each traced launch has four events: its start and end on its own stream,
// and, when helper workgroups on another stream join its tile queue, one
// before and one after the helper launch (kEv events per slot).
constexpr int kEv = 4;
struct Trace {
  std::mutex mu;
  bool on = false;
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev;
  std::vector<char> tail;
  double flops = 0.0, bytes = 0.0;
};
Trace g_trace;

// The start / end events of one traced launch of an m x n x k update and its
// slot number (none, -1, once the capacity is used up or no trace is active).
int trace_slot(int m, int n, int k, hipEvent_t* e0, hipEvent_t* e1) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  if (g_trace.on && g_trace.used < g_trace.cap) {
    const int id = g_trace.used++;
    *e0 = g_trace.ev[kEv * id];
    *e1 = g_trace.ev[kEv * id + 1];
    g_trace.tail[id] = 0;
    g_trace.flops += 2.0 * m * (double)n * k;
    g_trace.bytes += 8.0 * (2.0 * m * (double)n + (double)m * k + (double)k * n);
    return id;
  }
  return -1;
}

// The events around a helper launch that joins traced launch `id`'s queue.
bool trace_tail(int id, hipEvent_t* pre, hipEvent_t* post) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  if (id < 0 || id >= g_trace.used) return false;
  *pre = g_trace.ev[kEv * id + 2];
  *post = g_trace.ev[kEv * id + 3];
  g_trace.tail[id] = 1;
  return true;
}

}  // namespace

hipError_t gemm_update(hipStream_t s, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                       double* C, int ldc, bool trailing, int prec, bool traced, const int32_t* skip) {
  if (skip != nullptr && trailing) return hipErrorInvalidValue;
  if (prec != kPrecF64 && prec != kPrecF32 && prec != kPrecBF16) return hipErrorInvalidValue;
  if (prec != kPrecF64 && !trailing) return hipErrorInvalidValue;
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  const int tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
  const long long tiles = (long long)tiles_m * tiles_n;
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  const bool vec = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 8 == 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (trailing && traced) (void)trace_slot(m, n, k, &e0, &e1);
  if (e0) {
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return e;
  }
  if (prec == kPrecF64 && tiles < kSmallTiles) {   // few big tiles: four times as many small ones
    const int sm = (m + SBM - 1) / SBM, sn = (n + SBN - 1) / SBN;
    if (vec) hipLaunchKernelGGL(k_gemm_small<true>, dim3((unsigned)(sm * sn)), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc, sm, sn, skip);
    else hipLaunchKernelGGL(k_gemm_small<false>, dim3((unsigned)(sm * sn)), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C, ldc, sm, sn, skip);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
    return e;
  }
  const dim3 grid((unsigned)tiles), block(256);
  if (trailing) {
    if (prec == kPrecF32) {
      if (vec) hipLaunchKernelGGL((k_gemm_trailing<true, kPrecF32>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
      else hipLaunchKernelGGL((k_gemm_trailing<false, kPrecF32>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
    } else if (prec == kPrecBF16) {
      if (vec) hipLaunchKernelGGL((k_gemm_trailing<true, kPrecBF16>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
      else hipLaunchKernelGGL((k_gemm_trailing<false, kPrecBF16>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
    } else {
      if (vec) hipLaunchKernelGGL((k_gemm_trailing<true, kPrecF64>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
      else hipLaunchKernelGGL((k_gemm_trailing<false, kPrecF64>), grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n);
    }
  } else {
    if (vec) hipLaunchKernelGGL(k_gemm_update<true>, grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, skip);
    else hipLaunchKernelGGL(k_gemm_update<false>, grid, block, 0, s, m, n, k, A, lda, B, ldb, C, ldc, tiles_m, tiles_n, skip);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
  return e;
}

hipError_t gemm_queue(hipStream_t s, int m, int n, int k, const double* A, int lda, const double* B, int ldb,
                      double* C, int ldc, unsigned* q, unsigned* clear, int reserve, int grid, bool traced,
                      int prec, int* trace_id, int tail_of, bool edges) {
  if (trace_id != nullptr) *trace_id = -1;
  if (prec != kPrecF64 && prec != kPrecF32 && prec != kPrecBF16) return hipErrorInvalidValue;
  if (m <= 0 || n <= 0 || k <= 0) {
    if (clear == nullptr) return hipSuccess;
    m = n = k = 0;   // still clear the next slot
  }
  // FP64 with whole K stages: the whole tiles go to the pipelined kernel, the
  // partial last tile row and column (if any) to the tile kernels, after it
  // and only with `edges` (the launch that owns the update, not its helpers)
  const bool whole = prec == kPrecF64 && k % BK == 0 && m >= BM && n >= BN;
  const int mi = whole ? m - m % BM : m, ni = whole ? n - n % BN : n;
  const int tiles_m = (mi + BM - 1) / BM, tiles_n = (ni + BN - 1) / BN;
  const long long tiles = (long long)tiles_m * tiles_n;
  if (tiles > 0x7fffffffLL / kXcd) return hipErrorInvalidValue;
  if (reserve < 0 || reserve >= 8) return hipErrorInvalidValue;
  const bool vec = ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) % 8 == 0);
  if (tiles == 0) {
    grid = 1;
    reserve = 0;
  }
  if (grid <= 0) {
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    grid = 2 * cus;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (traced && tiles > 0) {
    const int id = trace_slot(m, n, k, &e0, &e1);
    if (trace_id != nullptr) *trace_id = id;
  } else if (tail_of >= 0 && !trace_tail(tail_of, &e0, &e1)) {
    e0 = e1 = nullptr;
  }
  if (e0) {
    hipError_t e = hipEventRecord(e0, s);
    if (e != hipSuccess) return e;
  }
  if (prec == kPrecF32) {
    if (vec)
      hipLaunchKernelGGL((k_gemm_queue<true, kPrecF32>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
    else
      hipLaunchKernelGGL((k_gemm_queue<false, kPrecF32>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
  } else if (prec == kPrecBF16) {
    if (vec)
      hipLaunchKernelGGL((k_gemm_queue<true, kPrecBF16>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
    else
      hipLaunchKernelGGL((k_gemm_queue<false, kPrecBF16>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
  } else if (whole) {
    if (vec)
      hipLaunchKernelGGL(k_gemm_queue_whole<true>, dim3(grid), dim3(256), 0, s, k, A, lda, B, ldb, C, ldc, tiles_m,
                         tiles_n, q, clear, reserve);
    else
      hipLaunchKernelGGL(k_gemm_queue_whole<false>, dim3(grid), dim3(256), 0, s, k, A, lda, B, ldb, C, ldc, tiles_m,
                         tiles_n, q, clear, reserve);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && edges && mi < m)   // the last, partial tile row
      e = gemm_update(s, m - mi, n, k, A + (size_t)mi * lda, lda, B, ldb, C + (size_t)mi * ldc, ldc, true,
                      kPrecF64, false);
    if (e == hipSuccess && edges && ni < n)   // the last, partial tile column above it
      e = gemm_update(s, mi, n - ni, k, A, lda, B + ni, ldb, C + ni, ldc, true, kPrecF64, false);
    if (e != hipSuccess) return e;
  } else {
    if (vec)
      hipLaunchKernelGGL((k_gemm_queue<true, kPrecF64>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
    else
      hipLaunchKernelGGL((k_gemm_queue<false, kPrecF64>), dim3(grid), dim3(256), 0, s, m, n, k, A, lda, B, ldb, C,
                         ldc, tiles_m, tiles_n, q, clear, reserve);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && e1) e = hipEventRecord(e1, s);
  return e;
}

hipError_t trace_begin(int capacity) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  while ((int)g_trace.ev.size() < kEv * capacity) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    g_trace.ev.push_back(e);
  }
  if ((int)g_trace.tail.size() < capacity) g_trace.tail.resize(capacity);
  g_trace.cap = capacity;
  g_trace.used = 0;
  g_trace.flops = g_trace.bytes = 0.0;
  g_trace.on = true;
  return hipSuccess;
}

hipError_t trace_end(int* launches, double* ms, double* flops, double* bytes) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  g_trace.on = false;
  // A launch lasts from its start to its end, unless helpers joined its queue
  // before it ended (the event before the helper launch precedes its end):
  // then to the later of its end and the helpers' end.  Helpers that start
  // after it ended find the queue empty and add nothing.
  double total = 0.0;
  for (int i = 0; i < g_trace.used; ++i) {
    const hipEvent_t* ev = &g_trace.ev[kEv * i];
    hipError_t r = hipEventSynchronize(ev[1]);
    if (r != hipSuccess) return r;
    float t = 0.f;
    r = hipEventElapsedTime(&t, ev[0], ev[1]);
    if (r != hipSuccess) return r;
    if (g_trace.tail[i]) {
      float tp = 0.f, tq = 0.f;
      if ((r = hipEventSynchronize(ev[3])) != hipSuccess) return r;
      if ((r = hipEventElapsedTime(&tp, ev[0], ev[2])) != hipSuccess) return r;
      if ((r = hipEventElapsedTime(&tq, ev[0], ev[3])) != hipSuccess) return r;
      if (tp < t && tq > t) t = tq;
    }
    total += t;
  }
  *launches = g_trace.used;
  *ms = total;
  *flops = g_trace.flops;
  *bytes = g_trace.bytes;
  return hipSuccess;
}

}  // namespace mlu
