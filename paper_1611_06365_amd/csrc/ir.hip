// Mixed-precision LU with FP64 iterative refinement (the precision ladder over
// the paper's LU variants): factor with FP32 or BF16 products in the outer
// trailing updates (mlu_dsgetrf), solve, then refine with FP64 residuals on
// the GPU:
//   r = b - A x (FP64),  berr = ||r||_inf / (||A||_inf ||x||_inf + ||b||_inf),
//   stop when berr <= tol, else x := x + d with a correction d.
// mlu_dsgesv_ir (LU-IR): d = (LU)^-1 P r; everything is enqueued on the
// caller's stream, convergence is a device flag that the remaining launches
// of the refinement loop read, so that they do nothing once it is raised (no
// host synchronization).
// mlu_dsgesv_gmres_ir (GMRES-IR, Carson and Higham): d from GMRES on the
// LU-preconditioned system (below), or LU-IR corrections, or LU-IR until it
// stops halving berr; the host drives the loop and reads a small state after
// each step.
#include "mlu_internal.h"
#include "../../include/mlu.h"

#include <cmath>

namespace mlu {
namespace {

constexpr int kGmresMaxKrylov = MLU_GMRES_MAX_KRYLOV;

// refinement state in the workspace (non-negative doubles as their bit
// patterns, so that the maxima can be taken with integer atomics)
struct IrState {
  int32_t done;
  int32_t pad;
  unsigned long long anorm;
  double best;   // smallest backward error so far
};

// LU-IR stops as not converged once the backward error is not finite or has
// grown past this factor times the smallest one reached (the corrections then
// diverge: kappa(A) u_low is too large for plain refinement).
constexpr double kDivergeFactor = 2.0;
// GMRES-IR gives up after this many GMRES corrections in a row that each fail
// to halve the backward error.
constexpr int kGmresStalls = 2;
// The host enqueues Arnoldi steps in chunks of 1, 2, 4, 4, ... and reads the
// state once per chunk; a device flag set by the step that meets the GMRES
// tolerance makes the chunk's later steps return at once.
constexpr int kGmresChunkMax = 4;

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ __forceinline__ double bitsd(unsigned long long b) { return __longlong_as_double((long long)b); }

#define MLU_IR_TRY(x)                   \
  do {                                  \
    hipError_t e__ = (x);               \
    if (e__ != hipSuccess) return e__;  \
  } while (0)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__global__ void k_ir_copy(int rows, int cols, const double* __restrict__ src, int lds, double* __restrict__ dst,
                          int ldd, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / cols, c = e % cols;
    dst[r * ldd + c] = src[r * lds + c];
  }
}

// ||A||_inf = max_i sum_j |a_ij|: one wave per row
__global__ __launch_bounds__(256) void k_ir_anorm(int n, const double* __restrict__ A, int lda,
                                                  unsigned long long* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* a = A + (size_t)row * lda;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};   // four strided partial sums: four loads in flight
  int j = lane;
  for (; j + 192 < n; j += 256) {
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = a[j + 64 * u];
#pragma unroll
    for (int u = 0; u < 4; ++u) s4[u] += fabs(v[u]);
  }
  for (; j < n; j += 64) s4[0] += fabs(a[j]);
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  s = wave_sum(s);
  if (lane == 0) atomicMax(out, dbits(s));
}

// out[c] = max_i |M[i][c]| for the nrhs columns, as the bit patterns of
// non-negative doubles (whose integer order is their numeric order; a NaN
// compares above every number and so propagates).  Each wave strides over the
// rows of one column at a time and folds its lanes' maxima before a single
// atomic, so a column of n rows costs n / 64 atomics on its word instead of n
// (which serialize: about 190 us for one column of 16384).
__global__ __launch_bounds__(256) void k_ir_colmax(int n, int nrhs, const double* __restrict__ M, int ldm,
                                                   unsigned long long* __restrict__ out,
                                                   const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int lane = threadIdx.x & 63;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  if (wave * 64 >= (size_t)n) return;
  for (int c = 0; c < nrhs; ++c) {
    unsigned long long m = 0;
    for (size_t r = wave * 64 + lane; r < (size_t)n; r += stride) m = max(m, dbits(fabs(M[r * ldm + c])));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = max(m, (unsigned long long)__shfl_xor(m, off));
    if (lane == 0) atomicMax(&out[c], m);
  }
}

// Out = Y - A X, or Out = A X when Y is null (FP64; A rows x cols, X cols x
// nrhs): one wave per row of A, NQ right-hand sides at a time.  Out may be Y
// (each element is read and written by the same lane).  Serves as the
// residual (A n x n) and as the block steps of the triangular solves.
template <int NQ>
__global__ __launch_bounds__(256) void k_gemv(int rows, int cols, int nrhs, const double* __restrict__ A, int lda,
                                              const double* __restrict__ X, int ldx, const double* Y, int ldy,
                                              double* Out, int ldo, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const double* a = A + (size_t)row * lda;
  for (int c0 = 0; c0 < nrhs; c0 += NQ) {
    // right-hand sides past nrhs are read from the last one (clamped) and
    // dropped at the store: the loads are unconditional, four columns of A
    // per lane at a time, so they stay in flight together
    int cq[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) cq[q] = min(c0 + q, nrhs - 1);
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) s[q] = 0.0;
    int j = lane;
    for (; j + 192 < cols; j += 256) {
      double av[4], xv[4][NQ];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        av[u] = a[j + 64 * u];
#pragma unroll
        for (int q = 0; q < NQ; ++q) xv[u][q] = X[(size_t)(j + 64 * u) * ldx + cq[q]];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int q = 0; q < NQ; ++q) s[q] += av[u] * xv[u][q];
    }
    for (; j < cols; j += 64) {
      const double aj = a[j];
#pragma unroll
      for (int q = 0; q < NQ; ++q) s[q] += aj * X[(size_t)j * ldx + cq[q]];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double t = wave_sum(s[q]);
      if (lane == 0 && c0 + q < nrhs) {
        const double y = Y != nullptr ? Y[(size_t)row * ldy + c0 + q] : 0.0;
        Out[(size_t)row * ldo + c0 + q] = Y != nullptr ? y - t : t;
      }
    }
  }
}

// One right-hand side with x contiguous: the same one-wave-per-row product,
// each lane loading two neighbouring elements of the row and of x per 16-byte
// load (which needs only 8-byte alignment, so rows of an odd lda keep it),
// four such loads in flight, and A's loads marked non-temporal (each element of A is read
// once per product, so it need not displace x from the caches).  Moving 16
// bytes per lane per load instead of 8 takes the n = 16384 product from about
// 5.1 to 6.5 TB/s and the 1024-column block steps of the triangular solves
// from about 4.3 to 5.4 TB/s.  A lane accumulates even and odd elements
// apart and adds the two before the wave sum; an odd last column is added
// by lane 0.
__global__ __launch_bounds__(256) void k_gemv_x2(int rows, int cols, const double* __restrict__ A, int lda,
                                                 const double* __restrict__ X, const double* Y, int ldy,
                                                 double* Out, int ldo, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const dbl2_g* a = reinterpret_cast<const dbl2_g*>(A + (size_t)row * lda);
  const dbl2_g* x = reinterpret_cast<const dbl2_g*>(X);
  const int pairs = cols >> 1;
  double s0 = 0.0, s1 = 0.0;
  int j = lane;
  for (; j + 192 < pairs; j += 256) {
    dbl2_g av[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = __builtin_nontemporal_load(a + j + 64 * u);
      xv[u] = x[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      s0 += av[u].x * xv[u].x;
      s1 += av[u].y * xv[u].y;
    }
  }
  for (; j < pairs; j += 64) {
    const dbl2_g av = a[j], xv = x[j];
    s0 += av.x * xv.x;
    s1 += av.y * xv.y;
  }
  if ((cols & 1) && lane == 0) s0 += A[(size_t)row * lda + cols - 1] * X[cols - 1];
  const double t = wave_sum(s0 + s1);
  if (lane == 0) {
    const double y = Y != nullptr ? Y[(size_t)row * ldy] : 0.0;
    Out[(size_t)row * ldo] = Y != nullptr ? y - t : t;
  }
}

hipError_t gemv(hipStream_t s, int rows, int cols, int nrhs, const double* A, int lda, const double* X, int ldx,
                const double* Y, int ldy, double* Out, int ldo, const int32_t* skip) {
  if (rows <= 0 || nrhs <= 0) return hipSuccess;
  const dim3 grid((unsigned)((rows + 3) / 4)), block(256);
  const bool x2 = nrhs == 1 && ldx == 1 &&
                  ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(X)) & 7) == 0;
  if (x2)
    hipLaunchKernelGGL(k_gemv_x2, grid, block, 0, s, rows, cols, A, lda, X, Y, ldy, Out, ldo, skip);
  else if (nrhs == 1)
    hipLaunchKernelGGL(k_gemv<1>, grid, block, 0, s, rows, cols, nrhs, A, lda, X, ldx, Y, ldy, Out, ldo, skip);
  else
    hipLaunchKernelGGL(k_gemv<4>, grid, block, 0, s, rows, cols, nrhs, A, lda, X, ldx, Y, ldy, Out, ldo, skip);
  return hipGetLastError();
}

// perm := the row order of P from the sequential interchanges ipiv (1-based;
// (P b)[i] = b[perm[i]]): one workgroup, the permutation composed in LDS by
// one thread, n <= kPermMax (the callers' limit on n).
constexpr int kPermMax = kPanelMaxRows;
static_assert(kPermMax * sizeof(int32_t) <= 160 * 1024, "the permutation must fit in LDS");
__global__ __launch_bounds__(256) void k_perm_from_ipiv(int n, const int32_t* __restrict__ ipiv,
                                                        int32_t* __restrict__ perm) {
  __shared__ int32_t p[kPermMax];
  for (int i = threadIdx.x; i < n; i += 256) p[i] = i;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < n; ++c) {
      const int q = min(max(ipiv[c] - 1, c), n - 1);   // a legal interchange partner (c <= q < n)
      const int t = p[c];
      p[c] = p[q];
      p[q] = t;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += 256) perm[i] = p[i];
}

// Out[i] := X[perm[i]] (one right-hand side)
__global__ void k_gather(int n, const int32_t* __restrict__ perm, const double* __restrict__ X,
                         double* __restrict__ Out, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) Out[i] = X[perm[i]];
}

// every ib x ib block := identity
__global__ void k_identity_blocks(int n, int ib, double* __restrict__ Inv) {
  const int nblk = (n + ib - 1) / ib;
  const size_t total = (size_t)nblk * ib * ib;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = (e / ib) % ib, c = e % ib;
    Inv[e] = r == c ? 1.0 : 0.0;
  }
}

size_t inv_bytes(int n, int ib) { return (size_t)((n + ib - 1) / ib) * ib * ib * sizeof(double); }

// B := U^-1 L^-1 P B with the inverted ib x ib diagonal blocks (Linv, Uinv):
// per block row a GEMV with the block's inverse, then a GEMV update of the
// rows still to be solved.  tmp: n x nrhs (leading dimension nrhs).
// perm / ybuf (optional, one right-hand side): P is applied by a gather of B
// into ybuf through perm (k_perm_from_ipiv) instead of interchanges in place.
hipError_t getrs_blocked(hipStream_t s, int n, int nrhs, const double* LU, int ld, const int32_t* ipiv, int ib,
                         const double* Linv, const double* Uinv, double* Bx, int ldb, double* tmp,
                         const int32_t* skip, const int32_t* perm = nullptr, double* ybuf = nullptr) {
  double* Y = Bx;
  int ldy = ldb;
  if (perm != nullptr && nrhs == 1) {
    hipLaunchKernelGGL(k_gather, dim3((unsigned)min((n + 255) / 256, 65536)), dim3(256), 0, s, n, perm, Bx, ybuf, skip);
    MLU_IR_TRY(hipGetLastError());
    Y = ybuf;
    ldy = 1;
  } else if (laswp(s, Bx, ldb, n, 0, n, ipiv, 0, nrhs, 0, 0, nullptr, skip) != hipSuccess) {
    return hipErrorUnknown;
  }
  const int nblk = (n + ib - 1) / ib;
  const size_t bsz = (size_t)ib * ib;
  for (int k = 0; k < nblk; ++k) {   // L: y := P B (in place), x_k = Linv_k y_k -> tmp
    const int r0 = k * ib, nbk = min(ib, n - r0);
    MLU_IR_TRY(gemv(s, nbk, nbk, nrhs, Linv + k * bsz, ib, Y + (size_t)r0 * ldy, ldy, nullptr, 0,
                    tmp + (size_t)r0 * nrhs, nrhs, skip));
    if (r0 + nbk < n)
      MLU_IR_TRY(gemv(s, n - r0 - nbk, nbk, nrhs, LU + (size_t)(r0 + nbk) * ld + r0, ld, tmp + (size_t)r0 * nrhs,
                      nrhs, Y + (size_t)(r0 + nbk) * ldy, ldy, Y + (size_t)(r0 + nbk) * ldy, ldy, skip));
  }
  for (int k = nblk - 1; k >= 0; --k) {   // U: z := tmp (in place), x_k = Uinv_k z_k -> B
    const int r0 = k * ib, nbk = min(ib, n - r0);
    MLU_IR_TRY(gemv(s, nbk, nbk, nrhs, Uinv + k * bsz, ib, tmp + (size_t)r0 * nrhs, nrhs, nullptr, 0,
                    Bx + (size_t)r0 * ldb, ldb, skip));
    if (r0 > 0)
      MLU_IR_TRY(gemv(s, r0, nbk, nrhs, LU + r0, ld, Bx + (size_t)r0 * ldb, ldb, tmp, nrhs, tmp, nrhs, skip));
  }
  return hipSuccess;
}

// one thread: backward error of this round, stop test, and reset of the
// per-round maxima
__global__ void k_ir_check(int nrhs, IrState* st, unsigned long long* bnorm, unsigned long long* xnorm,
                           unsigned long long* rnorm, double tol, int it, int max_iter, int32_t* d_iters,
                           double* d_berr) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (st->done) return;
  const double an = bitsd(st->anorm);
  double berr = 0.0;
  for (int c = 0; c < nrhs; ++c) {
    const double den = an * bitsd(xnorm[c]) + bitsd(bnorm[c]);
    const double rn = bitsd(rnorm[c]);
    const double e = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
    berr = (e > berr || e != e) ? e : berr;   // NaN propagates
    xnorm[c] = 0ull;
    rnorm[c] = 0ull;
  }
  *d_berr = berr;
  const double best = it == 0 ? berr : fmin(st->best, berr);
  st->best = best;
  if (berr <= tol) {
    st->done = 1;
    *d_iters = it;
  } else if (it >= max_iter || !isfinite(berr) || !(berr <= kDivergeFactor * best)) {
    st->done = 1;
    *d_iters = -1;
  }
}

__global__ void k_ir_axpy(int n, int nrhs, const double* __restrict__ D, int ldd, double* __restrict__ X, int ldx,
                          const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const size_t total = (size_t)n * nrhs;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / nrhs, c = e % nrhs;
    X[r * ldx + c] += D[r * ldd + c];
  }
}

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct IrLayout {
  size_t lu, linv, uinv, r, t, state, norms, total;
};
IrLayout ir_layout(int n, int nrhs) {
  IrLayout L;
  const size_t inv = inv_bytes(n, kIrInvBlock);
  L.lu = align_up(workspace_bytes());
  L.linv = align_up(L.lu + (size_t)n * n * sizeof(double));
  L.uinv = align_up(L.linv + inv);
  L.r = align_up(L.uinv + inv);
  L.t = align_up(L.r + (size_t)n * nrhs * sizeof(double));
  L.state = align_up(L.t + (size_t)n * nrhs * sizeof(double));
  L.norms = align_up(L.state + sizeof(IrState));
  L.total = align_up(L.norms + 3 * (size_t)nrhs * sizeof(unsigned long long));
  return L;
}

unsigned grid_for(size_t work) {
  size_t g = (work + 255) / 256;
  if (g > 65536) g = 65536;
  return (unsigned)(g > 0 ? g : 1);
}


// ---------------------------------------------------------------- GMRES-IR
// Correction equation M^-1 A d = M^-1 r solved by GMRES (Carson and Higham's
// GMRES-IR; GMRES of Saad and Schultz), M = P^T L U the low-precision factors
// applied in FP64 by getrs_blocked.  The Krylov basis V is (m+1) vectors of n
// doubles, vector j at V + j * n; Arnoldi orthogonalizes against it by
// classical Gram-Schmidt applied twice (two rounds of dot products and one
// update each, instead of k dependent steps of modified Gram-Schmidt); H is
// kept column by column (column k at H + k * (m + 1)) and reduced by Givens
// rotations as it grows.  Every reduction runs in a fixed order, so results do
// not depend on scheduling.
struct GmresState {
  unsigned long long anorm, bnorm, xnorm, rnorm;   // bit patterns of non-negative doubles
  double berr;    // backward error of the current x
  double beta;    // ||z||_2 of the current correction's right-hand side
  double hnext;   // h(k+1, k) of the last Arnoldi step, before its rotation
  double resid;   // |g(k+1)|: GMRES residual norm after the last step
  int32_t stop;   // set by the Arnoldi step that ends the correction; later steps' kernels skip
  int32_t steps;  // Arnoldi steps made in the current correction
};

// out[j] = V_j . w for j < k (one workgroup per j, fixed-order reduction)
__global__ __launch_bounds__(256) void k_dots(int n, int k, const double* __restrict__ V, const double* __restrict__ w,
                                              double* __restrict__ out, const int32_t* __restrict__ skip) {
  __shared__ double part[4];
  const int j = blockIdx.x;
  if (j >= k || (skip != nullptr && *skip != 0)) return;
  const double* v = V + (size_t)j * n;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};   // four strided partial sums: four loads in flight
  int i = threadIdx.x;
  for (; i + 768 < n; i += 1024) {
    double a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = v[i + 256 * u];
      b[u] = w[i + 256 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s4[u] += a[u] * b[u];
  }
  for (; i < n; i += 256) s4[0] += v[i] * w[i];
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[j] = ((part[0] + part[1]) + part[2]) + part[3];
}

// w[i] += sign * sum_{j<k} V_j[i] h[j]  (the sum first, then one update)
__global__ __launch_bounds__(256) void k_basis_combine(int n, int k, const double* __restrict__ V,
                                                       const double* __restrict__ h, double sign,
                                                       double* __restrict__ w, const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  __shared__ double hs[kGmresMaxKrylov + 1];
  for (int j = threadIdx.x; j < k; j += 256) hs[j] = h[j];
  __syncthreads();
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s += V[(size_t)j * n + i] * hs[j];
  w[i] = w[i] + sign * s;
}

// v[i] := v[i] / *div
__global__ void k_div_by(int n, double* __restrict__ v, const double* __restrict__ div,
                         const int32_t* __restrict__ skip) {
  if (skip != nullptr && *skip != 0) return;
  const double d = *div;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) v[i] = v[i] / d;
}

// one thread: beta = sqrt(z . z), g = (beta, 0, ..., 0)
__global__ void k_gmres_start(GmresState* st, const double* __restrict__ zz, double* __restrict__ g, int m) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double beta = sqrt(*zz);
  st->beta = beta;
  st->stop = 0;
  st->steps = 0;
  g[0] = beta;
  for (int i = 1; i <= m; ++i) g[i] = 0.0;
}

// one thread: Arnoldi step k's column of H from the two Gram-Schmidt rounds
// (h1 + h2) and ||w||_2, the earlier rotations applied to it, a new rotation
// that zeroes h(k+1, k), and the rotated right-hand side g.  The step that
// brings the GMRES residual to tol * beta, or meets a zero h(k+1, k) (an
// invariant Krylov space), sets the stop flag.
__global__ void k_arnoldi(GmresState* st, int k, int m, const double* __restrict__ h1, const double* __restrict__ h2,
                          const double* __restrict__ ww, double* __restrict__ H, double* __restrict__ cs,
                          double* __restrict__ sn, double* __restrict__ g, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->stop != 0) return;
  double* col = H + (size_t)k * (m + 1);
  for (int j = 0; j <= k; ++j) col[j] = h1[j] + h2[j];
  const double hnext = sqrt(*ww);
  st->hnext = hnext;
  for (int j = 0; j < k; ++j) {
    const double a = col[j], b = col[j + 1];
    col[j] = cs[j] * a + sn[j] * b;
    col[j + 1] = -sn[j] * a + cs[j] * b;
  }
  const double a = col[k], b = hnext;
  const double rho = hypot(a, b);
  const double c = rho == 0.0 ? 1.0 : a / rho;
  const double s = rho == 0.0 ? 0.0 : b / rho;
  cs[k] = c;
  sn[k] = s;
  col[k] = rho;
  col[k + 1] = 0.0;
  g[k + 1] = -s * g[k];
  g[k] = c * g[k];
  st->resid = fabs(g[k + 1]);
  st->steps = k + 1;
  if (st->resid <= tol * st->beta || !(hnext > 0.0)) st->stop = 1;
}

// one thread: y = R^-1 g over the first `steps` columns of the rotated H
__global__ void k_hess_solve(int steps, int m, const double* __restrict__ H, const double* __restrict__ g,
                             double* __restrict__ y) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = steps - 1; i >= 0; --i) {
    double t = g[i];
    for (int j = i + 1; j < steps; ++j) t -= H[(size_t)j * (m + 1) + i] * y[j];
    y[i] = t / H[(size_t)i * (m + 1) + i];
  }
}

// one thread: berr of the current x from the maxima, and their reset
__global__ void k_gmres_berr(GmresState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double den = bitsd(st->anorm) * bitsd(st->xnorm) + bitsd(st->bnorm);
  const double rn = bitsd(st->rnorm);
  st->berr = den > 0.0 ? rn / den : (rn > 0.0 ? INFINITY : 0.0);
  st->xnorm = 0ull;
  st->rnorm = 0ull;
}

struct GmresLayout {
  size_t lu, linv, uinv, r, t, yb, perm, v, h, cs, sn, g, y, dots, state, total;
};
GmresLayout gmres_layout(int n, int m) {
  GmresLayout L;
  const size_t inv = inv_bytes(n, kGmresInvBlock);
  const size_t vec = (size_t)n * sizeof(double), small = (size_t)(m + 2) * sizeof(double);
  L.lu = align_up(workspace_bytes());
  L.linv = align_up(L.lu + (size_t)n * n * sizeof(double));
  L.uinv = align_up(L.linv + inv);
  L.r = align_up(L.uinv + inv);
  L.t = align_up(L.r + vec);
  L.yb = align_up(L.t + vec);
  L.perm = align_up(L.yb + vec);
  L.v = align_up(L.perm + (size_t)n * sizeof(int32_t));
  L.h = align_up(L.v + (size_t)(m + 1) * vec);
  L.cs = align_up(L.h + (size_t)m * (m + 1) * sizeof(double));
  L.sn = align_up(L.cs + small);
  L.g = align_up(L.sn + small);
  L.y = align_up(L.g + small);
  L.dots = align_up(L.y + small);
  L.state = align_up(L.dots + 3 * small);
  L.total = align_up(L.state + sizeof(GmresState));
  return L;
}

}  // namespace
}  // namespace mlu

using namespace mlu;

extern "C" {

int mlu_dsgesv_ir_workspace(int n, int nrhs, size_t* bytes) {
  if (n < 0) return -1;
  if (nrhs < 0) return -2;
  if (!bytes) return -3;
  *bytes = ir_layout(n, nrhs).total;
  (void)mlu_init();   // the library stream, outside any capture (as mlu_dgetrf_workspace)
  return 0;
}

int mlu_dsgesv_ir(void* stream, int n, int nrhs, const double* dA, int lda, const double* dB, int ldb, double* dX,
                  int ldx, int precision, double tol, int max_iter, int variant, int nb, int nb_inner,
                  int32_t* d_ipiv, int32_t* d_info, int32_t* d_iters, double* d_berr, void* d_work,
                  size_t work_bytes) {
  if (n < 0) return -2;
  if (nrhs < 0) return -3;
  if (n > 0 && !dA) return -4;
  if (lda < (n > 1 ? n : 1)) return -5;
  if (n > 0 && nrhs > 0 && !dB) return -6;
  if (ldb < (nrhs > 1 ? nrhs : 1)) return -7;
  if (n > 0 && nrhs > 0 && !dX) return -8;
  if (ldx < (nrhs > 1 ? nrhs : 1)) return -9;
  if (precision != MLU_PREC_FP64 && precision != MLU_PREC_FP32 && precision != MLU_PREC_BF16) return -10;
  if (!(tol >= 0.0)) return -11;
  if (max_iter < 0) return -12;
  if (!valid_variant(variant)) return -13;
  if (nb < 1) return -14;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -15;
  if (n > 0 && !d_ipiv) return -16;
  if (!d_info) return -17;
  if (!d_iters) return -18;
  if (!d_berr) return -19;
  if (!d_work) return -20;
  const IrLayout L = ir_layout(n, nrhs);
  if (work_bytes < L.total) return -21;
  if (n > kPanelMaxRows) return -2;

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(d_work);
  double* LU = reinterpret_cast<double*>(base + L.lu);
  double* R = reinterpret_cast<double*>(base + L.r);
  double* T = reinterpret_cast<double*>(base + L.t);
  double* Linv = reinterpret_cast<double*>(base + L.linv);
  double* Uinv = reinterpret_cast<double*>(base + L.uinv);
  IrState* st = reinterpret_cast<IrState*>(base + L.state);
  unsigned long long* bnorm = reinterpret_cast<unsigned long long*>(base + L.norms);
  unsigned long long* xnorm = bnorm + nrhs;
  unsigned long long* rnorm = xnorm + nrhs;
  const int32_t* done = &st->done;

  if (zero_bytes(s, d_iters, sizeof(int32_t)) != hipSuccess) return MLU_ERR_HIP;
  if (zero_bytes(s, d_berr, sizeof(double)) != hipSuccess) return MLU_ERR_HIP;
  if (n == 0 || nrhs == 0) return zero_bytes(s, d_info, sizeof(int32_t)) == hipSuccess ? 0 : MLU_ERR_HIP;
  if (zero_bytes(s, base + L.state, L.total - L.state) != hipSuccess) return MLU_ERR_HIP;

  const unsigned g2 = grid_for((size_t)n * n), gr = grid_for((size_t)n * nrhs), gw = (unsigned)((n + 3) / 4);
  // LU := A, factor with the low-precision trailing products
  hipLaunchKernelGGL(k_ir_copy, dim3(g2), dim3(256), 0, s, n, n, dA, lda, LU, n, nullptr);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  const int rc = getrf_entry(stream, n, n, LU, n, d_ipiv, d_info, variant, nb, nb_inner, MLU_RL, precision, nullptr, 0, -1,
                             d_work, work_bytes, 0);
  if (rc != 0) return rc == MLU_ERR_HIP ? rc : MLU_ERR_HIP;
  // inverses of the factors' 256 x 256 diagonal blocks (the solves below are
  // then GEMVs), the norms of A and B, then x := (LU)^-1 P b
  const unsigned gi = grid_for(inv_bytes(n, kIrInvBlock) / sizeof(double));
  hipLaunchKernelGGL(k_identity_blocks, dim3(gi), dim3(256), 0, s, n, kIrInvBlock, Linv);
  hipLaunchKernelGGL(k_identity_blocks, dim3(gi), dim3(256), 0, s, n, kIrInvBlock, Uinv);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  if (invert_diag_blocks(s, true, true, n, LU, n, Linv, kIrInvBlock) != hipSuccess) return MLU_ERR_HIP;
  if (invert_diag_blocks(s, false, false, n, LU, n, Uinv, kIrInvBlock) != hipSuccess) return MLU_ERR_HIP;
  hipLaunchKernelGGL(k_ir_anorm, dim3(gw), dim3(256), 0, s, n, dA, lda, &st->anorm);
  hipLaunchKernelGGL(k_ir_colmax, dim3(gr), dim3(256), 0, s, n, nrhs, dB, ldb, bnorm, nullptr);
  hipLaunchKernelGGL(k_ir_copy, dim3(gr), dim3(256), 0, s, n, nrhs, dB, ldb, dX, ldx, nullptr);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  if (getrs_blocked(s, n, nrhs, LU, n, d_ipiv, kIrInvBlock, Linv, Uinv, dX, ldx, T, nullptr) != hipSuccess)
    return MLU_ERR_HIP;
  // refinement: residual and stop test, then a correction, until converged
  for (int it = 0; it <= max_iter; ++it) {
    if (gemv(s, n, n, nrhs, dA, lda, dX, ldx, dB, ldb, R, nrhs, done) != hipSuccess) return MLU_ERR_HIP;
    hipLaunchKernelGGL(k_ir_colmax, dim3(gr), dim3(256), 0, s, n, nrhs, R, nrhs, rnorm, done);
    hipLaunchKernelGGL(k_ir_colmax, dim3(gr), dim3(256), 0, s, n, nrhs, dX, ldx, xnorm, done);
    hipLaunchKernelGGL(k_ir_check, dim3(1), dim3(64), 0, s, nrhs, st, bnorm, xnorm, rnorm, tol, it, max_iter,
                       d_iters, d_berr);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    if (it == max_iter) break;
    if (getrs_blocked(s, n, nrhs, LU, n, d_ipiv, kIrInvBlock, Linv, Uinv, R, nrhs, T, done) != hipSuccess)
      return MLU_ERR_HIP;
    hipLaunchKernelGGL(k_ir_axpy, dim3(gr), dim3(256), 0, s, n, nrhs, R, nrhs, dX, ldx, done);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  }
  return 0;
}

}  // extern "C"

namespace {

// the host's copy of the refinement state, after the stream has reached it
hipError_t read_state(hipStream_t s, const GmresState* d, GmresState* h) {
  MLU_IR_TRY(hipMemcpyAsync(h, d, sizeof(GmresState), hipMemcpyDeviceToHost, s));
  return hipStreamSynchronize(s);
}

}  // namespace

extern "C" {

int mlu_dsgesv_gmres_ir_workspace(int n, int max_krylov, size_t* bytes) {
  if (n < 0) return -1;
  if (max_krylov < 1 || max_krylov > MLU_GMRES_MAX_KRYLOV) return -2;
  if (!bytes) return -3;
  *bytes = gmres_layout(n, max_krylov).total;
  (void)mlu_init();
  return 0;
}

int mlu_dsgesv_gmres_ir(void* stream, int n, const double* dA, int lda, const double* db, double* dx, int precision,
                        int solver, double tol, int max_outer, int max_krylov, double gmres_tol, int variant, int nb,
                        int nb_inner, int32_t* d_ipiv, int32_t* d_info, int32_t* h_outer, int32_t* h_inner,
                        double* h_berr, void* d_work, size_t work_bytes) {
  if (n < 0 || n > kPanelMaxRows) return -2;
  if (n > 0 && !dA) return -3;
  if (lda < (n > 1 ? n : 1)) return -4;
  if (n > 0 && !db) return -5;
  if (n > 0 && !dx) return -6;
  if (precision != MLU_PREC_FP64 && precision != MLU_PREC_FP32 && precision != MLU_PREC_BF16) return -7;
  if (solver != MLU_IR_LU && solver != MLU_IR_GMRES && solver != MLU_IR_AUTO) return -8;
  if (!(tol >= 0.0)) return -9;
  if (max_outer < 0) return -10;
  if (max_krylov < 1 || max_krylov > MLU_GMRES_MAX_KRYLOV) return -11;
  if (!(gmres_tol >= 0.0)) return -12;
  if (!valid_variant(variant)) return -13;
  if (nb < 1) return -14;
  if (nb_inner < 0 || nb_inner > MLU_MAX_NB_INNER) return -15;
  if (n > 0 && !d_ipiv) return -16;
  if (!d_info) return -17;
  if (!h_outer) return -18;
  if (!h_inner) return -19;
  if (!h_berr) return -20;
  if (!d_work) return -21;
  const int m = max_krylov;
  const GmresLayout L = gmres_layout(n, m);
  if (work_bytes < L.total) return -22;

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  *h_outer = 0;
  *h_inner = 0;
  *h_berr = 0.0;
  if (n == 0) {
    if (zero_bytes(s, d_info, sizeof(int32_t)) != hipSuccess) return MLU_ERR_HIP;
    return hipStreamSynchronize(s) == hipSuccess ? 0 : MLU_ERR_HIP;
  }
  char* base = reinterpret_cast<char*>(d_work);
  double* LU = reinterpret_cast<double*>(base + L.lu);
  double* Linv = reinterpret_cast<double*>(base + L.linv);
  double* Uinv = reinterpret_cast<double*>(base + L.uinv);
  double* R = reinterpret_cast<double*>(base + L.r);
  double* T = reinterpret_cast<double*>(base + L.t);
  double* Yb = reinterpret_cast<double*>(base + L.yb);
  int32_t* perm = reinterpret_cast<int32_t*>(base + L.perm);
  double* V = reinterpret_cast<double*>(base + L.v);
  double* H = reinterpret_cast<double*>(base + L.h);
  double* cs = reinterpret_cast<double*>(base + L.cs);
  double* sn = reinterpret_cast<double*>(base + L.sn);
  double* g = reinterpret_cast<double*>(base + L.g);
  double* y = reinterpret_cast<double*>(base + L.y);
  double* h1 = reinterpret_cast<double*>(base + L.dots);
  double* h2 = h1 + (m + 2);
  double* ww = h2 + (m + 2);
  GmresState* st = reinterpret_cast<GmresState*>(base + L.state);
  if (zero_bytes(s, st, sizeof(GmresState)) != hipSuccess) return MLU_ERR_HIP;

  const unsigned g2 = grid_for((size_t)n * n), g1 = grid_for((size_t)n), gw = (unsigned)((n + 3) / 4);
  // LU := A, factored with the low-precision trailing products; the inverses
  // of its 256 x 256 diagonal blocks; the norms of A and b; x := M^-1 b
  hipLaunchKernelGGL(k_ir_copy, dim3(g2), dim3(256), 0, s, n, n, dA, lda, LU, n, nullptr);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  const int rc = getrf_entry(stream, n, n, LU, n, d_ipiv, d_info, variant, nb, nb_inner, MLU_RL, precision, nullptr, 0, -1,
                             d_work, work_bytes, 0);
  if (rc != 0) return rc == MLU_ERR_HIP ? rc : MLU_ERR_HIP;
  // the inverted diagonal blocks of the factors: those of mlu_dsgesv_ir for
  // plain corrections (the same arithmetic step for step), the larger ones
  // from the first GMRES correction on (built when it comes)
  int ib = 0;
  const auto invert = [&](int blk) -> int {
    ib = blk;
    const unsigned gi = grid_for(inv_bytes(n, ib) / sizeof(double));
    hipLaunchKernelGGL(k_identity_blocks, dim3(gi), dim3(256), 0, s, n, ib, Linv);
    hipLaunchKernelGGL(k_identity_blocks, dim3(gi), dim3(256), 0, s, n, ib, Uinv);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    if (invert_diag_blocks(s, true, true, n, LU, n, Linv, ib) != hipSuccess) return MLU_ERR_HIP;
    if (invert_diag_blocks(s, false, false, n, LU, n, Uinv, ib) != hipSuccess) return MLU_ERR_HIP;
    return 0;
  };
  if (invert(solver == MLU_IR_GMRES ? kGmresInvBlock : kIrInvBlock) != 0) return MLU_ERR_HIP;
  hipLaunchKernelGGL(k_ir_anorm, dim3(gw), dim3(256), 0, s, n, dA, lda, &st->anorm);
  hipLaunchKernelGGL(k_ir_colmax, dim3(g1), dim3(256), 0, s, n, 1, db, 1, &st->bnorm, nullptr);
  hipLaunchKernelGGL(k_ir_copy, dim3(g1), dim3(256), 0, s, n, 1, db, 1, dx, 1, nullptr);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  hipLaunchKernelGGL(k_perm_from_ipiv, dim3(1), dim3(256), 0, s, n, d_ipiv, perm);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  const auto precondition = [&](double* v, const int32_t* skip) {   // v := M^-1 v
    return getrs_blocked(s, n, 1, LU, n, d_ipiv, ib, Linv, Uinv, v, 1, T, skip, perm, Yb);
  };
  if (precondition(dx, nullptr) != hipSuccess) return MLU_ERR_HIP;

  const unsigned gc = (unsigned)((n + 255) / 256);
  bool gmres_mode = solver == MLU_IR_GMRES;
  bool last_gmres = false;   // the correction just applied was a GMRES one
  double prev_berr = 0.0, best_berr = 0.0;
  int inner = 0, stalled = 0;
  GmresState hs{};
  for (int it = 0;; ++it) {
    // r := b - A x and the backward error of x
    if (gemv(s, n, n, 1, dA, lda, dx, 1, db, 1, R, 1, nullptr) != hipSuccess) return MLU_ERR_HIP;
    hipLaunchKernelGGL(k_ir_colmax, dim3(g1), dim3(256), 0, s, n, 1, R, 1, &st->rnorm, nullptr);
    hipLaunchKernelGGL(k_ir_colmax, dim3(g1), dim3(256), 0, s, n, 1, dx, 1, &st->xnorm, nullptr);
    hipLaunchKernelGGL(k_gmres_berr, dim3(1), dim3(64), 0, s, st);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    if (read_state(s, st, &hs) != hipSuccess) return MLU_ERR_HIP;
    *h_berr = hs.berr;
    *h_inner = inner;
    if (hs.berr <= tol) {
      *h_outer = it;
      return 0;
    }
    best_berr = it == 0 ? hs.berr : fmin(best_berr, hs.berr);
    if (it >= max_outer) {
      *h_outer = -1;
      return 0;
    }
    if (solver == MLU_IR_LU && (!std::isfinite(hs.berr) || !(hs.berr <= kDivergeFactor * best_berr))) {
      *h_outer = -1;   // plain LU-IR diverges
      return 0;
    }
    if (solver == MLU_IR_AUTO && !gmres_mode && it > 0 && !(hs.berr <= 0.5 * prev_berr)) gmres_mode = true;
    // GMRES corrections that stall: two in a row that do not halve berr end
    // the solve (the preconditioner is too poor for this matrix)
    if (last_gmres) stalled = hs.berr <= 0.5 * prev_berr ? 0 : stalled + 1;
    if (stalled >= kGmresStalls || !std::isfinite(hs.berr)) {
      *h_outer = -1;
      return 0;
    }
    prev_berr = hs.berr;
    last_gmres = gmres_mode;
    if (gmres_mode && ib != kGmresInvBlock && invert(kGmresInvBlock) != 0) return MLU_ERR_HIP;
    // z := M^-1 r, into the first basis vector
    hipLaunchKernelGGL(k_ir_copy, dim3(g1), dim3(256), 0, s, n, 1, R, 1, V, 1, nullptr);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    if (precondition(V, nullptr) != hipSuccess) return MLU_ERR_HIP;
    if (!gmres_mode) {   // LU-IR: x := x + z
      hipLaunchKernelGGL(k_ir_axpy, dim3(g1), dim3(256), 0, s, n, 1, V, 1, dx, 1, nullptr);
      if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
      continue;
    }
    // GMRES on M^-1 A d = z from d = 0
    hipLaunchKernelGGL(k_dots, dim3(1), dim3(256), 0, s, n, 1, V, V, ww, nullptr);
    hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(64), 0, s, st, ww, g, m);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    if (read_state(s, st, &hs) != hipSuccess) return MLU_ERR_HIP;
    if (!(hs.beta > 0.0)) continue;   // z = 0 (or not finite): no correction to make
    hipLaunchKernelGGL(k_div_by, dim3(g1), dim3(256), 0, s, n, V, &st->beta, nullptr);
    // Arnoldi steps, enqueued a chunk at a time; every kernel of a step after
    // the one that sets the stop flag returns at once
    const int32_t* stop = &st->stop;
    int k = 0;
    for (int chunk = 1; k < m; chunk = std::min(2 * chunk, kGmresChunkMax)) {
      for (const int kend = std::min(m, k + chunk); k < kend; ++k) {
        double* w = V + (size_t)(k + 1) * n;   // the next basis vector, built in place
        if (gemv(s, n, n, 1, dA, lda, V + (size_t)k * n, 1, nullptr, 0, w, 1, stop) != hipSuccess)
          return MLU_ERR_HIP;
        if (precondition(w, stop) != hipSuccess) return MLU_ERR_HIP;
        hipLaunchKernelGGL(k_dots, dim3(k + 1), dim3(256), 0, s, n, k + 1, V, w, h1, stop);
        hipLaunchKernelGGL(k_basis_combine, dim3(gc), dim3(256), 0, s, n, k + 1, V, h1, -1.0, w, stop);
        hipLaunchKernelGGL(k_dots, dim3(k + 1), dim3(256), 0, s, n, k + 1, V, w, h2, stop);
        hipLaunchKernelGGL(k_basis_combine, dim3(gc), dim3(256), 0, s, n, k + 1, V, h2, -1.0, w, stop);
        hipLaunchKernelGGL(k_dots, dim3(1), dim3(256), 0, s, n, 1, w, w, ww, stop);
        hipLaunchKernelGGL(k_arnoldi, dim3(1), dim3(64), 0, s, st, k, m, h1, h2, ww, H, cs, sn, g, gmres_tol);
        hipLaunchKernelGGL(k_div_by, dim3(g1), dim3(256), 0, s, n, w, &st->hnext, stop);
        if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
      }
      if (read_state(s, st, &hs) != hipSuccess) return MLU_ERR_HIP;
      if (hs.stop != 0) break;
    }
    const int steps = hs.steps;
    // d = V y, x := x + d
    hipLaunchKernelGGL(k_hess_solve, dim3(1), dim3(64), 0, s, steps, m, H, g, y);
    hipLaunchKernelGGL(k_basis_combine, dim3(gc), dim3(256), 0, s, n, steps, V, y, 1.0, dx, nullptr);
    if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
    inner += steps;
  }
}

}  // extern "C"
