// Batched LU with partial pivoting of many independent matrices of different
// orders in one persistent launch (the method of Section 3 applied to each
// operand: blocked right-looking, Fig. "LU", with the panel factored
// unblocked, Fig. "LU" left).
//
// A device counting sort orders the matrices by decreasing order (the largest
// first, so that the launch's tail holds small ones); a persistent grid of
// 512-thread workgroups takes matrices from an atomic queue in that order.
// One workgroup factors one matrix at a time, NB (16 or 32) columns per step:
//   1. the (n - j) x NB panel is held in registers, one row per thread, and
//      factored with partial pivoting.  Diagonal pivots are tried first (a
//      pass with two barriers in all, checked as it goes, kept when every
//      check holds); otherwise, per column: rows are not moved, each thread
//      tracks the position its row has reached under the interchanges, a DPP
//      wave argmax (first position on ties), each wave's best row copied into
//      LDS, one barrier, then every thread picks the winner, reads its row
//      from LDS and updates its own row in registers;
//   2. the panel's interchanges are applied to the columns outside it,
//      gathered: a lane pair owns a column and loads every moved row before
//      storing any (no chain of dependent swaps);
//   3. per 64 columns of A12: U12 := trilu(A11)^-1 A12 by forward
//      substitution, eight threads per column; then A22 -= A21 U12 on the
//      matrix cores (v_mfma 16 x 16 x 4 in the operand precision), 16 x 16
//      blocks spread over the waves, A21 read from an LDS copy of the panel
//      or, in FP64 with 32-column panels (two workgroups per CU instead of
//      one), from global memory right after the panel was stored there.  That
//      form groups the panels in pairs: the columns beyond a pair take both
//      panels' updates in one pass.
// Waves that hold no row of the current panel only take part in its
// barriers.
// Matrices are row-major (element (i, j) at A[i*lda + j]), in place.
#include "mlu_internal.h"
#include "../../include/mlu.h"

#include <climits>
#include <mutex>
#include <type_traits>

namespace mlu {
namespace {

// A12 columns staged per chunk: eight threads per column in the solve for U12
template <int BT>
constexpr int chunk_cols() { return BT / 8; }
constexpr int kMaxN = MLU_BATCH_MAX_N;
constexpr int kBatchDefaultNB = 16;   // panel width when the caller passes 0
constexpr int kGroup = 2;             // panels whose updates of the columns beyond them go in one pass

// Whether the factored panel is kept in LDS for the trailing update (A21
// read from there) or read back from global memory: LDS for every form but
// FP64 with 32-column panels, whose 512 x 33 copy (135 KB) would leave room
// for one workgroup per CU; without it that form holds two.
template <typename T, int NB>
constexpr bool panel_in_lds() {
  return !(sizeof(T) == 8 && NB == 32);
}

// Size classes: a workgroup of BT threads (one panel row each) factors
// matrices of order at most BT; the batch is split into orders above 256,
// above 128, and the rest, each class a persistent launch of its own.
constexpr int kClasses = 3;
constexpr int class_threads(int cls) { return cls == 0 ? 512 : (cls == 1 ? 256 : 128); }

template <typename T, int NB, int BT>
struct BatchLds {
  static constexpr bool kPL = panel_in_lds<T, NB>();
  static constexpr int kP = NB + 1;   // LDS pitch of the panel
  T P[kPL ? BT * kP : NB * kP];       // the factored panel (L11\U11 over L21), or its diagonal block only
  static constexpr int kUC = chunk_cols<BT>();
  T U[kPL ? NB * kUC : kGroup * NB * kUC];   // U12 chunk (one per panel of a group in the grouped form)
  T cand[2][BT / kWave][NB];   // each wave's candidate pivot row, by column parity
  T wv[2][BT / kWave];
  int wr[2][BT / kWave];
  int16_t src[BT];         // after the panel: the row now at position r came from src[r]
  int piv[NB];
  int item;
};

// v_mfma 16 x 16 x 4 in the operand type: A fragment element (li, k), B
// fragment element (k, li) with k chosen by lane >> 4; the four outputs of a
// lane are rows row_of(lq, r) of column li.
template <typename T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of(int lq, int r) { return lq + 4 * r; }
};
template <>
struct Mfma<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of(int lq, int r) { return 4 * lq + r; }
};

// Cross-lane moves by DPP (no LDS traffic): quad_perm [1,0,3,2] (lane ^ 1),
// [2,3,0,1] (lane ^ 2), row_half_mirror and row_mirror combine the 16 lanes of
// a row; readlane combines the four rows.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ double lane_val(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}
__device__ __forceinline__ float lane_val(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ int lane_val(int v, int lane) { return __builtin_amdgcn_readlane(v, lane); }

template <typename T>
__device__ __forceinline__ T wave_max(T w) {
  auto mx = [](T a, T b) { return a > b ? a : b; };
  w = mx(w, dpp_mov<0xB1>(w));
  w = mx(w, dpp_mov<0x4E>(w));
  w = mx(w, dpp_mov<0x141>(w));
  w = mx(w, dpp_mov<0x140>(w));
  return mx(mx(lane_val(w, 0), lane_val(w, 16)), mx(lane_val(w, 32), lane_val(w, 48)));
}

// (largest value, smallest position among the lanes holding it) over the
// wave; the result is the same in every lane.  Values are never NaN here
// (non-candidates carry -1 and position INT_MAX).
template <typename T>
__device__ __forceinline__ void wave_argmax_t(T& v, int& r) {
  const T w = wave_max(v);
  const unsigned long long tie = __ballot(v == w);
  int rr;
  if (__popcll(tie) == 1) {
    rr = __builtin_amdgcn_readlane(r, __ffsll((long long)tie) - 1);
  } else {
    int x = (v == w) ? r : INT_MAX;
    x = min(x, dpp_mov<0xB1>(x));
    x = min(x, dpp_mov<0x4E>(x));
    x = min(x, dpp_mov<0x141>(x));
    x = min(x, dpp_mov<0x140>(x));
    rr = min(min(lane_val(x, 0), lane_val(x, 16)), min(lane_val(x, 32), lane_val(x, 48)));
  }
  v = w;
  r = rr;
}

template <typename T, int NB, int BT>
__device__ __forceinline__ void factor_one(int n, T* __restrict__ A, int lda, int32_t* __restrict__ ipiv,
                                           int32_t* __restrict__ info, BatchLds<T, NB, BT>& L) {
  constexpr int kP = BatchLds<T, NB, BT>::kP;
  constexpr bool kPL = BatchLds<T, NB, BT>::kPL;
  constexpr int kUC = BatchLds<T, NB, BT>::kUC;
  constexpr int kTG = BT / kUC;      // threads per column in the solve for U12 (n <= BT: one row per thread)
  static_assert(kTG >= 1 && NB % kTG == 0 && kWave % kTG == 0, "solve layout");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // scalar: LDS slots of the wave
  int zero_col = INT_MAX;
  bool spec = true;   // diagonal pivots tried first, until a panel of this matrix refutes them
  // Grouped blocking (the form whose A21 is read back from global memory):
  // panels go in groups of kGroup.  After each panel, the group's remaining
  // columns take its update at once, as in one-level blocking; the columns
  // beyond the group wait: per chunk of them, the panel's rows take the
  // group's earlier panels' updates and are solved for its U12 rows, and
  // after the group's last panel the rows below the group take all of the
  // group's updates in one register pass over their C entries (a fraction
  // of the trailing traffic of one pass per panel).  A panel's interchanges
  // reach the pending rows and the group's earlier L rows alike, so they
  // commute with the deferred updates, and every entry receives the same
  // products in the same order as with one pass per panel.
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int kWaves = BT / kWave, kSB = kUC / 16;
  const int li = lane & 15, lq = lane >> 4;
  // U12 := trilu(L11)^-1 A12 on rows jp..jp+NB-1 (the panel just factored,
  // its diagonal block in P) of the columns [col0, col0 + cw), kTG threads
  // per column; in place, and into U when it is given
  auto solve_u12 = [&](int jp, int col0, int cw, T* U) {
    const int c = tid / kTG, t = tid % kTG;
    const bool ok = c < cw;
    T* a = A + (size_t)jp * lda + col0 + c;
    T x[NB / kTG];
#pragma unroll
    for (int i = 0; i < NB / kTG; ++i) x[i] = ok ? a[(size_t)(kTG * i + t) * lda] : T(0);
#pragma unroll
    for (int k = 0; k < NB - 1; ++k) {
      const T xk = __shfl(x[k / kTG], (lane & ~(kTG - 1)) | (k % kTG));
#pragma unroll
      for (int i = k / kTG; i < NB / kTG; ++i)
        if (kTG * i + t > k) x[i] -= L.P[(kTG * i + t) * kP + k] * xk;
    }
#pragma unroll
    for (int i = 0; i < NB / kTG; ++i) {
      if (U != nullptr) U[(kTG * i + t) * kUC + c] = x[i];
      if (ok && kTG * i + t > 0) a[(size_t)(kTG * i + t) * lda] = x[i];
    }
  };
  // rows [r0, r1) of the columns [col0, col0 + cw) minus A21_p U_p for the
  // np panels p at columns s0 + p NB (U_p in buffer p),
  // on the matrix cores: wave w takes the 16-row bands w, w + 8, ...; per
  // band and panel a lane loads its A21 fragments (from the panel stored
  // just before, still in cache) once for all of the chunk's 16-column
  // blocks, and every C load of the band is issued before the first product
  auto c_update = [&](int r0, int r1, int col0, int cw, int np, int s0) {
    const int R = r1 - r0;
    const int nrb = (R + 15) / 16, nsb = (cw + 15) / 16;
    T* const C = A + (size_t)r0 * lda + col0;
    for (int rb = wave; rb < nrb; rb += kWaves) {
      const int arow = min(rb * 16 + li, R - 1);   // a clamped row is computed and not stored
      acc_t acc[kSB];
#pragma unroll
      for (int sb = 0; sb < kSB; ++sb) {
        const int col = min(sb * 16 + li, cw - 1);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = min(rb * 16 + Mfma<T>::row_of(lq, r), R - 1);
          acc[sb][r] = sb < nsb ? C[(size_t)row * lda + col] : T(0);
        }
      }
      for (int p = 0; p < np; ++p) {
        const T* const A21 = A + (size_t)r0 * lda + s0 + p * NB;
        const T* const U = L.U + p * NB * kUC;
        T af[NB / 4];
#pragma unroll
        for (int s4 = 0; s4 < NB / 4; ++s4) af[s4] = A21[(size_t)arow * lda + 4 * s4 + lq];
#pragma unroll
        for (int sb = 0; sb < kSB; ++sb) {
          if (sb < nsb) {
            const int col = min(sb * 16 + li, cw - 1);
#pragma unroll
            for (int s4 = 0; s4 < NB / 4; ++s4)
              acc[sb] = Mfma<T>::run(af[s4], -U[(4 * s4 + lq) * kUC + col], acc[sb]);
          }
        }
      }
#pragma unroll
      for (int sb = 0; sb < kSB; ++sb) {
        if (sb < nsb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rb * 16 + Mfma<T>::row_of(lq, r);
            if (sb * 16 + li < cw && row < R) C[(size_t)row * lda + sb * 16 + li] = acc[sb][r];
          }
        }
      }
    }
  };
  for (int j = 0; j < n; j += NB) {
    const int nb = min(NB, n - j), rows = n - j;
    // 1. the panel in registers, one row per thread.  Rows are not moved
    //    while the panel is factored: each thread keeps the position its row
    //    has reached under the interchanges so far (pos) and whether it is
    //    still below the diagonal (live); the search breaks ties by position.
    const int r = tid;
    T v[NB];
    auto load_panel = [&]() {
      const bool own = r < rows;
      const T* a = A + (size_t)(j + (own ? r : 0)) * lda + j;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc) v[cc] = (own && cc < nb) ? a[cc] : T(0);
    };
    load_panel();
    int pos = r;
    bool live = r < rows;
    // Speculative pass: the pivot of every column is taken to be the diagonal
    // row, which is the partial pivoting choice exactly when no row below it
    // holds a larger |a(r, c)| at its column step (a tie keeps the diagonal
    // row, as the first-position rule does) and the pivot is not a NaN.  Wave
    // 0, whose lanes hold rows 0..63 and so every pivot row, eliminates its
    // rows alone, each entry of the pivot row read from lane c as it is used
    // (the updates are selected, not branched, so every lane reads it); it
    // then writes the pivot rows into LDS, and the other waves eliminate
    // theirs against them with no barrier per column.  Every row goes through
    // the same operations, in the same order, as in the column steps below,
    // so a pass whose checks all hold leaves what they would leave; otherwise
    // the panel, still untouched in memory, is loaded again and factored by
    // the column steps, and the rest of the matrix goes without speculation.
    bool done = false;
    if (spec) {
      bool fail = false;
      if (wave == 0) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c < nb) {
            const T pv = lane_val(v[c], c);
            const bool below = r > c && r < rows;
            if (pv != pv || (below && fabs(v[c]) > fabs(pv))) fail = true;
            const bool upd = below && pv != T(0);
            const T l = upd ? v[c] / pv : T(0);
            v[c] = upd ? l : v[c];
#pragma unroll
            for (int cc = c + 1; cc < NB; ++cc) {
              const T x = lane_val(v[cc], c);   // lane c's row is not updated at its own column
              const T y = v[cc] - l * x;
              v[cc] = upd ? y : v[cc];
            }
          }
        }
        if (r < nb) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) L.P[r * kP + cc] = v[cc];
        }
      }
      __syncthreads();
      if (wave > 0 && r < rows) {
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          if (c < nb) {
            const T* prow = &L.P[c * kP];
            const T pv = prow[c];
            if (fabs(v[c]) > fabs(pv)) fail = true;
            if (pv != T(0)) {
              const T l = v[c] / pv;
              v[c] = l;
#pragma unroll
              for (int cc = c + 1; cc < NB; ++cc) v[cc] -= l * prow[cc];
            }
          }
        }
      }
      done = __syncthreads_or(fail ? 1 : 0) == 0;
      if (done) {
        for (int c = 0; c < nb; ++c)
          if (L.P[c * kP + c] == T(0) && j + c < zero_col) zero_col = j + c;
        if (tid < nb) L.piv[tid] = tid;
      } else {
        spec = false;
        load_panel();
      }
    }
    if (done) {
      // the rows keep their positions
    } else if (wave * kWave >= rows) {
      // a wave with no row of the panel takes part in the column steps'
      // barriers only (the same count: the second one comes with a column of
      // NaNs, known to every thread from LDS)
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        if (c < nb) {
          const int par = c & 1;
          if (lane == 0) {
            L.wv[par][wave] = T(-1);
            L.wr[par][wave] = INT_MAX;
          }
          __syncthreads();
          T pm = L.wv[par][0];
          int p = L.wr[par][0];
#pragma unroll
          for (int w = 1; w < BT / kWave; ++w)
            if (L.wv[par][w] > pm || (L.wv[par][w] == pm && L.wr[par][w] < p)) {
              pm = L.wv[par][w];
              p = L.wr[par][w];
            }
          if (__builtin_amdgcn_readfirstlane(p) >= rows) __syncthreads();
        }
      }
    } else {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nb) {   // uniform: only the last panel is narrower
        // one barrier per column: each wave's best lane copies its row into
        // LDS (buffers alternate with the column's parity, so the next
        // column's writes cannot meet this column's reads), and every thread
        // reads the winner's row from there
        const int par = c & 1;
        T bv = T(-1);
        int bp = INT_MAX;
        const T av = fabs(v[c]);
        if (live && av > bv) {
          bv = av;
          bp = pos;
        }
        const int mine = bp;
        wave_argmax_t(bv, bp);
        if (bp != INT_MAX && mine == bp) {
#pragma unroll
          for (int cc = 0; cc < NB; ++cc) L.cand[par][wave][cc] = v[cc];
        }
        if (lane == 0) {
          L.wv[par][wave] = bv;
          L.wr[par][wave] = bp;
        }
        __syncthreads();
        T pm = L.wv[par][0];
        int p = L.wr[par][0], ws = 0;
#pragma unroll
        for (int w = 1; w < BT / kWave; ++w)
          if (L.wv[par][w] > pm || (L.wv[par][w] == pm && L.wr[par][w] < p)) {
            pm = L.wv[par][w];
            p = L.wr[par][w];
            ws = w;
          }
        p = __builtin_amdgcn_readfirstlane(p);
        ws = __builtin_amdgcn_readfirstlane(ws);
        if (p >= rows) {   // no comparable entry (a column of NaNs): keep the row at position c
          p = c;
          ws = 0;
          if (live && pos == c) {
#pragma unroll
            for (int cc = 0; cc < NB; ++cc) L.cand[par][0][cc] = v[cc];
          }
          __syncthreads();
        }
        const T* prow = L.cand[par][ws];
        if (tid == 0) L.piv[c] = p;
        const bool me = live && pos == p;
        if (me) {   // the interchange of positions c and p
          live = false;
          pos = c;
        } else if (live && pos == c) {
          pos = p;
        }
        const T pv = prow[c];
        if (pv == T(0) && j + c < zero_col) zero_col = j + c;   // same value in every thread
        if (pv != T(0) && live) {   // the division and rank-1 update
          const T l = v[c] / pv;
          v[c] = l;
#pragma unroll
          for (int cc = c + 1; cc < NB; ++cc) v[cc] -= l * prow[cc];
        }
      }
    }
    }
    // the factored panel to its final rows, in global memory and in LDS
    // (all of it, or, when step 3 reads A21 back from global memory, the
    // diagonal block: the triangle of the solve for U12); src[t] := the
    // panel-start position of the row now at position t
    if (r < rows) {
      T* a = A + (size_t)(j + pos) * lda + j;
#pragma unroll
      for (int cc = 0; cc < NB; ++cc)
        if (cc < nb) a[cc] = v[cc];
      if (kPL || pos < NB) {
#pragma unroll
        for (int cc = 0; cc < NB; ++cc) L.P[pos * kP + cc] = v[cc];
      }
      L.src[pos] = (int16_t)r;
    }
    __syncthreads();
    if (tid < nb) ipiv[j + tid] = j + L.piv[tid] + 1;
    // 2. the interchanges outside the panel, gathered: the row at position t
    //    becomes the one from src[t] for t in {0..nb-1} and {piv[c]}; every
    //    other row is unmoved.  Two neighbouring lanes own a column, the even
    //    one the targets 0..nb-1, the odd one the targets piv[c]; the code
    //    between the loads and the stores has no branch, so both lanes' loads
    //    (one instruction each) complete before either lane's first store:
    //    no order among the swaps remains.
    bool any = false;
    for (int c = 0; c < nb; ++c) any |= L.piv[c] != c;
    if (any) {
      const int ncol = n - nb;
      for (int idx = tid; idx < 2 * ncol; idx += BT) {   // a lane pair is in range together
        const int col = idx >> 1, h = idx & 1;
        const int g = col < j ? col : col + nb;
        int tg[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) tg[k] = k < nb ? (h ? L.piv[k] : k) : 0;
        T st[NB];
#pragma unroll
        for (int k = 0; k < NB; ++k) st[k] = A[(size_t)(j + L.src[tg[k]]) * lda + g];
#pragma unroll
        for (int k = 0; k < NB; ++k) A[(size_t)(j + tg[k]) * lda + g] = st[k];   // equal values to equal rows
      }
    }
    __syncthreads();   // P, and the interchanged columns, visible to the workgroup
    if constexpr (!kPL) {
      // 3, grouped: panel q of the group starting at column s0
      const int q = (j / NB) % kGroup, s0 = j - q * NB;
      const int e = min(s0 + kGroup * NB, n);   // end of the group's columns
      const bool last = j + nb >= e;
      // the group's remaining columns: this panel's U12 rows, then its update
      for (int c0 = j + nb; c0 < e; c0 += kUC) {
        const int cw = min(kUC, e - c0);
        solve_u12(j, c0, cw, L.U);
        __syncthreads();
        c_update(j + nb, n, c0, cw, 1, j);
        __syncthreads();
      }
      // the columns beyond the group
      for (int c0 = e; c0 < n; c0 += kUC) {
        const int cw = min(kUC, n - c0);
        if (q > 0) {
          for (int x = tid; x < q * NB * kUC; x += BT) {   // the earlier panels' U12 rows of the chunk
            const int p = x / (NB * kUC), k = (x / kUC) % NB, c = x % kUC;
            L.U[x] = c < cw ? A[(size_t)(s0 + p * NB + k) * lda + c0 + c] : T(0);
          }
          __syncthreads();
          c_update(j, j + nb, c0, cw, q, s0);   // this panel's rows: their deferred updates
          __syncthreads();
        }
        solve_u12(j, c0, cw, last ? L.U + q * NB * kUC : nullptr);
        __syncthreads();
        if (last) {
          c_update(j + nb, n, c0, cw, q + 1, s0);   // the rows below the group: all its updates
          __syncthreads();
        }
      }
      continue;
    }
    // 3. per chunk of kUC right columns: U12 := trilu(A11)^-1 A12 (kTG
    //    threads per column, forward substitution), then A22 -= A21 U12 on
    //    the matrix cores, 16 x 16 blocks spread over the waves.  (Only a
    //    full panel has right columns: nb == NB here.)
    const int R = rows - nb;
    for (int c0 = 0; c0 < R; c0 += kUC) {
      const int cw = min(kUC, R - c0);
      {
        // thread (c, t) holds rows kTG * i + t of column c
        const int c = tid / kTG, t = tid % kTG;
        const bool ok = c < cw;
        T* a = A + (size_t)j * lda + j + nb + c0 + c;
        T x[NB / kTG];
#pragma unroll
        for (int i = 0; i < NB / kTG; ++i) x[i] = ok ? a[(size_t)(kTG * i + t) * lda] : T(0);
#pragma unroll
        for (int k = 0; k < NB - 1; ++k) {
          const T xk = __shfl(x[k / kTG], (lane & ~(kTG - 1)) | (k % kTG));
#pragma unroll
          for (int i = k / kTG; i < NB / kTG; ++i)
            if (kTG * i + t > k) x[i] -= L.P[(kTG * i + t) * kP + k] * xk;
        }
#pragma unroll
        for (int i = 0; i < NB / kTG; ++i) {
          L.U[(kTG * i + t) * kUC + c] = x[i];
          if (ok && kTG * i + t > 0) a[(size_t)(kTG * i + t) * lda] = x[i];
        }
      }
      __syncthreads();
      if constexpr (kPL) {
        // A22 -= A21 U12 on the matrix cores, A21 from LDS: each wave walks
        // its 16 x 16 blocks, with the next block's C loads issued before the
        // current one's products
        typedef typename Mfma<T>::acc_t acc_t;
        constexpr int kWaves = BT / kWave;
        const int li = lane & 15, lq = lane >> 4;
        const int nrb = (R + 15) / 16, nsb = (cw + 15) / 16, npair = nrb * nsb;
        T* const C = A + (size_t)(j + nb) * lda + j + nb + c0;
        auto load_c = [&](int pp, acc_t& acc) {
          const int rb = pp / nsb;
          const int cb = (pp - rb * nsb) * 16 + li;
          const int col = min(cb, cw - 1);   // a clamped lane is computed and not stored
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = min(rb * 16 + Mfma<T>::row_of(lq, r), R - 1);
            acc[r] = C[(size_t)row * lda + col];
          }
        };
        acc_t cur;
        int pp = wave;
        if (pp < npair) load_c(pp, cur);
        while (pp < npair) {
          const int pn = pp + kWaves;
          acc_t nxt;
          if (pn < npair) load_c(pn, nxt);
          const int rb = pp / nsb;
          const int cb = (pp - rb * nsb) * 16 + li;
          const int arow = nb + min(rb * 16 + li, R - 1);
          const int cbc = min(cb, cw - 1);
#pragma unroll
          for (int s4 = 0; s4 < NB / 4; ++s4) {
            const int k = 4 * s4 + lq;
            cur = Mfma<T>::run(L.P[arow * kP + k], -L.U[k * kUC + cbc], cur);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = rb * 16 + Mfma<T>::row_of(lq, r);
            if (cb < cw && row < R) C[(size_t)row * lda + cb] = cur[r];
          }
          cur = nxt;
          pp = pn;
        }
      } else {
        // A22 -= A21 U12 on the chunk, A21 from global memory: wave w takes the 16-row bands w, w + 8,
        // ...; per band a lane loads its A21 fragments (element (16 rb + li,
        // 4 s + lq), from the panel just stored, still in cache) once for all
        // of the chunk's 16-column blocks, and every C load of the band is
        // issued before the first product
        typedef typename Mfma<T>::acc_t acc_t;
        constexpr int kWaves = BT / kWave, kSB = kUC / 16;
        const int li = lane & 15, lq = lane >> 4;
        const int nrb = (R + 15) / 16, nsb = (cw + 15) / 16;
        T* const C = A + (size_t)(j + nb) * lda + j + nb + c0;
        const T* const A21 = A + (size_t)(j + nb) * lda + j;
        for (int rb = wave; rb < nrb; rb += kWaves) {
          const int arow = min(rb * 16 + li, R - 1);   // a clamped row is computed and not stored
          T af[NB / 4];
#pragma unroll
          for (int s4 = 0; s4 < NB / 4; ++s4) af[s4] = A21[(size_t)arow * lda + 4 * s4 + lq];
          acc_t acc[kSB];
#pragma unroll
          for (int sb = 0; sb < kSB; ++sb) {
            const int col = min(sb * 16 + li, cw - 1);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = min(rb * 16 + Mfma<T>::row_of(lq, r), R - 1);
              acc[sb][r] = sb < nsb ? C[(size_t)row * lda + col] : T(0);
            }
          }
#pragma unroll
          for (int sb = 0; sb < kSB; ++sb) {
            if (sb < nsb) {
              const int col = min(sb * 16 + li, cw - 1);
#pragma unroll
              for (int s4 = 0; s4 < NB / 4; ++s4)
                acc[sb] = Mfma<T>::run(af[s4], -L.U[(4 * s4 + lq) * kUC + col], acc[sb]);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int row = rb * 16 + Mfma<T>::row_of(lq, r);
                if (sb * 16 + li < cw && row < R) C[(size_t)row * lda + sb * 16 + li] = acc[sb][r];
              }
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) *info = zero_col == INT_MAX ? 0 : zero_col + 1;
}

// order[] := matrix indices by decreasing order n (counting sort, one
// workgroup); entries with an invalid order are placed last.  bounds[c] ..
// bounds[c + 1] is the range of size class c (orders above 256, above 128,
// the rest and the invalid ones); the classes' queue counters are cleared.
__global__ __launch_bounds__(1024) void k_batch_order(int batch, const int32_t* __restrict__ d_n, int max_n,
                                                      int32_t* __restrict__ order, unsigned* __restrict__ queue,
                                                      int32_t* __restrict__ bounds) {
  __shared__ int cnt[kMaxN + 2];
  const int tid = threadIdx.x;
  for (int b = tid; b < kMaxN + 2; b += blockDim.x) cnt[b] = 0;
  if (tid < kClasses) queue[tid] = 0u;
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
    // class c holds the orders above class_threads(c + 1): buckets below kMaxN - that
    bounds[0] = 0;
    for (int c = 1; c < kClasses; ++c) bounds[c] = cnt[kMaxN - class_threads(c)];
    bounds[kClasses] = batch;
  }
  __syncthreads();
  for (int i = tid; i < batch; i += blockDim.x) order[atomicAdd(&cnt[bucket(i)], 1)] = i;
}

// Waves per SIMD each instantiation is built for: 4 (two 512-thread
// workgroups per CU, four of 256, eight of 128), 6 for FP32 with 16-column
// panels, so that one matrix's panel, a latency chain, runs beside another's
// work.  Registers are held to it (the second launch bound is the minimum
// waves per execution unit).
template <typename T, int NB>
constexpr int batched_min_waves() {
  return sizeof(T) == 4 && NB == 16 ? 6 : 4;
}

// Persistent: workgroups take the matrices of size class `cls` (the range
// bounds[cls] .. bounds[cls + 1] of order[]) from that class's queue.
template <typename T, int NB, int BT>
__global__ __launch_bounds__(BT, (batched_min_waves<T, NB>())) void k_getrf_batched(
    int cls, const int32_t* __restrict__ d_n, T* const* d_A, const int32_t* __restrict__ d_lda,
    int32_t* const* d_ipiv, int32_t* __restrict__ d_info, int max_n, const int32_t* __restrict__ order,
    unsigned* queue, const int32_t* __restrict__ bounds) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  BatchLds<T, NB, BT>& L = *reinterpret_cast<BatchLds<T, NB, BT>*>(smem);
  const int lo = __builtin_amdgcn_readfirstlane(bounds[cls]);
  const int hi = __builtin_amdgcn_readfirstlane(bounds[cls + 1]);
  while (true) {
    if (threadIdx.x == 0) {
      const unsigned t = atomicAdd(&queue[cls], 1u);
      L.item = t < (unsigned)(hi - lo) ? order[lo + (int)t] : -1;
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
    // (an order above BT cannot be in this class: the sort put it in a larger one)
    const bool bad = n < 0 || n > max_n || n > BT || lda < (n > 1 ? n : 1);
    if (bad || n == 0) {
      if (threadIdx.x == 0) d_info[i] = bad ? -1 : 0;
    } else {
      factor_one<T, NB, BT>(n, d_A[i], lda, d_ipiv[i], &d_info[i], L);
    }
    __syncthreads();
  }
}

// Workgroups of k_getrf_batched<T, NB, class_threads(c)> resident per CU
// (registers and LDS), found once by batched_set_lds_limits.
int g_resident[2][2][kClasses] = {};

template <typename T, int NB, int C>
hipError_t launch_class(hipStream_t s, int batch, const int32_t* d_n, T* const* d_A, const int32_t* d_lda,
                        int32_t* const* d_ipiv, int32_t* d_info, int max_n, const int32_t* order, unsigned* queue,
                        const int32_t* bounds) {
  constexpr int BT = class_threads(C);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int per_cu = g_resident[sizeof(T) == 8 ? 0 : 1][NB == 16 ? 0 : 1][C];
  const int grid = cus * per_cu < batch ? cus * per_cu : batch;
  hipLaunchKernelGGL((k_getrf_batched<T, NB, BT>), dim3(grid), dim3(BT), sizeof(BatchLds<T, NB, BT>), s, C, d_n,
                     d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds);
  return hipGetLastError();
}

// One persistent launch per size class that can hold an order up to max_n
// (the last class also takes the invalid entries), largest first.
template <typename T, int NB>
hipError_t launch_nb(hipStream_t s, int batch, const int32_t* d_n, T* const* d_A, const int32_t* d_lda,
                     int32_t* const* d_ipiv, int32_t* d_info, int max_n, const int32_t* order, unsigned* queue,
                     const int32_t* bounds) {
  hipError_t e = hipSuccess;
  if (max_n > class_threads(1))
    e = launch_class<T, NB, 0>(s, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds);
  if (e == hipSuccess && max_n > class_threads(2))
    e = launch_class<T, NB, 1>(s, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds);
  if (e == hipSuccess)
    e = launch_class<T, NB, 2>(s, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds);
  return e;
}

template <typename T>
int launch_batched(void* stream, int batch, const int32_t* d_n, T* const* d_A, const int32_t* d_lda,
                   int32_t* const* d_ipiv, int32_t* d_info, int max_n, int nb, void* d_work, size_t work_bytes) {
  if (batch < 0) return -2;
  if (batch > 0 && !d_n) return -3;
  if (batch > 0 && !d_A) return -4;
  if (batch > 0 && !d_lda) return -5;
  if (batch > 0 && !d_ipiv) return -6;
  if (batch > 0 && !d_info) return -7;
  if (max_n < 0 || max_n > kMaxN) return -8;
  if (nb != 0 && nb != 16 && nb != 32) return -9;
  if (!d_work) return -10;
  if (work_bytes < batched_workspace_bytes(batch)) return -11;
  if (batch == 0) return 0;
  if (batched_set_lds_limits() != hipSuccess) return MLU_ERR_HIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // workspace: the classes' queue counters (words 0..2), their bounds in
  // order[] (words 16..19), then order[]
  unsigned* queue = reinterpret_cast<unsigned*>(d_work);
  int32_t* bounds = reinterpret_cast<int32_t*>(d_work) + 16;
  int32_t* order = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_work) + 256);
  hipLaunchKernelGGL(k_batch_order, dim3(1), dim3(1024), 0, s, batch, d_n, max_n, order, queue, bounds);
  if (hipGetLastError() != hipSuccess) return MLU_ERR_HIP;
  const int use = nb != 0 ? nb : kBatchDefaultNB;
  const hipError_t e =
      use == 16 ? launch_nb<T, 16>(s, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds)
                : launch_nb<T, 32>(s, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, order, queue, bounds);
  return e == hipSuccess ? 0 : MLU_ERR_HIP;
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
  hipError_t e = hipSuccess;
  auto set = [&](const void* fn, size_t bytes, int threads, int& resident) {
    if (e == hipSuccess) e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    int blocks = 0;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, threads, bytes);
    if (e == hipSuccess) resident = blocks < 1 ? 1 : (blocks > 16 ? 16 : blocks);
  };
  auto set_all = [&](auto tag, auto nbc, int ti, int ni) {
    typedef decltype(tag) T;
    constexpr int NB = decltype(nbc)::value;
    set(reinterpret_cast<const void*>(&k_getrf_batched<T, NB, 512>), sizeof(BatchLds<T, NB, 512>), 512,
        g_resident[ti][ni][0]);
    set(reinterpret_cast<const void*>(&k_getrf_batched<T, NB, 256>), sizeof(BatchLds<T, NB, 256>), 256,
        g_resident[ti][ni][1]);
    set(reinterpret_cast<const void*>(&k_getrf_batched<T, NB, 128>), sizeof(BatchLds<T, NB, 128>), 128,
        g_resident[ti][ni][2]);
  };
  set_all(double(), std::integral_constant<int, 16>(), 0, 0);
  set_all(double(), std::integral_constant<int, 32>(), 0, 1);
  set_all(float(), std::integral_constant<int, 16>(), 1, 0);
  set_all(float(), std::integral_constant<int, 32>(), 1, 1);
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
                       int32_t* const* d_ipiv, int32_t* d_info, int max_n, int nb, void* d_work, size_t work_bytes) {
  return launch_batched<double>(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes);
}

int mlu_sgetrf_batched(void* stream, int batch, const int32_t* d_n, float* const* d_A, const int32_t* d_lda,
                       int32_t* const* d_ipiv, int32_t* d_info, int max_n, int nb, void* d_work, size_t work_bytes) {
  return launch_batched<float>(stream, batch, d_n, d_A, d_lda, d_ipiv, d_info, max_n, nb, d_work, work_bytes);
}

}  // extern "C"
