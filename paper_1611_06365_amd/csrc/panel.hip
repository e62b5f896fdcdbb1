// Panel factorization with partial pivoting (LU_unb of Fig. "LU", left, applied
// to a block of at most 16 columns: the diagonal-block step RL1 / PF3 / LL3).
//
// The m x bw block is held in registers by nwg cooperating workgroups
// ("workers") of 512 threads.  Worker 0 (the leader) holds rows 0..511, one per
// thread; worker w >= 1 holds KR rows per thread, rows 512 + (w-1)*512*KR + t +
// 512*k (thread t, k < KR): one row per thread while that takes at most 32
// workers (m <= 16384: as many CUs as the look-ahead leaves to the panel), two
// beyond.  Rows 0..bw-1 (the diagonal rows) therefore always live in the
// leader.
//
// Per column c (exact mode):
//   1. each thread takes its best candidate |a(r, c)|, r >= c (first row on
//      ties); a DPP wave reduction gives the wave's, whose owner lane copies its
//      row into LDS; one workgroup barrier; every thread reduces the per-wave
//      results to the worker's;
//   2. with nwg > 1 the workers exchange candidates through device memory
//      (below); one more barrier hands the winner to every thread;
//   3. rows c and p are exchanged (inside the block only), a21 := a21 / alpha11
//      (a true division; a zero pivot is skipped and reported), and the rank-1
//      update a22 := a22 - a21 a12^T runs on the owned rows.
//
// Speculative mode (m > 64): one wave, the leader (rows 0..63), chooses each
// pivot among its own rows and streams the pivot rows one way; every other wave
// applies them without waiting for any other wave and checks that none of its
// rows beats the chosen pivot (its rows all come after the leader's, so a tie
// keeps the leader's row, exactly as the first-row rule does).  One exchange at the end combines
// the checks.  If every check held, the factorization IS the partial pivoting
// one and is kept; otherwise the block, still untouched in global memory, is
// reloaded and factored again in exact mode, and the rest of the call runs in
// exact mode.  The result never depends on which path ran.
//
// Registers and code size: the column loop is rolled over groups of U columns.
// Within a group the column index is a compile-time offset u; after each group
// every register row is rotated left by U, so the current column always sits at
// index u; LDS and exchanged rows use the same rotated frame and a final
// rotation restores the order.
//
// Exchange protocol, with no fence and no atomic: every published value travels
// in a 16-byte chunk {value, aux, tag} written by one device-coherent (sc1)
// buffer_store_dwordx4, so value and tag land together; readers poll with sc1
// loads until every tag they need matches.  The tag holds the launch epoch
// (unique per launch within a call, the area being cleared at the start of the
// call) and the column.  Exact-mode chunks are double-buffered by column
// parity: a worker writes column c+2 only after reading every worker's column
// c+1 chunk, which each wrote after finishing column c.  Speculative pivot rows
// get one slot per column.  Publishing and polling are done by different waves
// (a wave's loads would otherwise also wait for its own stores).  Every wait is
// bounded: a timeout reports MLU_INFO_SYNC_TIMEOUT, never a hang.
#include "mlu_internal.h"

#include <climits>
#include <cstddef>
#include <type_traits>
#include <utility>

namespace mlu {
namespace {

constexpr int NT = 512;   // threads per workgroup
constexpr int NWAVE = NT / kWave;
constexpr int U = 4;      // columns per rolled step

// Instrumented builds (MLU_PANEL_PROBE, a separate library, never the product
// one) record real-time stamps of the exact-mode column step of the first and
// the last worker: [worker][column % 64][phase], phases 0 column start, 1
// local argmax done, 2 poll issued, 3 poll complete, 4 barrier passed, 5 row
// update done.
#ifdef MLU_PANEL_PROBE
}  // namespace
__device__ unsigned long long g_probe_stamps[2][64][6];
namespace {
__device__ __forceinline__ void probe_stamp(int who, int c, int k, int tid) {
  if (who >= 0 && tid == 0) g_probe_stamps[who][c & 63][k] = __builtin_amdgcn_s_memrealtime();
}
#else
__device__ __forceinline__ void probe_stamp(int, int, int, int) {}
#endif
constexpr long long kSpinLimit = 1LL << 21;
constexpr int kRowNone = INT_MAX;
constexpr int kSc1 = 16;  // buffer cache policy of the publishing stores: device-coherent
constexpr unsigned kTagVerify = 62u;

typedef int v4i __attribute__((ext_vector_type(4)));

template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }


template <int CTRL>
__device__ __forceinline__ double dpp_max_step(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return dmax(v, __hiloint2double(hi, lo));
}

// value of `v` in lane `src` (any lane, per lane)
__device__ __forceinline__ double bpermute_f64(int src, double v) {
  return __hiloint2double(__builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v)),
                          __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v)));
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                          __builtin_amdgcn_readlane(__double2loint(v), lane));
}

// (max |value|, first row among the maxima) over the 64 lanes; the result is
// wave-uniform.  Values are >= -1 (-1 marks "no candidate").
__device__ __forceinline__ void wave_argmax(double& v, int& r) {
  double w = v;
  w = dpp_max_step<0xB1>(w);    // quad_perm [1,0,3,2]: lane ^ 1
  w = dpp_max_step<0x4E>(w);    // quad_perm [2,3,0,1]: lane ^ 2
  w = dpp_max_step<0x141>(w);   // row_half_mirror: the other quad of 8
  w = dpp_max_step<0x140>(w);   // row_mirror: the other half of 16
  w = dmax(dmax(readlane_f64(w, 0), readlane_f64(w, 16)), dmax(readlane_f64(w, 32), readlane_f64(w, 48)));
  const unsigned long long tie = __ballot(v == w);
  int rr;
  if (__popcll(tie) == 1) {
    rr = __builtin_amdgcn_readlane(r, __ffsll((long long)tie) - 1);
  } else {   // several lanes hold the maximum: the smallest row wins
    int x = (v == w) ? r : kRowNone;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off));
    rr = x;
  }
  v = w;
  r = rr;
}

__device__ __forceinline__ int wave_min_int(int x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x = min(x, __shfl_xor(x, off));
  return x;
}

template <int BW>
__device__ __forceinline__ void lds_put_row(double* dst, const double (&src)[BW]) {
#pragma unroll
  for (int j = 0; j < BW; j += 2) *reinterpret_cast<double2*>(dst + j) = make_double2(src[j], src[j + 1]);
}
template <int BW>
__device__ __forceinline__ void lds_get_row(double (&dst)[BW], const double* src) {
#pragma unroll
  for (int j = 0; j < BW; j += 2) {
    const double2 x = *reinterpret_cast<const double2*>(src + j);
    dst[j] = x.x;
    dst[j + 1] = x.y;
  }
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ void put_chunk(__amdgpu_buffer_rsrc_t rs, unsigned off, double v, unsigned aux,
                                          unsigned tag) {
  v4i x;
  x[0] = __double2loint(v);
  x[1] = __double2hiint(v);
  x[2] = (int)aux;
  x[3] = (int)tag;
  __builtin_amdgcn_raw_buffer_store_b128(x, rs, (int)off, 0, kSc1);
}
// Polled reads of chunks: device-coherent (sc1) 16-byte loads written as one
// volatile asm block that issues them all and waits for them all, so that a
// wait loop really reads memory again on every pass (the compiler may
// otherwise keep a load's value from an earlier pass) and every load has
// landed before its registers are used.  Lane-wise, chunk i is read at
// base + offs[i]; unused slots of a block repeat the last address.
template <int K>
__device__ __forceinline__ void get_chunks(const char* base, const unsigned (&offs)[K], v4i (&out)[K]) {
  static_assert(K >= 1 && K <= 12, "at most 12 chunks per poll");
  const v4i* p[12];
#pragma unroll
  for (int i = 0; i < 12; ++i) p[i] = reinterpret_cast<const v4i*>(base + offs[i < K ? i : K - 1]);
  v4i r[12];
  if constexpr (K <= 4) {
    asm volatile(
        "global_load_dwordx4 %0, %4, off sc1\n\t"
        "global_load_dwordx4 %1, %5, off sc1\n\t"
        "global_load_dwordx4 %2, %6, off sc1\n\t"
        "global_load_dwordx4 %3, %7, off sc1\n\t"
        "s_waitcnt vmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3])
        : "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3])
        : "memory");
  } else if constexpr (K <= 8) {
    asm volatile(
        "global_load_dwordx4 %0, %8, off sc1\n\t"
        "global_load_dwordx4 %1, %9, off sc1\n\t"
        "global_load_dwordx4 %2, %10, off sc1\n\t"
        "global_load_dwordx4 %3, %11, off sc1\n\t"
        "global_load_dwordx4 %4, %12, off sc1\n\t"
        "global_load_dwordx4 %5, %13, off sc1\n\t"
        "global_load_dwordx4 %6, %14, off sc1\n\t"
        "global_load_dwordx4 %7, %15, off sc1\n\t"
        "s_waitcnt vmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]),
          "=&v"(r[7])
        : "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3]), "v"(p[4]), "v"(p[5]), "v"(p[6]), "v"(p[7])
        : "memory");
  } else {
    asm volatile(
        "global_load_dwordx4 %0, %12, off sc1\n\t"
        "global_load_dwordx4 %1, %13, off sc1\n\t"
        "global_load_dwordx4 %2, %14, off sc1\n\t"
        "global_load_dwordx4 %3, %15, off sc1\n\t"
        "global_load_dwordx4 %4, %16, off sc1\n\t"
        "global_load_dwordx4 %5, %17, off sc1\n\t"
        "global_load_dwordx4 %6, %18, off sc1\n\t"
        "global_load_dwordx4 %7, %19, off sc1\n\t"
        "global_load_dwordx4 %8, %20, off sc1\n\t"
        "global_load_dwordx4 %9, %21, off sc1\n\t"
        "global_load_dwordx4 %10, %22, off sc1\n\t"
        "global_load_dwordx4 %11, %23, off sc1\n\t"
        "s_waitcnt vmcnt(0)"
        : "=&v"(r[0]), "=&v"(r[1]), "=&v"(r[2]), "=&v"(r[3]), "=&v"(r[4]), "=&v"(r[5]), "=&v"(r[6]),
          "=&v"(r[7]), "=&v"(r[8]), "=&v"(r[9]), "=&v"(r[10]), "=&v"(r[11])
        : "v"(p[0]), "v"(p[1]), "v"(p[2]), "v"(p[3]), "v"(p[4]), "v"(p[5]), "v"(p[6]), "v"(p[7]), "v"(p[8]),
          "v"(p[9]), "v"(p[10]), "v"(p[11])
        : "memory");
  }
#pragma unroll
  for (int i = 0; i < K; ++i) out[i] = r[i];
}

__device__ __forceinline__ double chunk_val(v4i x) { return __hiloint2double(x[1], x[0]); }

constexpr unsigned off_hdr(int par, int w) {
  return (unsigned)offsetof(PanelWork, hdr) + (unsigned)((par * kPanelMaxWG + w) * 16);
}
constexpr unsigned off_cand(int par, int w, int t) {
  return (unsigned)offsetof(PanelWork, cand) + (unsigned)(((par * kPanelMaxWG + w) * kPanelMaxCols + t) * 16);
}
constexpr unsigned off_diag(int par, int t) {
  return (unsigned)offsetof(PanelWork, diag) + (unsigned)((par * kPanelMaxCols + t) * 16);
}
constexpr unsigned off_spec(int c, int t) {
  return (unsigned)offsetof(PanelWork, spec) + (unsigned)((c * kPanelMaxCols + t) * 16);
}
constexpr unsigned off_verify(int w) { return (unsigned)offsetof(PanelWork, verify) + (unsigned)(w * 16); }

// worker that holds a given row (rows as laid out above; KR rows per thread
// outside the leader)
template <int KR>
__device__ __forceinline__ int worker_of(int r) { return r < NT ? 0 : 1 + (r - NT) / (KR * NT); }

struct PanelShared {
  double val[2][NWAVE];
  int row[2][NWAVE];
  int p[2];
  int fail[NWAVE];
  int gfail;
  int zero_col;
  int piv[kPanelMaxCols];
};

// Bounded poll of n chunks (lane i of the calling wave reads offs[i]) until all
// tags match; returns the chunks.  Lanes may repeat offsets.
template <int K>
__device__ __forceinline__ void poll_chunks(const char* base, const unsigned (&offs)[K], v4i (&out)[K],
                                            unsigned tag, int lane, int32_t* info) {
  long long spins = 0;
  while (true) {
    get_chunks<K>(base, offs, out);
    unsigned bad = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) bad |= (unsigned)out[i][3] ^ tag;
    if (__all(bad == 0u)) return;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      if (lane == 0) atomicExch(info, -999);
      return;
    }
  }
}

template <int BW, int MAXW, int KR>
struct Panel {
  static constexpr int kPoll = (MAXW * BW + kWave - 1) / kWave;   // candidate chunks per lane

  double* A;
  int lda, m, bw;
  int32_t* info;
  int nwg, wg, tid, lane, wave;
  unsigned epoch;
  __amdgpu_buffer_rsrc_t rs;
  const char* wbase;
  double (*s_cand)[NWAVE][BW];
  double (*s_drow)[BW];
  double (*s_prow)[BW];
  PanelShared* sh;
  double v[KR][BW];
  int rows[KR];

  __device__ __forceinline__ void load() {
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const bool ok = rows[k] < m;
      const double* src = A + (size_t)(ok ? rows[k] : 0) * lda;
#pragma unroll
      for (int c = 0; c < BW; ++c) v[k][c] = (ok && c < bw) ? src[c] : 0.0;
    }
  }
  __device__ __forceinline__ void store() {
#pragma unroll
    for (int k = 0; k < KR; ++k)
      if (rows[k] < m) {
        double* dst = A + (size_t)rows[k] * lda;
#pragma unroll
        for (int c = 0; c < BW; ++c)
          if (c < bw) dst[c] = v[k][c];
      }
  }
  __device__ __forceinline__ void rotate() {
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      double t[U];
#pragma unroll
      for (int j = 0; j < U; ++j) t[j] = v[k][j];
#pragma unroll
      for (int j = 0; j < BW - U; ++j) v[k][j] = v[k][j + U];
#pragma unroll
      for (int j = 0; j < U; ++j) v[k][BW - U + j] = t[j];
    }
  }
  // after the groups that covered bw columns, finish the cycle of rotations
  __device__ __forceinline__ void unrotate() {
    for (int g = (bw + U - 1) / U; g < BW / U; ++g) rotate();
  }

  // Steps 1 and the local reduction: this worker's best row and its values in
  // LDS; returns (value, row, wave holding it).
  template <int u, int par>
  __device__ __forceinline__ void local_best(int c, double& bv, int& br, int& wbest) {
    bv = -1.0;
    br = kRowNone;
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int r = rows[k];
      if (r < m && r >= c) {
        const double a = fabs(v[k][u]);
        if (a > bv) {
          bv = a;
          br = r;
        }
      }
    }
    wave_argmax(bv, br);
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      if (rows[k] == br) lds_put_row<BW>(s_cand[par][wave], v[k]);
      if (rows[k] == c) lds_put_row<BW>(s_drow[par], v[k]);
    }
    if (lane == 0) {
      sh->val[par][wave] = bv;
      sh->row[par][wave] = br;
    }
    lds_sync();
    double wv[NWAVE];
    int wr[NWAVE];
#pragma unroll
    for (int w = 0; w < NWAVE; ++w) {
      wv[w] = sh->val[par][w];
      wr[w] = sh->row[par][w];
    }
    bv = wv[0];
#pragma unroll
    for (int w = 1; w < NWAVE; ++w) bv = dmax(bv, wv[w]);
    wbest = 0;
    br = kRowNone;
#pragma unroll
    for (int w = NWAVE - 1; w >= 0; --w)
      if (wv[w] == bv && wr[w] <= br) {
        br = wr[w];
        wbest = w;
      }
  }

  // Step 3 with the pivot row `prow` and the old diagonal row `drow` (LDS).
  template <int u>
  __device__ __forceinline__ void apply(int c, int lim, int p, const double* prow, const double* drow) {
    const double piv = prow[u];
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      if (rows[k] == c) lds_get_row<BW>(v[k], prow);
      else if (rows[k] == p) lds_get_row<BW>(v[k], drow);
    }
#pragma unroll
    for (int k = 0; k < KR; ++k) {
      const int r = rows[k];
      if (r > c && r < m) {
        double l = v[k][u];
        if (piv != 0.0) {
          l = l / piv;
          v[k][u] = l;
        }
        // entries past this column and inside the block; finished columns
        // rotated to the end stay untouched
#pragma unroll
        for (int j = u + 1; j < BW; ++j) v[k][j] = v[k][j] - l * ((j < lim) ? prow[j] : 0.0);
      }
    }
    if (tid == 0) {
      sh->piv[c] = p;
      if (piv == 0.0 && sh->zero_col < 0) sh->zero_col = c;
    }
  }

  // One full pass in exact mode.
  __device__ __forceinline__ void exact_pass() {
    for (int c0 = 0; c0 < bw; c0 += U) {
      const int lim = bw - c0;
      static_for<U>([&](auto uidx) {
        constexpr int u = decltype(uidx)::value;
        constexpr int par = u & 1;
        const int c = c0 + u;
        if (c < bw) {
          const int who = wg == 0 ? 0 : (wg == nwg - 1 ? 1 : -1);
          probe_stamp(who, c, 0, tid);
          double bv;
          int br, wbest;
          local_best<u, par>(c, bv, br, wbest);
          probe_stamp(who, c, 1, tid);
          int p = br;
          const double* prow = s_cand[par][wbest];
          if (nwg > 1) {
            const unsigned tag = epoch * 64u + (unsigned)c;
            if (wave == NWAVE - 1) {   // publish
              if (lane < BW) put_chunk(rs, off_cand(par, wg, lane), s_cand[par][wbest][lane], 0u, tag);
              if (wg == 0 && lane >= 32 && lane - 32 < BW)
                put_chunk(rs, off_diag(par, lane - 32), s_drow[par][lane - 32], 0u, tag);
              if (lane == 63) put_chunk(rs, off_hdr(par, wg), bv, (unsigned)br, tag);
            } else if (wave == 0) {    // poll every worker's chunks of this column
              unsigned offs[kPoll + 2];
              v4i got[kPoll + 2];
              offs[0] = off_hdr(par, min(lane, nwg - 1));
              offs[1] = off_diag(par, lane % BW);
#pragma unroll
              for (int i = 0; i < kPoll; ++i) {
                const int f = min(lane + kWave * i, nwg * BW - 1);
                offs[2 + i] = off_cand(par, f / BW, f % BW);
              }
              probe_stamp(who, c, 2, tid);
              poll_chunks<kPoll + 2>(wbase, offs, got, tag, lane, info);
              probe_stamp(who, c, 3, tid);
              double gv = lane < nwg ? chunk_val(got[0]) : -1.0;
              int gr = lane < nwg ? got[0][2] : kRowNone;
              wave_argmax(gv, gr);
              const int gw = gr == kRowNone ? 0 : worker_of<KR>(gr);
              if (lane == 0) sh->p[par] = gr;
#pragma unroll
              for (int i = 0; i < kPoll; ++i) {
                const int f = lane + kWave * i;
                if (f < nwg * BW && f / BW == gw) s_prow[par][f % BW] = chunk_val(got[2 + i]);
              }
              if (lane < BW) s_drow[par][lane] = chunk_val(got[1]);
            }
            lds_sync();
            probe_stamp(who, c, 4, tid);
            p = sh->p[par];
            prow = s_prow[par];
          }
          apply<u>(c, lim, p, prow, s_drow[par]);
          probe_stamp(who, c, 5, tid);
        }
      });
      rotate();
    }
    unrotate();
  }

  // One pass in speculative mode; returns the first column at which one of this
  // thread's rows beat the leader's pivot (bw if none).  The leader is wave 0
  // of worker 0 (rows 0..63): it picks each pivot among its own rows with wave
  // operations only and publishes the pivot row.  Every other wave follows on
  // its own, with no barrier: it fetches the pivot rows of a whole group of U
  // columns at once (one memory round trip when the leader is ahead), checks
  // and updates its rows.  The two roles run separate loops: the leader's loop
  // issues stores only and never waits for them; the followers' loop loads only.
  __device__ __forceinline__ int spec_pass() {
    __builtin_amdgcn_s_waitcnt(0);   // the block's loads, before loops that must not wait in them
    if (wg == 0 && wave == 0) {
      spec_lead();
      return bw;   // the leader's rows never beat the maximum it chose
    }
    return spec_follow();
  }

  // The leader's column step uses cross-lane operations only (its rows are its
  // lanes): the two rows are interchanged with a lane permutation, the pivot
  // row is broadcast into scalar registers, published by lanes 0..BW-1, and
  // the leader's rows below the pivot are updated.
  __device__ __forceinline__ void spec_lead() {
    for (int c0 = 0; c0 < bw; c0 += U) {
      const int lim = bw - c0;
      static_for<U>([&](auto uidx) {
        constexpr int u = decltype(uidx)::value;
        const int c = c0 + u;
        if (c < bw) {
          const unsigned tag = epoch * 64u + (unsigned)c;
          const bool act = rows[0] < m && rows[0] >= c;
          double bv = act ? fabs(v[0][u]) : -1.0;
          int br = act ? rows[0] : kRowNone;
          wave_argmax(bv, br);
          const int p = br;   // leader rows are lanes: row p sits in lane p
          if (p != c) {
            const int src = lane == c ? p : (lane == p ? c : lane);
#pragma unroll
            for (int j = 0; j < BW; ++j) v[0][j] = bpermute_f64(src, v[0][j]);
          }
          double pr[BW];
#pragma unroll
          for (int j = 0; j < BW; ++j) pr[j] = (j < u) ? 0.0 : readlane_f64(v[0][j], c);
          double out = 0.0;
#pragma unroll
          for (int j = 0; j < BW; ++j) out = lane == j ? pr[j] : out;
          if (lane < BW) put_chunk(rs, off_spec(c, lane), out, 0u, tag);
          const double piv = pr[u];
          if (rows[0] > c && rows[0] < m) {
            double l = v[0][u];
            if (piv != 0.0) {
              l = l / piv;
              v[0][u] = l;
            }
#pragma unroll
            for (int j = u + 1; j < BW; ++j) v[0][j] = v[0][j] - l * ((j < lim) ? pr[j] : 0.0);
          }
          if (lane == 0) {
            sh->piv[c] = p;
            if (piv == 0.0 && sh->zero_col < 0) sh->zero_col = c;
          }
        }
      });
      rotate();
    }
    unrotate();
  }

  __device__ __forceinline__ int spec_follow() {
    int fail = bw;
    for (int c0 = 0; c0 < bw; c0 += U) {
      const int lim = bw - c0;
      v4i cache[U];
      static_for<U>([&](auto uidx) {
        constexpr int u = decltype(uidx)::value;
        const int c = c0 + u;
        if (c < bw) {
          const unsigned tag = epoch * 64u + (unsigned)c;
          unsigned offs[U];
#pragma unroll
          for (int i = 0; i < U; ++i) offs[i] = off_spec(min(c0 + i, bw - 1), lane % BW);
          if (u == 0) get_chunks<U>(wbase, offs, cache);   // the whole group's pivot rows in one go
          long long spins = 0;
          while (!__all((unsigned)cache[u][3] == tag)) {
            __builtin_amdgcn_s_sleep(1);
            get_chunks<U>(wbase, offs, cache);
            if (++spins > kSpinLimit) {
              if (lane == 0) atomicExch(info, -999);
              break;
            }
          }
          // lane j holds entry j of the pivot row: broadcast it
          const double mine = chunk_val(cache[u]);
          double pr[BW];
#pragma unroll
          for (int j = 0; j < BW; ++j) pr[j] = (j < u) ? 0.0 : readlane_f64(mine, j);
          const double piv = pr[u];
          const double apiv = fabs(piv);
#pragma unroll
          for (int k = 0; k < KR; ++k) {
            const int r = rows[k];
            if (r < m) {
              if (fabs(v[k][u]) > apiv && fail > c) fail = c;
              double l = v[k][u];
              if (piv != 0.0) {
                l = l / piv;
                v[k][u] = l;
              }
#pragma unroll
              for (int j = u + 1; j < BW; ++j) v[k][j] = v[k][j] - l * ((j < lim) ? pr[j] : 0.0);
            }
          }
        }
      });
      rotate();
    }
    unrotate();
    return fail;
  }

  // Combine the workers' checks: the first failing column over all workers.
  __device__ __forceinline__ int verify(int fail) {
    const int wf = wave_min_int(fail);
    if (lane == 0) sh->fail[wave] = wf;
    lds_sync();
    if (wave == 0) {
      int f = sh->fail[0];
#pragma unroll
      for (int w = 1; w < NWAVE; ++w) f = min(f, sh->fail[w]);
      const unsigned tag = epoch * 64u + kTagVerify;
      if (lane == 0) put_chunk(rs, off_verify(wg), (double)f, 0u, tag);
    } else if (wave == 1) {
      unsigned offs[1] = {off_verify(min(lane, nwg - 1))};
      v4i got[1];
      poll_chunks<1>(wbase, offs, got, epoch * 64u + kTagVerify, lane, info);
      const int g = wave_min_int((int)chunk_val(got[0]));
      if (lane == 0) sh->gfail = g;
    }
    lds_sync();
    return sh->gfail;
  }
};

// Epilogue of worker 0 when the block is part of a wider panel: the block's
// interchanges applied to the panel's other columns (cl columns to the left of
// the block, cr to its right; LAPACK laswp semantics, the sequential swaps
// composed into one permutation of the touched rows and every displaced row
// segment moved once through LDS), then the top rows of the first ns right
// columns solved with a unit lower triangle (A12 := trilu(A11)^-1 A12, the next
// step of the blocked RL algorithm inside the panel).  The triangle is the
// block's own (lb = 0), or, when the block is the second half of a 32-column
// diagonal block factored in two register passes (lb = 16), the whole 32 x 32
// triangle: the lb rows above the block and the block's rows, with the lb
// columns to the block's left.  No other worker touches these columns during
// the launch.
constexpr int kMvCols = 64;
constexpr int kTriMax = kPanelWideCols;   // rows of the largest triangle solved
static_assert(2 * kPanelRegCols <= kTriMax, "a two-pass block's triangle fits");

struct EpilogueShared {
  double mv[2 * kPanelWideCols][kMvCols];
  double T[kTriMax][kTriMax + 1];
  int slot[kPanelWideCols];
  int row[2 * kPanelWideCols];
  int label[2 * kPanelWideCols];
  int any;
};

// Kept out of line so that its registers do not add to the factorization's;
// es.T[lb + r][lb + c] (c < r < bw) already holds the block's strictly lower
// rows.
typedef __attribute__((address_space(1))) double gdouble;   // global memory

template <int BW, int LB>
__device__ __noinline__ void panel_epilogue(double* __restrict__ Ag, int lda, int bw, int cl, int cr, int ns,
                                            const int* piv, int tid, EpilogueShared* esp) {
  constexpr int lb = LB;
  // the matrix is global memory: accessed as such, the loads and stores are
  // global (vector-memory counter only) instead of flat, which would also
  // count against the LDS counter that every LDS wait below waits for
  gdouble* __restrict__ A = (gdouble*)Ag;
  EpilogueShared& es = *esp;
  const int ntouch = 2 * bw;
  if (tid < ntouch) {
    es.label[tid] = tid;
    es.row[tid] = tid < bw ? tid : -1;
  }
  if (tid == 0) es.any = 0;
  __syncthreads();
  if (tid < bw) {   // slot of step tid's partner row
    const int p = piv[tid];
    int slot;
    if (p < bw) {
      slot = p;
    } else {
      int first = tid;
      for (int q = 0; q < tid; ++q)
        if (piv[q] == p) {
          first = q;
          break;
        }
      slot = bw + first;
      if (first == tid) es.row[bw + tid] = p;
    }
    es.slot[tid] = slot;
    if (p != tid) es.any = 1;
  }
  __syncthreads();
  if (es.any) {
    if (tid == 0) {
      for (int c = 0; c < bw; ++c) {
        const int t = es.label[c];
        es.label[c] = es.label[es.slot[c]];
        es.label[es.slot[c]] = t;
      }
    }
    __syncthreads();
    const int ncols = cl + cr;
    for (int c0 = 0; c0 < ncols; c0 += kMvCols) {
      const int cc = tid % kMvCols;
      const int g = c0 + cc;
      const int col = g < cl ? g - cl : bw + (g - cl);   // relative to the block's first column
      // every slot's source is read, from a clamped row and column (an unused
      // slot's entry is never written back), all loads before the first store
      const int gc = min(g, ncols - 1);
      const int colc = gc < cl ? gc - cl : bw + (gc - cl);
      constexpr int kPer = 2 * BW / (NT / kMvCols);
      double mvv[kPer];
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int sl = min(tid / kMvCols + t * (NT / kMvCols), ntouch - 1);
        mvv[t] = A[(size_t)max(es.row[es.label[sl]], 0) * lda + colc];
      }
#pragma unroll
      for (int t = 0; t < kPer; ++t) {
        const int sl = tid / kMvCols + t * (NT / kMvCols);
        if (sl < ntouch) es.mv[sl][cc] = mvv[t];
      }
      __syncthreads();
      for (int sl = tid / kMvCols; sl < ntouch; sl += NT / kMvCols) {
        const int src = es.label[sl];
        if (g < ncols && es.row[sl] >= 0 && src != sl) A[(size_t)es.row[sl] * lda + col] = es.mv[sl][cc];
      }
      __syncthreads();
    }
  }
  if (ns <= 0) return;
  // the rest of the triangle: its lb rows above the block, and the block's
  // rows in the lb columns to its left (those rows were interchanged above)
  const int nt = lb + bw;
  for (int e = tid; e < nt * lb; e += NT) {
    const int r = e / lb, q = e % lb;
    es.T[r][q] = q < r ? (double)A[(ptrdiff_t)(r - lb) * lda + (q - lb)] : 0.0;
  }
  __syncthreads();
  // A12 := trilu(T)^-1 A12 on the first ns right columns, one column per thread
  constexpr int TM = BW + LB;
  typedef __attribute__((address_space(3))) double ldouble;
  ldouble(*Tl)[kTriMax + 1] = (ldouble(*)[kTriMax + 1])(es.T);
  for (int j = tid; j < ns; j += NT) {
    double x[TM];
    gdouble* colp = A + bw + j - (ptrdiff_t)lb * lda;
#pragma unroll
    for (int r = 0; r < TM; ++r) x[r] = (r < nt) ? colp[(size_t)r * lda] : 0.0;
    // column by column: x[r] -= T[r][q] x[q] for r > q, so every x[r]
    // receives its terms in the order q = 0, 1, ... of row-wise substitution;
    // T is read through an LDS pointer (ds_read, not flat loads), column q at
    // its step (the scheduling barrier keeps the compiler from reading the
    // whole triangle into registers up front)
#pragma unroll
    for (int q = 0; q < TM - 1; ++q) {
      __builtin_amdgcn_sched_barrier(0);
      if (q < nt - 1) {
        const double xq = x[q];
#pragma unroll
        for (int r = q + 1; r < TM; ++r)
          if (r < nt) x[r] = x[r] - Tl[r][q] * xq;
      }
    }
#pragma unroll
    for (int r = 1; r < TM; ++r)
      if (r < nt) colp[(size_t)r * lda] = x[r];
  }
}

template <int BW, int MAXW, int KR>
__global__ __launch_bounds__(NT) void k_panel(double* __restrict__ A, int lda, int m, int bw, int row0,
                                              int32_t* __restrict__ ipiv, int32_t* __restrict__ info,
                                              PanelWork* __restrict__ work, int nwg, unsigned epoch, int cl,
                                              int cr, int ns, int lb, const int32_t* __restrict__ skip) {
  static_assert(BW % U == 0, "BW must be a multiple of U");
  // the flag was written by an earlier launch on the stream, so every
  // workgroup reads the same value and they all leave or all stay
  if (skip != nullptr && *skip != 0) return;
  __shared__ __attribute__((aligned(16))) double s_cand[2][NWAVE][BW];
  __shared__ __attribute__((aligned(16))) double s_drow[2][BW];
  __shared__ __attribute__((aligned(16))) double s_prow[2][BW];
  __shared__ PanelShared sh;

  Panel<BW, MAXW, KR> P;
  P.A = A;
  P.lda = lda;
  P.m = m;
  P.bw = bw;
  P.info = info;
  P.nwg = nwg;
  P.wg = blockIdx.x;
  P.tid = threadIdx.x;
  P.lane = threadIdx.x & 63;
  P.wave = threadIdx.x >> 6;
  P.epoch = epoch;
  P.rs = rsrc_of(work);
  P.wbase = reinterpret_cast<const char*>(work);
  P.s_cand = s_cand;
  P.s_drow = s_drow;
  P.s_prow = s_prow;
  P.sh = &sh;
  if (P.wg == 0) {
    P.rows[0] = P.tid;
#pragma unroll
    for (int k = 1; k < KR; ++k) P.rows[k] = kRowNone;
  } else {
#pragma unroll
    for (int k = 0; k < KR; ++k) P.rows[k] = NT + (P.wg - 1) * KR * NT + k * NT + P.tid;
  }
  if (P.tid == 0) sh.zero_col = -1;
  P.load();

  bool done = false;
  if (m > kWave && work->spec_off == 0u) {
    const int fail = P.spec_pass();
    if (P.verify(fail) >= bw) {
      done = true;
    } else {
      if (P.wg == 0 && P.tid == 0) work->spec_off = 1u;
      if (P.tid == 0) sh.zero_col = -1;
      P.load();
      lds_sync();
    }
  }
  if (!done) P.exact_pass();

  P.store();
  if (P.wg == 0) {
    lds_sync();
    for (int c = P.tid; c < bw; c += NT) ipiv[c] = row0 + sh.piv[c] + 1;
    if (P.tid == 0 && sh.zero_col >= 0) atomicCAS(info, 0, row0 + sh.zero_col + 1);
    if (cl > 0 || cr > 0) {
      __shared__ EpilogueShared es;
      if (P.tid < bw) {
#pragma unroll
        for (int c = 0; c < BW; ++c) es.T[lb + P.tid][lb + c] = (c < P.tid) ? P.v[0][c] : 0.0;
      }
      if constexpr (BW > kPanelRegCols) {
        panel_epilogue<BW, 0>(A, lda, bw, cl, cr, ns, sh.piv, P.tid, &es);
      } else {
        if (lb == 0) panel_epilogue<BW, 0>(A, lda, bw, cl, cr, ns, sh.piv, P.tid, &es);
        else panel_epilogue<BW, kPanelRegCols>(A, lda, bw, cl, cr, ns, sh.piv, P.tid, &es);
      }
    }
  }
}

template <int BW>
hipError_t launch_panel(hipStream_t s, double* A, int lda, int m, int bw, int row0, int32_t* ipiv,
                        int32_t* info, PanelWork* work, unsigned epoch, int cl, int cr, int ns, int lb,
                        const int32_t* skip) {
  if constexpr (BW > kPanelRegCols) {   // wide blocks: one row per thread, at most kPanelWideWG workers
    const int nwg = m <= NT ? 1 : 1 + (m - NT + NT - 1) / NT;
    if (nwg > kPanelWideWG) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_panel<BW, kPanelWideWG, 1>), dim3(nwg), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv, info,
                       work, nwg, epoch, cl, cr, ns, lb, skip);
  } else {
    // one row per thread while that takes at most 32 workers (half the work
    // per thread in every column step), two rows per thread beyond
    const int nwg1 = m <= NT ? 1 : 1 + (m - NT + NT - 1) / NT;
    if (nwg1 <= 16) {
      hipLaunchKernelGGL((k_panel<BW, 16, 1>), dim3(nwg1), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv, info, work,
                         nwg1, epoch, cl, cr, ns, lb, skip);
      return hipGetLastError();
    }
    if (nwg1 <= 32) {
      hipLaunchKernelGGL((k_panel<BW, kPanelMaxWG, 1>), dim3(nwg1), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv,
                         info, work, nwg1, epoch, cl, cr, ns, lb, skip);
      return hipGetLastError();
    }
    const int nwg = m <= NT ? 1 : 1 + (m - NT + 2 * NT - 1) / (2 * NT);
    if (nwg > kPanelMaxWG) return hipErrorInvalidValue;
    if (nwg <= 16)
      hipLaunchKernelGGL((k_panel<BW, 16, 2>), dim3(nwg), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv, info, work,
                         nwg, epoch, cl, cr, ns, lb, skip);
    else
      hipLaunchKernelGGL((k_panel<BW, kPanelMaxWG, 2>), dim3(nwg), dim3(NT), 0, s, A, lda, m, bw, row0, ipiv,
                         info, work, nwg, epoch, cl, cr, ns, lb, skip);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t panel_factor(hipStream_t s, double* A, int lda, int m, int bw, int row0, int32_t* ipiv,
                        int32_t* info, PanelWork* work, unsigned epoch, int cl, int cr, const int32_t* skip,
                        int ns, int lb) {
  if (m <= 0 || bw <= 0) return hipSuccess;
  if (bw > kPanelWideCols || bw > m || m > kPanelMaxRows || cl < 0 || cr < 0) return hipErrorInvalidValue;
  if (bw > kPanelRegCols && m > kPanelWideRows) return hipErrorInvalidValue;
  if (ns < 0) ns = cr;
  if (ns > cr || (lb != 0 && lb != kPanelRegCols) || lb > cl || (lb != 0 && bw > kPanelRegCols))
    return hipErrorInvalidValue;
  ipiv += row0;
  if (bw <= 8) return launch_panel<8>(s, A, lda, m, bw, row0, ipiv, info, work, epoch, cl, cr, ns, lb, skip);
  if (bw <= 16) return launch_panel<16>(s, A, lda, m, bw, row0, ipiv, info, work, epoch, cl, cr, ns, lb, skip);
  return launch_panel<32>(s, A, lda, m, bw, row0, ipiv, info, work, epoch, cl, cr, ns, lb, skip);
}

size_t workspace_bytes() { return (sizeof(Workspace) + 4095) / 4096 * 4096; }

}  // namespace mlu

#ifdef MLU_PANEL_PROBE
// The stamps of the last instrumented panel call (2 x 64 x 6 values).
extern "C" int mlu_probe_stamps(unsigned long long* host) {
  return hipMemcpyFromSymbol(host, HIP_SYMBOL(mlu::g_probe_stamps), sizeof(mlu::g_probe_stamps)) == hipSuccess ? 0
                                                                                                             : -1;
}
#endif
