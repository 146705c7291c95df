// Fused, register-resident kernel for Algorithm 3 of Wolf et al. (arXiv
// 2108.10565, section "Block-wise back-substitution"), one object per degree
// N = STP_DEGREE.
//
// Mapping.  One lane per column (element e, quantity p, time mode u) of the
// element's right-hand side b_pmu (eq:b_pmu); kNQ (N+1) lanes per element,
// kElems elements per workgroup (512 lanes at most), lanes ordered
// quantity-major.
// Every lane keeps b[m] for all modes m below the top degree block in
// registers.  The green-block update
//     b[p, n, u] -= sum_j Khat^j[n, m] (A^{j*} X[:, m, u])_p ,  n < block_start(g)
// is lane-local once the star product y_j = (A^{j*} X[:, m, u])_p is known,
// so the lane applies it as a fully unrolled list of fused multiply-adds
// over the non-zeros of Khat (compile-time pattern, coefficients read with
// scalar loads from a device table), exactly the zeros the Lemma of section
// "Structure of the system matrix" and the Dubiner structure provide.
//
// Per chunk of up to kChunkMax modes m of degree block g (g = N .. 0):
//   1. every lane writes b[m] to LDS (top block: b = Q0 (S^-1 w), eq:b_pmu);
//   2. dark-blue blocks and G coupling: lane (e, p, s) forms X[p, m, s] =
//      row s of (Z - E*_pp I)^-1 times b[p, m, :] (float64).  For E*_pp = 0
//      that row is a row of Z^-1, which is tridiagonal with a zero diagonal
//      apart from its two corner entries (the Legendre integration
//      recurrence), so such lanes read two entries of b instead of T; the
//      dense rows are read only by waves holding a lane that needs them.
//      A quantity o whose row of the strict upper part G of E* holds one
//      coupling G_op to an uncoupled quantity p (the poroelastic u <- uf,
//      v <- vf, w <- wf) uses the closed form
//      X_o = Zinv_o (b_o + G_op X_p) = zr . b_o + dr . b_p,
//      dr = G_op (row of Zinv_o) Zinv_p, so no extra round is needed; any
//      other upper-triangular E is handled level by level (level = longest
//      coupling chain below a quantity);
//   3. X of the chunk goes from LDS to Q (and dt X[:, :, 0] to Qint) in
//      contiguous runs, with streaming stores issued before and early in
//      step 4;
//   4. green blocks: every lane reads X[q, m, u] of the quantities in its
//      star row, forms y_1..y_3 with its row of A^{1*}, A^{2*}, A^{3*}, and
//      subtracts Khat^j[n, m] y_j from its registers b[n].
// A^{j*} = dt A^j and E* = dt E are formed in-kernel, so every product runs
// with unit scaling (the paper's libxsmm alpha = 1 remark, section "Roofline
// model").
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "generated/khat_tables.h"

#ifndef STP_DEGREE
#error "compile once per degree with -DSTP_DEGREE=N"
#endif

namespace stp {
namespace {

// Quantities of the system this object is compiled for: 13 (poroelastic) or
// 6 (damped Maxwell, section "Other applications").
#ifndef STP_NQ
#error "compile once per quantity count with -DSTP_NQ=Q"
#endif
constexpr int kNQ = STP_NQ;
static_assert(supported_nq(kNQ), "quantity count without kernels");

// Tile shape of this degree: threads per workgroup (upper bound; rounded to
// whole elements and waves) and modes per chunk (degree blocks are split
// evenly).  Both come from the build, which takes them from the table the
// autotuner writes after timing every candidate shape on the device.
#if !defined(STP_TILE_THREADS) || !defined(STP_TILE_CHUNK)
#error "compile with -DSTP_TILE_THREADS=T -DSTP_TILE_CHUNK=C (the tile table of the build)"
#endif
constexpr int kTileThreadsN = STP_TILE_THREADS;
constexpr int kChunkMax = STP_TILE_CHUNK;
static_assert(kTileThreadsN >= 64 && kTileThreadsN <= 1024 && kChunkMax >= 1, "tile shape");
constexpr int kMaxElems = 16;
// Non-zero columns kept per lane of a star-matrix row (union over the three
// directions).  The poroelastic Jacobians need at most 6 (normal-stress and
// pressure rows couple to the 6 velocities; velocity rows to 3 stresses and
// the pressure); a workgroup holding any row with more falls back to reading
// the dense rows from global memory.
constexpr int kStarNnz = 6;

template <int I>
using ic = std::integral_constant<int, I>;
using ConstUint = __attribute__((address_space(4))) const unsigned;

template <int Begin, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(ic<Begin + I>{}), ...);
}
// Calls f(ic<i>) for i = Begin .. End-1 with compile-time i.
template <int Begin, int End, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (End > Begin) static_for_impl<Begin>(f, std::make_integer_sequence<int, End - Begin>{});
}

// Smallest S >= len with nq S = t (mod 16) (nq odd), or the smallest odd
// S >= len (nq even, where no such S exists for odd t).
__host__ __device__ constexpr int stride_for(int len, int t, int nq) {
  for (int s = len; s < len + 32; ++s) {
    if (nq % 2 == 1 ? ((nq * s - t) % 16 + 16) % 16 == 0 : s % 2 == 1) return s;
  }
  return len;
}

template <int N>
struct Cfg {
  static constexpr int B = n_modes(N);
  static constexpr int T = N + 1;
  static constexpr int LN = block_start(N);        // register-resident rows (below the top block)
  static constexpr int LR = LN > 0 ? LN : 1;
  static constexpr int DN = block_size(N);         // modes of the top block (largest block)
  static constexpr int kCols = kNQ * T;            // lanes per element
  static constexpr int kElems =                    // elements per workgroup
      (kTileThreadsN / kCols) < kMaxElems ? (kTileThreadsN / kCols) : kMaxElems;
  static_assert(kElems >= 1, "the tile must hold at least one element");
  static constexpr int kThreads = (kElems * kCols + 63) / 64 * 64;
  static constexpr int kSlots = kElems + 1;        // + one dummy slot for spare lanes
  static constexpr int kChunk = kChunkMax < DN ? kChunkMax : DN;
  // The chunk buffers hold one block of S doubles per (element, quantity) row
  // in the order of the rows in memory (element-major), so a row's block is
  // row * S: the output passes address LDS and memory from the same row
  // index.  S is padded so that kNQ S = T (mod 16) when kNQ is odd: the LDS
  // address of lane (e, p, u) (lanes quantity-major) is then congruent to the
  // lane index modulo 16 doubles, 13 S = 7 making S = 3 = kElems T at N = 6,
  // so 16 consecutive lanes cover one 128-byte span of the banks without a
  // conflict.  One extra block at the end takes the writes of the spare lanes
  // past the last element (their values are never read back).
  static constexpr int kChunkT = kChunk * T;
  static constexpr int S = stride_for(kChunkT, T, kNQ);
  static constexpr int kRows = kElems * kNQ;       // real blocks
  static constexpr int kBufSize = (kRows + 1) * S; // + the spare lanes' block
  // Offset of the block of row `row` = element * kNQ + quantity; rows past
  // the last element (spare lanes, the dummy slot) share the last block.
  static __device__ __forceinline__ int rowblk(int row) { return (row < kRows ? row : kRows) * S; }
  static __device__ __forceinline__ int blk(int e, int q) { return rowblk(e * kNQ + q); }
};

// Degree block g is processed in nchunks(g) chunks of near-equal size.
__host__ __device__ constexpr int nchunks(int g, int cmax) { return (block_size(g) + cmax - 1) / cmax; }
__host__ __device__ constexpr int chunk_size(int g, int cmax, int i) {
  return block_size(g) / nchunks(g, cmax) + (i < block_size(g) % nchunks(g, cmax) ? 1 : 0);
}
__host__ __device__ constexpr int chunk_start(int g, int cmax, int i) {
  return block_start(g) + i * (block_size(g) / nchunks(g, cmax)) +
         (i < block_size(g) % nchunks(g, cmax) ? i : block_size(g) % nchunks(g, cmax));
}

// Lane tid -> (element slot es, quantity p, time mode u), quantity-major:
// the lanes of one quantity are contiguous (kElems * T of them), so the few
// quantities that take the dense dark-blue path (a non-zero diagonal source
// term, or a coupling) occupy few waves and the other waves skip it.  Spare
// lanes past kElems * kCols go to the dummy slot kElems.
template <int N>
struct LaneId {
  int es, p, u;
  __device__ __forceinline__ explicit LaneId(int tid) {
    using C = Cfg<N>;
    constexpr int per_q = C::kElems * C::T;
    if (tid < C::kElems * C::kCols) {
      p = tid / per_q;
      es = (tid % per_q) / C::T;
      u = tid % C::T;
    } else {
      const int i = tid - C::kElems * C::kCols;
      es = C::kElems;
      p = (i / C::T) % kNQ;
      u = i % C::T;
    }
  }
};

template <int N, typename R>
struct Shared {
  using C = Cfg<N>;
  double G[C::kSlots][kNQ][kNQ];            // E* (lower part zeroed)
  double zr[C::kThreads][C::T];             // per lane (e, p, u): row u of (Z - E*_pp I)^-1
  double dr[C::kThreads][C::T];             // per lane: row of Zinv_o G_op Zinv_p (closure coupling)
  int level[C::kSlots][kNQ];
  int maxlevel;
  unsigned flags;
  union {
    double A[C::kSlots][3][kNQ][kNQ];       // setup only: A^{j*} = dt A^j
    struct {
      R bufB[C::kBufSize];                  // b of the chunk: [e][p] blocks of [chunk][T], stride S
      R bufX[C::kBufSize];                  // X of the chunk, same layout
    } c;
  } u;
};

// Solves (Z - z I)^T y = rhs by Gauss-Jordan elimination without pivoting.
// For z = dt E_pp < 0.5 (the range stp_validate admits) the pivots stay away
// from zero: over z in [-1e7, 0.5) and every degree N <= 7 the smallest is at
// least 3% of max|Z| + |z| (checked numerically).  With rhs = e_s, y is row s
// of (Z - z I)^-1.
template <int T>
__device__ __forceinline__ void zt_solve(double z, const double (&rhs)[T], double (&out)[T]) {
  double a[T][T + 1];
#pragma unroll
  for (int r = 0; r < T; ++r) {
#pragma unroll
    for (int c = 0; c < T; ++c) a[r][c] = z_entry(c, r) - (r == c ? z : 0.0);  // transpose
    a[r][T] = rhs[r];
  }
#pragma unroll
  for (int k = 0; k < T; ++k) {
    const double inv = 1.0 / a[k][k];
#pragma unroll
    for (int c = k; c <= T; ++c) a[k][c] *= inv;
#pragma unroll
    for (int r = 0; r < T; ++r) {
      if (r == k) continue;
      const double f = a[r][k];
#pragma unroll
      for (int c = k; c <= T; ++c) a[r][c] -= f * a[k][c];
    }
  }
#pragma unroll
  for (int r = 0; r < T; ++r) out[r] = a[r][T];
}

// The usage-ordered Khat table of degree N in precision R.  Kernels pass its
// address through an empty asm statement before reading it, so the compiler
// cannot fold the values into instruction literals and reads them with
// scalar loads instead.
template <int N, typename R>
__device__ __forceinline__ const R* khat_sparse() {
  if constexpr (sizeof(R) == 8) {
    if constexpr (N == 0) return stp_gen::kKhatSparse0;
    else if constexpr (N == 1) return stp_gen::kKhatSparse1;
    else if constexpr (N == 2) return stp_gen::kKhatSparse2;
    else if constexpr (N == 3) return stp_gen::kKhatSparse3;
    else if constexpr (N == 4) return stp_gen::kKhatSparse4;
    else if constexpr (N == 5) return stp_gen::kKhatSparse5;
    else if constexpr (N == 6) return stp_gen::kKhatSparse6;
    else return stp_gen::kKhatSparse7;
  } else {
    if constexpr (N == 0) return stp_gen::kKhatSparseF0;
    else if constexpr (N == 1) return stp_gen::kKhatSparseF1;
    else if constexpr (N == 2) return stp_gen::kKhatSparseF2;
    else if constexpr (N == 3) return stp_gen::kKhatSparseF3;
    else if constexpr (N == 4) return stp_gen::kKhatSparseF4;
    else if constexpr (N == 5) return stp_gen::kKhatSparseF5;
    else if constexpr (N == 6) return stp_gen::kKhatSparseF6;
    else return stp_gen::kKhatSparseF7;
  }
}

// Register pinning: an empty asm statement that reads (or reads and writes)
// a register value.  Volatile asm statements keep their program order, so
// these fix where a value must be complete and stop the compiler from
// sinking pure arithmetic or hoisting loads across them.
template <typename T>
__device__ __forceinline__ void pin_v(T& x) { asm volatile("" : "+v"(x)); }
template <typename T>
__device__ __forceinline__ void use_s(T x) { asm volatile("" ::"s"(x)); }

// Coefficients per scalar load: one s_load_dwordx16 (64 bytes).
template <typename R>
constexpr int kGroup = 64 / static_cast<int>(sizeof(R));

// Loads the coefficients [g0, g0 + gn) of the usage-ordered Khat table into
// scalar registers, from an address the compiler cannot see through.
template <typename R, int g0, int gn>
__device__ __forceinline__ void load_group(const R* kv, R (&v)[kGroup<R>]) {
  using CR = __attribute__((address_space(4))) const R;
  const R* kp = kv + g0;
  asm volatile("" : "+s"(kp));
  const CR* kc = (const CR*)kp;
#pragma unroll
  for (int i = 0; i < gn; ++i) v[i] = kc[i];
}

// Brings the Khat coefficients of columns [M0, M0 + CNT) into the scalar
// data cache: wave w loads one dword of each line w, w + nwaves, ... of the
// range (64-byte lines, table 64-byte aligned), issuing every load before
// waiting once, so the line fetches overlap each other and the other waves'
// work; the per-group loads of the green update then hit the cache.
template <int N, typename R, int M0, int CNT, int NWAVES>
__device__ __forceinline__ void prefetch_columns(const R* kv, int wave) {
  using P = stp_gen::KhatPattern<N>;
  constexpr int per_line = 64 / static_cast<int>(sizeof(R));
  constexpr int first = P::col_start[M0];
  constexpr int last = P::col_start[M0 + CNT - 1] + P::col_count[M0 + CNT - 1];
  if constexpr (last > first) {
    constexpr int line0 = first / per_line, line1 = (last + per_line - 1) / per_line;
    constexpr int per_wave = (line1 - line0 + NWAVES - 1) / NWAVES;
    const R* kp = kv + (line0 + wave) * per_line;
    asm volatile("" : "+s"(kp));
    const ConstUint* kc = (const ConstUint*)kp;
    const int avail = line1 - line0 - wave;  // lines this wave may touch: k * NWAVES < avail
    unsigned v[per_wave];
#pragma unroll
    for (int k = 0; k < per_wave; ++k) v[k] = (k * NWAVES < avail) ? kc[k * NWAVES * 16] : 0u;
#pragma unroll
    for (int k = 0; k < per_wave; ++k) asm volatile("" ::"s"(v[k]));
  }
}

// First coefficient group of column M of the usage-ordered Khat table
// (possibly partial), issued into `grp` without waiting for it.
template <int N, int M, typename R>
__device__ __forceinline__ void load_first_group(const R* kv, R (&grp)[kGroup<R>]) {
  using P = stp_gen::KhatPattern<N>;
  constexpr int GS = kGroup<R>;
  constexpr int count = P::col_count[M];
  if constexpr (count > 0) load_group<R, P::col_start[M], (count < GS ? count : GS)>(kv, grp);
}

// b[n] -= Khat^j[n, M] y_j for the non-zeros of column M (usage order of the
// generated pattern: directions, then rows ascending), in groups of
// kGroup<R> coefficients.  `cur` arrives holding the column's first group
// (issued earlier by load_first_group or by the previous column); each
// group's fused multiply-adds run while the next group's scalar load is in
// flight, and the last group issues the first group of column MNext (< 0:
// none), so that a column starts without waiting for its coefficients.
template <int N, int M, int MNext, typename R>
__device__ __forceinline__ void green_column(R (&b)[Cfg<N>::LR], R y0, R y1, R y2, const R* kv, R (&cur)[kGroup<R>]) {
  using P = stp_gen::KhatPattern<N>;
  constexpr int GS = kGroup<R>;
  constexpr int start = P::col_start[M];
  constexpr int count = P::col_count[M];
  constexpr int ngroups = (count + GS - 1) / GS;
  constexpr bool kNext = MNext >= 0 && MNext < Cfg<N>::B;
  constexpr int next_count = kNext ? P::col_count[kNext ? MNext : 0] : 0;
  if constexpr (count == 0) {
    if constexpr (next_count > 0) load_first_group<N, (kNext ? MNext : 0), R>(kv, cur);
  } else {
#pragma unroll
    for (int i = 0; i < (count < GS ? count : GS); ++i) use_s(cur[i]);
    static_for<0, ngroups>([&](auto G) __attribute__((always_inline)) {
      constexpr int gi = decltype(G)::value;
      constexpr int g0 = start + gi * GS;
      constexpr int gn = (start + count - g0) < GS ? (start + count - g0) : GS;
      constexpr int g1 = g0 + GS;
      constexpr int gn1 = (start + count - g1) < GS ? (start + count - g1) : GS;
      constexpr bool kLast = gi + 1 == ngroups;
      constexpr int nload = kLast ? (next_count < GS ? next_count : GS) : gn1;
      R nxt[GS];
      if constexpr (!kLast) load_group<R, g1, gn1>(kv, nxt);
      else if constexpr (next_count > 0) load_first_group<N, (kNext ? MNext : 0), R>(kv, nxt);
      static_for<0, gn>([&](auto I) __attribute__((always_inline)) {
        constexpr int e = g0 + decltype(I)::value;
        constexpr int n = P::row[e];
        constexpr int j = P::dir[e];
        const R y = (j == 0) ? y0 : ((j == 1) ? y1 : y2);
        b[n] = fma(-cur[decltype(I)::value], y, b[n]);
      });
      static_for<0, gn>([&](auto I) __attribute__((always_inline)) {
        pin_v(b[P::row[g0 + decltype(I)::value]]);
      });
      if constexpr (!kLast) {
#pragma unroll
        for (int i = 0; i < nload; ++i) {
          use_s(nxt[i]);
          cur[i] = nxt[i];
        }
      } else if constexpr (nload > 0) {
        // the next column's first group: handed over without waiting here
#pragma unroll
        for (int i = 0; i < nload; ++i) cur[i] = nxt[i];
      }
    });
  }
}

// Copies columns [m0 T, m0 T + PER) of the (element, quantity) rows of the
// group (a [n][kNQ][B T] array in memory) into the chunk buffer `buf` (block
// layout of Cfg::blk), converted to R.  Every lane issues all its loads
// before its LDS stores, so the group waits for one memory latency, not one
// per row segment.
template <int N, typename R, int PER, typename Src>
__device__ __forceinline__ void stage_rows(R* buf, const Src* src, int64_t e0, int m0T, int nloc, int tid) {
  using C = Cfg<N>;
  constexpr int kIters = (C::kElems * kNQ * PER + C::kThreads - 1) / C::kThreads;
  const int limit = nloc * kNQ * PER;
  Src v[kIters];
#pragma unroll
  for (int k = 0; k < kIters; ++k) {
    const int i = tid + k * C::kThreads;
    const int row = i / PER, r = i % PER;
    v[k] = i < limit ? src[(e0 * kNQ + row) * (C::B * C::T) + m0T + r] : Src(0);
  }
#pragma unroll
  for (int k = 0; k < kIters; ++k) {
    const int i = tid + k * C::kThreads;
    const int row = i / PER, r = i % PER;
    if (i < limit) buf[C::rowblk(row) + r] = static_cast<R>(v[k]);
  }
}

// The two halves of stage_rows, for callers that overlap the loads with
// other work: the loads of columns [m0 T, m0 T + PER) into registers, then
// their stores into the chunk buffer.
template <int N, int PER>
struct RowStage {
  using C = Cfg<N>;
  static constexpr int kIters = (C::kElems * kNQ * PER + C::kThreads - 1) / C::kThreads;
  double v[kIters];
  __device__ __forceinline__ void issue(const double* src, int64_t e0, int m0T, int nloc, int tid) {
    const int limit = nloc * kNQ * PER;
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
      const int i = tid + k * C::kThreads;
      const int row = i / PER, r = i % PER;
      v[k] = i < limit ? src[(e0 * kNQ + row) * (C::B * C::T) + m0T + r] : 0.0;
    }
  }
  __device__ __forceinline__ void commit(double* buf, int nloc, int tid) const {
    const int limit = nloc * kNQ * PER;
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
      const int i = tid + k * C::kThreads;
      const int row = i / PER, r = i % PER;
      if (i < limit) buf[C::rowblk(row) + r] = v[k];
    }
  }
};

// Q0 of the CM modes starting at m0 of the group, [element][quantity][mode],
// in the same two halves.
template <int N, int CM>
struct Q0Stage {
  using C = Cfg<N>;
  static constexpr int kIters = (C::kElems * kNQ * CM + C::kThreads - 1) / C::kThreads;
  double v[kIters];
  __device__ __forceinline__ void issue(const double* Q0, int64_t e0, int m0, int nloc, int tid) {
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
      const int i = tid + k * C::kThreads;
      v[k] = i < nloc * kNQ * CM ? Q0[(e0 * kNQ + i / CM) * C::B + m0 + i % CM] : 0.0;
    }
  }
  __device__ __forceinline__ void commit(double* buf, int nloc, int tid) const {
#pragma unroll
    for (int k = 0; k < kIters; ++k) {
      const int i = tid + k * C::kThreads;
      if (i < nloc * kNQ * CM) buf[i] = v[k];
    }
  }
};

// Position of chunk ci of degree block g in the chunk order (blocks from N
// down, chunks ascending), and the chunk that follows it.
__host__ __device__ constexpr int chunk_index(int N, int g, int ci, int cmax) {
  int s = 0;
  for (int h = N; h > g; --h) s += nchunks(h, cmax);
  return s + ci;
}
__host__ __device__ constexpr int next_block(int g, int ci, int cmax) { return ci + 1 < nchunks(g, cmax) ? g : g - 1; }
__host__ __device__ constexpr int next_chunk(int g, int ci, int cmax) { return ci + 1 < nchunks(g, cmax) ? ci + 1 : 0; }

// Modes of the solve kernel.
constexpr int kInit = 0;     // b = Q0 (S^-1 w); Q <- X
constexpr int kCorrect = 1;  // b = residual (float workspace); Q <- Q + X

// Per-lane setup shared by the solve and residual kernels: stages E* and
// A^{j*} of the group, then per lane the sparse star row, the G coupling of
// the lane's quantity, row u of (Z - E*_pp I)^-1 (to LDS) and the closure row
// dr (to LDS); the dependency levels of the strict upper part G of E* only
// when some coupling is not of the closure form.
template <int N, typename R>
struct LaneSetup {
  using C = Cfg<N>;
  R sa0[kStarNnz], sa1[kStarNnz], sa2[kStarNnz];
  int sq[kStarNnz];
  // LDS addresses of the star-row entries in one fixed chunk buffer (bind):
  // the reads of each mode then take the mode's offset as an immediate
  using LdsR = __attribute__((address_space(3))) const R;
  LdsR* sp[kStarNnz];
  int gp, gcount;
  double gcoef;
  bool dense_star, closure;
  int maxlevel, mylevel;

  __device__ __forceinline__ void run(Shared<N, R>& sh, const PredictArgs& a, int64_t e0, int nloc, int tid,
                                      int es, int p, int u, bool active, int cb) {
    constexpr int kThreads = C::kThreads, T = C::T;
    unsigned bad = 0;  // input conditions the elimination without pivoting cannot take
    // E and the star matrices of the group: every load is issued before the
    // first LDS store, so the group waits for one memory latency
    constexpr int kEIt = (C::kSlots * kNQ * kNQ + kThreads - 1) / kThreads;
    constexpr int kAIt = (C::kSlots * 3 * kNQ * kNQ + kThreads - 1) / kThreads;
    double ev[kEIt], av[kAIt];
#pragma unroll
    for (int k = 0; k < kEIt; ++k) {
      const int i = tid + k * kThreads;
      ev[k] = i < nloc * kNQ * kNQ ? a.E[e0 * (kNQ * kNQ) + i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kAIt; ++k) {
      const int i = tid + k * kThreads;
      av[k] = i < nloc * 3 * kNQ * kNQ ? a.star[e0 * (3 * kNQ * kNQ) + i] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kEIt; ++k) {
      const int i = tid + k * kThreads;
      const int r = (i / kNQ) % kNQ, c = i % kNQ;
      const double v = a.dt * ev[k];
      if (c < r && v != 0.0) bad |= kInputNotUpper;
      if (c == r && v >= 0.5) bad |= kInputSingular;
      if (i < C::kSlots * kNQ * kNQ) (&sh.G[0][0][0])[i] = c >= r ? v : 0.0;
    }
    if (bad && a.status) atomicOr(a.status, bad);
#pragma unroll
    for (int k = 0; k < kAIt; ++k) {
      const int i = tid + k * kThreads;
      if (i < C::kSlots * 3 * kNQ * kNQ) (&sh.u.A[0][0][0][0])[i] = a.dt * av[k];
    }
    if (tid == 0) {
      sh.maxlevel = 0;
      sh.flags = 0;
    }
    __syncthreads();
    // G coupling of this lane's quantity (the first non-zero right of the
    // diagonal and their count), and whether that partner couples further
    gcount = 0;
    gp = p;
    gcoef = 0.0;
#pragma unroll
    for (int q = 1; q < kNQ; ++q) {
      const double gq = sh.G[es][p][q];
      if (q > p && gq != 0.0) {
        if (gcount == 0) {
          gcoef = gq;
          gp = q;
        }
        ++gcount;
      }
    }
    bool partner_coupled = false;
#pragma unroll
    for (int q = 1; q < kNQ; ++q)
      partner_coupled = partner_coupled || (q > gp && sh.G[es][gp][q] != 0.0);
    // sparse row p of the three star matrices: the columns with a non-zero
    // in any direction, in ascending order (a bit mask, consumed lowest bit
    // first)
    unsigned mask = 0;
#pragma unroll
    for (int q = 0; q < kNQ; ++q) {
      const double v0 = sh.u.A[es][0][p][q], v1 = sh.u.A[es][1][p][q], v2 = sh.u.A[es][2][p][q];
      if (v0 != 0.0 || v1 != 0.0 || v2 != 0.0) mask |= 1u << q;
    }
    const bool overflow = active && __builtin_popcount(mask) > kStarNnz;
#pragma unroll
    for (int k = 0; k < kStarNnz; ++k) {
      const bool live = mask != 0;
      const int q = live ? __builtin_ctz(mask) : p;
      mask &= mask - 1;
      const double v0 = sh.u.A[es][0][p][q], v1 = sh.u.A[es][1][p][q], v2 = sh.u.A[es][2][p][q];
      sa0[k] = live ? static_cast<R>(v0) : R(0);
      sa1[k] = live ? static_cast<R>(v1) : R(0);
      sa2[k] = live ? static_cast<R>(v2) : R(0);
      sq[k] = (live ? C::blk(es, q) : cb) + u;
    }
    // row u of (Z - E*_pp I)^-1.  Without a diagonal source it is row u of
    // Z^-1, which has two non-zeros (generated table); otherwise it comes from
    // an elimination, done only by waves holding such a lane.
    {
      const double z = sh.G[es][p][p];
      using ZS = stp_gen::ZinvSparse<N>;
      double zr[T];
#pragma unroll
      for (int v = 0; v < T; ++v)
        zr[v] = (ZS::col[2 * u] == v ? ZS::val[2 * u] : 0.0) + (ZS::col[2 * u + 1] == v ? ZS::val[2 * u + 1] : 0.0);
      if (__builtin_amdgcn_ballot_w64(z != 0.0) != 0) {
        double e_u[T], zs[T];
#pragma unroll
        for (int v = 0; v < T; ++v) e_u[v] = (v == u) ? 1.0 : 0.0;
        zt_solve<T>(z, e_u, zs);
        if (z != 0.0) {
#pragma unroll
          for (int v = 0; v < T; ++v) zr[v] = zs[v];
        }
      }
#pragma unroll
      for (int v = 0; v < T; ++v) sh.zr[tid][v] = zr[v];
    }
    // one barrier for the workgroup-uniform flags (scalar branches, no exec
    // masking); it also orders the reads of A before the chunk buffers (which
    // share its storage) are written, and the rows of Zinv before their reads
    // below.  The closure form of the coupling applies when every coupled
    // quantity couples to one quantity that itself is uncoupled (the
    // poroelastic case).
    {
      const unsigned f = (overflow ? 1u : 0u) | ((active && (gcount > 1 || (gcount == 1 && partner_coupled))) ? 2u : 0u);
      if (f) atomicOr(&sh.flags, f);
    }
    __syncthreads();
    const unsigned flags = __builtin_amdgcn_readfirstlane(sh.flags);
    dense_star = (flags & 1u) != 0;
    closure = (flags & 2u) == 0;
    // closure row: X_o = Zinv_o (b_o + g X_p) = zr . b_o + dr . b_p with
    //   dr[w] = g sum_v (row u of Zinv_o)[v] Zinv_p[v][w],
    // the rows Zinv_p[v] being those of the partner's lanes (e, p, v)
    {
      double dr[T];
#pragma unroll
      for (int w = 0; w < T; ++w) dr[w] = 0.0;
      if (gcount == 1 && closure) {
        constexpr int per_q = C::kElems * T;
        double zr[T];
#pragma unroll
        for (int v = 0; v < T; ++v) zr[v] = sh.zr[tid][v];
#pragma unroll
        for (int v = 0; v < T; ++v) {
          const double cv = gcoef * zr[v];
#pragma unroll
          for (int w = 0; w < T; ++w) dr[w] = fma(cv, sh.zr[gp * per_q + es * T + v][w], dr[w]);
        }
      }
#pragma unroll
      for (int v = 0; v < T; ++v) sh.dr[tid][v] = dr[v];
    }
    maxlevel = 0;
    mylevel = 0;
    if (!closure) {
      // dependency levels of a general upper-triangular E (level = longest
      // coupling chain below a quantity), one thread per element
      if (tid < nloc) {
        int lev[kNQ];
        int mx = 0;
#pragma unroll
        for (int o = kNQ - 1; o >= 0; --o) {
          int l = 0;
#pragma unroll
          for (int q = o + 1; q < kNQ; ++q)
            if (sh.G[tid][o][q] != 0.0 && lev[q] + 1 > l) l = lev[q] + 1;
          lev[o] = l;
          sh.level[tid][o] = l;
          mx = l > mx ? l : mx;
        }
        atomicMax(&sh.maxlevel, mx);
      }
      __syncthreads();
      maxlevel = sh.maxlevel;
      mylevel = active ? sh.level[es][p] : 0;
    }
  }

  __device__ __forceinline__ void bind(const R* buf) {
#pragma unroll
    for (int k = 0; k < kStarNnz; ++k) sp[k] = (LdsR*)buf + sq[k];
  }
  // star() for the buffer given to bind(): no address arithmetic per mode
  template <int kk>
  __device__ __forceinline__ void star_bound(const R* bufX, const PredictArgs& a, int64_t e0, int es, int p, int u,
                                             bool active, R& y0, R& y1, R& y2) const {
    constexpr int T = C::T;
    y0 = y1 = y2 = R(0);
    if (!dense_star) {
#pragma unroll
      for (int k = 0; k < kStarNnz; ++k) {
        const R xq = sp[k][kk * T];
        y0 = fma(sa0[k], xq, y0);
        y1 = fma(sa1[k], xq, y1);
        y2 = fma(sa2[k], xq, y2);
      }
    } else {
      star<kk>(bufX, a, e0, es, p, u, active, y0, y1, y2);
    }
  }

  // y_j = (A^{j*} X[:, m, u])_p for j = 1..3 from the chunk buffer
  template <int kk>
  __device__ __forceinline__ void star(const R* bufX, const PredictArgs& a, int64_t e0, int es, int p, int u,
                                       bool active, R& y0, R& y1, R& y2) const {
    constexpr int T = C::T;
    y0 = y1 = y2 = R(0);
    // opaque per-mode offset: this mode's LDS reads stay here
    int xoff = kk * T;
    asm volatile("" : "+v"(xoff));
    const R* xs = bufX + xoff;
    if (!dense_star) {
#pragma unroll
      for (int k = 0; k < kStarNnz; ++k) {
        const R xq = xs[sq[k]];
        y0 = fma(sa0[k], xq, y0);
        y1 = fma(sa1[k], xq, y1);
        y2 = fma(sa2[k], xq, y2);
      }
    } else {
      const double* st = a.star + (active ? e0 + es : 0) * (3 * kNQ * kNQ) + p * kNQ;
#pragma unroll
      for (int q = 0; q < kNQ; ++q) {
        const R xq = xs[C::blk(es, q) + u];
        y0 = fma(static_cast<R>(a.dt * st[q]), xq, y0);
        y1 = fma(static_cast<R>(a.dt * st[kNQ * kNQ + q]), xq, y1);
        y2 = fma(static_cast<R>(a.dt * st[2 * kNQ * kNQ + q]), xq, y2);
      }
    }
  }
};

// Algorithm 3 over a group of elements in precision R (the dark-blue solves
// are float64 in every mode).  kInit: b = Q0 (S^-1 w), Q <- X.  kCorrect:
// b = the residual in `rin` (float), Q <- Q + X.
template <int N, typename R, int Mode>
__global__ __launch_bounds__(Cfg<N>::kThreads) void fused_solve_kernel(PredictArgs a, const float* rin) {
  using C = Cfg<N>;
  constexpr int B = C::B, T = C::T, kE = C::kElems, kThreads = C::kThreads;
  __shared__ Shared<N, R> sh;
  R* const bufB = sh.u.c.bufB;
  R* const bufX = sh.u.c.bufX;
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kE;
  const int64_t nloc64 = a.n - e0 < kE ? a.n - e0 : kE;
  const int nloc = static_cast<int>(nloc64);
  const LaneId<N> lid(tid);
  const int es = lid.es, p = lid.p, u = lid.u;
  const bool active = es < nloc;
  const int cb = C::blk(es, p);  // this lane's (element, quantity) block in bufB / bufX
  const R* kv = khat_sparse<N, R>();
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int64_t erow = ((active ? e0 + es : 0) * kNQ + p);  // (element, quantity) row of this lane

  // register rows of b below the top block, loaded after the per-element
  // setup (so that its loads do not wait behind them and its elimination
  // does not compete with them for registers); the float64 rows are scaled
  // just before the first green update, when they have arrived.
  constexpr bool kDeferRows = Mode == kInit && std::is_same_v<R, double>;
  R b[C::LR];
  const double w_u = sinv_w(u);
  const double* const q0row = a.Q0 + erow * B;
  // Q0 of the first chunk (top block): its loads are issued before the
  // per-element setup so that their latency overlaps it; the registers then
  // carry each following top-block chunk, loaded one chunk ahead
  constexpr int kFirstC = chunk_size(N, C::kChunk, 0), kFirstM = chunk_start(N, C::kChunk, 0);
  constexpr int kFirstPer = (kE * kNQ * kFirstC + kThreads - 1) / kThreads;
  double q_first[kFirstPer];
  if constexpr (Mode == kInit) {
#pragma unroll
    for (int k = 0; k < kFirstPer; ++k) {
      const int i = tid + k * kThreads;
      const int ee = i / (kNQ * kFirstC), pp = (i / kFirstC) % kNQ, kk = i % kFirstC;
      q_first[k] = (ee < nloc) ? a.Q0[((e0 + ee) * kNQ + pp) * B + kFirstM + kk] : 0.0;
    }
  }
  LaneSetup<N, R> L;
  L.run(sh, a, e0, nloc, tid, es, p, u, active, cb);
  if constexpr (kDeferRows) {
#pragma unroll
    for (int n = 0; n < C::LN; ++n) b[n] = q0row[n];
  } else if constexpr (Mode == kInit) {
    // b[p, n, u] = Q0[p, n] (S^-1 w)_u (eq:b_pmu), converted on arrival
#pragma unroll
    for (int n = 0; n < C::LN; ++n) b[n] = static_cast<R>(q0row[n] * w_u);
  } else if constexpr (Mode == kCorrect) {
    // the residual rows below the top block (after the setup, like the rows
    // of the float64 solve)
    const float* rrow = rin + erow * (B * T) + u;
#pragma unroll
    for (int n = 0; n < C::LN; ++n) b[n] = static_cast<R>(rrow[n * T]);
  }
  const int pb = C::blk(es, L.gp);  // block of the coupled quantity (own block if uncoupled)
  L.bind(bufX);
  // Quantities without a diagonal source (E*_pp = 0) solve with Z^-1, whose
  // rows have two non-zeros (columns zc0, zc1 of row u); the dense row u of
  // (Z - E*_pp I)^-1 and the closure row dr are read only by waves holding a
  // lane that needs them (wave-uniform flags, scalar branches).
  using ZS = stp_gen::ZinvSparse<N>;
  const int cz0 = cb + ZS::col[2 * u], cz1 = cb + ZS::col[2 * u + 1];
  const double zv0 = ZS::val[2 * u], zv1 = ZS::val[2 * u + 1];
  const bool wave_stiff = __builtin_amdgcn_ballot_w64(sh.G[es][p][p] != 0.0) != 0;
  const bool wave_coupled = __builtin_amdgcn_ballot_w64(L.gcount == 1) != 0;

  static_for<0, N + 1>([&](auto gi) __attribute__((always_inline)) {
    constexpr int g = N - decltype(gi)::value;
    static_for<0, nchunks(g, C::kChunk)>([&](auto ci) __attribute__((always_inline)) {
      constexpr int m0 = chunk_start(g, C::kChunk, decltype(ci)::value);
      constexpr int c = chunk_size(g, C::kChunk, decltype(ci)::value);
      constexpr int kOut = (kE * kNQ * c * T + kThreads - 1) / kThreads;  // output values per lane
      // kCorrect: the previous Q of this lane's output values, loaded at the
      // start of the chunk so that the latency overlaps steps 1 and 2
      double qpre[Mode == kCorrect ? kOut : 1];
      if constexpr (Mode == kCorrect) {
        constexpr int per = c * T;
#pragma unroll
        for (int k = 0; k < kOut; ++k) {
          const int i = tid + k * kThreads;
          qpre[k] = i < nloc * kNQ * per ? a.Q[(e0 * kNQ + i / per) * (B * T) + m0 * T + i % per] : 0.0;
        }
      }
      if constexpr (g > 0) prefetch_columns<N, R, m0, c, kThreads / 64>(kv, wave);
      // 1. right-hand side of the chunk to LDS; the top block has received no
      //    update yet, so it comes straight from memory
      if constexpr (g == N) {
        if constexpr (Mode == kInit) {
          constexpr int per_thread = (kE * kNQ * c + kThreads - 1) / kThreads;
          double q[per_thread];
          // chunk 0 was loaded before the setup, the others during the green
          // update of the chunk before them
          static_assert(per_thread <= kFirstPer && (decltype(ci)::value > 0 || m0 == kFirstM), "top chunks");
#pragma unroll
          for (int k = 0; k < per_thread; ++k) q[k] = q_first[k];
#pragma unroll
          for (int k = 0; k < per_thread; ++k) {
            const int i = tid + k * kThreads;
            const int ee = i / (kNQ * c), pp = (i / c) % kNQ, kk = i % c;
            if (ee < nloc) {
#pragma unroll
              for (int uu = 0; uu < T; ++uu)
                bufB[C::blk(ee, pp) + kk * T + uu] = static_cast<R>(q[k] * sinv_w(uu));
            }
          }
        } else {
          stage_rows<N, R, c * T>(bufB, rin, e0, m0 * T, nloc, tid);
        }
      } else {
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          bufB[cb + decltype(k)::value * T + u] = b[m0 + decltype(k)::value];
        });
      }
      __syncthreads();
      // 2. dark-blue blocks and G coupling (float64)
      if (L.closure) {
        // One straight-line variant per combination of the wave-uniform
        // flags, so that the LDS reads of all modes of the chunk can be in
        // flight together.
        auto dark_blue = [&](auto stiff_c, auto coupled_c) __attribute__((always_inline)) {
          constexpr bool kStiff = decltype(stiff_c)::value, kCoupled = decltype(coupled_c)::value;
          double zr[T], drr[T];
          if constexpr (kStiff) {
#pragma unroll
            for (int v = 0; v < T; ++v) zr[v] = sh.zr[tid][v];
          }
          if constexpr (kCoupled) {
#pragma unroll
            for (int v = 0; v < T; ++v) drr[v] = sh.dr[tid][v];
          }
          static_for<0, c>([&](auto k) __attribute__((always_inline)) {
            constexpr int kk = decltype(k)::value;
            double x;
            if constexpr (kStiff) {
              // dense row u of (Z - E*_pp I)^-1 (Z^-1 for the lanes without
              // a diagonal source in this wave)
              x = 0.0;
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(zr[v], static_cast<double>(bufB[cb + kk * T + v]), x);
            } else {
              x = fma(zv0, static_cast<double>(bufB[cz0 + kk * T]), zv1 * static_cast<double>(bufB[cz1 + kk * T]));
            }
            if constexpr (kCoupled) {
              // closure coupling dr . b_p (dr = 0 in uncoupled lanes)
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(drr[v], static_cast<double>(bufB[pb + kk * T + v]), x);
            }
            bufX[cb + kk * T + u] = static_cast<R>(x);
          });
        };
        using yes = std::true_type;
        using no = std::false_type;
        if (wave_stiff) {
          if (wave_coupled) dark_blue(yes{}, yes{});
          else dark_blue(yes{}, no{});
        } else {
          if (wave_coupled) dark_blue(no{}, yes{});
          else dark_blue(no{}, no{});
        }
      } else {
        double zr[T];
#pragma unroll
        for (int v = 0; v < T; ++v) zr[v] = sh.zr[tid][v];
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          constexpr int kk = decltype(k)::value;
          double x = 0.0;
#pragma unroll
          for (int v = 0; v < T; ++v) x = fma(zr[v], static_cast<double>(bufB[cb + kk * T + v]), x);
          bufX[cb + kk * T + u] = static_cast<R>(x);
        });
        // general upper-triangular E: level by level, each level after the
        // levels it depends on
        for (int r = 1; r <= L.maxlevel; ++r) {
          __syncthreads();
          if (L.mylevel == r) {
            static_for<0, c>([&](auto k) __attribute__((always_inline)) {
              constexpr int kk = decltype(k)::value;
              double acc[T];
#pragma unroll
              for (int v = 0; v < T; ++v) acc[v] = static_cast<double>(bufB[cb + kk * T + v]);
              for (int q = p + 1; q < kNQ; ++q) {
                const double gq = sh.G[es][p][q];
                if (gq != 0.0) {
                  const int qb = C::blk(es, q) + kk * T;
#pragma unroll
                  for (int v = 0; v < T; ++v) acc[v] = fma(gq, static_cast<double>(bufX[qb + v]), acc[v]);
                }
              }
              double x = 0.0;
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(zr[v], acc[v], x);
              bufX[cb + kk * T + u] = static_cast<R>(x);
            });
          }
        }
      }
      __syncthreads();
      // 3. outputs of the chunk from the X buffer: every (element, quantity)
      //    row of the chunk is one contiguous run of c*T doubles of Q, so
      //    consecutive lanes store consecutive doubles.  Each lane stores
      //    kOut values: kInit in nOut groups of kOutGroup (LDS reads issued
      //    before the stores) in a rolled loop, which keeps the registers of
      //    this step few; kCorrect adds the previous Q loaded at the start of
      //    the chunk, in one unrolled pass.  The streaming stores drain while
      //    the green update computes: kInit issues a quarter of its groups
      //    here and the rest after the first quarter of the chunk's green
      //    modes (measured ~1% faster at N=6 than issuing all of them here,
      //    where the burst waits on the compute unit's write queue).
      //    Q <- X (kInit) or Q <- Q + X (kCorrect); then Qint = dt X[:, :, 0]
      //    in its own pass (consecutive lanes, consecutive modes), so no store
      //    instruction runs with one lane in T.  The block stays open over
      //    step 4, which issues the remaining kInit groups.
      {
        constexpr int per = c * T;
        constexpr int kOutGroup = 3;
        constexpr int nOut = (kOut + kOutGroup - 1) / kOutGroup;
        constexpr int kOutEarly = (g > 0) ? (nOut + 3) / 4 : nOut;   // groups issued before step 4
        const int limit = nloc * kNQ * per;
        double* Qg = a.Q + e0 * (kNQ * B * T) + m0 * T;
        // value k of this lane: run index i = tid + k kThreads -> (row, r)
        auto lds_index = [&](int i) __attribute__((always_inline)) { return C::rowblk(i / per) + i % per; };
        // streaming stores: Q is written once and not read again here, so
        // it should not displace the Khat lines in L2
        auto store_groups = [&](int glo, int ghi) __attribute__((always_inline)) {
#pragma unroll 1
          for (int gi = glo; gi < ghi; ++gi) {
            double xv[kOutGroup];
#pragma unroll
            for (int k = 0; k < kOutGroup; ++k)
              xv[k] = static_cast<double>(bufX[lds_index(tid + (gi * kOutGroup + k) * kThreads)]);
#pragma unroll
            for (int k = 0; k < kOutGroup; ++k) {
              const int i = tid + (gi * kOutGroup + k) * kThreads;
              if (i < limit) __builtin_nontemporal_store(xv[k], &Qg[(i / per) * (B * T) + i % per]);
            }
          }
        };
        if constexpr (Mode == kInit) {
          store_groups(0, kOutEarly);
        } else {
          double xv[kOut];
#pragma unroll
          for (int k = 0; k < kOut; ++k) xv[k] = static_cast<double>(bufX[lds_index(tid + k * kThreads)]);
#pragma unroll
          for (int k = 0; k < kOut; ++k) {
            const int i = tid + k * kThreads;
            if (i < limit) __builtin_nontemporal_store(xv[k] + qpre[k], &Qg[(i / per) * (B * T) + i % per]);
          }
        }
        // Qint of the chunk: c contiguous values per (element, quantity) row.
        // kCorrect adds dt X to the previous Qint (read and written by the
        // same lane; Q itself is being rewritten by other lanes above).
        if (a.Qint) {
          double* Ig = a.Qint + e0 * (kNQ * B);
          constexpr int kInt = (kE * kNQ * c + kThreads - 1) / kThreads;
          const int ilimit = nloc * kNQ * c;
#pragma unroll
          for (int k = 0; k < kInt; ++k) {
            const int j = tid + k * kThreads;
            const int row = j / c, kk = j % c;
            double v = a.dt * static_cast<double>(bufX[C::rowblk(row) + kk * T]);
            if constexpr (Mode == kCorrect) v += j < ilimit ? Ig[row * B + m0 + kk] : 0.0;
            if (j < ilimit) __builtin_nontemporal_store(v, &Ig[row * B + m0 + kk]);
          }
        }
      // 4. green blocks (lane-local): star product, then Khat columns.  X of
      //    the chunk stays in bufX until the next chunk's step 2, so the
      //    remaining output groups are read from it here.
      if constexpr (g > 0) {
        if constexpr (kDeferRows && g == N && decltype(ci)::value == 0) {
          // b[p, n, u] = Q0[p, n] (S^-1 w)_u (eq:b_pmu)
#pragma unroll
          for (int n = 0; n < C::LN; ++n) b[n] *= w_u;
        }
        if constexpr (Mode == kInit && g == N && decltype(ci)::value + 1 < nchunks(N, C::kChunk)) {
          // Q0 of the next top-block chunk, in flight during this green update
          constexpr int cn = chunk_size(N, C::kChunk, decltype(ci)::value + 1);
          constexpr int mn = chunk_start(N, C::kChunk, decltype(ci)::value + 1);
          constexpr int per_next = (kE * kNQ * cn + kThreads - 1) / kThreads;
#pragma unroll
          for (int k = 0; k < per_next; ++k) {
            const int i = tid + k * kThreads;
            const int ee = i / (kNQ * cn), pp = (i / cn) % kNQ, kk = i % cn;
            q_first[k] = (ee < nloc) ? a.Q0[((e0 + ee) * kNQ + pp) * B + mn + kk] : 0.0;
          }
        }
        R kgrp[kGroup<R>];
        load_first_group<N, m0, R>(kv, kgrp);
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          constexpr int kk = decltype(k)::value;
          if constexpr (Mode == kInit && kk == c / 4) {
            store_groups(kOutEarly, nOut);
            __builtin_amdgcn_sched_barrier(0);
          }
          R y0, y1, y2;
          // the star reads take the mode offset as an immediate (measured
          // 2.3% faster in float64 and 4% in the float chain; the residual
          // kernel, whose chunk buffer alternates, keeps the per-mode form)
          L.template star_bound<kk>(bufX, a, e0, es, p, u, active, y0, y1, y2);
          green_column<N, m0 + kk, (kk + 1 < c ? m0 + kk + 1 : -1), R>(b, y0, y1, y2, kv, kgrp);
          // keep the scheduler from hoisting the next mode's LDS reads
          __builtin_amdgcn_sched_barrier(0);
        });
      }
      }  // output block of step 3
    });
  });
}

// ---------------------------------------------------------------------------
// Float32 chain with the green-block update on the matrix cores.
//
// The green update of a chunk is a product with a shared left operand:
//   b[n, col] -= sum_k Khat(k)[n] Y[k, col],   k = (mode mm of the chunk, direction j),
// Y[k, col] = (A^{j*} X[:, mm, u])_p for column col = (element, quantity p, time
// mode u), n below the block start.  It runs as v_mfma_f32_16x16x4f32 with
// float32 accumulation: wave w keeps the right-hand side rows below the top
// degree block of its own 64 columns (4 column tiles of 16) in accumulator
// tiles of 16 rows; the A operand is a 16-row slice of -Khat read from a
// generated table, the B operand the wave's Y rows, which its lanes compute
// (sparse star rows, vector ALU) into a per-wave LDS buffer.  The dark-blue
// solves stay float64 on the vector ALU, and the matrix-core instructions of a
// chunk overlap the vector work that follows them.  Accumulator layout of
// the 16x16x4 instruction: lane l holds column l % 16, rows 4 (l / 16) + r,
// r = 0..3; A operand A[l % 16][l / 16]; B operand B[l / 16][l % 16].
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMG = 4;        // modes per k group: 3 k-blocks of 4 (mode, direction) pairs
constexpr int kYStride = 80;  // floats per k row of a wave's Y buffer: 64 columns, padded against bank conflicts

template <int N>
struct MfmaCfg {
  using C = Cfg<N>;
  static constexpr int kWaves = C::kThreads / 64;
  static constexpr int RN = (C::LN + 15) / 16;  // accumulator row tiles (rows below the top block)
  static constexpr int RA = RN > 0 ? RN : 1;
  static constexpr int kRealCols = C::kElems * C::kCols;
};

template <int N>
struct SharedM {
  Shared<N, float> s;
  float ybuf[MfmaCfg<N>::kWaves][3 * kMG][kYStride];
};

template <int N>
__device__ __forceinline__ const float* khat_mfma() {
  if constexpr (N == 0) return stp_gen::kKhatMfma0;
  else if constexpr (N == 1) return stp_gen::kKhatMfma1;
  else if constexpr (N == 2) return stp_gen::kKhatMfma2;
  else if constexpr (N == 3) return stp_gen::kKhatMfma3;
  else if constexpr (N == 4) return stp_gen::kKhatMfma4;
  else if constexpr (N == 5) return stp_gen::kKhatMfma5;
  else if constexpr (N == 6) return stp_gen::kKhatMfma6;
  else return stp_gen::kKhatMfma7;
}

// Algorithm 3 in float32 with the green update on the matrix cores (dark-blue
// solves in float64).  kInit: b = Q0 (S^-1 w), Q <- X.  kCorrect: b = the
// residual in `rin` (float), Q <- Q + X.
template <int N, int Mode>
__global__ __launch_bounds__(Cfg<N>::kThreads) void mfma_solve_kernel(PredictArgs a, const float* rin) {
  using C = Cfg<N>;
  using MC = MfmaCfg<N>;
  using R = float;
  constexpr int B = C::B, T = C::T, kE = C::kElems, kThreads = C::kThreads;
  __shared__ SharedM<N> shm;
  Shared<N, R>& sh = shm.s;
  R* const bufB = sh.u.c.bufB;
  R* const bufX = sh.u.c.bufX;
  const int tid = threadIdx.x;
  const int lane = tid & 63, lrow = lane >> 4, lcol = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kE;
  const int64_t nloc64 = a.n - e0 < kE ? a.n - e0 : kE;
  const int nloc = static_cast<int>(nloc64);
  const LaneId<N> lid(tid);
  const int es = lid.es, p = lid.p, u = lid.u;
  const bool active = es < nloc;
  const int cb = C::blk(es, p);
  float* const yb = &shm.ybuf[wave][0][0];

  // Column tiles of this wave holding real columns (wave-uniform), and the
  // chunk-buffer offset blk(e, p) + u of this lane's column in each tile.
  const int nct = __builtin_amdgcn_readfirstlane(
      (MC::kRealCols - 64 * wave) >= 64 ? 4 : ((MC::kRealCols - 64 * wave) > 0 ? (MC::kRealCols - 64 * wave + 15) / 16 : 0));
  int coff[4];
  v4f acc[4][MC::RA];
  static_for<0, 4>([&](auto ctc) __attribute__((always_inline)) {
    constexpr int ct = decltype(ctc)::value;
    const LaneId<N> cid(64 * wave + 16 * ct + lcol);
    coff[ct] = C::blk(cid.es, cid.p) + cid.u;
    const bool cact = cid.es < nloc;
    const int64_t crow = (cact ? e0 + cid.es : 0) * kNQ + cid.p;
    // accumulators: b rows below the top block
    static_for<0, MC::RA>([&](auto rtc) __attribute__((always_inline)) {
      constexpr int rt = decltype(rtc)::value;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * rt + 4 * lrow + r;
        float v = 0.0f;
        if (cact && row < C::LN) {
          if constexpr (Mode == kInit) v = static_cast<float>(a.Q0[crow * B + row] * sinv_w(cid.u));
          else v = rin[crow * (B * T) + row * T + cid.u];
        }
        acc[ct][rt][r] = v;
      }
    });
  });
  for (int i = lane; i < 3 * kMG * kYStride; i += 64) yb[i] = 0.0f;
  const float* const ktab = khat_mfma<N>();

  constexpr int kFirstC = chunk_size(N, C::kChunk, 0), kFirstM = chunk_start(N, C::kChunk, 0);
  constexpr int kFirstPer = (kE * kNQ * kFirstC + kThreads - 1) / kThreads;
  double q_first[kFirstPer];
  if constexpr (Mode == kInit) {
#pragma unroll
    for (int k = 0; k < kFirstPer; ++k) {
      const int i = tid + k * kThreads;
      const int ee = i / (kNQ * kFirstC), pp = (i / kFirstC) % kNQ, kk = i % kFirstC;
      q_first[k] = (ee < nloc) ? a.Q0[((e0 + ee) * kNQ + pp) * B + kFirstM + kk] : 0.0;
    }
  }
  LaneSetup<N, R> L;
  L.run(sh, a, e0, nloc, tid, es, p, u, active, cb);
  const int pb = C::blk(es, L.gp);
  using ZS = stp_gen::ZinvSparse<N>;
  const int cz0 = cb + ZS::col[2 * u], cz1 = cb + ZS::col[2 * u + 1];
  const double zv0 = ZS::val[2 * u], zv1 = ZS::val[2 * u + 1];
  const bool wave_stiff = __builtin_amdgcn_ballot_w64(sh.G[es][p][p] != 0.0) != 0;
  const bool wave_coupled = __builtin_amdgcn_ballot_w64(L.gcount == 1) != 0;

  static_for<0, N + 1>([&](auto gi) __attribute__((always_inline)) {
    constexpr int g = N - decltype(gi)::value;
    static_for<0, nchunks(g, C::kChunk)>([&](auto ci) __attribute__((always_inline)) {
      constexpr int m0 = chunk_start(g, C::kChunk, decltype(ci)::value);
      constexpr int c = chunk_size(g, C::kChunk, decltype(ci)::value);
      constexpr int kOut = (kE * kNQ * c * T + kThreads - 1) / kThreads;
      // 1. right-hand side of the chunk to LDS
      if constexpr (g == N) {
        if constexpr (Mode == kInit) {
          constexpr int per_thread = (kE * kNQ * c + kThreads - 1) / kThreads;
          double q[per_thread];
          if constexpr (decltype(ci)::value == 0) {
#pragma unroll
            for (int k = 0; k < per_thread; ++k) q[k] = q_first[k];
          } else {
#pragma unroll
            for (int k = 0; k < per_thread; ++k) {
              const int i = tid + k * kThreads;
              const int ee = i / (kNQ * c), pp = (i / c) % kNQ, kk = i % c;
              q[k] = (ee < nloc) ? a.Q0[((e0 + ee) * kNQ + pp) * B + m0 + kk] : 0.0;
            }
          }
#pragma unroll
          for (int k = 0; k < per_thread; ++k) {
            const int i = tid + k * kThreads;
            const int ee = i / (kNQ * c), pp = (i / c) % kNQ, kk = i % c;
            if (ee < nloc) {
#pragma unroll
              for (int uu = 0; uu < T; ++uu) bufB[C::blk(ee, pp) + kk * T + uu] = static_cast<R>(q[k] * sinv_w(uu));
            }
          }
        } else {
          stage_rows<N, R, c * T>(bufB, rin, e0, m0 * T, nloc, tid);
        }
      } else {
        // rows m0 .. m0 + c - 1 leave the accumulators of this wave's columns
        constexpr int rt0 = m0 / 16, rt1 = (m0 + c - 1) / 16;
        static_for<0, 4>([&](auto ctc) __attribute__((always_inline)) {
          constexpr int ct = decltype(ctc)::value;
          if (ct < nct) {
            static_for<rt0, rt1 + 1>([&](auto rtc) __attribute__((always_inline)) {
              constexpr int rt = decltype(rtc)::value;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                const int mm = 16 * rt + 4 * lrow + r - m0;
                if (mm >= 0 && mm < c) bufB[coff[ct] + mm * T] = acc[ct][rt][r];
              }
            });
          }
        });
      }
      __syncthreads();
      // 2. dark-blue blocks and G coupling (float64)
      if (L.closure) {
        auto dark_blue = [&](auto stiff_c, auto coupled_c) __attribute__((always_inline)) {
          constexpr bool kStiff = decltype(stiff_c)::value, kCoupled = decltype(coupled_c)::value;
          double zr[T], drr[T];
          if constexpr (kStiff) {
#pragma unroll
            for (int v = 0; v < T; ++v) zr[v] = sh.zr[tid][v];
          }
          if constexpr (kCoupled) {
#pragma unroll
            for (int v = 0; v < T; ++v) drr[v] = sh.dr[tid][v];
          }
          static_for<0, c>([&](auto k) __attribute__((always_inline)) {
            constexpr int kk = decltype(k)::value;
            double x;
            if constexpr (kStiff) {
              x = 0.0;
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(zr[v], static_cast<double>(bufB[cb + kk * T + v]), x);
            } else {
              x = fma(zv0, static_cast<double>(bufB[cz0 + kk * T]), zv1 * static_cast<double>(bufB[cz1 + kk * T]));
            }
            if constexpr (kCoupled) {
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(drr[v], static_cast<double>(bufB[pb + kk * T + v]), x);
            }
            bufX[cb + kk * T + u] = static_cast<R>(x);
          });
        };
        using yes = std::true_type;
        using no = std::false_type;
        if (wave_stiff) {
          if (wave_coupled) dark_blue(yes{}, yes{});
          else dark_blue(yes{}, no{});
        } else {
          if (wave_coupled) dark_blue(no{}, yes{});
          else dark_blue(no{}, no{});
        }
      } else {
        double zr[T];
#pragma unroll
        for (int v = 0; v < T; ++v) zr[v] = sh.zr[tid][v];
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          constexpr int kk = decltype(k)::value;
          double x = 0.0;
#pragma unroll
          for (int v = 0; v < T; ++v) x = fma(zr[v], static_cast<double>(bufB[cb + kk * T + v]), x);
          bufX[cb + kk * T + u] = static_cast<R>(x);
        });
        for (int r = 1; r <= L.maxlevel; ++r) {
          __syncthreads();
          if (L.mylevel == r) {
            static_for<0, c>([&](auto k) __attribute__((always_inline)) {
              constexpr int kk = decltype(k)::value;
              double accd[T];
#pragma unroll
              for (int v = 0; v < T; ++v) accd[v] = static_cast<double>(bufB[cb + kk * T + v]);
              for (int q = p + 1; q < kNQ; ++q) {
                const double gq = sh.G[es][p][q];
                if (gq != 0.0) {
                  const int qb = C::blk(es, q) + kk * T;
#pragma unroll
                  for (int v = 0; v < T; ++v) accd[v] = fma(gq, static_cast<double>(bufX[qb + v]), accd[v]);
                }
              }
              double x = 0.0;
#pragma unroll
              for (int v = 0; v < T; ++v) x = fma(zr[v], accd[v], x);
              bufX[cb + kk * T + u] = static_cast<R>(x);
            });
          }
        }
      }
      __syncthreads();
      // 3. outputs of the chunk: Q <- X (kInit) or Q <- Q + X (kCorrect) in a
      //    rolled loop of groups of three values per lane, contiguous runs,
      //    streaming stores; then Qint
      {
        constexpr int per = c * T;
        const int limit = nloc * kNQ * per;
        double* Qg = a.Q + e0 * (kNQ * B * T) + m0 * T;
        auto lds_index = [&](int i) __attribute__((always_inline)) { return C::rowblk(i / per) + i % per; };
        {
          constexpr int kOutGroup = 3;
          constexpr int nOut = (kOut + kOutGroup - 1) / kOutGroup;
#pragma unroll 1
          for (int gi = 0; gi < nOut; ++gi) {
            double xv[kOutGroup], qv[kOutGroup];
#pragma unroll
            for (int k = 0; k < kOutGroup; ++k) {
              const int i = tid + (gi * kOutGroup + k) * kThreads;
              qv[k] = (Mode == kCorrect && i < limit) ? Qg[(i / per) * (B * T) + i % per] : 0.0;
              xv[k] = static_cast<double>(bufX[lds_index(i)]);
            }
#pragma unroll
            for (int k = 0; k < kOutGroup; ++k) {
              const int i = tid + (gi * kOutGroup + k) * kThreads;
              if (i < limit) __builtin_nontemporal_store(xv[k] + qv[k], &Qg[(i / per) * (B * T) + i % per]);
            }
          }
        }
        if (a.Qint) {
          double* Ig = a.Qint + e0 * (kNQ * B);
          constexpr int kInt = (kE * kNQ * c + kThreads - 1) / kThreads;
          const int ilimit = nloc * kNQ * c;
#pragma unroll
          for (int k = 0; k < kInt; ++k) {
            const int j = tid + k * kThreads;
            const int row = j / c, kk = j % c;
            double v = a.dt * static_cast<double>(bufX[C::rowblk(row) + kk * T]);
            if constexpr (Mode == kCorrect) v += j < ilimit ? Ig[row * B + m0 + kk] : 0.0;
            if (j < ilimit) __builtin_nontemporal_store(v, &Ig[row * B + m0 + kk]);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // 4. green blocks on the matrix cores, in groups of kMG modes
      if constexpr (g > 0) {
        constexpr int RG = (block_start(g) + 15) / 16;   // row tiles holding rows below block g
        static_for<0, (c + kMG - 1) / kMG>([&](auto grc) __attribute__((always_inline)) {
          constexpr int mg0 = decltype(grc)::value * kMG;
          constexpr int gm = (c - mg0) < kMG ? (c - mg0) : kMG;
          constexpr int nkb = (3 * gm + 3) / 4;
          // A = -Khat rows 16 rt + l % 16 of (mode, direction) k = 4 kb + l / 16,
          // loaded first so that the loads overlap the star products
          constexpr int base = stp_gen::KhatMfma<N>::off[m0 + mg0];
          float av[RG][nkb];
#pragma unroll
          for (int kb = 0; kb < nkb; ++kb) {
            // k past the group's 3 gm pairs pads the last k-block: A = 0 there
            // (the load address is clamped to the group's first pair)
            const int k = 4 * kb + lrow;
            const bool live = k < 3 * gm;
            const int kc = live ? k : 0;
            const int mm = kc / 3, j = kc - 3 * mm;
#pragma unroll
            for (int rt = 0; rt < RG; ++rt) {
              const float v = ktab[base + mm * (RG * 48) + (rt * 3 + j) * 16 + lcol];
              av[rt][kb] = live ? v : 0.0f;
            }
          }
          // star products of the group's modes -> Y rows k = 3 mm + j of this wave
          static_for<0, gm>([&](auto mmc) __attribute__((always_inline)) {
            constexpr int mm = decltype(mmc)::value;
            R y0, y1, y2;
            L.template star<mg0 + mm>(bufX, a, e0, es, p, u, active, y0, y1, y2);
            yb[(3 * mm + 0) * kYStride + lane] = y0;
            yb[(3 * mm + 1) * kYStride + lane] = y1;
            yb[(3 * mm + 2) * kYStride + lane] = y2;
          });
          // B = Y (k = 4 kb + l / 16, column l % 16 of tile ct)
          float bv[4][nkb];
          static_for<0, 4>([&](auto ctc) __attribute__((always_inline)) {
            constexpr int ct = decltype(ctc)::value;
#pragma unroll
            for (int kb = 0; kb < nkb; ++kb) bv[ct][kb] = yb[(4 * kb + lrow) * kYStride + 16 * ct + lcol];
          });
          // k-blocks outermost: consecutive instructions update different
          // accumulator tiles, so none waits on the previous one's result
#pragma unroll
          for (int kb = 0; kb < nkb; ++kb) {
            static_for<0, 4>([&](auto ctc) __attribute__((always_inline)) {
              constexpr int ct = decltype(ctc)::value;
              if (ct < nct) {
                static_for<0, RG>([&](auto rtc) __attribute__((always_inline)) {
                  constexpr int rt = decltype(rtc)::value;
                  acc[ct][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[rt][kb], bv[ct][kb], acc[ct][rt], 0, 0, 0);
                });
              }
            });
          }
        });
      }
    });
  });
}

// Float64 residual of the full element system for the current Q (the
// matrix-free form of eq:stp-lineq after the multiplication with M^-1 S^-1,
// section "Block-wise back-substitution"):
//   r[p,n,u] = (S^-1 w)_u Q0[p,n] - sum_s Z_us Q[p,n,s] + sum_q E*_pq Q[q,n,u]
//              - sum_j sum_q A^{j*}_pq sum_l Khat^j[n,l] Q[q,l,u],
// written to `rout` in float (the right-hand side of the correction solve).
// Same lane mapping and chunk order as the solve; the Khat term is the green
// update of the solve applied to the known Q, accumulated in float64.  The
// residual of a chunk is collected in LDS and written in contiguous runs.
template <int N>
__global__ __launch_bounds__(Cfg<N>::kThreads) void fused_residual_kernel(PredictArgs a, float* rout) {
  using C = Cfg<N>;
  using R = double;
  constexpr int B = C::B, T = C::T, kE = C::kElems, kThreads = C::kThreads;
  __shared__ Shared<N, R> sh;
  R* const bufR = sh.u.c.bufB;  // residual of the chunk, same layout, to memory after the chunk
  // Q of the chunks (and Q0 of the top-block chunks, [element][quantity][mode])
  // alternate between two buffers: the X chunk buffer and the per-lane rows
  // of the setup, which are not used after it.  Each chunk's loads are issued
  // during the previous chunk and stored to its buffer before that chunk's
  // green update, so only the first chunk waits for memory.  Where the second
  // buffer does not fit, every chunk stages its own rows.
  constexpr int kXSize = C::kBufSize, kQ0Size = C::kSlots * kNQ * C::kChunk;
  constexpr bool kTwoBuffers = kXSize + 2 * kQ0Size <= 2 * C::kThreads * T;
  static_assert(kQ0Size <= C::kThreads * T, "Q0 staging fits");
  double* const rows = &sh.zr[0][0];  // zr and dr: 2 kThreads T contiguous doubles
  auto xbuf = [&](int ci_index) -> R* { return (kTwoBuffers && (ci_index & 1)) ? rows : sh.u.c.bufX; };
  auto q0buf = [&](int ci_index) -> double* {
    return kTwoBuffers ? rows + kXSize + (ci_index & 1) * kQ0Size : rows;
  };
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kE;
  const int64_t nloc64 = a.n - e0 < kE ? a.n - e0 : kE;
  const int nloc = static_cast<int>(nloc64);
  const LaneId<N> lid(tid);
  const int es = lid.es, p = lid.p, u = lid.u;
  const bool active = es < nloc;
  const int cb = C::blk(es, p);
  const R* kv = khat_sparse<N, R>();
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int64_t erow = ((active ? e0 + es : 0) * kNQ + p);
  const double w = sinv_w(u);

  // rows below the top block, loaded after the setup so that its loads do
  // not wait behind them
  R r[C::LR];
  LaneSetup<N, R> L;
  L.run(sh, a, e0, nloc, tid, es, p, u, active, cb);
  {
    const double* q0row = a.Q0 + erow * B;
#pragma unroll
    for (int n = 0; n < C::LN; ++n) r[n] = q0row[n] * w;
  }
  const double zpp = sh.G[es][p][p];
  const bool general_g = __builtin_amdgcn_readfirstlane(__syncthreads_or(active && L.gcount > 1)) != 0;
  const int pb = C::blk(es, L.gp);
  double zrow[T];  // row u of Z
#pragma unroll
  for (int v = 0; v < T; ++v) zrow[v] = z_entry(u, v);

  static_for<0, N + 1>([&](auto gi) __attribute__((always_inline)) {
    constexpr int g = N - decltype(gi)::value;
    static_for<0, nchunks(g, C::kChunk)>([&](auto ci) __attribute__((always_inline)) {
      constexpr int m0 = chunk_start(g, C::kChunk, decltype(ci)::value);
      constexpr int c = chunk_size(g, C::kChunk, decltype(ci)::value);
      constexpr int CI = chunk_index(N, g, decltype(ci)::value, C::kChunk);
      R* const bufX = xbuf(CI);
      double* const q0s = q0buf(CI);
      if constexpr (g > 0) prefetch_columns<N, R, m0, c, kThreads / 64>(kv, wave);
      // stage Q of the chunk (and Q0 of the top block) in LDS, coalesced,
      // unless the previous chunk did
      if constexpr (!kTwoBuffers || CI == 0) {
        stage_rows<N, R, c * T>(bufX, static_cast<const double*>(a.Q), e0, m0 * T, nloc, tid);
        if constexpr (g == N) {
          Q0Stage<N, c> qs;
          qs.issue(a.Q0, e0, m0, nloc, tid);
          qs.commit(q0s, nloc, tid);
        }
      }
      __syncthreads();
      // loads of the next chunk, in flight during the local terms
      constexpr bool kHasNext = !(g == 0 && decltype(ci)::value + 1 == nchunks(g, C::kChunk));
      constexpr int gn = kHasNext ? next_block(g, decltype(ci)::value, C::kChunk) : 0;
      constexpr int cin = kHasNext ? next_chunk(g, decltype(ci)::value, C::kChunk) : 0;
      constexpr int mn = chunk_start(gn, C::kChunk, cin), cn = chunk_size(gn, C::kChunk, cin);
      constexpr bool kPrefetch = kTwoBuffers && kHasNext;
      RowStage<N, cn * T> nrows;
      Q0Stage<N, cn> nq0;
      if constexpr (kPrefetch) {
        nrows.issue(static_cast<const double*>(a.Q), e0, mn * T, nloc, tid);
        if constexpr (gn == N) nq0.issue(a.Q0, e0, mn, nloc, tid);
      }
      // local terms of the chunk's rows: their residual is now complete
      static_for<0, c>([&](auto k) __attribute__((always_inline)) {
        constexpr int kk = decltype(k)::value;
        constexpr int m = m0 + kk;
        double base;
        if constexpr (g == N) base = q0s[(es * kNQ + p) * c + kk] * w;
        else base = r[m];
        double zx = 0.0;
#pragma unroll
        for (int v = 0; v < T; ++v) zx = fma(zrow[v], bufX[cb + kk * T + v], zx);
        double ex = zpp * bufX[cb + kk * T + u];
        if (!general_g) {
          ex = fma(L.gcoef, bufX[pb + kk * T + u], ex);
        } else {
          for (int q = p + 1; q < kNQ; ++q) {
            const double gq = sh.G[es][p][q];
            if (gq != 0.0) ex = fma(gq, bufX[C::blk(es, q) + kk * T + u], ex);
          }
        }
        bufR[cb + kk * T + u] = base - zx + ex;
      });
      // the next chunk's rows to the other buffer (no wave reads it during
      // this chunk)
      if constexpr (kPrefetch) {
        nrows.commit(xbuf(CI + 1), nloc, tid);
        if constexpr (gn == N) nq0.commit(q0buf(CI + 1), nloc, tid);
      }
      // Khat term into the rows of lower blocks
      if constexpr (g > 0) {
        R kgrp[kGroup<R>];
        load_first_group<N, m0, R>(kv, kgrp);
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          constexpr int kk = decltype(k)::value;
          R y0, y1, y2;
          L.template star<kk>(bufX, a, e0, es, p, u, active, y0, y1, y2);
          green_column<N, m0 + kk, (kk + 1 < c ? m0 + kk + 1 : -1), R>(r, y0, y1, y2, kv, kgrp);
          __builtin_amdgcn_sched_barrier(0);
        });
      }
      __syncthreads();  // before the next chunk overwrites the buffers
      // the residual of the chunk to memory: every (element, quantity) row is
      // one contiguous run of c*T floats (consecutive lanes, consecutive
      // values), streaming stores; the next chunk writes the residual buffer
      // only after its own barrier
      {
        constexpr int per = c * T;
        constexpr int kGroupOut = 3;
        constexpr int iters = (kE * kNQ * per + kThreads - 1) / kThreads;
        constexpr int ngroups = (iters + kGroupOut - 1) / kGroupOut;
        const int limit = nloc * kNQ * per;
        float* const Rg = rout + e0 * (kNQ * B * T) + m0 * T;
#pragma unroll 1
        for (int gi = 0; gi < ngroups; ++gi) {
          float v[kGroupOut];
#pragma unroll
          for (int k = 0; k < kGroupOut; ++k) {
            const int i = tid + (gi * kGroupOut + k) * kThreads;
            v[k] = static_cast<float>(bufR[C::rowblk(i / per) + i % per]);
          }
#pragma unroll
          for (int k = 0; k < kGroupOut; ++k) {
            const int i = tid + (gi * kGroupOut + k) * kThreads;
            if (i < limit) __builtin_nontemporal_store(v[k], &Rg[(i / per) * (B * T) + i % per]);
          }
        }
      }
    });
  });
}

}  // namespace

template <>
hipError_t launch_fused<STP_NQ, STP_DEGREE>(const PredictArgs& a, int precision, int refine_steps,
                                            float* workspace, bool valu_float_chain, hipStream_t stream) {
  constexpr int N = STP_DEGREE;
  using C = Cfg<N>;
  const int64_t groups = (a.n + C::kElems - 1) / C::kElems;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 grid(static_cast<unsigned>(groups)), block(C::kThreads);
  if (precision == 0) {
    hipLaunchKernelGGL((fused_solve_kernel<N, double, kInit>), grid, block, 0, stream, a, nullptr);
    return hipGetLastError();
  }
  if (valu_float_chain)
    hipLaunchKernelGGL((fused_solve_kernel<N, float, kInit>), grid, block, 0, stream, a, nullptr);
  else
    hipLaunchKernelGGL((mfma_solve_kernel<N, kInit>), grid, block, 0, stream, a, nullptr);
  hipError_t err = hipGetLastError();
  for (int k = 0; k < refine_steps && err == hipSuccess; ++k) {
    hipLaunchKernelGGL((fused_residual_kernel<N>), grid, block, 0, stream, a, workspace);
    err = hipGetLastError();
    if (err != hipSuccess) break;
    if (valu_float_chain)
      hipLaunchKernelGGL((fused_solve_kernel<N, float, kCorrect>), grid, block, 0, stream, a,
                         static_cast<const float*>(workspace));
    else
      hipLaunchKernelGGL((mfma_solve_kernel<N, kCorrect>), grid, block, 0, stream, a,
                         static_cast<const float*>(workspace));
    err = hipGetLastError();
  }
  return err;
}

}  // namespace stp
