// Fused, register-resident kernel for Algorithm 3 of Wolf et al. (arXiv
// 2108.10565, section "Block-wise back-substitution"), one object per degree
// N = STP_DEGREE.
//
// Mapping.  One lane per column (element e, quantity p, time mode u) of the
// element's right-hand side b_pmu (eq:b_pmu); 13 (N+1) lanes per element,
// kElems elements per 512-lane workgroup.  Every lane keeps b[m] for all
// modes m below the top degree block in registers.  The green-block update
//     b[p, n, u] -= sum_j Khat^j[n, m] (A^{j*} X[:, m, u])_p ,  n < block_start(g)
// is lane-local once the star product y_j = (A^{j*} X[:, m, u])_p is known,
// so the lane applies it as a fully unrolled list of fused multiply-adds
// over the non-zeros of Khat (compile-time pattern, coefficients read with
// scalar loads from a device table), exactly the zeros the Lemma of section
// "Structure of the system matrix" and the Dubiner structure provide.
//
// Per chunk of kChunk modes m of degree block g (g = N .. 0):
//   1. every lane writes b[m] to LDS (top block: b = Q0 (S^-1 w), eq:b_pmu);
//   2. dark-blue blocks: lane (e, p, s) forms X[p, m, s] = row s of
//      (Z - E*_pp I)^-1 times b[p, m, :] (float64, Zinv row in registers);
//   3. G coupling in dependency levels: a quantity o whose row of the strict
//      upper part G of E* is non-empty recomputes
//      X[o] = (Z - E*_oo I)^-1 (b[o] + sum_p G_op X[p]) once every X[p] it
//      depends on is final (level = longest chain below it); for the
//      poroelastic E this is one extra round for u, v, w;
//   4. green blocks: every lane reads X[q, m, u] of the 13 quantities, forms
//      y_1..y_3 with its row of A^{1*}, A^{2*}, A^{3*}, and subtracts
//      Khat^j[n, m] y_j from its registers b[n]; the chunk of X is written to
//      Q (and dt X[:, :, 0] to Qint) with coalesced stores.
// A^{j*} = dt A^j and E* = dt E are formed in-kernel, so every product runs
// with unit scaling (the paper's libxsmm alpha = 1 remark, section "Roofline
// model").
#include <utility>

#include "common.hpp"
#include "generated/khat_tables.h"

#ifndef STP_DEGREE
#error "compile once per degree with -DSTP_DEGREE=N"
#endif

namespace stp {
namespace {

constexpr int kMaxThreads = 512;
constexpr int kMaxElems = 16;
constexpr int kChunk = 4;
// Non-zero columns kept per lane of a star-matrix row (union over the three
// directions).  The poroelastic Jacobians need at most 6 (normal-stress and
// pressure rows couple to the 6 velocities; velocity rows to 3 stresses and
// the pressure); a workgroup holding any row with more falls back to reading
// the dense rows from LDS.
constexpr int kStarNnz = 6;

template <int I>
using ic = std::integral_constant<int, I>;
using ConstDouble = __attribute__((address_space(4))) const double;

template <int Begin, class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(ic<Begin + I>{}), ...);
}
// Calls f(ic<i>) for i = Begin .. End-1 with compile-time i.
template <int Begin, int End, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (End > Begin) static_for_impl<Begin>(f, std::make_integer_sequence<int, End - Begin>{});
}

template <int N>
struct Cfg {
  static constexpr int B = n_modes(N);
  static constexpr int T = N + 1;
  static constexpr int TP = (T + 1) & ~1;          // time dimension padded for 16-byte LDS rows
  static constexpr int LN = block_start(N);        // register-resident rows
  static constexpr int LR = LN > 0 ? LN : 1;
  static constexpr int kCols = kNQ * T;            // lanes per element
  static constexpr int kElems =                    // elements per workgroup
      (kMaxThreads / kCols) < kMaxElems ? (kMaxThreads / kCols) : kMaxElems;
  static constexpr int kThreads = (kElems * kCols + 63) / 64 * 64;
};

// The usage-ordered Khat table of degree N.  Kernels pass its address through
// an empty asm statement before reading it, so the compiler cannot fold the
// values into instruction literals and reads them with scalar loads instead.
template <int N>
__device__ __forceinline__ const double* khat_sparse() {
  if constexpr (N == 0) return stp_gen::kKhatSparse0;
  else if constexpr (N == 1) return stp_gen::kKhatSparse1;
  else if constexpr (N == 2) return stp_gen::kKhatSparse2;
  else if constexpr (N == 3) return stp_gen::kKhatSparse3;
  else if constexpr (N == 4) return stp_gen::kKhatSparse4;
  else if constexpr (N == 5) return stp_gen::kKhatSparse5;
  else if constexpr (N == 6) return stp_gen::kKhatSparse6;
  else return stp_gen::kKhatSparse7;
}

template <int N, typename R>
struct Shared {
  using C = Cfg<N>;
  double q0[C::kElems][kNQ][C::B];          // initial spatial DOFs of the group
  double A[C::kElems][3][kNQ][kNQ];         // A^{j*} = dt A^j of the group
  double G[C::kElems][kNQ][kNQ];            // E* (lower part zeroed)
  R bufB[C::kElems][kNQ][kChunk][C::TP];    // b of the chunk
  R bufX[C::kElems][kNQ][kChunk][C::TP];    // X of the chunk
  int level[C::kElems][kNQ];
  int maxlevel;
};

// Row s of (Z - z I)^-1: solves (Z - z I)^T y = e_s by Gauss-Jordan
// elimination without pivoting (eigenvalues of Z have real part >= 1, so for
// z <= 0.5 the pivots stay away from zero; accurate to ~1e-15 there).
template <int T>
__device__ __forceinline__ void zinv_row(double z, int s, double (&out)[T]) {
  double a[T][T + 1];
#pragma unroll
  for (int r = 0; r < T; ++r) {
#pragma unroll
    for (int c = 0; c < T; ++c) a[r][c] = z_entry(c, r) - (r == c ? z : 0.0);  // transpose
    a[r][T] = (r == s) ? 1.0 : 0.0;
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

// Register pinning: an empty asm statement that reads (or reads and writes)
// a register value.  Volatile asm statements keep their program order, so
// these fix where a value must be complete and stop the compiler from
// sinking pure arithmetic or hoisting loads across them.
template <typename T>
__device__ __forceinline__ void pin_v(T& x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void use_s(double x) { asm volatile("" ::"s"(x)); }

constexpr int kGroup = 8;  // coefficients per scalar load (s_load_dwordx16)

// Loads the coefficients [g0, g0 + gn) of the usage-ordered Khat table into
// scalar registers, from an address the compiler cannot see through.
template <int g0, int gn>
__device__ __forceinline__ void load_group(const double* kv, double (&v)[kGroup]) {
  const double* kp = kv + g0;
  asm volatile("" : "+s"(kp));
  const ConstDouble* kc = (const ConstDouble*)kp;
#pragma unroll
  for (int i = 0; i < gn; ++i) v[i] = kc[i];
}

// b[n] -= Khat^j[n, M] y_j for the non-zeros of column M (usage order of the
// generated pattern: directions, then rows ascending), in groups of kGroup
// coefficients; the next group's scalar load is issued before the current
// group's fused multiply-adds and waited for after them.
template <int N, int M, typename R>
__device__ __forceinline__ void green_column(R (&b)[Cfg<N>::LR], R y0, R y1, R y2, const double* kv) {
  using P = stp_gen::KhatPattern<N>;
  constexpr int start = P::col_start[M];
  constexpr int count = P::col_count[M];
  constexpr int ngroups = (count + kGroup - 1) / kGroup;
  if constexpr (count > 0) {
    double cur[kGroup], nxt[kGroup];
    load_group<start, (count < kGroup ? count : kGroup)>(kv, cur);
#pragma unroll
    for (int i = 0; i < (count < kGroup ? count : kGroup); ++i) use_s(cur[i]);
    static_for<0, ngroups>([&](auto G) __attribute__((always_inline)) {
      constexpr int gi = decltype(G)::value;
      constexpr int g0 = start + gi * kGroup;
      constexpr int gn = (start + count - g0) < kGroup ? (start + count - g0) : kGroup;
      constexpr int g1 = g0 + kGroup;
      constexpr int gn1 = (start + count - g1) < kGroup ? (start + count - g1) : kGroup;
      if constexpr (gi + 1 < ngroups) load_group<g1, gn1>(kv, nxt);
      static_for<0, gn>([&](auto I) __attribute__((always_inline)) {
        constexpr int e = g0 + decltype(I)::value;
        constexpr int n = P::row[e];
        constexpr int j = P::dir[e];
        const R k = static_cast<R>(cur[decltype(I)::value]);
        const R y = (j == 0) ? y0 : ((j == 1) ? y1 : y2);
        b[n] = fma(-k, y, b[n]);
      });
      static_for<0, gn>([&](auto I) __attribute__((always_inline)) {
        pin_v(b[P::row[g0 + decltype(I)::value]]);
      });
      if constexpr (gi + 1 < ngroups) {
#pragma unroll
        for (int i = 0; i < gn1; ++i) {
          use_s(nxt[i]);
          cur[i] = nxt[i];
        }
      }
    });
  }
}

template <int N>
__global__ __launch_bounds__(Cfg<N>::kThreads) void fused_fp64_kernel(PredictArgs a) {
  using C = Cfg<N>;
  using R = double;
  constexpr int B = C::B, T = C::T, kE = C::kElems, kThreads = C::kThreads;
  __shared__ Shared<N, R> sh;
  const int tid = threadIdx.x;
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kE;
  const int64_t nloc64 = a.n - e0 < kE ? a.n - e0 : kE;
  const int nloc = static_cast<int>(nloc64);
  int es = tid / C::kCols;
  const int col = tid % C::kCols;
  const int p = col / T, u = col % T;
  const bool active = es < nloc;
  // spare lanes past kElems * kCols alias the last slot for their reads only;
  // they never write LDS or memory
  const bool spare = es >= kE;
  if (spare) es = kE - 1;
  const double* kv = khat_sparse<N>();

  // ---- stage Q0 and E* of the group (coalesced)
  {
    const double* src = a.Q0 + e0 * (kNQ * B);
    double* dst = &sh.q0[0][0][0];
    for (int i = tid; i < nloc * kNQ * B; i += kThreads) dst[i] = src[i];
    const double* Esrc = a.E + e0 * (kNQ * kNQ);
    double* Gd = &sh.G[0][0][0];
    for (int i = tid; i < kE * kNQ * kNQ; i += kThreads) {
      const int r = (i / kNQ) % kNQ, c = i % kNQ;
      Gd[i] = (i < nloc * kNQ * kNQ && c >= r) ? a.dt * Esrc[i] : 0.0;
    }
    if (tid == 0) sh.maxlevel = 0;
  }
  {
    const double* Asrc = a.star + e0 * (3 * kNQ * kNQ);
    double* Ad = &sh.A[0][0][0][0];
    for (int i = tid; i < nloc * 3 * kNQ * kNQ; i += kThreads) Ad[i] = a.dt * Asrc[i];
    for (int i = nloc * 3 * kNQ * kNQ + tid; i < kE * 3 * kNQ * kNQ; i += kThreads) Ad[i] = 0.0;
  }
  __syncthreads();
  // dependency levels of the strict upper part of E*, one thread per element
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
  double zr[T];
  zinv_row<T>(sh.G[es][p][p], u, zr);
  // sparse row p of the three star matrices: columns sq[k] (as LDS offsets
  // into the chunk buffer) and coefficients sa0..sa2[k]
  double sa0[kStarNnz], sa1[kStarNnz], sa2[kStarNnz];
  int sq[kStarNnz];
  bool overflow = false;
  {
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < kStarNnz; ++k) {
      sa0[k] = sa1[k] = sa2[k] = 0.0;
      sq[k] = 0;
    }
#pragma unroll
    for (int q = 0; q < kNQ; ++q) {
      const double v0 = sh.A[es][0][p][q], v1 = sh.A[es][1][p][q], v2 = sh.A[es][2][p][q];
      if (v0 != 0.0 || v1 != 0.0 || v2 != 0.0) {
#pragma unroll
        for (int k = 0; k < kStarNnz; ++k)
          if (k == cnt) {
            sa0[k] = v0;
            sa1[k] = v1;
            sa2[k] = v2;
            sq[k] = q * kChunk * C::TP;
          }
        ++cnt;
      }
    }
    overflow = active && cnt > kStarNnz;
  }
  R b[C::LR];
  {
    const double w = sinv_w(u);
#pragma unroll
    for (int n = 0; n < C::LN; ++n) b[n] = sh.q0[es][p][n] * w;
  }
  const bool dense_star = __syncthreads_or(overflow);
  const int mylevel = active ? sh.level[es][p] : 0;
  const int maxlevel = sh.maxlevel;

  static_for<0, N + 1>([&](auto gi) __attribute__((always_inline)) {
    constexpr int g = N - decltype(gi)::value;
    constexpr int L0 = block_start(g), D = block_size(g);
    constexpr int nchunks = (D + kChunk - 1) / kChunk;
    static_for<0, nchunks>([&](auto ci) __attribute__((always_inline)) {
      constexpr int m0 = L0 + decltype(ci)::value * kChunk;
      constexpr int c = (D - decltype(ci)::value * kChunk) < kChunk ? (D - decltype(ci)::value * kChunk) : kChunk;
      // 1. right-hand side of the chunk to LDS
      static_for<0, c>([&](auto k) __attribute__((always_inline)) {
        constexpr int m = m0 + decltype(k)::value;
        R v;
        if constexpr (g == N) v = sh.q0[es][p][m] * sinv_w(u);
        else v = b[m];
        if (!spare) sh.bufB[es][p][decltype(k)::value][u] = v;
      });
      __syncthreads();
      // 2. dark-blue solves: X[p, m, u] = sum_v Zinv_p[u][v] b[p, m, v]
      static_for<0, c>([&](auto k) __attribute__((always_inline)) {
        double x = 0.0;
#pragma unroll
        for (int v = 0; v < T; ++v) x = fma(zr[v], static_cast<double>(sh.bufB[es][p][decltype(k)::value][v]), x);
        if (!spare) sh.bufX[es][p][decltype(k)::value][u] = static_cast<R>(x);
      });
      __syncthreads();
      // 3. G coupling, level by level
      for (int r = 1; r <= maxlevel; ++r) {
        if (mylevel == r && !spare) {
          static_for<0, c>([&](auto k) __attribute__((always_inline)) {
            constexpr int kk = decltype(k)::value;
            double acc[T];
#pragma unroll
            for (int v = 0; v < T; ++v) acc[v] = static_cast<double>(sh.bufB[es][p][kk][v]);
            for (int q = p + 1; q < kNQ; ++q) {
              const double gq = sh.G[es][p][q];
              if (gq != 0.0) {
#pragma unroll
                for (int v = 0; v < T; ++v) acc[v] = fma(gq, static_cast<double>(sh.bufX[es][q][kk][v]), acc[v]);
              }
            }
            double x = 0.0;
#pragma unroll
            for (int v = 0; v < T; ++v) x = fma(zr[v], acc[v], x);
            sh.bufX[es][p][kk][u] = static_cast<R>(x);
          });
        }
        __syncthreads();
      }
      // 4. green blocks (lane-local) and output of the chunk
      if constexpr (g > 0) {
        static_for<0, c>([&](auto k) __attribute__((always_inline)) {
          constexpr int kk = decltype(k)::value;
          R y0 = 0, y1 = 0, y2 = 0;
          // opaque per-mode offset: this mode's LDS reads stay here
          int xoff = ((es * kNQ) * kChunk + kk) * C::TP + u;
          asm volatile("" : "+v"(xoff));
          const R* xs = &sh.bufX[0][0][0][0] + xoff;
          if (!dense_star) {
#pragma unroll
            for (int k = 0; k < kStarNnz; ++k) {
              const R xq = xs[sq[k]];
              y0 = fma(static_cast<R>(sa0[k]), xq, y0);
              y1 = fma(static_cast<R>(sa1[k]), xq, y1);
              y2 = fma(static_cast<R>(sa2[k]), xq, y2);
            }
          } else {
#pragma unroll
            for (int q = 0; q < kNQ; ++q) {
              const R xq = xs[q * kChunk * C::TP];
              y0 = fma(static_cast<R>(sh.A[es][0][p][q]), xq, y0);
              y1 = fma(static_cast<R>(sh.A[es][1][p][q]), xq, y1);
              y2 = fma(static_cast<R>(sh.A[es][2][p][q]), xq, y2);
            }
          }
          green_column<N, m0 + kk, R>(b, y0, y1, y2, kv);
          // keep the scheduler from hoisting the next mode's LDS reads
          __builtin_amdgcn_sched_barrier(0);
        });
      }
      {
        double* Qg = a.Q + e0 * (kNQ * B * T);
        constexpr int per = c * T;
        for (int i = tid; i < nloc * kNQ * per; i += kThreads) {
          const int ee = i / (kNQ * per), rem = i % (kNQ * per);
          const int pp = rem / per, r = rem % per;
          Qg[(ee * kNQ + pp) * (B * T) + m0 * T + r] = sh.bufX[ee][pp][r / T][r % T];
        }
        if (a.Qint) {
          double* Ig = a.Qint + e0 * (kNQ * B);
          for (int i = tid; i < nloc * kNQ * c; i += kThreads) {
            const int ee = i / (kNQ * c), rem = i % (kNQ * c);
            const int pp = rem / c, kk = rem % c;
            Ig[(ee * kNQ + pp) * B + m0 + kk] = a.dt * sh.bufX[ee][pp][kk][0];
          }
        }
      }
    });
  });
}

}  // namespace

template <>
hipError_t launch_fused_degree<STP_DEGREE>(const PredictArgs& a, int precision, int refine_steps,
                                           hipStream_t stream) {
  constexpr int N = STP_DEGREE;
  (void)refine_steps;
  if (precision != 0) return hipErrorNotSupported;
  const int64_t groups = (a.n + Cfg<N>::kElems - 1) / Cfg<N>::kElems;
  if (groups > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fused_fp64_kernel<N>, dim3(static_cast<unsigned>(groups)), dim3(Cfg<N>::kThreads), 0,
                     stream, a);
  return hipGetLastError();
}

}  // namespace stp
