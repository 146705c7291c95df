// Corrector of one ADER-DG time step (section "ADER-DG discretisation": the
// semi-discrete system eq:semi_discrete integrated over the step, with the
// predictor's time-integrated DOFs Qint = int Q dt in place of the solution):
//
//   Q <- Q + sum_j A^j Qint V^j + E Qint
//          - sum_f ( Gp_f Qint Fl_f + Gm_f Qint_nb(f) Fn_{f, j(f), h(f)} )
//
// V^j, Fl, Fn: reference volume / own-face / neighbour-face tables divided by
// the mass of the test function; Gp_f, Gm_f: the Godunov split of the face's
// normal Jacobian, scaled by 2 |S_f| / |J| (host-built per face).  The volume
// term is the integrated-by-parts flux form of A q_x + B q_y + C q_z, the face
// term Godunov's upwind flux An^+ q^- + An^- q^+ across each face.
//
// One workgroup (4 waves) per element, one kernel per (quantity count,
// degree).  The own and the four neighbours' Qint and the 12 operators (E
// and the 11 terms' G, with the terms' signs folded in) are staged in LDS;
// then, in groups of WN terms, W_m = G_m X_m (nq x B) is formed in LDS on
// the vector ALU and the products W_m T_m are accumulated on the matrix cores
// (v_mfma_f64_16x16x4f64): rows = quantities (padded to 16), columns = the
// element's modes in tiles of 16 (tile t on wave t mod 4), the inner
// dimension the table's rows in steps of 4.  The accumulators stay in
// registers over all 11 terms; E Qint is added on the vector ALU before the
// single read-modify-write of Q.  The tables are read from global memory
// (they are shared by all elements and stay in the caches).
#include "common.hpp"

namespace stp {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kCorrThreads = 256;
constexpr int kCorrWaves = kCorrThreads / 64;
constexpr int kTerms = 11;

template <int NQ, int N>
struct CorrCfg {
  static constexpr int B = n_modes(N);
  static constexpr int QB = NQ * B;
  static constexpr int Q2 = NQ * NQ;
  static constexpr int NT = (B + 15) / 16;                 // column tiles
  static constexpr int TPW = (NT + kCorrWaves - 1) / kCorrWaves;  // tiles per wave
  static constexpr int KS = (B + 3) / 4;                   // inner steps of 4
  static constexpr int WS = 4 * KS + 1;                    // W row stride (odd: no bank conflicts)
  static constexpr int kW = 16 * WS;                       // one term's W, 16 rows (zero past NQ)
  static constexpr size_t lds_doubles(int wn) {
    return static_cast<size_t>(5) * QB + static_cast<size_t>(12) * Q2 + static_cast<size_t>(wn) * kW;
  }
  // terms per group: the most that still let three workgroups share a
  // compute unit's 160 KB of LDS, else two, else one (at N=4 with 13
  // quantities, 3 workgroups of 4-term groups: 5.6 ms per 163,840 elements,
  // against 7.0 ms for 2 workgroups of 6-term groups and 8.3-11.3 ms for 4
  // workgroups of single terms)
  static constexpr int pick_wn() {
    constexpr int cand[6] = {11, 6, 4, 3, 2, 1};
    constexpr size_t limit[3] = {160 * 1024 / 3, 80 * 1024, 160 * 1024};
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < 6; ++i)
        if (lds_doubles(cand[i]) * 8 <= limit[b]) return cand[i];
    return 0;
  }
  static constexpr int WN = pick_wn();
  static_assert(WN >= 1, "the corrector tile does not fit LDS");
  static constexpr size_t kLds = lds_doubles(WN) * 8;
  // the next term's table entries are loaded while the current term's
  // matrix-core products run, when the two register sets are small
  static constexpr bool kPrefetch = TPW * KS <= 24;
  static constexpr int kBuf = kPrefetch ? 2 : 1;
  // staging loads per thread: each source's Qint rows, and the 12 operators
  // (all issued before the first LDS store; issuing the next element's
  // during the current one measured slower, as its registers cost a
  // workgroup per compute unit)
  static constexpr int kXPer = (QB + kCorrThreads - 1) / kCorrThreads;
  static constexpr int kGPer = (12 * Q2 + kCorrThreads - 1) / kCorrThreads;
};

// Position (row i, column j) of accumulator entry r of lane l in the 16x16
// tile of v_mfma_f64_16x16x4f64, whose operands are lane l's A[l % 16][l / 16]
// and B[l / 16][l % 16]: row l / 16 + 4 r, column l % 16 (unlike the float32
// 16x16x4 instruction, whose rows are 4 (l / 16) + r; checked on gfx950 with
// an in-bounds probe of one wave).
__device__ __forceinline__ void acc_pos(int l, int r, int& i, int& j) {
  i = l / 16 + 4 * r;
  j = l % 16;
}

template <int NQ, int N>
__global__ __launch_bounds__(kCorrThreads) void corrector_kernel(CorrectArgs a) {
  using C = CorrCfg<NQ, N>;
  constexpr int B = C::B, QB = C::QB, Q2 = C::Q2, WN = C::WN;
  extern __shared__ double lds[];
  double* X = lds;                 // [5][NQ][B]: own, neighbours 0..3
  double* G = X + 5 * QB;          // [12][NQ][NQ]: E, then the 11 terms' operators (signed)
  double* W = G + 12 * Q2;         // [WN][16][WS]
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  constexpr size_t BB = static_cast<size_t>(B) * B;
  const double* Vt = a.tables;                 // [3][B][B]
  const double* Fl = a.tables + 3 * BB;        // [4][B][B]
  const double* Fn = a.tables + 7 * BB;        // [4][4][6][B][B]
  // the padding of W (rows >= NQ, columns >= B) stays zero
  for (int i = tid; i < WN * C::kW; i += kCorrThreads) W[i] = 0.0;
  // staging of element e: every load issued before any LDS store
  double xs[5][C::kXPer], gs[C::kGPer];
  auto fetch = [&](int64_t e) __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 5; ++s) {
      const int64_t src = s == 0 ? e : a.neighbor[e * 4 + (s - 1)];
#pragma unroll
      for (int k = 0; k < C::kXPer; ++k) {
        const int i = tid + k * kCorrThreads;
        xs[s][k] = i < QB ? a.Qint[src * QB + i] : 0.0;
      }
    }
#pragma unroll
    for (int k = 0; k < C::kGPer; ++k) {
      const int i = tid + k * kCorrThreads;
      const int m = i / Q2, j = i % Q2;
      const double* src = m == 0 ? a.E + e * Q2
                        : m <= 3 ? a.star + (e * 3 + (m - 1)) * Q2
                        : m <= 7 ? a.Gp + (e * 4 + (m - 4)) * Q2
                                 : a.Gm + (e * 4 + (m - 8)) * Q2;
      gs[k] = i < 12 * Q2 ? src[j] : 0.0;
    }
  };
  auto stash = [&]() __attribute__((always_inline)) {
#pragma unroll
    for (int s = 0; s < 5; ++s)
#pragma unroll
      for (int k = 0; k < C::kXPer; ++k) {
        const int i = tid + k * kCorrThreads;
        if (i < QB) X[s * QB + i] = xs[s][k];
      }
#pragma unroll
    for (int k = 0; k < C::kGPer; ++k) {
      const int i = tid + k * kCorrThreads;
      if (i < 12 * Q2) G[i] = i / Q2 >= 4 ? -gs[k] : gs[k];  // face terms enter with a minus sign
    }
  };
  for (int64_t e = blockIdx.x; e < a.n; e += gridDim.x) {
    fetch(e);
    __syncthreads();  // the previous element's LDS reads are done
    stash();
    int code[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) code[f] = a.nb_code[e * 4 + f];
    // this wave's B operands (table entries) of term m: tile t = wave + 4 tt,
    // inner step s; zero outside the B x B table
    auto load_b = [&](int m, double (&bv)[C::TPW][C::KS]) __attribute__((always_inline)) {
      const double* T = m < 3 ? Vt + m * BB
                       : m < 7 ? Fl + (m - 3) * BB
                               : Fn + (static_cast<size_t>(m - 7) * 24 + code[m - 7]) * BB;
#pragma unroll
      for (int tt = 0; tt < C::TPW; ++tt) {
        const int col = 16 * (wave + kCorrWaves * tt) + lane % 16;
#pragma unroll
        for (int s = 0; s < C::KS; ++s) {
          const int row = 4 * s + lane / 16;
          bv[tt][s] = (row < B && col < B) ? T[row * B + col] : 0.0;
        }
      }
    };
    v4d acc[C::TPW];
#pragma unroll
    for (int tt = 0; tt < C::TPW; ++tt) acc[tt] = v4d{0.0, 0.0, 0.0, 0.0};
    double bv[C::kBuf][C::TPW][C::KS];
    if constexpr (C::kPrefetch) load_b(0, bv[1]);  // overlaps the first W phase
    for (int m0 = 0; m0 < kTerms; m0 += WN) {
      const int mcount = kTerms - m0 < WN ? kTerms - m0 : WN;
      __syncthreads();  // staging done (first group) / previous group's W reads done
      // W_m = G_m X_m for the group's terms (vector ALU)
      for (int i = tid; i < mcount * QB; i += kCorrThreads) {
        const int mm = i / QB, r = i % QB, p = r / B, l = r % B;
        const int m = m0 + mm;
        const double* Xm = X + (m < 7 ? 0 : (m - 6) * QB);
        const double* Gm = G + (1 + m) * Q2 + p * NQ;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) s = fma(Gm[q], Xm[q * B + l], s);
        W[mm * C::kW + p * C::WS + l] = s;
      }
      __syncthreads();
      // accumulate W_m T_m on the matrix cores: wave w owns column tiles
      // w, w + 4, ... (waves without a tile skip this, wave-uniformly)
      if (wave < C::NT) {
        for (int mm = 0; mm < mcount; ++mm) {
          const int m = m0 + mm;
          if constexpr (C::kPrefetch) {
#pragma unroll
            for (int tt = 0; tt < C::TPW; ++tt)
#pragma unroll
              for (int s = 0; s < C::KS; ++s) bv[0][tt][s] = bv[1][tt][s];
            if (m + 1 < kTerms) load_b(m + 1, bv[1]);
          } else {
            load_b(m, bv[0]);
          }
          const double* Wm = W + mm * C::kW + (lane % 16) * C::WS + lane / 16;
#pragma unroll
          for (int s = 0; s < C::KS; ++s) {
            const double av = Wm[4 * s];
#pragma unroll
            for (int tt = 0; tt < C::TPW; ++tt)
              if (wave + kCorrWaves * tt < C::NT)  // wave-uniform
                acc[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[0][tt][s], acc[tt], 0, 0, 0);
          }
        }
      }
    }
    // + E Qint, then Q += the accumulated update
#pragma unroll
    for (int tt = 0; tt < C::TPW; ++tt) {
      const int t = wave + kCorrWaves * tt;
      if (t < C::NT) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int i, j;
          acc_pos(lane, r, i, j);
          j += 16 * t;
          if (i < NQ && j < B) {
            double v = acc[tt][r];
#pragma unroll
            for (int q = 0; q < NQ; ++q) v = fma(G[i * NQ + q], X[q * B + j], v);
            a.Q[e * QB + i * B + j] += v;
          }
        }
      }
    }
  }
}

template <int NQ, int N>
hipError_t launch_one(const CorrectArgs& a, hipStream_t stream) {
  using C = CorrCfg<NQ, N>;
  const int64_t blocks64 = a.n < 65536 ? a.n : 65536;
  if (C::kLds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(corrector_kernel<NQ, N>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(C::kLds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((corrector_kernel<NQ, N>), dim3(static_cast<unsigned>(blocks64)), dim3(kCorrThreads), C::kLds,
                     stream, a);
  return hipGetLastError();
}

template <int NQ>
hipError_t launch_nq(const CorrectArgs& a, hipStream_t stream) {
  switch (a.B) {
    case n_modes(0): return launch_one<NQ, 0>(a, stream);
    case n_modes(1): return launch_one<NQ, 1>(a, stream);
    case n_modes(2): return launch_one<NQ, 2>(a, stream);
    case n_modes(3): return launch_one<NQ, 3>(a, stream);
    case n_modes(4): return launch_one<NQ, 4>(a, stream);
    case n_modes(5): return launch_one<NQ, 5>(a, stream);
    case n_modes(6): return launch_one<NQ, 6>(a, stream);
    case n_modes(7): return launch_one<NQ, 7>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool corrector_fits(int nq, int B) {
  if (!supported_nq(nq)) return false;
  for (int N = 0; N <= kMaxDegree; ++N)
    if (n_modes(N) == B) return true;
  return false;
}

hipError_t launch_corrector(const CorrectArgs& a, hipStream_t stream) {
  if (a.n <= 0) return hipSuccess;
  if (a.nq == kNQPoro) return launch_nq<kNQPoro>(a, stream);
  if (a.nq == kNQMaxwell) return launch_nq<kNQMaxwell>(a, stream);
  return hipErrorInvalidValue;
}

}  // namespace stp
