// Reference GPU kernel: Algorithm 3 of Wolf et al. (arXiv 2108.10565,
// section "Block-wise back-substitution") in its literal order, one element
// per workgroup, everything staged in LDS, float64.
//
// Per element:
//   b <- Q0 o (S^-1 w)
//   for degree block g = N .. 0 (modes m in [block_start(g), +block_size(g))):
//     for p = 12 .. 0:
//       Q[p, m, :] <- (Z - E*_pp I)^-1 b[p, m, :]          (dark-blue blocks)
//       b[o, m, :] += G_op Q[p, m, :]  for o < p           (G = strict upper E*)
//     if g > 0, for each direction j:                      (green blocks)
//       Y_j[p, m, u] = sum_q A^{j*}_pq Q[q, m, u]
//       b[p, n, u] -= sum_m Khat^j[n, m] Y_j[p, m, u]     for n < block_start(g)
// with A^{j*} = dt A^j and E* = dt E.  Z - z I is inverted by Gauss-Jordan
// elimination without pivoting (its eigenvalues have real part >= 1 for
// z <= 0.5, and the elimination is accurate to ~1e-15 there).
//
// Slow by design (13 barriers per degree block and per quantity), fully
// general in the upper-triangular E and in the star matrices.
#include "common.hpp"
#include "generated/khat_tables.h"

namespace stp {
namespace {

constexpr int kNQ = kNQPoro;  // the reference kernel is for the poroelastic system

template <int N>
__device__ __forceinline__ const double* khat_dense();
#define STP_KHAT_DENSE(NN) \
  template <> __device__ __forceinline__ const double* khat_dense<NN>() { return stp_gen::kKhatDense##NN; }
STP_KHAT_DENSE(0)
STP_KHAT_DENSE(1)
STP_KHAT_DENSE(2)
STP_KHAT_DENSE(3)
STP_KHAT_DENSE(4)
STP_KHAT_DENSE(5)
STP_KHAT_DENSE(6)
STP_KHAT_DENSE(7)
#undef STP_KHAT_DENSE

constexpr int kRefThreads = 256;

template <int N>
struct RefShared {
  static constexpr int B = n_modes(N), T = N + 1, D = block_size(N);
  static constexpr int kY = (kNQ * D * T > kNQ * T * 2 * T) ? kNQ * D * T : kNQ * T * 2 * T;
  double b[kNQ * B * T];   // right-hand side, overwritten block by block by Q
  double y[kY];            // Y_j of the current block; Gauss-Jordan scratch
  double A[3 * kNQ * kNQ]; // dt * star
  double Es[kNQ * kNQ];    // dt * E, lower part zeroed
  double Zinv[kNQ * T * T];
};

template <int N>
__global__ __launch_bounds__(kRefThreads) void stp_reference_kernel(PredictArgs a) {
  constexpr int B = n_modes(N), T = N + 1;
  __shared__ RefShared<N> s;
  const int tid = threadIdx.x;
  const double* Kd = khat_dense<N>();
  for (int64_t e = blockIdx.x; e < a.n; e += gridDim.x) {
    const double* star = a.star + e * (3 * kNQ * kNQ);
    const double* E = a.E + e * (kNQ * kNQ);
    const double* Q0 = a.Q0 + e * (kNQ * B);
    double* Q = a.Q + e * (kNQ * B * T);
    for (int t = tid; t < 3 * kNQ * kNQ; t += kRefThreads) s.A[t] = a.dt * star[t];
    unsigned bad = 0;
    for (int t = tid; t < kNQ * kNQ; t += kRefThreads) {
      const int r = t / kNQ, c = t % kNQ;
      const double v = a.dt * E[t];
      if (c < r && v != 0.0) bad |= kInputNotUpper;
      if (c == r && v >= 0.5) bad |= kInputSingular;
      s.Es[t] = (c >= r) ? v : 0.0;
    }
    if (bad && a.status) atomicOr(a.status, bad);
    __syncthreads();
    // (Z - E*_pp I)^-1 for every quantity, one thread each
    if (tid < kNQ) {
      const int p = tid;
      double* m = &s.y[p * T * 2 * T];
      const double z = s.Es[p * kNQ + p];
      for (int u = 0; u < T; ++u)
        for (int v = 0; v < 2 * T; ++v)
          m[u * 2 * T + v] = (v < T) ? (z_entry(u, v) - (u == v ? z : 0.0)) : ((v - T) == u ? 1.0 : 0.0);
      for (int k = 0; k < T; ++k) {
        const double inv = 1.0 / m[k * 2 * T + k];
        for (int v = 0; v < 2 * T; ++v) m[k * 2 * T + v] *= inv;
        for (int u = 0; u < T; ++u) {
          if (u == k) continue;
          const double f = m[u * 2 * T + k];
          for (int v = 0; v < 2 * T; ++v) m[u * 2 * T + v] -= f * m[k * 2 * T + v];
        }
      }
      for (int u = 0; u < T; ++u)
        for (int v = 0; v < T; ++v) s.Zinv[(p * T + u) * T + v] = m[u * 2 * T + T + v];
    }
    for (int t = tid; t < kNQ * B * T; t += kRefThreads) {
      const int u = t % T, pl = t / T;
      s.b[t] = Q0[pl] * sinv_w(u);
    }
    __syncthreads();
    for (int g = N; g >= 0; --g) {
      const int L0 = block_start(g), d = block_size(g);
      for (int p = kNQ - 1; p >= 0; --p) {
        // X[p, m, :] = Zinv_p b[p, m, :] for m in the block
        constexpr int kMaxPer = (block_size(N) * (N + 1) + kRefThreads - 1) / kRefThreads;
        double xv[kMaxPer];
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r) {
          const int t = tid + r * kRefThreads;
          xv[r] = 0.0;
          if (t < d * T) {
            const int m = L0 + t / T, sidx = t % T;
            const double* bb = &s.b[(p * B + m) * T];
            double acc = 0.0;
            for (int u = 0; u < T; ++u) acc += s.Zinv[(p * T + sidx) * T + u] * bb[u];
            xv[r] = acc;
          }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r) {
          const int t = tid + r * kRefThreads;
          if (t < d * T) s.b[(p * B + L0 + t / T) * T + t % T] = xv[r];
        }
        __syncthreads();
        // b[o, m, :] += G_op X[p, m, :] for o < p with G_op != 0
        bool any = false;
        for (int o = 0; o < p; ++o) any |= (s.Es[o * kNQ + p] != 0.0);
        if (any) {
          for (int t = tid; t < p * d * T; t += kRefThreads) {
            const int o = t / (d * T), r = t % (d * T);
            const double gop = s.Es[o * kNQ + p];
            if (gop != 0.0) s.b[(o * B + L0) * T + r] += gop * s.b[(p * B + L0) * T + r];
          }
          __syncthreads();
        }
      }
      // the block's space-time DOFs are final: write them out
      for (int t = tid; t < kNQ * d * T; t += kRefThreads) {
        const int p = t / (d * T), r = t % (d * T);
        Q[(p * B + L0) * T + r] = s.b[(p * B + L0) * T + r];
      }
      if (g == 0) break;
      for (int j = 0; j < 3; ++j) {
        for (int t = tid; t < kNQ * d * T; t += kRefThreads) {
          const int p = t / (d * T), r = t % (d * T);
          const int m = r / T, u = r % T;
          double acc = 0.0;
          for (int q = 0; q < kNQ; ++q) acc += s.A[(j * kNQ + p) * kNQ + q] * s.b[(q * B + L0 + m) * T + u];
          s.y[t] = acc;
        }
        __syncthreads();
        for (int t = tid; t < kNQ * L0 * T; t += kRefThreads) {
          const int p = t / (L0 * T), r = t % (L0 * T);
          const int n = r / T, u = r % T;
          double acc = 0.0;
          for (int m = 0; m < d; ++m)
            acc += Kd[(j * B + n) * B + L0 + m] * s.y[(p * d + m) * T + u];
          s.b[(p * B + n) * T + u] -= acc;
        }
        __syncthreads();
      }
    }
    if (a.Qint) {
      for (int t = tid; t < kNQ * B; t += kRefThreads) a.Qint[e * (kNQ * B) + t] = a.dt * s.b[t * T];
    }
    __syncthreads();
  }
}

template <int N>
hipError_t launch_ref(const PredictArgs& a, hipStream_t stream) {
  const int64_t blocks = a.n < 65536 ? a.n : 65536;
  hipLaunchKernelGGL(stp_reference_kernel<N>, dim3(static_cast<unsigned>(blocks)), dim3(kRefThreads), 0,
                     stream, a);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_reference_kernel(int N, const PredictArgs& a, hipStream_t stream) {
  switch (N) {
    case 0: return launch_ref<0>(a, stream);
    case 1: return launch_ref<1>(a, stream);
    case 2: return launch_ref<2>(a, stream);
    case 3: return launch_ref<3>(a, stream);
    case 4: return launch_ref<4>(a, stream);
    case 5: return launch_ref<5>(a, stream);
    case 6: return launch_ref<6>(a, stream);
    case 7: return launch_ref<7>(a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace stp
