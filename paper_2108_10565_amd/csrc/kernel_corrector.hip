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
// One workgroup per element: the own and the four neighbours' Qint are
// staged in LDS; each of the 11 operator terms is formed as W = G X (nq x B,
// LDS) and accumulated into the per-thread outputs as W T.
#include "common.hpp"

namespace stp {
namespace {

constexpr int kCorrThreads = 256;
constexpr int kMaxOut = 8;  // outputs per thread: nq * B <= kMaxOut * kCorrThreads

__global__ __launch_bounds__(kCorrThreads) void corrector_kernel(CorrectArgs a) {
  extern __shared__ double lds[];
  const int nq = a.nq, B = a.B, tid = threadIdx.x;
  const int QB = nq * B;
  double* X = lds;              // [5][nq][B]: own Qint, then the 4 neighbours'
  double* W = lds + 5 * QB;     // [nq][B]
  const size_t BB = static_cast<size_t>(B) * B;
  const double* V = a.tables;                 // [3][B][B]
  const double* Fl = a.tables + 3 * BB;       // [4][B][B]
  const double* Fn = a.tables + 7 * BB;       // [4][4][6][B][B]
  const size_t q2 = static_cast<size_t>(nq) * nq;
  for (int64_t e = blockIdx.x; e < a.n; e += gridDim.x) {
    __syncthreads();  // the previous element's LDS reads are done
    for (int s = 0; s < 5; ++s) {
      const int64_t src = s == 0 ? e : a.neighbor[e * 4 + (s - 1)];
      for (int i = tid; i < QB; i += kCorrThreads) X[s * QB + i] = a.Qint[src * QB + i];
    }
    __syncthreads();
    double out[kMaxOut];
    // source term E Qint
#pragma unroll
    for (int r = 0; r < kMaxOut; ++r) {
      const int o = tid + r * kCorrThreads;
      double acc = 0.0;
      if (o < QB) {
        const int p = o / B, k = o % B;
        const double* Erow = a.E + e * q2 + p * nq;
        for (int q = 0; q < nq; ++q) acc = fma(Erow[q], X[q * B + k], acc);
      }
      out[r] = acc;
    }
    for (int m = 0; m < 11; ++m) {
      // operator G (nq x nq), input X_m, table T (B x B) and sign of the term
      const double* G;
      const double* Xm = X;
      const double* T;
      double sgn;
      if (m < 3) {
        G = a.star + (e * 3 + m) * q2;
        T = V + m * BB;
        sgn = 1.0;
      } else if (m < 7) {
        const int f = m - 3;
        G = a.Gp + (e * 4 + f) * q2;
        T = Fl + f * BB;
        sgn = -1.0;
      } else {
        const int f = m - 7;
        const int code = a.nb_code[e * 4 + f];  // 6 j + h
        G = a.Gm + (e * 4 + f) * q2;
        Xm = X + (1 + f) * QB;
        T = Fn + (static_cast<size_t>(f) * 24 + code) * BB;
        sgn = -1.0;
      }
      for (int i = tid; i < QB; i += kCorrThreads) {
        const int p = i / B, l = i % B;
        double acc = 0.0;
        for (int q = 0; q < nq; ++q) acc = fma(G[p * nq + q], Xm[q * B + l], acc);
        W[i] = acc;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kMaxOut; ++r) {
        const int o = tid + r * kCorrThreads;
        if (o < QB) {
          const int p = o / B, k = o % B;
          double acc = 0.0;
          for (int l = 0; l < B; ++l) acc = fma(W[p * B + l], T[l * B + k], acc);
          out[r] = fma(sgn, acc, out[r]);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kMaxOut; ++r) {
      const int o = tid + r * kCorrThreads;
      if (o < QB) a.Q[e * QB + o] += out[r];
    }
  }
}

}  // namespace

size_t corrector_lds_bytes(int nq, int B) { return static_cast<size_t>(6) * nq * B * sizeof(double); }

bool corrector_fits(int nq, int B) {
  return nq * B <= kMaxOut * kCorrThreads && corrector_lds_bytes(nq, B) <= 160 * 1024;
}

hipError_t launch_corrector(const CorrectArgs& a, hipStream_t stream) {
  if (a.n <= 0) return hipSuccess;
  const int64_t blocks64 = a.n < 65536 ? a.n : 65536;
  const size_t lds = corrector_lds_bytes(a.nq, a.B);
  if (lds > 64 * 1024) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(corrector_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(corrector_kernel, dim3(static_cast<unsigned>(blocks64)), dim3(kCorrThreads), lds, stream, a);
  return hipGetLastError();
}

}  // namespace stp
