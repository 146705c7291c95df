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
// One workgroup per element: the own Qint is staged in LDS; for each of the
// 11 operator terms the table T (B x B), the operator G (nq x nq) and, for a
// neighbour term, that neighbour's Qint are staged too, W = G X (nq x B) is formed in LDS,
// and each thread accumulates W T for one column k and every (256 / B)-th row
// (the table entry T[l][k] is reused across its rows, W[p][l] is a
// broadcast read).
#include "common.hpp"

namespace stp {
namespace {

constexpr int kCorrThreads = 256;
constexpr int kMaxRows = 7;  // rows per thread: ceil(nq / (256 / B)) <= 7 for nq <= 13, B <= 120

// LDS: X [nq][B] (own Qint), Xn [nq][B] (the current face neighbour's
// Qint), W [nq][B], T [B][B] (the term's table), G [nq][nq] (the term's
// operator): 154 KB at degree 7 with 13 quantities.
__host__ __device__ constexpr size_t corrector_lds_doubles(int nq, int B) {
  return static_cast<size_t>(3) * nq * B + static_cast<size_t>(B) * B + static_cast<size_t>(nq) * nq;
}

__global__ __launch_bounds__(kCorrThreads) void corrector_kernel(CorrectArgs a) {
  extern __shared__ double lds[];
  const int nq = a.nq, B = a.B, tid = threadIdx.x;
  const int QB = nq * B;
  double* X = lds;                  // [nq][B]
  double* Xn = X + QB;              // [nq][B]
  double* W = Xn + QB;              // [nq][B]
  double* T = W + QB;               // [B][B]
  double* G = T + B * B;            // [nq][nq]
  const size_t BB = static_cast<size_t>(B) * B;
  const double* Vt = a.tables;                 // [3][B][B]
  const double* Fl = a.tables + 3 * BB;        // [4][B][B]
  const double* Fn = a.tables + 7 * BB;        // [4][4][6][B][B]
  const int q2 = nq * nq;
  // output block of this thread: column k, rows p0, p0 + groups, ...
  const int groups = kCorrThreads / B;             // >= 2 for B <= 120
  const int k = tid % B, p0 = tid / B;
  const bool has = tid < groups * B && p0 < nq;
  for (int64_t e = blockIdx.x; e < a.n; e += gridDim.x) {
    __syncthreads();  // the previous element's LDS reads are done
    for (int i = tid; i < QB; i += kCorrThreads) X[i] = a.Qint[e * QB + i];
    for (int i = tid; i < q2; i += kCorrThreads) G[i] = a.E[e * q2 + i];
    __syncthreads();
    double out[kMaxRows];
    // source term E Qint
#pragma unroll
    for (int r = 0; r < kMaxRows; ++r) {
      const int p = p0 + r * groups;
      double acc = 0.0;
      if (has && p < nq)
        for (int q = 0; q < nq; ++q) acc = fma(G[p * nq + q], X[q * B + k], acc);
      out[r] = acc;
    }
    for (int m = 0; m < 11; ++m) {
      // operator G (nq x nq), input Xm, table T (B x B) and sign of the term
      const double* Gg;
      const double* Tg;
      const double* Xm = X;
      double sgn = -1.0;
      if (m < 3) {
        Gg = a.star + (e * 3 + m) * q2;
        Tg = Vt + m * BB;
        sgn = 1.0;
      } else if (m < 7) {
        const int f = m - 3;
        Gg = a.Gp + (e * 4 + f) * q2;
        Tg = Fl + f * BB;
      } else {
        const int f = m - 7;
        const int code = a.nb_code[e * 4 + f];  // 6 j + h
        Gg = a.Gm + (e * 4 + f) * q2;
        Tg = Fn + (static_cast<size_t>(f) * 24 + code) * BB;
        Xm = Xn;
      }
      __syncthreads();  // the previous term's reads of G, Xn, W and T are done
      for (int i = tid; i < static_cast<int>(BB); i += kCorrThreads) T[i] = Tg[i];
      for (int i = tid; i < q2; i += kCorrThreads) G[i] = Gg[i];
      if (m >= 7) {
        const int64_t nb = a.neighbor[e * 4 + (m - 7)];
        for (int i = tid; i < QB; i += kCorrThreads) Xn[i] = a.Qint[nb * QB + i];
      }
      __syncthreads();
      for (int i = tid; i < QB; i += kCorrThreads) {
        const int p = i / B, l = i % B;
        double acc = 0.0;
        for (int q = 0; q < nq; ++q) acc = fma(G[p * nq + q], Xm[q * B + l], acc);
        W[i] = acc;
      }
      __syncthreads();
      if (has) {
        double acc[kMaxRows];
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) acc[r] = 0.0;
        for (int l = 0; l < B; ++l) {
          const double t = T[l * B + k];
#pragma unroll
          for (int r = 0; r < kMaxRows; ++r) {
            const int p = p0 + r * groups;
            if (p < nq) acc[r] = fma(W[p * B + l], t, acc[r]);
          }
        }
#pragma unroll
        for (int r = 0; r < kMaxRows; ++r) out[r] = fma(sgn, acc[r], out[r]);
      }
    }
    if (has) {
#pragma unroll
      for (int r = 0; r < kMaxRows; ++r) {
        const int p = p0 + r * groups;
        if (p < nq) a.Q[e * QB + p * B + k] += out[r];
      }
    }
  }
}

}  // namespace

size_t corrector_lds_bytes(int nq, int B) { return corrector_lds_doubles(nq, B) * sizeof(double); }

bool corrector_fits(int nq, int B) {
  const int groups = B <= kCorrThreads ? kCorrThreads / B : 0;
  return groups >= 1 && (nq + groups - 1) / groups <= kMaxRows && corrector_lds_bytes(nq, B) <= 160 * 1024;
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
