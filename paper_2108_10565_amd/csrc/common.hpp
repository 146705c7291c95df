// Compile-time sizes and temporal constants shared by the HIP kernels.
//
// Temporal basis chi_s(tau) = P_s(2 tau - 1) on [0, 1] (section "Space-Time
// predictor" of Wolf et al., arXiv 2108.10565):
//   S_rs = delta_rs / (2s+1),  W_rs = 1,  w_r = (-1)^r,
//   K^tau_rs = 2 if r > s and r - s odd, else 0,
// so Z = S^-1 (W - K^tau) (section "Block-wise back-substitution") has the
// integer entries Z_us = (2u+1) * (u > s and u - s odd ? -1 : 1), and
// (S^-1 w)_u = (2u+1) (-1)^u.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace stp {

// Quantity counts the fused kernels are compiled for: the poroelastic system
// and the damped Maxwell system of section "Other applications" (any system
// whose source matrix is upper triangular runs through the same kernels).
constexpr int kNQPoro = 13;
constexpr int kNQMaxwell = 6;
__host__ __device__ constexpr bool supported_nq(int nq) { return nq == kNQPoro || nq == kNQMaxwell; }
constexpr int kMaxDegree = 7;

__host__ __device__ constexpr int n_modes(int N) { return (N + 1) * (N + 2) * (N + 3) / 6; }
__host__ __device__ constexpr int block_size(int g) { return (g + 1) * (g + 2) / 2; }
__host__ __device__ constexpr int block_start(int g) { return g * (g + 1) * (g + 2) / 6; }

__host__ __device__ constexpr double z_entry(int u, int s) {
  return (2.0 * u + 1.0) * ((u > s && ((u - s) & 1)) ? -1.0 : 1.0);
}
__host__ __device__ constexpr double sinv_w(int u) { return (2.0 * u + 1.0) * ((u & 1) ? -1.0 : 1.0); }

// Launch arguments common to every kernel.  All pointers are device pointers.
struct PredictArgs {
  int64_t n;             // elements
  double dt;
  const double* star;    // [n][3][13][13]
  const double* E;       // [n][13][13]
  const double* Q0;      // [n][13][B]
  double* Q;             // [n][13][B][T]
  double* Qint;          // [n][13][B] or nullptr
  unsigned* status;      // device word the kernels OR input conditions into (kInput*), or nullptr
};

// Input conditions the prediction kernels report (they run without pivoting
// and take E as upper triangular; section "Block-wise back-substitution").
constexpr unsigned kInputSingular = 1u;  // some dt E_pp >= 0.5
constexpr unsigned kInputNotUpper = 2u;  // a non-zero below the diagonal of some E

// Arguments of the corrector kernel (device pointers except the sizes).
struct CorrectArgs {
  int64_t n;              // elements
  int nq, B;              // quantities, spatial modes
  const double* tables;   // V [3][B][B], Fl [4][B][B], Fn [4][4][6][B][B]
  const double* star;     // [n][3][nq][nq]
  const double* E;        // [n][nq][nq]
  const double* Gp;       // [n][4][nq][nq]
  const double* Gm;       // [n][4][nq][nq]
  const int32_t* neighbor;  // [n][4] element behind each face
  const int32_t* nb_code;   // [n][4] 6 j + h: neighbour's face j, vertex correspondence h
  const double* Qint;     // [n][nq][B]
  double* Q;              // [n][nq][B], updated in place
};
hipError_t launch_corrector(const CorrectArgs& a, hipStream_t stream);
bool corrector_fits(int nq, int B);

// Bytes of workspace the mixed-precision path needs: the float residual of
// every element between the residual and the correction kernels.
inline size_t workspace_bytes(int nq, int N, int64_t n, int precision, int refine_steps) {
  if (precision == 0 || refine_steps == 0 || n <= 0) return 0;
  const size_t raw = static_cast<size_t>(n) * nq * n_modes(N) * (N + 1) * sizeof(float);
  return (raw + 255) / 256 * 256;
}

// Launchers (one per kernel family); return hipSuccess or the launch error.
hipError_t launch_reference_kernel(int N, const PredictArgs& a, hipStream_t stream);
// The fused kernels are compiled once per (quantity count STP_NQ, degree
// STP_DEGREE); each object defines the specialisation for its pair.
// valu_float_chain: the float32 chain's green update as sparse fused
// multiply-adds on the vector ALU (default); false: on the matrix cores.
template <int NQ, int N>
hipError_t launch_fused(const PredictArgs& a, int precision, int refine_steps, float* workspace,
                        bool valu_float_chain, hipStream_t stream);
#define STP_DECLARE_FUSED(Q)                                                                             \
  template <> hipError_t launch_fused<Q, 0>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 1>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 2>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 3>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 4>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 5>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 6>(const PredictArgs&, int, int, float*, bool, hipStream_t);  \
  template <> hipError_t launch_fused<Q, 7>(const PredictArgs&, int, int, float*, bool, hipStream_t);
STP_DECLARE_FUSED(13)
STP_DECLARE_FUSED(6)
#undef STP_DECLARE_FUSED

template <int NQ>
inline hipError_t launch_fused_nq(int N, const PredictArgs& a, int precision, int refine_steps, float* workspace,
                                  bool valu_float_chain, hipStream_t stream) {
  switch (N) {
    case 0: return launch_fused<NQ, 0>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 1: return launch_fused<NQ, 1>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 2: return launch_fused<NQ, 2>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 3: return launch_fused<NQ, 3>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 4: return launch_fused<NQ, 4>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 5: return launch_fused<NQ, 5>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 6: return launch_fused<NQ, 6>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    case 7: return launch_fused<NQ, 7>(a, precision, refine_steps, workspace, valu_float_chain, stream);
    default: return hipErrorInvalidValue;
  }
}

inline hipError_t launch_fused_kernel(int nq, int N, const PredictArgs& a, int precision, int refine_steps,
                                      float* workspace, bool valu_float_chain, hipStream_t stream) {
  if (nq == kNQPoro) return launch_fused_nq<kNQPoro>(N, a, precision, refine_steps, workspace, valu_float_chain, stream);
  if (nq == kNQMaxwell)
    return launch_fused_nq<kNQMaxwell>(N, a, precision, refine_steps, workspace, valu_float_chain, stream);
  return hipErrorInvalidValue;
}

}  // namespace stp
