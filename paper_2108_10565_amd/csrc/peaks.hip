// Machine ceilings for the roofline (stp_measure_peaks, include/stp.h): the
// paper places its predictor against the peak FLOP/s and bandwidth measured
// on the node itself (subsection "Roofline model"); these kernels measure the
// same ceilings on the GPU.
//
// FMA loops: every thread runs kChains independent chains x <- x * a + b
// (runtime a, b, trip count), so the loop cannot be folded and the chains
// hide the FMA latency; one result per thread is stored so nothing is dead.
// Matrix cores: independent accumulators of the 16x16x4 float64 MFMA.
// Streams: grid-stride copy and fill of 16-byte vectors through HBM (best of
// three grid sizes, streaming and ordinary accesses).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/stp.h"

namespace {

constexpr int kPeakThreads = 256;
constexpr int kPeakBlocks = 2048;        // 8 workgroups of 4 waves per compute unit
constexpr int kChains = 16;
constexpr int kMfmaAcc = 8;
constexpr int kFmaIters = 65536;
constexpr int kMfmaIters = 8192;
constexpr int kMfmaUnroll = 16;
static_assert(kMfmaIters % kMfmaUnroll == 0, "whole unrolled bodies");
constexpr size_t kOutBytes = static_cast<size_t>(kPeakBlocks) * kPeakThreads * sizeof(double);

template <typename F>
__global__ __launch_bounds__(kPeakThreads) void fma_loop(F a, F b, int iters, F* out) {
  F x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = static_cast<F>(threadIdx.x + c) * static_cast<F>(1e-3);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], a, b);
  }
  F s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

using v4d = double __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kPeakThreads) void mfma_f64_loop(double a, double b, int iters, double* out) {
  v4d acc[kMfmaAcc];
#pragma unroll
  for (int k = 0; k < kMfmaAcc; ++k) acc[k] = v4d{0.0, 0.0, 0.0, 0.0};
  const double av = a + 1e-9 * threadIdx.x;
  // unrolled by kMfmaUnroll (iters is a multiple of it): the compiler keeps
  // the accumulators in the matrix-core registers across a whole unrolled
  // body and copies them to and from the vector registers only at the loop
  // back-edge, which a rolled loop does on every iteration
  for (int i = 0; i < iters; i += kMfmaUnroll) {
#pragma unroll
    for (int r = 0; r < kMfmaUnroll; ++r) {
#pragma unroll
      for (int k = 0; k < kMfmaAcc; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b, acc[k], 0, 0, 0);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kMfmaAcc; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

typedef double d2 __attribute__((ext_vector_type(2)));

// Streams: each thread moves kUnroll 16-byte vectors per iteration (all loads
// issued before the stores; one global_load_dwordx4 / global_store_dwordx4
// per vector), as streaming (non-temporal) or ordinary accesses; n is a
// multiple of kUnroll * threads in the grid.  The rate reported is the best
// of a few grid sizes and both access kinds.
constexpr int kUnroll = 4;

template <bool kStreaming>
__global__ __launch_bounds__(kPeakThreads) void copy_stream(const d2* src, d2* dst, int64_t n) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kPeakThreads;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kPeakThreads) + threadIdx.x; i < n; i += kUnroll * stride) {
    d2 v[kUnroll];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) v[k] = kStreaming ? __builtin_nontemporal_load(&src[i + k * stride]) : src[i + k * stride];
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if constexpr (kStreaming) __builtin_nontemporal_store(v[k], &dst[i + k * stride]);
      else dst[i + k * stride] = v[k];
    }
  }
}

template <bool kStreaming>
__global__ __launch_bounds__(kPeakThreads) void fill_stream(d2* dst, int64_t n, double v) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kPeakThreads;
  const d2 vv = {v, v};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kPeakThreads) + threadIdx.x; i < n; i += kUnroll * stride) {
#pragma unroll
    for (int k = 0; k < kUnroll; ++k) {
      if constexpr (kStreaming) __builtin_nontemporal_store(vv, &dst[i + k * stride]);
      else dst[i + k * stride] = vv;
    }
  }
}

// Launches `launch` once untimed, then `reps` times between two events;
// returns the mean milliseconds per launch (negative on a HIP error).
template <class L>
double time_ms(hipStream_t stream, int reps, L&& launch) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -1.0;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -1.0;
  }
  double ms = -1.0;
  launch();
  if (hipGetLastError() == hipSuccess && hipEventRecord(e0, stream) == hipSuccess) {
    for (int r = 0; r < reps; ++r) launch();
    float t = 0.0f;
    if (hipGetLastError() == hipSuccess && hipEventRecord(e1, stream) == hipSuccess &&
        hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&t, e0, e1) == hipSuccess)
      ms = static_cast<double>(t) / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}

}  // namespace

extern "C" stp_status stp_measure_peaks(stp_handle handle, void* hip_stream, void* scratch, size_t scratch_bytes,
                                        stp_peaks* peaks) {
  if (!handle || !scratch || !peaks) return STP_EINVAL;
  constexpr size_t kMinScratch = size_t{1} << 30;
  if (scratch_bytes < kMinScratch) return STP_EWORKSPACE;
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  const dim3 grid(kPeakBlocks), block(kPeakThreads);
  const double threads = static_cast<double>(kPeakBlocks) * kPeakThreads;

  double* out64 = static_cast<double*>(scratch);
  float* out32 = static_cast<float*>(scratch);
  const double t64 = time_ms(stream, 3, [&] {
    hipLaunchKernelGGL(fma_loop<double>, grid, block, 0, stream, 0.999999, 1e-7, kFmaIters, out64);
  });
  const double t32 = time_ms(stream, 3, [&] {
    hipLaunchKernelGGL(fma_loop<float>, grid, block, 0, stream, 0.999999f, 1e-7f, kFmaIters, out32);
  });
  const double tm = time_ms(stream, 3, [&] {
    hipLaunchKernelGGL(mfma_f64_loop, grid, block, 0, stream, 1e-3, 1e-3, kMfmaIters, out64);
  });
  // streams over the buffer past the FMA results, split in two halves; the
  // grid sizes (workgroups of 256) all divide the vector count
  constexpr int kGrids[3] = {4096, 1024, 512};
  const int64_t unit = static_cast<int64_t>(kUnroll) * kGrids[0] * kPeakThreads;   // vectors per largest sweep
  const int64_t n = static_cast<int64_t>((scratch_bytes - kOutBytes) / 2 / sizeof(d2)) / unit * unit;
  d2* half0 = reinterpret_cast<d2*>(static_cast<char*>(scratch) + kOutBytes);
  d2* half1 = half0 + n;
  double tf = 1e30, tc = 1e30;
  bool stream_error = false;
  for (int gi = 0; gi < 3; ++gi) {
    const dim3 sgrid(kGrids[gi]);
    for (int nt = 0; nt < 2; ++nt) {
      const double f = time_ms(stream, 5, [&] {
        if (nt) hipLaunchKernelGGL(fill_stream<true>, sgrid, block, 0, stream, half0, n, 1.0);
        else hipLaunchKernelGGL(fill_stream<false>, sgrid, block, 0, stream, half0, n, 1.0);
      });
      const double c = time_ms(stream, 5, [&] {
        if (nt) hipLaunchKernelGGL(copy_stream<true>, sgrid, block, 0, stream, static_cast<const d2*>(half0), half1, n);
        else hipLaunchKernelGGL(copy_stream<false>, sgrid, block, 0, stream, static_cast<const d2*>(half0), half1, n);
      });
      if (f <= 0 || c <= 0) stream_error = true;
      tf = f < tf ? f : tf;
      tc = c < tc ? c : tc;
    }
  }
  if (stream_error) tf = tc = -1.0;
  if (t64 <= 0 || t32 <= 0 || tm <= 0 || tf <= 0 || tc <= 0) {
    (void)hipGetLastError();
    return STP_EHIP;
  }
  const double fma_flop = threads * kFmaIters * kChains * 2.0;
  const double mfma_flop = threads / 64.0 * kMfmaIters * kMfmaAcc * (2.0 * 16 * 16 * 4);
  peaks->fp64_valu_tflops = fma_flop / (t64 * 1e-3) / 1e12;
  peaks->fp32_valu_tflops = fma_flop / (t32 * 1e-3) / 1e12;
  peaks->fp64_mfma_tflops = mfma_flop / (tm * 1e-3) / 1e12;
  peaks->hbm_write_gbs = static_cast<double>(n) * sizeof(d2) / (tf * 1e-3) / 1e9;
  peaks->hbm_copy_gbs = 2.0 * static_cast<double>(n) * sizeof(d2) / (tc * 1e-3) / 1e9;
  return STP_OK;
}
