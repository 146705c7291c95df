// C ABI of the space-time predictor library (declared in include/stp.h).
// Host-side argument checks, kernel dispatch, data validation, reference
// matrices and FLOP counts.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "../../include/stp.h"
#include "ader_host.hpp"
#include "basis.hpp"
#include "common.hpp"

struct stp_handle_s {
  std::string last_error;
};

struct stp_graph_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

stp_status fail(stp_handle h, stp_status s, const std::string& msg) {
  if (h) h->last_error = msg;
  return s;
}

stp_status hip_fail(stp_handle h, hipError_t err, const char* where) {
  return fail(h, STP_EHIP, std::string(where) + ": " + hipGetErrorString(err));
}

// Validation flags written by the validate kernel.
constexpr int kFlagNonFinite = 1;
constexpr int kFlagNotUpper = 2;
constexpr int kFlagSingular = 4;

__global__ void validate_kernel(int64_t n, int nq, int B, double dt, const double* star, const double* E,
                                const double* Q0, int* flags) {
  const int64_t q2 = static_cast<int64_t>(nq) * nq;
  const int64_t per = 4 * q2 + nq * static_cast<int64_t>(B);
  int f = 0;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n * per;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t e = t / per, r = t % per;
    double v;
    if (r < 3 * q2) {
      v = star[e * 3 * q2 + r];
    } else if (r < 4 * q2) {
      const int k = static_cast<int>(r - 3 * q2), row = k / nq, col = k % nq;
      v = E[e * q2 + k];
      if (row > col && v != 0.0) f |= kFlagNotUpper;
      if (row == col && dt * v >= 0.5) f |= kFlagSingular;
    } else {
      v = Q0[e * nq * B + (r - 4 * q2)];
    }
    if (!std::isfinite(v)) f |= kFlagNonFinite;
  }
  if (f) atomicOr(flags, f);
}

stp_status check_common(stp_handle h, int degree, int64_t n, double dt) {
  if (!h) return STP_EINVAL;
  if (degree < 0 || degree > STP_MAX_DEGREE)
    return fail(h, STP_EDEGREE, "degree must be in 0..7, got " + std::to_string(degree));
  if (n < 0) return fail(h, STP_EINVAL, "n_elements < 0");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(h, STP_EINVAL, "dt must be > 0 and finite");
  return STP_OK;
}

// Checks one prediction request (everything that needs no device access).
stp_status check_predict(stp_handle h, int degree, int64_t n, double dt, const double* star, const double* E,
                         const double* Q0, double* Q, stp_precision precision, int refine_steps,
                         const void* workspace, size_t workspace_bytes, unsigned flags,
                         bool workspace_checked = true, int nq = STP_NQ) {
  if (!stp::supported_nq(nq))
    return fail(h, STP_EINVAL, "no kernels for " + std::to_string(nq) + " quantities (13 or 6)");
  stp_status st = check_common(h, degree, n, dt);
  if (st != STP_OK) return st;
  if (precision != STP_FP64 && precision != STP_FP32_REFINE) return fail(h, STP_EINVAL, "unknown precision");
  if (refine_steps < 0 || refine_steps > STP_MAX_REFINE)
    return fail(h, STP_EINVAL, "refine_steps must be in 0..3");
  if (flags & ~(STP_FLAG_REFERENCE_KERNEL | STP_FLAG_MFMA_FLOAT_CHAIN)) return fail(h, STP_EINVAL, "unknown flags");
  if ((flags & STP_FLAG_REFERENCE_KERNEL) && precision != STP_FP64)
    return fail(h, STP_EINVAL, "the reference kernel is float64 only");
  if (n == 0) return STP_OK;
  if (!star || !E || !Q0 || !Q) return fail(h, STP_EINVAL, "NULL array pointer");
  if ((flags & STP_FLAG_REFERENCE_KERNEL) && nq != STP_NQ)
    return fail(h, STP_EINVAL, "the reference kernel is for the 13-quantity system only");
  const size_t need = stp::workspace_bytes(nq, degree, n, static_cast<int>(precision), refine_steps);
  if (workspace_checked && need > 0 && (!workspace || workspace_bytes < need))
    return fail(h, STP_EWORKSPACE,
                "workspace of " + std::to_string(need) + " bytes needed, got " + std::to_string(workspace_bytes));
  return STP_OK;
}

// Per-device words of the input report: [0] collects what the prediction
// kernels OR into it (stp::kInputSingular, stp::kInputNotUpper), [1]
// receives it when stp_check_inputs takes it.  Host code uses only the
// device address from hipGetSymbolAddress (each device holds its own copy).
static __device__ __align__(64) unsigned input_status[2];

constexpr int kMaxDevices = 64;
std::mutex g_status_mutex;
unsigned* g_status_ptr[kMaxDevices] = {};

// Device that runs `stream` (the NULL stream: the current device), or -1.
int stream_device(hipStream_t stream) {
  if (stream) {
    hipDevice_t d = 0;
    return hipStreamGetDevice(stream, &d) == hipSuccess ? static_cast<int>(d) : -1;
  }
  int cur = -1;
  return hipGetDevice(&cur) == hipSuccess ? cur : -1;
}

// Device address of `input_status` on device `dev`, taken on first use with
// `dev` current; nullptr if it cannot be had (the kernels then report nothing).
unsigned* status_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_status_mutex);
  if (!g_status_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess) return nullptr;
    if (cur != dev && hipSetDevice(dev) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    void* p = nullptr;
    const hipError_t err = hipGetSymbolAddress(&p, HIP_SYMBOL(input_status));
    if (cur != dev) (void)hipSetDevice(cur);
    if (err != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_status_ptr[dev] = static_cast<unsigned*>(p);
  }
  return g_status_ptr[dev];
}

__global__ void take_status_kernel(unsigned* s) { s[1] = atomicExch(&s[0], 0u); }

// Launches one checked prediction request on `stream`.
stp_status launch_predict(stp_handle h, hipStream_t stream, int degree, int64_t n, double dt, const double* star,
                          const double* E, const double* Q0, double* Q, double* Qint, stp_precision precision,
                          int refine_steps, void* workspace, unsigned flags, int nq = STP_NQ) {
  if (n == 0) return STP_OK;
  stp::PredictArgs a{n, dt, star, E, Q0, Q, Qint, status_address(stream_device(stream))};
  hipError_t err;
  if (flags & STP_FLAG_REFERENCE_KERNEL)
    err = stp::launch_reference_kernel(degree, a, stream);
  else
    err = stp::launch_fused_kernel(nq, degree, a, static_cast<int>(precision), refine_steps,
                                   static_cast<float*>(workspace), (flags & STP_FLAG_MFMA_FLOAT_CHAIN) == 0,
                                   stream);
  if (err != hipSuccess) return hip_fail(h, err, "kernel launch");
  return STP_OK;
}

stp_status check_batches(stp_handle h, int n_batches, const stp_batch* batches, stp_precision precision,
                         int refine_steps, const void* workspace, size_t workspace_bytes, unsigned flags) {
  if (n_batches < 0) return fail(h, STP_EINVAL, "n_batches < 0");
  if (n_batches > 0 && !batches) return fail(h, STP_EINVAL, "NULL batches");
  for (int i = 0; i < n_batches; ++i) {
    const stp_batch& b = batches[i];
    const stp_status st = check_predict(h, b.degree, b.n_elements, b.dt, b.star, b.E, b.Q0, b.Q, precision,
                                        refine_steps, workspace, workspace_bytes, flags);
    if (st != STP_OK) return fail(h, st, "batch " + std::to_string(i) + ": " + h->last_error);
  }
  return STP_OK;
}

stp_status launch_batches(stp_handle h, hipStream_t stream, int n_batches, const stp_batch* batches,
                          stp_precision precision, int refine_steps, void* workspace, unsigned flags) {
  for (int i = 0; i < n_batches; ++i) {
    const stp_batch& b = batches[i];
    const stp_status st = launch_predict(h, stream, b.degree, b.n_elements, b.dt, b.star, b.E, b.Q0, b.Q, b.Qint,
                                         precision, refine_steps, workspace, flags);
    if (st != STP_OK) return fail(h, st, "batch " + std::to_string(i) + ": " + h->last_error);
  }
  return STP_OK;
}

// Device scratch of stp_predict_static: the mixed-precision path's residual
// buffer lives here instead of in a caller workspace.  In host code `scratch`
// names a host-side stand-in, never the device array: its device address is
// taken once per device with hipGetSymbolAddress (each device holds its own
// copy) and only that address is passed to kernels.
constexpr size_t kScratchBytes = size_t(256) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the device that runs `stream` (the NULL
// stream: the current device), which must be the current device.
stp_status scratch_address(stp_handle h, hipStream_t stream, void** out) {
  int cur = 0;
  hipError_t err = hipGetDevice(&cur);
  if (err != hipSuccess) return hip_fail(h, err, "hipGetDevice");
  if (stream) {
    hipDevice_t sdev = 0;
    err = hipStreamGetDevice(stream, &sdev);
    if (err != hipSuccess) return hip_fail(h, err, "hipStreamGetDevice");
    if (static_cast<int>(sdev) != cur)
      return fail(h, STP_EINVAL, "the stream belongs to device " + std::to_string(sdev) + " but device " +
                                     std::to_string(cur) + " is current");
  }
  if (cur < 0 || cur >= kMaxDevices) return fail(h, STP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[cur]) {
    void* p = nullptr;
    err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (err != hipSuccess) return hip_fail(h, err, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[cur] = p;
  }
  *out = g_scratch_ptr[cur];
  return STP_OK;
}

// Parallel branches of a staged graph: the batches of one stage go round
// robin to this many streams.
constexpr int kBranches = 4;

stp_status check_stages(stp_handle h, int n_stages, const int* stage_sizes) {
  if (n_stages < 0) return fail(h, STP_EINVAL, "n_stages < 0");
  if (n_stages > 0 && !stage_sizes) return fail(h, STP_EINVAL, "NULL stage_sizes");
  for (int s = 0; s < n_stages; ++s)
    if (stage_sizes[s] < 0) return fail(h, STP_EINVAL, "stage " + std::to_string(s) + " has a negative size");
  return STP_OK;
}

}  // namespace

extern "C" {

size_t stp_static_scratch_bytes(void) { return kScratchBytes; }

stp_status stp_predict_static(stp_handle handle, void* hip_stream, int degree, int64_t n_elements, double dt,
                              const double* star, const double* E, const double* Q0, double* Q, double* Qint,
                              stp_precision precision, int refine_steps, unsigned flags) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  const stp_status st = check_predict(handle, degree, n_elements, dt, star, E, Q0, Q, precision, refine_steps,
                                      nullptr, 0, flags, /*workspace_checked=*/false);
  if (st != STP_OK) return st;
  const size_t need = stp::workspace_bytes(STP_NQ, degree, n_elements, static_cast<int>(precision), refine_steps);
  if (need > kScratchBytes)
    return fail(handle, STP_EWORKSPACE,
                "stp_predict_static: " + std::to_string(need) + " bytes of scratch needed, at most " +
                    std::to_string(kScratchBytes) + " available (split the call)");
  void* ws = nullptr;
  if (need > 0) {
    const stp_status sa = scratch_address(handle, static_cast<hipStream_t>(hip_stream), &ws);
    if (sa != STP_OK) return sa;
  }
  return launch_predict(handle, static_cast<hipStream_t>(hip_stream), degree, n_elements, dt, star, E, Q0, Q, Qint,
                        precision, refine_steps, ws, flags);
}

stp_status stp_create(stp_handle* handle) {
  if (!handle) return STP_EINVAL;
  *handle = new (std::nothrow) stp_handle_s();
  if (!*handle) return STP_ENOMEM;
  // the current device's input-report address, outside any graph capture
  (void)status_address(stream_device(nullptr));
  return STP_OK;
}

stp_status stp_destroy(stp_handle handle) {
  if (!handle) return STP_EINVAL;
  delete handle;
  return STP_OK;
}

stp_status stp_workspace_size(stp_handle handle, int degree, int64_t n_elements,
                              stp_precision precision, int refine_steps, size_t* bytes) {
  if (!handle || !bytes) return STP_EINVAL;
  if (degree < 0 || degree > STP_MAX_DEGREE) return fail(handle, STP_EDEGREE, "degree out of range");
  if (n_elements < 0) return fail(handle, STP_EINVAL, "n_elements < 0");
  if (precision != STP_FP64 && precision != STP_FP32_REFINE) return fail(handle, STP_EINVAL, "precision");
  if (refine_steps < 0 || refine_steps > STP_MAX_REFINE) return fail(handle, STP_EINVAL, "refine_steps");
  *bytes = stp::workspace_bytes(STP_NQ, degree, n_elements, static_cast<int>(precision), refine_steps);
  return STP_OK;
}

stp_status stp_workspace_size_nq(stp_handle handle, int n_quantities, int degree, int64_t n_elements,
                                 stp_precision precision, int refine_steps, size_t* bytes) {
  if (!handle || !bytes) return STP_EINVAL;
  if (!stp::supported_nq(n_quantities)) return fail(handle, STP_EINVAL, "unsupported quantity count");
  const stp_status st = stp_workspace_size(handle, degree, n_elements, precision, refine_steps, bytes);
  if (st != STP_OK) return st;
  *bytes = stp::workspace_bytes(n_quantities, degree, n_elements, static_cast<int>(precision), refine_steps);
  return STP_OK;
}

stp_status stp_predict_nq(stp_handle handle, void* hip_stream, int n_quantities, int degree, int64_t n_elements,
                          double dt, const double* star, const double* E, const double* Q0, double* Q,
                          double* Qint, stp_precision precision, int refine_steps, void* workspace,
                          size_t workspace_bytes, unsigned flags) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  const stp_status st = check_predict(handle, degree, n_elements, dt, star, E, Q0, Q, precision, refine_steps,
                                      workspace, workspace_bytes, flags, true, n_quantities);
  if (st != STP_OK) return st;
  return launch_predict(handle, static_cast<hipStream_t>(hip_stream), degree, n_elements, dt, star, E, Q0, Q, Qint,
                        precision, refine_steps, workspace, flags, n_quantities);
}

stp_status stp_predict(stp_handle handle, void* hip_stream, int degree, int64_t n_elements, double dt,
                       const double* star, const double* E, const double* Q0, double* Q, double* Qint,
                       stp_precision precision, int refine_steps, void* workspace,
                       size_t workspace_bytes, unsigned flags) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  const stp_status st = check_predict(handle, degree, n_elements, dt, star, E, Q0, Q, precision, refine_steps,
                                      workspace, workspace_bytes, flags);
  if (st != STP_OK) return st;
  return launch_predict(handle, static_cast<hipStream_t>(hip_stream), degree, n_elements, dt, star, E, Q0, Q, Qint,
                        precision, refine_steps, workspace, flags);
}

stp_status stp_batched_workspace_size(stp_handle handle, int n_batches, const stp_batch* batches,
                                      stp_precision precision, int refine_steps, size_t* bytes) {
  if (!handle || !bytes) return STP_EINVAL;
  if (n_batches < 0 || (n_batches > 0 && !batches)) return fail(handle, STP_EINVAL, "batches");
  size_t need = 0;
  for (int i = 0; i < n_batches; ++i) {
    size_t b = 0;
    const stp_status st = stp_workspace_size(handle, batches[i].degree, batches[i].n_elements, precision,
                                             refine_steps, &b);
    if (st != STP_OK) return fail(handle, st, "batch " + std::to_string(i) + ": " + handle->last_error);
    need = b > need ? b : need;
  }
  *bytes = need;
  return STP_OK;
}

stp_status stp_predict_batched(stp_handle handle, void* hip_stream, int n_batches, const stp_batch* batches,
                               stp_precision precision, int refine_steps, void* workspace,
                               size_t workspace_bytes, unsigned flags) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  const stp_status st =
      check_batches(handle, n_batches, batches, precision, refine_steps, workspace, workspace_bytes, flags);
  if (st != STP_OK) return st;
  return launch_batches(handle, static_cast<hipStream_t>(hip_stream), n_batches, batches, precision,
                        refine_steps, workspace, flags);
}

stp_status stp_graph_create(stp_handle handle, void* hip_stream, int n_batches, const stp_batch* batches,
                            stp_precision precision, int refine_steps, void* workspace,
                            size_t workspace_bytes, unsigned flags, stp_graph* graph) {
  if (!handle || !graph) return STP_EINVAL;
  *graph = nullptr;
  handle->last_error.clear();
  if (!hip_stream) return fail(handle, STP_EINVAL, "graph capture needs a non-NULL stream");
  stp_status st =
      check_batches(handle, n_batches, batches, precision, refine_steps, workspace, workspace_bytes, flags);
  if (st != STP_OK) return st;
  stp_graph g = new (std::nothrow) stp_graph_s();
  if (!g) return fail(handle, STP_ENOMEM, "out of host memory");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  (void)status_address(stream_device(stream));  // taken before the capture
  hipError_t err = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (err != hipSuccess) {
    delete g;
    return hip_fail(handle, err, "hipStreamBeginCapture");
  }
  st = launch_batches(handle, stream, n_batches, batches, precision, refine_steps, workspace, flags);
  const std::string launch_error = handle->last_error;
  err = hipStreamEndCapture(stream, &g->graph);
  if (st == STP_OK && err != hipSuccess) st = hip_fail(handle, err, "hipStreamEndCapture");
  if (st == STP_OK) {
    err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (err != hipSuccess) st = hip_fail(handle, err, "hipGraphInstantiate");
  } else if (!launch_error.empty()) {
    handle->last_error = launch_error;
  }
  if (st != STP_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *graph = g;
  return STP_OK;
}

stp_status stp_staged_workspace_size(stp_handle handle, int n_stages, const int* stage_sizes,
                                     const stp_batch* batches, stp_precision precision, int refine_steps,
                                     size_t* bytes) {
  if (!handle || !bytes) return STP_EINVAL;
  const stp_status st = check_stages(handle, n_stages, stage_sizes);
  if (st != STP_OK) return st;
  size_t need = 0;
  int b0 = 0;
  for (int s = 0; s < n_stages; ++s) {
    size_t stage = 0;
    for (int i = b0; i < b0 + stage_sizes[s]; ++i) {
      size_t b = 0;
      const stp_status bs = stp_workspace_size(handle, batches[i].degree, batches[i].n_elements, precision,
                                               refine_steps, &b);
      if (bs != STP_OK) return fail(handle, bs, "batch " + std::to_string(i) + ": " + handle->last_error);
      stage += (b + 255) / 256 * 256;
    }
    need = stage > need ? stage : need;
    b0 += stage_sizes[s];
  }
  *bytes = need;
  return STP_OK;
}

stp_status stp_graph_create_staged(stp_handle handle, void* hip_stream, int n_stages, const int* stage_sizes,
                                   const stp_batch* batches, stp_precision precision, int refine_steps,
                                   void* workspace, size_t workspace_bytes, unsigned flags, stp_graph* graph) {
  if (!handle || !graph) return STP_EINVAL;
  *graph = nullptr;
  handle->last_error.clear();
  if (!hip_stream) return fail(handle, STP_EINVAL, "graph capture needs a non-NULL stream");
  stp_status st = check_stages(handle, n_stages, stage_sizes);
  if (st != STP_OK) return st;
  int n_batches = 0;
  for (int s = 0; s < n_stages; ++s) n_batches += stage_sizes[s];
  // every batch is checked against the whole workspace here; the per-stage
  // split is checked below
  st = check_batches(handle, n_batches, batches, precision, refine_steps, workspace, workspace_bytes, flags);
  if (st != STP_OK) return st;
  size_t need = 0;
  st = stp_staged_workspace_size(handle, n_stages, stage_sizes, batches, precision, refine_steps, &need);
  if (st != STP_OK) return st;
  if (need > 0 && (!workspace || workspace_bytes < need))
    return fail(handle, STP_EWORKSPACE, "staged workspace of " + std::to_string(need) + " bytes needed");
  stp_graph g = new (std::nothrow) stp_graph_s();
  if (!g) return fail(handle, STP_ENOMEM, "out of host memory");
  hipStream_t s0 = static_cast<hipStream_t>(hip_stream);
  // branch streams (default priority) and fork / join events, used only
  // while capturing
  hipStream_t br[kBranches] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kBranches] = {};
  hipError_t err = hipSuccess;
  for (int i = 0; i < kBranches && err == hipSuccess; ++i) err = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
  if (err == hipSuccess) err = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming);
  for (int i = 0; i < kBranches && err == hipSuccess; ++i) err = hipEventCreateWithFlags(&join_ev[i], hipEventDisableTiming);
  bool capturing = false;
  (void)status_address(stream_device(s0));  // taken before the capture
  if (err == hipSuccess) {
    err = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    capturing = err == hipSuccess;
  }
  int b0 = 0;
  for (int s = 0; s < n_stages && err == hipSuccess && st == STP_OK; ++s) {
    const int nb = stage_sizes[s];
    const int used = nb < kBranches ? nb : kBranches;
    err = hipEventRecord(fork_ev, s0);
    for (int k = 0; k < used && err == hipSuccess; ++k) err = hipStreamWaitEvent(br[k], fork_ev, 0);
    size_t off = 0;
    for (int i = 0; i < nb && err == hipSuccess && st == STP_OK; ++i) {
      const stp_batch& b = batches[b0 + i];
      size_t wb = 0;
      (void)stp_workspace_size(handle, b.degree, b.n_elements, precision, refine_steps, &wb);
      void* ws = wb ? static_cast<void*>(static_cast<char*>(workspace) + off) : nullptr;
      off += (wb + 255) / 256 * 256;
      st = launch_predict(handle, br[i % kBranches], b.degree, b.n_elements, b.dt, b.star, b.E, b.Q0, b.Q, b.Qint,
                          precision, refine_steps, ws, flags);
      if (st != STP_OK) handle->last_error = "batch " + std::to_string(b0 + i) + ": " + handle->last_error;
    }
    for (int k = 0; k < used && err == hipSuccess; ++k) {
      err = hipEventRecord(join_ev[k], br[k]);
      if (err == hipSuccess) err = hipStreamWaitEvent(s0, join_ev[k], 0);
    }
    b0 += nb;
  }
  const std::string launch_error = handle->last_error;
  if (capturing) {
    const hipError_t e2 = hipStreamEndCapture(s0, &g->graph);
    if (err == hipSuccess) err = e2;
  }
  if (st == STP_OK && err != hipSuccess) st = hip_fail(handle, err, "staged graph capture");
  if (st == STP_OK) {
    err = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (err != hipSuccess) st = hip_fail(handle, err, "hipGraphInstantiate");
  } else if (!launch_error.empty()) {
    handle->last_error = launch_error;
  }
  for (int i = 0; i < kBranches; ++i) {
    if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
    if (br[i]) (void)hipStreamDestroy(br[i]);
  }
  if (fork_ev) (void)hipEventDestroy(fork_ev);
  if (st != STP_OK) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *graph = g;
  return STP_OK;
}

stp_status stp_graph_launch(stp_graph graph, void* hip_stream) {
  if (!graph || !graph->exec) return STP_EINVAL;
  return hipGraphLaunch(graph->exec, static_cast<hipStream_t>(hip_stream)) == hipSuccess ? STP_OK : STP_EHIP;
}

stp_status stp_graph_destroy(stp_graph graph) {
  if (!graph) return STP_EINVAL;
  hipError_t e1 = graph->exec ? hipGraphExecDestroy(graph->exec) : hipSuccess;
  hipError_t e2 = graph->graph ? hipGraphDestroy(graph->graph) : hipSuccess;
  delete graph;
  return (e1 == hipSuccess && e2 == hipSuccess) ? STP_OK : STP_EHIP;
}

stp_status stp_validate_nq(stp_handle handle, void* hip_stream, int n_quantities, int degree, int64_t n_elements,
                           double dt, const double* star, const double* E, const double* Q0) {
  stp_status st = check_common(handle, degree, n_elements, dt);
  if (st == STP_OK && !stp::supported_nq(n_quantities))
    st = fail(handle, STP_EINVAL, "unsupported quantity count");
  if (st != STP_OK) return st;
  handle->last_error.clear();
  if (n_elements == 0) return STP_OK;
  if (!star || !E || !Q0) return fail(handle, STP_EINVAL, "NULL array pointer");
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  int* dflags = nullptr;
  hipError_t err = hipMalloc(&dflags, sizeof(int));
  if (err != hipSuccess) return hip_fail(handle, err, "hipMalloc");
  int hflags = 0;
  err = hipMemcpyAsync(dflags, &hflags, sizeof(int), hipMemcpyHostToDevice, stream);
  if (err == hipSuccess) {
    const int B = stp::n_modes(degree);
    hipLaunchKernelGGL(validate_kernel, dim3(1024), dim3(256), 0, stream, n_elements, n_quantities, B, dt, star,
                       E, Q0,
                       dflags);
    err = hipGetLastError();
  }
  if (err == hipSuccess) err = hipMemcpyAsync(&hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  hipError_t ferr = hipFree(dflags);
  if (err != hipSuccess) return hip_fail(handle, err, "validate");
  if (ferr != hipSuccess) return hip_fail(handle, ferr, "hipFree");
  if (hflags & kFlagNonFinite) return fail(handle, STP_ENONFINITE, "non-finite value in star, E or Q0");
  if (hflags & kFlagNotUpper) return fail(handle, STP_ENOTUPPER, "E has a non-zero below its diagonal");
  if (hflags & kFlagSingular) return fail(handle, STP_ESINGULAR, "dt * E_pp >= 0.5 for some quantity");
  return STP_OK;
}

stp_status stp_validate(stp_handle handle, void* hip_stream, int degree, int64_t n_elements, double dt,
                        const double* star, const double* E, const double* Q0) {
  return stp_validate_nq(handle, hip_stream, STP_NQ, degree, n_elements, dt, star, E, Q0);
}

stp_status stp_check_inputs(stp_handle handle, void* hip_stream) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  unsigned* ds = status_address(stream_device(stream));
  if (!ds) return fail(handle, STP_EHIP, "input report word of the stream's device unavailable");
  unsigned hs = 0;
  hipLaunchKernelGGL(take_status_kernel, dim3(1), dim3(1), 0, stream, ds);
  hipError_t err = hipGetLastError();
  if (err == hipSuccess) err = hipMemcpyAsync(&hs, ds + 1, sizeof(unsigned), hipMemcpyDeviceToHost, stream);
  if (err == hipSuccess) err = hipStreamSynchronize(stream);
  if (err != hipSuccess) return hip_fail(handle, err, "check_inputs");
  if (hs & stp::kInputNotUpper)
    return fail(handle, STP_ENOTUPPER, "a predict call met an E with a non-zero below its diagonal");
  if (hs & stp::kInputSingular) return fail(handle, STP_ESINGULAR, "a predict call met dt * E_pp >= 0.5");
  return STP_OK;
}

stp_status stp_reference_matrices(stp_handle handle, int degree, double* Z, double* Sinv_w, double* Khat) {
  if (!handle) return STP_EINVAL;
  if (degree < 0 || degree > STP_MAX_DEGREE) return fail(handle, STP_EDEGREE, "degree out of range");
  try {
    const stp_host::ReferenceMatrices R = stp_host::build_reference_matrices(degree);
    if (Z) std::memcpy(Z, R.Z.data(), R.Z.size() * sizeof(double));
    if (Sinv_w) std::memcpy(Sinv_w, R.Sinv_w.data(), R.Sinv_w.size() * sizeof(double));
    if (Khat) std::memcpy(Khat, R.Khat.data(), R.Khat.size() * sizeof(double));
  } catch (const std::bad_alloc&) {
    return fail(handle, STP_ENOMEM, "out of host memory");
  } catch (...) {
    return fail(handle, STP_EINVAL, "reference matrices");
  }
  return STP_OK;
}

stp_status stp_flops(int degree, double* paper_bound, double* executed) {
  if (degree < 0 || degree > STP_MAX_DEGREE) return STP_EDEGREE;
  const double N = degree, B = stp::n_modes(degree), T = N + 1, Qn = 13;
  if (paper_bound) {
    // upper bound of Algorithm 3 (section "Block-wise back-substitution")
    *paper_bound = 2 * B * (Qn * T * T + 3 * T + 3 * T * Qn * Qn + 3 * T * Qn * B) + 3 * Qn * B * T * T;
  }
  if (executed) {
    // the fused float64 kernel: right-hand side init, dark-blue solves,
    // three G couplings of the poroelastic E, dense star products of every
    // mode above degree 0, non-zero Khat entries.
    const stp_host::ReferenceMatrices R = stp_host::build_reference_matrices(degree);
    double nnz = 0;
    for (int d = 0; d < 3; ++d)
      for (int g = 1; g <= degree; ++g)
        for (int n = 0; n < stp::block_start(g); ++n)
          for (int l = stp::block_start(g); l < stp::block_start(g) + stp::block_size(g); ++l)
            nnz += (R.Khat[(static_cast<size_t>(d) * R.B + n) * R.B + l] != 0.0);
    *executed = Qn * B * T + 2 * Qn * T * T * B + 3 * 2 * T * B + 2 * 3 * Qn * Qn * T * (B - 1) +
                2 * Qn * T * nnz;
  }
  return STP_OK;
}

// ---- corrector ---------------------------------------------------------------

stp_status stp_basis_eval(int degree, int64_t n_points, const double* xi, double* phi) {
  if (degree < 0 || degree > STP_MAX_DEGREE) return STP_EDEGREE;
  if (n_points < 0 || (n_points > 0 && (!xi || !phi))) return STP_EINVAL;
  const int B = stp::n_modes(degree);
  for (int64_t i = 0; i < n_points; ++i)
    stp_host::eval_dubiner(degree, xi[3 * i], xi[3 * i + 1], xi[3 * i + 2], phi + i * B);
  return STP_OK;
}

stp_status stp_reference_mass(int degree, double* M) {
  if (degree < 0 || degree > STP_MAX_DEGREE) return STP_EDEGREE;
  if (!M) return STP_EINVAL;
  try {
    const stp_host::ReferenceMatrices R = stp_host::build_reference_matrices(degree);
    std::memcpy(M, R.M.data(), R.M.size() * sizeof(double));
  } catch (...) {
    return STP_ENOMEM;
  }
  return STP_OK;
}

size_t stp_corrector_tables_size(int degree) {
  if (degree < 0 || degree > STP_MAX_DEGREE) return 0;
  const size_t B = stp::n_modes(degree);
  return (3 + 4 + 96) * B * B;
}

stp_status stp_corrector_tables(int degree, double* tables) {
  if (degree < 0 || degree > STP_MAX_DEGREE) return STP_EDEGREE;
  if (!tables) return STP_EINVAL;
  try {
    const stp_host::CorrectorTables C = stp_host::build_corrector_tables(degree);
    double* p = tables;
    for (const std::vector<double>* v : {&C.V, &C.Fl, &C.Fn}) {
      std::memcpy(p, v->data(), v->size() * sizeof(double));
      p += v->size();
    }
  } catch (...) {
    return STP_ENOMEM;
  }
  return STP_OK;
}

stp_status stp_upwind_split(int n_quantities, const double* An, double* Aplus, double* Aminus) {
  if (n_quantities <= 0 || !An || !Aplus || !Aminus) return STP_EINVAL;
  std::string err;
  return stp_host::upwind_split(n_quantities, An, Aplus, Aminus, &err) ? STP_OK : STP_ESINGULAR;
}

stp_status stp_face_operators(stp_handle handle, int n_quantities, int64_t n_elements, const double* ABC,
                              const double* vertices, double* Gp, double* Gm) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  if (n_quantities <= 0 || n_elements < 0) return fail(handle, STP_EINVAL, "bad sizes");
  if (n_elements == 0) return STP_OK;
  if (!ABC || !vertices || !Gp || !Gm) return fail(handle, STP_EINVAL, "NULL array pointer");
  std::string err;
  if (!stp_host::face_operators(n_quantities, n_elements, ABC, vertices, Gp, Gm, &err))
    return fail(handle, STP_ESINGULAR, err);
  return STP_OK;
}

stp_status stp_correct(stp_handle handle, void* hip_stream, int n_quantities, int degree, int64_t n_elements,
                       const double* tables, const double* star, const double* E, const double* Gp,
                       const double* Gm, const int32_t* neighbor, const int32_t* nb_code, const double* Qint,
                       double* Q) {
  if (!handle) return STP_EINVAL;
  handle->last_error.clear();
  if (degree < 0 || degree > STP_MAX_DEGREE) return fail(handle, STP_EDEGREE, "degree out of range");
  if (n_quantities <= 0 || n_elements < 0) return fail(handle, STP_EINVAL, "bad sizes");
  if (n_elements == 0) return STP_OK;
  if (!tables || !star || !E || !Gp || !Gm || !neighbor || !nb_code || !Qint || !Q)
    return fail(handle, STP_EINVAL, "NULL array pointer");
  const int B = stp::n_modes(degree);
  if (!stp::corrector_fits(n_quantities, B))
    return fail(handle, STP_EINVAL, "corrector: kernels for 13 or 6 quantities only, got " +
                                        std::to_string(n_quantities));
  stp::CorrectArgs a{n_elements, n_quantities, B, tables, star, E, Gp, Gm, neighbor, nb_code, Qint, Q};
  const hipError_t err = stp::launch_corrector(a, static_cast<hipStream_t>(hip_stream));
  if (err != hipSuccess) return hip_fail(handle, err, "corrector launch");
  return STP_OK;
}

const char* stp_status_string(stp_status status) {
  switch (status) {
    case STP_OK: return "STP_OK";
    case STP_EINVAL: return "STP_EINVAL: invalid argument";
    case STP_EDEGREE: return "STP_EDEGREE: degree out of range";
    case STP_ENOTUPPER: return "STP_ENOTUPPER: E is not upper triangular";
    case STP_ESINGULAR: return "STP_ESINGULAR: diagonal block not safely invertible";
    case STP_ENOMEM: return "STP_ENOMEM: out of memory";
    case STP_EHIP: return "STP_EHIP: HIP runtime error";
    case STP_EWORKSPACE: return "STP_EWORKSPACE: workspace too small";
    case STP_ENONFINITE: return "STP_ENONFINITE: non-finite input";
  }
  return "unknown status";
}

const char* stp_last_error(stp_handle handle) { return handle ? handle->last_error.c_str() : ""; }

}  // extern "C"
