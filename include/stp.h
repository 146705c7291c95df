/*
 * stp.h -- C ABI of the element-local space-time predictor of ADER-DG for
 * Biot poroelasticity, solved by block-wise back-substitution over the
 * spatial-degree blocks (Wolf et al., "An Efficient ADER-DG Local Time
 * Stepping Scheme for 3D HPC Simulation of Seismic Waves in Poroelastic
 * Media", arXiv 2108.10565).  Kernels are written for AMD MI355X (gfx950).
 *
 * What one call computes, per element (section "Space-Time predictor",
 * eq:stp-lineq / eq:linear_system, solved as in section "Block-wise
 * back-substitution", Algorithm 3):
 *
 *   ( d_pq W_rs M_kl - d_pq K^tau_rs M_kl - E*_pq S_rs M_kl
 *     + sum_j A^{j*}_pq S_rs K^j_kl ) Q_qls = d_pq w_r M_kl Q0_ql,
 *   A^{j*} = dt A^j,  E* = dt E,
 *
 * and the time-integrated DOFs Qint_pl = dt * sum_s Q_pls int_0^1 chi_s
 * = dt * Q_pl0.
 *
 * Conventions (part of the ABI):
 *  - quantities p = 0..12 in the order (sxx, syy, szz, sxy, syz, sxz,
 *    u, v, w, p, uf, vf, wf) of section "Governing equations";
 *  - temporal basis chi_s(tau) = P_s(2 tau - 1), s = 0..N (Legendre,
 *    unnormalised, chi_s(1) = 1) on the reference interval [0, 1];
 *  - spatial basis: Dubiner polynomials on the reference tetrahedron
 *    {x, y, z > 0, x + y + z < 1},
 *      phi_ijk = P_i(a)(1-y-z)^i P_j^(2i+1,0)(b)(1-z)^j P_k^(2i+2j+2,0)(c),
 *      a = 2x/(1-y-z) - 1, b = 2y/(1-z) - 1, c = 2z - 1,
 *    unnormalised, ordered by total degree n = i+j+k, then k = 0..n, then
 *    j = 0..n-k;  B = (N+1)(N+2)(N+3)/6 modes, T = N+1 time modes;
 *  - all arrays are C-contiguous (row-major), float64.
 *
 * Ownership: the caller owns every input, output and workspace buffer.
 * The library owns only the handle (host memory).  stp_predict allocates
 * nothing, never synchronises the stream and launches on the stream given.
 *
 * Errors: every entry point returns a stp_status and never aborts.  Cheap
 * argument checks are done on the host before any launch; checks that need
 * the data are in stp_validate (opt-in, synchronises), and the prediction
 * kernels report the inputs their elimination cannot take to a per-device
 * word that stp_check_inputs reads.  A HIP launch
 * failure is reported as STP_EHIP with the HIP message in stp_last_error.
 * A handle must not be used from two host threads at once.
 */
#ifndef STP_H
#define STP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define STP_NQ 13          /* quantities of the poroelastic system        */
#define STP_MAX_DEGREE 7   /* supported polynomial degrees N = 0..7       */
#define STP_MAX_REFINE 3   /* refinement steps of the mixed-precision path */

typedef struct stp_handle_s* stp_handle;

typedef enum stp_status {
  STP_OK = 0,
  STP_EINVAL = -1,      /* bad argument: NULL pointer with n > 0, n < 0,
                           dt <= 0 or not finite, bad enum or flags       */
  STP_EDEGREE = -2,     /* degree outside 0..STP_MAX_DEGREE               */
  STP_ENOTUPPER = -3,   /* (stp_validate, stp_check_inputs) an E has a
                           non-zero strictly below its diagonal           */
  STP_ESINGULAR = -4,   /* (stp_validate, stp_check_inputs) Z - dt E_pp I
                           is singular or dt E_pp > 0 makes it nearly so  */
  STP_ENOMEM = -5,      /* host allocation failed                         */
  STP_EHIP = -6,        /* HIP runtime error (see stp_last_error)         */
  STP_EWORKSPACE = -7,  /* workspace smaller than stp_workspace_size      */
  STP_ENONFINITE = -8   /* (stp_validate) NaN or Inf in an input          */
} stp_status;

typedef enum stp_precision {
  /* Algorithm 3 entirely in float64. */
  STP_FP64 = 0,
  /* Algorithm 3 in float32 with float32 accumulation (the star x stiffness
   * x time chain), stiff diagonal-block inverses kept in float64, then
   * refine_steps rounds of iterative refinement: float64 matrix-free
   * residual of the full element system, correction by the float32 chain,
   * float64 update.  Outputs are float64. */
  STP_FP32_REFINE = 1
} stp_precision;

/* flags of stp_predict */
#define STP_FLAG_NONE 0u
/* Use the one-element-per-workgroup LDS kernel (float64 only) instead of
 * the fused register-resident kernel.  Same results up to rounding; kept
 * as an independent GPU implementation and for debugging. */
#define STP_FLAG_REFERENCE_KERNEL 1u
/* STP_FP32_REFINE only: run the float32 chain's green-block update (the
 * star x stiffness x time products, Algorithm 3) on the matrix cores,
 * v_mfma_f32_16x16x4f32 with float32 accumulation, instead of as sparse
 * fused multiply-adds on the vector ALU.  Same results up to float32
 * rounding.  The dense 16 x 16 x 4 tiles execute ~3x the non-zero products
 * of the sparse update at twice the vector rate, so on MI355X this variant
 * is slower; it is kept selectable for comparison. */
#define STP_FLAG_MFMA_FLOAT_CHAIN 2u

/* Create / destroy a handle.  No device work is done by either. */
stp_status stp_create(stp_handle* handle);
stp_status stp_destroy(stp_handle handle);

/* Bytes of device workspace stp_predict needs for these arguments: 0 for
 * STP_FP64 (all intermediates live in registers, LDS or the output Q); for
 * STP_FP32_REFINE with refine_steps > 0, the float residual of every element
 * (n * 13 * B * T * 4 bytes, rounded up to 256). */
stp_status stp_workspace_size(stp_handle handle, int degree, int64_t n_elements,
                              stp_precision precision, int refine_steps,
                              size_t* bytes);

/* Predict n_elements independent elements on `hip_stream` (a hipStream_t,
 * NULL = default stream).  All array pointers are DEVICE pointers, 16-byte
 * aligned, float64, C-contiguous:
 *   star [n][3][13][13]  reference-element Jacobians A^1, A^2, A^3
 *                        (A^j = A dxi_j/dx + B dxi_j/dy + C dxi_j/dz,
 *                        subsection "Spatial discretisation"), NOT scaled
 *                        by dt;
 *   E    [n][13][13]     source matrix, upper triangular (section
 *                        "Governing equations"), NOT scaled by dt;
 *                        entries below the diagonal are never read;
 *   Q0   [n][13][B]      spatial DOFs at the start of the step;
 *   Q    [n][13][B][T]   out: space-time DOFs;
 *   Qint [n][13][B]      out: dt * time average over the step; may be NULL.
 * dt > 0 and finite (one time step for every element of the call).
 * refine_steps in 0..STP_MAX_REFINE (ignored for STP_FP64).
 * workspace: device buffer of at least stp_workspace_size bytes (may be NULL
 * when that size is 0), owned by the caller, contents ignored and clobbered;
 * too small -> STP_EWORKSPACE.
 * n_elements == 0 is a no-op returning STP_OK. */
stp_status stp_predict(stp_handle handle, void* hip_stream, int degree,
                       int64_t n_elements, double dt, const double* star,
                       const double* E, const double* Q0, double* Q,
                       double* Qint, stp_precision precision,
                       int refine_steps, void* workspace,
                       size_t workspace_bytes, unsigned flags);

/* Data checks (synchronises `hip_stream`): non-finite input -> STP_ENONFINITE,
 * a non-zero below the diagonal of some E -> STP_ENOTUPPER, dt E_pp >= 0.5
 * (the diagonal-block matrices Z - dt E_pp I are then not guaranteed
 * invertible by the kernels' elimination without pivoting) ->
 * STP_ESINGULAR.  Returns STP_OK when the inputs are fit for stp_predict. */
stp_status stp_validate(stp_handle handle, void* hip_stream, int degree,
                        int64_t n_elements, double dt, const double* star,
                        const double* E, const double* Q0);

/* Input report of the prediction kernels (section "Block-wise
 * back-substitution": the dark-blue blocks Z - dt E_pp I are inverted
 * without pivoting, which the kernels admit for dt E_pp < 0.5, and the G
 * coupling takes E as upper triangular).  The predict calls return before
 * their kernels run, so they cannot fail on such data; instead every
 * prediction kernel (stp_predict, stp_predict_nq, stp_predict_static,
 * stp_predict_batched, graph replays; every precision and the reference
 * kernel) ORs what it meets into a word held per device.  This call takes
 * and clears that word of the device running `hip_stream` (atomically, in a
 * one-thread kernel on that stream), synchronises the stream, and returns
 * STP_ENOTUPPER (some E had a non-zero strictly below its diagonal; the
 * kernels used only its upper part), else STP_ESINGULAR (some dt E_pp was
 * >= 0.5; those outputs are not to be trusted), else STP_OK.  The word
 * collects the calls of every stream and handle on the device since it was
 * last taken; calls that are still running when it is taken report to the
 * next call.  Not for use under graph capture. */
stp_status stp_check_inputs(stp_handle handle, void* hip_stream);

/* Reference matrices the kernels use for degree N, computed on the host by
 * Gauss quadrature in collapsed coordinates (HOST pointers, for tests):
 *   Z      [T][T]     S^-1 (W - K^tau)  (section "Block-wise back-substitution")
 *   Sinv_w [T]        S^-1 w
 *   Khat   [3][B][B]  M^-1 K^alpha, alpha = xi, eta, zeta
 * Any pointer may be NULL to skip it. */
stp_status stp_reference_matrices(stp_handle handle, int degree, double* Z,
                                  double* Sinv_w, double* Khat);

/* FLOP counts per element: the paper's upper bound of Algorithm 3 (Table
 * "tab:flop-count"), and the count this library executes in its fused
 * float64 kernel (useful FLOP: dense star matrices, non-zero Khat entries). */
stp_status stp_flops(int degree, double* paper_bound, double* executed);

/* ---- Other systems with a stiff upper-triangular source -------------------
 *
 * Algorithm 3 needs only that E is upper triangular; the Jacobians are data
 * (section "Other applications").  These entry points take the quantity
 * count nq of the system; the kernels are compiled for nq = STP_NQ (13, the
 * poroelastic system) and nq = STP_NQ_MAXWELL (6: the damped Maxwell
 * equations, quantities (Ex, Ey, Ez, Hx, Hy, Hz), source -sigma/eps on the
 * electric field); any other nq returns STP_EINVAL.  Arrays as for
 * stp_predict with 13 replaced by nq: star [n][3][nq][nq], E [n][nq][nq],
 * Q0 [n][nq][B], Q [n][nq][B][T], Qint [n][nq][B].  With nq = 13 these are
 * exactly stp_workspace_size / stp_predict / stp_validate.  The reference
 * kernel (STP_FLAG_REFERENCE_KERNEL) is for nq = 13 only. */
#define STP_NQ_MAXWELL 6
stp_status stp_workspace_size_nq(stp_handle handle, int n_quantities, int degree,
                                 int64_t n_elements, stp_precision precision,
                                 int refine_steps, size_t* bytes);
stp_status stp_predict_nq(stp_handle handle, void* hip_stream, int n_quantities,
                          int degree, int64_t n_elements, double dt,
                          const double* star, const double* E, const double* Q0,
                          double* Q, double* Qint, stp_precision precision,
                          int refine_steps, void* workspace, size_t workspace_bytes,
                          unsigned flags);
stp_status stp_validate_nq(stp_handle handle, void* hip_stream, int n_quantities,
                           int degree, int64_t n_elements, double dt,
                           const double* star, const double* E, const double* Q0);

/* ---- Corrector: one ADER-DG step with the predictor ------------------------
 *
 * Section "ADER-DG discretisation": the semi-discrete system eq:semi_discrete
 * (volume term after integration by parts, Godunov flux across the four
 * faces, source term) integrated over one time step with the predictor's
 * time-integrated DOFs Qint in place of the solution:
 *
 *   Q <- Q + sum_j A^j Qint V^j + E Qint
 *          - sum_f ( Gp_f Qint Fl_f + Gm_f Qint_nb(f) Fn_{f, j(f), h(f)} )
 *
 * with A^j the star matrices and E the source (both NOT dt-scaled; Qint
 * already integrates over the step).  Reference tables (divided by the mass
 * M_kk of the test function k; face integrals over the face's parameter
 * triangle {s, t >= 0, s + t <= 1}, faces of the reference tetrahedron with
 * local vertex triples (0,2,1), (0,1,3), (0,3,2), (1,2,3)):
 *   V^j_lk = int phi_l d_j phi_k / M_kk,  Fl_f,lk = int phi_l phi_k / M_kk,
 *   Fn_{f,j,h},lk = int phi_l(neighbour face j, correspondence h) phi_k / M_kk,
 * where correspondence h means own-face vertex r is neighbour-face vertex
 * perm_h[r], perm = {012, 021, 102, 120, 201, 210}.
 * Per face: Gp_f = (2 |S_f| / |J|) An^+, Gm_f = (2 |S_f| / |J|) An^-, the
 * Godunov split of An = nu_x A + nu_y B + nu_z C (outward unit normal nu,
 * physical Jacobians of the element; the flux assumes the same material on
 * both sides of a face).  The corrector does not synchronise or allocate. */

/* Basis of degree N at n_points reference points xi [n][3] -> phi [n][B]
 * (HOST pointers). */
stp_status stp_basis_eval(int degree, int64_t n_points, const double* xi, double* phi);
/* Diagonal of the reference mass matrix, M [B] (HOST). */
stp_status stp_reference_mass(int degree, double* M);
/* Number of doubles of the corrector tables of degree N: (3 + 4 + 96) B^2
 * (0 for a bad degree), and the tables themselves, V, Fl, Fn concatenated
 * (HOST pointer; the caller copies them to the device for stp_correct). */
size_t stp_corrector_tables_size(int degree);
stp_status stp_corrector_tables(int degree, double* tables);
/* Godunov split of one normal Jacobian An [nq][nq] (real spectrum,
 * diagonalisable): Aplus = R max(Lambda,0) R^-1, Aminus = An - Aplus (HOST).
 * STP_ESINGULAR if the spectrum is not real or the split is inaccurate. */
stp_status stp_upwind_split(int n_quantities, const double* An, double* Aplus, double* Aminus);
/* Gp, Gm [n][4][nq][nq] of a mesh (HOST): ABC [n][3][nq][nq] physical
 * Jacobians of every element, vertices [n][4][3] its corners (local vertex
 * order of the reference tetrahedron). */
stp_status stp_face_operators(stp_handle handle, int n_quantities, int64_t n_elements,
                              const double* ABC, const double* vertices, double* Gp, double* Gm);
/* One corrector step on `hip_stream` (DEVICE pointers): tables as returned
 * by stp_corrector_tables; star [n][3][nq][nq]; E [n][nq][nq]; Gp, Gm
 * [n][4][nq][nq]; neighbor [n][4] (int32, the element behind each face);
 * nb_code [n][4] (int32, 6 j + h); Qint [n][nq][B]; Q [n][nq][B] in/out.
 * Every neighbor entry must lie in 0..n-1 and every nb_code in 0..23 (they
 * index device arrays and are not checked).  Q must not alias Qint.
 * STP_EINVAL for a quantity count other than 13 or 6 (the kernels are
 * compiled per quantity count and degree). */
stp_status stp_correct(stp_handle handle, void* hip_stream, int n_quantities, int degree,
                       int64_t n_elements, const double* tables, const double* star,
                       const double* E, const double* Gp, const double* Gm,
                       const int32_t* neighbor, const int32_t* nb_code, const double* Qint,
                       double* Q);

/* ---- Prediction without a caller workspace --------------------------------
 *
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments (minus the workspace), kernels and results as stp_predict; the
 * mixed-precision path's residual buffer is a device array inside the
 * library instead, of stp_static_scratch_bytes() bytes (256 MiB) per device,
 * which each device holds from the first call on it until the process ends.
 * The call allocates nothing and does not synchronise.
 *  - A call whose stp_workspace_size exceeds the array returns
 *    STP_EWORKSPACE before launching anything (at N=6 with refinement: up to
 *    8,779 elements per call; split larger batches).  STP_FP64 and
 *    refine_steps == 0 need no scratch and have no size limit.
 *  - hip_stream must belong to the current device (STP_EINVAL otherwise).
 *  - Every call on a device shares that device's array, and no call relies
 *    on what an earlier one left in it.  Calls that overlap in time on one
 *    device (two streams, or two host threads) race on it and give wrong
 *    results; calls ordered on one stream do not. */
size_t stp_static_scratch_bytes(void);
stp_status stp_predict_static(stp_handle handle, void* hip_stream, int degree,
                              int64_t n_elements, double dt, const double* star,
                              const double* E, const double* Q0, double* Q,
                              double* Qint, stp_precision precision,
                              int refine_steps, unsigned flags);

/* ---- Several batches in one call, and a replayable graph of them ---------
 *
 * Clustered local time stepping (subsection "Temporal discretisation with
 * ADER"; its gain is measured in subsection "Scaling") updates elements that
 * need a smaller time step more often: with clusters of time steps
 * dt_k = r^k dt_0 (rate r), one cycle of the largest step predicts cluster k
 * r^(K-1-k) times.  A batch is one group of elements sharing one degree and
 * one time step (one cluster of one degree); a cycle is a list of batches,
 * a batch possibly repeated.  Arrays of a batch have the layout of
 * stp_predict. */
typedef struct stp_batch {
  int degree;            /* 0..STP_MAX_DEGREE                                  */
  int64_t n_elements;    /* >= 0                                               */
  double dt;             /* > 0 and finite                                     */
  const double* star;    /* [n][3][13][13] device                              */
  const double* E;       /* [n][13][13]    device                              */
  const double* Q0;      /* [n][13][B]     device                              */
  double* Q;             /* [n][13][B][T]  device, out                         */
  double* Qint;          /* [n][13][B]     device, out, may be NULL            */
} stp_batch;

/* Workspace for stp_predict_batched / stp_graph_create: the largest
 * stp_workspace_size of any batch (the batches run one after the other on
 * one stream and reuse it). */
stp_status stp_batched_workspace_size(stp_handle handle, int n_batches, const stp_batch* batches,
                                      stp_precision precision, int refine_steps, size_t* bytes);

/* Predicts batches[0..n_batches-1] in order on `hip_stream`, each exactly as
 * stp_predict would (same kernels, bitwise the same results).  Every batch is
 * checked before anything is launched: a bad batch returns its error, with
 * its index in stp_last_error, and launches nothing.  n_batches == 0 is a
 * no-op.  Allocates nothing; does not synchronise. */
stp_status stp_predict_batched(stp_handle handle, void* hip_stream, int n_batches, const stp_batch* batches,
                               stp_precision precision, int refine_steps, void* workspace,
                               size_t workspace_bytes, unsigned flags);

/* A HIP graph holding the launches of one stp_predict_batched call, captured
 * on `hip_stream` (which must not be the NULL stream; nothing runs during
 * capture).  The graph keeps the device pointers, sizes and time steps of
 * the batches as they were at capture: replaying it predicts from whatever
 * the input arrays then hold.  The graph owns host-side HIP objects only;
 * the caller keeps every array and the workspace alive while it may run.
 * No memset or allocation is recorded in it.  Destroy with
 * stp_graph_destroy (after its last launch has completed). */
typedef struct stp_graph_s* stp_graph;
stp_status stp_graph_create(stp_handle handle, void* hip_stream, int n_batches, const stp_batch* batches,
                            stp_precision precision, int refine_steps, void* workspace,
                            size_t workspace_bytes, unsigned flags, stp_graph* graph);
/* Launches the graph on `hip_stream` (any stream, NULL included); does not
 * synchronise. */
stp_status stp_graph_launch(stp_graph graph, void* hip_stream);
stp_status stp_graph_destroy(stp_graph graph);

/* Concurrent batches.  In a cycle of clustered local time stepping the
 * batches predicted at one sub-step (one per cluster due and degree) are
 * independent of each other.  batches[0 .. sum(stage_sizes)) are split into
 * n_stages consecutive stages of stage_sizes[s] batches: the batches of one
 * stage must write distinct outputs (inputs may be shared) and are captured
 * on parallel graph branches (up to 4 streams of default priority, batches
 * assigned round robin); each stage starts after the previous one has
 * completed.  Concurrent STP_FP32_REFINE batches need their own residual
 * buffers: the workspace is the largest sum over one stage of the batches'
 * stp_workspace_size (each rounded up to 256 bytes), as
 * stp_staged_workspace_size returns.  Otherwise as stp_graph_create; the
 * graph is launched and destroyed with stp_graph_launch / stp_graph_destroy. */
stp_status stp_staged_workspace_size(stp_handle handle, int n_stages, const int* stage_sizes,
                                     const stp_batch* batches, stp_precision precision,
                                     int refine_steps, size_t* bytes);
stp_status stp_graph_create_staged(stp_handle handle, void* hip_stream, int n_stages,
                                   const int* stage_sizes, const stp_batch* batches,
                                   stp_precision precision, int refine_steps, void* workspace,
                                   size_t workspace_bytes, unsigned flags, stp_graph* graph);

/* ---- Machine ceilings ----------------------------------------------------
 *
 * The roofline of subsection "Roofline model" places the predictor against
 * the peak FLOP/s and memory bandwidth measured on the machine itself.  This
 * call measures the corresponding ceilings of the GPU: FMA loops on the
 * vector ALUs (float64, and float32 without packed math, as the kernels are
 * built) and on the float64 matrix cores, a device-to-device copy and a
 * write-only stream through HBM.  Each kernel is warmed up, then timed with
 * HIP events on `hip_stream`; the call synchronises that stream.
 * `scratch` (device, owned by the caller, contents clobbered) holds the
 * streams: at least 1 GiB (the two halves are copied into each other) is
 * needed for a bandwidth reading that caches do not inflate; a smaller buffer
 * returns STP_EWORKSPACE. */
typedef struct stp_peaks {
  double fp64_valu_tflops;   /* v_fma_f64 over all compute units            */
  double fp32_valu_tflops;   /* v_fma_f32 (no packed float32 instructions)  */
  double fp64_mfma_tflops;   /* 16x16x4 float64 matrix-core instructions    */
  double hbm_copy_gbs;       /* bytes read + bytes written per second (best of grid sizes and access kinds) */
  double hbm_write_gbs;      /* bytes written per second (same)             */
} stp_peaks;

stp_status stp_measure_peaks(stp_handle handle, void* hip_stream, void* scratch, size_t scratch_bytes,
                             stp_peaks* peaks);

const char* stp_status_string(stp_status status);
/* Human-readable detail of the last failure on this handle ("" if none). */
const char* stp_last_error(stp_handle handle);

#ifdef __cplusplus
}
#endif

#endif /* STP_H */
