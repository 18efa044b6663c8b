/*
 * toprop — batched free-space propagation of sampled optical fields on
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow the TorchOptics paper (Filipovich & Lvovsky,
 * arXiv 2411.18591):
 *   - modulation by an element, Eq. (field_modulation): u_out = M u_in, and
 *     its Jones-matrix form for polarized fields (section "Polarization");
 *   - propagation by the angular-spectrum method, Eq. (field_propagation_tf)
 *     with the transfer function of Eq. (transfer_function), on a zero-padded
 *     grid ("configurable zero-padding"), or by the Fresnel transfer
 *     function (the paraxial alternative the same section mentions), or by
 *     direct integration (DI) of Eq. (field_propagation) with the impulse
 *     response of Eq. (impulse_response), and the automatic choice between
 *     AS and DI by the critical distance of Eq. (sampling_condition);
 *   - gradients of both for gradient-based optimization (section
 *     "Gradient-based optimization");
 *   - propagation of a mutual coherence function (section "Spatial
 *     coherence").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every array argument is DEVICE memory owned by the caller; the
 *   library reads or writes it only during the call's stream work and keeps
 *   no reference afterwards.  The library owns its workspace (scratch FFT
 *   buffers, twiddle tables, reduction partials), allocated on first use per
 *   device and grown as needed; to_release() frees it.
 * Layout.  Complex arrays are interleaved (re, im) — complex64 (float2) for
 *   TO_C64, complex128 (double2) for TO_C128 — row-major [field][comp][ny][nx]
 *   with x fastest.  Real arrays (phase masks, targets, weights, gradients)
 *   are float for TO_C64 and double for TO_C128, [ny][nx].
 * Grid.  Sample (y, x) sits at ((y - ny/2) dy + y0, (x - nx/2) dx + x0)
 *   (integer division), i.e. sample ny/2 is on the optical axis when the
 *   offset is zero.
 * Padding.  Propagation zero-pads the ny x nx field to the py x px grid of
 *   the job; the field may be ragged (e.g. 1000 x 1000 padded to 2048 x
 *   2048).  Padded extents are powers of two in [8, 8192] (the fused
 *   kernels) or other lengths in [3, 4096] (e.g. 2000: an unfused pipeline
 *   whose lines are transformed by a mixed-radix FFT when the length is
 *   2^a 3^b 5^c 7^d, else by Bluestein's method, chosen automatically,
 *   with a stream synchronization on the first use of each such length;
 *   coherence propagation on such grids runs its batched propagations one
 *   field at a time through that pipeline).  The operator is the circular
 *   convolution on the padded grid restricted to the field window, so the
 *   window position inside the padded grid does not change the result.
 * Transfer function (cycles, lambda = wavelength):
 *   TO_ASM:     H = exp(2 pi i z sqrt(1/lambda^2 - fx^2 - fy^2)),
 *               H = 0 where fx^2 + fy^2 > 1/lambda^2 (evanescent cut-off);
 *   TO_FRESNEL: H = exp(2 pi i (z/lambda - lambda z (fx^2 + fy^2) / 2)),
 *   with fx = k / (px dx), fy = k / (py dy) in FFT order (bins with
 *   2 k >= px are negative: k - px);
 *   TO_DI:      H = DFT of h(sy dy, sx dx) dx dy on the padded grid, h the
 *               impulse response of Eq. (impulse_response),
 *                 h = z / (i lambda d) (1 + i / (k d)) exp(i k d) / d,
 *                 d = sqrt(ox^2 + oy^2 + z^2), k = 2 pi / lambda,
 *               sampled at the signed circular offsets sy (= ky for
 *               ky < py/2, ky - py otherwise; likewise sx) with |sy| < ny and
 *               |sx| < nx, zero elsewhere.  The propagation is then the
 *               discrete Riemann sum of Eq. (field_propagation) over the
 *               field's samples (a linear convolution), which needs
 *               py >= 2 ny - 1, px >= 2 nx - 1 (TO_E_UNSUPPORTED otherwise)
 *               and z > 0 (TO_E_INVAL otherwise).  The table is built on the
 *               GPU (sampling, then a forward 2-D FFT) once per call for
 *               each distinct geometry, unless the job supplies one
 *               (to_job.tf_table, from to_transfer_table);
 *   TO_AUTO:    TO_DI when z >= z_crit, TO_ASM otherwise (including z <= 0),
 *               with z_crit = min(nx dx^2, ny dy^2) / lambda: the critical
 *               distance L dx / lambda of Eq. (sampling_condition) for the
 *               aperture length L = n d of each axis, the smaller one taken.
 *   The phase is evaluated in FP64 and reduced modulo one cycle before the
 *   sine and cosine; c64 fields then use FP32 arithmetic.
 * Gradients.  For a real loss L of a complex array u, the gradient array is
 *   dL/dRe(u) + i dL/dIm(u); for a linear operator A the backward map is
 *   A^H.  Parameter gradients are ACCUMULATED (+=) into caller buffers in a
 *   fixed order (bitwise deterministic).
 * Streams.  Every call only enqueues work on `stream` (a hipStream_t, NULL =
 *   the null stream) and returns; results are valid once the stream is
 *   synchronized.  No host synchronization happens inside a call except on
 *   the first use of a device (table upload) or when the workspace grows.
 * Errors.  Every entry point returns a to_status and never aborts.  All
 *   arguments are validated on the host before anything is enqueued;
 *   TO_E_INVAL for null pointers or out-of-range values, TO_E_UNSUPPORTED
 *   for sizes outside the supported set, TO_E_NOMEM if the workspace cannot
 *   be allocated, TO_E_HIP for a failing HIP call.  to_last_error() returns a
 *   description of the calling thread's last failure.  NaN/Inf in the data
 *   are propagated, not checked.
 */
#ifndef TOPROP_H
#define TOPROP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TO_OK = 0,
  TO_E_INVAL = -1,
  TO_E_UNSUPPORTED = -2,
  TO_E_NOMEM = -3,
  TO_E_HIP = -4
} to_status;

typedef enum { TO_ASM = 0, TO_FRESNEL = 1, TO_DI = 2, TO_AUTO = 3 } to_method;
typedef enum { TO_C64 = 0, TO_C128 = 1 } to_dtype;

/* Element applied before the propagation (fused into its first pass).  Flags
 * combine; the composite modulation is M(r) = P(r) C(r) T(r) J where
 *   TO_EL_PHASE   P = exp(i phi(r)), phi = el_phase [ny][nx] (radians);
 *   TO_EL_COMPLEX C = el_complex [ny][nx] (complex of the job's dtype);
 *   TO_EL_LENS    T = exp(-i pi r^2 / (lambda el_f)), r measured from the
 *                 optical axis (thin lens, no pupil);
 *   TO_EL_JONES   J = el_jones, a uniform 3x3 complex matrix mixing the
 *                 three components (needs ncomp == 3); a 2x2 Jones matrix is
 *                 embedded with J[2][2] = 1;
 *   TO_EL_JONES_MAP  J = J(r) from el_jones_map, a spatially varying 3x3
 *                 matrix (complex of the job's dtype, [3][3][ny][nx]: entry
 *                 (r, c) is the plane 3 r + c); needs ncomp == 3, excludes
 *                 TO_EL_JONES (section "Polarization": Jones matrices act per
 *                 pixel).                                                    */
#define TO_EL_PHASE 1u
#define TO_EL_COMPLEX 2u
#define TO_EL_LENS 4u
#define TO_EL_JONES 8u
#define TO_EL_JONES_MAP 16u

/* Epilogue of a forward propagation (fused into its last pass), computed per
 * component from the intensity I = |u|^2 of the propagated field:
 *   TO_EPI_MSE       loss += epi_scale * sum (I - T)^2 over fields, comps and
 *                    pixels (T = epi_ref, broadcast over fields/comps);
 *                    epi_grad = 4 epi_scale (I - T) u  (use epi_scale = 1/n
 *                    for a mean);
 *   TO_EPI_WEIGHTED  loss += epi_scale * sum W I  (W = epi_ref);
 *                    epi_grad = 2 epi_scale W u.
 *   TO_EPI_INTENSITY epi_out[b][y][x] += epi_scale * sum over components of
 *                    I (the detected intensity, section "Polarization", and
 *                    with one job per wavelength sharing epi_out, the
 *                    incoherent polychromatic sum of Eq. (I_poly), epi_scale
 *                    being the wavelength's weight).  `out` may be NULL (the
 *                    field is then not stored).  Its gradient, given dL/dI,
 *                    is the TO_EPI_WEIGHTED epilogue with W = dL/dI.
 * epi_loss is one device double, accumulated.                                */
typedef enum { TO_EPI_NONE = 0, TO_EPI_MSE = 1, TO_EPI_WEIGHTED = 2, TO_EPI_INTENSITY = 3 } to_epilogue;

/* One propagation job: `batch` fields of `ncomp` components, all on the same
 * grid, through the same element and the same free-space distance.          */
typedef struct to_job {
  int32_t ny, nx;     /* field grid (rows, columns), >= 1                      */
  int32_t py, px;     /* padded grid (see Padding above), py >= ny,
                         px >= nx (py = 2 ny, px = 2 nx is "2x padding")      */
  int32_t method;     /* to_method                                             */
  int32_t ncomp;      /* components per field: 1 (scalar) or 3 (polarized)    */
  double dy, dx;      /* sample spacing [m], > 0                               */
  double wavelength;  /* [m], > 0                                              */
  double z;           /* propagation distance [m], any sign (0 = identity)     */
  double y0, x0;      /* grid offset from the optical axis [m]                 */
  int64_t batch;      /* number of fields (0 = nothing to do)                  */
  uint32_t el_flags;  /* TO_EL_* (0 = free space only)                         */
  int32_t epi;        /* to_epilogue                                           */
  const void* el_phase;   /* TO_EL_PHASE: real [ny][nx]                         */
  const void* el_complex; /* TO_EL_COMPLEX: complex [ny][nx]                    */
  double el_f;            /* TO_EL_LENS: focal length [m], != 0                 */
  double el_jones[18];    /* TO_EL_JONES: row-major 3x3, (re, im) pairs          */
  const void* epi_ref;    /* MSE / WEIGHTED: real [ny][nx] target or weight      */
  double epi_scale;
  void* epi_grad;         /* MSE / WEIGHTED: complex, same layout as `out`       */
  double* epi_loss;       /* MSE / WEIGHTED: one device double, accumulated      */
  const void* in;         /* complex [batch][ncomp][ny][nx]                      */
  void* out;              /* complex [batch][ncomp][ny][nx]; may equal `in`      */
  void* epi_out;          /* INTENSITY: real [batch][ny][nx], accumulated        */
  const void* el_jones_map; /* TO_EL_JONES_MAP: complex [3][3][ny][nx]           */
  const void* tf_table;   /* TO_DI (also when TO_AUTO resolves to it): NULL, or
                             the job's transfer function as written by
                             to_transfer_table, complex [py][px]; read only.
                             Ignored for the other methods.                    */
} to_job;

/* Gradient buffers of one job for to_propagate_backward.                    */
typedef struct to_grad {
  const void* grad_out;  /* dL/d(out), layout of job.out                         */
  void* grad_in;         /* dL/d(in) (overwritten), layout of job.in, or NULL    */
  const void* saved_in;  /* the job's forward input; required when grad_phase or
                            grad_f is requested                                  */
  void* grad_phase;      /* TO_EL_PHASE: real [ny][nx], += dL/dphi summed over
                            fields and components, or NULL                       */
  double* grad_f;        /* TO_EL_LENS: one device double, += dL/df, or NULL     */
  uint32_t flags;        /* TO_GRAD_* (0 = none)                                 */
} to_grad;

/* grad_in is read by nothing but the next job of the same call (the link of
 * a backward chain, its grad_out): where the library fuses the two layers it
 * may leave grad_in unwritten (its contents are then unspecified).          */
#define TO_GRAD_IN_TRANSIENT 1u

/* Forward propagation of every job (Eq. (field_propagation_tf) after the
 * element of Eq. (field_modulation)): out = P_z (M in), with the optional
 * loss epilogue.  Jobs may differ in every field (the batch dimension of the
 * paper's tensors, generalised to uneven grids, wavelengths and distances).
 *
 * Scheduling: jobs whose device ranges conflict (one writes what another
 * reads or writes, judged from the pointers and sizes in the records) run
 * in call order; independent jobs are spread longest-first over up to four
 * "lanes": the caller's `stream` and three library streams (default
 * priority) that wait on an event recorded on `stream` at entry and are
 * joined back into it at exit.  All work therefore completes in `stream`
 * order, and the call may be captured into a HIP graph from `stream` (after
 * one uncaptured call of the same shapes has sized the workspaces; a later
 * call that grows a workspace invalidates graphs captured before it).  Jobs
 * whose intensity epilogues add into the same epi_out range do not conflict
 * with each other: such jobs on different lanes add into private zeroed
 * copies, which are added into epi_out in lane order after the lanes join
 * (deterministic for a given call; the order differs from the call order,
 * so sums agree with a one-job-per-call loop to rounding).  Calls issued
 * concurrently on different caller streams of one device share the lanes'
 * workspaces and must be serialised by the caller.                           */
to_status to_propagate(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * operation, arguments and results (to rounding) as to_propagate, with no
 * allocation of any kind: every workspace (the padded intermediate of a
 * chunk of fields, loss partial sums, transfer-function and twiddle tables)
 * lives in one static device array of TO_NOALLOC_SCRATCH_BYTES that each
 * GPU the library runs on holds from the library's first use on it until
 * the process ends.  Differences from to_propagate:
 *   - all work runs on `stream`, jobs in call order, one chunk of fields at
 *     a time (no library streams, no fused layer chains);
 *   - padded extents must be powers of two, direct integration (TO_DI, or
 *     TO_AUTO resolving to it) needs the job's tf_table, and one field's
 *     intermediate (ny x px complex values, times 3 for a Jones element or a
 *     three-component intensity epilogue) must fit the array less its
 *     tables (about 62 MiB: a 1024 x 1024 complex64 field padded to
 *     2048 x 2048 needs 16 MiB); otherwise TO_E_UNSUPPORTED with the sizes
 *     in to_last_error(), before anything is enqueued;
 *   - launches are not timed by to_profile_begin.
 * Every call on a GPU uses that GPU's one array: calls that overlap in time
 * on one GPU (different streams, or host threads) race and must be
 * serialised by the caller.  A call rebuilds the tables it reads and writes
 * every intermediate before reading it, so nothing carries over between
 * calls.  The call may itself be captured into a HIP graph.              */
#define TO_NOALLOC_SCRATCH_BYTES (64u << 20)
to_status to_propagate_noalloc(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream);

/* Modulation only (Eq. (field_modulation) / the Jones product):
 * out = M in, or out = M^H in when adjoint != 0.  The propagation fields of
 * the job (py, px, method, z) are ignored.   */
to_status to_modulate(const to_job* jobs, int32_t njobs, to_dtype dtype, int32_t adjoint,
                      void* stream);

/* Backward pass of to_propagate for each job (section "Gradient-based
 * optimization"): with g_mod = P_z^H grad_out,
 *   grad_in     = M^H g_mod,
 *   grad_phase += sum Im(g_mod conj(M saved_in)),
 *   grad_f     += sum (pi r^2 / (lambda f^2)) Im(g_mod conj(M saved_in)).
 * P_z^H is the same pipeline with conj(H).  The per-layer input is taken
 * from `saved_in` (recomputation: no padded spectra are stored).  The
 * job's epilogue fields are ignored.  grads[i] belongs to jobs[i].  Jobs
 * are scheduled over the lanes as in to_propagate; jobs that accumulate
 * into the same grad_phase or grad_f run in call order on one lane, so the
 * accumulation order (and the result) does not depend on the schedule.     */
to_status to_propagate_backward(const to_job* jobs, const to_grad* grads, int32_t njobs,
                                to_dtype dtype, void* stream);

/* Propagation of a mutual coherence function (section "Spatial coherence"):
 * job->in / job->out hold Gamma [ny][nx][ny][nx] (r1 = (y1, x1) major,
 * r2 = (y2, x2) minor), job->batch must be 1 and ncomp 1.
 *   adjoint == 0:  Gamma_out = P (M Gamma M^H) P^H
 *                  (M = diag of the job's scalar element; P = P_z);
 *   adjoint != 0:  Gamma_out = M^H (P^H Gamma P) M, the adjoint of the
 *                  forward map under Re tr(A^H B).
 * When adjoint != 0 and grad is not NULL, grad->saved_in is the forward
 * input Gamma_in (not aliasing job->out) and grad->grad_phase (+=) receives
 * dL/dphi of the phase element, with job->in holding dL/dGamma_out:
 *   dL/dphi(r) = sum_b Im(G[r,b] conj(Gm[r,b])) - sum_a Im(G[a,r] conj(Gm[a,r])),
 *   G = P^H (dL/dGamma_out) P, Gm = M Gamma_in M^H.
 * Forward epilogue (adjoint == 0) on the time-averaged intensity
 * I(r) = Re Gamma_out(r, r):  TO_EPI_MSE  loss += epi_scale sum (I - T)^2,
 * TO_EPI_WEIGHTED loss += epi_scale sum W I; epi_grad (complex, n x n)
 * receives dL/dGamma_out, zero off the diagonal; TO_EPI_INTENSITY
 * epi_out[y][x] += epi_scale I(r) (real [ny][nx]).
 * Computed as two batched propagations of the n = ny nx rows (P^H along r2,
 * then P along r1) around transposes; needs workspace for one extra copy of
 * Gamma.  n must not exceed 46340; no Jones element.                         */
to_status to_coherence_propagate(const to_job* job, to_dtype dtype, int32_t adjoint,
                                 const to_grad* grad, void* stream);

/* Unfused reference form of to_propagate / to_propagate_backward, kept as the
 * comparison baseline for the fused kernels: each field goes through one
 * kernel per step of Eq. (field_propagation_tf) — modulate, zero-pad into a
 * full py x px array, row FFTs, column FFTs, multiply by a stored table of
 * H, inverse FFTs, crop — with every intermediate in device memory.  Same
 * arguments and results (to rounding) as the fused entry points (a Jones
 * element is applied to the three components by a modulation kernel before
 * they are propagated one by one).  Workspace: two py x px and two ny x nx complex arrays. */
to_status to_propagate_plain(const to_job* jobs, int32_t njobs, to_dtype dtype, void* stream);
to_status to_propagate_backward_plain(const to_job* jobs, const to_grad* grads, int32_t njobs,
                                      to_dtype dtype, void* stream);

/* Launch schedule of one padded grid and dtype: the column-pass
 * configuration (0 .. 4: LDS budget, points per thread, prefetch and, for
 * complex64, the factorisation of the column FFT: 0, 1 and 4 take the split
 * transform (a radix pass across the column, sub-transforms inside one
 * wavefront), 2 and 3 the Stockham passes) and the budget of padded
 * intermediate per chunk of fields [MiB].                                  */
typedef struct to_plan {
  int32_t col_variant;
  int32_t chunk_mb;
  int32_t row_fpb;  /* fields per row-pass workgroup, 1 .. 8; 0: as many as
                       keep one round of resident workgroups per launch     */
  double us;  /* measured time of the tuned forward propagation [us]       */
} to_plan;

/* Autotuner (the schedules of the batch/schedule layer): times every column
 * configuration for several chunk sizes on this job, then the fields per
 * row-pass workgroup with the fastest of those (forward propagation,
 * element included, epilogue left out, into a temporary output), stores the
 * fastest in the plan table under (job->py, job->px, dtype), then runs the
 * job once with it (so job->out and the epilogue are as after
 * to_propagate).  Later calls for the same padded grid and dtype use the
 * plan.  Synchronizes `stream` and allocates: not for use under graph
 * capture.  If the environment variable TOPROP_PLAN_CACHE names a file,
 * the table is read from it on first use (a file that fails the format
 * checks of to_plan_load is ignored) and written back after each tuning.
 * `result` (may be NULL) receives the chosen plan.
 * Precedence when a job runs: TOPROP_COL_VARIANT / TOPROP_CHUNK_MB /
 * TOPROP_ROW_FPB (tuning overrides) > plan table > built-in defaults (variant 1; variant 0 for
 * complex64 columns of 4096 points and more; 128 MiB).                                         */
to_status to_autotune(const to_job* job, to_dtype dtype, void* stream, to_plan* result);

/* Plan table access (host only, no device work).  to_plan_get sets *found
 * to 1 and fills *plan when (py, px, dtype) has a plan, else *found = 0.
 * to_plan_set validates (py, px powers of two in [8, 8192], col_variant in
 * [0, 5), chunk_mb in [1, 65536], row_fpb in [0, 8], us >= 0) and stores.  */
to_status to_plan_get(int32_t py, int32_t px, to_dtype dtype, to_plan* plan, int32_t* found);
to_status to_plan_set(int32_t py, int32_t px, to_dtype dtype, const to_plan* plan);
to_status to_plan_clear(void);

/* Plan files: text, first line "toprop-plan 2", then one record per line
 * "<c64|c128> <py> <px> <col_variant> <chunk_mb> <row_fpb> <us>" ('#' lines
 * are comments); files headed "toprop-plan 1" hold the same records without
 * row_fpb (read as 0).  to_plan_load merges a file into the table only if every line
 * passes the checks of to_plan_set (and no key repeats); otherwise it
 * returns TO_E_INVAL naming the line and leaves the table unchanged.
 * to_plan_save writes the table atomically (temporary file + rename).     */
to_status to_plan_load(const char* path);
to_status to_plan_save(const char* path);

/* Description of the calling thread's last non-TO_OK status ("" if none).   */
const char* to_last_error(void);

/* Frees the library's workspace on every device (waits for the device).     */
to_status to_release(void);

/* Transfer function of the job's propagation (after TO_AUTO is resolved):
 * table[ky][kx] = H at padded-grid bin (ky, kx), FFT order, complex of
 * `dtype`, py x px, caller-owned device memory.  For TO_DI this is the table
 * a DI job may carry in tf_table, so that repeated calls with the same
 * geometry (ny, nx, py, px, dy, dx, wavelength, z) skip its construction;
 * it must not be written while a call that reads it is in flight.  The
 * job's field pointers, element and epilogue are ignored.                    */
to_status to_transfer_table(const to_job* job, to_dtype dtype, void* table, void* stream);

/* Resampling onto another grid (section "Computational Fourier optics":
 * where input and output grids have different spacings, the field is
 * propagated on the input spacing and then interpolated onto the output
 * grid, bilinearly or to the nearest sample).  A grid is ny x nx samples of
 * spacing (dy, dx), sample (y, x) at ((y - ny/2) dy + y0, (x - nx/2) dx + x0)
 * as everywhere in this library.  Along each axis, output sample j reads the
 * input at the fractional index
 *   t = ((j - n_out/2) (d_out / d_in) + (o_out - o_in) / d_in) + n_in/2
 * (FP64, evaluated in this order without fused multiply-adds, so identical
 * grids map exactly): TO_BILINEAR weights 1 - a and a (a = t - floor t) on
 * samples floor t and floor t + 1, TO_NEAREST takes sample floor(t + 1/2);
 * the 2-D weights are products of the axis weights, and samples outside the
 * input window read zero.
 *   adjoint == 0: src [batch][grid_in], dst [batch][grid_out], dst = R src;
 *   adjoint != 0: src [batch][grid_out], dst [batch][grid_in], dst = R^T src
 *                 (the gradient map: the weights are real), computed as a
 *                 gather in a fixed order (deterministic, no atomics).
 * dst is overwritten and must not overlap src (TO_E_INVAL).                  */
typedef enum { TO_NEAREST = 0, TO_BILINEAR = 1 } to_interp;
typedef struct to_grid {
  int32_t ny, nx;   /* samples, >= 1                                          */
  double dy, dx;    /* spacing [m], > 0                                       */
  double y0, x0;    /* offset of the grid from the optical axis [m]           */
} to_grid;
to_status to_resample(const void* src, void* dst, const to_grid* grid_in, const to_grid* grid_out, int64_t batch,
                      int32_t interp, int32_t adjoint, to_dtype dtype, void* stream);

/* The method a job runs with: job->method, or for TO_AUTO the choice by the
 * critical distance described with the transfer functions.  Host only.      */
to_status to_resolve_method(const to_job* job, int32_t* method);

/* Jones matrices of standard elements (section "Polarization"), host only,
 * written to out[18] in the layout of to_job.el_jones (row-major 3x3,
 * (re, im) pairs), the 2x2 Jones matrix acting on (Ex, Ey) embedded with
 * J_zz = 1 and no coupling to Ez.
 *   to_jones_linear_polarizer: transmission axis at theta [rad] from x, the
 *     projector [[c^2, c s], [c s, s^2]] (c = cos theta, s = sin theta);
 *   to_jones_waveplate: fast axis at theta, retardance Gamma [rad] of the
 *     slow axis, R(theta) diag(1, exp(i Gamma)) R(-theta) (Gamma = pi/2: a
 *     quarter-wave plate), no global phase;
 *   to_jones_compose: out = then * first (first acts first); out may alias
 *     either input.
 * TO_E_INVAL for a NULL pointer or a non-finite angle.                      */
to_status to_jones_linear_polarizer(double theta, double* out);
to_status to_jones_waveplate(double theta, double retardance, double* out);
to_status to_jones_compose(const double* first, const double* then, double* out);

/* Captured calls (the batch dimension of the paper's Overview, §2, run as
 * one HIP graph).  to_graph_create runs one to_propagate call (grads ==
 * NULL) or one to_propagate_backward call (grads != NULL) over `jobs` on
 * `stream` — its results are those of that call, and it sizes every
 * workspace — then synchronizes `stream` and captures the same call, all
 * lanes and job-queue launches included, into a HIP graph that the library
 * instantiates and owns.  to_graph_launch replays it on `stream`: the same
 * kernels with the same arguments, reading and writing the buffers the
 * records named at creation, so a replay equals the call on the buffers'
 * contents at replay time.  The caller keeps those buffers alive (and at
 * the same addresses) until to_graph_destroy, and does not let a replay
 * overlap another call of this library on the device (they share the
 * workspaces).  Allocates (the first call, the graph): not for use under
 * another capture.  Errors: TO_E_INVAL (NULL out, njobs < 1, invalid
 * jobs as in the call), TO_E_HIP (capture or instantiation failed; nothing
 * is created).                                                               */
typedef struct to_graph_s* to_graph;
to_status to_graph_create(const to_job* jobs, const to_grad* grads, int32_t njobs, to_dtype dtype,
                          void* stream, to_graph* out);
to_status to_graph_launch(to_graph graph, void* stream);
to_status to_graph_destroy(to_graph graph);

/* Library version, e.g. "toprop 0.1.0 gfx950".                              */
const char* to_version(void);

/* Kernel timing, for measurement only (not part of the computation).
 * to_profile_begin() clears previous results and, until to_profile_end(),
 * brackets every kernel the library launches with a pair of HIP events
 * recorded on the launch's own stream.  to_profile_end() waits for those
 * events and aggregates the elapsed GPU time per kernel name
 * ("<phase>.<kernel>_<dtype>_L<transform length>").  to_profile_count() and
 * to_profile_entry() read the aggregate: `name` receives at most name_len
 * bytes including the terminator.  Not thread-safe with concurrent calls
 * on other threads while enabled.                                            */
to_status to_profile_begin(void);
to_status to_profile_end(void);
int32_t to_profile_count(void);
to_status to_profile_entry(int32_t i, char* name, int32_t name_len, int64_t* launches,
                           double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* TOPROP_H */
