/*
 * fsa.h -- C ABI of the MI355X (gfx950) FSA convolution library.
 *
 * The library evaluates the convolution potential Phi = U * rho of a radial,
 * singular kernel U with a smooth, compactly supported density rho, sampled
 * on a uniform grid of the box prod_j [-L_j, L_j], with the far-field smooth
 * approximation (FSA) method of Liu & Zhang (arXiv 2504.19410):
 *
 *   - problem statement: Phi on the grid from rho on the same grid (Sec. 1);
 *   - grid: x_j = -L_j + i_j h_j, h_j = 2 L_j / N_j, i_j in [0, N_j)
 *     (eq. UniformMesh; anisotropic boxes as in Sec. 2.4);
 *   - kernel tensor T = T(1) + T(2): T(1) by trapezoidal sampling of the
 *     smooth far-field kernel U^eps (eq. Tensor1 / TensorAnis), T(2) from the
 *     whole-space Fourier transform of U - U^eps (eq. FouTran, Table 1,
 *     eq. Tensor2), built once per plan;
 *   - each evaluation: the discrete aperiodic convolution of eq. DiscConv as
 *     a 2x zero-padded FFT convolution (Sec. 2.2, 2.3).
 *
 * Conventions shared by every entry point
 *   - All array pointers passed to fsa_apply* and fsa_server_submit are
 *     DEVICE pointers on the device that was current when the plan's tensor
 *     was built; they are owned by the caller.  Streams are hipStream_t passed
 *     as void* (NULL = the null stream).
 *   - rho and phi are dense C-order arrays of shape (N_0, ..., N_{d-1}) in
 *     the plan precision (float for FSA_F32, double for FSA_F64); the element
 *     at index i sits at x_j = -L_j + i_j h_j.  The last axis is contiguous.
 *   - Every argument is validated synchronously.  On failure the call
 *     returns a non-zero fsa_status, out-parameters are left untouched, and
 *     fsa_last_error() describes the problem.  Asynchronous device errors
 *     surface as FSA_EDEVICE at the next call that synchronises.
 *   - No C++ exception crosses this interface.
 *   - A built plan is immutable: concurrent fsa_apply calls on one plan are
 *     safe when they use distinct workspaces.
 */
#ifndef FSA_H
#define FSA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FSA_OK = 0,
    FSA_EINVAL = 1,        /* invalid argument (shape, size, parameter)      */
    FSA_EUNSUPPORTED = 2,  /* valid but not supported (grid length, kernel)  */
    FSA_ENOMEM = 3,        /* device or host allocation failed               */
    FSA_EDEVICE = 4,       /* a HIP runtime call or kernel failed            */
    FSA_ESTATE = 5,        /* call out of order (e.g. apply before build)    */
    FSA_EBUDGET = 6,       /* server: request can never fit the HBM budget   */
    FSA_ECANCELLED = 7,    /* server: request was cancelled                  */
    FSA_ETIMEDOUT = 8      /* server: request waited past the queue timeout  */
} fsa_status;

/* Kernels U(r) with their FSA split (Table 1; eqs. KerAppr, lnrAppr):
 *   FSA_COULOMB_3D    U = 1/(4 pi r),            U^eps = U erf(r/eps)
 *   FSA_YUKAWA_3D     U = e^{-lam r}/(4 pi r),   Gaussian-screened split with
 *                     FT[U - U^eps] = (1 - e^{-(k^2+lam^2) eps^2/4})/(k^2+lam^2)
 *                     (the paper lists Yukawa in Sec. 5.3 without a split)
 *   FSA_LOG_2D        U = -(1/2pi) ln r,          eq. lnrAppr
 *   FSA_COULOMB_2D    U = 1/(2 pi r),             U^eps = U erf(r/eps)
 *   FSA_BIHARMONIC_3D U = r/(8 pi),               U^eps = U erf(r/eps)
 *   FSA_BIHARMONIC_2D U = -r^2 (ln r - 1)/(8 pi), Table 1
 *   FSA_DDI_3D        dipole-dipole interaction with dipole orientations n, m
 *                     (Sec. 5.3): Phi = -(m.n) rho - 3 Coulomb(d_nm rho),
 *                     d_nm = (n.grad)(m.grad), the Coulomb part by FSA and
 *                     d_nm rho as the spectral derivative of rho on its own
 *                     grid, periodic on the box (q_j = i_j for i_j < N_j/2,
 *                     else i_j - N_j; k_j = pi q_j / L_j; real part).
 *   FSA_YUKAWA_2D     U = K0(lam r)/(2 pi) (Sec. 5.3); general construction.
 *   FSA_QUASI2D_DDI   quasi-2D dipole-dipole interaction (Sec. 5.3) with the
 *                     confinement width eta and dipole orientation n:
 *                     Phi = U~ conv S,
 *                     U~(r) = (2 pi)^{-3/2} int e^{-s^2/2} (r^2 + eta^2 s^2)^{-1/2} ds
 *                           = (2 pi)^{-3/2} eta^{-1} e^x K0(x),  x = r^2/(4 eta^2),
 *                     S = -(3/2)(d_{n_perp n_perp} - n_3^2 Lap) rho, n_perp =
 *                     (n_0, n_1), as the spectral derivative on the grid (as for
 *                     FSA_DDI_3D); U~ by the general construction.
 *
 * General construction (Sec. 4, eq. GeneralApprox1; fsa_kernel.general != 0
 * for kinds 1-7, always for kinds 8 and 9):
 *   U^eps = U erf(r/eps) (1 - xi(r)),  xi(r) = erfc((r - 6 eps)/eps)/2 where
 *   U erf(r/eps) is not smooth at r = 0 (3D Yukawa, 2D log, 2D biharmonic,
 *   kinds 8 and 9), xi = 0 otherwise (then U^eps is Table 1's);
 *   W(k) = FT[U - U^eps](k) by quadrature of the radial transform (eq.
 *   Fourier-Symmetric), in FP64 on the device.  A windowed plan needs
 *   eps <= R0/12 (the window has decayed to 1e-17 at R0); its default eps is
 *   R0/16. */
typedef enum {
    FSA_COULOMB_3D = 1,
    FSA_YUKAWA_3D = 2,
    FSA_LOG_2D = 3,
    FSA_COULOMB_2D = 4,
    FSA_BIHARMONIC_3D = 5,
    FSA_BIHARMONIC_2D = 6,
    FSA_DDI_3D = 7,
    FSA_YUKAWA_2D = 8,
    FSA_QUASI2D_DDI = 9
} fsa_kernel_kind;

/* Arithmetic of the per-evaluation FFT convolution.  For FSA_F32 and
 * FSA_F64 the tensor is generated in FP64 and rounded to this precision once.
 *
 * FSA_DD is the extended-precision mode (the paper's quadruple-precision
 * runs, Sec. 5.1, Table 2): every real is a double-double pair (hi, lo) of
 * doubles, interleaved, value hi + lo (106-bit significand, rounding
 * ~1.2e-32).  rho and phi are arrays of N_0 x ... x N_{d-1} such pairs; the
 * tensor is generated and the convolution runs in double-double.  Only the
 * Coulomb kernels (FSA_COULOMB_3D, FSA_COULOMB_2D, closed-form construction)
 * and grids N_j = 2^a in [8, 1024] are supported (FSA_EUNSUPPORTED
 * otherwise); plans in this precision are not batched, served or tuned. */
typedef enum { FSA_F32 = 0, FSA_F64 = 1, FSA_DD = 2 } fsa_precision;

typedef struct {
    int kind;       /* fsa_kernel_kind                                        */
    double lambda;  /* Yukawa screening lam > 0; ignored by other kernels     */
    double eps;     /* split parameter; <= 0 selects the default R0/8 (R0/16
                       for the windowed general construction), R0 = 2 min_j
                       L_j (condition (b) of eq. ApproxProp, Remark 2.1 and
                       Appendix B)                                            */
    double n[3];    /* FSA_DDI_3D: dipole orientations n and m (finite, non-  */
    double m[3];    /* zero; used as given); FSA_QUASI2D_DDI: n (m ignored);
                       ignored by other kernels                               */
    double eta;     /* FSA_QUASI2D_DDI: confinement width eta > 0            */
    int general;    /* non-zero: the general construction for kinds 1-7      */
} fsa_kernel;

typedef struct fsa_plan_s* fsa_plan;

/* Creates a plan (host only; no device work).
 *   k   kernel and split parameter (see fsa_kernel).
 *   d   2 or 3; must match the kernel.
 *   L   d half-widths L_j > 0 of the box prod_j [-L_j, L_j] (host array).
 *   N   d grid sizes (host array): even, 8 <= N_j <= 2048, of the form 2^a or
 *       3*2^a (the padded transform length 2 N_j must factor into the
 *       supported radices).
 *   p   FSA_F32 or FSA_F64.
 * The split parameter must satisfy 0 < eps <= R0/4, and eps <= R0/12 for a
 * windowed general construction (FSA_EINVAL otherwise).
 * Double-precision accuracy needs eps <= R0/5.85 (condition (b) of eq.
 * ApproxProp, Appendix B) and eps >= 2 max_j h_j, which keeps the
 * trapezoidal error of the regular part, ~ e^{-pi^2 eps^2 / h^2}, below
 * 1e-17; the paper's coarse-grid experiments deliberately violate the latter.
 * FSA_EUNSUPPORTED for a grid length outside the supported set.  *out
 * receives the plan. */
fsa_status fsa_plan_create(const fsa_kernel* k, int d, const double* L, const int64_t* N,
                           fsa_precision p, fsa_plan* out);

/* Reports the plan's parameters; any out-pointer may be NULL.
 *   eps_used         the split parameter the plan uses.
 *   h                d mesh sizes h_j (host array of d doubles).
 *   tensor_bytes     device bytes of the plan's spectral tensor.
 *   workspace_bytes  device bytes of the scratch buffer fsa_apply needs. */
fsa_status fsa_plan_query(fsa_plan plan, double* eps_used, double* h, size_t* tensor_bytes,
                          size_t* workspace_bytes);

/* Generates the plan's spectral tensor on the current device, in FP64,
 * asynchronously on `stream` (Precomp in the paper's terms, Sec. 5.1
 * Example 2):  T^[p] = ( DFT(T(1))[p] + W(|k_p|) ) / prod_j 2N_j, with
 * k_j = pi p_j / (2 L_j); since T(2) = IDFT(W) (eq. Tensor2), DFT(T(2)) = W
 * exactly.  T^ is real and even in every p_j (Sec. 2.3), so only the octant
 * 0 <= p_j <= N_j is stored, in the plan precision.  The library allocates
 * and owns it, with the plan's twiddle tables and, for a 3D plan whose box
 * has equal sides, an order of the (N_1 + 1)(N_2 + 1) lines of axis 0
 * (4 bytes each, computed by the first build, reused by later ones).  May be
 * called again (rebuilds in place). */
fsa_status fsa_build_tensor(fsa_plan plan, void* stream);

/* One evaluation (Execution in the paper's terms): phi = crop(IDFT(T^ .
 * DFT(pad(rho)))) through 3 (2D) or 5 (3D) kernels enqueued on `stream`;
 * returns without host synchronisation.
 *   rho        device input, plan precision, shape N (read only).
 *   phi        device output, plan precision, shape N; may equal rho.
 *   workspace  device scratch of at least workspace_bytes (fsa_plan_query),
 *              256-byte aligned; contents on entry are ignored.
 * FSA_ESTATE if the tensor has not been built. */
fsa_status fsa_apply(fsa_plan plan, const void* rho, void* phi, void* workspace, void* stream);

/* Capacity of the workspace that fsa_apply_noalloc uses (128 MiB): plans
 * whose workspace_bytes fit, e.g. every 3D grid up to 128^3 in FP32 and FP64
 * and every 2D grid up to 2048^2 in FP32 and FP64. */
#define FSA_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): fsa_apply
 * with the workspace taken from a static device array of the library,
 * FSA_NOALLOC_SCRATCH_BYTES long, one per device, held from the first call on
 * that device until the process ends.  Makes no device or host allocation
 * (the first call on a device resolves the array's address once).
 *   rho, phi, stream  as for fsa_apply; the results are bitwise those of
 *                     fsa_apply with the same launch choices.
 * FSA_EINVAL if the plan's workspace_bytes exceed FSA_NOALLOC_SCRATCH_BYTES
 * (nothing is launched), FSA_ESTATE as fsa_apply.  Every call on one device
 * shares that device's array and may leave data in it (the passes write
 * every workspace entry they read): calls whose executions overlap on one
 * device -- on different streams or from different threads without ordering
 * -- race and give wrong results; order them on one stream. */
fsa_status fsa_apply_noalloc(fsa_plan plan, const void* rho, void* phi, void* stream);

/* Number of kernel launches of one evaluation with the plan's current
 * schedule (3 in 2D; 2 + 3 x slabs in 3D, see fsa_tune_set_slabs) and, if
 * `passes` is not NULL, the fsa_pass of each launch in order (cap entries
 * available). */
fsa_status fsa_plan_launches(fsa_plan plan, int* n, int* passes, int cap);

/* Profiling variant of fsa_apply: the same kernels on the same stream, with
 * hipEventRecord(events[2i], stream) right before launch i (of n, from
 * fsa_plan_launches) and hipEventRecord(events[2i + 1], stream) right after
 * it, so that hipEventElapsedTime(events[2i], events[2i + 1]) times launch i.
 * A pair of NULL entries leaves launch i untimed.  The events are hipEvent_t
 * handles created by the caller; n_events must equal 2n.  Events created
 * with hipEventDisableSystemFence disturb the timed work least (a default
 * event writes back and invalidates the caches when it is recorded, so the
 * next launch starts cold).  For profiling tools and benchmarks. */
fsa_status fsa_apply_events(fsa_plan plan, const void* rho, void* phi, void* workspace,
                            void* stream, void* const* events, int n_events);

/* Device bytes of the workspace fsa_apply_batched needs for these plans. */
fsa_status fsa_batch_workspace_bytes(int n, const fsa_plan* plans, size_t* bytes);

/* Evaluates n independent problems (plans may differ in kernel, box, grid
 * and precision) as one hipGraph of persistent launches: for each pass, in
 * dependency order, and each transform length that pass uses, ONE launch
 * walks the work items (problem, tile or pencil) of every problem that
 * shares the length.  The graph is captured on first use of a batch
 * signature and replayed afterwards.  A launch takes the tuning table's
 * choice for its total number of transforms (fsa_autotune_batched tunes
 * those); under the same launch choices each problem's result is bitwise
 * equal to fsa_apply on that problem alone, and under other choices it
 * agrees to rounding.
 *   plans, rho, phi  host arrays of n entries; rho[i]/phi[i] are device
 *                    pointers for plans[i].
 *   workspace        device scratch of >= fsa_batch_workspace_bytes bytes.
 * The device pointers are part of the captured graph: a call with the same
 * plans but different pointers re-captures.  Dipole-dipole plans
 * (FSA_DDI_3D, FSA_QUASI2D_DDI) and double-double plans are not batched:
 * FSA_EUNSUPPORTED. */
fsa_status fsa_apply_batched(int n, const fsa_plan* plans, const void* const* rho,
                             void* const* phi, void* workspace, size_t workspace_bytes,
                             void* stream);

/* Number of persistent launches in the graph captured for this batch
 * signature (one per pass and transform length); FSA_ESTATE if the batch
 * has not been run yet.  For tests and tools. */
fsa_status fsa_batch_launches(int n, const fsa_plan* plans, const void* const* rho,
                              void* const* phi, void* workspace, int* launches);

/* Releases the plan and its device tensor (after synchronising its device). */
fsa_status fsa_plan_destroy(fsa_plan plan);

/* Device pointer and octant extents of the built spectral tensor, for tests
 * and tools.  dims[0..d-1] receive (N_{d-1}+1, ..., N_0+1): the octant is
 * stored with the LAST grid axis outermost, i.e. index [p_{d-1}]...[p_0]. */
fsa_status fsa_plan_tensor(fsa_plan plan, const void** tensor, int64_t* dims);

/* ------------------------------------------------------------------------- */
/* Autotuner: launch choices per (precision, pass, transform length)          */
/* ------------------------------------------------------------------------- */

/* Passes of one evaluation (Sec. 2.3: the forward FFT, the pointwise
 * product with the tensor and the inverse FFT of eq. DiscConv, split by
 * axis).  Transform length: the half length M = N_{d-1} of the padded row
 * for FSA_PASS_R2C / FSA_PASS_C2R, the padded length P = 2 N_j otherwise. */
typedef enum {
    FSA_PASS_R2C = 0,   /* A: zero-pad + real FFT along the last axis       */
    FSA_PASS_FWD_T = 1, /* B (3D): zero-pad + FFT along axis 1              */
    FSA_PASS_CONV = 2,  /* C: FFT along axis 0, x tensor, inverse FFT, crop */
    FSA_PASS_INV_T = 3, /* D (3D): inverse FFT along axis 1, crop           */
    FSA_PASS_C2R = 4,   /* E: inverse real FFT along the last axis, crop    */
    FSA_PASS_SPECTRAL = 5 /* dipole-dipole kinds: the source derivative     */
} fsa_pass;
/* OR-ed into the pass of the tuning calls below: the entry of the batched
 * persistent launches of that pass (fsa_apply_batched), kept apart from the
 * single-evaluation entries.  A batched launch with no batched entry of its
 * (precision, pass, length) takes the single-evaluation entry. */
#define FSA_PASS_BATCHED 16

/* Every pass kernel exists in up to five compiled variants per length:
 *   0  default radix plan and workgroup size;
 *   1  alternate radix family (another radix split and number of threads
 *      per transform);
 *   2  half-size workgroups (half the lines per tile, or teams per group);
 *   3  the default plan with the stage exchanges that only trade register
 *      and lane bits of a one-wave team done across lanes (DPP and lane
 *      swaps) instead of through the LDS (the fused pass at length 512);
 *   4  the default plan with the first forward stage of the fused pass as
 *      a matrix product on the matrix cores (FP32 MFMA; length 512).
 * and its persistent grid may use `occupancy` resident workgroups per CU
 * (0 = as many as fit).  The library keeps one process-wide table of
 * choices; untuned entries use variant 0 at full occupancy.  fsa_apply,
 * fsa_apply_batched and the server read the table when they launch.  All
 * variants compute the same transform; results differ only by rounding.
 * On first use the table is loaded from the JSON file named by the
 * environment variable FSA_TUNE_CACHE, when that is set and exists. */

/* Times every distinct (variant, occupancy) candidate of every pass of a
 * built plan on `stream` with hipEvents (median of `reps`, 1..1000, taken in
 * rounds that run each candidate once, after a warm-up round; each candidate
 * runs inside a whole evaluation, only its own launch timed) and stores the
 * fastest in the table; for a 3D plan then times the slab schedules
 * (fsa_tune_set_slabs) the same way and keeps the fastest.
 * Synchronous.
 *   rho, phi, workspace  device buffers as for fsa_apply; on return phi holds
 *                        a valid evaluation of rho with the tuned choices.
 * Batch graphs captured before the call are re-captured on their next use. */
fsa_status fsa_autotune(fsa_plan plan, const void* rho, void* phi, void* workspace, void* stream,
                        int reps);
/* The launches of a batch (fsa_apply_batched) cover many problems at once,
 * a size class that the per-plan tuning does not reach: times every
 * distinct (variant, occupancy) candidate of every persistent launch of
 * this batch (median of `reps`, 1..1000, in rounds as fsa_autotune; the
 * launch of the fused pass has its input re-created before each run) and stores
 * the fastest under the launch's size class.  Same arguments and checks as
 * fsa_apply_batched; synchronous.  On return phi holds a valid evaluation
 * with the tuned choices, and batch graphs captured before are re-captured
 * on their next use. */
fsa_status fsa_autotune_batched(int n, const fsa_plan* plans, const void* const* rho,
                                void* const* phi, void* workspace, size_t workspace_bytes,
                                void* stream, int reps);

/* Sets / reads one entry (precision: fsa_precision, pass: fsa_pass, with
 * FSA_PASS_BATCHED for the batched launches).
 * Entries are kept per size class floor(log2(lines)), `lines` being the
 * number of transforms one launch runs (rows of the last axis for the real
 * passes, axis-1 lines for B and D, axis-0 pencils for C; summed over the
 * problems of a batched launch): the best variant of a length depends on the
 * amount of work.  A launch uses the entry of the nearest tuned class of its
 * (precision, pass, length); fsa_tune_get reports that choice.  A variant
 * that does not exist at that pass and length is FSA_EINVAL.  `us` receives
 * the measured time of the entry of exactly that class (0 if set by hand or
 * not tuned at that class; may be NULL). */
fsa_status fsa_tune_set(int precision, int pass, int length, int64_t lines, int variant,
                        int occupancy);
fsa_status fsa_tune_get(int precision, int pass, int length, int64_t lines, int* variant,
                        int* occupancy, double* us);
/* Schedule of a 3D grid: passes B, C, D run in `slabs` (1..16) slabs of the
 * bins p2 of the last axis, B-C-D of one slab back to back, so that the slab's
 * spectrum can stay in the device's memory-side cache between them (slabs = 1:
 * each pass over the whole grid).  Same results for every slab count.
 * N: the three grid lengths.  fsa_autotune times 1, 2, 4, 8, 16 slabs after
 * tuning the passes.  `us` (may be NULL) receives the measured evaluation
 * time of the chosen schedule (0 if set by hand or untuned). */
fsa_status fsa_tune_set_slabs(int precision, const int64_t* N, int slabs);
fsa_status fsa_tune_get_slabs(int precision, const int64_t* N, int* slabs, double* us);
/* Bit mask of the variants that exist at (precision, pass, length). */
fsa_status fsa_tune_variants(int precision, int pass, int length, int* mask);
/* Writes the table as JSON (format "fsa-tune-1", tagged with the device's
 * architecture name) / merges a saved table into the current one.  Loading
 * rejects, as a whole, a file that is malformed, was tuned on another
 * architecture or names a variant that does not exist (FSA_EINVAL). */
fsa_status fsa_tune_save(const char* path);
fsa_status fsa_tune_load(const char* path);
/* Forgets every entry (all passes back to variant 0, full occupancy). */
fsa_status fsa_tune_reset(void);

/* ------------------------------------------------------------------------- */
/* Served variant: continuous batching with HBM-budget admission             */
/* ------------------------------------------------------------------------- */

typedef struct fsa_server_s* fsa_server;

typedef struct {
    double p50_ms, p99_ms;      /* latency: completion - arrival (the arrival
                                   time given to fsa_server_submit_at, else the
                                   submission time), queueing included       */
    double throughput_rps;      /* completed requests per second of uptime   */
    double gpts_per_s;          /* output grid points per second of uptime   */
    uint64_t done, rejected, cancelled, cache_hits, cache_misses;
    size_t hbm_in_use, hbm_peak;
    uint64_t timed_out;         /* finished FSA_ETIMEDOUT in the queue       */
} fsa_stats;

/* Creates a server on the current device.
 *   hbm_budget_bytes  cap on cached tensors + in-flight workspaces.
 *   max_inflight      concurrent requests on the device (slots, >= 1).
 *   n_streams         device streams the slots rotate over (>= 1).
 * Requests of at least 2^23 grid points run in turn on the first stream, the
 * others rotate over the rest (with n_streams = 1 everything runs in turn).
 * A submitting thread admits and launches its request itself when a slot and
 * the budget allow; one host thread per stream sleeps until that stream's
 * oldest request finishes (a blocking-sync event), then admits what the freed
 * slot allows.  No thread polls. */
fsa_status fsa_server_create(size_t hbm_budget_bytes, int max_inflight, int n_streams,
                             fsa_server* out);

/* Queues one request; never blocks on the device.  rho/phi are device
 * pointers of the request's shape and precision, owned by the caller and
 * untouched until the ticket completes.  FSA_EBUDGET if the request alone
 * exceeds the budget; FSA_EUNSUPPORTED for the dipole-dipole kinds. */
fsa_status fsa_server_submit(fsa_server s, const fsa_kernel* k, int d, const double* L,
                             const int64_t* N, fsa_precision p, const void* rho, void* phi,
                             uint64_t* ticket);

/* As fsa_server_submit, for a request that arose at t_arrival (seconds on
 * the clock of fsa_server_clock, CLOCK_MONOTONIC; < 0: now): its latency in
 * fsa_stats is counted from then, so time the caller spent before
 * submitting (a client-side queue, a full buffer pool) is included. */
fsa_status fsa_server_submit_at(fsa_server s, const fsa_kernel* k, int d, const double* L,
                                const int64_t* N, fsa_precision p, const void* rho, void* phi,
                                double t_arrival, uint64_t* ticket);
/* The server's clock: seconds of the host's monotonic clock (CLOCK_MONOTONIC,
 * the clock of Python's time.monotonic). */
fsa_status fsa_server_clock(double* t);

fsa_status fsa_server_poll(fsa_server s, uint64_t ticket, int* done, fsa_status* result);
/* Blocks until the request has finished; *result receives its status. */
fsa_status fsa_server_wait(fsa_server s, uint64_t ticket, fsa_status* result);
/* As fsa_server_wait for at most timeout_ms (< 0: no limit): *done = 1 and
 * *result set if the request finished, *done = 0 if the time ran out (the
 * request stays queued or in flight; fsa_server_cancel drops a queued one). */
fsa_status fsa_server_wait_for(fsa_server s, uint64_t ticket, double timeout_ms, int* done,
                               fsa_status* result);
/* Cancels a request that has not been launched yet (FSA_ESTATE otherwise). */
fsa_status fsa_server_cancel(fsa_server s, uint64_t ticket);
/* Requests still queued (not launched) timeout_ms after their arrival finish
 * with FSA_ETIMEDOUT, so that a burst beyond the device's rate sheds load
 * instead of growing the queue without bound; 0 (the default) or less: no
 * limit.  A launched request always runs to completion (a kernel is not
 * preempted).  Checked whenever the queue is pumped (submissions and
 * completions) or a request is polled or waited for.  A device error
 * reported by a request's completion event fails that request with
 * FSA_EDEVICE; a fault that ends the device context fails every later one
 * the same way. */
fsa_status fsa_server_set_queue_timeout(fsa_server s, double timeout_ms);
fsa_status fsa_server_stats(fsa_server s, fsa_stats* out);
/* Starts a new statistics window: clears latency samples, counters and the
 * HBM peak; cached tensors and queued or in-flight requests are kept. */
fsa_status fsa_server_reset_stats(fsa_server s);
/* Waits for in-flight work, then frees the cache and the server. */
fsa_status fsa_server_destroy(fsa_server s);

/* Message of the last failure on the calling thread; valid until the next
 * call on that thread. */
const char* fsa_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FSA_H */
