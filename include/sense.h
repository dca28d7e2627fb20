/*
 * sense.h - C ABI of the MI355X (gfx950) CG-SENSE library.
 *
 * Multicoil Cartesian MRI encoding on one GPU:
 *
 *   E     y_c = M .* F(S_c .* x)                  forward model, per coil c
 *   E^H   x   = sum_c conj(S_c) .* F^H(M .* y_c)   adjoint
 *   A     q   = E^H E p + lambda p                 normal operator
 *   CG    conjugate gradients on A x = E^H y from x = 0 (CG-SENSE)
 *
 * F is the centred unitary DFT over the image axes (x = readout, y and z =
 * phase encodes): F = n^(-1/2) fftshift . DFT . ifftshift per axis, with the
 * forward direction exp(-2 pi i k n / N) taking images to k-space.  M is a
 * binary sampling mask over the phase-encode axes that broadcasts along x.
 * With M = 1, E^H is the reconstruction equation of the paper (arXiv
 * 1807.11830, Section "Sensitivity-weighted multicoil image reconstruction",
 * Eq. (1)): inverse transform of each coil image, product with the conjugate
 * sensitivity map, sum over the coils of a frame; the unitary inverse here
 * carries n^(-1/2) where an unscaled inverse DFT with 1/n would carry 1/n.
 *
 * Operator model (Section "Algorithm handling" and the discussion after the
 * reconstruction listings): every operation has inputs, outputs and
 * parameters, and its once-only initialisation (here: plan creation, which
 * validates sizes, builds twiddle and mask tables and allocates workspace)
 * is split from the launch (the apply calls, which only enqueue kernels).
 * Chained operations pass device buffers without copies.
 *
 * Conventions that hold for every call:
 *  - Layouts are row-major with x fastest, complex values interleaved
 *    (re, im):  x [B][Nz][Ny][Nx],  y [B][C][Nz][Ny][Nx],
 *    maps [B or 1][C][Nz][Ny][Nx]; 2D problems have Nz = 1 and ndim = 2.
 *  - complex64 = two float32; SENSE_BF16X2 / SENSE_FP16X2 = two 16-bit
 *    values (re at the lower address).  x, p, q are always complex64.
 *  - Pointers named d_* are device pointers on the plan's device, owned by
 *    the caller.  Pointers named h_* are host memory.  Device buffers of
 *    maps, images and k-space must be 16-byte aligned (the kernels use
 *    16-byte vector accesses), d_info and d_rho_hist 8-byte aligned; every
 *    allocation of the HIP runtime or of torch is, and so is every batch or
 *    coil slab of one, since each slab of a supported size is a multiple of
 *    16 bytes.  A misaligned pointer fails with SENSE_ERR_INVALID.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).
 *    Apply and solve calls are asynchronous: they enqueue work on the
 *    stream and return; results are valid once the stream is synchronised.
 *    They never allocate memory.  The calls of one plan share its
 *    workspace: calls of one plan on different streams must be ordered by
 *    the caller (events or synchronisation), or they race.  Different plans
 *    are independent.
 *  - Errors: every call returns a sense_status; on failure nothing is
 *    enqueued and sense_last_error() returns a message for the calling
 *    thread.  No C++ exception crosses this boundary.
 */
#ifndef SENSE_H
#define SENSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SENSE_API __attribute__((visibility("default")))
#else
#define SENSE_API
#endif

typedef struct sense_plan_s* sense_plan;

typedef enum {
  SENSE_OK = 0,
  SENSE_ERR_INVALID = 1,     /* bad argument: null pointer, bad size, aliasing */
  SENSE_ERR_UNSUPPORTED = 2, /* valid request outside what the library implements */
  SENSE_ERR_NOMEM = 3,       /* device allocation failed at plan creation */
  SENSE_ERR_DEVICE = 4,      /* a HIP runtime call or kernel launch failed */
  SENSE_ERR_STATE = 5        /* call not allowed in the plan's current state */
} sense_status;

typedef enum {
  SENSE_C64 = 0,    /* complex64: float32 re, float32 im */
  SENSE_BF16X2 = 1, /* bfloat16 re, bfloat16 im; converted to fp32 on load, RNE on store */
  SENSE_FP16X2 = 2  /* float16 re, float16 im; converted to fp32 on load, RNE on store */
} sense_storage;

/* CG stop reasons, one per batch element. */
typedef enum {
  SENSE_CG_MAXITER = 0,   /* ran max_iter iterations */
  SENSE_CG_CONVERGED = 1, /* sqrt(rho_k / rho_0) < rel_tol after an update */
  SENSE_CG_EXACT = 2,     /* rho_k == 0 at the start of an iteration */
  SENSE_CG_BREAKDOWN = 3, /* Re<p, A p> <= 0 */
  SENSE_CG_NONFINITE = 4  /* a reduction produced Inf or NaN */
} sense_cg_status;

typedef struct {
  int32_t ndim;           /* 2 or 3 */
  int64_t nx, ny, nz;     /* image size; nz = 1 when ndim = 2 */
  int32_t ncoils;         /* C >= 1 */
  int32_t batch;          /* B >= 1 independent problems */
  int32_t maps_storage;   /* sense_storage of the sensitivity maps */
  int32_t kspace_storage; /* sense_storage of k-space y */
  int32_t maps_shared;    /* 1: one [C][...] map set serves every batch element */
  int32_t kspace_compact; /* 0: full grid [B][C][Nz][Ny][Nx]; 1: sampled lines
                             only, [B][C][L][Nx] with the L sampled (z, y)
                             lines in increasing z * Ny + y order */
} sense_desc;

/* Per batch element result of sense_cg_solve (24 bytes). */
typedef struct {
  int32_t iters_run; /* completed updates of x */
  int32_t status;    /* sense_cg_status */
  double rho0;       /* <b, b>, b = E^H y */
  double rho_final;  /* <r, r> when the loop stopped */
} sense_cg_info;

/*
 * Device bytes a plan for this descriptor allocates (tables, workspace and
 * CG vectors), so a scheduler can admit work by memory footprint.  Returns 0
 * for an invalid or unsupported descriptor.
 */
SENSE_API size_t sense_plan_device_bytes(const sense_desc* desc);

/*
 * Create a plan on the current HIP device (the paper's init step).
 *   desc    sizes and storage formats (copied).
 *   d_maps  sensitivity maps in desc->maps_storage, layout as above.  The plan
 *           borrows the pointer: the buffer must stay valid and unchanged
 *           while the plan is used.
 *   h_mask  uint8 host array of Nz*Ny entries in centred order ([Nz][Ny],
 *           DC at index (Nz/2, Ny/2)); nonzero = sampled.  Copied.
 *   stream  stream used for the table uploads (synchronised before return).
 *   out     receives the plan.
 * Supported: ndim = 2 or 3; Ny (and Nz in 3D) from {8, 16, 32, 48, 64, 80,
 * 96, 128, 160, 192, 256, 320, 384}; Nx from the same set for E, E^H and
 * CG, while the normal operator alone accepts any Nx >= 1; one image must
 * be below 2^31 bytes.  Other sizes -> SENSE_ERR_UNSUPPORTED.
 */
SENSE_API sense_status sense_plan_create(const sense_desc* desc, const void* d_maps, const uint8_t* h_mask,
                               void* stream, sense_plan* out);

/*
 * Rebind the plan to another sensitivity-map buffer of the same layout and
 * storage (for pooled plans in a server: sizes and mask stay, maps change).
 * Drops the captured solve graph.  Not allowed while the plan is in an
 * engine slot.
 */
SENSE_API sense_status sense_plan_set_maps(sense_plan plan, const void* d_maps);

/* Release a plan and its device memory (synchronises the device first). */
SENSE_API sense_status sense_plan_destroy(sense_plan plan);

/*
 * Forward operator: d_y[B][C][Nz][Ny][Nx] (kspace_storage) = E d_x.
 * Unsampled locations are written as zeros (full grid) or not stored at all
 * (kspace_compact: d_y is [B][C][L][Nx]).  d_x complex64 [B][...].
 * d_x and d_y must not overlap.
 */
SENSE_API sense_status sense_apply_E(sense_plan plan, const void* d_x, void* d_y, void* stream);

/*
 * Adjoint operator: d_x[B][...] (complex64) = E^H d_y.  The mask is applied
 * to d_y again, so values of d_y at unsampled locations are ignored, and
 * d_y is never modified.  d_x and d_y must not overlap.
 */
SENSE_API sense_status sense_apply_EH(sense_plan plan, const void* d_y, void* d_x, void* stream);

/*
 * Root-sum-of-squares reconstruction (the paper's RSS, Section "Performance
 * comparison with other frameworks"): d_img[b] = sqrt( sum_c |F_c^H (M .*
 * y_c)|^2 ), real float32 [B][Nz][Ny][Nx], no sensitivities.  With the
 * plan's mask applied to y it is the zero-filled RSS; a fully sampled plan
 * gives the paper's fully sampled reconstruction.  d_y is never modified;
 * d_img and d_y must not overlap.
 */
SENSE_API sense_status sense_apply_rss(sense_plan plan, const void* d_y, float* d_img, void* stream);

/*
 * Normal operator: d_q = E^H E d_p + lambda d_p, complex64 [B][...].
 * Computed in one fused pass per column (readout transforms cancel).
 * d_p and d_q must not overlap.
 */
SENSE_API sense_status sense_apply_EHE(sense_plan plan, const void* d_p, void* d_q, double lambda,
                             void* stream);

/*
 * CG-SENSE on (E^H E + lambda I) x = E^H y, one independent problem per
 * batch element, starting from x = 0.  Per iteration: q = A p,
 * alpha = rho / Re<p, q>, x += alpha p, r -= alpha q, rho' = <r, r>,
 * beta = rho' / rho, p = r + beta p.  Inner products, alpha and beta are
 * fp64 and stay on the device; vectors are complex64.
 *   d_y        k-space [B][C][...] in kspace_storage.
 *   d_x        output image [B][...] complex64 (must not overlap d_y).
 *   max_iter   >= 0 iterations at most.
 *   rel_tol    stop when sqrt(rho'/rho_0) < rel_tol (0 disables).
 *   lambda     Tikhonov weight (0 = plain CG-SENSE).
 *   d_info     optional device array of B sense_cg_info (NULL = skip); the
 *              plan also keeps the last result for sense_plan_cg_info.
 *   d_rho_hist optional device array [B][max_iter + 1] of fp64 rho_k
 *              (entries past the stop iteration are left untouched).
 * 2D slices of at most 64 columns with Ny in {8, 16, 32, 48, 64} and one
 * coil group run the whole loop in one launch after E^H y (one workgroup
 * per batch element, vectors in registers, block reductions); larger
 * problems run one fused launch per iteration.  Both follow the loop above.
 */
SENSE_API sense_status sense_cg_solve(sense_plan plan, const void* d_y, void* d_x, int32_t max_iter,
                            double rel_tol, double lambda, sense_cg_info* d_info,
                            double* d_rho_hist, void* stream);

/*
 * The same CG-SENSE solve without a plan, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Every table and work vector of the
 * solve lives in one static device array of 64 MiB per GPU (held from the
 * library's load on that GPU until the process ends); the call allocates
 * nothing and enqueues: a few small table-copy kernels (the tables travel
 * in kernel arguments), E^H y, the iterations and the final test, on
 * stream.  Results equal those of sense_cg_solve on a plan with the same
 * descriptor, maps and mask.
 *   desc, d_maps, h_mask   as for sense_plan_create (d_maps only borrowed
 *                          for the call; h_mask read during the call).
 *   d_y, d_x, max_iter, rel_tol, lambda, d_info, d_rho_hist
 *                          as for sense_cg_solve.
 * Limits: ndim = 2, nx a supported length, and the plan workspace
 * sense_plan_device_bytes(desc) at most 64 MiB; larger problems return
 * SENSE_ERR_UNSUPPORTED (use a plan).  All calls on one GPU share its
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race and must be serialised by the caller.  The array keeps the last
 * call's contents; each call initialises everything it reads.
 */
SENSE_API sense_status sense_cg_solve_static(const sense_desc* desc, const void* d_maps, const uint8_t* h_mask,
                                             const void* d_y, void* d_x, int32_t max_iter, double rel_tol,
                                             double lambda, sense_cg_info* d_info, double* d_rho_hist,
                                             void* stream);

/*
 * Graph replay of whole solves (default on).  The first sense_cg_solve with a
 * given argument set (d_y, d_x, max_iter, rel_tol, lambda, d_info,
 * d_rho_hist) captures every kernel of the solve into a HIP graph on a
 * private stream; later calls with the same arguments replay it on the
 * caller's stream with one launch.  Different arguments re-capture.  While
 * profiling is enabled solves run eagerly, and so do the solves of slices
 * that run whole in one workgroup (at most 64 x 64 with one coil group:
 * two launches, where a graph launch costs more than it saves).  The
 * mask never changes for a plan and new maps drop the graph, so a replay
 * computes exactly what the eager launches do.
 */
SENSE_API sense_status sense_plan_set_graphs(sense_plan plan, int32_t enable);

/*
 * Coil groups of the 2D normal operator.  The fused kernel runs one block
 * per (column tile, batch element); when there are too few of those to fill
 * the GPU, the plan splits the coils into G contiguous groups, one block per
 * group, and a combine pass adds the G partial coil sums in group order.
 * The E^H column pass and RSS split the same way (their own combine).
 * The plan sizes its workspace at creation for the fill split Gmax (1 when
 * tiles x batch >= 512, else ceil(512 / (tiles x batch)) capped at coils / 2
 * and 16) and starts at G = Gmax, or at G = 1 when a slice has fewer than
 * 8192 voxels (there the combine pass costs more than the split saves).
 *   sense_plan_set_coil_groups: groups = 0 restores the plan's defaults;
 *     1 <= groups <= Gmax sets G for all of them (1 = no split).
 *     Larger values return SENSE_ERR_UNSUPPORTED.  Results depend on G only
 *     through the order of the coil sum (deterministic for a given G).
 *   sense_plan_coil_groups: the current G of E^H E and CG and the largest
 *     allowed (either output may be NULL).
 * 3D plans always use one group.
 */
SENSE_API sense_status sense_plan_set_coil_groups(sense_plan plan, int32_t groups);
SENSE_API sense_status sense_plan_coil_groups(sense_plan plan, int32_t* groups, int32_t* max_groups);

/* Copy the last sense_cg_solve result of every batch element to host memory
 * h_info[B]; synchronises the stream. */
SENSE_API sense_status sense_plan_cg_info(sense_plan plan, sense_cg_info* h_info, void* stream);

/*
 * Stage timing (the paper's per-launch profile parameters).  When enabled,
 * every fused E^H E launch is bracketed by HIP events on its stream; after
 * the stream is synchronised sense_plan_profile returns the number of timed
 * launches and their total duration in milliseconds, then clears the record.
 */
SENSE_API sense_status sense_plan_set_profiling(sense_plan plan, int32_t enable);
SENSE_API sense_status sense_plan_profile(sense_plan plan, int64_t* n_launches, double* total_ms);

/*
 * Serving engine: continuous batching of independent single-slice solves.
 *
 * A slot table holds the solves in flight.  Each request brings its own plan
 * (ndim 2, batch 1; maps, mask and sizes may differ between requests), its
 * k-space d_y and output image d_x.  Admission needs a free slot and
 * footprint_bytes (what the caller counts for this request: plan plus its
 * buffers) within the remaining budget; otherwise it returns
 * SENSE_ERR_STATE and the caller retries after poll has freed slots.  The
 * running slots form groups by (ny, maps storage, maps staging); a step
 * advances the slots of every group that is not already two steps ahead by
 * one CG iteration with one batched launch of the fused iteration (and,
 * where a problem splits its coils, one combine launch) per group, and
 * returns (when every group is two steps ahead it first waits until one is
 * not).  Each group runs on a stream (lane) of its own, so groups of small
 * slices are not held to the pace of groups of large ones.  Each problem
 * uses its own CG state, coil groups and reduction order, so its result is
 * bitwise the same as sense_cg_solve alone.  Requests admitted between steps
 * join at their group's next step; a small slice that sense_cg_solve runs in
 * one launch runs its whole solve at admission instead.  poll returns the
 * slots whose solves are complete (d_x written; sense_plan_cg_info gives the
 * info) and frees them.  The engine owns its streams: admissions run on its
 * own stream, and a lane waits for the latest admission before the first
 * step of a newly joined slot (sense_engine_sync waits for all streams).  A
 * plan in a slot must not be used or destroyed until its slot is polled.
 * All calls come from one host thread.
 */
typedef struct sense_engine_s* sense_engine;

SENSE_API sense_status sense_engine_create(size_t budget_bytes, int32_t max_slots, sense_engine* out);
SENSE_API sense_status sense_engine_destroy(sense_engine engine);
/*
 * Admit one solve.  stream is the caller's stream on which d_y was produced
 * and d_x was last used (NULL = the null stream): the engine's own stream
 * waits for everything enqueued there before this admission, so the solve
 * never reads k-space that is still being written.  The wait covers only
 * work enqueued before the call.  Results are in d_x once poll reports the
 * slot; the caller may then read them on any stream.  d_y and d_x must stay
 * allocated (and must not be reused) until then, or until the engine is
 * destroyed, which waits for its streams.
 */
SENSE_API sense_status sense_engine_admit(sense_engine engine, sense_plan plan, const void* d_y, void* d_x,
                                          int32_t max_iter, double rel_tol, double lambda,
                                          size_t footprint_bytes, void* stream, int32_t* slot);
SENSE_API sense_status sense_engine_step(sense_engine engine, int32_t* n_running);
SENSE_API sense_status sense_engine_poll(sense_engine engine, int32_t* done_slots, int32_t max_done,
                                         int32_t* n_done);
SENSE_API sense_status sense_engine_stats(sense_engine engine, size_t* used_bytes, size_t* budget_bytes,
                                          int32_t* active, int64_t* steps);
/* Wait for everything the engine has enqueued. */
SENSE_API sense_status sense_engine_sync(sense_engine engine);

/* Message of the last failed call on this thread ("" if none). */
SENSE_API const char* sense_last_error(void);

/* Library version string. */
SENSE_API const char* sense_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SENSE_H */
