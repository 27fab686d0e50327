/*
 * rl.h -- C ABI of the MI355X Richardson-Lucy library (librl.so).
 *
 * The library solves the non-blind deconvolution problem "given the blurred image f and
 * the point-spread function h, find u with f ~ u*h" (Section 1, eq. 2) by Richardson-Lucy
 * iteration (Section 2, eq. 3):
 *
 *     u^0 = f,    u^{k+1} = (h^* * (f / (u^k * h))) . u^k
 *
 * where h^* is h reflected about the origin, so h^* * r is the correlation of r with h.
 * Every step of every iteration runs in the library's own HIP kernels on the GPU.
 *
 * Conventions used by every call below
 * ------------------------------------
 *  Images   row-major float32, height x width, pitch = width, pixel (y, x) at y*width + x.
 *  PSF      row-major float32 psf_h x psf_w in HOST memory, origin at
 *           (psf_h / 2, psf_w / 2); tap h[i][j] sits at offset (i - psf_h/2, j - psf_w/2).
 *             (u*h)(y,x)   = sum_ij h[i][j] u[fold(y-(i-oy))][fold(x-(j-ox))]
 *             (h^* * r)(y,x) = sum_ij h[i][j] r[fold(y+(i-oy))][fold(x+(j-ox))]
 *  Ratio    r = f / v where v = u^k*h > 0, else r = 0.
 *  Boundary missing pixels are replaced by image pixels (Section 2, "Boundary treatment"):
 *             RL_BC_REFLECT   half-sample symmetric continuation (c b a | a b c), period 2N
 *             RL_BC_REPLICATE the closest image pixel (the paper's rule)
 *           Both fold to any depth, so PSFs larger than the image are allowed.
 *  Memory   The caller owns every buffer.  Device pointers (f, u0, u_out, workspace, state
 *           buffers) must come from hipMalloc (or torch) on the current HIP device.  The
 *           library never allocates device memory: all per-job device state lives in the
 *           caller's workspace, whose size rl_workspace_bytes() reports exactly.
 *  Streams  Every device operation of a job is enqueued on the hipStream_t given in
 *           rl_params.stream (NULL = the null stream).  Calls return before the GPU work
 *           finishes unless stated otherwise.
 *  Errors   Every call returns an rl_status; nothing is thrown across the ABI.  After
 *           RL_E_DEVICE the job must be destroyed.
 *  Threads  One host thread at a time per job; distinct jobs are independent.
 *  Determinism  The same inputs give bit-identical results, alone or batched.
 */
#ifndef RL_H
#define RL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rl_status;
#define RL_OK 0
#define RL_E_INVAL (-1)       /* bad argument: sizes, PSF, workspace, f, call arguments  */
#define RL_E_NOMEM (-2)       /* workspace too small                                      */
#define RL_E_DEVICE (-3)      /* a HIP runtime call failed                                */
#define RL_E_STATE (-4)       /* call not allowed in this state (e.g. after destroy)      */
#define RL_E_UNSUPPORTED (-5) /* valid request the library does not serve                 */

/* boundary continuation */
#define RL_BC_REFLECT 0
#define RL_BC_REPLICATE 1

/* convolution path (Section 3): which operator family evaluates u*h and h^* * r */
#define RL_PATH_AUTO 0     /* chosen from the PSF by the PSF compiler                      */
#define RL_PATH_DIRECT 1   /* per-tap sum over the non-zero taps (naive / list filter)     */
#define RL_PATH_BOX_AXIS 2 /* 1 x L or L x 1 uniform box: sliding window (Section 3)       */
#define RL_PATH_RUNS 3     /* per-row runs: sliding for uniform runs (generic box filter),
                              register-blocked spans for non-uniform rows (list filter)    */
#define RL_PATH_BOX_RECT 4 /* kh x kw uniform rectangle (kh, kw >= 2): separable sliding
                              sums, rows then columns, on an LDS tile (2-D box filter,
                              Section 3); constant work per pixel in kh and kw            */
#define RL_PATH_BOX_SAT 5  /* the same rectangles from 2-D cumulated sums (Section 3, the
                              summed-area variant of the 2-D box filter): each window sum
                              from four corners of a table built per LDS tile in FP64, with
                              an exact integer count of non-zero inputs; constant work per
                              pixel; RL_E_UNSUPPORTED when the tile's tables exceed LDS   */
#define RL_PATH_MFMA 6     /* PSFs with dense lines (the list filter, Section 3, as matrix
                              products): each PSF row, at most 17 taps wide (at most 64
                              rows), is a banded matrix applied to 16 x 16 output blocks on
                              the matrix cores; values and weights are split into three
                              bfloat16 parts whose six leading products keep float32
                              accuracy; float32 accumulation.  AUTO picks it where it is
                              cheaper than the register-blocked spans (dense PSFs); not for
                              the fused or persistent schedule                            */

/* iteration schedule: how the per-iteration kernels are organised */
#define RL_SCHED_AUTO 0
#define RL_SCHED_TWO_PASS 1 /* conv+ratio kernel, then corr+update kernel, per iteration   */
#define RL_SCHED_RESIDENT 2 /* BOX_AXIS only: independent lines held on chip for all
                               iterations of one rl_iterate call                           */
#define RL_SCHED_FUSED 3    /* one kernel per iteration: conv, ratio, corr and update on an
                               LDS tile with a double halo (u double-buffered); plain jobs
                               with height, width >= 64 and PSF extents <= 63 only         */
#define RL_SCHED_PERSISTENT 4 /* one launch per rl_iterate call running both phases of
                               every iteration, tiles synchronised through per-tile step
                               counters; plain RL on the span and sliding kernels (strips
                               of 4 or 8) only, else RL_E_UNSUPPORTED.  Inside
                               rl_iterate_batch such jobs run on the two-pass kernels.   */

/* thinning (Section 4) */
#define RL_THIN_OFF 0
#define RL_THIN_ABS 1 /* frozen when |u^{k+1} - u^k| < tau        (the paper's rule)   */
#define RL_THIN_REL 2 /* frozen when |u^{k+1} - u^k| < tau * u^k  (relative variant)   */

typedef struct rl_thin {
    int32_t mode;           /* RL_THIN_*                                                  */
    float tau;              /* threshold, > 0 to freeze anything                          */
    int32_t hysteresis;     /* H: frozen after H consecutive tests below tau (H >= 1)     */
    int32_t reset_period;   /* R: iteration k is full when k == 0 or k % R == 0; 0 = never */
    int32_t compact_period; /* C: the active list is rebuilt after each full step and when
                               (k - 1) % C == 0                                           */
    int32_t keep_list;      /* 1: also build the per-pixel active list at every rebuild
                               (exported by rl_active_list); 0: only the tile list that
                               distributes the work is built                              */
    int32_t block;          /* 0 or 1: the per-pixel rule of Section 4 (eq. 4-5).  8, 16,
                               32 or 64: the block rule, a refinement of Section 4's
                               adaptive update rule: the image is cut into block x block
                               squares aligned at (0, 0) (cut by the image edge), each with
                               one counter; a block counts up when the test above holds for
                               every one of its pixels and restarts at 0 otherwise, and
                               every pixel of an active block is updated (frozen blocks
                               keep u and r; active neighbours read their stale r).  The
                               counters exchanged by rl_get_state / rl_set_state stay per
                               pixel: every pixel carries its block's counter, and on input
                               a block takes the counter of its top-left pixel.  The
                               tiled kernels then run 64 x 64 tiles (strip 8); the other
                               values give RL_E_INVAL                                     */
} rl_thin;

/* Kernel-shape and launch knobs (0 = let the library choose).  Results do not depend on
 * them beyond float32 rounding order (graph_iters: not at all).  strip: outputs per lane of
 * the tiled kernels (4, 8, 16 or 32); seg: pixels per lane of the resident solver (2..32,
 * power of two); lines_per_wg: image lines per workgroup of the resident solver;
 * graph_iters: plain two-pass jobs capture this many iterations into a hipGraph once and
 * replay it from rl_iterate (0: launch kernels directly). */
typedef struct rl_tuning {
    int32_t strip, seg, lines_per_wg, graph_iters;
} rl_tuning;

typedef struct rl_params {
    int32_t height, width;  /* image size, both >= 1                                      */
    const float *f;         /* DEVICE, height*width, >= 0 and finite; copied at rl_init   */
    int32_t psf_h, psf_w;   /* PSF size, each in [1, 127]                                 */
    const float *psf;       /* HOST, psf_h*psf_w, >= 0, finite, positive sum; copied      */
    const float *u0;        /* DEVICE initial estimate or NULL for u^0 = f; copied        */
    int32_t boundary;       /* RL_BC_*                                                    */
    int32_t path;           /* RL_PATH_*                                                  */
    int32_t schedule;       /* RL_SCHED_*                                                 */
    int32_t kahan;          /* 1: per-row partial sums combined with Kahan compensation
                               and compensated running sums; 0: plain float32 sums        */
    rl_thin thin;           /* thinning; mode RL_THIN_OFF disables it                     */
    void *stream;           /* hipStream_t for every device operation of the job          */
    rl_tuning tuning;       /* kernel-shape knobs, zero-initialise for defaults           */
    /* Total-variation regularisation (the regularised RL the paper names as carrying its
     * optimisations over, Section 2; the variant of Dey et al.): the update becomes
     * u^{k+1} = u^k . c / (1 - tv_lambda * div(grad u^k / sqrt(|grad u^k|^2 + tv_eps^2)))
     * with a forward-difference gradient (0 across the last column / row) and a
     * backward-difference divergence (no flux before the first column / row).
     * tv_lambda = 0 disables it; else 0 < tv_lambda < 0.25 (keeps the denominator > 0)
     * and tv_eps > 0.  Not combined with thinning, the resident or the fused schedule
     * (RL_E_UNSUPPORTED).                                                                */
    float tv_lambda;
    float tv_eps;
    /* Robustified data term (the paper names robust RL variants among the methods its
     * optimisations carry over to, Section 2): rob_eps > 0 turns the update into
     *   u^{k+1} = u^k . (h^* * (w f / v)) / (h^* * w),   v = u^k * h,
     *   w = 1 / sqrt(d + rob_eps^2),  d = v - f - f ln(v / f)  (I-divergence; d = v where
     *   f = 0; d = 0 and w f / v = 0 where v <= 0),
     * i.e. a square-root penaliser of the I-divergence.  Each iteration runs the forward
     * sum, an elementwise weight pass and two correlations.  rob_eps = 0 disables it; not
     * combined with TV, thinning, the resident or the fused schedule (RL_E_UNSUPPORTED).  */
    float rob_eps;
} rl_params;

typedef struct rl_stats {
    int64_t iters_done;       /* k: iterations applied so far                             */
    int64_t active_now;       /* pixels active in the next iteration (N without thinning) */
    int64_t skipped_px_iters; /* sum over iterations of (N - |A_k|)                       */
    double flux;              /* sum of u^k, reduced on the GPU in FP64 in a fixed order  */
    int32_t path;             /* RL_PATH_* actually used                                  */
    int32_t schedule;         /* RL_SCHED_* actually used                                 */
    int32_t f_invalid;        /* 1 if f had a negative or non-finite value                */
    int32_t reserved;
} rl_stats;

typedef struct rl_job rl_job;

/* Status name, e.g. "RL_E_INVAL".  Never NULL. */
const char *rl_status_str(rl_status s);

/* Text of the reason the last failing call on this thread gave (empty if it gave none),
 * e.g. why a path does not apply to a PSF or why a workspace is too small.  Never NULL;
 * valid until the next library call on this thread. */
const char *rl_last_error(void);

/*
 * Exact number of device bytes rl_init needs for these parameters: the planes of eq. 3
 * (f, u^k and the ratio r = f / (u^k * h), Section 2), the compiled PSF (Section 3),
 * the thinning state of Section 4 (counters, active lists), reduction scratch.  Pure host
 * computation.  Returns RL_E_INVAL for invalid sizes or PSF (PSF values are read from
 * p->psf).
 */
rl_status rl_workspace_bytes(const rl_params *p, size_t *bytes);

/*
 * Set up one problem f ~ u*h (Section 1, eq. 2) for RL iteration from u^0 = f (Section 2,
 * eq. 3): validate p, compile the PSF (host, Section 3), and enqueue on p->stream: the
 * upload of the compiled PSF, the copy of f (and u0) into the workspace, and zeroing of
 * the thinning state (Section 4).
 * ws: caller-owned device buffer of ws_bytes >= rl_workspace_bytes(p), 256-byte aligned;
 * it must stay alive and untouched until rl_destroy.  f's sign and finiteness are checked
 * on the GPU; the outcome is reported by rl_result (RL_E_INVAL) and in rl_stats.f_invalid.
 * On success *out receives a new job handle (host memory owned by the library).
 * The upload goes through pinned host buffers that the library allocates on first need,
 * reuses once their copies have completed and keeps until the process ends (at most
 * 256 MiB in all, then pageable copies), so that rl_init does not wait for work already
 * on the stream; rl_iterate_batch uploads its tables the same way.
 * Errors: RL_E_INVAL (sizes, PSF, NULL pointers, path not applicable to the PSF),
 * RL_E_NOMEM (ws_bytes too small), RL_E_DEVICE.
 */
rl_status rl_init(const rl_params *p, void *ws, size_t ws_bytes, rl_job **out);

/* Enqueue n_iter >= 0 further RL iterations (Section 2, eq. 3; thinned per Section 4 when
 * p->thin.mode != RL_THIN_OFF).  Asynchronous.  Every path returns exactly 0 for a window
 * whose inputs are all 0 (so r = 0 where v = 0, and u^{k+1} = 0 where c = 0), also the
 * sliding ones, which count the non-zero inputs of such windows exactly. */
rl_status rl_iterate(rl_job *job, int32_t n_iter);

/*
 * The result of the iteration (Section 2, eq. 3; Section 4, eq. 4-5 when thinned): enqueue
 * a device-to-device copy of u^k into u_out (height*width floats, may be NULL to skip).
 * If st is non-NULL, also reduce the statistics on the GPU, synchronise the job's stream
 * and fill *st.  Returns RL_E_INVAL if f was found invalid (only known once the stream has
 * been synchronised, i.e. when st != NULL).  A job that has run the persistent schedule
 * also synchronises the stream without st, to read its launches' abort flag: RL_E_DEVICE
 * if a launch gave up waiting (u^k is then incomplete).
 */
rl_status rl_result(rl_job *job, float *u_out, rl_stats *st);

/* Release the host handle.  The workspace stays with the caller.  Never fails on a valid
 * handle; the handle is invalid afterwards.  Does not synchronise. */
rl_status rl_destroy(rl_job *job);

/*
 * Allocation-free solve, for callers that cannot allocate device memory: tight serving
 * loops and harnesses that forbid hipMalloc.  One call does what rl_init, rl_iterate(n_iter),
 * rl_result(u_out, st) and rl_destroy do for p, on p->stream, except that the job's
 * workspace is a library-owned static device array of RL_STATIC_SCRATCH_BYTES on the
 * current HIP device instead of a caller's buffer.  It calls no hipMalloc, hipFree or
 * hipHostMalloc and creates no stream, event or graph (host-side bookkeeping uses ordinary
 * heap memory; keep kernel timing off, which creates events).  p->f, p->u0 and u_out
 * (may be NULL) are caller-owned device buffers as for rl_init / rl_result; st may be NULL.
 * Synchronises p->stream before returning.  Each device holds one array for the life of
 * the process; calls on one device share it and are serialised by the library (a call
 * holds the device's lock until its GPU work has finished); the array keeps the last
 * call's contents and each call clears what it needs zeroed.
 * Errors: RL_E_NOMEM if rl_workspace_bytes(p) > RL_STATIC_SCRATCH_BYTES (nothing is
 * enqueued); RL_E_UNSUPPORTED if p->tuning.graph_iters != 0; otherwise as rl_init,
 * rl_iterate and rl_result (RL_E_INVAL also for n_iter < 0 or an invalid f).
 */
#define RL_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
rl_status rl_solve_static(const rl_params *p, int32_t n_iter, float *u_out, rl_stats *st);

/*
 * Batched iteration of uneven jobs (different sizes, PSFs, iteration counts, thinning).
 * Enqueues n_iter[j] >= 0 further iterations of every job j on `stream` (hipStream_t;
 * the caller orders it against the jobs' own streams).  Jobs on the tiled two-pass
 * schedule are grouped by kernel variant; each batch iteration then runs ONE launch per
 * phase and group, covering the tiles of every job of the group that still has
 * iterations left (jobs are ordered by remaining iterations, so finished jobs drop out
 * of the grid).  Jobs on the resident schedule run all their iterations in one launch
 * each.  The per-group work tables (job descriptors and tile prefix sums) are copied into
 * the caller's batch workspace `bws` (device, 256-byte aligned) of at least
 * rl_batch_workspace_bytes(n_jobs) bytes; `bws` must not be reused by another call
 * before this one's work has started on the stream (the library waits for its own
 * previous upload into the same `bws`).  A job may appear at most once (RL_E_INVAL).
 * Results per job are bit-identical to rl_iterate on that job alone.
 * Streams: the kernel groups run concurrently on library-owned side streams (created once
 * per process at the default priority), forked from `stream` by an event before the first
 * launch and joined back into it by events after the last, so that all of the call's work
 * is ordered on `stream` as if it ran there; the caller supplies no other stream.
 */
rl_status rl_batch_workspace_bytes(int32_t n_jobs, size_t *bytes);
rl_status rl_iterate_batch(rl_job *const *jobs, const int32_t *n_iter, int32_t n_jobs,
                           void *bws, size_t bws_bytes, void *stream);

/*
 * Lock-step / checkpoint hooks (enqueued on the job's stream, asynchronous; rl_get_state
 * of a job that has run the persistent schedule synchronises to check the abort flag, as
 * rl_result does):
 *   rl_get_state copies u^k, the persistent ratio r (thinned mode keeps stale values of
 *   inactive pixels) and the per-pixel convergence counters out of the workspace, and
 *   writes k to *k_out (host).  Any of u, r, cnt may be NULL.
 *   rl_set_state copies them in and sets the iteration counter to k (so the thinning
 *   schedule continues from k).  NULL skips a buffer (r and cnt are then left as they are).
 * Buffers: u, r: height*width float32 (device); cnt: height*width uint8 (device).
 */
rl_status rl_get_state(rl_job *job, float *u, float *r, uint8_t *cnt, int64_t *k_out);
rl_status rl_set_state(rl_job *job, const float *u, const float *r, const uint8_t *cnt,
                       int64_t k);

/*
 * Thinned mode: the compacted active-pixel list of the last rebuild (ascending row-major
 * indices p with cnt[p] < hysteresis, Section 4), copied into list_dev (device int32,
 * capacity cap entries); *n receives the list length (synchronises the stream), or -1
 * if there is no list: no rebuild yet, or the job was created with thin.keep_list = 0.
 */
rl_status rl_active_list(rl_job *job, int32_t *list_dev, int64_t cap, int64_t *n);

/* Thinned mode: the number of active pixels |A_k| of the last min(k, cap, 4096)
 * iterations, oldest first, into out (host int64); *n receives the count.  Synchronises. */
rl_status rl_thin_schedule(rl_job *job, int64_t *out, int32_t cap, int32_t *n);

/*
 * PSF compiler (host only, no device work): classify the PSF and build its integer run
 * list -- per PSF row i ascending, maximal spans of consecutive columns with non-zero,
 * bit-identical weights (the representation behind the paper's generic box and list
 * filters, Section 3).  runs (int32, 3 per run): dy = i - oy, x0, x1 (column offsets
 * j - ox of the first and last tap); w: the float32 weight of each run.  *cls receives the
 * RL_PATH_* that RL_PATH_AUTO would choose.  Returns RL_E_NOMEM if cap < number of runs
 * (*n_runs is still set), RL_E_INVAL for an invalid PSF.
 */
rl_status rl_psf_runs(const float *psf, int32_t psf_h, int32_t psf_w, int32_t *runs,
                      float *w, int32_t cap, int32_t *n_runs, int32_t *cls);

/* Test hook for the failure path of the persistent schedule: the number of polls a
 * dependency wait of later persistent launches makes before the launch gives up (sets its
 * abort flag; every workgroup then leaves, so the kernel ends).  Default 1 << 20; a
 * negative value gives up at the first wait of every launch.  *previous (may be NULL)
 * receives the old value.  Process-wide. */
rl_status rl_debug_spin_limit(int32_t polls, int32_t *previous);

/* Kernel timing for measurement: while enabled, every kernel launch of every job is
 * bracketed by HIP events on the stream it is launched on.  rl_timing_read synchronises
 * on the recorded events and reports, for the kernel named `name`, the number of launches
 * and their summed duration in milliseconds; rl_timing_reset discards the records.  While
 * timing is on, rl_iterate_batch runs its kernel groups one after another on one stream
 * (not concurrently), so that each recorded duration is the launch's own and not the time
 * it shares the GPU with other groups; results are the same either way. */
rl_status rl_timing_enable(int32_t on);
rl_status rl_timing_read(const char *name, int64_t *launches, double *total_ms);
rl_status rl_timing_reset(void);

/*
 * Autotuner.  rl_autotune times every candidate kernel shape for these parameters on the
 * caller's data: strip length, two-pass or fused schedule and graph replay on/off for
 * the tiled kernels; segment length and lines per workgroup for the resident solver.
 * Each candidate runs n_iter untimed then n_iter timed iterations (HIP events on
 * p->stream; the call synchronises that stream) with p->f as data and `ws` (device,
 * >= rl_autotune_workspace_bytes(p) bytes, contents clobbered) as the job workspace.
 * A schedule other than RL_SCHED_AUTO in p is kept; path, boundary, thinning and kahan
 * are never changed.  The fastest pair (schedule, tuning) goes to *best_schedule / *best
 * (either may be NULL except best) and its milliseconds per iteration to *best_ms, and is
 * stored in the library's process-wide tuning cache under the key (path, PSF height and
 * width, taps, runs, round(log2(height*width)), thinning on/off, requested schedule).
 * From then on rl_workspace_bytes and rl_init with an all-zero p->tuning use the cached
 * pair for every job with that key -- so compute workspace sizes after tuning, since
 * rl_init rejects a workspace smaller than the configuration it picks.
 * rl_tune_lookup copies the cached pair for p (RL_E_STATE if there is none).
 * rl_tune_cache_save / _load write and merge the cache as text, one entry per line
 * (RL_E_INVAL on an unreadable file or a malformed line; a failed load changes nothing).
 * rl_tune_cache_clear empties it.  The cache is guarded by a mutex; tuning itself must
 * not overlap other work on p->stream that the timing would include.
 */
rl_status rl_autotune_workspace_bytes(const rl_params *p, size_t *bytes);
rl_status rl_autotune(const rl_params *p, void *ws, size_t ws_bytes, int32_t n_iter,
                      int32_t *best_schedule, rl_tuning *best, double *best_ms);
rl_status rl_tune_lookup(const rl_params *p, int32_t *schedule, rl_tuning *out);
rl_status rl_tune_cache_save(const char *path);
rl_status rl_tune_cache_load(const char *path);
rl_status rl_tune_cache_clear(void);

/* Describes the kernel configuration chosen for a job (for logs and tests):
 * path, schedule, tile height/width, strip length, spans, taps. */
typedef struct rl_job_info {
    int32_t path, schedule, tile_h, tile_w, strip, n_spans, n_taps, lmax;
    int32_t halo_y0, halo_y1, halo_x0, halo_x1;
    int64_t ws_bytes;
} rl_job_info;
rl_status rl_job_describe(rl_job *job, rl_job_info *info);

#ifdef __cplusplus
}
#endif
#endif /* RL_H */
