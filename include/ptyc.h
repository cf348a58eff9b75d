/*
 * ptyc — live ePIE ptychographic reconstruction on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the shared library libptyc.so.  Plain pointers and sizes only.
 *
 * The method is ePIE (extended ptychographical iterative engine, Maiden &
 * Rodenburg 2009) as used by the paper "Live Iterative Ptychography"
 * (Weber et al. 2023), section "ePIE Implementation": for every scan
 * position j, taken in a randomly shuffled order each iteration,
 *
 *   psi   = P * S_j O                       exit wave (S_j O: N x N window)
 *   Psi   = F psi                           unnormalised 2D DFT
 *   Psi'  = sqrt(I_j) * sgn(Psi)            modulus replacement, sgn(0) = 0
 *   psi'  = F^-1 Psi'                       (includes 1/N^2)
 *   S_j O += alpha conj(P) (psi' - psi) / max|P|^2
 *   P     += beta conj(S_j O) (psi' - psi) / max|S_j O|^2
 *
 * with both right-hand sides taken before the update, max|P|^2 over the whole
 * probe and max|S_j O|^2 over the position's window.  The section "Extensions
 * of the ePIE implementation" asks that diffraction patterns can be added
 * while the reconstruction runs and that it can be stopped, continued and
 * read out; the Discussion asks for import and export of object, probe and
 * data through an API and a geometry fixed in advance.  This interface
 * provides exactly that: init (fixed geometry), add_positions (data grows),
 * sweep (step the iteration), get/set of object and probe.
 *
 * Coloured mode.  Positions are grouped into batches whose N x N windows are
 * pairwise disjoint.  All positions of batch b are updated from the same
 * probe P_b (their object steps touch disjoint pixels and commute), and the
 * probe then moves by the batch mean of the increments:
 *   P_{b+1} = P_b + (beta / |B_b|) sum_{j in B_b} conj(S_j O) Delta_j / max|S_j O|^2.
 * A batch of one position is exactly the sequential update above.  Strict
 * mode runs every position as its own batch.
 *
 * Conventions
 *   - complex data are interleaved float32 pairs (re, im), row-major,
 *     i.e. the layout of torch.complex64 / numpy complex64.
 *   - positions are int32 pairs (row, col): the top-left corner of the
 *     position's N x N window in the object; 0 <= row <= H-N, 0 <= col <= W-N.
 *   - DFT sign convention exp(-2 pi i k.r / N) forward, DC at [0, 0]; the
 *     intensities are stored unshifted (or pass PTYC_I_CENTERED).
 *   - mem_kind PTYC_MEM_HOST: pointer to host memory; PTYC_MEM_DEVICE:
 *     pointer to device memory on the context's device.  The library copies
 *     every input; the caller keeps ownership of its buffers.
 *   - all device work is enqueued on the stream given at init (a hipStream_t,
 *     NULL for the default stream).  get_* and sweep with err_out
 *     synchronise that stream; nothing else blocks except add_positions,
 *     which waits for its own validation.
 *   - a context is used from one thread at a time.
 *
 * Errors: every call returns PTYC_OK (0) or a negative status.  Argument
 * errors are detected on the host before any device work and leave the
 * context unchanged.  After PTYC_ERR_HIP the context is poisoned: every call
 * except ptyc_destroy and ptyc_last_error returns PTYC_ERR_STATE.  Recovery
 * is destroy + init from the last get_object/get_probe + re-adding the data.
 */
#ifndef PTYC_H
#define PTYC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PTYC_OK 0
#define PTYC_ERR_ARG (-1)         /* invalid argument (null, size, non-power-of-two, overlap) */
#define PTYC_ERR_BOUNDS (-2)      /* a window would leave the object */
#define PTYC_ERR_OOM (-3)         /* device or pinned host allocation failed */
#define PTYC_ERR_HIP (-4)         /* a HIP runtime call failed; context poisoned */
#define PTYC_ERR_STATE (-5)       /* context poisoned by an earlier PTYC_ERR_HIP */

#define PTYC_MEM_HOST 0
#define PTYC_MEM_DEVICE 1

#define PTYC_MODE_STRICT 0        /* one position per batch: sequential ePIE */
#define PTYC_MODE_COLOURED 1      /* disjoint-window batches, batch-mean probe step */

#define PTYC_I_IS_SQRT 1u         /* add_positions receives sqrt(I) instead of I */
#define PTYC_I_CENTERED 2u        /* patterns arrive with DC at (N/2, N/2); shifted at ingest */

typedef struct ptyc_config {
    int32_t n;          /* pattern and probe side N: a power of two in [16, 256] */
    int32_t h, w;       /* object rows and columns, each >= n and <= 65536 */
    float alpha, beta;  /* object and probe update strengths (the paper uses 1, 1) */
    int32_t mode;       /* PTYC_MODE_STRICT or PTYC_MODE_COLOURED */
    int32_t max_batch;  /* coloured mode: cap on positions per batch; 0 means 1024 */
    uint64_t seed;      /* seeds the library's own per-sweep shuffle (order == NULL) */
    uint32_t flags;     /* PTYC_I_* bits */
    int32_t reserved;   /* must be 0 */
} ptyc_config;

typedef struct ptyc_ctx ptyc_ctx;

/* Create a context on the current HIP device with the geometry of cfg
 * (fixed for the context's life, as the paper fixes object size and the
 * pixel relation at initialisation, section "Determine parameters").
 * probe0: N*N complex64, object0: H*W complex64, both in mem_kind memory,
 * copied.  hip_stream: a hipStream_t or NULL.  On success *out receives the
 * context.  Errors: PTYC_ERR_ARG (null pointer, N not a power of two in
 * [16, 256], H or W < N or > 65536, bad mode/mem_kind, reserved != 0,
 * alpha/beta not finite), PTYC_ERR_OOM, PTYC_ERR_HIP (no usable device). */
int ptyc_init(ptyc_ctx** out, const ptyc_config* cfg, const void* probe0,
              const void* object0, int mem_kind, void* hip_stream);

/* Append `count` scan positions (indices n_loaded .. n_loaded+count-1, in
 * the given order) with their diffraction intensities, while the
 * reconstruction continues ("Extensions of the ePIE implementation").
 * pos_yx: count*2 int32 (row, col) window corners; intensities:
 * count raw frames of frame_h*frame_w float32 (N*N unless ptyc_set_ingest
 * says otherwise; photon counts, or sqrt when PTYC_I_IS_SQRT), both in
 * mem_kind memory.  All or nothing: PTYC_ERR_BOUNDS if a window leaves the
 * object, PTYC_ERR_ARG if an intensity is negative or not finite; then
 * nothing is appended.  count == 0 is a no-op.  Extends the coloured
 * schedule incrementally (greedy first-fit, earlier batches unchanged). */
int ptyc_add_positions(ptyc_ctx* ctx, int64_t count, const int32_t* pos_yx,
                       const float* intensities, int mem_kind);

/* Preprocessing applied by add_positions to every raw detector frame (the
 * paper's "ePIE Implementation" and "Preprocessing" sections: patterns are
 * cropped to 2^n and rotated or flipped to match the handedness of the
 * position encoders; its Discussion asks for masking invalid pixels).
 * Frames are frame_h x frame_w float32; the n x n crop starting at
 * (crop_y, crop_x) is kept; orient selects one of the 8 symmetries of the
 * square (bit 0: transpose, then bit 1: flip rows, then bit 2: flip
 * columns); PTYC_I_CENTERED moves DC from (n/2, n/2) to (0, 0); counts are
 * multiplied by scale (a detector gain) before the square root
 * (PTYC_I_IS_SQRT: the frames hold amplitudes, multiplied by sqrt(scale)).
 * The default is frame n x n, crop (0, 0), orient 0, scale 1 and the flags
 * of the config.  Must be called before set_mask and before any data.
 * Errors: PTYC_ERR_ARG (crop outside the frame, orient not in 0..7, scale
 * not finite and positive, unknown flags, reserved != 0, data present). */
typedef struct ptyc_ingest {
    int32_t frame_h, frame_w;
    int32_t crop_y, crop_x;
    int32_t orient;
    float scale;
    uint32_t flags;
    int32_t reserved;   /* must be 0 */
} ptyc_ingest;
int ptyc_set_ingest(ptyc_ctx* ctx, const ptyc_ingest* spec);

/* Detector mask (the masking of invalid pixels the paper's Discussion asks
 * for) in raw frame coordinates (frame_h * frame_w bytes, nonzero
 * = a measured pixel), in mem_kind memory, copied.  At a masked pixel there
 * is no measurement: the modulus replacement keeps the model's value there,
 * the pixel adds nothing to the error metric or to the amplitude loss, and
 * it is stored as 0.  Must be set before any data.  Errors: PTYC_ERR_ARG. */
int ptyc_set_mask(ptyc_ctx* ctx, const uint8_t* mask, int mem_kind);

/* Copy the stored amplitudes sqrt(I) of positions first .. first+count-1
 * (count * N * N float32, row-major, after the preprocessing of section
 * "Preprocessing"; the export of data the Discussion asks for) to mem_kind
 * memory (the library keeps them in blocks of 16 columns and reorders them
 * on the way out).
 * Synchronises.  Errors: PTYC_ERR_ARG for a range outside the loaded data. */
int ptyc_get_patterns(ptyc_ctx* ctx, int64_t first, int64_t count, float* out, int mem_kind);

/* Run n_sweeps passes (iterations) over the loaded positions: the ePIE
 * update of section "ePIE Implementation" (the method of Maiden and
 * Rodenburg 2009 with alpha and beta, a fixed number of iterations, the
 * position order shuffled anew in every iteration), in strict mode one
 * position after another, in coloured mode in batches of disjoint windows
 * whose probe increments are averaged at the end of the batch.
 * order == NULL: the library's schedule; each sweep draws a fresh random
 *   order from (seed, sweep counter) — strict mode: a permutation of all
 *   positions; coloured mode: the colour batches in shuffled order,
 *   ascending indices inside a batch.  ptyc_get_schedule exports it.
 * order != NULL: host array of order_len position indices (each < n_loaded)
 *   used for every sweep.  In coloured mode batch_offsets (host, n_batches+1
 *   entries, 0 = first, last = order_len, non-decreasing) splits order into
 *   batches, each of which must hold pairwise disjoint windows (checked on
 *   the host, PTYC_ERR_ARG otherwise); in strict mode batch_offsets must be
 *   NULL.
 * err_out: NULL or n_sweeps doubles receiving the running Fourier error
 *   sum_j sum_k (|Psi_j| - sqrt I_j)^2 / sum_j sum_k I_j of each sweep
 *   (this synchronises the stream).  With no positions loaded a sweep is a
 *   no-op (error 0). */
int ptyc_sweep(ptyc_ctx* ctx, int32_t n_sweeps, const int64_t* order,
               int64_t order_len, const int64_t* batch_offsets,
               int64_t n_batches, double* err_out);

/* ptyc_sweep for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sweeps with the same arguments, schedule, result bytes and errors as
 * ptyc_sweep in the per-batch launch form (PTYC_FORM_BATCH, the context's
 * tile variant), but every per-call buffer (the spectrum exchange between
 * the stages, the partial maxima of the windows, the error partials and
 * sums, the device copy of a sweep's order) lives in one fixed device array
 * of PTYC_NOALLOC_BYTES bytes that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing (no hipMalloc,
 * hipFree, pinned host memory or torch allocation); the context's own
 * buffers (object, probe, patterns) were allocated by init and
 * add_positions.  The orders are copied from pageable host memory, one
 * sweep at a time, and the call synchronises the stream before it returns.
 * Work memory needed: about 16 B per position of a sweep, 8 N^2 B per
 * position of the largest batch, 8 B per error partial (1, 4, 8, 32 and 64
 * per position at 16, 32, 64, 128 and 256 px) and 8 B per sweep;
 * PTYC_ERR_ARG (nothing run) if that exceeds PTYC_NOALLOC_BYTES.  All calls
 * on one GPU share that array, whose contents are left from the last call:
 * calls that overlap in time on one GPU (other threads, other streams)
 * race on it and must be serialised by the caller. */
#define PTYC_NOALLOC_BYTES 33554432   /* 32 MiB */
int ptyc_sweep_noalloc(ptyc_ctx* ctx, int32_t n_sweeps, const int64_t* order,
                       int64_t order_len, const int64_t* batch_offsets,
                       int64_t n_batches, double* err_out);

/* Run n_sweeps sweeps on each of n_ctx independent contexts together
 * (several scans of uneven size and pattern size at once).  Every context
 * follows its own default schedule, exactly as ptyc_sweep(ctx, n_sweeps,
 * NULL, ...) would, and produces the same bytes.  How the call is launched
 * (one persistent kernel with per-scan barriers, or one batch of every
 * scan per step) is described at ptyc_tune_multi below.  All contexts
 * must use the same device and stream; n_ctx <= PTYC_MULTI_MAX.  err_out:
 * NULL or n_ctx * n_sweeps doubles (context-major) receiving each sweep's
 * running Fourier error (this synchronises).  The call synchronises the
 * stream once before it enqueues work.  Errors: PTYC_ERR_ARG (NULL or
 * repeated context, mixed streams, too many contexts). */
#define PTYC_MULTI_MAX 64
int ptyc_sweep_multi(ptyc_ctx* const* ctxs, int32_t n_ctx, int32_t n_sweeps, double* err_out);

/* How ptyc_sweep_multi runs, chosen per call by its first context.  Variants
 * 0 .. ptyc_multi_variant_count()-1; all produce the same bytes.  With every
 * context of pattern size 64, 128 or 256 the persistent variants (0-3) run
 * the call as ONE persistent kernel: each scan is served by its own group
 * of workgroups (sized in proportion to its work, capped at what its
 * largest stage can use) and advances through its batches at its own pace,
 * its three stages per batch separated by barriers over that group only;
 * the variants differ in the inverse-stage tile at 64 and 128 px and in
 * how workgroups are shared.  Variants 4-6 (and any call with a 16 or 32 px
 * context) advance every scan by one batch per step with three launches
 * per step for all scans together; 5 and 6 give scans whose largest batch
 * holds at most 8 (16) positions an inverse-stage tile with fewer slots.
 * The default is 6.  The launch form of the first context
 * applies: PTYC_FORM_GRAPH replays the persistent launch as a HIP graph
 * (rebuilt when the scan count or the grid changes), the other forms
 * launch it cooperatively.  ptyc_tune_multi times every variant on `reps`
 * runs of one joint sweep (each from the same state), keeps the fastest on
 * the first context if it beats the current one by 2 %, restores every
 * context's object, probe and sweep counter, and reports each variant's
 * best time in ms_out (nullable, PTYC_MULTI_VARIANTS entries).  Errors:
 * PTYC_ERR_ARG for a variant out of range, reps outside 1..100 or a bad
 * context list; ptyc_get_multi_variant returns -1 for NULL. */
#define PTYC_MULTI_VARIANTS 8
int ptyc_multi_variant_count(void);
int ptyc_set_multi_variant(ptyc_ctx* first, int variant);
int ptyc_get_multi_variant(const ptyc_ctx* first);
int ptyc_tune_multi(ptyc_ctx* const* ctxs, int32_t n_ctx, int32_t reps, int32_t* variant_out,
                    double* ms_out);

/* Replace the object and the probe of each of n_ctx contexts by their mean
 * over the contexts (summed in list order).  This is the synchronisation
 * step of the paper's parallel processing scheme ("Simulating live and
 * parallel processing": independent iterations on disjoint subsets of the
 * data, with the object and the illumination averaged between them).  All
 * contexts must share N, H, W, device and stream; n_ctx <= PTYC_MULTI_MAX.
 * Errors: PTYC_ERR_ARG. */
int ptyc_average(ptyc_ctx* const* ctxs, int32_t n_ctx);

/* Export the schedule the next sweep with order == NULL would run:
 * order receives n_loaded indices, batch_offsets n_batches+1 offsets (host
 * arrays with room for n_loaded and n_loaded+1 entries; either may be NULL
 * to query n_batches only). */
int ptyc_get_schedule(ptyc_ctx* ctx, int64_t* order, int64_t* batch_offsets,
                      int64_t* n_batches);

/* Copy the object (H*W complex64) / probe (N*N complex64) out to, or in
 * from, mem_kind memory: reading out intermediate results while the
 * reconstruction continues ("Extensions of the ePIE implementation") and
 * the import and export of object and probe the Discussion asks for
 * (restart from a saved state).  get_* synchronise the stream.  Errors:
 * PTYC_ERR_ARG for NULL buffers or an unknown mem_kind. */
int ptyc_get_object(ptyc_ctx* ctx, void* out, int mem_kind);
int ptyc_get_probe(ptyc_ctx* ctx, void* out, int mem_kind);
int ptyc_set_object(ptyc_ctx* ctx, const void* in, int mem_kind);
int ptyc_set_probe(ptyc_ctx* ctx, const void* in, int mem_kind);

/* Launch form of a sweep: PTYC_FORM_BATCH (the default) launches three
 * kernels per batch; PTYC_FORM_PERSISTENT runs each sweep as one cooperative
 * kernel whose stages are separated by grid-wide barriers (in strict mode at
 * pattern sizes up to 64: one workgroup that walks the whole order with the
 * probe on chip, updating it after every position, the sequential ePIE of
 * the paper's "ePIE Implementation"); PTYC_FORM_GRAPH
 * replays one instantiated HIP graph per sweep (the batch form's kernels as
 * a chain of nodes that read their batch extents from device memory; built
 * on the first sweep and again whenever the batch count grows, the largest
 * batch grows or a buffer moves, e.g. after positions are added; each
 * replay is preceded by two device-to-device copies of the sweep's order and
 * offsets).  All forms produce the same bytes.  PTYC_FORM_DEFAULT selects
 * PTYC_FORM_BATCH.  Errors: PTYC_ERR_ARG for an unknown form or a
 * persistent grid the device cannot hold.  Every barrier wait of the
 * persistent kernels (this form and the persistent ptyc_sweep_multi) is
 * bounded: after PTYC_SPIN_LIMIT polls (environment variable read by
 * ptyc_init, default 4194304, about 0.1 s) the kernel raises a fault flag and
 * all its workgroups leave; the next call that synchronises (a sweep with
 * err_out, get_object, get_probe) then returns PTYC_ERR_HIP and the
 * context is unusable afterwards. */
#define PTYC_FORM_DEFAULT 0
#define PTYC_FORM_BATCH 1
#define PTYC_FORM_PERSISTENT 2
#define PTYC_FORM_GRAPH 3
int ptyc_set_form(ptyc_ctx* ctx, int form);
/* The current launch form (-1 for a NULL context). */
int ptyc_get_form(const ptyc_ctx* ctx);

/* Tile variants of the per-batch kernels (batch and graph forms).  The three
 * kernels of a batch can group rows, columns and slots into workgroups in
 * several ways (ptyc_tile_count variants at the context's pattern size,
 * variant 0 the default); every variant produces the same object and probe
 * bit for bit and they differ only in speed.  ptyc_tune times each variant
 * on `reps` runs of one sweep over the loaded positions (each from the same
 * state with the same schedule; a variant's time is its best run), switches
 * to the fastest if it beats the current variant by at least 2 % (else
 * keeps the current one, so that noise does not flip the choice), and
 * restores the object,
 * the probe and the sweep counter, so tuning leaves the reconstruction as it
 * was.  tile_out (nullable) receives the choice; ms_out (nullable,
 * PTYC_TILE_MAX entries) each variant's best sweep time in milliseconds (0
 * for entries past the count).  With no positions loaded nothing is timed
 * and the current variant is kept.  Synchronises the stream.  Errors:
 * PTYC_ERR_ARG for reps outside 1..100 or a tile outside
 * 0..ptyc_tile_count()-1; ptyc_tile_count and ptyc_get_tile return -1 for
 * a NULL context. */
#define PTYC_TILE_MAX 8
int ptyc_tile_count(const ptyc_ctx* ctx);
int ptyc_set_tile(ptyc_ctx* ctx, int tile);
int ptyc_get_tile(const ptyc_ctx* ctx);
int ptyc_tune(ptyc_ctx* ctx, int32_t reps, int32_t* tile_out, double* ms_out);

/* Per-kernel timing.  While enabled, every batch-form kernel is launched
 * with a start and an end event bound to its own dispatch, so the interval
 * is the kernel's execution (as a kernel trace reports it); the persistent
 * sweep kernel is bracketed by events on the stream.  This adds a little
 * host work per launch.  ptyc_profile_read synchronises the stream and returns,
 * for one kernel kind, the summed event time in milliseconds, the number of
 * launches and the number of position updates those launches processed.
 * ptyc_profile(ctx, enable) resets the totals.  Errors: PTYC_ERR_ARG for an
 * unknown kind or NULL outputs. */
#define PTYC_KERNEL_ROWS_FWD 0    /* exit wave and row FFTs */
#define PTYC_KERNEL_COLS 1        /* column FFTs, modulus replacement, inverse column FFTs */
#define PTYC_KERNEL_ROWS_INV 2    /* inverse row FFTs, object step, batch probe step */
#define PTYC_KERNEL_SWEEP 3       /* the persistent sweep kernel */
#define PTYC_KERNEL_GRAPH 4       /* one replay of the sweep graph (graph form) */
#define PTYC_KERNEL_STRICT 5      /* the sequential one-workgroup sweep kernel */
#define PTYC_KERNEL_KINDS 6
int ptyc_profile(ptyc_ctx* ctx, int enable);
int ptyc_profile_read(ptyc_ctx* ctx, int kind, double* total_ms, int64_t* launches,
                      int64_t* positions);

/* Number of loaded positions (-1 for a NULL context). */
int64_t ptyc_num_positions(const ptyc_ctx* ctx);
/* Number of completed sweeps (drives the default shuffle). */
int64_t ptyc_sweep_count(const ptyc_ctx* ctx);
/* Wait for all work enqueued by this context. */
int ptyc_synchronize(ptyc_ctx* ctx);
/* Release the context and its device memory (NULL is a no-op). */
void ptyc_destroy(ptyc_ctx* ctx);
/* Text of the last error on this context (never NULL). */
const char* ptyc_last_error(const ptyc_ctx* ctx);
/* Text of the last error of a failed ptyc_init on this thread. */
const char* ptyc_init_error(void);

/* Amplitude loss and its gradient, for gradient-based reconstruction beside
 * ePIE (not in the paper; the same forward model F(P * S_j O)):
 *   L = sum_{j in idx} sum_k (|F(P * S_j O)|_k - sqrt(I_j,k))^2
 * obj (H*W) and probe (N*N): device complex64 buffers holding the current
 * estimate (the context's own object and probe are not used or changed);
 * idx: host array of `count` loaded position indices (a minibatch; windows
 * may overlap); loss_out: host double receiving L.  If grad_obj and
 * grad_probe (device complex64, H*W and N*N) are given they are overwritten
 * with grad_scale * dL/dO and grad_scale * dL/dP in PyTorch's convention
 * for real functions of complex variables (dL/dRe + i dL/dIm):
 *   g_Psi = 2 (|Psi| - sqrt I) sgn(Psi), g_psi = F^H g_Psi,
 *   dL/dO[window j] += conj(P) g_psi,  dL/dP += conj(S_j O) g_psi.
 * The whole minibatch is transformed at once (forward and adjoint); the
 * contributions of overlapping windows to dL/dO and those of all positions
 * to dL/dP are then summed in a fixed order (minibatch order for every
 * object pixel; dL/dP in groups of 16 consecutive positions, then over the
 * groups), so the result is deterministic.  Work buffers grow to the
 * minibatch size (about N^2 complex64 per position).  Synchronises the
 * stream.  Errors:
 * PTYC_ERR_ARG for NULL buffers, an index that is not loaded, only one
 * gradient buffer, a non-finite scale, more than 2^24 positions. */
int ptyc_amp_loss(ptyc_ctx* ctx, const void* obj, const void* probe, const int64_t* idx,
                  int64_t count, float grad_scale, void* grad_obj, void* grad_probe,
                  double* loss_out);

/* ptyc_amp_loss without waiting for the result: the loss is written to the
 * device double loss_dev and the gradients (grad_scale 1) to grad_obj and
 * grad_probe (both or neither) when the enqueued work runs; nothing on the
 * host waits for the stream (only for the previous upload of an index
 * list, if it is still in flight).  For an optimiser loop: the autograd
 * wrapper computes loss and gradients in its forward and scales the saved
 * gradients by the upstream gradient (ptyc_scale_c64) in its backward.
 * Errors as for ptyc_amp_loss. */
int ptyc_amp_loss_async(ptyc_ctx* ctx, const void* obj, const void* probe, const int64_t* idx,
                        int64_t count, void* grad_obj, void* grad_probe, double* loss_dev);

/* Multiply `count` complex64 values at the device pointer data in place by
 * the device double *scale_dev (rounded to float), on the context's
 * stream.  Errors: PTYC_ERR_ARG for NULL buffers or a negative count. */
int ptyc_scale_c64(ptyc_ctx* ctx, void* data, int64_t count, const double* scale_dev);

/* ---- host-only helpers (no device needed) ---- */

/* Greedy first-fit colouring of window corners in index order: position j
 * joins the lowest colour that has fewer than max_batch members and no
 * window overlapping j's (two N x N windows overlap when |dy| < N and
 * |dx| < N).  colour_out: count int32.  *n_colours receives the count. */
int ptyc_colour(int64_t count, const int32_t* pos_yx, int32_t n,
                int32_t max_batch, int32_t* colour_out, int32_t* n_colours);

/* Check a batch schedule against window corners: offsets span the order,
 * indices are < count, windows inside each batch are pairwise disjoint.
 * Returns PTYC_OK or PTYC_ERR_ARG. */
int ptyc_check_batches(int64_t count, const int32_t* pos_yx, int32_t n,
                       const int64_t* order, int64_t order_len,
                       const int64_t* batch_offsets, int64_t n_batches);

/* Library version as major*10000 + minor*100 + patch. */
int ptyc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PTYC_H */
