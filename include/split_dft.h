/*
 * split_dft.h - batched complex DFT on separate real and imaginary planes,
 * for AMD Instinct MI355X (gfx950).
 *
 * Operation (Cariow, arXiv 2504.07264, Section II, eqs. (3)-(5)): for each of
 * `batch` independent rows of length N,
 *
 *     yr = C_N xr + S_N xi,      yi = C_N xi - S_N xr,
 *
 * with c_{k,n} = cos(2 pi k n / N) and s_{k,n} = sin(2 pi k n / N), i.e. the
 * forward DFT of eq. (1) (negative exponent, no normalisation) with the real
 * and imaginary parts held in separate arrays.  It is evaluated through the
 * decimation-in-time Kronecker factorisation of eq. (6) (Section III): a
 * bit-reversal permutation, then m = log2 N stages, each a twiddle factor
 * D^(i) (2x2 rotations omega^(i,q)) followed by a butterfly factor W^(i).
 *
 * Every FP32 result equals, bit for bit, the factors of eq. (6) applied in
 * order with these operation forms: rotation of (ar, ai) by omega^(i,q) =
 * [[c, s], [-s, c]] as (fmaf(c, ar, s*ai), fmaf(c, ai, -(s*ar))); butterfly
 * (u + v, u - v); c and s the round-to-nearest FP32 values of cos and sin of
 * 2 pi q / 2^i computed in FP64 with exact values at multiples of pi/4.
 *
 * Layout: each plane is a contiguous row-major [batch][N] array of float.
 *
 * Ownership: all data pointers are device memory owned by the caller.  A plan
 * owns its device tables (twiddles; matrix-core constants), allocated by
 * split_dft_plan and freed by split_dft_destroy.  Two-pass lengths (and
 * grouped plans that contain them) also need a workspace of
 * split_dft_workspace_bytes(plan) bytes: by default the plan allocates and
 * owns one; a plan created with SPLIT_DFT_CALLER_WORKSPACE allocates none,
 * and every call then takes the caller's (the *_ws entry points; the Python
 * binding allocates it through torch's caching allocator on the calling
 * stream), so that large allocations go through the caller's allocator and
 * calls on several streams never share one.
 *
 * Errors: every entry point returns a status and never aborts or throws.
 * Arguments are validated before any HIP call; on a validation failure no
 * kernel is launched and outputs are untouched.  Launches are asynchronous on
 * the caller's stream: a device fault surfaces at the caller's next
 * synchronisation.  split_dft_last_error() returns a message for the most
 * recent failure on the calling thread.
 *
 * Threads and streams: a plan is immutable after creation; exec and adjoint
 * may run concurrently on different streams with the same plan, except on a
 * two-pass plan through its own workspace (see split_dft_exec_ws).  A plan
 * runs on the HIP device that was current when it was created; calling exec
 * or adjoint (or building a graph) with another device current returns
 * SPLIT_DFT_ERR_INVALID_PLAN.
 *
 * Alignment: 16-byte aligned planes are required; planes that start on a
 * 128-byte line run fastest (torch allocations do).
 *
 * Environment (read when a plan is created):
 *   SPLIT_DFT_LOG=1          print each plan's schedule to stderr;
 *   SPLIT_DFT_CHUNK_MIB=k    two-pass workspace chunks of at most k MiB
 *                            (k clamped to 65536) instead of 256 (a
 *                            tuning override);
 *   SPLIT_DFT_FAIL_ALLOC=1   make plan creation fail with
 *                            SPLIT_DFT_ERR_OUT_OF_MEMORY (to test callers'
 *                            error paths).
 */
#ifndef SPLIT_DFT_H
#define SPLIT_DFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct split_dft_plan_s *split_dft_plan_t;

typedef enum {
    SPLIT_DFT_OK = 0,
    SPLIT_DFT_ERR_INVALID_LENGTH = 1, /* N not a power of two in [1, 2^16]  */
    SPLIT_DFT_ERR_INVALID_BATCH = 2,  /* batch < 1, or N*batch*4 overflows  */
    SPLIT_DFT_ERR_NULL_POINTER = 3,   /* a required pointer is NULL         */
    SPLIT_DFT_ERR_MISALIGNED = 4,     /* a data pointer not 16-byte aligned */
    SPLIT_DFT_ERR_ALIASING = 5,       /* outputs overlap illegally          */
    SPLIT_DFT_ERR_UNSUPPORTED = 6,    /* flags or variant not supported     */
    SPLIT_DFT_ERR_OUT_OF_MEMORY = 7,  /* device allocation failed           */
    SPLIT_DFT_ERR_HIP = 8,            /* a HIP runtime call failed          */
    SPLIT_DFT_ERR_INVALID_PLAN = 9    /* NULL, destroyed or foreign plan    */
} split_dft_status;

/* Plan flags, bits 0-7: precision of the arithmetic. */
#define SPLIT_DFT_FP32 0u /* FP32 throughout (the default); bit-exact eq. (6) */
/* Matrix-core modes (n = 256 only): the two 16-point sub-DFT stages of the
 * factorisation (stages 1-4 and 5-8 of eq. (6), grouped) run as dense
 * contractions with the block matrix of eq. (5) at N = 16 on the MI355X
 * matrix cores, operands split into low-precision parts, FP32 accumulation;
 * the twiddle between them is FP32.  Results are approximations of the DFT
 * (not bit-exact): */
#define SPLIT_DFT_BF16X2 1u /* bf16 hi+lo, 3 products: rel. error ~4e-6         */
#define SPLIT_DFT_FP16X2 2u /* fp16 hi+lo (lo scaled by 2^11), 3 products;
                               each row scaled by a power of two into fp16's
                               range (any finite input)                         */
#define SPLIT_DFT_BF16X3 3u /* bf16 hi+mid+lo, 6 products                       */
/* Bits 8-15: 0 = default kernel schedule, k = compiled FP32 schedule k-1
 * (used by tuning; split_dft_plan_describe names each).  At n = 2^15 and
 * 2^16 one compiled schedule, described as "fused", runs both passes of eq.
 * (6) in one persistent launch, handing each transform's intermediate
 * between the workgroups of one XCD through a ring in the workspace that the
 * XCD's L2 caches (Section III's regrouped factors); its workspace is the
 * ring (24 / 32 MiB) whatever the batch.  Its workgroups wait for each
 * other: at least 4 (2^15) or 8 (2^16) of them must be able to run at once
 * on each XCD, which holds unless other work fills the device for seconds (a
 * wait that times out ends the launch with undefined results). */
/* Bit 24: evaluate through the decimation-in-frequency factorisation of
 * eq. (9), y_2N = S D^(1) W^(1) ... D^(m) W^(m) x_2N (stages m down to 1,
 * butterfly before rotation, the bit reversal last), FP32, every n (two
 * passes from 2^15: stages m..9 on columns, then stages 8..1 on blocks); results
 * are bit-identical to those factors applied in that order with the
 * operation forms above. */
#define SPLIT_DFT_DIF (1u << 24)
/* Bit 30 (batched and grouped plans): allocate no workspace; calls on a plan
 * whose workspace_bytes is nonzero must then pass one (a NULL workspace
 * fails with SPLIT_DFT_ERR_NULL_POINTER). */
#define SPLIT_DFT_CALLER_WORKSPACE (1u << 30)
/* (Batched plans: bits 16-23, 25-29 and 31 must be 0.) */

/* Largest supported log2 N. */
#define SPLIT_DFT_MAX_LOG2N 16

/*
 * Create a plan for `batch` transforms of length n = 2^m, 0 <= m <= 16
 * (the paper's own domain is m >= 2, Section III; m = 0 and m = 1 follow from
 * the same formulas).  Builds the twiddle table omega^(i,q) (Section III,
 * definitions under eq. 6) on the host in FP64, rounds it to FP32 and copies
 * it to the current HIP device.  *out is set only on success.
 */
split_dft_status split_dft_plan(split_dft_plan_t *out, int64_t n, int64_t batch, uint32_t flags);

/*
 * Forward transform, eqs. (5)/(6): yr = C xr + S xi, yi = C xi - S xr for
 * every row.  xr, xi, yr, yi: device pointers to [batch][n] floats, 16-byte
 * aligned.  In place is allowed (yr == xr and/or yi == xi, or the planes
 * swapped); yr == yi and any partial overlap of an output with another array
 * are rejected with SPLIT_DFT_ERR_ALIASING.  `stream` is a hipStream_t
 * (NULL = the default stream).
 */
split_dft_status split_dft_exec(split_dft_plan_t plan, const float *xr, const float *xi,
                                float *yr, float *yi, void *stream);

/*
 * Adjoint (transpose) transform: gxr = C gr - S gi, gxi = S gr + C gi, the
 * transpose of E_2N of eq. (5) (C and S are symmetric).  This is N times the
 * inverse DFT; it is the vector-Jacobian product of split_dft_exec.  Same
 * argument rules as split_dft_exec.
 */
split_dft_status split_dft_adjoint(split_dft_plan_t plan, const float *gr, const float *gi,
                                   float *gxr, float *gxi, void *stream);

/*
 * As split_dft_exec / split_dft_adjoint, with a caller-owned workspace of at
 * least split_dft_workspace_bytes(plan) bytes (device memory, 16-byte
 * aligned, overlapping no data array).  Only two-pass plans (large n) use a
 * workspace; for them the plain entry points use one owned by the plan, so
 * concurrent calls on one two-pass plan from different streams must use these
 * variants with separate workspaces.  workspace may be NULL (plan-owned).
 */
split_dft_status split_dft_exec_ws(split_dft_plan_t plan, const float *xr, const float *xi,
                                   float *yr, float *yi, void *workspace, size_t workspace_bytes,
                                   void *stream);
split_dft_status split_dft_adjoint_ws(split_dft_plan_t plan, const float *gr, const float *gi,
                                      float *gxr, float *gxi, void *workspace,
                                      size_t workspace_bytes, void *stream);

/*
 * Forward transform of (xr, xi) into (yr, yi) and adjoint transform of
 * (gr, gi) into (gxr, gxi) in one call: eq. (5) and its transpose E_2N^T,
 * the two halves of a differentiable step when both inputs are at hand.
 * Single-pass FP32 schedules run both directions in one kernel launch (the
 * grid covers the forward rows, then the adjoint rows); two-pass and
 * matrix-core plans run them one after the other on the stream.  Each
 * direction follows the rules of split_dft_exec; in addition no array of one
 * direction may overlap an array of the other (SPLIT_DFT_ERR_ALIASING).
 * Results are bit-identical to split_dft_exec and split_dft_adjoint.
 */
split_dft_status split_dft_exec_adjoint(split_dft_plan_t plan, const float *xr, const float *xi, float *yr,
                                        float *yi, const float *gr, const float *gi, float *gxr, float *gxi,
                                        void *stream);
/* As split_dft_exec_adjoint, with a caller-owned workspace (rules of
 * split_dft_exec_ws; both directions use it one after the other). */
split_dft_status split_dft_exec_adjoint_ws(split_dft_plan_t plan, const float *xr, const float *xi, float *yr,
                                           float *yi, const float *gr, const float *gi, float *gxr, float *gxi,
                                           void *workspace, size_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops or harnesses that forbid hipMalloc): split_dft_exec
 * with the two-pass intermediate in a static device array of
 * SPLIT_DFT_NOALLOC_SCRATCH_BYTES instead of a workspace.  The call makes no
 * allocation of any kind; the plan (created beforehand, which allocates) and
 * the caller's inputs and outputs are used as by split_dft_exec, with the same
 * argument rules and bit-identical results.  Two-pass plans run in equal
 * chunks of at most SPLIT_DFT_NOALLOC_SCRATCH_BYTES / (8 n) transforms; a plan
 * on the fused two-pass schedule keeps its ring and control block there (32 MiB
 * at most) and runs the whole batch at once; other plans use no scratch.  A
 * transform whose intermediate (8 n bytes) exceeded the array would be
 * rejected with SPLIT_DFT_ERR_UNSUPPORTED (no supported length does).
 *
 * Each GPU holds its own copy of the array from the library's first use on it
 * until the process ends; its device address is looked up once per device,
 * when a two-pass plan is created or at the first call.  Every call on one
 * GPU uses that GPU's one array: calls that overlap in time on one GPU
 * (different streams or threads, with any plans) race on it and give wrong
 * results.  Nothing in the array needs clearing between calls (the fused
 * schedule clears its own control block with a kernel on the call's stream).
 */
#define SPLIT_DFT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
split_dft_status split_dft_exec_noalloc(split_dft_plan_t plan, const float *xr, const float *xi,
                                        float *yr, float *yi, void *stream);

/* Release a plan and its device table.  NULL is accepted and ignored. */
split_dft_status split_dft_destroy(split_dft_plan_t plan);

/* Workspace bytes a plan needs beyond inputs and outputs: 0 for lengths
 * handled in a single pass; for two-pass plans (n >= 2^15 by default) the
 * intermediate of one chunk of transforms, both planes (at most 256 MiB or one
 * transform).  0 for a NULL or destroyed plan. */
size_t split_dft_workspace_bytes(split_dft_plan_t plan);

/* Plan properties: length, batch, log2 length and the kernel schedule chosen
 * (elements per thread `ept` and transforms per workgroup `tpw`); any
 * pointer may be NULL. */
split_dft_status split_dft_plan_info(split_dft_plan_t plan, int64_t *n, int64_t *batch,
                                     int *log2n, int *ept, int *tpw);

/* Write a NUL-terminated description of the plan's kernel schedule (elements
 * per thread, transforms per workgroup, LDS bytes and data-movement options)
 * into buf, truncated to len bytes.  Makes no HIP call. */
split_dft_status split_dft_plan_describe(split_dft_plan_t plan, char *buf, size_t len);

/* Host-only: write the FP32 twiddle table the plans of length 2^m use, in
 * the layout entry[2^(i-1) + q] = omega^(i,q) for stage i = 1..m and
 * q < 2^(i-1), entry[0] = angle 0; c and s each hold 2^m floats.  Makes no
 * HIP call. */
split_dft_status split_dft_twiddle_table(int m, float *c, float *s);

/* ---- grouped execution: a ragged batch of mixed lengths --------------------
 *
 * `count` transforms of lengths lengths[k] = 2^m_k, 2 <= m_k <= 16, laid out
 * back to back in each plane: transform k occupies [offset_k, offset_k + N_k)
 * with offset_0 = 0 and offset_(k+1) = offset_k + N_k (split_dft_many_offsets).
 * Each transform is the operation of split_dft_exec (eq. (6) applied in order,
 * bit-identical to it), and the adjoint that of split_dft_adjoint.
 *
 * The shorter lengths run in one persistent kernel launch: workgroups take
 * work items (a group of short transforms of one length) from a device
 * counter, largest first.  By default each length from 2^12 up (a plan flag
 * moves this threshold) runs in its own launches of the single-length kernels,
 * addressed through the transforms' offsets (two passes through the plan's
 * workspace from 2^15), all on the caller's stream before the persistent
 * launch; with
 * SPLIT_DFT_MANY_ONE_KERNEL every length runs in the persistent kernel (one
 * transform of length >= 2^14 per work item, through a per-workgroup
 * workspace).  The counter returns to zero at the end of every launch, so
 * calls can be replayed from a graph; calls on one grouped plan must not
 * overlap in time (use one stream).  Pointer rules as for split_dft_exec
 * (16-byte aligned, outputs may coincide exactly with their own direction's
 * inputs). */
typedef struct split_dft_many_s *split_dft_many_t;
typedef struct split_dft_graph_s *split_dft_graph_t;

/* flags: bits 0-7 precision (SPLIT_DFT_FP32 only); bits 8-15 kernel build
 * (0 = default, k = build k-1: 0 two workgroups per CU, 1 one); bits 16-23
 * workgroups per CU (0 = as many as fit); SPLIT_DFT_MANY_ONE_KERNEL; bits
 * 25-29: t, the lengths from 2^t up run in per-length launches (0 = the
 * default 12; 10 <= t <= 17, 17 = none).
 * Allocates the device-side item list, offsets and twiddle table, and
 * (unless SPLIT_DFT_CALLER_WORKSPACE is set) a workspace: with
 * SPLIT_DFT_MANY_ONE_KERNEL and some length >= 2^14, 512 KiB per persistent
 * workgroup; by default, when some length is 2^15 or more, one two-pass chunk
 * (at most 256 MiB). */
#define SPLIT_DFT_MANY_ONE_KERNEL (1u << 24)
split_dft_status split_dft_many_plan(split_dft_many_t *out, const int64_t *lengths, int64_t count,
                                     uint32_t flags);
/* offsets: count + 1 entries (the last is the total number of points). */
split_dft_status split_dft_many_offsets(split_dft_many_t plan, int64_t *offsets);
/* Any pointer may be NULL. */
split_dft_status split_dft_many_info(split_dft_many_t plan, int64_t *count, int64_t *points,
                                     int *workgroups, int *items, size_t *workspace_bytes);
/* Workspace bytes the grouped plan's calls need (0 if none; the plan's own
 * unless it was created with SPLIT_DFT_CALLER_WORKSPACE); 0 for a NULL or
 * destroyed plan. */
size_t split_dft_many_workspace_bytes(split_dft_many_t plan);
/* Forward transforms of every (xr, xi) row into (yr, yi). */
split_dft_status split_dft_many_exec(split_dft_many_t plan, const float *xr, const float *xi,
                                     float *yr, float *yi, void *stream);
/* Adjoint transforms of every (gr, gi) row into (gxr, gxi). */
split_dft_status split_dft_many_adjoint(split_dft_many_t plan, const float *gr, const float *gi,
                                        float *gxr, float *gxi, void *stream);
/* Both in one launch (forward of x, adjoint of g); the forward and adjoint
 * arrays must not overlap each other. */
split_dft_status split_dft_many_exec_adjoint(split_dft_many_t plan, const float *xr, const float *xi,
                                             float *yr, float *yi, const float *gr, const float *gi,
                                             float *gxr, float *gxi, void *stream);
/* The three calls above with a caller-owned workspace of at least
 * split_dft_many_workspace_bytes(plan) bytes (device memory, 16-byte
 * aligned, overlapping no data array); NULL = the plan's own (an error for a
 * SPLIT_DFT_CALLER_WORKSPACE plan that needs one).  Everything is validated
 * before the first HIP call. */
split_dft_status split_dft_many_exec_ws(split_dft_many_t plan, const float *xr, const float *xi, float *yr,
                                        float *yi, void *workspace, size_t workspace_bytes, void *stream);
split_dft_status split_dft_many_adjoint_ws(split_dft_many_t plan, const float *gr, const float *gi, float *gxr,
                                           float *gxi, void *workspace, size_t workspace_bytes, void *stream);
split_dft_status split_dft_many_exec_adjoint_ws(split_dft_many_t plan, const float *xr, const float *xi,
                                                float *yr, float *yi, const float *gr, const float *gi,
                                                float *gxr, float *gxi, void *workspace,
                                                size_t workspace_bytes, void *stream);
/* Capture split_dft_many_exec_adjoint (or split_dft_many_exec when gr, gi,
 * gxr, gxi are all NULL) on these fixed buffers into an instantiated HIP
 * graph, using a private capturing stream.  The graph refers to the data
 * arrays (and the caller's workspace, _ws form) by address: the caller keeps
 * them allocated while the graph exists.  It also uses the plan's device
 * data, which the library keeps allocated until the plan AND every graph
 * captured from it are destroyed, in any order: after split_dft_many_destroy
 * the plan handle is invalid for every other call, but its graphs still
 * launch correctly. */
split_dft_status split_dft_many_graph(split_dft_many_t plan, const float *xr, const float *xi,
                                      float *yr, float *yi, const float *gr, const float *gi,
                                      float *gxr, float *gxi, split_dft_graph_t *out);
split_dft_status split_dft_many_graph_ws(split_dft_many_t plan, const float *xr, const float *xi, float *yr,
                                         float *yi, const float *gr, const float *gi, float *gxr, float *gxi,
                                         void *workspace, size_t workspace_bytes, split_dft_graph_t *out);
split_dft_status split_dft_graph_launch(split_dft_graph_t graph, void *stream);
split_dft_status split_dft_graph_destroy(split_dft_graph_t graph);
split_dft_status split_dft_many_destroy(split_dft_many_t plan);

/* Name of a status code; any other int gives "unknown status". */
const char *split_dft_status_string(int status);
const char *split_dft_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SPLIT_DFT_H */
