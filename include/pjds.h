/*
 * pjds.h -- C interface of libpjds, sparse matrix-vector multiplication in the padded
 * jagged diagonals storage (pJDS) format on AMD Instinct MI355X (gfx950).
 *
 * Paper: Kreutzer, Hager, Wellein, Fehske, Basermann, Bishop, "Sparse matrix-vector
 * multiplication on GPGPU clusters: a new storage format and a scalable implementation",
 * arXiv:1112.5588.  Section numbers below refer to it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Types      Row pointers and every offset are int64_t; column indices, permutations and
 *            row lengths are int32_t (so n_rows, n_cols < 2^31).  Matrix values, x and y
 *            are double (dtype PJDS_F64) or float (PJDS_F32); one dtype per call.
 * Memory     "host" arguments are ordinary CPU pointers; "device" arguments are HIP device
 *            pointers on the current device.  The caller allocates and frees every buffer;
 *            the library keeps no pointer beyond a call, except inside a batch handle
 *            (pjds_batch_*), which the caller destroys explicitly.
 * Streams    `stream` is a hipStream_t passed as void* (NULL = the default stream).  Device
 *            work is enqueued on it and the call returns without synchronising.
 * Errors     Every function returns PJDS_OK (0) or a negative PJDS_ERR_* code and leaves a
 *            message for pjds_last_error() (thread-local).  Arguments are validated before
 *            any output is written, so a failing call writes nothing.  Faults inside a
 *            kernel surface at the caller's next synchronisation, not here.
 * Threads    All functions are reentrant; concurrent calls on one device are safe unless
 *            they share an output or a workspace.
 */
#ifndef PJDS_H
#define PJDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define PJDS_OK               0
#define PJDS_ERR_ARG         (-1)  /* bad size, flag, dtype, block height or NULL pointer   */
#define PJDS_ERR_INDEX       (-2)  /* row_ptr not monotone / not starting at 0, column out of range */
#define PJDS_ERR_OVERFLOW    (-3)  /* a size or offset exceeds what the format can address   */
#define PJDS_ERR_NOMEM       (-4)  /* host allocation failed                                 */
#define PJDS_ERR_HIP         (-5)  /* the HIP runtime reported an error (launch, graph, event) */
#define PJDS_ERR_UNSUPPORTED (-6)  /* valid request outside what the library implements     */

/* ---- value types ------------------------------------------------------------------- */
#define PJDS_F64 0
#define PJDS_F32 1

/* ---- flags ------------------------------------------------------------------------- */
/* Conversion flags (pjds_plan). */
#define PJDS_LAYOUT_JD     0x0u  /* column j of the whole matrix contiguous, Listing 2's col_start
                                    addressing; needs a global sort                              */
#define PJDS_LAYOUT_BLOCK  0x1u  /* every block its own b_r x M_b column-major tile; any sort window */
#define PJDS_SYMMETRIC     0x2u  /* renumber columns into the permuted basis (square matrices):
                                    the kernel then computes (P A P^T)(P x), the way the paper runs
                                    an iterative solver entirely in the permuted basis (Sect. 2.1)  */
/* Product flags (pjds_spmv, pjds_spmmv). */
#define PJDS_Y_PERMUTED    0x4u  /* write y in the permuted row basis: y[i] = (A x)[perm[i]],
                                    coalesced; default scatters y to the original row order       */
#define PJDS_XCD_REMAP     0x8u  /* renumber workgroups so each of the 8 XCDs processes one
                                    contiguous range of row blocks (default: hardware round robin) */
#define PJDS_TWO_ROWS      0x10u /* pjds_spmv and pjds_spmv_xlds: each lane takes two adjacent
                                    sorted rows, reading both rows' values (and indices) with one
                                    2-wide load; same sums, bit for bit.  pjds_spmv needs no
                                    long-row work items (ERR_UNSUPPORTED) and a global sort or a
                                    window that is a multiple of 128 (ERR_ARG); pjds_lanczos's
                                    LDS path uses it                                              */
#define PJDS_ROW_LEN8      0x20u /* pjds_spmv_xlds: d_row_len points to n_pad one-byte lengths
                                    (uint8_t, written by pjds_pack_lengths) instead of int32:
                                    a quarter of the bytes, the same sums bit for bit; needs
                                    max_row_len <= 255 (ERR_UNSUPPORTED)                         */
/* Lanes per row (conversion flag, with PJDS_LAYOUT_BLOCK): PJDS_LANES(k) lets T = 2^k lanes
 * (k = 1..6) share each sorted row, the idea of the sliced ELLR-T format that the outlook of
 * Sect. 4 names beside pJDS.  The block height must then be b_r = 64 / T, so one block fills
 * one 64-lane wavefront.  A block of longest row M_b stores W_b = ceil(M_b / T) steps of 64
 * slots; entry j of sorted row i sits at
 *     block_start[i / b_r] + (j / T) * 64 + (i mod b_r) * T + (j mod T),
 * so lane t of a row takes entries t, t + T, t + 2T, ... and every step of the wave is one
 * contiguous 64-slot segment.  nnz_stored = 64 * sum_b W_b.  PJDS_LANES(0) is the plain
 * block layout.  Long-row splitting does not apply (n_chunks = 0); pjds_spmv and
 * pjds_spmv_axpby accept such matrices, the other products return PJDS_ERR_UNSUPPORTED. */
#define PJDS_LANES_SHIFT   8
#define PJDS_LANES_MASK    (0x7u << PJDS_LANES_SHIFT)
#define PJDS_LANES(k)      ((uint32_t)(k) << PJDS_LANES_SHIFT)

/* ---- pJDS -------------------------------------------------------------------------- */
/*
 * Sizes of a pJDS matrix, filled by pjds_plan (Sect. 2.1, "sort" and "pad" steps).
 *
 * Rows are sorted by their number of non-zeros, longest first; rows of equal length keep
 * their original order.  With sort_window < n_rows the sort happens only inside each
 * window of sort_window consecutive original rows (windows hold whole blocks).  The row
 * count is padded with empty rows to n_pad, a multiple of the block height b_r, and every
 * block of b_r consecutive sorted rows is padded to its longest row M_b; the stored entry
 * count is nnz_stored = b_r * sum_b M_b.  Padding slots hold value 0 and column 0.
 *
 * Offsets: JD layout -> n_offsets = max_row_len + 1 entries col_start[j] (start of jagged
 * diagonal j; entry j of sorted row i is at col_start[j] + i, as in Listing 2).  Block
 * layout -> n_offsets = n_blocks + 1 entries block_start[b] (entry j of sorted row i is at
 * block_start[i / b_r] + j * b_r + i % b_r).  The last offset equals nnz_stored.
 *
 * Long rows: wave groups (64 consecutive sorted rows, one GPU wavefront) whose longest row
 * exceeds split_len are processed as n_chunks work items of at most split_len entries
 * each, whose partial sums are combined in a fixed order; their schedule (4 int32 per work
 * item) is written by pjds_convert and they need a device workspace (pjds_workspace_size).
 */
typedef struct pjds_info {
    int64_t  n_rows, n_cols;
    int64_t  n_pad;          /* rows after padding, multiple of block_height             */
    int64_t  n_blocks;       /* n_pad / block_height                                      */
    int64_t  nnz;            /* entries of the input                                       */
    int64_t  nnz_stored;     /* entries of the padded format                               */
    int64_t  sort_window;    /* effective window; n_rows for a global sort                 */
    int64_t  n_offsets;      /* entries of the offsets array                               */
    int32_t  block_height;   /* b_r: 32, 64 or 128                                         */
    int32_t  max_row_len;    /* longest row                                                */
    uint32_t flags;          /* PJDS_LAYOUT_* | PJDS_SYMMETRIC | PJDS_LANES(k), as planned  */
    int32_t  split_len;      /* long-row threshold and work-item length; 0 = never split  */
    int64_t  n_chunks;       /* work items of split wave groups (0 if none)               */
    int64_t  n_split_groups; /* wave groups that are split                                 */
} pjds_info;

/*
 * Validate row_ptr (host, n_rows + 1 entries, row_ptr[0] = 0, non-decreasing) and size the
 * pJDS format.  block_height must be 32, 64 or 128 (the MI355X wavefront is 64 lanes), or
 * 64 / T with PJDS_LANES(k), T = 2^k.  sort_window <= 0 or >= n_rows means a global sort;
 * otherwise it must be a positive multiple of 64 and of block_height.  flags:
 * PJDS_LAYOUT_* | PJDS_SYMMETRIC | PJDS_LANES(k); the JD layout needs a global sort, and
 * PJDS_LANES(k > 0) needs the block layout.  split_len < 0 disables long-row splitting, 0 picks the default
 * (128), > 0 sets it (a multiple of 8).
 * Errors: ERR_ARG, ERR_INDEX, ERR_OVERFLOW (nnz_stored or n_pad >= 2^31 rows).
 */
int pjds_plan(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, int32_t block_height,
              int64_t sort_window, uint32_t flags, int32_t split_len, pjds_info *out);

/*
 * Build the pJDS arrays on the host (Sect. 2.1; addressing of Listing 2).
 *   row_ptr  [n_rows+1], col_idx [nnz], val [nnz] (dtype)      host, input CSR
 *   perm     [n_rows]     int32   host, out: perm[i] = original row of sorted row i
 *   row_len  [n_pad]      int32   host, out: length of sorted row i, 0 for padding rows
 *   offsets  [n_offsets]  int64   host, out: col_start (JD) or block_start (block)
 *   col_p    [nnz_stored] int32   host, out: column index per stored entry (padding 0;
 *                                 with PJDS_SYMMETRIC the renumbered column invperm[col])
 *   val_p    [nnz_stored] dtype   host, out: value per stored entry (padding 0), bit copies
 *   sched    [4*n_chunks] int32   host, out: long-row work items; may be NULL if n_chunks = 0
 * `info` must come from pjds_plan on the same row_ptr.  Column indices are checked to lie
 * in [0, n_cols) before anything is written.  Deterministic; uses several host threads.
 */
int pjds_convert(const pjds_info *info, const int64_t *row_ptr, const int32_t *col_idx,
                 const void *val, int32_t dtype, int32_t *perm, int32_t *row_len,
                 int64_t *offsets, int32_t *col_p, void *val_p, int32_t *sched);

/* Device workspace for the long-row work items: bytes needed (0 when n_chunks == 0). */
int pjds_workspace_size(const pjds_info *info, int32_t dtype, int64_t *bytes);

/* Zero the workspace's completion counters (once after allocating it; the product leaves
 * them zero again).  Enqueued on `stream`; uses a kernel, not a memset. */
int pjds_workspace_init(const pjds_info *info, int32_t dtype, void *d_work, void *stream);

/*
 * y = A x on the device with the pJDS arrays (Listing 2; one GPU lane per sorted row, one
 * 64-lane wavefront per 64 consecutive sorted rows).
 *   d_row_len, d_offsets, d_col_p, d_val_p  device copies of pjds_convert's outputs
 *   d_perm    device perm; may be NULL when flags has PJDS_Y_PERMUTED
 *   d_sched, d_work  device schedule and workspace; may be NULL when info->n_chunks == 0
 *   d_x       [n_cols] dtype, device: in the original column basis, or in the permuted
 *             basis (x_p[i] = x[perm[i]]) if the matrix was converted with PJDS_SYMMETRIC
 *   d_y       [n_rows] dtype, device, out: original row order, or the permuted order with
 *             PJDS_Y_PERMUTED.  Written, never read.
 * Sums run over each row's entries in stored order with fused multiply-add; long rows are
 * summed per work item and the partial sums added in item order, so results are
 * bitwise reproducible from run to run.  Padding never enters the arithmetic.
 */
int pjds_spmv(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
              const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
              const int32_t *d_sched, void *d_work, int32_t dtype, const void *d_x, void *d_y,
              uint32_t flags, void *stream);

/*
 * pjds_spmv for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same product, kernels and
 * results (bitwise) as pjds_spmv, with the long-row workspace taken from a fixed array in the
 * library's own device memory instead of a d_work argument.  Nothing is allocated, by the
 * library or by anything it calls.
 *   Arguments as for pjds_spmv, without d_work.
 *   Limit: the workspace pjds_workspace_size reports for `info` must not exceed
 *   PJDS_NOALLOC_SCRATCH_BYTES (16 MiB); larger plans are rejected with PJDS_ERR_OVERFLOW
 *   before anything is launched.  Each GPU the library runs on holds one such array until
 *   the process ends; its address is looked up on the first call made with that device
 *   current, so call with the stream's device current.
 *   Every call on one GPU shares that GPU's array: calls that overlap in time on one GPU
 *   (different streams, or several host threads) race and give wrong results.  Each call
 *   clears the completion counters it uses (a fill kernel on `stream`, no memset) before the
 *   product, so a call never depends on what an earlier one left behind.
 */
#define PJDS_NOALLOC_SCRATCH_BYTES (16ll << 20)
int pjds_spmv_noalloc(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                      const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                      const int32_t *d_sched, int32_t dtype, const void *d_x, void *d_y,
                      uint32_t flags, void *stream);

/*
 * y = alpha (A x) + beta z, the product with a fused update (pjds_spmv's arguments plus
 * alpha, beta and d_z; d_z NULL means beta is ignored).  z is indexed like y (permuted order
 * with PJDS_Y_PERMUTED, original order otherwise) and may be y itself, which accumulates:
 * this is how the product of a matrix split into a local and a non-local column part is
 * assembled, y = A_local x, then y = A_nonlocal x + y (Sect. 3.1, vector mode with overlap,
 * where the result vector is written twice).  z may not be x.
 */
int pjds_spmv_axpby(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                    const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                    const int32_t *d_sched, void *d_work, int32_t dtype, const void *d_x,
                    double alpha, double beta, const void *d_z, void *d_y, uint32_t flags,
                    void *stream);

/*
 * y = A x like pjds_spmv, with the right-hand side staged in LDS.  Needs the block layout and
 * a sort window that is a multiple of 256.  Sorting never moves a row out of its window of
 * original rows, so a workgroup owning `tile_rows` consecutive sorted rows (a multiple of 256
 * that divides, or is divided by, the window; 0 -> max(window, 1024)) works on original rows
 * inside the windows it touches, [lo, hi).  It copies x[lo - x_halo, hi + x_halo) (clipped to
 * [0, n_cols)) into LDS once, then entries whose column falls in that range read x from LDS
 * and the others from global memory.  For matrices whose non-zeros cluster near the diagonal
 * this replaces most scattered global gathers with LDS reads (the right-hand-side reuse that
 * eq. (1) calls alpha).  The staged range, (max(tile_rows, window) + 2*x_halo) values, must
 * fit 64 KiB; ERR_ARG otherwise.  Rows are not split (no schedule or workspace).  Tiles go
 * to the 8 XCDs in runs of 16 consecutive tiles, so neighbours that share halo values share
 * an L2; PJDS_XCD_REMAP gives each XCD one contiguous range instead.
 */
int pjds_spmv_xlds(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                   const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm, int32_t dtype,
                   const void *d_x, void *d_y, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                   void *stream);

/*
 * One-byte copies of the row lengths for the staged product's PJDS_ROW_LEN8 form:
 * d_row_len8[i] = d_row_len[i] for i < n_pad (device arrays; d_row_len8 holds n_pad bytes).
 * The lengths are the paper's rowmax array (Listing 2); at most 255 fits a byte, so a matrix
 * with longer rows is refused with PJDS_ERR_UNSUPPORTED before anything is launched.
 */
int pjds_pack_lengths(const pjds_info *info, const int32_t *d_row_len, uint8_t *d_row_len8, void *stream);

/*
 * Y = A X for k right-hand sides stored row-major (interleaved): X[c*k + v], Y[r*k + v]
 * (Y in the permuted row order with PJDS_Y_PERMUTED).  A tile of t = vectors_per_tile
 * consecutive right-hand sides is handled by t / vectors_per_lane lanes per row (1, 2, 4, 8,
 * 16 or 32), each applying the row's entries to vectors_per_lane (1, 2 or 4) adjacent
 * right-hand sides with one wide load; a matrix entry is loaded once per tile, so the matrix
 * is streamed ceil(k / t) times.  k must be a multiple of vectors_per_lane, and X and Y
 * aligned to vectors_per_lane values.  Arguments otherwise as pjds_spmv; long rows are not
 * split (no workspace needed).
 */
int pjds_spmmv(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
               const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
               int32_t dtype, int32_t k, int32_t vectors_per_tile, int32_t vectors_per_lane,
               const void *d_X, void *d_Y, uint32_t flags, void *stream);

/*
 * Y = A X as pjds_spmmv, with X staged in LDS (the idea of pjds_spmv_xlds for k right-hand
 * sides).  Needs the block layout and a sort window; t / vectors_per_lane lanes per row must
 * be 1, 2 or 4.  A 512-thread workgroup owns `tile_rows` consecutive sorted rows (a multiple
 * of 64; 0 -> max(window, 1024)) and one tile of t right-hand sides; it copies the rows of X
 * that the original rows of its sort windows cover, widened by x_halo (>= 0) on each side,
 * for those t vectors into LDS (at most 64 KiB: two workgroups per CU), then reads an X row
 * from LDS where staged and from global memory otherwise.  Row tiles go to the XCDs in runs
 * of 16, as in pjds_spmv_xlds.  The same FMAs in the same order as
 * pjds_spmmv: results equal it bit for bit, for any halo.  No flag other than PJDS_Y_PERMUTED.
 * Errors: ERR_ARG (layout, sizes, alignment, halo), ERR_UNSUPPORTED (several lanes per row).
 */
int pjds_spmmv_xlds(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                    const int32_t *d_col_p, const void *d_val_p, const int32_t *d_perm,
                    int32_t dtype, int32_t k, int32_t vectors_per_tile, int32_t vectors_per_lane,
                    const void *d_X, void *d_Y, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                    void *stream);

/* ---- the product inside an iterative solver ----------------------------------------- */
/*
 * `steps` steps of the symmetric Lanczos recurrence on a square matrix converted with
 * PJDS_SYMMETRIC, entirely in the permuted basis (the solver use of Sect. 2.1: permute once
 * before and once after the iteration):
 *   v_0 = v/||v||, beta_0 = 0;  w = A v_j - beta_j v_{j-1};  alpha_j = w.v_j;
 *   w = w - alpha_j v_j;  beta_{j+1} = ||w||;  v_{j+1} = w / beta_{j+1}.
 * FP64 only.  d_v0 [n_rows] is the start vector in the permuted basis (x_p[i] = x[perm[i]]).
 * Outputs (device): d_alpha [steps], d_beta [steps + 1] (beta_0 = 0).  The scalars stay on the
 * device; nothing synchronises with the host, so the call may be captured in a graph.  The
 * Lanczos vectors are held unnormalised (v_j = u_j / s_j, the 1/s_j factors applied inside
 * the product and the updates), which saves the rescaling pass; d_v0 is only read.
 * x_halo >= 0 uses the LDS-staged product (pjds_spmv_xlds's conditions), otherwise the plain
 * one (d_sched/d_work as for pjds_spmv).  flags: 0, or PJDS_ROW_LEN8 with x_halo >= 0 (the
 * staged product then reads one-byte row lengths: d_row_len addresses the n_pad bytes
 * pjds_pack_lengths writes; rows of at most 255 entries, else PJDS_ERR_UNSUPPORTED); any other
 * flag, or PJDS_ROW_LEN8 without x staging, is PJDS_ERR_ARG.  d_vectors and d_scratch are device buffers of the
 * sizes pjds_lanczos_workspace reports (three vectors; reduction partials).  A zero beta
 * (invariant subspace found) makes the following steps non-finite: stop before it.
 * Reductions use a fixed grid and fixed trees: results are reproducible bit for bit.
 */
int pjds_lanczos_workspace(const pjds_info *info, int64_t *vector_bytes, int64_t *scratch_bytes);
int pjds_lanczos(const pjds_info *info, const int32_t *d_row_len, const int64_t *d_offsets,
                 const int32_t *d_col_p, const void *d_val_p, const int32_t *d_sched, void *d_work,
                 const double *d_v0, int32_t steps, int32_t x_halo, int32_t tile_rows, uint32_t flags,
                 double *d_alpha, double *d_beta, void *d_vectors, void *d_scratch, void *stream);

/* ---- many matrices in one call ------------------------------------------------------ */
/*
 * A batch computes y_m = A_m x_m for every member m (each member a pJDS matrix of the same
 * block height and layout, any sizes).  Modes:
 *   PJDS_BATCH_PERSISTENT  one persistent kernel: the members' rows are cut into tiles of
 *                          `groups_per_tile` wave groups (64 sorted rows each; <= 0 -> 8),
 *                          member by member, largest member first; each wave pulls tiles
 *                          from one device counter until none is left.  A fill kernel resets
 *                          the counter first.  Both are captured once in a HIP graph.
 *   PJDS_BATCH_GRAPH       one pjds_spmv launch per member, captured in a HIP graph.
 *   PJDS_BATCH_DIRECT      one pjds_spmv launch per member, issued on every launch call.
 * Rows are never split into work items here, so members need no workspace.
 * Ownership: the handle copies the pjds_info structs but keeps the device pointers; the
 * caller keeps those buffers alive until pjds_batch_destroy.  The handle owns its device
 * tables and graph.  Launches of one handle must not overlap (they share the tile
 * counter); different handles are independent.
 */
#define PJDS_BATCH_PERSISTENT 0
#define PJDS_BATCH_GRAPH      1
#define PJDS_BATCH_DIRECT     2

typedef struct pjds_batch_member {
    const pjds_info *info;       /* host: the member's plan                                */
    const int32_t *d_row_len;    /* device arrays of the member, as for pjds_spmv          */
    const int64_t *d_offsets;
    const int32_t *d_col_p;
    const void    *d_val_p;
    const int32_t *d_perm;       /* may be NULL with PJDS_Y_PERMUTED                        */
    const void    *d_x;          /* device, [n_cols] dtype                                 */
    void          *d_y;          /* device, [n_rows] dtype, written                         */
} pjds_batch_member;

typedef struct pjds_batch pjds_batch;

/* flags: 0 or PJDS_Y_PERMUTED.  Errors: ERR_ARG (inconsistent members), ERR_HIP, ERR_NOMEM. */
int pjds_batch_create(int32_t n_members, const pjds_batch_member *members, int32_t dtype,
                      uint32_t flags, int32_t mode, int32_t groups_per_tile, pjds_batch **out);
/*
 * A persistent batch (as PJDS_BATCH_PERSISTENT) whose kernel stages x in LDS, the idea of
 * pjds_spmv_xlds applied per tile: 512-thread workgroups pull tiles of `groups_per_tile` wave
 * groups (<= 0 -> 32, i.e. 2048 rows, when every member is sorted in windows of whole 128-row
 * groups, else 8); a workgroup copies x[lo, hi) of its member into LDS,
 * where [lo, hi) are the original rows of the sort windows its sorted rows lie in (the whole
 * member for a global sort) widened by `x_halo` (>= 0) on each side and clipped to the
 * member's columns, then its waves pull the tile's wave groups and read x from LDS wherever
 * the column falls in the staged range, from global memory elsewhere.  The staged range is
 * cut at 78 KiB (two workgroups per CU on gfx950's 160 KB of LDS); columns past the cut are
 * read from global memory, so any halo gives the same results, bit for bit those of
 * PJDS_BATCH_PERSISTENT and pjds_spmv.  Suits members sorted in windows whose non-zeros lie
 * within about x_halo of the diagonal.  Errors: as pjds_batch_create; ERR_ARG for x_halo < 0.
 */
int pjds_batch_create_xlds(int32_t n_members, const pjds_batch_member *members, int32_t dtype,
                           uint32_t flags, int32_t groups_per_tile, int32_t x_halo, pjds_batch **out);
/* Enqueue one evaluation of the whole batch on `stream` (asynchronous). */
int pjds_batch_launch(pjds_batch *batch, void *stream);
/* Tile count and persistent grid size (workgroups) of a handle; either pointer may be NULL. */
int pjds_batch_info(const pjds_batch *batch, int32_t *n_tiles, int32_t *grid);
/* Free the handle, its device tables and graph (synchronise first if launches may still run). */
int pjds_batch_destroy(pjds_batch *batch);

/* ---- local / non-local split (Sect. 3.1, vector mode) ------------------------------- */
/*
 * A row-distributed product splits its rows' entries by column: A = A_loc + A_nl, where A_loc
 * holds the entries whose column lies in [c0, c1) (the columns of x the process owns) and
 * A_nl the rest.  The local product can then start while the non-local x entries are still
 * being exchanged, and the non-local product adds into y afterwards.  Both parts keep A's
 * n_rows x n_cols shape and each row's entries in their stored order, so they convert and
 * multiply like any CSR matrix (pjds_spmv for A_loc, pjds_spmv_axpby with b = 1, z = y for
 * A_nl).  Host arrays only.
 *
 * pjds_split_count: *nnz_local = entries of A_loc (A_nl has nnz - *nnz_local).
 * pjds_split_columns: writes rp_loc[n_rows+1], col_loc/val_loc[nnz_local] and
 *   rp_nl[n_rows+1], col_nl/val_nl[nnz - nnz_local]; values of type dtype are copied bit for
 *   bit.  0 <= c0 <= c1 <= n_cols, else ERR_ARG; row_ptr and columns are validated as by
 *   pjds_plan and pjds_convert before anything is written.
 */
int pjds_split_count(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, const int32_t *col_idx,
                     int64_t c0, int64_t c1, int64_t *nnz_local);
int pjds_split_columns(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, const int32_t *col_idx,
                       const void *val, int32_t dtype, int64_t c0, int64_t c1, int64_t *rp_loc,
                       int32_t *col_loc, void *val_loc, int64_t *rp_nl, int32_t *col_nl, void *val_nl);

/* ---- ELLPACK-R (Sect. 2.1, Listing 1) ---------------------------------------------- */
/*
 * Rows keep their order; the non-zeros of each row are shifted left and the
 * n_pad x max_row_len rectangle is stored column by column: entry j of row i at
 * j * n_pad + i, with n_pad = n_rows rounded up to a multiple of 64.  rowmax[i] holds the
 * length of row i.  pjds_info is reused: block_height = 64, nnz_stored = n_pad*max_row_len,
 * n_offsets = 0.  ellr_plan reports the size even when it is too large to allocate; the
 * caller decides.  ERR_OVERFLOW if nnz_stored does not fit int64.
 */
int ellr_plan(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, pjds_info *out);
int ellr_convert(const pjds_info *info, const int64_t *row_ptr, const int32_t *col_idx,
                 const void *val, int32_t dtype, int32_t *rowmax, int32_t *col_e, void *val_e);
/* y = A x with the ELLPACK-R arrays (Listing 1): one lane per row, y in row order. */
int ellr_spmv(const pjds_info *info, const int32_t *d_rowmax, const int32_t *d_col_e,
              const void *d_val_e, int32_t dtype, const void *d_x, void *d_y, void *stream);

/* ---- CSR on the GPU (the format of the paper's CPU comparison, Table 1) -------------- */
/*
 * y = A x straight from CSR device arrays.  variant 1: one lane per row (scalar);
 * 4, 16 or 64: that many lanes per row, each summing a strided subset of the row, then a
 * fixed-order butterfly reduction (vector).  Deterministic.
 */
int csr_spmv(int64_t n_rows, int64_t n_cols, const int64_t *d_row_ptr, const int32_t *d_col,
             const void *d_val, int32_t dtype, const void *d_x, void *d_y, int32_t variant,
             void *stream);

/* ---- learned tuner: features -------------------------------------------------------- */
/*
 * 24 features of a CSR matrix (host arrays) for the configuration tuner, written to out[24]:
 *  0 log2 N, 1 log2(nnz+1), 2-5 mean, std, skewness, excess kurtosis of the row lengths,
 *  6 min, 7 log2(max+1), 8 max/mean, 9 empty-row fraction, 10-12 p50/p90/p99 over the mean,
 *  13 log2 of ELLPACK-R stored/nnz, 14-15 pJDS stored/nnz at block height 64 with a global
 *  sort and with a 4096-row sort window (the padding of Sect. 2.1), 16-18 max/mean/std of
 *  |col-row| / max(N, n_cols), 19-20 fractions with |col-row| <= 64 and <= 4096, 21 log of
 *  distinct offsets per entry, 22 share of the 16 most used offsets, 23 entries per distinct
 *  128-byte x line in 64-row blocks (a proxy of the right-hand-side reuse alpha of eq. (1)).
 * Offset statistics use every s-th entry, s = ceil(nnz / 2^20).  O(N log N + nnz).
 */
int pjds_features(int64_t n_rows, int64_t n_cols, const int64_t *row_ptr, const int32_t *col_idx,
                  float *out);

/* ---- learned tuner: the network ----------------------------------------------------- */
/*
 * Three-layer perceptron d_in -> 64 -> 64 -> d_out with ReLU after the hidden layers,
 * binary32, predicting a standardised run time per kernel configuration.  Parameters are
 * one packed device array [W1 (d_in x 64) | b1 (64) | W2 (64 x 64) | b2 (64) | W3 (64 x
 * d_out) | b3 (d_out)], weights (fan_in, fan_out) row-major; 1 <= d_in, d_out <= 64.
 * X [batch x d_in], T and M [batch x d_out] are row-major device arrays; M is a 0/1 mask of
 * the labels present.  Loss = sum(M (P - T)^2) / sum(M).  Deterministic: the gradient is
 * summed over 64-row tiles in tile order.  Asynchronous on `stream`.
 */
int mlp_param_count(int32_t d_in, int32_t d_out, int64_t *n);
/* Device workspace of mlp_backward for a batch (bytes). */
int mlp_workspace_size(int32_t d_in, int32_t d_out, int64_t batch, int64_t *bytes);
/* P [batch x d_out] = network(X). */
int mlp_forward(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
                float *d_P, void *stream);
/* d_grad [n_params] = gradient of the loss; *d_loss (device, may be NULL) = the loss. */
int mlp_backward(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
                 const float *d_T, const float *d_M, float *d_grad, float *d_loss, void *d_work,
                 void *stream);
/* One Adam update (Kingma and Ba, 2015) at 1-based `step` with bias correction. */
int mlp_adam_step(float *d_params, const float *d_grad, float *d_m, float *d_v, int64_t n,
                  int32_t step, float lr, float beta1, float beta2, float eps, void *stream);
/* Per row: idx = argmin over outputs c with valid[c] != 0 of P*scale[c] + shift[c] (scale,
 * shift, valid may be NULL = 1, 0, all valid) and margin = runner-up minus best. */
int mlp_infer(const float *d_params, int32_t d_in, int32_t d_out, int64_t batch, const float *d_X,
              const float *d_scale, const float *d_shift, const float *d_valid, int32_t *d_idx,
              float *d_margin, void *stream);

/* ---- measurement helpers ------------------------------------------------------------ */
/* Stream probes for the achievable bandwidth ceiling: each workgroup streams a contiguous chunk
 * with 16-byte loads, several in flight per thread.  mode 0 reads n doubles with non-temporal
 * loads and writes one partial sum per workgroup to d_out (1024 values), mode 1 copies n doubles d_in -> d_out, mode 2
 * reads like mode 0 with ordinary cached loads: a read-only pass that evicts what the caches
 * (the Infinity Cache included) held before, leaving no dirty line to write back.  d_in and
 * d_out are device arrays of n doubles (mode 1) or of n and 2048 doubles (modes 0, 2). */
int pjds_probe(int32_t mode, const double *d_in, double *d_out, int64_t n, void *stream);
/* Kernel timing hook, for benchmarks (it computes nothing).  Arms the calling thread: the main
 * kernel of the next call on this thread to pjds_spmv, pjds_spmv_xlds, pjds_spmv_noalloc,
 * pjds_spmmv, pjds_spmmv_xlds, ellr_spmv, csr_spmv or pjds_probe (or to an entry point built
 * on them, such as pjds_lanczos, whose first product kernel takes it) is launched with
 * hipExtLaunchKernel, whose dispatch records `start_event` when the kernel starts and
 * `stop_event` when it ends; hipEventElapsedTime on the two then gives the kernel's own
 * duration, without the time the stream spends between separately recorded events and the
 * dispatch.  Both are hipEvent_t values the caller created (hipEventCreate) and owns.  The
 * launch that takes the events disarms the hook; (NULL, NULL) disarms it without a launch.
 * Leave it disarmed while a stream is being captured into a graph: events are not graph
 * nodes here.  PJDS_ERR_ARG if exactly one of the two is NULL (the hook is then left as it
 * was). */
int pjds_time_next_launch(void *start_event, void *stop_event);

/* ---- diagnostics ------------------------------------------------------------------- */
const char *pjds_last_error(void);
/* Library version string. */
const char *pjds_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PJDS_H */
