/*
 * blip.h -- C ABI of libblip: periodic cubic B-spline ("blip") orbital
 * evaluation on AMD Instinct MI355X (gfx950).
 *
 * The operation (Sec. II.B "Orbital evaluation", Eqs. (11.12.24.1),
 * (11.12.24.2) and (7)): every orbital psi_l is a sum over a periodic grid
 * of coefficients a_{l,s} times a tensor product of 1-D cubic B-splines;
 * at a position only the 4x4x4 sites around it contribute.  libblip keeps
 * the coefficient table resident on the GPU (loaded once, as the paper's
 * precomputed input file is) and evaluates psi_l, grad psi_l and
 * lap psi_l for all L orbitals at a block of positions -- the block of
 * trial moves that quasi-simultaneous updating (Sec. IV.A, Eqs.
 * (11.12.23.1)-(11.12.23.2)) produces once per Monte Carlo step.
 *
 * Conventions shared by every call:
 *  - Device pointers are HIP device memory of the current device; host
 *    pointers are ordinary host memory.  Sizes are in elements.
 *  - Positions are Cartesian bohr, float64, [npos][3], unwrapped: the
 *    library wraps them into the cell in FP64.
 *  - Outputs are orbital-contiguous rows: val [npos][L], grad [npos][3][L],
 *    lap [npos][L]; float for real tables, float2 (re, im) for complex ones.
 *    Accumulation is FP32 (FP64 in the debug kernel of blip_eval_ex).
 *  - Gradients are in bohr^-1, Laplacians in bohr^-2.
 *  - Every call returns BLIP_OK (0) or a negative status; the message for
 *    the last non-zero status on the calling thread is blip_last_error().
 *    Argument errors are reported before anything is enqueued.
 *  - Evaluation calls are asynchronous and stream-ordered on the caller's
 *    stream (a hipStream_t passed as void*, NULL = the null stream); they
 *    never synchronise.  Faults on the device surface at the caller's next
 *    synchronisation as HIP errors.
 *  - A table is immutable after blip_load; evaluation calls on one table may
 *    run concurrently on different streams.
 *  - Non-finite positions never cause out-of-bounds reads: their output
 *    rows are NaN.
 */
#ifndef BLIP_H
#define BLIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLIP_API __attribute__((visibility("default")))

typedef struct blip_table_s* blip_table;   /* opaque; owned by the library */

/* Storage dtype of the resident table.  The caller always hands over an
 * FP32 master (float, or float2 for complex); reduced-precision storage is
 * produced on the device by round-to-nearest-even. */
typedef enum {
    BLIP_F32 = 0,     /* real, float                                      */
    BLIP_BF16 = 1,    /* real, bfloat16                                   */
    BLIP_F16 = 2,     /* real, IEEE half with a power-of-two table scale  */
    BLIP_C64 = 3,     /* complex, float2                                  */
    BLIP_CBF16 = 4,   /* complex, bfloat16 (re, im) pairs                 */
    BLIP_CF16 = 5     /* complex, half (re, im) pairs with a 2^e scale    */
} blip_dtype;

enum {
    BLIP_OK = 0,
    BLIP_E_ARG = -1,     /* bad argument (sizes, NULL, singular lattice)   */
    BLIP_E_OOM = -2,     /* device allocation failed                       */
    BLIP_E_HIP = -3,     /* a HIP runtime call failed                      */
    BLIP_E_DTYPE = -4,   /* dtype not valid for this table / request       */
    BLIP_E_ALIGN = -5,   /* pointer not aligned as the call requires       */
    BLIP_E_STATE = -6,   /* invalid handle or object state                 */
    BLIP_E_NODEV = -7    /* no usable gfx950 device                        */
};

/* Evaluation kernels selectable through blip_eval_ex. */
typedef enum {
    BLIP_KERNEL_AUTO = 0,   /* tuned tiled kernel (what blip_eval runs)        */
    BLIP_KERNEL_PLAIN = 1,  /* one workgroup per position, one lane per orbital,
                               64 x 5 weights in LDS: the paper's coalesced
                               mapping (Sec. IV.B) written for wave64         */
    BLIP_KERNEL_TILED = 2,  /* P positions per workgroup, separable 1-D weights,
                               o orbitals per lane with wide loads             */
    BLIP_KERNEL_F64ACC = 3, /* tiled kernel with FP64 weights, accumulation and
                               outputs (debug; real FP32 tables only): val, grad
                               and lap are double arrays of the same shapes    */
    BLIP_KERNEL_SITE = 4    /* one wavefront per (position, orbital), one lane
                               per stencil site, the 64 products summed across
                               the wavefront: the paper's non-coalesced
                               comparison mapping (Sec. IV.C, implementation
                               (2)); called with npos = 1 per electron it is
                               implementation (1).  For measurement: every
                               load is uncoalesced by design                   */
} blip_kernel;

typedef struct {
    int kernel;          /* blip_kernel                                       */
    int tile_pos;        /* P: positions per workgroup (1..64), 0 = tuned     */
    int vec;             /* o: table elements per lane per load (1, 2, 4, 8),
                            0 = tuned                                          */
} blip_eval_opts;

/*
 * blip_load -- copy a coefficient table to the device and keep it resident.
 * (The precomputed coefficients a~_{l,s~} of Eq. (7), loaded once at start.)
 *
 *  lattice     host double[9]: rows a_1, a_2, a_3 of the periodic cell, bohr.
 *              Must be finite and non-singular.
 *  n1, n2, n3  grid points along a_1, a_2, a_3; each >= 4.  Site (i1,i2,i3)
 *              sits at sum_d (i_d / n_d) a_d.
 *  norb        number of orbitals L >= 1.
 *  coeffs_host host array [n1][n2][n3][norb] in C order (orbital fastest):
 *              float for real storage dtypes, float2 (re, im) for complex.
 *              Read during the call only; the library keeps its own copy.
 *  storage     blip_dtype of the resident copy.
 *  kvec        host double[3] k-point (bohr^-1) for complex tables, giving
 *              psi = exp(i k.r) u with u the spline sum; NULL = Gamma.
 *              A kvec with a real storage dtype is BLIP_E_DTYPE.
 *  out         receives the handle (NULL on failure).
 * Device memory: n1*n2*n3 rows of roundup(L * element bytes, 128) bytes;
 * n3 times that row size must stay below 2 GiB (BLIP_E_ARG otherwise).
 * Synchronous: returns after the table is resident.  Errors: BLIP_E_ARG,
 * BLIP_E_DTYPE, BLIP_E_OOM, BLIP_E_HIP, BLIP_E_NODEV.
 */
BLIP_API int blip_load(const double lattice[9], int n1, int n2, int n3,
                       int norb, const void* coeffs_host, blip_dtype storage,
                       const double kvec[3], blip_table* out);

/*
 * blip_eval -- evaluate all orbitals at a block of positions (Eq.
 * (11.12.24.1) for every j of the block; the N x L independent evaluations
 * of quasi-simultaneous updating, Sec. IV.A).
 *
 *  t     handle from blip_load.
 *  pos   device double[npos][3], Cartesian bohr, any values (wrapped in FP64).
 *  npos  >= 0; 0 returns BLIP_OK and enqueues nothing.
 *  val   device [npos][L] float (real) or float2 (complex); required.
 *  grad  device [npos][3][L]; lap device [npos][L].  Pass both or neither:
 *        grad == lap == NULL runs the values-only kernel.
 *  stream hipStream_t (as void*), NULL = null stream.
 * pos must be 8-byte and val/grad/lap 4-byte aligned (BLIP_E_ALIGN); outputs
 * whose base addresses are 16-byte aligned get whole-vector stores.  The
 * caller owns them and keeps them alive until the stream has run the work.
 * Runs the tuned tiled kernel.  No allocation, no synchronisation.
 */
BLIP_API int blip_eval(blip_table t, const double* pos, int64_t npos,
                       void* val, void* grad, void* lap, void* stream);

/*
 * blip_eval_ex -- blip_eval with an explicit kernel choice (opts may be NULL
 * for the defaults).  Same arguments, layouts and errors as blip_eval;
 * BLIP_E_ARG for P outside 1..64 or an unsupported o for the storage dtype,
 * BLIP_E_DTYPE for BLIP_KERNEL_F64ACC on anything but BLIP_F32.
 * Every kernel and every (P, o) computes each output with the same sequence
 * of operations, so results agree bit for bit across tilings
 * (BLIP_KERNEL_PLAIN, BLIP_KERNEL_SITE and BLIP_KERNEL_F64ACC round
 * differently).  tile_pos and vec are ignored by the plain and site kernels.
 */
BLIP_API int blip_eval_ex(blip_table t, const double* pos, int64_t npos,
                          void* val, void* grad, void* lap,
                          const blip_eval_opts* opts, void* stream);

/*
 * blip_eval_batched -- evaluate the move blocks of many walkers in one
 * persistent launch (quasi-simultaneous updating makes every moved electron
 * of every walker an independent evaluation, Sec. IV.A, Eq. (11.12.23.1)).
 *
 *  pos       device double[capacity][3]: the walkers' blocks concatenated;
 *            walker w owns rows offsets[w] .. offsets[w+1]-1.
 *  offsets   device int64[nw+1], offsets[0] == 0, non-decreasing.  Only
 *            offsets[nw] (the total) is read, on the device, so the host
 *            need not know it; a total above capacity is clamped to capacity.
 *  nw        number of walkers (0: nothing is enqueued).
 *  capacity  host bound on the total: the size of pos and of the outputs.
 *  val, grad, lap  as blip_eval, with capacity rows; row j belongs to the
 *            same position as pos row j.  Rows past the total are untouched.
 *  workspace device scratch of at least blip_workspace_size(t, capacity)
 *            bytes, 256-byte aligned, owned by the caller; calls that share
 *            a workspace must be ordered on one stream.
 * The positions are sorted by space on the device (counting sort by brick of
 * cells) so that positions sharing stencil rows are evaluated together; each
 * output is still computed in the fixed order of blip_eval, so results equal
 * the per-walker blip_eval results bit for bit.  Enqueues five kernels on the
 * stream; no allocation, no synchronisation, and no memset (capturable).
 */
BLIP_API int blip_eval_batched(blip_table t, const double* pos, const int64_t* offsets, int nw,
                               int64_t capacity, void* val, void* grad, void* lap,
                               void* workspace, size_t workspace_bytes, void* stream);

/* blip_workspace_size -- bytes of workspace blip_eval_batched needs for a
 * batch of up to `capacity` positions on table t. */
BLIP_API int blip_workspace_size(blip_table t, int64_t capacity, size_t* bytes);

/*
 * blip_eval_batched_static -- blip_eval_batched without a workspace argument
 * and without any allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The sort workspace lives in a fixed 4.5 MiB device array inside
 * the library, one per device, held until the process ends; its device
 * address is looked up once per device on the first call with that device
 * current.
 *
 *  t, pos, offsets, nw, val, grad, lap, stream: as blip_eval_batched.
 *  capacity  as blip_eval_batched, at most 131,072 positions (BLIP_E_ARG
 *            beyond; the 4.5 MiB covers the sort of that many positions on
 *            any table).
 * Results equal blip_eval_batched's bit for bit (the same kernels and launch
 * shape).  Every call on a device shares that device's array and the kernels
 * clear what must start at zero, so consecutive calls need nothing from the
 * caller; calls that overlap on one device (different streams, or host
 * threads racing to enqueue) race on the array and must be serialised by the
 * caller, e.g. on one stream.  No hipMalloc, hipFree or memset.
 */
BLIP_API int blip_eval_batched_static(blip_table t, const double* pos, const int64_t* offsets,
                                      int nw, int64_t capacity, void* val, void* grad, void* lap,
                                      void* stream);

/*
 * Plans: blip_eval_batched captured once into a HIP graph on fixed buffers,
 * then replayed with one hipGraphLaunch.  Between launches the caller may
 * rewrite the contents of pos and offsets (the device-side total may change
 * from launch to launch up to capacity); the buffers themselves must stay
 * alive until blip_plan_free.  The launch shape is fixed at creation.
 */
typedef struct blip_plan_s* blip_plan;
BLIP_API int blip_plan_create(blip_table t, const double* pos, const int64_t* offsets, int nw,
                              int64_t capacity, void* val, void* grad, void* lap,
                              void* workspace, size_t workspace_bytes, blip_plan* out);
BLIP_API int blip_plan_launch(blip_plan p, void* stream);
BLIP_API int blip_plan_free(blip_plan p);

/*
 * blip_submit -- one launch of a serving loop in one call: the requests'
 * positions (the moved electrons of several walkers, each an independent
 * evaluation, Sec. IV.A, Eq. (11.12.23.1)) are copied from host memory to
 * the launch's device buffer, evaluated, and an event is recorded, all on
 * stream, so that a scheduler pays one library call per launch.
 *
 *  plan == NULL: copy npos positions host_pos -> dev_pos, then blip_eval_ex
 *            (opts; NULL = the tuned kernel) on dev_pos with outputs
 *            val/grad/lap of at least npos rows.  host_off, noff, dev_off
 *            are ignored.
 *  plan != NULL: the plan's graph (blip_plan_create) on its own buffers:
 *            dev_pos and dev_off must be the buffers the plan captured,
 *            npos <= its capacity, and noff its nw + 1 offsets (host_off,
 *            offsets[nw] the total) are copied to dev_off before the replay;
 *            opts must be NULL and val/grad/lap are ignored (the plan's).
 *  host_pos  host double[npos][3]; pinned memory (hipHostMalloc) makes the
 *            copy asynchronous, and must then stay unchanged until event
 *            (or the stream) has completed; pageable memory is copied
 *            before the call returns.
 *  event     hipEventRecord'ed on stream after the launch (NULL: none).
 * Argument errors are returned before anything is enqueued.  No allocation.
 */
BLIP_API int blip_submit(blip_table t, blip_plan plan, const blip_eval_opts* opts,
                         const double* host_pos, int64_t npos, double* dev_pos,
                         const int64_t* host_off, int noff, int64_t* dev_off, void* val,
                         void* grad, void* lap, void* stream, void* event);

/*
 * blip_autotune -- time every launch shape (P positions per workgroup x o
 * table elements per lane) on the caller's buffers and keep the fastest for
 * this table and this size bucket (npos in [2^k, 2^(k+1))).  offsets == NULL
 * tunes blip_eval on blocks of npos positions (P in {1,2,4,8}): pos then
 * holds `rotate` consecutive blocks and timed launch i uses block i mod
 * rotate, so that a launch does not find its rows left in the caches by the
 * previous one; otherwise (rotate must be 1) it tunes blip_eval_batched with
 * capacity npos (P in {4,8,16,32,64}).  o runs over
 * {1,2,4} (FP32 storage) or {2,4,8} (16-bit storage).  Each shape is timed
 * as bursts of max(8, rotate) back-to-back launches (one untimed burst, then
 * five timed), the figure being the median over bursts of the mean time per
 * launch: the rate of a stream of steps, not the latency of one launch.
 * Synchronous: it synchronises the stream after each burst.  The outputs are
 * overwritten.  results (may be NULL) receives up to max_results timings;
 * best receives the winner.
 */
typedef struct {
    int tile_pos;   /* P */
    int vec;        /* o */
    double us;      /* per-launch time, microseconds (median over bursts) */
} blip_tune_result;
BLIP_API int blip_autotune(blip_table t, const double* pos, const int64_t* offsets, int nw,
                           int64_t npos, int rotate, void* val, void* grad, void* lap,
                           void* workspace, size_t workspace_bytes, void* stream,
                           blip_tune_result* results, int max_results, int* n_results,
                           blip_tune_result* best);

/* Launch-shape modes of blip_set_shape / blip_get_shape: the single-block
 * launch and the sorted persistent batch, each plain (orbitals stored) or
 * with the acceptance-ratio epilogue (blip_eval_ratio* calls).  A ratio
 * mode with no shape of its own runs its plain mode's shape, capped as the
 * epilogue needs (P <= 16 positions, at most 16 orbital chunks). */
typedef enum {
    BLIP_SHAPE_BLOCK = 0,          /* blip_eval, blip_eval_ex (tiled)          */
    BLIP_SHAPE_BATCHED = 1,        /* blip_eval_batched, plans                 */
    BLIP_SHAPE_BLOCK_RATIO = 2,    /* blip_eval_ratio, blip_eval_ratio_values  */
    BLIP_SHAPE_BATCHED_RATIO = 3   /* blip_eval_ratio_batched,
                                      blip_eval_ratio_values_batched           */
} blip_shape_mode;

/* blip_set_shape / blip_get_shape -- set or read the launch shape that mode
 * (a blip_shape_mode) uses for npos's size bucket, the power-of-two range
 * [2^k, 2^(k+1)) holding npos, e.g. to restore a cached autotuning result.
 * A size whose bucket has no shape of its own uses one set for an adjacent
 * bucket of the same mode (the larger if both are), else the built-in
 * default.  blip_get_shape reports what a launch of npos positions in that
 * mode would run.  Errors: BLIP_E_STATE (handle), BLIP_E_ARG (mode, npos < 1,
 * tile_pos outside 1..64, vec not valid for the table's storage). */
BLIP_API int blip_set_shape(blip_table t, int mode, int64_t npos, int tile_pos, int vec);
BLIP_API int blip_get_shape(blip_table t, int mode, int64_t npos, int* tile_pos, int* vec);

/*
 * blip_eval_ratio -- quasi-simultaneous acceptance ratios of the Slater part
 * (Eq. (11.12.23.1)) against the old inverse, fused into the evaluation so
 * that N numbers are written instead of N x L orbitals (real tables only):
 *
 *   ratio[j]         = sum_l psi_l(r'_j)      Dinv[l, c_j]
 *   grad_ratio[j][:] = sum_l grad psi_l(r'_j) Dinv[l, c_j]
 *   lap_ratio[j]     = sum_l lap psi_l(r'_j)  Dinv[l, c_j]
 *
 * ratio[j] is det(D')/det(D) for the Slater matrix D[i][l] = psi_l(r_i) with
 * row c_j replaced by the orbitals at the trial position r'_j; grad_ratio/ratio
 * and lap_ratio/ratio are its gradient and Laplacian in r'_j.
 *
 *  pos        device double[npos][3] trial positions (as blip_eval).
 *  inv_rows   device double: row r at inv_rows + r * inv_ld holds
 *             Dinv[l, c] for l = 0..L-1 (a column of the inverse, stored as a
 *             row: the transposed inverse); inv_ld >= L.
 *  row_of     device int64[npos]: the row position j uses (NULL: row j).
 *  ratio      device double[npos]; grad_ratio [npos][3] and lap_ratio [npos]
 *             device doubles, both or neither (NULL: values-only kernel).
 * The orbitals are summed in FP32 exactly as blip_eval does; the dot products
 * with the inverse are FP64 in a fixed order.  Pointers 8-byte aligned.
 * BLIP_E_DTYPE for complex tables; BLIP_E_ARG if L exceeds 16 lane chunks
 * (4,096 orbitals in FP32).  Asynchronous on the stream, no allocation.
 */
BLIP_API int blip_eval_ratio(blip_table t, const double* pos, int64_t npos,
                             const double* inv_rows, int64_t inv_ld, const int64_t* row_of,
                             double* ratio, double* grad_ratio, double* lap_ratio,
                             void* stream);

/*
 * blip_eval_ratio_values -- blip_eval_ratio that also writes the orbital
 * values, val [npos][L] float, exactly as blip_eval writes them: one pass
 * gives a quasi-simultaneous step both its ratios and the new orbital rows
 * that the inverse update (blip_sm_update*) needs for the accepted moves.
 * With grad_ratio, lap_ratio and lap (all three, or none) it is the full
 * blip_eval_ratio and also writes the Laplacian rows, lap [npos][L] float as
 * blip_eval writes them: the rows a caller keeps to evaluate the local
 * kinetic energy of the configuration it accepts without evaluating the
 * orbitals again (blip_qs_lap_ratios).  Same arguments and errors as
 * blip_eval_ratio; val is required; val and lap 4-byte aligned.
 */
BLIP_API int blip_eval_ratio_values(blip_table t, const double* pos, int64_t npos,
                                    const double* inv_rows, int64_t inv_ld, const int64_t* row_of,
                                    double* ratio, double* grad_ratio, double* lap_ratio,
                                    void* val, void* lap, void* stream);

/*
 * blip_eval_ratio_batched -- blip_eval_ratio for many walkers in one
 * persistent launch: positions concatenated and offsets as in
 * blip_eval_batched (only offsets[nw] is read, on the device), row_of[j]
 * (NULL: row j) selecting each position's row of the stacked transposed
 * inverses of all walkers; ratio outputs have capacity rows, of which the
 * first offsets[nw] are written.  Same workspace as blip_eval_batched.
 */
BLIP_API int blip_eval_ratio_batched(blip_table t, const double* pos, const int64_t* offsets,
                                     int nw, int64_t capacity, const double* inv_rows,
                                     int64_t inv_ld, const int64_t* row_of, double* ratio,
                                     double* grad_ratio, double* lap_ratio, void* workspace,
                                     size_t workspace_bytes, void* stream);

/*
 * blip_eval_ratio_values_batched -- blip_eval_ratio_values in the sorted
 * persistent launch of blip_eval_ratio_batched: the moved electrons of many
 * walkers (both spins) evaluated as one set of positions (Eq. (11.12.23.1)
 * makes every trial move independent), in spatial order so that moves of
 * different walkers near the same grid sites share the rows they read.
 * val [capacity][L] float is required.  grad_ratio [capacity][3] double,
 * lap_ratio [capacity] double and lap [capacity][L] float go together or not
 * at all, as in blip_eval_ratio_values.  Rows j < offsets[nw] are written at
 * index j (the caller's order).  The values and Laplacian rows equal
 * blip_eval's bit for bit; the ratios equal blip_eval_ratio_values' when both
 * run with the same orbitals per lane (blip_set_shape with
 * BLIP_SHAPE_BLOCK_RATIO and BLIP_SHAPE_BATCHED_RATIO), as they sum the same per-lane products
 * in the same order.  Same workspace and errors as blip_eval_ratio_batched,
 * plus BLIP_E_ARG without val and BLIP_E_ALIGN for val or lap not 4-byte
 * aligned.  Asynchronous on the stream; the sort and the evaluation make five
 * launches, capturable in a graph.
 */
BLIP_API int blip_eval_ratio_values_batched(blip_table t, const double* pos,
                                            const int64_t* offsets, int nw, int64_t capacity,
                                            const double* inv_rows, int64_t inv_ld,
                                            const int64_t* row_of, double* ratio, double* gratio,
                                            double* lratio, void* val, void* lap, void* workspace,
                                            size_t workspace_bytes, void* stream);

/*
 * blip_sm_update -- bring the inverse Slater matrix up to date after the
 * accepted moves of a step (Sec. VI.D; the Slater matrix of Eq. (5)):
 * the moves are applied in the given order, each as the Sherman-Morrison
 * rank-1 update of one electron's row.
 *
 * Conventions are those of blip_eval_ratio: D[i][l] = psi_l(r_i), one
 * electron per row, and the inverse is held transposed, B[i][l] = Dinv[l][i]
 * (the column of Dinv that electron i pairs with, stored as a row).  Moving
 * electron c replaces row c of D by u[l] = psi_l(r'_c); then
 *   ratio  = sum_l u[l] B[c][l],      v_i = sum_l u[l] B[i][l],
 *   B'[c]  = B[c] / ratio,            B'[i] = B[i] - (v_i / ratio) B[c]  (i != c).
 *
 *  n          matrix order (electrons of one spin = orbitals), 1..4096.
 *  inv        device double, B with row i at inv + i * inv_ld; updated in place.
 *  u          device float [u_nrows][u_ld], u_ld >= n: the new orbital rows
 *             (columns l < n are read) -- typically the val output of
 *             blip_eval for the step's trial positions.
 *  cols       HOST int64[k]: the accepted electrons, in the order the moves
 *             are applied; an electron may appear more than once.
 *  u_row      HOST int64[k] or NULL: the row of u holding move m's new
 *             orbitals (NULL: row cols[m], i.e. u ordered by electron).
 *  ratios     device double[k] or NULL: ratios[m] = det(D^(m)) / det(D^(m-1)),
 *             the ratio of move m against the matrix that already holds moves
 *             0..m-1 (so their product is det(D_new) / det(D_old)).
 *  workspace  device memory of blip_sm_workspace_size(n) bytes, 8-byte aligned,
 *             not shared with another call in flight.
 * Computed in FP64 (u converted exactly).  Up to 32 consecutive moves are
 * applied per launch in the equivalent rank-k (Woodbury) form, eliminating
 * the k x k block of moved rows without pivoting in move order -- the same
 * divisions by the sequential ratios the rank-1 updates make, so a ratio of
 * zero yields non-finite rows exactly as the rank-1 form would.
 * Asynchronous on the stream, no allocation; ceil(k/32)+1 launches (about
 * one more per repeated electron).  k = 0 enqueues nothing.  BLIP_E_ARG for
 * a size or index out of range, or when inv or u spans 2 GiB or more (the
 * kernels address a matrix with 31-bit byte offsets; at n <= 4096 only a
 * leading dimension far above n gets there), BLIP_E_ALIGN for misaligned
 * pointers.
 */
BLIP_API int blip_sm_update(int64_t n, double* inv, int64_t inv_ld, const float* u,
                            int64_t u_nrows, int64_t u_ld, const int64_t* cols,
                            const int64_t* u_row, int64_t k, double* ratios, void* workspace,
                            size_t workspace_bytes, void* stream);

/* blip_sm_workspace_size -- bytes of workspace blip_sm_update needs for
 * order n (0 if n is out of range). */
BLIP_API size_t blip_sm_workspace_size(int64_t n);

/*
 * blip_sm_update_batched -- blip_sm_update for many matrices at once (the
 * walkers and spins of a Monte Carlo step), with the accepted moves on the
 * device, as a quasi-simultaneous step produces them (Sec. IV.A; the update
 * of Sec. VI.D).
 *
 *  nmat        matrices, 0..65535; matrix q has order n (1..4096).
 *  inv         device double: B of matrix q at inv + q * inv_mstride, row i
 *              at + i * inv_ld (the layout of blip_sm_update); in place.
 *  u           device float: the new orbitals of electron c of matrix q at
 *              u + q * u_mstride + c * u_ld (u ordered by electron; n rows
 *              per matrix, columns l < n read).
 *  acc_cols    device int32 [nmat][acc_ld]: matrix q's accepted electrons in
 *              the order the moves are applied; each electron at most once
 *              per matrix (a quasi-simultaneous step moves each once).
 *  acc_count   device int32 [nmat]: moves of matrix q, clamped to [0, max_k].
 *  max_k       host bound on every count (0..n); sets the number of launches,
 *              2 * ceil(max_k / 32) + 2, whatever the counts are.
 *  ratios      device double [nmat][ratio_ld] or NULL: the sequential ratios,
 *              slot m of matrix q for its move m.
 *  workspace   blip_sm_batched_workspace_size(nmat, n) bytes, 16-byte aligned.
 * Entries of acc_cols outside [0, n) are clamped into it: wrong input gives
 * wrong results, never an out-of-bounds access; a repeated electron within a
 * matrix gives wrong results.  The arithmetic and its order are exactly those
 * of blip_sm_update on the same list, so the results are bitwise equal.
 * Everything is read on the device and the launch sequence depends only on
 * nmat, n and max_k: a step can be captured in a graph.  Asynchronous, no
 * allocation.  BLIP_E_ARG / BLIP_E_ALIGN on host-checkable errors (as for
 * blip_sm_update, one matrix of inv or u must span less than 2 GiB).
 */
BLIP_API int blip_sm_update_batched(int nmat, int64_t n, double* inv, int64_t inv_mstride,
                                    int64_t inv_ld, const float* u, int64_t u_mstride,
                                    int64_t u_ld, const int32_t* acc_cols, int64_t acc_ld,
                                    const int32_t* acc_count, int max_k, double* ratios,
                                    int64_t ratio_ld, void* workspace, size_t workspace_bytes,
                                    void* stream);

/* blip_sm_batched_workspace_size -- bytes of workspace blip_sm_update_batched
 * needs (0 if an argument is out of range). */
BLIP_API size_t blip_sm_batched_workspace_size(int nmat, int64_t n);

/*
 * Quasi-simultaneous Monte Carlo step helpers (Sec. IV.A; the step of Sec.
 * II.B: trial move, ratio, accept/reject, local energy).  Matrices are
 * (walker, spin) pairs q = 2 * walker + spin with n electrons each; arrays
 * indexed by electron are [nmat][n] (positions [nmat][n][3], bohr), so
 * electron j of matrix q is entry q * n + j.  All device pointers; all
 * asynchronous on the stream, no allocation.
 *
 * blip_qs_propose -- trial[p] = pos[p] + eta[p] for npos positions (the
 *   random displacements are the caller's).
 *
 * blip_qs_accept -- for every matrix, candidates j in [j0, j1) (all n for a
 *   quasi-simultaneous step; one electron for a configuration-by-
 *   configuration move): accepted when uniform < ratio^2, the Metropolis test
 *   for p = |Psi|^2 with the ratio of blip_eval_ratio against the old
 *   configuration (a NaN ratio is rejected).  Accepted electrons get
 *   pos = trial and are listed in increasing order in acc_cols[q * acc_ld ..]
 *   with acc_count[q] entries: the inputs of blip_sm_update_batched.
 *   acc_ld >= n; nmat <= 65535.
 *
 * blip_qs_kinetic -- e_kin[w] = -1/2 sum_{j < nel} lap_ratio[w * nel + j]:
 *   the local kinetic energy of walker w from the Laplacian ratios of
 *   blip_eval_ratio at its current positions against its current inverses
 *   (sum_l lap psi_l(r_j) Dinv[l, j] = lap_j Psi_D / Psi_D), summed in a fixed
 *   order.  nwalk <= 65535.
 *
 * blip_qs_copy_rows -- for each (walker, spin) matrix q < nmat, the rows
 *   q * n + acc_cols[q * acc_ld + i], i < acc_count[q], of src (row stride
 *   src_ld floats) copied to the same rows of dst (stride dst_ld): len floats
 *   each.  Carries the orbital rows evaluated at the trial positions (the
 *   Laplacian rows of blip_eval_ratio_values) into the rows kept for the
 *   current configuration, for the electrons blip_qs_accept accepted.
 *   Counts are clamped to [0, n] and list entries to [0, n).  acc_ld >= n,
 *   src_ld and dst_ld >= len; nmat <= 65535.
 *
 * blip_qs_lap_ratios -- lap_ratio[r] = sum_{l < len} lap[r][l] inv_rows[r][l]
 *   (FP64 sums of the FP32 rows in a fixed order), r < nrows: with the
 *   Laplacian rows of the orbitals at the current positions and the rows of
 *   the current transposed inverses, the Laplacian ratios lap_j Psi_D /
 *   Psi_D that blip_qs_kinetic sums, without evaluating the orbitals.
 *   lap_ld, inv_ld >= len; lap 4-byte, inv_rows and lap_ratio 8-byte aligned.
 */
BLIP_API int blip_qs_propose(int64_t npos, const double* pos, const double* eta, double* trial,
                             void* stream);
BLIP_API int blip_qs_accept(int nmat, int n, int j0, int j1, const double* ratio,
                            const double* uniform, const double* trial, double* pos,
                            int32_t* acc_cols, int64_t acc_ld, int32_t* acc_count, void* stream);
BLIP_API int blip_qs_kinetic(int nwalk, int nel, const double* lap_ratio, double* e_kin,
                             void* stream);
BLIP_API int blip_qs_copy_rows(int nmat, int n, int len, const int32_t* acc_cols, int64_t acc_ld,
                              const int32_t* acc_count, const float* src, int64_t src_ld,
                              float* dst, int64_t dst_ld, void* stream);
BLIP_API int blip_qs_lap_ratios(int64_t nrows, int len, const float* lap, int64_t lap_ld,
                               const double* inv_rows, int64_t inv_ld, double* lap_ratio,
                               void* stream);

/*
 * blip_stream_read -- measurement helper: read a device buffer once,
 * streaming, and write per-workgroup sums.  It gives the achievable HBM read
 * rate on this GPU, the second denominator (beside the 8 TB/s peak) for the
 * bandwidth fraction of the orbital evaluation, whose bound is the reading
 * of coefficient rows (a gather-weighted sum, Eq. (7)).
 *
 *  buf      device memory, 16-byte aligned, read as float4.
 *  bytes    a positive multiple of 16.
 *  partial  device float[nblocks]: partial[b] = FP32 sum of the floats that
 *           workgroup b read (the 32 KB pieces b, b + nblocks, ...), so that
 *           the sum of all partials covers every element once.
 *  nblocks  workgroups of 256 threads, 1..65535.
 * Asynchronous on the stream, no allocation.  BLIP_E_ARG / BLIP_E_ALIGN.
 */
BLIP_API int blip_stream_read(const void* buf, size_t bytes, float* partial, int nblocks,
                              void* stream);

/*
 * blip_stream_read_runs -- measurement helper, scattered form: read runs of
 * run_bytes contiguous bytes at the given offsets, the access pattern of a
 * block's coefficient rows (the 4 rows along a3 of a stencil line are one
 * run of 4 L floats at a scattered offset, Eq. (7)).  It gives the read rate
 * such a launch can reach, the ceiling for the orbital kernel's traffic.
 *
 *  buf          device memory of `bytes` bytes (a positive multiple of 16),
 *               16-byte aligned.
 *  run_offsets  device int64[nruns], byte offsets of the runs.  A run that is
 *               not 16-byte aligned or does not lie inside the buffer is
 *               skipped (never read out of bounds).
 *  run_bytes    4096, 8192, 12288, 16384, 24576 or 49152.
 *  partial      device float[nblocks]: partial[b] = FP32 sum of the floats
 *               of the runs b, b + nblocks, ... that workgroup b read.
 *  nblocks      workgroups of 256 threads, 1..65535.
 * Asynchronous on the stream, no allocation.  BLIP_E_ARG / BLIP_E_ALIGN.
 */
BLIP_API int blip_stream_read_runs(const void* buf, size_t bytes, const int64_t* run_offsets,
                                   int nruns, int run_bytes, float* partial, int nblocks,
                                   void* stream);

/* blip_table_info -- describe a table: L, storage dtype, row stride in bytes,
 * total device bytes.  Any output pointer may be NULL. */
BLIP_API int blip_table_info(blip_table t, int* norb, int* storage,
                             int64_t* row_bytes, int64_t* device_bytes);

/* blip_free -- release the table's device memory (synchronises the device
 * first so in-flight work finishes).  NULL is accepted and ignored. */
BLIP_API int blip_free(blip_table t);

/* blip_last_error -- thread-local message for the last non-zero status
 * returned on the calling thread ("" if none).  Owned by the library. */
BLIP_API const char* blip_last_error(void);

/* blip_version -- library version string (static storage). */
BLIP_API const char* blip_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BLIP_H */
