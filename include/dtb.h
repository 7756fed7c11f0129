/*
 * dtb.h -- libdtb: the j2d5pt iterative stencil under deep temporal blocking
 * on AMD Instinct MI355X (gfx950).
 *
 * The operation (Zhang et al., "Exploiting Scratchpad Memory for Deep
 * Temporal Blocking", GPGPU '23; Listing 1 gives the update, Section 3.1 and
 * the caption of Figure 1 repeat it for T time steps):
 *
 *   for t in 0 .. T-1, for every interior cell (i, j):
 *     u'[i][j] = w*u[i][j-1] + e*u[i][j+1] + s*u[i-1][j] + c*u[i][j] + n*u[i+1][j]
 *   then u = u'  (every read of a step sees the previous step's values).
 *
 * Storage: a device buffer of (rows + 2) lines of `pitch` elements,
 * row-major.  The interior is rows 1..rows, columns 1..cols; the one-cell ring
 * around it (rows 0 and rows+1, columns 0 and cols+1) is a fixed Dirichlet
 * halo: it is read but never written.  Corner halo cells are never read.
 * Elements past column cols+1 (pitch padding) are never touched.
 * Column j is the contiguous index (x in Listing 1), row i the strided one
 * (y); hence W = (i, j-1), E = (i, j+1), S = (i-1, j), N = (i+1, j).
 *
 * Coefficients are passed as five doubles in the order (c, n, s, e, w).  They
 * need not sum to 1 and are copied at the call.  DTB_F32 rounds them to float.
 *
 * The 3 x 3 box (j2d9pt), the next stencil shape of the same method (a plan
 * made with dtb_plan_opts.stencil = 9): every interior cell becomes the
 * weighted sum of the 3 x 3 block of cells centred on it,
 *     sw*u[i-1][j-1] + s*u[i-1][j] + se*u[i-1][j+1] + w*u[i][j-1] + c*u[i][j]
 *   + e*u[i][j+1] + nw*u[i+1][j-1] + n*u[i+1][j] + ne*u[i+1][j+1],
 * with the nine coefficients passed in that order (sw, s, se, w, c, e, nw, n,
 * ne) and summed in that order (fused multiply-adds by default, separately
 * rounded products with exact = 1).  The halo's corner cells are read.
 *
 * Arithmetic: by default each cell is a chain of one multiply and four fused
 * multiply-adds in the order W, E, S, C, N.  With dtb_plan_opts.exact = 1
 * the products are rounded separately and summed left to right in that same
 * order, which reproduces a plain CPU loop bit for bit.  No flush to zero.
 *
 * Every function returns a dtb_status; none aborts or prints.  Invalid
 * arguments are rejected before any HIP call.  Launches are asynchronous on
 * the given stream (a hipStream_t passed as void*; NULL is the default
 * stream).  The caller owns the grid and keeps it alive until the stream has
 * finished the work.
 */
#ifndef LIBDTB_DTB_H
#define LIBDTB_DTB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { DTB_F64 = 0, DTB_F32 = 1 } dtb_dtype;

typedef enum {
    DTB_OK = 0,
    DTB_ERR_INVALID_ARG = -1,    /* a NULL pointer, rows/cols < 1, pitch < cols+2, T < 0, bad dtype/option */
    DTB_ERR_UNSUPPORTED = -2,    /* shape or option the library does not handle */
    DTB_ERR_NOT_CORESIDENT = -3, /* the plan needs more workgroups than can run at once */
    DTB_ERR_OUT_OF_MEMORY = -4,  /* workspace allocation failed */
    DTB_ERR_HIP = -5,            /* a HIP runtime call or kernel launch failed */
    DTB_ERR_TIMEOUT = -6,        /* a bounded in-kernel wait expired (a workgroup never arrived) */
    DTB_ERR_NOT_PLANNED = -7,    /* the call needs a plan that does not exist */
    DTB_ERR_MISMATCH = -8        /* grid/dtype do not match the plan */
} dtb_status;

/* Execution paths a plan can take. */
typedef enum {
    DTB_PATH_AUTO = 0,     /* resident DTB when the grid fits on chip, else the tile-serial sweep */
    DTB_PATH_STEP = 1,     /* the untiled baseline: one kernel launch per time step, HBM to HBM */
    DTB_PATH_RESIDENT = 2, /* deep temporal blocking, whole grid held on chip for all T steps */
    DTB_PATH_SWEEP = 3,    /* deep temporal blocking, big tiles processed one after another (tile-serial) */
    DTB_PATH_OVERLAPPED = 4, /* overlapped per-workgroup blocking (Section 2's "overlapped tiling within
                               thread blocks"): one launch per depth_D steps, each workgroup loads its tile
                               with a depth_D-deep ring from HBM, advances it depth_D steps with no
                               synchronisation between workgroups and stores its owned cells; for comparison */
    DTB_PATH_STREAM3D = 5  /* j3d7pt (dtb_plan3d): 2.5D streaming with temporal blocking, ghost_k steps per
                              launch (see dtb_plan3d) */
} dtb_path;

/* A grid in device memory (see the storage description above). */
typedef struct {
    void* data;     /* device pointer to halo cell (0, 0); caller-owned */
    int64_t rows;   /* interior rows N >= 1 */
    int64_t cols;   /* interior columns M >= 1 */
    int64_t pitch;  /* elements per storage row, >= cols + 2 */
} dtb_grid;

/* Plan options.  Zero-initialise and set what you need; 0 means "choose". */
typedef struct {
    int32_t path;        /* dtb_path */
    int32_t ghost_k;     /* steps between inter-workgroup halo exchanges (ghost ring depth); 0 = auto */
    int32_t depth_D;     /* sweep: steps per round (temporal depth of a big tile); overlapped path: steps
                            per launch (ring depth of a tile); 0 = auto */
    int32_t rows_per_lane; /* register tile height per lane; 0 = auto.  Instantiated: FP64 8, 16, 24
                              (2 columns per lane) and 12 (4 columns per lane); FP32 8, 16, 24, 28
                              (4 columns per lane).  Tiles are 8 waves x rows_per_lane rows high. */
    int32_t max_wg;      /* cap on workgroups; 0 = every compute unit */
    int32_t exact;       /* 1: separately rounded products, plain left-to-right sum (bitwise CPU parity) */
    int32_t debug_flags; /* DTB_DEBUG_* bits; 0 in production */
    int32_t tune;        /* 1: time the best few candidate tilings on a scratch grid and keep the fastest
                            (results cached per shape/precision/device, and in the text file named by the
                            environment variable DTB_TUNE_CACHE if set); 0: static cost model only */
    int32_t waves;       /* waves per workgroup of the resident path: 8, or 4 (FP64, 24 rows per lane:
                            half-height tiles, two workgroups per compute unit so that one's exchange
                            overlaps the other's steps); 0 = choose */
    int32_t sync;        /* resident path, what a workgroup waits for at an exchange: 0 = the workgroups
                            whose cells it reads (neighbour epoch flags); 1 = every workgroup, at a
                            device-wide barrier (the grid-level barrier of Section 3.2; for comparison) */
    int32_t stencil;     /* 0 or 5: j2d5pt (five coefficients); 9: the 3 x 3 box (nine coefficients, see
                            above): step, resident and sweep paths, 8 waves, neighbour flags; register
                            tiles FP64 4 x 8 and FP32 4 x 16 per lane (rows_per_lane 8 / 16); 7: j3d7pt,
                            dtb_plan3d only */
    int32_t cols_per_lane; /* dtb_plan3d's streaming path only (0 elsewhere): columns per lane of the register
                              tile, 0 = choose.  Instantiated: FP64 2; FP32 4 and 3 (tiles 256 and 192 columns
                              wide; "choose" takes the one whose overlapping tiles compute fewer columns,
                              4 on a tie).  Any other value: DTB_ERR_UNSUPPORTED. */
} dtb_plan_opts;

/* A 3-D grid in device memory (dtb_plan3d): (depth + 2) planes of plane_pitch elements, each plane
   (rows + 2) lines of pitch elements; interior planes 1..depth, rows 1..rows, columns 1..cols; the one-cell
   shell around the interior is a fixed Dirichlet halo, read but never written (its edges and corners are
   never read). */
typedef struct {
    void* data;          /* device pointer to cell (0, 0, 0); caller-owned */
    int64_t depth;       /* interior planes >= 1 */
    int64_t rows;        /* interior rows >= 1 */
    int64_t cols;        /* interior columns >= 1 */
    int64_t pitch;       /* elements per row, >= cols + 2 */
    int64_t plane_pitch; /* elements per plane, >= (rows + 2) * pitch */
} dtb_grid3d;

/* Debug bits for dtb_plan_opts.debug_flags. */
#define DTB_DEBUG_TINY_SPIN 1 /* bounded in-kernel waits give up after a few polls: exercises the
                                 DTB_ERR_TIMEOUT path (results are then wrong, the kernel still drains) */
#define DTB_DEBUG_POISON 2    /* NaN-fill the exchange buffers before each run and every register cell
                                 outside the k-deep fresh region at each exchange: a stale or unsynchronised
                                 read, or a hole in the ghost ring, turns results into NaN */
#define DTB_DEBUG_TIMING 4    /* per-workgroup phase clocks (steps, publishing border strips, waiting for
                                 neighbours, loading the ghost ring): read them with dtb_plan_timing */
#define DTB_DEBUG_DIRECT_XCHG 8 /* move border strips lane by lane between registers and the exchange
                                   buffer instead of through the LDS staging area (same results) */

typedef struct dtb_plan_s* dtb_plan_t;

/* One problem of a batch: a grid, its coefficients (c, n, s, e, w), its step count and precision. */
typedef struct {
    dtb_grid grid;
    double coeffs[5];
    int64_t T;
    int32_t dtype;   /* dtb_dtype */
    int32_t reserved;
} dtb_problem;

/*
 * Build a plan for grids of this shape and precision: chooses the path, the
 * tile decomposition, the exchange depth and the workgroup count, checks that
 * every workgroup can be resident at once, and allocates the plan's device
 * workspace (exchange buffers, epoch flags, error word, descriptor tables).
 * (The paper: the whole-GPU tiling of the Abstract and Section 1 -- tiles
 * sized to the on-chip memory of all compute units; several steps per tile
 * between exchanges, Section 3.2; tiles processed one after another when the
 * grid is larger than the chip, Section 3.3 and Figure 1.)
 * T_hint is the expected step count (0 = unknown).  opts may be NULL.
 * On success *out receives the plan; release it with dtb_plan_destroy.
 * Allocates; not for use under stream capture.
 */
dtb_status dtb_plan(dtb_plan_t* out, int64_t rows, int64_t cols, int64_t pitch, dtb_dtype dtype,
                    int64_t T_hint, const dtb_plan_opts* opts);

/*
 * Advance grid->data by T steps in place with an explicit plan (Listing 1's
 * update repeated T times, Section 3.1 and Figure 1; the 3 x 3 box for a plan
 * made with stencil = 9).  coeffs: five doubles (c, n, s, e, w), or nine (sw,
 * s, se, w, c, e, nw, n, ne) for a box plan.  The grid's
 * rows, cols, pitch and dtype must match the plan.  T == 0 returns DTB_OK
 * without launching.  The plan's workspace serves one run at a time: a call
 * on another stream than the plan's previous run waits for that run first
 * (outside stream capture; inside it, runs are ordered by the capturing
 * stream).  Calls on other plans may overlap.  Does not allocate.
 */
dtb_status dtb_run_plan(dtb_plan_t plan, const dtb_grid* grid, const double* coeffs, int64_t T,
                        void* stream);

/*
 * Advance grid->data by T steps in place (Listing 1's update repeated T
 * times, Section 3.1 and Figure 1), using a plan cached by (rows, cols,
 * pitch, dtype, device), created on first use with default options.
 * Creating the plan allocates; later calls do not.  Calls on the same cached
 * plan are ordered: a call on another stream than the previous one waits for
 * the previous run first (outside stream capture).
 */
dtb_status dtb_run(const dtb_grid* grid, const double coeffs[5], int64_t T, dtb_dtype dtype,
                   void* stream);

/*
 * Run `count` independent problems (uneven shapes, step counts and
 * precisions) in one persistent launch -- each problem the operation of
 * dtb_run (Listing 1, Section 3.1).  The first call for a given set of
 * shapes/precisions/step counts plans each problem, packs their workgroups
 * onto the compute units and captures the launch in a HIP graph; later calls
 * with the same signature update the grid pointers and coefficients and
 * replay the graph.  Each grid is updated in place as dtb_run would.  The
 * planner picks, per problem, the register-tile shape (two per precision),
 * the exchange depth and, for grids larger than the chip, the round depth.
 * Calls with the same signature share one descriptor table: a call on
 * another stream than the previous one waits for it first.
 */
dtb_status dtb_run_batched(const dtb_problem* problems, int32_t count, void* stream);

/*
 * Wait for `stream` and report an in-kernel failure (DTB_ERR_TIMEOUT)
 * recorded by any batched launch since the previous check; clears it.
 */
dtb_status dtb_batch_check(void* stream);

/*
 * Wait for the plan's last run on `stream` and report an in-kernel failure
 * (DTB_ERR_TIMEOUT) recorded since the previous check; clears it.
 */
dtb_status dtb_plan_check(dtb_plan_t plan, void* stream);

/*
 * Phase clocks of a plan made with DTB_DEBUG_TIMING, accumulated over its runs
 * since the previous call (which this call resets): waits for `stream`, then
 * fills up to `n` uint64 values, 11 per workgroup in launch order: ticks (of
 * the GPU's 100 MHz real-time clock) spent in steps, publishing border strips,
 * waiting for neighbours, loading the ghost ring; number of exchanges; total
 * ticks of those; then, when border strips go through the LDS staging area,
 * the ticks spent moving the published strips from registers to LDS and the
 * loaded ring from the buffer to LDS (not counted in the publishing and
 * loading figures); then ticks spent loading extended tiles, storing owned
 * cells, and (tile-serial sweep) in the barriers between big tiles (the
 * split-phase wait inside a round, the device-wide barrier at its end; these
 * three outside the total).  DTB_ERR_NOT_PLANNED if the plan has no
 * clocks.
 */
dtb_status dtb_plan_timing(dtb_plan_t plan, uint64_t* out, int32_t n, void* stream);

/*
 * Describe a plan: fills up to `n` int64 values in this order: path,
 * workgroups, ghost_k, depth_D, ext_rows, ext_cols, tiles_rows, tiles_cols,
 * rows_per_lane, cols_per_lane, big_tiles, exact, waves, sync, stencil (5 or 9).
 * Returns DTB_OK.
 */
dtb_status dtb_plan_describe(dtb_plan_t plan, int64_t* values, int32_t n);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: dtb_run for
 * grids held on chip (the resident path, default fused chain), with no
 * allocation of any kind.  The kernels' workspace (descriptor table, epoch
 * flags, error word, two exchange buffers) lives in a fixed area of
 * DTB_NOALLOC_SCRATCH_BYTES that the library reserves on every GPU it runs on
 * and holds until the process ends; each call lays the table out there and
 * clears the flags before its launch, and the host plans with fixed-size
 * arrays.  Results equal dtb_run's bit for bit.
 *
 * grid, coeffs, T, dtype: as for dtb_run.  The grid's storage,
 * (rows + 2) * pitch elements, must fit one exchange buffer,
 * DTB_NOALLOC_MAX_BUFFER_BYTES (FP64: 2,359,296 elements, e.g. 1534 x 1534;
 * FP32: twice that), else DTB_ERR_UNSUPPORTED; a grid that does not fit on
 * chip in one wave of workgroups (at most 256, 32 per axis) gives
 * DTB_ERR_NOT_CORESIDENT.  Both are decided before any launch; invalid
 * arguments are rejected before any HIP call.
 * err_flag: NULL, or a caller-owned device int32 into which the run ORs a
 * nonzero value if one of its bounded in-kernel waits expired (the caller
 * clears it and reads it when the stream has finished).
 * Every call on one GPU shares that GPU's area, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads) race
 * and must be ordered by the caller.  Three launches on `stream`: table
 * set-up, the persistent kernel, and (with err_flag) the error report.
 */
#define DTB_NOALLOC_MAX_BUFFER_BYTES (18u << 20)
#define DTB_NOALLOC_SCRATCH_BYTES (40960u + 1048576u + 256u + 2u * DTB_NOALLOC_MAX_BUFFER_BYTES)
dtb_status dtb_run_noalloc(const dtb_grid* grid, const double coeffs[5], int64_t T, dtb_dtype dtype,
                           int32_t* err_flag, void* stream);

/*
 * The 3-D seven-point stencil j3d7pt -- Listing 1's update with the two
 * neighbours of the third axis, repeated T times (Section 3.1, Figure 1); the
 * 2.5D tiling of 3-D stencils is among the designs of Section 2:
 *   u'[z][i][j] = w*u[z][i][j-1] + e*u[z][i][j+1] + s*u[z][i-1][j] + c*u[z][i][j]
 *               + n*u[z][i+1][j] + b*u[z-1][i][j] + t*u[z+1][i][j],
 * products summed in that order (fused multiply-adds by default, separately
 * rounded products with exact = 1); coefficients passed as (c, n, s, e, w, t, b).
 *
 * dtb_plan3d: plan for 3-D grids of this shape and precision and allocate the
 * workspace (a second grid buffer, the tile table).  Paths: DTB_PATH_AUTO or
 * DTB_PATH_STREAM3D -- 2.5D streaming: each workgroup owns an (x, y) column
 * tile over a block of depth_D planes, streams it plane by plane and advances
 * it ghost_k (1 .. 3, default 3) steps per launch through a register pipeline
 * of time levels, with a ghost_k-deep ring of redundant cells in every axis
 * and no synchronisation between workgroups -- or DTB_PATH_STEP (one launch per
 * step, HBM to HBM).  Options other than path, ghost_k, depth_D (0 = chosen by
 * the planner), rows_per_lane (0 or the instance's: 4), cols_per_lane (0 or an
 * instance's: FP64 2 x 4, FP32 4 x 4 and 3 x 4 cells per lane and plane),
 * max_wg, exact and stencil (0 or 7) must be 0: DTB_ERR_UNSUPPORTED.  Invalid shapes: DTB_ERR_INVALID_ARG, before any HIP
 * call.  Allocates; describe() reports big_tiles = z-blocks and stencil = 7.
 */
dtb_status dtb_plan3d(dtb_plan_t* out, int64_t depth, int64_t rows, int64_t cols, int64_t pitch,
                      int64_t plane_pitch, dtb_dtype dtype, const dtb_plan_opts* opts);

/*
 * Advance a 3-D grid by T steps in place with a plan from dtb_plan3d; coeffs:
 * seven doubles (c, n, s, e, w, t, b).  The grid's shape must match the plan
 * (DTB_ERR_MISMATCH; also for a 2-D plan).  Ordering as dtb_run_plan (one run
 * at a time per plan; a run on another stream waits for the previous run).
 * Does not allocate.
 */
dtb_status dtb_run3d_plan(dtb_plan_t plan, const dtb_grid3d* grid, const double* coeffs, int64_t T,
                          void* stream);

/* Release a plan and its workspace (after its work has completed).  NULL is a no-op. */
void dtb_plan_destroy(dtb_plan_t plan);

/* Drop every cached plan (dtb_run's and dtb_run_batched's); call when no work is in flight. */
void dtb_cache_clear(void);

/* A static string naming the status. */
const char* dtb_status_string(dtb_status s);

#ifdef __cplusplus
}
#endif

#endif /* LIBDTB_DTB_H */
