/*
 * eik.h -- C ABI of the MI355X (gfx950) Eikonal solver.
 *
 * Solves the first-order upwind discretisation of |grad u| F = 1 on a uniform 3D grid
 * (Chacon & Vladimirsky, "A parallel Heap-Cell Method for Eikonal equations", Section 1.1,
 * eq. (2)): at every node outside the exit set,
 *     sum over axes of max(D^-U, -D^+U, 0)^2 = 1 / F^2,
 * with U = q on the exit nodes and U = +inf beyond the grid (the exit set Q of eq. (1); the rest
 * of the boundary is non-inflow).  The solver follows the Heap-Cell Method (Section 4,
 * Algorithms 1 and 2) and its parallel form (Section 5, Algorithm 3): the grid is split into
 * cubic cells of `cell` nodes per side, cells are swept with Gauss-Seidel / locking-sweeping
 * updates, and a worklist of the cells whose boundary changed decides which cells are swept: by
 * default every queued cell in each round; with a band (eik_options.delta) only those whose cell
 * value (eq. (3)) lies within delta of the smallest queued one.
 * The discrete solution is unique, so the result does not depend on cell size, schedule or
 * processing order (Section 4, "Assigning Cell Values") beyond rounding.
 *
 * Conventions
 *   grid    dims = {nx, ny, nz}; node (i, j, k) lies at (i h, j h, k h).  Every node array is
 *           row-major with i fastest: index = i + nx * (j + ny * k), i.e. C order [nz][ny][nx].
 *   memory  Pointers marked "device" must be device memory of the current HIP device (or
 *           managed memory).  The caller owns every buffer it passes; the library owns only
 *           its per-stream workspace, which it allocates on first use, grows when a larger
 *           problem arrives on the same stream, and frees in eik_release().
 *   streams All GPU work of a call is enqueued on `stream` (NULL = the default stream) and the
 *           call returns once it is enqueued.  Calls on different streams may run concurrently;
 *           each stream has its own workspace.  Calls on one stream are ordered by the stream.
 *   process The solve kernel is a cooperative launch, which the HIP runtime grants to one
 *           process per device at a time.  While another process holds it, a solve falls back
 *           to one ordinary launch per round, driven by the calling thread (EIK_SCHED_AUTO,
 *           see eik_options.schedule), which blocks the call until the solve ends.  Serve many
 *           callers of one GPU from one process (streams, batches, a server).
 *   errors  A negative return value is a synchronous error: nothing was enqueued and u_out is
 *           untouched.  Conditions found on the device (invalid speeds, a cap on rounds) are
 *           recorded in the stream's workspace and returned by eik_stream_status(); u_out then
 *           holds an upper bound of the solution (values only decrease during the solve).
 */
#ifndef EIK_H_
#define EIK_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define EIK_OK 0
#define EIK_EINVAL (-1)     /* invalid argument                                              */
#define EIK_ENOMEM (-2)     /* device or pinned-host allocation failed                       */
#define EIK_EHIP (-3)       /* a HIP runtime call failed                                     */
#define EIK_ENOCONV (-4)    /* the round cap was reached before the worklist emptied         */
#define EIK_ECANCELLED (-5) /* the solve was stopped by the device watchdog                  */
#define EIK_EBUSY (-6)      /* a server has no room for the problem now (retry after a step)  */
#define EIK_ETOOBIG (-7)    /* eik_solve_noalloc: the workspace exceeds its static scratch    */

/* Element types of F. */
#define EIK_F64 0
#define EIK_F32 1

/* Arithmetic modes (eik_options.mode). */
#define EIK_MODE_FP64 0  /* all storage and arithmetic in FP64                            */
/* Values stored and swept in FP32 (half the value and face bytes, FP32 comparisons and sorting,
 * FP32 one- and two-term roots) with the three-term root of eq. (2) computed in FP64 from the
 * FP32 inputs and rounded once; the result is widened to FP64 in u_out.  Accuracy is that of
 * FP32 storage accumulated along characteristics (max relative error about 1e-5, mean about
 * 1e-7 on the grids here), not the FP64 bar; exit values are rounded to FP32. */
#define EIK_MODE_FP32 1
/* FP32 bulk, FP64 polish: the method runs in EIK_MODE_FP32, its result is lifted (times
 * 1 + max(2^-12, n 2^-20), n the longest side: an empirical margin over the FP32 error, not a
 * proven bound), the exits are re-seeded at their exact values, and the FP64 method runs from
 * there: the exits' cells decrease first and every changed face tags the cell downwind of it,
 * so only cells whose boundary changes are swept.  Values only decrease, so the polish ends at
 * the FP64 solution wherever the lifted start was not below it.  The polished result is then
 * checked against eq. (2) at every node (each node's local solve must return its own value to
 * within 1e-11 s + 2^-46 U); a grid that fails is solved again from +inf in FP64 on the same
 * stream (counted in eik_stats.polish_redone), so the result meets the EIK_MODE_FP64 accuracy
 * either way.  With tol > 0 the check is skipped (early termination stops above the fixed
 * point by design).  The polish costs about as much as an FP64 solve from +inf (it needs the
 * same chain of rounds), so the mode is slower than EIK_MODE_FP64 by the FP32 phase.  Single
 * solves and batches only. */
#define EIK_MODE_MIXED 2

/* Cell values (eik_options.cell_value), the keys of the priority band:
 *   EIK_CELL_VALUE_NEW  the cell value of Section 4 ("Assigning Cell Values", eq. (3)): the
 *                       smallest newly decreased inflow value across the shared face; reset to
 *                       +inf whenever the cell is taken.
 *   EIK_CELL_VALUE_OLD  the authors' earlier heuristic (Section 6, "Other cell values",
 *                       eq. (4)): the largest such value plus (r h + h) / 2 over the speed at
 *                       the middle of the tagged cell, combined by min with the cell's previous
 *                       value, which is never reset. */
#define EIK_CELL_VALUE_NEW 0
#define EIK_CELL_VALUE_OLD 1

/* How the rounds of a solve are driven (eik_options.schedule):
 *   EIK_SCHED_AUTO         one cooperative launch runs every round, with a grid barrier between
 *                          rounds; if the runtime refuses the cooperative launch (another
 *                          process on the device holds one, or the device cannot host the
 *                          grid at once) the call falls back to EIK_SCHED_HOST_LOOP.
 *   EIK_SCHED_COOPERATIVE  the cooperative launch only (EIK_EHIP if it is refused).
 *   EIK_SCHED_HOST_LOOP    one ordinary launch per round, enqueued by the calling thread in
 *                          batches; it waits for the stream after each batch to see whether the
 *                          worklist has emptied, so the call blocks until the solve ends.  Needs
 *                          no co-residency of the workgroups.  Same results. */
#define EIK_SCHED_AUTO 0
#define EIK_SCHED_COOPERATIVE 1
#define EIK_SCHED_HOST_LOOP 2
/*   EIK_SCHED_ASYNC        no rounds (the pHCM main loop of Section 5 without per-thread heaps):
 *                          one cooperative launch in which every wave pops a queued cell from
 *                          a device ring, visits it and pushes the neighbours it tags, with no
 *                          barrier between visits.  With delta = 0 cells are taken in the
 *                          order they were queued; with delta > 0 they are kept in 64 buckets
 *                          of cell values of width delta (the heap of Algorithm 1 coarsened to
 *                          buckets) and each wave takes a cell of the lowest non-empty bucket
 *                          (the workspace then holds 64 rings of cells + 16384 8-byte entries).
 *                          When nothing is queued or being visited
 *                          the launch checks every cell against eq. (2) and re-queues any cell
 *                          with a node above its local solve, so the result is the same fixed
 *                          point.  Single solves and batches (EIK_EINVAL for a server); falls
 *                          back to EIK_SCHED_HOST_LOOP if the cooperative launch is refused. */
#define EIK_SCHED_ASYNC 3

/* In-cell solvers (eik_options.inner).  All solve the cell sub-problem of Section 4 exactly:
 *   EIK_INNER_SWEEP  locking sweeps (Algorithm 2) in the 8 directions, each sweep visiting the
 *                    diagonal planes x'+y'+z' = p of the cell in order (one plane per wave step);
 *   EIK_INNER_LIST   relaxation over a compacted list of active nodes: every pass evaluates the
 *                    listed nodes in dense 64-lane chunks and a node that decreases lists its
 *                    larger neighbours (Algorithm 2 activation without an ordering of nodes);
 *   EIK_INNER_DUAL   the locking sweeps run as two streams on the cell at once, half a sweep
 *                    apart, with directions that never put one node in both streams' planes;
 *                    cells of 4 and 8 only (EIK_EINVAL at 16).
 * At r = 16 a plane holds up to 192 nodes and is swept in up to three 64-node steps; a worker's
 * cell takes 78 KiB of LDS in FP64 (39 KiB in FP32), so a CU holds two (four) such workers. */
#define EIK_INNER_SWEEP 1
#define EIK_INNER_LIST 2
#define EIK_INNER_DUAL 3
/*   EIK_INNER_PAIR   the locking sweeps of EIK_INNER_SWEEP on two cells of a round at once, one
 *                    wave sweeping both half a sweep apart (each cell its own directions, stop
 *                    test and cap), so a wave instruction serves up to twice the nodes; cells
 *                    of 4 and 8 only, not with EIK_SCHED_ASYNC (EIK_EINVAL).  A CU holds half
 *                    as many such waves in FP64 (two cells' LDS each). */
#define EIK_INNER_PAIR 4

/* Exit set Q' and its values q (Section 4 notation: Q' = X intersect Q, values prescribed). */
typedef struct eik_sources {
    int64_t n;            /* number of exit nodes, >= 0 (0: every value is +inf)            */
    const int64_t* idx3;  /* n x 3 node indices (i, j, k), 0 <= i < nx etc.                 */
    const double* q;      /* n exit values, finite and >= 0; a node listed twice keeps min q */
    int on_device;        /* 0: idx3 and q are host memory (validated synchronously);
                             1: device memory (validated on the device, see errors above)   */
} eik_sources;

/* Optional knobs; zero-initialise for the defaults. */
typedef struct eik_options {
    int mode;             /* EIK_MODE_*; default EIK_MODE_FP64                               */
    double delta;         /* width of the cell-value band swept per round (the lowest bucket
                             of the priority worklist): cells with value < min + delta are
                             swept, the rest wait.  0 = default (+inf: every queued cell).
                             In a batch of several grids and in a server, min is taken per
                             grid (the smallest value queued in that grid).                 */
    int64_t max_rounds;   /* cap on worklist rounds; 0 = default (1 << 20)                    */
    int max_sweeps;       /* cap on sweeps (list passes) per cell visit: a visit that reaches
                             it publishes its changes, keeps its active nodes and re-queues
                             the cell; 0 = default (8 for sweeps, 512 otherwise)            */
    int workers;          /* persistent workgroups (one fills a CU); 0 = one per CU          */
    uint64_t shuffle;     /* 0 = natural order; otherwise seed of a pseudo-random permutation
                             of the order in which queued cells are taken (order tests)     */
    int timing;           /* 1: record HIP events around the solve kernel and the whole solve
                             of every call on the stream (read with eik_kernel_times)       */
    int64_t* round_log;   /* NULL, or a device array of 2 * round_log_len int64: for round t
                             < round_log_len, [2t] = cells in the round's list and [2t+1] =
                             shader-clock cycle count when the round ended (analysis)       */
    int64_t round_log_len;
    int inner;            /* in-cell solver: 0 = default (EIK_INNER_SWEEP at cell 8 and 16,
                             EIK_INNER_LIST at cell 4), or one of EIK_INNER_*                */
    int cell_value;       /* EIK_CELL_VALUE_NEW (default) or EIK_CELL_VALUE_OLD; only the
                             priority band (delta) reads cell values                        */
    int schedule;         /* EIK_SCHED_*; default EIK_SCHED_AUTO                             */
    uint64_t jitter;      /* 0 = none; otherwise seed of pseudo-random delays (0 to ~50 us)
                             before every cell visit, which make the visits of a round, or of
                             the ring, interleave in different orders (tests of the races that
                             Section 5.1 declares benign); the result is the same             */
} eik_options;

/* Per-solve counters, filled by eik_stream_status(). */
typedef struct eik_stats {
    int64_t rounds;       /* worklist rounds executed                                        */
    int64_t visits;       /* cell visits (one pop-and-sweep of one cell)                     */
    int64_t sweeps;       /* directional sweeps over all visits                              */
    int64_t updates;      /* local solves evaluated (grid-node updates)                      */
    int64_t deferred;     /* queued cells left for a later round by the priority band       */
    int64_t requeued;     /* visits that hit max_sweeps and re-queued their cell             */
    int64_t cells;        /* cells in the decomposition                                      */
    int64_t status;       /* same as the return value of eik_stream_status()                 */
    int64_t workers;      /* persistent workers (wave64) that ran                            */
    int64_t cycles_pop;   /* shader-clock cycles summed over workers: taking cells off the list */
    int64_t cycles_stage; /*   loading cells, halos and speeds into LDS                       */
    int64_t cycles_sweep; /*   in-cell sweeps                                                 */
    int64_t cycles_write; /*   write-back and tagging of neighbour cells                      */
    int64_t cycles_wait;  /*   publishing the next list and waiting at the round barrier      */
    int64_t sweep_hist[32];             /* visits by sweep count (bucket 31: 31 or more)      */
    int64_t visit_cycles_log2_hist[32]; /* visits by duration, bucket floor(log2(cycles))     */
    int64_t polish_redone; /* polished grids (EIK_MODE_MIXED, u_approx) whose result failed the
                              eq. (2) check and were solved again from +inf in FP64           */
} eik_stats;

/*
 * eik_solve -- solve eq. (2) on one grid.
 *   dims     host array {nx, ny, nz}, each >= 2, product < 2^31, and the grid rounded up to
 *            whole cells (ceil(n / cell) * cell per axis) also below 2^31 nodes.
 *   h        grid step, finite and > 0.
 *   F        device array of nx*ny*nz speeds of type f_dtype, each finite and > 0, with
 *            s = h / F between 2^-500 and 2^500 (between 2^-60 and 2^60 in EIK_MODE_FP32 and
 *            EIK_MODE_MIXED), the range in which the local solve's squares stay normal numbers;
 *            checked on the device, a violation yields EIK_EINVAL from eik_stream_status().
 *   f_dtype  EIK_F64 or EIK_F32.  Speeds are widened exactly to FP64; s = h / F is formed in
 *            FP64 (and rounded once to FP32 in EIK_MODE_FP32).
 *   sources  exit nodes and values (see eik_sources).
 *   u_out    device array of nx*ny*nz doubles; receives U (+inf where no exit node is reachable,
 *            q at exit nodes).  May not alias F.
 *   cell     cell side r in nodes: 4, 8 or 16.  Cells are anchored at node 0; the last layer of
 *            cells along an axis is partial when r does not divide the node count.
 *   tol      kappa >= 0, the early-termination threshold of the "early sweep termination"
 *            subsection: sweeping inside a cell stops after a sweep whose largest decrease is
 *            <= tol.  0 runs every cell to an exact floating-point fixed point.  Neighbour
 *            cells are re-queued on any strict decrease of a border value regardless of tol.
 *   stream   hipStream_t to enqueue on.
 * Returns EIK_OK or a negative code (nothing enqueued).
 */
int eik_solve(const int64_t dims[3], double h, const void* F, int f_dtype,
              const eik_sources* sources, double* u_out, int cell, double tol,
              hipStream_t stream);

/* eik_solve with options (NULL options = defaults). */
int eik_solve_ex(const int64_t dims[3], double h, const void* F, int f_dtype,
                 const eik_sources* sources, double* u_out, int cell, double tol,
                 hipStream_t stream, const eik_options* options);

/*
 * eik_solve_noalloc -- eik_solve_ex for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation.  Same arguments, results and
 * device-side status (eik_stream_status, eik_batch_status) as eik_solve_ex, but the call
 * allocates nothing: no hipMalloc, hipFree, pinned or staging buffer and no events.  Its
 * workspace is a static device array of 384 MiB (EIK_NOALLOC_SCRATCH_BYTES) that every device
 * the library runs this entry point on holds until the process ends; the slot table and
 * host-side exits reach the device through kernel arguments.
 *   limits   the workspace (eik_query_workspace(dims, cell, f_dtype, mode) plus 1 KiB for
 *            host-side exits) must fit the scratch, else EIK_ETOOBIG and nothing is enqueued:
 *            up to 257^3 nodes at cell 8 in EIK_MODE_FP64 with FP32 speeds, 248^3 in
 *            EIK_MODE_MIXED.  Host-side exits: at most 32 (EIK_EINVAL beyond; pass device
 *            arrays, sources.on_device = 1, for more).  options.timing must be 0 (EIK_EINVAL).
 *   set-up   the first call on a device (and the first after eik_release) looks up that
 *            device's copy of the array and creates the two events that order solve kernels
 *            on the device; later calls do no set-up.
 *   sharing  every call on a device uses that device's one array, which keeps the last call's
 *            contents (each call initialises what it reads).  Calls whose work overlaps on one
 *            GPU race on the array and corrupt each other's results: serialise them (one
 *            stream, or events).  A call that falls back to the host-driven round loop
 *            (EIK_SCHED_AUTO with the cooperative launch refused) blocks as described there.
 * Returns EIK_OK, EIK_EINVAL, EIK_ETOOBIG or EIK_EHIP (nothing enqueued on failure).
 */
#define EIK_NOALLOC_SCRATCH_BYTES ((size_t)384 << 20)
int eik_solve_noalloc(const int64_t dims[3], double h, const void* F, int f_dtype,
                      const eik_sources* sources, double* u_out, int cell, double tol,
                      hipStream_t stream, const eik_options* options);

/* Device bytes of the workspace one solve of this size needs (for admission control).
 * f_dtype as in eik_solve.  Returns EIK_OK or EIK_EINVAL. */
int eik_query_workspace(const int64_t dims[3], int cell, int f_dtype, int mode, size_t* bytes);

/* Device bytes of one grid's arrays inside a server pool (values, speeds, face copies) in the
 * given mode (EIK_MODE_*).  Returns EIK_OK or EIK_EINVAL. */
int eik_problem_bytes(const int64_t dims[3], int cell, int f_dtype, int mode, size_t* bytes);

/* Waits for all work on `stream`, then returns the device-side status of the last solve
 * enqueued on it (EIK_OK, EIK_EINVAL, EIK_ENOCONV, EIK_ECANCELLED) and, if stats != NULL,
 * its counters.  Returns EIK_EINVAL if no solve was ever enqueued on the stream. */
int eik_stream_status(hipStream_t stream, eik_stats* stats);

/* Asks every solve enqueued on `stream` so far (eik_solve, eik_solve_ex, eik_solve_batch) to
 * stop: a running solve kernel stops at its next round boundary (or within a few visits without
 * rounds) and the stream's status becomes EIK_ECANCELLED; u_out then holds an upper bound of
 * the solution, as after any early stop.  Solves enqueued after the call are not affected.  The
 * request is a store into host memory that the device reads; it does not wait.  Not for
 * eik_solve_noalloc or servers.  Returns EIK_OK, or EIK_EINVAL if nothing was ever solved on
 * the stream. */
int eik_cancel(hipStream_t stream);

/* Durations of the last n timed solves on `stream` (those enqueued with options.timing = 1),
 * oldest first: solve_ms[i] = the persistent solve kernel alone, total_ms[i] = the whole call
 * (staging, seeding, solve, output).  Either array may be NULL.  Waits for the stream.  At most
 * the last 256 solves are kept.  Returns the number of entries written (0 if none), or a
 * negative code. */
int eik_kernel_times(hipStream_t stream, int n, double* solve_ms, double* total_ms);

/* One configuration tried by eik_autotune and its time. */
typedef struct eik_tune_entry {
    int cell;             /* r: 4, 8 or 16                                                    */
    int inner;            /* EIK_INNER_SWEEP, EIK_INNER_LIST, EIK_INNER_DUAL or EIK_INNER_PAIR  */
    int workers;          /* persistent workgroups (0 = one per CU)                            */
    double delta;         /* priority band width (0 = every queued cell each round)            */
    double ms;            /* fastest of `reps` whole eik_solve_ex calls (stream events);       */
                          /* +inf if the configuration did not finish with EIK_OK               */
    int status;           /* device status of its last run                                    */
} eik_tune_entry;

/*
 * eik_autotune -- time the solver's configurations on one problem and return the fastest.
 * The best cell size, in-cell solver, worker count and priority band depend on the problem
 * (Section 6 finds the best cell size problem-dependent), so they are measured, not guessed:
 * every combination of r in {8, 4, 16}, inner in {SWEEP, LIST, DUAL, PAIR} (DUAL and PAIR up to
 * r = 8) and
 * workers in {all, half the CUs} with no band, then the best of those with bands of 4, 16 and 64 cell
 * crossings (delta = 4 r h, 16 r h, 64 r h).  Each configuration is solved once to warm up and `reps` (1..100)
 * times timed; the problem's arguments are those of eik_solve_ex (u_out receives the result of
 * the last run; every configuration computes the same U up to rounding).  Blocks until done.
 * table (cap entries, may be NULL if cap = 0) receives every configuration tried, *n_out their
 * number (may be NULL); *best the fastest one.  Returns EIK_OK, EIK_EINVAL (invalid problem or
 * arguments), a host error, or EIK_ECANCELLED if no configuration finished with EIK_OK.
 */
int eik_autotune(const int64_t dims[3], double h, const void* F, int f_dtype,
                 const eik_sources* sources, double* u_out, double tol, hipStream_t stream,
                 int reps, eik_tune_entry* table, int cap, int* n_out, eik_tune_entry* best);

/*
 * One problem of a batch or of a server: the arguments of eik_solve for one grid, and
 * optionally an approximation to polish.
 *
 * u_approx (device, nx*ny*nz doubles in the layout of u_out, or NULL): a solution of eq. (2)
 * that is accurate to about single precision, e.g. the u_out of an EIK_MODE_FP32 solve of the
 * same problem.  The solver then starts from |u_approx| * (1 + m), m = max(2^-12, n 2^-20)
 * with n the longest side, instead of +inf (NaN and +inf entries start at +inf) and sets the
 * exits to their exact values, as the second phase of EIK_MODE_MIXED does; the corrections
 * spread from the exits, and only cells whose boundary changes are swept.  Values only
 * decrease from their start, so the polish reaches the FP64 solution wherever the scaled start
 * is not below it (u_approx an upper bound, or at most about m relative below the solution).
 * The result is checked against eq. (2) at every node as in EIK_MODE_MIXED; a grid whose start
 * lay too low somewhere fails the check and is solved again from +inf (in a batch: on the
 * stream, counted in eik_stats.polish_redone; in a server: at the step that would have retired
 * it, counted by eik_server_polish_redone), so the result has the FP64 accuracy either way
 * (tol = 0; with tol > 0 the check is skipped).  u_approx is
 * read when the problem starts (in the batch call or at the server step that admits it) and may
 * be the same buffer as u_out.  Ignored for problems without exits (their solution is +inf).
 * Not allowed with EIK_MODE_MIXED (EIK_EINVAL).
 */
typedef struct eik_problem {
    int64_t dims[3];      /* as in eik_solve                                                  */
    double h;
    const void* F;        /* device speeds of the batch's / server's f_dtype                   */
    eik_sources sources;
    double* u_out;        /* device, nx*ny*nz doubles                                          */
    double tol;
    const double* u_approx;  /* device approximation to polish, or NULL (solve from scratch)   */
} eik_problem;

/*
 * eik_solve_batch -- solve n independent problems in one persistent launch.  Every problem is
 * validated as in eik_solve (any invalid one: EIK_EINVAL, nothing enqueued); all share f_dtype,
 * cell and options.  The grids' cells are swept together round by round, so many small grids
 * fill the device.  Each result equals the result of solving the problem alone (up to rounding
 * order).  eik_batch_status() returns the per-problem device status after the stream finishes.
 */
int eik_solve_batch(int n, const eik_problem* problems, int f_dtype, int cell, hipStream_t stream,
                    const eik_options* options);

/* Waits for `stream` and writes the device status of each problem of the last batch (or of
 * the single problem of the last eik_solve) into status[0 .. n-1].  Returns the number written
 * or a negative code. */
int eik_batch_status(hipStream_t stream, int n, int* status);

/*
 * Continuous-batching server.  A server owns a device pool (grids' arrays) and a cell-id
 * space; problems are admitted while they fit, swept together with the problems already on
 * the device, and retired (their u_out written) as soon as their own cells leave the worklist,
 * independently of the others.  Work happens in steps: a step starts the problems admitted
 * since the last step (staging, seeding into the next round's worklist), runs up to `rounds`
 * worklist rounds of every problem on the device in one persistent launch, then retires the
 * problems none of whose cells is queued.  A problem's result equals the result of solving it
 * alone (up to rounding order).  All calls of one server must come from one thread; its stream
 * must not be used for anything else while the server exists.
 *   eik_server_create   pool_bytes of device memory for grid arrays, at most max_cells cells
 *                       and max_problems problems on the device at once; cell, f_dtype and
 *                       options (delta, max_sweeps, workers, inner) fixed for its lifetime.
 *                       Returns EIK_EINVAL, EIK_ENOMEM or EIK_EHIP on failure (*out untouched).
 *   eik_server_submit   admits one problem if it fits now (pool space eik_problem_bytes(),
 *                       ncell cells, a free problem slot), else returns EIK_EBUSY (retry after
 *                       a step retired something); EIK_EINVAL if it is invalid or could never
 *                       fit.  On success *ticket (0, 1, 2, ... per server) identifies it.  F,
 *                       host-side sources and u_out must stay valid until the next
 *                       eik_server_step returned (F and the sources are read by it); u_out
 *                       until the problem is reported finished.
 *   eik_server_step     one step, blocking until it ran; *finished (may be NULL) receives the
 *                       number of problems retired in it.  Returns EIK_OK, EIK_EINVAL
 *                       (rounds < 1), a host error, or EIK_ECANCELLED if the device watchdog
 *                       stopped the launch: then every problem on the device is retired with
 *                       that status and the server starts again empty.
 *   eik_server_poll     up to max retired problems not yet polled, oldest first: tickets and
 *                       statuses (EIK_OK, EIK_EINVAL for an invalid speed, EIK_ECANCELLED).
 *   eik_server_load     problems on the device (admitted, not retired), cells and pool bytes
 *                       they occupy; any pointer may be NULL.
 *   eik_server_destroy  waits for the stream and frees everything.
 */
typedef struct eik_server eik_server;
int eik_server_create(eik_server** out, size_t pool_bytes, int64_t max_cells, int max_problems,
                      int cell, int f_dtype, hipStream_t stream, const eik_options* options);
int eik_server_submit(eik_server* srv, const eik_problem* problem, int64_t* ticket);
int eik_server_step(eik_server* srv, int64_t rounds, int* finished);
int eik_server_poll(eik_server* srv, int max, int64_t* tickets, int* status, int* n_out);
int eik_server_load(eik_server* srv, int* problems, int64_t* cells, size_t* pool_used);
int eik_server_destroy(eik_server* srv);
/* Problems of this server that started from u_approx, failed the eq. (2) check of their
 * polished result and were restarted from +inf (see eik_problem.u_approx); EIK_EINVAL if srv is
 * NULL. */
int64_t eik_server_polish_redone(const eik_server* srv);

/* Human-readable name of a status code (static storage). */
const char* eik_strerror(int code);

/* Frees every workspace and the library's per-device events and pinned words, after waiting
 * for every device that holds them (hipDeviceSynchronize; the streams they were used on may
 * already be destroyed).  Must not run concurrently with any other call of the library; a
 * later call allocates afresh. */
void eik_release(void);

/* Library version string (static storage). */
const char* eik_version(void);

#ifdef __cplusplus
}
#endif

#endif /* EIK_H_ */
