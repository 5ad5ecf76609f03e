/*
 * pi.h -- C ABI of the MI355X (gfx950) library for grid-binned short-range
 * pair interactions with a cutoff radius when each cell holds few particles.
 *
 * Method: Algis, Bramas, Darles, Aveneau, "Efficient GPU Implementation of
 * Particle Interactions with Cutoff Radius and Few Particles per Cell"
 * (arXiv 2406.16091).  The library implements the paper's GPU pipeline of
 * Sec. 2 ("Background"): per-particle cell index, per-cell counts, exclusive
 * prefix sum, scatter into a cell-sorted particle order, then the
 * 27-neighbour-cell interaction sweep over every pair i != j with
 * r_ij < r_c, with the sweep organisations of Sec. 4 (one thread per
 * particle, no shared memory) and Sec. 5 (X-pencil and full sub-box tiles
 * staged in LDS).
 *
 * Conventions for every entry point:
 *   - All particle arrays are structure-of-arrays, float32 or int32, in
 *     DEVICE memory, owned by the caller, and must stay valid until the work
 *     queued on `stream` has completed.
 *   - `stream` is a hipStream_t passed as an opaque pointer (NULL = the null
 *     stream).  Every call only queues work on it and returns; nothing
 *     blocks except pi_sync and pi_timing_read.
 *   - Errors the host can see (bad pointers, sizes, grid) are returned at
 *     once and nothing is queued.  Errors only the device can see (a particle
 *     outside the box) are latched in the pi_cells object and returned by the
 *     next pi_sync on it; the outputs of the failing call are unspecified but
 *     every kernel stays inside its buffers.
 *   - No call throws; every call is safe to make from any host thread as
 *     long as one pi_cells object is not used by two calls at once.
 */
#ifndef PI_H
#define PI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pi_status;
#define PI_OK          0
#define PI_EINVAL     (-1)  /* bad argument: pointer, size, grid, option */
#define PI_ENOMEM     (-2)  /* device allocation failed / budget exceeded */
#define PI_ERANGE     (-3)  /* a particle lies outside the grid's box */
#define PI_EDEVICE    (-4)  /* a HIP runtime call failed */
#define PI_EAGAIN     (-5)  /* try again later (queue or slots full) */
#define PI_ENOTFOUND  (-6)  /* unknown handle or ticket */
#define PI_ESTATE     (-7)  /* call out of order (e.g. interact before bin) */
#define PI_ESTEP      (-8)  /* a time step moved a particle further than half a
                               cell width on an axis (its displacement was cut) */

typedef void *pi_stream; /* hipStream_t */

/*
 * Regular grid over the box [origin, origin + dims * cell_w) (Sec. 2: the
 * domain is divided into a regular grid; Sec. 3: the cell width is at least
 * the cutoff, so every neighbour of a particle lies in its cell or one of
 * the 26 cells around it).  The grid is not periodic: the 27-cell stencil is
 * clipped at its faces.
 *   dims[a] >= 1, each <= 2^24, dims[0]*dims[1]*dims[2] < 2^31;
 *   0 < rc <= cell_w, both finite.
 * Cells are numbered X fastest: c = ix + dims[0] * (iy + dims[1] * iz)
 * (Fig. 1).  Particle axis index: t = (x - origin) / cell_w evaluated in
 * float32 with IEEE rounding, inside iff 0 <= t < dims, index floor(t).
 */
typedef struct pi_grid {
    float origin[3];
    int32_t dims[3];
    float cell_w;
    float rc;
} pi_grid;

typedef struct pi_ctx pi_ctx;     /* one per device */
typedef struct pi_cells pi_cells; /* a binned system, resident in HBM */

/* Create a context on HIP device `device` (made current for the calling
 * thread).  *out receives the handle.  PI_EDEVICE if the device is absent. */
pi_status pi_ctx_create(int32_t device, pi_ctx **out);
/* Destroy a context.  All pi_cells made from it must be destroyed first. */
pi_status pi_ctx_destroy(pi_ctx *ctx);

/* Create an empty cell structure.  Device buffers are allocated by pi_bin
 * and grown when a later pi_bin needs more; they are freed by
 * pi_cells_destroy.  The object is owned by the caller. */
pi_status pi_cells_create(pi_ctx *ctx, pi_cells **out);
/* Free a cell structure and its device buffers (synchronises its last
 * stream first). */
pi_status pi_cells_destroy(pi_cells *cells);

/*
 * Binning (Sec. 2; Fig. 1).  For the n particles (x, y, z, w) on the grid:
 *   1. cell of every particle (float32 decision, see pi_grid);
 *   2. counts[c] = particles in cell c, and max_per_cell (the paper's M_C,
 *      Sec. 5.1);
 *   3. offsets[c] = exclusive prefix sum of counts, n_cells + 1 entries,
 *      offsets[n_cells] = n (Fig. 1);
 *   4. the cell-sorted order: perm[k] = original index of the k-th particle,
 *      ascending original index inside each cell (a stable counting sort:
 *      the paper places particles inside a cell with atomics, in any order;
 *      this library fixes the order so that results are reproducible);
 *   5. sorted, cell-relative float32 coordinates
 *      xs[k] = fma(-ix, cell_w, x[perm[k]] - origin[0]) (one rounding; exact
 *      when positions lie on a power-of-two lattice), same for ys, zs, and
 *      ws[k] = w[perm[k]].
 * n may be 0.  n < 2^31.  An out-of-box particle sets PI_ERANGE on the object
 * (returned by pi_sync); the results of that call are then unspecified (the
 * particle is put in the last cell so that every kernel stays in bounds).
 * Buffers may be (re)allocated here; when they grow, the call first waits
 * for the object's previous stream.  A call that returns an error leaves the
 * object without a binned system: pi_interact, pi_tuner_choice and
 * pi_cells_get_view then return PI_ESTATE (and launch nothing) until a
 * pi_bin on it succeeds.
 */
pi_status pi_bin(pi_ctx *ctx, pi_cells *cells,
                 const float *x, const float *y, const float *z, const float *w,
                 int64_t n, const pi_grid *grid, pi_stream stream);

/* Device pointers into a binned system (valid until the next pi_bin or
 * pi_cells_destroy on it).  All arrays are int32/float32 in device memory.
 * The library keeps the sorted coordinates as one 16-byte record per slot;
 * the first view taken after a pi_bin writes the four arrays xs, ys, zs, ws
 * from those records, asynchronously on the stream of that pi_bin, so read
 * them once that stream's work has completed. */
typedef struct pi_cells_view {
    int64_t n;                /* particles binned by the last pi_bin */
    int64_t n_cells;
    pi_grid grid;
    const int32_t *counts;    /* [n_cells] */
    const int32_t *offsets;   /* [n_cells + 1] */
    const int32_t *perm;      /* [n] original index of sorted slot k */
    const int32_t *cell;      /* [n] cell of sorted slot k */
    const float *xs, *ys, *zs, *ws; /* [n] sorted, cell-relative */
    const int32_t *max_per_cell;    /* [1] */
} pi_cells_view;

pi_status pi_cells_get_view(pi_cells *cells, pi_cells_view *out);

/* Accumulation precision of the sweep. */
#define PI_PREC_COMPENSATED 0 /* FP32 terms with an error-free h^2 - r^2 for
                                 q > 1/2, FP32 Kahan-compensated sums */
#define PI_PREC_PLAIN       1 /* FP32 terms (1 - q from q), plain FP32 sums */
#define PI_PREC_FP64ACC     2 /* compensated FP32 terms, FP64 sums */

/* Organisation of the sweep. */
#define PI_SWEEP_AUTO   0 /* chosen by the library's tuner */
#define PI_SWEEP_NOLDS  1 /* one thread per target, sources read through the
                             caches (Sec. 4.1, Par-Part-NoLoop, Algorithm 1) */
#define PI_SWEEP_PENCIL 2 /* a workgroup owns an X-run of target cells; the 9
                             neighbour X-runs are staged in LDS (Sec. 5.2,
                             X-pencil, Algorithm 5) */
#define PI_SWEEP_SUBBOX 3 /* a workgroup owns a 3-D sub-box of target cells;
                             the sub-box and its ghost shell are staged in LDS
                             (Sec. 5.1, All-in-SM, Algorithm 4) */
#define PI_SWEEP_STREAM 4 /* as NOLDS (nothing staged), with accepted pairs
                             queued per thread in LDS and evaluated by the
                             whole wavefront at once (works at any occupancy) */
#define PI_SWEEP_PENCILREG 5 /* a workgroup owns a sub-box of target cells held
                             in registers, one target per thread; the halo's
                             X-pencils stream through LDS one Z-sheet at a time,
                             the targets' own particles copied from registers
                             (Sec. 5.3, X-pencil-reg); shapes 8x8x4 and 4x4x2 */
#define PI_SWEEP_CELL   6 /* cell-based with LDS staging (Sec. 4.4, Par-Cell-SM,
                             Algorithm 3), as a path for dense cells: a
                             one-wavefront workgroup owns a run of tile[0]
                             cells of an X-row and takes each cell holding at
                             least tile[1] particles, 64 targets at a time; the
                             cell's 9 neighbour rows stream through LDS and
                             every lane walks them in step.  tile[1] = 1: every
                             cell (the paper's organisation); larger: the
                             no-LDS walk takes the targets of the other cells.
                             Shapes (s, d, 1): (1, 1), (4, 1), (2, 16),
                             (2, 32), (2, 64) */

/* Order of the per-particle outputs. */
#define PI_ORDER_SORTED   0 /* output[k] belongs to sorted slot k */
#define PI_ORDER_ORIGINAL 1 /* output[i] belongs to input particle i */

typedef struct pi_interact_opts {
    int32_t precision; /* PI_PREC_* */
    int32_t sweep;     /* PI_SWEEP_* */
    int32_t order;     /* PI_ORDER_* */
    int32_t tile[3];   /* target cells per tile for PENCIL/SUBBOX/PENCILREG/
                          CELL; 0 = tuned */
} pi_interact_opts;

/* Global invariants, reduced in FP64 on the device. */
typedef struct pi_invariants {
    int64_t pairs;   /* sum_i count_i (ordered pairs; always even) */
    double net[3];   /* sum_i w_i G_i: zero up to rounding, since the pair
                        terms are antisymmetric (Newton's third law) */
    double scale;    /* sum_i w_i A_i, A_i = sum_j w_j |W'(r_ij)| */
    double rho_sum;  /* sum_i rho_i */
} pi_invariants;

/*
 * Interaction sweep (Sec. 2; Algorithms 1, 4, 5).  For every binned particle
 * i (target), over the 27 neighbour cells of its cell clipped at the grid
 * faces, and over every source j != i there with r_ij < rc (exact real
 * predicate for lattice inputs):
 *   count[i] = number of such j                                 (int32)
 *   rho[i]   = sum_j w_j W(r_ij)                                (float32)
 *   g*[i]    = sum_j w_j W'(r_ij) (x_i - x_j) / r_ij, 0 at r=0  (float32)
 * with the cubic B-spline of support h = rc, q = r/h, sigma = 8/(pi h^3):
 *   W = sigma (6q^3 - 6q^2 + 1) for q <= 1/2, 2 sigma (1-q)^3 for q < 1.
 * Terms are accumulated in a fixed canonical order (neighbour cells in
 * (dz, dy, dx) lexicographic order, sources in sorted order).
 * Exactness.  When the origin, the cell width and every coordinate are
 * multiples of one power of two 2^-p and every coordinate, measured from the
 * origin, stays below 2^(24-p) in magnitude, the cell-relative coordinates
 * and every pair difference are exact in float32: the neighbour counts then
 * equal the exact predicate r_ij < rc on the float32 inputs, and every sweep
 * organisation gives bit-identical outputs.  Otherwise each cell-relative
 * coordinate is rounded once, and the pair differences once or twice more
 * in the frame the organisation computes in: the results are then those of
 * the method on positions displaced by a small delta per pair, with, per
 * axis, delta <= 4 ulp(cell_w) for NOLDS and STREAM and
 * delta <= 2 ulp(cell_w) + ulp(E) for a tile whose halo box spans E cell
 * widths on that axis (T + 2 for a tile of T cells; a 254-cell pencil thus
 * loses about 8 bits along x).  A pair with |r_ij - rc| <= |delta| may be
 * counted differently from the exact predicate, and the floats may move by
 * what such a displacement changes (|delta| A_i for rho_i) beyond the
 * accuracy stated for exact inputs.
 * Outputs are caller-owned device arrays of n entries (n of the last
 * pi_bin); any of rho, gx, gy, gz, count may be NULL only if all the float
 * outputs are NULL together (count-only sweep).  `inv` (optional, device
 * memory) receives the invariants.  opts may be NULL (defaults: compensated,
 * auto, sorted).
 */
pi_status pi_interact(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts *opts,
                      float *rho, float *gx, float *gy, float *gz, int32_t *count,
                      pi_invariants *inv, pi_stream stream);

/*
 * pi_interact that allocates nothing, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Arguments, outputs and results are those
 * of pi_interact (bit-identical for the same organisation).  Differences:
 *   - the FP64 invariant partials (one 64-byte record per sweep workgroup,
 *     plus one per 1024 of them) go to a fixed device array of
 *     PI_NOALLOC_SCRATCH_RECORDS records (32 MiB), one copy per GPU the
 *     library runs on, held until the process ends;
 *   - a call whose invariants need more records returns PI_ENOMEM and queues
 *     nothing (a tile sweep takes one workgroup per tile, NOLDS and STREAM
 *     one per 256 particles); with PI_SWEEP_AUTO the no-LDS sweep is taken
 *     instead when the tiling would not fit; inv == NULL needs no records;
 *   - AUTO never runs timed trials (it takes the tuner's cached choice for
 *     the system's class, else the static rule), the call never waits, and
 *     it records no timing events (pi_timing_*).
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (no record needs to start at zero: each one read is first written
 * by the same call).  Calls whose work overlaps on one GPU -- on different
 * streams, or from different threads -- race on the array: queue them on
 * one stream.
 */
#define PI_NOALLOC_SCRATCH_RECORDS (1 << 19)
pi_status pi_interact_noalloc(pi_ctx *ctx, const pi_cells *cells, const pi_interact_opts *opts,
                              float *rho, float *gx, float *gy, float *gz, int32_t *count,
                              pi_invariants *inv, pi_stream stream);

/*
 * The pair kernels of the paper's timing experiments (Sec. 7.1: the
 * Lennard-Jones potential with a softening factor; Fig. 8: kernels of 5 and
 * 168 FLOP per interaction) on a binned system.  They are evaluated on every
 * candidate pair -- each source j != i whose cell is one of the 27 around
 * the target's cell, clipped at the grid faces -- since the interactions
 * those experiments count are the candidates (Table 1, first column); no
 * cutoff test is applied.  For every binned particle i:
 *   v[i]     = sum_j K(i, j)                                       (float32)
 *   count[i] = number of candidates j                               (int32)
 * with, for s^2 = r_ij^2 + eps^2 and u = sigma^2 / s^2:
 *   PI_PAIRFN_LJ:       K = 4 e0 (u^6 - u^3) = 4 e0 ((sigma/s)^12 - (sigma/s)^6)
 *   PI_PAIRFN_LOWFLOP:  K = (x_i - x_j) + (y_i - y_j) + (z_i - z_j)
 *   PI_PAIRFN_HIGHFLOP: the LJ value passed through 75 multiply-adds
 *                       y <- y a + b with run-time a = 1, b = 0 (150 more
 *                       FLOP, the same value)
 * Terms are accumulated in the canonical order of pi_interact, so every
 * organisation gives bit-identical outputs on lattice inputs (pi_interact's
 * exactness condition).  `inv` (optional, device memory): pairs = sum of
 * count, scale = sum_i sum_j |terms| (4 |e0| (u^6 + u^3), or |dx|+|dy|+|dz|),
 * rho_sum = sum_i v[i], net = 0.
 * Options: kernel; precision PI_PREC_COMPENSATED (Kahan sums) or
 * PI_PREC_PLAIN; sweep PI_SWEEP_NOLDS, PI_SWEEP_PENCIL (tiles of tile[0] x 1
 * x 1 cells, tile[0] <= 254), PI_SWEEP_SUBBOX (tile[0] x t x t with
 * t = tile[1] = tile[2] in {2, 4}, tile[0] <= 158 or 94; 0: 4 if its halo
 * fits, else 2) or PI_SWEEP_AUTO (with the timed tuner mode, every
 * organisation is timed once per size and occupancy class and the fastest
 * reused, as in pi_interact; in static mode: no LDS from 6 particles per
 * cell up, else the widest sub-box whose halo fits).  tile[0] = 0 sizes a
 * tile for about 384 targets, within the LDS capacity and the grid, and
 * shortens it while the launch has fewer than two workgroups per compute
 * unit; with AUTO a tile[0] beyond the chosen shape's limit is clamped to it
 * (PI_EINVAL for an explicit shape).  sigma, eps, e0: 0
 * selects rc/2, rc/4 and 1.  v is required (n > 0), count may be NULL.
 * PI_EINVAL for other options, PI_ESTATE before a successful pi_bin.
 */
#define PI_PAIRFN_LJ       1
#define PI_PAIRFN_LOWFLOP  2
#define PI_PAIRFN_HIGHFLOP 3

typedef struct pi_pairfn_opts {
    int32_t kernel;    /* PI_PAIRFN_* */
    int32_t precision; /* PI_PREC_COMPENSATED or PI_PREC_PLAIN */
    int32_t sweep;     /* PI_SWEEP_AUTO, _NOLDS, _PENCIL or _SUBBOX */
    int32_t order;     /* PI_ORDER_* */
    int32_t tile[3];
    float sigma, eps, e0;
} pi_pairfn_opts;

pi_status pi_interact_pairfn(pi_ctx *ctx, const pi_cells *cells, const pi_pairfn_opts *opts,
                             float *v, int32_t *count, pi_invariants *inv, pi_stream stream);

/*
 * Time stepping (Sec. 2: after the interactions the particles' positions are
 * updated).  The state of a binned system stays on the GPU in its
 * cell-sorted order.  With the B-spline as a soft pair potential
 *   E = (kappa / 2) sum_i sum_{j != i} w_i w_j W(r_ij)
 * and w_i taken as the mass, the force on i is -kappa w_i G_i (G as
 * pi_interact computes it), and one pi_step is:
 *   1. the sweep of pi_interact (opts->precision, opts->sweep) at the
 *      current positions;
 *   2. symplectic Euler, per axis: v <- v - dt kappa G; x <- x + dt v, with
 *      the displacement cut to half a cell width (PI_ESTEP is then latched
 *      and returned by the next pi_sync: reduce dt), reflection at the box
 *      faces (the velocity component changes sign), and, when lattice > 0,
 *      the coordinate measured from the origin rounded down to a multiple of
 *      it (a power of two keeps lattice inputs on the lattice, so counts stay
 *      exact);
 *   3. the re-binning of the new positions, incrementally: the result is
 *      what pi_bin gives on them (counts, offsets, M_C, the stable order,
 *      cell-relative records), computed from the previous binning since a
 *      particle moves to one of the 26 neighbouring cells at most.
 * pi_state_set_velocity gives the velocities (caller's device arrays in the
 * input order of the last pi_bin) and must follow every pi_bin before a
 * pi_step (else PI_ESTATE).  pi_state_get writes positions and velocities in
 * that input order; positions are origin + cell corner + cell-relative part,
 * which are the stepped values whenever they lie on a common power-of-two
 * lattice with the origin and cell width.  With rho .. gz (all or none) it
 * also writes the sweep outputs of the last step (at the positions before
 * it; PI_ESTATE before the first step).  The first call allocates 88 bytes
 * per particle and 12 per cell of stepping buffers on the object.
 */
typedef struct pi_step_opts {
    float dt;         /* time step (>= 0) */
    float kappa;      /* force scale */
    float lattice;    /* > 0: positions rounded down to multiples of it; 0: none */
    int32_t precision;/* PI_PREC_* of the sweep */
    int32_t sweep;    /* PI_SWEEP_* of the sweep */
    int32_t tile[3];  /* tile shape of the sweep, as in pi_interact_opts */
} pi_step_opts;

pi_status pi_state_set_velocity(pi_ctx *ctx, pi_cells *cells, const float *vx, const float *vy,
                                const float *vz, pi_stream stream);
/* inv (optional, device memory): the invariants of the step's sweep. */
pi_status pi_step(pi_ctx *ctx, pi_cells *cells, const pi_step_opts *opts, pi_invariants *inv,
                  pi_stream stream);
pi_status pi_state_get(pi_ctx *ctx, pi_cells *cells, float *x, float *y, float *z,
                       float *vx, float *vy, float *vz, float *rho, float *gx, float *gy, float *gz,
                       pi_stream stream);

/* Wait for `stream` and return the first device-detected error latched on
 * `cells` (PI_ERANGE for out-of-box particles), then clear it.  cells may be
 * NULL (only waits). */
pi_status pi_sync(pi_ctx *ctx, pi_cells *cells, pi_stream stream);

/*
 * Tuner.  The paper concludes that which organisation is fastest is hard to
 * predict and needs a profiling step per configuration (Sec. 8).  With
 * PI_SWEEP_AUTO the library times every compiled organisation (no-LDS, the
 * stream, each pencil / sub-box / pencil-reg tile, the cell-SM dense-cell
 * passes from two particles per cell on and the cell-SM over every cell from
 * 16 on) once per size and occupancy class -- buckets
 * of log2(n) and of the mean particles per cell -- on the caller's stream,
 * and reuses the fastest for that class afterwards (per context).  Tuning
 * runs each candidate once untimed, then keeps the fastest of up to three
 * timed runs (a candidate already 1.5x slower than the best so far stops
 * after one), and waits for the stream.  In
 * PI_TUNE_STATIC mode (or with PI_AUTOTUNE=off in the environment) AUTO uses
 * a fixed rule on the mean occupancy instead: the 6x6x6 sub-box while its
 * staged halo is expected to fit in LDS (mean + 6 standard deviations of a
 * Poisson count, up to about 1.2 particles per cell), then 4x4x4 (up to
 * about 6), then no LDS.  The same fit test picks the tile of PI_SWEEP_PENCIL
 * and PI_SWEEP_SUBBOX when tile[] is zero; PI_SWEEP_CELL with tile[] zero
 * takes every cell (one per workgroup) from 32 particles per cell on, else
 * the cells holding 32 or more with the no-LDS walk for the rest.
 */
#define PI_TUNE_STATIC 0
#define PI_TUNE_TIMED  1
pi_status pi_tuner_mode(pi_ctx *ctx, int32_t mode);
/* The organisation AUTO uses for this binned system and precision (tuning
 * it now if the class is new and the mode is timed).  out->sweep is
 * PI_SWEEP_NOLDS, _STREAM, _PENCIL or _SUBBOX and out->tile its shape. */
pi_status pi_tuner_choice(pi_ctx *ctx, const pi_cells *cells, int32_t precision, pi_interact_opts *out,
                          pi_stream stream);

/*
 * Batches: many independent systems binned and swept together (the
 * pipeline of Sec. 2 applied to a set of systems).  The systems' particles
 * are concatenated in the caller's arrays, system s occupying
 * [offset, offset + n) with offset = sum of the previous systems' n; each
 * system has its own grid and cutoff.  One radix sort over global cell ids
 * and one work-list sweep cover all systems; the launch sequence is
 * captured into a hipGraph the first time a layout (systems, pointers,
 * options, stream) is seen and replayed by later calls with the same
 * layout.  On the null stream nothing is captured.
 */
typedef struct pi_batch pi_batch;

typedef struct pi_system_desc {
    int64_t offset;   /* first particle of the system in the concatenated arrays */
    int64_t n;        /* particles of the system (>= 0) */
    pi_grid grid;     /* the system's grid and cutoff */
} pi_system_desc;

pi_status pi_batch_create(pi_ctx *ctx, pi_batch **out);
pi_status pi_batch_destroy(pi_batch *batch);
/*
 * Bin and sweep nsys >= 1 systems (descriptions in host memory).  x, y, z, w
 * and the outputs are concatenated device arrays of sum(n) entries; with
 * PI_ORDER_ORIGINAL output i belongs to input particle i, with
 * PI_ORDER_SORTED to sorted slot i (systems stay in order either way).  inv,
 * if not NULL, receives nsys records (device memory).  Same precision and
 * organisation options as pi_interact; AUTO picks one tile shape for the
 * batch from its mean occupancy.  Sum(n) and the total cell count must stay
 * below 2^31.  Errors as pi_bin / pi_interact; device errors surface through
 * pi_batch_sync.
 */
pi_status pi_batch_run(pi_ctx *ctx, pi_batch *batch, int32_t nsys, const pi_system_desc *sys,
                       const float *x, const float *y, const float *z, const float *w,
                       const pi_interact_opts *opts, float *rho, float *gx, float *gy, float *gz,
                       int32_t *count, pi_invariants *inv, pi_stream stream);
/* View of the concatenated binned arrays of the last run (cell ids in
 * `cell` are local to their system; counts/offsets are indexed by global
 * cell = cell_base[s] + local cell).  cell_base (host, max_sys entries) may
 * be NULL. */
pi_status pi_batch_get_view(pi_batch *batch, pi_cells_view *out, int64_t *cell_base, int32_t max_sys);
/* pi_sync for a batch. */
pi_status pi_batch_sync(pi_ctx *ctx, pi_batch *batch, pi_stream stream);

/*
 * Serving.  Particle systems submitted over time, each swept n_sweeps
 * times; before every sweep after the first, each particle is displaced by
 * a Gaussian step (counter-based RNG, reflected at the box faces, rounded to
 * a lattice) and the system is re-binned in place: its cell list stays
 * resident on the GPU for the whole request.  A scheduler thread admits
 * queued requests first-in first-out while fewer than max_slots are in
 * flight and their device-memory footprints fit the budget, and runs the
 * requests it admits at one time as one batch on a free lane (one of
 * n_streams streams): one upload per request, then per sweep one batched
 * displacement and one batched re-binning and sweep of all of them
 * (pi_batch_run), then one download per request.  Lanes run side by side,
 * so requests that arrive while batches are on the GPU are admitted onto
 * another lane as soon as one is free.  A batch holds requests of the same
 * n_sweeps, precision and sweep, each under 2^18 particles; a larger
 * request, or one admitted alone, runs the plain single-system path (pi_bin,
 * pi_interact).  A request's results are the same whatever it shares its
 * batch with.  Results stay in pinned host memory owned by
 * the server until pi_release.  All calls are thread-safe.
 */
typedef struct pi_server pi_server;

typedef struct pi_server_opts {
    int64_t hbm_budget;      /* device bytes the admitted requests may hold together */
    int32_t max_slots;       /* requests in flight at once, over all lanes (1..4096) */
    int32_t n_streams;       /* lanes: streams that each run one batch at a time (1..16) */
    int32_t queue_capacity;  /* requests waiting for admission; beyond -> PI_EAGAIN */
    int32_t pad;
} pi_server_opts;

typedef struct pi_request {
    const float *x, *y, *z, *w; /* host arrays of n entries, copied by pi_submit */
    int64_t n;
    pi_grid grid;
    int32_t n_sweeps;           /* >= 1 */
    int32_t precision;          /* PI_PREC_* */
    int32_t sweep;              /* PI_SWEEP_* */
    float jitter_sigma;         /* per-axis standard deviation of a displacement (0: none) */
    float lattice;              /* displaced positions rounded down to multiples of this (0: no rounding) */
    int32_t pad;
    uint64_t seed;              /* RNG seed of the displacements */
} pi_request;

typedef struct pi_result {
    int32_t done;               /* 1 once the request has finished */
    int32_t status;             /* PI_OK or the error that ended it */
    int64_t n;
    int32_t sweeps;
    int32_t pad;
    int64_t pairs_total;        /* ordered pairs summed over all sweeps */
    double t_submit, t_start, t_done; /* seconds (CLOCK_MONOTONIC): submitted, admitted, finished */
    const float *rho, *gx, *gy, *gz;  /* last sweep, input order (pinned host memory) */
    const int32_t *count;
    const float *x, *y, *z;     /* positions of the last sweep */
    const pi_invariants *invariants; /* [sweeps] */
} pi_result;

typedef struct pi_server_stats_t {
    int32_t queued;
    int32_t running;
    int64_t hbm_in_use;
} pi_server_stats_t;

/* opts may be NULL (64 GiB budget, 8 slots, 4 streams, queue of 1024). */
pi_status pi_server_create(pi_ctx *ctx, const pi_server_opts *opts, pi_server **out);
/* Admitted requests finish first; queued ones end with PI_EAGAIN. */
pi_status pi_server_destroy(pi_server *server);
/* PI_EAGAIN if the queue is full, PI_ENOMEM if the request alone exceeds the
 * budget, PI_ERANGE if a particle lies outside its box (by the binning's own
 * float32 decision), PI_EINVAL for a bad request.  *ticket identifies the
 * request. */
pi_status pi_submit(pi_server *server, const pi_request *req, uint64_t *ticket);
/* Non-blocking: out->done tells whether the request has finished. */
pi_status pi_poll(pi_server *server, uint64_t ticket, pi_result *out);
/* Blocks until the request has finished. */
pi_status pi_wait(pi_server *server, uint64_t ticket, pi_result *out);
/* Frees a finished request's results (PI_EAGAIN while it is running). */
pi_status pi_release(pi_server *server, uint64_t ticket);
pi_status pi_server_stats(pi_server *server, pi_server_stats_t *out);

/*
 * Kernel timing (instrumentation for measurement).  While enabled on a
 * context, every kernel the library launches is bracketed by two hipEvents
 * recorded on the stream it is launched on; pi_timing_read waits for the
 * recorded events and returns, per kernel name, the number of launches and
 * the summed device time since the last reset.  Off by default (no events
 * are recorded).  Not for use inside graph capture.
 */
typedef struct pi_kernel_time {
    char name[48];
    int64_t launches;
    double total_ms;
} pi_kernel_time;

pi_status pi_timing_enable(pi_ctx *ctx, int32_t on);
/* Restrict timing to the launches whose kernel name (as pi_timing_read
 * reports it) equals `name`; NULL or "" times every launch again.  Each
 * timed launch adds two event records to its stream, which costs device time
 * between kernels, so a measurement of one kernel inside a timed loop times
 * that kernel alone.  Returns PI_EINVAL for a name longer than 47 bytes. */
pi_status pi_timing_only(pi_ctx *ctx, const char *name);
/* Fill out[0 .. *n_out) (at most `max` records, in first-launch order). */
pi_status pi_timing_read(pi_ctx *ctx, pi_kernel_time *out, int32_t max, int32_t *n_out);
pi_status pi_timing_reset(pi_ctx *ctx);

/* Human-readable name of a status code (static string). */
const char *pi_status_str(pi_status status);

/* Library version string (static). */
const char *pi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PI_H */
