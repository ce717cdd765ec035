/*
 * swept.h -- C ABI of libswept, a two-dimensional swept-rule stencil solver
 * for one AMD Instinct MI355X (gfx950).
 *
 * Method: Walker & Niemeyer, "The Two-Dimensional Swept Rule Applied on
 * Heterogeneous Architectures" (arXiv:2105.10332).  The swept rule solves
 * as many (x, y, t) points of an explicit stencil time integration as the
 * data at hand allows before exchanging anything (Sec. 3.3), in four kinds
 * of space-time shapes: Up-Pyramid, X-/Y-Bridge, Octahedron, Down-Pyramid
 * (Figs. 1-2).  On one GPU every shape instance is one workgroup that keeps
 * its shape in LDS for up to b/(2n) levels between HBM round trips (Eq. 1),
 * and every phase is one kernel launch.  The Standard solver (Sec. 3.1)
 * takes one time step per launch.  Both use the same per-cell arithmetic,
 * so their results are bit-identical.
 *
 * Problems (App. A and B), on periodic square grids of nx = ny cells:
 *   SWEPT_HEAT   forward-Euler heat diffusion, 5-point stencil (n = 1);
 *   SWEPT_EULER  2D compressible Euler, finite volume with a pressure-ratio
 *                minmod limiter, Rusanov-form flux, explicit-midpoint RK2
 *                (n = 2 per RK stage; a stage is one swept level).
 *
 * Memory and ownership.  The caller owns every device buffer (allocated
 * through PyTorch or hipMalloc) and passes plain device pointers:
 *   - the state, nvar planes of nx*ny values (nvar = 1 heat: T;
 *     nvar = 4 Euler: rho, rho*u, rho*v, E), row-major with x fastest
 *     (index = var*nx*ny + j*nx + i), in the problem's dtype;
 *   - one workspace of swept_workspace_bytes() bytes: the second
 *     level-parity copy of the state (its first state_bytes bytes), reduction
 *     scratch and a per-level launch table written by swept_init.  It belongs
 *     to the library from swept_init to swept_destroy: the caller must not
 *     write it in between (its first state_bytes bytes may be overwritten
 *     freely between calls; they are scratch).
 * The library allocates no device memory; it owns only its host-side
 * context.  All work is enqueued on the caller's HIP stream (hipStream_t
 * passed as void*, NULL = default stream) and is asynchronous, except the
 * calls documented as synchronising.  The state is advanced in place.
 *
 * Errors.  Every call returns 0 (SWEPT_OK) or a negative SWEPT_E* code and
 * throws nothing.  Argument validation finishes before any HIP call.  A
 * thread-local message describing the last error is available from
 * swept_last_error().  Concurrent calls on one context are not allowed.
 */
#ifndef SWEPT_H
#define SWEPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SWEPT_OK = 0,
    SWEPT_EINVAL = -1,      /* null pointer or meaningless value            */
    SWEPT_ESHAPE = -2,      /* grid/tile geometry not supported (see init)  */
    SWEPT_EUNSTABLE = -3,   /* heat: 4r > 1, or dt <= 0                     */
    SWEPT_ENOTSUP = -4,     /* operation not available for this problem     */
    SWEPT_EWORKSPACE = -5,  /* workspace too small                          */
    SWEPT_EHIP = -6,        /* HIP runtime error (message has the details)  */
    SWEPT_ENONFINITE = -7   /* a conserved sum is NaN or infinite           */
};

enum { SWEPT_HEAT = 0, SWEPT_EULER = 1 };
enum { SWEPT_F64 = 0, SWEPT_F32 = 1 };

/* The problem as the paper states it (App. A/B; Sec. 4 parameters): grid,
 * physical parameters and time step.  The initial state is the device
 * buffer given to swept_init. */
typedef struct {
    int32_t kind;   /* SWEPT_HEAT or SWEPT_EULER                              */
    int32_t dtype;  /* SWEPT_F64 or SWEPT_F32: state and stencil arithmetic   */
    int32_t nx;     /* cells along x                                          */
    int32_t ny;     /* cells along y (must equal nx)                          */
    double lx;      /* domain length along x (heat: 1, Euler vortex: 10)      */
    double ly;      /* domain length along y                                  */
    double dt;      /* time step (> 0)                                        */
    double alpha;   /* heat diffusivity; r = alpha*dt/dx^2 with dx = lx/nx    */
    double gamma;   /* Euler ratio of specific heats (> 1)                    */
    int32_t scheme; /* Euler scheme variant bits (0 for heat), see below       */
    int32_t boundary; /* SWEPT_BC_*: periodic (0) or walls, see below         */
    double boundary_value; /* SWEPT_BC_DIRICHLET: the fixed ghost-cell value   */
} swept_problem;

/* Boundaries.  The paper's solver is periodic and notes that other
 * conditions fit the same decomposition (Sec. 3.3); heat also takes
 * SWEPT_BC_DIRICHLET (every neighbour outside the square reads the constant
 * boundary_value) and SWEPT_BC_NEUMANN (zero flux: an outside neighbour
 * reads the edge cell itself).  A cell's dependencies are then a subset of
 * its periodic ones, so the same shapes and phases apply unchanged.  The
 * heat adjoint takes the walls too (the walled step is affine: lambda runs
 * its homogeneous part, and dJ/dalpha pairs with the walled Laplacian
 * including the ghosts), and so does the batch.
 * Euler takes SWEPT_BC_NEUMANN (zero gradient: the two ghost cells beyond an
 * edge hold the edge cell) and SWEPT_BC_REFLECT (slip wall: ghost cell k
 * beyond the edge holds the k-th cell inside, mirrored, with its momentum
 * normal to the wall negated); a face's four-cell run reads ghosts from its
 * own side, so each wall face exists once per side.  SWEPT_BC_DIRICHLET is
 * SWEPT_ENOTSUP for Euler, SWEPT_BC_REFLECT is SWEPT_EINVAL for heat, and
 * the batch runs Euler periodic only (SWEPT_ENOTSUP). */
#define SWEPT_BC_PERIODIC 0
#define SWEPT_BC_DIRICHLET 1
#define SWEPT_BC_NEUMANN 2
#define SWEPT_BC_REFLECT 3

/* Euler scheme variants (App. B prints the limiter and the spectral radius
 * ambiguously).  0: pressure-ratio minmod face states, Q_L = Q_i +
 * min(1/r_i,1)/2 (Q_{i+1}-Q_i) and Q_R = Q_{i+1} + min(r_{i+1},1)/2
 * (Q_i-Q_{i+1}) with r_i = (p_{i+1}-p_i)/(p_i-p_{i-1}) (first order where
 * r_i is not in (0, inf)), and the Rusanov speed s = max(|u_L|+c_L,
 * |u_R|+c_R).  SWEPT_LIMITER_LITERAL takes the factors with the exponents as
 * printed, min(r_i,1)/2 and min(1/r_{i+1},1)/2.  SWEPT_SPEED_ROE takes s =
 * |u~|+c~ at the Roe-averaged state of Q_L and Q_R.  Bits combine.  The
 * single-problem calls and the batch accept every combination. */
#define SWEPT_LIMITER_LITERAL 1
#define SWEPT_SPEED_ROE 2

/* Launch tuning.  tile = block size b of Sec. 3.2 (0: library default);
 * wg = threads per workgroup (0: 256; a multiple of 64, at most 1024). */
typedef struct {
    int32_t tile;
    int32_t wg;
} swept_tuning;

/* What swept_init derived from the problem (for callers and tests). */
typedef struct {
    int32_t nvar;            /* 1 heat, 4 Euler                                 */
    int32_t n;               /* stencil radius per level: heat 1, Euler 2        */
    int32_t levels_per_step; /* heat 1, Euler 2 (RK stages)                      */
    int32_t tile;            /* b                                                */
    int32_t h;               /* b/(2n): levels per swept window (Eq. 1: k+1)     */
    int32_t wg;              /* threads per workgroup                            */
    double r;                /* heat: alpha*dt/dx^2 as used by the kernels       */
    double dx, dy;
    size_t state_bytes;      /* nvar*nx*ny*sizeof(scalar)                        */
    size_t lds_bytes;        /* LDS per swept workgroup                          */
} swept_info;

typedef struct swept_ctx swept_ctx;

/* Bytes of device workspace swept_init needs for this problem and tuning
 * (a second level-parity copy of the state plus reduction scratch).
 * Returns 0 and writes *bytes, or an error code. */
int swept_workspace_bytes(const swept_problem* prob, const swept_tuning* tune, size_t* bytes);

/* Validate the problem and create a context bound to the caller's state,
 * workspace and stream.  Geometry rules (Sec. 3.2, Eq. 1): nx == ny;
 * tile % (2n) == 0 and tile > 2n (b in (2n, b_max]); nx % tile == 0
 * (arrays divisible by the block size); nx >= 2*tile; the LDS window
 * (tile+2n)^2 * nvar * 2 levels must fit in 160 KiB.  Heat requires
 * 4r <= 1 (SWEPT_EUNSTABLE otherwise).  No device memory is allocated. */
int swept_init(swept_ctx** ctx, const swept_problem* prob, const swept_tuning* tune, void* d_state,
               void* d_work, size_t work_bytes, void* hip_stream);

/* Query derived parameters. */
int swept_query(const swept_ctx* ctx, swept_info* info);

/* Rebind the stream used by later calls. */
int swept_set_stream(swept_ctx* ctx, void* hip_stream);

/* Advance the state n_steps time steps with the swept rule (Sec. 3.3):
 * one Up-Pyramid, then alternating Bridge and Octahedron phases, closing
 * with the Down-Pyramid; one kernel launch per phase, 1 + 2*ceil(L/h)
 * launches for L = n_steps*levels_per_step levels.  Unlike the paper,
 * which stops at whole phases, every shape is cut at the final level, so
 * exactly n_steps steps are taken.  In place, asynchronous. */
int swept_advance(swept_ctx* ctx, int64_t n_steps);

/* Advance n_steps with the Standard solver (Sec. 3.1): one launch per time
 * step (Euler: both RK stages fused in one launch).  Bit-identical to
 * swept_advance.  In place, asynchronous. */
int standard_advance(swept_ctx* ctx, int64_t n_steps);

/* Per-plane sums of the current state in double, fixed reduction order
 * (reproducible): sum T (heat) or sum rho, rho*u, rho*v, E (Euler); out
 * must hold nvar doubles.  Synchronises the stream.  Returns
 * SWEPT_ENONFINITE if any sum is NaN or infinite (the values are still
 * written). */
int swept_conserved(swept_ctx* ctx, double* out);

/* Euler time step for a CFL number: dt = cfl / max over cells of
 * (|u|+c)/dx + (|v|+c)/dy, c = sqrt(gamma p / rho), evaluated in double.
 * d_state is an Euler state of prob's shape and dtype; d_work needs
 * swept_workspace_bytes(prob) bytes.  Synchronises the stream.  (The paper
 * states no time step; this fixes one.) */
int swept_cfl_dt(const swept_problem* prob, const void* d_state, double cfl, void* d_work, size_t work_bytes,
                 void* hip_stream, double* dt_out);

/* swept_cfl_dt without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as swept_cfl_dt, bit for bit
 * (the same kernels and reduction order); the 1024 partial maxima and the
 * result live in a static device array of 8200 bytes inside the library,
 * which holds one copy per GPU until the process ends and serves any grid
 * the library accepts (nx <= 32768; larger grids are SWEPT_ESHAPE).  The
 * array's device address is looked up on the first call on each device.
 * All calls on one GPU share that array, so calls that overlap on one GPU
 * (other threads, other streams) race; nothing in it needs clearing between
 * calls.  Synchronises the stream; calls no allocating routine. */
int swept_cfl_dt_noalloc(const swept_problem* prob, const void* d_state, double cfl, void* hip_stream,
                         double* dt_out);

/* ---- Adjoint of the swept heat advance (not in the paper) ------------------
 * For J(T^M) and g = dJ/dT^M, the discrete adjoint of n_steps heat steps
 * T^{m+1} = A T^m (A = I + r L) gives dJ/dT^0 = (A^T)^n g and
 * dJ/dalpha = (dt/dx^2) sum_{m<n} <lambda^{m+1}, L T^m>, lambda^m = (A^T)^{n-m} g.
 * The forward run keeps the flat state at the start of every swept cycle of
 * h = tile/2 steps (a "tape"); the reverse sweep recomputes each cycle
 * inside its reverse Octahedra, Bridges and Pyramids in LDS.  Heat only;
 * the tile must satisfy the LDS limit of the reverse shapes (tile <= 32). */

/* Bytes of tape for an n_steps adjoint: ceil(n_steps/h) checkpoints, four
 * state-sized buffers per full cycle (the forward's Up-Pyramid and Bridge
 * strips, kept so that the reverse sweep need not recompute them), two
 * double planes for lambda (carried in double for both state precisions),
 * (n_steps mod h) stored levels and the partial sums.  SWEPT_ENOTSUP for Euler, SWEPT_ESHAPE if the tile is too
 * large for the adjoint. */
int swept_tape_bytes(const swept_ctx* ctx, int64_t n_steps, size_t* bytes);

/* swept_advance(n_steps) that also records the checkpoints and each cycle's
 * forward strips in d_tape (device memory of swept_tape_bytes bytes,
 * caller-owned).  Same result as swept_advance.  Asynchronous. */
int swept_advance_checkpointed(swept_ctx* ctx, int64_t n_steps, void* d_tape, size_t tape_bytes);

/* Reverse sweep for the run recorded in d_tape (same ctx and n_steps):
 * d_gTM = dJ/dT^M (state layout and dtype, read-only), d_gT0 = dJ/dT^0
 * (written), *dJ_dalpha = dJ/dalpha (pairing sums accumulated in double in
 * a fixed order).  The tape's scratch is overwritten; its checkpoints are
 * kept.  Does not touch the context's state.  Synchronises the stream. */
int swept_adjoint(swept_ctx* ctx, int64_t n_steps, void* d_tape, size_t tape_bytes, const void* d_gTM,
                  void* d_gT0, double* dJ_dalpha);

int swept_destroy(swept_ctx* ctx);

/* ---- Batched ensemble in one persistent launch (not in the paper) ---------
 * count problems of uneven size and kind (heat and Euler mixed, one dtype)
 * advanced together by a single cooperative kernel: the grid holds what the
 * GPU keeps resident, and every workgroup walks global phases g = 0, 1, ...,
 * taking the shape instances of phase g of every problem (each problem has
 * 1 + 2 ceil(L/h) phases for its own tile) from a per-phase atomic counter,
 * with a grid barrier between global phases.  Every problem's result equals
 * its own swept_advance bit for bit.  The workspace holds each problem's
 * second level-parity buffer and level table, the launch arguments and the
 * two phase counters; calls that overlap on one workspace race.  Workgroups have 512 threads (FP32) or 256 (FP64);
 * tunes[q].tile (or 0 = default) picks each problem's tile, tunes may be
 * NULL.  swept_batch_advance is by default a cooperative launch: it has been
 * seen to return SWEPT_EHIP (HIP: operation cannot be performed in the
 * present state) in a process started while another live process on the same
 * GPU had made cooperative launches.  Such a process can switch the batch to
 * one ordinary launch per global phase (swept_batch_set_mode), where stream
 * order replaces the grid barrier; the results are the same bit for bit. */
typedef struct swept_batch swept_batch;

#define SWEPT_BATCH_COOPERATIVE 0 /* one persistent launch per advance (default) */
#define SWEPT_BATCH_PER_PHASE 1   /* one launch per global phase */

int swept_batch_workspace_bytes(const swept_problem* probs, const swept_tuning* tunes, int32_t count,
                                size_t* bytes);
/* d_states[q]: problem q's state (layout as above), advanced in place. */
int swept_batch_init(swept_batch** ctx, const swept_problem* probs, const swept_tuning* tunes,
                     void* const* d_states, int32_t count, void* d_work, size_t work_bytes, void* hip_stream);
/* n_steps time steps for every problem: one persistent launch, or one launch
 * per global phase in SWEPT_BATCH_PER_PHASE mode.  Asynchronous. */
int swept_batch_advance(swept_batch* ctx, int64_t n_steps);
/* SWEPT_BATCH_COOPERATIVE or SWEPT_BATCH_PER_PHASE for later advances;
 * SWEPT_EINVAL for any other value. */
int swept_batch_set_mode(swept_batch* ctx, int32_t mode);
int swept_batch_query(const swept_batch* ctx, int32_t q, swept_info* info);
/* Workgroups of the persistent launch (resident capacity for its LDS). */
int swept_batch_grid(const swept_batch* ctx, int32_t* grid);
int swept_batch_set_stream(swept_batch* ctx, void* hip_stream);
int swept_batch_destroy(swept_batch* ctx);

/* ---- Heterogeneous share: GPU and host cores together (Sec. 3.2, Eq. 2) ----
 * The paper divides the work of every phase between GPU and CPU by a GPU
 * share s = G/W of the blocks.  Here the tile rows jy < G = floor(s T + 1/2)
 * (T = nx/tile rows of tiles) run on the GPU, as one launch of the phase
 * kernel restricted to those rows, while host worker threads run the shape
 * instances of the other rows at the same time, each on the same memory
 * protocol and per-cell arithmetic (so the result equals swept_advance bit
 * for bit for every s).  After every phase the two sides exchange the rows
 * within tile of the two split lines (the GPU's copy of those rows is fetched
 * into pinned host memory, merged with the cells the host wrote, and sent
 * back); at the end the host's rows of the final level go to the GPU.  The
 * paper splits along x; this layout is x-fastest, so the split runs along y,
 * where each exchanged band is contiguous (the problems and the
 * decomposition are symmetric in x and y).  Periodic problems, heat and
 * Euler (every scheme variant); SWEPT_ENOTSUP for walls.
 *
 * swept_hetero_init binds to ctx (which must outlive it; no other call may
 * run on ctx concurrently) and holds pinned host memory of two state copies
 * plus the exchange band (no device memory).  cpu_threads = 0 takes
 * OMP_NUM_THREADS, else the host's hardware threads.  gpu_share in [0, 1]:
 * 1 is the all-GPU swept_advance, 0 runs every instance on the host.
 * swept_hetero_advance runs on ctx's stream and synchronises it. */
typedef struct swept_hetero swept_hetero;
int swept_hetero_init(swept_hetero** h, swept_ctx* ctx, double gpu_share, int32_t cpu_threads);
int swept_hetero_advance(swept_hetero* h, int64_t n_steps);
/* Tile rows on each side and the host worker threads. */
int swept_hetero_query(const swept_hetero* h, int32_t* gpu_rows, int32_t* cpu_rows, int32_t* threads);
int swept_hetero_destroy(swept_hetero* h);

/* Message for the last error on this thread ("" if none). */
const char* swept_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT_H */
