/*
 * rbf.h -- C ABI of librbf, a GPU library for implicit surface
 * reconstruction with Gaussian radial basis functions on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: Cuomo, Galletti, Giunta, Starace, "Surface Reconstruction from
 * Scattered Point via RBF Interpolation on GPU" (arXiv 1305.5179):
 *   1. extend the cloud by off-surface points along the normals (Sec. II.A.1);
 *   2. solve the Gaussian interpolation system A c = b with GMRES
 *      (Sec. II.B eq. RBFsys, Sec. III.A eqs. matrixEntries);
 *   3. evaluate the interpolant on a grid (Sec. II.B eq. matxvet, Sec. II.A.3).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers (hipMalloc'ed or torch tensors on
 *     the GPU) owned by the caller; they must stay valid until the work
 *     enqueued on `stream` has finished.  Host pointers are rejected with
 *     RBF_EINVAL.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; calls that must read a result back (rbf_setup,
 *     rbf_solve, rbf_count_pairs) synchronise with it before returning.
 *   - Centre order is the paper's: centre i is point i, centre N+i the
 *     outside point x_i + eps*n_i, centre 2N+i the inside point
 *     x_i - eps*n_i (Sec. II.A.1).  Vectors of length 3N (x, y, b, c) are in
 *     that order; any internal reordering is invisible to the caller.
 *   - The kernel is phi(r) = exp(-r^2 / (2 sigma^2)); A_ij = phi(|x_i - x_j|)
 *     when |x_i - x_j|^2 <= cutoff^2 (decided in float64, with
 *     r^2 = (dx*dx + dy*dy) + dz*dz), else 0.  cutoff = +INFINITY keeps every
 *     pair.  The paper's 1/(sqrt(2 pi) sigma) factor is left out: a constant
 *     factor scales the weights and leaves the interpolant unchanged.
 *   - Every function returns an rbf_status; nothing aborts.  After an error
 *     rbf_last_error() describes it.  One context must not be used from two
 *     host threads at once.
 */
#ifndef RBF_H
#define RBF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rbf_ctx rbf_ctx;

typedef enum {
    RBF_OK = 0,
    RBF_EINVAL = -1,      /* bad argument (NaN/Inf input, sigma/eps/cutoff <= 0, zero normal, n <= 0, host pointer, ...) */
    RBF_ENOMEM = -2,      /* device allocation failed */
    RBF_EDEVICE = -3,     /* no usable gfx950 device, or a HIP runtime error */
    RBF_ENOCONV = -4,     /* rbf_solve stopped at its iteration limit; c and info hold the best iterate */
    RBF_EBREAKDOWN = -5   /* a non-finite value appeared in the solve */
} rbf_status;

typedef enum { RBF_FP32 = 0, RBF_FP64 = 1 } rbf_prec;

typedef enum {
    RBF_SOLVE_PLAIN_FP64 = 0,  /* restarted GMRES, float64 operator throughout */
    RBF_SOLVE_IR_FP32 = 1      /* float64 outer refinement, GMRES cycles on the float32 operator */
} rbf_mode;

typedef enum {
    RBF_PRECOND_NONE = 0,
    RBF_PRECOND_SCHWARZ = 1    /* the context's Schwarz preconditioner (rbf_schwarz_setup), applied on the right */
} rbf_precond;

typedef struct {
    double tol;        /* stop when |b - A c|_2 / |b|_2 <= tol, float64 operator (default 1e-8) */
    int restart;       /* GMRES restart length m, 1..64 (default 30) */
    int max_outer;     /* maximum restarts / refinement steps (default 1000) */
    int max_iters;     /* maximum operator applications inside GMRES cycles (default 30000) */
    int mode;          /* rbf_mode (default RBF_SOLVE_IR_FP32) */
    int precond;       /* rbf_precond (default RBF_PRECOND_NONE) */
    int basis;         /* rbf_prec in which the refinement's inner GMRES stores its Krylov basis and
                          the operator's output: RBF_FP32 (default) or RBF_FP64.  Its dot products,
                          norms, updates and least squares are float64 either way.  The plain method
                          always stores float64 and ignores this field. */
    int graph;         /* 1 (default): the Arnoldi steps of a full GMRES cycle (operator,
                          preconditioner and orthogonalisation launches) are captured once into a
                          HIP graph on the context and replayed for every full cycle; 0: launched
                          one by one.  The same kernels in the same order: identical results.  Not
                          used while launch profiling (rbf_profile_begin) is on. */
} rbf_solve_opts;

typedef struct {
    int max_block;     /* largest subdomain, core + overlap centres, 3..1024 (default 192) */
    int overlap_pct;   /* overlap size in percent of the core, 0..100 (default 10) */
    int restricted;    /* 1: restricted additive Schwarz (core rows of each local solution);
                          0: additive (every row, summed) (default 0) */
    int min_block;     /* 0: every octree leaf is a core (default); > 0: consecutive leaves are
                          joined while the block (core + overlap) is below min_block and the
                          cap allows, 0..max_block */
    double shift;      /* added to the unit diagonal of every local block, >= 0 (default 0.3) */
    int tune;          /* 1: time the apply kernel's launch shapes at setup and keep the
                          fastest (default); 0: no timing: workgroups of the smallest of
                          128, 256, 512 threads whose task covers the largest block's rows
                          (two rows per thread with half), one workgroup per task */
    int half;          /* 1: the local inverses stored in float16 (half the apply's bytes; each
                          entry then carries a relative rounding of at most 2^-11, and the
                          apply's products and sums are float32; this changes the
                          preconditioner, not the solution: the solver's residual stays the
                          float64 one); 0: float32 entries, float64 sums (default) */
} rbf_schwarz_opts;

typedef struct {
    int64_t n_sub;         /* subdomains */
    int64_t n_members;     /* sum of the subdomain sizes (core + overlap) */
    int64_t max_members;   /* the largest subdomain */
    int64_t inverse_bytes; /* device memory of the local inverses */
    int retries;           /* local blocks redone with a larger shift */
    double max_shift;      /* the largest shift a block ended with */
    int64_t min_members;   /* the smallest subdomain */
    int apply_threads;     /* launch shape of the apply: threads per workgroup (rows per task:
                              one per thread, two with half) */
    int apply_blocks;      /* and workgroups of its persistent launch */
    double factor_ms;      /* device time of the local inverses (all blocks, one launch) */
} rbf_schwarz_info;

typedef struct {
    int iters;               /* operator applications inside GMRES cycles */
    int outer;               /* restarts (plain) or refinement steps (IR) performed */
    double rel_resid;        /* final |b - A c|_2 / |b|_2 with the float64 operator */
    int status;              /* same value rbf_solve returned */
    int n_history;
    const double* history;   /* host array: true relative residual at the start of each outer
                                step and at the end; owned by the context, valid until the next
                                call on it */
    const double* history_ms;  /* host array, same length: milliseconds since the call began
                                  when each history entry was known */
} rbf_solve_info;

typedef struct {
    double origin[3];   /* node (i,j,k) = origin + (i*h[0], j*h[1], k*h[2]) */
    double h[3];
    int64_t dims[3];    /* nodes per axis; output index i + dims[0]*(j + dims[1]*k) (x fastest) */
} rbf_grid;

typedef struct {
    int64_t n_points;        /* N */
    int64_t n_centres;       /* 3N */
    int64_t n_groups;        /* target groups of 16 centres */
    int64_t list_entries;    /* source-list entries over all groups (padded) */
    int64_t useful_pairs;    /* nonzeros of A: pairs with r^2 <= cutoff^2 (3N^2 without cutoff) */
    int64_t examined_pairs;  /* pairs one matvec evaluates (list entries x 16) */
    int64_t n_cells;         /* occupied cells of the neighbour lattice */
    double cell_size;        /* side of a lattice cell */
    double sigma, cutoff, eps;
    int64_t inner_entries;   /* list entries in the groups' leading inner chunks (every pair inside
                                the cutoff: the pair kernels apply no test there) */
} rbf_stats;

/* Fill `opts` with the defaults listed in rbf_solve_opts. */
int rbf_default_solve_opts(rbf_solve_opts* opts);

/* Step 1 of the paper's Alg. 1 plus the neighbour structure for truncation
 * (Sec. II.A.1; Sec. III.A, the finite-bandwidth remark).
 *   points, normals: device, n x 3 float64, row-major (x, y, z per row).
 *     Normals need not be unit length; a normal shorter than 1e-12 is
 *     RBF_EINVAL.  Coordinates must be finite.
 *   off_surface_eps > 0: the offset delta along the unit normals.
 *   sigma > 0, cutoff > 0 (or +INFINITY).
 * Copies everything it needs; keeps no caller pointer.  *out receives a new
 * context (NULL on failure). */
int rbf_setup(const double* points, const double* normals, int64_t n,
              double off_surface_eps, double sigma, double cutoff,
              void* stream, rbf_ctx** out);

/* The extended centre set and default data values (Sec. II.A.1-2).
 * centres: device, 3n x 3 float64 (paper order); values: device, 3n float64,
 * 0 / +eps / -eps.  Either pointer may be NULL. */
int rbf_centres(rbf_ctx* ctx, double* centres, double* values, void* stream);

/* y = A x (Sec. II.B eq. RBFsys), matrix-free.  x, y: device, 3n float64.
 * RBF_FP32 evaluates the pair sums in float32 (cutoff still decided as in
 * float64); RBF_FP64 entirely in float64.  x and y may not overlap.
 * (Inside rbf_solve's refinement mode the inner GMRES keeps its Krylov
 * basis in float32; its products and updates are formed in float64.) */
int rbf_matvec(rbf_ctx* ctx, const double* x, double* y, int prec, void* stream);

/* Weights c with A c = b (Sec. III.A: GMRES on the interpolation system).
 *   b: device 3n float64, or NULL for the default values (0, +eps, -eps).
 *   x0: device 3n initial guess, or NULL for zero.  c: device 3n output
 *   (may alias x0).  opts: NULL for defaults.  info: may be NULL.
 *   opts->precond = RBF_PRECOND_SCHWARZ preconditions every GMRES cycle on the
 *   right with the context's Schwarz preconditioner (RBF_EINVAL without one).
 * Blocks the host until done.  Returns RBF_OK when the float64 relative
 * residual reached opts->tol, RBF_ENOCONV when a limit stopped it (c and
 * info still hold the last iterate), RBF_EBREAKDOWN on non-finite values. */
int rbf_solve(rbf_ctx* ctx, const double* b, const double* x0, double* c,
              const rbf_solve_opts* opts, rbf_solve_info* info, void* stream);

/* f on a regular grid (Sec. II.A.3; Sec. II.B eq. matxvet).
 *   c: device 3n float64 weights.  out: device, dims[0]*dims[1]*dims[2]
 *   values, float32 when prec == RBF_FP32, float64 when RBF_FP64.
 * Nodes farther than cutoff from every centre get exactly 0.  With a
 * cutoff, float32 grids whose spacing is fine against sigma are summed
 * brick by brick from the neighbour cells without source lists (same
 * truncation, decided in float64); other grids go through lists. */
int rbf_eval_grid(rbf_ctx* ctx, const double* c, const rbf_grid* grid, void* out,
                  int prec, void* stream);

/* f at m arbitrary points (Sec. II.B eq. matxvet: the interpolant at
 * evaluation points is the rectangular matrix phi(|xi_k - x_j|), truncated as
 * the operator, times the weights).
 *   c: device 3n float64 weights (paper order).
 *   pts: device m x 3 float64, row-major; out: device m float64.
 *   prec: RBF_FP32 sums in float32 (truncation decided in float64),
 *   RBF_FP64 entirely in float64.  m = 0 does nothing.  Points farther than
 *   cutoff from every centre get exactly 0. */
int rbf_eval_points(rbf_ctx* ctx, const double* c, const double* pts, int64_t m,
                    double* out, int prec, void* stream);

/* Density measures of the point cloud the context was built from (Sec. IV,
 * eqs. sepDist, fillDist, hmax) and the choices of sigma the paper derives
 * from them (eqs. h1, h2):
 *   q          = 1/2 min_{i != j} |x_i - x_j| over the n cloud points;
 *   h_max      = max_j min_{i != j} |x_i - x_j|;
 *   h_fill     = max over the `samples` (device, n_samples x 3 float64, points
 *                of the domain chosen by the caller) of min_j |s - x_j|, the
 *                sampled fill distance; NaN when samples is NULL;
 *   h          = h_fill, or sqrt(2) h_max (eq. hmax) without samples;
 *   sigma_sep  = 2 q (eq. h1);
 *   sigma_fill = sqrt(2) h (eq. h2).
 * Exact float64 minima (all pairs); q, h_max are NaN for n < 2.
 * out: HOST pointer.  Synchronises with `stream`. */
typedef struct {
    double q, h_max, h_fill, h, sigma_sep, sigma_fill;
} rbf_density_info;

int rbf_density(rbf_ctx* ctx, const double* samples, int64_t n_samples, rbf_density_info* out, void* stream);

/* The Arnoldi process of rbf_solve's GMRES (Sec. III.A) for m steps from v0,
 * with no restart and no stopping test, so that its invariants can be
 * inspected: V_{k+1}^T V_{k+1} = I and A V_k = V_{k+1} H_k.
 *   v0: device 3n float64 (paper order), not zero.
 *   op_prec: the operator's precision (RBF_FP32 / RBF_FP64); basis: the
 *   storage of the basis and of the operator's output (RBF_FP32 / RBF_FP64),
 *   as rbf_solve_opts.basis.  The orthogonalisation is rbf_solve's: classical
 *   Gram-Schmidt applied twice, products in float64.
 *   V: device (m+1) x 3n float64, row k = basis vector k in paper order.
 *   H: HOST (m+1) x m float64, row-major, the Hessenberg matrix before any
 *   Givens rotation (zero below the subdiagonal).
 *   *steps: columns computed.  It is m unless |w| became exactly 0 at step
 *   *steps - 1 (an invariant Krylov space); then rows 0 .. *steps - 1 of V
 *   are the basis and the rest of V and H is 0.
 * 1 <= m <= 64.  RBF_EBREAKDOWN on a non-finite value.  Synchronises. */
int rbf_arnoldi(rbf_ctx* ctx, const double* v0, int m, int op_prec, int basis, double* V, double* H, int* steps,
                void* stream);

/* Overlapping Schwarz preconditioner for rbf_solve (Sec. III.A: overlapping
 * subdomains whose local systems are solved independently; their solutions
 * added up (additive Schwarz) or kept on the non-overlapping parts only
 * (restricted additive Schwarz) precondition GMRES).
 *   Subdomains: the cores are the leaves of an octree over the surface
 *   points (root cube at their componentwise minimum, side = their largest
 *   extent, 10 levels), a cell being split while it holds more than p points,
 *   p the largest count with 3p + ceil(3p overlap_pct / 100) <= max_block; a
 *   core holds the three centres of each of its points.  The overlap adds
 *   the ceil(overlap_pct |core| / 100) centres outside the core nearest to it
 *   (squared float64 distance to the nearest core centre, ties by index).
 *   With min_block > 0 the leaves, in the octree's depth-first order
 *   (children by the digit bx + 2 by + 4 bz of their cell), are joined into
 *   runs: the core being built is closed before the next leaf once its block
 *   reaches min_block or when the leaf would take it above p points.
 *   Local matrices: the Gaussian of the subdomain without truncation plus
 *   shift * I, inverted in float64 (a block found indefinite is redone with
 *   ten times the shift, at most 8 times), kept in float32.  All blocks are
 *   inverted by one persistent launch, largest first.
 *   Apply: one persistent launch takes strips of rows of the blocks
 *   (largest first, cyclic over its workgroups); the additive form adds a
 *   second launch that sums each centre's rows in subdomain order.
 * opts: NULL for defaults.  Replaces the context's previous preconditioner.
 * Synchronises with `stream`.  RBF_EBREAKDOWN when a block stays indefinite. */
int rbf_default_schwarz_opts(rbf_schwarz_opts* opts);
int rbf_schwarz_setup(rbf_ctx* ctx, const rbf_schwarz_opts* opts, void* stream);

/* z = M^{-1} r with the context's Schwarz preconditioner.  r, z: device, 3n
 * float64, paper order, not overlapping. */
int rbf_schwarz_apply(rbf_ctx* ctx, const double* r, double* z, void* stream);

/* Sizes of the context's Schwarz preconditioner (host call). */
int rbf_schwarz_get_info(const rbf_ctx* ctx, rbf_schwarz_info* info);

/* The subdomains, into HOST arrays: offsets (n_sub + 1), n_core (n_sub),
 * members (n_members, paper centre indices).  Subdomain i holds
 * members[offsets[i] .. offsets[i+1]): its n_core[i] core centres, then its
 * overlap, nearest first. */
int rbf_schwarz_subdomains(const rbf_ctx* ctx, int64_t* offsets, int32_t* n_core, int64_t* members);

/* Learned narrow-band cull (Sec. II.A.3: the interpolant is needed only in a
 * narrow volume around the surface).  A network
 *   u = (x - centre) * scale -> 128 -> 128 -> 128 -> 128 -> y,
 * SiLU after every hidden layer, predicts f(x) / tau.  Parameters, float32,
 * RBF_NET_PARAMS of them in this order: W1 [128][3], b1 [128], W2 [128][128],
 * b2, W3 [128][128], b3, W4 [128][128], b4, w5 [128], b5 [1] (W_l[out][in]).
 * The three 128 x 128 layers run on the matrix cores in bf16 with float32
 * accumulation, the others in float32. */
#define RBF_NET_PARAMS 50177

typedef struct {
    int64_t support_bricks;   /* bricks of 4 x 2 x 2 nodes with a centre within the cutoff */
    int64_t kept_bricks;      /* of those, evaluated exactly */
    int64_t useful_pairs;     /* node-centre pairs with r^2 <= cutoff^2 of the kept bricks */
    int64_t examined_pairs;   /* pairs the exact sum computed */
} rbf_cull_stats;

/* Install a network on the context (params: HOST array of RBF_NET_PARAMS
 * floats; centre: host double[3]); resets the Adam state.  Synchronises. */
int rbf_net_set(rbf_ctx* ctx, const float* params, const double centre[3], double scale, double tau,
                void* stream);
/* Current parameters into a HOST array of RBF_NET_PARAMS floats.  Synchronises. */
int rbf_net_get(rbf_ctx* ctx, float* params, void* stream);
/* y = network(x) for n positions x (device n x 3 float64); y: device n float32. */
int rbf_net_forward(rbf_ctx* ctx, const double* x, int64_t n, float* y, void* stream);
/* Gradient of the loss mean_i (y_i - f_i / tau)^2 over the n samples
 * (x: device n x 3, f: device n float64 values of the interpolant) into grad
 * (device, RBF_NET_PARAMS floats, the parameter order above); *loss (host,
 * may be NULL) gets the loss.  Synchronises. */
int rbf_net_gradient(rbf_ctx* ctx, const double* x, const double* f, int64_t n, float* grad, double* loss,
                     void* stream);
/* Adam (lr, b1 = 0.9, b2 = 0.999, eps = 1e-8) over `epochs` passes of the n
 * samples in their given order, `batch` consecutive samples a step.
 * *loss (host, may be NULL) gets the mean loss of the last pass.
 * Synchronises. */
int rbf_net_train(rbf_ctx* ctx, const double* x, const double* f, int64_t n, int batch, int epochs, double lr,
                  double* loss, void* stream);
/* f on a grid with the learned cull: nodes outside the support (no centre
 * within the cutoff of their brick) get 0; the network runs on every node of
 * the support; a support brick is evaluated exactly (float32 pair sums, as
 * rbf_eval_grid) when one of its nodes has |y| < e_val or has a support node
 * of the opposite sign of y within 3 grid steps along every axis; every other
 * support node gets tau * y.  out: device float32, x fastest.  stats: host,
 * may be NULL.  Synchronises. */
int rbf_eval_grid_culled(rbf_ctx* ctx, const double* c, const rbf_grid* grid, float* out, double e_val,
                         rbf_cull_stats* stats, void* stream);

/* Sizes and pair counts of the context (host call, no device work). */
int rbf_get_stats(const rbf_ctx* ctx, rbf_stats* stats);

/* rbf_eval_grid in float32 for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, hosts that forbid
 * allocation): it calls no hipMalloc/hipFree and no allocating library
 * routine.  The same result as rbf_eval_grid(..., RBF_FP32, ...), bit for
 * bit (the same kernels); its scratch memory (the marks of the bricks of
 * 4 x 2 x 2 nodes with a centre in reach, and the list of the tiles of two
 * bricks that hold them) is a fixed array of 48 MiB + 64 KiB in device memory
 * that the library holds on every device it runs on until the process ends.
 *   c: device 3n float64 weights; out: device float32, dims[0]*dims[1]*dims[2]
 *   values, x fastest.
 * Limits (RBF_EINVAL with a message beyond them): a context with a cutoff,
 * a grid whose spacing is fine against sigma (the brick sums apply; else use
 * rbf_eval_grid), at most 2^21 bricks (e.g. 256^3 nodes = 2^20 bricks)
 * whose marks and tile list fit the array, the context's device current.  Every call on a device shares that device's
 * array and the context's work vectors: calls that overlap on one device
 * (two streams, two threads) race.  Synchronises with `stream`. */
int rbf_eval_grid_noalloc(rbf_ctx* ctx, const double* c, const rbf_grid* grid, float* out, void* stream);

/* Pairs one rbf_eval_grid over `grid` evaluates: useful = node-centre pairs
 * with r^2 <= cutoff^2 (decided in float64), examined = pairs the kernel
 * computes.  Synchronises with `stream`. */
int rbf_count_grid_pairs(rbf_ctx* ctx, const rbf_grid* grid, int64_t* useful,
                         int64_t* examined, void* stream);

/* Kernel timing for measurement tools (process-wide, off by default).
 * Between rbf_profile_begin() and rbf_profile_end() pair-sum kernel launches
 * carry HIP start/stop events in their dispatch on the stream they run on:
 * every launch, except float32 operator launches, of which one in three is
 * timed (the first, fourth, ...).  rbf_profile_end() waits for them and
 * reports, per launch kind (operator = rbf_matvec and the solves,
 * evaluation = grid and point evaluation) and precision, the timed launches,
 * their summed device time and the pairs they evaluated.  Not thread-safe. */
typedef struct {
    int64_t launches[2][2];        /* timed launches [kind: 0 operator, 1 evaluation][RBF_FP32 / RBF_FP64] */
    double kernel_ms[2][2];        /* summed event-to-event time of those launches */
    int64_t useful_pairs[2][2];    /* pairs with r^2 <= cutoff^2 they evaluated (float32 grids
                                      with a cutoff, summed without lists, count none:
                                      rbf_count_grid_pairs gives their pairs) */
    int64_t examined_pairs[2][2];  /* pairs they computed (list entries x 16) */
} rbf_profile;

int rbf_profile_begin(void);
int rbf_profile_end(rbf_profile* out);

/* Issue rates of the current device's vector ALU, measured by
 * register-resident loops that fill every wave slot (eight waves per SIMD),
 * as evidence for the float32 pair kernel's roofline (measurement, not part
 * of the method): float32 FMAs (VOP2, unpacked; eight independent chains per
 * lane), the same FMA in its DPP row-broadcast form, v_exp_f32, chains of one
 * v_exp_f32 with three or seven FMAs, and the float32 pair kernel's own
 * 16-step chunk bodies (inner and masked) on register operands, without the
 * kernel's list reads, gathers and per-chunk set-up.  Runs seven short
 * kernels (milliseconds each) on `stream` and synchronises with it;
 * allocates a 2 MB output from the library's cache. */
typedef struct {
    int compute_units;
    double fma_per_s;                /* lane FMAs per second (VOP2) */
    double exp_per_s;                /* lane exponentials per second */
    double exp_3fma_per_s;           /* lane (exp + 3 FMA) chains per second */
    double exp_7fma_per_s;           /* lane (exp + 7 FMA) chains per second */
    double dpp_fma_per_s;            /* lane FMAs per second, DPP row-broadcast form */
    double inner_pair_steps_per_s;   /* pair steps per second of the inner chunk body */
    double masked_pair_steps_per_s;  /* pair steps per second of the masked chunk body */
} rbf_rates;

int rbf_measure_rates(rbf_rates* out, void* stream);

/* Release every resource of the context (NULL is ignored).  Waits for work
 * enqueued by the context. */
void rbf_destroy(rbf_ctx* ctx);

/* Message describing the last error on `ctx`, or on the calling thread when
 * ctx is NULL (e.g. after a failed rbf_setup).  Never NULL. */
const char* rbf_last_error(const rbf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RBF_H */
