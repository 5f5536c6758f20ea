/*
 * mg.h - C ABI of the MI355X (gfx950) variable-coefficient multigrid pressure
 * solver.
 *
 * The solver computes the pressure of the projection step of a two-phase
 * incompressible flow solver: the non-separable Poisson equation
 *     div( (1/rho) grad p ) = S                                   (paper eq. 9)
 * discretised with the cell-centred second-order scheme of eq. (10) on a
 * uniform grid of cubic cells, homogeneous Neumann walls.  In three dimensions
 * and with the h^2 of eq. (10) folded into the right-hand side b:
 *     (L p)_c = sum over the 6 faces f of c of  beta_f (p_nb(f) - p_c) = b_c,
 * beta_f = the face value of alpha = 1/rho (for example the harmonic estimate of
 * eqs. 11-12 or an arithmetic average; the library takes faces, not cells).
 *
 * The result is the unique mean-zero p with L p = b - mean(b) (the Neumann
 * problem is solvable only for the mean-free part of b).  It is reached with the
 * modified V-cycle of Sec. 2.3 (features 1-6): red-black Gauss-Seidel smoothing,
 * residual restriction by linear interpolation, flux-conserving prolongation
 * (eqs. 13-14), coarse operators rediscretised from averaged faces, an exact
 * coarsest-grid solve, and convergence reported with the average reduction rate
 * gamma of eq. (15).  An FP32-refined mode runs the V-cycles in FP32 inside an
 * FP64 iterative refinement loop.
 *
 * ---------------------------------------------------------------------------
 * Layout (all arrays device memory, C order, i fastest):
 *   cells   p, b:  [nz][ny][nx]          double
 *   x-faces bx:    [nz][ny][nx+1]        face i lies between cells i-1 and i
 *   y-faces by:    [nz][ny+1][nx]        face j lies between cells j-1 and j
 *   z-faces bz:    [nz+1][ny][nx]        face k lies between cells k-1 and k
 * Wall faces (i = 0 or nx, j = 0 or ny, k = 0 or nz) are ignored and treated
 * as 0.  Every interior face coefficient must be finite and > 0.
 *
 * Streams are hipStream_t passed as void* (NULL = the default stream).  Every
 * call returns an mg_status; no C++ exception crosses this boundary.  A handle
 * is not thread-safe; a server is.
 * ---------------------------------------------------------------------------
 */
#ifndef MG_H_
#define MG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_PENDING = 1,             /* mg_poll: request not finished yet */
    MG_E_INVALID = -1,          /* bad argument, grid, option or coefficient */
    MG_E_WORKSPACE = -2,        /* workspace missing, misaligned or too small */
    MG_E_HIP = -3,              /* a HIP runtime call failed (message in mg_last_error) */
    MG_E_NOT_CONVERGED = -4,    /* max_cycles reached; p holds the last iterate */
    MG_E_DIVERGED = -5,         /* residual became NaN or grew by > 1e6 */
    MG_E_BUDGET = -6,           /* request footprint exceeds the server arena */
    MG_E_NOT_FOUND = -7         /* unknown ticket */
} mg_status;

typedef enum { MG_FP64 = 0, MG_FP32_REFINED = 1 } mg_precision;
typedef enum { MG_BC_NEUMANN = 0 } mg_bc;

typedef struct {
    int nx, ny, nz; /* cells per direction, each >= 2 */
} mg_grid;

#define MG_MAX_LEVELS 24
#define MG_MAX_COARSE_CELLS 512   /* the coarsest grid is solved by a dense inverse */
#define MG_MAX_HISTORY 256

typedef struct {
    int precision;   /* mg_precision */
    int nu1, nu2;    /* pre- and post-smoothing red-black sweeps (default 2, 2) */
    int n_coarsest;  /* halve every dimension while all are even and the largest
                        exceeds n_coarsest (default 4); the coarsest grid must have
                        <= MG_MAX_COARSE_CELLS cells */
    int inner_m;     /* FP32 V-cycles per FP64 outer iteration (refined mode, default 3) */
    int max_cycles;  /* V-cycles (FP64) or outer iterations (refined), default 100 */
    int profile;     /* nonzero: time every kernel launch with HIP events (stats.kernel_*) */
    int tile;        /* smoother kernel: 0 = automatic (each level's variant is chosen by
                        timing every variant at setup; choices are cached per grid size and
                        precision, in memory and, if the environment variable MG_TUNE_CACHE
                        names a file, in that JSON-lines file), -1 = reference
                        one-colour-per-pass kernels on every level, 1..MG_NUM_TILES = one fixed
                        variant of the fused red-black sweep on every level that has a
                        ping-pong buffer.  With nu1 = 2 in refined mode, a level's
                        pre-smoothing pass may also form and restrict the residual (chosen by
                        the same timing; always, for a fixed variant that has such a pass).
                        Every choice gives bit-identical results. */
    int graph;       /* nonzero: capture one iteration's launches into a hipGraph on the first
                        iteration of a solve and replay it for the others (fewer host launches;
                        identical results).  Ignored when profile is set.  The server always
                        uses graphs. */
    int krylov;      /* MG_KRYLOV_NONE (default): iterate V-cycles.  MG_KRYLOV_FCG (FP64 precision
                        only): flexible conjugate gradients on -L (Notay's FCG(1)) with one V-cycle
                        from zero as the preconditioner of every iteration; each new direction is
                        made -L-orthogonal to the previous one explicitly, which the V-cycle needs
                        since its restriction and prolongation are not transposes.  The residual
                        b_bar - L p is recomputed every iteration, so history and tolerance mean
                        the same as for the V-cycle iteration; stats.cycles counts iterations (one
                        V-cycle each).  Needs 32 more bytes of workspace per cell. */
    /* Paper-faithful cycle variants (the defaults give the standard cycle).  Any omega, and
       restrict64, run through the fused passes (bit-identical to the reference kernels); with
       restrict64 the residual is restricted by a separate pass (the fused pre-smoothing passes
       restrict with the 8-child mean only). */
    double omega;          /* SOR factor of the red-black smoother, 0 < omega < 2 (feature 5);
                              default 1 = Gauss-Seidel */
    int restrict64;        /* 1: 64-point restriction (transpose of trilinear interpolation, times 4)
                              instead of the 8-child mean (feature 3); default 0 */
    int coarse_gmres;      /* 0 (default): exact coarsest solve; 1..MG_GMRES_MAX_M: restarted
                              GMRES(coarse_gmres) on the coarsest grid (feature 6), FP64 */
    int coarse_gmres_maxit;  /* GMRES iteration cap, default 200 */
    double coarse_gmres_tol; /* GMRES relative residual target, default 1e-3 */
} mg_options;

#define MG_GMRES_MAX_M 16

enum { MG_KRYLOV_NONE = 0, MG_KRYLOV_FCG = 1 };

/* Fused sweep variants: variant v uses tile (v-1)/3 of the list 64x8, 128x4,
   128x8, 64x16 (one sweep per pass), 64x4, 64x8, 128x8, 64x16 (two sweeps per
   pass), with a target of about 256, 1024 or 4096 workgroups for (v-1) mod 3 =
   0, 1, 2.  The last two two-sweep tiles exist in FP32 only; in FP64 they run
   as 64x8. */
#define MG_NUM_TILES 24

/* Kernel classes reported in mg_stats when options.profile is set. */
enum {
    MG_K_SMOOTH = 0,      /* red-black Gauss-Seidel sweeps on the coarse levels (level >= 1) */
    MG_K_RESTRICT = 1,    /* residual + restriction, all levels */
    MG_K_PROLONG = 2,     /* prolongation + correction, all levels */
    MG_K_COARSE = 3,      /* coarsest dense solve */
    MG_K_NORM = 4,        /* convergence residual + norm (FP64 mode) */
    MG_K_REFINE = 5,      /* FP64 refinement residual and update (refined mode) */
    MG_K_OTHER = 6,       /* projections, reductions, fills */
    MG_K_SMOOTH_FINE = 7, /* the smoother on the finest level (level 0); the classes are disjoint */
    MG_K_KRYLOV = 8,      /* Krylov vector passes: dot products, direction, update, residual */
    MG_K_COUNT = 9
};

typedef struct {
    int status;                       /* mg_status of the solve */
    int levels;                       /* hierarchy depth */
    int cycles;                       /* V-cycles run (FP32 cycles in refined mode) */
    int outer;                        /* outer iterations (refined) or = cycles (FP64) */
    int nhist;                        /* entries in history */
    double history[MG_MAX_HISTORY];   /* relative residual ||b_bar - L p|| / ||b_bar||
                                         before the first cycle and after each cycle
                                         (FP64) or outer iteration (refined) */
    double rel_residual;              /* final relative residual */
    double gamma;                     /* eq. (15): (R_nc / R_0)^(1/nc) */
    double mean_b;                    /* mean of b removed before solving */
    double norm_b;                    /* ||b - mean(b)||_2 */
    double solve_ms;                  /* wall time of mg_solve (stream synchronised) */
    double kernel_ms[MG_K_COUNT];     /* summed kernel time per class (profile only) */
    long long kernel_launches[MG_K_COUNT];
    double kernel_bytes[MG_K_COUNT];  /* algorithmic HBM bytes per class (profile only) */
} mg_stats;

typedef struct mg_handle mg_handle;

/* Fill *o with the defaults listed above.  Returns MG_E_INVALID if o is NULL. */
mg_status mg_default_options(mg_options *o);

/*
 * Bytes of device workspace mg_setup needs for grid g and options o (hierarchy
 * faces, cell weights, per-level unknowns/right-hand sides, the FP32 copy in
 * refined mode, the coarsest dense inverse, reduction scratch).  Pure; no device
 * call.  Errors: MG_E_INVALID for NULL arguments, a dimension < 2, or a coarsest
 * grid larger than MG_MAX_COARSE_CELLS.
 */
mg_status mg_workspace_bytes(const mg_grid *g, const mg_options *o, size_t *bytes);

/*
 * Build the hierarchy for one coefficient field of the pressure equation (9),
 * discretised by eq. (10) with face coefficients such as those of eqs. (11)-(12)
 * (Sec. 2.3): copy faces with zero walls, coarsen faces level by level on the
 * power-of-two hierarchy of Sec. 2.3 (coarse face = mean of the 2x2 fine faces it
 * covers: restriction and prolongation are not tied to each other, feature list of
 * Sec. 2.3), cell weights for the flux-conserving prolongation of eqs. (13)-(14)
 * (feature 4), dense inverse of the coarsest operator (the exact limit of the
 * coarsest-grid GMRES of feature 6), FP32 copies in refined mode.
 * bx, by, bz: device double arrays in the layout above; read on `stream`, the
 * caller may reuse them once the call returns.  ws: caller-owned device
 * workspace of ws_bytes >= mg_workspace_bytes(), 256-byte aligned, which must
 * outlive the handle; the library owns its contents until mg_destroy.
 * bc must be MG_BC_NEUMANN.  Blocking: the stream is synchronised before return.
 * Errors: MG_E_INVALID (NULL pointer, bad bc, a non-finite or non-positive
 * interior coefficient found by the device check), MG_E_WORKSPACE, MG_E_HIP.
 */
mg_status mg_setup(const mg_grid *g, const mg_options *o, const double *bx, const double *by,
                   const double *bz, mg_bc bc, void *ws, size_t ws_bytes, void *stream,
                   mg_handle **out);

/*
 * Solve L p = b - mean(b) (eq. 9 in the discrete form of eq. 10, Neumann walls) with
 * the modified V-cycle of Sec. 2.3 (red-black Gauss-Seidel smoothing, feature 5;
 * residual restriction by linear interpolation, feature 3; flux-conserving
 * prolongation, feature 4 with eqs. 13-14; exact coarsest solve, feature 6) to
 * relative residual ||b_bar - L p||_2 / ||b_bar||_2 <= tol (the convergence test
 * below eq. 15; the average reduction rate gamma of eq. (15) is reported in st).
 * rhs: device double [nz][ny][nx], not modified.  p: device double, in/out;
 * on entry the initial guess, on return the mean-zero solution (or the last
 * iterate).  Both must be 16-byte aligned (the finest-level passes access them
 * as 16-byte vectors; torch allocations are).  st (optional, host): statistics.
 * Blocking on return.  A zero b_bar gives p = 0 and MG_OK.
 * Errors: MG_E_NOT_CONVERGED (p = last iterate, st valid), MG_E_DIVERGED,
 * MG_E_INVALID (NULL handle/array, rhs or p not 16-byte aligned, tol not finite
 * or < 0; nothing is launched), MG_E_HIP.
 */
mg_status mg_solve(mg_handle *h, const double *rhs, double *p, double tol, mg_stats *st,
                   void *stream);

/* Release host-side state.  The workspace belongs to the caller.  NULL is ignored. */
void mg_destroy(mg_handle *h);

/*
 * For callers that cannot allocate memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): mg_setup followed by mg_solve
 * on one coefficient field, with the workspace taken from a device array of
 * MG_STATIC_WORKSPACE_BYTES inside the library instead of the caller.  The call
 * makes no device or pinned allocation (no hipMalloc, hipFree, hipHostMalloc,
 * graph or event); each GPU the library runs on holds its own copy of the array
 * from the first call on it until the process ends.  Grids whose workspace
 * (mg_workspace_bytes) exceeds MG_STATIC_WORKSPACE_BYTES are refused: every grid
 * up to 128^3 fits in both precisions.
 * Arguments and results as mg_setup and mg_solve (g, o, faces, bc; rhs, p, tol,
 * st); stream must belong to the current device.  options.profile and
 * options.graph are ignored (both would allocate); smoother variants come from
 * the tuning cache of earlier setups of the same grid size, else one fixed
 * variant (every variant gives bit-identical results).  Blocking on return.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU
 * (two host threads, or streams the caller has not ordered) race and give
 * undefined results.  Nothing in the array needs to survive between calls; each
 * call initialises what it reads.
 * Errors: those of mg_setup and mg_solve; MG_E_WORKSPACE for a grid larger than
 * the static workspace (nothing is launched).
 */
#define MG_STATIC_WORKSPACE_BYTES (160u * 1024u * 1024u)
mg_status mg_solve_static(const mg_grid *g, const mg_options *o, const double *bx, const double *by,
                          const double *bz, mg_bc bc, const double *rhs, double *p, double tol, mg_stats *st,
                          void *stream);

/* Hierarchy inspection (for tests): number of levels and dims of level l. */
mg_status mg_level_dims(const mg_handle *h, int l, int *nx, int *ny, int *nz);

/* Smoother variant used on level l (-1 reference, 1..MG_NUM_TILES fused; the
   coarsest level, which is not smoothed, reports 0). */
mg_status mg_level_tile(const mg_handle *h, int l, int *tile);

/*
 * Copy level l's FP64 faces and cell weights into caller device buffers of the
 * layout above (a has [nz][ny][nx]); any pointer may be NULL to skip it.
 * Runs on `stream` and synchronises it.  Errors: MG_E_INVALID, MG_E_HIP.
 */
mg_status mg_copy_level(const mg_handle *h, int l, double *bx, double *by, double *bz, double *a,
                        void *stream);

/* ------------------------------------------------------------------------- */
/* Projection step around the solve                                           */
/* ------------------------------------------------------------------------- */
/*
 * The pressure equation (9) comes from the flow solver's Chorin projection on
 * the staggered MAC mesh (Sec. 2.2): velocity components on the faces normal to
 * them (u on x-faces, v on y-faces, w on z-faces, the face layout above),
 * pressure in the cells, centred differences.  Its source is S = div(u*) / dt,
 * u* the velocity before projection, and the projected velocity is
 * u = u* - dt (1/rho)_f grad p.  With cubic cells of side h and the h^2 of
 * eq. (10) folded into b, the three calls below compute
 *     b_c = (h/dt) * sum_d (u_d(upper face of c) - u_d(lower face of c))
 *     u_f = u*_f - (dt/h) * beta_f * (p(c+) - p(c-))     (interior faces f)
 * so that the discrete divergence of the projected field is (dt/h^2)(b - L p),
 * zero to the solve's tolerance.  Wall faces of the velocity are used as given
 * by the divergence (a nonzero wall flux gives b a nonzero mean, which the solve
 * removes) and never changed by the correction.  Evaluation order is fixed and
 * has no fused multiply-adds: b = scale*((du + dv) + dw) and
 * u_f = u_f - (scale*beta_f)*(p(c+) - p(c-)).  FP64 throughout.
 */

/*
 * b = scale * (net outflow of the face velocity out of each cell); scale = h/dt
 * gives the right-hand side of the projection step.  g: cells per direction
 * (each >= 0; an empty grid is a no-op).  u, v, w: device double face arrays
 * (x-, y-, z-faces, walls included and read); b: device double [nz][ny][nx],
 * written.  Asynchronous on `stream` (no synchronisation); the caller keeps the
 * arrays alive until the stream has passed this call.
 * Errors: MG_E_INVALID (NULL grid/array, negative dimension, non-finite scale,
 * grid too large for one launch), MG_E_HIP (launch failure).
 */
mg_status mg_divergence(const mg_grid *g, const double *u, const double *v, const double *w, double scale,
                        double *b, void *stream);

/*
 * u -= scale * beta * (p(c+) - p(c-)) on every interior face, beta the handle's
 * level-0 face coefficients (the ones mg_setup received); scale = dt/h gives the
 * velocity correction of the projection step.  Wall faces are not touched.
 * p: device double cells; u, v, w: device double face arrays, in/out, of the
 * handle's grid.  Asynchronous on `stream`.  Errors: MG_E_INVALID (NULL
 * handle/array, non-finite scale), MG_E_HIP.
 */
mg_status mg_correct_velocity(const mg_handle *h, const double *p, double scale, double *u, double *v,
                              double *w, void *stream);

/*
 * The whole projection step for the handle's coefficient field: b =
 * mg_divergence(u, v, w, h/dt); mg_solve(b, p, tol); on MG_OK,
 * mg_correct_velocity(p, dt/h, u, v, w).  dt: time step, hcell: cell size h
 * (both finite and > 0).  b: device double cells, receives the right-hand side
 * (workspace owned by the caller).  p: in/out as in mg_solve (initial guess in,
 * mean-zero pressure out, in the h^2-scaled units of eq. 10).  u, v, w: in/out:
 * u* in, projected velocity out.  st: as in mg_solve.  Blocking on return.
 * If the solve does not succeed, its status is returned and u, v, w are left
 * unchanged (b and p hold what the solve left).  b and p must be 16-byte aligned,
 * as in mg_solve.  Errors: those of mg_solve, and MG_E_INVALID for a bad dt or h.
 */
mg_status mg_project(mg_handle *h, double *u, double *v, double *w, double dt, double hcell, double *b,
                     double *p, double tol, mg_stats *st, void *stream);

/* ------------------------------------------------------------------------- */
/* Material properties from a level set                                       */
/* ------------------------------------------------------------------------- */
/*
 * Face coefficients for mg_setup built on the device from a level set phi
 * (Sec. 2.2): the indicator is the smoothed Heaviside of half-width eps (the
 * paper resolves it over three to four cells; eps = 1.5 h is typical),
 *     I = 0 (phi <= -eps), 1 (phi >= eps), (1/2)(1 + x + sin(pi x)/pi), x = phi/eps,
 * the density rho = rho_g + (rho_l - rho_g) I (eq. 8), alpha = 1/rho, and each
 * interior face gets the arithmetic mean of its two cells' alpha (harmonic = 0)
 * or their harmonic mean, eqs. (11)-(12) (harmonic = 1).  Wall faces are 0.
 * Fixed evaluation order without fused multiply-adds: x = phi/eps,
 * I = 0.5*((1 + x) + sin(pi*x)/pi), alpha = 1/(rho_g + (rho_l - rho_g)*I),
 * 0.5*(a + b) or (2*a*b)/(a + b).
 * g: cells per direction (each >= 1).  phi: device double [nz][ny][nx], positive
 * in the liquid.  bx, by, bz: device double face arrays (layout above), every
 * entry written.  rho_l, rho_g, eps finite and > 0.  Asynchronous on `stream`.
 * Errors: MG_E_INVALID (NULL grid/array, a dimension < 1, a bad density, eps or
 * harmonic flag, a grid too large for one launch), MG_E_HIP (launch failure).
 */
mg_status mg_faces_from_levelset(const mg_grid *g, const double *phi, double rho_l, double rho_g, double eps,
                                 int harmonic, double *bx, double *by, double *bz, void *stream);

/* ------------------------------------------------------------------------- */
/* Continuous-batching solve server                                           */
/* ------------------------------------------------------------------------- */

typedef struct mg_server mg_server;

typedef struct {
    mg_options solver;    /* options for every request (precision, sweeps, ...) */
    int max_slots;        /* concurrent resident problems, 1..256 */
    int nstreams;         /* entries of `streams`, 0..256; 0: the server creates max_slots HIP
                             streams of its own (default priority) */
    void *const *streams; /* caller-created hipStream_t handles (for example torch streams, which
                             must have the default priority); the server runs all device work of
                             its requests on them and never destroys them.  They must outlive the
                             server.  The array itself is copied by mg_server_create. */
} mg_server_options;

typedef struct {
    mg_grid grid;
    const double *bx, *by, *bz;   /* device faces, layout above */
    const double *rhs;            /* device right-hand side */
    double *p;                    /* device in/out: initial guess, then the solution */
    double tol;
    void *stream;                 /* the stream on which the caller produced bx, by, bz, rhs and p
                                     (NULL: the default stream).  mg_batch_submit records an event
                                     on it; the server's work on the request starts after that
                                     event, so writes enqueued there before the submit are seen. */
} mg_request;

typedef struct {
    int status;                   /* final mg_status of the request */
    mg_stats stats;
    double submit_ms, start_ms, finish_ms;   /* server clock */
} mg_result;

typedef struct {
    int classes;                  /* size classes seen (one per distinct grid) */
    int graphs;                   /* iteration graphs built (one per class and batch capacity) */
    long long replays;            /* graph replays (one outer iteration of a whole class each) */
    long long problem_iterations; /* outer iterations summed over problems (members per replay) */
    int max_batch;                /* most problems advanced by one replay */
    int resident;                 /* problems resident now */
    long long completed;          /* requests finished (any status) */
} mg_server_info;

/*
 * Arena bytes one request of grid g takes in a server whose solver options are
 * o: its workspace (mg_workspace_bytes) plus a copy of p (8 bytes per cell), the
 * server iterating on the copy so that all of a problem's arrays share one
 * layout, rounded up to 256 bytes.  Pure; no device call.  Errors: as
 * mg_workspace_bytes.
 */
mg_status mg_server_request_bytes(const mg_grid *g, const mg_options *o, size_t *bytes);

/*
 * Create a server that keeps each admitted request's hierarchy resident in
 * `arena` (caller-owned device memory of arena_bytes, 256-byte aligned; the HBM
 * budget; it must outlive the server).  A scheduler thread admits requests in
 * arrival order as soon as fewer than max_slots are resident and their footprint
 * (mg_server_request_bytes) fits in the free part of the arena (first fit), and
 * builds their hierarchy in place.  Requests of one grid size form a size class
 * that advances together: each replay of the class's HIP graph is one outer
 * iteration (a V-cycle, or the inner FP32 V-cycles and the FP64 refinement step)
 * of every resident problem of the class, each kernel launch covering all of
 * them (the batched execution of Sec. 2.3's cycle for same-size problems); one
 * graph is built per size class and batch capacity (a power of two).  Converged
 * problems leave at once and release their memory; waiting requests join at the
 * next replay.  Classes run on the given streams (class k on streams[k mod
 * nstreams]) and overlap on the device.  The same request gives the same result
 * alone (mg_solve) or in any mix, bit for bit.  Errors: MG_E_INVALID, MG_E_HIP.
 */
mg_status mg_server_create(void *arena, size_t arena_bytes, const mg_server_options *o,
                           mg_server **out);

/*
 * Queue one solve (the pressure equation (9) in the form of eq. (10), as mg_solve).
 * The request's arrays must stay valid until mg_poll reports a final status; the
 * server reads them only after the work the caller enqueued on r->stream before
 * this call (an event is recorded there now).  When mg_poll reports a final status
 * the solution in r->p is complete (the server has synchronised its own stream).
 * rhs and p must be 16-byte aligned, as in mg_solve.
 * Thread-safe.  Errors: MG_E_BUDGET (workspace larger than the whole arena),
 * MG_E_INVALID, MG_E_HIP (event record failed).
 */
mg_status mg_batch_submit(mg_server *s, const mg_request *r, uint64_t *ticket);

/*
 * Non-blocking.  Returns MG_PENDING while the request is queued or running, else
 * its final status with *out filled (stats, timestamps); the ticket is then
 * forgotten.  Thread-safe.  Errors: MG_E_NOT_FOUND.
 */
mg_status mg_poll(mg_server *s, uint64_t ticket, mg_result *out);

/* Counters of the server's batched execution (a snapshot).  Errors: MG_E_INVALID. */
mg_status mg_server_stats(mg_server *s, mg_server_info *out);

/* Stop the scheduler after finishing all queued work, then free host state. */
void mg_server_destroy(mg_server *s);

/* Static description of a status code. */
const char *mg_status_string(mg_status s);

/* Message of the last failed call on this thread (empty string if none). */
const char *mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MG_H_ */
