/*
 * rok4e.h -- C ABI of the batched ROK4E reaction substep on MI355X (gfx950).
 *
 * Every cell of a batch is an independent adiabatic 0-D reactor at constant pressure
 * (the paper's reaction substep of the Simpler balanced splitting, Sec. 3.3
 * eq. e:simpler_balanced, and the reactor model of Sec. 4.4 eq. e:cv_reactor, read with
 * c_p and h_k).  Each cell integrates u = (Y_1..Y_ns, T) over [0, dt] with the
 * four-stage Rosenbrock-Krylov method ROK4E (Sec. 4, Algorithm a:ROK4E): a Krylov
 * basis of dimension M from finite-difference Jacobian-vector products (Sec. 4.3),
 * the transformed stages e:s_stage_row_transformed with the projected solve
 * e:solve_kry_jac, the embedded error estimate and the PI step-size controller.
 *
 * Conventions
 *  - All state arrays are device pointers in the structure-of-arrays layout:
 *    Y[k * n_cells + c] (species-major), T[c], p[c].  FP64 always.
 *  - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *    Calls that launch work are asynchronous on that stream.
 *  - Return value: ROK4E_OK (0) or a negative ROK4E_E* code; rok4e_strerror() names it.
 *    Argument errors are detected on the host before anything is launched.
 *  - Per-cell outcomes cannot be known synchronously; they go to per-cell status
 *    codes (ROK4E_CELL_*) readable through rok4e_cell_stats_ptr / rok4e_get_stats.
 *  - Units: W kg/mol, cp J/(kg K), hf J/kg at 298.15 K, A in cm-mol-s (ln A given),
 *    Ea J/mol, T K, p Pa, dt s.
 */
#ifndef ROK4E_H
#define ROK4E_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define ROK4E_OK 0
#define ROK4E_EINVAL (-1)    /* invalid argument (null pointer with n_cells > 0, sizes, tolerances, M) */
#define ROK4E_ENOMEM (-2)    /* device allocation failed */
#define ROK4E_EHIP (-3)      /* HIP runtime or launch error */
#define ROK4E_ECAPTURE (-4)  /* workspace too small, or PER_ATTEMPT, while the stream is being captured */
#define ROK4E_ENOTSUP (-5)   /* no kernel variant for this (n_species, M, precision, layout) */
#define ROK4E_ESTATIC (-6)   /* n_cells above ROK4E_STATIC_MAX_CELLS (rok4e_integrate_static) */

/* Per-cell status codes. */
#define ROK4E_CELL_OK 0
#define ROK4E_CELL_MAX_ATTEMPTS 1  /* attempt limit reached before dt; state = last accepted */
#define ROK4E_CELL_STEP_UNDERFLOW 2 /* step fell below 16 eps dt; state = last accepted */
#define ROK4E_CELL_BAD_INPUT 3     /* non-finite Y/T/p, T <= 0 or p <= 0; state untouched */

/* Precision of the right-hand side, Krylov basis and projected solve.  The state
 * update, the finite-difference perturbation and difference, the error norm and
 * the step controller are FP64 in both modes. */
#define ROK4E_FP64 0
#define ROK4E_MIXED 1

/* Cell scheduling (bitwise identical results).  PERSISTENT: one launch; segments pull
 * cells from a device work queue and integrate each to dt.  PER_ATTEMPT: one launch per
 * attempt over the cells still active, the per-cell integrator state (t, h, controller
 * memory, counters, f(u_n) and the Krylov basis) carried in device memory between
 * launches; the call synchronises the stream once per launch and returns
 * ROK4E_ECAPTURE inside a stream capture.  A reference schedule for comparison. */
#define ROK4E_PERSISTENT 0
#define ROK4E_PER_ATTEMPT 1

/* Integration method.  ROK4E: Algorithm a:ROK4E (the library's purpose).  RKDP45: the
 * explicit Dormand-Prince 5(4) pair (published tableau, first-same-as-last, the same error
 * norm, controller h* = h min(5, max(0.2, 0.9 err^(-1/5))), h0 = dt), the explicit
 * reference integrator of the efficiency study of Sec. 5; persistent schedule only
 * (ROK4E_ENOTSUP otherwise); M and the Krylov options are ignored. */
#define ROK4E_METHOD_ROK4E 0
#define ROK4E_METHOD_RKDP45 1

/* Order in which the persistent schedule hands out cells (bitwise neutral: every cell's
 * result is independent of it).  HOT_FIRST: by decreasing temperature, in bins of 16 K
 * (cells with invalid T last), so that the cells that take the most attempts start
 * first and the launch does not end on a few long cells; batches of fewer than eight
 * cells per segment in flight keep array order.  ARRAY: in array order. */
#define ROK4E_ORDER_HOT_FIRST 0
#define ROK4E_ORDER_ARRAY 1

/* Where the Jacobian-vector products of the Arnoldi process (Sec. 4.3) read the base-state
 * concentrations of each lane's reactions (bitwise neutral: the same values either way).
 * LDS: from the segment's LDS arrays.  PRIVATE: from a copy gathered into lane-private
 * memory once per basis (64-lane, one-slot layouts with M <= 8 only; elsewhere LDS).
 * AUTO: LDS, unless rok4e_tune chose otherwise. */
#define ROK4E_GATHER_AUTO 0
#define ROK4E_GATHER_LDS 1
#define ROK4E_GATHER_PRIVATE 2

typedef struct rok4e_mech rok4e_mech;   /* opaque handle */

/* Mechanism description; host arrays, copied to the device by rok4e_mech_create. */
typedef struct {
  int32_t n_species;          /* ns >= 1 */
  int32_t n_reactions;        /* nr >= 0 */
  const double* W;            /* [ns] molecular weight */
  const double* cp;           /* [ns] constant heat capacity */
  const double* hf;           /* [ns] formation enthalpy at 298.15 K */
  const int32_t* reac;        /* [nr * 2] reactant species of reaction j at 2j, 2j+1; -1 if absent */
  const int32_t* prod;        /* [nr * 2] product species, same layout */
  const double* lnAf;         /* [nr] ln of forward pre-exponential factor */
  const double* bf;           /* [nr] forward temperature exponent */
  const double* Ef;           /* [nr] forward activation energy */
  const double* lnAr;         /* [nr] reverse triple, same meaning */
  const double* br;
  const double* Er;
  int32_t n_elements;         /* E >= 0; 0: no element table (no balance check) */
  const int8_t* elem;         /* [ns * E] atoms of element e in species k at k*E + e, or NULL
                                 when E = 0.  rok4e_mech_create refuses (EINVAL) a mechanism
                                 in which a reaction changes the count of any element: the
                                 mass-action source then conserves elements and, with
                                 element-consistent weights, mass (Sec. 4.4) */
} rok4e_mech_desc;

typedef struct {
  int32_t M;              /* Krylov dimension, 1..16 (the method's implicitness; not tuned) */
  int32_t precision;      /* ROK4E_FP64 or ROK4E_MIXED */
  int32_t max_attempts;   /* attempts allowed per cell; <= 0 means 1000000 */
  int32_t fixed_steps;    /* 0: adaptive; n > 0: n equal steps, no error control */
  int32_t lanes_per_cell; /* 0: automatic; else 16, 32 or 64.  Changes the order in which
                             the production sums accumulate: results agree to rounding */
  int32_t waves_per_block;/* 0: automatic; 1..16 waves of 64 lanes per block (bitwise neutral;
                             at most 4 for one-slot layouts, 8 for two-slot ones, 16 with
                             waves_per_simd = 4) */
  int32_t blocks_per_cu;  /* 0: automatic; persistent-grid blocks per compute unit
                             (bitwise neutral) */
  int32_t scheduling;     /* ROK4E_PERSISTENT or ROK4E_PER_ATTEMPT (bitwise neutral) */
  int32_t method;         /* ROK4E_METHOD_ROK4E (default) or ROK4E_METHOD_RKDP45 */
  int32_t cell_order;     /* ROK4E_ORDER_HOT_FIRST (default) or ROK4E_ORDER_ARRAY (bitwise
                             neutral; persistent schedule) */
  int32_t jvp_gather;     /* ROK4E_GATHER_AUTO (default), _LDS or _PRIVATE (bitwise neutral;
                             persistent schedule) */
  int32_t waves_per_simd; /* 4: the persistent ROK4E kernel compiled for four waves per SIMD
                             (64-lane one-slot layouts with M <= 8, LDS reads; blocks of up to
                             16 waves); 3: three waves for one-slot layouts (two for others);
                             0 (automatic): the four-wave build for FP64 when the layout has
                             it, waves_per_block and blocks_per_cu are automatic and the JVP
                             gather is not private, else as 3.  Bitwise neutral */
  double h0;              /* first trial step; <= 0 means dt */
} rok4e_options;

/* Outcome of rok4e_tune. */
typedef struct {
  int32_t lanes_per_cell;  /* the chosen launch layout, also written to the handle's options */
  int32_t waves_per_block;
  int32_t blocks_per_cu;
  int32_t jvp_gather;
  int32_t waves_per_simd;
  float ms;                /* time of one integration of the batch with the choice */
  float ms_default;        /* the same with the options the handle had before (0 on a cache hit) */
  int32_t candidates;      /* layouts timed (0 on a cache hit) */
  int32_t from_cache;      /* 1: the choice came from the tuning cache and nothing was timed */
} rok4e_tune_result;

/* Bins of the attempt histogram: bin 0 counts cells with no attempt (invalid input), bin
 * b >= 1 cells with 2^(b-1) <= accepted + rejected < 2^b (the last bin also takes more). */
#define ROK4E_HIST_BINS 22

typedef struct {
  int64_t n_cells;        /* cells of the last integrate call */
  int64_t accepted;       /* accepted attempts, summed over cells */
  int64_t rejected;       /* rejected attempts, summed over cells */
  int64_t max_attempts;   /* largest accepted + rejected of any cell */
  int64_t status_count[4];/* cells per ROK4E_CELL_* status */
  int64_t attempt_histogram[ROK4E_HIST_BINS]; /* cells per attempt-count bin (above) */
} rok4e_stats;

/* Fills *o with the defaults (M = 4, FP64, automatic layout, persistent). */
void rok4e_options_default(rok4e_options* o);

/* Creates a handle on the current HIP device: validates the description (species
 * indices in range, finite parameters, W > 0, cp > 0), builds the device tables
 * (reaction parameters, species-major production lists) and selects the kernel
 * variant.  o may be NULL (defaults).  The caller keeps ownership of d and o. */
int rok4e_mech_create(const rok4e_mech_desc* d, const rok4e_options* o, rok4e_mech** out);

/* Frees the handle and its device memory (synchronises the device). NULL is a no-op. */
int rok4e_mech_destroy(rok4e_mech* m);

/* Replaces the launch options (layout, waves, grid, scheduling, M, precision,
 * max_attempts, fixed_steps, h0) of an existing handle. */
int rok4e_set_options(rok4e_mech* m, const rok4e_options* o);
int rok4e_get_options(const rok4e_mech* m, rok4e_options* o);

/* Sizes the per-cell workspace for up to max_cells cells.  integrate grows the
 * workspace on demand outside stream capture; inside a capture it returns
 * ROK4E_ECAPTURE instead, so call this before capturing. */
int rok4e_reserve(rok4e_mech* m, int64_t max_cells);

/* Integrates n_cells cells in place over [0, dt] (Algorithm a:ROK4E with relative
 * and absolute tolerances rtol > 0, atol >= 0).  Y, T are read and overwritten; p is
 * read only and constant over the substep.  n_cells == 0 is a no-op. */
int rok4e_integrate(int64_t n_cells, rok4e_mech* mech, double* Y, double* T, const double* p,
                    double dt, double rtol, double atol, void* stream);

/* As rok4e_integrate with a constant forcing added to f: S[(ns+1) * n_cells] in the
 * state layout (T last), the balancing term T(U_n) of the Simpler balanced splitting
 * (e:simpler_balanced: c_n = -T(U_n), reaction substep u' = R(u) - c_n).  S may be NULL. */
int rok4e_integrate_forced(int64_t n_cells, rok4e_mech* mech, double* Y, double* T,
                           const double* p, const double* S, double dt, double rtol,
                           double atol, void* stream);

/* As rok4e_integrate_forced with per-cell first trial steps (the h_0 input of Algorithm
 * a:ROK4E), for a caller that integrates the same cells over consecutive substeps:
 * h_io[n_cells] (device, FP64, may be NULL) holds on input each cell's first trial step
 * (<= 0 or non-finite: the option h0, else dt) and on output the step to start the next
 * call from: the controller's proposal after the cell's last attempt, or, when the last
 * accepted step had been shortened to end at dt, the larger of that proposal and the one
 * made before the shortening.  Cells with invalid input keep their entry.  ROK4E only
 * (ROK4E_ENOTSUP with a non-NULL h_io and ROK4E_METHOD_RKDP45).  S as for
 * rok4e_integrate_forced. */
int rok4e_integrate_ex(int64_t n_cells, rok4e_mech* mech, double* Y, double* T, const double* p,
                       const double* S, double* h_io, double dt, double rtol, double atol,
                       void* stream);

/* Reaction substep in the conservative variables of a compressible flow solver with the
 * auxiliary temperature equation (Sec. 5, e:chemical_source_balanced and
 * e:aux_t_equation).  U[(ns+5) * n_cells] (device, FP64, structure of arrays with stride
 * n_cells; read and overwritten) holds per cell rho Y_1 .. rho Y_ns (kg/m^3), rho,
 * rho u_x, rho u_y, rho u_z (kg/(m^2 s)) and rho E (J/m^3, E the total energy per unit
 * mass including the formation enthalpies: E = sum_k Y_k e_k(T) + |u|^2 / 2 with
 * e_k = h_f,k + c_p,k (T - 298.15) - Ru T / W_k).  S (same layout, may be NULL) holds
 * each row's balancing constant, the transport term of the conservative variables at the
 * start of the step.  The temperature is computed from U at the start of each cell's
 * integration and integrated with the state (ns + 6 rows: the species, T, rho, rho u,
 * rho E) with the source
 *   dT/dt = (-sum_k e_k F_k + |u|^2/2 F_rho - u . F_m + F_E) / (rho c_v),
 * F the forced derivatives of the conservative rows and rho c_v = sum_k rho Y_k
 * (c_p,k - Ru / W_k); the species energy of e:aux_t_equation is read as the internal
 * energy, under which the auxiliary temperature equals the temperature of U along the
 * exact solution.  The chemistry is that of a constant-volume reactor (c_k = rho Y_k /
 * W_k).  T_aux[n_cells] (device, may be NULL) receives the auxiliary temperature at dt.
 * A cell with non-finite input, rho <= 0, rho c_v <= 0 or a temperature <= 0 keeps U
 * (and its T_aux entry) and reports status 3.  Persistent schedule, FP64, ROK4E only
 * (ROK4E_ENOTSUP otherwise).  The handle's lane layout is used when it holds ns + 6
 * rows; otherwise the call uses the smallest layout that does (same options) and builds
 * its table image on first use, which returns ROK4E_ECAPTURE inside a stream capture.
 * Cells are handed out in array order; per-cell statistics as for rok4e_integrate. */
int rok4e_integrate_conservative(int64_t n_cells, rok4e_mech* mech, double* U, const double* S,
                                 double* T_aux, double dt, double rtol, double atol, void* stream);

/* Largest batch of rok4e_integrate_static: the size of its static device scratch. */
#define ROK4E_STATIC_MAX_CELLS (1 << 21)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): rok4e_integrate_forced that calls no
 * hipMalloc, hipFree or other allocating routine.  The same kernels and results (bit for
 * bit, on the persistent schedule whatever the handle's scheduling option; the handle's
 * method, M, precision, layout and cell order apply).  The per-call scratch (work-queue
 * counter, queue-order bins and the order of up to ROK4E_STATIC_MAX_CELLS cells, 8 MiB)
 * lives in a static device array of the library, one per GPU, held until the process
 * ends; its address is looked up when a handle is first created on that GPU.  Every call
 * on one GPU shares that array and keeps the last call's contents: calls that overlap on
 * one GPU (two streams, two host threads, two handles) race and must be serialised by the
 * caller.  The caller owns and passes the outputs: acc, rej, status (device int32
 * [n_cells] each, required for n_cells > 0) receive each cell's accepted and rejected
 * attempts and ROK4E_CELL_* status; rok4e_get_stats and the handle's per-cell arrays do
 * not describe this call.  Y, T, p, S, dt, rtol, atol as for rok4e_integrate_forced (S may
 * be NULL).  ROK4E_ESTATIC for n_cells > ROK4E_STATIC_MAX_CELLS; ROK4E_EINVAL for the
 * argument errors of rok4e_integrate_forced or a missing output; n_cells == 0 is a
 * no-op. */
int rok4e_integrate_static(int64_t n_cells, rok4e_mech* mech, double* Y, double* T,
                           const double* p, const double* S, double dt, double rtol,
                           double atol, int32_t* acc, int32_t* rej, int32_t* status,
                           void* stream);

/* Launch tuner (autotuning of the persistent kernel's result-neutral launch choices):
 * integrates a copy of the given batch (Y, T, p as for rok4e_integrate; the caller's
 * arrays are not modified) with each candidate launch layout and keeps the fastest in the
 * handle's options.  Candidates: every lane layout (lanes_per_cell 16, 32, 64) that holds
 * the ns + 1 state rows and M Krylov vectors, at its largest block and at half of it, and
 * for the layouts that have them the private-memory JVP gather (jvp_gather) and the
 * kernel held to four waves per SIMD (waves_per_simd).  Each is timed
 * with HIP events as the faster of two runs after a warm-up run.  Within a lane layout the
 * choices do not change any result bit; across lane layouts the production sums add in
 * another order (results agree to rounding).  The choice is kept in a process-wide cache
 * keyed by (GPU architecture and compute-unit count, n_species, n_reactions, M,
 * precision, method): a later call with the same key (on any handle) applies the cached
 * choice without timing anything, unless force is non-zero.  Allocates scratch for one
 * copy of Y and T, rebuilds the handle's tables for each lane layout and synchronises the
 * stream; ROK4E_ECAPTURE inside a stream capture, ROK4E_EINVAL for n_cells == 0.  out may
 * be NULL. */
int rok4e_tune(int64_t n_cells, rok4e_mech* mech, const double* Y, const double* T, const double* p,
               double dt, double rtol, double atol, int32_t force, rok4e_tune_result* out,
               void* stream);

/* ---- Splitting around the reaction substep (Sec. 3.3) ------------------------------
 * Model transport operator on an nx x ny x nz grid of cubic cells (cell
 * c = x + nx (y + ny z), the cell index of the state arrays): advection with velocity vel
 * along x and diffusion with diffusivity diff, second-order central differences, applied
 * to every state row (mass fractions and temperature):
 *   T(U)_r = -vel (U_{x+1} - U_{x-1}) / (2 dx) + diff (sum of six neighbours - 6 U) / dx^2
 * y and z are periodic.  Along x the grid is periodic, or open: the neighbour before x = 0
 * is a ghost cell holding a fixed inflow state, the neighbour after x = nx - 1 repeats that
 * cell (zero-gradient outflow).  An open grid has steady states that are not uniform (a
 * premixed stream reacting as it flows through), the discrete steady states the balanced
 * splitting is built to keep (definition d:steady_state_preserving). */
#define ROK4E_X_PERIODIC 0
#define ROK4E_X_INFLOW_OUTFLOW 1

typedef struct {
  int32_t nx, ny, nz;
  double dx;     /* m, > 0 */
  double vel;    /* m/s */
  double diff;   /* m^2/s, >= 0 */
  int32_t x_boundary;    /* ROK4E_X_PERIODIC or ROK4E_X_INFLOW_OUTFLOW */
  const double* inflow;  /* INFLOW_OUTFLOW: device array [n_species + 1], the inflow ghost
                            state (Y_1..Y_ns, T), owned by the caller and read by every call
                            that takes the grid; PERIODIC: NULL */
} rok4e_grid;

#define ROK4E_SPLIT_SIMPLER 0  /* Simpler balanced splitting, e:simpler_balanced */
#define ROK4E_SPLIT_STRANG 1   /* Strang splitting, e:strang_t1..e:strang_t3 (control) */

/* S[r * n + c] = T(U)_r at cell c (n = nx ny nz) for the state (Y, T).  Device pointers;
 * EINVAL for a bad grid (sizes, dx, diff, an unknown x_boundary, an inflow pointer missing
 * on an open grid or given on a periodic one) or null pointers. */
int rok4e_transport(const rok4e_grid* g, int32_t n_species, const double* Y, const double* T, double* S,
                    void* stream);

/* Device workspace bytes rok4e_split_step needs: six [ns + 1][n] FP64 arrays. */
size_t rok4e_split_workspace_bytes(const rok4e_grid* g, int32_t n_species);

/* One splitting step of size h for u' = T(u) + R(u) + src on the grid, in place in (Y, T):
 *   SIMPLER: c_n = -T(U_n); the reaction substep u' = R(u) + src - c_n over h (the batched
 *            ROK4E integration of the handle, forcing src - c_n); then the transport
 *            substep u' = T(u) + c_n over h / 2 (the balanced form's first transport half
 *            step is at rest and is skipped).  A steady state of T + R + src is kept.
 *   STRANG:  transport u' = T(u) over h / 2, reaction u' = R(u) + src over h, transport
 *            over h / 2.
 * Transport substeps use nsub >= 1 classical fourth-order Runge-Kutta steps.  src is an
 * optional cell-local constant source [(ns + 1) * n] (NULL: none), p the pressure per
 * cell.  work: device buffer of at least rok4e_split_workspace_bytes bytes, owned by the
 * caller.  Per-cell counts and status of the reaction substep as for rok4e_integrate. */
int rok4e_split_step(rok4e_mech* mech, const rok4e_grid* g, int32_t scheme, double* Y, double* T,
                     const double* p, const double* src, double h, double rtol, double atol, int32_t nsub,
                     void* work, size_t work_bytes, void* stream);

/* Evaluates the reactor right-hand side f(u) for every cell (Sec. 4.4, e:cv_reactor):
 * dY[k * n_cells + c], dT[c].  Inputs are not modified. */
int rok4e_rhs(int64_t n_cells, rok4e_mech* mech, const double* Y, const double* T, const double* p,
              double* dY, double* dT, void* stream);

/* Arnoldi process of Sec. 4.1 (e:jac_proj) at each cell's state, with the handle's M and
 * precision: Q[(c * M + j) * (ns+1) + r] (column j of cell c), H[(c * M + i) * M + j],
 * Meff[c].  Device output buffers sized by the caller.  For tests and diagnostics. */
int rok4e_arnoldi(int64_t n_cells, rok4e_mech* mech, const double* Y, const double* T,
                  const double* p, double* Q, double* H, int32_t* Meff, void* stream);

/* Diagnostic, not part of the method: the attainable FP64 vector FMA rate, the compute
 * roofline the integration kernel is measured against.  n_threads threads (a multiple of
 * 256) each run iters rounds of eight independent fused multiply-add chains and store
 * their sum in out[thread] (device, [n_threads], owned by the caller): 16 * n_threads *
 * iters FP64 operations.  EINVAL for a bad size or a null out. */
int rok4e_fma_probe(int64_t n_threads, int32_t iters, double* out, void* stream);

/* Copies the summary of the last integrate call to the host (synchronises stream). */
int rok4e_get_stats(rok4e_mech* m, rok4e_stats* out, void* stream);

/* Device pointers to the per-cell accepted/rejected/status arrays of the last call
 * (valid until the next reserve or destroy; owned by the handle). */
int rok4e_cell_stats_ptr(rok4e_mech* m, const int32_t** acc, const int32_t** rej,
                         const int32_t** status);

/* Copies the per-cell accepted/rejected/status counts of the last call into caller
 * buffers of n_cells int32 each (host or device pointers; any may be NULL), ordered on
 * stream.  Does not synchronise. */
int rok4e_copy_cell_stats(rok4e_mech* m, int32_t* acc, int32_t* rej, int32_t* status, void* stream);

/* Human-readable name of a return code (static string). */
const char* rok4e_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* ROK4E_H */
