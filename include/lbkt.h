/*
 * lbkt.h - C ABI of the MI355X (gfx950) finite-difference lattice Boltzmann step.
 *
 * Method: Pan, Xu, Zhang & Jiang, "Lattice Boltzmann approach to high-speed
 * compressible flows" (2007). One time step of the Kataoka-Tsutahara D2V9
 * discrete-velocity model (Sec. 2, Eqs. (e14)-(e18)) advanced by the forward
 * Euler / beta-mixed upwind finite-difference scheme (Eqs. (SEC-VON-1),
 * (SEC-VON-2a/2b)) with the added dissipation term lambda_i Laplacian(f_i)
 * (Eqs. (SEC-VON-11), (SEC-VON-13)):
 *
 *   f_i' = f_i - dt v_ia D_a f_i + dt lambda_i (d2/dx2 + d2/dy2) f_i + (f_i^eq - f_i)/tau
 *
 * with rho, u, T from Eqs. (e4), (e5), (e7) (R = 1, b = 2/(gamma-1)) and f^eq
 * from Eq. (e16). tau is in units of dt (the paper sets dt equal to the Knudsen
 * number). dx is used for both axes (the paper takes dx = dy).
 *
 * Data layout ("SoA planes"): a distribution array holds 9 planes, plane i in
 * the velocity order of Eq. (e14):
 *     0:(0,0) 1:(-c1,0) 2:(0,-c1) 3:(c1,0) 4:(0,c1)
 *     5:(-s,-s) 6:(s,-s) 7:(s,s) 8:(-s,s),   s = c2/sqrt(2)
 * Element (i, y, x) is at  f[i*pitch*ny + y*pitch + x]  (x fastest, pitch >= nx,
 * pitch a multiple of 64 elements, base pointer 256-byte aligned; the step
 * and the adjoint step write unspecified values into the padding columns
 * nx <= x < pitch, and no entry point reads them as data). Site (x, y)
 * has centre ((x+0.5) dx, (y+0.5) dx). Macroscopic fields (rho, ux, uy, p or T)
 * are dense row-major (ny, nx) float64 arrays. Sizes: pitch <= 2^27 elements,
 * nx and ny up to 2^31 - 1; an array may exceed 4 GiB (device memory is the
 * limit), except one problem of a batch (below 4 GiB).
 *
 * Precision: LB_F64 stores f in float64; LB_F32 stores f in float32 and widens
 * every load to float64, so moments, the division by rho, T, f^eq and the
 * stencil run in float64 and only the store rounds to float32. Adjoint fields
 * are always float64.
 *
 * Boundaries: one ghost cell per edge (the stencil is a 5-point cross, corners
 * are never read), edge order x-, x+, y-, y+:
 *   LB_BC_PERIODIC  wrap (both edges of an axis must be periodic)
 *   LB_BC_OUTFLOW   zero gradient: the ghost copies the adjacent interior cell
 *   LB_BC_WALL      reflecting wall on the cell face: ghost = adjacent interior
 *                   cell with the velocity planes mirrored across the wall
 *   LB_BC_INFLOW    Dirichlet: ghost = f^eq of state a
 *   LB_BC_SHOCK     (y edges only) ghost = f^eq(a) where its centre x lies behind
 *                   x_s = x0 + y/tan(angle) + speed t / sin(angle), t = step*dt,
 *                   and f^eq(b) elsewhere (a moving straight shock)
 *   split > 0       the first `split` ghost cells along the edge use f^eq(a)
 *                   whatever the kind (a wall that starts downstream).
 *
 * Conventions of every call:
 *   - All device pointers are caller-allocated (e.g. by PyTorch); the library
 *     never frees caller memory and returns no caller-visible allocation.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *     are asynchronous on that stream unless stated otherwise.
 *   - Parameter, size and alias errors are detected on the host before any
 *     launch and return a negative lb_status; lb_last_error() gives detail
 *     text (thread-local). HIP errors map to LB_EHIP.
 *   - Numerical blow-up is asynchronous: lb_moments records it in a device flags
 *     word, and lb_check_flags turns that word into LB_ENONFINITE.
 */
#ifndef LBKT_H
#define LBKT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LB_OK = 0,
  LB_EINVAL = -1,      /* null pointer, bad size, pitch or alignment */
  LB_EPARAM = -2,      /* c1 == c2, c1,c2,eta0,dx,dt,tau <= 0, beta outside [0,0.5], gamma <= 1, lambda < 0 */
  LB_EALIAS = -3,      /* input and output arrays overlap */
  LB_ENONFINITE = -4,  /* lb_check_flags: some site was non-finite or had rho <= 0 */
  LB_EHIP = -5,        /* a HIP runtime call failed */
  LB_ENOMEM = -6,      /* internal metadata allocation failed */
  LB_EUNSUPPORTED = -7 /* valid request the library does not implement */
} lb_status;

/* Storage precision. Entry points take it as an int32_t `prec` holding one of
 * these codes (as lb_edge.kind holds an lb_bc_kind): any other value returns
 * LB_EINVAL. */
typedef enum { LB_F64 = 0, LB_F32 = 1 } lb_prec;

typedef enum {
  LB_BC_PERIODIC = 0,
  LB_BC_OUTFLOW = 1,
  LB_BC_WALL = 2,
  LB_BC_INFLOW = 3,
  LB_BC_SHOCK = 4
} lb_bc_kind;

/* flags word bits written by lb_moments */
enum { LB_FLAG_NONFINITE = 1u, LB_FLAG_RHO_NONPOS = 2u, LB_FLAG_T_NONPOS = 4u };

typedef struct { double rho, ux, uy, p; } lb_state;

typedef struct {
  int32_t kind;        /* lb_bc_kind */
  int32_t split;       /* first `split` ghost cells along the edge are f^eq(a) */
  lb_state a, b;       /* INFLOW: a; SHOCK: a behind, b ahead */
  double x0, angle_deg, speed; /* SHOCK geometry */
} lb_edge;

typedef struct {
  int32_t nx, ny;      /* interior sites */
  int64_t pitch;       /* row pitch in elements (multiple of 64, >= nx) */
  double dx, dt;       /* grid spacing (both axes) and time step */
  double c1, c2, eta0; /* Eqs. (e14)-(e15) */
  double gamma;        /* specific-heat ratio, b = 2/(gamma-1) */
  double tau;          /* relaxation time in units of dt */
  double beta;         /* upwind mixing of Eqs. (SEC-VON-2a/2b), 0 <= beta <= 0.5 */
  double lambda[9];    /* dissipation coefficients lambda_i of Eq. (SEC-VON-11) */
  lb_edge edge[4];     /* x-, x+, y-, y+ */
} lb_grid;

/* Launch shape of the step kernels. The grid is cut into tiles of block_x
 * columns (64, 128 or 256: one thread per column) by `rows` rows (>= 1).
 * blocks = 0 launches one block per tile; blocks > 0 launches that many
 * persistent blocks (rounded down to a multiple of 8 where tiles are dealt to
 * the XCDs in bands), each looping over tiles. All zero (or a NULL tile) = the
 * default: 256 x 32 tiles, one block per tile, shrunk on small grids (rows down
 * to 2, then columns) to give at least 1024 tiles; one step per launch on a
 * float array takes about 52 rows where the row chunks then number a multiple
 * of 8 (each XCD's band of tiles is whole chunk rows) and there are at least
 * 1024 tiles of at least 32 rows, else 64 rows shrunk alike; the two-step pass takes at
 * most 11 rows (double) or 23 rows (float) by default, the three-step pass
 * 128 x 12 tiles. In the two-step pass a wavefront of 64 threads produces 60 columns, in
 * the three-step pass 58, so a tile is block_x / 64 * 60 (58) columns wide. */
typedef struct {
  int32_t block_x, rows, blocks;
  int32_t steps;   /* lb_run only: time steps per pass over the array, 1, 2 or 3; 0 = the
                      default: 3 for FP64 arrays below 4 GiB with ny >= 32; 16 on grids
                      of 4 rows with a periodic y axis, at least 64 columns and an array
                      below 4 GiB (a strip of 32 columns per block of four wavefronts,
                      one row each, its state kept on chip between the steps); else 2 (1 when
                      ny < 2). Several steps per pass keep the intermediate states in
                      registers (temporal blocking): 1/2 or 1/3 of the HBM traffic per
                      step, bitwise the result of single steps. An explicit 3 runs on
                      FP64 arrays below 4 GiB with ny >= 3; elsewhere LB_EUNSUPPORTED
                      from lb_run. */
} lb_tile;

/* Fill grid->lambda with Eq. (SEC-VON-13): c1 dx, c1 dx/10 (i = 1..4), 0 (i = 5..8). */
lb_status lb_default_lambda(lb_grid* grid);

/* Host-only validation of every field of *grid (no GPU needed): LB_EINVAL for
 * sizes and pitch, LB_EPARAM for scheme parameters and edge states,
 * LB_EUNSUPPORTED for pitch > 2^27 or lambda_1..4 (lambda_5..8) not all equal. */
lb_status lb_validate(const lb_grid* grid);

/* Number of elements of one distribution array (9 * pitch * ny). */
int64_t lb_array_elems(const lb_grid* grid);

/* Initialisation (Sec. 4.2: the field starts at equilibrium): f := f^eq(rho, u, p/rho)
 * from dense float64 device fields. f has the storage type of `prec`. */
lb_status lb_init(const lb_grid* grid, int32_t prec, const double* rho, const double* ux,
                  const double* uy, const double* p, void* f, void* stream);

/* One time step f_out = S(f_in) at time index `step` (t = step*dt, used by SHOCK
 * edges). f_in and f_out must not overlap. */
lb_status lb_step(const lb_grid* grid, int32_t prec, const void* f_in, void* f_out, int64_t step,
                  void* stream);

/* lb_step with an explicit launch shape (tile NULL = default). Every tile gives
 * bitwise the same result. */
lb_status lb_step_tiled(const lb_grid* grid, int32_t prec, const void* f_in, void* f_out,
                        int64_t step, const lb_tile* tile, void* stream);

/* nsteps ping-pong steps from f_a at time index step0. The result is in f_a when
 * nsteps is even, else in f_b; the other array is left holding an intermediate
 * state (with several steps per pass, not necessarily that of step nsteps-1).
 * With two steps per pass: 0-3 single steps, then an even number of two-step
 * passes; with three: 0-2 single steps, then nsteps / 3 three-step passes; with
 * sixteen: the steps beyond an even number of sixteen-step passes as with two,
 * then those passes.
 * use_graph != 0 captures the launches in a HIP graph (cached: a repeated call with
 * the same arguments replays it). Every launch shape and steps setting gives
 * bitwise the same result. */
lb_status lb_run(const lb_grid* grid, int32_t prec, void* f_a, void* f_b, int64_t step0,
                 int32_t nsteps, int32_t use_graph, const lb_tile* tile, void* stream);

/* Moments of f (Eqs. (e4), (e5), (e7)) into dense float64 device fields (any of
 * rho/ux/uy/T may be NULL), and, if flags != NULL, a device uint32[4]:
 * flags[0] = OR of LB_FLAG_* over all sites, flags[1..3] = number of sites that are
 * non-finite, have rho <= 0, have T <= 0. The flags array is cleared by the call. */
lb_status lb_moments(const lb_grid* grid, int32_t prec, const void* f, double* rho, double* ux,
                     double* uy, double* T, uint32_t* flags, void* stream);

/* Blow-up as a status (Sec. 3: outside its linear-stability range the scheme
 * grows without bound; a finite f^eq needs rho != 0, Eq. (e16) divides by it).
 * flags: the device uint32[4] that lb_moments filled (its work must be on
 * `stream` or finished). Waits for `stream` (synchronous), copies the four words
 * to host_flags (host uint32[4], may be NULL) and returns LB_ENONFINITE when
 * flags[0] has LB_FLAG_NONFINITE or LB_FLAG_RHO_NONPOS (lb_last_error gives the
 * counts), LB_OK otherwise. T <= 0 alone is not an error: f^eq is a polynomial
 * in T. LB_EINVAL for flags == NULL, LB_EHIP if the copy fails. */
lb_status lb_check_flags(const uint32_t* flags, uint32_t* host_flags, void* stream);

/* Domain totals of the collision invariants into a device double[4]: the sums
 * over sites of rho = sum_i f_i (Eq. (e4)), rho ux and rho uy = sum_i f_i v_i
 * (Eq. (e5)) and rho (b T + u^2) = sum_i f_i (v_i^2 + eta_i^2) (Eq. (e7)).
 * Deterministic (fixed reduction order). Uses a per-device workspace allocated
 * on first use (and grown when a larger grid needs more partial sums); calls on
 * different streams are ordered on it (each waits for the previous call's
 * kernels before writing it). */
lb_status lb_invariants(const lb_grid* grid, int32_t prec, const void* f, double* out4,
                        void* stream);

/* lb_invariants for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results (bitwise), with the partial sums in a fixed array of the
 * library instead of a workspace: 4096 records of 4 doubles (128 KiB) per
 * device, set up on the first call on a device and held until the process ends.
 * Calls no hipMalloc, hipFree or other allocating routine. Every call on a
 * device shares that device's array, and the array keeps the last call's
 * partial sums (each call writes every record it reads, so nothing needs
 * clearing): calls that overlap on one device (on different streams or host
 * threads) race on it. LB_EINVAL if the grid needs more than 4096 partial
 * records (the partition never does: it caps the number of row blocks at 4096),
 * and the argument errors of lb_invariants. */
lb_status lb_invariants_noalloc(const lb_grid* grid, int32_t prec, const void* f, double* out4,
                                void* stream);

/* Adjoint (vector-Jacobian product) of lb_step at f_n: g_n = (dS/df)^T g_np1.
 * g_np1 and g_n are float64 arrays of the distribution layout; f_n has the
 * storage type of `prec` (the float32 rounding of the store is treated as the
 * identity). g_np1 and g_n must not overlap. The paper has no adjoint: this is
 * the exact transpose of the step's linearisation (upwinding by the fixed sign
 * of v, no limiter, so the step is smooth in f where rho != 0). */
lb_status lb_step_adjoint(const lb_grid* grid, int32_t prec, const void* f_n, const double* g_np1,
                          double* g_n, int64_t step, void* stream);

/* nsteps steps from f0, keeping every state: out[j] (a host array of nsteps
 * device pointers, each a distribution array of the storage type) receives the
 * state after step step0 + j. Used to recompute a checkpointed segment.
 * Consecutive arrays (f0, out[0]; out[j], out[j+1]) must not overlap
 * (LB_EALIAS). Steps run two per pass, the first step's state stored on the way
 * (bitwise the state of a single step), wherever the pass's input and both of
 * its outputs are distinct arrays below 4 GiB and ny >= 2; elsewhere one step
 * per launch. */
lb_status lb_run_record(const lb_grid* grid, int32_t prec, const void* f0, void* const* out, int64_t step0,
                        int32_t nsteps, void* stream);

/* Reverse sweep over nsteps steps: f[j] (host array of nsteps device pointers) is
 * the state at time index step0 + j; g holds g^{step0+nsteps} on entry. Applies
 * lb_step_adjoint for j = nsteps-1 .. 0, alternating between g and work (both
 * float64 distribution arrays, not overlapping); g^{step0} ends in g when nsteps
 * is even, else in work. */
lb_status lb_adjoint_run(const lb_grid* grid, int32_t prec, const void* const* f, double* g, double* work,
                         int64_t step0, int32_t nsteps, void* stream);

/* Adjoint of lb_init with respect to rho at fixed u and p:
 * g_rho[x] = sum_i g_f0_i(x) d f_i^eq(rho, u, p/rho) / d rho. */
lb_status lb_init_adjoint(const lb_grid* grid, const double* rho, const double* ux,
                          const double* uy, const double* p, const double* g_f0, double* g_rho,
                          void* stream);

/* Batched independent problems (a batch of 1D/2D grids with their own
 * parameters) stored back to back in one packed array. */
typedef struct lb_batch lb_batch;

/* Build a batch from a host array of grids (pitch fields are ignored and
 * recomputed). Uploads per-problem constants and a work list. Errors as
 * lb_validate, LB_EUNSUPPORTED for a SHOCK edge or a problem whose array
 * reaches 4 GiB. */
lb_status lb_batch_create(int32_t nprob, const lb_grid* grids, int32_t prec, lb_batch** out);

/* Element offset of each problem's array inside the packed array (host int64[nprob])
 * and the total element count; each problem p is a normal distribution array with
 * the pitch written to pitches[p] (host int64[nprob], may be NULL). */
lb_status lb_batch_layout(const lb_batch* b, int64_t* offsets, int64_t* pitches, int64_t* total);

/* Set the launch shape of the batched step: block_x threads per work item (a
 * work item covers all rows of a strip of its problem); steps: time steps per
 * pass, 0 = the default, 1, 2, or 4, 6, 8 for a batch whose problems all have 4
 * rows and a periodic y axis (the whole state of a strip then stays on chip for
 * all the steps of a pass, and a strip of 64 lanes produces 64 - 2 * steps
 * columns; in FP32 storage at block_x 64 a strip's four rows run on the four
 * wavefronts of a 256-thread block, one row each, exchanged through LDS);
 * the default for such a batch is 4 steps and width 64 in FP32 and 8 steps in FP64
 * storage (width 256 unless set), else 2 (1
 * when a problem has ny < 2). blocks = 0: one launch per pass (the default). blocks > 0: all
 * two-step passes of a call in ONE launch of at most `blocks` co-resident
 * blocks (fewer if fewer fit on the device at once), each block taking its
 * share of the work items pass after pass and waiting, before
 * each pass of an item, until the items whose columns it reads have finished the
 * previous pass (progress counters with release/acquire atomics); results are
 * bitwise those of the per-pass launches. rows (persistent launch only): polls
 * per wait before a block gives up (0 = the default, 2^20); a block that gives up
 * flags the batch and ends, and so do the others at their next wait, so the launch
 * always terminates, with an incomplete result that lb_batch_status reports. Other
 * work on the device that keeps blocks of the launch from being resident can make
 * it give up. LB_EINVAL for a bad width, steps, or negative blocks or rows, for
 * more than 2 steps on a batch that is not all 4-row y-periodic problems, or for
 * more than 2 steps with blocks > 0 (the persistent launch runs two steps per
 * pass; steps = 0 with blocks > 0 selects that). */
lb_status lb_batch_set_tile(lb_batch* b, const lb_tile* tile);

/* nsteps steps of every problem, all problems per launch, the launches captured
 * once in a HIP graph and replayed as one graph launch. Several time steps per
 * pass over the packed array (as lb_batch_set_tile's steps sets: an even number of
 * passes of that many steps, then two-step passes and single steps for the rest)
 * unless a problem has ny < 2 or lb_batch_set_tile asked for steps = 1; results
 * are bitwise the same either way.
 * Result in f_a when nsteps is even, else f_b. step index starts at 0 on the
 * first call and continues across calls. */
lb_status lb_step_batched(lb_batch* b, void* f_a, void* f_b, int32_t nsteps, void* stream);

/* Status of the persistent launches of a batch since the last call: waits for
 * `stream`, and returns LB_EHIP (and clears the flag) if a block gave up waiting
 * for a neighbouring strip, so that some problems did not advance; LB_OK
 * otherwise. Synchronous. */
lb_status lb_batch_status(lb_batch* b, void* stream);

void lb_batch_destroy(lb_batch* b);

/* Time each candidate launch shape for (grid, prec) with HIP events on `stream`
 * (reps launches each, captured in a HIP graph and timed as one replay when
 * stream != NULL, as lb_run with use_graph runs them), for one step per launch,
 * two and (where they run) three steps per pass, and on 4-row grids with a
 * periodic y axis the sixteen-step pass, and return the fastest per time step in
 * *best (best->steps tells which, 0 for the sixteen-step pass, which lb_run takes
 * by default there; pass it to lb_run as is) and its time per step in *best_ms;
 * f_a/f_b are scratch state. Synchronises `stream`. */
lb_status lb_autotune(const lb_grid* grid, int32_t prec, void* f_a, void* f_b, int32_t reps,
                      lb_tile* best, float* best_ms, void* stream);

/* ------------------------------------------------------------ von Neumann scan
 *
 * Linear stability of the step about a uniform equilibrium, Sec. 3: a Fourier
 * perturbation F exp(i k.x) of the 9 distributions at the equilibrium of
 * (rho, u, T) is multiplied per step by the 9x9 complex matrix
 *     G(k) = diag(s_i(k)) + (1/tau) d f^eq / d f,
 * Eqs. (SEC-VON-8), (SEC-VON-9) with the dissipation term of Eq. (SEC-VON-12)
 * (the "-1" of Eq. (SEC-VON-4) read as -delta_ij; tau general), where s_i(k) is
 * the Fourier symbol of the linear part of the step for plane i: the same
 * stencil coefficients the step kernels use, so the scan analyses exactly the
 * implemented scheme. The scheme is linearly stable at (state, parameters, k)
 * when the spectral radius max_j |omega_j(k)| does not exceed 1. The
 * eigenvalues are computed per (case, k) on the GPU: Householder reduction to
 * Hessenberg form, then single-shift QR with Wilkinson shifts and deflation,
 * in complex double precision. */

/* One scan case: the uniform state and every parameter G depends on. Edges and
 * grid sizes play no part (the analysis is for the periodic, unbounded grid). */
typedef struct {
  double rho, ux, uy, T;    /* equilibrium state, rho > 0, T > 0 (T = p / rho) */
  double c1, c2, eta0, gamma;
  double tau, beta, dt, dx;
  double lambda[9];         /* as in lb_grid: one value per velocity group */
} lb_vn_case;

/* Spectral radius of G(k) for every (case, wave vector). cases: host array of
 * ncases (copied to the device; the call waits for that copy, i.e. it
 * synchronises `stream` once). kdx, kdy: device float64[nk], the wave vector
 * times dx (radians; k.dy = kdy, dy = dx). reduce = 0: out is device
 * float64[ncases * nk], out[c * nk + q] = radius at (case c, k_q); reduce = 1:
 * out is device float64[ncases], the maximum over q. A case whose QR iteration
 * does not converge gives NaN (NaN wins the maximum). Errors: LB_EINVAL for
 * NULL pointers, ncases < 1, nk < 1 or ncases * nk >= 2^31; LB_EPARAM (message
 * names the case) for parameters lb_validate would reject or a state with
 * rho <= 0 or T <= 0. */
lb_status lb_vn_scan(const lb_vn_case* cases, int32_t ncases, const double* kdx, const double* kdy, int32_t nk,
                     int32_t reduce, double* out, void* stream);

/* Largest stable time step per case among candidates: for each case c (its own
 * dt ignored) the largest dts[c * ndt + j] such that every candidate
 * dts[c * ndt + 0 .. j] gives a spectral radius <= 1 + tol over all nk wave
 * vectors; 0 when the first candidate already fails. dts: host
 * float64[ncases * ndt], each case's row ascending and > 0. kdx, kdy as in
 * lb_vn_scan. dt_out: host float64[ncases]. Synchronous (returns after the
 * scan finished); LB_EINVAL for bad candidates or tol < 0. */
lb_status lb_vn_max_stable_dt(const lb_vn_case* cases, int32_t ncases, const double* dts, int32_t ndt,
                              const double* kdx, const double* kdy, int32_t nk, double tol, double* dt_out,
                              void* stream);

/* ABI self-description for bindings: sizeof(lb_grid) (which = 0), sizeof(lb_edge)
 * (1), sizeof(lb_state) (2), sizeof(lb_tile) (3), sizeof(lb_vn_case) (4); -1 for
 * other values. */
int64_t lb_struct_size(int32_t which);

const char* lb_status_str(int32_t status);
const char* lb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBKT_H */
