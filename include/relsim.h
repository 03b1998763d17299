/*
 * relsim.h - C ABI of the MI355X (gfx950) library for the per-particle hot
 * path of the relativistic semi-implicit PIC step (RelSIM, an energy-
 * conserving ECsim-type scheme; Schoeffler et al. 2025, Sec. 2: explicit
 * pusher, implicit field solve, mass-matrix linearised current).
 *
 * The step n -> n+1, with x at half-integer and u = gamma v at integer times:
 *   S1 gather B^n at x^{n+1/2}                  (CIC from cell centres)
 *   S2 gbar = gamma(u^n), b = beta_s B_p/(gbar c), beta_s = q_s dt/(2 m_s),
 *      alpha = (I - [b]x + b b^T)/(1 + b^2)
 *   S3 Jhat_g = V^-1 sum_p w q W_g alpha u/gbar,
 *      M_{g,g'} = V^-1 sum_p (w q beta/gbar) W_g W_g' alpha
 *   S4 [I + (c th dt)^2 C_CN C_NC + 4 pi th dt M] E_th = E^n + c th dt C_CN B^n - 4 pi th dt Jhat
 *   S5 B^{n+1} = B^n - c dt C_NC E_th,  E^{n+1} = (E_th - (1 - th) E^n)/th
 *   S6 E_p = sum_g W_g E_th_g, ubar = alpha (u + beta E_p), u^{n+1} = 2 ubar - u,
 *      x^{n+3/2} = x^{n+1/2} + dt u^{n+1}/gamma(u^{n+1})
 *   S7 W = sum_p w m c^2 (gamma - 1) + V/(8 pi) (sum |E|^2 + sum |B|^2)
 *
 * Conventions
 *   - Gaussian units.  Periodic grid nx x ny (x nz), every extent >= 3.
 *     E, Jhat and M live at nodes (i,j,k)*dx, B at cell centres
 *     (i+1/2, j+1/2, k+1/2)*dx.  Node and cell (i,j,k) share the linear index
 *     i + nx*(j + ny*k); N = nx*ny*nz (nz = 1 in 2D, where d/dz = 0).
 *   - Grid arrays are FP64, component-major: E, B, Jhat [3][N].  M is
 *     summed in FP64 and stored in FP64, or in FP32 when the context was
 *     created with mass_fp32 = 1 (mixed precision only: the per-cell moments
 *     it is summed from are FP32 there, so the FP32 store rounds values that
 *     already carry FP32 rounding, and it halves M's memory and the S4
 *     operator's largest read; the S4 products and sums are FP64 either
 *     way).
 *     M holds the node-pair blocks M_{g,g+delta} for the 9 (2D) or 27 (3D)
 *     offsets delta in {-1,0,1}^dim, numbered o = sum_d (delta_d + 1) 3^d (x
 *     fastest).  The block is symmetric in the pair, M_{g,g'} = M_{g',g}
 *     (one 3x3 block; Sec. 2, the mass matrices are sums of W_g W_g' alpha_p
 *     over the particles), so only the upper half o >= c is stored, c = 4
 *     (2D) or 13 (3D): M is [m_slots][9][N], m_slots = 5 (2D) or 14 (3D).
 *     Entry [h][3r+s][g] couples E_s at node g+delta(c+h) into row r of node
 *     g; the block of offset o < c at node g is slot c - o of node
 *     g+delta(o).  Each 3x3 block is row-major.
 *   - Every array argument is a DEVICE pointer owned by the caller.  The
 *     library allocates no device memory after relsim_init: it carves the
 *     caller's workspace.  Host scalars returned (iters, residuals, energies)
 *     make the call synchronous; all other calls are asynchronous on the
 *     stream given to relsim_init.
 *   - Return value: RELSIM_OK (0) or a negative error code; relsim_strerror
 *     and relsim_last_error give text.  No exception crosses the ABI.  A
 *     context is not thread safe; several contexts may coexist.
 */
#ifndef RELSIM_H
#define RELSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RELSIM_OK 0
#define RELSIM_EINVAL (-1)        /* bad parameter, size or pointer            */
#define RELSIM_ENOTCONVERGED (-2) /* linear solve hit its iteration limit       */
#define RELSIM_EHIP (-3)          /* a HIP runtime call failed (text captured)  */
#define RELSIM_ENONFINITE (-4)    /* NaN/Inf met in a reduction or the solve    */
#define RELSIM_ERANGE (-5)        /* a particle moved more than one cell, or a
                                     bin exceeded 65535 particles              */
#define RELSIM_EINTERNAL (-6)     /* an internal consistency check failed      */

#define RELSIM_FP64 0  /* particle state and particle arithmetic in double    */
#define RELSIM_MIXED 1 /* particle state/arithmetic in float, per-cell moments
                          reduced in float, grid accumulation, solve and
                          energy in double                                   */

typedef struct relsim_ctx relsim_ctx;

typedef struct {
  int32_t dim;                 /* 2 or 3                                          */
  int32_t nx, ny, nz;          /* cells per dimension (nz ignored in 2D), >= 3    */
  double dx, dy, dz;           /* cell sizes                                      */
  double dt, c, theta;         /* time step, speed of light, time centring of E   */
  int32_t precision;           /* RELSIM_FP64 or RELSIM_MIXED                     */
  int32_t nspecies;            /* 1..8                                            */
  double q[8], m[8];           /* charge and mass per species                    */
  int64_t max_particles;       /* capacity of every particle array (< 2^31)       */
  double gmres_rtol;           /* stop when ||r - A E_th|| <= rtol ||r||          */
  int32_t gmres_restart;       /* Krylov dimension (1..64)                        */
  int32_t gmres_maxit;         /* total Arnoldi steps allowed                     */
  int32_t nonrelativistic;     /* 1: gamma == 1, kinetic energy m|u|^2/2          */
  int32_t group;               /* lanes per cell in the 2D deposit and the
                                  kinetic-energy kernel: 0 = choose from the
                                  mean occupancy, else 4, 8, 16, 32 or 64 (the
                                  3D deposit always splits a cell's moments
                                  over 4 lanes; the push passes size their
                                  row segments themselves)                      */
  int32_t mass_fp32;           /* 0: M stored in double (the default); 1 (only
                                  with RELSIM_MIXED): M stored in float, see
                                  Conventions                                   */
} relsim_params;

/* Particle state, sorted by bin = cell * nspecies + s, so that the
 * particles of (cell, species) occupy [bin_start[bin], bin_start[bin+1]).
 * Element type T is double for RELSIM_FP64 and float for RELSIM_MIXED.  In
 * 2D the record of particle p is split over two packed arrays: xy[p] =
 * (off_x, off_y) (2 T, aligned to 2 T) and uw[p] = (u_x, u_y, u_z, w) (4 T,
 * aligned to 4 T).  In 3D it is one block of 8 T at xy, (off_x, off_y, off_z,
 * 0, u_x, u_y, u_z, w), aligned to 8 T (one 32-byte memory sector in FP32);
 * uw and z are not used and may be NULL.  off in [0,1) is the position inside
 * the cell in units of the cell size; u = gamma v; w = number of physical
 * particles represented.  Each array exists twice ("front" and "back"); the
 * re-sort writes into the back set and then swaps the two sets (and the two
 * bin_start arrays) inside this struct. */
typedef struct {
  int64_t n;                   /* particles in use                                */
  int32_t *bin_start;          /* [ncells*nspecies + 1]                           */
  int32_t *cell;               /* [capacity] linear cell index: input of
                                  relsim_sort, written by relsim_sort and
                                  relsim_fill_cells; relsim_push leaves it
                                  stale (the bins already say where each
                                  particle is, and the re-sort saves the
                                  4-byte write per particle)                    */
  void *xy;                    /* [capacity][2] T (2D), [capacity][8] T (3D)      */
  void *uw;                    /* [capacity][4] T (2D; unused in 3D)              */
  void *z;                     /* unused (NULL)                                   */
  int32_t *bin_start_back;
  int32_t *cell_back;
  void *xy_back;
  void *uw_back;
  void *z_back;
  const uint8_t *species;      /* [n] species id, read only by relsim_sort        */
} relsim_particles;

/* Bytes of device workspace relsim_init needs for these parameters. */
size_t relsim_workspace_bytes(const relsim_params *p);

/* Validate parameters and create a context bound to the current HIP device
 * and to `hip_stream` (a hipStream_t; NULL = default stream).  `workspace`
 * must be a device buffer of at least relsim_workspace_bytes(p) bytes that
 * stays valid, and unused by the caller, until relsim_finalize.  Allocates a
 * small pinned host buffer and timing events; no device memory. */
int relsim_init(const relsim_params *p, void *hip_stream, void *workspace, size_t workspace_bytes,
                relsim_ctx **out);
void relsim_finalize(relsim_ctx *ctx);

/* a1 (general form): stable sort of arbitrary particles by bin.  Reads
 * part->cell and part->species for the front set, writes the sorted state to
 * the back set and swaps.  bin_start is rebuilt. */
int relsim_sort(relsim_ctx *ctx, relsim_particles *part);

/* a2-a4 (S1-S3): gather B^n, form alpha per particle and deposit Jhat [3][N]
 * and M [m_slots][9][N] (the stored half of the node-pair blocks, see
 * Conventions; both overwritten; Jhat FP64, M in its storage type and aligned
 * to it).
 * Particles must be bin-sorted. */
int relsim_deposit_moments(relsim_ctx *ctx, const relsim_particles *part, const double *B_n, double *Jhat,
                           void *M);

/* a5 (S4-S5): restarted GMRES for E_th from the initial guess E^n, then the
 * field update.  E_theta, E_np1, B_np1 are written.  iters / rel_resid (host
 * pointers, may be NULL) receive the Arnoldi steps taken and the final true
 * relative residual.  Synchronous (one small device-to-host copy per Arnoldi
 * step).  Returns RELSIM_ENOTCONVERGED with the last iterate written when
 * gmres_maxit is reached. */
int relsim_field_solve(relsim_ctx *ctx, const void *M, const double *Jhat, const double *E_n, const double *B_n,
                       double *E_theta, double *E_np1, double *B_np1, int32_t *iters, double *rel_resid);

/* a5 (S4-S5) from a caller's initial guess: as relsim_field_solve, with
 * the GMRES started from the values E_theta holds on entry (device, [3][N],
 * finite) instead of E^n.  For the passes of a fixed-point iteration whose
 * systems change little from one pass to the next (the energy-conserving
 * variant below): started from the previous pass's E_th, GMRES needs fewer
 * Arnoldi steps to the same relative tolerance.  The stopping rule and
 * everything else are relsim_field_solve's. */
int relsim_field_solve_guess(relsim_ctx *ctx, const void *M, const double *Jhat, const double *E_n,
                             const double *B_n, double *E_theta, double *E_np1, double *B_np1, int32_t *iters,
                             double *rel_resid);

/* a6 (S6, +a1 when resort != 0): push every particle with E_th and B^n and
 * move it across at most one cell face per dimension (periodic).  With
 * resort, the pushed state is written into the back set in the new bin
 * order (a stable counting sort over the neighbour moves: a first pass
 * reads the particles and counts the moves, a second pushes them again and
 * writes each one to its new place) and the sets are swapped, so that the
 * back set then holds the state before the push.  With resort == 0 the
 * particles are pushed in place and stay in their old bins; their offsets,
 * still relative to the old cell, may lie in [-1, 2), and the state is then
 * only good for reading out.  new_index (device, [n], may be NULL; used only
 * with resort) receives, for every particle in the old order, its position
 * in the new order.  A particle that moves more than one cell is reported as
 * RELSIM_ERANGE by the next synchronous call (the state is then
 * undefined). */
int relsim_push(relsim_ctx *ctx, relsim_particles *part, const double *E_theta, const double *B_n, int32_t resort,
                int32_t *new_index);

/* Energy-conserving relativistic variant.  The methods paragraph of Sec. 2
 * says the scheme conserves energy exactly only without relativity; with the
 * Lorentz factor of S2-S3 and S6 taken as gbar = (gamma(u^n) +
 * gamma(u^{n+1}))/2 the work done on each particle equals its kinetic energy
 * change, and the step conserves energy exactly, but gbar then depends on the
 * step's own result.  A caller finds it by fixed-point iteration:
 *   gbar = NULL (gamma(u^n));
 *   repeat: relsim_deposit_moments_ec(gbar) -> relsim_field_solve (after
 *           the first pass: relsim_field_solve_guess from the last E_th) ->
 *           relsim_gamma_mean(gbar -> gbar_next, change); swap gbar, gbar_next
 *   until change is small; then relsim_push_ec with the gbar the last
 *   relsim_gamma_mean was given (the one the field solve used).
 * gbar / gbar_next: device arrays of part->n elements of the particle type T
 * (double for RELSIM_FP64, float for RELSIM_MIXED, aligned to it), one per
 * particle in the current (front) order, owned by the caller.  A NULL gbar
 * means gamma(u^n), which makes the first two calls the standard ones.  In the
 * non-relativistic limit gbar is ignored (gamma = 1). */

/* Optional acceleration of that fixed point (the plain update above is the
 * default): after relsim_gamma_mean(gbar -> gbar_next), with each particle's
 * residual r = gbar_next - gbar of this pass and of the last (kept in g_prev,
 * r_prev), gbar_next[p] becomes gbar - r (gbar - g_prev) / (r - r_prev), the
 * root of the line through the particle's last two residuals, where that
 * line falls with a slope in [-10, -0.1] and the step is measurable (|gbar -
 * g_prev| > 1e-12 gbar); elsewhere it stays the plain update.  The result is
 * kept >= 1 (a NaN passes through).  Each particle's gbar is nearly its own
 * scalar fixed point, which the field couples only weakly, so a secant per
 * particle follows each one's contraction rate.  The fixed point, the
 * stopping test and the final relsim_push_ec are unchanged.
 * gbar, gbar_next: n elements of the particle type T (as relsim_gamma_mean);
 * g_prev, r_prev: device arrays of n elements of T owned by the caller,
 * written on every call; first != 0 (a step's first pass) only records them.
 * The step is formed in FP64; g_prev holds gbar itself (exact in T), r_prev
 * the residual rounded to T (exact in FP32 too while gbar_next lies within a
 * factor 2 of gbar, by Sterbenz's lemma).
 * n <= max_particles.  Asynchronous. */
int relsim_gamma_secant(relsim_ctx *ctx, int64_t n, const void *gbar, void *gbar_next, void *g_prev, void *r_prev,
                        int first);

/* relsim_deposit_moments with gbar in place of gamma(u^n). */
int relsim_deposit_moments_ec(relsim_ctx *ctx, const relsim_particles *part, const double *B_n, const void *gbar,
                              double *Jhat, void *M);

/* One fixed-point pass: pushes every particle as relsim_push would with
 * gbar (state untouched), writes gbar_next[p] = (gamma(u^n_p) +
 * gamma(u^{n+1}_p))/2, and stores in *max_rel_change (host) the largest
 * |gbar_next - gbar| / gbar over the particles (infinity if any is not
 * finite).  gbar_next must not alias gbar.  Synchronous (one 8-byte copy). */
int relsim_gamma_mean(relsim_ctx *ctx, const relsim_particles *part, const double *E_theta, const double *B_n,
                      const void *gbar, void *gbar_next, double *max_rel_change);

/* relsim_push with gbar in place of gamma(u^n). */
int relsim_push_ec(relsim_ctx *ctx, relsim_particles *part, const double *E_theta, const double *B_n,
                   const void *gbar, int32_t resort, int32_t *new_index);

/* Particles that the re-sort's second pass placed on a face of the cell the
 * first pass counted them in, because the recomputed offset came out within
 * rounding (1e-4 cell) outside that cell, summed over every relsim_push and
 * relsim_push_ec with resort since the last call; *count receives the sum
 * and the counter restarts at zero.  Both passes evaluate one function with
 * the same operands, so the count is expected to stay 0 (a difference
 * larger than rounding is reported as RELSIM_EINTERNAL instead).
 * Synchronous. */
int relsim_placement_clamps(relsim_ctx *ctx, int64_t *count);

/* Write part->cell (front set) from bin_start: particle p of bin b gets cell
 * b / nspecies.  Needed after relsim_push before anything reads the cell
 * ids (the adjoint entry points read state_n->cell). */
int relsim_fill_cells(relsim_ctx *ctx, relsim_particles *part);

/* a7 (S7): out[0..3] = kinetic, electric, magnetic, total energy (host
 * array), accumulated in FP64 in both precisions.  Synchronous. */
int relsim_energy(relsim_ctx *ctx, const relsim_particles *part, const double *E, const double *B, double out[4]);

/* a7 fused into a6: the S7 energy of the particle state written by the
 * last relsim_push or relsim_push_ec with resort on this context, whose
 * second pass summed each pushed particle's FP64 kinetic term per wave (in
 * a fixed order, so the result is deterministic; it equals relsim_energy's
 * to rounding order), plus the field energies of E and B as in
 * relsim_energy.  No pass over the particles.  The caller must not have
 * changed the particle arrays since that push.  RELSIM_EINVAL if no push
 * with resort happened since the context was made or since relsim_sort or
 * a relsim_push without resort.  Synchronous. */
int relsim_energy_pushed(relsim_ctx *ctx, const double *E, const double *B, double out[4]);

/* relsim_energy for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * No context and no workspace: the reduction partials live in a file-scope
 * device array of this library (4 MiB, one copy per device, held until the
 * process ends; its device address is looked up once per device on the first
 * call there).  p: the parameters a context would be created with (validated
 * as relsim_init does); hip_stream: the stream to enqueue on (NULL = default
 * stream); part: bin-sorted particles (front set); E, B: FP64 [3][N] device
 * arrays; out: device array of 4 doubles that receives kinetic, electric,
 * magnetic and total energy, the same values relsim_energy returns for the
 * same inputs, bit for bit.  Asynchronous (no host copy, no synchronisation,
 * no allocation): non-finite values are not reported, and the deferred
 * range flags of a context's push are not checked.  Returns RELSIM_EINVAL
 * for bad parameters or pointers and RELSIM_ERANGE when the grid needs more
 * kinetic partials (one per 64/group cells) than the scratch holds (about
 * 520,000: 4.2M cells at 8 lanes per cell).  Calls that overlap on one
 * device (other streams, other threads) share the array and race. */
int relsim_energy_noalloc(const relsim_params *p, void *hip_stream, const relsim_particles *part, const double *E,
                          const double *B, double *out);

/* Field operators, exposed for tests and for the adjoint (all FP64 [3][N]).
 * out = C_NC in (nodes -> centres), C_CN in (centres -> nodes), or the S4
 * operator A applied to x. */
int relsim_curl_nc(relsim_ctx *ctx, const double *in, double *out);
int relsim_curl_cn(relsim_ctx *ctx, const double *in, double *out);
int relsim_apply_A(relsim_ctx *ctx, const void *M, const double *x, double *out);

/* out = A^T x, the transposed S4 operator (each block of M transposed; the
 * curl-curl term is symmetric). */
int relsim_apply_AT(relsim_ctx *ctx, const void *M, const double *x, double *out);

/* a8: reverse-mode adjoint of one step, RELSIM_FP64 contexts only.  All
 * cotangent arrays are FP64 device arrays: particle ones [dim][n] for
 * positions (per unit of physical length) and [3][n] for momenta, in the
 * particle order of `state_n`; grid ones [3][N].  The step is
 *   (x^{n+1/2}, u^n, E^n, B^n) -> (x^{n+3/2}, u^{n+1}, E^{n+1}, B^{n+1}).
 * Call order for one step backwards: relsim_push_adjoint, then
 * relsim_field_solve_adjoint, then relsim_deposit_adjoint, with the grid
 * accumulators zeroed by the caller first.
 *
 * relsim_push_adjoint (adjoint of S1, S2, S6): state_n is the particle state
 * before the push (bin-sorted, with its cell ids written, e.g. by
 * relsim_fill_cells); new_index maps it to the
 * order of lam_x_in / lam_u_in (the cotangents of x^{n+3/2}, u^{n+1}; NULL =
 * same order).  Writes lam_x_out, lam_u_out (cotangents of x^{n+1/2}, u^n
 * through the push) and ADDS into lam_E_theta and lam_B_n. */
int relsim_push_adjoint(relsim_ctx *ctx, const relsim_particles *state_n, const double *E_theta, const double *B_n,
                        const int32_t *new_index, const double *lam_x_in, const double *lam_u_in, double *lam_x_out,
                        double *lam_u_out, double *lam_E_theta, double *lam_B_n);

/* relsim_field_solve_adjoint (adjoint of S4, S5): given lam_E_theta (from the
 * push adjoint) and the cotangents of E^{n+1}, B^{n+1}, solves
 * A^T mu = lam_E_theta + lam_E_np1/theta - c dt C_NC^T lam_B_np1 by GMRES
 * (same tolerance as the forward solve, initial guess 0), writes mu, and ADDS
 * -(1-theta)/theta lam_E_np1 + mu into lam_E_n and lam_B_np1 +
 * c theta dt C_CN^T mu into lam_B_n.  M is the step's mass matrix.
 * Synchronous; RELSIM_ENOTCONVERGED as for relsim_field_solve. */
int relsim_field_solve_adjoint(relsim_ctx *ctx, const void *M, const double *lam_E_theta, const double *lam_E_np1,
                               const double *lam_B_np1, double *mu, double *lam_E_n, double *lam_B_n, int32_t *iters,
                               double *rel_resid);

/* relsim_deposit_adjoint (adjoint of S1-S3 through J-bar = Jhat + M E_th):
 * with mu from relsim_field_solve_adjoint, ADDS the particle cotangents into
 * lam_x, lam_u and the field cotangent into lam_B_n. */
int relsim_deposit_adjoint(relsim_ctx *ctx, const relsim_particles *state_n, const double *B_n, const double *E_theta,
                           const double *mu, double *lam_x, double *lam_u, double *lam_B_n);

/* Per-kernel timing with HIP events on the context's stream.  When enabled,
 * every kernel launch is bracketed by events; relsim_timing_read
 * synchronises and returns, per kernel name, the summed milliseconds and the
 * launch count (up to `cap` entries, names copied into `names` as
 * NUL-terminated strings of at most 47 characters).  Returns the number of
 * entries or a negative error. */
int relsim_timing_enable(relsim_ctx *ctx, int32_t on);
int relsim_timing_reset(relsim_ctx *ctx);
int relsim_timing_read(relsim_ctx *ctx, int32_t cap, char (*names)[48], double *ms, int64_t *count);

const char *relsim_strerror(int code);
const char *relsim_last_error(const relsim_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RELSIM_H */
