/*
 * lion.h -- C ABI of the MI355X trapped-ion engine.
 *
 * One call per step of the problem as the paper states it ("Overview": create
 * the ions with their masses and charges, add a linear Paul trap with the full
 * fields of eq. (field), add laser cooling, then evolve N steps with a fixed
 * time step; "Implementation details": SI units, unscreened Coulomb pair
 * interaction summed over all pairs, Newtonian (velocity-Verlet) integration).
 *
 * Physics computed by every step (all ions i of one trap, t in seconds):
 *   E_c,i  = k_e sum_{j != i} Q_j (r_i - r_j) / |r_i - r_j|^3       (no cutoff)
 *   E_ext  = (V0/R0^2) cos(Omega t) (x, -y, 0) + (kappa U0/Z0^2) (x, y, -2z)
 *            (the dc term is taken as axially confining, the sign for which
 *            eq. (Mathieuaq) holds)
 *   a_i    = (Q_i/M_i) (E_c,i + E_ext(r_i, t))
 *   step   v <- f v; v <- v + (dt/2) a; x <- x + dt v; a <- a(x, t_{k+1});
 *          v <- v + (dt/2) a; v <- f v;   f = exp(-gamma dt/2),
 *          t_k = t_call_start + k dt within one lion_step call.
 * Exactly coincident ions exert no force on each other.
 *
 * Conventions
 *   - SI units throughout: m, m/s, kg, C, V, rad/s, s.
 *   - Host arrays (double, length n_total, trap order for batches) are read or
 *     written during the call only and stay owned by the caller.
 *   - Device memory: the caller allocates one workspace of
 *     lion_workspace_bytes(...) bytes (256-byte aligned) and keeps it alive
 *     until lion_destroy; the library carves all device arrays from it and
 *     never allocates or frees device memory itself (lion_normal_modes takes
 *     a second caller-owned workspace for its eigen-solver).  The HIP runtime
 *     allocates what it needs to instantiate launch graphs.
 *   - Every call runs on the HIP stream given at creation (a hipStream_t
 *     passed as void*, NULL = the default stream) and returns once its work is
 *     queued, except lion_get_state / lion_compute_accel / lion_get_energy,
 *     which synchronise the stream before returning host data.
 *   - A handle is not thread-safe; calls on one handle must not overlap.
 *   - Every call returns LION_OK or a negative status; lion_last_error gives a
 *     message for the last failure on that handle.
 */
#ifndef LION_H
#define LION_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lion_sim lion_sim;

/* Arithmetic of the pair sum.  Positions, velocities, the trap field, the rf
 * phase and the Verlet update are FP64 in every mode.
 *   LION_FP64          pair differences, r^-3 and accumulation in FP64
 *   LION_MIXED_F64ACC  pair arithmetic in FP32 on float-float positions,
 *                      accumulated in FP32 over short runs of sources and
 *                      flushed into FP64 sums (each workgroup's FP64 sum per
 *                      source slice or tile pair is rounded once to FP32 when
 *                      stored; the slices are added in FP64)
 *   LION_MIXED_KAHAN   pair arithmetic in FP32, compensated (Kahan) FP32 sums */
enum lion_precision { LION_FP64 = 0, LION_MIXED_F64ACC = 1, LION_MIXED_KAHAN = 2 };

enum lion_status {
    LION_OK = 0,
    LION_ERR_ARG = -1,         /* invalid argument (message says which)          */
    LION_ERR_STATE = -2,       /* call out of order, e.g. step before set_state  */
    LION_ERR_HIP = -3,         /* a HIP runtime call failed                       */
    LION_ERR_WORKSPACE = -4,   /* workspace missing, too small or misaligned     */
    LION_ERR_NONFINITE = -5,   /* non-finite state detected                      */
    LION_ERR_UNSUPPORTED = -6  /* option not available for this handle           */
};

/* Bytes of device workspace needed for n_total ions in n_traps traps (1 for a
 * single trap) at the given precision.  Returns 0 for invalid arguments.
 * Host-only; the workspace holds every per-ion array of the handle (section
 * "Creating the simulation": one object holds all the simulation's state). */
size_t lion_workspace_bytes(int64_t n_total, int32_t n_traps, int precision);

/* One trap of n ions (n >= 1) with masses (kg, > 0, finite) and charges (C,
 * finite) (section "Adding ions": each ion is defined by its charge and mass;
 * here both are per ion and in SI units, where the paper gives charge in units
 * of e and mass in atomic mass units).  masses_kg and charges_C are host
 * arrays of length n, copied during the call.  dev_workspace: caller-owned
 * device memory of at least lion_workspace_bytes(n, 1, precision) bytes,
 * 256-byte aligned, alive until lion_destroy.  hip_stream: the hipStream_t
 * every call of this handle runs on (NULL: the default stream).  Ions are
 * created with zero position and velocity; call lion_set_state before
 * stepping.  No trap field and no damping until set.  On failure *out is NULL
 * and lion_last_error(NULL) says why: LION_ERR_ARG (n < 1, a mass not finite
 * and > 0, a charge not finite, unknown precision), LION_ERR_WORKSPACE
 * (missing, misaligned or too small), LION_ERR_HIP. */
int lion_create(lion_sim **out, int64_t n, const double *masses_kg, const double *charges_C,
                int precision, void *dev_workspace, size_t ws_bytes, void *hip_stream);

/* n_traps independent traps (1 <= n_traps, 1 <= n_per_trap[k] <= 1024); trap k
 * owns the n_per_trap[k] ions that follow those of trap k-1 in every array.
 * No force acts between traps; each trap has its own field, damping, time step
 * and clock.  All traps of a batch run in one persistent launch per chunk. */
int lion_create_batch(lion_sim **out, int32_t n_traps, const int64_t *n_per_trap,
                      const double *masses_kg, const double *charges_C, int precision,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream);

/* Positions (m) and velocities (m/s) of all ions and the current time t (s; for
 * a batch every trap's clock is set to t) (section "Adding ions": ions placed
 * at given coordinates, placeAtoms; the velocities are the initial condition
 * of the equations of motion of section "Dynamics of trapped ions").  Six host
 * arrays of length n_total, copied during the call.  Computes the
 * accelerations at (x, t) with the kernels that step the handle.  Non-finite
 * input or a NULL array -> LION_ERR_ARG.  Synchronises. */
int lion_set_state(lion_sim *sim, const double *x, const double *y, const double *z,
                   const double *vx, const double *vy, const double *vz, double t);

/* Linear Paul trap of eq. (field) for trap `trap` (-1 = every trap): rf
 * amplitude V_rf (V) at angular frequency Omega (rad/s), end-cap voltage U_dc
 * (V), lengths r0, z0 (m, > 0), geometry factor kappa.  Recomputes the cached
 * accelerations at the current positions and time.  Omega <= 0 with V_rf != 0,
 * r0 or z0 <= 0, or any non-finite value -> LION_ERR_ARG. */
int lion_set_trap(lion_sim *sim, int32_t trap, double V_rf, double Omega_rad_s, double U_dc,
                  double r0, double z0, double kappa);

/* Rigid bodies as an exclusion mask (section "Charged rigid body": ions of a
 * group are bound together, so their mutual Coulomb forces are internal to the
 * body).  body_id[i] >= 0 names the body of ion i, -1 marks a free ion; pairs
 * of ions with the same body id are left out of the pair sum.  NULL (or all
 * -1) clears the mask.  Ions keep per-ion integration (lion_set_rigid_bodies
 * adds rigid integration); energies still count every pair.  Fastest when each
 * body's ions are consecutive in index order.  Single-trap handles only.  In
 * the pair-once kernels (lion_kernel_config.symmetric = 2) a pair of 256-ion
 * tiles (ions 256 t .. 256 t + 255) that both hold ions of one body only is
 * skipped; tile pairs whose body ids may meet compare body ids per pair.
 * Batched handles -> LION_ERR_UNSUPPORTED; ids < -1 -> LION_ERR_ARG.
 * Recomputes the cached accelerations. */
int lion_set_bodies(lion_sim *sim, const int32_t *body_id);

/* Laser cooling (section "Cooling the motion of ions") as an isotropic viscous
 * force -M gamma v on every ion of trap `trap` (-1 = every trap); gamma in 1/s,
 * >= 0 and finite.  Applied as exact exp(-gamma dt/2) velocity scalings. */
int lion_set_damping(lion_sim *sim, int32_t trap, double gamma_per_s);

/* Rigid bodies (section "Charged rigid body", and the rigid integrator of
 * section "Integration"): ions with equal body_id >= 0 keep their relative
 * positions and move as one body under the summed force and torque of their
 * ions; -1 marks a free ion.  Pairs inside a body are left out of the field
 * (as lion_set_bodies).  Set-up uses the current state: body mass, centre of
 * mass R, COM velocity V, angular momentum L about R, and the principal axes of
 * the inertia tensor as the body frame (moments below 1e-10 of the largest
 * count as zero, e.g. along a rod); member velocities are replaced by the rigid
 * motion V + w x (r - R), w = I^-1 L.  Each step: V, L damped by
 * exp(-gamma dt/2) and half-kicked (F/M, torque); R drifts; the orientation
 * quaternion advances with L held fixed by Richardson extrapolation of
 * normalised Euler steps of dq/dt = (1/2)(0, w) q (one of dt, two of dt/2);
 * members are placed; forces; half kick and damping again.  Beams and baths
 * act on free ions only.  lion_set_state re-runs the set-up from the new
 * state.  body_id NULL turns rigid bodies and the exclusion off.  Batched
 * handles -> LION_ERR_UNSUPPORTED; state not set -> LION_ERR_STATE; ids < -1 ->
 * LION_ERR_ARG. */
int lion_set_rigid_bodies(lion_sim *sim, const int32_t *body_id);

/* Body state, bodies in ascending body-id order: *nbodies, and (each output
 * optional, NULL to skip) com [3 nb], com_velocity [3 nb], angular_momentum
 * [3 nb] (about the COM, space frame) and quaternion [4 nb] (w, x, y, z; body
 * frame = principal axes, ascending moments). */
int lion_get_rigid_state(lion_sim *sim, int32_t *nbodies, double *com, double *com_velocity,
                         double *angular_momentum, double *quaternion);

/* Species labels (>= 0) used to select ions for beams and baths; NULL sets
 * every ion to species 0 (the default).  Negative labels -> LION_ERR_ARG. */
int lion_set_species(lion_sim *sim, const int32_t *species);

/* Single-beam laser cooling (section "Cooling the motion of ions": a viscous
 * force along the beam direction only, on one species).  Beam `beam` (0..3)
 * acts on ions of species `species` (-1: every species) with force
 * -M gamma (k.v) k, k = (kx, ky, kz) normalised here; each velocity half-step
 * applies it exactly: v <- v - (1 - exp(-gamma dt/2)) (k.v) k.  gamma = 0
 * turns the beam off.  Applies to every trap of the handle.  Non-finite input,
 * gamma < 0 or a zero direction with gamma > 0 -> LION_ERR_ARG. */
int lion_set_beam(lion_sim *sim, int32_t beam, int32_t species, double kx, double ky,
                  double kz, double gamma_per_s);

/* Langevin bath (section "Cooling the motion of ions": damping plus random kicks
 * that thermalise the ions at temperature T with 1/e velocity-relaxation time
 * tau).  Bath `bath` (0..3) acts on ions of species `species` (-1: every
 * species); each velocity half-step applies the exact Ornstein-Uhlenbeck update
 * v <- c v + sqrt(k_B T / M (1 - c^2)) xi, c = exp(-dt / (2 tau)), with xi
 * three standard normals from Philox4x32-10 (Salmon et al. 2011) keyed by
 * `seed`, counter (ion index, run-wide step number, bath << 8 | half-step),
 * Box-Muller of the four output words.  tau = 0 turns the bath off.  Order in a
 * half-step: isotropic damping, beams 0..3, baths 0..3.  Applies to every trap
 * of the handle (lion_step_batch with unequal dt -> LION_ERR_UNSUPPORTED). */
int lion_set_bath(lion_sim *sim, int32_t bath, int32_t species, double temperature_K,
                  double damping_time_s, uint64_t seed);

/* Run-wide step count that numbers the bath draws (steps completed so far; it
 * grows by nsteps in every lion_step).  Set it when resuming a run so that the
 * bath draws continue the same sequence.  steps_done < 0 -> LION_ERR_ARG. */
int lion_set_step_index(lion_sim *sim, int64_t steps_done);
int64_t lion_get_step_index(const lion_sim *sim);

/* Time average of the ion velocities (section "Writing/reading data": timeAvg,
 * a per-ion average over a duration such as one rf period, written once per
 * duration).  window_steps >= 1 starts averaging at the current run-wide step
 * count S0 (see lion_get_step_index): window k covers steps S0 + (k-1) W + 1 ..
 * S0 + k W, each contributing the velocity at the end of that step, and the
 * average of a window is the plain mean of its W samples.  0 turns it off.
 * Each call clears the sums and the last average.  Later changes of the step
 * index do not move S0: call this again after lion_set_step_index.
 * window_steps < 0 -> LION_ERR_ARG. */
int lion_set_time_average(lion_sim *sim, int32_t window_steps);

/* Average velocities [n] of the last completed window and the run-wide step at
 * which it closed.  Averaging off, or no window completed yet ->
 * LION_ERR_STATE; NULL outputs -> LION_ERR_ARG. */
int lion_get_time_average(lion_sim *sim, double *vx, double *vy, double *vz,
                          int64_t *window_end_step);

/* Pseudopotential trap (section "Electric fields and confinement": the
 * linearPseudoPT trap; eq. (pseudopot) with the Mathieu coefficients of
 * eq. (Mathieuaq)).  Same parameters as lion_set_trap; the rf is replaced by
 * the static radial field -(Q/M) (V_rf/r0^2)^2 / (2 Omega^2) (x, y, 0), so each
 * ion feels the secular frequency of its own Q/M (one trap serves every
 * species).  The dc field is unchanged.  lion_get_energy's trap energy then
 * includes the radial potential (1/2) Q (Q/M) (V_rf/r0^2)^2/(2 Omega^2)(x^2+y^2).
 * lion_set_trap switches back to the full field.  Errors as lion_set_trap. */
int lion_set_pseudo_trap(lion_sim *sim, int32_t trap, double V_rf, double Omega_rad_s,
                         double U_dc, double r0, double z0, double kappa);

/* Energy minimisation (section "Minimisation": damped dynamics that extract
 * energy and cap each ion's move per step).  With F_i = M_i a_i at the current
 * positions, each iteration: stop if max_i |F_i| <= ftol_N (or max_iter
 * iterations were done); keep only the component of the 3N velocity along the
 * 3N force (v <- (v.F / F.F) F if v.F > 0, else 0); v <- v + dt a; scale any
 * ion's velocity so that dt |v_i| <= dmax_m; x <- x + dt v; forces at the new
 * positions.  Starts from the current velocities and leaves the minimiser's
 * velocities in the state; the trap clock does not advance.  The trap must be
 * time independent (pseudopotential trap, or V_rf = 0) -> else
 * LION_ERR_UNSUPPORTED, as are batched handles and rigid bodies.  State not
 * set -> LION_ERR_STATE; dt, dmax <= 0, ftol < 0, max_iter < 0 or non-finite
 * -> LION_ERR_ARG.  *iterations (optional) gets the iterations that moved the
 * ions, *fmax_N (optional) the largest |F_i| at the final positions. */
int lion_minimize(lion_sim *sim, double dt, double dmax_m, double ftol_N, int64_t max_iter,
                  int64_t *iterations, double *fmax_N);

/* Device bytes lion_normal_modes needs for this handle's n ions: the (3n)^2
 * Hessian, two vectors of 3n, a status word and the scratch of rocSOLVER's
 * dsyevd for a 3n x 3n problem.  The scratch size is asked of rocSOLVER in
 * rocBLAS's size-query mode (nothing runs on the GPU and no device memory is
 * allocated); the call creates the handle's rocBLAS handle on first use (kept
 * until lion_destroy).  0 on failure (message in lion_last_error). */
size_t lion_normal_modes_workspace_bytes(lion_sim *sim);

/* Normal modes at the current positions (section "Normal modes of motion":
 * mode frequencies are the eigenvalues of the Hessian of eq. (fullPotential)).
 * A HIP kernel builds the mass-weighted Hessian D = H / sqrt(M_i M_j) of the
 * Coulomb pairs plus the static trap (pseudopotential and dc curvatures) in
 * FP64, in dev_work (caller-owned device memory, 256-byte aligned, at least
 * lion_normal_modes_workspace_bytes(sim) bytes); rocSOLVER's dsyevd
 * diagonalises it on the GPU, with its scratch memory taken from the tail of
 * dev_work (rocblas_set_workspace: rocBLAS allocates nothing for it).  Outputs
 * (host): omega2 [3n] squared angular frequencies, ascending (rad^2/s^2); modes
 * [3n * 3n] or NULL: column k (stride 3n, column-major) is the mass-weighted
 * eigenvector of omega2[k], component 3i + axis.  A minimum of the potential
 * (lion_minimize) gives omega2 >= 0.  Time-dependent trap, batched handle or
 * rigid bodies -> LION_ERR_UNSUPPORTED; workspace too small or misaligned ->
 * LION_ERR_WORKSPACE; solver failure -> LION_ERR_HIP.  Synchronises. */
int lion_normal_modes(lion_sim *sim, void *dev_work, size_t bytes, double *omega2,
                      double *modes);

/* Advance every trap by nsteps (>= 0) steps of size dt (s, > 0, finite)
 * (section "Time evolution": evolve(N) integrates the Newtonian equations of
 * motion for N steps of the set time step; section "Integration": velocity
 * Verlet; the step is written out at the top of this header).  nsteps = 0 is
 * a no-op.  Time afterwards: t + nsteps dt; within the call
 * t_k = t_call_start + k dt.  Runs as captured launch graphs of
 * lion_kernel_config.chunk_steps steps; returns once they are queued.
 * Requires lion_set_state first (else LION_ERR_STATE); nsteps < 0 or a bad
 * dt -> LION_ERR_ARG. */
int lion_step(lion_sim *sim, int64_t nsteps, double dt);

/* As lion_step with a per-trap time step dt[k] (batches only). */
int lion_step_batch(lion_sim *sim, int64_t nsteps, const double *dt_per_trap);

/* Capture and instantiate the launch graphs that a following lion_step (or
 * lion_step_batch) of nsteps steps replays, without running anything: no
 * state, clock or step index changes.  For callers that keep graph
 * instantiation out of a timed or latency-critical region.  The graphs hold
 * the current launch shape and cooling switches; a later change of either
 * drops them (they are then captured again on use).  nsteps < 0 ->
 * LION_ERR_ARG; nsteps = 0 or plain launches (use_graph = 2) do nothing. */
int lion_prepare_step(lion_sim *sim, int64_t nsteps);

/* Copy the state to host arrays of length n_total (any pointer may be NULL to
 * skip it); *t receives the time (trap 0's clock for a batch) (section
 * "Writing/reading data": the per-ion coordinates x, y, z and velocities vx,
 * vy, vz that dump writes, in ion index order).  Synchronises. */
int lion_get_state(const lion_sim *sim, double *x, double *y, double *z, double *vx,
                   double *vy, double *vz, double *t);

/* Accelerations (m/s^2) at the current positions and time, recomputed now by
 * the kernels that step the handle (length n_total host arrays): a_i =
 * (Q_i/M_i)(E_c,i + E_ext(r_i, t)), eq. (field) with the Coulomb sum of eq.
 * (fullPotential) (section "Dynamics of trapped ions"; the force of section
 * "Forces and fields" that evolve integrates).  NULL output -> LION_ERR_ARG;
 * state not set -> LION_ERR_STATE.  Synchronises. */
int lion_compute_accel(lion_sim *sim, double *ax, double *ay, double *az);

/* Kinetic energy sum M v^2/2, Coulomb energy sum_{i<j} k_e Q_i Q_j / r_ij
 * (the pair term of eq. (fullPotential)) and dc-trap energy
 * sum Q_i (kappa U0/Z0^2)(z^2 - (x^2 + y^2)/2), in J, summed over all traps.
 * Synchronises. */
int lion_get_energy(lion_sim *sim, double *kinetic, double *coulomb, double *dc_trap);

/* LION_ERR_NONFINITE if any position or velocity is NaN or infinite, else
 * LION_OK.  Synchronises. */
int lion_check_finite(lion_sim *sim);

/* Lost-ion check (section "Simulation domain": the integration volume is
 * expanded as ions leave it; here there is no volume, and ions that escape an
 * unstable trap show up in this count instead): *count receives the number of ions,
 * over every trap of the handle, farther than r_lost_m (m) from the trap
 * centre or with a non-finite position.  r_lost_m <= 0 or non-finite, or
 * count NULL -> LION_ERR_ARG.  Changes no state.  Synchronises. */
int lion_count_lost(lion_sim *sim, double r_lost_m, int64_t *count);

/* Message of the last failure on this handle ("" if none; a static string for
 * sim == NULL). */
const char *lion_last_error(const lion_sim *sim);

/* Release host-side objects and cached launch graphs.  The workspace stays
 * owned by the caller. */
void lion_destroy(lion_sim *sim);

/* Launch shape of the hot kernels; any field <= 0 keeps the built-in choice.
 * Values outside the listed sets -> LION_ERR_ARG. */
typedef struct {
    int32_t i_per_lane;   /* target ions per lane in the pair kernel: 1, 2 or 4          */
    int32_t j_split;      /* source slices per step (1..64; clipped to one per 64 sources),
                             partial sums reduced in slice order                           */
    int32_t chunk_steps;  /* steps per captured launch graph (1..1000).  Built-in: 1000
                             for a single trap on the one-workgroup path and for batches
                             of traps of at most 64 ions, else 100                        */
    int32_t flush_len;    /* LION_MIXED_F64ACC: sources per FP32 run: 4, 8 or 16           */
    int32_t batch_block;  /* threads per trap in batched mode and on the one-workgroup path:
                             64 (traps of at most 64 ions only), 256, 512 or 1024.  Built-in:
                             batched, 64 when the largest trap holds at most 16 ions, 1024
                             when it holds 256 or more, else 256; a lone trap on the
                             one-workgroup path, 64 up to 16 ions, 256 up to 32, 512 up to
                             64, 1024 above.  64 runs the wave kernel on one wave (target
                             state in registers, source parts in consecutive lanes); 256,
                             512 or 1024 run it on that many threads for traps of at most
                             48 ions and threads / 8, the batched kernel otherwise          */
    int32_t use_graph;    /* 1: replay captured graphs, 2: plain stream launches           */
    int32_t lds_sources;  /* FP32 pair modes: 1: sources by scalar loads, 2: LDS tiles        */
    int32_t symmetric;    /* 1: all ordered pairs; 2: each pair once (Newton's third law);
                             one trap of N <= 131072 (else LION_ERR_UNSUPPORTED).  Built-in
                             (0): each pair once where that is allowed and N >= 8192.
                             With
                             LION_MIXED_KAHAN the FP32 runs of each 256 x 256 tile pair are
                             added in compensated FP32 and the tile-pair totals in FP64       */
    int32_t sym_variant;  /* pair-once kernel variant, 1..9 (built-in: 9 for
                             LION_MIXED_F64ACC, 6 for LION_FP64; LION_MIXED_KAHAN always
                             runs the shape of 7).  FP32 pairs: reaction sums
                             per chunk of 8 or 4 sources, sources unrolled, register budget,
                             next source prefetched: 1: 8, two, 4 waves/SIMD; 2: 4, one,
                             5 waves; 3: 4, one, 6 waves; 4: 8, one, 5-wave budget; 5: 4, one,
                             4 waves; 6: 8, one, 5-wave budget, prefetch; 7: 8, two, 4 waves,
                             prefetch; the target sums in FP32 runs of 8 sources (1-7),
                             16 (8: the shape of 7) or 64 (9: the shape of 7).  FP64: 1: two
                             sources unrolled, 3 waves/SIMD; 2: one, 4 waves; 3: one,
                             3 waves; 4: two, 4 waves (spills); 5: two, 2 waves; 6: one,
                             4 waves, prefetch; 7, 8, 9: two, 3 waves, prefetch              */
    int32_t update_waves; /* waves that share the slice sums of 64 ions in the step
                             epilogue: 4, 8 or 16 (built-in: 4)                               */
    int32_t small_trap;   /* single trap: 1: always the multi-workgroup kernels; 2: step the
                             trap inside one workgroup, many steps per launch (the batched
                             kernel with one trap; N <= 1024, no body exclusion or rigid
                             bodies, else the multi-workgroup kernels run).  Built-in: 2
                             for N <= LION_SMALL_TRAP_IONS, else 1                           */
    int32_t batch_tpt;    /* batched kernel (and the one-workgroup path): targets per thread
                             for traps of 128 ions or more: 1, 2 or 4 (at most 2 with 1024
                             threads per trap; 2 or 4 is raised where the threads times the
                             count fall short of the trap's ions).  Built-in: 2 (4 below
                             1024 threads) from 256 ions, 2 from 128 in a batch; 1 below    */
    int32_t step_launches; /* single trap stepped by the multi-workgroup kernels: 1: one
                             launch per step (each workgroup owns a few targets, takes all
                             sources, reduces over the workgroup and ends the step for its
                             targets; positions alternate between two buffers); 2: the pair
                             kernel, then the epilogue.  Handles with body exclusion or
                             rigid bodies take 2.  Built-in: 1 for N <= LION_ONE_LAUNCH_IONS
                             when the all-pairs kernels are selected, else 2                  */
} lion_kernel_config;

/* Ion count up to which a single trap is stepped inside one workgroup by default. */
#define LION_SMALL_TRAP_IONS 128

/* Ion count up to which a single trap on the multi-workgroup kernels takes one
 * launch per step by default. */
#define LION_ONE_LAUNCH_IONS 2048

int lion_set_kernel_config(lion_sim *sim, const lion_kernel_config *cfg);
int lion_get_kernel_config(const lion_sim *sim, lion_kernel_config *cfg);

/* Measurement helper: launches the pair-field kernel of this handle once to
 * warm up, then `reps` times (1..10000) back to back on the handle's stream at
 * the current positions between two HIP events recorded on that stream, and
 * returns the mean duration per launch in *ms_avg.  Changes no state (only the
 * partial-sum scratch).  Single-trap handles only (LION_ERR_UNSUPPORTED for
 * batches).  Synchronises. */
int lion_time_pair_kernel(lion_sim *sim, int32_t reps, double *ms_avg);

/* As lion_time_pair_kernel for the batched kernel: `reps` back-to-back
 * launches of `nsteps` in-kernel steps each (no warm-up launch).  The state
 * advances by reps * nsteps steps.  Batched handles only.  Synchronises. */
int lion_time_batch_kernel(lion_sim *sim, int32_t reps, int32_t nsteps, double dt,
                           double *ms_avg);

/* Allocation-free force evaluation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The accelerations (m/s^2) that lion_compute_accel gives
 * on a single-trap handle of these ions with this trap (lion_set_trap's
 * parameters, full rf field, no bodies) at time t, from the same all-pairs
 * kernels: a_i = (Q_i/M_i)(E_c,i + E_ext(r_i, t)).  No handle, no workspace:
 * x, y, z (m), charges_C, masses_kg and the outputs ax, ay, az are device
 * arrays of n doubles owned by the caller; the packed source streams, Q/M,
 * the trap and the per-slice partial sums live in one 8 MiB device array of
 * the library (a file-scope __device__ array, its address taken once per
 * device on the first call there, held until the process ends).  Hence
 * 1 <= n <= 65536 (else LION_ERR_ARG, before any device work), and calls on
 * one GPU share that array: calls that overlap on one GPU (other streams,
 * other threads) race and must be ordered by the caller.  Runs on hip_stream
 * (NULL: the default stream) and returns once queued; calls no hipMalloc,
 * hipFree or allocating library routine.  NULL pointers, a bad trap (as
 * lion_set_trap), a non-finite t or an unknown precision -> LION_ERR_ARG;
 * lion_last_error(NULL) gives the message. */
int lion_accel_noalloc(int64_t n, const double *x, const double *y, const double *z,
                       const double *charges_C, const double *masses_kg, double V_rf,
                       double Omega_rad_s, double U_dc, double r0, double z0, double kappa,
                       double t, int precision, double *ax, double *ay, double *az,
                       void *hip_stream);

/* Host-only helper, eq. (Mathieuaq): the (V0, U0) giving Mathieu coefficients
 * (q_x, a_x) to an ion of mass M (kg) and charge Q (C) in a trap of angular
 * frequency Omega and geometry (r0, z0, kappa).  LION_ERR_ARG on invalid input. */
int lion_mathieu_to_voltages(double q_x, double a_x, double M, double Q, double Omega,
                             double r0, double z0, double kappa, double *V0, double *U0);

/* Physical constants used by the library (CODATA 2018): elementary charge (C),
 * vacuum permittivity (F/m), atomic mass unit (kg). */
void lion_constants(double *e_charge, double *eps0, double *amu);

#ifdef __cplusplus
}
#endif

#endif /* LION_H */
