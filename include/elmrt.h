/*
 * elmrt.h -- C ABI of the MI355X (gfx950) library that advances the entropic
 * multi-relaxation-time two-phase lattice Boltzmann model of Hosseini,
 * Dorschner & Karlin ("Entropic multi-relaxation-time lattice Boltzmann model
 * for large density ratio two-phase flows", arXiv:2201.12404).
 *
 * One time step (Sec. 2, eq. LBGK) is: pull-streaming of the populations,
 * moments rho and rho u (Sec. 2.2), Peng-Robinson pressure and pseudo-potential
 * psi (Sec. 2.3, 3.1), the psi and capillary force stencils of reach 2
 * (Sec. 2.3), the diagonal correction Phi (Sec. 2.2), the product-form f^eq
 * and f* (Sec. 2.1-2.2), the k + s + h split in the modified central Hermite
 * basis (Appendix A), the entropic stabiliser gamma (Sec. 2.4) and the
 * post-collision state.
 *
 * Conventions
 *   - Every call returns elmrt_status; nothing throws across the ABI.  On an
 *     error elmrt_last_error() returns a message (per thread).
 *   - Lattice units dt = dr = 1, cs^2 = 1/3, P0 = rho cs^2 (Sec. 2.3).
 *   - Cells are numbered cell = x + nx*(y + ny*z); host vector fields are
 *     component-major: u[a*N + cell].
 *   - Velocities are numbered i = (cx+1) + 3(cy+1) + 9(cz+1);
 *     elmrt_velocities() returns the table.
 *   - Device memory is caller-owned: a workspace of elmrt_workspace_bytes()
 *     bytes, 256-byte aligned, that must outlive the handle.  The library
 *     never allocates device memory for a simulation.
 *   - Work is enqueued on the caller's HIP stream; elmrt_step never
 *     synchronises.  Calls on one handle must come from one host thread at a
 *     time.
 */
#ifndef ELMRT_H
#define ELMRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct elmrt_sim elmrt_sim;   /* opaque, library-owned */

typedef enum {
    ELMRT_OK = 0,
    ELMRT_E_INVALID = 1,   /* bad argument or parameter; nothing was enqueued */
    ELMRT_E_NOMEM = 2,     /* workspace too small or host allocation failed */
    ELMRT_E_DEVICE = 3,    /* a HIP call failed; the handle may be unusable */
    ELMRT_E_UNSTABLE = 4,  /* a non-finite, non-positive or >= 1/b density was seen (sticky) */
    ELMRT_E_STATE = 5      /* call out of order (e.g. step before init_fields) */
} elmrt_status;

enum { ELMRT_D2Q9 = 0, ELMRT_D3Q27 = 1 };
enum { ELMRT_FP32 = 0, ELMRT_FP64 = 1 };
enum { ELMRT_ENTROPIC = 0, ELMRT_BGK = 1 };
enum { ELMRT_PERIODIC = 0, ELMRT_WALL = 1 };
/* Readings of points the paper leaves open (elmrt_params.readings, a bit set;
 * 0 = the default reading of each). */
enum {
    ELMRT_READING_TRACE_IN_S = 1,        /* the trace of the second-order central moments relaxes
                                            with omega as part of s; default: part of h, under
                                            entropic control (Sec. 3.1.2, Appendix A) */
    ELMRT_READING_PHI_FLUID_VELOCITY = 2 /* the flux q of Phi (Sec. 2.2) uses the fluid velocity
                                            u + F dt/(2 rho); default: the bare u = sum c f / rho */
};

/* Problem statement.  struct_size must be sizeof(elmrt_params). */
typedef struct {
    uint32_t struct_size;
    int32_t  lattice;        /* ELMRT_D2Q9 or ELMRT_D3Q27 (Sec. 2.1) */
    int32_t  precision;      /* ELMRT_FP32: populations, density and fluxes stored in FP32;
                                per-cell scalars (moments, EOS, force sums, f^eq, f*) are
                                formed in FP64 registers, the small non-equilibrium terms
                                in FP32, one rounding per stored population.
                                ELMRT_FP64: storage and arithmetic in FP64. */
    int32_t  collision;      /* ELMRT_ENTROPIC (gamma of Sec. 2.4) or ELMRT_BGK (gamma = 2) */
    int64_t  n[3];           /* nx, ny, nz; nz = 1 for D2Q9; each >= 4 */
    int32_t  bc[3];          /* per axis: ELMRT_PERIODIC, or ELMRT_WALL (half-way
                                bounce-back at both ends; stencil ghosts mirror
                                the density about the wall plane) */
    int32_t  readings;       /* 0, or ELMRT_READING_* bits */
    /* Peng-Robinson equation of state (Sec. 3.1): a, b, R, acentric factor,
       and the temperature as T/Tc with Tc = 0.0778 a / (0.45724 b R). */
    double   eos_a, eos_b, eos_R, acentric, T_over_Tc;
    double   kappa_tilde;    /* capillarity kappa~ = kappa dr^2 of the force stencil (Sec. 2.3), >= 0;
                                with target_W > 0 it must be 0 and is derived from W */
    /* Kinematic viscosity nu (omega = 1/(3 nu + 1/2), Sec. 2): nu_vapour at
       rho <= rho_vapour, nu_liquid at rho >= rho_liquid, linear in between.
       With nu_liquid == nu_vapour the two densities are not used. */
    double   nu_liquid, nu_vapour;
    double   rho_liquid, rho_vapour;
    /* Uniform body acceleration g: the force of Sec. 2 (F in the extended
       equilibrium f*) gains rho g in every cell.  Components beyond the
       lattice's dimension must be 0. */
    double   body_accel[3];
    /* > 0: interface width W = (rho_l - rho_v) / max |grad rho| (Sec. 3.1.1)
       from which kappa_tilde is derived (elmrt_kappa_for_width); 0: use
       kappa_tilde as given. */
    double   target_W;
} elmrt_params;

/* Bytes of device workspace the problem needs (populations twice, density
 * and Phi-flux fields, a small status/reduction area). */
elmrt_status elmrt_workspace_bytes(const elmrt_params* p, size_t* bytes);

/* Validate p and bind a handle to the caller's workspace (device pointer,
 * 256-byte aligned, >= elmrt_workspace_bytes) and HIP stream (hipStream_t, or
 * NULL for the null stream).  Fails with ELMRT_E_INVALID on: unknown lattice,
 * precision, collision or bc; n < 4 on an axis (nz != 1 for D2Q9); cells
 * >= 2^31; Q x (cells per plane normal to the last axis) x value size
 * >= 2^31 bytes; a, b, R <= 0; T/Tc outside (0, 1); kappa_tilde < 0;
 * nu <= 0; rho_liquid <= rho_vapour when the viscosities differ; unknown
 * readings bits; a non-finite body acceleration, or one along an axis the
 * lattice lacks; target_W < 0, or target_W > 0 with kappa_tilde != 0, or a
 * temperature without a two-phase region when target_W > 0. */
elmrt_status elmrt_create(const elmrt_params* p, void* dev_workspace, size_t workspace_bytes,
                          void* hip_stream, elmrt_sim** out);

/* Set the state to f = f^eq(rho0, u0 - F(rho0) dt / (2 rho0)) (product form,
 * Sec. 2.2), with F the force of Sec. 2.3 on the initial density: u0 is the
 * fluid velocity u + F dt/(2 rho) of the exact-difference forcing, so a drop
 * given u0 = 0 starts at rest.  rho0[N] and u0[D*N] are host FP64 arrays read
 * before the call returns; rho0 must be finite and positive and u0 finite
 * (else ELMRT_E_INVALID).  Synchronises the stream. */
elmrt_status elmrt_init_fields(elmrt_sim* s, const double* rho0, const double* u0);

/* Enqueue nsteps >= 0 time steps on the stream (two kernels per step). */
elmrt_status elmrt_step(elmrt_sim* s, int64_t nsteps);

/* Like elmrt_step, and also time each kernel with HIP events on the stream;
 * synchronises.  ms[0] = summed duration of the moment kernels, ms[1] = of
 * the collision kernels (milliseconds). */
elmrt_status elmrt_step_timed(elmrt_sim* s, int64_t nsteps, double ms[2]);

/* Read rho(t) and the bare velocity u = sum c f / rho (Sec. 2.2) of the
 * current state into host FP64 arrays (either may be NULL), and the sums
 * [sum rho, sum rho u_x, sum rho u_y, sum rho u_z] (sums may be NULL),
 * accumulated in FP64 with Neumaier's compensated summation per thread,
 * across the lanes of each wavefront, the wavefronts of each workgroup and
 * the 1024 workgroup partials in order.  Synchronises.  Returns
 * ELMRT_E_UNSTABLE (outputs still filled) once a non-finite or non-positive
 * density, or one at or beyond 1/b (the pole of the Peng-Robinson pressure,
 * Sec. 3.1), has been seen by a step or a read-out. */
elmrt_status elmrt_read_macros(elmrt_sim* s, double* rho, double* u, double* sums);

/* For callers that cannot allocate memory or synchronise the host -- code
 * under HIP graph capture, serving loops that poll the diagnostics of
 * resident simulations -- the sums of elmrt_read_macros and the instability
 * flag, left in device memory.  Enqueues on the sim's stream, without
 * waiting: dev_sums[0..3] (device FP64) receives [sum rho, sum rho u_x,
 * sum rho u_y, sum rho u_z] of the current state, bitwise equal to the sums
 * elmrt_read_macros returns for it, and *dev_flag (device, may be NULL) the
 * instability flag word (nonzero: unstable).  No field is written; the host
 * allocates nothing and the library calls no hipMalloc.  The partial sums go
 * to a static device array of the library (one per device, 64 KiB: the 1024
 * workgroup partials of the reduction, for any grid the library accepts).
 * The sim's device must be current (else ELMRT_E_INVALID).  Calls on one
 * device share that array: calls enqueued on different streams that may run
 * at the same time race; order them (one stream, or events).  ELMRT_E_STATE
 * before elmrt_init_fields; ELMRT_E_DEVICE if the array's device address
 * cannot be looked up. */
elmrt_status elmrt_read_sums_noalloc(elmrt_sim* s, double* dev_sums, uint32_t* dev_flag);

/* Fluid velocity u + F dt/(2 rho) of the exact-difference forcing (Sec. 2.3,
 * F on the read-out density) at time t, u[D][N] FP64 host.  In a resting
 * two-phase state the bare velocity of elmrt_read_macros equals -F/(2 rho)
 * near interfaces; this is the velocity whose maximum measures spurious
 * currents (Sec. 3.1.2).  Same errors as elmrt_read_macros. */
elmrt_status elmrt_read_fluid_velocity(elmrt_sim* s, double* u);

/* Enqueue on the sim's stream a copy of its sticky instability flag (nonzero
 * once a non-finite or non-positive density has been seen) into *host_word,
 * without waiting: the word holds the flag as of the work enqueued before
 * this call once the stream has reached it.  host_word should be pinned host
 * memory (hipHostMalloc); a pageable word makes the copy synchronous. */
elmrt_status elmrt_poll_unstable(elmrt_sim* s, uint32_t* host_word);

/* ---- Checkpoints --------------------------------------------------------
 *
 * A snapshot holds everything the next steps depend on: the populations of
 * the current time (in the library's device layout), the instability flag and
 * the fall-back count, behind a header naming the lattice, precision and
 * grid.  It lives in caller-owned device memory of elmrt_state_bytes bytes.
 * Restoring it into any sim of the same lattice, precision and grid and
 * stepping gives bitwise the same states as the run it was taken from. */
elmrt_status elmrt_state_bytes(const elmrt_sim* s, size_t* bytes);

/* Copy the current state into dev_dst (device memory, >= elmrt_state_bytes
 * bytes), asynchronously on the sim's stream.  ELMRT_E_STATE before
 * elmrt_init_fields. */
elmrt_status elmrt_save_state(elmrt_sim* s, void* dev_dst, size_t bytes);

/* Replace the state of s by a snapshot (reads its header: synchronises the
 * stream; the copies are then asynchronous).  ELMRT_E_INVALID for a buffer
 * that is not a snapshot, or one of a different lattice, precision or grid.
 * Marks s initialised. */
elmrt_status elmrt_load_state(elmrt_sim* s, const void* dev_src, size_t bytes);

/* Number of cell updates since elmrt_init_fields in which the entropic
 * gamma fell back to 2/omega, i.e. h was relaxed to equilibrium because some
 * f*_i <= 0 or <dh|dh> <= eps^2 rho with eps = 2^-53 (Sec. 2.4; the
 * stabiliser is undefined there).  0 for BGK.  The test of <dh|dh> is taken in
 * the build's working precision, so the FP32 and FP64 builds may count
 * differently near equilibrium.  Synchronises the stream. */
elmrt_status elmrt_gamma_fallbacks(elmrt_sim* s, int64_t* cells);

/* Read the populations f_i(r, t) (post-streaming) into host FP64 f[i*N + cell]. */
elmrt_status elmrt_read_populations(elmrt_sim* s, double* f);

/* Velocity table: c[3*i + a] for i < Q (9 or 27); returns Q, or -1. */
int32_t elmrt_velocities(int32_t lattice, int32_t* c);

/* Coexistence densities and saturation pressure of the Peng-Robinson EOS
 * from the Maxwell equal-area rule (Sec. 3.1.1), host FP64. */
elmrt_status elmrt_coexistence(const elmrt_params* p, double* rho_vapour, double* rho_liquid,
                               double* p_sat);

/* Capillarity kappa~ for an interface of width W (> 0) of the EOS in p at its
 * T/Tc, host FP64: the square-gradient first integral (kappa~/2) rho'^2 =
 * omega(rho) of a flat interface, with the excess grand potential omega(rho)
 * = rho int_{rho_v}^{rho} (P(s) - P_sat)/s^2 ds between the Maxwell densities
 * (textbook van der Waals theory; the paper does not give kappa~), makes the
 * steepest gradient sqrt(2 max omega / kappa~), so kappa~ = 2 max(omega) W^2
 * / (rho_l - rho_v)^2.  The integral is the closed-form antiderivative of P/s^2.
 * The model's converged interfaces approach W as W grows (at W = 5 they are
 * some 30 % wider: the stencils' own discretisation). */
elmrt_status elmrt_kappa_for_width(const elmrt_params* p, double W, double* kappa);

/* Peng-Robinson pressure P(rho) (Sec. 3.1) of the EOS in p at its T/Tc, for
 * n host FP64 densities (post-processing: Laplace pressure jumps). */
elmrt_status elmrt_pressure(const elmrt_params* p, const double* rho, double* P, int64_t n);

/* Move s to another HIP stream (NULL: the null stream): its later calls
 * enqueue there.  Work already enqueued for s on the old stream is not moved:
 * the caller orders it before the new stream's work (synchronise the old
 * stream, or record an event there and wait for it).  A batch member must
 * share the batch's stream when it is stepped (rebuild the batch after
 * moving a member). */
elmrt_status elmrt_set_stream(elmrt_sim* s, void* stream);

/* Tile shape of the collision kernel: tx x ty cells per workgroup, marched
 * over tm planes along the last axis.  Compiled shapes:
 * D2Q9 ty = 1 with tx = 64, 128 or 256; D3Q27 (tx, ty) = (64, 4), (64, 2),
 * (32, 8) or (128, 2).  Other shapes, or tm < 0, return ELMRT_E_INVALID and
 * leave the tiling unchanged.  tm = 0 (the default, with 64 x 1 or 64 x 4)
 * picks the depth automatically: the deepest of 16, 8, 4, 2, 1 (at most the
 * last grid extent) for which the launch -- the sim stepped alone, or all
 * members of a batch together -- still has >= 2048 (D3Q27) or 4096 (D2Q9)
 * wavefronts.  Every tiling gives bitwise the same result. */
elmrt_status elmrt_set_tiling(elmrt_sim* s, int32_t tx, int32_t ty, int32_t tm);

/* The current tiling (tm = 0: automatic depth); any pointer may be NULL. */
elmrt_status elmrt_get_tiling(const elmrt_sim* s, int32_t* tx, int32_t* ty, int32_t* tm);

/* Pick the collision tiling of s by measurement, in two stages: every
 * compiled tile shape of the lattice at marching depths 1, 2, 4, 8, 16, 32,
 * 64, then the fastest shape at depths 6..62 (even), 96 and 128; the three
 * fastest candidates are then timed again over 3 x trial_steps.  Each
 * candidate runs 1 + trial_steps steps (the extra step untimed), timed with
 * HIP events on the sim's stream; the fastest is kept.  The trial steps advance the simulation (results do
 * not depend on the tiling); their number is written to *steps_taken (may be
 * NULL).  Synchronises the stream.  trial_steps >= 1. */
elmrt_status elmrt_autotune(elmrt_sim* s, int32_t trial_steps, int64_t* steps_taken);

/* ---- Batches: many independent simulations advanced together ------------
 *
 * A batch advances several initialised simulations of the same lattice,
 * precision and stream with one moment launch and one collision launch per
 * tile shape per step, whose workgroups cover the tiles of every member
 * (a device job table maps each workgroup to its simulation and tile).  Pairs
 * of steps are captured once into a HIP graph and replayed.  Each member
 * evolves exactly as if stepped alone with the same tiling (bitwise), and
 * keeps working through its own handle: elmrt_read_macros etc. see the
 * batch's steps, and stepping a member alone between batch steps is allowed
 * (the table is rebuilt).  The job table lives in a caller-owned device
 * workspace of elmrt_batch_workspace_bytes(count) bytes (256-byte aligned),
 * which must outlive the batch; the members must outlive it too. */
typedef struct elmrt_batch elmrt_batch;

elmrt_status elmrt_batch_workspace_bytes(int32_t count, size_t* bytes);

/* Fails with ELMRT_E_INVALID for count < 1, a NULL or repeated member,
 * members of different lattice, precision or stream, or a small or
 * misaligned workspace; ELMRT_E_STATE if a member is not initialised.
 * Uploads the job table (synchronises the stream). */
elmrt_status elmrt_batch_create(elmrt_sim* const* sims, int32_t count, void* dev_workspace,
                                size_t workspace_bytes, elmrt_batch** out);

/* Advance every member by nsteps (asynchronous on the members' stream; the
 * graph is captured on a private stream at first use).  ELMRT_E_STATE if a
 * member has been moved to another stream since the batch was created. */
elmrt_status elmrt_batch_step(elmrt_batch* b, int64_t nsteps);

/* use_graph = 0: enqueue the launches directly instead of replaying the
 * captured graph (same results). */
elmrt_status elmrt_batch_set_graph(elmrt_batch* b, int32_t use_graph);

/* Pick one collision tiling for all members by measurement: every compiled
 * tile shape at depths 1, 2, 4, 8, 16, 32, 64 (the first stage of
 * elmrt_autotune); each candidate runs 2 + trial_steps batch steps, the
 * marching depth capped at each member's last extent.  The
 * trial steps advance every member; their number goes to *steps_taken. */
elmrt_status elmrt_batch_autotune(elmrt_batch* b, int32_t trial_steps, int64_t* steps_taken);

/* Release the batch (not the members or the workspace).  NULL is ignored. */
void elmrt_batch_destroy(elmrt_batch* b);

/* Release the handle (not the workspace).  NULL is ignored. */
void elmrt_destroy(elmrt_sim* s);

/* ---- Serving: a request loop over resident simulations ------------------
 *
 * Jobs (a problem statement as for elmrt_create, initial fields as for
 * elmrt_init_fields, a step count) are queued by elmrt_server_submit and
 * admitted in arrival order while their workspace fits a caller-owned device
 * pool (first fit; a job that does not fit waits, and so do the ones behind
 * it).  Admitted jobs stay resident and are advanced in rounds enqueued by
 * elmrt_server_run: a round takes the resident jobs first in the scheduling
 * order (elmrt_server_set_policy: arrival order -- the default -- least
 * remaining work -- cells x steps -- first, or that with the oldest job
 * always first): the first of them, and after it those that fit the rest of
 * a fill budget (elmrt_server_set_fill, default 2^21 cells), and advances them as one batch per lattice and
 * precision (the elmrt_batch_* machinery, without graphs; a lattice and
 * precision with one job in the round steps it as elmrt_step): the costliest
 * batch by chunk_steps, a cheaper one by proportionally more steps (bytes
 * per step: D2Q9 132 B, D3Q27 356 B per cell), none beyond the fewest steps a
 * member still needs, so every job stops exactly at its step count.
 * A scheduling pass (one per 'rounds' of elmrt_server_run) never waits for
 * the device: it reads out the jobs whose last round has completed (fields
 * and sums kept on the host until elmrt_server_result) and returns their
 * memory to the pool, uploads and initialises newly admitted jobs -- both on
 * a second stream the server creates (non-blocking, default priority) --
 * and enqueues the next round on the compute stream (the caller's) while
 * fewer than two rounds are in flight; a pass with nothing to do pauses for
 * 0.1 ms.  After its steps in a round, each job's instability flag is
 * copied to pinned host memory (elmrt_poll_unstable); a job seen unstable is
 * evicted: it is not advanced further, and is read out (status
 * ELMRT_E_UNSTABLE, fields as they stand) and its memory freed while the
 * others continue.  A job's result is bitwise the same as the same
 * simulation run alone.  The server owns its job records; the pool and the
 * stream are the caller's and must outlive it.  Not thread-safe: one thread
 * drives a server. */
typedef struct elmrt_server elmrt_server;

/* dev_pool: device memory (256-byte aligned, >= 4096 bytes) the server carves
 * job workspaces and batch tables from; stream: hipStream_t or NULL, the
 * compute stream.  ELMRT_E_DEVICE if the server's own stream or events cannot
 * be created. */
elmrt_status elmrt_server_create(void* dev_pool, size_t pool_bytes, void* stream, int64_t chunk_steps,
                                 elmrt_server** out);

/* Fill budget: cells a round advances at most, its first job aside (which
 * always runs); a later job joins the round only if it fits.  >= 1. */
elmrt_status elmrt_server_set_fill(elmrt_server* s, int64_t cells);

/* Scheduling order of resident jobs: 0 arrival (the default), 1 least
 * remaining work (cells x remaining steps) first, 2 as 1 but the oldest
 * resident job always first (it advances every round, so none starves). */
elmrt_status elmrt_server_set_policy(elmrt_server* s, int32_t policy);

/* Queue a job; the fields (rho0[N], u0[D][N], FP64 host) are copied.  Fails
 * with ELMRT_E_INVALID when elmrt_create would reject p.  *job_id > 0. */
elmrt_status elmrt_server_submit(elmrt_server* s, const elmrt_params* p, const double* rho0, const double* u0,
                                 int64_t steps, int64_t* job_id);

/* Run up to 'rounds' scheduling passes (retirement of jobs whose last round
 * has completed, admission, and a new round while fewer than two are in
 * flight); returns early when no job is queued or resident.  *queued,
 * *resident (may be NULL) count the jobs waiting and on the device (including
 * finished ones not yet read out). */
elmrt_status elmrt_server_run(elmrt_server* s, int32_t rounds, int32_t* queued, int32_t* resident);

/* State of a job (0 queued, 1 resident, 2 done, 3 failed), its submit /
 * admit / finish times in seconds of a monotonic host clock, and the steps it
 * has taken.  Any pointer may be NULL. */
elmrt_status elmrt_server_job(elmrt_server* s, int64_t job_id, int32_t* state, double times[3],
                              int64_t* steps_done);

/* Copy out the final rho[N], u[D][N] and sums[4] of a finished job (as
 * elmrt_read_macros; ELMRT_E_UNSTABLE if its flag was set, outputs still
 * written).  ELMRT_E_STATE while the job is queued or resident.  The result
 * is released after the call. */
elmrt_status elmrt_server_result(elmrt_server* s, int64_t job_id, double* rho, double* u, double* sums);

/* Lattice updates (cells x steps) advanced so far and the pool's free bytes. */
elmrt_status elmrt_server_stats(elmrt_server* s, int64_t* lattice_updates, size_t* pool_free);

/* Release every resident simulation and the server (not the pool).  NULL is
 * ignored. */
void elmrt_server_destroy(elmrt_server* s);

/* Message of the last failed call on this thread ("" if none). */
const char* elmrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
