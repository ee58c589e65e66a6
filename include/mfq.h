/*
 * mfq.h -- monitored free-fermion quantum trajectories on AMD MI355X (gfx950).
 *
 * C ABI of the library libmfq.so.  It implements the quantum-trajectory method
 * of arXiv:2508.18468 (Fan, Yin, Garcia-Garcia, "Entanglement dynamics of
 * monitored noninteracting fermions on graphics processing units") for
 * noninteracting U(1) fermions with nearest-neighbour hopping:
 *
 *   state     Slater determinant of N orbitals: an L x N complex matrix U with
 *             U^+ U = 1, correlation matrix C = U U^+      (Appendix A, Eq. (A3))
 *   step      U <- exp(-i Ht dt) U, then either projective measurements of n_i
 *             (Eq. (A1), Eq. (A2) with the sign of its rank-1 term corrected)
 *             or the homodyne factor of Eq. (A4); then re-orthonormalisation
 *             (Appendix A, QR after each step; done here by Cholesky-QR2)
 *   observe   S_A from the eigenvalues of C restricted to A (Sec. II entropy
 *             formula), mutual information I2 = S_A + S_B - S_AuB (Sec. IV)
 *
 * Conventions shared by every call:
 *   - Complex numbers are interleaved (re, im) IEEE doubles (16 bytes).
 *   - U of trajectory t is column-major L x N with leading dimension L; the
 *     n_traj trajectories are stored one after another (stride L*N), so the
 *     whole batch is one column-major L x (N*n_traj) matrix.
 *   - Sites are numbered i = x + Lx*y (y = 0 in 1d).  Regions are lists of
 *     distinct site ids in [0, L), strictly ascending; otherwise MFQ_EINVAL.
 *   - All device work is ordered on the context's HIP stream.  mfq_step is
 *     asynchronous; calls that return host data synchronise the stream.
 *   - Random numbers: Philox4x64-10, key = (seed, uid of the trajectory),
 *     counter = (absolute step index n >= 1, site i, purpose, 0); purpose 0
 *     = projective (word 0 selects the site, word 1 decides the outcome),
 *     purpose 1 = homodyne (words 0 and 1 give one Box-Muller normal).  The
 *     draws of a trajectory depend only on (seed, uid, n, i): one call of n
 *     steps equals n calls of one step, and batching never changes results.
 *   - Every call returns MFQ_OK (0) or a negative error code; none aborts and
 *     none throws.  mfq_last_error() describes the last failure on a context.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef MFQ_H
#define MFQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfq_ctx mfq_ctx;
typedef int32_t mfq_status;

#define MFQ_OK 0
#define MFQ_EINVAL (-1)   /* bad argument (null pointer, size, region, order) */
#define MFQ_ENOMEM (-2)   /* device allocation failed or workspace too small */
#define MFQ_EDEVICE (-3)  /* HIP runtime error */
#define MFQ_ENUMERIC (-4) /* Cholesky breakdown or a non-finite value */
#define MFQ_ESTATE (-5)   /* call out of order (e.g. step before init_state) */
#define MFQ_PENDING 1     /* serving engine: job not finished yet */

#define MFQ_PROJECTIVE 0  /* projective n_i measurements, Appendix A (PM) */
#define MFQ_HOMODYNE 1    /* homodyne / quantum state diffusion, Eq. (A4) (QSD) */

#define MFQ_FP64 0        /* every step in FP64 */
#define MFQ_FP32_BULK 1   /* propagator product in FP32 on the matrix cores, written as
                             U + (P - I) U with the identity term in FP64; Born
                             probabilities, homodyne / projective updates, Cholesky-QR2
                             and the eigensolver in FP64 */

/* Lattice of Sec. II (1d ring) or Sec. IV (2d torus); periodic boundaries,
 * nearest-neighbour hopping Ht_ij = J.  dim = 1: L = Lx (Ly ignored);
 * dim = 2: L = Lx*Ly.  Lx (and Ly for dim 2) must be >= 2. */
typedef struct {
  int32_t dim;
  int32_t Lx;
  int32_t Ly;
  int32_t reserved;
  double J;
} mfq_lattice;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to
 * order all work on, or NULL (the library then creates and owns a stream).
 * The first context on a device also resolves that device's address of the static
 * buffer of mfq_density_correlation_noalloc.
 * *out receives the context.  Errors: MFQ_EINVAL, MFQ_EDEVICE. */
mfq_status mfq_create(int device, void *hip_stream, mfq_ctx **out);

/* Destroy a context and free what the library allocated (never the caller's
 * workspace).  NULL is accepted. */
mfq_status mfq_destroy(mfq_ctx *ctx);

/* Text of the last error on ctx; owned by ctx, valid until the next call on
 * ctx.  Never NULL. */
const char *mfq_last_error(const mfq_ctx *ctx);

/* Device workspace, in bytes, that mfq_init_state needs for this problem
 * (state double buffer, propagator, Gram / Cholesky buffers, scratch). */
mfq_status mfq_workspace_bytes(const mfq_lattice *lat, int32_t N, int32_t n_traj,
                               int32_t precision, size_t *bytes);

/* Set up n_traj trajectories of N particles on lattice *lat and put each into
 * the initial product state of Appendix A: orbital k = e_{occupied[k]}.
 * occupied: N ascending site ids, or NULL for the Neel state (even sites in
 * 1d) / checkerboard (x+y even in 2d), which needs N = L/2 and even L.
 * traj_uid: n_traj host values that key each trajectory's random numbers.
 * dev_ws: caller-owned device memory of ws_bytes >= mfq_workspace_bytes(),
 * borrowed until the next init_state or destroy, or NULL to let the library
 * allocate it.  Resets the step counter to 0.  1 <= N < L, n_traj >= 1.
 * Errors: MFQ_EINVAL, MFQ_ENOMEM, MFQ_EDEVICE. */
mfq_status mfq_init_state(mfq_ctx *ctx, const mfq_lattice *lat, int32_t N, int32_t n_traj,
                          const uint64_t *traj_uid, const int32_t *occupied, int32_t precision,
                          void *dev_ws, size_t ws_bytes);

/* Advance every trajectory by n_steps steps of length dt with the given
 * protocol; gamma is a host array of n_traj monitoring rates (>= 0).
 * Projective: each site is measured with probability min(gamma*dt, 1) per
 * step; measured sites are projected in ascending order with their
 * conditional Born probabilities (Appendix A; the paper draws Poisson
 * waiting times instead).  Homodyne: rows of U are scaled by
 * exp(xi_i + gamma (2<n_i> - 1) dt), xi_i ~ N(0, gamma dt) (Eq. (A4), applied
 * after the propagator).  The propagator exp(-i Ht dt) is rebuilt when dt
 * changes.  Asynchronous, except projective steps in the blocked form (see
 * mfq_set_pm_path), which synchronise the stream twice per step; numeric
 * failures (Cholesky breakdown) surface as MFQ_ENUMERIC from the next
 * synchronising call.
 * Errors: MFQ_EINVAL, MFQ_ESTATE, MFQ_EDEVICE. */
mfq_status mfq_step(mfq_ctx *ctx, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                    int32_t n_steps);

/* Entanglement entropy S_A (Sec. II) of region A = region[0..n_sites) for
 * every trajectory: S_host[t], caller-owned, n_traj doubles.  Computed from
 * the eigenvalues of C_A = U_A U_A^+ (or of U_A^+ U_A when n_sites > N, same
 * nonzero spectrum), clamped to [0, 1].  Synchronises.
 * Errors: MFQ_EINVAL, MFQ_ESTATE, MFQ_ENUMERIC, MFQ_EDEVICE. */
mfq_status mfq_entropy(mfq_ctx *ctx, const int32_t *region, int32_t n_sites, double *S_host);

/* Eigenvalues of C_A (ascending, not clamped) for every trajectory:
 * lam_host[t * m + k], m = min(n_sites, N), caller-owned.  Synchronises. */
mfq_status mfq_region_spectrum(mfq_ctx *ctx, const int32_t *region, int32_t n_sites,
                               double *lam_host);

/* Mutual information I2 = S_A + S_B - S_{A u B} (Sec. IV) per trajectory;
 * A and B must be disjoint.  I_host: n_traj doubles.  Synchronises. */
mfq_status mfq_mutual_info(mfq_ctx *ctx, const int32_t *A, int32_t nA, const int32_t *B,
                           int32_t nB, double *I_host);

/* Density-density correlation of Sec. II, Eq. (2), on a 1d ring: by Wick's theorem
 * C_ij = -D_ij D_ji = -|C_ij|^2 for i != j, and C(r) is its average over the ordered site
 * pairs at ring distance r = min(|i - j|, L - |i - j|).  Cr_host[t * (L/2) + r - 1] for
 * r = 1 .. L/2, one trajectory each (the average over trajectories is the caller's).
 * Computed from the upper triangle of C = U U^+ on the matrix cores with the sums of
 * |C_ij|^2 along each diagonal formed in the product's epilogue (C is never stored).
 * Allocates a buffer on first use.  Synchronises.
 * Errors: MFQ_EINVAL (not a 1d lattice, NULL output), MFQ_ESTATE, MFQ_ENOMEM, MFQ_EDEVICE. */
mfq_status mfq_density_correlation(mfq_ctx *ctx, double *Cr_host);

/* Bytes of the per-GPU static buffer of mfq_density_correlation_noalloc (64 MiB). */
#define MFQ_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* mfq_density_correlation for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops that must not call hipMalloc, harnesses that forbid it): the
 * same kernels and the same result, bitwise, but the tile partials and the L/2 bins of every
 * trajectory go to a static device buffer of MFQ_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends, resolved once per device by mfq_create.
 * Nothing is allocated or freed on the device by this call.
 * Limit: (tile partials + L/2) x n_traj doubles must fit the buffer (for example L = 1024 with
 * up to 384 trajectories); larger requests fail with MFQ_ENOMEM before any launch.
 * The buffer is shared by every call on that GPU: calls that overlap on one GPU (contexts on
 * different streams or threads running this call at the same time) race and give wrong
 * results; sequential calls are safe (the call synchronises its stream before it returns,
 * and every value it reads from the buffer is written earlier in the same call).
 * Errors: as mfq_density_correlation, plus MFQ_ENOMEM above the limit. */
mfq_status mfq_density_correlation_noalloc(mfq_ctx *ctx, double *Cr_host);

/* Particle-number covariance of Sec. IV, Eq. (5): G_AB = -sum_{i in A, j in B} C_ij
 * = sum_{i in A, j in B} |C_ij|^2 for disjoint site lists A and B (ascending), i.e. minus
 * the covariance of the particle numbers of A and B; G_host[t] per trajectory.  Computed
 * from C_AB = U_A U_B^+ on the matrix cores with |C_ij|^2 summed in the product's epilogue.
 * Allocates a buffer on first use.  Synchronises.
 * Errors: MFQ_EINVAL (overlapping or invalid regions, NULL output), MFQ_ESTATE, MFQ_ENOMEM,
 * MFQ_EDEVICE. */
mfq_status mfq_particle_covariance(mfq_ctx *ctx, const int32_t *A, int32_t nA, const int32_t *B,
                                   int32_t nB, double *G_host);

/* Born probabilities <n_i> = sum_k |U_ik|^2 of the current state (Appendix A):
 * p_host[t * L + i], caller-owned.  Synchronises. */
mfq_status mfq_occupations(mfq_ctx *ctx, double *p_host);

/* Projective measurements made by the most recent step: for trajectory t,
 * counts[t] events (at most max_events are copied), event e at index
 * t * max_events + e: site, outcome (0/1) and conditional Born probability.
 * Any of the three output arrays may be NULL.  Synchronises. */
mfq_status mfq_pm_events(mfq_ctx *ctx, int32_t max_events, int32_t *counts, int32_t *sites,
                         int32_t *outcomes, double *probs);

/* Continuous-time projective protocol (Appendix A, PM protocol with Poisson waiting times).
 * Runs n_events event slots.  In each slot every trajectory t whose clock is below t_end
 * takes one event:
 *   tau = -ln(eta) / (gamma[t] N), eta uniform in (0, 1), N the particle number (the total
 *     event rate is gamma N, the per-site rate gamma N / L); the clock advances by tau;
 *   U <- exp(-i Ht tau) U, exact for every tau: the ring row of Bessel terms
 *     (-i)^|n| J_|n|(2 J tau) kept while above 1e-20 of the largest (or, when the band
 *     would wrap, the full row from its plane-wave sum); on the torus P_y (x) P_x;
 *   a site j uniform over the L sites, p_j = <n_j>, outcome 1 iff p_c <= p_j with p_c
 *     uniform, and the exact projection of the Slater determinant (Eq. (A1); Eq. (A2)
 *     with the sign of its rank-1 term corrected).
 * Trajectories whose clock has reached t_end (t_end = +inf: never) keep their state.
 * Random numbers: Philox4x64-10, key (seed, uid), counter (n, 0, 2, 0) with n the
 * trajectory's own step index (shared with mfq_step; each slot advances it by one);
 * word 0 -> eta, word 1 -> j = high 64 bits of word1 * L, word 2 -> p_c.
 * gamma: n_traj host doubles, each > 0.  reorth_every = R > 0: both Cholesky-QR passes
 * after every slot whose absolute step index is a multiple of R (0: never; each event
 * is exactly unitary up to rounding).  Asynchronous (stream-ordered).
 * Errors: MFQ_EINVAL (gamma NULL or not positive and finite, n_events < 0, t_end NaN,
 * reorth_every < 0), MFQ_ESTATE, MFQ_EDEVICE. */
mfq_status mfq_ct_events(mfq_ctx *ctx, const double *gamma, uint64_t seed, int32_t n_events,
                         double t_end, int32_t reorth_every);

/* Deferred events: with block = K in 1 .. 64, mfq_ct_events keeps up to
 * K consecutive events of every trajectory in factored form -- each event taken back to the
 * block's start, where its projection is a rank-2 right factor of U plus a rank-1 term
 * (Eq. (A1) / Eq. (A2) on U) -- and applies the block with two batched matrix products and one
 * band propagation exp(-i Ht s) over the block's time s (on the torus its two ring factors).  The events (sites, outcomes, Born
 * probabilities, waiting times) are those of the event-by-event form and the state agrees with
 * it to rounding.  A block is applied when full, before a scheduled Cholesky-QR and at the end
 * of every call.  block = 0 (default): event by event.
 * Needs (5 N + 3 L) K complex doubles per trajectory, allocated by the first blocked call.
 * Errors: MFQ_EINVAL (block outside 0 .. 64); the first blocked call may return MFQ_ENOMEM. */
mfq_status mfq_set_ct_block(mfq_ctx *ctx, int32_t block);

/* Record of the latest event slot of mfq_ct_events, per trajectory t (host arrays of
 * n_traj entries, any may be NULL): measured site, outcome (0/1), Born probability p_j
 * and waiting time tau; site = outcome = -1 and p = tau = 0 where the trajectory took
 * no event (or no slot has run since mfq_init_state).  Synchronises. */
mfq_status mfq_ct_last_events(mfq_ctx *ctx, int32_t *site, int32_t *outcome, double *prob,
                              double *tau);

/* Clocks of the continuous-time protocol (t_host: n_traj host doubles).  They start at 0
 * in mfq_init_state and mfq_reset_trajectory and advance only in mfq_ct_events.
 * mfq_set_times restores them (finite values) with a checkpoint.  Both synchronise.
 * Errors: MFQ_EINVAL (NULL, non-finite), MFQ_ESTATE, MFQ_EDEVICE. */
mfq_status mfq_get_times(mfq_ctx *ctx, double *t_host);
mfq_status mfq_set_times(mfq_ctx *ctx, const double *t_host);

/* Checkpoint: copy the current U of all trajectories (L*N*n_traj complex
 * doubles, layout as above) to host memory and report the absolute step
 * index.  Synchronises. */
mfq_status mfq_get_state(mfq_ctx *ctx, void *U_host, int64_t *step);

/* Restore a checkpoint written by mfq_get_state (same problem shape).
 * Columns must be orthonormal for the physics to hold; the library does not
 * re-orthonormalise on load. */
mfq_status mfq_set_state(mfq_ctx *ctx, const void *U_host, int64_t step);

/* The rest of a checkpoint of trajectories admitted by mfq_reset_trajectory: per trajectory
 * its uid (which keys its random numbers) and the context step at which its own step count
 * restarted (its Philox step counter is the context step minus this base).  Host arrays of
 * n_traj entries.  mfq_set_slots restores them after mfq_set_state (bases within
 * [0, the context's step]), so that a resumed context draws exactly what the uninterrupted one
 * would.  Both synchronise.  Errors: MFQ_EINVAL (NULL, base out of range), MFQ_ESTATE,
 * MFQ_EDEVICE. */
mfq_status mfq_get_slots(mfq_ctx *ctx, uint64_t *uid_host, int64_t *step_base_host);
mfq_status mfq_set_slots(mfq_ctx *ctx, const uint64_t *uid_host, const int64_t *step_base_host);

/* Wait for all work on the context's stream; reports deferred numeric errors
 * (MFQ_ENUMERIC) and clears them. */
mfq_status mfq_synchronize(mfq_ctx *ctx);

/* Run n_steps steps (as mfq_step) and record S_A of one region after every
 * step whose absolute index is a multiple of obs_every (0: no observation).
 * S_host receives n_obs x n_traj doubles, observation-major, where *n_obs_out
 * = number of such steps in the run.  Execution path (mfq_set_path): on the
 * fused path one workgroup per trajectory runs every step and observation
 * with its state in LDS, in a single launch (lattices whose state, Gram and
 * factor fit in a compute unit's LDS, e.g. L = 64); otherwise the per-phase
 * kernels run (graph-replayed) with the entropy pipeline on schedule.  Both
 * paths use the same random numbers.  Synchronises. */
mfq_status mfq_run(mfq_ctx *ctx, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                   int32_t n_steps, int32_t obs_every, const int32_t *region, int32_t n_sites,
                   double *S_host, int32_t *n_obs_out);

/* Several contexts advanced together (execution form: trajectories of uneven lattices,
 * protocols and monitoring rates batched into one launch or one graph).
 * ctx[k] runs args[k].n_steps steps of its own protocol, gamma (n_traj host doubles), dt and
 * seed, with S of its own region observed after every step whose absolute index is a
 * multiple of obs_every (0: none) into args[k].S_host (n_obs x n_traj doubles, observation-
 * major; args[k].n_obs is set on return).  1 <= n <= 8 distinct contexts on one device.
 * When every context fits the fused path (split-step integrator): ONE launch of the fused
 * kernel, each workgroup finding its context in a table and running one trajectory with its
 * state in LDS, exactly as mfq_run on the fused path does (same random numbers, same
 * results), enqueued on ctx[0]'s stream after the work already queued on the others' streams.
 * Otherwise every context takes its per-phase kernels: ONE graph holds two steps of every
 * context, each context on a parallel branch, and is replayed while all of them have two
 * steps left before their next observation or their end; the other steps run per context on
 * its own stream.  The results equal mfq_run of each context alone (same kernels, same random
 * numbers).  This form needs steps that a graph can hold: no blocked projective measurement
 * (mfq_set_pm_path), graphs enabled and profiling off.  The call synchronises.
 * Errors: MFQ_EINVAL (as mfq_run, too many or repeated contexts, different devices, steps a
 * graph cannot hold), MFQ_ESTATE, MFQ_ENUMERIC (per context, the first one reported),
 * MFQ_ENOMEM (RK4 scratch), MFQ_EDEVICE. */
typedef struct {
  int32_t protocol;
  const double *gamma;
  double dt;
  uint64_t seed;
  int32_t n_steps;
  int32_t obs_every;
  const int32_t *region;
  int32_t n_sites;
  double *S_host;
  int32_t n_obs; /* out */
} mfq_run_args;
mfq_status mfq_run_group(mfq_ctx *const *ctx, mfq_run_args *args, int32_t n);

/* Integrator of homodyne steps (mfq_step, mfq_run, Appendix A, Eq. (A4)).
 * MFQ_INTEGRATOR_SPLIT (default): U <- P U with the exact propagator P = exp(-i Ht dt), then
 *   each row scaled by exp(dW_i + (2 p_i - 1) gamma dt) with p of the propagated U.
 * MFQ_INTEGRATOR_RK4: the paper's fourth-order Runge-Kutta step of Eq. (A4) with its exponent
 *   A = -i Ht dt + diag(dW + (2 p - 1) gamma dt) frozen over the step (p of the state entering
 *   the step, the same normals dW_i = sqrt(gamma dt) z_i): U <- U + (k1 + 2 k2 + 2 k3 + k4)/6,
 *   evaluated as the degree-4 Taylor polynomial of exp(A) in Horner form, four nearest-
 *   neighbour passes over U and no L x L propagator.  Needs a third state buffer
 *   (16 L N n_traj bytes), allocated by the first RK4 step.  The fused path integrates by
 *   split step only, so mfq_run takes the per-phase kernels under RK4.
 * Projective steps are unaffected.  Errors: MFQ_EINVAL (unknown integrator); the first RK4
 * step may return MFQ_ENOMEM. */
#define MFQ_INTEGRATOR_SPLIT 0
#define MFQ_INTEGRATOR_RK4 1
mfq_status mfq_set_integrator(mfq_ctx *ctx, int32_t integrator);

/* Form in which exp(-i Ht dt) is applied (Appendix A free evolution).
 *   MFQ_PROP_DENSE     the dense L x L propagator as one GEMM over the batch (default; FP32
 *                      planes with MFQ_FP32_BULK);
 *   MFQ_PROP_FACTORED  on a ring, a banded stencil of the generating row: entries beyond the
 *                      band are below 1e-20 of the largest, so the result equals the dense
 *                      product to rounding (band <= 128 and narrower than the ring, else the
 *                      dense form is used); on a torus, the exact factors P = P_y (x) P_x
 *                      applied as two GEMMs (P U = vec(P_x X P_y) per column, X the Lx x Ly
 *                      view).  Always FP64.
 * mfq_propagator_band reports the ring band w (taps -w..w; -1: none narrower than the ring,
 * -2: torus) for the dt of the most recent step. */
#define MFQ_PROP_DENSE 0
#define MFQ_PROP_FACTORED 1
mfq_status mfq_set_propagator(mfq_ctx *ctx, int32_t form);
mfq_status mfq_propagator_band(mfq_ctx *ctx, int32_t *band);

/* How projective measurements of a step are carried out (Appendix A, Eq. (A1),
 * Eq. (A2) sign-corrected).  Both forms give the same outcomes and
 * conditional probabilities from the same random numbers, and the same state
 * up to the choice of orthonormal basis of its orbital space.
 *   MFQ_PM_WORKGROUP  one workgroup per trajectory projects the measured
 *                     sites one after another (each a pass over U);
 *   MFQ_PM_BLOCKED    the outcomes are drawn from C_MM = U_M U_M^+ of the
 *                     measured sites M by sequential elimination, then U is
 *                     updated at once: LQ of the outcome-1 rows and a
 *                     compact-WY product on the matrix cores.  The host reads
 *                     the per-step counts (two stream synchronisations per
 *                     step; such steps are not graph-replayed).  Needs N >= 128
 *                     and at most N measured sites in a step, else the step
 *                     falls back to the workgroup form;
 *   MFQ_PM_AUTO       blocked for N >= 128, workgroup below (default). */
#define MFQ_PM_AUTO 0
#define MFQ_PM_WORKGROUP 1
#define MFQ_PM_BLOCKED 2
mfq_status mfq_set_pm_path(mfq_ctx *ctx, int32_t path);

/* Form of the Householder reduction to tridiagonal form inside the entropy, spectrum and
 * mutual-information calls (the eigenvalues of C_A, Sec. II entropy formula).  Same
 * eigenvalues to rounding either way:
 *   MFQ_EIG_ONE_STAGE  one reflector at a time on the dense Gram (in LDS for small orders,
 *                      otherwise grid-wide sweeps or panels of 32 reflectors that read the
 *                      trailing matrix once per reflector);
 *   MFQ_EIG_TWO_STAGE  dense -> band of half-width 32 by block reflectors whose two-sided
 *                      updates are matrix-core products on the lower triangle (the column
 *                      steps of a panel in one kernel whose workgroups wait on each other;
 *                      such kernels of several streams are admitted only while they fit the
 *                      GPU together), then band -> tridiagonal by bulge chasing in a
 *                      persistent kernel whose workgroups wait on each other through progress
 *                      words (any wait beyond 10 s makes the call return MFQ_EDEVICE); used
 *                      for orders >= 66 where the Rinv region holds its storage (about
 *                      n^2 / 8 + 160 n complex entries per trajectory for n >= 512, 19077 at
 *                      n = 66), else one stage;
 *   MFQ_EIG_AUTO       two stages from order 4096 on, one below (default; measured on the
 *                      MI355X, two stages are faster from about that order). */
#define MFQ_EIG_AUTO 0
#define MFQ_EIG_ONE_STAGE 1
#define MFQ_EIG_TWO_STAGE 2
mfq_status mfq_set_eig_path(mfq_ctx *ctx, int32_t path);

/* GEMM tile choice of a context (all its contractions, the propagator included). */
#define MFQ_TILE_AUTO 0   /* 128 x 128 tiles for large contractions, 64 x 64 otherwise */
#define MFQ_TILE_SMALL 1  /* always 64 x 64 (4 waves) */
#define MFQ_TILE_LARGE 2  /* 128 x 128 (8 waves) whenever every dimension is >= 128 */

/* Workgroup -> tile order of the GEMMs (mfq_set_tile_order): XCD groups all tiles of one
 * batch entry (or one column panel of a single wide product) on one XCD so that they share
 * its L2; LINEAR hands tile i to workgroup i.  Results are bitwise the same either way. */
#define MFQ_ORDER_XCD 0
#define MFQ_ORDER_LINEAR 1

#define MFQ_TUNE_MAX_CANDIDATES 16

/* Result of mfq_autotune. */
typedef struct {
  int32_t path;             /* chosen mfq_run path: MFQ_PATH_FUSED or MFQ_PATH_LAUNCHES */
  int32_t tile;             /* chosen MFQ_TILE_* */
  double ms_per_step;       /* wall time per step of the chosen configuration */
  int32_t n_candidates;     /* entries used in the candidate arrays */
  int32_t order;            /* chosen MFQ_ORDER_* */
  int32_t pm_path;          /* chosen MFQ_PM_* (the context's setting when not searched) */
  int32_t reserved;
  double candidate_ms[MFQ_TUNE_MAX_CANDIDATES];   /* ms per step of each candidate probed */
  int32_t cand_path[MFQ_TUNE_MAX_CANDIDATES];     /* its path, */
  int32_t cand_tile[MFQ_TUNE_MAX_CANDIDATES];     /* tile, */
  int32_t cand_order[MFQ_TUNE_MAX_CANDIDATES];    /* tile order */
  int32_t cand_pm[MFQ_TUNE_MAX_CANDIDATES];       /* and projective form */
} mfq_tuning;

/* Autotuner of the execution form of a step (the batched launch of the hot
 * path): times probe_steps steps of the given protocol and parameters under
 * each candidate, after one warm-up run (a candidate whose warm-up takes ten
 * times the best time so far is not timed again), coordinate by coordinate:
 * for projective steps with N >= 128 the measurement form (blocked or one
 * workgroup per trajectory), then with that form every GEMM tile size (AUTO,
 * SMALL, LARGE) in both tile orders (MFQ_ORDER_*), then the fused
 * LDS-resident kernel when the problem fits.  The fastest becomes the
 * context's path (for mfq_run), tile size and order (for every call) and
 * projective form.  The state, the step index and the events of the last step
 * are saved before and restored after the probes, so tuning does not change
 * any trajectory.  Allocates a temporary device copy of the state.
 * Synchronises.  Errors: MFQ_EINVAL, MFQ_ESTATE, MFQ_ENOMEM / MFQ_EDEVICE, or
 * the first error a probe reports (the previous choice is then kept). */
mfq_status mfq_autotune(mfq_ctx *ctx, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                        int32_t probe_steps, mfq_tuning *out);

/* Tile order of the context's GEMMs (MFQ_ORDER_XCD default, or MFQ_ORDER_LINEAR).
 * Errors: MFQ_EINVAL for another value. */
mfq_status mfq_set_tile_order(mfq_ctx *ctx, int32_t order);

/* Apply a previously tuned choice (e.g. from a cache) without probing. */
mfq_status mfq_set_tuning(mfq_ctx *ctx, int32_t path, int32_t tile);

#define MFQ_PATH_AUTO 0     /* fused when the problem fits in LDS, else per-phase kernels */
#define MFQ_PATH_FUSED 1    /* force the fused single-launch path (MFQ_EINVAL if it does not fit) */
#define MFQ_PATH_LAUNCHES 2 /* force the per-phase kernels */
mfq_status mfq_set_path(mfq_ctx *ctx, int32_t path);

/* Continuous batching: put trajectory `slot` back into the initial state of
 * mfq_init_state with a new uid, without touching the other trajectories.
 * Its own step index restarts at 0 (its random numbers are those of a fresh
 * trajectory with this uid: counter step = context step - step at reset).
 * Stream-ordered, asynchronous. */
mfq_status mfq_reset_trajectory(mfq_ctx *ctx, int32_t slot, uint64_t uid);

/* Multi-step calls (n_steps >= 2) replay a captured HIP graph of two steps
 * (default on; off while phase timing is enabled).  enable = 0 launches every
 * kernel directly.  Results are identical either way. */
mfq_status mfq_use_graphs(mfq_ctx *ctx, int32_t enable);

/* Phase timing with HIP events recorded on the context's stream around each
 * phase of a step (no extra synchronisation while enabled). */
#define MFQ_PHASE_PROPAGATE 0 /* propagator GEMM U <- P U: exactly one kernel launch per step */
#define MFQ_PHASE_MEASURE 1   /* Born probabilities + homodyne factor, or projective measurement */
#define MFQ_PHASE_REORTH 2    /* both Cholesky-QR passes */
#define MFQ_PHASE_OBSERVE 3   /* region Gram, tridiagonalisation, bisection, entropy */
#define MFQ_NPHASES 4

/* enable != 0 starts timing (and clears accumulated times); 0 stops it. */
mfq_status mfq_profile(mfq_ctx *ctx, int32_t enable);

/* Accumulated milliseconds and number of timed intervals per phase since
 * timing was enabled; ms and count are host arrays of MFQ_NPHASES entries
 * (either may be NULL).  Synchronises. */
mfq_status mfq_phase_times(mfq_ctx *ctx, double *ms, int64_t *count);

/* ------------------------------------------------------------------------
 * Serving engine: continuous batching of trajectory jobs of different
 * lattices, sizes and protocols on one device.  A worker thread admits queued
 * jobs into batch groups (one context per shape = lattice, N, protocol,
 * precision, dt, seed) by device-memory footprint, refills slots as jobs
 * finish while the other slots keep running, and runs the groups' steps on
 * separate streams so that they overlap on the device.  Every job starts
 * from the Neel / checkerboard state (N = L/2) and keeps its own random
 * numbers (key (seed, uid), counter = its own step index), so its result is
 * the same alone and in any mix.
 * ------------------------------------------------------------------------ */
typedef struct mfq_engine mfq_engine;

typedef struct {
  mfq_lattice lat;
  int32_t N;          /* 0 or L/2 */
  int32_t protocol;   /* MFQ_PROJECTIVE or MFQ_HOMODYNE */
  int32_t precision;  /* MFQ_FP64 or MFQ_FP32_BULK */
  int32_t n_steps;    /* >= 1 */
  int32_t obs_every;  /* S of `region` after every obs_every-th step of the job; 0: after the last */
  int32_t n_region;
  double gamma;       /* monitoring rate, >= 0 */
  double dt;          /* > 0 */
  uint64_t seed;
  uint64_t uid;       /* keys the job's random numbers */
  const int32_t *region;  /* n_region ascending site ids, copied at submission */
} mfq_job;

typedef struct {
  uint64_t bytes_in_use;  /* device memory held by the engine's batch groups */
  uint64_t peak_bytes;
  uint64_t budget_bytes;
  int64_t queued;         /* jobs waiting for a slot or for memory */
  int32_t groups;         /* live batch groups */
  int32_t reserved;
} mfq_engine_stats_t;

/* Start an engine on `device` that keeps at most hbm_budget_bytes of device
 * workspace (0: 64 GiB) and at most max_slots trajectories per batch group. */
mfq_status mfq_engine_create(int device, size_t hbm_budget_bytes, int32_t max_slots, mfq_engine **out);
/* Stop the worker (running jobs are abandoned) and free everything. */
mfq_status mfq_engine_destroy(mfq_engine *engine);
const char *mfq_engine_last_error(const mfq_engine *engine);
/* Queue a job (non-blocking); *job_id identifies it.  A job whose footprint
 * alone exceeds the budget fails (poll returns MFQ_ENOMEM). */
mfq_status mfq_engine_submit(mfq_engine *engine, const mfq_job *job, uint64_t *job_id);
/* MFQ_PENDING (1) until the job is done; then copies up to max_obs entropies
 * (in order of observation) to S_host, their number to *n_obs and the time
 * from submission to completion to *latency_s (any output may be NULL). */
mfq_status mfq_engine_poll(mfq_engine *engine, uint64_t job_id, double *S_host, int32_t max_obs,
                           int32_t *n_obs, double *latency_s);
/* Block until the job is done (MFQ_OK), failed (its error) or timeout_s
 * elapsed (MFQ_PENDING). */
mfq_status mfq_engine_wait(mfq_engine *engine, uint64_t job_id, double timeout_s);
mfq_status mfq_engine_stats(mfq_engine *engine, mfq_engine_stats_t *out);

#ifdef __cplusplus
}
#endif

#endif /* MFQ_H */
