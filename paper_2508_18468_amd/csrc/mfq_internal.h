// Internal declarations shared by the HIP translation units of libmfq.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "cplx.h"
#include "workspace_layout.h"

namespace mfq {

// ---------------------------------------------------------------- batched complex GEMM
// D[b] = alpha * op(A[b]) * op(B[b]) + beta * Cin[b], column-major, complex FP64.
// op = 0: as stored; op = 2: conjugate transpose.  Storage row indices of A and
// B may be gathered through idxA / idxB (applied to the stored matrix rows).
enum { OP_N = 0, OP_C = 2 };
enum { TRI_NONE = 0, TRI_UPPER = 1, TRI_LOWER = 2 };

struct GemmDesc {
  int M, N, K, batch;
  const cplx *A; long lda, sA; const int *idxA; int opA;
  const cplx *B; long ldb, sB; const int *idxB; int opB;
  const cplx *Cin; long ldcin, sCin;
  cplx *D; long ldd, sD;
  cplx alpha, beta;        // beta == 0 -> Cin is not read
  int tri;                 // TRI_UPPER / TRI_LOWER: only the tiles touching that triangle of D
                           // (TRI_LOWER writes its entries on and below the diagonal only)
  int aUpper;              // op(A) is upper triangular: A[m][k] taken as 0 for k < m (not read);
                           // 2: strictly upper (also 0 for k == m)
  int bUpper;              // op(B) is upper triangular: B[k][n] taken as 0 for k > n (not read)
  int aLower;              // op(A) is lower triangular: A[m][k] taken as 0 for k > m (not read)
  // Global K index of this launch's K index 0 for the triangular masks (products split over K):
  // kofs, plus kofs2 for each step of the second batch index (see batch2).  kend_glob > 0: the
  // global K range ends there (a split whose last slice is shorter than K).
  int kofs, kofs2, kend_glob;
  const double *skip_if_le;  // if set and *skip_if_le <= skip_thr, the launch does nothing
  double skip_thr;
  long sIdxA, sIdxB;       // batch stride of idxA / idxB (0: one index list for all entries)
  // Near-identity epilogue of an upper Gram (square, TRI_UPPER, alpha = 1, beta = 0): with
  // E = D - I, also writes the upper triangle of R1 = I - triu(E, 1) - diag(E)/2 (ld and
  // batch stride as D) and raises *maxdev to max |Re E|+|Im E| (a NaN or an infinity
  // raises it to NaN).  *maxdev must be zeroed beforehand.
  cplx *R1;
  double *maxdev;
  // Reduction epilogues (D is then not written): with part set, a TRI_UPPER square product
  // stores per tile the sums of |D_ij|^2 (i < j) along each diagonal j - i, a general one
  // stores per tile the sum of |D_ij|^2 (see zgemm_partials, zgemm_ring_bins, zgemm_tile_sum).
  double *part;
  // Two batch dimensions: with batch2 > 1, entry b of the batch is (b / batch2, b % batch2)
  // and its operands sit at X + (b / batch2) sX + (b % batch2) sX2 (batch2 <= 1: X + b sX).
  int batch2;
  long sA2, sB2, sD2, sCin2;
  // Workgroup -> tile order, set by zgemm from the calling thread's choice
  // (set_gemm_tile_order): 0 XCD-grouped, 1 plain linear.
  int linear_order;
  // Nonzero: large tiles are allowed from K = 64 on (rank-64 updates of a large result).
  int short_k_large;
};

hipError_t zgemm(const GemmDesc &g, hipStream_t s);
// Tile choice for the GEMMs launched by the calling thread: AUTO (64 x 64 unless every
// dimension is >= 128 and the work fills the chip), SMALL (always 64 x 64, the propagator
// included), LARGE (128 x 128 whenever every dimension is >= 128).  Set by the context
// around its launches from its tuned choice.
enum { GEMM_TILE_AUTO = 0, GEMM_TILE_SMALL = 1, GEMM_TILE_LARGE = 2 };
void set_gemm_tile_mode(int mode);
int gemm_tile_mode();
// Order in which the workgroups of a GEMM walk its tiles, for the calling thread:
// XCD (all tiles of one batch entry, or one column panel, on one XCD and its L2) or
// LINEAR (tile index = workgroup index).  Results are bitwise the same either way.
enum { GEMM_ORDER_XCD = 0, GEMM_ORDER_LINEAR = 1 };
void set_gemm_tile_order(int order);
int gemm_tile_order();
// Doubles of partial results that a reduction-epilogue product g writes (0 if none).
size_t zgemm_partials(const GemmDesc &g);
// From the diagonal partials of the upper product C = U U^+ (M = N = L): for every batch entry
// and ring distance r = 1 .. L/2, out[b * (L/2) + r - 1] = C(r) = -(sum over ordered pairs
// i != j at ring distance r of |C_ij|^2) / (their number).  Launches the product as well.
hipError_t zgemm_ring_bins(const GemmDesc &g, int L, double *out, hipStream_t s);
// Launches the product and sums its tile partials per batch entry: out[b] = sum |D_ij|^2.
hipError_t zgemm_tile_sum(const GemmDesc &g, double *out, hipStream_t s);
// Same contraction (op N, op N), launched under a distinct kernel name.
hipError_t zgemm_propagator(const GemmDesc &g, hipStream_t s);

// FP32-bulk propagator U' = U + (P - I) U: planes of P - I in FP32, product on
// the FP32 matrix cores, identity term and output in FP64.  U and D are
// column-major L x ncols (ld = L) and must not overlap.
hipError_t make_delta_planes(const cplx *P, float *Pr, float *Pi, int L, hipStream_t s);
hipError_t propagator_delta_f32(const float *Pr, const float *Pi, const cplx *U, cplx *D, int L,
                                int ncols, hipStream_t s);

// ---------------------------------------------------------------- state kernels
hipError_t expand_propagator(cplx *P, const cplx *gx, const cplx *gy, int dim, int Lx, int Ly,
                             hipStream_t s);
hipError_t init_state(cplx *U, int L, int N, int B, const int *occ, hipStream_t s);
// D = P U for the ring propagator P_ab = g[(a - b) mod L] truncated to |a - b| <= w (band);
// U and D are column-major L x ncols and must not overlap; 2 w + 1 <= L, w <= 128.
hipError_t ring_stencil(const cplx *U, cplx *D, const cplx *g, int L, int w, long ncols, hipStream_t s);
// The absolute step index n of a step is read on the device as *step_ptr + step_offset,
// so that a captured graph of steps can be replayed unchanged.
hipError_t set_step(int64_t *step_ptr, int64_t value, bool add, hipStream_t s);
// step_base[b] (per trajectory) is subtracted: trajectory b's own step index is
// *step_ptr + step_offset - step_base[b].
hipError_t born_homodyne(cplx *U, double *p, int L, int N, int B, const double *gamma, double dt,
                         uint64_t seed, const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                         const int64_t *step_base, hipStream_t s);
hipError_t reset_slot(cplx *U, int L, int N, int slot, const int *occ, uint64_t *uid, uint64_t new_uid,
                      int64_t *step_base, int64_t base, hipStream_t s);
hipError_t born_only(const cplx *U, double *p, int L, int N, int B, hipStream_t s);
hipError_t pm_measure(cplx *U, int L, int N, int B, const double *gamma, double dt, uint64_t seed,
                      const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                      const int64_t *step_base, int *sites, int *outcomes, double *probs, int *counts,
                      cplx *vbuf, cplx *wbuf, hipStream_t s);
hipError_t fill_zero(void *p, size_t bytes, hipStream_t s);

// Blocked projective measurement for large lattices (selection, conditional
// outcomes from C_MM, LQ of the outcome-1 rows, compact-WY update of U).
struct PmBlockedWork {
  int *sites, *outcomes, *counts;  // L, L, 1 per trajectory (the events of the step)
  double *probs, *udraw, *tau;     // L per trajectory
  int *m1, *k1, *code;             // L, 1, L per trajectory
  cplx *G, *R;                     // N x N per trajectory (free during the measurement)
  cplx *T;                         // N x 64 per trajectory
};
// U: L x N per trajectory (updated in place); scratch: L x N per trajectory.
// Synchronises the stream twice (the host sizes the launches by the counts).
// *fallback is set, with U untouched, when the step cannot be done in this
// form (more measured sites than N, or N < 128); the caller then measures
// with pm_measure.
hipError_t pm_blocked(cplx *U, cplx *scratch, int L, int N, int B, const double *gamma, double dt,
                      uint64_t seed, const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                      const int64_t *step_base, const PmBlockedWork &w, bool *fallback,
                      hipStream_t s);
// Smallest N for the blocked form (the Gram and T factor of a 64-wide WY block share
// one N x N scratch).
constexpr int PM_BLOCKED_MIN_N = 128;

// ---------------------------------------------------------------- continuous-time protocol
// Appendix A, PM protocol with Poisson waiting times: one event per active
// trajectory (clock t < t_end) per call of cont_event.
struct ContWork {
  double *t;      // B: clock of each trajectory
  cplx *g;        // B x (Lx + Ly): ring rows of P(tau), x row at 0, y row at Lx (1d: Ly = 1)
  double *jn;     // B x jcap: Bessel-recurrence scratch
  int *info;      // B x 4: site j, outcome, band x, band y of the last event (band x < 0: none)
  double *dinfo;  // B x 4: tau, p_j, tau of the reflector, unused
  cplx *v;        // B x N: reflector vector
  cplx *y;        // B x L: tau_h U v
  cplx *yp;       // B x L: P(tau) y
  int jcap;
};
hipError_t cont_clock_set(double *t, int first, int count, double value, hipStream_t s);
// One event on every trajectory whose clock is below t_end.  Ua holds the state;
// the result lands in Ub on the ring (*state_in_b = true) and back in Ua on the
// torus.  The event index of trajectory b is *step_ptr + step_offset - step_base[b].
hipError_t cont_event(cplx *Ua, cplx *Ub, int L, int N, int B, int dim, int Lx, int Ly, double J,
                      const double *gamma, double t_end, uint64_t seed, const uint64_t *uid,
                      const int64_t *step_ptr, int step_offset, const int64_t *step_base,
                      const ContWork &w, bool *state_in_b, hipStream_t s);

// Deferred events on the ring: blocks of up to K (<= 64) events kept in factored form
// (V = V0 (I + WL WR^+) + G Z, taken back to the block's start) and applied by cont_block_flush.
struct BlockWork {
  cplx *WL, *WR;  // N x 2K per trajectory
  cplx *Zc;       // N x K per trajectory (conj(Z)^T)
  cplx *G;        // L x K per trajectory
  cplx *T1;       // L x 2K per trajectory (flush scratch)
  double *s;      // B: time since the block's start
  int *fb;        // 2 per trajectory: bands of P(s) along x and y at the flush
  int K;
};
// Event e (0-based) of the current block for every trajectory with clock below t_end; U (the
// state at the block's start) is only read.
hipError_t cont_block_event(const cplx *U, int L, int N, int B, int e, int dim, int Lx, int Ly, double J,
                            const double *gamma, double t_end, uint64_t seed, const uint64_t *uid, const int64_t *step_ptr,
                            int step_offset, const int64_t *step_base, const ContWork &w, const BlockWork &bw,
                            hipStream_t s);
// Apply the block's e events: Ua (block start) is overwritten by V, then U = P(s) V lands in Ub
// on the ring (*state_in_b = true) and back in Ua on the torus.
hipError_t cont_block_flush(cplx *Ua, cplx *Ub, int L, int N, int B, int e, int dim, int Lx, int Ly, double J,
                            const ContWork &w, const BlockWork &bw, bool *state_in_b, hipStream_t s);

// ---------------------------------------------------------------- RK4 homodyne step
// Appendix A: the homodyne step with Eq. (A4)'s exponent frozen over the step and
// integrated by RK4 (the degree-4 Taylor polynomial of exp(A), in Horner form).
// U (L x N per trajectory) is updated in place; p holds the Born probabilities of U;
// V1, V2 (L x N per trajectory) and a (L per trajectory) are scratch.
hipError_t rk4_homodyne(cplx *U, cplx *V1, cplx *V2, const double *p, double *a, int L, int N, int B, int dim,
                        int Lx, int Ly, double J, const double *gamma, double dt, uint64_t seed,
                        const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                        const int64_t *step_base, hipStream_t s);

// ---------------------------------------------------------------- Cholesky-QR
struct CholWork {
  cplx *G;              // N x N per trajectory (upper triangle used)
  cplx *Rinv;           // N x N per trajectory
  cplx *T;              // N x NB per trajectory
  int *flag;            // device error flag
  BreakdownInfo *info;  // where the first breakdown was seen (set with the flag)
  double *dev;          // device scalar: max |G - I| of the latest near-identity check
};
// Largest |U^+ U - I| entry for which the second pass uses the first-order factor.
constexpr double CHOL_FIRST_ORDER_MAX = 1e-8;
// Largest |U^+ U - I| entry for which the second pass keeps U as it is: the first pass
// already delivered an orthonormal basis to that accuracy, which the second pass's own
// rounding (about L eps per entry of the Gram) would not improve on.
constexpr double CHOL_KEEP_MAX = 1e-13;
// Cholesky-QR2 of the L x N matrices U (batch B): the orthonormal factor ends in T, and U
// is overwritten (scratch).  Pass 1: T = U R^{-1}, R = chol(U^+ U).  Pass 2 tests the Gram
// of T against I on the device: max |G - I| <= CHOL_KEEP_MAX keeps T as it is (the pass's
// launches exit at once); otherwise R^{-1} = I - triu(E) + diag(E)/2 for E = G - I below
// CHOL_FIRST_ORDER_MAX (the Cholesky factor of I + E to O(|E|^2), i.e. to rounding), else
// the full factorisation, and T R^{-1} is formed in U and copied back into T.
hipError_t cholqr2(cplx *U, cplx *T, int L, int N, int B, const CholWork &w, hipStream_t s);

// ---------------------------------------------------------------- fused small-lattice path
struct FusedArgs {
  const cplx *P;
  const cplx *gx, *gy;      // generating rows of P: P = P_y (x) P_x (1d: gy = {1})
  int Lx, Ly;
  cplx *U;                  // L x N per trajectory, updated in place
  int L, N;
  const double *gamma;
  double dt;
  uint64_t seed;
  const uint64_t *uid;
  const int64_t *step_base; // per-trajectory step base (trajectory step = context step - base)
  int64_t step0;            // absolute index of the last completed step
  int n_steps, protocol;
  int obs_every;            // observe S after steps n with n % obs_every == 0 (0: never)
  const int *region;
  int nreg, max_obs;
  double *S_out;            // [obs][trajectory]
  int *ev_sites, *ev_out, *ev_cnt;  // projective events of the last step (L per trajectory)
  double *ev_prob;
  int *flag;
  BreakdownInfo *info;
  int B;                    // trajectories of this context (row length of S_out)
};
bool fused_fits(int L, int N, int Lx, int Ly);
size_t fused_lds_bytes(int L, int N, int Lx, int Ly);
hipError_t fused_run(const FusedArgs &a, int B, hipStream_t s);
// Several contexts (different lattices, protocols, rates and step counts) in one launch:
// workgroups first[k] .. first[k+1]-1 run the trajectories of ctx[k] with its own args.
constexpr int FUSED_GROUP_MAX = 8;
struct FusedGroup {
  int n;
  int first[FUSED_GROUP_MAX + 1];
  FusedArgs g[FUSED_GROUP_MAX];
};
hipError_t fused_run_group(const FusedGroup &grp, hipStream_t s);

// ---------------------------------------------------------------- eigen / entropy
struct EigWork {
  cplx *A;      // n x n per trajectory (Gram of the region)
  cplx *v;      // 2 n per trajectory: two Householder vector slots
  cplx *w;      // n per trajectory: w of the pending rank-2 update
  cplx *p;      // n per trajectory: A v of the newest reflector
  double *tau;  // 2 per trajectory: tau of the two reflector slots
  double *d, *e, *lam, *S;
  cplx *panel;        // blocked reductions: panel factors and partial sums (trd_panel_elems(n),
                      // trd2_scratch_elems(n))
  long panel_stride;  // between trajectories
  int *flag;                // the context's error word and breakdown record (a bulge-chase wait
  BreakdownInfo *info;      // beyond its limit is reported through them)
};
// The blocked Householder reduction (panel width TRD_NB, storage trd_panel_elems) takes
// batches of n >= TRD_BLOCKED_MIN with B n^2 >= TRD_BLOCKED_WORK (below that the per-reflector
// sweep, with fewer launches per column, is faster: launch latency rather than HBM traffic
// bounds the reduction there).
constexpr double TRD_BLOCKED_WORK = 16777216.0;
hipError_t region_gram(const cplx *U, int L, int N, int B, const int *region, int nreg, cplx *A,
                       int *n_out, hipStream_t s);
hipError_t tridiagonalize(const EigWork &w, int n, int B, hipStream_t s);
// Two-stage reduction (eig2.hip) of n x n Grams, n >= 2 TRD2_SB + 2, needing
// panel_stride >= trd2_scratch_elems(n); wait_ticks bounds each dependency wait of its bulge
// chase (wall-clock ticks).
hipError_t tridiagonalize_two_stage(const EigWork &w, int n, int B, long long wait_ticks, hipStream_t s);
// Reduction form of tridiagonalize for the calling thread: AUTO (by size), ONE_STAGE, TWO_STAGE
// (where it applies).  Set by the context around its launches.
enum { EIG_PATH_AUTO = 0, EIG_PATH_ONE_STAGE = 1, EIG_PATH_TWO_STAGE = 2 };
constexpr int TRD2_AUTO_MIN = 4096;  // AUTO takes the two-stage form from this order on
void set_eig_path(int mode);
int eig_path();
hipError_t bisect_eigvals(const EigWork &w, int n, int B, hipStream_t s);
hipError_t entropy_sum(const EigWork &w, int n, int B, hipStream_t s);

}  // namespace mfq
