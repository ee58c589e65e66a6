// Internal declarations shared by the HIP translation units of libmfq.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace mfq {

struct cplx {
  double re, im;
};

// ---------------------------------------------------------------- batched complex GEMM
// D[b] = alpha * op(A[b]) * op(B[b]) + beta * Cin[b], column-major, complex FP64.
// op = 0: as stored; op = 2: conjugate transpose.  Storage row indices of A and
// B may be gathered through idxA / idxB (applied to the stored matrix rows).
enum { OP_N = 0, OP_C = 2 };
enum { TRI_NONE = 0, TRI_UPPER = 1 };

struct GemmDesc {
  int M, N, K, batch;
  const cplx *A; long lda, sA; const int *idxA; int opA;
  const cplx *B; long ldb, sB; const int *idxB; int opB;
  const cplx *Cin; long ldcin, sCin;
  cplx *D; long ldd, sD;
  cplx alpha, beta;        // beta == 0 -> Cin is not read
  int tri;                 // TRI_UPPER: only tiles touching the upper triangle of D
  int aUpper;              // op(A) is upper triangular: A[m][k] = 0 for k < m
  int bUpper;              // op(B) is upper triangular: B[k][n] = 0 for k > n
  const double *skip_if_le;  // if set and *skip_if_le <= skip_thr, the launch does nothing
  double skip_thr;
};

hipError_t zgemm(const GemmDesc &g, hipStream_t s);
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
// The absolute step index n of a step is read on the device as *step_ptr + step_offset,
// so that a captured graph of steps can be replayed unchanged.
hipError_t set_step(int64_t *step_ptr, int64_t value, bool add, hipStream_t s);
hipError_t born_homodyne(cplx *U, double *p, int L, int N, int B, const double *gamma, double dt,
                         uint64_t seed, const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                         hipStream_t s);
hipError_t born_only(const cplx *U, double *p, int L, int N, int B, hipStream_t s);
hipError_t pm_measure(cplx *U, int L, int N, int B, const double *gamma, double dt, uint64_t seed,
                      const uint64_t *uid, const int64_t *step_ptr, int step_offset, int *sites,
                      int *outcomes, double *probs, int *counts, cplx *vbuf, cplx *wbuf, hipStream_t s);
hipError_t fill_zero(void *p, size_t bytes, hipStream_t s);

// ---------------------------------------------------------------- Cholesky-QR
struct CholWork {
  cplx *G;       // N x N per trajectory (upper triangle used)
  cplx *Rinv;    // N x N per trajectory
  cplx *T;       // N x NB per trajectory
  int *flag;     // device error flag
  double *dev;   // device scalar: max |G - I| of the latest near-identity check
};
constexpr int CHOL_NB = 64;
// Largest |U^+ U - I| entry for which the second pass uses the first-order factor.
constexpr double CHOL_FIRST_ORDER_MAX = 1e-8;
// One Cholesky-QR pass: Uout = Uin * R^{-1}, R = chol(Uin^+ Uin).  With
// near_identity, the Gram is first tested against I: if every entry of
// E = G - I is below CHOL_FIRST_ORDER_MAX, R^{-1} = I - triu(E) + diag(E)/2 (the
// Cholesky factor of I + E to O(|E|^2), i.e. to rounding); otherwise the full
// factorisation runs.  The choice is made on the device.
hipError_t cholqr_pass(const cplx *Uin, cplx *Uout, int L, int N, int B, const CholWork &w,
                       bool near_identity, hipStream_t s);

// ---------------------------------------------------------------- eigen / entropy
struct EigWork {
  cplx *A;      // n x n per trajectory (Gram of the region)
  cplx *v, *w;  // n per trajectory (Householder scratch)
  double *d, *e, *lam, *S;
};
hipError_t region_gram(const cplx *U, int L, int N, int B, const int *region, int nreg, cplx *A,
                       int *n_out, hipStream_t s);
hipError_t tridiagonalize(const EigWork &w, int n, int B, hipStream_t s);
hipError_t bisect_eigvals(const EigWork &w, int n, int B, hipStream_t s);
hipError_t entropy_sum(const EigWork &w, int n, int B, hipStream_t s);

}  // namespace mfq
