// Spectrum of the region correlation matrix and the entanglement entropy.
//
// S_A (Sec. II entropy formula) needs every eigenvalue of the Hermitian
// C_A = U_A U_A^+.  Pipeline: Gram of the region rows on the matrix cores
// (U_A^+ U_A instead when the region has more sites than particles: same
// nonzero spectrum), Householder reduction to a real symmetric tridiagonal
// (one workgroup per matrix; in LDS when it fits), Sturm-sequence bisection
// for all eigenvalues (one lane per eigenvalue), and the entropy sum with a
// fixed reduction order.
#include "device_common.h"

namespace mfq {

namespace {

constexpr int LDS_MAX_N = 88;  // 88 * 88 * 16 B = 121 KiB

__global__ __launch_bounds__(256) void tridiag_global_kernel(EigWork w, int n) {
  const int b = blockIdx.x;
  __shared__ double red[4];
  tridiag_body(w.A + (long)b * n * n, n, n, w.v + (long)b * n, w.w + (long)b * n,
               w.d + (long)b * n, w.e + (long)b * n, red);
}

__global__ __launch_bounds__(256) void tridiag_lds_kernel(EigWork w, int n) {
  const int b = blockIdx.x;
  __shared__ cplx As[LDS_MAX_N * LDS_MAX_N];
  __shared__ cplx vs[LDS_MAX_N], ps[LDS_MAX_N];
  __shared__ double red[4];
  const cplx *Ab = w.A + (long)b * n * n;
  for (int i = threadIdx.x; i < n * n; i += 256) As[i] = Ab[i];
  __syncthreads();
  tridiag_body(As, n, n, vs, ps, w.d + (long)b * n, w.e + (long)b * n, red);
}

// Eigenvalue k (ascending) of tridiagonal b (see bisect_eigenvalue).
__global__ __launch_bounds__(256) void bisect_kernel(EigWork w, int n) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  w.lam[(long)b * n + k] = bisect_eigenvalue(w.d + (long)b * n, w.e + (long)b * n, n, k);
}

// S = sum_k h(lambda_k), h(x) = -x ln x - (1 - x) ln(1 - x), lambda clamped to [0, 1].
__global__ __launch_bounds__(256) void entropy_kernel(EigWork w, int n) {
  const int b = blockIdx.x;
  __shared__ double red[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) s += binary_entropy(w.lam[(long)b * n + k]);
  s = block_sum256(s, red);
  if (threadIdx.x == 0) w.S[b] = s;
}

}  // namespace

hipError_t region_gram(const cplx *U, int L, int N, int B, const int *region, int nreg, cplx *A,
                       int *n_out, hipStream_t s) {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  g.batch = B;
  if (nreg <= N) {  // C_A = U_A U_A^+  (nreg x nreg)
    g.M = nreg; g.N = nreg; g.K = N;
    g.A = U; g.lda = L; g.sA = (long)L * N; g.opA = OP_N; g.idxA = region;
    g.B = U; g.ldb = L; g.sB = (long)L * N; g.opB = OP_C; g.idxB = region;
    g.D = A; g.ldd = nreg; g.sD = (long)nreg * nreg;
    *n_out = nreg;
  } else {          // U_A^+ U_A  (N x N), same nonzero eigenvalues
    g.M = N; g.N = N; g.K = nreg;
    g.A = U; g.lda = L; g.sA = (long)L * N; g.opA = OP_C; g.idxA = region;
    g.B = U; g.ldb = L; g.sB = (long)L * N; g.opB = OP_N; g.idxB = region;
    g.D = A; g.ldd = N; g.sD = (long)N * N;
    *n_out = N;
  }
  return zgemm(g, s);
}

hipError_t tridiagonalize(const EigWork &w, int n, int B, hipStream_t s) {
  if (n <= LDS_MAX_N) hipLaunchKernelGGL(tridiag_lds_kernel, dim3(B), dim3(256), 0, s, w, n);
  else hipLaunchKernelGGL(tridiag_global_kernel, dim3(B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

hipError_t bisect_eigvals(const EigWork &w, int n, int B, hipStream_t s) {
  hipLaunchKernelGGL(bisect_kernel, dim3((n + 255) / 256, B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

hipError_t entropy_sum(const EigWork &w, int n, int B, hipStream_t s) {
  hipLaunchKernelGGL(entropy_kernel, dim3(B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

}  // namespace mfq
