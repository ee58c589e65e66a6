// Spectrum of the region correlation matrix and the entanglement entropy.
//
// S_A (Sec. II entropy formula) needs every eigenvalue of the Hermitian
// C_A = U_A U_A^+.  Pipeline: Gram of the region rows on the matrix cores
// (U_A^+ U_A instead when the region has more sites than particles: same
// nonzero spectrum), Householder reduction to a real symmetric tridiagonal
// (one workgroup per matrix; in LDS when it fits), Sturm-sequence bisection
// for all eigenvalues (one lane per eigenvalue), and the entropy sum with a
// fixed reduction order.
#include "mfq_internal.h"

namespace mfq {

namespace {

constexpr int LDS_MAX_N = 88;  // 88 * 88 * 16 B = 121 KiB

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum256(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Householder tridiagonalisation of the Hermitian n x n matrix A (column-major,
// leading dimension ld, full storage), destroying A.  Step k reflects
// x = A[k+1:, k] onto alpha e_0 with H = I - tau v v^+, v = x - alpha e_0,
// alpha = -phase(x_0) |x|, and applies A22 <- H A22 H as
// A22 -= v w^+ + w v^+, w = p - (tau/2)(v^+ p) v, p = tau A22 v.
// Output: d[0:n] (diagonal), e[0:n-1] = |off-diagonal| (a diagonal unitary
// similarity makes the off-diagonal real and nonnegative).
__device__ void tridiag_body(cplx *A, int ld, int n, cplx *v, cplx *p, double *d, double *e,
                             double *red) {
  const int tid = threadIdx.x;
  __shared__ double s_tau, s_kr, s_ki;
  __shared__ int s_skip;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    cplx *x = A + (k + 1) + (long)k * ld;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += 256) part += x[i].re * x[i].re + x[i].im * x[i].im;
    const double tail2 = block_sum256(part, red);
    if (tid == 0) {
      const cplx x0 = x[0];
      const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im);
      d[k] = A[k + (long)k * ld].re;
      if (tail2 == 0.0) {
        e[k] = ax0;
        s_skip = 1;
      } else {
        const double nx = sqrt(ax0 * ax0 + tail2);
        const double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
        const double v0r = x0.re + phr * nx, v0i = x0.im + phi * nx;
        s_tau = 2.0 / (tail2 + v0r * v0r + v0i * v0i);
        e[k] = nx;
        s_skip = 0;
        v[0] = cplx{v0r, v0i};
      }
    }
    for (int i = 1 + tid; i < m; i += 256) v[i] = x[i];
    __syncthreads();
    if (s_skip) continue;
    const double tau = s_tau;
    cplx *A22 = A + (k + 1) + (long)(k + 1) * ld;
    // p = tau A22 v
    for (int i = tid; i < m; i += 256) {
      double ar = 0.0, ai = 0.0;
      for (int j = 0; j < m; ++j) {
        const cplx a = A22[i + (long)j * ld], vj = v[j];
        ar += a.re * vj.re - a.im * vj.im;
        ai += a.re * vj.im + a.im * vj.re;
      }
      p[i] = cplx{tau * ar, tau * ai};
    }
    __syncthreads();
    // K = (tau/2) v^+ p
    double pr = 0.0, pi = 0.0;
    for (int i = tid; i < m; i += 256) {
      const cplx vi = v[i], q = p[i];
      pr += vi.re * q.re + vi.im * q.im;
      pi += vi.re * q.im - vi.im * q.re;
    }
    const double kr = 0.5 * tau * block_sum256(pr, red);
    const double ki = 0.5 * tau * block_sum256(pi, red);
    // w = p - K v  (overwrites p)
    for (int i = tid; i < m; i += 256) {
      const cplx vi = v[i];
      cplx q = p[i];
      q.re -= kr * vi.re - ki * vi.im;
      q.im -= kr * vi.im + ki * vi.re;
      p[i] = q;
    }
    __syncthreads();
    // A22 -= v w^+ + w v^+
    for (int i = tid; i < m; i += 256) {
      const cplx vi = v[i], wi = p[i];
      for (int j = 0; j < m; ++j) {
        const cplx vj = v[j], wj = p[j];
        cplx a = A22[i + (long)j * ld];
        a.re -= (vi.re * wj.re + vi.im * wj.im) + (wi.re * vj.re + wi.im * vj.im);
        a.im -= (vi.im * wj.re - vi.re * wj.im) + (wi.im * vj.re - wi.re * vj.im);
        A22[i + (long)j * ld] = a;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) + (long)(n - 2) * ld].re;
      const cplx t = A[(n - 1) + (long)(n - 2) * ld];
      e[n - 2] = sqrt(t.re * t.re + t.im * t.im);
    }
    d[n - 1] = A[(n - 1) + (long)(n - 1) * ld].re;
  }
}

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

// Number of eigenvalues of the tridiagonal (d, e) smaller than x (Sturm count
// of the LDL^T pivots of T - x I, tiny pivots replaced by -pivmin).
__device__ __forceinline__ int sturm_count(const double *d, const double *e, int n, double x,
                                           double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++c;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - (e[i - 1] * e[i - 1]) / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++c;
  }
  return c;
}

// Eigenvalue k (ascending) of tridiagonal b by bisection on the Gershgorin
// interval, to an absolute width of ~4 ulp(1).
__global__ __launch_bounds__(256) void bisect_kernel(EigWork w, int n) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double *d = w.d + (long)b * n, *e = w.e + (long)b * n;
  double lo = d[0], hi = d[0], emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? e[i - 1] : 0.0) + (i + 1 < n ? e[i] : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
  }
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double span = fmax(fabs(lo), fabs(hi));
  lo -= 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  hi += 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  const double tol = 4.0 * 2.220446049250313e-16 * fmax(1.0, span);
  for (int it = 0; it < 200 && hi - lo > tol; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(d, e, n, mid, pivmin) > k) hi = mid;
    else lo = mid;
  }
  w.lam[(long)b * n + k] = 0.5 * (lo + hi);
}

// S = sum_k h(lambda_k), h(x) = -x ln x - (1 - x) ln(1 - x), lambda clamped to [0, 1].
__global__ __launch_bounds__(256) void entropy_kernel(EigWork w, int n) {
  const int b = blockIdx.x;
  __shared__ double red[4];
  double s = 0.0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double x = fmin(fmax(w.lam[(long)b * n + k], 0.0), 1.0);
    if (x > 0.0 && x < 1.0) s -= x * log(x) + (1.0 - x) * log1p(-x);
  }
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
