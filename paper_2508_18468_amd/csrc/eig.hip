// Spectrum of the region correlation matrix and the entanglement entropy.
//
// S_A (Sec. II entropy formula) needs every eigenvalue of the Hermitian
// C_A = U_A U_A^+.  Pipeline: Gram of the region rows on the matrix cores
// (U_A^+ U_A instead when the region has more sites than particles: same
// nonzero spectrum), Householder reduction to a real symmetric tridiagonal,
// Sturm-sequence bisection for all eigenvalues, and the entropy sum with a
// fixed reduction order.
//
// Householder reduction: a matrix that fits in LDS is reduced by one
// workgroup; a larger one by a grid-wide sweep per reflector (all matrices of
// the batch in the same launches):
//   tri_col(k)   one workgroup per matrix: finishes w of reflector k-1 from
//                the previous sweep's p (w = tau p - (tau^2/2)(v^+ p) v),
//                applies the pending rank-2 update to column k, records d_k
//                and forms reflector k of column k (v_k, tau_k, e_k);
//   tri_sweep(k) one wave per group of columns j > k: applies the pending
//                update A -= v w^+ + w v^+ of reflector k-1 to column j and
//                forms p_j = sum_i conj(A_ij) v_k,i, i.e. (A v_k)_j for
//                Hermitian A.
// Every sweep reads and writes the trailing matrix once (HBM-bound).
// Bisection: one lane per eigenvalue when the batch offers enough of them,
// otherwise one wave per eigenvalue that splits its interval at 64 points per
// Sturm pass (65-fold narrowing per pass instead of 2-fold).
#include "device_common.h"

namespace mfq {

namespace {

constexpr int LDS_MAX_N = 88;  // 88 * 88 * 16 B = 121 KiB
// below this many eigenvalues in a batch, one wave per eigenvalue (multisection)
constexpr long BISECT_LANES_MIN = 131072;

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

__device__ __forceinline__ double wave_sum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ cplx *v_slot(const EigWork &W, int b, int n, int k) {
  return W.v + ((long)b * 2 + (k & 1)) * n;
}

// Reflector step k of the grid-wide reduction on matrix blockIdx.x (see the
// file comment).  Vectors are indexed by absolute row; reflector k lives in
// slot k & 1 and has entries in rows k+1 .. n-1.
__global__ __launch_bounds__(256) void tri_col_kernel(EigWork W, int n, int k) {
  const int b = blockIdx.x, tid = threadIdx.x;
  cplx *col = W.A + (long)b * n * n + (long)k * n;
  cplx *vc = v_slot(W, b, n, k);
  const cplx *vp = v_slot(W, b, n, k + 1);  // slot of reflector k-1
  cplx *w = W.w + (long)b * n;
  const cplx *p = W.p + (long)b * n;
  double *d = W.d + (long)b * n, *e = W.e + (long)b * n;
  __shared__ double red[4];
  __shared__ double sh_dk;
  __shared__ cplx sh_x0;
  const double tp = k >= 1 ? W.tau[2 * b + ((k + 1) & 1)] : 0.0;
  // K = (tp^2 / 2) v^+ p over rows >= k
  double Kr = 0.0, Ki = 0.0;
  if (tp != 0.0) {
    double kr = 0.0, ki = 0.0;
    for (int i = k + tid; i < n; i += 256) {
      const cplx vi = vp[i], q = p[i];
      kr += vi.re * q.re + vi.im * q.im;
      ki += vi.re * q.im - vi.im * q.re;
    }
    kr = block_sum256(kr, red);
    ki = block_sum256(ki, red);
    Kr = 0.5 * tp * tp * kr;
    Ki = 0.5 * tp * tp * ki;
  }
  // w_i = tp p_i - K v_i
  auto w_at = [&](int i) {
    const cplx vi = vp[i], q = p[i];
    return cplx{tp * q.re - (Kr * vi.re - Ki * vi.im), tp * q.im - (Kr * vi.im + Ki * vi.re)};
  };
  cplx vk{0.0, 0.0}, wk{0.0, 0.0};
  if (tp != 0.0 && k < n) {
    vk = vp[k];
    wk = w_at(k);
  }
  double mx = 0.0;
  for (int i = k + tid; i < n; i += 256) {
    cplx a = col[i];
    if (tp != 0.0) {
      const cplx vi = vp[i], wi = w_at(i);
      w[i] = wi;
      a.re -= (vi.re * wk.re + vi.im * wk.im) + (wi.re * vk.re + wi.im * vk.im);
      a.im -= (vi.im * wk.re - vi.re * wk.im) + (wi.im * vk.re - wi.re * vk.im);
      col[i] = a;
    }
    if (i == k) sh_dk = a.re;
    else mx = fmax(mx, cmax_abs(a));
    if (i == k + 1) sh_x0 = a;
  }
  // the reflector is formed from the column scaled by its largest component
  // (the barriers of the reduction publish the updated column to all threads)
  const double s = block_max256(mx, red);
  const double inv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
  double part = 0.0;
  for (int i = k + 2 + tid; i < n; i += 256) {
    const cplx a{col[i].re * inv, col[i].im * inv};
    part += a.re * a.re + a.im * a.im;
    vc[i] = a;
  }
  const double tail2 = block_sum256(part, red);  // its barriers publish sh_dk, sh_x0
  if (tid != 0) return;
  d[k] = sh_dk;
  if (k + 1 >= n) return;  // n == 1
  const cplx x0 = sh_x0;
  const double ax0 = hypot(x0.re, x0.im);
  if (k == n - 2) {  // last off-diagonal, and the last diagonal entry with the pending update
    e[k] = ax0;
    const cplx *cn = W.A + (long)b * n * n + (long)(n - 1) * n;
    double dn = cn[n - 1].re;
    if (tp != 0.0) {
      const cplx vi = vp[n - 1], wi = w_at(n - 1);
      dn -= 2.0 * (vi.re * wi.re + vi.im * wi.im);
    }
    d[n - 1] = dn;
    return;
  }
  if (tail2 == 0.0) {  // already reduced (or below REFLECT_TINY): H = I
    e[k] = ax0;
    W.tau[2 * b + (k & 1)] = 0.0;
    return;
  }
  const Reflector h = make_reflector(cplx{x0.re * inv, x0.im * inv}, tail2, s);
  vc[k + 1] = h.v0;
  e[k] = h.norm;
  W.tau[2 * b + (k & 1)] = h.tau;
}

// Sweep of reflector k over columns k+1 .. n-1 of matrix blockIdx.y; each wave
// owns CPW consecutive columns and walks their rows k+1 .. n-1 once.
template <int CPW>
__global__ __launch_bounds__(256) void tri_sweep_kernel(EigWork W, int n, int k) {
  const int b = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j0 = k + 1 + (blockIdx.x * 4 + wave) * CPW;
  if (j0 >= n) return;
  cplx *A = W.A + (long)b * n * n;
  const cplx *vc = v_slot(W, b, n, k);
  const cplx *vp = v_slot(W, b, n, k + 1);
  const cplx *w = W.w + (long)b * n;
  cplx *p = W.p + (long)b * n;
  const double tp = k >= 1 ? W.tau[2 * b + ((k + 1) & 1)] : 0.0;
  const double tc = W.tau[2 * b + (k & 1)];
  const bool upd = tp != 0.0, form = tc != 0.0;
  if (!upd && !form) return;
  cplx sv[CPW], sw[CPW];
  double pr[CPW], pim[CPW];
  int jc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    jc[c] = min(j0 + c, n - 1);  // columns past the end repeat the last one, unwritten
    sv[c] = upd ? vp[jc[c]] : cplx{0.0, 0.0};
    sw[c] = upd ? w[jc[c]] : cplx{0.0, 0.0};
    pr[c] = pim[c] = 0.0;
  }
  for (int i = k + 1 + lane; i < n; i += 64) {
    const cplx xv = upd ? vp[i] : cplx{0.0, 0.0};
    const cplx xw = upd ? w[i] : cplx{0.0, 0.0};
    const cplx xc = form ? vc[i] : cplx{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      cplx *ap = A + i + (long)jc[c] * n;
      cplx a = *ap;
      if (upd) {
        a.re -= (xv.re * sw[c].re + xv.im * sw[c].im) + (xw.re * sv[c].re + xw.im * sv[c].im);
        a.im -= (xv.im * sw[c].re - xv.re * sw[c].im) + (xw.im * sv[c].re - xw.re * sv[c].im);
        if (j0 + c < n) *ap = a;
      }
      pr[c] += a.re * xc.re + a.im * xc.im;
      pim[c] += a.re * xc.im - a.im * xc.re;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    const double sr = wave_sum(pr[c]), si = wave_sum(pim[c]);
    if (lane == 0 && j0 + c < n) p[j0 + c] = cplx{sr, si};
  }
}

// Eigenvalue k (ascending) of tridiagonal b (see bisect_eigenvalue).
__global__ __launch_bounds__(256) void bisect_kernel(EigWork w, int n) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  w.lam[(long)b * n + k] = bisect_eigenvalue(w.d + (long)b * n, w.e + (long)b * n, n, k);
}

// Eigenvalue blockIdx.x * 4 + wave of tridiagonal blockIdx.y by multisection:
// the 64 lanes evaluate the Sturm count at 64 interior points of the current
// interval, which shrinks to the gap between the last point below lambda_k
// and the first above it.  Same interval, pivmin and stopping width as
// bisect_eigenvalue.
__global__ __launch_bounds__(256) void bisect_multi_kernel(EigWork w, int n) {
  const int b = blockIdx.y, lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= n) return;
  const double *d = w.d + (long)b * n, *e = w.e + (long)b * n;
  double lo = d[0], hi = d[0], emax2 = 0.0;
  for (int i = lane; i < n; i += 64) {
    const double r = (i > 0 ? e[i - 1] : 0.0) + (i + 1 < n ? e[i] : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double span = fmax(fabs(lo), fabs(hi));
  lo -= 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  hi += 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  const double tol = 4.0 * 2.220446049250313e-16 * fmax(1.0, span);
  for (int it = 0; it < 40 && hi - lo > tol; ++it) {
    const double x = lo + (hi - lo) * ((double)(lane + 1) / 65.0);
    const bool above = sturm_count(d, e, n, x, pivmin) > k;
    const unsigned long long m = __ballot(above);
    const int first = m ? __ffsll((long long)m) - 1 : 64;
    const double nhi = __shfl(x, first < 64 ? first : 0, 64);
    const double nlo = __shfl(x, first > 0 ? first - 1 : 0, 64);
    if (first < 64) hi = nhi;
    if (first > 0) lo = nlo;
  }
  if (lane == 0) w.lam[(long)b * n + k] = bracket_estimate(lo, hi);
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
  if (n <= LDS_MAX_N) {
    hipLaunchKernelGGL(tridiag_lds_kernel, dim3(B), dim3(256), 0, s, w, n);
    return hipGetLastError();
  }
  for (int k = 0; k <= n - 2; ++k) {
    hipLaunchKernelGGL(tri_col_kernel, dim3(B), dim3(256), 0, s, w, n, k);
    if (k == n - 2) break;
    // columns per wave: as many as keep ~512 workgroups busy
    const long m = n - k - 1;
    if ((m + 15) / 16 * B >= 512)
      hipLaunchKernelGGL(tri_sweep_kernel<4>, dim3((unsigned)((m + 15) / 16), B), dim3(256), 0, s, w, n, k);
    else if ((m + 7) / 8 * B >= 512)
      hipLaunchKernelGGL(tri_sweep_kernel<2>, dim3((unsigned)((m + 7) / 8), B), dim3(256), 0, s, w, n, k);
    else
      hipLaunchKernelGGL(tri_sweep_kernel<1>, dim3((unsigned)((m + 3) / 4), B), dim3(256), 0, s, w, n, k);
  }
  return hipGetLastError();
}

hipError_t bisect_eigvals(const EigWork &w, int n, int B, hipStream_t s) {
  if ((long)n * B >= BISECT_LANES_MIN)
    hipLaunchKernelGGL(bisect_kernel, dim3((n + 255) / 256, B), dim3(256), 0, s, w, n);
  else
    hipLaunchKernelGGL(bisect_multi_kernel, dim3((n + 3) / 4, B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

hipError_t entropy_sum(const EigWork &w, int n, int B, hipStream_t s) {
  hipLaunchKernelGGL(entropy_kernel, dim3(B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

}  // namespace mfq
