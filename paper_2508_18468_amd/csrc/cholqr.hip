// Cholesky-QR re-orthonormalisation: U <- U R^{-1}, R^+ R = U^+ U.
//
// The paper keeps U^+ U = 1 by a QR decomposition after every step
// (Appendix A).  Here one pass is: Gram G = U^+ U on the matrix cores (upper
// triangle only), blocked right-looking Cholesky G = R^+ R (upper R, block
// 64: the diagonal block factorised and inverted in LDS, the block row solved
// and the trailing matrix updated by the batched GEMM), the triangular
// inverse R^{-1} assembled block column by block column from GEMMs, and the
// triangular product U R^{-1} (zero blocks of R^{-1} skipped).  Two passes
// (Cholesky-QR2) bring U^+ U to identity at working precision for the
// condition numbers a step produces.
#include "mfq_internal.h"

namespace mfq {

namespace {

constexpr int NB = CHOL_NB;

// Factorise the w x w diagonal block at (c0, c0) of G[b] (upper triangle),
// write R_JJ back into G and R_JJ^{-1} (full block, zeros below the diagonal)
// into Rinv[b].  A non-positive or non-finite pivot raises *flag.
__global__ __launch_bounds__(256) void potrf_diag_kernel(cplx *G, cplx *Rinv, int N, int c0, int w,
                                                         int *flag, const double *skip_if_le,
                                                         double skip_thr) {
  if (skip_if_le && *skip_if_le <= skip_thr) return;
  const int b = blockIdx.x, tid = threadIdx.x;
  cplx *Gb = G + (long)b * N * N;
  cplx *Rb = Rinv + (long)b * N * N;
  __shared__ cplx a[NB][NB + 1];  // a[c][r] = element (row r, col c) of the block
  __shared__ cplx x[NB][NB + 1];  // x[c][r] = element (r, c) of the inverse
  __shared__ int bad;
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < w * w; idx += 256) {
    const int r = idx % w, c = idx / w;
    a[c][r] = (r <= c) ? Gb[(c0 + r) + (long)(c0 + c) * N] : cplx{0.0, 0.0};
  }
  __syncthreads();
  for (int k = 0; k < w; ++k) {
    if (tid == 0) {
      double d = a[k][k].re;
      if (!(d > 0.0) || !isfinite(d)) {
        bad = 1;
        d = 1.0;
      }
      a[k][k] = cplx{sqrt(d), 0.0};
    }
    __syncthreads();
    const double rkk = a[k][k].re;
    for (int j = k + 1 + tid; j < w; j += 256) {
      a[j][k].re /= rkk;
      a[j][k].im /= rkk;
    }
    __syncthreads();
    // trailing: a(i, j) -= conj(R_ki) R_kj for k < i <= j < w
    const int m = w - k - 1;
    for (int idx = tid; idx < m * m; idx += 256) {
      const int i = k + 1 + idx % m, j = k + 1 + idx / m;
      if (i > j) continue;
      const cplx rki = a[i][k], rkj = a[j][k];
      a[j][i].re -= rki.re * rkj.re + rki.im * rkj.im;
      a[j][i].im -= rki.re * rkj.im - rki.im * rkj.re;
    }
    __syncthreads();
  }
  // inverse of the upper triangular block by back substitution, one column per thread
  if (tid < w) {
    const int j = tid;
    for (int i = w - 1; i > j; --i) x[j][i] = cplx{0.0, 0.0};
    x[j][j] = cplx{1.0 / a[j][j].re, 0.0};
    for (int i = j - 1; i >= 0; --i) {
      double sr = 0.0, si = 0.0;
      for (int k = i + 1; k <= j; ++k) {
        const cplx r = a[k][i], t = x[j][k];
        sr += r.re * t.re - r.im * t.im;
        si += r.re * t.im + r.im * t.re;
      }
      const double inv = 1.0 / a[i][i].re;
      x[j][i] = cplx{-sr * inv, -si * inv};
    }
  }
  __syncthreads();
  for (int idx = tid; idx < w * w; idx += 256) {
    const int r = idx % w, c = idx / w;
    if (r <= c) Gb[(c0 + r) + (long)(c0 + c) * N] = a[c][r];
    Rb[(c0 + r) + (long)(c0 + c) * N] = x[c][r];
  }
  if (tid == 0 && bad) atomicOr(flag, 1);
}

// E = G - I over the upper triangle of every Gram: writes the first-order
// inverse factor R^{-1} = I - triu(E, 1) - diag(E)/2 and raises *maxdev to the
// largest |E_ij| (non-negative doubles order like their bit patterns; a NaN
// compares above every finite value and so selects the full factorisation).
__global__ __launch_bounds__(256) void near_identity_kernel(const cplx *G, cplx *Rinv, int N,
                                                            double *maxdev) {
  const int c = blockIdx.x, b = blockIdx.y;  // one column of one Gram per workgroup
  const long NN = (long)N * N;
  const cplx *Gc = G + b * NN + (long)c * N;
  cplx *Rc = Rinv + b * NN + (long)c * N;
  const double qnan = __longlong_as_double(0x7ff8000000000000ll);
  double m = 0.0;
  for (int r = threadIdx.x; r < N; r += 256) {
    cplx out{0.0, 0.0};
    if (r <= c) {
      const cplx e = Gc[r];
      const double d = (r == c) ? e.re - 1.0 : e.re;
      const double a = fabs(d) + fabs(e.im);
      m = (!(a <= 1e300) || m != m) ? qnan : fmax(m, a);
      out = (r == c) ? cplx{1.0 - 0.5 * d, 0.0} : cplx{-e.re, -e.im};
    }
    Rc[r] = out;
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const double x = red[threadIdx.x], y = red[threadIdx.x + o];
      red[threadIdx.x] = (x != x || y != y) ? qnan : fmax(x, y);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    atomicMax(reinterpret_cast<unsigned long long *>(maxdev),
              (unsigned long long)__double_as_longlong(red[0]));
}

GemmDesc desc() {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  return g;
}

}  // namespace

hipError_t cholqr_pass(const cplx *Uin, cplx *Uout, int L, int N, int B, const CholWork &wk,
                       bool near_identity, hipStream_t s) {
  hipError_t e;
  const long NN = (long)N * N;
  // full-factorisation launches are skipped on the device when the near-identity
  // test passed (max |E| <= threshold)
  const double *skip = near_identity ? wk.dev : nullptr;
  const double thr = CHOL_FIRST_ORDER_MAX;
  // G = Uin^+ Uin (upper triangle)
  {
    GemmDesc g = desc();
    g.M = N; g.N = N; g.K = L; g.batch = B;
    g.A = Uin; g.lda = L; g.sA = (long)L * N; g.opA = OP_C;
    g.B = Uin; g.ldb = L; g.sB = (long)L * N; g.opB = OP_N;
    g.D = wk.G; g.ldd = N; g.sD = NN;
    g.tri = TRI_UPPER;
    if ((e = zgemm(g, s)) != hipSuccess) return e;
  }
  if (near_identity) {
    if ((e = fill_zero(wk.dev, sizeof(double), s)) != hipSuccess) return e;
    hipLaunchKernelGGL(near_identity_kernel, dim3(N, B), dim3(256), 0, s, wk.G, wk.Rinv, N, wk.dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const int nJ = (N + NB - 1) / NB;
  for (int J = 0; J < nJ; ++J) {
    const int c0 = J * NB, w = std::min(NB, N - c0);
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(B), dim3(256), 0, s, wk.G, wk.Rinv, N, c0, w, wk.flag,
                       skip, thr);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int r0 = c0 + w, nr = N - r0;
    if (nr <= 0) break;
    // block row: R_J,rest = R_JJ^{-+} G_J,rest (in place; one row tile, so every
    // workgroup reads its whole column panel before writing it)
    {
      GemmDesc g = desc();
      g.skip_if_le = skip; g.skip_thr = thr;
      g.M = w; g.N = nr; g.K = w; g.batch = B;
      g.A = wk.Rinv + c0 + (long)c0 * N; g.lda = N; g.sA = NN; g.opA = OP_C;
      g.B = wk.G + c0 + (long)r0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
      g.D = wk.G + c0 + (long)r0 * N; g.ldd = N; g.sD = NN;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    // trailing: G_rest,rest -= R_J,rest^+ R_J,rest (upper)
    {
      GemmDesc g = desc();
      g.skip_if_le = skip; g.skip_thr = thr;
      g.M = nr; g.N = nr; g.K = w; g.batch = B;
      g.A = wk.G + c0 + (long)r0 * N; g.lda = N; g.sA = NN; g.opA = OP_C;
      g.B = wk.G + c0 + (long)r0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
      g.Cin = wk.G + r0 + (long)r0 * N; g.ldcin = N; g.sCin = NN;
      g.D = wk.G + r0 + (long)r0 * N; g.ldd = N; g.sD = NN;
      g.alpha = cplx{-1.0, 0.0};
      g.beta = cplx{1.0, 0.0};
      g.tri = TRI_UPPER;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
  }
  // R^{-1}: block column J = -(R^{-1})_{0:J,0:J} R_{0:J,J} (R_JJ)^{-1}
  for (int J = 1; J < nJ; ++J) {
    const int c0 = J * NB, w = std::min(NB, N - c0);
    {
      GemmDesc g = desc();
      g.skip_if_le = skip; g.skip_thr = thr;
      g.M = c0; g.N = w; g.K = c0; g.batch = B;
      g.A = wk.Rinv; g.lda = N; g.sA = NN; g.opA = OP_N; g.aUpper = 1;
      g.B = wk.G + (long)c0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
      g.D = wk.T; g.ldd = N; g.sD = (long)N * NB;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    {
      GemmDesc g = desc();
      g.skip_if_le = skip; g.skip_thr = thr;
      g.M = c0; g.N = w; g.K = w; g.batch = B;
      g.A = wk.T; g.lda = N; g.sA = (long)N * NB; g.opA = OP_N;
      g.B = wk.Rinv + c0 + (long)c0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N; g.bUpper = 1;
      g.D = wk.Rinv + (long)c0 * N; g.ldd = N; g.sD = NN;
      g.alpha = cplx{-1.0, 0.0};
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
  }
  // Uout = Uin R^{-1}
  {
    GemmDesc g = desc();
    g.M = L; g.N = N; g.K = N; g.batch = B;
    g.A = Uin; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
    g.B = wk.Rinv; g.ldb = N; g.sB = NN; g.opB = OP_N; g.bUpper = 1;
    g.D = Uout; g.ldd = L; g.sD = (long)L * N;
    if ((e = zgemm(g, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mfq
