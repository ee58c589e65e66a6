// Fused small-lattice trajectory kernel: one workgroup advances one trajectory
// through many steps with its state resident in LDS, observing S_A on
// schedule, in a single launch.
//
// For small L (e.g. the L = 64 ring, U = 32 KiB) the per-phase kernels of a
// step are each far too small to fill the GPU and the step is dominated by
// launch and synchronisation latency.  Here every phase of Appendix A's step
// runs back to back inside the workgroup:
//   U' = P U (a dense product over all L^2 entries of P on the matrix cores,
//   the entries generated from the ring's circulant row -- or, on the torus,
//   the two rows of P = P_y (x) P_x -- held in LDS),
//   Born probabilities + homodyne factor (Eq. (A4)) or projective
//   measurements (Eq. (A1), Eq. (A2)), two Cholesky-QR passes (Gram on the
//   matrix cores, Cholesky and triangular solve U R^{-1} in LDS; the second
//   pass keeps a state its Gram certifies), and, when the absolute step is a
//   multiple of obs_every, S_A of one region (Gram of the region rows,
//   Householder tridiagonalisation, bisection, entropy sum; Sec. II).
// Random numbers are the same Philox draws as the per-phase kernels, so the
// two paths compute the same trajectory up to rounding.
#include <atomic>
#include <algorithm>

#include "device_common.h"

namespace mfq {

namespace {

struct FusedLayout {
  size_t ua, ub, g, r, v, w, site, outc, prob, d, e, lam, gx, gy, total;
};

__host__ __device__ inline size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__host__ __device__ inline FusedLayout fused_layout(int L, int N, int Lx, int Ly) {
  FusedLayout f;
  size_t o = 0;
  // leading dimensions padded by one element: consecutive columns then start
  // 16 bytes apart modulo the bank width, so lanes walking a row hit distinct banks
  f.ua = o; o = al16(o + sizeof(cplx) * (size_t)(L + 1) * N);
  f.ub = o; o = al16(o + sizeof(cplx) * (size_t)(L + 1) * N);
  f.g = o; o = al16(o + sizeof(cplx) * (size_t)(N + 1) * N);
  f.r = o; o = al16(o + sizeof(cplx) * (size_t)(N + 1) * N);
  f.v = o; o = al16(o + sizeof(cplx) * (size_t)N);
  f.w = o; o = al16(o + sizeof(cplx) * (size_t)L);
  f.site = o; o = al16(o + sizeof(int) * (size_t)L);
  f.outc = o; o = al16(o + sizeof(int) * (size_t)L);
  f.prob = o; o = al16(o + sizeof(double) * (size_t)L);
  f.d = o; o = al16(o + sizeof(double) * (size_t)N);
  f.e = o; o = al16(o + sizeof(double) * (size_t)N);
  f.lam = o; o = al16(o + sizeof(double) * (size_t)N);
  f.gx = o; o = al16(o + sizeof(cplx) * (size_t)Lx);
  f.gy = o; o = al16(o + sizeof(cplx) * (size_t)Ly);
  f.total = o;
  return f;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

// C = A B for small LDS-resident operands on the matrix cores (v_mfma_f64_16x16x4f64, four
// real products per complex one): the M x Nc result in 16 x 16 blocks, spread over the
// workgroup's four waves; a(m, k) and b(k, n) give the operands (zero outside M x K and
// K x Nc) and put(m, n, v) receives each entry of C inside M x Nc.  upper: only the blocks
// that meet the upper triangle (m <= n) are formed.  Operand lane layout: A lane l holds
// A[l % 16][l / 16], B lane l holds B[l / 16][l % 16]; result register r of lane l is
// C[l / 16 + 4 r][l % 16].
template <class FA, class FB, class FPut>
__device__ __forceinline__ void mfma_product(int M, int Nc, int K, FA a, FB b, FPut put, bool upper) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int bm_n = (M + 15) / 16, bn_n = (Nc + 15) / 16;
  for (int blk = wave; blk < bm_n * bn_n; blk += 4) {
    const int bm = blk % bm_n, bn = blk / bm_n;
    if (upper && bm > bn) continue;
    const int m = bm * 16 + (lane & 15), n = bn * 16 + (lane & 15);
    f64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + (lane >> 4);
      const cplx av = (m < M && k < K) ? a(m, k) : cplx{0.0, 0.0};
      const cplx bv = (k < K && n < Nc) ? b(k, n) : cplx{0.0, 0.0};
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.re, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.re, bv.im, ci, 0, 0, 0);
      cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-av.im, bv.im, cr, 0, 0, 0);
      ci = __builtin_amdgcn_mfma_f64_16x16x4f64(av.im, bv.re, ci, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = bm * 16 + (lane >> 4) + 4 * r, col = bn * 16 + (lane & 15);
      if (row < M && col < Nc) put(row, col, cplx{cr[r], ci[r]});
    }
  }
}

// Householder tridiagonalisation of the n x n Hermitian A (leading dimension ld, n <= 64)
// by one wave, lane i owning row i: the same reflectors and updates as tridiag_body
// (scaled reflector, p = tau A22 v, w = p - (tau/2)(v^+ p) v, A22 -= v w^+ + w v^+), with
// wave reductions and wave-level ordering in place of workgroup barriers.  Output as
// tridiag_body: d[0:n], e[0:n-1] = |off-diagonal|.  v, p: n scratch entries each.
__device__ void tridiag_wave(cplx *A, int ld, int n, cplx *v, cplx *p, double *d, double *e) {
  const int lane = threadIdx.x & 63;
  auto wave_order = []() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const cplx *x = A + (k + 1) + (long)k * ld;
    const cplx xi = lane < m ? x[lane] : cplx{0.0, 0.0};
    double s = cmax_abs(xi);
    for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o, 64));
    const double inv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
    const cplx a{xi.re * inv, xi.im * inv};
    double tail2 = lane >= 1 && lane < m ? a.re * a.re + a.im * a.im : 0.0;
    for (int o = 32; o > 0; o >>= 1) tail2 += __shfl_xor(tail2, o, 64);
    const cplx x0 = x[0];
    if (lane == 0) d[k] = A[k + (long)k * ld].re;
    if (tail2 == 0.0) {  // nothing below x0 (or all below REFLECT_TINY): H = I
      if (lane == 0) e[k] = hypot(x0.re, x0.im);
      wave_order();
      continue;
    }
    const Reflector h = make_reflector(cplx{x0.re * inv, x0.im * inv}, tail2, s);
    const double tau = h.tau;
    if (lane == 0) {
      e[k] = h.norm;
      v[0] = h.v0;
    } else if (lane < m) {
      v[lane] = a;
    }
    wave_order();
    cplx *A22 = A + (k + 1) + (long)(k + 1) * ld;
    cplx pi{0.0, 0.0};
    if (lane < m) {
      double ar = 0.0, ai = 0.0;
      for (int j = 0; j < m; ++j) {
        const cplx aij = A22[lane + (long)j * ld], vj = v[j];
        ar += aij.re * vj.re - aij.im * vj.im;
        ai += aij.re * vj.im + aij.im * vj.re;
      }
      pi = cplx{tau * ar, tau * ai};
    }
    const cplx vi = lane < m ? v[lane] : cplx{0.0, 0.0};
    double pr = vi.re * pi.re + vi.im * pi.im, pim = vi.re * pi.im - vi.im * pi.re;
    for (int o = 32; o > 0; o >>= 1) {
      pr += __shfl_xor(pr, o, 64);
      pim += __shfl_xor(pim, o, 64);
    }
    const double kr = 0.5 * tau * pr, ki = 0.5 * tau * pim;
    const cplx wi{pi.re - (kr * vi.re - ki * vi.im), pi.im - (kr * vi.im + ki * vi.re)};
    if (lane < m) p[lane] = wi;
    wave_order();
    if (lane < m) {
      for (int j = 0; j < m; ++j) {
        const cplx vj = v[j], wj = p[j];
        cplx aij = A22[lane + (long)j * ld];
        aij.re -= (vi.re * wj.re + vi.im * wj.im) + (wi.re * vj.re + wi.im * vj.im);
        aij.im -= (vi.im * wj.re - vi.re * wj.im) + (wi.im * vj.re - wi.re * vj.im);
        A22[lane + (long)j * ld] = aij;
      }
    }
    wave_order();
  }
  if (lane == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) + (long)(n - 2) * ld].re;
      const cplx t = A[(n - 1) + (long)(n - 2) * ld];
      e[n - 2] = hypot(t.re, t.im);
    }
    d[n - 1] = A[(n - 1) + (long)(n - 1) * ld].re;
  }
}

// Eigenvalues lam[0:n] (ascending) of the tridiagonal (d, e) by multisection over the
// workgroup: eight adjacent lanes per eigenvalue evaluate the Sturm count at eight interior
// points of its bracket and keep the sub-interval where the count passes k (a ninth of the
// bracket per round, against a half for bisection), on the same Gershgorin start, pivmin and
// stopping width as bisect_eigenvalue.
__device__ void multisect_eigenvalues(const double *d, const double *e, int n, double *lam) {
  const int tid = threadIdx.x, lane = tid & 63, sub = tid & 7, base = lane & ~7;
  double lo0 = d[0], hi0 = d[0], emax2 = 0.0;
  for (int i = 0; i < n; ++i) {
    const double r = (i > 0 ? e[i - 1] : 0.0) + (i + 1 < n ? e[i] : 0.0);
    lo0 = fmin(lo0, d[i] - r);
    hi0 = fmax(hi0, d[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
  }
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
  const double span = fmax(fabs(lo0), fabs(hi0));
  lo0 -= 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  hi0 += 2.0 * 2.220446049250313e-16 * span + 2.0 * pivmin;
  const double tol = 4.0 * 2.220446049250313e-16 * fmax(1.0, span);
  for (int k0 = 0; k0 < n; k0 += 32) {  // 32 groups of eight lanes per round
    const int k = k0 + (tid >> 3);
    double lo = lo0, hi = hi0;
    for (int it = 0; it < 40 && k < n && hi - lo > tol; ++it) {
      const double x = lo + (hi - lo) * ((double)(sub + 1) / 9.0);
      const bool above = sturm_count(d, e, n, x, pivmin) > k;
      const unsigned mask = (unsigned)(__ballot(above) >> base) & 0xffu;
      const int first = mask ? __ffs(mask) - 1 : 8;  // first of the eight points above k
      const double nhi = __shfl(x, base + (first < 8 ? first : 0), 64);
      const double nlo = __shfl(x, base + (first > 0 ? first - 1 : 0), 64);
      if (first < 8) hi = nhi;
      if (first > 0) lo = nlo;
    }
    if (k < n && sub == 0) lam[k] = bracket_estimate(lo, hi);
  }
}

// One Cholesky-QR pass in LDS, in place: X <- X R^{-1}, R^+ R = X^+ X (upper
// R).  X has leading dimension lu (>= L); G (the Gram, then R) has leading
// dimension lg (>= N); rdiag receives the diagonal of R; rowk (N entries) is
// scratch.  Gram on the matrix cores (upper blocks), right-looking Cholesky, then
// the triangular solve Y R = X (Y overwrites X) by four lanes per row.  A non-positive or
// non-finite pivot sets *bad to its column + 1 and *bad_pivot to its value (first one only).
// With certify, X is kept as it is when its Gram is within CHOL_KEEP_MAX of the identity
// entrywise (|Re| + |Im| of G - I), as the second pass of the per-phase path does.
__device__ void cholqr_lds(cplx *X, cplx *G, double *rdiag, cplx *rowk, int L, int N, int lu, int lg,
                           int *bad, double *bad_pivot, bool certify) {
  const int tid = threadIdx.x;
  // largest deviation as the bit pattern of a non-negative double (NaN orders above all)
  __shared__ unsigned long long dev_bits;
  if (tid == 0) dev_bits = 0ull;
  __syncthreads();
  double dmax = 0.0;
  mfma_product(
      N, N, L, [&](int m, int k) { const cplx v = X[k + m * lu]; return cplx{v.re, -v.im}; },
      [&](int k, int n) { return X[k + n * lu]; },
      [&](int r, int c, cplx g) {
        if (r > c) return;
        G[r + c * lg] = g;
        const double dv = fabs(r == c ? g.re - 1.0 : g.re) + fabs(g.im);
        dmax = (dv != dv || dmax != dmax) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(dmax, dv);
      },
      true);
  if (certify) atomicMax(&dev_bits, (unsigned long long)__double_as_longlong(dmax));
  __syncthreads();  // the Gram is written by every wave
  if (certify && __longlong_as_double((long long)dev_bits) <= CHOL_KEEP_MAX) return;
  // Right-looking Cholesky over the whole workgroup: at step k the scaled row k of R is
  // also copied to rowk, whose entries the trailing update of that step reads (a separate
  // buffer, so that those loads do not wait for the update's stores).
  for (int k = 0; k < N; ++k) {
    double d = G[k + k * lg].re;
    const bool ok = d > 0.0 && isfinite(d);
    if (tid == 0 && !ok && *bad == 0) {
      *bad = k + 1;
      *bad_pivot = d;
    }
    if (!ok) d = 1.0;
    const double rkk = sqrt(d);
    if (tid == 0) rdiag[k] = rkk;
    for (int j = k + 1 + tid; j < N; j += 256) {
      cplx r = G[k + j * lg];
      r.re /= rkk;
      r.im /= rkk;
      G[k + j * lg] = r;
      rowk[j] = r;
    }
    __syncthreads();
    const int m = N - k - 1;
    const cplx *__restrict__ rk = rowk + (k + 1);
    cplx *__restrict__ g = G + (k + 1) + (long)(k + 1) * lg;
    for (int idx = tid; idx < m * m; idx += 256) {
      const int i = idx % m, j = idx / m;
      if (i > j) continue;
      const cplx rki = rk[i], rkj = rk[j];
      cplx a = g[i + j * lg];
      a.re -= rki.re * rkj.re + rki.im * rkj.im;
      a.im -= rki.re * rkj.im - rki.im * rkj.re;
      g[i + j * lg] = a;
    }
    __syncthreads();
  }
  // Y R = X: each row is an independent forward substitution, run by four lanes
  // of one wave (64 rows per pass), which split the updates of the later
  // columns; only wave-level ordering is needed between the column steps.
  {
    const int q = tid & 3;
    for (int i0 = 0; i0 < L; i0 += 64) {
      const int i = i0 + (tid >> 2);
      const bool row = i < L;
      for (int j = 0; j < N; ++j) {
        const double inv = 1.0 / rdiag[j];
        cplx y{0.0, 0.0};
        if (row) {
          y = X[i + j * lu];
          y.re *= inv;
          y.im *= inv;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (row) {
          if (q == 0) X[i + j * lu] = y;
          const cplx *__restrict__ rj = G + j;
          cplx *__restrict__ xi = X + i;
          for (int c = j + 1 + q; c < N; c += 4) {
            const cplx r = rj[c * lg];
            cplx x = xi[c * lu];
            x.re -= y.re * r.re - y.im * r.im;
            x.im -= y.re * r.im + y.im * r.re;
            xi[c * lu] = x;
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
  }
  __syncthreads();
}

// All steps and observations of trajectory b of the context described by a, in LDS.
__device__ __forceinline__ void fused_body(const FusedArgs &a, int b, unsigned char *smem) {
  const FusedLayout f = fused_layout(a.L, a.N, a.Lx, a.Ly);
  cplx *Ua = reinterpret_cast<cplx *>(smem + f.ua);
  cplx *Ub = reinterpret_cast<cplx *>(smem + f.ub);
  cplx *G = reinterpret_cast<cplx *>(smem + f.g);
  cplx *R = reinterpret_cast<cplx *>(smem + f.r);
  cplx *vv = reinterpret_cast<cplx *>(smem + f.v);
  cplx *ww = reinterpret_cast<cplx *>(smem + f.w);
  int *site = reinterpret_cast<int *>(smem + f.site);
  int *outc = reinterpret_cast<int *>(smem + f.outc);
  double *prob = reinterpret_cast<double *>(smem + f.prob);
  double *dd = reinterpret_cast<double *>(smem + f.d);
  double *ee = reinterpret_cast<double *>(smem + f.e);
  double *lam = reinterpret_cast<double *>(smem + f.lam);
  cplx *gx = reinterpret_cast<cplx *>(smem + f.gx);
  cplx *gy = reinterpret_cast<cplx *>(smem + f.gy);
  __shared__ double red[4];
  __shared__ int bad;
  __shared__ double bad_pivot;

  const int tid = threadIdx.x;
  const int L = a.L, N = a.N, lu = L + 1, lg = N + 1;
  cplx *Ug = a.U + (long)b * L * N;
  const double g = a.gamma[b];
  const uint64_t key1 = a.uid[b];
  const int64_t base = a.step_base[b];
  if (tid == 0) bad = 0;
  for (int idx = tid; idx < L * N; idx += 256) Ua[idx % L + (idx / L) * lu] = Ug[idx];
  for (int i = tid; i < a.Lx; i += 256) gx[i] = a.gx[i];
  for (int i = tid; i < a.Ly; i += 256) gy[i] = a.gy[i];
  __syncthreads();
  const int Lx = a.Lx, Ly = a.Ly;

  int n_obs = 0, last_cnt = 0;
  for (int s = 1; s <= a.n_steps; ++s) {
    const uint64_t n = (uint64_t)(a.step0 + s - base);  // this trajectory's own step index
    const int64_t n_ctx = a.step0 + s;                   // the context's step (observation schedule)
    // propagate: Ub = P Ua on the matrix cores, with the dense P_ik = gx[(xi - xk) mod Lx]
    // gy[(yi - yk) mod Ly] generated from the generating rows held in LDS (all L^2 terms)
    mfma_product(
        L, N, L,
        [&](int i, int k) {
          int dx = i % Lx - k % Lx, dy = i / Lx - k / Lx;
          dx += dx < 0 ? Lx : 0;
          dy += dy < 0 ? Ly : 0;
          const cplx px = gx[dx], py = gy[dy];
          return cplx{px.re * py.re - px.im * py.im, px.re * py.im + px.im * py.re};
        },
        [&](int k, int j) { return Ua[k + j * lu]; }, [&](int i, int j, cplx v) { Ub[i + j * lu] = v; },
        false);
    __syncthreads();
    if (a.protocol == 1) {
      // Born probability and homodyne factor, one row per thread
      for (int i = tid; i < L; i += 256) {
        double pi = 0.0;
        for (int k = 0; k < N; ++k) {
          const cplx u = Ub[i + k * lu];
          pi += u.re * u.re + u.im * u.im;
        }
        const u64x4 w = philox4x64_10(a.seed, key1, n, (uint64_t)i, PURPOSE_HOMODYNE, 0);
        const double z = sqrt(-2.0 * log(u01(w.v[0]))) * cos(6.283185307179586 * u01(w.v[1]));
        const double fac = exp(sqrt(g * a.dt) * z + g * (2.0 * pi - 1.0) * a.dt);
        for (int k = 0; k < N; ++k) {
          Ub[i + k * lu].re *= fac;
          Ub[i + k * lu].im *= fac;
        }
      }
      __syncthreads();
    } else {
      last_cnt = pm_measure_block(Ub, L, N, fmin(g * a.dt, 1.0), a.seed, key1, n, site, outc, prob, vv, ww,
                                  lu);
      __syncthreads();
    }
    cholqr_lds(Ub, G, lam, vv, L, N, lu, lg, &bad, &bad_pivot, false);
    cholqr_lds(Ub, G, lam, vv, L, N, lu, lg, &bad, &bad_pivot, true);
    // state now in Ub: swap so that it is in Ua for the next step
    cplx *t = Ua;
    Ua = Ub;
    Ub = t;

    if (a.obs_every > 0 && n_ctx % a.obs_every == 0) {
      const int nreg = a.nreg;
      double S = 0.0;
      if (nreg > 0) {
        const int m = nreg <= N ? nreg : N;
        if (nreg <= N) {  // C_A = U_A U_A^+
          for (int idx = tid; idx < m * m; idx += 256) {
            const int r1 = a.region[idx % m], r2 = a.region[idx / m];
            double sr = 0.0, si = 0.0;
            for (int k = 0; k < N; ++k) {
              const cplx x = Ua[r1 + k * lu], y = Ua[r2 + k * lu];
              sr += x.re * y.re + x.im * y.im;
              si += x.im * y.re - x.re * y.im;
            }
            G[idx] = cplx{sr, si};
          }
        } else {          // U_A^+ U_A, same nonzero spectrum
          for (int idx = tid; idx < m * m; idx += 256) {
            const int c1 = idx % m, c2 = idx / m;
            double sr = 0.0, si = 0.0;
            for (int q = 0; q < nreg; ++q) {
              const int r = a.region[q];
              const cplx x = Ua[r + c1 * lu], y = Ua[r + c2 * lu];
              sr += x.re * y.re + x.im * y.im;
              si += x.re * y.im - x.im * y.re;
            }
            G[idx] = cplx{sr, si};
          }
        }
        __syncthreads();
        if (m <= 64) {  // one wave: no workgroup barriers inside the reduction
          if (tid < 64) tridiag_wave(G, m, m, vv, R, dd, ee);
        } else {
          tridiag_body(G, m, m, vv, R, dd, ee, red);
        }
        __syncthreads();
        multisect_eigenvalues(dd, ee, m, lam);
        __syncthreads();
        double part = 0.0;
        for (int k = tid; k < m; k += 256) part += binary_entropy(lam[k]);
        S = block_sum256(part, red);
      }
      if (tid == 0 && n_obs < a.max_obs) a.S_out[(long)n_obs * a.B + b] = S;
      ++n_obs;
      __syncthreads();
    }
  }
  for (int idx = tid; idx < L * N; idx += 256) Ug[idx] = Ua[idx % L + (idx / L) * lu];
  if (a.protocol == 0 && a.n_steps > 0) {
    for (int e = tid; e < last_cnt; e += 256) {
      a.ev_sites[(long)b * L + e] = site[e];
      a.ev_out[(long)b * L + e] = outc[e];
      a.ev_prob[(long)b * L + e] = prob[e];
    }
    if (tid == 0) a.ev_cnt[b] = last_cnt;
  }
  if (tid == 0 && bad) {
    atomicOr(a.flag, 1);
    if (atomicCAS(&a.info->set, 0, 1) == 0) {
      a.info->source = 3;
      a.info->traj = b;
      a.info->col = bad - 1;
      a.info->pivot = bad_pivot;
    }
  }
}

__global__ __launch_bounds__(256) void fused_trajectory_kernel(FusedArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  fused_body(a, blockIdx.x, smem);
}

// One launch for several contexts: the workgroup finds its context in the table (the
// range of workgroups of each) and runs that context's trajectory with its own arguments.
__global__ __launch_bounds__(256) void fused_group_kernel(FusedGroup grp) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int id = blockIdx.x;
  int k = 0;
  while (k + 1 < grp.n && id >= grp.first[k + 1]) ++k;
  fused_body(grp.g[k], id - grp.first[k], smem);
}

hipError_t set_fused_lds_limit() {
  static std::atomic<bool> done{false};
  if (done.load()) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fused_trajectory_kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(fused_group_kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
  if (e == hipSuccess) done = true;
  return e;
}

}  // namespace

size_t fused_lds_bytes(int L, int N, int Lx, int Ly) { return fused_layout(L, N, Lx, Ly).total; }

bool fused_fits(int L, int N, int Lx, int Ly) {
  // dynamic LDS plus the kernel's static scratch must stay within one CU's 160 KiB
  return fused_layout(L, N, Lx, Ly).total <= 150 * 1024 && N <= 256;
}

hipError_t fused_run(const FusedArgs &a, int B, hipStream_t s) {
  if (B != a.B || !fused_fits(a.L, a.N, a.Lx, a.Ly)) return hipErrorInvalidValue;
  const size_t bytes = fused_lds_bytes(a.L, a.N, a.Lx, a.Ly);
  hipError_t e = set_fused_lds_limit();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fused_trajectory_kernel, dim3(B), dim3(256), bytes, s, a);
  return hipGetLastError();
}

hipError_t fused_run_group(const FusedGroup &grp, hipStream_t s) {
  if (grp.n < 1 || grp.n > FUSED_GROUP_MAX || grp.first[0] != 0) return hipErrorInvalidValue;
  size_t bytes = 0;
  for (int k = 0; k < grp.n; ++k) {
    const FusedArgs &a = grp.g[k];
    if (grp.first[k + 1] - grp.first[k] != a.B || a.B < 1 || !fused_fits(a.L, a.N, a.Lx, a.Ly))
      return hipErrorInvalidValue;
    bytes = std::max(bytes, fused_lds_bytes(a.L, a.N, a.Lx, a.Ly));
  }
  hipError_t e = set_fused_lds_limit();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fused_group_kernel, dim3(grp.first[grp.n]), dim3(256), bytes, s, grp);
  return hipGetLastError();
}

}  // namespace mfq
