// Fused small-lattice trajectory kernel: one workgroup advances one trajectory
// through many steps with its state resident in LDS, observing S_A on
// schedule, in a single launch.
//
// For small L (e.g. the L = 64 ring, U = 32 KiB) the per-phase kernels of a
// step are each far too small to fill the GPU and the step is dominated by
// launch and synchronisation latency.  Here every phase of Appendix A's step
// runs back to back inside the workgroup:
//   U' = P U (a dense product over all L^2 entries of P, whose entries are
//   generated from the ring's circulant row -- or, on the torus, the two
//   rows of P = P_y (x) P_x -- held in LDS),
//   Born probabilities + homodyne factor (Eq. (A4)) or projective
//   measurements (Eq. (A1), Eq. (A2)), two Cholesky-QR passes (Gram, Cholesky
//   and triangular inverse in LDS, U R^{-1}), and, when the absolute step is a
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

// One Cholesky-QR pass in LDS, in place: X <- X R^{-1}, R^+ R = X^+ X (upper
// R).  X has leading dimension lu (>= L); G (the Gram, then R) has leading
// dimension lg (>= N); rdiag receives the diagonal of R.  Gram with four
// independent partial sums per entry, right-looking Cholesky in one wave, then
// the triangular solve Y R = X (Y overwrites X) one row per thread.  A non-positive or
// non-finite pivot sets *bad to its column + 1 and *bad_pivot to its value (first one only).
// With certify, X is kept as it is when its Gram is within CHOL_KEEP_MAX of the identity
// entrywise (|Re| + |Im| of G - I), as the second pass of the per-phase path does.
__device__ void cholqr_lds(cplx *X, cplx *G, double *rdiag, int L, int N, int lu, int lg, int *bad,
                           double *bad_pivot, bool certify) {
  const int tid = threadIdx.x;
  // largest deviation as the bit pattern of a non-negative double (NaN orders above all)
  __shared__ unsigned long long dev_bits;
  if (tid == 0) dev_bits = 0ull;
  __syncthreads();
  double dmax = 0.0;
  for (int idx = tid; idx < N * N; idx += 256) {
    const int a = idx % N, c = idx / N;
    if (a > c) continue;
    const cplx *xa = X + a * lu, *xc = X + c * lu;
    double sr[4] = {0.0, 0.0, 0.0, 0.0}, si[4] = {0.0, 0.0, 0.0, 0.0};
    int i = 0;
    for (; i + 4 <= L; i += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const cplx p = xa[i + u], q = xc[i + u];
        sr[u] += p.re * q.re + p.im * q.im;
        si[u] += p.re * q.im - p.im * q.re;
      }
    }
    for (; i < L; ++i) {
      const cplx p = xa[i], q = xc[i];
      sr[0] += p.re * q.re + p.im * q.im;
      si[0] += p.re * q.im - p.im * q.re;
    }
    const cplx gac{(sr[0] + sr[1]) + (sr[2] + sr[3]), (si[0] + si[1]) + (si[2] + si[3])};
    G[a + c * lg] = gac;
    const double dv = fabs(a == c ? gac.re - 1.0 : gac.re) + fabs(gac.im);
    dmax = (dv != dv || dmax != dmax) ? __longlong_as_double(0x7ff8000000000000ll) : fmax(dmax, dv);
  }
  if (certify) atomicMax(&dev_bits, (unsigned long long)__double_as_longlong(dmax));
  __syncthreads();  // the Gram is written by every wave
  if (certify && __longlong_as_double((long long)dev_bits) <= CHOL_KEEP_MAX) return;
  // Cholesky by wave 0 alone: lanes of one wave run in lockstep, so the
  // column steps need only wave-level ordering, not workgroup barriers
  if (tid < 64) {
    const int lane = tid;
    for (int k = 0; k < N; ++k) {
      double d = G[k + k * lg].re;
      const bool ok = d > 0.0 && isfinite(d);
      if (lane == 0 && !ok && *bad == 0) {
        *bad = k + 1;
        *bad_pivot = d;
      }
      if (!ok) d = 1.0;
      const double rkk = sqrt(d);
      if (lane == 0) rdiag[k] = rkk;
      for (int j = k + 1 + lane; j < N; j += 64) {
        G[k + j * lg].re /= rkk;
        G[k + j * lg].im /= rkk;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const int m = N - k - 1;
      for (int idx = lane; idx < m * m; idx += 64) {
        const int i = k + 1 + idx % m, j = k + 1 + idx / m;
        if (i > j) continue;
        const cplx rki = G[k + i * lg], rkj = G[k + j * lg];
        G[i + j * lg].re -= rki.re * rkj.re + rki.im * rkj.im;
        G[i + j * lg].im -= rki.re * rkj.im - rki.im * rkj.re;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  // Y R = X row by row: each row is an independent forward substitution, so a
  // thread owns a row and no barrier is needed inside
  for (int i = tid; i < L; i += 256) {
    for (int j = 0; j < N; ++j) {
      const double inv = 1.0 / rdiag[j];
      cplx y = X[i + j * lu];
      y.re *= inv;
      y.im *= inv;
      X[i + j * lu] = y;
      for (int c = j + 1; c < N; ++c) {
        const cplx r = G[j + c * lg];
        cplx x = X[i + c * lu];
        x.re -= y.re * r.re - y.im * r.im;
        x.im -= y.re * r.im + y.im * r.re;
        X[i + c * lu] = x;
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
    // propagate: Ub = P Ua, with the dense P_ik = gx[(xi - xk) mod Lx] gy[(yi - yk) mod Ly]
    // generated from the generating rows held in LDS (all L^2 terms are summed)
    for (int idx = tid; idx < L * N; idx += 256) {
      const int i = idx % L, j = idx / L;
      const int xi = i % Lx, yi = i / Lx;
      const cplx *uj = Ua + j * lu;
      double sr = 0.0, si = 0.0;
      for (int yk = 0; yk < Ly; ++yk) {
        const int dy = yi - yk;
        const cplx py = gy[dy < 0 ? dy + Ly : dy];
        double tr4[4] = {0.0, 0.0, 0.0, 0.0}, ti4[4] = {0.0, 0.0, 0.0, 0.0};
        int xk = 0;
        for (; xk + 4 <= Lx; xk += 4) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int dx = xi - (xk + q);
            const cplx px = gx[dx < 0 ? dx + Lx : dx], u = uj[xk + q + yk * Lx];
            tr4[q] += px.re * u.re - px.im * u.im;
            ti4[q] += px.re * u.im + px.im * u.re;
          }
        }
        for (; xk < Lx; ++xk) {
          const int dx = xi - xk;
          const cplx px = gx[dx < 0 ? dx + Lx : dx], u = uj[xk + yk * Lx];
          tr4[0] += px.re * u.re - px.im * u.im;
          ti4[0] += px.re * u.im + px.im * u.re;
        }
        const double tr = (tr4[0] + tr4[1]) + (tr4[2] + tr4[3]);
        const double ti = (ti4[0] + ti4[1]) + (ti4[2] + ti4[3]);
        sr += py.re * tr - py.im * ti;
        si += py.re * ti + py.im * tr;
      }
      Ub[i + j * lu] = cplx{sr, si};
    }
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
    cholqr_lds(Ub, G, lam, L, N, lu, lg, &bad, &bad_pivot, false);
    cholqr_lds(Ub, G, lam, L, N, lu, lg, &bad, &bad_pivot, true);
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
        tridiag_body(G, m, m, vv, R, dd, ee, red);
        __syncthreads();
        for (int k = tid; k < m; k += 256) lam[k] = bisect_eigenvalue(dd, ee, m, k);
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
