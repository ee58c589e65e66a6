// Device routines shared by the per-phase kernels and the fused small-lattice
// trajectory kernel.  All of them run on one 256-thread workgroup and accept
// generic (global or LDS) pointers.
#pragma once
#include "mfq_internal.h"
#include "philox.h"

namespace mfq {

// Sum over the 256 threads of a workgroup in a fixed order (wave shuffles, then
// the four wave partials); every thread receives the result.
__device__ __forceinline__ double block_sum256(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Maximum over the 256 threads of a workgroup; every thread receives it.
__device__ __forceinline__ double block_max256(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// Sum / maximum over the NT threads of a workgroup (wave shuffles, then the wave partials in
// a fixed order); every thread receives the result.  red: NT / 64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum_nt(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) s += red[q];
  return s;
}
template <int NT>
__device__ __forceinline__ double block_max_nt(double v, double *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double m = 0.0;
#pragma unroll
  for (int q = 0; q < NT / 64; ++q) m = fmax(m, red[q]);
  return m;
}

// Vectors whose largest component is below this are treated as zero when a
// reflector is formed (dropping them changes the result by less than that).
constexpr double REFLECT_TINY = 1e-290;

// Householder reflector H = I - tau v v^+ with H x = alpha e_0,
// alpha = -phase(x_0)|x|, v = x - alpha e_0, formed from the vector scaled by
// s = its largest component magnitude (s >= REFLECT_TINY): x0s = x_0 / s,
// tail2s = sum_{i>=1} |x_i / s|^2.  The returned v0 is the first entry of the
// scaled v (the other entries are x_i / s) and tau belongs to the scaled v;
// norm = |x|.  Scaling keeps every square away from underflow, so tau is
// consistent with v and H is unitary to rounding for any magnitude of x.
struct Reflector {
  cplx v0;
  double tau, norm;
};
__device__ __forceinline__ Reflector make_reflector(cplx x0s, double tail2s, double s) {
  const double ax0 = hypot(x0s.re, x0s.im);
  const double nx = sqrt(ax0 * ax0 + tail2s);
  const double phr = ax0 > 0.0 ? x0s.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0s.im / ax0 : 0.0;
  Reflector r;
  r.v0 = cplx{x0s.re + phr * nx, x0s.im + phi * nx};
  r.tau = 2.0 / (tail2s + r.v0.re * r.v0.re + r.v0.im * r.v0.im);
  r.norm = s * nx;
  return r;
}

__device__ __forceinline__ double cmax_abs(cplx a) { return fmax(fabs(a.re), fabs(a.im)); }

// Projective measurements of one step on one trajectory (Appendix A, Eq. (A1),
// Eq. (A2) with the sign fixed), by the whole workgroup.  Ub: column-major L x N
// state with leading dimension ld; site/outcomes/probs: at least L entries;
// v: N scratch; w: L scratch.
// Sites are selected with probability q (Philox purpose 0, word 0) and
// projected in ascending order, each with its conditional Born probability
// p = |row j|^2: x = conj(row j), Householder H = I - tau v v^+ with
// H x = beta e_0, U <- U H (row j confined to column 0); outcome 1 iff
// u (word 1) <= p; outcome 1: column 0 := e_j; outcome 0: U_j0 := 0 and
// column 0 renormalised.  Returns the number of measured sites.
__device__ int pm_measure_block(cplx *Ub, int L, int N, double q, uint64_t seed, uint64_t key1,
                                uint64_t step, int *site, int *outcomes, double *probs, cplx *v,
                                cplx *w, int ld) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ int wave_cnt[4];
  __shared__ int total;
  __shared__ double red[4];
  __shared__ double sh_tau;
  __shared__ int sh_outcome, sh_skip;

  // ---- selection with ascending compaction
  if (tid == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < L; base += 256) {
    const int i = base + tid;
    bool sel = false;
    if (i < L) {
      const u64x4 r = philox4x64_10(seed, key1, step, (uint64_t)i, PURPOSE_PROJECTIVE, 0);
      sel = u01(r.v[0]) < q;
    }
    const unsigned long long m = __ballot(sel);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int off = total;
    for (int wv = 0; wv < wave; ++wv) off += wave_cnt[wv];
    if (sel) site[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
    __syncthreads();
    if (tid == 0) total += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
  const int cnt = total;

  for (int e = 0; e < cnt; ++e) {
    const int j = site[e];
    // x = conj(row j), p = |x|^2, s = largest component
    double part = 0.0, mx = 0.0;
    for (int k = tid; k < N; k += 256) {
      const cplx a = Ub[j + (long)k * ld];
      v[k] = cplx{a.re, -a.im};
      part += a.re * a.re + a.im * a.im;
      mx = fmax(mx, cmax_abs(a));
    }
    const double p = block_sum256(part, red);
    const double s = block_max256(mx, red);
    // the reflector is formed from x / s (each thread rescales its own entries)
    double part2 = 0.0;
    if (s >= REFLECT_TINY) {
      const double inv = 1.0 / s;
      for (int k = tid; k < N; k += 256) {
        const cplx a{v[k].re * inv, v[k].im * inv};
        v[k] = a;
        if (k >= 1) part2 += a.re * a.re + a.im * a.im;
      }
    }
    const double tail2 = block_sum256(part2, red);
    if (tid == 0) {
      const u64x4 r = philox4x64_10(seed, key1, step, (uint64_t)j, PURPOSE_PROJECTIVE, 0);
      const int outcome = (u01(r.v[1]) <= p) ? 1 : 0;
      sh_outcome = outcome;
      outcomes[e] = outcome;
      probs[e] = p;
      if (!(s >= REFLECT_TINY)) {
        sh_skip = 1;
      } else {
        sh_skip = 0;
        const Reflector h = make_reflector(v[0], tail2, s);
        sh_tau = h.tau;
        v[0] = h.v0;
      }
    }
    __syncthreads();
    if (sh_skip) {  // empty row (below REFLECT_TINY): outcome 0 leaves the state unchanged
      __syncthreads();
      continue;
    }
    const double tau = sh_tau;
    const int outcome = sh_outcome;
    // w = U v
    for (int i = tid; i < L; i += 256) {
      double ar = 0.0, ai = 0.0;
      for (int k = 0; k < N; ++k) {
        const cplx u = Ub[i + (long)k * ld], vk = v[k];
        ar += u.re * vk.re - u.im * vk.im;
        ai += u.re * vk.im + u.im * vk.re;
      }
      w[i] = cplx{ar * tau, ai * tau};
    }
    // U <- U - (tau w) v^+ ; row j exactly confined to column 0
    double part0 = 0.0;
    for (int i = tid; i < L; i += 256) {
      const cplx wi = w[i];
      for (int k = 1; k < N; ++k) {
        cplx u = Ub[i + (long)k * ld];
        const cplx vk = v[k];
        if (i == j) {
          u = cplx{0.0, 0.0};
        } else {
          u.re -= wi.re * vk.re + wi.im * vk.im;
          u.im -= wi.im * vk.re - wi.re * vk.im;
        }
        Ub[i + (long)k * ld] = u;
      }
      cplx c0;
      if (outcome == 1) {
        c0 = cplx{i == j ? 1.0 : 0.0, 0.0};
      } else if (i == j) {
        c0 = cplx{0.0, 0.0};
      } else {
        c0 = Ub[i];
        const cplx v0 = v[0];
        c0.re -= wi.re * v0.re + wi.im * v0.im;
        c0.im -= wi.im * v0.re - wi.re * v0.im;
        part0 += c0.re * c0.re + c0.im * c0.im;
      }
      Ub[i] = c0;
    }
    if (outcome == 0) {
      const double n0 = block_sum256(part0, red);
      const double sc = 1.0 / sqrt(n0);
      for (int i = tid; i < L; i += 256) {
        cplx c0 = Ub[i];
        c0.re *= sc;
        c0.im *= sc;
        Ub[i] = c0;
      }
    }
    __syncthreads();
  }
  return cnt;
}

// Householder tridiagonalisation of the Hermitian n x n matrix A (column-major,
// leading dimension ld, full storage), destroying A.  Step k reflects
// x = A[k+1:, k] onto alpha e_0 with H = I - tau v v^+, v = x - alpha e_0,
// alpha = -phase(x_0) |x|, and applies A22 <- H A22 H as
// A22 -= v w^+ + w v^+, w = p - (tau/2)(v^+ p) v, p = tau A22 v.
// Output: d[0:n] (diagonal), e[0:n-1] = |off-diagonal| (a diagonal unitary
// similarity makes the off-diagonal real and nonnegative).
__device__ inline void tridiag_body(cplx *A, int ld, int n, cplx *v, cplx *p, double *d, double *e,
                             double *red) {
  const int tid = threadIdx.x;
  __shared__ double s_tau;
  __shared__ int s_skip;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    cplx *x = A + (k + 1) + (long)k * ld;
    double mx = 0.0;
    for (int i = tid; i < m; i += 256) mx = fmax(mx, cmax_abs(x[i]));
    const double s = block_max256(mx, red);
    const double inv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += 256) {
      const cplx a{x[i].re * inv, x[i].im * inv};
      v[i] = a;
      part += a.re * a.re + a.im * a.im;
    }
    const double tail2 = block_sum256(part, red);
    if (tid == 0) {
      const cplx x0 = x[0];
      d[k] = A[k + (long)k * ld].re;
      if (tail2 == 0.0) {  // nothing below x0 (or all below REFLECT_TINY): H = I
        e[k] = hypot(x0.re, x0.im);
        s_skip = 1;
      } else {
        const Reflector h = make_reflector(cplx{x0.re * inv, x0.im * inv}, tail2, s);
        s_tau = h.tau;
        e[k] = h.norm;
        s_skip = 0;
        v[0] = h.v0;
      }
    }
    __syncthreads();
    if (s_skip) continue;
    const double tau = s_tau;
    cplx *A22 = A + (k + 1) + (long)(k + 1) * ld;
    // p = tau A22 v: tpr adjacent lanes per row (as many as 256 threads allow, up to 8),
    // each summing every tpr-th column, then a shuffle tree within the lanes of the row
    const int tpr = m <= 32 ? 8 : m <= 64 ? 4 : m <= 128 ? 2 : 1;
    const int sub = tid % tpr;
    for (int i0 = 0; i0 < m; i0 += 256 / tpr) {
      const int i = i0 + tid / tpr;
      double ar = 0.0, ai = 0.0;
      if (i < m)
        for (int j = sub; j < m; j += tpr) {
          const cplx a = A22[i + (long)j * ld], vj = v[j];
          ar += a.re * vj.re - a.im * vj.im;
          ai += a.re * vj.im + a.im * vj.re;
        }
      for (int o = tpr / 2; o > 0; o >>= 1) {
        ar += __shfl_xor(ar, o, 64);
        ai += __shfl_xor(ai, o, 64);
      }
      if (i < m && sub == 0) p[i] = cplx{tau * ar, tau * ai};
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
    // A22 -= v w^+ + w v^+ (entry by entry over the workgroup when m^2 is small)
    if (m <= 128) {
      for (int idx = tid; idx < m * m; idx += 256) {
        const int i = idx % m, j = idx / m;
        const cplx vi = v[i], wi = p[i], vj = v[j], wj = p[j];
        cplx a = A22[i + (long)j * ld];
        a.re -= (vi.re * wj.re + vi.im * wj.im) + (wi.re * vj.re + wi.im * vj.im);
        a.im -= (vi.im * wj.re - vi.re * wj.im) + (wi.im * vj.re - wi.re * vj.im);
        A22[i + (long)j * ld] = a;
      }
    } else {
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
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = A[(n - 2) + (long)(n - 2) * ld].re;
      const cplx t = A[(n - 1) + (long)(n - 2) * ld];
      e[n - 2] = hypot(t.re, t.im);
    }
    d[n - 1] = A[(n - 1) + (long)(n - 1) * ld].re;
  }
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

// Estimate from a final bisection bracket [lo, hi].  The spectrum of a region
// correlation matrix lies in [0, 1]; when the bracket holds 0 or 1 that bound
// is returned (exact for the 0/1 eigenvalues of product states), otherwise
// the midpoint.  Either is within the bracket width of the eigenvalue.
__device__ __forceinline__ double bracket_estimate(double lo, double hi) {
  if (lo <= 0.0 && 0.0 <= hi) return 0.0;
  if (lo <= 1.0 && 1.0 <= hi) return 1.0;
  return 0.5 * (lo + hi);
}

// Eigenvalue k (ascending) of the tridiagonal (d, e) of order n by bisection on
// its Gershgorin interval, to an absolute width of ~4 ulp(1).
__device__ inline double bisect_eigenvalue(const double *d, const double *e, int n, int k) {
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
  return bracket_estimate(lo, hi);
}

// h(x) = -x ln x - (1 - x) ln(1 - x) for x clamped to [0, 1] (Sec. II entropy formula).
__device__ inline double binary_entropy(double x) {
  x = fmin(fmax(x, 0.0), 1.0);
  if (x > 0.0 && x < 1.0) return -(x * log(x) + (1.0 - x) * log1p(-x));
  return 0.0;
}

}  // namespace mfq
