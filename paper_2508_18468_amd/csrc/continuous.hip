// Continuous-time projective protocol (Appendix A, PM protocol): one event per
// active trajectory and launch sequence.
//
// An event of trajectory b: waiting time tau = -ln(eta) / (gamma N), U <- P(tau) U
// with P(tau) = exp(-i H tau), a site j uniform over the L sites, p_j = |row j of U|^2,
// outcome 1 iff p_c <= p_j, and the exact projection of the Slater determinant
// (a Householder reflector confines row j to column 0; column 0 becomes e_j for
// outcome 1, or loses its row-j entry and is renormalised for outcome 0).  This is
// Eq. (A1) / Eq. (A2) (sign of its rank-1 term corrected) on C = U U^+, done on U.
//
// Launches per event:
//   cont_draw_kernel   one workgroup per trajectory: draws, clock, the ring rows
//                      of P(tau) (Bessel band or plane-wave sum), row j of P U,
//                      Born decision and the reflector v (H = I - tau_h v v^+)
//   cont_gemv_kernel   y = tau_h U v                         (reads U once)
//   cont_prop_kernel   yp = P(tau) y                         (vectors only)
//   cont_apply_kernel  U' = P(tau) U - yp v^+, row j / column 0 fixed
//                      (reads U once, writes U' once; on the torus the x factor
//                      runs first in a plain pass, the y factor with the update)
//   cont_norm_kernel   outcome 0: column 0 renormalised      (column 0 only)
//
// P(tau) on the ring is the circulant with generating row
// g[d] = sum over integers n = d (mod L) of (-i)^|n| J_|n|(2 J tau) (Jacobi-Anger);
// on the torus P = P_y (x) P_x with the rows of both rings.  While the Bessel
// terms beyond order M fall below 1e-20 of the largest and 2 M + 1 <= L, the row
// is the band |d| <= w (taps below that bound dropped); otherwise the full row
// comes from its plane-wave sum (1/L) sum_m exp(-i z cos k_m + i k_m d).
#include <algorithm>
#include <cmath>

#include "mfq_internal.h"
#include "device_common.h"

namespace mfq {

namespace {

constexpr double BAND_REL = 1e-20;

// Taps of one ring direction: band |d| <= w, or the whole ring (w >= period).
struct Taps {
  int lo, hi;
};
__device__ __forceinline__ Taps taps_of(int w, int period) {
  if (w < 0) return Taps{0, 0};                 // no event: identity
  if (w >= period) return Taps{0, period - 1};  // full ring
  return Taps{-w, w};
}

__device__ __forceinline__ int wrap(int a, int p) {
  a %= p;
  return a < 0 ? a + p : a;
}

// Smallest order M beyond which |J_n(x)| < BAND_REL max|J| for x = |z|: the
// transition region of J_n(x) around n = x is O(x^(1/3)) wide and the decay past
// it is faster than exp(-(n - x)^(3/2) / x^(1/2)); for x <= 1 the series
// (x/2)^n / n! is below 1e-20 by n = 25.
__device__ __forceinline__ int bessel_order_bound(double x) {
  return (int)ceil(x + 15.0 * cbrt(x) + 25.0);
}

// Miller's backward recurrence J_{n-1} = (2n/x) J_n - J_{n+1} from order ms down
// to 0 (J_{ms+1} = 0, J_ms = tiny), normalised by J_0 + 2 sum_k J_2k = 1.  The
// recurrence is stable for the decaying solution J_n in this direction; values are
// rescaled by 1e-250 whenever one exceeds 1e250 (for x >= 1e-50 one step grows a value
// by at most 2 ms / x < 1e55, so nothing overflows).  Writes jn[0..ms].
__device__ void bessel_miller(double x, int ms, double *jn) {
  double up = 0.0, cur = 1e-300;
  jn[ms] = cur;
  for (int n = ms; n >= 1; --n) {
    const double nxt = (2.0 * n / x) * cur - up;
    up = cur;
    cur = nxt;
    jn[n - 1] = nxt;
    if (fabs(nxt) > 1e250) {
      for (int k = n - 1; k <= ms; ++k) jn[k] *= 1e-250;
      up *= 1e-250;
      cur *= 1e-250;
    }
  }
  double sum = jn[0];
  for (int k = 2; k <= ms; k += 2) sum += 2.0 * jn[k];
  const double inv = 1.0 / sum;
  for (int k = 0; k <= ms; ++k) jn[k] *= inv;
}

// Ring row of P(tau) for one direction (period Lr) into g[0..Lr); returns the band
// w (w >= Lr: full ring).  Called by the whole workgroup; thread 0 runs the
// recurrence.  z = 2 J tau (any sign: J_n(-x) = (-1)^n J_n(x)).
__device__ int ring_row_dev(double z, int Lr, cplx *g, double *jn, int jcap, int *sh_w) {
  const int tid = threadIdx.x;
  const double x = fabs(z);
  if (x < 1e-50) {  // J_1(x) < 1e-50: the identity to far below rounding
    if (tid == 0) g[0] = cplx{1.0, 0.0};
    __syncthreads();
    return 0;
  }
  const int M = bessel_order_bound(x);
  const int ms = M + (int)ceil(sqrt(160.0 * (M + 1))) + 20;
  const bool band = 2 * M + 1 <= Lr && ms + 1 <= jcap;
  if (band) {
    if (tid == 0) {
      bessel_miller(x, ms, jn);
      double mx = 0.0;
      for (int n = 0; n <= M; ++n) mx = fmax(mx, fabs(jn[n]));
      int w = 0;
      for (int n = 1; n <= M; ++n)
        if (fabs(jn[n]) > BAND_REL * mx) w = n;
      *sh_w = w;
    }
    __syncthreads();
    const int w = *sh_w;
    for (int d = -w + tid; d <= w; d += blockDim.x) {
      const int n = d < 0 ? -d : d;
      double v = jn[n];
      if (z < 0.0 && (n & 1)) v = -v;
      cplx ph;
      switch (n & 3) {  // (-i)^n
        case 0: ph = cplx{v, 0.0}; break;
        case 1: ph = cplx{0.0, -v}; break;
        case 2: ph = cplx{-v, 0.0}; break;
        default: ph = cplx{0.0, v}; break;
      }
      g[wrap(d, Lr)] = ph;
    }
    __syncthreads();
    return w;
  }
  // full ring: g[d] = (1/Lr) sum_m exp(-i z cos k_m) exp(i k_m d), the integer
  // product m d reduced modulo Lr before it becomes an angle
  const double two_pi = 6.283185307179586;
  for (int d = tid; d < Lr; d += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    for (int m = 0; m < Lr; ++m) {
      const double km = two_pi * m / Lr;
      const double th = two_pi * (double)(((long)m * d) % Lr) / Lr - z * cos(km);
      double sn, cs;
      sincos(th, &sn, &cs);
      ar += cs;
      ai += sn;
    }
    g[d] = cplx{ar / Lr, ai / Lr};
  }
  __syncthreads();
  return Lr;
}

struct DrawArgs {
  const cplx *U;
  int L, N, dim, Lx, Ly;
  double J;
  const double *gamma;
  double t_end;
  uint64_t seed;
  const uint64_t *uid;
  const int64_t *step_ptr;
  int step_offset;
  const int64_t *step_base;
  ContWork w;
};

__global__ __launch_bounds__(256) void cont_draw_kernel(DrawArgs a) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int L = a.L, N = a.N, Lx = a.Lx, Ly = a.Ly;
  int *info = a.w.info + 4 * b;
  double *dinfo = a.w.dinfo + 4 * b;
  const double t0 = a.w.t[b];
  if (!(t0 < a.t_end)) {  // the trajectory has reached the end time: no event
    if (tid == 0) {
      info[0] = -1; info[1] = 0; info[2] = -1; info[3] = -1;
      dinfo[0] = 0.0; dinfo[1] = 0.0; dinfo[2] = 0.0;
    }
    return;
  }
  __shared__ double sh_tau, sh_pc, red[4];
  __shared__ int sh_j, sh_w;
  if (tid == 0) {
    const uint64_t n = (uint64_t)(*a.step_ptr + a.step_offset - a.step_base[b]);
    const u64x4 r = philox4x64_10(a.seed, a.uid[b], n, 0, PURPOSE_CONTINUOUS, 0);
    sh_tau = -log(u01(r.v[0])) / (a.gamma[b] * N);
    sh_j = (int)__umul64hi(r.v[1], (uint64_t)L);
    sh_pc = u01(r.v[2]);
  }
  __syncthreads();
  const double tau = sh_tau;
  const int j = sh_j;
  cplx *gx = a.w.g + (long)b * (Lx + Ly);
  cplx *gy = gx + Lx;
  double *jn = a.w.jn + (long)b * a.w.jcap;
  const double z = 2.0 * a.J * tau;
  const int wx = ring_row_dev(z, Lx, gx, jn, a.w.jcap, &sh_w);
  int wy = 0;
  if (a.dim == 2) {
    wy = ring_row_dev(z, Ly, gy, jn, a.w.jcap, &sh_w);
  } else if (tid == 0) {
    gy[0] = cplx{1.0, 0.0};
  }
  __syncthreads();
  // x = conj(row j of P U), p = |x|^2
  const Taps tx = taps_of(wx, Lx), ty = taps_of(a.dim == 2 ? wy : 0, Ly);
  const int xj = j % Lx, yj = j / Lx;
  const cplx *Ub = a.U + (long)b * L * N;
  cplx *v = a.w.v + (long)b * N;
  double part = 0.0, mx = 0.0;
  for (int k = tid; k < N; k += 256) {
    const cplx *Uk = Ub + (long)k * L;
    double ar = 0.0, ai = 0.0;
    for (int dy = ty.lo; dy <= ty.hi; ++dy) {
      const cplx gyv = gy[wrap(dy, Ly)];
      const int row = Lx * wrap(yj - dy, Ly);
      double sr = 0.0, si = 0.0;
      for (int dx = tx.lo; dx <= tx.hi; ++dx) {
        const cplx gv = gx[wrap(dx, Lx)], u = Uk[row + wrap(xj - dx, Lx)];
        sr += gv.re * u.re - gv.im * u.im;
        si += gv.re * u.im + gv.im * u.re;
      }
      ar += gyv.re * sr - gyv.im * si;
      ai += gyv.re * si + gyv.im * sr;
    }
    v[k] = cplx{ar, -ai};
    part += ar * ar + ai * ai;
    mx = fmax(mx, fmax(fabs(ar), fabs(ai)));
  }
  const double p = block_sum256(part, red);
  const double s = block_max256(mx, red);
  double part2 = 0.0;
  if (s >= REFLECT_TINY) {
    const double inv = 1.0 / s;
    for (int k = tid; k < N; k += 256) {
      const cplx q{v[k].re * inv, v[k].im * inv};
      v[k] = q;
      if (k >= 1) part2 += q.re * q.re + q.im * q.im;
    }
  }
  const double tail2 = block_sum256(part2, red);
  if (tid == 0) {
    double tau_h = 0.0;
    if (s >= REFLECT_TINY) {
      const Reflector h = make_reflector(v[0], tail2, s);
      v[0] = h.v0;
      tau_h = h.tau;
    }
    info[0] = j;
    info[1] = (sh_pc <= p) ? 1 : 0;
    info[2] = wx;
    info[3] = a.dim == 2 ? wy : 0;
    dinfo[0] = tau;
    dinfo[1] = p;
    dinfo[2] = tau_h;
    a.w.t[b] = t0 + tau;
  }
}

// y = tau_h U v: 64 rows per workgroup (one per lane), the four waves split the
// columns and their partial sums are added in a fixed order.
__global__ __launch_bounds__(256) void cont_gemv_kernel(const cplx *U, int L, int N, ContWork w) {
  const int b = blockIdx.y;
  if (w.info[4 * b + 2] < 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  __shared__ double sr[4][64], si[4][64];
  double ar = 0.0, ai = 0.0;
  if (i < L) {
    const cplx *Ub = U + (long)b * L * N;
    const cplx *v = w.v + (long)b * N;
    for (int k = wave; k < N; k += 4) {
      const cplx u = Ub[i + (long)k * L], vk = v[k];
      ar += u.re * vk.re - u.im * vk.im;
      ai += u.re * vk.im + u.im * vk.re;
    }
  }
  sr[wave][lane] = ar;
  si[wave][lane] = ai;
  __syncthreads();
  if (wave == 0 && i < L) {
    const double th = w.dinfo[4 * b + 2];
    const double yr = (sr[0][lane] + sr[1][lane]) + (sr[2][lane] + sr[3][lane]);
    const double yi = (si[0][lane] + si[1][lane]) + (si[2][lane] + si[3][lane]);
    w.y[(long)b * L + i] = cplx{th * yr, th * yi};
  }
}

// yp = P(tau) y (both ring factors).
__global__ __launch_bounds__(256) void cont_prop_kernel(int L, int Lx, int Ly, ContWork w) {
  const int b = blockIdx.y;
  const int *info = w.info + 4 * b;
  if (info[2] < 0) return;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= L) return;
  const cplx *gx = w.g + (long)b * (Lx + Ly), *gy = gx + Lx;
  const cplx *y = w.y + (long)b * L;
  const Taps tx = taps_of(info[2], Lx), ty = taps_of(info[3], Ly);
  const int xi = i % Lx, yi = i / Lx;
  double ar = 0.0, ai = 0.0;
  for (int dy = ty.lo; dy <= ty.hi; ++dy) {
    const cplx gyv = gy[wrap(dy, Ly)];
    const int row = Lx * wrap(yi - dy, Ly);
    double sr = 0.0, si = 0.0;
    for (int dx = tx.lo; dx <= tx.hi; ++dx) {
      const cplx gv = gx[wrap(dx, Lx)], u = y[row + wrap(xi - dx, Lx)];
      sr += gv.re * u.re - gv.im * u.im;
      si += gv.re * u.im + gv.im * u.re;
    }
    ar += gyv.re * sr - gyv.im * si;
    ai += gyv.re * si + gyv.im * sr;
  }
  w.yp[(long)b * L + i] = cplx{ar, ai};
}

// One ring factor of P(tau) applied along a direction of the lattice: site i has
// coordinate c = (i / stride) % period along it, and the tap d reads site
// i + stride ((c - d) mod period - c).  UPDATE: also subtract yp v^+ and fix row j
// and column 0 (the last factor of the event).  64 rows x 16 columns per
// workgroup: lane = row, each wave 4 columns; every load is 64 consecutive rows of
// one column except where a tap wraps around the ring.
constexpr int CONT_CPW = 4;
constexpr int RING_ROWS = 256, RING_CT = 8, RING_WMAX = 32;

// Bands the LDS ring kernel takes (ring direction of a 1d lattice only).
__device__ __forceinline__ bool ring_lds_band(int band, int L) {
  return band >= 0 && band <= RING_WMAX && 2 * band + 1 <= L;
}

template <bool UPDATE>
__device__ __forceinline__ void cont_apply_tile(const cplx *U, cplx *D, int L, int N, int stride, int period,
                                                int g_off, int band, int rb, int cb, int Lx, int Ly,
                                                const ContWork &w) {
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = rb * 64 + lane;
  const int k0 = cb * (4 * CONT_CPW) + wave * CONT_CPW;
  if (i >= L || k0 >= N) return;
  const int *info = w.info + 4 * b;
  const cplx *g = w.g + (long)b * (Lx + Ly) + g_off;
  const Taps t = taps_of(band, period);
  const cplx *Ub = U + (long)b * L * N;
  cplx *Db = D + (long)b * L * N;
  const int c = (i / stride) % period;
  const int base = i - stride * c;
  const int nk = min(CONT_CPW, N - k0);
  double ar[CONT_CPW], ai[CONT_CPW];
#pragma unroll
  for (int q = 0; q < CONT_CPW; ++q) ar[q] = ai[q] = 0.0;
  if (band < 0) {  // no event: copy
#pragma unroll
    for (int q = 0; q < CONT_CPW; ++q)
      if (q < nk) {
        const cplx u = Ub[i + (long)(k0 + q) * L];
        ar[q] = u.re;
        ai[q] = u.im;
      }
  } else {
    for (int d = t.lo; d <= t.hi; ++d) {
      const cplx gv = g[wrap(d, period)];
      const long src = base + (long)stride * wrap(c - d, period);
#pragma unroll
      for (int q = 0; q < CONT_CPW; ++q)
        if (q < nk) {
          const cplx u = Ub[src + (long)(k0 + q) * L];
          ar[q] += gv.re * u.re - gv.im * u.im;
          ai[q] += gv.re * u.im + gv.im * u.re;
        }
    }
  }
  if (UPDATE && band >= 0) {
    const int j = info[0], outcome = info[1];
    const cplx yi = w.yp[(long)b * L + i];
    const cplx *v = w.v + (long)b * N;
#pragma unroll
    for (int q = 0; q < CONT_CPW; ++q)
      if (q < nk) {
        const int k = k0 + q;
        const cplx vk = v[k];
        // - yp_i conj(v_k)
        ar[q] -= yi.re * vk.re + yi.im * vk.im;
        ai[q] -= yi.im * vk.re - yi.re * vk.im;
        if (k == 0) {
          if (outcome == 1) {
            ar[q] = i == j ? 1.0 : 0.0;
            ai[q] = 0.0;
          } else if (i == j) {
            ar[q] = ai[q] = 0.0;
          }
        } else if (i == j) {
          ar[q] = ai[q] = 0.0;
        }
      }
  }
#pragma unroll
  for (int q = 0; q < CONT_CPW; ++q)
    if (q < nk) Db[i + (long)(k0 + q) * L] = cplx{ar[q], ai[q]};
}

// Tiles of 64 rows x 16 columns; the workgroups of a trajectory stride over its ntiles
// tiles (gridDim.x of them per trajectory).
template <bool UPDATE>
__global__ __launch_bounds__(256) void cont_apply_kernel(const cplx *U, cplx *D, int L, int N, int stride,
                                                         int period, int g_off, const int *bands, int bstride,
                                                         int band_slot, int nrb, int ntiles, int Lx, int Ly,
                                                         int skip_lds_bands, ContWork w) {
  const int b = blockIdx.y;
  const int band = bands[bstride * b + band_slot];
  if (skip_lds_bands && ring_lds_band(band, L)) return;  // done by cont_ring_kernel
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
    cont_apply_tile<UPDATE>(U, D, L, N, stride, period, g_off, band, tile % nrb, tile / nrb, Lx, Ly, w);
}

// Ring (1d) event pass for bands w <= RING_WMAX: 256 rows x 8 columns per workgroup; the
// rows r0 - w .. r0 + 255 + w of those columns are staged in LDS by coalesced loads
// (the halo wraps around the ring), then each thread forms its row of P U for the eight
// columns from LDS (lanes read consecutive rows: no bank conflicts), subtracts yp v^+
// and fixes row j / column 0 like cont_apply_kernel<true>.
template <bool UPDATE>
__global__ __launch_bounds__(256) void cont_ring_kernel(const cplx *U, cplx *D, int L, int N, int nrb,
                                                        const int *bands, int bstride, int band_slot, ContWork w) {
  const int b = blockIdx.y;
  const int rb = blockIdx.x % nrb, cb = blockIdx.x / nrb;
  const int *info = w.info + 4 * b;
  const int band = bands[bstride * b + band_slot];
  if (!ring_lds_band(band, L)) return;
  __shared__ cplx s[RING_CT][RING_ROWS + 2 * RING_WMAX];
  __shared__ cplx gs[2 * RING_WMAX + 1];
  const int tid = threadIdx.x;
  const int r0 = rb * RING_ROWS, k0 = cb * RING_CT;
  const int nk = min(RING_CT, N - k0);
  const int nrows = RING_ROWS + 2 * band;
  const cplx *Ub = U + (long)b * L * N + (long)k0 * L;
  // every load of a thread is issued before the first LDS store (rows tid and 256 + tid)
  for (int r = tid; r < nrows; r += 256) {
    int rr = (r0 - band + r) % L;  // rings shorter than the tile wrap more than once
    if (rr < 0) rr += L;
    cplx x[RING_CT];
#pragma unroll
    for (int c = 0; c < RING_CT; ++c) x[c] = c < nk ? Ub[rr + (long)c * L] : cplx{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < RING_CT; ++c) s[c][r] = x[c];
  }
  const cplx *g = w.g + (long)b * (L + 1);
  for (int d = tid - band; d <= band; d += 256) gs[d + band] = g[d < 0 ? d + L : d];
  __syncthreads();
  const int i = r0 + tid;
  if (i >= L) return;
  double ar[RING_CT], ai[RING_CT];
#pragma unroll
  for (int c = 0; c < RING_CT; ++c) ar[c] = ai[c] = 0.0;
  for (int d = -band; d <= band; ++d) {
    const cplx gv = gs[d + band];
    const int r = tid + band - d;
#pragma unroll
    for (int c = 0; c < RING_CT; ++c) {
      const cplx u = s[c][r];
      ar[c] += gv.re * u.re - gv.im * u.im;
      ai[c] += gv.re * u.im + gv.im * u.re;
    }
  }
  cplx *Db = D + (long)b * L * N;
  if (!UPDATE) {  // the band alone (the deferred propagation of a block of events)
#pragma unroll
    for (int c = 0; c < RING_CT; ++c)
      if (c < nk) Db[i + (long)(k0 + c) * L] = cplx{ar[c], ai[c]};
    return;
  }
  const int j = info[0], outcome = info[1];
  const cplx yi = w.yp[(long)b * L + i];
  const cplx *v = w.v + (long)b * N;
#pragma unroll
  for (int c = 0; c < RING_CT; ++c) {
    if (c >= nk) break;
    const int k = k0 + c;
    const cplx vk = v[k];
    double xr = ar[c] - (yi.re * vk.re + yi.im * vk.im);
    double xi = ai[c] - (yi.im * vk.re - yi.re * vk.im);
    if (k == 0) {
      if (outcome == 1) {
        xr = i == j ? 1.0 : 0.0;
        xi = 0.0;
      } else if (i == j) {
        xr = xi = 0.0;
      }
    } else if (i == j) {
      xr = xi = 0.0;
    }
    Db[i + (long)k * L] = cplx{xr, xi};
  }
}

// Outcome 0: column 0 (row j already zero) renormalised.
__global__ __launch_bounds__(256) void cont_norm_kernel(cplx *U, int L, int N, ContWork w) {
  const int b = blockIdx.x;
  const int *info = w.info + 4 * b;
  if (info[2] < 0 || info[1] != 0) return;
  __shared__ double red[4];
  cplx *c0 = U + (long)b * L * N;
  double part = 0.0;
  for (int i = threadIdx.x; i < L; i += 256) part += c0[i].re * c0[i].re + c0[i].im * c0[i].im;
  const double n0 = block_sum256(part, red);
  if (!(n0 > 0.0)) return;
  const double sc = 1.0 / sqrt(n0);
  for (int i = threadIdx.x; i < L; i += 256) c0[i] = cplx{c0[i].re * sc, c0[i].im * sc};
}

// ---- deferred events on the ring (blocks of up to K events) ----
// Within a block every event is taken back to the block's start (all propagators commute):
// the state is V = V0 (I + WL WR^+) + G Z with U = P(s) V, s the time since the block's start.
// Event e (0-based in the block) reads the combined row r = sum_d g_s[d] V[j - d, :] =
// u (I + WL WR^+) + sum_f gamma_f z_f, u = sum_d g_s[d] V0[j - d, :], gamma_f = sum_d g_s[d]
// G[j - d, f]; its projection is the factor D_e = (I - tau v v^+)(I + delta e0 e0^T) =
// I + X Y^+ with X = [-tau v, delta (e0 - tau conj(v0) v)], Y = [v, e0], followed by the
// additive term g_e c_e e0^T, g_e = P(-s) e_j (the band conj(g_s[i - j]) around j):
// outcome 1: delta = -1, c_e = 1; outcome 0: delta = 1/nu - 1, c_e = -conj(alpha)/nu,
// nu = sqrt(1 - p_j), alpha the reflector's image of x = conj(r).  Hence WL gains the
// columns X + WL (WR^+ X), WR the columns Y, every earlier z_f the term (z_f X) Y^+ and
// z_e = c_e e0^T.  Storage per trajectory, column-major: WL, WR N x 2K; Zc = conj(Z)^T N x K;
// G L x K.  One workgroup per trajectory; O((2w + 1) N + N e) work per event.
struct BlockArgs {
  const cplx *U;
  int L, N, e, dim, Lx, Ly;
  double J;
  const double *gamma;
  double t_end;
  uint64_t seed;
  const uint64_t *uid;
  const int64_t *step_ptr;
  int step_offset;
  const int64_t *step_base;
  ContWork w;
  BlockWork bw;
};

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

constexpr int BLOCK_KMAX = 64;
constexpr int BLOCK_EVENT_THREADS = 512;  // two workgroups per compute unit (1024 threads: one, and a second round past 256 trajectories)

template <int NT>
__global__ __launch_bounds__(NT) void cont_block_event_kernel(BlockArgs a) {
  constexpr int NW = NT / 64;
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int L = a.L, N = a.N, K = a.bw.K, e = a.e;
  cplx *WL = a.bw.WL + (long)b * N * 2 * K;
  cplx *WR = a.bw.WR + (long)b * N * 2 * K;
  cplx *Zc = a.bw.Zc + (long)b * N * K;
  cplx *G = a.bw.G + (long)b * L * K;
  int *info = a.w.info + 4 * b;
  double *dinfo = a.w.dinfo + 4 * b;
  for (int i = tid; i < L; i += NT) G[i + (long)e * L] = cplx{0.0, 0.0};
  const double t0 = a.w.t[b];
  if (!(t0 < a.t_end)) {  // no event: the factor is the identity, no additive term
    for (int k = tid; k < N; k += NT) {
      WL[k + (long)(2 * e) * N] = WL[k + (long)(2 * e + 1) * N] = cplx{0.0, 0.0};
      WR[k + (long)(2 * e) * N] = WR[k + (long)(2 * e + 1) * N] = cplx{0.0, 0.0};
      Zc[k + (long)e * N] = cplx{0.0, 0.0};
    }
    if (tid == 0) {
      info[0] = -1; info[1] = 0; info[2] = -1;
      dinfo[0] = 0.0; dinfo[1] = 0.0; dinfo[2] = 0.0;
    }
    return;
  }
  __shared__ double sh_tau, sh_pc, red[NW];
  __shared__ int sh_j, sh_w;
  __shared__ cplx sh_q[2 * BLOCK_KMAX], sh_gam[BLOCK_KMAX], sh_h[2 * BLOCK_KMAX][2], sh_a[BLOCK_KMAX][2];
  __shared__ double sh_tauh, sh_delta;
  __shared__ cplx sh_c;
  if (tid == 0) {
    const uint64_t n = (uint64_t)(*a.step_ptr + a.step_offset - a.step_base[b]);
    const u64x4 r = philox4x64_10(a.seed, a.uid[b], n, 0, PURPOSE_CONTINUOUS, 0);
    sh_tau = -log(u01(r.v[0])) / (a.gamma[b] * N);
    sh_j = (int)__umul64hi(r.v[1], (uint64_t)L);
    sh_pc = u01(r.v[2]);
  }
  __syncthreads();
  const double tau = sh_tau, s_new = a.bw.s[b] + tau;
  const int j = sh_j;
  const int Lx = a.Lx, Ly = a.Ly;
  cplx *gx = a.w.g + (long)b * (Lx + Ly);
  cplx *gy = gx + Lx;
  double *jn = a.w.jn + (long)b * a.w.jcap;
  const int wb = ring_row_dev(2.0 * a.J * s_new, Lx, gx, jn, a.w.jcap, &sh_w);
  int wy = 0;
  if (a.dim == 2) {
    wy = ring_row_dev(2.0 * a.J * s_new, Ly, gy, jn, a.w.jcap, &sh_w);
  } else if (tid == 0) {
    gy[0] = cplx{1.0, 0.0};
  }
  __syncthreads();
  const Taps tx = taps_of(wb, Lx), ty = taps_of(a.dim == 2 ? wy : 0, Ly);
  const int xj = j % Lx, yj = j / Lx;
  // sum over the band of P(s) around site j of column c (stride ld between columns)
  auto band_row = [&](const cplx *col) -> cplx {
    double ar = 0.0, ai = 0.0;
    for (int dy = ty.lo; dy <= ty.hi; ++dy) {
      const cplx gyv = gy[wrap(dy, Ly)];
      const int row = Lx * wrap(yj - dy, Ly);
      double sr = 0.0, si = 0.0;
      for (int dx = tx.lo; dx <= tx.hi; ++dx) {
        const cplx gv = gx[wrap(dx, Lx)], v = col[row + wrap(xj - dx, Lx)];
        sr += gv.re * v.re - gv.im * v.im;
        si += gv.re * v.im + gv.im * v.re;
      }
      ar += gyv.re * sr - gyv.im * si;
      ai += gyv.re * si + gyv.im * sr;
    }
    return cplx{ar, ai};
  };
  const cplx *V0 = a.U + (long)b * L * N;
  cplx *x = a.w.v + (long)b * N;  // u, then x = conj(r), then the scaled reflector
  for (int k = tid; k < N; k += NT) x[k] = band_row(V0 + (long)k * L);
  for (int f = tid; f < e; f += NT) sh_gam[f] = band_row(G + (long)f * L);
  __syncthreads();
  // q = u WL (one wave per column, lanes over rows)
  for (int c = wave; c < 2 * e; c += NW) {
    const cplx *Wc = WL + (long)c * N;
    double qr = 0.0, qi = 0.0;
    for (int k = lane; k < N; k += 64) {
      const cplx u = x[k], w = Wc[k];
      qr += u.re * w.re - u.im * w.im;
      qi += u.re * w.im + u.im * w.re;
    }
    qr = wave_sum(qr);
    qi = wave_sum(qi);
    if (lane == 0) sh_q[c] = cplx{qr, qi};
  }
  __syncthreads();
  // r = u + q WR^+ + sum_f gamma_f z_f; x = conj(r); p = |r|^2
  double part = 0.0, mx = 0.0;
  for (int k = tid; k < N; k += NT) {
    cplx r = x[k];
    for (int c = 0; c < 2 * e; ++c) {  // + q_c conj(WR[k, c])
      const cplx q = sh_q[c], w = WR[k + (long)c * N];
      r.re += q.re * w.re + q.im * w.im;
      r.im += q.im * w.re - q.re * w.im;
    }
    for (int f = 0; f < e; ++f) {  // + gamma_f z_f[k], z_f[k] = conj(Zc[k, f])
      const cplx gm = sh_gam[f], z = Zc[k + (long)f * N];
      r.re += gm.re * z.re + gm.im * z.im;
      r.im += gm.im * z.re - gm.re * z.im;
    }
    x[k] = cplx{r.re, -r.im};
    part += r.re * r.re + r.im * r.im;
    mx = fmax(mx, fmax(fabs(r.re), fabs(r.im)));
  }
  const double p = block_sum_nt<NT>(part, red);
  const double smax = block_max_nt<NT>(mx, red);
  double part2 = 0.0;
  if (smax >= REFLECT_TINY) {
    const double inv = 1.0 / smax;
    for (int k = tid; k < N; k += NT) {
      const cplx q{x[k].re * inv, x[k].im * inv};
      x[k] = q;
      if (k >= 1) part2 += q.re * q.re + q.im * q.im;
    }
  }
  const double tail2 = block_sum_nt<NT>(part2, red);
  if (tid == 0) {
    double tau_h = 0.0;
    cplx alpha_c{0.0, 0.0};  // conj(alpha), alpha = -phase(x0) |x|
    if (smax >= REFLECT_TINY) {
      const cplx x0 = x[0];
      const Reflector h = make_reflector(x0, tail2, smax);
      const double ax0 = hypot(x0.re, x0.im);
      const double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
      alpha_c = cplx{-phr * h.norm, phi * h.norm};
      x[0] = h.v0;
      tau_h = h.tau;
    } else {
      for (int k = 0; k < N; ++k) x[k] = cplx{0.0, 0.0};
    }
    const int outcome = (sh_pc <= p) ? 1 : 0;
    sh_tauh = tau_h;
    if (outcome == 1) {
      sh_delta = -1.0;
      sh_c = cplx{1.0, 0.0};
    } else {
      const double nu = sqrt(fmax(1.0 - p, 1e-300));
      sh_delta = 1.0 / nu - 1.0;
      sh_c = cplx{-alpha_c.re / nu, -alpha_c.im / nu};
    }
    info[0] = j; info[1] = outcome; info[2] = wb;
    dinfo[0] = tau; dinfo[1] = p; dinfo[2] = tau_h;
  }
  __syncthreads();
  const double th = sh_tauh, dl = sh_delta;
  const cplx v0 = x[0];
  // X[k] = (-th v_k, dl (delta_k0 - th conj(v0) v_k))
  auto Xk = [&](int k, int m) -> cplx {
    const cplx v = x[k];
    if (m == 0) return cplx{-th * v.re, -th * v.im};
    // conj(v0) v
    const double cr = v0.re * v.re + v0.im * v.im, ci = v0.re * v.im - v0.im * v.re;
    return cplx{dl * ((k == 0 ? 1.0 : 0.0) - th * cr), -dl * th * ci};
  };
  // h = WR^+ X (2e x 2) and a_f = z_f X (e x 2), z_f[k] = conj(Zc[k, f])
  for (int c = wave; c < 2 * e + e; c += NW) {
    const bool isW = c < 2 * e;
    const cplx *col = isW ? WR + (long)c * N : Zc + (long)(c - 2 * e) * N;
    double r0 = 0.0, i0 = 0.0, r1 = 0.0, i1 = 0.0;
    for (int k = lane; k < N; k += 64) {
      const cplx w = col[k];  // conj(w) X for both (WR^+ and conj(Zc))
      const cplx X0 = Xk(k, 0), X1 = Xk(k, 1);
      r0 += w.re * X0.re + w.im * X0.im;
      i0 += w.re * X0.im - w.im * X0.re;
      r1 += w.re * X1.re + w.im * X1.im;
      i1 += w.re * X1.im - w.im * X1.re;
    }
    r0 = wave_sum(r0); i0 = wave_sum(i0); r1 = wave_sum(r1); i1 = wave_sum(i1);
    if (lane == 0) {
      if (isW) {
        sh_h[c][0] = cplx{r0, i0};
        sh_h[c][1] = cplx{r1, i1};
      } else {
        sh_a[c - 2 * e][0] = cplx{r0, i0};
        sh_a[c - 2 * e][1] = cplx{r1, i1};
      }
    }
  }
  __syncthreads();
  for (int k = tid; k < N; k += NT) {
    // WL columns 2e, 2e+1: X + WL h
    cplx n0 = Xk(k, 0), n1 = Xk(k, 1);
    for (int c = 0; c < 2 * e; ++c) {
      const cplx w = WL[k + (long)c * N], h0 = sh_h[c][0], h1 = sh_h[c][1];
      n0.re += w.re * h0.re - w.im * h0.im;
      n0.im += w.re * h0.im + w.im * h0.re;
      n1.re += w.re * h1.re - w.im * h1.im;
      n1.im += w.re * h1.im + w.im * h1.re;
    }
    WL[k + (long)(2 * e) * N] = n0;
    WL[k + (long)(2 * e + 1) * N] = n1;
    const cplx vk = x[k];
    WR[k + (long)(2 * e) * N] = vk;
    WR[k + (long)(2 * e + 1) * N] = cplx{k == 0 ? 1.0 : 0.0, 0.0};
    // earlier additive rows: z_f += a_f0 conj(Y0) + a_f1 conj(Y1), stored conjugated
    for (int f = 0; f < e; ++f) {
      const cplx a0 = sh_a[f][0], a1 = sh_a[f][1];
      cplx z = Zc[k + (long)f * N];
      // + conj(a0) v_k + conj(a1) delta_k0
      z.re += a0.re * vk.re + a0.im * vk.im;
      z.im += a0.re * vk.im - a0.im * vk.re;
      if (k == 0) {
        z.re += a1.re;
        z.im -= a1.im;
      }
      Zc[k + (long)f * N] = z;
    }
    Zc[k + (long)e * N] = k == 0 ? cplx{sh_c.re, -sh_c.im} : cplx{0.0, 0.0};
  }
  // g_e = P(-s) e_j: G[(xj + dx, yj + dy), e] = conj(gx[dx] gy[dy]) over the band
  {
    const int nx = tx.hi - tx.lo + 1, ny = ty.hi - ty.lo + 1;
    for (int q = tid; q < nx * ny; q += NT) {
      const int dx = tx.lo + q % nx, dy = ty.lo + q / nx;
      const cplx u = gx[wrap(dx, Lx)], v = gy[wrap(dy, Ly)];
      const double pr = u.re * v.re - u.im * v.im, pi = u.re * v.im + u.im * v.re;
      G[wrap(xj + dx, Lx) + Lx * wrap(yj + dy, Ly) + (long)e * L] = cplx{pr, -pi};
    }
  }
  if (tid == 0) {
    a.bw.s[b] = s_new;
    a.w.t[b] = t0 + tau;
  }
}

// Ring rows of P(s) for the time accumulated since the block's start (bands in fb: x, y);
// the block clock restarts.
__global__ __launch_bounds__(256) void cont_block_rows_kernel(int dim, int Lx, int Ly, double J, ContWork w,
                                                              BlockWork bw) {
  const int b = blockIdx.x;
  __shared__ int sh_w;
  const double sb = bw.s[b];
  cplx *gx = w.g + (long)b * (Lx + Ly);
  double *jn = w.jn + (long)b * w.jcap;
  const int wx = ring_row_dev(2.0 * J * sb, Lx, gx, jn, w.jcap, &sh_w);
  int wy = 0;
  if (dim == 2) wy = ring_row_dev(2.0 * J * sb, Ly, gx + Lx, jn, w.jcap, &sh_w);
  else if (threadIdx.x == 0) gx[Lx] = cplx{1.0, 0.0};
  if (threadIdx.x == 0) {
    bw.fb[2 * b] = wx;
    bw.fb[2 * b + 1] = wy;
    bw.s[b] = 0.0;
  }
}

__global__ void clock_set_kernel(double *t, int first, int count, double value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) t[first + i] = value;
}

}  // namespace

hipError_t cont_clock_set(double *t, int first, int count, double value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(clock_set_kernel, dim3((count + 255) / 256), dim3(256), 0, s, t, first, count, value);
  return hipGetLastError();
}

hipError_t cont_event(cplx *Ua, cplx *Ub, int L, int N, int B, int dim, int Lx, int Ly, double J,
                      const double *gamma, double t_end, uint64_t seed, const uint64_t *uid,
                      const int64_t *step_ptr, int step_offset, const int64_t *step_base,
                      const ContWork &w, bool *state_in_b, hipStream_t s) {
  if (L != Lx * (dim == 2 ? Ly : 1) || N < 1 || B < 1 || w.jcap < 1) return hipErrorInvalidValue;
  if (dim == 1 && Ly != 1) return hipErrorInvalidValue;
  DrawArgs a{Ua, L, N, dim, Lx, Ly, J, gamma, t_end, seed, uid, step_ptr, step_offset, step_base, w};
  hipLaunchKernelGGL(cont_draw_kernel, dim3(B), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cont_gemv_kernel, dim3((L + 63) / 64, B), dim3(256), 0, s, (const cplx *)Ua, L, N, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cont_prop_kernel, dim3((L + 255) / 256, B), dim3(256), 0, s, L, Lx, Ly, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nrb = (L + 63) / 64, ncb = (N + 4 * CONT_CPW - 1) / (4 * CONT_CPW), ntiles = nrb * ncb;
  cplx *out;
  if (dim == 1) {
    // narrow bands through LDS; wide bands, full rows and trajectories without an event
    // by the direct pass, whose few workgroups per trajectory exit at once otherwise
    const int rnb = (L + RING_ROWS - 1) / RING_ROWS, rcb = (N + RING_CT - 1) / RING_CT;
    hipLaunchKernelGGL(cont_ring_kernel<true>, dim3((unsigned)(rnb * rcb), B), dim3(256), 0, s, (const cplx *)Ua,
                       Ub, L, N, rnb, (const int *)w.info, 4, 2, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const dim3 few((unsigned)std::min(ntiles, 8), B);
    hipLaunchKernelGGL(cont_apply_kernel<true>, few, dim3(256), 0, s, (const cplx *)Ua, Ub, L, N, 1, Lx, 0,
                       (const int *)w.info, 4, 2, nrb, ntiles, Lx, Ly, 1, w);
    out = Ub;
    *state_in_b = true;
  } else {
    const dim3 grid((unsigned)ntiles, B);
    hipLaunchKernelGGL(cont_apply_kernel<false>, grid, dim3(256), 0, s, (const cplx *)Ua, Ub, L, N, 1, Lx, 0,
                       (const int *)w.info, 4, 2, nrb, ntiles, Lx, Ly, 0, w);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(cont_apply_kernel<true>, grid, dim3(256), 0, s, (const cplx *)Ub, Ua, L, N, Lx, Ly, Lx,
                       (const int *)w.info, 4, 3, nrb, ntiles, Lx, Ly, 0, w);
    out = Ua;
    *state_in_b = false;
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(cont_norm_kernel, dim3(B), dim3(256), 0, s, out, L, N, w);
  return hipGetLastError();
}

hipError_t cont_block_event(const cplx *U, int L, int N, int B, int e, int dim, int Lx, int Ly, double J,
                            const double *gamma,
                            double t_end, uint64_t seed, const uint64_t *uid, const int64_t *step_ptr,
                            int step_offset, const int64_t *step_base, const ContWork &w, const BlockWork &bw,
                            hipStream_t s) {
  if (bw.K < 1 || bw.K > BLOCK_KMAX || e < 0 || e >= bw.K || N < 1 || B < 1) return hipErrorInvalidValue;
  if (L != Lx * (dim == 2 ? Ly : 1) || (dim == 1 && Ly != 1)) return hipErrorInvalidValue;
  BlockArgs a{U, L, N, e, dim, Lx, Ly, J, gamma, t_end, seed, uid, step_ptr, step_offset, step_base, w, bw};
  hipLaunchKernelGGL(cont_block_event_kernel<BLOCK_EVENT_THREADS>, dim3(B), dim3(BLOCK_EVENT_THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t cont_block_flush(cplx *Ua, cplx *Ub, int L, int N, int B, int e, int dim, int Lx, int Ly, double J,
                            const ContWork &w, const BlockWork &bw, bool *state_in_b, hipStream_t s) {
  if (e < 1 || e > bw.K) return hipErrorInvalidValue;
  const int K = bw.K;
  hipError_t err;
  {  // T1 = V0 WL
    GemmDesc g{};
    g.alpha = cplx{1.0, 0.0};
    g.M = L; g.N = 2 * e; g.K = N; g.batch = B;
    g.A = Ua; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
    g.B = bw.WL; g.ldb = N; g.sB = (long)N * 2 * K; g.opB = OP_N;
    g.D = bw.T1; g.ldd = L; g.sD = (long)L * 2 * K;
    if ((err = zgemm(g, s)) != hipSuccess) return err;
  }
  {  // V0 += T1 WR^+  (in place: each entry is read and written by one thread)
    GemmDesc g{};
    g.alpha = cplx{1.0, 0.0};
    g.beta = cplx{1.0, 0.0};
    g.M = L; g.N = N; g.K = 2 * e; g.batch = B;
    g.A = bw.T1; g.lda = L; g.sA = (long)L * 2 * K; g.opA = OP_N;
    g.B = bw.WR; g.ldb = N; g.sB = (long)N * 2 * K; g.opB = OP_C;
    g.Cin = Ua; g.ldcin = L; g.sCin = (long)L * N;
    g.D = Ua; g.ldd = L; g.sD = (long)L * N;
    if ((err = zgemm(g, s)) != hipSuccess) return err;
  }
  {  // V0 += G Z, Z = Zc^+
    GemmDesc g{};
    g.alpha = cplx{1.0, 0.0};
    g.beta = cplx{1.0, 0.0};
    g.M = L; g.N = N; g.K = e; g.batch = B;
    g.A = bw.G; g.lda = L; g.sA = (long)L * K; g.opA = OP_N;
    g.B = bw.Zc; g.ldb = N; g.sB = (long)N * K; g.opB = OP_C;
    g.Cin = Ua; g.ldcin = L; g.sCin = (long)L * N;
    g.D = Ua; g.ldd = L; g.sD = (long)L * N;
    if ((err = zgemm(g, s)) != hipSuccess) return err;
  }
  // U = P(s) V: the rows for each trajectory's time since the block's start, then the band(s)
  hipLaunchKernelGGL(cont_block_rows_kernel, dim3(B), dim3(256), 0, s, dim, Lx, Ly, J, w, bw);
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int nrb = (L + 63) / 64, ncb = (N + 4 * CONT_CPW - 1) / (4 * CONT_CPW), ntiles = nrb * ncb;
  if (dim == 1) {
    const int rnb = (L + RING_ROWS - 1) / RING_ROWS, rcb = (N + RING_CT - 1) / RING_CT;
    hipLaunchKernelGGL(cont_ring_kernel<false>, dim3((unsigned)(rnb * rcb), B), dim3(256), 0, s, (const cplx *)Ua,
                       Ub, L, N, rnb, (const int *)bw.fb, 2, 0, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(cont_apply_kernel<false>, dim3((unsigned)std::min(ntiles, 8), B), dim3(256), 0, s,
                       (const cplx *)Ua, Ub, L, N, 1, L, 0, (const int *)bw.fb, 2, 0, nrb, ntiles, L, 1, 1, w);
    *state_in_b = true;
  } else {  // P_x then P_y, back into Ua
    const dim3 grid((unsigned)ntiles, B);
    hipLaunchKernelGGL(cont_apply_kernel<false>, grid, dim3(256), 0, s, (const cplx *)Ua, Ub, L, N, 1, Lx, 0,
                       (const int *)bw.fb, 2, 0, nrb, ntiles, Lx, Ly, 0, w);
    if ((err = hipGetLastError()) != hipSuccess) return err;
    hipLaunchKernelGGL(cont_apply_kernel<false>, grid, dim3(256), 0, s, (const cplx *)Ub, Ua, L, N, Lx, Ly, Lx,
                       (const int *)bw.fb, 2, 1, nrb, ntiles, Lx, Ly, 0, w);
    *state_in_b = false;
  }
  return hipGetLastError();
}

}  // namespace mfq
