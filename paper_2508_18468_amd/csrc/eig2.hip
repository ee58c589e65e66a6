// Two-stage reduction of large Hermitian region Grams to real symmetric tridiagonal form, for
// the eigenvalues of the Sec. II entropy formula (the spectrum of C restricted to A).
//
// The one-stage blocked reduction (eig.hip) reads the trailing matrix once per reflector:
// about 8 n^3 / 3 bytes per matrix, bound by HBM.  Here the matrix is first reduced to a band
// of half-width TRD2_SB by block reflectors whose two-sided updates are matrix-core products
// (about 16 n^3 / 3 flop; the lower triangle of the trailing matrix is read three times and
// written once per panel of TRD2_SB columns),
// then the band is reduced to tridiagonal form by bulge chasing, whose work is O(n^2 TRD2_SB):
//
//   stage 1, per panel of TRD2_SB columns starting at column j (rows below the band:
//     m = n - j - TRD2_SB): Householder QR of the m x TRD2_SB panel, column by column (rows
//     spread over the grid; every workgroup reduces the per-workgroup column statistics of the
//     previous column in the same fixed order, so all of them form the same reflector) in one
//     kernel whose workgroups meet at a counter before each column, or one launch per column
//     where that grid would not fit the GPU at once,
//     leaving R in the band and zeros below it; then with Q = I - V T V^+ (compact WY),
//     A22 <- Q^+ A22 Q = A22 - V W^+ - W V^+,  W = X - (1/2) V (T^+ (V^+ X)),  X = A22 (V T),
//     the deep products split over K into slices summed in a fixed order.  Only the lower
//     triangle of A22 is kept: X is formed as tril(A22) (V T) + (strictly lower part)^+ (V T),
//     and the update writes the tiles on and below the diagonal;
//   stage 2, sweep j (column j) and task t: a reflector of length <= TRD2_SB removes column j
//     below the sub-diagonal (t = 0) or the first column of the bulge task t - 1 created
//     (t >= 1), applied to the rows it mixes (left), to its diagonal block (two-sided) and to
//     the block below (right), which creates the next bulge.  The rest of a bulge is removed
//     by later sweeps, so the lower triangle never holds entries beyond distance 2 TRD2_SB - 1
//     from the diagonal; stage 2 reads and writes only those.  Task t of sweep j shares entries
//     with tasks up to t + 2 of sweep j - 1 and with none beyond, so workgroups take sweeps in
//     order from a counter and start task t once sweep j - 1 has finished task t + 2 (a
//     bounded wait on its progress word: a wait beyond the limit sets the error word and every
//     workgroup leaves).
//
// Reflectors are Hermitian, H = I - tau v v^+ with real tau (make_reflector), formed from the
// vector scaled by its largest component.  The final tridiagonal has complex sub-diagonal
// entries; a diagonal unitary similarity makes them |e_i| without changing the spectrum.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "device_common.h"
#include "panel_admission.h"

namespace mfq {

namespace {

constexpr int SB = TRD2_SB;
constexpr int PAYC = 2 + 2 * SB;  // complex entries of one workgroup's column statistics
constexpr int P1_RPW = TRD2_RPW;  // panel rows per workgroup of the column launches

// Per-matrix scratch inside EigWork::panel (complex units from the matrix's base).
struct Scratch {
  cplx *X, *Y, *VT, *KP, *S, *T, *Z, *M2, *TAU, *PAY;
  int *prog;   // n progress words, the sweep counter at prog[n], the abort word at prog[n + 1],
               // the panel counter of stage 1 at prog[n + 2]
};
__host__ __device__ inline Scratch scratch_of(cplx *base, int n, int g1) {
  Scratch s;
  s.X = base;
  s.Y = s.X + 2L * SB * n;
  s.VT = s.Y + 2L * SB * n;
  s.KP = s.VT + (long)SB * n;
  s.S = s.KP + trd2_kp_elems(n);
  s.T = s.S + SB * SB;
  s.Z = s.T + SB * SB;
  s.M2 = s.Z + SB * SB;
  s.TAU = s.M2 + SB * SB;
  s.PAY = s.TAU + SB;
  s.prog = reinterpret_cast<int *>(s.PAY + (long)g1 * 2 * PAYC);
  return s;
}

__device__ __forceinline__ cplx conj_mul(cplx a, cplx b) {  // conj(a) b
  return cplx{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

__device__ __forceinline__ double wsum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// ------------------------------------------------------------------ stage 1: panel QR
// Launch k (0 <= k < kmax) of the panel at column j: reduces the statistics of column k that
// launch k - 1 left (parity k & 1), forms reflector k, applies it to the workgroup's rows of
// columns k+1 .. SB-1, writes column k of V (the X buffer) and column k of the panel (alpha
// on the pivot row, zeros below), and leaves the statistics of column k + 1 (parity
// (k + 1) & 1).  Launch k = -1 only leaves the statistics of column 0 (and zeroes V and tau).
// Statistics of workgroup g for column c: its largest |x_i| over rows i >= c (s_g), the sum of
// |x_i / s_g|^2 over rows i > c, the sums conj(x_i / s_g) P[i, c'] over rows i > c for every
// c' > c, and, from the workgroup holding row c, the pivot row P[c, c'] (c' >= c).
__device__ __forceinline__ void p1_col_step(const EigWork &W, int n, int j, int m, int k, int kmax, int g1,
                                            int gm) {
  const int b = blockIdx.y, g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cplx *A = W.A + (long)b * n * n;
  cplx *P = A + (j + SB) + (long)j * n;  // panel: rows 0 .. m-1, columns 0 .. SB-1, ld n
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  const int r_lo = g * P1_RPW, r_hi = min(m, r_lo + P1_RPW);
  __shared__ double red[4];
  constexpr int NG = 256 / SB;
  __shared__ cplx sw[SB], spiv[SB], dpart[NG][SB];
  __shared__ cplx lx[P1_RPW], lx1[P1_RPW];
  static_assert(P1_RPW <= 256, "one row per thread for columns k and k + 1");
  __shared__ double s_tau, s_inv;
  __shared__ cplx s_v0, s_alpha;
  __shared__ int s_skip;
  const int kk = k + 1;  // column whose statistics this launch leaves
  // this workgroup's panel entries, loaded first so that their latency overlaps the reduction
  // of the statistics: columns k and kk of row r_lo + tid, and the rows of columns c > k
  // (wave c % 4) in registers
  constexpr int CU = SB / 4, CH = P1_RPW / 64;
  cplx xk{0.0, 0.0}, xkk{0.0, 0.0};
  if (r_lo + tid < r_hi) {
    if (k >= 0) xk = P[r_lo + tid + (long)k * n];
    if (kk < SB) xkk = P[r_lo + tid + (long)kk * n];
  }
  cplx yv[CU][CH];
#pragma unroll
  for (int u = 0; u < CU; ++u)
#pragma unroll
    for (int h2 = 0; h2 < CH; ++h2) {
      const int c = k + 1 + wave + 4 * u, r = r_lo + lane + 64 * h2;
      yv[u][h2] = (c < SB && c != kk && r < r_hi) ? P[r + (long)c * n] : cplx{0.0, 0.0};
    }
  if (k < 0) {
    // zero V and tau for the panel (columns >= kmax keep tau = 0 and an empty V column)
    for (int c = wave; c < SB; c += 4)
      for (int r = r_lo + lane; r < r_hi; r += 64) sc.X[r + (long)c * n] = cplx{0.0, 0.0};
    if (g == 0 && tid < SB) sc.TAU[tid] = cplx{0.0, 0.0};
    if (tid == 0) { s_tau = 0.0; s_skip = 1; s_inv = 0.0; s_v0 = cplx{0.0, 0.0}; }
  } else {
    // reduce the statistics of column k over the workgroups, in the same order everywhere
    const cplx *pay = sc.PAY + (long)(k & 1) * g1 * PAYC;
    double mx = 0.0;
    for (int q = tid; q < gm; q += 256) mx = fmax(mx, pay[(long)q * PAYC].re);
    const double s = block_max256(mx, red);
    const double sinv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
    double part = 0.0;
    for (int q = tid; q < gm; q += 256) {
      const cplx st = pay[(long)q * PAYC];
      const double f = st.re * sinv;
      part += f * f * st.im;
    }
    const double tail2 = block_sum256(part, red);
    {
      const int c = tid % SB, grp = tid / SB;  // NG = 256 / SB groups of workgroups' statistics
      double dr = 0.0, di = 0.0;
      if (c > k)
#pragma unroll 16
        for (int q = grp; q < gm; q += NG) {
          const cplx *pq = pay + (long)q * PAYC;
          const double f = pq[0].re * sinv;
          dr += f * pq[2 + SB + c].re;
          di += f * pq[2 + SB + c].im;
        }
      dpart[grp][c] = cplx{dr, di};
      const int owner = k / P1_RPW;
      if (grp == 0) spiv[c] = pay[(long)owner * PAYC + 2 + c];
    }
    __syncthreads();
    if (tid == 0) {
      const cplx x0 = spiv[k];
      if (!(tail2 > 0.0)) {  // nothing below the pivot (or all below REFLECT_TINY): H = I
        s_skip = 1;
        s_tau = 0.0;
        s_alpha = x0;
        s_v0 = cplx{1.0, 0.0};
        s_inv = 0.0;
      } else {
        const Reflector h = make_reflector(cplx{x0.re * sinv, x0.im * sinv}, tail2, s);
        const double ax0 = hypot(x0.re, x0.im);
        const double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
        s_skip = 0;
        s_tau = h.tau;
        s_v0 = h.v0;
        s_inv = sinv;
        s_alpha = cplx{-phr * h.norm, -phi * h.norm};
      }
    }
    __syncthreads();
    if (tid < SB) {  // w_c = v^+ P[:, c] = conj(v0) P[k, c] + sum_{i>k} conj(x_i / s) P[i, c]
      cplx wc{0.0, 0.0};
      if (tid > k && !s_skip) {
        cplx d{0.0, 0.0};
#pragma unroll
        for (int g2 = 0; g2 < NG; ++g2) {
          d.re += dpart[g2][tid].re;
          d.im += dpart[g2][tid].im;
        }
        const cplx t = conj_mul(s_v0, spiv[tid]);
        wc = cplx{t.re + d.re, t.im + d.im};
      }
      sw[tid] = wc;
    }
    if (g == 0 && tid == 0) sc.TAU[k] = cplx{s_tau, 0.0};
  }
  // old column k (rows of this workgroup) and the updated column kk
  if (r_lo + tid < r_hi) {
    lx[tid] = xk;
    lx1[tid] = xkk;
  }
  __syncthreads();
  const bool upd = k >= 0 && !s_skip;
  const double tau = s_tau, inv = s_inv;
  const cplx v0 = s_v0;
  auto vrow = [&](int r) -> cplx {  // entry r of the scaled reflector vector
    if (r == k) return v0;
    const cplx x = lx[r - r_lo];
    return cplx{x.re * inv, x.im * inv};
  };
  if (kk < SB && upd) {
    const cplx w1 = sw[kk];
    for (int r = max(r_lo, k) + tid; r < r_hi; r += 256) {
      const cplx v = vrow(r);
      cplx y = lx1[r - r_lo];
      y.re -= tau * (v.re * w1.re - v.im * w1.im);
      y.im -= tau * (v.re * w1.im + v.im * w1.re);
      lx1[r - r_lo] = y;
    }
  }
  __syncthreads();
  // statistics of column kk over rows >= kk (scale) and > kk (sum of squares)
  double sg = 0.0, ss = 0.0;
  if (kk < kmax) {
    double mxl = 0.0;
    for (int r = max(r_lo, kk) + tid; r < r_hi; r += 256) mxl = fmax(mxl, cmax_abs(lx1[r - r_lo]));
    sg = block_max256(mxl, red);
    const double gi = sg >= REFLECT_TINY ? 1.0 / sg : 0.0;
    double pt = 0.0;
    for (int r = max(r_lo, kk + 1) + tid; r < r_hi; r += 256) {
      const cplx y = lx1[r - r_lo];
      const double a = y.re * gi, bb = y.im * gi;
      pt += a * a + bb * bb;
    }
    ss = block_sum256(pt, red);
  }
  const double gi = sg >= REFLECT_TINY ? 1.0 / sg : 0.0;
  cplx *payo = sc.PAY + ((long)(kk & 1) * g1 + g) * PAYC;
  const bool owns_kk = kk < kmax && kk >= r_lo && kk < r_hi;
  // columns c > k (wave c % 4): all of this workgroup's rows loaded at once, then updated, the
  // dots with column kk formed (c > kk) and the pivot row of kk recorded
#pragma unroll
  for (int u = 0; u < CU; ++u) {
    const int c = k + 1 + wave + 4 * u;
    if (c >= SB) break;  // uniform over the wave
    double dr = 0.0, di = 0.0;
    const cplx wc = upd ? sw[c] : cplx{0.0, 0.0};
#pragma unroll
    for (int h2 = 0; h2 < CH; ++h2) {
      const int r = r_lo + lane + 64 * h2;
      if (r >= r_hi) continue;
      cplx y;
      if (c == kk) {
        y = lx1[r - r_lo];
      } else {
        y = yv[u][h2];
        if (upd && r >= k) {
          const cplx v = vrow(r);
          y.re -= tau * (v.re * wc.re - v.im * wc.im);
          y.im -= tau * (v.re * wc.im + v.im * wc.re);
        }
      }
      if (upd && r >= k) P[r + (long)c * n] = y;
      if (kk < kmax && c > kk && r > kk) {
        const cplx xs{lx1[r - r_lo].re * gi, lx1[r - r_lo].im * gi};
        const cplx t = conj_mul(xs, y);
        dr += t.re;
        di += t.im;
      }
      if (owns_kk && r == kk) payo[2 + c] = y;
    }
    if (kk < kmax && c > kk) {
      dr = wsum(dr);
      di = wsum(di);
      if (lane == 0) payo[2 + SB + c] = cplx{dr, di};
    }
  }
  if (tid == 0 && kk < kmax) {
    payo[0] = cplx{sg, ss};
    payo[1] = cplx{owns_kk ? 1.0 : 0.0, 0.0};
  }
  // column k: V (scaled reflector vector, zero above the pivot) and the panel's column
  // (alpha on the pivot row, zeros below)
  if (k >= 0) {
    for (int r = r_lo + tid; r < r_hi; r += 256) {
      cplx v{0.0, 0.0};
      if (r >= k) v = s_skip ? (r == k ? cplx{1.0, 0.0} : cplx{0.0, 0.0}) : vrow(r);
      sc.X[r + (long)k * n] = v;
      if (r == k) P[r + (long)k * n] = s_alpha;
      else if (r > k) P[r + (long)k * n] = cplx{0.0, 0.0};
    }
  }
}

__global__ __launch_bounds__(256) void p1_col_kernel(EigWork W, int n, int j, int m, int k, int kmax, int g1,
                                                     int gm) {
  p1_col_step(W, n, j, m, k, kmax, g1, gm);
}

// All column launches of one panel as one kernel: before column k (k >= 0) every workgroup
// waits until all gm workgroups of its matrix have finished column k - 1, counted on a
// per-matrix counter that started the panel at `base` (the statistics that column k reduces
// are then complete, and the buffer that column k overwrites is no longer read).  Workgroups
// therefore depend on workgroups that may not have started: the host launches this kernel only
// when its grid, with those of the panel kernels of other streams that may run beside it, fits
// the GPU at once (launch_panel).  A wait longer than `limit` wall-clock ticks sets the abort
// word and the context's error flag, and every workgroup leaves.
__global__ __launch_bounds__(256) void p1_panel_kernel(EigWork W, int n, int j, int m, int kmax, int g1, int gm,
                                                       int base, long long limit) {
  const int b = blockIdx.y, tid = threadIdx.x;
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  int *ctr = sc.prog + n + 2, *abort_w = sc.prog + n + 1;
  __shared__ int s_go;
  for (int k = -1; k < kmax; ++k) {
    if (k >= 0) {
      if (tid == 0) {
        int go = 1;
        const int need = base + gm * (k + 1);
        long long t0 = -1;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (__hip_atomic_load(abort_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            go = 0;
            break;
          }
          const long long now = wall_clock64();
          if (t0 < 0) t0 = now;
          if (now - t0 > limit) {
            __hip_atomic_store(abort_w, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(W.flag, 1);
            if (atomicCAS(&W.info->set, 0, 1) == 0) {
              W.info->source = 5;
              W.info->traj = b;
              W.info->col = j + k;
              W.info->pivot = 0.0;
            }
            go = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        s_go = go;
      }
      __syncthreads();
      if (!s_go) return;
    }
    p1_col_step(W, n, j, m, k, kmax, g1, gm);
    // the barrier completes every wave's stores of column k, thread 0 releases them
    __syncthreads();
    if (tid == 0) __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// T of the panel's compact-WY factor from the Gram S = V^+ V: T_kk = tau_k,
// T[0:k, k] = -tau_k T[0:k, 0:k] S[0:k, k]; thread i owns row i of T (in LDS, beside S).
// Zeros below the diagonal.
__global__ __launch_bounds__(SB) void p1_tfactor_kernel(EigWork W, int n, int g1) {
  const int b = blockIdx.x, i = threadIdx.x;
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  __shared__ cplx Ss[SB][SB + 1], Ts[SB][SB + 1];  // [column][row]
  __shared__ double tau[SB];
  for (int k = 0; k < SB; ++k) Ss[k][i] = sc.S[i + k * SB];
  tau[i] = sc.TAU[i].re;
  __syncthreads();
  for (int k = 0; k < SB; ++k) {
    const double tk = tau[k];
    cplx t{0.0, 0.0};
    if (i == k) {
      t = cplx{tk, 0.0};
    } else if (i < k && tk != 0.0) {
      double ar = 0.0, ai = 0.0;
      for (int l = i; l < k; ++l) {
        const cplx a = Ts[l][i], s = Ss[k][l];
        ar += a.re * s.re - a.im * s.im;
        ai += a.re * s.im + a.im * s.re;
      }
      t = cplx{-tk * ar, -tk * ai};
    }
    Ts[k][i] = t;
  }
  for (int k = 0; k < SB; ++k) sc.T[i + k * SB] = Ts[k][i];
}

// out = sum over the ks slices of part (each rows x cols, ld rows), in slice order.
__global__ __launch_bounds__(256) void p1_ksum_kernel(EigWork W, int n, int g1, int which, int rows, int ks,
                                                      long ldo) {
  const int b = blockIdx.y;
  const long idx = blockIdx.x * 256L + threadIdx.x;
  if (idx >= (long)rows * SB) return;
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  const long r = idx % rows, c = idx / rows;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < ks; ++q) {
    const cplx x = sc.KP[(long)q * rows * SB + idx];
    re += x.re;
    im += x.im;
  }
  cplx *out = which == 0 ? sc.S : (which == 1 ? sc.Z : sc.X + (long)SB * n);
  out[r + c * ldo] = cplx{re, im};
}

// Y = [W V] from X = [V W] (rows 0 .. m-1).
__global__ __launch_bounds__(256) void p1_swap_kernel(EigWork W, int n, int g1, int m) {
  const int b = blockIdx.y;
  const long idx = blockIdx.x * 256L + threadIdx.x;
  if (idx >= (long)m * 2 * SB) return;
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  const long r = idx % m, c = idx / m;
  const long src = c < SB ? c + SB : c - SB;
  sc.Y[r + c * n] = sc.X[r + src * n];
}

// ------------------------------------------------------------------ stage 2: bulge chasing
constexpr int CH_THREADS = 256;

__device__ __forceinline__ int ntask(int n, int j) { return (n - 2 - j) / SB + 1; }

// Progress words, the sweep counter, the abort word and the panel counter of every matrix.
__global__ __launch_bounds__(256) void p2_clear_kernel(EigWork W, int n, int g1) {
  const Scratch sc = scratch_of(W.panel + (long)blockIdx.y * W.panel_stride, n, g1);
  for (int i = blockIdx.x * 256 + threadIdx.x; i <= n + 2; i += gridDim.x * 256) sc.prog[i] = 0;
}

// One task's entries are loaded into registers at once, so that a task costs about one memory
// latency.  With CG = 256 / SB: of the diagonal block and the block below, thread tid holds row
// r = tid % SB of the columns q = tid / SB + CG u (u < SB / CG); of the left block, thread
// (column q = tid / CG, part = tid % CG) holds rows part + CG i (i < SB / CG), so that each
// column's dot product with v is log2(CG) exchanges between neighbouring lanes.  Wave 0 loads
// column c for the reflector.
constexpr int CG = CH_THREADS / SB, CU2 = SB / CG;
static_assert(SB <= 64 && CG * SB == CH_THREADS && CU2 * CG == SB, "chase layout");

__global__ __launch_bounds__(CH_THREADS) void p2_chase_kernel(EigWork W, int n, int g1, long long limit) {
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rr = tid % SB, grp = tid / SB;   // diagonal block and block below
  const int lq = tid / CG, lp = tid % CG;    // left block
  cplx *A = W.A + (long)b * n * n;
  const Scratch sc = scratch_of(W.panel + (long)b * W.panel_stride, n, g1);
  __shared__ cplx D[SB][SB + 1];  // D[q][r]: row r, column q of the diagonal block (full Hermitian)
  __shared__ cplx sv[SB], sp[CG][SB], swv[SB];
  __shared__ int s_j, s_go, s_skip;
  __shared__ double s_tau;
  __shared__ cplx s_alpha;
  for (;;) {
    if (tid == 0) s_j = atomicAdd(&sc.prog[n], 1);
    __syncthreads();
    const int j = s_j;
    __syncthreads();
    if (j >= n - 2) return;
    const int nt = ntask(n, j);
    for (int t = 0; t < nt; ++t) {
      // wait until sweep j - 1 has finished task t + 2 (or all of its tasks); thread 0's acquire
      // fence and the barrier order the loads below after that task's stores
      if (tid == 0) {
        int go = 1;
        if (j > 0) {
          const int need = min(ntask(n, j - 1), t + 3);
          long long t0 = -1;
          while (__hip_atomic_load(&sc.prog[j - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            if (__hip_atomic_load(&sc.prog[n + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
              go = 0;
              break;
            }
            const long long now = wall_clock64();
            if (t0 < 0) t0 = now;
            if (now - t0 > limit) {  // leave, and make the context report it
              __hip_atomic_store(&sc.prog[n + 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              atomicOr(W.flag, 1);
              if (atomicCAS(&W.info->set, 0, 1) == 0) {
                W.info->source = 4;
                W.info->traj = b;
                W.info->col = j;
                W.info->pivot = 0.0;
              }
              go = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
          // the polls above do not touch the caches; one acquire fence orders the task's loads
          // after the stores that sweep j - 1 released
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        s_go = go;
      }
      __syncthreads();
      if (!s_go) return;
      const int r0 = j + t * SB + 1, r1 = min(j + (t + 1) * SB, n - 1), len = r1 - r0 + 1;
      const int c = t == 0 ? j : j + (t - 1) * SB + 1;
      const int ncl = r0 - c;              // columns of the left block (1 or SB)
      const int nb = min(SB, n - 1 - r1);  // rows of the block below
      // all loads of the task at once
      cplx Lr[CU2], Dr[CU2], Br[CU2];
      const cplx xc = (wave == 0 && lane < len) ? A[r0 + lane + (long)c * n] : cplx{0.0, 0.0};
#pragma unroll
      for (int u = 0; u < CU2; ++u) {
        const int q = grp + CG * u, rl = lp + CG * u;
        Lr[u] = (rl < len && lq < ncl) ? A[r0 + rl + (long)(c + lq) * n] : cplx{0.0, 0.0};
        Dr[u] = (rr < len && q <= rr) ? A[r0 + rr + (long)(r0 + q) * n] : cplx{0.0, 0.0};
        Br[u] = (rr < nb && q < len) ? A[r1 + 1 + rr + (long)(r0 + q) * n] : cplx{0.0, 0.0};
      }
      // reflector from x = column c (wave 0)
      if (wave == 0) {
        const cplx x = xc;
        double mx = cmax_abs(x);
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        const double inv = mx >= REFLECT_TINY ? 1.0 / mx : 0.0;
        const cplx xs{x.re * inv, x.im * inv};
        const double tail2 = wsum(lane >= 1 ? xs.re * xs.re + xs.im * xs.im : 0.0);
        const cplx x0{__shfl(x.re, 0, 64), __shfl(x.im, 0, 64)};
        if (!(tail2 > 0.0)) {
          if (lane == 0) {
            s_skip = 1;
            s_tau = 0.0;
          }
        } else {
          const Reflector h = make_reflector(cplx{x0.re * inv, x0.im * inv}, tail2, mx);
          if (lane == 0) {
            const double ax0 = hypot(x0.re, x0.im);
            const double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
            s_skip = 0;
            s_tau = h.tau;
            s_alpha = cplx{-phr * h.norm, -phi * h.norm};
          }
          if (lane < SB) sv[lane] = lane == 0 ? h.v0 : (lane < len ? xs : cplx{0.0, 0.0});
        }
      }
#pragma unroll
      for (int u = 0; u < CU2; ++u) {
        const int q = grp + CG * u;
        if (rr < len && q <= rr) {
          D[q][rr] = Dr[u];
          D[rr][q] = cplx{Dr[u].re, -Dr[u].im};
        }
      }
      __syncthreads();
      if (!s_skip) {
        const double tau = s_tau;
        const cplx vr = rr < len ? sv[rr] : cplx{0.0, 0.0};
        // (a) the left block from the left: column c -> alpha e_0, the others y -= tau v (v^+ y)
        if (lq < ncl) {
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int u = 0; u < CU2; ++u) {
            const int rl = lp + CG * u;
            if (rl < len) {
              const cplx d = conj_mul(sv[rl], Lr[u]);
              sr += d.re;
              si += d.im;
            }
          }
#pragma unroll
          for (int o = 1; o < CG; o <<= 1) {
            sr += __shfl_xor(sr, o, 64);
            si += __shfl_xor(si, o, 64);
          }
#pragma unroll
          for (int u = 0; u < CU2; ++u) {
            const int rl = lp + CG * u;
            if (rl >= len) continue;
            cplx y = Lr[u];
            if (lq == 0) {
              y = rl == 0 ? s_alpha : cplx{0.0, 0.0};
            } else {
              const cplx vv = sv[rl];
              y.re -= tau * (vv.re * sr - vv.im * si);
              y.im -= tau * (vv.re * si + vv.im * sr);
            }
            A[r0 + rl + (long)(c + lq) * n] = y;
          }
        }
        // (b) the diagonal block, two-sided: p = tau D v, w = p - (tau/2)(v^+ p) v, D -= v w^+ + w v^+
        {
          cplx acc{0.0, 0.0};
#pragma unroll
          for (int u = 0; u < CU2; ++u) {
            const int q = grp + CG * u;
            if (rr < len && q < len) {
              const cplx a = D[q][rr], vq = sv[q];
              acc.re += a.re * vq.re - a.im * vq.im;
              acc.im += a.re * vq.im + a.im * vq.re;
            }
          }
          sp[grp][rr] = acc;
        }
        __syncthreads();
        if (wave == 0) {
          cplx p{0.0, 0.0};
          if (lane < len) {
#pragma unroll
            for (int g = 0; g < CG; ++g) {
              p.re += sp[g][lane].re;
              p.im += sp[g][lane].im;
            }
            p.re *= tau;
            p.im *= tau;
          }
          const cplx vl = lane < len ? sv[lane] : cplx{0.0, 0.0};
          const cplx d = conj_mul(vl, p);
          const double kr = 0.5 * tau * wsum(d.re), ki = 0.5 * tau * wsum(d.im);
          if (lane < SB) swv[lane] = cplx{p.re - (kr * vl.re - ki * vl.im), p.im - (kr * vl.im + ki * vl.re)};
        }
        __syncthreads();
        const cplx wr = swv[rr];
        cplx acc{0.0, 0.0};
#pragma unroll
        for (int u = 0; u < CU2; ++u) {
          const int q = grp + CG * u;
          if (rr < len && q <= rr) {  // D_rq -= v_r conj(w_q) + w_r conj(v_q)
            const cplx vq = sv[q], wq = swv[q];
            cplx a = Dr[u];
            a.re -= (vr.re * wq.re + vr.im * wq.im) + (wr.re * vq.re + wr.im * vq.im);
            a.im -= (vr.im * wq.re - vr.re * wq.im) + (wr.im * vq.re - wr.re * vq.im);
            A[r0 + rr + (long)(r0 + q) * n] = a;
          }
          // (c) partial s_r = sum_q B_rq v_q of the block below
          if (q < len) {
            const cplx vq = sv[q];
            acc.re += Br[u].re * vq.re - Br[u].im * vq.im;
            acc.im += Br[u].re * vq.im + Br[u].im * vq.re;
          }
        }
        if (nb > 0) {
          __syncthreads();  // every wave is done with sp
          sp[grp][rr] = acc;
          __syncthreads();
          double sr = 0.0, si = 0.0;
#pragma unroll
          for (int g = 0; g < CG; ++g) {
            sr += sp[g][rr].re;
            si += sp[g][rr].im;
          }
          sr *= tau;
          si *= tau;
#pragma unroll
          for (int u = 0; u < CU2; ++u) {
            const int q = grp + CG * u;
            if (rr < nb && q < len) {  // B_rq -= (tau s_r) conj(v_q)
              const cplx vq = sv[q];
              A[r1 + 1 + rr + (long)(r0 + q) * n] =
                  cplx{Br[u].re - (sr * vq.re + si * vq.im), Br[u].im - (si * vq.re - sr * vq.im)};
            }
          }
        }
      }
      // publish the task: the barrier completes every wave's stores, thread 0 releases them
      __syncthreads();
      if (tid == 0) __hip_atomic_store(&sc.prog[j], t + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// d_i = Re A_ii, e_i = |A_{i+1,i}| of the reduced matrix.
__global__ __launch_bounds__(256) void p2_extract_kernel(EigWork W, int n) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const cplx *A = W.A + (long)b * n * n;
  W.d[(long)b * n + i] = A[i + (long)i * n].re;
  if (i + 1 < n) {
    const cplx e = A[i + 1 + (long)i * n];
    W.e[(long)b * n + i] = hypot(e.re, e.im);
  }
}

GemmDesc gdesc() {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  return g;
}

int groups_for(int n) { return trd2_groups(n); }

// Workgroups of p1_panel_kernel that the current GPU holds at once (0 if unknown).
long panel_capacity() {
  static std::atomic<long> cap[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  long c = cap[dev].load(std::memory_order_relaxed);
  if (c == 0) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, p1_panel_kernel, 256, 0) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return 0;
    c = per_cu > 0 && cus > 0 ? (long)per_cu * cus : -1;
    cap[dev].store(c, std::memory_order_relaxed);
  }
  return c > 0 ? c : 0;
}

// Panel kernels that may run at once on one device: the records of panel_admission.h, one per
// (device, stream).  A record's event is recorded on a stream of the library's own, made to wait
// for the panel kernel first: a query of an event last recorded on a context's stream has failed
// (hipErrorCapturedEvent) once that stream had been captured into its step-pair graphs, while the
// library's stream is never captured.  Records, their events and the library's streams are kept
// until the process ends (one per stream and device that ran a panel kernel).
struct PanelSlot {
  hipEvent_t ev = nullptr;
  mfq_panel::Record rec;
};
std::mutex g_panel_mu;
std::map<std::pair<int, hipStream_t>, PanelSlot> g_panel_slots;
std::map<int, hipStream_t> g_panel_streams;
long g_panel_seq = 0;

hipError_t launch_panel(const EigWork &w, int n, int j, int m, int kmax, int g1, int gm, int B, int base,
                        long long wait_ticks, long cap, hipStream_t s) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const long wgs = (long)gm * B;
  std::lock_guard<std::mutex> lock(g_panel_mu);
  hipStream_t &own = g_panel_streams[dev];
  if (!own && (e = hipStreamCreateWithFlags(&own, hipStreamNonBlocking)) != hipSuccess) {
    own = nullptr;
    return e;
  }
  std::vector<PanelSlot *> slots;
  std::vector<mfq_panel::Record> others;
  for (auto &kv : g_panel_slots) {
    PanelSlot &p = kv.second;
    if (kv.first.first != dev || kv.first.second == s || p.rec.wgs == 0) continue;
    const hipError_t q = hipEventQuery(p.ev);
    if (q == hipSuccess) {
      p.rec.wgs = 0;
      continue;
    }
    if (q != hipErrorNotReady) return q;
    slots.push_back(&p);
    others.push_back(p.rec);
  }
  for (int i : mfq_panel::waits_for(others, wgs, cap))
    if ((e = hipStreamWaitEvent(s, slots[i]->ev, 0)) != hipSuccess) return e;
  // this stream's earlier panel kernels are not queried here: the bound keeps their grid until
  // another stream finds the record finished
  PanelSlot &mine = g_panel_slots[{dev, s}];
  const bool finished = mine.rec.wgs == 0;
  hipLaunchKernelGGL(p1_panel_kernel, dim3(gm, B), dim3(256), 0, s, w, n, j, m, kmax, g1, gm, base, wait_ticks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the record's event: on the library's stream, after the panel kernel
  hipEvent_t after = nullptr;
  if ((e = hipEventCreateWithFlags(&after, hipEventDisableTiming)) != hipSuccess) return e;
  e = hipEventRecord(after, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(own, after, 0);
  (void)hipEventDestroy(after);
  if (e != hipSuccess) return e;
  if (!mine.ev && (e = hipEventCreateWithFlags(&mine.ev, hipEventDisableTiming)) != hipSuccess) return e;
  if ((e = hipEventRecord(mine.ev, own)) != hipSuccess) return e;
  mine.rec.wgs = mfq_panel::recorded_wgs(mine.rec.wgs, finished, wgs);
  mine.rec.seq = ++g_panel_seq;
  return hipSuccess;
}

// g (depth K) split over K in one launch into trd2_slice_count(K, ks) slices: slice q covers K
// indices [q kc, min((q + 1) kc, K)), kc = trd2_slice_depth(K, ks), its partial into D + q sDq.
// dA, dB: operand offsets per unit of K.  The slices' partials are summed by p1_ksum_kernel.
hipError_t ksplit(GemmDesc g, int B, int K, int ks, long dA, long dB, long sDq, hipStream_t s) {
  const int kc = trd2_slice_depth(K, ks);
  ks = trd2_slice_count(K, ks);
  g.K = kc; g.batch = B * ks; g.batch2 = ks;
  g.sA2 = kc * dA; g.sB2 = kc * dB; g.sD2 = sDq;
  g.kofs = 0; g.kofs2 = kc; g.kend_glob = K;
  return zgemm(g, s);
}

}  // namespace

hipError_t tridiagonalize_two_stage(const EigWork &w, int n, int B, long long wait_ticks, hipStream_t s) {
  if (n < 2 * SB + 2 || !w.panel || w.panel_stride < trd2_scratch_elems(n) || !w.flag || !w.info)
    return hipErrorInvalidValue;
  const int g1 = groups_for(n);
  hipError_t e;
  const Scratch s0 = scratch_of(w.panel, n, g1);  // matrix 0; the others at multiples of panel_stride
  const long ps = w.panel_stride, nn = (long)n * n;
  const long cap = panel_capacity();
  int base = 0;  // the panel counter's value at the start of the next panel kernel
  hipLaunchKernelGGL(p2_clear_kernel, dim3((n + 256) / 256, B), dim3(256), 0, s, w, n, g1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int j = 0; n - j - SB >= 2; j += SB) {
    const int m = n - j - SB, kmax = std::min(m, SB), gm = (m + P1_RPW - 1) / P1_RPW;
    cplx *A22 = w.A + (j + SB) + (long)(j + SB) * n;
    if ((long)gm * B <= cap * 3 / 4) {  // a quarter of the GPU left to other work
      if ((e = launch_panel(w, n, j, m, kmax, g1, gm, B, base, wait_ticks, cap, s)) != hipSuccess) return e;
      base += gm * (kmax + 1);
    } else {
      for (int k = -1; k < kmax; ++k) {
        hipLaunchKernelGGL(p1_col_kernel, dim3(gm, B), dim3(256), 0, s, w, n, j, m, k, kmax, g1, gm);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    {  // S = V^+ V
      const int ks = trd2_sb_slices(n, m, B);
      if ((long)ks * SB * SB > trd2_kp_elems(n)) return hipErrorInvalidValue;
      GemmDesc g = gdesc();
      g.M = SB; g.N = SB; g.batch = B;
      g.A = s0.X; g.lda = n; g.sA = ps; g.opA = OP_C;
      g.B = s0.X; g.ldb = n; g.sB = ps; g.opB = OP_N;
      g.D = s0.KP; g.ldd = SB; g.sD = ps;
      if ((e = ksplit(g, B, m, ks, 1, 1, (long)SB * SB, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(p1_ksum_kernel, dim3((SB * SB + 255) / 256, B), dim3(256), 0, s, w, n, g1, 0, SB, ks,
                         (long)SB);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(p1_tfactor_kernel, dim3(B), dim3(SB), 0, s, w, n, g1);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {  // VT = V T
      GemmDesc g = gdesc();
      g.M = m; g.N = SB; g.K = SB; g.batch = B;
      g.A = s0.X; g.lda = n; g.sA = ps; g.opA = OP_N;
      g.B = s0.T; g.ldb = SB; g.sB = ps; g.opB = OP_N; g.bUpper = 1;
      g.D = s0.VT; g.ldd = n; g.sD = ps;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    {  // X = A22 (V T) from the lower triangle of A22: tril(A22) (V T) + striu(A22^+) (V T),
       // each split over K, all partials summed into the W columns of X
      const int ks = trd2_x_slices(n, m, B);
      if (2L * ks * m * SB > trd2_kp_elems(n)) return hipErrorInvalidValue;
      GemmDesc g = gdesc();
      g.M = m; g.N = SB; g.batch = B;
      g.A = A22; g.lda = n; g.sA = nn; g.opA = OP_N; g.aLower = 1;
      g.B = s0.VT; g.ldb = n; g.sB = ps; g.opB = OP_N;
      g.D = s0.KP; g.ldd = m; g.sD = ps;
      if ((e = ksplit(g, B, m, ks, n, 1, (long)m * SB, s)) != hipSuccess) return e;
      g.opA = OP_C; g.aLower = 0; g.aUpper = 2;
      g.D = s0.KP + (long)ks * m * SB;
      if ((e = ksplit(g, B, m, ks, 1, 1, (long)m * SB, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(p1_ksum_kernel, dim3((unsigned)(((long)m * SB + 255) / 256), B), dim3(256), 0, s, w, n, g1,
                         2, m, 2 * ks, (long)n);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {  // Z = V^+ X
      const int ks = trd2_sb_slices(n, m, B);
      if ((long)ks * SB * SB > trd2_kp_elems(n)) return hipErrorInvalidValue;
      GemmDesc g = gdesc();
      g.M = SB; g.N = SB; g.batch = B;
      g.A = s0.X; g.lda = n; g.sA = ps; g.opA = OP_C;
      g.B = s0.X + (long)SB * n; g.ldb = n; g.sB = ps; g.opB = OP_N;
      g.D = s0.KP; g.ldd = SB; g.sD = ps;
      if ((e = ksplit(g, B, m, ks, 1, 1, (long)SB * SB, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(p1_ksum_kernel, dim3((SB * SB + 255) / 256, B), dim3(256), 0, s, w, n, g1, 1, SB, ks,
                         (long)SB);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    {  // M2 = T^+ Z
      GemmDesc g = gdesc();
      g.M = SB; g.N = SB; g.K = SB; g.batch = B;
      g.A = s0.T; g.lda = SB; g.sA = ps; g.opA = OP_C;
      g.B = s0.Z; g.ldb = SB; g.sB = ps; g.opB = OP_N;
      g.D = s0.M2; g.ldd = SB; g.sD = ps;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    {  // W = X - (1/2) V M2, in place
      GemmDesc g = gdesc();
      g.M = m; g.N = SB; g.K = SB; g.batch = B;
      g.A = s0.X; g.lda = n; g.sA = ps; g.opA = OP_N;
      g.B = s0.M2; g.ldb = SB; g.sB = ps; g.opB = OP_N;
      g.Cin = s0.X + (long)SB * n; g.ldcin = n; g.sCin = ps;
      g.D = s0.X + (long)SB * n; g.ldd = n; g.sD = ps;
      g.alpha = cplx{-0.5, 0.0};
      g.beta = cplx{1.0, 0.0};
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(p1_swap_kernel, dim3((unsigned)(((long)m * 2 * SB + 255) / 256), B), dim3(256), 0, s, w, n,
                       g1, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    {  // A22 -= [V W] [W V]^+, on and below the diagonal
      GemmDesc g = gdesc();
      g.M = m; g.N = m; g.K = 2 * SB; g.batch = B; g.tri = TRI_LOWER;
      g.A = s0.X; g.lda = n; g.sA = ps; g.opA = OP_N;
      g.B = s0.Y; g.ldb = n; g.sB = ps; g.opB = OP_C;
      g.Cin = A22; g.ldcin = n; g.sCin = nn;
      g.D = A22; g.ldd = n; g.sD = nn;
      g.alpha = cplx{-1.0, 0.0};
      g.beta = cplx{1.0, 0.0};
      g.short_k_large = 1;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
  }
  // stage 2
  hipLaunchKernelGGL(p2_clear_kernel, dim3((n + 256) / 256, B), dim3(256), 0, s, w, n, g1);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int g2 = std::max(1, std::min(n / (3 * SB) + 2, std::max(1, 480 / B)));
  hipLaunchKernelGGL(p2_chase_kernel, dim3(g2, B), dim3(CH_THREADS), 0, s, w, n, g1, wait_ticks);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(p2_extract_kernel, dim3((n + 255) / 256, B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

}  // namespace mfq
