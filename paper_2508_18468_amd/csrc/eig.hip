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
// Every sweep reads and writes the trailing matrix once (HBM-bound).  Batches
// with enough work take the blocked form below instead (panels of TRD_NB
// reflectors, only the lower triangle of the trailing matrix read per reflector,
// the matrix written once per panel by a GEMM): about a quarter of that traffic.
// Bisection: one lane per eigenvalue when the batch offers enough of them,
// otherwise P lanes per eigenvalue that split its interval at P points per Sturm
// pass ((P + 1)-fold narrowing per pass instead of 2-fold), P as large as keeps
// the batch within about two waves per SIMD.
#include <algorithm>

#include "device_common.h"

namespace mfq {

namespace {

constexpr int LDS_MAX_N = 88;  // 88 * 88 * 16 B = 121 KiB
// below this many eigenvalues in a batch, multisection with P lanes per eigenvalue, P the
// largest power of two up to 64 that keeps n B P within BISECT_MULTI_LANES (two waves per
// SIMD; two 8192-site spectra: P = 8 18.6 ms, 16 22.9 ms, 32 33.4 ms, 64 54 ms)
constexpr long BISECT_LANES_MIN = 131072;
constexpr long BISECT_MULTI_LANES = 131072;

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

// ---------------------------------------------------------------- blocked reduction
// Matrices of n >= TRD_BLOCKED_MIN are reduced in panels of TRD_NB columns.  Within a panel
// the trailing matrix is not written: A_cur = A - sum_t (v_t w_t^+ + w_t v_t^+) over the
// panel's earlier reflectors t, so that
//   A_cur v = A v - sum_t (v_t (w_t^+ v) + w_t (v_t^+ v))
// reads the trailing matrix once, read-only, and column k is corrected only when it is
// reduced.  At the end of the panel the trailing matrix takes all of the panel's reflectors in
// one GEMM, A -= [V W] [W V]^+, on the matrix cores; the last LDS_MAX_N columns are reduced in
// LDS.  For reflector r of a panel (column k0 + r) three launches:
//   trd_hemv(r)    grid: A v over the trailing block of columns c > k0 + r (from 64 x 64 tiles
//                  of its lower triangle, or from whole columns when the block is small), and,
//                  in the first TRD_ZCH workgroups, partial sums over row chunks of
//                  z = (W^+ v, V^+ v) against the panel's earlier reflectors;
//   trd_panel(r+1) grid over rows i >= k = k0 + r + 1: y_i corrected by the panel,
//                  partial sums of v^+ y, and column k corrected by the panel except for the
//                  part of reflector r's w that needs v^+ y;
//   trd_reflect(r+1) one workgroup per matrix: w_r = tau y - (tau^2/2)(v^+ y) v, the rest of
//                  column k, d_k and reflector r + 1 of column k.
// Every pass over the panel runs grid-wide; the one-workgroup step is O(n).  Panel storage per
// matrix (ld n): X = [V W] (v_t in column t, w_t in column jp + t), Y = [W V] at column offset
// 2 TRD_NB, then the z and v^+ y partial sums.  The corrected y goes to the first n entries of
// the reflector slots v (the hemv output y stays in p).
constexpr int TRD_REFLECT_THREADS = 1024;
constexpr int TRD_ZCH = 16;        // row chunks of the z partial sums
constexpr int TRD_PANEL_TPR = 8;    // threads per row of the row pass
constexpr int TRD_PANEL_ROWS = 32;  // rows per workgroup of the row pass
static_assert(TRD_ZCH == 16 && TRD_PANEL_ROWS == 32, "trd_panel_elems sizes the panel storage for these");

__device__ __forceinline__ cplx cmul_conj_a(cplx a, cplx x) {  // conj(a) x
  return cplx{a.re * x.re + a.im * x.im, a.re * x.im - a.im * x.re};
}
__device__ __forceinline__ cplx cmul(cplx a, cplx x) {
  return cplx{a.re * x.re - a.im * x.im, a.re * x.im + a.im * x.re};
}

struct PanelPtrs {
  cplx *X, *Y, *zpart, *kpart, *part, *dotpart;
};
__device__ __forceinline__ PanelPtrs panel_ptrs(const EigWork &W, int b, int n) {
  PanelPtrs q;
  q.X = W.panel + (long)b * W.panel_stride;
  q.Y = q.X + (long)2 * TRD_NB * n;
  q.zpart = q.Y + (long)2 * TRD_NB * n;
  q.kpart = q.zpart + TRD_ZCH * 2 * TRD_NB;
  q.part = q.kpart + (n + TRD_PANEL_ROWS - 1) / TRD_PANEL_ROWS;
  q.dotpart = q.part + (long)((n + 63) / 64) * n;
  return q;
}

// y = A v_r over columns c > k0 + r from the lower triangle only: with T the trailing block,
//   y_c = sum_{i >= c} conj(T_ic) v_i + sum_{i < c} T_ci v_i,
// the first sum read down column c, the second from the entries T_ci (c > i) of earlier
// columns.  The lower triangle is cut into 64 x 64 tiles (row tile t >= column tile p), TRD_TPW
// consecutive ones per workgroup: each tile is staged in LDS (the next one loaded into registers
// meanwhile), and the workgroup writes its row sums
// sum_c T_ic v_c (strictly below the diagonal) to part[p][i] and its column sums
// sum_i conj(T_ic) v_i (on and below the diagonal) to dotpart[t][c]; the row pass adds them up
// in a fixed order.  Workgroups below TRD_ZCH also form the partial sums of z = (W^+ v, V^+ v)
// over row chunks.
constexpr int TRD_TILE = 64;

__device__ __forceinline__ void lower_tile(long id, int &t, int &p) {  // id = t (t + 1) / 2 + p
  int c = (int)((sqrt(8.0 * (double)id + 1.0) - 1.0) * 0.5);
  while ((long)c * (c + 1) / 2 > id) --c;
  while ((long)(c + 1) * (c + 2) / 2 <= id) ++c;
  t = c;
  p = (int)(id - (long)c * (c + 1) / 2);
}

constexpr int TRD_HEMV_THREADS = 512;
constexpr int TRD_TPW = 4;  // tiles per workgroup, one loaded while the previous is reduced

__global__ __launch_bounds__(TRD_HEMV_THREADS) void trd_hemv_kernel(EigWork W, int n, int k0, int jp, int r) {
  constexpr int NW = TRD_HEMV_THREADS / 64, SUB = TRD_HEMV_THREADS / TRD_TILE;
  const int b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = k0 + r;
  if (W.tau[2 * b + (k & 1)] == 0.0) return;
  const PanelPtrs q = panel_ptrs(W, b, n);
  const cplx *v = q.X + (long)r * n;
  if (blockIdx.x < TRD_ZCH && r > 0) {  // z_t = w_t^+ v, z_{r+t} = v_t^+ v over this row chunk
    const int rows = n - k - 1, csz = (rows + TRD_ZCH - 1) / TRD_ZCH;
    const int i0 = k + 1 + blockIdx.x * csz, i1 = min(n, i0 + csz);
    for (int t2 = wave; t2 < 2 * r; t2 += NW) {
      const cplx *c = q.X + (long)(t2 < r ? jp + t2 : t2 - r) * n;
      double zr = 0.0, zi = 0.0;
      for (int i = i0 + lane; i < i1; i += 64) {
        const cplx x = cmul_conj_a(c[i], v[i]);
        zr += x.re;
        zi += x.im;
      }
      for (int o = 32; o > 0; o >>= 1) {
        zr += __shfl_down(zr, o, 64);
        zi += __shfl_down(zi, o, 64);
      }
      if (lane == 0) q.zpart[blockIdx.x * 2 * TRD_NB + t2] = cplx{zr, zi};
    }
  }
  const int c0 = k + 1, T = (n - c0 + TRD_TILE - 1) / TRD_TILE;
  const long ntile = (long)T * (T + 1) / 2;
  const long id0 = (long)blockIdx.x * TRD_TPW;
  if (id0 >= ntile) return;  // uniform over the workgroup
  const cplx *A = W.A + (long)b * n * n;
  // tile[c][i]: row r0 + i, column cb + c; a row stride of 72 entries (8 mod 16) spreads both
  // read patterns below over all LDS banks
  __shared__ cplx tile[TRD_TILE][TRD_TILE + 8];
  __shared__ cplx vrow[TRD_TILE], vcol[TRD_TILE];
  // the next tile is loaded into registers while the current one is reduced from LDS
  constexpr int PER = TRD_TILE / NW;  // columns per wave
  cplx nxt[PER], vnx{0.0, 0.0};
  auto fetch = [&](long id) {
    int tt, pp;
    lower_tile(id, tt, pp);
    const int rr0 = c0 + TRD_TILE * tt, cc0 = c0 + TRD_TILE * pp;
    const int row = rr0 + lane;
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int col = cc0 + wave + NW * m;
      nxt[m] = (row < n && col < n) ? A[row + (long)col * n] : cplx{0.0, 0.0};
    }
    if (tid < TRD_TILE) vnx = rr0 + tid < n ? v[rr0 + tid] : cplx{0.0, 0.0};
    else if (tid < 2 * TRD_TILE) vnx = cc0 + tid - TRD_TILE < n ? v[cc0 + tid - TRD_TILE] : cplx{0.0, 0.0};
  };
  fetch(id0);
  // row / column o of the tile; the other index runs over u = qq, qq + SUB, ... (the SUB threads
  // of one o read neighbouring LDS entries)
  const int o = tid / SUB, qq = tid % SUB;
  for (int s = 0; s < TRD_TPW; ++s) {
    const long id = id0 + s;
    if (id >= ntile) break;  // uniform
    __syncthreads();         // the previous tile's reads are done
#pragma unroll
    for (int m = 0; m < PER; ++m) tile[wave + NW * m][lane] = nxt[m];
    if (tid < TRD_TILE) vrow[tid] = vnx;
    else if (tid < 2 * TRD_TILE) vcol[tid - TRD_TILE] = vnx;
    __syncthreads();
    if (s + 1 < TRD_TPW && id + 1 < ntile) fetch(id + 1);
    int t, p;
    lower_tile(id, t, p);
    const int r0 = c0 + TRD_TILE * t, cb = c0 + TRD_TILE * p;
    const bool diag = t == p;
    double ar = 0.0, ai = 0.0, dr = 0.0, di = 0.0;
#pragma unroll
    for (int u = qq; u < TRD_TILE; u += SUB) {
      if (!diag || o > u) {  // row sums: T_{o,u} v_u, strictly lower
        const cplx a = tile[u][o], x = vcol[u];
        ar += a.re * x.re - a.im * x.im;
        ai += a.re * x.im + a.im * x.re;
      }
      if (!diag || u >= o) {  // column sums: conj(T_{u,o}) v_u, on and below the diagonal
        const cplx a = tile[o][u], x = vrow[u];
        dr += a.re * x.re + a.im * x.im;
        di += a.re * x.im - a.im * x.re;
      }
    }
    for (int m = 1; m < SUB; m <<= 1) {
      ar += __shfl_xor(ar, m, 64);
      ai += __shfl_xor(ai, m, 64);
      dr += __shfl_xor(dr, m, 64);
      di += __shfl_xor(di, m, 64);
    }
    if (qq == 0) {
      if (r0 + o < n) q.part[(long)p * n + r0 + o] = cplx{ar, ai};
      if (cb + o < n) q.dotpart[(long)t * n + cb + o] = cplx{dr, di};
    }
  }
}

// The same A v from whole columns (trailing blocks below TRD_TILED_MIN): one wave per CPW
// columns reads rows k0 + r + 1 .. n-1 of each and writes y_c = sum_i conj(A_ic) v_i (A Hermitian)
// to W.p; twice the bytes of the tiled form, but far fewer, fuller workgroups for small blocks.
constexpr int TRD_TILED_MIN = 1024;

template <int CPW>
__global__ __launch_bounds__(256) void trd_hemv_cols_kernel(EigWork W, int n, int k0, int jp, int r) {
  const int b = blockIdx.y, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int k = k0 + r;
  if (W.tau[2 * b + (k & 1)] == 0.0) return;
  const PanelPtrs q = panel_ptrs(W, b, n);
  const cplx *v = q.X + (long)r * n;
  if (blockIdx.x < TRD_ZCH && r > 0) {  // z_t = w_t^+ v, z_{r+t} = v_t^+ v over this row chunk
    const int rows = n - k - 1, csz = (rows + TRD_ZCH - 1) / TRD_ZCH;
    const int i0 = k + 1 + blockIdx.x * csz, i1 = min(n, i0 + csz);
    for (int t2 = wave; t2 < 2 * r; t2 += 4) {
      const cplx *c = q.X + (long)(t2 < r ? jp + t2 : t2 - r) * n;
      double zr = 0.0, zi = 0.0;
      for (int i = i0 + lane; i < i1; i += 64) {
        const cplx x = cmul_conj_a(c[i], v[i]);
        zr += x.re;
        zi += x.im;
      }
      for (int o = 32; o > 0; o >>= 1) {
        zr += __shfl_down(zr, o, 64);
        zi += __shfl_down(zi, o, 64);
      }
      if (lane == 0) q.zpart[blockIdx.x * 2 * TRD_NB + t2] = cplx{zr, zi};
    }
  }
  const int c0 = k + 1 + (blockIdx.x * 4 + wave) * CPW;
  if (c0 >= n) return;
  const cplx *A = W.A + (long)b * n * n;
  cplx *y = W.p + (long)b * n;
  double pr[CPW], pim[CPW];
  int jc[CPW];
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    jc[c] = min(c0 + c, n - 1);  // columns past the end repeat the last one, unwritten
    pr[c] = pim[c] = 0.0;
  }
  for (int i = k + 1 + lane; i < n; i += 64) {
    const cplx xv = v[i];
#pragma unroll
    for (int c = 0; c < CPW; ++c) {
      const cplx x = cmul_conj_a(A[i + (long)jc[c] * n], xv);
      pr[c] += x.re;
      pim[c] += x.im;
    }
  }
#pragma unroll
  for (int c = 0; c < CPW; ++c) {
    double sr = pr[c], si = pim[c];
    for (int o = 32; o > 0; o >>= 1) {
      sr += __shfl_down(sr, o, 64);
      si += __shfl_down(si, o, 64);
    }
    if (lane == 0 && c0 + c < n) y[c0 + c] = cplx{sr, si};
  }
}

// Rows i >= k = k0 + r + 1 of matrix blockIdx.y (TRD_PANEL_ROWS per workgroup, TRD_PANEL_TPR
// threads per row sharing its sums), for reflector r:
//   y_i = (A v_r)_i - sum_{t<r} (v_t[i] z_t + w_t[i] z_{r+t})     (into W.v)
//   partial sum of conj(v_r[i]) y_i                             (into kpart)
//   with_col: a_i = A_ik - sum_{t<r} (v_t[i] conj(w_t[k]) + w_t[i] conj(v_t[k]))
//                        - tau_r (v_r[i] conj(y_k) + y_i conj(v_r[k]))   (into column k)
// tiled: (A v_r)_i is the sum of the tiles' column sums dotpart[t][i] (t >= the tile of i) and row
// sums part[p][i] (p <= it), in a fixed order; otherwise it is W.p[i].
__global__ __launch_bounds__(TRD_PANEL_TPR * TRD_PANEL_ROWS) void trd_panel_kernel(EigWork W, int n, int k0, int jp, int r,
                                                                       int with_col, int tiled) {
  constexpr int NT = TRD_PANEL_TPR * TRD_PANEL_ROWS, S = TRD_PANEL_TPR;
  const int b = blockIdx.y, tid = threadIdx.x, sub = tid % S;
  const int k = k0 + r + 1;
  const int i = k + blockIdx.x * TRD_PANEL_ROWS + tid / S;
  const bool live = i < n;
  const int row = live ? i : n - 1;  // rows past the end compute on the last row, unwritten
  const PanelPtrs q = panel_ptrs(W, b, n);
  const double tp = W.tau[2 * b + ((k - 1) & 1)];
  __shared__ cplx zs[2 * TRD_NB], rowk[2 * TRD_NB];
  __shared__ double red[NT / 64];
  __shared__ cplx sh_yk;
  if (tp != 0.0)
    for (int t2 = tid; t2 < 2 * r; t2 += NT) {  // z summed over the row chunks in order
      cplx acc{0.0, 0.0};
      for (int c = 0; c < TRD_ZCH; ++c) {
        const cplx x = q.zpart[c * 2 * TRD_NB + t2];
        acc.re += x.re;
        acc.im += x.im;
      }
      zs[t2] = acc;
    }
  if (with_col)
    for (int t2 = tid; t2 < 2 * r; t2 += NT)  // v_t[k], w_t[k]
      rowk[t2] = q.X[k + (long)(t2 < r ? t2 : jp + t2 - r) * n];
  __syncthreads();
  cplx *ycor = W.v + (long)b * 2 * n;
  const int T = (n - k + TRD_TILE - 1) / TRD_TILE;
  // y at row rw, summed by the S threads of the row (each takes every S-th term)
  const cplx *ycols = W.p + (long)b * n;
  auto y_at = [&](int rw) {
    double yr = 0.0, yi = 0.0;
    if (tiled) {
      const int pr = (rw - k) / TRD_TILE;
      for (int t = pr + sub; t < T; t += S) {
        const cplx x = q.dotpart[(long)t * n + rw];
        yr += x.re;
        yi += x.im;
      }
      for (int p = sub; p <= pr; p += S) {
        const cplx x = q.part[(long)p * n + rw];
        yr += x.re;
        yi += x.im;
      }
    } else if (sub == 0) {
      yr = ycols[rw].re;
      yi = ycols[rw].im;
    }
    for (int t = sub; t < r; t += S) {
      const cplx a = cmul(q.X[rw + (long)t * n], zs[t]), c = cmul(q.X[rw + (long)(jp + t) * n], zs[r + t]);
      yr -= a.re + c.re;
      yi -= a.im + c.im;
    }
    for (int m = 1; m < S; m <<= 1) {
      yr += __shfl_xor(yr, m, 64);
      yi += __shfl_xor(yi, m, 64);
    }
    return cplx{yr, yi};
  };
  if (tid < S) {
    const cplx yk = tp != 0.0 ? y_at(k) : cplx{0.0, 0.0};
    if (tid == 0) sh_yk = yk;
  }
  __syncthreads();
  const cplx *vr = q.X + (long)r * n;
  double kr = 0.0, ki = 0.0;
  cplx yv{0.0, 0.0};
  if (tp != 0.0) {
    yv = y_at(row);
    if (live && sub == 0) {
      ycor[row] = yv;
      const cplx x = cmul_conj_a(vr[row], yv);
      kr = x.re;
      ki = x.im;
    }
  }
  if (with_col) {
    cplx *col = W.A + (long)b * n * n + (long)k * n;
    double sr = 0.0, si = 0.0;
    for (int t = sub; t < r; t += S) {
      const cplx vi = q.X[row + (long)t * n], wi = q.X[row + (long)(jp + t) * n];
      const cplx vk = rowk[t], wk = rowk[r + t];
      sr += (vi.re * wk.re + vi.im * wk.im) + (wi.re * vk.re + wi.im * vk.im);
      si += (vi.im * wk.re - vi.re * wk.im) + (wi.im * vk.re - wi.re * vk.im);
    }
    for (int m = 1; m < S; m <<= 1) {
      sr += __shfl_xor(sr, m, 64);
      si += __shfl_xor(si, m, 64);
    }
    if (live && sub == 0) {
      cplx a = col[row];
      a.re -= sr;
      a.im -= si;
      if (tp != 0.0) {  // - tau (v_r[i] conj(y_k) + y_i conj(v_r[k]))
        const cplx vi = vr[row], vk = vr[k], yk = sh_yk;
        a.re -= tp * ((vi.re * yk.re + vi.im * yk.im) + (yv.re * vk.re + yv.im * vk.im));
        a.im -= tp * ((vi.im * yk.re - vi.re * yk.im) + (yv.im * vk.re - yv.re * vk.im));
      }
      col[row] = a;
    }
  }
  kr = block_sum_nt<NT>(kr, red);
  ki = block_sum_nt<NT>(ki, red);
  if (tid == 0) q.kpart[blockIdx.x] = cplx{kr, ki};
}

// One workgroup per matrix: for r = j - 1 >= 0, K = (tau^2/2) v_r^+ y and w_r = tau y - K v_r
// (rows >= k = k0 + j), and the last part of column k's correction, 2 Re(K) v_r[i] conj(v_r[k]);
// for j < jp, d_k and reflector j of column k.
template <int NT>
__global__ __launch_bounds__(NT) void trd_reflect_kernel(EigWork W, int n, int k0, int jp, int j) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const int k = k0 + j;
  const PanelPtrs q = panel_ptrs(W, b, n);
  double *d = W.d + (long)b * n, *e = W.e + (long)b * n;
  __shared__ double red[NT / 64];
  __shared__ double sh_dk, sh_tau;
  __shared__ cplx sh_x0;
  cplx *col = W.A + (long)b * n * n + (long)k * n;
  double two_kr = 0.0;
  const cplx *vr = q.X + (long)(j > 0 ? j - 1 : 0) * n;
  if (j >= 1) {
    const int r = j - 1;
    const double tp = W.tau[2 * b + ((k - 1) & 1)];
    cplx K{0.0, 0.0};
    if (tp != 0.0) {  // the row pass's partial sums, reduced in a fixed order
      const int nch = (n - k + TRD_PANEL_ROWS - 1) / TRD_PANEL_ROWS;
      double kr = 0.0, ki = 0.0;
      for (int c = tid; c < nch; c += NT) {
        kr += q.kpart[c].re;
        ki += q.kpart[c].im;
      }
      K.re = 0.5 * tp * tp * block_sum_nt<NT>(kr, red);
      K.im = 0.5 * tp * tp * block_sum_nt<NT>(ki, red);
    }
    two_kr = 2.0 * K.re;
    const cplx *y = W.v + (long)b * 2 * n;
    cplx *wx = q.X + (long)(jp + r) * n, *wy = q.Y + (long)r * n;
    for (int i = k + tid; i < n; i += NT) {
      cplx wi{0.0, 0.0};
      if (tp != 0.0) {
        const cplx vi = vr[i], yi = y[i];
        wi = cplx{tp * yi.re - (K.re * vi.re - K.im * vi.im), tp * yi.im - (K.re * vi.im + K.im * vi.re)};
      }
      wx[i] = wi;
      wy[i] = wi;
    }
  }
  if (j == jp) return;  // the panel's last w only
  const cplx vrk = j >= 1 ? vr[k] : cplx{0.0, 0.0};
  double mx = 0.0;
  for (int i = k + tid; i < n; i += NT) {
    cplx a = col[i];
    if (j >= 1 && two_kr != 0.0) {  // + 2 Re(K) v_r[i] conj(v_r[k])
      const cplx x = cmul_conj_a(vrk, vr[i]);
      a.re += two_kr * x.re;
      a.im += two_kr * x.im;
      col[i] = a;
    }
    if (i == k) sh_dk = a.re;
    else mx = fmax(mx, cmax_abs(a));
    if (i == k + 1) sh_x0 = a;
  }
  // reflector of rows k+1 .. n-1, formed from the column scaled by its largest component
  const double s = block_max_nt<NT>(mx, red);
  const double inv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
  cplx *vk = q.X + (long)j * n, *vy = q.Y + (long)(jp + j) * n;
  double part = 0.0;
  for (int i = k + tid; i < n; i += NT) {  // each thread rereads the entries it wrote
    if (i < k + 2) continue;
    const cplx a{col[i].re * inv, col[i].im * inv};
    part += a.re * a.re + a.im * a.im;
    vk[i] = a;
  }
  const double tail2 = block_sum_nt<NT>(part, red);  // its barriers publish sh_dk, sh_x0
  if (tid == 0) {
    d[k] = sh_dk;
    const cplx x0 = sh_x0;
    double tau = 0.0;
    if (tail2 == 0.0) {  // nothing below x0 (or all below REFLECT_TINY): H = I
      e[k] = hypot(x0.re, x0.im);
    } else {
      const Reflector h = make_reflector(cplx{x0.re * inv, x0.im * inv}, tail2, s);
      vk[k + 1] = h.v0;
      e[k] = h.norm;
      tau = h.tau;
    }
    W.tau[2 * b + (k & 1)] = tau;
    sh_tau = tau;
  }
  __syncthreads();
  const bool zero = sh_tau == 0.0;  // H = I: a zero column, so that its w and corrections vanish
  for (int i = k + 1 + tid; i < n; i += NT) {
    if (zero) vk[i] = cplx{0.0, 0.0};
    vy[i] = vk[i];
  }
}

// The trailing block from column k0 on (at most LDS_MAX_N) reduced in LDS: d[k0 ..],
// e[k0 ..].
__global__ __launch_bounds__(256) void trd_tail_kernel(EigWork w, int n, int k0) {
  const int b = blockIdx.x, m = n - k0;
  __shared__ cplx As[LDS_MAX_N * LDS_MAX_N];
  __shared__ cplx vs[LDS_MAX_N], ps[LDS_MAX_N];
  __shared__ double red[4];
  const cplx *Ab = w.A + (long)b * n * n + (long)k0 * (n + 1);
  for (int q = threadIdx.x; q < m * m; q += 256) As[q] = Ab[q % m + (long)(q / m) * n];
  __syncthreads();
  tridiag_body(As, m, m, vs, ps, w.d + (long)b * n + k0, w.e + (long)b * n + k0, red);
}

// Eigenvalue k (ascending) of tridiagonal b (see bisect_eigenvalue).
__global__ __launch_bounds__(256) void bisect_kernel(EigWork w, int n) {
  const int b = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  w.lam[(long)b * n + k] = bisect_eigenvalue(w.d + (long)b * n, w.e + (long)b * n, n, k);
}

// Eigenvalues of tridiagonal blockIdx.y by multisection with P lanes per eigenvalue (P a power
// of two, 2 <= P <= 64; 64 / P eigenvalues per wave, eigenvalue k = (blockIdx.x * 4 + wave) *
// (64 / P) + lane / P): the P lanes of an eigenvalue evaluate the Sturm count at P interior
// points of its interval, which shrinks to the gap between the last point below lambda_k and
// the first above it.  Same interval, pivmin and stopping width as bisect_eigenvalue.
__global__ __launch_bounds__(256) void bisect_multi_kernel(EigWork w, int n, int P) {
  const int b = blockIdx.y, lane = threadIdx.x & 63;
  const int G = 64 / P, grp = lane / P, pl = lane % P;
  const int k0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * G;
  if (k0 >= n) return;  // uniform over the wave
  const int k = k0 + grp;
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
  // each pass divides the interval by P + 1; 60 halvings cover any start width over tol
  const int max_it = (int)(60.0 / log2((double)(P + 1))) + 4;
  const unsigned long long gmask = (P == 64 ? ~0ull : ((1ull << P) - 1)) << (grp * P);
  for (int it = 0; it < max_it; ++it) {
    const bool open = k < n && hi - lo > tol;  // uniform over the eigenvalue's lanes
    if (__ballot(open) == 0) break;
    const double x = lo + (hi - lo) * ((double)(pl + 1) / (double)(P + 1));
    const bool above = open && sturm_count(d, e, n, x, pivmin) > k;
    const unsigned long long m = __ballot(above) & gmask;
    const int first = m ? __ffsll((long long)m) - 1 - grp * P : P;  // first point above, in the group
    const double nhi = __shfl(x, grp * P + (first < P ? first : 0), 64);
    const double nlo = __shfl(x, grp * P + (first > 0 ? first - 1 : 0), 64);
    if (open) {
      if (first < P) hi = nhi;
      if (first > 0) lo = nlo;
    }
  }
  if (k < n && pl == 0) w.lam[(long)b * n + k] = bracket_estimate(lo, hi);
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

// The strictly lower triangle of each n x n Hermitian matrix from its upper triangle:
// A[i][j] = conj(A[j][i]) for i > j (column-major, ld n).  Workgroups walk 32 x 32 blocks
// of the lower triangle; the block's mirror image is staged through LDS so that both the
// reads and the writes run along columns.
__global__ __launch_bounds__(256) void hermitian_lower_kernel(cplx *A, int n) {
  const int nb = (n + 31) / 32;
  const int b = blockIdx.y;
  cplx *Ab = A + (long)b * n * n;
  __shared__ cplx t[32][33];
  for (int blk = blockIdx.x; blk < nb * (nb + 1) / 2; blk += gridDim.x) {
    int bj = (int)((sqrt(8.0 * blk + 1.0) - 1.0) * 0.5);  // block column of the upper triangle
    while (bj * (bj + 1) / 2 > blk) --bj;
    while ((bj + 1) * (bj + 2) / 2 <= blk) ++bj;
    const int bi = blk - bj * (bj + 1) / 2;  // bi <= bj: upper block (bi, bj) mirrors to (bj, bi)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {  // read upper block rows bi*32 + tx, columns bj*32 + r
      const int i = bi * 32 + tx, j = bj * 32 + r;
      if (i < n && j < n) t[r][tx] = Ab[i + (long)j * n];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {  // write lower block rows bj*32 + tx, columns bi*32 + r
      const int i = bj * 32 + tx, j = bi * 32 + r;
      if (i < n && j < n && i > j) {
        const cplx v = t[tx][r];
        Ab[i + (long)j * n] = cplx{v.re, -v.im};
      }
    }
  }
}

}  // namespace

hipError_t region_gram(const cplx *U, int L, int N, int B, const int *region, int nreg, cplx *A,
                       int *n_out, hipStream_t s) {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  g.batch = B;
  g.tri = TRI_UPPER;  // the upper triangle on the matrix cores, the lower one mirrored
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
  hipError_t e = zgemm(g, s);
  if (e != hipSuccess) return e;
  const int n = *n_out, nb = (n + 31) / 32;
  const unsigned blocks = (unsigned)std::min(nb * (nb + 1) / 2, 1024);
  hipLaunchKernelGGL(hermitian_lower_kernel, dim3(blocks, B), dim3(256), 0, s, A, n);
  return hipGetLastError();
}

namespace {

hipError_t tridiagonalize_blocked(const EigWork &w, int n, int B, hipStream_t s) {
  const int kstop = n - LDS_MAX_N;  // columns reduced in panels; the rest in LDS
  hipError_t err;
  const dim3 one(B), rt(TRD_REFLECT_THREADS);
  for (int k0 = 0; k0 < kstop; k0 += TRD_NB) {
    const int jp = std::min(TRD_NB, kstop - k0);
    for (int j = 0; j <= jp; ++j) {
      if (j >= 1) {  // y of reflector j - 1 and column k0 + j corrected by the panel
        const int rows = n - (k0 + j);
        const int tiled = rows >= TRD_TILED_MIN ? 1 : 0;  // the form of A v for reflector j - 1 (m = rows)
        hipLaunchKernelGGL(trd_panel_kernel, dim3((unsigned)((rows + TRD_PANEL_ROWS - 1) / TRD_PANEL_ROWS), B),
                           dim3(TRD_PANEL_TPR * TRD_PANEL_ROWS), 0, s, w, n, k0, jp, j - 1, j < jp ? 1 : 0,
                           tiled);
      }
      hipLaunchKernelGGL(trd_reflect_kernel<TRD_REFLECT_THREADS>, one, rt, 0, s, w, n, k0, jp, j);
      if ((err = hipGetLastError()) != hipSuccess) return err;
      if (j == jp) break;
      const long m = n - (k0 + j) - 1;
      if (m >= TRD_TILED_MIN) {
        const long T = (m + TRD_TILE - 1) / TRD_TILE, wgs = (T * (T + 1) / 2 + TRD_TPW - 1) / TRD_TPW;
        hipLaunchKernelGGL(trd_hemv_kernel, dim3((unsigned)std::max<long>(wgs, TRD_ZCH), B),
                           dim3(TRD_HEMV_THREADS), 0, s, w, n, k0, jp, j);
      } else {
        long gx;
        if ((gx = (m + 15) / 16) * B >= 512)
          hipLaunchKernelGGL(trd_hemv_cols_kernel<4>, dim3((unsigned)std::max<long>(gx, TRD_ZCH), B), dim3(256), 0,
                             s, w, n, k0, jp, j);
        else if ((gx = (m + 7) / 8) * B >= 512)
          hipLaunchKernelGGL(trd_hemv_cols_kernel<2>, dim3((unsigned)std::max<long>(gx, TRD_ZCH), B), dim3(256), 0,
                             s, w, n, k0, jp, j);
        else
          hipLaunchKernelGGL(trd_hemv_cols_kernel<1>, dim3((unsigned)std::max<long>((m + 3) / 4, TRD_ZCH), B),
                             dim3(256), 0, s, w, n, k0, jp, j);
      }
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    // A22 -= [V W] [W V]^+ over the trailing block
    const int k1 = k0 + jp, m = n - k1;
    GemmDesc g{};
    g.alpha = cplx{-1.0, 0.0};
    g.beta = cplx{1.0, 0.0};
    g.M = m; g.N = m; g.K = 2 * jp; g.batch = B;
    g.A = w.panel + k1; g.lda = n; g.sA = w.panel_stride; g.opA = OP_N;
    g.B = w.panel + (long)2 * TRD_NB * n + k1; g.ldb = n; g.sB = w.panel_stride; g.opB = OP_C;
    g.Cin = w.A + (long)k1 * (n + 1); g.ldcin = n; g.sCin = (long)n * n;
    g.D = w.A + (long)k1 * (n + 1); g.ldd = n; g.sD = (long)n * n;
    if ((err = zgemm(g, s)) != hipSuccess) return err;
  }
  hipLaunchKernelGGL(trd_tail_kernel, dim3(B), dim3(256), 0, s, w, n, kstop);
  return hipGetLastError();
}

}  // namespace

thread_local int tl_eig_path = EIG_PATH_AUTO;
void set_eig_path(int mode) { tl_eig_path = mode; }
int eig_path() { return tl_eig_path; }

namespace {

// Wall-clock ticks of the bulge chase's dependency-wait limit (10 s; a task takes microseconds).
long long chase_wait_ticks() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) !=
                                              hipSuccess || khz <= 0)
    return 1000000000LL;
  return 10000LL * khz;
}

}  // namespace

hipError_t tridiagonalize(const EigWork &w, int n, int B, hipStream_t s) {
  const bool two_ok = n >= 2 * TRD2_SB + 2 && w.panel && w.panel_stride >= trd2_scratch_elems(n) && w.flag && w.info;
  if (two_ok && (tl_eig_path == EIG_PATH_TWO_STAGE || (tl_eig_path == EIG_PATH_AUTO && n >= TRD2_AUTO_MIN)))
    return tridiagonalize_two_stage(w, n, B, chase_wait_ticks(), s);
  if (n <= LDS_MAX_N) {
    hipLaunchKernelGGL(tridiag_lds_kernel, dim3(B), dim3(256), 0, s, w, n);
    return hipGetLastError();
  }
  if (n >= TRD_BLOCKED_MIN && (double)n * n * B >= TRD_BLOCKED_WORK && w.panel &&
      w.panel_stride >= trd_panel_elems(n))
    return tridiagonalize_blocked(w, n, B, s);
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
  const long nb = (long)n * B;
  if (nb >= BISECT_LANES_MIN) {
    hipLaunchKernelGGL(bisect_kernel, dim3((n + 255) / 256, B), dim3(256), 0, s, w, n);
  } else {
    int P = 64;
    while (P > 2 && nb * P > BISECT_MULTI_LANES) P /= 2;
    const int per_wg = 4 * (64 / P);
    hipLaunchKernelGGL(bisect_multi_kernel, dim3((n + per_wg - 1) / per_wg, B), dim3(256), 0, s, w, n, P);
  }
  return hipGetLastError();
}

hipError_t entropy_sum(const EigWork &w, int n, int B, hipStream_t s) {
  hipLaunchKernelGGL(entropy_kernel, dim3(B), dim3(256), 0, s, w, n);
  return hipGetLastError();
}

}  // namespace mfq
