// Projective measurements of one step in blocked form, for lattices too large
// for one workgroup per trajectory (Appendix A: Eq. (A1), Eq. (A2) with the
// sign fixed).
//
// Measuring n_j = 1 keeps e_j and the part of the orbital space with zero
// amplitude on j; measuring n_j = 0 removes the amplitude on j.  For the sites
// M of a step with outcomes M1 (1) and M0 (0) the new orbital space is
//   span{e_j : j in M1}  +  P_M0 ( S  intersected with {u : u_j = 0, j in M1} ),
// S = range(U), P_M0 zeroing the rows M0, whatever the order.  The outcome
// draws of the sites, in ascending order, use the conditional Born
// probabilities, which depend only on C_MM = U_M U_M^+: p_t is the t-th
// diagonal entry of the Schur complement of the previous sites, eliminated
// with pivot C_tt (outcome 1, Eq. (A1)) or C_tt - 1 (outcome 0: adding
// C_.t C_t. / (1 - C_tt), Eq. (A2) with the sign fixed).  So a step is
//   1. selection: sites with u_sel < q in ascending order, their outcome draws;
//   2. C_MM on the matrix cores (gathered rows);
//   3. sequential elimination on C_MM with the outcome decided at each pivot;
//   4. LQ of the outcome-1 rows X = U_M1 by Householder reflectors from the
//      right (X Q = [L 0]), reflectors collected into V, in panels of LQ_PANEL
//      rows: each panel's reflectors one launch each on the panel's rows only,
//      then the rows below take the whole panel at once, X <- X (I - V T V^+),
//      as three GEMMs (X is kept conjugated and row-major, i.e. X^+ column-major,
//      so the update reads (I - V T^+ V^+) X^+);
//   5. U <- U Q in compact WY blocks of 128 where the N x N scratch holds them,
//      else 64 (U -= (U V T) V^+, three GEMMs; one pass over U per block);
//   6. columns 0..k1-1 := e_j (j in M1), measured rows of the other columns := 0.
// The Cholesky-QR of the step then normalises the columns that lost their
// M0 amplitude.  The host reads the site and outcome-1 counts (two stream
// synchronisations per step) to size steps 3-5.
#include <algorithm>
#include <vector>

#include "device_common.h"

namespace mfq {

namespace {

constexpr int WY = 64;    // width of a compact-WY block, and of one T-factor launch
constexpr int WY2 = 128;  // wide compact-WY block: two T factors of WY joined by GEMMs

__device__ __forceinline__ double wsum(double x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ double wmax(double x) {
  for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
  return x;
}

// One workgroup per trajectory: the measured sites in ascending order, their
// outcome draws (Philox purpose 0, words 0 and 1) and the count; entries past
// the count are set to site 0 (a valid row for padded gathers).
__global__ __launch_bounds__(256) void pm_select_kernel(int L, const double *gamma, double dt,
                                                        uint64_t seed, const uint64_t *uid,
                                                        const int64_t *step_ptr, int step_offset,
                                                        const int64_t *step_base, int *sites,
                                                        double *udraw, int *counts) {
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double q = fmin(gamma[b] * dt, 1.0);
  const uint64_t step = (uint64_t)(*step_ptr + step_offset - step_base[b]);
  int *sb = sites + (long)b * L;
  double *ub = udraw + (long)b * L;
  __shared__ int wave_cnt[4];
  __shared__ int total;
  if (tid == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < L; base += 256) {
    const int i = base + tid;
    bool sel = false;
    double u = 0.0;
    if (i < L) {
      const u64x4 r = philox4x64_10(seed, uid[b], step, (uint64_t)i, PURPOSE_PROJECTIVE, 0);
      sel = u01(r.v[0]) < q;
      u = u01(r.v[1]);
    }
    const unsigned long long m = __ballot(sel);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int off = total;
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    if (sel) {
      const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
      sb[pos] = i;
      ub[pos] = u;
    }
    __syncthreads();
    if (tid == 0) total += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
  const int k = total;
  for (int t = k + tid; t < L; t += 256) sb[t] = 0;
  if (tid == 0) counts[b] = k;
}

// Pivot t of the elimination on S = C_MM (lower triangle, ld = ld, per
// trajectory at S + b * sS): p = S_tt, outcome 1 iff u_t <= p, then
// S[i, j] -= S[i, t] conj(S[j, t]) / d for t < j <= i < k with d = p (outcome 1)
// or p - 1 (outcome 0).  One wave per column j.
__global__ __launch_bounds__(256) void pm_pivot_kernel(cplx *S, long sS, int ld, const int *counts,
                                                       const double *udraw, int L, int t,
                                                       int *outcomes, double *probs) {
  const int b = blockIdx.y;
  const int k = counts[b];
  if (t >= k) return;
  cplx *Sb = S + (long)b * sS;
  const double p = Sb[t + (long)t * ld].re;
  const double u = udraw[(long)b * L + t];
  const int outcome = u <= p ? 1 : 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    outcomes[(long)b * L + t] = outcome;
    probs[(long)b * L + t] = p;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = t + 1 + blockIdx.x * 4 + wave;
  if (j >= k) return;
  // u <= p > 0 for outcome 1 and p < u < 1 for outcome 0: d != 0
  const double inv = 1.0 / (outcome ? p : p - 1.0);
  const cplx cj = Sb[j + (long)t * ld];
  const double fr = cj.re * inv, fi = -cj.im * inv;  // conj(S[j, t]) / d
  for (int i = j + lane; i < k; i += 64) {
    const cplx ci = Sb[i + (long)t * ld];
    cplx s = Sb[i + (long)j * ld];
    s.re -= ci.re * fr - ci.im * fi;
    s.im -= ci.re * fi + ci.im * fr;
    Sb[i + (long)j * ld] = s;
  }
}

// One workgroup per trajectory: outcome-1 sites in ascending order (m1, k1)
// and a row code: -1 not measured, -2 outcome 0, c >= 0 outcome 1 (column c).
__global__ __launch_bounds__(256) void pm_split_kernel(const int *sites, const int *outcomes,
                                                       const int *counts, int L, int *m1, int *k1,
                                                       int *code) {
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = counts[b];
  const int *sb = sites + (long)b * L;
  const int *ob = outcomes + (long)b * L;
  int *mb = m1 + (long)b * L;
  int *cb = code + (long)b * L;
  for (int i = tid; i < L; i += 256) cb[i] = -1;
  __shared__ int wave_cnt[4];
  __shared__ int total;
  if (tid == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < k; base += 256) {
    const int t = base + tid;
    const bool one = t < k && ob[t] == 1;
    const unsigned long long m = __ballot(one);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int off = total;
    for (int w = 0; w < wave; ++w) off += wave_cnt[w];
    if (t < k) {
      if (one) {
        const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
        mb[pos] = sb[t];
        cb[sb[t]] = pos;
      } else {
        cb[sb[t]] = -2;
      }
    }
    __syncthreads();
    if (tid == 0) total += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
  if (tid == 0) k1[b] = total;
}

constexpr int LQ_PANEL = 32;  // reflectors per panel of the blocked LQ
constexpr int LQ_THREADS = 1024;  // one workgroup per row: few rows per launch, long rows
constexpr int LQ_KSPLIT = 16;  // K slices of the short, deep products (C_MM, the LQ panel's)

// X[r][:] = conj(U[m1[r], :]) (row-major, ld = N) for r < k1; grid (rows, trajectories).
// Used for the measured rows (m1 = sites, k1 = counts) and for the outcome-1 rows.
__global__ __launch_bounds__(256) void pm_gather_kernel(const cplx *U, int L, int N, const int *m1,
                                                        const int *k1, cplx *X, long sX) {
  const int r = blockIdx.x, b = blockIdx.y;
  if (r >= k1[b]) return;
  const cplx *Ub = U + (long)b * L * N;
  const int row = m1[(long)b * L + r];
  cplx *xr = X + (long)b * sX + (long)r * N;
  for (int c = threadIdx.x; c < N; c += 256) {
    const cplx u = Ub[row + (long)c * L];
    xr[c] = cplx{u.re, -u.im};
  }
}

// Columns k1 .. ncol-1 of V (N x ncol per trajectory, ld = N) set to zero.
__global__ __launch_bounds__(256) void pm_vpad_kernel(cplx *V, long sV, int N, const int *k1, int ncol) {
  const int c = blockIdx.x, b = blockIdx.y;
  if (c < k1[b] || c >= ncol) return;
  cplx *vc = V + (long)b * sV + (long)c * N;
  for (int i = threadIdx.x; i < N; i += 256) vc[i] = cplx{0.0, 0.0};
}

// Reflector t of the LQ of X (k1 x N), applied to the rows t+1 .. rend-1.  X is stored
// conjugated and row-major (Xs = conj(X)).  With z = Xs[t, t:] scaled by its largest component,
// H = I - tau v v^+, v = z - alpha e_0, alpha = -phase(z_0)|z|, so that x_t H is zero past
// column t.  One workgroup per row r in t .. rend-1, each forming (v, tau) from row t itself:
// row t's workgroup writes v into column t of V (zero above row t) and tau, the others apply
// x_r <- x_r H, i.e. Xs[r] -= tau conj(s) v with s = x_r v.
__global__ __launch_bounds__(LQ_THREADS) void pm_lq_kernel(cplx *X, long sX, int N, const int *k1, int t,
                                                           int rend, cplx *V, long sV, double *tau, int L) {
  const int b = blockIdx.y, tid = threadIdx.x;
  const int kb = min(k1[b], rend);
  const int r = t + blockIdx.x;
  if (t >= k1[b] || r >= kb) return;  // uniform over the workgroup
  __shared__ double red[LQ_THREADS / 64];
  cplx *Xb = X + (long)b * sX;
  const cplx *xt = Xb + (long)t * N;  // conj(x_t)
  // v scaled by its largest component (see make_reflector)
  double mx = 0.0;
  for (int c = t + tid; c < N; c += LQ_THREADS) mx = fmax(mx, cmax_abs(xt[c]));
  const double s = block_max_nt<LQ_THREADS>(mx, red);
  const double inv = s >= REFLECT_TINY ? 1.0 / s : 0.0;
  double tail = 0.0;
  for (int c = t + 1 + tid; c < N; c += LQ_THREADS) {
    const double re = xt[c].re * inv, im = xt[c].im * inv;
    tail += re * re + im * im;
  }
  tail = block_sum_nt<LQ_THREADS>(tail, red);
  double tt = 0.0;
  cplx v0{0.0, 0.0};
  if (tail > 0.0) {
    const Reflector h = make_reflector(cplx{xt[t].re * inv, xt[t].im * inv}, tail, s);
    v0 = h.v0;
    tt = h.tau;
  }
  if (r == t) {
    cplx *vt = V + (long)b * sV + (long)t * N;
    for (int c = tid; c < N; c += LQ_THREADS) {
      cplx v{0.0, 0.0};
      if (tt != 0.0 && c >= t) v = c == t ? v0 : cplx{xt[c].re * inv, xt[c].im * inv};
      vt[c] = v;
    }
    if (tid == 0) tau[(long)b * L + t] = tt;
    return;
  }
  if (tt == 0.0) return;
  cplx *xr = Xb + (long)r * N;
  double sr = 0.0, si = 0.0;  // s = x_r v = sum_c conj(Xs[r, c]) v_c
  for (int c = t + tid; c < N; c += LQ_THREADS) {
    const cplx v = c == t ? v0 : cplx{xt[c].re * inv, xt[c].im * inv};
    const cplx x = xr[c];
    sr += x.re * v.re + x.im * v.im;
    si += x.re * v.im - x.im * v.re;
  }
  sr = block_sum_nt<LQ_THREADS>(sr, red) * tt;
  si = block_sum_nt<LQ_THREADS>(si, red) * tt;
  for (int c = t + tid; c < N; c += LQ_THREADS) {  // Xs[r, c] -= tau conj(s) v_c
    const cplx v = c == t ? v0 : cplx{xt[c].re * inv, xt[c].im * inv};
    cplx x = xr[c];
    x.re -= sr * v.re + si * v.im;
    x.im -= sr * v.im - si * v.re;
    xr[c] = x;
  }
}

// out[b][i] = sum_s part[b][s][i] (i < n) in a fixed order: the K-split partial products of a
// short, deep product (C_MM, the LQ panel's V^+ [V X^+]; K = N).
__global__ __launch_bounds__(256) void pm_ksum_kernel(const cplx *part, long sPart, int ks, long n, cplx *out,
                                                      long sOut) {
  const int b = blockIdx.y;
  const long i = blockIdx.x * 256L + threadIdx.x;
  if (i >= n) return;
  const cplx *pb = part + (long)b * sPart;
  double re = 0.0, im = 0.0;
  for (int q = 0; q < ks; ++q) {
    const cplx x = pb[(long)q * n + i];
    re += x.re;
    im += x.im;
  }
  out[(long)b * sOut + i] = cplx{re, im};
}

// Triangular factor of a compact-WY block (columns c0 .. c0+w-1 of V):
// H_c0 ... H_c0+w-1 = I - V_b T V_b^+, T upper triangular with T_tt = tau_t and
// T[0:t, t] = -tau_t T[0:t, 0:t] (V_b^+ V_b)[0:t, t].  Thread i owns row i of T
// (row i of T depends only on row i and the Gram), so no barriers are needed.  G and T
// have leading dimensions ldg and ldt (sub-blocks of a wider block's Gram and T).
__global__ __launch_bounds__(64) void pm_tfactor_kernel(const cplx *Gb, long sG, int ldg, cplx *T, long sT,
                                                        int ldt, int w, const double *tau, const int *k1,
                                                        int c0, int L) {
  const int b = blockIdx.x, i = threadIdx.x;
  if (i >= w) return;
  const cplx *G = Gb + (long)b * sG;
  cplx *Tb = T + (long)b * sT;
  const int kb = k1[b];
  for (int t = 0; t < w; ++t) {
    const double tt = c0 + t < kb ? tau[(long)b * L + c0 + t] : 0.0;
    cplx out{0.0, 0.0};
    if (i < t) {
      double sr = 0.0, si = 0.0;
      for (int l = i; l < t; ++l) {
        const cplx a = Tb[i + (long)l * ldt], g = G[l + (long)t * ldg];
        sr += a.re * g.re - a.im * g.im;
        si += a.re * g.im + a.im * g.re;
      }
      out = cplx{-tt * sr, -tt * si};
    } else if (i == t) {
      out = cplx{tt, 0.0};
    }
    Tb[i + (long)t * ldt] = out;
  }
}

// Final form: column c < k1 := e_{m1[c]}; every measured row of the other
// columns := 0.  One workgroup per (column, trajectory).
__global__ __launch_bounds__(256) void pm_fix_kernel(cplx *U, int L, int N, const int *sites,
                                                     const int *counts, const int *k1,
                                                     const int *code) {
  const int c = blockIdx.x, b = blockIdx.y;
  cplx *col = U + (long)b * L * N + (long)c * L;
  const int kb = counts[b];
  if (kb == 0) return;
  if (c < k1[b]) {
    const int *cb = code + (long)b * L;
    for (int i = threadIdx.x; i < L; i += 256) col[i] = cplx{cb[i] == c ? 1.0 : 0.0, 0.0};
  } else {
    const int *sb = sites + (long)b * L;
    for (int t = threadIdx.x; t < kb; t += 256) col[sb[t]] = cplx{0.0, 0.0};
  }
}

GemmDesc desc() {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  return g;
}

}  // namespace

hipError_t pm_blocked(cplx *U, cplx *scratch, int L, int N, int B, const double *gamma, double dt,
                      uint64_t seed, const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                      const int64_t *step_base, const PmBlockedWork &w, bool *fallback,
                      hipStream_t s) {
  hipError_t e;
  *fallback = false;
  static_assert(PM_BLOCKED_MIN_N == 2 * WY, "the Gram and T of a WY block share one N x N scratch");
  if (N < PM_BLOCKED_MIN_N) {
    *fallback = true;
    return hipSuccess;
  }
  const long NN = (long)N * N;
  hipLaunchKernelGGL(pm_select_kernel, dim3(B), dim3(256), 0, s, L, gamma, dt, seed, uid, step_ptr,
                     step_offset, step_base, w.sites, w.udraw, w.counts);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  std::vector<int> cnt(B);
  if ((e = hipMemcpyAsync(cnt.data(), w.counts, B * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  int kmax = 0;
  for (int v : cnt) kmax = std::max(kmax, v);
  if (kmax == 0) return hipSuccess;
  if (kmax > N) {  // C_MM would not fit the N x N scratch
    *fallback = true;
    return hipSuccess;
  }
  // 2. C_MM = U_M U_M^+ into G (ld kmax): the measured rows gathered, conjugated, into R
  // (Y = U_M^+, N x kmax, ld N), then C_MM = Y^+ Y, a short (kmax rows) and deep (K = N)
  // product split over K into slices summed in a fixed order, partials in the idle state buffer
  // (rows past a trajectory's count are left unwritten: they reach only C_MM entries that the
  // elimination does not read)
  {
    hipLaunchKernelGGL(pm_gather_kernel, dim3(kmax, B), dim3(256), 0, s, U, L, N, w.sites, w.counts, w.R,
                       NN);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const long sPart = (long)L * N, n = (long)kmax * kmax;
    int ks = LQ_KSPLIT;  // slices of at least 128 rows, dividing N, partials within one state
    while (ks > 1 && (N % ks != 0 || N / ks < 128 || ks * n > sPart)) ks /= 2;
    const int kc = N / ks;
    GemmDesc g = desc();
    g.M = kmax; g.N = kmax; g.K = kc; g.batch = B * ks; g.batch2 = ks;
    g.A = w.R; g.lda = N; g.sA = NN; g.sA2 = kc; g.opA = OP_C;
    g.B = w.R; g.ldb = N; g.sB = NN; g.sB2 = kc; g.opB = OP_N;
    g.D = scratch; g.ldd = kmax; g.sD = sPart; g.sD2 = n;
    if ((e = zgemm(g, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(pm_ksum_kernel, dim3((unsigned)((n + 255) / 256), B), dim3(256), 0, s,
                       (const cplx *)scratch, sPart, ks, n, w.G, NN);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // 3. elimination with the outcome decided at each pivot
  for (int t = 0; t < kmax; ++t) {
    const int cols = std::max(1, (kmax - t - 1 + 3) / 4);
    hipLaunchKernelGGL(pm_pivot_kernel, dim3(cols, B), dim3(256), 0, s, w.G, NN, kmax, w.counts,
                       w.udraw, L, t, w.outcomes, w.probs);
  }
  hipLaunchKernelGGL(pm_split_kernel, dim3(B), dim3(256), 0, s, w.sites, w.outcomes, w.counts, L,
                     w.m1, w.k1, w.code);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(cnt.data(), w.k1, B * sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess)
    return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  int k1max = 0;
  for (int v : cnt) k1max = std::max(k1max, v);
  if (k1max > N) {  // more outcomes 1 than particles: only by rounding; U is still untouched
    *fallback = true;
    return hipSuccess;
  }
  if (k1max > 0) {
    // 4. LQ of the outcome-1 rows: X (row-major k1 x N) in R, reflectors in V = G (N x k1max)
    hipLaunchKernelGGL(pm_gather_kernel, dim3(k1max, B), dim3(256), 0, s, U, L, N, w.m1, w.k1, w.R, NN);
    hipLaunchKernelGGL(pm_vpad_kernel, dim3(k1max, B), dim3(256), 0, s, w.G, NN, N, w.k1, k1max);
    // panels of LQ_PANEL reflectors; the rows below a panel take it as X <- X (I - V T V^+) on the
    // stored X^+ (column-major N x k1max, ld N): Wh = V^+ X^+, Zh = T^+ Wh, X^+ -= V Zh.  Scratch:
    // the panel's Gram and T after X in R, Wh and Zh in w.T.
    const bool blocked_lq = k1max > LQ_PANEL && (long)k1max * N + 2L * LQ_PANEL * LQ_PANEL <= NN;
    const int panel = blocked_lq ? LQ_PANEL : k1max;
    for (int t0 = 0; t0 < k1max; t0 += panel) {
      const int t1 = std::min(k1max, t0 + panel);
      for (int t = t0; t < t1; ++t)
        hipLaunchKernelGGL(pm_lq_kernel, dim3(t1 - t, B), dim3(LQ_THREADS), 0, s, w.R, NN, N, w.k1, t, t1,
                           w.G, NN, w.tau, L);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int m = k1max - t1, wb = t1 - t0;
      if (!blocked_lq || m <= 0) continue;
      const cplx *Vb = w.G + (long)t0 * N;
      cplx *Gb = w.R + (long)k1max * N, *Tb = Gb + LQ_PANEL * LQ_PANEL;
      cplx *Wh = w.T, *Zh = w.T + (long)LQ_PANEL * k1max;
      cplx *Xr = w.R + (long)t1 * N;  // rows t1 .. of X, i.e. columns t1 .. of X^+
      // Gram V_b^+ V_b and Wh = V_b^+ X^+: short (wb rows) and deep (K = N) products, split over
      // K into LQ_KSPLIT slices (second batch dimension) and summed in a fixed order; partials in
      // the idle state buffer
      const long sPart = (long)L * N;
      int ks = LQ_KSPLIT;  // slices of at least 128 rows, dividing N, partials within one state
      while (ks > 1 && (N % ks != 0 || N / ks < 128 || (long)ks * LQ_PANEL * k1max > sPart)) ks /= 2;
      const int kc = N / ks;
      for (int which = 0; which < 2; ++which) {
        const int ncol = which == 0 ? wb : m;
        const long n = (long)wb * ncol;
        GemmDesc g = desc();
        g.M = wb; g.N = ncol; g.K = kc; g.batch = B * ks; g.batch2 = ks;
        g.A = Vb; g.lda = N; g.sA = NN; g.sA2 = kc; g.opA = OP_C;
        g.B = which == 0 ? Vb : Xr; g.ldb = N; g.sB = NN; g.sB2 = kc; g.opB = OP_N;
        g.D = scratch; g.ldd = wb; g.sD = sPart; g.sD2 = n;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(pm_ksum_kernel, dim3((unsigned)((n + 255) / 256), B), dim3(256), 0, s,
                           (const cplx *)scratch, sPart, ks, n, which == 0 ? Gb : Wh,
                           which == 0 ? NN : (long)N * WY);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (which == 0) {
          hipLaunchKernelGGL(pm_tfactor_kernel, dim3(B), dim3(64), 0, s, Gb, NN, wb, Tb, NN, wb, wb, w.tau,
                             w.k1, t0, L);
          if ((e = hipGetLastError()) != hipSuccess) return e;
        }
      }
      {  // Zh = T^+ Wh
        GemmDesc g = desc();
        g.M = wb; g.N = m; g.K = wb; g.batch = B;
        g.A = Tb; g.lda = wb; g.sA = NN; g.opA = OP_C;
        g.B = Wh; g.ldb = wb; g.sB = (long)N * WY; g.opB = OP_N;
        g.D = Zh; g.ldd = wb; g.sD = (long)N * WY;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
      {  // X^+ -= V_b Zh
        GemmDesc g = desc();
        g.M = N; g.N = m; g.K = wb; g.batch = B;
        g.A = Vb; g.lda = N; g.sA = NN; g.opA = OP_N;
        g.B = Zh; g.ldb = wb; g.sB = (long)N * WY; g.opB = OP_N;
        g.Cin = Xr; g.ldcin = N; g.sCin = NN;
        g.D = Xr; g.ldd = N; g.sD = NN;
        g.alpha = cplx{-1.0, 0.0};
        g.beta = cplx{1.0, 0.0};
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
    }
    // 5. U <- U Q, block by block.  In R: the Gram V_b^+ V_b and T (wb x wb each), then, for
    // blocks of WY2, V_b T (N x wb); for blocks of WY, V_b T in w.T.  W = U V_b T in scratch.
    // A block of WY2 columns takes T = [T1, -T1 G12 T2; 0, T2] from the T factors of its two
    // halves (G12: the Gram's off-diagonal block; -T1 G12 T2 via G12 T2 in w.T).
    const int wy = 2L * WY2 * WY2 + (long)N * WY2 <= NN ? WY2 : WY;
    for (int c0 = 0; c0 < k1max; c0 += wy) {
      const int wb = std::min(wy, k1max - c0);
      const int w1 = std::min(WY, wb), w2 = wb - w1;
      const cplx *Vb = w.G + (long)c0 * N;
      cplx *Gb = w.R;
      cplx *Tb = w.R + (long)wy * wy;
      cplx *VT = wy == WY2 ? w.R + 2L * WY2 * WY2 : w.T;
      const long sVT = wy == WY2 ? NN : (long)N * WY;
      {
        GemmDesc g = desc();
        g.M = wb; g.N = wb; g.K = N; g.batch = B;
        g.A = Vb; g.lda = N; g.sA = NN; g.opA = OP_C;
        g.B = Vb; g.ldb = N; g.sB = NN; g.opB = OP_N;
        g.D = Gb; g.ldd = wb; g.sD = NN;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
      hipLaunchKernelGGL(pm_tfactor_kernel, dim3(B), dim3(64), 0, s, Gb, NN, wb, Tb, NN, wb, w1, w.tau, w.k1,
                         c0, L);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      if (w2 > 0) {
        const long d2 = w1 + (long)w1 * wb;  // offset of the second half's diagonal block
        hipLaunchKernelGGL(pm_tfactor_kernel, dim3(B), dim3(64), 0, s, Gb + d2, NN, wb, Tb + d2, NN, wb, w2,
                           w.tau, w.k1, c0 + w1, L);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        {  // G12 T2 (w1 x w2) in w.T
          GemmDesc g = desc();
          g.M = w1; g.N = w2; g.K = w2; g.batch = B;
          g.A = Gb + (long)w1 * wb; g.lda = wb; g.sA = NN; g.opA = OP_N;
          g.B = Tb + d2; g.ldb = wb; g.sB = NN; g.opB = OP_N;
          g.D = w.T; g.ldd = w1; g.sD = (long)N * WY;
          if ((e = zgemm(g, s)) != hipSuccess) return e;
        }
        {  // T12 = -T1 (G12 T2)
          GemmDesc g = desc();
          g.M = w1; g.N = w2; g.K = w1; g.batch = B;
          g.A = Tb; g.lda = wb; g.sA = NN; g.opA = OP_N;
          g.B = w.T; g.ldb = w1; g.sB = (long)N * WY; g.opB = OP_N;
          g.D = Tb + (long)w1 * wb; g.ldd = wb; g.sD = NN;
          g.alpha = cplx{-1.0, 0.0};
          if ((e = zgemm(g, s)) != hipSuccess) return e;
        }
      }
      {  // V_b T: the first w1 columns are V_1 T1, the rest V_b [T12; T2]
        GemmDesc g = desc();
        g.M = N; g.N = w1; g.K = w1; g.batch = B;
        g.A = Vb; g.lda = N; g.sA = NN; g.opA = OP_N;
        g.B = Tb; g.ldb = wb; g.sB = NN; g.opB = OP_N;
        g.D = VT; g.ldd = N; g.sD = sVT;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
        if (w2 > 0) {
          g.N = w2; g.K = wb;
          g.B = Tb + (long)w1 * wb;
          g.D = VT + (long)w1 * N;
          if ((e = zgemm(g, s)) != hipSuccess) return e;
        }
      }
      {
        GemmDesc g = desc();
        g.M = L; g.N = wb; g.K = N; g.batch = B;
        g.A = U; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
        g.B = VT; g.ldb = N; g.sB = sVT; g.opB = OP_N;
        g.D = scratch; g.ldd = L; g.sD = (long)L * N;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
      {
        GemmDesc g = desc();
        g.M = L; g.N = N; g.K = wb; g.batch = B;
        g.A = scratch; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
        g.B = Vb; g.ldb = N; g.sB = NN; g.opB = OP_C;
        g.Cin = U; g.ldcin = L; g.sCin = (long)L * N;
        g.D = U; g.ldd = L; g.sD = (long)L * N;
        g.alpha = cplx{-1.0, 0.0};
        g.beta = cplx{1.0, 0.0};
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
    }
  }
  // 6. e_j columns for M1, measured rows cleared elsewhere
  hipLaunchKernelGGL(pm_fix_kernel, dim3(N, B), dim3(256), 0, s, U, L, N, w.sites, w.counts, w.k1, w.code);
  return hipGetLastError();
}

}  // namespace mfq
