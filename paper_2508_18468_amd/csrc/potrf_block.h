// Factorisation and inversion of one CHOL_NB x CHOL_NB diagonal block of the blocked
// Cholesky of a Cholesky-QR pass (Appendix A: QR after each step).  Each function is the
// work of one thread (tid of a 256-thread workgroup) in one phase; the device kernel
// (potrf_diag_kernel) separates the phases by workgroup barriers, and a host harness
// (tests/cholesky_block_harness.cpp) runs the 256 threads of a phase one after another, so
// both execute this same code.
//
// The elimination runs without square roots: step k subtracts conj(G_ki) G_kj / G_kk from
// the trailing upper triangle, each thread owning a fixed 4 x 4 set of (row, column)
// positions; the rows of R are then scaled by 1/sqrt(G_kk).  The inverse is formed by back
// substitution with four lanes per column: lane q sums the terms l = i+1+q, i+5+q, ... of
// row i, the four partial sums are combined by two exchanges (xor 1, then xor 2), and it is
// kept transposed in the free lower triangle of the same array (its diagonal apart).
#pragma once

#include "cplx.h"
#include "workspace_layout.h"

#if defined(__HIPCC__)
#define MFQ_HD __host__ __device__
#else
#define MFQ_HD
#endif
#if defined(__clang__)
#define MFQ_UNROLL _Pragma("unroll")
#else
#define MFQ_UNROLL
#endif

namespace mfq {

constexpr int PB = CHOL_NB;
constexpr int PB_THREADS = 256;
constexpr int CHOL_OUTER = 8 * CHOL_NB;  // rows of R per outer panel of the blocked Cholesky

struct PotrfLds {
  // a[c][r], r <= c: element (row r, col c) of the block, then of R; a[r][c], r < c: element
  // (r, c) of R^{-1}
  cplx a[PB][PB + 1];
  double xd[PB];   // the diagonal of R^{-1}
  double rs[PB];   // square roots of the pivots
  double piv[PB];  // the pivots
};

// The upper triangle of the w x w block at (c0, c0) of the column-major N x N matrix Gb.
MFQ_HD inline void potrf_load(PotrfLds &s, const cplx *Gb, long N, int c0, int w, int tid) {
  for (int c = tid >> 6; c < w; c += 4)
    for (int r = tid & 63; r < w; r += 64)
      s.a[c][r] = (r <= c) ? Gb[(c0 + r) + (long)(c0 + c) * N] : cplx{0.0, 0.0};
}

// Elimination step k: rows and columns i, j > k of the trailing upper triangle.
MFQ_HD inline void potrf_eliminate(PotrfLds &s, int k, int w, int tid) {
  const int ti = tid & 15, tj = tid >> 4;  // rows ti + 16 p, columns tj + 16 q
  double d = s.a[k][k].re;
  if (!(d > 0.0) || !__builtin_isfinite(d)) d = 1.0;  // flagged by potrf_pivot
  const double inv = 1.0 / d;
MFQ_UNROLL
  for (int q = 0; q < PB / 16; ++q) {
    const int j = tj + 16 * q;
    if (j <= k || j >= w) continue;
    const cplx gkj = s.a[j][k];
    const double fr = gkj.re * inv, fi = gkj.im * inv;
MFQ_UNROLL
    for (int p = 0; p < PB / 16; ++p) {
      const int i = ti + 16 * p;
      if (i <= k || i > j) continue;
      const cplx gki = s.a[i][k];  // a[j][i] -= conj(G_ki) G_kj / G_kk
      s.a[j][i].re -= gki.re * fr + gki.im * fi;
      s.a[j][i].im -= gki.re * fi - gki.im * fr;
    }
  }
}

// Pivot t (t < w) after the elimination; true when it is non-positive or not finite (its
// square root is then taken as 1 so that the block stays finite).
MFQ_HD inline bool potrf_pivot(PotrfLds &s, int t) {
  const double d = s.a[t][t].re;
  s.piv[t] = d;
  const bool bad = !(d > 0.0) || !__builtin_isfinite(d);
  s.rs[t] = bad ? 1.0 : __builtin_sqrt(d);
  return bad;
}

// Rows of R: row r of the eliminated block divided by sqrt(pivot r), diagonal sqrt(pivot r).
MFQ_HD inline void potrf_scale(PotrfLds &s, int w, int tid) {
  for (int c = tid >> 6; c < w; c += 4)
    for (int r = tid & 63; r <= c; r += 64) {
      const double sc = 1.0 / s.rs[r];
      s.a[c][r] = r == c ? cplx{s.rs[r], 0.0} : cplx{s.a[c][r].re * sc, s.a[c][r].im * sc};
    }
}

// Lane q's part of sum_{l=i+1..j} R_il (R^{-1})_lj for column j (dj = 1 / R_jj).
MFQ_HD inline void potrf_inv_partial(const PotrfLds &s, int i, int j, int q, double dj, double &sr,
                                     double &si) {
  sr = 0.0;
  si = 0.0;
  for (int l = i + 1 + q; l <= j; l += 4) {
    const cplx r = s.a[l][i], t = l == j ? cplx{dj, 0.0} : s.a[l][j];
    sr += r.re * t.re - r.im * t.im;
    si += r.re * t.im + r.im * t.re;
  }
}

// (R^{-1})_ij = -(sum) / R_ii.
MFQ_HD inline void potrf_inv_store(PotrfLds &s, int i, int j, double sr, double si) {
  const double inv = 1.0 / s.a[i][i].re;
  s.a[i][j] = cplx{-sr * inv, -si * inv};
}

// R_JJ back into the upper triangle of the block of Gb, R_JJ^{-1} (zeros below its diagonal)
// into the block of Rb.
MFQ_HD inline void potrf_store(const PotrfLds &s, cplx *Gb, cplx *Rb, long N, int c0, int w, int tid) {
  for (int c = tid >> 6; c < w; c += 4)
    for (int r = tid & 63; r < w; r += 64) {
      if (r <= c) Gb[(c0 + r) + (long)(c0 + c) * N] = s.a[c][r];
      Rb[(c0 + r) + (long)(c0 + c) * N] =
          r < c ? s.a[r][c] : (r == c ? cplx{s.xd[r], 0.0} : cplx{0.0, 0.0});
    }
}

}  // namespace mfq
