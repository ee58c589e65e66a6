// Host harness of the blocked Cholesky of a Cholesky-QR pass: the diagonal blocks go through
// the device kernel's own per-thread phase code (potrf_block.h), the 256 threads of each
// phase run one after another in three orders (ascending, descending, a fixed shuffle) that
// must give bitwise the same block (a read of another thread's write inside a phase, i.e. a
// missing barrier, would make them differ); the four lanes of a back-substitution column are
// combined as the two exchanges do and must agree bitwise.  The block rows, trailing updates
// and the level-by-level inverse are plain loops in the order of the device's launches.
//
// Usage: cholesky_block_harness in.bin out.bin
//   in:  int32 N, then the N x N complex Gram (column-major, upper triangle used)
//   out: int32 first bad column (-1: none), float64 its pivot, int32 order mismatches,
//        then R (N x N, upper, zeros below) and R^{-1} (N x N), complex column-major
// Built with the address and undefined-behaviour sanitizers by test_cholesky_block.py.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../paper_2508_18468_amd/csrc/potrf_block.h"

using mfq::cplx;
using mfq::PotrfLds;

static int mismatches = 0;

static bool same(const PotrfLds &x, const PotrfLds &y) { return std::memcmp(&x, &y, sizeof(PotrfLds)) == 0; }

// One phase for every thread, in the given order.
template <class F>
static void phase(PotrfLds &s, const std::vector<int> &order, F f) {
  for (int tid : order) f(s, tid);
}

// The phase in three thread orders from the same start; the results must agree bitwise.
template <class F>
static void checked_phase(PotrfLds &s, const std::vector<std::vector<int>> &orders, F f) {
  PotrfLds ref = s;
  phase(ref, orders[0], f);
  for (size_t o = 1; o < orders.size(); ++o) {
    PotrfLds alt = s;
    phase(alt, orders[o], f);
    if (!same(ref, alt)) ++mismatches;
  }
  s = ref;
}

// The device kernel's block factorisation: returns the first bad column of the block (w: none).
static int potrf_block_host(cplx *G, cplx *Rinv, long N, int c0, int w, double *bad_pivot,
                            const std::vector<std::vector<int>> &orders) {
  static PotrfLds s;  // large: keep it off the stack
  std::memset(&s, 0, sizeof(s));
  checked_phase(s, orders, [&](PotrfLds &t, int tid) { mfq::potrf_load(t, G, N, c0, w, tid); });
  for (int k = 0; k + 1 < w; ++k)
    checked_phase(s, orders, [&](PotrfLds &t, int tid) { mfq::potrf_eliminate(t, k, w, tid); });
  int first_bad = w;
  for (int t = 0; t < w; ++t)
    if (mfq::potrf_pivot(s, t)) first_bad = std::min(first_bad, t);
  checked_phase(s, orders, [&](PotrfLds &t, int tid) { mfq::potrf_scale(t, w, tid); });
  // back substitution: a wave's lane groups (one column each) are independent; the four lanes
  // of a group run in lockstep and exchange partial sums
  for (int j = 0; j < w; ++j) {
    const double dj = 1.0 / s.a[j][j].re;
    s.xd[j] = dj;
    for (int i = j - 1; i >= 0; --i) {
      double pr[4], pi[4];
      for (int q = 0; q < 4; ++q) mfq::potrf_inv_partial(s, i, j, q, dj, pr[q], pi[q]);
      double tr[4], ti[4], ur[4], ui[4];
      for (int q = 0; q < 4; ++q) {
        tr[q] = pr[q] + pr[q ^ 1];
        ti[q] = pi[q] + pi[q ^ 1];
      }
      for (int q = 0; q < 4; ++q) {
        ur[q] = tr[q] + tr[q ^ 2];
        ui[q] = ti[q] + ti[q ^ 2];
      }
      for (int q = 1; q < 4; ++q)
        if (std::memcmp(&ur[q], &ur[0], 8) || std::memcmp(&ui[q], &ui[0], 8)) ++mismatches;
      mfq::potrf_inv_store(s, i, j, ur[0], ui[0]);
    }
  }
  // the store reads the block only and writes each global element from one thread
  for (int tid = 0; tid < mfq::PB_THREADS; ++tid) mfq::potrf_store(s, G, Rinv, N, c0, w, tid);
  if (first_bad < w) *bad_pivot = s.piv[first_bad];
  return first_bad;
}

static cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
static cplx cmulc(cplx a, cplx b) { return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a) b

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t N32 = 0;
  if (std::fread(&N32, 4, 1, f) != 1 || N32 < 1 || N32 > 4096) return 2;
  const long N = N32;
  std::vector<cplx> G(N * N), Rinv(N * N, cplx{0.0, 0.0});
  if (std::fread(G.data(), sizeof(cplx), G.size(), f) != G.size()) return 2;
  std::fclose(f);
  auto g = [&](long r, long c) -> cplx & { return G[r + c * N]; };
  auto ri = [&](long r, long c) -> cplx & { return Rinv[r + c * N]; };

  std::vector<std::vector<int>> orders(3);
  for (int t = 0; t < mfq::PB_THREADS; ++t) {
    orders[0].push_back(t);
    orders[1].push_back(mfq::PB_THREADS - 1 - t);
    orders[2].push_back((t * 97 + 31) % mfq::PB_THREADS);  // 97 is odd: a permutation
  }

  const int NB = mfq::CHOL_NB;
  int first_bad = -1;
  double bad_pivot = 0.0;
  for (long p0 = 0; p0 < N; p0 += mfq::CHOL_OUTER) {
    const long p1 = std::min(N, p0 + (long)mfq::CHOL_OUTER);
    for (long c0 = p0; c0 < p1; c0 += NB) {
      const int w = (int)std::min<long>(NB, p1 - c0);
      double piv = 0.0;
      const int fb = potrf_block_host(G.data(), Rinv.data(), N, (int)c0, w, &piv, orders);
      if (fb < w && first_bad < 0) {
        first_bad = (int)c0 + fb;
        bad_pivot = piv;
      }
      const long r0 = c0 + w, nr = N - r0;
      if (nr <= 0) break;
      // block row: G[c0:c0+w, r0:] = R_JJ^{-+} G[c0:c0+w, r0:]
      std::vector<cplx> tmp((size_t)w * nr);
      for (long c = 0; c < nr; ++c)
        for (int m = 0; m < w; ++m) {
          cplx acc{0.0, 0.0};
          for (int k = 0; k < w; ++k) {
            const cplx a = ri(c0 + k, c0 + m), b = g(c0 + k, r0 + c);  // (R^{-1})^+_{mk} = conj(Rinv_km)
            const cplx t = cmulc(a, b);
            acc.re += t.re;
            acc.im += t.im;
          }
          tmp[m + c * w] = acc;
        }
      for (long c = 0; c < nr; ++c)
        for (int m = 0; m < w; ++m) g(c0 + m, r0 + c) = tmp[m + c * w];
      // the panel's later block rows (upper part): G[r0:p1, r0:] -= G[c0.., r0:p1]^+ G[c0.., r0:]
      for (long c = r0; c < N; ++c)
        for (long r = r0; r < std::min(p1, c + 1); ++r) {
          cplx acc{0.0, 0.0};
          for (int k = 0; k < w; ++k) {
            const cplx t = cmulc(g(c0 + k, r), g(c0 + k, c));
            acc.re += t.re;
            acc.im += t.im;
          }
          g(r, c).re -= acc.re;
          g(r, c).im -= acc.im;
        }
    }
    // below the panel (upper part): G[p1:, p1:] -= G[p0:p1, p1:]^+ G[p0:p1, p1:]
    for (long c = p1; c < N; ++c)
      for (long r = p1; r <= c; ++r) {
        cplx acc{0.0, 0.0};
        for (long k = p0; k < p1; ++k) {
          const cplx t = cmulc(g(k, r), g(k, c));
          acc.re += t.re;
          acc.im += t.im;
        }
        g(r, c).re -= acc.re;
        g(r, c).im -= acc.im;
      }
  }
  // R^{-1} level by level: [R11 R12; 0 R22]^{-1} has the block -R11^{-1} R12 R22^{-1}
  for (long S = NB; S < N; S *= 2)
    for (long r0 = 0; r0 + S < N; r0 += 2 * S) {
      const long wR = std::min(S, N - r0 - S);
      std::vector<cplx> T((size_t)S * wR);
      for (long c = 0; c < wR; ++c)
        for (long m = 0; m < S; ++m) {
          cplx acc{0.0, 0.0};
          for (long k = m; k < S; ++k) {
            const cplx t = cmul(ri(r0 + m, r0 + k), g(r0 + k, r0 + S + c));
            acc.re += t.re;
            acc.im += t.im;
          }
          T[m + c * S] = acc;
        }
      for (long c = 0; c < wR; ++c)
        for (long m = 0; m < S; ++m) {
          cplx acc{0.0, 0.0};
          for (long k = 0; k <= c; ++k) {
            const cplx t = cmul(T[m + k * S], ri(r0 + S + k, r0 + S + c));
            acc.re += t.re;
            acc.im += t.im;
          }
          ri(r0 + m, r0 + S + c) = cplx{-acc.re, -acc.im};
        }
    }
  FILE *o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  const int32_t fb32 = first_bad, mm = mismatches;
  std::fwrite(&fb32, 4, 1, o);
  std::fwrite(&bad_pivot, 8, 1, o);
  std::fwrite(&mm, 4, 1, o);
  for (long c = 0; c < N; ++c)
    for (long r = 0; r < N; ++r) {
      const cplx v = r <= c ? g(r, c) : cplx{0.0, 0.0};
      std::fwrite(&v, sizeof(cplx), 1, o);
    }
  std::fwrite(Rinv.data(), sizeof(cplx), Rinv.size(), o);
  std::fclose(o);
  std::printf("N=%ld first_bad=%d mismatches=%d\n", N, first_bad, mismatches);
  return 0;
}
