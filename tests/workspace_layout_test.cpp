// Host-only checks of the device workspace layout (workspace_layout.h), built with the
// address and undefined-behaviour sanitizers by test_workspace_layout.py:
// * every region starts on a 256-byte boundary and lies inside the workspace;
// * no two regions overlap, and each device word (error flag, breakdown record,
//   near-identity deviation, step counter) owns a whole 256-byte slot, so that clearing one
//   slot never touches another;
// * the regions that other phases reuse are large enough for that reuse: the blocked
//   tridiagonalisation's panels in the Rinv region (n <= N), the Cholesky level products'
//   temporaries (N^2 / 2 entries) in the other state buffer (L N entries), the blocked
//   projective step's C_MM (k <= N rows) in G;
// * the sizes are computed without overflow for the largest shapes the API accepts.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "../paper_2508_18468_amd/csrc/workspace_layout.h"

using namespace mfq;

static int failures = 0;
#define CHECK(c)                                                                  \
  do {                                                                            \
    if (!(c)) {                                                                   \
      std::printf("FAIL line %d: %s (shape %s)\n", __LINE__, #c, name);           \
      ++failures;                                                                 \
    }                                                                             \
  } while (0)

struct Shape {
  const char *name;
  int dim, Lx, Ly, N, B;
};

static void check(const Shape &sh, bool fp32) {
  const char *name = sh.name;
  const WsLayout w = plan_workspace(sh.dim, sh.Lx, sh.Ly, sh.N, sh.B, fp32);
  const unsigned __int128 L = (unsigned __int128)sh.Lx * (sh.dim == 2 ? sh.Ly : 1);
  std::vector<std::pair<size_t, int>> present;
  unsigned __int128 sum = 0;
  for (int r = 0; r < WS_COUNT; ++r) {
    CHECK(w.off[r] % 256 == 0);
    CHECK(w.elem[r] > 0);
    // exact size, recomputed in 128-bit arithmetic: no wrap-around in the 64-bit plan
    const unsigned __int128 b = (unsigned __int128)w.count[r] * w.elem[r];
    CHECK(b == (unsigned __int128)w.bytes(r));
    CHECK((unsigned __int128)w.off[r] + b <= w.total);
    sum += (b + 255) / 256 * 256;
    if (w.count[r]) present.push_back({w.off[r], r});
  }
  CHECK(sum == w.total);
  std::sort(present.begin(), present.end());
  for (size_t i = 0; i + 1 < present.size(); ++i) {
    const int r = present[i].second, s = present[i + 1].second;
    CHECK(w.off[r] + w.bytes(r) <= w.off[s]);
  }
  // each device word in its own 256-byte slot
  const int words[] = {WS_FLAG, WS_INFO, WS_DEV, WS_STEP};
  for (int a : words) {
    CHECK(w.count[a] == 1);
    CHECK(w.bytes(a) <= 256);
    for (int b : words)
      if (a != b) CHECK(w.off[a] + 256 <= w.off[b] || w.off[b] + 256 <= w.off[a]);
    for (int r = 0; r < WS_COUNT; ++r)
      if (r != a && w.count[r]) CHECK(w.off[a] + 256 <= w.off[r] || w.off[r] + w.bytes(r) <= w.off[a]);
  }
  CHECK(sizeof(BreakdownInfo) <= 256);
  // state buffers and the N x N regions
  const unsigned __int128 LN = L * sh.N, NN = (unsigned __int128)sh.N * sh.N;
  CHECK(w.bytes(WS_X0) == LN * sh.B * 16 && w.bytes(WS_X1) == LN * sh.B * 16);
  CHECK(w.bytes(WS_G) == NN * sh.B * 16 && w.bytes(WS_RINV) == NN * sh.B * 16);
  CHECK(w.bytes(WS_P) == L * L * 16);
  CHECK((w.count[WS_PR32] != 0) == fp32);
  // reuse: tridiagonalisation panels in Rinv for every region size n <= N that takes them
  for (int n = TRD_BLOCKED_MIN; n <= sh.N; n += std::max(1, sh.N / 97))
    CHECK((unsigned __int128)trd_panel_elems(n) <= NN);
  if (sh.N >= TRD_BLOCKED_MIN) CHECK((unsigned __int128)trd_panel_elems(sh.N) <= NN);
  // two-stage reduction storage in Rinv for every region order n <= N the default form gives it
  for (int n = 1024; n <= sh.N; n += std::max(1, sh.N / 97))
    CHECK((unsigned __int128)trd2_scratch_elems(n) <= NN);
  if (sh.N >= 1024) CHECK((unsigned __int128)trd2_scratch_elems(sh.N) <= NN);
  // Cholesky level temporaries (at most N^2 / 2 per trajectory) in the other state buffer
  CHECK(NN / 2 <= LN);
  // per-site vectors of the projective and continuous-time steps: L per trajectory
  CHECK(w.count[WS_PM_SITES] == (size_t)(L * sh.B) && w.count[WS_CT_YP] == (size_t)(L * sh.B));
}

int main() {
  const Shape shapes[] = {
      {"ring64 x16", 1, 64, 1, 32, 16},
      {"ring1024 x384", 1, 1024, 1, 512, 384},
      {"ring16384 x2", 1, 16384, 1, 8192, 2},
      {"torus160 x3", 2, 160, 160, 12800, 3},
      {"ring200 N100 x7", 1, 200, 1, 100, 7},
      {"torus8x6 x5", 2, 8, 6, 24, 5},
      {"torus56x4", 2, 56, 4, 112, 1},
      {"ring4 N1", 1, 4, 1, 1, 1},
      {"ring64 x65535", 1, 64, 1, 32, 65535},
      {"ring 2^20 x1", 1, 1 << 20, 1, 1 << 19, 1},
      {"torus 1024^2 x1", 2, 1024, 1024, 1 << 19, 1},
      {"ring4096 N4095 x3", 1, 4096, 1, 4095, 3},
  };
  for (const Shape &s : shapes) {
    check(s, false);
    check(s, true);
  }
  // K-split partials of the two-stage reduction: one slice of both halves of X = A22 (V T) (m
  // rows, m <= n - TRD2_SB) and the most slices of the deep TRD2_SB x TRD2_SB products
  const char *name = "two-stage partials";
  for (int n = 2 * TRD2_SB + 2; n <= 70000; n += (n < 2048 ? 1 : 97)) {
    CHECK(trd2_kp_elems(n) >= 2L * TRD2_SB * (n - TRD2_SB));
    CHECK(trd2_kp_elems(n) >= (long)trd2_ks_max(n) * TRD2_SB * TRD2_SB);
  }
  // the panel products' K splits as the reduction forms them: slices non-empty, whole K chunks
  // when split, and both halves of X (and the 32 x 32 products) within the partial storage
  name = "two-stage K splits";
  const int batches[] = {1, 2, 3, 16, 384};
  for (int n = 2 * TRD2_SB + 2; n <= 20000; n += (n < 1024 ? 7 : 331))
    for (int B : batches)
      for (int j = 0; n - j - TRD2_SB >= 2; j += TRD2_SB) {
        const int m = n - j - TRD2_SB;
        const int kx = trd2_x_slices(n, m, B), ks = trd2_sb_slices(n, m, B);
        for (int q : {kx, ks}) {
          const int kc = trd2_slice_depth(m, q);
          CHECK(q >= 1 && q <= TRD2_KS);
          CHECK((long)(q - 1) * kc < m && m <= (long)q * kc);
          CHECK(q == 1 || kc % 16 == 0);
          CHECK(trd2_slice_count(m, q) == q);  // asking again for q slices gives the same split
        }
        CHECK(2L * kx * m * TRD2_SB <= trd2_kp_elems(n));
        CHECK((long)ks * TRD2_SB * TRD2_SB <= trd2_kp_elems(n));
      }
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("all passed\n");
  return 0;
}
