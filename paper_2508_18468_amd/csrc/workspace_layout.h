// Byte layout of a context's device workspace.  Host code only (no HIP types), so that the
// library and its host-side checks (tests/workspace_layout_test.cpp, built with the address
// and undefined-behaviour sanitizers) use one definition.
//
// Every region starts on a 256-byte boundary of the (256-aligned) workspace base and holds
// `count` elements of `elem` bytes; absent regions have count 0.  The device words of a
// context (error flag, breakdown record, near-identity deviation, step counter) each get a
// region of their own.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>

// Size helpers that device code also calls (the two-stage reduction's scratch layout).
#if defined(__HIPCC__)
#define MFQ_LAYOUT_HD __host__ __device__
#else
#define MFQ_LAYOUT_HD
#endif

namespace mfq {

constexpr int CHOL_NB = 64;  // diagonal block of the blocked Cholesky (and width of its T panel)

// Panel width of the blocked Householder reduction, which keeps its per-matrix panel storage
// in the Rinv region (free outside a step), see trd_panel_elems.
constexpr int TRD_NB = 32;
constexpr int TRD_BLOCKED_MIN = 512;
// Complex entries of the blocked reduction's per-matrix storage: X and Y (n x 2 TRD_NB each),
// 16 row chunks of z partial sums (2 TRD_NB each), one v^+ y partial per 32 rows, and the row
// and column sums of A v per 64 x 64 tile (two n-vectors per tile row or column).
inline long trd_panel_elems(int n) {
  return (long)4 * TRD_NB * n + 16L * 2 * TRD_NB + (n + 31) / 32 + 2L * ((n + 63) / 64) * n;
}

// Two-stage reduction of region Grams (eig2.hip): band half-width of the first stage, panel
// rows per workgroup of its column launches, K slices of its deep products, and its per-matrix
// storage in the Rinv region (complex entries): X = [V W] and Y = [W V] (n x 2 TRD2_SB each),
// V T (n x TRD2_SB), the K-split partials, four TRD2_SB^2 blocks (V^+ V, T, V^+ X, T^+ V^+ X),
// tau, the column statistics of the column launches (two per workgroup), and n + 64 ints of
// progress words and counters of the bulge chase and the panel kernel.
constexpr int TRD2_SB = 32;
constexpr int TRD2_RPW = 128;
constexpr int TRD2_KS = 64;
MFQ_LAYOUT_HD inline int trd2_groups(int n) { return (n - TRD2_SB + TRD2_RPW - 1) / TRD2_RPW; }
// Most K slices of the deep TRD2_SB x TRD2_SB products of an order-n reduction (one per 128
// rows, at most TRD2_KS).
MFQ_LAYOUT_HD inline int trd2_ks_max(int n) {
  const int k = n / 128;
  return k < 1 ? 1 : (k > TRD2_KS ? TRD2_KS : k);
}
// K-split partials, the largest of: n^2 / 8 + n entries (the two m x TRD2_SB products of X take
// up to n^2 / (512 m) slices each), one slice of each of them (2 TRD2_SB n), and trd2_ks_max(n)
// slices of a TRD2_SB x TRD2_SB block.
MFQ_LAYOUT_HD inline long trd2_kp_elems(int n) {
  const long a = (long)n * n / 8 + n, b = (long)trd2_ks_max(n) * TRD2_SB * TRD2_SB, c = 2L * TRD2_SB * n;
  const long ab = a > b ? a : b;
  return ab > c ? ab : c;
}
// K splits of the band reduction's deep products (eig2.hip).  kslices: the largest power of two
// up to ksmax with at most `wgs` workgroups in all (`tiles` output tiles per matrix, B matrices)
// and slices at least `depth` deep.  A split of depth K asked for ks slices forms slices of
// trd2_slice_depth(K, ks) (whole K chunks of 16 when split), trd2_slice_count(K, ks) of them,
// every one non-empty.
MFQ_LAYOUT_HD inline int trd2_kslices(long tiles, int K, int B, long wgs, int depth, int ksmax) {
  int ks = 1;
  while (ks * 2 <= ksmax && tiles * B * ks * 2 <= wgs && K / (2 * ks) >= depth) ks *= 2;
  return ks;
}
MFQ_LAYOUT_HD inline int trd2_slice_depth(int K, int ks) {
  const int kc = (K + ks - 1) / ks;
  return ks > 1 ? (kc + 15) / 16 * 16 : kc;
}
MFQ_LAYOUT_HD inline int trd2_slice_count(int K, int ks) {
  return (K + trd2_slice_depth(K, ks) - 1) / trd2_slice_depth(K, ks);
}
MFQ_LAYOUT_HD inline long trd2_scratch_elems(int n) {
  return (long)n * 5 * TRD2_SB + trd2_kp_elems(n) + 4L * TRD2_SB * TRD2_SB + TRD2_SB +
         (long)trd2_groups(n) * 2 * (2 + 2 * TRD2_SB) + (n + 64 + 3) / 4;
}

// Slices of the panel products of order n with m rows below the band and B matrices: the two
// halves of X = A22 (V T) (m x TRD2_SB each, both sets of partials within trd2_kp_elems) and the
// TRD2_SB x TRD2_SB products V^+ V and V^+ X.
MFQ_LAYOUT_HD inline int trd2_x_slices(int n, int m, int B) {
  int ks = trd2_kslices((m + 63) / 64, m, B, 4096, 128, TRD2_KS);
  while (ks > 1 && 2L * ks * m * TRD2_SB > trd2_kp_elems(n)) ks /= 2;
  return trd2_slice_count(m, ks);
}
MFQ_LAYOUT_HD inline int trd2_sb_slices(int n, int m, int B) {
  return trd2_slice_count(m, trd2_kslices(1, m, B, 512, 64, trd2_ks_max(n)));
}

// Bessel-recurrence scratch length per trajectory (continuous-time protocol) for rings up to
// max(Lx, Ly): half the ring plus the recurrence's start-order margin.
inline int cont_jcap(int Lx, int Ly) {
  const int Lm = Lx > Ly ? Lx : Ly;
  return Lm / 2 + (int)std::ceil(std::sqrt(80.0 * Lm + 160.0)) + 64;
}

// Device record of the first Cholesky breakdown since the flag was last cleared.
struct BreakdownInfo {
  int32_t set;     // 0 until a breakdown is recorded
  int32_t source;  // 1: Cholesky-QR pass 1, 2: pass 2, 3: fused small-lattice kernel,
                   // 4: a dependency wait of the bulge chase exceeded its limit (no pivot),
                   // 5: a panel wait of the band reduction exceeded its limit (no pivot)
  int32_t traj;    // trajectory (batch index) of the pivot
  int32_t col;     // column of the pivot in the N x N Gram
  double pivot;    // its value (non-positive or not finite)
};

enum WsRegion {
  WS_X0, WS_X1, WS_P, WS_GX, WS_GY, WS_PKX, WS_PKY, WS_G, WS_RINV, WS_T,
  WS_BORN, WS_GAMMA, WS_UID, WS_OCC, WS_REGION,
  WS_FLAG, WS_INFO, WS_DEV, WS_STEP,
  WS_PM_SITES, WS_PM_OUT, WS_PM_CNT, WS_PM_PROB, WS_PM_V, WS_PM_W, WS_PM_U, WS_PM_TAU,
  WS_PM_M1, WS_PM_K1, WS_PM_CODE,
  WS_EV, WS_EW, WS_EP, WS_ETAU, WS_ED, WS_EE, WS_ELAM, WS_ES,
  WS_STEP_BASE,
  WS_CT_T, WS_CT_G, WS_CT_JN, WS_CT_INFO, WS_CT_DINFO, WS_CT_V, WS_CT_Y, WS_CT_YP,
  WS_PR32, WS_PI32,
  WS_COUNT
};

struct WsLayout {
  size_t off[WS_COUNT];
  size_t count[WS_COUNT];  // elements
  size_t elem[WS_COUNT];   // bytes per element
  size_t total;            // bytes from the aligned base to the end of the last region
  size_t bytes(int r) const { return count[r] * elem[r]; }
};

inline size_t ws_align(size_t x) { return (x + 255) & ~size_t(255); }

// Layout for a lattice (dim 1: Ly = 1) of L = Lx Ly sites, N particles, B trajectories;
// fp32_planes adds the FP32 planes of P - I of the FP32-bulk propagator.
inline WsLayout plan_workspace(int dim, int Lx, int Ly, int N, int B, bool fp32_planes) {
  const size_t L = (size_t)Lx * (dim == 2 ? Ly : 1), n = (size_t)N, b = (size_t)B;
  const size_t LN = L * n, NN = n * n;
  const int Lyr = dim == 2 ? Ly : 1;
  const size_t C = 16, D = 8, I = 4, F = 4;  // complex FP64, double / 64-bit int, int, float
  WsLayout w{};
  size_t off = 0;
  auto take = [&](int r, size_t count, size_t elem) {
    w.off[r] = off;
    w.count[r] = count;
    w.elem[r] = elem;
    off = ws_align(off + count * elem);
  };
  take(WS_X0, LN * b, C);
  take(WS_X1, LN * b, C);
  take(WS_P, L * L, C);
  take(WS_GX, L, C);
  take(WS_GY, L, C);
  take(WS_PKX, dim == 2 ? (size_t)Lx * Lx : 0, C);
  take(WS_PKY, dim == 2 ? (size_t)Ly * Ly : 0, C);
  take(WS_G, NN * b, C);
  take(WS_RINV, NN * b, C);
  take(WS_T, n * CHOL_NB * b, C);
  take(WS_BORN, L * b, D);
  take(WS_GAMMA, b, D);
  take(WS_UID, b, D);
  take(WS_OCC, n, I);
  take(WS_REGION, L, I);
  take(WS_FLAG, 1, I);
  take(WS_INFO, 1, sizeof(BreakdownInfo));
  take(WS_DEV, 1, D);
  take(WS_STEP, 1, D);
  take(WS_PM_SITES, L * b, I);
  take(WS_PM_OUT, L * b, I);
  take(WS_PM_CNT, b, I);
  take(WS_PM_PROB, L * b, D);
  take(WS_PM_V, n * b, C);
  take(WS_PM_W, L * b, C);
  take(WS_PM_U, L * b, D);
  take(WS_PM_TAU, L * b, D);
  take(WS_PM_M1, L * b, I);
  take(WS_PM_K1, b, I);
  take(WS_PM_CODE, L * b, I);
  take(WS_EV, 2 * n * b, C);
  take(WS_EW, n * b, C);
  take(WS_EP, n * b, C);
  take(WS_ETAU, 2 * b, D);
  take(WS_ED, n * b, D);
  take(WS_EE, n * b, D);
  take(WS_ELAM, n * b, D);
  take(WS_ES, b, D);
  take(WS_STEP_BASE, b, D);
  take(WS_CT_T, b, D);
  take(WS_CT_G, (size_t)(Lx + Lyr) * b, C);
  take(WS_CT_JN, (size_t)cont_jcap(Lx, Lyr) * b, D);
  take(WS_CT_INFO, 4 * b, I);
  take(WS_CT_DINFO, 4 * b, D);
  take(WS_CT_V, n * b, C);
  take(WS_CT_Y, L * b, C);
  take(WS_CT_YP, L * b, C);
  take(WS_PR32, fp32_planes ? L * L : 0, F);
  take(WS_PI32, fp32_planes ? L * L : 0, F);
  w.total = off;
  return w;
}

}  // namespace mfq
