// Batched complex FP64 GEMM on the CDNA4 FP64 matrix cores.
//
// Used for every dense contraction of a step: the propagator product U <- P U,
// the Gram matrices of the Cholesky-QR passes and of a region (C_A = U_A U_A^+),
// the trailing updates of the blocked Cholesky, the triangular inverse and the
// product U R^{-1}.
//
// Complex arithmetic is done as four real products on v_mfma_f64_16x16x4f64:
//   Re D += Ar*Br - Ai*Bi,  Im D += Ar*Bi + Ai*Br
// (8 real flops per complex multiply-add).  Real and imaginary parts are
// de-interleaved into separate LDS planes so that each MFMA operand is one
// double per lane.
//
// Tiling: a workgroup owns an MT x NT complex tile of D; its wave64s form a
// 2 x (NT/32) grid and each owns a block of 16 x 16 MFMA outputs with separate
// real and imaginary accumulators.  Shapes:
//   64 x 64,   4 waves, 32 x 32 per wave   small or thin contractions;
//   128 x 128, 8 waves, 64 x 32 per wave   the large ones: half the L2->CU
//              bytes per flop of the small tile, 64 accumulator doubles per
//              lane (more per wave would overflow the register file);
//   128 x 64,  4 waves, 64 x 32 per wave   the other large products with
//              op(A) = A and a general result (the products with R^-1 among them);
//   64 x 32 and 32 x 32, 2 waves           results at most 32 columns wide.
// K advances in chunks of 16; the next chunk is fetched into registers while the
// current one feeds the matrix cores.  Products with op(A) = A (the propagator among
// them) store it into their one LDS buffer between two barriers (66 KiB for
// 128 x 128 tiles, whose ~208 VGPRs per lane allow one 512-thread workgroup per
// compute unit; 128 x 64 tiles fit two); the Gram-shaped products
// (op(A) = A^+) and the reduction
// epilogues keep two buffers, store the next chunk after the first MFMA k-step of the
// current one and pass one barrier per chunk.
//
// Workgroup -> tile mapping is XCD-aware: the dispatcher hands workgroup i to
// XCD i mod 8, so the 1-D grid is ordered such that all tiles of one batch
// entry (or, for a single wide matrix, all row tiles of one column panel) run
// on the same XCD and share its L2.
//
// MFMA lane layout (gfx950, checked on hardware): operand A lane l holds
// A[l % 16][l / 16], operand B holds B[l / 16][l % 16]; output register r of
// lane l is D[l / 16 + 4 r][l % 16].
#include "mfq_internal.h"

namespace mfq {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int PAD = 1, NXCD = 8;

struct TileMap {
  int tilesM, tilesN, groups, per_group;  // group = batch entry, or (batch, column panel)
  bool by_panel, upper;                   // upper: only tiles with tm <= tn are launched
  bool linear;                            // fewer groups than XCDs: plain linear order
};

__host__ __device__ inline TileMap make_map(int M, int N, int batch, int MT, int NT, int tri,
                                            int linear_order) {
  TileMap t;
  t.tilesM = (M + MT - 1) / MT;
  t.tilesN = (N + NT - 1) / NT;
  t.upper = tri == TRI_UPPER && MT == NT && t.tilesM == t.tilesN;
  t.by_panel = !t.upper && batch < NXCD;
  t.groups = t.by_panel ? batch * t.tilesN : batch;
  t.per_group = t.by_panel ? t.tilesM
              : t.upper ? t.tilesM * (t.tilesM + 1) / 2 : t.tilesM * t.tilesN;
  t.linear = linear_order != 0 || t.groups < NXCD;
  return t;
}

// Index t of the upper-triangle tiles, column by column: (0,0), (0,1), (1,1), (0,2), ...
__device__ inline void upper_tile(int t, int &tm, int &tn) {
  int c = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (c * (c + 1) / 2 > t) --c;
  while ((c + 1) * (c + 2) / 2 <= t) ++c;
  tn = c;
  tm = t - c * (c + 1) / 2;
}

// FL: compile-time features, so that the plain contractions carry none of their code.
enum { FL_MASK = 1,      // triangular operands (aUpper / bUpper) masked at load
       FL_NEAR_ID = 2,   // near-identity epilogue (R1, maxdev)
       FL_SQSUM = 4,     // per-tile sum of |D_ij|^2 into part (D not written)
       FL_DIAG = 8 };    // per-tile sums of |D_ij|^2, i < j, along each diagonal (D not written)

// Reduction epilogues.  scratch: the A-plane LDS of the tile (2 KT (MT + 1) doubles), free
// once the K loop is over.  Every sum runs in a fixed order, so results are reproducible.
template <int MT, int NT, int KT, bool EDGE, int FL, int IM, int JN>
__device__ __forceinline__ void reduce_epilogue(const GemmDesc &g, const d4 (&acc_re)[IM][JN],
                                                const d4 (&acc_im)[IM][JN], double *scratch, int b,
                                                int t, int tm, int tn, int m0, int n0, int n_upper,
                                                int n_tiles) {
  constexpr int WM = 2, WN = NT / 32, NTHR = 64 * WM * WN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WM, wc = wave / WM;
  auto value = [&](int i, int j, int r, int &lr, int &lc) {
    lr = wr * (MT / WM) + i * 16 + (lane >> 4) + 4 * r;
    lc = wc * (NT / WN) + j * 16 + (lane & 15);
    const int row = m0 + lr, col = n0 + lc;
    bool ok = !EDGE || (row < g.M && col < g.N);
    if ((FL & FL_DIAG) != 0) ok = ok && row < col;
    if (!ok) return 0.0;
    const double xr = acc_re[i][j][r], xi = acc_im[i][j][r];
    const double yr = g.alpha.re * xr - g.alpha.im * xi, yi = g.alpha.re * xi + g.alpha.im * xr;
    return yr * yr + yi * yi;
  };
  if constexpr ((FL & FL_SQSUM) != 0) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < IM; ++i)
#pragma unroll
      for (int j = 0; j < JN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int lr, lc;
          s += value(i, j, r, lr, lc);
        }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    __syncthreads();
    if (lane == 0) scratch[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int w = 0; w < NTHR / 64; ++w) tot += scratch[w];
      g.part[(long)b * n_tiles + tm + (long)tn * ((g.M + MT - 1) / MT)] = tot;
    }
  } else {
    // diagonal d = lc - lr in [-(MT-1), NT-1], offset o = d + MT - 1; the tile passes
    // through the scratch CR rows at a time
    constexpr int ND = MT + NT - 1, CR = 2 * KT * (MT + 1) / NT, NQ = (ND + NTHR - 1) / NTHR;
    double accd[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) accd[q] = 0.0;
    for (int r0 = 0; r0 < MT; r0 += CR) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            int lr, lc;
            const double v = value(i, j, r, lr, lc);
            if (lr >= r0 && lr < r0 + CR) scratch[(lr - r0) * NT + lc] = v;
          }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int o = tid + NTHR * q;
        if (o >= ND) continue;
        const int d = o - (MT - 1);
        for (int lr = r0; lr < r0 + CR; ++lr) {
          const int lc = lr + d;
          if (lc >= 0 && lc < NT) accd[q] += scratch[(lr - r0) * NT + lc];
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int o = tid + NTHR * q;
      if (o < ND) g.part[((long)b * n_upper + t) * ND + o] = accd[q];
    }
  }
}

// GATHER: storage rows of A / B are looked up through idxA / idxB.
// EDGE: bounds-checked loads and stores (M, N or K not multiples of the tile).

// Offset of batch entry b for the strides (s, s2) of one operand.
__device__ __forceinline__ long batch_offset(const GemmDesc &g, int b, long s, long s2) {
  if (g.batch2 <= 1) return (long)b * s;
  return (long)(b / g.batch2) * s + (long)(b % g.batch2) * s2;
}

template <int OPA, int OPB, int MT, int NT, int KT, bool GATHER, bool EDGE, int FL = 0>
__device__ __forceinline__ void zgemm_body(const GemmDesc &g) {
  // waves: 2 along M; NT/32 along N (2 for 64x64 tiles, 4 for 128x128 tiles)
  constexpr int WM = 2, WN = NT / 32, NTHR = 64 * WM * WN;
  constexpr int IM = MT / WM / 16, JN = NT / WN / 16;  // 16x16 blocks per wave
  constexpr int LA = MT * KT / NTHR, LB = NT * KT / NTHR;
  if (g.skip_if_le && *g.skip_if_le <= g.skip_thr) return;
  const TileMap map = make_map(g.M, g.N, g.batch, MT, NT, g.tri, g.linear_order);
  const int id = blockIdx.x;
  const int k_on_xcd = map.linear ? id : id / NXCD;
  const int grp = map.linear ? id / map.per_group : id % NXCD + NXCD * (k_on_xcd / map.per_group);
  const int t = k_on_xcd % map.per_group;
  if (grp >= map.groups) return;
  int b, tm, tn;
  if (map.by_panel) {
    b = grp / map.tilesN;
    tn = grp % map.tilesN;
    tm = t;
  } else if (map.upper) {
    b = grp;
    upper_tile(t, tm, tn);
  } else {
    b = grp;
    tm = t % map.tilesM;
    tn = t / map.tilesM;
  }
  const int m0 = tm * MT, n0 = tn * NT;
  if (g.tri == TRI_UPPER && m0 > n0 + NT - 1) return;  // tile entirely below the diagonal
  if (g.tri == TRI_LOWER && n0 > m0 + MT - 1) return;  // tile entirely above the diagonal
  // global K index of local index 0 (the triangular masks compare it with m and n)
  const int kg0 = g.kofs + (g.batch2 > 1 ? (b % g.batch2) * g.kofs2 : 0);
  int kbeg = 0, kend = g.K;
  if (g.aUpper && m0 > kg0) kbeg = ((m0 - kg0) / KT) * KT;
  if (g.bUpper) kend = min(kend, max(0, n0 + NT - kg0));
  if (g.aLower) kend = min(kend, max(0, m0 + MT - kg0));
  if (g.kend_glob > 0) kend = min(kend, max(0, g.kend_glob - kg0));

  // Two buffers for the Gram-shaped products (op(A) = A^+) and the reduction epilogues: the
  // next chunk is stored into the idle buffer after the current one's first k-step, and one
  // barrier per chunk remains (Gram U^+U at L = 1024, N = 512, 384 trajectories: 0.667 ->
  // 0.695 of the FP64 peak).  The propagator product gains nothing from it and keeps one, and
  // so do the 32-column tiles, whose load must then land only at the end of the chunk and
  // whose single buffer lets four workgroups share a compute unit (the conjugate half of the
  // band reduction's X: 93 -> 82 ms per two 8192-site Grams).
  constexpr int NBUF = ((FL & (FL_SQSUM | FL_DIAG)) != 0 || (OPA == OP_C && NT > 32)) ? 2 : 1;
  __shared__ double Ar[NBUF][KT][MT + PAD], Ai[NBUF][KT][MT + PAD];
  __shared__ double Br[NBUF][KT][NT + PAD], Bi[NBUF][KT][NT + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WM, wc = wave / WM;
  const cplx *A = g.A + batch_offset(g, b, g.sA, g.sA2);
  const cplx *B = g.B + batch_offset(g, b, g.sB, g.sB2);
  const int *idxA = GATHER && g.idxA ? g.idxA + (long)b * g.sIdxA : nullptr;
  const int *idxB = GATHER && g.idxB ? g.idxB + (long)b * g.sIdxB : nullptr;

  // per-thread tile coordinates: element i of this thread is (m_a, k_a + i*da) of the
  // A tile and (k_b + i*db, n_b) of the B tile
  constexpr int DA = OPA == OP_N ? NTHR / MT : NTHR / KT;
  constexpr int DB = OPB == OP_N ? NTHR / KT : NTHR / NT;
  const int a_fast = OPA == OP_N ? tid % MT : tid % KT;  // contiguous direction in storage
  const int a_slow = OPA == OP_N ? tid / MT : tid / KT;
  const int b_fast = OPB == OP_N ? tid % KT : tid % NT;
  const int b_slow = OPB == OP_N ? tid / KT : tid / NT;

  double ra_re[LA], ra_im[LA], rb_re[LB], rb_im[LB];

  // Gathered rows that stay fixed over the K loop, read once: with op(A) = A every element of
  // this thread lies in tile row a_fast, with op(B) = B^+ in tile column b_fast.
  long a_row = 0, b_row = 0;
  if constexpr (OPA == OP_N) {
    const int gm = m0 + a_fast;
    a_row = (GATHER && idxA) ? (gm < g.M ? idxA[gm] : 0) : gm;
  }
  if constexpr (OPB == OP_C) {
    const int gn = n0 + b_fast;
    b_row = (GATHER && idxB) ? (gn < g.N ? idxB[gn] : 0) : gn;
  }

  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int m = OPA == OP_N ? a_fast : a_slow + DA * i;
      const int k = OPA == OP_N ? a_slow + DA * i : a_fast;
      const int gm = m0 + m, gk = k0 + k;
      double re = 0.0, im = 0.0;
      const int kgl = gk + kg0;  // global K index
      const bool zero = (FL & FL_MASK) && ((g.aUpper && (kgl < gm || (g.aUpper == 2 && kgl == gm))) ||
                                           (g.aLower && kgl > gm));
      if ((!EDGE || (gm < g.M && gk < kend)) && !zero) {
        cplx v;
        if (OPA == OP_N) {
          v = A[a_row + (long)gk * g.lda];
        } else {
          const long row = idxA ? idxA[gk] : gk;
          v = A[row + (long)gm * g.lda];
          v.im = -v.im;
        }
        re = v.re; im = v.im;
      }
      ra_re[i] = re; ra_im[i] = im;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int n = OPB == OP_N ? b_slow + DB * i : b_fast;
      const int k = OPB == OP_N ? b_fast : b_slow + DB * i;
      const int gn = n0 + n, gk = k0 + k;
      double re = 0.0, im = 0.0;
      if ((!EDGE || (gn < g.N && gk < kend)) && !((FL & FL_MASK) && g.bUpper && gk + kg0 > gn)) {
        cplx v;
        if (OPB == OP_N) {
          const long row = idxB ? idxB[gk] : gk;
          v = B[row + (long)gn * g.ldb];
        } else {
          v = B[b_row + (long)gk * g.ldb];
          v.im = -v.im;
        }
        re = v.re; im = v.im;
      }
      rb_re[i] = re; rb_im[i] = im;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int m = OPA == OP_N ? a_fast : a_slow + DA * i;
      const int k = OPA == OP_N ? a_slow + DA * i : a_fast;
      Ar[buf][k][m] = ra_re[i];
      Ai[buf][k][m] = ra_im[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int n = OPB == OP_N ? b_slow + DB * i : b_fast;
      const int k = OPB == OP_N ? b_fast : b_slow + DB * i;
      Br[buf][k][n] = rb_re[i];
      Bi[buf][k][n] = rb_im[i];
    }
  };

  d4 acc_re[IM][JN], acc_im[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      acc_re[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      acc_im[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    }

  const int nk = kend > kbeg ? (kend - kbeg + KT - 1) / KT : 0;
  if (nk > 0) {
    load(kbeg);
    store(0);
    __syncthreads();
  }
  for (int it = 0; it < nk; ++it) {
    const int buf = NBUF == 2 ? (it & 1) : 0;
    if (it + 1 < nk) load(kbeg + (it + 1) * KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      // the idle buffer was last read in the previous chunk, before its closing barrier
      if (NBUF == 2 && kk == 4 && it + 1 < nk) store(buf ^ 1);
      const int k = kk + (lane >> 4);
      double a_re[IM], a_im[IM], b_re[JN], b_im[JN];
#pragma unroll
      for (int i = 0; i < IM; ++i) {
        const int row = wr * (MT / WM) + i * 16 + (lane & 15);
        a_re[i] = Ar[buf][k][row];
        a_im[i] = Ai[buf][k][row];
      }
#pragma unroll
      for (int j = 0; j < JN; ++j) {
        const int col = wc * (NT / WN) + j * 16 + (lane & 15);
        b_re[j] = Br[buf][k][col];
        b_im[j] = Bi[buf][k][col];
      }
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_re[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_im[j], acc_im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < IM; ++i) {
        const double a_nim = -a_im[i];
#pragma unroll
        for (int j = 0; j < JN; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_nim, b_im[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_im[i], b_re[j], acc_im[i][j], 0, 0, 0);
        }
      }
    }
    if (NBUF == 1) {
      __syncthreads();  // every wave is done with the buffer
      if (it + 1 < nk) store(0);
    }
    __syncthreads();
  }

  if constexpr ((FL & (FL_SQSUM | FL_DIAG)) != 0) {
    reduce_epilogue<MT, NT, KT, EDGE, FL>(g, acc_re, acc_im, &Ar[0][0][0], b, t, tm, tn, m0, n0,
                                          map.per_group, map.tilesM * map.tilesN);
    return;
  }
  // epilogue: D = alpha * acc + beta * Cin
  const bool useC = (g.beta.re != 0.0 || g.beta.im != 0.0);
  const cplx *Cin = g.Cin ? g.Cin + batch_offset(g, b, g.sCin, g.sCin2) : nullptr;
  cplx *D = g.D + batch_offset(g, b, g.sD, g.sD2);
  cplx *R1 = (FL & FL_NEAR_ID) ? g.R1 + batch_offset(g, b, g.sD, g.sD2) : nullptr;
  double dmax = 0.0;
  const double qnan = __longlong_as_double(0x7ff8000000000000ll);
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * (MT / WM) + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wc * (NT / WN) + j * 16 + (lane & 15);
        if (EDGE && (row >= g.M || col >= g.N)) continue;
        if (g.tri == TRI_UPPER && row > col) continue;
        if (g.tri == TRI_LOWER && row < col) continue;
        const double xr = acc_re[i][j][r], xi = acc_im[i][j][r];
        double yr = g.alpha.re * xr - g.alpha.im * xi;
        double yi = g.alpha.re * xi + g.alpha.im * xr;
        if (useC) {
          const cplx c = Cin[row + (long)col * g.ldcin];
          yr += g.beta.re * c.re - g.beta.im * c.im;
          yi += g.beta.re * c.im + g.beta.im * c.re;
        }
        D[row + (long)col * g.ldd] = cplx{yr, yi};
        if (FL & FL_NEAR_ID) {
          const double er = row == col ? yr - 1.0 : yr;
          const double a = fabs(er) + fabs(yi);
          dmax = (!(a <= 1e300) || dmax != dmax) ? qnan : fmax(dmax, a);
          R1[row + (long)col * g.ldd] = row == col ? cplx{1.0 - 0.5 * er, 0.0} : cplx{-yr, -yi};
        }
      }
  if (FL & FL_NEAR_ID) {  // non-negative doubles order like their bit patterns; NaN is above them all
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(dmax, o, 64);
      dmax = (y != y || dmax != dmax) ? qnan : fmax(dmax, y);
    }
    if (lane == 0)
      atomicMax(reinterpret_cast<unsigned long long *>(g.maxdev),
                (unsigned long long)__double_as_longlong(dmax));
  }
}

template <int MT>
constexpr int kchunk() { return 16; }
template <int NT>
constexpr int nthreads() { return 64 * 2 * (NT / 32); }

template <int OPA, int OPB, int MT, int NT, bool GATHER, bool EDGE, int FL = 0>
__global__ __launch_bounds__(nthreads<NT>()) void zgemm_kernel(GemmDesc g) {
  zgemm_body<OPA, OPB, MT, NT, kchunk<MT>(), GATHER, EDGE, FL>(g);
}

// The propagator product U <- P U gets its own symbols so that profilers can
// tell it apart from the other contractions of a step.  It keeps 128 x 128 tiles:
// the 128 x 64 form of the other op(A) = A products ran it 0.5-1.6 % faster on the
// 160x160 torus but fetched twice the HBM bytes (6.7 against 3.3 TB per launch).
template <bool EDGE>
__global__ __launch_bounds__(512) void propagator_zgemm_kernel(GemmDesc g) {
  zgemm_body<OP_N, OP_N, 128, 128, kchunk<128>(), false, EDGE>(g);
}
template <bool EDGE>
__global__ __launch_bounds__(256) void propagator_zgemm_kernel_t64(GemmDesc g) {
  zgemm_body<OP_N, OP_N, 64, 64, kchunk<64>(), false, EDGE>(g);
}

// Tile choice and tile order of the calling thread (see set_gemm_tile_mode and
// set_gemm_tile_order).
thread_local int tl_tile_mode = GEMM_TILE_AUTO;
thread_local int tl_tile_order = GEMM_ORDER_XCD;

template <int MT, int NT>
unsigned grid_size(const GemmDesc &g) {
  const TileMap t = make_map(g.M, g.N, g.batch, MT, NT, g.tri, g.linear_order);
  if (t.linear) return (unsigned)((long)t.groups * t.per_group);
  const long groups_per_xcd = (t.groups + NXCD - 1) / NXCD;
  return (unsigned)(groups_per_xcd * NXCD * t.per_group);
}

template <int MT, int NT>
bool needs_edge(const GemmDesc &g) {
  constexpr int KT = kchunk<MT>();
  return (g.M % MT) || (g.N % NT) || (g.K % KT) || (g.kend_glob % KT);
}

template <int MT, int NT, bool GATHER, bool EDGE, int FL = 0>
void launch_ops(const GemmDesc &g, dim3 grid, hipStream_t s) {
  const dim3 block(nthreads<NT>());
  if (g.opA == OP_N && g.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_N, MT, NT, GATHER, EDGE, FL>), grid, block, 0, s, g);
  else if (g.opA == OP_C && g.opB == OP_N)
    hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_N, MT, NT, GATHER, EDGE, FL>), grid, block, 0, s, g);
  else if (g.opA == OP_N && g.opB == OP_C)
    hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, GATHER, EDGE, FL>), grid, block, 0, s, g);
  else
    hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_C, MT, NT, GATHER, EDGE, FL>), grid, block, 0, s, g);
}

// Large products with op(A) = A and a general result (no triangular result, no epilogue;
// the propagator has its own kernel) take 128 x 64 tiles held to two waves per SIMD: two
// workgroups share a compute unit, and a triangular op(B) skips K in steps of 64 columns
// instead of 128 (U R^-1 shaped products, 384 x (1024 x 256 x 256): 0.49 -> 0.56 of the FP64
// peak against 4 L N^2; 3 x (25600 x 6400 x 6400): 0.77 -> 0.80).
template <int OPB, bool GATHER, bool EDGE, int FL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void zgemm_wide_kernel(GemmDesc g) {
  zgemm_body<OP_N, OPB, 128, 64, kchunk<128>(), GATHER, EDGE, FL>(g);
}

template <int OPB>
void launch_wide_ops(const GemmDesc &g, hipStream_t s) {
  const dim3 grid(grid_size<128, 64>(g)), block(256);
  const bool edge = needs_edge<128, 64>(g);
  if (g.idxA || g.idxB)
    hipLaunchKernelGGL((zgemm_wide_kernel<OPB, true, true, 0>), grid, block, 0, s, g);
  else if (g.aUpper || g.bUpper || g.aLower) {
    if (edge) hipLaunchKernelGGL((zgemm_wide_kernel<OPB, false, true, FL_MASK>), grid, block, 0, s, g);
    else hipLaunchKernelGGL((zgemm_wide_kernel<OPB, false, false, FL_MASK>), grid, block, 0, s, g);
  } else if (edge) {
    hipLaunchKernelGGL((zgemm_wide_kernel<OPB, false, true, 0>), grid, block, 0, s, g);
  } else {
    hipLaunchKernelGGL((zgemm_wide_kernel<OPB, false, false, 0>), grid, block, 0, s, g);
  }
}

hipError_t launch_wide(const GemmDesc &g, hipStream_t s) {
  if (g.opB == OP_N) launch_wide_ops<OP_N>(g, s);
  else launch_wide_ops<OP_C>(g, s);
  return hipGetLastError();
}

// Results at most 32 columns wide (the panels of the band reduction: m x 32 products and the
// deep 32 x 32 ones split over K) take two-wave tiles of 64 x 32 or 32 x 32: a 64 x 64 tile
// would spend half its matrix-core work on zero columns.
template <int MT, int NT>
hipError_t launch_thin(const GemmDesc &g, hipStream_t s) {
  const dim3 grid(grid_size<MT, NT>(g));
  const bool edge = needs_edge<MT, NT>(g);
  if (g.idxA || g.idxB) {
    launch_ops<MT, NT, true, true>(g, grid, s);
  } else if (g.aUpper || g.bUpper || g.aLower) {
    if (edge) launch_ops<MT, NT, false, true, FL_MASK>(g, grid, s);
    else launch_ops<MT, NT, false, false, FL_MASK>(g, grid, s);
  } else if (edge) {
    launch_ops<MT, NT, false, true>(g, grid, s);
  } else {
    launch_ops<MT, NT, false, false>(g, grid, s);
  }
  return hipGetLastError();
}

template <int MT, int NT>
hipError_t launch(const GemmDesc &g, hipStream_t s) {
  const dim3 grid(grid_size<MT, NT>(g));
  const dim3 block(nthreads<NT>());
  const bool edge = needs_edge<MT, NT>(g);
  if (g.part) {  // reduction epilogues: products U_X U_Y^+ only
    if (g.tri == TRI_LOWER || g.opA != OP_N || g.opB != OP_C || g.R1 || g.aUpper || g.bUpper || g.aLower) return hipErrorInvalidValue;
    if (g.tri == TRI_UPPER) {
      if (g.M != g.N || g.idxA || g.idxB) return hipErrorInvalidValue;
      if (edge) hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, false, true, FL_DIAG>), grid, block, 0, s, g);
      else hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, false, false, FL_DIAG>), grid, block, 0, s, g);
    } else if (g.idxA || g.idxB) {
      hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, true, true, FL_SQSUM>), grid, block, 0, s, g);
    } else if (edge) {
      hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, false, true, FL_SQSUM>), grid, block, 0, s, g);
    } else {
      hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C, MT, NT, false, false, FL_SQSUM>), grid, block, 0, s, g);
    }
    return hipGetLastError();
  }
  if (g.R1) {  // near-identity epilogue: the upper Gram U^+ U of a Cholesky-QR pass
    if (g.opA != OP_C || g.opB != OP_N || g.idxA || g.idxB || g.aUpper || g.bUpper || g.aLower)
      return hipErrorInvalidValue;
    if (edge) hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_N, MT, NT, false, true, FL_NEAR_ID>), grid,
                                 dim3(nthreads<NT>()), 0, s, g);
    else hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_N, MT, NT, false, false, FL_NEAR_ID>), grid,
                            dim3(nthreads<NT>()), 0, s, g);
  } else if (g.idxA || g.idxB) {
    launch_ops<MT, NT, true, true>(g, grid, s);
  } else if (g.aUpper || g.bUpper || g.aLower) {
    if (edge) launch_ops<MT, NT, false, true, FL_MASK>(g, grid, s);
    else launch_ops<MT, NT, false, false, FL_MASK>(g, grid, s);
  } else if (edge) {
    launch_ops<MT, NT, false, true>(g, grid, s);
  } else {
    launch_ops<MT, NT, false, false>(g, grid, s);
  }
  return hipGetLastError();
}

}  // namespace

void set_gemm_tile_mode(int mode) { tl_tile_mode = mode; }
int gemm_tile_mode() { return tl_tile_mode; }
void set_gemm_tile_order(int order) { tl_tile_order = order; }
int gemm_tile_order() { return tl_tile_order; }

hipError_t zgemm_propagator(const GemmDesc &g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return hipSuccess;
  GemmDesc g = g0;
  g.linear_order = tl_tile_order;
  if (tl_tile_mode == GEMM_TILE_SMALL) {
    const dim3 grid(grid_size<64, 64>(g));
    if (needs_edge<64, 64>(g)) hipLaunchKernelGGL(propagator_zgemm_kernel_t64<true>, grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(propagator_zgemm_kernel_t64<false>, grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  const dim3 grid(grid_size<128, 128>(g));
  if (needs_edge<128, 128>(g)) hipLaunchKernelGGL(propagator_zgemm_kernel<true>, grid, dim3(512), 0, s, g);
  else hipLaunchKernelGGL(propagator_zgemm_kernel<false>, grid, dim3(512), 0, s, g);
  return hipGetLastError();
}

// Tile edge the dispatcher uses for g: large tiles only when every dimension fills them
// (and, by default, when there is enough work to occupy the chip with them).
int pick_tile(const GemmDesc &g) {
  if (tl_tile_mode == GEMM_TILE_SMALL) return 64;
  const long work = (long)g.M * g.N * g.batch;
  if (g.M >= 128 && g.N >= 128 && g.K >= (g.short_k_large ? 64 : 128) &&
      (tl_tile_mode == GEMM_TILE_LARGE || work >= (1L << 22)))
    return 128;
  return 64;
}

hipError_t zgemm(const GemmDesc &g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return hipSuccess;
  GemmDesc g = g0;
  g.linear_order = tl_tile_order;
  if (g.N <= 32 && !g.part && !g.R1 && g.tri != TRI_UPPER)  // thin results: no idle tile columns
    return g.M <= 32 ? launch_thin<32, 32>(g, s) : launch_thin<64, 32>(g, s);
  if (pick_tile(g) != 128) return launch<64, 64>(g, s);
  if (g.opA == OP_N && g.tri != TRI_UPPER && !g.part && !g.R1) return launch_wide(g, s);
  return launch<128, 128>(g, s);
}

size_t zgemm_partials(const GemmDesc &g) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return 0;
  const long T = pick_tile(g), tm = (g.M + T - 1) / T, tn = (g.N + T - 1) / T;
  if (g.tri == TRI_UPPER) return (size_t)g.batch * (tm * (tm + 1) / 2) * (2 * T - 1);
  return (size_t)g.batch * tm * tn;
}

namespace {

// C(r) from the diagonal partials (see zgemm_ring_bins): thread per distance r; the upper
// pair (i, j), j - i = e, lies at ring distance min(e, L - e).
__global__ __launch_bounds__(256) void ring_bins_kernel(const double *part, int L, int T, int n_upper,
                                                        double *out) {
  const int b = blockIdx.y, r = 1 + blockIdx.x * 256 + threadIdx.x;
  if (r > L / 2) return;
  const int ND = 2 * T - 1;
  const double *pb = part + (long)b * n_upper * ND;
  const int e1 = r, e2 = L - r;
  double s = 0.0;
  for (int t = 0; t < n_upper; ++t) {
    int tm, tn;
    upper_tile(t, tm, tn);
    const int delta = (tn - tm) * T;
    int o = e1 - delta + (T - 1);
    if (o >= 0 && o < ND) s += pb[(long)t * ND + o];
    if (e2 != e1) {
      o = e2 - delta + (T - 1);
      if (o >= 0 && o < ND) s += pb[(long)t * ND + o];
    }
  }
  // ordered pairs at distance r: 2L (r < L/2) or L (r = L/2); s counts each once
  out[(long)b * (L / 2) + r - 1] = 2 * r == L ? -2.0 * s / L : -s / L;
}

__global__ __launch_bounds__(64) void tile_sum_kernel(const double *part, long n_tiles, double *out) {
  const int b = blockIdx.x;
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (long t = 0; t < n_tiles; ++t) s += part[(long)b * n_tiles + t];
  out[b] = s;
}

}  // namespace

hipError_t zgemm_ring_bins(const GemmDesc &g, int L, double *out, hipStream_t s) {
  if (!g.part || g.tri != TRI_UPPER || g.M != L || g.N != L) return hipErrorInvalidValue;
  hipError_t e = zgemm(g, s);
  if (e != hipSuccess) return e;
  const int T = pick_tile(g), tiles = (L + T - 1) / T;
  hipLaunchKernelGGL(ring_bins_kernel, dim3((L / 2 + 255) / 256, g.batch), dim3(256), 0, s, g.part, L, T,
                     tiles * (tiles + 1) / 2, out);
  return hipGetLastError();
}

hipError_t zgemm_tile_sum(const GemmDesc &g, double *out, hipStream_t s) {
  if (!g.part || g.tri != TRI_NONE) return hipErrorInvalidValue;
  hipError_t e = zgemm(g, s);
  if (e != hipSuccess) return e;
  const long T = pick_tile(g), n_tiles = ((g.M + T - 1) / T) * ((g.N + T - 1) / T);
  hipLaunchKernelGGL(tile_sum_kernel, dim3(g.batch), dim3(64), 0, s, g.part, n_tiles, out);
  return hipGetLastError();
}

}  // namespace mfq
