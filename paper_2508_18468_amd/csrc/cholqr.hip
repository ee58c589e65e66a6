// Cholesky-QR re-orthonormalisation: U <- U R^{-1}, R^+ R = U^+ U.
//
// The paper keeps U^+ U = 1 by a QR decomposition after every step
// (Appendix A).  Here one pass is: Gram G = U^+ U on the matrix cores (upper
// triangle only), blocked Cholesky G = R^+ R (upper R, block 64: the diagonal
// block factorised and inverted in LDS, the block row solved and the later rows
// updated by the batched GEMM, right-looking inside panels of 512 rows and one
// rank-512 update of the rest per panel), the triangular
// inverse R^{-1} assembled block column by block column from GEMMs, and the
// triangular product U R^{-1} (zero blocks of R^{-1} skipped).  Two passes
// (Cholesky-QR2) bring U^+ U to identity at working precision for the
// condition numbers a step produces; the second pass keeps the first pass's
// result in place when its Gram certifies |U^+ U - I| <= CHOL_KEEP_MAX entrywise,
// so that, as in every step of the workloads here, it costs one Gram and no copy.
#include "mfq_internal.h"
#include "potrf_block.h"

namespace mfq {

namespace {

constexpr int NB = CHOL_NB;
static_assert(PB == NB, "one diagonal block size");

// Factorise the w x w diagonal block at (c0, c0) of G[b] (upper triangle),
// write R_JJ back into G and R_JJ^{-1} (full block, zeros below the diagonal)
// into Rinv[b], by the phases of potrf_block.h separated by barriers.  A
// non-positive or non-finite pivot raises *flag, and the first such pivot of a
// call sequence is recorded in *info (source: 1 or 2 for the pass, the
// trajectory, its column and its value).  The block and its inverse share one
// LDS array, so that two workgroups fit on a compute unit.
__global__ __launch_bounds__(PB_THREADS) void potrf_diag_kernel(cplx *G, cplx *Rinv, int N, int c0, int w,
                                                                int *flag, BreakdownInfo *info, int source,
                                                                const double *skip_if_le, double skip_thr) {
  if (skip_if_le && *skip_if_le <= skip_thr) return;
  const int b = blockIdx.x, tid = threadIdx.x;
  cplx *Gb = G + (long)b * N * N;
  cplx *Rb = Rinv + (long)b * N * N;
  __shared__ PotrfLds s;
  __shared__ int first_bad;  // smallest column of a bad pivot (w: none)
  if (tid == 0) first_bad = w;
  potrf_load(s, Gb, N, c0, w, tid);
  __syncthreads();
  for (int k = 0; k + 1 < w; ++k) {
    potrf_eliminate(s, k, w, tid);
    __syncthreads();
  }
  if (tid < w && potrf_pivot(s, tid)) atomicMin(&first_bad, tid);
  __syncthreads();
  potrf_scale(s, w, tid);
  __syncthreads();
  // column j of the inverse by lanes 4j .. 4j+3 of one wave
  const int j = tid >> 2, q = tid & 3;
  if (j < w) {
    const double dj = 1.0 / s.a[j][j].re;
    if (q == 0) s.xd[j] = dj;
    for (int i = j - 1; i >= 0; --i) {
      double sr, si;
      potrf_inv_partial(s, i, j, q, dj, sr, si);
      sr += __shfl_xor(sr, 1, 64);
      si += __shfl_xor(si, 1, 64);
      sr += __shfl_xor(sr, 2, 64);
      si += __shfl_xor(si, 2, 64);
      potrf_inv_store(s, i, j, sr, si);  // the four lanes store the same value
    }
  }
  __syncthreads();
  potrf_store(s, Gb, Rb, N, c0, w, tid);
  if (tid == 0 && first_bad < w) {
    atomicOr(flag, 1);
    if (atomicCAS(&info->set, 0, 1) == 0) {
      info->source = source;
      info->traj = b;
      info->col = c0 + first_bad;
      info->pivot = s.piv[first_bad];
    }
  }
}

// Pass 2 did not certify its input (max |G - I| above thr or not finite): its product,
// formed in src, becomes the result in dst.  Otherwise every workgroup exits at once.
__global__ __launch_bounds__(256) void keep_or_copy_kernel(const double2 *src, double2 *dst, long n,
                                                           const double *dev, double thr) {
  if (*dev <= thr) return;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) dst[i] = src[i];
}

GemmDesc desc() {
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.beta = cplx{0.0, 0.0};
  return g;
}

// One pass: Uout = Uin R^{-1}.  near_identity (pass 2): Uout is not written when the Gram
// certifies Uin (max |G - I| <= CHOL_KEEP_MAX, left in wk.dev).  Otherwise Uin may be
// overwritten (pass 1 solves its right block in place).
hipError_t cholqr_pass(cplx *Uin, cplx *Uout, int L, int N, int B, const CholWork &wk,
                       bool near_identity, hipStream_t s) {
  hipError_t e;
  const long NN = (long)N * N;
  // full-factorisation launches are skipped on the device when the near-identity
  // test passed (max |E| <= threshold)
  const double *skip = near_identity ? wk.dev : nullptr;
  const double thr = CHOL_FIRST_ORDER_MAX;
  // G = Uin^+ Uin (upper triangle); with near_identity the Gram's epilogue also
  // writes the first-order factor into Rinv and the largest |G - I| into wk.dev
  if (near_identity && (e = fill_zero(wk.dev, sizeof(double), s)) != hipSuccess) return e;
  {
    GemmDesc g = desc();
    g.M = N; g.N = N; g.K = L; g.batch = B;
    g.A = Uin; g.lda = L; g.sA = (long)L * N; g.opA = OP_C;
    g.B = Uin; g.ldb = L; g.sB = (long)L * N; g.opB = OP_N;
    g.D = wk.G; g.ldd = N; g.sD = NN;
    g.tri = TRI_UPPER;
    if (near_identity) {
      g.R1 = wk.Rinv;
      g.maxdev = wk.dev;
    }
    if ((e = zgemm(g, s)) != hipSuccess) return e;
  }
  // Two levels: outer panels of CHOL_OUTER rows of R.  Inside a panel, block J (NB rows) is
  // factorised, its block row solved to the end of the matrix, and only the panel's later block
  // rows updated (K = NB); the rows below the panel get one update per panel (K = CHOL_OUTER),
  // which has CHOL_OUTER / NB times the flops per byte of a per-block trailing update.
  for (int p0 = 0; p0 < N; p0 += CHOL_OUTER) {
    const int p1 = std::min(N, p0 + CHOL_OUTER);
    for (int c0 = p0; c0 < p1; c0 += NB) {
      const int w = std::min(NB, p1 - c0);
      hipLaunchKernelGGL(potrf_diag_kernel, dim3(B), dim3(256), 0, s, wk.G, wk.Rinv, N, c0, w, wk.flag,
                         wk.info, near_identity ? 2 : 1, skip, thr);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      const int r0 = c0 + w, nr = N - r0;
      if (nr <= 0) break;
      // block row: R_J,rest = R_JJ^{-+} G_J,rest (in place; one row tile, so every
      // workgroup reads its whole column panel before writing it)
      {
        GemmDesc g = desc();
        g.skip_if_le = skip; g.skip_thr = thr;
        g.M = w; g.N = nr; g.K = w; g.batch = B;
        g.A = wk.Rinv + c0 + (long)c0 * N; g.lda = N; g.sA = NN; g.opA = OP_C;
        g.B = wk.G + c0 + (long)r0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
        g.D = wk.G + c0 + (long)r0 * N; g.ldd = N; g.sD = NN;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
      // the panel's later block rows: G_r0..p1, r0.. -= R_J,r0..p1^+ R_J,r0.. (upper part)
      if (r0 < p1) {
        GemmDesc g = desc();
        g.skip_if_le = skip; g.skip_thr = thr;
        g.M = p1 - r0; g.N = nr; g.K = w; g.batch = B;
        g.A = wk.G + c0 + (long)r0 * N; g.lda = N; g.sA = NN; g.opA = OP_C;
        g.B = wk.G + c0 + (long)r0 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
        g.Cin = wk.G + r0 + (long)r0 * N; g.ldcin = N; g.sCin = NN;
        g.D = wk.G + r0 + (long)r0 * N; g.ldd = N; g.sD = NN;
        g.alpha = cplx{-1.0, 0.0};
        g.beta = cplx{1.0, 0.0};
        g.tri = TRI_UPPER;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
    }
    // below the panel: G_p1..,p1.. -= R_P,p1..^+ R_P,p1.. (upper)
    const int nr = N - p1;
    if (nr > 0) {
      GemmDesc g = desc();
      g.skip_if_le = skip; g.skip_thr = thr;
      g.M = nr; g.N = nr; g.K = p1 - p0; g.batch = B;
      g.A = wk.G + p0 + (long)p1 * N; g.lda = N; g.sA = NN; g.opA = OP_C;
      g.B = wk.G + p0 + (long)p1 * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
      g.Cin = wk.G + p1 + (long)p1 * N; g.ldcin = N; g.sCin = NN;
      g.D = wk.G + p1 + (long)p1 * N; g.ldd = N; g.sD = NN;
      g.alpha = cplx{-1.0, 0.0};
      g.beta = cplx{1.0, 0.0};
      g.tri = TRI_UPPER;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
  }
  // R^{-1} from the inverted diagonal blocks, level by level: adjacent aligned diagonal
  // blocks [R11 R12; 0 R22] of size S (S = NB, 2 NB, ...) have the inverse
  // [R11^{-1}, -R11^{-1} R12 R22^{-1}; 0, R22^{-1}], so one level is two batched products
  // over all its block pairs and all trajectories (T = R11^{-1} R12, then -T R22^{-1}); the
  // last pair of a level may have a narrower right block.  T lives in Uout, which is free
  // until the final product (at most N^2 / 2 <= L N entries per trajectory).
  // Pass 1 stops below the top level: with R = [R11 R12; 0 R22] split at S_top (the largest
  // level, S_top < N <= 2 S_top), Q = U R^{-1} is Q1 = U1 R11^{-1}, then U2 -= Q1 R12 in place and
  // Q2 = U2 R22^{-1}: the same flops as U R^{-1} without forming -R11^{-1} R12 R22^{-1}.
  const bool split = !near_identity && N > NB;
  long S_top = NB;
  while (2 * S_top < N) S_top *= 2;
  for (long S = NB; S < N; S *= 2) {
    if (split && S == S_top) break;
    const int full = (int)(N / (2 * S));                        // pairs with a complete right block
    const int w2 = (int)(N - (long)full * 2 * S - S);           // right width of a last, narrower pair
    for (int part = 0; part < 2; ++part) {
      const int npairs = part == 0 ? full : (w2 > 0 ? 1 : 0);
      if (npairs == 0) continue;
      const long r0 = part == 0 ? 0 : (long)full * 2 * S;       // first pair's left block
      const int wR = part == 0 ? (int)S : w2;                   // right block width
      cplx *T = Uout + (part == 0 ? 0 : (long)full * S * S);
      const long step = 2 * S * ((long)N + 1);                  // between pairs along the diagonal
      {  // T = R11^{-1} R12
        GemmDesc g = desc();
        g.skip_if_le = skip; g.skip_thr = thr;
        g.M = (int)S; g.N = wR; g.K = (int)S; g.batch = B * npairs; g.batch2 = npairs;
        g.A = wk.Rinv + r0 * ((long)N + 1); g.lda = N; g.sA = NN; g.sA2 = step; g.opA = OP_N; g.aUpper = 1;
        g.B = wk.G + r0 + (r0 + S) * N; g.ldb = N; g.sB = NN; g.sB2 = step; g.opB = OP_N;
        g.D = T; g.ldd = S; g.sD = (long)L * N; g.sD2 = S * S;
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
      {  // (R^{-1})_12 = -T R22^{-1}
        GemmDesc g = desc();
        g.skip_if_le = skip; g.skip_thr = thr;
        g.M = (int)S; g.N = wR; g.K = wR; g.batch = B * npairs; g.batch2 = npairs;
        g.A = T; g.lda = S; g.sA = (long)L * N; g.sA2 = S * S; g.opA = OP_N;
        g.B = wk.Rinv + (r0 + S) * ((long)N + 1); g.ldb = N; g.sB = NN; g.sB2 = step; g.opB = OP_N;
        g.bUpper = 1;
        g.D = wk.Rinv + r0 + (r0 + S) * N; g.ldd = N; g.sD = NN; g.sD2 = step;
        g.alpha = cplx{-1.0, 0.0};
        if ((e = zgemm(g, s)) != hipSuccess) return e;
      }
    }
  }
  if (split) {
    const int w1 = (int)S_top, w2 = N - (int)S_top;
    {  // Q1 = U1 R11^{-1}
      GemmDesc g = desc();
      g.M = L; g.N = w1; g.K = w1; g.batch = B;
      g.A = Uin; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
      g.B = wk.Rinv; g.ldb = N; g.sB = NN; g.opB = OP_N; g.bUpper = 1;
      g.D = Uout; g.ldd = L; g.sD = (long)L * N;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    {  // U2 -= Q1 R12 (each entry reads only itself from U2)
      GemmDesc g = desc();
      g.M = L; g.N = w2; g.K = w1; g.batch = B;
      g.A = Uout; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
      g.B = wk.G + S_top * N; g.ldb = N; g.sB = NN; g.opB = OP_N;
      g.Cin = Uin + S_top * L; g.ldcin = L; g.sCin = (long)L * N;
      g.D = Uin + S_top * L; g.ldd = L; g.sD = (long)L * N;
      g.alpha = cplx{-1.0, 0.0};
      g.beta = cplx{1.0, 0.0};
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    {  // Q2 = U2 R22^{-1}
      GemmDesc g = desc();
      g.M = L; g.N = w2; g.K = w2; g.batch = B;
      g.A = Uin + S_top * L; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
      g.B = wk.Rinv + S_top * ((long)N + 1); g.ldb = N; g.sB = NN; g.opB = OP_N; g.bUpper = 1;
      g.D = Uout + S_top * L; g.ldd = L; g.sD = (long)L * N;
      if ((e = zgemm(g, s)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  // Uout = Uin R^{-1}; in the second pass skipped on the device when Uin is already
  // orthonormal to CHOL_KEEP_MAX
  {
    GemmDesc g = desc();
    g.M = L; g.N = N; g.K = N; g.batch = B;
    g.A = Uin; g.lda = L; g.sA = (long)L * N; g.opA = OP_N;
    g.B = wk.Rinv; g.ldb = N; g.sB = NN; g.opB = OP_N; g.bUpper = 1;
    g.D = Uout; g.ldd = L; g.sD = (long)L * N;
    if (near_identity) {
      g.skip_if_le = wk.dev;
      g.skip_thr = CHOL_KEEP_MAX;
    }
    if ((e = zgemm(g, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t cholqr2(cplx *U, cplx *T, int L, int N, int B, const CholWork &wk, hipStream_t s) {
  if (U == T) return hipErrorInvalidValue;
  hipError_t e = cholqr_pass(U, T, L, N, B, wk, false, s);
  if (e != hipSuccess) return e;
  if ((e = cholqr_pass(T, U, L, N, B, wk, true, s)) != hipSuccess) return e;
  const long n = (long)L * N * B;
  const unsigned blocks = (unsigned)std::min<long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(keep_or_copy_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const double2 *>(U),
                     reinterpret_cast<double2 *>(T), n, (const double *)wk.dev, CHOL_KEEP_MAX);
  return hipGetLastError();
}

}  // namespace mfq
