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
// Tiling: a 256-thread workgroup (4 wave64) owns a 64 x 64 complex tile of D;
// each wave owns a 32 x 32 quadrant = 2 x 2 MFMA blocks, with separate real and
// imaginary accumulators (8 x 4 doubles per lane).  K advances in chunks of 16
// through double-buffered LDS (64 KiB); the next chunk is fetched into
// registers while the current one feeds the matrix cores.
//
// MFMA lane layout (gfx950, checked on hardware): operand A lane l holds
// A[l % 16][l / 16], operand B holds B[l / 16][l % 16]; output register r of
// lane l is D[l / 16 + 4 r][l % 16].
#include "mfq_internal.h"

namespace mfq {

typedef double d4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int MT = 64, NT = 64, KT = 16, PAD = 1;

template <int OPA, int OPB>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmDesc g) {
  const int tm = blockIdx.x, tn = blockIdx.y, b = blockIdx.z;
  const int m0 = tm * MT, n0 = tn * NT;
  if (g.tri == TRI_UPPER && m0 > n0 + NT - 1) return;  // tile entirely below the diagonal
  int kbeg = 0, kend = g.K;
  if (g.aUpper) kbeg = (m0 / KT) * KT;
  if (g.bUpper) kend = min(g.K, n0 + NT);

  __shared__ double Ar[2][KT][MT + PAD], Ai[2][KT][MT + PAD];
  __shared__ double Br[2][KT][NT + PAD], Bi[2][KT][NT + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const cplx *A = g.A + (long)b * g.sA;
  const cplx *B = g.B + (long)b * g.sB;

  double ra_re[4], ra_im[4], rb_re[4], rb_im[4];

  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      if (OPA == OP_N) { m = tid & 63; k = (tid >> 6) + 4 * i; }
      else { k = tid & 15; m = (tid >> 4) + 16 * i; }
      const int gm = m0 + m, gk = k0 + k;
      double re = 0.0, im = 0.0;
      if (gm < g.M && gk < kend) {
        if (OPA == OP_N) {
          const long row = g.idxA ? g.idxA[gm] : gm;
          const cplx v = A[row + (long)gk * g.lda];
          re = v.re; im = v.im;
        } else {
          const long row = g.idxA ? g.idxA[gk] : gk;
          const cplx v = A[row + (long)gm * g.lda];
          re = v.re; im = -v.im;
        }
      }
      ra_re[i] = re; ra_im[i] = im;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int n, k;
      if (OPB == OP_N) { k = tid & 15; n = (tid >> 4) + 16 * i; }
      else { n = tid & 63; k = (tid >> 6) + 4 * i; }
      const int gn = n0 + n, gk = k0 + k;
      double re = 0.0, im = 0.0;
      if (gn < g.N && gk < kend) {
        if (OPB == OP_N) {
          const long row = g.idxB ? g.idxB[gk] : gk;
          const cplx v = B[row + (long)gn * g.ldb];
          re = v.re; im = v.im;
        } else {
          const long row = g.idxB ? g.idxB[gn] : gn;
          const cplx v = B[row + (long)gk * g.ldb];
          re = v.re; im = -v.im;
        }
      }
      rb_re[i] = re; rb_im[i] = im;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int m, k;
      if (OPA == OP_N) { m = tid & 63; k = (tid >> 6) + 4 * i; }
      else { k = tid & 15; m = (tid >> 4) + 16 * i; }
      Ar[buf][k][m] = ra_re[i];
      Ai[buf][k][m] = ra_im[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int n, k;
      if (OPB == OP_N) { k = tid & 15; n = (tid >> 4) + 16 * i; }
      else { n = tid & 63; k = (tid >> 6) + 4 * i; }
      Br[buf][k][n] = rb_re[i];
      Bi[buf][k][n] = rb_im[i];
    }
  };

  d4 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
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
    const int buf = it & 1;
    if (it + 1 < nk) load(kbeg + (it + 1) * KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int k = kk + (lane >> 4);
      double a_re[2], a_im[2], a_nim[2], b_re[2], b_im[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int row = wr * 32 + i * 16 + (lane & 15);
        a_re[i] = Ar[buf][k][row];
        a_im[i] = Ai[buf][k][row];
        a_nim[i] = -a_im[i];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = wc * 32 + j * 16 + (lane & 15);
        b_re[j] = Br[buf][k][col];
        b_im[j] = Bi[buf][k][col];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_re[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_re[i], b_im[j], acc_im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_nim[i], b_im[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_im[i], b_re[j], acc_im[i][j], 0, 0, 0);
        }
    }
    if (it + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // epilogue: D = alpha * acc + beta * Cin
  const bool useC = (g.beta.re != 0.0 || g.beta.im != 0.0);
  const cplx *Cin = g.Cin ? g.Cin + (long)b * g.sCin : nullptr;
  cplx *D = g.D + (long)b * g.sD;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int col = n0 + wc * 32 + j * 16 + (lane & 15);
        if (row >= g.M || col >= g.N) continue;
        if (g.tri == TRI_UPPER && row > col) continue;
        const double xr = acc_re[i][j][r], xi = acc_im[i][j][r];
        double yr = g.alpha.re * xr - g.alpha.im * xi;
        double yi = g.alpha.re * xi + g.alpha.im * xr;
        if (useC) {
          const cplx c = Cin[row + (long)col * g.ldcin];
          yr += g.beta.re * c.re - g.beta.im * c.im;
          yi += g.beta.re * c.im + g.beta.im * c.re;
        }
        D[row + (long)col * g.ldd] = cplx{yr, yi};
      }
}

}  // namespace

hipError_t zgemm(const GemmDesc &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  dim3 grid((g.M + MT - 1) / MT, (g.N + NT - 1) / NT, g.batch);
  dim3 block(256);
  if (g.opA == OP_N && g.opB == OP_N) hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_N>), grid, block, 0, s, g);
  else if (g.opA == OP_C && g.opB == OP_N) hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_N>), grid, block, 0, s, g);
  else if (g.opA == OP_N && g.opB == OP_C) hipLaunchKernelGGL((zgemm_kernel<OP_N, OP_C>), grid, block, 0, s, g);
  else hipLaunchKernelGGL((zgemm_kernel<OP_C, OP_C>), grid, block, 0, s, g);
  return hipGetLastError();
}

}  // namespace mfq
