// FP32-bulk propagator: U' = U + (P - I) U with the product on the FP32 matrix
// cores (v_mfma_f32_16x16x4f32, twice the FP64 matrix rate) and the sum in FP64.
//
// Writing the step as the identity plus a small correction ("delta form")
// keeps the FP32 rounding on the correction only: |P - I| ~ 2J dt, so the
// per-step error is ~2J dt times that of a plain FP32 product.  P - I is kept
// as two FP32 planes (real, imaginary); U is read in FP64, rounded to FP32 on
// its way into LDS, and read again in FP64 for the exact identity term.
//
// Tiling as the FP64 kernel: 128 x 128 complex tile per 512-thread workgroup,
// 8 wave64 in a 2 x 4 grid, 64 x 32 outputs per wave as 4 x 2 MFMA blocks with
// separate real / imaginary FP32 accumulators, K chunks of 16 through
// double-buffered LDS, XCD-aware ordering of the column panels.
//
// FP32 MFMA lane layout (gfx950, checked on hardware): operand A lane l holds
// A[l % 16][l / 16], operand B holds B[l / 16][l % 16]; output register r of
// lane l is D[4 (l / 16) + r][l % 16].
#include "mfq_internal.h"

namespace mfq {

typedef float f4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int MT = 128, NT = 128, KT = 16, WM = 2, WN = 4, NTHR = 512, PAD = 1, NXCD = 8;
constexpr int IM = MT / WM / 16, JN = NT / WN / 16;
#ifndef F32_MIN_WAVES
#define F32_MIN_WAVES 4  // waves per SIMD: two workgroups per CU
#endif
constexpr int LA = MT * KT / NTHR, LB = NT * KT / NTHR;

__global__ void delta_planes_kernel(const cplx *P, float *Pr, float *Pi, long L) {
  const long total = L * L;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long r = idx % L, c = idx / L;
    const cplx p = P[idx];
    Pr[idx] = (float)(r == c ? p.re - 1.0 : p.re);
    Pi[idx] = (float)p.im;
  }
}

template <bool EDGE>
__global__ __launch_bounds__(NTHR, F32_MIN_WAVES) void propagator_delta_f32_kernel(const float *Pr, const float *Pi,
                                                                    const cplx *U, cplx *D, int L,
                                                                    int ncols) {
  const int tilesM = (L + MT - 1) / MT, tilesN = (ncols + NT - 1) / NT;
  const int id = blockIdx.x;
  const bool linear = tilesN < NXCD;
  const int k_on_xcd = linear ? id : id / NXCD;
  const int tn = linear ? id / tilesM : id % NXCD + NXCD * (k_on_xcd / tilesM);
  const int tm = k_on_xcd % tilesM;
  if (tn >= tilesN) return;
  const int m0 = tm * MT, n0 = tn * NT;

  __shared__ float Ar[2][KT][MT + PAD], Ai[2][KT][MT + PAD];
  __shared__ float Br[2][KT][NT + PAD], Bi[2][KT][NT + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave % WM, wc = wave / WM;
  // A = P - I (column-major planes): contiguous in m
  const int a_m = tid % MT, a_k = tid / MT;          // k = a_k + (NTHR / MT) * i
  // B = U (column-major, FP64 complex): contiguous in k
  const int b_k = tid % KT, b_n = tid / KT;          // n = b_n + (NTHR / KT) * i

  float ra_re[LA], ra_im[LA], rb_re[LB], rb_im[LB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int gm = m0 + a_m, gk = k0 + a_k + (NTHR / MT) * i;
      float re = 0.f, im = 0.f;
      if (!EDGE || (gm < L && gk < L)) {
        re = Pr[gm + (long)gk * L];
        im = Pi[gm + (long)gk * L];
      }
      ra_re[i] = re; ra_im[i] = im;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int gk = k0 + b_k, gn = n0 + b_n + (NTHR / KT) * i;
      float re = 0.f, im = 0.f;
      if (!EDGE || (gk < L && gn < ncols)) {
        const cplx v = U[gk + (long)gn * L];
        re = (float)v.re; im = (float)v.im;
      }
      rb_re[i] = re; rb_im[i] = im;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int k = a_k + (NTHR / MT) * i;
      Ar[buf][k][a_m] = ra_re[i];
      Ai[buf][k][a_m] = ra_im[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int n = b_n + (NTHR / KT) * i;
      Br[buf][b_k][n] = rb_re[i];
      Bi[buf][b_k][n] = rb_im[i];
    }
  };

  f4 acc_re[IM][JN], acc_im[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      acc_re[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc_im[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  const int nk = (L + KT - 1) / KT;
  load(0);
  store(0);
  __syncthreads();
  for (int it = 0; it < nk; ++it) {
    const int buf = it & 1;
    if (it + 1 < nk) load((it + 1) * KT);
#pragma unroll
    for (int kk = 0; kk < KT; kk += 4) {
      const int k = kk + (lane >> 4);
      float a_re[IM], a_im[IM], b_re[JN], b_im[JN];
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
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re[i], b_re[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_re[i], b_im[j], acc_im[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < IM; ++i) {
        const float a_nim = -a_im[i];
#pragma unroll
        for (int j = 0; j < JN; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_nim, b_im[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_im[i], b_re[j], acc_im[i][j], 0, 0, 0);
        }
      }
    }
    if (it + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // D = U + acc  (identity term exact in FP64)
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * (MT / WM) + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wc * (NT / WN) + j * 16 + (lane & 15);
        if (EDGE && (row >= L || col >= ncols)) continue;
        const long idx = row + (long)col * L;
        const cplx u = U[idx];
        D[idx] = cplx{u.re + (double)acc_re[i][j][r], u.im + (double)acc_im[i][j][r]};
      }
}

}  // namespace

hipError_t make_delta_planes(const cplx *P, float *Pr, float *Pi, int L, hipStream_t s) {
  const long total = (long)L * L;
  const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(delta_planes_kernel, dim3(blocks), dim3(256), 0, s, P, Pr, Pi, (long)L);
  return hipGetLastError();
}

hipError_t propagator_delta_f32(const float *Pr, const float *Pi, const cplx *U, cplx *D, int L,
                                int ncols, hipStream_t s) {
  if (L <= 0 || ncols <= 0) return hipSuccess;
  const int tilesM = (L + MT - 1) / MT, tilesN = (ncols + NT - 1) / NT;
  const bool linear = tilesN < NXCD;
  const long grid = linear ? (long)tilesM * tilesN : (long)((tilesN + NXCD - 1) / NXCD) * NXCD * tilesM;
  const bool edge = (L % MT) || (ncols % NT) || (L % KT);
  if (edge)
    hipLaunchKernelGGL(propagator_delta_f32_kernel<true>, dim3((unsigned)grid), dim3(NTHR), 0, s, Pr, Pi,
                       U, D, L, ncols);
  else
    hipLaunchKernelGGL(propagator_delta_f32_kernel<false>, dim3((unsigned)grid), dim3(NTHR), 0, s, Pr, Pi,
                       U, D, L, ncols);
  return hipGetLastError();
}

}  // namespace mfq
