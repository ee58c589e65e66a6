// State kernels: initial state, propagator expansion, Born probabilities with
// the fused homodyne update, and the projective measurement.
//
// Layout: U of trajectory b is column-major L x N (ld = L) at U + b*L*N.  A
// thread owns rows, so every load/store of a column is coalesced across the
// wave (64 consecutive rows = 1 KiB per column).
#include "mfq_internal.h"
#include "device_common.h"

namespace mfq {

namespace {

__global__ void fill_zero_kernel(uint64_t *p, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = 0ull;
}

// P_ab = g[(a - b) mod L] (1d ring, circulant); on the torus P = P_y (x) P_x,
// P_(xa,ya),(xb,yb) = gx[(xa - xb) mod Lx] * gy[(ya - yb) mod Ly].
__global__ void expand_propagator_kernel(cplx *P, const cplx *gx, const cplx *gy, int dim, int Lx,
                                         int Ly, long L) {
  const long total = L * L;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long a = idx % L, b = idx / L;
    if (dim == 1) {
      P[idx] = gx[((a - b) % L + L) % L];
    } else {
      const int xa = (int)(a % Lx), ya = (int)(a / Lx), xb = (int)(b % Lx), yb = (int)(b / Lx);
      const cplx u = gx[((xa - xb) % Lx + Lx) % Lx], v = gy[((ya - yb) % Ly + Ly) % Ly];
      P[idx] = cplx{u.re * v.re - u.im * v.im, u.re * v.im + u.im * v.re};
    }
  }
}

// U[:, k] = e_{occ[k]} for every trajectory.
__global__ void init_state_kernel(cplx *U, int L, int N, long total, const int *occ) {
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const long within = idx % ((long)L * N);
    const int i = (int)(within % L), k = (int)(within / L);
    U[idx] = cplx{occ[k] == i ? 1.0 : 0.0, 0.0};
  }
}

// p_i = sum_k |U_ik|^2; homodyne: U_i. *= exp(xi_i + gamma (2 p_i - 1) dt),
// xi_i = sqrt(gamma dt) z_i, z_i = Box-Muller normal from Philox (purpose 1).
template <bool HOMODYNE>
__global__ __launch_bounds__(256) void born_kernel(cplx *U, double *p, int L, int N,
                                                   const double *gamma, double dt, uint64_t seed,
                                                   const uint64_t *uid, const int64_t *step_ptr,
                                                   int step_offset, const int64_t *step_base) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  cplx *Ub = U + (long)b * L * N;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 4 <= N; k += 4) {
    const cplx a0 = Ub[i + (long)k * L], a1 = Ub[i + (long)(k + 1) * L];
    const cplx a2 = Ub[i + (long)(k + 2) * L], a3 = Ub[i + (long)(k + 3) * L];
    s0 += a0.re * a0.re + a0.im * a0.im;
    s1 += a1.re * a1.re + a1.im * a1.im;
    s2 += a2.re * a2.re + a2.im * a2.im;
    s3 += a3.re * a3.re + a3.im * a3.im;
  }
  for (; k < N; ++k) {
    const cplx a = Ub[i + (long)k * L];
    s0 += a.re * a.re + a.im * a.im;
  }
  const double pi = (s0 + s1) + (s2 + s3);
  p[(long)b * L + i] = pi;
  if (!HOMODYNE) return;
  const double g = gamma[b];
  const uint64_t step = (uint64_t)(*step_ptr + step_offset - step_base[b]);
  const u64x4 w = philox4x64_10(seed, uid[b], step, (uint64_t)i, PURPOSE_HOMODYNE, 0);
  const double z = sqrt(-2.0 * log(u01(w.v[0]))) * cos(6.283185307179586 * u01(w.v[1]));
  const double f = exp(sqrt(g * dt) * z + g * (2.0 * pi - 1.0) * dt);
  for (k = 0; k < N; ++k) {
    cplx a = Ub[i + (long)k * L];
    a.re *= f;
    a.im *= f;
    Ub[i + (long)k * L] = a;
  }
}

// Same operation with the rows held in registers between the reduction and
// the scaling, so U is read once and written once: a workgroup owns 16
// consecutive rows of one trajectory; thread t holds row t % 16 at columns
// t / 16 + 16 v (v < VPT, N <= 16 VPT).  The 16 partial sums of a row are
// combined in a fixed order (wave shuffles, then the four waves in LDS).
template <bool HOMODYNE, int VPT>
__global__ __launch_bounds__(256) void born_rows_kernel(cplx *U, double *p, int L, int N,
                                                        const double *gamma, double dt, uint64_t seed,
                                                        const uint64_t *uid, const int64_t *step_ptr,
                                                        int step_offset, const int64_t *step_base) {
  const int b = blockIdx.y, tid = threadIdx.x;
  const int r = tid & 15, c0 = tid >> 4;
  const int i = blockIdx.x * 16 + r;
  const bool row_ok = i < L;
  cplx *Ub = U + (long)b * L * N;
  cplx a[VPT];
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    const int k = c0 + 16 * v;
    a[v] = (row_ok && k < N) ? Ub[i + (long)k * L] : cplx{0.0, 0.0};
    s += a[v].re * a[v].re + a[v].im * a[v].im;
  }
  // lanes r, r+16, r+32, r+48 of a wave hold the same row
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  __shared__ double part[4][16];
  if ((tid & 63) < 16) part[tid >> 6][r] = s;
  __syncthreads();
  const double pi = (part[0][r] + part[1][r]) + (part[2][r] + part[3][r]);
  if (c0 == 0 && row_ok) p[(long)b * L + i] = pi;
  if (!HOMODYNE || !row_ok) return;
  const double g = gamma[b];
  const uint64_t step = (uint64_t)(*step_ptr + step_offset - step_base[b]);
  const u64x4 w = philox4x64_10(seed, uid[b], step, (uint64_t)i, PURPOSE_HOMODYNE, 0);
  const double z = sqrt(-2.0 * log(u01(w.v[0]))) * cos(6.283185307179586 * u01(w.v[1]));
  const double f = exp(sqrt(g * dt) * z + g * (2.0 * pi - 1.0) * dt);
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    const int k = c0 + 16 * v;
    if (k < N) Ub[i + (long)k * L] = cplx{a[v].re * f, a[v].im * f};
  }
}

// Banded ring propagator: D[a, c] = sum_{|d| <= w} g[d mod L] U[(a - d) mod L, c], the
// circulant exp(-i Ht dt) with the generating-row entries beyond distance w dropped (the
// caller picks w so that they are below the rounding of the kept ones).  One workgroup per
// (256-row block, column): the rows it needs, with a halo of w on each side, go through LDS.
constexpr int STENCIL_WMAX = 128;
__global__ __launch_bounds__(256) void ring_stencil_kernel(const cplx *U, cplx *D, const cplx *g, int L,
                                                           int w, int nrb) {
  __shared__ cplx s[256 + 2 * STENCIL_WMAX];
  const long id = blockIdx.x;
  const int rb = (int)(id % nrb);
  const long c = id / nrb;
  const int r0 = rb * 256;
  const cplx *Uc = U + c * L;
  for (int t = threadIdx.x; t < 256 + 2 * w; t += 256) {
    int r = (r0 - w + t) % L;
    if (r < 0) r += L;
    s[t] = Uc[r];
  }
  __syncthreads();
  const int i = r0 + threadIdx.x;
  if (i >= L) return;
  double ar = 0.0, ai = 0.0;
  for (int d = -w; d <= w; ++d) {
    const cplx gd = g[d < 0 ? d + L : d], u = s[threadIdx.x + w - d];
    ar += gd.re * u.re - gd.im * u.im;
    ai += gd.re * u.im + gd.im * u.re;
  }
  D[c * L + i] = cplx{ar, ai};
}

// Projective measurement of one step, one trajectory per workgroup (see
// pm_measure_block).
__global__ __launch_bounds__(256) void pm_kernel(cplx *U, int L, int N, const double *gamma,
                                                 double dt, uint64_t seed, const uint64_t *uid,
                                                 const int64_t *step_ptr, int step_offset,
                                                 const int64_t *step_base, int *sites, int *outcomes,
                                                 double *probs, int *counts, cplx *vbuf,
                                                 cplx *wbuf) {
  const int b = blockIdx.x;
  const uint64_t step = (uint64_t)(*step_ptr + step_offset - step_base[b]);
  const int cnt = pm_measure_block(U + (long)b * L * N, L, N, fmin(gamma[b] * dt, 1.0), seed, uid[b],
                                   step, sites + (long)b * L, outcomes + (long)b * L,
                                   probs + (long)b * L, vbuf + (long)b * N, wbuf + (long)b * L, L);
  if (threadIdx.x == 0) counts[b] = cnt;
}

// Trajectory `slot` back to its initial state U[:, k] = e_{occ[k]}, with a new
// uid and its own step count restarting at 0 (base = the context's step).
__global__ void reset_slot_kernel(cplx *U, int L, int N, int slot, const int *occ, uint64_t *uid,
                                  uint64_t new_uid, int64_t *step_base, int64_t base) {
  cplx *Us = U + (long)slot * L * N;
  for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < (long)L * N;
       idx += (long)gridDim.x * blockDim.x) {
    const int i = (int)(idx % L), k = (int)(idx / L);
    Us[idx] = cplx{occ[k] == i ? 1.0 : 0.0, 0.0};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uid[slot] = new_uid;
    step_base[slot] = base;
  }
}

__global__ void set_step_kernel(int64_t *step_ptr, int64_t value, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step_ptr = add ? *step_ptr + value : value;
}

}  // namespace

hipError_t reset_slot(cplx *U, int L, int N, int slot, const int *occ, uint64_t *uid, uint64_t new_uid,
                      int64_t *step_base, int64_t base, hipStream_t s) {
  const int blocks = (int)std::min<long>(((long)L * N + 255) / 256, 1024);
  hipLaunchKernelGGL(reset_slot_kernel, dim3(blocks), dim3(256), 0, s, U, L, N, slot, occ, uid, new_uid,
                     step_base, base);
  return hipGetLastError();
}

hipError_t set_step(int64_t *step_ptr, int64_t value, bool add, hipStream_t s) {
  hipLaunchKernelGGL(set_step_kernel, dim3(1), dim3(64), 0, s, step_ptr, value, add ? 1 : 0);
  return hipGetLastError();
}

hipError_t fill_zero(void *p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 8;
  if (n == 0) return hipSuccess;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint64_t *)p, n);
  return hipGetLastError();
}

hipError_t expand_propagator(cplx *P, const cplx *gx, const cplx *gy, int dim, int Lx, int Ly,
                             hipStream_t s) {
  const long L = (long)Lx * (dim == 2 ? Ly : 1);
  const long total = L * L;
  const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(expand_propagator_kernel, dim3(blocks), dim3(256), 0, s, P, gx, gy, dim, Lx,
                     Ly, L);
  return hipGetLastError();
}

hipError_t init_state(cplx *U, int L, int N, int B, const int *occ, hipStream_t s) {
  const long total = (long)L * N * B;
  const int blocks = (int)std::min<long>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(init_state_kernel, dim3(blocks), dim3(256), 0, s, U, L, N, total, occ);
  return hipGetLastError();
}

hipError_t ring_stencil(const cplx *U, cplx *D, const cplx *g, int L, int w, long ncols, hipStream_t s) {
  if (w < 0 || w > STENCIL_WMAX || 2 * w + 1 > L) return hipErrorInvalidValue;
  const int nrb = (L + 255) / 256;
  hipLaunchKernelGGL(ring_stencil_kernel, dim3((unsigned)(nrb * ncols)), dim3(256), 0, s, U, D, g, L, w, nrb);
  return hipGetLastError();
}

hipError_t born_homodyne(cplx *U, double *p, int L, int N, int B, const double *gamma, double dt,
                         uint64_t seed, const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                         const int64_t *step_base, hipStream_t s) {
  if (N <= 16 * 32) {  // rows in registers: one read and one write of U
    const dim3 g16((L + 15) / 16, B);
    if (N <= 16 * 8)
      hipLaunchKernelGGL((born_rows_kernel<true, 8>), g16, dim3(256), 0, s, U, p, L, N, gamma, dt, seed,
                         uid, step_ptr, step_offset, step_base);
    else if (N <= 16 * 16)
      hipLaunchKernelGGL((born_rows_kernel<true, 16>), g16, dim3(256), 0, s, U, p, L, N, gamma, dt, seed,
                         uid, step_ptr, step_offset, step_base);
    else
      hipLaunchKernelGGL((born_rows_kernel<true, 32>), g16, dim3(256), 0, s, U, p, L, N, gamma, dt, seed,
                         uid, step_ptr, step_offset, step_base);
    return hipGetLastError();
  }
  dim3 grid((L + 255) / 256, B);
  hipLaunchKernelGGL(born_kernel<true>, grid, dim3(256), 0, s, U, p, L, N, gamma, dt, seed, uid,
                     step_ptr, step_offset, step_base);
  return hipGetLastError();
}

hipError_t born_only(const cplx *U, double *p, int L, int N, int B, hipStream_t s) {
  dim3 grid((L + 255) / 256, B);
  hipLaunchKernelGGL(born_kernel<false>, grid, dim3(256), 0, s, const_cast<cplx *>(U), p, L, N,
                     nullptr, 0.0, 0ull, nullptr, nullptr, 0, nullptr);
  return hipGetLastError();
}

hipError_t pm_measure(cplx *U, int L, int N, int B, const double *gamma, double dt, uint64_t seed,
                      const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                      const int64_t *step_base, int *sites, int *outcomes, double *probs, int *counts,
                      cplx *vbuf, cplx *wbuf, hipStream_t s) {
  hipLaunchKernelGGL(pm_kernel, dim3(B), dim3(256), 0, s, U, L, N, gamma, dt, seed, uid, step_ptr,
                     step_offset, step_base, sites, outcomes, probs, counts, vbuf, wbuf);
  return hipGetLastError();
}

}  // namespace mfq
