// State kernels: initial state, propagator expansion, Born probabilities with
// the fused homodyne update, and the projective measurement.
//
// Layout: U of trajectory b is column-major L x N (ld = L) at U + b*L*N.  A
// thread owns rows, so every load/store of a column is coalesced across the
// wave (64 consecutive rows = 1 KiB per column).
#include "mfq_internal.h"
#include "philox.h"

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
                                                   const uint64_t *uid, uint64_t step) {
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

__device__ __forceinline__ double block_sum(double v, double *red) {
  // 256 threads: wave reduction, then across the 4 waves (fixed order)
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  return r;
}

// Projective measurement of one step for one trajectory per workgroup.
// Sites are selected with probability q = min(gamma dt, 1) (Philox purpose 0,
// word 0) and projected in ascending order.  Each projection: x = conj(U_j.),
// Householder H = I - tau v v^+ with H x = beta e_0, U <- U H (row j is then
// confined to column 0), outcome 1 iff u (word 1) <= p = |x|^2; outcome 1:
// column 0 := e_j; outcome 0: U_j0 := 0 and column 0 renormalised.
__global__ __launch_bounds__(256) void pm_kernel(cplx *U, int L, int N, const double *gamma,
                                                 double dt, uint64_t seed, const uint64_t *uid,
                                                 uint64_t step, int *sites, int *outcomes,
                                                 double *probs, int *counts, cplx *vbuf,
                                                 cplx *wbuf) {
  const int b = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  cplx *Ub = U + (long)b * L * N;
  cplx *v = vbuf + (long)b * N;
  cplx *w = wbuf + (long)b * L;
  int *site = sites + (long)b * L;
  const uint64_t key1 = uid[b];
  const double q = fmin(gamma[b] * dt, 1.0);
  __shared__ int wave_cnt[4];
  __shared__ int total;
  __shared__ double red[4];
  __shared__ double sh_tau, sh_v0re, sh_v0im;
  __shared__ int sh_outcome, sh_skip;

  // ---- selection with ascending compaction
  if (tid == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < L; base += 256) {
    const int i = base + tid;
    bool sel = false;
    if (i < L) {
      const u64x4 r = philox4x64_10(seed, key1, step, (uint64_t)i, PURPOSE_PROJECTIVE, 0);
      sel = u01(r.v[0]) < q;
    }
    const unsigned long long m = __ballot(sel);
    if (lane == 0) wave_cnt[wave] = __popcll(m);
    __syncthreads();
    int off = total;
    for (int wv = 0; wv < wave; ++wv) off += wave_cnt[wv];
    if (sel) site[off + __popcll(m & ((1ull << lane) - 1ull))] = i;
    __syncthreads();
    if (tid == 0) total += wave_cnt[0] + wave_cnt[1] + wave_cnt[2] + wave_cnt[3];
    __syncthreads();
  }
  const int cnt = total;
  if (tid == 0) counts[b] = cnt;

  for (int e = 0; e < cnt; ++e) {
    const int j = site[e];
    // x = conj(row j), |x|^2
    double part = 0.0;
    for (int k = tid; k < N; k += 256) {
      const cplx a = Ub[j + (long)k * L];
      v[k] = cplx{a.re, -a.im};
      part += a.re * a.re + a.im * a.im;
    }
    const double p = block_sum(part, red);
    if (tid == 0) {
      const u64x4 r = philox4x64_10(seed, key1, step, (uint64_t)j, PURPOSE_PROJECTIVE, 0);
      const int outcome = (u01(r.v[1]) <= p) ? 1 : 0;
      sh_outcome = outcome;
      outcomes[(long)b * L + e] = outcome;
      probs[(long)b * L + e] = p;
      const cplx x0 = v[0];
      const double ax0 = sqrt(x0.re * x0.re + x0.im * x0.im);
      const double nx = sqrt(p);
      if (nx == 0.0) {
        sh_skip = 1;
      } else {
        sh_skip = 0;
        const double phr = ax0 > 0.0 ? x0.re / ax0 : 1.0, phi = ax0 > 0.0 ? x0.im / ax0 : 0.0;
        const double br = -phr * nx, bi = -phi * nx;  // beta
        const double v0r = x0.re - br, v0i = x0.im - bi;
        const double vn2 = (p - ax0 * ax0) + (v0r * v0r + v0i * v0i);
        sh_tau = 2.0 / vn2;
        sh_v0re = v0r;
        sh_v0im = v0i;
        v[0] = cplx{v0r, v0i};
      }
    }
    __syncthreads();
    if (sh_skip) {  // empty row: p = 0, outcome 0 leaves the state unchanged
      __syncthreads();
      continue;
    }
    const double tau = sh_tau;
    const int outcome = sh_outcome;
    // w = U v
    for (int i = tid; i < L; i += 256) {
      double ar = 0.0, ai = 0.0;
      for (int k = 0; k < N; ++k) {
        const cplx u = Ub[i + (long)k * L], vk = v[k];
        ar += u.re * vk.re - u.im * vk.im;
        ai += u.re * vk.im + u.im * vk.re;
      }
      w[i] = cplx{ar * tau, ai * tau};
    }
    // U <- U - (tau w) v^+ ; row j exactly confined to column 0
    double part0 = 0.0;
    for (int i = tid; i < L; i += 256) {
      const cplx wi = w[i];
      for (int k = 1; k < N; ++k) {
        cplx u = Ub[i + (long)k * L];
        const cplx vk = v[k];
        if (i == j) {
          u = cplx{0.0, 0.0};
        } else {
          u.re -= wi.re * vk.re + wi.im * vk.im;
          u.im -= wi.im * vk.re - wi.re * vk.im;
        }
        Ub[i + (long)k * L] = u;
      }
      cplx c0;
      if (outcome == 1) {
        c0 = cplx{i == j ? 1.0 : 0.0, 0.0};
      } else if (i == j) {
        c0 = cplx{0.0, 0.0};
      } else {
        c0 = Ub[i];
        const cplx v0 = v[0];
        c0.re -= wi.re * v0.re + wi.im * v0.im;
        c0.im -= wi.im * v0.re - wi.re * v0.im;
        part0 += c0.re * c0.re + c0.im * c0.im;
      }
      Ub[i] = c0;
    }
    if (outcome == 0) {
      const double n0 = block_sum(part0, red);
      const double sc = 1.0 / sqrt(n0);
      for (int i = tid; i < L; i += 256) {
        cplx c0 = Ub[i];
        c0.re *= sc;
        c0.im *= sc;
        Ub[i] = c0;
      }
    }
    __syncthreads();
  }
}

}  // namespace

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

hipError_t born_homodyne(cplx *U, double *p, int L, int N, int B, const double *gamma, double dt,
                         uint64_t seed, const uint64_t *uid, int64_t step, hipStream_t s) {
  dim3 grid((L + 255) / 256, B);
  hipLaunchKernelGGL(born_kernel<true>, grid, dim3(256), 0, s, U, p, L, N, gamma, dt, seed, uid,
                     (uint64_t)step);
  return hipGetLastError();
}

hipError_t born_only(const cplx *U, double *p, int L, int N, int B, hipStream_t s) {
  dim3 grid((L + 255) / 256, B);
  hipLaunchKernelGGL(born_kernel<false>, grid, dim3(256), 0, s, const_cast<cplx *>(U), p, L, N,
                     nullptr, 0.0, 0ull, nullptr, 0ull);
  return hipGetLastError();
}

hipError_t pm_measure(cplx *U, int L, int N, int B, const double *gamma, double dt, uint64_t seed,
                      const uint64_t *uid, int64_t step, int *sites, int *outcomes, double *probs,
                      int *counts, cplx *vbuf, cplx *wbuf, hipStream_t s) {
  hipLaunchKernelGGL(pm_kernel, dim3(B), dim3(256), 0, s, U, L, N, gamma, dt, seed, uid,
                     (uint64_t)step, sites, outcomes, probs, counts, vbuf, wbuf);
  return hipGetLastError();
}

}  // namespace mfq
