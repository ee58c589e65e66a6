// Homodyne step integrated by RK4 (Appendix A: Eq. (A4) with the fourth-order
// Runge-Kutta method).  Over the step the exponent of Eq. (A4),
//   A = -i Ht dt + diag(a),  a_i = dW_i + (2 p_i - 1) gamma dt,  dW_i = sqrt(gamma dt) z_i,
// is frozen at the start of the step, so one classical RK4 step of dU/ds = (A/dt) U over
// [0, dt] equals the degree-4 Taylor polynomial of exp(A) applied to U, evaluated here in
// Horner form:
//   V1 = U + (A/4) U,  V2 = U + (A/3) V1,  V3 = U + (A/2) V2,  U' = U + A V3.
// A is the nearest-neighbour hopping (two neighbours on the ring, four on the torus, site
// i = x + Lx y) plus the diagonal, so each stage is one pass over the state: it reads U and
// V (neighbour rows of V from cache) and writes the next V; the last stage writes U' over U
// (each element of U is read only by the thread that overwrites it).
#include "mfq_internal.h"
#include "device_common.h"

namespace mfq {

namespace {

// a_i = sqrt(gamma dt) z_i + (2 p_i - 1) gamma dt with the homodyne normals of the split
// step (Philox purpose 1, site i, the trajectory's own step index).
__global__ __launch_bounds__(256) void rk4_diag_kernel(const double *p, double *a, int L, const double *gamma,
                                                       double dt, uint64_t seed, const uint64_t *uid,
                                                       const int64_t *step_ptr, int step_offset,
                                                       const int64_t *step_base) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= L) return;
  const double g = gamma[b];
  const uint64_t step = (uint64_t)(*step_ptr + step_offset - step_base[b]);
  const u64x4 w = philox4x64_10(seed, uid[b], step, (uint64_t)i, PURPOSE_HOMODYNE, 0);
  const double z = sqrt(-2.0 * log(u01(w.v[0]))) * cos(6.283185307179586 * u01(w.v[1]));
  a[(long)b * L + i] = sqrt(g * dt) * z + (2.0 * p[(long)b * L + i] - 1.0) * g * dt;
}

// Vout = U + inv_m (A Vin): 64 rows (one per lane) x 16 columns per workgroup, each wave
// four columns.  Vin must not alias Vout; Vout may alias U.
constexpr int RK_CPW = 4;
__global__ __launch_bounds__(256) void rk4_stage_kernel(const cplx *U, const cplx *Vin, cplx *Vout, int L, int N,
                                                        int dim, int Lx, int Ly, double cJ, double inv_m,
                                                        const double *a, int nrb) {
  const int b = blockIdx.y;
  const int rb = blockIdx.x % nrb, cb = blockIdx.x / nrb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = rb * 64 + lane;
  const int k0 = cb * (4 * RK_CPW) + wave * RK_CPW;
  if (i >= L || k0 >= N) return;
  int nb[4], nn;
  if (dim == 1) {
    nb[0] = i == 0 ? L - 1 : i - 1;
    nb[1] = i == L - 1 ? 0 : i + 1;
    nn = 2;
  } else {
    const int x = i % Lx, y = i / Lx;
    nb[0] = (x == 0 ? Lx - 1 : x - 1) + Lx * y;
    nb[1] = (x == Lx - 1 ? 0 : x + 1) + Lx * y;
    nb[2] = x + Lx * (y == 0 ? Ly - 1 : y - 1);
    nb[3] = x + Lx * (y == Ly - 1 ? 0 : y + 1);
    nn = 4;
  }
  const double ai = a[(long)b * L + i];
  const long base = (long)b * L * N;
#pragma unroll
  for (int q = 0; q < RK_CPW; ++q) {
    const int k = k0 + q;
    if (k >= N) break;
    const long col = base + (long)k * L;
    double sr = 0.0, si = 0.0;
    for (int t = 0; t < nn; ++t) {
      const cplx v = Vin[col + nb[t]];
      sr += v.re;
      si += v.im;
    }
    const cplx v = Vin[col + i], u = U[col + i];
    // A V = -i cJ S + a_i V
    const double avr = cJ * si + ai * v.re;
    const double avi = -cJ * sr + ai * v.im;
    Vout[col + i] = cplx{u.re + inv_m * avr, u.im + inv_m * avi};
  }
}

}  // namespace

hipError_t rk4_homodyne(cplx *U, cplx *V1, cplx *V2, const double *p, double *a, int L, int N, int B, int dim,
                        int Lx, int Ly, double J, const double *gamma, double dt, uint64_t seed,
                        const uint64_t *uid, const int64_t *step_ptr, int step_offset,
                        const int64_t *step_base, hipStream_t s) {
  if (L != Lx * (dim == 2 ? Ly : 1) || N < 1 || B < 1 || U == V1 || U == V2 || V1 == V2)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(rk4_diag_kernel, dim3((L + 255) / 256, B), dim3(256), 0, s, p, a, L, gamma, dt, seed, uid,
                     step_ptr, step_offset, step_base);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nrb = (L + 63) / 64, ncb = (N + 4 * RK_CPW - 1) / (4 * RK_CPW);
  const dim3 grid((unsigned)(nrb * ncb), B);
  const double cJ = dt * J;
  // V1 = U + (A/4) U; V2 = U + (A/3) V1; V1 = U + (A/2) V2; U = U + A V1
  const cplx *vin[4] = {U, V1, V2, V1};
  cplx *vout[4] = {V1, V2, V1, U};
  const double inv[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
  for (int st = 0; st < 4; ++st) {
    hipLaunchKernelGGL(rk4_stage_kernel, grid, dim3(256), 0, s, (const cplx *)U, vin[st], vout[st], L, N, dim, Lx,
                       Ly, cJ, inv[st], (const double *)a, nrb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace mfq
