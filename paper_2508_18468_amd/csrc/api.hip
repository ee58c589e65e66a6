// C ABI of libmfq: context, device memory plan and the step / observable
// drivers.  Every arithmetic step runs in the HIP kernels of this library;
// the host only validates arguments, computes the propagator's generating
// row (a Bessel series, once per dt) and orders launches on the stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mfq.h"
#include "group_schedule.h"

#include "mfq_internal.h"

using namespace mfq;

// Static device buffer of mfq_density_correlation_noalloc.  Each GPU holds its own copy for
// the lifetime of the process; host code may use only the per-device address resolved by
// hipGetSymbolAddress (the name itself is a host-side stand-in, not a device address).
static __device__ __align__(256) double scratch[MFQ_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_dev;  // per device; null until resolved

// Resolves `device`'s address of the static buffer once (the device must be current).
hipError_t resolve_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= device) g_scratch_dev.resize(device + 1, nullptr);
  if (g_scratch_dev[device]) return hipSuccess;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_dev[device] = static_cast<double *>(ptr);
  return hipSuccess;
}

double *scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device < (int)g_scratch_dev.size() ? g_scratch_dev[device] : nullptr;
}

}  // namespace

struct mfq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  // problem
  bool ready = false;
  mfq_lattice lat{};
  int L = 0, N = 0, B = 0, precision = 0;
  int64_t step = 0;
  double dt_cached = NAN;
  // workspace
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  cplx *X[2] = {nullptr, nullptr};
  int cur = 0;
  cplx *P = nullptr, *gx = nullptr, *gy = nullptr;
  // factored propagator: band of the ring stencil (1d) or the factors P_x, P_y (2d)
  int prop_form = 0;  // MFQ_PROP_DENSE
  int band_w = -1;    // -1: no band narrower than the ring
  cplx *Pkx = nullptr, *Pky = nullptr;
  int g_prop = -1;    // propagator form the cached graph was captured with
  float *Pr32 = nullptr, *Pi32 = nullptr;  // FP32-bulk: planes of P - I
  CholWork chol{};
  EigWork eig{};
  double *p = nullptr, *gamma = nullptr;
  uint64_t *uid = nullptr;
  int *occ = nullptr, *region = nullptr, *flag = nullptr;
  BreakdownInfo *info = nullptr;  // where the flag's breakdown was seen
  int *pm_sites = nullptr, *pm_out = nullptr, *pm_cnt = nullptr;
  double *pm_prob = nullptr;
  cplx *pm_v = nullptr, *pm_w = nullptr;
  PmBlockedWork pmb{};
  int pm_path = 0;  // MFQ_PM_AUTO
  ContWork ct{};    // continuous-time protocol: clocks, ring rows, event records
  int integrator = 0;       // MFQ_INTEGRATOR_SPLIT
  int g_integ = -1;         // integrator the cached graph was captured with
  void *rk_buf = nullptr;   // RK4 scratch (a third state buffer and the diagonal), on first use
  size_t rk_cap = 0;
  bool ct_any = false;  // an event batch has run since mfq_init_state
  int ct_block = 0;     // deferred continuous-time events per block (0: event by event)
  BlockWork bw{};
  void *blk_buf = nullptr;
  size_t blk_cap = 0;
  std::vector<double> gamma_host;
  // phase timing
  bool profiling = false;
  std::vector<hipEvent_t> events;     // pool, reused after every read-out
  size_t events_used = 0;
  std::vector<int> rec_phase;         // interval i: phase, events 2i and 2i+1
  double phase_ms[MFQ_NPHASES] = {0, 0, 0, 0};
  int64_t phase_n[MFQ_NPHASES] = {0, 0, 0, 0};
  // step counter on the device and the cached two-step graph
  int64_t *step_dev = nullptr;
  int64_t *step_base = nullptr;  // per trajectory: own step = step - step_base[b]
  bool use_graphs = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_protocol = -1, g_cur = -1;
  double g_dt = NAN;
  uint64_t g_seed = 0;
  // mfq_run: execution path and its observation buffer; GEMM tile choice
  int run_path = 0;   // MFQ_PATH_AUTO
  int tile_mode = 0;  // MFQ_TILE_AUTO
  int tile_order = 0;  // MFQ_ORDER_XCD
  int eig_mode = 0;   // MFQ_EIG_AUTO
  // correlation observables: tile partials and results (allocated on first use)
  double *red_buf = nullptr;
  size_t red_cap = 0;
  int g_tile = -1;    // tile choice the cached graph was captured with
  int g_order = -1;   // tile order the cached graph was captured with
  double *run_S = nullptr;
  size_t run_S_cap = 0;
};

namespace {

mfq_status fail(mfq_ctx *c, mfq_status code, const std::string &msg) {
  if (c) c->err = msg;
  return code;
}

mfq_status hip_fail(mfq_ctx *c, hipError_t e, const char *where) {
  return fail(c, MFQ_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(expr, where)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(c, e_, where); \
  } while (0)

bool lattice_ok(const mfq_lattice *lat) {
  if (!lat) return false;
  if (lat->dim == 1) return lat->Lx >= 2 && lat->Lx <= (1 << 20) && std::isfinite(lat->J);
  if (lat->dim == 2)
    return lat->Lx >= 2 && lat->Ly >= 2 && (long)lat->Lx * lat->Ly <= (1 << 20) &&
           std::isfinite(lat->J);
  return false;
}

int lattice_L(const mfq_lattice *lat) { return lat->dim == 1 ? lat->Lx : lat->Lx * lat->Ly; }

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Sub-buffers of the workspace at `base` (256-aligned), from the layout of workspace_layout.h.
void carve(char *base, const WsLayout &w, const mfq_lattice &lat, int N, mfq_ctx *c) {
  auto at = [&](int r) -> void * { return w.count[r] ? base + w.off[r] : nullptr; };
  const long NN = (long)N * N;
  cplx *G = (cplx *)at(WS_G), *Rinv = (cplx *)at(WS_RINV), *T = (cplx *)at(WS_T);
  c->Pr32 = (float *)at(WS_PR32); c->Pi32 = (float *)at(WS_PI32);
  c->X[0] = (cplx *)at(WS_X0); c->X[1] = (cplx *)at(WS_X1); c->P = (cplx *)at(WS_P);
  c->gx = (cplx *)at(WS_GX); c->gy = (cplx *)at(WS_GY);
  c->Pkx = (cplx *)at(WS_PKX); c->Pky = (cplx *)at(WS_PKY);
  c->flag = (int *)at(WS_FLAG);
  c->info = (BreakdownInfo *)at(WS_INFO);
  c->chol = CholWork{G, Rinv, T, c->flag, c->info, (double *)at(WS_DEV)};
  c->step_dev = (int64_t *)at(WS_STEP);
  c->step_base = (int64_t *)at(WS_STEP_BASE);
  // the blocked reduction keeps its panels in Rinv (free outside a step; trd_panel_elems(n) <= N^2
  // for TRD_BLOCKED_MIN <= n <= N)
  c->eig = EigWork{G, (cplx *)at(WS_EV), (cplx *)at(WS_EW), (cplx *)at(WS_EP), (double *)at(WS_ETAU),
                   (double *)at(WS_ED), (double *)at(WS_EE), (double *)at(WS_ELAM), (double *)at(WS_ES),
                   Rinv, NN, c->flag, c->info};
  c->p = (double *)at(WS_BORN); c->gamma = (double *)at(WS_GAMMA); c->uid = (uint64_t *)at(WS_UID);
  c->occ = (int *)at(WS_OCC); c->region = (int *)at(WS_REGION);
  c->pm_sites = (int *)at(WS_PM_SITES); c->pm_out = (int *)at(WS_PM_OUT); c->pm_cnt = (int *)at(WS_PM_CNT);
  c->pm_prob = (double *)at(WS_PM_PROB);
  c->pm_v = (cplx *)at(WS_PM_V); c->pm_w = (cplx *)at(WS_PM_W);
  c->pmb = PmBlockedWork{c->pm_sites, c->pm_out, c->pm_cnt, c->pm_prob, (double *)at(WS_PM_U),
                         (double *)at(WS_PM_TAU), (int *)at(WS_PM_M1), (int *)at(WS_PM_K1),
                         (int *)at(WS_PM_CODE), G, Rinv, T};
  const int Lyr = lat.dim == 2 ? lat.Ly : 1;
  c->ct = ContWork{(double *)at(WS_CT_T), (cplx *)at(WS_CT_G), (double *)at(WS_CT_JN), (int *)at(WS_CT_INFO),
                   (double *)at(WS_CT_DINFO), (cplx *)at(WS_CT_V), (cplx *)at(WS_CT_Y), (cplx *)at(WS_CT_YP),
                   cont_jcap(lat.Lx, Lyr)};
}

WsLayout layout_of(const mfq_lattice &lat, int N, int B, int precision) {
  return plan_workspace(lat.dim, lat.Lx, lat.dim == 2 ? lat.Ly : 1, N, B, precision == MFQ_FP32_BULK);
}

// Generating row of the ring propagator exp(-i Ht dt) from the Jacobi-Anger
// expansion exp(-i z cos k) = sum_n (-i)^n J_n(z) e^{ink}, z = 2 J dt:
// g[d] = sum over integers n = d (mod Lr) of (-i)^|n| J_|n|(z).
void ring_row(int Lr, double J, double dt, std::vector<std::complex<double>> &g) {
  g.assign(Lr, std::complex<double>(0.0, 0.0));
  const double z = 2.0 * J * dt, az = std::fabs(z);
  const std::complex<double> mi(0.0, -1.0);
  // J_n(|z|) falls below 1e-300 of J_0 long before n = |z| + 80 for |z| <= 100
  const int nmax = (int)az + 80;
  std::vector<double> jn(nmax + 1);
  for (int n = 0; n <= nmax; ++n) {
    double v = (az == 0.0) ? (n == 0 ? 1.0 : 0.0) : std::cyl_bessel_j((double)n, az);
    if (z < 0.0 && (n & 1)) v = -v;  // J_n(-x) = (-1)^n J_n(x)
    jn[n] = v;
  }
  for (int n = -nmax; n <= nmax; ++n) {
    const int an = n < 0 ? -n : n;
    std::complex<double> ph(1.0, 0.0);
    switch (an & 3) {
      case 1: ph = mi; break;
      case 2: ph = -1.0; break;
      case 3: ph = -mi; break;
      default: break;
    }
    const int d = ((n % Lr) + Lr) % Lr;
    g[d] += ph * jn[an];
  }
}

// Record an event on the stream (phase timing); returns false on failure.
bool record_event(mfq_ctx *c) {
  if (c->events_used == c->events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return false;
    c->events.push_back(e);
  }
  return hipEventRecord(c->events[c->events_used++], c->stream) == hipSuccess;
}

struct PhaseTimer {
  mfq_ctx *c;
  int phase;
  bool on;
  PhaseTimer(mfq_ctx *c_, int ph) : c(c_), phase(ph), on(c_->profiling) {
    if (on) on = record_event(c);
  }
  ~PhaseTimer() {
    if (on && record_event(c)) c->rec_phase.push_back(phase);
    else if (on) c->events_used--;
  }
};

mfq_status collect_phase_times(mfq_ctx *c) {
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  for (size_t i = 0; i < c->rec_phase.size(); ++i) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, c->events[2 * i], c->events[2 * i + 1]), "event time");
    c->phase_ms[c->rec_phase[i]] += ms;
    c->phase_n[c->rec_phase[i]] += 1;
  }
  c->rec_phase.clear();
  c->events_used = 0;
  return MFQ_OK;
}

// Clears the error flag and the breakdown record (each in its own 256-byte region).
hipError_t clear_flag(mfq_ctx *c) {
  hipError_t e = fill_zero(c->flag, 256, c->stream);
  if (e == hipSuccess) e = fill_zero(c->info, 256, c->stream);
  return e;
}

mfq_status check_flag(mfq_ctx *c) {
  int f = 0;
  BreakdownInfo info{};
  HIPCHK(hipMemcpyAsync(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "flag read");
  HIPCHK(hipMemcpyAsync(&info, c->info, sizeof(info), hipMemcpyDeviceToHost, c->stream), "breakdown read");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  if (f) {
    HIPCHK(clear_flag(c), "flag clear");
    HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
    if (info.set && info.source == 4)
      return fail(c, MFQ_EDEVICE, "tridiagonal reduction: a bulge-chase dependency wait exceeded its limit "
                                  "(trajectory " + std::to_string(info.traj) + ", sweep " +
                                  std::to_string(info.col) + ")");
    if (info.set && info.source == 5)
      return fail(c, MFQ_EDEVICE, "band reduction: a wait for the other workgroups of a panel exceeded its "
                                  "limit (trajectory " + std::to_string(info.traj) + ", column " +
                                  std::to_string(info.col) + ")");
    static const char *src[] = {"unknown source", "Cholesky-QR pass 1", "Cholesky-QR pass 2", "fused kernel"};
    char where[192] = "";
    if (info.set)
      std::snprintf(where, sizeof(where), ": %s, trajectory %d, column %d, pivot %.17g",
                    src[(info.source >= 1 && info.source <= 3) ? info.source : 0], info.traj, info.col,
                    info.pivot);
    return fail(c, MFQ_ENUMERIC, std::string("Cholesky breakdown (non-positive or non-finite pivot)") + where);
  }
  return MFQ_OK;
}

mfq_status build_propagator(mfq_ctx *c, double dt) {
  std::vector<std::complex<double>> gx, gy;
  ring_row(c->lat.Lx, c->lat.J, dt, gx);
  if (c->lat.dim == 2) ring_row(c->lat.Ly, c->lat.J, dt, gy);
  else gy.assign(1, std::complex<double>(1.0, 0.0));
  for (auto &z : gx)
    if (!std::isfinite(z.real()) || !std::isfinite(z.imag()))
      return fail(c, MFQ_EINVAL, "propagator not finite for this dt");
  HIPCHK(hipMemcpyAsync(c->gx, gx.data(), gx.size() * sizeof(cplx), hipMemcpyHostToDevice, c->stream),
         "propagator row upload");
  HIPCHK(hipMemcpyAsync(c->gy, gy.data(), gy.size() * sizeof(cplx), hipMemcpyHostToDevice, c->stream),
         "propagator row upload");
  HIPCHK(expand_propagator(c->P, c->gx, c->gy, c->lat.dim, c->lat.Lx, c->lat.Ly, c->stream),
         "expand_propagator");
  // factored form: band of the ring row (entries beyond it are below 1e-20 of the largest,
  // far under the rounding of the kept terms), or the two ring factors of the torus
  c->band_w = -1;
  if (c->lat.dim == 1) {
    double gmax = 0.0;
    for (auto &z : gx) gmax = std::max(gmax, std::abs(z));
    int w = 0;
    for (int d = 1; d <= c->lat.Lx / 2; ++d)
      if (std::abs(gx[d]) > 1e-20 * gmax || std::abs(gx[c->lat.Lx - d]) > 1e-20 * gmax) w = d;
    if (2 * w + 1 <= c->lat.Lx && w <= 128) c->band_w = w;
  } else {
    HIPCHK(expand_propagator(c->Pkx, c->gx, c->gy, 1, c->lat.Lx, 1, c->stream), "expand P_x");
    HIPCHK(expand_propagator(c->Pky, c->gy, c->gx, 1, c->lat.Ly, 1, c->stream), "expand P_y");
  }
  if (c->precision == MFQ_FP32_BULK)
    HIPCHK(make_delta_planes(c->P, c->Pr32, c->Pi32, c->L, c->stream), "delta planes");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  c->dt_cached = dt;
  return MFQ_OK;
}

mfq_status validate_region(mfq_ctx *c, const int32_t *r, int32_t n) {
  if (n < 0 || n > c->L) return fail(c, MFQ_EINVAL, "region size out of range");
  if (n > 0 && !r) return fail(c, MFQ_EINVAL, "region is NULL");
  for (int i = 0; i < n; ++i) {
    if (r[i] < 0 || r[i] >= c->L) return fail(c, MFQ_EINVAL, "region site out of range");
    if (i > 0 && r[i] <= r[i - 1]) return fail(c, MFQ_EINVAL, "region not strictly ascending");
  }
  return MFQ_OK;
}

// Eigenvalues of C_A for every trajectory into c->eig.lam; *n_out = their count.
mfq_status region_spectrum_dev(mfq_ctx *c, const int32_t *region, int32_t n, int *n_out) {
  mfq_status st = validate_region(c, region, n);
  if (st) return st;
  *n_out = 0;
  if (n == 0) return MFQ_OK;
  PhaseTimer t(c, MFQ_PHASE_OBSERVE);
  HIPCHK(hipMemcpyAsync(c->region, region, n * sizeof(int), hipMemcpyHostToDevice, c->stream),
         "region upload");
  int m = 0;
  HIPCHK(region_gram(c->X[c->cur], c->L, c->N, c->B, c->region, n, c->eig.A, &m, c->stream),
         "region_gram");
  HIPCHK(tridiagonalize(c->eig, m, c->B, c->stream), "tridiagonalize");
  HIPCHK(bisect_eigvals(c->eig, m, c->B, c->stream), "bisect");
  *n_out = m;
  return MFQ_OK;
}

mfq_status entropy_dev(mfq_ctx *c, const int32_t *region, int32_t n, double *S_host) {
  int m = 0;
  mfq_status st = region_spectrum_dev(c, region, n, &m);
  if (st) return st;
  if (m == 0) {
    for (int b = 0; b < c->B; ++b) S_host[b] = 0.0;
    return MFQ_OK;
  }
  {
    PhaseTimer t(c, MFQ_PHASE_OBSERVE);
    HIPCHK(entropy_sum(c->eig, m, c->B, c->stream), "entropy");
  }
  HIPCHK(hipMemcpyAsync(S_host, c->eig.S, c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream),
         "entropy download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return MFQ_OK;
}


mfq_status validate_step(mfq_ctx *c, int protocol, const double *gamma, double dt, int n_steps) {
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (protocol != MFQ_PROJECTIVE && protocol != MFQ_HOMODYNE) return fail(c, MFQ_EINVAL, "bad protocol");
  if (!gamma) return fail(c, MFQ_EINVAL, "gamma is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(c, MFQ_EINVAL, "dt must be positive and finite");
  if (n_steps < 0) return fail(c, MFQ_EINVAL, "n_steps < 0");
  for (int b = 0; b < c->B; ++b)
    if (!(gamma[b] >= 0.0) || !std::isfinite(gamma[b])) return fail(c, MFQ_EINVAL, "gamma must be >= 0");
  return MFQ_OK;
}

// Propagator for dt and the monitoring rates on the device.
mfq_status prepare_step(mfq_ctx *c, const double *gamma, double dt) {
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  if (!(dt == c->dt_cached)) {
    mfq_status st = build_propagator(c, dt);
    if (st) return st;
  }
  if (std::memcmp(c->gamma_host.data(), gamma, c->B * sizeof(double)) != 0) {
    std::memcpy(c->gamma_host.data(), gamma, c->B * sizeof(double));
    HIPCHK(hipMemcpyAsync(c->gamma, c->gamma_host.data(), c->B * sizeof(double), hipMemcpyHostToDevice,
                          c->stream), "gamma upload");
  }
  return MFQ_OK;
}

// Projective steps use the blocked measurement wherever it applies (N >= 128): measured
// on rings of 256 to 2048 sites with 1 to 384 trajectories it takes 0.2-0.75x the
// per-workgroup form's time (0.06x for one trajectory of 1024 sites).  It synchronises
// the stream, so such steps are never captured in a graph.
bool blocked_pm(const mfq_ctx *c) {
  if (c->pm_path == MFQ_PM_BLOCKED) return true;
  return c->pm_path == MFQ_PM_AUTO && c->N >= PM_BLOCKED_MIN_N;
}

size_t rk4_state_bytes(const mfq_ctx *c) {
  return align_up((size_t)c->L * c->N * c->B * sizeof(cplx));
}

// RK4 scratch: a third state buffer and the diagonal (L per trajectory), allocated on first
// use outside any graph capture.
mfq_status ensure_rk4(mfq_ctx *c) {
  const size_t need = rk4_state_bytes(c) + (size_t)c->L * c->B * sizeof(double);
  if (c->rk_cap >= need) return MFQ_OK;
  if (c->rk_buf) {
    HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
    (void)hipFree(c->rk_buf);
    c->rk_buf = nullptr;
    c->rk_cap = 0;
  }
  if (hipMalloc(&c->rk_buf, need) != hipSuccess) {
    c->rk_buf = nullptr;
    return fail(c, MFQ_ENOMEM, "hipMalloc of the RK4 scratch failed");
  }
  c->rk_cap = need;
  return MFQ_OK;
}

bool factored_propagator(const mfq_ctx *c) {
  return c->prop_form == MFQ_PROP_FACTORED && (c->lat.dim == 2 || c->band_w >= 0);
}

// Enqueue one step on the stream; the step index is read on the device as
// *step_dev + step_offset.  The propagated state lands in X[1-cur] (dense form,
// ring band) or, for the torus factors and RK4, back in X[cur]; the measurement
// works in place, and Cholesky-QR2 leaves the orthonormal factor in the other
// buffer, which becomes the current one.
mfq_status enqueue_step(mfq_ctx *c, int protocol, double dt, uint64_t seed, int step_offset) {
  const int L = c->L, N = c->N, B = c->B;
  cplx *Xa = c->X[c->cur], *Xb = c->X[1 - c->cur];
  int pidx = 1 - c->cur;
  const bool rk4 = protocol == MFQ_HOMODYNE && c->integrator == MFQ_INTEGRATOR_RK4;
  if (rk4) {  // homodyne step by RK4: the whole step in place on the current buffer
    PhaseTimer t(c, MFQ_PHASE_PROPAGATE);
    const int Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
    cplx *V2 = reinterpret_cast<cplx *>(c->rk_buf);
    double *a = reinterpret_cast<double *>(reinterpret_cast<char *>(c->rk_buf) + rk4_state_bytes(c));
    HIPCHK(born_only(Xa, c->p, L, N, B, c->stream), "born");
    HIPCHK(rk4_homodyne(Xa, Xb, V2, c->p, a, L, N, B, c->lat.dim, c->lat.Lx, Ly, c->lat.J, c->gamma, dt, seed,
                        c->uid, c->step_dev, step_offset, c->step_base, c->stream), "rk4 homodyne");
    pidx = c->cur;
  }
  if (!rk4) {
    PhaseTimer t(c, MFQ_PHASE_PROPAGATE);
    if (factored_propagator(c) && c->lat.dim == 1) {
      HIPCHK(ring_stencil(Xa, Xb, c->gx, L, c->band_w, (long)N * B, c->stream), "propagator band");
    } else if (factored_propagator(c)) {
      // P U = vec(P_x X P_y^T) column by column, X the Lx x Ly view of a column (P_y = P_y^T)
      const int Lx = c->lat.Lx, Ly = c->lat.Ly;
      GemmDesc g{};
      g.alpha = cplx{1.0, 0.0};
      g.M = Lx; g.N = Ly * N * B; g.K = Lx; g.batch = 1;
      g.A = c->Pkx; g.lda = Lx; g.opA = OP_N;
      g.B = Xa; g.ldb = Lx; g.opB = OP_N;
      g.D = Xb; g.ldd = Lx;
      HIPCHK(zgemm(g, c->stream), "propagator P_x");
      GemmDesc h{};
      h.alpha = cplx{1.0, 0.0};
      h.M = Lx; h.N = Ly; h.K = Ly; h.batch = N * B;
      h.A = Xb; h.lda = Lx; h.sA = L; h.opA = OP_N;
      h.B = c->Pky; h.ldb = Ly; h.sB = 0; h.opB = OP_N;
      h.D = Xa; h.ldd = Lx; h.sD = L;
      HIPCHK(zgemm(h, c->stream), "propagator P_y");
      pidx = c->cur;
    } else if (c->precision == MFQ_FP32_BULK) {
      HIPCHK(propagator_delta_f32(c->Pr32, c->Pi32, Xa, Xb, L, N * B, c->stream), "propagator f32");
    } else {  // dense: Xb = P Xa, the batch as one L x (N*B) matrix
      GemmDesc g{};
      g.M = L; g.N = N * B; g.K = L; g.batch = 1;
      g.A = c->P; g.lda = L; g.opA = OP_N;
      g.B = Xa; g.ldb = L; g.opB = OP_N;
      g.D = Xb; g.ldd = L;
      g.alpha = cplx{1.0, 0.0};
      HIPCHK(zgemm_propagator(g, c->stream), "propagator gemm");
    }
  }
  Xb = c->X[pidx];          // propagated state
  Xa = c->X[1 - pidx];      // free buffer
  if (!rk4) {
    PhaseTimer t(c, MFQ_PHASE_MEASURE);
    if (protocol == MFQ_HOMODYNE) {
      HIPCHK(born_homodyne(Xb, c->p, L, N, B, c->gamma, dt, seed, c->uid, c->step_dev, step_offset,
                           c->step_base, c->stream), "homodyne");
    } else {
      bool fallback = true;
      if (blocked_pm(c))
        HIPCHK(pm_blocked(Xb, Xa, L, N, B, c->gamma, dt, seed, c->uid, c->step_dev, step_offset,
                          c->step_base, c->pmb, &fallback, c->stream), "projective (blocked)");
      if (fallback)
        HIPCHK(pm_measure(Xb, L, N, B, c->gamma, dt, seed, c->uid, c->step_dev, step_offset,
                          c->step_base, c->pm_sites, c->pm_out, c->pm_prob, c->pm_cnt, c->pm_v, c->pm_w,
                          c->stream), "projective");
    }
  }
  {
    PhaseTimer t(c, MFQ_PHASE_REORTH);
    HIPCHK(cholqr2(Xb, Xa, L, N, B, c->chol, c->stream), "cholqr2");
  }
  c->cur = 1 - pidx;  // the orthonormal factor is in Xa
  return MFQ_OK;
}

// The context's GEMM tile choice and reduction form for the launches of one ABI call.
struct TileScope {
  int saved, saved_order, saved_eig;
  explicit TileScope(const mfq_ctx *c)
      : saved(gemm_tile_mode()), saved_order(gemm_tile_order()), saved_eig(eig_path()) {
    set_gemm_tile_mode(c->tile_mode);
    set_gemm_tile_order(c->tile_order);
    set_eig_path(c->eig_mode);
  }
  ~TileScope() {
    set_gemm_tile_mode(saved);
    set_gemm_tile_order(saved_order);
    set_eig_path(saved_eig);
  }
};

void drop_graph(mfq_ctx *c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

// A graph of two consecutive steps (so the state returns to the same buffer)
// plus the step-counter advance; rebuilt when protocol, dt, seed or buffer
// parity change.  Replayed with hipGraphLaunch for each pair of steps.
mfq_status ensure_step_graph(mfq_ctx *c, int protocol, double dt, uint64_t seed) {
  if (c->gexec && c->g_protocol == protocol && c->g_dt == dt && c->g_seed == seed && c->g_cur == c->cur &&
      c->g_tile == c->tile_mode && c->g_order == c->tile_order && c->g_prop == c->prop_form &&
      c->g_integ == c->integrator)
    return MFQ_OK;
  drop_graph(c);
  const int cur0 = c->cur;
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed), "begin capture");
  mfq_status st = enqueue_step(c, protocol, dt, seed, 1);
  if (!st) st = enqueue_step(c, protocol, dt, seed, 2);
  hipError_t e = st ? hipSuccess : set_step(c->step_dev, 2, true, c->stream);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
  c->cur = cur0;
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_fail(c, e, "capture");
  if (e2 != hipSuccess) return hip_fail(c, e2, "end capture");
  c->graph = graph;
  HIPCHK(hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0), "graph instantiate");
  c->g_protocol = protocol;
  c->g_dt = dt;
  c->g_seed = seed;
  c->g_cur = cur0;
  c->g_tile = c->tile_mode;
  c->g_order = c->tile_order;
  c->g_prop = c->prop_form;
  c->g_integ = c->integrator;
  return MFQ_OK;
}

// Contexts of one mfq_run_group call that advance through their per-phase kernels: one graph
// holds two steps of every member context, each on a branch of its own (a side stream joined
// to the capture), so that the contexts' kernels can overlap; it is replayed while every
// member has two steps left before its next stop (its last step or an observation).  Steps
// outside such pairs run per context, and each context observes on its own schedule.
struct GroupRun {
  mfq_ctx *const *ctxs;
  const mfq_run_args *args;
  int n;
  std::vector<hipStream_t> side;  // one per context, and the origin of the capture at [n]
  std::vector<hipEvent_t> evs;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> key;           // members and their buffer parity when the graph was captured
  ~GroupRun() {
    for (hipStream_t st : side) (void)hipStreamSynchronize(st);
    drop();
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
    for (hipStream_t st : side) (void)hipStreamDestroy(st);
  }
  void drop() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
  hipEvent_t event(size_t i) { return evs[i]; }
};

// Capture two steps of each member context into one graph on the origin stream.
mfq_status capture_group(GroupRun &g, const std::vector<int> &members) {
  mfq_ctx *c = g.ctxs[members[0]];
  hipStream_t origin = g.side[g.n];
  g.drop();
  HIPCHK(hipStreamBeginCapture(origin, hipStreamCaptureModeRelaxed), "begin group capture");
  hipError_t e = hipEventRecord(g.event(0), origin);
  mfq_status st = MFQ_OK;
  for (size_t i = 0; i < members.size() && e == hipSuccess && !st; ++i) {
    mfq_ctx *ck = g.ctxs[members[i]];
    const mfq_run_args &r = g.args[members[i]];
    hipStream_t sk = g.side[members[i]];
    if ((e = hipStreamWaitEvent(sk, g.event(0), 0)) != hipSuccess) break;
    TileScope tiles(ck);
    hipStream_t own = ck->stream;
    const int cur0 = ck->cur;
    ck->stream = sk;
    st = enqueue_step(ck, r.protocol, r.dt, r.seed, 1);
    if (!st) st = enqueue_step(ck, r.protocol, r.dt, r.seed, 2);
    if (!st) e = set_step(ck->step_dev, 2, true, sk);
    ck->stream = own;
    ck->cur = cur0;
    if (!st && e == hipSuccess && (e = hipEventRecord(g.event(1 + members[i]), sk)) == hipSuccess)
      e = hipStreamWaitEvent(origin, g.event(1 + members[i]), 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t e2 = hipStreamEndCapture(origin, &graph);
  if (st || e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    if (st) return st;
    return hip_fail(c, e != hipSuccess ? e : e2, "group capture");
  }
  g.graph = graph;
  HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0), "group graph instantiate");
  for (int k : members) {
    g.key.push_back(k);
    g.key.push_back(g.ctxs[k]->cur);
  }
  return MFQ_OK;
}

mfq_status run_group_graph(mfq_ctx *const *ctxs, const mfq_run_args *args, int n) {
  mfq_ctx *c = ctxs[0];
  GroupRun g;
  g.ctxs = ctxs;
  g.args = args;
  g.n = n;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  for (int k = 0; k <= n; ++k) {
    hipStream_t st = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking), "stream create");
    g.side.push_back(st);
  }
  for (int k = 0; k < n + 2; ++k) {  // fork, one join per context, the group's completion
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
    g.evs.push_back(ev);
  }
  std::vector<hipEvent_t> ready(n, nullptr);
  for (int k = 0; k < n; ++k) {
    hipEvent_t ev = nullptr;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "event create");
    g.evs.push_back(ev);
    ready[k] = ev;
  }
  std::vector<int64_t> left(n), now(n);
  std::vector<int> every(n), k_obs(n, 0);
  for (int k = 0; k < n; ++k) {
    mfq_ctx *ck = ctxs[k];
    mfq_status st = prepare_step(ck, args[k].gamma, args[k].dt);
    if (!st && args[k].protocol == MFQ_HOMODYNE && ck->integrator == MFQ_INTEGRATOR_RK4) st = ensure_rk4(ck);
    if (st) return st;
    left[k] = args[k].n_steps;
    every[k] = args[k].obs_every;
  }
  for (;;) {
    for (int k = 0; k < n; ++k) now[k] = ctxs[k]->step;
    const mfq_group::Round round = mfq_group::plan_round(left, now, every);
    if (round.members.empty() && round.singles.empty()) break;
    const std::vector<int> &members = round.members;
    const int64_t pairs = round.pairs;
    if (!members.empty()) {
      std::vector<int> key;
      for (int k : members) {
        key.push_back(k);
        key.push_back(ctxs[k]->cur);
      }
      if (!g.exec || key != g.key) {
        mfq_status st = capture_group(g, members);
        if (st) return st;
      }
      hipStream_t origin = g.side[n];
      for (int k : members) {  // the graph after the work queued on the members' streams
        mfq_ctx *ck = ctxs[k];
        HIPCHK(set_step(ck->step_dev, ck->step, false, ck->stream), "step counter");
        HIPCHK(hipEventRecord(ready[k], ck->stream), "event record");
        HIPCHK(hipStreamWaitEvent(origin, ready[k], 0), "stream wait");
      }
      for (int64_t q = 0; q < pairs; ++q) HIPCHK(hipGraphLaunch(g.exec, origin), "group graph launch");
      HIPCHK(hipEventRecord(g.event(n + 1), origin), "event record");
      for (int k : members) {  // and the members' later work after it
        HIPCHK(hipStreamWaitEvent(ctxs[k]->stream, g.event(n + 1), 0), "stream wait");
        ctxs[k]->step += 2 * pairs;
        left[k] -= 2 * pairs;
      }
    }
    // contexts one step from their stop take it on their own stream
    for (int k : round.singles) {
      mfq_ctx *ck = ctxs[k];
      TileScope tiles(ck);
      HIPCHK(set_step(ck->step_dev, ck->step, false, ck->stream), "step counter");
      mfq_status st = enqueue_step(ck, args[k].protocol, args[k].dt, args[k].seed, 1);
      if (st) return st;
      ++ck->step;
      --left[k];
    }
    // every context that moved observes when it reached a multiple of its obs_every (the
    // schedule never takes it past one)
    for (int k = 0; k < n; ++k) {
      mfq_ctx *ck = ctxs[k];
      const bool moved = std::find(members.begin(), members.end(), k) != members.end() ||
                         std::find(round.singles.begin(), round.singles.end(), k) != round.singles.end();
      if (moved && every[k] > 0 && ck->step % every[k] == 0) {
        if (k_obs[k] >= args[k].n_obs) return fail(ck, MFQ_EDEVICE, "observation schedule");
        TileScope tiles(ck);
        mfq_status st = entropy_dev(ck, args[k].region, args[k].n_sites, args[k].S_host + (size_t)k_obs[k] * ck->B);
        if (st) return st;
        ++k_obs[k];
      }
    }
  }
  for (int k = 0; k < n; ++k) {
    mfq_ctx *ck = ctxs[k];
    const hipError_t se = hipStreamSynchronize(ck->stream);
    if (se != hipSuccess) return hip_fail(ck, se, "synchronize");
  }
  mfq_status worst = MFQ_OK;
  for (int k = 0; k < n; ++k) {
    const mfq_status st = check_flag(ctxs[k]);
    if (st && !worst) worst = st;
  }
  return worst;
}

}  // namespace

extern "C" {

mfq_status mfq_create(int device, void *hip_stream, mfq_ctx **out) {
  if (!out) return MFQ_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MFQ_EINVAL;
  mfq_ctx *c = new (std::nothrow) mfq_ctx();
  if (!c) return MFQ_ENOMEM;
  c->device = device;
  if (hipSetDevice(device) != hipSuccess || resolve_scratch(device) != hipSuccess) {
    delete c;
    return MFQ_EDEVICE;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) {
      delete c;
      return MFQ_EDEVICE;
    }
    c->own_stream = true;
  }
  *out = c;
  return MFQ_OK;
}

mfq_status mfq_destroy(mfq_ctx *c) {
  if (!c) return MFQ_OK;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->events) (void)hipEventDestroy(e);
  drop_graph(c);
  if (c->run_S) (void)hipFree(c->run_S);
  if (c->red_buf) (void)hipFree(c->red_buf);
  if (c->rk_buf) (void)hipFree(c->rk_buf);
  if (c->blk_buf) (void)hipFree(c->blk_buf);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return MFQ_OK;
}

const char *mfq_last_error(const mfq_ctx *c) {
  if (!c) return "null context";
  return c->err.c_str();
}

mfq_status mfq_workspace_bytes(const mfq_lattice *lat, int32_t N, int32_t n_traj, int32_t precision,
                               size_t *bytes) {
  if (!lattice_ok(lat) || !bytes || n_traj < 1 || (precision != MFQ_FP64 && precision != MFQ_FP32_BULK))
    return MFQ_EINVAL;
  const int L = lattice_L(lat);
  if (N < 1 || N >= L) return MFQ_EINVAL;
  *bytes = layout_of(*lat, N, n_traj, precision).total + 256;
  return MFQ_OK;
}

mfq_status mfq_init_state(mfq_ctx *c, const mfq_lattice *lat, int32_t N, int32_t n_traj,
                          const uint64_t *traj_uid, const int32_t *occupied, int32_t precision,
                          void *dev_ws, size_t ws_bytes) {
  if (!c) return MFQ_EINVAL;
  c->ready = false;
  if (!lattice_ok(lat)) return fail(c, MFQ_EINVAL, "invalid lattice");
  if (precision != MFQ_FP64 && precision != MFQ_FP32_BULK)
    return fail(c, MFQ_EINVAL, "unsupported precision");
  const int L = lattice_L(lat);
  if (N < 1 || N >= L) return fail(c, MFQ_EINVAL, "need 1 <= N < L");
  if (n_traj < 1 || n_traj > 65535) return fail(c, MFQ_EINVAL, "need 1 <= n_traj <= 65535");
  if (!traj_uid) return fail(c, MFQ_EINVAL, "traj_uid is NULL");
  std::vector<int> occ(N);
  if (occupied) {
    for (int k = 0; k < N; ++k) {
      occ[k] = occupied[k];
      if (occ[k] < 0 || occ[k] >= L || (k > 0 && occ[k] <= occ[k - 1]))
        return fail(c, MFQ_EINVAL, "occupied sites must be ascending and in [0, L)");
    }
  } else {
    if (2 * N != L) return fail(c, MFQ_EINVAL, "default (Neel) state needs N = L/2");
    if (lat->dim == 1 && L % 2) return fail(c, MFQ_EINVAL, "Neel state needs even L");
    if (lat->dim == 2 && (lat->Lx % 2 || lat->Ly % 2))
      return fail(c, MFQ_EINVAL, "checkerboard state needs even Lx and Ly");
    int k = 0;
    for (int i = 0; i < L; ++i) {
      const int x = i % lat->Lx, y = i / lat->Lx;
      if ((x + y) % 2 == 0) occ[k++] = i;
    }
  }
  if (hipSetDevice(c->device) != hipSuccess) return fail(c, MFQ_EDEVICE, "hipSetDevice");
  const WsLayout wl = layout_of(*lat, N, n_traj, precision);
  const size_t need = wl.total + 256;
  if (c->own_ws && c->ws) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->own_ws = false;
  }
  if (dev_ws) {
    if (ws_bytes < need) return fail(c, MFQ_ENOMEM, "workspace too small");
    c->ws = dev_ws;
    c->ws_bytes = ws_bytes;
  } else {
    if (hipMalloc(&c->ws, need) != hipSuccess) {
      c->ws = nullptr;
      return fail(c, MFQ_ENOMEM, "hipMalloc of the workspace failed");
    }
    c->own_ws = true;
    c->ws_bytes = need;
  }
  drop_graph(c);
  carve(reinterpret_cast<char *>(align_up(reinterpret_cast<size_t>(c->ws))), wl, *lat, N, c);
  c->lat = *lat;
  c->L = L; c->N = N; c->B = n_traj; c->precision = precision;
  c->step = 0; c->cur = 0; c->dt_cached = NAN; c->ct_any = false;
  c->gamma_host.assign(n_traj, -1.0);
  HIPCHK(hipMemcpyAsync(c->uid, traj_uid, n_traj * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream),
         "uid upload");
  HIPCHK(hipMemcpyAsync(c->occ, occ.data(), N * sizeof(int), hipMemcpyHostToDevice, c->stream),
         "occupied upload");
  HIPCHK(clear_flag(c), "flag clear");
  HIPCHK(fill_zero(c->step_dev, 256, c->stream), "step counter clear");
  HIPCHK(fill_zero(c->pm_cnt, ((size_t)n_traj * sizeof(int) + 7) / 8 * 8, c->stream), "event clear");
  HIPCHK(fill_zero(c->step_base, (size_t)n_traj * sizeof(int64_t), c->stream), "step base clear");
  HIPCHK(cont_clock_set(c->ct.t, 0, n_traj, 0.0, c->stream), "clock clear");
  HIPCHK(fill_zero(c->ct.info, (size_t)4 * n_traj * sizeof(int), c->stream), "event record clear");
  HIPCHK(init_state(c->X[0], L, N, n_traj, c->occ, c->stream), "init_state");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  c->ready = true;
  return MFQ_OK;
}

mfq_status mfq_step(mfq_ctx *c, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                    int32_t n_steps) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  mfq_status sv = validate_step(c, protocol, gamma, dt, n_steps);
  if (sv) return sv;
  if (n_steps == 0) return MFQ_OK;
  mfq_status st0 = prepare_step(c, gamma, dt);
  if (st0) return st0;
  if (protocol == MFQ_HOMODYNE && c->integrator == MFQ_INTEGRATOR_RK4 && (st0 = ensure_rk4(c))) return st0;
  HIPCHK(set_step(c->step_dev, c->step, false, c->stream), "step counter");
  int done = 0;
  const bool capturable = !(protocol == MFQ_PROJECTIVE && blocked_pm(c));
  if (c->use_graphs && !c->profiling && n_steps >= 2 && capturable) {
    mfq_status st = ensure_step_graph(c, protocol, dt, seed);
    if (st) return st;
    for (; done + 2 <= n_steps; done += 2) HIPCHK(hipGraphLaunch(c->gexec, c->stream), "graph launch");
  }
  for (; done < n_steps; ++done) {
    mfq_status st = enqueue_step(c, protocol, dt, seed, 1);
    if (st) return st;
    HIPCHK(set_step(c->step_dev, 1, true, c->stream), "step counter");
  }
  c->step += n_steps;
  return MFQ_OK;
}

// Scratch of the deferred events (per trajectory WL, WR, Zc, G, T1 and the block clock),
// allocated on first use; the block clocks start at zero.
mfq_status ensure_blk(mfq_ctx *c) {
  const long K = c->ct_block, L = c->L, N = c->N, B = c->B;
  const size_t cpl = align_up((size_t)(5 * N * K + 3 * L * K) * B * sizeof(cplx));
  const size_t need = cpl + (size_t)B * sizeof(double) + (size_t)2 * B * sizeof(int);
  if (c->blk_cap < need) {
    if (c->blk_buf) {
      HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
      (void)hipFree(c->blk_buf);
      c->blk_buf = nullptr;
      c->blk_cap = 0;
    }
    if (hipMalloc(&c->blk_buf, need) != hipSuccess) {
      c->blk_buf = nullptr;
      return fail(c, MFQ_ENOMEM, "hipMalloc of the deferred-event scratch failed");
    }
    c->blk_cap = need;
  }
  cplx *p = reinterpret_cast<cplx *>(c->blk_buf);
  c->bw.WL = p; p += 2 * N * K * B;
  c->bw.WR = p; p += 2 * N * K * B;
  c->bw.Zc = p; p += N * K * B;
  c->bw.G = p; p += L * K * B;
  c->bw.T1 = p;
  c->bw.s = reinterpret_cast<double *>(reinterpret_cast<char *>(c->blk_buf) + cpl);
  c->bw.fb = reinterpret_cast<int *>(c->bw.s + B);
  c->bw.K = (int)K;
  HIPCHK(fill_zero(c->bw.s, (size_t)B * sizeof(double), c->stream), "block clock clear");
  return MFQ_OK;
}

mfq_status mfq_ct_events(mfq_ctx *c, const double *gamma, uint64_t seed, int32_t n_events, double t_end,
                         int32_t reorth_every) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!gamma) return fail(c, MFQ_EINVAL, "gamma is NULL");
  for (int b = 0; b < c->B; ++b)
    if (!(gamma[b] > 0.0) || !std::isfinite(gamma[b]))
      return fail(c, MFQ_EINVAL, "gamma must be positive and finite");
  if (n_events < 0) return fail(c, MFQ_EINVAL, "n_events < 0");
  if (std::isnan(t_end)) return fail(c, MFQ_EINVAL, "t_end is NaN");
  if (reorth_every < 0) return fail(c, MFQ_EINVAL, "reorth_every < 0");
  if (n_events == 0) return MFQ_OK;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  if (std::memcmp(c->gamma_host.data(), gamma, c->B * sizeof(double)) != 0) {
    std::memcpy(c->gamma_host.data(), gamma, c->B * sizeof(double));
    HIPCHK(hipMemcpyAsync(c->gamma, c->gamma_host.data(), c->B * sizeof(double), hipMemcpyHostToDevice,
                          c->stream), "gamma upload");
  }
  HIPCHK(set_step(c->step_dev, c->step, false, c->stream), "step counter");
  const int Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
  if (c->ct_block > 0) {  // deferred events, flushed every ct_block slots
    mfq_status st = ensure_blk(c);
    if (st) return st;
    int e = 0;
    for (int slot = 0; slot < n_events; ++slot) {
      {
        PhaseTimer t(c, MFQ_PHASE_MEASURE);
        HIPCHK(cont_block_event(c->X[c->cur], c->L, c->N, c->B, e, c->lat.dim, c->lat.Lx, Ly, c->lat.J, c->gamma,
                                t_end, seed, c->uid, c->step_dev, 1, c->step_base, c->ct, c->bw, c->stream),
               "deferred event");
      }
      ++e;
      HIPCHK(set_step(c->step_dev, 1, true, c->stream), "step counter");
      c->step += 1;
      c->ct_any = true;
      const bool reorth = reorth_every > 0 && c->step % reorth_every == 0;
      if (e == c->ct_block || slot + 1 == n_events || reorth) {
        bool in_b = false;
        {
          PhaseTimer t(c, MFQ_PHASE_PROPAGATE);
          HIPCHK(cont_block_flush(c->X[c->cur], c->X[1 - c->cur], c->L, c->N, c->B, e, c->lat.dim, c->lat.Lx, Ly,
                                  c->lat.J, c->ct, c->bw, &in_b, c->stream), "deferred events flush");
        }
        if (in_b) c->cur = 1 - c->cur;
        e = 0;
      }
      if (reorth) {
        PhaseTimer t(c, MFQ_PHASE_REORTH);
        HIPCHK(cholqr2(c->X[c->cur], c->X[1 - c->cur], c->L, c->N, c->B, c->chol, c->stream), "cholqr2");
        c->cur = 1 - c->cur;
      }
    }
    return MFQ_OK;
  }
  for (int e = 0; e < n_events; ++e) {
    bool in_b = false;
    {
      PhaseTimer t(c, MFQ_PHASE_MEASURE);
      HIPCHK(cont_event(c->X[c->cur], c->X[1 - c->cur], c->L, c->N, c->B, c->lat.dim, c->lat.Lx, Ly,
                        c->lat.J, c->gamma, t_end, seed, c->uid, c->step_dev, 1, c->step_base, c->ct,
                        &in_b, c->stream), "continuous-time event");
    }
    if (in_b) c->cur = 1 - c->cur;
    HIPCHK(set_step(c->step_dev, 1, true, c->stream), "step counter");
    c->step += 1;
    c->ct_any = true;
    if (reorth_every > 0 && c->step % reorth_every == 0) {
      PhaseTimer t(c, MFQ_PHASE_REORTH);
      HIPCHK(cholqr2(c->X[c->cur], c->X[1 - c->cur], c->L, c->N, c->B, c->chol, c->stream), "cholqr2");
      c->cur = 1 - c->cur;
    }
  }
  return MFQ_OK;
}

mfq_status mfq_ct_last_events(mfq_ctx *c, int32_t *site, int32_t *outcome, double *prob, double *tau) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int B = c->B;
  std::vector<int> info((size_t)4 * B);
  std::vector<double> dinfo((size_t)4 * B);
  if (c->ct_any) {
    HIPCHK(hipMemcpyAsync(info.data(), c->ct.info, info.size() * sizeof(int), hipMemcpyDeviceToHost,
                          c->stream), "event record download");
    HIPCHK(hipMemcpyAsync(dinfo.data(), c->ct.dinfo, dinfo.size() * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream), "event record download");
    HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  }
  for (int b = 0; b < B; ++b) {
    const bool ev = c->ct_any && info[4 * b + 2] >= 0;
    if (site) site[b] = ev ? info[4 * b] : -1;
    if (outcome) outcome[b] = ev ? info[4 * b + 1] : -1;
    if (prob) prob[b] = ev ? dinfo[4 * b + 1] : 0.0;
    if (tau) tau[b] = ev ? dinfo[4 * b] : 0.0;
  }
  return check_flag(c);
}

mfq_status mfq_get_times(mfq_ctx *c, double *t_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!t_host) return fail(c, MFQ_EINVAL, "t_host is NULL");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(t_host, c->ct.t, c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream),
         "clock download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

mfq_status mfq_set_times(mfq_ctx *c, const double *t_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!t_host) return fail(c, MFQ_EINVAL, "t_host is NULL");
  for (int b = 0; b < c->B; ++b)
    if (!std::isfinite(t_host[b])) return fail(c, MFQ_EINVAL, "clock values must be finite");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(c->ct.t, t_host, c->B * sizeof(double), hipMemcpyHostToDevice, c->stream),
         "clock upload");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return MFQ_OK;
}

mfq_status mfq_set_ct_block(mfq_ctx *c, int32_t block) {
  if (!c) return MFQ_EINVAL;
  if (block < 0 || block > 64) return fail(c, MFQ_EINVAL, "block length must be in 0 .. 64");
  c->ct_block = block;
  return MFQ_OK;
}

mfq_status mfq_set_integrator(mfq_ctx *c, int32_t integrator) {
  if (!c) return MFQ_EINVAL;
  if (integrator != MFQ_INTEGRATOR_SPLIT && integrator != MFQ_INTEGRATOR_RK4)
    return fail(c, MFQ_EINVAL, "unknown integrator");
  c->integrator = integrator;
  drop_graph(c);
  return MFQ_OK;
}

mfq_status mfq_run_group(mfq_ctx *const *ctxs, mfq_run_args *args, int32_t n) {
  if (!ctxs || !args || n < 1) return MFQ_EINVAL;
  if (n > FUSED_GROUP_MAX) return fail(ctxs[0], MFQ_EINVAL, "too many contexts for one launch");
  bool all_fused = true;
  for (int k = 0; k < n; ++k) {
    mfq_ctx *c = ctxs[k];
    if (!c) return MFQ_EINVAL;
    for (int q = 0; q < k; ++q)
      if (ctxs[q] == c) return fail(c, MFQ_EINVAL, "a context appears twice");
    if (c->device != ctxs[0]->device) return fail(c, MFQ_EINVAL, "contexts on different devices");
    const mfq_run_args &r = args[k];
    mfq_status st = validate_step(c, r.protocol, r.gamma, r.dt, r.n_steps);
    if (st) return st;
    if (r.obs_every < 0) return fail(c, MFQ_EINVAL, "obs_every < 0");
    if (r.obs_every > 0 && (st = validate_region(c, r.region, r.n_sites))) return st;
    const int Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
    if (!fused_fits(c->L, c->N, c->lat.Lx, Ly) || (r.protocol == MFQ_HOMODYNE && c->integrator == MFQ_INTEGRATOR_RK4))
      all_fused = false;
    const int n_obs = r.obs_every > 0 ? (int)((c->step + r.n_steps) / r.obs_every - c->step / r.obs_every) : 0;
    if (n_obs > 0 && !r.S_host) return fail(c, MFQ_EINVAL, "S_host is NULL");
    args[k].n_obs = n_obs;
  }
  if (!all_fused) {
    for (int k = 0; k < n; ++k) {
      mfq_ctx *c = ctxs[k];
      if (args[k].protocol == MFQ_PROJECTIVE && blocked_pm(c))
        return fail(c, MFQ_EINVAL, "blocked projective steps synchronise and cannot join a group graph");
      if (!c->use_graphs || c->profiling)
        return fail(c, MFQ_EINVAL, "graphs are disabled or profiling is on for this context");
    }
    return run_group_graph(ctxs, args, n);
  }
  mfq_ctx *c0 = ctxs[0];
  FusedGroup grp{};
  grp.n = n;
  grp.first[0] = 0;
  for (int k = 0; k < n; ++k) {
    mfq_ctx *c = ctxs[k];
    const mfq_run_args &r = args[k];
    mfq_status st = prepare_step(c, r.gamma, r.dt);
    if (st) return st;
    const size_t need = (size_t)std::max(r.n_obs, 1) * c->B;
    if (need > c->run_S_cap) {
      HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
      if (c->run_S) (void)hipFree(c->run_S);
      c->run_S = nullptr;
      c->run_S_cap = 0;
      HIPCHK(hipMalloc(&c->run_S, need * sizeof(double)), "observation buffer");
      c->run_S_cap = need;
    }
    if (r.obs_every > 0 && r.n_sites > 0)
      HIPCHK(hipMemcpyAsync(c->region, r.region, r.n_sites * sizeof(int), hipMemcpyHostToDevice, c->stream),
             "region upload");
    FusedArgs &a = grp.g[k];
    a.P = c->P; a.U = c->X[c->cur]; a.L = c->L; a.N = c->N;
    a.gx = c->gx; a.gy = c->gy; a.Lx = c->lat.Lx; a.Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
    a.gamma = c->gamma; a.dt = r.dt; a.seed = r.seed; a.uid = c->uid; a.step_base = c->step_base;
    a.step0 = c->step; a.n_steps = r.n_steps; a.protocol = r.protocol;
    a.obs_every = r.obs_every; a.region = c->region; a.nreg = r.obs_every > 0 ? r.n_sites : 0;
    a.max_obs = r.n_obs; a.S_out = c->run_S;
    a.ev_sites = c->pm_sites; a.ev_out = c->pm_out; a.ev_cnt = c->pm_cnt; a.ev_prob = c->pm_prob;
    a.flag = c->flag;
    a.info = c->info;
    a.B = c->B;
    grp.first[k + 1] = grp.first[k] + c->B;
  }
  // the launch goes on the first context's stream, ordered after the work already queued on
  // the others' streams, and theirs after it
  std::vector<hipEvent_t> evs;
  auto cleanup = [&]() {
    for (hipEvent_t ev : evs) (void)hipEventDestroy(ev);
  };
  for (int k = 1; k < n; ++k) {
    if (ctxs[k]->stream == c0->stream) continue;
    hipEvent_t ev;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return fail(c0, MFQ_EDEVICE, "event create");
    }
    evs.push_back(ev);
    if (hipEventRecord(ev, ctxs[k]->stream) != hipSuccess || hipStreamWaitEvent(c0->stream, ev, 0) != hipSuccess) {
      cleanup();
      return fail(c0, MFQ_EDEVICE, "stream ordering");
    }
  }
  hipError_t le = fused_run_group(grp, c0->stream);
  if (le != hipSuccess) {
    cleanup();
    return hip_fail(c0, le, "fused group kernel");
  }
  for (int k = 0; k < n; ++k) {
    mfq_ctx *c = ctxs[k];
    if (args[k].n_obs > 0 &&
        hipMemcpyAsync(args[k].S_host, c->run_S, (size_t)args[k].n_obs * c->B * sizeof(double),
                       hipMemcpyDeviceToHost, c0->stream) != hipSuccess) {
      cleanup();
      return fail(c, MFQ_EDEVICE, "observation download");
    }
  }
  const hipError_t se = hipStreamSynchronize(c0->stream);
  cleanup();
  if (se != hipSuccess) return hip_fail(c0, se, "synchronize");
  mfq_status worst = MFQ_OK;
  for (int k = 0; k < n; ++k) {
    ctxs[k]->step += args[k].n_steps;
    const mfq_status st = check_flag(ctxs[k]);
    if (st && !worst) worst = st;
  }
  return worst;
}

mfq_status mfq_set_propagator(mfq_ctx *c, int32_t form) {
  if (!c) return MFQ_EINVAL;
  if (form != MFQ_PROP_DENSE && form != MFQ_PROP_FACTORED)
    return fail(c, MFQ_EINVAL, "unknown propagator form");
  c->prop_form = form;
  drop_graph(c);
  return MFQ_OK;
}

mfq_status mfq_propagator_band(mfq_ctx *c, int32_t *band) {
  if (!c || !band) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  *band = c->lat.dim == 1 ? c->band_w : -2;
  return MFQ_OK;
}

mfq_status mfq_set_pm_path(mfq_ctx *c, int32_t path) {
  if (!c) return MFQ_EINVAL;
  if (path != MFQ_PM_AUTO && path != MFQ_PM_WORKGROUP && path != MFQ_PM_BLOCKED)
    return fail(c, MFQ_EINVAL, "unknown projective-measurement path");
  c->pm_path = path;
  return MFQ_OK;
}

mfq_status mfq_set_eig_path(mfq_ctx *c, int32_t path) {
  if (!c) return MFQ_EINVAL;
  if (path != MFQ_EIG_AUTO && path != MFQ_EIG_ONE_STAGE && path != MFQ_EIG_TWO_STAGE)
    return fail(c, MFQ_EINVAL, "unknown reduction form");
  c->eig_mode = path;
  return MFQ_OK;
}

mfq_status mfq_set_path(mfq_ctx *c, int32_t path) {
  if (!c) return MFQ_EINVAL;
  if (path != MFQ_PATH_AUTO && path != MFQ_PATH_FUSED && path != MFQ_PATH_LAUNCHES)
    return fail(c, MFQ_EINVAL, "unknown path");
  c->run_path = path;
  return MFQ_OK;
}

mfq_status mfq_run(mfq_ctx *c, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                   int32_t n_steps, int32_t obs_every, const int32_t *region, int32_t n_sites,
                   double *S_host, int32_t *n_obs_out) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  mfq_status st = validate_step(c, protocol, gamma, dt, n_steps);
  if (st) return st;
  if (obs_every < 0) return fail(c, MFQ_EINVAL, "obs_every < 0");
  if (obs_every > 0) {
    if ((st = validate_region(c, region, n_sites))) return st;
  }
  int n_obs = 0;
  if (obs_every > 0)
    n_obs = (int)((c->step + n_steps) / obs_every - c->step / obs_every);
  if (n_obs > 0 && !S_host) return fail(c, MFQ_EINVAL, "S_host is NULL");
  if (n_obs_out) *n_obs_out = n_obs;
  if (n_steps == 0) return MFQ_OK;
  const int Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
  const bool fits = fused_fits(c->L, c->N, c->lat.Lx, Ly) &&
                    !(protocol == MFQ_HOMODYNE && c->integrator == MFQ_INTEGRATOR_RK4);
  if (c->run_path == MFQ_PATH_FUSED && !fits)
    return fail(c, MFQ_EINVAL, "problem does not fit the fused path (LDS)");
  const bool fused = c->run_path == MFQ_PATH_FUSED || (c->run_path == MFQ_PATH_AUTO && fits);
  if (!fused) {
    int done = 0, k = 0;
    while (done < n_steps) {
      int chunk = n_steps - done;
      if (obs_every > 0) chunk = std::min<int64_t>(chunk, obs_every - c->step % obs_every);
      if ((st = mfq_step(c, protocol, gamma, dt, seed, chunk))) return st;
      done += chunk;
      if (obs_every > 0 && c->step % obs_every == 0) {
        if ((st = entropy_dev(c, region, n_sites, S_host + (size_t)k * c->B))) return st;
        ++k;
      }
    }
    return check_flag(c);
  }
  if ((st = prepare_step(c, gamma, dt))) return st;
  const size_t need = (size_t)std::max(n_obs, 1) * c->B;
  if (need > c->run_S_cap) {
    if (c->run_S) (void)hipFree(c->run_S);
    c->run_S = nullptr;
    c->run_S_cap = 0;
    HIPCHK(hipMalloc(&c->run_S, need * sizeof(double)), "observation buffer");
    c->run_S_cap = need;
  }
  if (obs_every > 0 && n_sites > 0)
    HIPCHK(hipMemcpyAsync(c->region, region, n_sites * sizeof(int), hipMemcpyHostToDevice, c->stream),
           "region upload");
  FusedArgs a{};
  a.P = c->P; a.U = c->X[c->cur]; a.L = c->L; a.N = c->N;
  a.gx = c->gx; a.gy = c->gy; a.Lx = c->lat.Lx; a.Ly = Ly;
  a.gamma = c->gamma; a.dt = dt; a.seed = seed; a.uid = c->uid; a.step_base = c->step_base;
  a.step0 = c->step; a.n_steps = n_steps; a.protocol = protocol;
  a.obs_every = obs_every; a.region = c->region; a.nreg = obs_every > 0 ? n_sites : 0;
  a.max_obs = n_obs; a.S_out = c->run_S;
  a.ev_sites = c->pm_sites; a.ev_out = c->pm_out; a.ev_cnt = c->pm_cnt; a.ev_prob = c->pm_prob;
  a.flag = c->flag;
  a.info = c->info;
  a.B = c->B;
  {
    PhaseTimer t(c, MFQ_PHASE_PROPAGATE);
    HIPCHK(fused_run(a, c->B, c->stream), "fused trajectory kernel");
  }
  if (n_obs > 0)
    HIPCHK(hipMemcpyAsync(S_host, c->run_S, (size_t)n_obs * c->B * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream), "observation download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  c->step += n_steps;
  return check_flag(c);
}

namespace {

mfq_status ensure_red(mfq_ctx *c, size_t n) {
  if (n <= c->red_cap) return MFQ_OK;
  if (c->red_buf) (void)hipFree(c->red_buf);
  c->red_buf = nullptr;
  c->red_cap = 0;
  if (hipMalloc(&c->red_buf, n * sizeof(double)) != hipSuccess)
    return fail(c, MFQ_ENOMEM, "correlation buffer");
  c->red_cap = n;
  return MFQ_OK;
}

}  // namespace

namespace {

// C(r) of every trajectory with its tile partials and bins in `buf` (cap doubles; null: the
// context's buffer, grown on demand).
mfq_status density_correlation(mfq_ctx *c, double *Cr_host, double *buf, size_t cap) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!Cr_host) return fail(c, MFQ_EINVAL, "Cr_host is NULL");
  if (c->lat.dim != 1) return fail(c, MFQ_EINVAL, "C(r) is defined for 1d rings");
  TileScope tiles(c);
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int L = c->L, half = L / 2;
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.M = L; g.N = L; g.K = c->N; g.batch = c->B;
  g.A = c->X[c->cur]; g.lda = L; g.sA = (long)L * c->N; g.opA = OP_N;
  g.B = c->X[c->cur]; g.ldb = L; g.sB = (long)L * c->N; g.opB = OP_C;
  g.tri = TRI_UPPER;
  const size_t np = zgemm_partials(g), nout = (size_t)half * c->B;
  if (buf) {
    if (np + nout > cap)
      return fail(c, MFQ_ENOMEM, "C(r) needs " + std::to_string((np + nout) * sizeof(double)) +
                                     " bytes of partials and bins, above the static buffer's " +
                                     std::to_string(cap * sizeof(double)));
  } else {
    mfq_status st = ensure_red(c, np + nout);
    if (st) return st;
    buf = c->red_buf;
  }
  g.part = buf;
  {
    PhaseTimer t(c, MFQ_PHASE_OBSERVE);
    HIPCHK(zgemm_ring_bins(g, L, buf + np, c->stream), "density correlation");
  }
  HIPCHK(hipMemcpyAsync(Cr_host, buf + np, nout * sizeof(double), hipMemcpyDeviceToHost, c->stream),
         "C(r) download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

}  // namespace

mfq_status mfq_density_correlation(mfq_ctx *c, double *Cr_host) {
  return density_correlation(c, Cr_host, nullptr, 0);
}

mfq_status mfq_density_correlation_noalloc(mfq_ctx *c, double *Cr_host) {
  if (!c) return MFQ_EINVAL;
  double *buf = scratch_of(c->device);
  if (!buf) return fail(c, MFQ_EDEVICE, "static buffer of this device not resolved");
  return density_correlation(c, Cr_host, buf, MFQ_NOALLOC_SCRATCH_BYTES / sizeof(double));
}

mfq_status mfq_particle_covariance(mfq_ctx *c, const int32_t *A, int32_t nA, const int32_t *B, int32_t nB,
                                   double *G_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!G_host) return fail(c, MFQ_EINVAL, "G_host is NULL");
  mfq_status st = validate_region(c, A, nA);
  if (st) return st;
  if ((st = validate_region(c, B, nB))) return st;
  for (int i = 0, j = 0; i < nA && j < nB;) {  // both ascending: disjoint iff no common entry
    if (A[i] == B[j]) return fail(c, MFQ_EINVAL, "regions A and B must be disjoint");
    if (A[i] < B[j]) ++i;
    else ++j;
  }
  if (nA == 0 || nB == 0) {
    for (int b = 0; b < c->B; ++b) G_host[b] = 0.0;
    return MFQ_OK;
  }
  TileScope tiles(c);
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(c->region, A, nA * sizeof(int), hipMemcpyHostToDevice, c->stream), "region upload");
  HIPCHK(hipMemcpyAsync(c->region + nA, B, nB * sizeof(int), hipMemcpyHostToDevice, c->stream),
         "region upload");
  const int L = c->L;
  GemmDesc g{};
  g.alpha = cplx{1.0, 0.0};
  g.M = nA; g.N = nB; g.K = c->N; g.batch = c->B;
  g.A = c->X[c->cur]; g.lda = L; g.sA = (long)L * c->N; g.opA = OP_N; g.idxA = c->region;
  g.B = c->X[c->cur]; g.ldb = L; g.sB = (long)L * c->N; g.opB = OP_C; g.idxB = c->region + nA;
  const size_t np = zgemm_partials(g);
  if ((st = ensure_red(c, np + c->B))) return st;
  g.part = c->red_buf;
  {
    PhaseTimer t(c, MFQ_PHASE_OBSERVE);
    HIPCHK(zgemm_tile_sum(g, c->red_buf + np, c->stream), "particle covariance");
  }
  HIPCHK(hipMemcpyAsync(G_host, c->red_buf + np, c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream),
         "G_AB download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

mfq_status mfq_set_tuning(mfq_ctx *c, int32_t path, int32_t tile) {
  if (!c) return MFQ_EINVAL;
  if (path != MFQ_PATH_AUTO && path != MFQ_PATH_FUSED && path != MFQ_PATH_LAUNCHES)
    return fail(c, MFQ_EINVAL, "unknown path");
  if (tile != MFQ_TILE_AUTO && tile != MFQ_TILE_SMALL && tile != MFQ_TILE_LARGE)
    return fail(c, MFQ_EINVAL, "unknown tile choice");
  c->run_path = path;
  c->tile_mode = tile;
  drop_graph(c);
  return MFQ_OK;
}

mfq_status mfq_set_tile_order(mfq_ctx *c, int32_t order) {
  if (!c) return MFQ_EINVAL;
  if (order != MFQ_ORDER_XCD && order != MFQ_ORDER_LINEAR) return fail(c, MFQ_EINVAL, "unknown tile order");
  c->tile_order = order;
  drop_graph(c);
  return MFQ_OK;
}

mfq_status mfq_autotune(mfq_ctx *c, int32_t protocol, const double *gamma, double dt, uint64_t seed,
                        int32_t probe_steps, mfq_tuning *out) {
  if (!c) return MFQ_EINVAL;
  if (!out) return fail(c, MFQ_EINVAL, "out is NULL");
  mfq_status st = validate_step(c, protocol, gamma, dt, probe_steps);
  if (st) return st;
  if (probe_steps < 1 || probe_steps > 1000) return fail(c, MFQ_EINVAL, "need 1 <= probe_steps <= 1000");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  // the state and the events of the last step are saved and restored around the probes
  const size_t ubytes = (size_t)c->L * c->N * c->B * sizeof(cplx);
  const size_t ev = (size_t)c->L * c->B;
  const size_t ebytes = ev * (2 * sizeof(int) + sizeof(double)) + c->B * sizeof(int);
  char *save = nullptr;
  HIPCHK(hipMalloc(&save, ubytes + ebytes), "autotune save buffer");
  auto copy_events = [&](bool to_save) -> hipError_t {
    char *p = save + ubytes;
    struct Piece { void *dev; size_t n; } pieces[4] = {{c->pm_sites, ev * sizeof(int)},
                                                        {c->pm_out, ev * sizeof(int)},
                                                        {c->pm_prob, ev * sizeof(double)},
                                                        {c->pm_cnt, c->B * sizeof(int)}};
    for (const Piece &q : pieces) {
      hipError_t e = to_save ? hipMemcpyAsync(p, q.dev, q.n, hipMemcpyDeviceToDevice, c->stream)
                             : hipMemcpyAsync(q.dev, p, q.n, hipMemcpyDeviceToDevice, c->stream);
      if (e != hipSuccess) return e;
      p += q.n;
    }
    return hipSuccess;
  };
  const int cur0 = c->cur;
  const int64_t step0 = c->step;
  hipError_t he = hipMemcpyAsync(save, c->X[cur0], ubytes, hipMemcpyDeviceToDevice, c->stream);
  if (he == hipSuccess) he = copy_events(true);
  auto restore = [&]() -> hipError_t {
    c->cur = cur0;
    c->step = step0;
    hipError_t e = hipMemcpyAsync(c->X[cur0], save, ubytes, hipMemcpyDeviceToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return e;
  };
  // Candidates, searched coordinate by coordinate: the projective measurement form first (when
  // both apply), then GEMM tile size x tile order with that form, then the fused kernel.
  struct Cand { int path, tile, order, pm; };
  const int path0 = c->run_path, tile0 = c->tile_mode, order0 = c->tile_order, pm0 = c->pm_path;
  std::memset(out, 0, sizeof(*out));
  int n = 0;
  double best_ms = 0.0;
  Cand best{path0, tile0, order0, pm0};
  bool have_best = false;
  auto probe = [&](const Cand &k) {
    if (he != hipSuccess || st != MFQ_OK || n >= MFQ_TUNE_MAX_CANDIDATES) return;
    c->run_path = k.path;
    c->tile_mode = k.tile;
    c->tile_order = k.order;
    c->pm_path = k.pm;
    double ms = 0.0;
    for (int rep = 0; rep < 2 && he == hipSuccess && st == MFQ_OK; ++rep) {  // warm-up, then timed
      if ((he = restore()) != hipSuccess) break;
      int32_t n_obs = 0;
      const auto t0 = std::chrono::steady_clock::now();
      st = mfq_run(c, protocol, gamma, dt, seed, probe_steps, 0, nullptr, 0, nullptr, &n_obs);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      // a warm-up ten times slower than the best so far is not worth a timed run
      if (rep == 0 && have_best && ms > 10.0 * best_ms) break;
    }
    out->candidate_ms[n] = ms / probe_steps;
    out->cand_path[n] = k.path;
    out->cand_tile[n] = k.tile;
    out->cand_order[n] = k.order;
    out->cand_pm[n] = k.pm;
    ++n;
    if (st == MFQ_OK && (!have_best || ms < best_ms)) {
      best = k;
      best_ms = ms;
      have_best = true;
    }
  };
  int pm = pm0;
  if (protocol == MFQ_PROJECTIVE && c->N >= PM_BLOCKED_MIN_N) {
    probe({MFQ_PATH_LAUNCHES, MFQ_TILE_AUTO, MFQ_ORDER_XCD, MFQ_PM_BLOCKED});
    probe({MFQ_PATH_LAUNCHES, MFQ_TILE_AUTO, MFQ_ORDER_XCD, MFQ_PM_WORKGROUP});
    pm = best.pm;
  }
  for (int tile : {MFQ_TILE_AUTO, MFQ_TILE_SMALL, MFQ_TILE_LARGE})
    for (int order : {MFQ_ORDER_XCD, MFQ_ORDER_LINEAR}) {
      const Cand k{MFQ_PATH_LAUNCHES, tile, order, pm};
      bool seen = false;
      for (int i = 0; i < n; ++i)
        seen = seen || (out->cand_path[i] == k.path && out->cand_tile[i] == k.tile &&
                        out->cand_order[i] == k.order && out->cand_pm[i] == k.pm);
      if (!seen) probe(k);
    }
  const int Ly = c->lat.dim == 2 ? c->lat.Ly : 1;
  if (fused_fits(c->L, c->N, c->lat.Lx, Ly) && !(protocol == MFQ_HOMODYNE && c->integrator == MFQ_INTEGRATOR_RK4))
    probe({MFQ_PATH_FUSED, MFQ_TILE_AUTO, MFQ_ORDER_XCD, pm});
  out->n_candidates = n;
  const std::string probe_err = c->err;
  if (he == hipSuccess) he = restore();
  if (he == hipSuccess) he = copy_events(false);
  if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
  (void)hipFree(save);
  drop_graph(c);
  auto keep_previous = [&]() {
    c->run_path = path0;
    c->tile_mode = tile0;
    c->tile_order = order0;
    c->pm_path = pm0;
  };
  if (he != hipSuccess) {
    keep_previous();
    return hip_fail(c, he, "autotune");
  }
  if (st != MFQ_OK || !have_best) {
    keep_previous();
    return fail(c, st ? st : MFQ_EDEVICE, "autotune probe failed: " + probe_err);
  }
  c->run_path = best.path;
  c->tile_mode = best.tile;
  c->tile_order = best.order;
  c->pm_path = best.pm;
  out->path = best.path;
  out->tile = best.tile;
  out->order = best.order;
  out->pm_path = best.pm;
  out->ms_per_step = best_ms / probe_steps;
  return MFQ_OK;
}

mfq_status mfq_reset_trajectory(mfq_ctx *c, int32_t slot, uint64_t uid) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (slot < 0 || slot >= c->B) return fail(c, MFQ_EINVAL, "slot out of range");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(reset_slot(c->X[c->cur], c->L, c->N, slot, c->occ, c->uid, uid, c->step_base, c->step, c->stream),
         "reset slot");
  HIPCHK(cont_clock_set(c->ct.t, slot, 1, 0.0, c->stream), "clock reset");
  return MFQ_OK;
}

mfq_status mfq_use_graphs(mfq_ctx *c, int32_t enable) {
  if (!c) return MFQ_EINVAL;
  c->use_graphs = enable != 0;
  if (!c->use_graphs) drop_graph(c);
  return MFQ_OK;
}

mfq_status mfq_entropy(mfq_ctx *c, const int32_t *region, int32_t n_sites, double *S_host) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!S_host) return fail(c, MFQ_EINVAL, "S_host is NULL");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  mfq_status st = entropy_dev(c, region, n_sites, S_host);
  if (st) return st;
  return check_flag(c);
}

mfq_status mfq_region_spectrum(mfq_ctx *c, const int32_t *region, int32_t n_sites, double *lam_host) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!lam_host) return fail(c, MFQ_EINVAL, "lam_host is NULL");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  int m = 0;
  mfq_status st = region_spectrum_dev(c, region, n_sites, &m);
  if (st) return st;
  if (m > 0)
    HIPCHK(hipMemcpyAsync(lam_host, c->eig.lam, (size_t)m * c->B * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream), "spectrum download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

mfq_status mfq_mutual_info(mfq_ctx *c, const int32_t *A, int32_t nA, const int32_t *B, int32_t nB,
                           double *I_host) {
  if (!c) return MFQ_EINVAL;
  TileScope tiles(c);
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!I_host) return fail(c, MFQ_EINVAL, "I_host is NULL");
  mfq_status st = validate_region(c, A, nA);
  if (st) return st;
  if ((st = validate_region(c, B, nB))) return st;
  std::vector<int32_t> AB;
  AB.reserve(nA + nB);
  int i = 0, j = 0;
  while (i < nA || j < nB) {
    if (j >= nB || (i < nA && A[i] < B[j])) AB.push_back(A[i++]);
    else if (i >= nA || B[j] < A[i]) AB.push_back(B[j++]);
    else return fail(c, MFQ_EINVAL, "regions A and B overlap");
  }
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  std::vector<double> sa(c->B), sb(c->B), sab(c->B);
  if ((st = entropy_dev(c, A, nA, sa.data()))) return st;
  if ((st = entropy_dev(c, B, nB, sb.data()))) return st;
  if ((st = entropy_dev(c, AB.data(), (int32_t)AB.size(), sab.data()))) return st;
  for (int b = 0; b < c->B; ++b) I_host[b] = sa[b] + sb[b] - sab[b];
  return check_flag(c);
}

mfq_status mfq_occupations(mfq_ctx *c, double *p_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!p_host) return fail(c, MFQ_EINVAL, "p_host is NULL");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(born_only(c->X[c->cur], c->p, c->L, c->N, c->B, c->stream), "born");
  HIPCHK(hipMemcpyAsync(p_host, c->p, (size_t)c->L * c->B * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream), "occupations download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

mfq_status mfq_pm_events(mfq_ctx *c, int32_t max_events, int32_t *counts, int32_t *sites,
                         int32_t *outcomes, double *probs) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (max_events < 0 || !counts) return fail(c, MFQ_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  const int L = c->L, B = c->B;
  std::vector<int> cnt(B), st(max_events > 0 ? (size_t)L * B : 0), oc(st.size());
  std::vector<double> pr(st.size());
  HIPCHK(hipMemcpyAsync(cnt.data(), c->pm_cnt, B * sizeof(int), hipMemcpyDeviceToHost, c->stream), "events");
  if (max_events > 0) {
    HIPCHK(hipMemcpyAsync(st.data(), c->pm_sites, st.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream), "events");
    HIPCHK(hipMemcpyAsync(oc.data(), c->pm_out, oc.size() * sizeof(int), hipMemcpyDeviceToHost, c->stream), "events");
    HIPCHK(hipMemcpyAsync(pr.data(), c->pm_prob, pr.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream), "events");
  }
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  for (int b = 0; b < B; ++b) {
    counts[b] = cnt[b];
    const int m = std::min(cnt[b], max_events);
    for (int e = 0; e < m; ++e) {
      if (sites) sites[(size_t)b * max_events + e] = st[(size_t)b * L + e];
      if (outcomes) outcomes[(size_t)b * max_events + e] = oc[(size_t)b * L + e];
      if (probs) probs[(size_t)b * max_events + e] = pr[(size_t)b * L + e];
    }
  }
  return MFQ_OK;
}

mfq_status mfq_get_state(mfq_ctx *c, void *U_host, int64_t *step) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  if (U_host)
    HIPCHK(hipMemcpyAsync(U_host, c->X[c->cur], (size_t)c->L * c->N * c->B * sizeof(cplx),
                          hipMemcpyDeviceToHost, c->stream), "state download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  if (step) *step = c->step;
  return check_flag(c);
}

mfq_status mfq_set_state(mfq_ctx *c, const void *U_host, int64_t step) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!U_host || step < 0) return fail(c, MFQ_EINVAL, "bad arguments");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(c->X[c->cur], U_host, (size_t)c->L * c->N * c->B * sizeof(cplx),
                        hipMemcpyHostToDevice, c->stream), "state upload");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  c->step = step;
  return MFQ_OK;
}

mfq_status mfq_get_slots(mfq_ctx *c, uint64_t *uid_host, int64_t *step_base_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!uid_host || !step_base_host) return fail(c, MFQ_EINVAL, "NULL output");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(uid_host, c->uid, (size_t)c->B * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream),
         "uid download");
  HIPCHK(hipMemcpyAsync(step_base_host, c->step_base, (size_t)c->B * sizeof(int64_t), hipMemcpyDeviceToHost,
                        c->stream), "step base download");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return check_flag(c);
}

mfq_status mfq_set_slots(mfq_ctx *c, const uint64_t *uid_host, const int64_t *step_base_host) {
  if (!c) return MFQ_EINVAL;
  if (!c->ready) return fail(c, MFQ_ESTATE, "mfq_init_state has not succeeded");
  if (!uid_host || !step_base_host) return fail(c, MFQ_EINVAL, "NULL input");
  for (int b = 0; b < c->B; ++b)
    if (step_base_host[b] < 0 || step_base_host[b] > c->step)
      return fail(c, MFQ_EINVAL, "step base outside [0, step of the context]");
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipMemcpyAsync(c->uid, uid_host, (size_t)c->B * sizeof(uint64_t), hipMemcpyHostToDevice, c->stream),
         "uid upload");
  HIPCHK(hipMemcpyAsync(c->step_base, step_base_host, (size_t)c->B * sizeof(int64_t), hipMemcpyHostToDevice,
                        c->stream), "step base upload");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  return MFQ_OK;
}

mfq_status mfq_synchronize(mfq_ctx *c) {
  if (!c) return MFQ_EINVAL;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  HIPCHK(hipStreamSynchronize(c->stream), "synchronize");
  if (!c->ready) return MFQ_OK;
  return check_flag(c);
}

}  // extern "C"

extern "C" {

mfq_status mfq_profile(mfq_ctx *c, int32_t enable) {
  if (!c) return MFQ_EINVAL;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  if (enable) {
    mfq_status st = collect_phase_times(c);
    if (st) return st;
    for (int i = 0; i < MFQ_NPHASES; ++i) {
      c->phase_ms[i] = 0.0;
      c->phase_n[i] = 0;
    }
  }
  c->profiling = enable != 0;
  return MFQ_OK;
}

mfq_status mfq_phase_times(mfq_ctx *c, double *ms, int64_t *count) {
  if (!c) return MFQ_EINVAL;
  HIPCHK(hipSetDevice(c->device), "hipSetDevice");
  mfq_status st = collect_phase_times(c);
  if (st) return st;
  for (int i = 0; i < MFQ_NPHASES; ++i) {
    if (ms) ms[i] = c->phase_ms[i];
    if (count) count[i] = c->phase_n[i];
  }
  return MFQ_OK;
}

}  // extern "C"
