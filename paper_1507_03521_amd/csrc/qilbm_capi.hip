// C ABI of the quasi-incompressible phase-field LBE library (include/qilbm.h).
// Host code only: argument validation, derivation of the model coefficients,
// workspace layout, and dispatch of the kernels on the context's stream.
#include <math.h>
#include <mutex>
#include <new>
#include <string.h>

#include "../../include/qilbm.h"
#include "qilbm_adjoint.hpp"
#include "qilbm_internal.hpp"

using namespace qilbm;

struct lbm_ctx {
  lbm_params prm;
  double beta, kappa, lam, alpha, gamma, drho;
  Geom geom;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  char* pop[2];
  int cur;
  char* fields;       // phi, mu, p scratch (compute type, Ns elements each)
  double* part;       // reduction partials, 4 per block
  int nred;
  double* red_out;    // 8 doubles
  int64_t t;
  int seg_rows;
  int resident;       // fused workgroups resident at once on this device
  int pass_steps;     // time steps per pass of the fused kernel (1 or 2)
  int pass_seg_rows;  // rows per segment of the two-step kernel (0: automatic)
  int resident2;      // two-step workgroups resident at once
  int64_t pbytes;
  AdjointState adj;
};

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool finite_all(const lbm_params* p) {
  const double v[] = {p->rho_A, p->rho_B, p->sigma, p->W, p->M, p->tau_f, p->tau_g,
                      p->gx,    p->gy,    p->rho_ref, p->trt_magic};
  for (double d : v)
    if (!isfinite(d)) return false;
  return true;
}

bool valid(const lbm_params* p) {
  if (!p) return false;
  if (p->nx < 3 || p->ny < 3) return false;
  // 32-bit byte offsets inside a population plane (8-byte values, plane
  // stride below 2^29 elements including the stagger)
  if ((int64_t)p->nx * (int64_t)p->ny > ((int64_t)1 << 29) - 4096) return false;
  if (!finite_all(p)) return false;
  if (!(p->rho_A > 0.0) || !(p->rho_B > 0.0)) return false;
  if (!(p->sigma > 0.0) || !(p->W > 0.0) || !(p->M > 0.0)) return false;
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5)) return false;
  if (p->bc != LBM_BC_PERIODIC && p->bc != LBM_BC_WALLS_Y) return false;
  if (p->precision < LBM_FP64 || p->precision > LBM_FP16_STORE) return false;
  if (p->flags & ~(uint32_t)(LBM_FLAG_NO_GAMMA | LBM_FLAG_UNFUSED)) return false;
  if (!(p->trt_magic >= 0.0)) return false;
  return true;
}

Geom make_geom(const lbm_params* p) {
  Geom g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.walls = p->bc == LBM_BC_WALLS_Y;
  g.N = (int64_t)p->nx * p->ny;
  g.Ns = plane_stride(g.N);
  return g;
}

// Coefficients of Sec. II-III with phi_A = 1, phi_B = 0:
// beta = 12 sigma / W, kappa = 3 sigma W / 2 (from the interface width
// W = sqrt(8 kappa / beta) and sigma = sqrt(2 kappa beta) / 6),
// lambda = M, alpha = lambda / (c_s^2 (tau_g - 1/2)),
// gamma = rho_A / rho_B - 1, d rho / d phi = rho_A - rho_B.
void derive(const lbm_params* p, double out[6]) {
  out[0] = 12.0 * p->sigma / p->W;
  out[1] = 1.5 * p->sigma * p->W;
  out[2] = p->M;
  out[3] = p->M / ((p->tau_g - 0.5) / 3.0);
  out[4] = (p->flags & LBM_FLAG_NO_GAMMA) ? 0.0 : p->rho_A / p->rho_B - 1.0;
  out[5] = p->rho_A - p->rho_B;
}

struct Layout {
  size_t pop0, pop1, fields, part, red, total;
  int nred;
};

Layout layout(const lbm_params* p) {
  const Geom g = make_geom(p);
  Layout L;
  const size_t pb = up((size_t)pop_bytes(p->precision, g.Ns));
  L.nred = (int)((g.N + 255) / 256);
  if (L.nred > 2048) L.nred = 2048;
  L.pop0 = 0;
  L.pop1 = L.pop0 + pb;
  L.fields = L.pop1 + pb;
  L.part = L.fields + up(3 * (size_t)g.Ns * 8);
  L.red = L.part + up((size_t)L.nred * 4 * 8);
  L.total = L.red + up(8 * 8);
  return L;
}

// Kernel coefficients in the compute type from the parameters and their
// derived coefficients d[6] (derive()).
template <typename T>
Coef<T> coef_of(const lbm_params& p, const double d[6]) {
  Coef<T> k;
  k.beta4 = T(4.0 * d[0]);
  k.kappa = T(d[1]);
  k.lam = T(d[2]);
  k.alpha = T(d[3]);
  k.gamma = T(d[4]);
  k.drho = T(d[5]);
  k.rho_B = T(p.rho_B);
  k.rho_ref = T(p.rho_ref);
  k.gx = T(p.gx);
  k.gy = T(p.gy);
  k.inv_tau_f = T(1.0 / p.tau_f);
  k.inv_tau_g = T(1.0 / p.tau_g);
  k.kf = T(1.0 - 0.5 / p.tau_f);
  k.kg = T(1.0 - 0.5 / p.tau_g);
  // odd part of the TRT collision: tau_- = 1/2 + magic / (tau_f - 1/2)
  const double tau_m = p.trt_magic > 0.0 ? 0.5 + p.trt_magic / (p.tau_f - 0.5) : p.tau_f;
  k.inv_tau_m = T(1.0 / tau_m);
  k.km = T(1.0 - 0.5 / tau_m);
  return k;
}

template <typename T>
Coef<T> coef_t(const lbm_ctx* c) {
  const double d[6] = {c->beta, c->kappa, c->lam, c->alpha, c->gamma, c->drho};
  return coef_of<T>(c->prm, d);
}

bool trt_of(const lbm_ctx* c) { return c->prm.trt_magic > 0.0; }

lbm_status st(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

char* phi_f(lbm_ctx* c) { return c->fields; }
char* mu_f(lbm_ctx* c) { return c->fields + c->geom.Ns * 8; }
char* p_f(lbm_ctx* c) { return c->fields + 2 * c->geom.Ns * 8; }

// n steps; with recs not null, step k also writes the record of the state it
// starts from into recs[k] (planes phi, mu, p, S, jx, jy of the compute type
// at stride Ns). Pairs of steps run as one two-step launch when the context
// uses two steps per pass (a pair's records come from that launch).
template <int P>
lbm_status step_p(lbm_ctx* c, int64_t n, void* const* recs) {
  using T = typename PrecT<P>::T;
  const Coef<T> k = coef_t<T>(c);
  const bool unfused = c->prm.flags & LBM_FLAG_UNFUSED;
  const bool trt = trt_of(c);
  if (trt && recs) return LBM_EINVAL;
  const int64_t pl = c->geom.Ns;
  int64_t done = 0;
  if (!unfused && c->pass_steps == 2 && n >= 2) {
    const FusedShape sh2 = fused2_shape<P>(c->geom, c->pass_seg_rows, c->resident2);
    for (; n - done >= 2; done += 2) {
      void* r0 = recs ? recs[done] : nullptr;
      void* r1 = recs ? recs[done + 1] : nullptr;
      if (launch_step2_fused<P>(c->pop[c->cur], c->pop[c->cur ^ 1], k, c->geom, sh2, r0, r1,
                                c->stream, trt) != hipSuccess)
        return LBM_EDEVICE;
      c->cur ^= 1;
      c->t += 2;
    }
  }
  const FusedShape sh = fused_shape<P>(c->geom, c->seg_rows, c->resident);
  for (; done < n; ++done) {
    void* rec = recs ? recs[done] : nullptr;
    hipError_t e;
    if (unfused && rec)
      e = launch_step_unfused<P>(c->pop[c->cur], c->pop[c->cur ^ 1], (T*)rec, (T*)rec + pl,
                                 (T*)rec + 2 * pl, (T*)rec + 3 * pl, k, c->geom, c->stream);
    else if (unfused)
      e = launch_step_unfused<P>(c->pop[c->cur], c->pop[c->cur ^ 1], phi_f(c), mu_f(c), p_f(c),
                                 nullptr, k, c->geom, c->stream, trt);
    else
      e = launch_step_fused<P>(c->pop[c->cur], c->pop[c->cur ^ 1], k, c->geom, sh, rec,
                               c->stream, trt);
    if (e != hipSuccess) return LBM_EDEVICE;
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

template <int P>
lbm_status moments_p(lbm_ctx* c, const MomentOut& mo) {
  using T = typename PrecT<P>::T;
  const Coef<T> k = coef_t<T>(c);
  hipError_t e = launch_fields<P>(c->pop[c->cur], phi_f(c), mu_f(c), k, c->geom, c->stream);
  if (e != hipSuccess) return LBM_EDEVICE;
  return st(launch_macro<P>(c->pop[c->cur], phi_f(c), mu_f(c), nullptr, nullptr, mo, k, c->geom,
                            c->stream));
}

template <int P>
lbm_status mass_p(lbm_ctx* c) {
  using T = typename PrecT<P>::T;
  return st(launch_mass<P>(c->pop[c->cur], phi_f(c), mu_f(c), c->part, c->nred, c->red_out,
                           coef_t<T>(c), coef_t<double>(c), c->geom, c->stream));
}

// ------------------------------------------- totals without any allocation
// lbm_mass_noalloc runs lbm_mass's kernels on a caller's raw state with their
// scratch -- the phi and mu fields and the per-block partials -- in a static
// device array instead of a context workspace.
constexpr int64_t NOALLOC_MAX_NODES = int64_t(1) << 21;
constexpr size_t NOALLOC_FIELD_BYTES = size_t(NOALLOC_MAX_NODES) * 8;
constexpr int NOALLOC_MAX_PARTS = 2048;   // the workspace layout's cap of nred
constexpr size_t NOALLOC_BYTES = 2 * NOALLOC_FIELD_BYTES + size_t(NOALLOC_MAX_PARTS) * 4 * 8;

}  // namespace

// One copy per GPU for the life of the process. Host code never passes this
// name to a kernel: it is a host-side stand-in, not the device address; the
// address comes from hipGetSymbolAddress, per device (noalloc_scratch).
static __device__ __align__(256) char scratch[NOALLOC_BYTES];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[NOALLOC_MAX_DEVICES];   // device address of scratch, per device

// Device address of the current device's copy of scratch, looked up once per
// device with that device current.
lbm_status noalloc_scratch(char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_EDEVICE;
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return LBM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EDEVICE;
    g_noalloc_ptr[dev] = (char*)ptr;
  }
  *out = g_noalloc_ptr[dev];
  return LBM_OK;
}

template <int P>
hipError_t mass_noalloc_p(const lbm_params& p, const void* state, double* out, char* sc,
                          hipStream_t s) {
  using T = typename PrecT<P>::T;
  double d[6];
  derive(&p, d);
  const Geom g = make_geom(&p);
  // same partial count as a context's workspace (layout()), so the totals
  // are those of lbm_mass bit for bit
  int nred = (int)((g.N + 255) / 256);
  if (nred > NOALLOC_MAX_PARTS) nred = NOALLOC_MAX_PARTS;
  return launch_mass<P>(state, sc, sc + NOALLOC_FIELD_BYTES, (double*)(sc + 2 * NOALLOC_FIELD_BYTES),
                        nred, out, coef_of<T>(p, d), coef_of<double>(p, d), g, s);
}

}  // namespace

// Precision dispatch: calls FN<P>(args...) for the context's precision.
#define QILBM_DISPATCH(prec, FN, ...)                  \
  ((prec) == LBM_FP64   ? FN<P_F64>(__VA_ARGS__)       \
   : (prec) == LBM_FP32 ? FN<P_F32>(__VA_ARGS__)       \
                        : FN<P_F16>(__VA_ARGS__))

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* params) {
  if (!valid(params)) return 0;
  return layout(params).total;
}

lbm_status lbm_coefficients(const lbm_params* params, double out[6]) {
  if (!valid(params) || !out) return LBM_EINVAL;
  derive(params, out);
  return LBM_OK;
}

lbm_status lbm_init(lbm_ctx** out, const lbm_params* params, void* workspace_dev,
                    size_t workspace_bytes, const double* phi0_dev, void* stream) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!valid(params) || !workspace_dev || !phi0_dev) return LBM_EINVAL;
  if ((uintptr_t)workspace_dev % ALIGN != 0) return LBM_EINVAL;
  const Layout L = layout(params);
  if (workspace_bytes < L.total) return LBM_ENOMEM;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  c->prm = *params;
  double d[6];
  derive(params, d);
  c->beta = d[0];
  c->kappa = d[1];
  c->lam = d[2];
  c->alpha = d[3];
  c->gamma = d[4];
  c->drho = d[5];
  c->geom = make_geom(params);
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace_dev;
  c->ws_bytes = workspace_bytes;
  c->pop[0] = c->ws + L.pop0;
  c->pop[1] = c->ws + L.pop1;
  c->cur = 0;
  c->fields = c->ws + L.fields;
  c->part = (double*)(c->ws + L.part);
  c->nred = L.nred;
  c->red_out = (double*)(c->ws + L.red);
  c->t = 0;
  c->seg_rows = 0;
  c->resident = QILBM_DISPATCH(params->precision, fused_resident);
  // two steps per pass where it is the faster kernel (FP32, FP64); FP16
  // storage keeps one (its two-step kernel measured slower: the binary16
  // conversions of the intermediate state make it arithmetic-bound)
  c->pass_steps = params->precision == LBM_FP16_STORE ? 1 : 2;
  c->pass_seg_rows = 0;
  c->resident2 = QILBM_DISPATCH(params->precision, fused2_resident);
  c->pbytes = pop_bytes(params->precision, c->geom.Ns);
  Coef<double> k = coef_t<double>(c);
  // both population buffers start zeroed, padding included, so that raw
  // snapshots of equal states are equal byte for byte
  hipError_t e = launch_zero(c->ws + L.pop0, L.fields - L.pop0, c->stream);
  if (e == hipSuccess)
    e = QILBM_DISPATCH(params->precision, launch_init, phi0_dev, c->pop[0], k, c->geom,
                       c->stream);
  if (e != hipSuccess) {
    delete c;
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  return QILBM_DISPATCH(c->prm.precision, step_p, c, nsteps, (void* const*)nullptr);
}

size_t lbm_record_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  return up(6 * (size_t)c->geom.Ns * (c->prm.precision == LBM_FP64 ? 8 : 4));
}

lbm_status lbm_step_record(lbm_ctx* c, void* record_dev) {
  if (!c || !record_dev || trt_of(c)) return LBM_EINVAL;
  if ((uintptr_t)record_dev % ALIGN != 0) return LBM_EINVAL;
  void* const recs[1] = {record_dev};
  return QILBM_DISPATCH(c->prm.precision, step_p, c, 1, recs);
}

lbm_status lbm_step_records(lbm_ctx* c, int64_t nsteps, void* const* records) {
  if (!c || nsteps < 0 || (nsteps > 0 && !records) || trt_of(c)) return LBM_EINVAL;
  for (int64_t k = 0; k < nsteps; ++k)
    if (!records[k] || (uintptr_t)records[k] % ALIGN != 0) return LBM_EINVAL;
  return QILBM_DISPATCH(c->prm.precision, step_p, c, nsteps, records);
}

lbm_status lbm_moments(lbm_ctx* c, double* phi, double* rho, double* ux, double* uy, double* p,
                       double* mu) {
  if (!c) return LBM_EINVAL;
  MomentOut mo;
  mo.phi = phi;
  mo.rho = rho;
  mo.ux = ux;
  mo.uy = uy;
  mo.p = p;
  mo.mu = mu;
  return QILBM_DISPATCH(c->prm.precision, moments_p, c, mo);
}

lbm_status lbm_mass(lbm_ctx* c, double out[4]) {
  if (!c || !out) return LBM_EINVAL;
  lbm_status s = QILBM_DISPATCH(c->prm.precision, mass_p, c);
  if (s != LBM_OK) return s;
  if (hipMemcpyAsync(out, c->red_out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_EDEVICE;
  for (int k = 0; k < 4; ++k)
    if (!isfinite(out[k])) return LBM_EDIVERGED;
  return LBM_OK;
}

lbm_status lbm_mass_noalloc(const lbm_params* params, const void* state_dev, double* out_dev,
                            void* stream) {
  if (!valid(params) || !state_dev || !out_dev) return LBM_EINVAL;
  if ((uintptr_t)state_dev % ALIGN != 0 || (uintptr_t)out_dev % 8 != 0) return LBM_EINVAL;
  if ((int64_t)params->nx * params->ny > NOALLOC_MAX_NODES) return LBM_EINVAL;
  char* sc = nullptr;
  lbm_status s = noalloc_scratch(&sc);
  if (s != LBM_OK) return s;
  return st(QILBM_DISPATCH(params->precision, mass_noalloc_p, *params, state_dev, out_dev, sc,
                           (hipStream_t)stream));
}

lbm_status lbm_get_state(lbm_ctx* c, double* f, double* g) {
  if (!c || !f || !g) return LBM_EINVAL;
  return st(QILBM_DISPATCH(c->prm.precision, launch_to_canonical, c->pop[c->cur], f, g, c->geom,
                           c->stream));
}

lbm_status lbm_set_state(lbm_ctx* c, const double* f, const double* g) {
  if (!c || !f || !g) return LBM_EINVAL;
  return st(QILBM_DISPATCH(c->prm.precision, launch_from_canonical, f, g, c->pop[c->cur], c->geom,
                           c->stream));
}

size_t lbm_state_bytes(const lbm_ctx* c) { return c ? (size_t)c->pbytes : 0; }

lbm_status lbm_save_raw(lbm_ctx* c, void* dst) {
  if (!c || !dst) return LBM_EINVAL;
  return st(hipMemcpyAsync(dst, c->pop[c->cur], c->pbytes, hipMemcpyDeviceToDevice, c->stream));
}

lbm_status lbm_load_raw(lbm_ctx* c, const void* src, int64_t t) {
  if (!c || !src || t < 0) return LBM_EINVAL;
  c->t = t;
  return st(hipMemcpyAsync(c->pop[c->cur], src, c->pbytes, hipMemcpyDeviceToDevice, c->stream));
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

lbm_status lbm_set_stream(lbm_ctx* c, void* stream) {
  if (!c) return LBM_EINVAL;
  c->stream = (hipStream_t)stream;
  return LBM_OK;
}

lbm_status lbm_set_launch(lbm_ctx* c, int32_t seg_rows) {
  if (!c || seg_rows < 0) return LBM_EINVAL;
  c->seg_rows = seg_rows;
  return LBM_OK;
}

lbm_status lbm_launch_info(const lbm_ctx* c, int32_t out[4]) {
  if (!c || !out) return LBM_EINVAL;
  const FusedShape sh =
      c->prm.precision == LBM_FP64
          ? fused_shape<P_F64>(c->geom, c->seg_rows, c->resident)
          : (c->prm.precision == LBM_FP32 ? fused_shape<P_F32>(c->geom, c->seg_rows, c->resident)
                                          : fused_shape<P_F16>(c->geom, c->seg_rows, c->resident));
  out[0] = sh.nstrips;
  out[1] = sh.nseg;
  out[2] = sh.seg_rows;
  out[3] = sh.threads;
  return LBM_OK;
}

lbm_status lbm_set_pass(lbm_ctx* c, int32_t steps, int32_t seg_rows) {
  if (!c || seg_rows < 0 || (steps != 1 && steps != 2)) return LBM_EINVAL;
  c->pass_steps = steps;
  c->pass_seg_rows = seg_rows;
  return LBM_OK;
}

lbm_status lbm_pass_info(const lbm_ctx* c, int32_t out[5]) {
  if (!c || !out) return LBM_EINVAL;
  FusedShape sh;
  if (c->pass_steps == 2)
    sh = c->prm.precision == LBM_FP64
             ? fused2_shape<P_F64>(c->geom, c->pass_seg_rows, c->resident2)
             : (c->prm.precision == LBM_FP32
                    ? fused2_shape<P_F32>(c->geom, c->pass_seg_rows, c->resident2)
                    : fused2_shape<P_F16>(c->geom, c->pass_seg_rows, c->resident2));
  else
    sh = c->prm.precision == LBM_FP64
             ? fused_shape<P_F64>(c->geom, c->seg_rows, c->resident)
             : (c->prm.precision == LBM_FP32
                    ? fused_shape<P_F32>(c->geom, c->seg_rows, c->resident)
                    : fused_shape<P_F16>(c->geom, c->seg_rows, c->resident));
  out[0] = c->pass_steps;
  out[1] = sh.nstrips;
  out[2] = sh.nseg;
  out[3] = sh.seg_rows;
  out[4] = sh.threads;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) { delete c; }

const char* lbm_strerror(lbm_status s) {
  switch (s) {
    case LBM_OK: return "success";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small or host allocation failed";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_EDIVERGED: return "non-finite lattice total (diverged)";
    case LBM_ESTATE: return "call not valid in the current state";
  }
  return "unknown status";
}

int32_t lbm_abi_version(void) { return QILBM_ABI_VERSION; }

}  // extern "C"

// ------------------------------------------------------------------ adjoint
// The adjoint entry points live in qilbm_adjoint.hip; they reach the context
// through these accessors.
namespace qilbm {
CtxView ctx_view(lbm_ctx* c) {
  CtxView v;
  v.prm = &c->prm;
  v.beta = c->beta;
  v.kappa = c->kappa;
  v.lam = c->lam;
  v.alpha = c->alpha;
  v.gamma = c->gamma;
  v.drho = c->drho;
  v.geom = c->geom;
  v.stream = c->stream;
  v.adj = &c->adj;
  v.pbytes = c->pbytes;
  return v;
}
}  // namespace qilbm
