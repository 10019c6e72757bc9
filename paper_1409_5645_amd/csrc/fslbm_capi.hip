// Host side of the C interface declared in include/fslbm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fslbm.h"
#include "fslbm_internal.hpp"

using namespace fslbm;

struct fslbm_ctx {
  fslbm_params p;
  Common com;
  double thr_hi, thr_lo;
  void* f[2];
  uint8_t* flags;
  double* mass;
  double* phi[2];
  hipStream_t stream;
  int cur = 0;          // index of the buffers holding time t
  int step = 0;         // steps done (also the epoch stamp of the next step)
  // workspace carve-out
  double* aux_rho;
  double* aux_u;
  int32_t *f_epoch, *new_epoch, *recv_epoch, *conv_epoch;
  int32_t *listF, *listE, *listEP, *listNI, *listNL, *listR, *listI;
  int32_t* counters;    // 2 sets of NCOUNT
  double* reservoir;
  double* acc;
  int32_t* err;
  int32_t* cnt;
  std::string last_error;
  // sweep timing (fslbm_timing)
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  int pairs = 1;  // FP16 sweep with two cells per lane (FSLBM_FP16_PAIRS=0 disables)
};

namespace {

thread_local std::string g_init_error;

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t aux_rho, aux_u, epochs[4], lists[7], counters, scalars, total;
};

Layout layout(size_t N) {
  Layout L{};
  size_t o = 0;
  L.aux_rho = o;
  o = align_up(o + 8 * N);
  L.aux_u = o;
  o = align_up(o + 24 * N);
  for (int i = 0; i < 4; ++i) {
    L.epochs[i] = o;
    o = align_up(o + 4 * N);
  }
  for (int i = 0; i < 7; ++i) {
    L.lists[i] = o;
    o = align_up(o + 4 * N);
  }
  L.counters = o;
  o = align_up(o + 2 * NCOUNT * sizeof(int32_t));
  L.scalars = o;  // reservoir, acc, err(int), cnt[4] (int)
  o = align_up(o + 2 * sizeof(double) + 8 * sizeof(int32_t));
  L.total = o;
  return L;
}

fslbm_status check_params(const fslbm_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return FSLBM_E_INVALID; }
  if (p->abi_version != FSLBM_ABI_VERSION) { why = "abi_version mismatch"; return FSLBM_E_INVALID; }
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) { why = "dimensions must be >= 1"; return FSLBM_E_INVALID; }
  const double n = (double)p->nx * (double)p->ny * (double)p->nz;
  // 32-bit element offsets address the 19 population planes of a buffer
  if (19.0 * n > 4294967295.0) { why = "too many cells (19 N must be < 2^32)"; return FSLBM_E_INVALID; }
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) { why = "tau must exceed 1/2"; return FSLBM_E_INVALID; }
  if (!(p->magic > 0.0) || !std::isfinite(p->magic)) { why = "magic (Lambda) must be positive"; return FSLBM_E_INVALID; }
  if (p->precision < FSLBM_FP64 || p->precision > FSLBM_FP16S) { why = "unknown precision"; return FSLBM_E_INVALID; }
  if (p->fp16_scale_log2 < 0 || p->fp16_scale_log2 > 24) { why = "fp16_scale_log2 must be in 0..24"; return FSLBM_E_INVALID; }
  if (!(p->rho_gas > 0.0)) { why = "rho_gas must be positive"; return FSLBM_E_INVALID; }
  if (!(p->conv_eps >= 0.0)) { why = "conv_eps must be >= 0"; return FSLBM_E_INVALID; }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->g[a])) { why = "g must be finite"; return FSLBM_E_INVALID; }
  return FSLBM_OK;
}

size_t storage_bytes(int precision) { return precision == FSLBM_FP64 ? 8 : (precision == FSLBM_FP32 ? 4 : 2); }

fslbm_status dev_fail(fslbm_ctx* c, hipError_t e, const char* what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  if (c) c->last_error = m; else g_init_error = m;
  return FSLBM_E_DEVICE;
}

// Constants of the model (section 2.1 and 3.1), derived once in double.
void make_constants(const fslbm_params& p, Common& com, double& thr_hi, double& thr_lo) {
  const bool shifted = p.precision != FSLBM_FP64;
  const double lp = -1.0 / p.tau;              // lambda_+
  const double Lp = p.tau - 0.5;               // Lambda_+
  const double Lm = p.magic / Lp;              // Lambda_-
  const double lm = -1.0 / (Lm + 0.5);         // lambda_-
  Consts<double>& d = com.kd;
  d.lp = lp;
  d.lm = lm;
  d.inv1p = 1.0 / (1.0 + lp);
  for (int a = 0; a < 3; ++a) {
    d.g[a] = p.g[a];
    d.hg[a] = 0.5 * p.g[a];
    d.glm[a] = p.g[a] / lm;
  }
  d.rhob_s = shifted ? p.rho_gas - 1.0 : p.rho_gas;
  d.rho0b = p.incompressible ? 1.0 : p.rho_gas;
  Consts<float>& f = com.kf;
  f.lp = (float)d.lp;
  f.lm = (float)d.lm;
  f.inv1p = (float)d.inv1p;
  for (int a = 0; a < 3; ++a) {
    f.g[a] = (float)d.g[a];
    f.hg[a] = (float)d.hg[a];
    f.glm[a] = (float)d.glm[a];
  }
  f.rhob_s = (float)d.rhob_s;
  f.rho0b = (float)d.rho0b;
  com.incomp = p.incompressible ? 1 : 0;
  com.stokes = p.stokes ? 1 : 0;
  com.scale = std::ldexp(1.0f, p.fp16_scale_log2);
  com.inv_scale = std::ldexp(1.0f, -p.fp16_scale_log2);
  com.grid.nx = p.nx;
  com.grid.ny = p.ny;
  com.grid.nz = p.nz;
  com.grid.N = p.nx * p.ny * p.nz;
  com.grid.px = p.periodic[0] ? 1 : 0;
  com.grid.py = p.periodic[1] ? 1 : 0;
  com.grid.pz = p.periodic[2] ? 1 : 0;
  thr_hi = 1.0 + p.conv_eps;
  thr_lo = -p.conv_eps;
}

#define HIPCHK(c, expr, what)                 \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return dev_fail(c, e_, what); \
  } while (0)

}  // namespace

extern "C" {

fslbm_status fslbm_workspace_size(const fslbm_params* p, size_t* bytes) {
  std::string why;
  fslbm_status s = check_params(p, why);
  if (s != FSLBM_OK) { g_init_error = why; return s; }
  if (!bytes) { g_init_error = "bytes is NULL"; return FSLBM_E_INVALID; }
  *bytes = layout((size_t)p->nx * p->ny * p->nz).total;
  return FSLBM_OK;
}

fslbm_status fslbm_init(const fslbm_params* p, const fslbm_buffers* b, fslbm_ctx** out) {
  std::string why;
  fslbm_status s = check_params(p, why);
  if (s != FSLBM_OK) { g_init_error = why; return s; }
  if (!b || !out) { g_init_error = "buffers or out is NULL"; return FSLBM_E_INVALID; }
  if (!b->f[0] || !b->f[1] || !b->flags || !b->mass || !b->phi[0] || !b->phi[1] || !b->workspace) {
    g_init_error = "a device buffer is NULL";
    return FSLBM_E_INVALID;
  }
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const Layout L = layout(N);
  if (b->workspace_bytes < L.total) { g_init_error = "workspace too small"; return FSLBM_E_INVALID; }
  if (((uintptr_t)b->workspace) % ALIGN) { g_init_error = "workspace not 256-byte aligned"; return FSLBM_E_INVALID; }

  fslbm_ctx* c = new (std::nothrow) fslbm_ctx();
  if (!c) { g_init_error = "out of host memory"; return FSLBM_E_INVALID; }
  c->p = *p;
  make_constants(*p, c->com, c->thr_hi, c->thr_lo);
  c->f[0] = b->f[0];
  c->f[1] = b->f[1];
  c->flags = b->flags;
  c->mass = b->mass;
  c->phi[0] = b->phi[0];
  c->phi[1] = b->phi[1];
  c->stream = (hipStream_t)b->stream;
  if (const char* e = std::getenv("FSLBM_FP16_PAIRS")) c->pairs = std::atoi(e) != 0;
  char* w = (char*)b->workspace;
  c->aux_rho = (double*)(w + L.aux_rho);
  c->aux_u = (double*)(w + L.aux_u);
  int32_t** ep[4] = {&c->f_epoch, &c->new_epoch, &c->recv_epoch, &c->conv_epoch};
  for (int i = 0; i < 4; ++i) *ep[i] = (int32_t*)(w + L.epochs[i]);
  int32_t** ls[7] = {&c->listF, &c->listE, &c->listEP, &c->listNI, &c->listNL, &c->listR, &c->listI};
  for (int i = 0; i < 7; ++i) *ls[i] = (int32_t*)(w + L.lists[i]);
  c->counters = (int32_t*)(w + L.counters);
  c->reservoir = (double*)(w + L.scalars);
  c->acc = c->reservoir + 1;
  c->err = (int32_t*)(c->reservoir + 2);
  c->cnt = c->err + 1;

  auto fail = [&](fslbm_status st) {
    g_init_error = c->last_error;
    delete c;
    return st;
  };
  hipError_t e;
  void* st = (void*)c->stream;
  for (int i = 0; i < 4; ++i)
    if ((e = launch_fill_i32(*ep[i], N, -1, st)) != hipSuccess) return fail(dev_fail(c, e, "init epochs"));
  if ((e = launch_fill_i32(c->counters, 2 * NCOUNT, 0, st)) != hipSuccess) return fail(dev_fail(c, e, "init counters"));
  if ((e = launch_fill_i32(c->err, 5, 0, st)) != hipSuccess) return fail(dev_fail(c, e, "init scalars"));
  if ((e = launch_fill_f64(c->reservoir, 2, 0.0, st)) != hipSuccess) return fail(dev_fail(c, e, "init scalars"));
  if ((e = launch_check_flags(c->flags, c->com.grid, c->err, st)) != hipSuccess) return fail(dev_fail(c, e, "check flags"));
  int32_t herr = 0;
  if ((e = hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "read flag check"));
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail(dev_fail(c, e, "init sync"));
  if (herr & 1) { c->last_error = "unknown cell class in flags"; return fail(FSLBM_E_INVALID); }
  if (herr & 2) { c->last_error = "a liquid cell has a gas neighbour"; return fail(FSLBM_E_INVALID); }
  *out = c;
  return FSLBM_OK;
}

static InitArgs init_args(fslbm_ctx* c) {
  InitArgs a;
  a.c = c->com;
  a.f = c->f[c->cur];
  a.flags = c->flags;
  a.mass = c->mass;
  a.phi = c->phi[c->cur];
  a.aux_rho = c->aux_rho;
  a.aux_u = c->aux_u;
  return a;
}

fslbm_status fslbm_set_equilibrium(fslbm_ctx* c, const double* rho, const double* u, const double* fill) {
  if (!c) return FSLBM_E_INVALID;
  if (!rho || !u || !fill) { c->last_error = "NULL field"; return FSLBM_E_INVALID; }
  HIPCHK(c, launch_set_equilibrium(init_args(c), c->p.precision, rho, u, fill, c->stream), "set_equilibrium");
  HIPCHK(c, hipStreamSynchronize(c->stream), "set_equilibrium sync");
  return FSLBM_OK;
}

fslbm_status fslbm_set_state(fslbm_ctx* c, const double* f, const double* mass, const double* fill,
                             double reservoir) {
  if (!c) return FSLBM_E_INVALID;
  if (!f || !mass || !fill) { c->last_error = "NULL field"; return FSLBM_E_INVALID; }
  HIPCHK(c, launch_set_state(init_args(c), c->p.precision, f, mass, fill, c->stream), "set_state");
  HIPCHK(c, launch_fill_f64(c->reservoir, 1, reservoir, c->stream), "set reservoir");
  HIPCHK(c, hipStreamSynchronize(c->stream), "set_state sync");
  return FSLBM_OK;
}

fslbm_status fslbm_step(fslbm_ctx* c, int32_t n, int32_t rule) {
  if (!c) return FSLBM_E_INVALID;
  if (n < 0) { c->last_error = "n must be >= 0"; return FSLBM_E_INVALID; }
  if (rule != FSLBM_RULE_FSK && rule != FSLBM_RULE_FSL) { c->last_error = "unknown rule"; return FSLBM_E_INVALID; }
  if (rule == FSLBM_RULE_FSL && c->p.tau == 1.0) {
    c->last_error = "FSL needs tau != 1 (n+ is not recoverable from a fully relaxed state)";
    return FSLBM_E_UNSUPPORTED;
  }
  for (int32_t i = 0; i < n; ++i) {
    StepLaunch L;
    const int a = c->cur, b = 1 - c->cur;
    SweepArgs& s = L.sweep;
    s.c = c->com;
    s.fin = c->f[a];
    s.fout = c->f[b];
    s.flags = c->flags;
    s.mass = c->mass;
    s.phi_in = c->phi[a];
    s.phi_out = c->phi[b];
    s.aux_rho = c->aux_rho;
    s.aux_u = c->aux_u;
    s.f_epoch = c->f_epoch;
    s.listF = c->listF;
    s.listE = c->listE;
    s.listI = c->listI;
    s.counters = c->counters + (c->step & 1) * NCOUNT;
    s.counters_next = c->counters + ((c->step + 1) & 1) * NCOUNT;
    s.thr_hi = c->thr_hi;
    s.thr_lo = c->thr_lo;
    s.step = c->step;
    s.freeze = c->p.freeze ? 1 : 0;
    s.cpr = 0;
    s.pairs = c->pairs;
    ConvArgs& v = L.conv;
    v.c = c->com;
    v.fout = c->f[b];
    v.flags = c->flags;
    v.mass = c->mass;
    v.phi_out = c->phi[b];
    v.aux_rho = c->aux_rho;
    v.aux_u = c->aux_u;
    v.f_epoch = c->f_epoch;
    v.new_epoch = c->new_epoch;
    v.recv_epoch = c->recv_epoch;
    v.conv_epoch = c->conv_epoch;
    v.listF = c->listF;
    v.listE = c->listE;
    v.listEP = c->listEP;
    v.listNI = c->listNI;
    v.listNL = c->listNL;
    v.listR = c->listR;
    v.counters = s.counters;
    v.reservoir = c->reservoir;
    v.step = c->step;
    L.stream = (void*)c->stream;
    if (c->timing) {
      while (c->events.size() < c->events_used + 2) {
        hipEvent_t ev;
        HIPCHK(c, hipEventCreate(&ev), "event create");
        c->events.push_back(ev);
      }
      HIPCHK(c, hipEventRecord(c->events[c->events_used], c->stream), "event record");
    }
    HIPCHK(c, launch_sweep(L, c->p.precision, rule), "sweep launch");
    if (c->timing) {
      HIPCHK(c, hipEventRecord(c->events[c->events_used + 1], c->stream), "event record");
      c->events_used += 2;
    }
    HIPCHK(c, launch_iface(L, c->p.precision, rule), "interface launch");
    if (!c->p.freeze) HIPCHK(c, launch_convert(L, c->p.precision), "conversion launch");
    c->cur = b;
    c->step += 1;
  }
  return FSLBM_OK;
}

fslbm_status fslbm_fields(fslbm_ctx* c, uint32_t mask, void* const* dst) {
  if (!c) return FSLBM_E_INVALID;
  if (mask && !dst) { c->last_error = "dst is NULL"; return FSLBM_E_INVALID; }
  for (int i = 0; i < 8; ++i)
    if ((mask >> i) & 1u)
      if (!dst[i]) { c->last_error = "dst entry for a selected field is NULL"; return FSLBM_E_INVALID; }
  if (mask >> 8) { c->last_error = "unknown field bit"; return FSLBM_E_INVALID; }
  FieldArgs a;
  a.c = c->com;
  a.f = c->f[c->cur];
  a.flags = c->flags;
  a.mass = c->mass;
  a.phi = c->phi[c->cur];
  a.aux_rho = c->aux_rho;
  a.aux_u = c->aux_u;
  auto sel = [&](int bit) { return ((mask >> bit) & 1u) ? dst[bit] : nullptr; };
  a.rho_out = (double*)sel(0);
  a.u_out = (double*)sel(1);
  a.phi_out = (double*)sel(2);
  a.flags_out = (uint8_t*)sel(3);
  a.f_out = (double*)sel(4);
  a.mass_out = (double*)sel(5);
  a.rhoc_out = (double*)sel(6);
  a.uc_out = (double*)sel(7);
  HIPCHK(c, launch_fields(a, c->p.precision, c->stream), "fields");
  HIPCHK(c, hipStreamSynchronize(c->stream), "fields sync");
  return FSLBM_OK;
}

fslbm_status fslbm_stats(fslbm_ctx* c, double* total_mass, double* reservoir, int64_t counts[8]) {
  if (!c) return FSLBM_E_INVALID;
  HIPCHK(c, launch_fill_f64(c->acc, 1, 0.0, c->stream), "stats init");
  HIPCHK(c, launch_fill_i32(c->cnt, 4, 0, c->stream), "stats init");
  StatArgs a;
  a.c = c->com;
  a.f = c->f[c->cur];
  a.flags = c->flags;
  a.mass = c->mass;
  a.acc = c->acc;
  a.cnt = c->cnt;
  HIPCHK(c, launch_stats(a, c->p.precision, c->stream), "stats");
  double sc[2];
  int32_t cn[4];
  int32_t last[NCOUNT] = {0};
  HIPCHK(c, hipMemcpyAsync(sc, c->reservoir, sizeof(sc), hipMemcpyDeviceToHost, c->stream), "stats copy");
  HIPCHK(c, hipMemcpyAsync(cn, c->cnt, sizeof(cn), hipMemcpyDeviceToHost, c->stream), "stats copy");
  if (c->step > 0)
    HIPCHK(c, hipMemcpyAsync(last, c->counters + ((c->step - 1) & 1) * NCOUNT, sizeof(last), hipMemcpyDeviceToHost,
                             c->stream), "stats copy");
  HIPCHK(c, hipStreamSynchronize(c->stream), "stats sync");
  if (total_mass) *total_mass = sc[1] + sc[0];
  if (reservoir) *reservoir = sc[0];
  if (counts) {
    counts[0] = last[C_F];
    counts[1] = last[C_E];
    counts[2] = last[C_EP];
    counts[3] = last[C_NI];
    counts[4] = last[C_NL];
    counts[5] = cn[2];
    counts[6] = cn[0];
    counts[7] = c->step;
  }
  if (cn[1] != 0) {
    c->last_error = std::to_string(cn[1]) + " cells with NaN or non-positive density";
    return FSLBM_E_UNSTABLE;
  }
  return FSLBM_OK;
}

fslbm_status fslbm_conversions(fslbm_ctx* c, int32_t* const* out, int32_t cap, int32_t n_out[5]) {
  if (!c) return FSLBM_E_INVALID;
  if (!n_out || cap < 0) { c->last_error = "n_out is NULL or cap < 0"; return FSLBM_E_INVALID; }
  int32_t last[NCOUNT] = {0};
  if (c->step > 0) {
    HIPCHK(c, hipMemcpyAsync(last, c->counters + ((c->step - 1) & 1) * NCOUNT, sizeof(last), hipMemcpyDeviceToHost,
                             c->stream), "conversions copy");
    HIPCHK(c, hipStreamSynchronize(c->stream), "conversions sync");
  }
  const int which[5] = {C_F, C_E, C_EP, C_NI, C_NL};
  int32_t* lists[5] = {c->listF, c->listE, c->listEP, c->listNI, c->listNL};
  fslbm_status st = FSLBM_OK;
  for (int i = 0; i < 5; ++i) {
    const int n = last[which[i]];
    n_out[i] = n;
    if (n == 0) continue;
    std::vector<int32_t> h(n);
    HIPCHK(c, hipMemcpy(h.data(), lists[i], sizeof(int32_t) * n, hipMemcpyDeviceToHost), "conversions copy");
    std::sort(h.begin(), h.end());
    if (out && out[i]) std::memcpy(out[i], h.data(), sizeof(int32_t) * std::min(n, cap));
    if (n > cap) st = FSLBM_E_CAPACITY;
  }
  if (st != FSLBM_OK) c->last_error = "a conversion list exceeds cap";
  return st;
}

fslbm_status fslbm_timing(fslbm_ctx* c, int32_t enable, double* sweep_ms, int64_t* sweeps) {
  if (!c) return FSLBM_E_INVALID;
  if (sweep_ms || sweeps) {
    HIPCHK(c, hipStreamSynchronize(c->stream), "timing sync");
    double tot = 0.0;
    for (size_t i = 0; i + 1 < c->events_used; i += 2) {
      float ms = 0.0f;
      HIPCHK(c, hipEventElapsedTime(&ms, c->events[i], c->events[i + 1]), "event elapsed");
      tot += ms;
    }
    if (sweep_ms) *sweep_ms = tot;
    if (sweeps) *sweeps = (int64_t)(c->events_used / 2);
  }
  if (enable) c->events_used = 0;
  c->timing = enable != 0;
  return FSLBM_OK;
}

fslbm_status fslbm_destroy(fslbm_ctx* c) {
  if (!c) return FSLBM_E_INVALID;
  hipError_t e = hipStreamSynchronize(c->stream);
  for (hipEvent_t ev : c->events) (void)hipEventDestroy(ev);
  delete c;
  return e == hipSuccess ? FSLBM_OK : FSLBM_E_DEVICE;
}

const char* fslbm_last_error(const fslbm_ctx* c) {
  return c ? c->last_error.c_str() : g_init_error.c_str();
}

}  // extern "C"
