// Host side of the C interface declared in include/fslbm.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
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
  double* aux;  // [N][4] collision density and velocity of interface cells
  int32_t *f_epoch, *new_epoch, *recv_epoch, *conv_epoch;
  int32_t *listF, *listE, *listEP, *listNI, *listNL, *listR, *listI;
  int32_t* counters;    // 2 sets of NCOUNT
  // interface kernel before the sweep (the plain step with the four-lane
  // interface kernel): cell -> list entry, the list-ordered populations the
  // sweep stores, and whether listI / islot / the counter of the current step
  // hold the list of the current state (else the step builds it first)
  int32_t* islot = nullptr;
  void* rbuf = nullptr;
  int rcap = 0;
  bool reorder = false;
  bool list_ok = false;
  double* reservoir;
  double* kappa = nullptr;  // surface tension only
  double* khf = nullptr;    // surface tension with plic = 2 only
  double* wall_t = nullptr; // moving-wall terms [6][19]
  bool has_solid = false;   // the flags hold solid cells
  const int32_t* wcells = nullptr;  // wall table (caller's device memory, fslbm_set_walls)
  const double* wdelta = nullptr;
  const double* wuw = nullptr;
  int nwall = -1;           // -1: no table set
  const double* surf_n = nullptr;   // prescribed surface (caller's device memory, fslbm_set_surface)
  const double* surf_d = nullptr;
  double* acc;
  int32_t* err;
  int32_t* cnt;
  std::string last_error;
  // sweep timing (fslbm_timing)
  bool timing = false;
  std::vector<hipEvent_t> events;
  size_t events_used = 0;
  int pairs = 1;  // FP16 sweep with two cells per lane (FSLBM_FP16_PAIRS=0 disables)
  int quad = 2;   // interface kernel: 2 four lanes per cell in XCD-aware order (FSLBM_IFACE_QUAD: 1 plain order, 0 one lane per cell)
  int check_every = 0;  // health check after every K-th step (0: none)
  int static_device = -1;  // device whose static workspace this context holds (fslbm_init_static)
  int dflt_T = -1, dflt_K = 0;  // default checkpoint spacing chosen for windows of length dflt_T
  // Rows the sweep launches: every ext_every steps the extent of the fluid
  // cells is measured on the device and copied into pinned host memory
  // without a wait; a step launches only the rows within the latest extent
  // that has arrived, widened by one cell per step since it was taken (the
  // fluid region grows by at most one cell per step: new interface cells are
  // neighbours of filled ones).  Off (every row) for fslbm_init_static.
  int ext_every = 0;
  int32_t* ext_dev = nullptr;        // workspace: the kernel's output
  int32_t* ext_host = nullptr;       // pinned: two slots of 4 values
  hipEvent_t ext_ev[2] = {nullptr, nullptr};
  int ext_step[2] = {-1, -1};        // step whose flags each slot describes
  int ext_pending = -1, ext_valid = -1;
  double u_max2 = 0.16; // square of the |u| bound of the health check
};

namespace {

thread_local std::string g_init_error;

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Layout {
  size_t aux, epochs[4], lists[7], counters, scalars, extent, wall_t, kappa, khf, islot, rbuf, rcap, total;
};

// Entries of the list-ordered population buffer of the interface-first step:
// every cell on small lattices, else an eighth of them (at least 32768); an
// interface list longer than that writes the rest straight into the cells.
size_t rbuf_entries(size_t N) { return N <= 32768 ? N : std::max<size_t>(32768, N / 8); }

// Moving-wall bounce-back terms per face (x-, x+, y-, y+, z-, z+) and link:
// 2 w_q (c_q . u_w) / c_s^2 in FP64 (zero on periodic axes and for walls at
// rest), computed on the host as (c_x u_x + c_y u_y) + c_z u_z, times 6 w_q.
void wall_table(const fslbm_params& p, double out[6 * Q]) {
  static const int CV[Q][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                               {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                               {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                               {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
  for (int f = 0; f < 6; ++f)
    for (int q = 0; q < Q; ++q) {
      const double* u = p.wall_u[f];
      const double cu = (CV[q][0] * u[0] + CV[q][1] * u[1]) + CV[q][2] * u[2];
      const double w = q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
      out[f * Q + q] = (p.periodic[f / 2] || cu == 0.0) ? 0.0 : 6.0 * w * cu;
    }
}

// kappa: with surface tension, one Laplace-pressure correction per listed cell;
// hf: with surface tension and plic = 2, the height-function kappa per cell;
// reorder: room for the interface-first step (cell -> list entry, 19
// populations of s bytes per list entry)
Layout layout(size_t N, bool kappa, bool hf, size_t s, bool reorder) {
  Layout L{};
  size_t o = 0;
  L.aux = o;
  o = align_up(o + 32 * N);
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
  L.scalars = o;  // reservoir, acc, err(int), cnt[8] (int)
  o = align_up(o + 2 * sizeof(double) + 16 * sizeof(int32_t));
  L.extent = o;
  o = align_up(o + EXT_BYTES);
  L.wall_t = o;
  o = align_up(o + 8 * 6 * Q);
  L.kappa = o;
  if (kappa) o = align_up(o + 8 * N);
  L.khf = o;
  if (kappa && hf) o = align_up(o + 8 * N);
  L.rcap = reorder ? rbuf_entries(N) : 0;
  L.islot = o;
  if (reorder) o = align_up(o + 4 * N);
  L.rbuf = o;
  if (reorder) o = align_up(o + (size_t)Q * s * L.rcap);
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
  if (!(p->sigma >= 0.0) || !std::isfinite(p->sigma)) { why = "sigma must be finite and >= 0"; return FSLBM_E_INVALID; }
  if (p->plic < 0 || p->plic > 2) { why = "plic must be 0, 1 or 2"; return FSLBM_E_INVALID; }
  if (p->check_every < 0) { why = "check_every must be >= 0"; return FSLBM_E_INVALID; }
  if (!(p->u_max >= 0.0) || !std::isfinite(p->u_max)) { why = "u_max must be finite and >= 0"; return FSLBM_E_INVALID; }
  for (int f = 0; f < 6; ++f)
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->wall_u[f][a])) { why = "wall_u must be finite"; return FSLBM_E_INVALID; }
  for (int i = 0; i < 6; ++i)
    if (!std::isfinite(p->shear_b[i])) { why = "shear_b must be finite"; return FSLBM_E_INVALID; }
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
  d.ilm = 1.0 / lm;
  for (int a = 0; a < 3; ++a) {
    d.g[a] = p.g[a];
    d.hg[a] = 0.5 * p.g[a];
    d.glm[a] = p.g[a] / lm;
  }
  d.rhob_s = shifted ? p.rho_gas - 1.0 : p.rho_gas;
  d.rho0b = p.incompressible ? 1.0 : p.rho_gas;
  d.Lp = Lp;
  Consts<float>& f = com.kf;
  f.lp = (float)d.lp;
  f.lm = (float)d.lm;
  f.inv1p = (float)d.inv1p;
  f.ilm = (float)d.ilm;
  for (int a = 0; a < 3; ++a) {
    f.g[a] = (float)d.g[a];
    f.hg[a] = (float)d.hg[a];
    f.glm[a] = (float)d.glm[a];
  }
  f.rhob_s = (float)d.rhob_s;
  f.rho0b = (float)d.rho0b;
  f.Lp = (float)d.Lp;
  com.incomp = p.incompressible ? 1 : 0;
  com.stokes = p.stokes ? 1 : 0;
  com.moving = 0;
  for (int f = 0; f < 6; ++f)
    for (int a = 0; a < 3; ++a)
      if (!p.periodic[f / 2] && p.wall_u[f][a] != 0.0) com.moving = 1;
  for (int i = 0; i < 6; ++i) com.shear_b[i] = p.shear_b[i];
  com.sigma = p.sigma;
  com.plic = p.plic;
  com.rho_gas = p.rho_gas;
  com.scale = std::ldexp(1.0f, p.fp16_scale_log2);
  com.inv_scale = std::ldexp(1.0f, -p.fp16_scale_log2);
  com.grid.nx = p.nx;
  com.grid.ny = p.ny;
  com.grid.nz = p.nz;
  com.grid.N = p.nx * p.ny * p.nz;
  com.grid.px = p.periodic[0] ? 1 : 0;
  com.grid.py = p.periodic[1] ? 1 : 0;
  com.grid.pz = p.periodic[2] ? 1 : 0;
  com.grid.rx = grid_recip(p.nx);
  com.grid.ry = grid_recip(p.ny);
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
  *bytes = layout((size_t)p->nx * p->ny * p->nz, p->sigma != 0.0, p->plic == 2, storage_bytes(p->precision),
                  p->precision != FSLBM_FP16S).total;
  return FSLBM_OK;
}

}  // extern "C"

namespace {

// fslbm_init with the workspace given separately (the caller's buffer, or the
// library's static array for fslbm_init_static); parameters already checked.
fslbm_status init_impl(const fslbm_params* p, const fslbm_buffers* b, void* workspace, size_t workspace_bytes,
                       bool reorder, fslbm_ctx** out) {
  if (!b->f[0] || !b->f[1] || !b->flags || !b->mass || !b->phi[0] || !b->phi[1] || !workspace) {
    g_init_error = "a device buffer is NULL";
    return FSLBM_E_INVALID;
  }
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const Layout L = layout(N, p->sigma != 0.0, p->plic == 2, storage_bytes(p->precision), reorder);
  if (workspace_bytes < L.total) { g_init_error = "workspace too small"; return FSLBM_E_INVALID; }
  if (((uintptr_t)workspace) % ALIGN) { g_init_error = "workspace not 256-byte aligned"; return FSLBM_E_INVALID; }

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
  if (const char* e = std::getenv("FSLBM_IFACE_QUAD")) c->quad = std::max(0, std::min(2, std::atoi(e)));
  c->check_every = p->check_every;
  if (const char* e = std::getenv("FSLBM_CHECK_EVERY")) c->check_every = std::max(0, std::atoi(e));
  {
    const double um = p->u_max > 0.0 ? p->u_max : 0.4;
    c->u_max2 = um * um;
  }
  char* w = (char*)workspace;
  c->aux = (double*)(w + L.aux);
  int32_t** ep[4] = {&c->f_epoch, &c->new_epoch, &c->recv_epoch, &c->conv_epoch};
  for (int i = 0; i < 4; ++i) *ep[i] = (int32_t*)(w + L.epochs[i]);
  int32_t** ls[7] = {&c->listF, &c->listE, &c->listEP, &c->listNI, &c->listNL, &c->listR, &c->listI};
  for (int i = 0; i < 7; ++i) *ls[i] = (int32_t*)(w + L.lists[i]);
  c->counters = (int32_t*)(w + L.counters);
  c->reservoir = (double*)(w + L.scalars);
  c->ext_dev = (int32_t*)(w + L.extent);
  if (p->sigma != 0.0) c->kappa = (double*)(w + L.kappa);
  if (p->sigma != 0.0 && p->plic == 2) c->khf = (double*)(w + L.khf);
  c->wall_t = (double*)(w + L.wall_t);
  if (reorder) {
    c->islot = (int32_t*)(w + L.islot);
    c->rbuf = (void*)(w + L.rbuf);
    c->rcap = (int)L.rcap;
    // On by default in the FP32 form.  In FP64 the 512x320x512 tank's step
    // got 0.9 % slower with it (the sweep lost more than the interface kernel
    // saved); the FP16 sweeps always keep the other order.  FSLBM_REORDER=0 /
    // 1: off / on in the FP32 and FP64 forms; FSLBM_RCAP: fewer list entries
    // in the population buffer (the rest are written straight into the cells)
    c->reorder = p->precision == FSLBM_FP32;
    if (const char* e = std::getenv("FSLBM_REORDER")) c->reorder = std::atoi(e) != 0 && p->precision != FSLBM_FP16S;
    if (const char* e = std::getenv("FSLBM_RCAP")) c->rcap = std::max(0, std::min(c->rcap, std::atoi(e)));
  }
  {
    double tab[6 * Q];
    wall_table(*p, tab);
    HIPCHK(c, hipMemcpyAsync(c->wall_t, tab, sizeof(tab), hipMemcpyHostToDevice, c->stream), "wall terms");
    HIPCHK(c, hipStreamSynchronize(c->stream), "wall terms sync");
  }
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
  if ((e = launch_fill_i32(c->err, 16, 0, st)) != hipSuccess) return fail(dev_fail(c, e, "init scalars"));
  if ((e = launch_extent_init(c->ext_dev, st)) != hipSuccess) return fail(dev_fail(c, e, "init extent"));
  if ((e = launch_fill_f64(c->reservoir, 2, 0.0, st)) != hipSuccess) return fail(dev_fail(c, e, "init scalars"));
  if ((e = launch_check_flags(c->flags, c->com.grid, c->err, st)) != hipSuccess) return fail(dev_fail(c, e, "check flags"));
  int32_t herr = 0;
  if ((e = hipMemcpyAsync(&herr, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "read flag check"));
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail(dev_fail(c, e, "init sync"));
  if (herr & 1) { c->last_error = "unknown cell class in flags"; return fail(FSLBM_E_INVALID); }
  if (herr & 2) { c->last_error = "a liquid cell has a gas neighbour"; return fail(FSLBM_E_INVALID); }
  c->has_solid = (herr & 4) != 0;
  *out = c;
  return FSLBM_OK;
}

// The allocation-free workspace: one array per device, in the library's own
// device memory from the load of the code object until the process ends.  Its
// device address comes from hipGetSymbolAddress (once per device, with that
// device current); the name itself is only a host-side stand-in.
__device__ __align__(256) unsigned char scratch[FSLBM_STATIC_WORKSPACE_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
bool g_scratch_busy[MAX_DEVICES] = {};

}  // namespace

extern "C" {

fslbm_status fslbm_init(const fslbm_params* p, const fslbm_buffers* b, fslbm_ctx** out) {
  std::string why;
  fslbm_status s = check_params(p, why);
  if (s != FSLBM_OK) { g_init_error = why; return s; }
  if (!b || !out) { g_init_error = "buffers or out is NULL"; return FSLBM_E_INVALID; }
  // the interface-first buffers: FP32 and FP64 forms (FP16 keeps the other order)
  s = init_impl(p, b, b->workspace, b->workspace_bytes, p->precision != FSLBM_FP16S, out);
  if (s != FSLBM_OK) return s;
  fslbm_ctx* c = *out;
  c->ext_every = 16;
  if (const char* e = std::getenv("FSLBM_EXTENT_EVERY")) c->ext_every = std::max(0, std::atoi(e));
  if (c->ext_every > 0) {
    hipError_t e = hipHostMalloc((void**)&c->ext_host, 8 * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ext_ev[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ext_ev[1], hipEventDisableTiming);
    if (e != hipSuccess) {
      fslbm_destroy(c);
      *out = nullptr;
      return dev_fail(nullptr, e, "extent buffers");
    }
  }
  return FSLBM_OK;
}

fslbm_status fslbm_init_static(const fslbm_params* p, const fslbm_buffers* b, fslbm_ctx** out) {
  std::string why;
  fslbm_status s = check_params(p, why);
  if (s != FSLBM_OK) { g_init_error = why; return s; }
  if (!b || !out) { g_init_error = "buffers or out is NULL"; return FSLBM_E_INVALID; }
  const size_t need =
      layout((size_t)p->nx * p->ny * p->nz, p->sigma != 0.0, p->plic == 2, storage_bytes(p->precision), false).total;
  if (need > (size_t)FSLBM_STATIC_WORKSPACE_BYTES) {
    g_init_error = "the lattice needs " + std::to_string(need) + " bytes of workspace, more than the " +
                   std::to_string((size_t)FSLBM_STATIC_WORKSPACE_BYTES) + " of the static workspace";
    return FSLBM_E_CAPACITY;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_fail(nullptr, e, "current device");
  if (dev < 0 || dev >= MAX_DEVICES) { g_init_error = "device index beyond the static workspace table"; return FSLBM_E_UNSUPPORTED; }
  void* ws = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_busy[dev]) {
      g_init_error = "the static workspace of this device is held by another context (destroy it first)";
      return FSLBM_E_INVALID;
    }
    if (!g_scratch_ptr[dev]) {
      void* ptr = nullptr;
      e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess) return dev_fail(nullptr, e, "static workspace address");
      g_scratch_ptr[dev] = ptr;
    }
    ws = g_scratch_ptr[dev];
    g_scratch_busy[dev] = true;
  }
  s = init_impl(p, b, ws, (size_t)FSLBM_STATIC_WORKSPACE_BYTES, false, out);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (s != FSLBM_OK) g_scratch_busy[dev] = false;
  else (*out)->static_device = dev;
  return s;
}

// A new state may put fluid anywhere: the next step measures the extent
// again and launches every row until it has arrived (the stream is idle here,
// so no copy into the host slots is still in flight), and builds the
// interface list of the new classes.
static void forget_extent(fslbm_ctx* c) {
  c->ext_valid = -1;
  c->ext_pending = -1;
  c->list_ok = false;
}

static InitArgs init_args(fslbm_ctx* c) {
  InitArgs a;
  a.c = c->com;
  a.f = c->f[c->cur];
  a.flags = c->flags;
  a.mass = c->mass;
  a.phi = c->phi[c->cur];
  a.aux = c->aux;
  return a;
}

fslbm_status fslbm_set_equilibrium(fslbm_ctx* c, const double* rho, const double* u, const double* fill) {
  if (!c) return FSLBM_E_INVALID;
  if (!rho || !u || !fill) { c->last_error = "NULL field"; return FSLBM_E_INVALID; }
  HIPCHK(c, launch_set_equilibrium(init_args(c), c->p.precision, rho, u, fill, c->stream), "set_equilibrium");
  HIPCHK(c, hipStreamSynchronize(c->stream), "set_equilibrium sync");
  forget_extent(c);
  return FSLBM_OK;
}

fslbm_status fslbm_set_state(fslbm_ctx* c, const double* f, const double* mass, const double* fill,
                             double reservoir) {
  if (!c) return FSLBM_E_INVALID;
  if (!f || !mass || !fill) { c->last_error = "NULL field"; return FSLBM_E_INVALID; }
  HIPCHK(c, launch_set_state(init_args(c), c->p.precision, f, mass, fill, c->stream), "set_state");
  HIPCHK(c, launch_fill_f64(c->reservoir, 1, reservoir, c->stream), "set reservoir");
  HIPCHK(c, hipStreamSynchronize(c->stream), "set_state sync");
  forget_extent(c);
  return FSLBM_OK;
}

}  // extern "C"

namespace {

// Health check and totals of the current state: mass sum (FP64), counts and
// failing cells (k_stats).  Synchronises.  Returns FSLBM_E_INVARIANT or
// FSLBM_E_UNSTABLE (with the message set) if a check fails.
fslbm_status health(fslbm_ctx* c, double sc[2], int32_t cn[8], int32_t last[NCOUNT]) {
  HIPCHK(c, launch_fill_f64(c->acc, 1, 0.0, c->stream), "stats init");
  HIPCHK(c, launch_fill_i32(c->cnt, 8, 0, c->stream), "stats init");
  StatArgs a;
  a.c = c->com;
  a.f = c->f[c->cur];
  a.flags = c->flags;
  a.mass = c->mass;
  a.acc = c->acc;
  a.cnt = c->cnt;
  a.u_max2 = c->u_max2;
  HIPCHK(c, launch_stats(a, c->p.precision, c->stream), "stats");
  HIPCHK(c, hipMemcpyAsync(sc, c->reservoir, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream), "stats copy");
  HIPCHK(c, hipMemcpyAsync(cn, c->cnt, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "stats copy");
  for (int i = 0; i < NCOUNT; ++i) last[i] = 0;
  if (c->step > 0)
    HIPCHK(c, hipMemcpyAsync(last, c->counters + ((c->step - 1) & 1) * NCOUNT, NCOUNT * sizeof(int32_t),
                             hipMemcpyDeviceToHost, c->stream), "stats copy");
  HIPCHK(c, hipStreamSynchronize(c->stream), "stats sync");
  const std::string at = " (after " + std::to_string(c->step) + " steps)";
  if (cn[5] != 0) {
    c->last_error = std::to_string(cn[5]) + " cells break the cell-class rule (unknown class, or a liquid cell next "
                    "to a gas cell)" + at;
    return FSLBM_E_INVARIANT;
  }
  if (cn[1] != 0 || cn[4] != 0) {
    c->last_error = std::to_string(cn[1]) + " cells with NaN or non-positive density, " + std::to_string(cn[4]) +
                    " cells with |u| above " + std::to_string(std::sqrt(c->u_max2)) + " or NaN" + at;
    return FSLBM_E_UNSTABLE;
  }
  return FSLBM_OK;
}

// Rows the sweep of the next step launches (SweepArgs box), from the latest
// fluid extent that has arrived, widened by one cell per step since it was
// measured; a new measurement (of the rows of this box) starts every
// ext_every steps.  The host reads the extents back without waiting, except
// that it lets the device fall at most 2 ext_every steps behind: when the
// extent in use is that old and the next one has not arrived, it waits for
// that one, so that the box stays within 2 ext_every cells of the fluid.
hipError_t sweep_box(fslbm_ctx* c, SweepArgs& s) {
  s.box = 0;
  if (c->ext_every <= 0) return hipSuccess;
  if (c->ext_pending >= 0) {
    hipError_t q = hipEventQuery(c->ext_ev[c->ext_pending]);
    if (q == hipErrorNotReady && c->ext_valid >= 0 && c->step - c->ext_step[c->ext_valid] >= 2 * c->ext_every)
      q = hipEventSynchronize(c->ext_ev[c->ext_pending]);
    if (q == hipSuccess) {
      c->ext_valid = c->ext_pending;
      c->ext_pending = -1;
    } else if (q != hipErrorNotReady) {
      return q;
    }
  }
  const Grid& g = c->com.grid;
  int by0 = 0, bny = g.ny, bz0 = 0, bnz = g.nz;
  bool empty = false;
  if (c->ext_valid >= 0) {
    const int32_t* ex = c->ext_host + 4 * c->ext_valid;
    const int d = c->step - c->ext_step[c->ext_valid];
    if (ex[1] < 0) {
      empty = true;  // no fluid cell
    } else {
      by0 = g.py ? 0 : std::max(0, ex[0] - d);
      bny = g.py ? g.ny : std::min(g.ny - 1, ex[1] + d) - by0 + 1;
      bz0 = g.pz ? 0 : std::max(0, ex[2] - d);
      bnz = g.pz ? g.nz : std::min(g.nz - 1, ex[3] + d) - bz0 + 1;
    }
  }
  if (c->ext_pending < 0 && (c->ext_valid < 0 || c->step - c->ext_step[c->ext_valid] >= c->ext_every)) {
    const int slot = c->ext_valid == 0 ? 1 : 0;
    // the fluid of this step lies in this step's box (every row before the first extent)
    hipError_t e = empty ? launch_extent(c->flags, g, 0, 1, 0, 1, c->ext_dev, (void*)c->stream)
                         : launch_extent(c->flags, g, by0, bny, bz0, bnz, c->ext_dev, (void*)c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->ext_host + 4 * slot, c->ext_dev, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ext_ev[slot], c->stream);
    if (e != hipSuccess) return e;
    c->ext_step[slot] = c->step;
    c->ext_pending = slot;
  }
  if (c->ext_valid < 0) return hipSuccess;
  s.box = 1;
  if (empty) {  // one row (the sweep still resets the next counters)
    s.by0 = s.bz0 = 0;
    s.bny = s.bnz = 1;
    return hipSuccess;
  }
  s.by0 = by0;
  s.bny = bny;
  s.bz0 = bz0;
  s.bnz = bnz;
  return hipSuccess;
}

}  // namespace

extern "C" {

fslbm_status fslbm_step(fslbm_ctx* c, int32_t n, int32_t rule) {
  if (!c) return FSLBM_E_INVALID;
  if (n < 0) { c->last_error = "n must be >= 0"; return FSLBM_E_INVALID; }
  if (rule < FSLBM_RULE_FSK || rule > FSLBM_RULE_FSL_SHEAR) { c->last_error = "unknown rule"; return FSLBM_E_INVALID; }
  if (rule != FSLBM_RULE_FSK && c->p.tau == 1.0) {
    c->last_error = "this rule needs tau != 1 (n+ is not recoverable from a fully relaxed state)";
    return FSLBM_E_UNSUPPORTED;
  }
  if (c->has_solid && c->nwall < 0) {
    c->last_error = "solid cells present: set their wall table with fslbm_set_walls first";
    return FSLBM_E_INVALID;
  }
  for (int32_t i = 0; i < n; ++i) {
    StepLaunch L{};
    const int a = c->cur, b = 1 - c->cur;
    SweepArgs& s = L.sweep;
    s.c = c->com;
    s.fin = c->f[a];
    s.fout = c->f[b];
    s.flags = c->flags;
    s.mass_in = c->mass;
    s.mass = c->mass;
    s.phi_in = c->phi[a];
    s.phi_out = c->phi[b];
    s.aux = c->aux;
    s.f_epoch = c->f_epoch;
    s.listF = c->listF;
    s.listE = c->listE;
    s.listI = c->listI;
    s.counters = c->counters + (c->step & 1) * NCOUNT;
    s.counters_next = c->counters + ((c->step + 1) & 1) * NCOUNT;
    s.thr_hi = c->thr_hi;
    s.thr_lo = c->thr_lo;
    s.step = c->step;
    s.freeze = (c->p.freeze || c->p.hold_fill) ? 1 : 0;  // a held surface keeps its classes
    s.hold = c->p.hold_fill ? 1 : 0;
    s.cpr = 0;
    s.pairs = c->pairs;
    s.quad = c->quad;
    s.u_out = nullptr;
    s.kappa = c->kappa;
    s.khf = c->khf;
    s.wall_t = c->wall_t;
    s.wcells = c->wcells;
    s.wdelta = c->wdelta;
    s.wuw = c->wuw;
    s.nwall = c->nwall > 0 ? c->nwall : 0;
    s.surf_n = c->surf_n;
    s.surf_d = c->surf_d;
    // the plain step with the four-lane interface kernel runs it before the
    // sweep (the other variants after it)
    const bool extra = s.c.moving || s.c.sigma != 0.0 || s.c.plic || s.c.solid || s.c.surface;
    const bool order = c->reorder && c->quad && !extra;
    s.order = order ? 1 : 0;
    s.islot = c->islot;
    s.rbuf = c->rbuf;
    s.rcap = c->rcap;
    HIPCHK(c, sweep_box(c, s), "extent");
    ConvArgs& v = L.conv;
    v.c = c->com;
    v.fout = c->f[b];
    v.flags = c->flags;
    v.mass = c->mass;
    v.phi_out = c->phi[b];
    v.aux = c->aux;
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
    v.order = s.order;
    v.listI = c->listI;
    v.islot = c->islot;
    v.counters_next = s.counters_next;
    L.stream = (void*)c->stream;
    if (order) {
      // the interface list of the current classes, when no step has left it
      if (!c->list_ok)
        HIPCHK(c, launch_list_append(c->flags, c->com.grid, s.counters + C_I, c->listI, c->islot, c->stream),
               "interface list");
      HIPCHK(c, launch_iface(L, c->p.precision, rule), "interface launch");
    }
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
    if (!order) {
      if (s.nwall > 0) HIPCHK(c, launch_wall(L, c->p.precision), "wall launch");
      if (c->kappa) HIPCHK(c, launch_curvature(L), "curvature launch");
      HIPCHK(c, launch_iface(L, c->p.precision, rule), "interface launch");
    }
    if (!s.freeze) HIPCHK(c, launch_convert(L, c->p.precision), "conversion launch");
    c->list_ok = order;
    c->cur = b;
    c->step += 1;
    if (c->check_every > 0 && c->step % c->check_every == 0) {
      double sc[2];
      int32_t cn[8], last[NCOUNT];
      const fslbm_status hs = health(c, sc, cn, last);
      if (hs != FSLBM_OK) return hs;
    }
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
  a.aux = c->aux;
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
  double sc[2] = {0.0, 0.0};
  int32_t cn[8] = {0}, last[NCOUNT] = {0};
  const fslbm_status hs = health(c, sc, cn, last);
  if (hs == FSLBM_E_DEVICE) return hs;
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
  return hs;
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
  for (hipEvent_t ev : c->ext_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (c->ext_host) (void)hipHostFree(c->ext_host);
  if (c->static_device >= 0) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    g_scratch_busy[c->static_device] = false;
  }
  delete c;
  return e == hipSuccess ? FSLBM_OK : FSLBM_E_DEVICE;
}

const char* fslbm_last_error(const fslbm_ctx* c) {
  return c ? c->last_error.c_str() : g_init_error.c_str();
}

}  // extern "C"

// ------------------------------------------------------------ adjoint window
// Storage (all in the caller's window workspace):
//   - two hot states that the forward and recompute steps ping-pong between;
//   - a full checkpoint every K steps (state 0, K, 2K, ...);
//   - a ring of K step records: what the adjoint of a step needs, namely the
//     collision velocity of the liquid cells and, per interface cell in list
//     order, the pulled and own populations, fill and mass of time t.
// The backward pass rebuilds the records of a segment by re-running it from its
// checkpoint (the last segment's records are kept from the forward pass), then
// runs the reverse steps of the segment from the records.
struct fslbm_window {
  fslbm_ctx* ctx = nullptr;
  Common com;           // constants at forward time (g, rho_b, relaxation)
  int T = 0, K = 0, C = 0, rule = 0, precision = 0;
  int n_i = 0, cap = 1, nb_sweep = 0, nb_iface = 0;
  size_t N = 0;
  struct State {
    void* f;
    double* m;
    double* phi;
  };
  struct Record {
    void* u;       // [3][N] compute type
    void* f;       // [Q][cap] compute type
    void* own;     // [Q][cap] compute type
    double* phi;   // [cap]
    double* m;     // [cap]
    void* ui;      // [3][cap] compute type: collision velocity of the interface cells
    double* rho;   // [cap] collision density of the interface cells
  };
  std::vector<State> ckpt;  // states at t = jK
  State hot[2];             // hot[*].m is one shared array (mass is updated in place)
  std::vector<Record> rec;  // records of steps jK + k, k = 0..K-1, of one segment
  int rec_seg = -1;         // segment whose records the ring holds
  uint8_t* flags = nullptr;  // cell classes, fixed over the window
  void* lam[2] = {nullptr, nullptr};
  double* lam_m = nullptr;
  double* lphi[2] = {nullptr, nullptr};
  int32_t *listI = nullptr, *islot = nullptr, *bcount = nullptr, *n_dev = nullptr;
  uint64_t* ncls = nullptr;
  int32_t* nslot = nullptr;
  void* own = nullptr;
  double* phic = nullptr;
  double *part_sweep = nullptr, *part_iface = nullptr, *grads = nullptr;
  double* aux = nullptr;  // recompute steps (the context's stays untouched)
  int32_t* counters = nullptr;
  int32_t* fixed_count = nullptr;  // counter set whose interface count is n_i (for the fixed list)
  int32_t* listI_fwd = nullptr;
};

namespace {

struct WinLayout {
  // head (independent of the interface count)
  size_t flags, listI, islot, bcount, n_dev;
  // rest
  size_t ckpt, state_bytes, st_m, st_phi;
  size_t hot[2], hot_m;
  size_t rec, rec_bytes, rc_f, rc_own, rc_phi, rc_m, rc_ui, rc_rho;
  size_t ncls, nslot, lam[2], lam_m, lphi[2], own, phic, part_sweep, part_iface, grads, aux, counters,
      fixed_count, listI_fwd;
  size_t total;
};

WinLayout win_layout(const Grid& g, int precision, int T, int K, int n_i) {
  const size_t N = (size_t)g.N;
  const size_t sb = storage_bytes(precision);
  const size_t rb = precision == FSLBM_FP64 ? 8 : 4;  // compute type of the adjoint
  const size_t cap = (size_t)std::max(n_i, 1);
  const int C = (T + K - 1) / K;
  WinLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  L.flags = take(N);
  L.listI = take(4 * N);
  L.islot = take(4 * N);
  L.bcount = take(4 * (size_t)list_blocks(g));
  L.n_dev = take(4);
  // full state: f, mass, fill
  L.st_m = align_up(Q * N * sb);
  L.st_phi = L.st_m + align_up(8 * N);
  L.state_bytes = L.st_phi + align_up(8 * N);
  L.ckpt = take(L.state_bytes * (size_t)C);
  L.hot[0] = take(Q * N * sb + 0);
  L.hot[1] = take(Q * N * sb);
  L.hot_m = take(8 * N);
  const size_t hot_phi0 = take(8 * N);
  const size_t hot_phi1 = take(8 * N);
  (void)hot_phi0;
  (void)hot_phi1;
  // step record
  L.rc_f = align_up(3 * N * rb);
  L.rc_own = L.rc_f + align_up(Q * cap * rb);
  L.rc_phi = L.rc_own + align_up(Q * cap * rb);
  L.rc_m = L.rc_phi + align_up(8 * cap);
  L.rc_ui = L.rc_m + align_up(8 * cap);
  L.rc_rho = L.rc_ui + align_up(3 * cap * rb);
  L.rec_bytes = L.rc_rho + align_up(8 * cap);
  L.rec = take(L.rec_bytes * (size_t)K);
  L.ncls = take(8 * cap);
  L.nslot = take(4 * Q * cap);
  L.lam[0] = take(Q * N * rb);
  L.lam[1] = take(Q * N * rb);
  L.lam_m = take(8 * N);
  L.lphi[0] = take(8 * N);
  L.lphi[1] = take(8 * N);
  L.own = take(Q * cap * rb);
  L.phic = take(Q * cap * 8);
  L.part_sweep = take(3 * 8 * (size_t)adj_sweep_slots(g));
  L.part_iface = take(4 * 8 * (size_t)adj_iface_blocks(n_i));
  L.grads = take(4 * 8);
  L.aux = take(32 * N);
  L.counters = take(2 * NCOUNT * sizeof(int32_t));
  L.fixed_count = take(NCOUNT * sizeof(int32_t));
  L.listI_fwd = take(4 * N);
  L.total = o;
  return L;
}

fslbm_status window_checks(fslbm_ctx* c, int32_t T, int32_t K) {
  if (T < 1) { c->last_error = "window length T must be >= 1"; return FSLBM_E_INVALID; }
  if (K < 0) { c->last_error = "checkpoint spacing K must be >= 0 (0: ceil(sqrt(T)))"; return FSLBM_E_INVALID; }
  if (c->p.precision == FSLBM_FP16S) {
    c->last_error = "the adjoint window supports the FP64 and FP32 forms";
    return FSLBM_E_UNSUPPORTED;
  }
  if (!c->p.incompressible || c->p.stokes) {
    c->last_error = "the adjoint window supports the incompressible equilibrium with its quadratic term";
    return FSLBM_E_UNSUPPORTED;
  }
  if (c->p.sigma != 0.0) {
    c->last_error = "the adjoint window does not support surface tension";
    return FSLBM_E_UNSUPPORTED;
  }
  if (c->p.plic) {
    c->last_error = "the adjoint window does not support the PLIC interface position";
    return FSLBM_E_UNSUPPORTED;
  }
  if (c->has_solid) {
    c->last_error = "the adjoint window does not support solid cells";
    return FSLBM_E_UNSUPPORTED;
  }
  if (c->p.hold_fill || c->com.surface) {
    c->last_error = "the adjoint window does not support held fills or a prescribed surface";
    return FSLBM_E_UNSUPPORTED;
  }
  return FSLBM_OK;
}

int sqrt_spacing(int32_t T) {
  int k = (int)std::ceil(std::sqrt((double)T));
  while ((long long)k * k < T) ++k;
  return std::max(k, 1);
}

// Checkpoint spacing K of a window: as given (at most T), or for K = 0 the
// default: every step's record (K = T, no recompute pass in the backward
// pass) when that workspace fits in half the device memory free now, else
// ceil(sqrt T).  The default chosen for a window length is kept in the
// context, so that fslbm_window_workspace_size and fslbm_window_forward agree
// even though the caller allocates the workspace in between.
int window_spacing(fslbm_ctx* c, int32_t T, int32_t K, int n_i) {
  if (K != 0) return std::min(K, T);
  if (c->dflt_T == T) return c->dflt_K;
  const size_t all = win_layout(c->com.grid, c->p.precision, T, T, n_i).total;
  size_t free_b = 0, total_b = 0;
  const bool fits = hipMemGetInfo(&free_b, &total_b) == hipSuccess && all <= free_b / 2;
  c->dflt_T = T;
  c->dflt_K = fits ? T : sqrt_spacing(T);
  return c->dflt_K;
}

// One frozen forward step from state A (time t) to state B (time t+1) that
// also writes the step's record R.  The sweep stores the liquid cells'
// collision velocity; the interface kernel takes the window's fixed ascending
// list (so records are in list order) and stores its cells' inputs.
hipError_t window_step(fslbm_window* w, const fslbm_window::State& A, const fslbm_window::State& B,
                       const fslbm_window::Record& R, int parity, bool forward_pass) {
  fslbm_ctx* c = w->ctx;
  StepLaunch L{};
  SweepArgs& s = L.sweep;
  s.c = w->com;
  s.fin = A.f;
  s.fout = B.f;
  s.flags = w->flags;
  s.mass_in = A.m;
  s.mass = B.m;
  s.phi_in = A.phi;
  s.phi_out = B.phi;
  // the forward pass leaves the context's collision moments at the final state
  s.aux = forward_pass ? c->aux : w->aux;
  s.f_epoch = c->f_epoch;
  s.listF = c->listF;
  s.listE = c->listE;
  s.listI = w->listI_fwd;
  s.counters = w->counters + (parity & 1) * NCOUNT;
  s.counters_next = w->counters + ((parity + 1) & 1) * NCOUNT;
  s.thr_hi = c->thr_hi;
  s.thr_lo = c->thr_lo;
  s.step = 0;
  s.freeze = 1;
  s.cpr = 0;
  s.pairs = c->pairs;
  s.quad = c->quad;
  s.u_out = R.u;
  s.wall_t = c->wall_t;
  L.stream = (void*)c->stream;
  hipError_t e = launch_sweep(L, w->precision, w->rule);
  if (e != hipSuccess) return e;
  StepLaunch Li = L;
  Li.sweep.listI = w->listI;
  Li.sweep.counters = w->fixed_count;
  Li.sweep.rec_f = R.f;
  Li.sweep.rec_own = R.own;
  Li.sweep.rec_phi = R.phi;
  Li.sweep.rec_m = R.m;
  Li.sweep.rec_u = R.ui;
  Li.sweep.rec_rho = R.rho;
  Li.sweep.rec_cap = w->cap;
  return launch_iface(Li, w->precision, w->rule);
}

// State of time t during a pass over the window: checkpoint at multiples of K,
// else a hot buffer (t = T included).
const fslbm_window::State& state_at(const fslbm_window* w, int t) {
  if (t % w->K == 0 && t < w->T) return w->ckpt[t / w->K];
  return w->hot[t & 1];
}

// Steps t0 .. t1-1 writing records k = t - t0.  In the forward pass every
// state goes where state_at says (so checkpoints are written); in a recompute
// the outputs stay in the hot buffers.
hipError_t window_run(fslbm_window* w, int t0, int t1, bool forward_pass) {
  for (int t = t0; t < t1; ++t) {
    const fslbm_window::State& A = state_at(w, t);
    const fslbm_window::State& B = forward_pass ? state_at(w, t + 1) : w->hot[(t + 1) & 1];
    hipError_t e = window_step(w, A, B, w->rec[t - t0], t, forward_pass);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

extern "C" {

fslbm_status fslbm_set_walls(fslbm_ctx* c, int32_t n, const int32_t* cells, const double* delta,
                             const double* wall_u) {
  if (!c) return FSLBM_E_INVALID;
  if (n < 0) { c->last_error = "n must be >= 0"; return FSLBM_E_INVALID; }
  if (n > 0 && (!cells || !delta || !wall_u)) { c->last_error = "cells, delta or wall_u is NULL"; return FSLBM_E_INVALID; }
  HIPCHK(c, launch_fill_i32(c->err, 1, 0, c->stream), "wall check init");
  HIPCHK(c, launch_fill_i32(c->cnt + 3, 1, 0, c->stream), "wall check init");
  HIPCHK(c, launch_check_walls(c->flags, c->com.grid, cells, n, delta, wall_u, c->err, c->cnt + 3, c->stream),
         "wall check");
  int32_t h[2] = {0, 0};
  HIPCHK(c, hipMemcpyAsync(&h[0], c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "wall check copy");
  HIPCHK(c, hipMemcpyAsync(&h[1], c->cnt + 3, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "wall check copy");
  HIPCHK(c, hipStreamSynchronize(c->stream), "wall check sync");
  if (h[0] & 1) { c->last_error = "wall list: cell index out of range"; return FSLBM_E_INVALID; }
  if (h[0] & 2) { c->last_error = "wall list: cells not strictly ascending"; return FSLBM_E_INVALID; }
  if (h[0] & 4) { c->last_error = "wall list: a listed cell is solid"; return FSLBM_E_INVALID; }
  if (h[0] & 32) { c->last_error = "wall list: a listed cell has no link into a solid cell"; return FSLBM_E_INVALID; }
  if (h[0] & 8) { c->last_error = "wall distance outside (0, 1] on a link into a solid cell"; return FSLBM_E_INVALID; }
  if (h[0] & 16) { c->last_error = "wall velocity not finite"; return FSLBM_E_INVALID; }
  if (h[1] != n) {
    c->last_error = "wall list must hold every non-solid cell next to a solid cell (" + std::to_string(h[1]) +
                    " such cells, " + std::to_string(n) + " listed)";
    return FSLBM_E_INVALID;
  }
  c->wcells = cells;
  c->wdelta = delta;
  c->wuw = wall_u;
  c->nwall = n;
  c->com.solid = n > 0 ? 1 : 0;
  return FSLBM_OK;
}

fslbm_status fslbm_set_surface(fslbm_ctx* c, const double* normal, const double* offset) {
  if (!c) return FSLBM_E_INVALID;
  if (!normal || !offset) {
    c->surf_n = c->surf_d = nullptr;
    c->com.surface = 0;
    return FSLBM_OK;
  }
  if (!c->p.hold_fill) {
    c->last_error = "a prescribed surface needs params.hold_fill (the surface must stay where it is given)";
    return FSLBM_E_INVALID;
  }
  c->surf_n = normal;
  c->surf_d = offset;
  c->com.surface = 1;
  return FSLBM_OK;
}

fslbm_status fslbm_set_forcing(fslbm_ctx* c, const double g[3], double rho_gas) {
  if (!c) return FSLBM_E_INVALID;
  if (!g) { c->last_error = "g is NULL"; return FSLBM_E_INVALID; }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(g[a])) { c->last_error = "g must be finite"; return FSLBM_E_INVALID; }
  if (!(rho_gas > 0.0) || !std::isfinite(rho_gas)) { c->last_error = "rho_gas must be positive"; return FSLBM_E_INVALID; }
  for (int a = 0; a < 3; ++a) c->p.g[a] = g[a];
  c->p.rho_gas = rho_gas;
  make_constants(c->p, c->com, c->thr_hi, c->thr_lo);
  return FSLBM_OK;
}

fslbm_status fslbm_window_workspace_size(fslbm_ctx* c, int32_t T, int32_t K, size_t* bytes) {
  if (!c) return FSLBM_E_INVALID;
  if (!bytes) { c->last_error = "bytes is NULL"; return FSLBM_E_INVALID; }
  fslbm_status st = window_checks(c, T, K);
  if (st != FSLBM_OK) return st;
  HIPCHK(c, launch_fill_i32(c->cnt + 3, 1, 0, c->stream), "count init");
  HIPCHK(c, launch_count_iface(c->flags, c->com.grid, c->cnt + 3, c->stream), "count interface cells");
  int32_t n_i = 0;
  HIPCHK(c, hipMemcpyAsync(&n_i, c->cnt + 3, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "count copy");
  HIPCHK(c, hipStreamSynchronize(c->stream), "count sync");
  c->dflt_T = -1;  // a fresh default for this call
  *bytes = win_layout(c->com.grid, c->p.precision, T, window_spacing(c, T, K, n_i), n_i).total;
  return FSLBM_OK;
}

fslbm_status fslbm_window_forward(fslbm_ctx* c, int32_t T, int32_t K, int32_t rule, void* workspace,
                                  size_t workspace_bytes, fslbm_window** out) {
  if (!c) return FSLBM_E_INVALID;
  if (!out || !workspace) { c->last_error = "out or workspace is NULL"; return FSLBM_E_INVALID; }
  if (((uintptr_t)workspace) % ALIGN) { c->last_error = "window workspace not 256-byte aligned"; return FSLBM_E_INVALID; }
  c->list_ok = false;  // the window's steps keep their own lists; the next plain step rebuilds
  if (rule >= FSLBM_RULE_FSK_STRESS && rule <= FSLBM_RULE_FSL_SHEAR) {
    c->last_error = "the adjoint window supports the FSK and FSL rules (D = 0)";
    return FSLBM_E_UNSUPPORTED;
  }
  if (rule != FSLBM_RULE_FSK && rule != FSLBM_RULE_FSL) { c->last_error = "unknown rule"; return FSLBM_E_INVALID; }
  if (rule == FSLBM_RULE_FSL && c->p.tau == 1.0) {
    c->last_error = "FSL needs tau != 1 (n+ is not recoverable from a fully relaxed state)";
    return FSLBM_E_UNSUPPORTED;
  }
  fslbm_status st = window_checks(c, T, K);
  if (st != FSLBM_OK) return st;
  const Grid& g = c->com.grid;
  const size_t N = (size_t)g.N;
  char* wsp = (char*)workspace;
  // the head of the layout does not depend on the interface count
  const WinLayout H = win_layout(g, c->p.precision, T, 1, 0);
  if (workspace_bytes < H.ckpt) { c->last_error = "window workspace too small"; return FSLBM_E_INVALID; }
  fslbm_window* w = new (std::nothrow) fslbm_window();
  if (!w) { c->last_error = "out of host memory"; return FSLBM_E_INVALID; }
  auto fail = [&](fslbm_status s) {
    delete w;
    return s;
  };
  w->ctx = c;
  w->com = c->com;
  w->T = T;
  w->C = 0;
  w->rule = rule;
  w->precision = c->p.precision;
  w->N = N;
  w->flags = (uint8_t*)(wsp + H.flags);
  w->listI = (int32_t*)(wsp + H.listI);
  w->islot = (int32_t*)(wsp + H.islot);
  w->bcount = (int32_t*)(wsp + H.bcount);
  w->n_dev = (int32_t*)(wsp + H.n_dev);
  hipError_t e;
  if ((e = hipMemcpyAsync(w->flags, c->flags, N, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "window flags copy"));
  if ((e = launch_iface_list(w->flags, g, w->bcount, w->listI, w->islot, w->n_dev, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "interface list"));
  int32_t n_i = 0;
  if ((e = hipMemcpyAsync(&n_i, w->n_dev, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "interface count copy"));
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return fail(dev_fail(c, e, "window sync"));
  w->K = window_spacing(c, T, K, n_i);
  w->C = (T + w->K - 1) / w->K;
  const WinLayout L = win_layout(g, c->p.precision, T, w->K, n_i);
  if (workspace_bytes < L.total) {
    c->last_error = "window workspace too small (" + std::to_string(workspace_bytes) + " < " +
                    std::to_string(L.total) + " bytes)";
    return fail(FSLBM_E_INVALID);
  }
  w->n_i = n_i;
  w->cap = std::max(n_i, 1);
  w->nb_sweep = (int)adj_sweep_slots(g);
  w->nb_iface = (int)adj_iface_blocks(n_i);
  for (int j = 0; j < w->C; ++j) {
    char* b = wsp + L.ckpt + (size_t)j * L.state_bytes;
    w->ckpt.push_back({b, (double*)(b + L.st_m), (double*)(b + L.st_phi)});
  }
  // hot states: own population and fill buffers, one mass array (in place)
  w->hot[0] = {wsp + L.hot[0], (double*)(wsp + L.hot_m), (double*)(wsp + L.hot_m + align_up(8 * N))};
  w->hot[1] = {wsp + L.hot[1], (double*)(wsp + L.hot_m), (double*)(wsp + L.hot_m + 2 * align_up(8 * N))};
  for (int k = 0; k < w->K; ++k) {
    char* b = wsp + L.rec + (size_t)k * L.rec_bytes;
    w->rec.push_back({b, b + L.rc_f, b + L.rc_own, (double*)(b + L.rc_phi), (double*)(b + L.rc_m), b + L.rc_ui,
                      (double*)(b + L.rc_rho)});
  }
  w->ncls = (uint64_t*)(wsp + L.ncls);
  w->nslot = (int32_t*)(wsp + L.nslot);
  for (int i = 0; i < 2; ++i) {
    w->lam[i] = wsp + L.lam[i];
    w->lphi[i] = (double*)(wsp + L.lphi[i]);
  }
  w->lam_m = (double*)(wsp + L.lam_m);
  w->own = wsp + L.own;
  w->phic = (double*)(wsp + L.phic);
  w->part_sweep = (double*)(wsp + L.part_sweep);
  w->part_iface = (double*)(wsp + L.part_iface);
  w->grads = (double*)(wsp + L.grads);
  w->aux = (double*)(wsp + L.aux);
  w->counters = (int32_t*)(wsp + L.counters);
  w->fixed_count = (int32_t*)(wsp + L.fixed_count);
  w->listI_fwd = (int32_t*)(wsp + L.listI_fwd);
  if ((e = launch_fill_i32(w->fixed_count, NCOUNT, 0, c->stream)) != hipSuccess ||
      (e = launch_fill_i32(w->fixed_count + C_I, 1, n_i, c->stream)) != hipSuccess ||
      (e = launch_adj_topo(w->flags, g, w->listI, w->islot, n_i, w->cap, w->ncls, w->nslot, c->stream)) !=
          hipSuccess)
    return fail(dev_fail(c, e, "window topology"));

  // checkpoint 0: the current state of the context
  const size_t fb = Q * N * storage_bytes(c->p.precision);
  const fslbm_window::State& c0 = w->ckpt[0];
  if ((e = hipMemcpyAsync(c0.f, c->f[c->cur], fb, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c0.m, c->mass, 8 * N, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c0.phi, c->phi[c->cur], 8 * N, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "checkpoint copy"));
  if ((e = launch_fill_i32(w->counters, 2 * NCOUNT, 0, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "window counters"));
  // forward: segment by segment, records into the ring (the last segment's
  // stay for the backward pass), checkpoints at multiples of K
  for (int j = 0; j < w->C; ++j) {
    const int t0 = j * w->K, t1 = std::min(T, t0 + w->K);
    if ((e = window_run(w, t0, t1, true)) != hipSuccess) return fail(dev_fail(c, e, "window step"));
  }
  w->rec_seg = w->C - 1;
  // the final state becomes the context's current state
  const fslbm_window::State& fin = state_at(w, T);
  if ((e = hipMemcpyAsync(c->f[c->cur], fin.f, fb, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c->mass, fin.m, 8 * N, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(c->phi[c->cur], fin.phi, 8 * N, hipMemcpyDeviceToDevice, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "final state copy"));
  // no conversions happened: the last-step counters of the context read zero
  if ((e = launch_fill_i32(c->counters, 2 * NCOUNT, 0, c->stream)) != hipSuccess)
    return fail(dev_fail(c, e, "counters reset"));
  c->step += T;
  *out = w;
  return FSLBM_OK;
}

fslbm_status fslbm_window_backward(fslbm_window* w, const double* dL_df, const double* dL_dm, const double* dL_dphi,
                                   double* dL_df0, double* dL_dm0, double* dL_dphi0, double grads[4]) {
  if (!w || !w->ctx) return FSLBM_E_INVALID;
  fslbm_ctx* c = w->ctx;
  hipStream_t st = c->stream;
  const int T = w->T;
  HIPCHK(c, launch_adj_seed(w->com, w->flags, w->precision, dL_df, dL_dm, dL_dphi, w->lam[T & 1],
                            w->lam[(T + 1) & 1], w->lam_m, w->lphi[T & 1], w->lphi[(T + 1) & 1], st),
         "adjoint seed");
  HIPCHK(c, launch_fill_f64(w->part_sweep, 3 * (size_t)w->nb_sweep, 0.0, st), "adjoint partials");
  HIPCHK(c, launch_fill_f64(w->part_iface, 4 * (size_t)w->nb_iface, 0.0, st), "adjoint partials");
  for (int j = w->C - 1; j >= 0; --j) {
    const int t0 = j * w->K, t1 = std::min(T, t0 + w->K);
    if (w->rec_seg != j) {
      // rebuild the segment's records from its checkpoint
      HIPCHK(c, launch_fill_i32(w->counters, 2 * NCOUNT, 0, st), "window counters");
      HIPCHK(c, window_run(w, t0, t1, false), "recompute step");
      w->rec_seg = j;
    }
    for (int t = t1 - 1; t >= t0; --t) {
      const fslbm_window::Record& R = w->rec[t - t0];
      AdjArgs a{};
      a.c = w->com;
      a.u = R.u;
      a.rec_f = R.f;
      a.rec_own = R.own;
      a.rec_phi = R.phi;
      a.rec_m = R.m;
      a.rec_u = R.ui;
      a.rec_rho = R.rho;
      a.ncls = w->ncls;
      a.nslot = w->nslot;
      a.flags = w->flags;
      a.lam_in = w->lam[(t + 1) & 1];
      a.lam_out = w->lam[t & 1];
      a.lam_m = w->lam_m;
      a.lphi_in = w->lphi[(t + 1) & 1];
      a.lphi_out = w->lphi[t & 1];
      a.listI = w->listI;
      a.islot = w->islot;
      a.own = w->own;
      a.phic = w->phic;
      a.part_sweep = w->part_sweep;
      a.part_iface = w->part_iface;
      a.n_i = w->n_i;
      a.cap = w->cap;
      a.cpr = 0;
      HIPCHK(c, launch_adj_sweep(a, w->precision, st), "adjoint sweep");
      HIPCHK(c, launch_adj_iface(a, w->precision, w->rule, st), "adjoint interface");
      HIPCHK(c, launch_adj_iface2(a, w->precision, st), "adjoint gather");
    }
  }
  HIPCHK(c, launch_adj_out(w->com, w->flags, w->precision, w->lam[0], w->lam_m, w->lphi[0], dL_df0, dL_dm0,
                           dL_dphi0, st), "adjoint output");
  HIPCHK(c, launch_adj_reduce(w->part_sweep, w->nb_sweep, w->part_iface, w->nb_iface, w->grads, st),
         "adjoint reduce");
  double h[4] = {0.0, 0.0, 0.0, 0.0};
  HIPCHK(c, hipMemcpyAsync(h, w->grads, sizeof(h), hipMemcpyDeviceToHost, st), "gradient copy");
  HIPCHK(c, hipStreamSynchronize(st), "adjoint sync");
  if (grads)
    for (int i = 0; i < 4; ++i) grads[i] = h[i];
  return FSLBM_OK;
}

fslbm_status fslbm_window_info(const fslbm_window* w, int32_t info[4]) {
  if (!w || !info) return FSLBM_E_INVALID;
  info[0] = w->T;
  info[1] = w->K;
  info[2] = w->C;
  info[3] = w->n_i;
  return FSLBM_OK;
}

fslbm_status fslbm_window_destroy(fslbm_window* w) {
  if (!w) return FSLBM_E_INVALID;
  const hipError_t e = w->ctx ? hipStreamSynchronize(w->ctx->stream) : hipSuccess;
  delete w;
  return e == hipSuccess ? FSLBM_OK : FSLBM_E_DEVICE;
}

}  // extern "C"
