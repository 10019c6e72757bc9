// HIP kernels of the free-surface LBM step for gfx950.
//
// Per time step t (stream order, no host synchronisation):
//   k_sweep   pull stream + bounce-back + (interface cells) mass exchange,
//             interface geometry, FSK/FSL reconstruction; TRT collision;
//             fill update and filled/emptied classification with list append.
//   k_mark    E' = E minus N(F); new interface cells from gas next to filled
//             cells (initialised from their interface neighbours) and from
//             liquid next to E' cells.
//   k_commit  new cell classes; excess of filled cells.
//   k_share   excess split over interface neighbours; receiver list.
//   k_gather  receivers add the shares in ascending link order; fill refresh.
// Membership marks are step-stamped int arrays ("epochs"), so nothing needs to
// be cleared between steps; list counters are double buffered by step parity
// and the sweep of step t zeroes the set of step t+1.
#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"
#include "fslbm_stencil.hpp"

#include <algorithm>
#include <type_traits>

namespace fslbm {

constexpr int BLOCK = 256;

// ------------------------------------------------------------------ sweep
// Update of one interface cell from its loaded neighbourhood: mass exchange,
// geometry, reconstruction of the gas-side populations, TRT collision.  On exit
// d.f holds the post-collision populations; returns the new mass, the density
// (storage convention) and the velocity of the collision.
template <class F, int RULE>
__device__ __forceinline__ double iface_compute(IfaceData<F>& d, const Common& cm, typename F::R& rho_s,
                                                typename F::R (&u)[3]) {
  using R = typename F::R;
  constexpr bool SH = F::shifted;
  const Consts<R>& k = pick_consts<R>(cm);
  const bool incomp = cm.incomp, stokes = cm.stokes;

  // ---- mass exchange (FP64): dm = sum_q w (ft_q(x-c_q) - ft_qbar(x)); weight 1
  // to liquid, (phi_x + phi_s)/2 to interface, nothing from gas or walls
  uint32_t gasmask = 0;
  double dm = 0.0;
#define FSLBM_EXCH(q)                                              \
  {                                                                \
    const uint8_t ts = d.ty[q];                                    \
    if (ts == GAS) gasmask |= 1u << q;                             \
    if (ts == LIQ || ts == IFACE) {                                \
      const double diff = (double)d.f[q] - (double)d.own[OPP[q]];  \
      if (ts == LIQ) {                                             \
        dm = dm + diff;                                            \
      } else {                                                     \
        const double wgt = 0.5 * (d.phix + d.ph[q]);               \
        dm = dm + wgt * diff;                                      \
      }                                                            \
    }                                                              \
  }
  FSLBM_LINKS(FSLBM_EXCH)
#undef FSLBM_EXCH
  const double m_new = d.m + dm;

  if (gasmask) {
    // ---- interface geometry: n = -grad(phi)/|grad(phi)| by central
    // differences over the six axis neighbours (pull sources of links 1..6 are
    // x-1, x+1, y-1, y+1, z-1, z+1)
    const double gx = 0.5 * (phi_seen(d, 2) - phi_seen(d, 1));
    const double gy = 0.5 * (phi_seen(d, 4) - phi_seen(d, 3));
    const double gz = 0.5 * (phi_seen(d, 6) - phi_seen(d, 5));
    const double nrm2 = (gx * gx + gy * gy) + gz * gz;
    const bool have_n = nrm2 > 0.0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (have_n) {
      const double nrm = sqrt(nrm2);
      nv[0] = -gx / nrm;
      nv[1] = -gy / nrm;
      nv[2] = -gz / nrm;
    }
    const double dist = d.phix - 0.5;
    // ---- moments of time t from the own post-collision populations
    R rho_t, u_t[3];
    recover_moments<R, SH>(d.own, k, incomp, rho_t, u_t);
    const R rho0_t = rho0_of<R, SH>(rho_t, incomp);
    const R usq_t = usq_of(u_t);
#define FSLBM_REBUILD(q) rebuild<F, RULE, q>(d, gasmask, have_n, nv, dist, rho_t, rho0_t, u_t, usq_t, k, incomp, stokes);
    FSLBM_LINKS(FSLBM_REBUILD)
#undef FSLBM_REBUILD
  }

  // ---- TRT collision, Eq. (lbe2)
  if constexpr (sizeof(R) == 4)
    collide_f32<SH>(d.f, k, incomp, stokes, rho_s, u);
  else
    collide<R, SH>(d.f, k, incomp, stokes, rho_s, u);
  return m_new;
}

// Stream/collide sweep over liquid cells, one cell per lane; a block covers a
// chunk of one lattice row, so the row, its y and z and the source rows of
// every link are uniform (scalar) values.  Interface cells are appended to the
// interface list (one atomic per wavefront) and updated by k_iface; gas cells
// are skipped.
//
// Pull, Eq. (lbe1): f_q(x) = ft_q(x - c_q).  A source beyond a wall gives
// halfway bounce-back f_q(x) = ft_qbar(x).  Every load is unconditional with a
// 32-bit element offset from the buffer start (selected per lane), so all 19
// loads of a cell are in flight together.  MODEL 1 fixes the incompressible
// non-Stokes equilibrium at compile time; MODEL 0 reads both switches.

template <class F, int MODEL, bool WITH_U = false>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NCOUNT; ++i) a.counters_next[i] = 0;
  }
  const int row = (int)blockIdx.x / a.cpr;
  const int chunk = (int)blockIdx.x - row * a.cpr;
  const int y = row % g.ny, z = row / g.ny;
  const int x = chunk * BLOCK + (int)threadIdx.x;
  const unsigned rbase = (unsigned)row * (unsigned)g.nx;
  const uint8_t t = x < g.nx ? a.flags[rbase + x] : GAS;
  const int lane = (int)threadIdx.x & 63;
  {
    // interface cells -> list (wavefront-aggregated append)
    const unsigned long long b = __ballot(t == IFACE);
    if (b) {
      const int leader = __ffsll((long long)b) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&a.counters[C_I], __popcll(b));
      base = __shfl(base, leader);
      if (t == IFACE) a.listI[base + __popcll(b & ((1ull << lane) - 1ull))] = (int)(rbase + x);
    }
  }
  if (t != LIQ) return;

  // source rows (element offsets) of the nine (c_y, c_z) combinations
  const int ym = step_axis(y, -1, g.ny, g.py), yp = step_axis(y, 1, g.ny, g.py);
  const int zm = step_axis(z, -1, g.nz, g.pz), zp = step_axis(z, 1, g.nz, g.pz);
  auto row_of = [&](int sy, int sz) -> unsigned {
    return (sy < 0 || sz < 0) ? WALL_ROW : (unsigned)(sy + g.ny * sz) * (unsigned)g.nx;
  };
  // index: (c_y + 1) + 3 (c_z + 1); source row is (y - c_y, z - c_z)
  const unsigned srow[9] = {row_of(yp, zp), row_of(y, zp), row_of(ym, zp),
                            row_of(yp, z),  rbase,         row_of(ym, z),
                            row_of(yp, zm), row_of(y, zm), row_of(ym, zm)};
  // source columns (-1 beyond a wall at a row end: bounce-back)
  const int xm = step_axis(x, -1, g.nx, g.px), xp = step_axis(x, 1, g.nx, g.px);
  const unsigned N = (unsigned)g.N;  // 19 N < 2^32 is checked at init
  const S* __restrict__ fin = reinterpret_cast<const S*>(a.fin);

  // Every load is unconditional with a 32-bit element offset (selected per
  // lane), so all 19 loads of a cell are in flight together.  F::load_raw
  // keeps the FP16 form in its storage units (the collision absorbs the scale).
  R f[Q];
#define FSLBM_PULL(q)                                                                               \
  {                                                                                                 \
    const unsigned ro = srow[(CY[q] + 1) + 3 * (CZ[q] + 1)];                                        \
    const int sx = CX[q] == 1 ? xm : (CX[q] == -1 ? xp : x);                                        \
    const unsigned off = (ro == WALL_ROW || sx < 0) ? (unsigned)OPP[q] * N + rbase + (unsigned)x     \
                                                    : (unsigned)q * N + ro + (unsigned)sx;          \
    f[q] = F::load_raw(fin + off);                                                                  \
  }
  FSLBM_PULL(0)
  FSLBM_LINKS(FSLBM_PULL)
#undef FSLBM_PULL

  // ---- TRT collision, Eq. (lbe2)
  const Consts<R>& k = pick_consts<R>(a.c);
  const bool incomp = MODEL == 1 ? true : (bool)a.c.incomp;
  const bool stokes = MODEL == 1 ? false : (bool)a.c.stokes;
  R rho_s, u[3];
  if constexpr (sizeof(R) == 4)
    collide_f32_scaled<SH, F::scaled>(f, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  else
    collide<R, SH>(f, k, incomp, stokes, rho_s, u);
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
#pragma unroll
  for (int q = 0; q < Q; ++q) F::store_raw(fout + ((unsigned)q * N + rbase + (unsigned)x), f[q]);
  if constexpr (WITH_U) {
    // collision velocity, kept for the adjoint of this step
    R* __restrict__ uo = reinterpret_cast<R*>(a.u_out);
#pragma unroll
    for (int c = 0; c < 3; ++c) uo[(unsigned)c * N + rbase + (unsigned)x] = u[c];
  }
}

// FP16-storage sweep with two cells per lane (rows of even length): the 19
// populations of a pair are 4-byte aligned loads; the x-shifted neighbour comes
// from the adjacent lane by a wavefront shift (DPP), and the one element beyond
// the wavefront (or the row end: periodic wrap, or bounce-back at a wall) is a
// broadcast load from a wavefront-uniform address.  Liquid cells only; a pair
// store also covers an interface or gas partner (k_iface, which runs after this
// kernel, writes interface cells; gas slots are never read).
constexpr int DPP_WAVE_SHR1 = 0x138;  // lane i receives lane i-1
constexpr int DPP_WAVE_SHL1 = 0x130;  // lane i receives lane i+1

__device__ __forceinline__ float h_lo(uint32_t p) {
  return (float)__builtin_bit_cast(_Float16, (uint16_t)(p & 0xffffu));
}
__device__ __forceinline__ float h_hi(uint32_t p) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(p >> 16)); }
__device__ __forceinline__ float h_one(uint16_t v) { return (float)__builtin_bit_cast(_Float16, v); }
__device__ __forceinline__ uint32_t h_pack(float a, float b) {
  return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)a) |
         ((uint32_t)__builtin_bit_cast(uint16_t, (_Float16)b) << 16);
}

// Pull of the 19 populations of a lane's cell pair (see k_sweep_h2).  Phase 1
// issues all loads (19 pairs, 10 wavefront-edge elements); phase 2 shifts and
// selects, so no load waits on another link's data movement.
template <bool WALLS>
__device__ __forceinline__ void pull_pair(float (&f0)[Q], float (&f1)[Q], const uint16_t* __restrict__ fin,
                                          const Grid& g, size_t N, const unsigned (&srow)[9], unsigned rbase,
                                          int xl, int wx0, int wend, bool row_end) {
  uint32_t p[Q], e[Q];
#define FSLBM_LOAD2(q)                                                                            \
  {                                                                                               \
    const unsigned ro = srow[(CY[q] + 1) + 3 * (CZ[q] + 1)];                                      \
    const bool wall = WALLS && ro == WALL_ROW;                                                    \
    const uint16_t* own_qb = fin + (size_t)OPP[q] * N + rbase;                                    \
    const uint16_t* src = wall ? own_qb : fin + (size_t)q * N + ro;                               \
    p[q] = *reinterpret_cast<const uint32_t*>(src + xl);                                          \
    if (CX[q] == 1) {                                                                             \
      const uint16_t* ep = wx0 > 0 ? src + (wx0 - 1) : (g.px ? src + (g.nx - 1) : own_qb);        \
      e[q] = (uint32_t)*ep << 16;                                                                 \
    } else if (CX[q] == -1) {                                                                     \
      const uint16_t* ep = wend < g.nx ? src + wend : (g.px ? src : own_qb + (g.nx - 1));         \
      e[q] = (uint32_t)*ep;                                                                       \
    }                                                                                             \
  }
  FSLBM_LOAD2(0)
  FSLBM_LINKS(FSLBM_LOAD2)
#undef FSLBM_LOAD2
#define FSLBM_SHIFT2(q)                                                                           \
  {                                                                                               \
    const bool wall = WALLS && srow[(CY[q] + 1) + 3 * (CZ[q] + 1)] == WALL_ROW;                   \
    uint32_t lo = p[q], hi = p[q];                                                                \
    if (CX[q] == 1) {                                                                             \
      /* cell x0 <- x0-1 (lane 0: the edge element as the shift's fill), cell x0+1 <- x0 */       \
      const uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp((int)e[q], (int)p[q], DPP_WAVE_SHR1, 0xf, 0xf, false); \
      lo = wall ? p[q] : (nb >> 16);                                                              \
      hi = wall ? p[q] : (p[q] << 16);                                                            \
    } else if (CX[q] == -1) {                                                                     \
      /* cell x0 <- x0+1, cell x0+1 <- x0+2 (lane 63 and the row's last pair: the edge element) */ \
      const uint32_t nb = (uint32_t)__builtin_amdgcn_update_dpp((int)e[q], (int)p[q], DPP_WAVE_SHL1, 0xf, 0xf, false); \
      const uint32_t nx2 = row_end ? e[q] : nb;                                                   \
      lo = wall ? p[q] : (p[q] >> 16);                                                            \
      hi = wall ? p[q] : (nx2 << 16);                                                             \
    }                                                                                             \
    f0[q] = h_lo(lo);                                                                             \
    f1[q] = h_hi(hi);                                                                             \
  }
  FSLBM_SHIFT2(0)
  FSLBM_LINKS(FSLBM_SHIFT2)
#undef FSLBM_SHIFT2
}

template <int MODEL>
__global__ __launch_bounds__(BLOCK) void k_sweep_h2(SweepArgs a) {
  const Grid g = a.c.grid;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NCOUNT; ++i) a.counters_next[i] = 0;
  }
  const int row = (int)blockIdx.x / a.cpr;
  const int chunk = (int)blockIdx.x - row * a.cpr;
  const int y = row % g.ny, z = row / g.ny;
  const int x0 = (chunk * BLOCK + (int)threadIdx.x) * 2;
  const bool valid = x0 < g.nx;
  const int xl = valid ? x0 : 0;  // in-bounds pair for lanes past the row end
  const unsigned rbase = (unsigned)row * (unsigned)g.nx;
  const uint16_t fl2 = valid ? *reinterpret_cast<const uint16_t*>(a.flags + rbase + xl) : (uint16_t)0;
  const uint8_t tt[2] = {(uint8_t)(fl2 & 0xffu), (uint8_t)(fl2 >> 8)};
  const int lane = (int)threadIdx.x & 63;
  // interface cells -> list (wavefront-aggregated append, one cell of the pair at a time)
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const unsigned long long b = __ballot(tt[j] == IFACE);
    if (b) {
      const int leader = __ffsll((long long)b) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&a.counters[C_I], __popcll(b));
      base = __shfl(base, leader);
      if (tt[j] == IFACE) a.listI[base + __popcll(b & ((1ull << lane) - 1ull))] = (int)rbase + x0 + j;
    }
  }
  const bool liq = tt[0] == LIQ || tt[1] == LIQ;
  if (__ballot(liq) == 0) return;  // lanes exchange data below: whole wavefronts only

  const int ym = step_axis(y, -1, g.ny, g.py), yp = step_axis(y, 1, g.ny, g.py);
  const int zm = step_axis(z, -1, g.nz, g.pz), zp = step_axis(z, 1, g.nz, g.pz);
  auto row_of = [&](int sy, int sz) -> unsigned {
    return (sy < 0 || sz < 0) ? WALL_ROW : (unsigned)(sy + g.ny * sz) * (unsigned)g.nx;
  };
  const unsigned srow[9] = {row_of(yp, zp), row_of(y, zp), row_of(ym, zp),
                            row_of(yp, z),  rbase,         row_of(ym, z),
                            row_of(yp, zm), row_of(y, zm), row_of(ym, zm)};
  // first column of the wavefront (uniform over it; readfirstlane says so) and after it
  const int wx0 = __builtin_amdgcn_readfirstlane((chunk * BLOCK + ((int)threadIdx.x & ~63)) * 2);
  const int wend = wx0 + 128;
  const bool row_end = xl + 2 == g.nx;  // last pair of the row (its right neighbour is past the row)
  const size_t N = (size_t)g.N;
  const uint16_t* __restrict__ fin = reinterpret_cast<const uint16_t*>(a.fin);

  float f0[Q], f1[Q];
  // interior blocks (no source row beyond a y/z wall) take a select-only pull;
  // the few blocks on the y/z faces take the general one
  bool wall_rows = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) wall_rows = wall_rows || srow[i] == WALL_ROW;
  if (!wall_rows)
    pull_pair<false>(f0, f1, fin, g, N, srow, rbase, xl, wx0, wend, row_end);
  else
    pull_pair<true>(f0, f1, fin, g, N, srow, rbase, xl, wx0, wend, row_end);

  // ---- TRT collision, Eq. (lbe2), in storage units
  const Consts<float>& k = a.c.kf;
  const bool incomp = MODEL == 1 ? true : (bool)a.c.incomp;
  const bool stokes = MODEL == 1 ? false : (bool)a.c.stokes;
  float rho_s, u[3];
  collide_f32_scaled<true, true>(f0, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  collide_f32_scaled<true, true>(f1, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  if (liq) {
    uint16_t* __restrict__ fout = reinterpret_cast<uint16_t*>(a.fout) + rbase + x0;
#pragma unroll
    for (int q = 0; q < Q; ++q) *reinterpret_cast<uint32_t*>(fout + (size_t)q * N) = h_pack(f0[q], f1[q]);
  }
}

// Interface cells of the list built by the sweep: one cell per thread, in
// three phases -- load the whole neighbourhood (independent loads), compute in
// registers, store.
constexpr int IBLOCK = 64;  // interface-list kernels: one wavefront per block

template <class F, int RULE, bool REC = false>
__global__ __launch_bounds__(IBLOCK) void k_iface(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  const int n_i = a.counters[C_I];
  const S* __restrict__ fin = reinterpret_cast<const S*>(a.fin);
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
  const size_t N = (size_t)g.N;
  const float isc = a.c.inv_scale;
  for (int i = blockIdx.x * IBLOCK + threadIdx.x; i < n_i; i += gridDim.x * IBLOCK) {
    const int idx = a.listI[i];
    Nbr n;
    coords(g, idx, n.x, n.y, n.z);
    n.xm = step_axis(n.x, -1, g.nx, g.px);
    n.xp = step_axis(n.x, 1, g.nx, g.px);
    n.ym = step_axis(n.y, -1, g.ny, g.py);
    n.yp = step_axis(n.y, 1, g.ny, g.py);
    n.zm = step_axis(n.z, -1, g.nz, g.pz);
    n.zp = step_axis(n.z, 1, g.nz, g.pz);
    // ---- phase 1: loads.  Pull, Eq. (lbe1): f_q(x) = ft_q(x - c_q); beyond a
    // wall halfway bounce-back f_q(x) = ft_qbar(x).
    IfaceData<F> d;
    d.f[0] = F::load(fin + idx, isc);
    d.own[0] = d.f[0];
    d.ty[0] = IFACE;
    d.ph[0] = 0.0;
#define FSLBM_ILOAD(q)                                                                     \
  {                                                                                        \
    const int s = pull_source<q>(g, n);                                                    \
    const int sc = s >= 0 ? s : idx;                                                       \
    const size_t off = s >= 0 ? (size_t)q * N + (size_t)s : (size_t)OPP[q] * N + idx;      \
    d.f[q] = F::load(fin + off, isc);                                                      \
    d.own[q] = F::load(fin + (size_t)q * N + idx, isc);                                    \
    const uint8_t ts = a.flags[sc];                                                        \
    d.ty[q] = s >= 0 ? ts : WALL_CLASS;                                                    \
    d.ph[q] = a.phi_in[sc];                                                                \
  }
    FSLBM_LINKS(FSLBM_ILOAD)
#undef FSLBM_ILOAD
    d.m = a.mass_in[idx];
    d.phix = a.phi_in[idx];
    if constexpr (REC) {
      // what the adjoint of this step needs at this cell, in list order
      using RR = typename F::R;
      RR* rf = reinterpret_cast<RR*>(a.rec_f);
      RR* ro = reinterpret_cast<RR*>(a.rec_own);
      const unsigned cap = (unsigned)a.rec_cap;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        rf[(unsigned)q * cap + (unsigned)i] = d.f[q];
        ro[(unsigned)q * cap + (unsigned)i] = d.own[q];
      }
      a.rec_phi[i] = d.phix;
      a.rec_m[i] = d.m;
    }
    // ---- phase 2: interface treatment and collision
    R rho_s, u[3];
    const double m_new = iface_compute<F, RULE>(d, a.c, rho_s, u);
    // ---- phase 3: populations, fill level and classification (FP64 bookkeeping)
#pragma unroll
    for (int q = 0; q < Q; ++q) F::store(fout + (size_t)q * N + idx, d.f[q], a.c.scale);
    const double rho = SH ? 1.0 + (double)rho_s : (double)rho_s;
    a.mass[idx] = m_new;
    a.phi_out[idx] = m_new / rho;
    a.aux_rho[idx] = rho;
    a.aux_u[idx] = (double)u[0];
    a.aux_u[N + idx] = (double)u[1];
    a.aux_u[2 * N + idx] = (double)u[2];
    if (!a.freeze) {
      if (m_new > a.thr_hi * rho) {
        a.f_epoch[idx] = a.step;
        a.listF[atomicAdd(&a.counters[C_F], 1)] = idx;
      }
      if (m_new < a.thr_lo * rho) a.listE[atomicAdd(&a.counters[C_E], 1)] = idx;
    }
  }
}

// ------------------------------------------------------------ conversions
template <class F>
__device__ void init_new_from_gas(const ConvArgs& a, int c) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid& g = a.c.grid;
  int x, y, z;
  coords(g, c, x, y, z);
  double rs = 0.0, us0 = 0.0, us1 = 0.0, us2 = 0.0;
  int cnt = 0;
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    if (s < 0 || a.flags[s] == GAS) continue;
    rs = rs + a.aux_rho[s];
    us0 = us0 + a.aux_u[s];
    us1 = us1 + a.aux_u[(size_t)g.N + s];
    us2 = us2 + a.aux_u[2 * (size_t)g.N + s];
    ++cnt;
  }
  const double rbar = rs / (double)cnt;
  R ubar[3] = {(R)(us0 / (double)cnt), (R)(us1 / (double)cnt), (R)(us2 / (double)cnt)};
  const R rs_store = SH ? (R)(rbar - 1.0) : (R)rbar;
  const Consts<R>& k = pick_consts<R>(a.c);
  R out[Q];
  equilibrium_post<R, SH>(rs_store, ubar, k, a.c.incomp, a.c.stokes, out);
  S* fo = reinterpret_cast<S*>(a.fout);
#pragma unroll
  for (int q = 0; q < Q; ++q) F::store(fo + (size_t)q * g.N + c, out[q], a.c.scale);
  a.mass[c] = 0.0;
  a.aux_rho[c] = rbar;
}

template <class F>
__device__ void init_new_from_liquid(const ConvArgs& a, int c) {
  using S = typename F::S;
  const S* fo = reinterpret_cast<const S*>(a.fout);
  double r;
  if (F::shifted) {
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s = s + (double)F::load(fo + (size_t)q * a.c.grid.N + c, a.c.inv_scale);
    r = 1.0 + s;
  } else {
    r = (double)F::load(fo + c, a.c.inv_scale);
    for (int q = 1; q < Q; ++q) r = r + (double)F::load(fo + (size_t)q * a.c.grid.N + c, a.c.inv_scale);
  }
  a.mass[c] = r;
  a.aux_rho[c] = r;
}

template <class F>
__global__ __launch_bounds__(BLOCK) void k_mark(ConvArgs a) {
  const int nF = a.counters[C_F], nE = a.counters[C_E];
  const Grid& g = a.c.grid;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < nF + nE; i += gridDim.x * BLOCK) {
    const int c = i < nF ? a.listF[i] : a.listE[i - nF];
    int x, y, z;
    coords(g, c, x, y, z);
    if (i < nF) {
      for (int q = 1; q < Q; ++q) {
        const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
        if (s < 0 || a.flags[s] != GAS) continue;
        if (atomicExch(&a.new_epoch[s], a.step) != a.step) {
          a.listNI[atomicAdd(&a.counters[C_NI], 1)] = s;
          init_new_from_gas<F>(a, s);
        }
      }
    } else {
      bool protect = false;
      for (int q = 1; q < Q; ++q) {
        const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
        if (s >= 0 && a.f_epoch[s] == a.step) protect = true;
      }
      if (protect) continue;
      a.listEP[atomicAdd(&a.counters[C_EP], 1)] = c;
      for (int q = 1; q < Q; ++q) {
        const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
        if (s < 0 || a.flags[s] != LIQ) continue;
        if (atomicExch(&a.new_epoch[s], a.step) != a.step) {
          a.listNL[atomicAdd(&a.counters[C_NL], 1)] = s;
          init_new_from_liquid<F>(a, s);
        }
      }
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_commit(ConvArgs a) {
  const int nF = a.counters[C_F], nEP = a.counters[C_EP], nNI = a.counters[C_NI], nNL = a.counters[C_NL];
  const int tot = nF + nEP + nNI + nNL;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < tot; i += gridDim.x * BLOCK) {
    if (i < nF) {
      const int c = a.listF[i];
      a.flags[c] = LIQ;
      a.mass[c] = a.mass[c] - a.aux_rho[c];  // excess of a filled cell
    } else if (i < nF + nEP) {
      a.flags[a.listEP[i - nF]] = GAS;      // excess of an emptied cell: its mass
    } else if (i < nF + nEP + nNI) {
      a.flags[a.listNI[i - nF - nEP]] = IFACE;
    } else {
      a.flags[a.listNL[i - nF - nEP - nNI]] = IFACE;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_share(ConvArgs a) {
  const int nF = a.counters[C_F], nEP = a.counters[C_EP];
  const Grid& g = a.c.grid;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < nF + nEP; i += gridDim.x * BLOCK) {
    const int c = i < nF ? a.listF[i] : a.listEP[i - nF];
    int x, y, z;
    coords(g, c, x, y, z);
    int n_elig = 0;
    for (int q = 1; q < Q; ++q) {
      const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
      if (s >= 0 && a.flags[s] == IFACE) ++n_elig;
    }
    if (n_elig == 0) {
      atomicAdd(a.reservoir, a.mass[c]);
      continue;
    }
    a.mass[c] = a.mass[c] / (double)n_elig;
    a.conv_epoch[c] = a.step;
    for (int q = 1; q < Q; ++q) {
      const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
      if (s < 0 || a.flags[s] != IFACE) continue;
      if (atomicExch(&a.recv_epoch[s], a.step) != a.step) a.listR[atomicAdd(&a.counters[C_R], 1)] = s;
    }
  }
}

__global__ __launch_bounds__(BLOCK) void k_gather(ConvArgs a) {
  const int nR = a.counters[C_R];
  const Grid& g = a.c.grid;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < nR; i += gridDim.x * BLOCK) {
    const int r = a.listR[i];
    int x, y, z;
    coords(g, r, x, y, z);
    double m = a.mass[r];
    for (int q = 1; q < Q; ++q) {
      const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
      if (s >= 0 && a.conv_epoch[s] == a.step) m = m + a.mass[s];
    }
    a.mass[r] = m;
    a.phi_out[r] = m / a.aux_rho[r];
  }
}

// --------------------------------------------------------- init / export
__global__ __launch_bounds__(BLOCK) void k_fill_i32(int32_t* p, size_t n, int32_t v) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK) p[i] = v;
}

__global__ __launch_bounds__(BLOCK) void k_fill_f64(double* p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (size_t)gridDim.x * BLOCK) p[i] = v;
}

// cell classes valid and no liquid cell next to a gas cell
__global__ __launch_bounds__(BLOCK) void k_check_flags(const uint8_t* flags, Grid g, int32_t* err) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= g.N) return;
  const uint8_t t = flags[idx];
  if (t > LIQ) {
    atomicOr(err, 1);
    return;
  }
  if (t != LIQ) return;
  int x, y, z;
  coords(g, idx, x, y, z);
  for (int q = 1; q < Q; ++q) {
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    if (s >= 0 && flags[s] == GAS) atomicOr(err, 2);
  }
}

template <class F>
__global__ __launch_bounds__(BLOCK) void k_set_equilibrium(InitArgs a, const double* rho, const double* u,
                                                           const double* fill) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= a.c.grid.N) return;
  const uint8_t t = a.flags[idx];
  if (t == GAS) return;
  const size_t N = a.c.grid.N;
  const Consts<R>& k = pick_consts<R>(a.c);
  const double r = rho[idx];
  R uu[3] = {(R)u[idx], (R)u[N + idx], (R)u[2 * N + idx]};
  R out[Q];
  equilibrium_post<R, SH>(SH ? (R)(r - 1.0) : (R)r, uu, k, a.c.incomp, a.c.stokes, out);
  S* fo = reinterpret_cast<S*>(a.f);
#pragma unroll
  for (int q = 0; q < Q; ++q) F::store(fo + (size_t)q * N + idx, out[q], a.c.scale);
  if (t == IFACE) {
    a.phi[idx] = fill[idx];
    a.mass[idx] = fill[idx] * r;
    a.aux_rho[idx] = r;
    a.aux_u[idx] = u[idx];
    a.aux_u[N + idx] = u[N + idx];
    a.aux_u[2 * N + idx] = u[2 * N + idx];
  }
}

template <class F>
__global__ __launch_bounds__(BLOCK) void k_set_state(InitArgs a, const double* fsrc, const double* mass,
                                                     const double* fill) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= a.c.grid.N) return;
  const uint8_t t = a.flags[idx];
  if (t == GAS) return;
  const size_t N = a.c.grid.N;
  const Consts<R>& k = pick_consts<R>(a.c);
  S* fo = reinterpret_cast<S*>(a.f);
  R fl[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const double v = fsrc[(size_t)q * N + idx];
    fl[q] = SH ? (R)(v - WD[q]) : (R)v;
    F::store(fo + (size_t)q * N + idx, fl[q], a.c.scale);
    fl[q] = F::load(fo + (size_t)q * N + idx, a.c.inv_scale);
  }
  if (t == IFACE) {
    R rs, uu[3];
    recover_moments<R, SH>(fl, k, a.c.incomp, rs, uu);
    a.phi[idx] = fill[idx];
    a.mass[idx] = mass[idx];
    a.aux_rho[idx] = SH ? 1.0 + (double)rs : (double)rs;
    a.aux_u[idx] = uu[0];
    a.aux_u[N + idx] = uu[1];
    a.aux_u[2 * N + idx] = uu[2];
  }
}

template <class F>
__global__ __launch_bounds__(BLOCK) void k_fields(FieldArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= a.c.grid.N) return;
  const size_t N = a.c.grid.N;
  const uint8_t t = a.flags[idx];
  const S* fi = reinterpret_cast<const S*>(a.f);
  const Consts<R>& k = pick_consts<R>(a.c);
  if (a.flags_out) a.flags_out[idx] = t;
  if (a.phi_out) a.phi_out[idx] = t == LIQ ? 1.0 : (t == GAS ? 0.0 : a.phi[idx]);
  if (a.mass_out) a.mass_out[idx] = t == IFACE ? a.mass[idx] : 0.0;
  if (a.rhoc_out) a.rhoc_out[idx] = t == IFACE ? a.aux_rho[idx] : 0.0;
  if (a.uc_out)
    for (int d = 0; d < 3; ++d) a.uc_out[d * N + idx] = t == IFACE ? a.aux_u[d * N + idx] : 0.0;
  R fl[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) fl[q] = F::load(fi + (size_t)q * N + idx, a.c.inv_scale);
  if (a.f_out) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      a.f_out[(size_t)q * N + idx] = t == GAS ? 0.0 : (SH ? (double)fl[q] + WD[q] : (double)fl[q]);
  }
  if (a.rho_out || a.u_out) {
    R rs, uu[3];
    recover_moments<R, SH>(fl, k, a.c.incomp, rs, uu);
    const double r = SH ? 1.0 + (double)rs : (double)rs;
    if (a.rho_out) a.rho_out[idx] = t == GAS ? 0.0 : r;
    if (a.u_out)
      for (int d = 0; d < 3; ++d) a.u_out[d * N + idx] = t == GAS ? 0.0 : (double)uu[d];
  }
}

// total mass and health check: block partial sums into acc[0]; counts of
// liquid cells into cnt[0], bad cells into cnt[1], interface cells into cnt[2]
template <class F>
__global__ __launch_bounds__(BLOCK) void k_stats(StatArgs a) {
  using S = typename F::S;
  __shared__ double sm[BLOCK / 64];
  __shared__ int sl[BLOCK / 64];
  __shared__ int si[BLOCK / 64];
  double v = 0.0;
  int nl = 0, ni = 0;
  const S* fi = reinterpret_cast<const S*>(a.f);
  for (int idx = blockIdx.x * BLOCK + threadIdx.x; idx < a.c.grid.N; idx += gridDim.x * BLOCK) {
    const uint8_t t = a.flags[idx];
    if (t == GAS) continue;
    double r = 0.0;
    for (int q = 0; q < Q; ++q) r = r + (double)F::load(fi + (size_t)q * a.c.grid.N + idx, a.c.inv_scale);
    if (F::shifted) r = 1.0 + r;
    if (!(r > 0.0) || !isfinite(r)) atomicAdd(&a.cnt[1], 1);
    if (t == LIQ) {
      v += r;
      nl += 1;
    } else {
      v += a.mass[idx];
      ni += 1;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    v += __shfl_down(v, o);
    nl += __shfl_down(nl, o);
    ni += __shfl_down(ni, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sm[threadIdx.x >> 6] = v;
    sl[threadIdx.x >> 6] = nl;
    si[threadIdx.x >> 6] = ni;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    int cl = 0, ci = 0;
    for (int w = 0; w < BLOCK / 64; ++w) {
      s += sm[w];
      cl += sl[w];
      ci += si[w];
    }
    atomicAdd(a.acc, s);
    atomicAdd(&a.cnt[0], cl);
    atomicAdd(&a.cnt[2], ci);
  }
}

// ------------------------------------------------------------ launchers
static inline unsigned blocks_for(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }
static constexpr unsigned LIST_GRID = 512;
static constexpr unsigned IFACE_GRID = 8192;

template <class F>
static void sweep_form(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  SweepArgs a = L.sweep;
  const Grid& g = a.c.grid;
  a.cpr = (g.nx + BLOCK - 1) / BLOCK;
  const unsigned nb = (unsigned)a.cpr * (unsigned)g.ny * (unsigned)g.nz;
  if (a.u_out && a.c.incomp && !a.c.stokes)
    k_sweep<F, 1, true><<<nb, BLOCK, 0, st>>>(a);
  else if (a.c.incomp && !a.c.stokes)
    k_sweep<F, 1><<<nb, BLOCK, 0, st>>>(a);
  else
    k_sweep<F, 0><<<nb, BLOCK, 0, st>>>(a);
}

template <class F>
static void iface_form(const StepLaunch& L, int rule) {
  hipStream_t st = (hipStream_t)L.stream;
  // the interface count is on the device: enough one-wavefront blocks for
  // every cell up to IFACE_GRID * IBLOCK, grid-stride beyond
  const unsigned nb = std::min<unsigned>(IFACE_GRID, (unsigned)((L.sweep.c.grid.N + IBLOCK - 1) / IBLOCK));
  if (L.sweep.rec_f) {
    if (rule == 0)
      k_iface<F, 0, true><<<nb, IBLOCK, 0, st>>>(L.sweep);
    else
      k_iface<F, 1, true><<<nb, IBLOCK, 0, st>>>(L.sweep);
  } else if (rule == 0) {
    k_iface<F, 0><<<nb, IBLOCK, 0, st>>>(L.sweep);
  } else {
    k_iface<F, 1><<<nb, IBLOCK, 0, st>>>(L.sweep);
  }
}

template <class F>
static void convert_form(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  k_mark<F><<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_commit<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_share<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_gather<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
}

static void sweep_h2(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  SweepArgs a = L.sweep;
  const Grid& g = a.c.grid;
  a.cpr = (g.nx + 2 * BLOCK - 1) / (2 * BLOCK);
  const unsigned nb = (unsigned)a.cpr * (unsigned)g.ny * (unsigned)g.nz;
  if (a.c.incomp && !a.c.stokes)
    k_sweep_h2<1><<<nb, BLOCK, 0, st>>>(a);
  else
    k_sweep_h2<0><<<nb, BLOCK, 0, st>>>(a);
}

hipError_t launch_sweep(const StepLaunch& L, int precision, int rule) {
  (void)rule;  // the sweep covers liquid cells only; the rule acts in k_iface
  if (precision == 0) sweep_form<FormF64>(L);
  else if (precision == 1) sweep_form<FormF32>(L);
  else if (L.sweep.c.grid.nx % 2 == 0 && L.sweep.pairs) sweep_h2(L);
  else sweep_form<FormF16>(L);
  return hipGetLastError();
}

hipError_t launch_iface(const StepLaunch& L, int precision, int rule) {
  if (precision == 0) iface_form<FormF64>(L, rule);
  else if (precision == 1) iface_form<FormF32>(L, rule);
  else iface_form<FormF16>(L, rule);
  return hipGetLastError();
}

hipError_t launch_convert(const StepLaunch& L, int precision) {
  if (precision == 0) convert_form<FormF64>(L);
  else if (precision == 1) convert_form<FormF32>(L);
  else convert_form<FormF16>(L);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, void* stream) {
  k_fill_i32<<<1024, BLOCK, 0, (hipStream_t)stream>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, size_t n, double v, void* stream) {
  k_fill_f64<<<1024, BLOCK, 0, (hipStream_t)stream>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_check_flags(const uint8_t* flags, const Grid& g, int32_t* err, void* stream) {
  k_check_flags<<<blocks_for(g.N), BLOCK, 0, (hipStream_t)stream>>>(flags, g, err);
  return hipGetLastError();
}

template <class F>
static void set_eq_form(const InitArgs& a, const double* rho, const double* u, const double* fill, void* s) {
  k_set_equilibrium<F><<<blocks_for(a.c.grid.N), BLOCK, 0, (hipStream_t)s>>>(a, rho, u, fill);
}
hipError_t launch_set_equilibrium(const InitArgs& a, int precision, const double* rho, const double* u,
                                  const double* fill, void* stream) {
  if (precision == 0) set_eq_form<FormF64>(a, rho, u, fill, stream);
  else if (precision == 1) set_eq_form<FormF32>(a, rho, u, fill, stream);
  else set_eq_form<FormF16>(a, rho, u, fill, stream);
  return hipGetLastError();
}

template <class F>
static void set_state_form(const InitArgs& a, const double* f, const double* m, const double* fill, void* s) {
  k_set_state<F><<<blocks_for(a.c.grid.N), BLOCK, 0, (hipStream_t)s>>>(a, f, m, fill);
}
hipError_t launch_set_state(const InitArgs& a, int precision, const double* f, const double* mass,
                            const double* fill, void* stream) {
  if (precision == 0) set_state_form<FormF64>(a, f, mass, fill, stream);
  else if (precision == 1) set_state_form<FormF32>(a, f, mass, fill, stream);
  else set_state_form<FormF16>(a, f, mass, fill, stream);
  return hipGetLastError();
}

hipError_t launch_fields(const FieldArgs& a, int precision, void* stream) {
  const unsigned nb = blocks_for(a.c.grid.N);
  hipStream_t s = (hipStream_t)stream;
  if (precision == 0) k_fields<FormF64><<<nb, BLOCK, 0, s>>>(a);
  else if (precision == 1) k_fields<FormF32><<<nb, BLOCK, 0, s>>>(a);
  else k_fields<FormF16><<<nb, BLOCK, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_stats(const StatArgs& a, int precision, void* stream) {
  const unsigned nb = std::min<unsigned>(2048u, blocks_for(a.c.grid.N));
  hipStream_t s = (hipStream_t)stream;
  if (precision == 0) k_stats<FormF64><<<nb, BLOCK, 0, s>>>(a);
  else if (precision == 1) k_stats<FormF32><<<nb, BLOCK, 0, s>>>(a);
  else k_stats<FormF16><<<nb, BLOCK, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace fslbm
