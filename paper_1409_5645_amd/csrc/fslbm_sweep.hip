// Stream/collide sweep of the liquid cells for gfx950: the kernel that moves
// the populations (Eq. lbe1, lbe2), in one file of its own.  Every other step
// of the method is in fslbm_kernels.hip.
#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"
#include "fslbm_stencil.hpp"

namespace fslbm {

constexpr int BLOCK = 256;

// Stream/collide sweep over liquid cells, one cell per lane; a block covers a
// chunk of one lattice row, so the row, its y and z and the source rows of
// every link are uniform (scalar) values.  Interface cells are appended to the
// interface list (one atomic per wavefront) and updated by the interface
// kernel.  A wavefront without liquid cells exits; in one with liquid cells
// every lane of the row (but solid cells) pulls, collides and stores, so that
// its stores cover whole cache lines: a partly written line costs the memory
// system more than a whole one.  What it writes into gas cells is not a
// result (gas populations are never read; a cell that becomes interface is
// initialised in full).  The interface cells take one of two orders:
//   - order 0: the interface kernel runs after this one and overwrites them
//     (the FP16 and FP64 forms, a step with walls, surface tension, PLIC,
//     solids or an adjoint record, or any step with FSLBM_REORDER=0);
//   - order 1 (k_sweep<..., ORDER1>, the plain FP32 step, and FP64 with
//     FSLBM_REORDER=1): the interface kernel ran before this one and left
//     their populations in a list-ordered buffer; a wavefront with liquid or
//     interface cells stores them with its whole row segment, and the list
//     built here is that of the next step.  Not in the FP16 forms: there the
//     compiler fuses the collision's last FMA and the FP16 conversion into
//     one instruction where it can, and a choice between two values before
//     the store changes where it can, so the two FP16 sweeps would no longer
//     give the same bits (rounding explicitly cost the pair sweep 3 %).
//
// Pull, Eq. (lbe1): f_q(x) = ft_q(x - c_q).  A source beyond a wall gives
// halfway bounce-back f_q(x) = ft_qbar(x).  Every load is unconditional with a
// 32-bit element offset from the buffer start (selected per lane), so all 19
// loads of a cell are in flight together.  MODEL 1 fixes the incompressible
// non-Stokes equilibrium at compile time; MODEL 0 reads both switches.

template <class F, int MODEL, bool WITH_U = false, bool ORDER1 = false>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  if (!ORDER1 && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NCOUNT; ++i) a.counters_next[i] = 0;
  }
  const int brow = (int)blockIdx.x / a.cpr;
  const int chunk = (int)blockIdx.x - brow * a.cpr;
  const int y = a.box ? a.by0 + brow % a.bny : brow % g.ny;
  const int z = a.box ? a.bz0 + brow / a.bny : brow / g.ny;
  const int row = y + g.ny * z;
  const int x = chunk * (int)blockDim.x + (int)threadIdx.x;
  const unsigned rbase = (unsigned)row * (unsigned)g.nx;
  const uint8_t t = x < g.nx ? a.flags[rbase + x] : GAS;
  const int lane = (int)threadIdx.x & 63;
  if constexpr (!ORDER1) {
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
  // with the interface kernel first, a wavefront without liquid cells that
  // holds interface cells pulls nothing: it only stores their populations
  // from the list buffer
  const bool wliq = __ballot(t == LIQ) != 0ull;
  if (!wliq && (!ORDER1 || __ballot(t == IFACE) == 0ull)) return;
  if (x >= g.nx || t == SOLID) return;

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
  R rho_s = R(0.0), u[3] = {R(0.0), R(0.0), R(0.0)};
  if (ORDER1 && !wliq) {
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = R(0.0);
  } else {
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
  if (a.c.moving) {
    // moving walls (uniform branch): halfway bounce-back gains 2 w_q (c_q . u_w) / c_s^2,
    // in storage units for the FP16 form
    const double su = F::scaled ? (double)a.c.scale : 1.0;
#define FSLBM_WALLU(q)                                                         \
  {                                                                            \
    const double t = wall_term<q>(a.wall_t, xm, xp, ym, yp, zm, zp);           \
    if (t != 0.0) f[q] = f[q] + (R)(t * su);                                   \
  }
    FSLBM_LINKS(FSLBM_WALLU)
#undef FSLBM_WALLU
  }

  // ---- TRT collision, Eq. (lbe2)
  const Consts<R>& k = pick_consts<R>(a.c);
  const bool incomp = MODEL == 1 ? true : (bool)a.c.incomp;
  const bool stokes = MODEL == 1 ? false : (bool)a.c.stokes;
  if constexpr (sizeof(R) == 4)
    collide_f32_scaled<SH, F::scaled>(f, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  else
    collide<R, SH>(f, k, incomp, stokes, rho_s, u);
  }
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
  if constexpr (!ORDER1) {
#pragma unroll
    for (int q = 0; q < Q; ++q) F::store_raw(fout + ((unsigned)q * N + rbase + (unsigned)x), f[q]);
  } else {
    // With the interface kernel first (a wavefront with interface cells has
    // come this far, and every lane of the row but none past its end): the
    // list entry of time t of an interface cell, then its entry in the next
    // list.  The map is read at interface cells only; a wavefront with
    // interface cells writes its whole segment of it (-1 elsewhere), so no
    // line of it is left partly written.  An interface cell stores what the
    // interface kernel computed for it (a list entry beyond rcap: written
    // there directly, left alone here).
    const bool it = t == IFACE;
    int oslot = -1;
    if (it) oslot = a.islot[rbase + x];
    const int pos = wave_append_at(it, &a.counters_next[C_I], a.listI, (int)(rbase + x));
    if (__ballot(it) != 0ull) a.islot[rbase + x] = pos;
    const bool keep = it && (unsigned)oslot >= (unsigned)a.rcap;
    if (it && !keep) {
      const S* __restrict__ rb = reinterpret_cast<const S*>(a.rbuf) + oslot;
#pragma unroll
      for (int q = 0; q < Q; ++q) f[q] = F::load_raw(rb + (unsigned)q * (unsigned)a.rcap);
    }
    if (!keep) {
#pragma unroll
      for (int q = 0; q < Q; ++q) F::store_raw(fout + ((unsigned)q * N + rbase + (unsigned)x), f[q]);
    }
  }
  if constexpr (WITH_U) {
    // collision velocity of the row segment, kept for the adjoint of this step,
    // which reads it at liquid cells only: whole lines, and non-temporal
    // stores, as it is read once, in the reverse pass, long after (cached
    // stores would evict the window's hot state)
    {
      R* __restrict__ uo = reinterpret_cast<R*>(a.u_out);
#pragma unroll
      for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(u[c], &uo[(unsigned)c * N + rbase + (unsigned)x]);
    }
  }
}

// FP16-storage sweep with two cells per lane (rows of even length; always the
// order with the interface kernel after the sweep): the 19
// populations of a pair are 4-byte aligned loads; the x-shifted neighbour comes
// from the adjacent lane by a wavefront shift (DPP), and the one element beyond
// the wavefront (or the row end: periodic wrap, or bounce-back at a wall) is a
// broadcast load from a wavefront-uniform address.  As in k_sweep, a wavefront
// with liquid cells stores every pair of the row (but pairs with a solid cell),
// so that its stores cover whole cache lines; its results are those of the
// liquid cells.
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
// selects, so no load waits on another link's data movement.  A lane whose
// two cells are gas loads no pair: no liquid cell pulls from a gas cell (the
// interface layer lies between them), so its values reach only gas or
// interface slots, which the sweep's results do not use.
// All addresses are 32-bit byte offsets from the buffer start (the two-cells
// form is used only while 19 N populations of 2 bytes stay below 2^32 bytes),
// so the per-link source and edge offsets are a few 32-bit scalar operations
// and every load is base + 32-bit offset.
template <bool WALLS>
__device__ __forceinline__ void pull_pair(float (&f0)[Q], float (&f1)[Q], const char* __restrict__ fb,
                                          const Grid& g, unsigned N2, const unsigned (&srow2)[9], unsigned rbase2,
                                          unsigned xl2, int wx0, int wend, bool row_end, bool ld) {
  uint32_t p[Q], e[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) p[q] = 0u;
#define FSLBM_LOAD2(q)                                                                            \
  {                                                                                               \
    const unsigned ro = srow2[(CY[q] + 1) + 3 * (CZ[q] + 1)];                                     \
    const bool wall = WALLS && ro == WALL_ROW;                                                    \
    const unsigned own_qb = (unsigned)OPP[q] * N2 + rbase2;                                       \
    const unsigned src = wall ? own_qb : (unsigned)q * N2 + ro;                                   \
    if (ld) p[q] = *reinterpret_cast<const uint32_t*>(fb + (src + xl2));                          \
    if (CX[q] == 1) {                                                                             \
      const unsigned eo = wx0 > 0 ? src + 2u * (unsigned)(wx0 - 1)                                \
                                  : (g.px ? src + 2u * (unsigned)(g.nx - 1) : own_qb);            \
      e[q] = (uint32_t)*reinterpret_cast<const uint16_t*>(fb + eo) << 16;                         \
    } else if (CX[q] == -1) {                                                                     \
      const unsigned eo = wend < g.nx ? src + 2u * (unsigned)wend                                 \
                                      : (g.px ? src : own_qb + 2u * (unsigned)(g.nx - 1));        \
      e[q] = (uint32_t)*reinterpret_cast<const uint16_t*>(fb + eo);                               \
    }                                                                                             \
  }
  FSLBM_LOAD2(0)
  FSLBM_LINKS(FSLBM_LOAD2)
#undef FSLBM_LOAD2
#define FSLBM_SHIFT2(q)                                                                           \
  {                                                                                               \
    const bool wall = WALLS && srow2[(CY[q] + 1) + 3 * (CZ[q] + 1)] == WALL_ROW;                  \
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
  const int brow = (int)blockIdx.x / a.cpr;
  const int chunk = (int)blockIdx.x - brow * a.cpr;
  const int y = a.box ? a.by0 + brow % a.bny : brow % g.ny;
  const int z = a.box ? a.bz0 + brow / a.bny : brow / g.ny;
  const int row = y + g.ny * z;
  const int x0 = (chunk * (int)blockDim.x + (int)threadIdx.x) * 2;
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
  const int wx0 = __builtin_amdgcn_readfirstlane((chunk * (int)blockDim.x + ((int)threadIdx.x & ~63)) * 2);
  const int wend = wx0 + 128;
  const bool row_end = xl + 2 == g.nx;  // last pair of the row (its right neighbour is past the row)
  const unsigned N2 = 2u * (unsigned)g.N;  // bytes per population plane
  const char* __restrict__ fb = reinterpret_cast<const char*>(a.fin);
  unsigned srow2[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) srow2[i] = srow[i] == WALL_ROW ? WALL_ROW : 2u * srow[i];

  float f0[Q], f1[Q];
  // interior blocks (no source row beyond a y/z wall) take a select-only pull;
  // the few blocks on the y/z faces take the general one
  bool wall_rows = false;
#pragma unroll
  for (int i = 0; i < 9; ++i) wall_rows = wall_rows || srow[i] == WALL_ROW;
  const bool ld = tt[0] != GAS || tt[1] != GAS;  // lanes past the row end read as gas
  if (!wall_rows)
    pull_pair<false>(f0, f1, fb, g, N2, srow2, 2u * rbase, 2u * (unsigned)xl, wx0, wend, row_end, ld);
  else
    pull_pair<true>(f0, f1, fb, g, N2, srow2, 2u * rbase, 2u * (unsigned)xl, wx0, wend, row_end, ld);

  // ---- TRT collision, Eq. (lbe2), in storage units
  const Consts<float>& k = a.c.kf;
  const bool incomp = MODEL == 1 ? true : (bool)a.c.incomp;
  const bool stokes = MODEL == 1 ? false : (bool)a.c.stokes;
  float rho_s, u[3];
  collide_f32_scaled<true, true>(f0, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  collide_f32_scaled<true, true>(f1, k, incomp, stokes, a.c.scale, a.c.inv_scale, rho_s, u);
  if (valid && tt[0] != SOLID && tt[1] != SOLID) {
    char* __restrict__ fo = reinterpret_cast<char*>(a.fout);
    const unsigned o = 2u * (rbase + (unsigned)x0);
#pragma unroll
    for (int q = 0; q < Q; ++q) *reinterpret_cast<uint32_t*>(fo + ((unsigned)q * N2 + o)) = h_pack(f0[q], f1[q]);
  }
}

// Extent of the fluid (liquid and interface) cells in y and z: ext[0..3] =
// (ymin, ymax, zmin, zmax).  Only the rows of the box [y0, y0 + ny) x
// [z0, z0 + nz) are read (the caller knows the fluid lies inside it).  A lane
// reads 16 flag bytes of a row (one 16-byte load where the row allows); each
// block adds its extent to one of EXT_COPIES partial extents (one atomic per
// value; spread over copies so that the blocks do not queue on one address),
// and k_extent_final reduces the copies into ext[0..3] and resets them for the
// next measurement (k_extent_init sets them once, when the context is made).
constexpr int EBLOCK = 256;
constexpr int ECELLS = 16;
constexpr int ESTRIDE = 32;  // int32 between partial extents: one 128-byte line each

__device__ __forceinline__ void extent_reset(int32_t* e) {
  e[0] = 0x7fffffff;
  e[1] = -1;
  e[2] = 0x7fffffff;
  e[3] = -1;
}

__global__ void k_extent_init(int32_t* ext) {
  extent_reset(ext + ESTRIDE * (1 + (int)threadIdx.x));  // one thread per partial extent
}

__global__ __launch_bounds__(EBLOCK) void k_extent(const uint8_t* __restrict__ flags, Grid g, int y0, int ny, int z0,
                                                   int nz, int32_t* ext) {
  __shared__ int sm[4][EBLOCK / 64];
  const int lpr = (g.nx + ECELLS - 1) / ECELLS;
  const int total = ny * nz * lpr;  // < N / 16 + ny nz < 2^31
  int ymin = 0x7fffffff, ymax = -1, zmin = 0x7fffffff, zmax = -1;
  for (int k = (int)blockIdx.x * EBLOCK + (int)threadIdx.x; k < total; k += (int)gridDim.x * EBLOCK) {
    const int brow = k / lpr;
    const int x0 = (k - brow * lpr) * ECELLS;
    const int by = brow % ny;
    const int y = y0 + by, z = z0 + (brow - by) / ny;
    const size_t o = ((size_t)z * g.ny + (size_t)y) * (size_t)g.nx + (size_t)x0;
    bool fluid = false;
    if (x0 + ECELLS <= g.nx && (o & 15u) == 0u) {
      const uint4 v = *reinterpret_cast<const uint4*>(flags + o);
      const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int j = 0; j < ECELLS; ++j) {
        const uint32_t b = (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
        fluid = fluid || b == IFACE || b == LIQ;
      }
    } else {
      for (int j = 0; j < ECELLS && x0 + j < g.nx; ++j) fluid = fluid || flags[o + j] == IFACE || flags[o + j] == LIQ;
    }
    if (fluid) {
      ymin = min(ymin, y);
      ymax = max(ymax, y);
      zmin = min(zmin, z);
      zmax = max(zmax, z);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    ymin = min(ymin, __shfl_down(ymin, off));
    ymax = max(ymax, __shfl_down(ymax, off));
    zmin = min(zmin, __shfl_down(zmin, off));
    zmax = max(zmax, __shfl_down(zmax, off));
  }
  if ((threadIdx.x & 63) == 0) {
    sm[0][threadIdx.x >> 6] = ymin;
    sm[1][threadIdx.x >> 6] = ymax;
    sm[2][threadIdx.x >> 6] = zmin;
    sm[3][threadIdx.x >> 6] = zmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < EBLOCK / 64; ++w) {
      ymin = min(ymin, sm[0][w]);
      ymax = max(ymax, sm[1][w]);
      zmin = min(zmin, sm[2][w]);
      zmax = max(zmax, sm[3][w]);
    }
    if (ymax >= 0) {
      int32_t* e = ext + ESTRIDE * (1 + (int)(blockIdx.x % EXT_COPIES));
      atomicMin(&e[0], ymin);
      atomicMax(&e[1], ymax);
      atomicMin(&e[2], zmin);
      atomicMax(&e[3], zmax);
    }
  }
}

__global__ void k_extent_final(int32_t* ext) {
  const int c = (int)threadIdx.x;  // EXT_COPIES threads: one wavefront
  int v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = ext[ESTRIDE * (1 + c) + i];
  extent_reset(ext + ESTRIDE * (1 + c));
  for (int off = 32; off > 0; off >>= 1) {
    v[0] = min(v[0], __shfl_down(v[0], off));
    v[1] = max(v[1], __shfl_down(v[1], off));
    v[2] = min(v[2], __shfl_down(v[2], off));
    v[3] = max(v[3], __shfl_down(v[3], off));
  }
  if (c == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) ext[i] = v[i];
}

hipError_t launch_extent_init(int32_t* ext, void* stream) {
  static_assert(EXT_COPIES == 64, "k_extent_init and k_extent_final use one wavefront of EXT_COPIES lanes");
  k_extent_init<<<1, EXT_COPIES, 0, (hipStream_t)stream>>>(ext);
  return hipGetLastError();
}

hipError_t launch_extent(const uint8_t* flags, const Grid& g, int y0, int ny, int z0, int nz, int32_t* ext,
                         void* stream) {
  const long long total = (long long)ny * nz * ((g.nx + ECELLS - 1) / ECELLS);
  const unsigned nb = (unsigned)std::max<long long>(1, std::min<long long>(4096, (total + EBLOCK - 1) / EBLOCK));
  k_extent<<<nb, EBLOCK, 0, (hipStream_t)stream>>>(flags, g, y0, ny, z0, nz, ext);
  k_extent_final<<<1, EXT_COPIES, 0, (hipStream_t)stream>>>(ext);
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
template <class F>
static void sweep_form(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  SweepArgs a = L.sweep;
  const Grid& g = a.c.grid;
  // whole wavefronts, no more than a row needs (short rows would idle lanes)
  const int threads = std::min(BLOCK, 64 * ((g.nx + 63) / 64));
  a.cpr = (g.nx + threads - 1) / threads;
  const unsigned nb = (unsigned)a.cpr * (a.box ? (unsigned)a.bny * (unsigned)a.bnz : (unsigned)g.ny * (unsigned)g.nz);
  if constexpr (!F::scaled) {
    if (a.order) {
      // the interface kernel first (FP32 and FP64 forms; never with an adjoint record)
      if (a.c.incomp && !a.c.stokes)
        k_sweep<F, 1, false, true><<<nb, threads, 0, st>>>(a);
      else
        k_sweep<F, 0, false, true><<<nb, threads, 0, st>>>(a);
      return;
    }
  }
  if (a.u_out && a.c.incomp && !a.c.stokes)
    k_sweep<F, 1, true><<<nb, threads, 0, st>>>(a);
  else if (a.c.incomp && !a.c.stokes)
    k_sweep<F, 1><<<nb, threads, 0, st>>>(a);
  else
    k_sweep<F, 0><<<nb, threads, 0, st>>>(a);
}

static void sweep_h2(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  SweepArgs a = L.sweep;
  const Grid& g = a.c.grid;
  // whole wavefronts of cell pairs, no more than a row needs
  const int threads = std::min(BLOCK, 64 * ((g.nx + 127) / 128));
  a.cpr = (g.nx + 2 * threads - 1) / (2 * threads);
  const unsigned nb = (unsigned)a.cpr * (a.box ? (unsigned)a.bny * (unsigned)a.bnz : (unsigned)g.ny * (unsigned)g.nz);
  if (a.c.incomp && !a.c.stokes)
    k_sweep_h2<1><<<nb, threads, 0, st>>>(a);
  else
    k_sweep_h2<0><<<nb, threads, 0, st>>>(a);
}

hipError_t launch_sweep(const StepLaunch& L, int precision, int rule) {
  (void)rule;  // the sweep covers liquid cells only; the rule acts in k_iface
  if (L.sweep.order && precision == 2) return hipErrorInvalidValue;  // FP16 storage: interface kernel after the sweep
  if (precision == 0) sweep_form<FormF64>(L);
  else if (precision == 1) sweep_form<FormF32>(L);
  else if (L.sweep.c.grid.nx % 2 == 0 && L.sweep.pairs && !L.sweep.c.moving &&
           38.0 * (double)L.sweep.c.grid.N < 4294967296.0)
    sweep_h2(L);  // two cells per lane (moving walls take the one-cell form)
  else sweep_form<FormF16>(L);
  return hipGetLastError();
}

}  // namespace fslbm
