// HIP kernels of the free-surface LBM step for gfx950.
//
// Per time step t (stream order, no host synchronisation):
//   k_sweep   (fslbm_sweep.hip) pull stream + bounce-back + TRT collision of
//             the liquid cells; builds the interface-cell list.
//   k_iface   interface cells (k_iface4 in fslbm_iface4.hip for the plain
//             step): mass exchange, interface geometry, FSK/FSL
//             reconstruction, TRT collision, fill update and filled/emptied
//             classification with list append.
//   The plain step of the FP32 form runs k_iface4 first, on the list the
//   step before built, and k_sweep stores its populations (the
//   interface-first order of SweepArgs::order).
//   k_mark    E' = E minus N(F); new interface cells from gas next to filled
//             cells (initialised from their interface neighbours) and from
//             liquid next to E' cells.
//   k_share   excess of the filled and E' cells split over the neighbours
//             that are interface cells after the conversions; receiver list.
//   k_gather  receivers add the shares in ascending link order; fill refresh;
//             new cell classes.
// Membership marks are step-stamped int arrays ("epochs"), so nothing needs to
// be cleared between steps; list counters are double buffered by step parity
// and the sweep of step t (the interface kernel, when it runs first) zeroes
// the set of step t+1.  The cell classes keep
// their values of time t until k_gather: k_share takes the classes after the
// conversions from the marks (iface_after).
#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"
#include "fslbm_stencil.hpp"

#include <algorithm>
#include <type_traits>

namespace fslbm {

constexpr int BLOCK = 256;

// ------------------------------------------------------------------ sweep
// Boundary shear rate S^b (section 3.4) of the rules with D != 0, for an
// interface cell with a normal.  S is extrapolated from the bulk at order zero:
// it is read from the non-equilibrium of time t of the liquid neighbour x + c_k
// whose link points most directly into the liquid (largest -c_k.n / |c_k|,
// lowest k on ties; the cell's own populations if no neighbour is liquid), by
// Eq. (nqp) at leading order with the fourth-moment isotropy of D3Q19:
//   M = sum_q c_q c_q n+_q,   S = (lambda_+ / (2 c_s^2)) (M - I tr M / 5).
// In the basis {t1, t2, n} the tangential block of S is kept, the
// tangential-normal entries are zero (Eq. proj2) and the normal entry is S_nn/3
// (the closure holds P - P_b = Lambda_+ (S_nn - S^b_nn) on the links it
// rebuilds; Eq. (proj1) with sigma = 0 asks 2 nu S_nn = (2/3) Lambda_+ S_nn):
//   S^b = S - (S n) n^T - n (S n)^T + (n.S.n + S_nn/3) n n^T.
// Components [xx, yy, zz, xy, xz, yz]; the geometry is FP64.
template <class F>
__device__ __forceinline__ void boundary_shear(const IfaceData<F>& d, const Nbr& n, const Grid& g,
                                               const typename F::S* __restrict__ fin, float isc,
                                               const double (&nv)[3], const Consts<typename F::R>& k,
                                               bool incomp, bool stokes, typename F::R (&Sb)[6]) {
  using R = typename F::R;
  constexpr bool SH = F::shifted;
  int best = -1, bx = 0, by = 0, bz = 0;
  double best_v = 0.0;
#define FSLBM_BULK(kk)                                                               \
  if (d.ty[OPP[kk]] == LIQ) { /* x + c_k is the pull source of link kbar */           \
    const double cn = -cdot<kk>(nv);                                                 \
    const double len2 = kk <= 6 ? 1.0 : 2.0;                                         \
    const double v = cn < 0.0 ? -(cn * cn) / len2 : (cn * cn) / len2;                \
    if (best < 0 || v > best_v) {                                                    \
      best = kk;                                                                     \
      best_v = v;                                                                    \
      bx = CX[kk];                                                                   \
      by = CY[kk];                                                                   \
      bz = CZ[kk];                                                                   \
    }                                                                                \
  }
  FSLBM_LINKS(FSLBM_BULK)
#undef FSLBM_BULK
  R f[Q];
  if (best < 0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = d.own[q];
  } else {
    const int sx = step_axis(n.x, bx, g.nx, g.px), sy = step_axis(n.y, by, g.ny, g.py);
    const int sz = step_axis(n.z, bz, g.nz, g.pz);
    const unsigned s = (unsigned)(sx + g.nx * (sy + g.ny * sz));  // a liquid cell: inside the lattice
#pragma unroll
    for (int q = 0; q < Q; ++q) f[q] = F::load(fin + ((unsigned)q * (unsigned)g.N + s), isc);
  }
  R rho_n, u_n[3];
  recover_moments<R, SH>(f, k, incomp, rho_n, u_n);
  const R rho0_n = rho0_of<R, SH>(rho_n, incomp);
  const R usq_n = usq_of(u_n);
  R M[6] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
#define FSLBM_MNEQ(q)                                                                \
  {                                                                                  \
    const R fplus = R(0.5) * (f[q] + f[q + 1]);                                      \
    const R np = (fplus - e_plus<q>(rho_n, rho0_n, incomp, stokes, u_n, usq_n)) * k.inv1p; \
    const R n2 = R(2.0) * np;                                                        \
    M[0] = M[0] + R(CX[q] * CX[q]) * n2;                                             \
    M[1] = M[1] + R(CY[q] * CY[q]) * n2;                                             \
    M[2] = M[2] + R(CZ[q] * CZ[q]) * n2;                                             \
    M[3] = M[3] + R(CX[q] * CY[q]) * n2;                                             \
    M[4] = M[4] + R(CX[q] * CZ[q]) * n2;                                             \
    M[5] = M[5] + R(CY[q] * CZ[q]) * n2;                                             \
  }
  FSLBM_MNEQ(1) FSLBM_MNEQ(3) FSLBM_MNEQ(5) FSLBM_MNEQ(7) FSLBM_MNEQ(9) FSLBM_MNEQ(11) FSLBM_MNEQ(13)
  FSLBM_MNEQ(15) FSLBM_MNEQ(17)
#undef FSLBM_MNEQ
  const R tr5 = ((M[0] + M[1]) + M[2]) / R(5.0);
  const R fs = R(1.5) * k.lp;  // lambda_+ / (2 c_s^2)
  double S[6];
  S[0] = (double)(fs * (M[0] - tr5));
  S[1] = (double)(fs * (M[1] - tr5));
  S[2] = (double)(fs * (M[2] - tr5));
  S[3] = (double)(fs * M[3]);
  S[4] = (double)(fs * M[4]);
  S[5] = (double)(fs * M[5]);
  // normal entry of the boundary value: n.S.n / 3
  const double ndg = (S[0] * (nv[0] * nv[0]) + S[1] * (nv[1] * nv[1])) + S[2] * (nv[2] * nv[2]);
  const double nof = (S[3] * (nv[0] * nv[1]) + S[4] * (nv[0] * nv[2])) + S[5] * (nv[1] * nv[2]);
  const double s_nn = (ndg + 2.0 * nof) / 3.0;
  // S^b = P S P + s_nn n n^T
  double Sn[3];
  Sn[0] = (S[0] * nv[0] + S[3] * nv[1]) + S[4] * nv[2];
  Sn[1] = (S[3] * nv[0] + S[1] * nv[1]) + S[5] * nv[2];
  Sn[2] = (S[4] * nv[0] + S[5] * nv[1]) + S[2] * nv[2];
  const double kk = ((nv[0] * Sn[0] + nv[1] * Sn[1]) + nv[2] * Sn[2]) + s_nn;
  constexpr int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int i = 0; i < 6; ++i)
    Sb[i] = (R)(((S[i] - Sn[A[i]] * nv[B[i]]) - nv[A[i]] * Sn[B[i]]) + kk * (nv[A[i]] * nv[B[i]]));
}

// Update of one interface cell from its loaded neighbourhood: mass exchange,
// geometry, reconstruction of the gas-side populations, TRT collision.  On exit
// d.f holds the post-collision populations; returns the new mass, the density
// (storage convention) and the velocity of the collision.
template <class F, int RULE, bool EXTRA>
__device__ __forceinline__ double iface_compute(IfaceData<F>& d, const Common& cm, typename F::R& rho_s,
                                                typename F::R (&u)[3], const Nbr& nb,
                                                const typename F::S* __restrict__ fin, double drho,
                                                const uint8_t* __restrict__ flags = nullptr,
                                                const double* __restrict__ phi = nullptr,
                                                const double* __restrict__ surf_n = nullptr,
                                                const double* __restrict__ surf_d = nullptr) {
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
    bool have_n = nrm2 > 0.0;
    double nv[3] = {0.0, 0.0, 0.0};
    if (have_n) {
      const double nrm = sqrt(nrm2);
      nv[0] = -gx / nrm;
      nv[1] = -gy / nrm;
      nv[2] = -gz / nrm;
    }
    double dist = d.phix - 0.5;
    if constexpr (EXTRA && (RULE & 1) != 0) {
      // FSL link distances from the plane that cuts the cell's fill (PLIC),
      // with the height-function normal where its columns are complete
      if (cm.plic == 2 && have_n) hf_normal(cm.grid, nb.x, nb.y, nb.z, flags, phi, nv);
      if (cm.plic && have_n) dist = plic_plane_offset(d.phix, nv);
    }
    if constexpr (EXTRA) {
      // a prescribed surface: the given plane (section 2.2: each boundary link
      // meets it at x_b + delta c_q)
      if (cm.surface) {
        const size_t ci = (size_t)nb.x + (size_t)cm.grid.nx * ((size_t)nb.y + (size_t)cm.grid.ny * (size_t)nb.z);
        const size_t Nn = (size_t)cm.grid.N;
        nv[0] = surf_n[ci];
        nv[1] = surf_n[Nn + ci];
        nv[2] = surf_n[2 * Nn + ci];
        dist = surf_d[ci];
        have_n = true;
      }
    }
    // ---- moments of time t from the own post-collision populations
    R rho_t, u_t[3];
    recover_moments<R, SH>(d.own, k, incomp, rho_t, u_t);
    const R rho0_t = rho0_of<R, SH>(rho_t, incomp);
    const R usq_t = usq_of(u_t);
    // boundary shear rate for the rules with D != 0: from the bulk (needs the
    // local basis) or prescribed
    R Sb[6] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
    const bool stress = ((RULE & 2) && have_n) || (RULE & 4);
    if constexpr ((RULE & 2) != 0) {
      if (stress) boundary_shear<F>(d, nb, cm.grid, fin, cm.inv_scale, nv, k, incomp, stokes, Sb);
    }
    if constexpr ((RULE & 4) != 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) Sb[i] = (R)cm.shear_b[i];
    }
    // Laplace pressure: the boundary term takes P_b - sigma kappa (Eq.
    // freeboundary); drho = 3 sigma kappa comes from k_curvature (0 without a normal)
    R rhob_c = k.rhob_s, rho0b_c = k.rho0b;
    if constexpr (EXTRA) {
      if (cm.sigma != 0.0) {
        rhob_c = (R)((double)k.rhob_s - drho);
        if (!incomp) rho0b_c = (R)(cm.rho_gas - drho);
      }
    }
#define FSLBM_REBUILD(q) \
  rebuild<F, RULE, q>(d, gasmask, have_n, nv, dist, rho_t, rho0_t, u_t, usq_t, k, incomp, stokes, Sb, stress, \
                      rhob_c, rho0b_c);
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

// Interface cells of the list built by the sweep: one cell per thread, in
// three phases -- load the whole neighbourhood (independent loads), compute in
// registers, store.
constexpr int IBLOCK = 64;  // interface-list kernels: one wavefront per block

// EXTRA: moving walls, surface tension or the PLIC interface position present
// (a separate instantiation, so that the plain path keeps its registers).
// Waves per SIMD the FP32-arithmetic forms are compiled for (the FP64 form
// takes what it needs): 4 (128 VGPRs) for the plain FSK and FSL rules, 3 (168)
// for the rules with a boundary shear and the EXTRA variants, 2 for the EXTRA
// variant of FSL with a prescribed shear; each without spills.
template <class F, int RULE, bool EXTRA>
constexpr int iface_waves() {
  if (sizeof(typename F::R) != 4) return 1;
  if (EXTRA) return RULE == 5 ? 2 : 3;
  return (RULE & 6) ? 3 : 4;
}

template <class F, int RULE, bool REC = false, bool EXTRA = false>
__global__ __launch_bounds__(IBLOCK, (iface_waves<F, RULE, EXTRA>())) void k_iface(SweepArgs a) {
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
    if (EXTRA && a.c.moving) {
      // moving walls (uniform branch): halfway bounce-back gains 2 w_q (c_q . u_w) / c_s^2
#define FSLBM_IWALLU(q)                                                                        \
  {                                                                                            \
    const double t = wall_term<q>(a.wall_t, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp);               \
    if (t != 0.0) d.f[q] = d.f[q] + (R)t;                                                      \
  }
      FSLBM_LINKS(FSLBM_IWALLU)
#undef FSLBM_IWALLU
    }
    d.m = a.mass_in[idx];
    d.phix = a.phi_in[idx];
    if constexpr (EXTRA) {
      if (a.c.solid) {
        // solid pull sources (class SOLID, inside the grid): the cell's own fill
        // for the geometry, the wall closure for the populations
        uint32_t sm = 0, up = 0;
#define FSLBM_ISOLID(q)                                                       \
  if (d.ty[q] == WALL_CLASS && pull_source<q>(g, n) >= 0) sm |= 1u << q;      \
  if (d.ty[q] == LIQ || d.ty[q] == IFACE) up |= 1u << q;
        FSLBM_LINKS(FSLBM_ISOLID)
#undef FSLBM_ISOLID
        if (sm) {
          const int slot = wall_slot(a.wcells, a.nwall, idx);
          if (slot >= 0) solid_links<R>(d.f, d.own, sm, up, slot, a.nwall, a.wdelta, a.wuw);
#pragma unroll
          for (int q = 1; q < Q; ++q)
            if ((sm >> q) & 1u) d.ph[q] = d.phix;
        }
      }
    }
    if constexpr (REC) {
      // what the adjoint of this step needs at this cell, in list order
      // (non-temporal stores: read once, in the reverse pass)
      using RR = typename F::R;
      RR* rf = reinterpret_cast<RR*>(a.rec_f);
      RR* ro = reinterpret_cast<RR*>(a.rec_own);
      const unsigned cap = (unsigned)a.rec_cap;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        __builtin_nontemporal_store(d.f[q], &rf[(unsigned)q * cap + (unsigned)i]);
        __builtin_nontemporal_store(d.own[q], &ro[(unsigned)q * cap + (unsigned)i]);
      }
      __builtin_nontemporal_store(d.phix, &a.rec_phi[i]);
      __builtin_nontemporal_store(d.m, &a.rec_m[i]);
    }
    // ---- phase 2: interface treatment and collision
    R rho_s, u[3];
    const double drho = (EXTRA && a.c.sigma != 0.0) ? a.kappa[i] : 0.0;
    const double m_new = iface_compute<F, RULE, EXTRA>(d, a.c, rho_s, u, n, fin, drho, a.flags, a.phi_in, a.surf_n,
                                                       a.surf_d);
    // ---- phase 3: populations, fill level and classification (FP64 bookkeeping)
#pragma unroll
    for (int q = 0; q < Q; ++q) F::store(fout + (size_t)q * N + idx, d.f[q], a.c.scale);
    const double rho = SH ? 1.0 + (double)rho_s : (double)rho_s;
    if constexpr (REC) {
      typename F::R* ru = reinterpret_cast<typename F::R*>(a.rec_u);
      const unsigned cap = (unsigned)a.rec_cap;
#pragma unroll
      for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(u[c], &ru[(unsigned)c * cap + (unsigned)i]);
      __builtin_nontemporal_store(rho, &a.rec_rho[i]);
    }
    a.mass[idx] = a.hold ? d.m : m_new;
    a.phi_out[idx] = a.hold ? d.phix : m_new / rho;
    *reinterpret_cast<double4*>(a.aux + 4 * (size_t)idx) = make_double4(rho, (double)u[0], (double)u[1], (double)u[2]);
    if (!a.freeze) {
      const bool filled = m_new > a.thr_hi * rho;
      if (filled) a.f_epoch[idx] = a.step;
      wave_append(filled, &a.counters[C_F], a.listF, idx);
      wave_append(m_new < a.thr_lo * rho, &a.counters[C_E], a.listE, idx);
    }
  }
}

// Laplace-pressure correction of each listed interface cell (surface tension):
// kappa[i] = 3 sigma kappa, with kappa = -div n from the fill seen over the
// D3Q19 neighbourhood (Eq. freeboundary; see curvature), or with plic = 2 from
// the height function where its columns are complete.  Runs between the
// sweep (which builds the list) and k_iface, only when sigma != 0.
__global__ __launch_bounds__(IBLOCK) void k_curvature(SweepArgs a) {
  const Grid g = a.c.grid;
  const int n_i = a.counters[C_I];
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
    IfaceData<FormF64> d;
    d.phix = a.phi_in[idx];
#define FSLBM_CLOAD(q)                                            \
  {                                                               \
    const int s = pull_source<q>(g, n);                           \
    const int sc = s >= 0 ? s : idx;                              \
    d.ty[q] = s >= 0 ? a.flags[sc] : WALL_CLASS;                  \
    d.ph[q] = a.phi_in[sc];                                       \
  }
    FSLBM_LINKS(FSLBM_CLOAD)
#undef FSLBM_CLOAD
    if (a.c.solid) {
      // a solid source is a wall: the cell's own fill
#pragma unroll
      for (int q = 1; q < Q; ++q)
        if (d.ty[q] == WALL_CLASS) d.ph[q] = d.phix;
    }
    const double kap = curvature(d);
    if (a.c.plic == 2) {
      // height-function kappa where the columns along the axis of the
      // central-difference normal are complete (NaN otherwise) for
      // k_curvature_hf, which also takes the final value; kappa[i] keeps the
      // central-difference kappa for cells with no height-function kappa near
      double khf = __builtin_nan("");
      const double gx = 0.5 * (phi_seen(d, 2) - phi_seen(d, 1));
      const double gy = 0.5 * (phi_seen(d, 4) - phi_seen(d, 3));
      const double gz = 0.5 * (phi_seen(d, 6) - phi_seen(d, 5));
      const double nrm2 = (gx * gx + gy * gy) + gz * gz;
      if (nrm2 > 0.0) {
        const double nrm = sqrt(nrm2);
        const double nv[3] = {-gx / nrm, -gy / nrm, -gz / nrm};
        hf_curvature(g, n.x, n.y, n.z, a.flags, a.phi_in, nv, khf);
      }
      a.khf[idx] = khf;
      a.kappa[i] = kap;
    } else {
      a.kappa[i] = 3.0 * a.c.sigma * kap;
    }
  }
}

// Height-function curvature with plic = 2, after k_curvature: a listed cell
// takes its own height-function kappa; where its columns are not complete,
// the mean of those of its D3Q19 interface neighbours that have one (summed
// in link order: the neighbours lie on the same stretch of surface, while the
// central-difference kappa of the raw fills is biased by the fill itself);
// with no such neighbour the central-difference kappa.  kappa[i] = 3 sigma
// kappa.  Every interface cell is listed, so khf holds this step's value at
// every interface neighbour.
__global__ __launch_bounds__(IBLOCK) void k_curvature_hf(SweepArgs a) {
  const Grid g = a.c.grid;
  const int n_i = a.counters[C_I];
  for (int i = blockIdx.x * IBLOCK + threadIdx.x; i < n_i; i += gridDim.x * IBLOCK) {
    const int idx = a.listI[i];
    double kap = a.khf[idx];
    if (isnan(kap)) {
      int x, y, z;
      coords(g, idx, x, y, z);
      double sum = 0.0;
      int cnt = 0;
#pragma unroll
      for (int q = 1; q < Q; ++q) {
        const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
        if (s < 0 || a.flags[s] != IFACE) continue;
        const double v = a.khf[s];
        if (isnan(v)) continue;
        sum = sum + v;
        ++cnt;
      }
      kap = cnt ? sum / (double)cnt : a.kappa[i];
    }
    a.kappa[i] = 3.0 * a.c.sigma * kap;
  }
}

// ------------------------------------------------------------ conversions
// Classes and auxiliary rows of the 18 neighbours of a new interface cell c
// from gas (a neighbour beyond a wall reads the cell's own row and counts as
// gas).  Split from the arithmetic so that the loads can go out before the
// thread knows that it initialises c.  Nothing here is written by k_mark: the
// non-gas neighbours of a gas cell are interface cells (a liquid cell never
// touches gas), and k_mark writes rows of new cells only.
struct GasNbrs {
  uint8_t tn[Q];
  double4 vn[Q];
};

__device__ __forceinline__ void load_gas_nbrs(const ConvArgs& a, int c, GasNbrs& nb) {
  const Grid& g = a.c.grid;
  int x, y, z;
  coords(g, c, x, y, z);
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    const int sc = s >= 0 ? s : c;
    nb.tn[q] = s >= 0 ? a.flags[sc] : (uint8_t)GAS;
    nb.vn[q] = *reinterpret_cast<const double4*>(a.aux + 4 * (size_t)sc);
  }
}

// f = f^eq of the mean collision density and velocity of the non-gas
// neighbours, mass 0.
template <class F>
__device__ void init_new_from_gas(const ConvArgs& a, int c, const GasNbrs& nb) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid& g = a.c.grid;
  double rs = 0.0, us0 = 0.0, us1 = 0.0, us2 = 0.0;
  int cnt = 0;
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    if (nb.tn[q] == GAS || nb.tn[q] == SOLID) continue;
    rs = rs + nb.vn[q].x;
    us0 = us0 + nb.vn[q].y;
    us1 = us1 + nb.vn[q].z;
    us2 = us2 + nb.vn[q].w;
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
  a.aux[4 * (size_t)c] = rbar;
}

// A new interface cell from liquid keeps its populations (of time t+1, written
// by the sweep); m = rho.  The populations are loaded by the caller.
template <class F>
__device__ void init_new_from_liquid(const ConvArgs& a, int c, const typename F::R (&fl)[Q]) {
  double r;
  if (F::shifted) {
    double s = 0.0;
    for (int q = 0; q < Q; ++q) s = s + (double)fl[q];
    r = 1.0 + s;
  } else {
    r = (double)fl[0];
    for (int q = 1; q < Q; ++q) r = r + (double)fl[q];
  }
  a.mass[c] = r;
  a.aux[4 * (size_t)c] = r;
}

// Mark of an E' cell in new_epoch: below every step stamp (>= 0) and the
// initial -1, and distinct for every step.  E' cells are interface cells and
// new_epoch's step stamps go to gas and liquid cells only.
__device__ __forceinline__ int ep_stamp(int step) { return -2 - step; }

// One thread per (converted cell, link): a cell's 18 neighbours are handled by
// 18 threads, so the work of a step is not the longest serial chain of one
// cell's new neighbours.  Which thread wins a new cell's epoch mark does not
// change the result (its initialisation reads only pre-conversion classes).
template <class F>
__global__ __launch_bounds__(BLOCK) void k_mark(ConvArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  const int nF = a.counters[C_F], nE = a.counters[C_E];
  const Grid& g = a.c.grid;
  const S* fo = reinterpret_cast<const S*>(a.fout);
  // 18 N < 19 N < 2^32 (the lattice limit): the pair index fits in 32 unsigned bits
  const unsigned total = (unsigned)(nF + nE) * (unsigned)(Q - 1);
  for (unsigned i = blockIdx.x * BLOCK + threadIdx.x; i < total; i += gridDim.x * BLOCK) {
    const int e = (int)(i / (unsigned)(Q - 1));
    const int q = 1 + (int)(i - (unsigned)e * (unsigned)(Q - 1));
    const int c = e < nF ? a.listF[e] : a.listE[e - nF];
    int x, y, z;
    coords(g, c, x, y, z);
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    const uint8_t ts = s >= 0 ? a.flags[s] : (uint8_t)SOLID;
    if (e < nF) {
      // a gas neighbour: its initialisation data load with the claim
      bool win = false;
      GasNbrs nb;
      if (ts == GAS) {
        load_gas_nbrs(a, s, nb);
        win = atomicExch(&a.new_epoch[s], a.step) != a.step;
      }
      wave_append(win, &a.counters[C_NI], a.listNI, s);
      if (win) init_new_from_gas<F>(a, s, nb);
    } else {
      // E' = E minus N(F): every thread of the cell takes the same decision
      bool protect = false;
#pragma unroll
      for (int p = 1; p < Q; ++p) {
        const int t = neighbor(g, x, y, z, CX[p], CY[p], CZ[p]);
        if (t >= 0 && a.f_epoch[t] == a.step) protect = true;
      }
      if (protect) continue;
      if (q == 1) a.new_epoch[c] = ep_stamp(a.step);
      wave_append(q == 1, &a.counters[C_EP], a.listEP, c);
      // a liquid neighbour: its populations load with the claim
      bool win = false;
      R fl[Q];
      if (ts == LIQ) {
#pragma unroll
        for (int p = 0; p < Q; ++p) fl[p] = F::load(fo + (size_t)p * g.N + s, a.c.inv_scale);
        win = atomicExch(&a.new_epoch[s], a.step) != a.step;
      }
      wave_append(win, &a.counters[C_NL], a.listNL, s);
      if (win) init_new_from_liquid<F>(a, s, fl);
    }
  }
}

// Whether cell t is an interface cell after this step's conversions: a new
// interface cell, or an interface cell of time t that neither filled nor is in
// E'.  Three loads, no branch, so that a caller's 18 neighbours load in one
// batch.
__device__ __forceinline__ bool iface_after(const ConvArgs& a, int t) {
  const int ne = a.new_epoch[t];
  const int fe = a.f_epoch[t];
  const uint8_t fl = a.flags[t];
  return (ne == a.step) | ((fl == IFACE) & (fe != a.step) & (ne != ep_stamp(a.step)));
}

// One thread per (converted cell, link), as in k_mark: every thread of a cell
// counts its eligible neighbours; the link-1 thread takes the excess (a filled
// cell's mass minus its density, an emptied cell's mass), divides it (or hands
// it to the reservoir) and marks the cell, each thread lists its own receiver.
__global__ __launch_bounds__(BLOCK) void k_share(ConvArgs a) {
  const int nF = a.counters[C_F], nEP = a.counters[C_EP];
  const Grid& g = a.c.grid;
  // 18 N < 19 N < 2^32 (the lattice limit): the pair index fits in 32 unsigned bits
  const unsigned total = (unsigned)(nF + nEP) * (unsigned)(Q - 1);
  for (unsigned i = blockIdx.x * BLOCK + threadIdx.x; i < total; i += gridDim.x * BLOCK) {
    const int e = (int)(i / (unsigned)(Q - 1));
    const int q = 1 + (int)(i - (unsigned)e * (unsigned)(Q - 1));
    const bool filled = e < nF;
    const int c = filled ? a.listF[e] : a.listEP[e - nF];
    int x, y, z;
    coords(g, c, x, y, z);
    int n_elig = 0;
    bool recv = false;
#pragma unroll
    for (int p = 1; p < Q; ++p) {
      const int t = neighbor(g, x, y, z, CX[p], CY[p], CZ[p]);
      const bool el = (t >= 0) & iface_after(a, t >= 0 ? t : c);
      n_elig += el ? 1 : 0;
      if (p == q) recv = el;
    }
    if (q == 1) {
      const double ex = filled ? a.mass[c] - a.aux[4 * (size_t)c] : a.mass[c];
      if (n_elig == 0) {
        atomicAdd(a.reservoir, ex);
        if (filled) a.mass[c] = ex;
      } else {
        a.mass[c] = ex / (double)n_elig;
        a.conv_epoch[c] = a.step;
      }
    }
    if (!recv) continue;
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    wave_append(atomicExch(&a.recv_epoch[s], a.step) != a.step, &a.counters[C_R], a.listR, s);
  }
}

// Receivers (first nR threads) and the new cell classes (the rest; with the
// interface kernel first, the new interface cells also join the next list).
__global__ __launch_bounds__(BLOCK) void k_gather(ConvArgs a) {
  const int nR = a.counters[C_R];
  const int nF = a.counters[C_F], nEP = a.counters[C_EP], nNI = a.counters[C_NI], nNL = a.counters[C_NL];
  const int tot = nR + nF + nEP + nNI + nNL;
  const Grid& g = a.c.grid;
  for (int i = blockIdx.x * BLOCK + threadIdx.x; i < tot; i += gridDim.x * BLOCK) {
    if (i >= nR) {
      int j = i - nR, cell;
      uint8_t cls;
      if (j < nF) {
        cell = a.listF[j];
        cls = LIQ;
      } else if ((j -= nF) < nEP) {
        cell = a.listEP[j];
        cls = GAS;
      } else if ((j -= nEP) < nNI) {
        cell = a.listNI[j];
        cls = IFACE;
      } else {
        cell = a.listNL[j - nNI];
        cls = IFACE;
      }
      a.flags[cell] = cls;
      if (a.order) {
        // a new interface cell joins the list of the next step
        const bool join = cls == IFACE;
        const int pos = wave_append_at(join, &a.counters_next[C_I], a.listI, cell);
        if (join) a.islot[cell] = pos;
      }
      continue;
    }
    const int r = a.listR[i];
    int x, y, z;
    coords(g, r, x, y, z);
    double m = a.mass[r];
    // marks and masses of all neighbours in one batch of loads, then the sum
    // in link order (a neighbour beyond a wall reads the cell's own entries)
    int ep[Q];
    double mn[Q];
#pragma unroll
    for (int q = 1; q < Q; ++q) {
      const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
      const int sc = s >= 0 ? s : r;
      ep[q] = s >= 0 ? a.conv_epoch[sc] : -1;
      mn[q] = a.mass[sc];
    }
#pragma unroll
    for (int q = 1; q < Q; ++q)
      if (ep[q] == a.step) m = m + mn[q];
    a.mass[r] = m;
    a.phi_out[r] = m / a.aux[4 * (size_t)r];
  }
}

// The interface cells of the current classes into list and islot (cell -> list
// entry), in wavefront order; *counter (zero before) becomes their number.  For
// the first step with the interface kernel first after a new state.
__global__ __launch_bounds__(BLOCK) void k_list_append(const uint8_t* __restrict__ flags, int N, int32_t* counter,
                                                       int32_t* list, int32_t* islot) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  const bool it = i < N && flags[i] == IFACE;
  const int pos = wave_append_at(it, counter, list, i);
  if (it) islot[i] = pos;
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
  if (t > SOLID) {
    atomicOr(err, 1);
    return;
  }
  if (t == SOLID) atomicOr(err, 4);  // solid cells present
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
  if (t == SOLID) {
    // obstacles hold no fluid: zero populations (never read by the step)
    S* fz = reinterpret_cast<S*>(a.f);
#pragma unroll
    for (int q = 0; q < Q; ++q) fz[(size_t)q * N + idx] = S(0);
    return;
  }
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
    *reinterpret_cast<double4*>(a.aux + 4 * idx) = make_double4(r, u[idx], u[N + idx], u[2 * N + idx]);
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
  if (t == SOLID) {
#pragma unroll
    for (int q = 0; q < Q; ++q) fo[(size_t)q * N + idx] = S(0);
    return;
  }
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
    *reinterpret_cast<double4*>(a.aux + 4 * idx) =
        make_double4(SH ? 1.0 + (double)rs : (double)rs, (double)uu[0], (double)uu[1], (double)uu[2]);
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
  if (a.phi_out) a.phi_out[idx] = t == LIQ ? 1.0 : (t == IFACE ? a.phi[idx] : 0.0);
  if (a.mass_out) a.mass_out[idx] = t == IFACE ? a.mass[idx] : 0.0;
  if (a.rhoc_out) a.rhoc_out[idx] = t == IFACE ? a.aux[4 * idx] : 0.0;
  if (a.uc_out)
    for (int d = 0; d < 3; ++d) a.uc_out[d * N + idx] = t == IFACE ? a.aux[4 * idx + 1 + d] : 0.0;
  R fl[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) fl[q] = F::load(fi + (size_t)q * N + idx, a.c.inv_scale);
  if (a.f_out) {
#pragma unroll
    for (int q = 0; q < Q; ++q)
      a.f_out[(size_t)q * N + idx] = (t == GAS || t == SOLID) ? 0.0 : (SH ? (double)fl[q] + WD[q] : (double)fl[q]);
  }
  if (a.rho_out || a.u_out) {
    R rs, uu[3];
    recover_moments<R, SH>(fl, k, a.c.incomp, rs, uu);
    const double r = SH ? 1.0 + (double)rs : (double)rs;
    const bool fluid = t == LIQ || t == IFACE;
    if (a.rho_out) a.rho_out[idx] = fluid ? r : 0.0;
    if (a.u_out)
      for (int d = 0; d < 3; ++d) a.u_out[d * N + idx] = fluid ? (double)uu[d] : 0.0;
  }
}

// Bits j + 1 of gas and liq for the cells x0 + j, j = -1 .. 16, of the row
// starting at rbase (a cell beyond a wall sets no bit, beyond a periodic face
// the wrapped one; positions past the row end set none, and the right
// neighbour of the row's last cell is at bit nx - x0 + 1).  One 16-byte load
// where the row allows.
__device__ __forceinline__ void row_masks(const uint8_t* __restrict__ f, const Grid& g, unsigned rbase, int x0,
                                          uint32_t& gas, uint32_t& liq) {
  gas = liq = 0u;
  const int n = min(16, g.nx - x0);  // cells of this chunk
  if (n == 16 && ((rbase + (unsigned)x0) & 15u) == 0u) {
    const uint4 v = *reinterpret_cast<const uint4*>(f + rbase + (unsigned)x0);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const uint32_t b = (w[j >> 2] >> (8 * (j & 3))) & 0xffu;
      gas |= (b == GAS ? 1u : 0u) << (j + 1);
      liq |= (b == LIQ ? 1u : 0u) << (j + 1);
    }
  } else {
    for (int j = 0; j < n; ++j) {
      const uint8_t b = f[rbase + (unsigned)(x0 + j)];
      gas |= (b == GAS ? 1u : 0u) << (j + 1);
      liq |= (b == LIQ ? 1u : 0u) << (j + 1);
    }
  }
  const int xl = x0 > 0 ? x0 - 1 : (g.px ? g.nx - 1 : -1);
  if (xl >= 0 && f[rbase + (unsigned)xl] == GAS) gas |= 1u;
  const int xr = x0 + n < g.nx ? x0 + n : (g.px ? 0 : -1);
  if (xr >= 0 && f[rbase + (unsigned)xr] == GAS) gas |= 1u << (n + 1);
}

// The layer rule of the health check: liquid cells with a gas cell among
// their 18 neighbours, added to cnt[5].  A lane takes 16 cells of a row and
// the masks of its eight neighbour rows (the rows at y +- 1 or z +- 1 give
// neighbours at x - 1, x, x + 1, the four diagonal rows only at x), one
// 16-byte load per row.
__global__ __launch_bounds__(BLOCK) void k_layer(const uint8_t* __restrict__ flags, Grid g, int32_t* cnt) {
  __shared__ int sb[BLOCK / 64];
  const int lpr = (g.nx + 15) / 16;
  const int total = g.ny * g.nz * lpr;  // < N / 16 + ny nz < 2^31
  int bad = 0;
  for (int k = (int)blockIdx.x * BLOCK + (int)threadIdx.x; k < total; k += (int)gridDim.x * BLOCK) {
    const int row = k / lpr;
    const int x0 = (k - row * lpr) * 16;
    const int y = row % g.ny, z = row / g.ny;
    uint32_t gas, liq;
    row_masks(flags, g, (unsigned)row * (unsigned)g.nx, x0, gas, liq);
    if (liq == 0u) continue;
    uint32_t near = (gas << 1) | (gas >> 1);
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz) {
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy) {
        if (dy == 0 && dz == 0) continue;
        const int ys = step_axis(y, dy, g.ny, g.py), zs = step_axis(z, dz, g.nz, g.pz);
        if (ys < 0 || zs < 0) continue;
        uint32_t gr, lr;
        row_masks(flags, g, (unsigned)(ys + g.ny * zs) * (unsigned)g.nx, x0, gr, lr);
        near |= (dy != 0 && dz != 0) ? gr : (gr | (gr << 1) | (gr >> 1));
      }
    }
    bad += __popc(liq & near);
  }
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_down(bad, o);
  if ((threadIdx.x & 63) == 0) sb[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < BLOCK / 64; ++w) t += sb[w];
    if (t > 0) atomicAdd(&cnt[5], t);
  }
}

// Total mass and health check: block partial sums of the mass into acc[0];
// counts of liquid and interface cells, and of the cells that fail a check
// (see StatArgs::cnt; the layer rule is k_layer's).  The mass sum is FP64 in
// every form.
template <class F>
__global__ __launch_bounds__(BLOCK) void k_stats(StatArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  __shared__ double sm[BLOCK / 64];
  __shared__ int sl[BLOCK / 64];
  __shared__ int si[BLOCK / 64];
  double v = 0.0;
  int nl = 0, ni = 0;
  const S* fi = reinterpret_cast<const S*>(a.f);
  const Grid& g = a.c.grid;
  const Consts<R>& k = pick_consts<R>(a.c);
  for (int idx = blockIdx.x * BLOCK + threadIdx.x; idx < g.N; idx += gridDim.x * BLOCK) {
    const uint8_t t = a.flags[idx];
    if (t > SOLID) {
      atomicAdd(&a.cnt[5], 1);
      continue;
    }
    if (t == GAS || t == SOLID) continue;
    R fl[Q];
    double r = 0.0;
    for (int q = 0; q < Q; ++q) {
      fl[q] = F::load(fi + (size_t)q * g.N + idx, a.c.inv_scale);
      r = r + (double)fl[q];
    }
    if (F::shifted) r = 1.0 + r;
    if (!(r > 0.0) || !isfinite(r)) atomicAdd(&a.cnt[1], 1);
    R rs, u[3];
    recover_moments<R, SH>(fl, k, a.c.incomp, rs, u);
    const double usq = ((double)u[0] * (double)u[0] + (double)u[1] * (double)u[1]) + (double)u[2] * (double)u[2];
    if (!(usq <= a.u_max2)) atomicAdd(&a.cnt[4], 1);
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

template <class F, int RULE, bool REC, bool EXTRA>
static void iface_go(const StepLaunch& L, unsigned nb) {
  k_iface<F, RULE, REC, EXTRA><<<nb, IBLOCK, 0, (hipStream_t)L.stream>>>(L.sweep);
}

template <class F>
static void iface_form(const StepLaunch& L, int rule) {
  // the interface count is on the device: enough one-wavefront blocks for
  // every cell up to IFACE_GRID * IBLOCK, grid-stride beyond
  const unsigned nb = std::min<unsigned>(IFACE_GRID, (unsigned)((L.sweep.c.grid.N + IBLOCK - 1) / IBLOCK));
  const bool extra =
      L.sweep.c.moving || L.sweep.c.sigma != 0.0 || L.sweep.c.plic || L.sweep.c.solid || L.sweep.c.surface;
  if (L.sweep.rec_f) {
    // a window step (rules 0 and 1): the list is fixed and its length (rec_cap)
    // known here; the four-lane kernel records as well where the plain step
    // would take it
    if (!extra && L.sweep.quad) {
      (void)launch_iface4(L, std::is_same<F, FormF64>::value ? 0 : (std::is_same<F, FormF32>::value ? 1 : 2), rule);
      return;
    }
    const unsigned nbr = std::min<unsigned>(nb, (unsigned)((L.sweep.rec_cap + IBLOCK - 1) / IBLOCK));
    if (rule == 0)
      extra ? iface_go<F, 0, true, true>(L, nbr) : iface_go<F, 0, true, false>(L, nbr);
    else
      extra ? iface_go<F, 1, true, true>(L, nbr) : iface_go<F, 1, true, false>(L, nbr);
    return;
  }
  if (!extra && L.sweep.quad) {
    (void)launch_iface4(L, std::is_same<F, FormF64>::value ? 0 : (std::is_same<F, FormF32>::value ? 1 : 2), rule);
    return;
  }
  switch (rule) {
    case 0: extra ? iface_go<F, 0, false, true>(L, nb) : iface_go<F, 0, false, false>(L, nb); break;
    case 1: extra ? iface_go<F, 1, false, true>(L, nb) : iface_go<F, 1, false, false>(L, nb); break;
    case 2: extra ? iface_go<F, 2, false, true>(L, nb) : iface_go<F, 2, false, false>(L, nb); break;
    case 3: extra ? iface_go<F, 3, false, true>(L, nb) : iface_go<F, 3, false, false>(L, nb); break;
    case 4: extra ? iface_go<F, 4, false, true>(L, nb) : iface_go<F, 4, false, false>(L, nb); break;
    default: extra ? iface_go<F, 5, false, true>(L, nb) : iface_go<F, 5, false, false>(L, nb); break;
  }
}

template <class F>
static void convert_form(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  k_mark<F><<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_share<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_gather<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
}

// Liquid cells next to solid cells (the wall list; interface cells there are
// done by k_iface, gas cells need nothing): the sweep has written them with
// values pulled from solid cells, so this kernel redoes their step after it:
// pull (halfway bounce-back at wall faces, the wall closure on solid links),
// TRT collision, store.  One cell per thread.
template <class F>
__global__ __launch_bounds__(IBLOCK) void k_wall(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  const S* __restrict__ fin = reinterpret_cast<const S*>(a.fin);
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
  const size_t N = (size_t)g.N;
  const float isc = a.c.inv_scale;
  const Consts<R>& k = pick_consts<R>(a.c);
  const bool incomp = a.c.incomp, stokes = a.c.stokes;
  for (int i = blockIdx.x * IBLOCK + threadIdx.x; i < a.nwall; i += gridDim.x * IBLOCK) {
    const int idx = a.wcells[i];
    if (a.flags[idx] != LIQ) continue;
    Nbr n;
    coords(g, idx, n.x, n.y, n.z);
    n.xm = step_axis(n.x, -1, g.nx, g.px);
    n.xp = step_axis(n.x, 1, g.nx, g.px);
    n.ym = step_axis(n.y, -1, g.ny, g.py);
    n.yp = step_axis(n.y, 1, g.ny, g.py);
    n.zm = step_axis(n.z, -1, g.nz, g.pz);
    n.zp = step_axis(n.z, 1, g.nz, g.pz);
    R f[Q], own[Q];
    uint32_t sm = 0, up = 0;
    f[0] = F::load(fin + idx, isc);
    own[0] = f[0];
#define FSLBM_WLOAD(q)                                                                     \
  {                                                                                        \
    const int s = pull_source<q>(g, n);                                                    \
    const size_t off = s >= 0 ? (size_t)q * N + (size_t)s : (size_t)OPP[q] * N + idx;      \
    f[q] = F::load(fin + off, isc);                                                        \
    own[q] = F::load(fin + (size_t)q * N + idx, isc);                                      \
    const uint8_t ts = s >= 0 ? a.flags[s] : WALL_CLASS;                                   \
    if (s >= 0 && ts == SOLID) sm |= 1u << q;                                              \
    if (ts == LIQ || ts == IFACE) up |= 1u << q;                                           \
  }
    FSLBM_LINKS(FSLBM_WLOAD)
#undef FSLBM_WLOAD
    if (a.c.moving) {
#define FSLBM_WWALLU(q)                                                                        \
  {                                                                                            \
    const double t = wall_term<q>(a.wall_t, n.xm, n.xp, n.ym, n.yp, n.zm, n.zp);               \
    if (t != 0.0) f[q] = f[q] + (R)t;                                                          \
  }
      FSLBM_LINKS(FSLBM_WWALLU)
#undef FSLBM_WWALLU
    }
    solid_links<R>(f, own, sm, up, i, a.nwall, a.wdelta, a.wuw);
    R rho_s, u[3];
    if constexpr (sizeof(R) == 4)
      collide_f32<SH>(f, k, incomp, stokes, rho_s, u);
    else
      collide<R, SH>(f, k, incomp, stokes, rho_s, u);
#pragma unroll
    for (int q = 0; q < Q; ++q) F::store(fout + (size_t)q * N + idx, f[q], a.c.scale);
  }
}

hipError_t launch_wall(const StepLaunch& L, int precision) {
  if (L.sweep.nwall <= 0) return hipSuccess;
  const unsigned nb = std::min<unsigned>(IFACE_GRID, (unsigned)((L.sweep.nwall + IBLOCK - 1) / IBLOCK));
  hipStream_t st = (hipStream_t)L.stream;
  if (precision == 0) k_wall<FormF64><<<nb, IBLOCK, 0, st>>>(L.sweep);
  else if (precision == 1) k_wall<FormF32><<<nb, IBLOCK, 0, st>>>(L.sweep);
  else k_wall<FormF16><<<nb, IBLOCK, 0, st>>>(L.sweep);
  return hipGetLastError();
}

// Wall table checks: cells ascending, in range, not solid, each with a link
// into a solid cell whose distance is in (0, 1] and velocity finite (err bits
// 1, 2, 4, 32, 8, 16); count[0] += the number of non-solid cells with a link
// into a solid cell (k_count_walls), to be compared with n.
__global__ __launch_bounds__(BLOCK) void k_check_walls(const uint8_t* flags, Grid g, const int32_t* cells, int n,
                                                       const double* delta, const double* uw, int32_t* err) {
  const int i = blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const int idx = cells[i];
  if (idx < 0 || idx >= g.N) {
    atomicOr(err, 1);
    return;
  }
  if (i > 0 && cells[i - 1] >= idx) atomicOr(err, 2);
  if (flags[idx] == SOLID) atomicOr(err, 4);
  int x, y, z;
  coords(g, idx, x, y, z);
  bool any = false;
  for (int q = 1; q < Q; ++q) {
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    if (s < 0 || flags[s] != SOLID) continue;
    any = true;
    const double d = delta[(size_t)q * n + i];
    if (!(d > 0.0 && d <= 1.0)) atomicOr(err, 8);
    for (int c = 0; c < 3; ++c)
      if (!isfinite(uw[((size_t)c * Q + q) * n + i])) atomicOr(err, 16);
  }
  if (!any) atomicOr(err, 32);
}

__global__ __launch_bounds__(BLOCK) void k_count_walls(const uint8_t* flags, Grid g, int32_t* count) {
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx >= g.N || flags[idx] == SOLID) return;
  int x, y, z;
  coords(g, idx, x, y, z);
  for (int q = 1; q < Q; ++q) {
    const int s = neighbor(g, x, y, z, CX[q], CY[q], CZ[q]);
    if (s >= 0 && flags[s] == SOLID) {
      atomicAdd(count, 1);
      return;
    }
  }
}

hipError_t launch_check_walls(const uint8_t* flags, const Grid& g, const int32_t* cells, int n, const double* delta,
                              const double* uw, int32_t* err, int32_t* count, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (n > 0) k_check_walls<<<blocks_for(n), BLOCK, 0, st>>>(flags, g, cells, n, delta, uw, err);
  k_count_walls<<<blocks_for(g.N), BLOCK, 0, st>>>(flags, g, count);
  return hipGetLastError();
}

hipError_t launch_curvature(const StepLaunch& L) {
  const unsigned nb = std::min<unsigned>(IFACE_GRID, (unsigned)((L.sweep.c.grid.N + IBLOCK - 1) / IBLOCK));
  k_curvature<<<nb, IBLOCK, 0, (hipStream_t)L.stream>>>(L.sweep);
  if (L.sweep.c.plic == 2) k_curvature_hf<<<nb, IBLOCK, 0, (hipStream_t)L.stream>>>(L.sweep);
  return hipGetLastError();
}

hipError_t launch_iface(const StepLaunch& L, int precision, int rule) {
  if (precision == 0) iface_form<FormF64>(L, rule);
  else if (precision == 1) iface_form<FormF32>(L, rule);
  else iface_form<FormF16>(L, rule);
  return hipGetLastError();
}

hipError_t launch_list_append(const uint8_t* flags, const Grid& g, int32_t* counter, int32_t* list, int32_t* islot,
                              void* stream) {
  hipStream_t st = (hipStream_t)stream;
  k_fill_i32<<<1, BLOCK, 0, st>>>(counter, 1, 0);
  k_list_append<<<blocks_for((size_t)g.N), BLOCK, 0, st>>>(flags, g.N, counter, list, islot);
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

// k_stats with 16 bytes of every population plane per lane: G = 16 / s cells
// (8 in the FP16 form, whose 2-byte elements would otherwise take a load
// instruction per element and per cell), for lattices whose N is a multiple
// of G (the planes then start on 16-byte boundaries).  Same checks and sums
// as k_stats, cell by cell.
template <class F>
__global__ __launch_bounds__(BLOCK) void k_stats_vec(StatArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  constexpr int G = 16 / (int)sizeof(S);
  __shared__ double sm[BLOCK / 64];
  __shared__ int sl[BLOCK / 64];
  __shared__ int si[BLOCK / 64];
  double v = 0.0;
  int nl = 0, ni = 0;
  const S* fi = reinterpret_cast<const S*>(a.f);
  const Grid& g = a.c.grid;
  const unsigned N = (unsigned)g.N;
  const unsigned ng = N / (unsigned)G;
  const Consts<R>& k = pick_consts<R>(a.c);
  for (unsigned gi = blockIdx.x * BLOCK + threadIdx.x; gi < ng; gi += gridDim.x * BLOCK) {
    const unsigned base = gi * (unsigned)G;
    uint8_t t[G];
#pragma unroll
    for (int c = 0; c < G; ++c) t[c] = a.flags[base + (unsigned)c];
    bool any = false;
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (t[c] > SOLID) atomicAdd(&a.cnt[5], 1);
      any = any || t[c] == LIQ || t[c] == IFACE;
    }
    if (!any) continue;
    uint4 vq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) vq[q] = *reinterpret_cast<const uint4*>(fi + ((size_t)q * N + base));
#pragma unroll
    for (int c = 0; c < G; ++c) {
      if (t[c] != LIQ && t[c] != IFACE) continue;
      R fl[Q];
      double r = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        fl[q] = F::load(reinterpret_cast<const S*>(&vq[q]) + c, a.c.inv_scale);
        r = r + (double)fl[q];
      }
      if (F::shifted) r = 1.0 + r;
      if (!(r > 0.0) || !isfinite(r)) atomicAdd(&a.cnt[1], 1);
      R rs, u[3];
      recover_moments<R, SH>(fl, k, a.c.incomp, rs, u);
      const double usq = ((double)u[0] * (double)u[0] + (double)u[1] * (double)u[1]) + (double)u[2] * (double)u[2];
      if (!(usq <= a.u_max2)) atomicAdd(&a.cnt[4], 1);
      if (t[c] == LIQ) {
        v += r;
        nl += 1;
      } else {
        v += a.mass[base + (unsigned)c];
        ni += 1;
      }
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

template <class F>
static void stats_form(const StatArgs& a, hipStream_t s) {
  constexpr int G = 16 / (int)sizeof(typename F::S);
  const unsigned nb = std::min<unsigned>(2048u, blocks_for(a.c.grid.N));
  if (a.c.grid.N % G == 0)
    k_stats_vec<F><<<std::min<unsigned>(2048u, blocks_for(a.c.grid.N / G)), BLOCK, 0, s>>>(a);
  else
    k_stats<F><<<nb, BLOCK, 0, s>>>(a);
}

hipError_t launch_stats(const StatArgs& a, int precision, void* stream) {
  hipStream_t s = (hipStream_t)stream;
  if (precision == 0) stats_form<FormF64>(a, s);
  else if (precision == 1) stats_form<FormF32>(a, s);
  else stats_form<FormF16>(a, s);
  const Grid& g = a.c.grid;
  const long long lanes = (long long)g.ny * g.nz * ((g.nx + 15) / 16);
  const unsigned nl = (unsigned)std::max<long long>(1, std::min<long long>(2048, (lanes + BLOCK - 1) / BLOCK));
  k_layer<<<nl, BLOCK, 0, s>>>(a.flags, g, a.cnt);
  return hipGetLastError();
}

}  // namespace fslbm
