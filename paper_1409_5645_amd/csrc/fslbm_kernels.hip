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

namespace fslbm {

constexpr int BLOCK = 256;

// ------------------------------------------------------------------ sweep
// Neighbour coordinates of one cell (-1 beyond a wall).
struct Nbr {
  int x, y, z, xm, xp, ym, yp, zm, zp;
};

// linear index of the source x - c_q of the pull, or -1 beyond a wall
template <int q>
__device__ __forceinline__ int pull_source(const Grid& g, const Nbr& n) {
  const int sx = CX[q] == 1 ? n.xm : (CX[q] == -1 ? n.xp : n.x);
  const int sy = CY[q] == 1 ? n.ym : (CY[q] == -1 ? n.yp : n.y);
  const int sz = CZ[q] == 1 ? n.zm : (CZ[q] == -1 ? n.zp : n.z);
  return ((sx | sy | sz) < 0) ? -1 : sx + g.nx * (sy + g.ny * sz);
}

template <class F>
struct IfaceCtx {
  using R = typename F::R;
  using S = typename F::S;
  const S* fin;
  size_t N;
  int idx;
  float isc;
  uint32_t gasmask;
  bool have_n;
  double nv[3];
  double dist;
  R rho_t, rho0_t, u_t[3], usq_t;
  const Consts<R>* k;
  bool incomp, stokes;
};

// Mass exchange over link q (FP64): weight 1 to liquid, (phi_x+phi_s)/2 to
// interface, nothing from gas or walls.
template <class F, int q>
__device__ __forceinline__ void exchange(double& dm, const typename F::R (&f)[Q], const Grid& g, const Nbr& n,
                                         const uint8_t* flags, const double* phi, double phix,
                                         const typename F::S* fin, int idx, float isc, uint32_t& gasmask) {
  const int s = pull_source<q>(g, n);
  if (s < 0) return;
  const uint8_t ts = flags[s];
  if (ts == GAS) {
    gasmask |= 1u << q;
    return;
  }
  const double own_qb = (double)F::load(fin + (size_t)OPP[q] * g.N + idx, isc);
  const double diff = (double)f[q] - own_qb;
  if (ts == LIQ) {
    dm = dm + diff;
  } else {
    const double wgt = 0.5 * (phix + phi[s]);
    dm = dm + wgt * diff;
  }
}

// Reconstruction of the population f_q that would stream in from a gas cell.
// With o = qbar the link pointing to gas, the closure Eq. (closure) gives
//   f_q = a0 ft_o(x) + a0bar ft_q(x) + a1 f_o(x,t+1) + C n+_o(x,t) + alpha_+ e+_o(rho_b,u_b)
// with the FSK row of Table 1 (Eq. koerner) or Eq. (fsli1)-(fsli4) at alpha_+ = 1.
template <class F, int RULE, int q>
__device__ __forceinline__ void rebuild(typename F::R (&f)[Q], const IfaceCtx<F>& c) {
  using R = typename F::R;
  if (!((c.gasmask >> q) & 1u)) return;
  constexpr int o = OPP[q];
  const R own_o = F::load(c.fin + (size_t)o * c.N + c.idx, c.isc);
  const R e_b = e_plus<o>(c.k->rhob_s, c.k->rho0b, c.incomp, c.stokes, c.u_t, c.usq_t);
  if (RULE == 1 && c.have_n && !((c.gasmask >> o) & 1u)) {
    // link distance delta: plane with normal n at offset phi - 1/2
    double nc = 0.0;
    if (CX[o] == 1) nc = nc + c.nv[0];
    if (CX[o] == -1) nc = nc - c.nv[0];
    if (CY[o] == 1) nc = nc + c.nv[1];
    if (CY[o] == -1) nc = nc - c.nv[1];
    if (CZ[o] == 1) nc = nc + c.nv[2];
    if (CZ[o] == -1) nc = nc - c.nv[2];
    if (nc > 0.0) {
      double d = c.dist / nc;
      if (d < 0.0) d = 0.0;
      if (d > 1.0) d = 1.0;
      const R delta = (R)d;
      const R own_q = F::load(c.fin + (size_t)q * c.N + c.idx, c.isc);
      // n+_o(x,t) from ft+ = e+ + (1 + lambda_+) n+
      const R e_o_t = e_plus<o>(c.rho_t, c.rho0_t, c.incomp, c.stokes, c.u_t, c.usq_t);
      const R n_plus = (R(0.5) * (own_o + own_q) - e_o_t) * c.k->inv1p;
      const R a0 = R(1.0) - (R(0.5) + delta);
      const R a1 = delta - R(1.0);
      const R Cc = c.k->lp * (R(0.5) + delta) - R(2.0) * c.k->lp;
      f[q] = (((a0 * own_o + R(0.5) * own_q) + a1 * f[o]) + Cc * n_plus) + e_b;
      return;
    }
  }
  f[q] = R(2.0) * e_b - own_o;  // FSK: -ft_o + 2 e+_o(rho_b, u_b)
}

#define FSLBM_LINKS(M) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) M(17) M(18)

template <class F, int RULE>
__global__ __launch_bounds__(BLOCK) void k_sweep(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  if (idx == 0) {
#pragma unroll
    for (int i = 0; i < NCOUNT; ++i) a.counters_next[i] = 0;
  }
  if (idx >= g.N) return;
  const uint8_t t = a.flags[idx];
  if (t == GAS) return;

  Nbr n;
  coords(g, idx, n.x, n.y, n.z);
  n.xm = step_axis(n.x, -1, g.nx, g.px);
  n.xp = step_axis(n.x, 1, g.nx, g.px);
  n.ym = step_axis(n.y, -1, g.ny, g.py);
  n.yp = step_axis(n.y, 1, g.ny, g.py);
  n.zm = step_axis(n.z, -1, g.nz, g.pz);
  n.zp = step_axis(n.z, 1, g.nz, g.pz);
  const S* __restrict__ fin = reinterpret_cast<const S*>(a.fin);
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
  const size_t N = (size_t)g.N;
  const Consts<R>& k = pick_consts<R>(a.c);
  const float isc = a.c.inv_scale;
  const bool incomp = a.c.incomp, stokes = a.c.stokes;

  // ---- pull stream, Eq. (lbe1): f_q(x) = ft_q(x - c_q); a source beyond a
  // wall gives halfway bounce-back f_q(x) = ft_qbar(x).
  R f[Q];
#define FSLBM_PULL(q)                                                                       \
  {                                                                                         \
    const int s = pull_source<q>(g, n);                                                     \
    const size_t off = s >= 0 ? (size_t)q * N + (size_t)s : (size_t)OPP[q] * N + idx;       \
    f[q] = F::load(fin + off, isc);                                                         \
  }
  f[0] = F::load(fin + idx, isc);
  FSLBM_LINKS(FSLBM_PULL)
#undef FSLBM_PULL

  double m_new = 0.0;
  if (t == IFACE) {
    const double phix = a.phi_in[idx];
    IfaceCtx<F> c;
    c.gasmask = 0;
    // ---- mass exchange (FP64), fills the gas-link mask on the way
    double dm = 0.0;
#define FSLBM_EXCH(q) exchange<F, q>(dm, f, g, n, a.flags, a.phi_in, phix, fin, idx, isc, c.gasmask);
    FSLBM_LINKS(FSLBM_EXCH)
#undef FSLBM_EXCH
    m_new = a.mass[idx] + dm;

    if (c.gasmask) {
      // ---- interface geometry: n = -grad(phi)/|grad(phi)| by central
      // differences; liquid 1, gas 0, beyond a wall phi(x)
      auto phi_at = [&](int s) -> double {
        if (s < 0) return phix;
        const uint8_t ts = a.flags[s];
        if (ts == LIQ) return 1.0;
        if (ts == GAS) return 0.0;
        return a.phi_in[s];
      };
      // pull sources of links 1..6 are x-1, x+1, y-1, y+1, z-1, z+1
      const double gx = 0.5 * (phi_at(pull_source<2>(g, n)) - phi_at(pull_source<1>(g, n)));
      const double gy = 0.5 * (phi_at(pull_source<4>(g, n)) - phi_at(pull_source<3>(g, n)));
      const double gz = 0.5 * (phi_at(pull_source<6>(g, n)) - phi_at(pull_source<5>(g, n)));
      const double nrm2 = (gx * gx + gy * gy) + gz * gz;
      c.have_n = nrm2 > 0.0;
      c.nv[0] = c.nv[1] = c.nv[2] = 0.0;
      if (c.have_n) {
        const double nrm = sqrt(nrm2);
        c.nv[0] = -gx / nrm;
        c.nv[1] = -gy / nrm;
        c.nv[2] = -gz / nrm;
      }
      c.dist = phix - 0.5;
      // ---- moments of time t from the own post-collision populations
      {
        R own[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) own[q] = F::load(fin + (size_t)q * N + idx, isc);
        recover_moments<R, SH>(own, k, incomp, c.rho_t, c.u_t);
      }
      c.rho0_t = rho0_of<R, SH>(c.rho_t, incomp);
      c.usq_t = usq_of(c.u_t);
      c.fin = fin;
      c.N = N;
      c.idx = idx;
      c.isc = isc;
      c.k = &k;
      c.incomp = incomp;
      c.stokes = stokes;
#define FSLBM_REBUILD(q) rebuild<F, RULE, q>(f, c);
      FSLBM_LINKS(FSLBM_REBUILD)
#undef FSLBM_REBUILD
    }
  }

  // ---- TRT collision, Eq. (lbe2)
  R rho_s, u[3];
  collide<R, SH>(f, k, incomp, stokes, rho_s, u);
#pragma unroll
  for (int q = 0; q < Q; ++q) F::store(fout + (size_t)q * N + idx, f[q], a.c.scale);

  const bool iface = t == IFACE;
  if (iface) {
    // ---- fill level and classification (FP64 bookkeeping)
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
  // count interface cells (one atomic per wavefront)
  const unsigned long long b = __ballot(iface);
  if (b && (int)(threadIdx.x & 63) == __ffsll((long long)b) - 1) atomicAdd(&a.counters[C_I], __popcll(b));
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
  const int idx = blockIdx.x * BLOCK + threadIdx.x;
  double v = 0.0;
  int nl = 0, ni = 0;
  if (idx < a.c.grid.N) {
    const uint8_t t = a.flags[idx];
    const S* fi = reinterpret_cast<const S*>(a.f);
    if (t != GAS) {
      double r = 0.0;
      for (int q = 0; q < Q; ++q) r = r + (double)F::load(fi + (size_t)q * a.c.grid.N + idx, a.c.inv_scale);
      if (F::shifted) r = 1.0 + r;
      if (!(r > 0.0) || !isfinite(r)) atomicAdd(&a.cnt[1], 1);
      if (t == LIQ) {
        v = r;
        nl = 1;
      } else {
        v = a.mass[idx];
        ni = 1;
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

// ------------------------------------------------------------ launchers
static inline unsigned blocks_for(size_t n) { return (unsigned)((n + BLOCK - 1) / BLOCK); }
static constexpr unsigned LIST_GRID = 512;

template <class F>
static void sweep_form(const StepLaunch& L, int rule) {
  hipStream_t st = (hipStream_t)L.stream;
  const unsigned nb = blocks_for(L.sweep.c.grid.N);
  if (rule == 0)
    k_sweep<F, 0><<<nb, BLOCK, 0, st>>>(L.sweep);
  else
    k_sweep<F, 1><<<nb, BLOCK, 0, st>>>(L.sweep);
}

template <class F>
static void convert_form(const StepLaunch& L) {
  hipStream_t st = (hipStream_t)L.stream;
  k_mark<F><<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_commit<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_share<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
  k_gather<<<LIST_GRID, BLOCK, 0, st>>>(L.conv);
}

hipError_t launch_sweep(const StepLaunch& L, int precision, int rule) {
  if (precision == 0) sweep_form<FormF64>(L, rule);
  else if (precision == 1) sweep_form<FormF32>(L, rule);
  else sweep_form<FormF16>(L, rule);
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
  const unsigned nb = blocks_for(a.c.grid.N);
  hipStream_t s = (hipStream_t)stream;
  if (precision == 0) k_stats<FormF64><<<nb, BLOCK, 0, s>>>(a);
  else if (precision == 1) k_stats<FormF32><<<nb, BLOCK, 0, s>>>(a);
  else k_stats<FormF16><<<nb, BLOCK, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace fslbm
