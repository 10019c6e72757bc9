// Interface cells of the step with four lanes per cell (a quad), for the
// rules and forms of the plain step (no moving walls, surface tension, PLIC or
// solid cells, no adjoint record; those take k_iface).  Run before the sweep
// (SweepArgs::order), it takes the list the step before built and writes the
// populations into a list-ordered buffer that the sweep stores with its rows,
// instead of 19 scattered 2-, 4- or 8-byte stores per cell.
//
// The 18 moving links form 9 pairs of opposites (q, q + 1), q odd; lane s of
// the quad owns pairs s and s + 4, lane 0 also pair 8 and lane 1 the rest
// link.  Everything a reconstruction of f_q needs besides the cell's scalars
// lives in the lane of its pair (its own populations ft_q, ft_qbar, the value
// pulled along qbar, the class of both pull sources), and so does the halfway
// bounce-back partner of a pull beyond a wall.  So a lane loads and writes
// only its own links: a quarter of the cell's scattered loads per lane.
//
// The cell's scalars are sums over all links: mass change, moments of time t,
// the normal, the bulk shear rate, the moments of the collision.  Each is
// formed in every lane of the quad in ascending link order from values
// broadcast out of their owner lanes by DPP, with the same operations as the
// one-lane form (k_iface): in the FP64 form the two give the same bits.
#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"
#include "fslbm_quad.hpp"
#include "fslbm_stencil.hpp"

#include <algorithm>
#include <type_traits>

namespace fslbm {

constexpr int QBLOCK = 256;               // threads per block
constexpr int QCELLS = QBLOCK / QUAD;     // cells per block
constexpr unsigned IFACE4_GRID = 16384;   // blocks at most (grid-stride beyond); a multiple of NXCD
constexpr int NXCD = 8;                   // XCDs of the device

// owner lane, pair slot and half (0: the odd link 2p + 1, 1: the even one) of
// link q >= 1: pair p = (q - 1) / 2 lives in lane p % 4, slot p / 4
template <int q>
struct Own {
  static constexpr int p = (q - 1) / 2;
  static constexpr int lane = p % 4;
  static constexpr int slot = p / 4;
  static constexpr int half = (q - 1) % 2;
};

// Per-lane link data of a cell: pair slots s = 0..2 (slot 2 only in lane 0),
// A = the odd link of the pair, B = its opposite; the rest link in lane 1.
template <class R>
struct QuadLinks {
  R fA[3], fB[3];     // pulled populations f_q(x, t+1)
  R oA[3], oB[3];     // own post-collision populations of time t
  int tA[3], tB[3];   // classes of the pull sources (WALL_CLASS beyond a wall)
  double pA[3], pB[3];// fills of the pull sources (own fill beyond a wall)
  R f0;               // rest link (lane 1): pulled = own
};

template <int q, class R>
__device__ __forceinline__ R bq(const R (&A)[3], const R (&B)[3], R r0) {
  if constexpr (q == 0) {
    return qbcast<1>(r0);
  } else {
    using O = Own<q>;
    return qbcast<O::lane>(O::half ? B[O::slot] : A[O::slot]);
  }
}

// even equilibrium e+ of a link with c.u = cu and weight wq (Eq. eqEven), the
// operations of e_plus<q>
template <class R>
__device__ __forceinline__ R e_plus_w(R wq, R cu, R rho_s, R rho0, bool incomp, bool stokes, R usq) {
  if (stokes) return wq * rho_s;
  R nl = R(4.5) * (cu * cu) - R(1.5) * usq;
  if (!incomp) nl = rho0 * nl;
  return wq * (rho_s + nl);
}

// c c : S for a direction d (components in {-1, 0, 1}), the operations of c_S_c<q>
template <class R>
__device__ __forceinline__ R dSd(const int (&d)[3], const R (&S)[6]) {
  const R dg = (R(d[0] * d[0]) * S[0] + R(d[1] * d[1]) * S[1]) + R(d[2] * d[2]) * S[2];
  const R of = (R(d[0] * d[1]) * S[3] + R(d[0] * d[2]) * S[4]) + R(d[1] * d[2]) * S[5];
  return dg + R(2.0) * of;
}

// Moments of 19 populations held by the quad (rest in lane 1), the same in
// all four lanes.  FP64: ascending q, the operations of moments() (so that the
// form reproduces the one-lane kernel bit for bit).  FP32 (whose results are
// not reproduced bit for bit anyway): per-lane partial sums combined by two
// quad exchanges.
template <class R>
__device__ __forceinline__ void quad_moments(const R (&A)[3], const R (&B)[3], R r0, R& rho_s, R (&j)[3],
                                             const int (&dI)[3][3], int nsl, int sub) {
  if constexpr (sizeof(R) == 8) {
    R r = bq<0>(A, B, r0);
    R jx = R(0.0), jy = R(0.0), jz = R(0.0);
#define FSLBM_QM(q)                                   \
  {                                                   \
    const R v = bq<q>(A, B, r0);                      \
    r = r + v;                                        \
    if (CX[q] == 1) jx = jx + v;                      \
    if (CX[q] == -1) jx = jx - v;                     \
    if (CY[q] == 1) jy = jy + v;                      \
    if (CY[q] == -1) jy = jy - v;                     \
    if (CZ[q] == 1) jz = jz + v;                      \
    if (CZ[q] == -1) jz = jz - v;                     \
  }
    FSLBM_LINKS(FSLBM_QM)
#undef FSLBM_QM
    rho_s = r;
    j[0] = jx;
    j[1] = jy;
    j[2] = jz;
  } else {
    R r = sub == 1 ? r0 : R(0.0), jx = R(0.0), jy = R(0.0), jz = R(0.0);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (s < nsl) {
        r = r + (A[s] + B[s]);
        const R dd = A[s] - B[s];
        jx = jx + R(dI[s][0]) * dd;
        jy = jy + R(dI[s][1]) * dd;
        jz = jz + R(dI[s][2]) * dd;
      }
    }
    rho_s = quad_sum(r);
    j[0] = quad_sum(jx);
    j[1] = quad_sum(jy);
    j[2] = quad_sum(jz);
  }
}

// Reconstruction of the gas-side populations of one pair (the operations of
// rebuild<F, RULE, q>).  Link A (c = d) or B (c = -d) is pulled from gas when
// its source is (gA, gB).  For link q with o = qbar the link to gas, Eq.
// (closure) takes ft_o, ft_q, the value pulled along o, n+_o and e+_o(rho_b,
// u_b).  Both links of a pair share e+ (it depends on (c.u)^2) and n+ (on the
// pair's sum); only the link with n.c_o > 0 can take the FSL row, so a pair
// needs one FSL evaluation at most.
// d . v for an integer direction and a geometry vector of type G
template <class G>
__device__ __forceinline__ G idot(const int (&d)[3], const G (&v)[3]) {
  return ((G)d[0] * v[0] + (G)d[1] * v[1]) + (G)d[2] * v[2];
}

template <class R, int RULE, class G>
__device__ __forceinline__ void rebuild_pair(R& fA, R& fB, R oA, R oB, bool gA, bool gB, const int (&d)[3], R w,
                                             R w3, bool have_n, const G (&nv)[3], G dist, R rho_t,
                                             R rho0_t, const R (&u_t)[3], R usq_t, const Consts<R>& k, bool incomp,
                                             bool stokes, const R (&Sb)[6], bool stress) {
  const R dR[3] = {R(d[0]), R(d[1]), R(d[2])};
  const R cu = ddot(dR, u_t);
  const R e_b = e_plus_w(w, cu, k.rhob_s, k.rho0b, incomp, stokes, usq_t);
  R dS = R(0.0);
  if constexpr ((RULE & 6) != 0) dS = dSd(d, Sb);
  const R fA0 = fA, fB0 = fB;
  // FSK: -ft_o + 2 e+_o(rho_b, u_b) (+ D c_o c_o : S^b, alpha_+ = 2)
  R vA = R(2.0) * e_b - oB, vB = R(2.0) * e_b - oA;
  if constexpr ((RULE & 6) != 0) {
    if (stress) {
      const R D2 = -((R(2.0) * k.Lp) * w3);
      vA = vA + D2 * dS;
      vB = vB + D2 * dS;
    }
  }
  if constexpr ((RULE & 1) != 0) {
    // link A: o = B, c_o = -d, n.c_o = -(d.n); link B: o = A, n.c_o = d.n
    const G dn = idot(d, nv);
    const bool useA = gA && !gB && have_n && -dn > G(0.0);
    const bool useB = gB && !gA && have_n && dn > G(0.0);
    if (useA || useB) {
      const G nc = useA ? -dn : dn;
      G dl;
      if constexpr (sizeof(G) == 8) dl = dist / nc;
      else dl = dist * __builtin_amdgcn_rcpf(nc);  // FP32 geometry: hardware reciprocal (1 ulp)
      if (dl < G(0.0)) dl = G(0.0);
      if (dl > G(1.0)) dl = G(1.0);
      const R delta = (R)dl;
      const R own_o = useA ? oB : oA, own_q = useA ? oA : oB, f_o = useA ? fB0 : fA0;
      const R e_o_t = e_plus_w(w, cu, rho_t, rho0_t, incomp, stokes, usq_t);
      const R n_plus = (R(0.5) * (own_o + own_q) - e_o_t) * k.inv1p;
      const R a0 = R(1.0) - (R(0.5) + delta);
      const R a1 = delta - R(1.0);
      const R Cc = k.lp * (R(0.5) + delta) - R(2.0) * k.lp;
      R v = (((a0 * own_o + R(0.5) * own_q) + a1 * f_o) + Cc * n_plus) + e_b;
      if constexpr ((RULE & 6) != 0) {
        if (stress) v = v + (-((R(1.0) * k.Lp) * w3)) * dS;  // alpha_+ = 1
      }
      if (useA) vA = v;
      else vB = v;
    }
  }
  if (gA) fA = vA;
  if (gB) fB = vB;
}

// REC: a step of an adjoint window, which also stores what the reverse step
// needs at each listed cell, in list order (rules 0 and 1).
template <class F, int RULE, bool REC = false>
__global__ __launch_bounds__(QBLOCK) void k_iface4(SweepArgs a) {
  using R = typename F::R;
  using S = typename F::S;
  // the interface geometry (normal, link distances): FP64 in the FP64 form,
  // FP32 in the FP32-arithmetic forms
  using G = typename std::conditional<sizeof(R) == 8, double, float>::type;
  constexpr bool SH = F::shifted;
  const Grid g = a.c.grid;
  const int n_i = a.counters[C_I];
  // before the sweep (order 1) this kernel opens the counters of the next step
  if (a.order && blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NCOUNT; ++c) a.counters_next[c] = 0;
  }
  const S* __restrict__ fin = reinterpret_cast<const S*>(a.fin);
  S* __restrict__ fout = reinterpret_cast<S*>(a.fout);
  S* __restrict__ rbuf = reinterpret_cast<S*>(a.rbuf);
  const unsigned N = (unsigned)g.N;  // 19 N < 2^32 is checked at init
  const float isc = a.c.inv_scale;
  const Consts<R>& k = pick_consts<R>(a.c);
  const bool incomp = a.c.incomp, stokes = a.c.stokes;
  const int sub = (int)threadIdx.x & (QUAD - 1);
  const int nsl = sub == 0 ? 3 : 2;  // pair slots of this lane
  const bool lead = sub == 0;        // lane that stores the cell's scalars
  int dI[3][3], qa[3], lo[3];
  R wq[3], w3[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int p = s == 2 ? PAIRS - 1 : sub + 4 * s;
    pair_dir(p, dI[s]);
    qa[s] = 2 * p + 1;
    wq[s] = R(p < 3 ? WD[1] : WD[7]);
    w3[s] = R(p < 3 ? W3D[1] : W3D[7]);
    lo[s] = dI[s][0] + g.nx * (dI[s][1] + g.ny * dI[s][2]);  // index offset of direction d
  }
  // Chunks of QCELLS consecutive list entries.  Workgroups go to the eight
  // XCDs round robin (workgroup b to XCD b mod 8); with a.quad == 2 the chunks
  // are dealt so that each XCD takes one contiguous stretch of the list, whose
  // cells share rows and so the lines of their neighbourhoods in that XCD's
  // L2; else chunk b, b + grid, ...
  const int nchunk = (n_i + QCELLS - 1) / QCELLS;
  const bool xcd_order = a.quad == 2;
  const int per = (nchunk + NXCD - 1) / NXCD;
  const int k0 = xcd_order ? (int)blockIdx.x / NXCD : (int)blockIdx.x;
  const int kstride = xcd_order ? (int)gridDim.x / NXCD : (int)gridDim.x;
  const int kend = xcd_order ? per : nchunk;
  for (int kk = k0; kk < kend; kk += kstride) {
    const int chunk = xcd_order ? ((int)blockIdx.x % NXCD) * per + kk : kk;
    const int i = chunk * QCELLS + ((int)threadIdx.x >> 2);
    if (chunk >= nchunk || i >= n_i) continue;  // quad-uniform
    const int idx = a.listI[i];
    // the list of order 1 comes from the step before: an entry whose cell has
    // since filled or emptied is skipped (quad-uniform)
    if (a.order && a.flags[idx] != IFACE) continue;
    Nbr n;
    coords(g, idx, n.x, n.y, n.z);
    // ---- pull sources: link A (c = d) pulls from x - d, link B (c = -d)
    // from x + d; -1 beyond a wall.  A cell off every face of the lattice
    // (no wall, no periodic wrap around it) takes them as idx -/+ the offset of d.
    int srcA[3], srcB[3];
    const bool inner = (unsigned)(n.x - 1) < (unsigned)(g.nx - 2) && (unsigned)(n.y - 1) < (unsigned)(g.ny - 2) &&
                       (unsigned)(n.z - 1) < (unsigned)(g.nz - 2);
    if (inner) {
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        srcA[s] = idx - lo[s];
        srcB[s] = idx + lo[s];
      }
    } else {
      n.xm = step_axis(n.x, -1, g.nx, g.px);
      n.xp = step_axis(n.x, 1, g.nx, g.px);
      n.ym = step_axis(n.y, -1, g.ny, g.py);
      n.yp = step_axis(n.y, 1, g.ny, g.py);
      n.zm = step_axis(n.z, -1, g.nz, g.pz);
      n.zp = step_axis(n.z, 1, g.nz, g.pz);
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int* d = dI[s];
        const int xa = d[0] == 1 ? n.xm : (d[0] == -1 ? n.xp : n.x);
        const int ya = d[1] == 1 ? n.ym : (d[1] == -1 ? n.yp : n.y);
        const int za = d[2] == 1 ? n.zm : (d[2] == -1 ? n.zp : n.z);
        const int xb = d[0] == 1 ? n.xp : (d[0] == -1 ? n.xm : n.x);
        const int yb = d[1] == 1 ? n.yp : (d[1] == -1 ? n.ym : n.y);
        const int zb = d[2] == 1 ? n.zp : (d[2] == -1 ? n.zm : n.z);
        srcA[s] = ((xa | ya | za) < 0) ? -1 : xa + g.nx * (ya + g.ny * za);
        srcB[s] = ((xb | yb | zb) < 0) ? -1 : xb + g.nx * (yb + g.ny * zb);
      }
    }
    // ---- loads.  Pull, Eq. (lbe1): f_q(x) = ft_q(x - c_q); beyond a wall
    // halfway bounce-back f_q(x) = ft_qbar(x).
    QuadLinks<R> L;
    // classes of the pull sources first: the value pulled from a gas source
    // is replaced by the reconstruction and the fill of a source counts only
    // where it is an interface cell, so those loads are made only where needed
    // (a wall source takes the cell's own fill)
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      L.tA[s] = L.tB[s] = GAS;
      if (s < nsl) {
        const int sa = srcA[s], sb = srcB[s];
        const uint8_t ta = a.flags[sa >= 0 ? sa : idx], tb = a.flags[sb >= 0 ? sb : idx];
        L.tA[s] = sa >= 0 ? (int)ta : (int)WALL_CLASS;
        L.tB[s] = sb >= 0 ? (int)tb : (int)WALL_CLASS;
      }
    }
    const double m_old = a.mass_in[idx];
    const double phix = a.phi_in[idx];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      L.oA[s] = L.oB[s] = R(0.0);
      if (s < nsl) {
        const unsigned qA = (unsigned)qa[s], qB = qA + 1u;
        L.oA[s] = F::load(fin + (qA * N + (unsigned)idx), isc);
        L.oB[s] = F::load(fin + (qB * N + (unsigned)idx), isc);
      }
    }
    L.f0 = sub == 1 ? F::load(fin + (unsigned)idx, isc) : R(0.0);
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      L.fA[s] = L.fB[s] = R(0.0);
      L.pA[s] = L.pB[s] = phix;
      if (s < nsl) {
        const int sa = srcA[s], sb = srcB[s];
        const unsigned qA = (unsigned)qa[s], qB = qA + 1u;
        const unsigned offA = sa >= 0 ? qA * N + (unsigned)sa : qB * N + (unsigned)idx;
        const unsigned offB = sb >= 0 ? qB * N + (unsigned)sb : qA * N + (unsigned)idx;
        if (L.tA[s] != GAS) L.fA[s] = F::load(fin + offA, isc);
        if (L.tB[s] != GAS) L.fB[s] = F::load(fin + offB, isc);
        if (L.tA[s] == IFACE) L.pA[s] = a.phi_in[sa];
        if (L.tB[s] == IFACE) L.pB[s] = a.phi_in[sb];
      }
    }

    if constexpr (REC) {
      // the record: pulled and own populations of time t (each lane its links,
      // lane 1 the rest link), fill and mass.  A value pulled from a gas source
      // is not loaded and is recorded as 0: the reverse step reads the pulled
      // values of liquid and interface sources only.  Non-temporal stores: the
      // record is read once, in the reverse pass.
      R* __restrict__ rf = reinterpret_cast<R*>(a.rec_f);
      R* __restrict__ ro = reinterpret_cast<R*>(a.rec_own);
      const unsigned cap = (unsigned)a.rec_cap, ui = (unsigned)i;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (s < nsl) {
          const unsigned qA = (unsigned)qa[s], qB = qA + 1u;
          __builtin_nontemporal_store(L.fA[s], &rf[qA * cap + ui]);
          __builtin_nontemporal_store(L.fB[s], &rf[qB * cap + ui]);
          __builtin_nontemporal_store(L.oA[s], &ro[qA * cap + ui]);
          __builtin_nontemporal_store(L.oB[s], &ro[qB * cap + ui]);
        }
      }
      if (sub == 1) {
        __builtin_nontemporal_store(L.f0, &rf[ui]);
        __builtin_nontemporal_store(L.f0, &ro[ui]);
      }
      if (lead) {
        __builtin_nontemporal_store(phix, &a.rec_phi[i]);
        __builtin_nontemporal_store(m_old, &a.rec_m[i]);
      }
    }

    // ---- link classes of the cell (bit q: source of link q is gas / liquid /
    // takes part in the mass exchange), OR-combined over the quad
    uint32_t gm = 0, lm = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (s < nsl) {
        gm |= (L.tA[s] == GAS ? 1u : 0u) << qa[s];
        gm |= (L.tB[s] == GAS ? 1u : 0u) << (qa[s] + 1);
        lm |= (L.tA[s] == LIQ ? 1u : 0u) << qa[s];
        lm |= (L.tB[s] == LIQ ? 1u : 0u) << (qa[s] + 1);
      }
    }
    gm |= qperm<QP_XOR1>(gm);
    gm |= qperm<QP_XOR2>(gm);
    lm |= qperm<QP_XOR1>(lm);
    lm |= qperm<QP_XOR2>(lm);
    const uint32_t gasmask = gm, liqmask = lm;

    // ---- mass exchange (FP64): dm = sum_q w (ft_q(x-c_q) - ft_qbar(x)); weight 1
    // to liquid, (phi_x + phi_s)/2 to interface, nothing from gas or walls.  Each
    // link's term is formed in its lane and summed in link order in every lane.
    double tmA[3], tmB[3];
    uint32_t xm = 0;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      tmA[s] = tmB[s] = 0.0;
      if (s < nsl) {
        const double dA = (double)L.fA[s] - (double)L.oB[s];
        const double dB = (double)L.fB[s] - (double)L.oA[s];
        if (L.tA[s] == LIQ) tmA[s] = dA;
        if (L.tA[s] == IFACE) tmA[s] = (0.5 * (phix + L.pA[s])) * dA;
        if (L.tB[s] == LIQ) tmB[s] = dB;
        if (L.tB[s] == IFACE) tmB[s] = (0.5 * (phix + L.pB[s])) * dB;
        xm |= ((L.tA[s] == LIQ || L.tA[s] == IFACE) ? 1u : 0u) << qa[s];
        xm |= ((L.tB[s] == LIQ || L.tB[s] == IFACE) ? 1u : 0u) << (qa[s] + 1);
      }
    }
    xm |= qperm<QP_XOR1>(xm);
    xm |= qperm<QP_XOR2>(xm);
    double dm = 0.0;
    if constexpr (sizeof(R) == 8) {
#define FSLBM_QDM(q)                                    \
  {                                                     \
    const double t = bq<q>(tmA, tmB, 0.0);              \
    if ((xm >> q) & 1u) dm = dm + t;                    \
  }
      FSLBM_LINKS(FSLBM_QDM)
#undef FSLBM_QDM
    } else {
#pragma unroll
      for (int s = 0; s < 3; ++s) dm = dm + (tmA[s] + tmB[s]);
      dm = quad_sum(dm);
    }
    const double m_new = m_old + dm;

    if (gasmask) {
      // ---- interface geometry: n = -grad(phi)/|grad(phi)| by central
      // differences over the six axis neighbours (links 1..6: lanes 0, 1, 2, slot 0)
      const G psA = L.tA[0] == LIQ ? G(1.0) : (L.tA[0] == GAS ? G(0.0) : (G)L.pA[0]);
      const G psB = L.tB[0] == LIQ ? G(1.0) : (L.tB[0] == GAS ? G(0.0) : (G)L.pB[0]);
      const G p1 = qbcast<0>(psA), p2 = qbcast<0>(psB);
      const G p3 = qbcast<1>(psA), p4 = qbcast<1>(psB);
      const G p5 = qbcast<2>(psA), p6 = qbcast<2>(psB);
      const G gx = G(0.5) * (p2 - p1);
      const G gy = G(0.5) * (p4 - p3);
      const G gz = G(0.5) * (p6 - p5);
      const G nrm2 = (gx * gx + gy * gy) + gz * gz;
      const bool have_n = nrm2 > G(0.0);
      G nv[3] = {G(0.0), G(0.0), G(0.0)};
      if (have_n) {
        if constexpr (sizeof(G) == 8) {
          const G nrm = sqrt(nrm2);
          nv[0] = -gx / nrm;
          nv[1] = -gy / nrm;
          nv[2] = -gz / nrm;
        } else {
          // FP32 geometry: hardware reciprocal square root (1 ulp)
          const G r = __builtin_amdgcn_rsqf(nrm2);
          nv[0] = -gx * r;
          nv[1] = -gy * r;
          nv[2] = -gz * r;
        }
      }
      const G dist = (G)phix - G(0.5);
      // ---- moments of time t from the own post-collision populations
      R rho_t, j_t[3], u_t[3];
      quad_moments(L.oA, L.oB, L.f0, rho_t, j_t, dI, nsl, sub);
      const R rho0_t = rho0_of<R, SH>(rho_t, incomp);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R U = incomp ? j_t[c] : j_t[c] / rho0_t;
        u_t[c] = (U - k.g[c]) + k.hg[c];
      }
      const R usq_t = usq_of(u_t);
      // ---- boundary shear rate for the rules with D != 0: from the bulk
      // (needs the local basis) or prescribed
      R Sb[6] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
      const bool stress = ((RULE & 2) && have_n) || (RULE & 4);
      if constexpr ((RULE & 2) != 0) {
        if (stress) {
          // liquid neighbour x + c_k whose link points most directly into the
          // liquid (largest -c_k.n / |c_k|, lowest k on ties); x + c_k is the
          // pull source of link kbar
          int best = -1, bx = 0, by = 0, bz = 0;
          double best_v = 0.0;
          const double nvd[3] = {(double)nv[0], (double)nv[1], (double)nv[2]};
#define FSLBM_QBULK(kk)                                                              \
  if ((liqmask >> OPP[kk]) & 1u) {                                                   \
    const double cn = -cdot<kk>(nvd);                                                \
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
          FSLBM_LINKS(FSLBM_QBULK)
#undef FSLBM_QBULK
          R bA[3], bB[3], b0;
          if (best < 0) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
              bA[s] = L.oA[s];
              bB[s] = L.oB[s];
            }
            b0 = L.f0;
          } else {
            const int sx = step_axis(n.x, bx, g.nx, g.px), sy = step_axis(n.y, by, g.ny, g.py);
            const int sz = step_axis(n.z, bz, g.nz, g.pz);
            const unsigned sn = (unsigned)(sx + g.nx * (sy + g.ny * sz));  // a liquid cell: inside the lattice
#pragma unroll
            for (int s = 0; s < 3; ++s) {
              bA[s] = bB[s] = R(0.0);
              if (s < nsl) {
                bA[s] = F::load(fin + ((unsigned)qa[s] * N + sn), isc);
                bB[s] = F::load(fin + ((unsigned)(qa[s] + 1) * N + sn), isc);
              }
            }
            b0 = sub == 1 ? F::load(fin + sn, isc) : R(0.0);
          }
          R rho_n, j_n[3], u_n[3];
          quad_moments(bA, bB, b0, rho_n, j_n, dI, nsl, sub);
          const R rho0_n = rho0_of<R, SH>(rho_n, incomp);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const R U = incomp ? j_n[c] : j_n[c] / rho0_n;
            u_n[c] = (U - k.g[c]) + k.hg[c];
          }
          const R usq_n = usq_of(u_n);
          // 2 n+ of each pair in its lane, M = sum over pairs in link order
          R n2[3];
#pragma unroll
          for (int s = 0; s < 3; ++s) {
            const R dR[3] = {R(dI[s][0]), R(dI[s][1]), R(dI[s][2])};
            const R fplus = R(0.5) * (bA[s] + bB[s]);
            const R np = (fplus - e_plus_w(wq[s], ddot(dR, u_n), rho_n, rho0_n, incomp, stokes, usq_n)) * k.inv1p;
            n2[s] = R(2.0) * np;
          }
          R M[6] = {R(0.0), R(0.0), R(0.0), R(0.0), R(0.0), R(0.0)};
#define FSLBM_QMNEQ(q)                                                 \
  {                                                                    \
    const R v = bq<q>(n2, n2, R(0.0));                                 \
    M[0] = M[0] + R(CX[q] * CX[q]) * v;                                \
    M[1] = M[1] + R(CY[q] * CY[q]) * v;                                \
    M[2] = M[2] + R(CZ[q] * CZ[q]) * v;                                \
    M[3] = M[3] + R(CX[q] * CY[q]) * v;                                \
    M[4] = M[4] + R(CX[q] * CZ[q]) * v;                                \
    M[5] = M[5] + R(CY[q] * CZ[q]) * v;                                \
  }
          FSLBM_QMNEQ(1) FSLBM_QMNEQ(3) FSLBM_QMNEQ(5) FSLBM_QMNEQ(7) FSLBM_QMNEQ(9) FSLBM_QMNEQ(11)
          FSLBM_QMNEQ(13) FSLBM_QMNEQ(15) FSLBM_QMNEQ(17)
#undef FSLBM_QMNEQ
          const R tr5 = ((M[0] + M[1]) + M[2]) / R(5.0);
          const R fs = R(1.5) * k.lp;  // lambda_+ / (2 c_s^2)
          double Sd[6];
          Sd[0] = (double)(fs * (M[0] - tr5));
          Sd[1] = (double)(fs * (M[1] - tr5));
          Sd[2] = (double)(fs * (M[2] - tr5));
          Sd[3] = (double)(fs * M[3]);
          Sd[4] = (double)(fs * M[4]);
          Sd[5] = (double)(fs * M[5]);
          // normal entry of the boundary value: n.S.n / 3; S^b = P S P + s_nn n n^T
          const double ndg = (Sd[0] * (nvd[0] * nvd[0]) + Sd[1] * (nvd[1] * nvd[1])) + Sd[2] * (nvd[2] * nvd[2]);
          const double nof = (Sd[3] * (nvd[0] * nvd[1]) + Sd[4] * (nvd[0] * nvd[2])) + Sd[5] * (nvd[1] * nvd[2]);
          const double s_nn = (ndg + 2.0 * nof) / 3.0;
          double Sn[3];
          Sn[0] = (Sd[0] * nvd[0] + Sd[3] * nvd[1]) + Sd[4] * nvd[2];
          Sn[1] = (Sd[3] * nvd[0] + Sd[1] * nvd[1]) + Sd[5] * nvd[2];
          Sn[2] = (Sd[4] * nvd[0] + Sd[5] * nvd[1]) + Sd[2] * nvd[2];
          const double kk = ((nvd[0] * Sn[0] + nvd[1] * Sn[1]) + nvd[2] * Sn[2]) + s_nn;
          constexpr int IA[6] = {0, 1, 2, 0, 0, 1}, IB[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
          for (int c = 0; c < 6; ++c)
            Sb[c] = (R)(((Sd[c] - Sn[IA[c]] * nvd[IB[c]]) - nvd[IA[c]] * Sn[IB[c]]) + kk * (nvd[IA[c]] * nvd[IB[c]]));
        }
      }
      if constexpr ((RULE & 4) != 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) Sb[c] = (R)a.c.shear_b[c];
      }
      // ---- reconstruction of every population pulled from gas, Eq. (closure)
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        if (s < nsl) {
          const bool gA = (gasmask >> qa[s]) & 1u, gB = (gasmask >> (qa[s] + 1)) & 1u;
          if (gA || gB)
            rebuild_pair<R, RULE, G>(L.fA[s], L.fB[s], L.oA[s], L.oB[s], gA, gB, dI[s], wq[s], w3[s], have_n, nv, dist,
                                  rho_t, rho0_t, u_t, usq_t, k, incomp, stokes, Sb, stress);
        }
      }
    }

    // ---- TRT collision, Eq. (lbe2): moments of the quad in link order, then
    // each lane relaxes its own pairs (and lane 1 the rest link)
    R rho_s, j[3], u[3], ueq[3];
    quad_moments(L.fA, L.fB, L.f0, rho_s, j, dI, nsl, sub);
    const R rho0 = rho0_of<R, SH>(rho_s, incomp);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const R U = incomp ? j[c] : j[c] / rho0;
      u[c] = U + k.hg[c];
      ueq[c] = U - k.glm[c];
    }
    if constexpr (sizeof(R) == 8) {
      const R usq = usq_of(u);
      if (sub == 1) {
        const R ep = e_plus_w(R(WD[0]), R(0.0), rho_s, rho0, incomp, stokes, usq);
        L.f0 = L.f0 + k.lp * (L.f0 - ep);
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const R dR[3] = {R(dI[s][0]), R(dI[s][1]), R(dI[s][2])};
        const R fp = R(0.5) * (L.fA[s] + L.fB[s]);
        const R fm = R(0.5) * (L.fA[s] - L.fB[s]);
        const R np = fp - e_plus_w(wq[s], ddot(dR, u), rho_s, rho0, incomp, stokes, usq);
        R cue = ddot(dR, ueq);
        if (!incomp) cue = rho0 * cue;
        const R nm = fm - w3[s] * cue;
        const R A0 = L.fA[s], B0 = L.fB[s];
        L.fA[s] = (A0 + k.lp * np) + k.lm * nm;
        L.fB[s] = (B0 + k.lp * np) - k.lm * nm;
      }
    } else {
      // the FP32 collision with fused multiply-adds (collide_f32)
      const float m15usq = -1.5f * usq_of(u);
      const float rho0f = rho0;
      auto ep_of = [&](float w, float cu) -> float {
        const float wr = w * rho_s;
        if (stokes) return wr;
        float nl = __builtin_fmaf(4.5f * cu, cu, m15usq);
        if (!incomp) nl = rho0f * nl;
        return __builtin_fmaf(w, nl, wr);
      };
      if (sub == 1) {
        const float ep = ep_of(float(WD[0]), 0.0f);
        L.f0 = __builtin_fmaf(k.lp, L.f0 - ep, L.f0);
      }
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const float dR[3] = {float(dI[s][0]), float(dI[s][1]), float(dI[s][2])};
        const float cu = ddot(dR, u);
        const float cue = ddot(dR, ueq);
        const float em = w3[s] * (incomp ? cue : rho0f * cue);
        const float ep = ep_of(wq[s], cu);
        const float A0 = L.fA[s], B0 = L.fB[s];
        const float np = 0.5f * (A0 + B0) - ep;
        const float nm = 0.5f * (A0 - B0) - em;
        const float lpn = k.lp * np;
        L.fA[s] = __builtin_fmaf(k.lm, nm, A0 + lpn);
        L.fB[s] = __builtin_fmaf(-k.lm, nm, B0 + lpn);
      }
    }
    // ---- stores: populations of the lane's links (order 1: into list entry
    // i of rbuf, which the sweep stores with its rows; past rcap, and in
    // order 0, into the cell); the cell's scalars (FP64 bookkeeping) and
    // classification from lane 0
    const bool to_r = a.order && i < a.rcap;
    S* const pb = to_r ? rbuf + i : fout + idx;
    const unsigned ps = to_r ? (unsigned)a.rcap : N;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      if (s < nsl) {
        F::store(pb + (unsigned)qa[s] * ps, L.fA[s], a.c.scale);
        F::store(pb + (unsigned)(qa[s] + 1) * ps, L.fB[s], a.c.scale);
      }
    }
    if (sub == 1) F::store(pb, L.f0, a.c.scale);
    const double rho = SH ? 1.0 + (double)rho_s : (double)rho_s;
    bool filled = false, emptied = false;
    if (REC && lead) {
      R* __restrict__ ru = reinterpret_cast<R*>(a.rec_u);
      const unsigned cap = (unsigned)a.rec_cap;
#pragma unroll
      for (int c = 0; c < 3; ++c) __builtin_nontemporal_store(u[c], &ru[(unsigned)c * cap + (unsigned)i]);
      __builtin_nontemporal_store(rho, &a.rec_rho[i]);
    }
    if (lead) {
      a.mass[idx] = a.hold ? m_old : m_new;
      a.phi_out[idx] = a.hold ? phix : m_new / rho;
      *reinterpret_cast<double4*>(a.aux + 4 * (size_t)idx) = make_double4(rho, (double)u[0], (double)u[1], (double)u[2]);
      if (!a.freeze) {
        filled = m_new > a.thr_hi * rho;
        emptied = m_new < a.thr_lo * rho;
        if (filled) a.f_epoch[idx] = a.step;
      }
    }
    if (!a.freeze) {
      wave_append(filled, &a.counters[C_F], a.listF, idx);
      wave_append(emptied, &a.counters[C_E], a.listE, idx);
    }
  }
}

template <class F, int RULE, bool REC = false>
static void iface4_go(const StepLaunch& L) {
  // a window step's list is fixed and its length (rec_cap) known here
  const size_t cells = REC ? (size_t)L.sweep.rec_cap : (size_t)L.sweep.c.grid.N;
  unsigned nb = std::min<unsigned>(IFACE4_GRID, (unsigned)std::max<size_t>(1, (cells + QCELLS - 1) / QCELLS));
  nb = (nb + NXCD - 1) / NXCD * NXCD;
  k_iface4<F, RULE, REC><<<nb, QBLOCK, 0, (hipStream_t)L.stream>>>(L.sweep);
}

template <class F>
static void iface4_form(const StepLaunch& L, int rule) {
  if (L.sweep.rec_f) {  // a window step (rules 0 and 1)
    if (rule == 0) iface4_go<F, 0, true>(L);
    else iface4_go<F, 1, true>(L);
    return;
  }
  switch (rule) {
    case 0: iface4_go<F, 0>(L); break;
    case 1: iface4_go<F, 1>(L); break;
    case 2: iface4_go<F, 2>(L); break;
    case 3: iface4_go<F, 3>(L); break;
    case 4: iface4_go<F, 4>(L); break;
    default: iface4_go<F, 5>(L); break;
  }
}

hipError_t launch_iface4(const StepLaunch& L, int precision, int rule) {
  if (precision == 0) iface4_form<FormF64>(L, rule);
  else if (precision == 1) iface4_form<FormF32>(L, rule);
  else iface4_form<FormF16>(L, rule);
  return hipGetLastError();
}

}  // namespace fslbm
