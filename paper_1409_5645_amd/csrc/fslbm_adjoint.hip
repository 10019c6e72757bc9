// Reverse-mode (adjoint) kernels of the free-surface LBM step over a window of
// steps with frozen cell classes (no conversions), for the incompressible
// equilibrium with its quadratic term.
//
// A forward step maps the state (ft, m, phi) of time t to time t+1:
//   pull (Eq. lbe1) -> [interface cells: mass exchange; normal from the fill
//   gradient; FSK / FSL reconstruction of the gas-side populations, Eq.
//   (closure) with Table 1 or Eq. (fsli1)-(fsli4)] -> TRT collision (Eq. lbe2)
//   -> [interface cells: phi = m / rho].
// The adjoint maps lambda = dL/d(state) of time t+1 to time t.  The adjoint of
// the pull is a push: the adjoint of a pulled value is written to the very
// element the pull read (the source population, or the cell's own opposite
// population at a wall).  Every element is read by exactly one pull, so the
// push needs no atomics.
//
//   k_adj_sweep    liquid cells: pull of time t (for the collision velocity),
//                  collision adjoint, push.
//   k_adj_iface    interface cells, four lanes per cell: recompute of the
//                  exchange, normal and moments of time t (the collision state
//                  is in the record);
//                  adjoint of phi = m/rho, of the collision, reconstruction,
//                  normal and mass exchange; push; own-population and fill
//                  terms to per-cell scratch.
//   k_adj_iface2   interface cells: add the own-population terms (set them where
//                  the pull that reads the element comes from gas) and gather the
//                  fill adjoint from the cell and its interface neighbours.
// Parameter gradients (dL/drho_b, dL/dg) are summed per wavefront or block in
// FP64 into fixed slots and reduced at the end in a fixed order: a run is reproducible
// bit for bit.
#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"
#include "fslbm_quad.hpp"
#include "fslbm_stencil.hpp"

#include <algorithm>
#include <type_traits>

namespace fslbm {

constexpr int ABLOCK = 256;
constexpr int AIBLOCK = 64;  // interface-list kernels: one wavefront per block
static constexpr unsigned ADJ_IFACE_GRID = 16384;

// v += c_q t
template <int q, class R>
__device__ __forceinline__ void cadd(R (&v)[3], R t) {
  if (CX[q] == 1) v[0] = v[0] + t;
  if (CX[q] == -1) v[0] = v[0] - t;
  if (CY[q] == 1) v[1] = v[1] + t;
  if (CY[q] == -1) v[1] = v[1] - t;
  if (CZ[q] == 1) v[2] = v[2] + t;
  if (CZ[q] == -1) v[2] = v[2] - t;
}

// Adjoint of the TRT collision, Eq. (lbe2), with the force in
// u = U + g/2, u_eq = U - g/lambda_- (incompressible: U = sum_q c_q f_q).
// ob = dL/d(post-collision f), u = collision velocity, rho_extra = dL/drho
// from elsewhere.  Returns fb = dL/d(pre-collision f) and gb = dL/dg.
//   out_q    = f_q    + lambda_+ n+ + lambda_- n-
//   out_qbar = f_qbar + lambda_+ n+ - lambda_- n-,  n+- = (f_q +- f_qbar)/2 - e+-_q
template <class R>
__device__ __forceinline__ void collide_adjoint(const R (&ob)[Q], const R (&u)[3], R rho_extra, const Consts<R>& k,
                                                R (&fb)[Q], R (&gb)[3]) {
  R rb = R(0.0);                         // sum_q w_q dL/de+_q
  R s9[3] = {R(0.0), R(0.0), R(0.0)};    // sum_q w_q dL/de+_q (c_q.u) c_q
  R ue[3] = {R(0.0), R(0.0), R(0.0)};    // dL/du_eq = sum_q 3 w_q dL/de-_q c_q
  R hp[Q], hm[Q];                        // half of dL/dn+ and dL/dn- per pair
  {
    const R np_b = k.lp * ob[0];
    rb = rb + R(WD[0]) * (-np_b);
  }
#define FSLBM_CADJ(q)                                   \
  {                                                     \
    const R np_b = k.lp * (ob[q] + ob[q + 1]);          \
    const R nm_b = k.lm * (ob[q] - ob[q + 1]);          \
    const R we = R(WD[q]) * (-np_b);                    \
    rb = rb + we;                                       \
    cadd<q>(s9, we * cdot<q>(u));                       \
    cadd<q>(ue, R(W3D[q]) * (-nm_b));                   \
    hp[q] = R(0.5) * np_b;                              \
    hm[q] = R(0.5) * nm_b;                              \
  }
  FSLBM_CADJ(1) FSLBM_CADJ(3) FSLBM_CADJ(5) FSLBM_CADJ(7) FSLBM_CADJ(9) FSLBM_CADJ(11) FSLBM_CADJ(13)
  FSLBM_CADJ(15) FSLBM_CADJ(17)
#undef FSLBM_CADJ
  R jb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const R ub = R(9.0) * s9[a] - R(3.0) * (u[a] * rb);  // dL/du
    jb[a] = ub + ue[a];                                   // u and u_eq both move with U = j
    gb[a] = R(0.5) * ub - ue[a] * k.ilm;                  // u = U + g/2, u_eq = U - g/lambda_-
  }
  const R rt = rb + rho_extra;
  fb[0] = (R(1.0) + k.lp) * ob[0] + rt;
#define FSLBM_FADJ(q)                                   \
  {                                                     \
    const R cj = cdot<q>(jb);                           \
    fb[q] = ((ob[q] + hp[q]) + hm[q]) + (rt + cj);      \
    fb[q + 1] = ((ob[q + 1] + hp[q]) - hm[q]) + (rt - cj); \
  }
  FSLBM_FADJ(1) FSLBM_FADJ(3) FSLBM_FADJ(5) FSLBM_FADJ(7) FSLBM_FADJ(9) FSLBM_FADJ(11) FSLBM_FADJ(13)
  FSLBM_FADJ(15) FSLBM_FADJ(17)
#undef FSLBM_FADJ
}

// row_ror:4 and row_ror:8: lane i of a row of 16 receives lane (i - 4) mod 16, (i - 8) mod 16
constexpr int DPP_ROW_ROR4 = 0x124;
constexpr int DPP_ROW_ROR8 = 0x128;

__device__ __forceinline__ double read_lane(double v, int lane) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// *slot += v as an atomic add without return: the wavefront need not wait for
// its stores to complete (a load of the slot would).  Every slot is owned by one
// wavefront per launch and launches are ordered, so the additions into a slot
// happen in the same order on every run.
__device__ __forceinline__ void slot_add(double* slot, double v) { (void)atomicAdd(slot, v); }

// Sum of v over the wavefront in a fixed order (quads, rows of 16, then the
// four rows), the same value in every lane; all 64 lanes must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v = quad_sum(v);
  v = v + qperm<DPP_ROW_ROR4>(v);
  v = v + qperm<DPP_ROW_ROR8>(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// ------------------------------------------------------------ liquid cells
// Same row mapping and pull offsets as the forward sweep; the push writes the
// adjoint of each pulled value to the offset the pull read.  The collision
// adjoint needs only the collision velocity, which the forward step stored.
// OFF32: every population plane array is below 4 GiB, so elements are reached
// as base + 32-bit byte offset (one VALU op less per access).
template <class F, bool OFF32>
__global__ __launch_bounds__(ABLOCK) void k_adj_sweep(AdjArgs a) {
  using R = typename F::R;
  auto elem = [](auto* base, unsigned e) -> auto& {
    if constexpr (OFF32)
      return *reinterpret_cast<std::remove_pointer_t<decltype(base)>*>(
          reinterpret_cast<std::conditional_t<std::is_const_v<std::remove_pointer_t<decltype(base)>>, const char*,
                                              char*>>(base) +
          e * (unsigned)sizeof(R));
    else
      return base[e];
  };
  const Grid g = a.c.grid;
  const int row = (int)blockIdx.x / a.cpr;
  const int chunk = (int)blockIdx.x - row * a.cpr;
  const int y = row % g.ny, z = row / g.ny;
  const int x = chunk * ABLOCK + (int)threadIdx.x;
  const unsigned rbase = (unsigned)row * (unsigned)g.nx;
  const uint8_t t = x < g.nx ? a.flags[rbase + x] : GAS;
  const bool liq = t == LIQ;
  if (__ballot(liq) == 0) return;  // whole wavefronts leave together (the sum below exchanges lanes)
  double gs[3] = {0.0, 0.0, 0.0};
  if (liq) {
    const int ym = step_axis(y, -1, g.ny, g.py), yp = step_axis(y, 1, g.ny, g.py);
    const int zm = step_axis(z, -1, g.nz, g.pz), zp = step_axis(z, 1, g.nz, g.pz);
    auto row_of = [&](int sy, int sz) -> unsigned {
      return (sy < 0 || sz < 0) ? WALL_ROW : (unsigned)(sy + g.ny * sz) * (unsigned)g.nx;
    };
    const unsigned srow[9] = {row_of(yp, zp), row_of(y, zp), row_of(ym, zp),
                              row_of(yp, z),  rbase,         row_of(ym, z),
                              row_of(yp, zm), row_of(y, zm), row_of(ym, zm)};
    const int xm = step_axis(x, -1, g.nx, g.px), xp = step_axis(x, 1, g.nx, g.px);
    const unsigned N = (unsigned)g.N;
    const R* __restrict__ lin = reinterpret_cast<const R*>(a.lam_in);
    const R* __restrict__ un = reinterpret_cast<const R*>(a.u);
    unsigned off[Q];
    R ob[Q];
#define FSLBM_APULL(q)                                                                            \
  {                                                                                               \
    const unsigned ro = srow[(CY[q] + 1) + 3 * (CZ[q] + 1)];                                      \
    const int sx = CX[q] == 1 ? xm : (CX[q] == -1 ? xp : x);                                      \
    off[q] = (ro == WALL_ROW || sx < 0) ? (unsigned)OPP[q] * N + rbase + (unsigned)x              \
                                        : (unsigned)q * N + ro + (unsigned)sx;                    \
    ob[q] = elem(lin, (unsigned)q * N + rbase + (unsigned)x);                                     \
  }
    FSLBM_APULL(0)
    FSLBM_LINKS(FSLBM_APULL)
#undef FSLBM_APULL
    const Consts<R>& k = pick_consts<R>(a.c);
    const R u[3] = {elem(un, rbase + (unsigned)x), elem(un, N + rbase + (unsigned)x),
                    elem(un, 2u * N + rbase + (unsigned)x)};
    R fb[Q], gb[3];
    collide_adjoint(ob, u, R(0.0), k, fb, gb);
    R* __restrict__ lout = reinterpret_cast<R*>(a.lam_out);
#pragma unroll
    for (int q = 0; q < Q; ++q) elem(lout, off[q]) = fb[q];
#pragma unroll
    for (int i = 0; i < 3; ++i) gs[i] = (double)gb[i];
  }
  // dL/dg of the wavefront, added to its own slot
#pragma unroll
  for (int c = 0; c < 3; ++c) gs[c] = wave_sum(gs[c]);
  if ((threadIdx.x & 63) == 0) {
    double* slot = a.part_sweep + 3 * ((size_t)blockIdx.x * (ABLOCK / 64) + (threadIdx.x >> 6));
#pragma unroll
    for (int c = 0; c < 3; ++c) slot_add(slot + c, gs[c]);
  }
}

// --------------------------------------------------------- interface cells
// Four lanes per interface cell (a quad).  The 18 moving links form 9 pairs of
// opposites (q, q+1), q odd; lane s of the quad owns pairs s and s + 4, lane 0
// also pair 8 and lane 1 the rest link.  The reconstruction of a gas-side f_q
// involves only q and its opposite, and the mass exchange of link q only q and
// its opposite, so all per-link work of a pair stays in its lane.  Sums over
// the links (moments, mass change, collision and reconstruction adjoints) are
// per-lane partial sums combined across the quad by two DPP exchanges, which
// leave the same bits in all four lanes.
constexpr int CELLS_PER_BLOCK = AIBLOCK / QUAD;

template <class F, int RULE>
__global__ __launch_bounds__(AIBLOCK) void k_adj_iface(AdjArgs a) {
  using R = typename F::R;
  const Grid g = a.c.grid;
  const unsigned N = (unsigned)g.N;
  const unsigned cap = (unsigned)a.cap;
  const R* __restrict__ rf = reinterpret_cast<const R*>(a.rec_f);
  const R* __restrict__ ro = reinterpret_cast<const R*>(a.rec_own);
  const R* __restrict__ ru = reinterpret_cast<const R*>(a.rec_u);
  const R* __restrict__ lin = reinterpret_cast<const R*>(a.lam_in);
  R* __restrict__ lout = reinterpret_cast<R*>(a.lam_out);
  R* __restrict__ own_t = reinterpret_cast<R*>(a.own);
  const Consts<R>& k = pick_consts<R>(a.c);
  const int sub = (int)threadIdx.x & (QUAD - 1);
  const int nsl = sub == 0 ? 3 : 2;  // pairs of this lane
  const bool rest = sub == 1;        // lane with the rest link
  const bool lead = sub == 0;        // lane that stores the cell's scalars
  int pp[3], dI[3][3];
  R dR[3][3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    pp[s] = s == 2 ? PAIRS - 1 : sub + 4 * s;
    pair_dir(pp[s], dI[s]);
#pragma unroll
    for (int c = 0; c < 3; ++c) dR[s][c] = R(dI[s][c]);
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // dL/drho_b, dL/dg (lead lanes)
  static_assert(AIBLOCK == 64, "one wavefront per block");
  for (int i = (int)(blockIdx.x * CELLS_PER_BLOCK) + ((int)threadIdx.x >> 2); i < a.n_i;
       i += (int)gridDim.x * CELLS_PER_BLOCK) {
    const int idx = a.listI[i];
    const unsigned ui = (unsigned)i;
    int x, y, z;
    coords(g, idx, x, y, z);
    // ---- loads: the cell's scalars (all four lanes) and the lane's pairs, from
    // the step's record (list order) and the fixed topology
    const uint64_t cls = a.ncls[i];
    const double phix = a.rec_phi[i];
    const double m0 = a.rec_m[i];
    const double lam_m = a.lam_m[idx];
    const double lam_p = a.lphi_in[idx];
    const double rho = a.rec_rho[i];
    const R u[3] = {ru[ui], ru[cap + ui], ru[2u * cap + ui]};
    R f[3][2], own[3][2], ob[3][2];
    int ty[3][2];
    double ph[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        f[s][h] = own[s][h] = ob[s][h] = R(0.0);
        ty[s][h] = GAS;
        ph[s][h] = 0.0;
        if (s < nsl) {
          const unsigned L = 2u * (unsigned)pp[s] + 1u + (unsigned)h;
          f[s][h] = rf[L * cap + ui];
          own[s][h] = ro[L * cap + ui];
          ob[s][h] = lin[L * N + (unsigned)idx];
          ty[s][h] = (int)(cls >> (2 * L)) & 3;  // 0 gas, 1 interface, 2 liquid, 3 beyond a wall
          ph[s][h] = ty[s][h] == WALL_CLASS ? phix : a.rec_phi[a.nslot[L * cap + ui]];
        }
      }
    const R own0 = rest ? ro[ui] : R(0.0);
    const R ob0 = rest ? lin[idx] : R(0.0);

    // ---- forward recompute of what the reverse steps need (the collision's
    // velocity and density come from the record)
    // mass exchange: dm = sum_q w (f_q(pulled) - ft_qbar), w = 1 liquid, (phi_x + phi_s)/2 interface
    double dm = 0.0;
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int t = ty[s][h];
        if (s < nsl && (t == LIQ || t == IFACE)) {
          const double diff = (double)f[s][h] - (double)own[s][1 - h];
          dm = dm + (t == LIQ ? diff : (0.5 * (phix + ph[s][h])) * diff);
        }
      }
    dm = quad_sum(dm);
    const double m_new = m0 + dm;
    // normal n = -grad(phi)/|grad(phi)|, central differences over the axis pull
    // sources (pairs 0, 1, 2 are the x, y, z axes: link 2p+2 sees x + e_p)
    auto seen = [&](int s, int h) -> double {
      return ty[s][h] == LIQ ? 1.0 : (ty[s][h] == GAS ? 0.0 : ph[s][h]);
    };
    double gr[3] = {0.0, 0.0, 0.0};
    {
      const double ga = sub < 3 ? 0.5 * (seen(0, 1) - seen(0, 0)) : 0.0;
      gr[0] = quad_sum(sub == 0 ? ga : 0.0);
      gr[1] = quad_sum(sub == 1 ? ga : 0.0);
      gr[2] = quad_sum(sub == 2 ? ga : 0.0);
    }
    const double nrm2 = (gr[0] * gr[0] + gr[1] * gr[1]) + gr[2] * gr[2];
    const bool have_n = nrm2 > 0.0;
    double nrm = 0.0, nv[3] = {0.0, 0.0, 0.0};
    if (have_n) {
      nrm = sqrt(nrm2);
#pragma unroll
      for (int c = 0; c < 3; ++c) nv[c] = -gr[c] / nrm;
    }
    const double dist = phix - 0.5;
    // moments of time t from the own populations: rho_t = sum ft, u_t = (sum c ft - g) + g/2
    R rho_t, u_t[3];
    {
      R rs = own0, js[3] = {R(0.0), R(0.0), R(0.0)};
#pragma unroll
      for (int s = 0; s < 3; ++s)
        if (s < nsl) {
          rs = rs + (own[s][0] + own[s][1]);
          const R dl = own[s][0] - own[s][1];
#pragma unroll
          for (int c = 0; c < 3; ++c) js[c] = js[c] + dR[s][c] * dl;
        }
      rho_t = quad_sum(rs);
#pragma unroll
      for (int c = 0; c < 3; ++c) u_t[c] = (quad_sum(js[c]) - k.g[c]) + k.hg[c];
    }
    const R usq_t = usq_of(u_t);
    const double phi_new = m_new / rho;

    // ---- adjoint
    // phi(t+1) = m(t+1) / rho: dL/dm(t+1) and the density term of the collision
    const double mb = lam_m + lam_p / rho;
    const double rho_b_phi = -lam_p * phi_new / rho;
    // collision, Eq. (lbe2): out_q = f_q + lambda_+ n+ + lambda_- n-, with
    // n+- = (f_q +- f_qbar)/2 - e+-_q and u = U + g/2, u_eq = U - g/lambda_-
    R fb[3][2], hp[3], hm[3], gb[3];
    R fb0;
    {
      R rb = rest ? R(WD[0]) * (-(k.lp * ob0)) : R(0.0);
      R s9[3] = {R(0.0), R(0.0), R(0.0)}, ue[3] = {R(0.0), R(0.0), R(0.0)};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        hp[s] = hm[s] = R(0.0);
        if (s < nsl) {
          const R w = pp[s] < 3 ? R(WD[1]) : R(WD[7]);
          const R w3 = pp[s] < 3 ? R(W3D[1]) : R(W3D[7]);
          const R np_b = k.lp * (ob[s][0] + ob[s][1]);
          const R nm_b = k.lm * (ob[s][0] - ob[s][1]);
          const R we = w * (-np_b);
          rb = rb + we;
          const R t9 = we * ddot(dR[s], u);
          const R te = w3 * (-nm_b);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            s9[c] = s9[c] + dR[s][c] * t9;
            ue[c] = ue[c] + dR[s][c] * te;
          }
          hp[s] = R(0.5) * np_b;
          hm[s] = R(0.5) * nm_b;
        }
      }
      rb = quad_sum(rb);
      R jb[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s9[c] = quad_sum(s9[c]);
        ue[c] = quad_sum(ue[c]);
        const R ub = R(9.0) * s9[c] - R(3.0) * (u[c] * rb);  // dL/du
        jb[c] = ub + ue[c];                                   // u and u_eq both move with U = j
        gb[c] = R(0.5) * ub - ue[c] * k.ilm;                  // u = U + g/2, u_eq = U - g/lambda_-
      }
      const R rt = rb + (R)rho_b_phi;
      fb0 = (R(1.0) + k.lp) * ob0 + rt;
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const R cj = ddot(dR[s], jb);
        fb[s][0] = ((ob[s][0] + hp[s]) + hm[s]) + (rt + cj);
        fb[s][1] = ((ob[s][1] + hp[s]) - hm[s]) + (rt - cj);
      }
    }
    // reconstruction of the gas-side populations (see rebuild): the adjoint r
    // of a rebuilt f_q is spread over the own populations, the pulled f_o,
    // n+_o (and through it rho_t, u_t), e+_o(rho_b, u_t) and, for the FSL rule,
    // the link distance delta = clamp((phi - 1/2)/(c_o.n), 0, 1)
    R ownb[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s) ownb[s][0] = ownb[s][1] = R(0.0);
    R ownb0 = R(0.0);
    double nvb[3] = {0.0, 0.0, 0.0}, distb = 0.0;
    R rtb = R(0.0), utb[3] = {R(0.0), R(0.0), R(0.0)}, rbb = R(0.0);
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!(s < nsl && ty[s][h] == GAS)) continue;
        const int o = 1 - h;                    // the opposite link o = qbar, in the same pair
        const R sgo = h == 0 ? R(-1.0) : R(1.0);  // c_o = sgo * (direction of the pair's odd link)
        R cob[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) cob[c] = sgo * dR[s][c];
        const R w = pp[s] < 3 ? R(WD[1]) : R(WD[7]);
        const R r = fb[s][h];
        fb[s][h] = R(0.0);  // reconstructed, not pulled: nothing to push
        R ebb = R(0.0);     // dL/de+_o(rho_b, u_t)
        bool fsl = false;
        if (RULE == 1 && have_n && ty[s][o] != GAS) {
          const double nc = h == 0 ? -ddot(dI[s], nv) : ddot(dI[s], nv);
          if (nc > 0.0) {
            fsl = true;
            const double raw = dist / nc;
            double dl = raw;
            if (dl < 0.0) dl = 0.0;
            if (dl > 1.0) dl = 1.0;
            const bool inside = !(raw < 0.0) && !(raw > 1.0);
            const R delta = (R)dl;
            const R own_o = own[s][o], own_q = own[s][h];
            const R cu = ddot(cob, u_t);
            const R e_o_t = w * (rho_t + (R(4.5) * (cu * cu) - R(1.5) * usq_t));
            const R n_plus = (R(0.5) * (own_o + own_q) - e_o_t) * k.inv1p;
            const R a0 = R(1.0) - (R(0.5) + delta);
            const R a1 = delta - R(1.0);
            const R Cc = k.lp * (R(0.5) + delta) - R(2.0) * k.lp;
            // f_q = a0 ft_o + ft_q / 2 + a1 f_o + C n+_o + e+_o(rho_b, u_t)
            ownb[s][o] = ownb[s][o] + a0 * r;
            ownb[s][h] = ownb[s][h] + R(0.5) * r;
            fb[s][o] = fb[s][o] + a1 * r;
            ebb = r;
            const R npb = Cc * r;
            // da0/ddelta = -1, da1/ddelta = 1, dC/ddelta = lambda_+
            const R deltab = r * ((f[s][o] - own_o) + k.lp * n_plus);
            // n+_o = ((ft_o + ft_q)/2 - e+_o(rho_t, u_t)) / (1 + lambda_+)
            const R hb = R(0.5) * (k.inv1p * npb);
            ownb[s][o] = ownb[s][o] + hb;
            ownb[s][h] = ownb[s][h] + hb;
            {  // adjoint of e+_o(rho_t, u_t) for dL/de = -npb/(1 + lambda_+)
              const R we = w * (-(k.inv1p * npb));
              rtb = rtb + we;
              const R t = R(9.0) * (we * cu);
#pragma unroll
              for (int c = 0; c < 3; ++c) utb[c] = (utb[c] + cob[c] * t) - R(3.0) * (we * u_t[c]);
            }
            if (inside) {
              distb += (double)deltab / nc;
              const double ncb = -(double)deltab * raw / nc;
              const double so = h == 0 ? -1.0 : 1.0;
#pragma unroll
              for (int c = 0; c < 3; ++c) nvb[c] += (so * (double)dI[s][c]) * ncb;
            }
          }
        }
        if (!fsl) {  // FSK: f_q = -ft_o + 2 e+_o(rho_b, u_t)
          ownb[s][o] = ownb[s][o] - r;
          ebb = R(2.0) * r;
        }
        {  // adjoint of e+_o(rho_b, u_t): dL/drho_b and dL/du_t (u_b = u_t)
          const R we = w * ebb;
          rbb = rbb + we;
          const R t = R(9.0) * (we * ddot(cob, u_t));
#pragma unroll
          for (int c = 0; c < 3; ++c) utb[c] = (utb[c] + cob[c] * t) - R(3.0) * (we * u_t[c]);
        }
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      nvb[c] = quad_sum(nvb[c]);
      utb[c] = quad_sum(utb[c]);
    }
    distb = quad_sum(distb);
    rtb = quad_sum(rtb);
    rbb = quad_sum(rbb);
    // normal: dL/dgrad = (-nb + n (nb.n)) / |grad|, grad_p = (phi(x+e_p) - phi(x-e_p))/2
    double geo[2] = {0.0, 0.0};  // fill adjoint of the axis pull sources of pair 0 of this lane
    double phis = lead ? distb : 0.0;  // fill adjoint of the cell itself (dist = phi - 1/2)
    if (RULE == 1 && have_n && sub < 3) {
      const double nd = (nvb[0] * nv[0] + nvb[1] * nv[1]) + nvb[2] * nv[2];
      const double nvb_a = sub == 0 ? nvb[0] : (sub == 1 ? nvb[1] : nvb[2]);  // axis of this lane's pair 0
      const double nv_a = sub == 0 ? nv[0] : (sub == 1 ? nv[1] : nv[2]);
      const double gbp = (-nvb_a + nv_a * nd) / nrm;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double v = h == 1 ? 0.5 * gbp : -0.5 * gbp;
        if (ty[0][h] == IFACE) geo[h] += v;
        else if (ty[0][h] == WALL_CLASS) phis += v;  // beyond a wall the cell's own fill is used
      }
    }
    // rho_t = sum_q ft_q, u_t = (sum_q c_q ft_q - g) + g/2
    ownb0 = ownb0 + rtb;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const R cu = ddot(dR[s], utb);
      ownb[s][0] = ownb[s][0] + (rtb + cu);
      ownb[s][1] = ownb[s][1] + (rtb - cu);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) gb[c] = gb[c] - R(0.5) * utb[c];
    // mass exchange: m(t+1) = m + sum_q w_q (f_q(pulled) - ft_qbar)
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!(s < nsl)) continue;
        const unsigned L = 2u * (unsigned)pp[s] + 1u + (unsigned)h;
        const int t = ty[s][h];
        double pc = s == 0 ? geo[h] : 0.0;
        if (t == LIQ || t == IFACE) {
          const double w = t == LIQ ? 1.0 : 0.5 * (phix + ph[s][h]);
          const R wm = (R)(w * mb);
          fb[s][h] = fb[s][h] + wm;
          ownb[s][1 - h] = ownb[s][1 - h] - wm;
          if (t == IFACE) {
            const double half = 0.5 * ((double)f[s][h] - (double)own[s][1 - h]) * mb;
            phis += half;
            pc += half;
          }
        }
        a.phic[L * cap + ui] = pc;
      }
    phis = quad_sum(phis);

    // ---- stores: push of the pulled populations' adjoints (to the element each
    // pull read), own-population terms, the cell's scalars
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!(s < nsl)) continue;
        const unsigned L = 2u * (unsigned)pp[s] + 1u + (unsigned)h;
        own_t[L * cap + ui] = ownb[s][h];
        if (ty[s][h] == GAS) continue;
        // pull source x - c_L (c_L = +-d for the odd / even link of the pair)
        const int sg = h == 0 ? -1 : 1;
        const int sx = step_axis(x, sg * dI[s][0], g.nx, g.px);
        const int sy = step_axis(y, sg * dI[s][1], g.ny, g.py);
        const int sz = step_axis(z, sg * dI[s][2], g.nz, g.pz);
        const unsigned Lo = (L & 1u) ? L + 1u : L - 1u;  // beyond a wall: the cell's own opposite population
        const unsigned off = ((sx | sy | sz) < 0) ? Lo * N + (unsigned)idx
                                                  : L * N + (unsigned)(sx + g.nx * (sy + g.ny * sz));
        lout[off] = fb[s][h];
      }
    if (rest) {
      lout[idx] = fb0;
      own_t[ui] = ownb0;
    }
    if (lead) {
      a.phic[ui] = phis;
      a.lam_m[idx] = mb;
      acc[0] += (double)rbb;
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[1 + c] += (double)gb[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = wave_sum(acc[c]);
  if (threadIdx.x == 0) {
    double* slot = a.part_iface + 4 * (size_t)blockIdx.x;
#pragma unroll
    for (int c = 0; c < 4; ++c) slot_add(slot + c, acc[c]);
  }
}

// Own-population terms and the fill adjoint of each interface cell y.  The
// element ft_q(y) is read by the pull of the cell y + c_q, the pull source of
// link qbar of y (beyond a wall: by y itself).  If that cell is gas nothing was
// pushed there this step.  Classes and list positions come from the fixed
// topology, so the loads are two independent batches.
template <class F>
__global__ __launch_bounds__(AIBLOCK) void k_adj_iface2(AdjArgs a) {
  using R = typename F::R;
  const unsigned N = (unsigned)a.c.grid.N;
  const unsigned cap = (unsigned)a.cap;
  R* __restrict__ lout = reinterpret_cast<R*>(a.lam_out);
  const R* __restrict__ own_t = reinterpret_cast<const R*>(a.own);
  for (int i = blockIdx.x * AIBLOCK + threadIdx.x; i < a.n_i; i += gridDim.x * AIBLOCK) {
    const unsigned yc = (unsigned)a.listI[i];
    const unsigned ui = (unsigned)i;
    const uint64_t cls = a.ncls[i];
    R v[Q], cur[Q];
    double pc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      v[q] = own_t[(unsigned)q * cap + ui];
      cur[q] = lout[(unsigned)q * N + yc];
    }
    pc[0] = a.phic[ui];
#define FSLBM_A2PC(q) pc[q] = a.phic[(unsigned)q * cap + (unsigned)a.nslot[(unsigned)OPP[q] * cap + ui]];
    FSLBM_LINKS(FSLBM_A2PC)
#undef FSLBM_A2PC
    lout[yc] = cur[0] + v[0];
    double pb = pc[0];
#define FSLBM_A2ST(q)                                                           \
  {                                                                             \
    const unsigned c2 = (unsigned)(cls >> (2 * OPP[q])) & 3u; /* class of y + c_q */ \
    lout[(unsigned)q * N + yc] = c2 == 0 ? v[q] : cur[q] + v[q];                \
    if (c2 == 1) pb += pc[q];                                                   \
  }
    FSLBM_LINKS(FSLBM_A2ST)
#undef FSLBM_A2ST
    a.lphi_out[yc] = pb;
  }
}

// Fixed topology of the interface cells (list order): the class of the pull
// source of every link (2 bits each: 0 gas, 1 interface, 2 liquid, 3 beyond a
// wall) and, for interface sources, their list position (else the cell's own).
__global__ __launch_bounds__(ABLOCK) void k_adj_topo(const uint8_t* flags, Grid g, const int32_t* list,
                                                     const int32_t* islot, int n_i, int cap, uint64_t* ncls,
                                                     int32_t* nslot) {
  const int i = blockIdx.x * ABLOCK + threadIdx.x;
  if (i >= n_i) return;
  const int idx = list[i];
  Nbr n;
  coords(g, idx, n.x, n.y, n.z);
  n.xm = step_axis(n.x, -1, g.nx, g.px);
  n.xp = step_axis(n.x, 1, g.nx, g.px);
  n.ym = step_axis(n.y, -1, g.ny, g.py);
  n.yp = step_axis(n.y, 1, g.ny, g.py);
  n.zm = step_axis(n.z, -1, g.nz, g.pz);
  n.zp = step_axis(n.z, 1, g.nz, g.pz);
  uint64_t cls = 1;  // link 0: the cell itself
  nslot[i] = i;
#define FSLBM_TOPO(q)                                                                       \
  {                                                                                         \
    const int s = pull_source<q>(g, n);                                                     \
    const uint8_t t = s >= 0 ? flags[s] : (uint8_t)0xff;                                    \
    const uint64_t c2 = s < 0 ? 3u : (t == GAS ? 0u : (t == IFACE ? 1u : 2u));              \
    cls |= c2 << (2 * q);                                                                   \
    nslot[(size_t)q * cap + i] = (s >= 0 && t == IFACE) ? islot[s] : i;                     \
  }
  FSLBM_LINKS(FSLBM_TOPO)
#undef FSLBM_TOPO
  ncls[i] = cls;
}

// ------------------------------------------------------- seed / output
template <class R>
__global__ __launch_bounds__(ABLOCK) void k_adj_seed(Grid g, const uint8_t* flags, const double* dLdf,
                                                     const double* dLdm, const double* dLdphi, R* lam, R* lam2,
                                                     double* lam_m, double* lphi, double* lphi2) {
  const size_t N = (size_t)g.N;
  for (size_t idx = (size_t)blockIdx.x * ABLOCK + threadIdx.x; idx < N; idx += (size_t)gridDim.x * ABLOCK) {
    const uint8_t t = flags[idx];
    const bool act = t != GAS, itf = t == IFACE;
    for (int q = 0; q < Q; ++q) {
      lam[(size_t)q * N + idx] = (act && dLdf) ? (R)dLdf[(size_t)q * N + idx] : R(0.0);
      lam2[(size_t)q * N + idx] = R(0.0);
    }
    lam_m[idx] = (itf && dLdm) ? dLdm[idx] : 0.0;
    lphi[idx] = (itf && dLdphi) ? dLdphi[idx] : 0.0;
    lphi2[idx] = 0.0;
  }
}

template <class R>
__global__ __launch_bounds__(ABLOCK) void k_adj_out(Grid g, const uint8_t* flags, const R* lam, const double* lam_m,
                                                    const double* lphi, double* dLdf, double* dLdm, double* dLdphi) {
  const size_t N = (size_t)g.N;
  for (size_t idx = (size_t)blockIdx.x * ABLOCK + threadIdx.x; idx < N; idx += (size_t)gridDim.x * ABLOCK) {
    const uint8_t t = flags[idx];
    if (dLdf)
      for (int q = 0; q < Q; ++q) dLdf[(size_t)q * N + idx] = t != GAS ? (double)lam[(size_t)q * N + idx] : 0.0;
    if (dLdm) dLdm[idx] = t == IFACE ? lam_m[idx] : 0.0;
    if (dLdphi) dLdphi[idx] = t == IFACE ? lphi[idx] : 0.0;
  }
}

// fixed-order sum of the block partials: out4 = {dL/drho_b, dL/dg}
__global__ __launch_bounds__(ABLOCK) void k_adj_reduce(const double* ps, int nbs, const double* pi, int nbi,
                                                       double* out4) {
  __shared__ double sm[ABLOCK][4];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nbs; b += ABLOCK)
    for (int c = 0; c < 3; ++c) v[1 + c] += ps[3 * (size_t)b + c];
  for (int b = threadIdx.x; b < nbi; b += ABLOCK)
    for (int c = 0; c < 4; ++c) v[c] += pi[4 * (size_t)b + c];
  for (int c = 0; c < 4; ++c) sm[threadIdx.x][c] = v[c];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int c = 0; c < 4; ++c) {
      double s = 0.0;
      for (int t = 0; t < ABLOCK; ++t) s += sm[t][c];
      out4[c] = s;
    }
  }
}

// ------------------------------------------- ascending interface-cell list
// per block of ABLOCK cells: number of interface cells
__global__ __launch_bounds__(ABLOCK) void k_list_count(const uint8_t* flags, int N, int32_t* bcount) {
  const int idx = blockIdx.x * ABLOCK + threadIdx.x;
  const bool it = idx < N && flags[idx] == IFACE;
  const int c = __syncthreads_count(it);
  if (threadIdx.x == 0) bcount[blockIdx.x] = c;
}

// exclusive scan of bcount[0..nb) in place (one block of SCAN threads); total to n_out
constexpr int SCAN = 1024;
__global__ __launch_bounds__(SCAN) void k_list_scan(int32_t* bcount, int nb, int32_t* n_out) {
  __shared__ int32_t sm[SCAN];
  const int per = (nb + SCAN - 1) / SCAN;
  const int b0 = (int)threadIdx.x * per;
  const int b1 = min(nb, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += bcount[b];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < SCAN; o <<= 1) {
    const int v = (int)threadIdx.x >= o ? sm[threadIdx.x - o] : 0;
    __syncthreads();
    sm[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x > 0 ? sm[threadIdx.x - 1] : 0;
  for (int b = b0; b < b1; ++b) {
    const int c = bcount[b];
    bcount[b] = run;
    run += c;
  }
  if (threadIdx.x == SCAN - 1) *n_out = sm[SCAN - 1];
}

__global__ __launch_bounds__(ABLOCK) void k_list_write(const uint8_t* flags, int N, const int32_t* boff,
                                                       int32_t* list, int32_t* islot) {
  __shared__ int32_t wc[ABLOCK / 64];
  const int idx = blockIdx.x * ABLOCK + threadIdx.x;
  const bool it = idx < N && flags[idx] == IFACE;
  const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
  const unsigned long long b = __ballot(it);
  if (lane == 0) wc[w] = __popcll(b);
  __syncthreads();
  int base = boff[blockIdx.x];
  for (int k = 0; k < w; ++k) base += wc[k];
  if (it) {
    const int pos = base + __popcll(b & ((1ull << lane) - 1ull));
    list[pos] = idx;
    islot[idx] = pos;
  }
}

// number of interface cells (atomic add of per-block counts into *out)
__global__ __launch_bounds__(ABLOCK) void k_count_iface(const uint8_t* flags, int N, int32_t* out) {
  const int idx = blockIdx.x * ABLOCK + threadIdx.x;
  const int c = __syncthreads_count(idx < N && flags[idx] == IFACE);
  if (threadIdx.x == 0 && c) atomicAdd(out, c);
}

// ------------------------------------------------------------ launchers
static inline unsigned ablocks(size_t n) { return (unsigned)((n + ABLOCK - 1) / ABLOCK); }

unsigned adj_sweep_blocks(const Grid& g) {
  return (unsigned)((g.nx + ABLOCK - 1) / ABLOCK) * (unsigned)g.ny * (unsigned)g.nz;
}
unsigned adj_sweep_slots(const Grid& g) { return adj_sweep_blocks(g) * (ABLOCK / 64); }
unsigned adj_iface_blocks(int n_i) {  // blocks of the quad kernel (their partial sums are reduced)
  return std::max(1u, std::min(ADJ_IFACE_GRID, (unsigned)(((size_t)n_i + CELLS_PER_BLOCK - 1) / CELLS_PER_BLOCK)));
}
static unsigned adj_iface2_blocks(int n_i) {
  return std::max(1u, std::min(ADJ_IFACE_GRID, (unsigned)(((size_t)n_i + AIBLOCK - 1) / AIBLOCK)));
}
unsigned list_blocks(const Grid& g) { return ablocks((size_t)g.N); }

hipError_t launch_iface_list(const uint8_t* flags, const Grid& g, int32_t* bcount, int32_t* list, int32_t* islot,
                             int32_t* n_out, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const unsigned nb = list_blocks(g);
  k_list_count<<<nb, ABLOCK, 0, st>>>(flags, g.N, bcount);
  k_list_scan<<<1, SCAN, 0, st>>>(bcount, (int)nb, n_out);
  k_list_write<<<nb, ABLOCK, 0, st>>>(flags, g.N, bcount, list, islot);
  return hipGetLastError();
}

hipError_t launch_adj_topo(const uint8_t* flags, const Grid& g, const int32_t* list, const int32_t* islot, int n_i,
                           int cap, uint64_t* ncls, int32_t* nslot, void* stream) {
  if (n_i <= 0) return hipSuccess;
  k_adj_topo<<<ablocks((size_t)n_i), ABLOCK, 0, (hipStream_t)stream>>>(flags, g, list, islot, n_i, cap, ncls, nslot);
  return hipGetLastError();
}

hipError_t launch_count_iface(const uint8_t* flags, const Grid& g, int32_t* out, void* stream) {
  k_count_iface<<<list_blocks(g), ABLOCK, 0, (hipStream_t)stream>>>(flags, g.N, out);
  return hipGetLastError();
}

hipError_t launch_adj_seed(const Common& c, const uint8_t* flags, int precision, const double* dLdf,
                           const double* dLdm, const double* dLdphi, void* lam, void* lam_other, double* lam_m,
                           double* lphi, double* lphi_other, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const unsigned nb = std::min(8192u, ablocks((size_t)c.grid.N));
  if (precision == 0)
    k_adj_seed<double><<<nb, ABLOCK, 0, st>>>(c.grid, flags, dLdf, dLdm, dLdphi, (double*)lam, (double*)lam_other,
                                              lam_m, lphi, lphi_other);
  else
    k_adj_seed<float><<<nb, ABLOCK, 0, st>>>(c.grid, flags, dLdf, dLdm, dLdphi, (float*)lam, (float*)lam_other,
                                             lam_m, lphi, lphi_other);
  return hipGetLastError();
}

template <class F>
static void adj_sweep_form(const AdjArgs& a0, hipStream_t st) {
  AdjArgs a = a0;
  a.cpr = (a.c.grid.nx + ABLOCK - 1) / ABLOCK;
  if ((double)Q * (double)a.c.grid.N * (double)sizeof(typename F::R) < 4294967296.0)
    k_adj_sweep<F, true><<<adj_sweep_blocks(a.c.grid), ABLOCK, 0, st>>>(a);
  else
    k_adj_sweep<F, false><<<adj_sweep_blocks(a.c.grid), ABLOCK, 0, st>>>(a);
}

template <class F>
static void adj_iface_form(const AdjArgs& a, int rule, hipStream_t st) {
  if (a.n_i <= 0) return;
  const unsigned nbi = adj_iface_blocks(a.n_i);
  if (rule == 0)
    k_adj_iface<F, 0><<<nbi, AIBLOCK, 0, st>>>(a);
  else
    k_adj_iface<F, 1><<<nbi, AIBLOCK, 0, st>>>(a);
}

template <class F>
static void adj_iface2_form(const AdjArgs& a, hipStream_t st) {
  if (a.n_i <= 0) return;
  k_adj_iface2<F><<<adj_iface2_blocks(a.n_i), AIBLOCK, 0, st>>>(a);
}

hipError_t launch_adj_sweep(const AdjArgs& a, int precision, void* stream) {
  if (precision == 0) adj_sweep_form<FormF64>(a, (hipStream_t)stream);
  else adj_sweep_form<FormF32>(a, (hipStream_t)stream);
  return hipGetLastError();
}

hipError_t launch_adj_iface(const AdjArgs& a, int precision, int rule, void* stream) {
  if (precision == 0) adj_iface_form<FormF64>(a, rule, (hipStream_t)stream);
  else adj_iface_form<FormF32>(a, rule, (hipStream_t)stream);
  return hipGetLastError();
}

hipError_t launch_adj_iface2(const AdjArgs& a, int precision, void* stream) {
  if (precision == 0) adj_iface2_form<FormF64>(a, (hipStream_t)stream);
  else adj_iface2_form<FormF32>(a, (hipStream_t)stream);
  return hipGetLastError();
}

hipError_t launch_adj_out(const Common& c, const uint8_t* flags, int precision, const void* lam,
                          const double* lam_m, const double* lphi, double* dLdf, double* dLdm, double* dLdphi,
                          void* stream) {
  hipStream_t st = (hipStream_t)stream;
  const unsigned nb = std::min(8192u, ablocks((size_t)c.grid.N));
  if (precision == 0)
    k_adj_out<double><<<nb, ABLOCK, 0, st>>>(c.grid, flags, (const double*)lam, lam_m, lphi, dLdf, dLdm, dLdphi);
  else
    k_adj_out<float><<<nb, ABLOCK, 0, st>>>(c.grid, flags, (const float*)lam, lam_m, lphi, dLdf, dLdm, dLdphi);
  return hipGetLastError();
}

hipError_t launch_adj_reduce(const double* part_sweep, int nb_sweep, const double* part_iface, int nb_iface,
                             double* out4, void* stream) {
  k_adj_reduce<<<1, ABLOCK, 0, (hipStream_t)stream>>>(part_sweep, nb_sweep, part_iface, nb_iface, out4);
  return hipGetLastError();
}

}  // namespace fslbm
