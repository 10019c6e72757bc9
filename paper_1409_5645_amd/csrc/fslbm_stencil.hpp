// Stencil helpers shared by the step and adjoint kernels: pull sources, the
// neighbourhood of an interface cell, the link macro.
#pragma once

#include "fslbm_device.hpp"
#include "fslbm_internal.hpp"

namespace fslbm {

#define FSLBM_LINKS(M) M(1) M(2) M(3) M(4) M(5) M(6) M(7) M(8) M(9) M(10) M(11) M(12) M(13) M(14) M(15) M(16) M(17) M(18)

// row offset marking a pull source row beyond a wall
constexpr unsigned WALL_ROW = 0xffffffffu;

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

constexpr uint8_t WALL_CLASS = 3;  // class recorded for a pull source beyond a wall (= SOLID)

// Neighbourhood of one interface cell, loaded in a single pass (all loads
// independent, so the cell costs one memory round trip, not a chain of them).
template <class F>
struct IfaceData {
  using R = typename F::R;
  R f[Q];         // pulled populations f_q(x, t+1) (gas links: placeholder)
  R own[Q];       // own post-collision populations of time t
  uint8_t ty[Q];  // class of the pull source x - c_q (WALL_CLASS beyond a wall)
  double ph[Q];   // fill of the pull source (own fill beyond a wall)
  double m, phix;
};

// As wave_append below, returning the list position of the lane's value (-1
// where pred is false).
__device__ __forceinline__ int wave_append_at(bool pred, int32_t* counter, int32_t* list, int32_t value) {
  const unsigned long long b = __ballot(pred);
  if (b == 0ull) return -1;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)b) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(b));
  base = __shfl(base, leader);
  const int pos = base + __popcll(b & ((1ull << lane) - 1ull));
  if (pred) list[pos] = value;
  return pred ? pos : -1;
}

// Append value to list for every active lane with pred set, with one atomic
// per wavefront: the lowest such lane reserves the slots, each lane writes at
// its rank among them (lanes that have left the branch take no part).
__device__ __forceinline__ void wave_append(bool pred, int32_t* counter, int32_t* list, int32_t value) {
  const unsigned long long b = __ballot(pred);
  if (b == 0ull) return;
  const int lane = (int)__lane_id();
  const int leader = __ffsll((long long)b) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(counter, __popcll(b));
  base = __shfl(base, leader);
  if (pred) list[base + __popcll(b & ((1ull << lane) - 1ull))] = value;
}

template <class F>
__device__ __forceinline__ double phi_seen(const IfaceData<F>& d, int q) {
  // fill level seen from the cell: liquid 1, gas 0, interface its fill,
  // beyond a wall the cell's own fill
  return d.ty[q] == LIQ ? 1.0 : (d.ty[q] == GAS ? 0.0 : d.ph[q]);
}

// Halfway bounce-back off a moving wall: the population pulled along q from
// beyond a wall face gains 2 w_q (c_q . u_w) / c_s^2 (rho_w = 1), read from the
// table wt[face * 19 + q].  The face is the first one the pull source x - c_q
// crosses, in axis order x, y, z (faces x-, x+, y-, y+, z-, z+); the arguments
// are the neighbour coordinates (-1 beyond a wall).  Every candidate face is
// known at compile time from c_q.  0 if the link is not a wall link.
template <int q>
__device__ __forceinline__ double wall_term(const double* __restrict__ wt, int xm, int xp, int ym, int yp, int zm,
                                            int zp) {
  if (CX[q] == 1 && xm < 0) return wt[0 * Q + q];
  if (CX[q] == -1 && xp < 0) return wt[1 * Q + q];
  if (CY[q] == 1 && ym < 0) return wt[2 * Q + q];
  if (CY[q] == -1 && yp < 0) return wt[3 * Q + q];
  if (CZ[q] == 1 && zm < 0) return wt[4 * Q + q];
  if (CZ[q] == -1 && zp < 0) return wt[5 * Q + q];
  return 0.0;
}

// Curvature kappa = -div n = (|g|^2 tr H - g.H.g) / |g|^3 of the fill field seen
// from an interface cell (Eq. freeboundary: the gas pressure becomes P_b -
// sigma kappa; a sphere of radius R has kappa = -2/R), with the gradient g and
// Hessian H by central differences over the D3Q19 neighbourhood.  The pull
// source of link q sits at offset -c_q.  Zero if g = 0.  FP64.
template <class F>
__device__ __forceinline__ double curvature(const IfaceData<F>& d) {
  double v[3][3][3];
  v[1][1][1] = d.phix;
#define FSLBM_KV(q) v[1 - CX[q]][1 - CY[q]][1 - CZ[q]] = phi_seen(d, q);
  FSLBM_LINKS(FSLBM_KV)
#undef FSLBM_KV
  const double c = v[1][1][1];
  double g[3], H[3][3];
  g[0] = 0.5 * (v[2][1][1] - v[0][1][1]);
  g[1] = 0.5 * (v[1][2][1] - v[1][0][1]);
  g[2] = 0.5 * (v[1][1][2] - v[1][1][0]);
  H[0][0] = (v[2][1][1] - 2.0 * c) + v[0][1][1];
  H[1][1] = (v[1][2][1] - 2.0 * c) + v[1][0][1];
  H[2][2] = (v[1][1][2] - 2.0 * c) + v[1][1][0];
  H[0][1] = H[1][0] = 0.25 * (((v[2][2][1] - v[2][0][1]) - v[0][2][1]) + v[0][0][1]);
  H[0][2] = H[2][0] = 0.25 * (((v[2][1][2] - v[2][1][0]) - v[0][1][2]) + v[0][1][0]);
  H[1][2] = H[2][1] = 0.25 * (((v[1][2][2] - v[1][2][0]) - v[1][0][2]) + v[1][0][0]);
  const double g2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
  if (!(g2 > 0.0)) return 0.0;
  const double trH = (H[0][0] + H[1][1]) + H[2][2];
  double gHg = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) gHg = gHg + g[a] * ((H[a][0] * g[0] + H[a][1] * g[1]) + H[a][2] * g[2]);
  const double gn = sqrt(g2);
  return (g2 * trH - gHg) / (g2 * gn);
}

// Slot of a cell in the ascending wall list (binary search), -1 if absent.
__device__ __forceinline__ int wall_slot(const int32_t* __restrict__ cells, int n, int idx) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (cells[mid] < idx) lo = mid + 1;
    else hi = mid;
  }
  return (lo < n && cells[lo] == idx) ? lo : -1;
}

// Solid walls of the rotated channels (section 4.2).  Link q whose pull source
// x - c_q is a solid cell (bit q of `solid`): with p = qbar the link towards
// the wall point x + delta c_p, the closure f_q(x,t+1) = a0 ft_p(x) +
// a0bar ft_q(x) + a1 ft_p(x - c_p) + f^b of Eq. (closure) with the fitting
// conditions alpha_+ = 0 and beta_+ / lambda_+ = alpha_- delta (Eq. fitting,
// cl1; momentum of the wall matched to first order, no pressure term), C = 0
// and a0 = 1: kappa = (1 - 2 delta)/(1 + 2 delta), a1 = kappa, a0bar = -kappa,
// f^b = -4/(1 + 2 delta) e-_p(u_w), i.e. 2/(1 + 2 delta) times the halfway
// bounce-back term 2 w_q (c_q . u_w)/c_s^2 (rho_w = 1).  ft_p(x - c_p) is the
// value pulled along p; where its source is not a fluid cell (bit p of `up`
// clear) the link takes halfway bounce-back.  f[p] of a fluid source is never
// modified here, so the links can be done in any order.
template <class R>
__device__ __forceinline__ void solid_links(R (&f)[Q], const R (&own)[Q], uint32_t solid, uint32_t up, int slot,
                                            int nw, const double* __restrict__ delta,
                                            const double* __restrict__ uw) {
#define FSLBM_SOLID(q)                                                                                  \
  if ((solid >> q) & 1u) {                                                                              \
    constexpr int p = OPP[q];                                                                           \
    const double dl = delta[(size_t)p * nw + slot];                                                     \
    const double u0 = uw[(size_t)p * nw + slot];                                                        \
    const double u1 = uw[((size_t)Q + p) * nw + slot];                                                  \
    const double u2 = uw[((size_t)2 * Q + p) * nw + slot];                                              \
    const double bb = 6.0 * WD[q] * ((CX[q] * u0 + CY[q] * u1) + CZ[q] * u2);                            \
    if ((up >> p) & 1u) {                                                                               \
      const double kap = (1.0 - 2.0 * dl) / (1.0 + 2.0 * dl);                                           \
      f[q] = (own[p] + (R)kap * (f[p] - own[q])) + (R)(bb * (2.0 / (1.0 + 2.0 * dl)));                  \
    } else {                                                                                            \
      f[q] = own[p] + (R)bb;                                                                            \
    }                                                                                                   \
  }
  FSLBM_LINKS(FSLBM_SOLID)
#undef FSLBM_SOLID
}

// Second-order interface position (section 5): the offset d of the plane
// n.(x - x_node) = d that leaves the fill fraction phi of the unit cell on the
// liquid side, for a unit normal n.  The cut volume is the forward relation of
// Scardovelli & Zaleski (J. Comput. Phys. 164, 2000): components sorted
// s1 <= s2 <= s3 and scaled to sum 1, offset reflected into [0, 1/2], the
// quotients over s1 in closed form so near-axis normals lose nothing to
// cancellation.  The offset is found by bisection on [0, 1/2] (54 halvings
// reach the spacing of doubles there).
__device__ __forceinline__ double plic_lower_volume(double al, double s1, double s2, double s3) {
  if (al <= s1) return (al * al * al) / (6.0 * s1 * s2 * s3);
  const double w = 1.0 / (6.0 * s2 * s3);
  const double base = 3.0 * al * (al - s1) + s1 * s1;
  if (al <= s2) return base * w;
  const double r2 = al - s2;
  const double s12 = s1 + s2;
  if (al <= s3) {
    if (al <= s12) return (base - r2 * r2 * r2 / s1) * w;
    return (al - 0.5 * s12) / s3;
  }
  const double r3 = al - s3;
  return (base - (r2 * r2 * r2 + r3 * r3 * r3) / s1) * w;
}

// Height-function columns of an interface cell (the second-order
// reconstruction of section 5).  Along the axis a of the largest component of
// the central-difference normal nv (lowest axis on ties), the fills of the
// 3 x 3 columns of 7 cells around the cell are summed (liquid 1, gas 0,
// interface its fill).  With every column complete (fill >= 1 at the liquid
// end, <= 0 at the gas end, no wall face or solid cell in it) the sums h are
// the surface heights; sg is the side of the gas along a.  False otherwise.
__device__ __forceinline__ bool hf_heights(const Grid& g, int x, int y, int z, const uint8_t* __restrict__ flags,
                                           const double* __restrict__ phi, const double (&nv)[3],
                                           double (&h)[3][3], int& a, int& sg) {
  a = 0;
  if (fabs(nv[1]) > fabs(nv[a])) a = 1;
  if (fabs(nv[2]) > fabs(nv[a])) a = 2;
  sg = nv[a] > 0.0 ? 1 : -1;
  const int e1 = a == 2 ? 0 : a + 1, e2 = a == 0 ? 2 : (a == 1 ? 0 : 1);
  const int n3[3] = {g.nx, g.ny, g.nz};
  const int p3[3] = {g.px, g.py, g.pz};
  const int c0[3] = {x, y, z};
  for (int i = -1; i <= 1; ++i)
    for (int j = -1; j <= 1; ++j) {
      double sum = 0.0;
      for (int k = -3; k <= 3; ++k) {
        int d[3];
        d[a] = k;
        d[e1] = i;
        d[e2] = j;
        int cc[3];
        for (int b = 0; b < 3; ++b) {
          int v = c0[b] + d[b];
          if (v < 0 || v >= n3[b]) {
            if (!p3[b]) return false;
            v = ((v % n3[b]) + n3[b]) % n3[b];
          }
          cc[b] = v;
        }
        const int s = cc[0] + g.nx * (cc[1] + g.ny * cc[2]);
        const uint8_t t = flags[s];
        if (t == SOLID) return false;
        const double v = t == LIQ ? 1.0 : (t == GAS ? 0.0 : phi[s]);
        if (k == -3 * sg && !(v >= 1.0)) return false;
        if (k == 3 * sg && !(v <= 0.0)) return false;
        sum = sum + v;
      }
      h[i + 1][j + 1] = sum;
    }
  return true;
}

// Height-function normal: with central differences H_1, H_2 of the column
// heights across the axis a, nv becomes (s e_a - H_1 e_1 - H_2 e_2)/|.|, s the
// side of the gas.  Exact for a plane whose slope against a is at most 1.
// Leaves nv as it is where a column is not complete.
__device__ __forceinline__ void hf_normal(const Grid& g, int x, int y, int z, const uint8_t* __restrict__ flags,
                                       const double* __restrict__ phi, double (&nv)[3]) {
  double h[3][3];
  int a, sg;
  if (!hf_heights(g, x, y, z, flags, phi, nv, h, a, sg)) return;
  const int e1 = a == 2 ? 0 : a + 1, e2 = a == 0 ? 2 : (a == 1 ? 0 : 1);
  const double h1 = 0.5 * (h[2][1] - h[0][1]);
  const double h2 = 0.5 * (h[1][2] - h[1][0]);
  double v[3];
  v[a] = (double)sg;
  v[e1] = -h1;
  v[e2] = -h2;
  const double nrm = sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]);
  nv[0] = v[0] / nrm;
  nv[1] = v[1] / nrm;
  nv[2] = v[2] / nrm;
}

// Height-function curvature for the Laplace pressure of Eq. (freeboundary):
// kappa = -div n = [H_11 (1 + H_2^2) + H_22 (1 + H_1^2) - 2 H_12 H_1 H_2] /
// (1 + H_1^2 + H_2^2)^(3/2) with central differences of the column heights (a
// sphere of radius R: -2/R).  Leaves kappa as it is where a column is not
// complete.
__device__ __forceinline__ void hf_curvature(const Grid& g, int x, int y, int z, const uint8_t* __restrict__ flags,
                                          const double* __restrict__ phi, const double (&nv)[3], double& kappa) {
  double h[3][3];
  int a, sg;
  if (!hf_heights(g, x, y, z, flags, phi, nv, h, a, sg)) return;
  const double h1 = 0.5 * (h[2][1] - h[0][1]);
  const double h2 = 0.5 * (h[1][2] - h[1][0]);
  const double h11 = (h[2][1] - 2.0 * h[1][1]) + h[0][1];
  const double h22 = (h[1][2] - 2.0 * h[1][1]) + h[1][0];
  const double h12 = 0.25 * (((h[2][2] - h[2][0]) - h[0][2]) + h[0][0]);
  const double q = (1.0 + h1 * h1) + h2 * h2;
  const double num = (h11 * (1.0 + h2 * h2) + h22 * (1.0 + h1 * h1)) - 2.0 * ((h12 * h1) * h2);
  kappa = num / (q * sqrt(q));
}

__device__ __forceinline__ double plic_plane_offset(double phi, const double (&nv)[3]) {
  const double a = fabs(nv[0]), b = fabs(nv[1]), c = fabs(nv[2]);
  const double sum = a + b + c;
  const double lo3 = fmin(a, fmin(b, c)), hi3 = fmax(a, fmax(b, c));
  const double inv = 1.0 / sum;
  const double s1 = lo3 * inv, s3 = hi3 * inv, s2 = ((sum - lo3) - hi3) * inv;
  const double v = fmin(fmax(phi, 0.0), 1.0);
  const bool upper = v > 0.5;
  const double t = upper ? 1.0 - v : v;
  double lo = 0.0, hi = 0.5;
  for (int it = 0; it < 54; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (plic_lower_volume(mid, s1, s2, s3) < t) lo = mid;
    else hi = mid;
  }
  const double al = 0.5 * (lo + hi);
  return sum * ((upper ? 1.0 - al : al) - 0.5);
}

// c_q . S . c_q for a symmetric S = [xx, yy, zz, xy, xz, yz]
template <int q, class R>
__device__ __forceinline__ R c_S_c(const R (&S)[6]) {
  const R dg = (R(CX[q] * CX[q]) * S[0] + R(CY[q] * CY[q]) * S[1]) + R(CZ[q] * CZ[q]) * S[2];
  const R of = (R(CX[q] * CY[q]) * S[3] + R(CX[q] * CZ[q]) * S[4]) + R(CY[q] * CZ[q]) * S[5];
  return dg + R(2.0) * of;
}

// Reconstruction of the population f_q that would stream in from a gas cell
// (rhob_s: the cell's gas density in storage convention, rho0b its rho_0).
// With o = qbar the link pointing to gas, the closure Eq. (closure) gives
//   f_q = a0 ft_o(x) + a0bar ft_q(x) + a1 f_o(x,t+1) + C n+_o(x,t) + alpha_+ e+_o(rho_b,u_b)
// with the FSK row of Table 1 (Eq. koerner) or Eq. (fsli1)-(fsli4) at alpha_+ = 1
// (RULE bit 0), plus, with RULE bit 1 (S^b from the bulk) or bit 2 (S^b
// prescribed), the shear-rate part of the boundary value Eq. (bterm):
// D c_o c_o : S^b with D = -alpha_+ Lambda_+ w_o / c_s^2 (Table 1).
template <class F, int RULE, int q>
__device__ __forceinline__ void rebuild(IfaceData<F>& d, uint32_t gasmask, bool have_n, const double (&nv)[3],
                                        double dist, typename F::R rho_t, typename F::R rho0_t,
                                        const typename F::R (&u_t)[3], typename F::R usq_t,
                                        const Consts<typename F::R>& k, bool incomp, bool stokes,
                                        const typename F::R (&Sb)[6], bool stress, typename F::R rhob_s,
                                        typename F::R rho0b) {
  using R = typename F::R;
  if (!((gasmask >> q) & 1u)) return;
  constexpr int o = OPP[q];
  const R own_o = d.own[o];
  const R e_b = e_plus<o>(rhob_s, rho0b, incomp, stokes, u_t, usq_t);
  if ((RULE & 1) && have_n && !((gasmask >> o) & 1u)) {
    // link distance delta: plane with normal n at offset phi - 1/2
    double nc = 0.0;
    if (CX[o] == 1) nc = nc + nv[0];
    if (CX[o] == -1) nc = nc - nv[0];
    if (CY[o] == 1) nc = nc + nv[1];
    if (CY[o] == -1) nc = nc - nv[1];
    if (CZ[o] == 1) nc = nc + nv[2];
    if (CZ[o] == -1) nc = nc - nv[2];
    if (nc > 0.0) {
      double dl = dist / nc;
      if (dl < 0.0) dl = 0.0;
      if (dl > 1.0) dl = 1.0;
      const R delta = (R)dl;
      const R own_q = d.own[q];
      // n+_o(x,t) from ft+ = e+ + (1 + lambda_+) n+
      const R e_o_t = e_plus<o>(rho_t, rho0_t, incomp, stokes, u_t, usq_t);
      const R n_plus = (R(0.5) * (own_o + own_q) - e_o_t) * k.inv1p;
      const R a0 = R(1.0) - (R(0.5) + delta);
      const R a1 = delta - R(1.0);
      const R Cc = k.lp * (R(0.5) + delta) - R(2.0) * k.lp;
      d.f[q] = (((a0 * own_o + R(0.5) * own_q) + a1 * d.f[o]) + Cc * n_plus) + e_b;
      if constexpr ((RULE & 6) != 0) {
        if (stress) d.f[q] = d.f[q] + (-((R(1.0) * k.Lp) * R(3.0 * WD[o]))) * c_S_c<o>(Sb);  // alpha_+ = 1
      }
      return;
    }
  }
  d.f[q] = R(2.0) * e_b - own_o;  // FSK: -ft_o + 2 e+_o(rho_b, u_b)
  if constexpr ((RULE & 6) != 0) {
    if (stress) d.f[q] = d.f[q] + (-((R(2.0) * k.Lp) * R(3.0 * WD[o]))) * c_S_c<o>(Sb);  // alpha_+ = 2
  }
}

}  // namespace fslbm
