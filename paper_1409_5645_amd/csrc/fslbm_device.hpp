// Device-side building blocks of the free-surface LBM step on gfx950:
// D3Q19 lattice tables, precision forms, equilibria and the TRT collision.
//
// Floating-point expression order is fixed (ascending-q sums, no FMA
// contraction: the library is compiled with -ffp-contract=off) so that the FP64
// form is reproducible bit for bit on any IEEE machine.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fslbm {

constexpr int Q = 19;

// D3Q19 velocities: rest, axis links, diagonals; odd q has its opposite at q+1.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

// Lattice weights w_q (Qian et al.; c_s^2 = 1/3) and 3 w_q = w_q / c_s^2.
constexpr double WD[Q] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
constexpr double W3D[Q] = {3.0 * (1.0 / 3.0),  3.0 * (1.0 / 18.0), 3.0 * (1.0 / 18.0), 3.0 * (1.0 / 18.0),
                           3.0 * (1.0 / 18.0), 3.0 * (1.0 / 18.0), 3.0 * (1.0 / 18.0), 3.0 * (1.0 / 36.0),
                           3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0),
                           3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0),
                           3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0), 3.0 * (1.0 / 36.0)};

enum : uint8_t { GAS = 0, IFACE = 1, LIQ = 2, SOLID = 3 };  // SOLID: obstacle, never converted

// ---------------------------------------------------------------- forms
// R: compute type; S: storage type.  Shifted forms store g_q = f_q - w_q, so
// that "density" in storage convention is delta rho = rho - 1.
struct FormF64 {
  using R = double;
  using S = double;
  static constexpr bool shifted = false;
  static constexpr bool scaled = false;
  __device__ static R load(const S* p, float) { return *p; }
  __device__ static void store(S* p, R v, float) { *p = v; }
  __device__ static R load_raw(const S* p) { return *p; }
  __device__ static void store_raw(S* p, R v) { *p = v; }
};
struct FormF32 {
  using R = float;
  using S = float;
  static constexpr bool shifted = true;
  static constexpr bool scaled = false;
  __device__ static R load(const S* p, float) { return *p; }
  __device__ static void store(S* p, R v, float) { *p = v; }
  __device__ static R load_raw(const S* p) { return *p; }
  __device__ static void store_raw(S* p, R v) { *p = v; }
};
struct FormF16 {
  using R = float;
  using S = _Float16;
  static constexpr bool shifted = true;
  // stored value = 2^k g in binary16 (round to nearest even); scale factors
  // are exact powers of two
  static constexpr bool scaled = true;
  __device__ static R load(const S* p, float inv_scale) { return (float)(*p) * inv_scale; }
  __device__ static void store(S* p, R v, float scale) { *p = (_Float16)(v * scale); }
  // scaled units: the stored value 2^k g itself (the sweep collides in these units)
  __device__ static R load_raw(const S* p) { return (float)(*p); }
  __device__ static void store_raw(S* p, R v) { *p = (_Float16)v; }
};

// Per-form constants (all derived on the host in double, then rounded once).
template <class R>
struct Consts {
  R lp, lm, inv1p;        // lambda_+, lambda_-, 1/(1+lambda_+)
  R ilm;                  // 1/lambda_-
  R g[3], hg[3], glm[3];  // g, g/2, g/lambda_-
  R rhob_s;               // gas density in storage convention
  R rho0b;                // rho_0 used with the gas density
  R Lp;                   // Lambda_+ = -(1/2 + 1/lambda_+) = tau - 1/2
};

// c_q . v with the non-zero components only, in axis order
template <int q, class R>
__device__ __forceinline__ R cdot(const R v[3]) {
  R s = R(0.0);
  if (CX[q] == 1) s = s + v[0];
  if (CX[q] == -1) s = s - v[0];
  if (CY[q] == 1) s = s + v[1];
  if (CY[q] == -1) s = s - v[1];
  if (CZ[q] == 1) s = s + v[2];
  if (CZ[q] == -1) s = s - v[2];
  return s;
}

template <class R>
__device__ __forceinline__ R usq_of(const R u[3]) {
  return (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
}

// even equilibrium e+_q (Eq. eqEven) in storage convention:
// w_q (rho_s + rho_0 (4.5 (c.u)^2 - 1.5 u.u)); rho_s is rho or rho - 1
template <int q, class R>
__device__ __forceinline__ R e_plus(R rho_s, R rho0, bool incomp, bool stokes, const R u[3], R usq) {
  if (stokes) return R(WD[q]) * rho_s;
  R cu = cdot<q>(u);
  R nl = R(4.5) * (cu * cu) - R(1.5) * usq;
  if (!incomp) nl = rho0 * nl;
  return R(WD[q]) * (rho_s + nl);
}

// odd equilibrium e-_q (Eq. eqOdd): 3 w_q rho_0 c_q.u_eq
template <int q, class R>
__device__ __forceinline__ R e_minus(R rho0, bool incomp, const R ueq[3]) {
  R cu = cdot<q>(ueq);
  if (!incomp) cu = rho0 * cu;
  return R(W3D[q]) * cu;
}

// zeroth moment (storage convention) and first moment, ascending q
template <class R>
__device__ __forceinline__ void moments(const R f[Q], R& rho_s, R j[3]) {
  R r = f[0];
#pragma unroll
  for (int q = 1; q < Q; ++q) r = r + f[q];
  rho_s = r;
  R jx = R(0.0), jy = R(0.0), jz = R(0.0);
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (CX[q] == 1) jx = jx + f[q];
    if (CX[q] == -1) jx = jx - f[q];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (CY[q] == 1) jy = jy + f[q];
    if (CY[q] == -1) jy = jy - f[q];
  }
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    if (CZ[q] == 1) jz = jz + f[q];
    if (CZ[q] == -1) jz = jz - f[q];
  }
  j[0] = jx;
  j[1] = jy;
  j[2] = jz;
}

template <class R, bool SHIFTED>
__device__ __forceinline__ R rho0_of(R rho_s, bool incomp) {
  if (incomp) return R(1.0);
  return SHIFTED ? R(1.0) + rho_s : rho_s;
}

// TRT collision, Eq. (lbe2), force through u_eq = U - g/lambda_- (F = rho_0 g).
// Overwrites f with the post-collision populations; returns rho_s and u.
template <class R, bool SHIFTED>
__device__ __forceinline__ void collide(R f[Q], const Consts<R>& k, bool incomp, bool stokes, R& rho_s,
                                        R u[3]) {
  R j[3];
  moments(f, rho_s, j);
  const R rho0 = rho0_of<R, SHIFTED>(rho_s, incomp);
  R ueq[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R U = incomp ? j[a] : j[a] / rho0;
    u[a] = U + k.hg[a];
    ueq[a] = U - k.glm[a];
  }
  const R usq = usq_of(u);
  {
    R ep = e_plus<0>(rho_s, rho0, incomp, stokes, u, usq);
    f[0] = f[0] + k.lp * (f[0] - ep);
  }
#define FSLBM_PAIR(q)                                            \
  {                                                              \
    R fp = R(0.5) * (f[q] + f[q + 1]);                           \
    R fm = R(0.5) * (f[q] - f[q + 1]);                           \
    R np = fp - e_plus<q>(rho_s, rho0, incomp, stokes, u, usq);  \
    R nm = fm - e_minus<q>(rho0, incomp, ueq);                   \
    R a = f[q], b = f[q + 1];                                    \
    f[q] = (a + k.lp * np) + k.lm * nm;                          \
    f[q + 1] = (b + k.lp * np) - k.lm * nm;                      \
  }
  FSLBM_PAIR(1) FSLBM_PAIR(3) FSLBM_PAIR(5) FSLBM_PAIR(7) FSLBM_PAIR(9) FSLBM_PAIR(11) FSLBM_PAIR(13)
  FSLBM_PAIR(15) FSLBM_PAIR(17)
#undef FSLBM_PAIR
}

// The same collision for the FP32 forms, written with fused multiply-adds (the
// reduced-precision forms are not reproduced bit for bit, so the contraction
// that saves issue slots is taken here and only here).  With SCALED, f holds
// populations in units of 1/sc (the FP16 storage scale), which the collision is
// linear in except for the quadratic equilibrium term and the velocity; sc is
// folded into those constants instead of rescaling all 19 values.
template <bool SHIFTED, bool SCALED>
__device__ __forceinline__ void collide_f32_scaled(float f[Q], const Consts<float>& k, bool incomp, bool stokes,
                                                   float sc, float isc, float& rho_s, float u[3]) {
  float j[3];
  moments(f, rho_s, j);  // rho_s, j in units of 1/sc
  const float rho0 = incomp ? 1.0f : (SHIFTED ? (SCALED ? __builtin_fmaf(rho_s, isc, 1.0f) : 1.0f + rho_s)
                                              : rho_s);
  float ueq[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float Js = SCALED ? j[a] * isc : j[a];
    const float U = incomp ? Js : Js / rho0;
    u[a] = U + k.hg[a];
    ueq[a] = U - k.glm[a];
  }
  const float c45 = SCALED ? 4.5f * sc : 4.5f;
  const float m15usq = (SCALED ? -1.5f * sc : -1.5f) * usq_of(u);
  const float wr[3] = {float(WD[0]) * rho_s, float(WD[1]) * rho_s, float(WD[7]) * rho_s};
  const float r0s = SCALED ? rho0 * sc : rho0;  // rho_0 in units of 1/sc
  auto ep_of = [&](float cu, int q, int cls) -> float {
    if (stokes) return wr[cls];
    float nl = __builtin_fmaf(c45 * cu, cu, m15usq);
    if (!incomp) nl = rho0 * nl;
    return __builtin_fmaf(float(WD[q]), nl, wr[cls]);
  };
  {
    const float ep = ep_of(0.0f, 0, 0);
    f[0] = __builtin_fmaf(k.lp, f[0] - ep, f[0]);
  }
#define FSLBM_PAIR32(q)                                                   \
  {                                                                       \
    const float cu = cdot<q>(u);                                          \
    const float cue = cdot<q>(ueq);                                       \
    const float em = float(W3D[q]) * (incomp && !SCALED ? cue : r0s * cue); \
    const float ep = ep_of(cu, q, q <= 6 ? 1 : 2);                        \
    const float a = f[q], b = f[q + 1];                                   \
    const float np = 0.5f * (a + b) - ep;                                 \
    const float nm = 0.5f * (a - b) - em;                                 \
    const float lpn = k.lp * np;                                          \
    f[q] = __builtin_fmaf(k.lm, nm, a + lpn);                             \
    f[q + 1] = __builtin_fmaf(-k.lm, nm, b + lpn);                        \
  }
  FSLBM_PAIR32(1) FSLBM_PAIR32(3) FSLBM_PAIR32(5) FSLBM_PAIR32(7) FSLBM_PAIR32(9) FSLBM_PAIR32(11)
  FSLBM_PAIR32(13) FSLBM_PAIR32(15) FSLBM_PAIR32(17)
#undef FSLBM_PAIR32
}

template <bool SHIFTED>
__device__ __forceinline__ void collide_f32(float f[Q], const Consts<float>& k, bool incomp, bool stokes,
                                            float& rho_s, float u[3]) {
  collide_f32_scaled<SHIFTED, false>(f, k, incomp, stokes, 1.0f, 1.0f, rho_s, u);
}

// Post-collision state of a resting-frame equilibrium (rho, u):
// e+(rho, u) + e-(rho_0, u + g/2).  rho_s in storage convention.
template <class R, bool SHIFTED>
__device__ __forceinline__ void equilibrium_post(R rho_s, const R u[3], const Consts<R>& k, bool incomp,
                                                 bool stokes, R out[Q]) {
  const R rho0 = rho0_of<R, SHIFTED>(rho_s, incomp);
  R v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = u[a] + k.hg[a];
  const R usq = usq_of(u);
  out[0] = e_plus<0>(rho_s, rho0, incomp, stokes, u, usq);
#define FSLBM_EQ(q)                                             \
  {                                                             \
    R ep = e_plus<q>(rho_s, rho0, incomp, stokes, u, usq);      \
    R em = e_minus<q>(rho0, incomp, v);                         \
    out[q] = ep + em;                                           \
    out[q + 1] = ep - em;                                       \
  }
  FSLBM_EQ(1) FSLBM_EQ(3) FSLBM_EQ(5) FSLBM_EQ(7) FSLBM_EQ(9) FSLBM_EQ(11) FSLBM_EQ(13) FSLBM_EQ(15)
  FSLBM_EQ(17)
#undef FSLBM_EQ
}

// Moments of time t recovered from post-collision populations (the collision
// keeps rho and adds rho_0 g to the momentum): u = (j/rho_0 - g) + g/2.
template <class R, bool SHIFTED>
__device__ __forceinline__ void recover_moments(const R f[Q], const Consts<R>& k, bool incomp, R& rho_s,
                                                R u[3]) {
  R j[3];
  moments(f, rho_s, j);
  const R rho0 = rho0_of<R, SHIFTED>(rho_s, incomp);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R U = incomp ? j[a] : j[a] / rho0;
    u[a] = (U - k.g[a]) + k.hg[a];
  }
}

// ------------------------------------------------------------- geometry
struct Grid {
  int nx, ny, nz, N;
  int px, py, pz;
  unsigned rx, ry;  // floor(2^32 / nx), floor(2^32 / ny) (2^32 - 1 for 1): see coords
};

// floor(2^32 / d) for d >= 2, 2^32 - 1 for d = 1: the reciprocal coords divides by
inline unsigned grid_recip(int d) {
  return d <= 1 ? 0xffffffffu : (unsigned)(4294967296ull / (unsigned long long)d);
}

// coordinate one step along an axis; -1 if beyond a wall
__device__ __forceinline__ int step_axis(int c, int d, int n, int per) {
  int s = c + d;
  if (s < 0) return per ? n - 1 : -1;
  if (s >= n) return per ? 0 : -1;
  return s;
}

// neighbour index of (x,y,z) at offset (dx,dy,dz); -1 beyond a wall
__device__ __forceinline__ int neighbor(const Grid& g, int x, int y, int z, int dx, int dy, int dz) {
  int sx = dx ? step_axis(x, dx, g.nx, g.px) : x;
  int sy = dy ? step_axis(y, dy, g.ny, g.py) : y;
  int sz = dz ? step_axis(z, dz, g.nz, g.pz) : z;
  if ((sx | sy | sz) < 0) return -1;
  return sx + g.nx * (sy + g.ny * sz);
}

// n / d and n % d for 0 <= n < 2^31 with m = grid_recip(d): since
// n / d - 1 < n m / 2^32 <= n / d, the high word of n m is the quotient or one
// less, and one comparison of the remainder fixes it
__device__ __forceinline__ unsigned divmod_recip(unsigned n, unsigned d, unsigned m, unsigned& r) {
  unsigned q = __umulhi(n, m);
  r = n - q * d;
  if (r >= d) {
    q += 1u;
    r -= d;
  }
  return q;
}

__device__ __forceinline__ void coords(const Grid& g, int idx, int& x, int& y, int& z) {
  unsigned rx, ry;
  const unsigned row = divmod_recip((unsigned)idx, (unsigned)g.nx, g.rx, rx);
  z = (int)divmod_recip(row, (unsigned)g.ny, g.ry, ry);
  x = (int)rx;
  y = (int)ry;
}

}  // namespace fslbm
