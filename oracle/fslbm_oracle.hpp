// Serial reference implementation of the free-surface lattice Boltzmann time
// step (Bogner, Ammer, Ruede: "Boundary Conditions for Free Interfaces with the
// Lattice Boltzmann Method").
//
// TEST INFRASTRUCTURE ONLY.  This oracle exists so that tests, the smoke check
// and the CPU-baseline leg of the benchmark can check the GPU library against
// a plain, slow, obviously correct implementation.  It shares no code, header,
// table or constant with the GPU library and must never be called by it.
//
// Everything is serial, in ascending linear cell order idx = x + nx*(y + ny*z),
// and templated on the scalar type T so that a dual-number scalar can give exact
// directional derivatives (adjoint checks).  T = double is the FP64 oracle.
//
// Parity status per function is listed in the test files; every function here
// is pinned by at least one closed form, invariant or special case, with one
// exception.  Parity unpinned: the weight of the mass exchange between two
// interface cells, (phi_x + phi_s) / 2 in step S4.  The paper leaves it to the
// interface tracking it cites; any symmetric weight conserves mass and passes
// every pin, so only the antisymmetry (mass conservation) is pinned.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

namespace fsref {

// ---------------------------------------------------------------------------
// D3Q19 lattice (section 2.1; experiments use D3Q19, section 4).
// Velocity order: rest, the six axis links, then the twelve diagonals; every
// odd index q has its opposite at q+1.
// ---------------------------------------------------------------------------
static const int Q = 19;
static const int CV[Q][3] = {
    {0, 0, 0},
    {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},  {0, -1, 0}, {0, 0, 1},  {0, 0, -1},
    {1, 1, 0},  {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

// opposite direction: c_qbar = -c_q (section 2.1)
inline int opposite(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

// Lattice weights of Qian et al. for D3Q19 (section 2.1 names them; the values
// 1/3, 1/18, 1/36 are the textbook ones for c_s^2 = 1/3).
inline double weight(int q) {
  if (q == 0) return 1.0 / 3.0;
  if (q <= 6) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

enum CellType : uint8_t { GAS = 0, INTERFACE = 1, LIQUID = 2, SOLID = 3 };
// Rules: bit 0 selects the FSL construction (else the FSK row of Table 1).
// Bit 1 adds the shear-rate entry D c_a c_b S^b_ab of Eq. (bterm) (Table 1,
// column D; section 3.4) with S^b from the bulk; bit 2 adds it with a
// prescribed S^b (section 4.2, linear Couette flow).  Without either, D = 0.
enum Rule { FSK = 0, FSL = 1, FSK_STRESS = 2, FSL_STRESS = 3, FSK_SHEAR = 4, FSL_SHEAR = 5 };

// Model parameters.  tau is the symmetric relaxation time (lambda_+ = -1/tau),
// Lambda = Lambda_+ Lambda_- fixes lambda_- (section 3.1).  g is the body
// acceleration; rho_gas the gas density with P_b = rho_gas / 3 (section 2.3).
struct Params {
  int nx, ny, nz;
  int periodic[3];
  double tau, Lambda;
  int incompressible;  // rho_0 = 1 (He-Luo) if nonzero, else rho_0 = rho
  int stokes;          // drop the quadratic part N_q of e+ (section 2.1)
  double g[3];
  double rho_gas;
  double eps;          // conversion threshold margin
  double wall_u[6][3]; // velocity of the wall faces x-, x+, y-, y+, z-, z+
  double shear_b[6];   // prescribed S^b [xx, yy, zz, xy, xz, yz] (rules with bit 2)
  double sigma;        // surface tension coefficient (0: none)
  int plic;            // FSL link distance: 0 phi - 1/2; 1 the PLIC plane; 2 the PLIC
                       // plane with the height-function normal where its columns are
                       // complete, and the height-function curvature (own or borrowed)
  int hold;            // nonzero: fill levels and interface masses keep their values (a
                       // surface held at a known position; with frozen classes)
};

// ---------------------------------------------------------------------------
// The simulation state and one time step.
// ---------------------------------------------------------------------------
template <class T>
struct Oracle {
  Params p{};
  int N = 0;
  // relaxation constants (section 2.1 and 3.1)
  T lam_p, lam_m;       // lambda_+, lambda_-
  T inv_1p_lam_p;       // 1/(1+lambda_+): recovers n+ from post-collision f
  T gvec[3], half_g[3], g_over_lam_m[3];
  T thr_hi, thr_lo;     // (1+eps), (-eps)
  T rho_b;              // gas density rho_b = 3 P_b of the boundary term
  T Lam_p;              // Lambda_+ = -(1/2 + 1/lambda_+) = tau - 1/2 (section 3.1)

  std::vector<uint8_t> type;  // cell classes
  std::vector<T> ft;          // post-collision populations ft[q*N + cell]
  std::vector<T> mass;        // interface mass m (FP64 bookkeeping)
  std::vector<T> phi;         // fill level at interface cells
  std::vector<T> rho_c;       // density of the last collision at I cells
  std::vector<T> u_c;         // velocity of the last collision u_c[a*N+cell]
  T reservoir = T(0.0);
  bool freeze = false;        // frozen flag topology (no conversions)
  long long steps_done = 0;
  // Record of the branches the FSL closure took (diagnostics for finite
  // differences: two runs with equal counts and signature took the same
  // branch at every link of every step): link distance clamped at 0, at 1,
  // FSK fallback; signature = sum mod 2^64 of a hash of (step, cell, link,
  // branch) over those events, so it does not depend on their order.
  unsigned long long branch_count[3] = {0, 0, 0};
  unsigned long long branch_sig = 0;
  void note_branch(int cell, int q, int code) {
    unsigned long long k = ((unsigned long long)steps_done << 37) ^ ((unsigned long long)cell << 5) ^ (unsigned long long)q;
    k = k * 4ull + (unsigned long long)code;
    k += 0x9e3779b97f4a7c15ull;  // splitmix64 finaliser
    k = (k ^ (k >> 30)) * 0xbf58476d1ce4e5b9ull;
    k = (k ^ (k >> 27)) * 0x94d049bb133111ebull;
    k = k ^ (k >> 31);
    branch_count[code] += 1;
    branch_sig += k;
  }

  // conversion lists of the last step, ascending cell index
  std::vector<int> listF, listE, listEp, listNI, listNL;

  // Solid obstacles (class SOLID, never converted): the non-solid cells with a
  // link into a solid cell, ascending, and per listed cell i and link p
  // (from the cell towards c_p) the wall distance delta in (0, 1] of the wall
  // point x + delta c_p and the wall velocity, where x + c_p is solid.
  bool any_solid = false;
  std::vector<int> wall_cells;
  // A prescribed surface (with held fills): for each interface cell the unit
  // normal towards the gas, surf_n[a*N + cell], and the signed offset of the
  // plane from the node along it, surf_d[cell]; empty if not set.
  std::vector<double> surf_n, surf_d;
  std::vector<double> wall_delta;  // [19][n]
  std::vector<double> wall_uvel;   // [3][19][n]

  // ---------------------------------------------------------------- setup
  void set_params(const Params& q) {
    p = q;
    if (p.nx <= 0 || p.ny <= 0 || p.nz <= 0) throw std::runtime_error("dims must be positive");
    if (!(p.tau > 0.5)) throw std::runtime_error("tau must exceed 1/2");
    if (!(p.Lambda > 0.0)) throw std::runtime_error("Lambda must be positive");
    N = p.nx * p.ny * p.nz;
    // lambda_+ = -1/tau; nu = -(1/3)(1/lambda_+ + 1/2) = (tau - 1/2)/3  (section 2.1)
    // Lambda_+ = -(1/2 + 1/lambda_+) = tau - 1/2 ; Lambda_- = Lambda / Lambda_+ ;
    // lambda_- = -1/(Lambda_- + 1/2)                                (section 3.1)
    double lp = -1.0 / p.tau;
    double Lp = p.tau - 0.5;
    double Lm = p.Lambda / Lp;
    double lm = -1.0 / (Lm + 0.5);
    lam_p = T(lp);
    lam_m = T(lm);
    inv_1p_lam_p = T(1.0 / (1.0 + lp));
    for (int a = 0; a < 3; ++a) {
      gvec[a] = T(p.g[a]);
      half_g[a] = T(0.5 * p.g[a]);
      g_over_lam_m[a] = T(p.g[a] / lm);
    }
    thr_hi = T(1.0 + p.eps);
    thr_lo = T(-p.eps);
    rho_b = T(p.rho_gas);
    Lam_p = T(Lp);
  }

  // Velocity of the wall a link's source lies beyond: the first non-periodic
  // face crossed, in axis order x, y, z (faces x-, x+, y-, y+, z-, z+).
  const double* wall_velocity(int x, int y, int z, int q) const {
    static const double zero[3] = {0.0, 0.0, 0.0};
    const int c[3] = {x - CV[q][0], y - CV[q][1], z - CV[q][2]};
    const int n[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
      if (p.periodic[a]) continue;
      if (c[a] < 0) return p.wall_u[2 * a];
      if (c[a] >= n[a]) return p.wall_u[2 * a + 1];
    }
    return zero;
  }

  // cell at offset d from (x,y,z) (periodic wrap); -1 beyond a wall face
  int raw_neighbor(int x, int y, int z, int dx, int dy, int dz) const {
    int c[3] = {x + dx, y + dy, z + dz};
    int n[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
      if (c[a] < 0 || c[a] >= n[a]) {
        if (!p.periodic[a]) return -1;
        c[a] = (c[a] + n[a]) % n[a];
      }
    }
    return c[0] + p.nx * (c[1] + p.ny * c[2]);
  }
  // neighbour of cell (x,y,z) at offset d; -1 if it lies beyond a wall face or
  // is solid (a solid cell is a wall to the fluid)
  int neighbor(int x, int y, int z, int dx, int dy, int dz) const {
    int s = raw_neighbor(x, y, z, dx, dy, dz);
    return (s >= 0 && type[s] == SOLID) ? -1 : s;
  }
  // slot of a cell in the wall list (binary search), -1 if not listed
  int wall_slot(int cell) const {
    auto it = std::lower_bound(wall_cells.begin(), wall_cells.end(), cell);
    return (it != wall_cells.end() && *it == cell) ? (int)(it - wall_cells.begin()) : -1;
  }

  // The wall table: validated against the classes (every non-solid cell with
  // a link into a solid cell listed, nothing else; delta in (0, 1] on those
  // links).  NULL delta: 1/2 (halfway); NULL velocities: resting walls.
  void set_surface(const double* n3, const double* d) {
    surf_n.assign(n3, n3 + (size_t)3 * N);
    surf_d.assign(d, d + (size_t)N);
  }

  void set_walls(int n, const int* cells, const double* delta, const double* uvel) {
    std::vector<int> need;
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] == SOLID) continue;
      int x, y, z;
      coords(cell, x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = raw_neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && type[s] == SOLID) { need.push_back(cell); break; }
      }
    }
    if (n != (int)need.size()) throw std::runtime_error("wall list must hold exactly the non-solid cells next to solid cells");
    for (int i = 0; i < n; ++i)
      if (cells[i] != need[i]) throw std::runtime_error("wall list must hold exactly the non-solid cells next to solid cells, ascending");
    wall_cells.assign(cells, cells + n);
    wall_delta.assign((size_t)Q * n, 0.5);
    wall_uvel.assign((size_t)3 * Q * n, 0.0);
    for (int i = 0; i < n; ++i) {
      int x, y, z;
      coords(cells[i], x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = raw_neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s < 0 || type[s] != SOLID) continue;
        double d = delta ? delta[(size_t)q * n + i] : 0.5;
        if (!(d > 0.0 && d <= 1.0)) throw std::runtime_error("wall distance outside (0, 1]");
        wall_delta[(size_t)q * n + i] = d;
        if (uvel)
          for (int a = 0; a < 3; ++a) {
            double v = uvel[((size_t)a * Q + q) * n + i];
            if (!std::isfinite(v)) throw std::runtime_error("wall velocity must be finite");
            wall_uvel[((size_t)a * Q + q) * n + i] = v;
          }
      }
    }
  }
  void coords(int cell, int& x, int& y, int& z) const {
    x = cell % p.nx;
    y = (cell / p.nx) % p.ny;
    z = cell / (p.nx * p.ny);
  }

  // The invariant the free-surface model relies on: a liquid cell is never a
  // direct neighbour of a gas cell (the interface layer separates them).
  void check_layer_invariant() const {
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] > SOLID) throw std::runtime_error("unknown cell type");
      if (type[cell] != LIQUID) continue;
      int x, y, z;
      coords(cell, x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && type[s] == GAS)
          throw std::runtime_error("liquid cell " + std::to_string(cell) + " has a gas neighbour");
      }
    }
  }

  // ----------------------------------------------------- equilibria (2.1)
  T rho0_of(const T& rho) const { return p.incompressible ? T(1.0) : rho; }

  // c_q . v: the sum of the (at most two) non-zero components
  static T cdot(int q, const T v[3]) {
    T s = T(0.0);
    for (int a = 0; a < 3; ++a) {
      if (CV[q][a] == 1) s = s + v[a];
      if (CV[q][a] == -1) s = s - v[a];
    }
    return s;
  }

  // even equilibrium e+_q = (w_q/c_s^2)(P + N_q), P = rho/3,
  // N_q = (rho_0/2) u_a u_b (3 c_a c_b - delta_ab)    (Eq. eqEven)
  //     => e+_q = w_q (rho + rho_0 (4.5 (c.u)^2 - 1.5 u.u))
  T e_plus(int q, const T& rho, const T& rho0, const T u[3]) const {
    if (p.stokes) return T(weight(q)) * rho;
    T cu = cdot(q, u);
    T usq = (u[0] * u[0] + u[1] * u[1]) + u[2] * u[2];
    return T(weight(q)) * (rho + rho0 * (T(4.5) * (cu * cu) - T(1.5) * usq));
  }
  // odd equilibrium e-_q = (w_q/c_s^2) rho_0 c_q.u_eq      (Eq. eqOdd)
  T e_minus(int q, const T& rho0, const T ueq[3]) const {
    T cu = cdot(q, ueq);
    return T(3.0 * weight(q)) * (rho0 * cu);
  }

  // Zeroth and first moments (Eq. density, Eq. momentum).
  static void moments(const T f[Q], T& rho, T j[3]) {
    rho = f[0];
    for (int q = 1; q < Q; ++q) rho = rho + f[q];
    for (int a = 0; a < 3; ++a) {
      j[a] = T(0.0);
      for (int q = 0; q < Q; ++q) {
        if (CV[q][a] == 1) j[a] = j[a] + f[q];
        if (CV[q][a] == -1) j[a] = j[a] - f[q];
      }
    }
  }

  // TRT collision, Eq. (lbe2), with the force through
  // u_eq = U - F/lambda_- and rho_0 U = rho_0 u - F/2 = sum c f (section 2.1);
  // F = rho_0 g (g is an acceleration).  Returns rho and u of the pre-collision
  // state.
  void collide(const T f[Q], T out[Q], T& rho, T u[3]) const {
    T j[3];
    moments(f, rho, j);
    T rho0 = rho0_of(rho);
    T U[3], ueq[3];
    for (int a = 0; a < 3; ++a) {
      U[a] = j[a] / rho0;
      u[a] = U[a] + half_g[a];
      ueq[a] = U[a] - g_over_lam_m[a];
    }
    out[0] = f[0] + lam_p * (f[0] - e_plus(0, rho, rho0, u));
    for (int q = 1; q < Q; q += 2) {
      int qb = q + 1;
      T fp = T(0.5) * (f[q] + f[qb]);  // f+_q
      T fm = T(0.5) * (f[q] - f[qb]);  // f-_q
      T np = fp - e_plus(q, rho, rho0, u);
      T nm = fm - e_minus(q, rho0, ueq);
      out[q] = (f[q] + lam_p * np) + lam_m * nm;
      out[qb] = (f[qb] + lam_p * np) - lam_m * nm;
    }
  }

  // Post-collision state of a pre-collision equilibrium with density rho and
  // velocity u: even part e+(rho,u), odd part e-(rho_0, u + g/2) (the collision
  // of such a state adds rho_0 g to its momentum).  Used for the initial state
  // and for cells that newly join the interface.
  void equilibrium_post(const T& rho, const T u[3], T out[Q]) const {
    T rho0 = rho0_of(rho);
    T v[3];
    for (int a = 0; a < 3; ++a) v[a] = u[a] + half_g[a];
    out[0] = e_plus(0, rho, rho0, u);
    for (int q = 1; q < Q; q += 2) {
      T ep = e_plus(q, rho, rho0, u);
      T em = e_minus(q, rho0, v);
      out[q] = ep + em;
      out[q + 1] = ep - em;
    }
  }

  // Moments at time t recovered from post-collision populations: rho is
  // unchanged by the collision, the momentum grew by rho_0 g.
  void recover_moments(const T ftl[Q], T& rho, T u[3]) const {
    T j[3];
    moments(ftl, rho, j);
    T rho0 = rho0_of(rho);
    for (int a = 0; a < 3; ++a) u[a] = (j[a] / rho0 - gvec[a]) + half_g[a];
  }

  // ------------------------------------------- closure coefficients (3.3)
  // General linear closure Eq. (closure) with f^{p.c.} = C n+ (Eq. correction)
  // and f^b = alpha_+ e+(rho_b, u_b) (Eq. bterm with S^b = 0).
  struct Coeffs { T a0, a0bar, a1, alpha_p, C; };
  // FSK row of Table 1 (D = 0): the rule of Eq. (koerner).
  Coeffs coeffs_fsk() const { return {T(-1.0), T(0.0), T(0.0), T(2.0), T(0.0)}; }
  // FSL construction with free parameter alpha_+, Eq. (fsli1)-(fsli4).
  Coeffs coeffs_fsli(const T& alpha_p, const T& delta) const {
    Coeffs c;
    c.a0 = T(1.0) - alpha_p * (T(0.5) + delta);
    c.a0bar = T(1.0) - T(0.5) * alpha_p;
    c.a1 = delta * alpha_p - T(1.0);
    c.alpha_p = alpha_p;
    c.C = (alpha_p * lam_p) * (T(0.5) + delta) - T(2.0) * lam_p;
    return c;
  }

  // ------------------------------------------ boundary shear rate (3.4)
  // Shear rate S_ab = (d_a j_b + d_b j_a)/2 from the even non-equilibrium of
  // post-collision populations of time t.  At leading order Eq. (nqp) gives
  // n+_q = (1/lambda_+)(w_q/c_s^2) c_qa c_qb S_ab, and the fourth moment of the
  // D3Q19 weights, sum_q w_q c_a c_b c_c c_d = c_s^4 (d_ab d_cd + d_ac d_bd +
  // d_ad d_bc), turns M_ab = sum_q c_qa c_qb n+_q into
  // (c_s^2/lambda_+)(d_ab tr S + 2 S_ab); hence tr S = lambda_+ tr M / (5 c_s^2)
  // and S = (lambda_+ / (2 c_s^2)) (M - d tr M / 5).  n+_q is recovered from
  // ft+ = e+ + (1 + lambda_+) n+ with the moments (rho, u) of time t.
  // Components: [xx, yy, zz, xy, xz, yz].
  void shear_from_own(const T own[Q], const T& rho, const T& rho0, const T u[3], T S[6]) const {
    T M[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
    for (int q = 1; q < Q; q += 2) {  // n+ is even: each pair once, counted twice
      T fplus = T(0.5) * (own[q] + own[q + 1]);
      T np = (fplus - e_plus(q, rho, rho0, u)) * inv_1p_lam_p;
      T n2 = T(2.0) * np;
      const int* c = CV[q];
      M[0] = M[0] + T(c[0] * c[0]) * n2;
      M[1] = M[1] + T(c[1] * c[1]) * n2;
      M[2] = M[2] + T(c[2] * c[2]) * n2;
      M[3] = M[3] + T(c[0] * c[1]) * n2;
      M[4] = M[4] + T(c[0] * c[2]) * n2;
      M[5] = M[5] + T(c[1] * c[2]) * n2;
    }
    T tr5 = ((M[0] + M[1]) + M[2]) / T(5.0);
    T f = T(1.5) * lam_p;  // lambda_+ / (2 c_s^2)
    S[0] = f * (M[0] - tr5);
    S[1] = f * (M[1] - tr5);
    S[2] = f * (M[2] - tr5);
    S[3] = f * M[3];
    S[4] = f * M[4];
    S[5] = f * M[5];
  }

  // Boundary value S^b of section 3.4: in a local orthonormal basis {t1, t2, n}
  // the tangential block of S is kept, the tangential-normal entries are set by
  // Eq. (proj2) (d_t j_n + d_n j_t = 0, i.e. zero) and the normal-normal entry
  // by Eq. (proj1) with sigma = 0 (d_n j_n = s_nn).  In the standard basis that
  // is S^b = P S P + s_nn n n^T with the tangential projector P = I - n n^T,
  // whatever t1 and t2 are:  S^b = S - (S n) n^T - n (S n)^T + (n.S.n + s_nn) n n^T.
  static void boundary_shear(const T S[6], const T n[3], const T& s_nn, T Sb[6]) {
    // full matrix view of the symmetric S
    const int ix[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
    T Sn[3];
    for (int a = 0; a < 3; ++a) Sn[a] = (S[ix[a][0]] * n[0] + S[ix[a][1]] * n[1]) + S[ix[a][2]] * n[2];
    T nSn = (n[0] * Sn[0] + n[1] * Sn[1]) + n[2] * Sn[2];
    T k = nSn + s_nn;
    const int ab[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    for (int i = 0; i < 6; ++i) {
      int a = ab[i][0], b = ab[i][1];
      Sb[i] = ((S[i] - Sn[a] * n[b]) - n[a] * Sn[b]) + k * (n[a] * n[b]);
    }
  }

  // Liquid neighbour x + c_k with the largest -c_k.n / |c_k| (lowest k on
  // ties), or -1 if no neighbour is liquid.  |c_k| is 1 or sqrt 2, so the
  // comparison is made on (c_k.n)^2 / |c_k|^2 with the sign of -c_k.n.
  int bulk_neighbour(int x, int y, int z, const T n[3]) const {
    int best = -1;
    T best_v = T(0.0);
    for (int k = 1; k < Q; ++k) {
      int s = neighbor(x, y, z, CV[k][0], CV[k][1], CV[k][2]);
      if (s < 0 || type[s] != LIQUID) continue;
      T cn = -cdot(k, n);
      T len2 = T(k <= 6 ? 1.0 : 2.0);
      T v = cn < T(0.0) ? -(cn * cn) / len2 : (cn * cn) / len2;
      if (best < 0 || v > best_v) {
        best = s;
        best_v = v;
      }
    }
    return best;
  }

  // ----------------------------------------------------- curvature (2.3)
  // Curvature kappa of the free boundary for the pressure jump of Eq.
  // (freeboundary): with the fill gradient g and Hessian H by central
  // differences over the D3Q19 neighbourhood (v[dx+1][dy+1][dz+1]: fill seen
  // from the cell, corners unused), the normal n = -g/|g| points to the gas and
  //   kappa = div(g/|g|) = (|g|^2 tr H - g.H.g) / |g|^3 = -div n,
  // so that P = P_b - sigma kappa is the Laplace pressure P_b + sigma div n
  // (a sphere of radius R: kappa = -2/R).  Zero if g = 0.
  static T curvature(const T v[3][3][3]) {
    const T c = v[1][1][1];
    T g[3], H[3][3];
    g[0] = T(0.5) * (v[2][1][1] - v[0][1][1]);
    g[1] = T(0.5) * (v[1][2][1] - v[1][0][1]);
    g[2] = T(0.5) * (v[1][1][2] - v[1][1][0]);
    H[0][0] = (v[2][1][1] - T(2.0) * c) + v[0][1][1];
    H[1][1] = (v[1][2][1] - T(2.0) * c) + v[1][0][1];
    H[2][2] = (v[1][1][2] - T(2.0) * c) + v[1][1][0];
    H[0][1] = H[1][0] = T(0.25) * (((v[2][2][1] - v[2][0][1]) - v[0][2][1]) + v[0][0][1]);
    H[0][2] = H[2][0] = T(0.25) * (((v[2][1][2] - v[2][1][0]) - v[0][1][2]) + v[0][1][0]);
    H[1][2] = H[2][1] = T(0.25) * (((v[1][2][2] - v[1][2][0]) - v[1][0][2]) + v[1][0][0]);
    T g2 = (g[0] * g[0] + g[1] * g[1]) + g[2] * g[2];
    if (!(g2 > T(0.0))) return T(0.0);
    T trH = (H[0][0] + H[1][1]) + H[2][2];
    T gHg = T(0.0);
    for (int a = 0; a < 3; ++a) {
      T r = (H[a][0] * g[0] + H[a][1] * g[1]) + H[a][2] * g[2];
      gHg = gHg + g[a] * r;
    }
    using std::sqrt;
    T gn = sqrt(g2);
    return (g2 * trH - gHg) / (g2 * gn);
  }

  // ------------------------------------------ PLIC plane offset (sec. 5)
  // Volume of the unit cube [0,1]^3 below the plane m.x = a, m_i >= 0 (not all
  // zero).  The forward relation of Scardovelli & Zaleski (J. Comput. Phys.
  // 164, 2000) by regions of the normalised offset, with the components sorted
  // m1 <= m2 <= m3 and scaled to sum 1; the offset is reflected to the lower
  // half (V(a) = 1 - V(1 - a)).  Regions that divide by m1 carry the
  // difference quotients in closed form, so a vanishing component (a plane
  // parallel to an axis) leaves no cancelled difference divided by it.
  static T cut_volume(const T m[3], const T& a) {
    T s = (m[0] + m[1]) + m[2];
    T m1 = m[0] / s, m2 = m[1] / s, m3 = m[2] / s;
    if (m1 > m2) std::swap(m1, m2);
    if (m2 > m3) std::swap(m2, m3);
    if (m1 > m2) std::swap(m1, m2);
    T b = a / s;
    if (b <= T(0.0)) return T(0.0);
    if (b >= T(1.0)) return T(1.0);
    bool upper = b > T(0.5);
    T al = upper ? T(1.0) - b : b;
    T m12 = m1 + m2;
    T v;
    if (al <= m1) {
      // corner tetrahedron
      v = ((al * al) * al) / (T(6.0) * ((m1 * m2) * m3));
    } else if (al <= m2) {
      // the plane has passed the corner on the smallest axis
      v = (al * (al - m1)) / (T(2.0) * (m2 * m3)) + (m1 * m1) / (T(6.0) * (m2 * m3));
    } else if (al <= m12 && al <= m3) {
      // [al^3 - (al - m1)^3 - (al - m2)^3] / (6 m1 m2 m3), the first
      // difference divided by m1 in closed form
      T t = al - m2;
      T q = ((T(3.0) * (al * al) - T(3.0) * (al * m1)) + m1 * m1) - ((t * t) * t) / m1;
      v = q / (T(6.0) * (m2 * m3));
    } else if (al <= m3) {
      // m1 + m2 <= al <= m3: a prism under a sloped roof, linear in al
      v = ((T(2.0) * al) - m12) / (T(2.0) * m3);
    } else {
      // m3 < al <= 1/2 (only when m3 < m1 + m2): all three corners passed
      T t2 = al - m2, t3 = al - m3;
      T q = ((T(3.0) * (al * al) - T(3.0) * (al * m1)) + m1 * m1) - (((t2 * t2) * t2) + ((t3 * t3) * t3)) / m1;
      v = q / (T(6.0) * (m2 * m3));
    }
    return upper ? T(1.0) - v : v;
  }

  // Offset d of the plane n.(x - x_node) = d (n a unit normal, liquid below)
  // that cuts the fill fraction phi from the cell: V(a) = phi with
  // a = d + (|n_x| + |n_y| + |n_z|)/2, by 64 bisection steps on [0, sum |n_i|].
  // For an axis-aligned normal d = phi - 1/2.
  static T plic_offset(const T& phi, const T n[3]) {
    // (the bisection carries no derivative: the dual-number path never sets plic)
    T m[3];
    for (int i = 0; i < 3; ++i) m[i] = n[i] < T(0.0) ? -n[i] : n[i];
    T sum = (m[0] + m[1]) + m[2];
    T lo = T(0.0), hi = sum;
    for (int it = 0; it < 64; ++it) {
      T mid = T(0.5) * (lo + hi);
      if (cut_volume(m, mid) < phi) lo = mid;
      else hi = mid;
    }
    return T(0.5) * (lo + hi) - T(0.5) * sum;
  }

  // n . S . n for a symmetric S given as [xx, yy, zz, xy, xz, yz]
  static T normal_normal(const T S[6], const T n[3]) {
    T d = (S[0] * (n[0] * n[0]) + S[1] * (n[1] * n[1])) + S[2] * (n[2] * n[2]);
    T o = (S[3] * (n[0] * n[1]) + S[4] * (n[0] * n[2])) + S[5] * (n[1] * n[2]);
    return d + T(2.0) * o;
  }

  // c_q . S . c_q for a symmetric S given as [xx, yy, zz, xy, xz, yz]
  static T cSc(int q, const T S[6]) {
    const int* c = CV[q];
    T d = (T(c[0] * c[0]) * S[0] + T(c[1] * c[1]) * S[1]) + T(c[2] * c[2]) * S[2];
    T o = (T(c[0] * c[1]) * S[3] + T(c[0] * c[2]) * S[4]) + T(c[1] * c[2]) * S[5];
    return d + T(2.0) * o;
  }

  // --------------------------------------------------------------- init
  // flags: cell classes; rho, u (u[a*N+cell]): initial macroscopic state;
  // fill: fill level (used at interface cells; m = fill * rho there).
  void init_from_fields(const uint8_t* flags, const double* rho, const double* u, const double* fill) {
    type.assign(flags, flags + N);
    check_layer_invariant();
    ft.assign((size_t)Q * N, T(0.0));
    mass.assign(N, T(0.0));
    phi.assign(N, T(0.0));
    rho_c.assign(N, T(0.0));
    u_c.assign((size_t)3 * N, T(0.0));
    reservoir = T(0.0);
    any_solid = false;
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] == SOLID) any_solid = true;
      if (type[cell] == GAS || type[cell] == SOLID) continue;
      T r = T(rho[cell]);
      T uu[3] = {T(u[cell]), T(u[N + cell]), T(u[2 * N + cell])};
      T out[Q];
      equilibrium_post(r, uu, out);
      for (int q = 0; q < Q; ++q) ft[(size_t)q * N + cell] = out[q];
      if (type[cell] == INTERFACE) {
        phi[cell] = T(fill[cell]);
        mass[cell] = T(fill[cell]) * r;
        rho_c[cell] = r;
        for (int a = 0; a < 3; ++a) u_c[(size_t)a * N + cell] = uu[a];
      }
    }
  }

  // Restart / adjoint entry: the state given directly.
  void init_from_state(const uint8_t* flags, const T* ftin, const T* m, const T* fill, const T& res) {
    type.assign(flags, flags + N);
    check_layer_invariant();
    any_solid = std::find(type.begin(), type.end(), (uint8_t)SOLID) != type.end();
    ft.assign(ftin, ftin + (size_t)Q * N);
    mass.assign(m, m + N);
    phi.assign(fill, fill + N);
    rho_c.assign(N, T(0.0));
    u_c.assign((size_t)3 * N, T(0.0));
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] != INTERFACE) continue;
      T f[Q], r, uu[3];
      for (int q = 0; q < Q; ++q) f[q] = ft[(size_t)q * N + cell];
      recover_moments(f, r, uu);
      rho_c[cell] = r;
      for (int a = 0; a < 3; ++a) u_c[(size_t)a * N + cell] = uu[a];
    }
    reservoir = res;
  }

  // fill level seen by neighbours: liquid 1, gas 0, interface its own value
  T phi_of(int s) const {
    if (type[s] == LIQUID) return T(1.0);
    if (type[s] == GAS) return T(0.0);
    return phi[s];
  }

  // Interface normal n = -grad(phi)/|grad(phi)| (towards the gas) by central
  // differences over the six axis neighbours (a wall or solid: the cell's own
  // fill).  False (n = 0) where the gradient vanishes.
  bool cd_normal(int x, int y, int z, const T& phix, T nvec[3]) const {
    T grad[3];
    for (int a = 0; a < 3; ++a) {
      int d[3] = {0, 0, 0};
      d[a] = 1;
      int sp = neighbor(x, y, z, d[0], d[1], d[2]);
      int sm = neighbor(x, y, z, -d[0], -d[1], -d[2]);
      T vp = sp < 0 ? phix : phi_of(sp);
      T vm = sm < 0 ? phix : phi_of(sm);
      grad[a] = T(0.5) * (vp - vm);
    }
    T nrm2 = (grad[0] * grad[0] + grad[1] * grad[1]) + grad[2] * grad[2];
    for (int a = 0; a < 3; ++a) nvec[a] = T(0.0);
    if (!(nrm2 > T(0.0))) return false;
    using std::sqrt;  // the dual-number sqrt is found by argument lookup
    T nrm = sqrt(nrm2);
    for (int a = 0; a < 3; ++a) nvec[a] = -grad[a] / nrm;
    return true;
  }

  // cell at offset d (periodic wrap, any |d|); -1 beyond a wall face or solid
  int stencil_cell(int x, int y, int z, const int d[3]) const {
    int c[3] = {x + d[0], y + d[1], z + d[2]};
    int n[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a) {
      if (c[a] < 0 || c[a] >= n[a]) {
        if (!p.periodic[a]) return -1;
        c[a] = ((c[a] % n[a]) + n[a]) % n[a];
      }
    }
    int s = c[0] + p.nx * (c[1] + p.ny * c[2]);
    return type[s] == SOLID ? -1 : s;
  }

  // Column heights of the height function: along the axis a where nvec is
  // largest (lowest axis on ties), h[i+1][j+1] = the fill summed over the 7
  // cells of the column at offsets i, j across a; sg is the side of the gas
  // along a.  False where a column is not complete (fill 1 at its liquid end,
  // 0 at its gas end, no wall or solid in it).
  bool hf_heights(int x, int y, int z, const T nvec[3], T h[3][3], int& a, int& sg) const {
    a = 0;
    for (int b = 1; b < 3; ++b) {
      T ab = nvec[b] < T(0.0) ? -nvec[b] : nvec[b];
      T aa = nvec[a] < T(0.0) ? -nvec[a] : nvec[a];
      if (ab > aa) a = b;
    }
    sg = nvec[a] > T(0.0) ? 1 : -1;
    const int e1 = (a + 1) % 3, e2 = (a + 2) % 3;
    for (int i = -1; i <= 1; ++i)
      for (int j = -1; j <= 1; ++j) {
        T sum = T(0.0);
        for (int k = -3; k <= 3; ++k) {
          int d[3];
          d[a] = k;
          d[e1] = i;
          d[e2] = j;
          int s = stencil_cell(x, y, z, d);
          if (s < 0) return false;
          T v = phi_of(s);
          if (k == -3 * sg && !(v >= T(1.0))) return false;
          if (k == 3 * sg && !(v <= T(0.0))) return false;
          sum = sum + v;
        }
        h[i + 1][j + 1] = sum;
      }
    return true;
  }

  // Height-function normal: with the surface height H known on the 3 x 3
  // columns and central differences H_1, H_2 across them, the normal towards
  // the gas is (s e_a - H_1 e_1 - H_2 e_2)/|.|.  Exact for a plane whose slope
  // against a is at most 1.  Leaves nvec unchanged (and returns false) where a
  // column is not complete.
  bool hf_normal(int x, int y, int z, T nvec[3]) const {
    T h[3][3];
    int a, sg;
    if (!hf_heights(x, y, z, nvec, h, a, sg)) return false;
    const int e1 = (a + 1) % 3, e2 = (a + 2) % 3;
    T h1 = T(0.5) * (h[2][1] - h[0][1]);
    T h2 = T(0.5) * (h[1][2] - h[1][0]);
    T v[3];
    v[a] = T((double)sg);
    v[e1] = -h1;
    v[e2] = -h2;
    T nrm2 = (v[0] * v[0] + v[1] * v[1]) + v[2] * v[2];
    using std::sqrt;
    T nrm = sqrt(nrm2);
    for (int b = 0; b < 3; ++b) nvec[b] = v[b] / nrm;
    return true;
  }

  // Height-function curvature (the second-order reconstruction applied to
  // kappa of Eq. freeboundary): with the axis from the central-difference
  // normal and the 3 x 3 column heights, kappa = -div n = [H_11 (1 + H_2^2) +
  // H_22 (1 + H_1^2) - 2 H_12 H_1 H_2] / (1 + H_1^2 + H_2^2)^(3/2), central
  // differences throughout (a sphere of radius R has kappa = -2/R).  False
  // where there is no normal or a column is not complete.
  bool hf_curvature(int x, int y, int z, const T& phix, T& kappa) const {
    T n[3], h[3][3];
    int a, sg;
    if (!cd_normal(x, y, z, phix, n)) return false;
    if (!hf_heights(x, y, z, n, h, a, sg)) return false;
    T h1 = T(0.5) * (h[2][1] - h[0][1]);
    T h2 = T(0.5) * (h[1][2] - h[1][0]);
    T h11 = (h[2][1] - T(2.0) * h[1][1]) + h[0][1];
    T h22 = (h[1][2] - T(2.0) * h[1][1]) + h[1][0];
    T h12 = T(0.25) * (((h[2][2] - h[2][0]) - h[0][2]) + h[0][0]);
    T q = (T(1.0) + h1 * h1) + h2 * h2;
    using std::sqrt;
    T num = (h11 * (T(1.0) + h2 * h2) + h22 * (T(1.0) + h1 * h1)) - T(2.0) * ((h12 * h1) * h2);
    kappa = num / (q * sqrt(q));
    return true;
  }

  // Height-function kappa of an interface cell with a normal (false where
  // it has none or a column is not complete).
  bool hf_kappa_at(int cell, T& kappa) const {
    if (type[cell] != INTERFACE) return false;
    int x, y, z;
    coords(cell, x, y, z);
    return hf_curvature(x, y, z, phi[cell], kappa);
  }

  // The curvature of the Laplace pressure (Eq. freeboundary) with plic = 2,
  // the second-order reconstruction asked for in section 5 applied to kappa:
  // the cell's own height-function kappa; where
  // its columns are not complete, the mean of the height-function kappa of
  // its D3Q19 interface neighbours that have one (summed in link order);
  // without such a neighbour kcd, the central-difference kappa.  A cell
  // next to complete columns lies on the same stretch of surface, and the
  // central-difference kappa of the raw fills is biased by the fill itself
  // (of the wrong sign at small fills), so borrowing keeps the mean of kappa
  // over the surface.  hf(c, k): hf_kappa_at of cell c (computed or looked up).
  template <class HF>
  T hf_or_borrowed(int x, int y, int z, int cell, const T& kcd, const HF& hf) const {
    T k;
    if (hf(cell, k)) return k;
    T sum = T(0.0);
    int cnt = 0;
    for (int q = 1; q < Q; ++q) {
      int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
      if (s < 0 || !hf(s, k)) continue;
      sum = sum + k;
      ++cnt;
    }
    return cnt ? sum / T((double)cnt) : kcd;
  }

  void hf_kappa_field(std::vector<uint8_t>& have, std::vector<T>& khf) const {
    have.assign(N, 0);
    khf.assign(N, T(0.0));
    for (int c = 0; c < N; ++c) have[c] = hf_kappa_at(c, khf[c]) ? 1 : 0;
  }

  // The curvature a step uses at an interface cell (for tests): the
  // central-difference kappa of the D3Q19 fill block, or with plic = 2 the
  // height-function kappa, own or borrowed (hf_or_borrowed); 0 without a
  // normal.
  T interface_curvature(int cell) const {
    int x, y, z;
    coords(cell, x, y, z);
    T n[3];
    const T phix = phi[cell];
    if (!cd_normal(x, y, z, phix, n)) return T(0.0);
    T v[3][3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int cc = 0; cc < 3; ++cc) {
          v[a][b][cc] = T(0.0);
          int nz_ = (a != 1) + (b != 1) + (cc != 1);
          if (nz_ == 0) { v[a][b][cc] = phix; continue; }
          if (nz_ == 3) continue;
          int sN = neighbor(x, y, z, a - 1, b - 1, cc - 1);
          v[a][b][cc] = sN < 0 ? phix : phi_of(sN);
        }
    T kap = curvature(v);
    if (p.plic == 2) kap = hf_or_borrowed(x, y, z, cell, kap, [this](int c, T& k) { return hf_kappa_at(c, k); });
    return kap;
  }

  // The normal a step uses at an interface cell for a rule (for tests).
  bool interface_normal(int cell, int rule, T nvec[3]) const {
    int x, y, z;
    coords(cell, x, y, z);
    bool ok = cd_normal(x, y, z, phi[cell], nvec);
    if (p.plic == 2 && ok && (rule & 1)) hf_normal(x, y, z, nvec);
    return ok;
  }

  // ------------------------------------------------------------ one step
  std::vector<T> ftn;  // second population buffer (pull scheme ping-pong)

  void step(int rule) {
    if (any_solid && wall_cells.empty()) throw std::runtime_error("solid cells present but no wall table set");
    ftn.resize((size_t)Q * N);
    std::vector<T> massn = mass;
    std::vector<T> phin = phi;
    // height-function kappa of every interface cell at time t (plic = 2)
    std::vector<uint8_t> hf_have;
    std::vector<T> hf_k;
    if (p.sigma != 0.0 && p.plic == 2) hf_kappa_field(hf_have, hf_k);

    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] == GAS || type[cell] == SOLID) continue;
      int x, y, z;
      coords(cell, x, y, z);
      const bool iface = type[cell] == INTERFACE;

      // own post-collision populations of time t
      T own[Q];
      for (int q = 0; q < Q; ++q) own[q] = ft[(size_t)q * N + cell];

      // ---- S1 stream, Eq. (lbe1) in pull form: f_q(x) = ft_q(x - c_q).
      // A source beyond a wall gives halfway bounce-back f_q(x) = ft_qbar(x).
      T f[Q];
      bool gaslink[Q] = {false};
      int src[Q];
      bool solidlink[Q] = {false};
      for (int q = 0; q < Q; ++q) {
        int s = neighbor(x, y, z, -CV[q][0], -CV[q][1], -CV[q][2]);
        src[q] = s;
        if (s < 0 && q > 0) {
          int r = raw_neighbor(x, y, z, -CV[q][0], -CV[q][1], -CV[q][2]);
          solidlink[q] = r >= 0;  // a solid source (not a wall face)
        }
        if (s < 0 && solidlink[q]) {
          f[q] = own[opposite(q)];  // completed below (CLI)
        } else if (s < 0) {
          // halfway bounce-back off a wall moving with u_w (section 4.1):
          // f_q = ft_qbar + 2 w_q (c_q . u_w) / c_s^2, with rho_w = 1
          f[q] = own[opposite(q)];
          const double* uw = wall_velocity(x, y, z, q);
          double cu = (CV[q][0] * uw[0] + CV[q][1] * uw[1]) + CV[q][2] * uw[2];
          if (cu != 0.0) f[q] = f[q] + T(6.0 * weight(q) * cu);
        } else if (type[s] == GAS) {
          if (!iface) throw std::runtime_error("liquid cell with gas neighbour");
          gaslink[q] = true;
          f[q] = T(0.0);
        } else {
          f[q] = ft[(size_t)q * N + s];
        }
      }

      // Solid walls: the linear-interpolation closure (CLI) for the link p =
      // qbar that points from the cell to the wall point x + delta c_p.  In the
      // closure f_q(x,t+1) = a0 ft_p(x) + a0bar ft_q(x) + a1 ft_p(x - c_p) + f^b
      // the fitting conditions alpha_+ = 0 (no pressure term) and beta_+ /
      // lambda_+ = alpha_- delta (momentum at the wall point to first order,
      // Eq. fitting and cl1) with C = 0 leave one free coefficient; a0 = 1
      // gives kappa = (1 - 2 delta)/(1 + 2 delta), a1 = kappa, a0bar = -kappa,
      // and f^b = alpha_- e-_p(u_w) with alpha_- = -4/(1 + 2 delta).  Exact for
      // linear velocity profiles; halfway bounce-back at delta = 1/2.  Where
      // ft_p(x - c_p) is not a fluid population (a wall, a solid or gas there)
      // the link takes halfway bounce-back.
      if (any_solid) {
        const int slot = wall_slot(cell);
        const int nw = (int)wall_cells.size();
        for (int q = 1; q < Q; ++q) {
          if (!solidlink[q]) continue;
          if (slot < 0) throw std::runtime_error("cell next to a solid missing from the wall table");
          const int pl = opposite(q);
          const double d = wall_delta[(size_t)pl * nw + slot];
          double uw[3];
          for (int a = 0; a < 3; ++a) uw[a] = wall_uvel[((size_t)a * Q + pl) * nw + slot];
          // 2 w (c_q . u_w) / c_s^2 of halfway bounce-back (rho_w = 1)
          const double bb = 6.0 * weight(q) * ((CV[q][0] * uw[0] + CV[q][1] * uw[1]) + CV[q][2] * uw[2]);
          const bool upstream = src[pl] >= 0 && type[src[pl]] != GAS;
          if (upstream) {
            const double kap = (1.0 - 2.0 * d) / (1.0 + 2.0 * d);
            f[q] = (own[pl] + T(kap) * (f[pl] - own[q])) + T(bb * (2.0 / (1.0 + 2.0 * d)));
          } else {
            f[q] = own[pl] + T(bb);
          }
        }
      }

      T m_new = T(0.0);
      if (iface) {
        const T phix = phi[cell];

        // ---- S4 mass exchange (interface tracking of the cited FSLBM):
        // dm = sum_q w_xs (ft_q(x - c_q) - ft_qbar(x)), weight 1 to liquid,
        // (phi_x + phi_s)/2 to interface, 0 to gas and walls.
        T dm = T(0.0);
        for (int q = 1; q < Q; ++q) {
          int s = src[q];
          if (s < 0 || type[s] == GAS) continue;
          T diff = ft[(size_t)q * N + s] - own[opposite(q)];
          if (type[s] == LIQUID) {
            dm = dm + diff;
          } else {
            T wgt = T(0.5) * (phix + phi[s]);  // parity unpinned (see the header)
            dm = dm + wgt * diff;
          }
        }
        m_new = mass[cell] + dm;

        // ---- S2 interface geometry: normal from the fill-level gradient
        // (central differences over the six axis neighbours), surface plane
        // at signed distance phi - 1/2 from the node along the normal.
        T nvec[3];
        bool have_normal = cd_normal(x, y, z, phix, nvec);
        // second-order reconstruction (section 5): the FSL rules may take the
        // normal from height functions where their columns are complete
        if (p.plic == 2 && have_normal && (rule & 1)) hf_normal(x, y, z, nvec);
        T dist = phix - T(0.5);
        // second-order interface position (section 5): the plane that cuts the
        // cell's fill fraction with the normal n (PLIC) instead of phi - 1/2
        if (p.plic && have_normal && (rule & 1)) dist = plic_offset(phix, nvec);
        // a prescribed surface: the given plane (section 2.2: the boundary
        // link meets it at x_b + delta c_q)
        if (!surf_d.empty()) {
          for (int a = 0; a < 3; ++a) nvec[a] = T(surf_n[(size_t)a * N + cell]);
          dist = T(surf_d[cell]);
          have_normal = true;
        }

        // Laplace pressure: the boundary term takes P_b - sigma kappa (Eq.
        // freeboundary), i.e. rho_b - 3 sigma kappa
        T rho_bc = rho_b;
        if (p.sigma != 0.0 && have_normal) {
          T v[3][3][3];
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
              for (int cc = 0; cc < 3; ++cc) {
                v[a][b][cc] = T(0.0);
                int nz_ = (a != 1) + (b != 1) + (cc != 1);
                if (nz_ == 0) { v[a][b][cc] = phix; continue; }
                if (nz_ == 3) continue;  // corners: not D3Q19 neighbours, unused
                int sN = neighbor(x, y, z, a - 1, b - 1, cc - 1);
                v[a][b][cc] = sN < 0 ? phix : phi_of(sN);
              }
          T kap = curvature(v);
          if (p.plic == 2)
            kap = hf_or_borrowed(x, y, z, cell, kap, [&](int c, T& k) {
              if (!hf_have[c]) return false;
              k = hf_k[c];
              return true;
            });
          rho_bc = rho_b - T(3.0 * p.sigma) * kap;
        }

        // ---- S3 reconstruction of every population streaming in from gas.
        // In the paper's notation the link to gas is o (x + c_o is gas) and the
        // unknown is f_{obar} = f_q.  Moments of time t from the own state:
        T rho_t, u_t[3];
        recover_moments(own, rho_t, u_t);
        const T rho0_t = rho0_of(rho_t);
        const T rho0_b = rho0_of(rho_bc);
        // Boundary shear rate for the rules with D != 0 (section 3.4): S
        // extrapolated from the bulk at order zero, i.e. taken from the
        // non-equilibrium of time t of the liquid neighbour x + c_k whose link
        // points most directly into the liquid (largest -c_k.n / |c_k|, lowest
        // k on ties; the cell itself if no neighbour is liquid).  In the basis
        // {t1, t2, n}: tangential block kept,
        // tangential-normal entries zero (Eq. proj2), normal-normal entry
        // S_nn / 3.  The closure, Taylor-expanded at the surface point, holds
        // P - P_b = Lambda_+ (S_nn - S^b_nn) on the links it reconstructs;
        // Eq. (proj1) with sigma = 0 asks P - P_b = 2 nu S_nn, and with
        // nu = c_s^2 Lambda_+ that is S^b_nn = (1 - 2 c_s^2) S_nn = S_nn / 3.
        // Without a normal there is no local basis and the term is left out.
        const bool stress = ((rule & 2) && have_normal) || (rule & 4);
        T Sb[6] = {T(0.0), T(0.0), T(0.0), T(0.0), T(0.0), T(0.0)};
        if (rule & 4) {
          for (int i = 0; i < 6; ++i) Sb[i] = T(p.shear_b[i]);  // prescribed boundary value
        } else if (stress) {
          int nb = bulk_neighbour(x, y, z, nvec);
          T fb[Q];
          for (int q = 0; q < Q; ++q) fb[q] = nb < 0 ? own[q] : ft[(size_t)q * N + nb];
          T rho_n, u_n[3];
          recover_moments(fb, rho_n, u_n);
          T S[6];
          shear_from_own(fb, rho_n, rho0_of(rho_n), u_n, S);
          T s_nn = normal_normal(S, nvec) / T(3.0);
          boundary_shear(S, nvec, s_nn, Sb);
        }
        for (int q = 1; q < Q; ++q) {
          if (!gaslink[q]) continue;
          int o = opposite(q);
          // n+_o(x,t): pre-collision even non-equilibrium recovered from
          // ft+ = e+ + (1 + lambda_+) n+
          T fplus = T(0.5) * (own[o] + own[q]);
          T n_plus = (fplus - e_plus(o, rho_t, rho0_t, u_t)) * inv_1p_lam_p;
          T e_b = e_plus(o, rho_bc, rho0_b, u_t);  // boundary value, u_b = u(x,t)
          Coeffs k = coeffs_fsk();
          T f_o_next = T(0.0);
          if (rule & 1) {
            // ft_o(x - c_o, t) = f_o(x, t+1): the value the pull delivers
            // along o; unavailable when that source is gas too.
            bool ok = have_normal && !gaslink[o];
            T nc = cdot(o, nvec);
            if (ok && nc > T(0.0)) {
              T delta = dist / nc;
              if (delta < T(0.0)) { delta = T(0.0); note_branch(cell, q, 0); }
              if (delta > T(1.0)) { delta = T(1.0); note_branch(cell, q, 1); }
              k = coeffs_fsli(T(1.0), delta);
              f_o_next = f[o];
            } else {
              note_branch(cell, q, 2);
            }
          }
          // Eq. (closure): f_{obar}(x,t+1) = a0 ft_o + a0bar ft_obar + a1 ft_o(x-c_o)
          //                                  + C n+_o + alpha_+ e+_o(rho_b,u_b)
          f[q] = (((k.a0 * own[o] + k.a0bar * own[q]) + k.a1 * f_o_next) + k.C * n_plus) +
                 k.alpha_p * e_b;
          // + D c_o c_o : S^b with D = -alpha_+ Lambda_+ w/c_s^2 (Eq. bterm, Table 1)
          if (stress) {
            T D = -((k.alpha_p * Lam_p) * T(3.0 * weight(o)));
            f[q] = f[q] + D * cSc(o, Sb);
          }
        }
      }

      // ---- S5 collide
      T out[Q], rho, u[3];
      collide(f, out, rho, u);
      for (int q = 0; q < Q; ++q) ftn[(size_t)q * N + cell] = out[q];

      if (iface) {
        // ---- S6 fill level and classification
        massn[cell] = p.hold ? mass[cell] : m_new;
        phin[cell] = p.hold ? phi[cell] : m_new / rho;
        rho_c[cell] = rho;
        for (int a = 0; a < 3; ++a) u_c[(size_t)a * N + cell] = u[a];
      }
    }

    ft.swap(ftn);
    mass.swap(massn);
    phi.swap(phin);

    listF.clear(); listE.clear(); listEp.clear(); listNI.clear(); listNL.clear();
    if (!freeze && !p.hold) convert();  // a held surface keeps its classes
    ++steps_done;
  }

  // ---------------------------------------------- S6/S7 cell conversions
  // Filled: m > (1+eps) rho; emptied: m < -eps rho (rho of the last collision).
  void convert() {
    std::vector<uint8_t> filled(N, 0), emptied(N, 0);
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] != INTERFACE) continue;
      if (mass[cell] > thr_hi * rho_c[cell]) { filled[cell] = 1; listF.push_back(cell); }
      if (mass[cell] < thr_lo * rho_c[cell]) { emptied[cell] = 1; listE.push_back(cell); }
    }
    auto near_filled = [&](int cell) {
      int x, y, z;
      coords(cell, x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && filled[s]) return true;
      }
      return false;
    };
    // E' = E minus the neighbourhood of F
    std::vector<uint8_t> emptied2(N, 0);
    for (int cell : listE)
      if (!near_filled(cell)) { emptied2[cell] = 1; listEp.push_back(cell); }
    // NI: gas next to a filled cell; NL: liquid next to an E' cell
    std::vector<uint8_t> newI(N, 0), newL(N, 0);
    for (int cell : listF) {
      int x, y, z;
      coords(cell, x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && type[s] == GAS) newI[s] = 1;
      }
    }
    for (int cell : listEp) {
      int x, y, z;
      coords(cell, x, y, z);
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && type[s] == LIQUID) newL[s] = 1;
      }
    }
    for (int cell = 0; cell < N; ++cell) {
      if (newI[cell]) listNI.push_back(cell);
      if (newL[cell]) listNL.push_back(cell);
    }
    // New interface cells from gas: post-collision equilibrium with the mean
    // density and velocity of their interface neighbours (before conversion).
    for (int cell : listNI) {
      int x, y, z;
      coords(cell, x, y, z);
      T rs = T(0.0), us[3] = {T(0.0), T(0.0), T(0.0)};
      int cnt = 0;
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s < 0 || type[s] == GAS) continue;
        rs = rs + rho_c[s];
        for (int a = 0; a < 3; ++a) us[a] = us[a] + u_c[(size_t)a * N + s];
        ++cnt;
      }
      T rbar = rs / T((double)cnt);
      T ubar[3];
      for (int a = 0; a < 3; ++a) ubar[a] = us[a] / T((double)cnt);
      T out[Q];
      equilibrium_post(rbar, ubar, out);
      for (int q = 0; q < Q; ++q) ft[(size_t)q * N + cell] = out[q];
      mass[cell] = T(0.0);
      rho_c[cell] = rbar;
      for (int a = 0; a < 3; ++a) u_c[(size_t)a * N + cell] = ubar[a];
    }
    // New interface cells from liquid keep their populations; m = rho.
    for (int cell : listNL) {
      T r = ft[cell];
      for (int q = 1; q < Q; ++q) r = r + ft[(size_t)q * N + cell];
      mass[cell] = r;
      rho_c[cell] = r;
      T f[Q], rr, uu[3];
      for (int q = 0; q < Q; ++q) f[q] = ft[(size_t)q * N + cell];
      recover_moments(f, rr, uu);
      for (int a = 0; a < 3; ++a) u_c[(size_t)a * N + cell] = uu[a];
    }
    // excess mass of converted cells
    std::vector<T> excess(N, T(0.0));
    for (int cell : listF) excess[cell] = mass[cell] - rho_c[cell];
    for (int cell : listEp) excess[cell] = mass[cell];
    // commit the new classes
    for (int cell : listF) type[cell] = LIQUID;
    for (int cell : listEp) type[cell] = GAS;
    for (int cell : listNI) type[cell] = INTERFACE;
    for (int cell : listNL) type[cell] = INTERFACE;
    // share of each converted cell: split equally over its interface
    // neighbours after conversion; none -> reservoir (ascending order).
    std::vector<T> share(N, T(0.0));
    std::vector<uint8_t> converted(N, 0);
    std::vector<int> conv = listF;
    conv.insert(conv.end(), listEp.begin(), listEp.end());
    std::sort(conv.begin(), conv.end());
    for (int cell : conv) {
      converted[cell] = 1;
      int x, y, z;
      coords(cell, x, y, z);
      int n_elig = 0;
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && type[s] == INTERFACE) ++n_elig;
      }
      if (n_elig == 0) {
        reservoir = reservoir + excess[cell];
        converted[cell] = 0;
      } else {
        share[cell] = excess[cell] / T((double)n_elig);
      }
    }
    // every interface cell gathers the shares of its converted neighbours
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] != INTERFACE) continue;
      int x, y, z;
      coords(cell, x, y, z);
      bool got = false;
      T m = mass[cell];
      for (int q = 1; q < Q; ++q) {
        int s = neighbor(x, y, z, CV[q][0], CV[q][1], CV[q][2]);
        if (s >= 0 && converted[s]) { m = m + share[s]; got = true; }
      }
      if (got) {
        mass[cell] = m;
        phi[cell] = m / rho_c[cell];
      }
    }
    for (int cell : listF) { mass[cell] = T(0.0); phi[cell] = T(0.0); }
    for (int cell : listEp) { mass[cell] = T(0.0); phi[cell] = T(0.0); }
  }

  // ------------------------------------------------------- diagnostics
  // M = sum over liquid of sum_q ft + sum over interface of m + reservoir
  T total_mass() const {
    T M = T(0.0);
    for (int cell = 0; cell < N; ++cell) {
      if (type[cell] == LIQUID) {
        T r = ft[cell];
        for (int q = 1; q < Q; ++q) r = r + ft[(size_t)q * N + cell];
        M = M + r;
      } else if (type[cell] == INTERFACE) {
        M = M + mass[cell];
      }
    }
    return M + reservoir;
  }
};

}  // namespace fsref
