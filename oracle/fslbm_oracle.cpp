// C entry points of the serial FP64 oracle (test infrastructure only; see
// fslbm_oracle.hpp).  Loaded by the tests through ctypes.
#include <cstdio>
#include <memory>

#include "dual.hpp"
#include "fslbm_oracle.hpp"

using fsref::Dual;
using fsref::Oracle;
using fsref::Params;

namespace {
struct Handle {
  Oracle<double> sim;
  std::string err;
};
thread_local std::string g_create_error;
}  // namespace

extern "C" {

struct ref_params {
  int nx, ny, nz;
  int px, py, pz;
  double tau, Lambda;
  int incompressible, stokes;
  double gx, gy, gz;
  double rho_gas, eps;
  double wall_u[18];  // faces x-, x+, y-, y+, z-, z+
  double shear_b[6];  // prescribed S^b [xx, yy, zz, xy, xz, yz]
  double sigma;       // surface tension coefficient
  int plic;           // FSL link distance from the PLIC plane
  int hold;           // fill levels and interface masses held
};

static Params to_params(const ref_params* r) {
  Params p{};
  p.nx = r->nx;
  p.ny = r->ny;
  p.nz = r->nz;
  p.periodic[0] = r->px;
  p.periodic[1] = r->py;
  p.periodic[2] = r->pz;
  p.tau = r->tau;
  p.Lambda = r->Lambda;
  p.incompressible = r->incompressible;
  p.stokes = r->stokes;
  p.g[0] = r->gx;
  p.g[1] = r->gy;
  p.g[2] = r->gz;
  p.rho_gas = r->rho_gas;
  p.eps = r->eps;
  for (int f = 0; f < 6; ++f)
    for (int a = 0; a < 3; ++a) p.wall_u[f][a] = r->wall_u[3 * f + a];
  for (int i = 0; i < 6; ++i) p.shear_b[i] = r->shear_b[i];
  p.sigma = r->sigma;
  p.plic = r->plic;
  p.hold = r->hold;
  return p;
}

// Create from macroscopic fields (flags, rho, u[3][N], fill).  Returns NULL on
// invalid input; ref_create_error() then says why.
void* ref_create(const ref_params* rp, const uint8_t* flags, const double* rho, const double* u,
                 const double* fill) {
  try {
    auto h = std::make_unique<Handle>();
    h->sim.set_params(to_params(rp));
    h->sim.init_from_fields(flags, rho, u, fill);
    return h.release();
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return nullptr;
  }
}

// Create from a full state: flags, post-collision populations ft[19][N], mass,
// fill, reservoir.
void* ref_create_state(const ref_params* rp, const uint8_t* flags, const double* ft, const double* mass,
                       const double* fill, double reservoir) {
  try {
    auto h = std::make_unique<Handle>();
    h->sim.set_params(to_params(rp));
    h->sim.init_from_state(flags, ft, mass, fill, reservoir);
    return h.release();
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return nullptr;
  }
}

const char* ref_create_error() { return g_create_error.c_str(); }

// Solid walls: the ascending list of the n non-solid cells next to solid
// cells, per listed cell and link p the wall distance delta[p*n + i] (NULL:
// 1/2) and the wall velocity uvel[(a*19 + p)*n + i] (NULL: at rest).  Returns
// 0, or -1 with ref_error() saying why.
int ref_set_walls(void* hp, int n, const int* cells, const double* delta, const double* uvel) {
  auto* h = static_cast<Handle*>(hp);
  try {
    h->sim.set_walls(n, cells, delta, uvel);
    return 0;
  } catch (const std::exception& e) {
    h->err = e.what();
    return -1;
  }
}

// Prescribed surface: normal[3 N] (unit, towards the gas) and offset[N] of the
// plane from each interface cell's node.
void ref_set_surface(void* hp, const double* normal, const double* offset) {
  static_cast<Handle*>(hp)->sim.set_surface(normal, offset);
}

void ref_destroy(void* hp) { delete static_cast<Handle*>(hp); }

const char* ref_error(void* hp) { return static_cast<Handle*>(hp)->err.c_str(); }

void ref_set_freeze(void* hp, int freeze) { static_cast<Handle*>(hp)->sim.freeze = freeze != 0; }

// n steps with rule 0 = FSK, 1 = FSL, 2 / 3 = FSK / FSL with the shear-rate
// boundary term (D of Table 1) from the bulk, 4 / 5 = the same with the
// prescribed S^b.  Returns 0, or 1 with ref_error() set.
int ref_step(void* hp, int n, int rule) {
  auto* h = static_cast<Handle*>(hp);
  if (rule < 0 || rule > 5) {
    h->err = "unknown rule";
    return 1;
  }
  try {
    for (int i = 0; i < n; ++i) h->sim.step(rule);
    return 0;
  } catch (const std::exception& e) {
    h->err = e.what();
    return 1;
  }
}

void ref_get_populations(void* hp, double* out) {
  auto& s = static_cast<Handle*>(hp)->sim;
  std::memcpy(out, s.ft.data(), sizeof(double) * s.ft.size());
}
void ref_get_flags(void* hp, uint8_t* out) {
  auto& s = static_cast<Handle*>(hp)->sim;
  std::memcpy(out, s.type.data(), s.type.size());
}
void ref_get_mass(void* hp, double* out) {
  auto& s = static_cast<Handle*>(hp)->sim;
  std::memcpy(out, s.mass.data(), sizeof(double) * s.mass.size());
}
void ref_get_phi(void* hp, double* out) {
  auto& s = static_cast<Handle*>(hp)->sim;
  std::memcpy(out, s.phi.data(), sizeof(double) * s.phi.size());
}
// density and velocity of the last collision at interface cells
void ref_get_collision_moments(void* hp, double* rho, double* u) {
  auto& s = static_cast<Handle*>(hp)->sim;
  std::memcpy(rho, s.rho_c.data(), sizeof(double) * s.rho_c.size());
  std::memcpy(u, s.u_c.data(), sizeof(double) * s.u_c.size());
}
// rho and u at every non-gas cell recovered from the current post-collision
// populations (gas cells get 0)
void ref_get_macro(void* hp, double* rho, double* u) {
  auto& s = static_cast<Handle*>(hp)->sim;
  const int N = s.N;
  for (int cell = 0; cell < N; ++cell) {
    if (s.type[cell] == fsref::GAS) {
      rho[cell] = 0.0;
      u[cell] = u[N + cell] = u[2 * N + cell] = 0.0;
      continue;
    }
    double f[fsref::Q], r, uu[3];
    for (int q = 0; q < fsref::Q; ++q) f[q] = s.ft[(size_t)q * N + cell];
    s.recover_moments(f, r, uu);
    rho[cell] = r;
    for (int a = 0; a < 3; ++a) u[(size_t)a * N + cell] = uu[a];
  }
}
double ref_total_mass(void* hp) { return static_cast<Handle*>(hp)->sim.total_mass(); }
double ref_reservoir(void* hp) { return static_cast<Handle*>(hp)->sim.reservoir; }

// Branches of the FSL closure so far: out = {clamped at 0, clamped at 1, FSK
// fallback, order-independent signature of (step, cell, link, branch)}.
void ref_branch_stats(void* hp, unsigned long long* out) {
  const auto& s = static_cast<Handle*>(hp)->sim;
  for (int i = 0; i < 3; ++i) out[i] = s.branch_count[i];
  out[3] = s.branch_sig;
}

// which: 0 = filled, 1 = emptied, 2 = emptied and converted, 3 = new interface
// from gas, 4 = new interface from liquid.  Copies up to cap entries and
// returns the list length.
int ref_list(void* hp, int which, int* out, int cap) {
  auto& s = static_cast<Handle*>(hp)->sim;
  const std::vector<int>* L[5] = {&s.listF, &s.listE, &s.listEp, &s.listNI, &s.listNL};
  if (which < 0 || which > 4) return -1;
  const auto& v = *L[which];
  int n = (int)v.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = v[i];
  return n;
}

// Relaxation constants as the oracle derives them (for tests).
void ref_constants(void* hp, double* out4) {
  auto& s = static_cast<Handle*>(hp)->sim;
  out4[0] = s.lam_p;
  out4[1] = s.lam_m;
  out4[2] = s.inv_1p_lam_p;
  out4[3] = s.thr_hi;
}

// Pointwise building blocks, exposed for the identity tests.
void ref_equilibrium_post(void* hp, double rho, const double* u, double* out19) {
  static_cast<Handle*>(hp)->sim.equilibrium_post(rho, u, out19);
}
void ref_collide(void* hp, const double* f19, double* out19, double* rho, double* u3) {
  static_cast<Handle*>(hp)->sim.collide(f19, out19, *rho, u3);
}
// Shear rate S = [xx, yy, zz, xy, xz, yz] of section 3.4 from 19 post-collision
// populations of time t (moments recovered from them).
void ref_shear(void* hp, const double* own19, double* S6) {
  auto& s = static_cast<Handle*>(hp)->sim;
  double rho, u[3];
  s.recover_moments(own19, rho, u);
  s.shear_from_own(own19, rho, s.rho0_of(rho), u, S6);
}
// Curvature of the fill field from the 3x3x3 block v27[(dx+1) + 3(dy+1) + 9(dz+1)]
// around a cell (corners unused); kappa = -div n, n = -grad/|grad|.
double ref_curvature(const double* v27) {
  double v[3][3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) v[a][b][c] = v27[a + 3 * b + 9 * c];
  return fsref::Oracle<double>::curvature(v);
}

// PLIC: volume of the unit cube below m.x = a (m_i >= 0), and the plane offset
// d from the cell centre (n unit, liquid below) that cuts the fraction phi.
// The interface normal the step would use at a cell for a rule (towards the
// gas); returns 0 where there is none.
int ref_interface_normal(void* hp, int cell, int rule, double* n3) {
  auto* h = static_cast<Handle*>(hp);
  return h->sim.interface_normal(cell, rule, n3) ? 1 : 0;
}

double ref_interface_curvature(void* hp, int cell) {
  return static_cast<Handle*>(hp)->sim.interface_curvature(cell);
}

double ref_cut_volume(const double* m3, double a) { return fsref::Oracle<double>::cut_volume(m3, a); }
double ref_plic_offset(double phi, const double* n3) { return fsref::Oracle<double>::plic_offset(phi, n3); }

// Boundary value S^b = P S P + s_nn n n^T of section 3.4 (n a unit vector).
void ref_boundary_shear(const double* S6, const double* n3, double s_nn, double* Sb6) {
  fsref::Oracle<double>::boundary_shear(S6, n3, s_nn, Sb6);
}

// Closure coefficients: rule 0 = FSK row, rule 1 = Eq. (fsli) with alpha_+.
void ref_coeffs(void* hp, int rule, double alpha_p, double delta, double* out5) {
  auto& s = static_cast<Handle*>(hp)->sim;
  auto k = rule == 0 ? s.coeffs_fsk() : s.coeffs_fsli(alpha_p, delta);
  out5[0] = k.a0;
  out5[1] = k.a0bar;
  out5[2] = k.a1;
  out5[3] = k.alpha_p;
  out5[4] = k.C;
}

// Frozen-topology window with a loss and its exact directional derivative.
//
// From the state (flags, ft0, m0, phi0), T steps with conversions disabled;
// then L = sum over interface cells of |u_T - u*|^2 + (phi_T - phi*)^2, where
// u_T is recovered from the post-collision populations of time T, plus
// sum over non-gas cells and q of a_q ft_q(T) when the weights a (f_weight,
// 19 N values) are given.  The run is
// made on dual numbers, so next to L it yields dL along the input direction
// (dft0, dm0, dphi0, drho_b, dg): the exact derivative of the same arithmetic.
// Any direction pointer may be NULL (no change); with u_target and phi_target
// both NULL the interface term is left out.  out2 = {L, dL}; fT, mT, phiT
// (optional) receive the value part of the final state.  Returns 0, or 1 with
// the message in ref_create_error().
int ref_window_dual(const ref_params* rp, const uint8_t* flags, const double* ft0, const double* m0,
                    const double* phi0, const double* dft0, const double* dm0, const double* dphi0,
                    double drho_b, const double* dg, int T, int rule, const double* u_target,
                    const double* phi_target, const double* f_weight, double* out2, double* fT, double* mT,
                    double* phiT) {
  try {
    auto s = std::make_unique<Oracle<Dual>>();
    s->set_params(to_params(rp));
    // the derivative is exact for the rules without a D term and without the
    // options whose arithmetic it does not follow (the PLIC root finder) or
    // that need a wall table (solid cells)
    if (rule != fsref::FSK && rule != fsref::FSL) throw std::runtime_error("dual window: rules 0 and 1 only");
    if (s->p.plic) throw std::runtime_error("dual window: no PLIC interface position");
    if (s->p.sigma != 0.0) throw std::runtime_error("dual window: no surface tension");
    if (s->p.hold) throw std::runtime_error("dual window: no held fills");
    for (size_t i = 0; i < (size_t)s->N; ++i)
      if (flags[i] == fsref::SOLID) throw std::runtime_error("dual window: no solid cells");
    const int N = s->N;
    // seed the parameter directions: rho_b, g and the constants derived from g
    s->rho_b.d = drho_b;
    if (dg) {
      const double lm = s->lam_m.v;
      for (int a = 0; a < 3; ++a) {
        s->gvec[a].d = dg[a];
        s->half_g[a].d = 0.5 * dg[a];
        s->g_over_lam_m[a].d = dg[a] / lm;
      }
    }
    std::vector<Dual> F((size_t)fsref::Q * N), M(N), P(N);
    for (size_t i = 0; i < F.size(); ++i) F[i] = Dual(ft0[i], dft0 ? dft0[i] : 0.0);
    for (int i = 0; i < N; ++i) {
      M[i] = Dual(m0[i], dm0 ? dm0[i] : 0.0);
      P[i] = Dual(phi0[i], dphi0 ? dphi0[i] : 0.0);
    }
    s->init_from_state(flags, F.data(), M.data(), P.data(), Dual(0.0));
    s->freeze = true;
    for (int t = 0; t < T; ++t) s->step(rule);
    Dual L(0.0);
    for (int cell = 0; cell < N && u_target && phi_target; ++cell) {
      if (s->type[cell] != fsref::INTERFACE) continue;
      Dual f[fsref::Q], r, u[3];
      for (int q = 0; q < fsref::Q; ++q) f[q] = s->ft[(size_t)q * N + cell];
      s->recover_moments(f, r, u);
      for (int a = 0; a < 3; ++a) {
        const Dual e = u[a] - Dual(u_target[(size_t)a * N + cell]);
        L = L + e * e;
      }
      const Dual e = s->phi[cell] - Dual(phi_target[cell]);
      L = L + e * e;
    }
    if (f_weight) {
      for (int cell = 0; cell < N; ++cell) {
        if (s->type[cell] == fsref::GAS) continue;
        for (int q = 0; q < fsref::Q; ++q) {
          const size_t i = (size_t)q * N + cell;
          L = L + Dual(f_weight[i]) * s->ft[i];
        }
      }
    }
    out2[0] = L.v;
    out2[1] = L.d;
    if (fT)
      for (size_t i = 0; i < F.size(); ++i) fT[i] = s->ft[i].v;
    for (int i = 0; i < N; ++i) {
      if (mT) mT[i] = s->mass[i].v;
      if (phiT) phiT[i] = s->phi[i].v;
    }
    return 0;
  } catch (const std::exception& e) {
    g_create_error = e.what();
    return 1;
  }
}

}  // extern "C"
