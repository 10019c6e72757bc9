// Internal interface between the C-ABI host code and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "fslbm_device.hpp"

namespace fslbm {

// list counters of one step (two sets, selected by step parity)
enum { C_F = 0, C_E = 1, C_EP = 2, C_NI = 3, C_NL = 4, C_I = 5, C_R = 6, NCOUNT = 8 };

struct Common {
  Grid grid;
  Consts<double> kd;
  Consts<float> kf;
  int incomp, stokes;
  float scale, inv_scale;  // FP16 storage scaling (powers of two)
  int moving;              // some wall face moves (then SweepArgs::wall_t holds the terms)
  double shear_b[6];       // prescribed S^b [xx, yy, zz, xy, xz, yz] (rules 4, 5)
  double sigma;            // surface tension coefficient (0: none)
  double rho_gas;          // gas density rho_b (actual, not in storage convention)
  int plic;                // FSL link distances from the PLIC plane instead of phi - 1/2
  int solid;               // solid cells present (SweepArgs carries their wall table)
  int surface;             // a prescribed surface plane per interface cell (SweepArgs surf_n, surf_d)
};

template <class R>
__device__ __forceinline__ const Consts<R>& pick_consts(const Common& c);
template <>
__device__ __forceinline__ const Consts<double>& pick_consts<double>(const Common& c) {
  return c.kd;
}
template <>
__device__ __forceinline__ const Consts<float>& pick_consts<float>(const Common& c) {
  return c.kf;
}

struct SweepArgs {
  Common c;
  const void* fin;
  void* fout;
  const uint8_t* flags;
  const double* mass_in;  // interface mass of time t (may equal mass)
  double* mass;           // interface mass of time t+1
  const double* phi_in;
  double* phi_out;
  // collision density and velocity of the interface cells of the step, [N][4]
  // (rho, u_x, u_y, u_z; 32 bytes per cell, one store)
  double* aux;
  int32_t* f_epoch;
  int32_t* listF;
  int32_t* listE;
  int32_t* listI;  // interface cells of time t (built by the sweep)
  int32_t* counters;
  int32_t* counters_next;
  double thr_hi, thr_lo;
  int step;
  int freeze;
  int hold;   // fill levels and interface masses held
  int cpr;   // blocks per lattice row (set by the launcher)
  // box of rows the sweep launches (box != 0): y in [by0, by0 + bny), z in
  // [bz0, bz0 + bnz); every liquid cell lies inside it.  0: every row.
  int box, by0, bny, bz0, bnz;
  int pairs; // FP16 form: two cells per lane when rows have even length
  int quad;  // interface cells of the plain step with four lanes per cell (k_iface4); 2: XCD-aware order
  // order != 0: the interface kernel runs before the sweep.  It takes the
  // list of time t that the previous step built (listI, counters[C_I]; with
  // holes where a cell has left the interface) and writes the populations of
  // t+1 of list entry i to rbuf[q * rcap + i] (i < rcap; beyond that straight
  // into fout).  The sweep then stores them with the rows it writes whole,
  // lists the interface cells of time t for the next step (counters_next,
  // islot: cell -> list entry) and leaves the counter zeroing to the
  // interface kernel.
  int order;
  int32_t* islot;
  void* rbuf;
  int rcap;
  void* u_out;  // optional (FP64 / FP32 forms): collision velocity of liquid cells, [3][N] compute type
  // optional per-step record of the interface cells (list order, capacity
  // rec_cap): pulled and own populations of time t (compute type, [Q][cap]),
  // fill and mass of time t, collision velocity ([3][cap], compute type) and
  // density of the step
  void* rec_f;
  void* rec_own;
  double* rec_phi;
  double* rec_m;
  void* rec_u;
  double* rec_rho;
  int rec_cap;
  double* kappa;  // surface tension: 3 sigma kappa per listed interface cell (list order)
  double* khf;    // surface tension with plic = 2: height-function kappa per cell (NaN: none)
  const double* wall_t;  // moving walls: [6 faces][19 links] bounce-back terms 2 w_q (c_q.u_w)/c_s^2
  // solid walls: ascending list of the non-solid cells next to a solid cell,
  // per listed cell i and link p the wall distance delta[p*nwall + i] and
  // velocity uw[(a*19 + p)*nwall + i] of the wall point x + delta c_p
  // prescribed surface: unit normal towards the gas [3][N] and plane offset
  // from the node [N] of the interface cells (caller's device memory)
  const double* surf_n;
  const double* surf_d;
  const int32_t* wcells;
  const double* wdelta;
  const double* wuw;
  int nwall;
};

struct ConvArgs {
  Common c;
  void* fout;  // populations of time t+1
  uint8_t* flags;
  double* mass;
  double* phi_out;
  double* aux;  // [N][4] as in SweepArgs
  int32_t* f_epoch;
  int32_t* new_epoch;
  int32_t* recv_epoch;
  int32_t* conv_epoch;
  int32_t *listF, *listE, *listEP, *listNI, *listNL, *listR;
  int32_t* counters;
  double* reservoir;
  int step;
  // order != 0 (SweepArgs::order): the new interface cells join the list of
  // the next step (listI, counters_next[C_I], islot)
  int order;
  int32_t* listI;
  int32_t* islot;
  int32_t* counters_next;
};

struct StepLaunch {
  SweepArgs sweep;
  ConvArgs conv;
  void* stream;
};

struct InitArgs {
  Common c;
  void* f;
  const uint8_t* flags;
  double* mass;
  double* phi;
  // collision density and velocity of the interface cells of the step, [N][4]
  // (rho, u_x, u_y, u_z; 32 bytes per cell, one store)
  double* aux;
};

struct FieldArgs {
  Common c;
  const void* f;
  const uint8_t* flags;
  const double* mass;
  const double* phi;
  const double* aux;  // [N][4] as in SweepArgs
  double* rho_out;
  double* u_out;
  double* phi_out;
  uint8_t* flags_out;
  double* f_out;
  double* mass_out;
  double* rhoc_out;
  double* uc_out;
};

struct StatArgs {
  Common c;
  const void* f;
  const uint8_t* flags;
  const double* mass;
  double* acc;    // [0] mass sum
  // [0] liquid cells, [1] cells with a NaN or non-positive density, [2]
  // interface cells, [3] unused here, [4] cells with |u| above the bound (or
  // a NaN velocity), [5] cells breaking the class rule (unknown class, or a
  // liquid cell next to a gas cell)
  int32_t* cnt;
  double u_max2;  // square of the |u| bound
};

// One reverse step t+1 -> t of a window with frozen cell classes.
struct AdjArgs {
  Common c;
  // record of the step t -> t+1 (written by the forward step)
  const void* u;          // collision velocity at liquid cells ([3][N], compute type)
  const void* rec_f;      // interface cells: pulled populations ([Q][cap], compute type)
  const void* rec_own;    // interface cells: own post-collision populations of time t
  const double* rec_phi;  // interface cells: fill of time t
  const double* rec_m;    // interface cells: mass of time t
  const void* rec_u;      // interface cells: collision velocity ([3][cap], compute type)
  const double* rec_rho;  // interface cells: collision density
  // fixed topology of the interface cells (list order)
  const uint64_t* ncls;   // class of the pull source of each link, 2 bits per link (gas, interface, liquid, wall)
  const int32_t* nslot;   // [Q][cap] list position of an interface pull source, else the cell's own
  const uint8_t* flags;   // cell classes (fixed over the window)
  const void* lam_in;     // dL/dft of time t+1 (compute type)
  void* lam_out;          // dL/dft of time t (compute type)
  double* lam_m;          // dL/dm: time t+1 on entry, time t on exit (interface cells)
  const double* lphi_in;  // dL/dphi of time t+1 (interface cells)
  double* lphi_out;       // dL/dphi of time t (interface cells)
  const int32_t* listI;   // interface cells, ascending
  const int32_t* islot;   // cell -> position in listI (interface cells only)
  void* own;              // [Q][cap] own-population adjoint terms (compute type)
  double* phic;           // [Q][cap] fill adjoint terms per pull source (0: the cell itself)
  double* part_sweep;     // [sweep wavefronts][3] dL/dg partial sums
  double* part_iface;     // [interface blocks][4] dL/drho_b, dL/dg partial sums
  int n_i, cap, cpr;
};

hipError_t launch_sweep(const StepLaunch& L, int precision, int rule);
// y and z extent of the fluid cells into ext = (ymin, ymax, zmin, zmax); (INT_MAX, -1, ...) if none
// partial extents of k_extent (ext holds (1 + EXT_COPIES) lines of 32 int32:
// the result in the first, the partials after it)
constexpr int EXT_COPIES = 64;
constexpr size_t EXT_BYTES = (size_t)(1 + EXT_COPIES) * 32 * sizeof(int32_t);
hipError_t launch_extent_init(int32_t* ext, void* stream);
hipError_t launch_extent(const uint8_t* flags, const Grid& g, int y0, int ny, int z0, int nz, int32_t* ext,
                         void* stream);
hipError_t launch_iface(const StepLaunch& L, int precision, int rule);
hipError_t launch_iface4(const StepLaunch& L, int precision, int rule);  // fslbm_iface4.hip
hipError_t launch_curvature(const StepLaunch& L);  // one or (plic = 2) two list kernels
hipError_t launch_convert(const StepLaunch& L, int precision);
// interface cells of the current classes -> list, islot, *counter (a step with
// the interface kernel first after a new state)
hipError_t launch_list_append(const uint8_t* flags, const Grid& g, int32_t* counter, int32_t* list, int32_t* islot,
                              void* stream);
hipError_t launch_fill_i32(int32_t* p, size_t n, int32_t v, void* stream);
hipError_t launch_fill_f64(double* p, size_t n, double v, void* stream);
hipError_t launch_check_flags(const uint8_t* flags, const Grid& g, int32_t* err, void* stream);
hipError_t launch_wall(const StepLaunch& L, int precision);
hipError_t launch_check_walls(const uint8_t* flags, const Grid& g, const int32_t* cells, int n, const double* delta,
                              const double* uw, int32_t* err, int32_t* count, void* stream);
hipError_t launch_set_equilibrium(const InitArgs& a, int precision, const double* rho, const double* u,
                                  const double* fill, void* stream);
hipError_t launch_set_state(const InitArgs& a, int precision, const double* f, const double* mass,
                            const double* fill, void* stream);
hipError_t launch_fields(const FieldArgs& a, int precision, void* stream);
hipError_t launch_stats(const StatArgs& a, int precision, void* stream);

// adjoint window (fslbm_adjoint.hip)
unsigned adj_sweep_blocks(const Grid& g);
unsigned adj_sweep_slots(const Grid& g);  // dL/dg partial-sum slots of the sweep (one per wavefront)
unsigned adj_iface_blocks(int n_i);
unsigned list_blocks(const Grid& g);
hipError_t launch_count_iface(const uint8_t* flags, const Grid& g, int32_t* out, void* stream);
hipError_t launch_adj_topo(const uint8_t* flags, const Grid& g, const int32_t* list, const int32_t* islot, int n_i,
                           int cap, uint64_t* ncls, int32_t* nslot, void* stream);
hipError_t launch_iface_list(const uint8_t* flags, const Grid& g, int32_t* bcount, int32_t* list, int32_t* islot,
                             int32_t* n_out, void* stream);
hipError_t launch_adj_seed(const Common& c, const uint8_t* flags, int precision, const double* dLdf,
                           const double* dLdm, const double* dLdphi, void* lam, void* lam_other, double* lam_m,
                           double* lphi, double* lphi_other, void* stream);
// one reverse step = adj_sweep (liquid cells) and adj_iface (interface cells;
// independent of adj_sweep, may run concurrently), then adj_iface2 after both
hipError_t launch_adj_sweep(const AdjArgs& a, int precision, void* stream);
hipError_t launch_adj_iface(const AdjArgs& a, int precision, int rule, void* stream);
hipError_t launch_adj_iface2(const AdjArgs& a, int precision, void* stream);
hipError_t launch_adj_out(const Common& c, const uint8_t* flags, int precision, const void* lam,
                          const double* lam_m, const double* lphi, double* dLdf, double* dLdm, double* dLdphi,
                          void* stream);
hipError_t launch_adj_reduce(const double* part_sweep, int nb_sweep, const double* part_iface, int nb_iface,
                             double* out4, void* stream);

}  // namespace fslbm
