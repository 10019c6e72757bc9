// Quads of lanes working on one interface cell (the forward and adjoint
// interface kernels): DPP exchanges inside a quad and the pair layout of the
// D3Q19 links over its four lanes.
#pragma once

#include "fslbm_device.hpp"

namespace fslbm {

// quad_perm DPP controls: lanes (1,0,3,2) and (2,3,0,1) of each quad
constexpr int QP_XOR1 = 0xB1;
constexpr int QP_XOR2 = 0x4E;

template <int CTRL>
__device__ __forceinline__ uint32_t qperm(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double qperm(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint64_t r = (uint64_t)qperm<CTRL>((uint32_t)b) | ((uint64_t)qperm<CTRL>((uint32_t)(b >> 32)) << 32);
  return __longlong_as_double((long long)r);
}
template <int CTRL>
__device__ __forceinline__ float qperm(float v) {
  return __uint_as_float(qperm<CTRL>(__float_as_uint(v)));
}
// (v0 + v1) + (v2 + v3) in every lane of the quad (addition is commutative in
// IEEE arithmetic, so the four lanes agree bit for bit); the whole quad must be
// active
template <class T>
__device__ __forceinline__ T quad_sum(T v) {
  v = v + qperm<QP_XOR1>(v);
  return v + qperm<QP_XOR2>(v);
}

// broadcast of lane L of each quad to all four lanes (quad_perm [L, L, L, L])
template <int L, class T>
__device__ __forceinline__ T qbcast(T v) {
  return qperm<L * 0x55>(v);
}

constexpr int QUAD = 4;
constexpr int PAIRS = 9;

// direction of the odd link 2p + 1 of every pair p, 6 bits per pair
constexpr uint64_t pack_pair_dirs() {
  uint64_t c = 0;
  for (int p = 0; p < PAIRS; ++p) {
    const int q = 2 * p + 1;
    c |= (uint64_t)((CX[q] + 1) | ((CY[q] + 1) << 2) | ((CZ[q] + 1) << 4)) << (6 * p);
  }
  return c;
}
constexpr uint64_t PAIR_DIRS = pack_pair_dirs();
static_assert(WD[1] == WD[6] && WD[7] == WD[18], "axis and diagonal weights");

__device__ __forceinline__ void pair_dir(int p, int (&d)[3]) {
  const unsigned c = (unsigned)(PAIR_DIRS >> (6 * p)) & 63u;
  d[0] = (int)(c & 3u) - 1;
  d[1] = (int)((c >> 2) & 3u) - 1;
  d[2] = (int)(c >> 4) - 1;
}

// d . v for a direction with components in {-1, 0, 1}
template <class R>
__device__ __forceinline__ R ddot(const R (&d)[3], const R (&v)[3]) {
  return (d[0] * v[0] + d[1] * v[1]) + d[2] * v[2];
}
__device__ __forceinline__ double ddot(const int (&d)[3], const double (&v)[3]) {
  return ((double)d[0] * v[0] + (double)d[1] * v[1]) + (double)d[2] * v[2];
}

}  // namespace fslbm
