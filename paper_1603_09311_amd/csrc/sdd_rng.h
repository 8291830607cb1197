// Device helpers shared by the walk kernels: Philox4x32-10 with per-path
// precomputed rounds, wave-uniform broadcasts, FP64 uniforms and normals, and
// the boundary tables' interpolation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdd_math64.h"

namespace sdd {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): ten rounds of two 32x32->64-bit
// products with a Weyl key schedule (the key is wave-uniform, so the
// schedule runs on the scalar unit).  Each output word's double XOR is one
// gfx950 three-input bit operation (truth table 0x96 = a ^ b ^ c).
// ---------------------------------------------------------------------------
constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                             uint32_t k1) {
  const uint64_t p0 = (uint64_t)kM0 * (uint64_t)c0;
  const uint64_t p1 = (uint64_t)kM1 * (uint64_t)c2;
  const uint32_t n0 = xor3((uint32_t)(p1 >> 32), c1, k0);
  const uint32_t n2 = xor3((uint32_t)(p0 >> 32), c3, k1);
  c1 = (uint32_t)p1;
  c3 = (uint32_t)p0;
  c0 = n0;
  c2 = n2;
}

// Every counter this walk uses has the form (c0, path, node, c3): words 1 and
// 2 are fixed for a path.  Round 1 then depends on c0 only through M0*c0, and
// round 2 multiplies a word that is fixed for the path; both products are made
// once per path.
struct PhiloxPath {
  uint32_t x1;   // lo(M1 node)             (round-1 output word 1)
  uint32_t hb;   // hi(M0 x0), x0 = hi(M1 node) ^ path ^ k0 (round-1 word 0)
  uint32_t lb;   // lo(M0 x0)
};

__device__ __forceinline__ PhiloxPath philox_path(uint32_t path, uint32_t node, uint32_t k0) {
  const uint64_t A = (uint64_t)kM1 * (uint64_t)node;
  const uint32_t x0 = xor3((uint32_t)(A >> 32), path, k0);
  const uint64_t B = (uint64_t)kM0 * (uint64_t)x0;
  PhiloxPath pp;
  pp.x1 = (uint32_t)A;
  pp.hb = (uint32_t)(B >> 32);
  pp.lb = (uint32_t)B;
  return pp;
}

// Philox4x32-10 of the counter (c0, path, node, c3) given P0 = M0 * c0.
__device__ __forceinline__ uint4 philox_pp(uint64_t P0, uint32_t c3, const PhiloxPath &pp, uint32_t k0,
                                           uint32_t k1) {
  // round 1 gives (x0, x1, hi(P0) ^ c3 ^ k1, lo(P0)); round 2 (key + W).
  // c3 ^ k1 is wave-uniform: one scalar XOR, then one vector XOR.
  const uint32_t r1w2 = (uint32_t)(P0 >> 32) ^ (c3 ^ k1);
  const uint32_t r1w3 = (uint32_t)P0;
  const uint64_t p1 = (uint64_t)kM1 * (uint64_t)r1w2;
  uint32_t w0 = xor3((uint32_t)(p1 >> 32), pp.x1, k0 + kW0);
  uint32_t w1 = (uint32_t)p1;
  uint32_t w2 = xor3(pp.hb, r1w3, k1 + kW1);
  uint32_t w3 = pp.lb;
#pragma unroll
  for (uint32_t r = 2; r < 10; ++r) philox_round(w0, w1, w2, w3, k0 + r * kW0, k1 + r * kW1);
  return make_uint4(w0, w1, w2, w3);
}

// ---------------------------------------------------------------------------
// Wave-uniform broadcasts.
// ---------------------------------------------------------------------------
// readfirstlane returns a signed int: every use goes through uint32_t so no
// value is ever sign-extended when widened.
__device__ __forceinline__ uint32_t uni(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float unif(float v) { return __builtin_bit_cast(float, uni(__builtin_bit_cast(uint32_t, v))); }
__device__ __forceinline__ double unid(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint64_t r = ((uint64_t)uni((uint32_t)(u >> 32)) << 32) | (uint64_t)uni((uint32_t)u);
  return __builtin_bit_cast(double, r);
}

// ---------------------------------------------------------------------------
// FP64 uniforms in (0, 1) and Box-Muller normals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double u01_64(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

__device__ __forceinline__ void normals64(uint32_t a, uint32_t b, double &n0, double &n1) {
  const double r = sqrt(-2.0 * log_unit64(u01_64(a)));
  double sn, cs;
  sincos_2pi64(u01_64(b), sn, cs);   // the angle 2 pi u, both from one reduction
  n0 = r * cs;
  n1 = r * sn;
}

// g at the tangential coordinate t of wall `wall` (0 top, 1 right, 2 bottom,
// 3 left): the wall's table, linear between its M + 1 equispaced samples.
__device__ __forceinline__ void g_table(const double *g, int M, double y_lo, double y_hi, double z_lo, double z_hi,
                                        int wall, double t, double &gre, double &gim) {
  const bool along_y = (wall == 0) || (wall == 2);
  const double t0 = along_y ? y_lo : z_lo;
  const double t1 = along_y ? y_hi : z_hi;
  const double h = (t1 - t0) / (double)M;
  const double u = (t - t0) / h;
  int i = (int)floor(u);
  i = i < 0 ? 0 : i;
  i = i > M - 1 ? M - 1 : i;
  const double lam = u - (double)i;
  const double *gw = g + (size_t)wall * (size_t)(M + 1) * 2;
  const double2 ga = *reinterpret_cast<const double2 *>(gw + 2 * i);
  const double2 gb = *reinterpret_cast<const double2 *>(gw + 2 * i + 2);
  gre = (1.0 - lam) * ga.x + lam * gb.x;
  gim = (1.0 - lam) * ga.y + lam * gb.y;
}

}  // namespace sdd
