// HIP kernels for gfx950: the walk of (1/2) div(kappa grad u) - lambda u = 0
// (Eq. 9) when kappa and lambda are constant on each side of one vertical
// interface y = y_if (Secs. 2.2 and 3.1): walk_kappa64 in FP64 (the parity
// form) and walk_kappa32, FP32-mixed, on the same random numbers.
//
// Away from the interface the process is sqrt(kappa_i) times Brownian motion
// (Eq. 10): a step is the Euler-Maruyama proposal of Eq. (13) with kappa_i.
// The outer boundary is tested first (crossing, or the Brownian-bridge test
// of Eq. 14 with kappa_i on the nearer wall per axis).  Then the interface:
// a crossing, or a same-side bridge hit whose time t_gamma (Eq. 14, first
// case) is within the step, means the process reached it; it then resumes
// from a uniform point of a disc of radius h = sqrt(kappa_i dt) that touches
// the interface from side i (probability p_i of Eq. 12) or from side j, and
// the step's time is split between the two occupation times (Sec. 3.1, with
// the second share of a side change read as (1/2)(dt - t_gamma)(2 - p_j) so
// that the shares sum to dt).  A disc point outside the rectangle ends the
// walk at the nearest boundary point.  When kappa_0 == kappa_1 the proposal
// is kept and the step's time goes to the side of the proposal.  The record
// is g(exit) exp(-(lambda_0 T_0 + lambda_1 T_1)).
//
// Random numbers (Philox4x32-10 keyed by the seed): counter (n/2, p, j, 4s)
// gives the normals of steps n, n + 1 (words 0,1 / 2,3); (n, p, j, 4s + 1)
// the outer bridge uniforms (words 0, 1), the interface bridge uniform
// (word 2) and the side uniform (word 3); (n, p, j, 4s + 2) the disc point
// (radius word 0, angle word 1).  Uniforms are drawn only where the paper's
// tests can use them, which changes no result.
//
// Scheduling: persistent waves; a wave claims tiles of one node's paths with
// one atomic and refills every lane whose path has ended (ballot + mbcnt
// rank), so a wave never waits for its longest path.  Each path writes its
// own record: results are independent of the launch shape.
//
// Compiled with -ffp-contract=off: every operation rounds on its own, in the
// order a plain FP64 reading of the scheme evaluates it.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sdd_device.h"
#include "sdd_rng.h"

namespace sdd {
namespace {

constexpr uint32_t kKappaThreads = 256;

struct KWalker {
  double y, z;
  double T0, T1;     // occupation times of side 0 and side 1
  uint32_t n;        // steps taken
  uint64_t rec;      // record slot
  PhiloxPath pp;
};

// Where and when a path ended.
struct KExit {
  double t;          // tangential coordinate on the wall
  double tau;        // exit time
  int wall;          // 0 top, 1 right, 2 bottom, 3 left; -1 unfinished
};

// The record of a path that ended at step n: g at the exit point times
// exp(-(lambda_0 T_0 + lambda_1 T_1)).
__device__ __forceinline__ PathRec kfinish(const KReq &Q, double T0, double T1, uint32_t n, const KExit &X) {
  double gre, gim;
  g_table(Q.g, (int)Q.M, Q.y_lo, Q.y_hi, Q.z_lo, Q.z_hi, X.wall, X.t, gre, gim);
  const double er = -(Q.lre[0] * T0 + Q.lre[1] * T1);
  const double ei = -(Q.lim[0] * T0 + Q.lim[1] * T1);
  const double m = exp(er);
  const double cr = m * cos(ei), ci = m * sin(ei);
  PathRec r;
  r.w_re = gre * cr - gim * ci;
  r.w_im = gre * ci + gim * cr;
  r.tau = X.tau;
  r.steps = n + 1u;
  r.wall = X.wall;
  return r;
}

// One step with normals (n0, n1).  Returns true when the path ends at the
// boundary; where and when is then in `X`.
__device__ __forceinline__ bool kstep(const KReq &Q, KWalker &W, double n0, double n1, KExit &X) {
  const bool s1 = !(W.y < Q.y_if);                 // side of the current point
  const double kdt = s1 ? Q.kdt[1] : Q.kdt[0];
  const double s = s1 ? Q.s[1] : Q.s[0];
  const double thr = s1 ? Q.thr[1] : Q.thr[0];
  const double yn = W.y + s * n0;
  const double zn = W.z + s * n1;

  // outer boundary: nearer wall per axis (a tie goes to the lower wall)
  const double dly = W.y - Q.y_lo, dhy = Q.y_hi - W.y;
  const bool upy = !(dly <= dhy);
  const double d0y = upy ? dhy : dly;
  const double d1y = upy ? (Q.y_hi - yn) : (yn - Q.y_lo);
  const double dlz = W.z - Q.z_lo, dhz = Q.z_hi - W.z;
  const bool upz = !(dlz <= dhz);
  const double d0z = upz ? dhz : dlz;
  const double d1z = upz ? (Q.z_hi - zn) : (zn - Q.z_lo);
  const bool cy = d1y <= 0.0, cz = d1z <= 0.0;
  const double qy = (2.0 * d0y) * d1y, qz = (2.0 * d0z) * d1z;
  const bool by = !cy && (qy <= thr), bz = !cz && (qz <= thr);

  // interface candidates
  const bool sn1 = !(yn < Q.y_if);
  const bool jump = !Q.equal_kappa;
  const double e0 = fabs(W.y - Q.y_if);
  const double e1 = fabs(yn - Q.y_if);
  const bool crossed = jump && (sn1 != s1);
  const bool bridge_if = jump && !crossed && ((2.0 * e0) * e1 <= thr);

  uint4 u = make_uint4(0u, 0u, 0u, 0u);
  if (by || bz || crossed || bridge_if) {
    const uint64_t Pn = (uint64_t)kM0 * (uint64_t)W.n;
    u = philox_pp(Pn, Q.ctr3 + 1u, W.pp, Q.key0, Q.key1);
  }

  bool hy = cy, hz = cz;
  double fy = 0.0, fz = 0.0;
  if (by) {
    const double L = -log_unit64(u01_64(u.x));
    if (qy <= kdt * L) { hy = true; fy = qy / (kdt * L); }
  }
  if (bz) {
    const double L = -log_unit64(u01_64(u.y));
    if (qz <= kdt * L) { hz = true; fz = qz / (kdt * L); }
  }
  if (hy || hz) {
    if (cy) fy = d0y / (d0y - d1y);
    if (cz) fz = d0z / (d0z - d1z);
    double f;
    if (hy && (!hz || fy <= fz)) {
      f = fy;
      X.wall = upy ? 1 : 3;
      X.t = fmin(fmax(W.z + fy * (zn - W.z), Q.z_lo), Q.z_hi);
    } else {
      f = fz;
      X.wall = upz ? 2 : 0;
      X.t = fmin(fmax(W.y + fz * (yn - W.y), Q.y_lo), Q.y_hi);
    }
    const double occ = f * Q.dt;
    if (s1) W.T1 = W.T1 + occ; else W.T0 = W.T0 + occ;
    X.tau = ((double)W.n + f) * Q.dt;
    return true;
  }

  if (!jump) {                                     // equal kappa: no regime change
    if (sn1) W.T1 = W.T1 + Q.dt; else W.T0 = W.T0 + Q.dt;
    W.y = yn;
    W.z = zn;
    return false;
  }
  double tg = 0.0;
  bool reached = crossed;
  if (crossed) {
    tg = Q.dt * fabs(e0 / (yn - W.y));
  } else if (bridge_if) {
    const double ki = s1 ? Q.kappa[1] : Q.kappa[0];
    tg = ((-2.0 * e0) * e1) / (ki * log_unit64(u01_64(u.z)));
    reached = tg <= Q.dt;
  }
  if (!reached) {
    if (s1) W.T1 = W.T1 + Q.dt; else W.T0 = W.T0 + Q.dt;
    W.y = yn;
    W.z = zn;
    return false;
  }

  // resume inside a disc touching the interface from side i or side j
  const double pi = s1 ? Q.p[1] : Q.p[0];
  const double pj = 1.0 - pi;
  const double zg = W.z + (tg / Q.dt) * (zn - W.z);   // interface point
  const double towards = s1 ? -1.0 : 1.0;             // from side i towards side j
  const double half = 0.5 * (Q.dt - tg);
  double cyc, add_i, add_j;
  if (u01_64(u.w) < pi) {
    cyc = Q.y_if - towards * s;
    add_i = Q.dt - half * pi;
    add_j = half * pi;
  } else {
    cyc = Q.y_if + towards * s;
    add_i = tg + half * pj;
    add_j = half * (2.0 - pj);
  }
  W.T0 = W.T0 + (s1 ? add_j : add_i);
  W.T1 = W.T1 + (s1 ? add_i : add_j);
  const uint64_t Pn = (uint64_t)kM0 * (uint64_t)W.n;
  const uint4 d = philox_pp(Pn, Q.ctr3 + 2u, W.pp, Q.key0, Q.key1);
  const double r = s * sqrt(u01_64(d.x));
  double sth, cth;
  sincos_2pi64(u01_64(d.y), sth, cth);   // the angle 2 pi u
  const double y = cyc + r * cth;
  const double z = zg + r * sth;
  if (!(y > Q.y_lo && y < Q.y_hi && z > Q.z_lo && z < Q.z_hi)) {
    // the nearest boundary point (ties in the order left, right, top, bottom)
    const double dl = y - Q.y_lo, dr = Q.y_hi - y, dtp = z - Q.z_lo, db = Q.z_hi - z;
    double m = dl;
    int wall = 3;
    if (dr < m) { m = dr; wall = 1; }
    if (dtp < m) { m = dtp; wall = 0; }
    if (db < m) { m = db; wall = 2; }
    const double yy = fmin(fmax(y, Q.y_lo), Q.y_hi), zz = fmin(fmax(z, Q.z_lo), Q.z_hi);
    X.wall = wall;
    X.t = (wall == 0 || wall == 2) ? yy : zz;
    X.tau = ((double)W.n + 1.0) * Q.dt;
    return true;
  }
  W.y = y;
  W.z = z;
  return false;
}


// ---------------------------------------------------------------------------
// FP32-mixed walk: positions relative to the domain centre in FP32, the
// hardware log2, sqrt, sin and cos (angles in revolutions), the same random
// numbers as the FP64 walk (so the two are paired); full steps counted per
// side in integers, the interface shares and the exit fraction of the
// occupation times summed in FP64, the weight in FP64.
// ---------------------------------------------------------------------------
struct KWalker32 {
  float a, b;        // y - ymid, z - zmid
  float m;           // kdist32 of (a, b)
  uint32_t c0, c1;   // full steps on side 0 / side 1
  double f0, f1;     // the rest of the occupation times (interface shares, exit fraction)
  uint32_t n;
  uint64_t rec;
  PhiloxPath pp;
};

__device__ __forceinline__ float one_frac_k(uint32_t w) {
  return __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, w, 9u));
}
// (2 (w >> 9) + 1) 2^-24, exact, in (0, 1)
__device__ __forceinline__ float u01_k(uint32_t w) { return one_frac_k(w) - 0x1.fffffep-1f; }
// -ln u
__device__ __forceinline__ float neglog_k(uint32_t w) {
  return -0.69314718055994531f * __builtin_amdgcn_logf(u01_k(w));
}

// The per-side FP32 constants of the walk in scalar registers: a choice
// between two fields of the request by the lane's side is otherwise compiled
// to a per-lane load from the request.
__device__ __forceinline__ float uni_f(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
struct KSide32 {
  float K[2], thr[2], kdt[2], kappa[2], p[2], s[2], r[2];
  __device__ __forceinline__ void load(const KReq &Q) {
    for (int i = 0; i < 2; ++i) {
      K[i] = uni_f(Q.fK[i]);
      thr[i] = uni_f(Q.fthr[i]);
      // the least float r with fl(2 r r) > thr: two distances above r give a
      // rounded product 2 d0 d1 above thr (rounding is monotone)
      float rr = __builtin_sqrtf(0.5f * thr[i]);
      while (rr > 0.f && (2.f * rr) * rr > thr[i]) rr = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, rr) - 1u);
      while (!((2.f * rr) * rr > thr[i])) rr = __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, rr) + 1u);
      r[i] = uni_f(rr);
      kdt[i] = uni_f(Q.fkdt[i]);
      kappa[i] = uni_f(Q.fkappa[i]);
      p[i] = uni_f(Q.fp[i]);
      s[i] = uni_f(Q.fs[i]);
    }
  }
};

__device__ __forceinline__ bool kstep32(const KReq &Q, const KSide32 &S, KWalker32 &W, uint32_t wa, uint32_t wb,
                                        KExit &X) {
  const bool s1 = !(W.a < Q.fa_if);
  const float K = s1 ? S.K[1] : S.K[0];
  const float thr = s1 ? S.thr[1] : S.thr[0];
  const float rk = K * __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u01_k(wa)));
  const float ang = one_frac_k(wb);
  const float an = __builtin_fmaf(__builtin_amdgcn_cosf(ang), rk, W.a);
  const float bn = __builtin_fmaf(__builtin_amdgcn_sinf(ang), rk, W.b);

  // outer boundary: nearer wall per axis (a tie goes to the lower wall)
  const bool upy = W.a > 0.f, upz = W.b > 0.f;
  const float d0y = Q.fhy - fabsf(W.a), d0z = Q.fhz - fabsf(W.b);
  const float d1y = upy ? (Q.fhy - an) : (Q.fhy + an);
  const float d1z = upz ? (Q.fhz - bn) : (Q.fhz + bn);
  const bool cy = d1y <= 0.f, cz = d1z <= 0.f;
  const float qy = (2.f * d0y) * d1y, qz = (2.f * d0z) * d1z;
  const bool by = !cy && (qy <= thr), bz = !cz && (qz <= thr);

  // interface candidates
  const bool sn1 = !(an < Q.fa_if);
  const bool jump = !Q.equal_kappa;
  const float e0 = fabsf(W.a - Q.fa_if), e1 = fabsf(an - Q.fa_if);
  const bool crossed = jump && (sn1 != s1);
  const bool bridge_if = jump && !crossed && ((2.f * e0) * e1 <= thr);

  uint4 u = make_uint4(0u, 0u, 0u, 0u);
  if (by || bz || crossed || bridge_if) {
    const uint64_t Pn = (uint64_t)kM0 * (uint64_t)W.n;
    u = philox_pp(Pn, Q.ctr3 + 1u, W.pp, Q.key0, Q.key1);
  }
  const float kdt = s1 ? S.kdt[1] : S.kdt[0];
  bool hy = cy, hz = cz;
  float fy = 0.f, fz = 0.f;
  if (by) {
    const float L = kdt * neglog_k(u.x);
    if (qy <= L) { hy = true; fy = qy * __builtin_amdgcn_rcpf(L); }
  }
  if (bz) {
    const float L = kdt * neglog_k(u.y);
    if (qz <= L) { hz = true; fz = qz * __builtin_amdgcn_rcpf(L); }
  }
  if (hy || hz) {
    if (cy) fy = d0y * __builtin_amdgcn_rcpf(d0y - d1y);
    if (cz) fz = d0z * __builtin_amdgcn_rcpf(d0z - d1z);
    float f, t;
    if (hy && (!hz || fy <= fz)) {
      f = fminf(fy, 1.f);
      X.wall = upy ? 1 : 3;
      t = fminf(fmaxf(__builtin_fmaf(f, bn - W.b, W.b), -Q.fhz), Q.fhz);
      X.t = (double)t + Q.zmid;
    } else {
      f = fminf(fz, 1.f);
      X.wall = upz ? 2 : 0;
      t = fminf(fmaxf(__builtin_fmaf(f, an - W.a, W.a), -Q.fhy), Q.fhy);
      X.t = (double)t + Q.ymid;
    }
    const double occ = (double)f * Q.dt;
    if (s1) W.f1 += occ; else W.f0 += occ;
    X.tau = ((double)W.n + (double)f) * Q.dt;
    return true;
  }

  if (!jump) {                                     // equal kappa: no regime change
    if (sn1) W.c1 += 1u; else W.c0 += 1u;
    W.a = an;
    W.b = bn;
    return false;
  }
  float tg = 0.f;
  bool reached = crossed;
  if (crossed) {
    tg = Q.fdt * (e0 * __builtin_amdgcn_rcpf(fabsf(an - W.a)));
  } else if (bridge_if) {
    const float ki = s1 ? S.kappa[1] : S.kappa[0];
    tg = ((2.f * e0) * e1) * __builtin_amdgcn_rcpf(ki * neglog_k(u.z));
    reached = tg <= Q.fdt;
  }
  if (!reached) {
    if (s1) W.c1 += 1u; else W.c0 += 1u;
    W.a = an;
    W.b = bn;
    return false;
  }

  // resume inside a disc touching the interface from side i or side j
  const float pi = s1 ? S.p[1] : S.p[0];
  const float h = s1 ? S.s[1] : S.s[0];
  const float zg = __builtin_fmaf(fminf(tg * Q.frdt, 1.f), bn - W.b, W.b);   // interface point
  const float towards = s1 ? -1.f : 1.f;
  const double half = 0.5 * (Q.dt - (double)tg);
  float cyc;
  double add_i, add_j;
  if (u01_k(u.w) < pi) {
    cyc = Q.fa_if - towards * h;
    add_i = Q.dt - half * (double)pi;
    add_j = half * (double)pi;
  } else {
    const double pj = 1.0 - (double)pi;
    cyc = Q.fa_if + towards * h;
    add_i = (double)tg + half * pj;
    add_j = half * (2.0 - pj);
  }
  W.f0 += s1 ? add_j : add_i;
  W.f1 += s1 ? add_i : add_j;
  const uint64_t Pn = (uint64_t)kM0 * (uint64_t)W.n;
  const uint4 d = philox_pp(Pn, Q.ctr3 + 2u, W.pp, Q.key0, Q.key1);
  const float r = h * __builtin_amdgcn_sqrtf(u01_k(d.x));
  const float th = one_frac_k(d.y);
  const float a = __builtin_fmaf(__builtin_amdgcn_cosf(th), r, cyc);
  const float bb = __builtin_fmaf(__builtin_amdgcn_sinf(th), r, zg);
  if (!(fabsf(a) < Q.fhy && fabsf(bb) < Q.fhz)) {
    // the nearest boundary point (ties in the order left, right, top, bottom)
    const float dl = Q.fhy + a, dr = Q.fhy - a, dtp = Q.fhz + bb, db = Q.fhz - bb;
    float m = dl;
    int wall = 3;
    if (dr < m) { m = dr; wall = 1; }
    if (dtp < m) { m = dtp; wall = 0; }
    if (db < m) { m = db; wall = 2; }
    const float yy = fminf(fmaxf(a, -Q.fhy), Q.fhy), zz = fminf(fmaxf(bb, -Q.fhz), Q.fhz);
    X.wall = wall;
    X.t = (wall == 0 || wall == 2) ? (double)yy + Q.ymid : (double)zz + Q.zmid;
    X.tau = ((double)W.n + 1.0) * Q.dt;
    return true;
  }
  W.a = a;
  W.b = bb;
  return false;
}

// The least distance of (a, b) to the outer boundary and (kappa jumping) to
// the interface.
__device__ __forceinline__ float kdist32(const KReq &Q, float a, float b) {
  const float e = Q.equal_kappa ? __builtin_inff() : fabsf(a - Q.fa_if);
  return fminf(fminf(Q.fhy - fabsf(a), Q.fhz - fabsf(b)), e);
}

// kstep32 for a step that none of its tests flags: the same proposal, then
// a screen that passes only steps kstep32 would not flag (no crossing of the
// interface, and the start and the proposal both farther than r from the
// outer boundary and the interface: each distance kstep32 takes is at least
// the one here, so every product 2 d0 d1 it forms rounds above thr and no
// distance is <= 0), the move and the count of the step's side (with a jump
// in kappa the proposal stayed on the start's side).  Returns false, leaving
// W as it was, for any other step; kstep32 on the same words then takes it.
__device__ __forceinline__ bool kstep32_plain(const KReq &Q, const KSide32 &S, KWalker32 &W, uint32_t wa, uint32_t wb) {
  const bool s1 = !(W.a < Q.fa_if);
  const float K = s1 ? S.K[1] : S.K[0];
  const float r = s1 ? S.r[1] : S.r[0];
  const float rk = K * __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u01_k(wa)));
  const float ang = one_frac_k(wb);
  const float an = __builtin_fmaf(__builtin_amdgcn_cosf(ang), rk, W.a);
  const float bn = __builtin_fmaf(__builtin_amdgcn_sinf(ang), rk, W.b);
  const float m1 = kdist32(Q, an, bn);
  const bool sn1 = !(an < Q.fa_if);
  const bool crossed = !Q.equal_kappa && (sn1 != s1);
  if (!(fminf(W.m, m1) > r) || crossed) return false;
  if (sn1) W.c1 += 1u; else W.c0 += 1u;
  W.a = an;
  W.b = bn;
  W.m = m1;
  return true;
}

// Lanes whose step is flagged park it until the wave runs the full step
// logic for all parked lanes at once: when kParkLanes lanes are parked,
// kParkIters iterations after a lane first parked, or when no lane is left
// that can step.  Near the interface a few lanes of a wave are flagged in
// most steps; run step by step, every flagged step would cost the wave the
// whole branch (a second Philox call, a bridge, a resume).  A record depends
// only on its path's random numbers, so parking changes when a step runs,
// not what it computes.
constexpr uint32_t kParkLanes = 24;
constexpr uint32_t kParkIters = 8;

struct K32 {
  using Walker = KWalker32;
  static __device__ __forceinline__ void start(const KReq &Q, Walker &W, double2 xy, uint32_t p, uint32_t node,
                                               uint64_t rec, uint32_t k0) {
    W.a = (float)(xy.x - Q.ymid);
    W.b = (float)(xy.y - Q.zmid);
    W.m = kdist32(Q, W.a, W.b);
    W.c0 = 0u;
    W.c1 = 0u;
    W.f0 = 0.0;
    W.f1 = 0.0;
    W.n = 0u;
    W.rec = rec;
    W.pp = philox_path(p, node, k0);
  }
  static __device__ __forceinline__ PathRec finish(const KReq &Q, const Walker &W, const KExit &X) {
    const double T0 = Q.dt * (double)W.c0 + W.f0;
    const double T1 = Q.dt * (double)W.c1 + W.f1;
    return kfinish(Q, T0, T1, W.n, X);
  }
};

// The two walks keep separate kernels, so that each gets the register
// allocation of its own step; the FP32-mixed one parks flagged steps.
__global__ void __launch_bounds__(kKappaThreads) walk_kappa32(const KReq *__restrict__ qp) {
  using T = K32;
  const KReq &Q = *qp;
  KSide32 S;
  S.load(Q);
  const uint32_t lane = __lane_id();
  typename T::Walker W;
  bool active = false;
  bool exhausted = false;
  bool parked = false;
  uint32_t wz = 0, ww = 0;   // words of the odd step of the walker's current pair
  uint32_t pa = 0, pb = 0;   // words of the parked step
  uint32_t waited = 0;       // iterations the parked lanes have waited (wave-uniform)
  // wave-uniform tile cursor
  uint32_t t_node = 0, t_p0 = 0, t_next = 0, t_end = 0;
  uint64_t t_rec0 = 0;

  for (;;) {
    const uint64_t freemask = __builtin_amdgcn_ballot_w64(!active);
    if (freemask != 0ull && !exhausted) {
      const uint32_t nfree = (uint32_t)__popcll(freemask);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(freemask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)freemask, 0u));
      uint32_t given = 0;
      while (given < nfree) {
        if (t_next == t_end) {
          uint32_t t = 0;
          if (lane == 0) t = atomicAdd(Q.tile_counter, 1u);
          t = uni(t);
          if (t >= Q.n_tiles) { exhausted = true; break; }
          const DevTile Tl = Q.tiles[t];
          t_node = uni(Tl.node);
          t_p0 = uni(Tl.p0);
          t_next = t_p0;
          t_end = t_p0 + uni(Tl.count);
          t_rec0 = ((uint64_t)uni((uint32_t)(Tl.rec0 >> 32)) << 32) | uni((uint32_t)Tl.rec0);
        }
        const uint32_t take = min(t_end - t_next, nfree - given);
        if (!active && rank >= given && rank < given + take) {
          const uint32_t p = t_next + (rank - given);
          const double2 xy = *reinterpret_cast<const double2 *>(Q.nodes + 2 * (size_t)t_node);
          T::start(Q, W, xy, p, t_node, t_rec0 + (p - t_p0), Q.key0);
          active = true;
        }
        t_next += take;
        given += take;
      }
    }
    if (__builtin_amdgcn_ballot_w64(!active) == ~0ull) break;   // no work left for this wave

    // flagged steps first, every parked lane at once; a walker whose parked
    // step was even then takes the odd one below in the same iteration, so
    // the walkers of a wave stay at one parity
    int st = 0;   // 0 running, 1 exited (X), 2 step cap
    KExit X;
    X.wall = -1;
    const uint64_t pmask = __builtin_amdgcn_ballot_w64(parked);
    if (pmask != 0ull) {
      waited += 1u;
      const bool stuck = __builtin_amdgcn_ballot_w64(active && !parked) == 0ull;
      if ((uint32_t)__popcll(pmask) >= kParkLanes || waited >= kParkIters || stuck) {
        waited = 0;
        if (parked) {
          parked = false;
          if (kstep32(Q, S, W, pa, pb, X)) {
            st = 1;
          } else {
            W.m = kdist32(Q, W.a, W.b);
            W.n += 1u;
            if (W.n >= Q.max_steps) st = 2;
          }
        }
      }
    }
    // unflagged steps: two per normal draw (steps 2k and 2k + 1 take words
    // 0, 1 and 2, 3 of the draw at 2k)
    if (active && !parked && st == 0) {
      if ((W.n & 1u) == 0u) {
        const uint64_t P = (uint64_t)kM0 * (uint64_t)(W.n >> 1);
        const uint4 w = philox_pp(P, Q.ctr3, W.pp, Q.key0, Q.key1);
        wz = w.z;
        ww = w.w;
        if (kstep32_plain(Q, S, W, w.x, w.y)) {
          W.n += 1u;
          if (W.n >= Q.max_steps) st = 2;
        } else {
          parked = true;
          pa = w.x;
          pb = w.y;
        }
      }
      if (st == 0 && !parked) {
        if (kstep32_plain(Q, S, W, wz, ww)) {
          W.n += 1u;
          if (W.n >= Q.max_steps) st = 2;
        } else {
          parked = true;
          pa = wz;
          pb = ww;
        }
      }
    }
    if (st != 0) {
      PathRec r;
      if (st == 1) {
        r = T::finish(Q, W, X);
      } else {   // step cap: max_steps steps drawn
        r.w_re = 0.0;
        r.w_im = 0.0;
        r.tau = -1.0;
        r.steps = W.n;
        r.wall = -1;
      }
      Q.recs[W.rec] = r;
      active = false;
    }
  }
}

__global__ void __launch_bounds__(kKappaThreads) walk_kappa64(const KReq *__restrict__ qp) {
  const KReq &Q = *qp;
  const uint32_t lane = __lane_id();
  KWalker W;
  bool active = false;
  bool exhausted = false;
  // wave-uniform tile cursor
  uint32_t t_node = 0, t_p0 = 0, t_next = 0, t_end = 0;
  uint64_t t_rec0 = 0;

  for (;;) {
    const uint64_t freemask = __builtin_amdgcn_ballot_w64(!active);
    if (freemask != 0ull && !exhausted) {
      const uint32_t nfree = (uint32_t)__popcll(freemask);
      const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(freemask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)freemask, 0u));
      uint32_t given = 0;
      while (given < nfree) {
        if (t_next == t_end) {
          uint32_t t = 0;
          if (lane == 0) t = atomicAdd(Q.tile_counter, 1u);
          t = uni(t);
          if (t >= Q.n_tiles) { exhausted = true; break; }
          const DevTile Tl = Q.tiles[t];
          t_node = uni(Tl.node);
          t_p0 = uni(Tl.p0);
          t_next = t_p0;
          t_end = t_p0 + uni(Tl.count);
          t_rec0 = ((uint64_t)uni((uint32_t)(Tl.rec0 >> 32)) << 32) | uni((uint32_t)Tl.rec0);
        }
        const uint32_t take = min(t_end - t_next, nfree - given);
        if (!active && rank >= given && rank < given + take) {
          const uint32_t p = t_next + (rank - given);
          const double2 xy = *reinterpret_cast<const double2 *>(Q.nodes + 2 * (size_t)t_node);
          W.y = xy.x;
          W.z = xy.y;
          W.T0 = 0.0;
          W.T1 = 0.0;
          W.n = 0u;
          W.rec = t_rec0 + (p - t_p0);
          W.pp = philox_path(p, t_node, Q.key0);
          active = true;
        }
        t_next += take;
        given += take;
      }
    }
    if (__builtin_amdgcn_ballot_w64(!active) == ~0ull) break;   // no work left for this wave

    if (active) {
      // two steps per normal draw; a walker is at an even step here
      const uint64_t P = (uint64_t)kM0 * (uint64_t)(W.n >> 1);
      const uint4 w = philox_pp(P, Q.ctr3, W.pp, Q.key0, Q.key1);
      double a0, a1, b0, b1;
      normals64(w.x, w.y, a0, a1);
      normals64(w.z, w.w, b0, b1);
      KExit X;
      X.wall = -1;
      bool end = kstep(Q, W, a0, a1, X);
      if (!end) {
        W.n += 1u;
        end = W.n >= Q.max_steps;
        if (!end) {
          end = kstep(Q, W, b0, b1, X);
          if (!end) {
            W.n += 1u;
            end = W.n >= Q.max_steps;
          }
        }
      }
      if (end) {
        PathRec r;
        if (X.wall >= 0) {
          r = kfinish(Q, W.T0, W.T1, W.n, X);
        } else {   // step cap: W.n == max_steps steps drawn
          r.w_re = 0.0;
          r.w_im = 0.0;
          r.tau = -1.0;
          r.steps = W.n;
          r.wall = -1;
        }
        Q.recs[W.rec] = r;
        active = false;
      }
    }
  }
}

}  // namespace

hipError_t launch_walk_kappa(int precision, const KReq *req_dev, uint32_t blocks, hipStream_t st) {
  if (blocks == 0) return hipSuccess;
  if (precision == 1) hipLaunchKernelGGL(walk_kappa32, dim3(blocks), dim3(kKappaThreads), 0, st, req_dev);
  else hipLaunchKernelGGL(walk_kappa64, dim3(blocks), dim3(kKappaThreads), 0, st, req_dev);
  return hipGetLastError();
}

int kappa_blocks_per_cu(int precision) {
  int nb = 0;
  const hipError_t e = precision == 1
      ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kappa32, (int)kKappaThreads, 0)
      : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, walk_kappa64, (int)kKappaThreads, 0);
  return e == hipSuccess ? nb : 0;
}

uint32_t kappa_threads() { return kKappaThreads; }

}  // namespace sdd
