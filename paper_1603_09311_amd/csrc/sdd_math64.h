// FP64 logarithm and sine/cosine of a full turn for the FP64 walks, on the
// arguments they take: log u and (sin 2 pi u, cos 2 pi u) for uniforms u in
// (0, 1).  Written out from their series:
//
//   log u:  u = f 2^e with f in [sqrt(1/2), sqrt(2)); log f = 2 atanh(s) with
//           s = (f - 1) / (f + 1), |s| <= 0.1716, summed to s^21 (the next
//           term is below 1e-18 of the sum); e ln 2 added with ln 2 split in
//           two parts so that e times the high part is exact.
//   sin 2 pi u, cos 2 pi u:  u = t + q / 4 with q = rint(4 u) and |t| <= 1/8
//           (t exact: Sterbenz), x = 2 pi t with 2 pi split in two parts,
//           |x| <= pi / 4; the Taylor series of sin x to x^17 and of cos x to
//           x^18 (next terms below 1e-19), then the q quarter turns.
//
// Both stay within 2 ulp of the exact values (tests/test_math64.py checks
// them against long-double references on the host).  The reduction is exact
// and each series a fixed chain of FMAs, about a third of the instructions of
// the general library routines, which handle any argument.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace sdd {

// 2 pi = kTwoPiHi + kTwoPiLo (kTwoPiHi the double nearest 2 pi); ln 2 =
// kLn2Hi + kLn2Lo with kLn2Hi rounded to 42 significant bits, so e kLn2Hi is
// exact for |e| < 2^11.
constexpr double kTwoPiHi = 0x1.921fb54442d18p+2;
constexpr double kTwoPiLo = 0x1.1a62633145c07p-52;
constexpr double kLn2Hi = 0x1.62e42fefa3800p-1;
constexpr double kLn2Lo = 0x1.ef35793c76730p-45;
constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;

// log u for u in (0, 1].
__host__ __device__ inline double log_unit64(double u) {
  int e;
  double f = frexp(u, &e);   // u = f 2^e, f in [1/2, 1)
  if (f < kSqrtHalf) {
    f = f + f;
    e -= 1;
  }
  const double s = (f - 1.0) / (f + 1.0);   // f - 1 is exact
  const double z = s * s;
  // 2 atanh(s) = 2 s + s z (2/3 + 2 z/5 + ... + 2 z^9/21)
  double p = 2.0 / 21.0;
  p = fma(p, z, 2.0 / 19.0);
  p = fma(p, z, 2.0 / 17.0);
  p = fma(p, z, 2.0 / 15.0);
  p = fma(p, z, 2.0 / 13.0);
  p = fma(p, z, 2.0 / 11.0);
  p = fma(p, z, 2.0 / 9.0);
  p = fma(p, z, 2.0 / 7.0);
  p = fma(p, z, 2.0 / 5.0);
  p = fma(p, z, 2.0 / 3.0);
  const double lf = fma(s * z, p, 2.0 * s);
  const double ed = (double)e;
  return fma(ed, kLn2Hi, fma(ed, kLn2Lo, lf));
}

// (sin 2 pi u, cos 2 pi u) for u in [0, 1].
__host__ __device__ inline void sincos_2pi64(double u, double &sn, double &cs) {
  const double qd = rint(4.0 * u);
  const double t = fma(qd, -0.25, u);                // exact
  const double x = fma(t, kTwoPiHi, t * kTwoPiLo);   // 2 pi t
  const double z = x * x;
  // sin x = x + x z (-1/3! + z/5! - ... - z^7/17!)
  double ps = -1.0 / 355687428096000.0;   // 1/17!
  ps = fma(ps, z, 1.0 / 1307674368000.0);
  ps = fma(ps, z, -1.0 / 6227020800.0);
  ps = fma(ps, z, 1.0 / 39916800.0);
  ps = fma(ps, z, -1.0 / 362880.0);
  ps = fma(ps, z, 1.0 / 5040.0);
  ps = fma(ps, z, -1.0 / 120.0);
  ps = fma(ps, z, 1.0 / 6.0);
  const double s = fma(-(x * z), ps, x);
  // cos x = 1 + z (-1/2! + z/4! - ... + z^8/18!)
  double pc = 1.0 / 6402373705728000.0;   // 1/18!
  pc = fma(pc, z, -1.0 / 20922789888000.0);
  pc = fma(pc, z, 1.0 / 87178291200.0);
  pc = fma(pc, z, -1.0 / 479001600.0);
  pc = fma(pc, z, 1.0 / 3628800.0);
  pc = fma(pc, z, -1.0 / 40320.0);
  pc = fma(pc, z, 1.0 / 720.0);
  pc = fma(pc, z, -1.0 / 24.0);
  pc = fma(pc, z, 0.5);
  const double c = fma(-z, pc, 1.0);
  // 2 pi u = x + q pi / 2
  const int q = (int)qd;
  const double a = (q & 1) ? c : s;
  const double b = (q & 1) ? s : c;
  sn = (q & 2) ? -a : a;
  cs = ((q + 1) & 2) ? -b : b;
}

}  // namespace sdd
