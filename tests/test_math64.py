"""The FP64 walks' logarithm and full-turn sine/cosine (csrc/sdd_math64.h)
against long-double references, on the host: every uniform the walks form,
u = (w + 1/2) / 2^32, for 2^21 seeded 32-bit words w, the ends of the range
and the words next to each eighth of a turn (where the reduction changes
quarter or the series reaches its widest argument).  The sine and cosine
references take the nearest quarter turn off u exactly in long double before
sinl/cosl, so that near the functions' zeros the reference is accurate
relative to the value.  Bar: 2 ulp of the double nearest the reference.
CPU only (the header is compiled as host code)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1603_09311_amd", "csrc")

HARNESS = r"""
#include <cmath>
#include <cstdint>
#include <cstdio>
#include "sdd_math64.h"

static double ulp_of(long double r) {
  const double d = std::fabs((double)r);
  return std::nextafter(d, INFINITY) - d;
}

int main() {
  const long double two_pi = 6.283185307179586476925286766559005768394L;
  double worst_log = 0, worst_sin = 0, worst_cos = 0;
  uint64_t x = 0x9E3779B97F4A7C15ull;
  auto check = [&](uint32_t w) {
    const double u = ((double)w + 0.5) * (1.0 / 4294967296.0);
    const double l = sdd::log_unit64(u);
    const long double lr = logl((long double)u);
    worst_log = std::fmax(worst_log, (double)(fabsl((long double)l - lr) / ulp_of(lr)));
    double s, c;
    sdd::sincos_2pi64(u, s, c);
    // reference: the nearest quarter turn taken off exactly in long double,
    // so that the long-double product's rounding stays relative to the
    // values near their zeros
    const long double k = rintl(4.0L * (long double)u);
    const long double a = two_pi * ((long double)u - k / 4.0L);
    const int q = (int)k;
    const long double s0 = sinl(a), c0 = cosl(a);
    const long double sa = (q & 1) ? c0 : s0, ca = (q & 1) ? s0 : c0;
    const long double sr = (q & 2) ? -sa : sa;
    const long double cr = ((q + 1) & 2) ? -ca : ca;
    worst_sin = std::fmax(worst_sin, (double)(fabsl((long double)s - sr) / ulp_of(sr)));
    worst_cos = std::fmax(worst_cos, (double)(fabsl((long double)c - cr) / ulp_of(cr)));
  };
  for (int i = 0; i < (1 << 21); ++i) {   // xorshift64*
    x ^= x >> 12; x ^= x << 25; x ^= x >> 27;
    check((uint32_t)((x * 0x2545F4914F6CDD1Dull) >> 32));
  }
  const uint32_t ends[] = {0u, 1u, 2u, 3u, 0xFFFFFFFFu, 0xFFFFFFFEu, 0x7FFFFFFFu, 0x80000000u};
  for (uint32_t w : ends) check(w);
  for (uint64_t k = 1; k < 8; ++k)
    for (int d = -64; d <= 64; ++d) check((uint32_t)((k << 29) + (int64_t)d));
  std::printf("%.4f %.4f %.4f\n", worst_log, worst_sin, worst_cos);
  return 0;
}
"""


@pytest.fixture(scope="module")
def worst(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    d = tmp_path_factory.mktemp("math64")
    src = d / "harness.hip"
    src.write_text(HARNESS)
    exe = d / "harness"
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-ffp-contract=off", "-w",
                        "-I", CSRC, str(src), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    return [float(v) for v in out]


def test_log_within_two_ulp(worst):
    assert worst[0] <= 2.0, worst


def test_sin_cos_within_two_ulp(worst):
    assert worst[1] <= 2.0 and worst[2] <= 2.0, worst
