"""The colatitude cosine of the device pixel code (cos_0pi in csrc/common.h),
compiled for the host from the same source lines and measured against
80-bit long-double cos: within one ulp on [0, pi], which is what the pixel
parity checks assume (a device pixel may differ from the oracle's only where
cos theta lies within one ulp of a pixel edge).

The functions are plain IEEE double arithmetic with explicit fma and no
contraction, so the host build evaluates exactly what the device evaluates.
"""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COMMON = os.path.join(ROOT, "paper_2603_19600_amd", "csrc", "common.h")

HARNESS = r"""
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <random>
#define __device__
#define __forceinline__ inline
using std::fma;
%(FUNCS)s
static double ulp_err(double got, long double ref) {
  const double r = (double)ref;
  const double u = std::nextafter(std::fabs(r), INFINITY) - std::fabs(r);
  return (double)(std::fabs((long double)got - ref) / (long double)u);
}
int main() {
  double worst = 0.0, at = 0.0;
  auto check = [&](double t) {
    const double e = ulp_err(cos_0pi(t), cosl((long double)t));
    if (e > worst) { worst = e; at = t; }
  };
  // every FP32 angle in [0, pi] on a stride (about 4e6 of them), every FP32
  // angle around the sub-range edges pi/4, pi/2 and 3 pi/4 and the ends
  const float top = 3.14159250f;   // the largest float below pi
  uint32_t hi; std::memcpy(&hi, &top, 4);
  for (uint32_t b = 0; b <= hi; b += 257) { float f; std::memcpy(&f, &b, 4); check(f); }
  for (double c : {0.0, 0.7853981633974483, 1.5707963267948966, 2.356194490192345,
                   3.141592653589793}) {
    float f = (float)c;
    uint32_t b; std::memcpy(&b, &f, 4);
    for (int d = -20000; d <= 20000; ++d) {
      const int64_t bb = (int64_t)b + d;
      if (bb < 0 || bb > (int64_t)hi) continue;
      const uint32_t u = (uint32_t)bb; float g; std::memcpy(&g, &u, 4); check(g);
    }
  }
  // FP64 angles: uniform, and packed near 0, pi/2 and pi
  std::mt19937_64 rng(7);
  std::uniform_real_distribution<double> U(0.0, 3.141592653589793);
  for (int i = 0; i < 2000000; ++i) {
    double t = U(rng);
    if (i %% 4 == 1) t = 1.5707963267948966 + (U(rng) - 1.5707963267948966) * 1e-9;
    if (i %% 4 == 2) t = U(rng) * 1e-4;
    if (i %% 4 == 3) t = 3.141592653589793 - U(rng) * 1e-4;
    check(t);
  }
  std::printf("%%.6f %%.17g %%.17g %%.17g %%.17g\n", worst, at, cos_0pi(0.0),
              cos_0pi(3.141592653589793), cos_0pi(1.5707963267948966));
  return 0;
}
"""


def _functions():
    src = open(COMMON).read()
    start = src.index("__device__ __forceinline__ double sin_kernel(")
    end = src.index("// Ring pixel of (theta, phi)")
    funcs = src[start:end]
    assert "cos_0pi" in funcs and "cos_kernel" in funcs
    return funcs


@pytest.fixture(scope="module")
def result():
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "cos_check.cpp")
        exe = os.path.join(d, "cos_check")
        with open(src, "w") as fh:
            fh.write(HARNESS % {"FUNCS": _functions()})
        subprocess.run([cxx, "-O2", "-std=c++17", "-ffp-contract=off", src, "-o", exe],
                       check=True, capture_output=True, text=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    worst, at, c0, cpi, cpio2 = (float(x) for x in out.split())
    return worst, at, c0, cpi, cpio2


def test_cos_0pi_is_within_one_ulp(result):
    worst, at, _, _, _ = result
    assert worst < 1.0, f"{worst} ulp at theta = {at!r}"


def test_cos_0pi_special_values(result):
    _, _, c0, cpi, cpio2 = result
    assert c0 == 1.0 and cpi == -1.0
    # cos(RN(pi/2)) = pi/2 - RN(pi/2) to first order: the tail of pi/2
    assert cpio2 == pytest.approx(6.123233995736766e-17, rel=1e-15)


def test_the_extracted_source_is_the_device_source():
    funcs = _functions()
    assert re.search(r"__device__ __forceinline__ double cos_0pi\(double t\)", funcs)
    assert "pix_of_z(n, cos_0pi(theta), phi)" in open(COMMON).read()
