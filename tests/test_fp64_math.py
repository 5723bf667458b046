"""Host-side accuracy of the library's double-precision logarithm, sine/cosine
of 2 pi u and square root (gmf_math.hpp), which replace the generic device
math in the FP64 Box-Muller transform (the host path refines single-precision
estimates where the device refines its v_rcp_f64 / v_rsq_f64 estimates).  The header compiles for the host; the errors
are measured against long-double libm on every argument form the kernel can
produce, and the constants are regenerated from their definitions."""
import os
import subprocess
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2601_03806_amd", "csrc")

DRIVER = r"""
#include "gmf_math.hpp"
#include <cmath>
#include <cstdio>
#include <random>
int main() {
    std::mt19937_64 g(12345);
    const long double pil = 3.14159265358979323846264338327950288L;
    double maxlog = 0, maxs = 0, maxc = 0, maxsq = 0;
    for (long i = 0; i < 2000000; ++i) {
        uint32_t x = (uint32_t)(i < 4096 ? (i < 2048 ? i : 0xFFFFFFFFu - (uint32_t)(i - 2048)) : g());
        double u = ((double)x + 0.5) * 0x1p-32;
        long double ref = logl((long double)u);
        double got = gmf::fp64::log_unit(u);
        double ulp = nextafter(fabs((double)ref), INFINITY) - fabs((double)ref);
        maxlog = fmax(maxlog, fabs((double)((long double)got - ref)) / ulp);
        double s, c;
        gmf::fp64::sincos_2pi(u, &s, &c);
        long double a = 2 * pil * (long double)u;
        maxs = fmax(maxs, fabs((double)((long double)s - sinl(a))));
        maxc = fmax(maxc, fabs((double)((long double)c - cosl(a))));
        // the Box-Muller radius: sqrt of x = -2 ln u in [2^-32, 46]
        double xr = -2.0 * got;
        long double rs = sqrtl((long double)xr);
        double sq = gmf::fp64::sqrt_pos(xr);
        double ulq = nextafter((double)rs, INFINITY) - (double)rs;
        maxsq = fmax(maxsq, fabs((double)((long double)sq - rs)) / ulq);
    }
    printf("%.6e %.6e %.6e %.6e\n", maxlog, maxs, maxc, maxsq);
    return 0;
}
"""


def test_log_and_sincos_accuracy(tmp_path):
    src = tmp_path / "drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    subprocess.run(["g++", "-O2", "-ffp-contract=off", f"-I{CSRC}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    max_log_ulp, max_sin, max_cos, max_sqrt_ulp = map(float, out)
    assert max_log_ulp <= 2.0, max_log_ulp
    assert max_sin <= 2.5e-16 and max_cos <= 2.5e-16, (max_sin, max_cos)
    assert max_sqrt_ulp <= 1.0, max_sqrt_ulp


def test_constants_match_generator():
    gen = subprocess.run([sys.executable, os.path.join(CSRC, "gen_fp64_coeffs.py")], capture_output=True, text=True,
                         check=True).stdout
    header = open(os.path.join(CSRC, "gmf_math.hpp")).read()
    for line in gen.splitlines():
        if line.startswith("constexpr"):
            name_values = line.split("=", 1)[1].strip()
            assert name_values in header, line
