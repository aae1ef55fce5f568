"""The kernels' attenuation factors (vrc_math.h), built for the host, against long-double references.

g = exp(-x) and em = 1 - exp(-x) come from one Cody-Waite reduction and a
Taylor polynomial; here both are compared with x87 long-double expl/expm1l
over optical thicknesses from 1e-12 to the cut-off, in ulps of the working
precision.  (FMA, ldexp and rint round the same on the host and the GPU.)
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1706_07476_amd", "csrc")

SRC = r"""
#include <cstdio>
#include <cmath>
#include <cfloat>
#include <random>
#include "vrc_math.h"

template <typename R> long double ulp_of(long double v) {
    int e; std::frexp((double)v, &e);
    const int mant = std::is_same<R, float>::value ? 24 : 53;
    return std::ldexp(1.0L, e - mant);
}

template <typename R> void run(const char *name, R xmax) {
    std::mt19937_64 rng(12345);
    long double worst_g = 0, worst_em = 0;
    R at_g = 0, at_em = 0;
    const int N = 2000000;
    for (int i = 0; i < N; ++i) {
        R x;
        if (i < N / 2) {
            std::uniform_real_distribution<double> d(-12.0, std::log10((double)xmax));
            x = (R)std::pow(10.0, d(rng));
        } else {
            std::uniform_real_distribution<double> d(0.0, 3.0);
            x = (R)d(rng);
        }
        R g, em;
        vrc::attenuation(x, g, em);
        long double xg = (long double)x;
        long double rg = std::exp(-xg), rem = -std::expm1(-xg);
        long double eg = std::fabs((long double)g - rg) / ulp_of<R>(rg);
        long double eem = std::fabs((long double)em - rem) / ulp_of<R>(rem);
        if (eg > worst_g) { worst_g = eg; at_g = x; }
        if (eem > worst_em) { worst_em = eem; at_em = x; }
    }
    // special values
    R g, em;
    vrc::attenuation((R)0, g, em);
    int zero_ok = (g == 1 && em == 0);
    vrc::attenuation(xmax * 2, g, em);
    int big_ok = (g == 0 && em == 1);
    vrc::attenuation((R)NAN, g, em);
    int nan_ok = (g == 0 && em == 1);
    std::printf("%s %.3Lf %.9g %.3Lf %.9g %d %d %d\n", name, worst_g, (double)at_g, worst_em, (double)at_em,
                zero_ok, big_ok, nan_ok);
}

int main() {
    run<double>("f64", 708.0);
    run<float>("f32", 87.0f);
    return 0;
}
"""


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    d = tmp_path_factory.mktemp("vrcmath")
    src = d / "t.cpp"
    src.write_text(SRC)
    exe = d / "t"
    subprocess.run(["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-I", HDR, "-o", str(exe), str(src)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.strip().splitlines():
        name, wg, xg, wem, xem, z, b, n = line.split()
        res[name] = dict(worst_g=float(wg), at_g=float(xg), worst_em=float(wem), at_em=float(xem),
                         zero=z == "1", big=b == "1", nan=n == "1")
    return res


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_attenuation_factors_within_a_few_ulp(results, prec):
    r = results[prec]
    assert r["worst_g"] <= 4.0, r
    assert r["worst_em"] <= 4.0, r


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_attenuation_special_values(results, prec):
    r = results[prec]
    assert r["zero"] and r["big"] and r["nan"], r
