"""The library's double-precision Box-Muller pieces (csrc/bm_math.h: ln of
(v / 2^32) and cos of the double product 2pi * w / 2^32 with exact argument
reduction), compiled for the host and checked against the C library: within
two double ulp on random and edge words, and the fp32 weights they give equal
the library-function formula on every sampled word (including the words
around the zeros of the cosine, with mean-zero weights)."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HEADER = os.path.join(HERE, "..", "paper_2512_09502_amd", "csrc", "bm_math.h")

SRC = r'''
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <random>
#include "HEADER"
using namespace snnc;
static double ulps(double a, double b) {
    if (a == b) return 0;
    return std::fabs(a - b) / std::fabs(std::nextafter(b, INFINITY) - b);
}
static int64_t ordf(float f) { int32_t i; std::memcpy(&i, &f, 4); return i < 0 ? -(int64_t)(i & 0x7fffffff) : i; }
static float wref(uint32_t w0, uint32_t w1, double mean, double sd) {
    volatile double r = std::sqrt(-2.0 * std::log(((double)w0 + 1.0) * (1.0 / 4294967296.0)));
    volatile double z = r * std::cos(6.283185307179586 * ((double)w1 * (1.0 / 4294967296.0)));
    volatile double s = sd * z;
    return (float)(mean + s);
}
static float wlib(uint32_t w0, uint32_t w1, double mean, double sd) {
    volatile double r = std::sqrt(-2.0 * log_u32_frac((uint64_t)w0 + 1));
    volatile double z = r * cos_2pi_u32(w1);
    volatile double s = sd * z;
    return (float)(mean + s);
}
int main() {
    std::mt19937_64 rng(7);
    double mlog = 0, mcos = 0;
    auto check = [&](uint32_t w) {
        mlog = std::fmax(mlog, ulps(log_u32_frac((uint64_t)w + 1), std::log(((double)w + 1.0) / 4294967296.0)));
        mcos = std::fmax(mcos, ulps(cos_2pi_u32(w), std::cos(6.283185307179586 * ((double)w / 4294967296.0))));
    };
    for (long i = 0; i < 2000000; ++i) check((uint32_t)rng());
    for (uint32_t c : {0u, 0x20000000u, 0x40000000u, 0x60000000u, 0x80000000u, 0xa0000000u, 0xc0000000u, 0xe0000000u})
        for (int k = -300; k <= 300; ++k) check(c + (uint32_t)k);
    check(0xffffffffu);
    long diff = 0;
    const double ms[][2] = {{0.1, 0.01}, {-0.5, 0.05}, {0.0, 1.0}, {100.0, 10.0}};
    for (const auto& p : ms)
        for (long i = 0; i < 1000000; ++i) {
            const uint64_t r = rng();
            if (ordf(wlib((uint32_t)r, (uint32_t)(r >> 32), p[0], p[1])) != ordf(wref((uint32_t)r, (uint32_t)(r >> 32), p[0], p[1]))) ++diff;
        }
    for (uint32_t c : {0x40000000u, 0xc0000000u})
        for (int k = -2000; k <= 2000; ++k)
            for (uint32_t w0 : {0u, 99u, 0x80000000u, 0xfffffff0u, 0xffffffffu})
                if (ordf(wlib(w0, c + (uint32_t)k, 0.0, 1.0)) != ordf(wref(w0, c + (uint32_t)k, 0.0, 1.0))) ++diff;
    std::printf("%.3f %.3f %ld\n", mlog, mcos, diff);
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_box_muller_pieces_match_the_c_library():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        open(src, "w").write(SRC.replace("HEADER", os.path.abspath(HEADER)))
        exe = os.path.join(d, "t")
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-o", exe, src, "-lm"])
        out = subprocess.check_output([exe], timeout=120).decode().split()
    max_log_ulp, max_cos_ulp, weight_diffs = float(out[0]), float(out[1]), int(out[2])
    assert max_log_ulp <= 2.0
    assert max_cos_ulp <= 2.0
    assert weight_diffs == 0
