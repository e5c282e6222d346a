// Host-side twiddle table for the plans.
//
// The factor D^(i) of eq. (6) (Section III) rotates by the 2x2 blocks
// omega^(i,q) = [[cos a, sin a], [-sin a, cos a]], a = 2*pi*q / 2^i.  The
// table keeps (cos a, sin a) at entry 2^(i-1) + q for stages i = 1..m, and
// the angle 0 at entry 0.
//
// Values are computed in FP64 and rounded to nearest FP32.  So that 0, +-1
// and the equality cos = sin at odd multiples of pi/4 come out exact, the
// angle fraction q / 2^i is split into a whole number of quarter turns and a
// remainder in (-1/8, 1/8] of a turn: libm evaluates cos and sin only of the
// remainder angle |phi| = pi * |r| / (2 * 2^i) (|phi| <= pi/4, with
// |phi| = pi/4 given the value sqrt(1/2) for both), and the quarter turns are
// applied by exchanging and negating.  Negative zeros become +0.
#include "internal.h"

#include <cmath>

namespace splitdft {

namespace {

struct CosSin {
    double c, s;
};

// cos and sin of 2*pi * num / 2^lg, exact at multiples of pi/4.
CosSin turn_fraction(int64_t num, int lg)
{
    const int64_t den = int64_t{1} << lg;
    // 4*num = quarters * den + rem, with rem moved into (-den/2, den/2].
    num &= den - 1;  // whole turns
    int64_t quarters = (num * 4) / den;
    int64_t rem = (num * 4) - quarters * den;
    if (rem * 2 > den) {
        rem -= den;
        quarters += 1;
    }
    const int64_t mag = rem < 0 ? -rem : rem;
    double lc, ls;
    if (mag * 2 == den) {
        lc = std::sqrt(0.5);
        ls = lc;
    } else {
        const double phi = (M_PI * static_cast<double>(mag)) / (2.0 * static_cast<double>(den));
        lc = std::cos(phi);
        ls = std::sin(phi);
    }
    if (rem < 0)
        ls = -ls;
    CosSin out{};
    switch (quarters & 3) {
    case 0: out = {lc, ls}; break;       // a = phi
    case 1: out = {-ls, lc}; break;      // a = phi + pi/2
    case 2: out = {-lc, -ls}; break;     // a = phi + pi
    default: out = {ls, -lc}; break;     // a = phi + 3pi/2
    }
    out.c += 0.0;
    out.s += 0.0;
    return out;
}

}  // namespace

void turn_fraction_f64(int64_t num, int lg, double* c, double* s)
{
    const CosSin v = turn_fraction(num, lg);
    *c = v.c;
    *s = v.s;
}

void build_twiddles_f32(int m, float* c, float* s)
{
    c[0] = 1.0f;
    s[0] = 0.0f;
    for (int i = 1; i <= m; ++i) {
        const int64_t r = int64_t{1} << (i - 1);
        for (int64_t q = 0; q < r; ++q) {
            const CosSin v = turn_fraction(q, i);
            c[r + q] = static_cast<float>(v.c) + 0.0f;
            s[r + q] = static_cast<float>(v.s) + 0.0f;
        }
    }
}

}  // namespace splitdft
