// Host tables of the length-256 matrix-core kernel.
//
// The kernel computes two 16-point DFTs per transform as real contractions
// with the block matrix [[C16, S16], [-S16, C16]] of eq. (5) at N = 16
// (c_kn = cos(2 pi k n / 16), s_kn = sin(2 pi k n / 16)).  Each lane of a
// wave holds, for each of four constant operands, 8 entries (register r of
// lane quarter q, column or row lane % 16).  The entries are formed in FP64
// and split into hi (+ lo (+ lo2)) parts exactly representable in the
// low-precision type; the FP16 lo part is scaled by 2^11.
#include "internal.h"

#include <cmath>

namespace splitdft {

namespace {

// Round to nearest (ties to even) with `bits` significand bits; the
// constants here are far from the under/overflow limits of bf16 and fp16.
double round_bits(double v, int bits)
{
    if (v == 0.0)
        return 0.0;
    const int e = std::ilogb(v);
    const double scale = std::ldexp(1.0, bits - 1 - e);
    return std::nearbyint(v * scale) / scale;
}

void split(double v, int mode, float* parts)
{
    if (mode == kModeFP16X2) {
        const double h = round_bits(v, 11);
        parts[0] = static_cast<float>(h);
        parts[1] = static_cast<float>(round_bits((v - h) * 2048.0, 11));
        parts[2] = 0.0f;
    } else {
        const double h = round_bits(v, 8);
        const double l = round_bits(v - h, 8);
        parts[0] = static_cast<float>(h);
        parts[1] = static_cast<float>(l);
        parts[2] = mode == kModeBF16X3 ? static_cast<float>(round_bits(v - h - l, 8)) : 0.0f;
    }
}

double cos16(int k) { double c, s; turn_fraction_f64(k & 15, 4, &c, &s); return c; }
double sin16(int k) { double c, s; turn_fraction_f64(k & 15, 4, &c, &s); return s; }

}  // namespace

void build_mfma256_constants(int mode, float* out)
{
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, c = lane & 15;
        for (int r = 0; r < 8; ++r) {
            // step 1, B operand: slot (q, r) = plane q >> 1, n1 = 8 (q & 1) + r; column k1 = c
            const int n1 = 8 * (q & 1) + r;
            const bool re = (q >> 1) == 0;
            const double b1r = re ? cos16(n1 * c) : sin16(n1 * c);
            const double b1i = re ? -sin16(n1 * c) : cos16(n1 * c);
            // step 3, A operand: row k2 = c; slot (q, r) = real n0 = 4q + r for r < 4,
            // imaginary n0 = 4q + r - 4 for r >= 4
            const int n0 = 4 * q + (r & 3);
            const bool re3 = r < 4;
            const double a3r = re3 ? cos16(c * n0) : sin16(c * n0);
            const double a3i = re3 ? -sin16(c * n0) : cos16(c * n0);
            const double vals[4] = {b1r, b1i, a3r, a3i};
            for (int mat = 0; mat < 4; ++mat)
                split(vals[mat], mode, out + ((mat * 64 + lane) * 8 + r) * 3);
        }
    }
}

void build_tw256(float* cs)
{
    for (int t = 0; t < 256; ++t) {
        double c, s;
        turn_fraction_f64(t, 8, &c, &s);
        cs[2 * t] = static_cast<float>(c) + 0.0f;
        cs[2 * t + 1] = static_cast<float>(s) + 0.0f;
    }
}

}  // namespace splitdft
