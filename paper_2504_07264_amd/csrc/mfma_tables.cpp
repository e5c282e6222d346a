// Host tables of the length-256 matrix-core kernel.
//
// The kernel computes two 16-point DFTs per transform as real contractions
// with the block matrix [[C16, S16], [-S16, C16]] of eq. (5) at N = 16
// (c_kn = cos(2 pi k n / 16), s_kn = sin(2 pi k n / 16)).  Each lane of a
// wave holds, for each of two constant operands (the real and the imaginary
// output rows), 8 entries (register r of lane quarter q, index lane % 16).
// C16 and S16 are symmetric, and both contractions order K alike (slot
// (q, r) = plane r >= 4, n = 4q + (r & 3)), so the same registers are the B
// operand of the first contraction (column k1 = lane % 16) and the A operand
// of the second (row k2 = lane % 16).  The entries are formed in FP64
// and split into hi (+ lo (+ lo2)) parts exactly representable in the
// low-precision type; the FP16 lo part is scaled by 2^11.  The parts are
// stored in the type's encoding, so that each lane loads one (operand, part)
// as one 16-byte vector.
#include "internal.h"

#include <cmath>
#include <cstdint>
#include <cstring>

namespace splitdft {

namespace {

// Round to nearest (ties to even) with `bits` significand bits; the
// constants here are far from the under/overflow limits of bf16 and fp16
// (every nonzero part is a normal number of its type).
double round_bits(double v, int bits)
{
    if (v == 0.0)
        return 0.0;
    const int e = std::ilogb(v);
    const double scale = std::ldexp(1.0, bits - 1 - e);
    return std::nearbyint(v * scale) / scale;
}

// Encoding of v, exactly representable in the type: bf16 is the upper half
// of the FP32 encoding; fp16 through the compiler's conversion.
uint16_t encode(double v, int mode)
{
    if (mode == kModeFP16X2) {
        const _Float16 h = static_cast<_Float16>(static_cast<float>(v));
        uint16_t bits;
        std::memcpy(&bits, &h, sizeof bits);
        return bits;
    }
    const float f = static_cast<float>(v);
    uint32_t bits;
    std::memcpy(&bits, &f, sizeof bits);
    return static_cast<uint16_t>(bits >> 16);
}

void split(double v, int mode, uint16_t* parts)
{
    if (mode == kModeFP16X2) {
        const double h = round_bits(v, 11);
        parts[0] = encode(h, mode);
        parts[1] = encode(round_bits((v - h) * 2048.0, 11), mode);
        parts[2] = 0;
    } else {
        const double h = round_bits(v, 8);
        const double l = round_bits(v - h, 8);
        parts[0] = encode(h, mode);
        parts[1] = encode(l, mode);
        parts[2] = mode == kModeBF16X3 ? encode(round_bits(v - h - l, 8), mode) : 0;
    }
}

double cos16(int k) { double c, s; turn_fraction_f64(k & 15, 4, &c, &s); return c; }
double sin16(int k) { double c, s; turn_fraction_f64(k & 15, 4, &c, &s); return s; }

}  // namespace

void build_mfma256_constants(int mode, uint16_t* out)
{
    for (int lane = 0; lane < 64; ++lane) {
        const int q = lane >> 4, c = lane & 15;
        for (int r = 0; r < 8; ++r) {
            // slot (q, r): real part of input n = 4q + r for r < 4, imaginary
            // part of n = 4q + r - 4 for r >= 4; output index c
            const int n = 4 * q + (r & 3);
            const bool re = r < 4;
            const double er = re ? cos16(c * n) : sin16(c * n);
            const double ei = re ? -sin16(c * n) : cos16(c * n);
            const double vals[2] = {er, ei};
            for (int mat = 0; mat < 2; ++mat) {
                uint16_t parts[3];
                split(vals[mat], mode, parts);
                for (int k = 0; k < 3; ++k)
                    out[((mat * 3 + k) * 64 + lane) * 8 + r] = parts[k];
            }
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
