// Internal declarations shared by the plan/ABI code and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace splitdft {

// One compiled single-pass kernel: transforms of length 2^m, 2^rb elements per
// thread, tpw transforms per workgroup, plus data-movement options.
struct Variant {
    int m;
    int rb;
    int tpw;
    int threads;  // workgroup size = tpw * 2^(m - rb)
    int lds_bytes;
    bool split;   // LDS exchange one plane at a time
    bool nt;      // nontemporal streaming loads/stores
    bool twl;     // twiddles of passes >= 1 staged in LDS
    int wpe;      // occupancy hint (minimum waves per SIMD)
    bool f4io;    // 16-byte global I/O staged through LDS
    hipError_t (*launch)(const float* xr, const float* xi, float* yr, float* yi,
                         const float2* tw, int64_t batch, hipStream_t stream);
};

// All compiled variants for length 2^m (count returned through *count).
const Variant* variants_for(int m, int* count);

// Default variant for a length and batch.
const Variant* default_variant(int m, int64_t batch);

// Host twiddle table: entry 2^(i-1)+q = (cos, sin) of 2*pi*q/2^i, FP32.
void build_twiddles_f32(int m, float* c, float* s);

}  // namespace splitdft
