// Internal declarations shared by the plan/ABI code and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/split_dft.h"

namespace splitdft {

// The message split_dft_last_error() returns on this thread.
void set_last_error(const std::string& msg);

// Planes of a second direction run in the same launch as the first (a fused
// forward + adjoint: the adjoint's planes are passed already exchanged).
struct Dir2 {
    const float* xr;
    const float* xi;
    float* yr;
    float* yi;
};

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
    int twl;      // twiddles of passes >= 1 in LDS: 0 no, 1 table slice, 2 quarter turn
    int wpe;      // occupancy hint (minimum waves per SIMD)
    int f4io;     // 16-byte global I/O staged through LDS: 0 no, 1 both ways, 2 loads
    // rows: NULL for a contiguous [batch][n] layout, else the element offset
    // of each transform (accepted when rows_ok); second: NULL, or the planes
    // of a second direction over the same rows, run in the same launch
    hipError_t (*launch)(const float* xr, const float* xi, float* yr, float* yi,
                         const float2* tw, int64_t batch, const int64_t* rows, hipStream_t stream,
                         const Dir2* second);
    bool pf = false;       // persistent workgroups, next block's loads prefetched
    bool rows_ok = false;  // takes per-transform offsets (one transform per workgroup)
};

// A two-pass schedule for large lengths: pass 1 runs stages 1..a on blocks of
// 2^a positions into a workspace, pass 2 runs stages a+1..m on columns.
struct TwoPass {
    int m;
    int a;
    int c1, c2;              // groups per workgroup in each pass
    int threads1, threads2;  // workgroup sizes
    int lds1, lds2;          // LDS bytes
    bool gf2;                // pass 2 lanes run over columns first
    // rows: NULL for contiguous transforms, else the element offset of each
    // transform in the data arrays (the workspace side is always contiguous)
    hipError_t (*pass1)(const float* xr, const float* xi, float* wr, float* wi, const float2* tw, int64_t batch,
                        const int64_t* rows, hipStream_t stream);
    hipError_t (*pass2)(const float* wr, const float* wi, float* yr, float* yi, const float2* tw, int64_t batch,
                        const int64_t* rows, hipStream_t stream);
    bool wst;  // workspace in pass-2 tile order (else natural position order)
    // both passes in one launch, the intermediate handed over through a ring of
    // `slots` transforms per XCD in the workspace (NULL: separate passes)
    hipError_t (*fused)(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                        const int64_t* rows, float* ws, hipStream_t stream) = nullptr;
    int slots = 0;
    // decimation in frequency (eq. (9)): pass 1 runs stages m..a+1 on c1
    // columns per workgroup, pass 2 stages a..1 on c2 blocks
    bool dif = false;
};

// Workspace bytes of a fused two-pass schedule (ring and control block).
size_t fused_workspace_bytes(const TwoPass* t);

// Offset in floats, modulo 32, of a plane pointer from a 128-byte line.
inline int line_offset(const float* p) { return static_cast<int>((reinterpret_cast<uintptr_t>(p) >> 2) & 31); }

// Compiled two-pass schedules for length 2^m (count returned through *count);
// dif_two_pass_for: those of the decimation-in-frequency order.
const TwoPass* two_pass_for(int m, int* count);
const TwoPass* dif_two_pass_for(int m, int* count);

// ---- grouped (ragged, mixed-length) execution --------------------------
constexpr int kManyThreads = 512;         // workgroup size of the grouped kernel
constexpr int kManyMinLog2N = 2;          // supported lengths 2^2 .. 2^16
constexpr int kManyMaxLog2N = 16;
constexpr int64_t kManyMaxN = int64_t{1} << kManyMaxLog2N;
// default mode: lengths from 2^12 up run by the per-length kernels (single
// pass to 2^14, two passes from 2^15 through chunks of at most this many
// bytes); the threshold is a plan flag, from 2^10
constexpr int kManyPerLengthLog2N = 12;
constexpr int kManyPerLengthMinLog2N = 10;
constexpr int kManyTwoPassLog2N = 15;
// (measured on the 20000-transform ragged workload: 256 MiB chunks 2.24 ms,
// 128 MiB 2.33 ms, 512 MiB 2.64 ms once the intermediate outgrows the
// memory-side cache)
constexpr int64_t kManyChunkBytes = int64_t{256} << 20;

// One unit of work: `count` transforms of length 2^m, entries [first, first +
// count) of the length-sorted transform list.
struct ManyItem {
    int32_t m;
    int32_t dir;    // index into ManyArgs' plane pointers (0 or 1)
    int32_t count;
    int32_t pad;
    int64_t first;
};

struct ManyArgs {
    const float* in_r[2];
    const float* in_i[2];
    float* out_r[2];
    float* out_i[2];
    const int64_t* offsets;  // element offset in every plane of each transform of the length-sorted list
    const ManyItem* items;
    int nitems;
    int* queue;              // [0] next item, [1] workgroups finished
    float* ws;               // per-workgroup intermediate: 2 * kManyMaxN floats each
    const float2* tw;        // twiddle table of length 2^16 (its entries serve every length)
};

// Grouped-kernel builds: 0 = 128-VGPR budget (two workgroups per CU),
// 1 = no register limit (one workgroup per CU).
constexpr int kManyKernelVariants = 2;
// large: items of length >= 2^14 may occur (the build that carries them)
hipError_t launch_many(int variant, bool large, const ManyArgs& args, int grid, hipStream_t stream);
hipError_t many_max_active_per_cu(int variant, bool large, int* blocks);
int many_items_per_group(int m);

// All compiled variants for length 2^m (count returned through *count).
const Variant* variants_for(int m, int* count);

// Compiled decimation-in-frequency (eq. 9) variants for length 2^m, m <= 13.
const Variant* dif_variants_for(int m, int* count);

// Default variant for a length and batch.
const Variant* default_variant(int m, int64_t batch);

// Host twiddle table: entry 2^(i-1)+q = (cos, sin) of 2*pi*q/2^i, FP32.
void build_twiddles_f32(int m, float* c, float* s);

// cos and sin of 2*pi*num/2^lg in FP64, exact at multiples of pi/4.
void turn_fraction_f64(int64_t num, int lg, double* c, double* s);

// Split-precision matrix-core modes (plan flag values).
constexpr int kModeFP32 = 0;
constexpr int kModeBF16X2 = 1;
constexpr int kModeFP16X2 = 2;
constexpr int kModeBF16X3 = 3;

// 32-bit words of the per-mode constant table of the length-256 matrix-core
// kernel: 2 operands x 3 parts x 64 lanes x 8 16-bit values.
constexpr int kMfmaConstFloats = 2 * 3 * 64 * 8 / 2;

// Host: constant operands of the length-256 matrix-core kernel for `mode`,
// split from FP64 into parts exactly representable in the low-precision type
// and stored as that type's 16-bit encodings, 8 per lane and (operand, part):
// entry ((mat * 3 + part) * 64 + lane) * 8 + r.
void build_mfma256_constants(int mode, uint16_t* out);

// Host: (cos, sin) of 2*pi*t/256 for t = 0..255 (exact at multiples of pi/4).
void build_tw256(float* cs);

// Launch the matrix-core kernel (only length 2^8 is supported).
hipError_t launch_mfma(int mode, int m, const float* xr, const float* xi, float* yr, float* yi, const float* consts,
                       const float2* tw256, int64_t batch, hipStream_t stream);

// ---- no-allocation entry point ------------------------------------------
// Device address and size of the static scratch array on `device` (which must
// be the current device); looked up once per device.
using ScratchLookup = hipError_t (*)(int device, float** ptr, size_t* bytes);
// Set-up: look the array up on the current device (errors are reported by the
// entry point's own lookup).
void prepare_noalloc_scratch(int device);
// split_dft_exec with two-pass intermediates in the scratch array `lookup`
// returns, in chunks that fit it; validates before any HIP call.
split_dft_status exec_in_scratch(split_dft_plan_t p, const float* xr, const float* xi, float* yr, float* yi,
                                 void* stream, ScratchLookup lookup);

}  // namespace splitdft
