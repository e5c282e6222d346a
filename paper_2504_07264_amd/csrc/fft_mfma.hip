// Split-format FFT of length 256 with the two 16-point sub-DFT stages on the
// matrix cores (gfx950 v_mfma_f32_16x16x32_{bf16,f16}), split precision.
//
// Grouping of the factors of eq. (6) (Section III) for N = 256 = 16 * 16:
// after the bit reversal, stages 1..4 act within blocks of 16 consecutive
// positions: block n0 holds x[16*n1 + n0] (n1 = 0..15) and the four stages
// produce its 16-point DFT X_n0[k1] = sum_n1 x[16 n1 + n0] W16^(n1 k1).
// Stages 5..8 act on the positions k1 + 16*a; their product is the twiddle
// W256^(n0 k1) followed by a 16-point DFT over n0:
//     y[k1 + 16 k2] = sum_n0 W16^(n0 k2) * (W256^(n0 k1) X_n0[k1]).
// Each 16-point DFT is the real block matrix of eq. (5) at N = 16,
// [[C16, S16], [-S16, C16]], applied as a dense contraction with K = 32
// (16 real + 16 imaginary inputs): exactly the case where the stage is a
// contraction.
//
// One wave computes TPI transforms per iteration; rows are loaded with
// 16-byte vectors into wave-private LDS, and each transform goes through:
//   step 1  D = A * B, A = data (row n0 = lane % 16, K = (plane, n1)),
//           B = [C; S] or [-S; C] (K x k1), giving X[n0][k1];
//   step 2  X[n0][k1] *= W256^(n0 k1) in FP32 (VALU);
//   step 3  D = A3 * B3, A3 = constant (row k2, K = (plane, n0)), B3 = the
//           twiddled X exactly as step 1 left it in the accumulator layout
//           (lane holds n0 = 4*(lane/16) + r, k1 = lane % 16 for r < 4), so
//           no data moves between lanes.
// The K order is the same slot (lane quarter q, register r) in both
// operands of each product, so it only needs to be consistent, not equal to
// any particular hardware order.
//
// Split precision (FP32 accumulate): each operand v = hi + lo (+ lo2) in the
// low-precision type; products are summed smallest first:
//   BF16X2: lo*hi + hi*lo + hi*hi                     (3 MFMAs per product)
//   BF16X3: lo2*hi + hi*lo2 + lo*lo + lo*hi + hi*lo + hi*hi  (6 MFMAs)
//   FP16X2: lo parts scaled by 2^11 (kept normal), accumulated separately
//           and scaled back: hi*hi + 2^-11 (lo*hi + hi*lo)   (3 MFMAs)
// The constant matrices are split on the host from FP64 values.
#include "internal.h"

#include <atomic>
#include <climits>

namespace splitdft {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
struct Prec;

template <>
struct Prec<kModeBF16X2> {
    using V = bf16x8;
    static constexpr int PARTS = 2;
};
template <>
struct Prec<kModeBF16X3> {
    using V = bf16x8;
    static constexpr int PARTS = 3;
};
template <>
struct Prec<kModeFP16X2> {
    using V = f16x8;
    static constexpr int PARTS = 2;
};

__device__ __forceinline__ f32x4 mma(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mma(f16x8 a, f16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Split 8 floats into the parts of MODE.
template <int MODE>
__device__ __forceinline__ void split8(const float (&v)[8], typename Prec<MODE>::V (&p)[Prec<MODE>::PARTS])
{
    if constexpr (MODE == kModeFP16X2) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const _Float16 h = static_cast<_Float16>(v[r]);
            p[0][r] = h;
            p[1][r] = static_cast<_Float16>((v[r] - static_cast<float>(h)) * 2048.0f);
        }
    } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const __bf16 h = static_cast<__bf16>(v[r]);
            const float rest = v[r] - static_cast<float>(h);
            const __bf16 l = static_cast<__bf16>(rest);
            p[0][r] = h;
            p[1][r] = l;
            if constexpr (Prec<MODE>::PARTS == 3)
                p[2][r] = static_cast<__bf16>(rest - static_cast<float>(l));
        }
    }
}

// A * B with split operands, FP32 accumulate.
template <int MODE>
__device__ __forceinline__ f32x4 product(const typename Prec<MODE>::V (&a)[Prec<MODE>::PARTS],
                                         const typename Prec<MODE>::V (&b)[Prec<MODE>::PARTS])
{
    const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (MODE == kModeBF16X2) {
        f32x4 acc = mma(a[1], b[0], z);
        acc = mma(a[0], b[1], acc);
        return mma(a[0], b[0], acc);
    } else if constexpr (MODE == kModeBF16X3) {
        f32x4 acc = mma(a[2], b[0], z);
        acc = mma(a[0], b[2], acc);
        acc = mma(a[1], b[1], acc);
        acc = mma(a[1], b[0], acc);
        acc = mma(a[0], b[1], acc);
        return mma(a[0], b[0], acc);
    } else {
        f32x4 corr = mma(a[1], b[0], z);
        corr = mma(a[0], b[1], corr);
        const f32x4 main = mma(a[0], b[0], z);
        f32x4 out;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            out[r] = __builtin_fmaf(corr[r], 1.0f / 2048.0f, main[r]);
        return out;
    }
}

template <int MODE>
__device__ __forceinline__ void load_const(const float* tab, int mat, int lane,
                                           typename Prec<MODE>::V (&p)[Prec<MODE>::PARTS])
{
    const float* src = tab + ((mat * 64 + lane) * 8) * 3;
#pragma unroll
    for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int k = 0; k < Prec<MODE>::PARTS; ++k) {
            if constexpr (MODE == kModeFP16X2)
                p[k][r] = static_cast<_Float16>(src[r * 3 + k]);
            else
                p[k][r] = static_cast<__bf16>(src[r * 3 + k]);
        }
}

constexpr int kWaves = 4;
// LDS words of one staged plane: 256 floats with 16 pad words after each 128,
// so the operand reads of lane quarters 0/1 (and 2/3) fall on different banks.
constexpr int kPlaneWords = 256 + 32;
__device__ __forceinline__ int pad256(int n) { return n + 16 * (n >> 7); }

typedef float v4f __attribute__((ext_vector_type(4)));

// Orders a wave's own LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 16-byte loads of the TPI rows from b0 (zeros past the batch).
template <int TPI>
__device__ __forceinline__ void load_rows(v4f (&in)[TPI][2], const float* xr, const float* xi, int64_t b0,
                                          int64_t batch, int lane)
{
#pragma unroll
    for (int t = 0; t < TPI; ++t) {
        if (b0 + t < batch) {
            in[t][0] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xr + (b0 + t) * 256) + lane);
            in[t][1] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xi + (b0 + t) * 256) + lane);
        } else {
            in[t][0] = in[t][1] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
}

// TPI transforms per wave iteration; rows are staged through wave-private
// LDS so that global loads and stores are 16-byte and fully coalesced.
template <int MODE, int TPI>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(Prec<MODE>::PARTS == 2 ? 4 : 3)))
split_fft256_mfma_kernel(const float* xr, const float* xi, float* yr, float* yi, const float* __restrict__ consts,
                         const float2* __restrict__ tw256, int64_t batch)
{
    using P = Prec<MODE>;
    using V = typename P::V;
    __shared__ __attribute__((aligned(16))) float lds[kWaves * TPI * 2 * kPlaneWords];
    const int lane = threadIdx.x & 63;
    const int q = lane >> 4;
    const int c = lane & 15;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * kWaves + (threadIdx.x >> 6);
    const int64_t nwaves = static_cast<int64_t>(gridDim.x) * kWaves;
    float* my = lds + (threadIdx.x >> 6) * (TPI * 2 * kPlaneWords);

    V b1r[P::PARTS], b1i[P::PARTS], a3r[P::PARTS], a3i[P::PARTS];
    load_const<MODE>(consts, 0, lane, b1r);
    load_const<MODE>(consts, 1, lane, b1i);
    load_const<MODE>(consts, 2, lane, a3r);
    load_const<MODE>(consts, 3, lane, a3i);
    float2 w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        w[r] = tw256[((4 * q + r) * c) & 255];

    // step-1 operand: lane (q, c) reads plane q >> 1 at n = 16 * (8 (q & 1) + r) + c
    const int a_off = (q >> 1) * kPlaneWords + pad256(128 * (q & 1) + c);
    // the grid is resident: each wave loops with a stride and issues the
    // next rows' loads before the current rows' arithmetic
    v4f in[TPI][2];
    if (wave * TPI < batch)
        load_rows<TPI>(in, xr, xi, wave * TPI, batch, lane);
    for (int64_t b0 = wave * TPI; b0 < batch; b0 += nwaves * TPI) {
#pragma unroll
        for (int t = 0; t < TPI; ++t)
#pragma unroll
            for (int p = 0; p < 2; ++p)
                *reinterpret_cast<v4f*>(my + (2 * t + p) * kPlaneWords + pad256(4 * lane)) = in[t][p];
        wave_lds_sync();
        if (b0 + nwaves * TPI < batch)
            load_rows<TPI>(in, xr, xi, b0 + nwaves * TPI, batch, lane);
#pragma unroll
        for (int t = 0; t < TPI; ++t) {
            const float* src = my + 2 * t * kPlaneWords + a_off;
            float v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                v[r] = src[16 * r];
            V a[P::PARTS];
            split8<MODE>(v, a);
            const f32x4 xr4 = product<MODE>(a, b1r);
            const f32x4 xi4 = product<MODE>(a, b1i);
            // twiddle W256^(n0 k1), n0 = 4q + r, k1 = c; B3 slot r < 4 real, r >= 4 imaginary
            float z[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                z[r] = __builtin_fmaf(w[r].x, xr4[r], w[r].y * xi4[r]);
                z[r + 4] = __builtin_fmaf(w[r].x, xi4[r], -(w[r].y * xr4[r]));
            }
            V b3[P::PARTS];
            split8<MODE>(z, b3);
            const f32x4 yr4 = product<MODE>(a3r, b3);
            const f32x4 yi4 = product<MODE>(a3i, b3);
            // lane holds k2 = 4q + r, k1 = c: output index k1 + 16 k2 (the
            // transform's operand reads above are complete: the MFMAs used them)
            float* dr = my + 2 * t * kPlaneWords;
            float* di = dr + kPlaneWords;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dr[pad256(c + 16 * (4 * q + r))] = yr4[r];
                di[pad256(c + 16 * (4 * q + r))] = yi4[r];
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < TPI; ++t) {
            if (b0 + t < batch) {
                const v4f o_r = *reinterpret_cast<const v4f*>(my + 2 * t * kPlaneWords + pad256(4 * lane));
                const v4f o_i = *reinterpret_cast<const v4f*>(my + (2 * t + 1) * kPlaneWords + pad256(4 * lane));
                __builtin_nontemporal_store(o_r, reinterpret_cast<v4f*>(yr + (b0 + t) * 256) + lane);
                __builtin_nontemporal_store(o_i, reinterpret_cast<v4f*>(yi + (b0 + t) * 256) + lane);
            }
        }
        // the next iteration's staging writes reuse this wave's LDS
        wave_lds_sync();
    }
}

constexpr int kMaxDevices = 64;

template <int MODE>
hipError_t launch_mfma256(const float* xr, const float* xi, float* yr, float* yi, const float* consts,
                          const float2* tw256, int64_t batch, hipStream_t stream)
{
    constexpr int TPI = 4;
    auto kernel = split_fft256_mfma_kernel<MODE, TPI>;
    // as many workgroups as can be resident (looked up once per device)
    static std::atomic<int> resident_of[kMaxDevices];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    int resident = (dev >= 0 && dev < kMaxDevices) ? resident_of[dev].load(std::memory_order_relaxed) : 0;
    if (resident <= 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64 * kWaves, 0);
        if (e != hipSuccess)
            return e;
        if (per_cu < 1 || cus < 1)
            return hipErrorInvalidConfiguration;
        resident = cus * per_cu;
        if (dev >= 0 && dev < kMaxDevices)
            resident_of[dev].store(resident, std::memory_order_relaxed);
    }
    const int64_t per_block = kWaves * TPI;
    const int64_t blocks = (batch + per_block - 1) / per_block;
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(grid)), dim3(64 * kWaves), 0, stream, xr, xi, yr, yi, consts,
                       tw256, batch);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_mfma(int mode, int m, const float* xr, const float* xi, float* yr, float* yi, const float* consts,
                       const float2* tw256, int64_t batch, hipStream_t stream)
{
    if (m != 8)
        return hipErrorInvalidValue;
    switch (mode) {
    case kModeBF16X2: return launch_mfma256<kModeBF16X2>(xr, xi, yr, yi, consts, tw256, batch, stream);
    case kModeFP16X2: return launch_mfma256<kModeFP16X2>(xr, xi, yr, yi, consts, tw256, batch, stream);
    case kModeBF16X3: return launch_mfma256<kModeBF16X3>(xr, xi, yr, yi, consts, tw256, batch, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace splitdft
