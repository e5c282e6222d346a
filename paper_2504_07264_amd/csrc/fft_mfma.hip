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
// any particular hardware order.  Step 3's order is fixed by the accumulator
// layout (slot (q, r) = plane r >= 4, index 4q + (r & 3)); step 1 reads its
// data in the same order, and as C16 and S16 are symmetric, A3 is then, lane
// by lane and register by register, the step-1 B operand: one set of
// constant registers serves both steps.
//
// Split precision (FP32 accumulate): each operand v = hi + lo (+ lo2) in the
// low-precision type; products are summed smallest first:
//   BF16X2: lo*hi + hi*lo + hi*hi                     (3 MFMAs per product)
//   BF16X3: lo2*hi + hi*lo2 + lo*lo + lo*hi + hi*lo + hi*hi  (6 MFMAs)
//   FP16X2: lo parts scaled by 2^11 (kept normal), accumulated separately
//           and scaled back: hi*hi + 2^-11 (lo*hi + hi*lo)   (3 MFMAs);
//           a row outside FP16's comfortable range is first scaled by a
//           power of two (row_shift), so any finite input is accepted
// The constant matrices are split on the host from FP64 values.
#include "internal.h"

#include <atomic>
#include <climits>
#include <type_traits>

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
        // lo = (v - h) 2^11 rounded once to FP16: v - h and the scaling are
        // exact, so the fused form below has the same value and lets the
        // compiler read h as an FP16 operand (mixed-precision FMA) instead
        // of converting it back first
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const _Float16 h = static_cast<_Float16>(v[r]);
            p[0][r] = h;
            p[1][r] = static_cast<_Float16>(__builtin_fmaf(-static_cast<float>(h), 2048.0f, v[r] * 2048.0f));
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

// Operand `mat` (0..3) of this lane, every part: one 16-byte load each from
// the table of 16-bit encodings.
template <int MODE>
__device__ __forceinline__ void load_const(const float* tab, int mat, int lane,
                                           typename Prec<MODE>::V (&p)[Prec<MODE>::PARTS])
{
    using V = typename Prec<MODE>::V;
    const V* src = reinterpret_cast<const V*>(tab);
#pragma unroll
    for (int k = 0; k < Prec<MODE>::PARTS; ++k)
        p[k] = src[(mat * 3 + k) * 64 + lane];
}

constexpr int kWaves = 4;
// LDS words of one staged plane: 256 floats with 16 pad words after each 64.
// The operand reads and result writes touch n = 64q + 16r + c for lane
// (q, c) and register r: lane quarter q then starts 80q words in, i.e. on
// bank group 16q of 64 banks, and the 64 lanes hit 64 different banks.
constexpr int kPlaneWords = 256 + 64;
__device__ __forceinline__ int plane_word(int n) { return n + 16 * (n >> 6); }

typedef float v4f __attribute__((ext_vector_type(4)));

// Orders a wave's own LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Maximum over the wave of a nonnegative value, wave-uniform: DPP row shifts
// reduce each row of 16 lanes into its lane 15, two row broadcasts carry the
// rows into lane 63, which is read back as a scalar.  Lanes a DPP move has no
// source for read 0, the identity here.
template <int CTRL, int ROW_MASK, int BANK_MASK>
__device__ __forceinline__ float dpp_max_step(float x)
{
    const int y = __builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, BANK_MASK, false);
    return __builtin_fmaxf(x, __int_as_float(y));
}

__device__ __forceinline__ float wave_max_nonneg(float v)
{
    v = dpp_max_step<0x111, 0xf, 0xf>(v);  // row_shr:1
    v = dpp_max_step<0x112, 0xf, 0xf>(v);  // row_shr:2
    v = dpp_max_step<0x114, 0xf, 0xe>(v);  // row_shr:4
    v = dpp_max_step<0x118, 0xf, 0xc>(v);  // row_shr:8
    v = dpp_max_step<0x142, 0xa, 0xf>(v);  // row_bcast:15
    v = dpp_max_step<0x143, 0xc, 0xf>(v);  // row_bcast:31
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// FP16X2 range: the exponent k by which a row is scaled (x * 2^-k) before its
// FP16 split, and its outputs scaled back (y * 2^k).  A 16-point DFT grows
// magnitudes at most 32-fold (16 complex terms), so with the row's largest
// magnitude m below 2^10 both contractions' operands stay below 2^15 < 65504;
// and with m at least 2^-4 the row's significant values are normal FP16
// numbers.  Rows with m in [2^-4, 2^10) are not scaled (k = 0); the others
// are scaled to m * 2^-k in [2^9, 2^10), whatever their scale (k in
// [-158, 118]; ldexp of the values themselves, so no scale factor has to be
// representable).  Scaling by a power of two commutes with FP16 and FP32
// rounding.  All-zero and non-finite rows are not scaled.  k is wave-uniform.
__device__ __forceinline__ int row_shift(const v4f (&row)[2])
{
    float m = 0.0f;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int e = 0; e < 4; ++e)
            m = __builtin_fmaxf(m, __builtin_fabsf(row[p][e]));
    // the common case from two wave votes: the wave's maximum is in
    // [2^-4, 2^10) exactly when no lane's is 2^10 or more and some lane's is
    // 2^-4 or more (m is never NaN: fmax drops NaN operands)
    if (__builtin_amdgcn_ballot_w64(m >= 1024.0f) == 0 && __builtin_amdgcn_ballot_w64(m >= 0.0625f) != 0)
        return 0;
    m = wave_max_nonneg(m);
    if (!(m > 0.0f) || m == __builtin_inff() || (m >= 0.0625f && m < 1024.0f))
        return 0;
    // m = f * 2^e with f in [0.5, 1): m * 2^-k in [2^9, 2^10) for k = e - 10
    return __builtin_amdgcn_frexp_expf(m) - 10;
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

// The TPI rows from b0, all inside the batch.
template <int TPI>
__device__ __forceinline__ void load_rows_full(v4f (&in)[TPI][2], const float* xr, const float* xi, int64_t b0,
                                               int lane)
{
#pragma unroll
    for (int t = 0; t < TPI; ++t) {
        in[t][0] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xr + (b0 + t) * 256) + lane);
        in[t][1] = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(xi + (b0 + t) * 256) + lane);
    }
}

// TPI transforms per wave iteration; rows are staged through wave-private
// LDS so that global loads and stores are 16-byte and fully coalesced.
template <int MODE, int TPI>
__global__ void __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(4)))
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

    // the constant operands of both contractions (real and imaginary rows)
    V er[P::PARTS], ei[P::PARTS];
    load_const<MODE>(consts, 0, lane, er);
    load_const<MODE>(consts, 1, lane, ei);
    float2 w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
        w[r] = tw256[((4 * q + r) * c) & 255];

    // step-1 operand: lane (q, c), register r reads plane r >= 4 at
    // n = 16 (4q + (r & 3)) + c (input index n1 = 4q + (r & 3), row n0 = c)
    const int a_off = plane_word(64 * q + c);
    // the grid is resident: each wave loops with a stride and issues the
    // next rows' loads before the current rows' arithmetic
    const int64_t stride = nwaves * TPI;
    // Rows go to LDS ("staged") one iteration ahead: an iteration issues the
    // next rows' loads, computes the staged rows, stores their results, and
    // then stages the next rows.  The loads are thus issued before the
    // stores, and waiting for them (stores count in the same counter) does
    // not wait for the stores.  FP16X2 also carries each staged row's scale
    // exponent.
    v4f in[TPI][2];
    int shift[TPI];
    auto stage = [&]() {
#pragma unroll
        for (int t = 0; t < TPI; ++t) {
#pragma unroll
            for (int p = 0; p < 2; ++p)
                *reinterpret_cast<v4f*>(my + (2 * t + p) * kPlaneWords + plane_word(4 * lane)) = in[t][p];
            shift[t] = MODE == kModeFP16X2 ? row_shift(in[t]) : 0;
        }
        wave_lds_sync();
    };
    // One iteration over the staged rows b0 .. b0 + TPI - 1.  FULL: these
    // rows and the next iteration's are all in the batch, so every load and
    // store is unconditional and the compiler counts them exactly.
    auto iteration = [&](int64_t b0, auto full) {
        constexpr bool FULL = decltype(full)::value;
        const bool more = FULL || b0 + stride < batch;
        if constexpr (FULL)
            load_rows_full<TPI>(in, xr, xi, b0 + stride, lane);
        else if (more)
            load_rows<TPI>(in, xr, xi, b0 + stride, batch, lane);
#pragma unroll
        for (int t = 0; t < TPI; ++t) {
            const float* src = my + 2 * t * kPlaneWords + a_off;
            float v[8];
#pragma unroll
            for (int r = 0; r < 8; ++r)
                v[r] = src[(r >> 2) * kPlaneWords + 16 * (r & 3)];
            if (MODE == kModeFP16X2 && shift[t] != 0)  // wave-uniform
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    v[r] = __builtin_ldexpf(v[r], -shift[t]);
            V a[P::PARTS];
            split8<MODE>(v, a);
            const f32x4 xr4 = product<MODE>(a, er);
            const f32x4 xi4 = product<MODE>(a, ei);
            // twiddle W256^(n0 k1), n0 = 4q + r, k1 = c; B3 slot r < 4 real, r >= 4 imaginary
            float z[8];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                z[r] = __builtin_fmaf(w[r].x, xr4[r], w[r].y * xi4[r]);
                z[r + 4] = __builtin_fmaf(w[r].x, xi4[r], -(w[r].y * xr4[r]));
            }
            V b3[P::PARTS];
            split8<MODE>(z, b3);
            const f32x4 yr4 = product<MODE>(er, b3);
            const f32x4 yi4 = product<MODE>(ei, b3);
            // lane holds k2 = 4q + r, k1 = c: output index k1 + 16 k2 (the
            // transform's operand reads above are complete: the MFMAs used them)
            float* dr = my + 2 * t * kPlaneWords;
            float* di = dr + kPlaneWords;
            f32x4 outr = yr4, outi = yi4;
            if (MODE == kModeFP16X2 && shift[t] != 0)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    outr[r] = __builtin_ldexpf(yr4[r], shift[t]);
                    outi[r] = __builtin_ldexpf(yi4[r], shift[t]);
                }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                dr[plane_word(c + 16 * (4 * q + r))] = outr[r];
                di[plane_word(c + 16 * (4 * q + r))] = outi[r];
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int t = 0; t < TPI; ++t) {
            if (FULL || b0 + t < batch) {
                const v4f o_r = *reinterpret_cast<const v4f*>(my + 2 * t * kPlaneWords + plane_word(4 * lane));
                const v4f o_i = *reinterpret_cast<const v4f*>(my + (2 * t + 1) * kPlaneWords + plane_word(4 * lane));
                __builtin_nontemporal_store(o_r, reinterpret_cast<v4f*>(yr + (b0 + t) * 256) + lane);
                __builtin_nontemporal_store(o_i, reinterpret_cast<v4f*>(yi + (b0 + t) * 256) + lane);
            }
        }
        // the staging writes below reuse this wave's LDS
        wave_lds_sync();
        if (more)
            stage();
    };
    int64_t b0 = wave * TPI;
    if (b0 < batch) {
        load_rows<TPI>(in, xr, xi, b0, batch, lane);
        stage();
    }
    for (; b0 + stride + TPI <= batch; b0 += stride)
        iteration(b0, std::true_type{});
    // at most two more iterations, partly outside the batch
    for (; b0 < batch; b0 += stride)
        iteration(b0, std::false_type{});
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
