// Single-pass split-format FFT kernels for gfx950.
//
// Each workgroup owns `TPW` whole transforms of length N = 2^M.  Within a
// transform, thread t holds E = 2^RB complex elements as two register arrays
// (real plane, imaginary plane) and applies the factors of eq. (6) of the
// paper (Section III) in order:
//
//   S        bit reversal: folded into the global-load addresses;
//   D^(i)    the upper element of each pair at distance 2^(i-1) is rotated
//            by omega^(i,q) = [[c, s], [-s, c]];
//   W^(i)    butterfly (u + v, u - v) on each plane separately.
//
// Only the twiddle factor mixes the planes; permutation and butterflies act
// on each plane alone (the interleaved factors of eq. (6) are I_2-blocked
// once x_2N is written as two planes).
//
// Stages are taken RB at a time ("passes").  Position j of a transform (the
// index of eq. (6)'s working vector after the bit reversal) is held during the
// pass that starts after stage S and combines RP stages by
//
//   thread t, register u = uu + (g << RP):
//     o  = t + (g << LT)                       (LT = M - RB, T = 2^LT threads)
//     j  = (o mod 2^S) + (uu << S) + ((o >> S) << (S + RP))
//
// so the RP stages of the pass pair registers of one thread.  Between passes
// the working vector goes through LDS.  The first pass is always full (RP =
// RB), which makes the bit-reversed loads coalesced: for fixed u the threads
// of a transform read a contiguous run of T floats.  In the last pass
// (o >> S) = 0 and j = o + (uu << S), so the stores are coalesced too.
//
// Every rotation is fmaf(c, ar, s*ai), fmaf(c, ai, -(s*ar)) with FP32
// twiddles from the plan's table (entry 2^(i-1) + q holds omega^(i,q)); in the
// first pass the twiddles with q = 0 (identity) and angle pi/2 (swap and
// negate) are applied as such, which gives the same values as the general
// form with the table's exact 1 and 0.  The results therefore equal, bit for
// bit, the factors of eq. (6) applied one after the other in FP32.
#include "internal.h"

#include <climits>

namespace splitdft {
namespace {

__device__ __forceinline__ int rev_bits(int x, int bits)
{
    return bits == 0 ? 0 : static_cast<int>(__builtin_bitreverse32(static_cast<unsigned>(x)) >> (32 - bits));
}

// LDS word of in-transform position j: one pad word after every 32 words, so
// that the strided accesses of a pass transition spread over the banks.
__host__ __device__ constexpr int lds_index(int j) { return j + (j >> 5); }

template <int LT, int S, int RP>
__device__ __forceinline__ int position(int t, int u)
{
    const int g = u >> RP;
    const int uu = u & ((1 << RP) - 1);
    const int o = t + (g << LT);
    return (o & ((1 << S) - 1)) + (uu << S) + ((o >> S) << (S + RP));
}

// (ar, ai) <- omega (ar, ai), omega = [[c, s], [-s, c]].
__device__ __forceinline__ void rotate(float& ar, float& ai, float c, float s)
{
    const float tr = __builtin_fmaf(c, ar, s * ai);
    const float ti = __builtin_fmaf(c, ai, -(s * ar));
    ar = tr;
    ai = ti;
}

// Stages S+1 .. S+RP of eq. (6) on the E registers of one thread.
template <int E, int LT, int S, int RP>
__device__ __forceinline__ void stages(float (&vr)[E], float (&vi)[E], int t, const float2* __restrict__ tw)
{
#pragma unroll
    for (int k = 1; k <= RP; ++k) {
        const int half = 1 << (k - 1);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u & half)
                continue;
            const int v = u + half;
            float ar = vr[v], ai = vi[v];
            if constexpr (S == 0) {
                const int q = u & (half - 1);
                if (q == 0) {
                    // omega^(k,0) = I
                } else if (2 * q == half) {
                    // omega at angle pi/2 = [[0, 1], [-1, 0]]
                    const float tr = ai;
                    ai = -ar;
                    ar = tr;
                } else {
                    const float2 w = tw[half + q];
                    rotate(ar, ai, w.x, w.y);
                }
            } else {
                const int o = t + ((u >> RP) << LT);
                const int q = (o & ((1 << S) - 1)) + ((u & (half - 1)) << S);
                const float2 w = tw[(1 << (S + k - 1)) + q];
                rotate(ar, ai, w.x, w.y);
            }
            const float ur = vr[u], ui = vi[u];
            vr[u] = ur + ar;
            vi[u] = ui + ai;
            vr[v] = ur - ar;
            vi[v] = ui - ai;
        }
    }
}

template <int M, int RB, int P>
struct Pass {
    static constexpr int S = P * RB;
    static constexpr int RP = (S + RB <= M) ? RB : (M - S);
};

template <int E, int LT, int S0, int RP0, int S1, int RP1>
__device__ __forceinline__ void lds_put(const float (&v)[E], float* lds, int t)
{
#pragma unroll
    for (int u = 0; u < E; ++u)
        lds[lds_index(position<LT, S0, RP0>(t, u))] = v[u];
}

template <int E, int LT, int S1, int RP1>
__device__ __forceinline__ void lds_get(float (&v)[E], const float* lds, int t)
{
#pragma unroll
    for (int u = 0; u < E; ++u)
        v[u] = lds[lds_index(position<LT, S1, RP1>(t, u))];
}

// Passes P, P+1, ... : exchange through LDS, then the pass's stages.
template <int M, int RB, int P, bool SPLIT, int E>
__device__ __forceinline__ void later_passes(float (&vr)[E], float (&vi)[E], float* lr, float* li, int t,
                                             const float2* __restrict__ tw)
{
    if constexpr (P * RB < M) {
        constexpr int LT = M - RB;
        using Prev = Pass<M, RB, P - 1>;
        using Cur = Pass<M, RB, P>;
        if constexpr (SPLIT) {  // one plane at a time through the same LDS
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            __syncthreads();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            __syncthreads();
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, lr, t);
            __syncthreads();
            lds_get<E, LT, Cur::S, Cur::RP>(vi, lr, t);
            __syncthreads();
        } else {
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, li, t);
            __syncthreads();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            lds_get<E, LT, Cur::S, Cur::RP>(vi, li, t);
            __syncthreads();
        }
        stages<E, LT, Cur::S, Cur::RP>(vr, vi, t, tw);
        later_passes<M, RB, P + 1, SPLIT, E>(vr, vi, lr, li, t, tw);
    }
}

template <int M, int RB, int TPW, bool SPLIT>
struct Shape {
    static constexpr int N = 1 << M;
    static constexpr int E = 1 << RB;
    static constexpr int LT = M - RB;
    static constexpr int T = 1 << LT;
    static constexpr int NP = (M + RB - 1) / RB;
    static constexpr int THREADS = TPW * T;
    static constexpr int PADN = lds_index(N);
    static constexpr int LDS_WORDS = (NP > 1) ? TPW * PADN * (SPLIT ? 1 : 2) : 1;
};

template <int M, int RB, int TPW, bool SPLIT>
__global__ void __launch_bounds__(TPW << (M - RB))
split_fft_lds_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                     int64_t batch)
{
    using Sh = Shape<M, RB, TPW, SPLIT>;
    constexpr int N = Sh::N, E = Sh::E, LT = Sh::LT, T = Sh::T, NP = Sh::NP;
    __shared__ float lds[Sh::LDS_WORDS];

    const int tid = threadIdx.x;
    const int slot = tid >> LT;
    const int t = tid & (T - 1);
    const int64_t b = static_cast<int64_t>(blockIdx.x) * TPW + slot;
    const bool active = b < batch;
    const int64_t row = b * N;

    float vr[E], vi[E];
    if constexpr (T == 1) {
        // A whole transform per thread: natural-order vector loads; the bit
        // reversal is a renaming of registers.
        if (active) {
            if constexpr (N >= 4) {
                const float4* pr = reinterpret_cast<const float4*>(xr + row);
                const float4* pi = reinterpret_cast<const float4*>(xi + row);
#pragma unroll
                for (int c = 0; c < N / 4; ++c) {
                    const float4 a = pr[c], z = pi[c];
                    vr[rev_bits(4 * c + 0, M)] = a.x;
                    vr[rev_bits(4 * c + 1, M)] = a.y;
                    vr[rev_bits(4 * c + 2, M)] = a.z;
                    vr[rev_bits(4 * c + 3, M)] = a.w;
                    vi[rev_bits(4 * c + 0, M)] = z.x;
                    vi[rev_bits(4 * c + 1, M)] = z.y;
                    vi[rev_bits(4 * c + 2, M)] = z.z;
                    vi[rev_bits(4 * c + 3, M)] = z.w;
                }
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    vr[rev_bits(n, M)] = xr[row + n];
                    vi[rev_bits(n, M)] = xi[row + n];
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u)
                vr[u] = vi[u] = 0.0f;
        }
    } else {
        // Position u + (t << RB) holds x[rev_M(u + (t << RB))]
        //   = x[rev_LT(t) + (rev_RB(u) << LT)].
        const int tb = rev_bits(t, LT);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t idx = row + tb + (rev_bits(u, RB) << LT);
            vr[u] = active ? xr[idx] : 0.0f;
            vi[u] = active ? xi[idx] : 0.0f;
        }
    }

    stages<E, LT, 0, Pass<M, RB, 0>::RP>(vr, vi, t, tw);

    if constexpr (NP > 1) {
        float* lr = lds + slot * Sh::PADN;
        float* li = SPLIT ? lr : lr + TPW * Sh::PADN;
        later_passes<M, RB, 1, SPLIT, E>(vr, vi, lr, li, t, tw);
    }

    if (!active)
        return;
    using Last = Pass<M, RB, NP - 1>;
    if constexpr (T == 1) {
        if constexpr (N >= 4) {
            float4* pr = reinterpret_cast<float4*>(yr + row);
            float4* pi = reinterpret_cast<float4*>(yi + row);
#pragma unroll
            for (int c = 0; c < N / 4; ++c) {
                pr[c] = make_float4(vr[4 * c], vr[4 * c + 1], vr[4 * c + 2], vr[4 * c + 3]);
                pi[c] = make_float4(vi[4 * c], vi[4 * c + 1], vi[4 * c + 2], vi[4 * c + 3]);
            }
        } else {
#pragma unroll
            for (int n = 0; n < N; ++n) {
                yr[row + n] = vr[n];
                yi[row + n] = vi[n];
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t idx = row + position<LT, Last::S, Last::RP>(t, u);
            yr[idx] = vr[u];
            yi[idx] = vi[u];
        }
    }
}

// N = 1: the transform is the identity.
__global__ void __launch_bounds__(256) split_fft_len1_kernel(const float* xr, const float* xi, float* yr, float* yi,
                                                             int64_t batch)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (b < batch) {
        const float r = xr[b], i = xi[b];
        yr[b] = r;
        yi[b] = i;
    }
}

hipError_t launch_len1(const float* xr, const float* xi, float* yr, float* yi, const float2*, int64_t batch,
                       hipStream_t stream)
{
    const int64_t blocks = (batch + 255) / 256;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(split_fft_len1_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, xr, xi, yr,
                       yi, batch);
    return hipGetLastError();
}

template <int M, int RB, int TPW, bool SPLIT>
hipError_t launch_lds(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                      hipStream_t stream)
{
    using Sh = Shape<M, RB, TPW, SPLIT>;
    const int64_t blocks = (batch + TPW - 1) / TPW;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((split_fft_lds_kernel<M, RB, TPW, SPLIT>), dim3(static_cast<unsigned>(blocks)),
                       dim3(Sh::THREADS), 0, stream, xr, xi, yr, yi, tw, batch);
    return hipGetLastError();
}

#define SDFT_V(M, RB, TPW, SPLIT)                                                                              \
    Variant                                                                                                    \
    {                                                                                                          \
        M, RB, TPW, Shape<M, RB, TPW, SPLIT>::THREADS,                                                         \
            static_cast<int>(sizeof(float)) * Shape<M, RB, TPW, SPLIT>::LDS_WORDS, &launch_lds<M, RB, TPW, SPLIT> \
    }

// Compiled schedules per length; the first entry of each list is the default.
const Variant kV0[] = {Variant{0, 0, 256, 256, 0, &launch_len1}};
const Variant kV1[] = {SDFT_V(1, 1, 256, false)};
const Variant kV2[] = {SDFT_V(2, 2, 256, false)};
const Variant kV3[] = {SDFT_V(3, 3, 256, false)};
const Variant kV4[] = {SDFT_V(4, 4, 256, false), SDFT_V(4, 4, 64, false)};
const Variant kV5[] = {SDFT_V(5, 5, 128, false), SDFT_V(5, 4, 128, false)};
const Variant kV6[] = {SDFT_V(6, 3, 32, false), SDFT_V(6, 4, 64, false)};
const Variant kV7[] = {SDFT_V(7, 4, 32, false), SDFT_V(7, 4, 16, false)};
const Variant kV8[] = {SDFT_V(8, 4, 16, false), SDFT_V(8, 4, 4, false)};
const Variant kV9[] = {SDFT_V(9, 5, 16, false), SDFT_V(9, 4, 8, false)};
const Variant kV10[] = {SDFT_V(10, 5, 8, false), SDFT_V(10, 5, 2, false), SDFT_V(10, 4, 4, false),
                        SDFT_V(10, 5, 8, true)};
const Variant kV11[] = {SDFT_V(11, 4, 2, false), SDFT_V(11, 5, 4, false)};
const Variant kV12[] = {SDFT_V(12, 4, 1, false), SDFT_V(12, 5, 2, false)};
const Variant kV13[] = {SDFT_V(13, 5, 1, false), SDFT_V(13, 4, 1, false)};
const Variant kV14[] = {SDFT_V(14, 5, 1, false), SDFT_V(14, 5, 1, true)};
const Variant kV15[] = {SDFT_V(15, 5, 1, true)};

#undef SDFT_V

struct VariantList {
    const Variant* v;
    int count;
};

#define SDFT_L(a) VariantList{a, static_cast<int>(sizeof(a) / sizeof(a[0]))}
const VariantList kLists[] = {SDFT_L(kV0),  SDFT_L(kV1),  SDFT_L(kV2),  SDFT_L(kV3),  SDFT_L(kV4),  SDFT_L(kV5),
                              SDFT_L(kV6),  SDFT_L(kV7),  SDFT_L(kV8),  SDFT_L(kV9),  SDFT_L(kV10), SDFT_L(kV11),
                              SDFT_L(kV12), SDFT_L(kV13), SDFT_L(kV14), SDFT_L(kV15)};
#undef SDFT_L

}  // namespace

const Variant* variants_for(int m, int* count)
{
    if (m < 0 || m >= static_cast<int>(sizeof(kLists) / sizeof(kLists[0]))) {
        *count = 0;
        return nullptr;
    }
    *count = kLists[m].count;
    return kLists[m].v;
}

const Variant* default_variant(int m, int64_t /*batch*/)
{
    int count = 0;
    const Variant* v = variants_for(m, &count);
    return count > 0 ? &v[0] : nullptr;
}

}  // namespace splitdft
