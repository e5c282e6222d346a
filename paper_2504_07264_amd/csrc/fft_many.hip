// Grouped execution: many split-format transforms of different power-of-two
// lengths (a ragged batch), forward and adjoint, in one persistent launch.
// (By default the plan sends its longer lengths to the single-length kernels
// instead; this kernel then only meets group items.)
//
// Each transform k occupies [offset_k, offset_k + N_k) of every plane.  The
// host sorts the transforms by length and cuts the work into items:
//   * a group item: up to 512 / T transforms of one length N <= 2^13, run by
//     the single-pass scheme of eq. (6) (register passes, LDS exchanges, bit
//     reversal folded into the LDS reads, 16-byte staged global I/O);
//   * a large item: one transform of length 2^14..2^16, run by the two-pass
//     scheme (stages 1..8 on 256-point blocks, then the remaining stages on
//     columns) by a single workgroup, through a workspace region private to
//     that workgroup, so no inter-workgroup dependency exists.
// Items are listed largest first; persistent workgroups take them from an
// atomic counter.  The last workgroup to leave resets the counter, so the
// launch can be replayed from a graph without any memset.
// The arithmetic is exactly eq. (6) in order, as in the other kernels, so each
// transform's result equals theirs bit for bit; the adjoint is the forward
// scheme with both plane pairs exchanged (the host swaps the pointers).
#include "fft_tile.h"

#include <climits>

namespace splitdft {
namespace {

constexpr int kMT = kManyThreads;
constexpr int kRB = 4;

// LDS words of a group item of length 2^M (one plane at a time).
template <int M>
struct GroupShape {
    static constexpr int RB = M < kRB ? M : kRB;
    static constexpr int N = 1 << M;
    static constexpr int E = 1 << RB;
    static constexpr int LT = M - RB;
    static constexpr int T = 1 << LT;
    static constexpr int NP = (M + RB - 1) / RB;
    static constexpr int SLOTS = kMT / T;
    static constexpr int SLOT = T >= 32 ? lds_index(N) : (lds_index(N) | 1);
    static constexpr int WORDS = SLOTS * SLOT;
    // sync group: a wave when transforms fit one wave, else the workgroup
    static constexpr int GT = T <= 64 ? 64 : kMT;
    static constexpr int GSLOTS = GT / T;
};

// workspace in pass-2 tile order (see TileCfg)
using P1_14 = TileCfg<14, 8, 1, 4, 32, true, false, 128>;
using P2_14 = TileCfg<14, 8, 2, 4, 128, true, true, 128>;
using P1_15 = TileCfg<15, 8, 1, 4, 32, true, false, 64>;
using P2_15 = TileCfg<15, 8, 2, 4, 64, true, true, 64>;
using P1_16 = TileCfg<16, 8, 1, 4, 32, true, false, 32>;
using P2_16 = TileCfg<16, 8, 2, 4, 32, true, true, 32>;

constexpr int cmax(int a, int b) { return a > b ? a : b; }
template <int M>
constexpr int group_words_upto()
{
    if constexpr (M < 2)
        return 0;
    else
        return cmax(GroupShape<M>::WORDS, group_words_upto<M - 1>());
}
constexpr int kGroupLdsWords = group_words_upto<13>();
constexpr int kLdsWords =
    cmax(kGroupLdsWords,
         cmax(cmax(P1_16::LDS_WORDS, P2_16::LDS_WORDS),
              cmax(cmax(P2_15::LDS_WORDS, P2_14::LDS_WORDS), cmax(P1_15::LDS_WORDS, P1_14::LDS_WORDS))));
static_assert(P1_16::THREADS == kMT && P2_16::THREADS == kMT && P1_15::THREADS == kMT && P2_15::THREADS == kMT &&
                  P1_14::THREADS == kMT && P2_14::THREADS == kMT,
              "tile shapes must use the grouped kernel's workgroup size");

// Planes of one item (the host has already exchanged them for the adjoint).
struct Planes {
    const float* xr;
    const float* xi;
    float* yr;
    float* yi;
};

// Twiddles of the group items' later passes: the first quarter turn of stage
// kGroupTwM (the longest group length) in LDS, in TwQuarterLds slot order;
// omega^(i,q) of every shorter length has an equal-valued entry there.
constexpr int kGroupTwM = 13;
using GroupTw = TwQuarterLds<kGroupTwM>;
constexpr int kGroupTwEntries = 1 << (kGroupTwM - 2);

// Group item: transforms first .. first + count - 1 of the length-sorted list,
// of length 2^M.
template <int M>
__device__ __forceinline__ void many_group_body(Planes pl, const int64_t* __restrict__ offsets,
                                                int64_t first, int count, const float2* __restrict__ tw,
                                                const float2* s_tw, float* lds,
                                                int64_t* s_off, int tid)
{
    using G = GroupShape<M>;
    constexpr int E = G::E, LT = G::LT, T = G::T, RB = G::RB, N = G::N;
    const float* xr = pl.xr;
    const float* xi = pl.xi;
    float* yr = pl.yr;
    float* yi = pl.yi;
    if (tid < count)
        s_off[tid] = offsets[first + tid];
    __syncthreads();

    const int slot = tid >> LT;
    const int t = tid & (T - 1);
    const int gtid = tid & (G::GT - 1);
    const int gslot0 = (tid / G::GT) * G::GSLOTS;
    float* gl = lds + gslot0 * G::SLOT;
    float* lr = lds + slot * G::SLOT;
    int valid_slots = count - gslot0;
    valid_slots = valid_slots < 0 ? 0 : (valid_slots > G::GSLOTS ? G::GSLOTS : valid_slots);
    const int valid = valid_slots * N;

    float vr[E], vi[E];
    // the 16-byte loads of both planes are issued first; then, one plane at a
    // time, each slot's row goes into LDS and the registers of the first pass
    // are read from it in bit-reversed order
    v4f ld[2][E / 4];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const float* src = p == 0 ? xr : xi;
#pragma unroll
        for (int c = 0; c < E / 4; ++c) {
            const int f = 4 * (gtid + c * G::GT);
            if (f < valid)
                ld[p][c] = load4<true>(src + s_off[gslot0 + (f >> M)] + (f & (N - 1)));
        }
    }
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int c = 0; c < E / 4; ++c) {
            const int f = 4 * (gtid + c * G::GT);
            if (f < valid) {
                float* d = gl + (f >> M) * G::SLOT + lds_index(f & (N - 1));
                d[0] = ld[p][c][0];
                d[1] = ld[p][c][1];
                d[2] = ld[p][c][2];
                d[3] = ld[p][c][3];
            }
        }
        xsync<T>();
        const int tb = rev_bits(t, LT);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const float w = lr[lds_index(tb + (rev_bits(u, RB) << LT))];
            if (p == 0)
                vr[u] = w;
            else
                vi[u] = w;
        }
        xsync<T>();
    }

    stages<E, LT, 0, Pass<M, RB, 0>::RP>(vr, vi, t, tw);
    if constexpr (G::NP > 1)
        later_passes<M, RB, 1, true, E, GroupTw>(vr, vi, lr, lr, t, s_tw);

    using Last = Pass<M, RB, G::NP - 1>;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
#pragma unroll
        for (int u = 0; u < E; ++u)
            lr[lds_index(position<LT, Last::S, Last::RP>(t, u))] = p == 0 ? vr[u] : vi[u];
        xsync<T>();
        float* dst = p == 0 ? yr : yi;
#pragma unroll
        for (int c = 0; c < E / 4; ++c) {
            const int f = 4 * (gtid + c * G::GT);
            if (f < valid) {
                const float* s = gl + (f >> M) * G::SLOT + lds_index(f & (N - 1));
                store4<true>(dst + s_off[gslot0 + (f >> M)] + (f & (N - 1)), v4f{s[0], s[1], s[2], s[3]});
            }
        }
        xsync<T>();
    }
    // s_off and the LDS slots are reused by the next item
    __syncthreads();
}

// Out of line: each length's item keeps its own register allocation (inlined
// into one dispatch, the twelve lengths' code would share, and spill, one).
template <int M, int WPE>
__device__ __noinline__ void many_group(Planes pl, const int64_t* __restrict__ offsets,
                                        int64_t first, int count, const float2* __restrict__ tw,
                                        const float2* s_tw, float* lds, int64_t* s_off, int tid)
{
    many_group_body<M>(pl, offsets, first, count, tw, s_tw, lds, s_off, tid);
}

// Large item: one transform through this workgroup's workspace region.
template <class P1, class P2, int WPE>
__device__ __noinline__ void many_large(Planes pl, int64_t off, float* ws, const float2* __restrict__ tw,
                                           float* lds, int tid)
{
    const float* xr = pl.xr + off;
    const float* xi = pl.xi + off;
    float* yr = pl.yr + off;
    float* yi = pl.yi + off;
    float* wr = ws + static_cast<int64_t>(blockIdx.x) * (2 * kManyMaxN);
    float* wi = wr + kManyMaxN;
    for (int tile = 0; tile < P1::TILES; ++tile) {
        tile_process<P1>(xr, xi, wr, wi, tw, TileCols<false>{tile * P1::C}, lds, tid);
        __syncthreads();
    }
    // the workgroup's own workspace stores are visible to its loads after the
    // barrier above
    for (int tile = 0; tile < P2::TILES; ++tile) {
        tile_process<P2>(wr, wi, yr, yi, tw, TileCols<false>{tile * P2::C}, lds, tid);
        __syncthreads();
    }
}

// WPE: minimum waves per SIMD the register allocation must allow (1 = no
// limit, one workgroup per CU; 4 = two workgroups per CU, 128 VGPRs).
// LARGE: whether items of length >= 2^14 can occur (else their code, LDS and
// registers are left out).
template <int WPE, bool LARGE>
__global__ void __launch_bounds__(kMT) __attribute__((amdgpu_waves_per_eu(WPE)))
split_fft_many_kernel(const float* in_r0, const float* in_i0, float* out_r0, float* out_i0, const float* in_r1,
                      const float* in_i1, float* out_r1, float* out_i1, const int64_t* __restrict__ offsets,
                      const ManyItem* __restrict__ items, int nitems, int* queue,
                      float* ws, const float2* __restrict__ tw)
{
    __shared__ float lds[LARGE ? kLdsWords : kGroupLdsWords];
    __shared__ int64_t s_off[kMT];
    __shared__ int s_item;
    __shared__ float2 s_tw[kGroupTwEntries];
    const int tid = threadIdx.x;
    // stage kGroupTwM's block starts at table entry 2^(kGroupTwM - 1); the
    // barrier at the top of the item loop orders these writes before any read
    for (int k = tid; k < kGroupTwEntries; k += kMT)
        s_tw[GroupTw::slot(k)] = tw[(1 << (kGroupTwM - 1)) + k];
    for (;;) {
        if (tid == 0)
            s_item = atomicAdd(&queue[0], 1);
        __syncthreads();
        // uniform across the workgroup: keep it scalar so that the dispatch
        // below is a scalar branch and the item fields are scalar loads
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= nitems)
            break;
        const int m = __builtin_amdgcn_readfirstlane(items[item].m);
        const int dir = __builtin_amdgcn_readfirstlane(items[item].dir);
        const int count = __builtin_amdgcn_readfirstlane(items[item].count);
        const int64_t first = items[item].first;
        const Planes pl = dir == 0 ? Planes{in_r0, in_i0, out_r0, out_i0} : Planes{in_r1, in_i1, out_r1, out_i1};
        switch (m) {
#define SDFT_GROUP(MM)                                                                   \
    case MM:                                                                             \
        many_group<MM, WPE>(pl, offsets, first, count, tw, s_tw, lds, s_off, tid);        \
        break;
            SDFT_GROUP(2)
            SDFT_GROUP(3)
            SDFT_GROUP(4)
            SDFT_GROUP(5)
            SDFT_GROUP(6)
            SDFT_GROUP(7)
            SDFT_GROUP(8)
            SDFT_GROUP(9)
            SDFT_GROUP(10)
            SDFT_GROUP(11)
            SDFT_GROUP(12)
            SDFT_GROUP(13)
#undef SDFT_GROUP
        case 14:
            if constexpr (LARGE)
                many_large<P1_14, P2_14, WPE>(pl, offsets[first], ws, tw, lds, tid);
            break;
        case 15:
            if constexpr (LARGE)
                many_large<P1_15, P2_15, WPE>(pl, offsets[first], ws, tw, lds, tid);
            break;
        case 16:
            if constexpr (LARGE)
                many_large<P1_16, P2_16, WPE>(pl, offsets[first], ws, tw, lds, tid);
            break;
        default: break;
        }
    }
    // the last workgroup out resets the queue for the next launch
    if (tid == 0) {
        __threadfence();
        if (atomicAdd(&queue[1], 1) == static_cast<int>(gridDim.x) - 1) {
            atomicExch(&queue[0], 0);
            atomicExch(&queue[1], 0);
        }
    }
}

template <bool LARGE>
auto many_kernel(int variant)
{
    return variant == 0 ? split_fft_many_kernel<4, LARGE> : split_fft_many_kernel<1, LARGE>;
}

}  // namespace

hipError_t launch_many(int variant, bool large, const ManyArgs& a, int grid, hipStream_t stream)
{
    auto k = large ? many_kernel<true>(variant) : many_kernel<false>(variant);
    hipLaunchKernelGGL(k, dim3(static_cast<unsigned>(grid)), dim3(kMT), 0, stream, a.in_r[0], a.in_i[0], a.out_r[0],
                       a.out_i[0], a.in_r[1], a.in_i[1], a.out_r[1], a.out_i[1], a.offsets, a.items,
                       a.nitems, a.queue, a.ws, a.tw);
    return hipGetLastError();
}

hipError_t many_max_active_per_cu(int variant, bool large, int* blocks)
{
    auto k = large ? many_kernel<true>(variant) : many_kernel<false>(variant);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k, kMT, 0);
}

int many_items_per_group(int m)
{
    // transforms of length 2^m that one group item holds
    return m < 2 || m > 13 ? 1 : kMT >> (m - (m < kRB ? m : kRB));
}

}  // namespace splitdft
