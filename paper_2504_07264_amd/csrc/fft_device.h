// Device building blocks shared by the split-format FFT kernels: the stages
// of eq. (6) (Section III) on registers, position maps of register passes,
// LDS exchanges and streaming load/store helpers.
//
// Position j of a group of 2^M positions (a whole transform, or a sub-block of
// one) is held during the pass that starts after stage S and combines RP
// stages by thread t, register u = uu + (g << RP):
//     o = t + (g << LT)                       (LT = M - RB, T = 2^LT threads)
//     j = (o mod 2^S) + (uu << S) + ((o >> S) << (S + RP))
// so the RP stages of the pass pair registers of one thread.
//
// Every rotation (factor D^(i)) is fmaf(c, ar, s*ai), fmaf(c, ai, -(s*ar))
// with FP32 twiddles from the plan's table (entry 2^(i-1) + q holds
// omega^(i,q)); every butterfly (factor W^(i)) is (u + v, u - v) per plane.
// In a first pass without stage shift, q = 0 (identity) and the angle pi/2
// (swap and negate) are applied as such, which gives the same values as the
// general form with the table's exact 1 and 0.
#pragma once

#include "internal.h"

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

// Twiddle sources: omega^(i,q) for stage i ("level") and index q < 2^(i-1).
//
// TwTable<OFF>: the plan's table, entry 2^(i-1) + q read at tw[entry - OFF]
// (OFF > 0 when only the upper part of the table is staged).
template <int OFF>
struct TwTable {
    static __device__ __forceinline__ float2 get(const float2* __restrict__ tw, int level, int q)
    {
        return tw[(1 << (level - 1)) - OFF + q];
    }
    // q = qt + qc with qt and qc on disjoint bits (qt per thread, qc fixed
    // per register)
    static __device__ __forceinline__ float2 get2(const float2* __restrict__ tw, int level, int qt, int qc)
    {
        return get(tw, level, qt + qc);
    }
};

// TwQuarter<MQ>: only the first quarter turn of stage MQ's twiddles,
// tw[k] = omega^(MQ, k) for k < 2^(MQ-2).  omega^(i,q) has the angle of
// omega^(MQ, q 2^(MQ-i)) and the table holds the same FP32 value for equal
// angles; an angle a + pi/2 in the upper quarter has (cos, sin) =
// (-sin a, cos a), which the table's quadrant rule also gives exactly (with
// +0 for -0, hence 0 - s rather than a negation).
template <int MQ>
struct TwQuarter {
    static __device__ __forceinline__ float2 get(const float2* __restrict__ tw, int level, int q)
    {
        constexpr int H = 1 << (MQ - 2);
        const int idx = q << (MQ - level);
        const float2 w = tw[idx & (H - 1)];
        const bool upper = (idx & H) != 0;
        return make_float2(upper ? 0.0f - w.y : w.x, upper ? w.x : w.y);
    }
    static __device__ __forceinline__ float2 get2(const float2* __restrict__ tw, int level, int qt, int qc)
    {
        return get(tw, level, qt + qc);
    }
};

// TwQuarterLds<MQ>: the values of TwQuarter<MQ> from a copy of its table in
// LDS that holds entry k at slot(k).  Later passes read the table at strides
// of 2^(MQ - level) entries, which in the plain layout fall into few LDS banks
// (up to 16 lanes on one bank); slot(k) XORs the higher 5-bit groups of k
// into its low 5 bits, which spreads any run of 2^s-strided entries over 32
// consecutive 8-byte slots, i.e. over all banks.  slot() is linear over XOR,
// so with q = qt + qc on disjoint bits the per-thread part slot(qt ...) is
// computed once per stage and each register only XORs a constant.  slot()
// keeps bits 5 and up and XORs the low 5 bits with a function of them, so it
// maps [0, H) onto itself and is its own inverse.
template <int MQ>
struct TwQuarterLds {
    static constexpr int H = 1 << (MQ - 2);
    static __host__ __device__ constexpr int slot(int k) { return k ^ (((k >> 5) ^ (k >> 10) ^ (k >> 15)) & 31); }
    static __device__ __forceinline__ float2 get2(const float2* tw, int level, int qt, int qc)
    {
        const int it = qt << (MQ - level), ic = qc << (MQ - level);
        const float2 w = tw[slot(it & (H - 1)) ^ slot(ic & (H - 1))];
        const bool upper = ((it ^ ic) & H) != 0;
        return make_float2(upper ? 0.0f - w.y : w.x, upper ? w.x : w.y);
    }
    static __device__ __forceinline__ float2 get(const float2* tw, int level, int q) { return get2(tw, level, q, 0); }
};
static_assert(TwQuarterLds<16>::slot(TwQuarterLds<16>::slot(12345)) == 12345 &&
                  TwQuarterLds<16>::slot(32) == 33 && TwQuarterLds<16>::slot(1024) == 1025,
              "slot layout of the LDS quarter table");

// Stages S+1 .. S+RP of a group of 2^MA positions on the E registers of one
// thread.  The group's position p is the transform's position lo_g + (p << A)
// (A = 0, lo_g = 0 for a whole transform), so its local stage s is stage A + s
// of eq. (6) and a local twiddle index ql becomes q = lo_g + (ql << A).  TW is
// the twiddle source for the non-trivial rotations.
template <int E, int LT, int S, int RP, class TW = TwTable<0>, int A = 0>
__device__ __forceinline__ void stages(float (&vr)[E], float (&vi)[E], int t, const float2* __restrict__ tw,
                                       int lo_g = 0)
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
            if constexpr (S == 0 && A == 0) {
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
                // ql = (o & (2^S - 1)) + (u mod half) 2^S with o = t + (u >> RP) 2^LT,
                // split into the thread's part and the register's (t < 2^LT)
                const int qt = lo_g + ((t & ((1 << S) - 1)) << A);
                const int qc = ((((u >> RP) << LT) & ((1 << S) - 1)) + ((u & (half - 1)) << S)) << A;
                const float2 w = TW::get2(tw, A + S + k, qt, qc);
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

// Stages S+RP .. S+1 of the decimation-in-frequency factorisation, eq. (9),
// on the E registers of one thread (positions as in the DIT passes): for each
// stage, highest first, the butterfly W^(i) (u + v, u - v) and then the
// rotation D^(i) of the upper element by omega^(i,q), q as in stages().  The
// pass with S = 0 takes its uniform twiddles from the plan's table tw; the
// other passes read theirs from the source TW at tws.
template <int E, int LT, int S, int RP, class TW = TwTable<0>>
__device__ __forceinline__ void stages_dif(float (&vr)[E], float (&vi)[E], int t, const float2* __restrict__ tw,
                                           const float2* __restrict__ tws)
{
#pragma unroll
    for (int k = RP; k >= 1; --k) {
        const int half = 1 << (k - 1);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            if (u & half)
                continue;
            const int v = u + half;
            const float ur = vr[u], ui = vi[u], wr = vr[v], wi = vi[v];
            vr[u] = ur + wr;
            vi[u] = ui + wi;
            float dr = ur - wr, di = ui - wi;
            if constexpr (S == 0) {
                const int q = u & (half - 1);
                if (q == 0) {
                    // omega^(k,0) = I
                } else if (2 * q == half) {
                    const float tr = di;  // angle pi/2
                    di = -dr;
                    dr = tr;
                } else {
                    const float2 w = tw[half + q];
                    rotate(dr, di, w.x, w.y);
                }
            } else {
                const int qt = t & ((1 << S) - 1);  // as in stages()
                const int qc = (((u >> RP) << LT) & ((1 << S) - 1)) + ((u & (half - 1)) << S);
                const float2 w = TW::get2(tws, S + k, qt, qc);
                rotate(dr, di, w.x, w.y);
            }
            vr[v] = dr;
            vi[v] = di;
        }
    }
}

// Orders a wave's LDS writes before its later LDS reads by other lanes of the
// same wave (LDS operations of one wave complete in order).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Synchronisation of an LDS exchange among the T threads of one transform:
// a transform of at most 64 threads lies within one wave.
template <int T>
__device__ __forceinline__ void xsync()
{
    if constexpr (T <= 64)
        wave_lds_sync();
    else
        __syncthreads();
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

// Passes of the decimation-in-frequency order: pass 0 covers the top RP0
// bits (RP0 = M - RB (NP - 1), the partial one), later passes RB bits each,
// downwards, the last one bits 0 .. RB-1.
template <int M, int RB, int P>
struct PassD {
    static constexpr int NP = (M + RB - 1) / RB;
    static constexpr int RP0 = M - RB * (NP - 1);
    static constexpr int RP = P == 0 ? RP0 : RB;
    static constexpr int S = M - RP0 - RB * P;
};

// Whether the DIF exchange into pass P stays inside one wave.  Pass P covers
// bits S .. S+RB-1 of the position and the full pass P-1 the RB bits above;
// position j moves from thread (j mod 2^(S+RB)) + ((j >> (S+2RB)) << (S+RB)) to
// thread (j mod 2^S) + ((j >> (S+RB)) << S), both in the aligned run of
// 2^(S+RB) consecutive threads numbered from (j >> (S+2RB)) << (S+RB).  With
// 2^(S+RB) <= 64 that run lies in one wave.  S decreases from pass to pass,
// so once an exchange is wave-local every later one is too.
template <int M, int RB, int P>
__host__ __device__ constexpr bool dif_wave_local_exchange()
{
    return P >= 1 && P < PassD<M, RB, 0>::NP && (1 << (M - RB)) > 64 && PassD<M, RB, P - 1>::RP == RB &&
           (1 << (PassD<M, RB, P>::S + RB)) <= 64;
}

// Whether the last DIF exchange was ordered per wave only: the caller then
// needs a workgroup barrier before its next LDS writes.
template <int M, int RB>
__host__ __device__ constexpr bool dif_last_exchange_local()
{
    return dif_wave_local_exchange<M, RB, PassD<M, RB, 0>::NP - 1>();
}

static_assert(dif_last_exchange_local<11, 4>() && dif_last_exchange_local<14, 4>() &&
                  dif_last_exchange_local<13, 5>() && !dif_wave_local_exchange<14, 4, 2>() &&
                  !dif_wave_local_exchange<14, 4, 1>() && !dif_last_exchange_local<10, 4>(),
              "wave-local exchanges of the DIF passes");

// DIF passes P, P+1, ...: exchange through LDS, then the pass's stages
// (twiddle sources as in stages_dif).  Wave-local exchanges
// (dif_wave_local_exchange) are ordered per wave.
template <int M, int RB, int P, bool SPLIT, int E, class TW = TwTable<0>>
__device__ __forceinline__ void later_passes_dif(float (&vr)[E], float (&vi)[E], float* lr, float* li, int t,
                                                 const float2* __restrict__ tw, const float2* __restrict__ tws)
{
    if constexpr (P < PassD<M, RB, 0>::NP) {
        constexpr int LT = M - RB;
        constexpr int T = dif_wave_local_exchange<M, RB, P>() ? 64 : (1 << LT);
        using Prev = PassD<M, RB, P - 1>;
        using Cur = PassD<M, RB, P>;
        if constexpr (SPLIT) {
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            xsync<T>();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            xsync<T>();
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, lr, t);
            xsync<T>();
            lds_get<E, LT, Cur::S, Cur::RP>(vi, lr, t);
            xsync<T>();
        } else {
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, li, t);
            xsync<T>();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            lds_get<E, LT, Cur::S, Cur::RP>(vi, li, t);
            xsync<T>();
        }
        stages_dif<E, LT, Cur::S, Cur::RP, TW>(vr, vi, t, tw, tws);
        later_passes_dif<M, RB, P + 1, SPLIT, E, TW>(vr, vi, lr, li, t, tw, tws);
    }
}

// Whether the exchange into pass P of a group of 2^M positions stays inside
// one wave.  Between two full passes (RP = RB) position j moves from thread
// (j mod 2^S') + ((j >> S) << S') to thread (j mod 2^S) + ((j >> (S + RB)) << S)
// (S' = S - RB): both lie in the run of 2^S threads numbered from
// (j >> (S + RB)) << S, so the exchange never leaves an aligned run of 2^S
// consecutive threads.  When the group's threads are the consecutive lanes
// 0 .. 2^(M-RB) - 1 of aligned runs (SYNC_T = 2^(M-RB)) and 2^S <= 64, each
// run lies in one wave, and wave-level ordering suffices where SYNC_T alone
// would ask for workgroup barriers.
template <int M, int RB, int P, int SYNC_T>
__host__ __device__ constexpr bool wave_local_exchange()
{
    return P >= 1 && P * RB < M && SYNC_T == (1 << (M - RB)) && SYNC_T > 64 && Pass<M, RB, P>::RP == RB &&
           (1 << Pass<M, RB, P>::S) <= 64;
}

// The cases the position-map tests enumerate: with 16 elements per thread
// the first exchange of 2^11 .. 2^14 stays in a wave and the second does not;
// with 32, the first of 2^12 .. 2^15; a transform of one wave needs no rule,
// and neither does a sync group other than the transform's own lanes.
static_assert(wave_local_exchange<11, 4, 1, 128>() && wave_local_exchange<14, 4, 1, 1024>() &&
                  !wave_local_exchange<14, 4, 2, 1024>() && !wave_local_exchange<14, 4, 3, 1024>() &&
                  wave_local_exchange<15, 5, 1, 1024>() && !wave_local_exchange<10, 4, 1, 64>() &&
                  !wave_local_exchange<14, 4, 1, 1025>(),
              "wave-local exchanges of the DIT passes");

// Passes P, P+1, ... of a group of 2^M positions: exchange through LDS, then
// the pass's stages (A, lo_g as for stages()).  SYNC_T is the thread count
// whose exchange ordering is needed (the group's own T when its threads are
// consecutive lanes; anything above 64 forces workgroup barriers).  An
// exchange that stays inside each wave (wave_local_exchange) orders only its
// wave's accesses; the next exchange that does not then starts with a
// workgroup barrier, so that no wave writes slots that another wave may still
// be reading.
template <int M, int RB, int P, bool SPLIT, int E, class TW, int A = 0, int SYNC_T = (1 << (M - RB))>
__device__ __forceinline__ void later_passes(float (&vr)[E], float (&vi)[E], float* lr, float* li, int t,
                                             const float2* __restrict__ tw, int lo_g = 0)
{
    if constexpr (P * RB < M) {
        constexpr int LT = M - RB;
        using Prev = Pass<M, RB, P - 1>;
        using Cur = Pass<M, RB, P>;
        constexpr bool LOCAL = wave_local_exchange<M, RB, P, SYNC_T>();
        constexpr int XT = LOCAL ? 64 : SYNC_T;
        if constexpr (!LOCAL && wave_local_exchange<M, RB, P - 1, SYNC_T>())
            xsync<SYNC_T>();
        if constexpr (SPLIT) {  // one plane at a time through the same LDS
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            xsync<XT>();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            xsync<XT>();
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, lr, t);
            xsync<XT>();
            lds_get<E, LT, Cur::S, Cur::RP>(vi, lr, t);
            xsync<XT>();
        } else {
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
            lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, li, t);
            xsync<XT>();
            lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
            lds_get<E, LT, Cur::S, Cur::RP>(vi, li, t);
            xsync<XT>();
        }
        stages<E, LT, Cur::S, Cur::RP, TW, A>(vr, vi, t, tw, lo_g);
        later_passes<M, RB, P + 1, SPLIT, E, TW, A, SYNC_T>(vr, vi, lr, li, t, tw, lo_g);
    }
}

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ float load1(const float* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT>
__device__ __forceinline__ void store1(float* p, float v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT>
__device__ __forceinline__ v4f load4(const float* p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    else
        return *reinterpret_cast<const v4f*>(p);
}

template <bool NT>
__device__ __forceinline__ void store4(float* p, v4f v)
{
    if constexpr (NT)
        __builtin_nontemporal_store(v, reinterpret_cast<v4f*>(p));
    else
        *reinterpret_cast<v4f*>(p) = v;
}


}  // namespace
}  // namespace splitdft
