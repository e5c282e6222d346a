// Single-pass split-format FFT kernels for gfx950.
//
// Each workgroup owns `TPW` whole transforms of length N = 2^M.  Within a
// transform, thread t holds E = 2^RB complex elements as two register arrays
// (real plane, imaginary plane) and applies the factors of eq. (6) of the
// paper (Section III) in order:
//
//   S        bit reversal: folded into the global-load addresses, or into
//            the LDS reads of the first pass when the rows are staged;
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
// twiddles from the plan's table (entry 2^(i-1) + q holds omega^(i,q)), or
// from an equal-valued copy (a table slice or the quarter-turn table in LDS);
// in the first pass the twiddles with q = 0 (identity) and angle pi/2 (swap
// and negate) are applied as such, which gives the same values as the general
// form with the table's exact 1 and 0.  The results therefore equal, bit for
// bit, the factors of eq. (6) applied one after the other in FP32.
//
// Two kernels share this scheme: split_fft_lds_kernel (one block of TPW
// transforms per workgroup) and split_fft_pf_kernel (a resident grid looping
// over blocks, prefetching the next block's rows).  The same kernels also run
// the decimation-in-frequency factorisation of eq. (9) (Cfg::DIF).  Each
// compiled schedule is one Cfg; every length has a list of them, the first
// being the default.
#include "fft_device.h"

#include <atomic>
#include <climits>
#include <type_traits>

namespace splitdft {
namespace {

constexpr int kMaxDevices = 64;

// Compile-time schedule of one kernel instance.
//   M      log2 of the transform length
//   RB     log2 of the elements each thread holds (stages per full pass)
//   TPW    transforms per workgroup
//   SPLIT  exchange one plane at a time through LDS (half the LDS)
//   NT     nontemporal hints on the streaming global loads and stores
//   TWL    twiddles of passes >= 1: 0 read from the table in global memory;
//          staged once per workgroup in LDS: 1 table entries [2^RB, N),
//          2 the first quarter turn of stage M, in the bank-spreading slot
//          order of TwQuarterLds; 3 that quarter turn read from global memory
//          (TwQuarter)
//   WPE    minimum waves per SIMD the register allocation must allow (1 = any)
//   F4IO   global I/O as 16-byte vectors over the workgroup's contiguous
//          rows, staged through LDS: 0 none, 1 loads and stores, 2 loads only
//   PF     persistent workgroups with a grid-stride loop over blocks of TPW
//          transforms; the 16-byte loads of the next block are issued into
//          registers before the current block's passes (needs F4IO != 0)
//   DIF    the decimation-in-frequency factorisation, eq. (9): registers of
//          the first pass at natural positions (top bits first), stages m..1,
//          the bit reversal applied on the way out
template <int M_, int RB_, int TPW_, bool SPLIT_, bool NT_, int TWL_, int WPE_, int F4IO_ = 0, bool PF_ = false,
          bool DIF_ = false>
struct Cfg {
    static constexpr int M = M_, RB = RB_, TPW = TPW_, WPE = WPE_, TWL = TWL_;
    static constexpr bool SPLIT = SPLIT_, NT = NT_, PF = PF_, DIF = DIF_;
    static constexpr bool F4IN = F4IO_ != 0, F4OUT = F4IO_ == 1;
    static constexpr int F4IO = F4IO_;
    static constexpr int N = 1 << M;
    static constexpr int E = 1 << RB;
    static constexpr int LT = M - RB;
    static constexpr int T = 1 << LT;
    static constexpr int NP = (M + RB - 1) / RB;
    static constexpr int THREADS = TPW * T;
    // LDS words per transform: the padded length, made odd when one wave
    // spans many transforms so that their slots start on different banks
    static constexpr int SLOT = T >= 32 ? lds_index(N) : (lds_index(N) | 1);
    static constexpr bool USES_XCH = NP > 1 || F4IN;
    static constexpr int XCH_WORDS = USES_XCH ? TPW * SLOT * (SPLIT ? 1 : 2) : 1;
    // twiddle entries [2^RB, N) are the ones passes >= 1 read
    static constexpr int TW_LDS = (TWL == 1 && NP > 1) ? (N - E) : 0;
    // quarter-turn table of stage M
    static constexpr int TWQ = (TWL == 2 && NP > 1) ? (N / 4) : 0;
    static constexpr int LDS_BYTES = 4 * XCH_WORDS + 8 * TW_LDS + 8 * TWQ;
    static_assert(!F4IN || E >= 4, "16-byte I/O needs at least 4 elements per thread");
    static_assert(TWL < 2 || M >= 3, "the quarter-turn table needs N >= 8");
    static_assert(!PF || F4IN, "the prefetching form loads through the 16-byte staging");
};

// The quarter-turn table of stage M (entries [N/2, N/2 + N/4) of the plan's
// table) into LDS, entry k at TwQuarterLds slot k; consecutive k of one
// 32-entry run go to a permutation of that run, so the writes do not collide.
template <class C>
__device__ __forceinline__ void stage_quarter(const float2* __restrict__ tw, float2* lds_q, int tid)
{
    using Q = TwQuarterLds<(C::M >= 3 ? C::M : 3)>;
    const float2* src = tw + C::N / 2;
    for (int k = tid; k < C::TWQ; k += C::THREADS)
        lds_q[Q::slot(k)] = src[k];
}

// 16-byte loads of one plane of a sync group's rows (valid floats only) into
// LDS; float f of the group's block lands in slot f / N at lds_index(f mod N).
// GT threads share the work (a wave when transforms fit one wave, else the
// workgroup), so each group stages only the rows its own exchange syncs cover.
template <class C, int GT>
__device__ __forceinline__ void stage_in(const float* x, float* area, int64_t base, int valid, int gtid)
{
#pragma unroll
    for (int c = 0; c < C::E / 4; ++c) {
        const int f = 4 * (gtid + c * GT);
        if (f < valid) {
            const v4f v = load4<C::NT>(x + base + f);
            float* d = area + (f >> C::M) * C::SLOT + lds_index(f & (C::N - 1));
            d[0] = v[0];
            d[1] = v[1];
            d[2] = v[2];
            d[3] = v[3];
        }
    }
}

// stage_in in two steps, so that the loads can be issued early: the valid
// 16-byte vectors of one plane of a sync group's rows into registers ...
template <class C, int GT>
__device__ __forceinline__ void load_rows(v4f (&r)[C::E / 4], const float* x, int64_t base, int valid, int gtid)
{
#pragma unroll
    for (int c = 0; c < C::E / 4; ++c) {
        const int f = 4 * (gtid + c * GT);
        if (f < valid)
            r[c] = load4<C::NT>(x + base + f);
    }
}

// ... and from the registers into the LDS slots (layout of stage_in).
template <class C, int GT>
__device__ __forceinline__ void put_rows(const v4f (&r)[C::E / 4], float* area, int valid, int gtid)
{
#pragma unroll
    for (int c = 0; c < C::E / 4; ++c) {
        const int f = 4 * (gtid + c * GT);
        if (f < valid) {
            float* d = area + (f >> C::M) * C::SLOT + lds_index(f & (C::N - 1));
            d[0] = r[c][0];
            d[1] = r[c][1];
            d[2] = r[c][2];
            d[3] = r[c][3];
        }
    }
}

// The reverse of stage_in: LDS slots to 16-byte global stores.
template <class C, int GT>
__device__ __forceinline__ void stage_out(float* y, const float* area, int64_t base, int valid, int gtid)
{
#pragma unroll
    for (int c = 0; c < C::E / 4; ++c) {
        const int f = 4 * (gtid + c * GT);
        if (f < valid) {
            const float* s = area + (f >> C::M) * C::SLOT + lds_index(f & (C::N - 1));
            store4<C::NT>(y + base + f, v4f{s[0], s[1], s[2], s[3]});
        }
    }
}

// Registers of the first pass from an LDS slot holding a transform in
// natural order: position u + (t << RB) holds x[rev_LT(t) + (rev_RB(u) << LT)].
// (DIF: position j of the first DIF pass holds x[j].)
template <class C>
__device__ __forceinline__ void regs_from_natural(float (&v)[C::E], const float* slot_area, int t)
{
    if constexpr (C::DIF) {
        using First = PassD<C::M, C::RB, 0>;
#pragma unroll
        for (int u = 0; u < C::E; ++u)
            v[u] = slot_area[lds_index(position<C::LT, First::S, First::RP>(t, u))];
    } else {
        const int tb = rev_bits(t, C::LT);
#pragma unroll
        for (int u = 0; u < C::E; ++u)
            v[u] = slot_area[lds_index(tb + (rev_bits(u, C::RB) << C::LT))];
    }
}

// The last pass's registers into an LDS slot in natural output order (DIF:
// position j is output rev_M(j)).
template <class C>
__device__ __forceinline__ void regs_to_natural(const float (&v)[C::E], float* slot_area, int t)
{
    if constexpr (C::DIF) {
        using Last = PassD<C::M, C::RB, C::NP - 1>;
#pragma unroll
        for (int u = 0; u < C::E; ++u)
            slot_area[lds_index(rev_bits(position<C::LT, Last::S, Last::RP>(t, u), C::M))] = v[u];
    } else {
        using Last = Pass<C::M, C::RB, C::NP - 1>;
#pragma unroll
        for (int u = 0; u < C::E; ++u)
            slot_area[lds_index(position<C::LT, Last::S, Last::RP>(t, u))] = v[u];
    }
}

// Direct stores of the last pass (T > 1): DIT positions are natural output
// indices; a DIF position j is output rev_M(j) (last pass on bits
// 0..RB-1: rev_M(u + (t << RB)) = (rev_RB(u) << LT) + rev_LT(t), coalesced
// over t).
template <class C>
__device__ __forceinline__ void store_last(float* yr, float* yi, int64_t row, const float (&vr)[C::E],
                                           const float (&vi)[C::E], int t)
{
    if constexpr (C::DIF) {
        using Last = PassD<C::M, C::RB, C::NP - 1>;
#pragma unroll
        for (int u = 0; u < C::E; ++u) {
            const int64_t idx = row + rev_bits(position<C::LT, Last::S, Last::RP>(t, u), C::M);
            store1<C::NT>(yr + idx, vr[u]);
            store1<C::NT>(yi + idx, vi[u]);
        }
    } else {
        using Last = Pass<C::M, C::RB, C::NP - 1>;
#pragma unroll
        for (int u = 0; u < C::E; ++u) {
            const int64_t idx = row + position<C::LT, Last::S, Last::RP>(t, u);
            store1<C::NT>(yr + idx, vr[u]);
            store1<C::NT>(yi + idx, vi[u]);
        }
    }
}

// Every stage of the transform on the registers (first pass included), in the
// order of eq. (6) (DIT) or eq. (9) (DIF).  lds_tw: the twiddles staged in LDS
// (TWL 1 or 2), else unused.
template <class C>
__device__ __forceinline__ void run_stages(float (&vr)[C::E], float (&vi)[C::E], float* lr, float* li, int t,
                                           const float2* __restrict__ tw, const float2* lds_tw)
{
    constexpr int M = C::M, RB = C::RB, E = C::E, LT = C::LT;
    using TW = typename std::conditional<
        (C::TW_LDS > 0), TwTable<E>,
        typename std::conditional<
            (C::TWQ > 0), TwQuarterLds<(M >= 3 ? M : 3)>,
            typename std::conditional<(C::TWL == 3), TwQuarter<(M >= 3 ? M : 3)>, TwTable<0>>::type>::type>::type;
    const float2* tws = (C::TW_LDS > 0 || C::TWQ > 0) ? lds_tw : (C::TWL == 3 ? tw + C::N / 2 : tw);
    if constexpr (C::DIF) {
        using First = PassD<M, RB, 0>;
        stages_dif<E, LT, First::S, First::RP, TW>(vr, vi, t, tw, tws);
        if constexpr (C::NP > 1)
            later_passes_dif<M, RB, 1, C::SPLIT, E, TW>(vr, vi, lr, li, t, tw, tws);
        // a last exchange ordered per wave: other waves may still be reading
        // slots that the next LDS writes (output staging, next block) reuse
        if constexpr (C::NP > 1 && dif_last_exchange_local<M, RB>())
            __syncthreads();
    } else {
        stages<E, LT, 0, Pass<M, RB, 0>::RP>(vr, vi, t, tw);
        if constexpr (C::NP > 1)
            later_passes<M, RB, 1, C::SPLIT, E, TW>(vr, vi, lr, li, t, tws);
    }
}

// DUAL: the grid covers two directions over the same rows, the first
// ceil(batch / TPW) workgroups the planes (xr, xi, yr, yi), the rest those of
// d2 (a fused forward + adjoint); otherwise d2 is unused.
template <class C, bool DUAL>
__global__ void __launch_bounds__(C::THREADS) __attribute__((amdgpu_waves_per_eu(C::WPE)))
split_fft_lds_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                     int64_t batch, const int64_t* __restrict__ rows, Dir2 d2)
{
    constexpr int M = C::M, RB = C::RB, TPW = C::TPW;
    constexpr int N = C::N, E = C::E, LT = C::LT, T = C::T, NP = C::NP;
    constexpr bool NT = C::NT;
    __shared__ float lds[C::XCH_WORDS];
    __shared__ v4f lds_tw4[C::TW_LDS > 0 ? C::TW_LDS / 2 : (C::TWQ > 0 ? C::TWQ / 2 : 1)];

    const int tid = threadIdx.x;
    const int slot = tid >> LT;
    const int t = tid & (T - 1);
    int64_t wg = blockIdx.x;
    if constexpr (DUAL) {
        const int64_t nb = (batch + TPW - 1) / TPW;
        if (wg >= nb) {
            wg -= nb;
            xr = d2.xr;
            xi = d2.xi;
            yr = d2.yr;
            yi = d2.yi;
        }
    }
    const int64_t b0 = wg * TPW;
    const int64_t b = b0 + slot;
    const bool active = b < batch;
    // rows (one transform per workgroup only): element offset of each transform
    const bool indirect = TPW == 1 && rows != nullptr;
    const int64_t row = indirect ? (active ? rows[b] : 0) : b * N;
    float* lr = lds + slot * C::SLOT;
    float* li = C::SPLIT ? lr : lr + TPW * C::SLOT;
    // sync group of the LDS exchanges: one wave when a transform fits in it
    constexpr int GT = (T <= 64) ? (C::THREADS < 64 ? C::THREADS : 64) : C::THREADS;
    constexpr int GSLOTS = GT / T;
    const int gtid = tid & (GT - 1);
    const int gslot0 = (tid / GT) * GSLOTS;

    // Stage the twiddles of passes >= 1 (entries [E, N)) in LDS, entry idx
    // at LDS element idx - E, before the data loads are issued, so that the
    // barrier making them visible waits only for the table's own loads.
    if constexpr (C::TW_LDS > 0) {
        const v4f* src = reinterpret_cast<const v4f*>(tw + E);
        for (int k = tid; k < C::TW_LDS / 2; k += C::THREADS)
            lds_tw4[k] = src[k];
        __syncthreads();
    } else if constexpr (C::TWQ > 0) {
        stage_quarter<C>(tw, reinterpret_cast<float2*>(lds_tw4), tid);
        __syncthreads();
    }

    float vr[E], vi[E];
    if constexpr (C::F4IN) {
        const int64_t rows_left = batch - (b0 + gslot0);
        const int valid = static_cast<int>(rows_left < GSLOTS ? (rows_left > 0 ? rows_left : 0) : GSLOTS) * N;
        const int64_t base = indirect ? row : (b0 + gslot0) * N;
        float* gr = lds + gslot0 * C::SLOT;
        if constexpr (C::SPLIT) {
            // both planes' loads in flight at once; LDS holds one plane at a time
            v4f pr[E / 4], pi[E / 4];
            load_rows<C, GT>(pr, xr, base, valid, gtid);
            load_rows<C, GT>(pi, xi, base, valid, gtid);
            put_rows<C, GT>(pr, gr, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vr, lr, t);
            xsync<T>();
            put_rows<C, GT>(pi, gr, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vi, lr, t);
        } else {
            stage_in<C, GT>(xr, gr, base, valid, gtid);
            stage_in<C, GT>(xi, gr + TPW * C::SLOT, base, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vr, lr, t);
            regs_from_natural<C>(vi, li, t);
        }
        // the next LDS writes (exchange or output staging) reuse these slots
        xsync<T>();
    } else if constexpr (T == 1) {
        // A whole transform per thread: natural-order vector loads; the bit
        // reversal is a renaming of registers.
        // (DIF: no reversal on the way in; it is applied to the stores.)
        constexpr int RIN = C::DIF ? 0 : M;
        if (active) {
            if constexpr (N >= 4) {
#pragma unroll
                for (int c = 0; c < N / 4; ++c) {
                    const v4f a = load4<NT>(xr + row + 4 * c), z = load4<NT>(xi + row + 4 * c);
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        vr[RIN ? rev_bits(4 * c + e, RIN) : 4 * c + e] = a[e];
                        vi[RIN ? rev_bits(4 * c + e, RIN) : 4 * c + e] = z[e];
                    }
                }
            } else {
#pragma unroll
                for (int n = 0; n < N; ++n) {
                    vr[RIN ? rev_bits(n, RIN) : n] = load1<NT>(xr + row + n);
                    vi[RIN ? rev_bits(n, RIN) : n] = load1<NT>(xi + row + n);
                }
            }
        } else {
#pragma unroll
            for (int u = 0; u < E; ++u)
                vr[u] = vi[u] = 0.0f;
        }
    } else if constexpr (C::DIF) {
        // position j of the first DIF pass holds x[j]: coalesced over t
        using First = PassD<M, RB, 0>;
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t idx = row + position<LT, First::S, First::RP>(t, u);
            vr[u] = active ? load1<NT>(xr + idx) : 0.0f;
            vi[u] = active ? load1<NT>(xi + idx) : 0.0f;
        }
    } else {
        // Position u + (t << RB) holds x[rev_M(u + (t << RB))]
        //   = x[rev_LT(t) + (rev_RB(u) << LT)].
        const int tb = rev_bits(t, LT);
#pragma unroll
        for (int u = 0; u < E; ++u) {
            const int64_t idx = row + tb + (rev_bits(u, RB) << LT);
            vr[u] = active ? load1<NT>(xr + idx) : 0.0f;
            vi[u] = active ? load1<NT>(xi + idx) : 0.0f;
        }
    }

    run_stages<C>(vr, vi, lr, li, t, tw, reinterpret_cast<const float2*>(lds_tw4));

    if constexpr (C::F4OUT) {
        const int64_t rows_left = batch - (b0 + gslot0);
        const int valid = static_cast<int>(rows_left < GSLOTS ? (rows_left > 0 ? rows_left : 0) : GSLOTS) * N;
        const int64_t base = indirect ? row : (b0 + gslot0) * N;
        float* gr = lds + gslot0 * C::SLOT;
        if constexpr (C::SPLIT) {
            regs_to_natural<C>(vr, lr, t);
            xsync<T>();
            stage_out<C, GT>(yr, gr, base, valid, gtid);
            xsync<T>();
            regs_to_natural<C>(vi, lr, t);
            xsync<T>();
            stage_out<C, GT>(yi, gr, base, valid, gtid);
        } else {
            regs_to_natural<C>(vr, lr, t);
            regs_to_natural<C>(vi, li, t);
            xsync<T>();
            stage_out<C, GT>(yr, gr, base, valid, gtid);
            stage_out<C, GT>(yi, gr + TPW * C::SLOT, base, valid, gtid);
        }
        return;
    }

    if (!active)
        return;
    if constexpr (T == 1) {
        // (DIF: output k is register rev_M(k).)
        constexpr int ROUT = C::DIF ? M : 0;
        auto reg = [](int k) { return ROUT ? rev_bits(k, ROUT) : k; };
        if constexpr (N >= 4) {
#pragma unroll
            for (int c = 0; c < N / 4; ++c) {
                store4<NT>(yr + row + 4 * c, v4f{vr[reg(4 * c)], vr[reg(4 * c + 1)], vr[reg(4 * c + 2)],
                                                 vr[reg(4 * c + 3)]});
                store4<NT>(yi + row + 4 * c, v4f{vi[reg(4 * c)], vi[reg(4 * c + 1)], vi[reg(4 * c + 2)],
                                                 vi[reg(4 * c + 3)]});
            }
        } else {
#pragma unroll
            for (int n = 0; n < N; ++n) {
                store1<NT>(yr + row + n, vr[reg(n)]);
                store1<NT>(yi + row + n, vi[reg(n)]);
            }
        }
    } else {
        store_last<C>(yr, yi, row, vr, vi, t);
    }
}

// The values must exist in registers at this point of the program.
template <int E>
__device__ __forceinline__ void pin_regs(float (&v)[E])
{
#pragma unroll
    for (int u = 0; u < E; ++u)
        asm volatile("" : "+v"(v[u]));
}

// Persistent form of split_fft_lds_kernel (C::PF): the same arithmetic and
// data movement per block of TPW transforms, but each workgroup loops over
// blocks blockIdx.x, blockIdx.x + gridDim.x, ...  The twiddles are staged in
// LDS once per workgroup, and the 16-byte loads of the next block go into
// registers right after the current block has left them, so that they are
// in flight during the current block's passes and stores.  DUAL: blocks
// ceil(batch / TPW) and up run on the planes of d2 (as in
// split_fft_lds_kernel).
template <class C, bool DUAL>
__global__ void __launch_bounds__(C::THREADS) __attribute__((amdgpu_waves_per_eu(C::WPE)))
split_fft_pf_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                    int64_t batch, const int64_t* __restrict__ rows, Dir2 d2)
{
    constexpr int M = C::M, RB = C::RB, TPW = C::TPW;
    constexpr int N = C::N, E = C::E, LT = C::LT, T = C::T, NP = C::NP;
    constexpr bool NT = C::NT;
    static_assert(C::PF && C::F4IN, "persistent form of the staged-load schedules");
    __shared__ float lds[C::XCH_WORDS];
    __shared__ v4f lds_tw4[C::TW_LDS > 0 ? C::TW_LDS / 2 : (C::TWQ > 0 ? C::TWQ / 2 : 1)];
    const int tid = threadIdx.x;
    const int slot = tid >> LT;
    const int t0 = tid & (T - 1);
    float* lr = lds + slot * C::SLOT;
    float* li = C::SPLIT ? lr : lr + TPW * C::SLOT;
    constexpr int GT = (T <= 64) ? (C::THREADS < 64 ? C::THREADS : 64) : C::THREADS;
    constexpr int GSLOTS = GT / T;
    const int gtid = tid & (GT - 1);
    const int gslot0 = (tid / GT) * GSLOTS;
    float* gr = lds + gslot0 * C::SLOT;
    float* gi = C::SPLIT ? gr : gr + TPW * C::SLOT;

    if constexpr (C::TW_LDS > 0) {
        const v4f* src = reinterpret_cast<const v4f*>(tw + E);
        for (int k = tid; k < C::TW_LDS / 2; k += C::THREADS)
            lds_tw4[k] = src[k];
        __syncthreads();
    } else if constexpr (C::TWQ > 0) {
        stage_quarter<C>(tw, reinterpret_cast<float2*>(lds_tw4), tid);
        __syncthreads();
    }

    const int64_t nb = (batch + TPW - 1) / TPW;  // blocks of one direction
    const int64_t blocks = DUAL ? 2 * nb : nb;
    // block of its own direction, and that direction's planes
    auto local = [&](int64_t blk) { return (DUAL && blk >= nb) ? blk - nb : blk; };
    auto src_r = [&](int64_t blk) { return (DUAL && blk >= nb) ? d2.xr : xr; };
    auto src_i = [&](int64_t blk) { return (DUAL && blk >= nb) ? d2.xi : xi; };
    // rows (one transform per workgroup only): element offset of each transform
    const bool indirect = TPW == 1 && rows != nullptr;
    auto group_base = [&](int64_t blk) {
        const int64_t lb = local(blk);
        return indirect ? rows[lb] : (lb * TPW + gslot0) * N;
    };
    // floats of the sync group's rows that exist in block blk
    auto group_valid = [&](int64_t blk) {
        const int64_t rows_left = batch - (local(blk) * TPW + gslot0);
        return static_cast<int>(rows_left < GSLOTS ? (rows_left > 0 ? rows_left : 0) : GSLOTS) * N;
    };

    v4f pr[E / 4], pi[E / 4];
    int64_t blk = blockIdx.x;
    // With one transform per workgroup the offsets of the next two blocks are
    // carried (uniform values), so that an offset read from `rows` has arrived
    // by the time the prefetch needs it.
    int64_t ahead[2] = {0, 0};
    if (blk < blocks) {
        const int valid = group_valid(blk);
        const int64_t base = group_base(blk);
        load_rows<C, GT>(pr, src_r(blk), base, valid, gtid);
        load_rows<C, GT>(pi, src_i(blk), base, valid, gtid);
        if constexpr (TPW == 1) {
            ahead[0] = base;
            if (blk + gridDim.x < blocks)
                ahead[1] = group_base(blk + gridDim.x);
        }
    }
    for (; blk < blocks; blk += gridDim.x) {
        const int valid = group_valid(blk);
        const int64_t base = TPW == 1 ? ahead[0] : group_base(blk);
        float* dst_r = (DUAL && blk >= nb) ? d2.yr : yr;
        float* dst_i = (DUAL && blk >= nb) ? d2.yi : yi;
        // the position and twiddle addresses below depend only on t; an
        // opaque copy per iteration keeps the compiler from hoisting all of
        // them out of the loop into registers that the prefetch needs
        int t = t0;
        asm volatile("" : "+v"(t));
        float vr[E], vi[E];
        if constexpr (C::SPLIT) {
            put_rows<C, GT>(pr, gr, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vr, lr, t);
            xsync<T>();
            put_rows<C, GT>(pi, gr, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vi, lr, t);
        } else {
            put_rows<C, GT>(pr, gr, valid, gtid);
            put_rows<C, GT>(pi, gi, valid, gtid);
            xsync<T>();
            regs_from_natural<C>(vr, lr, t);
            regs_from_natural<C>(vi, li, t);
        }
        // The LDS reads above must complete before the barrier: the compiler
        // has been seen to sink them past it into the block after the
        // prefetch branch, where faster waves already overwrite the slots.
        // Taking the values through an opaque definition here pins them.
        pin_regs<E>(vr);
        pin_regs<E>(vi);
        xsync<T>();

        // the next block's loads, in flight during this block's work
        const int64_t nblk = blk + gridDim.x;
        if (nblk < blocks) {
            const int nvalid = group_valid(nblk);
            const int64_t nbase = TPW == 1 ? ahead[1] : group_base(nblk);
            load_rows<C, GT>(pr, src_r(nblk), nbase, nvalid, gtid);
            load_rows<C, GT>(pi, src_i(nblk), nbase, nvalid, gtid);
        }
        if constexpr (TPW == 1) {
            ahead[0] = ahead[1];
            ahead[1] = nblk + gridDim.x < blocks ? group_base(nblk + gridDim.x) : 0;
        }

        run_stages<C>(vr, vi, lr, li, t, tw, reinterpret_cast<const float2*>(lds_tw4));

        if constexpr (C::F4OUT) {
            if constexpr (C::SPLIT) {
                regs_to_natural<C>(vr, lr, t);
                xsync<T>();
                stage_out<C, GT>(dst_r, gr, base, valid, gtid);
                xsync<T>();
                regs_to_natural<C>(vi, lr, t);
                xsync<T>();
                stage_out<C, GT>(dst_i, gr, base, valid, gtid);
            } else {
                regs_to_natural<C>(vr, lr, t);
                regs_to_natural<C>(vi, li, t);
                xsync<T>();
                stage_out<C, GT>(dst_r, gr, base, valid, gtid);
                stage_out<C, GT>(dst_i, gi, base, valid, gtid);
            }
            // the next block's put_rows reuses the slots
            xsync<T>();
        } else {
            // the last exchange ended with a sync, so the slots are free
            const int64_t b = local(blk) * TPW + slot;
            if (b < batch)
                store_last<C>(dst_r, dst_i, indirect ? base : b * N, vr, vi, t);
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
                       const int64_t* rows, hipStream_t stream, const Dir2* second)
{
    if (rows)
        return hipErrorInvalidValue;
    const int64_t blocks = (batch + 255) / 256;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(split_fft_len1_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, xr, xi, yr,
                       yi, batch);
    if (second)
        hipLaunchKernelGGL(split_fft_len1_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream,
                           second->xr, second->xi, second->yr, second->yi, batch);
    return hipGetLastError();
}

template <class C>
hipError_t launch_lds(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                      const int64_t* rows, hipStream_t stream, const Dir2* second)
{
    if (rows && C::TPW != 1)
        return hipErrorInvalidValue;
    const int64_t blocks = (batch + C::TPW - 1) / C::TPW;
    if (blocks > INT_MAX / 2)
        return hipErrorInvalidConfiguration;
    if (second)
        hipLaunchKernelGGL((split_fft_lds_kernel<C, true>), dim3(static_cast<unsigned>(2 * blocks)),
                           dim3(C::THREADS), 0, stream, xr, xi, yr, yi, tw, batch, rows, *second);
    else
        hipLaunchKernelGGL((split_fft_lds_kernel<C, false>), dim3(static_cast<unsigned>(blocks)), dim3(C::THREADS),
                           0, stream, xr, xi, yr, yi, tw, batch, rows, Dir2{});
    return hipGetLastError();
}

// Workgroups of the persistent form: as many as can be resident at once.
template <class C, bool DUAL>
hipError_t launch_pf_dir(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                         const int64_t* rows, hipStream_t stream, const Dir2& second)
{
    const int64_t blocks = (batch + C::TPW - 1) / C::TPW * (DUAL ? 2 : 1);
    // resident workgroups per device, looked up once (launches are frequent)
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
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, split_fft_pf_kernel<C, DUAL>, C::THREADS, 0);
        if (e != hipSuccess)
            return e;
        if (per_cu < 1 || cus < 1)
            return hipErrorInvalidConfiguration;
        resident = cus * per_cu;
        if (dev >= 0 && dev < kMaxDevices)
            resident_of[dev].store(resident, std::memory_order_relaxed);
    }
    const int64_t grid = blocks < resident ? blocks : resident;
    hipLaunchKernelGGL((split_fft_pf_kernel<C, DUAL>), dim3(static_cast<unsigned>(grid)), dim3(C::THREADS), 0,
                       stream, xr, xi, yr, yi, tw, batch, rows, second);
    return hipGetLastError();
}

template <class C>
hipError_t launch_pf(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                     const int64_t* rows, hipStream_t stream, const Dir2* second)
{
    if (rows && C::TPW != 1)
        return hipErrorInvalidValue;
    if (second)
        return launch_pf_dir<C, true>(xr, xi, yr, yi, tw, batch, rows, stream, *second);
    return launch_pf_dir<C, false>(xr, xi, yr, yi, tw, batch, rows, stream, Dir2{});
}

template <class C>
constexpr Variant make_variant()
{
    if constexpr (C::PF)
        return Variant{C::M,  C::RB,  C::TPW, C::THREADS, C::LDS_BYTES,  C::SPLIT,
                       C::NT, C::TWL, C::WPE, C::F4IO,    &launch_pf<C>, true,     C::TPW == 1};
    else
        return Variant{C::M,  C::RB,  C::TPW, C::THREADS, C::LDS_BYTES,   C::SPLIT,
                       C::NT, C::TWL, C::WPE, C::F4IO,    &launch_lds<C>, false,    C::TPW == 1};
}

// Compiled schedules per length; the first entry of each list is the default.
//                              M   RB  TPW  SPLIT  NT     TWL    WPE
const Variant kV0[] = {Variant{0, 0, 256, 256, 0, false, false, false, 1, false, &launch_len1}};
template <int M, int RB, int TPW, bool SPLIT, bool NT, int TWL, int WPE, int F4IO = 0, bool PF = false>
constexpr Variant V()
{
    return make_variant<Cfg<M, RB, TPW, SPLIT, NT, TWL, WPE, F4IO, PF>>();
}

// decimation-in-frequency schedules (eq. 9)
template <int M, int RB, int TPW, bool SPLIT, bool NT, int TWL, int WPE, int F4IO = 0, bool PF = false>
constexpr Variant DV()
{
    return make_variant<Cfg<M, RB, TPW, SPLIT, NT, TWL, WPE, F4IO, PF, true>>();
}

constexpr bool Y = true, _ = false;
//                      M   RB TPW SPLIT NT TWL WPE F4IO
const Variant kV1[] = {V<1, 1, 256, _, _, _, 1>()};
const Variant kV2[] = {V<2, 2, 256, _, _, _, 1>()};
const Variant kV3[] = {V<3, 3, 256, _, _, _, 1>()};
const Variant kV4[] = {V<4, 4, 64, _, Y, _, 4, 1, Y>(), V<4, 4, 64, _, Y, _, 1, Y>(), V<4, 4, 256, _, Y, _, 4, 1, Y>(),
                       V<4, 4, 64, _, _, _, 1>()};
const Variant kV5[] = {V<5, 4, 64, _, Y, 2, 4, 1, Y>(), V<5, 4, 64, _, Y, Y, 1, Y>(), V<5, 5, 128, _, _, _, 1>()};
const Variant kV6[] = {V<6, 4, 64, _, Y, 2, 4, 1, Y>(), V<6, 4, 32, _, Y, 2, 4, 1, Y>(), V<6, 4, 64, _, Y, Y, 1, Y>(),
                       V<6, 3, 32, _, _, _, 1>()};
const Variant kV7[] = {V<7, 4, 32, Y, Y, 2, 4, 1, Y>(), V<7, 4, 16, _, Y, 2, 4, 1, Y>(), V<7, 4, 16, _, Y, Y, 1, Y>(),
                       V<7, 4, 32, _, _, _, 1>()};
const Variant kV8[] = {V<8, 4, 16, Y, Y, Y, 4, Y>(), V<8, 4, 16, Y, Y, 2, 4, 1, Y>(), V<8, 4, 32, Y, Y, 2, 4, 1, Y>(),
                       V<8, 4, 16, _, _, _, 1>()};
const Variant kV9[] = {V<9, 4, 8, Y, Y, 2, 4, 1, Y>(), V<9, 4, 8, Y, Y, 2, 4, 2, Y>(), V<9, 4, 4, Y, Y, 2, 4, 2, Y>(),
                       V<9, 4, 8, Y, Y, Y, 4, Y>(),    V<9, 4, 8, _, Y, Y, 1>(),       V<9, 4, 8, Y, Y, 2, 4, 2>()};
const Variant kV10[] = {V<10, 4, 4, _, Y, 2, 4, 2, Y>(), V<10, 4, 4, Y, Y, 2, 4, 2, Y>(), V<10, 4, 4, Y, Y, 1, 4, 2, Y>(),
                        V<10, 4, 4, Y, Y, 2, 3, 2, Y>(), V<10, 4, 8, Y, Y, 2, 3, 2, Y>(), V<10, 4, 2, Y, Y, 2, 4, 2, Y>(),
                        V<10, 4, 8, Y, Y, 2, 4, 2, Y>(), V<10, 4, 8, Y, Y, Y, 4>(),       V<10, 5, 8, Y, Y, Y, 1>(),
                        V<10, 4, 4, Y, Y, 2, 4, 2>(),    V<10, 4, 8, Y, Y, 2, 4, 2>(),    V<10, 5, 8, Y, Y, 2, 2, 2>(),
                        V<10, 5, 4, Y, Y, 2, 2, 2>(),    V<10, 5, 8, _, Y, 2, 2, 2>(),    V<10, 5, 4, Y, Y, 2, 2, 2, Y>(),
                        V<10, 5, 8, Y, Y, 2, 3, 2>(),
                        V<10, 4, 1, Y, Y, 2, 4, 2, Y>()};
const Variant kV11[] = {V<11, 4, 2, Y, Y, 2, 4, 2>(),    V<11, 4, 1, Y, Y, 2, 4, 2>(),    V<11, 4, 1, Y, Y, 2, 4, 2, Y>(),
                        V<11, 4, 2, Y, Y, 2, 4, 2, Y>(), V<11, 4, 2, Y, Y, 2, 4>(),       V<11, 5, 4, Y, Y, Y, 1>()};
const Variant kV12[] = {V<12, 4, 1, Y, Y, 2, 4, 2>(),    V<12, 5, 2, Y, Y, 2, 2>(),    V<12, 4, 1, Y, Y, 2, 3, 2, Y>(),
                        V<12, 5, 2, Y, Y, Y, 2>(),       V<12, 5, 1, Y, Y, 2, 2, 2>(), V<12, 4, 2, Y, Y, 2, 4, 2>()};
const Variant kV13[] = {V<13, 4, 1, Y, Y, 2, 4, 2>(),    V<13, 5, 1, Y, Y, 0, 2, 2>(), V<13, 5, 1, Y, Y, 2, 2, 2>(),
                        V<13, 4, 1, Y, Y, 2, 4, 2, Y>(), V<13, 5, 1, Y, Y, 2, 4, 2>(), V<13, 5, 1, _, Y, _, 1>()};
const Variant kV14[] = {V<14, 4, 1, Y, Y, 2, 1, 1, Y>(), V<14, 4, 1, Y, Y, 2, 1, 2, Y>(), V<14, 4, 1, Y, Y, 3, 1, 2, Y>(),
                        V<14, 5, 1, Y, Y, 2, 2, 2, Y>(), V<14, 4, 1, Y, Y, 2, 1, 2>(),    V<14, 5, 1, Y, Y, 3, 4, 2>(),
                        V<14, 5, 1, Y, Y, 3, 2, 2>(),    V<14, 5, 1, Y, Y, 2, 2, 2>()};
const Variant kV15[] = {V<15, 5, 1, Y, Y, 3, 1, 2>(), V<15, 5, 1, Y, Y, _, 1>()};

struct VariantList {
    const Variant* v;
    int count;
};

#define SDFT_L(a) VariantList{a, static_cast<int>(sizeof(a) / sizeof(a[0]))}
const VariantList kLists[] = {SDFT_L(kV0),  SDFT_L(kV1),  SDFT_L(kV2),  SDFT_L(kV3),  SDFT_L(kV4),  SDFT_L(kV5),
                              SDFT_L(kV6),  SDFT_L(kV7),  SDFT_L(kV8),  SDFT_L(kV9),  SDFT_L(kV10), SDFT_L(kV11),
                              SDFT_L(kV12), SDFT_L(kV13), SDFT_L(kV14), SDFT_L(kV15)};

// decimation-in-frequency schedules; the first entry of each list is the default
//                      M   RB TPW SPLIT NT TWL WPE F4IO PF
const Variant kD1[] = {DV<1, 1, 256, _, _, _, 1>()};
const Variant kD2[] = {DV<2, 2, 256, _, _, _, 1>()};
const Variant kD3[] = {DV<3, 3, 256, _, _, _, 1>()};
const Variant kD4[] = {DV<4, 4, 64, _, Y, _, 4, 1, Y>(), DV<4, 4, 64, _, _, _, 1>()};
const Variant kD5[] = {DV<5, 4, 64, _, Y, 2, 4, 1, Y>(), DV<5, 4, 64, _, _, _, 1>()};
const Variant kD6[] = {DV<6, 4, 64, _, Y, 2, 4, 1, Y>(), DV<6, 4, 32, _, _, _, 1>()};
const Variant kD7[] = {DV<7, 4, 32, Y, Y, 2, 4, 1, Y>(), DV<7, 4, 16, _, _, _, 1>()};
const Variant kD8[] = {DV<8, 4, 16, Y, Y, 2, 4, 1, Y>(), DV<8, 4, 16, Y, _, _, 4>()};
const Variant kD9[] = {DV<9, 4, 8, Y, Y, 2, 4, 1, Y>(), DV<9, 4, 8, Y, Y, 2, 4, 2, Y>(), DV<9, 4, 8, Y, Y, _, 4>()};
const Variant kD10[] = {DV<10, 4, 4, _, Y, 2, 4, 2, Y>(), DV<10, 4, 4, _, Y, 2, 4, 1, Y>(), DV<10, 4, 4, Y, Y, _, 4>()};
// (the last DIF pass scatters its direct stores once T > 64: stage them)
const Variant kD11[] = {DV<11, 4, 2, Y, Y, 2, 4, 1>(), DV<11, 4, 2, Y, Y, 2, 4, 2>(), DV<11, 4, 2, Y, Y, _, 4>()};
const Variant kD12[] = {DV<12, 4, 1, Y, Y, 2, 4, 1>(), DV<12, 4, 2, Y, Y, 2, 4, 1>(), DV<12, 4, 1, Y, Y, _, 4>()};
const Variant kD13[] = {DV<13, 5, 1, Y, Y, 2, 2, 1>(), DV<13, 4, 1, Y, Y, 2, 4, 1>()};
const Variant kD14[] = {DV<14, 4, 1, Y, Y, 2, 1, 1, Y>(), DV<14, 4, 1, Y, Y, 2, 1, 1>()};

const VariantList kDLists[] = {SDFT_L(kV0),  SDFT_L(kD1),  SDFT_L(kD2),  SDFT_L(kD3),  SDFT_L(kD4),
                               SDFT_L(kD5),  SDFT_L(kD6),  SDFT_L(kD7),  SDFT_L(kD8),  SDFT_L(kD9),
                               SDFT_L(kD10), SDFT_L(kD11), SDFT_L(kD12), SDFT_L(kD13), SDFT_L(kD14)};
#undef SDFT_L

}  // namespace

const Variant* dif_variants_for(int m, int* count)
{
    if (m < 0 || m >= static_cast<int>(sizeof(kDLists) / sizeof(kDLists[0]))) {
        *count = 0;
        return nullptr;
    }
    *count = kDLists[m].count;
    return kDLists[m].v;
}

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
