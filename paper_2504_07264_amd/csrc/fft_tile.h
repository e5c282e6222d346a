// Device code of one tile of the two-pass schedule (see fft_tile.hip for the
// decomposition of eq. (6) into the two passes).
#pragma once

#include "fft_device.h"

#include <type_traits>

namespace splitdft {
namespace {

// GF: lanes run over the tile's groups first (thread t of group g is
// tid = g + C * t), so that the per-group twiddles of pass 2 (index
// lo + (ql << A), lo = the group's column) are contiguous across a wave; the
// groups then span waves and exchanges use workgroup barriers.
//
// WSC: layout of the workspace between the passes.  0: natural position
// order (pass 1 writes whole blocks, pass 2 reads rows of C columns strided by
// 2^A).  WSC = pass 2's C: "tiled", position c 2^A + p of a transform at
//     (p / WSC) (2^(M-A) WSC) + rev_(M-A)(c) WSC + p mod WSC,
// so that one pass-2 tile (WSC columns, all rows) is one contiguous run and a
// pass-1 tile (consecutive input columns k = rev(c)) writes runs of
// C1 x WSC floats.  Pass 2 puts run row k at tile row rev_(M-A)(k).
template <int M_, int A_, int PASS_, int RB_, int C_, bool SPLIT_, bool GF_ = false, int WSC_ = 0>
struct TileCfg {
    static constexpr int M = M_, A = A_, PASS = PASS_, RB = RB_, C = C_, WSC = WSC_;
    static constexpr bool SPLIT = SPLIT_, GF = GF_;
    static constexpr int N = 1 << M;
    static constexpr int MA = PASS == 1 ? A : M - A;  // log2 positions per group
    static constexpr int R = 1 << MA;
    static constexpr int E = 1 << RB;
    static constexpr int LT = MA - RB;
    static constexpr int T = 1 << LT;  // threads per group
    static constexpr int NP = (MA + RB - 1) / RB;
    static constexpr int THREADS = C * T;
    static constexpr int SLOT = lds_index(R) | 1;
    static constexpr int LDS_WORDS = C * SLOT * (SPLIT ? 1 : 2);
    static constexpr int TW_SHIFT = PASS == 1 ? 0 : A;
    static constexpr int GROUPS = PASS == 1 ? (1 << (M - A)) : (1 << A);  // per transform
    static constexpr int TILES = GROUPS / C;                               // per transform
    static constexpr int R2 = 1 << (M - A);  // rows of a pass-2 column (blocks of pass 1)
    static_assert(C % 4 == 0 && E >= 4 && GROUPS % C == 0, "tile shape");
    static_assert(M <= 16, "32-bit offsets within a transform");
    static_assert(WSC == 0 || (WSC % 4 == 0 && (1 << A) % WSC == 0 && (PASS == 1 || WSC == C)),
                  "tiled workspace: pass 2's tile width");
};

// Tile row of source row r (the tiled workspace stores pass-2 rows in
// bit-reversed order).
template <class TC>
__device__ __forceinline__ int tile_lds_row(int r)
{
    if constexpr (TC::PASS == 2 && TC::WSC > 0)
        return rev_bits(r, TC::MA);
    else
        return r;
}

// The columns of one tile.  Tile column i is column (col0 - rot + i) mod
// GROUPS of the pass.  Pass 1 reads its rows of C floats straight from the
// data; rotating the windows by the data's offset from a 128-byte line (rot
// floats, a multiple of 4) makes each of those segments start on a line,
// wherever the transform sits.  (Pass 2 is not rotated: its data side is
// the stores, which lose little to a misaligned start, and its rotated build
// needs more registers than that gains.)  TileCols<false> is the unrotated
// case, with rot = 0 known at compile time.
template <bool ROT>
struct TileCols {
    static constexpr bool ROTATES = true;
    int col0;  // C x tile index
    int rot;   // rotation of the columns
};
template <>
struct TileCols<false> {
    static constexpr bool ROTATES = false;
    static constexpr int rot = 0;
    int col0;
};

template <class TC, class CS>
__device__ __forceinline__ int tile_col(const CS& tc, int i)
{
    static_assert(TC::PASS == 1 || !CS::ROTATES, "only pass 1 rotates its columns");
    if constexpr (CS::ROTATES)
        return (tc.col0 - tc.rot + i) & (TC::GROUPS - 1);
    else
        return tc.col0 + i;
}

// Tile row r, tile columns i .. i+3 (i a multiple of 4) in the source of the
// pass (offsets within one transform are below N <= 2^16, so 32-bit offsets
// from the uniform plane pointer suffice).
template <class TC, class CS>
__device__ __forceinline__ int tile_src_offset(int r, int i, const CS& tc)
{
    if constexpr (TC::PASS == 1)
        return r * (TC::N >> TC::A) + tile_col<TC, CS>(tc, i);  // x row r
    else if constexpr (TC::WSC > 0)
        return tc.col0 * TC::R + r * TC::C + i;  // tiled: one contiguous run
    else
        return tile_col<TC, CS>(tc, i) + (r << TC::A);  // workspace row r
}

// Sources of a tile's plane: a pointer read with 16-byte loads (nontemporal
// for the data side of pass 1) ...
template <bool NT>
struct PlaneSrc {
    const float* p;
    __device__ __forceinline__ v4f load(int off) const { return load4<NT>(p + off); }
};

// ... or a plane another workgroup of the same XCD has just written, read
// through a buffer resource with loads that bypass the CU's own cache and read
// the XCD's L2 (cache policy sc1), so that no line the CU cached before the
// other workgroup's stores can be returned.
struct L2Src {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ v4f load(int off) const
    {
        return __builtin_bit_cast(v4f, __builtin_amdgcn_raw_buffer_load_b128(rsrc, static_cast<unsigned>(off) * 4u,
                                                                             0, 16));
    }
};

// Buffer resource over `floats` floats from p (raw 32-bit format, offsets in
// bytes; accesses beyond the range read 0 instead of faulting).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(float* p, int floats)
{
    return __builtin_amdgcn_make_buffer_rsrc(p, static_cast<short>(0), floats * 4, 0x00020000);
}

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// tile_in in two steps, so that both planes' loads can be in flight at once:
// this thread's 16-byte vectors of one plane of the tile ...
// Vector c of a thread covers tile row tid / C4 + c * THREADS / C4 and tile
// columns 4 * (tid % C4) .. + 3 (THREADS is a multiple of C4 = C / 4).
template <class TC, class CS, class Src>
__device__ __forceinline__ void tile_load(v4f (&r)[TC::E / 4], const Src& src, const CS& tc, int tid)
{
    constexpr int C4 = TC::C / 4, RSTEP = TC::THREADS / C4;
    const int c4 = tid % C4, r0 = tid / C4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c)
        r[c] = src.load(tile_src_offset<TC, CS>(r0 + c * RSTEP, 4 * c4, tc));
}

// ... and into the LDS slots (layout of tile_in).
template <class TC>
__device__ __forceinline__ void tile_put(const v4f (&r)[TC::E / 4], float* lds, int tid)
{
    constexpr int C4 = TC::C / 4, RSTEP = TC::THREADS / C4;
    const int c4 = tid % C4, r0 = tid / C4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int row = tile_lds_row<TC>(r0 + c * RSTEP);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            lds[(4 * c4 + e) * TC::SLOT + lds_index(row)] = r[c][e];
    }
}

// Tile (R rows x C columns, one plane) into LDS: column i in slot i, row r at
// lds_index(r) of the slot.
template <class TC, class CS>
__device__ __forceinline__ void tile_in(const float* src, float* lds, const CS& tc, int tid)
{
    constexpr int C4 = TC::C / 4, RSTEP = TC::THREADS / C4;
    const int c4 = tid % C4, r0 = tid / C4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int r = r0 + c * RSTEP;
        const v4f v = load4<TC::PASS == 1>(src + tile_src_offset<TC, CS>(r, 4 * c4, tc));
        const int row = tile_lds_row<TC>(r);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            lds[(4 * c4 + e) * TC::SLOT + lds_index(row)] = v[e];
    }
}

// Pass 1 output: block c of group i is contiguous in the workspace.
template <class TC, class CS>
__device__ __forceinline__ void blocks_out(float* dst, const float* lds, const CS& tc, int tid)
{
    if constexpr (TC::WSC > 0) {
        // tiled workspace: for each group of WSC positions, the tile's C
        // blocks (input columns tile_col(i)) form runs of WSC floats at
        // consecutive columns (one run of C x WSC floats unless the tile's
        // columns wrap around)
        constexpr int W4 = TC::WSC / 4;
        constexpr bool LINEAR = TC::THREADS % (W4 * TC::C) == 0;  // i, p4w fixed per thread
#pragma unroll
        for (int c = 0; c < TC::E / 4; ++c) {
            const int f4 = tid + c * TC::THREADS;
            const int p4w = (LINEAR ? tid : f4) % W4, rest = (LINEAR ? tid : f4) / W4;
            const int i = rest % TC::C;
            const int pg = LINEAR ? rest / TC::C + c * (TC::THREADS / (W4 * TC::C)) : rest / TC::C;
            const float* s = lds + i * TC::SLOT + lds_index(pg * TC::WSC + 4 * p4w);
            *reinterpret_cast<v4f*>(dst + (pg * (TC::R2 * TC::WSC) + tile_col<TC, CS>(tc, i) * TC::WSC + 4 * p4w)) =
                v4f{s[0], s[1], s[2], s[3]};
        }
        return;
    }
    constexpr int R4 = TC::R / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int i = f4 / R4, p4 = f4 % R4;
        const float* s = lds + i * TC::SLOT + lds_index(4 * p4);
        const int blk = rev_bits(tile_col<TC, CS>(tc, i), TC::M - TC::A);
        *reinterpret_cast<v4f*>(dst + (blk * TC::R + 4 * p4)) = v4f{s[0], s[1], s[2], s[3]};
    }
}

// Pass 2 output: natural positions lo + (p << A), along tile rows
// (nontemporal stores unless NT is false).
template <class TC, class CS, bool NT = true>
__device__ __forceinline__ void rows_out(float* dst, const float* lds, const CS& tc, int tid)
{
    constexpr int C4 = TC::C / 4, RSTEP = TC::THREADS / C4;
    const int c4 = tid % C4, r0 = tid / C4;
    // the output is in natural order whatever the workspace layout
    const int col = tile_col<TC, CS>(tc, 4 * c4);
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int r = r0 + c * RSTEP;
        const float* s = lds + (4 * c4) * TC::SLOT + lds_index(r);
        store4<NT>(dst + (col + (r << TC::A)), v4f{s[0], s[TC::SLOT], s[2 * TC::SLOT], s[3 * TC::SLOT]});
    }
}

// Registers of the group's first local pass: position u + (t << RB); in
// pass 1 that position is tile row rev_MA(position).
template <class TC>
__device__ __forceinline__ void tile_regs(float (&v)[TC::E], const float* slot, int t)
{
#pragma unroll
    for (int u = 0; u < TC::E; ++u) {
        if constexpr (TC::PASS == 1)
            v[u] = slot[lds_index(rev_bits(t, TC::LT) + (rev_bits(u, TC::RB) << TC::LT))];
        else
            v[u] = slot[lds_index(u + (t << TC::RB))];
    }
}

template <class TC>
__device__ __forceinline__ void regs_tile(const float (&v)[TC::E], float* slot, int t)
{
    using Last = Pass<TC::MA, TC::RB, TC::NP - 1>;
#pragma unroll
    for (int u = 0; u < TC::E; ++u)
        slot[lds_index(position<TC::LT, Last::S, Last::RP>(t, u))] = v[u];
}

// One tile of a pass: the C groups (columns) tile_col(tc, 0 .. C - 1) of the
// transform whose source planes are sr, si and whose destination planes start
// at yr, yi.  lds holds LDS_WORDS floats; every thread of the workgroup takes
// part.  after_loads() runs once every thread's loads of the tile have been
// consumed (behind a workgroup barrier; split-plane tiles only).
template <class TC, class CS, class Src, class Hook>
__device__ __forceinline__ void tile_process(const Src& sr, const Src& si, float* yr, float* yi,
                                             const float2* __restrict__ tw, const CS& tc, float* lds, int tid,
                                             const Hook& after_loads)
{
    constexpr int E = TC::E, LT = TC::LT, T = TC::T, C = TC::C;
    const int g = TC::GF ? tid % C : tid >> LT;  // group (column) within the tile
    const int t = TC::GF ? tid / C : tid & (T - 1);
    float* lr = lds + g * TC::SLOT;
    float* li = TC::SPLIT ? lr : lr + C * TC::SLOT;
    float* area_i = TC::SPLIT ? lds : lds + C * TC::SLOT;

    float vr[E], vi[E];
    if constexpr (TC::SPLIT) {
        // both planes' loads in flight at once; LDS holds one plane at a time
        v4f pr[E / 4], pi[E / 4];
        tile_load<TC, CS>(pr, sr, tc, tid);
        tile_load<TC, CS>(pi, si, tc, tid);
        tile_put<TC>(pr, lds, tid);
        __syncthreads();
        tile_regs<TC>(vr, lr, t);
        __syncthreads();
        tile_put<TC>(pi, lds, tid);
        __syncthreads();
        after_loads();
        tile_regs<TC>(vi, lr, t);
    } else {
        static_assert(std::is_same<Hook, NoHook>::value, "load hooks need split-plane tiles");
        tile_in<TC, CS>(sr.p, lds, tc, tid);
        tile_in<TC, CS>(si.p, area_i, tc, tid);
        __syncthreads();
        tile_regs<TC>(vr, lr, t);
        tile_regs<TC>(vi, li, t);
    }
    // the group's exchanges reuse its slot
    __syncthreads();

    const int lo_g = TC::PASS == 1 ? 0 : tile_col<TC, CS>(tc, g);
    stages<E, LT, 0, Pass<TC::MA, TC::RB, 0>::RP, TwTable<0>, TC::TW_SHIFT>(vr, vi, t, tw, lo_g);
    if constexpr (TC::NP > 1)
        later_passes<TC::MA, TC::RB, 1, TC::SPLIT, E, TwTable<0>, TC::TW_SHIFT, TC::GF ? 1024 : T>(vr, vi, lr, li, t, tw,
                                                                                       lo_g);

    // the group's slot is free again (its last exchange ended with a sync)
    if constexpr (TC::SPLIT) {
        regs_tile<TC>(vr, lr, t);
        __syncthreads();
        if constexpr (TC::PASS == 1)
            blocks_out<TC, CS>(yr, lds, tc, tid);
        else
            rows_out<TC, CS>(yr, lds, tc, tid);
        __syncthreads();
        regs_tile<TC>(vi, lr, t);
        __syncthreads();
        if constexpr (TC::PASS == 1)
            blocks_out<TC, CS>(yi, lds, tc, tid);
        else
            rows_out<TC, CS>(yi, lds, tc, tid);
    } else {
        regs_tile<TC>(vr, lr, t);
        regs_tile<TC>(vi, li, t);
        __syncthreads();
        if constexpr (TC::PASS == 1) {
            blocks_out<TC, CS>(yr, lds, tc, tid);
            blocks_out<TC, CS>(yi, area_i, tc, tid);
        } else {
            rows_out<TC, CS>(yr, lds, tc, tid);
            rows_out<TC, CS>(yi, area_i, tc, tid);
        }
    }
}

// ---- decimation in frequency, eq. (9), in two passes ---------------------
// The stages run m down to 1 on the natural-order input, the bit reversal
// last.  Split at a: stages m..a+1 act on bits m-1..a, so the positions
// lo + (p << a) (lo < 2^a) form independent columns; this first pass has the
// column geometry of a TileCfg with PASS 2 (natural layout on both sides:
// columns read from the input, rows written to the workspace).  Stages a..1
// act on blocks of 2^a consecutive positions (the block geometry of PASS 1);
// position c 2^a + j is output rev_m(c 2^a + j) = rev_a(j) 2^(m-a) +
// rev_(m-a)(c), so with the tile's blocks c = rev_(m-a)(k) for consecutive k
// every output row rev_a(j) is a run of C contiguous floats.

// Stages S+RP .. S+1 of eq. (9) for a group of 2^MA positions whose position p
// is the transform's lo_g + (p << A): per stage, highest first, the butterfly
// W^(i) (u + v, u - v), then the rotation D^(i) of the upper element by
// omega^(i,q), q = lo_g + (ql << A) (the index mapping of stages()).
template <int E, int LT, int S, int RP, class TW, int A>
__device__ __forceinline__ void stages_dif_group(float (&vr)[E], float (&vi)[E], int t, const float2* __restrict__ tw,
                                                 int lo_g)
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
            if constexpr (S == 0 && A == 0) {
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
                const int qt = lo_g + ((t & ((1 << S) - 1)) << A);
                const int qc = ((((u >> RP) << LT) & ((1 << S) - 1)) + ((u & (half - 1)) << S)) << A;
                const float2 w = TW::get2(tw, A + S + k, qt, qc);
                rotate(dr, di, w.x, w.y);
            }
            vr[v] = dr;
            vi[v] = di;
        }
    }
}

// DIF passes P, P+1, ... of a group (exchange through the group's LDS slot,
// SYNC_T as for later_passes), then the pass's stages.
template <int M, int RB, int P, int E, class TW, int A, int SYNC_T>
__device__ __forceinline__ void later_passes_dif_group(float (&vr)[E], float (&vi)[E], float* lr, int t,
                                                       const float2* __restrict__ tw, int lo_g)
{
    if constexpr (P < PassD<M, RB, 0>::NP) {
        constexpr int LT = M - RB;
        using Prev = PassD<M, RB, P - 1>;
        using Cur = PassD<M, RB, P>;
        lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vr, lr, t);
        xsync<SYNC_T>();
        lds_get<E, LT, Cur::S, Cur::RP>(vr, lr, t);
        xsync<SYNC_T>();
        lds_put<E, LT, Prev::S, Prev::RP, Cur::S, Cur::RP>(vi, lr, t);
        xsync<SYNC_T>();
        lds_get<E, LT, Cur::S, Cur::RP>(vi, lr, t);
        xsync<SYNC_T>();
        stages_dif_group<E, LT, Cur::S, Cur::RP, TW, A>(vr, vi, t, tw, lo_g);
        later_passes_dif_group<M, RB, P + 1, E, TW, A, SYNC_T>(vr, vi, lr, t, tw, lo_g);
    }
}

// Second DIF pass input: this thread's 16-byte vectors of one plane of the
// tile's blocks (block rev_(m-a)(tile column i), contiguous in the workspace)
// ...
template <class TC, class CS, class Src>
__device__ __forceinline__ void blocks_load(v4f (&r)[TC::E / 4], const Src& src, const CS& tc, int tid)
{
    constexpr int R4 = TC::R / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int i = f4 / R4, p4 = f4 % R4;
        const int blk = rev_bits(tile_col<TC, CS>(tc, i), TC::M - TC::A);
        r[c] = src.load(blk * TC::R + 4 * p4);
    }
}

// ... into the LDS slots: block position j of tile column i at lds_index(j).
template <class TC>
__device__ __forceinline__ void blocks_put(const v4f (&r)[TC::E / 4], float* lds, int tid)
{
    constexpr int R4 = TC::R / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int i = f4 / R4, p4 = f4 % R4;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            lds[i * TC::SLOT + lds_index(4 * p4 + e)] = r[c][e];
    }
}

// Second DIF pass output: output row r holds block position rev_a(r) of
// every tile column, at r 2^(m-a) + (tile column).
template <class TC, class CS>
__device__ __forceinline__ void bitrev_rows_out(float* dst, const float* lds, const CS& tc, int tid)
{
    constexpr int C4 = TC::C / 4, RSTEP = TC::THREADS / C4;
    const int c4 = tid % C4, r0 = tid / C4;
    const int col = tile_col<TC, CS>(tc, 4 * c4);
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int r = r0 + c * RSTEP;
        const float* s = lds + (4 * c4) * TC::SLOT + lds_index(rev_bits(r, TC::MA));
        store4<true>(dst + (r * (TC::N >> TC::A) + col), v4f{s[0], s[TC::SLOT], s[2 * TC::SLOT], s[3 * TC::SLOT]});
    }
}

// Tiled DIF workspace (WSX > 0): with C1 columns per first-pass tile and C2
// blocks per second-pass tile, row p = rev_(m-a)(k) of column lo sits at
//     (k / C2) (C2 2^a) + (lo / C1) (C2 C1) + (k mod C2) C1 + lo mod C1,
// each intersection of a first-pass and a second-pass tile contiguous: a
// second-pass tile (C2 consecutive k) reads one run of C2 2^a floats, and a
// first-pass tile writes runs of C2 C1 floats.

// First-pass output into the tiled workspace (C2: the second pass's tile width).
template <class TC, class CS, int C2>
__device__ __forceinline__ void dif_tiled_rows_out(float* dst, const float* lds, const CS& tc, int tid)
{
    constexpr int C1 = TC::C, C4 = C1 / 4, RSTEP = TC::THREADS / C4;
    static_assert(TC::PASS == 2 && (1 << TC::MA) % C2 == 0, "first DIF pass, whole second-pass tiles");
    const int c4 = tid % C4, r0 = tid / C4;
    const int t1 = tc.col0 / C1;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int k = r0 + c * RSTEP;  // rows in bit-reversed order
        const float* s = lds + (4 * c4) * TC::SLOT + lds_index(rev_bits(k, TC::MA));
        const int off = (k / C2) * (C2 << TC::A) + t1 * (C2 * C1) + (k % C2) * C1 + 4 * c4;
        store4<false>(dst + off, v4f{s[0], s[TC::SLOT], s[2 * TC::SLOT], s[3 * TC::SLOT]});
    }
}

// Second-pass input from the tiled workspace: the tile's run, this thread's
// 16-byte vectors ...
template <class TC, class CS, class Src>
__device__ __forceinline__ void dif_tiled_blocks_load(v4f (&r)[TC::E / 4], const Src& src, const CS& tc, int tid)
{
    static_assert(TC::PASS == 1, "second DIF pass");
    const int base = (tc.col0 / TC::C) * (TC::C * TC::R);
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c)
        r[c] = src.load(base + 4 * (tid + c * TC::THREADS));
}

// ... into the LDS slots (C1: the first pass's tile width): block k of the
// tile (slot k mod C2) at position lo.
template <class TC, int C1>
__device__ __forceinline__ void dif_tiled_blocks_put(const v4f (&r)[TC::E / 4], float* lds, int tid)
{
    constexpr int C2 = TC::C;
    static_assert(TC::R % C1 == 0 && C1 % 4 == 0, "whole first-pass tiles");
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f = 4 * (tid + c * TC::THREADS);
        const int t1 = f / (C2 * C1), rem = f % (C2 * C1);
        const int i = rem / C1, lo = t1 * C1 + rem % C1;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            lds[i * TC::SLOT + lds_index(lo + e)] = r[c][e];
    }
}

// One tile of a DIF pass: TC::PASS 2 is the first (columns of the input into
// the workspace), TC::PASS 1 the second (workspace blocks into the output).
// WSX: the other pass's tile width for the tiled workspace layout, 0 for
// natural position order.  The group's positions sit in natural order in its
// LDS slot on the way in and on the way out.
template <class TC, class CS, int WSX, class Src>
__device__ __forceinline__ void tile_process_dif(const Src& sr, const Src& si, float* yr, float* yi,
                                                 const float2* __restrict__ tw, const CS& tc, float* lds, int tid)
{
    static_assert(TC::SPLIT && TC::WSC == 0, "split-plane tiles (the DIF layouts are chosen by WSX)");
    constexpr int E = TC::E, LT = TC::LT, T = TC::T, C = TC::C;
    using First = PassD<TC::MA, TC::RB, 0>;
    using Last = PassD<TC::MA, TC::RB, First::NP - 1>;
    const int g = TC::GF ? tid % C : tid >> LT;
    const int t = TC::GF ? tid / C : tid & (T - 1);
    float* lr = lds + g * TC::SLOT;

    float vr[E], vi[E];
    v4f pr[E / 4], pi[E / 4];
    if constexpr (TC::PASS == 2) {
        tile_load<TC, CS>(pr, sr, tc, tid);
        tile_load<TC, CS>(pi, si, tc, tid);
        tile_put<TC>(pr, lds, tid);
    } else if constexpr (WSX > 0) {
        dif_tiled_blocks_load<TC, CS>(pr, sr, tc, tid);
        dif_tiled_blocks_load<TC, CS>(pi, si, tc, tid);
        dif_tiled_blocks_put<TC, WSX>(pr, lds, tid);
    } else {
        blocks_load<TC, CS>(pr, sr, tc, tid);
        blocks_load<TC, CS>(pi, si, tc, tid);
        blocks_put<TC>(pr, lds, tid);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < E; ++u)
        vr[u] = lr[lds_index(position<LT, First::S, First::RP>(t, u))];
    __syncthreads();
    if constexpr (TC::PASS == 2)
        tile_put<TC>(pi, lds, tid);
    else if constexpr (WSX > 0)
        dif_tiled_blocks_put<TC, WSX>(pi, lds, tid);
    else
        blocks_put<TC>(pi, lds, tid);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < E; ++u)
        vi[u] = lr[lds_index(position<LT, First::S, First::RP>(t, u))];
    __syncthreads();

    const int lo_g = TC::PASS == 1 ? 0 : tile_col<TC, CS>(tc, g);
    stages_dif_group<E, LT, First::S, First::RP, TwTable<0>, TC::TW_SHIFT>(vr, vi, t, tw, lo_g);
    if constexpr (First::NP > 1)
        later_passes_dif_group<TC::MA, TC::RB, 1, E, TwTable<0>, TC::TW_SHIFT, TC::GF ? 1024 : T>(vr, vi, lr, t, tw,
                                                                                                 lo_g);

    // natural position order in the slot, one plane at a time
#pragma unroll
    for (int u = 0; u < E; ++u)
        lr[lds_index(position<LT, Last::S, Last::RP>(t, u))] = vr[u];
    __syncthreads();
    if constexpr (TC::PASS == 2 && WSX > 0)
        dif_tiled_rows_out<TC, CS, WSX>(yr, lds, tc, tid);
    else if constexpr (TC::PASS == 2)
        rows_out<TC, CS, false>(yr, lds, tc, tid);
    else
        bitrev_rows_out<TC, CS>(yr, lds, tc, tid);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < E; ++u)
        lr[lds_index(position<LT, Last::S, Last::RP>(t, u))] = vi[u];
    __syncthreads();
    if constexpr (TC::PASS == 2 && WSX > 0)
        dif_tiled_rows_out<TC, CS, WSX>(yi, lds, tc, tid);
    else if constexpr (TC::PASS == 2)
        rows_out<TC, CS, false>(yi, lds, tc, tid);
    else
        bitrev_rows_out<TC, CS>(yi, lds, tc, tid);
}

// The same from plane pointers (nontemporal loads on pass 1's data side).
template <class TC, class CS>
__device__ __forceinline__ void tile_process(const float* xr, const float* xi, float* yr, float* yi,
                                             const float2* __restrict__ tw, const CS& tc, float* lds, int tid)
{
    tile_process<TC, CS>(PlaneSrc<TC::PASS == 1>{xr}, PlaneSrc<TC::PASS == 1>{xi}, yr, yi, tw, tc, lds, tid,
                         NoHook{});
}

}  // namespace
}  // namespace splitdft
