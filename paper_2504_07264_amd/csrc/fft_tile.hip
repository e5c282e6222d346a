// Two-pass split-format FFT for lengths whose working vector does not fit in
// one workgroup's registers and LDS (N = 2^15, 2^16).
//
// The Kronecker structure of eq. (6) (Section III) splits the m stages at a:
//   pass 1: stages 1..a.  Every factor is I_(2^(m-i)) (x) (...) with i <= a,
//           so after the bit reversal the working vector falls into 2^(m-a)
//           independent blocks of 2^a consecutive positions.  Block c holds
//           x[rev_a(p) * 2^(m-a) + rev_(m-a)(c)] at its position p.
//   pass 2: stages a+1..m.  Stage a+s pairs positions whose index differs in
//           bit a+s-1, so the positions lo + (p << a) (lo < 2^a) form
//           2^a independent groups ("columns"); within column lo, local
//           stage s is stage a+s with twiddle index q = lo + (ql << a).
// The working vector between the passes lives in a workspace (row-major,
// natural position order) that stays in the L2 / Infinity Cache when the
// batch is processed in chunks.
//
// A workgroup handles a tile of C groups (columns) x R = 2^MA rows.  The tile
// is loaded and stored with 16-byte vectors along rows (C contiguous floats)
// and transposed through LDS into one slot per group; the group then runs the
// register passes of the single-pass kernel (exchanges within a group need
// only wave-level ordering when the group fits in one wave).  The arithmetic
// is exactly that of eq. (6) in order, so results equal the single-pass
// kernels' bit for bit.
#include "fft_device.h"

#include <climits>

namespace splitdft {
namespace {

// GF: lanes run over the tile's groups first (thread t of group g is
// tid = g + C * t), so that the per-group twiddles of pass 2 (index
// lo + (ql << A), lo = the group's column) are contiguous across a wave; the
// groups then span waves and exchanges use workgroup barriers.
template <int M_, int A_, int PASS_, int RB_, int C_, bool SPLIT_, bool GF_ = false>
struct TileCfg {
    static constexpr int M = M_, A = A_, PASS = PASS_, RB = RB_, C = C_;
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
    static_assert(C % 4 == 0 && E >= 4 && GROUPS % C == 0, "tile shape");
};

// Row r of the tile (C contiguous floats) in the source of the pass.
template <class TC>
__device__ __forceinline__ int64_t tile_row_offset(int r, int col0)
{
    if constexpr (TC::PASS == 1)
        return static_cast<int64_t>(r) * (TC::N >> TC::A) + col0;  // x row r, blocks col0..
    else
        return col0 + (static_cast<int64_t>(r) << TC::A);           // workspace row r, columns col0..
}

// Tile (R rows x C columns, one plane) into LDS: column i in slot i, row r at
// lds_index(r) of the slot.
template <class TC>
__device__ __forceinline__ void tile_in(const float* src, float* lds, int col0, int tid)
{
    constexpr int C4 = TC::C / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int r = f4 / C4, c4 = f4 % C4;
        const v4f v = load4<TC::PASS == 1>(src + tile_row_offset<TC>(r, col0) + 4 * c4);
#pragma unroll
        for (int e = 0; e < 4; ++e)
            lds[(4 * c4 + e) * TC::SLOT + lds_index(r)] = v[e];
    }
}

// Pass 1 output: block c of group i is contiguous in the workspace.
template <class TC>
__device__ __forceinline__ void blocks_out(float* dst, const float* lds, int col0, int tid)
{
    constexpr int R4 = TC::R / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int i = f4 / R4, p4 = f4 % R4;
        const float* s = lds + i * TC::SLOT + lds_index(4 * p4);
        const int blk = rev_bits(col0 + i, TC::M - TC::A);
        *reinterpret_cast<v4f*>(dst + static_cast<int64_t>(blk) * TC::R + 4 * p4) = v4f{s[0], s[1], s[2], s[3]};
    }
}

// Pass 2 output: natural positions lo + (p << A), along tile rows.
template <class TC>
__device__ __forceinline__ void rows_out(float* dst, const float* lds, int col0, int tid)
{
    constexpr int C4 = TC::C / 4;
#pragma unroll
    for (int c = 0; c < TC::E / 4; ++c) {
        const int f4 = tid + c * TC::THREADS;
        const int r = f4 / C4, c4 = f4 % C4;
        const float* s = lds + (4 * c4) * TC::SLOT + lds_index(r);
        store4<true>(dst + tile_row_offset<TC>(r, col0) + 4 * c4,
                     v4f{s[0], s[TC::SLOT], s[2 * TC::SLOT], s[3 * TC::SLOT]});
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

template <class TC>
__global__ void __launch_bounds__(TC::THREADS)
split_fft_tile_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                      int tiles_per_transform)
{
    constexpr int E = TC::E, LT = TC::LT, T = TC::T, C = TC::C;
    __shared__ float lds[TC::LDS_WORDS];
    const int tid = threadIdx.x;
    const int g = TC::GF ? tid % C : tid >> LT;  // group (column) within the tile
    const int t = TC::GF ? tid / C : tid & (T - 1);
    const int64_t b = blockIdx.x / tiles_per_transform;
    const int col0 = (blockIdx.x % tiles_per_transform) * C;
    const int64_t base = b * TC::N;
    float* lr = lds + g * TC::SLOT;
    float* li = TC::SPLIT ? lr : lr + C * TC::SLOT;
    float* area_i = TC::SPLIT ? lds : lds + C * TC::SLOT;

    float vr[E], vi[E];
    tile_in<TC>(xr + base, lds, col0, tid);
    if constexpr (TC::SPLIT) {
        __syncthreads();
        tile_regs<TC>(vr, lr, t);
        __syncthreads();
        tile_in<TC>(xi + base, lds, col0, tid);
        __syncthreads();
        tile_regs<TC>(vi, lr, t);
    } else {
        tile_in<TC>(xi + base, area_i, col0, tid);
        __syncthreads();
        tile_regs<TC>(vr, lr, t);
        tile_regs<TC>(vi, li, t);
    }
    // the group's exchanges reuse its slot
    __syncthreads();

    const int lo_g = TC::PASS == 1 ? 0 : col0 + g;
    stages<E, LT, 0, Pass<TC::MA, TC::RB, 0>::RP, 0, TC::TW_SHIFT>(vr, vi, t, tw, lo_g);
    if constexpr (TC::NP > 1)
        later_passes<TC::MA, TC::RB, 1, TC::SPLIT, E, 0, TC::TW_SHIFT, TC::GF ? 1024 : T>(vr, vi, lr, li, t, tw,
                                                                                       lo_g);

    // the group's slot is free again (its last exchange ended with a sync)
    if constexpr (TC::SPLIT) {
        regs_tile<TC>(vr, lr, t);
        __syncthreads();
        if constexpr (TC::PASS == 1)
            blocks_out<TC>(yr + base, lds, col0, tid);
        else
            rows_out<TC>(yr + base, lds, col0, tid);
        __syncthreads();
        regs_tile<TC>(vi, lr, t);
        __syncthreads();
        if constexpr (TC::PASS == 1)
            blocks_out<TC>(yi + base, lds, col0, tid);
        else
            rows_out<TC>(yi + base, lds, col0, tid);
    } else {
        regs_tile<TC>(vr, lr, t);
        regs_tile<TC>(vi, li, t);
        __syncthreads();
        if constexpr (TC::PASS == 1) {
            blocks_out<TC>(yr + base, lds, col0, tid);
            blocks_out<TC>(yi + base, area_i, col0, tid);
        } else {
            rows_out<TC>(yr + base, lds, col0, tid);
            rows_out<TC>(yi + base, area_i, col0, tid);
        }
    }
}

template <class TC>
hipError_t launch_tile(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                       hipStream_t stream)
{
    const int64_t blocks = batch * TC::TILES;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(split_fft_tile_kernel<TC>, dim3(static_cast<unsigned>(blocks)), dim3(TC::THREADS), 0, stream,
                       xr, xi, yr, yi, tw, TC::TILES);
    return hipGetLastError();
}

template <int M, int A, int RB1, int C1, bool SPLIT1, int RB2, int C2, bool SPLIT2, bool GF2 = false>
constexpr TwoPass make_two_pass()
{
    using P1 = TileCfg<M, A, 1, RB1, C1, SPLIT1>;
    using P2 = TileCfg<M, A, 2, RB2, C2, SPLIT2, GF2>;
    return TwoPass{M,  A,  C1, C2, P1::THREADS, P2::THREADS, 4 * P1::LDS_WORDS, 4 * P2::LDS_WORDS, GF2,
                   &launch_tile<P1>, &launch_tile<P2>};
}

//                                   M   A  RB1 C1 SPLIT1 RB2 C2 SPLIT2 GF2
const TwoPass kTwoPass14[] = {make_two_pass<14, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<14, 8, 4, 32, true, 4, 32, true>()};
const TwoPass kTwoPass15[] = {make_two_pass<15, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 32, true>(),
                              make_two_pass<15, 8, 4, 16, false, 4, 32, false>()};
const TwoPass kTwoPass16[] = {make_two_pass<16, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 32, true>(),
                              make_two_pass<16, 8, 4, 16, false, 4, 16, false>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 64, true, true>()};

}  // namespace

const TwoPass* two_pass_for(int m, int* count)
{
    switch (m) {
    case 14: *count = 2; return kTwoPass14;
    case 15: *count = 3; return kTwoPass15;
    case 16: *count = 4; return kTwoPass16;
    default: *count = 0; return nullptr;
    }
}

}  // namespace splitdft
