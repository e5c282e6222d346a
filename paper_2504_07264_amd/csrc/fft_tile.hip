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
// The working vector between the passes lives in a workspace that the batch
// is processed through in chunks; by default it is stored in pass-2 tile order
// (see TileCfg), so that pass 1 writes and pass 2 reads long contiguous runs
// and only the inherently strided sides (pass 1's gather of each block, pass
// 2's natural-order output) use 128-byte segments.  When a transform's data
// does not start on a 128-byte line (ragged batches), its pass-1 tiles take
// their columns rotated so that the read segments start on lines again
// (TileCols).
//
// A workgroup handles a tile of C groups (columns) x R = 2^MA rows.  The tile
// is loaded and stored with 16-byte vectors along rows (C contiguous floats)
// and transposed through LDS into one slot per group; the group then runs the
// register passes of the single-pass kernel (exchanges within a group need
// only wave-level ordering when the group fits in one wave).  The arithmetic
// is exactly that of eq. (6) in order, so results equal the single-pass
// kernels' bit for bit.
#include "fft_tile.h"

#include <climits>
#include <cstdint>

namespace splitdft {
namespace {

// ROT (pass 1 only): rotate the tile columns by the data's offset from a
// 128-byte line (ragged transforms, or planes off a line); the unrotated build
// serves the rest.
template <class TC, bool ROT>
__global__ void __launch_bounds__(TC::THREADS)
split_fft_tile_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                      int tiles_per_transform, const int64_t* __restrict__ rows)
{
    __shared__ float lds[TC::LDS_WORDS];
    const int64_t t = blockIdx.x / tiles_per_transform;
    // the workspace side is contiguous; the data side may be given per transform
    const int64_t wbase = t * TC::N;
    const int64_t dbase = rows ? rows[t] : wbase;
    const int64_t ibase = TC::PASS == 1 ? dbase : wbase;
    const int64_t obase = TC::PASS == 1 ? wbase : dbase;
    const int col0 = (blockIdx.x % tiles_per_transform) * TC::C;
    if constexpr (ROT) {
        const int rot = static_cast<int>(((reinterpret_cast<uintptr_t>(xr) >> 2) + dbase) & 31);
        const TileCols<true> tc{col0, rot};
        tile_process<TC>(xr + ibase, xi + ibase, yr + obase, yi + obase, tw, tc, lds, threadIdx.x);
    } else {
        const TileCols<false> tc{col0};
        tile_process<TC>(xr + ibase, xi + ibase, yr + obase, yi + obase, tw, tc, lds, threadIdx.x);
    }
}

template <class TC>
hipError_t launch_tile(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                       const int64_t* rows, hipStream_t stream)
{
    const int64_t blocks = batch * TC::TILES;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    // contiguous transforms (N a multiple of 32) share the plane's own line
    // offset, so the unrotated build serves them when it is zero
    if constexpr (TC::PASS == 1) {
        if (rows != nullptr || line_offset(xr) != 0) {
            hipLaunchKernelGGL((split_fft_tile_kernel<TC, true>), dim3(static_cast<unsigned>(blocks)),
                               dim3(TC::THREADS), 0, stream, xr, xi, yr, yi, tw, TC::TILES, rows);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((split_fft_tile_kernel<TC, false>), dim3(static_cast<unsigned>(blocks)), dim3(TC::THREADS), 0,
                       stream, xr, xi, yr, yi, tw, TC::TILES, rows);
    return hipGetLastError();
}

template <int M, int A, int RB1, int C1, bool SPLIT1, int RB2, int C2, bool SPLIT2, bool GF2 = false,
          bool WST = false>
constexpr TwoPass make_two_pass()
{
    constexpr int WSC = WST ? C2 : 0;
    using P1 = TileCfg<M, A, 1, RB1, C1, SPLIT1, false, WSC>;
    using P2 = TileCfg<M, A, 2, RB2, C2, SPLIT2, GF2, WSC>;
    return TwoPass{M,  A,  C1, C2, P1::THREADS, P2::THREADS, 4 * P1::LDS_WORDS, 4 * P2::LDS_WORDS, GF2,
                   &launch_tile<P1>, &launch_tile<P2>, WST};
}

//                                   M   A  RB1 C1 SPLIT1 RB2 C2 SPLIT2 GF2
const TwoPass kTwoPass14[] = {make_two_pass<14, 8, 4, 32, true, 4, 128, true, true, true>(),
                              make_two_pass<14, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<14, 8, 4, 32, true, 4, 32, true, true>()};
const TwoPass kTwoPass15[] = {make_two_pass<15, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<15, 8, 4, 64, true, 4, 64, true, true, true>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 128, true, true, true>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<15, 8, 4, 16, false, 4, 32, false>()};
const TwoPass kTwoPass16[] = {make_two_pass<16, 8, 4, 32, true, 4, 32, true, true, true>(),
                              make_two_pass<16, 8, 4, 64, true, 4, 32, true, true, true>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<16, 8, 4, 16, false, 4, 16, false>()};

}  // namespace

const TwoPass* two_pass_for(int m, int* count)
{
    switch (m) {
    case 14: *count = static_cast<int>(sizeof(kTwoPass14) / sizeof(kTwoPass14[0])); return kTwoPass14;
    case 15: *count = static_cast<int>(sizeof(kTwoPass15) / sizeof(kTwoPass15[0])); return kTwoPass15;
    case 16: *count = static_cast<int>(sizeof(kTwoPass16) / sizeof(kTwoPass16[0])); return kTwoPass16;
    default: *count = 0; return nullptr;
    }
}

}  // namespace splitdft
