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
#include "fft_xcd.h"

#include <atomic>
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

// A pass of the decimation-in-frequency two-pass schedule (TC::PASS 2: the
// first, input columns into the workspace; TC::PASS 1: the second, workspace
// blocks into the output in bit-reversed order).
template <class TC, int WSX>
__global__ void __launch_bounds__(TC::THREADS)
split_fft_tile_dif_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                          int tiles_per_transform, const int64_t* __restrict__ rows)
{
    __shared__ float lds[TC::LDS_WORDS];
    const int64_t t = blockIdx.x / tiles_per_transform;
    const int64_t wbase = t * TC::N;
    const int64_t dbase = rows ? rows[t] : wbase;
    const int64_t ibase = TC::PASS == 2 ? dbase : wbase;
    const int64_t obase = TC::PASS == 2 ? wbase : dbase;
    const TileCols<false> tc{static_cast<int>(blockIdx.x % tiles_per_transform) * TC::C};
    tile_process_dif<TC, TileCols<false>, WSX>(PlaneSrc<TC::PASS == 2>{xr + ibase}, PlaneSrc<TC::PASS == 2>{xi + ibase},
                                               yr + obase, yi + obase, tw, tc, lds, threadIdx.x);
}

template <class TC, int WSX>
hipError_t launch_tile_dif(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                           const int64_t* rows, hipStream_t stream)
{
    const int64_t blocks = batch * TC::TILES;
    if (blocks > INT_MAX)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((split_fft_tile_dif_kernel<TC, WSX>), dim3(static_cast<unsigned>(blocks)), dim3(TC::THREADS),
                       0, stream, xr, xi, yr, yi, tw, TC::TILES, rows);
    return hipGetLastError();
}

// DIF two-pass schedule: C1 input columns per first-pass tile (lanes over
// columns first when GF1), C2 blocks per second-pass tile; WST: the tiled
// workspace layout (see tile_process_dif), else natural position order.
template <int M, int A, int RB1, int C1, bool GF1, int RB2, int C2, bool WST = true>
constexpr TwoPass make_two_pass_dif()
{
    using P1 = TileCfg<M, A, 2, RB1, C1, true, GF1, 0>;
    using P2 = TileCfg<M, A, 1, RB2, C2, true, false, 0>;
    return TwoPass{M,     A,   C1,  C2, P1::THREADS, P2::THREADS, 4 * P1::LDS_WORDS, 4 * P2::LDS_WORDS,
                   GF1,   &launch_tile_dif<P1, WST ? C2 : 0>, &launch_tile_dif<P2, WST ? C1 : 0>,
                   WST,   nullptr, 0, true};
}

// Polls per wait of the fused schedule before it gives up (each poll sleeps
// up to about 0.4 us after a load from L2: seconds in all).
constexpr int kXcdPollLimit = 1 << 22;

// Launch of the fused schedule: the control block (after the ring in ws)
// cleared by a kernel (graph-safe), then one persistent launch sized to the
// device's resident capacity.
template <class P1, class P2, int SLOTS>
hipError_t launch_xcd(const float* xr, const float* xi, float* yr, float* yi, const float2* tw, int64_t batch,
                      const int64_t* rows, float* ws, hipStream_t stream)
{
    static_assert(SLOTS >= 1 && SLOTS <= kXcdMaxSlots, "ring slots");
    if (batch < 1 || batch >= kClaimedEmpty)
        return hipErrorInvalidValue;
    float* ring = ws;
    auto* ctl = reinterpret_cast<XcdControl*>(ws + xcd_ring_floats(P1::M, SLOTS));
    const bool rot = rows != nullptr || line_offset(xr) != 0;
    auto kernel = rot ? split_fft_xcd_kernel<P1, P2, true> : split_fft_xcd_kernel<P1, P2, false>;
    static std::atomic<int> resident_of[2][64];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    const bool cache = dev >= 0 && dev < 64;
    int resident = cache ? resident_of[rot][dev].load(std::memory_order_relaxed) : 0;
    if (resident <= 0) {
        int cus = 0, per_cu = 0;
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, P1::THREADS, 0);
        if (e != hipSuccess)
            return e;
        if (per_cu < 1 || cus < 1)
            return hipErrorInvalidConfiguration;
        resident = cus * per_cu;
        if (cache)
            resident_of[rot][dev].store(resident, std::memory_order_relaxed);
    }
    // As many workgroups as are resident at once, fewer for small batches
    // (more than the items would only take empty ones) but never fewer than
    // T per XCD: the T tiles of a transform wait on each other, and workgroups
    // are dispatched to the XCDs in turn.
    const int64_t items = batch * P1::TILES;
    const int64_t least = int64_t{kXcds} * P1::TILES;
    int64_t grid = items > least ? items : least;
    if (grid > resident)
        grid = resident;
    if (resident < least)
        return hipErrorInvalidConfiguration;
    static_assert(xcd_control_bytes() % 16 == 0, "whole 16-byte words");
    hipLaunchKernelGGL(xcd_control_clear, dim3(4), dim3(256), 0, stream, reinterpret_cast<float4*>(ctl),
                       static_cast<int>(xcd_control_bytes() / 16));
    hipLaunchKernelGGL(kernel, dim3(static_cast<unsigned>(grid)), dim3(P1::THREADS), 0, stream, xr, xi, yr, yi, tw,
                       batch, rows, ring, ctl, SLOTS, kXcdPollLimit);
    return hipGetLastError();
}

template <int M, int A, int RB1, int C1, bool SPLIT1, int RB2, int C2, bool SPLIT2, bool GF2 = false,
          bool WST = false, int SLOTS = 0>
constexpr TwoPass make_two_pass()
{
    constexpr int WSC = WST ? C2 : 0;
    using P1 = TileCfg<M, A, 1, RB1, C1, SPLIT1, false, WSC>;
    using P2 = TileCfg<M, A, 2, RB2, C2, SPLIT2, GF2, WSC>;
    if constexpr (SLOTS > 0)
        return TwoPass{M,  A,  C1, C2, P1::THREADS, P2::THREADS, 4 * P1::LDS_WORDS, 4 * P2::LDS_WORDS, GF2,
                       &launch_tile<P1>, &launch_tile<P2>, WST, &launch_xcd<P1, P2, SLOTS>, SLOTS};
    else
        return TwoPass{M,  A,  C1, C2, P1::THREADS, P2::THREADS, 4 * P1::LDS_WORDS, 4 * P2::LDS_WORDS, GF2,
                       &launch_tile<P1>, &launch_tile<P2>, WST};
}

//                                   M   A  RB1 C1 SPLIT1 RB2 C2 SPLIT2 GF2
const TwoPass kTwoPass14[] = {make_two_pass<14, 8, 4, 32, true, 4, 128, true, true, true>(),
                              make_two_pass<14, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<14, 8, 4, 32, true, 4, 32, true, true>()};
// (split at stage 7 at 2^15 and at stage 9 at 2^16, appended after the fused
// entries: within 1-2% of the stage-8 defaults; 16 blocks per pass-1 tile at
// stage 9 and a stage-7 split at 2^16 measured 20-30% slower)
// the fused entries of the 2^15 and 2^16 lists: both passes in one launch
// through a ring of 12 (2^15, 3 MiB) or 8 (2^16, 4 MiB) transforms per XCD, the
// fastest ring sizes measured (112 / 110 us per 2^24 points against 90 / 92
// for the separate passes, so not the default)
const TwoPass kTwoPass15[] = {make_two_pass<15, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<15, 8, 4, 64, true, 4, 64, true, true, true>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 128, true, true, true>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<15, 8, 4, 16, false, 4, 32, false>(),
                              make_two_pass<15, 8, 4, 32, true, 4, 64, true, true, true, 12>(),
                              make_two_pass<15, 7, 4, 64, true, 4, 32, true, true, true>(),
                              make_two_pass<15, 7, 4, 32, true, 4, 32, true, true, true>()};
const TwoPass kTwoPass16[] = {make_two_pass<16, 8, 4, 32, true, 4, 32, true, true, true>(),
                              make_two_pass<16, 8, 4, 64, true, 4, 32, true, true, true>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 64, true, true, true>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 32, true, true>(),
                              make_two_pass<16, 8, 4, 16, false, 4, 16, false>(),
                              make_two_pass<16, 8, 4, 32, true, 4, 32, true, true, true, 8>(),
                              make_two_pass<16, 9, 4, 32, true, 4, 64, true, true, true>()};

}  // namespace

//                                              M   A  RB1 C1 GF1 RB2 C2
// (swept: 128 columns or lanes over rows first in the first pass, 64 blocks in
// the second at 2^16, or 16 columns at 2^16, measured 2-30% slower)
const TwoPass kDifTwoPass15[] = {make_two_pass_dif<15, 8, 4, 64, true, 4, 32>(),
                                 make_two_pass_dif<15, 8, 4, 64, true, 4, 32, false>(),
                                 make_two_pass_dif<15, 8, 4, 64, true, 4, 16>(),
                                 make_two_pass_dif<15, 8, 4, 32, true, 4, 32>()};
const TwoPass kDifTwoPass16[] = {make_two_pass_dif<16, 8, 4, 32, true, 4, 32>(),
                                 make_two_pass_dif<16, 8, 4, 32, true, 4, 32, false>(),
                                 make_two_pass_dif<16, 8, 4, 64, true, 4, 32>(),
                                 make_two_pass_dif<16, 8, 4, 32, true, 4, 16>()};

size_t fused_workspace_bytes(const TwoPass* t)
{
    return static_cast<size_t>(xcd_ring_floats(t->m, t->slots)) * sizeof(float) + xcd_control_bytes();
}

const TwoPass* dif_two_pass_for(int m, int* count)
{
    switch (m) {
    case 15: *count = static_cast<int>(sizeof(kDifTwoPass15) / sizeof(kDifTwoPass15[0])); return kDifTwoPass15;
    case 16: *count = static_cast<int>(sizeof(kDifTwoPass16) / sizeof(kDifTwoPass16[0])); return kDifTwoPass16;
    default: *count = 0; return nullptr;
    }
}

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
