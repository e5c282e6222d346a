// Both passes of the two-pass schedule in one persistent launch, the
// intermediate of each transform handed from its pass-1 tiles to its pass-2
// tiles through the L2 cache of one XCD (accelerator complex die: 32 CUs
// sharing a 4 MB L2) instead of a workspace round trip through memory.
//
// Work items.  Every XCD has its own queue of items; item k of an XCD is tile
// r = k mod T of the XCD's local transform l = k / T (both passes have T
// tiles per transform).  The workgroup holding it runs pass-1 tile r into the
// local transform's ring slot, waits until all of the transform's pass-1 tiles
// are there, then runs pass-2 tile r out of the slot.  Which transform of the
// batch local transform l is gets decided when its tile 0 is taken: that
// workgroup claims the next transform from one counter shared by all XCDs.
// Claims of one XCD are ordered (a ticket passed from local transform to local
// transform), so an XCD's transforms come in increasing order and the first
// claim past the batch marks the end of that XCD's queue: every later item of
// it is empty, and a workgroup that takes an empty item leaves.  An XCD that
// runs no workgroup of the launch claims nothing.
//
// Ring.  Each XCD has S slots of one transform's intermediate (both planes,
// the tiled workspace layout of the separate passes); local transform l uses
// slot l mod S once the S-th previous transform's pass-2 tiles have all read
// it.  Hand-over within an XCD needs no agent-scope release (which would write
// L2 back to memory): a pass-1 tile's stores are acknowledged by the XCD's L2
// (a wait on the memory counter) before the slot's counter is incremented
// there, and pass-2 tiles read the slot with loads that bypass the CU's own
// cache.  The waits are bounded: a wait that exceeds its poll limit sets the
// abort word, after which every wait returns at once, so a launch always ends
// (its results are then not defined).  Workgroups wait only on items taken
// before theirs, except that a transform's T tiles wait on each other, which
// needs T workgroups of the launch resident on an XCD at once; the launch is
// sized to the device's resident capacity.
//
// The arithmetic of every tile is that of the separate pass kernels
// (tile_process), so the results equal theirs bit for bit.
#pragma once

#include "fft_tile.h"

#include <climits>

namespace splitdft {
namespace {

constexpr int kXcds = 8;       // queues; workgroups use queue (XCC_ID mod 8)
constexpr int kLineInts = 32;  // every counter on its own 128-byte line
constexpr int kXcdMaxSlots = 16;
constexpr int kClaimedEmpty = 1 << 30;  // ticket flag: the claim past the batch happened

struct XcdControl {
    int head[kXcds][kLineInts];                            // next item of each queue
    unsigned long long next_transform[kLineInts / 2];      // claims, all queues
    int ticket[kXcds][kLineInts];                          // local transforms claimed (| kClaimedEmpty)
    unsigned long long owner[kXcds][kXcdMaxSlots][kLineInts / 2];  // (l + 1) | transform << 32
    int written[kXcds][kXcdMaxSlots][kLineInts];           // pass-1 tiles written per slot
    int gathered[kXcds][kXcdMaxSlots][kLineInts];          // pass-2 tiles read per slot
    int failed;                                            // workgroups whose waits gave up
    int abort_word;
};

__device__ __forceinline__ int xcd_queue()
{
    // HW_REG_XCC_ID (hardware register 20), bits 0..3
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11)) & (kXcds - 1);
}

__device__ __forceinline__ int load_agent(const int* p)
{
    return __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

__device__ __forceinline__ void nap(int& n)
{
    for (int j = 0; j < n; ++j)
        __builtin_amdgcn_s_sleep(2);
    n = n < 8 ? 2 * n : 8;
}

// Polls *p until it is >= target; run by a whole wave, decisions on
// wave-uniform values only.  false: gave up (abort word set).
__device__ __forceinline__ bool xcd_wait_geq(const int* p, int target, XcdControl* ctl, int limit)
{
    int n = 1;
    for (int i = 0; i < limit; ++i) {
        if (load_agent(p) >= target)
            return true;
        if (load_agent(&ctl->abort_word))
            return false;
        nap(n);
    }
    __hip_atomic_store(&ctl->abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

// The ticket of queue x once local transform l may claim: the value
// (l | kClaimedEmpty for an earlier empty claim included), or -1 (gave up).
__device__ __forceinline__ int xcd_wait_ticket(XcdControl* ctl, int x, int l, int limit)
{
    int n = 1;
    for (int i = 0; i < limit; ++i) {
        const int t = load_agent(&ctl->ticket[x][0]);
        if ((t & ~kClaimedEmpty) >= l || (t & kClaimedEmpty))
            return t;
        if (load_agent(&ctl->abort_word))
            return -1;
        nap(n);
    }
    __hip_atomic_store(&ctl->abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return -1;
}

// The transform local transform l of queue x was given (-1: none, or gave up).
__device__ __forceinline__ int xcd_wait_owner(XcdControl* ctl, int x, int slot, int l, int limit)
{
    int n = 1;
    for (int i = 0; i < limit; ++i) {
        const unsigned long long o =
            __hip_atomic_load(&ctl->owner[x][slot][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int lo = __builtin_amdgcn_readfirstlane(static_cast<int>(o & 0xffffffffu));
        const int hi = __builtin_amdgcn_readfirstlane(static_cast<int>(o >> 32));
        if (lo == l + 1)
            return hi;
        const int t = load_agent(&ctl->ticket[x][0]);
        if ((t & kClaimedEmpty) && (t & ~kClaimedEmpty) - 1 <= l)
            return -1;
        if (load_agent(&ctl->abort_word))
            return -1;
        nap(n);
    }
    __hip_atomic_store(&ctl->abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return -1;
}

template <class P1, class P2, bool ROT>
__global__ void __launch_bounds__(P1::THREADS)
split_fft_xcd_kernel(const float* xr, const float* xi, float* yr, float* yi, const float2* __restrict__ tw,
                     int64_t batch, const int64_t* __restrict__ rows, float* ring, XcdControl* ctl, int slots,
                     int limit)
{
    static_assert(P1::PASS == 1 && P2::PASS == 2 && P1::M == P2::M && P1::A == P2::A, "one length, both passes");
    static_assert(P1::THREADS == P2::THREADS && P1::SPLIT && P2::SPLIT && P1::WSC == P2::WSC,
                  "one workgroup shape, split-plane tiles, one workspace layout");
    constexpr int N = P1::N;
    constexpr int T1 = P1::TILES, T2 = P2::TILES, T = T1;
    static_assert(T1 == T2, "every item runs one tile of each pass");
    constexpr int LDS_WORDS = P1::LDS_WORDS > P2::LDS_WORDS ? P1::LDS_WORDS : P2::LDS_WORDS;
    __shared__ float lds[LDS_WORDS];
    __shared__ int s_word;
    const int tid = threadIdx.x;
    const int x = xcd_queue();
    const bool wave0 = __builtin_amdgcn_readfirstlane(tid) == 0;
    int ok = 1;
    for (;;) {
        if (tid == 0)
            s_word = __hip_atomic_fetch_add(&ctl->head[x][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_word);
        __syncthreads();
        const int l = k / T, r = k % T, slot = l % slots, gen = l / slots;
        // the thread index, opaque to the compiler once per item: its tile
        // address arithmetic is redone per item instead of being hoisted out
        // of the loop and held in registers for all of it
        int lane_tid = tid;
        asm volatile("" : "+v"(lane_tid));
        // which transform local transform l is (wave 0 decides, the workgroup follows)
        if (wave0) {
            int g = -1;
            if (r == 0) {
                const int t = xcd_wait_ticket(ctl, x, l, limit);
                if (t >= 0 && !(t & kClaimedEmpty)) {
                    unsigned long long c = 0;
                    if (tid == 0)
                        c = __hip_atomic_fetch_add(&ctl->next_transform[0], 1ull, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                    const unsigned lo = static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(c)));
                    const unsigned hi =
                        static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(c >> 32)));
                    c = lo | (static_cast<unsigned long long>(hi) << 32);
                    const bool valid = c < static_cast<unsigned long long>(batch);
                    if (tid == 0)
                        __hip_atomic_store(&ctl->ticket[x][0], (l + 1) | (valid ? 0 : kClaimedEmpty),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (valid) {
                        g = static_cast<int>(c);
                        // the slot's previous transform has been read by all its pass-2 tiles
                        ok &= xcd_wait_geq(&ctl->gathered[x][slot][0], T2 * gen, ctl, limit);
                        if (tid == 0)
                            __hip_atomic_store(&ctl->owner[x][slot][0],
                                               static_cast<unsigned long long>(l + 1) |
                                                   (static_cast<unsigned long long>(g) << 32),
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
            } else {
                g = xcd_wait_owner(ctl, x, slot, l, limit);
            }
            if (tid == 0)
                s_word = g;
        }
        __syncthreads();
        const int g = __builtin_amdgcn_readfirstlane(s_word);
        if (g < 0)
            break;
        const int64_t dbase = rows ? rows[g] : static_cast<int64_t>(g) * N;
        float* wr = ring + (static_cast<int64_t>(x) * slots + slot) * (2 * N);
        float* wi = wr + N;
        // pass-1 tile r into the slot
        if constexpr (ROT) {
            const int rot = static_cast<int>(((reinterpret_cast<uintptr_t>(xr) >> 2) + dbase) & 31);
            tile_process<P1>(PlaneSrc<true>{xr + dbase}, PlaneSrc<true>{xi + dbase}, wr, wi, tw,
                             TileCols<true>{r * P1::C, rot}, lds, lane_tid, NoHook{});
        } else {
            tile_process<P1>(PlaneSrc<true>{xr + dbase}, PlaneSrc<true>{xi + dbase}, wr, wi, tw,
                             TileCols<false>{r * P1::C}, lds, lane_tid, NoHook{});
        }
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores acknowledged by L2
        __syncthreads();
        if (tid == 0)
            __hip_atomic_fetch_add(&ctl->written[x][slot][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // the transform's other pass-1 tiles
        if (wave0) {
            const bool w = xcd_wait_geq(&ctl->written[x][slot][0], T1 * (gen + 1), ctl, limit);
            if (tid == 0)
                s_word = w;
        }
        __syncthreads();
        ok &= __builtin_amdgcn_readfirstlane(s_word);
        // pass-2 tile r out of the slot, which is released as soon as its
        // loads have been consumed
        int* gathered = &ctl->gathered[x][slot][0];
        auto release = [gathered, tid]() {
            if (tid == 0)
                __hip_atomic_fetch_add(gathered, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        tile_process<P2>(L2Src{plane_rsrc(wr, N)}, L2Src{plane_rsrc(wi, N)}, yr + dbase, yi + dbase, tw,
                         TileCols<false>{r * P2::C}, lds, lane_tid, release);
    }
    if (!ok && tid == 0)
        atomicAdd(&ctl->failed, 1);
}

// Zeroes the control block (vec4s 16-byte words, the block's rounded size).
__global__ void __launch_bounds__(256) xcd_control_clear(float4* ctl, int vec4s)
{
    for (int i = blockIdx.x * 256 + threadIdx.x; i < vec4s; i += gridDim.x * 256)
        ctl[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace

// Floats of the ring of a length-2^m schedule with `slots` slots per XCD.
constexpr int64_t xcd_ring_floats(int m, int slots) { return int64_t{kXcds} * slots * 2 * (int64_t{1} << m); }

constexpr size_t xcd_control_bytes() { return (sizeof(XcdControl) + 255) / 256 * 256; }

}  // namespace splitdft
