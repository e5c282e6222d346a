// Data-movement model of a two-pass transform whose intermediate stays in the
// L2 cache of one XCD (accelerator complex die), without the transform's
// arithmetic: how fast pass-1 tiles can be handed to pass-2 tiles of the same
// transform by workgroups of one XCD, and how many of the intermediate's bytes
// still reach memory.  Benchmark library only (libsplitdft_bench.so).
//
// A "transform" is T tiles of 64 KB.  Pass-1 tile r is the input's tile r;
// pass-2 tile c gathers chunk c (64 KB / T) of every pass-1 tile, so every
// pass-2 tile depends on every pass-1 tile, as in the two passes of eq. (6)
// regrouped (Section III).  Output tile c, float j * (16384 / T) + e, is input
// tile j, float c * (16384 / T) + e.
//
// Each XCD has its own queue of items (tile r = k mod T of local transform
// k / T) and a ring of R transform-sized slots in device memory that its L2
// caches.  A workgroup takes an item, loads its input tile (nontemporal),
// waits until its ring slot is free, writes the tile there, waits until all T
// pass-1 tiles of the transform are written, gathers its pass-2 tile from the
// ring (loads that miss the CU's own cache and read L2), and writes it to the
// output (nontemporal).  The hand-over needs no agent-scope release: a store
// is acknowledged by the XCD's L2 (the wait on the store counter) before the
// counter that publishes it is incremented there, and the readers, on the same
// XCD, read L2.  A transform's T workgroups must be resident on the XCD at
// once (items are taken in order, so they are unless fewer than T workgroups
// of the launch are resident per XCD).  Every wait is bounded: after
// spin_limit polls a wait gives up, counts a timeout and sets the abort word,
// after which every wait returns at once, so the launch always finishes.
// "self" mode: each workgroup reads back its own pass-1 tile (no waiting on
// other workgroups), which isolates the cost of the ring round trip.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kTileFloats = 16384;  // 64 KB
constexpr int kXcds = 8;
constexpr int kLineInts = 32;       // every counter on its own 128-byte line
constexpr int kMaxSlots = 32;

struct Control {
    int head[kXcds][kLineInts];                   // next item per XCD
    int written[kXcds][kMaxSlots][kLineInts];     // pass-1 tiles written per slot (monotonic)
    int gathered[kXcds][kMaxSlots][kLineInts];    // pass-2 tiles gathered per slot (monotonic)
    int timeouts;
    int foreign_xcd;  // workgroups on an XCD index >= kXcds (did nothing)
    int abort_word;
};

__device__ __forceinline__ int xcd_index()
{
    // HW_REG_XCC_ID (register 20), bits 0..3: the XCD this wave runs on
    return __builtin_amdgcn_s_getreg(20 | (0 << 6) | ((4 - 1) << 11));
}

// Run by a whole wave, every decision on wave-uniform values: the loop has
// scalar branches only.
__device__ __forceinline__ bool wait_at_least(int* p, int target, int limit, int* abort_word)
{
    int nap = 1;
    for (int i = 0; i < limit; ++i) {
        const int v = __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (v >= target)
            return true;
        const int ab =
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (ab)
            return false;
        for (int j = 0; j < nap; ++j)
            __builtin_amdgcn_s_sleep(2);
        nap = nap < 8 ? 2 * nap : 8;
    }
    __hip_atomic_store(abort_word, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
}

template <int T>
__global__ void __launch_bounds__(kThreads)
l2_handover_kernel(const float* __restrict__ in, float* __restrict__ out, float* ring, Control* ctl,
                   int per_xcd, int slots, int spin_limit, int self)
{
    constexpr int TF = T * kTileFloats;  // floats per transform
    constexpr int CH = kTileFloats / T;  // floats per gathered chunk
    constexpr int V = kTileFloats / 4 / kThreads;
    __shared__ int s_item;
    __shared__ int s_ok;
    const int x = xcd_index();
    if (x >= kXcds) {
        if (threadIdx.x == 0)
            atomicAdd(&ctl->foreign_xcd, 1);
        return;
    }
    float* my_ring = ring + static_cast<size_t>(x) * slots * TF;
    const __amdgpu_buffer_rsrc_t rsrc =
        __builtin_amdgcn_make_buffer_rsrc(my_ring, static_cast<short>(0), slots * TF * 4, 0x00020000);
    const int nitems = per_xcd * T;
    auto wait_all = [&](int* p, int target) {
        if (__builtin_amdgcn_readfirstlane(threadIdx.x) == 0) {  // wave 0
            const bool ok = wait_at_least(p, target, spin_limit, &ctl->abort_word);
            if (threadIdx.x == 0)
                s_ok = ok;
        }
        __syncthreads();
        return __builtin_amdgcn_readfirstlane(s_ok);
    };
    int k = 0;
    do {
        if (threadIdx.x == 0)
            s_item = __hip_atomic_fetch_add(&ctl->head[x][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        k = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (k < nitems) {
            const int lt = k / T, r = k % T;
            const int slot = lt % slots, gen = lt / slots;
            const size_t g = static_cast<size_t>(lt) * kXcds + x;  // transform index in the arrays
            const v4f* src = reinterpret_cast<const v4f*>(in + g * TF + r * kTileFloats);
            v4f v[V];
#pragma unroll
            for (int j = 0; j < V; ++j)
                v[j] = __builtin_nontemporal_load(src + threadIdx.x + j * kThreads);
            int ok = wait_all(&ctl->gathered[x][slot][0], T * gen);
            v4f* dst = reinterpret_cast<v4f*>(my_ring + static_cast<size_t>(slot) * TF + r * kTileFloats);
#pragma unroll
            for (int j = 0; j < V; ++j)
                dst[threadIdx.x + j * kThreads] = v[j];
            __builtin_amdgcn_s_waitcnt(0);  // every store acknowledged by L2
            __syncthreads();
            if (threadIdx.x == 0)
                __hip_atomic_fetch_add(&ctl->written[x][slot][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!self)
                ok &= wait_all(&ctl->written[x][slot][0], T * (gen + 1));
#pragma unroll
            for (int j = 0; j < V; ++j) {
                const int f = 4 * (threadIdx.x + j * kThreads);
                const int part = f / CH, e = f % CH;
                const int fl = self ? slot * TF + r * kTileFloats + f : slot * TF + part * kTileFloats + r * CH + e;
                // aux 16: the load bypasses the CU's cache and reads L2
                v[j] = __builtin_bit_cast(
                    v4f, __builtin_amdgcn_raw_buffer_load_b128(rsrc, static_cast<unsigned>(fl) * 4u, 0, 16));
            }
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (threadIdx.x == 0) {
                __hip_atomic_fetch_add(&ctl->gathered[x][slot][0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (!ok)
                    atomicAdd(&ctl->timeouts, 1);
            }
            v4f* o = reinterpret_cast<v4f*>(out + g * TF + r * kTileFloats);
#pragma unroll
            for (int j = 0; j < V; ++j)
                __builtin_nontemporal_store(v[j], o + threadIdx.x + j * kThreads);
        }
    } while (k < nitems);
}

}  // namespace

extern "C" {

// Bytes of the control block (zeroed by the caller before each launch; its
// last three ints are the timeout count, the count of workgroups that found no
// XCD index below 8, and the abort word).
int64_t splitdft_bench_l2_control_bytes() { return static_cast<int64_t>(sizeof(Control)); }

// One launch of the hand-over model on `stream`: per_xcd transforms of T = tiles
// (4 or 8) 64-KB tiles per XCD, in and out each 8 * per_xcd * tiles * 16384
// floats, ring 8 * slots * tiles * 16384 floats (slots 1..32), control as above,
// grid workgroups of 256 threads (at least tiles per XCD must be resident at
// once), spin_limit polls per wait.  self != 0: read back the own tile.  All
// pointers 16-byte aligned device memory.  Returns a hipError_t value.
int splitdft_bench_l2_handover(const float* in, float* out, float* ring, void* control, int grid, int per_xcd,
                               int tiles, int slots, int self, int spin_limit, void* stream)
{
    const bool aligned = in && out && ring && control && reinterpret_cast<uintptr_t>(in) % 16 == 0 &&
                         reinterpret_cast<uintptr_t>(out) % 16 == 0 && reinterpret_cast<uintptr_t>(ring) % 16 == 0;
    if (!aligned || grid < 1 || per_xcd < 1 || slots < 1 || slots > kMaxSlots || spin_limit < 1 ||
        (tiles != 4 && tiles != 8) || static_cast<int64_t>(per_xcd) * kXcds * tiles * kTileFloats > INT64_MAX / 8 ||
        static_cast<int64_t>(slots) * tiles * kTileFloats * 4 > INT_MAX)
        return static_cast<int>(hipErrorInvalidValue);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    Control* ctl = static_cast<Control*>(control);
    if (tiles == 4)
        hipLaunchKernelGGL(l2_handover_kernel<4>, dim3(grid), dim3(kThreads), 0, st, in, out, ring, ctl, per_xcd,
                           slots, spin_limit, self);
    else
        hipLaunchKernelGGL(l2_handover_kernel<8>, dim3(grid), dim3(kThreads), 0, st, in, out, ring, ctl, per_xcd,
                           slots, spin_limit, self);
    return static_cast<int>(hipGetLastError());
}

}  // extern "C"
