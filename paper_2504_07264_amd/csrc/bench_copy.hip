// Plain HBM streaming kernels that measure the achievable memory rate for the
// benchmark's byte counts: read-only, write-only and copy, with 16-byte
// nontemporal accesses like the transform kernels.  Built into a separate
// library (libsplitdft_bench.so); the transform library does not export them.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstddef>
#include <cstdint>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kVecPerThread = 4;  // 16-byte vectors per thread, strided by the workgroup

// mode 0: dst = src; 1: read src only; 2: write dst only.  The read-only
// kernel keeps its sum live by storing it where no value can match.
template <int MODE>
__global__ void __launch_bounds__(kThreads) stream_kernel(const v4f* __restrict__ src, v4f* __restrict__ dst,
                                                          int64_t nvec, float* sink)
{
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kThreads * kVecPerThread) + threadIdx.x;
    v4f v[kVecPerThread];
    if constexpr (MODE != 2) {
#pragma unroll
        for (int k = 0; k < kVecPerThread; ++k) {
            const int64_t i = base + k * kThreads;
            v[k] = i < nvec ? __builtin_nontemporal_load(src + i) : v4f{0.f, 0.f, 0.f, 0.f};
        }
    } else {
#pragma unroll
        for (int k = 0; k < kVecPerThread; ++k)
            v[k] = v4f{1.f, 2.f, 3.f, static_cast<float>(threadIdx.x)};
    }
    if constexpr (MODE != 1) {
#pragma unroll
        for (int k = 0; k < kVecPerThread; ++k) {
            const int64_t i = base + k * kThreads;
            if (i < nvec)
                __builtin_nontemporal_store(v[k], dst + i);
        }
    } else {
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < kVecPerThread; ++k)
            s += v[k][0] + v[k][1] + v[k][2] + v[k][3];
        if (s == -1.2345e30f)  // never for finite test data; keeps the loads
            sink[0] = s;
    }
}

// The transform's streams: two source planes to two destination planes
// (each n floats), VPP 16-byte vectors per plane per thread.
template <int VPP>
__global__ void __launch_bounds__(kThreads) planar_copy_kernel(const v4f* __restrict__ xr, const v4f* __restrict__ xi,
                                                               v4f* __restrict__ yr, v4f* __restrict__ yi, int64_t nvec)
{
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kThreads * VPP) + threadIdx.x;
    v4f a[VPP], b[VPP];
#pragma unroll
    for (int k = 0; k < VPP; ++k) {
        const int64_t i = base + k * kThreads;
        const bool in = i < nvec;
        a[k] = in ? __builtin_nontemporal_load(xr + i) : v4f{0.f, 0.f, 0.f, 0.f};
        b[k] = in ? __builtin_nontemporal_load(xi + i) : v4f{0.f, 0.f, 0.f, 0.f};
    }
#pragma unroll
    for (int k = 0; k < VPP; ++k) {
        const int64_t i = base + k * kThreads;
        if (i < nvec) {
            __builtin_nontemporal_store(a[k], yr + i);
            __builtin_nontemporal_store(b[k], yi + i);
        }
    }
}

// One 16-byte vector per thread (the fastest single-array copy measured).
__global__ void __launch_bounds__(kThreads) copy1_kernel(const v4f* __restrict__ src, v4f* __restrict__ dst, int64_t nvec)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (i < nvec)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" {

// Stream n_floats floats (a multiple of 4, 16-byte aligned pointers) on the
// given hipStream_t.  mode 0 copies src to dst, 1 reads src, 2 writes dst;
// 3 copies the two halves of src (two planes) to the two halves of dst, four
// vectors per plane per thread, as the transform kernels stream them (n_floats
// a multiple of 8); 4 copies src to dst with one vector per thread; sink: one
// float of device memory (mode 1).  Returns a hipError_t value.
int splitdft_bench_stream(const float* src, float* dst, int64_t n_floats, int mode, float* sink, void* stream)
{
    if (n_floats <= 0 || n_floats % 4 != 0 || mode < 0 || mode > 4 || (mode == 3 && n_floats % 8 != 0))
        return static_cast<int>(hipErrorInvalidValue);
    if ((mode != 2 && (!src || reinterpret_cast<uintptr_t>(src) % 16 != 0)) ||
        (mode != 1 && (!dst || reinterpret_cast<uintptr_t>(dst) % 16 != 0)) || (mode == 1 && !sink))
        return static_cast<int>(hipErrorInvalidValue);
    const int64_t nvec = n_floats / 4;
    const int64_t blocks = (nvec + kThreads * kVecPerThread - 1) / (kThreads * kVecPerThread);
    if (blocks > INT_MAX)
        return static_cast<int>(hipErrorInvalidValue);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const v4f* s = reinterpret_cast<const v4f*>(src);
    v4f* d = reinterpret_cast<v4f*>(dst);
    const dim3 grid(static_cast<unsigned>(blocks)), block(kThreads);
    if (mode == 3) {
        const int64_t half = nvec / 2;
        const int64_t pblocks = (half + kThreads * 4 - 1) / (kThreads * 4);
        hipLaunchKernelGGL(planar_copy_kernel<4>, dim3(static_cast<unsigned>(pblocks)), block, 0, st, s, s + half, d,
                           d + half, half);
        return static_cast<int>(hipGetLastError());
    }
    if (mode == 4) {
        const int64_t blocks1 = (nvec + kThreads - 1) / kThreads;
        if (blocks1 > INT_MAX)
            return static_cast<int>(hipErrorInvalidValue);
        hipLaunchKernelGGL(copy1_kernel, dim3(static_cast<unsigned>(blocks1)), block, 0, st, s, d, nvec);
        return static_cast<int>(hipGetLastError());
    }
    if (mode == 0)
        hipLaunchKernelGGL(stream_kernel<0>, grid, block, 0, st, s, d, nvec, sink);
    else if (mode == 1)
        hipLaunchKernelGGL(stream_kernel<1>, grid, block, 0, st, s, d, nvec, sink);
    else
        hipLaunchKernelGGL(stream_kernel<2>, grid, block, 0, st, s, d, nvec, sink);
    return static_cast<int>(hipGetLastError());
}

}  // extern "C"
