// C ABI of the split-format DFT library: plans, argument validation, launch.
#include "../../include/split_dft.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

struct split_dft_plan_s {
    int64_t n;
    int64_t batch;
    int m;
    uint32_t flags;
    int device;
    float2* d_tw;  // 2^m entries: (cos, sin) of omega^(i,q) at 2^(i-1)+q
    const splitdft::Variant* variant;  // FP32 schedule (mode == kModeFP32)
    int mode;                          // precision mode (plan flags & 0xff)
    float* d_mfma;  // matrix-core modes: constant operands, then 256 (cos, sin) pairs
    const splitdft::TwoPass* two;  // two-pass schedule (large lengths), else NULL
    int64_t chunk;                 // transforms per two-pass chunk
    float* d_ws;                   // plan-owned workspace: 2 planes x chunk x n floats
    size_t ws_bytes;
};

namespace {

thread_local std::string g_last_error;

// Lengths 2^15 and 2^16 use the two-pass schedule by default.  A transform of
// 2^16 (512 KiB) does not fit a CU's LDS and registers; one of 2^15 does, but
// the single-workgroup kernel (one transform per CU) is bound by its
// arithmetic and latency rather than by memory, and measured slower than two
// passes on most devices.  Lengths up to 2^14 run in a single pass.
constexpr int kTwoPassDefaultLog2N = 15;
// Workspace per two-pass chunk (both planes); measured on MI355X, chunks of
// 256 MiB beat smaller ones (fewer, larger launches: 85.3 / 88.0 µs per 2^24
// points at 2^15 / 2^16 against 88.6 / 91.8 µs with 128 MiB, for batches of
// 2^25 points and more) and larger ones (the intermediate outgrows the
// memory-side cache).
constexpr int64_t kTwoPassChunkBytes = int64_t{256} << 20;

std::mutex g_plans_mu;
std::unordered_set<const split_dft_plan_s*>& live_plans()
{
    static auto* s = new std::unordered_set<const split_dft_plan_s*>();
    return *s;
}

split_dft_status fail(split_dft_status st, const std::string& msg)
{
    g_last_error = msg;
    return st;
}

}  // namespace

void splitdft::set_last_error(const std::string& msg) { g_last_error = msg; }

namespace {

split_dft_status fail_hip(hipError_t e, const char* what)
{
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return SPLIT_DFT_ERR_HIP;
}

bool log_enabled()
{
    const char* v = std::getenv("SPLIT_DFT_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
}

int exact_log2(int64_t n)
{
    if (n < 1)
        return -1;
    int m = 0;
    while ((int64_t{1} << m) < n && m < 62)
        ++m;
    return (int64_t{1} << m) == n ? m : -1;
}

bool plan_is_live(const split_dft_plan_s* p)
{
    std::lock_guard<std::mutex> g(g_plans_mu);
    return live_plans().count(p) != 0;
}

bool overlaps(const void* a, const void* b, size_t bytes)
{
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

// [a, a + abytes) and [b, b + bbytes) intersect
bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

split_dft_status validate_io(const split_dft_plan_s* p, const float* xr, const float* xi, const float* yr,
                             const float* yi)
{
    if (!xr || !xi || !yr || !yi)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "a data pointer is NULL");
    for (const void* q : {static_cast<const void*>(xr), static_cast<const void*>(xi), static_cast<const void*>(yr),
                          static_cast<const void*>(yi)})
        if (reinterpret_cast<uintptr_t>(q) % 16 != 0)
            return fail(SPLIT_DFT_ERR_MISALIGNED, "data pointers must be 16-byte aligned");
    const size_t bytes = static_cast<size_t>(p->n) * static_cast<size_t>(p->batch) * sizeof(float);
    if (overlaps(yr, yi, bytes))
        return fail(SPLIT_DFT_ERR_ALIASING, "the two output planes overlap");
    for (const float* out : {yr, yi})
        for (const float* in : {xr, xi})
            if (out != in && overlaps(out, in, bytes))
                return fail(SPLIT_DFT_ERR_ALIASING, "an output partially overlaps an input");
    return SPLIT_DFT_OK;
}

// Planes of one direction of a call.
struct Io {
    const float* xr;
    const float* xi;
    float* yr;
    float* yi;
};

// Arguments of one or two directions (dir[1].xr == NULL: one); makes no HIP
// call.  A second direction may run in the same launch as the first, so its
// arrays may not overlap the first direction's.
split_dft_status validate_call(split_dft_plan_t p, const Io* dir, int ndir)
{
    if (!p || !plan_is_live(p))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "plan is NULL, destroyed or not created by split_dft_plan");
    for (int k = 0; k < ndir; ++k) {
        const split_dft_status vs = validate_io(p, dir[k].xr, dir[k].xi, dir[k].yr, dir[k].yi);
        if (vs != SPLIT_DFT_OK)
            return vs;
    }
    const size_t bytes = static_cast<size_t>(p->n) * static_cast<size_t>(p->batch) * sizeof(float);
    if (ndir == 2) {
        // the directions may run concurrently: no output of one may touch the other's arrays
        for (int k = 0; k < 2; ++k)
            for (const float* out : {dir[k].yr, dir[k].yi})
                for (const float* other : {dir[1 - k].xr, dir[1 - k].xi, static_cast<const float*>(dir[1 - k].yr),
                                           static_cast<const float*>(dir[1 - k].yi)})
                    if (ranges_overlap(out, bytes, other, bytes))
                        return fail(SPLIT_DFT_ERR_ALIASING, "forward and adjoint arrays overlap");
    }
    return SPLIT_DFT_OK;
}

// The plan's tables live on the device it was created on.
split_dft_status check_device(const split_dft_plan_s* p)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device)
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "the plan belongs to HIP device " + std::to_string(p->device) +
                                                    ", the current device is " + std::to_string(cur));
    return SPLIT_DFT_OK;
}

// Launch validated directions on the stream.  Two-pass plans go through the
// workspace w in chunks of `chunk` transforms (w holds 2 * chunk * n floats);
// single-pass FP32 schedules run a second direction in the same launch.
split_dft_status launch_dirs(const split_dft_plan_s* p, const Io* dir, int ndir, float* w, int64_t chunk,
                             hipStream_t st)
{
    if (p->two && p->two->fused) {
        // both passes in one launch per direction, the ring and its control block in w
        for (int k = 0; k < ndir; ++k) {
            const hipError_t e =
                p->two->fused(dir[k].xr, dir[k].xi, dir[k].yr, dir[k].yi, p->d_tw, p->batch, nullptr, w, st);
            if (e != hipSuccess)
                return fail_hip(e, "fused two-pass kernel launch");
        }
        return SPLIT_DFT_OK;
    }
    if (p->two) {
        float* wr = w;
        float* wi = w + chunk * p->n;
        for (int k = 0; k < ndir; ++k)
            for (int64_t s0 = 0; s0 < p->batch; s0 += chunk) {
                const int64_t c = p->batch - s0 < chunk ? p->batch - s0 : chunk;
                const int64_t off = s0 * p->n;
                hipError_t e = p->two->pass1(dir[k].xr + off, dir[k].xi + off, wr, wi, p->d_tw, c, nullptr, st);
                if (e == hipSuccess)
                    e = p->two->pass2(wr, wi, dir[k].yr + off, dir[k].yi + off, p->d_tw, c, nullptr, st);
                if (e != hipSuccess)
                    return fail_hip(e, "two-pass kernel launch");
            }
        return SPLIT_DFT_OK;
    }
    if (p->mode == splitdft::kModeFP32) {
        const splitdft::Dir2 second{dir[1].xr, dir[1].xi, dir[1].yr, dir[1].yi};
        const hipError_t e = p->variant->launch(dir[0].xr, dir[0].xi, dir[0].yr, dir[0].yi, p->d_tw, p->batch,
                                                nullptr, st, ndir == 2 ? &second : nullptr);
        if (e != hipSuccess)
            return fail_hip(e, "kernel launch");
        return SPLIT_DFT_OK;
    }
    for (int k = 0; k < ndir; ++k) {
        const hipError_t e =
            splitdft::launch_mfma(p->mode, p->m, dir[k].xr, dir[k].xi, dir[k].yr, dir[k].yi, p->d_mfma,
                                  reinterpret_cast<const float2*>(p->d_mfma + splitdft::kMfmaConstFloats), p->batch,
                                  st);
        if (e != hipSuccess)
            return fail_hip(e, "kernel launch");
    }
    return SPLIT_DFT_OK;
}

// One or two directions on the caller's stream, through the caller's
// workspace ws (NULL: the plan's own).
split_dft_status run(split_dft_plan_t p, const Io* dir, int ndir, void* ws, size_t ws_bytes, void* stream)
{
    split_dft_status vs = validate_call(p, dir, ndir);
    if (vs != SPLIT_DFT_OK)
        return vs;
    const size_t bytes = static_cast<size_t>(p->n) * static_cast<size_t>(p->batch) * sizeof(float);
    float* w = static_cast<float*>(ws);
    if (p->two) {
        if (!w) {
            w = p->d_ws;
            if (!w)
                return fail(SPLIT_DFT_ERR_NULL_POINTER,
                            "the plan was created with SPLIT_DFT_CALLER_WORKSPACE: pass a workspace of "
                            "split_dft_workspace_bytes(plan) = " + std::to_string(p->ws_bytes) + " bytes");
        } else {
            if (ws_bytes < p->ws_bytes)
                return fail(SPLIT_DFT_ERR_INVALID_BATCH, "workspace smaller than split_dft_workspace_bytes");
            if (reinterpret_cast<uintptr_t>(w) % 16 != 0)
                return fail(SPLIT_DFT_ERR_MISALIGNED, "workspace must be 16-byte aligned");
            for (int k = 0; k < ndir; ++k)
                for (const void* q : {static_cast<const void*>(dir[k].xr), static_cast<const void*>(dir[k].xi),
                                      static_cast<const void*>(dir[k].yr), static_cast<const void*>(dir[k].yi)})
                    if (ranges_overlap(w, p->ws_bytes, q, bytes))
                        return fail(SPLIT_DFT_ERR_ALIASING, "workspace overlaps a data array");
        }
    }
    vs = check_device(p);
    if (vs != SPLIT_DFT_OK)
        return vs;
    return launch_dirs(p, dir, ndir, w, p->chunk, static_cast<hipStream_t>(stream));
}

// C gr - S gi = imaginary part and S gr + C gi = real part of the forward
// transform of (gi, gr): the adjoint is the forward kernel with both plane
// pairs exchanged.
Io adjoint_io(const float* gr, const float* gi, float* gxr, float* gxi) { return Io{gi, gr, gxi, gxr}; }

}  // namespace

namespace splitdft {

split_dft_status exec_in_scratch(split_dft_plan_t p, const float* xr, const float* xi, float* yr, float* yi,
                                 void* stream, ScratchLookup lookup)
{
    const Io io[2] = {{xr, xi, yr, yi}, {}};
    split_dft_status vs = validate_call(p, io, 1);
    if (vs != SPLIT_DFT_OK)
        return vs;
    vs = check_device(p);
    if (vs != SPLIT_DFT_OK)
        return vs;
    float* w = nullptr;
    int64_t chunk = p->chunk;
    if (p->two) {
        size_t cap = 0;
        const hipError_t e = lookup(p->device, &w, &cap);
        if (e != hipSuccess)
            return fail_hip(e, "address of the static scratch array");
        if (p->two->fused) {
            if (cap < splitdft::fused_workspace_bytes(p->two))
                return fail(SPLIT_DFT_ERR_UNSUPPORTED, "the fused schedule's ring (" +
                                                           std::to_string(splitdft::fused_workspace_bytes(p->two)) +
                                                           " bytes) exceeds the static scratch (" +
                                                           std::to_string(cap) + " bytes)");
            return launch_dirs(p, io, 1, w, chunk, static_cast<hipStream_t>(stream));
        }
        const int64_t per = p->n * 2 * static_cast<int64_t>(sizeof(float));
        const int64_t fit = static_cast<int64_t>(cap) / per;
        if (fit < 1)
            return fail(SPLIT_DFT_ERR_UNSUPPORTED, "one transform's intermediate (" + std::to_string(per) +
                                                       " bytes) exceeds the static scratch (" +
                                                       std::to_string(cap) + " bytes)");
        if (fit < chunk) {
            // equal chunks of at most `fit` transforms
            const int64_t nchunks = (p->batch + fit - 1) / fit;
            chunk = (p->batch + nchunks - 1) / nchunks;
        }
    }
    return launch_dirs(p, io, 1, w, chunk, static_cast<hipStream_t>(stream));
}

}  // namespace splitdft

extern "C" {

split_dft_status split_dft_plan(split_dft_plan_t* out, int64_t n, int64_t batch, uint32_t flags)
{
    if (!out)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "out is NULL");
    const int m = exact_log2(n);
    if (m < 0 || m > SPLIT_DFT_MAX_LOG2N)
        return fail(SPLIT_DFT_ERR_INVALID_LENGTH, "n must be 2^m with 0 <= m <= 16, got " + std::to_string(n));
    if (batch < 1)
        return fail(SPLIT_DFT_ERR_INVALID_BATCH, "batch must be >= 1, got " + std::to_string(batch));
    if (batch > INT64_MAX / n / static_cast<int64_t>(sizeof(float)))
        return fail(SPLIT_DFT_ERR_INVALID_BATCH, "n * batch * 4 bytes overflows int64");
    const uint32_t precision = flags & 0xffu;
    const uint32_t vsel = (flags >> 8) & 0xffu;  // 0 = default schedule, k = compiled schedule k-1
    const bool dif = (flags & SPLIT_DFT_DIF) != 0;
    const bool caller_ws = (flags & SPLIT_DFT_CALLER_WORKSPACE) != 0;
    if (precision > SPLIT_DFT_BF16X3 || ((flags & ~(SPLIT_DFT_DIF | SPLIT_DFT_CALLER_WORKSPACE)) >> 16) != 0)
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "unsupported flags " + std::to_string(flags));
    const int mode = static_cast<int>(precision);
    if (mode != splitdft::kModeFP32 && (m != 8 || vsel != 0 || dif))
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "matrix-core precision modes support n = 256 (DIT) only");

    // schedules: the compiled single-pass variants, then the two-pass ones;
    // selector 0 = the default for the length
    int count = 0, count2 = 0;
    const splitdft::Variant* list =
        dif ? splitdft::dif_variants_for(m, &count) : splitdft::variants_for(m, &count);
    const splitdft::TwoPass* list2 = dif ? splitdft::dif_two_pass_for(m, &count2) : splitdft::two_pass_for(m, &count2);
    if (dif && count == 0 && count2 == 0)
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "no decimation-in-frequency schedule for n = " + std::to_string(n));
    const splitdft::Variant* v = nullptr;
    const splitdft::TwoPass* two = nullptr;
    if (vsel == 0) {
        if (mode != splitdft::kModeFP32 || count > 0)
            v = dif ? &list[0] : splitdft::default_variant(m, batch);
        if ((!dif && m >= kTwoPassDefaultLog2N) || !v)
            two = count2 > 0 ? &list2[0] : nullptr;
        if (two)
            v = nullptr;
    } else if (static_cast<int>(vsel) <= count) {
        v = &list[vsel - 1];
    } else if (static_cast<int>(vsel) <= count + count2) {
        two = &list2[vsel - 1 - count];
    }
    if (!v && !two)
        return fail(SPLIT_DFT_ERR_UNSUPPORTED,
                    "no compiled schedule for n = " + std::to_string(n) + " (selector " + std::to_string(vsel) + ")");

    const char* inj = std::getenv("SPLIT_DFT_FAIL_ALLOC");
    if (inj && *inj && std::strcmp(inj, "0") != 0)
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "allocation failure forced by SPLIT_DFT_FAIL_ALLOC");

    std::vector<float> c(static_cast<size_t>(n)), s(static_cast<size_t>(n));
    splitdft::build_twiddles_f32(m, c.data(), s.data());
    std::vector<float2> tw(static_cast<size_t>(n));
    for (int64_t j = 0; j < n; ++j)
        tw[static_cast<size_t>(j)] = make_float2(c[static_cast<size_t>(j)], s[static_cast<size_t>(j)]);

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return fail_hip(e, "hipGetDevice");
    float2* d_tw = nullptr;
    e = hipMalloc(&d_tw, sizeof(float2) * static_cast<size_t>(n));
    if (e == hipErrorOutOfMemory)
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "hipMalloc of the twiddle table failed");
    if (e != hipSuccess)
        return fail_hip(e, "hipMalloc");
    e = hipMemcpy(d_tw, tw.data(), sizeof(float2) * static_cast<size_t>(n), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_tw);
        return fail_hip(e, "hipMemcpy of the twiddle table");
    }
    float* d_mfma = nullptr;
    if (mode != splitdft::kModeFP32) {
        std::vector<float> tab(splitdft::kMfmaConstFloats + 2 * 256);
        std::vector<uint16_t> enc(2 * splitdft::kMfmaConstFloats);
        splitdft::build_mfma256_constants(mode, enc.data());
        std::memcpy(tab.data(), enc.data(), sizeof(uint16_t) * enc.size());
        splitdft::build_tw256(tab.data() + splitdft::kMfmaConstFloats);
        e = hipMalloc(&d_mfma, sizeof(float) * tab.size());
        if (e == hipSuccess)
            e = hipMemcpy(d_mfma, tab.data(), sizeof(float) * tab.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (d_mfma)
                (void)hipFree(d_mfma);
            (void)hipFree(d_tw);
            return e == hipErrorOutOfMemory ? fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "hipMalloc of the matrix-core tables")
                                            : fail_hip(e, "matrix-core tables");
        }
    }
    int64_t chunk = 0;
    size_t ws_bytes = 0;
    float* d_ws = nullptr;
    if (two) {
        int64_t chunk_bytes = kTwoPassChunkBytes;
        if (const char* cb = std::getenv("SPLIT_DFT_CHUNK_MIB"))  // tuning override, 1 MiB .. 64 GiB
            if (std::atoll(cb) > 0)
                chunk_bytes = std::min<int64_t>(std::atoll(cb), int64_t{1} << 16) << 20;
        chunk = chunk_bytes / (n * 2 * static_cast<int64_t>(sizeof(float)));
        chunk = chunk < 1 ? 1 : (chunk > batch ? batch : chunk);
        // equal chunks: no short launch at the end
        const int64_t nchunks = (batch + chunk - 1) / chunk;
        chunk = (batch + nchunks - 1) / nchunks;
        ws_bytes = static_cast<size_t>(chunk) * static_cast<size_t>(n) * 2 * sizeof(float);
        if (two->fused) {
            // one launch over the whole batch through the ring
            chunk = batch;
            ws_bytes = splitdft::fused_workspace_bytes(two);
        }
        e = caller_ws ? hipSuccess : hipMalloc(&d_ws, ws_bytes);
        if (e != hipSuccess) {
            if (d_mfma)
                (void)hipFree(d_mfma);
            (void)hipFree(d_tw);
            return e == hipErrorOutOfMemory ? fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "hipMalloc of the workspace")
                                            : fail_hip(e, "hipMalloc of the workspace");
        }
    }
    if (two)
        splitdft::prepare_noalloc_scratch(dev);  // set-up: the no-allocation entry point's array
    auto* p = new (std::nothrow)
        split_dft_plan_s{n, batch, m, flags, dev, d_tw, v, mode, d_mfma, two, chunk, d_ws, ws_bytes};
    if (!p) {
        if (d_mfma)
            (void)hipFree(d_mfma);
        if (d_ws)
            (void)hipFree(d_ws);
        (void)hipFree(d_tw);
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "host allocation of the plan failed");
    }
    {
        std::lock_guard<std::mutex> g(g_plans_mu);
        live_plans().insert(p);
    }
    if (log_enabled()) {
        char desc[256];
        split_dft_plan_describe(p, desc, sizeof(desc));
        std::fprintf(stderr, "[split_dft] plan n=%lld batch=%lld %s\n", static_cast<long long>(n),
                     static_cast<long long>(batch), desc);
    }
    *out = p;
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_exec(split_dft_plan_t plan, const float* xr, const float* xi, float* yr, float* yi,
                                void* stream)
{
    const Io io[2] = {{xr, xi, yr, yi}, {}};
    return run(plan, io, 1, nullptr, 0, stream);
}

split_dft_status split_dft_exec_ws(split_dft_plan_t plan, const float* xr, const float* xi, float* yr, float* yi,
                                   void* workspace, size_t workspace_bytes, void* stream)
{
    const Io io[2] = {{xr, xi, yr, yi}, {}};
    return run(plan, io, 1, workspace, workspace_bytes, stream);
}

split_dft_status split_dft_adjoint(split_dft_plan_t plan, const float* gr, const float* gi, float* gxr, float* gxi,
                                   void* stream)
{
    const Io io[2] = {adjoint_io(gr, gi, gxr, gxi), {}};
    return run(plan, io, 1, nullptr, 0, stream);
}

split_dft_status split_dft_adjoint_ws(split_dft_plan_t plan, const float* gr, const float* gi, float* gxr,
                                      float* gxi, void* workspace, size_t workspace_bytes, void* stream)
{
    const Io io[2] = {adjoint_io(gr, gi, gxr, gxi), {}};
    return run(plan, io, 1, workspace, workspace_bytes, stream);
}

split_dft_status split_dft_exec_adjoint(split_dft_plan_t plan, const float* xr, const float* xi, float* yr,
                                        float* yi, const float* gr, const float* gi, float* gxr, float* gxi,
                                        void* stream)
{
    const Io io[2] = {{xr, xi, yr, yi}, adjoint_io(gr, gi, gxr, gxi)};
    return run(plan, io, 2, nullptr, 0, stream);
}

split_dft_status split_dft_exec_adjoint_ws(split_dft_plan_t plan, const float* xr, const float* xi, float* yr,
                                           float* yi, const float* gr, const float* gi, float* gxr, float* gxi,
                                           void* workspace, size_t workspace_bytes, void* stream)
{
    const Io io[2] = {{xr, xi, yr, yi}, adjoint_io(gr, gi, gxr, gxi)};
    return run(plan, io, 2, workspace, workspace_bytes, stream);
}

split_dft_status split_dft_destroy(split_dft_plan_t plan)
{
    if (!plan)
        return SPLIT_DFT_OK;
    {
        std::lock_guard<std::mutex> g(g_plans_mu);
        if (live_plans().erase(plan) == 0)
            return fail(SPLIT_DFT_ERR_INVALID_PLAN, "plan is destroyed or not created by split_dft_plan");
    }
    int cur = 0;
    const bool switch_dev = hipGetDevice(&cur) == hipSuccess && cur != plan->device;
    if (switch_dev)
        (void)hipSetDevice(plan->device);
    hipError_t e = hipFree(plan->d_tw);
    if (plan->d_ws) {
        const hipError_t e2 = hipFree(plan->d_ws);
        if (e == hipSuccess)
            e = e2;
    }
    if (plan->d_mfma) {
        const hipError_t e2 = hipFree(plan->d_mfma);
        if (e == hipSuccess)
            e = e2;
    }
    if (switch_dev)
        (void)hipSetDevice(cur);
    delete plan;
    if (e != hipSuccess)
        return fail_hip(e, "hipFree");
    return SPLIT_DFT_OK;
}

size_t split_dft_workspace_bytes(split_dft_plan_t plan)
{
    if (!plan || !plan_is_live(plan))
        return 0;
    return plan->ws_bytes;
}

split_dft_status split_dft_plan_info(split_dft_plan_t plan, int64_t* n, int64_t* batch, int* log2n, int* ept,
                                     int* tpw)
{
    if (!plan || !plan_is_live(plan))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "plan is NULL, destroyed or not created by split_dft_plan");
    if (n)
        *n = plan->n;
    if (batch)
        *batch = plan->batch;
    if (log2n)
        *log2n = plan->m;
    if (ept)
        *ept = plan->variant ? 1 << plan->variant->rb : 16;
    if (tpw)
        *tpw = plan->variant ? plan->variant->tpw : 0;
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_plan_describe(split_dft_plan_t plan, char* buf, size_t len)
{
    if (!plan || !plan_is_live(plan))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "plan is NULL, destroyed or not created by split_dft_plan");
    if (!buf || len == 0)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "buf is NULL or len is 0");
    if (plan->mode != splitdft::kModeFP32) {
        static const char* names[] = {"fp32", "bf16x2", "fp16x2", "bf16x3"};
        std::snprintf(buf, len, "mfma16x16x32 %s two 16-point contractions, 4 waves/workgroup", names[plan->mode]);
        return SPLIT_DFT_OK;
    }
    if (plan->two) {
        const splitdft::TwoPass* t = plan->two;
        if (t->fused) {
            std::snprintf(buf, len,
                          "two-pass fused a=%d: %d blocks / %d columns per tile, %d threads, lds=%d, "
                          "ring %d transforms per XCD",
                          t->a, t->c1, t->c2, t->threads1, t->lds1 > t->lds2 ? t->lds1 : t->lds2, t->slots);
            return SPLIT_DFT_OK;
        }
        if (t->dif) {
            std::snprintf(buf, len,
                          "dif two-pass a=%d: pass1 %d columns/wg %d threads lds=%d gf=%d, pass2 %d blocks/wg %d "
                          "threads lds=%d ws=%s, chunk=%lld",
                          t->a, t->c1, t->threads1, t->lds1, t->gf2 ? 1 : 0, t->c2, t->threads2, t->lds2,
                          t->wst ? "tiled" : "natural", static_cast<long long>(plan->chunk));
            return SPLIT_DFT_OK;
        }
        std::snprintf(buf, len,
                      "two-pass a=%d: pass1 %d blocks/wg %d threads lds=%d, pass2 %d columns/wg %d threads lds=%d "
                      "gf=%d ws=%s, chunk=%lld",
                      t->a, t->c1, t->threads1, t->lds1, t->c2, t->threads2, t->lds2, t->gf2 ? 1 : 0,
                      t->wst ? "tiled" : "natural", static_cast<long long>(plan->chunk));
        return SPLIT_DFT_OK;
    }
    const splitdft::Variant* v = plan->variant;
    std::snprintf(buf, len, "%sept=%d tpw=%d threads=%d lds=%d split=%d nt=%d twl=%d wpe=%d f4io=%d%s",
                  (plan->flags & SPLIT_DFT_DIF) ? "dif " : "", 1 << v->rb,
                  v->tpw, v->threads, v->lds_bytes, v->split ? 1 : 0, v->nt ? 1 : 0, v->twl, v->wpe,
                  v->f4io, v->pf ? " persistent" : "");
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_twiddle_table(int m, float* c, float* s)
{
    if (!c || !s)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "c or s is NULL");
    if (m < 0 || m > SPLIT_DFT_MAX_LOG2N)
        return fail(SPLIT_DFT_ERR_INVALID_LENGTH, "m must be in [0, 16]");
    splitdft::build_twiddles_f32(m, c, s);
    return SPLIT_DFT_OK;
}

const char* split_dft_status_string(int status)
{
    switch (status) {
    case SPLIT_DFT_OK: return "ok";
    case SPLIT_DFT_ERR_INVALID_LENGTH: return "invalid length";
    case SPLIT_DFT_ERR_INVALID_BATCH: return "invalid batch";
    case SPLIT_DFT_ERR_NULL_POINTER: return "null pointer";
    case SPLIT_DFT_ERR_MISALIGNED: return "misaligned pointer";
    case SPLIT_DFT_ERR_ALIASING: return "illegal aliasing";
    case SPLIT_DFT_ERR_UNSUPPORTED: return "unsupported";
    case SPLIT_DFT_ERR_OUT_OF_MEMORY: return "out of memory";
    case SPLIT_DFT_ERR_HIP: return "HIP runtime error";
    case SPLIT_DFT_ERR_INVALID_PLAN: return "invalid plan";
    }
    return "unknown status";
}

const char* split_dft_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
