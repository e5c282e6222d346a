// C ABI of grouped execution: a ragged batch of transforms of different
// power-of-two lengths, forward and/or adjoint, in one persistent launch,
// optionally captured once into a HIP graph.
#include "../../include/split_dft.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <unordered_set>
#include <vector>

// Transforms of one length >= 2^14 in the default (hybrid) mode: run by the
// per-length kernels, addressed through their element offsets.
struct ManyLarge {
    int m;
    int64_t count;
    int64_t* d_rows;                     // element offsets, count entries
    const splitdft::Variant* variant;    // single-pass schedule, or
    const splitdft::TwoPass* two;        // two-pass schedule through d_ws
    int64_t chunk;                       // transforms per workspace chunk
};

struct split_dft_many_s {
    int64_t count;
    int64_t points;
    int device;
    bool one_kernel;  // every length in the grouped kernel
    bool large_items; // the persistent kernel meets lengths >= 2^14 (its larger build)
    std::vector<ManyLarge> large;
    int variant;  // grouped-kernel build
    int grid;     // persistent workgroups
    std::vector<int64_t> offsets;  // host copy, count + 1 entries
    int64_t* d_offsets;  // offsets of the transforms in length order
    splitdft::ManyItem* d_items_one;   // forward only (direction 0)
    int n_one;
    splitdft::ManyItem* d_items_both;  // forward (0) and adjoint (1) interleaved
    int n_both;
    int* d_queue;
    float* d_ws;     // plan-owned workspace (NULL with SPLIT_DFT_CALLER_WORKSPACE)
    size_t ws_bytes; // workspace the plan's launches need
    float2* d_tw;
    // device data stays allocated while the handle is live or any captured
    // graph refers to it: destroy drops the handle's reference, each graph
    // holds one (guarded by g_mu)
    int refs;
};

struct split_dft_graph_s {
    hipGraph_t graph;
    hipGraphExec_t exec;
    split_dft_many_s* plan;  // whose device data the graph's kernels use
};

namespace {

std::mutex g_mu;
std::unordered_set<const void*>& live()
{
    static auto* s = new std::unordered_set<const void*>();
    return *s;
}

bool is_live(const void* p)
{
    std::lock_guard<std::mutex> g(g_mu);
    return live().count(p) != 0;
}

void set_live(const void* p, bool on)
{
    std::lock_guard<std::mutex> g(g_mu);
    if (on)
        live().insert(p);
    else
        live().erase(p);
}

// Remove p from the live set; false if it was not there.
bool take_live(const void* p)
{
    std::lock_guard<std::mutex> g(g_mu);
    return live().erase(p) != 0;
}

bool ranges_overlap(const void* a, size_t abytes, const void* b, size_t bbytes)
{
    const auto x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bbytes && y < x + abytes;
}

// Free a grouped plan's device data and host record (its device current).
void free_many(split_dft_many_s* p)
{
    for (ManyLarge& g : p->large)
        if (g.d_rows)
            (void)hipFree(g.d_rows);
    for (void* q : {static_cast<void*>(p->d_offsets), static_cast<void*>(p->d_items_one),
                    static_cast<void*>(p->d_items_both),
                    static_cast<void*>(p->d_queue), static_cast<void*>(p->d_ws), static_cast<void*>(p->d_tw)})
        if (q)
            (void)hipFree(q);
    delete p;
}

// Drop one reference to a plan's device data; the last one frees it (on the
// plan's device).
void release_many(split_dft_many_s* p)
{
    {
        std::lock_guard<std::mutex> g(g_mu);
        if (--p->refs > 0)
            return;
    }
    int cur = 0;
    const bool sw = hipGetDevice(&cur) == hipSuccess && cur != p->device;
    if (sw)
        (void)hipSetDevice(p->device);
    free_many(p);
    if (sw)
        (void)hipSetDevice(cur);
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src)
{
    *dst = nullptr;
    if (src.empty())
        return hipSuccess;
    hipError_t e = hipMalloc(dst, sizeof(T) * src.size());
    if (e == hipSuccess)
        e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
    return e;
}

// Planes of one direction: inputs and outputs, checked for NULL, alignment
// and partial overlap (an output may coincide exactly with an input of its
// own direction: every item reads its transforms before writing them).
split_dft_status check_dir(const split_dft_many_s* p, const float* ar, const float* ai, const float* br,
                           const float* bi, std::string* msg)
{
    if (!ar || !ai || !br || !bi) {
        *msg = "a data pointer is NULL";
        return SPLIT_DFT_ERR_NULL_POINTER;
    }
    for (const void* q : {static_cast<const void*>(ar), static_cast<const void*>(ai), static_cast<const void*>(br),
                          static_cast<const void*>(bi)})
        if (reinterpret_cast<uintptr_t>(q) % 16 != 0) {
            *msg = "data pointers must be 16-byte aligned";
            return SPLIT_DFT_ERR_MISALIGNED;
        }
    const size_t bytes = static_cast<size_t>(p->points) * sizeof(float);
    if (ranges_overlap(br, bytes, bi, bytes)) {
        *msg = "the two output planes overlap";
        return SPLIT_DFT_ERR_ALIASING;
    }
    for (const float* out : {br, bi})
        for (const float* in : {ar, ai})
            if (out != in && ranges_overlap(out, bytes, in, bytes)) {
                *msg = "an output partially overlaps an input";
                return SPLIT_DFT_ERR_ALIASING;
            }
    return SPLIT_DFT_OK;
}

// Validate a grouped call (plan, planes of each direction, cross-direction
// overlap, workspace); makes no HIP call.
split_dft_status many_validate(split_dft_many_t p, const float* xr, const float* xi, float* yr, float* yi,
                               const float* gr, const float* gi, float* gxr, float* gxi, bool fwd, bool adj,
                               const void* ws, size_t ws_bytes, std::string* msg)
{
    if (!p || !is_live(p)) {
        *msg = "grouped plan is NULL, destroyed or not created by split_dft_many_plan";
        return SPLIT_DFT_ERR_INVALID_PLAN;
    }
    const size_t bytes = static_cast<size_t>(p->points) * sizeof(float);
    split_dft_status st = SPLIT_DFT_OK;
    if (fwd && (st = check_dir(p, xr, xi, yr, yi, msg)) != SPLIT_DFT_OK)
        return st;
    if (adj && (st = check_dir(p, gr, gi, gxr, gxi, msg)) != SPLIT_DFT_OK)
        return st;
    if (fwd && adj) {
        // the two directions run concurrently: no output of one may touch the other's arrays
        for (const float* out : {yr, yi})
            for (const float* other : {gr, gi, static_cast<const float*>(gxr), static_cast<const float*>(gxi)})
                if (ranges_overlap(out, bytes, other, bytes)) {
                    *msg = "forward and adjoint arrays overlap";
                    return SPLIT_DFT_ERR_ALIASING;
                }
        for (const float* out : {gxr, gxi})
            for (const float* other : {xr, xi})
                if (ranges_overlap(out, bytes, other, bytes)) {
                    *msg = "forward and adjoint arrays overlap";
                    return SPLIT_DFT_ERR_ALIASING;
                }
    }
    if (p->ws_bytes > 0) {
        if (!ws && !p->d_ws) {
            *msg = "the grouped plan was created with SPLIT_DFT_CALLER_WORKSPACE: pass a workspace of "
                   "split_dft_many_workspace_bytes(plan) = " + std::to_string(p->ws_bytes) + " bytes";
            return SPLIT_DFT_ERR_NULL_POINTER;
        }
        if (ws) {
            if (ws_bytes < p->ws_bytes) {
                *msg = "workspace smaller than split_dft_many_workspace_bytes";
                return SPLIT_DFT_ERR_INVALID_BATCH;
            }
            if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) {
                *msg = "workspace must be 16-byte aligned";
                return SPLIT_DFT_ERR_MISALIGNED;
            }
            for (const void* q : {static_cast<const void*>(xr), static_cast<const void*>(xi),
                                  static_cast<const void*>(yr), static_cast<const void*>(yi),
                                  static_cast<const void*>(gr), static_cast<const void*>(gi),
                                  static_cast<const void*>(gxr), static_cast<const void*>(gxi)})
                if (q && ranges_overlap(ws, p->ws_bytes, q, bytes)) {
                    *msg = "workspace overlaps a data array";
                    return SPLIT_DFT_ERR_ALIASING;
                }
        }
    }
    return SPLIT_DFT_OK;
}

// Validate, then launch on `stream`.  ws: the caller's workspace, or NULL for
// the plan's own.
split_dft_status many_launch(split_dft_many_t p, const float* xr, const float* xi, float* yr, float* yi,
                             const float* gr, const float* gi, float* gxr, float* gxi, bool fwd, bool adj,
                             void* ws, size_t ws_bytes, hipStream_t stream, std::string* msg)
{
    split_dft_status st = many_validate(p, xr, xi, yr, yi, gr, gi, gxr, gxi, fwd, adj, ws, ws_bytes, msg);
    if (st != SPLIT_DFT_OK)
        return st;
    int cur = -1;  // the plan's tables and workspace live on the device it was created on
    if (hipGetDevice(&cur) != hipSuccess || cur != p->device) {
        *msg = "the grouped plan belongs to HIP device " + std::to_string(p->device) + ", the current device is " +
               std::to_string(cur);
        return SPLIT_DFT_ERR_INVALID_PLAN;
    }
    float* work = ws ? static_cast<float*>(ws) : p->d_ws;
    splitdft::ManyArgs a{};
    int d = 0;
    if (fwd) {
        a.in_r[d] = xr, a.in_i[d] = xi, a.out_r[d] = yr, a.out_i[d] = yi;
        ++d;
    }
    if (adj) {
        // C g_r - S g_i and S g_r + C g_i: the forward scheme on (g_i, g_r), outputs exchanged
        a.in_r[d] = gi, a.in_i[d] = gr, a.out_r[d] = gxi, a.out_i[d] = gxr;
        ++d;
    }
    // lengths >= 2^14 (default mode): per-length kernels, one direction at a time
    for (const ManyLarge& g : p->large) {
        for (int k = 0; k < d; ++k) {
            hipError_t e = hipSuccess;
            if (g.variant) {
                e = g.variant->launch(a.in_r[k], a.in_i[k], a.out_r[k], a.out_i[k], p->d_tw, g.count, g.d_rows,
                                      stream, nullptr);
            } else {
                float* wr = work;
                float* wi = work + g.chunk * (int64_t{1} << g.m);
                for (int64_t s0 = 0; s0 < g.count && e == hipSuccess; s0 += g.chunk) {
                    const int64_t c = g.count - s0 < g.chunk ? g.count - s0 : g.chunk;
                    e = g.two->pass1(a.in_r[k], a.in_i[k], wr, wi, p->d_tw, c, g.d_rows + s0, stream);
                    if (e == hipSuccess)
                        e = g.two->pass2(wr, wi, a.out_r[k], a.out_i[k], p->d_tw, c, g.d_rows + s0, stream);
                }
            }
            if (e != hipSuccess) {
                *msg = std::string("per-length kernel launch: ") + hipGetErrorString(e);
                return SPLIT_DFT_ERR_HIP;
            }
        }
    }
    if ((d == 2 ? p->n_both : p->n_one) == 0)
        return SPLIT_DFT_OK;
    a.offsets = p->d_offsets;
    a.items = d == 2 ? p->d_items_both : p->d_items_one;
    a.nitems = d == 2 ? p->n_both : p->n_one;
    a.queue = p->d_queue;
    a.ws = work;
    a.tw = p->d_tw;
    const hipError_t e = splitdft::launch_many(p->variant, p->large_items, a, p->grid, stream);
    if (e != hipSuccess) {
        *msg = std::string("grouped kernel launch: ") + hipGetErrorString(e);
        return SPLIT_DFT_ERR_HIP;
    }
    return SPLIT_DFT_OK;
}

split_dft_status fail(split_dft_status st, const std::string& msg)
{
    splitdft::set_last_error(msg);
    return st;
}

}  // namespace

extern "C" {

split_dft_status split_dft_many_plan(split_dft_many_t* out, const int64_t* lengths, int64_t count, uint32_t flags)
{
    using namespace splitdft;
    if (!out || !lengths)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "out or lengths is NULL");
    if (count < 1 || count > INT32_MAX)
        return fail(SPLIT_DFT_ERR_INVALID_BATCH, "count must be in [1, 2^31 - 1]");
    const bool caller_ws = (flags & SPLIT_DFT_CALLER_WORKSPACE) != 0;
    if ((flags & 0xffu) != SPLIT_DFT_FP32 || ((flags & ~SPLIT_DFT_CALLER_WORKSPACE) >> 30) != 0)
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "unsupported flags " + std::to_string(flags));
    const bool one_kernel = (flags & SPLIT_DFT_MANY_ONE_KERNEL) != 0;
    // bits 25-29: log2 of the shortest length run by per-length launches
    const int split_sel = static_cast<int>((flags >> 25) & 0x1fu);
    if (split_sel != 0 && (split_sel < kManyPerLengthMinLog2N || split_sel > kManyMaxLog2N + 1))
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "per-length threshold must be 2^" +
                                                   std::to_string(kManyPerLengthMinLog2N) + " .. 2^" +
                                                   std::to_string(kManyMaxLog2N + 1));
    const int per_length_from = split_sel == 0 ? kManyPerLengthLog2N : split_sel;
    const int variant_sel = static_cast<int>((flags >> 8) & 0xffu);  // 0 = default build, k = build k-1
    const int wg_per_cu = static_cast<int>((flags >> 16) & 0xffu);   // 0 = as many as fit
    if (variant_sel > kManyKernelVariants)
        return fail(SPLIT_DFT_ERR_UNSUPPORTED, "unknown grouped kernel build");

    std::vector<int64_t> offs(static_cast<size_t>(count) + 1, 0);
    std::vector<int> logs(static_cast<size_t>(count));
    bool any_large = false;
    for (int64_t k = 0; k < count; ++k) {
        const int64_t n = lengths[k];
        int m = 0;
        while (m < 62 && (int64_t{1} << m) < n)
            ++m;
        if (n < 1 || (int64_t{1} << m) != n || m < kManyMinLog2N || m > kManyMaxLog2N)
            return fail(SPLIT_DFT_ERR_INVALID_LENGTH,
                        "length " + std::to_string(k) + " = " + std::to_string(n) + " is not 2^m, 2 <= m <= 16");
        logs[static_cast<size_t>(k)] = m;
        // lengths >= 2^14 that stay in the persistent kernel need its large build
        any_large = any_large || (m > 13 && (one_kernel || m < per_length_from));
        if (offs[static_cast<size_t>(k)] > INT64_MAX / 8 - n)
            return fail(SPLIT_DFT_ERR_INVALID_BATCH, "total length overflows");
        offs[static_cast<size_t>(k) + 1] = offs[static_cast<size_t>(k)] + n;
    }

    // transforms grouped by length, longest first; items listed longest first
    std::vector<int32_t> order(static_cast<size_t>(count));
    for (int64_t k = 0; k < count; ++k)
        order[static_cast<size_t>(k)] = static_cast<int32_t>(k);
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return logs[static_cast<size_t>(a)] > logs[static_cast<size_t>(b)]; });
    std::vector<ManyItem> one, both;
    struct LargeHost {
        int m;
        std::vector<int64_t> rows;
    };
    std::vector<LargeHost> large_host;
    for (size_t i = 0; i < order.size();) {
        const int m = logs[static_cast<size_t>(order[i])];
        size_t j = i;
        while (j < order.size() && logs[static_cast<size_t>(order[j])] == m)
            ++j;
        if (!one_kernel && m >= per_length_from) {
            LargeHost g{m, {}};
            for (size_t s = i; s < j; ++s)
                g.rows.push_back(offs[static_cast<size_t>(order[s])]);
            large_host.push_back(std::move(g));
            i = j;
            continue;
        }
        const size_t per = static_cast<size_t>(many_items_per_group(m));
        for (size_t s = i; s < j; s += per) {
            const int cnt = static_cast<int>(std::min(per, j - s));
            const ManyItem it{m, 0, cnt, 0, static_cast<int64_t>(s)};
            one.push_back(it);
            both.push_back(it);
            ManyItem it2 = it;
            it2.dir = 1;
            both.push_back(it2);
        }
        i = j;
    }

    const char* inj = std::getenv("SPLIT_DFT_FAIL_ALLOC");
    if (inj && *inj && std::strcmp(inj, "0") != 0)
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "allocation failure forced by SPLIT_DFT_FAIL_ALLOC");

    auto* p = new (std::nothrow) split_dft_many_s{};
    if (!p)
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "host allocation of the plan failed");
    p->count = count;
    p->points = offs.back();
    p->offsets = offs;
    p->one_kernel = one_kernel;
    p->large_items = any_large;
    p->variant = variant_sel == 0 ? 0 : variant_sel - 1;
    hipError_t e = hipGetDevice(&p->device);
    int cus = 0, per_cu = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device);
    if (e == hipSuccess)
        e = many_max_active_per_cu(p->variant, any_large, &per_cu);
    if (e != hipSuccess) {
        free_many(p);
        return fail(SPLIT_DFT_ERR_HIP, std::string("device query: ") + hipGetErrorString(e));
    }
    if (wg_per_cu > 0 && wg_per_cu < per_cu)
        per_cu = wg_per_cu;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t items = static_cast<int64_t>(both.size());
    p->grid = static_cast<int>(std::min<int64_t>(static_cast<int64_t>(cus) * per_cu, std::max<int64_t>(items, 1)));

    std::vector<float> c(static_cast<size_t>(kManyMaxN)), s(static_cast<size_t>(kManyMaxN));
    build_twiddles_f32(kManyMaxLog2N, c.data(), s.data());
    std::vector<float2> tw(static_cast<size_t>(kManyMaxN));
    for (size_t j = 0; j < tw.size(); ++j)
        tw[j] = make_float2(c[j], s[j]);
    std::vector<int> queue_init(2, 0);
    // the kernel reads each item's offsets in length order: one load, no
    // indirection through the sort
    std::vector<int64_t> offs_dev(order.size());
    for (size_t i = 0; i < order.size(); ++i)
        offs_dev[i] = offs[static_cast<size_t>(order[i])];
    e = upload(&p->d_offsets, offs_dev);
    if (e == hipSuccess)
        e = upload(&p->d_items_one, one);
    if (e == hipSuccess)
        e = upload(&p->d_items_both, both);
    if (e == hipSuccess)
        e = upload(&p->d_queue, queue_init);
    if (e == hipSuccess)
        e = upload(&p->d_tw, tw);
    // one workspace serves both users, which run one after the other on the
    // stream: the persistent kernel's per-workgroup regions (lengths >= 2^14
    // in it) and the per-length two-pass chunks
    size_t ws1 = any_large ? static_cast<size_t>(p->grid) * 2 * static_cast<size_t>(kManyMaxN) * sizeof(float) : 0;
    size_t ws2 = 0;
    for (LargeHost& h : large_host) {
        if (e != hipSuccess)
            break;
        ManyLarge g{h.m, static_cast<int64_t>(h.rows.size()), nullptr, nullptr, nullptr, 0};
        // the length's default schedule if it takes per-transform offsets,
        // else the first one that does
        const Variant* v = default_variant(h.m, g.count);
        if (v && !v->rows_ok) {
            int nv = 0;
            const Variant* list = variants_for(h.m, &nv);
            v = nullptr;
            for (int k = 0; k < nv && !v; ++k)
                if (list[k].rows_ok)
                    v = &list[k];
        }
        int c2 = 0;
        const TwoPass* two = two_pass_for(h.m, &c2);
        if (h.m < kManyTwoPassLog2N && v) {
            g.variant = v;
        } else if (two && c2 > 0) {
            g.two = &two[0];
            const int64_t n = int64_t{1} << h.m;
            int64_t chunk_bytes = kManyChunkBytes;
            if (const char* cb = std::getenv("SPLIT_DFT_CHUNK_MIB"))  // tuning override, 1 MiB .. 64 GiB
                if (std::atoll(cb) > 0)
                    chunk_bytes = std::min<int64_t>(std::atoll(cb), int64_t{1} << 16) << 20;
            g.chunk = std::max<int64_t>(1, std::min<int64_t>(g.count, chunk_bytes / (n * 2 * 4)));
            const int64_t nchunks = (g.count + g.chunk - 1) / g.chunk;
            g.chunk = (g.count + nchunks - 1) / nchunks;  // equal chunks
            ws2 = std::max(ws2, static_cast<size_t>(g.chunk) * static_cast<size_t>(n) * 2 * sizeof(float));
        } else {
            e = hipErrorInvalidConfiguration;
            break;
        }
        e = upload(&g.d_rows, h.rows);
        p->large.push_back(g);
    }
    if (e == hipSuccess && std::max(ws1, ws2) > 0) {
        p->ws_bytes = std::max(ws1, ws2);
        if (!caller_ws)
            e = hipMalloc(&p->d_ws, p->ws_bytes);
    }
    if (e != hipSuccess) {
        free_many(p);
        return e == hipErrorOutOfMemory ? fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "device allocation for the grouped plan")
                                        : fail(SPLIT_DFT_ERR_HIP, std::string("grouped plan: ") + hipGetErrorString(e));
    }
    p->n_one = static_cast<int>(one.size());
    p->n_both = static_cast<int>(both.size());
    p->refs = 1;
    set_live(p, true);
    *out = p;
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_many_offsets(split_dft_many_t plan, int64_t* offsets)
{
    if (!plan || !is_live(plan))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "grouped plan is NULL or destroyed");
    if (!offsets)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "offsets is NULL");
    std::memcpy(offsets, plan->offsets.data(), sizeof(int64_t) * plan->offsets.size());
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_many_info(split_dft_many_t plan, int64_t* count, int64_t* points, int* workgroups,
                                     int* items, size_t* workspace_bytes)
{
    if (!plan || !is_live(plan))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "grouped plan is NULL or destroyed");
    if (count)
        *count = plan->count;
    if (points)
        *points = plan->points;
    if (workgroups)
        *workgroups = plan->grid;
    if (items)
        *items = plan->n_both;
    if (workspace_bytes)
        *workspace_bytes = plan->ws_bytes;
    return SPLIT_DFT_OK;
}

size_t split_dft_many_workspace_bytes(split_dft_many_t plan)
{
    if (!plan || !is_live(plan))
        return 0;
    return plan->ws_bytes;
}

split_dft_status split_dft_many_exec(split_dft_many_t plan, const float* xr, const float* xi, float* yr, float* yi,
                                     void* stream)
{
    return split_dft_many_exec_ws(plan, xr, xi, yr, yi, nullptr, 0, stream);
}

split_dft_status split_dft_many_exec_ws(split_dft_many_t plan, const float* xr, const float* xi, float* yr,
                                        float* yi, void* workspace, size_t workspace_bytes, void* stream)
{
    std::string msg;
    const split_dft_status st = many_launch(plan, xr, xi, yr, yi, nullptr, nullptr, nullptr, nullptr, true, false,
                                            workspace, workspace_bytes, static_cast<hipStream_t>(stream), &msg);
    return st == SPLIT_DFT_OK ? st : fail(st, msg);
}

split_dft_status split_dft_many_adjoint(split_dft_many_t plan, const float* gr, const float* gi, float* gxr,
                                        float* gxi, void* stream)
{
    return split_dft_many_adjoint_ws(plan, gr, gi, gxr, gxi, nullptr, 0, stream);
}

split_dft_status split_dft_many_adjoint_ws(split_dft_many_t plan, const float* gr, const float* gi, float* gxr,
                                           float* gxi, void* workspace, size_t workspace_bytes, void* stream)
{
    std::string msg;
    const split_dft_status st = many_launch(plan, nullptr, nullptr, nullptr, nullptr, gr, gi, gxr, gxi, false, true,
                                            workspace, workspace_bytes, static_cast<hipStream_t>(stream), &msg);
    return st == SPLIT_DFT_OK ? st : fail(st, msg);
}

split_dft_status split_dft_many_exec_adjoint(split_dft_many_t plan, const float* xr, const float* xi, float* yr,
                                             float* yi, const float* gr, const float* gi, float* gxr, float* gxi,
                                             void* stream)
{
    return split_dft_many_exec_adjoint_ws(plan, xr, xi, yr, yi, gr, gi, gxr, gxi, nullptr, 0, stream);
}

split_dft_status split_dft_many_exec_adjoint_ws(split_dft_many_t plan, const float* xr, const float* xi, float* yr,
                                                float* yi, const float* gr, const float* gi, float* gxr, float* gxi,
                                                void* workspace, size_t workspace_bytes, void* stream)
{
    std::string msg;
    const split_dft_status st = many_launch(plan, xr, xi, yr, yi, gr, gi, gxr, gxi, true, true, workspace,
                                            workspace_bytes, static_cast<hipStream_t>(stream), &msg);
    return st == SPLIT_DFT_OK ? st : fail(st, msg);
}

split_dft_status split_dft_many_graph(split_dft_many_t plan, const float* xr, const float* xi, float* yr, float* yi,
                                      const float* gr, const float* gi, float* gxr, float* gxi,
                                      split_dft_graph_t* out)
{
    return split_dft_many_graph_ws(plan, xr, xi, yr, yi, gr, gi, gxr, gxi, nullptr, 0, out);
}

split_dft_status split_dft_many_graph_ws(split_dft_many_t plan, const float* xr, const float* xi, float* yr,
                                         float* yi, const float* gr, const float* gi, float* gxr, float* gxi,
                                         void* workspace, size_t workspace_bytes, split_dft_graph_t* out)
{
    if (!out)
        return fail(SPLIT_DFT_ERR_NULL_POINTER, "out is NULL");
    const bool adj = gr || gi || gxr || gxi;
    // validate before touching the runtime
    {
        std::string msg;
        const split_dft_status st = many_validate(plan, xr, xi, yr, yi, gr, gi, gxr, gxi, true, adj, workspace,
                                                  workspace_bytes, &msg);
        if (st != SPLIT_DFT_OK)
            return fail(st, msg);
    }
    auto* g = new (std::nothrow) split_dft_graph_s{nullptr, nullptr, plan};
    if (!g)
        return fail(SPLIT_DFT_ERR_OUT_OF_MEMORY, "host allocation of the graph");
    hipStream_t s = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete g;
        return fail(SPLIT_DFT_ERR_HIP, std::string("hipStreamCreate: ") + hipGetErrorString(e));
    }
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    std::string msg;
    split_dft_status st = SPLIT_DFT_OK;
    if (e == hipSuccess) {
        st = many_launch(plan, xr, xi, yr, yi, gr, gi, gxr, gxi, true, adj, workspace, workspace_bytes, s, &msg);
        const hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (st == SPLIT_DFT_OK && e2 != hipSuccess)
            e = e2;
    }
    (void)hipStreamDestroy(s);
    if (st != SPLIT_DFT_OK) {
        if (graph)
            (void)hipGraphDestroy(graph);
        delete g;
        return fail(st, msg);
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess)
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        delete g;
        return fail(SPLIT_DFT_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    }
    g->graph = graph;
    g->exec = exec;
    {
        // the graph's kernels use the plan's device data: hold a reference
        // (a plan destroyed meanwhile would be gone from the live set)
        std::lock_guard<std::mutex> lk(g_mu);
        if (live().count(plan) == 0) {
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            delete g;
            return fail(SPLIT_DFT_ERR_INVALID_PLAN, "grouped plan destroyed during graph capture");
        }
        ++plan->refs;
        live().insert(g);
    }
    *out = g;
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_graph_launch(split_dft_graph_t graph, void* stream)
{
    if (!graph || !is_live(graph))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "graph is NULL or destroyed");
    const hipError_t e = hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(SPLIT_DFT_ERR_HIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    return SPLIT_DFT_OK;
}

split_dft_status split_dft_graph_destroy(split_dft_graph_t graph)
{
    if (!graph)
        return SPLIT_DFT_OK;
    if (!take_live(graph))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "graph is destroyed");
    hipError_t e = hipGraphExecDestroy(graph->exec);
    const hipError_t e2 = hipGraphDestroy(graph->graph);
    split_dft_many_s* plan = graph->plan;
    delete graph;
    release_many(plan);
    if (e == hipSuccess)
        e = e2;
    return e == hipSuccess ? SPLIT_DFT_OK : fail(SPLIT_DFT_ERR_HIP, hipGetErrorString(e));
}

split_dft_status split_dft_many_destroy(split_dft_many_t plan)
{
    if (!plan)
        return SPLIT_DFT_OK;
    if (!take_live(plan))
        return fail(SPLIT_DFT_ERR_INVALID_PLAN, "grouped plan is destroyed");
    release_many(plan);
    return SPLIT_DFT_OK;
}

}  // extern "C"
