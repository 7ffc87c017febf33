// flic_api.cpp -- C ABI of the FLIC clustering library: argument checks,
// contexts (descriptor + scratch ring), batch layout, plans (hipGraph),
// pass timing and error reporting.
#include "../../include/flic.h"

#include <hip/hip_runtime.h>

#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "flic_internal.h"

using flic::ScanDesc;

static_assert(FLIC_NOALLOC_SCRATCH_BYTES == flic::kNoAllocScratchBytes, "header and library agree");

namespace {

thread_local std::string g_last_error;

flic_status fail(flic_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
flic_status fail(flic_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                              \
    do {                                                                           \
        hipError_t e_ = (expr);                                                    \
        if (e_ != hipSuccess)                                                      \
            return fail(FLIC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const char* a0 = static_cast<const char*>(a);
    const char* b0 = static_cast<const char*>(b);
    return a0 < b0 + nb && b0 < a0 + na;
}

// Host-side check of one scan's arguments; nothing touches the device.
flic_status check_scan(const float* range, int32_t H, int32_t W, const flic_alpha_tables* t,
                       float threshold, int32_t N, const int32_t* labels, int idx) {
    if (!range || !labels || !t || !t->cos_v || !t->cos_h)
        return fail(FLIC_EINVAL, "scan %d: null pointer", idx);
    if (H < 1 || W < 1) return fail(FLIC_EINVAL, "scan %d: H=%d W=%d", idx, H, W);
    if (N < 1 || N > FLIC_MAX_SKIP)
        return fail(FLIC_EINVAL, "scan %d: skip_depth %d outside 1..%d", idx, N, FLIC_MAX_SKIP);
    if (2 * N >= W) return fail(FLIC_EINVAL, "scan %d: need 2*skip_depth < W (N=%d W=%d)", idx, N, W);
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX)
        return fail(FLIC_EINVAL, "scan %d: H*W exceeds INT32_MAX", idx);
    if (!(threshold >= 0.0f) || !std::isfinite(threshold))
        return fail(FLIC_EINVAL, "scan %d: threshold must be finite and >= 0", idx);
    const size_t px = (size_t)H * (size_t)W;
    if (overlaps(range, px * 4, labels, px * 4))
        return fail(FLIC_EINVAL, "scan %d: range_img and labels_out overlap", idx);
    if (overlaps(t->cos_v, (size_t)N * H * 4, labels, px * 4) ||
        overlaps(t->cos_h, (size_t)N * W * 4, labels, px * 4))
        return fail(FLIC_EINVAL, "scan %d: a table overlaps labels_out", idx);
    return FLIC_OK;
}

flic_status check_scans(const flic_scan* scans, int32_t n) {
    if (n < 0) return fail(FLIC_EINVAL, "n < 0");
    if (n > 0 && !scans) return fail(FLIC_EINVAL, "scans is null");
    for (int32_t i = 0; i < n; ++i) {
        const flic_scan& s = scans[i];
        flic_status st = check_scan(s.range_img, s.H, s.W, &s.tables, s.threshold, s.skip_depth,
                                    s.labels_out, i);
        if (st != FLIC_OK) return st;
        if (s.min_points < 0) return fail(FLIC_EINVAL, "scan %d: min_points %d < 0", i, s.min_points);
        if (s.map_connections != 0 && s.map_connections != 1)
            return fail(FLIC_EINVAL, "scan %d: map_connections %d not 0 or 1", i, s.map_connections);
    }
    // no scan may write into another scan's buffers
    for (int32_t i = 0; i < n; ++i) {
        const size_t pi = (size_t)scans[i].H * scans[i].W * 4;
        for (int32_t j = 0; j < n; ++j) {
            if (i == j) continue;
            const size_t pj = (size_t)scans[j].H * scans[j].W * 4;
            if (overlaps(scans[i].labels_out, pi, scans[j].labels_out, pj) ||
                overlaps(scans[i].labels_out, pi, scans[j].range_img, pj))
                return fail(FLIC_EINVAL, "scan %d labels_out overlaps scan %d buffers", i, j);
        }
    }
    return FLIC_OK;
}

hipError_t launch_cluster(const flic::BatchRef& ref, int tile_w, int skip, bool sized, bool maps,
                          int n_tiles, int n_scans, hipStream_t stream, hipEvent_t* events = nullptr) {
    if (n_tiles <= 0 || n_scans <= 0) return hipSuccess;
    switch (tile_w * 2 + (maps ? 1 : 0)) {
        case 128: return flic::launch_cluster_tw<64, false>(ref, skip, sized, n_tiles, n_scans, stream, events);
        case 129: return flic::launch_cluster_tw<64, true>(ref, skip, sized, n_tiles, n_scans, stream, events);
        case 256: return flic::launch_cluster_tw<128, false>(ref, skip, sized, n_tiles, n_scans, stream, events);
        case 257: return flic::launch_cluster_tw<128, true>(ref, skip, sized, n_tiles, n_scans, stream, events);
        case 512: return flic::launch_cluster_tw<256, false>(ref, skip, sized, n_tiles, n_scans, stream, events);
        case 513: return flic::launch_cluster_tw<256, true>(ref, skip, sized, n_tiles, n_scans, stream, events);
        default: return hipErrorInvalidValue;
    }
}

// The kernels of one launch group (count in *n_out), for graph nodes.
hipError_t cluster_passes(int tile_w, int skip, bool sized, bool maps, int n_tiles, flic::PassLaunch* out,
                          int* n_out) {
    *n_out = 0;
    if (n_tiles <= 0) return hipErrorInvalidValue;
    switch (tile_w * 2 + (maps ? 1 : 0)) {
        case 128: *n_out = flic::cluster_passes_tw<64, false>(skip, sized, n_tiles, out); break;
        case 129: *n_out = flic::cluster_passes_tw<64, true>(skip, sized, n_tiles, out); break;
        case 256: *n_out = flic::cluster_passes_tw<128, false>(skip, sized, n_tiles, out); break;
        case 257: *n_out = flic::cluster_passes_tw<128, true>(skip, sized, n_tiles, out); break;
        case 512: *n_out = flic::cluster_passes_tw<256, false>(skip, sized, n_tiles, out); break;
        case 513: *n_out = flic::cluster_passes_tw<256, true>(skip, sized, n_tiles, out); break;
        default: break;
    }
    return *n_out > 0 ? hipSuccess : hipErrorInvalidValue;
}

hipError_t set_device(int dev) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    return cur == dev ? hipSuccess : hipSetDevice(dev);
}

}  // namespace

// ---------------------------------------------------------------------------
// Context: a ring of launch slots.  Each slot owns a pinned + device copy of a
// batch's descriptor blob and a device scratch buffer; a slot is reused only
// after the event recorded behind its last launch has completed, so launches
// in flight on any streams never share scratch.
// ---------------------------------------------------------------------------

struct flic_ctx {
    int device = 0;
    size_t budget = 0;          // 0 = unlimited
    size_t used = 0;            // device bytes held by this context and its plans
    int tile_override = 0;
    int plan_parts = 1;         // launch sequences per shape group in a plan
    struct TileRule { int32_t H, W, N, tile_w; };
    std::vector<TileRule> rules;   // exact-shape tile widths (autotuner output)
    static constexpr int kRing = 4;
    struct Slot {
        void* host = nullptr;   // pinned descriptor staging
        void* dev = nullptr;    // device descriptors
        size_t cap = 0;
        void* scratch = nullptr;
        size_t scratch_cap = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    } ring[kRing];
    int next = 0;
    bool timing = false;
    std::vector<std::array<hipEvent_t, flic::kPasses + 1>> timed;   // recorded, not yet read
    std::vector<std::array<hipEvent_t, flic::kPasses + 1>> spare;   // recycled
};

struct flic_plan {
    flic_ctx* ctx = nullptr;
    int32_t n = 0;
    std::vector<flic_scan> shapes;     // shapes as planned
    struct Group {                     // scans sharing tile width, skip depth, sizing and skip-edge mode
        int tile_w;
        int skip;
        bool sized;
        bool maps;
        int n_tiles;
        size_t desc_off;               // byte offset of ScanDesc[members] in the blob
        std::vector<int> members;      // scan indices
    };
    std::vector<Group> groups;
    size_t blob_bytes = 0;
    char* host_blob = nullptr;         // pinned copy of the device descriptor blob
    void* dev_mem = nullptr;           // descriptors
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool launched = false;
};

namespace {

int choose_tile_w(const flic_ctx* ctx, int32_t H, int32_t W, int32_t N) {
    if (ctx && ctx->tile_override > 0) return ctx->tile_override;
    if (ctx)
        for (const auto& r : ctx->rules)
            if (r.H == H && r.W == W && r.N == N) return r.tile_w;
    // One tile row whenever the scan fits: 128 rows x 64 columns, 64 x 128
    // or 32 x 256 (every tile holds kTilePx pixels).
    if (H <= 32 && W >= 256) return 256;
    if (H <= 64 && W >= 128) return 128;
    return 64;
}

bool sized(const flic_scan& s) { return s.min_points > 0; }
// Map Connections matter only with skip edges (N >= 2).
bool maps(const flic_scan& s) { return s.map_connections != 0 && s.skip_depth >= 2; }

ScanDesc make_desc(const flic_scan& s, int tile_w, int32_t tile_begin, char* scratch) {
    ScanDesc d{};
    d.range = s.range_img;
    d.labels = s.labels_out;
    d.cos_v = s.tables.cos_v;
    d.cos_h = s.tables.cos_h;
    d.H = s.H;
    d.W = s.W;
    d.N = s.skip_depth;
    d.t2 = s.threshold * s.threshold;      // binary32 product, as in Eq. (4)
    d.tile_w = tile_w;
    d.tile_h = flic::tile_h_for(tile_w);
    d.tiles_x = (s.W + tile_w - 1) / tile_w;
    d.tiles_y = (s.H + d.tile_h - 1) / d.tile_h;
    d.chunks_per_row = (s.W + 63) / 64;
    d.tile_begin = tile_begin;
    d.min_points = s.min_points;
    const flic::ScratchLayout S = flic::scratch_layout(s.H, s.W, s.skip_depth, tile_w, sized(s));
    d.masks = reinterpret_cast<ulonglong2*>(scratch + S.masks);
    d.runs = reinterpret_cast<uint16_t*>(scratch + S.runs);
    d.parent = reinterpret_cast<int32_t*>(scratch + S.parent);
    d.counts = sized(s) ? reinterpret_cast<int32_t*>(scratch + S.counts) : nullptr;
    d.bcol_v = reinterpret_cast<float*>(scratch + S.bcol_v);
    d.bcol_r = reinterpret_cast<int32_t*>(scratch + S.bcol_r);
    d.brow_v = reinterpret_cast<float*>(scratch + S.brow_v);
    d.brow_r = reinterpret_cast<int32_t*>(scratch + S.brow_r);
    return d;
}

size_t scratch_bytes(const flic_ctx* ctx, const flic_scan* scans, int32_t n) {
    size_t total = 0;
    for (int32_t i = 0; i < n; ++i)
        total += flic::scratch_layout(scans[i].H, scans[i].W, scans[i].skip_depth,
                                      choose_tile_w(ctx, scans[i].H, scans[i].W, scans[i].skip_depth),
                                      sized(scans[i])).total;
    return total;
}

// Descriptors + block maps for a batch, grouped by (tile width, skip depth,
// size threshold or not),
// as one byte image: per group ScanDesc[members] then int32 block_scan[tiles].
// Scans take consecutive scratch regions starting at `scratch`.
struct Layout {
    std::vector<char> blob;
    struct G {
        int tile_w, skip;
        bool sized, maps;
        int n_tiles;
        size_t desc_off, map_off;
        std::vector<int> members;
    };
    std::vector<G> groups;
};

// parts > 1 splits every group into up to `parts` launch sequences over
// consecutive member ranges (plans make them parallel graph branches).
void build_layout(const flic_ctx* ctx, const flic_scan* scans, int32_t n, char* scratch, Layout& L,
                  int parts = 1) {
    L.blob.clear();
    L.groups.clear();
    std::vector<char*> base(n);
    size_t off = 0;
    for (int32_t i = 0; i < n; ++i) {
        base[i] = scratch + off;
        off += flic::scratch_layout(scans[i].H, scans[i].W, scans[i].skip_depth,
                                    choose_tile_w(ctx, scans[i].H, scans[i].W, scans[i].skip_depth),
                                    sized(scans[i])).total;
    }
    const int widths[3] = {64, 128, 256};
    constexpr int kShapes = 3 * FLIC_MAX_SKIP;
    for (int gi = 0; gi < 4 * kShapes; ++gi) {
        const int gw = gi % kShapes, mode = gi / kShapes;
        Layout::G all{widths[gw / FLIC_MAX_SKIP], 1 + gw % FLIC_MAX_SKIP, (mode & 1) != 0, (mode & 2) != 0,
                      0, 0, 0, {}};
        for (int32_t i = 0; i < n; ++i)
            if (choose_tile_w(ctx, scans[i].H, scans[i].W, scans[i].skip_depth) == all.tile_w &&
                scans[i].skip_depth == all.skip && sized(scans[i]) == all.sized && maps(scans[i]) == all.maps)
                all.members.push_back(i);
        if (all.members.empty()) continue;
        const size_t np = std::min<size_t>(std::max(parts, 1), all.members.size());
        for (size_t part = 0; part < np; ++part) {
            Layout::G g = all;
            g.members.assign(all.members.begin() + all.members.size() * part / np,
                             all.members.begin() + all.members.size() * (part + 1) / np);
            std::vector<ScanDesc> descs;
            std::vector<int32_t> map;
            int32_t tiles = 0;
            for (size_t m = 0; m < g.members.size(); ++m) {
                const int i = g.members[m];
                ScanDesc d = make_desc(scans[i], g.tile_w, tiles, base[i]);
                const int32_t t = d.tiles_x * d.tiles_y;
                for (int32_t k = 0; k < t; ++k) map.push_back((int32_t)m);
                tiles += t;
                descs.push_back(d);
            }
            g.n_tiles = tiles;
            auto align = [&](size_t a) { L.blob.resize((L.blob.size() + a - 1) / a * a); };
            align(256);
            g.desc_off = L.blob.size();
            L.blob.resize(L.blob.size() + descs.size() * sizeof(ScanDesc));
            memcpy(L.blob.data() + g.desc_off, descs.data(), descs.size() * sizeof(ScanDesc));
            align(256);
            g.map_off = L.blob.size();
            L.blob.resize(L.blob.size() + map.size() * sizeof(int32_t));
            memcpy(L.blob.data() + g.map_off, map.data(), map.size() * sizeof(int32_t));
            L.groups.push_back(std::move(g));
        }
    }
}

// Events for one timed launch (null when timing is off).
hipEvent_t* timing_events(flic_ctx* ctx, hipError_t* err) {
    *err = hipSuccess;
    if (!ctx || !ctx->timing) return nullptr;
    std::array<hipEvent_t, flic::kPasses + 1> ev{};
    if (!ctx->spare.empty()) {
        ev = ctx->spare.back();
        ctx->spare.pop_back();
    } else {
        for (auto& e : ev)
            if ((*err = hipEventCreate(&e)) != hipSuccess) return nullptr;
    }
    ctx->timed.push_back(ev);
    return ctx->timed.back().data();
}

flic_status enqueue_layout(const Layout& L, const char* dev_base, hipStream_t stream,
                           flic_ctx* timing_ctx) {
    for (const auto& g : L.groups) {
        flic::BatchRef ref{};
        ref.descs = reinterpret_cast<const ScanDesc*>(dev_base + g.desc_off);
        ref.block_scan = reinterpret_cast<const int32_t*>(dev_base + g.map_off);
        hipError_t e;
        hipEvent_t* ev = timing_events(timing_ctx, &e);
        HIP_TRY(e);
        HIP_TRY(launch_cluster(ref, g.tile_w, g.skip, g.sized, g.maps, g.n_tiles, (int)g.members.size(),
                               stream, ev));
    }
    return FLIC_OK;
}

// The plan's graph: per group (a shape group, or a part of one) a chain of
// its pass kernels; the chains share no edge, so the groups' passes overlap
// one another.  Built node by node (no stream capture, no extra streams).
hipError_t build_plan_graph(const Layout& L, const char* dev_base, hipGraph_t* graph) {
    hipError_t e = hipGraphCreate(graph, 0);
    if (e != hipSuccess) return e;
    for (const auto& g : L.groups) {
        flic::BatchRef ref{};
        ref.descs = reinterpret_cast<const ScanDesc*>(dev_base + g.desc_off);
        ref.block_scan = reinterpret_cast<const int32_t*>(dev_base + g.map_off);
        flic::PassLaunch pass[flic::kMaxPassKernels];
        int n_pass = 0;
        e = cluster_passes(g.tile_w, g.skip, g.sized, g.maps, g.n_tiles, pass, &n_pass);
        if (e != hipSuccess) return e;
        hipGraphNode_t prev = nullptr;
        for (int k = 0; k < n_pass; ++k) {
            void* args[] = {&ref};                   // copied into the node
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(pass[k].fn);
            kp.gridDim = dim3(pass[k].grid);
            kp.blockDim = dim3(pass[k].block);
            kp.sharedMemBytes = 0;
            kp.kernelParams = args;
            kp.extra = nullptr;
            hipGraphNode_t node;
            e = hipGraphAddKernelNode(&node, *graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
            if (e != hipSuccess) return e;
            prev = node;
        }
    }
    return hipSuccess;
}

size_t round_cap(size_t need) {
    size_t cap = 4096;
    while (cap < need) cap *= 2;
    return cap;
}

// Next ring slot with at least `desc_bytes` of descriptors and
// `scratch_need` of scratch, after its previous launch has finished.
flic_status acquire_slot(flic_ctx* ctx, size_t desc_bytes, size_t scratch_need, flic_ctx::Slot** out) {
    flic_ctx::Slot& slot = ctx->ring[ctx->next];
    ctx->next = (ctx->next + 1) % flic_ctx::kRing;
    if (slot.pending) {
        HIP_TRY(hipEventSynchronize(slot.done));
        slot.pending = false;
    }
    if (!slot.done) HIP_TRY(hipEventCreateWithFlags(&slot.done, hipEventDisableTiming));
    if (desc_bytes > slot.cap) {
        const size_t cap = round_cap(desc_bytes);
        if (ctx->budget && ctx->used - slot.cap + cap > ctx->budget)
            return fail(FLIC_ENOMEM, "descriptor buffer of %zu bytes exceeds the HBM budget", cap);
        if (slot.dev) HIP_TRY(hipFree(slot.dev));
        if (slot.host) HIP_TRY(hipHostFree(slot.host));
        ctx->used -= slot.cap;
        slot.dev = slot.host = nullptr;
        slot.cap = 0;
        if (hipMalloc(&slot.dev, cap) != hipSuccess) return fail(FLIC_ENOMEM, "hipMalloc(%zu) failed", cap);
        if (hipHostMalloc(&slot.host, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(slot.dev);
            slot.dev = nullptr;
            return fail(FLIC_ENOMEM, "hipHostMalloc(%zu) failed", cap);
        }
        slot.cap = cap;
        ctx->used += cap;
    }
    if (scratch_need > slot.scratch_cap) {
        const size_t cap = round_cap(scratch_need);
        if (ctx->budget && ctx->used - slot.scratch_cap + cap > ctx->budget)
            return fail(FLIC_ENOMEM, "scratch of %zu bytes exceeds the HBM budget", cap);
        if (slot.scratch) HIP_TRY(hipFree(slot.scratch));
        ctx->used -= slot.scratch_cap;
        slot.scratch = nullptr;
        slot.scratch_cap = 0;
        if (hipMalloc(&slot.scratch, cap) != hipSuccess)
            return fail(FLIC_ENOMEM, "hipMalloc(%zu) for scratch failed", cap);
        slot.scratch_cap = cap;
        ctx->used += cap;
    }
    *out = &slot;
    return FLIC_OK;
}

std::mutex g_default_mu;
flic_ctx* g_default_ctx[64] = {};

}  // namespace

extern "C" {

const char* flic_last_error(void) { return g_last_error.c_str(); }

flic_status flic_ctx_create(flic_ctx** out, int device, size_t hbm_budget_bytes) {
    if (!out) return fail(FLIC_EINVAL, "out is null");
    if (device < 0) return fail(FLIC_EINVAL, "device %d", device);
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device >= count) return fail(FLIC_EINVAL, "device %d of %d", device, count);
    flic_ctx* c = new flic_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    *out = c;
    return FLIC_OK;
}

void flic_ctx_destroy(flic_ctx* ctx) {
    if (!ctx) return;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(ctx->device);
    for (auto* v : {&ctx->timed, &ctx->spare})
        for (auto& ev : *v)
            for (auto e : ev) { (void)hipEventSynchronize(e); (void)hipEventDestroy(e); }
    for (auto& s : ctx->ring) {
        if (s.done) { (void)hipEventSynchronize(s.done); (void)hipEventDestroy(s.done); }
        if (s.dev) (void)hipFree(s.dev);
        if (s.host) (void)hipHostFree(s.host);
        if (s.scratch) (void)hipFree(s.scratch);
    }
    (void)hipSetDevice(prev);
    delete ctx;
}

flic_status flic_set_tile_override(flic_ctx* ctx, int32_t tile_w) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    if (tile_w != 0 && tile_w != 64 && tile_w != 128 && tile_w != 256)
        return fail(FLIC_EINVAL, "tile_w %d not in {0, 64, 128, 256}", tile_w);
    ctx->tile_override = tile_w;
    return FLIC_OK;
}

flic_status flic_ctx_set_tile_rule(flic_ctx* ctx, int32_t H, int32_t W, int32_t skip_depth,
                                   int32_t tile_w) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    if (H < 1 || W < 1 || skip_depth < 1 || skip_depth > FLIC_MAX_SKIP)
        return fail(FLIC_EINVAL, "bad shape %dx%d N=%d", H, W, skip_depth);
    if (tile_w != 0 && tile_w != 64 && tile_w != 128 && tile_w != 256)
        return fail(FLIC_EINVAL, "tile_w %d not in {0, 64, 128, 256}", tile_w);
    auto& v = ctx->rules;
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i].H == H && v[i].W == W && v[i].N == skip_depth) { v.erase(v.begin() + i); break; }
    if (tile_w) v.push_back({H, W, skip_depth, tile_w});
    return FLIC_OK;
}

flic_status flic_ctx_set_plan_parts(flic_ctx* ctx, int32_t parts) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    if (parts < 1 || parts > 64) return fail(FLIC_EINVAL, "parts %d outside 1..64", parts);
    ctx->plan_parts = parts;
    return FLIC_OK;
}

flic_status flic_ctx_tile_for(const flic_ctx* ctx, int32_t H, int32_t W, int32_t skip_depth,
                              int32_t* tile_w) {
    if (!ctx || !tile_w) return fail(FLIC_EINVAL, "null argument");
    *tile_w = choose_tile_w(ctx, H, W, skip_depth);
    return FLIC_OK;
}

flic_status flic_batch_bytes(const flic_ctx* ctx, const flic_scan* scans, int32_t n,
                             size_t* desc_bytes, size_t* scratch) {
    if (!ctx || !desc_bytes || !scratch) return fail(FLIC_EINVAL, "null argument");
    flic_status st = check_scans(scans, n);
    if (st != FLIC_OK) return st;
    Layout L;
    build_layout(ctx, scans, n, nullptr, L);
    *desc_bytes = L.blob.size();
    *scratch = scratch_bytes(ctx, scans, n);
    return FLIC_OK;
}

flic_status flic_ctx_reserve(flic_ctx* ctx, size_t desc_bytes, size_t scratch) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    HIP_TRY(set_device(ctx->device));
    for (int i = 0; i < flic_ctx::kRing; ++i) {
        flic_ctx::Slot* slot = nullptr;
        flic_status st = acquire_slot(ctx, desc_bytes, scratch, &slot);
        if (st != FLIC_OK) return st;
    }
    return FLIC_OK;
}

flic_status flic_ctx_bytes_in_use(const flic_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return fail(FLIC_EINVAL, "null argument");
    *bytes = ctx->used;
    return FLIC_OK;
}

flic_status flic_ctx_set_pass_timing(flic_ctx* ctx, int32_t enable) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    ctx->timing = enable != 0;
    return FLIC_OK;
}

flic_status flic_ctx_pass_times(flic_ctx* ctx, float* total_ms, int32_t* n_launches) {
    if (!ctx || !total_ms || !n_launches) return fail(FLIC_EINVAL, "null argument");
    for (int i = 0; i < flic::kPasses; ++i) total_ms[i] = 0.0f;
    *n_launches = (int32_t)ctx->timed.size();
    for (auto& ev : ctx->timed) {
        HIP_TRY(hipEventSynchronize(ev[flic::kPasses]));
        for (int i = 0; i < flic::kPasses; ++i) {
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            total_ms[i] += ms;
        }
        ctx->spare.push_back(ev);
    }
    ctx->timed.clear();
    return FLIC_OK;
}

flic_status flic_cluster_async(flic_ctx* ctx, const float* range_img, int32_t H, int32_t W,
                               const flic_alpha_tables* alpha_tables, float threshold,
                               int32_t skip_depth, int32_t* labels_out, void* hip_stream) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    flic_status st = check_scan(range_img, H, W, alpha_tables, threshold, skip_depth, labels_out, 0);
    if (st != FLIC_OK) return st;
    const flic_scan s{range_img, H, W, *alpha_tables, threshold, skip_depth, labels_out, 0, 0};
    const int tw = choose_tile_w(ctx, H, W, skip_depth);
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(set_device(ctx->device));
    flic_ctx::Slot* slot = nullptr;
    st = acquire_slot(ctx, 0, flic::scratch_layout(H, W, skip_depth, tw, false).total, &slot);
    if (st != FLIC_OK) return st;
    flic::BatchRef ref{};
    ref.one = make_desc(s, tw, 0, static_cast<char*>(slot->scratch));
    hipError_t e;
    hipEvent_t* ev = timing_events(ctx, &e);
    HIP_TRY(e);
    HIP_TRY(launch_cluster(ref, tw, skip_depth, false, false, ref.one.tiles_x * ref.one.tiles_y, 1, stream, ev));
    HIP_TRY(hipEventRecord(slot->done, stream));
    slot->pending = true;
    return FLIC_OK;
}

flic_status flic_cluster(const float* range_img, int32_t H, int32_t W,
                         const flic_alpha_tables* alpha_tables, float threshold,
                         int32_t skip_depth, int32_t* labels_out) {
    flic_status st = check_scan(range_img, H, W, alpha_tables, threshold, skip_depth, labels_out, 0);
    if (st != FLIC_OK) return st;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(FLIC_EINVAL, "device %d", dev);
    {
        // one shared context per device: the launch is serialised, the wait
        // for its completion is not
        std::lock_guard<std::mutex> lk(g_default_mu);
        if (!g_default_ctx[dev]) {
            st = flic_ctx_create(&g_default_ctx[dev], dev, 0);
            if (st != FLIC_OK) return st;
        }
        st = flic_cluster_async(g_default_ctx[dev], range_img, H, W, alpha_tables, threshold,
                                skip_depth, labels_out, nullptr);
        if (st != FLIC_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(nullptr));
    return FLIC_OK;
}

flic_status flic_cluster_noalloc(const float* range_img, int32_t H, int32_t W,
                                 const flic_alpha_tables* alpha_tables, float threshold,
                                 int32_t skip_depth, int32_t* labels_out, void* hip_stream) {
    flic_status st = check_scan(range_img, H, W, alpha_tables, threshold, skip_depth, labels_out, 0);
    if (st != FLIC_OK) return st;
    const int tw = choose_tile_w(nullptr, H, W, skip_depth);
    const size_t need = flic::scratch_layout(H, W, skip_depth, tw, false).total;
    if (need > flic::kNoAllocScratchBytes)
        return fail(FLIC_EINVAL, "a %dx%d scan with skip_depth %d needs %zu bytes of scratch; "
                    "flic_cluster_noalloc holds %zu", H, W, skip_depth, need, flic::kNoAllocScratchBytes);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= flic::kMaxDevices) return fail(FLIC_EINVAL, "device %d", dev);
    void* scratch = nullptr;
    HIP_TRY(flic::noalloc_scratch(dev, &scratch));
    const flic_scan s{range_img, H, W, *alpha_tables, threshold, skip_depth, labels_out, 0, 0};
    flic::BatchRef ref{};
    ref.one = make_desc(s, tw, 0, static_cast<char*>(scratch));
    HIP_TRY(launch_cluster(ref, tw, skip_depth, false, false, ref.one.tiles_x * ref.one.tiles_y, 1,
                           static_cast<hipStream_t>(hip_stream)));
    return FLIC_OK;
}

flic_status flic_cluster_batched(flic_ctx* ctx, const flic_scan* scans, int32_t n,
                                 void* hip_stream) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    flic_status st = check_scans(scans, n);
    if (st != FLIC_OK) return st;
    if (n == 0) return FLIC_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(set_device(ctx->device));
    // sizes first (the blob size does not depend on the scratch address)
    Layout L;
    build_layout(ctx, scans, n, nullptr, L);
    flic_ctx::Slot* slot = nullptr;
    st = acquire_slot(ctx, L.blob.size(), scratch_bytes(ctx, scans, n), &slot);
    if (st != FLIC_OK) return st;
    build_layout(ctx, scans, n, static_cast<char*>(slot->scratch), L);
    memcpy(slot->host, L.blob.data(), L.blob.size());
    HIP_TRY(hipMemcpyAsync(slot->dev, slot->host, L.blob.size(), hipMemcpyHostToDevice, stream));
    st = enqueue_layout(L, static_cast<const char*>(slot->dev), stream, ctx);
    if (st != FLIC_OK) return st;
    HIP_TRY(hipEventRecord(slot->done, stream));
    slot->pending = true;
    return FLIC_OK;
}

flic_status flic_cluster_batched_host(flic_ctx* ctx, const flic_scan* scans, int32_t n,
                                      const float* const* host_ranges, int32_t* const* host_labels,
                                      void* hip_stream) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    flic_status st = check_scans(scans, n);
    if (st != FLIC_OK) return st;
    if (n == 0) return FLIC_OK;
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(set_device(ctx->device));
    if (host_ranges)
        for (int32_t i = 0; i < n; ++i)
            if (host_ranges[i])
                HIP_TRY(hipMemcpyAsync(const_cast<float*>(scans[i].range_img), host_ranges[i],
                                       (size_t)scans[i].H * scans[i].W * sizeof(float), hipMemcpyHostToDevice,
                                       stream));
    st = flic_cluster_batched(ctx, scans, n, hip_stream);
    if (st != FLIC_OK) return st;
    if (host_labels)
        for (int32_t i = 0; i < n; ++i)
            if (host_labels[i])
                HIP_TRY(hipMemcpyAsync(host_labels[i], scans[i].labels_out,
                                       (size_t)scans[i].H * scans[i].W * sizeof(int32_t), hipMemcpyDeviceToHost,
                                       stream));
    return FLIC_OK;
}

flic_status flic_plan_create(flic_ctx* ctx, const flic_scan* scans, int32_t n, flic_plan** out) {
    if (!ctx || !out) return fail(FLIC_EINVAL, "null ctx or out");
    if (n < 1) return fail(FLIC_EINVAL, "a plan needs n >= 1");
    flic_status st = check_scans(scans, n);
    if (st != FLIC_OK) return st;
    Layout L;
    const int parts = ctx->plan_parts;
    build_layout(ctx, scans, n, nullptr, L, parts);
    const size_t scratch = scratch_bytes(ctx, scans, n);
    if (ctx->budget && ctx->used + L.blob.size() + scratch > ctx->budget)
        return fail(FLIC_ENOMEM, "plan of %zu bytes exceeds the HBM budget", L.blob.size() + scratch);
    HIP_TRY(set_device(ctx->device));
    flic_plan* p = new flic_plan();
    p->ctx = ctx;
    p->n = n;
    p->shapes.assign(scans, scans + n);
    auto cleanup = [&](flic_status s) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->done) (void)hipEventDestroy(p->done);
        if (p->dev_mem) { (void)hipFree(p->dev_mem); ctx->used -= p->blob_bytes; }
        if (p->scratch) { (void)hipFree(p->scratch); ctx->used -= p->scratch_bytes; }
        if (p->host_blob) (void)hipHostFree(p->host_blob);
        delete p;
        return s;
    };
    if (hipMalloc(&p->scratch, scratch) != hipSuccess) {
        p->scratch = nullptr;
        return cleanup(fail(FLIC_ENOMEM, "hipMalloc(%zu) for scratch failed", scratch));
    }
    p->scratch_bytes = scratch;
    ctx->used += scratch;
    build_layout(ctx, scans, n, static_cast<char*>(p->scratch), L, parts);
    p->blob_bytes = L.blob.size();
    for (const auto& g : L.groups)
        p->groups.push_back({g.tile_w, g.skip, g.sized, g.maps, g.n_tiles, g.desc_off, g.members});
    if (hipMalloc(&p->dev_mem, p->blob_bytes) != hipSuccess) {
        p->dev_mem = nullptr;
        return cleanup(fail(FLIC_ENOMEM, "hipMalloc(%zu) failed", p->blob_bytes));
    }
    ctx->used += p->blob_bytes;
    if (hipHostMalloc((void**)&p->host_blob, p->blob_bytes, hipHostMallocDefault) != hipSuccess) {
        p->host_blob = nullptr;
        return cleanup(fail(FLIC_ENOMEM, "hipHostMalloc(%zu) failed", p->blob_bytes));
    }
    memcpy(p->host_blob, L.blob.data(), p->blob_bytes);
    if (hipMemcpy(p->dev_mem, p->host_blob, p->blob_bytes, hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(FLIC_EHIP, "descriptor upload failed"));
    hipError_t e = build_plan_graph(L, static_cast<const char*>(p->dev_mem), &p->graph);
    if (e != hipSuccess) return cleanup(fail(FLIC_EHIP, "plan graph: %s", hipGetErrorString(e)));
    e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return cleanup(fail(FLIC_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e)));
    if (hipEventCreateWithFlags(&p->done, hipEventDisableTiming) != hipSuccess)
        return cleanup(fail(FLIC_EHIP, "hipEventCreate failed"));
    *out = p;
    return FLIC_OK;
}

flic_status flic_plan_launch(flic_plan* plan, const flic_scan* scans, int32_t n, void* hip_stream) {
    if (!plan) return fail(FLIC_EINVAL, "plan is null");
    if (n != plan->n) return fail(FLIC_EINVAL, "plan holds %d scans, got %d", plan->n, n);
    flic_status st = check_scans(scans, n);
    if (st != FLIC_OK) return st;
    for (int32_t i = 0; i < n; ++i) {
        const flic_scan& a = scans[i];
        const flic_scan& b = plan->shapes[i];
        if (a.H != b.H || a.W != b.W || a.skip_depth != b.skip_depth)
            return fail(FLIC_EINVAL, "scan %d shape differs from the plan", i);
        if (sized(a) != sized(b))
            return fail(FLIC_EINVAL, "scan %d: min_points %s 0 in the plan but %d now", i,
                        sized(b) ? ">" : "==", a.min_points);
        if (maps(a) != maps(b))
            return fail(FLIC_EINVAL, "scan %d: map_connections differs from the plan", i);
    }
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(set_device(plan->ctx->device));
    // Refresh descriptors whose pointers, threshold or min_points changed (scratch stays
    // the plan's own).  The pinned staging copy is rewritten only after the
    // previous launch, and with it the previous upload, has completed.
    std::vector<std::pair<size_t, ScanDesc>> changed;
    for (const auto& g : plan->groups) {
        for (size_t m = 0; m < g.members.size(); ++m) {
            const size_t off = g.desc_off + m * sizeof(ScanDesc);
            ScanDesc old;
            memcpy(&old, plan->host_blob + off, sizeof old);
            ScanDesc nd = old;
            const flic_scan& s = scans[g.members[m]];
            nd.range = s.range_img;
            nd.labels = s.labels_out;
            nd.cos_v = s.tables.cos_v;
            nd.cos_h = s.tables.cos_h;
            nd.t2 = s.threshold * s.threshold;
            nd.min_points = s.min_points;
            if (memcmp(&nd, &old, sizeof nd) != 0) changed.push_back({off, nd});
        }
    }
    if (!changed.empty()) {
        if (plan->launched) HIP_TRY(hipEventSynchronize(plan->done));
        for (const auto& c : changed) memcpy(plan->host_blob + c.first, &c.second, sizeof(ScanDesc));
        HIP_TRY(hipMemcpyAsync(plan->dev_mem, plan->host_blob, plan->blob_bytes,
                               hipMemcpyHostToDevice, stream));
        plan->shapes.assign(scans, scans + n);
    }
    // Launches of one plan share its scratch: a launch on another stream
    // waits for the previous one on the device (a no-op on the same stream).
    if (plan->launched) HIP_TRY(hipStreamWaitEvent(stream, plan->done, 0));
    HIP_TRY(hipGraphLaunch(plan->exec, stream));
    HIP_TRY(hipEventRecord(plan->done, stream));
    plan->launched = true;
    return FLIC_OK;
}

flic_status flic_ground_remove(flic_ctx* ctx, const float* range_in, int32_t n_scans,
                               int32_t H, int32_t W, const flic_ground_tables* t,
                               float* range_out, uint8_t* ground_mask, void* hip_stream) {
    if (!ctx) return fail(FLIC_EINVAL, "ctx is null");
    if (!t || !t->sin_a || !t->cos_a || !t->tan_lo || !t->tan_hi || !t->sin_d || !t->cos_d)
        return fail(FLIC_EINVAL, "null table pointer");
    if (n_scans < 0 || n_scans > 65535) return fail(FLIC_EINVAL, "n_scans %d outside 0..65535", n_scans);
    if (H < 1 || W < 1) return fail(FLIC_EINVAL, "H=%d W=%d", H, W);
    if ((int64_t)H * (int64_t)W > (int64_t)INT32_MAX) return fail(FLIC_EINVAL, "H*W exceeds INT32_MAX");
    if (!std::isfinite(t->sensor_height) || !std::isfinite(t->tan_theta))
        return fail(FLIC_EINVAL, "sensor_height and tan_theta must be finite");
    if (n_scans == 0) return FLIC_OK;                // nothing to read or write
    if (!range_in || !range_out) return fail(FLIC_EINVAL, "null range pointer");
    const size_t px = (size_t)n_scans * H * W;
    if (overlaps(range_in, px * 4, range_out, px * 4))
        return fail(FLIC_EINVAL, "range_in and range_out overlap");
    if (ground_mask && (overlaps(ground_mask, px, range_in, px * 4) || overlaps(ground_mask, px, range_out, px * 4)))
        return fail(FLIC_EINVAL, "ground_mask overlaps a range buffer");
    for (const float* tab : {t->sin_a, t->cos_a, t->tan_lo, t->tan_hi, t->sin_d, t->cos_d})
        if (overlaps(tab, (size_t)H * 4, range_out, px * 4) ||
            (ground_mask && overlaps(tab, (size_t)H * 4, ground_mask, px)))
            return fail(FLIC_EINVAL, "a table overlaps an output");
    HIP_TRY(set_device(ctx->device));
    flic::GroundArgs a{range_in, range_out, ground_mask, t->sin_a, t->cos_a, t->tan_lo, t->tan_hi,
                       t->sin_d, t->cos_d, t->sensor_height, t->tan_theta, H, W};
    HIP_TRY(flic::launch_ground(a, n_scans, static_cast<hipStream_t>(hip_stream)));
    return FLIC_OK;
}

void flic_plan_destroy(flic_plan* plan) {
    if (!plan) return;
    (void)set_device(plan->ctx->device);
    if (plan->launched) (void)hipEventSynchronize(plan->done);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->done) (void)hipEventDestroy(plan->done);
    if (plan->dev_mem) (void)hipFree(plan->dev_mem);
    if (plan->scratch) (void)hipFree(plan->scratch);
    if (plan->host_blob) (void)hipHostFree(plan->host_blob);
    plan->ctx->used -= plan->blob_bytes + plan->scratch_bytes;
    delete plan;
}

}  // extern "C"

void flic::record_error(const char* msg) { g_last_error = msg; }

int flic::ctx_device(const flic_ctx* ctx) { return ctx->device; }
