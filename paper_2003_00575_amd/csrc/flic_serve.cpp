// flic_serve.cpp -- the serving runtime: many sensors' frames clustered as
// they arrive (the real-time, frame-by-frame use of Section IV.A), frames that
// are ready together sharing one batched launch.  Admission against an HBM
// budget, FIFO per sensor with drop-oldest backpressure, per-sensor device
// frame slots, continuous batching over several launch streams.  A launch is
// the frames' copies in, flic_cluster_batched on the context the caller owns,
// and the labels' copies out: one DMA copy per frame and direction
// (flic_cluster_batched_host), or one staging kernel per direction for the
// whole batch (k_stage, flic_stage.hip).
#include "../../include/flic.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <limits>
#include <thread>
#include <vector>

#include "flic_internal.h"

namespace {

flic_status sfail(flic_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
flic_status sfail(flic_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    flic::record_error(buf);
    return st;
}

#define SRV_HIP(expr)                                                                \
    do {                                                                             \
        const hipError_t e_ = (expr);                                                \
        if (e_ != hipSuccess)                                                        \
            return sfail(FLIC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

constexpr double kNaN = std::numeric_limits<double>::quiet_NaN();
constexpr double kInf = std::numeric_limits<double>::infinity();

struct Sensor {
    int32_t H = 0, W = 0, N = 0;
    float T = 0.0f;
    float* tables = nullptr;               // device: cos_v [N][H] then cos_h [N][W]
    std::vector<float*> range;             // device frame slots
    std::vector<int32_t*> labels;
    std::vector<int32_t> free_slots;       // the last one freed is taken first
    std::deque<int32_t> waiting;           // frame indices, oldest first
    uint64_t resident = 0;                 // tables + slots, bytes
};

struct Frame {
    int32_t sensor = 0, slot = -1, batch = -1;
    bool staged = false;                   // its host buffers go through the copy kernels
    int64_t tag = 0;
    const float* h_in = nullptr;
    int32_t* h_out = nullptr;
    double t_arrival = 0.0, t_admit = kNaN, t_launch = kNaN, t_done = kNaN;
};

struct Inflight {
    bool busy = false;
    double t_launch = 0.0;
    std::vector<int32_t> frames;
};

}  // namespace

struct flic_server {
    flic_ctx* ctx = nullptr;               // null: simulated device
    int device = 0;
    flic_server_config cfg{};
    std::vector<Sensor> sensors;
    std::vector<Frame> frames;
    std::deque<int32_t> admitted;          // frame indices, in admission order
    std::vector<Inflight> inflight;        // per stream
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> done;
    uint64_t reserved = 0;                 // the sensors' resident bytes
    int64_t dropped = 0, launches = 0;
    std::chrono::steady_clock::time_point t0;
    // launch staging, reused
    std::vector<flic_scan> scans;
    std::vector<const float*> h_in;
    std::vector<int32_t*> h_out;
    std::vector<char> direct;              // per frame of the launch being built: passes use its host buffers
};

namespace {

bool device_mode(const flic_server* s) { return s->ctx != nullptr; }

// Whether the device can read and write [p, p + bytes) at the same addresses
// (pinned host memory mapped into the device's address space), both ends
// asked of the HIP runtime for every frame (an address seen before may since
// belong to another allocation).
bool device_visible(const void* p, size_t bytes) {
    if (!p || bytes == 0 || (reinterpret_cast<uintptr_t>(p) & 15)) return false;
    const char* ends[2] = {static_cast<const char*>(p), static_cast<const char*>(p) + bytes - 1};
    for (const char* q : ends) {
        hipPointerAttribute_t a{};
        if (hipPointerGetAttributes(&a, q) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        if (a.type != hipMemoryTypeHost || a.devicePointer != q) return false;
    }
    return true;
}

void free_sensor(Sensor& sn) {
    for (float* p : sn.range) (void)hipFree(p);
    for (int32_t* p : sn.labels) (void)hipFree(p);
    if (sn.tables) (void)hipFree(sn.tables);
    sn.range.clear();
    sn.labels.clear();
    sn.tables = nullptr;
}

// A scan struct for flic_batch_bytes: only its shape matters there; the
// pointers are distinct, non-overlapping and never dereferenced.
flic_scan shape_only(int32_t H, int32_t W, int32_t N, float T) {
    flic_scan s{};
    s.range_img = reinterpret_cast<const float*>(uintptr_t(1) << 40);
    s.H = H;
    s.W = W;
    s.tables.cos_v = reinterpret_cast<const float*>(uintptr_t(3) << 40);
    s.tables.cos_h = reinterpret_cast<const float*>(uintptr_t(4) << 40);
    s.threshold = T;
    s.skip_depth = N;
    s.labels_out = reinterpret_cast<int32_t*>(uintptr_t(2) << 40);
    return s;
}

// Whether frame k's host buffers, used directly by the passes, would overlap
// the host buffers of an earlier direct frame of the same launch (the batch's
// output buffers must be disjoint from every other buffer of the batch);
// such a frame goes through its device slot instead.
bool overlaps_direct(const flic_server* s, int k, const float* in, const int32_t* out, const Sensor& sn) {
    const size_t bytes = (size_t)sn.H * sn.W * 4;
    const char* ia = reinterpret_cast<const char*>(in);
    const char* oa = reinterpret_cast<const char*>(out);
    if (ia < oa + bytes && oa < ia + bytes) return true;
    for (int q = 0; q < k; ++q) {
        if (!s->direct[q]) continue;
        const flic_scan& o = s->scans[q];
        const size_t ob = (size_t)o.H * o.W * 4;
        const char* qi = reinterpret_cast<const char*>(o.range_img);
        const char* qo = reinterpret_cast<const char*>(o.labels_out);
        // this frame's labels against the other's range and labels; this
        // frame's range against the other's labels
        if ((oa < qi + ob && qi < oa + bytes) || (oa < qo + ob && qo < oa + bytes) ||
            (ia < qo + ob && qo < ia + bytes))
            return true;
    }
    return false;
}

// Frames of `sensor` waiting for a slot take free slots, oldest first.
void admit(flic_server* s, int32_t sensor, double now) {
    Sensor& sn = s->sensors[sensor];
    while (!sn.waiting.empty() && !sn.free_slots.empty()) {
        const int32_t f = sn.waiting.front();
        sn.waiting.pop_front();
        Frame& fr = s->frames[f];
        fr.slot = sn.free_slots.back();
        sn.free_slots.pop_back();
        fr.t_admit = now;
        s->admitted.push_back(f);
    }
}

// 1 when stream i's launch is done, 0 when not yet, < 0 on an error.
int stream_done(flic_server* s, int i, double now) {
    if (!device_mode(s)) return now >= s->inflight[i].t_launch + s->cfg.sim_launch_s ? 1 : 0;
    const hipError_t e = hipEventQuery(s->done[i]);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    sfail(FLIC_EHIP, "hipEventQuery failed: %s", hipGetErrorString(e));
    return -1;
}

flic_status launch(flic_server* s, int i, double now) {
    Inflight& fl = s->inflight[i];
    const int n = (int)std::min<size_t>(s->admitted.size(), (size_t)s->cfg.max_batch);
    fl.frames.clear();
    for (int k = 0; k < n; ++k) {
        const int32_t f = s->admitted.front();
        s->admitted.pop_front();
        Frame& fr = s->frames[f];
        fr.t_launch = now;
        fr.batch = (int32_t)s->launches;
        fl.frames.push_back(f);
    }
    fl.busy = true;
    fl.t_launch = now;
    ++s->launches;
    if (!device_mode(s)) return FLIC_OK;
    s->scans.resize(n);
    s->h_in.resize(n);
    s->h_out.resize(n);
    s->direct.assign(n, 0);
    for (int k = 0; k < n; ++k) {
        const Frame& fr = s->frames[fl.frames[k]];
        const Sensor& sn = s->sensors[fr.sensor];
        flic_scan& sc = s->scans[k];
        sc = flic_scan{};
        sc.range_img = sn.range[fr.slot];
        sc.H = sn.H;
        sc.W = sn.W;
        sc.tables.cos_v = sn.tables;
        sc.tables.cos_h = sn.tables + (size_t)sn.N * sn.H;
        sc.threshold = sn.T;
        sc.skip_depth = sn.N;
        sc.labels_out = sn.labels[fr.slot];
        if (s->cfg.stage_kernels == 2 && fr.staged && !overlaps_direct(s, k, fr.h_in, fr.h_out, sn)) {
            sc.range_img = fr.h_in;                   // the passes read and write the host buffers
            sc.labels_out = fr.h_out;
            s->direct[k] = 1;
        }
        s->h_in[k] = fr.h_in;
        s->h_out[k] = fr.h_out;
    }
    if (!s->cfg.stage_kernels) {
        const flic_status st = flic_cluster_batched_host(s->ctx, s->scans.data(), n, s->h_in.data(),
                                                         s->h_out.data(), s->streams[i]);
        if (st != FLIC_OK) return st;
    } else {
        // frames in: one copy kernel per kStageMax staged frames, a DMA copy
        // for any other; then the batched launch; then the labels out
        for (int dir = 0; dir < 2; ++dir) {
            if (dir == 1) {
                const flic_status st = flic_cluster_batched(s->ctx, s->scans.data(), n, s->streams[i]);
                if (st != FLIC_OK) return st;
            }
            flic::StageList list{};
            int m = 0;
            uint64_t most = 0;
            for (int k = 0; k < n; ++k) {
                const Frame& fr = s->frames[fl.frames[k]];
                const flic_scan& sc = s->scans[k];
                const size_t bytes = (size_t)sc.H * sc.W * 4;
                if (s->direct[k]) continue;                 // no copy at all
                const void* src = dir == 0 ? static_cast<const void*>(fr.h_in) : sc.labels_out;
                void* dst = dir == 0 ? const_cast<float*>(sc.range_img) : static_cast<void*>(fr.h_out);
                if (!fr.staged) {
                    SRV_HIP(hipMemcpyAsync(dst, src, bytes, dir == 0 ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost,
                                           s->streams[i]));
                    continue;
                }
                list.item[m++] = flic::StageItem{src, dst, bytes};
                most = std::max<uint64_t>(most, bytes);
                if (m == flic::kStageMax || k == n - 1) {
                    SRV_HIP(flic::launch_stage(list, m, most, s->streams[i]));
                    m = 0;
                    most = 0;
                }
            }
            if (m > 0) SRV_HIP(flic::launch_stage(list, m, most, s->streams[i]));
        }
    }
    SRV_HIP(hipEventRecord(s->done[i], s->streams[i]));
    return FLIC_OK;
}

bool busy(const flic_server* s) {
    if (!s->admitted.empty()) return true;
    for (const Inflight& fl : s->inflight)
        if (fl.busy) return true;
    for (const Sensor& sn : s->sensors)
        if (!sn.waiting.empty()) return true;
    return false;
}

bool launch_idle(const flic_server* s) {
    if (!s->admitted.empty()) return false;
    for (const Inflight& fl : s->inflight)
        if (fl.busy) return false;
    return true;
}

}  // namespace

extern "C" {

flic_status flic_server_create(flic_ctx* ctx, const flic_server_config* cfg, flic_server** out) {
    if (!out || !cfg) return sfail(FLIC_EINVAL, "null cfg or out");
    const flic_server_config& c = *cfg;
    if (c.n_streams < 1 || c.n_streams > 8) return sfail(FLIC_EINVAL, "n_streams %d outside 1..8", c.n_streams);
    if (c.max_batch < 1 || c.max_batch > 1024) return sfail(FLIC_EINVAL, "max_batch %d outside 1..1024", c.max_batch);
    if (c.slots_per_sensor < 1 || c.slots_per_sensor > 16)
        return sfail(FLIC_EINVAL, "slots_per_sensor %d outside 1..16", c.slots_per_sensor);
    if (c.max_queue < 1) return sfail(FLIC_EINVAL, "max_queue %d < 1", c.max_queue);
    if (c.stage_kernels < 0 || c.stage_kernels > 2)
        return sfail(FLIC_EINVAL, "stage_kernels %d outside 0..2", c.stage_kernels);
    if (!ctx && !(std::isfinite(c.sim_launch_s) && c.sim_launch_s >= 0.0))
        return sfail(FLIC_EINVAL, "sim_launch_s must be finite and >= 0");
    flic_server* s = new flic_server();
    s->ctx = ctx;
    s->cfg = c;
    s->inflight.resize(c.n_streams);
    s->t0 = std::chrono::steady_clock::now();
    if (ctx) {
        s->device = flic::ctx_device(ctx);
        hipError_t e = hipSetDevice(s->device);
        for (int i = 0; e == hipSuccess && i < c.n_streams; ++i) {
            hipStream_t st = nullptr;
            hipEvent_t ev = nullptr;
            e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);   // default priority
            if (e == hipSuccess) s->streams.push_back(st);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) s->done.push_back(ev);
        }
        if (e != hipSuccess) {
            flic_server_destroy(s);
            return sfail(FLIC_EHIP, "stream or event creation failed: %s", hipGetErrorString(e));
        }
    }
    *out = s;
    return FLIC_OK;
}

flic_status flic_server_add_sensor(flic_server* s, int32_t H, int32_t W, const flic_alpha_tables* host_tables,
                                   float threshold, int32_t skip_depth, int32_t* sensor_out) {
    if (!s || !sensor_out || !host_tables) return sfail(FLIC_EINVAL, "null server, tables or sensor_out");
    if (skip_depth < 1 || skip_depth > FLIC_MAX_SKIP)
        return sfail(FLIC_EINVAL, "skip_depth %d outside 1..%d", skip_depth, FLIC_MAX_SKIP);
    if (H < 1 || W <= 2 * skip_depth || (int64_t)H * W > INT32_MAX)
        return sfail(FLIC_EINVAL, "shape %dx%d (need H >= 1, W > 2*skip_depth, H*W <= INT32_MAX)", H, W);
    if (!(std::isfinite(threshold) && threshold >= 0.0f))
        return sfail(FLIC_EINVAL, "threshold must be finite and >= 0");
    if (device_mode(s) && (!host_tables->cos_v || !host_tables->cos_h)) return sfail(FLIC_EINVAL, "null table");
    Sensor sn;
    sn.H = H;
    sn.W = W;
    sn.N = skip_depth;
    sn.T = threshold;
    const size_t px = (size_t)H * W;
    const size_t table_bytes = (size_t)skip_depth * ((size_t)H + W) * sizeof(float);
    sn.resident = table_bytes + (size_t)s->cfg.slots_per_sensor * px * (sizeof(float) + sizeof(int32_t));
    // the launch ring must hold max_batch frames of the largest shape
    int32_t bigH = H, bigW = W, bigN = skip_depth;
    for (const Sensor& o : s->sensors)
        if ((size_t)o.H * o.W > (size_t)bigH * bigW) bigH = o.H, bigW = o.W, bigN = o.N;
    if (device_mode(s)) {
        SRV_HIP(hipSetDevice(s->device));
        size_t desc = 0, scratch = 0;
        const flic_scan one = shape_only(bigH, bigW, bigN, threshold);
        flic_status st = flic_batch_bytes(s->ctx, &one, 1, &desc, &scratch);
        if (st != FLIC_OK) return st;
        st = flic_ctx_reserve(s->ctx, desc * s->cfg.max_batch, scratch * s->cfg.max_batch);
        if (st != FLIC_OK) return st;
        size_t ring = 0;
        st = flic_ctx_bytes_in_use(s->ctx, &ring);
        if (st != FLIC_OK) return st;
        if (s->cfg.hbm_budget && s->reserved + sn.resident + ring > s->cfg.hbm_budget)
            return sfail(FLIC_ENOMEM, "sensor %zu: %llu bytes would exceed the budget of %llu", s->sensors.size(),
                         (unsigned long long)(s->reserved + sn.resident + ring),
                         (unsigned long long)s->cfg.hbm_budget);
        bool ok = hipMalloc(&sn.tables, table_bytes) == hipSuccess;
        if (!ok) sn.tables = nullptr;
        for (int k = 0; ok && k < s->cfg.slots_per_sensor; ++k) {
            float* r = nullptr;
            int32_t* l = nullptr;
            ok = hipMalloc(&r, px * sizeof(float)) == hipSuccess;
            if (ok) sn.range.push_back(r);
            ok = ok && hipMalloc(&l, px * sizeof(int32_t)) == hipSuccess;
            if (ok) sn.labels.push_back(l);
        }
        ok = ok && hipMemcpy(sn.tables, host_tables->cos_v, (size_t)skip_depth * H * sizeof(float),
                             hipMemcpyHostToDevice) == hipSuccess;
        ok = ok && hipMemcpy(sn.tables + (size_t)skip_depth * H, host_tables->cos_h,
                             (size_t)skip_depth * W * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        if (!ok) {
            free_sensor(sn);
            return sfail(FLIC_ENOMEM, "device buffers for a %dx%d sensor", H, W);
        }
    } else if (s->cfg.hbm_budget && s->reserved + sn.resident > s->cfg.hbm_budget) {
        return sfail(FLIC_ENOMEM, "sensor %zu: %llu bytes would exceed the budget of %llu", s->sensors.size(),
                     (unsigned long long)(s->reserved + sn.resident), (unsigned long long)s->cfg.hbm_budget);
    }
    for (int k = 0; k < s->cfg.slots_per_sensor; ++k) sn.free_slots.push_back(k);
    s->reserved += sn.resident;
    *sensor_out = (int32_t)s->sensors.size();
    s->sensors.push_back(std::move(sn));
    return FLIC_OK;
}

flic_status flic_server_submit(flic_server* s, double now, double t_arrival, int32_t sensor,
                               const float* host_range, int32_t* host_labels, int64_t tag) {
    if (!s) return sfail(FLIC_EINVAL, "null server");
    if (sensor < 0 || sensor >= (int32_t)s->sensors.size()) return sfail(FLIC_EINVAL, "unknown sensor %d", sensor);
    if (device_mode(s) && (!host_range || !host_labels)) return sfail(FLIC_EINVAL, "null host buffer");
    Sensor& sn = s->sensors[sensor];
    Frame fr;
    fr.sensor = sensor;
    fr.tag = tag;
    fr.h_in = host_range;
    fr.h_out = host_labels;
    fr.t_arrival = t_arrival;
    if (device_mode(s) && s->cfg.stage_kernels) {
        const size_t bytes = (size_t)sn.H * sn.W * 4;
        fr.staged = device_visible(host_range, bytes) && device_visible(host_labels, bytes);
    }
    const int32_t idx = (int32_t)s->frames.size();
    s->frames.push_back(fr);
    if ((int32_t)sn.waiting.size() >= s->cfg.max_queue) {
        s->frames[sn.waiting.front()].t_done = kInf;
        sn.waiting.pop_front();
        ++s->dropped;
    }
    sn.waiting.push_back(idx);
    admit(s, sensor, now);
    return FLIC_OK;
}

flic_status flic_server_progress(flic_server* s, double now, int32_t* completed) {
    if (!s) return sfail(FLIC_EINVAL, "null server");
    int32_t n = 0;
    for (int i = 0; i < s->cfg.n_streams; ++i) {
        Inflight& fl = s->inflight[i];
        if (!fl.busy) continue;
        const int d = stream_done(s, i, now);
        if (d < 0) return FLIC_EHIP;
        if (d == 0) continue;
        for (int32_t f : fl.frames) {
            Frame& fr = s->frames[f];
            fr.t_done = now;
            s->sensors[fr.sensor].free_slots.push_back(fr.slot);
            ++n;
        }
        fl.busy = false;
        // waiting frames of the batch's sensors take the freed slots (each
        // sensor once, in the order the batch first names it)
        for (size_t k = 0; k < fl.frames.size(); ++k) {
            const int32_t sensor = s->frames[fl.frames[k]].sensor;
            bool seen = false;
            for (size_t q = 0; q < k && !seen; ++q) seen = s->frames[fl.frames[q]].sensor == sensor;
            if (!seen) admit(s, sensor, now);
        }
    }
    for (int i = 0; i < s->cfg.n_streams; ++i) {
        if (s->inflight[i].busy || s->admitted.empty()) continue;
        const flic_status st = launch(s, i, now);
        if (st != FLIC_OK) return st;
    }
    if (completed) *completed = n;
    return FLIC_OK;
}

double flic_server_now(const flic_server* s) {
    if (!s) return kNaN;
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

flic_status flic_server_replay(flic_server* s, const flic_arrival* a, int32_t n) {
    if (!s) return sfail(FLIC_EINVAL, "null server");
    if (n < 0 || (n > 0 && !a)) return sfail(FLIC_EINVAL, "bad arrival list");
    for (int32_t i = 0; i < n; ++i) {
        if (!std::isfinite(a[i].t) || (i > 0 && a[i].t < a[i - 1].t))
            return sfail(FLIC_EINVAL, "arrival %d: times must be finite and non-decreasing", i);
        if (a[i].sensor < 0 || a[i].sensor >= (int32_t)s->sensors.size())
            return sfail(FLIC_EINVAL, "arrival %d: unknown sensor %d", i, a[i].sensor);
        if (device_mode(s) && (!a[i].host_range || !a[i].host_labels))
            return sfail(FLIC_EINVAL, "arrival %d: null host buffer", i);
    }
    const double t0 = flic_server_now(s);
    int32_t i = 0;
    while (i < n || busy(s)) {
        const double now = flic_server_now(s);
        while (i < n && a[i].t <= now - t0) {
            const flic_status st = flic_server_submit(s, flic_server_now(s), t0 + a[i].t, a[i].sensor,
                                                      a[i].host_range, a[i].host_labels, (int64_t)i);
            if (st != FLIC_OK) return st;
            ++i;
        }
        const flic_status st = flic_server_progress(s, flic_server_now(s), nullptr);
        if (st != FLIC_OK) return st;
        if (launch_idle(s) && i < n) {
            const double wait = a[i].t - (flic_server_now(s) - t0);
            if (wait > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(std::min(wait, 1e-3)));
        }
    }
    return FLIC_OK;
}

flic_status flic_server_records(const flic_server* s, flic_frame_record* out, int64_t n_max, int64_t* n_out,
                                int64_t* dropped, int64_t* launches) {
    if (!s || !n_out || n_max < 0 || (n_max > 0 && !out)) return sfail(FLIC_EINVAL, "bad arguments");
    const int64_t n = (int64_t)s->frames.size();
    for (int64_t i = 0; i < std::min(n, n_max); ++i) {
        const Frame& fr = s->frames[i];
        out[i] = flic_frame_record{fr.sensor, std::isinf(fr.t_done) ? -1 : fr.batch, fr.tag, fr.t_arrival,
                                   fr.t_admit, fr.t_launch, fr.t_done};
    }
    *n_out = n;
    if (dropped) *dropped = s->dropped;
    if (launches) *launches = s->launches;
    return FLIC_OK;
}

flic_status flic_server_clear(flic_server* s) {
    if (!s) return sfail(FLIC_EINVAL, "null server");
    if (busy(s)) return sfail(FLIC_EINVAL, "frames are still waiting, admitted or in flight");
    s->frames.clear();
    s->dropped = 0;
    s->launches = 0;
    return FLIC_OK;
}

void flic_server_destroy(flic_server* s) {
    if (!s) return;
    if (device_mode(s)) {
        (void)hipSetDevice(s->device);
        for (hipStream_t st : s->streams) (void)hipStreamSynchronize(st);
        for (Sensor& sn : s->sensors) free_sensor(sn);
        for (hipEvent_t ev : s->done) (void)hipEventDestroy(ev);
        for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    }
    delete s;
}

}  // extern "C"
