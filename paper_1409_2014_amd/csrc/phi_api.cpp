// C ABI of the solver (declared in include/phi_solve.h): parameter checks,
// plan lifetime, device tables and workspace, and the stream-ordered entry
// points.  No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "api_errors.hpp"
#include "phi_solve.h"
#include "plan_host.hpp"
#include "solver_kernels.hpp"

struct phi_plan_s {
    // single plan: host tables and the device view
    phi::HostPlan host;
    phi::DevPlan dev;
    phi::StreamSet streams;     // side stream + fork/join events of the node-side chain
    phi_params params;
    // batched plan (n_members > 0): members share a table set when their
    // parameters are equal; each member has its own workspace
    int n_members = 0;
    std::vector<phi::HostPlan> sets;        // distinct table sets
    std::vector<int> member_set;            // table set of each member
    std::vector<int64_t> offsets;           // packed element offsets, n_members + 1
    phi::BatchDev batch;
    int device = 0;
    void* block = nullptr;      // one device allocation: tables + workspace
    size_t block_bytes = 0;
    std::string last_error;
    phi::KernelTimer timer;     // events of phi_solve_timed, created on first use
    bool timer_ready = false;
};

namespace {

std::mutex g_registry_mutex;
std::set<phi_plan_t>& registry() {
    static std::set<phi_plan_t> live;
    return live;
}
thread_local std::string g_thread_error;

bool is_live(phi_plan_t p) {
    std::lock_guard<std::mutex> lock(g_registry_mutex);
    return p != nullptr && registry().count(p) != 0;
}

phi_status fail(phi_plan_t plan, phi_status st, const std::string& msg) {
    g_thread_error = msg;
    if (plan) plan->last_error = msg;
    return st;
}

phi_status device_fail(phi_plan_t plan, hipError_t e, const char* where) {
    std::string msg = std::string(where) + ": " + hipGetErrorString(e);
    return fail(plan, PHI_ERR_DEVICE, msg);
}

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }


phi_status check_plan(phi_plan_t plan) {
    if (!is_live(plan)) return fail(nullptr, PHI_ERR_INVALID_ARG, "plan is NULL or was destroyed");
    return PHI_OK;
}

phi_status check_device(phi_plan_t plan) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return device_fail(plan, e, "hipGetDevice");
    if (cur != plan->device) return fail(plan, PHI_ERR_INVALID_ARG, "current device differs from the plan's device");
    return PHI_OK;
}

// ---- device layout of tables and workspaces ---------------------------------
struct Part {
    size_t off = 0, bytes = 0;
};
struct Layout {
    size_t cursor = 0;
    Part take(size_t bytes) {
        Part p{cursor, bytes};
        cursor = align256(cursor + bytes);
        return p;
    }
};
// everything a plan reads and never writes
struct TableParts {
    Part deconv, gx, gy, gyr, q, cell, sub, cst, con, taps, twr, twn;
};
// everything a solve writes
struct WorkParts {
    Part xt, tt, win, pts, tiles, u;
};

TableParts layout_tables(const phi::HostPlan& hp, size_t es, Layout& L) {
    TableParts t;
    const size_t n = hp.n, f = hp.n_fine, m = hp.n_nodes;
    t.deconv = L.take(n * 8);
    t.gx = L.take(2 * (f / 2 + 1) * 8);
    t.gy = L.take(2 * f * 8);
    t.gyr = L.take(2 * f * es);
    t.q = L.take(m * 8);
    t.cell = L.take(hp.cell.size() * 4);
    t.sub = L.take(hp.sub.size() * 4);
    t.cst = L.take(hp.contrib_start.size() * 4);
    t.con = L.take(hp.contrib.size() * 4);
    t.taps = L.take(hp.taps.size() * es);
    t.twr = L.take(hp.twr.size() * es);
    t.twn = L.take(hp.twn.size() * es);
    return t;
}

// Column stride of the column-major spectra: N plus 64 elements, so that the
// rows of one block, written across all columns at once, do not fall into a
// few cache sets (a power-of-two stride maps every column to the same sets).
size_t column_stride(const phi::HostPlan& hp) { return static_cast<size_t>(hp.n) + 64; }

WorkParts layout_work(const phi::HostPlan& hp, size_t es, Layout& L) {
    WorkParts w;
    const size_t n = hp.n, f = hp.n_fine, q = hp.patch, m = hp.n_nodes, cs = column_stride(hp);
    w.xt = L.take((f / 2 + 1) * cs * 2 * es);
    w.tt = L.take(q * cs * 2 * es);
    w.win = L.take(q * q * 2 * es);
    w.pts = L.take(m * 2 * es);
    w.tiles = L.take(static_cast<size_t>(hp.n_sub) * hp.tile * hp.tile * 2 * es);
    w.u = L.take(n * q * 2 * es);
    return w;
}

// Enqueues the copies of one table set; `keep` holds the rounded FP32 copies
// until the caller has synchronised the stream.
hipError_t upload_tables(const phi::HostPlan& hp, const TableParts& t, char* base, bool f32, hipStream_t s,
                         std::vector<std::vector<float>>& keep) {
    auto up = [&](const Part& pt, const void* src) -> hipError_t {
        if (pt.bytes == 0) return hipSuccess;
        return hipMemcpyAsync(base + pt.off, src, pt.bytes, hipMemcpyHostToDevice, s);
    };
    // kernel taps, FFT twiddles and the y factors of g1 are rounded once from FP64
    // to the data precision
    auto narrow = [&](const std::vector<double>& v) -> const void* {
        if (!f32) return v.data();
        keep.emplace_back(v.begin(), v.end());
        return keep.back().data();
    };
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = up(t.deconv, hp.deconv.data());
    if (e == hipSuccess) e = up(t.gx, hp.gx.data());
    if (e == hipSuccess) e = up(t.gy, hp.gy.data());
    if (e == hipSuccess) e = up(t.gyr, narrow(hp.gy));
    if (e == hipSuccess) e = up(t.q, hp.q.data());
    if (e == hipSuccess) e = up(t.cell, hp.cell.data());
    if (e == hipSuccess) e = up(t.sub, hp.sub.data());
    if (e == hipSuccess) e = up(t.cst, hp.contrib_start.data());
    if (e == hipSuccess) e = up(t.con, hp.contrib.data());
    if (e == hipSuccess) e = up(t.taps, narrow(hp.taps));
    const void* twr = hp.twr.data();
    if (f32) {
        keep.emplace_back();
        phi::round_unit_pairs(hp.twr, &keep.back());
        twr = keep.back().data();
    }
    if (e == hipSuccess) e = up(t.twr, twr);
    const void* twn = hp.twn.data();
    if (f32) {
        keep.emplace_back();
        phi::round_unit_pairs(hp.twn, &keep.back());
        twn = keep.back().data();
    }
    if (e == hipSuccess) e = up(t.twn, twn);
    return e;
}

// Points the workspace of the device view into the memory at `base`.
void point_work(char* base, const WorkParts& w, phi::DevPlan* d) {
    d->xt = base + w.xt.off;
    d->tt = base + w.tt.off;
    d->win = base + w.win.off;
    d->pts = base + w.pts.off;
    d->tiles = base + w.tiles.off;
    d->u = base + w.u.off;
}

void fill_dev(const phi::HostPlan& hp, phi_dtype dtype, char* base, const TableParts& t,
              const WorkParts& w, phi::DevPlan* d) {
    const double f = hp.n_fine;
    d->dtype = dtype;
    d->n = hp.n;
    d->n_fine = hp.n_fine;
    d->log_fine = hp.log_fine;
    d->log_n = hp.log_n;
    d->patch = hp.patch;
    d->patch_lo = hp.patch_lo;
    d->width = hp.width;
    d->n_nodes = hp.n_nodes;
    d->component = hp.component;
    d->partition_erfc = hp.partition_erfc;
    d->inv_sigma = 1.0 / hp.sigma;
    // The two branches of a solve share the GPU, and the one enqueued first is
    // served first: the node-side chain (the same few small kernels at every N)
    // unless the high-frequency columns carry at least the work they have in a
    // 2048^2 FP32 solve (N F log2 F times the element size), where they are the
    // longer branch.  Graph replay on MI355X: 2048^2 FP32 98.2 -> 95.8..97.2 us
    // with the columns first, 1024^2 FP64 60.5 -> 70.5 us (so chain first there).
    const double col_work = (f / 2) * f * std::log2(f) * (dtype == PHI_F32 ? 4.0 : 8.0);
    d->highfreq_first = col_work >= 2048.0 * 4096.0 * 12.0 * 4.0 ? 1 : 0;
    // Padded sides up to 1024 (both precisions) and FP32 solves on padded side
    // 2048 run the one-stream layout: cols_type2, nodes, then the type-1 window
    // columns and every I1 column in one launch.  Graph replay on MI355X, two
    // runs each (µs): 64^2 FP64 42.5, 43.4 -> 36.3, 36.2; 128^2 FP64 44.9, 51.4
    // -> 37.7, 37.6; 256^2 FP32 51.5, 45.1 -> 36.7, 36.8; 256^2 FP64 48.4, 50.9 ->
    // 41.1, 41.0 (against the one launch with device-counter waits that these
    // sides used before); 512^2 FP32 63.7 -> 38.8, 512^2 FP64 52.5..71 -> 44.8;
    // 1024^2 FP32 49..58 -> 48.6 (against the two-stream layout, whose time
    // there varies from run to run).  Splitting the I1 columns over the three
    // chain launches instead was slower at every size (e.g. 512^2 FP64 50.7,
    // 1024^2 FP32 50.1).  Where the I1 columns are the longer branch the
    // two-stream layout is faster: 1024^2 FP64 60..63 against 63.3, 2048^2 FP32
    // 96.5..97 against 100.3, 2048^2 FP64 143..145 against 152.
    d->shared = (!hp.two_streams && hp.width <= phi::kMaxEsWidth && hp.log_fine >= phi::kSharedMinLogFine &&
                 (hp.log_fine <= 10 || (dtype == PHI_F32 && hp.log_fine <= 11))) ? 1 : 0;
    d->freq_scale = 1.0 / (f * hp.h * hp.sigma);
    d->col_stride = static_cast<int>(column_stride(hp));
    d->h2 = hp.h * hp.h;
    d->inv_f2 = 1.0 / (f * f);
    d->deconv = reinterpret_cast<const double*>(base + t.deconv.off);
    d->gx = reinterpret_cast<const double*>(base + t.gx.off);
    d->gy = reinterpret_cast<const double*>(base + t.gy.off);
    d->gyr = base + t.gyr.off;
    d->q = reinterpret_cast<const double*>(base + t.q.off);
    d->cell = reinterpret_cast<const int*>(base + t.cell.off);
    d->taps = base + t.taps.off;
    d->sub = reinterpret_cast<const int*>(base + t.sub.off);
    d->contrib_start = reinterpret_cast<const int*>(base + t.cst.off);
    d->contrib = reinterpret_cast<const int*>(base + t.con.off);
    d->n_sub = hp.n_sub;
    d->bin = hp.bin;
    d->tile = hp.tile;
    d->twr = base + t.twr.off;
    d->twr_count = static_cast<int>(hp.twr.size() / 2);
    d->twn = base + t.twn.off;
    d->twn_count = static_cast<int>(hp.twn.size() / 2);
    point_work(base, w, d);
}

phi_status create_streams(phi_plan_t plan) {
    // the node-side chain runs on a second stream of the plan's device, default priority
    hipError_t e = hipStreamCreateWithFlags(&plan->streams.side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->streams.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->streams.join, hipEventDisableTiming);
    if (e != hipSuccess) return device_fail(nullptr, e, "plan streams");
    return PHI_OK;
}

void release(phi_plan_t plan) {
    if (plan->timer_ready) {
        for (int i = 0; i < 2 * phi::KernelTimer::kMax; ++i) (void)hipEventDestroy(plan->timer.ev[i]);
    }
    if (plan->streams.join) (void)hipEventDestroy(plan->streams.join);
    if (plan->streams.fork) (void)hipEventDestroy(plan->streams.fork);
    if (plan->streams.side) (void)hipStreamDestroy(plan->streams.side);
    if (plan->block) (void)hipFree(plan->block);
    plan->block = nullptr;
}

phi_status register_plan(phi_plan_t plan, phi_plan_t* out) {
    std::lock_guard<std::mutex> lock(g_registry_mutex);
    registry().insert(plan);
    *out = plan;
    return PHI_OK;
}

// A single plan on the current device, not yet registered.  On failure
// nothing is left allocated.
phi_status create_single(const phi_params* p, hipStream_t s, phi_plan_s** out) {
    *out = nullptr;
    std::unique_ptr<phi_plan_s> plan(new phi_plan_s());
    std::string err;
    phi_status st = phi::build_host_plan(p, &plan->host, &err);
    if (st != PHI_OK) return fail(nullptr, st, err);
    plan->params = *p;
    const phi::HostPlan& hp = plan->host;
    hipError_t e = hipGetDevice(&plan->device);
    if (e != hipSuccess) return device_fail(nullptr, e, "hipGetDevice");
    const bool f32 = (p->dtype == PHI_F32);
    const size_t es = f32 ? 4 : 8;
    Layout L;
    const TableParts tp = layout_tables(hp, es, L);
    const WorkParts wp = layout_work(hp, es, L);
    plan->block_bytes = L.cursor;
    e = hipMalloc(&plan->block, L.cursor);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        plan->block = nullptr;
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    char* base = static_cast<char*>(plan->block);
    std::vector<std::vector<float>> keep;
    e = upload_tables(hp, tp, base, f32, s, keep);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        release(plan.get());
        return device_fail(nullptr, e, "table upload");
    }
    st = create_streams(plan.get());
    if (st != PHI_OK) {
        release(plan.get());
        return st;
    }
    fill_dev(hp, p->dtype, base, tp, wp, &plan->dev);
    *out = plan.release();
    return PHI_OK;
}

void destroy_unregistered(phi_plan_s* plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    release(plan);
    delete plan;
}

// Picks the bin side and subproblem size of the node sort by timing whole
// solves of a zero density with every candidate on the current device (two
// warm-up solves, then the median of five).  *best = *p with the fastest
// candidate's bin / sub_nodes and the autotune flag cleared.
phi_status autotune(const phi_params* p, hipStream_t s, phi_params* best) {
    static const int kBins[] = {4, 8, 16};
    static const int kSubs[] = {32, 64};
    phi::HostPlan probe;
    std::string err;
    phi_status st = phi::derive(p, &probe, &err);
    if (st != PHI_OK) return fail(nullptr, st, err);
    const size_t es = (p->dtype == PHI_F32) ? 4 : 8;
    const size_t grid_bytes = static_cast<size_t>(probe.n) * probe.n * es;
    void* io = nullptr;
    hipError_t e = hipMalloc(&io, 2 * grid_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipMemsetAsync(io, 0, grid_bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    *best = *p;
    best->flags &= ~PHI_AUTOTUNE;
    float best_ms = -1.f;
    for (int b : kBins) {
        for (int sn : kSubs) {
            if (e != hipSuccess || st != PHI_OK) break;
            if (b + probe.width - 1 > phi::kMaxTile) continue;   // tile too large for this kernel
            phi_params cand = *best;
            cand.bin = b;
            cand.sub_nodes = sn;
            phi_plan_s* pl = nullptr;
            st = create_single(&cand, s, &pl);
            if (st != PHI_OK) break;
            void* in = io;
            void* out_buf = static_cast<char*>(io) + grid_bytes;
            std::vector<float> ms;
            for (int it = 0; it < 7 && e == hipSuccess; ++it) {
                if (it >= 2) e = hipEventRecord(ev[0], s);
                if (e == hipSuccess) e = phi::enqueue(pl->dev, pl->streams, phi::Stage::Solve, in, out_buf, 0, s);
                if (e == hipSuccess && it >= 2) e = hipEventRecord(ev[1], s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                float t = 0.f;
                if (e == hipSuccess && it >= 2) e = hipEventElapsedTime(&t, ev[0], ev[1]);
                if (e == hipSuccess && it >= 2) ms.push_back(t);
            }
            destroy_unregistered(pl);
            if (e != hipSuccess) break;
            std::nth_element(ms.begin(), ms.begin() + ms.size() / 2, ms.end());
            const float med = ms[ms.size() / 2];
            if (best_ms < 0.f || med < best_ms) {
                best_ms = med;
                best->bin = b;
                best->sub_nodes = sn;
            }
        }
    }
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
    (void)hipFree(io);
    if (st != PHI_OK) return st;
    if (e != hipSuccess) return device_fail(nullptr, e, "autotune");
    return PHI_OK;
}

hipError_t enqueue_any(phi_plan_t plan, phi::Stage stage, const void* in, void* out, int adjoint, hipStream_t s,
                       phi::KernelTimer* timer) {
    if (plan->n_members > 0) return phi::enqueue_batch(plan->batch, plan->streams, in, out, adjoint, s, timer);
    return phi::enqueue(plan->dev, plan->streams, stage, in, out, adjoint, s, timer);
}

phi_status run(phi_plan_t plan, phi::Stage stage, const void* in, void* out, int adjoint, void* stream) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!in || !out) return fail(plan, PHI_ERR_INVALID_ARG, "NULL data pointer");
    if (in == out) return fail(plan, PHI_ERR_INVALID_ARG, "input and output must not alias");
    if (plan->n_members > 0 && stage != phi::Stage::Solve)
        return fail(plan, PHI_ERR_UNSUPPORTED, "stage entry points take single plans only");
    st = check_device(plan);
    if (st != PHI_OK) return st;
    hipError_t e = enqueue_any(plan, stage, in, out, adjoint, static_cast<hipStream_t>(stream), nullptr);
    if (e != hipSuccess) return device_fail(plan, e, "kernel launch");
    return PHI_OK;
}

// Field-wise equality of every field of phi_params (the struct's padding
// bytes are not compared); members that differ only in their node sort get
// table sets of their own.
bool same_params(const phi_params& a, const phi_params& b) {
    return a.nx == b.nx && a.ny == b.ny && a.hx == b.hx && a.hy == b.hy && a.n_r == b.n_r &&
           a.n_theta == b.n_theta && a.tol == b.tol && a.pad == b.pad && a.sigma == b.sigma &&
           a.cutoff == b.cutoff && a.dtype == b.dtype && a.flags == b.flags && a.bin == b.bin &&
           a.sub_nodes == b.sub_nodes;
}

// Work items of one member and stage: first row / column / subproblem of each
// block.  Members are listed largest first, so the last blocks to start are short.
void push_items(std::vector<phi::WorkItem>* v, int member, int kind, int count, int step) {
    for (int i = 0; i < count; i += step) v->push_back({member, i, kind, 0});
}

}  // namespace

phi_status phi::thread_error(phi_status st, const std::string& msg) {
    g_thread_error = msg;
    return st;
}

extern "C" {

const char* phi_status_string(phi_status s) {
    switch (s) {
        case PHI_OK: return "PHI_OK";
        case PHI_ERR_INVALID_ARG: return "PHI_ERR_INVALID_ARG";
        case PHI_ERR_UNSUPPORTED: return "PHI_ERR_UNSUPPORTED";
        case PHI_ERR_TOL_UNREACHABLE: return "PHI_ERR_TOL_UNREACHABLE";
        case PHI_ERR_OUT_OF_MEMORY: return "PHI_ERR_OUT_OF_MEMORY";
        case PHI_ERR_DEVICE: return "PHI_ERR_DEVICE";
        case PHI_ERR_INTERNAL: return "PHI_ERR_INTERNAL";
    }
    return "PHI_STATUS_UNKNOWN";
}

const char* phi_last_error(phi_plan_t plan) {
    if (plan && is_live(plan)) return plan->last_error.c_str();
    return g_thread_error.c_str();
}

phi_status phi_params_default(phi_params* p, int32_t n, double h, phi_dtype dtype) {
    if (!p) return fail(nullptr, PHI_ERR_INVALID_ARG, "NULL params");
    return phi::fill_defaults(p, n, h, dtype);
}

static void fill_info(const phi::HostPlan& hp, size_t bytes, phi_plan_info* info) {
    info->n = hp.n;
    info->n_fine = hp.n_fine;
    info->n_nodes = hp.n_nodes;
    info->kernel_width = hp.width;
    info->patch = hp.patch;
    info->patch_lo = hp.patch_lo;
    info->max_cell_nodes = hp.max_cell_nodes;
    info->max_gather = hp.max_gather;
    info->bin = hp.bin;
    info->tile = hp.tile;
    info->n_sub = hp.n_sub;
    info->sub_nodes = hp.sub_nodes;
    info->n_contrib = static_cast<int64_t>(hp.contrib.size());
    info->h = hp.h;
    info->half_width = hp.half_width;
    info->sigma = hp.sigma;
    info->cutoff = hp.cutoff;
    info->beta = hp.beta;
    info->device_bytes = bytes;
}

phi_status phi_describe(const phi_params* p, phi_plan_info* info) {
    if (!p || !info) return fail(nullptr, PHI_ERR_INVALID_ARG, "NULL argument");
    try {
        phi::HostPlan hp;
        std::string err;
        phi_status st = phi::build_host_plan(p, &hp, &err);
        if (st != PHI_OK) return fail(nullptr, st, err);
        fill_info(hp, 0, info);
        return PHI_OK;
    } catch (const std::bad_alloc&) {
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(nullptr, PHI_ERR_INTERNAL, "unexpected exception");
    }
}

phi_status phi_plan(const phi_params* p, void* stream, phi_plan_t* out) {
    if (!p || !out) return fail(nullptr, PHI_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    try {
        hipStream_t s = static_cast<hipStream_t>(stream);
        phi_params chosen = *p;
        if (p->flags & PHI_AUTOTUNE) {
            phi_status st = autotune(p, s, &chosen);
            if (st != PHI_OK) return st;
        }
        phi_plan_s* plan = nullptr;
        phi_status st = create_single(&chosen, s, &plan);
        if (st != PHI_OK) return st;
        return register_plan(plan, out);
    } catch (const std::bad_alloc&) {
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(nullptr, PHI_ERR_INTERNAL, "unexpected exception");
    }
}

phi_status phi_plan_batch(const phi_params* members, int32_t count, void* stream, phi_plan_t* out) {
    if (!members || !out || count < 1) return fail(nullptr, PHI_ERR_INVALID_ARG, "NULL argument or empty batch");
    *out = nullptr;
    phi_plan_s* plan = nullptr;
    try {
        plan = new phi_plan_s();
        plan->n_members = count;
        plan->member_set.resize(count);
        const phi_dtype dtype = members[0].dtype;
        std::vector<phi_params> set_params;
        for (int i = 0; i < count; ++i) {
            const phi_params& p = members[i];
            if (p.dtype != dtype) {
                delete plan;
                return fail(nullptr, PHI_ERR_INVALID_ARG, "all members of a batch must have the same dtype");
            }
            int found = -1;
            for (size_t k = 0; k < set_params.size(); ++k)
                if (same_params(set_params[k], p)) found = static_cast<int>(k);
            if (found < 0) {
                phi::HostPlan hp;
                std::string err;
                phi_params chosen = p;
                if (p.flags & PHI_AUTOTUNE) {
                    phi_status st = autotune(&p, static_cast<hipStream_t>(stream), &chosen);
                    if (st != PHI_OK) {
                        delete plan;
                        return st;
                    }
                }
                phi_status st = phi::build_host_plan(&chosen, &hp, &err);
                if (st != PHI_OK) {
                    delete plan;
                    return fail(nullptr, st, "member " + std::to_string(i) + ": " + err);
                }
                if (hp.component == 3) {
                    delete plan;
                    return fail(nullptr, PHI_ERR_UNSUPPORTED,
                                "member " + std::to_string(i) + ": the Coulomb multiplier is not batched");
                }
                if (hp.log_fine < phi::kBatchMinLogFine || hp.log_fine > phi::kBatchMaxLogFine) {
                    delete plan;
                    return fail(nullptr, PHI_ERR_UNSUPPORTED,
                                "member " + std::to_string(i) + ": batched members need a padded side of 256 .. 4096");
                }
                set_params.push_back(p);
                plan->sets.push_back(std::move(hp));
                found = static_cast<int>(plan->sets.size()) - 1;
            }
            plan->member_set[i] = found;
        }
        plan->params = members[0];
        hipError_t e = hipGetDevice(&plan->device);
        if (e != hipSuccess) {
            delete plan;
            return device_fail(nullptr, e, "hipGetDevice");
        }
        const bool f32 = (dtype == PHI_F32);
        const size_t es = f32 ? 4 : 8;
        // packed element offsets
        plan->offsets.assign(count + 1, 0);
        for (int i = 0; i < count; ++i) {
            const int64_t n = plan->sets[plan->member_set[i]].n;
            plan->offsets[i + 1] = plan->offsets[i] + n * n;
        }
        // work tables, members in decreasing size order
        std::vector<int> order(count);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return plan->sets[plan->member_set[a]].n > plan->sets[plan->member_set[b]].n;
        });
        std::vector<phi::WorkItem> rows, cols, cols_t2, cols_mixed, nodes, cols1;
        for (int i : order) {
            const phi::HostPlan& hp = plan->sets[plan->member_set[i]];
            const int g = phi::batch_lines(hp.log_fine);
            push_items(&rows, i, 0, hp.n, g);
            push_items(hp.component == 2 ? &cols_mixed : &cols, i, 0, hp.n_fine / 2 + 1, g);
            push_items(&cols_t2, i, 1, hp.patch, g);
            push_items(&nodes, i, 0, hp.n_sub, 1);
            push_items(&cols1, i, 0, hp.patch, g);
        }
        // one allocation: table sets, member workspaces, device views, work tables
        Layout L;
        std::vector<TableParts> tparts;
        for (const phi::HostPlan& hp : plan->sets) tparts.push_back(layout_tables(hp, es, L));
        std::vector<WorkParts> wparts;
        for (int i = 0; i < count; ++i) wparts.push_back(layout_work(plan->sets[plan->member_set[i]], es, L));
        const Part p_dev = L.take(sizeof(phi::DevPlan) * count);
        const Part p_off = L.take(sizeof(int64_t) * (count + 1));
        const Part p_rows = L.take(sizeof(phi::WorkItem) * rows.size());
        const Part p_cols = L.take(sizeof(phi::WorkItem) * cols.size());
        const Part p_cols_t2 = L.take(sizeof(phi::WorkItem) * cols_t2.size());
        const Part p_cols_mixed = L.take(sizeof(phi::WorkItem) * cols_mixed.size());
        const Part p_nodes = L.take(sizeof(phi::WorkItem) * nodes.size());
        const Part p_cols1 = L.take(sizeof(phi::WorkItem) * cols1.size());
        plan->block_bytes = L.cursor;
        e = hipMalloc(&plan->block, L.cursor);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            plan->block = nullptr;
            delete plan;
            return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        char* base = static_cast<char*>(plan->block);
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<std::vector<float>> keep;
        for (size_t k = 0; k < plan->sets.size() && e == hipSuccess; ++k)
            e = upload_tables(plan->sets[k], tparts[k], base, f32, s, keep);
        std::vector<phi::DevPlan> devs(count);
        for (int i = 0; i < count; ++i)
            fill_dev(plan->sets[plan->member_set[i]], dtype, base, tparts[plan->member_set[i]], wparts[i],
                     &devs[i]);
        auto up = [&](const Part& pt, const void* src) -> hipError_t {
            if (pt.bytes == 0) return hipSuccess;
            return hipMemcpyAsync(base + pt.off, src, pt.bytes, hipMemcpyHostToDevice, s);
        };
        if (e == hipSuccess) e = up(p_dev, devs.data());
        if (e == hipSuccess) e = up(p_off, plan->offsets.data());
        if (e == hipSuccess) e = up(p_rows, rows.data());
        if (e == hipSuccess) e = up(p_cols, cols.data());
        if (e == hipSuccess) e = up(p_cols_t2, cols_t2.data());
        if (e == hipSuccess) e = up(p_cols_mixed, cols_mixed.data());
        if (e == hipSuccess) e = up(p_nodes, nodes.data());
        if (e == hipSuccess) e = up(p_cols1, cols1.data());
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            release(plan);
            delete plan;
            return device_fail(nullptr, e, "table upload");
        }
        phi::BatchDev& b = plan->batch;
        b.dtype = dtype;
        b.members = reinterpret_cast<const phi::DevPlan*>(base + p_dev.off);
        b.offsets = reinterpret_cast<const int64_t*>(base + p_off.off);
        b.rows = reinterpret_cast<const phi::WorkItem*>(base + p_rows.off);
        b.cols = reinterpret_cast<const phi::WorkItem*>(base + p_cols.off);
        b.cols_t2 = reinterpret_cast<const phi::WorkItem*>(base + p_cols_t2.off);
        b.cols_mixed = reinterpret_cast<const phi::WorkItem*>(base + p_cols_mixed.off);
        b.nodes = reinterpret_cast<const phi::WorkItem*>(base + p_nodes.off);
        b.cols1 = reinterpret_cast<const phi::WorkItem*>(base + p_cols1.off);
        b.n_rows = static_cast<int>(rows.size());
        b.n_cols = static_cast<int>(cols.size());
        b.n_cols_t2 = static_cast<int>(cols_t2.size());
        b.n_cols_mixed = static_cast<int>(cols_mixed.size());
        for (const phi::HostPlan& hp : plan->sets) b.wide_kernel |= (hp.width > phi::kMaxEsWidth) ? 1 : 0;
        b.n_nodes = static_cast<int>(nodes.size());
        b.n_cols1 = static_cast<int>(cols1.size());
        plan->host = plan->sets[plan->member_set[0]];
        phi_status sst = create_streams(plan);
        if (sst != PHI_OK) {
            release(plan);
            delete plan;
            return sst;
        }
        return register_plan(plan, out);
    } catch (const std::bad_alloc&) {
        if (plan) {
            release(plan);
            delete plan;
        }
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        if (plan) {
            release(plan);
            delete plan;
        }
        return fail(nullptr, PHI_ERR_INTERNAL, "unexpected exception");
    }
}

phi_status phi_batch_layout(phi_plan_t plan, int32_t* count, int64_t* offsets) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!count) return fail(plan, PHI_ERR_INVALID_ARG, "NULL count");
    if (plan->n_members == 0) {
        *count = 1;
        if (offsets) {
            offsets[0] = 0;
            offsets[1] = static_cast<int64_t>(plan->host.n) * plan->host.n;
        }
        return PHI_OK;
    }
    *count = plan->n_members;
    if (offsets) std::memcpy(offsets, plan->offsets.data(), sizeof(int64_t) * (plan->n_members + 1));
    return PHI_OK;
}

phi_status phi_batch_member_info(phi_plan_t plan, int32_t member, phi_plan_info* info) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!info) return fail(plan, PHI_ERR_INVALID_ARG, "NULL info");
    const int count = plan->n_members > 0 ? plan->n_members : 1;
    if (member < 0 || member >= count) return fail(plan, PHI_ERR_INVALID_ARG, "member index out of range");
    if (plan->n_members == 0) {
        fill_info(plan->host, plan->block_bytes, info);
    } else {
        fill_info(plan->sets[plan->member_set[member]], 0, info);
    }
    return PHI_OK;
}

phi_status phi_destroy(phi_plan_t plan) {
    if (!plan) return PHI_OK;
    {
        std::lock_guard<std::mutex> lock(g_registry_mutex);
        if (registry().erase(plan) == 0) return fail(nullptr, PHI_ERR_INVALID_ARG, "plan was already destroyed");
    }
    phi_status st = PHI_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != plan->device) (void)hipSetDevice(plan->device);
    hipError_t e = hipDeviceSynchronize();   // the plan's last stream work may still read its tables
    if (e == hipSuccess) {
        release(plan);
    } else {
        st = fail(nullptr, PHI_ERR_DEVICE, std::string("phi_destroy: ") + hipGetErrorString(e));
    }
    if (prev >= 0 && prev != plan->device) (void)hipSetDevice(prev);
    delete plan;
    return st;
}

phi_status phi_plan_get_info(phi_plan_t plan, phi_plan_info* info) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!info) return fail(plan, PHI_ERR_INVALID_ARG, "NULL info");
    fill_info(plan->host, plan->block_bytes, info);
    return PHI_OK;
}

phi_status phi_plan_nodes(phi_plan_t plan, double* kx, double* ky, double* q) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (plan->n_members > 0) return fail(plan, PHI_ERR_UNSUPPORTED, "node tables of batched plans are per member");
    const size_t m = plan->host.n_nodes;
    if (kx) std::memcpy(kx, plan->host.kx.data(), m * sizeof(double));
    if (ky) std::memcpy(ky, plan->host.ky.data(), m * sizeof(double));
    if (q) std::memcpy(q, plan->host.q.data(), m * sizeof(double));
    return PHI_OK;
}

phi_status phi_solve(phi_plan_t plan, const void* rho, void* phi_out, void* stream) {
    return run(plan, phi::Stage::Solve, rho, phi_out, 0, stream);
}

phi_status phi_solve_noalloc(phi_plan_t plan, const void* rho, void* phi_out, void* stream) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!rho || !phi_out) return fail(plan, PHI_ERR_INVALID_ARG, "NULL data pointer");
    if (rho == phi_out) return fail(plan, PHI_ERR_INVALID_ARG, "input and output must not alias");
    if (plan->n_members > 0) return fail(plan, PHI_ERR_UNSUPPORTED, "phi_solve_noalloc takes single plans only");
    st = check_device(plan);
    if (st != PHI_OK) return st;
    // the same workspace layout as the plan's own, placed in the static scratch
    const size_t es = plan->host.dtype == PHI_F32 ? 4 : 8;
    Layout L;
    const WorkParts wp = layout_work(plan->host, es, L);
    if (L.cursor > phi::scratch_capacity()) {
        char msg[200];
        std::snprintf(msg, sizeof(msg),
                      "phi_solve_noalloc: this plan needs %zu bytes of scratch; the static scratch holds %zu",
                      L.cursor, phi::scratch_capacity());
        return fail(plan, PHI_ERR_UNSUPPORTED, msg);
    }
    void* base = nullptr;
    hipError_t e = phi::scratch_region(plan->device, &base);
    if (e != hipSuccess) return device_fail(plan, e, "static scratch address");
    phi::DevPlan d = plan->dev;
    point_work(static_cast<char*>(base), wp, &d);
    e = phi::enqueue(d, plan->streams, phi::Stage::Solve, rho, phi_out, 0, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(plan, e, "kernel launch");
    return PHI_OK;
}

phi_status phi_solve_adjoint(phi_plan_t plan, const void* g_phi, void* g_rho, void* stream) {
    return run(plan, phi::Stage::Solve, g_phi, g_rho, 1, stream);
}

phi_status phi_solve_highfreq(phi_plan_t plan, const void* rho, void* i1, void* stream) {
    return run(plan, phi::Stage::HighFreq, rho, i1, 0, stream);
}

phi_status phi_solve_lowfreq(phi_plan_t plan, const void* rho, void* i2, void* stream) {
    return run(plan, phi::Stage::LowFreq, rho, i2, 0, stream);
}

phi_status phi_nodes_type2(phi_plan_t plan, const void* rho, void* rho_hat, void* stream) {
    return run(plan, phi::Stage::Type2, rho, rho_hat, 0, stream);
}

phi_status phi_nodes_type1(phi_plan_t plan, const void* coef, void* field, void* stream) {
    return run(plan, phi::Stage::Type1, coef, field, 0, stream);
}

phi_status phi_solve_periodic(phi_plan_t plan, const void* rho, void* phi_out, void* stream) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (plan->n_members == 0 && plan->host.component == 3)
        return fail(plan, PHI_ERR_UNSUPPORTED, "the periodic solver takes the DS multipliers, not the Coulomb one");
    if (plan->n_members == 0 && (plan->host.log_n < 4 || plan->host.log_n > 12))
        return fail(plan, PHI_ERR_UNSUPPORTED, "the periodic solver takes power-of-two grid sides 16 .. 4096");
    return run(plan, phi::Stage::Periodic, rho, phi_out, 0, stream);
}

phi_status phi_solve_timed(phi_plan_t plan, const void* in, void* out, int32_t adjoint, void* stream,
                           float* kernel_ms, const char** names, int32_t capacity, int32_t* count) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!in || !out || !count || (capacity > 0 && (!kernel_ms || !names)) || capacity < 0)
        return fail(plan, PHI_ERR_INVALID_ARG, "NULL or invalid argument");
    if (in == out) return fail(plan, PHI_ERR_INVALID_ARG, "input and output must not alias");
    st = check_device(plan);
    if (st != PHI_OK) return st;
    hipError_t e = hipSuccess;
    phi::KernelTimer& t = plan->timer;
    if (!plan->timer_ready) {
        for (int i = 0; i < 2 * phi::KernelTimer::kMax; ++i) {
            e = hipEventCreate(&t.ev[i]);
            if (e != hipSuccess) {
                for (int k = 0; k < i; ++k) (void)hipEventDestroy(t.ev[k]);
                return device_fail(plan, e, "hipEventCreate");
            }
        }
        plan->timer_ready = true;
    }
    t.count = 0;
    hipStream_t s = static_cast<hipStream_t>(stream);
    e = enqueue_any(plan, phi::Stage::Solve, in, out, adjoint ? 1 : 0, s, &t);
    if (e != hipSuccess) return device_fail(plan, e, "kernel launch");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_fail(plan, e, "hipStreamSynchronize");
    *count = t.count;
    for (int i = 0; i < t.count && i < capacity; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]);
        if (e != hipSuccess) return device_fail(plan, e, "hipEventElapsedTime");
        kernel_ms[i] = ms;
        names[i] = t.names[i];
    }
    return PHI_OK;
}

phi_status phi_host_gauss_legendre(int32_t n, double* x, double* w) {
    if (n < 1 || !x || !w) return fail(nullptr, PHI_ERR_INVALID_ARG, "bad Gauss-Legendre arguments");
    phi::gauss_legendre(n, x, w);
    return PHI_OK;
}

phi_status phi_host_gauss_jacobi01(int32_t n, double* x, double* w) {
    if (n < 1 || !x || !w) return fail(nullptr, PHI_ERR_INVALID_ARG, "bad Gauss-Jacobi arguments");
    phi::gauss_jacobi01(n, x, w);
    return PHI_OK;
}

phi_status phi_host_es_kernel(int32_t count, const double* z, double beta, double* out) {
    if (count < 0 || (count > 0 && (!z || !out))) return fail(nullptr, PHI_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < count; ++i) out[i] = phi::es_kernel(z[i], beta);
    return PHI_OK;
}

phi_status phi_host_es_transform(int32_t count, const double* omega, double beta, double* out) {
    if (count < 0 || (count > 0 && (!omega || !out))) return fail(nullptr, PHI_ERR_INVALID_ARG, "bad arguments");
    for (int i = 0; i < count; ++i) out[i] = phi::es_transform(omega[i], beta);
    return PHI_OK;
}

phi_status phi_host_polar_nodes(const phi_params* p, double* kx, double* ky, double* q) {
    if (!p) return fail(nullptr, PHI_ERR_INVALID_ARG, "NULL params");
    try {
        phi::HostPlan hp;
        std::string err;
        phi_status st = phi::build_host_plan(p, &hp, &err);
        if (st != PHI_OK) return fail(nullptr, st, err);
        const size_t m = hp.n_nodes;
        if (kx) std::memcpy(kx, hp.kx.data(), m * sizeof(double));
        if (ky) std::memcpy(ky, hp.ky.data(), m * sizeof(double));
        if (q) std::memcpy(q, hp.q.data(), m * sizeof(double));
        return PHI_OK;
    } catch (...) {
        return fail(nullptr, PHI_ERR_INTERNAL, "unexpected exception");
    }
}

}  // extern "C"
