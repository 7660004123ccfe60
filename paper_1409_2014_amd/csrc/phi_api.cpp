// C ABI of the solver (declared in include/phi_solve.h): parameter checks,
// plan lifetime, device tables and workspace, and the stream-ordered entry
// points.  No C++ exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <vector>

#include "phi_solve.h"
#include "plan_host.hpp"
#include "solver_kernels.hpp"

struct phi_plan_s {
    phi::HostPlan host;
    phi::DevPlan dev;
    phi::StreamSet streams;     // side stream + fork/join events of the node-side chain
    phi_params params;
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

phi_status run(phi_plan_t plan, phi::Stage stage, const void* in, void* out, int adjoint, void* stream) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!in || !out) return fail(plan, PHI_ERR_INVALID_ARG, "NULL data pointer");
    if (in == out) return fail(plan, PHI_ERR_INVALID_ARG, "input and output must not alias");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return device_fail(plan, e, "hipGetDevice");
    if (cur != plan->device) {
        return fail(plan, PHI_ERR_INVALID_ARG, "current device differs from the plan's device");
    }
    e = phi::enqueue(plan->dev, plan->streams, stage, in, out, adjoint, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return device_fail(plan, e, "kernel launch");
    return PHI_OK;
}

}  // namespace

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
    phi_plan_s* plan = nullptr;
    try {
        plan = new phi_plan_s();
        std::string err;
        phi_status st = phi::build_host_plan(p, &plan->host, &err);
        if (st != PHI_OK) {
            delete plan;
            return fail(nullptr, st, err);
        }
        plan->params = *p;
        const phi::HostPlan& hp = plan->host;
        hipError_t e = hipGetDevice(&plan->device);
        if (e != hipSuccess) {
            delete plan;
            return device_fail(nullptr, e, "hipGetDevice");
        }
        const size_t es = (p->dtype == PHI_F32) ? 4 : 8;   // real element size
        const size_t n = hp.n, f = hp.n_fine, q = hp.patch, m = hp.n_nodes;
        // layout of the single allocation
        struct Part { size_t off, bytes; };
        size_t cursor = 0;
        auto take = [&](size_t bytes) { Part pt{cursor, bytes}; cursor = align256(cursor + bytes); return pt; };
        Part p_deconv = take(n * 8);
        Part p_gx = take(2 * (n + 1) * 8);
        Part p_gy = take(2 * f * 8);
        Part p_gyr = take(2 * f * es);
        Part p_q = take(m * 8);
        Part p_cell = take(hp.cell.size() * 4);
        Part p_sub = take(hp.sub.size() * 4);
        Part p_cst = take(hp.contrib_start.size() * 4);
        Part p_con = take(hp.contrib.size() * 4);
        Part p_taps = take(hp.taps.size() * es);
        Part p_twr = take(hp.twr.size() * es);
        Part p_xt = take((n + 1) * n * 2 * es);
        Part p_tt = take(q * n * 2 * es);
        Part p_win = take(q * q * 2 * es);
        Part p_pts = take(m * 2 * es);
        Part p_tiles = take(static_cast<size_t>(hp.n_sub) * hp.tile * hp.tile * 2 * es);
        Part p_u = take(n * q * 2 * es);
        plan->block_bytes = cursor;
        e = hipMalloc(&plan->block, cursor);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete plan;
            return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        char* base = static_cast<char*>(plan->block);
        hipStream_t s = static_cast<hipStream_t>(stream);
        auto up = [&](const Part& pt, const void* src) -> hipError_t {
            if (pt.bytes == 0) return hipSuccess;
            return hipMemcpyAsync(base + pt.off, src, pt.bytes, hipMemcpyHostToDevice, s);
        };
        // kernel taps and FFT twiddles are rounded once from FP64 to the data precision
        std::vector<float> taps32, twr32, gy32;
        if (p->dtype == PHI_F32) {
            gy32.assign(hp.gy.begin(), hp.gy.end());
            taps32.assign(hp.taps.begin(), hp.taps.end());
            twr32.assign(hp.twr.begin(), hp.twr.end());
        }
        const bool f32 = (p->dtype == PHI_F32);
        hipError_t ce = hipSuccess;
        if (ce == hipSuccess) ce = up(p_deconv, hp.deconv.data());
        if (ce == hipSuccess) ce = up(p_gx, hp.gx.data());
        if (ce == hipSuccess) ce = up(p_gy, hp.gy.data());
        if (ce == hipSuccess) ce = up(p_gyr, f32 ? static_cast<const void*>(gy32.data())
                                                 : static_cast<const void*>(hp.gy.data()));
        if (ce == hipSuccess) ce = up(p_q, hp.q.data());
        if (ce == hipSuccess) ce = up(p_cell, hp.cell.data());
        if (ce == hipSuccess) ce = up(p_sub, hp.sub.data());
        if (ce == hipSuccess) ce = up(p_cst, hp.contrib_start.data());
        if (ce == hipSuccess) ce = up(p_con, hp.contrib.data());
        if (ce == hipSuccess) ce = up(p_taps, f32 ? static_cast<const void*>(taps32.data())
                                                  : static_cast<const void*>(hp.taps.data()));
        if (ce == hipSuccess) ce = up(p_twr, f32 ? static_cast<const void*>(twr32.data())
                                                 : static_cast<const void*>(hp.twr.data()));
        if (ce == hipSuccess) ce = hipStreamSynchronize(s);
        // the node-side chain runs on a second stream of the plan's device, default priority
        if (ce == hipSuccess) ce = hipStreamCreateWithFlags(&plan->streams.side, hipStreamNonBlocking);
        if (ce == hipSuccess) ce = hipEventCreateWithFlags(&plan->streams.fork, hipEventDisableTiming);
        if (ce == hipSuccess) ce = hipEventCreateWithFlags(&plan->streams.join, hipEventDisableTiming);
        if (ce != hipSuccess) {
            if (plan->streams.join) (void)hipEventDestroy(plan->streams.join);
            if (plan->streams.fork) (void)hipEventDestroy(plan->streams.fork);
            if (plan->streams.side) (void)hipStreamDestroy(plan->streams.side);
            (void)hipFree(plan->block);
            delete plan;
            return device_fail(nullptr, ce, "plan setup");
        }
        phi::DevPlan& d = plan->dev;
        d.dtype = p->dtype;
        d.n = hp.n;
        d.n_fine = hp.n_fine;
        d.log_fine = hp.log_fine;
        d.patch = hp.patch;
        d.patch_lo = hp.patch_lo;
        d.width = hp.width;
        d.n_nodes = hp.n_nodes;
        d.component_y = hp.component_y;
        d.n_cu = 0;
        if (hipDeviceGetAttribute(&d.n_cu, hipDeviceAttributeMultiprocessorCount, plan->device) != hipSuccess ||
            d.n_cu < 1)
            d.n_cu = 1;
        d.h2 = hp.h * hp.h;
        d.inv_f2 = 1.0 / (static_cast<double>(f) * static_cast<double>(f));
        d.deconv = reinterpret_cast<const double*>(base + p_deconv.off);
        d.gx = reinterpret_cast<const double*>(base + p_gx.off);
        d.gy = reinterpret_cast<const double*>(base + p_gy.off);
        d.gyr = base + p_gyr.off;
        d.q = reinterpret_cast<const double*>(base + p_q.off);
        d.cell = reinterpret_cast<const int*>(base + p_cell.off);
        d.sub = reinterpret_cast<const int*>(base + p_sub.off);
        d.contrib_start = reinterpret_cast<const int*>(base + p_cst.off);
        d.contrib = reinterpret_cast<const int*>(base + p_con.off);
        d.n_sub = hp.n_sub;
        d.bin = hp.bin;
        d.tile = hp.tile;
        d.taps = base + p_taps.off;
        d.twr = base + p_twr.off;
        d.twr_count = static_cast<int>(hp.twr.size() / 2);
        d.xt = base + p_xt.off;
        d.tt = base + p_tt.off;
        d.win = base + p_win.off;
        d.pts = base + p_pts.off;
        d.tiles = base + p_tiles.off;
        d.u = base + p_u.off;
        {
            std::lock_guard<std::mutex> lock(g_registry_mutex);
            registry().insert(plan);
        }
        *out = plan;
        return PHI_OK;
    } catch (const std::bad_alloc&) {
        if (plan) {
            if (plan->block) (void)hipFree(plan->block);
            delete plan;
        }
        return fail(nullptr, PHI_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        if (plan) {
            if (plan->block) (void)hipFree(plan->block);
            delete plan;
        }
        return fail(nullptr, PHI_ERR_INTERNAL, "unexpected exception");
    }
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
    if (e == hipSuccess && plan->timer_ready) {
        for (int i = 0; i < 2 * phi::KernelTimer::kMax; ++i) (void)hipEventDestroy(plan->timer.ev[i]);
    }
    if (e == hipSuccess) {
        (void)hipEventDestroy(plan->streams.join);
        (void)hipEventDestroy(plan->streams.fork);
        (void)hipStreamDestroy(plan->streams.side);
    }
    if (e == hipSuccess) e = hipFree(plan->block);
    if (e != hipSuccess) st = fail(nullptr, PHI_ERR_DEVICE, std::string("phi_destroy: ") + hipGetErrorString(e));
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
    const size_t m = plan->host.n_nodes;
    if (kx) std::memcpy(kx, plan->host.kx.data(), m * sizeof(double));
    if (ky) std::memcpy(ky, plan->host.ky.data(), m * sizeof(double));
    if (q) std::memcpy(q, plan->host.q.data(), m * sizeof(double));
    return PHI_OK;
}

phi_status phi_solve(phi_plan_t plan, const void* rho, void* phi_out, void* stream) {
    return run(plan, phi::Stage::Solve, rho, phi_out, 0, stream);
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

phi_status phi_solve_timed(phi_plan_t plan, const void* in, void* out, int32_t adjoint, void* stream,
                           float* kernel_ms, const char** names, int32_t capacity, int32_t* count) {
    phi_status st = check_plan(plan);
    if (st != PHI_OK) return st;
    if (!in || !out || !count || (capacity > 0 && (!kernel_ms || !names)) || capacity < 0)
        return fail(plan, PHI_ERR_INVALID_ARG, "NULL or invalid argument");
    if (in == out) return fail(plan, PHI_ERR_INVALID_ARG, "input and output must not alias");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return device_fail(plan, e, "hipGetDevice");
    if (cur != plan->device) return fail(plan, PHI_ERR_INVALID_ARG, "current device differs from the plan's device");
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
    e = phi::enqueue(plan->dev, plan->streams, phi::Stage::Solve, in, out, adjoint ? 1 : 0, s, &t);
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
