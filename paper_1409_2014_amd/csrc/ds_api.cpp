// C ABI of the DS time stepper (declared in include/phi_ds.h): the Fourier
// multipliers of the linear substep, the workspace, and the orchestration of
// the split-step passes around the potential solves.
#include <hip/hip_runtime.h>

#include <cmath>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "api_errors.hpp"
#include "ds_kernels.hpp"
#include "phi_ds.h"
#include "phi_solve.h"
#include "plan_host.hpp"

struct phi_ds_s {
    phi_plan_t plan = nullptr;   // potential solve of the stepper's grid
    phi::DsDev dev{};
    int device = 0;
    int n = 0;
    size_t elem = 0;             // bytes of one real value
    void* block = nullptr;       // tables + workspace
    void* work_c = nullptr;      // N^2 complex: v or g_w
    void* work_r1 = nullptr;     // N^2 real: rho or s
    void* work_r2 = nullptr;     // N^2 real: Phi or A^T s
};

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

std::mutex g_ds_mutex;
std::set<phi_ds_t>& live() {
    static std::set<phi_ds_t> s;
    return s;
}

bool is_live(phi_ds_t ds) {
    std::lock_guard<std::mutex> lock(g_ds_mutex);
    return ds != nullptr && live().count(ds) != 0;
}

phi_status err(phi_status st, const std::string& msg) { return phi::thread_error(st, msg); }

phi_status hip_err(hipError_t e, const char* where) {
    return err(PHI_ERR_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

phi_status check(phi_ds_t ds) {
    if (!is_live(ds)) return err(PHI_ERR_INVALID_ARG, "stepper is NULL or was destroyed");
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_err(e, "hipGetDevice");
    if (cur != ds->device) return err(PHI_ERR_INVALID_ARG, "current device differs from the stepper's device");
    return PHI_OK;
}

size_t align256(size_t v) { return (v + 255) & ~static_cast<size_t>(255); }

// e^{i sign 4 pi^2 c k_m^2 s} for the N Fourier modes of the box in FFT order
// (k_m = m/(N h), m - N for m >= N/2), interleaved (re, im), FP64
std::vector<double> multiplier(int n, double h, double c, double s, double sign) {
    std::vector<double> out(2 * static_cast<size_t>(n));
    for (int m = 0; m < n; ++m) {
        const int ms = (m < n / 2) ? m : m - n;
        const double k = ms / (n * h);
        const double th = sign * 4.0 * kPi * kPi * c * k * k * s;
        out[2 * m] = std::cos(th);
        out[2 * m + 1] = std::sin(th);
    }
    return out;
}

void release(phi_ds_s* ds) {
    if (ds->block) (void)hipFree(ds->block);
    ds->block = nullptr;
    if (ds->plan) (void)phi_destroy(ds->plan);
    ds->plan = nullptr;
}

#define DS_TRY(expr, where)                               \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_err(e_, where);  \
    } while (0)

}  // namespace

extern "C" {

phi_status phi_ds_create(const phi_params* solve, double alpha, double beta, double tau, void* stream,
                         phi_ds_t* out) {
    if (!solve || !out) return err(PHI_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!std::isfinite(alpha) || !std::isfinite(beta) || !std::isfinite(tau))
        return err(PHI_ERR_INVALID_ARG, "alpha, beta and tau must be finite");
    if (solve->nx < 16 || solve->nx > 4096)
        return err(PHI_ERR_UNSUPPORTED, "the stepper takes grid sides 16 .. 4096");
    try {
        std::unique_ptr<phi_ds_s> ds(new phi_ds_s());
        phi_status st = phi_plan(solve, stream, &ds->plan);
        if (st != PHI_OK) return st;   // message already recorded
        phi_plan_info info;
        st = phi_plan_get_info(ds->plan, &info);
        if (st != PHI_OK) {
            release(ds.get());
            return st;
        }
        hipError_t e = hipGetDevice(&ds->device);
        if (e != hipSuccess) {
            release(ds.get());
            return hip_err(e, "hipGetDevice");
        }
        const int n = info.n;
        int log_n = 0;
        while ((1 << log_n) < n) ++log_n;
        const bool f32 = solve->dtype == PHI_F32;
        const size_t es = f32 ? 4 : 8;
        const size_t nn = static_cast<size_t>(n) * n;
        ds->n = n;
        ds->elem = es;
        std::vector<double> twr;
        phi::fft_stage_twiddles(log_n, &twr);
        const double h = info.h;
        std::vector<double> tabs[4] = {multiplier(n, h, 1.0, 0.5 * tau, -1.0), multiplier(n, h, 1.0, tau, -1.0),
                                       multiplier(n, h, alpha, 0.5 * tau, 1.0), multiplier(n, h, alpha, tau, 1.0)};
        // layout: 4 multiplier tables, twiddles, partial sums, spec, work_c, work_r1, work_r2
        size_t off = 0;
        size_t o_tab[4];
        for (int i = 0; i < 4; ++i) {
            o_tab[i] = off;
            off = align256(off + 2 * n * es);
        }
        const size_t o_twr = off;
        off = align256(off + twr.size() * es);
        const size_t o_part = off;
        off = align256(off + 2 * phi::kDsReduceBlocks * sizeof(double));
        const size_t o_spec = off;
        off = align256(off + 2 * nn * es);
        const size_t o_wc = off;
        off = align256(off + 2 * nn * es);
        const size_t o_r1 = off;
        off = align256(off + nn * es);
        const size_t o_r2 = off;
        off = align256(off + nn * es);
        e = hipMalloc(&ds->block, off);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ds->block = nullptr;
            release(ds.get());
            return err(PHI_ERR_OUT_OF_MEMORY, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        char* base = static_cast<char*>(ds->block);
        hipStream_t s = static_cast<hipStream_t>(stream);
        std::vector<std::vector<float>> keep;
        // every table here holds unit-modulus pairs
        auto narrow = [&](const std::vector<double>& v) -> const void* {
            if (!f32) return v.data();
            keep.emplace_back();
            phi::round_unit_pairs(v, &keep.back());
            return keep.back().data();
        };
        for (int i = 0; i < 4 && e == hipSuccess; ++i)
            e = hipMemcpyAsync(base + o_tab[i], narrow(tabs[i]), 2 * n * es, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && !twr.empty())
            e = hipMemcpyAsync(base + o_twr, narrow(twr), twr.size() * es, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            release(ds.get());
            return hip_err(e, "table upload");
        }
        phi::DsDev& d = ds->dev;
        d.dtype = solve->dtype;
        d.n = n;
        d.log_n = log_n;
        d.tau = tau;
        d.beta = beta;
        d.h2 = h * h;
        d.ex_half = base + o_tab[0];
        d.ex_full = base + o_tab[1];
        d.ey_half = base + o_tab[2];
        d.ey_full = base + o_tab[3];
        d.twr = base + o_twr;
        d.twr_count = static_cast<int>(twr.size() / 2);
        d.spec = base + o_spec;
        d.partials = reinterpret_cast<double*>(base + o_part);
        ds->work_c = base + o_wc;
        ds->work_r1 = base + o_r1;
        ds->work_r2 = base + o_r2;
        std::lock_guard<std::mutex> lock(g_ds_mutex);
        live().insert(ds.get());
        *out = ds.release();
        return PHI_OK;
    } catch (const std::bad_alloc&) {
        return err(PHI_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return err(PHI_ERR_INTERNAL, "unexpected exception");
    }
}

phi_status phi_ds_destroy(phi_ds_t ds) {
    if (!ds) return PHI_OK;
    {
        std::lock_guard<std::mutex> lock(g_ds_mutex);
        if (live().erase(ds) == 0) return err(PHI_ERR_INVALID_ARG, "stepper was already destroyed");
    }
    int prev = -1;
    (void)hipGetDevice(&prev);
    if (prev != ds->device) (void)hipSetDevice(ds->device);
    hipError_t e = hipDeviceSynchronize();
    release(ds);
    if (prev >= 0 && prev != ds->device) (void)hipSetDevice(prev);
    delete ds;
    if (e != hipSuccess) return hip_err(e, "phi_ds_destroy");
    return PHI_OK;
}

phi_status phi_ds_plan(phi_ds_t ds, phi_plan_t* plan) {
    if (!is_live(ds) || !plan) return err(PHI_ERR_INVALID_ARG, "NULL or destroyed stepper");
    *plan = ds->plan;
    return PHI_OK;
}

phi_status phi_ds_forward(phi_ds_t ds, void* u, int32_t steps, void* v_store, void* phi_store, void* stream) {
    phi_status st = check(ds);
    if (st != PHI_OK) return st;
    if (!u || steps < 0) return err(PHI_ERR_INVALID_ARG, "NULL field or negative step count");
    if (steps == 0) return PHI_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const phi::DsDev& D = ds->dev;
    const size_t nn = static_cast<size_t>(ds->n) * ds->n;
    char* vs = static_cast<char*>(v_store);
    char* ps = static_cast<char*>(phi_store);
    // e^{A tau/2}, then per step: complete the linear substep (v_i, rho_i), Phi_i,
    // the nonlinear substep fused into the next linear substep (a full step
    // between steps, a half step after the last)
    DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Plain, 0, 0, u, nullptr, nullptr, nullptr, nullptr, s),
           "ds rows_forward");
    DS_TRY(phi::ds_cols(D, 0, 0, s), "ds cols");
    for (int i = 0; i < steps; ++i) {
        void* v = vs ? static_cast<void*>(vs + i * nn * 2 * ds->elem) : ds->work_c;
        void* pot = ps ? static_cast<void*>(ps + i * nn * ds->elem) : ds->work_r2;
        DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Density, v, ds->work_r1, nullptr, nullptr, s),
               "ds rows_inverse");
        st = phi_solve(ds->plan, ds->work_r1, pot, stream);
        if (st != PHI_OK) return st;
        const int full = (i + 1 < steps) ? 1 : 0;
        DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Nonlinear, 0, full, v, nullptr, pot, nullptr, nullptr, s),
               "ds rows_forward");
        DS_TRY(phi::ds_cols(D, 0, full, s), "ds cols");
    }
    DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Field, u, nullptr, nullptr, nullptr, s), "ds rows_inverse");
    return PHI_OK;
}

phi_status phi_ds_backward(phi_ds_t ds, void* g, int32_t steps, const void* v_store, const void* phi_store,
                           void* stream) {
    phi_status st = check(ds);
    if (st != PHI_OK) return st;
    if (!g || steps < 0) return err(PHI_ERR_INVALID_ARG, "NULL gradient or negative step count");
    if (steps == 0) return PHI_OK;
    if (!v_store || !phi_store) return err(PHI_ERR_INVALID_ARG, "the reverse pass needs both stores");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const phi::DsDev& D = ds->dev;
    const size_t nn = static_cast<size_t>(ds->n) * ds->n;
    const char* vs = static_cast<const char*>(v_store);
    const char* ps = static_cast<const char*>(phi_store);
    // adjoint of the trailing e^{A tau/2}; then per step, last to first: the
    // gradient at the nonlinear substep's output and its source s, A^T s, the
    // adjoint nonlinear update fused into the adjoint of the preceding linear substep
    DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Plain, 1, 0, g, nullptr, nullptr, nullptr, nullptr, s),
           "ds rows_forward");
    DS_TRY(phi::ds_cols(D, 1, 0, s), "ds cols");
    for (int i = steps - 1; i >= 0; --i) {
        const void* v = vs + i * nn * 2 * ds->elem;
        const void* pot = ps + i * nn * ds->elem;
        DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::AdjointSource, ds->work_c, ds->work_r1, v, pot, s),
               "ds rows_inverse");
        st = phi_solve_adjoint(ds->plan, ds->work_r1, ds->work_r2, stream);
        if (st != PHI_OK) return st;
        const int full = (i > 0) ? 1 : 0;
        DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Adjoint, 1, full, ds->work_c, v, pot, ds->work_r1,
                                    ds->work_r2, s),
               "ds rows_forward");
        DS_TRY(phi::ds_cols(D, 1, full, s), "ds cols");
    }
    DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Field, g, nullptr, nullptr, nullptr, s), "ds rows_inverse");
    return PHI_OK;
}

phi_status phi_ds_moments(phi_ds_t ds, const void* u, double* out, void* stream) {
    phi_status st = check(ds);
    if (st != PHI_OK) return st;
    if (!u || !out) return err(PHI_ERR_INVALID_ARG, "NULL argument");
    DS_TRY(phi::ds_moments(ds->dev, u, out, static_cast<hipStream_t>(stream)), "ds moments");
    return PHI_OK;
}

phi_status phi_ds_loss_grad(phi_ds_t ds, const void* u, void* g, void* stream) {
    phi_status st = check(ds);
    if (st != PHI_OK) return st;
    if (!u || !g) return err(PHI_ERR_INVALID_ARG, "NULL argument");
    DS_TRY(phi::ds_loss_grad(ds->dev, u, g, static_cast<hipStream_t>(stream)), "ds loss gradient");
    return PHI_OK;
}

}  // extern "C"
