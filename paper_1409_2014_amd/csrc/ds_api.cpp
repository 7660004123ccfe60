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
    int potential = PHI_DS_SPLIT;
    double tau = 0;
    // one step: e^{A lin[0]} e^{B non[0]} e^{A lin[1]} ... e^{B non[K-1]} e^{A lin[K]}
    // (durations in units of tau); the tables hold the distinct linear durations
    // first (lin[0]), interior, between steps (lin[K] + lin[0]) and last (lin[K])
    std::vector<double> non;         // K nonlinear durations
    std::vector<int> lin_inner_table;  // tables of lin[1 .. K-1]
    int lin_first_table = 0, lin_between_table = 0, lin_last_table = 0;
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

// The scheme's substep durations (fractions of tau).
void composition(int scheme, std::vector<double>* lin, std::vector<double>* non) {
    if (scheme == PHI_DS_YOSHIDA4) {
        const double b1 = 1.0 / (2.0 - std::cbrt(2.0));
        const double b2 = -std::cbrt(2.0) * b1;
        const double a1 = 0.5 * b1, a2 = 0.5 * (b1 + b2);
        *lin = {a1, a2, a2, a1};
        *non = {b1, b2, b1};
    } else {
        *lin = {0.5, 0.5};
        *non = {1.0};
    }
}

// Index of duration d in the table list (added when new).
int table_of(std::vector<double>* times, double d) {
    for (size_t i = 0; i < times->size(); ++i)
        if (std::fabs((*times)[i] - d) <= 1e-15 * std::fabs(d)) return static_cast<int>(i);
    times->push_back(d);
    return static_cast<int>(times->size()) - 1;
}

phi_status solve_potential(phi_ds_s* ds, const void* in, void* out, bool transpose, void* stream) {
    if (ds->potential == PHI_DS_PERIODIC) return phi_solve_periodic(ds->plan, in, out, stream);
    return transpose ? phi_solve_adjoint(ds->plan, in, out, stream) : phi_solve(ds->plan, in, out, stream);
}

// Linear-substep table after nonlinear substep k (0-based) of a run of
// `total` nonlinear substeps, K per step.
int table_after(const phi_ds_s* ds, int k, int total) {
    const int K = static_cast<int>(ds->non.size());
    const int j = k % K;
    if (j + 1 < K) return ds->lin_inner_table[j];
    return (k + 1 < total) ? ds->lin_between_table : ds->lin_last_table;
}

#define DS_TRY(expr, where)                               \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_err(e_, where);  \
    } while (0)

}  // namespace

extern "C" {

phi_status phi_ds_create(const phi_params* solve, const phi_ds_options* opt, void* stream, phi_ds_t* out) {
    if (!solve || !opt || !out) return err(PHI_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (!std::isfinite(opt->alpha) || !std::isfinite(opt->c_local) || !std::isfinite(opt->c_potential) ||
        !std::isfinite(opt->tau))
        return err(PHI_ERR_INVALID_ARG, "alpha, the phase coefficients and tau must be finite");
    if (opt->scheme != PHI_DS_STRANG && opt->scheme != PHI_DS_YOSHIDA4)
        return err(PHI_ERR_INVALID_ARG, "unknown scheme");
    if (opt->potential != PHI_DS_SPLIT && opt->potential != PHI_DS_PERIODIC)
        return err(PHI_ERR_INVALID_ARG, "unknown potential solver");
    if (solve->flags & (PHI_COMPONENT_COULOMB | PHI_PARTITION_GAUSS))
        return err(PHI_ERR_UNSUPPORTED, "the DS stepper takes the DS multiplier, not the Coulomb one");
    if (solve->nx < 16 || solve->nx > 4096 || (solve->nx & (solve->nx - 1)) != 0)
        return err(PHI_ERR_UNSUPPORTED, "the stepper takes power-of-two grid sides 16 .. 4096");
    try {
        std::unique_ptr<phi_ds_s> ds(new phi_ds_s());
        ds->potential = opt->potential;
        ds->tau = opt->tau;
        std::vector<double> lin;
        composition(opt->scheme, &lin, &ds->non);
        const int K = static_cast<int>(ds->non.size());
        std::vector<double> times;     // distinct linear durations, fractions of tau
        ds->lin_first_table = table_of(&times, lin[0]);
        for (int j = 1; j < K; ++j) ds->lin_inner_table.push_back(table_of(&times, lin[j]));
        ds->lin_between_table = table_of(&times, lin[K] + lin[0]);
        ds->lin_last_table = table_of(&times, lin[K]);
        if (static_cast<int>(times.size()) > phi::kDsMaxTimes) return err(PHI_ERR_INTERNAL, "too many substep durations");
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
        const int nt = static_cast<int>(times.size());
        std::vector<std::vector<double>> tabs;
        for (int i = 0; i < nt; ++i) tabs.push_back(multiplier(n, h, 1.0, times[i] * opt->tau, -1.0));
        for (int i = 0; i < nt; ++i) tabs.push_back(multiplier(n, h, opt->alpha, times[i] * opt->tau, 1.0));
        // layout: 2 nt multiplier tables, twiddles, partial sums, spec, work_c, work_r1, work_r2
        size_t off = 0;
        std::vector<size_t> o_tab(tabs.size());
        for (size_t i = 0; i < tabs.size(); ++i) {
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
        for (size_t i = 0; i < tabs.size() && e == hipSuccess; ++i)
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
        d.c_local = opt->c_local;
        d.c_potential = opt->c_potential;
        d.h2 = h * h;
        d.n_times = nt;
        for (int i = 0; i < nt; ++i) {
            d.ex[i] = base + o_tab[i];
            d.ey[i] = base + o_tab[nt + i];
        }
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

phi_status phi_ds_substeps(phi_ds_t ds, int32_t* per_step) {
    if (!is_live(ds) || !per_step) return err(PHI_ERR_INVALID_ARG, "NULL or destroyed stepper");
    *per_step = static_cast<int32_t>(ds->non.size());
    return PHI_OK;
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
    const int K = static_cast<int>(ds->non.size());
    const int total = steps * K;
    char* vs = static_cast<char*>(v_store);
    char* ps = static_cast<char*>(phi_store);
    // the first linear substep; then per nonlinear substep: complete the linear
    // substep (v_k, rho_k), Phi_k, the nonlinear substep fused into the next
    // linear substep (consecutive linear substeps of two steps merged)
    const int t0 = ds->lin_first_table;
    DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Plain, 0, t0, u, nullptr, nullptr, nullptr, nullptr, 0.0, s),
           "ds rows_forward");
    DS_TRY(phi::ds_cols(D, 0, t0, s), "ds cols");
    for (int k = 0; k < total; ++k) {
        const double ntau = ds->non[k % K] * ds->tau;
        void* v = vs ? static_cast<void*>(vs + static_cast<size_t>(k) * nn * 2 * ds->elem) : ds->work_c;
        void* pot = ps ? static_cast<void*>(ps + static_cast<size_t>(k) * nn * ds->elem) : ds->work_r2;
        DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Density, v, ds->work_r1, nullptr, nullptr, ntau, s),
               "ds rows_inverse");
        st = solve_potential(ds, ds->work_r1, pot, false, stream);
        if (st != PHI_OK) return st;
        const int tn = table_after(ds, k, total);
        DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Nonlinear, 0, tn, v, nullptr, pot, nullptr, nullptr, ntau, s),
               "ds rows_forward");
        DS_TRY(phi::ds_cols(D, 0, tn, s), "ds cols");
    }
    DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Field, u, nullptr, nullptr, nullptr, 0.0, s), "ds rows_inverse");
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
    const int K = static_cast<int>(ds->non.size());
    const int total = steps * K;
    const char* vs = static_cast<const char*>(v_store);
    const char* ps = static_cast<const char*>(phi_store);
    // adjoint of the last linear substep; then per nonlinear substep, last to
    // first: the gradient at its output and the source q, A^T q, the adjoint
    // update fused into the adjoint of the linear substep before it
    const int tl = ds->lin_last_table;
    DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Plain, 1, tl, g, nullptr, nullptr, nullptr, nullptr, 0.0, s),
           "ds rows_forward");
    DS_TRY(phi::ds_cols(D, 1, tl, s), "ds cols");
    for (int k = total - 1; k >= 0; --k) {
        const double ntau = ds->non[k % K] * ds->tau;
        const void* v = vs + static_cast<size_t>(k) * nn * 2 * ds->elem;
        const void* pot = ps + static_cast<size_t>(k) * nn * ds->elem;
        DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::AdjointSource, ds->work_c, ds->work_r1, v, pot, ntau, s),
               "ds rows_inverse");
        st = solve_potential(ds, ds->work_r1, ds->work_r2, true, stream);
        if (st != PHI_OK) return st;
        const int tp = (k > 0) ? table_after(ds, k - 1, total) : ds->lin_first_table;
        DS_TRY(phi::ds_rows_forward(D, phi::DsRowIn::Adjoint, 1, tp, ds->work_c, v, pot, ds->work_r1, ds->work_r2,
                                    ntau, s),
               "ds rows_forward");
        DS_TRY(phi::ds_cols(D, 1, tp, s), "ds cols");
    }
    DS_TRY(phi::ds_rows_inverse(D, phi::DsRowOut::Field, g, nullptr, nullptr, nullptr, 0.0, s), "ds rows_inverse");
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
