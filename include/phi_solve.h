/*
 * phi_solve.h -- C ABI of the MI355X (gfx950) solver for the nonlocal
 * Davey-Stewartson potential
 *
 *     Phi = F^-1[ -kx^2/|k|^2 rho_hat ],   rho_hat(k) = int rho e^{-2 pi i k.x} dx
 *
 * (Mauser, Stimming, Zhang, "A novel nonlocal potential solver based on
 * nonuniform FFT for efficient simulation of the Davey-Stewartson equations",
 * Sec. 1, eqs. 4-5), evaluated with the split of Sec. 2.1, eqs. 8-12:
 *
 *   I1  high-frequency part: trapezoidal rule on the zero-padded box, i.e. a
 *       padded 2-D FFT, the multiplier g1(k) = -(kx^2/|k|^2)(1 - e^{-|k|^2/sigma^2}),
 *       and the inverse FFT (Sec. 2.1, eq. 9);
 *   I2  low-frequency part: polar quadrature on the disk |k| <= c (radial
 *       Gauss-Legendre x azimuthal trapezoid, eq. 12), where rho_hat at the
 *       polar nodes is a type-2 NUFFT and the sum back onto the grid a type-1
 *       NUFFT (Sec. 2.2, eqs. 15-16).
 *
 * Conventions shared by every entry point
 *   - Grid: N x N points x_n = -L + n h, n = 0..N-1, L = N h / 2 (the periodic
 *     box [-L, L)^2; Sec. 3).  Arrays are row-major [iy][ix], x fastest,
 *     contiguous, element type fixed by the plan's dtype (double or float).
 *   - All array arguments of phi_solve* / phi_nodes_* are DEVICE pointers on
 *     the plan's device, owned by the caller; they must not alias each other.
 *   - Streams are passed as void* holding a hipStream_t (NULL = null stream).
 *     Solves only enqueue work on that stream: they are asynchronous,
 *     stream-ordered and never synchronize with the host.
 *   - A plan owns its tables and workspace.  One solve may be in flight per
 *     plan at a time (the workspace is shared): order solves on one stream, or
 *     use one plan per concurrent stream.
 *   - Errors are returned as phi_status; no C++ exception crosses the ABI.
 *     phi_last_error() gives a human-readable message for the last failure.
 */
#ifndef PHI_SOLVE_H
#define PHI_SOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phi_plan_s* phi_plan_t;

typedef enum {
    PHI_OK = 0,
    PHI_ERR_INVALID_ARG = 1,     /* NULL pointer, destroyed plan, bad size/spacing */
    PHI_ERR_UNSUPPORTED = 2,     /* valid for the paper, not implemented here     */
    PHI_ERR_TOL_UNREACHABLE = 3, /* NUFFT tolerance outside the dtype's range     */
    PHI_ERR_OUT_OF_MEMORY = 4,   /* device or host allocation failed              */
    PHI_ERR_DEVICE = 5,          /* a HIP call failed; see phi_last_error         */
    PHI_ERR_INTERNAL = 6
} phi_status;

typedef enum { PHI_F64 = 0, PHI_F32 = 1 } phi_dtype;

/* phi_params.flags */
#define PHI_COMPONENT_Y 1u   /* multiplier -ky^2/|k|^2 instead of -kx^2/|k|^2 (their sum is -1) */
#define PHI_COMPONENT_XY 8u  /* multiplier -kx ky/|k|^2: the mixed second derivative of the inverse
                                Laplacian, with -kx^2/|k|^2 and -ky^2/|k|^2 the whole tensor
                                -k_i k_j/|k|^2 (Sec. 2.1, Remark: the split needs only the
                                multiplier's values; this one is also bounded, even, and degree-0
                                homogeneous, so I1 stays smooth at k = 0).  Not with PHI_COMPONENT_Y. */
#define PHI_COMPONENT_COULOMB 64u /* multiplier 1/|k|: the 2-D Coulomb potential int rho(y)/|x - y| dy
                                (Sec. 2.1, Remark: the split applies to any multiplier whose
                                transform is known).  1/|k| cancels the polar Jacobian r, so
                                q_j = (c/2) w_i (2 pi/N_theta) p(r_i) with Gauss-Legendre radial
                                nodes (PHI_RADIAL_JACOBI is refused), and the I1 multiplier is
                                (1 - p(k))/|k|.  The partition is p = erfc(|k|/sigma) unless
                                PHI_PARTITION_GAUSS is set: both integrands are then smooth
                                (erf(r)/r is even and entire), and the solve reaches the NUFFT
                                tolerance.  Not with PHI_COMPONENT_Y / _XY; not in batches, the
                                periodic solver or the stepper (PHI_ERR_UNSUPPORTED). */
#define PHI_PARTITION_GAUSS 128u /* with PHI_COMPONENT_COULOMB: the paper's partition
                                p = e^{-|k|^2/sigma^2}, which leaves a cone |k|/sigma^2 in the I1
                                integrand at k = 0; the padded trapezoidal rule then resolves I1
                                only to about 3e-4 relative at L = 8 (falling like 1/L at the
                                default sigma).  Kept to reproduce that limit. */
#define PHI_RADIAL_JACOBI 4u /* radial rule Gauss-Jacobi(0, 1) on [0, c] (weight r built in; the rule
                                Sec. 2.1 names) instead of Gauss-Legendre with r in the weight */
#define PHI_KERNEL_GAUSSIAN 16u /* NUFFT spreading kernel: the truncated Gaussian of Greengard-Lee
                                gridding (the NUFFT Sec. 2.1 uses), psi(t) = exp(-(3 pi / (4 M)) t^2)
                                over w = 2M fine-grid cells, M = ceil(1.5 ln(1/tol) / pi), with the
                                Gaussian's Fourier transform as deconvolution, instead of the
                                exponential of semicircle.  Needs bin + w - 1 <= 31 (tol >= 5e-13
                                at bin 4); other cases return PHI_ERR_UNSUPPORTED. */
#define PHI_TWO_STREAMS 32u /* run the node-side chain as its own three launches on a second stream,
                                concurrently with the I1 column pass, also where a plan would
                                otherwise keep the solve on one stream: on padded sides up to 1024
                                (and 2048 in FP32) a solve by default runs cols_type2 and the node
                                subproblems in their own launches on the solve's stream, then the
                                type-1 window columns and every I1 column in one launch.  Results
                                are bit-identical in both layouts.
                                Larger sides and the Gaussian kernel above 16 cells always use
                                the two-stream layout. */
#define PHI_AUTOTUNE 2u      /* phi_plan / phi_plan_batch time the candidate bin sides {4, 8, 16} and
                                subproblem sizes {32, 64} on the device and keep the fastest; the
                                choice is visible in phi_plan_info.bin / .sub_nodes.  Results of
                                different choices differ by rounding only.  The candidates are timed
                                as eager whole solves; for solves replayed from a captured graph,
                                and for batches, the default (bin 4, 64 nodes) measured as fast or
                                faster on MI355X. */

/* Problem statement as the paper gives it (Sec. 2.1): the density on a uniform
 * box with spacing, the padding factor kappa, the partition width sigma and
 * disk radius c, the polar node counts and the NUFFT accuracy. */
typedef struct {
    int32_t nx, ny;        /* grid points per side; must be equal, even and >= 8 (Sec. 3); the
                              padded side F below must not exceed 8192                         */
    double hx, hy;         /* spacings; must be equal and > 0; box side = n h, centred at 0     */
    int32_t n_r;           /* radial Gauss-Legendre nodes, 1..1024                              */
    int32_t n_theta;       /* azimuthal trapezoid nodes, even, 2..4096                          */
    double tol;            /* NUFFT relative accuracy: F64 [1e-15, 1e-1], F32 [1e-7, 1e-1]      */
    int32_t pad;           /* zero-padding factor kappa of the I1 box, 2..8 (0: 2).  The padded
                              box (Sec. 2.1, kappa >= 2) has the side F = the smallest power of
                              two >= kappa N; F is also the NUFFT fine grid (oversampling F/N)  */
    double sigma;          /* partition width (<= 0: sqrt(ln 1e16) / (2 pi (F/N - 1) L), the
                              reading of Sec. 2.1 with the padding factor F/N of the box used) */
    double cutoff;         /* disk radius c   (<= 0: sqrt(ln 1e16) * sigma)                     */
    phi_dtype dtype;       /* data precision of rho / Phi; node and deconvolution tables are FP64 */
    uint32_t flags;        /* PHI_COMPONENT_Y, PHI_COMPONENT_XY or PHI_COMPONENT_COULOMB
                              (| PHI_PARTITION_GAUSS) | PHI_AUTOTUNE | PHI_RADIAL_JACOBI
                              | PHI_KERNEL_GAUSSIAN | PHI_TWO_STREAMS                              */
    int32_t bin;           /* bin side of the node sort in fine-grid cells: 4, 8 or 16 (0: 4)    */
    int32_t sub_nodes;     /* most nodes per spreading / interpolation block, 8..64 (0: 64)      */
} phi_params;

/* Derived quantities of a plan (filled by phi_describe / phi_plan_get_info). */
typedef struct {
    int32_t n;             /* grid side N                                        */
    int32_t n_fine;        /* FFT / fine-grid side F: smallest power of two >= kappa N */
    int32_t n_nodes;       /* M = n_r * n_theta                                  */
    int32_t kernel_width;  /* exponential-of-semicircle kernel width w (cells)   */
    int32_t patch;         /* side Q of the fine-grid window the nodes touch     */
    int32_t patch_lo;      /* lowest fine-grid index of that window (= -Q/2)     */
    int32_t max_cell_nodes;/* most nodes whose first kernel tap is one cell      */
    int32_t max_gather;    /* most tile entries summed into one window cell      */
    int32_t bin;           /* bin side of the node sort (cells)                  */
    int32_t tile;          /* spread tile side bin + w - 1                       */
    int32_t n_sub;         /* node blocks (runs of <= sub_nodes nodes of one bin) */
    int32_t sub_nodes;     /* most nodes per node block                          */
    double h, half_width, sigma, cutoff, beta;   /* beta: ES shape, or the Gaussian's 3 pi / (4 M) */
    size_t device_bytes;   /* tables + workspace allocated by phi_plan           */
    int64_t n_contrib;     /* tile entries summed onto the fine-grid window      */
} phi_plan_info;

/* Fill *p with defaults for an n x n grid of spacing h: 64 x 128 polar nodes,
 * kappa = 2, default sigma and c, tol 1e-12 (F64) or 1e-7 (F32). */
phi_status phi_params_default(phi_params* p, int32_t n, double h, phi_dtype dtype);

/* Validate *p and compute the derived quantities without touching a GPU. */
phi_status phi_describe(const phi_params* p, phi_plan_info* info);

/* Build a plan on the current HIP device: host-side FP64 tables (Gauss-Legendre
 * nodes, polar weights, kernel deconvolution factors, twiddles, multiplier
 * tables, bin sort) are computed and copied to device memory on `stream`.
 * This is the only host-to-device transfer; the copy is complete on return. */
phi_status phi_plan(const phi_params* p, void* stream, phi_plan_t* out);

/* Batch of independent solves (Sec. 2.1 applied to each member on its own box):
 * one plan for `count` members, each with its own parameters (grid side
 * with a padded side F of 256..4096, spacing, node counts, tolerance); all members share one dtype.
 * Members with equal parameters (field by field) share their device tables; every
 * member has its own workspace.  phi_solve / phi_solve_adjoint on a batch plan
 * take packed buffers: member i's N_i x N_i array starts at element offset
 * offsets[i] (phi_batch_layout).  Each stage of the chain is one launch over
 * all members.  The stage entry points (phi_solve_highfreq, phi_nodes_type2,
 * ...) and phi_plan_nodes return PHI_ERR_UNSUPPORTED on batch plans;
 * phi_plan_get_info describes member 0 and the plan's total device bytes. */
phi_status phi_plan_batch(const phi_params* members, int32_t count, void* stream, phi_plan_t* out);

/* Packed layout of a plan's input and output: *count = members (1 for a single
 * plan); offsets (may be NULL) receives count + 1 element offsets, member i
 * occupying [offsets[i], offsets[i+1]). */
phi_status phi_batch_layout(phi_plan_t plan, int32_t* count, int64_t* offsets);

/* Derived quantities of member `member` of a batch plan, as phi_plan_get_info
 * gives them for a single plan, except device_bytes = 0 (the batch's total is
 * in phi_plan_get_info).  On a single plan member 0 is the plan itself.
 * PHI_ERR_INVALID_ARG for a member index out of range. */
phi_status phi_batch_member_info(phi_plan_t plan, int32_t member, phi_plan_info* info);

/* Phi = A rho (Sec. 2.1, eq. 8: I1 + I2).  rho, phi: N x N device arrays. */
phi_status phi_solve(phi_plan_t plan, const void* rho, void* phi, void* stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): the same solve as
 * phi_solve, with the same kernels and the same results bit for bit, whose
 * workspace is a static device array of the library (80 MiB, one copy per
 * device, held until the process ends) instead of the plan's own.  It calls no
 * allocating routine; the plan itself is made beforehand by phi_plan.
 * rho, phi: N x N device arrays as for phi_solve (caller-owned).
 * Single plans only (PHI_ERR_UNSUPPORTED on a batch plan).  A plan whose
 * workspace exceeds the scratch (beyond N = 2048 at the default node counts)
 * returns PHI_ERR_UNSUPPORTED with the sizes in phi_last_error; nothing is
 * enqueued then.  Every call on one device shares that device's scratch and
 * leaves its contents behind: calls that overlap in time on one device (on
 * different streams, or from different threads) race and give wrong results;
 * order them on one stream. */
phi_status phi_solve_noalloc(phi_plan_t plan, const void* rho, void* phi, void* stream);

/* g_rho = A^T g_phi: the transposed chain (every transform direction reversed:
 * the grid-to-node NUFFT becomes the transpose of the node-to-grid one and vice
 * versa, the diagonal multipliers are their own transposes).  Used for the
 * gradient of a loss of Phi with respect to rho. */
phi_status phi_solve_adjoint(phi_plan_t plan, const void* g_phi, void* g_rho, void* stream);

/* Frees the plan's device memory after synchronizing its device.  NULL is a no-op. */
phi_status phi_destroy(phi_plan_t plan);

phi_status phi_plan_get_info(phi_plan_t plan, phi_plan_info* info);

/* Host copies (FP64, plan order, M entries) of the polar nodes k_j (in the
 * 2 pi convention of eq. 5) and the I2 weights q_j of eq. 12 (without h^2). */
phi_status phi_plan_nodes(phi_plan_t plan, double* kx, double* ky, double* q);

/* Type-2 stage alone (Sec. 2.2, eq. 16; the trapezoidal rule for eq. 5 at the
 * polar nodes): rho_hat[j] = h^2 sum_n rho_n e^{-2 pi i k_j.x_n}, j in plan
 * order.  rho: N x N device array; rho_hat: M interleaved (re, im) pairs. */
phi_status phi_nodes_type2(phi_plan_t plan, const void* rho, void* rho_hat, void* stream);

/* Type-1 stage alone (Sec. 2.2, eq. 15): field_n = Re sum_j coef_j e^{+2 pi i k_j.x_n}.
 * coef: M interleaved (re, im) pairs in plan order; field: N x N device array. */
phi_status phi_nodes_type1(phi_plan_t plan, const void* coef, void* field, void* stream);

/* The standard periodic FFT solver the paper compares against (Sec. 1; Sec. 3.1,
 * Tables 1 and 4): Phi_hat(k_m) = -kx^2/|k|^2 rho_hat(k_m) on the plan's N x N
 * periodic grid, k_m = m/(N h) in FFT order, Phi_hat(0) = 0 (-ky^2/|k|^2 with
 * PHI_COMPONENT_Y).  rho, phi: N x N device arrays as for phi_solve.  The
 * operator is symmetric, so it is also its own transpose.  Uses the plan's
 * workspace (one call in flight per plan, as phi_solve).  N = 16 .. 4096;
 * PHI_ERR_UNSUPPORTED for smaller grids and for batch plans. */
phi_status phi_solve_periodic(phi_plan_t plan, const void* rho, void* phi, void* stream);

/* I1 alone (Sec. 2.1, eq. 9) and I2 alone (eq. 12); phi_solve = their sum. */
phi_status phi_solve_highfreq(phi_plan_t plan, const void* rho, void* i1, void* stream);
phi_status phi_solve_lowfreq(phi_plan_t plan, const void* rho, void* i2, void* stream);

/* Measurement only: enqueues the same kernels as phi_solve (adjoint = 0) or
 * phi_solve_adjoint (adjoint = 1) with a HIP event recorded on `stream` before
 * each kernel and after the last, then waits for the stream.  Writes the
 * number of kernels to *count and, for i < min(*count, capacity), the i-th
 * kernel's duration in milliseconds to kernel_ms[i] and its name (a static
 * string owned by the library) to names[i].  Unlike phi_solve it blocks the
 * calling thread. */
phi_status phi_solve_timed(phi_plan_t plan, const void* in, void* out, int32_t adjoint, void* stream,
                           float* kernel_ms, const char** names, int32_t capacity, int32_t* count);

/* Host-only helpers used by the plan (exported for CPU tests). */
phi_status phi_host_gauss_legendre(int32_t n, double* x, double* w);
/* Gauss-Jacobi rule for int_{-1}^{1} f(x) (1 + x) dx, nodes ascending. */
phi_status phi_host_gauss_jacobi01(int32_t n, double* x, double* w);
/* Exponential-of-semicircle kernel phi(z) = exp(beta (sqrt(1 - z^2) - 1)), |z| < 1,
 * and its Fourier integral int_{-1}^{1} phi(z) cos(omega z) dz at omega[i]. */
phi_status phi_host_es_kernel(int32_t count, const double* z, double beta, double* out);
phi_status phi_host_es_transform(int32_t count, const double* omega, double beta, double* out);
/* Polar nodes and q_j exactly as phi_plan builds them (plan order, without h^2). */
phi_status phi_host_polar_nodes(const phi_params* p, double* kx, double* ky, double* q);

const char* phi_status_string(phi_status s);
/* Message of the last failure on this plan (plan != NULL) or of the last failure
 * in this thread (plan == NULL).  Valid until the next call on the same object. */
const char* phi_last_error(phi_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* PHI_SOLVE_H */
