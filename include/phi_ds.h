/* Split-step time integration of the DS system on one GPU: the consumer of the
 * potential solve (include/phi_solve.h).
 *
 *   i u_t = -u_xx + alpha u_yy - 2 beta |u|^2 u - 4 beta Phi u,
 *   Phi_hat = -kx^2/|k|^2 rho_hat,  rho = |u|^2             (Sec. 1, eqs. 1-2)
 *
 * on the periodic box of the solve's grid (Sec. 2.3).  A step of length tau is a
 * composition of the exact flows of
 *   A: i v_t = (-d_xx + alpha d_yy) v, exact in Fourier space:
 *      v_hat <- v_hat e^{-i 4 pi^2 (kx^2 - alpha ky^2) s}, k = m/(N h);
 *   B: w = v e^{i s (c_l |v|^2 + c_p Phi[|v|^2])}, pointwise (Sec. 2.3),
 *      Phi from one potential solve of the stepper's own plan; c_l = 2 beta and
 *      c_p = 4 beta for eq. 1 (the E-E system of Sec. 3.3, i u_t = -(u_xx + u_yy)
 *      + chi |u|^2 u + gamma Phi u, has alpha = -1, c_l = -chi, c_p = -gamma):
 *   PHI_DS_STRANG    e^{A tau/2} e^{B tau} e^{A tau/2}            (1 solve per step)
 *   PHI_DS_YOSHIDA4  e^{A a1 tau} e^{B b1 tau} e^{A a2 tau} e^{B b2 tau}
 *                    e^{A a2 tau} e^{B b1 tau} e^{A a1 tau}, b1 = 1/(2 - 2^(1/3)),
 *                    b2 = -2^(1/3) b1, a1 = b1/2, a2 = (b1 + b2)/2 (3 solves per
 *                    step; the fourth-order composition of Sec. 2.3).
 * The last A of a step and the first A of the next are applied as one.
 * The potential solver is the split solver (phi_solve, PHI_DS_SPLIT) or the
 * standard periodic FFT solver (phi_solve_periodic, PHI_DS_PERIODIC).
 *
 * Fields are N x N complex arrays in device memory, row-major [y][x] with x
 * contiguous, interleaved (re, im) in the data precision of the solve
 * parameters (F32 -> complex64, F64 -> complex128).  Gradients of a real loss
 * J are fields g = dJ/dRe(u) + i dJ/dIm(u).  All calls only enqueue work on
 * `stream` (stream-ordered, asynchronous); one call in flight per stepper.
 * Errors are reported by status; the message is phi_last_error(NULL). */
#ifndef PHI_DS_H
#define PHI_DS_H

#include <stdint.h>

#include "phi_solve.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct phi_ds_s* phi_ds_t;

typedef enum { PHI_DS_STRANG = 0, PHI_DS_YOSHIDA4 = 1 } phi_ds_scheme;
typedef enum { PHI_DS_SPLIT = 0, PHI_DS_PERIODIC = 1 } phi_ds_potential;

typedef struct {
    double alpha;          /* coefficient of u_yy in eq. 1 (finite)              */
    double c_local;        /* phase coefficient of |u|^2: 2 beta for eq. 1       */
    double c_potential;    /* phase coefficient of Phi: 4 beta for eq. 1         */
    double tau;            /* time step (finite)                                 */
    int32_t scheme;        /* phi_ds_scheme                                 */
    int32_t potential;     /* phi_ds_potential                              */
} phi_ds_options;

/* Creates a stepper on the current device: a potential-solve plan for *solve
 * (grid side 16..4096, spacing, polar nodes, tolerance, dtype, flags), the
 * Fourier multipliers of the scheme's linear substeps (FP64, rounded to the
 * data precision) and a workspace of 2 complex and 2 real N x N fields. */
phi_status phi_ds_create(const phi_params* solve, const phi_ds_options* options, void* stream, phi_ds_t* out);

/* Nonlinear substeps (= potential solves) per step: 1 (Strang) or 3 (Yoshida). */
phi_status phi_ds_substeps(phi_ds_t ds, int32_t* per_step);

/* Frees the stepper and its plan after synchronizing its device.  NULL is a no-op. */
phi_status phi_ds_destroy(phi_ds_t ds);

/* The potential-solve plan the stepper owns (valid until phi_ds_destroy). */
phi_status phi_ds_plan(phi_ds_t ds, phi_plan_t* plan);

/* Advances u in place by `steps` (>= 0) steps.  v_store (may be NULL) receives
 * the input v_i of the i-th nonlinear substep (i = 0 .. steps * substeps - 1) at
 * element offset i N^2 (complex fields), phi_store (may be NULL) the potential
 * Phi_i of that substep at offset i N^2 (real fields): what phi_ds_backward
 * needs to run the reverse pass of the same steps.  One potential solve per
 * nonlinear substep. */
phi_status phi_ds_forward(phi_ds_t ds, void* u, int32_t steps, void* v_store, void* phi_store, void* stream);

/* Reverse pass of `steps` steps: g holds the gradient with respect to the
 * state after the steps and is overwritten with the gradient with respect to
 * the state before them.  v_store and phi_store are the stores a phi_ds_forward
 * of the same steps from that earlier state wrote (both required).  Each step
 * nonlinear substep of duration s takes one transposed potential solve
 * (phi_solve_adjoint; the periodic operator is symmetric): with
 * w = v e^{i phi}, phi = s (c_l |v|^2 + c_p Phi),
 *   g_v = g_w e^{-i phi} + 2 s (c_l q + c_p A^T q) v,  q = -Im(conj(g_w) w),
 * and the linear substeps run backwards in time (their adjoints). */
phi_status phi_ds_backward(phi_ds_t ds, void* g, int32_t steps, const void* v_store, const void* phi_store,
                           void* stream);

/* out[0] = h^2 sum |u|^2 (mass), out[1] = h^2 sum |u|^4; out: 2 doubles in device
 * memory, FP64 sums in a fixed order. */
phi_status phi_ds_moments(phi_ds_t ds, const void* u, double* out, void* stream);

/* g = 4 h^2 |u|^2 u: the gradient of J = h^2 sum |u|^4. */
phi_status phi_ds_loss_grad(phi_ds_t ds, const void* u, void* g, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* PHI_DS_H */
