// Host-side (CPU, FP64) construction of a solve plan: parameter defaults and
// validation, the polar quadrature of Sec. 2.1 (eq. 12), the NUFFT kernel and
// its deconvolution factors, the I1 multiplier tables, FFT twiddles and the
// bin sort of the polar nodes.  No HIP calls: everything here runs and is
// tested without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "phi_solve.h"

namespace phi {

constexpr int kMaxLogFine = 13;        // padded / fine grid up to 8192 (N up to 4096 at kappa = 2)
constexpr int kMinLogFine = 4;         // padded / fine grid from 16
constexpr int kMinGrid = 8;            // smallest grid side
constexpr int kMaxPad = 8;             // largest padding factor kappa
constexpr int kMaxKernelWidth = 28;   // widest kernel: ES up to 16, the Gaussian up to 28
constexpr int kMaxEsWidth = 16;       // widest ES kernel (node blocks for it need less LDS)
constexpr int kMaxTile = 31;          // largest spread tile side bin + w - 1
constexpr int kBinSize = 4;            // default bin side in fine-grid cells (measured best or equal)
constexpr int kMaxBinSize = 16;        // largest bin side
constexpr int kMaxNodesPerSub = 64;    // most nodes per interp / spread subproblem

struct HostPlan {
    // problem
    int n = 0;            // grid side N (even)
    int n_fine = 0;       // FFT side F: the smallest power of two >= kappa N (padded I1 box
                          // and NUFFT fine grid, oversampling F / N >= 2)
    int log_fine = 0;
    int log_n = -1;       // log2 N when N is a power of two (the periodic solver), else -1
    int kappa = 2;        // requested padding factor
    int n_r = 0, n_theta = 0, n_nodes = 0;
    int component = 0;          // multiplier -k_a k_b/|k|^2: 0 (a,b) = (x,x), 1 (y,y), 2 (x,y); 3: 1/|k|
    int partition_erfc = 0;     // Coulomb with the partition erfc(|k|/sigma) (else the Gaussian)
    int radial_jacobi = 0;      // Gauss-Jacobi(0, 1) radial rule instead of Gauss-Legendre
    int two_streams = 0;        // node-side chain as separate launches on a second stream
    int gaussian_kernel = 0;    // Greengard-Lee Gaussian gridding instead of the ES kernel
    phi_dtype dtype = PHI_F64;
    double h = 0, half_width = 0, sigma = 0, cutoff = 0;
    // NUFFT kernel: phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| < 1, z = offset / (w/2);
    // with gaussian_kernel, psi(t) = exp(-beta t^2), t = offset in cells, |t| < w/2
    int width = 0;
    double beta = 0;
    // fine-grid window touched by the nodes' kernel taps: [patch_lo, patch_lo + patch)
    int patch = 0, patch_lo = 0;

    // node data in plan order: sorted by bin (bin x bin window cells) of the first kernel tap
    std::vector<double> kx, ky, q;      // k_j and q_j of eq. 12 (q without h^2)
    std::vector<int32_t> cell;          // [2 M] first-tap window cell (x, y), 0 <= c < patch
    std::vector<double> taps;           // [M][2][w] psi(u_j - l0_j - t), x then y
    int bin = 8, nb = 0;                // bin side in cells, bins per window side
    int sub_nodes = 64;                 // most nodes per subproblem
    int tile = 0;                       // spread tile side E = bin + w - 1
    std::vector<int32_t> sub;           // [4 n_sub] bin x, bin y, first node, node count (<= 64)
    int n_sub = 0;
    // reduction of the subproblem tiles onto the window: for window cell c = x * patch + y,
    // entries contrib_start[c] .. contrib_start[c+1]-1 of contrib hold flat tile indices
    std::vector<int32_t> contrib_start, contrib;
    int max_cell_nodes = 0;             // most nodes of one subproblem's bin
    int max_gather = 0;                 // most tile entries summed into one window cell
    // tables
    std::vector<double> deconv;         // [N] 2 pi / (n_fine psi_hat(n')), n' = i - N/2
    std::vector<double> gx;             // [2 (F/2+1)] (a, 1 - e^{-a}),  a = kx^2 / sigma^2, kx = m/(n_fine h)
    std::vector<double> gy;             // [2 n_fine] (b, 1 - e^{-b}), signed frequency
    std::vector<double> twr;            // (re, im) per-stage twiddles of the register FFT of length n_fine
    std::vector<double> twn;            // the same for length N (the periodic solver; N a power of two >= 16)
};

phi_status fill_defaults(phi_params* p, int32_t n, double h, phi_dtype dtype);
// Checks the parameters and derives the scalar quantities (no tables).
phi_status derive(const phi_params* p, HostPlan* hp, std::string* err);
// derive() plus every table.
phi_status build_host_plan(const phi_params* p, HostPlan* hp, std::string* err);

void gauss_legendre(int n, double* x, double* w);
// Gauss-Jacobi rule for the weight (1 + x) on [-1, 1], nodes ascending.
void gauss_jacobi01(int n, double* x, double* w);
// e^{-2 pi i m / n} with the angle reduced to the first octant (FP64).
void unit_root(long long m, long long n, double* re, double* im);
// Twiddles of the register-resident FFT of length 2^log (layout documented in
// fft_reg.hpp): stage s >= 1 of radix R and span p holds W_{pR}^{t k},
// t = 1..R-1, k = 0..p-1, at (t-1) p + k; stages back to back.
void fft_stage_twiddles(int log, std::vector<double>* out);
// FP32 copies of unit-modulus (re, im) pairs (twiddles, phase multipliers):
// each pair is taken among the floats within one ulp of its components such
// that re^2 + im^2 is closest to 1 (ties: the nearest pair), so rounding does
// not bias the modulus of long products of such factors.
void round_unit_pairs(const std::vector<double>& in, std::vector<float>* out);
double es_kernel(double z, double beta);
// int_{-1}^{1} phi(z) cos(omega z) dz
double es_transform(double omega, double beta);
// Polar nodes and weights in the natural (radial-major) order.
void polar_nodes(const HostPlan& hp, std::vector<double>* kx, std::vector<double>* ky,
                 std::vector<double>* q);

}  // namespace phi
