// Host-only driver of the plan construction code, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: builds plans
// over the supported range of sides, node counts, tolerances and node sorts and
// checks the structural invariants of the node tables.
#include <cstdio>
#include <string>

#include "plan_host.hpp"

int main() {
    int failures = 0;
    const int sides[] = {8, 16, 64, 256, 1024};
    const double tols[] = {1e-3, 1e-7, 1e-12};
    const int bins[] = {0, 4, 16};
    for (int n : sides) {
        for (double tol : tols) {
            for (int bin : bins) {
                phi_params p;
                phi::fill_defaults(&p, n, 16.0 / n, tol < 1e-7 ? PHI_F64 : PHI_F32);
                p.tol = tol;
                p.n_r = 16;
                p.n_theta = 32;
                p.bin = bin;
                p.sub_nodes = (bin == 16) ? 8 : 0;
                phi::HostPlan hp;
                std::string err;
                if (phi::build_host_plan(&p, &hp, &err) != PHI_OK) {
                    std::printf("plan n=%d tol=%g bin=%d failed: %s\n", n, tol, bin, err.c_str());
                    ++failures;
                    continue;
                }
                // every node in exactly one subproblem, in order; entries in range
                int next = 0;
                for (int s = 0; s < hp.n_sub; ++s) {
                    if (hp.sub[4 * s + 2] != next || hp.sub[4 * s + 3] < 1 || hp.sub[4 * s + 3] > hp.sub_nodes) ++failures;
                    next += hp.sub[4 * s + 3];
                }
                if (next != hp.n_nodes) ++failures;
                const long long tile_cells = static_cast<long long>(hp.n_sub) * hp.tile * hp.tile;
                for (int c : hp.contrib)
                    if (c < 0 || c >= tile_cells) ++failures;
                if (hp.contrib_start.back() != static_cast<int>(hp.contrib.size())) ++failures;
                std::vector<float> unit;
                phi::round_unit_pairs(hp.twr, &unit);
                if (unit.size() != hp.twr.size()) ++failures;
            }
        }
    }
    std::printf("%s (%d failures)\n", failures ? "FAIL" : "OK", failures);
    return failures ? 1 : 0;
}
