// Host-only driver for the address and undefined-behaviour sanitizer build of
// the library's planning and reference-data code (plan.cpp, fe.cpp): builds
// the partition plan (Algorithm 3 Step 2, band numbering, owner tables), the
// Krylov strips, the reference-element tables, the exact nodal values and the
// source loads of one problem, and prints a few totals.  No device call.
//
// usage: host_sanitize_driver n_coarse refine nsx nsy overlap strip_width [cuts...]
// Prints "ok <ports> <conduits> <local_dofs> <max_bw> <strips> <checksum>" or
// "rejected <reason>" (exit 0 either way; a sanitizer finding aborts).
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "lp_internal.h"

int main(int argc, char **argv) {
    if (argc < 7) {
        std::fprintf(stderr, "usage: %s n_coarse refine nsx nsy overlap strip_width [cuts...]\n", argv[0]);
        return 2;
    }
    lp_mesh m{2, std::atoi(argv[1]), std::atoi(argv[2])};
    std::vector<int32_t> cuts;
    for (int i = 7; i < argc; ++i) cuts.push_back(std::atoi(argv[i]));
    lp_partition p{{std::atoi(argv[3]), std::atoi(argv[4])}, std::atoi(argv[5]), cuts.empty() ? nullptr : cuts.data()};
    const int width = std::atoi(argv[6]);
    lp::Plan P;
    std::string why;
    if (!lp::build_plan(m, p, P, why)) {
        std::printf("rejected %s\n", why.c_str());
        return 0;
    }
    int nstrip = 0;
    if (width > 0) {
        lp::Plan Q = P;
        if (lp::build_strips(Q, width, 2, 159, why)) nstrip = (int)Q.strip.size();
        else std::printf("strips rejected %s\n", why.c_str());
    }
    lp::RefData ref;
    lp::build_refdata(ref);
    std::vector<double> ex[6];
    lp::exact_spatial(P.Nh, ex);
    lp_params prm{};
    for (int i = 0; i < 3; ++i) { prm.phi[i] = 1.0; prm.C[i] = 1.0; prm.k[i] = 0.1 * (i + 1); }
    prm.mu_tilde = prm.sigma = prm.sigma_star = prm.rho = prm.alpha = prm.eta = 1.0;
    prm.nu = 0.5;
    prm.dt = 0.01;
    std::vector<double> ld[5][3];
    lp::source_loads(P.Nh, prm, ld);
    double sum = 0.0;
    for (int f = 0; f < 6; ++f)
        for (double v : ex[f]) sum += v;
    for (int f = 0; f < 5; ++f)
        for (int k = 0; k < 3; ++k)
            for (double v : ld[f][k]) sum += v;
    long long idx = 0;
    for (int32_t d : P.dof2) idx += d;
    for (int32_t d : P.dof1) idx += d;
    std::printf("ok %zu %zu %lld %d %d %.6e %lld\n", P.por.size(), P.ose.size(), (long long)P.local_dofs, (int)P.max_bw,
                nstrip, sum, idx);
    return 0;
}
