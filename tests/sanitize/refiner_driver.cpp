// Drives the library's host-side bisection refiner (ocp_refiner_*, compiled
// into this program from its source) on a small Kuhn mesh: several Doerfler
// refinements with a localised indicator, the size and array queries, and the
// argument checks, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer.  Exit status 0 when every call behaves.
#include <cmath>
#include <cstdio>
#include <vector>

#include "kuhn.h"
#include "ocpamg.h"

int main() {
    san_mesh m = san_kuhn(3, 0.0);
    ocp_refiner *r = nullptr;
    int bad = 0;
    bad |= ocp_refiner_create(m.xyz, (int32_t)m.nv, m.tets, (int32_t)m.nt, &r) != OCP_OK;
    for (int step = 0; step < 6 && !bad; ++step) {
        int32_t nv = 0, nt = 0;
        bad |= ocp_refiner_sizes(r, &nv, &nt) != OCP_OK;
        std::vector<double> xyz(3 * (size_t)nv);
        std::vector<int32_t> tets(4 * (size_t)nt);
        std::vector<uint8_t> dir((size_t)nv);
        bad |= ocp_refiner_get(r, xyz.data(), tets.data(), dir.data()) != OCP_OK;
        std::vector<double> eta2((size_t)nt);
        for (int32_t e = 0; e < nt; ++e) {
            double c[3] = {0, 0, 0};
            for (int a = 0; a < 4; ++a)
                for (int d = 0; d < 3; ++d) c[d] += 0.25 * xyz[3 * (size_t)tets[4 * (size_t)e + a] + d];
            const double q = (c[0] - 0.3) * (c[0] - 0.3) + (c[1] - 0.3) * (c[1] - 0.3) + (c[2] - 0.3) * (c[2] - 0.3);
            eta2[(size_t)e] = std::exp(-20.0 * q);
        }
        int32_t marked = 0;
        bad |= ocp_refiner_refine(r, eta2.data(), 0.5, &marked) != OCP_OK;
        bad |= marked <= 0;
        int32_t nv2 = 0, nt2 = 0;
        bad |= ocp_refiner_sizes(r, &nv2, &nt2) != OCP_OK;
        bad |= !(nt2 > nt && nv2 > nv);
        for (size_t e = 0; e < 4 * (size_t)nt && !bad; ++e) bad |= tets[e] < 0 || tets[e] >= nv;
    }
    // argument checks
    double eta_bad[1] = {-1.0};
    int32_t mk = 0;
    bad |= ocp_refiner_refine(r, nullptr, 0.5, &mk) != OCP_ERR_INVALID_ARG;
    bad |= ocp_refiner_refine(r, eta_bad, 0.0, &mk) != OCP_ERR_INVALID_ARG;
    ocp_refiner *r2 = nullptr;
    const int32_t badtet[4] = {0, 1, 2, 99};
    bad |= ocp_refiner_create(m.xyz, 4, badtet, 1, &r2) != OCP_ERR_BAD_MESH;
    bad |= r2 != nullptr;
    ocp_refiner_destroy(r);
    san_free(&m);
    std::printf(bad ? "refiner driver: FAILED\n" : "refiner driver: ok\n");
    return bad;
}
