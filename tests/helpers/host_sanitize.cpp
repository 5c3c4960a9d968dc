// Drives the library's host-only calls (the +-J instance generator and the
// rho_f reduction, csrc/instances.cpp) with valid and invalid arguments, so
// that a build with AddressSanitizer and UndefinedBehaviorSanitizer checks
// them.  Links instances.cpp directly; set_error is provided here.
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/pamc.h"

namespace pamc {
static std::string g_err;
void set_error(const std::string &m) { g_err = m; }
}

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main()
{
    for (int L = 2; L <= 32; ++L) {
        std::vector<int8_t> J(3 * (size_t)L * L * L, 0);
        CHECK(pamc_make_pm_j(L, 0xFFFFFFFFFFFFFFFFull - (uint64_t)L, J.data()) == PAMC_OK);
        for (int8_t v : J) CHECK(v == 1 || v == -1);
    }
    std::vector<int8_t> small(3 * 8);
    CHECK(pamc_make_pm_j(1, 1, small.data()) == PAMC_ERR_INVALID);
    CHECK(pamc_make_pm_j(33, 1, small.data()) == PAMC_ERR_INVALID);
    CHECK(pamc_make_pm_j(2, 1, nullptr) == PAMC_ERR_INVALID);
    for (int runs = 2; runs <= 9; ++runs)
        for (int nT = 1; nT <= 5; ++nT) {
            std::vector<double> bf((size_t)runs * nT), R(nT, 1000.0), m(nT), v(nT), rf(nT);
            for (size_t i = 0; i < bf.size(); ++i) bf[i] = -50.0 + 0.01 * (double)(i % 7);
            CHECK(pamc_rho_f(bf.data(), runs, nT, R.data(), m.data(), v.data(), rf.data()) == PAMC_OK);
            for (int k = 0; k < nT; ++k) CHECK(v[k] >= 0.0 && std::isfinite(rf[k]));
            CHECK(pamc_rho_f(bf.data(), runs, nT, R.data(), nullptr, nullptr, nullptr) == PAMC_OK);
        }
    double one[3] = {0, 0, 0}, r3[3] = {1, 1, 1};
    CHECK(pamc_rho_f(one, 1, 3, r3, nullptr, nullptr, nullptr) == PAMC_ERR_INVALID);
    CHECK(pamc_rho_f(nullptr, 2, 3, r3, nullptr, nullptr, nullptr) == PAMC_ERR_INVALID);
    CHECK(pamc_rho_f(one, 2, 0, r3, nullptr, nullptr, nullptr) == PAMC_ERR_INVALID);
    std::printf("host sanitizer run ok\n");
    return 0;
}
