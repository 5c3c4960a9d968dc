// instances.cpp -- host-side calls of the C ABI that need no device:
// the +-J instance generator and the free-energy variance rho_f.
//
// pamc_make_pm_j draws the couplings of Sec. II.A (+-1 with probability 1/2
// each) from the library's own counter-based generator, Philox4x32-10 keyed
// by the disorder seed, so that a C caller reproduces any instance from
// (L, seed) alone.  pamc_rho_f evaluates Eq. (4), rho_f = R var(beta F),
// over independent runs of one instance.
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/pamc.h"

// Host code only (no HIP), so that it also builds with a plain C++ compiler
// (the sanitizer test does that).
namespace pamc {
void set_error(const std::string &msg);
}

namespace {

// Coupling stream tag, the top four bits of counter word 3 (1..4 are the
// initial spins, the sweeps, the resampling and the cluster moves).
constexpr uint32_t kTagCoupling = 0x50000000u;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), host form: ten rounds,
// each multiplying counter words 0 and 2 by the round multipliers (full
// 64-bit products), the high halves mixed with words 1 and 3 and the round
// key by XOR; the key advances by the Weyl constants after each round.
void philox_host(const uint32_t in[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t x = in[0], y = in[1], z = in[2], w = in[3];
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * x;
        const uint64_t b = (uint64_t)0xCD9E8D57u * z;
        const uint32_t nx = (uint32_t)(b >> 32) ^ y ^ k0;
        const uint32_t ny = (uint32_t)b;
        const uint32_t nz = (uint32_t)(a >> 32) ^ w ^ k1;
        const uint32_t nw = (uint32_t)a;
        x = nx;
        y = ny;
        z = nz;
        w = nw;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x;
    out[1] = y;
    out[2] = z;
    out[3] = w;
}

int invalid(const char *m)
{
    pamc::set_error(m);
    return PAMC_ERR_INVALID;
}

}  // namespace

extern "C" {

int pamc_make_pm_j(int L, uint64_t disorder_seed, int8_t *out)
{
    if (L < 2 || L > 32) return invalid("pamc_make_pm_j: L must be in [2, 32]");
    if (!out) return invalid("pamc_make_pm_j: out is NULL");
    const int64_t nb = 3 * (int64_t)L * L * L;  // bonds, b = d N + s
    const uint32_t k0 = (uint32_t)disorder_seed, k1 = (uint32_t)(disorder_seed >> 32);
    for (int64_t blk = 0; 4 * blk < nb; ++blk) {
        const uint32_t ctr[4] = {(uint32_t)blk, 0u, 0u, kTagCoupling};
        uint32_t v[4];
        philox_host(ctr, k0, k1, v);
        for (int j = 0; j < 4 && 4 * blk + j < nb; ++j) out[4 * blk + j] = (v[j] >> 31) ? 1 : -1;
    }
    return PAMC_OK;
}

int pamc_rho_f(const double *betaF, int runs, int n_temps, const double *nominal_R, double *mean_betaF,
               double *var_betaF, double *rho_f)
{
    if (!betaF || !nominal_R) return invalid("pamc_rho_f: NULL input");
    if (runs < 2) return invalid("pamc_rho_f: rho_f needs at least two independent runs");
    if (n_temps < 1) return invalid("pamc_rho_f: n_temps must be >= 1");
    for (int k = 0; k < n_temps; ++k) {
        // mean, then the sum of squared deviations from it, both in run order
        double s = 0.0;
        for (int i = 0; i < runs; ++i) s += betaF[(size_t)i * n_temps + k];
        const double m = s / (double)runs;
        double q = 0.0;
        for (int i = 0; i < runs; ++i) {
            const double d = betaF[(size_t)i * n_temps + k] - m;
            q += d * d;
        }
        const double v = q / (double)(runs - 1);
        if (mean_betaF) mean_betaF[k] = m;
        if (var_betaF) var_betaF[k] = v;
        if (rho_f) rho_f[k] = nominal_R[k] * v;
    }
    return PAMC_OK;
}

}  // extern "C"
