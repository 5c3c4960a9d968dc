// pamc_api.cpp -- the extern "C" boundary declared in include/pamc.h.
// Argument validation, handle bookkeeping and status codes; the work is
// done by pamc::Runner and the gfx950 kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "runner.h"

namespace pamc {
const char *last_error_cstr();
}

using pamc::HostInst;
using pamc::Runner;

struct pamc_ctx {
    Runner run;
};

struct pamc_batch {
    Runner run;
    int n = 0;
};

namespace pamc {
int make_inst(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int nT, int NS,
              uint64_t seed, const pamc_options &opt, HostInst &h);
bool shape_valid(const HostInst &h, int tile_rows, int rp, const char **why);
void default_shape(HostInst &h, int gmax);
int tune_shape(HostInst &h, const pamc_options &opt, double *ns_per_attempt);
}

namespace {

int invalid(const std::string &m)
{
    pamc::set_error(m);
    return PAMC_ERR_INVALID;
}

}  // namespace

// Validates one instance and fills the host description.  Exactly one of J
// (+-1 couplings) and Jq (real couplings, units of 2^-20) is used: Jq when
// it is not NULL.
int pamc::make_inst(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int nT, int NS,
                    uint64_t seed, const pamc_options &opt, HostInst &h)
{
    const int dim = opt.dim == 0 ? 3 : opt.dim;
    if (dim != 2 && dim != 3) return invalid("dim must be 2 or 3");
    if (dim == 3 && (L < 2 || L > 32)) return invalid("L must be in [2, 32]");
    if (dim == 2 && (L < 2 || L > 64)) return invalid("square lattice: L must be in [2, 64]");
    if (!J && !Jq) return invalid("couplings is NULL");
    if (dim == 2 && !Jq) return invalid("the square lattice takes real couplings (+-J as +-2^20)");
    if (!beta) return invalid("beta is NULL");
    if (R < 1) return invalid("R must be >= 1");
    if (nT < 1) return invalid("n_temps must be >= 1");
    if (NS < 1) return invalid("sweeps must be >= 1");
    const int N = dim == 3 ? L * L * L : L * L;
    const bool real = Jq != nullptr;
    int64_t absJ = 0;  // sum of |j|: bounds |E| (units of 2^-20)
    if (real) {
        for (int i = 0; i < dim * N; ++i) {
            if (Jq[i] <= -(1 << 23) || Jq[i] >= (1 << 23)) return invalid("real couplings must satisfy |J| < 8");
            absJ += Jq[i] < 0 ? -(int64_t)Jq[i] : (int64_t)Jq[i];
        }
    } else {
        for (int i = 0; i < 3 * N; ++i)
            if (J[i] != 1 && J[i] != -1) return invalid("couplings must be +1 or -1");
    }
    // the initial replicas are independent random spins, the beta = 0
    // equilibrium, and ln Z is anchored there at N ln 2 (Sec. II.B)
    if (beta[0] != 0.0) return invalid("beta[0] must be 0 (random initial spins are the beta = 0 sample)");
    for (int k = 0; k < nT; ++k) {
        if (!std::isfinite(beta[k]) || beta[k] < 0.0) return invalid("beta must be finite and >= 0");
        if (k > 0 && beta[k] < beta[k - 1]) return invalid("beta must be non-decreasing");
    }
    int64_t peak = R;
    if (opt.pop_schedule) {
        if (opt.pop_schedule[0] != R) return invalid("pop_schedule[0] must equal R");
        for (int k = 0; k < nT; ++k) {
            if (opt.pop_schedule[k] < 1) return invalid("pop_schedule entries must be >= 1");
            peak = std::max(peak, (int64_t)opt.pop_schedule[k]);
        }
    }
    const int64_t cap = opt.capacity > 0 ? opt.capacity : pamc::default_capacity(peak);
    if (cap < R) return invalid("capacity must be >= R");
    if (cap >= ((int64_t)1 << 31) - 1024) return invalid("capacity must stay below 2^31");
    if (opt.spin_format != PAMC_SPINS_INT8 && opt.spin_format != PAMC_SPINS_PACKED)
        return invalid("unknown spin format");
    if (opt.icm_rounds < 0 || opt.icm_rounds > 8) return invalid("icm_rounds must be in [0, 8]");
    if (!std::isfinite(opt.icm_beta_min)) return invalid("icm_beta_min must be finite");
    if (opt.icm_rounds > 0 && opt.spin_format == PAMC_SPINS_PACKED)
        return invalid("cluster moves need int8 spin storage");
    if (real && (__int128)absJ * cap >= ((__int128)1 << 62))
        return invalid("capacity times the sum of |couplings| must stay below 2^62");
    // the normaliser's tree folds at most 2^19 roots of 1024-row blocks
    if (real && cap > ((int64_t)1 << 29)) return invalid("real couplings: capacity must stay at or below 2^29");
    const pamc::LayoutInfo li = pamc::layout_for(L, real, dim);
    if (li.layout < 0) return invalid("real couplings need even L <= 20 or odd L <= 21");
    h.dim = dim;
    h.L = L;
    h.N = N;
    h.ncol = li.ncol;
    h.layout = li.layout;
    h.variant = li.variant;
    h.row_bytes = li.row_bytes;
    h.packed = opt.spin_format == PAMC_SPINS_PACKED ? 1 : 0;
    h.srow_bytes = pamc::stored_row_bytes(li.row_bytes, h.packed != 0);
    h.tpr = li.tpr;
    h.R = R;
    h.Rcap = cap;
    h.nT = nT;
    h.NS = NS;
    h.seed = seed;
    h.beta.assign(beta, beta + nT);
    h.pop.assign((size_t)nT, (double)R);
    if (opt.pop_schedule)
        for (int k = 0; k < nT; ++k) h.pop[(size_t)k] = (double)opt.pop_schedule[k];
    h.real = real ? 1 : 0;
    h.icm = opt.icm_rounds;
    h.icm_bmin = opt.icm_beta_min;
    if (real)
        h.Jq.assign(Jq, Jq + (size_t)dim * N);
    else
        h.J.assign(J, J + 3 * N);
    h.ovl_slot.assign(nT, -1);
    h.ovl_n = 0;
    if (opt.overlap_steps && opt.n_overlap_steps > 0) {
        for (int j = 0; j < opt.n_overlap_steps; ++j) {
            const int k = opt.overlap_steps[j];
            if (k < 0 || k >= nT) return invalid("overlap step out of range");
            if (h.ovl_slot[k] < 0) h.ovl_slot[k] = h.ovl_n++;
        }
    } else {
        h.ovl_slot[nT - 1] = h.ovl_n++;
    }
    // sweep workgroup shape: explicit, tuned by measurement, or the default
    pamc::default_shape(h, li.gmax);
    if (opt.tile_rows < 0 || opt.tile_rows > 4096) return invalid("tile_rows out of range");
    if (opt.group_replicas < 0 || opt.group_replicas > 1024) return invalid("group_replicas out of range");
    const bool cm = h.variant == pamc::kSweepCM2 || h.variant == pamc::kSweepCM2T || h.variant == pamc::kSweepCM3 ||
                    h.variant == pamc::kSweepCM3T ||
                    h.variant == pamc::kSweepCQ2 || h.variant == pamc::kSweepCQ3 || h.variant == pamc::kSweepSQ2 ||
                    h.variant == pamc::kSweepSQ3;
    if (opt.tile_rows > 0 || (cm && opt.group_replicas > 0)) {
        // the colour-major kernel sweeps replicas in fours
        if (cm && opt.group_replicas % 4) return invalid("group_replicas must be a multiple of four for this lattice");
        const int rp = cm && opt.group_replicas > 0 ? opt.group_replicas / 4 : h.rp;
        // without an explicit tile: the default number of passes per workgroup
        int tr = opt.tile_rows > 0 ? opt.tile_rows : (cm ? h.tile_rows / h.rp * rp : h.tile_rows);
        // the even/odd-x kernel sweeps a fixed number of replicas per pass
        if (h.variant == pamc::kSweepEO8 || h.variant == pamc::kSweepEO16) {
            const int p = pamc::eo_replicas_per_pass(L);
            tr = (tr + p - 1) / p * p;
        }
        const char *why = nullptr;
        if (!pamc::shape_valid(h, tr, rp, &why)) return invalid(why);
        h.tile_rows = tr;
        h.rp = rp;
    } else if (opt.autotune) {
        const int st = pamc::tune_shape(h, opt, nullptr);
        if (st != PAMC_OK) return st;
    }
    return PAMC_OK;
}

namespace {

pamc_options resolve(const pamc_options *opt)
{
    pamc_options o;
    pamc_default_options(&o);
    if (opt) o = *opt;
    return o;
}

}  // namespace

extern "C" {

void pamc_default_options(pamc_options *opt)
{
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->spin_format = PAMC_SPINS_INT8;
    opt->fuse_gather = 1;
    opt->graphs = 1;
    opt->device = -1;
}

const char *pamc_status_string(int s)
{
    switch (s) {
    case PAMC_OK: return "ok";
    case PAMC_ERR_INVALID: return "invalid argument";
    case PAMC_ERR_NOMEM: return "out of memory";
    case PAMC_ERR_CAPACITY: return "population capacity exceeded";
    case PAMC_ERR_EXTINCT: return "population extinct";
    case PAMC_ERR_DEVICE: return "device error";
    case PAMC_ERR_STATE: return "invalid state for this call";
    case PAMC_ERR_BUSY: return "busy";
    case PAMC_ERR_REJECTED: return "rejected";
    default: return "unknown status";
    }
}

const char *pamc_last_error(void) { return pamc::last_error_cstr(); }

int64_t pamc_footprint(int L, int64_t R, int n_temps, const pamc_options *opt)
{
    const pamc_options o = resolve(opt);
    const int dim = o.dim == 0 ? 3 : o.dim;
    if ((dim != 2 && dim != 3) || L < 2 || L > (dim == 3 ? 32 : 64) || R < 1 || n_temps < 1) return -1;
    if ((o.real_couplings || dim == 2) && pamc::layout_for(L, true, dim).layout < 0) return -1;
    const bool real = o.real_couplings != 0 || dim == 2;
    const int64_t cap = o.capacity > 0 ? o.capacity : pamc::default_capacity(R);
    const int nov = (o.overlap_steps && o.n_overlap_steps > 0) ? o.n_overlap_steps : 1;
    if (o.capacity <= 0 && o.pop_schedule) {
        int64_t peak = R;
        for (int k = 0; k < n_temps; ++k) peak = std::max(peak, (int64_t)o.pop_schedule[k]);
        const int64_t c = pamc::default_capacity(peak);
        return (int64_t)pamc::inst_device_bytes(L, c, n_temps, nov, o.spin_format == PAMC_SPINS_PACKED, real,
                                                dim);
    }
    return (int64_t)pamc::inst_device_bytes(L, cap, n_temps, nov, o.spin_format == PAMC_SPINS_PACKED, real, dim);
}

}  // extern "C"

namespace {

int create_one(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int n_temps, int sweeps,
               uint64_t seed, const pamc_options *opt, pamc_ctx **out)
{
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    const pamc_options o = resolve(opt);
    std::vector<HostInst> v(1);
    int st = pamc::make_inst(L, J, Jq, R, beta, n_temps, sweeps, seed, o, v[0]);
    if (st != PAMC_OK) return st;
    std::unique_ptr<pamc_ctx> c(new (std::nothrow) pamc_ctx());
    if (!c) return PAMC_ERR_NOMEM;
    st = c->run.setup(o, 1);
    if (st != PAMC_OK) return st;
    const int slot = c->run.add_instance(std::move(v[0]));
    if (slot < 0) return slot;
    st = c->run.init_instances({slot});
    if (st != PAMC_OK) return st;
    st = c->run.build_work({slot});
    if (st != PAMC_OK) return st;
    *out = c.release();
    return PAMC_OK;
}

}  // namespace

extern "C" {

int pamc_create(int L, const int8_t *couplings, int64_t R, const double *beta, int n_temps, int sweeps,
                uint64_t seed, const pamc_options *opt, pamc_ctx **out)
{
    if (!couplings) {
        if (out) *out = nullptr;
        return invalid("couplings is NULL");
    }
    return create_one(L, couplings, nullptr, R, beta, n_temps, sweeps, seed, opt, out);
}

int pamc_create_real(int L, const int32_t *couplings, int64_t R, const double *beta, int n_temps, int sweeps,
                     uint64_t seed, const pamc_options *opt, pamc_ctx **out)
{
    if (!couplings) {
        if (out) *out = nullptr;
        return invalid("couplings is NULL");
    }
    return create_one(L, nullptr, couplings, R, beta, n_temps, sweeps, seed, opt, out);
}

int pamc_anneal_async(pamc_ctx *ctx, int n_steps)
{
    if (!ctx) return invalid("ctx is NULL");
    if (ctx->run.poisoned()) return PAMC_ERR_DEVICE;
    const int n = n_steps < 0 ? ctx->run.inst(0).nT : n_steps;
    return ctx->run.enqueue_steps(n);
}

int pamc_sync(pamc_ctx *ctx)
{
    if (!ctx) return invalid("ctx is NULL");
    int st = ctx->run.sync();
    if (st != PAMC_OK) return st;
    return ctx->run.inst_status(0, nullptr, nullptr);
}

int pamc_anneal(pamc_ctx *ctx, int n_steps)
{
    int st = pamc_anneal_async(ctx, n_steps);
    if (st != PAMC_OK) return st;
    return pamc_sync(ctx);
}

int pamc_observables(const pamc_ctx *ctx, pamc_step_obs *out, int n)
{
    if (!ctx || !out) return invalid("NULL argument");
    return const_cast<pamc_ctx *>(ctx)->run.observables(0, out, n);
}

int pamc_overlap_hist(const pamc_ctx *ctx, int step, int64_t *hist)
{
    if (!ctx || !hist) return invalid("NULL argument");
    return const_cast<pamc_ctx *>(ctx)->run.overlap_hist(0, step, hist);
}

int pamc_step_sums(const pamc_ctx *ctx, double *S, double *T, int n)
{
    if (!ctx) return invalid("ctx is NULL");
    return const_cast<pamc_ctx *>(ctx)->run.step_sums(0, S, T, n);
}

int pamc_sweep_shape(const pamc_ctx *ctx, int *tile_rows, int *group_replicas)
{
    if (!ctx) return invalid("ctx is NULL");
    const HostInst &h = ctx->run.inst(0);
    if (tile_rows) *tile_rows = h.tile_rows;
    if (group_replicas) *group_replicas = 4 * h.rp;
    return PAMC_OK;
}

int pamc_autotune(int L, int64_t R, int sweeps, const pamc_options *opt, int *tile_rows, int *group_replicas,
                  double *ns_per_attempt)
{
    pamc_options o = resolve(opt);
    const int dim = o.dim == 0 ? 3 : o.dim;
    if (dim != 2 && dim != 3) return invalid("dim must be 2 or 3");
    if (L < 2 || L > (dim == 3 ? 32 : 64)) return invalid("L out of range");
    o.tile_rows = 0;
    o.group_replicas = 0;
    o.autotune = 0;
    o.pop_schedule = nullptr;
    // seeded couplings (splitmix64): +-1, or real ones spread over
    // (-2, 2); the sweep's speed does not depend on their values
    const int N = dim == 3 ? L * L * L : L * L;
    std::vector<int8_t> J((size_t)dim * N);
    std::vector<int32_t> Jq(o.real_couplings || dim == 2 ? (size_t)dim * N : 0);
    uint64_t x = 0x2545F4914F6CDD1Dull;
    for (size_t i = 0; i < J.size(); ++i) {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        J[i] = (z >> 63) ? 1 : -1;
        if (!Jq.empty()) Jq[i] = (int32_t)(z >> 42) - (1 << 21);
    }
    const double beta[2] = {0.0, 0.5};
    HostInst h;
    int st = pamc::make_inst(L, J.data(), Jq.empty() ? nullptr : Jq.data(), R, beta, 2, sweeps, 1, o, h);
    if (st != PAMC_OK) return st;
    st = pamc::tune_shape(h, o, ns_per_attempt);
    if (st != PAMC_OK) return st;
    if (tile_rows) *tile_rows = h.tile_rows;
    if (group_replicas) *group_replicas = 4 * h.rp;
    return PAMC_OK;
}

int pamc_get_shape(const pamc_ctx *ctx, int *step, int64_t *R)
{
    if (!ctx) return invalid("ctx is NULL");
    Runner &r = const_cast<pamc_ctx *>(ctx)->run;
    int st = r.sync();
    if (st != PAMC_OK) return st;
    st = r.inst_status(0, step, R);
    // after a failed resampling the population is that of the failing step
    if (st == PAMC_ERR_CAPACITY || st == PAMC_ERR_EXTINCT) return PAMC_OK;
    return st;
}

int pamc_get_state(pamc_ctx *ctx, pamc_state *st)
{
    if (!ctx || !st) return invalid("NULL argument");
    return ctx->run.get_state(0, st);
}

int pamc_set_state(pamc_ctx *ctx, const pamc_state *st)
{
    if (!ctx || !st) return invalid("NULL argument");
    return ctx->run.set_state(0, st);
}

int pamc_thresholds(const pamc_ctx *ctx, uint32_t *out, uint8_t *accept_all)
{
    if (!ctx) return invalid("ctx is NULL");
    return const_cast<pamc_ctx *>(ctx)->run.thresholds(0, out, accept_all);
}

int pamc_phase_times(pamc_ctx *ctx, double *sweep_ms, double *resample_ms, double *gather_ms, int64_t *n_steps)
{
    if (!ctx) return invalid("ctx is NULL");
    return ctx->run.phase_times(sweep_ms, resample_ms, gather_ms, n_steps);
}

void pamc_destroy(pamc_ctx *ctx) { delete ctx; }

// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kGroupShapeRows = 200000;  // population batch shapes are tuned for (at most)
}

int pamc_batch_create(int n, const pamc_instance *inst, const pamc_options *opt, pamc_batch **out)
{
    if (!out) return invalid("out is NULL");
    *out = nullptr;
    if (n < 1 || !inst) return invalid("need at least one instance");
    const pamc_options o = resolve(opt);
    // Instances of one lattice (and kernel) sweep as one launch per step:
    // with autotuning and no explicit shape, that launch's shape is the one
    // tuned for the group's population (up to kGroupShapeRows rows), not
    // for each instance alone, whose own tuning favours small tiles to fill
    // the chip by itself.
    const bool group_tune = o.autotune && o.tile_rows == 0 && o.group_replicas == 0;
    std::vector<HostInst> v((size_t)n);
    for (int i = 0; i < n; ++i) {
        const pamc_instance &p = inst[i];
        pamc_options oi = o;
        oi.pop_schedule = p.pop_schedule;
        if (group_tune) oi.autotune = 0;
        int st = pamc::make_inst(p.L, p.real_couplings ? nullptr : p.couplings, p.real_couplings, p.R, p.beta,
                                 p.n_temps, p.sweeps, p.seed, oi, v[(size_t)i]);
        if (st != PAMC_OK) {
            pamc::set_error("instance " + std::to_string(i) + ": " + pamc_last_error());
            return st;
        }
    }
    if (group_tune) {
        using GKey = std::tuple<int, int, int, int, int>;  // variant, dim, L, sweeps, packed
        auto gkey = [](const HostInst &h) { return GKey(h.variant, h.dim, h.L, h.NS, h.packed); };
        std::map<GKey, int64_t> rows;
        for (const HostInst &h : v) rows[gkey(h)] += h.R;
        std::map<GKey, std::pair<int, int>> shape;
        for (auto &kv : rows) {
            HostInst t;
            for (const HostInst &h : v)
                if (gkey(h) == kv.first) {
                    t = h;
                    break;
                }
            t.R = std::min<int64_t>(kv.second, kGroupShapeRows);
            t.Rcap = pamc::default_capacity(t.R);
            const int st = pamc::tune_shape(t, o, nullptr);
            if (st != PAMC_OK) return st;
            shape[kv.first] = {t.tile_rows, t.rp};
        }
        for (HostInst &h : v) {
            const auto s = shape[gkey(h)];
            if (pamc::shape_valid(h, s.first, s.second, nullptr)) {
                h.tile_rows = s.first;
                h.rp = s.second;
            }
        }
    }
    std::unique_ptr<pamc_batch> b(new (std::nothrow) pamc_batch());
    if (!b) return PAMC_ERR_NOMEM;
    int st = b->run.setup(o, n);
    if (st != PAMC_OK) return st;
    std::vector<int> slots;
    for (int i = 0; i < n; ++i) {
        const int slot = b->run.add_instance(std::move(v[(size_t)i]));
        if (slot < 0) return slot;
        slots.push_back(slot);
    }
    st = b->run.init_instances(slots);
    if (st != PAMC_OK) return st;
    st = b->run.build_work(slots);
    if (st != PAMC_OK) return st;
    b->n = n;
    *out = b.release();
    return PAMC_OK;
}

int pamc_batch_anneal(pamc_batch *b)
{
    if (!b) return invalid("batch is NULL");
    int maxT = 0;
    for (int i = 0; i < b->n; ++i) maxT = std::max(maxT, b->run.inst(i).nT);
    int st = b->run.enqueue_steps(maxT);
    if (st != PAMC_OK) return st;
    st = b->run.sync();
    if (st != PAMC_OK) return st;
    int worst = PAMC_OK;
    for (int i = 0; i < b->n; ++i) {
        const int s = b->run.inst_status(i, nullptr, nullptr);
        if (s != PAMC_OK) worst = s;
    }
    return worst;
}

int pamc_batch_observables(const pamc_batch *b, int i, pamc_step_obs *out, int n)
{
    if (!b || !out) return invalid("NULL argument");
    if (i < 0 || i >= b->n) return invalid("instance index out of range");
    return const_cast<pamc_batch *>(b)->run.observables(i, out, n);
}

int pamc_batch_get_state(pamc_batch *b, int i, pamc_state *st)
{
    if (!b || !st) return invalid("NULL argument");
    if (i < 0 || i >= b->n) return invalid("instance index out of range");
    return b->run.get_state(i, st);
}

int pamc_batch_shape(const pamc_batch *b, int i, int *step, int64_t *R)
{
    if (!b) return invalid("batch is NULL");
    if (i < 0 || i >= b->n) return invalid("instance index out of range");
    Runner &r = const_cast<pamc_batch *>(b)->run;
    int st = r.inst_status(i, step, R);
    if (st == PAMC_ERR_CAPACITY || st == PAMC_ERR_EXTINCT) return PAMC_OK;
    return st;
}

void pamc_batch_destroy(pamc_batch *b) { delete b; }

}  // extern "C"
