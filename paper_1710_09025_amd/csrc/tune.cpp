// tune.cpp -- sweep workgroup shapes chosen by measurement.
//
// How fast the sweep runs depends on how many replica rows one workgroup
// holds (tile_rows) and, for the colour-major kernel, on how many replica
// quads it sweeps at once: a small population needs small
// tiles to spread over the 256 compute units, a large one amortises the tile
// load, the energy epilogue and the measurement tail over more rows.  The
// tuner runs each candidate shape on a throw-away run of the instance (its
// couplings, L, R, capacity and sweeps per step) at a constant beta = 2
// after the beta = 0 start, where every replica gets one copy on average
// and the population stays near R, and keeps the shape whose fastest timed
// step (HIP events, after a warm-up step) is shortest; a burn-in first
// brings the energies to that temperature.
// Every shape gives bit-identical results, so the choice only affects
// speed.  Choices are cached for the life of the process, keyed by device
// (architecture and compute units), kernel, lattice (dimension and L),
// sweeps per step, the capacity rounded up to a power of two and the spin
// storage format; the cache starts from the file tune_cache.jsonl beside
// the library and from the file PAMC_TUNE_CACHE names, and new choices are
// appended to the latter, so a later process finds them.
#include <dlfcn.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "runner.h"

namespace pamc {

int make_inst(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int nT, int NS,
              uint64_t seed, const pamc_options &opt, HostInst &h);

namespace {

constexpr int64_t kMaxLds = kMaxSweepLds;  // dynamic LDS of one sweep workgroup
constexpr int kTimedSteps = 3;      // timed steps per candidate shape (after one warm-up)
constexpr int kBurnIn = 8;          // steps before the first candidate
constexpr double kTuneBeta = 2.0;   // inside the low-temperature part where an anneal spends most steps

bool is_cm(const HostInst &h)
{
    return h.variant == kSweepCM2 || h.variant == kSweepCM2T || h.variant == kSweepCM3 || h.variant == kSweepCM3T ||
           h.variant == kSweepCQ2 || h.variant == kSweepCQ3 || h.variant == kSweepSQ2 || h.variant == kSweepSQ3;
}
bool is_cq(const HostInst &h)
{
    return h.variant == kSweepCQ2 || h.variant == kSweepCQ3 || h.variant == kSweepSQ2 || h.variant == kSweepSQ3;
}
bool is_eo(const HostInst &h) { return h.variant == kSweepEO8 || h.variant == kSweepEO16; }

int64_t sweep_lds(const HostInst &h, int tile_rows, int rp)
{
    if (is_cq(h)) return (int64_t)cm_slot_bytes(h.row_bytes, h.tpr, 4) * rp + 32 + 8 * (int64_t)tile_rows;
    if (is_cm(h))
        return (int64_t)cm_slot_bytes(h.row_bytes, h.tpr, 8) * rp + 32 + 4 * (int64_t)tile_rows +
               cm_table_bytes(h.variant, h.tpr);
    return (int64_t)tile_rows * h.row_bytes + 32 + 4 * (int64_t)tile_rows;
}

struct Choice {
    int tile_rows, rp;
    double ns_per_attempt;
};

using Key = std::tuple<int, int, int, int, int, int>;  // variant, dim, L, sweeps, log2 capacity, packed

std::mutex g_mu;
std::map<std::pair<std::string, Key>, Choice> g_cache;  // by device and key
bool g_loaded = false;
std::string g_save_path;  // where new choices are appended ("" = nowhere)

// The device a choice was measured on: architecture and compute units.
std::string device_tag()
{
    int dev = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    std::string arch = p.gcnArchName;
    const size_t c = arch.find(':');
    if (c != std::string::npos) arch.resize(c);
    return arch + "-" + std::to_string(p.multiProcessorCount) + "cu";
}

// One choice per line, as a JSON object with these fields in this order
// (read with kLineFmt, written with kLineOut).
#define PAMC_TUNE_LINE(DEV, NS)                                                                     \
    "{\"device\": \"" DEV "\", \"variant\": %d, \"dim\": %d, \"L\": %d, \"sweeps\": %d, "  \
    "\"cap_log2\": %d, \"packed\": %d, \"tile_rows\": %d, \"group_quads\": %d, "               \
    "\"ns_per_attempt\": " NS "}"
const char *kLineFmt = PAMC_TUNE_LINE("%63[^\"]", "%lf");
const char *kLineOut = PAMC_TUNE_LINE("%s", "%.6e");
#undef PAMC_TUNE_LINE

void load_file(const std::string &path)
{
    FILE *f = std::fopen(path.c_str(), "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof line, f)) {
        char dev[64];
        int v, d, L, ns, cl, pk, tr, rp;
        double npa;
        if (std::sscanf(line, kLineFmt, dev, &v, &d, &L, &ns, &cl, &pk, &tr, &rp, &npa) != 10) continue;
        g_cache[{dev, Key(v, d, L, ns, cl, pk)}] = Choice{tr, rp, npa};
    }
    std::fclose(f);
}

// The tuning cache file shipped beside the library (choices measured on
// MI355X for common sizes), then PAMC_TUNE_CACHE when it names a file;
// new choices are appended to PAMC_TUNE_CACHE.  Call with g_mu held.
void load_persistent()
{
    if (g_loaded) return;
    g_loaded = true;
    Dl_info info;
    if (dladdr((void *)&load_persistent, &info) && info.dli_fname) {
        std::string dir = info.dli_fname;
        const size_t sl = dir.rfind('/');
        dir = sl == std::string::npos ? std::string(".") : dir.substr(0, sl);
        load_file(dir + "/tune_cache.jsonl");
    }
    const char *env = std::getenv("PAMC_TUNE_CACHE");
    if (env && *env) {
        g_save_path = env;
        load_file(g_save_path);
    }
}

void save_choice(const std::string &dev, const Key &k, const Choice &c)
{
    if (g_save_path.empty()) return;
    FILE *f = std::fopen(g_save_path.c_str(), "a");
    if (!f) return;
    std::fprintf(f, kLineOut, dev.c_str(), std::get<0>(k), std::get<1>(k), std::get<2>(k), std::get<3>(k),
                 std::get<4>(k), std::get<5>(k), c.tile_rows, c.rp, c.ns_per_attempt);
    std::fputc('\n', f);
    std::fclose(f);
}

int ceil_log2(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << b) < v) ++b;
    return b;
}

}  // namespace

// Whether (tile_rows, rp) is a shape the instance's sweep kernel can run;
// on failure *why says what is wrong.
bool shape_valid(const HostInst &h, int tile_rows, int rp, const char **why)
{
    const char *w = nullptr;
    if (tile_rows < 1 || tile_rows > 4096) {
        w = "tile_rows must be in [1, 4096]";
    } else if (is_eo(h) && tile_rows % eo_replicas_per_pass(h.L) != 0) {
        w = "tile_rows must be a multiple of the replicas one pass sweeps";
    } else if (is_cm(h) && (rp < 1 || (h.tpr <= 64 && (h.tpr * rp) % 64 != 0) ||
                            cm_launch_threads(h.tpr, rp) > 1024)) {
        w = "group_replicas must be a multiple of four giving at most 1024 threads (whole waves when a quad "
            "takes at most 64)";
    } else if (sweep_lds(h, tile_rows, is_cm(h) ? rp : 0) > kMaxLds) {
        w = "the workgroup's tile does not fit in LDS";
    }
    if (why) *why = w;
    return w == nullptr;
}

// The shape used without tuning: enough workgroups to fill the chip when
// the population is small, up to four passes per workgroup when it is
// large.  gmax: Philox blocks of the largest colour.
void default_shape(HostInst &h, int gmax)
{
    const int64_t target = 512;  // workgroups: two per compute unit
    if (is_eo(h)) {
        const int rp = eo_replicas_per_pass(h.L);
        const int64_t m = std::max<int64_t>(1, std::min<int64_t>(4, h.Rcap / (target * rp)));
        h.tile_rows = (int)(m * rp);
        h.rp = 0;
    } else if (is_cm(h)) {
        h.rp = cm_replicas_per_block(h.tpr);
        const int64_t m = std::max<int64_t>(1, std::min<int64_t>(4, h.Rcap / (target * 4 * h.rp)));
        h.tile_rows = (int)(m * 4 * h.rp);
    } else {
        // per-site kernel: about 512 Philox blocks of work per workgroup
        int tr = (512 + gmax - 1) / gmax;
        tr = std::min(tr, std::max(1, 16384 / h.row_bytes));
        h.tile_rows = std::max(1, tr);
        h.rp = 0;
    }
}

std::vector<std::pair<int, int>> shape_candidates(const HostInst &h)
{
    std::vector<std::pair<int, int>> c;
    // tile sizes between the powers of two matter: the number of tiles
    // against the number of resident workgroups decides how full the last
    // round of workgroups is
    if (is_eo(h)) {
        const int rp = eo_replicas_per_pass(h.L);
        for (int m = 1; m <= 16; ++m)
            if (shape_valid(h, m * rp, 0, nullptr) && m * rp <= 2 * h.Rcap) c.emplace_back(m * rp, 0);
    } else if (is_cm(h)) {
        static const int kPasses[] = {1, 2, 3, 4, 6, 8};
        // quads of up to 64 threads: groups of whole waves; wider quads: any
        // count whose last wave is at least 80% used
        for (int rp = 1; cm_launch_threads(h.tpr, rp) <= 1024; rp = h.tpr <= 64 ? 2 * rp : rp + 1) {
            if (h.tpr <= 64 && (h.tpr * rp) % 64 != 0) continue;
            if (h.tpr > 64 && rp > 1 && 5 * h.tpr * rp < 4 * cm_launch_threads(h.tpr, rp)) continue;
            for (int m : kPasses)
                if (shape_valid(h, 4 * m * rp, rp, nullptr) && 4 * m * rp <= 2 * h.Rcap)
                    c.emplace_back(4 * m * rp, rp);
        }
    } else {
        for (int t = 1; t <= 4096; t *= 2)
            if (shape_valid(h, t, 0, nullptr) && t <= 2 * h.Rcap) c.emplace_back(t, 0);
    }
    return c;
}

int tune_shape(HostInst &h, const pamc_options &opt, double *ns_per_attempt)
{
    const Key k0(h.variant, h.dim, h.L, h.NS, ceil_log2(h.Rcap), h.packed);
    const auto key = std::make_pair(device_tag(), k0);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        load_persistent();
        auto it = g_cache.find(key);
        if (it != g_cache.end() && shape_valid(h, it->second.tile_rows, it->second.rp, nullptr)) {
            h.tile_rows = it->second.tile_rows;
            h.rp = it->second.rp;
            if (ns_per_attempt) *ns_per_attempt = it->second.ns_per_attempt;
            return PAMC_OK;
        }
    }
    const auto cand = shape_candidates(h);
    if (cand.empty()) {
        set_error("no valid sweep shape for this lattice");
        return PAMC_ERR_INVALID;
    }
    // throw-away run at a constant beta: a burn-in that brings the energies
    // to that temperature (the epilogue's cost depends on how many distinct
    // energies a wave holds), then 1 + kTimedSteps steps per candidate
    pamc_options o = opt;
    o.timing = 1;
    o.graphs = 0;
    o.overlap_steps = nullptr;
    o.n_overlap_steps = 0;
    o.capacity = h.Rcap;
    o.tile_rows = 0;
    o.group_replicas = 0;
    o.autotune = 0;
    o.pop_schedule = nullptr;
    o.fuse_gather = 1;
    o.icm_rounds = 0;  // the shape concerns the sweep alone
    // (beta_0 = 0, where every run starts; then the constant tuning beta)
    const int nT = 1 + kBurnIn + (1 + kTimedSteps) * (int)cand.size();
    std::vector<double> beta((size_t)nT, kTuneBeta);
    beta[0] = 0.0;
    HostInst t;
    int st = make_inst(h.L, h.real ? nullptr : h.J.data(), h.real ? h.Jq.data() : nullptr, h.R, beta.data(), nT,
                       h.NS, h.seed, o, t);
    if (st != PAMC_OK) return st;
    Runner run;
    st = run.setup(o, 1);
    if (st != PAMC_OK) return st;
    const int slot = run.add_instance(std::move(t));
    if (slot < 0) return slot;
    st = run.init_instances({slot});
    if (st == PAMC_OK) st = run.build_work({slot});
    if (st != PAMC_OK) return st;
    const double attempts = (double)h.R * h.N * h.NS;
    st = run.enqueue_steps(kBurnIn);
    if (st == PAMC_OK) st = run.sync();
    if (st == PAMC_OK) st = run.phase_times(nullptr, nullptr, nullptr, nullptr);
    if (st != PAMC_OK) return st;
    Choice best{h.tile_rows, h.rp, INFINITY};
    for (const auto &c : cand) {
        // one warm-up step, then the fastest of three timed steps
        st = run.set_shape(slot, c.first, c.second);
        double best_ms = INFINITY;
        for (int rep = 0; rep < 1 + kTimedSteps && st == PAMC_OK; ++rep) {
            double sw = 0.0;
            st = run.enqueue_steps(1);
            if (st == PAMC_OK) st = run.sync();
            if (st == PAMC_OK) st = run.phase_times(&sw, nullptr, nullptr, nullptr);
            if (rep > 0) best_ms = std::min(best_ms, sw);
        }
        if (st == PAMC_OK) st = run.inst_status(slot, nullptr, nullptr);
        if (st != PAMC_OK) return st;
        const double ns = best_ms * 1e6 / attempts;
        if (ns < best.ns_per_attempt) best = Choice{c.first, c.second, ns};
    }
    {
        std::lock_guard<std::mutex> lk(g_mu);
        g_cache[key] = best;
        save_choice(key.first, k0, best);
    }
    h.tile_rows = best.tile_rows;
    h.rp = best.rp;
    if (ns_per_attempt) *ns_per_attempt = best.ns_per_attempt;
    return PAMC_OK;
}

// Loads the persistent choices now (the serving loop does this before its
// first request arrives).
void tune_cache_load()
{
    std::lock_guard<std::mutex> lk(g_mu);
    load_persistent();
}

}  // namespace pamc
