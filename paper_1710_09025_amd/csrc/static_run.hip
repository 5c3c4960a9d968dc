// static_run.hip -- a whole anneal without device allocation, for callers
// that cannot call hipMalloc (code under graph capture, tight serving loops,
// harnesses that forbid it).
//
// Every device buffer of the run (the population, its tables, the work
// lists, the n ln n table, the instance descriptor) is carved, 256-byte
// aligned, from one file-scope device array of kStaticBytes, so the call
// allocates no device memory: the library reads the array's device address
// once per device with hipGetSymbolAddress and hands the kernels pointers
// into it exactly as it hands them pointers into hipMalloc'ed memory in
// pamc_create.  The run is the one pamc_create + pamc_anneal would do, with
// the fixed sweep shape rule, direct kernel launches (no graph) and the
// caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "runner.h"

namespace pamc {
int make_inst(int L, const int8_t *J, const int32_t *Jq, int64_t R, const double *beta, int nT, int NS,
              uint64_t seed, const pamc_options &opt, HostInst &h);
}

namespace {

constexpr size_t kStaticBytes = size_t(64) << 20;  // per device, held until the process ends

// The array itself.  In host code its name is a host-side stand-in, never a
// device address: only the address hipGetSymbolAddress returns is used.
__device__ __align__(256) uint8_t scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;                        // one call at a time per process
uint8_t *g_scratch[kMaxDevices] = {};   // device address of the array, per device

struct Bump {
    uint8_t *base = nullptr;
    size_t cap = 0, off = 0;
    bool overflow = false;
};

void *bump_alloc(size_t bytes, void *user)
{
    Bump *b = static_cast<Bump *>(user);
    const size_t o = (b->off + 255) & ~size_t(255);
    if (o > b->cap || bytes > b->cap - o) {
        b->overflow = true;
        return nullptr;
    }
    b->off = o + bytes;
    return b->base + o;
}

void bump_free(void *, void *) {}

size_t up256(size_t x) { return (x + 255) & ~size_t(255); }

// Device bytes the run takes from the array: the instance's block, the
// descriptor table and coupling pointer, the n ln n table, the work lists of
// the step kernels, the initial population's work list and the export's
// gather lists.
size_t static_need(const pamc::HostInst &h)
{
    using namespace pamc;
    const int64_t cap = h.Rcap;
    const int64_t blocks = (cap + kRowsPerBlock - 1) / kRowsPerBlock;
    int64_t fp2 = 1;
    while (fp2 < h.R) fp2 <<= 1;
    const int64_t g = std::max(1, std::min(1024, 32768 / h.srow_bytes));
    const int64_t gather = (cap + g - 1) / g;
    const int64_t sweep = (cap + h.tile_rows - 1) / h.tile_rows;
    const int64_t post = blocks + std::max<int64_t>(1, fp2 / 2048) + (cap / 2 + kOvlPairs - 1) / kOvlPairs + 1;
    const size_t w = sizeof(Work);
    size_t n = inst_device_bytes(h.L, cap, h.nT, h.ovl_n, h.packed != 0, h.real != 0, h.dim);
    n += up256(sizeof(Inst)) + up256(sizeof(void *));
    n += up256(8 * (size_t)(cap + 1));
    n += up256(w * sweep) + up256(w * blocks) + up256(w * gather) + up256(w * post) + up256(4);
    n += up256(w * ((h.R + kRowsPerBlock - 1) / kRowsPerBlock));
    n += up256(w * gather) + up256(4);
    return n;
}

int fail(int status, const std::string &m)
{
    pamc::set_error("pamc_anneal_static: " + m);
    return status;
}

}  // namespace

extern "C" int pamc_anneal_static(int L, const int8_t *couplings, int64_t R, const double *beta, int n_temps,
                                  int sweeps, uint64_t seed, void *stream, pamc_step_obs *obs, pamc_state *final_state)
{
    using namespace pamc;
    if (!couplings || !beta || !obs) return fail(PAMC_ERR_INVALID, "NULL argument");
    pamc_options o;
    pamc_default_options(&o);
    o.graphs = 0;
    o.stream = stream;
    HostInst h;
    int st = make_inst(L, couplings, nullptr, R, beta, n_temps, sweeps, seed, o, h);
    if (st != PAMC_OK) return st;
    const size_t need = static_need(h);
    if (need > kStaticBytes)
        return fail(PAMC_ERR_INVALID, "the run needs " + std::to_string(need) + " bytes of device memory, more than the " +
                                          std::to_string(kStaticBytes) + " bytes of the allocation-free path");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(PAMC_ERR_DEVICE, "no usable current device");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(PAMC_ERR_DEVICE, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_scratch[dev] = static_cast<uint8_t *>(p);
    }
    Bump bump;
    bump.base = g_scratch[dev];
    bump.cap = kStaticBytes;
    o.alloc = bump_alloc;
    o.free = bump_free;
    o.alloc_user = &bump;
    {
        Runner run;
        st = run.setup(o, 1, true);
        const int slot = st == PAMC_OK ? run.add_instance(std::move(h)) : st;
        st = slot < 0 ? slot : PAMC_OK;
        if (st == PAMC_OK) st = run.init_instances({slot});
        if (st == PAMC_OK) st = run.build_work({slot});
        if (st == PAMC_OK) st = run.enqueue_steps(n_temps);
        if (st == PAMC_OK) st = run.sync();
        int status = PAMC_OK;
        if (st == PAMC_OK) {
            status = run.inst_status(slot, nullptr, nullptr);
            if (status == PAMC_ERR_DEVICE) st = status;
        }
        if (st == PAMC_OK) st = run.observables(slot, obs, n_temps);
        if (st == PAMC_OK && final_state) st = run.get_state(slot, final_state);
        if (st == PAMC_OK) st = status;
        if (bump.overflow) return fail(PAMC_ERR_NOMEM, "the static device array ran out (" + std::to_string(need) +
                                                           " bytes estimated)");
        return st;
    }
}
