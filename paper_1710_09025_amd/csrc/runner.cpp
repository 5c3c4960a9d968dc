// runner.cpp -- host orchestration: validation results are assumed, this
// file builds the host tables (thresholds, weights' rho, n ln n), lays out
// each instance's device memory, builds the work lists of the segmented
// kernels and enqueues the per-step launch sequence.
#include "runner.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace pamc {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

void *Allocator::get(size_t bytes)
{
    if (bytes == 0) bytes = 256;
    if (alloc) return alloc(bytes, user);
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    return p;
}

void Allocator::put(void *p)
{
    if (!p) return;
    if (free)
        free(p, user);
    else
        (void)hipFree(p);
}

int64_t default_capacity(int64_t R) { return R + (int64_t)std::ceil(8.0 * std::sqrt((double)R)) + 64; }


// Colour of site (x, y, z): checkerboard for even L; for odd L the proper
// three-colouring (g(x) + g(y) + g(z)) mod 3 with g(v) = v mod 2 below L-1
// and g(L-1) = 2.
static int colour_of(int L, int x, int y, int z)
{
    if ((L & 1) == 0) return (x + y + z) & 1;
    auto g = [L](int v) { return v == L - 1 ? 2 : (v & 1); };
    return (g(x) + g(y) + g(z)) % 3;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// L = 8, 16: even/odd-x rows (SWAR words aligned to rows).  Otherwise the
// colour-major layout when its largest colour fits a workgroup of 1024
// threads, the slot offsets fit 16 bits and a replica quad's slot fits the
// workgroup's LDS (even L up to 20, odd L up to 21); else lexicographic.
// Real couplings: the colour-major layout wherever it fits (a quad slot of
// four planes), L = 8 and 16 included; no kernel beyond it.  The square
// lattice (dim = 2) runs only with real couplings, in the same layout.
LayoutInfo layout_for(int L, bool real, int dim)
{
    LayoutInfo li{};
    const int Lz = dim == 3 ? L : 1;
    const int N = L * L * Lz;
    li.ncol = (L & 1) ? 3 : 2;
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) li.ncs[colour_of(L, x, y, z)]++;
    li.gmax = 1;
    for (int c = 0; c < 3; ++c) li.gmax = std::max(li.gmax, (li.ncs[c] + 3) / 4);
    li.row_bytes = (N + 15) & ~15;
    if (!real && dim != 3) {
        li.layout = -1;
        li.variant = -1;
        return li;
    }
    if (!real && (L == 8 || L == 16)) {
        li.layout = kLayoutEO;
        li.variant = L == 8 ? kSweepEO8 : kSweepEO16;
        return li;
    }
    int cb = 0;
    for (int c = 0; c < li.ncol; ++c) {
        li.cbase[c] = cb;
        cb += (li.ncs[c] + 3) & ~3;
    }
    const int rb = (cb + 15) & ~15;
    // threads per replica quad: one per Philox block of the largest colour;
    // up to 64 blocks rounded up to a power of two, so that whole quads fit
    // in a wave and sync with wave barriers
    int tpr = 1;
    if (li.gmax <= 64) {
        while (tpr < li.gmax) tpr <<= 1;
    } else {
        tpr = li.gmax;
    }
    if (real) {
        if (tpr <= 1024 && 2 * rb <= 65535 &&
            (size_t)cm_slot_bytes(rb, tpr, 4) * cm_replicas_per_block(tpr) + 32 + 8 * 64 <= kMaxSweepLds) {
            li.layout = kLayoutCM;
            li.variant = dim == 2 ? (li.ncol == 2 ? kSweepSQ2 : kSweepSQ3) : (li.ncol == 2 ? kSweepCQ2 : kSweepCQ3);
            li.row_bytes = rb;
            li.tpr = tpr;
        } else {
            li.layout = -1;
            li.variant = -1;
        }
        return li;
    }
    // The neighbour table in LDS instead of registers: three colours always
    // (136 VGPRs without spills against 168 with 38 spilled: 10-20% faster
    // at L = 5 ... 13), two colours with quads of at most 128 threads
    // (L <= 10: four waves per SIMD instead of three, 7-12% faster; above,
    // the extra table reads and adds cost what the occupancy gains).  The
    // table holds 16-bit slot offsets, so the slot must stay within 64 KB,
    // and slot and table must fit the workgroup's LDS; otherwise the
    // register form.
    auto fits = [&](int v) {
        const size_t tab = (size_t)cm_table_bytes(v, tpr);
        return (size_t)cm_slot_bytes(rb, tpr, 8) * cm_replicas_per_block(tpr) + 32 + 4 * 64 + tab <= kMaxSweepLds &&
               (tab == 0 || 8 * (size_t)cm_plane_bytes(rb) <= 65536);
    };
    const int tab_form = li.ncol == 2 ? (tpr <= 128 ? kSweepCM2T : -1) : kSweepCM3T;
    const int reg_form = li.ncol == 2 ? kSweepCM2 : kSweepCM3;
    const int cmv = tab_form >= 0 && fits(tab_form) ? tab_form : fits(reg_form) ? reg_form : -1;
    if (tpr <= 1024 && 2 * rb <= 65535 && cmv >= 0) {
        li.layout = kLayoutCM;
        li.variant = cmv;
        li.row_bytes = rb;
        li.tpr = tpr;
        return li;
    }
    li.layout = kLayoutLex;
    li.variant = kSweepLex;
    return li;
}

namespace {
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += align256(bytes);
        return o;
    }
};

struct InstLayout {
    size_t ctl, status, sync, spins0, spins1, E0, E1, f0, f1, map, loff, bsum, boff, hist, BF, cnt, fpart, thr,
        beta, rho, Rt, site, grp, jeo, J, pos, lexof, cmdesc, Rk, rec, ovl_slot, qhist, Eq0, Eq1, wrep, wpart, emom, cmj,
        bq, gpw, total;
};

InstLayout layout_of(int L, int64_t R, int64_t Rcap, int nT, int n_ovl, bool packed, bool real, int dim)
{
    const int N = dim == 3 ? L * L * L : L * L;
    const LayoutInfo li = layout_for(L, real, dim);
    const int row_bytes = stored_row_bytes(li.row_bytes, packed);
    const int ncol = li.ncol;
    const int nblk = (int)((Rcap + kRowsPerBlock - 1) / kRowsPerBlock);
    const int nlev = 3 * N + 1;
    int64_t fp2 = 1;
    while (fp2 < R) fp2 <<= 1;
    const int gmax = li.gmax;
    Carve c;
    InstLayout l{};
    l.ctl = c.take(16);
    l.status = c.take(8);
    l.sync = c.take(16);
    l.spins0 = c.take((size_t)Rcap * row_bytes);
    l.spins1 = c.take((size_t)Rcap * row_bytes);
    l.E0 = c.take(real ? 16 : (size_t)Rcap * 4);
    l.E1 = c.take(real ? 16 : (size_t)Rcap * 4);
    l.f0 = c.take((size_t)Rcap * 4);
    l.f1 = c.take((size_t)Rcap * 4);
    l.map = c.take((size_t)Rcap * 4);
    l.loff = c.take((size_t)Rcap * 4);
    l.bsum = c.take((size_t)nblk * 4);
    l.boff = c.take((size_t)nblk * 4);
    l.hist = c.take((size_t)nlev * 4);
    l.BF = c.take((size_t)nlev * 8);
    l.cnt = c.take((size_t)R * 4);
    l.fpart = c.take((size_t)std::max<int64_t>(1, fp2 / 2048) * 8);
    l.thr = c.take((size_t)nT * 16);
    l.beta = c.take((size_t)nT * 8);
    l.rho = c.take((size_t)nT * 8);
    l.Rt = c.take((size_t)nT * 8);
    l.site = c.take((size_t)N * 16);
    l.grp = c.take((size_t)ncol * gmax * 4 * 2);
    l.jeo = c.take((size_t)2 * (N / 8 + 1) * 6 * 4);
    l.J = c.take((size_t)dim * N * (real ? 4 : 1));
    l.pos = c.take((size_t)N * 2);
    l.lexof = c.take((size_t)li.row_bytes * 2);
    l.cmdesc = li.layout == kLayoutCM ? c.take((size_t)ncol * gmax * 32 * 2) : c.take(16);
    l.Rk = c.take((size_t)(nT + 1) * 4);
    l.rec = c.take((size_t)nT * sizeof(StepRec));
    l.ovl_slot = c.take((size_t)nT * 4);
    l.qhist = c.take((size_t)std::max(1, n_ovl) * (2 * N + 1) * 4);
    // real couplings: 64-bit energies, per-row weights, block roots, moments,
    // couplings per neighbour word and the per-step scalars
    l.Eq0 = c.take(real ? (size_t)Rcap * 8 : 16);
    l.Eq1 = c.take(real ? (size_t)Rcap * 8 : 16);
    l.wrep = c.take(real ? (size_t)Rcap * 8 : 16);
    l.wpart = c.take(real ? (size_t)nblk * 8 : 16);
    l.emom = c.take(sizeof(EMoments));
    l.cmj = c.take(real ? (size_t)ncol * gmax * 24 * 4 : 16);
    l.bq = c.take((size_t)nT * 4);
    l.gpw = c.take(real ? (size_t)nT * 40 * 8 : 16);
    l.total = c.off;
    return l;
}
}  // namespace

int stored_row_bytes(int row_bytes, bool packed) { return packed ? (row_bytes + 127) / 128 * 16 : row_bytes; }

size_t inst_device_bytes(int L, int64_t Rcap, int nT, int n_ovl, bool packed, bool real, int dim)
{
    // R <= Rcap; use Rcap for the family counters as an upper bound
    return layout_of(L, Rcap, Rcap, nT, n_ovl, packed, real, dim).total;
}

Runner::~Runner()
{
    if (stream_) (void)hipStreamSynchronize(stream_);
    if (side_) (void)hipStreamSynchronize(side_);
    for (hipStream_t s : aux_) (void)hipStreamSynchronize(s);
    (void)release_fenced(true);
    for (size_t i = 0; i < inst_.size(); ++i)
        if (used_[i]) alloc_.put(inst_[i].block);
    for (void *p : work_allocs_) alloc_.put(p);
    for (hipEvent_t e : ev_pool_) (void)hipEventDestroy(e);
    for (hipEvent_t e : fence_pool_) (void)hipEventDestroy(e);
    if (stage_) (void)hipHostFree(stage_);
    if (side_) (void)hipStreamDestroy(side_);
    drop_graph();
    alloc_.put(d_insts_);
    alloc_.put(d_nlnn_);
    alloc_.put(d_Jptr_);
    for (hipEvent_t e : ev_join_) (void)hipEventDestroy(e);
    if (ev_fork_) (void)hipEventDestroy(ev_fork_);
    for (hipStream_t s : aux_) (void)hipStreamDestroy(s);
    if (own_stream_ && stream_) (void)hipStreamDestroy(stream_);
}

int Runner::dev_fail(hipError_t e, const char *what)
{
    poisoned_ = true;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return PAMC_ERR_DEVICE;
}

#define HIPCHK(call, what)                                   \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return dev_fail(e_, what);     \
    } while (0)

int Runner::setup(const pamc_options &opt, int max_slots, bool external_stream)
{
    alloc_.alloc = opt.alloc;
    alloc_.free = opt.free;
    alloc_.user = opt.alloc_user;
    fuse_ = opt.fuse_gather != 0;
    timing_ = opt.timing != 0;
    graphs_ = opt.graphs != 0 && !timing_;
    max_slots_ = max_slots;
    if (opt.device >= 0) HIPCHK(hipSetDevice(opt.device), "hipSetDevice");
    HIPCHK(hipGetDevice(&device_), "hipGetDevice");
    HIPCHK(sweep_kernels_init(), "hipFuncSetAttribute (sweep LDS)");
    HIPCHK(icm_kernels_init(), "hipFuncSetAttribute (cluster-move LDS)");
    if (opt.stream || external_stream) {
        stream_ = (hipStream_t)opt.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking), "hipStreamCreate");
        own_stream_ = true;
    }
    if (max_slots > 1) {
        for (int a = 0; a < kAuxStreams; ++a) {
            hipStream_t s = nullptr;
            hipEvent_t e = nullptr;
            HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate (sweep groups)");
            aux_.push_back(s);
            HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate (sweep groups)");
            ev_join_.push_back(e);
        }
        HIPCHK(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming), "hipEventCreate (sweep groups)");
    }
    inst_.resize((size_t)max_slots);
    used_.assign((size_t)max_slots, 0);
    held_.assign((size_t)max_slots, 0);
    d_insts_ = (Inst *)alloc_.get(sizeof(Inst) * (size_t)max_slots);
    d_Jptr_ = (const int8_t **)alloc_.get(sizeof(void *) * (size_t)max_slots);
    if (!d_insts_ || !d_Jptr_) {
        set_error("device allocation failed (instance table)");
        return PAMC_ERR_NOMEM;
    }
    return PAMC_OK;
}

int Runner::enable_async(size_t staging_bytes)
{
    if (async_) return PAMC_OK;
    HIPCHK(hipStreamCreateWithFlags(&side_, hipStreamNonBlocking), "hipStreamCreate (uploads)");
    HIPCHK(hipHostMalloc((void **)&stage_, staging_bytes, hipHostMallocDefault), "hipHostMalloc (staging)");
    stage_cap_ = staging_bytes;
    stage_used_ = 0;
    async_ = true;
    return PAMC_OK;
}

int Runner::h2d(void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return PAMC_OK;
    if (!async_) {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream_), "upload");
        return PAMC_OK;
    }
    const uint8_t *s = static_cast<const uint8_t *>(src);
    uint8_t *d = static_cast<uint8_t *>(dst);
    while (bytes > 0) {
        // the staging is reused once the copies issued from it have landed
        if (stage_used_ == stage_cap_) {
            HIPCHK(hipStreamSynchronize(side_), "staging sync");
            stage_used_ = 0;
        }
        const size_t n = std::min(bytes, stage_cap_ - stage_used_);
        std::memcpy(stage_ + stage_used_, s, n);
        HIPCHK(hipMemcpyAsync(d, stage_ + stage_used_, n, hipMemcpyHostToDevice, side_), "staged upload");
        stage_used_ = std::min(stage_cap_, stage_used_ + ((n + 63) & ~size_t(63)));
        s += n;
        d += n;
        bytes -= n;
    }
    return PAMC_OK;
}

int Runner::upload_sync()
{
    HIPCHK(hipStreamSynchronize(up_stream()), "upload sync");
    stage_used_ = 0;
    return PAMC_OK;
}

int Runner::d2h(void *dst, const void *src, size_t bytes)
{
    if (bytes == 0) return PAMC_OK;
    HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, up_stream()), "read back");
    HIPCHK(hipStreamSynchronize(up_stream()), "read back sync");
    return PAMC_OK;
}

int Runner::fence(std::vector<void *> ptrs, std::vector<int> slots)
{
    hipEvent_t e = nullptr;
    if (!fence_pool_.empty()) {
        e = fence_pool_.back();
        fence_pool_.pop_back();
    } else {
        HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate (fence)");
    }
    HIPCHK(hipEventRecord(e, stream_), "hipEventRecord (fence)");
    for (int i : slots) held_[(size_t)i] = 1;
    fenced_.push_back(Fenced{e, std::move(ptrs), std::move(slots)});
    return PAMC_OK;
}

int Runner::release_fenced(bool wait)
{
    for (size_t j = 0; j < fenced_.size();) {
        Fenced &f = fenced_[j];
        hipError_t q = wait ? hipEventSynchronize(f.ev) : hipEventQuery(f.ev);
        if (q == hipErrorNotReady) {
            ++j;
            continue;
        }
        if (q != hipSuccess) return dev_fail(q, "fence");
        for (void *p : f.ptrs) alloc_.put(p);
        for (int i : f.slots) held_[(size_t)i] = 0;
        fence_pool_.push_back(f.ev);
        fenced_.erase(fenced_.begin() + (long)j);
    }
    return PAMC_OK;
}

int Runner::free_slots() const
{
    int n = 0;
    for (int i = 0; i < max_slots_; ++i)
        if (!used_[i] && !held_[i]) ++n;
    return n;
}

// n ln n for n = 0 .. len-1 (host libm), shared by all instances; grows when
// an instance with a larger capacity arrives.
int Runner::ensure_nlnn(int64_t len)
{
    if (len <= nlnn_len_) return PAMC_OK;
    // every queued step reads the table that is replaced
    HIPCHK(hipStreamSynchronize(stream_), "nlnn sync");
    if (side_) HIPCHK(hipStreamSynchronize(side_), "nlnn sync");
    const int64_t n = std::max(len, 2 * nlnn_len_);
    std::vector<double> nl((size_t)n);
    nl[0] = 0.0;
    for (int64_t q = 1; q < n; ++q) nl[(size_t)q] = (double)q * std::log((double)q);
    double *d = (double *)alloc_.get(nl.size() * 8);
    if (!d) {
        set_error("device allocation failed (n ln n table)");
        return PAMC_ERR_NOMEM;
    }
    HIPCHK(hipMemcpy(d, nl.data(), nl.size() * 8, hipMemcpyHostToDevice), "upload nlnn");
    for (size_t i = 0; i < inst_.size(); ++i) {
        if (!used_[i]) continue;
        inst_[i].dev.nlnn = d;
        HIPCHK(hipMemcpy(d_insts_ + i, &inst_[i].dev, sizeof(Inst), hipMemcpyHostToDevice), "update instance");
    }
    alloc_.put(d_nlnn_);
    d_nlnn_ = d;
    nlnn_len_ = n;
    return PAMC_OK;
}

int Runner::add_instance(HostInst &&h)
{
    int slot = -1;
    for (int i = 0; i < max_slots_; ++i)
        if (!used_[i] && !held_[i]) {
            slot = i;
            break;
        }
    if (slot < 0) {
        set_error("no free instance slot");
        return PAMC_ERR_BUSY;
    }
    int st = ensure_nlnn(h.Rcap + 1);
    if (st != PAMC_OK) return st;
    inst_[slot] = std::move(h);
    st = upload_inst(slot);
    if (st != PAMC_OK) {
        alloc_.put(inst_[slot].block);
        inst_[slot].block = nullptr;
        return st;
    }
    used_[slot] = 1;
    const int8_t *jp = inst_[slot].Jdev;
    st = h2d(d_insts_ + slot, &inst_[slot].dev, sizeof(Inst));
    if (st == PAMC_OK) st = h2d(d_Jptr_ + slot, &jp, sizeof(void *));
    if (st == PAMC_OK) st = upload_sync();
    if (st != PAMC_OK) return st;
    return slot;
}

void Runner::remove_instance(int slot)
{
    if (slot < 0 || slot >= max_slots_ || !used_[slot]) return;
    if (async_) {
        // queued steps may still read the instance: release it behind them
        (void)fence({inst_[slot].block}, {slot});
    } else {
        (void)hipStreamSynchronize(stream_);
        alloc_.put(inst_[slot].block);
    }
    inst_[slot] = HostInst();
    used_[slot] = 0;
}

int Runner::upload_inst(int i)
{
    HostInst &h = inst_[i];
    const int L = h.L, N = h.N;
    const InstLayout lay = layout_of(L, h.R, h.Rcap, h.nT, h.ovl_n, h.packed != 0, h.real != 0, h.dim);
    h.bytes = lay.total;
    h.block = alloc_.get(lay.total);
    if (!h.block) {
        set_error("device allocation of " + std::to_string(lay.total) + " bytes failed");
        return PAMC_ERR_NOMEM;
    }
    uint8_t *b = (uint8_t *)h.block;
    HIPCHK(hipMemsetAsync(b, 0, lay.total, up_stream()), "clear instance memory");
    Inst &d = h.dev;
    std::memset(&d, 0, sizeof(d));
    d.L = L;
    d.N = N;
    d.dim = h.dim;
    d.ncol = h.ncol;
    d.layout = h.layout;
    d.row_bytes = h.row_bytes;
    d.packed = h.packed;
    d.srow_bytes = h.srow_bytes;
    d.nT = h.nT;
    d.NS = h.NS;
    d.key0 = (uint32_t)h.seed;
    d.key1 = (uint32_t)(h.seed >> 32);
    d.R = (int32_t)h.R;
    d.Rcap = (int32_t)h.Rcap;
    d.nblk = (int32_t)((h.Rcap + kRowsPerBlock - 1) / kRowsPerBlock);
    d.nlev = 3 * N + 1;
    int64_t fp2 = 1;
    while (fp2 < h.R) fp2 <<= 1;
    d.fam_pow2 = (int32_t)fp2;
    d.ovl_n = h.ovl_n;
    d.spins[0] = b + lay.spins0;
    d.spins[1] = b + lay.spins1;
    d.E[0] = (int32_t *)(b + lay.E0);
    d.E[1] = (int32_t *)(b + lay.E1);
    d.fam[0] = (uint32_t *)(b + lay.f0);
    d.fam[1] = (uint32_t *)(b + lay.f1);
    d.map = (uint32_t *)(b + lay.map);
    d.loff = (uint32_t *)(b + lay.loff);
    d.bsum = (uint32_t *)(b + lay.bsum);
    d.boff = (uint32_t *)(b + lay.boff);
    d.hist = (uint32_t *)(b + lay.hist);
    d.BF = (uint2 *)(b + lay.BF);
    d.cnt = (uint32_t *)(b + lay.cnt);
    d.fpart = (double *)(b + lay.fpart);
    d.thr = (const uint4 *)(b + lay.thr);
    d.beta = (const double *)(b + lay.beta);
    d.rho = (const double *)(b + lay.rho);
    d.Rt = (const double *)(b + lay.Rt);
    d.nlnn = d_nlnn_;
    d.site = (const uint4 *)(b + lay.site);
    d.grp = (const uint16_t *)(b + lay.grp);
    d.jeo = (const uint32_t *)(b + lay.jeo);
    d.pos = (const uint16_t *)(b + lay.pos);
    d.lexof = (const uint16_t *)(b + lay.lexof);
    d.cmdesc = (const uint16_t *)(b + lay.cmdesc);
    d.k = (int32_t *)(b + lay.ctl);
    d.cur = d.k + 1;
    d.mapped = d.k + 2;
    d.Rk = (uint32_t *)(b + lay.Rk);
    d.rec = (StepRec *)(b + lay.rec);
    d.ovl_slot = (int32_t *)(b + lay.ovl_slot);
    d.qhist = (uint32_t *)(b + lay.qhist);
    d.status = (uint32_t *)(b + lay.status);
    d.sync = (uint32_t *)(b + lay.sync);
    d.real = h.real;
    d.icm = h.icm;
    d.icm_bmin = h.icm_bmin;
    d.Eq[0] = (int64_t *)(b + lay.Eq0);
    d.Eq[1] = (int64_t *)(b + lay.Eq1);
    d.wrep = (double *)(b + lay.wrep);
    d.wpart = (double *)(b + lay.wpart);
    d.emom = (EMoments *)(b + lay.emom);
    d.cmj = (const int32_t *)(b + lay.cmj);
    d.bq = (const float *)(b + lay.bq);
    d.gpw = (const double *)(b + lay.gpw);
    d.Jtot = 0;
    for (int32_t v : h.Jq) d.Jtot += v;
    d.tile_rows = h.tile_rows;
    d.sweep_tiles = (int32_t)((h.Rcap + h.tile_rows - 1) / h.tile_rows);
    {
        const int64_t nchunks = std::max<int64_t>(1, fp2 / 2048);
        const int64_t novl = (h.Rcap / 2 + kOvlPairs - 1) / kOvlPairs;
        d.post_blocks = (int32_t)(d.nblk + nchunks + novl);
    }
    h.ctl = d.k;
    h.Jdev = (int8_t *)(b + lay.J);

    // --- thresholds: T_k(dE) = floor(exp(-beta_k dE) 2^32), capped; beta = 0
    // accepts every move
    std::vector<uint32_t> thr((size_t)h.nT * 4);
    for (int k = 0; k < h.nT; ++k) {
        const double bk = h.beta[k];
        for (int j = 0; j < 3; ++j) {
            const double p = std::exp(-bk * (4.0 * (j + 1)));
            const double x = std::floor(p * 4294967296.0);
            thr[4 * k + j] = x >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)x;
        }
        thr[4 * k + 3] = bk == 0.0 ? 1u : 0u;
    }
    // --- rho_k = exp(-2 (beta_{k+1} - beta_k)): weight ratio of adjacent levels
    std::vector<double> rho((size_t)h.nT, 1.0);
    for (int k = 0; k + 1 < h.nT; ++k) {
        const double db = h.beta[k + 1] - h.beta[k];
        rho[k] = std::exp(-2.0 * db);
    }
    // --- colours and colour ranks
    const int Lz = h.dim == 3 ? L : 1;
    std::vector<int> col(N), rank(N);
    int ncs[3] = {0, 0, 0};
    for (int z = 0; z < Lz; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                const int s = x + L * (y + L * z);
                col[s] = colour_of(L, x, y, z);
                rank[s] = ncs[col[s]]++;
            }
    for (int c = 0; c < 3; ++c) {
        d.ncs[c] = ncs[c];
        d.gcs[c] = (ncs[c] + 3) / 4;
    }
    d.gmax = std::max(d.gcs[0], std::max(d.gcs[1], d.gcs[2]));
    // coupling of bond (dir, s): +-1, or j (units of 2^-20) for real couplings
    auto J = [&](int dir, int s) { return h.real ? (int)h.Jq[(size_t)dir * N + s] : (int)h.J[(size_t)dir * N + s]; };
    auto site_of = [L, Lz](int x, int y, int z) {
        return ((x % L + L) % L) + L * (((y % L + L) % L) + L * ((z % Lz + Lz) % Lz));
    };
    const LayoutInfo li = layout_for(L, h.real != 0, h.dim);
    for (int c = 0; c < 3; ++c) d.cbase[c] = li.cbase[c];
    d.tpr = li.tpr;
    d.plane_bytes = cm_plane_bytes(h.row_bytes);
    d.slot_bytes = cm_slot_bytes(h.row_bytes, li.tpr, h.real ? 4 : 8);
    // storage position of each site
    h.lex_pos.resize(N);
    std::vector<uint16_t> pos16((size_t)N);
    for (int s = 0; s < N; ++s) {
        const int x = s % L, yz = s / L;
        if (h.layout == kLayoutLex)
            h.lex_pos[s] = s;
        else if (h.layout == kLayoutEO)
            h.lex_pos[s] = col[s] * (N / 2) + yz * (L / 2) + (x >> 1);
        else
            h.lex_pos[s] = li.cbase[col[s]] + rank[s];
        pos16[s] = (uint16_t)h.lex_pos[s];
    }
    // its inverse over the storage positions of a row (cluster moves read
    // rows in storage order)
    std::vector<uint16_t> lexof16((size_t)h.row_bytes, (uint16_t)0xFFFF);
    for (int s = 0; s < N; ++s) lexof16[(size_t)h.lex_pos[s]] = (uint16_t)s;
    std::vector<uint16_t> cmdesc;
    std::vector<int32_t> cmj;
    std::vector<uint32_t> site((size_t)N * 4, 0u);
    std::vector<uint16_t> grp((size_t)h.ncol * d.gmax * 4, (uint16_t)0xFFFF);
    std::vector<uint32_t> jeo((size_t)2 * (N / 8 + 1) * 6, 0u);
    if (h.layout == kLayoutLex) {
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    const int s = site_of(x, y, z);
                    const int nb[6] = {site_of(x + 1, y, z), site_of(x - 1, y, z), site_of(x, y + 1, z),
                                       site_of(x, y - 1, z), site_of(x, y, z + 1), site_of(x, y, z - 1)};
                    // couplings of the six bonds; the bond to s - e_d is
                    // stored at the lower site
                    const int jv[6] = {J(0, s), J(0, nb[1]), J(1, s), J(1, nb[3]), J(2, s), J(2, nb[5])};
                    uint32_t jm = 0;
                    for (int q = 0; q < 6; ++q)
                        if (jv[q] < 0) jm |= 1u << q;
                    site[4 * s + 0] = (uint32_t)nb[0] | ((uint32_t)nb[1] << 16);
                    site[4 * s + 1] = (uint32_t)nb[2] | ((uint32_t)nb[3] << 16);
                    site[4 * s + 2] = (uint32_t)nb[4] | ((uint32_t)nb[5] << 16);
                    site[4 * s + 3] = jm;
                    const int c = col[s], r = rank[s];
                    grp[((size_t)c * d.gmax + (r >> 2)) * 4 + (r & 3)] = (uint16_t)s;
                }
    } else if (h.layout == kLayoutCM) {
        // per colour, Philox block and site: the LDS offsets of its six
        // neighbours, in the complemented copy (+row_bytes) for a -1 bond;
        // for real couplings the plain copy, with the couplings alongside.
        // On the square lattice the two z entries of a site point at the
        // site itself with coupling 0: they add nothing to its field or to
        // the energy, so the sweep kernel runs unchanged.
        std::vector<int> site_at((size_t)3 * N, -1);
        for (int s = 0; s < N; ++s) site_at[(size_t)col[s] * N + rank[s]] = s;
        cmdesc.assign((size_t)h.ncol * d.gmax * 32, 0);
        if (h.real) cmj.assign((size_t)h.ncol * d.gmax * 24, 0);
        for (int c = 0; c < h.ncol; ++c)
            for (int g = 0; g < d.gcs[c]; ++g) {
                uint16_t *e = cmdesc.data() + ((size_t)c * d.gmax + g) * 32;
                uint32_t vmask = 0;
                for (int bb = 0; bb < 4; ++bb) {
                    const int i = 4 * g + bb;
                    if (i >= ncs[c]) {
                        // padding byte: no site; point at itself (value 0)
                        for (int dd = 0; dd < 6; ++dd) e[4 * dd + bb] = (uint16_t)(li.cbase[c] + i);
                        continue;
                    }
                    vmask |= 1u << (8 * bb);
                    const int s = site_at[(size_t)c * N + i];
                    const int x = s % L, y = (s / L) % L, z = s / (L * L);
                    const bool sq = h.dim == 2;
                    const int nb[6] = {site_of(x + 1, y, z), site_of(x - 1, y, z), site_of(x, y + 1, z),
                                       site_of(x, y - 1, z), sq ? s : site_of(x, y, z + 1),
                                       sq ? s : site_of(x, y, z - 1)};
                    const int jv[6] = {J(0, s), J(0, nb[1]), J(1, s), J(1, nb[3]), sq ? 0 : J(2, s),
                                       sq ? 0 : J(2, nb[5])};
                    for (int dd = 0; dd < 6; ++dd) {
                        if (h.real) {
                            e[4 * dd + bb] = (uint16_t)h.lex_pos[nb[dd]];
                            cmj[((size_t)c * d.gmax + g) * 24 + 4 * dd + bb] = jv[dd];
                        } else {
                            e[4 * dd + bb] = (uint16_t)(h.lex_pos[nb[dd]] + (jv[dd] < 0 ? h.row_bytes : 0));
                        }
                    }
                }
                e[24] = (uint16_t)(vmask & 0xFFFFu);
                e[25] = (uint16_t)(vmask >> 16);
            }
    } else {
        const int H = L / 2, GPR = L / 8, G = N / 8;
        for (int c = 0; c < 2; ++c)
            for (int g = 0; g < G; ++g) {
                const int row = g / GPR, jb = g % GPR;
                const int y = row % L, z = row / L;
                const int p = (c + y + z) & 1;
                uint32_t w[6] = {0, 0, 0, 0, 0, 0};
                for (int bb = 0; bb < 4; ++bb) {
                    const int x = 2 * (4 * jb + bb) + p;
                    const int s = site_of(x, y, z);
                    const int xm = site_of(x - 1, y, z), ym = site_of(x, y - 1, z), zm = site_of(x, y, z - 1);
                    // aligned x neighbour: x+1 for p = 0, x-1 for p = 1
                    const int ja = p == 0 ? J(0, s) : J(0, xm);
                    const int js = p == 0 ? J(0, xm) : J(0, s);
                    const int jv[6] = {ja, js, J(1, s), J(1, ym), J(2, s), J(2, zm)};
                    for (int q = 0; q < 6; ++q)
                        if (jv[q] < 0) w[q] |= 1u << (8 * bb);
                }
                for (int q = 0; q < 6; ++q) jeo[((size_t)c * G + g) * 6 + q] = w[q];
                (void)H;
            }
    }
    // real couplings: beta_k 2^-20 in binary32 and the weight factors
    // exp(-(beta_{k+1} - beta_k) 2^(b-20)), b < 40, host libm
    std::vector<float> bq((size_t)h.nT);
    for (int k = 0; k < h.nT; ++k) bq[(size_t)k] = (float)(h.beta[k] * 0x1p-20);
    std::vector<double> gpw;
    if (h.real) {
        gpw.assign((size_t)h.nT * 40, 1.0);
        for (int k = 0; k + 1 < h.nT; ++k) {
            const double db = h.beta[k + 1] - h.beta[k];
            for (int bb = 0; bb < 40; ++bb) gpw[(size_t)k * 40 + bb] = std::exp(-db * std::ldexp(1.0, bb - 20));
        }
    }
    EMoments em{};
    em.emin = std::numeric_limits<long long>::max();
    em.emax = std::numeric_limits<long long>::min();
    std::vector<uint32_t> Rk0((size_t)h.nT + 1, 0u);
    Rk0[0] = (uint32_t)h.R;
    int32_t ctl[4] = {0, 0, 0, 0};
    int st = PAMC_OK;
    auto put = [&](size_t off, const void *src, size_t bytes) {
        if (st == PAMC_OK) st = h2d(b + off, src, bytes);
    };
    put(lay.ctl, ctl, 16);
    put(lay.thr, thr.data(), thr.size() * 4);
    put(lay.beta, h.beta.data(), h.beta.size() * 8);
    put(lay.rho, rho.data(), rho.size() * 8);
    put(lay.Rt, h.pop.data(), h.pop.size() * 8);
    put(lay.site, site.data(), site.size() * 4);
    put(lay.grp, grp.data(), grp.size() * 2);
    put(lay.jeo, jeo.data(), jeo.size() * 4);
    if (h.real)
        put(lay.J, h.Jq.data(), h.Jq.size() * 4);
    else
        put(lay.J, h.J.data(), h.J.size());
    put(lay.bq, bq.data(), bq.size() * 4);
    put(lay.emom, &em, sizeof(em));
    if (!gpw.empty()) put(lay.gpw, gpw.data(), gpw.size() * 8);
    if (!cmj.empty()) put(lay.cmj, cmj.data(), cmj.size() * 4);
    put(lay.pos, pos16.data(), pos16.size() * 2);
    put(lay.lexof, lexof16.data(), lexof16.size() * 2);
    if (!cmdesc.empty()) put(lay.cmdesc, cmdesc.data(), cmdesc.size() * 2);
    put(lay.Rk, Rk0.data(), Rk0.size() * 4);
    put(lay.ovl_slot, h.ovl_slot.data(), h.ovl_slot.size() * 4);
    // host vectors must outlive the async copies
    if (st == PAMC_OK) st = upload_sync();
    if (st != PAMC_OK) return st;
    h.k_enq = 0;
    h.k_base = 0;
    h.lnZ_base = (double)N * std::log(2.0);
    return PAMC_OK;
}

std::vector<Work> gather_items(uint32_t slot, int64_t Rcap, int row_bytes)
{
    const int g = std::max(1, std::min(1024, 32768 / row_bytes));
    std::vector<Work> v;
    for (int64_t r = 0; r < Rcap; r += g) v.push_back(Work{slot, (uint32_t)r, 0u, (uint32_t)g});
    return v;
}

int Runner::set_shape(int i, int tile_rows, int rp)
{
    if (i < 0 || i >= max_slots_ || !used_[i]) return PAMC_ERR_STATE;
    HostInst &h = inst_[i];
    h.tile_rows = tile_rows;
    h.rp = rp;
    h.dev.tile_rows = tile_rows;
    h.dev.sweep_tiles = (int32_t)((h.Rcap + tile_rows - 1) / tile_rows);
    HIPCHK(hipStreamSynchronize(stream_), "set_shape sync");
    HIPCHK(hipMemcpy(d_insts_ + i, &h.dev, sizeof(Inst), hipMemcpyHostToDevice), "update instance shape");
    return build_work(active_);
}

int Runner::build_work(const std::vector<int> &active)
{
    if (async_) {
        // the lists being replaced serve the steps already queued
        if (!work_allocs_.empty()) {
            const int st = fence(std::move(work_allocs_), {});
            if (st != PAMC_OK) return st;
        }
    } else {
        HIPCHK(hipStreamSynchronize(stream_), "build_work sync");
        drop_graph();
        for (void *p : work_allocs_) alloc_.put(p);
    }
    work_allocs_.clear();
    sweep_groups_.clear();
    active_ = active;
    auto upload = [&](const void *src, size_t bytes) -> void * {
        void *p = alloc_.get(bytes);
        if (!p) return nullptr;
        work_allocs_.push_back(p);
        if (h2d(p, src, bytes) != PAMC_OK) return nullptr;
        return p;
    };
    std::map<std::tuple<int, int, int, int, int, int, int>, std::vector<Work>> groups;
    std::vector<Work> rows, post, gath, wblk, icm;
    icm_rounds_ = 0;
    icm_N_ = 0;
    std::vector<uint32_t> list;
    for (int i : active) {
        const HostInst &h = inst_[i];
        const uint32_t ii = (uint32_t)i;
        auto &g = groups[std::make_tuple(h.variant, h.L, h.tile_rows, h.row_bytes, h.tpr, h.rp, h.icm > 0 ? 1 : 0)];
        if (h.icm > 0) {
            for (int64_t j = 0; j < h.Rcap / 2; ++j) icm.push_back(Work{ii, (uint32_t)j, 0u, 0u});
            icm_rounds_ = std::max(icm_rounds_, h.icm);
            icm_N_ = std::max(icm_N_, h.N);
        }
        for (int64_t r = 0; r < h.Rcap; r += h.tile_rows) g.push_back(Work{ii, (uint32_t)r, 0u, 0u});
        for (int64_t r = 0; r < h.Rcap; r += kRowsPerBlock) {
            rows.push_back(Work{ii, (uint32_t)r, 0u, 0u});
            post.push_back(Work{ii, (uint32_t)r, kRoleCopies, 0u});
            if (h.real) wblk.push_back(Work{ii, (uint32_t)r, 0u, 0u});
        }
        for (const Work &w : gather_items(ii, h.Rcap, h.srow_bytes)) gath.push_back(w);
        int64_t fp2 = 1;
        while (fp2 < h.R) fp2 <<= 1;
        for (int64_t f = 0; f < fp2; f += 2048) post.push_back(Work{ii, (uint32_t)f, kRoleFamilies, 0u});
        for (int64_t r = 0; r < h.Rcap / 2; r += kOvlPairs) post.push_back(Work{ii, (uint32_t)r, kRoleOverlap, 0u});
        list.push_back(ii);
    }
    for (auto &kv : groups) {
        SweepGroup sg;
        sg.variant = std::get<0>(kv.first);
        sg.tile_rows = std::get<2>(kv.first);
        sg.row_bytes = std::get<3>(kv.first);
        sg.tpr = std::get<4>(kv.first);
        sg.rp = std::get<5>(kv.first);
        sg.icm = std::get<6>(kv.first);
        sg.nwork = (int)kv.second.size();
        sg.work = (Work *)upload(kv.second.data(), kv.second.size() * sizeof(Work));
        if (!sg.work) return dev_fail(hipErrorOutOfMemory, "upload sweep work");
        sweep_groups_.push_back(sg);
    }
    d_rows_ = (Work *)upload(rows.data(), rows.size() * sizeof(Work));
    d_gather_ = (Work *)upload(gath.data(), gath.size() * sizeof(Work));
    ngather_ = (int)gath.size();
    d_post_ = (Work *)upload(post.data(), post.size() * sizeof(Work));
    d_list_ = (uint32_t *)upload(list.data(), list.size() * 4);
    d_icm_ = nullptr;
    nicm_ = (int)icm.size();
    if (nicm_) {
        d_icm_ = (Work *)upload(icm.data(), icm.size() * sizeof(Work));
        if (!d_icm_) return dev_fail(hipErrorOutOfMemory, "upload pair work");
    }
    d_wblk_ = nullptr;
    nwblk_ = (int)wblk.size();
    if (nwblk_) {
        d_wblk_ = (Work *)upload(wblk.data(), wblk.size() * sizeof(Work));
        if (!d_wblk_) return dev_fail(hipErrorOutOfMemory, "upload weight work");
    }
    if (!d_rows_ || !d_post_ || !d_list_ || !d_gather_) return dev_fail(hipErrorOutOfMemory, "upload work lists");
    const int ust = upload_sync();
    if (ust != PAMC_OK) return ust;
    nrows_work_ = (int)rows.size();
    npost_ = (int)post.size();
    nlist_ = (int)list.size();
    return PAMC_OK;
}

int Runner::init_instances(const std::vector<int> &slots)
{
    std::vector<Work> w;
    for (int i : slots)
        for (int64_t r = 0; r < inst_[i].R; r += kRowsPerBlock) w.push_back(Work{(uint32_t)i, (uint32_t)r, 0u, 0u});
    if (w.empty()) return PAMC_OK;
    Work *d = (Work *)alloc_.get(w.size() * sizeof(Work));
    if (!d) return PAMC_ERR_NOMEM;
    int st = h2d(d, w.data(), w.size() * sizeof(Work));
    if (st != PAMC_OK) return st;
    size_t lds = 0;
    for (int i : slots)
        if (inst_[i].packed) lds = std::max(lds, (size_t)std::max(16384, inst_[i].row_bytes));
    launch_init(d_insts_, d, (int)w.size(), lds, up_stream());
    launch_energy(d_insts_, d, (int)w.size(), d_Jptr_, up_stream());
    HIPCHK(hipGetLastError(), "init launch");
    st = upload_sync();
    if (st != PAMC_OK) return st;
    alloc_.put(d);
    return PAMC_OK;
}

void Runner::drop_graph()
{
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    if (chunk_exec_) (void)hipGraphExecDestroy(chunk_exec_);
    if (chunk_graph_) (void)hipGraphDestroy(chunk_graph_);
    graph_exec_ = nullptr;
    graph_ = nullptr;
    chunk_exec_ = nullptr;
    chunk_graph_ = nullptr;
}

// The kernels of one temperature step, for every active instance.  Their
// arguments do not change from step to step (the step index and the
// population size live on the device), so the sequence can be captured once.
int Runner::launch_step_kernels()
{
    // the shape groups touch disjoint instances: with several of them, fork
    // them onto the auxiliary streams, the largest first, and join before
    // the resampling (a launch's last workgroups then share the chip with
    // the next group's first ones)
    std::vector<const SweepGroup *> plain;
    for (auto &g : sweep_groups_)
        if (!g.icm) plain.push_back(&g);
    const int ns = std::min((int)aux_.size(), (int)plain.size() - 1);
    if (ns <= 0) {
        for (const SweepGroup *g : plain)
            launch_sweep(g->variant, d_insts_, g->work, g->nwork, g->tile_rows, g->row_bytes, g->tpr, g->rp, 0, stream_);
    } else {
        std::stable_sort(plain.begin(), plain.end(), [](const SweepGroup *a, const SweepGroup *b) {
            return (double)a->nwork * a->tile_rows * a->row_bytes > (double)b->nwork * b->tile_rows * b->row_bytes;
        });
        HIPCHK(hipEventRecord(ev_fork_, stream_), "hipEventRecord (fork)");
        for (int a = 0; a < ns; ++a) HIPCHK(hipStreamWaitEvent(aux_[a], ev_fork_, 0), "hipStreamWaitEvent (fork)");
        for (size_t j = 0; j < plain.size(); ++j) {
            const int lane = (int)(j % (size_t)(ns + 1));
            const SweepGroup *g = plain[j];
            launch_sweep(g->variant, d_insts_, g->work, g->nwork, g->tile_rows, g->row_bytes, g->tpr, g->rp, 0,
                         lane == 0 ? stream_ : aux_[lane - 1]);
        }
        for (int a = 0; a < ns; ++a) {
            HIPCHK(hipEventRecord(ev_join_[a], aux_[a]), "hipEventRecord (join)");
            HIPCHK(hipStreamWaitEvent(stream_, ev_join_[a], 0), "hipStreamWaitEvent (join)");
        }
    }
    // runs with cluster moves split their sweeps around the ICM rounds
    if (nicm_) {
        for (auto &g : sweep_groups_)
            if (g.icm)
                launch_sweep(g.variant, d_insts_, g.work, g.nwork, g.tile_rows, g.row_bytes, g.tpr, g.rp, 1, stream_);
        for (int rd = 0; rd < icm_rounds_; ++rd) launch_icm(d_insts_, d_icm_, nicm_, icm_N_, rd, stream_);
        for (auto &g : sweep_groups_)
            if (g.icm)
                launch_sweep(g.variant, d_insts_, g.work, g.nwork, g.tile_rows, g.row_bytes, g.tpr, g.rp, 2, stream_);
    }
    if (timing_) HIPCHK(hipEventRecord(ev_pool_[ev_used_ - 3], stream_), "hipEventRecord");
    launch_weights(d_insts_, d_wblk_, nwblk_, stream_);
    launch_post(d_insts_, d_post_, npost_, stream_);
    launch_expand(d_insts_, d_rows_, nrows_work_, stream_);
    if (timing_) HIPCHK(hipEventRecord(ev_pool_[ev_used_ - 2], stream_), "hipEventRecord");
    if (!fuse_) {
        launch_gather(d_insts_, d_gather_, ngather_, stream_);
        launch_flip(d_insts_, d_list_, nlist_, stream_);
    }
    return PAMC_OK;
}

int Runner::enqueue_step()
{
    if (poisoned_) return PAMC_ERR_DEVICE;
    if (timing_) {
        while (ev_pool_.size() < ev_used_ + 4) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e), "hipEventCreate");
            ev_pool_.push_back(e);
        }
        ev_used_ += 4;
        HIPCHK(hipEventRecord(ev_pool_[ev_used_ - 4], stream_), "hipEventRecord");
    }
    if (graphs_) {
        if (!graph_exec_) {
            HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
            launch_step_kernels();
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamEndCapture(stream_, &g), "hipStreamEndCapture");
            graph_ = g;
            HIPCHK(hipGraphInstantiate(&graph_exec_, graph_, nullptr, nullptr, 0), "hipGraphInstantiate");
        }
        HIPCHK(hipGraphLaunch(graph_exec_, stream_), "hipGraphLaunch");
    } else {
        int st = launch_step_kernels();
        if (st != PAMC_OK) return st;
    }
    if (timing_) HIPCHK(hipEventRecord(ev_pool_[ev_used_ - 1], stream_), "hipEventRecord");
    HIPCHK(hipGetLastError(), "step launch");
    count_enqueued(1);
    return PAMC_OK;
}

void Runner::count_enqueued(int steps)
{
    for (int i : active_) {
        HostInst &h = inst_[i];
        h.k_enq = std::min(h.nT, h.k_enq + steps);
    }
}

// kChunkSteps steps as one graph launch (the step kernels read the step
// index from the device, so consecutive steps are the same kernel
// sequence; steps past an instance's last temperature do nothing).
int Runner::enqueue_chunk()
{
    if (poisoned_) return PAMC_ERR_DEVICE;
    if (!chunk_exec_) {
        HIPCHK(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
        for (int s = 0; s < kChunkSteps; ++s) launch_step_kernels();
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamEndCapture(stream_, &g), "hipStreamEndCapture");
        chunk_graph_ = g;
        HIPCHK(hipGraphInstantiate(&chunk_exec_, chunk_graph_, nullptr, nullptr, 0), "hipGraphInstantiate");
    }
    HIPCHK(hipGraphLaunch(chunk_exec_, stream_), "hipGraphLaunch");
    HIPCHK(hipGetLastError(), "chunk launch");
    count_enqueued(kChunkSteps);
    return PAMC_OK;
}

int Runner::phase_times(double *sweep_ms, double *resample_ms, double *gather_ms, int64_t *n_steps)
{
    if (!timing_) {
        set_error("timing is off for this run");
        return PAMC_ERR_STATE;
    }
    HIPCHK(hipStreamSynchronize(stream_), "timing sync");
    double t[3] = {0.0, 0.0, 0.0};
    for (size_t j = 0; j + 4 <= ev_used_; j += 4)
        for (int p = 0; p < 3; ++p) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, ev_pool_[j + p], ev_pool_[j + p + 1]), "hipEventElapsedTime");
            t[p] += ms;
        }
    if (sweep_ms) *sweep_ms = t[0];
    if (resample_ms) *resample_ms = t[1];
    if (gather_ms) *gather_ms = t[2];
    if (n_steps) *n_steps = (int64_t)(ev_used_ / 4);
    ev_used_ = 0;
    return PAMC_OK;
}

int Runner::enqueue_steps(int n)
{
    // steps left for the active instance that is furthest from its end
    int left = 0;
    for (int i : active_) left = std::max(left, inst_[i].nT - inst_[i].k_enq);
    n = std::min(n, left);
    while (n > 0) {
        int st;
        if (graphs_ && n >= kChunkSteps) {
            st = enqueue_chunk();
            n -= kChunkSteps;
        } else {
            st = enqueue_step();
            --n;
        }
        if (st != PAMC_OK) return st;
    }
    return PAMC_OK;
}

int Runner::sync()
{
    if (poisoned_) return PAMC_ERR_DEVICE;
    HIPCHK(hipStreamSynchronize(stream_), "hipStreamSynchronize");
    return PAMC_OK;
}

int Runner::read_ctl(int i, int32_t ctl[3], uint32_t status[2])
{
    const HostInst &h = inst_[i];
    // in serving mode the instance's steps have completed: read on the
    // upload path, without waiting for the steps queued behind them
    const hipStream_t s = async_ ? side_ : stream_;
    HIPCHK(hipMemcpyAsync(ctl, h.ctl, 12, hipMemcpyDeviceToHost, s), "read ctl");
    HIPCHK(hipMemcpyAsync(status, h.dev.status, 8, hipMemcpyDeviceToHost, s), "read status");
    HIPCHK(hipStreamSynchronize(s), "read ctl sync");
    return PAMC_OK;
}

int Runner::inst_status(int i, int *step, int64_t *Rk)
{
    int32_t ctl[3];
    uint32_t status[2];
    int st = read_ctl(i, ctl, status);
    if (st != PAMC_OK) return st;
    const HostInst &h = inst_[i];
    uint32_t r = 0;
    const int k = ctl[0];
    // after the last step the population is that of step nT - 1
    st = d2h(&r, h.dev.Rk + std::min(k, h.nT - 1), 4);
    if (st != PAMC_OK) return st;
    if (step) *step = k;
    if (Rk) *Rk = r;
    if (status[0] & 1u) {
        set_error("resampling at step " + std::to_string(status[1]) + " exceeded the capacity");
        return PAMC_ERR_CAPACITY;
    }
    if (status[0] & 2u) {
        set_error("resampling at step " + std::to_string(status[1]) + " left no replica");
        return PAMC_ERR_EXTINCT;
    }
    return PAMC_OK;
}

int Runner::observables(int i, pamc_step_obs *out, int n)
{
    const HostInst &h = inst_[i];
    if (n < 0 || n > h.nT) {
        set_error("observables: n out of range");
        return PAMC_ERR_INVALID;
    }
    int32_t ctl[3];
    uint32_t status[2];
    int st = read_ctl(i, ctl, status);
    if (st != PAMC_OK) return st;
    std::vector<StepRec> rec((size_t)h.nT);
    std::vector<uint32_t> q((size_t)std::max(1, h.ovl_n) * (2 * h.N + 1));
    st = d2h(rec.data(), h.dev.rec, rec.size() * sizeof(StepRec));
    if (st == PAMC_OK) st = d2h(q.data(), h.dev.qhist, q.size() * 4);
    if (st != PAMC_OK) return st;
    // steps measured: those below the device step, plus the failing step
    int kdone = ctl[0];
    if (status[0]) kdone = (int)status[1] + 1;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const int N = h.N;
    double lnZ = h.lnZ_base;
    for (int k = 0; k < n; ++k) {
        pamc_step_obs &o = out[k];
        std::memset(&o, 0, sizeof(o));
        o.beta = h.beta[k];
        o.mean_E = o.e = o.C_V = o.lnQ = o.lnZ = o.betaF = o.f = o.S_f = o.rho_s = nan;
        o.q_abs = o.q2 = o.q4 = o.g_SG = nan;
        if (k < h.k_base || k >= kdone) continue;
        const StepRec &r = rec[k];
        o.measured = 1;
        o.R = r.R;
        o.sum_E = r.sumE;
        o.sum_E2 = (int64_t)r.sumE2;
        o.sum_E2_hi = r.sumE2_hi;
        o.E_min = r.Emin;
        o.E_max = r.Emax;
        const double Rd = (double)r.R;
        // energies in units of 2^-20 for real couplings (exact scalings)
        const double sc = h.real ? 0x1p-20 : 1.0;
        o.mean_E = ((double)r.sumE * sc) / Rd;
        o.e = o.mean_E / (double)N;
        const __int128 sum2 = (__int128)(((unsigned __int128)(uint64_t)r.sumE2_hi << 64) | r.sumE2);
        const __int128 num = (__int128)r.R * sum2 - (__int128)r.sumE * (__int128)r.sumE;
        const double var = ((double)num / (Rd * Rd)) * (sc * sc);
        o.C_V = (o.beta * o.beta) * var / (double)N;
        o.lnZ = lnZ;
        o.betaF = -lnZ;
        o.f = o.beta > 0.0 ? -lnZ / (o.beta * (double)N) : nan;
        o.S_f = std::log(Rd) - r.T / Rd;
        o.rho_s = Rd / std::exp(o.S_f);
        if (k < h.nT - 1 && k + 1 < kdone + (status[0] ? 0 : 1)) {
            const double db = h.beta[k + 1] - h.beta[k];
            o.lnQ = (-db * ((double)r.Emin * sc)) + std::log(r.S) - std::log(Rd);
            lnZ = lnZ + o.lnQ;
        }
        const int slot = h.ovl_slot[k];
        if (slot >= 0) {
            const uint32_t *hq = q.data() + (size_t)slot * (2 * N + 1);
            int64_t cnt = 0;
            double m1 = 0.0, m2 = 0.0, m4 = 0.0;
            for (int Q = -N; Q <= N; ++Q) {
                const int64_t c = hq[Q + N];
                if (c == 0) continue;
                const double qq = (double)Q / (double)N;
                cnt += c;
                m1 += (double)c * std::fabs(qq);
                m2 += (double)c * (qq * qq);
                m4 += (double)c * ((qq * qq) * (qq * qq));
            }
            if (cnt > 0) {
                o.q_abs = m1 / (double)cnt;
                o.q2 = m2 / (double)cnt;
                o.q4 = m4 / (double)cnt;
                o.g_SG = 0.5 * (3.0 - o.q4 / (o.q2 * o.q2));
            }
        }
    }
    return PAMC_OK;
}

int Runner::overlap_hist(int i, int step, int64_t *hist)
{
    const HostInst &h = inst_[i];
    if (step < 0 || step >= h.nT || h.ovl_slot[step] < 0) {
        set_error("not an overlap step");
        return PAMC_ERR_STATE;
    }
    int32_t ctl[3];
    uint32_t status[2];
    int st = read_ctl(i, ctl, status);
    if (st != PAMC_OK) return st;
    if (step >= ctl[0]) {
        set_error("overlap step has not run");
        return PAMC_ERR_STATE;
    }
    std::vector<uint32_t> q((size_t)(2 * h.N + 1));
    HIPCHK(hipMemcpy(q.data(), h.dev.qhist + (size_t)h.ovl_slot[step] * (2 * h.N + 1), q.size() * 4,
                     hipMemcpyDeviceToHost),
           "read qhist");
    for (size_t j = 0; j < q.size(); ++j) hist[j] = q[j];
    return PAMC_OK;
}

int Runner::step_sums(int i, double *S, double *T, int n)
{
    const HostInst &h = inst_[i];
    if (n < 0 || n > h.nT) return PAMC_ERR_INVALID;
    std::vector<StepRec> rec((size_t)h.nT);
    HIPCHK(hipStreamSynchronize(stream_), "sync");
    HIPCHK(hipMemcpy(rec.data(), h.dev.rec, rec.size() * sizeof(StepRec), hipMemcpyDeviceToHost), "read rec");
    for (int k = 0; k < n; ++k) {
        if (S) S[k] = rec[k].S;
        if (T) T[k] = rec[k].T;
    }
    return PAMC_OK;
}

// Bring a pending copy map into the other buffer so that rows are stored
// in order (used before export).
int Runner::materialise(int i)
{
    HostInst &h = inst_[i];
    int32_t ctl[3];
    uint32_t status[2];
    int st = read_ctl(i, ctl, status);
    if (st != PAMC_OK) return st;
    if (!ctl[2]) return PAMC_OK;
    const std::vector<Work> rows = gather_items((uint32_t)i, h.Rcap, h.srow_bytes);
    Work *d = (Work *)alloc_.get(rows.size() * sizeof(Work));
    uint32_t *l = (uint32_t *)alloc_.get(4);
    if (!d || !l) {
        alloc_.put(d);
        alloc_.put(l);
        return PAMC_ERR_NOMEM;
    }
    const uint32_t idx = (uint32_t)i;
    HIPCHK(hipMemcpy(d, rows.data(), rows.size() * sizeof(Work), hipMemcpyHostToDevice), "upload rows");
    HIPCHK(hipMemcpy(l, &idx, 4, hipMemcpyHostToDevice), "upload list");
    launch_gather(d_insts_, d, (int)rows.size(), stream_);
    launch_flip(d_insts_, l, 1, stream_);
    HIPCHK(hipGetLastError(), "gather launch");
    HIPCHK(hipStreamSynchronize(stream_), "gather sync");
    alloc_.put(d);
    alloc_.put(l);
    return PAMC_OK;
}

int Runner::get_state(int i, pamc_state *stt)
{
    HostInst &h = inst_[i];
    int st = sync();
    if (st != PAMC_OK) return st;
    st = materialise(i);
    if (st != PAMC_OK) return st;
    int32_t ctl[3];
    uint32_t status[2];
    st = read_ctl(i, ctl, status);
    if (st != PAMC_OK) return st;
    uint32_t Rk = 0;
    HIPCHK(hipMemcpy(&Rk, h.dev.Rk + std::min(ctl[0], h.nT - 1), 4, hipMemcpyDeviceToHost), "read Rk");
    if (status[0]) {
        // the failing step's population after its sweeps
        HIPCHK(hipMemcpy(&Rk, h.dev.Rk + status[1], 4, hipMemcpyDeviceToHost), "read Rk");
    }
    stt->step = ctl[0];
    stt->R = Rk;
    // ln Z at the current step
    {
        std::vector<pamc_step_obs> obs((size_t)h.nT);
        st = observables(i, obs.data(), h.nT);
        if (st != PAMC_OK) return st;
        double lnZ = h.lnZ_base;
        for (int k = h.k_base; k < ctl[0] && k < h.nT; ++k)
            if (!std::isnan(obs[k].lnQ)) lnZ = lnZ + obs[k].lnQ;
        stt->lnZ = lnZ;
    }
    const int cur = ctl[1];
    if (stt->spins) {
        std::vector<uint8_t> buf((size_t)Rk * h.srow_bytes);
        HIPCHK(hipMemcpy(buf.data(), h.dev.spins[cur], buf.size(), hipMemcpyDeviceToHost), "read spins");
        for (uint32_t r = 0; r < Rk; ++r) {
            const uint8_t *row = buf.data() + (size_t)r * h.srow_bytes;
            int8_t *o = stt->spins + (size_t)r * h.N;
            for (int s = 0; s < h.N; ++s) {
                const int p = h.lex_pos[s];
                const int up = h.packed ? (row[p >> 3] >> (p & 7)) & 1 : row[p];
                o[s] = up ? 1 : -1;
            }
        }
    }
    if (h.real) {
        if (stt->E_fixed)
            HIPCHK(hipMemcpy(stt->E_fixed, h.dev.Eq[cur], (size_t)Rk * 8, hipMemcpyDeviceToHost), "read E");
    } else if (stt->E) {
        HIPCHK(hipMemcpy(stt->E, h.dev.E[cur], (size_t)Rk * 4, hipMemcpyDeviceToHost), "read E");
    }
    if (stt->family)
        HIPCHK(hipMemcpy(stt->family, h.dev.fam[cur], (size_t)Rk * 4, hipMemcpyDeviceToHost), "read family");
    return PAMC_OK;
}

int Runner::set_state(int i, const pamc_state *st)
{
    HostInst &h = inst_[i];
    if (!st || !st->spins || !st->family || st->step < 0 || st->step >= h.nT || st->R < 1 || st->R > h.Rcap) {
        set_error("set_state: invalid state");
        return PAMC_ERR_INVALID;
    }
    const int64_t R = st->R;
    std::vector<uint8_t> buf((size_t)R * h.srow_bytes, 0);
    for (int64_t r = 0; r < R; ++r) {
        const int8_t *in = st->spins + (size_t)r * h.N;
        uint8_t *row = buf.data() + (size_t)r * h.srow_bytes;
        for (int s = 0; s < h.N; ++s) {
            if (in[s] != 1 && in[s] != -1) {
                set_error("set_state: spins must be +-1");
                return PAMC_ERR_INVALID;
            }
            const int p = h.lex_pos[s];
            if (h.packed) {
                if (in[s] > 0) row[p >> 3] |= (uint8_t)(1u << (p & 7));
            } else {
                row[p] = in[s] > 0 ? 1 : 0;
            }
        }
        if ((int64_t)st->family[r] >= h.R) {
            set_error("set_state: family id out of range");
            return PAMC_ERR_INVALID;
        }
    }
    int stt = sync();
    if (stt != PAMC_OK) return stt;
    const int32_t ctl[3] = {st->step, 0, 0};
    const uint32_t status[2] = {0, 0};
    const uint32_t Rk = (uint32_t)R;
    HIPCHK(hipMemcpy(h.dev.spins[0], buf.data(), buf.size(), hipMemcpyHostToDevice), "write spins");
    HIPCHK(hipMemcpy(h.dev.fam[0], st->family, (size_t)R * 4, hipMemcpyHostToDevice), "write family");
    HIPCHK(hipMemcpy(h.ctl, ctl, 12, hipMemcpyHostToDevice), "write ctl");
    HIPCHK(hipMemcpy(h.dev.status, status, 8, hipMemcpyHostToDevice), "write status");
    HIPCHK(hipMemcpy(h.dev.Rk + st->step, &Rk, 4, hipMemcpyHostToDevice), "write Rk");
    // energies from the spins (Eq. (1)) for the imported rows
    std::vector<Work> rows;
    for (int64_t r = 0; r < R; r += kRowsPerBlock) rows.push_back(Work{(uint32_t)i, (uint32_t)r, 0u, 0u});
    Work *d = (Work *)alloc_.get(rows.size() * sizeof(Work));
    if (!d) return PAMC_ERR_NOMEM;
    HIPCHK(hipMemcpy(d, rows.data(), rows.size() * sizeof(Work), hipMemcpyHostToDevice), "upload rows");
    launch_energy(d_insts_, d, (int)rows.size(), d_Jptr_, stream_);
    HIPCHK(hipGetLastError(), "energy launch");
    HIPCHK(hipStreamSynchronize(stream_), "energy sync");
    alloc_.put(d);
    h.k_enq = st->step;
    h.k_base = st->step;
    h.lnZ_base = st->lnZ;
    return PAMC_OK;
}

int Runner::thresholds(int i, uint32_t *out, uint8_t *acc)
{
    const HostInst &h = inst_[i];
    if (h.real) {
        set_error("thresholds: runs with real couplings take their acceptance per move (no table)");
        return PAMC_ERR_STATE;
    }
    std::vector<uint32_t> thr((size_t)h.nT * 4);
    HIPCHK(hipMemcpy(thr.data(), h.dev.thr, thr.size() * 4, hipMemcpyDeviceToHost), "read thr");
    for (int k = 0; k < h.nT; ++k) {
        if (out)
            for (int j = 0; j < 3; ++j) out[3 * k + j] = thr[4 * k + j];
        if (acc) acc[k] = (uint8_t)thr[4 * k + 3];
    }
    return PAMC_OK;
}

}  // namespace pamc
