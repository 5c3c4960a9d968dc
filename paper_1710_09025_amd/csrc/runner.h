// runner.h -- host orchestration of the population annealing kernels.
//
// A Runner owns a set of instances (one for pamc_create, many for a batch or
// the serving loop), their device memory, the work lists the segmented
// kernels run over, and the stream.  Steps are enqueued without host
// synchronisation: the temperature index, the population size and the
// buffer roles of every instance live on the device.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/pamc.h"
#include "launch.h"
#include "pamc_dev.h"

namespace pamc {

struct HostInst {
    int dim = 3;                       // lattice dimension (2 or 3), N = L^dim
    int L = 0, N = 0, ncol = 0, layout = 0, variant = 0;
    int row_bytes = 0, tile_rows = 0;
    int packed = 0;                    // spins stored one bit per position
    int real = 0;                      // real couplings in fixed point (Jq)
    int icm = 0;                       // cluster-move rounds per step
    double icm_bmin = 0.0;             // ... at steps with beta_k >= icm_bmin
    int srow_bytes = 0;                // bytes per stored spin row
    int tpr = 0;                       // colour-major sweep: threads per replica
    int rp = 0;                        // colour-major sweep: replica quads per workgroup
    int64_t R = 0, Rcap = 0;
    int nT = 0, NS = 0;
    uint64_t seed = 0;
    std::vector<double> beta;
    std::vector<double> pop;           // [nT] nominal population R(beta_k)
    std::vector<int8_t> J;             // [3][N] +-1 couplings
    std::vector<int32_t> Jq;           // [dim][N] real couplings, J = Jq 2^-20
    std::vector<int32_t> ovl_slot;     // [nT]
    int ovl_n = 0;
    int k_enq = 0;                     // steps enqueued so far
    double lnZ_base = 0.0;             // ln Z at step k_base
    int k_base = 0;
    std::vector<int> lex_pos;          // lexicographic site -> storage position
    // device memory
    void *block = nullptr;             // everything of this instance
    size_t bytes = 0;
    int8_t *Jdev = nullptr;
    int32_t *ctl = nullptr;            // k, cur, mapped
    Inst dev{};                        // descriptor as uploaded
    bool poisoned = false;
};

struct Allocator {
    void *(*alloc)(size_t, void *) = nullptr;
    void (*free)(void *, void *) = nullptr;
    void *user = nullptr;
    void *get(size_t bytes);
    void put(void *p);
};

// Footprint and table construction helpers.
size_t inst_device_bytes(int L, int64_t Rcap, int nT, int n_ovl, bool packed, bool real = false, int dim = 3);
// Bytes per stored spin row: row_bytes, or one bit per position rounded up
// to 16 bytes.
int stored_row_bytes(int row_bytes, bool packed);
int64_t default_capacity(int64_t R);
// Storage layout for lattice size L, and the shape it implies.
struct LayoutInfo {
    int layout, variant, ncol;  // layout < 0: no kernel for this lattice
    int ncs[3];       // sites per colour
    int cbase[3];     // colour-major: first byte of each colour
    int row_bytes;    // bytes per replica row (multiple of 16)
    int gmax;         // Philox blocks of the largest colour
    int tpr;          // colour-major: threads per replica
};
// Real couplings use the colour-major layout for every L it covers (L = 8
// and 16 included).
LayoutInfo layout_for(int L, bool real = false, int dim = 3);

class Runner {
public:
    Runner() = default;
    ~Runner();
    // Stream, allocator and slot capacity of the device instance table.
    // external_stream: run on opt.stream even when it is NULL (the null
    // stream) instead of creating a stream of the library's own.
    int setup(const pamc_options &opt, int max_slots, bool external_stream = false);
    // Allocates an instance's device memory and tables; returns its slot
    // (>= 0) or a negative status.  The population is not initialised.
    int add_instance(HostInst &&h);
    void remove_instance(int slot);
    // Random initial population (step 0) and energies of these instances.
    int init_instances(const std::vector<int> &slots);
    // Device work lists of the segmented kernels for this active set.
    int build_work(const std::vector<int> &active);
    // Enqueue one step of every active instance not yet finished.
    int enqueue_step();
    // Enqueue up to n steps, in lock step.
    int enqueue_steps(int n);
    int sync();
    // Status of slot i after a sync: PAMC_OK / CAPACITY / EXTINCT, and its
    // device step and population.
    int inst_status(int i, int *step, int64_t *Rk);
    int observables(int i, pamc_step_obs *out, int n);
    int overlap_hist(int i, int step, int64_t *hist);
    int step_sums(int i, double *S, double *T, int n);
    int get_state(int i, pamc_state *st);
    int set_state(int i, const pamc_state *st);
    int thresholds(int i, uint32_t *out, uint8_t *acc);
    // Changes the sweep workgroup shape of slot i (between steps; results
    // do not depend on it) and rebuilds the work lists of the active set.
    int set_shape(int i, int tile_rows, int rp);
    const HostInst &inst(int i) const { return inst_[i]; }
    HostInst &inst(int i) { return inst_[i]; }
    const std::vector<int> &active() const { return active_; }
    hipStream_t stream() const { return stream_; }
    bool fused() const { return fuse_; }
    bool poisoned() const { return poisoned_; }
    // Sums of the recorded per-step event intervals since the last call.
    int phase_times(double *sweep_ms, double *resample_ms, double *gather_ms, int64_t *n_steps);
    bool timing() const { return timing_; }

    // Serving mode.  Instance uploads, initial populations, work-list
    // uploads and result reads go through a second stream from pinned
    // staging, so they never wait for the steps queued on the main stream;
    // an instance removed or a work list replaced while queued steps may
    // still read it is released only when an event recorded behind those
    // steps has completed (its slot is not reused before).  Reads of an
    // instance's results assume its last step has completed.
    int enable_async(size_t staging_bytes);
    bool async() const { return async_; }
    // Releases what retired fences hold once their events have completed
    // (wait: waits for all of them first).
    int release_fenced(bool wait);
    // Slots free for add_instance (not in use, not held by a fence).
    int free_slots() const;
    // Sizes the shared n ln n table for populations up to len - 1 rows.
    int reserve_nlnn(int64_t len) { return ensure_nlnn(len); }

private:
    // Host-to-device copy through the upload path (the main stream, or in
    // serving mode the second stream from pinned staging); upload_sync
    // waits for the path's copies and kernels.
    int h2d(void *dst, const void *src, size_t bytes);
    int upload_sync();
    // Device-to-host copy of data no queued work still writes, waited for.
    int d2h(void *dst, const void *src, size_t bytes);
    hipStream_t up_stream() const { return async_ ? side_ : stream_; }
    // Holds ptrs and slots until the steps enqueued so far have run.
    int fence(std::vector<void *> ptrs, std::vector<int> slots);
    int upload_inst(int i);
    int ensure_nlnn(int64_t len);
    int read_ctl(int i, int32_t ctl[3], uint32_t status[2]);
    int materialise(int i);
    int dev_fail(hipError_t e, const char *what);

    std::vector<HostInst> inst_;   // by slot
    std::vector<char> used_;       // slot in use
    Allocator alloc_;
    hipStream_t stream_ = nullptr;
    bool own_stream_ = false;
    bool fuse_ = true;
    bool poisoned_ = false;
    int device_ = 0;
    int max_slots_ = 0;

    // shared device data
    Inst *d_insts_ = nullptr;      // [max_slots]
    const int8_t **d_Jptr_ = nullptr;
    double *d_nlnn_ = nullptr;
    int64_t nlnn_len_ = 0;

    // work lists for the current active set
    struct SweepGroup {
        int variant, tile_rows, row_bytes, tpr, rp, icm;
        Work *work;
        int nwork;
    };
    std::vector<SweepGroup> sweep_groups_;
    // Runs of several instances sweep their shape groups side by side: the
    // groups go round-robin to the main stream and these, which start after
    // the fork event on the main stream and rejoin it before the resampling.
    static constexpr int kAuxStreams = 2;
    std::vector<hipStream_t> aux_;
    hipEvent_t ev_fork_ = nullptr;
    std::vector<hipEvent_t> ev_join_;
    Work *d_rows_ = nullptr;   // 1024-row blocks (expand)
    int nrows_work_ = 0;
    Work *d_wblk_ = nullptr;   // 1024-row blocks of instances with real couplings (weights)
    int nwblk_ = 0;
    Work *d_icm_ = nullptr;    // replica pairs of instances with cluster moves
    int nicm_ = 0, icm_rounds_ = 0, icm_N_ = 0;
    Work *d_gather_ = nullptr; // row blocks of about 32 KB of spins (stand-alone gather)
    int ngather_ = 0;
    Work *d_post_ = nullptr;   // post-launch workgroups with their roles
    int npost_ = 0;
    uint32_t *d_list_ = nullptr;
    int nlist_ = 0;
    std::vector<void *> work_allocs_;
    std::vector<int> active_;
    // one captured temperature step, replayed for every step, and a
    // captured chunk of kChunkSteps steps for runs of whole chunks
    static constexpr int kChunkSteps = 16;
    bool graphs_ = true;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr;
    hipGraph_t chunk_graph_ = nullptr;
    hipGraphExec_t chunk_exec_ = nullptr;
    void drop_graph();
    int launch_step_kernels();
    int enqueue_chunk();
    void count_enqueued(int steps);
    // timing: four events per enqueued step (before the sweeps, after the
    // sweeps, after the resampling, after the stand-alone gather), reused
    // from a pool
    bool timing_ = false;
    std::vector<hipEvent_t> ev_pool_;
    size_t ev_used_ = 0;
    // serving mode
    bool async_ = false;
    hipStream_t side_ = nullptr;
    uint8_t *stage_ = nullptr;       // pinned host staging
    size_t stage_cap_ = 0, stage_used_ = 0;
    struct Fenced {
        hipEvent_t ev;
        std::vector<void *> ptrs;
        std::vector<int> slots;
    };
    std::vector<Fenced> fenced_;
    std::vector<hipEvent_t> fence_pool_;
    std::vector<char> held_;         // slot retired, its fence pending
};

void set_error(const std::string &msg);
// Work items of the stand-alone gather of instance slot i: blocks of about
// 32 KB of spin rows, the row count in Work::pad.
std::vector<Work> gather_items(uint32_t slot, int64_t Rcap, int row_bytes);

}  // namespace pamc
