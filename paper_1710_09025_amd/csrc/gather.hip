// gather.hip -- stand-alone copy of the surviving replicas into the other
// population buffer (the gather step of the resampling, paper Sec. II.B), for
// gfx950.  The default path fuses this copy into the next sweep's tile load;
// this kernel serves runs with the fusion off and the export of a population.
#include "launch.h"
#include "pamc_dev.h"

namespace pamc {

// ---------------------------------------------------------------------------
// Stand-alone gather of surviving replicas: destination row d of the other
// buffer receives source row map[d] (spins, energy, family).  Used when the
// gather is not fused into the next sweep and to materialise a population
// for export.  Runs after the step index has moved to the new population;
// a one-workgroup launch then moves the buffer roles on.  (Having the last
// workgroup of the gather do that instead costs a device-scope release fence
// in every one of its many short workgroups, which slowed the gather about
// five-fold.)
// A work item is a block of w.pad destination rows (about 32 KB of spins);
// each thread keeps four 16-byte loads in flight before its stores.  The
// rows are written with nontemporal (streaming) stores: the new population
// is not read again before the next sweep, and ordinary stores let it evict
// the source rows from the caches, which costs a third to half of the
// bandwidth at these sizes.
// ---------------------------------------------------------------------------
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_streaming(uint4 *p, uint4 v)
{
    const u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4 *>(p));
}

__global__ __launch_bounds__(256) void k_gather(const Inst *insts, const Work *work)
{
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (k >= I.nT || I.status[0] || !*I.mapped) return;
    const int Rn = (int)I.Rk[k];
    const int row0 = (int)w.row0;
    const int rows = min((int)w.pad, Rn - row0);
    if (rows <= 0) return;
    const int cur = *I.cur;
    const int per_row = I.srow_bytes >> 4;
    const int total = rows * per_row;
    const uint4 *src = reinterpret_cast<const uint4 *>(I.spins[cur]);
    uint4 *dst = reinterpret_cast<uint4 *>(I.spins[cur ^ 1]);
    const int nt = (int)blockDim.x;
    for (int base = threadIdx.x; base < total; base += 4 * nt) {
        uint4 v[4];
        size_t to[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int it = base + u * nt;
            if (it < total) {
                const int q = it / per_row, c = it - q * per_row;
                const uint32_t d = (uint32_t)(row0 + q);
                v[u] = src[(size_t)I.map[d] * per_row + c];
                to[u] = (size_t)d * per_row + c;
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (base + u * nt < total) store_streaming(dst + to[u], v[u]);
    }
    for (int q = threadIdx.x; q < rows; q += nt) {
        const uint32_t d = (uint32_t)(row0 + q), s = I.map[d];
        if (I.real)
            I.Eq[cur ^ 1][d] = I.Eq[cur][s];
        else
            I.E[cur ^ 1][d] = I.E[cur][s];
        I.fam[cur ^ 1][d] = I.fam[cur][s];
    }
}

void launch_gather(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_gather<<<nwork, 256, 0, st>>>(insts, work);
}

}  // namespace pamc
