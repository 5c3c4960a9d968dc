// resample.hip -- resampling and the per-step statistics (paper Sec. II.B,
// Eq. (2), Sec. V.A) for gfx950.
//
// After the sweep kernel (which also measured the step and prepared the
// (floor(tau), frac(tau) 2^32) table), one post launch runs three kinds of
// workgroups per instance:
//   copies    n_r = floor(tau) + [u_r < frac(tau) 2^32] for 1024 rows, with
//             their exclusive scan inside the workgroup;
//   families  n ln n of 2048 family ids, summed by the pairwise tree;
//   overlap   spin overlaps of 1024 replica pairs (at overlap steps).
// The last workgroup of an instance to finish scans the per-workgroup
// totals into offsets, sets R_{k+1} and the capacity / extinction status,
// folds the family partial sums, and advances the step.  An expand launch
// then writes the copy map (destination row -> source row, stable order),
// which the next sweep reads its tile through.
#include "launch.h"
#include "pamc_dev.h"
#include "step_common.h"

namespace pamc {

// Exclusive scan over the workgroup (1024 threads, 16 waves).
__device__ __forceinline__ uint32_t block_exscan(uint32_t v, uint32_t *sh, uint32_t *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < nw; ++i) {
            const uint32_t t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[16] = acc;
    }
    __syncthreads();
    *total = sh[16];
    const uint32_t r = sh[wave] + x - v;
    __syncthreads();
    return r;
}

// Copy counts of rows [row0, row0 + 1024) and their offsets in the block.
__device__ void copies_role(const Inst &I, int k, uint32_t row0, uint32_t *sh)
{
    const int Rk = (int)I.Rk[k];
    const int r = (int)row0 + (int)threadIdx.x;
    uint32_t n = 0;
    if (r < Rk) {
        const int m = (I.E[*I.cur][r] - I.rec[k].Emin) >> 1;
        const uint2 bf = I.BF[m];
        const uint32_t u = philox10(make_uint4(0u, (uint32_t)r, (uint32_t)k, kTagResample), I.key0, I.key1).x;
        n = bf.x + (u < bf.y ? 1u : 0u);
    }
    uint32_t total;
    const uint32_t off = block_exscan(n, sh, &total);
    if (r < I.Rcap) {
        I.ncopy[r] = n;
        I.loff[r] = off;
    }
    if (threadIdx.x == 0) I.bsum[row0 / kRowsPerBlock] = total;
}

// Pairwise tree of n ln n over family ids [base, base + 2048) (zero for ids
// without descendants and beyond R); the counts are cleared for the next
// step.
__device__ void families_role(const Inst &I, int k, uint32_t base, double *a)
{
    const int n = min(2048, I.fam_pow2);
    const int t = threadIdx.x;
    double v = 0.0;
    if (2 * t < n) {
        const int f0 = (int)base + 2 * t, f1 = f0 + 1;
        double l0 = 0.0, l1 = 0.0;
        if (f0 < I.R) {
            l0 = I.nlnn[I.cnt[f0]];
            I.cnt[f0] = 0u;
        }
        if (n >= 2 && f1 < I.R) {
            l1 = I.nlnn[I.cnt[f1]];
            I.cnt[f1] = 0u;
        }
        v = n >= 2 ? l0 + l1 : l0;
    }
    a[t] = v;
    __syncthreads();
    const double s = lds_pairwise(a, n >= 2 ? n / 2 : 1);
    if (threadIdx.x == 0) {
        if (I.fam_pow2 <= 2048)
            I.rec[k].T = s;
        else
            I.fpart[base / 2048] = s;
    }
}

// Overlap histogram: row r pairs with r + floor(R_k / 2).  Spins are 0/1
// bytes, so the number of differing sites is the popcount of the XOR.
__device__ void overlap_role(const Inst &I, int k, uint32_t row0)
{
    const int slot = I.ovl_slot[k];
    if (slot < 0) return;
    const int h = (int)I.Rk[k] / 2;
    const uint8_t *sp = I.spins[*I.cur];
    const int words = I.row_bytes >> 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    for (int q = wave; q < kRowsPerBlock; q += nw) {
        const int r = (int)row0 + q;
        if (r >= h) break;
        const uint32_t *a = reinterpret_cast<const uint32_t *>(sp + (size_t)r * I.row_bytes);
        const uint32_t *b = reinterpret_cast<const uint32_t *>(sp + (size_t)(r + h) * I.row_bytes);
        int diff = 0;
        for (int i = lane; i < words; i += 64) diff += __builtin_popcount(a[i] ^ b[i]);
        for (int off = 32; off > 0; off >>= 1) diff += __shfl_xor(diff, off);
        if (lane == 0) atomicAdd(&I.qhist[(size_t)slot * (2 * I.N + 1) + (I.N - 2 * diff) + I.N], 1u);
    }
}

// Last workgroup of an instance in a post launch.
__device__ void post_finish(const Inst &I, int k, uint32_t *sh, double *a)
{
    if (I.fam_pow2 > 2048) {
        const int n = I.fam_pow2 / 2048;  // power of two
        const double s = tree_sum<1024>(n, [&](int i) { return I.fpart[i]; }, a, a + 1024);
        if (threadIdx.x == 0) I.rec[k].T = s;
    }
    bool ok = true;
    if (k < I.nT - 1) {
        const int nb = ((int)I.Rk[k] + kRowsPerBlock - 1) / kRowsPerBlock;
        uint64_t carry = 0;
        for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
            const int b = b0 + (int)threadIdx.x;
            const uint32_t v = b < nb ? I.bsum[b] : 0u;
            uint32_t total;
            const uint32_t off = block_exscan(v, sh, &total);
            if (b < nb) I.boff[b] = (uint32_t)(carry + off);
            carry += total;
        }
        ok = carry > 0 && carry <= (uint64_t)I.Rcap;
        if (threadIdx.x == 0) {
            I.Rk[k + 1] = carry > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)carry;
            if (!ok) {
                I.status[1] = (uint32_t)k;
                I.status[0] |= carry == 0 ? 2u : 1u;
            } else {
                *I.mapped = 1;
            }
        }
    }
    if (threadIdx.x == 0 && ok) *I.k = k + 1;
}

__global__ __launch_bounds__(1024) void k_post(const Inst *insts, const Work *work)
{
    __shared__ uint32_t sh[17];
    __shared__ double a[2048];
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    if (w.role == kRoleCopies) {
        if (k < I.nT - 1) copies_role(I, k, w.row0, sh);
    } else if (w.role == kRoleFamilies) {
        families_role(I, k, w.row0, a);
    } else {
        overlap_role(I, k, w.row0);
    }
    if (last_workgroup(&I.sync[1], I.post_blocks)) post_finish(I, k, sh, a);
}

// Copy map of the resampling of step k - 1 (the step index has advanced):
// source row r owns destination rows [off_r, off_r + n_r).
__global__ __launch_bounds__(1024) void k_expand(const Inst *insts, const Work *work)
{
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k == 0 || !*I.mapped) return;
    const int Rold = (int)I.Rk[k - 1];
    const int r = (int)w.row0 + (int)threadIdx.x;
    if (r < Rold) {
        const uint32_t o = I.boff[w.row0 / kRowsPerBlock] + I.loff[r];
        const uint32_t n = I.ncopy[r];
        for (uint32_t j = 0; j < n; ++j)
            if (o + j < (uint32_t)I.Rcap) I.map[o + j] = (uint32_t)r;
    }
}

// After a stand-alone gather the population lives in the other buffer.
__global__ void k_flip(const Inst *insts, const uint32_t *list)
{
    const Inst &I = insts[list[blockIdx.x]];
    const int k = *I.k;
    if (threadIdx.x == 0 && inst_live(I, k) && *I.mapped) {
        *I.cur ^= 1;
        *I.mapped = 0;
    }
}

// ---------------------------------------------------------------------------
void launch_post(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_post<<<nwork, 1024, 0, st>>>(insts, work);
}
void launch_expand(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_expand<<<nwork, 1024, 0, st>>>(insts, work);
}
void launch_flip(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_flip<<<n, 64, 0, st>>>(insts, list);
}

}  // namespace pamc
