// resample.hip -- resampling and the per-step statistics (paper Sec. II.B,
// Eq. (2), Sec. V.A) for gfx950.
//
// After the sweep kernel (which also measured the step and prepared the
// (floor(tau), frac(tau) 2^32) table), one post launch runs three kinds of
// workgroups per instance:
//   copies    n_r = floor(tau) + [u_r < frac(tau) 2^32] for 1024 rows, with
//             their exclusive scan inside the workgroup; each also clears
//             a slice of the step's energy histogram;
//   families  n ln n of 2048 family ids, summed by the pairwise tree;
//   overlap   spin overlaps of 2048 replica pairs (at overlap steps).
// The last workgroup of an instance to finish scans the per-workgroup
// totals into offsets, sets R_{k+1} and the capacity / extinction status,
// folds the family partial sums, and advances the step.  An expand launch
// then writes the copy map (destination row -> source row, stable order),
// which the next sweep reads its tile through.
#include "launch.h"
#include "pamc_dev.h"
#include "step_common.h"

namespace pamc {

// Resampling weights with real couplings (Sec. II.B), for rows
// [row0, row0 + 1024) of one instance after the sweeps of step k:
// w_r = exp(-dbeta (E_r - E_min)) as the product over the set bits b of
// E_r - E_min (units of 2^-20) of exp(-dbeta 2^(b-20)), in ascending b.  The
// block's 1024 leaves (zero beyond R_k) form an aligned subtree of the
// pairwise tree over rows 0 .. P-1 (P the smallest power of two >= R_k); the
// last workgroup of the instance folds the block roots (zero for blocks
// beyond R_k) into the normaliser S.  For P < 1024 the block tree adds only
// zeros above the P-leaf subtree, which leaves its sum unchanged.
__global__ __launch_bounds__(512) void k_weights(const Inst *insts, const Work *work)
{
    __shared__ double pw[40];
    __shared__ double a[512];
    __shared__ double roots[512];
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k >= I.nT - 1) return;
    const int Rk = (int)I.Rk[k];
    const int t = threadIdx.x;
    if (t < 40) pw[t] = I.gpw[(size_t)k * 40 + t];
    __syncthreads();
    const long long Emin = I.rec[k].Emin;
    const int64_t *E = I.Eq[*I.cur];
    double l[2] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int r = (int)w.row0 + 2 * t + j;
        if (r < Rk) {
            const double x = weight64(pw, (uint64_t)(E[r] - Emin));
            I.wrep[r] = x;
            l[j] = x;
        }
    }
    a[t] = l[0] + l[1];
    __syncthreads();
    const double root = lds_pairwise(a, 512);
    if (t == 0) I.wpart[w.row0 / kRowsPerBlock] = root;
    if (last_workgroup(&I.sync[2], I.nblk)) {
        int P = 1;
        while (P < Rk) P <<= 1;
        const int nroot = P > kRowsPerBlock ? P / kRowsPerBlock : 1;
        const double S = tree_sum<512>(
            nroot, [&](int b) { return b * kRowsPerBlock < Rk ? I.wpart[b] : 0.0; }, a, roots);
        if (t == 0) I.rec[k].S = S;
    }
}

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
        const uint32_t u = philox10(make_uint4(0u, (uint32_t)r, (uint32_t)k, kTagResample), I.key0, I.key1).x;
        if (I.real) {
            // per-replica weight from the weights launch
            const double tau = (I.Rt[k + 1] * I.wrep[r]) / I.rec[k].S;
            const double fl = __builtin_floor(tau);
            n = (uint32_t)fl + (u < (uint32_t)__builtin_floor((tau - fl) * 4294967296.0) ? 1u : 0u);
        } else {
            const int m = (int)((I.E[*I.cur][r] - I.rec[k].Emin) >> 1);
            const uint2 bf = I.BF[m];
            n = bf.x + (u < bf.y ? 1u : 0u);
        }
    }
    uint32_t total;
    const uint32_t off = block_exscan(n, sh, &total);
    if (r < I.Rcap) I.loff[r] = off;
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

// Overlap histogram: row r pairs with r + floor(R_k / 2); this workgroup
// takes the kOvlPairs pairs from row p0.  Spins are 0/1 bytes, so the number
// of differing sites is the popcount of the XOR.  A pair is read by a group
// of lanes sized to its row (16-byte loads), several pairs per wave for
// short rows.  Low temperatures put most pairs into a few bins, so the
// counts go to an LDS histogram first and only its non-empty bins reach
// global memory.
__device__ void overlap_role(const Inst &I, int k, uint32_t p0, uint32_t *qh)
{
    const int slot = I.ovl_slot[k];
    if (slot < 0) return;
    const int h = (int)I.Rk[k] / 2;
    if ((int)p0 >= h) return;
    const int npairs = min(kOvlPairs, h - (int)p0);
    const int nb = 2 * I.N + 1;
    uint32_t *gh = I.qhist + (size_t)slot * nb;
    const bool local = nb <= kOvlLdsBins;
    if (local) {
        for (int i = threadIdx.x; i < nb; i += blockDim.x) qh[i] = 0u;
        __syncthreads();
    }
    const uint8_t *sp = I.spins[*I.cur];
    // 16-byte words of a stored row: bytes 0/1, or bits (both count the
    // differing sites as the popcount of the XOR)
    const int words = I.srow_bytes >> 4;
    int lpp = 1;  // lanes per pair, a power of two <= 64
    while (lpp < words && lpp < 64) lpp <<= 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int sub = lane / lpp, j = lane & (lpp - 1), ppw = 64 / lpp;
    for (int q0 = wave * ppw; q0 < npairs; q0 += nw * ppw) {
        const int q = q0 + sub;
        int diff = 0;
        if (q < npairs) {
            const int r = (int)p0 + q;
            const uint4 *a = reinterpret_cast<const uint4 *>(sp + (size_t)r * I.srow_bytes);
            const uint4 *b = reinterpret_cast<const uint4 *>(sp + (size_t)(r + h) * I.srow_bytes);
            for (int i = j; i < words; i += lpp) {
                const uint4 x = a[i], y = b[i];
                diff += __builtin_popcount(x.x ^ y.x) + __builtin_popcount(x.y ^ y.y) +
                        __builtin_popcount(x.z ^ y.z) + __builtin_popcount(x.w ^ y.w);
            }
        }
        for (int off = lpp >> 1; off > 0; off >>= 1) diff += __shfl_xor(diff, off);
        if (q < npairs && j == 0) {
            const int bin = (I.N - 2 * diff) + I.N;
            if (local)
                atomicAdd(&qh[bin], 1u);
            else
                atomicAdd(&gh[bin], 1u);
        }
    }
    if (local) {
        __syncthreads();
        for (int i = threadIdx.x; i < nb; i += blockDim.x) {
            const uint32_t c = qh[i];
            if (c) atomicAdd(&gh[i], c);
        }
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
    // pairwise-tree scratch, or the LDS overlap histogram
    __shared__ double a[kOvlLdsBins / 2 + 1];
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    if (w.role == kRoleCopies) {
        // the step's energy histogram (+-1 couplings) has been measured:
        // the nblk copies workgroups clear it for the next sweep, a slice
        // each, off the measurement's serial path
        if (!I.real) {
            const int per = (I.nlev + I.nblk - 1) / I.nblk;
            const int m0 = (int)(w.row0 / kRowsPerBlock) * per, m1 = min(I.nlev, m0 + per);
            for (int m = m0 + (int)threadIdx.x; m < m1; m += blockDim.x) I.hist[m] = 0u;
        }
        if (k < I.nT - 1) copies_role(I, k, w.row0, sh);
    } else if (w.role == kRoleFamilies) {
        families_role(I, k, w.row0, a);
    } else {
        overlap_role(I, k, w.row0, reinterpret_cast<uint32_t *>(a));
    }
    if (last_workgroup(&I.sync[1], I.post_blocks)) post_finish(I, k, sh, a);
}

// Copy map of the resampling of step k - 1 (the step index has advanced):
// source row r owns destination rows [off_r, off_r + n_r).  A few rows can
// own thousands of copies when the temperature step is large, so the
// workgroup of a row block walks the block's destinations instead of its
// rows: destination j belongs to the last row whose local offset is <= j.
__global__ __launch_bounds__(1024) void k_expand(const Inst *insts, const Work *work)
{
    __shared__ uint32_t off[kRowsPerBlock];
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k == 0 || !*I.mapped) return;
    const int Rold = (int)I.Rk[k - 1];
    const int row0 = (int)w.row0;
    if (row0 >= Rold) return;
    const int nrow = min(kRowsPerBlock, Rold - row0);
    const uint32_t total = I.bsum[row0 / kRowsPerBlock];
    const uint32_t base = I.boff[row0 / kRowsPerBlock];
    if (total == 0u) return;
    for (int t = threadIdx.x; t < nrow; t += blockDim.x) off[t] = I.loff[row0 + t];
    __syncthreads();
    const uint32_t lim = (uint32_t)I.Rcap - min(base, (uint32_t)I.Rcap);
    const uint32_t end = min(total, lim);
    for (uint32_t j = threadIdx.x; j < end; j += blockDim.x) {
        int p = 0;  // off[0] = 0 <= j
        for (int step = kRowsPerBlock / 2; step > 0; step >>= 1)
            if (p + step < nrow && off[p + step] <= j) p += step;
        I.map[base + j] = (uint32_t)(row0 + p);
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
void launch_weights(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_weights<<<nwork, 512, 0, st>>>(insts, work);
}
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
