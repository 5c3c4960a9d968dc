// resample.hip -- measurement and resampling (paper Sec. II.B, Eq. (2),
// Sec. V.A, Eq. (9)) for gfx950.
//
// Per temperature step k, after the sweeps:
//   k_measure    one block per instance: E_min, E_max, sum E, sum E^2 from
//                the energy histogram (exact integers); for k < nT-1 the
//                level weights w[m] = exp(-2 dbeta m) as a fixed product of
//                rho^(2^b), their normaliser S by a pairwise tree, and the
//                table (floor(tau), frac(tau) 2^32) with tau = R w / S;
//   k_famcount   descendants per family (wave-aggregated atomics);
//   k_famtree    pairwise tree of n ln n over family ids;
//   k_overlap    spin-overlap histogram at selected steps;
//   k_copycount  n_r = floor(tau) + [u_r < frac(tau) 2^32], block scan;
//   k_scan       prefix over blocks, R_{k+1}, capacity / extinction check;
//   k_expand     copy map: destination row -> source row (stable order).
// The floating-point work is IEEE double +, *, / in a fixed order; no
// transcendental is evaluated on the device (exp and log come from host
// tables), so results are reproducible bit for bit.
#include "pamc_dev.h"
#include "launch.h"

#pragma clang fp contract(off)

namespace pamc {

__device__ __forceinline__ bool inst_live(const Inst &I, int k) { return k < I.nT && I.status[0] == 0; }

// Block-wide reductions over 1024 threads (16 waves).
template <typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T *sh, Op op)
{
    for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    T r = sh[0];
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 1; i < nw; ++i) r = op(r, sh[i]);
    __syncthreads();
    return r;
}

// Pairwise tree sum of the n = 2^p values a[0..n) held in LDS (destroys a).
// Level by level, node i of the next level is a[2i] + a[2i+1].
__device__ double lds_pairwise(double *a, int n)
{
    for (; n > 1; n >>= 1) {
        const int h = n >> 1;
        double v = 0.0;
        if ((int)threadIdx.x < h) v = a[2 * threadIdx.x] + a[2 * threadIdx.x + 1];
        __syncthreads();
        if ((int)threadIdx.x < h) a[threadIdx.x] = v;
        __syncthreads();
    }
    return a[0];
}

// w[m] = product over the set bits b of m, ascending, of pw[b] = rho^(2^b).
__device__ __forceinline__ double level_weight(const double *pw, uint32_t m)
{
    double x = 1.0;
    for (int b = 0; m != 0; ++b, m >>= 1)
        if (m & 1u) x = x * pw[b];
    return x;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_measure(const Inst *insts, const uint32_t *list)
{
    __shared__ int64_t sh64[16];
    __shared__ int32_t sh32[16];
    __shared__ double tree[1024];
    __shared__ double pw[40];
    const Inst &I = insts[list[blockIdx.x]];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    const int N3 = 3 * I.N;
    int64_t s1 = 0, s2 = 0;
    int32_t lmin = 0x7FFFFFFF, lmax = -1;
    for (int m = threadIdx.x; m < I.nlev; m += blockDim.x) {
        const uint32_t c = I.hist[m];
        if (c) {
            const int64_t e = 2 * m - N3;
            s1 += (int64_t)c * e;
            s2 += (int64_t)c * e * e;
            lmin = min(lmin, m);
            lmax = max(lmax, m);
        }
    }
    s1 = block_reduce<int64_t>(s1, sh64, [](int64_t a, int64_t b) { return a + b; });
    s2 = block_reduce<int64_t>(s2, sh64, [](int64_t a, int64_t b) { return a + b; });
    lmin = block_reduce<int32_t>(lmin, sh32, [](int32_t a, int32_t b) { return min(a, b); });
    lmax = block_reduce<int32_t>(lmax, sh32, [](int32_t a, int32_t b) { return max(a, b); });
    StepRec *rec = I.rec + k;
    if (threadIdx.x == 0) {
        rec->R = I.Rk[k];
        rec->sumE = s1;
        rec->sumE2 = s2;
        rec->Emin = 2 * lmin - N3;
        rec->Emax = 2 * lmax - N3;
        rec->S = __builtin_nan("");
    }
    if (k < I.nT - 1) {
        if (threadIdx.x == 0) {
            pw[0] = I.rho[k];
            for (int b = 1; b < 40; ++b) pw[b] = pw[b - 1] * pw[b - 1];
        }
        __syncthreads();
        const int nl = lmax - lmin + 1;
        int P = 1;
        while (P < nl) P <<= 1;
        // each thread folds an aligned chunk of C leaves (a subtree of the
        // global pairwise tree), then the block folds the chunk roots
        const int C = P > 1024 ? P / 1024 : 1;
        const int nthr = P / C;
        double part = 0.0;
        if ((int)threadIdx.x < nthr) {
            double stack[24];
            int sp = 0;
            const int m0 = threadIdx.x * C;
            for (int i = 0; i < C; ++i) {
                const int m = m0 + i;
                double v = 0.0;
                if (m < nl) v = (double)I.hist[lmin + m] * level_weight(pw, (uint32_t)m);
                for (int j = i; j & 1; j >>= 1) v = stack[--sp] + v;
                stack[sp++] = v;
            }
            part = stack[0];
        }
        tree[threadIdx.x] = part;
        __syncthreads();
        const double S = lds_pairwise(tree, nthr);
        const double Rd = (double)I.R;
        for (int m = threadIdx.x; m < nl; m += blockDim.x) {
            const double tau = (Rd * level_weight(pw, (uint32_t)m)) / S;
            const double fl = __builtin_floor(tau);
            uint2 bf;
            bf.x = (uint32_t)fl;
            bf.y = (uint32_t)__builtin_floor((tau - fl) * 4294967296.0);
            I.BF[m] = bf;
        }
        if (threadIdx.x == 0) rec->S = S;
    }
    __syncthreads();
    for (int m = threadIdx.x; m < I.nlev; m += blockDim.x) I.hist[m] = 0u;
    // the sweep of this step moved the population to the other buffer
    if (threadIdx.x == 0 && *I.mapped) {
        *I.cur ^= 1;
        *I.mapped = 0;
    }
}

// ---------------------------------------------------------------------------
// Family sizes.  The family array is sorted, so runs of equal ids inside a
// wave are added with one atomic per run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_famcount(const Inst *insts, const Work *work)
{
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    const int Rk = (int)I.Rk[k];
    const int r = (int)w.row0 + (int)threadIdx.x;
    const bool in = r < Rk;
    const uint32_t f = in ? I.fam[*I.cur][r] : 0xFFFFFFFFu;
    const int lane = threadIdx.x & 63;
    const uint32_t fprev = __shfl_up(f, 1);
    const bool start = in && (lane == 0 || fprev != f);
    const uint64_t starts = __ballot(start);
    const uint64_t valid = __ballot(in);
    if (start) {
        const uint64_t later = lane == 63 ? 0ull : (starts >> (lane + 1));
        const int next = later ? lane + 1 + __builtin_ctzll(later) : 64;
        const int last_valid = 63 - __builtin_clzll(valid);
        const int end = min(next, last_valid + 1);
        atomicAdd(&I.cnt[f], (uint32_t)(end - lane));
    }
}

// Pairwise tree of n ln n over family ids f in [0, fam_pow2) (zero for
// families without descendants and for f >= R), in aligned chunks of 2048
// leaves; counts are cleared for the next step.
__global__ __launch_bounds__(1024) void k_famtree(const Inst *insts, const Work *chunks)
{
    __shared__ double a[1024];
    const Work w = chunks[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    const int n = min(2048, I.fam_pow2);
    const int base = (int)w.row0;
    double v = 0.0;
    const int t = threadIdx.x;
    if (2 * t < n) {
        const int f0 = base + 2 * t, f1 = f0 + 1;
        double l0 = 0.0, l1 = 0.0;
        if (f0 < I.R) {
            l0 = I.nlnn[I.cnt[f0]];
            I.cnt[f0] = 0u;
        }
        if (f1 < I.R) {
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

__global__ __launch_bounds__(1024) void k_famfinal(const Inst *insts, const uint32_t *list)
{
    __shared__ double a[1024];
    const Inst &I = insts[list[blockIdx.x]];
    const int k = *I.k;
    if (!inst_live(I, k) || I.fam_pow2 <= 2048) return;
    const int n = I.fam_pow2 / 2048;  // power of two
    // first fold pairs into LDS, then the tree
    const int C = n > 1024 ? n / 1024 : 1;
    const int nthr = n / C;
    double part = 0.0;
    if ((int)threadIdx.x < nthr) {
        double stack[24];
        int sp = 0;
        for (int i = 0; i < C; ++i) {
            double v = I.fpart[threadIdx.x * C + i];
            for (int j = i; j & 1; j >>= 1) v = stack[--sp] + v;
            stack[sp++] = v;
        }
        part = stack[0];
    }
    a[threadIdx.x] = part;
    __syncthreads();
    const double s = lds_pairwise(a, nthr);
    if (threadIdx.x == 0) I.rec[k].T = s;
}

// ---------------------------------------------------------------------------
// Overlap histogram: row r pairs with r + floor(R_k / 2).  Spins are 0/1
// bytes, so the number of differing sites is the popcount of the XOR.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_overlap(const Inst *insts, const Work *work)
{
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k)) return;
    const int slot = I.ovl_slot[k];
    if (slot < 0) return;
    const int h = (int)I.Rk[k] / 2;
    const uint8_t *sp = I.spins[*I.cur];
    const int words = I.row_bytes >> 2;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int q = wave; q < kRowsPerBlock; q += 4) {
        const int r = (int)w.row0 + q;
        if (r >= h) break;
        const uint32_t *a = reinterpret_cast<const uint32_t *>(sp + (size_t)r * I.row_bytes);
        const uint32_t *b = reinterpret_cast<const uint32_t *>(sp + (size_t)(r + h) * I.row_bytes);
        int diff = 0;
        for (int i = lane; i < words; i += 64) diff += __builtin_popcount(a[i] ^ b[i]);
        for (int off = 32; off > 0; off >>= 1) diff += __shfl_xor(diff, off);
        if (lane == 0) atomicAdd(&I.qhist[(size_t)slot * (2 * I.N + 1) + (I.N - 2 * diff) + I.N], 1u);
    }
}

// ---------------------------------------------------------------------------
// Copy counts and block-local exclusive scan (1024 rows per block).
// ---------------------------------------------------------------------------
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
    return sh[wave] + x - v;
}

__global__ __launch_bounds__(1024) void k_copycount(const Inst *insts, const Work *work)
{
    __shared__ uint32_t sh[17];
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k >= I.nT - 1) return;
    const int Rk = (int)I.Rk[k];
    if ((int)w.row0 >= Rk) {
        if (threadIdx.x == 0) I.bsum[w.row0 / kRowsPerBlock] = 0u;
        return;
    }
    const int r = (int)w.row0 + (int)threadIdx.x;
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
    if (threadIdx.x == 0) I.bsum[w.row0 / kRowsPerBlock] = total;
}

__global__ __launch_bounds__(1024) void k_scan(const Inst *insts, const uint32_t *list)
{
    __shared__ uint32_t sh[17];
    const Inst &I = insts[list[blockIdx.x]];
    const int k = *I.k;
    if (!inst_live(I, k) || k >= I.nT - 1) return;
    const int nb = ((int)I.Rk[k] + kRowsPerBlock - 1) / kRowsPerBlock;
    uint64_t carry = 0;
    for (int b0 = 0; b0 < nb; b0 += blockDim.x) {
        const int b = b0 + (int)threadIdx.x;
        const uint32_t v = b < nb ? I.bsum[b] : 0u;
        uint32_t total;
        const uint32_t off = block_exscan(v, sh, &total);
        if (b < nb) I.boff[b] = (uint32_t)(carry + off);
        carry += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        I.Rk[k + 1] = carry > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)carry;
        if (carry > (uint64_t)I.Rcap) {
            I.status[1] = (uint32_t)k;
            I.status[0] |= 1u;
        } else if (carry == 0) {
            I.status[1] = (uint32_t)k;
            I.status[0] |= 2u;
        }
    }
}

__global__ __launch_bounds__(1024) void k_expand(const Inst *insts, const Work *work)
{
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k >= I.nT - 1) return;
    const int Rk = (int)I.Rk[k];
    const int r = (int)w.row0 + (int)threadIdx.x;
    if (r < Rk) {
        const uint32_t o = I.boff[w.row0 / kRowsPerBlock] + I.loff[r];
        const uint32_t n = I.ncopy[r];
        for (uint32_t j = 0; j < n; ++j)
            if (o + j < (uint32_t)I.Rcap) I.map[o + j] = (uint32_t)r;
    }
    if (w.row0 == 0 && threadIdx.x == 0) *I.mapped = 1;
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

__global__ void k_advance(const Inst *insts, const uint32_t *list)
{
    const Inst &I = insts[list[blockIdx.x]];
    if (threadIdx.x == 0) {
        const int k = *I.k;
        if (inst_live(I, k)) *I.k = k + 1;
    }
}

// ---------------------------------------------------------------------------
void launch_measure(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_measure<<<n, 1024, 0, st>>>(insts, list);
}
void launch_famcount(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_famcount<<<nwork, 1024, 0, st>>>(insts, work);
}
void launch_famtree(const Inst *insts, const Work *chunks, int nchunks, hipStream_t st)
{
    if (nchunks) k_famtree<<<nchunks, 1024, 0, st>>>(insts, chunks);
}
void launch_famfinal(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_famfinal<<<n, 1024, 0, st>>>(insts, list);
}
void launch_overlap(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_overlap<<<nwork, 256, 0, st>>>(insts, work);
}
void launch_copycount(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_copycount<<<nwork, 1024, 0, st>>>(insts, work);
}
void launch_scan(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_scan<<<n, 1024, 0, st>>>(insts, list);
}
void launch_expand(const Inst *insts, const Work *work, int nwork, hipStream_t st)
{
    if (nwork) k_expand<<<nwork, 1024, 0, st>>>(insts, work);
}
void launch_flip(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_flip<<<n, 64, 0, st>>>(insts, list);
}
void launch_advance(const Inst *insts, const uint32_t *list, int n, hipStream_t st)
{
    if (n) k_advance<<<n, 64, 0, st>>>(insts, list);
}

}  // namespace pamc
