// step_common.h -- device routines shared by the sweep and resampling
// kernels: the Philox4x32-10 generator, block reductions, the fixed pairwise
// summation tree, counting with one atomic per distinct address of a wave,
// the end-of-launch detection of the last workgroup of an instance, and the
// measurement of a temperature step (paper Sec. II.B: reweighting factors
// exp[-(beta'-beta) E_i] normalised to the nominal population R(beta')).
#pragma once
#include "pamc_dev.h"

#pragma clang fp contract(off)

namespace pamc {

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation with
// the truth table of a three-way exclusive or.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Each round multiplies
// counter words 0 and 2 by the round multipliers, the high halves mixed with
// words 1 and 3 and the round key; the key advances by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t a = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t b = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        uint4 n;
        n.x = xor3((uint32_t)(b >> 32), c.y, k0);
        n.y = (uint32_t)b;
        n.z = xor3((uint32_t)(a >> 32), c.w, k1);
        n.w = (uint32_t)a;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t word_of(uint4 v, int i)
{
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

__device__ __forceinline__ bool inst_live(const Inst &I, int k) { return k < I.nT && I.status[0] == 0; }

// Reduction over the block (any multiple of 64 threads up to 1024); sh holds
// one value per wave.
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

// Pairwise tree sum of the n = 2^p values a[0..n) held in LDS (destroys a):
// level by level, node i of the next level is a[2i] + a[2i+1].
// n <= 2 blockDim.
__device__ __forceinline__ double lds_pairwise(double *a, int n)
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

// Pairwise tree sum of n = 2^p leaves leaf(0..n).  T = the largest power of
// two <= min(blockDim, NT) threads take part: aligned chunks of 2T leaves
// are subtrees of the global tree; each is folded in LDS, then the chunk
// roots are folded.  a and roots hold NT doubles each; n <= 2 T NT.
template <int NT, typename Leaf>
__device__ __forceinline__ double tree_sum(int n, Leaf leaf, double *a, double *roots)
{
    const int t = threadIdx.x;
    int T = 1;
    while (2 * T <= (int)blockDim.x && 2 * T <= NT) T <<= 1;
    if (n == 1) {
        if (t == 0) a[0] = leaf(0);
        __syncthreads();
        const double r = a[0];
        __syncthreads();
        return r;
    }
    const int chunk = 2 * T;
    if (n <= chunk) {
        if (t < T) a[t] = 2 * t < n ? leaf(2 * t) + leaf(2 * t + 1) : 0.0;
        __syncthreads();
        return lds_pairwise(a, n / 2);
    }
    const int nchunks = n / chunk;
    for (int c = 0; c < nchunks; ++c) {
        if (t < T) a[t] = leaf(c * chunk + 2 * t) + leaf(c * chunk + 2 * t + 1);
        __syncthreads();
        const double r = lds_pairwise(a, T);
        if (t == 0) roots[c] = r;
    }
    __syncthreads();
    return lds_pairwise(roots, nchunks);
}

// w[m] = product over the set bits b of m, ascending, of pw[b] = rho^(2^b).
__device__ __forceinline__ double level_weight(const double *pw, uint32_t m)
{
    double x = 1.0;
    for (int b = 0; m != 0; ++b, m >>= 1)
        if (m & 1u) x = x * pw[b];
    return x;
}

// w = product over the set bits b of D (< 2^40), ascending, of pw[b].
__device__ __forceinline__ double weight64(const double *pw, uint64_t D)
{
    double x = 1.0;
    for (int b = 0; D != 0; ++b, D >>= 1)
        if (D & 1u) x = x * pw[b];
    return x;
}

// ---------------------------------------------------------------------------
// Metropolis acceptance with real couplings.  exp(x) in binary32 for
// -23 <= x <= 0 by a fixed recipe of correctly rounded steps: Cody-Waite
// reduction x = n ln 2 + r, n = rint(x log2 e), with ln 2 split into a head
// of 16 significant bits (n times it is exact) and a tail; the Taylor
// polynomial of degree 7 in r (|r| <= ln(2)/2) by Horner's rule with fused
// multiply-adds; scaling by 2^n.  Any IEEE implementation of the same steps
// returns the same bits, so decisions are reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float exp_recipe(float x)
{
    const float n = __builtin_rintf(x * 1.44269504f);
    float r = __builtin_fmaf(-n, 0.693145751953125f, x);
    r = __builtin_fmaf(-n, 1.42860677e-06f, r);
    float p = 1.0f / 5040.0f;
    p = __builtin_fmaf(p, r, 1.0f / 720.0f);
    p = __builtin_fmaf(p, r, 1.0f / 120.0f);
    p = __builtin_fmaf(p, r, 1.0f / 24.0f);
    p = __builtin_fmaf(p, r, 1.0f / 6.0f);
    p = __builtin_fmaf(p, r, 0.5f);
    p = __builtin_fmaf(p, r, 1.0f);
    p = __builtin_fmaf(p, r, 1.0f);
    return __builtin_ldexpf(p, (int)n);
}

// A move with dE > 0 (units of 2^-20) at bq = beta 2^-20 (binary32) is
// accepted when x = -(bq dE) >= -23 and e = exp(x) >= 1 or u < floor(e 2^32).
// The recipe's argument is x clamped to [-24, 0] (dE <= 0 taken as 0): every
// decision is unchanged and its conversions stay in range for any dE.
__device__ __forceinline__ bool real_accept(float bq, int32_t dE, uint32_t u)
{
    const float x = -(bq * (float)max(dE, 0));
    const float e = exp_recipe(__builtin_fmaxf(x, -24.0f));
    const uint32_t T = (uint32_t)((e < 1.0f ? e : 0.0f) * 4294967296.0f);
    return x >= -23.0f && (e >= 1.0f || u < T);
}

// Adds one count per valid lane to arr[idx], one atomic per distinct index
// of the wave: at low temperature most replicas share a few energies (and
// sorted families share ids), and per-lane atomics on one address would
// serialise.  Every lane of the wave must call it.
__device__ __forceinline__ void count_wave(uint32_t *arr, uint32_t idx, bool valid)
{
    const int lane = threadIdx.x & 63;
    uint64_t pending = __ballot(valid);
    while (pending) {
        const int leader = __builtin_ctzll(pending);
        const uint32_t li = __shfl(idx, leader);
        const uint64_t same = __ballot(valid && idx == li) & pending;
        if (lane == leader) atomicAdd(&arr[li], (uint32_t)__builtin_popcountll(same));
        pending &= ~same;
    }
}

// Called by every workgroup of an instance at the end of its work in a
// launch: returns true in exactly one workgroup, the last to finish, after
// which the writes of all the others are visible to it.  Each workgroup
// releases its writes (device scope: an L2 write-back, the L2s of the XCDs
// not being coherent) before it counts itself in; only the last one
// acquires (an L2 invalidate).  A full fence in every workgroup would also
// invalidate the L2 under all the workgroups still running.
__device__ __forceinline__ bool last_workgroup(uint32_t *counter, int expected)
{
    __shared__ int is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        is_last = atomicAdd(counter, 1u) == (uint32_t)(expected - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *counter = 0u;
    return true;
}

// Measurement of step k after its sweeps, by one workgroup (blockDim a power
// of two, <= 1024): E_min, E_max, sum E, sum E^2 from the energy histogram
// (exact integers), and for k < nT-1 the level weights w[m] = exp(-2 dbeta m)
// as a fixed product of rho^(2^b), their normaliser S by the pairwise tree
// over 2^ceil(log2(M+1)) levels, and the table (floor(tau), floor(frac(tau)
// 2^32)) with tau = R w / S.  Moves the buffer roles on when the sweep wrote
// the other buffer; the post launch that follows clears the histogram.  NT
// bounds the workgroup size (scratch capacity); any workgroup of a multiple
// of 64 threads works.  This runs in one workgroup while the rest of the GPU
// waits, so every global load it needs is issued as early as possible.
template <int NT>
__device__ void measure_step(const Inst &I, int k)
{
    __shared__ int64_t sh64[2][16];
    __shared__ int32_t sh32[2][16];
    __shared__ double tree[NT];
    __shared__ double roots[NT];
    __shared__ double pw[40];
    const bool resample = k < I.nT - 1;
    // loaded before the histogram pass so that their latency overlaps it
    const double rho_k = resample ? I.rho[k] : 1.0;
    const double Rd = resample ? I.Rt[k + 1] : 0.0;  // nominal population at beta_{k+1}
    const uint32_t Rk = I.Rk[k];
    const int N3 = 3 * I.N, nlev = I.nlev, nt = (int)blockDim.x;
    int64_t s1 = 0, s2 = 0;
    int32_t lmin = 0x7FFFFFFF, lmax = -1;
    // the counts come from memory (the election invalidated the L2): each
    // thread issues its loads eight at a time before using any of them, so
    // the pass waits for about one memory latency per eight levels per
    // thread rather than one per level
    for (int base = threadIdx.x; base < nlev; base += 8 * nt) {
        uint32_t c[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int m = base + u * nt;
            c[u] = m < nlev ? I.hist[m] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            if (!c[u]) continue;
            const int m = base + u * nt;
            const int64_t e = 2 * m - N3;
            s1 += (int64_t)c[u] * e;
            s2 += (int64_t)c[u] * e * e;
            lmin = min(lmin, m);
            lmax = max(lmax, m);
        }
    }
    // the four reductions in one pass: within each wave, then over the waves
    for (int off = 32; off > 0; off >>= 1) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
        lmin = min(lmin, __shfl_xor(lmin, off));
        lmax = max(lmax, __shfl_xor(lmax, off));
    }
    {
        const int wave = threadIdx.x >> 6, nw = (nt + 63) >> 6;
        if ((threadIdx.x & 63) == 0) {
            sh64[0][wave] = s1;
            sh64[1][wave] = s2;
            sh32[0][wave] = lmin;
            sh32[1][wave] = lmax;
        }
        __syncthreads();
        s1 = sh64[0][0];
        s2 = sh64[1][0];
        lmin = sh32[0][0];
        lmax = sh32[1][0];
        for (int i = 1; i < nw; ++i) {
            s1 += sh64[0][i];
            s2 += sh64[1][i];
            lmin = min(lmin, sh32[0][i]);
            lmax = max(lmax, sh32[1][i]);
        }
    }
    StepRec *rec = I.rec + k;
    if (threadIdx.x == 0) {
        rec->R = Rk;
        rec->sumE = s1;
        rec->sumE2 = (uint64_t)s2;
        rec->sumE2_hi = 0;
        rec->Emin = 2 * lmin - N3;
        rec->Emax = 2 * lmax - N3;
        rec->S = __builtin_nan("");
    }
    if (resample) {
        if (threadIdx.x == 0) {
            pw[0] = rho_k;
            for (int b = 1; b < 40; ++b) pw[b] = pw[b - 1] * pw[b - 1];
        }
        __syncthreads();
        const int nl = lmax - lmin + 1;
        int P = 1;
        while (P < nl) P <<= 1;
        const double S = tree_sum<NT>(
            P,
            [&](int m) { return m < nl ? (double)I.hist[lmin + m] * level_weight(pw, (uint32_t)m) : 0.0; },
            tree, roots);
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
    // the sweep of this step moved the population to the other buffer
    if (threadIdx.x == 0 && *I.mapped) {
        *I.cur ^= 1;
        *I.mapped = 0;
    }
}

// Measurement of step k with real couplings, by the last sweep workgroup:
// the energy moments the tiles accumulated (exact integers) go to the step
// record and are reset for the next step; the weights and the normaliser
// follow in the weights launch.  Moves the buffer roles on when the sweep
// wrote the other buffer.
__device__ __forceinline__ void measure_step_real(const Inst &I, int k)
{
    if (threadIdx.x != 0) return;
    EMoments *m = I.emom;
    StepRec *rec = I.rec + k;
    rec->R = I.Rk[k];
    rec->sumE = (int64_t)m->sum;
    rec->sumE2 = m->sq_lo;
    rec->sumE2_hi = (int64_t)m->sq_hi;
    rec->Emin = m->emin;
    rec->Emax = m->emax;
    rec->S = __builtin_nan("");
    m->emin = 0x7FFFFFFFFFFFFFFFll;
    m->emax = -0x7FFFFFFFFFFFFFFFll - 1;
    m->sum = 0ull;
    m->sq_lo = 0ull;
    m->sq_hi = 0ull;
    if (*I.mapped) {
        *I.cur ^= 1;
        *I.mapped = 0;
    }
}

}  // namespace pamc
