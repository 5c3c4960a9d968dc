// icm.hip -- isoenergetic cluster moves between replica pairs (paper Sec. IV,
// the Houdayer-type update in the variant the paper describes) for gfx950.
//
// At every step after a resampling the sweep launch stops after floor(N_S/2)
// sweeps; then each ICM round pairs the rows of the population at random and
// updates every pair at once (pairs are disjoint), and the remaining sweeps
// follow.  One update: the overlap q_s = S^a_s S^b_s splits the sites into
// the sector where the replicas differ (q = -1) and where they agree
// (q = +1); the sector with fewer sites (the differing one on a tie) is
// taken, a site of it is drawn, and the island of that site -- the sites of
// the sector connected to it through lattice bonds -- is flipped in both
// replicas, which leaves their summed energy unchanged (the move is always
// accepted).
//
// Random numbers: round rd pairs rows pi(2j) and pi(2j+1), j < floor(R_k/2),
// with pi a keyed pseudo-random permutation of [0, R_k): a four-round
// balanced Feistel network on 2h-bit words (4^h >= R_k) whose round function
// j is word 0 of Philox at counter (half-word, j, k, TAG_ICM | rd), applied
// repeatedly until the value falls in [0, R_k) (cycle walking).  The drawn
// site is the m-th site of the sector in lexicographic order,
// m = floor(u count / 2^32), u = word 0 of Philox at (j, 4, k, TAG_ICM | rd).
#include "launch.h"
#include "pamc_dev.h"
#include "step_common.h"

namespace pamc {

__device__ uint32_t icm_perm(uint32_t key0, uint32_t key1, uint32_t i, uint32_t n, int k, int round)
{
    int h = 0;
    while (((uint64_t)1 << (2 * h)) < (uint64_t)n) ++h;
    const uint32_t mask = h == 0 ? 0u : (uint32_t)(((uint64_t)1 << h) - 1);
    uint32_t x = i;
    do {
        uint32_t l = h == 0 ? 0u : x >> h, r = x & mask;
        for (int j = 0; j < 4; ++j) {
            const uint32_t f =
                philox10(make_uint4(r, (uint32_t)j, (uint32_t)k, kTagIcm | (uint32_t)round), key0, key1).x & mask;
            const uint32_t t = l ^ f;
            l = r;
            r = t;
        }
        x = h == 0 ? 0u : ((l << h) | r);
    } while (x >= n);
    return x;
}

// LDS of one pair: the sector flag of every lexicographic site (bytes), the
// visited bits, and the island queue (site indices, N <= 32768).
__host__ __device__ inline size_t icm_lds_bytes(int N)
{
    return (size_t)((N + 15) & ~15) + 4 * (size_t)((N + 31) / 32) + 2 * (size_t)N + 16;
}

// Exclusive scan over the workgroup (a multiple of 64 threads, <= 1024).
__device__ __forceinline__ int icm_exscan(int v, int *sh, int *total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)blockDim.x >> 6;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < nw; ++i) {
            const int t = sh[i];
            sh[i] = acc;
            acc += t;
        }
        sh[16] = acc;
    }
    __syncthreads();
    *total = sh[16];
    const int r = sh[wave] + x - v;
    __syncthreads();
    return r;
}

// One ICM round: work item = (instance, pair index j).
__global__ __launch_bounds__(256) void k_icm(const Inst *insts, const Work *work, int round)
{
    extern __shared__ __align__(16) uint8_t lds[];
    __shared__ uint32_t rows[2];
    __shared__ int sh[17];
    __shared__ int sh_tail;
    const Work w = work[blockIdx.x];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k == 0 || round >= I.icm) return;
    const uint32_t n = I.Rk[k];
    const uint32_t j = w.row0;
    if (j >= n / 2) return;
    const int N = I.N, L = I.L, t = (int)threadIdx.x, bd = (int)blockDim.x;
    uint8_t *member = lds;
    uint32_t *vis = reinterpret_cast<uint32_t *>(lds + ((N + 15) & ~15));
    uint16_t *queue = reinterpret_cast<uint16_t *>(lds + ((N + 15) & ~15) + 4 * ((N + 31) / 32));
    if (t == 0) {
        rows[0] = icm_perm(I.key0, I.key1, 2 * j, n, k, round);
        rows[1] = icm_perm(I.key0, I.key1, 2 * j + 1, n, k, round);
    }
    __syncthreads();
    uint8_t *sp = I.spins[*I.cur];
    uint8_t *A = sp + (size_t)rows[0] * I.srow_bytes;
    uint8_t *B = sp + (size_t)rows[1] * I.srow_bytes;
    // sites where the replicas differ
    int nd = 0;
    for (int s = t; s < N; s += bd) {
        const int p = I.pos[s];
        const uint8_t d = A[p] != B[p] ? 1 : 0;
        member[s] = d;
        nd += d;
    }
    for (int i = t; i < (N + 31) / 32; i += bd) vis[i] = 0u;
    int total;
    (void)icm_exscan(nd, sh, &total);
    nd = total;
    const bool want = nd <= N - nd;
    const int cnt = want ? nd : N - nd;
    if (cnt == 0) return;  // empty sector: no move (uniform over the workgroup)
    if (!want)
        for (int s = t; s < N; s += bd) member[s] ^= 1u;
    __syncthreads();
    // the m-th site of the sector, found through per-thread chunk counts
    const uint32_t u = philox10(make_uint4(j, 4u, (uint32_t)k, kTagIcm | (uint32_t)round), I.key0, I.key1).x;
    const int m = (int)(((uint64_t)u * (uint64_t)cnt) >> 32);
    const int chunk = (N + bd - 1) / bd;
    const int s_begin = min(N, t * chunk), s_end = min(N, s_begin + chunk);
    int c = 0;
    for (int s = s_begin; s < s_end; ++s) c += member[s];
    const int off = icm_exscan(c, sh, &total);
    if (off <= m && m < off + c) {
        int seen = off;
        for (int s = s_begin; s < s_end; ++s)
            if (member[s]) {
                if (seen == m) {
                    queue[0] = (uint16_t)s;
                    vis[s >> 5] = 1u << (s & 31);
                    break;
                }
                ++seen;
            }
    }
    if (t == 0) sh_tail = 1;
    __syncthreads();
    // breadth-first growth of the island, one frontier per iteration; the
    // queue only grows and holds each site once, so this ends within N
    // iterations
    int head = 0;
    while (true) {
        const int tail = sh_tail;
        if (head >= tail) break;
        __syncthreads();
        for (int idx = head + t; idx < tail; idx += bd) {
            const int s = queue[idx];
            const int x = s % L, yz = s / L, y = yz % L, z = yz / L;
            const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
            const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
            const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
            const int nb[6] = {xp + L * yz, xm + L * yz, x + L * (yp + L * z), x + L * (ym + L * z),
                               x + L * (y + L * zp), x + L * (y + L * zm)};
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                const int q = nb[d];
                if (!member[q]) continue;
                const uint32_t bit = 1u << (q & 31);
                if (atomicOr(&vis[q >> 5], bit) & bit) continue;
                queue[atomicAdd(&sh_tail, 1)] = (uint16_t)q;
            }
        }
        head = tail;
        __syncthreads();
    }
    // flip the island in both replicas
    const int size = sh_tail;
    for (int idx = t; idx < size; idx += bd) {
        const int p = I.pos[queue[idx]];
        A[p] ^= 1u;
        B[p] ^= 1u;
    }
}

hipError_t icm_kernels_init()
{
    return hipFuncSetAttribute(reinterpret_cast<const void *>(&k_icm), hipFuncAttributeMaxDynamicSharedMemorySize,
                               kMaxSweepLds);
}

void launch_icm(const Inst *insts, const Work *work, int nwork, int N, int round, hipStream_t st)
{
    if (nwork) k_icm<<<nwork, 256, icm_lds_bytes(N), st>>>(insts, work, round);
}

}  // namespace pamc
