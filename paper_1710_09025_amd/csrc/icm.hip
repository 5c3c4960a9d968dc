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
#include <algorithm>

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

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_sum(int v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// One ICM round.  Each wave of the workgroup updates one pair (work item =
// instance, pair index j) on its own slice of LDS, so the island search
// synchronises only inside its wave.
__global__ __launch_bounds__(256) void k_icm(const Inst *insts, const Work *work, int nwork, int round, int pair_bytes)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const int item = (int)blockIdx.x * ((int)blockDim.x >> 6) + wave;
    if (item >= nwork) return;
    const Work w = work[item];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k == 0 || round >= I.icm || !(I.beta[k] >= I.icm_bmin)) return;
    const uint32_t n = I.Rk[k];
    const uint32_t j = w.row0;
    if (j >= n / 2) return;
    const int N = I.N, L = I.L, nnb = 2 * I.dim;
    uint8_t *base = lds + (size_t)wave * pair_bytes;
    uint8_t *member = base;
    uint32_t *vis = reinterpret_cast<uint32_t *>(base + ((N + 15) & ~15));
    uint16_t *queue = reinterpret_cast<uint16_t *>(base + ((N + 15) & ~15) + 4 * ((N + 31) / 32));
    int *tailp = reinterpret_cast<int *>(base + pair_bytes - 16);
    // the pair's rows: pi(2j) on lane 0, pi(2j + 1) on lane 1
    uint32_t row = 0;
    if (lane < 2) row = icm_perm(I.key0, I.key1, 2 * j + (uint32_t)lane, n, k, round);
    const uint32_t ra = __shfl(row, 0), rb = __shfl(row, 1);
    uint8_t *sp = I.spins[*I.cur];
    uint8_t *A = sp + (size_t)ra * I.srow_bytes;
    uint8_t *B = sp + (size_t)rb * I.srow_bytes;
    // sites where the replicas differ
    int nd = 0;
    for (int s = lane; s < N; s += 64) {
        const int p = I.pos[s];
        const uint8_t d = A[p] != B[p] ? 1 : 0;
        member[s] = d;
        nd += d;
    }
    for (int i = lane; i < (N + 31) / 32; i += 64) vis[i] = 0u;
    nd = wave_sum(nd);
    const bool want = nd <= N - nd;
    const int cnt = want ? nd : N - nd;
    if (cnt == 0) return;  // empty sector: no move (uniform over the wave)
    if (!want)
        for (int s = lane; s < N; s += 64) member[s] ^= 1u;
    wave_sync();
    // the m-th site of the sector, through per-lane chunk counts
    const uint32_t u = philox10(make_uint4(j, 4u, (uint32_t)k, kTagIcm | (uint32_t)round), I.key0, I.key1).x;
    const int m = (int)(((uint64_t)u * (uint64_t)cnt) >> 32);
    const int chunk = (N + 63) / 64;
    const int s_begin = min(N, lane * chunk), s_end = min(N, s_begin + chunk);
    int c = 0;
    for (int s = s_begin; s < s_end; ++s) c += member[s];
    int incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
    }
    const int excl = incl - c;
    if (excl <= m && m < incl) {
        int seen = excl;
        for (int s = s_begin; s < s_end; ++s)
            if (member[s]) {
                if (seen == m) {
                    queue[0] = (uint16_t)s;
                    vis[s >> 5] = 1u << (s & 31);
                    *tailp = 1;
                    break;
                }
                ++seen;
            }
    }
    wave_sync();
    // breadth-first growth of the island, one frontier per iteration; the
    // queue only grows and holds each site once, so this ends within N
    // iterations
    int head = 0;
    while (true) {
        const int tail = *reinterpret_cast<volatile int *>(tailp);
        if (head >= tail) break;
        wave_sync();
        for (int idx = head + lane; idx < tail; idx += 64) {
            const int s = queue[idx];
            const int x = s % L, yz = s / L, y = yz % L, z = yz / L;
            const int xp = x + 1 == L ? 0 : x + 1, xm = x == 0 ? L - 1 : x - 1;
            const int yp = y + 1 == L ? 0 : y + 1, ym = y == 0 ? L - 1 : y - 1;
            const int zp = z + 1 == L ? 0 : z + 1, zm = z == 0 ? L - 1 : z - 1;
            // on the square lattice (z = 0) only the first four are bonds
            const int nb[6] = {xp + L * yz, xm + L * yz, x + L * (yp + L * z), x + L * (ym + L * z),
                               x + L * (y + L * zp), x + L * (y + L * zm)};
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                if (d >= nnb) break;
                const int q = nb[d];
                if (!member[q]) continue;
                const uint32_t bit = 1u << (q & 31);
                if (atomicOr(&vis[q >> 5], bit) & bit) continue;
                queue[atomicAdd(tailp, 1)] = (uint16_t)q;
            }
        }
        head = tail;
        wave_sync();
    }
    // flip the island in both replicas
    const int size = *reinterpret_cast<volatile int *>(tailp);
    for (int idx = lane; idx < size; idx += 64) {
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
    if (!nwork) return;
    // one wave per pair, up to four pairs per workgroup within the LDS limit
    const int pb = icm_pair_bytes(N);
    const int ppw = std::max(1, std::min(4, kMaxSweepLds / pb));
    k_icm<<<(nwork + ppw - 1) / ppw, 64 * ppw, (size_t)ppw * pb, st>>>(insts, work, nwork, round, pb);
}

}  // namespace pamc
