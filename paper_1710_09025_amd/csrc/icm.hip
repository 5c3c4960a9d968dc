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

// Sum over the GS lanes of a lane group (GS a power of two <= 64).
template <int GS>
__device__ __forceinline__ int group_sum(int v)
{
    for (int off = GS / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GS);
    return v;
}

// One ICM round.  A lane group of GS lanes updates one pair (work item =
// instance, pair index j) on its own slice of LDS, so the island search
// synchronises only inside its wave; small lattices take 16 lanes per pair
// and four pairs per wave, since every phase of an update waits on memory
// or LDS latency and more pairs in flight hide it.  Every exit before the
// end is uniform over a group, and lanes only exchange values within their
// group.
template <int GS>
__global__ __launch_bounds__(256) void k_icm(const Inst *insts, const Work *work, int nwork, int round, int pair_bytes)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const int lane = (int)threadIdx.x & 63;
    const int gl = lane % GS;                  // lane in the group
    const int slot = (int)threadIdx.x / GS;    // group in the workgroup
    const int item = (int)blockIdx.x * ((int)blockDim.x / GS) + slot;
    if (item >= nwork) return;
    const Work w = work[item];
    const Inst &I = insts[w.inst];
    const int k = *I.k;
    if (!inst_live(I, k) || k == 0 || round >= I.icm || !(I.beta[k] >= I.icm_bmin)) return;
    const uint32_t n = I.Rk[k];
    const uint32_t j = w.row0;
    if (j >= n / 2) return;
    const int N = I.N, L = I.L, nnb = 2 * I.dim, N16 = (N + 15) & ~15;
    uint8_t *base = lds + (size_t)slot * pair_bytes;
    uint8_t *member = base;
    uint32_t *vis = reinterpret_cast<uint32_t *>(base + N16);
    uint16_t *queue = reinterpret_cast<uint16_t *>(base + N16 + ((4 * ((N + 31) / 32) + 15) & ~15));
    int *tailp = reinterpret_cast<int *>(base + pair_bytes - 16);
    // the pair's rows: pi(2j) on group lane 0, pi(2j + 1) on group lane 1
    uint32_t row = 0;
    if (gl < 2) row = icm_perm(I.key0, I.key1, 2 * j + (uint32_t)gl, n, k, round);
    const uint32_t ra = __shfl(row, 0, GS), rb = __shfl(row, 1, GS);
    uint8_t *sp = I.spins[*I.cur];
    uint8_t *A = sp + (size_t)ra * I.srow_bytes;
    uint8_t *B = sp + (size_t)rb * I.srow_bytes;
    uint4 *A4 = reinterpret_cast<uint4 *>(A), *B4 = reinterpret_cast<uint4 *>(B);
    const uint4 *X4 = reinterpret_cast<const uint4 *>(I.lexof);
    const int nvec = I.row_bytes >> 4;
    // sites where the replicas differ: both rows read in 16-byte vectors in
    // storage order (one round of loads per 16 positions), each byte
    // compared and its flag stored at the position's lexicographic site
    int nd = 0;
    for (int v = gl; v < nvec; v += GS) {
        const uint4 a = A4[v], b = B4[v], x0 = X4[2 * v], x1 = X4[2 * v + 1];
        const uint32_t dw[4] = {a.x ^ b.x, a.y ^ b.y, a.z ^ b.z, a.w ^ b.w};
        const uint32_t xw[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t s = (xw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
            if (s == 0xFFFFu) continue;  // padding position
            const uint8_t d = (dw[q >> 2] >> (8 * (q & 3))) & 0xFFu ? 1 : 0;
            member[s] = d;
            nd += d;
        }
    }
    // sector flags beyond N stay 0 (the site search reads 16-byte vectors)
    if (gl < N16 - N) member[N + gl] = 0;
    for (int i = gl; i < (N + 31) / 32; i += GS) vis[i] = 0u;
    nd = group_sum<GS>(nd);
    const bool want = nd <= N - nd;
    const int cnt = want ? nd : N - nd;
    if (cnt == 0) return;  // empty sector: no move (uniform over the group)
    wave_sync();
    if (!want)
        for (int s = gl; s < N; s += GS) member[s] ^= 1u;
    wave_sync();
    // the m-th site of the sector: per-lane counts over 16-byte chunks of
    // the flags (0 or 1 per byte), a scan over the group, and the owning
    // lane's walk through its chunk
    const uint32_t u = philox10(make_uint4(j, 4u, (uint32_t)k, kTagIcm | (uint32_t)round), I.key0, I.key1).x;
    const int m = (int)(((uint64_t)u * (uint64_t)cnt) >> 32);
    const int nch = N16 >> 4, per = (nch + GS - 1) / GS;
    const int c_begin = min(nch, gl * per), c_end = min(nch, c_begin + per);
    const uint4 *M4 = reinterpret_cast<const uint4 *>(member);
    int c = 0;
    for (int ch = c_begin; ch < c_end; ++ch) {
        const uint4 f = M4[ch];
        c += __builtin_popcount(f.x) + __builtin_popcount(f.y) + __builtin_popcount(f.z) + __builtin_popcount(f.w);
    }
    int incl = c;
    for (int off = 1; off < GS; off <<= 1) {
        const int y = __shfl_up(incl, off, GS);
        if (gl >= off) incl += y;
    }
    const int excl = incl - c;
    if (excl <= m && m < incl) {
        int seen = excl;
        for (int s = 16 * c_begin; s < 16 * c_end; ++s)
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
    // queue only grows and holds each site of the island once (at most
    // cnt <= N / 2 of them), so this ends within N iterations
    int head = 0;
    while (true) {
        const int tail = *reinterpret_cast<volatile int *>(tailp);
        if (head >= tail) break;
        wave_sync();
        for (int idx = head + gl; idx < tail; idx += GS) {
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
    // flip the island in both replicas: the visited bits are exactly the
    // island, so each 16-byte vector of the two rows (storage order) gets a
    // byte mask from the bits of its positions' sites and is rewritten when
    // any of its bytes flips; the rows and the site table are loaded
    // together, one round per vector whatever the island's size (the pairs
    // of a round are disjoint, so no other group writes these rows)
    for (int v = gl; v < nvec; v += GS) {
        const uint4 x0 = X4[2 * v], x1 = X4[2 * v + 1], a = A4[v], b = B4[v];
        const uint32_t xw[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        uint32_t fw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const uint32_t t = (xw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
            if (t != 0xFFFFu && ((vis[t >> 5] >> (t & 31)) & 1u)) fw[q >> 2] |= 1u << (8 * (q & 3));
        }
        if (fw[0] | fw[1] | fw[2] | fw[3]) {
            A4[v] = make_uint4(a.x ^ fw[0], a.y ^ fw[1], a.z ^ fw[2], a.w ^ fw[3]);
            B4[v] = make_uint4(b.x ^ fw[0], b.y ^ fw[1], b.z ^ fw[2], b.w ^ fw[3]);
        }
    }
}

hipError_t icm_kernels_init()
{
    const void *fns[] = {reinterpret_cast<const void *>(&k_icm<16>), reinterpret_cast<const void *>(&k_icm<32>),
                         reinterpret_cast<const void *>(&k_icm<64>)};
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxSweepLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Lanes per pair: 16 up to N = 1024 sites, 32 up to 4096, else a wave.
static int icm_group_lanes(int N) { return N <= 1024 ? 16 : N <= 4096 ? 32 : 64; }

void launch_icm(const Inst *insts, const Work *work, int nwork, int N, int round, hipStream_t st)
{
    if (!nwork) return;
    // a lane group per pair, up to four waves per workgroup within the LDS
    // limit
    const int pb = icm_pair_bytes(N);
    const int gs = icm_group_lanes(N), gpw = 64 / gs;
    const int waves = std::max(1, std::min(4, kMaxSweepLds / (pb * gpw)));
    const int ppb = waves * gpw;  // pairs per workgroup
    const int grid = (nwork + ppb - 1) / ppb;
    const size_t lds = (size_t)ppb * pb;
    if (gs == 16)
        k_icm<16><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
    else if (gs == 32)
        k_icm<32><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
    else
        k_icm<64><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
}

}  // namespace pamc
