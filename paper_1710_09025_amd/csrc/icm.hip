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

// Island growth on the square lattice as a bit-parallel flood fill: row y
// of the sector is the L-bit word Mr[y] (bit x = site x + L y) and the
// island so far is Vr[y].  A pass replaces each row's island bits by the runs
// of Mr[y] (cyclic in x) that contain an island bit or a site bonded to an
// island site of row y - 1 or y + 1 (same x); the set only grows and stays
// connected to the seed, and a pass that changes no row leaves it closed
// under the four bonds, i.e. it is then the seed's connected component, the
// same set the breadth-first search finds.
template <typename W>
__device__ __forceinline__ W bit_reverse(W v)
{
    if constexpr (sizeof(W) == 4)
        return __builtin_bitreverse32(v);
    else
        return __builtin_bitreverse64(v);
}

// Runs of m holding a bit of s (s within m) when no run wraps past the top
// bit.  Adding s to m carries from the lowest seed of each run to its top
// and out of it, so m & ~(m + s) is each seeded run from its lowest seed up,
// except for the higher seeds, which the sum leaves set: OR-ing s restores
// them.  The same on the bit-reversed words gives each run from its highest
// seed down.
template <typename W>
__device__ __forceinline__ W runs_linear(W m, W s)
{
    const W up = (m & ~(m + s)) | s;
    const W mr = bit_reverse(m), sr = bit_reverse(s);
    return up | bit_reverse((mr & ~(mr + sr)) | sr);
}

// Rotations within the low L bits (0 <= n < L).
template <typename W>
__device__ __forceinline__ W rot_right(W v, int n, int L, W mask)
{
    return n == 0 ? v : ((v >> n) | (v << (L - n))) & mask;
}

template <typename W>
__device__ __forceinline__ W rot_left(W v, int n, int L, W mask)
{
    return n == 0 ? v : ((v << n) | (v >> (L - n))) & mask;
}

// Cyclic runs of the L-bit row m holding a bit of seed: the row is rotated
// so that one of its empty sites sits at bit L - 1, where no run can cross
// the ends, and the linear form applies; a full row is one run.
template <typename W>
__device__ __forceinline__ W row_runs(W m, W seed, int L, W mask)
{
    const W s = seed & m;
    const W gaps = ~m & mask;
    if (s == 0 || gaps == 0) return s == 0 ? (W)0 : m;
    const int z = sizeof(W) == 4 ? __builtin_ctz((uint32_t)gaps) : __builtin_ctzll((uint64_t)gaps);
    const int n = z + 1 == L ? 0 : z + 1;
    return rot_left<W>(runs_linear<W>(rot_right<W>(m, n, L, mask), rot_right<W>(s, n, L, mask)), n, L, mask);
}

// The rows live in the pair's queue area: 2 L words of W fit there for
// 8 <= L (4-byte words up to L = 32, 8-byte words above, where N > 1024).
// Lane gl owns rows gl and gl + GS (L <= 2 GS on the square lattice).  On
// return the island's bits are ORed into vis (which holds the seed).
template <typename W, int GS>
__device__ __forceinline__ void flood_square(const uint8_t *member, int sel, uint32_t *vis, uint16_t *queue, int L,
                                             int gl)
{
    const int s0 = queue[0];
    wave_sync();  // the seed is read before the rows overwrite the queue
    W *Mr = reinterpret_cast<W *>(queue);
    W *Vr = Mr + L;
    const W mask = L == (int)(8 * sizeof(W)) ? ~(W)0 : (((W)1 << L) - 1);
    const int y0 = s0 / L, x0 = s0 - y0 * L;
    W m[2], v[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int y = gl + i * GS;
        m[i] = 0;
        v[i] = 0;
        if (y >= L) continue;
        const uint8_t *row = member + y * L;
        if ((L & 3) == 0) {
            for (int x = 0; x < L; x += 4) {
                const uint32_t w = *reinterpret_cast<const uint32_t *>(row + x) >> sel;
                m[i] |= (W)((w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u)) << x;
            }
        } else {
            for (int x = 0; x < L; ++x) m[i] |= (W)((row[x] >> sel) & 1u) << x;
        }
        v[i] = y == y0 ? (W)1 << x0 : (W)0;
        Vr[y] = v[i];
    }
    wave_sync();
    // every pass but the last adds a site, so at most N + 1 passes
    for (int pass = 0; pass <= L * L; ++pass) {
        int changed = 0;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int y = gl + i * GS;
            if (y >= L) continue;
            const W nbv = Vr[y == 0 ? L - 1 : y - 1] | Vr[y == L - 1 ? 0 : y + 1];
            const W f = row_runs<W>(m[i], v[i] | (m[i] & nbv), L, mask);
            if (f != v[i]) {
                v[i] = f;
                Vr[y] = f;
                changed = 1;
            }
        }
        changed = group_sum<GS>(changed);
        wave_sync();
        if (!changed) break;
    }
    // bits y L .. y L + L - 1 of the site bitmap: at most three words
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int y = gl + i * GS;
        if (y >= L || v[i] == 0) continue;
        const uint64_t f = (uint64_t)v[i];
        const int p = y * L, w = p >> 5, sh = p & 31;
        const uint32_t p0 = (uint32_t)(f << sh), p1 = (uint32_t)(f >> (32 - sh));
        const uint32_t p2 = sh ? (uint32_t)(f >> (64 - sh)) : 0u;
        if (p0) atomicOr(&vis[w], p0);
        if (p1) atomicOr(&vis[w + 1], p1);
        if (p2) atomicOr(&vis[w + 2], p2);
    }
}

// The same flood fill on the cubic lattice, from L = 8 on: row r = y + L z
// holds the L sites of x (bit x = site x + L r), its neighbouring rows are
// y +- 1 and z +- 1 (cyclic), and the sector and island rows, 4-byte words,
// live in the queue area (8 L^2 <= L^3 bytes).  Lane gl takes rows gl,
// gl + GS, ...; they stay in LDS (up to 16 per lane).
template <int GS>
__device__ __forceinline__ void flood_cubic(const uint8_t *member, int sel, uint32_t *vis, uint16_t *queue, int L,
                                            int gl)
{
    const int s0 = queue[0];
    wave_sync();  // the seed is read before the rows overwrite the queue
    const int nr = L * L;
    uint32_t *Mr = reinterpret_cast<uint32_t *>(queue);
    uint32_t *Vr = Mr + nr;
    const uint32_t mask = L == 32 ? ~0u : ((1u << L) - 1u);
    // r / L as (r mg) >> 16, exact for r < 1024 and L <= 32
    const uint32_t mg = (65536u + (uint32_t)L - 1u) / (uint32_t)L;
    const int r0 = s0 / L, x0 = s0 - r0 * L;
    for (int r = gl; r < nr; r += GS) {
        const uint8_t *row = member + r * L;
        uint32_t m = 0;
        if ((L & 3) == 0) {
            for (int x = 0; x < L; x += 4) {
                const uint32_t w = *reinterpret_cast<const uint32_t *>(row + x) >> sel;
                m |= ((w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u)) << x;
            }
        } else {
            for (int x = 0; x < L; ++x) m |= (uint32_t)((row[x] >> sel) & 1u) << x;
        }
        Mr[r] = m;
        Vr[r] = r == r0 ? 1u << x0 : 0u;
    }
    wave_sync();
    // every pass but the last adds a site, so at most N + 1 passes
    for (int pass = 0; pass <= L * nr; ++pass) {
        int changed = 0;
        for (int r = gl; r < nr; r += GS) {
            const uint32_t m = Mr[r];
            if (m == 0) continue;
            const uint32_t v = Vr[r];
            const int z = (int)(((uint32_t)r * mg) >> 16), y = r - z * L;
            const int ym = y == 0 ? r + L - 1 : r - 1, yp = y == L - 1 ? r - L + 1 : r + 1;
            const int zm = z == 0 ? r + nr - L : r - L, zp = z == L - 1 ? r - nr + L : r + L;
            const uint32_t nbv = Vr[ym] | Vr[yp] | Vr[zm] | Vr[zp];
            const uint32_t f = row_runs<uint32_t>(m, v | (m & nbv), L, mask);
            if (f != v) {
                Vr[r] = f;
                changed = 1;
            }
        }
        changed = group_sum<GS>(changed);
        wave_sync();
        if (!changed) break;
    }
    // bits r L .. r L + L - 1 of the site bitmap: at most two words
    for (int r = gl; r < nr; r += GS) {
        const uint64_t f = Vr[r];
        if (f == 0) continue;
        const int p = r * L, w = p >> 5, sh = p & 31;
        const uint32_t p0 = (uint32_t)(f << sh), p1 = (uint32_t)(f >> (32 - sh));
        if (p0) atomicOr(&vis[w], p0);
        if (p1) atomicOr(&vis[w + 1], p1);
    }
}

// One ICM round.  A lane group of GS lanes updates one pair (work item =
// instance, pair index j) on its own slice of LDS, so the island search
// synchronises only inside its wave; small lattices take 16 lanes per pair
// and four pairs per wave, since every phase of an update waits on memory
// or LDS latency and more pairs in flight hide it.  Every exit before the
// end is uniform over a group, and lanes only exchange values within their
// group.
//
// UF: row vectors a lane loads at once in the passes over the two rows
// (2 when a lane has at most two vectors of a row, else 4: more in flight
// costs registers and occupancy).
template <int GS, int UF>
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
    // (UF vectors per lane are loaded before the first is used, so that a
    // lattice of up to UF GS 16 positions costs one round trip to memory;
    // indexes past the row reload its last vector and are not used)
    int nd = 0;
    for (int v0 = gl; v0 < nvec; v0 += UF * GS) {
        uint4 a[UF], b[UF], x0[UF], x1[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int v = min(v0 + u * GS, nvec - 1);
            a[u] = A4[v];
            b[u] = B4[v];
            x0[u] = X4[2 * v];
            x1[u] = X4[2 * v + 1];
        }
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            if (v0 + u * GS >= nvec) continue;
            const uint32_t dw[4] = {a[u].x ^ b[u].x, a[u].y ^ b[u].y, a[u].z ^ b[u].z, a[u].w ^ b[u].w};
            const uint32_t xw[8] = {x0[u].x, x0[u].y, x0[u].z, x0[u].w, x1[u].x, x1[u].y, x1[u].z, x1[u].w};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t s = (xw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
                if (s == 0xFFFFu) continue;  // padding position
                const uint32_t d = (dw[q >> 2] >> (8 * (q & 3))) & 0xFFu ? 1u : 0u;
                member[s] = (uint8_t)(2u - d);  // bit 0: differ, bit 1: agree
                nd += (int)d;
            }
        }
    }
    // flags beyond N stay 0 in both bits (the site search reads 16-byte
    // vectors)
    if (gl < N16 - N) member[N + gl] = 0;
    for (int i = gl; i < (N + 31) / 32; i += GS) vis[i] = 0u;
    nd = group_sum<GS>(nd);
    const bool want = nd <= N - nd;
    const int cnt = want ? nd : N - nd;
    if (cnt == 0) return;  // empty sector: no move (uniform over the group)
    // the chosen sector's flag is bit sel of each byte
    const int sel = want ? 0 : 1;
    const uint32_t bm = 0x01010101u << sel;
    wave_sync();
    // the m-th site of the sector: per-lane counts over 16-byte chunks of
    // the flags, a scan over the group, and the owning lane's walk through
    // its chunk
    const uint32_t u = philox10(make_uint4(j, 4u, (uint32_t)k, kTagIcm | (uint32_t)round), I.key0, I.key1).x;
    const int m = (int)(((uint64_t)u * (uint64_t)cnt) >> 32);
    const int nch = N16 >> 4, per = (nch + GS - 1) / GS;
    const int c_begin = min(nch, gl * per), c_end = min(nch, c_begin + per);
    const uint4 *M4 = reinterpret_cast<const uint4 *>(member);
    int c = 0;
    for (int ch = c_begin; ch < c_end; ++ch) {
        const uint4 f = M4[ch];
        c += __builtin_popcount(f.x & bm) + __builtin_popcount(f.y & bm) + __builtin_popcount(f.z & bm) +
             __builtin_popcount(f.w & bm);
    }
    int incl = c;
    for (int off = 1; off < GS; off <<= 1) {
        const int y = __shfl_up(incl, off, GS);
        if (gl >= off) incl += y;
    }
    const int excl = incl - c;
    if (excl <= m && m < incl) {
        // skip whole 4-byte words by their counts, then walk the word that
        // holds the site
        int left = m - excl;
        const uint32_t *M1 = reinterpret_cast<const uint32_t *>(member);
        for (int wi = 4 * c_begin; wi < 4 * c_end; ++wi) {
            const uint32_t f = M1[wi] & bm;
            const int pc = __builtin_popcount(f);
            if (left >= pc) {
                left -= pc;
                continue;
            }
            int b = 0;
            for (;; ++b)
                if ((f >> (8 * b)) & 0xFFu) {
                    if (left == 0) break;
                    --left;
                }
            const int s = 4 * wi + b;
            queue[0] = (uint16_t)s;
            vis[s >> 5] = 1u << (s & 31);
            *tailp = 1;
            break;
        }
    }
    wave_sync();
    bool grown = false;
    if constexpr (GS <= 32) {
        if (I.dim == 2 && L >= 8) {
            if constexpr (GS == 16)
                flood_square<uint32_t, GS>(member, sel, vis, queue, L, gl);
            else
                flood_square<uint64_t, GS>(member, sel, vis, queue, L, gl);
            grown = true;
        }
    }
    if (I.dim == 3 && L >= 8) {
        flood_cubic<GS>(member, sel, vis, queue, L, gl);
        grown = true;
    }
    // otherwise breadth-first growth of the island, one frontier per
    // iteration; the queue only grows and holds each site of the island
    // once (at most cnt <= N / 2 of them), so this ends within N iterations
    int head = 0;
    while (!grown) {
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
                if (!((member[q] >> sel) & 1u)) continue;
                const uint32_t bit = 1u << (q & 31);
                if (atomicOr(&vis[q >> 5], bit) & bit) continue;
                queue[atomicAdd(tailp, 1)] = (uint16_t)q;
            }
        }
        head = tail;
        wave_sync();
    }
    wave_sync();
    // flip the island in both replicas: the visited bits are exactly the
    // island, so each 16-byte vector of the two rows (storage order) gets a
    // byte mask from the bits of its positions' sites and is rewritten when
    // any of its bytes flips; the rows and the site table are loaded
    // together, one round per vector whatever the island's size (the pairs
    // of a round are disjoint, so no other group writes these rows)
    for (int v0 = gl; v0 < nvec; v0 += UF * GS) {
        uint4 a[UF], b[UF], x0[UF], x1[UF];
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int v = min(v0 + u * GS, nvec - 1);
            x0[u] = X4[2 * v];
            x1[u] = X4[2 * v + 1];
            a[u] = A4[v];
            b[u] = B4[v];
        }
#pragma unroll
        for (int u = 0; u < UF; ++u) {
            const int v = v0 + u * GS;
            if (v >= nvec) continue;
            const uint32_t xw[8] = {x0[u].x, x0[u].y, x0[u].z, x0[u].w, x1[u].x, x1[u].y, x1[u].z, x1[u].w};
            uint32_t fw[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const uint32_t t = (xw[q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
                if (t != 0xFFFFu && ((vis[t >> 5] >> (t & 31)) & 1u)) fw[q >> 2] |= 1u << (8 * (q & 3));
            }
            if (fw[0] | fw[1] | fw[2] | fw[3]) {
                A4[v] = make_uint4(a[u].x ^ fw[0], a[u].y ^ fw[1], a[u].z ^ fw[2], a[u].w ^ fw[3]);
                B4[v] = make_uint4(b[u].x ^ fw[0], b[u].y ^ fw[1], b[u].z ^ fw[2], b[u].w ^ fw[3]);
            }
        }
    }
}

hipError_t icm_kernels_init()
{
    const void *fns[] = {reinterpret_cast<const void *>(&k_icm<16, 2>), reinterpret_cast<const void *>(&k_icm<16, 4>),
                         reinterpret_cast<const void *>(&k_icm<32, 4>), reinterpret_cast<const void *>(&k_icm<64, 4>)};
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
    // about N / 16 row vectors of 16 positions per row (a layout's padding
    // may add some; the choice only affects speed)
    const int per_lane = ((N + 15) / 16 + gs - 1) / gs;
    if (gs == 16 && per_lane <= 2)
        k_icm<16, 2><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
    else if (gs == 16)
        k_icm<16, 4><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
    else if (gs == 32)
        k_icm<32, 4><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
    else
        k_icm<64, 4><<<grid, 64 * waves, lds, st>>>(insts, work, nwork, round, pb);
}

}  // namespace pamc
