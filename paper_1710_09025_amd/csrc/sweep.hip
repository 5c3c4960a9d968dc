// sweep.hip -- initial population, energies and the checkerboard Metropolis
// sweeps (paper Sec. II.B and Sec. III.A) for gfx950.
//
// A block loads a tile of replica rows into LDS, runs all N_S sweeps of the
// current temperature on chip, recomputes each replica's energy (Eq. (1))
// from the final spins, and writes the rows back once.  When the previous
// resampling left a copy map, the tile is read through it, so the gather of
// surviving replicas costs no separate pass over HBM.  The epilogue adds the
// tile to the energy histogram and the family counts; the last workgroup of
// an instance to finish then measures the step and prepares the resampling
// table (measure_step).
//
// Random numbers: the draw for a site of colour c whose rank among the
// sites of that colour is i, in replica row r, step k and sweep t, is word
// (i & 3) of Philox4x32-10 at counter ((c << 24) | (i >> 2), r, k,
// TAG_SWEEP | t) under the run's key.  Acceptance for dE > 0 is u < T_k(dE)
// with uint32 thresholds prepared on the host.
#include "launch.h"
#include "pamc_dev.h"
#include "step_common.h"

namespace pamc {

__device__ __forceinline__ const Inst &inst_ref(const Inst *insts, uint32_t i) { return insts[i]; }

// Storage position of lexicographic site s in a replica row.
__device__ __forceinline__ int storage_pos(const Inst &I, int s) { return I.pos[s]; }

// Packed spin rows: bit p of a row (bit p & 7 of byte p >> 3) is the spin at
// storage position p.  Kernels work on one byte per position in LDS; 16
// stored bits are one 16-byte LDS vector.
__device__ __forceinline__ uint32_t bits_to_bytes4(uint32_t nib)
{
    // bit i of the nibble lands on bit 8 i: nib + (nib << 7) + (nib << 14) + (nib << 21)
    return (nib * 0x00204081u) & 0x01010101u;
}
__device__ __forceinline__ uint4 bits_to_bytes16(uint32_t b)
{
    return make_uint4(bits_to_bytes4(b & 15u), bits_to_bytes4((b >> 4) & 15u), bits_to_bytes4((b >> 8) & 15u),
                      bits_to_bytes4((b >> 12) & 15u));
}
__device__ __forceinline__ uint32_t bytes_to_bits4(uint32_t w)
{
    // byte i (0 or 1) lands on bit 24 + i of w * (2^24 + 2^17 + 2^10 + 2^3)
    return (uint32_t)(((uint64_t)w * 0x01020408ull) >> 24) & 15u;
}
__device__ __forceinline__ uint32_t bytes_to_bits16(uint4 v)
{
    return bytes_to_bits4(v.x) | (bytes_to_bits4(v.y) << 4) | (bytes_to_bits4(v.z) << 8) | (bytes_to_bits4(v.w) << 12);
}
// Spin (0/1) at storage position p of a stored row.
__device__ __forceinline__ int stored_spin(const Inst &I, const uint8_t *row, int p)
{
    return I.packed ? (row[p >> 3] >> (p & 7)) & 1 : row[p];
}

// ---------------------------------------------------------------------------
// Initial replicas (Sec. II.B: random configurations at beta = 0).  Site s
// of row r takes S = +1 when bit 31 of word (s & 3) of Philox at counter
// (s >> 2, r, 0, TAG_INIT) is set.  One thread per Philox block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_init(const Inst *insts, const Work *work)
{
    extern __shared__ __align__(16) uint8_t stage[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int nq = (I.N + 3) >> 2;
    const int rows = min(kRowsPerBlock, I.R - (int)w.row0);
    if (!I.packed) {
        uint8_t *sp = I.spins[0];
        for (int it = threadIdx.x; it < rows * nq; it += blockDim.x) {
            const int q = it / nq, b = it - q * nq;
            const uint32_t r = w.row0 + q;
            const uint4 v = philox10(make_uint4((uint32_t)b, r, 0u, kTagInit), I.key0, I.key1);
            for (int j = 0; j < 4; ++j) {
                const int s = 4 * b + j;
                if (s >= I.N) break;
                sp[(size_t)r * I.row_bytes + storage_pos(I, s)] = (uint8_t)(word_of(v, j) >> 31);
            }
        }
    } else {
        // rows staged as bytes in LDS (16 KB, or one row), then packed
        const int nvec = I.row_bytes >> 4;
        const int rpi = max(1, 16384 / I.row_bytes);
        uint4 *st16 = reinterpret_cast<uint4 *>(stage);
        for (int q0 = 0; q0 < rows; q0 += rpi) {
            const int nr = min(rpi, rows - q0);
            for (int i = threadIdx.x; i < nr * nvec; i += blockDim.x) st16[i] = make_uint4(0u, 0u, 0u, 0u);
            __syncthreads();
            for (int it = threadIdx.x; it < nr * nq; it += blockDim.x) {
                const int q = it / nq, b = it - q * nq;
                const uint32_t r = w.row0 + q0 + q;
                const uint4 v = philox10(make_uint4((uint32_t)b, r, 0u, kTagInit), I.key0, I.key1);
                for (int j = 0; j < 4; ++j) {
                    const int s = 4 * b + j;
                    if (s >= I.N) break;
                    stage[q * I.row_bytes + storage_pos(I, s)] = (uint8_t)(word_of(v, j) >> 31);
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < nr * nvec; i += blockDim.x) {
                const int q = i / nvec, c = i - q * nvec;
                uint16_t *dst = reinterpret_cast<uint16_t *>(I.spins[0] + (size_t)(w.row0 + q0 + q) * I.srow_bytes);
                dst[c] = (uint16_t)bytes_to_bits16(st16[i]);
            }
            __syncthreads();
        }
    }
    for (int q = threadIdx.x; q < rows; q += blockDim.x) I.fam[0][w.row0 + q] = w.row0 + q;
}

// ---------------------------------------------------------------------------
// Energies of the rows of the current buffer, Eq. (1): E = -sum over the
// D N bonds (s, s + e_d) of J S_s S_{s+e_d} (D = 3, or 2 on the square
// lattice, real couplings only).  One wave per row.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_energy(const Inst *insts, const Work *work, const int8_t *const *Jraw)
{
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT) return;
    const int Rk = (int)I.Rk[k];
    const int cur = *I.cur;
    const int8_t *J = Jraw[w.inst];
    const int L = I.L, N = I.N;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (I.real) {
        // real couplings: int32 [D][N] in units of 2^-20, 64-bit sums; on
        // the square lattice z = 0 and the z bond is absent
        const int32_t *Jq = reinterpret_cast<const int32_t *>(J);
        const int Lz = I.dim == 3 ? L : 1;
        for (int q = wave; q < kRowsPerBlock; q += 4) {
            const int r = (int)w.row0 + q;
            if (r >= Rk) break;
            const uint8_t *S = I.spins[cur] + (size_t)r * I.srow_bytes;
            long long e = 0;
            for (int s = lane; s < N; s += 64) {
                const int x = s % L, y = (s / L) % L, z = s / (L * L);
                const int ss = 2 * stored_spin(I, S, storage_pos(I, s)) - 1;
                const int nb[3] = {(x + 1) % L + L * (y + L * z), x + L * ((y + 1) % L + L * z),
                                   x + L * (y + L * ((z + 1) % Lz))};
                for (int d = 0; d < I.dim; ++d)
                    e -= (long long)Jq[d * N + s] * (ss * (2 * stored_spin(I, S, storage_pos(I, nb[d])) - 1));
            }
            for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
            if (lane == 0) I.Eq[cur][r] = e;
        }
        return;
    }
    for (int q = wave; q < kRowsPerBlock; q += 4) {
        const int r = (int)w.row0 + q;
        if (r >= Rk) break;
        const uint8_t *S = I.spins[cur] + (size_t)r * I.srow_bytes;
        int e = 0;
        for (int s = lane; s < N; s += 64) {
            const int x = s % L, y = (s / L) % L, z = s / (L * L);
            const int ss = 2 * stored_spin(I, S, storage_pos(I, s)) - 1;
            const int nb[3] = {(x + 1) % L + L * (y + L * z), x + L * ((y + 1) % L + L * z),
                               x + L * (y + L * ((z + 1) % L))};
            for (int d = 0; d < 3; ++d)
                e -= J[d * N + s] * ss * (2 * stored_spin(I, S, storage_pos(I, nb[d])) - 1);
        }
        for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
        if (lane == 0) I.E[cur][r] = e;
    }
}

// ---------------------------------------------------------------------------
// Shared tile load / store.  Rows of the tile come from buffer `cur`, either
// directly (in place) or through the copy map (then they go to the other
// buffer, with their family ids).
// ---------------------------------------------------------------------------
struct TileIO {
    const uint8_t *src;
    uint8_t *dst;
    const uint32_t *map;  // nullptr: identity
    const uint32_t *fsrc;
    uint32_t *fdst;
    int32_t *Edst;
    int64_t *Eqdst;       // real couplings: 64-bit energies
    int packed;           // stored rows hold one bit per position
    int srow;             // bytes per stored row
};

__device__ __forceinline__ TileIO tile_io(const Inst &I)
{
    TileIO io;
    const int cur = *I.cur;
    const int mapped = *I.mapped;
    io.src = I.spins[cur];
    io.map = mapped ? I.map : nullptr;
    io.dst = mapped ? I.spins[cur ^ 1] : I.spins[cur];
    io.fsrc = I.fam[cur];
    io.fdst = mapped ? I.fam[cur ^ 1] : nullptr;
    io.Edst = mapped ? I.E[cur ^ 1] : I.E[cur];
    io.Eqdst = I.real ? (mapped ? I.Eq[cur ^ 1] : I.Eq[cur]) : nullptr;
    io.packed = I.packed;
    io.srow = I.srow_bytes;
    return io;
}

// 16-byte LDS vector c of stored row `row`: a copy, or 16 stored bits
// expanded to bytes.
__device__ __forceinline__ uint4 stored_vec(const TileIO &io, const uint8_t *row, int c)
{
    if (io.packed) return bits_to_bytes16(reinterpret_cast<const uint16_t *>(row)[c]);
    return reinterpret_cast<const uint4 *>(row)[c];
}
__device__ __forceinline__ void store_vec(const TileIO &io, uint8_t *row, int c, uint4 v)
{
    if (io.packed)
        reinterpret_cast<uint16_t *>(row)[c] = (uint16_t)bytes_to_bits16(v);
    else
        reinterpret_cast<uint4 *>(row)[c] = v;
}

__device__ __forceinline__ void tile_load(const TileIO &io, uint8_t *tile, int r0, int nrows, int row_bytes)
{
    const int per_row = row_bytes >> 4;
    for (int it = threadIdx.x; it < nrows * per_row; it += blockDim.x) {
        const int q = it / per_row, c = it - q * per_row;
        const uint32_t r = (uint32_t)(r0 + q);
        const uint32_t sr = io.map ? io.map[r] : r;
        *reinterpret_cast<uint4 *>(tile + q * row_bytes + 16 * c) = stored_vec(io, io.src + (size_t)sr * io.srow, c);
    }
}

__device__ __forceinline__ void tile_store(const TileIO &io, const uint8_t *tile, int r0, int nrows, int row_bytes)
{
    const int per_row = row_bytes >> 4;
    for (int it = threadIdx.x; it < nrows * per_row; it += blockDim.x) {
        const int q = it / per_row, c = it - q * per_row;
        const uint4 v = *reinterpret_cast<const uint4 *>(tile + q * row_bytes + 16 * c);
        store_vec(io, io.dst + (size_t)(r0 + q) * io.srow, c, v);
    }
    if (io.map)
        for (int q = threadIdx.x; q < nrows; q += blockDim.x) io.fdst[r0 + q] = io.fsrc[io.map[r0 + q]];
}

// Energy -> histogram bin and stored energy, for the rows of the tile.
__device__ __forceinline__ void tile_energy_out(const Inst &I, const TileIO &io, const int *unsat, int r0, int nrows)
{
    for (int base = 0; base < nrows; base += blockDim.x) {
        const int q = base + (int)threadIdx.x;
        const bool valid = q < nrows;
        int E = 0;
        if (valid) {
            E = 2 * unsat[q] - 3 * I.N;
            io.Edst[r0 + q] = E;
        }
        count_wave(I.hist, (uint32_t)((E + 3 * I.N) >> 1), valid);
    }
}

// Descendants per family: the tile's rows counted under their family ids.
__device__ __forceinline__ void tile_family_count(const Inst &I, const TileIO &io, int r0, int nrows)
{
    for (int base = 0; base < nrows; base += blockDim.x) {
        const int q = base + (int)threadIdx.x;
        const bool valid = q < nrows;
        uint32_t f = 0;
        if (valid) f = io.map ? io.fsrc[io.map[r0 + q]] : io.fsrc[r0 + q];
        count_wave(I.cnt, f, valid);
    }
}

// A sweep launch runs the whole step (phase 0) or, for runs with cluster
// moves, the first floor(N_S/2) sweeps (phase 1: through the copy map, no
// energies) and later the remaining ones (phase 2: in place, with energies
// and the measurement).
__device__ __forceinline__ int phase_t0(const Inst &I, int phase) { return phase == 2 ? I.NS / 2 : 0; }
__device__ __forceinline__ int phase_t1(const Inst &I, int phase) { return phase == 1 ? I.NS / 2 : I.NS; }

// End of phase 1 in the last workgroup: the population now lives in the
// buffer the tiles were written to.
__device__ __forceinline__ void phase1_done(const Inst &I)
{
    const bool last = last_workgroup(&I.sync[0], I.sweep_tiles);
    if (last && threadIdx.x == 0 && *I.mapped) {
        *I.cur ^= 1;
        *I.mapped = 0;
    }
}

// End of a sweep workgroup: the last one of the instance measures the step.
__device__ __forceinline__ void sweep_done(const Inst &I, int k, int phase)
{
    if (phase == 1)
        phase1_done(I);
    else if (last_workgroup(&I.sync[0], I.sweep_tiles))
        measure_step<256>(I, k);
}

// ---------------------------------------------------------------------------
// General sweep: any L >= 2, two colours for even L, three for odd L.
// Storage is lexicographic.  Each work item is one Philox block (four
// consecutive sites of one colour) of one replica of the tile; per site the
// six neighbours and the couplings come from a per-site record.
// ---------------------------------------------------------------------------
__device__ void sweep_tile_lex(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows, int phase);

__global__ __launch_bounds__(256) void k_sweep_lex(const Inst *insts, const Work *work, int tile_rows, int phase)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT || I.status[0]) return;
    const int Rk = (int)I.Rk[k];
    const int r0 = (int)w.row0;
    const int nrows = min(tile_rows, Rk - r0);
    if (nrows > 0) sweep_tile_lex(I, k, lds, r0, nrows, tile_rows, phase);
    sweep_done(I, k, phase);
}

__device__ void sweep_tile_lex(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows, int phase)
{
    const int row_bytes = I.row_bytes;
    int *unsat = reinterpret_cast<int *>(lds + tile_rows * row_bytes);
    const TileIO io = tile_io(I);
    tile_load(io, lds, r0, nrows, row_bytes);
    for (int q = threadIdx.x; q < nrows; q += blockDim.x) unsat[q] = 0;
    const uint4 th = I.thr[k];
    const bool all = th.w != 0;
    const uint32_t key0 = I.key0, key1 = I.key1;
    __syncthreads();

    const int t1 = phase_t1(I, phase);
    for (int t = phase_t0(I, phase); t < t1; ++t) {
        for (int c = 0; c < I.ncol; ++c) {
            const int G = I.gcs[c];
            const int items = nrows * G;
            const uint16_t *grp = I.grp + (size_t)c * I.gmax * 4;
            for (int it = threadIdx.x; it < items; it += blockDim.x) {
                const int q = it / G, g = it - q * G;
                const uint32_t r = (uint32_t)(r0 + q);
                const uint4 u = philox10(make_uint4(((uint32_t)c << 24) | (uint32_t)g, r, (uint32_t)k,
                                                    kTagSweep | (uint32_t)t),
                                         key0, key1);
                uint8_t *S = lds + q * row_bytes;
                const uint16_t *gs = grp + 4 * g;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int pos = gs[j];
                    if (pos == 0xFFFF) break;
                    const uint4 rec = I.site[pos];
                    const uint32_t s0 = S[pos];
                    const uint32_t jm = rec.w;
                    // unsatisfied bonds: S_s S_nb J = -1  <=>  s ^ nb ^ [J = -1] = 1
                    const uint32_t n = (s0 ^ S[rec.x & 0xFFFF] ^ (jm & 1)) + (s0 ^ S[rec.x >> 16] ^ ((jm >> 1) & 1)) +
                                       (s0 ^ S[rec.y & 0xFFFF] ^ ((jm >> 2) & 1)) + (s0 ^ S[rec.y >> 16] ^ ((jm >> 3) & 1)) +
                                       (s0 ^ S[rec.z & 0xFFFF] ^ ((jm >> 4) & 1)) + (s0 ^ S[rec.z >> 16] ^ ((jm >> 5) & 1));
                    // dE = 12 - 4 n: n = 0, 1, 2 need the draw; n >= 3 is downhill
                    const uint32_t T = n == 0 ? th.z : (n == 1 ? th.y : th.x);
                    const bool acc = all || n >= 3 || word_of(u, j) < T;
                    if (acc) S[pos] = (uint8_t)(s0 ^ 1u);
                }
            }
            __syncthreads();
        }
    }

    if (phase == 1) {
        tile_store(io, lds, r0, nrows, row_bytes);
        return;
    }
    // energies: E = 2U - 3N with U the unsatisfied bonds (s, s + e_d)
    for (int it = threadIdx.x; it < nrows * I.N; it += blockDim.x) {
        const int q = it / I.N, s = it - q * I.N;
        const uint8_t *S = lds + q * row_bytes;
        const uint4 rec = I.site[s];
        const uint32_t s0 = S[s];
        const uint32_t jm = rec.w;
        const int n = (int)((s0 ^ S[rec.x & 0xFFFF] ^ (jm & 1)) + (s0 ^ S[rec.y & 0xFFFF] ^ ((jm >> 2) & 1)) +
                            (s0 ^ S[rec.z & 0xFFFF] ^ ((jm >> 4) & 1)));
        atomicAdd(&unsat[q], n);
    }
    __syncthreads();
    tile_store(io, lds, r0, nrows, row_bytes);
    tile_energy_out(I, io, unsat, r0, nrows);
    tile_family_count(I, io, r0, nrows);
}

// ---------------------------------------------------------------------------
// SWAR sweep for L in {8, 16}.  Storage layout kLayoutEO: the sites of
// colour c fill positions c N/2 ... with row (y, z) holding its L/2 sites of
// colour c, x >> 1 ascending, at c N/2 + (zL + y) L/2.  Philox block
// g = (row, jb) of colour c is the aligned 32-bit word at c N/2 + row L/2 +
// 4 jb, one byte per site; the sites of colour c in row (y, z) have x of
// parity p = (c + y + z) & 1.  Their neighbours are sites of the other
// colour: the word at the same place of rows y +- 1 and z +- 1, the word at
// the same place of the same row (one x neighbour), and that word shifted
// by one byte (the other x neighbour), built with a byte-align of two
// words.  Per byte the six terms s ^ nb ^ [J = -1] are summed without
// carries (<= 6 per byte).  Consecutive blocks are consecutive words, so
// the lanes of a wave read consecutive LDS words (no bank conflicts).
//
// A thread owns GPT Philox blocks of each colour in RPT replicas at once;
// the replicas of one thread lie a fixed distance apart in LDS, so their
// word addresses differ by an immediate offset.
// ---------------------------------------------------------------------------
template <int L>
struct EOShape {
    static constexpr int N = L * L * L;    // also the row stride in bytes
    static constexpr int H = L / 2;        // sites per half row
    static constexpr int GPR = L / 8;      // Philox blocks per half row
    static constexpr int G = N / 8;        // Philox blocks per colour
    static constexpr int TPR = G < 256 ? G : 256;  // threads per replica
    static constexpr int GPT = G / TPR;    // blocks per thread and colour
    static constexpr int RPT = 2;          // replicas per thread
    static constexpr int RPG = 256 / TPR;  // replica groups per workgroup
    static constexpr int RP = RPG * RPT;   // replicas swept at once
    static constexpr int RSTRIDE = RPG * N;  // LDS distance between a thread's replicas
    static constexpr bool kWaveLocal = TPR <= 64;
};

int eo_replicas_per_pass(int L) { return L == 8 ? EOShape<8>::RP : EOShape<16>::RP; }

// Orders the LDS accesses of the threads sweeping one replica between two
// colours.  When a replica lives inside one wave, the wave's LDS operations
// complete in issue order, so a compiler fence and wave barrier suffice.
template <bool kWaveLocal>
__device__ __forceinline__ void colour_barrier()
{
    if constexpr (kWaveLocal) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

struct EOGroup {
    uint32_t own, hi, lo, yp, ym, zp, zm;  // LDS byte offsets within a row
    uint32_t sh;                            // byte shift for the x neighbour
    uint32_t ctr;                           // Philox counter word 0
    uint32_t j[6];                          // coupling bytes (1: J = -1)
};

template <int L>
__device__ __forceinline__ void eo_group_setup(EOGroup &gr, const uint32_t *jeo, int c, int g)
{
    using S = EOShape<L>;
    const int row = g / S::GPR, jb = g - row * S::GPR;
    const int y = row % L, z = row / L;
    const int p = (c + y + z) & 1;
    const uint32_t base = (uint32_t)c * (S::N / 2), obase = (uint32_t)(1 - c) * (S::N / 2);
    gr.own = base + row * S::H + 4 * jb;
    const uint32_t oth = obase + row * S::H + 4 * jb;
    // p = 1: the other x neighbour is one site to the right (next word),
    // p = 0: one site to the left (previous word), with periodic wrap.
    const uint32_t adj = obase + row * S::H + 4 * ((jb + (p ? 1 : S::GPR - 1)) % S::GPR);
    gr.hi = p ? adj : oth;
    gr.lo = p ? oth : adj;
    gr.sh = p ? 1u : 3u;
    gr.yp = obase + (z * L + (y + 1) % L) * S::H + 4 * jb;
    gr.ym = obase + (z * L + (y + L - 1) % L) * S::H + 4 * jb;
    gr.zp = obase + (((z + 1) % L) * L + y) * S::H + 4 * jb;
    gr.zm = obase + (((z + L - 1) % L) * L + y) * S::H + 4 * jb;
    gr.ctr = ((uint32_t)c << 24) | (uint32_t)g;
    const uint32_t *jw = jeo + ((size_t)c * S::G + g) * 6;
#pragma unroll
    for (int d = 0; d < 6; ++d) gr.j[d] = jw[d];
}

__device__ __forceinline__ uint32_t lds32(const uint8_t *base, uint32_t off)
{
    return *reinterpret_cast<const uint32_t *>(base + off);
}

// Per byte: number of unsatisfied bonds of the four sites of the block.
__device__ __forceinline__ uint32_t eo_unsat(const uint8_t *row, const EOGroup &gr, uint32_t own)
{
    const uint32_t hi = lds32(row, gr.hi), lo = lds32(row, gr.lo);
    const uint32_t xa = gr.sh == 1u ? lo : hi;  // the aligned x neighbour word
    const uint32_t xs = __builtin_amdgcn_alignbyte(hi, lo, gr.sh);
    return (xor3(own, xa, gr.j[0]) + xor3(own, xs, gr.j[1]) + xor3(own, lds32(row, gr.yp), gr.j[2])) +
           (xor3(own, lds32(row, gr.ym), gr.j[3]) + xor3(own, lds32(row, gr.zp), gr.j[4]) +
            xor3(own, lds32(row, gr.zm), gr.j[5]));
}

// Metropolis decision of the four sites of a block: n >= 3 unsatisfied bonds
// (dE <= 0) always flips; otherwise site i flips when word i of the draw is
// below the threshold of its dE.  tab holds the thresholds by 4 n (bytes);
// every byte of n is <= 6, so 4 n stays inside its byte.
__device__ __forceinline__ uint32_t eo_flip(uint32_t n, uint4 u, const uint8_t *tab)
{
    const uint32_t n4 = n << 2;
    uint32_t flip = ((n + 0x05050505u) >> 3) & 0x01010101u;
    flip |= u.x < *reinterpret_cast<const uint32_t *>(tab + (n4 & 0x1Cu)) ? 0x00000001u : 0u;
    flip |= u.y < *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 8, 5)) ? 0x00000100u : 0u;
    flip |= u.z < *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 16, 5)) ? 0x00010000u : 0u;
    flip |= u.w < *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 24, 5)) ? 0x01000000u : 0u;
    return flip;
}

// eo_flip in two halves: the thresholds of the four bytes of n (and the
// mask of the bytes that always flip, returned) before the draw, the
// comparisons with it after.
__device__ __forceinline__ uint32_t eo_thresholds(uint32_t n, const uint8_t *tab, uint32_t (&th)[4])
{
    const uint32_t n4 = n << 2;
    th[0] = *reinterpret_cast<const uint32_t *>(tab + (n4 & 0x1Cu));
    th[1] = *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 8, 5));
    th[2] = *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 16, 5));
    th[3] = *reinterpret_cast<const uint32_t *>(tab + __builtin_amdgcn_ubfe(n4, 24, 5));
    return ((n + 0x05050505u) >> 3) & 0x01010101u;
}

__device__ __forceinline__ uint32_t eo_accept(uint32_t always, const uint32_t (&th)[4], uint4 u)
{
    uint32_t flip = always;
    flip |= u.x < th[0] ? 0x00000001u : 0u;
    flip |= u.y < th[1] ? 0x00000100u : 0u;
    flip |= u.z < th[2] ? 0x00010000u : 0u;
    flip |= u.w < th[3] ? 0x01000000u : 0u;
    return flip;
}

// All N_S sweeps of the replicas of the tile.  ALL: beta = 0, every move is
// accepted.  The replica groups of the last pass may run past the tile's
// rows into unused LDS rows (the tile holds a multiple of RP rows); their
// results are never stored.
template <int L, bool ALL>
__device__ __forceinline__ void eo_sweeps(const Inst &I, int k, uint8_t *lds, const EOGroup (&gr)[2][EOShape<L>::GPT],
                                          const uint8_t *tab, int *unsat, int r0, int nrows, int phase)
{
    using SH = EOShape<L>;
    const int qsub = threadIdx.x / SH::TPR;
    const uint32_t key0 = I.key0, key1 = I.key1;
    for (int qb = 0; qb < nrows; qb += SH::RP) {
        const int q0 = qb + qsub;
        uint8_t *row = lds + q0 * SH::N;
        const int t1 = phase_t1(I, phase);
        for (int t = phase_t0(I, phase); t < t1; ++t) {
#pragma unroll
            for (int c = 0; c < 2; ++c) {
#pragma unroll
                for (int gi = 0; gi < SH::GPT; ++gi) {
                    const EOGroup &g = gr[c][gi];
#pragma unroll
                    for (int j = 0; j < SH::RPT; ++j) {
                        uint8_t *rj = row + j * SH::RSTRIDE;
                        // raised issue priority for everything but the draw
                        // (see the colour-major kernel)
                        if constexpr (!ALL && L == 16) __builtin_amdgcn_s_setprio(1);
                        const uint32_t own = lds32(rj, g.own);
                        const uint32_t n = eo_unsat(rj, g, own);
                        uint32_t flip = 0x01010101u;
                        const uint32_t r = (uint32_t)(r0 + q0 + j * SH::RPG);
                        if constexpr (!ALL && L == 16) {
                            // the threshold reads go out before the draw,
                            // whose arithmetic covers their LDS latency; the
                            // scheduling barriers keep the compiler from
                            // moving the draw back in front (L = 16: 2303 ->
                            // 2438 attempts/ns at R = 5e5; at L = 8, whose
                            // launch holds fewer groups per thread, the
                            // compiler's own order is 3% faster)
                            uint32_t th[4];
                            const uint32_t fa = eo_thresholds(n, tab, th);
                            __builtin_amdgcn_sched_barrier(0);
                            __builtin_amdgcn_s_setprio(0);
                            const uint4 u = philox10(make_uint4(g.ctr, r, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
                            __builtin_amdgcn_sched_barrier(0);
                            __builtin_amdgcn_s_setprio(1);
                            flip = eo_accept(fa, th, u);
                        } else if constexpr (!ALL) {
                            const uint4 u = philox10(make_uint4(g.ctr, r, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
                            flip = eo_flip(n, u, tab);
                        }
                        *reinterpret_cast<uint32_t *>(rj + g.own) = own ^ flip;
                    }
                }
                colour_barrier<SH::kWaveLocal>();
            }
        }
        // energy: every bond joins a colour-0 and a colour-1 site, so the
        // unsatisfied bonds are the sum of n over colour-0 sites.
        if (phase == 1) continue;
#pragma unroll
        for (int j = 0; j < SH::RPT; ++j) {
            const uint8_t *rj = row + j * SH::RSTRIDE;
            uint32_t part = 0;
#pragma unroll
            for (int gi = 0; gi < SH::GPT; ++gi) {
                const uint32_t n = eo_unsat(rj, gr[0][gi], lds32(rj, gr[0][gi].own));
                part = __builtin_amdgcn_sad_u8(n, 0u, part);
            }
            atomicAdd(&unsat[q0 + j * SH::RPG], (int)part);
        }
        // the rows of the next pass belong to other replicas: no barrier
    }
    __syncthreads();
}

template <int L>
__device__ void sweep_tile_eo(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows, int phase);

// At most 128 VGPRs, so that four waves share each SIMD (the L = 16 kernel
// would take 145 and run three): the draws' long multiply chains and the LDS
// round trips of a colour phase hide behind the other waves.  L = 16 went
// from 1929 to 2110 attempts/ns at R = 5e5 (tile of 8 rows, four
// workgroups per compute unit); L = 8 needs 121 VGPRs either way.
template <int L>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_sweep_eo(const Inst *insts,
                                                                                            const Work *work,
                                                                                            int tile_rows, int phase)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT || I.status[0]) return;
    const int Rk = (int)I.Rk[k];
    const int r0 = (int)w.row0;
    const int nrows = min(tile_rows, Rk - r0);
    if (nrows > 0) sweep_tile_eo<L>(I, k, lds, r0, nrows, tile_rows, phase);
    sweep_done(I, k, phase);
}

// The tile holds tile_rows rows (a multiple of EOShape<L>::RP) of N bytes,
// then tile_rows unsatisfied-bond counters.
template <int L>
__device__ void sweep_tile_eo(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows, int phase)
{
    using SH = EOShape<L>;
    // thresholds by 4 n at a fixed LDS address: T(dE = 12, 8, 4) for
    // n = 0, 1, 2; unused above
    __shared__ uint32_t tab[8];
    int *unsat = reinterpret_cast<int *>(lds + tile_rows * SH::N);
    const TileIO io = tile_io(I);
    tile_load(io, lds, r0, nrows, SH::N);
    const uint4 th = I.thr[k];
    const bool all = th.w != 0;
    if (threadIdx.x < 8) tab[threadIdx.x] = threadIdx.x == 0 ? th.z : threadIdx.x == 1 ? th.y : threadIdx.x == 2 ? th.x : 0u;
    for (int q = threadIdx.x; q < tile_rows; q += blockDim.x) unsat[q] = 0;

    const int lane_r = threadIdx.x % SH::TPR;  // position inside the replica
    EOGroup gr[2][SH::GPT];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int gi = 0; gi < SH::GPT; ++gi) eo_group_setup<L>(gr[c][gi], I.jeo, c, lane_r + gi * SH::TPR);
    __syncthreads();
    const uint8_t *tb = reinterpret_cast<const uint8_t *>(tab);
    if (all)
        eo_sweeps<L, true>(I, k, lds, gr, tb, unsat, r0, nrows, phase);
    else
        eo_sweeps<L, false>(I, k, lds, gr, tb, unsat, r0, nrows, phase);
    // the output pointers are read again rather than held through the
    // sweeps: held, their registers spilled to scratch on every pass (the
    // empty asm's memory clobber keeps the compiler from reusing the first
    // reads)
    asm volatile("" ::: "memory");
    const TileIO out = tile_io(I);
    tile_store(out, lds, r0, nrows, SH::N);
    if (phase == 1) return;
    tile_energy_out(I, out, unsat, r0, nrows);
    tile_family_count(I, out, r0, nrows);
}

// ---------------------------------------------------------------------------
// Colour-major SWAR sweep for any L whose largest colour has at most 4096
// sites (two colours for even L, three for odd L).  Storage kLayoutCM: the
// four sites of a Philox block are consecutive storage positions.
//
// A thread group sweeps four replicas A, B, C, D at once from one LDS slot
// in which the byte lanes of a word are the replicas: storage position p of
// the four is the word [A B C D] at plane(p) plane_bytes + 4 (p >> 2), with
// plane(p) = p & 3 (threads of neighbouring Philox blocks read neighbouring
// words), followed by the same four planes of the complement (0/1 swapped).
// A bond with coupling -1 reads the neighbour from the complement, so one
// 32-bit neighbour read returns s_nb ^ [J = -1] of all four replicas; with m
// the per-site sum of the six words a site has n = m unsatisfied bonds when
// s = 0 and 6 - m when s = 1, i.e. (m ^ 7 s) - s per byte.  Each thread owns
// Philox block g of every colour, keeps the 24 neighbour addresses of its
// four sites in registers and runs the four replicas' draws side by side;
// site i of the block takes word i of each replica's draw.  Energy: every
// bond joins two sites of different colours, so U = (1/2) sum over all
// sites of their unsatisfied bonds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void replica_barrier(int tpr)
{
    if (tpr <= 64) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

struct CMBlock {
    uint32_t nb[24];  // LDS offsets of the neighbour words, [direction][site]
    uint32_t tabp;    // table form: LDS offset of the block's record in the table
    uint32_t own;     // LDS offset of site 0's word (site i at + i plane_bytes)
    uint32_t vbits;   // bit i set when site i of the block is a real site
    uint32_t ctr;     // Philox counter word 0
    bool has;
};

// Byte offset, in a replica-quad slot, of storage position p (p < row_bytes;
// the complement's positions follow at 4 plane_bytes).
__device__ __forceinline__ uint32_t quad_pos(uint32_t p, uint32_t plane_bytes)
{
    return (p & 3u) * plane_bytes + 4u * (p >> 2);
}

// 4 x 4 byte transpose: word k of the result holds byte k of w0, w1, w2, w3
// (v_perm selectors: bytes 0-3 of the second operand, 4-7 of the first).
// It is its own inverse.
__device__ __forceinline__ void transpose4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t (&o)[4])
{
    const uint32_t a_lo = __builtin_amdgcn_perm(w1, w0, 0x05010400u);  // [w0.0 w1.0 w0.1 w1.1]
    const uint32_t a_hi = __builtin_amdgcn_perm(w1, w0, 0x07030602u);  // [w0.2 w1.2 w0.3 w1.3]
    const uint32_t b_lo = __builtin_amdgcn_perm(w3, w2, 0x05010400u);
    const uint32_t b_hi = __builtin_amdgcn_perm(w3, w2, 0x07030602u);
    o[0] = __builtin_amdgcn_perm(b_lo, a_lo, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(b_lo, a_lo, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(b_hi, a_hi, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(b_hi, a_hi, 0x07060302u);
}

// Per byte (replica): unsatisfied bonds, (m ^ 7 s) - s, with 7 s as (s
// rotated left by 3) - s (s has no bits above bit 24, so the rotation is a
// shift and stays off the quarter-rate multiplier).
__device__ __forceinline__ uint32_t unsat_from_sum(uint32_t m, uint32_t own)
{
    const uint32_t own7 = __builtin_amdgcn_alignbit(own, own, 29) - own;
    return (m ^ own7) - own;
}

__device__ __forceinline__ uint32_t lds_word(const uint8_t *lds, uint32_t a)
{
    return *reinterpret_cast<const uint32_t *>(lds + a);
}

// The 24 neighbour addresses of block b in the quad slot at sbase: kept in
// registers, or (TAB) read from the block's record in the workgroup's LDS
// table, two 16-bit slot offsets a word (each extracted and added in one
// SDWA instruction).  The table form holds 24 fewer registers per colour:
// with two colours 125 VGPRs, four waves per SIMD instead of three.
template <bool TAB>
__device__ __forceinline__ void cm_neighbours(const uint8_t *lds, const CMBlock &b, uint32_t sbase,
                                              uint32_t (&nb)[24])
{
    if constexpr (TAB) {
        const uint4 *rq = reinterpret_cast<const uint4 *>(lds + b.tabp);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            const uint4 w = rq[v];
            nb[8 * v + 0] = sbase + (w.x & 0xFFFFu);
            nb[8 * v + 1] = sbase + (w.x >> 16);
            nb[8 * v + 2] = sbase + (w.y & 0xFFFFu);
            nb[8 * v + 3] = sbase + (w.y >> 16);
            nb[8 * v + 4] = sbase + (w.z & 0xFFFFu);
            nb[8 * v + 5] = sbase + (w.z >> 16);
            nb[8 * v + 6] = sbase + (w.w & 0xFFFFu);
            nb[8 * v + 7] = sbase + (w.w >> 16);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 24; ++j) nb[j] = b.nb[j];
    }
}

// Sweeps of the replicas of the tile, four per thread group at a time, each
// quad loaded into the group's LDS slot (through the copy map) and stored
// back after its N_S sweeps.  ALL: beta = 0, every move is accepted.
// Missing replicas of the last quad are swept as zeros and never stored.
// SF (sums first): the neighbour sums and threshold reads of a block before
// its draws, else the draws first.
template <int NCOL, bool ALL, bool TAB, bool SF>
__device__ __forceinline__ void cm_passes(const Inst &I, int k, uint8_t *lds, const CMBlock (&blk)[NCOL],
                                          const uint8_t *tab, int *unsat, const TileIO &io, int r0, int nrows,
                                          int phase)
{
    const int tpr = I.tpr;
    const int RPG = (int)blockDim.x / tpr;
    const int ps = I.plane_bytes;
    const int lane_r = (int)threadIdx.x % tpr, qsub = (int)threadIdx.x / tpr;
    uint8_t *slot = lds + qsub * I.slot_bytes;
    const uint32_t sbase = (uint32_t)(qsub * I.slot_bytes);
    const int nvec = I.row_bytes >> 4, pvec = ps >> 4;
    const uint32_t key0 = I.key0, key1 = I.key1;
    for (int qb = 0; qb < nrows; qb += 4 * RPG) {
        const int q0 = qb + 4 * qsub;
        const bool act = qsub < RPG && q0 < nrows;  // the last wave's spare lanes idle
        const uint32_t r0q = (uint32_t)(r0 + q0);
        if (act) {
            const uint8_t *src[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t r = r0q + j;
                src[j] = q0 + j < nrows ? io.src + (size_t)(io.map ? io.map[r] : r) * io.srow : nullptr;
            }
            // 16 bytes of a row are four blocks: their plane-k words are 16
            // contiguous bytes of plane k
            uint4 *sp = reinterpret_cast<uint4 *>(slot);
            for (int i = lane_r; i < nvec; i += tpr) {
                uint4 v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = src[j] ? stored_vec(io, src[j], i) : make_uint4(0u, 0u, 0u, 0u);
                uint32_t ox[4], oy[4], oz[4], ow[4];
                transpose4(v[0].x, v[1].x, v[2].x, v[3].x, ox);
                transpose4(v[0].y, v[1].y, v[2].y, v[3].y, oy);
                transpose4(v[0].z, v[1].z, v[2].z, v[3].z, oz);
                transpose4(v[0].w, v[1].w, v[2].w, v[3].w, ow);
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) {
                    const uint4 w = make_uint4(ox[pl], oy[pl], oz[pl], ow[pl]);
                    sp[pl * pvec + i] = w;
                    sp[(4 + pl) * pvec + i] =
                        make_uint4(w.x ^ 0x01010101u, w.y ^ 0x01010101u, w.z ^ 0x01010101u, w.w ^ 0x01010101u);
                }
            }
        }
        replica_barrier(tpr);
        const int t1 = phase_t1(I, phase);
        for (int t = phase_t0(I, phase); t < t1; ++t) {
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                const CMBlock &b = blk[c];
                if (act && b.has) {
                    // Sums first: the wave runs everything but the draws
                    // (its LDS reads, the sums that index the thresholds,
                    // the decisions and the writes) at raised priority and
                    // drops back for the draws, so that a wave whose reads
                    // or writes are due goes ahead of the others' long
                    // multiply chains instead of waiting behind them: more
                    // reads are in flight under the arithmetic and a colour
                    // step's last writes reach the barrier sooner (L = 10,
                    // 12, 14: +3.5, +4.5, +2%; the even/odd-x kernel at
                    // L = 16: +0.5-1%).
                    if constexpr (!ALL && SF) __builtin_amdgcn_s_setprio(1);
                    uint32_t own[4], flip[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        own[i] = lds_word(lds, b.own + i * ps);
                        flip[i] = ((b.vbits >> i) & 1u) * 0x01010101u;
                    }
                    if constexpr (!ALL && SF) {
                        // the neighbour sums and the threshold reads go out
                        // before the draws, whose arithmetic then covers
                        // their LDS latency; the scheduling barrier keeps the
                        // compiler from moving the draws back in front
                        uint32_t fa[4], th[4][4], nb[24];
                        cm_neighbours<TAB>(lds, b, sbase, nb);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint32_t m = (lds_word(lds, nb[i]) + lds_word(lds, nb[4 + i]) +
                                                lds_word(lds, nb[8 + i])) +
                                               (lds_word(lds, nb[12 + i]) + lds_word(lds, nb[16 + i]) +
                                                lds_word(lds, nb[20 + i]));
                            fa[i] = eo_thresholds(unsat_from_sum(m, own[i]), tab, th[i]);
                        }
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_setprio(0);
                        uint4 u[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            u[j] = philox10(make_uint4(b.ctr, r0q + j, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_setprio(1);
#pragma unroll
                        for (int i = 0; i < 4; ++i)
                            flip[i] &= eo_accept(fa[i], th[i], make_uint4(word_of(u[0], i), word_of(u[1], i),
                                                                          word_of(u[2], i), word_of(u[3], i)));
                    } else if constexpr (!ALL) {
                        // draws first (three colours in registers, or in a
                        // 1024-thread workgroup held to 128 VGPRs): the sums'
                        // registers stay short-lived; the reads that follow
                        // go out at raised priority (L = 9, 11, 13: +3, +5,
                        // +1.5%)
                        uint4 u[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            u[j] = philox10(make_uint4(b.ctr, r0q + j, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_setprio(1);
                        uint32_t nb[24];
                        cm_neighbours<TAB>(lds, b, sbase, nb);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const uint32_t m = (lds_word(lds, nb[i]) + lds_word(lds, nb[4 + i]) +
                                                lds_word(lds, nb[8 + i])) +
                                               (lds_word(lds, nb[12 + i]) + lds_word(lds, nb[16 + i]) +
                                                lds_word(lds, nb[20 + i]));
                            const uint32_t n = unsat_from_sum(m, own[i]);
                            flip[i] &= eo_flip(n, make_uint4(word_of(u[0], i), word_of(u[1], i), word_of(u[2], i),
                                                             word_of(u[3], i)),
                                               tab);
                        }
                        __builtin_amdgcn_s_setprio(0);
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t nw = own[i] ^ flip[i];
                        *reinterpret_cast<uint32_t *>(lds + b.own + i * ps) = nw;
                        *reinterpret_cast<uint32_t *>(lds + b.own + (4 + i) * ps) = nw ^ 0x01010101u;
                    }
                }
                replica_barrier(tpr);
            }
        }
        if (act && phase != 1) {
            // per byte (replica) at most 4 sites x 3 colours x 6 bonds = 72:
            // the sum stays inside its byte
            uint32_t acc = 0;
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                if (!blk[c].has) continue;
                uint32_t nb[24];
                cm_neighbours<TAB>(lds, blk[c], sbase, nb);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    if (!((blk[c].vbits >> i) & 1u)) continue;
                    const uint32_t m = (lds_word(lds, nb[i]) + lds_word(lds, nb[4 + i]) +
                                        lds_word(lds, nb[8 + i])) +
                                       (lds_word(lds, nb[12 + i]) + lds_word(lds, nb[16 + i]) +
                                        lds_word(lds, nb[20 + i]));
                    acc += unsat_from_sum(m, lds_word(lds, blk[c].own + i * ps));
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (q0 + j < nrows) atomicAdd(&unsat[q0 + j], (int)((acc >> (8 * j)) & 0xFFu));
        }
        if (act) {
            const uint4 *sp = reinterpret_cast<const uint4 *>(slot);
            for (int i = lane_r; i < nvec; i += tpr) {
                uint4 w[4];
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) w[pl] = sp[pl * pvec + i];
                uint32_t ox[4], oy[4], oz[4], ow[4];
                transpose4(w[0].x, w[1].x, w[2].x, w[3].x, ox);
                transpose4(w[0].y, w[1].y, w[2].y, w[3].y, oy);
                transpose4(w[0].z, w[1].z, w[2].z, w[3].z, oz);
                transpose4(w[0].w, w[1].w, w[2].w, w[3].w, ow);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (q0 + j < nrows)
                        store_vec(io, io.dst + (size_t)(r0q + j) * io.srow, i, make_uint4(ox[j], oy[j], oz[j], ow[j]));
            }
        }
        replica_barrier(tpr);
    }
}

template <int NCOL, bool TAB, bool SF>
__device__ __forceinline__ void sweep_tile_cm(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows,
                                              int phase)
{
    // thresholds by 4 n at a fixed LDS address (see eo_flip)
    __shared__ uint32_t tab[8];
    const int tpr = I.tpr;
    const int RPG = (int)blockDim.x / tpr;
    const int row_bytes = I.row_bytes;
    const int slot_bytes = I.slot_bytes;
    int *unsat = reinterpret_cast<int *>(lds + RPG * slot_bytes + 32);
    const TileIO io = tile_io(I);
    const int lane_r = (int)threadIdx.x % tpr, qsub = (int)threadIdx.x / tpr;
    const uint32_t slot = (uint32_t)(qsub * slot_bytes);
    const uint32_t rb = (uint32_t)row_bytes, ps = (uint32_t)I.plane_bytes;
    CMBlock blk[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
        const int g = lane_r;
        blk[c].has = g < I.gcs[c];
        blk[c].ctr = ((uint32_t)c << 24) | (uint32_t)g;
        const int gg = blk[c].has ? g : 0;
        const uint16_t *d = I.cmdesc + ((size_t)c * I.gmax + gg) * 32;
        // byte offset o of the single-replica slot [row | complement]: row
        // position o, or complement position o - row_bytes
        if constexpr (TAB) {
            // the table follows the row energies, 16-byte aligned; the
            // first quad's threads write it (slot offsets are the same for
            // every quad)
            const uint32_t tbase = ((uint32_t)(RPG * slot_bytes + 32 + 4 * tile_rows) + 15u) & ~15u;
            blk[c].tabp = tbase + 48u * (uint32_t)(c * tpr + g);
            if (qsub == 0) {
                uint32_t w[12];
#pragma unroll
                for (int i = 0; i < 24; ++i) {
                    const uint32_t o = d[i];
                    const uint32_t off = o < rb ? quad_pos(o, ps) : 4u * ps + quad_pos(o - rb, ps);
                    if (i & 1)
                        w[i >> 1] |= off << 16;
                    else
                        w[i >> 1] = off;
                }
                uint4 *rec = reinterpret_cast<uint4 *>(lds + blk[c].tabp);
                rec[0] = make_uint4(w[0], w[1], w[2], w[3]);
                rec[1] = make_uint4(w[4], w[5], w[6], w[7]);
                rec[2] = make_uint4(w[8], w[9], w[10], w[11]);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 24; ++i) {
                const uint32_t o = d[i];
                blk[c].nb[i] = slot + (o < rb ? quad_pos(o, ps) : 4u * ps + quad_pos(o - rb, ps));
            }
        }
        const uint32_t vm = blk[c].has ? (uint32_t)d[24] | ((uint32_t)d[25] << 16) : 0u;
        blk[c].vbits = (vm & 1u) | ((vm >> 7) & 2u) | ((vm >> 14) & 4u) | ((vm >> 21) & 8u);
        // position cbase + 4 g is a multiple of four: site 0 is in plane 0
        blk[c].own = slot + (uint32_t)(I.cbase[c] + 4 * gg);
    }
    const uint4 th = I.thr[k];
    const bool all = th.w != 0;
    if (threadIdx.x < 8) tab[threadIdx.x] = threadIdx.x == 0 ? th.z : threadIdx.x == 1 ? th.y : threadIdx.x == 2 ? th.x : 0u;
    for (int q = threadIdx.x; q < tile_rows; q += blockDim.x) unsat[q] = 0;
    __syncthreads();
    const uint8_t *tb = reinterpret_cast<const uint8_t *>(tab);
    if (all)
        cm_passes<NCOL, true, TAB, SF>(I, k, lds, blk, tb, unsat, io, r0, nrows, phase);
    else
        cm_passes<NCOL, false, TAB, SF>(I, k, lds, blk, tb, unsat, io, r0, nrows, phase);
    __syncthreads();
    // every bond was counted from both of its ends
    for (int q = threadIdx.x; q < nrows; q += blockDim.x) unsat[q] >>= 1;
    if (io.map)
        for (int q = threadIdx.x; q < nrows; q += blockDim.x) io.fdst[r0 + q] = io.fsrc[io.map[r0 + q]];
    if (phase == 1) return;
    __syncthreads();
    tile_energy_out(I, io, unsat, r0, nrows);
    tile_family_count(I, io, r0, nrows);
}

// MAXT: the largest workgroup the instantiation is built for.  Up to 768
// threads (12 waves, three per SIMD) the kernel keeps its 168 registers:
// every neighbour address stays in a register.  A 1024-thread workgroup
// needs four waves per SIMD and spills.  The 768-thread form lets quads
// wider than 64 threads come in threes and fours (L = 12: 3 x 216 threads
// in 11 waves, 92% of the lanes busy, against 84% for one quad).  Sums
// before draws wherever the registers allow it: two colours, and three in
// the table form up to 768 threads (142 VGPRs; L = 7, 9, 11: +2.7, +2.3,
// +1.1%); the 1024-thread three-colour table form would spill with that
// order (8% slower at L = 13) and keeps the draws first.
template <int NCOL, int MAXT, bool TAB = false>
__global__ __launch_bounds__(MAXT, MAXT <= 768 ? 3 : 4) void k_sweep_cm(const Inst *insts, const Work *work, int tile_rows,
                                                                       int phase)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT || I.status[0]) return;
    const int Rk = (int)I.Rk[k];
    const int r0 = (int)w.row0;
    const int nrows = min(tile_rows, Rk - r0);
    constexpr bool kSumsFirst = NCOL == 2 || (TAB && MAXT < 1024);
    if (nrows > 0) sweep_tile_cm<NCOL, TAB, kSumsFirst>(I, k, lds, r0, nrows, tile_rows, phase);
    if (phase == 1)
        phase1_done(I);
    else if (last_workgroup(&I.sync[0], I.sweep_tiles))
        measure_step<512>(I, k);
}

// ---------------------------------------------------------------------------
// Colour-major sweep with real couplings (Sec. II.A: Gaussian J in fixed
// point, J = j 2^-20).  Same replica quads as the +-1 kernel, without the
// complement planes, and with each spin held in LDS as a byte 0x00 / 0xFF
// (converted on load and store): one 32-bit read of a neighbour word returns
// that neighbour's spin in all four replicas, and its XOR with the site's own
// word is, per byte, 0 or -1 for sigma = [S != S_nb] = 0 or 1.  With
// S S_nb = 1 - 2 sigma,
//   dE = 2 S sum_d J_d S_d = 2 sum_d J_d - 4 sum_d sigma_d J_d,
// where sigma_d J_d is the sign-extended byte ANDed with j.  Each
// thread keeps the 4 NB neighbour addresses and couplings of its block of
// every colour in registers (NB = 6 on the cubic lattice; the square-lattice
// kernel reads the first NB = 4 directions of the same tables, whose z
// entries are zero bonds).  Energy: every bond is seen from both of its
// sites, so E = -sum_b J_b + sum over sites of sum_d sigma_d J_d.
// ---------------------------------------------------------------------------
template <int NB>
struct CQBlock {
    uint32_t nb[4 * NB];  // LDS offsets of the neighbour words, [direction][site]
    int32_t j[4 * NB];    // coupling of each of those bonds (units of 2^-20)
    int32_t j2[4];        // twice the sum of the couplings of each site
    uint32_t own;     // LDS offset of site 0's word (site i at + i plane_bytes)
    uint32_t vbits;   // bit i set when site i of the block is a real site
    uint32_t ctr;     // Philox counter word 0
    bool has;
};

// sum_d sigma_d J_d of site i of block b for the four replicas (bytes of the
// XOR words, 0x00 or 0xFF), given the site's own word.
template <int NB>
__device__ __forceinline__ void cq_field(const uint8_t *lds, const CQBlock<NB> &b, int i, uint32_t own,
                                         int32_t (&a)[4])
{
    a[0] = a[1] = a[2] = a[3] = 0;
#pragma unroll
    for (int d = 0; d < NB; ++d) {
        const uint32_t x = own ^ lds_word(lds, b.nb[4 * d + i]);
        const int32_t jj = b.j[4 * d + i];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] += (int32_t)(int8_t)(uint8_t)(x >> (8 * r)) & jj;
    }
}

// 0/1 spin bytes to 0x00/0xFF (255 b per byte, no carries) and back.
__device__ __forceinline__ uint32_t spin_ff(uint32_t w) { return (w << 8) - w; }
__device__ __forceinline__ uint4 spin_ff4(uint4 v)
{
    return make_uint4(spin_ff(v.x), spin_ff(v.y), spin_ff(v.z), spin_ff(v.w));
}
__device__ __forceinline__ uint4 spin_01(uint4 v)
{
    return make_uint4(v.x & 0x01010101u, v.y & 0x01010101u, v.z & 0x01010101u, v.w & 0x01010101u);
}

template <int NCOL, bool ALL, int NB>
__device__ __forceinline__ void cq_passes(const Inst &I, int k, uint8_t *lds, const CQBlock<NB> (&blk)[NCOL], float bq,
                                          unsigned long long *eacc, const TileIO &io, int r0, int nrows, int phase)
{
    const int tpr = I.tpr;
    const int RPG = (int)blockDim.x / tpr;
    const int ps = I.plane_bytes;
    const int lane_r = (int)threadIdx.x % tpr, qsub = (int)threadIdx.x / tpr;
    uint8_t *slot = lds + qsub * I.slot_bytes;
    const int nvec = I.row_bytes >> 4, pvec = ps >> 4;
    const uint32_t key0 = I.key0, key1 = I.key1;
    for (int qb = 0; qb < nrows; qb += 4 * RPG) {
        const int q0 = qb + 4 * qsub;
        const bool act = qsub < RPG && q0 < nrows;  // the last wave's spare lanes idle
        const uint32_t r0q = (uint32_t)(r0 + q0);
        if (act) {
            const uint8_t *src[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t r = r0q + j;
                src[j] = q0 + j < nrows ? io.src + (size_t)(io.map ? io.map[r] : r) * io.srow : nullptr;
            }
            uint4 *sp = reinterpret_cast<uint4 *>(slot);
            for (int i = lane_r; i < nvec; i += tpr) {
                uint4 v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) v[j] = src[j] ? stored_vec(io, src[j], i) : make_uint4(0u, 0u, 0u, 0u);
                uint32_t ox[4], oy[4], oz[4], ow[4];
                transpose4(v[0].x, v[1].x, v[2].x, v[3].x, ox);
                transpose4(v[0].y, v[1].y, v[2].y, v[3].y, oy);
                transpose4(v[0].z, v[1].z, v[2].z, v[3].z, oz);
                transpose4(v[0].w, v[1].w, v[2].w, v[3].w, ow);
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) sp[pl * pvec + i] = spin_ff4(make_uint4(ox[pl], oy[pl], oz[pl], ow[pl]));
            }
        }
        replica_barrier(tpr);
        const int t1 = phase_t1(I, phase);
        for (int t = phase_t0(I, phase); t < t1; ++t) {
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                const CQBlock<NB> &b = blk[c];
                if (act && b.has) {
                    // raised issue priority for the field reads, as in the
                    // +-1 colour-major kernel
                    if constexpr (!ALL) __builtin_amdgcn_s_setprio(1);
                    uint32_t own[4], flip[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        own[i] = lds_word(lds, b.own + i * ps);
                        flip[i] = (b.vbits >> i) & 1u ? 0xFFFFFFFFu : 0u;
                    }
                    if constexpr (!ALL) {
                        // the fields (24 neighbour reads) before the draws,
                        // whose arithmetic then covers the reads' latency
                        // (3-4% at L = 8, 12 and 32 in 2D)
                        int32_t aa[4][4];
#pragma unroll
                        for (int i = 0; i < 4; ++i) cq_field(lds, b, i, own[i], aa[i]);
                        __builtin_amdgcn_sched_barrier(0);
                        __builtin_amdgcn_s_setprio(0);
                        uint4 u[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            u[j] = philox10(make_uint4(b.ctr, r0q + j, (uint32_t)k, kTagSweep | (uint32_t)t), key0, key1);
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int32_t *a = aa[i];
                            uint32_t acc = 0;
#pragma unroll
                            for (int r = 0; r < 4; ++r) {
                                const int32_t dE = b.j2[i] - 4 * a[r];
                                const bool ok = dE <= 0 || real_accept(bq, dE, word_of(u[r], i));
                                acc |= (ok ? 0xFFu : 0u) << (8 * r);
                            }
                            flip[i] &= acc;
                        }
                    }
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        *reinterpret_cast<uint32_t *>(lds + b.own + i * ps) = own[i] ^ flip[i];
                }
                replica_barrier(tpr);
            }
        }
        if (act && phase != 1) {
            // per replica, sum over the thread's sites of sum_d sigma_d J_d:
            // at most 12 sites x 6 bonds x 2^23 < 2^30
            int32_t e[4] = {0, 0, 0, 0};
#pragma unroll
            for (int c = 0; c < NCOL; ++c) {
                if (!blk[c].has) continue;
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    int32_t a[4];
                    cq_field(lds, blk[c], i, lds_word(lds, blk[c].own + i * ps), a);
#pragma unroll
                    for (int r = 0; r < 4; ++r) e[r] += a[r];
                }
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (q0 + j < nrows) atomicAdd(&eacc[q0 + j], (unsigned long long)(long long)e[j]);
        }
        if (act) {
            const uint4 *sp = reinterpret_cast<const uint4 *>(slot);
            for (int i = lane_r; i < nvec; i += tpr) {
                uint4 w[4];
#pragma unroll
                for (int pl = 0; pl < 4; ++pl) w[pl] = spin_01(sp[pl * pvec + i]);
                uint32_t ox[4], oy[4], oz[4], ow[4];
                transpose4(w[0].x, w[1].x, w[2].x, w[3].x, ox);
                transpose4(w[0].y, w[1].y, w[2].y, w[3].y, oy);
                transpose4(w[0].z, w[1].z, w[2].z, w[3].z, oz);
                transpose4(w[0].w, w[1].w, w[2].w, w[3].w, ow);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (q0 + j < nrows)
                        store_vec(io, io.dst + (size_t)(r0q + j) * io.srow, i, make_uint4(ox[j], oy[j], oz[j], ow[j]));
            }
        }
        replica_barrier(tpr);
    }
}

// Energies of the tile's rows (E = -sum_b J_b + the accumulated sums) and
// their moments, added to the step's accumulators once per workgroup: min,
// max, sum E (two's complement) and sum E^2 as an exact 128-bit integer
// (low word added first; its carry goes into the high word).
__device__ __forceinline__ void tile_moments_real(const Inst &I, const TileIO &io, const unsigned long long *eacc,
                                                  int r0, int nrows)
{
    __shared__ long long smin[16], smax[16];
    __shared__ unsigned long long ssum[16], slo[16], shi[16];
    long long lmin = 0x7FFFFFFFFFFFFFFFll, lmax = -0x7FFFFFFFFFFFFFFFll - 1;
    unsigned long long s1 = 0ull, lo = 0ull, hi = 0ull;
    for (int q = threadIdx.x; q < nrows; q += blockDim.x) {
        const long long E = (long long)eacc[q] - I.Jtot;
        io.Eqdst[r0 + q] = E;
        lmin = E < lmin ? E : lmin;
        lmax = E > lmax ? E : lmax;
        s1 += (unsigned long long)E;
        const unsigned __int128 e2 = (unsigned __int128)((__int128)E * (__int128)E);
        const unsigned long long l2 = (unsigned long long)e2;
        const unsigned long long nl = lo + l2;
        hi += (unsigned long long)(e2 >> 64) + (nl < lo ? 1ull : 0ull);
        lo = nl;
    }
    for (int off = 32; off > 0; off >>= 1) {
        const long long omin = __shfl_xor(lmin, off), omax = __shfl_xor(lmax, off);
        const unsigned long long os = __shfl_xor(s1, off), ol = __shfl_xor(lo, off), oh = __shfl_xor(hi, off);
        lmin = omin < lmin ? omin : lmin;
        lmax = omax > lmax ? omax : lmax;
        s1 += os;
        const unsigned long long nl = lo + ol;
        hi += oh + (nl < lo ? 1ull : 0ull);
        lo = nl;
    }
    const int wave = threadIdx.x >> 6, nw = ((int)blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) {
        smin[wave] = lmin;
        smax[wave] = lmax;
        ssum[wave] = s1;
        slo[wave] = lo;
        shi[wave] = hi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < nw; ++v) {
            lmin = smin[v] < lmin ? smin[v] : lmin;
            lmax = smax[v] > lmax ? smax[v] : lmax;
            s1 += ssum[v];
            const unsigned long long nl = lo + slo[v];
            hi += shi[v] + (nl < lo ? 1ull : 0ull);
            lo = nl;
        }
        EMoments *m = I.emom;
        atomicMin(&m->emin, lmin);
        atomicMax(&m->emax, lmax);
        atomicAdd(&m->sum, s1);
        const unsigned long long old = atomicAdd(&m->sq_lo, lo);
        atomicAdd(&m->sq_hi, hi + (old + lo < old ? 1ull : 0ull));
    }
}

template <int NCOL, int NB>
__device__ __forceinline__ void sweep_tile_cq(const Inst &I, int k, uint8_t *lds, int r0, int nrows, int tile_rows,
                                              int phase)
{
    const int tpr = I.tpr;
    const int RPG = (int)blockDim.x / tpr;
    const int ps = I.plane_bytes;
    unsigned long long *eacc = reinterpret_cast<unsigned long long *>(lds + RPG * I.slot_bytes + 32);
    const TileIO io = tile_io(I);
    const int lane_r = (int)threadIdx.x % tpr, qsub = (int)threadIdx.x / tpr;
    const uint32_t slot = (uint32_t)(qsub * I.slot_bytes);
    CQBlock<NB> blk[NCOL];
#pragma unroll
    for (int c = 0; c < NCOL; ++c) {
        const int g = lane_r;
        blk[c].has = g < I.gcs[c];
        blk[c].ctr = ((uint32_t)c << 24) | (uint32_t)g;
        const int gg = blk[c].has ? g : 0;
        const uint16_t *d = I.cmdesc + ((size_t)c * I.gmax + gg) * 32;
        const int32_t *jd = I.cmj + ((size_t)c * I.gmax + gg) * 24;
#pragma unroll
        for (int i = 0; i < 4 * NB; ++i) {
            blk[c].nb[i] = slot + quad_pos((uint32_t)d[i], (uint32_t)ps);
            blk[c].j[i] = jd[i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int32_t s2 = 0;
#pragma unroll
            for (int dd = 0; dd < NB; ++dd) s2 += blk[c].j[4 * dd + i];
            blk[c].j2[i] = 2 * s2;
        }
        const uint32_t vm = blk[c].has ? (uint32_t)d[24] | ((uint32_t)d[25] << 16) : 0u;
        blk[c].vbits = (vm & 1u) | ((vm >> 7) & 2u) | ((vm >> 14) & 4u) | ((vm >> 21) & 8u);
        blk[c].own = slot + (uint32_t)(I.cbase[c] + 4 * gg);
    }
    const float bq = I.bq[k];
    const bool all = I.thr[k].w != 0;
    for (int q = threadIdx.x; q < tile_rows; q += blockDim.x) eacc[q] = 0ull;
    __syncthreads();
    if (all)
        cq_passes<NCOL, true, NB>(I, k, lds, blk, bq, eacc, io, r0, nrows, phase);
    else
        cq_passes<NCOL, false, NB>(I, k, lds, blk, bq, eacc, io, r0, nrows, phase);
    __syncthreads();
    if (io.map)
        for (int q = threadIdx.x; q < nrows; q += blockDim.x) io.fdst[r0 + q] = io.fsrc[io.map[r0 + q]];
    if (phase == 1) return;
    tile_moments_real(I, io, eacc, r0, nrows);
    tile_family_count(I, io, r0, nrows);
}

template <int NCOL, int MAXT>
__global__ __launch_bounds__(MAXT, 2) void k_sweep_cq(const Inst *insts, const Work *work, int tile_rows, int phase)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT || I.status[0]) return;
    const int Rk = (int)I.Rk[k];
    const int r0 = (int)w.row0;
    const int nrows = min(tile_rows, Rk - r0);
    if (nrows > 0) sweep_tile_cq<NCOL, 6>(I, k, lds, r0, nrows, tile_rows, phase);
    if (phase == 1)
        phase1_done(I);
    else if (last_workgroup(&I.sync[0], I.sweep_tiles))
        measure_step_real(I, k);
}

// The same on the square lattice: four neighbours per site.
template <int NCOL, int MAXT>
__global__ __launch_bounds__(MAXT, 2) void k_sweep_sq(const Inst *insts, const Work *work, int tile_rows, int phase)
{
    extern __shared__ __align__(16) uint8_t lds[];
    const Work w = work[blockIdx.x];
    const Inst &I = inst_ref(insts, w.inst);
    const int k = *I.k;
    if (k >= I.nT || I.status[0]) return;
    const int Rk = (int)I.Rk[k];
    const int r0 = (int)w.row0;
    const int nrows = min(tile_rows, Rk - r0);
    if (nrows > 0) sweep_tile_cq<NCOL, 4>(I, k, lds, r0, nrows, tile_rows, phase);
    if (phase == 1)
        phase1_done(I);
    else if (last_workgroup(&I.sync[0], I.sweep_tiles))
        measure_step_real(I, k);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
hipError_t sweep_kernels_init()
{
    const void *fns[] = {
        reinterpret_cast<const void *>(&k_sweep_lex),         reinterpret_cast<const void *>(&k_sweep_eo<8>),
        reinterpret_cast<const void *>(&k_sweep_eo<16>),      reinterpret_cast<const void *>(&k_sweep_cm<2, 512>),
        reinterpret_cast<const void *>(&k_sweep_cm<2, 1024>), reinterpret_cast<const void *>(&k_sweep_cm<3, 512>),
        reinterpret_cast<const void *>(&k_sweep_cm<3, 1024>), reinterpret_cast<const void *>(&k_sweep_cm<2, 768>),
        reinterpret_cast<const void *>(&k_sweep_cm<3, 768>),  reinterpret_cast<const void *>(&k_sweep_cm<2, 512, true>),
        reinterpret_cast<const void *>(&k_sweep_cm<2, 1024, true>),
        reinterpret_cast<const void *>(&k_sweep_cm<3, 512, true>),  reinterpret_cast<const void *>(&k_sweep_cm<3, 768, true>),
        reinterpret_cast<const void *>(&k_sweep_cm<3, 1024, true>), reinterpret_cast<const void *>(&k_sweep_cq<2, 512>),
        reinterpret_cast<const void *>(&k_sweep_cq<2, 1024>), reinterpret_cast<const void *>(&k_sweep_cq<3, 512>),
        reinterpret_cast<const void *>(&k_sweep_cq<3, 1024>), reinterpret_cast<const void *>(&k_sweep_sq<2, 512>),
        reinterpret_cast<const void *>(&k_sweep_sq<2, 1024>), reinterpret_cast<const void *>(&k_sweep_sq<3, 512>),
        reinterpret_cast<const void *>(&k_sweep_sq<3, 1024>),
    };
    for (const void *f : fns) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxSweepLds);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void launch_init(const Inst *insts, const Work *work, int nwork, size_t lds_bytes, hipStream_t st)
{
    if (nwork) k_init<<<nwork, 256, lds_bytes, st>>>(insts, work);
}

void launch_energy(const Inst *insts, const Work *work, int nwork, const int8_t *const *Jraw, hipStream_t st)
{
    if (nwork) k_energy<<<nwork, 256, 0, st>>>(insts, work, Jraw);
}

// Default workgroup shape of the colour-major sweep: 256 / tpr quads for
// quads of at most 64 threads; above, the number of quads (of at most 512
// threads together) that leaves the fewest idle lanes in the last wave, the
// one nearest 256 threads among equals.
int cm_replicas_per_block(int tpr)
{
    if (tpr <= 64) return 256 / tpr;
    int best = 1;
    double best_use = 0.0;
    for (int rp = 1; rp * tpr <= 512 || rp == 1; ++rp) {
        const int nt = rp * tpr;
        const double use = (double)nt / (double)cm_launch_threads(tpr, rp);
        const bool nearer = std::abs(nt - 256) < std::abs(best * tpr - 256);
        if (use > best_use + 1e-9 || (use > best_use - 1e-9 && nearer)) {
            best = rp;
            best_use = use;
        }
    }
    return best;
}

void launch_sweep(int variant, const Inst *insts, const Work *work, int nwork, int tile_rows, int row_bytes, int tpr,
                  int rp, int phase, hipStream_t st)
{
    if (!nwork) return;
    if (variant == kSweepCM2T || variant == kSweepCM3T) {
        // as below, with the neighbour table after the row energies
        const size_t lds = (size_t)cm_slot_bytes(row_bytes, tpr, 8) * rp + 32 + 4 * (size_t)tile_rows +
                           cm_table_bytes(variant, tpr);
        const int nt = cm_launch_threads(tpr, rp);
        if (variant == kSweepCM2T) {
            if (nt <= 512)
                k_sweep_cm<2, 512, true><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cm<2, 1024, true><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        } else {
            if (nt <= 512)
                k_sweep_cm<3, 512, true><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else if (nt <= 768)
                k_sweep_cm<3, 768, true><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cm<3, 1024, true><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        }
        return;
    }
    if (variant == kSweepCM2 || variant == kSweepCM3) {
        // rp replica quads, each four planes of the row and of the complement
        const size_t lds = (size_t)cm_slot_bytes(row_bytes, tpr, 8) * rp + 32 + 4 * (size_t)tile_rows;
        const int nt = cm_launch_threads(tpr, rp);
        if (variant == kSweepCM2) {
            if (nt <= 512)
                k_sweep_cm<2, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else if (nt <= 768)
                k_sweep_cm<2, 768><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cm<2, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        } else {
            if (nt <= 512)
                k_sweep_cm<3, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else if (nt <= 768)
                k_sweep_cm<3, 768><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cm<3, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        }
        return;
    }
    if (variant == kSweepSQ2 || variant == kSweepSQ3) {
        // as below, on the square lattice
        const size_t lds = (size_t)cm_slot_bytes(row_bytes, tpr, 4) * rp + 32 + 8 * (size_t)tile_rows;
        const int nt = cm_launch_threads(tpr, rp);
        if (variant == kSweepSQ2) {
            if (nt <= 512)
                k_sweep_sq<2, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_sq<2, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        } else {
            if (nt <= 512)
                k_sweep_sq<3, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_sq<3, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        }
        return;
    }
    if (variant == kSweepCQ2 || variant == kSweepCQ3) {
        // rp replica quads of four planes, and a 64-bit energy per tile row
        const size_t lds = (size_t)cm_slot_bytes(row_bytes, tpr, 4) * rp + 32 + 8 * (size_t)tile_rows;
        const int nt = cm_launch_threads(tpr, rp);
        if (variant == kSweepCQ2) {
            if (nt <= 512)
                k_sweep_cq<2, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cq<2, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        } else {
            if (nt <= 512)
                k_sweep_cq<3, 512><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
            else
                k_sweep_cq<3, 1024><<<nwork, nt, lds, st>>>(insts, work, tile_rows, phase);
        }
        return;
    }
    const size_t lds = (size_t)tile_rows * row_bytes + 32 + 4 * (size_t)tile_rows;
    switch (variant) {
    case kSweepLex: k_sweep_lex<<<nwork, 256, lds, st>>>(insts, work, tile_rows, phase); break;
    case kSweepEO8: k_sweep_eo<8><<<nwork, 256, lds, st>>>(insts, work, tile_rows, phase); break;
    case kSweepEO16: k_sweep_eo<16><<<nwork, 256, lds, st>>>(insts, work, tile_rows, phase); break;
    default: break;
    }
}

}  // namespace pamc
