// pamc_dev.h -- data layout shared by the host orchestrator and the gfx950
// kernels of the population annealing library.
//
// Every kernel is segmented by instance: it reads the instance descriptor
// `Inst` from device memory, so one run, a batch of mixed-size instances and
// the serving loop all use the same kernels.  The current temperature step
// k of each instance lives on the device, so a step can be captured once in
// a hipGraph and replayed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

// (Device arithmetic shared by the kernels -- Philox, the three-way xor --
// lives in step_common.h, which only the kernel sources include.)

namespace pamc {

// Philox stream tags, the top four bits of counter word 3.
constexpr uint32_t kTagInit = 0x10000000u;
constexpr uint32_t kTagSweep = 0x20000000u;
constexpr uint32_t kTagResample = 0x30000000u;
constexpr uint32_t kTagIcm = 0x40000000u;

// Spin storage layouts inside one replica row.
enum Layout : int32_t {
    // byte per site (0: S = -1, 1: S = +1), lexicographic s = x + L(y + Lz)
    kLayoutLex = 0,
    // byte per site, the sites of colour 0 then those of colour 1, each in
    // lexicographic order: pos = c N/2 + (zL + y)(L/2) + (x >> 1) for the
    // site of colour c = (x + y + z) & 1.  Used for L = 8 and 16 (L/2 a
    // multiple of four): the four sites of one Philox block are one aligned
    // 32-bit word inside one row (y, z), their y and z neighbours and one x
    // neighbour are the word at the same place of the other colour's rows,
    // and the other x neighbour is that word shifted by one byte.  Lanes
    // sweeping consecutive blocks read consecutive words.
    kLayoutEO = 1,
    // byte per site, colour-major: the sites of colour 0 in lexicographic
    // order, then colour 1 (and 2 for odd L), each colour padded to a
    // multiple of four, so the four sites of one Philox block are one
    // aligned 32-bit word for every L.
    kLayoutCM = 2,
};

constexpr int kRowsPerBlock = 1024;  // rows handled per block by row kernels
constexpr int kOvlPairs = 2048;      // replica pairs per overlap workgroup (few workgroups: most steps measure no overlap)
constexpr int kOvlLdsBins = 8194;    // overlap histograms up to this many bins (L <= 16) are built in LDS

// Per-step integer record written on the device.  Energies are in units of
// 2^-20 for real couplings.
struct StepRec {
    int64_t R;        // R_k
    int64_t sumE;     // sum of E
    uint64_t sumE2;   // sum of E^2: low 64 bits of the exact 128-bit sum
    int64_t sumE2_hi; //   and its high 64 bits
    int64_t Emin, Emax;
    double S;         // resampling normaliser (NaN at the last step)
    double T;         // family term sum n ln n
};

// Energy moments of a step's population with real couplings, accumulated
// with atomics by the sweep workgroups (one update per tile) and read and
// reset by the step measurement.  Sums are exact: E^2 as a 128-bit integer.
struct EMoments {
    long long emin, emax;
    unsigned long long sum;      // sum of E, two's complement
    unsigned long long sq_lo;    // sum of E^2, low 64 bits
    unsigned long long sq_hi;    //   high 64 bits (carries added)
    unsigned long long pad[3];
};

struct Inst {
    // problem
    int32_t L, N, ncol, layout;
    int32_t dim;        // lattice dimension: 3 (cubic, N = L^3) or 2 (square, N = L^2; real couplings only)
    int32_t row_bytes;  // bytes per replica row in LDS, one byte per storage position (>= N, multiple of 16)
    int32_t packed;     // 1: the spin buffers hold one bit per storage position
    int32_t srow_bytes; // bytes per replica row in the spin buffers (row_bytes, or row_bytes / 8 rounded up to 16)
    int32_t nT, NS;
    uint32_t key0, key1;
    int32_t R;          // nominal population
    int32_t Rcap;       // rows per buffer
    int32_t nblk;       // ceil(Rcap / kRowsPerBlock)
    int32_t nlev;       // 3N + 1 energy levels
    int32_t fam_pow2;   // smallest power of two >= R (family tree leaves)
    int32_t ovl_n;      // number of overlap steps
    int32_t real;       // 1: real couplings in fixed point, J = j 2^-20 (int32 j, |J| < 8)
    int32_t icm;        // cluster-move rounds per step (0: none)
    double icm_bmin;    // cluster moves only at steps with beta_k >= icm_bmin
    // double-buffered population
    uint8_t *spins[2];
    int32_t *E[2];
    uint32_t *fam[2];
    // resampling scratch
    uint32_t *map;      // [Rcap] destination row -> source row
    uint32_t *loff;     // [Rcap] first destination of each row inside its row block
    uint32_t *bsum;     // [nblk]
    uint32_t *boff;     // [nblk]
    uint32_t *sync;     // [4] workgroups finished in the current sweep / post / weights launch
    int32_t sweep_tiles;  // workgroups of this instance in a sweep launch
    int32_t post_blocks;  // workgroups of this instance in a post launch
    int32_t tile_rows;    // replica rows per sweep workgroup
    uint32_t *hist;     // [nlev] energy histogram, (E + 3N)/2
    uint2 *BF;          // [nlev] (floor(tau), frac(tau) 2^32) per level above E_min
    uint32_t *cnt;      // [R] descendants per family
    double *fpart;      // [max(1, fam_pow2 / 2048)] family tree partial sums
    // tables
    const uint4 *thr;   // [nT] (T(dE=4), T(8), T(12), accept_all)
    const double *beta; // [nT]
    const double *rho;  // [nT] exp(-2 (beta_{k+1} - beta_k)), host libm
    const double *Rt;   // [nT] nominal population R(beta_k) the resampling targets
    const double *nlnn; // [>= Rcap + 1] n ln n, host libm (shared)
    const uint4 *site;  // lex layout: [N] {nb+x|nb-x<<16, nb+y|nb-y<<16, nb+z|nb-z<<16, jmask}
    const uint16_t *grp;// lex layout: [ncol][gmax][4] sites of each Philox block (0xFFFF: none)
    const uint32_t *jeo;// EO layout: [2][N/8][6] coupling words per block
    const uint16_t *pos;// [N] storage position of each lexicographic site
    const uint16_t *lexof; // [row_bytes] lexicographic site at each storage position (0xFFFF: padding)
    // CM layout: per colour and Philox block, the 24 LDS byte offsets (within
    // a replica slot) of the 6 neighbours of its 4 sites, in the spin copy or,
    // for a -1 coupling, in the complemented copy at +row_bytes; word 24 is
    // the mask of real (non-padding) sites, one 0x01 per byte.
    const uint16_t *cmdesc;  // [ncol][gmax][32]
    int32_t cbase[3];   // CM layout: first byte of each colour
    int32_t tpr;        // CM layout: threads per replica
    int32_t plane_bytes;// CM layout: LDS stride of a replica quad's byte planes (>= row_bytes)
    int32_t slot_bytes; // CM layout: LDS stride of the replica quads' slots (bank-skewed)
    int32_t ncs[3];     // sites per colour
    int32_t gcs[3];     // Philox blocks per colour, ceil(ncs / 4)
    int32_t gmax;
    // real couplings (CM layout)
    int64_t *Eq[2];     // energies, units of 2^-20
    double *wrep;       // [Rcap] resampling weight of each row
    double *wpart;      // [nblk] pairwise-tree roots of the 1024-row blocks
    EMoments *emom;     // energy moments of the step being swept
    const int32_t *cmj; // [ncol][gmax][24] coupling of each neighbour bond, in cmdesc order
    const float *bq;    // [nT] beta_k 2^-20 rounded to binary32
    const double *gpw;  // [nT][40] exp(-(beta_{k+1} - beta_k) 2^(b-20)), host libm
    int64_t Jtot;       // sum of all couplings
    // progress and records
    int32_t *k;         // current step (device scalar)
    int32_t *cur;       // buffer holding the current population (0/1)
    int32_t *mapped;    // 1: rows of the current step still live in buffer
                        //    cur through `map` (gather pending)
    uint32_t *Rk;       // [nT + 1]
    StepRec *rec;       // [nT]
    int32_t *ovl_slot;  // [nT] slot in qhist or -1
    uint32_t *qhist;    // [ovl_n][2N + 1]
    uint32_t *status;   // bit 0 capacity, bit 1 extinct; word 1: failing step
};

// Work item of the row-parallel kernels and of the sweep: instance index,
// first row (or first family id), and the role of a post-kernel workgroup.
enum PostRole : uint32_t { kRoleCopies = 0, kRoleFamilies = 1, kRoleOverlap = 2 };
struct Work {
    uint32_t inst;
    uint32_t row0;
    uint32_t role;
    uint32_t pad;
};

}  // namespace pamc
