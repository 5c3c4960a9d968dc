// launch.h -- host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pamc_dev.h"

namespace pamc {

// CM: colour-major, +-1 couplings (CM2T, CM3T: two or three colours with the
// neighbour offsets in an LDS table); CQ: colour-major, real couplings; SQ: CQ on the
// square lattice (four neighbours)
enum SweepVariant {
    kSweepLex = 0,
    kSweepEO8 = 1,
    kSweepEO16 = 2,
    kSweepCM2 = 3,
    kSweepCM3 = 4,
    kSweepCQ2 = 5,
    kSweepCQ3 = 6,
    kSweepSQ2 = 7,
    kSweepSQ3 = 8,
    kSweepCM2T = 9,
    kSweepCM3T = 10
};

// Dynamic LDS a sweep workgroup may take: gfx950 gives one workgroup up to
// 160 KB, of which 12 KB stay for the kernels' static LDS (the step
// measurement's reduction trees).
constexpr int kMaxSweepLds = 160 * 1024 - 12 * 1024;
// Lets every sweep kernel launch with up to kMaxSweepLds bytes of dynamic
// LDS (above the default of 64 KB); returns the HIP status.
hipError_t sweep_kernels_init();

// LDS stride of the byte planes of a colour-major replica quad: rows of at
// most 64 bytes keep their length (their four planes fall in disjoint LDS
// banks); longer ones are padded to a multiple of 256 bytes, so that every
// plane starts at bank 0 and the lanes of a wave reading consecutive words
// of any planes never collide.
inline int cm_plane_bytes(int row_bytes) { return row_bytes <= 64 ? row_bytes : (row_bytes + 255) & ~255; }

// Threads of a colour-major sweep workgroup of rp quads of tpr threads:
// whole waves; quads above 64 threads leave the last wave's spare lanes
// idle (tpr * rp is a multiple of 64 below).
inline int cm_launch_threads(int tpr, int rp) { return (tpr * rp + 63) / 64 * 64; }

// LDS of the neighbour table of the table forms: per colour and Philox
// block (tpr records a colour) 24 slot offsets of 16 bits, 48 bytes; 16
// more for its alignment.
inline int cm_table_bytes(int variant, int tpr)
{
    return variant == kSweepCM2T ? 16 + 96 * tpr : variant == kSweepCM3T ? 16 + 144 * tpr : 0;
}

// LDS stride of one replica-quad slot of `planes` byte planes.  Below 64
// threads per quad one wave sweeps 64 / tpr quads side by side; unpadded,
// their slots (a multiple of 64 words for rows longer than 64 bytes, 128
// words at L = 4) would start in the same LDS bank and every plane read would
// conflict 64 / tpr ways.  The slot is padded so that its length in words is
// congruent to max(tpr, 4) modulo the 64 banks: quad q then starts q tpr
// banks on, and lane q tpr + g reading word g of a plane hits bank (lane +
// const) mod 64.  Quads of 64 or more threads fill whole waves and take no
// padding.  The result is a multiple of 16 bytes (slots hold 16-byte rows).
inline int cm_slot_bytes(int row_bytes, int tpr, int planes)
{
    const int base = planes * cm_plane_bytes(row_bytes);
    if (tpr >= 64) return base;
    const int want = 4 * (tpr < 4 ? 4 : tpr);  // bytes, modulo 256
    return base + (((want - base) % 256) + 256) % 256;
}

// LDS of one cluster-move pair (the island search of one lane group): the
// sector flags of every lexicographic site (a byte: bit 0 where the replicas
// differ, bit 1 where they agree), the visited bits, the
// island queue (16-bit site indices; an island lies in the smaller sector,
// so it holds at most (N + 1) / 2 sites) and its tail, each part a multiple
// of 16 bytes, so that every pair's slice starts 16-byte aligned.
constexpr int icm_pair_bytes(int N)
{
    return ((N + 15) & ~15) + ((4 * ((N + 31) / 32) + 15) & ~15) + ((2 * ((N + 1) / 2) + 15) & ~15) + 16;
}
// the largest lattice the library accepts (L = 32) fits one pair per workgroup
static_assert(icm_pair_bytes(32 * 32 * 32) <= kMaxSweepLds, "cluster-move pair exceeds the LDS of a workgroup");

// default number of replica quads a colour-major workgroup sweeps at once
// (tpr threads per quad)
int cm_replicas_per_block(int tpr);
// replicas swept at once by an even/odd-x workgroup (L = 8 or 16); its tile
// holds a multiple of this many rows
int eo_replicas_per_pass(int L);

// lds_bytes: staging for packed rows (max(16384, row_bytes) when any instance
// of the launch is packed, else 0)
void launch_init(const Inst *insts, const Work *work, int nwork, size_t lds_bytes, hipStream_t st);
void launch_energy(const Inst *insts, const Work *work, int nwork, const int8_t *const *Jraw, hipStream_t st);
// sweeps of one temperature step; the last workgroup of each instance also
// measures the step and prepares its resampling table
// (tpr, rp: threads per replica quad and replica quads per workgroup of the
// colour-major kernel; unused by the others).  phase 0: all N_S sweeps;
// with cluster moves, phase 1: the first floor(N_S/2) sweeps (no energies,
// no measurement), phase 2: the rest with energies and the measurement.
void launch_sweep(int variant, const Inst *insts, const Work *work, int nwork, int tile_rows, int row_bytes, int tpr,
                  int rp, int phase, hipStream_t st);
// resampling weights and their normaliser (instances with real couplings;
// work items are 1024-row blocks)
void launch_weights(const Inst *insts, const Work *work, int nwork, hipStream_t st);
// one round of isoenergetic cluster moves (work items: instance, pair
// index); N: the largest lattice of the launch (sizes the LDS)
void launch_icm(const Inst *insts, const Work *work, int nwork, int N, int round, hipStream_t st);
hipError_t icm_kernels_init();
// copy counts, family entropy, overlap; the last workgroup of each instance
// finishes the prefix sum and advances the step
void launch_post(const Inst *insts, const Work *work, int nwork, hipStream_t st);
// copy map of the resampling just done
void launch_expand(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_gather(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_flip(const Inst *insts, const uint32_t *list, int n, hipStream_t st);

}  // namespace pamc
