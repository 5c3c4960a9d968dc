// launch.h -- host-side launchers of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include "pamc_dev.h"

namespace pamc {

enum SweepVariant { kSweepLex = 0, kSweepEO8 = 1, kSweepEO16 = 2 };

void launch_init(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_energy(const Inst *insts, const Work *work, int nwork, const int8_t *const *Jraw, hipStream_t st);
void launch_sweep(int variant, const Inst *insts, const Work *work, int nwork, int tile_rows, int row_bytes,
                  hipStream_t st);
void launch_gather(const Inst *insts, const Work *work, int nwork, int koff, hipStream_t st);

// per-instance kernels take the list of instance indices
void launch_measure(const Inst *insts, const uint32_t *list, int n, hipStream_t st);
void launch_famcount(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_famtree(const Inst *insts, const Work *chunks, int nchunks, hipStream_t st);
void launch_famfinal(const Inst *insts, const uint32_t *list, int n, hipStream_t st);
void launch_overlap(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_copycount(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_scan(const Inst *insts, const uint32_t *list, int n, hipStream_t st);
void launch_expand(const Inst *insts, const Work *work, int nwork, hipStream_t st);
void launch_flip(const Inst *insts, const uint32_t *list, int n, hipStream_t st);
void launch_advance(const Inst *insts, const uint32_t *list, int n, hipStream_t st);

}  // namespace pamc
