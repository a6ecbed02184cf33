// mg_blocks.h -- operators on the MeshBlock layout (internal; see mg_blocks.hip for the layout).
//
// Levels are named by Lm = log2(cells per block side) and Lb = log2(blocks per side); the
// level has 2^(Lm+Lb) cells per side.  The coarse side of an operator on block level Lm = 1
// is the dense root grid of 2^Lb cells per side.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "mg_common.h"

namespace mg {

// Schedule of the block sweep: threads per workgroup, blocks staged per workgroup (G) and
// sweeps fused per launch (S, halo 2S).  Every valid schedule gives bitwise the same result:
// each cell's update is the same expression of the same operand values.
struct BlkTune {
  int threads;
  int G;
  int S;
};

constexpr int kBlkMaxLm = 4;   // blocks of up to 16^3 cells (the two-cell halo tile then fits in LDS)

int blk_periodic_mask(const LevelBC& bc);
size_t blk_sweep_lds(int Lm, int S, int G, size_t elem);
BlkTune blk_default_tune(int Lm, int Lb, size_t elem);
bool blk_tune_valid(const BlkTune& t, int Lm, int Lb, size_t elem, size_t lds_max);

template <typename T>
void blk_prepare(size_t lds_max);

// t.S red-then-black sweeps of every block in one launch: uin -> uout (distinct arrays).
template <typename T>
void blk_sweep(const T* uin, T* uout, const T* f, int Lm, int Lb, const BlkTune& t, double h, double omega,
               const LevelBC& bc, hipStream_t s);

// fc = restriction of the defect f - L u to the level below (block level Lm-1 or the root);
// uc0 (optional) = 0 on that level.
template <typename T>
void blk_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int Lm, int Lb, double h, const LevelBC& bc,
                         hipStream_t s);

// uc = restriction of uf (block level Lm) to the level below.
template <typename Tin, typename Tout>
void blk_restrict(const Tin* uf, Tout* uc, int Lm, int Lb, hipStream_t s);

// Block level Lm from the level below: cubic = 0: uf += trilinear(uc); cubic = 1: uf = tricubic(uc).
template <typename T>
void blk_prolong(const T* uc, T* uf, int Lm, int Lb, const LevelBC& bcc, int cubic, hipStream_t s);

// Partial sums of squared defects (returns their number) and optionally the FP32 defect.
int blk_defect_norm(const double* u, const double* f, float* r32, int Lm, int Lb, double h, const LevelBC& bc,
                    double* part, hipStream_t s);

}  // namespace mg
