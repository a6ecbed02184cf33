// mg_tile.h -- V-cycle legs of the small levels as one launch each (internal; see mg_tile.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mg_common.h"

namespace mg {

// Smallest and largest level side the region-tile legs take (the level must hold whole
// regions of 8 x 8 x 4 cells or more; above 128^3 the streaming passes move far fewer bytes).
constexpr int kTileMinN = 32;
constexpr int kTileMaxN = 128;

// Down step of a V-cycle level (Alg. 1 steps 1-3) in one launch: two smoothing sweeps of u
// (uin -> uout, distinct arrays), the defect restricted into fc and the coarse correction uc0
// cleared.  Lm > 0: the level is in the MeshBlock layout with blocks of 2^Lm cells per side
// and 2^Lb blocks per side (the coarse level in the layout below, or the dense root grid when
// Lm = 1); Lm = 0: dense.
template <typename T>
void tile_down(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, int Lm, int Lb, double h, double omega,
               const LevelBC& bc, hipStream_t s);

// The down step of a Full Approximation Scheme cycle (Alg. 3 steps 2-4; dense FP64 levels):
// as tile_down, and phibar (the mean of the 8 children of the swept u) written to pbar and to
// uc0, the coarse level's starting iterate.
template <typename T>
void tile_down_fas(const T* uin, T* uout, const T* f, T* fc, T* pbar, T* uc0, int n, double h, double omega,
                   const LevelBC& bc, hipStream_t s);

// Up step (Alg. 1 steps 5-7) in one launch: u += trilinear(ec) (ec's ghosts from the
// homogeneous description bcc), then two sweeps (uin -> uout).  part != nullptr: one partial
// sum of squared defects of the result per workgroup (returns their number, else 0).
template <typename T>
int tile_up(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, double* part, int n, int Lm, int Lb,
            double h, double omega, const LevelBC& bc, hipStream_t s);

template <typename T>
std::string tile_name(bool up, bool norm, bool blk = false);

}  // namespace mg
