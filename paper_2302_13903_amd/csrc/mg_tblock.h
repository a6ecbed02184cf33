// mg_tblock.h -- temporally blocked smoothing passes (internal; see mg_tblock.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mg_common.h"

namespace mg {

// nsweeps (1 or 2) full red-then-black sweeps of an n^3 level (n >= 64) in one pass:
// uin -> uout (distinct arrays).  With ec != nullptr, the trilinear prolongation of the coarse
// correction ec ((n/2)^3, ghosts from bcc) is added to u before the sweeps.
template <typename T>
void tb_sweeps(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int nsweeps, int n, double h,
               double omega, const LevelBC& bc, hipStream_t s);

// Kernel name as the profiler lists it.
template <typename T>
std::string tb_name(int nsweeps, bool pro);

}  // namespace mg
