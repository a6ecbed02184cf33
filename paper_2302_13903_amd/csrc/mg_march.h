// mg_march.h -- two-sweep streaming passes of the large levels (internal; see mg_march.hip).
//
// Each pass reads u from `uin` and writes the result to `uout` (uin != uout): tiles overlap in
// their halos, so the update cannot be in place.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mg_common.h"

namespace mg {

// Smallest level the two-sweep passes run on (a z chunk must hold many planes).
constexpr int kMarchMinN = 128;

// A second stream and two events for splitting a pass of a level with x or y walls into the
// interior tiles and the wall tiles, run concurrently (owned by the caller; unused when null).
struct MarchAux {
  hipStream_t s2 = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};

// Down step of a V-cycle level (Alg. 1 steps 1-3) in one pass: two smoothing sweeps of u, the
// defect of the result restricted into fc, and the coarse correction uc0 cleared.
// uin == nullptr: u is zero on input and is not read.
// Lm > 0: the level is in the MeshBlock layout with blocks of 2^Lm cells per side (the coarse
// level below in the layout with blocks of 2^(Lm-1), or the dense root grid when Lm = 1).
template <typename T>
void march_down(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, double h, double omega, const LevelBC& bc,
                hipStream_t s, int Lm = 0, const MarchAux* aux = nullptr);

// Up step (Alg. 1 steps 5-7) in one pass: u += trilinear(ec) (ec's ghosts from bcc) as u is
// loaded, then two smoothing sweeps.  part != nullptr: one partial sum of squared defects of
// the result per workgroup into part (the convergence norm, Sec. 2.3.7); returns the number of
// partials (0 without part).
template <typename T>
int march_up(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, double* part, int n, double h,
             double omega, const LevelBC& bc, hipStream_t s, int Lm = 0, const MarchAux* aux = nullptr);

// Down step of a Full Approximation Scheme cycle (Alg. 3 steps 1-4) in one pass: two sweeps,
// the defect of the result restricted into fc, the result itself restricted into pbar (phibar)
// and the coarse level started from it (uc0 = phibar).
template <typename T>
void march_down_fas(const T* uin, T* uout, const T* f, T* fc, T* pbar, T* uc0, int n, double h, double omega,
                    const LevelBC& bc, hipStream_t s);

template <typename T>
std::string march_fas_name(const LevelBC& bc);

// Names of the kernels as the profiler lists them (the wall form follows bc's kinds; blk:
// MeshBlock layout).
template <typename T>
std::string march_name(bool up, bool norm, const LevelBC& bc, bool blk = false);

}  // namespace mg
