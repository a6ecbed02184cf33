// mg_fused.h -- bandwidth-optimised fused smoothing kernels for the large levels.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mg_common.h"

namespace mg {

// True when the fused kernel handles an n^3 level in precision T.
template <typename T>
bool fused_supported(int n);

// `sweeps` red-then-black RB-SOR sweeps of u (eqs. rbsor1-2), identical in result to
// 2*sweeps single-colour launches.
template <typename T>
void launch_fused_smooth(T* u, const T* f, int n, double h, double omega, int sweeps, const LevelBC& bc,
                         hipStream_t s);

// Kernel name and algorithmic HBM bytes of one launch (for the roofline report).
template <typename T>
std::string fused_smooth_name(int n, int sweeps);
template <typename T>
double fused_smooth_bytes(int n, int sweeps);

}  // namespace mg
