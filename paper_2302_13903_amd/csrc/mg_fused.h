// mg_fused.h -- fused z-marching smoothing passes for the large levels (internal).
//
// Every pass reads u from `uin` and writes the swept u to `uout` (uin != uout): tiles overlap
// in their halos, so the update cannot be in place.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mg_common.h"

namespace mg {

// Smallest level size the fused passes can handle, and the smallest the solver uses them for
// by default (below it a z-marching workgroup has too few planes and tiles to hide latency,
// and one launch per operator is faster: measured on 512^3 V-cycles).
constexpr int kFusedMinN = 64;
constexpr int kFusedDefaultMinN = 256;

template <typename T>
bool fused_supported(int n);

// One red-then-black sweep.  uin == nullptr: u is zero on input (not read).
template <typename T>
void fused_sweep(const T* uin, T* uout, const T* f, int n, double h, double omega, const LevelBC& bc,
                 hipStream_t s);

// One sweep, then the defect restricted into fc (coarse level) and uc0 cleared.
template <typename T>
void fused_sweep_defect(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, double h, double omega,
                        const LevelBC& bc, hipStream_t s);

// u += trilinear(ec) on the fly (ec's ghosts from bcc), then one sweep.
template <typename T>
void fused_prolong_sweep(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int n, double h,
                         double omega, const LevelBC& bc, hipStream_t s);

// One sweep, then one partial sum of squared defects per block into part; returns the number
// of partials written.
template <typename T>
int fused_sweep_norm(const T* uin, T* uout, const T* f, double* part, int n, double h, double omega,
                     const LevelBC& bc, hipStream_t s);

// One sweep, and one partial sum of squared defects per block of the INPUT u (the residual of
// the iterate the sweep starts from); returns the number of partials.
template <typename T>
int fused_sweep_input_norm(const T* uin, T* uout, const T* f, double* part, int n, double h, double omega,
                           const LevelBC& bc, hipStream_t s);

// Mixed precision, FP64 part of one defect-correction step: phi_out = phi_in + e (e FP32),
// then the defect f - L phi_out, its FP32 copy r32 and one partial sum of squares per block;
// returns the number of partials.
int fused_mixed_update_defect(double* phi_in, double* phi_out, const float* e, const double* f, float* r32,
                              double* part, int n, double h, const LevelBC& bc, hipStream_t s);

// Defect-only streaming passes over the input u (nothing swept, u not written):
// the defect restricted into fc with uc0 cleared (Alg. 1 steps 2-3) ...
template <typename T>
void fused_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int n, double h, const LevelBC& bc, hipStream_t s);
// ... or one partial sum of squared defects per block into part (returns their number),
// with the defect's FP32 copy into r32 when given (the right-hand side of a mixed-precision
// correction cycle).
template <typename T>
int fused_defect_norm(const T* u, const T* f, double* part, int n, double h, const LevelBC& bc, hipStream_t s,
                      float* r32 = nullptr);

// The same streaming passes on a MeshBlock-layout level (blocks of 2^Lm cells, 2^Lb blocks per
// side; the coarse level is the layout below: blocks of 2^(Lm-1) cells, or the dense root
// grid when Lm = 1).  fused_blk_sweep: one sweep, with the prolonged correction ec added first
// when ec != nullptr.
template <typename T>
void fused_blk_sweep(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int Lm, int Lb, double h,
                     double omega, const LevelBC& bc, hipStream_t s);
template <typename T>
void fused_blk_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int Lm, int Lb, double h, const LevelBC& bc,
                               hipStream_t s);
template <typename T>
int fused_blk_defect_norm(const T* u, const T* f, double* part, int Lm, int Lb, double h, const LevelBC& bc,
                          hipStream_t s, float* r32 = nullptr);
template <typename T>
std::string fused_blk_pass_name(bool pro, int out);

// Names of the pass kernels as the profiler lists them (sweep = false: the defect-only pass).
template <typename T>
std::string fused_pass_name(bool pro, int out, bool sweep = true);

// Full Approximation Scheme (Alg. 3 steps 2-4) in one streaming pass over a dense FP64 level:
// fc = restricted defect f - L u, pbar = uc = restricted u.
void fused_fas_restrict(const double* u, const double* f, double* fc, double* pbar, double* uc, int n, double h,
                        const LevelBC& bc, hipStream_t s);
// One sweep, then the same restriction stage as fused_fas_restrict on the swept u (uout).
void fused_sweep_fas_restrict(const double* uin, double* uout, const double* f, double* fc, double* pbar, double* uc,
                              int n, double h, double omega, const LevelBC& bc, hipStream_t s);
std::string fused_fas_restrict_name(bool sweep = false);

}  // namespace mg
