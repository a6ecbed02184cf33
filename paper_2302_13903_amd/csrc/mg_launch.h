// mg_launch.h -- host-side declarations of the kernel launchers (internal to the library).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "mg_common.h"

namespace mg {

constexpr int kMaxPartials = 2048;   // per-block partial sums of the two-stage reductions

// Timing of the next launch (one per host thread).  The solver arms it with two created events
// before a timed launcher that takes it; a single kernel then carries the events in its own
// dispatch (start and end timestamps of that kernel, with no marker packet queued between it
// and its neighbours), a launcher of several kernels records them around its launches.
struct LaunchTiming {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  bool armed = false;
};
LaunchTiming& launch_timing();

// One kernel launch, timed through the armed hook when there is one.
template <typename K, typename... Args>
void launch_maybe_timed(K kern, dim3 grid, dim3 block, unsigned lds, hipStream_t s, Args... args) {
  LaunchTiming& t = launch_timing();
  if (t.armed) {
    t.armed = false;
    hipExtLaunchKernelGGL(kern, grid, block, lds, s, t.e0, t.e1, 0u, args...);
  } else {
    hipLaunchKernelGGL(kern, grid, block, lds, s, args...);
  }
}

inline int ilog2(long long n) {
  int l = 0;
  while ((1LL << l) < n) ++l;
  return l;
}

enum : int { TAIL_FMG = 1, TAIL_LOAD_U = 2, TAIL_FAS = 4 };

// Arguments of the coarse-tail kernel (all levels <= 16^3 of one hierarchy in LDS).
struct TailArgs {
  int top;            // highest level held (level 0 is one cell)
  int total;          // cells over levels 0..top (set by the launcher)
  int mode;           // TAIL_FMG / TAIL_LOAD_U bits
  int npre, npost;
  double omega;
  double h[5];        // cell width per level
  LevelBC bc_top;     // description of level `top` in V-cycle mode
  LevelBC hom;        // homogeneous description (coarse corrections)
  LevelBC phys[5];    // physical description per level (FMG mode)
  const void* fg[5];  // device source per level (FMG mode: all levels; V-cycle mode: top only)
  void* ug;           // device solution / correction of level `top` (in and out)
};

template <typename T>
void launch_half_sweep(T* u, const T* f, int n, double h, double omega, int colour, const LevelBC& bc,
                       hipStream_t s);
template <typename T>
void launch_defect(const T* u, const T* f, T* d, int n, double h, const LevelBC& bc, hipStream_t s);
template <typename T>
void launch_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int n, double h, const LevelBC& bc,
                            hipStream_t s);
template <typename Tin, typename Tout>
void launch_restrict(const Tin* uf, Tout* uc, int nc, hipStream_t s);
template <typename T>
void launch_prolong(const T* uc, T* uf, int nc, const LevelBC& bcc, int cubic, hipStream_t s);
template <typename T>
void launch_coarsest(T* u, const T* f, double h, const LevelBC& bc, hipStream_t s);
template <typename T>
void launch_tail(const TailArgs& a, hipStream_t s);
size_t tail_lds_bytes(int top, size_t elem);
// Allows the FP64 tail the LDS of its FAS form (u, f and phibar of levels 0..4); returns
// whether it fits.
bool tail_fas_prepare(size_t lds_per_block);
// Allows the FP64 tail its dynamic LDS; returns the highest level it can hold (3 or 4).
int tail_prepare(size_t lds_per_block);

// FAS (Alg. 3): fc = restricted defect, pbar = uc = restricted u; f += L pbar on the coarse
// level; u -= pbar (the coarse-grid correction)
void launch_fas_restrict(const double* u, const double* f, double* fc, double* pbar, double* uc, int n, double h,
                         const LevelBC& bc, hipStream_t s);
void launch_fas_source(const double* pbar, double* f, int n, double h, const LevelBC& bc, hipStream_t s);
void launch_fas_correction(double* u, const double* pbar, size_t n3, hipStream_t s);

// f = a rho + c (and its FP32 copy when f32 != nullptr); sumsq[0] = sum of f^2 (device).
// c = -a * rho_sum[0] / n3 when rho_sum (device) is given (the gauge-free source), else 0.
void launch_source(const double* rho, double* f, float* f32, size_t n3, double a, const double* rho_sum,
                   double* part, double* sumsq, hipStream_t s);
void launch_sub_mean(double* u, size_t n3, const double* sum_dev, hipStream_t s);
void launch_f32_to_f64(const float* a, double* b, size_t n3, hipStream_t s);
void launch_add_f32(double* phi, const float* e, size_t n3, hipStream_t s);

int reduce_blocks(size_t n3);
// what: 0 = sum x, 1 = sum x^2, 2 = count of non-finite values; result in out[0] (device)
void launch_sum(const double* x, size_t n3, int what, double* part, double* out, hipStream_t s);
// out[0] = sum of part[0..np) in index order (second stage of a deterministic reduction)
// Publish *src (device) to dst_host[0] and then seq to dst_host[1] (coherent pinned memory);
// done != nullptr: that event takes the end of the publishing kernel (from its own dispatch).
void launch_publish(const double* src, unsigned long long* dst_host, unsigned long long seq, hipStream_t s,
                    hipEvent_t done);
void launch_sum_partials(const double* part, int np, double* out, hipStream_t s);
void launch_defect_norm(const double* u, const double* f, float* r32, int n, double h, const LevelBC& bc,
                        double* part, double* out, hipStream_t s);

// zero `bytes` of device memory at p (8-byte aligned) with a kernel
void launch_zero(void* p, size_t bytes, hipStream_t s);

// out ((n+2)^3) = u with its ghost layer, edges and corners included, filled from bc
void launch_fill(const double* u, double* out, int n, const LevelBC& bc, hipStream_t s);

void launch_face_extend(const double* b, double* e, int n, hipStream_t s);
void launch_face_restrict(const double* ef, double* ec, int nc, hipStream_t s);

// multipole (mg_multipole.hip)
// moments[0..3] = (M, Mx, My, Mz) sums; origin[3]; q[25]
// rho of n^3 cells, dense (Lm = 0) or in the MeshBlock layout with 2^Lm-cell blocks
void launch_multipole_moments(const double* rho, int n, int Lm, double dx, int lmax, int use_origin,
                              const double* origin_host, double* part, double* scratch, hipStream_t s);
// faces[f]: (nl + 2 ext)^2 values over transverse positions (t + 1/2) hl, t = -ext .. nl - 1 + ext
void launch_multipole_faces(const double* scratch, int lmax, double G, int nl, double hl, double length,
                            double* faces[6], hipStream_t s, int ext = 1);
// Moments over the cells of up to kMpMaxBoxes boxes (dense, x fastest), skipping each box's
// covered sub-box [hlo, hhi); cell (i, j, k) of a box sits at ((o + i + 1/2) h, ..).  part holds
// multipole_box_blocks() * nbox * 25 doubles; scratch as above.
constexpr int kMpMaxBoxes = 9;
struct MpBox {
  const double* rho;
  int n[3], o[3], hlo[3], hhi[3];
  double h;
};
int multipole_box_blocks();
// returns MG_ERR_INVALID_ARG (nothing launched) unless 1 <= nbox <= kMpMaxBoxes
int launch_multipole_moments_boxes(const MpBox* boxes, int nbox, int lmax, int use_origin, const double* origin_host,
                                   double centre, double* part, double* scratch, hipStream_t s);

// gravitational acceleration (mg_gravity.hip): g, rhog (3 n^3 each) and gface (3 n^2 (n+1),
// dense layout only) from phi, any of them null; returns the number of workgroups launched
int launch_gravity(const double* phi, const double* rho, double* g, double* rhog, double* gface, int n, int Lm,
                   double dx, const LevelBC& bc, hipStream_t s);
std::string gravity_kernel_name(int n, int Lm, bool g, bool rhog, bool gface);

}  // namespace mg
