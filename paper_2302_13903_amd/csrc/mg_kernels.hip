// mg_kernels.hip -- per-operator HIP kernels (gfx950) of the multigrid solver, in FP64 and FP32.
//
// These are the plain one-operator-per-launch kernels used on every level below the fused
// large-level kernels, by the operator entry points, and as the building blocks of the
// FP32 inner cycle of the mixed-precision path.  Each kernel is a streaming loop with
// 64-bit indices and on-the-fly boundary ghosts (see mg_common.h).
#include <algorithm>

#include "mg_common.h"
#include "mg_launch.h"

namespace mg {

LaunchTiming& launch_timing() {
  static thread_local LaunchTiming t;
  return t;
}

constexpr int kBlock = 256;

static inline unsigned grid_for(size_t work, int per_thread = 1) {
  size_t threads = (work + per_thread - 1) / per_thread;
  size_t g = (threads + kBlock - 1) / kBlock;
  return (unsigned)(g == 0 ? 1 : g);
}

// ------------------------------------------------------------------ smoothing (eqs. rbsor1-2)

// One colour of the over-relaxed red-black Gauss-Seidel update.  Work item t covers the
// x-pair (2p, 2p+1) of row (j, k); exactly one of the two has the requested colour.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_half_sweep(T* __restrict__ u, const T* __restrict__ f, int n,
                                                        int L, T h2, T omega, int colour, LevelBC bc) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t pairs = (size_t)1 << (3 * L - 1);
  if (t >= pairs) return;
  const int p = (int)(t & (size_t)((n >> 1) - 1));
  const int j = (int)((t >> (L - 1)) & (size_t)(n - 1));
  const int k = (int)(t >> (2 * L - 1));
  const int i = 2 * p + ((j + k + colour) & 1);
  const size_t c = cidx(L, i, j, k);
  const T uc = u[c];
  const T nb = neighbour_sum(u, n, L, i, j, k, c, uc, bc);
  u[c] = uc + omega * ((nb - h2 * f[c]) * (T)(1.0 / 6.0) - uc);
}

template <typename T>
void launch_half_sweep(T* u, const T* f, int n, double h, double omega, int colour, const LevelBC& bc,
                       hipStream_t s) {
  const int L = ilog2(n);
  const size_t pairs = (size_t)1 << (3 * L - 1);
  hipLaunchKernelGGL(k_half_sweep<T>, dim3(grid_for(pairs)), dim3(kBlock), 0, s, u, f, n, L, (T)(h * h),
                     (T)omega, colour, bc);
}

// ------------------------------------------------------------------ defect (eq. defect)

template <typename T>
__global__ void __launch_bounds__(kBlock) k_defect(const T* __restrict__ u, const T* __restrict__ f,
                                                    T* __restrict__ d, int n, int L, T ih2, LevelBC bc) {
  const size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ((size_t)1 << (3 * L))) return;
  const int i = (int)(c & (size_t)(n - 1));
  const int j = (int)((c >> L) & (size_t)(n - 1));
  const int k = (int)(c >> (2 * L));
  const T uc = u[c];
  const T nb = neighbour_sum(u, n, L, i, j, k, c, uc, bc);
  d[c] = f[c] - (nb - (T)6 * uc) * ih2;
}

template <typename T>
void launch_defect(const T* u, const T* f, T* d, int n, double h, const LevelBC& bc, hipStream_t s) {
  const int L = ilog2(n);
  hipLaunchKernelGGL(k_defect<T>, dim3(grid_for((size_t)1 << (3 * L))), dim3(kBlock), 0, s, u, f, d, n, L,
                     (T)(1.0 / (h * h)), bc);
}

// Defect on the fine level restricted straight to the coarse level (Alg. 1 steps 2-3): one
// work item per coarse cell computes its 8 children's defects and their mean; it also clears
// the coarse correction (the recursion starts from zero, Alg. 1 step 4).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_defect_restrict(const T* __restrict__ u, const T* __restrict__ f,
                                                             T* __restrict__ fc, T* __restrict__ uc0, int n,
                                                             int L, T ih2, LevelBC bc) {
  const int nc = n >> 1, Lc = L - 1;
  const size_t C = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (C >= ((size_t)1 << (3 * Lc))) return;
  const int I = (int)(C & (size_t)(nc - 1));
  const int J = (int)((C >> Lc) & (size_t)(nc - 1));
  const int K = (int)(C >> (2 * Lc));
  T s = (T)0;
#pragma unroll
  for (int c3 = 0; c3 < 2; ++c3)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c3;
        const size_t c = cidx(L, i, j, k);
        const T ucv = u[c];
        const T nb = neighbour_sum(u, n, L, i, j, k, c, ucv, bc);
        s += f[c] - (nb - (T)6 * ucv) * ih2;
      }
  fc[C] = s * (T)0.125;
  if (uc0) uc0[C] = (T)0;
}

template <typename T>
void launch_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int n, double h, const LevelBC& bc,
                            hipStream_t s) {
  const int L = ilog2(n);
  hipLaunchKernelGGL(k_defect_restrict<T>, dim3(grid_for((size_t)1 << (3 * (L - 1)))), dim3(kBlock), 0, s, u,
                     f, fc, uc0, n, L, (T)(1.0 / (h * h)), bc);
}

// ------------------------------------------------------------------ FAS transfers (Alg. 3)

// Alg. 3 steps 2-4 and the coarse initial guess of step 6: per coarse cell the restricted
// defect of its 8 children (into fc), the restricted potential phibar (into pbar) and the
// coarse iterate set to phibar (into uc).
__global__ void __launch_bounds__(kBlock) k_fas_restrict(const double* __restrict__ u, const double* __restrict__ f,
                                                          double* __restrict__ fc, double* __restrict__ pbar,
                                                          double* __restrict__ uc, int n, int L, double ih2,
                                                          LevelBC bc) {
  const int nc = n >> 1, Lc = L - 1;
  const size_t C = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (C >= ((size_t)1 << (3 * Lc))) return;
  const int I = (int)(C & (size_t)(nc - 1));
  const int J = (int)((C >> Lc) & (size_t)(nc - 1));
  const int K = (int)(C >> (2 * Lc));
  double sd = 0.0, su = 0.0;
#pragma unroll
  for (int c3 = 0; c3 < 2; ++c3)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c3;
        const size_t c = cidx(L, i, j, k);
        const double ucv = u[c];
        const double nb = neighbour_sum(u, n, L, i, j, k, c, ucv, bc);
        sd += f[c] - (nb - 6.0 * ucv) * ih2;
        su += ucv;
      }
  fc[C] = sd * 0.125;
  const double pb = su * 0.125;
  pbar[C] = pb;
  uc[C] = pb;
}

void launch_fas_restrict(const double* u, const double* f, double* fc, double* pbar, double* uc, int n, double h,
                         const LevelBC& bc, hipStream_t s) {
  const int L = ilog2(n);
  hipLaunchKernelGGL(k_fas_restrict, dim3(grid_for((size_t)1 << (3 * (L - 1)))), dim3(kBlock), 0, s, u, f, fc, pbar,
                     uc, n, L, 1.0 / (h * h), bc);
}

// Alg. 3 step 5 on the coarse level: f += L phibar, with phibar's ghosts from the level's
// physical description.
__global__ void __launch_bounds__(kBlock) k_fas_source(const double* __restrict__ pbar, double* __restrict__ f, int n,
                                                        int L, double ih2, LevelBC bc) {
  const size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (c >= ((size_t)1 << (3 * L))) return;
  const int i = (int)(c & (size_t)(n - 1));
  const int j = (int)((c >> L) & (size_t)(n - 1));
  const int k = (int)(c >> (2 * L));
  const double pc = pbar[c];
  const double nb = neighbour_sum(pbar, n, L, i, j, k, c, pc, bc);
  f[c] = f[c] + (nb - 6.0 * pc) * ih2;
}

void launch_fas_source(const double* pbar, double* f, int n, double h, const LevelBC& bc, hipStream_t s) {
  const int L = ilog2(n);
  hipLaunchKernelGGL(k_fas_source, dim3(grid_for((size_t)1 << (3 * L))), dim3(kBlock), 0, s, pbar, f, n, L,
                     1.0 / (h * h), bc);
}

// Alg. 3 step 7: the coarse-grid correction psi - phibar, in place of psi.
__global__ void __launch_bounds__(kBlock) k_fas_correction(double* __restrict__ u, const double* __restrict__ pbar,
                                                            size_t n3) {
  const size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (c < n3) u[c] = u[c] - pbar[c];
}

void launch_fas_correction(double* u, const double* pbar, size_t n3, hipStream_t s) {
  hipLaunchKernelGGL(k_fas_correction, dim3(grid_for(n3)), dim3(kBlock), 0, s, u, pbar, n3);
}

// ------------------------------------------------------------------ restriction (eq. restriction)

template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlock) k_restrict(const Tin* __restrict__ uf, Tout* __restrict__ uc, int Lc) {
  const int nc = 1 << Lc, L = Lc + 1;
  const size_t C = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (C >= ((size_t)1 << (3 * Lc))) return;
  const int I = (int)(C & (size_t)(nc - 1));
  const int J = (int)((C >> Lc) & (size_t)(nc - 1));
  const int K = (int)(C >> (2 * Lc));
  Tin s = (Tin)0;
#pragma unroll
  for (int c3 = 0; c3 < 2; ++c3)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) s += uf[cidx(L, 2 * I + a, 2 * J + b, 2 * K + c3)];
  uc[C] = (Tout)(s * (Tin)0.125);
}

template <typename Tin, typename Tout>
void launch_restrict(const Tin* uf, Tout* uc, int nc, hipStream_t s) {
  const int Lc = ilog2(nc);
  hipLaunchKernelGGL((k_restrict<Tin, Tout>), dim3(grid_for((size_t)1 << (3 * Lc))), dim3(kBlock), 0, s, uf,
                     uc, Lc);
}

// ------------------------------------------------------------------ prolongation (Sec. 2.3.1)

// cubic = 0: uf += trilinear(uc) (eq. trilinear, Alg. 1 steps 5-6);
// cubic = 1: uf  = tricubic(uc)  (FMG prolongation, Alg. 2 step 3).
// One work item per coarse cell: it gathers the 3x3x3 coarse neighbourhood once (through the
// ghost rules only in the first and last rows and planes) and writes its 8 children as four
// 2-cell row segments.
// One-dimensional prolongation of the coarse values a, b, c at offsets -1, 0, +1 to the lower
// (upper = 0) or upper child, with the weights of lin_w / cub_w (zero weights left out).
template <typename T, int CUBIC>
__device__ __forceinline__ T interp3(int upper, T a, T b, T c) {
  if (CUBIC) {
    return upper ? ((T)(-3.0 / 32.0) * a + (T)(30.0 / 32.0) * b) + (T)(5.0 / 32.0) * c
                 : ((T)(5.0 / 32.0) * a + (T)(30.0 / 32.0) * b) + (T)(-3.0 / 32.0) * c;
  }
  return upper ? (T)0.75 * b + (T)0.25 * c : (T)0.25 * a + (T)0.75 * b;
}

template <typename T, int CUBIC>
__global__ void __launch_bounds__(kBlock) k_prolong(const T* __restrict__ uc, T* __restrict__ uf, int Lc,
                                                     LevelBC bcc) {
  const int nc = 1 << Lc, L = Lc + 1;
  const size_t C = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (C >= ((size_t)1 << (3 * Lc))) return;
  const int I = (int)(C & (size_t)(nc - 1));
  const int J = (int)((C >> Lc) & (size_t)(nc - 1));
  const int K = (int)(C >> (2 * Lc));
  // res[zc][yc][xc]: child (2I + xc, 2J + yc, 2K + zc), each the sum over the taps (cz, by, ax)
  // in that order of (wx * wy * wz) * tap (the same terms in the same order in both branches)
  T res[2][2][2];
  if (J > 0 && J < nc - 1 && K > 0 && K < nc - 1) {
    // rows inside in y and z (every row of the grid has its two x-boundary cells, so these
    // must not leave the fast path): the 27 taps read directly, the x-neighbour beyond an x
    // face given by that face's rule -- the wrapped cell, the cell itself (zero gradient) or
    // 2b - u (a value b on the face) -- as the ghost rules give it; every weight a constant
    const int Im = I > 0 ? I - 1 : nc - 1, Ip = I < nc - 1 ? I + 1 : 0;
    const bool wlo = I == 0 && bcc.kind[0] != BC_PERIODIC, whi = I == nc - 1 && bcc.kind[1] != BC_PERIODIC;
    T v[3][3][3];
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
      for (int by = 0; by < 3; ++by) {
        const int Jr = J + by - 1, Kr = K + cz - 1;
        const size_t row = cidx(Lc, 0, Jr, Kr);
        const T u0 = uc[row + (size_t)I];
        T um = uc[row + (size_t)Im], up = uc[row + (size_t)Ip];
        if (wlo) um = bcc.kind[0] == BC_ZERO_GRADIENT ? u0 : (T)(2.0 * face_b(bcc, 0, nc, Jr, Kr)) - u0;
        if (whi) up = bcc.kind[1] == BC_ZERO_GRADIENT ? u0 : (T)(2.0 * face_b(bcc, 1, nc, Jr, Kr)) - u0;
        v[cz][by][0] = um;
        v[cz][by][1] = u0;
        v[cz][by][2] = up;
      }
    // the weights are a product of one-dimensional ones: interpolate in x (nine rows), then in
    // y (three planes), then in z -- 114 multiply-adds for the eight children instead of 216
    T ex[3][3][2], ey[3][2][2];
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
      for (int by = 0; by < 3; ++by)
#pragma unroll
        for (int xc = 0; xc < 2; ++xc) ex[cz][by][xc] = interp3<T, CUBIC>(xc, v[cz][by][0], v[cz][by][1], v[cz][by][2]);
#pragma unroll
    for (int cz = 0; cz < 3; ++cz)
#pragma unroll
      for (int yc = 0; yc < 2; ++yc)
#pragma unroll
        for (int xc = 0; xc < 2; ++xc) ey[cz][yc][xc] = interp3<T, CUBIC>(yc, ex[cz][0][xc], ex[cz][1][xc], ex[cz][2][xc]);
#pragma unroll
    for (int zc = 0; zc < 2; ++zc)
#pragma unroll
      for (int yc = 0; yc < 2; ++yc)
#pragma unroll
        for (int xc = 0; xc < 2; ++xc) res[zc][yc][xc] = interp3<T, CUBIC>(zc, ey[0][yc][xc], ey[1][yc][xc], ey[2][yc][xc]);
  } else {
    // the first and last rows and planes: one tap at a time through the ghost rules (a loop,
    // so the ghost code is in the kernel once), added to all eight children
#pragma unroll
    for (int zc = 0; zc < 2; ++zc)
#pragma unroll
      for (int yc = 0; yc < 2; ++yc)
#pragma unroll
        for (int xc = 0; xc < 2; ++xc) res[zc][yc][xc] = (T)0;
#pragma unroll 1
    for (int t = 0; t < 27; ++t) {
      const int ax = t % 3, by = (t / 3) % 3, cz = t / 9;
      const T val = ghost_any(uc, nc, Lc, I + ax - 1, J + by - 1, K + cz - 1, bcc);
#pragma unroll
      for (int zc = 0; zc < 2; ++zc)
#pragma unroll
        for (int yc = 0; yc < 2; ++yc)
#pragma unroll
          for (int xc = 0; xc < 2; ++xc) {
            T wx[3], wy[3], wz[3];
            if (CUBIC) { cub_w<T>(xc, wx); cub_w<T>(yc, wy); cub_w<T>(zc, wz); }
            else { lin_w<T>(xc, wx); lin_w<T>(yc, wy); lin_w<T>(zc, wz); }
            // the weights of this tap (selects: no runtime-indexed arrays)
            const T a = ax == 0 ? wx[0] : (ax == 1 ? wx[1] : wx[2]);
            const T b = by == 0 ? wy[0] : (by == 1 ? wy[1] : wy[2]);
            const T c = cz == 0 ? wz[0] : (cz == 1 ? wz[1] : wz[2]);
            if (!CUBIC && (a == (T)0 || b == (T)0 || c == (T)0)) continue;
            res[zc][yc][xc] += (a * b * c) * val;
          }
    }
  }
  // the two x-children are adjacent (even index first): one vector access per child row; the
  // FMG result is written past the caches (it is read again only by the next pass, and kept
  // out of L2 it leaves room there for the coarse rows the neighbouring workgroups read:
  // 455 -> 360 us at 512^3)
  typedef T tv2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int zc = 0; zc < 2; ++zc)
#pragma unroll
    for (int yc = 0; yc < 2; ++yc) {
      tv2* fp = reinterpret_cast<tv2*>(uf + cidx(L, 2 * I, 2 * J + yc, 2 * K + zc));
      if (CUBIC) {
        __builtin_nontemporal_store(tv2{res[zc][yc][0], res[zc][yc][1]}, fp);
      } else {
        const tv2 o = *fp;
        *fp = tv2{o.x + res[zc][yc][0], o.y + res[zc][yc][1]};
      }
    }
}

template <typename T>
void launch_prolong(const T* uc, T* uf, int nc, const LevelBC& bcc, int cubic, hipStream_t s) {
  const int Lc = ilog2(nc);
  const dim3 g(grid_for((size_t)1 << (3 * Lc)));
  if (cubic) hipLaunchKernelGGL((k_prolong<T, 1>), g, dim3(kBlock), 0, s, uc, uf, Lc, bcc);
  else hipLaunchKernelGGL((k_prolong<T, 0>), g, dim3(kBlock), 0, s, uc, uf, Lc, bcc);
}

// ------------------------------------------------------------------ coarsest (Sec. 2.3.2)

// Single-cell solve: every ghost is alpha*u + beta (periodic / zero-gradient: alpha = 1,
// fixed: alpha = -1, beta = 2b), so u = (sum beta - h^2 f) / (6 - sum alpha); 0 if sum alpha = 6.
template <typename T>
__device__ __forceinline__ T coarsest_value(T f, T h2, const LevelBC& bc) {
  T sa = (T)0, sb = (T)0;
#pragma unroll
  for (int face = 0; face < 6; ++face) {
    if (bc_has_value(bc.kind[face])) { sa -= (T)1; sb += (T)(2.0 * face_b(bc, face, 1, 0, 0)); }
    else sa += (T)1;
  }
  return sa == (T)6 ? (T)0 : (sb - h2 * f) / ((T)6 - sa);
}

template <typename T>
__global__ void k_coarsest(T* u, const T* f, T h2, LevelBC bc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) u[0] = coarsest_value(f[0], h2, bc);
}

template <typename T>
void launch_coarsest(T* u, const T* f, double h, const LevelBC& bc, hipStream_t s) {
  hipLaunchKernelGGL(k_coarsest<T>, dim3(1), dim3(64), 0, s, u, f, (T)(h * h), bc);
}

// ------------------------------------------------------------------ coarse tail (levels <= 2^TL)

// All levels 0..T (T <= 4, at most 16^3 cells) of one hierarchy in LDS, one workgroup.
// mode bits: TAIL_FMG runs Alg. 2 on levels 0..T with the physical description of each level
// and writes u_T; otherwise one V-cycle (Alg. 1) at level T with bc_top (u_T loaded from
// global when TAIL_LOAD_U, else started from zero) and homogeneous descriptions below.
constexpr int kTailThreads = 1024;

// Start of level l within the LDS arrays (levels 0..top stored back to back): the cells of
// levels 0..l-1, sum of 8^q for q < l = (8^l - 1) / 7.
__host__ __device__ __forceinline__ constexpr int level_offset(int l) { return ((1 << (3 * l)) - 1) / 7; }

// KIND 1: every face of every description the launch uses is periodic.  Ghosts are then the
// opposite cells, read by wrapping the index; this leaves the boundary code of the other kinds
// out of the kernel image, which the tail's many short phases fetch cold otherwise (measured
// 36 against 98 us for the tail from 16^3).  KIND 2: no description carries face values (the
// homogeneous conditions of a V-cycle's coarse levels): a wall's ghost is kappa times the
// cell's own value, taken by a select after a wrapped (always in range) read, with no
// boundary branches either.  KIND 0: the general ghost rules.  Same values, same order of
// operations.
// The walls of a description without face values: per face, the ghost's factor on the cell's
// own value (0 for a periodic face: never used).
template <typename T>
struct WallRule {
  T k[6];
  __device__ __forceinline__ explicit WallRule(const LevelBC& bc) {
#pragma unroll
    for (int f = 0; f < 6; ++f)
      k[f] = bc.kind[f] == BC_PERIODIC ? (T)0 : (bc.kind[f] == BC_ZERO_GRADIENT ? (T)1 : (T)-1);
  }
};

// LDS index of cell (i, j, k) of a level of 2^L cells per side (32-bit: LDS arrays are small)
__device__ __forceinline__ int lds_idx(int L, int i, int j, int k) { return (k << (2 * L)) | (j << L) | i; }

template <typename T, int KIND>
__device__ __forceinline__ T lds_nb(const T* u, int n, int L, int i, int j, int k, T uc, const LevelBC& bc,
                                    const WallRule<T>& wr) {
  if (KIND != 0) {
    const int m = n - 1;
    T xm = u[lds_idx(L, (i - 1) & m, j, k)], xp = u[lds_idx(L, (i + 1) & m, j, k)];
    T ym = u[lds_idx(L, i, (j - 1) & m, k)], yp = u[lds_idx(L, i, (j + 1) & m, k)];
    T zm = u[lds_idx(L, i, j, (k - 1) & m)], zp = u[lds_idx(L, i, j, (k + 1) & m)];
    if (KIND == 2) {
      if (i == 0 && wr.k[0] != (T)0) xm = wr.k[0] * uc;
      if (i == m && wr.k[1] != (T)0) xp = wr.k[1] * uc;
      if (j == 0 && wr.k[2] != (T)0) ym = wr.k[2] * uc;
      if (j == m && wr.k[3] != (T)0) yp = wr.k[3] * uc;
      if (k == 0 && wr.k[4] != (T)0) zm = wr.k[4] * uc;
      if (k == m && wr.k[5] != (T)0) zp = wr.k[5] * uc;
    }
    return ((((xm + xp) + ym) + yp) + zm) + zp;
  }
  const size_t c = cidx(L, i, j, k);
  return neighbour_sum(u, n, L, i, j, k, c, uc, bc);
}

// KIND 2: a coarse index beyond a wall without values: wrapped (periodic) or clamped to the
// boundary cell with the sign of the wall's rule.
template <typename T>
__device__ __forceinline__ int wall_tap(int c, int nc, int klo, int khi, T& s) {
  if (c < 0) {
    if (klo == BC_PERIODIC) return nc - 1;
    if (klo != BC_ZERO_GRADIENT) s = -s;
    return 0;
  }
  if (c >= nc) {
    if (khi == BC_PERIODIC) return 0;
    if (khi != BC_ZERO_GRADIENT) s = -s;
    return nc - 1;
  }
  return c;
}

// One smoothing sweep on an LDS-resident level: work items enumerate only the cells of the
// current colour (the x-pair index p picks the pair's cell of that colour), so no lane idles.
template <typename T, int KIND>
__device__ __forceinline__ void tail_smooth(T* u, const T* f, int L, T h2, T omega, const LevelBC& bc) {
  const int n = 1 << L;
  const T inv6 = (T)(1.0 / 6.0);
  const int half = 1 << (3 * L - 1);
  const WallRule<T> wr(bc);
#pragma unroll 1
  for (int colour = 0; colour < 2; ++colour) {
#pragma unroll 1
    for (int t = threadIdx.x; t < half; t += blockDim.x) {
      const int p = t & ((n >> 1) - 1), j = (t >> (L - 1)) & (n - 1), k = t >> (2 * L - 1);
      const int i = 2 * p + ((j + k + colour) & 1);
      const int c = lds_idx(L, i, j, k);
      const T uc = u[c];
      const T nb = lds_nb<T, KIND>(u, n, L, i, j, k, uc, bc, wr);
      u[c] = uc + omega * ((nb - h2 * f[c]) * inv6 - uc);
    }
    __syncthreads();
  }
}

template <typename T, int KIND>
__device__ __forceinline__ void tail_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int L, T ih2, const LevelBC& bc) {
  const int n = 1 << L, Lc = L - 1, nc = n >> 1, nc3 = 1 << (3 * Lc);
  const WallRule<T> wr(bc);
#pragma unroll 1
  for (int C = threadIdx.x; C < nc3; C += blockDim.x) {
    const int I = C & (nc - 1), J = (C >> Lc) & (nc - 1), K = C >> (2 * Lc);
    T s = (T)0;
    for (int c3 = 0; c3 < 2; ++c3)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c3;
          const int c = lds_idx(L, i, j, k);
          const T ucv = u[c];
          s += f[c] - (lds_nb<T, KIND>(u, n, L, i, j, k, ucv, bc, wr) - (T)6 * ucv) * ih2;
        }
    fc[C] = s * (T)0.125;
    uc0[C] = (T)0;
  }
  __syncthreads();
}

template <typename T, int CUBIC, int KIND>
__device__ __forceinline__ void tail_prolong(const T* uc, T* uf, int L, const LevelBC& bcc) {
  const int n = 1 << L, n3 = 1 << (3 * L), Lc = L - 1, nc = n >> 1;
#pragma unroll 1
  for (int c = threadIdx.x; c < n3; c += blockDim.x) {
    const int i = c & (n - 1), j = (c >> L) & (n - 1), k = c >> (2 * L);
    const int I = i >> 1, J = j >> 1, K = k >> 1;
    const bool inner = I > 0 && I < nc - 1 && J > 0 && J < nc - 1 && K > 0 && K < nc - 1;
    T wx[3], wy[3], wz[3];
    if (CUBIC) { cub_w(i & 1, wx); cub_w(j & 1, wy); cub_w(k & 1, wz); }
    else { lin_w(i & 1, wx); lin_w(j & 1, wy); lin_w(k & 1, wz); }
    T s = (T)0;
    if (!CUBIC && KIND != 0) {
      // trilinear: on each axis the tap of weight zero is the third (even fine index) or the
      // first (odd), so the two others are slots o, o+1 with o = the index's parity; each
      // axis's two coarse indices (wrapped, or clamped with the wall's sign) are taken once,
      // and the eight terms are summed in the order of the 27-tap loop below
      const int ox = i & 1, oy = j & 1, oz = k & 1;
      int xo[2], yo[2], zo[2];
      T xs[2], ys[2], zs[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        xs[d] = ys[d] = zs[d] = (T)1;
        if (KIND == 1) {
          xo[d] = (I - 1 + ox + d) & (nc - 1);
          yo[d] = ((J - 1 + oy + d) & (nc - 1)) << Lc;
          zo[d] = ((K - 1 + oz + d) & (nc - 1)) << (2 * Lc);
        } else {
          xo[d] = wall_tap<T>(I - 1 + ox + d, nc, bcc.kind[0], bcc.kind[1], xs[d]);
          yo[d] = wall_tap<T>(J - 1 + oy + d, nc, bcc.kind[2], bcc.kind[3], ys[d]) << Lc;
          zo[d] = wall_tap<T>(K - 1 + oz + d, nc, bcc.kind[4], bcc.kind[5], zs[d]) << (2 * Lc);
        }
      }
#pragma unroll
      for (int cz = 0; cz < 2; ++cz)
#pragma unroll
        for (int by = 0; by < 2; ++by)
#pragma unroll
          for (int ax = 0; ax < 2; ++ax) {
            const T w = wx[ox + ax] * wy[oy + by] * wz[oz + cz];
            const T v = uc[zo[cz] | yo[by] | xo[ax]];
            if (KIND == 1) s += w * v;
            else s += w * (((xs[ax] * ys[by]) * zs[cz]) * v);
          }
      uf[c] += s;
      continue;
    }
#pragma unroll
    for (int cz = -1; cz <= 1; ++cz)
#pragma unroll
      for (int by = -1; by <= 1; ++by)
#pragma unroll
        for (int ax = -1; ax <= 1; ++ax) {
          const T w = wx[ax + 1] * wy[by + 1] * wz[cz + 1];
          if (w == (T)0) continue;
          if (KIND == 1) {
            s += w * uc[lds_idx(Lc, (I + ax) & (nc - 1), (J + by) & (nc - 1), (K + cz) & (nc - 1))];
          } else if (KIND == 2) {
            T sg = (T)1;
            const int Ic = wall_tap<T>(I + ax, nc, bcc.kind[0], bcc.kind[1], sg);
            const int Jc = wall_tap<T>(J + by, nc, bcc.kind[2], bcc.kind[3], sg);
            const int Kc = wall_tap<T>(K + cz, nc, bcc.kind[4], bcc.kind[5], sg);
            s += w * (sg * uc[lds_idx(Lc, Ic, Jc, Kc)]);
          } else {
            s += w * (inner ? uc[cidx(Lc, I + ax, J + by, K + cz)] : ghost_any(uc, nc, Lc, I + ax, J + by, K + cz, bcc));
          }
        }
    if (CUBIC) uf[c] = s;
    else uf[c] += s;
  }
  __syncthreads();
}

// Per-launch metadata copied to LDS once, so per-level lookups with a runtime level index
// read LDS instead of spilling the argument block to private memory.
struct TailMeta {
  LevelBC phys[5];
  LevelBC top;   // description of the top level in V-cycle mode
  LevelBC hom;
  double h2[5];
};

// V-cycle from level `topl` down to 0 and back, with bc_top on level topl and the
// homogeneous description below.
template <typename T, int KIND>
__device__ __forceinline__ void tail_vcycle(T* base, int total, int topl, const TailMeta& m, const LevelBC& bc_top, int npre,
                            int npost, T omega) {
#pragma unroll 1
  for (int l = topl; l >= 1; --l) {
    const LevelBC bc = l == topl ? bc_top : m.hom;   // by value: kinds in registers
    T* u = base + level_offset(l);
    T* f = base + total + level_offset(l);
    const T h2 = (T)m.h2[l];
#pragma unroll 1
    for (int it = 0; it < npre; ++it) tail_smooth<T, KIND>(u, f, l, h2, omega, bc);
    tail_defect_restrict<T, KIND>(u, f, base + total + level_offset(l - 1), base + level_offset(l - 1), l, (T)(1.0 / m.h2[l]),
                         bc);
  }
  const LevelBC hom = m.hom;
  if (threadIdx.x == 0) base[0] = coarsest_value(base[total], (T)m.h2[0], topl == 0 ? bc_top : hom);
  __syncthreads();
#pragma unroll 1
  for (int l = 1; l <= topl; ++l) {
    const LevelBC bc = l == topl ? bc_top : hom;
    T* u = base + level_offset(l);
    tail_prolong<T, 0, KIND>(base + level_offset(l - 1), u, l, hom);
#pragma unroll 1
    for (int it = 0; it < npost; ++it) tail_smooth<T, KIND>(u, base + total + level_offset(l), l, (T)m.h2[l], omega, bc);
  }
}

// FAS (Alg. 3 steps 2-7) on an LDS-resident level: the restricted defect into the coarse
// source, the restricted u (phibar) into the coarse level's phibar and starting iterate --
// the same terms in the same order as the per-operator FAS restriction
template <typename T, int KIND>
__device__ __forceinline__ void tail_fas_restrict(const T* u, const T* f, T* fc, T* pbar, T* uc, int L, T ih2,
                                                  const LevelBC& bc) {
  const int n = 1 << L, Lc = L - 1, nc = n >> 1, nc3 = 1 << (3 * Lc);
  const WallRule<T> wr(bc);
#pragma unroll 1
  for (int C = threadIdx.x; C < nc3; C += blockDim.x) {
    const int I = C & (nc - 1), J = (C >> Lc) & (nc - 1), K = C >> (2 * Lc);
    T sd = (T)0, su = (T)0;
    for (int c3 = 0; c3 < 2; ++c3)
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c3;
          const int c = lds_idx(L, i, j, k);
          const T ucv = u[c];
          sd += f[c] - (lds_nb<T, KIND>(u, n, L, i, j, k, ucv, bc, wr) - (T)6 * ucv) * ih2;
          su += ucv;
        }
    fc[C] = sd * (T)0.125;
    const T pb = su * (T)0.125;
    pbar[C] = pb;
    uc[C] = pb;
  }
  __syncthreads();
}

// f += L phibar on an LDS-resident level, phibar's ghosts from the level's physical description
template <typename T, int KIND>
__device__ __forceinline__ void tail_fas_source(const T* pbar, T* f, int L, T ih2, const LevelBC& bc) {
  const int n = 1 << L, n3 = 1 << (3 * L);
  const WallRule<T> wr(bc);
#pragma unroll 1
  for (int c = threadIdx.x; c < n3; c += blockDim.x) {
    const int i = c & (n - 1), j = (c >> L) & (n - 1), k = c >> (2 * L);
    const T pc = pbar[c];
    f[c] = f[c] + (lds_nb<T, KIND>(pbar, n, L, i, j, k, pc, bc, wr) - (T)6 * pc) * ih2;
  }
  __syncthreads();
}

// One FAS cycle (Alg. 3) from level topl down to 0 and back, each level with its physical
// description; phibar of each level at base + 2 total.  Only the forms without face values
// (KIND 1, 2).  The single cell is solved when a face fixes the zero point (a zero-valued
// fixed face) and otherwise keeps phibar (a zero correction), as in the per-operator cycle.
template <typename T, int KIND>
__device__ __forceinline__ void tail_fas_vcycle(T* base, int total, int topl, const TailMeta& m, int npre, int npost,
                                                T omega) {
  T* pbase = base + 2 * total;
#pragma unroll 1
  for (int l = topl; l >= 1; --l) {
    const LevelBC bc = m.phys[l];
    T* u = base + level_offset(l);
    T* f = base + total + level_offset(l);
#pragma unroll 1
    for (int it = 0; it < npre; ++it) tail_smooth<T, KIND>(u, f, l, (T)m.h2[l], omega, bc);
    tail_fas_restrict<T, KIND>(u, f, base + total + level_offset(l - 1), pbase + level_offset(l - 1),
                               base + level_offset(l - 1), l, (T)(1.0 / m.h2[l]), bc);
    const LevelBC bcc = m.phys[l - 1];
    tail_fas_source<T, KIND>(pbase + level_offset(l - 1), base + total + level_offset(l - 1), l - 1,
                             (T)(1.0 / m.h2[l - 1]), bcc);
  }
  if (threadIdx.x == 0) {
    const LevelBC b0 = m.phys[0];
    bool fixes = false;
    for (int f = 0; f < 6; ++f) fixes = fixes || bc_has_value(b0.kind[f]);
    if (fixes) base[0] = coarsest_value(base[total], (T)m.h2[0], b0);
  }
  __syncthreads();
  const LevelBC hom = m.hom;
#pragma unroll 1
  for (int l = 1; l <= topl; ++l) {
    // the coarse-grid correction psi - phibar, prolonged with the homogeneous conditions
    T* uc = base + level_offset(l - 1);
    const T* pc = pbase + level_offset(l - 1);
    const int nc3 = 1 << (3 * (l - 1));
    for (int c = threadIdx.x; c < nc3; c += blockDim.x) uc[c] = uc[c] - pc[c];
    __syncthreads();
    T* u = base + level_offset(l);
    tail_prolong<T, 0, KIND>(uc, u, l, hom);
    const LevelBC bc = m.phys[l];
#pragma unroll 1
    for (int it = 0; it < npost; ++it) tail_smooth<T, KIND>(u, base + total + level_offset(l), l, (T)m.h2[l], omega, bc);
  }
}

template <typename T, int KIND>
__global__ void __launch_bounds__(kTailThreads) k_tail(TailArgs a) {
  const T* const* fg = reinterpret_cast<const T* const*>(a.fg);
  T* ug = reinterpret_cast<T*>(a.ug);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ TailMeta m;
  T* base = reinterpret_cast<T*>(smem_raw);
  const int total = a.total, top = a.top;
  if (threadIdx.x == 0) {
    for (int l = 0; l < 5; ++l) {
      m.phys[l] = a.phys[l];
      m.h2[l] = a.h[l] * a.h[l];
    }
    m.top = a.bc_top;
    m.hom = a.hom;
  }
  __syncthreads();
  const int ntop = 1 << (3 * top);
  const T omega = (T)a.omega;
  const bool fmg = (a.mode & TAIL_FMG) != 0;
  if (fmg) {
    for (int l = 0; l <= top; ++l) {
      const int n3 = 1 << (3 * l);
      const T* src = fg[l];
      T* dst = base + total + level_offset(l);
      for (int c = threadIdx.x; c < n3; c += blockDim.x) dst[c] = src[c];
    }
    __syncthreads();
    if (threadIdx.x == 0) base[0] = coarsest_value(base[total], (T)m.h2[0], m.phys[0]);
  } else {
    T* u = base + level_offset(top);
    T* f = base + total + level_offset(top);
    const T* src = fg[top];
    for (int c = threadIdx.x; c < ntop; c += blockDim.x) {
      f[c] = src[c];
      u[c] = (a.mode & TAIL_LOAD_U) ? ug[c] : (T)0;
    }
  }
  __syncthreads();
  // Alg. 2 (FMG): on each level l = 1..top, the tricubic prolongation, then one V-cycle with
  // the level's own physical description (the V-cycle on level l overwrites the sources below
  // with restricted defects, which FMG no longer needs: it proceeds upwards).  V-cycle mode:
  // the one V-cycle on level top.  One copy of the V-cycle code serves both (a small kernel
  // image keeps the instruction cache warm across the many short phases).
  if ((a.mode & TAIL_FAS) != 0) {
    if constexpr (KIND != 0) tail_fas_vcycle<T, KIND>(base, total, top, m, a.npre, a.npost, omega);
  } else {
#pragma unroll 1
    for (int l = fmg ? 1 : top; l <= top; ++l) {
      if (fmg) {
        const LevelBC below = m.phys[l - 1];
        tail_prolong<T, 1, KIND>(base + level_offset(l - 1), base + level_offset(l), l, below);
      }
      const LevelBC here = fmg ? m.phys[l] : m.top;
      tail_vcycle<T, KIND>(base, total, l, m, here, a.npre, a.npost, omega);
    }
  }
  const T* u = base + level_offset(top);
  for (int c = threadIdx.x; c < ntop; c += blockDim.x) ug[c] = u[c];
}

template <typename T>
void launch_tail(const TailArgs& a, hipStream_t s) {
  TailArgs b = a;
  b.total = level_offset(a.top + 1);
  // FAS: phibar of every level beside u and f
  const size_t lds = ((b.mode & TAIL_FAS) ? 3 : 2) * (size_t)b.total * sizeof(T);
  // the periodic form when every description this launch reads is periodic
  auto periodic = [](const LevelBC& q) {
    for (int f = 0; f < 6; ++f)
      if (q.kind[f] != BC_PERIODIC) return false;
    return true;
  };
  // the wall form when no description carries face values
  auto valueless = [](const LevelBC& q) {
    for (int f = 0; f < 6; ++f)
      if (q.kind[f] != BC_PERIODIC && q.kind[f] != BC_ZERO_GRADIENT && q.b[f]) return false;
    return true;
  };
  // FMG and FAS read every level's physical description
  const bool fmg = (b.mode & (TAIL_FMG | TAIL_FAS)) != 0;
  bool per = periodic(b.hom) && (fmg || periodic(b.bc_top));
  bool walls = valueless(b.hom) && (fmg || valueless(b.bc_top));
  if (fmg)
    for (int l = 0; l <= b.top; ++l) {
      per = per && periodic(b.phys[l]);
      walls = walls && valueless(b.phys[l]);
    }
  if (per)
    hipLaunchKernelGGL((k_tail<T, 1>), dim3(1), dim3(kTailThreads), lds, s, b);
  else if (walls)
    hipLaunchKernelGGL((k_tail<T, 2>), dim3(1), dim3(kTailThreads), lds, s, b);
  else
    hipLaunchKernelGGL((k_tail<T, 0>), dim3(1), dim3(kTailThreads), lds, s, b);
}

// the FAS form (forms 1 and 2 only) holds phibar beside u and f
static size_t tail_fas_lds(int top) { return tail_lds_bytes(top, sizeof(double)) / 2 * 3; }

bool tail_fas_prepare(size_t lds_per_block) { return lds_per_block >= tail_fas_lds(4); }

int tail_prepare(size_t lds_per_block) {
  const size_t need64 = tail_lds_bytes(4, sizeof(double));
  const size_t need32 = tail_lds_bytes(4, sizeof(float));
  for (const void* k : {reinterpret_cast<const void*>(&k_tail<float, 0>), reinterpret_cast<const void*>(&k_tail<float, 1>),
                        reinterpret_cast<const void*>(&k_tail<float, 2>)})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)need32);
  if (lds_per_block < need64) return 3;
  // forms 1 and 2 also run the FAS cycle, with phibar beside u and f, where that fits
  const size_t need_fas = tail_fas_lds(4);
  const size_t need12 = lds_per_block >= need_fas ? need_fas : need64;
  const void* k64[3] = {reinterpret_cast<const void*>(&k_tail<double, 0>),
                        reinterpret_cast<const void*>(&k_tail<double, 1>),
                        reinterpret_cast<const void*>(&k_tail<double, 2>)};
  for (int q = 0; q < 3; ++q)
    if (hipFuncSetAttribute(k64[q], hipFuncAttributeMaxDynamicSharedMemorySize, (int)(q == 0 ? need64 : need12)) !=
        hipSuccess) {
      (void)hipGetLastError();
      return 3;
    }
  return 4;
}



size_t tail_lds_bytes(int top, size_t elem) {
  size_t total = 0;
  for (int l = 0; l <= top; ++l) total += (size_t)1 << (3 * l);
  return 2 * total * elem;
}

// ------------------------------------------------------------------ elementwise / set-up

// u += shift (gauge fix, Sec. 2.3.6)
__global__ void __launch_bounds__(kBlock) k_shift(double* __restrict__ u, size_t n3, const double* __restrict__ sum,
                                                   double scale) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n3) return;
  u[t] -= sum[0] * scale;
}

void launch_sub_mean(double* u, size_t n3, const double* sum_dev, hipStream_t s) {
  hipLaunchKernelGGL(k_shift, dim3(grid_for(n3)), dim3(kBlock), 0, s, u, n3, sum_dev, 1.0 / (double)n3);
}

template <typename Ta, typename Tb>
__global__ void __launch_bounds__(kBlock) k_copy_convert(const Ta* __restrict__ a, Tb* __restrict__ b, size_t n3) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n3) b[t] = (Tb)a[t];
}

void launch_f32_to_f64(const float* a, double* b, size_t n3, hipStream_t s) {
  hipLaunchKernelGGL((k_copy_convert<float, double>), dim3(grid_for(n3)), dim3(kBlock), 0, s, a, b, n3);
}

// phi64 += e32 (mixed precision correction, defect equation eq. defecteq)
__global__ void __launch_bounds__(kBlock) k_add_f32(double* __restrict__ phi, const float* __restrict__ e, size_t n3) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t < n3) phi[t] += (double)e[t];
}

void launch_add_f32(double* phi, const float* e, size_t n3, hipStream_t s) {
  hipLaunchKernelGGL(k_add_f32, dim3(grid_for(n3)), dim3(kBlock), 0, s, phi, e, n3);
}

// ------------------------------------------------------------------ reductions

// Deterministic two-stage sums: stage 1 writes one partial per block (grid-stride loop, fixed
// grid, fixed tree); stage 2 sums the partials in index order in one block.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int q = 0; q < kBlock / 64; ++q) r += red[q];
  }
  __syncthreads();
  return r;
}

// what: 0 = sum x, 1 = sum x^2, 2 = sum of squared non-finite flags (count of NaN/Inf)
__global__ void __launch_bounds__(kBlock) k_sum_partials(const double* __restrict__ x, size_t n3, int what,
                                                          double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n3; t += (size_t)gridDim.x * kBlock) {
    const double v = x[t];
    acc += what == 0 ? v : (what == 1 ? v * v : (isfinite(v) ? 0.0 : 1.0));
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(kBlock) k_sum_final(const double* __restrict__ part, int np, int stride,
                                                       double* __restrict__ out, int nvals) {
  // out[v] = sum_{b < np} part[b*stride + v] in index order, v < nvals
  __shared__ double red[kBlock / 64];
  for (int v = 0; v < nvals; ++v) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < np; b += kBlock) acc += part[(size_t)b * stride + v];
    const double r = block_sum(acc, red);
    if (threadIdx.x == 0) out[v] = r;
  }
}

int reduce_blocks(size_t n3) {
  size_t b = (n3 + (size_t)kBlock * 8 - 1) / ((size_t)kBlock * 8);
  if (b > (size_t)kMaxPartials) b = kMaxPartials;
  return (int)(b < 1 ? 1 : b);
}

// One device scalar copied into coherent pinned host memory (dst[0]), then the sequence number
// `seq` stored beside it (dst[1]) with system-scope release, so that a host that sees the number
// also sees the value.  Vector stores from one lane.
__global__ void k_publish(const double* __restrict__ src, unsigned long long* dst, unsigned long long seq) {
  if (threadIdx.x != 0) return;
  __hip_atomic_store(dst, __builtin_bit_cast(unsigned long long, src[0]), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_SYSTEM);
  __hip_atomic_store(dst + 1, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

void launch_publish(const double* src, unsigned long long* dst_host, unsigned long long seq, hipStream_t s,
                    hipEvent_t done) {
  if (done) hipExtLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, nullptr, done, 0u, src, dst_host, seq);
  else hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, src, dst_host, seq);
}

void launch_sum_partials(const double* part, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, np, 1, out, 1);
}

void launch_sum(const double* x, size_t n3, int what, double* part, double* out, hipStream_t s) {
  const int nb = reduce_blocks(n3);
  hipLaunchKernelGGL(k_sum_partials, dim3(nb), dim3(kBlock), 0, s, x, n3, what, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, nb, 1, out, 1);
}

// Defect of the finest level and its sum of squares (Sec. 2.3.7, eq. threshold); optionally
// the defect itself in FP32 (mixed precision: right-hand side of the inner correction cycle).
__global__ void __launch_bounds__(kBlock) k_defect_norm(const double* __restrict__ u, const double* __restrict__ f,
                                                         float* __restrict__ r32, int n, int L, double ih2, LevelBC bc,
                                                         double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  const size_t n3 = (size_t)1 << (3 * L);
  double acc = 0.0;
  for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < n3; c += (size_t)gridDim.x * kBlock) {
    const int i = (int)(c & (size_t)(n - 1));
    const int j = (int)((c >> L) & (size_t)(n - 1));
    const int k = (int)(c >> (2 * L));
    const double uc = u[c];
    const double nb = neighbour_sum(u, n, L, i, j, k, c, uc, bc);
    const double d = f[c] - (nb - 6.0 * uc) * ih2;
    acc += d * d;
    if (r32) r32[c] = (float)d;
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void launch_defect_norm(const double* u, const double* f, float* r32, int n, double h, const LevelBC& bc,
                        double* part, double* out, hipStream_t s) {
  const int L = ilog2(n);
  const size_t n3 = (size_t)1 << (3 * L);
  const int nb = reduce_blocks(n3);
  hipLaunchKernelGGL(k_defect_norm, dim3(nb), dim3(kBlock), 0, s, u, f, r32, n, L, 1.0 / (h * h), bc, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, nb, 1, out, 1);
}

// f = a * rho + c (the source 4 pi G rho, mean-shifted when gauge-free: c = -a * mean(rho),
// read from the device so that the host need not wait for the sum), in FP64, plus the
// FP32 copy when f32 != nullptr, and one partial sum of f^2 per block (fixed grid and tree,
// so the sum is reproducible).
__global__ void __launch_bounds__(kBlock) k_source(const double* __restrict__ rho, double* __restrict__ f,
                                                    float* __restrict__ f32, size_t n3, double a,
                                                    const double* __restrict__ rho_sum, double* __restrict__ part) {
  __shared__ double red[kBlock / 64];
  // gauge-free: c = -a * mean(rho), from the sum the previous launch left in device memory
  const double c = rho_sum ? -a * (rho_sum[0] / (double)n3) : 0.0;
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x; t < n3; t += (size_t)gridDim.x * kBlock) {
    const double v = a * rho[t] + c;
    f[t] = v;
    if (f32) f32[t] = (float)v;
    acc += v * v;
  }
  const double r = block_sum(acc, red);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

void launch_source(const double* rho, double* f, float* f32, size_t n3, double a, const double* rho_sum,
                   double* part, double* sumsq, hipStream_t s) {
  const int nb = reduce_blocks(n3);
  hipLaunchKernelGGL(k_source, dim3(nb), dim3(kBlock), 0, s, rho, f, f32, n3, a, rho_sum, part);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(kBlock), 0, s, part, nb, 1, sumsq, 1);
}

// ------------------------------------------------------------------ boundary face arrays

// Finest-level FIXED face: extend the caller's n^2 face-centre array to (n+2)^2, the ring
// taking the nearest face value.
__global__ void __launch_bounds__(kBlock) k_face_extend(const double* __restrict__ b, double* __restrict__ e, int n) {
  const int m = n + 2;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= m * m) return;
  const int t1 = t % m - 1, t2 = t / m - 1;
  const int c1 = t1 < 0 ? 0 : (t1 >= n ? n - 1 : t1);
  const int c2 = t2 < 0 ? 0 : (t2 >= n ? n - 1 : t2);
  e[t] = b ? b[(size_t)c2 * n + c1] : 0.0;
}

// Coarser FIXED face: 2x2 area mean of the finer face values, then the extension ring.
__global__ void __launch_bounds__(kBlock) k_face_restrict(const double* __restrict__ ef, double* __restrict__ ec, int nc) {
  const int m = nc + 2, nf = 2 * nc, mf = nf + 2;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= m * m) return;
  int t1 = t % m - 1, t2 = t / m - 1;
  t1 = t1 < 0 ? 0 : (t1 >= nc ? nc - 1 : t1);
  t2 = t2 < 0 ? 0 : (t2 >= nc ? nc - 1 : t2);
  const double* r0 = ef + (size_t)(2 * t2 + 1) * mf + 1;
  const double* r1 = ef + (size_t)(2 * t2 + 2) * mf + 1;
  ec[t] = (r0[2 * t1] + r0[2 * t1 + 1] + r1[2 * t1] + r1[2 * t1 + 1]) / 4.0;
}

// ------------------------------------------------------------------ clearing device memory

// Zero `words` 8-byte words (a kernel rather than a memset node, so the clear is an ordinary
// kernel wherever the stream's work is recorded).
__global__ void __launch_bounds__(kBlock) k_zero(unsigned long long* __restrict__ p, size_t words) {
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = t; i < words; i += stride) p[i] = 0ull;
}
__global__ void k_zero_bytes(unsigned char* __restrict__ p, size_t bytes) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < bytes) p[t] = 0;
}

void launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  const size_t words = bytes / 8, tail = bytes % 8;
  if (words) {
    const size_t g = std::min<size_t>((words + kBlock - 1) / kBlock, 8192);
    hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(kBlock), 0, s, reinterpret_cast<unsigned long long*>(p), words);
  }
  if (tail)
    hipLaunchKernelGGL(k_zero_bytes, dim3(1), dim3(8), 0, s, reinterpret_cast<unsigned char*>(p) + words * 8, tail);
}

// ------------------------------------------------------------------ ghost fill (Sec. 2.3.6)

// The ghost-filled copy of one level: out is (n+2)^3, x fastest, with active cell (i, j, k) at
// ((k+1)(n+2) + j+1)(n+2) + i+1 and every ghost -- faces, edges and corners -- set by the
// axis-ordered rule the prolongations read (x first, then y over the x ghosts, then z over
// both), i.e. the value ghost_any evaluates on the fly.
__global__ void __launch_bounds__(kBlock) k_fill(const double* __restrict__ u, double* __restrict__ out, int n,
                                                  int L, LevelBC bc) {
  const size_t m = (size_t)n + 2;
  const size_t t = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= m * m * m) return;
  const int i = (int)(t % m) - 1, j = (int)((t / m) % m) - 1, k = (int)(t / (m * m)) - 1;
  const bool inside = i >= 0 && i < n && j >= 0 && j < n && k >= 0 && k < n;
  out[t] = inside ? u[cidx(L, i, j, k)] : ghost_any(u, n, L, i, j, k, bc);
}

void launch_fill(const double* u, double* out, int n, const LevelBC& bc, hipStream_t s) {
  const size_t m = (size_t)n + 2;
  hipLaunchKernelGGL(k_fill, dim3(grid_for(m * m * m)), dim3(kBlock), 0, s, u, out, n, ilog2(n), bc);
}

void launch_face_extend(const double* b, double* e, int n, hipStream_t s) {
  const int m = n + 2;
  hipLaunchKernelGGL(k_face_extend, dim3((m * m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, b, e, n);
}

void launch_face_restrict(const double* ef, double* ec, int nc, hipStream_t s) {
  const int m = nc + 2;
  hipLaunchKernelGGL(k_face_restrict, dim3((m * m + kBlock - 1) / kBlock), dim3(kBlock), 0, s, ef, ec, nc);
}

// ------------------------------------------------------------------ explicit instantiations

#define MG_INST(T)                                                                                   \
  template void launch_half_sweep<T>(T*, const T*, int, double, double, int, const LevelBC&, hipStream_t); \
  template void launch_defect<T>(const T*, const T*, T*, int, double, const LevelBC&, hipStream_t);        \
  template void launch_defect_restrict<T>(const T*, const T*, T*, T*, int, double, const LevelBC&,         \
                                          hipStream_t);                                                    \
  template void launch_prolong<T>(const T*, T*, int, const LevelBC&, int, hipStream_t);                    \
  template void launch_coarsest<T>(T*, const T*, double, const LevelBC&, hipStream_t);                     \
  template void launch_tail<T>(const TailArgs&, hipStream_t);

MG_INST(double)
MG_INST(float)
template void launch_restrict<double, double>(const double*, double*, int, hipStream_t);
template void launch_restrict<float, float>(const float*, float*, int, hipStream_t);
template void launch_restrict<double, float>(const double*, float*, int, hipStream_t);

}  // namespace mg
