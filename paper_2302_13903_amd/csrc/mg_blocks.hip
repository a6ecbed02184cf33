// mg_blocks.hip -- multigrid operators on the MeshBlock layout (Sec. 3.2: the mesh split into
// equal cubic MeshBlocks, each block's levels coarsened down to one cell per block, those cells
// forming the root grid).
//
// Layout of a level whose blocks hold 2^Lm cells per side, with 2^Lb blocks per side: the
// blocks are stored one after another in Morton (Z-curve) order of their block coordinates,
// each block dense with x fastest.  The same block index owns the same region on every block
// level, so restriction and prolongation never leave a block; only the stencil halos reach
// into neighbouring blocks, and those are read directly from them (the device-memory
// equivalent of the paper's ghost exchange between MeshBlocks before each colour).  When the
// coarse side of an inter-level operator is one cell per block, it is the root grid, a dense
// (2^Lb)^3 array: restriction gathers into it, prolongation scatters from it.
#include <hip/hip_runtime.h>

#include "mg_blocks.h"
#include "mg_launch.h"

namespace mg {

namespace {

constexpr int kBlkThreads = 256;   // defect/restriction/prolongation/norm kernels

// Workgroups in a contiguous run per XCD (consecutive workgroups go round the 8 XCDs), so that
// Morton-neighbouring blocks, which share halos, are swept by the same XCD and its L2.
__device__ __forceinline__ unsigned xcd_remap(unsigned bid, unsigned nwg) {
  if ((nwg & 7u) != 0) return bid;
  return (bid & 7u) * (nwg >> 3) + (bid >> 3);
}

template <typename T>
__device__ __forceinline__ T wall_ghost(const LevelBC& bc, int face, int n, int t1, int t2, T uc) {
  if (bc.kind[face] == BC_ZERO_GRADIENT) return uc;
  return (T)(2.0 * face_b(bc, face, n, t1, t2)) - uc;
}

// Sum of the six face neighbours of cell (i, j, k) (value uc) on a block level, read from the
// neighbouring blocks where needed; same summation order as the dense kernels.
template <typename T>
__device__ __forceinline__ T blk_nsum(const T* __restrict__ u, int Lm, int n, int i, int j, int k, T uc,
                                      const LevelBC& bc, int per) {
  const int nm = n - 1;
  const T xm = (!(per & 1) && i == 0) ? wall_ghost(bc, 0, n, j, k, uc) : u[bidx(Lm, (i - 1) & nm, j, k)];
  const T xp = (!(per & 1) && i == nm) ? wall_ghost(bc, 1, n, j, k, uc) : u[bidx(Lm, (i + 1) & nm, j, k)];
  const T ym = (!(per & 2) && j == 0) ? wall_ghost(bc, 2, n, i, k, uc) : u[bidx(Lm, i, (j - 1) & nm, k)];
  const T yp = (!(per & 2) && j == nm) ? wall_ghost(bc, 3, n, i, k, uc) : u[bidx(Lm, i, (j + 1) & nm, k)];
  const T zm = (!(per & 4) && k == 0) ? wall_ghost(bc, 4, n, i, j, uc) : u[bidx(Lm, i, j, (k - 1) & nm)];
  const T zp = (!(per & 4) && k == nm) ? wall_ghost(bc, 5, n, i, j, uc) : u[bidx(Lm, i, j, (k + 1) & nm)];
  return ((((xm + xp) + ym) + yp) + zm) + zp;
}

// ------------------------------------------------------------------ one smoothing sweep

// S red-then-black sweeps (eqs. rbsor1-2) of G blocks per workgroup in one launch.  Each
// block is staged with a halo of 2S cells; colour pass q (red, black, red, ...) updates the
// block plus a ring of 2S-1-q cells, so every pass sees neighbours in exactly the state they
// would have after a ghost exchange; only the block itself is stored.  The rings are
// recomputed redundantly, never stored: uin and uout must differ.
template <typename T, int LM, int S>
__global__ void __launch_bounds__(1024) k_blk_sweep(const T* __restrict__ uin, T* __restrict__ uout,
                                                    const T* __restrict__ f, int Lb, int G, T h2, T omega,
                                                    LevelBC bc, int per) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  constexpr int md = 1 << LM, H = 2 * S, tw = md + 2 * H, tv = tw * tw * tw;
  const int n = md << Lb, nm = n - 1;
  const int b0 = (int)xcd_remap(blockIdx.x, gridDim.x) * G;

  for (int q = threadIdx.x; q < G * tv; q += blockDim.x) {
    const int gb = q / tv, r = q - gb * tv;
    const int tz = r / (tw * tw), r2 = r - tz * tw * tw, ty = r2 / tw, tx = r2 - ty * tw;
    int bx, by, bz;
    demorton3((unsigned)(b0 + gb), bx, by, bz);
    int i = (bx << LM) + tx - H, j = (by << LM) + ty - H, k = (bz << LM) + tz - H;
    bool in = true;
    if (per & 1) i &= nm; else in &= (unsigned)i < (unsigned)n;
    if (per & 2) j &= nm; else in &= (unsigned)j < (unsigned)n;
    if (per & 4) k &= nm; else in &= (unsigned)k < (unsigned)n;
    tile[q] = in ? uin[bidx(LM, i, j, k)] : (T)0;
  }
  __syncthreads();

#pragma unroll 1
  for (int pass = 0; pass < 2 * S; ++pass) {
    const int colour = pass & 1;
    const int ring = 2 * S - 1 - pass;
    const int o = -ring;                // region origin relative to the block
    const int R = md + 2 * ring;        // region side (even)
    const int half = R >> 1, per_blk = R * R * half;
    for (int q = threadIdx.x; q < G * per_blk; q += blockDim.x) {
      const int gb = q / per_blk, r = q - gb * per_blk;
      const int row = r / half, xi = r - row * half;
      const int ry = row % R, rz = row / R;
      int bx, by, bz;
      demorton3((unsigned)(b0 + gb), bx, by, bz);
      int j = (by << LM) + o + ry, k = (bz << LM) + o + rz;
      const int ib = (bx << LM) + o;
      const int rx = 2 * xi + ((colour - ib - j - k) & 1);
      int i = ib + rx;
      if (per & 1) i &= nm; else if ((unsigned)i >= (unsigned)n) continue;
      if (per & 2) j &= nm; else if ((unsigned)j >= (unsigned)n) continue;
      if (per & 4) k &= nm; else if ((unsigned)k >= (unsigned)n) continue;
      const int p = gb * tv + ((rz + o + H) * tw + (ry + o + H)) * tw + (rx + o + H);
      const T uc = tile[p];
      const T xm = (!(per & 1) && i == 0) ? wall_ghost(bc, 0, n, j, k, uc) : tile[p - 1];
      const T xp = (!(per & 1) && i == nm) ? wall_ghost(bc, 1, n, j, k, uc) : tile[p + 1];
      const T ym = (!(per & 2) && j == 0) ? wall_ghost(bc, 2, n, i, k, uc) : tile[p - tw];
      const T yp = (!(per & 2) && j == nm) ? wall_ghost(bc, 3, n, i, k, uc) : tile[p + tw];
      const T zm = (!(per & 4) && k == 0) ? wall_ghost(bc, 4, n, i, j, uc) : tile[p - tw * tw];
      const T zp = (!(per & 4) && k == nm) ? wall_ghost(bc, 5, n, i, j, uc) : tile[p + tw * tw];
      const T nb = ((((xm + xp) + ym) + yp) + zm) + zp;
      tile[p] = uc + omega * ((nb - h2 * f[bidx(LM, i, j, k)]) * (T)(1.0 / 6.0) - uc);
    }
    __syncthreads();
  }

  constexpr int m3 = md * md * md;
  for (int q = threadIdx.x; q < G * m3; q += blockDim.x) {
    const int gb = q >> (3 * LM), r = q & (m3 - 1);
    const int lx = r & (md - 1), ly = (r >> LM) & (md - 1), lz = r >> (2 * LM);
    uout[((size_t)(b0 + gb) << (3 * LM)) + r] = tile[gb * tv + ((lz + H) * tw + ly + H) * tw + lx + H];
  }
}

// ------------------------------------------------------------------ defect + restriction

// Coarse output index of coarse cell (I, J, K) of block blk: the coarse block level, or the
// root grid when the coarse level has one cell per block (Lc = 0).
__device__ __forceinline__ size_t coarse_out(int Lc, int Lb, size_t C, int bx, int by, int bz) {
  return Lc == 0 ? cidx(Lb, bx, by, bz) : C;
}

// fc = mean over the 8 children of the defect f - L u (Alg. 1 steps 2-3); uc0 = 0.
template <typename T>
__global__ void __launch_bounds__(kBlkThreads) k_blk_defect_restrict(const T* __restrict__ u, const T* __restrict__ f,
                                                                     T* __restrict__ fc, T* __restrict__ uc0, int Lm,
                                                                     int Lb, T ih2, LevelBC bc, int per) {
  const int Lc = Lm - 1, mc = 1 << Lc, n = 1 << (Lm + Lb);
  const size_t C = (size_t)blockIdx.x * kBlkThreads + threadIdx.x;
  if (C >= ((size_t)1 << (3 * (Lc + Lb)))) return;
  const int r = (int)(C & (size_t)((1 << (3 * Lc)) - 1));
  int bx, by, bz;
  demorton3((unsigned)(C >> (3 * Lc)), bx, by, bz);
  const int I = (bx << Lc) + (r & (mc - 1)), J = (by << Lc) + ((r >> Lc) & (mc - 1)), K = (bz << Lc) + (r >> (2 * Lc));
  T s = (T)0;
#pragma unroll
  for (int c3 = 0; c3 < 2; ++c3)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int i = 2 * I + a, j = 2 * J + b, k = 2 * K + c3;
        const size_t c = bidx(Lm, i, j, k);
        const T ucv = u[c];
        const T nb = blk_nsum(u, Lm, n, i, j, k, ucv, bc, per);
        s += f[c] - (nb - (T)6 * ucv) * ih2;
      }
  const size_t o = coarse_out(Lc, Lb, C, bx, by, bz);
  fc[o] = s * (T)0.125;
  if (uc0) uc0[o] = (T)0;
}

// uc = mean of the 8 children of uf (eq. restriction), block level -> block level or root.
template <typename Tin, typename Tout>
__global__ void __launch_bounds__(kBlkThreads) k_blk_restrict(const Tin* __restrict__ uf, Tout* __restrict__ uc,
                                                              int Lm, int Lb) {
  const int Lc = Lm - 1, mc = 1 << Lc;
  const size_t C = (size_t)blockIdx.x * kBlkThreads + threadIdx.x;
  if (C >= ((size_t)1 << (3 * (Lc + Lb)))) return;
  const int r = (int)(C & (size_t)((1 << (3 * Lc)) - 1));
  int bx, by, bz;
  demorton3((unsigned)(C >> (3 * Lc)), bx, by, bz);
  const int I = (bx << Lc) + (r & (mc - 1)), J = (by << Lc) + ((r >> Lc) & (mc - 1)), K = (bz << Lc) + (r >> (2 * Lc));
  Tin s = (Tin)0;
#pragma unroll
  for (int c3 = 0; c3 < 2; ++c3)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) s += uf[bidx(Lm, 2 * I + a, 2 * J + b, 2 * K + c3)];
  uc[coarse_out(Lc, Lb, C, bx, by, bz)] = (Tout)(s * (Tin)0.125);
}

// ------------------------------------------------------------------ prolongation

// Coarse value at (I, J, K), each in [-1, nc], edges and corners included, with the ghost
// rule filled axis by axis (x, then y, then z): the last axis is resolved first, each step an
// affine map value = s * inner + t.  The coarse level is the root grid (dense) when Lc = 0.
template <typename T>
__device__ __forceinline__ T coarse_any(const T* __restrict__ uc, int Lc, int Lb, int I, int J, int K,
                                        const LevelBC& bc) {
  const int nc = 1 << (Lc + Lb);
  T s = (T)1, t = (T)0;
  if (K < 0 || K >= nc) {
    const int face = K < 0 ? 4 : 5, kd = bc.kind[face];
    if (kd == BC_PERIODIC) {
      K = K < 0 ? nc - 1 : 0;
    } else {
      if (kd != BC_ZERO_GRADIENT) { t += s * (T)(2.0 * face_b(bc, face, nc, I, J)); s = -s; }
      K = K < 0 ? 0 : nc - 1;
    }
  }
  if (J < 0 || J >= nc) {
    const int face = J < 0 ? 2 : 3, kd = bc.kind[face];
    if (kd == BC_PERIODIC) {
      J = J < 0 ? nc - 1 : 0;
    } else {
      if (kd != BC_ZERO_GRADIENT) { t += s * (T)(2.0 * face_b(bc, face, nc, I, K)); s = -s; }
      J = J < 0 ? 0 : nc - 1;
    }
  }
  if (I < 0 || I >= nc) {
    const int face = I < 0 ? 0 : 1, kd = bc.kind[face];
    if (kd == BC_PERIODIC) {
      I = I < 0 ? nc - 1 : 0;
    } else {
      if (kd != BC_ZERO_GRADIENT) { t += s * (T)(2.0 * face_b(bc, face, nc, J, K)); s = -s; }
      I = I < 0 ? 0 : nc - 1;
    }
  }
  const size_t c = Lc == 0 ? cidx(Lb, I, J, K) : bidx(Lc, I, J, K);
  return s * uc[c] + t;
}

// Fine block level (2^Lm per block) from the coarse level below it: CUBIC = 0 adds the
// trilinear correction (eq. trilinear), CUBIC = 1 writes the tricubic FMG interpolant
// (Sec. 2.3.1).  One work item per coarse cell, in fine block order.
template <typename T, int CUBIC>
__global__ void __launch_bounds__(kBlkThreads) k_blk_prolong(const T* __restrict__ uc, T* __restrict__ uf, int Lm,
                                                             int Lb, LevelBC bcc) {
  const int Lc = Lm - 1, mc = 1 << Lc;
  const size_t C = (size_t)blockIdx.x * kBlkThreads + threadIdx.x;
  if (C >= ((size_t)1 << (3 * (Lc + Lb)))) return;
  const int r = (int)(C & (size_t)((1 << (3 * Lc)) - 1));
  int bx, by, bz;
  demorton3((unsigned)(C >> (3 * Lc)), bx, by, bz);
  const int I = (bx << Lc) + (r & (mc - 1)), J = (by << Lc) + ((r >> Lc) & (mc - 1)), K = (bz << Lc) + (r >> (2 * Lc));
  T v[3][3][3];
#pragma unroll
  for (int cz = 0; cz < 3; ++cz)
#pragma unroll
    for (int by2 = 0; by2 < 3; ++by2)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) v[cz][by2][ax] = coarse_any(uc, Lc, Lb, I + ax - 1, J + by2 - 1, K + cz - 1, bcc);
#pragma unroll
  for (int zc = 0; zc < 2; ++zc)
#pragma unroll
    for (int yc = 0; yc < 2; ++yc) {
      T wz[3], wy[3];
      if (CUBIC) { cub_w<T>(zc, wz); cub_w<T>(yc, wy); }
      else { lin_w<T>(zc, wz); lin_w<T>(yc, wy); }
#pragma unroll
      for (int xc = 0; xc < 2; ++xc) {
        T wx[3];
        if (CUBIC) cub_w<T>(xc, wx);
        else lin_w<T>(xc, wx);
        T acc = (T)0;
#pragma unroll
        for (int cz = 0; cz < 3; ++cz)
#pragma unroll
          for (int by2 = 0; by2 < 3; ++by2)
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
              if (!CUBIC && (wx[ax] == (T)0 || wy[by2] == (T)0 || wz[cz] == (T)0)) continue;
              acc += (wx[ax] * wy[by2] * wz[cz]) * v[cz][by2][ax];
            }
        const size_t fi = bidx(Lm, 2 * I + xc, 2 * J + yc, 2 * K + zc);
        if (CUBIC) uf[fi] = acc;
        else uf[fi] += acc;
      }
    }
}

// ------------------------------------------------------------------ finest-level defect norm

// Partial sums of squared defects per workgroup (fixed grid, fixed tree); r32 = FP32 defect.
__global__ void __launch_bounds__(kBlkThreads) k_blk_defect_norm(const double* __restrict__ u,
                                                                 const double* __restrict__ f, float* __restrict__ r32,
                                                                 int Lm, int Lb, double ih2, LevelBC bc, int per,
                                                                 double* __restrict__ part) {
  __shared__ double red[kBlkThreads / 64];
  const int n = 1 << (Lm + Lb), mm = (1 << Lm) - 1;
  const size_t n3 = (size_t)1 << (3 * (Lm + Lb));
  double acc = 0.0;
  for (size_t c = (size_t)blockIdx.x * kBlkThreads + threadIdx.x; c < n3; c += (size_t)gridDim.x * kBlkThreads) {
    int bx, by, bz;
    demorton3((unsigned)(c >> (3 * Lm)), bx, by, bz);
    const int r = (int)(c & (size_t)((1 << (3 * Lm)) - 1));
    const int i = (bx << Lm) + (r & mm), j = (by << Lm) + ((r >> Lm) & mm), k = (bz << Lm) + (r >> (2 * Lm));
    const double ucv = u[c];
    const double nb = blk_nsum(u, Lm, n, i, j, k, ucv, bc, per);
    const double d = f[c] - (nb - 6.0 * ucv) * ih2;
    acc += d * d;
    if (r32) r32[c] = (float)d;
  }
  acc = wave_sum(acc);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < kBlkThreads / 64; ++q) t += red[q];
    part[blockIdx.x] = t;
  }
}

unsigned grid_of(size_t work) {
  const size_t g = (work + kBlkThreads - 1) / kBlkThreads;
  return (unsigned)(g == 0 ? 1 : g);
}

template <typename T, int LM, int S>
void sweep_lms(const T* uin, T* uout, const T* f, int Lb, int G, int threads, double h, double omega,
               const LevelBC& bc, int per, hipStream_t s) {
  constexpr int tw = (1 << LM) + 4 * S;
  const size_t lds = (size_t)G * tw * tw * tw * sizeof(T);
  const unsigned nwg = (unsigned)((1u << (3 * Lb)) / (unsigned)G);
  hipLaunchKernelGGL((k_blk_sweep<T, LM, S>), dim3(nwg), dim3(threads), lds, s, uin, uout, f, Lb, G, (T)(h * h),
                     (T)omega, bc, per);
}

template <typename T, int LM>
void sweep_lm(const T* uin, T* uout, const T* f, int Lb, const BlkTune& t, double h, double omega, const LevelBC& bc,
              int per, hipStream_t s) {
  if (t.S == 2) sweep_lms<T, LM, 2>(uin, uout, f, Lb, t.G, t.threads, h, omega, bc, per, s);
  else sweep_lms<T, LM, 1>(uin, uout, f, Lb, t.G, t.threads, h, omega, bc, per, s);
}

template <typename T, int LM>
void set_lds(int bytes) {
  (void)hipFuncSetAttribute((const void*)k_blk_sweep<T, LM, 1>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  (void)hipFuncSetAttribute((const void*)k_blk_sweep<T, LM, 2>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

}  // namespace

int blk_periodic_mask(const LevelBC& bc) {
  return (bc.kind[0] == BC_PERIODIC ? 1 : 0) | (bc.kind[2] == BC_PERIODIC ? 2 : 0) | (bc.kind[4] == BC_PERIODIC ? 4 : 0);
}

size_t blk_sweep_lds(int Lm, int S, int G, size_t elem) {
  const size_t tw = (size_t)(1 << Lm) + 4 * (size_t)S;
  return (size_t)G * tw * tw * tw * elem;
}

BlkTune blk_default_tune(int Lm, int Lb, size_t elem) {
  // one sweep per launch, about 8000 staged cells per workgroup
  const int tw = (1 << Lm) + 4;
  int G = 1;
  while (G * 2 * tw * tw * tw <= 8000 && G * 2 <= (1 << (3 * Lb))) G *= 2;
  (void)elem;
  return BlkTune{Lm <= 1 ? 256 : 512, G, 1};
}

bool blk_tune_valid(const BlkTune& t, int Lm, int Lb, size_t elem, size_t lds_max) {
  if (Lm < 1 || Lm > kBlkMaxLm) return false;
  if (t.threads != 256 && t.threads != 512 && t.threads != 1024) return false;
  if (t.S != 1 && t.S != 2) return false;
  if (t.G < 1 || (t.G & (t.G - 1)) != 0 || t.G > (1 << (3 * Lb))) return false;
  return blk_sweep_lds(Lm, t.S, t.G, elem) <= lds_max;
}

template <typename T>
void blk_prepare(size_t lds_max) {
  const int bytes = (int)lds_max;
  set_lds<T, 1>(bytes);
  set_lds<T, 2>(bytes);
  set_lds<T, 3>(bytes);
  set_lds<T, 4>(bytes);
}

template <typename T>
void blk_sweep(const T* uin, T* uout, const T* f, int Lm, int Lb, const BlkTune& t, double h, double omega,
               const LevelBC& bc, hipStream_t s) {
  const int per = blk_periodic_mask(bc);
  switch (Lm) {
    case 1: sweep_lm<T, 1>(uin, uout, f, Lb, t, h, omega, bc, per, s); break;
    case 2: sweep_lm<T, 2>(uin, uout, f, Lb, t, h, omega, bc, per, s); break;
    case 3: sweep_lm<T, 3>(uin, uout, f, Lb, t, h, omega, bc, per, s); break;
    default: sweep_lm<T, 4>(uin, uout, f, Lb, t, h, omega, bc, per, s); break;
  }
}

template <typename T>
void blk_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int Lm, int Lb, double h, const LevelBC& bc,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_blk_defect_restrict<T>, dim3(grid_of((size_t)1 << (3 * (Lm - 1 + Lb)))), dim3(kBlkThreads), 0,
                     s, u, f, fc, uc0, Lm, Lb, (T)(1.0 / (h * h)), bc, blk_periodic_mask(bc));
}

template <typename Tin, typename Tout>
void blk_restrict(const Tin* uf, Tout* uc, int Lm, int Lb, hipStream_t s) {
  hipLaunchKernelGGL((k_blk_restrict<Tin, Tout>), dim3(grid_of((size_t)1 << (3 * (Lm - 1 + Lb)))), dim3(kBlkThreads),
                     0, s, uf, uc, Lm, Lb);
}

template <typename T>
void blk_prolong(const T* uc, T* uf, int Lm, int Lb, const LevelBC& bcc, int cubic, hipStream_t s) {
  const dim3 g(grid_of((size_t)1 << (3 * (Lm - 1 + Lb))));
  if (cubic) hipLaunchKernelGGL((k_blk_prolong<T, 1>), g, dim3(kBlkThreads), 0, s, uc, uf, Lm, Lb, bcc);
  else hipLaunchKernelGGL((k_blk_prolong<T, 0>), g, dim3(kBlkThreads), 0, s, uc, uf, Lm, Lb, bcc);
}

int blk_defect_norm(const double* u, const double* f, float* r32, int Lm, int Lb, double h, const LevelBC& bc,
                    double* part, hipStream_t s) {
  const size_t n3 = (size_t)1 << (3 * (Lm + Lb));
  size_t g = (n3 + (size_t)kBlkThreads * 8 - 1) / ((size_t)kBlkThreads * 8);
  if (g > (size_t)kMaxPartials) g = kMaxPartials;
  if (g == 0) g = 1;
  hipLaunchKernelGGL(k_blk_defect_norm, dim3((unsigned)g), dim3(kBlkThreads), 0, s, u, f, r32, Lm, Lb,
                     1.0 / (h * h), bc, blk_periodic_mask(bc), part);
  return (int)g;
}

template void blk_prepare<float>(size_t);
template void blk_prepare<double>(size_t);
template void blk_sweep<float>(const float*, float*, const float*, int, int, const BlkTune&, double, double,
                               const LevelBC&, hipStream_t);
template void blk_sweep<double>(const double*, double*, const double*, int, int, const BlkTune&, double, double,
                                const LevelBC&, hipStream_t);
template void blk_defect_restrict<float>(const float*, const float*, float*, float*, int, int, double, const LevelBC&,
                                         hipStream_t);
template void blk_defect_restrict<double>(const double*, const double*, double*, double*, int, int, double,
                                          const LevelBC&, hipStream_t);
template void blk_restrict<double, double>(const double*, double*, int, int, hipStream_t);
template void blk_restrict<float, float>(const float*, float*, int, int, hipStream_t);
template void blk_prolong<float>(const float*, float*, int, int, const LevelBC&, int, hipStream_t);
template void blk_prolong<double>(const double*, double*, int, int, const LevelBC&, int, hipStream_t);

}  // namespace mg
