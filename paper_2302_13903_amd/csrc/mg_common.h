// mg_common.h -- device-side definitions shared by the HIP kernels of the multigrid solver.
//
// Grid arrays are dense n^3, x fastest: (i, j, k) -> (k*n + j)*n + i.  n is a power of two,
// so index arithmetic uses shifts by L = log2(n).  Ghost cells are never stored: a kernel that
// reads a neighbour outside [0, n) evaluates the boundary rule of Sec. 2.3.6 on the fly, from
// the value the boundary cell holds at the start of the operator (which is exactly the value
// a ghost layer filled before the operator would hold).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mg {

enum : int { BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_FIXED = 2, BC_MULTIPOLE = 3 };

// Boundary description of one level, passed by value to kernels.  Faces -x,+x,-y,+y,-z,+z.
// b[face] is an extended face array of (n+2)^2 values indexed [t2+1][t1+1], t in [-1, n],
// (t1, t2) the two transverse axes in increasing order; nullptr means b = 0.
struct LevelBC {
  int kind[6];
  const double* b[6];
};

__host__ __device__ inline bool bc_has_value(int kind) { return kind >= BC_FIXED; }

__device__ __forceinline__ double face_b(const LevelBC& bc, int face, int n, int t1, int t2) {
  const double* b = bc.b[face];
  return b ? b[(size_t)(t2 + 1) * (size_t)(n + 2) + (size_t)(t1 + 1)] : 0.0;
}

__device__ __forceinline__ size_t cidx(int L, int i, int j, int k) {
  return ((size_t)k << (2 * L)) | ((size_t)j << L) | (size_t)i;
}

// ---- MeshBlock layout: blocks of 2^Lm cells per side, stored one after another in Morton
// (Z-curve) order of their block coordinates (x bit lowest), each block dense, x fastest.
__device__ __forceinline__ unsigned spread3(unsigned v) {
  v &= 0x3ffu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}
__device__ __forceinline__ unsigned compact3(unsigned v) {
  v &= 0x09249249u;
  v = (v | (v >> 2)) & 0x030C30C3u;
  v = (v | (v >> 4)) & 0x0300F00Fu;
  v = (v | (v >> 8)) & 0x030000FFu;
  v = (v | (v >> 16)) & 0x3ffu;
  return v;
}
__device__ __forceinline__ unsigned morton3(int bx, int by, int bz) {
  return spread3((unsigned)bx) | (spread3((unsigned)by) << 1) | (spread3((unsigned)bz) << 2);
}
__device__ __forceinline__ void demorton3(unsigned b, int& bx, int& by, int& bz) {
  bx = (int)compact3(b);
  by = (int)compact3(b >> 1);
  bz = (int)compact3(b >> 2);
}

// Storage index of global cell (i, j, k), all in [0, 2^(Lm+Lb)), of a MeshBlock-layout level.
__device__ __forceinline__ size_t bidx(int Lm, int i, int j, int k) {
  const int mm = (1 << Lm) - 1;
  return ((size_t)morton3(i >> Lm, j >> Lm, k >> Lm) << (3 * Lm)) |
         (size_t)(((k & mm) << (2 * Lm)) | ((j & mm) << Lm) | (i & mm));
}

// Storage index of cell (i, j, k) of a level of 2^L cells per side: dense when Lm = 0 (the
// dense layout, or a root grid), MeshBlock layout with 2^Lm-cell blocks otherwise.
__device__ __forceinline__ size_t lidx(int L, int Lm, int i, int j, int k) {
  return Lm == 0 ? cidx(L, i, j, k) : bidx(Lm, i, j, k);
}

// Value of a face-adjacent ghost for the 7-point stencil: `uc` is the boundary cell's own
// value, `opp` points at the opposite active cell (read only for periodic faces).
template <typename T>
__device__ __forceinline__ T ghost7(const LevelBC& bc, int face, int n, int t1, int t2, T uc,
                                    const T* __restrict__ opp) {
  const int kd = bc.kind[face];
  if (kd == BC_PERIODIC) return *opp;
  if (kd == BC_ZERO_GRADIENT) return uc;
  return (T)(2.0 * face_b(bc, face, n, t1, t2)) - uc;
}

// Sum of the six face neighbours of active cell (i, j, k) whose value is uc.
template <typename T>
__device__ __forceinline__ T neighbour_sum(const T* __restrict__ u, int n, int L, int i, int j, int k,
                                           size_t c, T uc, const LevelBC& bc) {
  const size_t sy = (size_t)1 << L, sz = (size_t)1 << (2 * L);
  T xm = i > 0 ? u[c - 1] : ghost7(bc, 0, n, j, k, uc, u + c + (n - 1));
  T xp = i < n - 1 ? u[c + 1] : ghost7(bc, 1, n, j, k, uc, u + c - (n - 1));
  T ym = j > 0 ? u[c - sy] : ghost7(bc, 2, n, i, k, uc, u + c + (size_t)(n - 1) * sy);
  T yp = j < n - 1 ? u[c + sy] : ghost7(bc, 3, n, i, k, uc, u + c - (size_t)(n - 1) * sy);
  T zm = k > 0 ? u[c - sz] : ghost7(bc, 4, n, i, j, uc, u + c + (size_t)(n - 1) * sz);
  T zp = k < n - 1 ? u[c + sz] : ghost7(bc, 5, n, i, j, uc, u + c - (size_t)(n - 1) * sz);
  return ((((xm + xp) + ym) + yp) + zm) + zp;
}

// Value at (i, j, k) with each index in [-1, n], edges and corners included, under the rule
// that ghosts are filled axis by axis (x, then y over the x ghosts, then z over both).  The
// last-filled axis is resolved first; each step maps value = s * inner + t.  Faces are picked
// with compile-time indices only (so a boundary description held in registers stays there).
// Lm > 0: u is a MeshBlock-layout level with 2^Lm-cell blocks.
template <typename T>
__device__ __forceinline__ void ghost_axis(const LevelBC& bc, int lo_face, int n, int& c, int t1, int t2, T& s,
                                           T& t) {
  if (c >= 0 && c < n) return;
  const bool lo = c < 0;
  const int kd = lo ? bc.kind[lo_face] : bc.kind[lo_face + 1];
  if (kd == BC_PERIODIC) {
    c = lo ? n - 1 : 0;
    return;
  }
  if (kd != BC_ZERO_GRADIENT) {
    const double* b = lo ? bc.b[lo_face] : bc.b[lo_face + 1];
    const double bv = b ? b[(size_t)(t2 + 1) * (size_t)(n + 2) + (size_t)(t1 + 1)] : 0.0;
    t += s * (T)(2.0 * bv);
    s = -s;
  }
  c = lo ? 0 : n - 1;
}

template <typename T>
__device__ __forceinline__ T ghost_any(const T* __restrict__ u, int n, int L, int i, int j, int k,
                                       const LevelBC& bc, int Lm = 0) {
  T s = (T)1, t = (T)0;
  ghost_axis<T>(bc, 4, n, k, i, j, s, t);
  ghost_axis<T>(bc, 2, n, j, i, k, s, t);
  ghost_axis<T>(bc, 0, n, i, j, k, s, t);
  return s * u[lidx(L, Lm, i, j, k)] + t;
}

// 1-D prolongation weights for coarse offsets -1, 0, +1 (Sec. 2.3.1): `upper` selects the
// odd fine child.  Trilinear: (1/4, 3/4, 0) / (0, 3/4, 1/4).  Tricubic (FMG):
// (5, 30, -3)/32 / (-3, 30, 5)/32.
template <typename T>
__device__ __forceinline__ void lin_w(int upper, T w[3]) {
  w[0] = upper ? (T)0 : (T)0.25;
  w[1] = (T)0.75;
  w[2] = upper ? (T)0.25 : (T)0;
}
template <typename T>
__device__ __forceinline__ void cub_w(int upper, T w[3]) {
  w[0] = upper ? (T)(-3.0 / 32.0) : (T)(5.0 / 32.0);
  w[1] = (T)(30.0 / 32.0);
  w[2] = upper ? (T)(5.0 / 32.0) : (T)(-3.0 / 32.0);
}

// ---- wavefront / workgroup reductions (deterministic fixed-shape trees) ------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mg
