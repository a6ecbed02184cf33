// mg_tile.hip -- V-cycle legs of the small levels (32^3 .. 128^3, and the MeshBlock levels
// below 256^3) as one launch each.
//
// On these levels a V-cycle leg is a handful of microseconds of work spread over many
// dependent launches (per colour, per operator), so the launch latency dominates.  Here one
// launch does a whole leg:
//   down (Alg. 1 steps 1-3): two red-black SOR sweeps (eqs. rbsor1-2), the defect of the
//        result (eq. defect) restricted to the coarse level (eq. restriction), the coarse
//        correction cleared;
//   up   (Alg. 1 steps 5-7): u += trilinear prolongation of the coarse correction (eq.
//        trilinear), two sweeps, optionally the sum of squared defects of the result
//        (Sec. 2.3.7).
// Each workgroup owns a region (16 x 16 x 8 cells on 128^3, smaller below) and stages it in
// LDS with a halo of 5 cells (four colour passes of radius 1 and the defect); colour pass s
// updates the region plus a ring of 4 - s cells, so every pass sees its neighbours exactly as
// a global sweep would, and only the region is written back.  The rings are recomputed by the neighbouring regions,
// never exchanged, so regions are independent.  The up leg first stages the coarse correction
// under the tile (homogeneous ghosts: periodic wrap, or the boundary cell with the face's
// sign) and adds its trilinear interpolant to every staged cell.  Boundary ghosts of the fine
// level are evaluated on the fly (Sec. 2.3.6).  The level may be dense or in the MeshBlock
// layout (the same code with the block-major index; the coarse side of the lowest block level
// is the dense root grid).
#include "mg_tile.h"

#include <cstring>
#include <type_traits>

#include "mg_launch.h"

namespace mg {

namespace {

constexpr int H = 5;   // staged halo: four colour passes of radius 1 and the defect

// Region shapes (cells per workgroup, all even): 16 x 16 x 8 on the 128^3 levels; smaller
// ones below, so that the few-microsecond legs of the 64^3 and 32^3 levels spread over more
// CUs with less serial work per workgroup (16 x 16 x 4: 256 regions at 64^3; 8 x 8 x 4: 128
// at 32^3).
struct Shape {
  int dx, dy, dz, threads;
};
constexpr Shape kShapes[3] = {{16, 16, 8, 1024}, {16, 16, 4, 1024}, {8, 8, 4, 1024}};
int shape_of(int n) { return n >= 128 ? 0 : n >= 64 ? 1 : 2; }

struct TileArgs {
  const void* uin;
  void* uout;
  const void* f;
  const void* ec;    // up: coarse correction
  void* fc;          // down: restricted defect
  void* uc0;         // down: coarse correction to clear (FAS: to start from phibar)
  void* pbar;        // FAS down: the restricted potential phibar
  double* part;      // up with norm: one partial sum per workgroup
  LevelBC bc;        // this level
  LevelBC bcc;       // up: coarse level (homogeneous)
  int n, L, Lm, per, nrx, nry;
  double h2, ih2, omega;
};

// Workgroups in contiguous runs per XCD (consecutive workgroups go round the 8 XCDs).
__device__ __forceinline__ unsigned xcd_order(unsigned bid, unsigned nwg) {
  if ((nwg & 7u) != 0) return bid;
  return (bid & 7u) * (nwg >> 3) + (bid >> 3);
}

template <typename T>
__device__ __forceinline__ T wall(const LevelBC& bc, int face, int n, int t1, int t2, T uc) {
  if (bc.kind[face] == BC_ZERO_GRADIENT) return uc;
  return (T)(2.0 * face_b(bc, face, n, t1, t2)) - uc;
}

// Storage index of cell (i, j, k) (in range) of this level (BLK: MeshBlock layout) and of the
// coarse level below.
template <bool BLK>
__device__ __forceinline__ size_t fine_at(const TileArgs& A, int i, int j, int k) {
  return BLK ? bidx(A.Lm, i, j, k) : cidx(A.L, i, j, k);
}
template <bool BLK>
__device__ __forceinline__ size_t coarse_idx(const TileArgs& A, int I, int J, int K) {
  return BLK && A.Lm > 1 ? bidx(A.Lm - 1, I, J, K) : cidx(A.L - 1, I, J, K);
}

// Coarse correction at (I, J, K) under homogeneous conditions: periodic indices wrap; on the
// other axes an index beyond the domain takes the boundary cell with the face's sign (+1 zero
// gradient, -1 zero-fixed), axis by axis (edges and corners: the product of the signs).
template <typename T, bool BLK>
__device__ __forceinline__ T coarse_hom(const TileArgs& A, const T* __restrict__ ec, int I, int J, int K) {
  const int nc = A.n >> 1, ncm = nc - 1;
  T s = (T)1;
  auto axis = [&](int v, int pbit, int lo_face) __attribute__((always_inline)) {
    if (A.per & pbit) return v & ncm;
    if (v < 0) {
      if (A.bcc.kind[lo_face] != BC_ZERO_GRADIENT) s = -s;
      return 0;
    }
    if (v > ncm) {
      if (A.bcc.kind[lo_face + 1] != BC_ZERO_GRADIENT) s = -s;
      return ncm;
    }
    return v;
  };
  const int Ic = axis(I, 1, 0), Jc = axis(J, 2, 2), Kc = axis(K, 4, 4);
  return s * ec[coarse_idx<BLK>(A, Ic, Jc, Kc)];
}

// One axis' share of coarse_hom, for the coordinate that is not 0 (the others must be 0, which
// every layout maps to index part 0 with sign +1): the part of the storage index, with bit 31
// set when the ghost rule negates the value.
template <bool BLK>
__device__ __forceinline__ unsigned coarse_part(const TileArgs& A, int I, int J, int K) {
  const int ncm = (A.n >> 1) - 1;
  bool neg = false;
  auto axis = [&](int v, int pbit, int lo_face) __attribute__((always_inline)) {
    if (A.per & pbit) return v & ncm;
    if (v < 0) {
      neg ^= A.bcc.kind[lo_face] != BC_ZERO_GRADIENT;
      return 0;
    }
    if (v > ncm) {
      neg ^= A.bcc.kind[lo_face + 1] != BC_ZERO_GRADIENT;
      return ncm;
    }
    return v;
  };
  const int Ic = axis(I, 1, 0), Jc = axis(J, 2, 2), Kc = axis(K, 4, 4);
  return (unsigned)coarse_idx<BLK>(A, Ic, Jc, Kc) | (neg ? 0x80000000u : 0u);
}

// FAS (down, dense; Alg. 3 steps 2-4): the restriction also writes phibar, the mean of the 8
// children of the swept u, into A.pbar and starts the coarse level from it (uc0 = phibar).
template <typename T, bool UP, bool NORM, bool BLK, bool FAS, int SH>
__global__ void __launch_bounds__(kShapes[SH].threads) k_tile_leg(TileArgs A) {
  constexpr int kThreads = kShapes[SH].threads;
  constexpr int DX = kShapes[SH].dx, DY = kShapes[SH].dy, DZ = kShapes[SH].dz;
  constexpr int WX = DX + 2 * H, WY = DY + 2 * H, WZ = DZ + 2 * H;   // staged tile
  constexpr int TV = WX * WY * WZ;
  // coarse cells under the tile: floor(x/2) - 1 .. floor(x/2) + 1 for every staged x
  constexpr int CX = DX / 2 + 8, CY = DY / 2 + 8, CZ = DZ / 2 + 8;
  constexpr int CV = CX * CY * CZ;
  __shared__ T tile[TV];
  __shared__ T ctile[UP ? CV : 1];
  __shared__ double red[kThreads / 64];
  const int tid = threadIdx.x;
  const int n = A.n, nm = n - 1, per = A.per;
  const T h2 = (T)A.h2, ih2 = (T)A.ih2, omega = (T)A.omega, inv6 = (T)(1.0 / 6.0);
  const T* __restrict__ uin = reinterpret_cast<const T*>(A.uin);
  T* __restrict__ uout = reinterpret_cast<T*>(A.uout);
  const T* __restrict__ fin = reinterpret_cast<const T*>(A.f);
  const int rid = (int)xcd_order(blockIdx.x, gridDim.x);
  const int rx = rid % A.nrx, ry = (rid / A.nrx) % A.nry, rz = rid / (A.nrx * A.nry);
  const int ox = rx * DX, oy = ry * DY, oz = rz * DZ;   // region origin (even)

  // wrapped coordinate on a periodic axis; -1 outside a non-periodic domain
  auto wrap = [&](int v, int pbit) __attribute__((always_inline)) {
    if (per & pbit) return v & nm;
    return (unsigned)v < (unsigned)n ? v : -1;
  };

  // MeshBlock layout: a storage index is the sum of an x part and a y-z part (disjoint bits of
  // the block-major index), tabulated once for the staged extent, so each access costs two LDS
  // reads instead of three bit spreads.  Entries of cells outside a non-periodic domain are
  // never used.  Up: the same for the coarse cells under the tile, with the homogeneous ghost
  // sign in bit 31 (the coarse level has at most 2^21 cells).
  __shared__ unsigned ix_part[BLK ? WX : 1], iyz_part[BLK ? WY * WZ : 1];
  __shared__ unsigned cx_part[BLK && UP ? CX : 1], cyz_part[BLK && UP ? CY * CZ : 1];
  const int cx0 = (ox >> 1) - 4, cy0 = (oy >> 1) - 4, cz0 = (oz >> 1) - 4;
  if constexpr (BLK) {
    constexpr int NF = WX + WY * WZ, NC = UP ? CX + CY * CZ : 0;
    for (int q = tid; q < NF + NC; q += kThreads) {
      if (q < WX) {
        const int i = wrap(ox + q - H, 1);
        ix_part[q] = i < 0 ? 0u : (unsigned)fine_at<BLK>(A, i, 0, 0);
      } else if (q < NF) {
        const int r = q - WX, j = wrap(oy + r % WY - H, 2), k = wrap(oz + r / WY - H, 4);
        iyz_part[r] = (j < 0 || k < 0) ? 0u : (unsigned)fine_at<BLK>(A, 0, j, k);
      } else if constexpr (UP) {
        const int r = q - NF;
        if (r < CX) {
          cx_part[r] = coarse_part<BLK>(A, cx0 + r, 0, 0);
        } else {
          const int t = r - CX;
          cyz_part[t] = coarse_part<BLK>(A, 0, cy0 + t % CY, cz0 + t / CY);
        }
      }
    }
    __syncthreads();
  }
  // storage index of the staged cell (tx, ty, tz) (tile coordinates), in the domain at (i, j, k)
  auto fat = [&](int tx, int ty, int tz, int i, int j, int k) __attribute__((always_inline)) -> size_t {
    if constexpr (BLK) return (size_t)(ix_part[tx] + iyz_part[tz * WY + ty]);
    else return cidx(A.L, i, j, k);
  };

  // ---- stage u on the region and its halo
  for (int q = tid; q < TV; q += kThreads) {
    const int tx = q % WX, ty = (q / WX) % WY, tz = q / (WX * WY);
    const int i = wrap(ox + tx - H, 1), j = wrap(oy + ty - H, 2), k = wrap(oz + tz - H, 4);
    tile[q] = (i >= 0 && j >= 0 && k >= 0) ? uin[fat(tx, ty, tz, i, j, k)] : (T)0;
  }
  if constexpr (UP) {
    const T* __restrict__ ec = reinterpret_cast<const T*>(A.ec);
    for (int q = tid; q < CV; q += kThreads) {
      const int cx = q % CX, cy = (q / CX) % CY, cz = q / (CX * CY);
      if constexpr (BLK) {
        const unsigned a = cx_part[cx], b = cyz_part[cz * CY + cy];
        const T v = ec[(a & 0x7fffffffu) + (b & 0x7fffffffu)];
        ctile[q] = ((a ^ b) >> 31) ? -v : v;
      } else {
        ctile[q] = coarse_hom<T, BLK>(A, ec, cx0 + cx, cy0 + cy, cz0 + cz);
      }
    }
    __syncthreads();
    // trilinear prolongation (weights 1/4, 3/4 per axis; the even child is the lower one)
    for (int q = tid; q < TV; q += kThreads) {
      const int tx = q % WX, ty = (q / WX) % WY, tz = q / (WX * WY);
      const int x = ox + tx - H, y = oy + ty - H, z = oz + tz - H;
      if (wrap(x, 1) < 0 || wrap(y, 2) < 0 || wrap(z, 4) < 0) continue;
      // lower tap and weight per axis: even child X-1 (1/4), X (3/4); odd child X (3/4), X+1 (1/4)
      const int ax = (x >> 1) - (x & 1 ? 0 : 1) - cx0, ay = (y >> 1) - (y & 1 ? 0 : 1) - cy0;
      const int az = (z >> 1) - (z & 1 ? 0 : 1) - cz0;
      const T wx0 = (x & 1) ? (T)0.75 : (T)0.25, wy0 = (y & 1) ? (T)0.75 : (T)0.25, wz0 = (z & 1) ? (T)0.75 : (T)0.25;
      const T wx[2] = {wx0, (T)1 - wx0}, wy[2] = {wy0, (T)1 - wy0}, wz[2] = {wz0, (T)1 - wz0};
      T acc = (T)0;
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a)
            acc += (wx[a] * wy[b] * wz[c]) * ctile[((az + c) * CY + (ay + b)) * CX + (ax + a)];
      tile[q] += acc;
    }
  }
  __syncthreads();

  // ---- four colour passes (red, black, red, black) on the region plus a shrinking ring (each
  // pass's extents are compile-time, so the index arithmetic divides by constants)
  auto pass_of = [&](auto cpass) __attribute__((always_inline)) {
    constexpr int pass = decltype(cpass)::value;
    constexpr int colour = pass & 1, ring = 4 - pass;
    constexpr int sx = DX + 2 * ring, sy = DY + 2 * ring, sz = DZ + 2 * ring, hx = sx >> 1;
    constexpr int cnt = hx * sy * sz;
    for (int q = tid; q < cnt; q += kThreads) {
      const int row = q / hx, xi = q - row * hx;
      const int ry2 = row % sy, rz2 = row / sy;
      const int j0 = oy - ring + ry2, k0 = oz - ring + rz2, ib = ox - ring;
      const int rx2 = 2 * xi + ((colour - ib - j0 - k0) & 1);   // the cell of this colour
      const int i = wrap(ib + rx2, 1), j = wrap(j0, 2), k = wrap(k0, 4);
      if (i < 0 || j < 0 || k < 0) continue;
      const int p = ((rz2 + H - ring) * WY + (ry2 + H - ring)) * WX + (rx2 + H - ring);
      const T uc = tile[p];
      const T xm = (!(per & 1) && i == 0) ? wall(A.bc, 0, n, j, k, uc) : tile[p - 1];
      const T xp = (!(per & 1) && i == nm) ? wall(A.bc, 1, n, j, k, uc) : tile[p + 1];
      const T ym = (!(per & 2) && j == 0) ? wall(A.bc, 2, n, i, k, uc) : tile[p - WX];
      const T yp = (!(per & 2) && j == nm) ? wall(A.bc, 3, n, i, k, uc) : tile[p + WX];
      const T zm = (!(per & 4) && k == 0) ? wall(A.bc, 4, n, i, j, uc) : tile[p - WX * WY];
      const T zp = (!(per & 4) && k == nm) ? wall(A.bc, 5, n, i, j, uc) : tile[p + WX * WY];
      const T nb = ((((xm + xp) + ym) + yp) + zm) + zp;
      tile[p] = uc + omega * ((nb - h2 * fin[fat(rx2 + H - ring, ry2 + H - ring, rz2 + H - ring, i, j, k)]) * inv6 - uc);
    }
    __syncthreads();
  };
  pass_of(std::integral_constant<int, 0>{});
  pass_of(std::integral_constant<int, 1>{});
  pass_of(std::integral_constant<int, 2>{});
  pass_of(std::integral_constant<int, 3>{});

  // defect of region cell (x, y, z) (region-local), from the final tile
  auto defect_at = [&](int x, int y, int z) __attribute__((always_inline)) {
    const int i = ox + x, j = oy + y, k = oz + z;   // in the domain: regions tile it
    const int p = ((z + H) * WY + (y + H)) * WX + (x + H);
    const T uc = tile[p];
    const T xm = (!(per & 1) && i == 0) ? wall(A.bc, 0, n, j, k, uc) : tile[p - 1];
    const T xp = (!(per & 1) && i == nm) ? wall(A.bc, 1, n, j, k, uc) : tile[p + 1];
    const T ym = (!(per & 2) && j == 0) ? wall(A.bc, 2, n, i, k, uc) : tile[p - WX];
    const T yp = (!(per & 2) && j == nm) ? wall(A.bc, 3, n, i, k, uc) : tile[p + WX];
    const T zm = (!(per & 4) && k == 0) ? wall(A.bc, 4, n, i, j, uc) : tile[p - WX * WY];
    const T zp = (!(per & 4) && k == nm) ? wall(A.bc, 5, n, i, j, uc) : tile[p + WX * WY];
    const T nb = ((((xm + xp) + ym) + yp) + zm) + zp;
    return fin[fat(x + H, y + H, z + H, i, j, k)] - (nb - (T)6 * uc) * ih2;
  };

  if constexpr (!UP) {
    // ---- restricted defect (mean over the 8 children) and the cleared coarse correction
    T* __restrict__ fc = reinterpret_cast<T*>(A.fc);
    T* __restrict__ uc0 = reinterpret_cast<T*>(A.uc0);
    for (int q = tid; q < (DX / 2) * (DY / 2) * (DZ / 2); q += kThreads) {
      const int cx = q % (DX / 2), cy = (q / (DX / 2)) % (DY / 2), cz = q / ((DX / 2) * (DY / 2));
      T s = (T)0;
#pragma unroll 1
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int a = 0; a < 2; ++a) s += defect_at(2 * cx + a, 2 * cy + b, 2 * cz + c);
      const size_t ci = coarse_idx<BLK>(A, (ox >> 1) + cx, (oy >> 1) + cy, (oz >> 1) + cz);
      fc[ci] = s * (T)0.125;
      if constexpr (FAS) {
        T su = (T)0;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) su += tile[((2 * cz + c + H) * WY + (2 * cy + b + H)) * WX + (2 * cx + a + H)];
        const T pb = su * (T)0.125;
        reinterpret_cast<T*>(A.pbar)[ci] = pb;
        uc0[ci] = pb;
      } else {
        uc0[ci] = (T)0;
      }
    }
  }
  double acc = 0.0;
  // ---- the region back to memory (and, for the norm, its defects)
  for (int q = tid; q < DX * DY * DZ; q += kThreads) {
    const int x = q % DX, y = (q / DX) % DY, z = q / (DX * DY);
    uout[fat(x + H, y + H, z + H, ox + x, oy + y, oz + z)] = tile[((z + H) * WY + (y + H)) * WX + (x + H)];
    if constexpr (UP && NORM) {
      const T d = defect_at(x, y, z);
      acc += (double)d * (double)d;
    }
  }
  if constexpr (UP && NORM) {
    acc = wave_sum(acc);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int q = 0; q < kThreads / 64; ++q) t += red[q];
      A.part[blockIdx.x] = t;
    }
  }
}

template <typename T>
TileArgs base_args(const T* uin, T* uout, const T* f, int n, int Lm, double h, double omega, const LevelBC& bc) {
  TileArgs A;
  std::memset(&A, 0, sizeof(A));
  A.uin = uin;
  A.uout = uout;
  A.f = f;
  A.bc = bc;
  A.n = n;
  A.L = ilog2(n);
  A.Lm = Lm;
  A.per = (bc.kind[0] == BC_PERIODIC ? 1 : 0) | (bc.kind[2] == BC_PERIODIC ? 2 : 0) | (bc.kind[4] == BC_PERIODIC ? 4 : 0);
  const Shape sh = kShapes[shape_of(n)];
  A.nrx = n / sh.dx;
  A.nry = n / sh.dy;
  A.h2 = h * h;
  A.ih2 = 1.0 / (h * h);
  A.omega = omega;
  return A;
}

int regions(int n) {
  const Shape sh = kShapes[shape_of(n)];
  return (n / sh.dx) * (n / sh.dy) * (n / sh.dz);
}

// One launch of the leg in the region shape of level side n.
template <typename T, bool UP, bool NORM, bool BLK, bool FAS = false>
void launch_leg(const TileArgs& A, hipStream_t s) {
  const dim3 g(regions(A.n)), b(kShapes[shape_of(A.n)].threads);
  switch (shape_of(A.n)) {
    case 0: launch_maybe_timed(k_tile_leg<T, UP, NORM, BLK, FAS, 0>, g, b, 0, s, A); break;
    case 1: launch_maybe_timed(k_tile_leg<T, UP, NORM, BLK, FAS, 1>, g, b, 0, s, A); break;
    default: launch_maybe_timed(k_tile_leg<T, UP, NORM, BLK, FAS, 2>, g, b, 0, s, A); break;
  }
}

}  // namespace

template <typename T>
void tile_down(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, int Lm, int Lb, double h, double omega,
               const LevelBC& bc, hipStream_t s) {
  (void)Lb;
  TileArgs A = base_args(uin, uout, f, n, Lm, h, omega, bc);
  A.fc = fc;
  A.uc0 = uc0;
  if (Lm > 0) launch_leg<T, false, false, true>(A, s);
  else launch_leg<T, false, false, false>(A, s);
}

template <typename T>
void tile_down_fas(const T* uin, T* uout, const T* f, T* fc, T* pbar, T* uc0, int n, double h, double omega,
                   const LevelBC& bc, hipStream_t s) {
  TileArgs A = base_args(uin, uout, f, n, 0, h, omega, bc);
  A.fc = fc;
  A.pbar = pbar;
  A.uc0 = uc0;
  launch_leg<T, false, false, false, true>(A, s);
}

template <typename T>
int tile_up(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, double* part, int n, int Lm, int Lb,
            double h, double omega, const LevelBC& bc, hipStream_t s) {
  (void)Lb;
  TileArgs A = base_args(uin, uout, f, n, Lm, h, omega, bc);
  A.ec = ec;
  A.bcc = bcc;
  A.part = part;
  if (part) {
    if (Lm > 0) launch_leg<T, true, true, true>(A, s);
    else launch_leg<T, true, true, false>(A, s);
    return regions(n);
  }
  if (Lm > 0) launch_leg<T, true, false, true>(A, s);
  else launch_leg<T, true, false, false>(A, s);
  return 0;
}

template <typename T>
std::string tile_name(bool up, bool norm, bool blk) {
  auto b = [](bool v) { return std::string(v ? "true" : "false"); };
  return std::string("k_tile_leg<") + (sizeof(T) == 8 ? "double" : "float") + ", " + b(up) + ", " + b(up && norm) + ", " +
         b(blk) + ">";
}

template void tile_down<double>(const double*, double*, const double*, double*, double*, int, int, int, double, double,
                                const LevelBC&, hipStream_t);
template void tile_down<float>(const float*, float*, const float*, float*, float*, int, int, int, double, double,
                               const LevelBC&, hipStream_t);
template void tile_down_fas<double>(const double*, double*, const double*, double*, double*, double*, int, double,
                                    double, const LevelBC&, hipStream_t);
template int tile_up<double>(const double*, double*, const double*, const double*, const LevelBC&, double*, int, int,
                             int, double, double, const LevelBC&, hipStream_t);
template int tile_up<float>(const float*, float*, const float*, const float*, const LevelBC&, double*, int, int, int,
                            double, double, const LevelBC&, hipStream_t);
template std::string tile_name<double>(bool, bool, bool);
template std::string tile_name<float>(bool, bool, bool);

}  // namespace mg
