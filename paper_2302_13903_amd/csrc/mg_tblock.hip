// mg_tblock.hip -- temporally blocked smoothing: NS full RB-SOR sweeps (eqs. rbsor1-2) per
// pass over HBM, for the large levels.
//
// A workgroup owns a tile of TX x TY cells in x-y (an output box plus a halo of 2 NS cells)
// and marches in z through a chunk of planes.  The last 2 NS + 2 planes of u live in LDS
// (plane ring); f of the planes still in flight lives in registers (each thread always owns
// the same x-pairs of the tile).  At the step that loads plane P, colour stage s (red, black,
// red, black, ...) runs on plane P-1-s: every stage reads its z-neighbours in exactly the
// colour state a sequence of whole-grid half-sweeps would give, and stage s is computed on a
// box that shrinks by one cell per stage, so the last stage is exact on the output box.  Only
// that box is written, to a separate array (tiles overlap in their halos).  With PRO the
// trilinear prolongation of the coarse correction (eq. trilinear; Alg. 1 steps 5-6) is added
// to u as it is loaded.  Boundary ghosts (Sec. 2.3.6) are evaluated on the fly from the
// boundary cell's own value.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include "mg_launch.h"
#include "mg_tblock.h"

namespace mg {

namespace {

constexpr int kTbTX = 64;          // tile width in x (32 pairs)
constexpr int kTbPairsX = kTbTX / 2;

struct TbArgs {
  const void* uin;
  void* uout;
  const void* f;
  const void* ec;      // PRO: coarse correction (n/2)^3
  LevelBC bc;
  LevelBC bcc;         // PRO: coarse level description (homogeneous)
  int n, L, tiles_x, tiles_y, chunks_z, ntiles, zc;
  double h2, omega;
};

template <typename T>
struct alignas(2 * sizeof(T)) TbPair {
  T a, b;
};

template <typename T>
__device__ __forceinline__ T tb_ghost(const LevelBC& bc, int face, int n, int t1, int t2, T c) {
  if (bc.kind[face] == BC_ZERO_GRADIENT) return c;
  return (T)(2.0 * face_b(bc, face, n, t1, t2)) - c;
}

template <typename T>
__device__ __forceinline__ T tb_coarse(const T* __restrict__ e, int nc, int Lc, int X, int Y, int Z,
                                       const LevelBC& bcc) {
  if ((unsigned)X < (unsigned)nc && (unsigned)Y < (unsigned)nc && (unsigned)Z < (unsigned)nc)
    return e[cidx(Lc, X, Y, Z)];
  return ghost_any(e, nc, Lc, X, Y, Z, bcc);
}

template <typename T, int NS, bool PRO, int TY, int THREADS>
__global__ void __launch_bounds__(THREADS) k_tb(TbArgs A) {
  constexpr int TX = kTbTX, H = 2 * NS, RING = 2 * NS + 2, NST = 2 * NS;
  constexpr int PAIRS = kTbPairsX * TY;
  static_assert(PAIRS % THREADS == 0, "whole pairs per thread");
  constexpr int PPT = PAIRS / THREADS;   // x-pairs per thread
  constexpr int FR = NST + 2;            // f ring slots (>= NST + 1 planes in flight; even, so
                                         // that the two prefetch slots are compile-time too)
  constexpr int PD = 2;                  // planes prefetched ahead
  __shared__ TbPair<T> us[RING][TY][kTbPairsX];

  const int tid = threadIdx.x;
  const int nb = gridDim.x, bid = blockIdx.x;
  const int tile = (nb & 7) == 0 ? (bid & 7) * (nb >> 3) + (bid >> 3) : bid;
  if (tile >= A.ntiles) return;   // whole workgroup: no barrier is skipped by part of it

  const int n = A.n, L = A.L, nm = n - 1;
  const int OX = TX - 2 * H, OY = TY - 2 * H;
  const int tx = tile % A.tiles_x;
  const int ty = (tile / A.tiles_x) % A.tiles_y;
  const int cz = tile / (A.tiles_x * A.tiles_y);
  const T* __restrict__ uin = reinterpret_cast<const T*>(A.uin);
  T* __restrict__ uout = reinterpret_cast<T*>(A.uout);
  const T* __restrict__ fin = reinterpret_cast<const T*>(A.f);
  const bool px = A.bc.kind[0] == BC_PERIODIC, py = A.bc.kind[2] == BC_PERIODIC, pz = A.bc.kind[4] == BC_PERIODIC;
  const T h2 = (T)A.h2, omega = (T)A.omega, inv6 = (T)(1.0 / 6.0);
  const int gx0 = tx * OX - H, gy0 = ty * OY - H;
  const int z0 = cz * A.zc, zend = min(z0 + A.zc, n);
  const int zstart = z0 - NST;
  const int nsteps = (zend - z0) + 2 * NST;

  // this thread's pairs: local (lxp, ly), global even column gx and row gy
  int lxp[PPT], ly[PPT], gxa[PPT], gxw[PPT], gy[PPT], gyw[PPT];
  bool inxy[PPT], outxy[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    const int pi = tid + q * THREADS;
    lxp[q] = pi % kTbPairsX;
    ly[q] = pi / kTbPairsX;
    gxa[q] = gx0 + 2 * lxp[q];
    gy[q] = gy0 + ly[q];
    gxw[q] = gxa[q] & nm;
    gyw[q] = gy[q] & nm;
    const bool inx = px || (gxa[q] >= 0 && gxa[q] < n);
    const bool iny = py || (gy[q] >= 0 && gy[q] < n);
    inxy[q] = inx && iny;
    const int lx = 2 * lxp[q];
    outxy[q] = lx >= H && lx < TX - H && ly[q] >= H && ly[q] < TY - H && gxa[q] < n && gy[q] < n && gxa[q] >= 0 &&
               gy[q] >= 0;
  }

  T fr[FR][2][PPT];     // f ring (slot = plane mod FR, compile-time after unrolling) by colour
  TbPair<T> pu[PD][PPT];  // prefetched u of the next PD planes (slot = plane mod PD)
  T pf[PD][PPT][2];       // prefetched f of the next PD planes

  auto fetch = [&](int P, TbPair<T> (&pu)[PPT], T (&pf)[PPT][2]) __attribute__((always_inline)) {
    const bool inz = pz || (P >= 0 && P < n);
    const int Pg = P & nm;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      if (inxy[q] && inz) {
        const size_t off = ((size_t)Pg << (2 * L)) + ((size_t)gyw[q] << L) + (size_t)gxw[q];
        pu[q] = *reinterpret_cast<const TbPair<T>*>(uin + off);
        const TbPair<T> vf = *reinterpret_cast<const TbPair<T>*>(fin + off);
        // stored by colour, not by column: [0] = f of the pair's red cell, [1] = of its black
        // cell, so the stages index the f ring with compile-time indices only
        const bool red_odd = ((gxa[q] + gy[q] + P) & 1) != 0;
        pf[q][0] = red_odd ? vf.b : vf.a;
        pf[q][1] = red_odd ? vf.a : vf.b;
        if (PRO) {
          // trilinear weights 1/4, 3/4 per axis: the even child takes coarse index I-1, I, the
          // odd child I, I+1
          const T* __restrict__ ec = reinterpret_cast<const T*>(A.ec);
          const int nc = n >> 1, Lc = L - 1;
          const int xg = px ? gxw[q] : gxa[q], yg = py ? gyw[q] : gy[q], zg = pz ? Pg : P;
          const int X = xg >> 1, Y = yg >> 1, Z = zg >> 1;
          const int ylo = (yg & 1) ? Y : Y - 1, zlo = (zg & 1) ? Z : Z - 1;
          const T wy0 = (yg & 1) ? (T)0.75 : (T)0.25, wz0 = (zg & 1) ? (T)0.75 : (T)0.25;
          const T wy1 = (T)1 - wy0, wz1 = (T)1 - wz0;
          T col[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            // z first, then y, then (below) x
            const int Xd = X - 1 + d;
            const T r0 = wz0 * tb_coarse(ec, nc, Lc, Xd, ylo, zlo, A.bcc) +
                         wz1 * tb_coarse(ec, nc, Lc, Xd, ylo, zlo + 1, A.bcc);
            const T r1 = wz0 * tb_coarse(ec, nc, Lc, Xd, ylo + 1, zlo, A.bcc) +
                         wz1 * tb_coarse(ec, nc, Lc, Xd, ylo + 1, zlo + 1, A.bcc);
            col[d] = wy0 * r0 + wy1 * r1;
          }
          pu[q].a += (T)0.25 * col[0] + (T)0.75 * col[1];
          pu[q].b += (T)0.75 * col[1] + (T)0.25 * col[2];
        }
      } else {
        pu[q] = TbPair<T>{(T)0, (T)0};
        pf[q][0] = pf[q][1] = (T)0;
      }
    }
  };

  // one colour stage on plane p for the cells of this thread that lie in the stage's box;
  // fp[q] holds f of this colour's cell of pair q
  auto stage = [&](int p, int colour, int s, const T (&fp)[PPT]) __attribute__((always_inline)) {
    const bool inz = pz || (p >= 0 && p < n);
    const int sp = ((p % RING) + RING) % RING, sm = ((p - 1) % RING + RING) % RING, spp = ((p + 1) % RING + RING) % RING;
    const int pw = p & nm;
    const bool bz0 = !pz && p == 0, bz1 = !pz && p == nm;
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
      const int lyq = ly[q];
      // which cell of the pair has this colour (the pair starts on an even column)
      const int odd = (gxa[q] + gy[q] + p + colour) & 1;
      const int lx = 2 * lxp[q] + odd;
      const bool inbox = lx >= 1 + s && lx < TX - 1 - s && lyq >= 1 + s && lyq < TY - 1 - s;
      if (!(inbox && inxy[q] && inz)) continue;
      const T* row = reinterpret_cast<const T*>(&us[sp][lyq][0]);
      const T c = row[lx];
      T xm = row[lx - 1], xp = row[lx + 1];
      T ym = reinterpret_cast<const T*>(&us[sp][lyq - 1][0])[lx];
      T yp = reinterpret_cast<const T*>(&us[sp][lyq + 1][0])[lx];
      T zm = reinterpret_cast<const T*>(&us[sm][lyq][0])[lx];
      T zp = reinterpret_cast<const T*>(&us[spp][lyq][0])[lx];
      const int gxc = gxa[q] + odd;
      if (!px && gxc == 0) xm = tb_ghost(A.bc, 0, n, gyw[q], pw, c);
      if (!px && gxc == nm) xp = tb_ghost(A.bc, 1, n, gyw[q], pw, c);
      if (!py && gy[q] == 0) ym = tb_ghost(A.bc, 2, n, gxw[q] + odd, pw, c);
      if (!py && gy[q] == nm) yp = tb_ghost(A.bc, 3, n, gxw[q] + odd, pw, c);
      if (bz0) zm = tb_ghost(A.bc, 4, n, gxw[q] + odd, gyw[q], c);
      if (bz1) zp = tb_ghost(A.bc, 5, n, gxw[q] + odd, gyw[q], c);
      const T fv = fp[q];
      const T nbs = ((((xm + xp) + ym) + yp) + zm) + zp;
      const T nv = c + omega * ((nbs - h2 * fv) * inv6 - c);
      reinterpret_cast<T*>(&us[sp][lyq][0])[lx] = nv;
    }
  };

  // step t makes plane P = zstart + t the newest (K = P mod FR, compile-time); steps -PD..-1
  // only prefetch the first planes
  auto step = [&](int g, auto kk) __attribute__((always_inline)) {
    constexpr int K = decltype(kk)::value;
    constexpr int Q = K % PD;   // prefetch slot of plane P (and of P + PD)
    const int t = g + K;
    if (t < -PD || t >= nsteps) return;
    const int P = zstart + t;
    if (t < 0) {
      fetch(P + PD, pu[Q], pf[Q]);
      return;
    }
    {
      // plane P replaces plane P-RING in the u ring (last read before the previous step's
      // final barrier) and plane P-FR in this thread's f ring
      const int sn = ((P % RING) + RING) % RING;
#pragma unroll
      for (int q = 0; q < PPT; ++q) {
        us[sn][ly[q]][lxp[q]] = pu[Q][q];
        fr[K][0][q] = pf[Q][q][0];
        fr[K][1][q] = pf[Q][q][1];
      }
    }
    __syncthreads();
    if (t + PD < nsteps) fetch(P + PD, pu[Q], pf[Q]);
    // stage s runs on plane P-1-s, whose f is in ring slot (K - 1 - s) mod FR
    stage(P - 1, 0, 0, fr[(K + FR - 1) % FR][0]);
    __syncthreads();
    stage(P - 2, 1, 1, fr[(K + FR - 2) % FR][1]);
    __syncthreads();
    if constexpr (NS == 2) {
      stage(P - 3, 0, 2, fr[(K + 2 * FR - 3) % FR][0]);
      __syncthreads();
      stage(P - 4, 1, 3, fr[(K + 2 * FR - 4) % FR][1]);
      __syncthreads();
    }
    // the last stage's plane is final on the output box
    const int po = P - NST;
    if (po >= z0 && po < zend) {
      const int pg = po & nm;
      const int so = ((po % RING) + RING) % RING;
#pragma unroll
      for (int q = 0; q < PPT; ++q)
        if (outxy[q]) {
          const size_t off = ((size_t)pg << (2 * L)) + ((size_t)gyw[q] << L) + (size_t)gxw[q];
          *reinterpret_cast<TbPair<T>*>(uout + off) = us[so][ly[q]][lxp[q]];
        }
    }
  };
  // steps are unrolled in groups of FR so every ring slot is a fixed register set: the group
  // index g is congruent to -(zstart mod FR), so step t = g + K holds plane P with
  // P mod FR = K; the first group starts early enough to include the prefetch-only steps
  const int k0 = ((zstart % FR) + FR) % FR;
  static_assert(FR % PD == 0 && FR <= 6, "unrolled group");
  for (int g = -k0 - FR; g < nsteps; g += FR) {
    step(g, std::integral_constant<int, 0>{});
    step(g, std::integral_constant<int, 1>{});
    step(g, std::integral_constant<int, 2>{});
    step(g, std::integral_constant<int, 3>{});
    if constexpr (FR > 4) {
      step(g, std::integral_constant<int, 4>{});
      step(g, std::integral_constant<int, 5>{});
    }
  }
}

int tb_zchunk(int n) {
  if (n >= 512) return 64;
  if (n >= 256) return 32;
  return 16;
}

// Tile height per precision and pass: FP64 64 x 32 (one x-pair per thread, 16 KB per LDS
// plane); FP32 64 x 64 (two pairs per thread) except with the prolongation, whose coarse
// taps need the registers of a second pair.
template <typename T, bool PRO>
struct TbCfg {
  static constexpr int TY = (sizeof(T) == 4 && !PRO) ? 64 : 32, THREADS = 1024;
};

template <typename T, int NS, bool PRO>
void tb_launch(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int n, double h, double omega,
               const LevelBC& bc, hipStream_t s) {
  constexpr int TY = TbCfg<T, PRO>::TY, THREADS = TbCfg<T, PRO>::THREADS;
  TbArgs A;
  std::memset(&A, 0, sizeof(A));
  A.uin = uin;
  A.uout = uout;
  A.f = f;
  A.ec = ec;
  A.bc = bc;
  A.bcc = bcc;
  A.n = n;
  A.L = ilog2(n);
  A.h2 = h * h;
  A.omega = omega;
  const int OX = kTbTX - 4 * NS, OY = TY - 4 * NS;
  A.zc = min(tb_zchunk(n), n);
  A.tiles_x = (n + OX - 1) / OX;
  A.tiles_y = (n + OY - 1) / OY;
  A.chunks_z = (n + A.zc - 1) / A.zc;
  A.ntiles = A.tiles_x * A.tiles_y * A.chunks_z;
  const int grid = (A.ntiles + 7) / 8 * 8;
  hipLaunchKernelGGL((k_tb<T, NS, PRO, TY, THREADS>), dim3(grid), dim3(THREADS), 0, s, A);
}

}  // namespace

template <typename T>
void tb_sweeps(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int nsweeps, int n, double h,
               double omega, const LevelBC& bc, hipStream_t s) {
  if (ec) {
    if (nsweeps == 2) tb_launch<T, 2, true>(uin, uout, f, ec, bcc, n, h, omega, bc, s);
    else tb_launch<T, 1, true>(uin, uout, f, ec, bcc, n, h, omega, bc, s);
  } else {
    if (nsweeps == 2) tb_launch<T, 2, false>(uin, uout, f, ec, bcc, n, h, omega, bc, s);
    else tb_launch<T, 1, false>(uin, uout, f, ec, bcc, n, h, omega, bc, s);
  }
}

template <typename T>
std::string tb_name(int nsweeps, bool pro) {
  const int TY = pro ? TbCfg<T, true>::TY : TbCfg<T, false>::TY;
  return std::string("k_tb<") + (sizeof(T) == 8 ? "double" : "float") + ", " + std::to_string(nsweeps) + ", " +
         (pro ? "true" : "false") + ", " + std::to_string(TY) + ", 1024>";
}

template void tb_sweeps<double>(const double*, double*, const double*, const double*, const LevelBC&, int, int,
                                double, double, const LevelBC&, hipStream_t);
template void tb_sweeps<float>(const float*, float*, const float*, const float*, const LevelBC&, int, int, double,
                               double, const LevelBC&, hipStream_t);
template std::string tb_name<double>(int, bool);
template std::string tb_name<float>(int, bool);

}  // namespace mg
