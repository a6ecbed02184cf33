// mg_march.inl -- two-sweep streaming passes of the large levels (the bandwidth path); included
// once per precision by mg_march_f64.hip and mg_march_f32.hip.
//
// One launch = the whole work of a V-cycle leg on one level, with u and f crossing HBM once:
//   down (Alg. 1 steps 1-3): two red-black SOR sweeps (eqs. rbsor1-2), then the defect
//        f - L u of the result (eq. defect) restricted to the coarse level (eq. restriction)
//        and the coarse correction cleared;
//   up   (Alg. 1 steps 5-7): u += trilinear prolongation of the coarse correction (eq.
//        trilinear) as u is loaded, then two sweeps, optionally followed by the defect of the
//        result summed as squares (the convergence norm of Sec. 2.3.7);
//   FAS down (Alg. 3 steps 2-4, k_march_fas): the down leg with the swept u restricted beside
//        the defect (phibar, also the coarse level's starting iterate).
//
// Work layout.  A workgroup of W = 8 waves owns a tile of 64 x 64 cells in x-y and marches a
// chunk of z planes.  Each half-wave holds a band of R = 4 rows, each lane the x-pair (2l, 2l+1)
// of those rows.  At the step that loads plane P the stages run on older planes:
//   red sweep 1 on P-1, black 1 on P-2, red 2 on P-3, black 2 on P-4, defect on P-4,
// so every stage reads its z-neighbours in the colour state it needs.  u of six planes lives in
// registers (a ring), f of plane P-1 in registers and of P-2..P-4 in per-thread LDS slots.
//
// The colour pattern is a compile-time constant: tile origins, halos and z-chunk starts are
// even, chunks start at multiples of 6 and the ring has 6 planes, so the parity of the plane a
// stage works on, and which cell of a lane's x-pair is red in each row, are template constants.
// A stage then updates exactly one cell per row with no operand selection: two cross-lane moves
// (DPP wave shifts) for the x-neighbour, in-lane rows or one LDS exchange of the band-edge rows
// for y, ring planes for z.
//
// The defect stage needs the final state of both neighbouring planes.  Black cells of P-4 have
// only red neighbours, final after red sweep 2; red cells of P-4 get their in-plane and lower
// neighbours now and the upper one (black, final one step later) at the next step, so the ring
// stays at six planes.  Tiles overlap by a halo of 6 cells (5 stages of radius 1, rounded up to
// even) and are recomputed, so tiles are independent and the result goes to another array.
//
// Non-periodic faces (Sec. 2.3.6): a ghost value is kappa * (the adjacent active cell's current
// value) + beta, with kappa = +1, beta = 0 for a zero-gradient face and kappa = -1, beta = 2 b
// for a fixed face.  beta enters only the stencil of that active cell, and there with the
// weight of a neighbour, so it is folded into the cell's source as f - beta / h^2 when f is
// loaded; what remains of the ghost is kappa times the cell's own current value:
//   x: the lane holding x = 0 (x = n-1) takes kappa * c in place of its left (right) neighbour;
//   y: with 52-row output tiles and a halo of 6 the rows beyond y = 0 and y = n-1 are always
//      rows 1 and 2 of the same lane as their active neighbour; before each stage the ghost
//      cells the stage reads are set to kappa times that neighbour (in-lane);
//   z: the ring plane beyond z = 0 or z = n-1 is set the same way before a stage on the
//      boundary plane.
// Cells outside the domain are loaded from their periodic image (every address in range, no
// predicated loads) and swept like the others; no active cell reads them.  The coarse
// correction's taps (homogeneous conditions) are clamped to the domain with the sign of each
// face's rule.
#include "mg_march.h"

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <utility>

#include "mg_launch.h"

namespace mg {

namespace {

constexpr int kLanes = 64;
constexpr int kR = 4;          // rows per lane (a band)
constexpr int kSL = 32;        // lanes per x segment (a half-wave)
constexpr int kTX = 2 * kSL;   // tile width
constexpr int kRing = 6;       // u planes held per lane
constexpr int kFSlots = 3;     // f planes held in LDS per lane
constexpr int kHalo = 6;       // tile overlap in x and y

struct MarchArgs {
  const void* uin;   // u on input (not read when zero_in)
  void* uout;
  const void* f;
  const void* ec;    // up: coarse correction (n/2)^3
  void* fc;          // down: restricted defect (n/2)^3
  void* uc0;         // down: coarse correction to clear (FAS: to start from phibar)
  void* pbar;        // FAS down: the restricted potential phibar
  double* part;      // norm: one partial sum per workgroup
  LevelBC bc;        // this level
  LevelBC bcc;       // up: coarse level (homogeneous)
  int n, L, xo, yo, zc, tiles_x, tiles_y, ntiles;
  int set;           // tiles of this launch: 0 all, 1 the interior ones, 2 the ring at the walls
  int zero_in;
  int Lm;            // BLK: log2 of the MeshBlock side on this level (the coarse level: Lm - 1)
  double h2, ih2, omega;
};

template <int N, typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl<N>(f, std::make_integer_sequence<int, N>{});
}

// Whole-wave shift by one lane through DPP: wave_shr:1 gives lane i the value of lane i-1,
// wave_shl:1 the value of lane i+1.  UNTIED: lanes without a source read zero (bound control),
// which leaves the destination untied from the source (no copy before each move; used by the
// all-periodic passes); otherwise they keep their own value (the non-periodic passes, whose
// register allocation fares better with it).  Those lanes, and the edge lanes of each
// half-wave, hold the outermost columns of a tile, inside its halo.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

template <int CTRL, bool UNTIED>
__device__ __forceinline__ int dpp_move32(int v) {
  if constexpr (UNTIED) return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
  else return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL, bool UNTIED>
__device__ __forceinline__ float dpp_move(float v) {
  return __builtin_bit_cast(float, dpp_move32<CTRL, UNTIED>(__builtin_bit_cast(int, v)));
}
template <int CTRL, bool UNTIED>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo2 = dpp_move32<CTRL, UNTIED>((int)(b & 0xffffffffLL));
  const int hi2 = dpp_move32<CTRL, UNTIED>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi2 << 32) | (long long)(unsigned)lo2);
}
template <bool UNTIED, typename T>
__device__ __forceinline__ T from_left(T v) {   // value of lane - 1
  return dpp_move<kDppWaveShr1, UNTIED>(v);
}
template <bool UNTIED, typename T>
__device__ __forceinline__ T from_right(T v) {  // value of lane + 1
  return dpp_move<kDppWaveShl1, UNTIED>(v);
}

// Ghost rule of a face as ghost = kappa * adjacent + beta: zero gradient kappa = 1, beta = 0;
// fixed (and multipole) kappa = -1, beta = 2 b at the face point (t1, t2).
template <typename T>
__device__ __forceinline__ T kappa_of(const LevelBC& bc, int face) {
  return bc.kind[face] == BC_ZERO_GRADIENT ? (T)1 : (T)-1;
}
template <typename T>
__device__ __forceinline__ T beta_of(const LevelBC& bc, int face, int n, int t1, int t2) {
  return bc.kind[face] == BC_ZERO_GRADIENT ? (T)0 : (T)(2.0 * face_b(bc, face, n, t1, t2));
}

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T a, b;
};

// MeshBlock storage index split into its x-y part and its z part (disjoint bits, so the index
// is their sum): the x-y part is fixed per lane and row, the z part is uniform per plane.  Both
// are 32-bit (a 64-bit index costs these passes register spills): the launcher sends only
// levels of fewer than 2^32 cells here.
__device__ __forceinline__ unsigned blk_xy(int Lm, int i, int j) {
  const int mm = (1 << Lm) - 1;
  return ((spread3((unsigned)(i >> Lm)) | (spread3((unsigned)(j >> Lm)) << 1)) << (3 * Lm)) |
         (unsigned)(((j & mm) << Lm) | (i & mm));
}
__device__ __forceinline__ unsigned blk_z(int Lm, int k) {
  const int mm = (1 << Lm) - 1;
  return ((spread3((unsigned)(k >> Lm)) << 2) << (3 * Lm)) | (unsigned)((k & mm) << (2 * Lm));
}

// Waves per workgroup: 8 (a 64 x 64 tile, 2 waves per SIMD with up to 256 registers per lane;
// FP32 on 16 waves, a 64 x 128 tile, needs more than the 128 registers that leaves per lane).
template <typename T>
constexpr int cfg_W() {
  return 8;
}

// WALLS: 0 = every face of the level is periodic (no boundary code compiled in); 1 = walls
// only across z (x and y periodic, or a tile that reaches no x or y wall with its halo: no x/y
// wall code compiled in); 2 = walls on any axis.  The launcher picks per tile.  BLK: the level is in the MeshBlock layout (blocks of 2^A.Lm cells, Morton order);
// the tile streams across block boundaries as across a dense array (an x-pair never straddles
// two blocks), and the coarse level is in the layout below (blocks of 2^(A.Lm-1) cells, or the
// dense root grid when that is one cell).
// FAS (down only, Alg. 3 steps 2-4): the restriction also writes the restricted potential
// phibar (mean of the 8 children of the pass's result) into A.pbar and starts the coarse level
// from it (uc0 = phibar instead of 0).
template <typename T, int W, bool UP, bool NORM, int WALLS, bool BLK, bool FAS>
__device__ __forceinline__ void march_body(const MarchArgs& A) {
  constexpr bool PER = WALLS == 0;                // every face periodic
  constexpr bool XYW = WALLS == 2;                // x or y walls may be in reach
  constexpr int R = kR, SL = kSL, NB = 2 * W, NT = kLanes * W;
  constexpr bool DEF = !UP;                       // down: restricted defect
  constexpr bool DSTAGE = DEF || NORM;            // a defect stage after the sweeps
  constexpr int HZ = DSTAGE ? 5 : 4;              // planes marched before (and after) the chunk
  __shared__ Pair<T> xch[2][NB][2][SL];
  __shared__ Pair<T> fl[kFSlots][R][NT];
  // walls with face values: -beta / h^2 of the wall cells of the plane being loaded, added to
  // their f when that plane's f is taken up at the end of the step (x walls: per band, side
  // and row; y walls: per side, column and cell)
  __shared__ T fdx[XYW ? NB : 1][2][R];
  __shared__ T fdy[2][XYW ? SL : 1][2];
  // non-periodic: the red cells' partial defects carried to the next step (registers are short)
  __shared__ T dredl[PER ? 1 : R][PER ? 1 : NT];

  const int tid = threadIdx.x;
  const int lane = tid & (kLanes - 1);
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int seg = lane >> 5;
  const int xl = lane & (SL - 1);
  const int band = 2 * w + seg;
  // XCD-aware order: consecutive block ids go to different XCDs, so give each XCD a
  // contiguous run of tiles (neighbouring tiles then share that XCD's L2 for their halos)
  const int nbk = gridDim.x, bid = blockIdx.x;
  const int tile = (bid & 7) * (nbk >> 3) + (bid >> 3);
  double acc = 0.0;
  if (tile < A.ntiles) {
    // tile coordinates and z-chunk: every tile; the interior rectangle [1, tiles_x - 1) x
    // [1, tiles_y - 1); or the ring around it (bottom row, top row, then the two side columns)
    int tx, ty, cz;
    if (A.set == 0) {
      tx = tile % A.tiles_x;
      ty = (tile / A.tiles_x) % A.tiles_y;
      cz = tile / (A.tiles_x * A.tiles_y);
    } else if (A.set == 1) {
      const int wi = A.tiles_x - 2, per = wi * (A.tiles_y - 2), t = tile % per;
      cz = tile / per;
      tx = 1 + t % wi;
      ty = 1 + t / wi;
    } else {
      const int per = 2 * A.tiles_x + 2 * (A.tiles_y - 2);
      int q = tile % per;
      cz = tile / per;
      if (q < A.tiles_x) {
        tx = q;
        ty = 0;
      } else if (q < 2 * A.tiles_x) {
        tx = q - A.tiles_x;
        ty = A.tiles_y - 1;
      } else {
        q -= 2 * A.tiles_x;
        tx = (q & 1) ? A.tiles_x - 1 : 0;
        ty = 1 + (q >> 1);
      }
    }
    const int n = A.n, L = A.L, nm = n - 1;
    const T* __restrict__ uin = reinterpret_cast<const T*>(A.uin);
    T* __restrict__ uout = reinterpret_cast<T*>(A.uout);
    const T* __restrict__ fin = reinterpret_cast<const T*>(A.f);
    // storage index of cell (X, Y, Z) of the coarse level below
    auto cdx = [&](int X, int Y, int Z) __attribute__((always_inline)) {
      return BLK ? lidx(L - 1, A.Lm - 1, X, Y, Z) : cidx(L - 1, X, Y, Z);
    };
    const bool px = !XYW || A.bc.kind[0] == BC_PERIODIC;
    const bool py = !XYW || A.bc.kind[2] == BC_PERIODIC;
    const bool pz = PER || A.bc.kind[4] == BC_PERIODIC;
    const T h2 = (T)A.h2, ih2 = (T)A.ih2, omega = (T)A.omega;
    const T inv6 = (T)(1.0 / 6.0);

    const int xs = tx * A.xo;                    // first output column (even)
    const int xa = xs - kHalo + 2 * xl;          // this lane's even column
    const int xag = xa & nm;
    const bool out_x = xa >= xs && xa < xs + A.xo && xa < n;
    // the lane whose even cell is x = 0, whose odd cell is x = n-1 (beside a wall)
    const bool wx0 = XYW && !px && xa == 0;
    [[maybe_unused]] const bool in_x = px || (xa >= 0 && xa < n);
    const bool wx1 = XYW && !px && xa == n - 2;

    const int ys = ty * A.yo;                    // first output row (even)
    int yv[R], ygv[R];
    bool out_y[R];
    [[maybe_unused]] bool in_y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = ys - kHalo + band * R + r;
      yv[r] = y;
      ygv[r] = y & nm;
      out_y[r] = y >= ys && y < ys + A.yo && y < n;
      in_y[r] = py || (y >= 0 && y < n);
    }
    // MeshBlock layout: the x-y part of each row's storage index (the z part is added per plane)
    unsigned rxy[BLK ? R : 1];
    if constexpr (BLK) {
#pragma unroll
      for (int r = 0; r < R; ++r) rxy[r] = blk_xy(A.Lm, xag, ygv[r]);
    }
    // storage index of row r of this lane on plane z
    auto fidr = [&](int r, int z) __attribute__((always_inline)) -> size_t {
      if constexpr (BLK) return (size_t)(rxy[r] + blk_z(A.Lm, z));
      else return cidx(L, xag, ygv[r], z);
    };
    // up, MeshBlock layout: the x-y part of the coarse taps' storage indices (rows Y0-1 ..
    // Y0+2 of the lane's coarse column, wrapped or clamped as the taps take them); the coarse
    // level is in blocks of 2^(Lm-1) cells, or the dense root grid when Lm = 1
    constexpr int NTAP = R / 2 + 2;
    unsigned cxy[UP ? NTAP : 1];
    if constexpr (UP) {
      const int nc = n >> 1, Lc = L - 1;
      int X = (px ? xag : xa) >> 1;
      if constexpr (XYW) X = min(max(X, 0), nc - 1);
      const int Y0 = (py ? ygv[0] : yv[0]) >> 1;
#pragma unroll
      for (int i = 0; i < NTAP; ++i) {
        int Y = Y0 - 1 + i;
        if (py) Y &= nc - 1;
        if constexpr (XYW) Y = min(max(Y, 0), nc - 1);
        cxy[i] = !BLK || A.Lm == 1 ? (unsigned)((Y << Lc) | X) : blk_xy(A.Lm - 1, X, Y);
      }
    }
    const int z0 = cz * A.zc;                    // a multiple of 6
    const int zend = min(z0 + A.zc, n);
    const int zstart = z0 - HZ;
    const int nsteps = (zend - z0) + 2 * HZ;
    // rows 1 and 2 of this lane are the ghost row beyond y = 0 and its active neighbour, or the
    // active row y = n-1 and the ghost beyond it
    const bool gy0 = XYW && !py && yv[1] == -1;
    const bool gy1 = XYW && !py && yv[2] == n;
    // does any cell of this wave sit beside a wall in x or y?
    const int wy0 = ys - kHalo + w * 2 * R, wy1 = wy0 + 2 * R - 1;
    const bool wave_x = XYW && !px && (xs - kHalo < 0 || xs - kHalo + kTX - 1 >= n);
    const bool wave_y = XYW && !py && (wy0 < 0 || wy1 >= n);
    // fold beta of the walls with face values into f (fixed and multipole faces)
    const bool fold_x = wave_x && (A.bc.b[0] || A.bc.b[1]);
    const bool fold_y = wave_y && (A.bc.b[2] || A.bc.b[3]);
    const T kx0 = kappa_of<T>(A.bc, 0), kx1 = kappa_of<T>(A.bc, 1), ky0 = kappa_of<T>(A.bc, 2);
    const T ky1 = kappa_of<T>(A.bc, 3), kz0 = kappa_of<T>(A.bc, 4), kz1 = kappa_of<T>(A.bc, 5);
    // up: the coarse correction's rules (homogeneous conditions)
    const T kcx0 = kappa_of<T>(A.bcc, 0), kcx1 = kappa_of<T>(A.bcc, 1), kcy0 = kappa_of<T>(A.bcc, 2);
    const T kcy1 = kappa_of<T>(A.bcc, 3), kcz0 = kappa_of<T>(A.bcc, 4), kcz1 = kappa_of<T>(A.bcc, 5);

    T u[kRing][R][2];
    T pu[R][2], pf[R][2];      // prefetched u of plane P+1 and f of plane P
    T fr[R][2];                // f of plane P-1
    T dred[PER ? R : 1];       // red cells' partial defects of plane P-4 (completed next step)
    // (non-periodic: in LDS)
    auto dred_get = [&](int r) __attribute__((always_inline)) -> T { return PER ? dred[PER ? r : 0] : dredl[PER ? 0 : r][PER ? 0 : tid]; };
    auto dred_set = [&](int r, T v) __attribute__((always_inline)) {
      if constexpr (PER) dred[r] = v;
      else dredl[r][tid] = v;
    };
    T pend[R / 2], stash[R / 2];   // down: row-pair defect sums (black cells of P-4; even plane)
    T stash_u[FAS ? R / 2 : 1];      // FAS: row-pair sums of u on the even plane of a coarse plane
    T pc[UP ? NTAP : 1][2];    // up: coarse rows Y0-1 .. Y0+2 on the two coarse planes of a fine plane
#pragma unroll
    for (int s = 0; s < kRing; ++s)
#pragma unroll
      for (int r = 0; r < R; ++r) u[s][r][0] = u[s][r][1] = (T)0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      fr[r][0] = fr[r][1] = (T)0;
      dred_set(r, (T)0);
#pragma unroll
      for (int q = 0; q < kFSlots; ++q) fl[q][r][tid] = Pair<T>{(T)0, (T)0};
    }
#pragma unroll
    for (int j = 0; j < R / 2; ++j) pend[j] = stash[j] = (T)0;
    if constexpr (FAS) {
#pragma unroll
      for (int j = 0; j < R / 2; ++j) stash_u[j] = (T)0;
    }

    // ---- loads of u on plane P (unless zero on input) and f on plane P-1 (the plane the red
    // stage of the next step works on), beta of the walls folded into f; up: the coarse taps
    // of plane P
    // cTAPS (up): 0 load both coarse planes of P, 1 (P odd) keep the upper plane of P-1 as the
    // lower one and load the upper, 2 (P even) keep the pair of P-1
    auto load_plane = [&](int P, auto cTAPS) __attribute__((always_inline)) {
      const int Pg = P & nm, Pfg = (P - 1) & nm;
      if constexpr (XYW) {
        // beta of the x and y walls (fixed and multipole faces) for this plane's f: loaded
        // before u and f, so waiting for them does not wait for the plane, and parked in LDS
        // until the f it belongs to is taken up; every lane loads (from a valid address) and
        // keeps its value or zero
        if (fold_x || fold_y) {
          const T bw = -(T)2 * ih2;   // f - beta / h^2 with beta = 2 b
          const size_t row = (size_t)(Pfg + 1) * (size_t)(n + 2);
          const double* bxa = A.bc.b[0] ? A.bc.b[0] : A.bc.b[1];
          const double* bxb = A.bc.b[1] ? A.bc.b[1] : A.bc.b[0];
          const double* bya = A.bc.b[2] ? A.bc.b[2] : A.bc.b[3];
          const double* byb = A.bc.b[3] ? A.bc.b[3] : A.bc.b[2];
          const bool hx = (wx0 && A.bc.b[0]) || (wx1 && A.bc.b[1]);
          const bool hy = (gy0 && A.bc.b[2]) || (gy1 && A.bc.b[3]);
          const double* bxp = wx1 ? bxb : bxa;
          const double* byp = gy1 ? byb : bya;
          T dx[R], dy[2];
#pragma unroll
          for (int r = 0; r < R; ++r) dx[r] = (T)0;
          dy[0] = dy[1] = (T)0;
          if (fold_x) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const double v = bxp[row + (size_t)(ygv[r] + 1)];
              dx[r] = hx ? bw * (T)v : (T)0;
            }
          }
          if (fold_y) {
#pragma unroll
            for (int e = 0; e < 2; ++e) {
              const double v = byp[row + (size_t)(((xag + e) & nm) + 1)];
              dy[e] = hy ? bw * (T)v : (T)0;
            }
          }
          if (wx0 || wx1) {
#pragma unroll
            for (int r = 0; r < R; ++r) fdx[band][wx1 ? 1 : 0][r] = dx[r];
          }
          if (gy0 || gy1) {
            fdy[gy1 ? 1 : 0][xl][0] = dy[0];
            fdy[gy1 ? 1 : 0][xl][1] = dy[1];
          }
        }
      }
      if constexpr (PER) {
        // (the range tests are trivially true here; written out, they keep the compiler's
        // register allocation of the periodic passes at its best)
        const bool in_z = pz || (P >= 0 && P < n);
        const bool in_zf = pz || (P - 1 >= 0 && P - 1 < n);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (in_x && in_y[r] && in_z && !A.zero_in) {
            const Pair<T> vu = *reinterpret_cast<const Pair<T>*>(uin + fidr(r, Pg));
            pu[r][0] = vu.a; pu[r][1] = vu.b;
          } else {
            pu[r][0] = pu[r][1] = (T)0;
          }
          if (in_x && in_y[r] && in_zf) {
            const Pair<T> vf = *reinterpret_cast<const Pair<T>*>(fin + fidr(r, Pfg));
            pf[r][0] = vf.a; pf[r][1] = vf.b;
          } else {
            pf[r][0] = pf[r][1] = (T)0;
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (!A.zero_in) {
            const Pair<T> vu = *reinterpret_cast<const Pair<T>*>(uin + fidr(r, Pg));
            pu[r][0] = vu.a; pu[r][1] = vu.b;
          } else {
            pu[r][0] = pu[r][1] = (T)0;
          }
          const Pair<T> vf = *reinterpret_cast<const Pair<T>*>(fin + fidr(r, Pfg));
          pf[r][0] = vf.a; pf[r][1] = vf.b;
        }
      }
      if constexpr (!PER) {
        // the z walls: beta on the first and last plane of the level (two planes per pass;
        // loaded and applied at once)
        if (!pz && (Pfg == 0 || Pfg == nm)) {
          const double* bz = Pfg == 0 ? A.bc.b[4] : A.bc.b[5];
          if (bz) {
            const T bw = -(T)2 * ih2;
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
              for (int e = 0; e < 2; ++e)
                pf[r][e] += bw * (T)bz[(size_t)(ygv[r] + 1) * (size_t)(n + 2) + (size_t)(((xag + e) & nm) + 1)];
          }
        }
      }
      if constexpr (UP) {
        // Trilinear prolongation (weights 1/4, 3/4 per axis) of the coarse correction: the
        // lane's coarse column X, coarse rows Y0-1 .. Y0+2 (rows 2j, 2j+1 of the band take
        // Y0+j-1 .. Y0+j+1) on the coarse planes (zlo, zlo+1) of fine plane P; the x-neighbour
        // columns come from the lanes beside (an edge lane of a segment gets zero or another
        // band's value: wrong, but only in the outermost column of the tile, inside the halo).  Fine
        // plane 2Z takes coarse planes (Z-1, Z), plane 2Z+1 (Z, Z+1), so the fine planes 2Z+1
        // and 2Z+2 take the same pair (also where the planes wrap or are clamped): an odd plane
        // loads one new coarse plane, an even one none (the parity is a template constant of
        // each pipeline step).
        constexpr int TAPS = decltype(cTAPS)::value;
        const T* __restrict__ ec = reinterpret_cast<const T*>(A.ec);
        const int nc = n >> 1, Lc = L - 1;
        const int X = (px ? xag : xa) >> 1;
        const int Y0 = (py ? ygv[0] : yv[0]) >> 1;
        const int Pz = pz ? (P & nm) : P;
        const int Z = Pz >> 1;
        const int zlo = (Pz & 1) ? Z : Z - 1;
        auto tap = [&](int i, int zz) __attribute__((always_inline)) {
          int Y = Y0 - 1 + i;
          if (py) Y &= nc - 1;
          if (pz) zz &= nc - 1;
          // the lane's x-y part (wrapped, or clamped into the domain) plus the plane's z part;
          // every face periodic: the wrapped indices are in range (no ghost code compiled);
          // otherwise the sign of the wall's rule when clamped (selects: no branches around
          // the load)
          const int Zc = PER ? zz : min(max(zz, 0), nc - 1);
          const size_t ci = (size_t)cxy[i] + (!BLK || A.Lm == 1 ? ((size_t)Zc << (2 * Lc)) : (size_t)blk_z(A.Lm - 1, Zc));
          if constexpr (PER) {
            return ec[ci];
          } else if constexpr (!XYW) {
            // x and y taps wrapped into the domain: only a z wall's sign (the same value as
            // the general form, whose x and y factors are 1 here)
            const T sz = zz < 0 ? kcz0 : (zz >= nc ? kcz1 : (T)1);
            return sz * ec[ci];
          } else {
            const T sx = X < 0 ? kcx0 : (X >= nc ? kcx1 : (T)1);
            const T sy = Y < 0 ? kcy0 : (Y >= nc ? kcy1 : (T)1);
            const T sz = zz < 0 ? kcz0 : (zz >= nc ? kcz1 : (T)1);
            return (sx * sy) * (sz * ec[ci]);
          }
        };
        if constexpr (TAPS == 0) {
#pragma unroll
          for (int i = 0; i < NTAP; ++i) {
            pc[i][0] = tap(i, zlo);
            pc[i][1] = tap(i, zlo + 1);
          }
        } else if constexpr (TAPS == 1) {
#pragma unroll
          for (int i = 0; i < NTAP; ++i) {
            pc[i][0] = pc[i][1];
            pc[i][1] = tap(i, zlo + 1);
          }
        }
      }
    };

    // ---- the parked wall terms of the f just taken up into fr
    auto fold_take = [&]() __attribute__((always_inline)) {
      if constexpr (XYW) {
        if (fold_x) {
#pragma unroll
          for (int r = 0; r < R; ++r) {
            const T d0 = fdx[band][0][r], d1 = fdx[band][1][r];
            fr[r][0] += wx0 ? d0 : (T)0;
            fr[r][1] += wx1 ? d1 : (T)0;
          }
        }
        if (fold_y) {
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const T d0 = fdy[0][xl][e], d1 = fdy[1][xl][e];
            fr[2][e] += gy0 ? d0 : (T)0;
            fr[1][e] += gy1 ? d1 : (T)0;
          }
        }
      }
    };

    // ---- add the prolonged correction fetched with plane P (parity PARP) to the prefetched u
    auto prolong_apply = [&](int P, auto cPAR) __attribute__((always_inline)) {
      if constexpr (UP) {
        constexpr int PARP = decltype(cPAR)::value;
        const T wz0 = PARP ? (T)0.75 : (T)0.25, wz1 = PARP ? (T)0.25 : (T)0.75;
        T czv[NTAP];
#pragma unroll
        for (int i = 0; i < NTAP; ++i) czv[i] = wz0 * pc[i][0] + wz1 * pc[i][1];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int j = r >> 1;
          const T c = (r & 1) ? (T)0.75 * czv[j + 1] + (T)0.25 * czv[j + 2] : (T)0.25 * czv[j] + (T)0.75 * czv[j + 1];
          const T cl = from_left<PER>(c), cr = from_right<PER>(c);
          pu[r][0] += (T)0.25 * cl + (T)0.75 * c;
          pu[r][1] += (T)0.75 * c + (T)0.25 * cr;
        }
      }
    };

    int xbuf = 0;

    // ---- ghost cells read by the active cells of colour COL (0 red, 1 black, 2 both) of plane p
    // (parity PAR, in uc; the planes beside it in um, up): y ghost rows and z ghost planes set
    // to kappa times those cells' current values (x walls are taken in the stencil)
    auto refresh = [&](auto cCOL, auto cPAR, T (&um)[R][2], T (&uc)[R][2], T (&up)[R][2], int p)
                       __attribute__((always_inline)) {
      if constexpr (!PER) {
        constexpr int COL = decltype(cCOL)::value, PAR = decltype(cPAR)::value;
        // does cell e of row r have a colour being refreshed?
        auto sel = [](int r, int e) constexpr { return COL == 2 || ((r + PAR + COL) & 1) == e; };
        if (wave_y) {
          static_for<2>([&](auto ee) __attribute__((always_inline)) {
            constexpr int e = decltype(ee)::value;
            if constexpr (sel(2, e))
              if (gy0) uc[1][e] = ky0 * uc[2][e];
            if constexpr (sel(1, e))
              if (gy1) uc[2][e] = ky1 * uc[1][e];
          });
        }
        // (two separate blocks: a store through a pointer chosen between the two ring planes
        // would move the ring out of registers)
        if (!pz && p == 0) {
          static_for<R>([&](auto rr) __attribute__((always_inline)) {
            constexpr int r = decltype(rr)::value;
            static_for<2>([&](auto ee) __attribute__((always_inline)) {
              constexpr int e = decltype(ee)::value;
              if constexpr (sel(r, e)) um[r][e] = kz0 * uc[r][e];
            });
          });
        }
        if (!pz && p == nm) {
          static_for<R>([&](auto rr) __attribute__((always_inline)) {
            constexpr int r = decltype(rr)::value;
            static_for<2>([&](auto ee) __attribute__((always_inline)) {
              constexpr int e = decltype(ee)::value;
              if constexpr (sel(r, e)) up[r][e] = kz1 * uc[r][e];
            });
          });
        }
      }
    };

    // ---- one colour C (0 red, 1 black) of the RB-SOR update (eqs. rbsor1-2) on plane p of
    // parity PAR held in uc, its z-neighbour planes in um (p-1) and up (p+1); f from the
    // registers (FS < 0) or LDS slot FS
    auto colour = [&](auto cC, auto cPAR, auto cFS, T (&um)[R][2], T (&uc)[R][2], T (&up)[R][2],
                      int p) __attribute__((always_inline)) {
      constexpr int C = decltype(cC)::value, PAR = decltype(cPAR)::value, FS = decltype(cFS)::value;
      refresh(cC, cPAR, um, uc, up, p);
      // the band-edge rows' cells of the other colour, for the bands below and above
      constexpr int q0 = (PAR + C) & 1, qL = (R - 1 + PAR + C) & 1;
      T* xt = reinterpret_cast<T*>(&xch[xbuf][0][0][0]);
      xt[(band * 2 + 0) * SL + xl] = uc[0][q0 ^ 1];
      xt[(band * 2 + 1) * SL + xl] = uc[R - 1][qL ^ 1];
      __syncthreads();
      const T below = xt[((band > 0 ? band - 1 : band) * 2 + 1) * SL + xl];
      const T above = xt[((band < NB - 1 ? band + 1 : band) * 2 + 0) * SL + xl];
      xbuf ^= 1;
      static_for<R>([&](auto rr) __attribute__((always_inline)) {
        constexpr int r = decltype(rr)::value;
        constexpr int q = (r + PAR + C) & 1;      // the cell of this colour in row r
        const T c = uc[r][q];
        T xm, xp, ym, yp;
        if constexpr (q == 0) {
          xm = from_left<PER>(uc[r][1]);
          xp = uc[r][1];
          if constexpr (XYW) xm = wx0 ? kx0 * c : xm;
        } else {
          xm = uc[r][0];
          xp = from_right<PER>(uc[r][0]);
          if constexpr (XYW) xp = wx1 ? kx1 * c : xp;
        }
        if constexpr (r > 0) ym = uc[r - 1][q]; else ym = below;
        if constexpr (r < R - 1) yp = uc[r + 1][q]; else yp = above;
        const T zm = um[r][q], zp = up[r][q];
        T fv;
        if constexpr (FS < 0) fv = fr[r][q];
        else fv = q ? fl[FS][r][tid].b : fl[FS][r][tid].a;
        const T nbs = ((((xm + xp) + ym) + yp) + zm) + zp;
        uc[r][q] = c + omega * ((nbs - h2 * fv) * inv6 - c);
      });
    };

    // ---- defect stage on plane p (parity PAR, final after black sweep 2, in uc; p-1 in um,
    // p+1 in up, final in its red cells): completes the red cells of p-1 with the black cells
    // of p above them, takes the black cells of p whole and the red cells of p without their
    // upper neighbour; then the restriction (down) or the sum of squares (norm)
    auto defect = [&](auto cPAR, auto cFS, T (&um)[R][2], T (&uc)[R][2], T (&up)[R][2], int p)
                      __attribute__((always_inline)) {
      constexpr int PAR = decltype(cPAR)::value, FS = decltype(cFS)::value;
      refresh(std::integral_constant<int, 2>{}, cPAR, um, uc, up, p);
      Pair<T>* xq = &xch[xbuf][0][0][0];
      xq[(band * 2 + 0) * SL + xl] = Pair<T>{uc[0][0], uc[0][1]};
      xq[(band * 2 + 1) * SL + xl] = Pair<T>{uc[R - 1][0], uc[R - 1][1]};
      __syncthreads();
      const Pair<T> vb = xq[((band > 0 ? band - 1 : band) * 2 + 1) * SL + xl];
      const Pair<T> va = xq[((band < NB - 1 ? band + 1 : band) * 2 + 0) * SL + xl];
      xbuf ^= 1;
      const T below[2] = {vb.a, vb.b}, above[2] = {va.a, va.b};
      const bool bnd_z1 = !PER && !pz && p == nm;
      // plane p-1: its red cells' upper neighbour is final now (unless p-1 is the top plane of
      // a non-periodic axis, whose ghost was taken at once)
      const bool top_prev = !pz && p - 1 == nm;
      const bool out_prev = p - 1 >= z0 && p - 1 < zend;
      const bool out_cur = p >= z0 && p < zend;
      T dprev[R], dblk[R];
      static_for<R>([&](auto rr) __attribute__((always_inline)) {
        constexpr int r = decltype(rr)::value;
        constexpr int qr_prev = (r + PAR + 1) & 1;   // red cell of row r on plane p-1 (parity PAR^1)
        const T dr = dred_get(r);
        dprev[r] = top_prev ? dr : dr - ih2 * uc[r][qr_prev];
      });
      static_for<R>([&](auto rr) __attribute__((always_inline)) {
        constexpr int r = decltype(rr)::value;
        const Pair<T> fp = fl[FS][r][tid];
        const T fpair[2] = {fp.a, fp.b};
        // q = 0: the black cell, whole; q = 1: the red cell, without its upper neighbour
        static_for<2>([&](auto qq) __attribute__((always_inline)) {
          constexpr int black = decltype(qq)::value == 0;
          constexpr int q = (r + PAR + (black ? 1 : 0)) & 1;
          const T c = uc[r][q];
          T xm, xp, ym, yp;
          if constexpr (q == 0) {
            xm = from_left<PER>(uc[r][1]);
            xp = uc[r][1];
            if constexpr (XYW) xm = wx0 ? kx0 * c : xm;
          } else {
            xm = uc[r][0];
            xp = from_right<PER>(uc[r][0]);
            if constexpr (XYW) xp = wx1 ? kx1 * c : xp;
          }
          if constexpr (r > 0) ym = uc[r - 1][q]; else ym = below[q];
          if constexpr (r < R - 1) yp = uc[r + 1][q]; else yp = above[q];
          const T zm = um[r][q], zp = up[r][q];
          const T s5 = (((xm + xp) + ym) + yp) + zm;
          if constexpr (black) {
            dblk[r] = fpair[q] - ((s5 + zp) - (T)6 * c) * ih2;
          } else {
            // the upper neighbour of a red cell on the top plane of a non-periodic axis is the
            // ghost plane (set now); elsewhere it is added at the next step
            dred_set(r, bnd_z1 ? fpair[q] - ((s5 + zp) - (T)6 * c) * ih2 : fpair[q] - (s5 - (T)6 * c) * ih2);
          }
        });
      });
      if constexpr (NORM) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (out_x && out_y[r]) {
            if (out_cur) acc += (double)dblk[r] * (double)dblk[r];
            if (out_prev) acc += (double)dprev[r] * (double)dprev[r];
          }
        }
      }
      if constexpr (DEF) {
        // plane p-1 is complete: its row-pair sums (black part from the previous step); the
        // even plane of a coarse plane waits in stash, the odd one writes the coarse cell
        constexpr int par_prev = PAR ^ 1;
        T* __restrict__ fcp = reinterpret_cast<T*>(A.fc);
        T* __restrict__ ucp = reinterpret_cast<T*>(A.uc0);
#pragma unroll
        for (int j = 0; j < R / 2; ++j) {
          const T sprev = pend[j] + (dprev[2 * j] + dprev[2 * j + 1]);
          // FAS: the final u of plane p-1 (um) over the same four cells
          T suprev = (T)0;
          if constexpr (FAS) suprev = (um[2 * j][0] + um[2 * j][1]) + (um[2 * j + 1][0] + um[2 * j + 1][1]);
          if constexpr (par_prev == 0) {
            stash[j] = sprev;
            if constexpr (FAS) stash_u[j] = suprev;
          } else {
            if (out_prev && out_x && out_y[2 * j]) {
              const size_t ci = cdx(xag >> 1, ygv[2 * j] >> 1, (p - 1) >> 1);
              fcp[ci] = (stash[j] + sprev) * (T)0.125;
              if constexpr (FAS) {
                const T pb = (stash_u[j] + suprev) * (T)0.125;
                reinterpret_cast<T*>(A.pbar)[ci] = pb;
                ucp[ci] = pb;
              } else {
                ucp[ci] = (T)0;
              }
            }
          }
          pend[j] = dblk[2 * j] + dblk[2 * j + 1];
        }
      }
    };

    load_plane(zstart, std::integral_constant<int, 0>{});
    prolong_apply(zstart, std::integral_constant<int, HZ & 1>{});
#pragma unroll
    for (int r = 0; r < R; ++r) {
      u[0][r][0] = pu[r][0]; u[0][r][1] = pu[r][1];
      fr[r][0] = pf[r][0]; fr[r][1] = pf[r][1];
    }
    if constexpr (XYW) {
      if (fold_x || fold_y) {
        fold_take();
      }
    }
    // one pipeline step: the plane in ring slot K is P = zstart + t, t = g + K with g a
    // multiple of 6, so P - j sits in slot (K - j) mod 6, has parity (HZ + K + j) mod 2, and
    // its f is in LDS slot (K - HZ - j) mod 3 (z0 is a multiple of 6)
    auto step = [&](int g, auto kk) __attribute__((always_inline)) {
      constexpr int K = decltype(kk)::value;
      const int t = g + K;
      if (t >= nsteps) return;
      const int P = zstart + t;
      // prefetch; consumed at the end of the step
      if (t + 1 < nsteps) load_plane(P + 1, std::integral_constant<int, ((HZ + K + 1) & 1) ? 1 : 2>{});
      constexpr int s0 = K, s1 = (K + 5) % 6, s2 = (K + 4) % 6, s3 = (K + 3) % 6, s4 = (K + 2) % 6,
                    s5 = (K + 1) % 6;
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using Par1 = std::integral_constant<int, (HZ + K + 1) & 1>;
      using Par2 = std::integral_constant<int, (HZ + K + 2) & 1>;
      using Par3 = std::integral_constant<int, (HZ + K + 3) & 1>;
      using Par4 = std::integral_constant<int, (HZ + K + 4) & 1>;
      using FsReg = std::integral_constant<int, -1>;
      using Fs2 = std::integral_constant<int, ((K - HZ - 2) % 3 + 6) % 3>;
      using Fs3 = std::integral_constant<int, ((K - HZ - 3) % 3 + 6) % 3>;
      using Fs4 = std::integral_constant<int, ((K - HZ - 4) % 3 + 6) % 3>;
      colour(I0{}, Par1{}, FsReg{}, u[s2], u[s1], u[s0], P - 1);   // red, sweep 1
      colour(I1{}, Par2{}, Fs2{}, u[s3], u[s2], u[s1], P - 2);     // black, sweep 1
      colour(I0{}, Par3{}, Fs3{}, u[s4], u[s3], u[s2], P - 3);     // red, sweep 2
      colour(I1{}, Par4{}, Fs4{}, u[s5], u[s4], u[s3], P - 4);     // black, sweep 2
      if constexpr (DSTAGE) defect(Par4{}, Fs4{}, u[s5], u[s4], u[s3], P - 4);
      // plane P-4 is final: out
      {
        const int p = P - 4;
        if (p >= z0 && p < zend && out_x) {
          const int pg = p & nm;
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (out_y[r]) {
              typedef T ntv2 __attribute__((ext_vector_type(2)));
              const ntv2 v = {u[s4][r][0], u[s4][r][1]};
              __builtin_nontemporal_store(v, reinterpret_cast<ntv2*>(uout + fidr(r, pg)));
            }
        }
      }
      if (t + 1 < nsteps) {
        prolong_apply(P + 1, std::integral_constant<int, (HZ + K + 1) & 1>{});
        // u(P+1) enters the ring in the slot of P-5; f(P-1) moves to the LDS slot of P-4 (done
        // with), f(P) into the registers
#pragma unroll
        for (int r = 0; r < R; ++r) {
          u[s5][r][0] = pu[r][0]; u[s5][r][1] = pu[r][1];
          fl[Fs4::value][r][tid] = Pair<T>{fr[r][0], fr[r][1]};
          fr[r][0] = pf[r][0]; fr[r][1] = pf[r][1];
        }
        if constexpr (XYW) {
          if (fold_x || fold_y) {
            fold_take();
          }
        }
      }
    };
    for (int g = 0; g < nsteps; g += kRing) {
      step(g, std::integral_constant<int, 0>{});
      step(g, std::integral_constant<int, 1>{});
      step(g, std::integral_constant<int, 2>{});
      step(g, std::integral_constant<int, 3>{});
      step(g, std::integral_constant<int, 4>{});
      step(g, std::integral_constant<int, 5>{});
    }
  }
  if constexpr (NORM) {
    // the exchange buffer is free once every wave has left the march
    double* red = reinterpret_cast<double*>(&xch[0][0][0][0]);
    acc = wave_sum(acc);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int q = 0; q < W; ++q) s += red[q];
      A.part[blockIdx.x] = s;
    }
  }
}

template <typename T, int W, bool UP, bool NORM, int WALLS, bool BLK>
__global__ void __launch_bounds__(kLanes* W) k_march(MarchArgs A) {
  march_body<T, W, UP, NORM, WALLS, BLK, false>(A);
}

// The down pass of a Full Approximation Scheme cycle (dense FP64 levels).
template <typename T, int W, int WALLS>
__global__ void __launch_bounds__(kLanes* W) k_march_fas(MarchArgs A) {
  march_body<T, W, false, false, WALLS, false, true>(A);
}

constexpr int kCUs = 256;

// Planes per workgroup: a multiple of 6 (the ring's period; chunks then start on planes whose
// ring slot, parity and f slot are compile-time).  One workgroup per CU is resident (LDS), so
// the grid runs in rounds of kCUs workgroups; the chunk minimises rounds x (planes marched,
// 2 hz halo planes included).
int march_zchunk(int n, int tiles_xy, int hz) {
  int best = (n + 5) / 6 * 6;
  long best_cost = -1;
  for (int zc = 6; zc <= (n + 5) / 6 * 6; zc += 6) {
    const long chunks = (n + zc - 1) / zc;
    if ((long)tiles_xy * chunks > (long)kMaxPartials * 32 - 8) continue;   // partials buffer
    const long rounds = ((long)tiles_xy * chunks + kCUs - 1) / kCUs;
    const long cost = rounds * (zc + 2 * hz);
    if (best_cost < 0 || cost < best_cost) best_cost = cost, best = zc;
  }
  return best;
}

// Interior and wall tiles of a level with x or y walls: the chunk lengths of the two sets
// (both launches resident together, in one round of kCUs workgroups) that balance the interior
// march against the wall march, whose steps cost kWallCost times as much.
constexpr double kWallCost = 1.3;

bool march_split_plan(int n, int nint, int nring, int hz, int& zi, int& zr) {
  double best = -1.0;
  const long cap = (long)kMaxPartials * 32 - 8;
  for (int ci = 1; ci <= (n + 5) / 6; ++ci) {
    const int zci = ((n + ci - 1) / ci + 5) / 6 * 6;
    const long ni = (long)nint * ((n + zci - 1) / zci);
    for (int cr = 1; cr <= (n + 5) / 6; ++cr) {
      const int zcr = ((n + cr - 1) / cr + 5) / 6 * 6;
      const long nr = (long)nring * ((n + zcr - 1) / zcr);
      const long tot = ((ni + 7) / 8 + (nr + 7) / 8) * 8;
      if (tot > kCUs || tot > cap) continue;
      const double t = std::max((double)(zci + 2 * hz), kWallCost * (zcr + 2 * hz));
      if (best < 0 || t < best) best = t, zi = zci, zr = zcr;
    }
  }
  return best > 0;
}

template <typename T, bool UP, bool NORM, bool BLK>
int launch_march(MarchArgs A, hipStream_t s, const MarchAux* aux) {
  bool per = true;
  for (int f = 0; f < 6; ++f) per = per && A.bc.kind[f] == BC_PERIODIC;
  bool xyper = true;
  for (int f = 0; f < 4; ++f) xyper = xyper && A.bc.kind[f] == BC_PERIODIC;
  constexpr int W = cfg_W<T>();
  constexpr int HZ = (!UP || NORM) ? 5 : 4;
  A.L = ilog2(A.n);
  A.xo = kTX - 2 * kHalo;
  A.yo = kR * 2 * W - 2 * kHalo;
  A.tiles_x = (A.n + A.xo - 1) / A.xo;
  A.tiles_y = (A.n + A.yo - 1) / A.yo;
  A.set = 0;
  int zi = 0, zr = 0;
  if (sizeof(T) == 8 && !per && !xyper && aux && aux->s2 && A.tiles_x >= 3 && A.tiles_y >= 3 &&
      march_split_plan(A.n, (A.tiles_x - 2) * (A.tiles_y - 2), 2 * A.tiles_x + 2 * (A.tiles_y - 2), HZ, zi, zr)) {
    // FP64 with x or y walls: the interior tiles (their halos reach no x or y wall) march in
    // the z-walls-only form on this stream, the ring of wall tiles in the full form on the
    // second stream, concurrently (fork and join through events); the ring's partials follow
    // the interior's.  (Measured at 512^3: down 1.18 -> 1.05 ms, up with the norm 1.54 ->
    // 1.36 ms.  Less than the two forms' own rates promise: the two sets march at different z,
    // so halo re-reads between them miss L2.  FP32, without spills in the full form, is
    // slower split: 0.52 -> 0.57 ms.)
    MarchArgs Ai = A, Ar = A;
    Ai.set = 1;
    Ai.zc = zi;
    Ai.ntiles = (A.tiles_x - 2) * (A.tiles_y - 2) * ((A.n + zi - 1) / zi);
    const int gi = (Ai.ntiles + 7) / 8 * 8;
    Ar.set = 2;
    Ar.zc = zr;
    Ar.ntiles = (2 * A.tiles_x + 2 * (A.tiles_y - 2)) * ((A.n + zr - 1) / zr);
    const int gr = (Ar.ntiles + 7) / 8 * 8;
    if (A.part) Ar.part = A.part + gi;
    LaunchTiming& lt = launch_timing();
    const bool timed = lt.armed;
    lt.armed = false;
    if (timed) (void)hipEventRecord(lt.e0, s);
    (void)hipEventRecord(aux->fork, s);
    (void)hipStreamWaitEvent(aux->s2, aux->fork, 0);
    hipLaunchKernelGGL((k_march<T, W, UP, NORM, 2, BLK>), dim3(gr), dim3(kLanes * W), 0, aux->s2, Ar);
    hipLaunchKernelGGL((k_march<T, W, UP, NORM, 1, BLK>), dim3(gi), dim3(kLanes * W), 0, s, Ai);
    (void)hipEventRecord(aux->join, aux->s2);
    (void)hipStreamWaitEvent(s, aux->join, 0);
    if (timed) (void)hipEventRecord(lt.e1, s);
    return gi + gr;
  }
  A.zc = march_zchunk(A.n, A.tiles_x * A.tiles_y, HZ);
  const int chunks = (A.n + A.zc - 1) / A.zc;
  A.ntiles = A.tiles_x * A.tiles_y * chunks;
  const int grid = (A.ntiles + 7) / 8 * 8;
  if (per) launch_maybe_timed(k_march<T, W, UP, NORM, 0, BLK>, dim3(grid), dim3(kLanes * W), 0, s, A);
  else if (xyper) launch_maybe_timed(k_march<T, W, UP, NORM, 1, BLK>, dim3(grid), dim3(kLanes * W), 0, s, A);
  else launch_maybe_timed(k_march<T, W, UP, NORM, 2, BLK>, dim3(grid), dim3(kLanes * W), 0, s, A);
  return grid;
}

// The FAS down pass: one launch over every tile, the wall form chosen by the level's faces.
template <typename T>
void launch_march_fas(MarchArgs A, hipStream_t s) {
  bool per = true, xyper = true;
  for (int f = 0; f < 6; ++f) per = per && A.bc.kind[f] == BC_PERIODIC;
  for (int f = 0; f < 4; ++f) xyper = xyper && A.bc.kind[f] == BC_PERIODIC;
  constexpr int W = cfg_W<T>();
  A.L = ilog2(A.n);
  A.xo = kTX - 2 * kHalo;
  A.yo = kR * 2 * W - 2 * kHalo;
  A.tiles_x = (A.n + A.xo - 1) / A.xo;
  A.tiles_y = (A.n + A.yo - 1) / A.yo;
  A.set = 0;
  A.zc = march_zchunk(A.n, A.tiles_x * A.tiles_y, 5);
  A.ntiles = A.tiles_x * A.tiles_y * ((A.n + A.zc - 1) / A.zc);
  const int grid = (A.ntiles + 7) / 8 * 8;
  if (per) launch_maybe_timed(k_march_fas<T, W, 0>, dim3(grid), dim3(kLanes * W), 0, s, A);
  else if (xyper) launch_maybe_timed(k_march_fas<T, W, 1>, dim3(grid), dim3(kLanes * W), 0, s, A);
  else launch_maybe_timed(k_march_fas<T, W, 2>, dim3(grid), dim3(kLanes * W), 0, s, A);
}

template <typename T>
MarchArgs base_args(const T* uin, T* uout, const T* f, int n, double h, double omega, const LevelBC& bc) {
  MarchArgs A;
  std::memset(&A, 0, sizeof(A));
  A.uin = uin;
  A.uout = uout;
  A.f = f;
  A.bc = bc;
  A.n = n;
  A.h2 = h * h;
  A.ih2 = 1.0 / (h * h);
  A.omega = omega;
  A.zero_in = uin == nullptr;
  return A;
}

}  // namespace

template <typename T>
void march_down(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, double h, double omega, const LevelBC& bc,
                hipStream_t s, int Lm, const MarchAux* aux) {
  MarchArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.fc = fc;
  A.uc0 = uc0;
  A.Lm = Lm;
  if (Lm > 0) launch_march<T, false, false, true>(A, s, aux);
  else launch_march<T, false, false, false>(A, s, aux);
}

template <typename T>
void march_down_fas(const T* uin, T* uout, const T* f, T* fc, T* pbar, T* uc0, int n, double h, double omega,
                    const LevelBC& bc, hipStream_t s) {
  MarchArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.fc = fc;
  A.pbar = pbar;
  A.uc0 = uc0;
  launch_march_fas<T>(A, s);
}

template <typename T>
int march_up(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, double* part, int n, double h,
             double omega, const LevelBC& bc, hipStream_t s, int Lm, const MarchAux* aux) {
  MarchArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.ec = ec;
  A.bcc = bcc;
  A.part = part;
  A.Lm = Lm;
  if (Lm > 0) {
    if (part) return launch_march<T, true, true, true>(A, s, aux);
    launch_march<T, true, false, true>(A, s, aux);
    return 0;
  }
  if (part) return launch_march<T, true, true, false>(A, s, aux);
  launch_march<T, true, false, false>(A, s, aux);
  return 0;
}

template <typename T>
std::string march_fas_name(const LevelBC& bc) {
  bool per = true, xyper = true;
  for (int f = 0; f < 6; ++f) per = per && bc.kind[f] == BC_PERIODIC;
  for (int f = 0; f < 4; ++f) xyper = xyper && bc.kind[f] == BC_PERIODIC;
  return std::string("k_march_fas<") + (sizeof(T) == 8 ? "double" : "float") + ", " + std::to_string(cfg_W<T>()) +
         ", " + std::to_string(per ? 0 : (xyper ? 1 : 2)) + ">";
}

template <typename T>
std::string march_name(bool up, bool norm, const LevelBC& bc, bool blk) {
  auto b = [](bool v) { return std::string(v ? "true" : "false"); };
  bool per = true, xyper = true;
  for (int f = 0; f < 6; ++f) per = per && bc.kind[f] == BC_PERIODIC;
  for (int f = 0; f < 4; ++f) xyper = xyper && bc.kind[f] == BC_PERIODIC;
  const int walls = per ? 0 : (xyper ? 1 : 2);
  return std::string("k_march<") + (sizeof(T) == 8 ? "double" : "float") + ", " + std::to_string(cfg_W<T>()) + ", " +
         b(up) + ", " + b(up && norm) + ", " + std::to_string(walls) + ", " + b(blk) + ">";
}

#ifndef MG_MARCH_T
#error "define MG_MARCH_T (the precision this translation unit instantiates)"
#endif
template void march_down<MG_MARCH_T>(const MG_MARCH_T*, MG_MARCH_T*, const MG_MARCH_T*, MG_MARCH_T*, MG_MARCH_T*, int,
                                     double, double, const LevelBC&, hipStream_t, int, const MarchAux*);
template int march_up<MG_MARCH_T>(const MG_MARCH_T*, MG_MARCH_T*, const MG_MARCH_T*, const MG_MARCH_T*, const LevelBC&,
                                  double*, int, double, double, const LevelBC&, hipStream_t, int, const MarchAux*);
template std::string march_name<MG_MARCH_T>(bool, bool, const LevelBC&, bool);
template std::string march_fas_name<MG_MARCH_T>(const LevelBC&);
template void march_down_fas<MG_MARCH_T>(const MG_MARCH_T*, MG_MARCH_T*, const MG_MARCH_T*, MG_MARCH_T*, MG_MARCH_T*,
                                         MG_MARCH_T*, int, double, double, const LevelBC&, hipStream_t);

}  // namespace mg
