// mg_fused.hip -- fused, z-marching RB-SOR passes for the large levels (bandwidth path).
//
// One launch = one full smoothing sweep (red half-sweep, then black; eqs. rbsor1-2) over the
// level, streamed through registers so u and f cross HBM once per sweep (24 B per cell in
// FP64 instead of 48 for two single-colour launches).  Optional fused stages:
//   PRO : on load, add the trilinear prolongation of the coarse correction (Alg. 1 steps 5-6);
//   OUT=1 (DEF) : after the sweep, the defect f - L u (eq. defect) restricted to the coarse
//         level (eq. restriction; Alg. 1 steps 2-3), and the coarse correction cleared;
//   OUT=2 (NORM): after the sweep, sum of squared defects for the stopping test (Sec. 2.3.7).
//
// Layout of one workgroup (W wavefronts, 64 lanes each): a tile of 128 x (R*W) cells in x-y,
// lane l holding the x-pair (x0+2l, x0+2l+1) of R consecutive rows, or (XS = 2) a tile of
// 64 x (2*R*W) cells with each half-wave on its own band of R rows; the workgroup marches in
// z over a chunk of planes.  Each cell keeps a ring of RING planes of u and f in registers:
// at the step that loads plane P, the red update runs on plane P-1, the black update on P-2
// and the defect on P-3, so every stage reads its z-neighbours in the right colour state.
// x-neighbours across lanes move by DPP wave shifts, y-neighbours across the wave bands
// through a double-buffered LDS exchange (one barrier per stage).  Tiles overlap by a halo of
// `hx` cells (the stages' dependency radius, rounded up to even) and are recomputed, so tiles
// are independent; results go to a separate output array (ping-pong), never in place.
// Boundary ghosts are evaluated on the fly (Sec. 2.3.6) for cells on non-periodic faces.
#include "mg_fused.h"

#include <cstring>
#include <type_traits>

#include "mg_launch.h"

namespace mg {

namespace {

constexpr int kLanes = 64;
constexpr int kTileX = 2 * kLanes;

struct FusedArgs {
  const void* uin;
  void* uout;
  const void* f;
  const void* ec;     // PRO: coarse correction (n/2)^3
  void* fc;           // DEF: coarse source (n/2)^3
  void* uc0;          // DEF: coarse correction to clear (FASDEF: coarse start = restricted u)
  void* pbar;         // FASDEF: restricted u
  double* part;       // NORM: one partial sum per block
  const float* e32;   // MIX: FP32 correction added to u on load
  float* r32;         // MIX: FP32 copy of the defect
  LevelBC bc;         // this level
  LevelBC bcc;        // PRO: coarse level (homogeneous)
  int n, L, hx, hy, xo, yo, zc, tiles_x, tiles_y, chunks_z, ntiles;
  int zero_in;        // u is known to be zero on input: it is not read
  int Lm;             // BLK: log2 of the block side on this level (the coarse level: Lm - 1)
  double h2, ih2, omega;
};

// Whole-wave shift by one lane through DPP (register-speed cross-lane move): wave_shr:1 gives
// lane i the value of lane i-1, wave_shl:1 the value of lane i+1; lanes without a source
// keep their own value.
constexpr int kDppWaveShr1 = 0x138;
constexpr int kDppWaveShl1 = 0x130;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  const int i = __builtin_bit_cast(int, v);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(i, i, CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = (int)(b & 0xffffffffLL), hi = (int)(b >> 32);
  const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi2 << 32) | (long long)(unsigned)lo2);
}
template <typename T>
__device__ __forceinline__ T shfl_from_left(T v) {   // value of lane-1 (lane 0 keeps its own)
  return dpp_move<kDppWaveShr1>(v);
}
template <typename T>
__device__ __forceinline__ T shfl_from_right(T v) {  // value of lane+1 (lane 63 keeps its own)
  return dpp_move<kDppWaveShl1>(v);
}

template <typename T>
__device__ __forceinline__ T ghost_of(const LevelBC& bc, int face, int n, int t1, int t2, T c) {
  if (bc.kind[face] == BC_ZERO_GRADIENT) return c;
  return (T)(2.0 * face_b(bc, face, n, t1, t2)) - c;
}

template <typename T>
__device__ __forceinline__ T coarse_at(const T* __restrict__ e, int nc, int Lc, int Lmc, int X, int Y, int Z,
                                       const LevelBC& bcc) {
  if ((unsigned)X < (unsigned)nc && (unsigned)Y < (unsigned)nc && (unsigned)Z < (unsigned)nc)
    return e[lidx(Lc, Lmc, X, Y, Z)];
  return ghost_any(e, nc, Lc, X, Y, Z, bcc, Lmc);
}

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T a, b;
};

// MODE selects the pass body:
//   MODE_SWEEP : one smoothing sweep, then the OUT stage on the swept u;
//   MODE_MIX   : no sweep, OUT = 2: u = u + e32 on load, written out, then the defect of the
//                updated u, its sum of squares and its FP32 copy -- the FP64 part of one
//                mixed-precision defect-correction step;
//   MODE_FASDEF: MODE_DEF with OUT = 1 for the Full Approximation Scheme (Alg. 3 steps 2-4):
//                besides the restricted defect, the restricted u goes to pbar and to the
//                coarse start uc0;
//   MODE_DEF   : no sweep, u is not written: only the OUT stage on the input u (the defect
//                restricted to the coarse level, or its sum of squares).
//   MODE_SWEEPFAS: one sweep, then the MODE_FASDEF stage on the swept u (the last pre-sweep
//                of a FAS cycle with its restriction).
enum : int { MODE_SWEEP = 0, MODE_MIX = 1, MODE_DEF = 2, MODE_FASDEF = 3, MODE_SWEEPFAS = 4 };

// Tile shape per precision and pass kind: R rows per lane, W waves per workgroup (tile
// 128 x R*W, or 64 x 2*R*W with split waves).  Measured: R = 2, W = 16 for most passes; the
// FP64 passes with the fused restricted defect (one more plane and the most temporaries live,
// ~155 registers) and the FP64 head pass (sweep + input norm, ~165) run 12 waves.  At 512^3
// the fused FP64 sweep + restricted defect takes 0.96 ms with R = 2, W = 12 and split waves,
// 1.28 ms with R = 4, W = 8, against 0.67 + 0.51 ms as a sweep and a defect-only pass.
// Passes without a sweep, and every pass with a norm, use R = 2, W = 16 (four rows per lane
// for the FP32 sweep measured slower: occupancy falls from 7 to 4 waves per SIMD).  The FP32
// prolongation pass (whole-wave tiles, 128 columns) takes four rows per lane on 12 waves: 48
// rows per tile, 0.46 against 0.51 ms at 512^3 (0.093 against 0.096 ms at 256^3).
template <typename T, bool PRO, int OUT, int MODE>
constexpr int cfg_R() {
  if (sizeof(T) == 4 && PRO) return 4;
  return 2;
}
template <typename T, bool PRO, int OUT, int MODE>
constexpr int cfg_W() {
  if (MODE != MODE_SWEEP && MODE != MODE_SWEEPFAS) return 16;
  if (sizeof(T) == 8 && (OUT == 1 || OUT == 3)) return 12;
  if (sizeof(T) == 4 && PRO) return 12;
  return 16;
}
// x-segments per wave: 1 = a wave spans the tile's 128 columns; 2 = each half-wave spans 64
// columns of its own band of R rows (tile 64 x 2RW: for the same cells per workgroup, a
// squarer tile re-reads fewer halo cells).  Measured at 512^3 with the chunking below: the
// sweep + input norm 0.89 -> 0.77 ms, the restricted defect 0.53 -> 0.51 ms, the FP32 sweep
// 0.40 -> 0.38 ms, the FP64 sweep unchanged.  The passes that would spill registers with
// the extra per-lane addressing (prolongation, the sweep + norm) keep 1.
template <typename T, bool PRO, int OUT, int MODE>
constexpr int cfg_XS() {
  if (PRO || (MODE == MODE_SWEEP && OUT == 2)) return 1;
  return 2;
}

// BLK: the level is in the MeshBlock layout (blocks of 2^A.Lm cells, Morton order); the tile
// streams across block boundaries exactly as across a dense array (an x-pair never straddles
// two blocks), and the coarse level is in the layout below it (blocks of 2^(A.Lm-1) cells, or
// the dense root grid when that is one cell).
template <typename T, int R, int W, bool PRO, int OUT, int MODE = MODE_SWEEP, bool BLK = false, int XS = 1>
__global__ void __launch_bounds__(kLanes* W) k_fused(FusedArgs A) {
  // XS = 2: the two halves of a wave hold two row bands; the colour of a lane's cells stays
  // wave-uniform because the bands are R (even) rows apart
  static_assert(XS == 1 || (XS == 2 && R % 2 == 0), "x-segments: 1, or 2 with an even row count");
  constexpr int SL = kLanes / XS;      // lanes per x-segment
  constexpr int TX = 2 * SL;           // tile width
  constexpr int NBAND = W * XS;        // row bands of R rows
  constexpr bool SWEEP = MODE == MODE_SWEEP || MODE == MODE_SWEEPFAS;
  constexpr bool MIX = MODE == MODE_MIX;
  constexpr bool WRITE_U = SWEEP || MODE == MODE_MIX;
  constexpr bool FASR = MODE == MODE_FASDEF || MODE == MODE_SWEEPFAS;
  static_assert(!FASR || OUT == 1, "the FAS restriction rides on the restricted-defect stage");
  // OUT = 3 (with a sweep): the sum of squared defects of the INPUT u, taken in the red stage
  // before it updates the plane (no defect stage behind the sweep)
  constexpr bool INNORM = SWEEP && OUT == 3;
  constexpr bool DSTAGE = OUT == 1 || OUT == 2;
  constexpr int DLAG = SWEEP ? 3 : 1;                  // the defect runs on plane P - DLAG
  constexpr int HZ = DSTAGE ? DLAG : 2;                // z planes loaded ahead of the chunk
  constexpr int kRing = DSTAGE ? DLAG + 2 : 4;         // u planes alive
  __shared__ Pair<T> xch[2][NBAND][2][SL];
  // f of planes P-1, P-2, P-3 for this thread's cells: private per thread (f is only read at
  // the cell itself), kept in LDS to leave the registers to the u ring
  // (a sweep without a defect stage needs f of P-1 and P-2 only)
  constexpr int NF = DSTAGE ? 3 : 2;
  // where the final plane is stored: after the end-of-step ring update for the FP64 passes
  // with the prolongation or the input norm (measured 2-4 % faster there, slower elsewhere)
  constexpr bool STORE_LAST = sizeof(T) == 8 && SWEEP && !DSTAGE && (PRO || OUT == 3);
  // leave out the stages that feed no output: planes before the chunk and halo-only waves
  // (measured 6 % faster on the FP64 sweep with the restricted defect and 11 % on the FP32
  // sweep at 512^3; 1-17 % slower on the other passes, where the compiler then schedules the
  // march worse)
  constexpr bool SKIP = (sizeof(T) == 8 && SWEEP && OUT == 1) || (sizeof(T) == 4 && MODE == MODE_SWEEP && !PRO && OUT == 0);
  __shared__ Pair<T> fl[NF][R][W * kLanes];
  // INNORM: input values of plane P-2, private per thread like f
  __shared__ Pair<T> uol[INNORM ? R : 1][INNORM ? W * kLanes : 1];

  const int lane = threadIdx.x & (kLanes - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int seg = XS == 1 ? 0 : lane / SL;
  const int xl = lane - seg * SL;        // lane within the x-segment
  const int band = w * XS + seg;
  const int tid = threadIdx.x;
  // XCD-aware order: consecutive block ids go to different XCDs, so give each XCD a
  // contiguous run of tiles (neighbouring tiles then share that XCD's L2 for their halos).
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  const int tile = (bid & 7) * (nb >> 3) + (bid >> 3);
  double acc = 0.0;
  if (tile < A.ntiles) {
    const int tx = tile % A.tiles_x;
    const int ty = (tile / A.tiles_x) % A.tiles_y;
    const int cz = tile / (A.tiles_x * A.tiles_y);
    const int n = A.n, L = A.L, nm = n - 1;
    const T* __restrict__ uin = reinterpret_cast<const T*>(A.uin);
    T* __restrict__ uout = reinterpret_cast<T*>(A.uout);
    const T* __restrict__ fin = reinterpret_cast<const T*>(A.f);
    // storage index of cell (x, y, z) of this level
    auto fidx = [&](int x, int y, int z) __attribute__((always_inline)) {
      return BLK ? bidx(A.Lm, x, y, z) : cidx(L, x, y, z);
    };
    const bool px = A.bc.kind[0] == BC_PERIODIC;
    const bool py = A.bc.kind[2] == BC_PERIODIC;
    const bool pz = A.bc.kind[4] == BC_PERIODIC;
    const T h2 = (T)A.h2, ih2 = (T)A.ih2, omega = (T)A.omega;
    const T inv6 = (T)(1.0 / 6.0);

    const int xs = tx * A.xo;                     // first output column
    const int xa = xs - A.hx + 2 * xl;            // this lane's even column
    const bool in_x = px || (xa >= 0 && xa < n);
    const int xag = xa & nm;
    const bool out_x = xa >= xs && xa < xs + A.xo && xa < n;
    const bool bnd_xl = !px && xa == 0;           // cell a on the -x face
    const bool bnd_xr = !px && xa + 1 == nm;      // cell b on the +x face

    const int ys = ty * A.yo;
    int yv[R], ygv[R];
    bool in_y[R], out_y[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = ys - A.hy + band * R + r;
      yv[r] = y;
      ygv[r] = y & nm;
      in_y[r] = py || (y >= 0 && y < n);
      out_y[r] = y >= ys && y < ys + A.yo && y < n;
    }
    const int z0 = cz * A.zc;
    const int zend = min(z0 + A.zc, n);
    const int zstart = z0 - HZ;
    const int nsteps = (zend - z0) + 2 * HZ;
    // does any cell of this wave touch a non-periodic face in x or y?
    const int wy0 = ys - A.hy + w * XS * R, wy1 = wy0 + XS * R - 1;   // rows of the whole wave
    const bool wave_bnd_xy = (!px && (xs - A.hx <= 0 || xs - A.hx + TX - 1 >= nm)) ||
                             (!py && (wy0 <= 0 || wy1 >= nm));
    // does this wave hold an output row?  (with SKIP a wave of halo rows leaves out the
    // defect stage)
    const bool wave_out = wy1 >= ys && wy0 < min(ys + A.yo, n);

    // u: ring of kRing planes (slot = plane index mod kRing, compile-time after unrolling);
    // f: LDS slots (plane mod 3) holding planes P-1, P-2, P-3.
    T u[kRing][R][2];
    T pu[R][2], pf[R][2];
    T pc[PRO ? R / 2 : 1][3][2];   // PRO: coarse taps (rows Y-1..Y+1, planes zlo, zlo+1) of the next plane
#pragma unroll
    for (int r = 0; r < (INNORM ? R : 0); ++r) uol[r][tid] = Pair<T>{(T)0, (T)0};
    T stash[R / 2 > 0 ? R / 2 : 1];
    T stash_u[FASR && R / 2 > 0 ? R / 2 : 1];   // FASDEF: restricted u of the even plane
#pragma unroll
    for (int s = 0; s < kRing; ++s)
#pragma unroll
      for (int r = 0; r < R; ++r) u[s][r][0] = u[s][r][1] = (T)0;
    auto fslot = [&](int p) __attribute__((always_inline)) { return ((p % NF) + NF) % NF; };
    auto fget = [&](int p, int r, int q) __attribute__((always_inline)) {
      const Pair<T> v = fl[fslot(p)][r][tid];
      return q ? v.b : v.a;
    };
#pragma unroll
    for (int q = 0; q < (R / 2 > 0 ? R / 2 : 1); ++q) stash[q] = (T)0;

    // ---- load of u on plane P (with the prolonged coarse correction added) and f on P-1
    auto load_plane = [&](int P, bool first) __attribute__((always_inline)) {
      const bool in_z = pz || (P >= 0 && P < n);
      const bool in_zf = pz || (P - 1 >= 0 && P - 1 < n);
      const int Pg = P & nm, Pfg = (P - 1) & nm;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (in_x && in_y[r] && in_z) {
          const size_t off = fidx(xag, ygv[r], Pg);
          if (A.zero_in) {
            pu[r][0] = pu[r][1] = (T)0;
          } else {
            const Pair<T> vu = *reinterpret_cast<const Pair<T>*>(uin + off);
            pu[r][0] = vu.a; pu[r][1] = vu.b;
          }
          if (MIX) {
            const float2 ve = *reinterpret_cast<const float2*>(A.e32 + off);
            pu[r][0] += (T)ve.x;
            pu[r][1] += (T)ve.y;
          }
        } else {
          pu[r][0] = pu[r][1] = (T)0;
        }
        if (in_x && in_y[r] && in_zf) {
          const size_t off = fidx(xag, ygv[r], Pfg);
          const Pair<T> vf = *reinterpret_cast<const Pair<T>*>(fin + off);
          pf[r][0] = vf.a; pf[r][1] = vf.b;
        } else {
          pf[r][0] = pf[r][1] = (T)0;
        }
      }
      if (PRO) {
        // Trilinear prolongation (weights 1/4, 3/4 per axis) of the coarse correction.  Rows
        // come in aligned pairs (2Y, 2Y+1) sharing coarse rows Y-1, Y, Y+1; the lane's coarse
        // column X is interpolated in y and z, and its x-neighbours come from lanes -+1.  Only
        // the loads are issued here; prolong_apply adds the correction when the plane enters
        // the ring, so the loads are in flight during the step like the u and f prefetch.
        // Fine plane 2Z takes coarse planes (Z-1, Z), plane 2Z+1 (Z, Z+1): an even plane
        // reuses the taps of the odd plane before it, an odd plane keeps its predecessor's
        // upper plane as its lower one and loads one new plane (the first plane of the
        // march loads both).
        const T* __restrict__ ec = reinterpret_cast<const T*>(A.ec);
        const int nc = n >> 1, Lc = L - 1, Lmc = BLK ? A.Lm - 1 : 0;
        const int X = (px ? xag : xa) >> 1;
        const int Pz = pz ? Pg : P;
        const int Z = Pz >> 1;
        const int zlo = (Pz & 1) ? Z : Z - 1;          // taps (zlo, zlo+1)
        if (first || (P & 1)) {
#pragma unroll
          for (int q2 = 0; q2 < R / 2; ++q2) {
            const int Y = (py ? ygv[2 * q2] : yv[2 * q2]) >> 1;   // the pair's coarse row
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
              pc[q2][dy][0] = first ? coarse_at(ec, nc, Lc, Lmc, X, Y - 1 + dy, zlo, A.bcc) : pc[q2][dy][1];
              pc[q2][dy][1] = coarse_at(ec, nc, Lc, Lmc, X, Y - 1 + dy, zlo + 1, A.bcc);
            }
          }
        }
      }
    };

    // ---- add the prolonged correction fetched with plane P to the prefetched u of P
    auto prolong_apply = [&](int P) __attribute__((always_inline)) {
      if (!PRO) return;
      const bool in_z = pz || (P >= 0 && P < n);
      const int Pz = pz ? (P & nm) : P;
      const T wz0 = (Pz & 1) ? (T)0.75 : (T)0.25, wz1 = (Pz & 1) ? (T)0.25 : (T)0.75;
#pragma unroll
      for (int q2 = 0; q2 < R / 2; ++q2) {
        T cz[3];
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) cz[dy] = wz0 * pc[q2][dy][0] + wz1 * pc[q2][dy][1];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
          const int r = 2 * q2 + rr;
          const T c = rr ? (T)0.75 * cz[1] + (T)0.25 * cz[2] : (T)0.25 * cz[0] + (T)0.75 * cz[1];
          // the edge lanes 0 and 63 get their own value back: wrong, but within the halo
          const T cl = shfl_from_left(c), cr = shfl_from_right(c);
          if (in_x && in_y[r] && in_z) {
            pu[r][0] += (T)0.25 * cl + (T)0.75 * c;
            pu[r][1] += (T)0.75 * c + (T)0.25 * cr;
          }
        }
      }
    };

    // ---- exchange of the band-edge rows of one plane between the wave bands
    int xbuf = 0;
    auto exchange = [&](const T (&pl)[R][2], T (&below)[2], T (&above)[2]) __attribute__((always_inline)) {
      xch[xbuf][band][0][xl] = Pair<T>{pl[0][0], pl[0][1]};
      xch[xbuf][band][1][xl] = Pair<T>{pl[R - 1][0], pl[R - 1][1]};
      __syncthreads();
      const Pair<T> vb = xch[xbuf][band > 0 ? band - 1 : band][1][xl];
      const Pair<T> va = xch[xbuf][band < NBAND - 1 ? band + 1 : band][0][xl];
      below[0] = vb.a; below[1] = vb.b;
      above[0] = va.a; above[1] = va.b;
      xbuf ^= 1;
    };

    // ---- one colour of the RB-SOR update (eqs. rbsor1-2) on plane p held in pc, its
    // z-neighbour planes in pm (p-1) and pp (p+1)
    auto half_sweep = [&](T (&pm)[R][2], T (&pc)[R][2], T (&pp)[R][2], int p,
                          int colour) __attribute__((always_inline)) {
      T below[2], above[2];
      exchange(pc, below, above);
      const bool in_z = pz || (p >= 0 && p < n);
      const bool bnd_z0 = !pz && p == 0, bnd_z1 = !pz && p == nm;
      const bool out_zn = INNORM && p >= z0 && p < zend;
      if (INNORM && colour == 0) {
        // defect of the input on plane p, black cells (the red cells' comes with their update
        // below, whose neighbour sum is the input's): pc, below/above and pp still hold input
        // values (the red update of p comes next, p+1 was only just loaded); a black cell's
        // z-neighbour below is red and already updated, so its input value comes from uol
        const int qr = __builtin_amdgcn_readfirstlane((yv[0] + p) & 1);
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int q = ((qr + r) & 1) ^ 1;   // the black cell of the pair (wave-uniform)
          const T ca = pc[r][0], cb = pc[r][1];
          const T c = q ? cb : ca;
          const T la = shfl_from_left(cb), rb = shfl_from_right(ca);
          T xm = q ? ca : la;
          T xp = q ? rb : cb;
          T ym = r > 0 ? (q ? pc[r - 1][1] : pc[r - 1][0]) : (q ? below[1] : below[0]);
          T yp = r < R - 1 ? (q ? pc[r + 1][1] : pc[r + 1][0]) : (q ? above[1] : above[0]);
          const Pair<T> zo = uol[r][tid];
          T zm = q ? zo.b : zo.a;
          T zp = q ? pp[r][1] : pp[r][0];
          if ((wave_bnd_xy || bnd_z0 || bnd_z1) && in_x && in_y[r] && in_z) {
            const int xw = xag + q, yw = ygv[r], pw = p & nm;
            if (q == 0 && bnd_xl) xm = ghost_of(A.bc, 0, n, yw, pw, c);
            if (q == 1 && bnd_xr) xp = ghost_of(A.bc, 1, n, yw, pw, c);
            if (!py && yv[r] == 0) ym = ghost_of(A.bc, 2, n, xw, pw, c);
            if (!py && yv[r] == nm) yp = ghost_of(A.bc, 3, n, xw, pw, c);
            if (bnd_z0) zm = ghost_of(A.bc, 4, n, xw, yw, c);
            if (bnd_z1) zp = ghost_of(A.bc, 5, n, xw, yw, c);
          }
          const T nbs = ((((xm + xp) + ym) + yp) + zm) + zp;
          const T d = fget(p, r, q) - (nbs - (T)6 * c) * ih2;
          if (out_zn && out_x && out_y[r]) acc += (double)d * (double)d;
          uol[r][tid] = Pair<T>{ca, cb};
        }
      }
      // 0: the even column of row 0 has this colour (the same for every lane of the wave)
      const int q0 = __builtin_amdgcn_readfirstlane((yv[0] + p + colour) & 1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int q = (q0 + r) & 1;                  // wave-uniform
        const T ca = pc[r][0], cb = pc[r][1];
        const T c = q ? cb : ca;
        // the cross-lane x neighbour: lane-1's odd column or lane+1's even column
        const T xo_l = shfl_from_left(cb), xo_r = shfl_from_right(ca);
        T xm = q ? ca : xo_l;
        T xp = q ? xo_r : cb;
        T ym = r > 0 ? (q ? pc[r - 1][1] : pc[r - 1][0]) : (q ? below[1] : below[0]);
        T yp = r < R - 1 ? (q ? pc[r + 1][1] : pc[r + 1][0]) : (q ? above[1] : above[0]);
        T zm = q ? pm[r][1] : pm[r][0];
        T zp = q ? pp[r][1] : pp[r][0];
        if ((wave_bnd_xy || bnd_z0 || bnd_z1) && in_x && in_y[r] && in_z) {
          // face-array coordinates in [0, n): wrapped on periodic axes, in range otherwise
          const int xw = xag + q, yw = ygv[r], pw = p & nm;
          if (q == 0 && bnd_xl) xm = ghost_of(A.bc, 0, n, yw, pw, c);
          if (q == 1 && bnd_xr) xp = ghost_of(A.bc, 1, n, yw, pw, c);
          if (!py && yv[r] == 0) ym = ghost_of(A.bc, 2, n, xw, pw, c);
          if (!py && yv[r] == nm) yp = ghost_of(A.bc, 3, n, xw, pw, c);
          if (bnd_z0) zm = ghost_of(A.bc, 4, n, xw, yw, c);
          if (bnd_z1) zp = ghost_of(A.bc, 5, n, xw, yw, c);
        }
        const T fv = fget(p, r, q);
        const T nbs = ((((xm + xp) + ym) + yp) + zm) + zp;
        if (INNORM && colour == 0) {
          // the red cell's input defect: every neighbour of a red cell is black, still input
          const T d = fv - (nbs - (T)6 * c) * ih2;
          if (out_zn && out_x && out_y[r]) acc += (double)d * (double)d;
        }
        const T nv = c + omega * ((nbs - h2 * fv) * inv6 - c);
        pc[r][0] = q ? ca : nv;
        pc[r][1] = q ? nv : cb;
      }
    };

    // ---- defect of both columns on plane p; restriction (DEF) or sum of squares (NORM)
    auto defect_out = [&](T (&pm)[R][2], T (&pc)[R][2], T (&pp)[R][2], int p) __attribute__((always_inline)) {
      T below[2], above[2];
      exchange(pc, below, above);
      if (SKIP && !wave_out) return;   // wave-uniform, after the barrier
      const bool in_z = pz || (p >= 0 && p < n);
      const bool bnd_z0 = !pz && p == 0, bnd_z1 = !pz && p == nm;
      const bool out_z = p >= z0 && p < zend;
      // defect of both columns of row r (eq. defect)
      auto row_defect = [&](int r, T (&d)[2]) __attribute__((always_inline)) {
        const T ca = pc[r][0], cb = pc[r][1];
        const T la = shfl_from_left(cb), rb = shfl_from_right(ca);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const T c = q ? cb : ca;
          T xm = q ? ca : la;
          T xp = q ? rb : cb;
          T ym = r > 0 ? pc[r - 1][q] : below[q];
          T yp = r < R - 1 ? pc[r + 1][q] : above[q];
          T zm = pm[r][q], zp = pp[r][q];
          if ((wave_bnd_xy || bnd_z0 || bnd_z1) && in_x && in_y[r] && in_z) {
            const int xw = xag + q, yw = ygv[r], pw = p & nm;
            if (q == 0 && bnd_xl) xm = ghost_of(A.bc, 0, n, yw, pw, c);
            if (q == 1 && bnd_xr) xp = ghost_of(A.bc, 1, n, yw, pw, c);
            if (!py && yv[r] == 0) ym = ghost_of(A.bc, 2, n, xw, pw, c);
            if (!py && yv[r] == nm) yp = ghost_of(A.bc, 3, n, xw, pw, c);
            if (bnd_z0) zm = ghost_of(A.bc, 4, n, xw, yw, c);
            if (bnd_z1) zp = ghost_of(A.bc, 5, n, xw, yw, c);
          }
          const T nbs = ((((xm + xp) + ym) + yp) + zm) + zp;
          d[q] = fget(p, r, q) - (nbs - (T)6 * c) * ih2;
        }
      };
      if (OUT == 2) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          T d[2];
          row_defect(r, d);
          if (out_z && out_x && out_y[r]) {
            acc += (double)d[0] * (double)d[0] + (double)d[1] * (double)d[1];
            if (MIX || (MODE == MODE_DEF && A.r32)) {
              const size_t off = fidx(xag, ygv[r], p & nm);
              *reinterpret_cast<float2*>(A.r32 + off) = make_float2((float)d[0], (float)d[1]);
            }
          }
        }
      } else if (OUT == 1) {
        T* __restrict__ fcp = reinterpret_cast<T*>(A.fc);
        T* __restrict__ ucp = reinterpret_cast<T*>(A.uc0);
        T* __restrict__ pbp = reinterpret_cast<T*>(A.pbar);
        const int pg = pz ? (p & nm) : p;
#pragma unroll
        for (int q2 = 0; q2 < R / 2; ++q2) {
          T d0[2], d1[2];
          row_defect(2 * q2, d0);
          row_defect(2 * q2 + 1, d1);
          const T s = (d0[0] + d0[1]) + (d1[0] + d1[1]);
          const T su = FASR ? (pc[2 * q2][0] + pc[2 * q2][1]) + (pc[2 * q2 + 1][0] + pc[2 * q2 + 1][1]) : (T)0;
          if ((pg & 1) == 0) {
            stash[q2] = s;
            if (FASR) stash_u[q2] = su;
          } else if (out_z && out_x && out_y[2 * q2]) {
            const int Lc = L - 1;
            const size_t ci = lidx(Lc, BLK ? A.Lm - 1 : 0, xag >> 1, ygv[2 * q2] >> 1, pg >> 1);
            fcp[ci] = (stash[q2] + s) * (T)0.125;
            if (FASR) {
              const T pb = (stash_u[q2] + su) * (T)0.125;
              pbp[ci] = pb;
              ucp[ci] = pb;
            } else {
              ucp[ci] = (T)0;
            }
          }
        }
      }
    };

    load_plane(zstart, true);
    prolong_apply(zstart);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      u[0][r][0] = pu[r][0]; u[0][r][1] = pu[r][1];
      fl[fslot(zstart - 1)][r][tid] = Pair<T>{pf[r][0], pf[r][1]};
    }
    // one pipeline step; K = t mod kRing is a compile-time constant so every ring slot is a
    // fixed register set
    auto step = [&](int g, auto kk) __attribute__((always_inline)) {
      constexpr int k = decltype(kk)::value;
      const int t = g + k;
      if (t >= nsteps) return;
      const int P = zstart + t;                  // plane held in slot k
      if (t + 1 < nsteps) load_plane(P + 1, false);   // prefetch; consumed at the end of the step
      constexpr int s1 = (k + kRing - 1) % kRing, s2 = (k + kRing - 2) % kRing;
      constexpr int s3 = (k + 2 * kRing - 3) % kRing, s4 = (k + 2 * kRing - 4) % kRing;
      // red on P-1 (neighbours P-2, P), black on P-2 (P-3, P-1), defect on P-3 (P-4, P-2);
      // without the sweep the (updated) plane P is final at once and the defect runs on P-1.
      // A stage runs only on planes that reach an output plane of the chunk: the defect on
      // planes >= z0, the black colour on planes >= z0 - 1 (>= z0 without a defect stage),
      // the red one plane further out (the same for the whole workgroup, barriers included)
      constexpr int kRedLo = DSTAGE ? 2 : 1, kBlackLo = DSTAGE ? 1 : 0;
      if (SWEEP) {
        if (!SKIP || P - 1 >= z0 - kRedLo) half_sweep(u[s2], u[s1], u[k], P - 1, 0);
        if (!SKIP || P - 2 >= z0 - kBlackLo) half_sweep(u[s3], u[s2], u[s1], P - 2, 1);
      }
      // the plane that is final this step goes out (ring slot sf)
      constexpr int sf = SWEEP ? s2 : k;
      auto store_final = [&]() __attribute__((always_inline)) {
        const int p = SWEEP ? P - 2 : P;
        if (p >= z0 && p < zend && out_x) {
          const int pg = p & nm;
#pragma unroll
          for (int r = 0; r < R; ++r)
            if (out_y[r]) {
              const size_t off = fidx(xag, ygv[r], pg);
              // nontemporal: the next pass over this level comes long after the caches have
              // turned over (measured 4 % faster on the FP64 sweep at 512^3)
              typedef T ntv2 __attribute__((ext_vector_type(2)));
              const ntv2 v = {u[sf][r][0], u[sf][r][1]};
              __builtin_nontemporal_store(v, reinterpret_cast<ntv2*>(uout + off));
            }
        }
      };
      if (WRITE_U && !STORE_LAST) store_final();
      if (DSTAGE) {
        if (SWEEP) {
          if (!SKIP || P - 3 >= z0) defect_out(u[s4], u[s3], u[s2], P - 3);
        } else if (!SKIP || P - 1 >= z0) {
          defect_out(u[s2], u[s1], u[k], P - 1);
        }
      }
      if (t + 1 < nsteps) {
        prolong_apply(P + 1);
        constexpr int sn = (k + 1) % kRing;
        // f(P) replaces f(P-3), which this thread's defect stage has finished reading
#pragma unroll
        for (int r = 0; r < R; ++r) {
          u[sn][r][0] = pu[r][0]; u[sn][r][1] = pu[r][1];
          fl[fslot(P)][r][tid] = Pair<T>{pf[r][0], pf[r][1]};
        }
      }
      // STORE_LAST: after the prefetched plane has entered the ring (sn is never sf), so the
      // wait for the prefetch does not cover these stores
      if (WRITE_U && STORE_LAST) store_final();
    };
    for (int g = 0; g < nsteps; g += kRing) {
      step(g, std::integral_constant<int, 0>{});
      step(g, std::integral_constant<int, 1>{});
      step(g, std::integral_constant<int, 2>{});
      if (kRing > 3) step(g, std::integral_constant<int, 3 % kRing>{});
      if (kRing > 4) step(g, std::integral_constant<int, 4 % kRing>{});
    }
  }
  if (OUT == 2 || OUT == 3) {
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

constexpr int kCUs = 256;

// Planes per workgroup (even, so restriction plane pairs never straddle two chunks).  One
// workgroup per CU is resident (LDS bound), so the grid runs in rounds of kCUs workgroups;
// the chunk count minimises (rounds) x (planes a workgroup marches, its 2 hz halo planes
// included).  At 512^3 this gives the 64 x 64 tiles one round of 3 chunks: the FP64 sweep
// takes 0.665 ms, against 0.77 ms with fixed 64-plane chunks (2.5 rounds).
int zchunk_for(int n, int tiles_xy, int hz) {
  if (n < 256) return min(16, n);
  int best = n;
  long best_cost = -1;
  for (int c = 1; c <= n / 16; ++c) {
    int zc = (n + c - 1) / c;
    zc += zc & 1;
    const long chunks = (n + zc - 1) / zc;
    // a norm pass writes one partial sum per workgroup: stay within the partials buffer
    if ((long)tiles_xy * chunks > (long)kMaxPartials * 32 - 8) continue;
    const long rounds = ((long)tiles_xy * chunks + kCUs - 1) / kCUs;
    const long cost = rounds * (zc + 2 * hz);
    if (best_cost < 0 || cost < best_cost) best_cost = cost, best = zc;
  }
  return best;
}

// Launches one pass; returns its grid size (the number of partial sums a norm pass writes).
template <typename T, bool PRO, int OUT, int MODE = MODE_SWEEP, bool BLK = false>
int launch_pass(FusedArgs A, hipStream_t s) {
  constexpr int R = cfg_R<T, PRO, OUT, MODE>(), W = cfg_W<T, PRO, OUT, MODE>();
  constexpr int XS = cfg_XS<T, PRO, OUT, MODE>();
  constexpr bool DSTAGE = OUT == 1 || OUT == 2;
  constexpr int HZ = DSTAGE ? (MODE == MODE_SWEEP || MODE == MODE_SWEEPFAS ? 3 : 1) : 2;   // the kernel's z halo
  A.xo = kTileX / XS - 2 * A.hx;
  A.yo = R * W * XS - 2 * A.hy;
  A.tiles_x = (A.n + A.xo - 1) / A.xo;
  A.tiles_y = (A.n + A.yo - 1) / A.yo;
  A.zc = zchunk_for(A.n, A.tiles_x * A.tiles_y, HZ);
  A.chunks_z = (A.n + A.zc - 1) / A.zc;
  A.ntiles = A.tiles_x * A.tiles_y * A.chunks_z;
  const int grid = (A.ntiles + 7) / 8 * 8;
  hipLaunchKernelGGL((k_fused<T, R, W, PRO, OUT, MODE, BLK, XS>), dim3(grid), dim3(kLanes * W), 0, s, A);
  return grid;
}

template <typename T>
FusedArgs base_args(const T* uin, T* uout, const T* f, int n, double h, double omega, const LevelBC& bc) {
  FusedArgs A;
  std::memset(&A, 0, sizeof(A));
  A.uin = uin;
  A.uout = uout;
  A.f = f;
  A.bc = bc;
  A.n = n;
  A.L = ilog2(n);
  A.h2 = h * h;
  A.ih2 = 1.0 / (h * h);
  A.omega = omega;
  return A;
}

}  // namespace

template <typename T>
bool fused_supported(int n) {
  return n >= kFusedMinN;
}

template <typename T>
void fused_sweep(const T* uin, T* uout, const T* f, int n, double h, double omega, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.zero_in = uin == nullptr;
  A.hx = 2;   // dependency radius of one sweep
  A.hy = 2;
  launch_pass<T, false, 0>(A, s);
}

template <typename T>
void fused_sweep_defect(const T* uin, T* uout, const T* f, T* fc, T* uc0, int n, double h, double omega,
                        const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.hx = 4;   // sweep (2) + defect (1), rounded up to even: restriction pairs align
  A.hy = 4;
  A.fc = fc;
  A.uc0 = uc0;
  launch_pass<T, false, 1>(A, s);
}

template <typename T>
void fused_prolong_sweep(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int n, double h,
                         double omega, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  // the prolongation of an edge lane lacks one coarse column, so the dependency radius of
  // this pass is 3 (2 for the sweep + 1); the halo is rounded up to even
  A.hx = 4;
  A.hy = 2;   // along y a row's prolongation needs no other row
  A.ec = ec;
  A.bcc = bcc;
  launch_pass<T, true, 0>(A, s);
}

template <typename T>
int fused_sweep_norm(const T* uin, T* uout, const T* f, double* part, int n, double h, double omega, const LevelBC& bc,
                     hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.hx = 4;   // sweep (2) + defect (1); even in x so lane pairs start on even columns
  A.hy = 3;
  A.part = part;
  return launch_pass<T, false, 2>(A, s);
}

template <typename T>
int fused_sweep_input_norm(const T* uin, T* uout, const T* f, double* part, int n, double h, double omega,
                           const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.hx = 2;   // the input defect's radius (1) is inside the sweep's
  A.hy = 2;
  A.part = part;
  return launch_pass<T, false, 3>(A, s);   // one partial per workgroup
}

int fused_mixed_update_defect(double* phi_in, double* phi_out, const float* e, const double* f, float* r32,
                              double* part, int n, double h, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args<double>(phi_in, phi_out, f, n, h, 1.0, bc);
  A.hx = 2;   // defect only: radius 1, rounded up to even
  A.hy = 1;
  A.part = part;
  A.e32 = e;
  A.r32 = r32;
  return launch_pass<double, false, 2, MODE_MIX>(A, s);
}

template <typename T>
void fused_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int n, double h, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(u, (T*)nullptr, f, n, h, 1.0, bc);
  A.hx = 2;   // defect only: radius 1, rounded up to even
  A.hy = 2;   // even, so that restriction row pairs align
  A.fc = fc;
  A.uc0 = uc0;
  launch_pass<T, false, 1, MODE_DEF>(A, s);
}

void fused_fas_restrict(const double* u, const double* f, double* fc, double* pbar, double* uc, int n, double h,
                        const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(u, (double*)nullptr, f, n, h, 1.0, bc);
  A.hx = 2;   // defect only: radius 1, rounded up to even
  A.hy = 2;   // even, so that restriction row pairs align
  A.fc = fc;
  A.uc0 = uc;
  A.pbar = pbar;
  launch_pass<double, false, 1, MODE_FASDEF>(A, s);
}

void fused_sweep_fas_restrict(const double* uin, double* uout, const double* f, double* fc, double* pbar, double* uc,
                              int n, double h, double omega, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, n, h, omega, bc);
  A.hx = 4;   // sweep (2) + defect (1), rounded up to even: restriction pairs align
  A.hy = 4;
  A.fc = fc;
  A.uc0 = uc;
  A.pbar = pbar;
  launch_pass<double, false, 1, MODE_SWEEPFAS>(A, s);
}

template <typename T>
int fused_defect_norm(const T* u, const T* f, double* part, int n, double h, const LevelBC& bc, hipStream_t s,
                      float* r32) {
  FusedArgs A = base_args(u, (T*)nullptr, f, n, h, 1.0, bc);
  A.hx = 2;
  A.hy = 1;
  A.part = part;
  A.r32 = r32;
  return launch_pass<T, false, 2, MODE_DEF>(A, s);
}

// ---- the same passes on a MeshBlock-layout level (blocks of 2^Lm cells, 2^Lb per side)

template <typename T>
void fused_blk_sweep(const T* uin, T* uout, const T* f, const T* ec, const LevelBC& bcc, int Lm, int Lb, double h,
                     double omega, const LevelBC& bc, hipStream_t s) {
  FusedArgs A = base_args(uin, uout, f, 1 << (Lm + Lb), h, omega, bc);
  A.Lm = Lm;
  A.hy = 2;
  if (ec) {
    A.hx = 4;
    A.ec = ec;
    A.bcc = bcc;
    launch_pass<T, true, 0, MODE_SWEEP, true>(A, s);
  } else {
    A.hx = 2;
    launch_pass<T, false, 0, MODE_SWEEP, true>(A, s);
  }
}

template <typename T>
void fused_blk_defect_restrict(const T* u, const T* f, T* fc, T* uc0, int Lm, int Lb, double h, const LevelBC& bc,
                               hipStream_t s) {
  FusedArgs A = base_args(u, (T*)nullptr, f, 1 << (Lm + Lb), h, 1.0, bc);
  A.Lm = Lm;
  A.hx = 2;
  A.hy = 2;
  A.fc = fc;
  A.uc0 = uc0;
  launch_pass<T, false, 1, MODE_DEF, true>(A, s);
}

template <typename T>
int fused_blk_defect_norm(const T* u, const T* f, double* part, int Lm, int Lb, double h, const LevelBC& bc,
                          hipStream_t s, float* r32) {
  const int n = 1 << (Lm + Lb);
  FusedArgs A = base_args(u, (T*)nullptr, f, n, h, 1.0, bc);
  A.Lm = Lm;
  A.hx = 2;
  A.hy = 1;
  A.part = part;
  A.r32 = r32;
  return launch_pass<T, false, 2, MODE_DEF, true>(A, s);
}

// The kernel name as the profiler lists it.
template <typename T, bool PRO, int OUT, int MODE, bool BLK>
std::string kname() {
  auto b = [](bool v) { return std::string(v ? "true" : "false"); };
  return std::string("k_fused<") + (sizeof(T) == 8 ? "double" : "float") + ", " +
         std::to_string(cfg_R<T, PRO, OUT, MODE>()) + ", " + std::to_string(cfg_W<T, PRO, OUT, MODE>()) + ", " +
         b(PRO) + ", " + std::to_string(OUT) + ", " + std::to_string(MODE) + ", " + b(BLK) + ", " +
         std::to_string(cfg_XS<T, PRO, OUT, MODE>()) + ">";
}

template <typename T>
std::string fused_blk_pass_name(bool pro, int out) {
  // the block passes: plain or prolonging sweeps, and the defect-only restricted defect
  if (out == 1) return kname<T, false, 1, MODE_DEF, true>();
  if (out == 2) return kname<T, false, 2, MODE_DEF, true>();
  if (pro) return kname<T, true, 0, MODE_SWEEP, true>();
  return kname<T, false, 0, MODE_SWEEP, true>();
}

template <typename T>
std::string fused_pass_name(bool pro, int out, bool sweep) {
  if (!sweep) return out == 2 ? kname<T, false, 2, MODE_DEF, false>() : kname<T, false, 1, MODE_DEF, false>();
  switch (out) {
    case 1: return kname<T, false, 1, MODE_SWEEP, false>();
    case 2: return kname<T, false, 2, MODE_SWEEP, false>();
    case 3: return kname<T, false, 3, MODE_SWEEP, false>();
    default: return pro ? kname<T, true, 0, MODE_SWEEP, false>() : kname<T, false, 0, MODE_SWEEP, false>();
  }
}

std::string fused_fas_restrict_name(bool sweep) {
  return sweep ? kname<double, false, 1, MODE_SWEEPFAS, false>() : kname<double, false, 1, MODE_FASDEF, false>();
}

#define MG_FUSED_INST(T)                                                                                        \
  template bool fused_supported<T>(int);                                                                        \
  template void fused_sweep<T>(const T*, T*, const T*, int, double, double, const LevelBC&, hipStream_t);        \
  template void fused_sweep_defect<T>(const T*, T*, const T*, T*, T*, int, double, double, const LevelBC&,       \
                                      hipStream_t);                                                             \
  template void fused_prolong_sweep<T>(const T*, T*, const T*, const T*, const LevelBC&, int, double, double,    \
                                       const LevelBC&, hipStream_t);                                            \
  template int fused_sweep_norm<T>(const T*, T*, const T*, double*, int, double, double, const LevelBC&,         \
                                   hipStream_t);                                                                \
  template int fused_sweep_input_norm<T>(const T*, T*, const T*, double*, int, double, double, const LevelBC&,    \
                                         hipStream_t);                                                          \
  template void fused_defect_restrict<T>(const T*, const T*, T*, T*, int, double, const LevelBC&, hipStream_t);  \
  template int fused_defect_norm<T>(const T*, const T*, double*, int, double, const LevelBC&, hipStream_t, float*); \
  template std::string fused_pass_name<T>(bool, int, bool);                                                     \
  template void fused_blk_sweep<T>(const T*, T*, const T*, const T*, const LevelBC&, int, int, double, double,   \
                                   const LevelBC&, hipStream_t);                                                \
  template void fused_blk_defect_restrict<T>(const T*, const T*, T*, T*, int, int, double, const LevelBC&,       \
                                             hipStream_t);                                                      \
  template int fused_blk_defect_norm<T>(const T*, const T*, double*, int, int, double, const LevelBC&,           \
                                        hipStream_t, float*);                                                   \
  template std::string fused_blk_pass_name<T>(bool, int);

MG_FUSED_INST(double)
MG_FUSED_INST(float)

}  // namespace mg
