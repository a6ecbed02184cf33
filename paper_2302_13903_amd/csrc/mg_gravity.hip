// mg_gravity.hip -- gravitational acceleration g = -grad phi (eq. acceleration) in the
// cell-centred source-term scheme of Sec. 2.4.
//
// For each axis a cell face carries the difference of its two adjacent potentials over the
// cell width (sign of -grad), a cell the mean of its two faces, and the momentum source is
// rho times the cell value.  Potentials across the domain surface are the ghosts of the
// Laplacian's boundary rule (Sec. 2.3.6), evaluated on the fly from the adjacent cell.
//
// The arithmetic is written in the order fl = (phi_left - phi) * (1/h),
// fr = (phi - phi_right) * (1/h), g = 0.5 (fl + fr) with contraction off, so for a power-of-two
// cell width every output is the correctly rounded result of the definition (1/h exact).
//
// Large grids (n >= 128): a streaming pass.  A wavefront owns a strip of 128 x R cells in x-y
// (lane l holds the x-pair 2l, 2l+1 of R consecutive rows) and marches in z over a chunk of
// planes, keeping planes k-1, k, k+1 of its cells in registers.  x-neighbours inside the strip
// move across lanes by DPP; y-neighbours are the same lane's other rows, plus one halo row on
// each side loaded from the cache; z-neighbours are the register planes.  phi crosses HBM
// once; every output is written once with 16-byte stores (8-byte for x faces, whose rows
// hold n+1 values).  Small grids: one thread per cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "mg_launch.h"

namespace mg {

namespace {

constexpr int kLanes = 64;
constexpr int kStripX = 2 * kLanes;

struct GravArgs {
  const double* phi;
  const double* rho;   // needed when rhog is set
  double* g;           // 3 n^3 or null
  double* rhog;        // 3 n^3 or null
  double* gf;          // 3 n^2 (n+1) or null (dense layout)
  LevelBC bc;
  int n, L, Lm;        // Lm > 0: MeshBlock layout with 2^Lm-cell blocks
  int tiles_x, strips, zc, ntiles;
  double ih;
};

constexpr int kDppWaveShr1 = 0x138;   // lane i receives lane i-1
constexpr int kDppWaveShl1 = 0x130;   // lane i receives lane i+1

// Whole-wave shift by one lane of `src`; the lane without a source (lane 0 for wave_shr,
// lane 63 for wave_shl) receives `old` instead.  Taking the edge value through the DPP's own
// old operand (rather than a per-lane select afterwards) keeps the move outside any
// lane-divergent branch: a DPP executed with its source lane masked off would return the
// destination's previous value instead of the neighbour's.
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double old, double src) {
  const long long o = __builtin_bit_cast(long long, old), v = __builtin_bit_cast(long long, src);
  const int lo2 = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffLL), (int)(v & 0xffffffffLL), CTRL, 0xf, 0xf, false);
  const int hi2 = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi2 << 32) | (long long)(unsigned)lo2);
}

// Ghost potential across non-periodic face `face` next to a cell holding `own`.
__device__ __forceinline__ double ghost(const LevelBC& bc, int face, int n, int t1, int t2, double own) {
  if (bc.kind[face] == BC_ZERO_GRADIENT) return own;
  return 2.0 * face_b(bc, face, n, t1, t2) - own;
}

struct D2 {
  double a, b;
};

__device__ __forceinline__ D2 ld2(const double* __restrict__ p, size_t i) {
  const double2 v = *reinterpret_cast<const double2*>(p + i);
  return D2{v.x, v.y};
}
// Outputs are written once and not read again by this pass: nontemporal 16-byte stores
// (measured 4 % faster than plain stores at 512^3).
typedef double nt_double2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void st2(double* __restrict__ p, size_t i, double a, double b) {
  const nt_double2 v = {a, b};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_double2*>(p + i));
}

// Face value from the potentials on its two sides (lower index first) and the cell value
// from its two faces, with the rounding of the definition.
__device__ __forceinline__ double face_g(double lo, double hi, double ih) {
#pragma clang fp contract(off)
  return (lo - hi) * ih;
}
__device__ __forceinline__ double cell_g(double fl, double fr) {
#pragma clang fp contract(off)
  return 0.5 * (fl + fr);
}

template <bool BLK>
__device__ __forceinline__ size_t at(const GravArgs& A, int x, int y, int z) {
  return BLK ? bidx(A.Lm, x, y, z) : cidx(A.L, x, y, z);
}

// Outputs written, as template bits (registers go only to the paths a launch takes).
enum : int { OUT_G = 1, OUT_RHOG = 2, OUT_FACE = 4 };

// ---- streaming pass, n >= 128 ------------------------------------------------------------
template <int R, int W, bool BLK, int OUTS>
__global__ void __launch_bounds__(kLanes* W) k_grav_stream(GravArgs A) {
  constexpr bool WG = OUTS & OUT_G, WR = OUTS & OUT_RHOG, WF = !BLK && (OUTS & OUT_FACE);
  const int lane = threadIdx.x & (kLanes - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nb = gridDim.x;
  const int bid = blockIdx.x;
  // consecutive workgroup ids go round the 8 XCDs: give each XCD a contiguous run of tiles,
  // so strips that share halo rows share an L2
  const int tile = (bid & 7) * (nb >> 3) + (bid >> 3);
  if (tile >= A.ntiles) return;
  const int n = A.n, nm = n - 1;
  const size_t n3 = (size_t)n * n * n;
  const int tx = tile % A.tiles_x;
  const int ty = (tile / A.tiles_x) % A.strips;
  const int cz = tile / (A.tiles_x * A.strips);
  const int x = tx * kStripX + 2 * lane;          // this lane's cells x, x+1
  const int y0 = (ty * W + w) * R;                // first row of this wave
  const int z0 = cz * A.zc, z1 = z0 + A.zc;
  const bool px = A.bc.kind[0] == BC_PERIODIC;
  const bool py = A.bc.kind[2] == BC_PERIODIC;
  const bool pz = A.bc.kind[4] == BC_PERIODIC;
  const double ih = A.ih;
  const double* __restrict__ phi = A.phi;
  const bool lo_lane = lane == 0, hi_lane = lane == kLanes - 1;
  const bool xl_edge = lo_lane && x == 0 && !px;          // cell a on the -x face
  const bool xr_edge = hi_lane && x + 1 == nm && !px;     // cell b on the +x face
  const int xl = (x - 1) & nm, xr = (x + 2) & nm;

  D2 cm[R], cc[R], cn[R];
  // plane z0 and the plane below it
#pragma unroll
  for (int r = 0; r < R; ++r) cc[r] = ld2(phi, at<BLK>(A, x, y0 + r, z0));
  if (z0 > 0 || pz) {
#pragma unroll
    for (int r = 0; r < R; ++r) cm[r] = ld2(phi, at<BLK>(A, x, y0 + r, (z0 - 1) & nm));
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r)
      cm[r] = D2{ghost(A.bc, 4, n, x, y0 + r, cc[r].a), ghost(A.bc, 4, n, x + 1, y0 + r, cc[r].b)};
  }

  for (int z = z0; z < z1; ++z) {
    // plane above
    if (z < nm || pz) {
      const int zn = (z + 1) & nm;
#pragma unroll
      for (int r = 0; r < R; ++r) cn[r] = ld2(phi, at<BLK>(A, x, y0 + r, zn));
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r)
        cn[r] = D2{ghost(A.bc, 5, n, x, y0 + r, cc[r].a), ghost(A.bc, 5, n, x + 1, y0 + r, cc[r].b)};
    }
    // halo rows of plane z
    D2 ylo, yhi;
    if (y0 > 0 || py) ylo = ld2(phi, at<BLK>(A, x, (y0 - 1) & nm, z));
    else ylo = D2{ghost(A.bc, 2, n, x, z, cc[0].a), ghost(A.bc, 2, n, x + 1, z, cc[0].b)};
    if (y0 + R < n || py) yhi = ld2(phi, at<BLK>(A, x, (y0 + R) & nm, z));
    else yhi = D2{ghost(A.bc, 3, n, x, z, cc[R - 1].a), ghost(A.bc, 3, n, x + 1, z, cc[R - 1].b)};
    // x-halo of the strip's edge lanes (lane 0: left of its cell a; lane 63: right of b)
    double hx[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      hx[r] = 0.0;
      if (lo_lane) hx[r] = xl_edge ? ghost(A.bc, 0, n, y0 + r, z, cc[r].a) : phi[at<BLK>(A, xl, y0 + r, z)];
      if (hi_lane) hx[r] = xr_edge ? ghost(A.bc, 1, n, y0 + r, z, cc[r].b) : phi[at<BLK>(A, xr, y0 + r, z)];
    }
    D2 rh[R];
    if (WR) {
#pragma unroll
      for (int r = 0; r < R; ++r) rh[r] = ld2(A.rho, at<BLK>(A, x, y0 + r, z));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int y = y0 + r;
      const D2 c = cc[r];
      const double left = dpp_shift<kDppWaveShr1>(hx[r], c.b);    // lane 0: its x-halo
      const double right = dpp_shift<kDppWaveShl1>(hx[r], c.a);   // lane 63: its x-halo
      const D2 yl = r == 0 ? ylo : cc[r - 1];
      const D2 yh = r == R - 1 ? yhi : cc[r + 1];
      const double fxa = face_g(left, c.a, ih), fxm = face_g(c.a, c.b, ih), fxb = face_g(c.b, right, ih);
      const double fya0 = face_g(yl.a, c.a, ih), fya1 = face_g(c.a, yh.a, ih);
      const double fyb0 = face_g(yl.b, c.b, ih), fyb1 = face_g(c.b, yh.b, ih);
      const double fza0 = face_g(cm[r].a, c.a, ih), fza1 = face_g(c.a, cn[r].a, ih);
      const double fzb0 = face_g(cm[r].b, c.b, ih), fzb1 = face_g(c.b, cn[r].b, ih);
      const double gxa = cell_g(fxa, fxm), gxb = cell_g(fxm, fxb);
      const double gya = cell_g(fya0, fya1), gyb = cell_g(fyb0, fyb1);
      const double gza = cell_g(fza0, fza1), gzb = cell_g(fzb0, fzb1);
      const size_t o = at<BLK>(A, x, y, z);
      if (WG) {
        st2(A.g, o, gxa, gxb);
        st2(A.g, n3 + o, gya, gyb);
        st2(A.g, 2 * n3 + o, gza, gzb);
      }
      if (WR) {
        st2(A.rhog, o, rh[r].a * gxa, rh[r].b * gxb);
        st2(A.rhog, n3 + o, rh[r].a * gya, rh[r].b * gyb);
        st2(A.rhog, 2 * n3 + o, rh[r].a * gza, rh[r].b * gzb);
      }
      if (WF) {
        const size_t nf = (size_t)n * n * (n + 1);
        double* __restrict__ fx = A.gf;
        double* __restrict__ fy = A.gf + nf;
        double* __restrict__ fz = A.gf + 2 * nf;
        const size_t rx = ((size_t)z * n + y) * (size_t)(n + 1) + x;
        fx[rx] = fxa;
        fx[rx + 1] = fxm;
        if (x + 1 == nm) fx[rx + 2] = fxb;
        st2(fy, ((size_t)z * (n + 1) + y) * n + x, fya0, fyb0);
        if (y == nm) st2(fy, ((size_t)z * (n + 1) + n) * n + x, fya1, fyb1);
        st2(fz, ((size_t)z * n + y) * n + x, fza0, fzb0);
        if (z == nm) st2(fz, ((size_t)n * n + y) * n + x, fza1, fzb1);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cm[r] = cc[r];
      cc[r] = cn[r];
    }
  }
}

// ---- one thread per cell (any n) ---------------------------------------------------------
template <bool BLK>
__global__ void __launch_bounds__(256) k_grav_cell(GravArgs A) {
  const int n = A.n, L = A.L, nm = n - 1;
  const size_t n3 = (size_t)n * n * n;
  const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= n3) return;
  const int i = (int)(id & nm), j = (int)((id >> L) & nm), k = (int)(id >> (2 * L));
  const double* __restrict__ phi = A.phi;
  const size_t c = at<BLK>(A, i, j, k);
  const double p = phi[c];
  auto nbr = [&](int face, int ii, int jj, int kk, int t1, int t2) __attribute__((always_inline)) {
    const bool out = (unsigned)ii >= (unsigned)n || (unsigned)jj >= (unsigned)n || (unsigned)kk >= (unsigned)n;
    if (!out) return phi[at<BLK>(A, ii, jj, kk)];
    if (A.bc.kind[face] == BC_PERIODIC) return phi[at<BLK>(A, ii & nm, jj & nm, kk & nm)];
    return ghost(A.bc, face, n, t1, t2, p);
  };
  const double ih = A.ih;
  const double fx0 = face_g(nbr(0, i - 1, j, k, j, k), p, ih), fx1 = face_g(p, nbr(1, i + 1, j, k, j, k), ih);
  const double fy0 = face_g(nbr(2, i, j - 1, k, i, k), p, ih), fy1 = face_g(p, nbr(3, i, j + 1, k, i, k), ih);
  const double fz0 = face_g(nbr(4, i, j, k - 1, i, j), p, ih), fz1 = face_g(p, nbr(5, i, j, k + 1, i, j), ih);
  const double gx = cell_g(fx0, fx1), gy = cell_g(fy0, fy1), gz = cell_g(fz0, fz1);
  if (A.g) {
    A.g[c] = gx;
    A.g[n3 + c] = gy;
    A.g[2 * n3 + c] = gz;
  }
  if (A.rhog) {
    const double r = A.rho[c];
    A.rhog[c] = r * gx;
    A.rhog[n3 + c] = r * gy;
    A.rhog[2 * n3 + c] = r * gz;
  }
  if (!BLK && A.gf) {
    const size_t nf = (size_t)n * n * (n + 1);
    double* __restrict__ fx = A.gf;
    double* __restrict__ fy = A.gf + nf;
    double* __restrict__ fz = A.gf + 2 * nf;
    fx[((size_t)k * n + j) * (size_t)(n + 1) + i] = fx0;
    if (i == nm) fx[((size_t)k * n + j) * (size_t)(n + 1) + n] = fx1;
    fy[((size_t)k * (n + 1) + j) * n + i] = fy0;
    if (j == nm) fy[((size_t)k * (n + 1) + n) * n + i] = fy1;
    fz[((size_t)k * n + j) * n + i] = fz0;
    if (k == nm) fz[((size_t)n * n + j) * n + i] = fz1;
  }
}

constexpr int kGravR = 4, kGravW = 4;

struct GravShape {
  bool stream;
  int tiles_x, strips, zc, ntiles, grid;
};

GravShape grav_shape(int n) {
  GravShape s{};
  s.stream = n >= kStripX;
  if (!s.stream) {
    const size_t n3 = (size_t)n * n * n;
    s.grid = (int)((n3 + 255) / 256);
    return s;
  }
  s.tiles_x = n / kStripX;
  s.strips = n / (kGravR * kGravW);
  // planes per chunk: enough workgroups to fill the chip (about 2048), chunks of 8..64 planes
  const long long cols = (long long)s.tiles_x * s.strips;
  int zc = 64;
  while (zc > 8 && cols * (n / zc) < 2048) zc >>= 1;
  s.zc = std::min(zc, n);
  s.ntiles = (int)(cols * (n / s.zc));
  s.grid = (s.ntiles + 7) / 8 * 8;
  return s;
}

template <int R, int W, bool BLK, int OUTS>
void launch_stream(const GravArgs& A, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_grav_stream<R, W, BLK, OUTS>), dim3(grid), dim3(kLanes * W), 0, s, A);
}

template <bool BLK>
void launch_stream_outs(const GravArgs& A, int outs, int grid, hipStream_t s) {
  switch (outs) {
    case 1: launch_stream<kGravR, kGravW, BLK, 1>(A, grid, s); break;
    case 2: launch_stream<kGravR, kGravW, BLK, 2>(A, grid, s); break;
    case 3: launch_stream<kGravR, kGravW, BLK, 3>(A, grid, s); break;
    case 4: launch_stream<kGravR, kGravW, BLK, 4>(A, grid, s); break;
    case 5: launch_stream<kGravR, kGravW, BLK, 5>(A, grid, s); break;
    case 6: launch_stream<kGravR, kGravW, BLK, 6>(A, grid, s); break;
    default: launch_stream<kGravR, kGravW, BLK, 7>(A, grid, s); break;
  }
}

int outs_of(const double* g, const double* rhog, const double* gface, int Lm) {
  return (g ? OUT_G : 0) | (rhog ? OUT_RHOG : 0) | (gface && Lm == 0 ? OUT_FACE : 0);
}

}  // namespace

int launch_gravity(const double* phi, const double* rho, double* g, double* rhog, double* gface, int n, int Lm,
                   double dx, const LevelBC& bc, hipStream_t s) {
  GravArgs A{};
  A.phi = phi;
  A.rho = rho;
  A.g = g;
  A.rhog = rhog;
  A.gf = Lm > 0 ? nullptr : gface;
  A.bc = bc;
  A.n = n;
  A.L = ilog2(n);
  A.Lm = Lm;
  A.ih = 1.0 / dx;
  const int outs = outs_of(g, rhog, gface, Lm);
  if (!outs) return 0;
  const GravShape sh = grav_shape(n);
  if (sh.stream) {
    A.tiles_x = sh.tiles_x;
    A.strips = sh.strips;
    A.zc = sh.zc;
    A.ntiles = sh.ntiles;
    if (Lm > 0) launch_stream_outs<true>(A, outs, sh.grid, s);
    else launch_stream_outs<false>(A, outs, sh.grid, s);
  } else {
    if (Lm > 0) hipLaunchKernelGGL((k_grav_cell<true>), dim3(sh.grid), dim3(256), 0, s, A);
    else hipLaunchKernelGGL((k_grav_cell<false>), dim3(sh.grid), dim3(256), 0, s, A);
  }
  return sh.grid;
}

std::string gravity_kernel_name(int n, int Lm, bool g, bool rhog, bool gface) {
  const std::string blk = Lm > 0 ? "true" : "false";
  const std::string args = "(mg::(anonymous namespace)::GravArgs)";
  if (n >= kStripX) {
    const int outs = (g ? OUT_G : 0) | (rhog ? OUT_RHOG : 0) | (gface && Lm == 0 ? OUT_FACE : 0);
    return "void mg::(anonymous namespace)::k_grav_stream<" + std::to_string(kGravR) + ", " + std::to_string(kGravW) +
           ", " + blk + ", " + std::to_string(outs) + ">" + args;
  }
  return "void mg::(anonymous namespace)::k_grav_cell<" + blk + ">" + args;
}

}  // namespace mg
