// mg_amr.hip -- the multigrid solver on a statically refined mesh (Sec. 3.3): FAS V-cycles
// (Alg. 3) over the MeshBlock levels, the Octet levels and the root grid.
//
// Mesh: NB^3 root MeshBlocks of nb^3 cells; refinement level lam = 1..Lam is one box of
// level-(lam-1) MeshBlocks refined 2:1, nested inside box lam-1 with a margin of at least one
// block.  On MG level k (2^k cells per MeshBlock side) each refinement level is one dense
// patch with a one-cell ghost layer; cells under the next finer box are covered.
//
// Level boundaries: before every colour of the smoother and before every defect, the fine
// patch's ghost faces are interpolated from the coarse patch (transverse coarse gradients,
// eqs. transgrad and piint, then eq. lbint between those points and the first fine cells) and
// the coarse side gets one ghost per hole face by extrapolation through the area mean of the
// first fine cells (eq. lbext), so the face fluxes match (eq. masscons).  Before a
// correction is prolongated, the normal level boundary restricts the finer patch into the
// covered coarse cells and prolongates the coarse patch into the finer patch's ghost shell.
//
// Every operator is one plain launch over a patch (the refined levels are small next to the
// uniform path; this is the correctness-first form of the refined solver).  Arithmetic follows
// the same expressions in the same order as the oracle, so results agree to rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mg355.h"
#include "mg_launch.h"

namespace mg {

namespace {

constexpr int kB = 256;

struct Dims {
  int n[3];   // active cells per axis (x, y, z)
};

__host__ __device__ inline size_t gx(const Dims& d, int x, int y, int z) {
  return ((size_t)(z + 1) * (size_t)(d.n[1] + 2) + (size_t)(y + 1)) * (size_t)(d.n[0] + 2) + (size_t)(x + 1);
}
inline size_t ghosted(const Dims& d) { return (size_t)(d.n[0] + 2) * (d.n[1] + 2) * (d.n[2] + 2); }
__device__ inline size_t ghosted_d(const Dims& d) { return (size_t)(d.n[0] + 2) * (d.n[1] + 2) * (d.n[2] + 2); }
__host__ __device__ inline size_t cells(const Dims& d) { return (size_t)d.n[0] * d.n[1] * d.n[2]; }
inline unsigned blocks(size_t work) { return (unsigned)std::max<size_t>(1, (work + kB - 1) / kB); }
// work items of one colour of k_smooth (x-pairs when the x extent is even)
__host__ __device__ inline size_t smooth_items(const Dims& d) { return (d.n[0] & 1) ? cells(d) : cells(d) / 2; }

struct Hole {
  int on;
  int lo[3], hi[3];       // covered cells, local [lo, hi)
  const double* cg[6];    // per hole face: ghost seen from the active cell outside it, [t2][t1]
};

__device__ inline bool covered(const Hole& H, int x, int y, int z) {
  return H.on && x >= H.lo[0] && x < H.hi[0] && y >= H.lo[1] && y < H.hi[1] && z >= H.lo[2] && z < H.hi[2];
}

// Neighbour value across one face of active cell (x, y, z): the stored neighbour, or the
// hole face's ghost when the neighbour is covered.
__device__ inline double nbv(const double* __restrict__ u, const Dims& d, const Hole& H, int x, int y, int z,
                             int axis, int dir) {
  int p[3] = {x, y, z};
  p[axis] += dir;
  if (covered(H, p[0], p[1], p[2])) {
    const int face = 2 * axis + (dir > 0 ? 0 : 1);   // entering through the hole's low face from below
    const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
    const int m1 = H.hi[t1] - H.lo[t1];
    return H.cg[face][(size_t)(p[t2] - H.lo[t2]) * m1 + (p[t1] - H.lo[t1])];
  }
  return u[gx(d, p[0], p[1], p[2])];
}

__device__ inline double nbsum(const double* __restrict__ u, const Dims& d, const Hole& H, int x, int y, int z) {
  const double xm = nbv(u, d, H, x, y, z, 0, -1), xp = nbv(u, d, H, x, y, z, 0, 1);
  const double ym = nbv(u, d, H, x, y, z, 1, -1), yp = nbv(u, d, H, x, y, z, 1, 1);
  const double zm = nbv(u, d, H, x, y, z, 2, -1), zp = nbv(u, d, H, x, y, z, 2, 1);
  return ((((xm + xp) + ym) + yp) + zm) + zp;
}

// Cell (x, y, z) of work item t < cells(d).  32-bit arithmetic: amr_plan admits patches of
// fewer than 2^31 cells only (a 64-bit division costs several times a 32-bit one, and the
// small kernels and the single-workgroup stages decode an index per item and phase).
__device__ inline void cell_of(size_t t, const Dims& d, int& x, int& y, int& z) {
  const unsigned tt = (unsigned)t, n0 = (unsigned)d.n[0], n1 = (unsigned)d.n[1];
  const unsigned q = tt / n0;
  x = (int)(tt - q * n0);
  y = (int)(q % n1);
  z = (int)(q / n1);
}

// ---- physical ghosts of the root patch (Sec. 2.3.6): filled axis by axis (x, then y over the
// x ghosts, then z over both); fixed faces read b (bn x bn, [t2][t1]) clamped to the face
struct Phys {
  int kind[6];
  const double* b[6];
  int bn;
};

// All ghosts in one launch: every ghost cell is composed from an active cell by the face
// rules in the order z, y, x (the last-filled axis outermost), value = s u + t, which is the
// axis-by-axis fill written out; one thread per cell of the six ghost faces (edge and corner
// cells are reached from two or three faces and written with the same value).
__device__ inline void fill_phys_body(double* __restrict__ u, const Dims& d, const Phys& P, int hom, size_t t) {
  const int n0 = d.n[0] + 2, n1 = d.n[1] + 2, n2 = d.n[2] + 2;
  const size_t f0 = (size_t)n1 * n2, f1 = (size_t)n0 * n2, f2 = (size_t)n0 * n1;
  int p[3];
  // (32-bit decoding, as cell_of)
  if (t < 2 * f0) {
    p[0] = t < f0 ? -1 : d.n[0];
    const unsigned r = (unsigned)(t < f0 ? t : t - f0);
    p[1] = (int)(r % (unsigned)n1) - 1;
    p[2] = (int)(r / (unsigned)n1) - 1;
  } else if ((t -= 2 * f0) < 2 * f1) {
    p[1] = t < f1 ? -1 : d.n[1];
    const unsigned r = (unsigned)(t < f1 ? t : t - f1);
    p[0] = (int)(r % (unsigned)n0) - 1;
    p[2] = (int)(r / (unsigned)n0) - 1;
  } else if ((t -= 2 * f1) < 2 * f2) {
    p[2] = t < f2 ? -1 : d.n[2];
    const unsigned r = (unsigned)(t < f2 ? t : t - f2);
    p[0] = (int)(r % (unsigned)n0) - 1;
    p[1] = (int)(r / (unsigned)n0) - 1;
  } else {
    return;
  }
  const int q[3] = {p[0], p[1], p[2]};
  double sgn = 1.0, add = 0.0;
  for (int axis = 2; axis >= 0; --axis) {
    const int c = p[axis], na = d.n[axis];
    if (c >= 0 && c < na) continue;
    const int side = c < 0 ? 0 : 1, face = 2 * axis + side;
    const int kd = P.kind[face];
    if (kd == BC_PERIODIC) {
      p[axis] = side ? 0 : na - 1;
      continue;
    }
    if (kd != BC_ZERO_GRADIENT) {
      double b = 0.0;
      if (!hom && P.b[face]) {
        // face value at the transverse position of the ghost (ring: the nearest face value)
        const int t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
        const int i1 = min(max(p[t1], 0), P.bn - 1), i2 = min(max(p[t2], 0), P.bn - 1);
        b = P.b[face][(size_t)i2 * P.bn + i1];
      }
      add += sgn * (2.0 * b);
      sgn = -sgn;
    }
    p[axis] = side ? na - 1 : 0;
  }
  u[gx(d, q[0], q[1], q[2])] = sgn * u[gx(d, p[0], p[1], p[2])] + add;
}
__global__ void __launch_bounds__(kB) k_fill_phys1(double* __restrict__ u, Dims d, Phys P, int hom) {
  fill_phys_body(u, d, P, hom, (size_t)blockIdx.x * kB + threadIdx.x);
}
// number of ghost cells of the six faces (edges and corners included)
__host__ __device__ inline size_t ghost_faces(const Dims& d) {
  return (size_t)2 * ((size_t)(d.n[1] + 2) * (d.n[2] + 2) + (size_t)(d.n[0] + 2) * (d.n[2] + 2) +
                      (size_t)(d.n[0] + 2) * (d.n[1] + 2));
}

// ---- conservative level boundary (eqs. transgrad, piint, lbint; lbext on the coarse side)
struct Cons {
  double* uf;
  Dims df;
  const double* uc;
  Dims dc;
  int lo[3], hi[3];   // the fine box in coarse local cells
  double* cg[6];      // coarse ghosts per face, or nullptr
};

__device__ inline void cons_body(const Cons& A, int axis, size_t t) {
  const int t1a = axis == 0 ? 1 : 0, t2a = axis == 2 ? 1 : 2;
  const int nf1 = A.df.n[t1a], nf2 = A.df.n[t2a];
  if (t >= (size_t)2 * nf1 * nf2) return;
  const unsigned face = (unsigned)nf1 * (unsigned)nf2, tt = (unsigned)t;
  const int side = tt >= face ? 1 : 0;
  const unsigned r = side ? tt - face : tt;
  const int j1 = (int)(r % (unsigned)nf1), j2 = (int)(r / (unsigned)nf1);
  const int J1 = A.lo[t1a] + (j1 >> 1), J2 = A.lo[t2a] + (j2 >> 1);
  const int cl = side ? A.hi[axis] : A.lo[axis] - 1;
  auto cidx = [&](int q1, int q2) {
    int p[3];
    p[axis] = cl;
    p[t1a] = q1;
    p[t2a] = q2;
    return gx(A.dc, p[0], p[1], p[2]);
  };
  auto fidx = [&](int layer, int q1, int q2) {
    int p[3];
    p[axis] = layer;
    p[t1a] = q1;
    p[t2a] = q2;
    return gx(A.df, p[0], p[1], p[2]);
  };
  const double C = A.uc[cidx(J1, J2)];
  const double d1 = A.uc[cidx(J1 + 1, J2)] - A.uc[cidx(J1 - 1, J2)];
  const double d2 = A.uc[cidx(J1, J2 + 1)] - A.uc[cidx(J1, J2 - 1)];
  const double s1 = (j1 & 1) ? 1.0 : -1.0, s2 = (j2 & 1) ? 1.0 : -1.0;
  const double cross = (C + s1 * (d1 * 0.125)) + s2 * (d2 * 0.125);
  const int first = side ? A.df.n[axis] - 1 : 0;
  const double F = A.uf[fidx(first, j1, j2)];
  A.uf[fidx(side ? A.df.n[axis] : -1, j1, j2)] = (1.0 / 3.0) * F + (2.0 / 3.0) * cross;
  if (A.cg[0] && !(j1 & 1) && !(j2 & 1)) {
    const double fr = 0.25 * (((F + A.uf[fidx(first, j1 + 1, j2)]) + A.uf[fidx(first, j1, j2 + 1)]) +
                              A.uf[fidx(first, j1 + 1, j2 + 1)]);
    const int m1 = A.hi[t1a] - A.lo[t1a];
    A.cg[2 * axis + side][(size_t)(J2 - A.lo[t2a]) * m1 + (J1 - A.lo[t1a])] = (4.0 / 3.0) * fr - (1.0 / 3.0) * C;
  }
}

// Batched launches: one launch runs one operator on several patches of a level, patch q on
// blockIdx.y (blockIdx.z), each with its own arguments; the blocks past a patch's own extent
// return at the bounds check of the shared body.
constexpr int kMaxSet = MG_AMR_MAX_LEVELS + 1;
template <typename A>
struct Set {
  A a[kMaxSet];
};

__global__ void __launch_bounds__(kB) k_cons(Cons A) { cons_body(A, blockIdx.y, (size_t)blockIdx.x * kB + threadIdx.x); }
// All ghosts of one level: the level boundaries of the ncons finer patches (axis on
// blockIdx.y, patch on blockIdx.z) and, on blockIdx.z = ncons, the physical ghosts of the root
// patch.  Each part reads active cells only and writes its own ghosts.
__global__ void __launch_bounds__(kB) k_ghosts_set(Set<Cons> S, int ncons, double* __restrict__ u0, Dims d0, Phys P0,
                                                   int hom0) {
  const size_t t = (size_t)blockIdx.x * kB + threadIdx.x;
  if ((int)blockIdx.z < ncons) cons_body(S.a[blockIdx.z], blockIdx.y, t);
  else if (blockIdx.y == 0) fill_phys_body(u0, d0, P0, hom0, t);
}

// ---- RB-SOR on the active cells of one colour (eqs. rbsor1-2); colour by global parity
// With an even x extent one work item per x-pair updates the pair's cell of this colour;
// otherwise one work item per cell.
__device__ inline void smooth_body(double* __restrict__ u, const double* __restrict__ f, const Dims& d, int o0, int o1,
                                   int o2, const Hole& H, double h2, double omega, int colour, size_t t) {
  int x, y, z;
  if ((d.n[0] & 1) == 0) {
    const Dims dp{{d.n[0] / 2, d.n[1], d.n[2]}};
    if (t >= cells(dp)) return;
    cell_of(t, dp, x, y, z);
    x = 2 * x + ((colour + o0 + (o1 + y) + (o2 + z)) & 1);
  } else {
    if (t >= cells(d)) return;
    cell_of(t, d, x, y, z);
  }
  if ((((o0 + x) + (o1 + y) + (o2 + z)) & 1) != colour || covered(H, x, y, z)) return;
  const size_t c = gx(d, x, y, z);
  const double uc = u[c];
  const double nb = nbsum(u, d, H, x, y, z);
  u[c] = uc + omega * ((nb - h2 * f[c]) / 6.0 - uc);
}
__global__ void __launch_bounds__(kB) k_smooth(double* __restrict__ u, const double* __restrict__ f, Dims d, int o0,
                                                int o1, int o2, Hole H, double h2, double omega, int colour) {
  smooth_body(u, f, d, o0, o1, o2, H, h2, omega, colour, (size_t)blockIdx.x * kB + threadIdx.x);
}
struct SmoothA {
  double* u;
  const double* f;
  Dims d;
  int o[3];
  Hole H;
  double h2;
};
__global__ void __launch_bounds__(kB) k_smooth_set(Set<SmoothA> S, double omega, int colour) {
  const SmoothA& A = S.a[blockIdx.y];
  smooth_body(A.u, A.f, A.d, A.o[0], A.o[1], A.o[2], A.H, A.h2, omega, colour, (size_t)blockIdx.x * kB + threadIdx.x);
}

// ---- out = a + s L u on the active cells (defect: a = f, s = -1; FAS source: a = restricted
// defect, s = +1); covered cells get 0
__device__ inline void lap_body(const double* __restrict__ u, const double* __restrict__ a, double* __restrict__ out,
                                const Dims& d, const Hole& H, double ih2, double s, size_t t) {
  if (t >= cells(d)) return;
  int x, y, z;
  cell_of(t, d, x, y, z);
  const size_t c = gx(d, x, y, z);
  if (covered(H, x, y, z)) {
    out[c] = 0.0;
    return;
  }
  const double L = (nbsum(u, d, H, x, y, z) - 6.0 * u[c]) * ih2;
  out[c] = a[c] + s * L;
}
__global__ void __launch_bounds__(kB) k_lap(const double* __restrict__ u, const double* __restrict__ a,
                                             double* __restrict__ out, Dims d, Hole H, double ih2, double s) {
  lap_body(u, a, out, d, H, ih2, s, (size_t)blockIdx.x * kB + threadIdx.x);
}
struct LapA {
  const double* u;
  const double* a;
  double* out;
  Dims d;
  Hole H;
  double ih2;
};
__global__ void __launch_bounds__(kB) k_lap_set(Set<LapA> S, double s) {
  const LapA& A = S.a[blockIdx.y];
  lap_body(A.u, A.a, A.out, A.d, A.H, A.ih2, s, (size_t)blockIdx.x * kB + threadIdx.x);
}

// ---- 8-cell mean (eq. restriction) of the fine patch into coarse cells [0, nr) written at
// coarse local offset o; covered fine cells count as 0 when the fine hole is given
__device__ inline void restrict_body(const double* __restrict__ uf, const Dims& df, const Hole& Hf, double* out1,
                                     double* out2, const Dims& dc, int o0, int o1, int o2, const Dims& nr, size_t t) {
  if (t >= cells(nr)) return;
  int X, Y, Z;
  cell_of(t, nr, X, Y, Z);
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int x = 2 * X + a, y = 2 * Y + b, z = 2 * Z + c;
        s += covered(Hf, x, y, z) ? 0.0 : uf[gx(df, x, y, z)];
      }
  const double v = s / 8.0;
  const size_t o = gx(dc, o0 + X, o1 + Y, o2 + Z);
  out1[o] = v;
  if (out2) out2[o] = v;
}
__global__ void __launch_bounds__(kB) k_restrict(const double* __restrict__ uf, Dims df, Hole Hf, double* out1,
                                                  double* out2, Dims dc, int o0, int o1, int o2, Dims nr) {
  restrict_body(uf, df, Hf, out1, out2, dc, o0, o1, o2, nr, (size_t)blockIdx.x * kB + threadIdx.x);
}
struct RestrictA {
  const double* uf;
  Dims df;
  Hole Hf;
  double* out1;
  double* out2;
  Dims dc;
  int o[3];
  Dims nr;
};
__global__ void __launch_bounds__(kB) k_restrict_set(Set<RestrictA> S) {
  const RestrictA& A = S.a[blockIdx.y];
  restrict_body(A.uf, A.df, A.Hf, A.out1, A.out2, A.dc, A.o[0], A.o[1], A.o[2], A.nr,
                (size_t)blockIdx.x * kB + threadIdx.x);
}

// ---- prolongation, separable x then y then z as in the oracle.  Fine cells [lo, hi) per axis
// (ghost indices allowed); parent coarse cell = (fine global >> 1) - coarse origin.
// mode 0: trilinear (eq. trilinear), added on active fine cells; 1: trilinear, set on the
// ghost shell only; 2: tricubic FMG prolongation (Sec. 2.3.1), set on active cells (0 on
// covered cells).
__device__ inline void prolong_body(const double* __restrict__ uc, const Dims& dc, int co0, int co1, int co2,
                                    double* __restrict__ uf, const Dims& df, int fo0, int fo1, int fo2, const Hole& Hf,
                                    int lx, int ly, int lz, const Dims& span, int mode, size_t t) {
  if (t >= cells(span)) return;
  int x, y, z;
  cell_of(t, span, x, y, z);
  x += lx;
  y += ly;
  z += lz;
  const bool shell = x < 0 || y < 0 || z < 0 || x >= df.n[0] || y >= df.n[1] || z >= df.n[2];
  if (mode != 1 && shell) return;
  if (mode == 0 && covered(Hf, x, y, z)) return;
  if (mode == 1 && !shell) return;
  if (mode == 2 && covered(Hf, x, y, z)) {
    uf[gx(df, x, y, z)] = 0.0;
    return;
  }
  const int gxg = fo0 + x, gyg = fo1 + y, gzg = fo2 + z;
  const int X = (gxg >> 1) - co0, Y = (gyg >> 1) - co1, Z = (gzg >> 1) - co2;
  const int ux = gxg & 1, uy = gyg & 1, uz = gzg & 1;
  // per axis: lower child 1/4 c[I-1] + 3/4 c[I]; upper 3/4 c[I] + 1/4 c[I+1]
  // tricubic: lower child (5 c[I-1] + 30 c[I] - 3 c[I+1]) / 32, upper (-3, 30, 5) / 32
  const bool cubic = mode == 2;
  auto lin = [cubic](double cm, double c0, double cp, int up) {
    if (cubic)
      return up ? ((-3.0 / 32.0) * cm + (30.0 / 32.0) * c0) + (5.0 / 32.0) * cp
                : ((5.0 / 32.0) * cm + (30.0 / 32.0) * c0) + (-3.0 / 32.0) * cp;
    return up ? 0.75 * c0 + 0.25 * cp : 0.25 * cm + 0.75 * c0;
  };
  double ty[3][3];
#pragma unroll
  for (int c = -1; c <= 1; ++c)
#pragma unroll
    for (int b = -1; b <= 1; ++b)
      ty[c + 1][b + 1] = lin(uc[gx(dc, X - 1, Y + b, Z + c)], uc[gx(dc, X, Y + b, Z + c)],
                             uc[gx(dc, X + 1, Y + b, Z + c)], ux);
  double tz[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) tz[c] = lin(ty[c][0], ty[c][1], ty[c][2], uy);
  const double v = lin(tz[0], tz[1], tz[2], uz);
  const size_t o = gx(df, x, y, z);
  uf[o] = mode == 0 ? uf[o] + v : v;
}
__global__ void __launch_bounds__(kB) k_prolong(const double* __restrict__ uc, Dims dc, int co0, int co1, int co2,
                                                 double* __restrict__ uf, Dims df, int fo0, int fo1, int fo2,
                                                 Hole Hf, int lx, int ly, int lz, Dims span, int mode) {
  prolong_body(uc, dc, co0, co1, co2, uf, df, fo0, fo1, fo2, Hf, lx, ly, lz, span, mode,
               (size_t)blockIdx.x * kB + threadIdx.x);
}
struct ProlongA {
  const double* uc;
  Dims dc;
  int co[3];
  double* uf;
  Dims df;
  int fo[3];
  Hole Hf;
  int l[3];
  Dims span;
};
__global__ void __launch_bounds__(kB) k_prolong_set(Set<ProlongA> S, int mode) {
  const ProlongA& A = S.a[blockIdx.y];
  prolong_body(A.uc, A.dc, A.co[0], A.co[1], A.co[2], A.uf, A.df, A.fo[0], A.fo[1], A.fo[2], A.Hf, A.l[0], A.l[1], A.l[2],
               A.span, mode, (size_t)blockIdx.x * kB + threadIdx.x);
}

// dst = src over the whole ghosted array
__global__ void __launch_bounds__(kB) k_copy(const double* __restrict__ src, double* __restrict__ dst, size_t n) {
  const size_t t = (size_t)blockIdx.x * kB + threadIdx.x;
  if (t < n) dst[t] = src[t];
}

// out = u - p on the active cells (0 on covered cells)
__device__ inline void sub_body(const double* __restrict__ u, const double* __restrict__ p, double* __restrict__ out,
                                const Dims& d, const Hole& H, size_t t) {
  if (t >= cells(d)) return;
  int x, y, z;
  cell_of(t, d, x, y, z);
  const size_t c = gx(d, x, y, z);
  out[c] = covered(H, x, y, z) ? 0.0 : u[c] - p[c];
}
__global__ void __launch_bounds__(kB) k_sub(const double* __restrict__ u, const double* __restrict__ p,
                                             double* __restrict__ out, Dims d, Hole H) {
  sub_body(u, p, out, d, H, (size_t)blockIdx.x * kB + threadIdx.x);
}
struct SubA {
  const double* u;
  const double* p;
  double* out;
  Dims d;
  Hole H;
};
__global__ void __launch_bounds__(kB) k_sub_set(Set<SubA> S) {
  const SubA& A = S.a[blockIdx.y];
  sub_body(A.u, A.p, A.out, A.d, A.H, (size_t)blockIdx.x * kB + threadIdx.x);
}

// kernel arguments are limited to 4 KiB
static_assert(sizeof(Set<Cons>) <= 4096 && sizeof(Set<SmoothA>) <= 4096 && sizeof(Set<LapA>) <= 4096 &&
                  sizeof(Set<RestrictA>) <= 4096 && sizeof(Set<ProlongA>) <= 4096 && sizeof(Set<SubA>) <= 4096,
              "batched launch arguments");

// dense caller array <-> ghosted patch: a*src + c on active cells, 0 on covered cells
__global__ void __launch_bounds__(kB) k_load(const double* __restrict__ src, double* __restrict__ dst, Dims d, Hole H,
                                              double a, double c) {
  const size_t t = (size_t)blockIdx.x * kB + threadIdx.x;
  if (t >= cells(d)) return;
  int x, y, z;
  cell_of(t, d, x, y, z);
  dst[gx(d, x, y, z)] = covered(H, x, y, z) ? 0.0 : a * src[t] + c;
}
__global__ void __launch_bounds__(kB) k_store(const double* __restrict__ src, double* __restrict__ dst, Dims d, Hole H,
                                               double c) {
  const size_t t = (size_t)blockIdx.x * kB + threadIdx.x;
  if (t >= cells(d)) return;
  int x, y, z;
  cell_of(t, d, x, y, z);
  dst[t] = covered(H, x, y, z) ? 0.0 : src[gx(d, x, y, z)] - c;
}

// dst = src on the active cells, 0 on covered cells (both ghosted arrays)
__global__ void __launch_bounds__(kB) k_load_ghosted(const double* __restrict__ src, double* __restrict__ dst, Dims d,
                                                      Hole H) {
  const size_t t = (size_t)blockIdx.x * kB + threadIdx.x;
  if (t >= cells(d)) return;
  int x, y, z;
  cell_of(t, d, x, y, z);
  const size_t c = gx(d, x, y, z);
  dst[c] = covered(H, x, y, z) ? 0.0 : src[c];
}

// per-block partial sums of g(v) over the active cells (what: 0 value, 1 square), fixed tree
// Partial sums over the active cells of several patches in one launch: patch q (blockIdx.y)
// uses its own nb blocks, block b summing cells b*kB + i + j*nb*kB into part[q * stride + b],
// so each patch's partials and their order are fixed by its own size.
struct SumA {
  const double* v;
  Dims d;
  Hole H;
  int nb;
};
__global__ void __launch_bounds__(kB) k_psum_set(Set<SumA> S, int what, double* __restrict__ part, int stride) {
  const SumA& A = S.a[blockIdx.y];
  if ((int)blockIdx.x >= A.nb) return;
  __shared__ double sh[kB];
  double acc = 0.0;
  for (size_t t = (size_t)blockIdx.x * kB + threadIdx.x; t < cells(A.d); t += (size_t)A.nb * kB) {
    int x, y, z;
    cell_of(t, A.d, x, y, z);
    if (covered(A.H, x, y, z)) continue;
    const double a = A.v[gx(A.d, x, y, z)];
    acc += what ? a * a : a;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(size_t)blockIdx.y * stride + blockIdx.x] = sh[0];
}

// 2 x 2 area mean of a face array (n x n) -> (n/2 x n/2)
__global__ void __launch_bounds__(kB) k_face_mean(const double* __restrict__ b, double* __restrict__ out, int nc) {
  const int t = blockIdx.x * kB + threadIdx.x;
  if (t >= nc * nc) return;
  const int i = t % nc, j = t / nc, n = 2 * nc;
  out[t] = 0.25 * (((b[(size_t)(2 * j) * n + 2 * i] + b[(size_t)(2 * j) * n + 2 * i + 1]) +
                    b[(size_t)(2 * j + 1) * n + 2 * i]) + b[(size_t)(2 * j + 1) * n + 2 * i + 1]);
}

// single root cell (Sec. 2.3.2): ghost = alpha u + beta per face; kept when nothing fixes it
__global__ void k_coarsest(double* u, const double* f, Phys P, double h2) {
  if (threadIdx.x || blockIdx.x) return;
  double sa = 0.0, sb = 0.0;
  for (int face = 0; face < 6; ++face) {
    if (P.kind[face] == BC_PERIODIC || P.kind[face] == BC_ZERO_GRADIENT) {
      sa += 1.0;
    } else {
      sa -= 1.0;
      sb += 2.0 * (P.b[face] ? P.b[face][0] : 0.0);
    }
  }
  const Dims d{{1, 1, 1}};
  if (sa != 6.0) u[gx(d, 0, 0, 0)] = (sb - h2 * f[gx(d, 0, 0, 0)]) / (6.0 - sa);
}

// ---- the small root levels (kRootTailN^3 cells and below) in one workgroup: the uniform FAS
// V-cycle of the root grid from level q0 down to the single cell and back, every operator a
// block-strided loop followed by a barrier (the levels are cached in the CU; its waves share
// the L1, so a barrier orders their global-memory accesses).  Same bodies, same order of
// operations as the per-operator launches.
constexpr int kRootTailN = 16;
constexpr int kRootTailThreads = 1024;
constexpr int kMaxRoot = 10;   // root levels 256^3 .. 1
struct RootLvl {
  Dims d;
  double h;
  double *u, *f, *pbar, *dres, *tmp;
  Phys phys;   // physical conditions at this level's face points
};
struct RootSet {
  RootLvl l[kMaxRoot];
};

template <typename F>
__device__ inline void forall(size_t work, F fn) {
  for (size_t t = threadIdx.x; t < work; t += blockDim.x) fn(t);
  __syncthreads();
}

__device__ void root_tail_run(const RootSet& S, int q0, int npre, int npost, double omega) {
  const Hole none{};
  auto smooth = [&](const RootLvl& L, int sweeps) {
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        forall(ghost_faces(L.d), [&](size_t t) { fill_phys_body(L.u, L.d, L.phys, 0, t); });
        forall(smooth_items(L.d),
               [&](size_t t) { smooth_body(L.u, L.f, L.d, 0, 0, 0, none, L.h * L.h, omega, colour, t); });
      }
  };
  int q = q0;
  // down: smooth, defect, FAS restriction of u and of the defect, coarse source
  while (S.l[q].d.n[0] > 1) {
    const RootLvl& L = S.l[q];
    const RootLvl& C = S.l[q + 1];
    smooth(L, npre);
    forall(ghost_faces(L.d), [&](size_t t) { fill_phys_body(L.u, L.d, L.phys, 0, t); });
    forall(cells(L.d), [&](size_t t) { lap_body(L.u, L.f, L.tmp, L.d, none, 1.0 / (L.h * L.h), -1.0, t); });
    forall(cells(C.d), [&](size_t t) {
      restrict_body(L.u, L.d, none, C.u, C.pbar, C.d, 0, 0, 0, C.d, t);
      restrict_body(L.tmp, L.d, none, C.dres, nullptr, C.d, 0, 0, 0, C.d, t);
    });
    forall(ghost_faces(C.d), [&](size_t t) { fill_phys_body(C.pbar, C.d, C.phys, 0, t); });
    forall(cells(C.d), [&](size_t t) { lap_body(C.pbar, C.dres, C.f, C.d, none, 1.0 / (C.h * C.h), 1.0, t); });
    ++q;
  }
  // the single cell
  if (threadIdx.x == 0) {
    const RootLvl& L = S.l[q];
    double sa = 0.0, sb = 0.0;
    for (int face = 0; face < 6; ++face) {
      if (L.phys.kind[face] == BC_PERIODIC || L.phys.kind[face] == BC_ZERO_GRADIENT) {
        sa += 1.0;
      } else {
        sa -= 1.0;
        sb += 2.0 * (L.phys.b[face] ? L.phys.b[face][0] : 0.0);
      }
    }
    if (sa != 6.0) L.u[gx(L.d, 0, 0, 0)] = (sb - L.h * L.h * L.f[gx(L.d, 0, 0, 0)]) / (6.0 - sa);
  }
  __syncthreads();
  // up: correction u - pbar, homogeneous ghosts, trilinear prolongation added, smooth
  for (--q; q >= q0; --q) {
    const RootLvl& L = S.l[q];
    const RootLvl& C = S.l[q + 1];
    forall(cells(C.d), [&](size_t t) { sub_body(C.u, C.pbar, C.tmp, C.d, none, t); });
    forall(ghost_faces(C.d), [&](size_t t) { fill_phys_body(C.tmp, C.d, C.phys, 1, t); });
    forall(cells(L.d), [&](size_t t) {
      prolong_body(C.tmp, C.d, 0, 0, 0, L.u, L.d, 0, 0, 0, none, 0, 0, 0, L.d, 0, t);
    });
    smooth(L, npost);
  }
}

__global__ void __launch_bounds__(kRootTailThreads) k_root_tail(RootSet S, int q0, int npre, int npost, double omega) {
  root_tail_run(S, q0, npre, npost, omega);
}

// ---- the middle of a refined-mesh V-cycle in one workgroup: the Octet levels (one cell per
// MeshBlock of each refinement level) finest first, the root grid, the Octet levels coarsest
// first -- the same operators in the same order as the per-operator launches, for meshes
// whose Octet patches and root grid are small
constexpr int kMidMaxCells = 4096;   // 16^3: four cells per thread and operator
struct OctL {
  Dims d;
  int o[3];
  double h;
  double *u, *f, *pbar, *dres, *tmp;
  int hlo[3], hhi[3];   // the covered box of the next level (patch lam < Lam), local cells
};
struct OctSet {
  OctL l[kMaxSet];
};

static_assert(sizeof(OctSet) + sizeof(RootSet) + 64 <= 4096, "k_mid arguments are limited to 4 KiB");
static_assert(kMpMaxBoxes >= MG_AMR_MAX_LEVELS + 1, "one multipole box per refinement level");

__device__ inline Cons oct_cons(const OctL& F, double* uf, const OctL& C, const double* uc) {
  Cons A;
  A.uf = uf;
  A.df = F.d;
  A.uc = uc;
  A.dc = C.d;
  for (int a = 0; a < 3; ++a) {
    A.lo[a] = C.hlo[a];
    A.hi[a] = C.hhi[a];
  }
  for (int f = 0; f < 6; ++f) A.cg[f] = nullptr;
  return A;
}

__device__ inline size_t cons_most(const Dims& df) {
  size_t m = 0;
  for (int axis = 0; axis < 3; ++axis) {
    const int t1a = axis == 0 ? 1 : 0, t2a = axis == 2 ? 1 : 2;
    m = max(m, (size_t)2 * df.n[t1a] * df.n[t2a]);
  }
  return m;
}

__global__ void __launch_bounds__(kRootTailThreads) k_mid(OctSet O, RootSet R, int Lam, int npre, int npost,
                                                          double omega) {
  const Hole none{};
  auto cons_all = [&](const Cons& A) {
    const size_t m = cons_most(A.df);
    forall(3 * m, [&](size_t t) { cons_body(A, (int)(t / m), t % m); });
  };
  auto oct_smooth = [&](const OctL& P, const OctL& C, int sweeps) {
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        cons_all(oct_cons(P, P.u, C, C.u));
        forall(smooth_items(P.d), [&](size_t t) {
          smooth_body(P.u, P.f, P.d, P.o[0], P.o[1], P.o[2], none, P.h * P.h, omega, colour, t);
        });
      }
  };
  // Octet levels, finest first
  for (int l = Lam; l >= 1; --l) {
    const OctL& P = O.l[l];
    const OctL& C = O.l[l - 1];
    cons_all(oct_cons(P, P.pbar, C, C.pbar));
    forall(cells(P.d), [&](size_t t) { lap_body(P.pbar, P.dres, P.f, P.d, none, 1.0 / (P.h * P.h), 1.0, t); });
    forall(ghosted_d(P.d), [&](size_t t) { P.u[t] = P.pbar[t]; });
    oct_smooth(P, C, npre);
    cons_all(oct_cons(P, P.u, C, C.u));
    forall(cells(P.d), [&](size_t t) { lap_body(P.u, P.f, P.tmp, P.d, none, 1.0 / (P.h * P.h), -1.0, t); });
    const Dims nr{{P.d.n[0] / 2, P.d.n[1] / 2, P.d.n[2] / 2}};
    forall(cells(nr), [&](size_t t) {
      restrict_body(P.u, P.d, none, C.pbar, C.u, C.d, C.hlo[0], C.hlo[1], C.hlo[2], nr, t);
      restrict_body(P.tmp, P.d, none, C.dres, nullptr, C.d, C.hlo[0], C.hlo[1], C.hlo[2], nr, t);
    });
  }
  // root grid
  {
    const RootLvl& L = R.l[0];
    forall(ghost_faces(L.d), [&](size_t t) { fill_phys_body(L.pbar, L.d, L.phys, 0, t); });
    forall(cells(L.d), [&](size_t t) { lap_body(L.pbar, L.dres, L.f, L.d, none, 1.0 / (L.h * L.h), 1.0, t); });
    forall(ghosted_d(L.d), [&](size_t t) { L.u[t] = L.pbar[t]; });
    root_tail_run(R, 0, npre, npost, omega);
  }
  // Octet levels, coarsest first
  for (int l = 1; l <= Lam; ++l) {
    const OctL& P = O.l[l];
    const OctL& C = O.l[l - 1];
    forall(cells(C.d), [&](size_t t) { sub_body(C.u, C.pbar, C.tmp, C.d, none, t); });
    if (l == 1) forall(ghost_faces(C.d), [&](size_t t) { fill_phys_body(C.tmp, C.d, R.l[0].phys, 1, t); });
    forall(cells(P.d), [&](size_t t) {
      prolong_body(C.tmp, C.d, C.o[0], C.o[1], C.o[2], P.u, P.d, P.o[0], P.o[1], P.o[2], none, 0, 0, 0, P.d, 0, t);
    });
    oct_smooth(P, C, npost);
  }
}

// =========================================================================== host plan

struct PatchL {
  Dims d;
  int o[3];       // global origin (cells) at (lam, k)
  double h;
  Hole hole;      // cg pointers filled per use
  double *u, *f, *pbar, *dres, *tmp;
  double* src;    // FMG: the source restricted to this level
  double* cg[6];  // coarse ghosts of the hole faces (lam < Lam)
};

struct Plan {
  int NB, nb, K, Lam, N;      // N = NB * nb root cells per side
  int lo[9][3], hi[9][3];     // boxes (level-(lam-1) block units), index lam - 1
  std::vector<std::vector<PatchL>> P;   // [lam][k]
  // root hierarchy below NB: n = NB/2 .. 1
  std::vector<PatchL> R;
  std::vector<double*> bface;           // per root-side size n (N, N/2, .., 1): 6 arrays
  std::vector<int> bface_n;
  double dx;
};

}  // namespace
}  // namespace mg

using namespace mg;

struct mg_amr_ws {
  void* mem = nullptr;
  size_t cap = 0;
};

namespace {

struct AmrRun {
  Plan pl;
  hipStream_t s;
  double* part;
  double* hpart;   // host copy of partials
  int kinds[6];
  int npre, npost;
  double omega;
  bool gauge_free;

  Phys phys_for(int n, bool hom) const {
    Phys P;
    for (int f = 0; f < 6; ++f) {
      P.kind[f] = kinds[f];
      P.b[f] = nullptr;
    }
    P.bn = n;
    if (!hom)
      for (size_t q = 0; q < pl.bface_n.size(); ++q)
        if (pl.bface_n[q] == n)
          for (int f = 0; f < 6; ++f) P.b[f] = pl.bface.empty() || !pl.bface[q] ? nullptr : pl.bface[q] + (size_t)f * n * n;
    return P;
  }

  void fill_phys(double* u, const Dims& d, bool hom) {
    const Phys P = phys_for(d.n[0], hom);
    hipLaunchKernelGGL(k_fill_phys1, dim3(blocks(ghost_faces(d))), dim3(kB), 0, s, u, d, P, hom ? 1 : 0);
  }

  // conservative ghosts between fine patch (lam) and coarse patch (lam-1) at level k, using
  // arrays uf / uc; writes the coarse ghosts when cg is non-null
  static Cons cons_args(const PatchL& fine, double* uf, const PatchL& coarse, const double* uc, double* const* cg,
                        size_t& most) {
    Cons A;
    A.uf = uf;
    A.df = fine.d;
    A.uc = uc;
    A.dc = coarse.d;
    for (int a = 0; a < 3; ++a) {
      A.lo[a] = coarse.hole.lo[a];
      A.hi[a] = coarse.hole.hi[a];
    }
    for (int f = 0; f < 6; ++f) A.cg[f] = cg ? cg[f] : nullptr;
    for (int axis = 0; axis < 3; ++axis) {
      const int t1a = axis == 0 ? 1 : 0, t2a = axis == 2 ? 1 : 2;
      most = std::max(most, (size_t)2 * fine.d.n[t1a] * fine.d.n[t2a]);
    }
    return A;
  }
  void cons(const PatchL& fine, double* uf, const PatchL& coarse, const double* uc, double* const* cg) {
    Cons A;
    A.uf = uf;
    A.df = fine.d;
    A.uc = uc;
    A.dc = coarse.d;
    for (int a = 0; a < 3; ++a) {
      A.lo[a] = coarse.hole.lo[a];
      A.hi[a] = coarse.hole.hi[a];
    }
    for (int f = 0; f < 6; ++f) A.cg[f] = cg ? cg[f] : nullptr;
    size_t most = 0;
    for (int axis = 0; axis < 3; ++axis) {
      const int t1a = axis == 0 ? 1 : 0, t2a = axis == 2 ? 1 : 2;
      most = std::max(most, (size_t)2 * fine.d.n[t1a] * fine.d.n[t2a]);
    }
    hipLaunchKernelGGL(k_cons, dim3(blocks(most), 3), dim3(kB), 0, s, A);
  }

  Hole hole_of(const PatchL& p) const {
    Hole H = p.hole;
    for (int f = 0; f < 6; ++f) H.cg[f] = p.cg[f];
    return H;
  }

  // ghosts of every patch at level k for the arrays sel(P) (0: u, 1: pbar): the physical
  // ghosts of the root patch, and the level boundary of every finer patch in one launch (each
  // reads active cells only and writes its own ghosts, so the patches are independent)
  void fill_level(int k, int which) {
    auto arr = [&](PatchL& p) { return which == 0 ? p.u : p.pbar; };
    Set<Cons> S{};
    size_t most = ghost_faces(pl.P[0][k].d);
    for (int l = 1; l <= pl.Lam; ++l)
      S.a[l - 1] = cons_args(pl.P[l][k], arr(pl.P[l][k]), pl.P[l - 1][k], arr(pl.P[l - 1][k]), pl.P[l - 1][k].cg, most);
    hipLaunchKernelGGL(k_ghosts_set, dim3(blocks(most), 3, pl.Lam + 1), dim3(kB), 0, s, S, pl.Lam, arr(pl.P[0][k]),
                       pl.P[0][k].d, phys_for(pl.P[0][k].d.n[0], false), 0);
  }

  void smooth_level(int k, int sweeps) {
    Set<SmoothA> S{};
    size_t most = 0;
    for (int l = 0; l <= pl.Lam; ++l) {
      PatchL& p = pl.P[l][k];
      S.a[l] = SmoothA{p.u, p.f, p.d, {p.o[0], p.o[1], p.o[2]}, hole_of(p), p.h * p.h};
      most = std::max(most, smooth_items(p.d));
    }
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        fill_level(k, 0);
        hipLaunchKernelGGL(k_smooth_set, dim3(blocks(most), pl.Lam + 1), dim3(kB), 0, s, S, omega, colour);
      }
  }

  // out[l] = a[l] + s L(arrays) at level k (ghosts filled first)
  void lap_level(int k, int which, int a_sel, int out_sel, double sgn) {
    fill_level(k, which);
    Set<LapA> S{};
    size_t most = 0;
    for (int l = 0; l <= pl.Lam; ++l) {
      PatchL& p = pl.P[l][k];
      const double* u = which == 0 ? p.u : p.pbar;
      const double* a = a_sel == 0 ? p.f : p.dres;
      double* out = out_sel == 0 ? p.tmp : p.f;
      S.a[l] = LapA{u, a, out, p.d, hole_of(p), 1.0 / (p.h * p.h)};
      most = std::max(most, cells(p.d));
    }
    hipLaunchKernelGGL(k_lap_set, dim3(blocks(most), pl.Lam + 1), dim3(kB), 0, s, S, sgn);
  }

  static RestrictA restrict_args(const PatchL& fine, const double* src, bool mask, double* out1, double* out2,
                                 const PatchL& coarse, const int o[3]) {
    RestrictA A;
    A.uf = src;
    A.df = fine.d;
    A.Hf = fine.hole;
    if (!mask) A.Hf.on = 0;
    A.out1 = out1;
    A.out2 = out2;
    A.dc = coarse.d;
    for (int a = 0; a < 3; ++a) A.o[a] = o[a];
    A.nr = Dims{{fine.d.n[0] / 2, fine.d.n[1] / 2, fine.d.n[2] / 2}};
    return A;
  }
  // the restrictions of every patch from level k to k-1: u into pbar and u (masked: covered
  // cells count as 0), the defect in tmp into dres
  void restrict_level(int k) {
    Set<RestrictA> Su{}, Sd{};
    size_t most = 0;
    const int o[3] = {0, 0, 0};
    for (int l = 0; l <= pl.Lam; ++l) {
      PatchL &p = pl.P[l][k], &c = pl.P[l][k - 1];
      Su.a[l] = restrict_args(p, p.u, true, c.pbar, c.u, c, o);
      Sd.a[l] = restrict_args(p, p.tmp, false, c.dres, nullptr, c, o);
      most = std::max(most, cells(Su.a[l].nr));
    }
    hipLaunchKernelGGL(k_restrict_set, dim3(blocks(most), pl.Lam + 1), dim3(kB), 0, s, Su);
    hipLaunchKernelGGL(k_restrict_set, dim3(blocks(most), pl.Lam + 1), dim3(kB), 0, s, Sd);
  }
  // every patch at level k-1 -> k: the prolongated correction tmp added to u (mode 0), or the
  // FMG start from u (mode 2)
  void prolong_level(int k, int mode) {
    Set<ProlongA> S{};
    size_t most = 0;
    for (int l = 0; l <= pl.Lam; ++l) {
      PatchL &c = pl.P[l][k - 1], &p = pl.P[l][k];
      ProlongA& A = S.a[l];
      A.uc = mode == 0 ? c.tmp : c.u;
      A.dc = c.d;
      A.uf = p.u;
      A.df = p.d;
      A.Hf = p.hole;
      for (int a = 0; a < 3; ++a) {
        A.co[a] = c.o[a];
        A.fo[a] = p.o[a];
        A.l[a] = 0;
      }
      A.span = p.d;
      most = std::max(most, cells(p.d));
    }
    hipLaunchKernelGGL(k_prolong_set, dim3(blocks(most), pl.Lam + 1), dim3(kB), 0, s, S, mode);
  }

  void restrict_into(const PatchL& fine, const double* src, bool mask, double* out1, double* out2, const PatchL& coarse,
                     const int o[3]) {
    Dims nr{{fine.d.n[0] / 2, fine.d.n[1] / 2, fine.d.n[2] / 2}};
    Hole H = fine.hole;
    if (!mask) H.on = 0;
    hipLaunchKernelGGL(k_restrict, dim3(blocks(cells(nr))), dim3(kB), 0, s, src, fine.d, H, out1, out2, coarse.d, o[0],
                       o[1], o[2], nr);
  }

  void prolong(const PatchL& coarse, const double* uc, const PatchL& fine, double* uf, int mode, const int lo[3],
               const int hi[3]) {
    Dims span{{hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]}};
    Hole H = fine.hole;
    hipLaunchKernelGGL(k_prolong, dim3(blocks(cells(span))), dim3(kB), 0, s, uc, coarse.d, coarse.o[0], coarse.o[1],
                       coarse.o[2], uf, fine.d, fine.o[0], fine.o[1], fine.o[2], H, lo[0], lo[1], lo[2], span, mode);
  }

  // normal level boundary for prolongation of the corrections held in tmp at level k
  // the arrays tmp (corrections, homogeneous root conditions) or u (the solution, FMG)
  void normal_fill(int k, bool on_u = false) {
    auto arr = [&](PatchL& p) { return on_u ? p.u : p.tmp; };
    for (int l = pl.Lam; l >= 1; --l) {
      PatchL &f = pl.P[l][k], &c = pl.P[l - 1][k];
      restrict_into(f, arr(f), false, arr(c), nullptr, c, c.hole.lo);
    }
    fill_phys(arr(pl.P[0][k]), pl.P[0][k].d, !on_u);
    for (int l = 1; l <= pl.Lam; ++l) {
      PatchL &f = pl.P[l][k], &c = pl.P[l - 1][k];
      const int lo[3] = {-1, -1, -1};
      const int hi[3] = {f.d.n[0] + 1, f.d.n[1] + 1, f.d.n[2] + 1};
      prolong(c, arr(c), f, arr(f), 1, lo, hi);
    }
  }

  void copy(const double* src, double* dst, const Dims& d) {
    hipLaunchKernelGGL(k_copy, dim3(blocks(ghosted(d))), dim3(kB), 0, s, src, dst, ghosted(d));
  }

  // root level n's arrays: n = NB is the root patch, below that pl.R
  PatchL root_level(int n) {
    if (n == pl.NB) {
      PatchL r = pl.P[0][0];
      r.hole.on = 0;
      return r;
    }
    for (auto& q : pl.R)
      if (q.d.n[0] == n) return q;
    return pl.R.back();
  }
  int root_index(int n) const {   // index into pl.R of the level below n
    int q = 0;
    for (int m = pl.NB / 2; m > n / 2 && q < (int)pl.R.size(); m /= 2) ++q;
    return q;
  }

  // cell-volume-weighted mean over the active cells of level k (all patches): one launch and
  // one copy of the partials, summed on the host patch by patch in block order
  double volume_mean(int k, int which_arr, int what) {
    Set<SumA> S{};
    int most = 1;
    for (int l = 0; l <= pl.Lam; ++l) {
      const PatchL& p = pl.P[l][k];
      const double* v = which_arr == 0 ? p.u : which_arr == 1 ? p.f : p.tmp;
      const int nb = (int)std::min<size_t>(kMaxPartials, std::max<size_t>(1, cells(p.d) / (kB * 4)));
      S.a[l] = SumA{v, p.d, hole_of(p), nb};
      most = std::max(most, nb);
    }
    hipLaunchKernelGGL(k_psum_set, dim3(most, pl.Lam + 1), dim3(kB), 0, s, S, what, part, kMaxPartials);
    (void)hipMemcpyAsync(hpart, part, sizeof(double) * kMaxPartials * (pl.Lam + 1), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    double sum = 0.0, vol = 0.0;
    for (int l = 0; l <= pl.Lam; ++l) {
      const PatchL& p = pl.P[l][k];
      const double w = p.h * p.h * p.h;
      double acc = 0.0;
      for (int i = 0; i < S.a[l].nb; ++i) acc += hpart[(size_t)l * kMaxPartials + i];
      sum += w * acc;
      size_t act = cells(p.d);
      if (p.hole.on) act -= (size_t)(p.hole.hi[0] - p.hole.lo[0]) * (p.hole.hi[1] - p.hole.lo[1]) * (p.hole.hi[2] - p.hole.lo[2]);
      vol += w * (double)act;
    }
    return sum / vol;
  }

  // one uniform FAS V-cycle on the root grid (NB^3 down to one cell), physical conditions
  // the root levels as the tail kernel sees them: entry 0 the NB^3 root patch, entry i the
  // level pl.R[i-1]
  RootSet root_set() {
    RootSet S{};
    for (int i = 0; i <= (int)pl.R.size() && i < kMaxRoot; ++i) {
      PatchL p = i == 0 ? pl.P[0][0] : pl.R[i - 1];
      S.l[i] = RootLvl{p.d, p.h, p.u, p.f, p.pbar, p.dres, p.tmp, phys_for(p.d.n[0], false)};
    }
    return S;
  }

  void root_fas(int q, PatchL& top, double* u, double* f) {
    // level q: q = 0 is the NB^3 root patch (u, f given), q >= 1 index into pl.R
    const int n = top.d.n[0];
    if (n <= kRootTailN && (int)pl.R.size() < kMaxRoot && u == top.u && f == top.f) {
      hipLaunchKernelGGL(k_root_tail, dim3(1), dim3(kRootTailThreads), 0, s, root_set(), q, npre, npost, omega);
      return;
    }
    if (n == 1) {
      hipLaunchKernelGGL(k_coarsest, dim3(1), dim3(64), 0, s, u, f, phys_for(1, false), top.h * top.h);
      return;
    }
    const Dims d = top.d;
    Hole none{};
    for (int it = 0; it < npre; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        fill_phys(u, d, false);
        hipLaunchKernelGGL(k_smooth, dim3(blocks(smooth_items(d))), dim3(kB), 0, s, u, f, d, 0, 0, 0, none, top.h * top.h, omega,
                           colour);
      }
    fill_phys(u, d, false);
    hipLaunchKernelGGL(k_lap, dim3(blocks(cells(d))), dim3(kB), 0, s, u, f, top.tmp, d, none, 1.0 / (top.h * top.h),
                       -1.0);
    PatchL& c = pl.R[q];
    const int o[3] = {0, 0, 0};
    restrict_into(top, u, false, c.u, c.pbar, c, o);
    restrict_into(top, top.tmp, false, c.dres, nullptr, c, o);
    fill_phys(c.pbar, c.d, false);
    hipLaunchKernelGGL(k_lap, dim3(blocks(cells(c.d))), dim3(kB), 0, s, c.pbar, c.dres, c.f, c.d, none,
                       1.0 / (c.h * c.h), 1.0);
    root_fas(q + 1, c, c.u, c.f);
    hipLaunchKernelGGL(k_sub, dim3(blocks(cells(c.d))), dim3(kB), 0, s, c.u, c.pbar, c.tmp, c.d, none);
    fill_phys(c.tmp, c.d, true);
    const int lo[3] = {0, 0, 0}, hi[3] = {d.n[0], d.n[1], d.n[2]};
    prolong(c, c.tmp, top, u, 0, lo, hi);
    for (int it = 0; it < npost; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        fill_phys(u, d, false);
        hipLaunchKernelGGL(k_smooth, dim3(blocks(smooth_items(d))), dim3(kB), 0, s, u, f, d, 0, 0, 0, none, top.h * top.h, omega,
                           colour);
      }
  }

  // Octet patch l at k = 0, all cells active, ghosts from patch l-1 (held fixed)
  PatchL octet(int l) const {
    PatchL p = pl.P[l][0];
    p.hole.on = 0;
    return p;
  }
  void octet_smooth(int l, int sweeps) {
    PatchL p = octet(l);
    PatchL& c = pl.P[l - 1][0];
    Hole none{};
    for (int it = 0; it < sweeps; ++it)
      for (int colour = 0; colour < 2; ++colour) {
        cons(p, p.u, c, c.u, nullptr);
        hipLaunchKernelGGL(k_smooth, dim3(blocks(smooth_items(p.d))), dim3(kB), 0, s, p.u, p.f, p.d, p.o[0], p.o[1], p.o[2], none,
                           p.h * p.h, omega, colour);
      }
  }

  // can the middle of a V-cycle (Octet levels, root grid) run in one workgroup?
  bool mid_fits() const {
    if (pl.NB > kRootTailN || (int)pl.R.size() + 1 > kMaxRoot) return false;
    for (int l = 0; l <= pl.Lam; ++l)
      if (cells(pl.P[l][0].d) > (size_t)kMidMaxCells) return false;
    return true;
  }

  // the middle of a V-cycle from its top level, one launch per operator: the Octet levels
  // finest first (from lam_top), the root grid, the Octet levels coarsest first
  void vcycle_middle(int kind, int lam_top) {
    Hole none{};
    // ---- Octet levels, finest first
    for (int l = lam_top; l >= 1; --l) {
      PatchL p = octet(l);
      PatchL& c = pl.P[l - 1][0];
      if (!(kind == 1 && l == lam_top)) {
        cons(p, p.pbar, c, c.pbar, nullptr);
        hipLaunchKernelGGL(k_lap, dim3(blocks(cells(p.d))), dim3(kB), 0, s, p.pbar, p.dres, p.f, p.d, none,
                           1.0 / (p.h * p.h), 1.0);
        (void)hipMemcpyAsync(p.u, p.pbar, ghosted(p.d) * sizeof(double), hipMemcpyDeviceToDevice, s);
      } else {
        copy(p.src, p.f, p.d);
      }
      octet_smooth(l, npre);
      cons(p, p.u, c, c.u, nullptr);
      hipLaunchKernelGGL(k_lap, dim3(blocks(cells(p.d))), dim3(kB), 0, s, p.u, p.f, p.tmp, p.d, none,
                         1.0 / (p.h * p.h), -1.0);
      restrict_into(p, p.u, false, c.pbar, c.u, c, c.hole.lo);
      restrict_into(p, p.tmp, false, c.dres, nullptr, c, c.hole.lo);
    }
    // ---- root grid
    {
      PatchL r = pl.P[0][0];
      r.hole.on = 0;
      fill_phys(r.pbar, r.d, false);
      hipLaunchKernelGGL(k_lap, dim3(blocks(cells(r.d))), dim3(kB), 0, s, r.pbar, r.dres, r.f, r.d, none,
                         1.0 / (r.h * r.h), 1.0);
      (void)hipMemcpyAsync(r.u, r.pbar, ghosted(r.d) * sizeof(double), hipMemcpyDeviceToDevice, s);
      root_fas(0, r, r.u, r.f);
    }
    // ---- Octet levels, coarsest first
    for (int l = 1; l <= lam_top; ++l) {
      PatchL p = octet(l);
      PatchL c = pl.P[l - 1][0];
      c.hole.on = 0;
      hipLaunchKernelGGL(k_sub, dim3(blocks(cells(c.d))), dim3(kB), 0, s, c.u, c.pbar, c.tmp, c.d, none);
      if (l - 1 == 0) fill_phys(c.tmp, c.d, true);
      const int lo[3] = {0, 0, 0}, hi[3] = {p.d.n[0], p.d.n[1], p.d.n[2]};
      prolong(c, c.tmp, p, p.u, 0, lo, hi);
      octet_smooth(l, npost);
    }
  }

  // one FAS V-cycle from the top level: kind 0 MeshBlock level `level`, 1 Octet level `level`,
  // 2 root level `level` (cells per side)
  void vcycle(int kind = 0, int level = -1) {
    const int K = pl.K, Lam = pl.Lam;
    Hole none{};
    if (kind == 2) {
      PatchL top = root_level(level);
      root_fas(root_index(level), top, top.u, top.f);
      return;
    }
    const int kt = kind == 0 ? (level < 0 ? K : level) : 0;
    const int lam_top = kind == 0 ? Lam : level;
    // ---- MeshBlock levels, down
    for (int k = kt; k >= 1; --k) {
      smooth_level(k, npre);
      lap_level(k, 0, 0, 0, -1.0);                      // tmp = f - L u
      restrict_level(k);
      if (k - 1 >= 1) lap_level(k - 1, 1, 1, 1, 1.0);   // f = dres + L pbar
    }
    if (kind == 1) {
      // the uncovered cells of the coarser patches belong to this Octet level's composite
      // problem: phibar = current value, restricted defect = their defect in that problem
      fill_phys(pl.P[0][0].u, pl.P[0][0].d, false);
      for (int l = 1; l <= lam_top; ++l) {
        PatchL f = pl.P[l][0];
        if (l == lam_top) f.hole.on = 0;
        cons(f, f.u, pl.P[l - 1][0], pl.P[l - 1][0].u, pl.P[l - 1][0].cg);
      }
      for (int l = 0; l < lam_top; ++l) {
        PatchL& p = pl.P[l][0];
        hipLaunchKernelGGL(k_lap, dim3(blocks(cells(p.d))), dim3(kB), 0, s, p.u, p.src, p.dres, p.d, hole_of(p),
                           1.0 / (p.h * p.h), -1.0);
        copy(p.u, p.pbar, p.d);
      }
    }
    if (kind == 0 && mid_fits()) {
      // the Octet levels, the root grid and the Octet levels back in one workgroup
      OctSet O{};
      for (int l = 0; l <= Lam; ++l) {
        const PatchL& p = pl.P[l][0];
        O.l[l] = OctL{p.d, {p.o[0], p.o[1], p.o[2]}, p.h, p.u, p.f, p.pbar, p.dres, p.tmp,
                      {p.hole.lo[0], p.hole.lo[1], p.hole.lo[2]}, {p.hole.hi[0], p.hole.hi[1], p.hole.hi[2]}};
      }
      hipLaunchKernelGGL(k_mid, dim3(1), dim3(kRootTailThreads), 0, s, O, root_set(), Lam, npre, npost, omega);
    } else {
      vcycle_middle(kind, lam_top);
    }
    // ---- MeshBlock levels, up
    for (int k = 1; k <= kt; ++k) {
      Set<SubA> S{};
      size_t most = 0;
      for (int l = 0; l <= Lam; ++l) {
        PatchL& c = pl.P[l][k - 1];
        S.a[l] = SubA{c.u, c.pbar, c.tmp, c.d, c.hole};
        most = std::max(most, cells(c.d));
      }
      hipLaunchKernelGGL(k_sub_set, dim3(blocks(most), Lam + 1), dim3(kB), 0, s, S);
      normal_fill(k - 1);
      prolong_level(k, 0);
      smooth_level(k, npost);
    }
  }

  // Alg. 2 on the refined hierarchy (FAS in place of the V-cycle)
  void fmg() {
    const int K = pl.K, Lam = pl.Lam;
    // sources on every level
    for (int k = K; k >= 1; --k)
      for (int l = 0; l <= Lam; ++l) {
        PatchL &p = pl.P[l][k], &c = pl.P[l][k - 1];
        const int o[3] = {0, 0, 0};
        restrict_into(p, p.f, false, c.f, nullptr, c, o);
      }
    for (int k = 0; k <= K; ++k)
      for (int l = 0; l <= Lam; ++l) copy(pl.P[l][k].f, pl.P[l][k].src, pl.P[l][k].d);
    for (int l = Lam; l >= 1; --l) {
      PatchL p = octet(l);
      PatchL& c = pl.P[l - 1][0];
      restrict_into(p, p.src, false, c.src, nullptr, c, c.hole.lo);
    }
    {
      PatchL prev = root_level(pl.NB);
      for (size_t q = 0; q < pl.R.size(); ++q) {
        const int o[3] = {0, 0, 0};
        restrict_into(prev, prev.src, false, pl.R[q].src, nullptr, pl.R[q], o);
        prev = pl.R[q];
      }
    }
    // root levels
    {
      PatchL one = root_level(1);
      copy(one.src, one.f, one.d);
      (void)hipMemsetAsync(one.u, 0, ghosted(one.d) * sizeof(double), s);
      hipLaunchKernelGGL(k_coarsest, dim3(1), dim3(64), 0, s, one.u, one.f, phys_for(1, false), one.h * one.h);
      for (int n = 2; n <= pl.NB; n *= 2) {
        PatchL c = root_level(n / 2), p = root_level(n);
        fill_phys(c.u, c.d, false);
        const int lo[3] = {0, 0, 0}, hi[3] = {n, n, n};
        prolong(c, c.u, p, p.u, 2, lo, hi);
        copy(p.src, p.f, p.d);
        vcycle(2, n);
      }
    }
    // Octet levels
    for (int l = 1; l <= Lam; ++l) {
      PatchL p = octet(l);
      PatchL c = pl.P[l - 1][0];
      c.hole.on = 0;
      const int lo[3] = {0, 0, 0}, hi[3] = {p.d.n[0], p.d.n[1], p.d.n[2]};
      prolong(c, c.u, p, p.u, 2, lo, hi);
      vcycle(1, l);
    }
    // MeshBlock levels
    for (int k = 1; k <= K; ++k) {
      for (int l = 0; l <= Lam; ++l) {
        PatchL& p = pl.P[l][k];
        hipLaunchKernelGGL(k_load_ghosted, dim3(blocks(cells(p.d))), dim3(kB), 0, s, p.src, p.f, p.d, p.hole);
      }
      normal_fill(k - 1, true);
      prolong_level(k, 2);
      vcycle(0, k);
    }
  }

  double residual(double rms_f) {
    lap_level(pl.K, 0, 0, 0, -1.0);
    const double rd = std::sqrt(volume_mean(pl.K, 2, 1));
    return rms_f > 0 ? rd / rms_f : rd;
  }
};

int fail_amr(std::string* err, int code, const char* msg) {
  if (err) *err = msg;
  return code;
}

}  // namespace

// Geometry and validation of a refined mesh: fills the plan's patch dimensions (no memory).
static int amr_plan(const mg_amr_mesh* m, Plan& pl, std::string* err) {
  if (!m) return fail_amr(err, MG_ERR_INVALID_ARG, "null mesh");
  auto pow2 = [](int v) { return v >= 1 && (v & (v - 1)) == 0; };
  if (!pow2(m->NB) || m->NB < 1 || m->NB > 256 || !pow2(m->nb) || m->nb < 2 || m->nb > 64)
    return fail_amr(err, MG_ERR_INVALID_ARG, "NB and nb must be powers of two (NB <= 256, 2 <= nb <= 64)");
  if (m->levels < 0 || m->levels > MG_AMR_MAX_LEVELS) return fail_amr(err, MG_ERR_INVALID_ARG, "levels out of range");
  pl.NB = m->NB;
  pl.nb = m->nb;
  pl.K = ilog2(m->nb);
  pl.Lam = m->levels;
  pl.N = m->NB * m->nb;
  for (int lam = 1; lam <= pl.Lam; ++lam)
    for (int a = 0; a < 3; ++a) {
      const int lo = m->box_lo[lam - 1][a], hi = m->box_hi[lam - 1][a];
      const int plo = lam == 1 ? 0 : 2 * m->box_lo[lam - 2][a];
      const int phi = lam == 1 ? m->NB : 2 * m->box_hi[lam - 2][a];
      if (!(plo + 1 <= lo && lo < hi && hi <= phi - 1))
        return fail_amr(err, MG_ERR_INVALID_ARG, "each box must lie inside its parent with a one-block margin");
      pl.lo[lam - 1][a] = lo;
      pl.hi[lam - 1][a] = hi;
    }
  pl.P.assign(pl.Lam + 1, std::vector<PatchL>(pl.K + 1));
  for (int lam = 0; lam <= pl.Lam; ++lam)
    for (int k = 0; k <= pl.K; ++k) {
      PatchL& p = pl.P[lam][k];
      std::memset(&p, 0, sizeof(p));
      const int c = 1 << k;
      for (int a = 0; a < 3; ++a) {
        const int bo = lam == 0 ? 0 : 2 * pl.lo[lam - 1][a];
        const int bn = lam == 0 ? pl.NB : 2 * (pl.hi[lam - 1][a] - pl.lo[lam - 1][a]);
        p.o[a] = bo * c;
        p.d.n[a] = bn * c;
      }
      p.h = 1.0 / ((double)pl.NB * (double)(1 << lam) * (double)c);
      p.hole.on = lam < pl.Lam;
      if (p.hole.on)
        for (int a = 0; a < 3; ++a) {
          p.hole.lo[a] = pl.lo[lam][a] * c - p.o[a];
          p.hole.hi[a] = pl.hi[lam][a] * c - p.o[a];
        }
    }
  // the kernels decode cell indices in 32 bits (cell_of)
  for (int lam = 0; lam <= pl.Lam; ++lam)
    if (cells(pl.P[lam][pl.K].d) >= ((size_t)1 << 31))
      return fail_amr(err, MG_ERR_UNSUPPORTED, "a refinement level's patch has 2^31 cells or more");
  pl.R.clear();
  for (int n = pl.NB / 2; n >= 1; n /= 2) {
    PatchL p;
    std::memset(&p, 0, sizeof(p));
    p.d = Dims{{n, n, n}};
    p.h = 1.0 / n;
    pl.R.push_back(p);
  }
  return MG_OK;
}

extern "C" {

int mg_amr_patch_dims(const mg_amr_mesh* m, int lam, int dims[3]) {
  Plan pl;
  const int st = amr_plan(m, pl, nullptr);
  if (st != MG_OK) return st;
  if (lam < 0 || lam > pl.Lam || !dims) return MG_ERR_INVALID_ARG;
  for (int a = 0; a < 3; ++a) dims[a] = pl.P[lam][pl.K].d.n[a];
  return MG_OK;
}

}  // extern "C"

// Solve on the refined mesh.  The workspace is the caller's pool (*pool, *pool_cap bytes),
// grown here when the mesh needs more (at most `room` bytes) and kept for the next call.
int amr_solve_impl(int device, const mg_params* p, const mg_amr_mesh* m, const mg_bc* bc, const double* const* rho,
                   double* const* phi, double* hist, int* n_hist, void* stream, double* part, double* hpart,
                   double** pool, size_t* pool_cap, size_t room, std::string* err) {
  Plan pl;
  int st = amr_plan(m, pl, err);
  if (st != MG_OK) return st;
  if (!p || !bc || !rho || !phi || !hist || !n_hist) return fail_amr(err, MG_ERR_INVALID_ARG, "null argument");
  if (p->mode != MG_MODE_MGI && p->mode != MG_MODE_FMG) return fail_amr(err, MG_ERR_INVALID_ARG, "bad mode");
  if (p->precision != MG_PREC_FP64) return fail_amr(err, MG_ERR_UNSUPPORTED, "the refined mesh runs in FP64");
  if (std::fabs(p->dx * pl.N - 1.0) > 1e-12) return fail_amr(err, MG_ERR_INVALID_ARG, "the refined mesh spans the unit cube: dx = 1/(NB nb)");
  bool any_mp = false;
  for (int f = 0; f < 6; ++f) {
    if (bc->kind[f] < 0 || bc->kind[f] > MG_BC_MULTIPOLE) return fail_amr(err, MG_ERR_INVALID_ARG, "bad face kind");
    any_mp |= bc->kind[f] == MG_BC_MULTIPOLE;
  }
  if (any_mp && (bc->lmax < 0 || bc->lmax > 4)) return fail_amr(err, MG_ERR_INVALID_ARG, "lmax outside 0..4");
  for (int a = 0; a < 3; ++a)
    if ((bc->kind[2 * a] == MG_BC_PERIODIC) != (bc->kind[2 * a + 1] == MG_BC_PERIODIC))
      return fail_amr(err, MG_ERR_INVALID_ARG, "periodic faces must be paired per axis");
  for (int l = 0; l <= pl.Lam; ++l)
    if (!rho[l] || !phi[l]) return fail_amr(err, MG_ERR_INVALID_ARG, "null patch array");
  *n_hist = 0;
  if (hipSetDevice(device) != hipSuccess) return fail_amr(err, MG_ERR_DEVICE, "hipSetDevice");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);

  // ---- memory: per patch and level u, f, pbar, dres, tmp (ghosted) and the hole-face ghosts;
  // root levels below NB; fixed-face arrays per root-side size
  size_t total = 0;
  auto take = [&](size_t doubles) {
    const size_t o = total;
    total += (doubles + 31) / 32 * 32;
    return o;
  };
  struct Off {
    size_t u, f, pbar, dres, tmp, src, cg[6];
  };
  std::vector<std::vector<Off>> off(pl.Lam + 1, std::vector<Off>(pl.K + 1));
  for (int l = 0; l <= pl.Lam; ++l)
    for (int k = 0; k <= pl.K; ++k) {
      const size_t g = ghosted(pl.P[l][k].d);
      Off& o = off[l][k];
      o.u = take(g);
      o.f = take(g);
      o.pbar = take(g);
      o.dres = take(g);
      o.tmp = take(g);
      o.src = take(g);
      for (int f = 0; f < 6; ++f) {
        o.cg[f] = (size_t)-1;
        if (pl.P[l][k].hole.on) {
          const Hole& H = pl.P[l][k].hole;
          const int axis = f / 2, t1 = axis == 0 ? 1 : 0, t2 = axis == 2 ? 1 : 2;
          o.cg[f] = take((size_t)(H.hi[t1] - H.lo[t1]) * (H.hi[t2] - H.lo[t2]));
        }
      }
    }
  std::vector<Off> roff(pl.R.size());
  for (size_t q = 0; q < pl.R.size(); ++q) {
    const size_t g = ghosted(pl.R[q].d);
    roff[q].u = take(g);
    roff[q].f = take(g);
    roff[q].pbar = take(g);
    roff[q].dres = take(g);
    roff[q].tmp = take(g);
    roff[q].src = take(g);
  }
  bool any_fixed = any_mp;
  for (int f = 0; f < 6; ++f) any_fixed |= bc->kind[f] == MG_BC_FIXED && bc->fixed_b[f];
  std::vector<size_t> boff;
  if (any_fixed)
    for (int n = pl.N; n >= 1; n /= 2) {
      pl.bface_n.push_back(n);
      boff.push_back(take((size_t)6 * n * n));
    }
  // multipole moments: per-block partials of every patch, then origin and Q_lm (32 values)
  const size_t mp_part = any_mp ? take((size_t)multipole_box_blocks() * (pl.Lam + 1) * 25) : 0;
  const size_t mp_scratch = any_mp ? take(32) : 0;
  const size_t need = total * sizeof(double);
  if (need > *pool_cap) {
    if (need > room) return fail_amr(err, MG_ERR_OOM, "refined-mesh workspace exceeds the context's HBM budget");
    if (*pool) {
      // the old workspace may still be read by earlier work on any stream
      (void)hipDeviceSynchronize();
      (void)hipFree(*pool);
      *pool = nullptr;
      *pool_cap = 0;
    }
    if (hipMalloc(pool, need) != hipSuccess) {
      (void)hipGetLastError();
      *pool = nullptr;
      return fail_amr(err, MG_ERR_OOM, "refined-mesh workspace");
    }
    *pool_cap = need;
  }
  double* mem = *pool;
  (void)hipMemsetAsync(mem, 0, total * sizeof(double), s);
  for (int l = 0; l <= pl.Lam; ++l)
    for (int k = 0; k <= pl.K; ++k) {
      PatchL& q = pl.P[l][k];
      const Off& o = off[l][k];
      q.u = mem + o.u;
      q.f = mem + o.f;
      q.pbar = mem + o.pbar;
      q.dres = mem + o.dres;
      q.tmp = mem + o.tmp;
      q.src = mem + o.src;
      for (int f = 0; f < 6; ++f) q.cg[f] = o.cg[f] == (size_t)-1 ? nullptr : mem + o.cg[f];
    }
  for (size_t q = 0; q < pl.R.size(); ++q) {
    pl.R[q].u = mem + roff[q].u;
    pl.R[q].f = mem + roff[q].f;
    pl.R[q].pbar = mem + roff[q].pbar;
    pl.R[q].dres = mem + roff[q].dres;
    pl.R[q].tmp = mem + roff[q].tmp;
    pl.R[q].src = mem + roff[q].src;
  }
  for (size_t q = 0; q < boff.size(); ++q) pl.bface.push_back(mem + boff[q]);
  if (any_fixed) {
    const int N = pl.N;
    for (int f = 0; f < 6; ++f) {
      if (bc->kind[f] == MG_BC_MULTIPOLE) continue;
      if (bc->kind[f] == MG_BC_FIXED && bc->fixed_b[f])
        (void)hipMemcpyAsync(pl.bface[0] + (size_t)f * N * N, bc->fixed_b[f], sizeof(double) * N * N,
                             hipMemcpyDeviceToDevice, s);
      for (size_t q = 1; q < pl.bface.size(); ++q) {
        const int nc = pl.bface_n[q];
        hipLaunchKernelGGL(k_face_mean, dim3(blocks((size_t)nc * nc)), dim3(kB), 0, s,
                           pl.bface[q - 1] + (size_t)f * 4 * nc * nc, pl.bface[q] + (size_t)f * nc * nc, nc);
      }
    }
  }
  if (any_mp) {
    // Appendix A over the composite grid: the active cells of every patch at the finest
    // level; the expansion is then evaluated at the face centres of every root level
    MpBox boxes[kMpMaxBoxes];
    for (int l = 0; l <= pl.Lam; ++l) {
      const PatchL& q = pl.P[l][pl.K];
      MpBox& B = boxes[l];
      B.rho = rho[l];
      B.h = q.h;
      for (int a = 0; a < 3; ++a) {
        B.n[a] = q.d.n[a];
        B.o[a] = q.o[a];
        B.hlo[a] = q.hole.on ? q.hole.lo[a] : 0;
        B.hhi[a] = q.hole.on ? q.hole.hi[a] : 0;
      }
    }
    double* mps = mem + mp_scratch;
    if (launch_multipole_moments_boxes(boxes, pl.Lam + 1, bc->lmax, bc->use_origin, bc->origin, 0.5, mem + mp_part,
                                       mps, s) != MG_OK) {
      (void)hipStreamSynchronize(s);
      return fail_amr(err, MG_ERR_INVALID_ARG, "too many refinement levels for the multipole moments");
    }
    const double G = p->four_pi_g / (4.0 * M_PI);
    for (size_t q = 0; q < pl.bface.size(); ++q) {
      const int n = pl.bface_n[q];
      double* out[6];
      for (int f = 0; f < 6; ++f)
        out[f] = bc->kind[f] == MG_BC_MULTIPOLE ? pl.bface[q] + (size_t)f * n * n : nullptr;
      launch_multipole_faces(mps, bc->lmax, G, n, 1.0 / n, 1.0, out, s, 0);
    }
  }

  AmrRun R;
  R.pl = pl;
  R.s = s;
  R.part = part;
  R.hpart = hpart;
  for (int f = 0; f < 6; ++f) R.kinds[f] = bc->kind[f] == MG_BC_MULTIPOLE ? MG_BC_FIXED : bc->kind[f];
  R.npre = p->npre;
  R.npost = p->npost;
  R.omega = p->omega;
  R.gauge_free = true;
  for (int f = 0; f < 6; ++f)
    if (bc->kind[f] == MG_BC_FIXED || bc->kind[f] == MG_BC_MULTIPOLE) R.gauge_free = false;

  // ---- source and initial guess on the finest level
  const int K = pl.K;
  for (int l = 0; l <= pl.Lam; ++l) {
    PatchL& q = R.pl.P[l][K];
    hipLaunchKernelGGL(k_load, dim3(blocks(cells(q.d))), dim3(kB), 0, s, rho[l], q.f, q.d, q.hole, p->four_pi_g, 0.0);
    hipLaunchKernelGGL(k_load, dim3(blocks(cells(q.d))), dim3(kB), 0, s, phi[l], q.u, q.d, q.hole, 1.0, 0.0);
  }
  if (R.gauge_free) {
    const double mean = R.volume_mean(K, 1, 0);
    for (int l = 0; l <= pl.Lam; ++l) {
      PatchL& q = R.pl.P[l][K];
      hipLaunchKernelGGL(k_load, dim3(blocks(cells(q.d))), dim3(kB), 0, s, rho[l], q.f, q.d, q.hole, p->four_pi_g,
                         -mean);
    }
  }
  const double rms_f = std::sqrt(R.volume_mean(K, 1, 1));
  if (p->mode == MG_MODE_FMG) R.fmg();
  double r = R.residual(rms_f);
  int nh = 0;
  hist[nh++] = r;
  const int ncyc = p->fixed_cycles > 0 ? p->fixed_cycles : p->max_cycles;
  int status = p->fixed_cycles > 0 ? MG_OK : MG_NOT_CONVERGED;
  int slow = 0;
  if (p->fixed_cycles > 0 || r > p->tol) {
    for (int c = 0; c < ncyc; ++c) {
      R.vcycle();
      const double rn = R.residual(rms_f);
      hist[nh++] = rn;
      if (p->fixed_cycles > 0) {
        r = rn;
        continue;
      }
      slow = rn > 0.9 * r ? slow + 1 : 0;
      r = rn;
      if (r <= p->tol) {
        status = MG_OK;
        break;
      }
      if (slow >= 2) {
        status = MG_STALLED;
        break;
      }
    }
  } else {
    status = MG_OK;
  }
  *n_hist = nh;
  double mean = 0.0;
  if (R.gauge_free) mean = R.volume_mean(K, 0, 0);
  for (int l = 0; l <= pl.Lam; ++l) {
    PatchL& q = R.pl.P[l][K];
    hipLaunchKernelGGL(k_store, dim3(blocks(cells(q.d))), dim3(kB), 0, s, q.u, phi[l], q.d, q.hole, mean);
  }
  const hipError_t e1 = hipStreamSynchronize(s);
  const hipError_t e2 = hipGetLastError();
  if (e1 != hipSuccess || e2 != hipSuccess) return fail_amr(err, MG_ERR_DEVICE, hipGetErrorString(e1 != hipSuccess ? e1 : e2));
  return status;
}
