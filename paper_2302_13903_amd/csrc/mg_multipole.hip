// mg_multipole.hip -- open boundaries from the multipole expansion of Appendix A.
//
// The expansion is phi(r) = -G sum_{l<=lmax} sum_m Q_lm sqrt(4 pi/(2l+1)) Y_lm(r) / r^(l+1)
// with Q_lm = sum rho dV sqrt(4 pi/(2l+1)) r'^l Y_lm(r'), positions relative to the origin
// (centre of mass by default).  The sign makes the monopole -GM/r, the potential that solves
// nabla^2 phi = +4 pi G rho.  Here the factor sqrt(4 pi/(2l+1)) is folded into the real
// harmonics of the paper's table, giving the Schmidt semi-normalised regular solid harmonics
// S_lm(r) = sqrt(4 pi/(2l+1)) r^l Y_lm, which are plain polynomials:
//   Q_lm = sum rho dV S_lm(r'),     phi = -G sum Q_lm S_lm(r) / r^(2l+1).
#include "mg355.h"
#include "mg_common.h"
#include "mg_launch.h"

namespace mg {

constexpr int kMBlock = 256;

// Schmidt semi-normalised regular solid harmonics for l <= 4, index l*l + l + m.
__device__ __forceinline__ void schmidt_solid(double x, double y, double z, double S[25]) {
  const double x2 = x * x, y2 = y * y, z2 = z * z, r2 = x2 + y2 + z2;
  const double s3 = 1.7320508075688772935;     // sqrt(3)
  const double s15 = 3.8729833462074168852;    // sqrt(15)
  const double s35 = 5.9160797830996160426;    // sqrt(35)
  const double s5_8 = 0.79056941504209483300;  // sqrt(5/8)
  const double s3_8 = 0.61237243569579452455;  // sqrt(3/8)
  const double s35_8 = 2.0916500663351888830;  // sqrt(35/8)
  const double s5_2 = 1.1180339887498948482;   // sqrt(5)/2
  S[0] = 1.0;
  S[1] = y;
  S[2] = z;
  S[3] = x;
  S[4] = s3 * x * y;
  S[5] = s3 * y * z;
  S[6] = 0.5 * (3.0 * z2 - r2);
  S[7] = s3 * x * z;
  S[8] = 0.5 * s3 * (x2 - y2);
  S[9] = s5_8 * y * (3.0 * x2 - y2);
  S[10] = s15 * x * y * z;
  S[11] = s3_8 * y * (5.0 * z2 - r2);
  S[12] = 0.5 * z * (5.0 * z2 - 3.0 * r2);
  S[13] = s3_8 * x * (5.0 * z2 - r2);
  S[14] = 0.5 * s15 * z * (x2 - y2);
  S[15] = s5_8 * x * (x2 - 3.0 * y2);
  S[16] = 0.5 * s35 * x * y * (x2 - y2);
  S[17] = s35_8 * y * z * (3.0 * x2 - y2);
  S[18] = s5_2 * x * y * (7.0 * z2 - r2);
  S[19] = s5_8 * y * z * (7.0 * z2 - 3.0 * r2);
  S[20] = 0.125 * (35.0 * z2 * z2 - 30.0 * z2 * r2 + 3.0 * r2 * r2);
  S[21] = s5_8 * x * z * (7.0 * z2 - 3.0 * r2);
  S[22] = 0.5 * s5_2 * (x2 - y2) * (7.0 * z2 - r2);
  S[23] = s35_8 * x * z * (x2 - 3.0 * y2);
  S[24] = 0.125 * s35 * (x2 * (x2 - 3.0 * y2) - y2 * (3.0 * x2 - y2));
}

// Block-wide sums of NV values per thread into part[row * NV + v] (fixed tree).
template <int NV>
__device__ __forceinline__ void block_sums(double* v, double* red, double* part, size_t row) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double a = wave_sum(v[q]);
    if (lane == 0) red[w * NV + q] = a;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double a = 0.0;
    for (int ww = 0; ww < kMBlock / 64; ++ww) a += red[ww * NV + threadIdx.x];
    part[row * NV + threadIdx.x] = a;
  }
}

// Cell (i, j, k) stored at index c of a level of 2^L cells per side: dense (Lm = 0), or the
// MeshBlock layout with 2^Lm-cell blocks in Morton order.
__device__ __forceinline__ void cell_of(size_t c, int L, int Lm, int& i, int& j, int& k) {
  if (Lm == 0) {
    const int n = 1 << L;
    i = (int)(c & (size_t)(n - 1));
    j = (int)((c >> L) & (size_t)(n - 1));
    k = (int)(c >> (2 * L));
    return;
  }
  int bx, by, bz;
  demorton3((unsigned)(c >> (3 * Lm)), bx, by, bz);
  const int r = (int)(c & (size_t)((1 << (3 * Lm)) - 1)), mm = (1 << Lm) - 1;
  i = (bx << Lm) + (r & mm);
  j = (by << Lm) + ((r >> Lm) & mm);
  k = (bz << Lm) + (r >> (2 * Lm));
}

// Mass and first moments: (sum rho dV, sum rho x dV, sum rho y dV, sum rho z dV).
__global__ void __launch_bounds__(kMBlock) k_mass_partials(const double* __restrict__ rho, int L, int Lm, double dx,
                                                            double* __restrict__ part) {
  __shared__ double red[4 * kMBlock / 64];
  const int n = 1 << L;
  const size_t n3 = (size_t)1 << (3 * L);
  const double dv = dx * dx * dx;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t c = (size_t)blockIdx.x * kMBlock + threadIdx.x; c < n3; c += (size_t)gridDim.x * kMBlock) {
    int i, j, k;
    cell_of(c, L, Lm, i, j, k);
    const double m = rho[c] * dv;
    v[0] += m;
    v[1] += m * ((i + 0.5) * dx);
    v[2] += m * ((j + 0.5) * dx);
    v[3] += m * ((k + 0.5) * dx);
  }
  block_sums<4>(v, red, part, blockIdx.x);
}

// scratch layout: [0..3] mass sums, [4..6] origin, [7..31] Q_lm
__global__ void k_set_origin(double* scratch, int use_origin, double ox, double oy, double oz, double centre) {
  if (threadIdx.x != 0) return;
  if (use_origin) {
    scratch[4] = ox; scratch[5] = oy; scratch[6] = oz;
  } else if (fabs(scratch[0]) < 1e-300) {
    scratch[4] = scratch[5] = scratch[6] = centre;
  } else {
    scratch[4] = scratch[1] / scratch[0];
    scratch[5] = scratch[2] / scratch[0];
    scratch[6] = scratch[3] / scratch[0];
  }
}

__global__ void __launch_bounds__(kMBlock) k_moment_partials(const double* __restrict__ rho, int L, int Lm,
                                                              double dx, int lmax, const double* __restrict__ scratch,
                                                              double* __restrict__ part) {
  __shared__ double red[25 * kMBlock / 64];
  const int n = 1 << L;
  const size_t n3 = (size_t)1 << (3 * L);
  const double dv = dx * dx * dx;
  const double ox = scratch[4], oy = scratch[5], oz = scratch[6];
  const int nq = (lmax + 1) * (lmax + 1);
  double acc[25];
#pragma unroll
  for (int q = 0; q < 25; ++q) acc[q] = 0.0;
  for (size_t c = (size_t)blockIdx.x * kMBlock + threadIdx.x; c < n3; c += (size_t)gridDim.x * kMBlock) {
    int i, j, k;
    cell_of(c, L, Lm, i, j, k);
    const double m = rho[c] * dv;
    double S[25];
    schmidt_solid((i + 0.5) * dx - ox, (j + 0.5) * dx - oy, (k + 0.5) * dx - oz, S);
#pragma unroll
    for (int q = 0; q < 25; ++q) acc[q] += q < nq ? m * S[q] : 0.0;
  }
  block_sums<25>(acc, red, part, blockIdx.x);
}

__global__ void __launch_bounds__(kMBlock) k_sum_columns(const double* __restrict__ part, int np, int nv,
                                                          double* __restrict__ out) {
  // out[v] = sum over blocks b (in order) of part[b*nv + v]; one wave per value
  __shared__ double red[kMBlock / 64];
  for (int v = 0; v < nv; ++v) {
    double a = 0.0;
    for (int b = threadIdx.x; b < np; b += kMBlock) a += part[(size_t)b * nv + v];
    a = wave_sum(a);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = 0.0;
      for (int ww = 0; ww < kMBlock / 64; ++ww) r += red[ww];
      out[v] = r;
    }
    __syncthreads();
  }
}

void launch_multipole_moments(const double* rho, int n, int Lm, double dx, int lmax, int use_origin,
                              const double* origin_host, double* part, double* scratch, hipStream_t s) {
  const int L = ilog2(n);
  const size_t n3 = (size_t)1 << (3 * L);
  int nb = reduce_blocks(n3);
  if (!use_origin) {
    hipLaunchKernelGGL(k_mass_partials, dim3(nb), dim3(kMBlock), 0, s, rho, L, Lm, dx, part);
    hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kMBlock), 0, s, part, nb, 4, scratch);
  }
  const double ox = use_origin ? origin_host[0] : 0.0, oy = use_origin ? origin_host[1] : 0.0,
               oz = use_origin ? origin_host[2] : 0.0;
  hipLaunchKernelGGL(k_set_origin, dim3(1), dim3(64), 0, s, scratch, use_origin, ox, oy, oz, 0.5 * n * dx);
  hipLaunchKernelGGL(k_moment_partials, dim3(nb), dim3(kMBlock), 0, s, rho, L, Lm, dx, lmax, scratch, part);
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kMBlock), 0, s, part, nb, 25, scratch + 7);
}

// sum over m of Q_lm S_lm for one l, in increasing m
template <int L>
__device__ __forceinline__ double mp_band(const double* __restrict__ Q, const double (&S)[25]) {
  double sl = 0.0;
#pragma unroll
  for (int q = L * L; q < (L + 1) * (L + 1); ++q) sl += Q[q] * S[q];
  return sl;
}

// Boundary values at the face points of one level: (nl + 2 ext)^2 arrays per face over the
// transverse positions (t + 1/2) hl, t = -ext .. nl - 1 + ext.
__global__ void __launch_bounds__(kMBlock) k_multipole_faces(const double* __restrict__ scratch, int lmax, double G,
                                                              int nl, int ext, double hl, double length, double* f0,
                                                              double* f1, double* f2, double* f3, double* f4,
                                                              double* f5) {
  const int m = nl + 2 * ext;
  const int t = blockIdx.x * kMBlock + threadIdx.x;
  const int face = blockIdx.y;
  if (t >= m * m) return;
  double* out = face == 0 ? f0 : face == 1 ? f1 : face == 2 ? f2 : face == 3 ? f3 : face == 4 ? f4 : f5;
  if (!out) return;
  const double a = (t % m - ext + 0.5) * hl, b = (t / m - ext + 0.5) * hl;
  const double pos = (face & 1) ? length : 0.0;
  const int axis = face >> 1;
  const double x = axis == 0 ? pos : a;
  const double y = axis == 0 ? a : (axis == 1 ? pos : b);
  const double z = axis == 2 ? pos : b;
  const double rx = x - scratch[4], ry = y - scratch[5], rz = z - scratch[6];
  const double r2 = rx * rx + ry * ry + rz * rz;
  const double r = sqrt(r2);
  double S[25];
  schmidt_solid(rx, ry, rz, S);
  const double* Q = scratch + 7;
  // one band per l with compile-time indices, so S stays in registers
  const double r3 = r * r2, r5 = r3 * r2, r7 = r5 * r2, r9 = r7 * r2;   // r^(2l+1)
  double phi = mp_band<0>(Q, S) / r;
  if (lmax >= 1) phi += mp_band<1>(Q, S) / r3;
  if (lmax >= 2) phi += mp_band<2>(Q, S) / r5;
  if (lmax >= 3) phi += mp_band<3>(Q, S) / r7;
  if (lmax >= 4) phi += mp_band<4>(Q, S) / r9;
  out[t] = -G * phi;
}

void launch_multipole_faces(const double* scratch, int lmax, double G, int nl, double hl, double length,
                            double* faces[6], hipStream_t s, int ext) {
  const int m = nl + 2 * ext;
  dim3 g((m * m + kMBlock - 1) / kMBlock, 6);
  hipLaunchKernelGGL(k_multipole_faces, g, dim3(kMBlock), 0, s, scratch, lmax, G, nl, ext, hl, length, faces[0],
                     faces[1], faces[2], faces[3], faces[4], faces[5]);
}

// ---- moments over a set of boxes (the active cells of a composite grid)

struct MpBoxSet {
  MpBox b[kMpMaxBoxes];
};

__device__ __forceinline__ bool box_cell(const MpBox& B, size_t c, int& i, int& j, int& k) {
  i = (int)(c % (size_t)B.n[0]);
  j = (int)((c / (size_t)B.n[0]) % (size_t)B.n[1]);
  k = (int)(c / ((size_t)B.n[0] * B.n[1]));
  return !(i >= B.hlo[0] && i < B.hhi[0] && j >= B.hlo[1] && j < B.hhi[1] && k >= B.hlo[2] && k < B.hhi[2]);
}

// Box blockIdx.y, grid-strided over its cells; partial row blockIdx.y * gridDim.x + blockIdx.x.
__global__ void __launch_bounds__(kMBlock) k_box_mass_partials(MpBoxSet S, double* __restrict__ part) {
  __shared__ double red[4 * kMBlock / 64];
  const MpBox& B = S.b[blockIdx.y];
  const size_t n3 = (size_t)B.n[0] * B.n[1] * B.n[2];
  const double dv = B.h * B.h * B.h;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (size_t c = (size_t)blockIdx.x * kMBlock + threadIdx.x; c < n3; c += (size_t)gridDim.x * kMBlock) {
    int i, j, k;
    if (!box_cell(B, c, i, j, k)) continue;
    const double m = B.rho[c] * dv;
    v[0] += m;
    v[1] += m * ((B.o[0] + i + 0.5) * B.h);
    v[2] += m * ((B.o[1] + j + 0.5) * B.h);
    v[3] += m * ((B.o[2] + k + 0.5) * B.h);
  }
  block_sums<4>(v, red, part, (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

__global__ void __launch_bounds__(kMBlock) k_box_moment_partials(MpBoxSet S, int lmax,
                                                                  const double* __restrict__ scratch,
                                                                  double* __restrict__ part) {
  __shared__ double red[25 * kMBlock / 64];
  const MpBox& B = S.b[blockIdx.y];
  const size_t n3 = (size_t)B.n[0] * B.n[1] * B.n[2];
  const double dv = B.h * B.h * B.h;
  const double ox = scratch[4], oy = scratch[5], oz = scratch[6];
  const int nq = (lmax + 1) * (lmax + 1);
  double acc[25];
#pragma unroll
  for (int q = 0; q < 25; ++q) acc[q] = 0.0;
  for (size_t c = (size_t)blockIdx.x * kMBlock + threadIdx.x; c < n3; c += (size_t)gridDim.x * kMBlock) {
    int i, j, k;
    if (!box_cell(B, c, i, j, k)) continue;
    const double m = B.rho[c] * dv;
    double S25[25];
    schmidt_solid((B.o[0] + i + 0.5) * B.h - ox, (B.o[1] + j + 0.5) * B.h - oy, (B.o[2] + k + 0.5) * B.h - oz,
                  S25);
#pragma unroll
    for (int q = 0; q < 25; ++q) acc[q] += q < nq ? m * S25[q] : 0.0;
  }
  block_sums<25>(acc, red, part, (size_t)blockIdx.y * gridDim.x + blockIdx.x);
}

int multipole_box_blocks() { return 256; }

int launch_multipole_moments_boxes(const MpBox* boxes, int nbox, int lmax, int use_origin, const double* origin_host,
                                   double centre, double* part, double* scratch, hipStream_t s) {
  if (nbox < 1 || nbox > kMpMaxBoxes) return MG_ERR_INVALID_ARG;
  MpBoxSet S{};
  for (int q = 0; q < nbox; ++q) S.b[q] = boxes[q];
  const int nb = multipole_box_blocks();
  const dim3 grid(nb, nbox);
  if (!use_origin) {
    hipLaunchKernelGGL(k_box_mass_partials, grid, dim3(kMBlock), 0, s, S, part);
    hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kMBlock), 0, s, part, nb * nbox, 4, scratch);
  }
  const double ox = use_origin ? origin_host[0] : 0.0, oy = use_origin ? origin_host[1] : 0.0,
               oz = use_origin ? origin_host[2] : 0.0;
  hipLaunchKernelGGL(k_set_origin, dim3(1), dim3(64), 0, s, scratch, use_origin, ox, oy, oz, centre);
  hipLaunchKernelGGL(k_box_moment_partials, grid, dim3(kMBlock), 0, s, S, lmax, scratch, part);
  hipLaunchKernelGGL(k_sum_columns, dim3(1), dim3(kMBlock), 0, s, part, nb * nbox, 25, scratch + 7);
  return MG_OK;
}

}  // namespace mg
