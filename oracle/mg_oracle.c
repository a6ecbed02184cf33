/*
 * mg_oracle.c -- plain FP64 CPU reference of the uniform-grid multigrid Poisson solver
 * of Tomida & Stone, "The Athena++ AMR framework: multigrid solvers for self-gravity"
 * (arXiv:2302.13903).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load this library.  It shares no code, header, table or constant with
 * the HIP path; the product never calls it.
 *
 * Everything is written for clarity, not speed: arrays carry one explicit ghost layer
 * (N_G = 1, Sec. 3.2.1), ghosts are filled before every operator that reads neighbours
 * (Sec. 2.3.6 and Sec. 3.2.4), every loop is a plain triple loop in FP64.
 *
 * Conventions (each a reading of the paper, see the design notes):
 *   - grid arrays are indexed [k][j][i] (x fastest), cell (i,j,k) centred at ((i+1/2)h, ...);
 *     domain [0, n*dx]^3;
 *   - red cells have (i+j+k) even with 0-based active indices (Sec. 2.2, RBGS);
 *   - boundary ghosts: periodic -> opposite active cell, zero-gradient -> adjacent active
 *     cell, fixed / multipole -> 2b - adjacent active cell so that the value on the domain
 *     surface equals b (Sec. 2.3.6); axes are filled x, then y, then z, each pass covering
 *     the ghosts the earlier passes filled, which defines edges and corners;
 *   - coarse-level corrections use homogeneous conditions: periodic and zero-gradient
 *     faces keep their kind, faces with prescribed values become zero-fixed (Sec. 2.3.6);
 *   - the convergence measure is RMS(defect)/RMS(source) on the finest level (Sec. 2.3.7,
 *     eq. threshold, normalised by the source so a relative tolerance can be given).
 *
 * Parity unpinned parts: none; every operator is pinned by the CPU tests.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PERIODIC 0
#define OR_ZERO_GRADIENT 1
#define OR_FIXED 2
#define OR_MULTIPOLE 3

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_STALLED 2
#define OR_ERR_INVALID -1
#define OR_ERR_NONFINITE -5

#define PI 3.14159265358979323846

/* ---------------------------------------------------------------- indexing */

static inline size_t gidx(int n, int i, int j, int k) {
  /* ghosted array of (n+2)^3, active indices 0..n-1, ghosts at -1 and n */
  size_t s = (size_t)(n + 2);
  return ((size_t)(k + 1) * s + (size_t)(j + 1)) * s + (size_t)(i + 1);
}

/* extended face array: (n+2)^2, transverse indices t1,t2 in -1..n */
static inline size_t fidx(int n, int t1, int t2) {
  return (size_t)(t2 + 1) * (size_t)(n + 2) + (size_t)(t1 + 1);
}

typedef struct {
  int kind[6];          /* faces -x,+x,-y,+y,-z,+z */
  const double *b[6];   /* extended face values (n+2)^2 or NULL (= 0) */
} obc;

static double face_b(const obc *bc, int face, int n, int t1, int t2) {
  if (bc->b[face] == NULL) return 0.0;
  return bc->b[face][fidx(n, t1, t2)];
}

/* --------------------------------------------------------- ghost filling */

/* Sec. 2.3.6: set the ghost layer of u from the boundary description. */
static void fill_ghosts(double *u, int n, const obc *bc) {
  for (int axis = 0; axis < 3; ++axis) {
    for (int side = 0; side < 2; ++side) {
      int face = 2 * axis + side;
      int g = side == 0 ? -1 : n;          /* ghost index along axis */
      int a = side == 0 ? 0 : n - 1;       /* adjacent active cell */
      int o = side == 0 ? n - 1 : 0;       /* opposite active cell (periodic) */
      /* transverse ranges: axes already filled include their ghosts */
      int lo1, hi1, lo2, hi2;
      if (axis == 0) { lo1 = 0; hi1 = n; lo2 = 0; hi2 = n; }          /* (y, z) */
      else if (axis == 1) { lo1 = -1; hi1 = n + 1; lo2 = 0; hi2 = n; } /* (x, z) */
      else { lo1 = -1; hi1 = n + 1; lo2 = -1; hi2 = n + 1; }          /* (x, y) */
      for (int t2 = lo2; t2 < hi2; ++t2) {
        for (int t1 = lo1; t1 < hi1; ++t1) {
          size_t ig, ia, io;
          if (axis == 0) { ig = gidx(n, g, t1, t2); ia = gidx(n, a, t1, t2); io = gidx(n, o, t1, t2); }
          else if (axis == 1) { ig = gidx(n, t1, g, t2); ia = gidx(n, t1, a, t2); io = gidx(n, t1, o, t2); }
          else { ig = gidx(n, t1, t2, g); ia = gidx(n, t1, t2, a); io = gidx(n, t1, t2, o); }
          switch (bc->kind[face]) {
            case OR_PERIODIC: u[ig] = u[io]; break;
            case OR_ZERO_GRADIENT: u[ig] = u[ia]; break;
            default: u[ig] = 2.0 * face_b(bc, face, n, t1, t2) - u[ia]; break;
          }
        }
      }
    }
  }
}

/* Homogeneous counterpart of a boundary description, used for the corrections on the
 * coarser levels (Sec. 2.3.6): faces with prescribed values become zero-fixed, periodic
 * faces stay periodic, and zero-gradient faces stay zero-gradient (a zero-gradient face
 * prescribes no value, so its homogeneous form is itself). */
static obc homogeneous(const obc *phys) {
  obc h;
  for (int f = 0; f < 6; ++f) {
    int k = phys->kind[f];
    h.kind[f] = (k == OR_PERIODIC || k == OR_ZERO_GRADIENT) ? k : OR_FIXED;
    h.b[f] = NULL;
  }
  return h;
}

/* ------------------------------------------------------------- operators */

/* eqs. rbsor1/rbsor2: one colour of the over-relaxed red-black Gauss-Seidel smoother. */
static void half_sweep(double *u, const double *f, int n, double h, double omega, int colour,
                       const obc *bc) {
  fill_ghosts(u, n, bc);
  double h2 = h * h;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        if (((i + j + k) & 1) != colour) continue;
        size_t c = gidx(n, i, j, k);
        double nb = u[gidx(n, i - 1, j, k)] + u[gidx(n, i + 1, j, k)] + u[gidx(n, i, j - 1, k)] +
                    u[gidx(n, i, j + 1, k)] + u[gidx(n, i, j, k - 1)] + u[gidx(n, i, j, k + 1)];
        u[c] = u[c] + omega * ((nb - h2 * f[c]) / 6.0 - u[c]);
      }
}

/* SMOOTH(): red half-sweep then black half-sweep (Sec. 2.3.2). */
static void smooth(double *u, const double *f, int n, double h, double omega, const obc *bc) {
  half_sweep(u, f, n, h, omega, 0, bc);
  half_sweep(u, f, n, h, omega, 1, bc);
}

/* eq. defect: d = f - L u with the 7-point Laplacian of eq. discretized2. */
static void defect(double *u, const double *f, double *d, int n, double h, const obc *bc) {
  fill_ghosts(u, n, bc);
  double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t c = gidx(n, i, j, k);
        double nb = u[gidx(n, i - 1, j, k)] + u[gidx(n, i + 1, j, k)] + u[gidx(n, i, j - 1, k)] +
                    u[gidx(n, i, j + 1, k)] + u[gidx(n, i, j, k - 1)] + u[gidx(n, i, j, k + 1)];
        d[c] = f[c] - (nb - 6.0 * u[c]) * ih2;
      }
}

/* eq. restriction: volume-weighted mean of the 8 children (1/8 each on a uniform grid). */
static void restrict8(const double *uf, double *uc, int nc) {
  int nf = 2 * nc;
#pragma omp parallel for schedule(static)
  for (int K = 0; K < nc; ++K)
    for (int J = 0; J < nc; ++J)
      for (int I = 0; I < nc; ++I) {
        double s = 0.0;
        for (int c = 0; c < 2; ++c)
          for (int b = 0; b < 2; ++b)
            for (int a = 0; a < 2; ++a) s += uf[gidx(nf, 2 * I + a, 2 * J + b, 2 * K + c)];
        uc[gidx(nc, I, J, K)] = s / 8.0;
      }
}

/* 1-D prolongation weights for offsets -1, 0, +1 of the coarse neighbour; lower child
 * (even fine index) and upper child (odd).  eq. trilinear and the tricubic FMG weights. */
static void weights(int cubic, int upper, double w[3]) {
  if (!cubic) {
    if (!upper) { w[0] = 0.25; w[1] = 0.75; w[2] = 0.0; }
    else { w[0] = 0.0; w[1] = 0.75; w[2] = 0.25; }
  } else {
    if (!upper) { w[0] = 5.0 / 32.0; w[1] = 30.0 / 32.0; w[2] = -3.0 / 32.0; }
    else { w[0] = -3.0 / 32.0; w[1] = 30.0 / 32.0; w[2] = 5.0 / 32.0; }
  }
}

/* Tensor-product prolongation of a ghost-filled coarse array uc (nc cells) to the fine
 * grid.  add != 0: uf += P uc (correction, Alg. 1 steps 5-6); else uf = P uc (Alg. 2 step 3). */
static void prolong(const double *uc, int nc, double *uf, int cubic, int add) {
  int nf = 2 * nc;
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nf; ++k)
    for (int j = 0; j < nf; ++j)
      for (int i = 0; i < nf; ++i) {
        double wx[3], wy[3], wz[3];
        weights(cubic, i & 1, wx);
        weights(cubic, j & 1, wy);
        weights(cubic, k & 1, wz);
        int I = i >> 1, J = j >> 1, K = k >> 1;
        double s = 0.0;
        for (int c = -1; c <= 1; ++c)
          for (int b = -1; b <= 1; ++b)
            for (int a = -1; a <= 1; ++a) {
              double w = wx[a + 1] * wy[b + 1] * wz[c + 1];
              if (w != 0.0) s += w * uc[gidx(nc, I + a, J + b, K + c)];
            }
        size_t t = gidx(nf, i, j, k);
        uf[t] = add ? uf[t] + s : s;
      }
}

/* COARSEST() on a single cell (Sec. 2.3.2).  Every ghost is an affine function of the
 * cell value, ghost = alpha*u + beta, so the one-cell equation is solved for its fixed
 * point: u = (sum beta - h^2 f) / (6 - sum alpha); u = 0 when sum alpha = 6 (no face
 * fixes the zero point). */
static void coarsest(double *u, const double *f, double h, const obc *bc) {
  double sa = 0.0, sb = 0.0;
  for (int face = 0; face < 6; ++face) {
    if (bc->kind[face] == OR_PERIODIC || bc->kind[face] == OR_ZERO_GRADIENT) {
      sa += 1.0;
    } else {
      sa += -1.0;
      sb += 2.0 * face_b(bc, face, 1, 0, 0);
    }
  }
  size_t c = gidx(1, 0, 0, 0);
  if (sa == 6.0) u[c] = 0.0;
  else u[c] = (sb - h * h * f[c]) / (6.0 - sa);
}

/* ------------------------------------------------------------- reductions */

/* Kahan-compensated sum of g(cell) over the active cells. */
static double sum_active(const double *u, int n, int square) {
  double s = 0.0, comp = 0.0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double v = u[gidx(n, i, j, k)];
        if (square) v = v * v;
        double y = v - comp;
        double t = s + y;
        comp = (t - s) - y;
        s = t;
      }
  return s;
}

/* ------------------------------------------------------------- multipole */

/* Regular solid harmonics r^l Y_{l,m} for l <= 4 written from the real spherical
 * harmonics table of Appendix A (each Y multiplied by r^l, so no division by r).
 * Output order: l = 0..4, m = -l..l  (25 entries). */
static void solid_harmonics(double x, double y, double z, double out[25]) {
  double r2 = x * x + y * y + z * z;
  double x2 = x * x, y2 = y * y, z2 = z * z;
  out[0] = sqrt(1.0 / (4.0 * PI));
  out[1] = sqrt(3.0 / (4.0 * PI)) * y;
  out[2] = sqrt(3.0 / (4.0 * PI)) * z;
  out[3] = sqrt(3.0 / (4.0 * PI)) * x;
  out[4] = sqrt(15.0 / (4.0 * PI)) * x * y;
  out[5] = sqrt(15.0 / (4.0 * PI)) * y * z;
  out[6] = sqrt(5.0 / (16.0 * PI)) * (3.0 * z2 - r2);
  out[7] = sqrt(15.0 / (4.0 * PI)) * x * z;
  out[8] = sqrt(15.0 / (4.0 * PI)) * (x2 - y2) / 2.0;
  out[9] = sqrt(35.0 / (32.0 * PI)) * y * (3.0 * x2 - y2);
  out[10] = sqrt(105.0 / (4.0 * PI)) * x * y * z;
  out[11] = sqrt(21.0 / (32.0 * PI)) * y * (5.0 * z2 - r2);
  out[12] = sqrt(7.0 / (16.0 * PI)) * z * (5.0 * z2 - 3.0 * r2);
  out[13] = sqrt(21.0 / (32.0 * PI)) * x * (5.0 * z2 - r2);
  out[14] = sqrt(105.0 / (4.0 * PI)) * z * (x2 - y2) / 2.0;
  out[15] = sqrt(35.0 / (32.0 * PI)) * x * (x2 - 3.0 * y2);
  out[16] = sqrt(315.0 / (4.0 * PI)) * x * y * (x2 - y2) / 2.0;
  out[17] = sqrt(315.0 / (32.0 * PI)) * y * z * (3.0 * x2 - y2);
  out[18] = sqrt(45.0 / (16.0 * PI)) * x * y * (7.0 * z2 - r2);
  out[19] = sqrt(45.0 / (32.0 * PI)) * y * z * (7.0 * z2 - 3.0 * r2);
  out[20] = sqrt(9.0 / (256.0 * PI)) * (35.0 * z2 * z2 - 30.0 * z2 * r2 + 3.0 * r2 * r2);
  out[21] = sqrt(45.0 / (32.0 * PI)) * x * z * (7.0 * z2 - 3.0 * r2);
  out[22] = sqrt(45.0 / (16.0 * PI)) * (x2 - y2) * (7.0 * z2 - r2) / 2.0;
  out[23] = sqrt(315.0 / (32.0 * PI)) * x * z * (x2 - 3.0 * y2);
  out[24] = sqrt(315.0 / (4.0 * PI)) * (x2 * (x2 - 3.0 * y2) - y2 * (3.0 * x2 - y2)) / 8.0;
}

/* Appendix A: origin (centre of mass unless given) and moments
 * Q_lm = sum rho dV sqrt(4 pi/(2l+1)) r'^l Y_lm(r'). */
void oracle_multipole_moments(int n, double dx, const double *rho, int lmax, int use_origin,
                              const double *origin_in, double *origin_out, double *q) {
  double dv = dx * dx * dx;
  double ox, oy, oz;
  if (use_origin) {
    ox = origin_in[0]; oy = origin_in[1]; oz = origin_in[2];
  } else {
    double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
          double r = rho[((size_t)k * n + j) * n + i] * dv;
          m += r;
          mx += r * (i + 0.5) * dx;
          my += r * (j + 0.5) * dx;
          mz += r * (k + 0.5) * dx;
        }
    if (fabs(m) < 1e-300) {
      ox = oy = oz = 0.5 * n * dx;
    } else {
      ox = mx / m; oy = my / m; oz = mz / m;
    }
  }
  origin_out[0] = ox; origin_out[1] = oy; origin_out[2] = oz;
  for (int t = 0; t < 25; ++t) q[t] = 0.0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        double r = rho[((size_t)k * n + j) * n + i] * dv;
        double s[25];
        solid_harmonics((i + 0.5) * dx - ox, (j + 0.5) * dx - oy, (k + 0.5) * dx - oz, s);
        for (int l = 0; l <= lmax; ++l) {
          double cl = sqrt(4.0 * PI / (2.0 * l + 1.0));
          for (int m = -l; m <= l; ++m) q[l * l + l + m] += r * cl * s[l * l + l + m];
        }
      }
}

/* Appendix A: potential of the truncated expansion at a point, with the sign fixed so
 * the monopole is -G M / r (the sign that solves eq. poisson). */
double oracle_multipole_potential(double x, double y, double z, const double *q, int lmax,
                                  const double *origin, double G) {
  double rx = x - origin[0], ry = y - origin[1], rz = z - origin[2];
  double r = sqrt(rx * rx + ry * ry + rz * rz);
  double s[25];
  solid_harmonics(rx, ry, rz, s);
  double phi = 0.0;
  for (int l = 0; l <= lmax; ++l) {
    double cl = sqrt(4.0 * PI / (2.0 * l + 1.0));
    double rl = pow(r, 2 * l + 1);   /* Y_lm / r^(l+1) = (r^l Y_lm) / r^(2l+1) */
    for (int m = -l; m <= l; ++m) phi += q[l * l + l + m] * cl * s[l * l + l + m] / rl;
  }
  return -G * phi;
}

/* Appendix A over a set of point masses (a composite mesh's active cells, each at its centre
 * with mass rho dV): origin (centre of mass unless given) and the moments Q_lm. */
void oracle_multipole_moments_points(int npts, const double *x, const double *y, const double *z,
                                     const double *mass, int lmax, int use_origin,
                                     const double *origin_in, double *origin_out, double *q) {
  double ox, oy, oz;
  if (use_origin) {
    ox = origin_in[0]; oy = origin_in[1]; oz = origin_in[2];
  } else {
    double m = 0.0, mx = 0.0, my = 0.0, mz = 0.0;
    for (int p = 0; p < npts; ++p) {
      m += mass[p];
      mx += mass[p] * x[p];
      my += mass[p] * y[p];
      mz += mass[p] * z[p];
    }
    if (fabs(m) < 1e-300) {
      ox = oy = oz = 0.5;
    } else {
      ox = mx / m; oy = my / m; oz = mz / m;
    }
  }
  origin_out[0] = ox; origin_out[1] = oy; origin_out[2] = oz;
  for (int t = 0; t < 25; ++t) q[t] = 0.0;
  for (int p = 0; p < npts; ++p) {
    double s[25];
    solid_harmonics(x[p] - ox, y[p] - oy, z[p] - oz, s);
    for (int l = 0; l <= lmax; ++l) {
      double cl = sqrt(4.0 * PI / (2.0 * l + 1.0));
      for (int m = -l; m <= l; ++m) q[l * l + l + m] += mass[p] * cl * s[l * l + l + m];
    }
  }
}

/* The truncated expansion at npts points. */
void oracle_multipole_potential_points(int npts, const double *x, const double *y, const double *z,
                                       const double *q, int lmax, const double *origin, double G,
                                       double *out) {
  for (int p = 0; p < npts; ++p) out[p] = oracle_multipole_potential(x[p], y[p], z[p], q, lmax, origin, G);
}

/* Multipole boundary values at the face points of a level with nl cells of width hl:
 * out[face] is an extended (nl+2)^2 array over transverse positions (t+1/2) hl, t=-1..nl. */
static void multipole_faces(int nl, double hl, double length, const double *q, int lmax,
                            const double *origin, double G, double *out[6]) {
  for (int face = 0; face < 6; ++face) {
    if (out[face] == NULL) continue;
    int axis = face / 2;
    double pos = (face & 1) ? length : 0.0;
    for (int t2 = -1; t2 <= nl; ++t2)
      for (int t1 = -1; t1 <= nl; ++t1) {
        double a = (t1 + 0.5) * hl, b = (t2 + 0.5) * hl, x, y, z;
        if (axis == 0) { x = pos; y = a; z = b; }
        else if (axis == 1) { x = a; y = pos; z = b; }
        else { x = a; y = b; z = pos; }
        out[face][fidx(nl, t1, t2)] = oracle_multipole_potential(x, y, z, q, lmax, origin, G);
      }
  }
}

/* ------------------------------------------------------------ the solver */

typedef struct {
  int n, L, npre, npost;
  double dx, omega, four_pi_g;
  int gauge_free;
  int *nl;            /* cells per side on each level */
  double *hl;         /* cell width on each level */
  double **u, **f, **d;
  obc *phys;          /* physical boundary description per level */
  obc hom;            /* homogeneous description (same on all levels) */
  double *bstore;     /* storage for all per-level face arrays */
  int fas;            /* 1: iterate with the Full Approximation Scheme (Alg. 3) */
  double **pbar;      /* FAS: restricted potential per level (Sec. 3.2.1's extra storage) */
  double rms_f;
  double q[25], origin[3];
} ostate;

static void vcycle(ostate *s, int l, const obc *bc);

/* Alg. 1 (MULTIGRID, correction scheme) on level l with boundary description bc. */
static void vcycle(ostate *s, int l, const obc *bc) {
  int n = s->nl[l];
  double h = s->hl[l];
  if (l == 0) {
    coarsest(s->u[0], s->f[0], h, bc);
    return;
  }
  for (int it = 0; it < s->npre; ++it) smooth(s->u[l], s->f[l], n, h, s->omega, bc);   /* 1 */
  defect(s->u[l], s->f[l], s->d[l], n, h, bc);                                         /* 2 */
  restrict8(s->d[l], s->f[l - 1], n / 2);                                                /* 3 */
  memset(s->u[l - 1], 0, sizeof(double) * (size_t)(n / 2 + 2) * (n / 2 + 2) * (n / 2 + 2));
  vcycle(s, l - 1, &s->hom);                                                             /* 4 */
  fill_ghosts(s->u[l - 1], n / 2, &s->hom);
  prolong(s->u[l - 1], n / 2, s->u[l], 0, 1);                                            /* 5, 6 */
  for (int it = 0; it < s->npost; ++it) smooth(s->u[l], s->f[l], n, h, s->omega, bc);   /* 7 */
}

/* out = L_h u (eq. discretized2) on the active cells, ghosts of u from bc. */
static void laplacian(double *u, double *out, int n, double h, const obc *bc) {
  fill_ghosts(u, n, bc);
  double ih2 = 1.0 / (h * h);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t c = gidx(n, i, j, k);
        double nb = u[gidx(n, i - 1, j, k)] + u[gidx(n, i + 1, j, k)] + u[gidx(n, i, j - 1, k)] +
                    u[gidx(n, i, j + 1, k)] + u[gidx(n, i, j, k - 1)] + u[gidx(n, i, j, k + 1)];
        out[c] = (nb - 6.0 * u[c]) * ih2;
      }
}

/* Alg. 3 (FAS) on level l.  Every level solves the original equation for the potential, so
 * every level uses the physical boundary description at its own geometry (Sec. 2.3.6); the
 * coarse-grid correction psi - phibar then obeys the homogeneous conditions, which its
 * prolongation uses.  On the single coarsest cell the equation is solved with the physical
 * conditions starting from phibar (Sec. 2.3.2): when no face fixes the zero point the cell's
 * value is arbitrary and phibar is kept (a zero correction). */
static void fas(ostate *s, int l) {
  int n = s->nl[l], nc = n / 2;
  double h = s->hl[l];
  const obc *bc = &s->phys[l];
  size_t g3c = (size_t)(nc + 2) * (nc + 2) * (nc + 2);
  for (int it = 0; it < s->npre; ++it) smooth(s->u[l], s->f[l], n, h, s->omega, bc);   /* 1 */
  defect(s->u[l], s->f[l], s->d[l], n, h, bc);                                         /* 2 */
  restrict8(s->d[l], s->d[l - 1], nc);                                                  /* 3 */
  restrict8(s->u[l], s->pbar[l - 1], nc);                                               /* 4 */
  laplacian(s->pbar[l - 1], s->f[l - 1], nc, s->hl[l - 1], &s->phys[l - 1]);            /* 5 */
  for (int k = 0; k < nc; ++k)
    for (int j = 0; j < nc; ++j)
      for (int i = 0; i < nc; ++i) {
        size_t c = gidx(nc, i, j, k);
        s->f[l - 1][c] = s->d[l - 1][c] + s->f[l - 1][c];
      }
  memcpy(s->u[l - 1], s->pbar[l - 1], sizeof(double) * g3c);                           /* 6 */
  if (l - 1 == 0) {
    double keep = s->u[0][gidx(1, 0, 0, 0)];
    coarsest(s->u[0], s->f[0], s->hl[0], &s->phys[0]);
    int fixes = 0;
    for (int face = 0; face < 6; ++face)
      fixes |= s->phys[0].kind[face] != OR_PERIODIC && s->phys[0].kind[face] != OR_ZERO_GRADIENT;
    if (!fixes) s->u[0][gidx(1, 0, 0, 0)] = keep;
  } else {
    fas(s, l - 1);
  }
  for (int k = 0; k < nc; ++k)                                                           /* 7 */
    for (int j = 0; j < nc; ++j)
      for (int i = 0; i < nc; ++i) {
        size_t c = gidx(nc, i, j, k);
        s->u[l - 1][c] = s->u[l - 1][c] - s->pbar[l - 1][c];
      }
  fill_ghosts(s->u[l - 1], nc, &s->hom);
  prolong(s->u[l - 1], nc, s->u[l], 0, 1);                                               /* 8, 9 */
  for (int it = 0; it < s->npost; ++it) smooth(s->u[l], s->f[l], n, h, s->omega, bc);   /* 10 */
}

/* one iteration on level l in the chosen scheme */
static void cycle(ostate *s, int l) {
  if (s->fas) {
    if (l == 0) coarsest(s->u[0], s->f[0], s->hl[0], &s->phys[0]);
    else fas(s, l);
  } else {
    vcycle(s, l, &s->phys[l]);
  }
}

/* Alg. 2 (FMG): coarsest solve, then per level tricubic prolongation and one V-cycle (or one
 * FAS iteration), each level using the physical boundary description evaluated at its own
 * geometry. */
static void fmg(ostate *s) {
  size_t n0 = 27;
  memset(s->u[0], 0, sizeof(double) * n0);
  coarsest(s->u[0], s->f[0], s->hl[0], &s->phys[0]);
  for (int l = 1; l <= s->L; ++l) {
    fill_ghosts(s->u[l - 1], s->nl[l - 1], &s->phys[l - 1]);
    prolong(s->u[l - 1], s->nl[l - 1], s->u[l], 1, 0);
    cycle(s, l);
  }
}

static double residual_norm(ostate *s) {
  int L = s->L, n = s->nl[L];
  defect(s->u[L], s->f[L], s->d[L], n, s->hl[L], &s->phys[L]);
  double sd = sqrt(sum_active(s->d[L], n, 1) / ((double)n * n * n));
  return s->rms_f > 0.0 ? sd / s->rms_f : sd;
}

static int is_pow2(int n) { return n >= 1 && (n & (n - 1)) == 0; }

void oracle_state_destroy(ostate *s) {
  if (!s) return;
  for (int l = 0; l <= s->L; ++l) { free(s->u[l]); free(s->f[l]); free(s->d[l]); free(s->pbar[l]); }
  free(s->u); free(s->f); free(s->d); free(s->pbar); free(s->nl); free(s->hl); free(s->phys); free(s->bstore);
  free(s);
}

/* Build the hierarchy, the source on every level and the per-level boundary values.
 * rho: n^3 (x fastest).  kind: 6 face kinds.  bfix: 6 pointers to n^2 arrays of face
 * values for FIXED faces (NULL = 0).  Returns NULL on invalid input (*err set). */
ostate *oracle_state_create(int n, double dx, double four_pi_g, const double *rho,
                            const int *kind, const double *const *bfix, int lmax,
                            int use_origin, const double *origin, int npre, int npost,
                            double omega, int *err) {
  *err = OR_OK;
  if (!is_pow2(n) || dx <= 0.0 || npre < 0 || npost < 0 || lmax < 0 || lmax > 4) {
    *err = OR_ERR_INVALID;
    return NULL;
  }
  for (int a = 0; a < 3; ++a)
    if ((kind[2 * a] == OR_PERIODIC) != (kind[2 * a + 1] == OR_PERIODIC)) {
      *err = OR_ERR_INVALID;
      return NULL;
    }
  size_t n3 = (size_t)n * n * n;
  for (size_t c = 0; c < n3; ++c)
    if (!isfinite(rho[c])) { *err = OR_ERR_NONFINITE; return NULL; }

  ostate *s = (ostate *)calloc(1, sizeof(ostate));
  s->n = n; s->dx = dx; s->omega = omega; s->four_pi_g = four_pi_g;
  s->npre = npre; s->npost = npost;
  int L = 0;
  while ((1 << L) < n) ++L;
  s->L = L;
  s->nl = (int *)calloc(L + 1, sizeof(int));
  s->hl = (double *)calloc(L + 1, sizeof(double));
  s->u = (double **)calloc(L + 1, sizeof(double *));
  s->f = (double **)calloc(L + 1, sizeof(double *));
  s->d = (double **)calloc(L + 1, sizeof(double *));
  s->pbar = (double **)calloc(L + 1, sizeof(double *));
  s->phys = (obc *)calloc(L + 1, sizeof(obc));
  for (int l = 0; l <= L; ++l) {
    int nl = 1 << l;
    size_t g3 = (size_t)(nl + 2) * (nl + 2) * (nl + 2);
    s->nl[l] = nl;
    s->hl[l] = dx * (double)(1 << (L - l));
    s->u[l] = (double *)calloc(g3, sizeof(double));
    s->f[l] = (double *)calloc(g3, sizeof(double));
    s->d[l] = (double *)calloc(g3, sizeof(double));
    s->pbar[l] = (double *)calloc(g3, sizeof(double));
  }

  /* source f = 4 pi G rho (eq. poisson); mean removed when no face fixes the zero point */
  s->gauge_free = 1;
  for (int face = 0; face < 6; ++face)
    if (kind[face] == OR_FIXED || kind[face] == OR_MULTIPOLE) s->gauge_free = 0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        s->f[L][gidx(n, i, j, k)] = four_pi_g * rho[((size_t)k * n + j) * n + i];
  if (s->gauge_free) {
    double mean = sum_active(s->f[L], n, 0) / (double)n3;
    for (int k = 0; k < n; ++k)
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) s->f[L][gidx(n, i, j, k)] -= mean;
  }
  s->rms_f = sqrt(sum_active(s->f[L], n, 1) / (double)n3);
  /* Alg. 2 step 1: restrict the source to every coarser level */
  for (int l = L; l >= 1; --l) restrict8(s->f[l], s->f[l - 1], s->nl[l - 1]);

  /* boundary values per level */
  size_t bsz = 0;
  for (int l = 0; l <= L; ++l) bsz += 6 * (size_t)(s->nl[l] + 2) * (s->nl[l] + 2);
  s->bstore = (double *)calloc(bsz, sizeof(double));
  double *bp = s->bstore;
  int any_mp = 0;
  for (int face = 0; face < 6; ++face) any_mp |= kind[face] == OR_MULTIPOLE;
  if (any_mp) {
    oracle_multipole_moments(n, dx, rho, lmax, use_origin, origin, s->origin, s->q);
  }
  double G = four_pi_g / (4.0 * PI);
  for (int l = L; l >= 0; --l) {
    int nl = s->nl[l];
    size_t fs = (size_t)(nl + 2) * (nl + 2);
    double *mp_out[6] = {0};
    for (int face = 0; face < 6; ++face) {
      s->phys[l].kind[face] = kind[face];
      s->phys[l].b[face] = NULL;
      if (kind[face] == OR_FIXED || kind[face] == OR_MULTIPOLE) {
        double *b = bp;
        bp += fs;
        s->phys[l].b[face] = b;
        if (kind[face] == OR_MULTIPOLE) {
          mp_out[face] = b;
        } else if (l == L) {
          /* caller's face-centre values; the extension ring copies the nearest value */
          for (int t2 = -1; t2 <= nl; ++t2)
            for (int t1 = -1; t1 <= nl; ++t1) {
              int c1 = t1 < 0 ? 0 : (t1 >= nl ? nl - 1 : t1);
              int c2 = t2 < 0 ? 0 : (t2 >= nl ? nl - 1 : t2);
              b[fidx(nl, t1, t2)] = bfix[face] ? bfix[face][(size_t)c2 * nl + c1] : 0.0;
            }
        } else {
          /* coarser face: area-weighted mean of the 4 finer face values, then extended */
          const double *bf = s->phys[l + 1].b[face];
          int nf = s->nl[l + 1];
          for (int t2 = 0; t2 < nl; ++t2)
            for (int t1 = 0; t1 < nl; ++t1)
              b[fidx(nl, t1, t2)] = (bf[fidx(nf, 2 * t1, 2 * t2)] + bf[fidx(nf, 2 * t1 + 1, 2 * t2)] +
                                     bf[fidx(nf, 2 * t1, 2 * t2 + 1)] + bf[fidx(nf, 2 * t1 + 1, 2 * t2 + 1)]) / 4.0;
          for (int t2 = -1; t2 <= nl; ++t2)
            for (int t1 = -1; t1 <= nl; ++t1) {
              if (t1 >= 0 && t1 < nl && t2 >= 0 && t2 < nl) continue;
              int c1 = t1 < 0 ? 0 : (t1 >= nl ? nl - 1 : t1);
              int c2 = t2 < 0 ? 0 : (t2 >= nl ? nl - 1 : t2);
              b[fidx(nl, t1, t2)] = b[fidx(nl, c1, c2)];
            }
        }
      }
    }
    if (any_mp) multipole_faces(nl, s->hl[l], n * dx, s->q, lmax, s->origin, G, mp_out);
  }
  s->hom = homogeneous(&s->phys[L]);
  return s;
}

void oracle_fmg(ostate *s) { fmg(s); }

/* scheme of the iterations: 0 = correction scheme (Alg. 1), 1 = FAS (Alg. 3) */
void oracle_set_scheme(ostate *s, int fas) { s->fas = fas != 0; }

/* Conditions of the corrections on the coarser levels: 0 = the homogeneous counterpart above
 * (the reading the solver follows), 1 = Sec. 2.3.6 taken literally, zero-fixed on every face
 * that is not periodic (zero-gradient faces too).  The literal rule is kept so that tests can
 * show why it is not the one followed; no solve uses it by default. */
void oracle_set_coarse_rule(ostate *s, int literal) {
  s->hom = homogeneous(&s->phys[s->L]);
  if (literal)
    for (int f = 0; f < 6; ++f)
      if (s->hom.kind[f] == OR_ZERO_GRADIENT) s->hom.kind[f] = OR_FIXED;
}

/* one V-cycle (or FAS iteration) on the finest level; returns the relative residual after it */
double oracle_vcycle(ostate *s) {
  cycle(s, s->L);
  return residual_norm(s);
}

double oracle_residual(ostate *s) { return residual_norm(s); }

void oracle_set_phi(ostate *s, const double *phi) {
  int n = s->n;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) s->u[s->L][gidx(n, i, j, k)] = phi[((size_t)k * n + j) * n + i];
}

/* Final potential; the mean is removed when no face fixes the zero point (Sec. 2.3.6). */
void oracle_get_phi(ostate *s, double *phi) {
  int n = s->n;
  double mean = 0.0;
  if (s->gauge_free) mean = sum_active(s->u[s->L], n, 0) / ((double)n * n * n);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) phi[((size_t)k * n + j) * n + i] = s->u[s->L][gidx(n, i, j, k)] - mean;
}

void oracle_get_origin_moments(ostate *s, double *origin, double *q) {
  for (int a = 0; a < 3; ++a) origin[a] = s->origin[a];
  for (int t = 0; t < 25; ++t) q[t] = s->q[t];
}

/* Whole solve (Sec. 2.3.7): FMG (mode 0) or V-cycles from the given phi (mode 1), with the
 * correction scheme (scheme 0, Alg. 1) or FAS (scheme 1, Alg. 3) as the iteration, then
 * V-cycles until the relative residual is <= tol, stalls (two consecutive cycles each
 * reducing it by less than 10 %), or max_cycles is reached; fixed_cycles > 0 runs exactly
 * that many cycles.  hist receives r after FMG (or of the initial guess) and after each
 * cycle; *n_hist its length. */
int oracle_solve(int n, double dx, double four_pi_g, const double *rho, const int *kind,
                 const double *const *bfix, int lmax, int use_origin, const double *origin,
                 int npre, int npost, double omega, int mode, int scheme, double tol, int max_cycles,
                 int fixed_cycles, double *phi, double *hist, int *n_hist) {
  int err;
  ostate *s = oracle_state_create(n, dx, four_pi_g, rho, kind, bfix, lmax, use_origin, origin,
                                  npre, npost, omega, &err);
  *n_hist = 0;
  if (!s) return err;
  s->fas = scheme != 0;
  if (mode == 0) fmg(s);
  else oracle_set_phi(s, phi);
  double r = residual_norm(s);
  hist[(*n_hist)++] = r;
  int status = OR_OK;
  if (fixed_cycles > 0) {
    for (int c = 0; c < fixed_cycles; ++c) hist[(*n_hist)++] = oracle_vcycle(s);
  } else {
    int slow = 0;
    status = OR_NOT_CONVERGED;
    for (int c = 0; c < max_cycles && r > tol; ++c) {
      double rn = oracle_vcycle(s);
      hist[(*n_hist)++] = rn;
      slow = rn > 0.9 * r ? slow + 1 : 0;
      r = rn;
      if (slow >= 2) { status = OR_STALLED; break; }
    }
    if (r <= tol) status = OR_OK;
  }
  oracle_get_phi(s, phi);
  oracle_state_destroy(s);
  return status;
}

/* ------------------------------------------- operator-level entry points (tests) */

/* The operator entry points take active arrays (n^3, x fastest) and a boundary
 * description given as 6 kinds and 6 extended face arrays ((n+2)^2, NULL = 0). */

static double *to_ghosted(const double *a, int n) {
  double *g = (double *)calloc((size_t)(n + 2) * (n + 2) * (n + 2), sizeof(double));
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) g[gidx(n, i, j, k)] = a[((size_t)k * n + j) * n + i];
  return g;
}

static void from_ghosted(const double *g, int n, double *a) {
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) a[((size_t)k * n + j) * n + i] = g[gidx(n, i, j, k)];
}

static obc make_bc(const int *kind, const double *const *bext) {
  obc bc;
  for (int f = 0; f < 6; ++f) { bc.kind[f] = kind[f]; bc.b[f] = bext ? bext[f] : NULL; }
  return bc;
}

/* ghost-filled copy: out is (n+2)^3 */
void oracle_op_fill(int n, const double *u, const int *kind, const double *const *bext, double *out) {
  obc bc = make_bc(kind, bext);
  double *g = to_ghosted(u, n);
  fill_ghosts(g, n, &bc);
  memcpy(out, g, sizeof(double) * (size_t)(n + 2) * (n + 2) * (n + 2));
  free(g);
}

void oracle_op_half_sweep(int n, double h, double omega, int colour, double *u, const double *f,
                          const int *kind, const double *const *bext) {
  obc bc = make_bc(kind, bext);
  double *gu = to_ghosted(u, n), *gf = to_ghosted(f, n);
  half_sweep(gu, gf, n, h, omega, colour, &bc);
  from_ghosted(gu, n, u);
  free(gu); free(gf);
}

void oracle_op_defect(int n, double h, const double *u, const double *f, double *d,
                      const int *kind, const double *const *bext) {
  obc bc = make_bc(kind, bext);
  double *gu = to_ghosted(u, n), *gf = to_ghosted(f, n), *gd = to_ghosted(f, n);
  defect(gu, gf, gd, n, h, &bc);
  from_ghosted(gd, n, d);
  free(gu); free(gf); free(gd);
}

void oracle_op_restrict(int nc, const double *uf, double *uc) {
  double *gf = to_ghosted(uf, 2 * nc);
  double *gc = (double *)calloc((size_t)(nc + 2) * (nc + 2) * (nc + 2), sizeof(double));
  restrict8(gf, gc, nc);
  from_ghosted(gc, nc, uc);
  free(gf); free(gc);
}

/* cubic = 0: uf += trilinear(uc); cubic = 1: uf = tricubic(uc); ghosts of uc from kind/bext */
void oracle_op_prolong(int nc, const double *uc, double *uf, int cubic, const int *kind,
                       const double *const *bext) {
  obc bc = make_bc(kind, bext);
  double *gc = to_ghosted(uc, nc);
  double *gf = to_ghosted(uf, 2 * nc);
  fill_ghosts(gc, nc, &bc);
  prolong(gc, nc, gf, cubic, !cubic);
  from_ghosted(gf, 2 * nc, uf);
  free(gc); free(gf);
}

void oracle_op_coarsest(double h, double *u, const double *f, const int *kind,
                        const double *const *bext) {
  obc bc = make_bc(kind, bext);
  double gu[27] = {0}, gf[27] = {0};
  gf[gidx(1, 0, 0, 0)] = f[0];
  coarsest(gu, gf, h, &bc);
  u[0] = gu[gidx(1, 0, 0, 0)];
}

/* Gravitational acceleration g = -grad phi (eq. acceleration) in the cell-centred source-term
 * scheme of Sec. 2.4: on each cell face the difference of the two adjacent potentials divided
 * by h, with the sign of -grad; in each cell the mean of its two faces along each axis; and the
 * momentum source rho g.  Ghost potentials across the domain surface follow the boundary rule
 * of Sec. 2.3.6 (fill_ghosts), so a fixed face gives -(phi_0 - b)/(h/2) and a zero-gradient face
 * gives 0.
 *   g     3 n^3: g_x, g_y, g_z, each x fastest;
 *   rhog  3 n^3 or NULL: rho g_x, rho g_y, rho g_z (rho must then be given);
 *   gface 3 n^2 (n+1) or NULL: the face values, x faces as [k][j][i'] with i' = 0..n (face
 *         i' between cells i'-1 and i'), then y faces [k][j'][i], then z faces [k'][j][i]. */
void oracle_gravity(int n, double h, const double *phi, const double *rho, const int *kind,
                    const double *const *bext, double *g, double *rhog, double *gface) {
  obc bc = make_bc(kind, bext);
  double *gp = to_ghosted(phi, n);
  fill_ghosts(gp, n, &bc);
  size_t n3 = (size_t)n * n * n, nf = (size_t)n * n * (n + 1);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) {
        size_t c = ((size_t)k * n + j) * n + i;
        double p0 = gp[gidx(n, i, j, k)];
        /* faces on the low and high side of the cell along x, y, z */
        double fx0 = -(p0 - gp[gidx(n, i - 1, j, k)]) / h, fx1 = -(gp[gidx(n, i + 1, j, k)] - p0) / h;
        double fy0 = -(p0 - gp[gidx(n, i, j - 1, k)]) / h, fy1 = -(gp[gidx(n, i, j + 1, k)] - p0) / h;
        double fz0 = -(p0 - gp[gidx(n, i, j, k - 1)]) / h, fz1 = -(gp[gidx(n, i, j, k + 1)] - p0) / h;
        double cg[3] = {0.5 * (fx0 + fx1), 0.5 * (fy0 + fy1), 0.5 * (fz0 + fz1)};
        for (int a = 0; a < 3; ++a) {
          g[a * n3 + c] = cg[a];
          if (rhog) rhog[a * n3 + c] = rho[c] * cg[a];
        }
        if (gface) {
          gface[((size_t)k * n + j) * (n + 1) + i] = fx0;
          gface[nf + ((size_t)k * (n + 1) + j) * n + i] = fy0;
          gface[2 * nf + ((size_t)k * n + j) * n + i] = fz0;
          if (i == n - 1) gface[((size_t)k * n + j) * (n + 1) + n] = fx1;
          if (j == n - 1) gface[nf + ((size_t)k * (n + 1) + n) * n + i] = fy1;
          if (k == n - 1) gface[2 * nf + ((size_t)n * n + j) * n + i] = fz1;
        }
      }
  free(gp);
}

/* per-level boundary face arrays computed by the solver set-up (for parity of set-up) */
int oracle_state_levels(ostate *s) { return s->L; }

void oracle_state_face(ostate *s, int level, int face, double *out) {
  int nl = s->nl[level];
  size_t fs = (size_t)(nl + 2) * (nl + 2);
  if (s->phys[level].b[face]) memcpy(out, s->phys[level].b[face], fs * sizeof(double));
  else memset(out, 0, fs * sizeof(double));
}

void oracle_state_source(ostate *s, int level, double *out) {
  from_ghosted(s->f[level], s->nl[level], out);
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
