/*
 * lbm_oracle3d.c -- TEST INFRASTRUCTURE, not product code.
 *
 * The three-dimensional form of the step on the D3Q19 lattice (and, compiled
 * from lbm_oracle3d27.c, on the D3Q27 lattice): the same
 * equations as lbm_oracle.c (Z. Guo, arXiv:2012.11075, Sec. II for the
 * standard LBE, Sec. III for the well-balanced one, Sec. IV for the double
 * well), written for D = 3.  Eq. (24) and Eq. (26) are stated for general
 * dimension; in Eq. (26) the last term carries (|c_i|^2/cs2 - D) with D = 3.
 *
 * Conventions (lattice units, cs2 = 1/3, periodic in x, y and z):
 *   - populations array-of-structures, f[((z*ny + y)*nx + x)*Q + i];
 *   - fields phi[(z*ny + y)*nx + x];
 *   - velocities: rest, the 6 axis directions (weight 1/18) and the 12 edge
 *     directions (weight 1/36), in the order listed below; on D3Q27 the 8
 *     corner directions follow, and the weights are 8/27, 2/27, 1/54, 1/216;
 *   - gradient (1/cs2) sum_i w_i c_i phi(x + c_i), Laplacian
 *     (2/cs2) sum_i w_i [phi(x + c_i) - phi(x)]: for a field that varies
 *     along one axis only they are the central difference and the 3-point
 *     Laplacian, as in two dimensions;
 *   - every loop in a fixed order; built with -ffp-contract=off.
 * The readings of lbm_oracle.c (collision sign, equilibrium signs, forcing
 * contraction, half-force velocity, initial populations) carry over.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Lattices smaller than this run their loops on one thread (thread start-up
 * would cost more than the work); the arithmetic is the same either way. */
#define ORC_OMP_MIN_NODES 16384L

#define CS2 (1.0 / 3.0)
#define DIM 3.0

#ifndef ORC3_D3Q27
/* D3Q19: functions orc3_*. */
#define Q3 19
#define ORC3(name) orc3_##name
static const int CX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double WT3[Q3] = {1.0 / 3.0,
                               1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
#else
/* D3Q27 (lbm_oracle3d27.c): rest (8/27), the 6 axis directions (2/27), the
 * 12 edge directions (1/54) in the D3Q19 order, then the 8 corners (1/216)
 * in opposite pairs.  Functions orc27_*. */
#define Q3 27
#define ORC3(name) orc27_##name
static const int CX3[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                            1, -1, 1, -1, 1, -1, -1, 1};
static const int CY3[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1,
                            1, -1, 1, -1, -1, 1, 1, -1};
static const int CZ3[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1,
                            1, -1, -1, 1, 1, -1, 1, -1};
static const double WT3[Q3] = {8.0 / 27.0,
                               2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0, 2.0 / 27.0,
                               1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                               1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0, 1.0 / 54.0,
                               1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0,
                               1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0, 1.0 / 216.0};
#endif

enum { ORC3_STANDARD = 0, ORC3_WELL_BALANCED = 1, ORC3_STANDARD_EQF = 2 };

/* Same layout as orc_params of lbm_oracle.c; force_stencil must be 0. */
typedef struct {
  double tau, beta, kappa, rho_l, rho_v, rho0;
  int force_stencil;
} orc3_params;

static inline int wrap3(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

static double mu0_3(const orc3_params *p, double rho) {
  return 2.0 * p->beta * (rho - p->rho_l) * (rho - p->rho_v) *
         (2.0 * rho - p->rho_l - p->rho_v);
}

/* Equilibrium: Eq. (3) standard, Eq. (24) WB (D = 3). */
void ORC3(feq)(int scheme, const orc3_params *p, double rho, double ux, double uy,
              double uz, double *feq) {
  double uu = ux * ux + uy * uy + uz * uz;
  for (int i = 0; i < Q3; ++i) {
    double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
    double poly = cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    if (scheme != ORC3_WELL_BALANCED)
      feq[i] = WT3[i] * rho * (1.0 + poly);
    else if (i == 0)
      feq[i] = rho - (1.0 - WT3[0]) * p->rho0 - WT3[0] * rho * uu / (2.0 * CS2);
    else
      feq[i] = WT3[i] * (p->rho0 + rho * poly);
  }
}

/* The standard LBE's other forcing term, named after Eq. (5):
 *   F_i = (c_i - u).F feq_i / (cs2 rho), feq of Eq. (3) at (rho, u). */
void ORC3(forcing_eq)(const double *feq, double rho, double ux, double uy, double uz,
                     double Fx, double Fy, double Fz, double *Fi) {
  for (int i = 0; i < Q3; ++i) {
    double cmuF = (CX3[i] - ux) * Fx + (CY3[i] - uy) * Fy + (CZ3[i] - uz) * Fz;
    Fi[i] = cmuF * feq[i] / (CS2 * rho);
  }
}

/* Forcing term: Eq. (5) standard; Eq. (26) WB with G = F + cs2 grad rho and
 * the term (1/2)(|c|^2/cs2 - D)(u . grad rho), D = 3. */
void ORC3(forcing)(int scheme, double ux, double uy, double uz, double Fx, double Fy,
                  double Fz, double grx, double gry, double grz, double *Fi) {
  double Gx = Fx, Gy = Fy, Gz = Fz;
  if (scheme == ORC3_WELL_BALANCED) {
    Gx = Fx + CS2 * grx;
    Gy = Fy + CS2 * gry;
    Gz = Fz + CS2 * grz;
  }
  double uG = ux * Gx + uy * Gy + uz * Gz;
  double ugr = ux * grx + uy * gry + uz * grz;
  for (int i = 0; i < Q3; ++i) {
    double cF = CX3[i] * Fx + CY3[i] * Fy + CZ3[i] * Fz;
    double cu = CX3[i] * ux + CY3[i] * uy + CZ3[i] * uz;
    double cG = CX3[i] * Gx + CY3[i] * Gy + CZ3[i] * Gz;
    double v = cF / CS2 + (cu * cG - CS2 * uG) / (CS2 * CS2);
    if (scheme == ORC3_WELL_BALANCED) {
      double c2 = (double)(CX3[i] * CX3[i] + CY3[i] * CY3[i] + CZ3[i] * CZ3[i]);
      v += 0.5 * (c2 / CS2 - DIM) * ugr;
    }
    Fi[i] = WT3[i] * v;
  }
}

static inline size_t idx3(int x, int y, int z, int nx, int ny) {
  return ((size_t)z * ny + y) * nx + x;
}

/* Isotropic central gradient, periodic. */
void ORC3(gradient)(int nx, int ny, int nz, const double *phi, double *gx, double *gy,
                   double *gz) {
#pragma omp parallel for schedule(static) if ((long)nx * ny * nz >= ORC_OMP_MIN_NODES)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int i = 1; i < Q3; ++i) {
          double v = phi[idx3(wrap3(x + CX3[i], nx), wrap3(y + CY3[i], ny), wrap3(z + CZ3[i], nz), nx, ny)];
          sx += WT3[i] * CX3[i] * v;
          sy += WT3[i] * CY3[i] * v;
          sz += WT3[i] * CZ3[i] * v;
        }
        size_t k = idx3(x, y, z, nx, ny);
        gx[k] = sx / CS2;
        gy[k] = sy / CS2;
        gz[k] = sz / CS2;
      }
}

/* Isotropic Laplacian, periodic. */
void ORC3(laplacian)(int nx, int ny, int nz, const double *phi, double *lap) {
#pragma omp parallel for schedule(static) if ((long)nx * ny * nz >= ORC_OMP_MIN_NODES)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx3(x, y, z, nx, ny);
        double c = phi[k], s = 0.0;
        for (int i = 1; i < Q3; ++i) {
          double v = phi[idx3(wrap3(x + CX3[i], nx), wrap3(y + CY3[i], ny), wrap3(z + CZ3[i], nz), nx, ny)];
          s += WT3[i] * (v - c);
        }
        lap[k] = 2.0 * s / CS2;
      }
}

/* rho, u, mu, F and grad rho of the state f (Eqs. 4, 6, 25 in 3-D). */
void ORC3(macro)(int scheme, const orc3_params *p, int nx, int ny, int nz, const double *f,
                double *rho, double *ux, double *uy, double *uz, double *mu, double *Fx,
                double *Fy, double *Fz, double *grx, double *gry, double *grz) {
  size_t n = (size_t)nx * ny * nz;
  double *lap = (double *)malloc(n * sizeof(double));
  double *gmx = (double *)malloc(3 * n * sizeof(double));
  double *gmy = gmx + n, *gmz = gmx + 2 * n;
  for (size_t k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = 0; i < Q3; ++i) s += f[k * Q3 + i];
    rho[k] = s;
  }
  ORC3(laplacian)(nx, ny, nz, rho, lap);
  for (size_t k = 0; k < n; ++k) mu[k] = mu0_3(p, rho[k]) - p->kappa * lap[k];
  ORC3(gradient)(nx, ny, nz, mu, gmx, gmy, gmz);
  ORC3(gradient)(nx, ny, nz, rho, grx, gry, grz);
  for (size_t k = 0; k < n; ++k) {
    double fx = -rho[k] * gmx[k], fy = -rho[k] * gmy[k], fz = -rho[k] * gmz[k];
    if (scheme != ORC3_WELL_BALANCED) {
      fx += CS2 * grx[k];
      fy += CS2 * gry[k];
      fz += CS2 * grz[k];
    }
    Fx[k] = fx;
    Fy[k] = fy;
    Fz[k] = fz;
    double mx = 0.0, my = 0.0, mz = 0.0;
    for (int i = 0; i < Q3; ++i) {
      mx += CX3[i] * f[k * Q3 + i];
      my += CY3[i] * f[k * Q3 + i];
      mz += CZ3[i] * f[k * Q3 + i];
    }
    ux[k] = (mx + 0.5 * fx) / rho[k];
    uy[k] = (my + 0.5 * fy) / rho[k];
    uz[k] = (mz + 0.5 * fz) / rho[k];
  }
  free(lap);
  free(gmx);
}

/* f_i = feq_i(rho, u); any of ux, uy, uz NULL means 0. */
void ORC3(init)(int scheme, const orc3_params *p, int nx, int ny, int nz, const double *rho,
               const double *ux, const double *uy, const double *uz, double *f) {
  size_t n = (size_t)nx * ny * nz;
  for (size_t k = 0; k < n; ++k)
    ORC3(feq)(scheme, p, rho[k], ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, uz ? uz[k] : 0.0, f + k * Q3);
}

/* n steps of Eq. (2): collide, then stream to x + c_i; f in place. */
void ORC3(step)(int scheme, const orc3_params *p, int nx, int ny, int nz, double *f,
               int64_t nsteps) {
  size_t n = (size_t)nx * ny * nz;
  double *buf = (double *)malloc(11 * n * sizeof(double));
  double *rho = buf, *ux = buf + n, *uy = buf + 2 * n, *uz = buf + 3 * n, *mu = buf + 4 * n;
  double *Fx = buf + 5 * n, *Fy = buf + 6 * n, *Fz = buf + 7 * n;
  double *grx = buf + 8 * n, *gry = buf + 9 * n, *grz = buf + 10 * n;
  double *g = (double *)malloc(n * Q3 * sizeof(double));
  double omega = 1.0 / p->tau, fpre = 1.0 - 0.5 / p->tau;
  for (int64_t s = 0; s < nsteps; ++s) {
    ORC3(macro)(scheme, p, nx, ny, nz, f, rho, ux, uy, uz, mu, Fx, Fy, Fz, grx, gry, grz);
#pragma omp parallel for schedule(static) if ((long)nx * ny * nz >= ORC_OMP_MIN_NODES)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          size_t k = idx3(x, y, z, nx, ny);
          double feq[Q3], Fi[Q3];
          ORC3(feq)(scheme, p, rho[k], ux[k], uy[k], uz[k], feq);
          if (scheme == ORC3_STANDARD_EQF)
            ORC3(forcing_eq)(feq, rho[k], ux[k], uy[k], uz[k], Fx[k], Fy[k], Fz[k], Fi);
          else
            ORC3(forcing)(scheme, ux[k], uy[k], uz[k], Fx[k], Fy[k], Fz[k], grx[k], gry[k], grz[k],
                         Fi);
          for (int i = 0; i < Q3; ++i) {
            double fs = f[k * Q3 + i] - omega * (f[k * Q3 + i] - feq[i]) + fpre * Fi[i];
            size_t d = idx3(wrap3(x + CX3[i], nx), wrap3(y + CY3[i], ny), wrap3(z + CZ3[i], nz), nx, ny);
            g[d * Q3 + i] = fs;
          }
        }
    memcpy(f, g, n * Q3 * sizeof(double));
  }
  free(buf);
  free(g);
}

static inline void neumaier3(double *sum, double *comp, double v) {
  double t = *sum + v;
  if (fabs(*sum) >= fabs(v))
    *comp += (*sum - t) + v;
  else
    *comp += (v - t) + *sum;
  *sum = t;
}

/* out[0] max|u|, out[1] mass (compensated), out[2] kinetic energy
 * (compensated), out[3] 1 if any rho or u is non-finite or rho <= 0,
 * out[4..6] total momentum sum rho u (compensated, half-force u of Eq. 4). */
void ORC3(observe)(int scheme, const orc3_params *p, int nx, int ny, int nz, const double *f,
                  double *out) {
  size_t n = (size_t)nx * ny * nz;
  double *b = (double *)malloc(11 * n * sizeof(double));
  ORC3(macro)(scheme, p, nx, ny, nz, f, b, b + n, b + 2 * n, b + 3 * n, b + 4 * n, b + 5 * n,
             b + 6 * n, b + 7 * n, b + 8 * n, b + 9 * n, b + 10 * n);
  double umax = 0.0, ms = 0.0, mc = 0.0, es = 0.0, ec = 0.0, bad = 0.0;
  double ps[3] = {0.0, 0.0, 0.0}, pc[3] = {0.0, 0.0, 0.0};
  for (size_t k = 0; k < n; ++k) {
    double r = b[k], u2 = b[n + k] * b[n + k] + b[2 * n + k] * b[2 * n + k] + b[3 * n + k] * b[3 * n + k];
    double um = sqrt(u2);
    if (!isfinite(r) || !isfinite(um) || !(r > 0.0)) bad = 1.0;
    if (um > umax) umax = um;
    neumaier3(&ms, &mc, r);
    neumaier3(&es, &ec, 0.5 * r * u2);
    for (int a = 0; a < 3; ++a) neumaier3(&ps[a], &pc[a], r * b[(size_t)(a + 1) * n + k]);
  }
  out[0] = umax;
  out[1] = ms + mc;
  out[2] = es + ec;
  out[3] = bad;
  for (int a = 0; a < 3; ++a) out[4 + a] = ps[a] + pc[a];
  free(b);
}
