/*
 * lbm_oracle.c -- TEST INFRASTRUCTURE, not product code.
 *
 * A plain, slow, double-precision CPU reference of the D2Q9 lattice Boltzmann
 * step for a two-phase fluid driven by a chemical potential, in the two forms
 * compared by Z. Guo, "Well-balanced lattice Boltzmann equation for two-phase
 * flows" (arXiv:2012.11075):
 *
 *   - the standard LBE  : Sec. II, Eqs. (2)-(5) with the potential-form force
 *                         F = grad(cs2 rho) - rho grad(mu)          (Eq. 6)
 *   - the standard LBE with the other forcing term the paper names after
 *     Eq. (5): F_i = (c_i - u).F feq_i / (cs2 rho), same equilibrium and
 *     force (scheme ORC_STANDARD_EQF)
 *   - the well-balanced : Sec. III, Eq. (2) with the equilibrium of Eq. (24),
 *     (WB) LBE            the force F = -rho grad(mu) of Eq. (25) and the
 *                         forcing term of Eq. (26)
 *
 * with the double-well bulk free energy of Sec. IV, Eqs. (36)-(37).
 *
 * Only tests, the smoke entry and the CPU-baseline leg of the benchmark may
 * load this file's library.  It shares no code with the GPU path.
 *
 * Conventions (lattice units, c = dx = dt = 1, cs2 = 1/3):
 *   - populations are stored array-of-structures, f[(y*nx + x)*9 + i];
 *   - scalar fields are stored row-major, phi[y*nx + x];
 *   - the lattice is periodic in x and y;
 *   - every loop runs in a fixed order; build with -ffp-contract=off so that
 *     no multiply-add is fused.
 *
 * Readings of the paper taken here (where the text is garbled or silent):
 *   - Eq. (2): the collision term enters with a minus sign, f - (f-feq)/tau;
 *     the steady-state relation below Eq. (8) follows only with that sign.
 *   - Eq. (2) text: the sixth velocity is c6 = -c8 = (-1, 1).
 *   - Eq. (3): quadratic terms are +(c.u)^2/(2 cs4) - u.u/(2 cs2), the signs
 *     that Eq. (24) prints and that give the second moment cs2 rho I + rho uu.
 *   - Eq. (5): uF:(cc - cs2 I) = (c.u)(c.F) - cs2 (u.F).
 *   - Gradients (Sec. II, isotropic central scheme): in 2-D the weighted
 *     central difference grad(phi) = (1/cs2) sum_i w_i c_i phi(x + c_i), which
 *     reduces to (phi_{j+1} - phi_{j-1})/2 for a one-dimensional field.
 *   - Laplacian in mu = mu0 - kappa lap(rho): the isotropic 9-point form of
 *     the same family, lap(phi) = (2/cs2) sum_i w_i [phi(x + c_i) - phi(x)],
 *     which reduces to phi_{j+1} - 2 phi_j + phi_{j-1} in 1-D.
 *   - The grad(rho) inside the WB forcing term (Eq. 26) and inside the
 *     standard force is the same isotropic gradient.
 *   - u inside feq and F_i is the half-force velocity of Eq. (4), with the
 *     force evaluated from the fields at time t (explicit; F does not depend
 *     on u).
 *   - The WB constant rho0 of Eq. (24) is a parameter; the paper uses 0.
 *   - Force-stencil variant (Sec. II, after Eq. 23: higher-order gradients in
 *     the force reduce but cannot remove the net force): with force_stencil
 *     = 1 every gradient in the force and in Eq. (26) is the fourth-order
 *     gradient grad(phi) - (1/6) grad(lap(phi)) built from the two stencils
 *     above; it removes the isotropic second-order error of the central
 *     scheme and reduces to (-phi_{j+2} + 8 phi_{j+1} - 8 phi_{j-1} +
 *     phi_{j-2})/12 in 1-D.
 *   - Initial populations: f_i(0) = feq_i(rho, u) of the scheme in use.
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

#define Q 9
#define CS2 (1.0 / 3.0)
#define DIM 2.0

/* D2Q9 velocities in the paper's numbering (Sec. II, below Eq. 2). */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Weights (below Eq. 3). */
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

enum { ORC_STANDARD = 0, ORC_WELL_BALANCED = 1, ORC_STANDARD_EQF = 2 };

typedef struct {
  double tau;   /* relaxation time, Eq. (2) */
  double beta;  /* double-well height, Eq. (36) */
  double kappa; /* gradient-energy coefficient, Sec. II and Eq. (35) */
  double rho_l; /* saturation liquid density, Eq. (36) */
  double rho_v; /* saturation vapour density, Eq. (36) */
  double rho0;  /* constant in the WB equilibrium, Eq. (24) */
  int force_stencil; /* gradients of the force: 0 the isotropic central
                        scheme (Sec. II), 1 the fourth-order form below */
} orc_params;

static inline int wrap(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

/* ---------------------------------------------------------------- node level */

/* Bulk chemical potential mu0 = d psi0 / d rho, psi0 = beta (rho-rl)^2
 * (rho-rv)^2 (Eqs. 36-37). */
double orc_mu0(const orc_params *p, double rho) {
  return 2.0 * p->beta * (rho - p->rho_l) * (rho - p->rho_v) *
         (2.0 * rho - p->rho_l - p->rho_v);
}

/* Bulk free energy psi0 (Eq. 36). */
double orc_psi0(const orc_params *p, double rho) {
  double a = rho - p->rho_l, b = rho - p->rho_v;
  return p->beta * a * a * b * b;
}

/* Thermodynamic pressure p0 = rho mu0 - psi0 (Eq. 37, read as rho dpsi0/drho
 * - psi0). */
double orc_p0(const orc_params *p, double rho) {
  return rho * orc_mu0(p, rho) - orc_psi0(p, rho);
}

/* Equilibrium populations.
 * Standard, Eq. (3):  feq_i = w_i rho [1 + c.u/cs2 + (c.u)^2/(2cs4) - u.u/(2cs2)]
 * WB, Eq. (24):       feq_0 = rho - (1-w0) rho0 - w0 rho u.u/(2cs2)
 *                     feq_i = w_i {rho0 + rho [c.u/cs2 + (c.u)^2/(2cs4)
 *                                               - u.u/(2cs2)]},   i != 0 */
void orc_feq(int scheme, const orc_params *p, double rho, double ux, double uy,
             double *feq) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < Q; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    double poly = cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2);
    if (scheme != ORC_WELL_BALANCED) {
      feq[i] = WT[i] * rho * (1.0 + poly);
    } else if (i == 0) {
      feq[i] = rho - (1.0 - WT[0]) * p->rho0 - WT[0] * rho * uu / (2.0 * CS2);
    } else {
      feq[i] = WT[i] * (p->rho0 + rho * poly);
    }
  }
}

/* Forcing term F_i of the standard LBE named after Eq. (5):
 *   F_i = (c_i - u).F feq_i / (cs2 rho)
 * with feq the standard equilibrium of Eq. (3) at (rho, u). */
void orc_forcing_eq(const double *feq, double rho, double ux, double uy,
                    double Fx, double Fy, double *Fi) {
  for (int i = 0; i < Q; ++i) {
    double cmuF = (CX[i] - ux) * Fx + (CY[i] - uy) * Fy;
    Fi[i] = cmuF * feq[i] / (CS2 * rho);
  }
}

/* Forcing term F_i.
 * Standard, Eq. (5): w_i [c.F/cs2 + uF:(cc - cs2 I)/cs4]
 * WB, Eq. (26):      w_i [c.F/cs2 + u(F + cs2 grad rho):(cc - cs2 I)/cs4
 *                         + (1/2)(|c|^2/cs2 - D)(u.grad rho)]
 * with aF:(cc - cs2 I) = (c.a)(c.F) - cs2 (a.F) for vectors a, F.
 * (grx, gry) = grad rho; unused by the standard scheme. */
void orc_forcing(int scheme, double ux, double uy, double Fx, double Fy,
                 double grx, double gry, double *Fi) {
  double Gx = Fx, Gy = Fy;
  if (scheme == ORC_WELL_BALANCED) {
    Gx = Fx + CS2 * grx;
    Gy = Fy + CS2 * gry;
  }
  double uG = ux * Gx + uy * Gy;
  double ugr = ux * grx + uy * gry;
  for (int i = 0; i < Q; ++i) {
    double cF = CX[i] * Fx + CY[i] * Fy;
    double cu = CX[i] * ux + CY[i] * uy;
    double cG = CX[i] * Gx + CY[i] * Gy;
    double c2 = (double)(CX[i] * CX[i] + CY[i] * CY[i]);
    double t = cF / CS2 + (cu * cG - CS2 * uG) / (CS2 * CS2);
    if (scheme == ORC_WELL_BALANCED) t += 0.5 * (c2 / CS2 - DIM) * ugr;
    Fi[i] = WT[i] * t;
  }
}

/* --------------------------------------------------------------- field level */

/* Isotropic central gradient, grad(phi)(x) = (1/cs2) sum_i w_i c_i phi(x+c_i),
 * periodic. */
void orc_gradient(int nx, int ny, const double *phi, double *gx, double *gy) {
#pragma omp parallel for schedule(static) if ((long)nx * ny >= ORC_OMP_MIN_NODES)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      double sx = 0.0, sy = 0.0;
      for (int i = 1; i < Q; ++i) {
        double v = phi[wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx)];
        sx += WT[i] * CX[i] * v;
        sy += WT[i] * CY[i] * v;
      }
      gx[y * nx + x] = sx / CS2;
      gy[y * nx + x] = sy / CS2;
    }
  }
}

/* Isotropic Laplacian, lap(phi)(x) = (2/cs2) sum_i w_i [phi(x+c_i) - phi(x)],
 * periodic. */
void orc_laplacian(int nx, int ny, const double *phi, double *lap) {
#pragma omp parallel for schedule(static) if ((long)nx * ny >= ORC_OMP_MIN_NODES)
  for (int y = 0; y < ny; ++y) {
    for (int x = 0; x < nx; ++x) {
      double c = phi[y * nx + x];
      double s = 0.0;
      for (int i = 1; i < Q; ++i) {
        double v = phi[wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx)];
        s += WT[i] * (v - c);
      }
      lap[y * nx + x] = 2.0 * s / CS2;
    }
  }
}

/* Fourth-order gradient: the isotropic central gradient of phi minus one
 * sixth of the isotropic central gradient of lap(phi).  The central
 * gradient's leading error is (1/6) grad(lap(phi)); subtracting it leaves a
 * fourth-order error.  Periodic. */
void orc_gradient4(int nx, int ny, const double *phi, double *gx, double *gy) {
  size_t n = (size_t)nx * ny;
  double *lap = (double *)malloc(n * sizeof(double));
  double *lx = (double *)malloc(n * sizeof(double));
  double *ly = (double *)malloc(n * sizeof(double));
  orc_laplacian(nx, ny, phi, lap);
  orc_gradient(nx, ny, phi, gx, gy);
  orc_gradient(nx, ny, lap, lx, ly);
  for (size_t k = 0; k < n; ++k) {
    gx[k] -= lx[k] / 6.0;
    gy[k] -= ly[k] / 6.0;
  }
  free(lap);
  free(lx);
  free(ly);
}

/* All macroscopic fields at time t from the populations f(t).
 *   rho = sum_i f_i                                         (Eq. 4)
 *   mu  = mu0(rho) - kappa lap(rho)                         (Sec. II, Eq. 37)
 *   F   = grad(cs2 rho) - rho grad(mu)  (standard, Eq. 6)
 *       = -rho grad(mu)                 (WB, Eq. 25)
 *   (grad: the central gradient, or the fourth-order one with
 *    force_stencil = 1)
 *   u   = (sum_i c_i f_i + F/2) / rho                       (Eq. 4)
 * Any output pointer may be NULL except those the next step needs; scratch is
 * allocated here. */
void orc_macro(int scheme, const orc_params *p, int nx, int ny,
               const double *f, double *rho, double *ux, double *uy,
               double *mu, double *Fx, double *Fy, double *grx, double *gry) {
  size_t n = (size_t)nx * ny;
  double *lap = (double *)malloc(n * sizeof(double));
  double *gmx = (double *)malloc(n * sizeof(double));
  double *gmy = (double *)malloc(n * sizeof(double));

  for (size_t k = 0; k < n; ++k) {
    double s = 0.0;
    for (int i = 0; i < Q; ++i) s += f[k * Q + i];
    rho[k] = s;
  }
  orc_laplacian(nx, ny, rho, lap);
  for (size_t k = 0; k < n; ++k) mu[k] = orc_mu0(p, rho[k]) - p->kappa * lap[k];
  if (p->force_stencil == 1) {
    orc_gradient4(nx, ny, mu, gmx, gmy);
    orc_gradient4(nx, ny, rho, grx, gry);
  } else {
    orc_gradient(nx, ny, mu, gmx, gmy);
    orc_gradient(nx, ny, rho, grx, gry);
  }
  for (size_t k = 0; k < n; ++k) {
    double fx = -rho[k] * gmx[k];
    double fy = -rho[k] * gmy[k];
    if (scheme != ORC_WELL_BALANCED) {
      fx += CS2 * grx[k];
      fy += CS2 * gry[k];
    }
    Fx[k] = fx;
    Fy[k] = fy;
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < Q; ++i) {
      mx += CX[i] * f[k * Q + i];
      my += CY[i] * f[k * Q + i];
    }
    ux[k] = (mx + 0.5 * fx) / rho[k];
    uy[k] = (my + 0.5 * fy) / rho[k];
  }
  free(lap);
  free(gmx);
  free(gmy);
}

/* Fields of the state f as a caller sees them: rho, u, mu (any may be NULL). */
void orc_fields(int scheme, const orc_params *p, int nx, int ny,
                const double *f, double *rho_out, double *ux_out,
                double *uy_out, double *mu_out) {
  size_t n = (size_t)nx * ny;
  double *buf = (double *)malloc(8 * n * sizeof(double));
  double *rho = buf, *ux = buf + n, *uy = buf + 2 * n, *mu = buf + 3 * n;
  double *Fx = buf + 4 * n, *Fy = buf + 5 * n, *grx = buf + 6 * n,
         *gry = buf + 7 * n;
  orc_macro(scheme, p, nx, ny, f, rho, ux, uy, mu, Fx, Fy, grx, gry);
  if (rho_out) memcpy(rho_out, rho, n * sizeof(double));
  if (ux_out) memcpy(ux_out, ux, n * sizeof(double));
  if (uy_out) memcpy(uy_out, uy, n * sizeof(double));
  if (mu_out) memcpy(mu_out, mu, n * sizeof(double));
  free(buf);
}

/* Initial populations f_i = feq_i(rho, u) of the given scheme; ux/uy NULL
 * means u = 0. */
void orc_init(int scheme, const orc_params *p, int nx, int ny,
              const double *rho, const double *ux, const double *uy,
              double *f) {
  size_t n = (size_t)nx * ny;
  for (size_t k = 0; k < n; ++k)
    orc_feq(scheme, p, rho[k], ux ? ux[k] : 0.0, uy ? uy[k] : 0.0, f + k * Q);
}

/* n time steps of Eq. (2): collide, then stream to x + c_i (periodic).
 *   f*_i(x) = f_i - (f_i - feq_i)/tau + (1 - 1/(2 tau)) F_i
 *   f_i(x + c_i, t+1) = f*_i(x)
 * f is updated in place (a second buffer is allocated here). */
void orc_step(int scheme, const orc_params *p, int nx, int ny, double *f,
              int64_t nsteps) {
  size_t n = (size_t)nx * ny;
  double *buf = (double *)malloc(7 * n * sizeof(double));
  double *rho = buf, *ux = buf + n, *uy = buf + 2 * n, *mu = buf + 3 * n;
  double *Fx = buf + 4 * n, *Fy = buf + 5 * n, *gr = buf + 6 * n;
  double *gry = (double *)malloc(n * sizeof(double));
  double *g = (double *)malloc(n * Q * sizeof(double));
  double omega = 1.0 / p->tau;
  double fpre = 1.0 - 0.5 / p->tau;

  for (int64_t s = 0; s < nsteps; ++s) {
    orc_macro(scheme, p, nx, ny, f, rho, ux, uy, mu, Fx, Fy, gr, gry);
#pragma omp parallel for schedule(static) if ((long)nx * ny >= ORC_OMP_MIN_NODES)
    for (int y = 0; y < ny; ++y) {
      for (int x = 0; x < nx; ++x) {
        size_t k = (size_t)y * nx + x;
        double feq[Q], Fi[Q];
        orc_feq(scheme, p, rho[k], ux[k], uy[k], feq);
        if (scheme == ORC_STANDARD_EQF)
          orc_forcing_eq(feq, rho[k], ux[k], uy[k], Fx[k], Fy[k], Fi);
        else
          orc_forcing(scheme, ux[k], uy[k], Fx[k], Fy[k], gr[k], gry[k], Fi);
        for (int i = 0; i < Q; ++i) {
          double fs = f[k * Q + i] - omega * (f[k * Q + i] - feq[i]) +
                      fpre * Fi[i];
          size_t d = (size_t)wrap(y + CY[i], ny) * nx + wrap(x + CX[i], nx);
          g[d * Q + i] = fs;
        }
      }
    }
    memcpy(f, g, n * Q * sizeof(double));
  }
  free(buf);
  free(gry);
  free(g);
}

/* Neumaier compensated summation step. */
static inline void neumaier(double *sum, double *comp, double v) {
  double t = *sum + v;
  if (fabs(*sum) >= fabs(v))
    *comp += (*sum - t) + v;
  else
    *comp += (v - t) + *sum;
  *sum = t;
}

/* Scalar observables of the state f:
 *   out[0] = max |u|, out[1] = total mass sum rho (compensated),
 *   out[2] = kinetic energy E = (1/2) sum rho |u|^2 (Sec. IV.A, compensated),
 *   out[3] = 1 if any rho, u is NaN/Inf or rho <= 0, else 0,
 *   out[4], out[5] = total momentum sum rho u_x, sum rho u_y (compensated;
 *   with u the half-force velocity of Eq. 4). */
void orc_observe(int scheme, const orc_params *p, int nx, int ny,
                 const double *f, double *out) {
  size_t n = (size_t)nx * ny;
  double *buf = (double *)malloc(3 * n * sizeof(double));
  double *rho = buf, *ux = buf + n, *uy = buf + 2 * n;
  orc_fields(scheme, p, nx, ny, f, rho, ux, uy, NULL);
  double umax = 0.0, ms = 0.0, mc = 0.0, es = 0.0, ec = 0.0, bad = 0.0;
  double pxs = 0.0, pxc = 0.0, pys = 0.0, pyc = 0.0;
  for (size_t k = 0; k < n; ++k) {
    double u2 = ux[k] * ux[k] + uy[k] * uy[k];
    double um = sqrt(u2);
    if (!isfinite(rho[k]) || !isfinite(um) || !(rho[k] > 0.0)) bad = 1.0;
    if (um > umax) umax = um;
    neumaier(&ms, &mc, rho[k]);
    neumaier(&es, &ec, 0.5 * rho[k] * u2);
    neumaier(&pxs, &pxc, rho[k] * ux[k]);
    neumaier(&pys, &pyc, rho[k] * uy[k]);
  }
  out[0] = umax;
  out[1] = ms + mc;
  out[2] = es + ec;
  out[3] = bad;
  out[4] = pxs + pxc;
  out[5] = pys + pyc;
  free(buf);
}

/* Thread count for the field loops (results do not depend on it: every node's
 * arithmetic is the same and the sums above run serially). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
