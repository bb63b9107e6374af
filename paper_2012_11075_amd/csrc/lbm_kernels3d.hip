// lbm_kernels3d.hip -- gfx950 kernels of the D3Q19 form of the two-phase
// LBE step (Eqs. 24 and 26 are stated for general D; here D = 3).
//
// Velocities: rest, the 6 axis directions (weight 1/18), the 12 edge
// directions (weight 1/36).  Gradient (1/cs2) sum w_i c_i phi(x+c_i) and
// Laplacian (2/cs2) sum w_i [phi(x+c_i) - phi(x)], as in 2-D.  FP64, three
// passes per step like the force-stencil variant: density, chemical
// potential, collide-stream on LDS tiles of rho and mu with a 1-node halo.
#include <hip/hip_runtime.h>

#include "lbm_kernels3d.h"

namespace lbmk {
namespace {

// Populations are addressed through global-address-space pointers, so the
// compiler emits global (not flat) loads and stores.
template <typename T>
using Global = __attribute__((address_space(1))) T;

__device__ __forceinline__ void c3(int i, int& cx, int& cy, int& cz) {
  const int X[Q3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  const int Y[Q3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  const int Z[Q3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  cx = X[i];
  cy = Y[i];
  cz = Z[i];
}

// Element offset (without the q * plane term) that the pull of population q
// of node (x, y, z) reads: the node (x, y, z) - c_q, periodic.
__device__ __forceinline__ long long src3(const Geometry3& g, int q, int x, int y, int z) {
  int cx, cy, cz;
  c3(q, cx, cy, cz);
  int xs = x - cx, ys = y - cy, zs = z - cz;
  xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
  ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
  zs = zs < 0 ? zs + g.nz : (zs >= g.nz ? zs - g.nz : zs);
  return (long long)zs * g.slab + (long long)ys * g.pitch + xs;
}

__device__ __forceinline__ double mu0_3(double r, const Physics3& p) {
  return 2.0 * p.beta * (r - p.rho_l) * (r - p.rho_v) * (2.0 * r - p.rho_l - p.rho_v);
}

// Equilibrium (Eq. 3 / Eq. 24) and forcing term (Eq. 5 / Eq. 26 with D = 3:
// the last term's coefficient (|c|^2/cs2 - 3)/2 is -3/2, 0, 3/2 for the
// rest, axis and edge directions), then BGK.
template <int SCHEME>
__device__ __forceinline__ void collide3(double (&f)[Q3], double rho, double ux, double uy,
                                         double uz, double Fx, double Fy, double Fz, double grx,
                                         double gry, double grz, const Physics3& p) {
  const double u15 = 1.5 * (ux * ux + uy * uy + uz * uz);
  double Gx = Fx, Gy = Fy, Gz = Fz;
  if (SCHEME == WELL_BALANCED) {
    Gx += grx * (1.0 / 3.0);
    Gy += gry * (1.0 / 3.0);
    Gz += grz * (1.0 / 3.0);
  }
  const double uG3 = 3.0 * (ux * Gx + uy * Gy + uz * Gz);
  const double ugr = ux * grx + uy * gry + uz * grz;
#pragma unroll
  for (int i = 0; i < Q3; ++i) {
    int cx, cy, cz;
    c3(i, cx, cy, cz);
    const double w = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    const double cu = cx * ux + cy * uy + cz * uz;
    const double cF = cx * Fx + cy * Fy + cz * Fz;
    const double cG = cx * Gx + cy * Gy + cz * Gz;
    const double poly = 3.0 * cu + 4.5 * cu * cu - u15;
    double feq, Fi;
    if (SCHEME == STANDARD) {
      feq = w * rho * (1.0 + poly);
      Fi = w * (3.0 * cF + 9.0 * cu * cG - uG3);
    } else {
      feq = i == 0 ? rho - (1.0 - w) * p.rho0 - w * rho * u15 : w * (p.rho0 + rho * poly);
      const double k = i == 0 ? -1.5 : (i < 7 ? 0.0 : 1.5);
      Fi = w * (3.0 * cF + 9.0 * cu * cG - uG3 + k * ugr);
    }
    f[i] = f[i] - p.omega * (f[i] - feq) + p.fpre * Fi;
  }
}

__global__ void __launch_bounds__(256)
    density3(Geometry3 g, const Global<double>* __restrict__ fin, double* __restrict__ rho) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < Q3; ++i) s += fin[(long long)i * g.plane + src3(g, i, x, y, z)];
  rho[((long long)z * g.ny + y) * g.nx + x] = s;
}

__global__ void __launch_bounds__(256)
    potential3(Geometry3 g, Physics3 p, const double* __restrict__ rho, double* __restrict__ mu) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  auto at = [&](int dx, int dy, int dz) {
    int a = x + dx, b = y + dy, c = z + dz;
    a = a < 0 ? a + g.nx : (a >= g.nx ? a - g.nx : a);
    b = b < 0 ? b + g.ny : (b >= g.ny ? b - g.ny : b);
    c = c < 0 ? c + g.nz : (c >= g.nz ? c - g.nz : c);
    return rho[((long long)c * g.ny + b) * g.nx + a];
  };
  const double c = at(0, 0, 0);
  double ax = 0.0, ed = 0.0;
#pragma unroll
  for (int i = 1; i < Q3; ++i) {
    int cx, cy, cz;
    c3(i, cx, cy, cz);
    if (i < 7)
      ax += at(cx, cy, cz);
    else
      ed += at(cx, cy, cz);
  }
  const double lap = (2.0 * ax + ed - 24.0 * c) * (1.0 / 6.0);
  mu[((long long)z * g.ny + y) * g.nx + x] = mu0_3(c, p) - p.kappa * lap;
}

constexpr int T3X = 32, T3Y = 4, T3Z = 2;  // collide-stream block (threads)

// Isotropic central gradient of an LDS tile at tile point (k, j, i).
__device__ __forceinline__ void grad3(const double (&a)[T3Z + 2][T3Y + 2][T3X + 2], int k, int j,
                                      int i, double& gx, double& gy, double& gz) {
  gx = (a[k][j][i + 1] - a[k][j][i - 1]) * (1.0 / 6.0) +
       ((a[k][j + 1][i + 1] - a[k][j + 1][i - 1]) + (a[k][j - 1][i + 1] - a[k][j - 1][i - 1]) +
        (a[k + 1][j][i + 1] - a[k + 1][j][i - 1]) + (a[k - 1][j][i + 1] - a[k - 1][j][i - 1])) *
           (1.0 / 12.0);
  gy = (a[k][j + 1][i] - a[k][j - 1][i]) * (1.0 / 6.0) +
       ((a[k][j + 1][i + 1] - a[k][j - 1][i + 1]) + (a[k][j + 1][i - 1] - a[k][j - 1][i - 1]) +
        (a[k + 1][j + 1][i] - a[k + 1][j - 1][i]) + (a[k - 1][j + 1][i] - a[k - 1][j - 1][i])) *
           (1.0 / 12.0);
  gz = (a[k + 1][j][i] - a[k - 1][j][i]) * (1.0 / 6.0) +
       ((a[k + 1][j][i + 1] - a[k - 1][j][i + 1]) + (a[k + 1][j][i - 1] - a[k - 1][j][i - 1]) +
        (a[k + 1][j + 1][i] - a[k - 1][j + 1][i]) + (a[k + 1][j - 1][i] - a[k - 1][j - 1][i])) *
           (1.0 / 12.0);
}

template <int SCHEME, bool OBSERVE>
__global__ void __launch_bounds__(T3X * T3Y * T3Z)
    collide3_kernel(Geometry3 g, Physics3 p, const Global<double>* __restrict__ fin,
                    Global<double>* __restrict__ fout, const double* __restrict__ rho,
                    const double* __restrict__ mu, ObserveOut3 obs) {
  __shared__ double rt[T3Z + 2][T3Y + 2][T3X + 2];
  __shared__ double mt[T3Z + 2][T3Y + 2][T3X + 2];
  const int tid = threadIdx.x;
  const int tx = tid % T3X, ty = (tid / T3X) % T3Y, tz = tid / (T3X * T3Y);
  const int x0 = blockIdx.x * T3X, y0 = blockIdx.y * T3Y, z0 = blockIdx.z * T3Z;
  constexpr int TILE = (T3Z + 2) * (T3Y + 2) * (T3X + 2);
  for (int e = tid; e < TILE; e += T3X * T3Y * T3Z) {
    const int i = e % (T3X + 2), j = (e / (T3X + 2)) % (T3Y + 2), k = e / ((T3X + 2) * (T3Y + 2));
    int xx = (x0 + i - 1) % g.nx, yy = (y0 + j - 1) % g.ny, zz = (z0 + k - 1) % g.nz;
    xx = xx < 0 ? xx + g.nx : xx;
    yy = yy < 0 ? yy + g.ny : yy;
    zz = zz < 0 ? zz + g.nz : zz;
    const long long o = ((long long)zz * g.ny + yy) * g.nx + xx;
    rt[k][j][i] = rho[o];
    mt[k][j][i] = mu[o];
  }
  __syncthreads();
  const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
  double umax = 0.0, mass = 0.0, ekin = 0.0, bad = 0.0;
  if (x < g.nx && y < g.ny && z < g.nz) {
    double f[Q3];
#pragma unroll
    for (int i = 0; i < Q3; ++i) f[i] = fin[(long long)i * g.plane + src3(g, i, x, y, z)];
    const double r = rt[tz + 1][ty + 1][tx + 1];
    double grx, gry, grz, gmx, gmy, gmz;
    grad3(rt, tz + 1, ty + 1, tx + 1, grx, gry, grz);
    grad3(mt, tz + 1, ty + 1, tx + 1, gmx, gmy, gmz);
    double Fx = -r * gmx, Fy = -r * gmy, Fz = -r * gmz;
    if (SCHEME == STANDARD) {
      Fx += grx * (1.0 / 3.0);
      Fy += gry * (1.0 / 3.0);
      Fz += grz * (1.0 / 3.0);
    }
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < Q3; ++i) {
      int cx, cy, cz;
      c3(i, cx, cy, cz);
      jx += cx * f[i];
      jy += cy * f[i];
      jz += cz * f[i];
    }
    const double inv = 1.0 / r;
    const double ux = (jx + 0.5 * Fx) * inv, uy = (jy + 0.5 * Fy) * inv, uz = (jz + 0.5 * Fz) * inv;
    if (!OBSERVE) {
      collide3<SCHEME>(f, r, ux, uy, uz, Fx, Fy, Fz, grx, gry, grz, p);
      Global<double>* dst = fout + (long long)z * g.slab + (long long)y * g.pitch + x;
#pragma unroll
      for (int i = 0; i < Q3; ++i) __builtin_nontemporal_store(f[i], dst + (long long)i * g.plane);
    } else {
      const long long o = ((long long)z * g.ny + y) * g.nx + x;
      if (obs.ux) obs.ux[o] = ux;
      if (obs.uy) obs.uy[o] = uy;
      if (obs.uz) obs.uz[o] = uz;
      const double u2 = ux * ux + uy * uy + uz * uz;
      const double um = sqrt(u2);
      if (!(isfinite(r) && r > 0.0 && isfinite(um))) bad = 1.0;
      umax = um;
      mass = r;
      ekin = 0.5 * r * u2;
    }
  }
  if (OBSERVE && obs.partials) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      umax = fmax(umax, __shfl_xor(umax, off));
      bad = fmax(bad, __shfl_xor(bad, off));
      mass += __shfl_xor(mass, off);
      ekin += __shfl_xor(ekin, off);
    }
    constexpr int NW = T3X * T3Y * T3Z / 64;
    __shared__ double red[NW][4];
    const int wv = tid >> 6;
    if ((tid & 63) == 0) {
      red[wv][0] = umax;
      red[wv][1] = mass;
      red[wv][2] = ekin;
      red[wv][3] = bad;
    }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, m = 0.0, e = 0.0, zb = 0.0;
      for (int w = 0; w < NW; ++w) {
        a = fmax(a, red[w][0]);
        m += red[w][1];
        e += red[w][2];
        zb = fmax(zb, red[w][3]);
      }
      const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
      double* out = obs.partials + 4 * b;
      out[0] = a;
      out[1] = m;
      out[2] = e;
      out[3] = zb;
    }
  }
}

// f = feq(rho, u) of every node, stored where the next pull reads it.
template <int SCHEME>
__global__ void __launch_bounds__(256)
    init3_kernel(Geometry3 g, Physics3 p, const double* __restrict__ rho,
                 const double* __restrict__ ux, const double* __restrict__ uy,
                 const double* __restrict__ uz, double* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  const long long k = ((long long)z * g.ny + y) * g.nx + x;
  const double r = rho[k];
  const double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0, vz = uz ? uz[k] : 0.0;
  const double u15 = 1.5 * (vx * vx + vy * vy + vz * vz);
  for (int i = 0; i < Q3; ++i) {
    int cx, cy, cz;
    c3(i, cx, cy, cz);
    const double w = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
    const double cu = cx * vx + cy * vy + cz * vz;
    const double poly = 3.0 * cu + 4.5 * cu * cu - u15;
    double q;
    if (SCHEME == STANDARD)
      q = w * r * (1.0 + poly);
    else
      q = i == 0 ? r - (1.0 - w) * p.rho0 - w * r * u15 : w * (p.rho0 + r * poly);
    f[(long long)i * g.plane + src3(g, i, x, y, z)] = q;
  }
}

// dense[m][z][y][x] <-> populations q0 .. q0+m-1 (pre-collision f at each node).
template <bool PACK>
__global__ void __launch_bounds__(256)
    pack3_kernel(Geometry3 g, int q0, int m, double* __restrict__ dense, double* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long k = ((long long)z * g.ny + y) * g.nx + x;
  for (int j = 0; j < m; ++j) {
    const int q = q0 + j;
    const long long o = (long long)q * g.plane + src3(g, q, x, y, z);
    if (PACK)
      f[o] = dense[j * n + k];
    else
      dense[j * n + k] = f[o];
  }
}

}  // namespace

namespace {

inline dim3 grid_rows3(const Geometry3& g) { return dim3((g.nx + 255) / 256, g.ny, g.nz); }

}  // namespace

int blocks3(const Geometry3& g) {
  return ((g.nx + T3X - 1) / T3X) * ((g.ny + T3Y - 1) / T3Y) * ((g.nz + T3Z - 1) / T3Z);
}

hipError_t launch_init3(int scheme, const Geometry3& g, const Physics3& ph, const double* rho,
                        const double* ux, const double* uy, const double* uz, void* f,
                        hipStream_t s) {
  if (scheme == STANDARD)
    hipLaunchKernelGGL(init3_kernel<STANDARD>, grid_rows3(g), dim3(256), 0, s, g, ph, rho, ux,
                       uy, uz, (double*)f);
  else
    hipLaunchKernelGGL(init3_kernel<WELL_BALANCED>, grid_rows3(g), dim3(256), 0, s, g, ph, rho,
                       ux, uy, uz, (double*)f);
  return hipGetLastError();
}

hipError_t launch_pack3(const Geometry3& g, const double* dense, int q0, int m, void* f,
                        hipStream_t s) {
  hipLaunchKernelGGL(pack3_kernel<true>, grid_rows3(g), dim3(256), 0, s, g, q0, m,
                     const_cast<double*>(dense), (double*)f);
  return hipGetLastError();
}

hipError_t launch_unpack3(const Geometry3& g, const void* f, int q0, int m, double* dense,
                          hipStream_t s) {
  hipLaunchKernelGGL(pack3_kernel<false>, grid_rows3(g), dim3(256), 0, s, g, q0, m, dense,
                     const_cast<double*>((const double*)f));
  return hipGetLastError();
}

namespace {

template <bool OBS>
hipError_t launch3(int scheme, const Geometry3& g, const Physics3& ph, const void* fin, void* fout,
                   double* rho, double* mu, const ObserveOut3& o, hipStream_t s) {
  const auto* in = (const Global<double>*)(const double*)fin;
  auto* out = (Global<double>*)(double*)fout;
  hipLaunchKernelGGL(density3, grid_rows3(g), dim3(256), 0, s, g, in, rho);
  hipLaunchKernelGGL(potential3, grid_rows3(g), dim3(256), 0, s, g, ph, (const double*)rho, mu);
  const dim3 gc((g.nx + T3X - 1) / T3X, (g.ny + T3Y - 1) / T3Y, (g.nz + T3Z - 1) / T3Z);
  if (scheme == STANDARD)
    hipLaunchKernelGGL((collide3_kernel<STANDARD, OBS>), gc, dim3(T3X * T3Y * T3Z), 0, s, g, ph,
                       in, out, (const double*)rho, (const double*)mu, o);
  else
    hipLaunchKernelGGL((collide3_kernel<WELL_BALANCED, OBS>), gc, dim3(T3X * T3Y * T3Z), 0, s, g,
                       ph, in, out, (const double*)rho, (const double*)mu, o);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step3(int scheme, const Geometry3& g, const Physics3& ph, const void* fin,
                        void* fout, double* rho, double* mu, hipStream_t s) {
  const ObserveOut3 none{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  return launch3<false>(scheme, g, ph, fin, fout, rho, mu, none, s);
}

hipError_t launch_observe3(int scheme, const Geometry3& g, const Physics3& ph, const void* f,
                           double* rho, double* mu, const ObserveOut3& o, hipStream_t s) {
  return launch3<true>(scheme, g, ph, f, nullptr, rho, mu, o, s);
}

}  // namespace lbmk
