// lbm_kernels.hip -- gfx950 kernels of the D2Q9 two-phase LBE step.
//
// Method: Z. Guo, "Well-balanced lattice Boltzmann equation for two-phase
// flows", arXiv:2012.11075.
//   rho, u            Eq. (4)  (half-force velocity)
//   mu = mu0 - k lap   Sec. II with mu0 of Eqs. (36)-(37)
//   grad, lap          isotropic central differences (Sec. II, Eq. 19 and the
//                      9-point Laplacian of the same family)
//   force              Eq. (6) potential form (standard) / Eq. (25) (WB)
//   equilibrium        Eq. (3) (standard) / Eq. (24) (WB)
//   forcing term       Eq. (5) (standard) / Eq. (26) (WB)
//   collide + stream   Eq. (2): f*_i = f_i - (f_i - feq_i)/tau + (1 - 1/2tau) F_i,
//                      f_i(x + c_i, t+1) = f*_i(x, t), periodic.
//
// Design (one HBM pass per step).  Populations live in 9 structure-of-arrays
// planes, x fastest.  A block of BW threads owns a strip of BW-4 output
// columns and marches down a chunk of rows.  Each thread loads the 9
// populations of one column per row (coalesced along x), keeps the last three
// rows in registers, and publishes rho of the row to a 5-row LDS ring; mu of
// the previous row goes to a 3-row LDS ring.  The 2-column x-halo of rho is
// recomputed by the edge threads (neighbouring strips overlap by 4 columns),
// the 2-row y-halo by reading two extra rows at each end of the chunk, so no
// block ever waits for another.  Collision and streaming are fused: the
// post-collision populations are pushed to x + c_i of the other buffer.
// rho, mu and u of every node come from the same device code in the step and
// in the observe pass.
#include <hip/hip_runtime.h>

#include "lbm_kernels.h"

namespace lbmk {
namespace {

template <typename R>
struct PhysR {
  R omega, fpre, beta, kappa, rho_l, rho_v, rho_ref;
  R c[Q];
};

template <typename R>
__device__ __forceinline__ PhysR<R> to_r(const Physics& p) {
  PhysR<R> q;
  q.omega = (R)p.omega;
  q.fpre = (R)p.fpre;
  q.beta = (R)p.beta;
  q.kappa = (R)p.kappa;
  q.rho_l = (R)p.rho_l;
  q.rho_v = (R)p.rho_v;
  q.rho_ref = (R)p.rho_ref;
#pragma unroll
  for (int i = 0; i < Q; ++i) q.c[i] = (R)p.geq_c[i];
  return q;
}

// Bulk chemical potential of the double well, mu0 = dpsi0/drho (Eq. 37).
template <typename R>
__device__ __forceinline__ R mu0(R rho, const PhysR<R>& p) {
  return (R)2 * p.beta * (rho - p.rho_l) * (rho - p.rho_v) * ((R)2 * rho - p.rho_l - p.rho_v);
}

template <typename R>
__device__ __forceinline__ R sum9(const R (&f)[Q]) {
  return (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) + f[8];
}

// Velocity of Eq. (4): u = (sum_i c_i f_i + F/2) / rho.
template <typename R>
__device__ __forceinline__ void velocity(const R (&f)[Q], R rho, R Fx, R Fy, R& ux, R& uy) {
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R inv = (R)1 / rho;
  ux = (jx + (R)0.5 * Fx) * inv;
  uy = (jy + (R)0.5 * Fy) * inv;
}

// Shifted equilibrium geq_i = feq_i(rho, u) - s_i and forcing term F_i.
//   standard: feq_i = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)     (Eq. 3)
//             F_i   = w_i (3 c.F + 9 (c.u)(c.F) - 3 u.F)              (Eq. 5)
//   WB:       feq_0 = rho - (1-w0) rho0 - 1.5 w0 rho u.u,
//             feq_i = w_i (rho0 + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)) (Eq. 24)
//             F_i   = w_i (3 c.F + 9 (c.u)(c.G) - 3 u.G
//                          + (3|c_i|^2 - 2)/2 (u.grad rho)),  G = F + grad(rho)/3  (Eq. 26)
// feq_i(rho, u) - feq_i(rho_ref, 0) is evaluated from drho = rho - rho_ref
// (the rho0 terms cancel); the constant feq_i(rho_ref, 0) - s_i is p.c[i].
template <typename R, int SCHEME>
__device__ __forceinline__ void collide(R (&f)[Q], R drho, R rho, R ux, R uy, R Fx, R Fy, R grx,
                                        R gry, const PhysR<R>& p) {
  const R w0 = (R)4 / (R)9, w1 = (R)1 / (R)9, w5 = (R)1 / (R)36;
  const R uu = ux * ux + uy * uy;
  const R u15 = (R)1.5 * uu;
  R Gx = Fx, Gy = Fy;
  if (SCHEME == WELL_BALANCED) {
    Gx = Fx + grx * ((R)1 / (R)3);
    Gy = Fy + gry * ((R)1 / (R)3);
  }
  const R uG3 = (R)3 * (ux * Gx + uy * Gy);
  const R ugr = ux * grx + uy * gry;
  // c_i . u, c_i . F, c_i . G for i = 1..8 (paper numbering)
  const R cu[Q] = {(R)0, ux, uy, -ux, -uy, ux + uy, uy - ux, -ux - uy, ux - uy};
  const R cF[Q] = {(R)0, Fx, Fy, -Fx, -Fy, Fx + Fy, Fy - Fx, -Fx - Fy, Fx - Fy};
  const R cG[Q] = {(R)0, Gx, Gy, -Gx, -Gy, Gx + Gy, Gy - Gx, -Gx - Gy, Gx - Gy};
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    const R w = (i == 0) ? w0 : (i < 5 ? w1 : w5);
    const R poly = (R)3 * cu[i] + (R)4.5 * cu[i] * cu[i] - u15;
    R geq, Fi;
    if (SCHEME == STANDARD) {
      geq = w * (drho + rho * poly);
      Fi = w * ((R)3 * cF[i] + (R)9 * cu[i] * cF[i] - uG3);
    } else {
      geq = (i == 0) ? drho - w0 * rho * u15 : w * rho * poly;
      const R k = (i == 0) ? (R)-1 : (i < 5 ? (R)0.5 : (R)2);
      Fi = w * ((R)3 * cF[i] + (R)9 * cu[i] * cG[i] - uG3 + k * ugr);
    }
    geq += p.c[i];
    f[i] = f[i] - p.omega * (f[i] - geq) + p.fpre * Fi;
  }
}

// Marching step / observe kernel.  T: storage and arithmetic type.
template <typename T, int SCHEME, int BW, bool OBSERVE>
__global__ void __launch_bounds__(BW)
    march(Geometry g, Physics phys, Tiling tl, const T* __restrict__ fin, T* __restrict__ fout,
          ObserveOut obs) {
  using R = T;
  __shared__ R rs[5][BW];  // rho ring: rows y-2 .. y+2 of the output row y
  __shared__ R ms[3][BW];  // mu ring: rows y-1 .. y+1
  const PhysR<R> p = to_r<R>(phys);
  const int t = threadIdx.x;

  // Tiles are assigned so that each XCD (blocks b, b+8, ...) walks a
  // contiguous range of tiles: neighbouring strips share halo lines in L2.
  const int nb = tl.strips * tl.chunks;
  const int b = blockIdx.x;
  const int xcd = b & 7, l = b >> 3, q8 = nb >> 3, r8 = nb & 7;
  const int tile = xcd * q8 + min(xcd, r8) + l;
  const int chunk = tile / tl.strips;
  const int strip = tile - chunk * tl.strips;

  const int x0 = strip * (BW - 4);
  int xc = (x0 - 2 + t) % g.nx;
  if (xc < 0) xc += g.nx;
  const bool outc = (t >= 2) && (t < BW - 2) && (x0 + t - 2 < g.nx);
  const int x = x0 + t - 2;
  const int y0 = chunk * tl.rows;
  const int H = min(tl.rows, g.ny - y0);
  const int K = H + 4;  // row index k <-> lattice row y0 - 2 + k

  auto row_of = [&](int k) {
    int y = (y0 - 2 + k) % g.ny;
    return y < 0 ? y + g.ny : y;
  };
  auto load_row = [&](int k, R(&dst)[Q]) {
    const long long off = (long long)row_of(k) * g.pitch + xc;
#pragma unroll
    for (int i = 0; i < Q; ++i) dst[i] = fin[(long long)i * g.plane + off];
  };

  double umax = 0.0, mass = 0.0, ekin = 0.0, bad = 0.0;

  R fo[Q], fm[Q], fc[Q], fn[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) fo[i] = fm[i] = fn[i] = (R)0;
  load_row(0, fc);

  for (int k = 0; k < K; ++k) {
    if (k + 1 < K) load_row(k + 1, fn);
    rs[k % 5][t] = p.rho_ref + sum9(fc);
    __syncthreads();
    if (k >= 2 && t >= 1 && t < BW - 1) {
      // mu at row index k-1: mu0(rho) - kappa lap(rho), 9-point Laplacian
      const int a = (k - 2) % 5, c0 = (k - 1) % 5, d = k % 5;
      const R r0 = rs[c0][t];
      const R ax = (rs[c0][t + 1] + rs[c0][t - 1]) + (rs[a][t] + rs[d][t]);
      const R dg = (rs[a][t + 1] + rs[a][t - 1]) + (rs[d][t + 1] + rs[d][t - 1]);
      const R lap = ((R)4 * ax + dg - (R)20 * r0) * ((R)1 / (R)6);
      ms[(k - 1) % 3][t] = mu0(r0, p) - p.kappa * lap;
    }
    __syncthreads();
    if (k >= 4 && outc) {
      const int sM = (k - 3) % 5, s0 = (k - 2) % 5, sP = (k - 1) % 5;
      const int mM = (k - 3) % 3, m0 = (k - 2) % 3, mP = (k - 1) % 3;
      const R third = (R)1 / (R)3, twelfth = (R)1 / (R)12;
      const R rho = rs[s0][t];
      const R grx = (rs[s0][t + 1] - rs[s0][t - 1]) * third +
                    ((rs[sP][t + 1] - rs[sP][t - 1]) + (rs[sM][t + 1] - rs[sM][t - 1])) * twelfth;
      const R gry = (rs[sP][t] - rs[sM][t]) * third +
                    ((rs[sP][t + 1] + rs[sP][t - 1]) - (rs[sM][t + 1] + rs[sM][t - 1])) * twelfth;
      const R gmx = (ms[m0][t + 1] - ms[m0][t - 1]) * third +
                    ((ms[mP][t + 1] - ms[mP][t - 1]) + (ms[mM][t + 1] - ms[mM][t - 1])) * twelfth;
      const R gmy = (ms[mP][t] - ms[mM][t]) * third +
                    ((ms[mP][t + 1] + ms[mP][t - 1]) - (ms[mM][t + 1] + ms[mM][t - 1])) * twelfth;
      R Fx = -rho * gmx, Fy = -rho * gmy;
      if (SCHEME == STANDARD) {
        Fx += grx * third;
        Fy += gry * third;
      }
      R ux, uy;
      velocity(fo, rho, Fx, Fy, ux, uy);
      const int y = y0 + k - 4;
      if (!OBSERVE) {
        const R drho = sum9(fo);
        collide<R, SCHEME>(fo, drho, rho, ux, uy, Fx, Fy, grx, gry, p);
        const int xe = (x + 1 == g.nx) ? 0 : x + 1;
        const int xw = (x == 0) ? g.nx - 1 : x - 1;
        const int yn = (y + 1 == g.ny) ? 0 : y + 1;
        const int ys = (y == 0) ? g.ny - 1 : y - 1;
        const long long P = g.plane;
        const long long ry = (long long)y * g.pitch, rn = (long long)yn * g.pitch,
                        rsy = (long long)ys * g.pitch;
        fout[ry + x] = fo[0];
        fout[P + ry + xe] = fo[1];
        fout[2 * P + rn + x] = fo[2];
        fout[3 * P + ry + xw] = fo[3];
        fout[4 * P + rsy + x] = fo[4];
        fout[5 * P + rn + xe] = fo[5];
        fout[6 * P + rn + xw] = fo[6];
        fout[7 * P + rsy + xw] = fo[7];
        fout[8 * P + rsy + xe] = fo[8];
      } else {
        const long long o = (long long)y * g.nx + x;
        const double drho = (double)rho, dux = (double)ux, duy = (double)uy;
        if (obs.rho) obs.rho[o] = drho;
        if (obs.ux) obs.ux[o] = dux;
        if (obs.uy) obs.uy[o] = duy;
        if (obs.mu) obs.mu[o] = (double)ms[m0][t];
        const double u2 = dux * dux + duy * duy;
        const double um = sqrt(u2);
        if (!(isfinite(drho) && drho > 0.0 && isfinite(um))) bad = 1.0;
        umax = fmax(umax, um);
        mass += drho;
        ekin += 0.5 * drho * u2;
      }
    }
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      fo[i] = fm[i];
      fm[i] = fc[i];
      fc[i] = fn[i];
    }
  }

  if (OBSERVE && obs.partials) {
    // wave butterfly, then waves in order: a fixed summation order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      umax = fmax(umax, __shfl_xor(umax, off));
      bad = fmax(bad, __shfl_xor(bad, off));
      mass += __shfl_xor(mass, off);
      ekin += __shfl_xor(ekin, off);
    }
    __shared__ double red[BW / 64][4];
    const int wv = t >> 6;
    if ((t & 63) == 0) {
      red[wv][0] = umax;
      red[wv][1] = mass;
      red[wv][2] = ekin;
      red[wv][3] = bad;
    }
    __syncthreads();
    if (t == 0) {
      double a = 0.0, m = 0.0, e = 0.0, z = 0.0;
      for (int w = 0; w < BW / 64; ++w) {
        a = fmax(a, red[w][0]);
        m += red[w][1];
        e += red[w][2];
        z = fmax(z, red[w][3]);
      }
      double* out = obs.partials + 4LL * tile;
      out[0] = a;
      out[1] = m;
      out[2] = e;
      out[3] = z;
    }
  }
}

// f = feq(rho, u) - s from dense fields; arithmetic in double, stored as T.
template <typename T, int SCHEME>
__global__ void init_kernel(Geometry g, Physics phys, const double* __restrict__ rho,
                            const double* __restrict__ ux, const double* __restrict__ uy,
                            T* __restrict__ f) {
  const long long n = (long long)g.nx * g.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int y = (int)(k / g.nx), x = (int)(k - (long long)y * g.nx);
  const PhysR<double> p = to_r<double>(phys);
  const double r = rho[k];
  const double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0;
  // feq with F = 0: the collision with omega = 1, fpre = 0 returns geq.
  double q[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) q[i] = 0.0;
  PhysR<double> p1 = p;
  p1.omega = 1.0;
  p1.fpre = 0.0;
  collide<double, SCHEME>(q, r - p.rho_ref, r, vx, vy, 0.0, 0.0, 0.0, 0.0, p1);
  const long long off = (long long)y * g.pitch + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) f[(long long)i * g.plane + off] = (T)q[i];
}

struct Shift {
  double s[Q];
};

inline Shift make_shift(const double* h) {
  Shift r;
  for (int i = 0; i < Q; ++i) r.s[i] = h ? h[i] : 0.0;
  return r;
}

template <typename T>
__global__ void pack_kernel(Geometry g, Shift shift, const double* __restrict__ dense, int q0,
                            T* __restrict__ f) {
  const long long n = (long long)g.nx * g.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= n) return;
  const int y = (int)(k / g.nx), x = (int)(k - (long long)y * g.nx);
  const int q = q0 + m;
  const double s = shift.s[q];
  f[(long long)q * g.plane + (long long)y * g.pitch + x] = (T)(dense[(long long)m * n + k] - s);
}

template <typename T>
__global__ void unpack_kernel(Geometry g, Shift shift, const T* __restrict__ f, int q0,
                              double* __restrict__ dense) {
  const long long n = (long long)g.nx * g.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (k >= n) return;
  const int y = (int)(k / g.nx), x = (int)(k - (long long)y * g.nx);
  const int q = q0 + m;
  const double s = shift.s[q];
  dense[(long long)m * n + k] = (double)f[(long long)q * g.plane + (long long)y * g.pitch + x] + s;
}

template <typename T>
__global__ void reshift_kernel(Geometry g, Physics d, T* __restrict__ f) {
  const long long n = (long long)g.nx * g.ny;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int y = (int)(k / g.nx), x = (int)(k - (long long)y * g.nx);
  const long long off = (long long)y * g.pitch + x;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    T* a = f + (long long)i * g.plane + off;
    *a = (T)((double)*a + d.geq_c[i]);
  }
}

template <typename T, int SCHEME, int BW, bool OBS>
hipError_t launch_march_t(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                          void* fout, const ObserveOut& o, hipStream_t s) {
  hipLaunchKernelGGL((march<T, SCHEME, BW, OBS>), dim3(t.blocks()), dim3(BW), 0, s, g, ph, t,
                     (const T*)fin, (T*)fout, o);
  return hipGetLastError();
}

template <typename T, int SCHEME, bool OBS>
hipError_t launch_march_w(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                          void* fout, const ObserveOut& o, hipStream_t s) {
  switch (t.block) {
    case 128: return launch_march_t<T, SCHEME, 128, OBS>(g, ph, t, fin, fout, o, s);
    case 192: return launch_march_t<T, SCHEME, 192, OBS>(g, ph, t, fin, fout, o, s);
    case 256: return launch_march_t<T, SCHEME, 256, OBS>(g, ph, t, fin, fout, o, s);
    case 320: return launch_march_t<T, SCHEME, 320, OBS>(g, ph, t, fin, fout, o, s);
    case 512: return launch_march_t<T, SCHEME, 512, OBS>(g, ph, t, fin, fout, o, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool OBS>
hipError_t launch_march(int storage, int scheme, const Geometry& g, const Physics& ph,
                        const Tiling& t, const void* fin, void* fout, const ObserveOut& o,
                        hipStream_t s) {
  if (t.blocks() <= 0) return hipErrorInvalidValue;
  if (storage == FP64) {
    return scheme == STANDARD
               ? launch_march_w<double, STANDARD, OBS>(g, ph, t, fin, fout, o, s)
               : launch_march_w<double, WELL_BALANCED, OBS>(g, ph, t, fin, fout, o, s);
  }
  return scheme == STANDARD ? launch_march_w<float, STANDARD, OBS>(g, ph, t, fin, fout, o, s)
                            : launch_march_w<float, WELL_BALANCED, OBS>(g, ph, t, fin, fout, o, s);
}

inline unsigned grid1(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

bool block_width_supported(int block) {
  return block == 128 || block == 192 || block == 256 || block == 320 || block == 512;
}

hipError_t launch_step(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const Tiling& t, const void* fin, void* fout, hipStream_t s) {
  ObserveOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
  return launch_march<false>(storage, scheme, g, ph, t, fin, fout, none, s);
}

hipError_t launch_observe(int storage, int scheme, const Geometry& g, const Physics& ph,
                          const Tiling& t, const void* f, const ObserveOut& o, hipStream_t s) {
  return launch_march<true>(storage, scheme, g, ph, t, f, nullptr, o, s);
}

hipError_t launch_init(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const double* rho, const double* ux, const double* uy, void* f,
                       hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  if (storage == FP64) {
    if (scheme == STANDARD)
      hipLaunchKernelGGL((init_kernel<double, STANDARD>), dim3(grid1(n)), dim3(256), 0, s, g, ph,
                         rho, ux, uy, (double*)f);
    else
      hipLaunchKernelGGL((init_kernel<double, WELL_BALANCED>), dim3(grid1(n)), dim3(256), 0, s, g,
                         ph, rho, ux, uy, (double*)f);
  } else {
    if (scheme == STANDARD)
      hipLaunchKernelGGL((init_kernel<float, STANDARD>), dim3(grid1(n)), dim3(256), 0, s, g, ph,
                         rho, ux, uy, (float*)f);
    else
      hipLaunchKernelGGL((init_kernel<float, WELL_BALANCED>), dim3(grid1(n)), dim3(256), 0, s, g,
                         ph, rho, ux, uy, (float*)f);
  }
  return hipGetLastError();
}

hipError_t launch_pack(int storage, const Geometry& g, const double* shift, const double* dense,
                       int q0, int m, void* f, hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  if (storage == FP64)
    hipLaunchKernelGGL(pack_kernel<double>, dim3(grid1(n), m), dim3(256), 0, s, g,
                       make_shift(shift), dense, q0, (double*)f);
  else
    hipLaunchKernelGGL(pack_kernel<float>, dim3(grid1(n), m), dim3(256), 0, s, g, make_shift(shift),
                       dense, q0, (float*)f);
  return hipGetLastError();
}

hipError_t launch_unpack(int storage, const Geometry& g, const double* shift, const void* f,
                         int q0, int m, double* dense, hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  if (storage == FP64)
    hipLaunchKernelGGL(unpack_kernel<double>, dim3(grid1(n), m), dim3(256), 0, s, g,
                       make_shift(shift), (const double*)f, q0, dense);
  else
    hipLaunchKernelGGL(unpack_kernel<float>, dim3(grid1(n), m), dim3(256), 0, s, g,
                       make_shift(shift), (const float*)f, q0, dense);
  return hipGetLastError();
}

hipError_t launch_reshift(int storage, const Geometry& g, const double* delta, void* f,
                          hipStream_t s) {
  Physics d{};
  for (int i = 0; i < Q; ++i) d.geq_c[i] = delta[i];
  const long long n = (long long)g.nx * g.ny;
  if (storage == FP64)
    hipLaunchKernelGGL(reshift_kernel<double>, dim3(grid1(n)), dim3(256), 0, s, g, d, (double*)f);
  else
    hipLaunchKernelGGL(reshift_kernel<float>, dim3(grid1(n)), dim3(256), 0, s, g, d, (float*)f);
  return hipGetLastError();
}

}  // namespace lbmk
