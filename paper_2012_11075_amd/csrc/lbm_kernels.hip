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
//   forcing term       Eq. (5) (standard) / Eq. (26) (WB); or, for the
//                      standard LBE, (c_i - u).F feq_i / (cs2 rho), the
//                      form named after Eq. (5) (STANDARD_EQF)
//   collide + stream   Eq. (2): f*_i = f_i - (f_i - feq_i)/tau + (1 - 1/2tau) F_i,
//                      f_i(x + c_i, t+1) = f*_i(x, t), periodic.
//
// Design (one HBM pass per step).  Populations are stored row-interleaved:
// lattice row y holds its nine population rows one after another (element
// (x, y, q) at y * pitch + q * plane + x, plane = nx rounded up to 32,
// pitch = 9 * plane), x fastest within each.  A block of BW threads owns an
// aligned strip of BW output columns and marches along a chunk of rows.  Each thread loads the 9
// populations of one column per row (coalesced along x) one row ahead of use,
// keeps the last three rows in registers, and publishes rho of the row to a 5-row LDS ring; mu of
// the previous row goes to a 3-row LDS ring.  The 2-column x-halo of rho is
// recomputed from populations that 36 lanes of the first wave load (one each),
// the 2-row y-halo by reading two extra rows at each end of the chunk, so no
// block ever waits for another.  Collision and streaming are fused in pull
// form: the buffers hold post-collision populations; a step reads f_i of node
// x from x - c_i of one buffer (misaligned loads are cheap) and writes the
// new post-collision values of x, aligned and non-temporal, to the other.
// rho, mu and u of every node come from the same device code in the step and
// in the observe pass.
#include <hip/hip_runtime.h>

#include "lbm_kernels.h"

// Multiply-adds are fused only within one source expression, never across
// statements: the fusion is then fixed by the code as written, not by how
// the compiler lays out a kernel's blocks, so kernels of different shape
// that evaluate a node with the same expressions (every tile, the observe
// pass, the batched step) round it the same way, bit for bit.
#pragma clang fp contract(on)

namespace lbmk {
namespace {

template <typename R>
struct PhysR {
  R omega, fpre, beta, kappa, rho_l, rho_v, rho_ref;
  R c[3];  // feq_i(rho_ref, 0) - s_i of the rest, axis and diagonal shells
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
  q.c[0] = (R)p.geq_c[0];
  q.c[1] = (R)p.geq_c[1];
  q.c[2] = (R)p.geq_c[5];
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

// 1/rho: the hardware reciprocal refined by two Newton steps (relative error
// a few units in the last place, far below the step's tolerances; the same
// function serves the step and the observe pass).
__device__ __forceinline__ double recip(double a) {
  double r = __builtin_amdgcn_rcp(a);
  r = r * (2.0 - a * r);
  return r * (2.0 - a * r);
}
__device__ __forceinline__ float recip(float a) {
  float r = __builtin_amdgcn_rcpf(a);
  return r * (2.0f - a * r);
}

// Velocity of Eq. (4): u = (sum_i c_i f_i + F/2) / rho.
template <typename R>
__device__ __forceinline__ void velocity(const R (&f)[Q], R rho, R Fx, R Fy, R& ux, R& uy) {
  const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
  const R jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
  const R inv = recip(rho);
  ux = (jx + (R)0.5 * Fx) * inv;
  uy = (jy + (R)0.5 * Fy) * inv;
}

// Collision of Eq. (2), f*_i = f_i - omega (f_i - geq_i) + fpre F_i, with the
// shifted equilibrium geq_i = feq_i(rho, u) - s_i and the forcing term F_i:
//   standard: feq_i = w_i rho (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)     (Eq. 3)
//             F_i   = w_i (3 c.F + 9 (c.u)(c.F) - 3 u.F)              (Eq. 5)
//   STANDARD_EQF: feq_i as above, F_i = 3 (c - u).F feq_i / rho
//             = w_i (1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u)(3 c.F - 3 u.F)
//   WB:       feq_0 = rho - (1-w0) rho0 - 1.5 w0 rho u.u,
//             feq_i = w_i (rho0 + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)) (Eq. 24)
//             F_i   = w_i (3 c.F + 9 (c.u)(c.G) - 3 u.G
//                          + (3|c_i|^2 - 2)/2 (u.grad rho)),  G = F + grad(rho)/3  (Eq. 26)
// feq_i(rho, u) - feq_i(rho_ref, 0) is evaluated from drho = rho - rho_ref
// (the rho0 terms cancel); feq_i(rho_ref, 0) - s_i is the shell constant
// p.c.  A velocity c_i and its opposite share every term of geq and F_i that
// is even in c_i, so each pair evaluates its even and odd parts once.  The
// relaxation keeps the form f - omega (f - geq), whose rounding stays
// proportional to the small non-equilibrium part (mass is conserved to
// round-off of that part, whatever the rounding of omega).
template <typename R, int SCHEME>
__device__ __forceinline__ void collide(R (&f)[Q], R drho, R rho, R ux, R uy, R Fx, R Fy, R grx,
                                        R gry, const PhysR<R>& p) {
  const R w0 = (R)4 / (R)9, w1 = (R)1 / (R)9, w2 = (R)1 / (R)36;
  const R u15 = (R)1.5 * (ux * ux + uy * uy);
  R Gx = Fx, Gy = Fy;
  if (SCHEME == WELL_BALANCED) {
    Gx = Fx + grx * ((R)1 / (R)3);
    Gy = Fy + gry * ((R)1 / (R)3);
  }
  const R uG3 = (R)3 * (ux * Gx + uy * Gy);
  const R ugr = ux * grx + uy * gry;
  const R om = p.omega, fp = p.fpre;
  // even forcing constant of a shell: k_i u.grad(rho) - 3 u.G (k = 1/2, 2 for WB)
  R ev1 = -uG3, ev2 = -uG3;
  if (SCHEME == WELL_BALANCED) {
    ev1 = (R)0.5 * ugr - uG3;
    ev2 = (R)2 * ugr - uG3;
  }
  auto pair = [&](int i, int j, R cu, R cF, R cG, R w, R c, R ev) {
    const R ep = (R)4.5 * (cu * cu) - u15;  // even part of poly_i
    const R wr = w * rho;
    // even and odd parts of geq_i, then of fpre F_i
    const R E = (SCHEME == WELL_BALANCED ? wr * ep : w * drho + wr * ep) + c;
    const R O = (R)3 * wr * cu;
    R Fe, Fo;
    if (SCHEME == STANDARD_EQF) {  // F_i = w (1 + ep + 3 cu)(3 cF - uG3)
      const R e1 = (R)1 + ep;
      Fe = w * ((R)9 * cu * cF + e1 * ev);
      Fo = (R)3 * w * (e1 * cF - cu * uG3);
    } else {
      Fe = w * ((R)9 * cu * (SCHEME == WELL_BALANCED ? cG : cF) + ev);
      Fo = (R)3 * w * cF;
    }
    const R Fp = fp * (Fe + Fo), Fm = fp * (Fe - Fo);
    f[i] = f[i] - om * ((f[i] - E) - O) + Fp;
    f[j] = f[j] - om * ((f[j] - E) + O) + Fm;
  };
  pair(1, 3, ux, Fx, Gx, w1, p.c[1], ev1);
  pair(2, 4, uy, Fy, Gy, w1, p.c[1], ev1);
  pair(5, 7, ux + uy, Fx + Fy, Gx + Gy, w2, p.c[2], ev2);
  pair(6, 8, uy - ux, Fy - Fx, Gy - Gx, w2, p.c[2], ev2);
  // rest population (c_0 = 0)
  R g0, F0;
  if (SCHEME == WELL_BALANCED) {
    g0 = (drho - w0 * rho * u15) + p.c[0];
    F0 = -w0 * (uG3 + ugr);
  } else {
    g0 = w0 * (drho - rho * u15) + p.c[0];
    F0 = SCHEME == STANDARD ? -w0 * uG3 : -w0 * ((R)1 - u15) * uG3;
  }
  f[0] = f[0] - om * (f[0] - g0) + fp * F0;
}

// Populations are addressed through global-address-space pointers.  A
// pointer read from device memory (the batched slot table) is otherwise
// generic to the compiler, which then emits flat loads and stores; those
// count against the LDS wait counter as well, so every LDS wait of the march
// would also wait for the rows in flight.
template <typename T>
using Global = __attribute__((address_space(1))) T;

// Marching step / observe kernel.  T: storage and arithmetic type; BW:
// threads per block = output columns per block; D: rows of populations in
// flight ahead of the row being summed.
template <typename T, int SCHEME, int BW, int D, bool OBSERVE>
__device__ __forceinline__ void march_tile(const Geometry& g, const Physics& phys,
                                           const Tiling& tl, int tile,
                                           const Global<T>* __restrict__ fin,
                                           Global<T>* __restrict__ fout,
                                           const ObserveOut& obs) {
  using R = T;
  // LDS column j of the rho ring holds lattice column x0 - 2 + j (periodic).
  __shared__ R rs[5][BW + 4];  // rho: rows y-2 .. y+2 of the output row y
  __shared__ R fl[2][Q][BW];   // populations of rows y and y+1, each thread its own column
  // mu stays in registers: each thread evaluates it at its own column and at
  // both neighbours, for the three rows that its node's gradient needs
  // (mu3[0..2] = row index k-3 .. k-1 at stage k; [.][0..2] = x-1, x, x+1).
  // Every value is computed by the same expression from the same rho, so it
  // is bit-identical to the value of the column's own thread; the price is
  // two extra evaluations per node, the gain one block-wide barrier per row.
  R mu3[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) mu3[a][b] = (R)0;
  const PhysR<R> p = to_r<R>(phys);
  const int t = threadIdx.x;
  const int chunk = tile / tl.strips;
  const int strip = tile - chunk * tl.strips;

  // Strips are BW columns wide and start on a multiple of BW, so loads and
  // stores of a row are aligned to whole cache lines.
  const int x0 = strip * BW;
  const int x = x0 + t;
  const bool outc = x < g.nx;
  const int xc = x % g.nx;
  const int y0 = chunk * tl.rows;
  const int H = min(tl.rows, g.ny - y0);
  const int K = H + 4;
  // Odd chunks march upward, so that vertically adjacent blocks read the two
  // halo rows they share at about the same time (L2 hits instead of a second
  // HBM fetch).  Row index k is lattice row y0 - 2 + k (down) or
  // y0 + H + 1 - k (up); the stencils are symmetric in y, and the y
  // gradients take the sign of the direction, so results are bit-identical.
  const bool up = (chunk & 1) != 0;
  auto wrapy = [&](int y) {
    y %= g.ny;
    return y < 0 ? y + g.ny : y;
  };
  auto row_of = [&](int k) { return wrapy(up ? y0 + H + 1 - k : y0 - 2 + k); };

  // Rows advance by one per stage in the march direction: the row loaded
  // next and the row of the node updated at the current stage are carried
  // from stage to stage (no division per stage).
  auto next_row = [&](int y) {
    y += up ? -1 : 1;
    return y < 0 ? y + g.ny : (y >= g.ny ? y - g.ny : y);
  };
  auto row_above = [&](int y) { return (y == 0) ? g.ny - 1 : y - 1; };
  auto row_below = [&](int y) { return (y + 1 == g.ny) ? 0 : y + 1; };

  // Pull streaming: the buffers hold post-collision populations, so f_i at
  // (x, y) is read from (x - c_ix, y - c_iy) of the previous step.  Each
  // access is a row base common to the wave (population q of lattice row y)
  // plus this lane's byte offset within that population row, which stays
  // below 2^32 (nx * 8 bytes), so loads and stores take a scalar base and a
  // 32-bit lane offset.
  const int xw = (xc == 0) ? g.nx - 1 : xc - 1;
  const int xe = (xc + 1 == g.nx) ? 0 : xc + 1;
  const unsigned bc = (unsigned)xc * (unsigned)sizeof(T), bw = (unsigned)xw * (unsigned)sizeof(T),
                 be = (unsigned)xe * (unsigned)sizeof(T);
  auto at = [](const Global<T>* row, unsigned b) -> T {
    return *(const Global<T>*)((const Global<char>*)row + b);
  };
  auto load_row = [&](int y, R(&dst)[Q]) {
    const long long P = g.plane;
    const Global<T>* r0 = fin + (long long)y * g.pitch;
    const Global<T>* ru = fin + (long long)row_above(y) * g.pitch;
    const Global<T>* rd = fin + (long long)row_below(y) * g.pitch;
    dst[0] = at(r0, bc);
    dst[1] = at(r0 + P, bw);
    dst[2] = at(ru + 2 * P, bc);
    dst[3] = at(r0 + 3 * P, be);
    dst[4] = at(rd + 4 * P, bc);
    dst[5] = at(ru + 5 * P, bw);
    dst[6] = at(ru + 6 * P, be);
    dst[7] = at(rd + 7 * P, be);
    dst[8] = at(rd + 8 * P, bw);
  };

  // The four halo columns x0-2, x0-1, x0+BW, x0+BW+1 need rho only.  Lane
  // L < 36 of wave 0 loads one population (column L/9, velocity L%9) per row;
  // the nine lanes of a column are gathered by shuffles and summed in the
  // same order as an interior column, so a node's rho is bit-identical in
  // every block that computes it.
  const bool hl = t < 4 * Q;
  const int hcol = t / Q, hq = t - Q * (t / Q);
  const int hslot = hcol < 2 ? hcol : BW + hcol;  // rho-ring column of the halo
  int hsx = 0, hcy = 0;
  long long hplane = 0;
  if (hl) {
    // c_x, c_y of velocity hq (paper numbering), without an indexed array
    // (which would live in scratch memory)
    const int cxq = (hq == 1 || hq == 5 || hq == 8) ? 1 : ((hq == 3 || hq == 6 || hq == 7) ? -1 : 0);
    const int cyq = (hq == 2 || hq == 5 || hq == 6) ? 1 : ((hq == 4 || hq == 7 || hq == 8) ? -1 : 0);
    int hc = hcol < 2 ? x0 - 2 + hcol : x0 + BW + hcol - 2;
    hc = ((hc % g.nx) + g.nx) % g.nx;
    hsx = hc - cxq;
    hsx = hsx < 0 ? hsx + g.nx : (hsx >= g.nx ? hsx - g.nx : hsx);
    hcy = cyq;
    hplane = (long long)hq * g.plane;
  }
  auto load_halo = [&](int y, R& dst) {
    if (hl) {
      const int hy = hcy > 0 ? row_above(y) : (hcy < 0 ? row_below(y) : y);
      dst = fin[hplane + (long long)hy * g.pitch + hsx];
    }
  };
  int yload = row_of(0);  // row of the next population load
  int yupd = row_of(-2);  // row of the node updated at the current stage

  NodeSums acc;

  // One row step: prefetch row k+D into `nxt`; publish rho of row k (`cur`,
  // which then parks in LDS for two rows); mu of row k-1; update the node of
  // row k-2.  One barrier per row: the rho ring slot written at stage k + 1
  // holds row index k - 4, which no thread reads at stage k, and a thread
  // cannot reach stage k + 2 before every thread has left stage k.
  auto stage = [&](int k, R(&nxt)[Q], R(&cur)[Q], R& hnxt, R& hcur) {
    load_row(yload, nxt);  // rows past the chunk are valid (periodic) and unused
    load_halo(yload, hnxt);
    yload = next_row(yload);
    const int sk = k % 5;
    rs[sk][t + 2] = p.rho_ref + sum9(cur);
    if (t < 64) {
      const int base = (hl ? hcol : 0) * Q;
      R v[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i] = __shfl(hcur, base + i);
      if (hl && hq == 0) rs[sk][hslot] = p.rho_ref + sum9(v);
    }
    R out[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      out[i] = fl[k & 1][i][t];  // row k-2 (garbage for k < 2, unused)
      fl[k & 1][i][t] = cur[i];
    }
    __syncthreads();
    if (k >= 2) {
      // mu at row index k-1: mu0(rho) - kappa lap(rho), 9-point Laplacian, at
      // ring column m (rho-ring columns m .. m+2), for this column and its
      // two neighbours (no exchange through LDS)
      const int a = (k - 2) % 5, c0 = (k - 1) % 5, d = sk;
      auto mu_at = [&](int m) {
        const R r0 = rs[c0][m + 1];
        const R ax = (rs[c0][m + 2] + rs[c0][m]) + (rs[a][m + 1] + rs[d][m + 1]);
        const R dg = (rs[a][m + 2] + rs[a][m]) + (rs[d][m + 2] + rs[d][m]);
        const R lap = ((R)4 * ax + dg - (R)20 * r0) * ((R)1 / (R)6);
        return mu0(r0, p) - p.kappa * lap;
      };
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        mu3[0][b] = mu3[1][b];
        mu3[1][b] = mu3[2][b];
      }
      mu3[2][0] = mu_at(t);
      mu3[2][1] = mu_at(t + 1);
      mu3[2][2] = mu_at(t + 2);
    }
    if (k >= 4 && k < K && outc) {
      const int sM = (k - 3) % 5, s0 = (k - 2) % 5, sP = (k - 1) % 5;
      const R third = (R)1 / (R)3, twelfth = (R)1 / (R)12;
      const R rho = rs[s0][t + 2];
      const R grx = (rs[s0][t + 3] - rs[s0][t + 1]) * third +
                    ((rs[sP][t + 3] - rs[sP][t + 1]) + (rs[sM][t + 3] - rs[sM][t + 1])) * twelfth;
      R gry = (rs[sP][t + 2] - rs[sM][t + 2]) * third +
              ((rs[sP][t + 3] + rs[sP][t + 1]) - (rs[sM][t + 3] + rs[sM][t + 1])) * twelfth;
      const R gmx = (mu3[1][2] - mu3[1][0]) * third +
                    ((mu3[2][2] - mu3[2][0]) + (mu3[0][2] - mu3[0][0])) * twelfth;
      R gmy = (mu3[2][1] - mu3[0][1]) * third +
              ((mu3[2][2] + mu3[2][0]) - (mu3[0][2] + mu3[0][0])) * twelfth;
      if (up) {
        gry = -gry;
        gmy = -gmy;
      }
      R Fx = -rho * gmx, Fy = -rho * gmy;
      if (SCHEME != WELL_BALANCED) {
        Fx += grx * third;
        Fy += gry * third;
      }
      R ux, uy;
      velocity(out, rho, Fx, Fy, ux, uy);
      const int y = yupd;
      if (!OBSERVE) {
        // FP64 storage carries no shift: rho = 0 + sum9 of the same values
        const R drho = sizeof(T) == 8 ? rho : sum9(out);
        collide<R, SCHEME>(out, drho, rho, ux, uy, Fx, Fy, grx, gry, p);
        // post-collision populations stay at their node (aligned, streaming stores)
        Global<T>* dst = fout + (long long)y * g.pitch;
        const unsigned bx = (unsigned)x * (unsigned)sizeof(T);
#pragma unroll
        for (int i = 0; i < Q; ++i)
          __builtin_nontemporal_store(
              out[i], (Global<T>*)((Global<char>*)(dst + (long long)i * g.plane) + bx));
      } else {
        const long long o = (long long)y * g.nx + x;
        const double drho = (double)rho, dux = (double)ux, duy = (double)uy;
        if (obs.rho) obs.rho[o] = drho;
        if (obs.ux) obs.ux[o] = dux;
        if (obs.uy) obs.uy[o] = duy;
        if (obs.mu) obs.mu[o] = (double)mu3[1][1];
        const double u2 = dux * dux + duy * duy;
        const double um = sqrt(u2);
        if (!(isfinite(drho) && drho > 0.0 && isfinite(um))) acc.bad = 1.0;
        acc.umax = fmax(acc.umax, um);
        acc.mass += drho;
        acc.ekin += 0.5 * drho * u2;
        acc.px += drho * dux;
        acc.py += drho * duy;
      }
    }
    yupd = next_row(yupd);
  };

  // Row r lives in register set r % (D+1).  The loop is unrolled by D+1 and
  // is straight-line (the trip count is rounded up; the extra stages store
  // nothing), so no set is copied and every prefetch stays in flight until
  // its row is summed.
  R s0[Q], s1[Q], s2[Q], s3[Q];
  R h0 = (R)0, h1 = (R)0, h2 = (R)0, h3 = (R)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) s0[i] = s1[i] = s2[i] = s3[i] = (R)0;
  load_row(yload, s0);
  load_halo(yload, h0);
  yload = next_row(yload);
  if (D >= 2) {
    load_row(yload, s1);
    load_halo(yload, h1);
    yload = next_row(yload);
  }
  if (D >= 3) {
    load_row(yload, s2);
    load_halo(yload, h2);
    yload = next_row(yload);
  }
  for (int k = 0; k < K; k += D + 1) {
    if (D == 1) {
      stage(k, s1, s0, h1, h0);
      stage(k + 1, s0, s1, h0, h1);
    } else if (D == 2) {
      stage(k, s2, s0, h2, h0);
      stage(k + 1, s0, s1, h0, h1);
      stage(k + 2, s1, s2, h1, h2);
    } else {
      stage(k, s3, s0, h3, h0);
      stage(k + 1, s0, s1, h0, h1);
      stage(k + 2, s1, s2, h1, h2);
      stage(k + 3, s2, s3, h2, h3);
    }
  }

  if (OBSERVE && obs.partials) write_block_partials<BW / 64>(acc, obs.partials + (long long)NPART * tile);
}

// One thread finishes the per-tile records in tile order: max of max|u| and
// of the non-finite flag, Neumaier sums of mass, kinetic energy and momentum
// (additions only, so no multiply-add contraction can change the rounding).
__global__ void __launch_bounds__(64) finish_partials_kernel(const double* __restrict__ part,
                                                             int count, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double umax = 0.0, bad = 0.0;
  double sum[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, comp[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < count; ++b) {
    const double* q = part + (long long)NPART * b;
    umax = fmax(umax, q[0]);
    bad = fmax(bad, q[3]);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const double v = q[k < 2 ? 1 + k : 2 + k];
      const double t = sum[k] + v;
      if (fabs(sum[k]) >= fabs(v))
        comp[k] += (sum[k] - t) + v;
      else
        comp[k] += (v - t) + sum[k];
      sum[k] = t;
    }
    if (!isfinite(q[1]) || !isfinite(q[2])) bad = 1.0;
  }
  out[0] = umax;
  out[1] = sum[0] + comp[0];
  out[2] = sum[1] + comp[1];
  out[3] = bad;
  out[4] = sum[2] + comp[2];
  out[5] = sum[3] + comp[3];
  out[6] = sum[4] + comp[4];
  out[7] = 0.0;
}

// Tiles are assigned so that each XCD (blocks b, b+8, ...) walks a contiguous
// range of tiles: neighbouring strips share halo lines in L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  const int xcd = b & 7, l = b >> 3, q8 = nb >> 3, r8 = nb & 7;
  return xcd * q8 + min(xcd, r8) + l;
}

// Two steps in one pass (temporal blocking): the step reads and writes each
// population once per two steps instead of once per step.  A block of BW
// threads (128 or 256) runs the first step on BW consecutive
// columns (xa0 .. xa0 + BW - 1, xa0 = x0 - 3) and keeps its output rows in
// LDS; the second step reads them there and writes columns x0 .. x0 + BW - 7
// of the state two steps on.  LDS: four first-step output rows of 9 x BW
// values, both steps' rho rings and the first step's parked rows: 513 bytes
// (FP64) or 257 (FP32) per thread, so 131 KB for a 256-thread FP64 block (one
// per CU) and 66 KB for a 128-thread FP64 or 256-thread FP32 block (two per
// CU).  The second step's node needs
// first-step populations at x +- 3 (its pull, then rho at x +- 2 for mu and
// the gradients), hence the 6 columns the first step computes in addition.
// Along y the first step runs 3 rows ahead of the second step's chunk on each
// side.  One barrier per row: every LDS value a thread reads after the
// barrier of row k was written before it, or, for the rings written after
// the barrier, in a slot no thread reads during row k.  Each node is
// evaluated by the same expressions as in the one-step kernel, so the result
// is bit-identical to two launches of it.
template <typename T, int SCHEME, int D, int BW>
__device__ __forceinline__ void march2_tile(Geometry g, Physics phys, int rows,
                                            int strips, int tile, const T* __restrict__ fin_,
                                            T* __restrict__ fout_) {
  constexpr int M2S = BW - 6;
  using R = T;
  const Global<T>* fin = (const Global<T>*)fin_;
  Global<T>* fout = (Global<T>*)fout_;
  __shared__ R rs[5][BW + 4];  // first step's rho, column j = lattice xa0 - 2 + j
  __shared__ R fl[2][Q][BW];   // first step's populations of rows y, y+1 (own column)
  __shared__ R f1[4][Q][BW];   // first step's post-collision rows, column t = xa0 + t
  __shared__ R r2[5][BW + 4];  // second step's rho, column j = xa0 - 2 + j
  R mu3[3][3], mb[3][3];       // mu of the two steps, rows r-1 .. r+1 at columns x-1 .. x+1
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) mu3[a][b] = mb[a][b] = (R)0;
  const PhysR<R> p = to_r<R>(phys);
  const int t = threadIdx.x;
  const int chunk = tile / strips;
  const int strip = tile - chunk * strips;
  const int x0 = strip * M2S, xa0 = x0 - 3;
  auto wrapx = [&](int x) {
    x %= g.nx;
    return x < 0 ? x + g.nx : x;
  };
  const int xc = wrapx(xa0 + t);
  const int y0 = chunk * rows;
  const int H = min(rows, g.ny - y0);
  const int K = H + 12;
  const int xb = xa0 + t;  // the second step's output column of this thread
  const bool outc = t >= 3 && t < BW - 3 && xb < g.nx;
  auto wrapy = [&](int y) {
    y %= g.ny;
    return y < 0 ? y + g.ny : y;
  };
  auto next_row = [&](int y) { return y + 1 == g.ny ? 0 : y + 1; };
  auto row_above = [&](int y) { return (y == 0) ? g.ny - 1 : y - 1; };
  auto row_below = [&](int y) { return (y + 1 == g.ny) ? 0 : y + 1; };

  const int xw = (xc == 0) ? g.nx - 1 : xc - 1;
  const int xe = (xc + 1 == g.nx) ? 0 : xc + 1;
  const unsigned bc = (unsigned)xc * (unsigned)sizeof(T), bw = (unsigned)xw * (unsigned)sizeof(T),
                 be = (unsigned)xe * (unsigned)sizeof(T);
  auto at = [](const Global<T>* row, unsigned b) -> T {
    return *(const Global<T>*)((const Global<char>*)row + b);
  };
  auto load_row = [&](int y, R(&dst)[Q]) {
    const long long P = g.plane;
    const Global<T>* r0 = fin + (long long)y * g.pitch;
    const Global<T>* ru = fin + (long long)row_above(y) * g.pitch;
    const Global<T>* rd = fin + (long long)row_below(y) * g.pitch;
    dst[0] = at(r0, bc);
    dst[1] = at(r0 + P, bw);
    dst[2] = at(ru + 2 * P, bc);
    dst[3] = at(r0 + 3 * P, be);
    dst[4] = at(rd + 4 * P, bc);
    dst[5] = at(ru + 5 * P, bw);
    dst[6] = at(ru + 6 * P, be);
    dst[7] = at(rd + 7 * P, be);
    dst[8] = at(rd + 8 * P, bw);
  };
  const bool hl = t < 4 * Q;
  const int hcol = t / Q, hq = t - Q * (t / Q);
  const int hslot = hcol < 2 ? hcol : BW + hcol;
  int hsx = 0, hcy = 0;
  long long hplane = 0;
  if (hl) {
    const int cxq = (hq == 1 || hq == 5 || hq == 8) ? 1 : ((hq == 3 || hq == 6 || hq == 7) ? -1 : 0);
    const int cyq = (hq == 2 || hq == 5 || hq == 6) ? 1 : ((hq == 4 || hq == 7 || hq == 8) ? -1 : 0);
    int hc = hcol < 2 ? xa0 - 2 + hcol : xa0 + BW + hcol - 2;
    hc = ((hc % g.nx) + g.nx) % g.nx;
    hsx = hc - cxq;
    hsx = hsx < 0 ? hsx + g.nx : (hsx >= g.nx ? hsx - g.nx : hsx);
    hcy = cyq;
    hplane = (long long)hq * g.plane;
  }
  auto load_halo = [&](int y, R& dst) {
    if (hl) {
      const int hy = hcy > 0 ? row_above(y) : (hcy < 0 ? row_below(y) : y);
      dst = fin[hplane + (long long)hy * g.pitch + hsx];
    }
  };
  // first step's row index i <-> lattice row y0 - 5 + i
  int yload = wrapy(y0 - 5);
  const int tw = t > 0 ? t - 1 : 0, te = t + 1 < BW ? t + 1 : BW - 1;
  const R third = (R)1 / (R)3, twelfth = (R)1 / (R)12;

  // Row step k: first step as in the one-step kernel (rho of row k, mu of row
  // k-1, node of row k-2 into f1); second step: rho of row k-4 from f1 (rows
  // k-5 .. k-3, written in earlier steps), its pulled populations into Bn;
  // mu of row k-6; node of row k-7 (populations in Bu, pulled at row k-3)
  // into fout.
  auto stage = [&](int k, R(&nxt)[Q], R(&cur)[Q], R& hnxt, R& hcur, R(&Bn)[Q], R(&Bu)[Q]) {
    load_row(yload, nxt);
    load_halo(yload, hnxt);
    yload = next_row(yload);
    const int sk = k % 5;
    rs[sk][t + 2] = p.rho_ref + sum9(cur);
    if (t < 64) {
      const int base = (hl ? hcol : 0) * Q;
      R v[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i] = __shfl(hcur, base + i);
      if (hl && hq == 0) rs[sk][hslot] = p.rho_ref + sum9(v);
    }
    R out[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      out[i] = fl[k & 1][i][t];
      fl[k & 1][i][t] = cur[i];
    }
    __syncthreads();
    auto lap_mu = [&](R(&ring)[5][BW + 4], int a, int c0, int d, int m) {
      const R r0 = ring[c0][m + 1];
      const R ax = (ring[c0][m + 2] + ring[c0][m]) + (ring[a][m + 1] + ring[d][m + 1]);
      const R dg = (ring[a][m + 2] + ring[a][m]) + (ring[d][m + 2] + ring[d][m]);
      const R lap = ((R)4 * ax + dg - (R)20 * r0) * ((R)1 / (R)6);
      return mu0(r0, p) - p.kappa * lap;
    };
    // first step
    if (k >= 2) {
      const int a = (k - 2) % 5, c0 = (k - 1) % 5, d = sk;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        mu3[0][b] = mu3[1][b];
        mu3[1][b] = mu3[2][b];
      }
      mu3[2][0] = lap_mu(rs, a, c0, d, t);
      mu3[2][1] = lap_mu(rs, a, c0, d, t + 1);
      mu3[2][2] = lap_mu(rs, a, c0, d, t + 2);
    }
    if (k >= 4) {
      const int sM = (k - 3) % 5, s0 = (k - 2) % 5, sP = (k - 1) % 5;
      const R rho = rs[s0][t + 2];
      const R grx = (rs[s0][t + 3] - rs[s0][t + 1]) * third +
                    ((rs[sP][t + 3] - rs[sP][t + 1]) + (rs[sM][t + 3] - rs[sM][t + 1])) * twelfth;
      const R gry = (rs[sP][t + 2] - rs[sM][t + 2]) * third +
                    ((rs[sP][t + 3] + rs[sP][t + 1]) - (rs[sM][t + 3] + rs[sM][t + 1])) * twelfth;
      const R gmx = (mu3[1][2] - mu3[1][0]) * third +
                    ((mu3[2][2] - mu3[2][0]) + (mu3[0][2] - mu3[0][0])) * twelfth;
      const R gmy = (mu3[2][1] - mu3[0][1]) * third +
                    ((mu3[2][2] + mu3[2][0]) - (mu3[0][2] + mu3[0][0])) * twelfth;
      R Fx = -rho * gmx, Fy = -rho * gmy;
      if (SCHEME != WELL_BALANCED) {
        Fx += grx * third;
        Fy += gry * third;
      }
      R ux, uy;
      velocity(out, rho, Fx, Fy, ux, uy);
      const R drho = sizeof(T) == 8 ? rho : sum9(out);
      collide<R, SCHEME>(out, drho, rho, ux, uy, Fx, Fy, grx, gry, p);
      const int so = (k - 2) & 3;
#pragma unroll
      for (int i = 0; i < Q; ++i) f1[so][i][t] = out[i];
    }
    // second step: rho of row k-4 (k >= 4)
    {
      const int sm = (k + 3) & 3, s0 = k & 3, sp = (k + 1) & 3;  // rows k-5, k-4, k-3
      Bn[0] = f1[s0][0][t];
      Bn[1] = f1[s0][1][tw];
      Bn[2] = f1[sm][2][t];
      Bn[3] = f1[s0][3][te];
      Bn[4] = f1[sp][4][t];
      Bn[5] = f1[sm][5][tw];
      Bn[6] = f1[sm][6][te];
      Bn[7] = f1[sp][7][te];
      Bn[8] = f1[sp][8][tw];
    }
    // mu of row k-6 from r2 rows k-7 .. k-5 (written at rows k-3 .. k-1)
    {
      const int a = (k + 3) % 5, c0 = (k + 4) % 5, d = k % 5;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        mb[0][b] = mb[1][b];
        mb[1][b] = mb[2][b];
      }
      mb[2][0] = lap_mu(r2, a, c0, d, t);
      mb[2][1] = lap_mu(r2, a, c0, d, t + 1);
      mb[2][2] = lap_mu(r2, a, c0, d, t + 2);
    }
    if (k >= 12 && k < K && outc) {
      const int sM = (k + 2) % 5, s0 = (k + 3) % 5, sP = (k + 4) % 5;  // rows k-8 .. k-6
      const R rho = r2[s0][t + 2];
      const R grx = (r2[s0][t + 3] - r2[s0][t + 1]) * third +
                    ((r2[sP][t + 3] - r2[sP][t + 1]) + (r2[sM][t + 3] - r2[sM][t + 1])) * twelfth;
      const R gry = (r2[sP][t + 2] - r2[sM][t + 2]) * third +
                    ((r2[sP][t + 3] + r2[sP][t + 1]) - (r2[sM][t + 3] + r2[sM][t + 1])) * twelfth;
      const R gmx = (mb[1][2] - mb[1][0]) * third +
                    ((mb[2][2] - mb[2][0]) + (mb[0][2] - mb[0][0])) * twelfth;
      const R gmy = (mb[2][1] - mb[0][1]) * third +
                    ((mb[2][2] + mb[2][0]) - (mb[0][2] + mb[0][0])) * twelfth;
      R Fx = -rho * gmx, Fy = -rho * gmy;
      if (SCHEME != WELL_BALANCED) {
        Fx += grx * third;
        Fy += gry * third;
      }
      R o2[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) o2[i] = Bu[i];
      R ux, uy;
      velocity(o2, rho, Fx, Fy, ux, uy);
      const R drho = sizeof(T) == 8 ? rho : sum9(o2);
      collide<R, SCHEME>(o2, drho, rho, ux, uy, Fx, Fy, grx, gry, p);
      Global<T>* dst = fout + (long long)(y0 + k - 12) * g.pitch;
      const unsigned bx = (unsigned)xb * (unsigned)sizeof(T);
#pragma unroll
      for (int i = 0; i < Q; ++i)
        __builtin_nontemporal_store(
            o2[i], (Global<T>*)((Global<char>*)(dst + (long long)i * g.plane) + bx));
    }
    // second step's rho of row k-4 (read from row k+1 on)
    r2[(k + 1) % 5][t + 2] = p.rho_ref + sum9(Bn);
  };

  R s0[Q], s1[Q], s2[Q], s3[Q], B0[Q], B1[Q], B2[Q], B3[Q];
  R h0 = (R)0, h1 = (R)0, h2 = (R)0, h3 = (R)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) s0[i] = s1[i] = s2[i] = s3[i] = B0[i] = B1[i] = B2[i] = B3[i] = (R)0;
  static_assert(D == 3, "the two-step kernel prefetches three rows");
  load_row(yload, s0);
  load_halo(yload, h0);
  yload = next_row(yload);
  load_row(yload, s1);
  load_halo(yload, h1);
  yload = next_row(yload);
  load_row(yload, s2);
  load_halo(yload, h2);
  yload = next_row(yload);
  for (int k = 0; k < K; k += 4) {
    stage(k, s3, s0, h3, h0, B0, B1);
    stage(k + 1, s0, s1, h0, h1, B1, B2);
    stage(k + 2, s1, s2, h1, h2, B2, B3);
    stage(k + 3, s2, s3, h2, h3, B3, B0);
  }
}

// One lattice, two steps: one block per tile of `strips` x `chunks`.
template <typename T, int SCHEME, int D, int BW>
__global__ void __launch_bounds__(BW)
    march2(Geometry g, Physics phys, int rows, int strips, int chunks, const T* __restrict__ fin,
           T* __restrict__ fout) {
  march2_tile<T, SCHEME, D, BW>(g, phys, rows, strips, xcd_tile(blockIdx.x, strips * chunks), fin,
                                fout);
}

// One lattice: one block per tile.
template <typename T, int SCHEME, int BW, int D, bool OBSERVE>
__global__ void __launch_bounds__(BW)
    march(Geometry g, Physics phys, Tiling tl, const T* __restrict__ fin, T* __restrict__ fout,
          ObserveOut obs) {
  const int tile = xcd_tile(blockIdx.x, tl.strips * tl.chunks);
  march_tile<T, SCHEME, BW, D, OBSERVE>(g, phys, tl, tile, (const Global<T>*)fin,
                                        (Global<T>*)fout, obs);
}

// Many lattices in one launch: one block per work item (one tile of one
// lattice) of the table's concatenated tile list, so the hardware dispatcher
// balances uneven lattices as blocks finish.  Items are mapped XCD-aware as
// in the single-lattice launch (blocks b, b+8, ... of one XCD walk a
// contiguous range of the list), so horizontally adjacent tiles run together
// on one XCD and share their halo lines in its L2.  The table lives in
// device memory; `parity` selects which of each slot's two buffers is read.
// Slot of work item `item`: the last slot whose first tile <= item (a
// search uniform over the block).
__device__ __forceinline__ int slot_of_item(const BatchTable* __restrict__ tab, int item) {
  int lo = 0, hi = tab->nslots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab->slot[mid].tile0 <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

template <typename T, int SCHEME, int BW, int D, bool OBSERVE>
__global__ void __launch_bounds__(BW) march_batch(const BatchTable* __restrict__ tab, int parity) {
  const int total = tab->total_tiles;
  const int item = xcd_tile(blockIdx.x, total);
  if (item >= total) return;
  const int lo = slot_of_item(tab, item);
  // The slot's record is copied into locals: read through a reference into
  // the table, its fields would be re-loaded after every population store
  // (the compiler cannot rule out that the stores alias the table), and each
  // scalar re-load waits on outstanding LDS traffic.
  const BatchSlot* sp = &tab->slot[lo];
  const Geometry g = sp->g;
  const Physics ph = sp->ph;
  const Tiling tl = sp->tl;
  const int which = sp->cur ^ parity;
  const Global<T>* fin = (const Global<T>*)(const T*)sp->buf[which];
  Global<T>* fout = (Global<T>*)(T*)sp->buf[which ^ 1];
  const ObserveOut o{nullptr, nullptr, nullptr, nullptr, sp->partials};
  march_tile<T, SCHEME, BW, D, OBSERVE>(g, ph, tl, item - sp->tile0, fin, fout, o);
}

// Two steps per launch over a batch: as march_batch, with each slot's tiling
// holding the two-step strips (BW - 6 columns) and chunks; the state moves
// from buffer `which` to the other one, two steps on.
template <typename T, int SCHEME, int BW>
__global__ void __launch_bounds__(BW) march2_batch(const BatchTable* __restrict__ tab, int parity) {
  const int total = tab->total_tiles;
  const int item = xcd_tile(blockIdx.x, total);
  if (item >= total) return;
  const BatchSlot* sp = &tab->slot[slot_of_item(tab, item)];
  const Geometry g = sp->g;
  const Physics ph = sp->ph;
  const int rows = sp->tl.rows, strips = sp->tl.strips, tile = item - sp->tile0;
  const int which = sp->cur ^ parity;
  march2_tile<T, SCHEME, 3, BW>(g, ph, rows, strips, tile, (const T*)sp->buf[which],
                                (T*)sp->buf[which ^ 1]);
}

// Offset, within a plane, of the slot the next pull reads population q of
// node (x, y) from: (x - c_qx, y - c_qy), periodic.
__device__ __forceinline__ long long src_offset(const Geometry& g, int q, int x, int y) {
  const int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  int xs = x - cx[q], ys = y - cy[q];
  xs = xs < 0 ? xs + g.nx : (xs >= g.nx ? xs - g.nx : xs);
  ys = ys < 0 ? ys + g.ny : (ys >= g.ny ? ys - g.ny : ys);
  return (long long)ys * g.pitch + xs;
}

// ---------------------------------------------------------------------------
// Force-stencil variant (Sec. II, after Eq. 23): the gradients of the force
// (and of Eq. 26) use the fourth-order form grad(phi) - (1/6) grad(lap phi)
// of the central gradient and the isotropic Laplacian above, which removes
// the central gradient's isotropic second-order error (1-D:
// (-phi_{j+2} + 8 phi_{j+1} - 8 phi_{j-1} + phi_{j-2})/12).  The paper's
// point is that this shrinks the net force of the standard scheme at
// equilibrium but cannot remove it.  FP64.  The step is one fused pass
// (`march4`); the observe pass takes three: density, chemical potential,
// then fields and reductions on LDS tiles of rho and mu with a 2-node halo.
// Expanded, the x-derivative's 5 x 5 weights are, for rows
// dy = 0, +-1, +-2 and columns dx = 1, 2 (odd in dx):
//   dy = 0:   1/2,    -1/24
//   dy = +-1: 5/54,   -1/54
//   dy = +-2: -1/108, -1/432
// and the y-derivative's are their transpose.

// The observe pass computes in the storage type T, as the step does (FP32
// storage: rho = rho_ref + sum_i g_i, then every stencil in FP32); fields
// are written as double.

// Pass 1: rho = sum_i f_i of every node (pulled populations, Eq. 4).
template <typename T>
__global__ void __launch_bounds__(256)
    density4(Geometry g, Physics phys, const Global<T>* __restrict__ fin,
             double* __restrict__ rho) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  T f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = fin[(long long)i * g.plane + src_offset(g, i, x, y)];
  rho[(long long)y * g.nx + x] = (double)((T)phys.rho_ref + sum9(f));
}

// Pass 2: mu = mu0(rho) - kappa lap(rho), 9-point isotropic Laplacian.
template <typename T>
__global__ void __launch_bounds__(256)
    potential4(Geometry g, Physics phys, const double* __restrict__ rho, double* __restrict__ mu) {
  using R = T;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y;
  if (x >= g.nx) return;
  const PhysR<R> p = to_r<R>(phys);
  const int xw = x == 0 ? g.nx - 1 : x - 1, xe = x + 1 == g.nx ? 0 : x + 1;
  const int ys = y == 0 ? g.ny - 1 : y - 1, yn = y + 1 == g.ny ? 0 : y + 1;
  const double* r0 = rho + (long long)y * g.nx;
  const double* rs = rho + (long long)ys * g.nx;
  const double* rn = rho + (long long)yn * g.nx;
  const R c = (R)r0[x];
  const R ax = ((R)r0[xe] + (R)r0[xw]) + ((R)rs[x] + (R)rn[x]);
  const R dg = ((R)rs[xe] + (R)rs[xw]) + ((R)rn[xe] + (R)rn[xw]);
  const R lap = ((R)4 * ax + dg - (R)20 * c) * ((R)1 / (R)6);
  mu[(long long)y * g.nx + x] = (double)(mu0(c, p) - p.kappa * lap);
}

constexpr int S4X = 64, S4Y = 4;  // collide-stream tile (threads)

// Fourth-order gradient at column j from the five rows y-2 .. y+2 (m2, m1,
// r0, p1, p2).  Swapping the rows (m2 <-> p2, m1 <-> p1) negates gy exactly
// and leaves gx unchanged.
template <typename R>
__device__ __forceinline__ void grad4r(const R* m2, const R* m1, const R* r0, const R* p1,
                                       const R* p2, int j, R& gx, R& gy) {
  auto dx1 = [&](const R* r) { return r[j + 1] - r[j - 1]; };
  auto dx2 = [&](const R* r) { return r[j + 2] - r[j - 2]; };
  auto dy1 = [&](int c) { return p1[c] - m1[c]; };
  auto dy2 = [&](int c) { return p2[c] - m2[c]; };
  const R a1 = (R)0.5, a2 = (R)1 / (R)24, b1 = (R)5 / (R)54, b2 = (R)1 / (R)54,
          c1 = (R)1 / (R)108, c2 = (R)1 / (R)432;
  gx = a1 * dx1(r0) - a2 * dx2(r0) + b1 * (dx1(p1) + dx1(m1)) - b2 * (dx2(p1) + dx2(m1)) -
       c1 * (dx1(p2) + dx1(m2)) - c2 * (dx2(p2) + dx2(m2));
  gy = a1 * dy1(j) - a2 * dy2(j) + b1 * (dy1(j + 1) + dy1(j - 1)) -
       b2 * (dy2(j + 1) + dy2(j - 1)) - c1 * (dy1(j + 2) + dy1(j - 2)) -
       c2 * (dy2(j + 2) + dy2(j - 2));
}

// Pass 3 of the observe pass: force with the fourth-order gradients and
// velocity of every node; writes the velocity fields and per-block partials
// (max|u|, mass, kinetic energy, non-finite).
template <typename T, int SCHEME>
__global__ void __launch_bounds__(S4X * S4Y)
    observe4_kernel(Geometry g, const Global<T>* __restrict__ fin,
                    const double* __restrict__ rho, const double* __restrict__ mu,
                    ObserveOut obs) {
  using R = T;
  __shared__ R rt[S4Y + 4][S4X + 4];
  __shared__ R mt[S4Y + 4][S4X + 4];
  const int tx = threadIdx.x % S4X, ty = threadIdx.x / S4X;
  const int x0 = blockIdx.x * S4X, y0 = blockIdx.y * S4Y;
  for (int e = threadIdx.x; e < (S4Y + 4) * (S4X + 4); e += S4X * S4Y) {
    const int i = e / (S4X + 4), j = e - i * (S4X + 4);
    int yy = (y0 + i - 2) % g.ny, xx = (x0 + j - 2) % g.nx;
    yy = yy < 0 ? yy + g.ny : yy;
    xx = xx < 0 ? xx + g.nx : xx;
    const long long o = (long long)yy * g.nx + xx;
    rt[i][j] = (R)rho[o];
    mt[i][j] = (R)mu[o];
  }
  __syncthreads();
  const int x = x0 + tx, y = y0 + ty;
  NodeSums acc;
  if (x < g.nx && y < g.ny) {
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = fin[(long long)i * g.plane + src_offset(g, i, x, y)];
    const R rr = rt[ty + 2][tx + 2];
    R grx, gry, gmx, gmy;
    const int i = ty + 2, j = tx + 2;
    grad4r<R>(rt[i - 2], rt[i - 1], rt[i], rt[i + 1], rt[i + 2], j, grx, gry);
    grad4r<R>(mt[i - 2], mt[i - 1], mt[i], mt[i + 1], mt[i + 2], j, gmx, gmy);
    R Fx = -rr * gmx, Fy = -rr * gmy;
    if (SCHEME != WELL_BALANCED) {
      Fx += grx * ((R)1 / (R)3);
      Fy += gry * ((R)1 / (R)3);
    }
    R uxr, uyr;
    velocity(f, rr, Fx, Fy, uxr, uyr);
    const double r = (double)rr, ux = (double)uxr, uy = (double)uyr;
    const long long o = (long long)y * g.nx + x;
    if (obs.ux) obs.ux[o] = ux;
    if (obs.uy) obs.uy[o] = uy;
    const double u2 = ux * ux + uy * uy;
    const double um = sqrt(u2);
    if (!(isfinite(r) && r > 0.0 && isfinite(um))) acc.bad = 1.0;
    acc.umax = um;
    acc.mass = r;
    acc.ekin = 0.5 * r * u2;
    acc.px = r * ux;
    acc.py = r * uy;
  }
  if (obs.partials)
    write_block_partials<S4Y * S4X / 64>(
        acc, obs.partials + (long long)NPART * ((long long)blockIdx.y * gridDim.x + blockIdx.x));
}

// Fused step of the force-stencil variant (FP64): one HBM pass per step, as
// `march`, with the fourth-order gradients.  The gradients reach two nodes
// and the Laplacian inside mu one more, so the rho ring holds 7 rows
// (y-3 .. y+3), the mu ring 5, the x-halo is 3 columns on each side (54
// lanes of wave 0 load one population each), and a row is updated 3 rows
// after it is loaded (rows k-3 .. k-1 wait in LDS).  Stencil sums pair the
// rows above and below, so the march direction changes no bit of the result.
template <typename T, int SCHEME, int BW, int D>
__device__ __forceinline__ void march4_tile(const Geometry& g, const Physics& phys,
                                            const Tiling& tl, int tile,
                                            const Global<T>* __restrict__ fin,
                                            Global<T>* __restrict__ fout) {
  using R = T;
  __shared__ R rs[7][BW + 6];  // column j: lattice column x0 - 3 + j
  __shared__ R ms[5][BW + 4];  // column m: lattice column x0 - 2 + m
  __shared__ R fl[3][Q][BW];   // populations of rows k-3 .. k-1, each thread its own column
  const PhysR<R> p = to_r<R>(phys);
  const int t = threadIdx.x;
  const int chunk = tile / tl.strips;
  const int strip = tile - chunk * tl.strips;
  const int x0 = strip * BW;
  const int x = x0 + t;
  const bool outc = x < g.nx;
  const int xc = x % g.nx;
  const int y0 = chunk * tl.rows;
  const int H = min(tl.rows, g.ny - y0);
  const int K = H + 6;
  // Odd chunks march upward (as in `march`); row index k is lattice row
  // y0 - 3 + k (down) or y0 + H + 2 - k (up).
  const bool up = (chunk & 1) != 0;
  auto wrapy = [&](int y) {
    y %= g.ny;
    return y < 0 ? y + g.ny : y;
  };
  auto row_of = [&](int k) { return wrapy(up ? y0 + H + 2 - k : y0 - 3 + k); };

  const int xw = (xc == 0) ? g.nx - 1 : xc - 1;
  const int xe = (xc + 1 == g.nx) ? 0 : xc + 1;
  auto load_row = [&](int k, R(&dst)[Q]) {
    const int y = row_of(k);
    const int yu = (y == 0) ? g.ny - 1 : y - 1;
    const int yd = (y + 1 == g.ny) ? 0 : y + 1;
    const long long P = g.plane;
    const long long r0 = (long long)y * g.pitch, ru = (long long)yu * g.pitch,
                    rd = (long long)yd * g.pitch;
    dst[0] = fin[r0 + xc];
    dst[1] = fin[P + r0 + xw];
    dst[2] = fin[2 * P + ru + xc];
    dst[3] = fin[3 * P + r0 + xe];
    dst[4] = fin[4 * P + rd + xc];
    dst[5] = fin[5 * P + ru + xw];
    dst[6] = fin[6 * P + ru + xe];
    dst[7] = fin[7 * P + rd + xe];
    dst[8] = fin[8 * P + rd + xw];
  };

  // Halo columns x0-3 .. x0-1 and x0+BW .. x0+BW+2: lane L < 54 of wave 0
  // loads population L%9 of halo column L/9; rho is gathered by shuffles and
  // summed in the interior order.
  const bool hl = t < 6 * Q;
  const int hcol = t / Q, hq = t - Q * (t / Q);
  const int hslot = hcol < 3 ? hcol : BW + hcol;  // rho-ring column of the halo
  int hsx = 0, hcy = 0;
  long long hplane = 0;
  if (hl) {
    // c_x, c_y of velocity hq (paper numbering), without an indexed array
    const int cxq = (hq == 1 || hq == 5 || hq == 8) ? 1 : ((hq == 3 || hq == 6 || hq == 7) ? -1 : 0);
    const int cyq = (hq == 2 || hq == 5 || hq == 6) ? 1 : ((hq == 4 || hq == 7 || hq == 8) ? -1 : 0);
    int hc = hcol < 3 ? x0 - 3 + hcol : x0 + BW + hcol - 3;
    hc = ((hc % g.nx) + g.nx) % g.nx;
    hsx = hc - cxq;
    hsx = hsx < 0 ? hsx + g.nx : (hsx >= g.nx ? hsx - g.nx : hsx);
    hcy = cyq;
    hplane = (long long)hq * g.plane;
  }
  auto load_halo = [&](int k, R& dst) {
    if (hl) dst = fin[hplane + (long long)wrapy(row_of(k) - hcy) * g.pitch + hsx];
  };

  // One row step: prefetch row k+D; publish rho of row k (`cur`); mu of row
  // k-1; update the node of row k-3.
  auto stage = [&](int k, R(&nxt)[Q], R(&cur)[Q], R& hnxt, R& hcur) {
    load_row(k + D, nxt);  // rows past the chunk are valid (periodic) and unused
    load_halo(k + D, hnxt);
    const int sk = k % 7;
    rs[sk][t + 3] = p.rho_ref + sum9(cur);
    if (t < 64) {
      const int base = (hl ? hcol : 0) * Q;
      R v[Q];
#pragma unroll
      for (int i = 0; i < Q; ++i) v[i] = __shfl(hcur, base + i);
      if (hl && hq == 0) rs[sk][hslot] = p.rho_ref + sum9(v);
    }
    const int fk = k % 3;
    R out[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) {
      out[i] = fl[fk][i][t];  // row k-3 (garbage for k < 3, unused)
      fl[fk][i][t] = cur[i];
    }
    __syncthreads();
    if (k >= 2) {
      // mu at row index k-1 and mu-ring column m (rho-ring columns m .. m+2)
      const int a = (k - 2) % 7, c0 = (k - 1) % 7, d = sk, mk = (k - 1) % 5;
      auto mu_at = [&](int m) {
        const R r0 = rs[c0][m + 1];
        const R ax = (rs[c0][m + 2] + rs[c0][m]) + (rs[a][m + 1] + rs[d][m + 1]);
        const R dg = (rs[a][m + 2] + rs[a][m]) + (rs[d][m + 2] + rs[d][m]);
        const R lap = ((R)4 * ax + dg - (R)20 * r0) * ((R)1 / (R)6);
        ms[mk][m] = mu0(r0, p) - p.kappa * lap;
      };
      mu_at(t + 2);
      if (t < 4) mu_at(t < 2 ? t : BW + t);
    }
    __syncthreads();
    if (k >= 6 && k < K && outc) {
      const int q2 = (k - 5) % 7, q1 = (k - 4) % 7, q0 = (k - 3) % 7, p1 = (k - 2) % 7,
                p2 = (k - 1) % 7;
      const int n2 = (k - 5) % 5, n1 = (k - 4) % 5, n0 = (k - 3) % 5, o1 = (k - 2) % 5,
                o2 = (k - 1) % 5;
      const R rho = rs[q0][t + 3];
      R grx, gry, gmx, gmy;
      grad4r<R>(rs[q2], rs[q1], rs[q0], rs[p1], rs[p2], t + 3, grx, gry);
      grad4r<R>(ms[n2], ms[n1], ms[n0], ms[o1], ms[o2], t + 2, gmx, gmy);
      if (up) {
        gry = -gry;
        gmy = -gmy;
      }
      R Fx = -rho * gmx, Fy = -rho * gmy;
      if (SCHEME != WELL_BALANCED) {
        Fx += grx * ((R)1 / (R)3);
        Fy += gry * ((R)1 / (R)3);
      }
      R ux, uy;
      velocity(out, rho, Fx, Fy, ux, uy);
      const R drho = sum9(out);
      collide<R, SCHEME>(out, drho, rho, ux, uy, Fx, Fy, grx, gry, p);
      Global<T>* dst = fout + (long long)row_of(k - 3) * g.pitch + x;
#pragma unroll
      for (int i = 0; i < Q; ++i) __builtin_nontemporal_store(out[i], dst + (long long)i * g.plane);
    }
  };

  // Row r lives in register set r % (D+1), as in `march`.
  R s0[Q], s1[Q], s2[Q], s3[Q];
  R h0 = (R)0, h1 = (R)0, h2 = (R)0, h3 = (R)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) s0[i] = s1[i] = s2[i] = s3[i] = (R)0;
  load_row(0, s0);
  load_halo(0, h0);
  if (D >= 2) {
    load_row(1, s1);
    load_halo(1, h1);
  }
  if (D >= 3) {
    load_row(2, s2);
    load_halo(2, h2);
  }
  for (int k = 0; k < K; k += D + 1) {
    if (D == 1) {
      stage(k, s1, s0, h1, h0);
      stage(k + 1, s0, s1, h0, h1);
    } else if (D == 2) {
      stage(k, s2, s0, h2, h0);
      stage(k + 1, s0, s1, h0, h1);
      stage(k + 2, s1, s2, h1, h2);
    } else {
      stage(k, s3, s0, h3, h0);
      stage(k + 1, s0, s1, h0, h1);
      stage(k + 2, s1, s2, h1, h2);
      stage(k + 3, s2, s3, h2, h3);
    }
  }
}

template <typename T, int SCHEME, int BW, int D>
__global__ void __launch_bounds__(BW)
    march4(Geometry g, Physics phys, Tiling tl, const Global<T>* __restrict__ fin,
           Global<T>* __restrict__ fout) {
  march4_tile<T, SCHEME, BW, D>(g, phys, tl, xcd_tile(blockIdx.x, tl.strips * tl.chunks), fin,
                                fout);
}

// The force-stencil variant's step over a batch table (as march_batch).
template <typename T, int SCHEME, int BW, int D>
__global__ void __launch_bounds__(BW) march4_batch(const BatchTable* __restrict__ tab, int parity) {
  const int total = tab->total_tiles;
  const int item = xcd_tile(blockIdx.x, total);
  if (item >= total) return;
  const BatchSlot* sp = &tab->slot[slot_of_item(tab, item)];
  const Geometry g = sp->g;
  const Physics ph = sp->ph;
  const Tiling tl = sp->tl;
  const int which = sp->cur ^ parity;
  march4_tile<T, SCHEME, BW, D>(g, ph, tl, item - sp->tile0,
                                (const Global<T>*)(const T*)sp->buf[which],
                                (Global<T>*)(T*)sp->buf[which ^ 1]);
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
#pragma unroll
  for (int i = 0; i < Q; ++i) f[(long long)i * g.plane + src_offset(g, i, x, y)] = (T)q[i];
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
  f[(long long)q * g.plane + src_offset(g, q, x, y)] = (T)(dense[(long long)m * n + k] - s);
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
  dense[(long long)m * n + k] = (double)f[(long long)q * g.plane + src_offset(g, q, x, y)] + s;
}

// Window (x0 .. x0+w-1, y0 .. y0+h-1, periodic) of populations q0 .. q0+m-1
// (one per blockIdx.y) as dense double planes [m][h][w], shift added back.
template <typename T>
__global__ void unpack_window_kernel(Geometry g, Shift shift, const T* __restrict__ f, int x0,
                                     int y0, int w, int h, int q0, double* __restrict__ dense) {
  const long long n = (long long)w * h;
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int j = (int)(k / w), i = (int)(k - (long long)j * w);
  const int x = (int)(((long long)x0 + i) % g.nx), y = (int)(((long long)y0 + j) % g.ny);
  const int q = q0 + (int)blockIdx.y;
  dense[(long long)blockIdx.y * n + k] =
      (double)f[(long long)q * g.plane + src_offset(g, q, x, y)] + shift.s[q];
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

template <typename T, int SCHEME, int BW, int D, bool OBS>
hipError_t launch_march_t(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                          void* fout, const ObserveOut& o, hipStream_t s) {
  hipLaunchKernelGGL((march<T, SCHEME, BW, D, OBS>), dim3(t.blocks()), dim3(BW), 0, s, g, ph, t,
                     (const T*)fin, (T*)fout, o);
  return hipGetLastError();
}

template <typename T, int SCHEME, int BW, bool OBS>
hipError_t launch_march_d(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                          void* fout, const ObserveOut& o, hipStream_t s) {
  if (OBS) return launch_march_t<T, SCHEME, BW, 1, OBS>(g, ph, t, fin, fout, o, s);
  switch (t.depth) {
    case 1: return launch_march_t<T, SCHEME, BW, 1, OBS>(g, ph, t, fin, fout, o, s);
    case 2: return launch_march_t<T, SCHEME, BW, 2, OBS>(g, ph, t, fin, fout, o, s);
    case 3: return launch_march_t<T, SCHEME, BW, 3, OBS>(g, ph, t, fin, fout, o, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int SCHEME, bool OBS>
hipError_t launch_march_w(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                          void* fout, const ObserveOut& o, hipStream_t s) {
  switch (t.block) {
    case 64: return launch_march_d<T, SCHEME, 64, OBS>(g, ph, t, fin, fout, o, s);
    case 128: return launch_march_d<T, SCHEME, 128, OBS>(g, ph, t, fin, fout, o, s);
    case 192: return launch_march_d<T, SCHEME, 192, OBS>(g, ph, t, fin, fout, o, s);
    case 256: return launch_march_d<T, SCHEME, 256, OBS>(g, ph, t, fin, fout, o, s);
    case 320: return launch_march_d<T, SCHEME, 320, OBS>(g, ph, t, fin, fout, o, s);
    case 512: return launch_march_d<T, SCHEME, 512, OBS>(g, ph, t, fin, fout, o, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool OBS>
hipError_t launch_march(int storage, int scheme, const Geometry& g, const Physics& ph,
                        const Tiling& t, const void* fin, void* fout, const ObserveOut& o,
                        hipStream_t s) {
  if (t.blocks() <= 0) return hipErrorInvalidValue;
  // the observe pass of STANDARD_EQF is the standard one (same force and u)
  if (OBS && scheme == STANDARD_EQF) scheme = STANDARD;
  if (storage == FP64) {
    if (scheme == STANDARD)
      return launch_march_w<double, STANDARD, OBS>(g, ph, t, fin, fout, o, s);
    if (!OBS && scheme == STANDARD_EQF)
      return launch_march_w<double, STANDARD_EQF, false>(g, ph, t, fin, fout, o, s);
    return launch_march_w<double, WELL_BALANCED, OBS>(g, ph, t, fin, fout, o, s);
  }
  if (scheme == STANDARD) return launch_march_w<float, STANDARD, OBS>(g, ph, t, fin, fout, o, s);
  if (!OBS && scheme == STANDARD_EQF)
    return launch_march_w<float, STANDARD_EQF, false>(g, ph, t, fin, fout, o, s);
  return launch_march_w<float, WELL_BALANCED, OBS>(g, ph, t, fin, fout, o, s);
}

inline unsigned grid1(long long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

bool block_width_supported(int block) {
  return block == 64 || block == 128 || block == 192 || block == 256 || block == 320 ||
         block == 512;
}

namespace {

template <typename T, int SCHEME, int BW, int D, bool OBS>
const void* batch_fn() {
  return (const void*)march_batch<T, SCHEME, BW, D, OBS>;
}

// Kernel of a batched group; null for unsupported combinations.  Batches use
// block widths 64, 128 and 256 and depth 1, 2 or 3 (observe: depth 1).
template <typename T, int SCHEME, bool OBS>
const void* batch_kernel_t(int block, int depth) {
  if (depth == 1) {
    switch (block) {
      case 64: return batch_fn<T, SCHEME, 64, 1, OBS>();
      case 128: return batch_fn<T, SCHEME, 128, 1, OBS>();
      case 256: return batch_fn<T, SCHEME, 256, 1, OBS>();
    }
  } else if (depth == 2 && !OBS) {
    switch (block) {
      case 64: return batch_fn<T, SCHEME, 64, 2, OBS>();
      case 128: return batch_fn<T, SCHEME, 128, 2, OBS>();
      case 256: return batch_fn<T, SCHEME, 256, 2, OBS>();
    }
  } else if (depth == 3 && !OBS) {
    switch (block) {
      case 64: return batch_fn<T, SCHEME, 64, 3, OBS>();
      case 128: return batch_fn<T, SCHEME, 128, 3, OBS>();
      case 256: return batch_fn<T, SCHEME, 256, 3, OBS>();
    }
  }
  return nullptr;
}

template <typename T, int SCHEME>
const void* batch4_kernel_t(int depth) {
  switch (depth) {
    case 1: return (const void*)march4_batch<T, SCHEME, kBatch4Block, 1>;
    case 2: return (const void*)march4_batch<T, SCHEME, kBatch4Block, 2>;
    case 3: return (const void*)march4_batch<T, SCHEME, kBatch4Block, 3>;
  }
  return nullptr;
}

template <typename T>
const void* batch4_kernel_s(int scheme, int depth) {
  if (scheme == STANDARD) return batch4_kernel_t<T, STANDARD>(depth);
  if (scheme == STANDARD_EQF) return batch4_kernel_t<T, STANDARD_EQF>(depth);
  return batch4_kernel_t<T, WELL_BALANCED>(depth);
}

const void* batch_kernel(int storage, int scheme, int block, int depth, bool observe) {
  if (scheme != STANDARD && scheme != WELL_BALANCED && scheme != STANDARD_EQF) return nullptr;
  if (observe) {
    depth = 1;
    if (scheme == STANDARD_EQF) scheme = STANDARD;  // same force, velocity and fields
  }
  if (storage == FP64) {
    if (scheme == STANDARD)
      return observe ? batch_kernel_t<double, STANDARD, true>(block, depth)
                     : batch_kernel_t<double, STANDARD, false>(block, depth);
    if (scheme == STANDARD_EQF) return batch_kernel_t<double, STANDARD_EQF, false>(block, depth);
    return observe ? batch_kernel_t<double, WELL_BALANCED, true>(block, depth)
                   : batch_kernel_t<double, WELL_BALANCED, false>(block, depth);
  }
  if (scheme == STANDARD)
    return observe ? batch_kernel_t<float, STANDARD, true>(block, depth)
                   : batch_kernel_t<float, STANDARD, false>(block, depth);
  if (scheme == STANDARD_EQF) return batch_kernel_t<float, STANDARD_EQF, false>(block, depth);
  return observe ? batch_kernel_t<float, WELL_BALANCED, true>(block, depth)
                 : batch_kernel_t<float, WELL_BALANCED, false>(block, depth);
}

}  // namespace

hipError_t launch_batch4(int storage, int scheme, int depth, const BatchTable* tab, int tiles,
                         int parity, hipStream_t s) {
  if (scheme != STANDARD && scheme != WELL_BALANCED && scheme != STANDARD_EQF) return hipErrorInvalidValue;
  const void* fn = storage == FP64 ? batch4_kernel_s<double>(scheme, depth)
                                   : batch4_kernel_s<float>(scheme, depth);
  if (!fn || tiles <= 0) return hipErrorInvalidValue;
  void* args[] = {(void*)&tab, (void*)&parity};
  return hipLaunchKernel(fn, dim3(tiles), dim3(kBatch4Block), args, 0, s);
}

namespace {
template <typename T, int B>
const void* batch2_kernel_t(int scheme) {
  return scheme == STANDARD        ? (const void*)march2_batch<T, STANDARD, B>
         : scheme == STANDARD_EQF  ? (const void*)march2_batch<T, STANDARD_EQF, B>
         : scheme == WELL_BALANCED ? (const void*)march2_batch<T, WELL_BALANCED, B>
                                   : nullptr;
}
}  // namespace

hipError_t launch_batch2(int storage, int scheme, int block, const BatchTable* tab, int tiles,
                         int parity, hipStream_t s) {
  if (tiles <= 0 || !step2_block_supported(block)) return hipErrorInvalidValue;
  const void* fn = storage == FP64
                       ? (block == 128 ? batch2_kernel_t<double, 128>(scheme)
                                       : batch2_kernel_t<double, 256>(scheme))
                       : (block == 128 ? batch2_kernel_t<float, 128>(scheme)
                                       : batch2_kernel_t<float, 256>(scheme));
  if (!fn) return hipErrorInvalidValue;
  void* args[] = {(void*)&tab, (void*)&parity};
  return hipLaunchKernel(fn, dim3(tiles), dim3(block), args, 0, s);
}

hipError_t launch_batch(int storage, int scheme, int block, int depth, bool observe,
                        const BatchTable* tab, int tiles, int parity, hipStream_t s) {
  const void* fn = batch_kernel(storage, scheme, block, depth, observe);
  if (!fn || tiles <= 0) return hipErrorInvalidValue;
  void* args[] = {(void*)&tab, (void*)&parity};
  const int grid = tiles;
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, s);
}

hipError_t launch_step(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const Tiling& t, const void* fin, void* fout, hipStream_t s) {
  ObserveOut none{nullptr, nullptr, nullptr, nullptr, nullptr};
  return launch_march<false>(storage, scheme, g, ph, t, fin, fout, none, s);
}

namespace {
template <typename T, int BW>
hipError_t launch_step2_t(int scheme, const Geometry& g, const Physics& ph, int rows,
                          const void* fin, void* fout, hipStream_t s) {
  const int sw = BW - 6;
  const int strips = (g.nx + sw - 1) / sw, chunks = (g.ny + rows - 1) / rows;
  if ((long long)strips * chunks > 0x7fffffffLL) return hipErrorInvalidValue;
  const dim3 grid(strips * chunks), block(BW);
  const T* in = (const T*)fin;
  T* out = (T*)fout;
  if (scheme == STANDARD)
    hipLaunchKernelGGL((march2<T, STANDARD, 3, BW>), grid, block, 0, s, g, ph, rows, strips,
                       chunks, in, out);
  else if (scheme == STANDARD_EQF)
    hipLaunchKernelGGL((march2<T, STANDARD_EQF, 3, BW>), grid, block, 0, s, g, ph, rows, strips,
                       chunks, in, out);
  else
    hipLaunchKernelGGL((march2<T, WELL_BALANCED, 3, BW>), grid, block, 0, s, g, ph, rows, strips,
                       chunks, in, out);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_step2(int storage, int scheme, int block, const Geometry& g, const Physics& ph,
                        int rows, const void* fin, void* fout, hipStream_t s) {
  if (rows < 1 || !step2_block_supported(block)) return hipErrorInvalidValue;
  if (storage == FP32)
    return block == 128 ? launch_step2_t<float, 128>(scheme, g, ph, rows, fin, fout, s)
                        : launch_step2_t<float, 256>(scheme, g, ph, rows, fin, fout, s);
  return block == 128 ? launch_step2_t<double, 128>(scheme, g, ph, rows, fin, fout, s)
                      : launch_step2_t<double, 256>(scheme, g, ph, rows, fin, fout, s);
}

hipError_t launch_observe(int storage, int scheme, const Geometry& g, const Physics& ph,
                          const Tiling& t, const void* f, const ObserveOut& o, hipStream_t s) {
  return launch_march<true>(storage, scheme, g, ph, t, f, nullptr, o, s);
}

hipError_t launch_finish_partials(const double* part, int count, double* out, hipStream_t s) {
  hipLaunchKernelGGL(finish_partials_kernel, dim3(1), dim3(64), 0, s, part, count, out);
  return hipGetLastError();
}

int stencil4_blocks(const Geometry& g) {
  return ((g.nx + S4X - 1) / S4X) * ((g.ny + S4Y - 1) / S4Y);
}

namespace {

template <typename T>
hipError_t launch4_observe(int scheme, const Geometry& g, const Physics& ph, const void* f,
                           double* rho, double* mu, const ObserveOut& o, hipStream_t s) {
  const dim3 g1((g.nx + 255) / 256, g.ny);
  const auto* in = (const Global<T>*)(const T*)f;
  hipLaunchKernelGGL(density4<T>, g1, dim3(256), 0, s, g, ph, in, rho);
  hipLaunchKernelGGL(potential4<T>, g1, dim3(256), 0, s, g, ph, (const double*)rho, mu);
  const dim3 g3((g.nx + S4X - 1) / S4X, (g.ny + S4Y - 1) / S4Y);
  if (scheme != WELL_BALANCED)
    hipLaunchKernelGGL((observe4_kernel<T, STANDARD>), g3, dim3(S4X * S4Y), 0, s, g, in,
                       (const double*)rho, (const double*)mu, o);
  else
    hipLaunchKernelGGL((observe4_kernel<T, WELL_BALANCED>), g3, dim3(S4X * S4Y), 0, s, g, in,
                       (const double*)rho, (const double*)mu, o);
  return hipGetLastError();
}

}  // namespace

namespace {

template <typename T, int SCHEME, int BW>
hipError_t launch_march4_d(const Geometry& g, const Physics& ph, const Tiling& t,
                           const Global<T>* in, Global<T>* out, hipStream_t s) {
  const dim3 grid(t.blocks()), block(BW);
  if (t.depth == 1)
    hipLaunchKernelGGL((march4<T, SCHEME, BW, 1>), grid, block, 0, s, g, ph, t, in, out);
  else if (t.depth == 2)
    hipLaunchKernelGGL((march4<T, SCHEME, BW, 2>), grid, block, 0, s, g, ph, t, in, out);
  else if (t.depth == 3)
    hipLaunchKernelGGL((march4<T, SCHEME, BW, 3>), grid, block, 0, s, g, ph, t, in, out);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T, int SCHEME>
hipError_t launch_march4(const Geometry& g, const Physics& ph, const Tiling& t, const void* fin,
                         void* fout, hipStream_t s) {
  const auto* in = (const Global<T>*)(const T*)fin;
  auto* out = (Global<T>*)(T*)fout;
  if (t.block == 256) return launch_march4_d<T, SCHEME, 256>(g, ph, t, in, out, s);
  if (t.block == 512) return launch_march4_d<T, SCHEME, 512>(g, ph, t, in, out, s);
  return hipErrorInvalidValue;
}

}  // namespace

bool stencil4_block_supported(int block) { return block == 256 || block == 512; }

hipError_t launch_step4(int storage, int scheme, const Geometry& g, const Physics& ph,
                        const Tiling& t, const void* fin, void* fout, hipStream_t s) {
  if (storage == FP64) {
    if (scheme == STANDARD) return launch_march4<double, STANDARD>(g, ph, t, fin, fout, s);
    if (scheme == STANDARD_EQF) return launch_march4<double, STANDARD_EQF>(g, ph, t, fin, fout, s);
    return launch_march4<double, WELL_BALANCED>(g, ph, t, fin, fout, s);
  }
  if (scheme == STANDARD) return launch_march4<float, STANDARD>(g, ph, t, fin, fout, s);
  if (scheme == STANDARD_EQF) return launch_march4<float, STANDARD_EQF>(g, ph, t, fin, fout, s);
  return launch_march4<float, WELL_BALANCED>(g, ph, t, fin, fout, s);
}

hipError_t launch_observe4(int storage, int scheme, const Geometry& g, const Physics& ph,
                           const void* f, double* rho, double* mu, const ObserveOut& o,
                           hipStream_t s) {
  return storage == FP64 ? launch4_observe<double>(scheme, g, ph, f, rho, mu, o, s)
                         : launch4_observe<float>(scheme, g, ph, f, rho, mu, o, s);
}

hipError_t launch_init(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const double* rho, const double* ux, const double* uy, void* f,
                       hipStream_t s) {
  const long long n = (long long)g.nx * g.ny;
  if (storage == FP64) {
    if (scheme != WELL_BALANCED)
      hipLaunchKernelGGL((init_kernel<double, STANDARD>), dim3(grid1(n)), dim3(256), 0, s, g, ph,
                         rho, ux, uy, (double*)f);
    else
      hipLaunchKernelGGL((init_kernel<double, WELL_BALANCED>), dim3(grid1(n)), dim3(256), 0, s, g,
                         ph, rho, ux, uy, (double*)f);
  } else {
    if (scheme != WELL_BALANCED)
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

hipError_t launch_unpack_window(int storage, const Geometry& g, const double* shift,
                                const void* f, int x0, int y0, int w, int h, int q0, int m,
                                double* dense, hipStream_t s) {
  const long long n = (long long)w * h;
  if (storage == FP64)
    hipLaunchKernelGGL(unpack_window_kernel<double>, dim3(grid1(n), m), dim3(256), 0, s, g,
                       make_shift(shift), (const double*)f, x0, y0, w, h, q0, dense);
  else
    hipLaunchKernelGGL(unpack_window_kernel<float>, dim3(grid1(n), m), dim3(256), 0, s, g,
                       make_shift(shift), (const float*)f, x0, y0, w, h, q0, dense);
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
