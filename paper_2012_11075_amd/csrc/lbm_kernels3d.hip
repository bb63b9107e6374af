// lbm_kernels3d.hip -- gfx950 kernels of the three-dimensional form of the
// two-phase LBE step (Eqs. 24 and 26 are stated for general D; here D = 3),
// on the D3Q19 and the D3Q27 lattice (template parameter Q).
//
// Velocities: rest, the 6 axis directions, the 12 edge directions and (D3Q27
// only) the 8 corner directions; weights 1/3, 1/18, 1/36 (D3Q19) or 8/27,
// 2/27, 1/54, 1/216 (D3Q27).  Gradient (1/cs2) sum w_i c_i phi(x+c_i) and
// Laplacian (2/cs2) sum w_i [phi(x+c_i) - phi(x)] with the lattice's
// weights, as in 2-D.  FP64 or FP32-shifted storage.
//
// Step (one HBM pass, `march3`).  A block of 32 x TY threads owns a 32 x TY
// column of nodes and marches along z through a chunk of planes.  Each
// plane's populations are loaded once: a thread pulls the Q populations of
// its own node and keeps them in registers for the two planes until that
// node's update; the 2-node ring of halo nodes around the tile, whose
// populations are needed for rho only, is spread over the waves (one node
// per lane).  rho of a plane goes to a 5-plane LDS ring, mu of the plane
// before to a 3-plane ring, and the node two planes back is collided and
// written.  Odd chunks march towards -z, so adjacent chunks read the planes
// they share at about the same time.  Every stencil sum is grouped
// symmetrically in z, so the direction of the march changes no bit of the
// result.
//
// Observe (three passes, off the stepping path): density, chemical
// potential, and fields and reductions on LDS tiles of rho and mu with a
// 1-node halo, through the same device functions as the step.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_kernels3d.h"

// Multiply-adds are fused only within one source expression (as in the 2-D
// kernels): the single-lattice and batched steps, every tiling and the
// observe pass then round a node the same way by construction.
#pragma clang fp contract(on)

namespace lbmk {
namespace {

// Populations are addressed through global-address-space pointers, so the
// compiler emits global (not flat) loads and stores.
template <typename T>
using Global = __attribute__((address_space(1))) T;

// Velocity c_i: indices 0..18 are D3Q19's, 19..26 the corners D3Q27 adds.
__device__ __forceinline__ void c3(int i, int& cx, int& cy, int& cz) {
  const int X[QMAX3] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1,
                        -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
  const int Y[QMAX3] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0,
                        0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
  const int Z[QMAX3] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1,
                        1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
  cx = X[i];
  cy = Y[i];
  cz = Z[i];
}

// Weight of a shell (0 rest, 1 axis, 2 edge, 3 corner) on the Q-velocity
// lattice, divided in the arithmetic type R.
template <int Q, typename R>
__device__ __forceinline__ R wshell(int shell) {
  if constexpr (Q == 19)
    return shell == 0 ? (R)1 / (R)3 : shell == 1 ? (R)1 / (R)18 : (R)1 / (R)36;
  else
    return shell == 0   ? (R)8 / (R)27
           : shell == 1 ? (R)2 / (R)27
           : shell == 2 ? (R)1 / (R)54
                        : (R)1 / (R)216;
}
__device__ __forceinline__ int shell_of(int i) { return i == 0 ? 0 : i < 7 ? 1 : i < 19 ? 2 : 3; }

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

template <typename R>
__device__ __forceinline__ R mu0_3(R r, const Physics3& p) {
  const R rl = (R)p.rho_l, rv = (R)p.rho_v;
  return (R)2 * (R)p.beta * (r - rl) * (r - rv) * ((R)2 * r - rl - rv);
}

// Equilibrium (Eq. 3 / Eq. 24) and forcing term (Eq. 5 / Eq. 26 with D = 3:
// the last term's coefficient (|c|^2/cs2 - 3)/2 is -3/2, 0, 3/2, 3 for the
// rest, axis, edge and corner directions), then BGK, f*_i = f_i - omega
// (f_i - feq_i) + fpre F_i; emit(i, f*_i) receives each post-collision
// population as soon as it is known.  The velocities come in opposite pairs
// (1,2), (3,4), ..., (Q-2,Q-1); every term of feq_i and F_i is even or odd
// in c_i, so a pair evaluates its even and odd parts once.  A scheduling
// barrier after every G pairs keeps the compiler from computing all Q at
// once (each result then dies at its store instead of holding a register).  FP32 storage holds
// g_i = f_i - s_i: the equilibrium is then taken as feq_i(rho, u) -
// feq_i(rho_ref, 0) from drho = rho - rho_ref, plus the constant
// c_i = feq_i(rho_ref, 0) - s_i (the rho0 terms cancel).
template <int Q, int SCHEME, int G, typename R, typename E>
__device__ __forceinline__ void collide3(const R (&f)[Q], R drho, R rho, R ux, R uy, R uz, R Fx,
                                         R Fy, R Fz, R grx, R gry, R grz, const Physics3& p,
                                         E&& emit) {
  constexpr bool SHIFTED = sizeof(R) == 4;
  const R u15 = (R)1.5 * (ux * ux + uy * uy + uz * uz);
  R Gx = Fx, Gy = Fy, Gz = Fz;
  if (SCHEME == WELL_BALANCED) {
    Gx += grx * ((R)1 / (R)3);
    Gy += gry * ((R)1 / (R)3);
    Gz += grz * ((R)1 / (R)3);
  }
  const R uG3 = (R)3 * (ux * Gx + uy * Gy + uz * Gz);
  const R ugr = ux * grx + uy * gry + uz * grz;
  const R omega = (R)p.omega, fpre = (R)p.fpre, rho0 = (R)p.rho0;
  // even forcing constant of a shell: k u.grad(rho) - 3 u.G (WB: k = 0 on the
  // axes, 3/2 on the edges, 3 at the corners)
  const R ev_axis = -uG3;
  const R ev_edge = SCHEME == WELL_BALANCED ? (R)1.5 * ugr - uG3 : -uG3;
  const R ev_corner = SCHEME == WELL_BALANCED ? (R)3 * ugr - uG3 : -uG3;
  auto pair = [&](int i, R cu, R cF, R cG, R w, R ev) {
    const R ep = (R)4.5 * (cu * cu) - u15;  // even part of poly_i
    const R wr = w * rho;
    R Ev;  // even part of the (shifted) equilibrium
    if (SCHEME == WELL_BALANCED)
      Ev = SHIFTED ? wr * ep + (R)p.c[i] : w * rho0 + wr * ep;
    else
      Ev = SHIFTED ? (w * drho + wr * ep) + (R)p.c[i] : wr + wr * ep;
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
    const R Fp = fpre * (Fe + Fo), Fm = fpre * (Fe - Fo);
    emit(i, f[i] - omega * ((f[i] - Ev) - O) + Fp);
    emit(i + 1, f[i + 1] - omega * ((f[i + 1] - Ev) + O) + Fm);
  };
  int np = 0;
  auto sched = [&]() {
    if (G > 0 && ++np % G == 0) __builtin_amdgcn_sched_barrier(0);
  };
  const R wa = wshell<Q, R>(1), we = wshell<Q, R>(2);
  // rest population (c_0 = 0)
  {
    const R w0 = wshell<Q, R>(0);
    R feq0, F0;
    if (SCHEME == WELL_BALANCED) {
      feq0 = SHIFTED ? (drho - w0 * rho * u15) + (R)p.c[0] : rho - ((R)1 - w0) * rho0 - w0 * rho * u15;
      F0 = -w0 * (uG3 + (R)1.5 * ugr);
    } else {
      feq0 = SHIFTED ? w0 * (drho - rho * u15) + (R)p.c[0] : w0 * rho * ((R)1 - u15);
      F0 = SCHEME == STANDARD ? -w0 * uG3 : -w0 * ((R)1 - u15) * uG3;
    }
    emit(0, f[0] - omega * (f[0] - feq0) + fpre * F0);
  }
  pair(1, ux, Fx, Gx, wa, ev_axis);
  sched();
  pair(3, uy, Fy, Gy, wa, ev_axis);
  sched();
  pair(5, uz, Fz, Gz, wa, ev_axis);
  sched();
  pair(7, ux + uy, Fx + Fy, Gx + Gy, we, ev_edge);
  sched();
  pair(9, ux - uy, Fx - Fy, Gx - Gy, we, ev_edge);
  sched();
  pair(11, ux + uz, Fx + Fz, Gx + Gz, we, ev_edge);
  sched();
  pair(13, ux - uz, Fx - Fz, Gx - Gz, we, ev_edge);
  sched();
  pair(15, uy + uz, Fy + Fz, Gy + Gz, we, ev_edge);
  sched();
  pair(17, uy - uz, Fy - Fz, Gy - Gz, we, ev_edge);
  if constexpr (Q == 27) {
    const R wc = wshell<Q, R>(3);
    sched();
    pair(19, (ux + uy) + uz, (Fx + Fy) + Fz, (Gx + Gy) + Gz, wc, ev_corner);
    sched();
    pair(21, (ux + uy) - uz, (Fx + Fy) - Fz, (Gx + Gy) - Gz, wc, ev_corner);
    sched();
    pair(23, (ux - uy) + uz, (Fx - Fy) + Fz, (Gx - Gy) + Gz, wc, ev_corner);
    sched();
    pair(25, (uy + uz) - ux, (Fy + Fz) - Fx, (Gy + Gz) - Gx, wc, ev_corner);
  }
}

// rho = sum_i f_i in a fixed order (every kernel sums a node the same way).
template <int Q, typename R>
__device__ __forceinline__ R sumq(const R (&f)[Q]) {
  R s = (R)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) s += f[i];
  return s;
}

// Isotropic Laplacian (2/cs2) sum_i w_i [phi(x + c_i) - phi(x)] from
// at(dx, dy, dz) = phi(x + (dx, dy, dz)); the sums pair +z with -z.  D3Q19:
// (2 axis + edge - 24 phi)/6; D3Q27: (16 axis + 4 edge + corner - 152 phi)/36.
template <int Q, typename R, typename A>
__device__ __forceinline__ R lapq(const A& at, R c) {
  const R ax = ((at(1, 0, 0) + at(-1, 0, 0)) + (at(0, 1, 0) + at(0, -1, 0))) +
               (at(0, 0, 1) + at(0, 0, -1));
  const R xy = (at(1, 1, 0) + at(-1, -1, 0)) + (at(1, -1, 0) + at(-1, 1, 0));
  const R xz = (at(1, 0, 1) + at(1, 0, -1)) + (at(-1, 0, -1) + at(-1, 0, 1));
  const R yz = (at(0, 1, 1) + at(0, 1, -1)) + (at(0, -1, -1) + at(0, -1, 1));
  if constexpr (Q == 19) {
    return ((R)2 * ax + ((xy + xz) + yz) - (R)24 * c) * ((R)1 / (R)6);
  } else {
    const R co = ((at(1, 1, 1) + at(1, 1, -1)) + (at(-1, -1, -1) + at(-1, -1, 1))) +
                 ((at(1, -1, 1) + at(1, -1, -1)) + (at(-1, 1, -1) + at(-1, 1, 1)));
    return (((R)16 * ax + (R)4 * ((xy + xz) + yz)) + (co - (R)152 * c)) * ((R)1 / (R)36);
  }
}

// Isotropic central gradient (1/cs2) sum_i w_i c_i phi(x + c_i) at row j,
// column i of the LDS plane a0, with am and ap the planes at z - 1 and z + 1.
// Swapping am and ap negates gz exactly and leaves gx, gy unchanged.
// Coefficients 3 w: D3Q19 axis 1/6, edge 1/12; D3Q27 axis 2/9, edge 1/18,
// corner 1/72.
template <int Q, int W, typename R>
__device__ __forceinline__ void grad3p(const R (*am)[W], const R (*a0)[W], const R (*ap)[W], int j,
                                       int i, R& gx, R& gy, R& gz) {
  const R sa = Q == 19 ? (R)1 / (R)6 : (R)2 / (R)9;
  const R se = Q == 19 ? (R)1 / (R)12 : (R)1 / (R)18;
  gx = (a0[j][i + 1] - a0[j][i - 1]) * sa +
       (((a0[j + 1][i + 1] - a0[j + 1][i - 1]) + (a0[j - 1][i + 1] - a0[j - 1][i - 1])) +
        ((ap[j][i + 1] - ap[j][i - 1]) + (am[j][i + 1] - am[j][i - 1]))) *
           se;
  gy = (a0[j + 1][i] - a0[j - 1][i]) * sa +
       (((a0[j + 1][i + 1] - a0[j - 1][i + 1]) + (a0[j + 1][i - 1] - a0[j - 1][i - 1])) +
        ((ap[j + 1][i] - ap[j - 1][i]) + (am[j + 1][i] - am[j - 1][i]))) *
           se;
  gz = (ap[j][i] - am[j][i]) * sa +
       (((ap[j][i + 1] - am[j][i + 1]) + (ap[j][i - 1] - am[j][i - 1])) +
        ((ap[j + 1][i] - am[j + 1][i]) + (ap[j - 1][i] - am[j - 1][i]))) *
           se;
  if constexpr (Q == 27) {
    const R sc = (R)1 / (R)72;
    gx += (((ap[j + 1][i + 1] - ap[j + 1][i - 1]) + (am[j + 1][i + 1] - am[j + 1][i - 1])) +
           ((ap[j - 1][i + 1] - ap[j - 1][i - 1]) + (am[j - 1][i + 1] - am[j - 1][i - 1]))) *
          sc;
    gy += (((ap[j + 1][i + 1] - ap[j - 1][i + 1]) + (am[j + 1][i + 1] - am[j - 1][i + 1])) +
           ((ap[j + 1][i - 1] - ap[j - 1][i - 1]) + (am[j + 1][i - 1] - am[j - 1][i - 1]))) *
          sc;
    gz += (((ap[j + 1][i + 1] - am[j + 1][i + 1]) + (ap[j + 1][i - 1] - am[j + 1][i - 1])) +
           ((ap[j - 1][i + 1] - am[j - 1][i + 1]) + (ap[j - 1][i - 1] - am[j - 1][i - 1]))) *
          sc;
  }
}

// Force (F = -rho grad mu for WB, Eq. 25; plus grad(rho)/3 for the standard
// scheme, Eq. 6) and the half-force velocity of Eq. (4).
template <int Q, int SCHEME, typename R>
__device__ __forceinline__ void force_velocity3(const R (&f)[Q], R r, R grx, R gry, R grz, R gmx,
                                                R gmy, R gmz, R& Fx, R& Fy, R& Fz, R& ux, R& uy,
                                                R& uz) {
  Fx = -r * gmx;
  Fy = -r * gmy;
  Fz = -r * gmz;
  if (SCHEME != WELL_BALANCED) {
    Fx += grx * ((R)1 / (R)3);
    Fy += gry * ((R)1 / (R)3);
    Fz += grz * ((R)1 / (R)3);
  }
  R jx = (R)0, jy = (R)0, jz = (R)0;
#pragma unroll
  for (int i = 0; i < Q; ++i) {
    int cx, cy, cz;
    c3(i, cx, cy, cz);
    if (cx) jx += cx > 0 ? f[i] : -f[i];
    if (cy) jy += cy > 0 ? f[i] : -f[i];
    if (cz) jz += cz > 0 ? f[i] : -f[i];
  }
  const R inv = (R)1 / r;
  ux = (jx + (R)0.5 * Fx) * inv;
  uy = (jy + (R)0.5 * Fy) * inv;
  uz = (jz + (R)0.5 * Fz) * inv;
}

__device__ __forceinline__ int wrapi(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

// Blocks b, b+8, ... run on one XCD; give each XCD a contiguous range of
// work items, so neighbouring tiles share their halo lines in its L2.
__device__ __forceinline__ int xcd_item(int b, int nb) {
  const int xcd = b & 7, l = b >> 3, q8 = nb >> 3, r8 = nb & 7;
  return xcd * q8 + min(xcd, r8) + l;
}

// Buffer addressing for the fused step.  Each z-plane of populations is
// below 4 GiB (the library checks), so a plane is one buffer resource (in
// scalar registers), a node's position in it a 32-bit per-lane byte offset
// and the population's offset q * plane a scalar offset: no 64-bit per-lane
// address arithmetic, which would otherwise take a large share of the
// registers.
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
constexpr int RSRC_WORD3 = 0x00020000;  // raw 32-bit data, no swizzle (gfx9 family)
constexpr int CPOL_NT = 2;              // non-temporal

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_buffer(const T* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(base), 0, (int)bytes, RSRC_WORD3);
}

// One element at a byte offset of a buffer, and its non-temporal store.
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t b, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(b, voff, soff, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(b, voff, soff, 0));
}

template <typename T>
__device__ __forceinline__ void buf_store_nt(T v, __amdgpu_buffer_rsrc_t b, unsigned voff,
                                             unsigned soff) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b, voff, soff, CPOL_NT);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b, voff, soff, CPOL_NT);
}

// Pull sources of one node (x, y) within a z-plane: byte offset of the node
// (x - c_x, y - c_y), periodic, at index [c_y + 1][c_x + 1].
struct Pull3 {
  unsigned off[3][3];
};

template <typename T>
__device__ __forceinline__ Pull3 pull_of(const Geometry3& g, int x, int y) {
  Pull3 s;
#pragma unroll
  for (int cy = -1; cy <= 1; ++cy) {
    const long long row = (long long)wrapi(y - cy, g.ny) * g.pitch;
#pragma unroll
    for (int cx = -1; cx <= 1; ++cx)
      s.off[cy + 1][cx + 1] = (unsigned)((row + wrapi(x - cx, g.nx)) * (long long)sizeof(T));
  }
  return s;
}

// The Q pulled populations of node s on a plane; b[c_z + 1] is the plane
// z - c_z, pb the bytes between populations.
template <int Q, typename T>
__device__ __forceinline__ void loadq(const __amdgpu_buffer_rsrc_t (&b)[3], unsigned pb,
                                      const Pull3& s, T (&f)[Q]) {
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int cx, cy, cz;
    c3(q, cx, cy, cz);
    f[q] = buf_load<T>(b[cz + 1], s.off[cy + 1][cx + 1], q * pb);
  }
}

// Fused step: one block per (32 x TY column, chunk of tl.zc planes).  D:
// planes of populations loaded ahead of the plane being summed (0 = none).
constexpr int CG = 1;  // velocity pairs per scheduling region of the collision
template <typename T, int SCHEME, int TY, int D, int Q>
__device__ __forceinline__ void march3_tile(const Geometry3& g, const Physics3& p,
                                            const Tiling3& tl, int item,
                                            const T* __restrict__ fin, T* __restrict__ fout) {
  using R = T;
  constexpr int NT = M3X * TY;
  constexpr int RX = M3X + 4, RY = TY + 4;  // rho region: tile and a 2-node halo
  constexpr int MX = M3X + 2, MY = TY + 2;  // mu region: tile and a 1-node halo
  constexpr int NH = RX * RY - NT;          // halo nodes of the rho region
  constexpr int NW = NT / 64, HPW = (NH + NW - 1) / NW;
  static_assert(HPW <= 64, "one halo node per lane");
  // Populations of planes k-1 .. k+D in a register ring, of plane k-2 in LDS
  // (each thread its own column); halo of planes k .. k+D-1.
  constexpr int RP = 2 + D, RH = D > 0 ? D : 1;
  constexpr int U = (RP % RH == 0) ? RP : RP * RH;  // unroll: slots are compile-time
  __shared__ R pk[Q][NT];
  __shared__ R rs[5][RY][RX];  // region (i, j) is lattice (x0 - 2 + i, y0 - 2 + j)
  __shared__ R ms[3][MY][MX];  // region (i, j) is lattice (x0 - 1 + i, y0 - 1 + j)
  const int t = threadIdx.x;
  const int per_plane = tl.tiles_x * tl.tiles_y;
  const int chunk = item / per_plane;
  const int rem = item - chunk * per_plane;
  const int by = rem / tl.tiles_x, bx = rem - by * tl.tiles_x;
  const int x0 = bx * M3X, y0 = by * TY, z0 = chunk * tl.zc;
  const int Z = min(tl.zc, g.nz - z0);
  const int K = Z + 4;  // planes z0-2 .. z0+Z+1
  const bool up = (chunk & 1) != 0;
  // plane index k of the march -> lattice plane
  auto plane_of = [&](int k) { return wrapi(up ? z0 + Z + 1 - k : z0 - 2 + k, g.nz); };

  const int tx = t % M3X, ty = t / M3X;
  const bool own = x0 + tx < g.nx && y0 + ty < g.ny;
  const Pull3 si = pull_of<T>(g, x0 + tx, y0 + ty);
  // Halo node of this lane: wave w takes halo nodes w*HPW .. w*HPW+HPW-1,
  // numbered along the two rows above the tile, the side columns, then the
  // two rows below.
  const int h = (t >> 6) * HPW + (t & 63);
  const bool hl = (t & 63) < HPW && h < NH;
  int hi = 0, hj = 0;
  if (hl) {
    if (h < 2 * RX) {
      hj = h / RX;
      hi = h - hj * RX;
    } else if (h < 2 * RX + 4 * TY) {
      const int e = h - 2 * RX, c = e & 3;
      hj = 2 + (e >> 2);
      hi = c < 2 ? c : RX - 4 + c;
    } else {
      const int e = h - 2 * RX - 4 * TY;
      hj = TY + 2 + e / RX;
      hi = e - (e / RX) * RX;
    }
  }
  const Pull3 sh = pull_of<T>(g, x0 - 2 + hi, y0 - 2 + hj);
  const R rho_ref = (R)p.rho_ref, kappa = (R)p.kappa;

  const unsigned pb = (unsigned)(g.plane * (long long)sizeof(T));
  const unsigned slab_bytes = (unsigned)(g.slab * (long long)sizeof(T));
  const unsigned own_off =
      (unsigned)(((long long)(y0 + ty) * g.pitch + (x0 + tx)) * (long long)sizeof(T));

  // Loads of plane k.
  auto load_plane = [&](int k, R(&Pl)[Q], R(&Hl)[Q]) {
    const int z = plane_of(k);
    __amdgpu_buffer_rsrc_t b[3];
#pragma unroll
    for (int c = -1; c <= 1; ++c)
      b[c + 1] = plane_buffer<T>(fin + (long long)wrapi(z - c, g.nz) * g.slab, slab_bytes);
    loadq<Q, T>(b, pb, si, Pl);
    if (hl) loadq<Q, T>(b, pb, sh, Hl);
  };

  // Plane step k: publish rho of plane k (populations in Pk, halo in Hk),
  // start the loads of plane k+D (into Pn, Hk), mu of plane k-1, update the
  // nodes of plane k-2 (populations parked in LDS), park plane k-1 (Pm).
  auto stage = [&](int k, R(&Pk)[Q], R(&Hk)[Q], R(&Pn)[Q], R(&Pm)[Q]) {
    if (D == 0) load_plane(k, Pk, Hk);
    const int sk = k % 5;
    rs[sk][ty + 2][tx + 2] = rho_ref + sumq<Q>(Pk);
    if (hl) rs[sk][hj][hi] = rho_ref + sumq<Q>(Hk);
    if (D > 0 && k + D < K) load_plane(k + D, Pn, Hk);
    __syncthreads();
    if (k >= 2) {
      const int sm = (k - 2) % 5, s0 = (k - 1) % 5, mk = (k - 1) % 3;
      for (int e = t; e < MX * MY; e += NT) {
        const int mj = e / MX, mi = e - mj * MX;
        const int i = mi + 1, j = mj + 1;
        auto at = [&](int dx, int dy, int dz) {
          return rs[dz < 0 ? sm : (dz > 0 ? sk : s0)][j + dy][i + dx];
        };
        const R r0 = rs[s0][j][i];
        ms[mk][mj][mi] = mu0_3(r0, p) - kappa * lapq<Q>(at, r0);
      }
    }
    __syncthreads();
    if (own) {
      // Gradients first, then plane k-2 out of LDS and plane k-1 in (each
      // thread its own column), then the collision: the scheduling barriers
      // keep the phases apart, so their temporaries are not live at once.
      const int c = k - 2;
      R grx = (R)0, gry = (R)0, grz = (R)0, gmx = (R)0, gmy = (R)0, gmz = (R)0, r = (R)1;
      if (k >= 4) {
        const int sM = (c - 1) % 5, s0 = c % 5, sP = (c + 1) % 5;
        const int mM = (c - 1) % 3, m0 = c % 3, mP = (c + 1) % 3;
        grad3p<Q, RX>(rs[sM], rs[s0], rs[sP], ty + 2, tx + 2, grx, gry, grz);
        grad3p<Q, MX>(ms[mM], ms[m0], ms[mP], ty + 1, tx + 1, gmx, gmy, gmz);
        r = rs[s0][ty + 2][tx + 2];
      }
      __builtin_amdgcn_sched_barrier(0);
      R f[Q];
      if (k >= 4) {
#pragma unroll
        for (int q = 0; q < Q; ++q) f[q] = pk[q][t];
      }
      if (k >= 3) {
#pragma unroll
        for (int q = 0; q < Q; ++q) pk[q][t] = Pm[q];
      }
      __builtin_amdgcn_sched_barrier(0);
      if (k >= 4) {
        if (up) {  // plane k-1 of the march lies at +z
          grz = -grz;
          gmz = -gmz;
        }
        R Fx, Fy, Fz, ux, uy, uz;
        force_velocity3<Q, SCHEME>(f, r, grx, gry, grz, gmx, gmy, gmz, Fx, Fy, Fz, ux, uy, uz);
        const __amdgpu_buffer_rsrc_t o =
            plane_buffer<T>(fout + (long long)plane_of(c) * g.slab, slab_bytes);
        const R drho = sumq<Q>(f);
        collide3<Q, SCHEME, CG>(f, drho, r, ux, uy, uz, Fx, Fy, Fz, grx, gry, grz, p,
                             [&](int q, R v) { buf_store_nt<T>(v, o, own_off, q * pb); });
      }
    }
  };

  R P[RP][Q], H[RH][Q];
#pragma unroll
  for (int k = 0; k < D; ++k) load_plane(k, P[k], H[k % RH]);
  for (int k0 = 0; k0 < K; k0 += U) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < K)
        stage(k0 + u, P[u % RP], H[u % RH], P[(u + D) % RP], P[(u + RP - 1) % RP]);
  }
}

template <typename T, int SCHEME, int TY, int D, int Q>
__global__ void __launch_bounds__(M3X * TY)
    march3(Geometry3 g, Physics3 p, Tiling3 tl, const T* __restrict__ fin, T* __restrict__ fout) {
  march3_tile<T, SCHEME, TY, D, Q>(
      g, p, tl, xcd_item(blockIdx.x, tl.tiles_x * tl.tiles_y * tl.chunks), fin, fout);
}

// Many 3-D lattices in one launch: one block per work item of the table's
// concatenated tile list (as the 2-D batched step), the slot found by a
// search uniform over the block.
template <typename T, int SCHEME, int D, int Q>
__global__ void __launch_bounds__(M3X * kBatch3Ty)
    march3_batch(const BatchTable3* __restrict__ tab, int parity) {
  const int total = tab->total_tiles;
  const int item = xcd_item(blockIdx.x, total);
  if (item >= total) return;
  int lo = 0, hi = tab->nslots - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tab->slot[mid].tile0 <= item)
      lo = mid;
    else
      hi = mid - 1;
  }
  const BatchSlot3* sp = &tab->slot[lo];
  const Geometry3 g = sp->g;
  const Physics3 ph = sp->ph;
  const Tiling3 tl = sp->tl;
  const int which = sp->cur ^ parity;
  march3_tile<T, SCHEME, kBatch3Ty, D, Q>(g, ph, tl, item - sp->tile0, (const T*)sp->buf[which],
                                          (T*)sp->buf[which ^ 1]);
}

// Observe pass, in the storage type's arithmetic as the step (FP32 storage:
// rho = rho_ref + sum_i g_i, then every stencil in FP32); fields as double.
template <typename T, int Q>
__global__ void __launch_bounds__(256)
    density3(Geometry3 g, Physics3 p, const Global<T>* __restrict__ fin, double* __restrict__ rho) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  T f[Q];
#pragma unroll
  for (int i = 0; i < Q; ++i) f[i] = fin[(long long)i * g.plane + src3(g, i, x, y, z)];
  rho[((long long)z * g.ny + y) * g.nx + x] = (double)((T)p.rho_ref + sumq<Q>(f));
}

template <typename T, int Q>
__global__ void __launch_bounds__(256)
    potential3(Geometry3 g, Physics3 p, const double* __restrict__ rho, double* __restrict__ mu) {
  using R = T;
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  auto at = [&](int dx, int dy, int dz) {
    const int a = wrapi(x + dx, g.nx), b = wrapi(y + dy, g.ny), c = wrapi(z + dz, g.nz);
    return (R)rho[((long long)c * g.ny + b) * g.nx + a];
  };
  const R c = at(0, 0, 0);
  mu[((long long)z * g.ny + y) * g.nx + x] = (double)(mu0_3(c, p) - (R)p.kappa * lapq<Q>(at, c));
}

constexpr int T3X = 32, T3Y = 4, T3Z = 2;  // observe block (threads)

// Fields and per-block partials (max|u|, mass, kinetic energy, non-finite
// flag, momentum) of the state f, from dense rho and mu.
template <typename T, int SCHEME, int Q>
__global__ void __launch_bounds__(T3X * T3Y * T3Z)
    observe3_kernel(Geometry3 g, const Global<T>* __restrict__ fin,
                    const double* __restrict__ rho, const double* __restrict__ mu,
                    ObserveOut3 obs) {
  using R = T;
  __shared__ R rt[T3Z + 2][T3Y + 2][T3X + 2];
  __shared__ R mt[T3Z + 2][T3Y + 2][T3X + 2];
  const int tid = threadIdx.x;
  const int tx = tid % T3X, ty = (tid / T3X) % T3Y, tz = tid / (T3X * T3Y);
  const int x0 = blockIdx.x * T3X, y0 = blockIdx.y * T3Y, z0 = blockIdx.z * T3Z;
  constexpr int TILE = (T3Z + 2) * (T3Y + 2) * (T3X + 2);
  for (int e = tid; e < TILE; e += T3X * T3Y * T3Z) {
    const int i = e % (T3X + 2), j = (e / (T3X + 2)) % (T3Y + 2), k = e / ((T3X + 2) * (T3Y + 2));
    const int xx = wrapi(x0 + i - 1, g.nx), yy = wrapi(y0 + j - 1, g.ny),
              zz = wrapi(z0 + k - 1, g.nz);
    const long long o = ((long long)zz * g.ny + yy) * g.nx + xx;
    rt[k][j][i] = (R)rho[o];
    mt[k][j][i] = (R)mu[o];
  }
  __syncthreads();
  const int x = x0 + tx, y = y0 + ty, z = z0 + tz;
  NodeSums acc;
  if (x < g.nx && y < g.ny && z < g.nz) {
    R f[Q];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = fin[(long long)i * g.plane + src3(g, i, x, y, z)];
    const R rr = rt[tz + 1][ty + 1][tx + 1];
    R grx, gry, grz, gmx, gmy, gmz;
    grad3p<Q, T3X + 2>(rt[tz], rt[tz + 1], rt[tz + 2], ty + 1, tx + 1, grx, gry, grz);
    grad3p<Q, T3X + 2>(mt[tz], mt[tz + 1], mt[tz + 2], ty + 1, tx + 1, gmx, gmy, gmz);
    R Fx, Fy, Fz, uxr, uyr, uzr;
    force_velocity3<Q, SCHEME>(f, rr, grx, gry, grz, gmx, gmy, gmz, Fx, Fy, Fz, uxr, uyr, uzr);
    const double r = (double)rr, ux = (double)uxr, uy = (double)uyr, uz = (double)uzr;
    const long long o = ((long long)z * g.ny + y) * g.nx + x;
    if (obs.ux) obs.ux[o] = ux;
    if (obs.uy) obs.uy[o] = uy;
    if (obs.uz) obs.uz[o] = uz;
    const double u2 = ux * ux + uy * uy + uz * uz;
    const double um = sqrt(u2);
    if (!(isfinite(r) && r > 0.0 && isfinite(um))) acc.bad = 1.0;
    acc.umax = um;
    acc.mass = r;
    acc.ekin = 0.5 * r * u2;
    acc.px = r * ux;
    acc.py = r * uy;
    acc.pz = r * uz;
  }
  if (obs.partials) {
    const long long b = ((long long)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    write_block_partials<T3X * T3Y * T3Z / 64>(acc, obs.partials + (long long)NPART * b);
  }
}

// f = feq(rho, u) of every node (in double), stored minus the storage shift
// s_i where the next pull reads it.
template <typename T, int SCHEME, int Q>
__global__ void __launch_bounds__(256)
    init3_kernel(Geometry3 g, Physics3 p, const double* __restrict__ rho,
                 const double* __restrict__ ux, const double* __restrict__ uy,
                 const double* __restrict__ uz, T* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  const long long k = ((long long)z * g.ny + y) * g.nx + x;
  const double r = rho[k];
  const double vx = ux ? ux[k] : 0.0, vy = uy ? uy[k] : 0.0, vz = uz ? uz[k] : 0.0;
  const double u15 = 1.5 * (vx * vx + vy * vy + vz * vz);
  for (int i = 0; i < Q; ++i) {
    int cx, cy, cz;
    c3(i, cx, cy, cz);
    const double w = wshell<Q, double>(shell_of(i));
    const double cu = cx * vx + cy * vy + cz * vz;
    const double poly = 3.0 * cu + 4.5 * cu * cu - u15;
    double q;
    if (SCHEME == STANDARD)
      q = w * r * (1.0 + poly);
    else
      q = i == 0 ? r - (1.0 - w) * p.rho0 - w * r * u15 : w * (p.rho0 + r * poly);
    f[(long long)i * g.plane + src3(g, i, x, y, z)] = (T)(q - p.s[i]);
  }
}

// dense[m][z][y][x] <-> populations q0 .. q0+m-1 (pre-collision f at each
// node), removing (to storage) or adding back (from storage) the shift s_q.
template <typename T, bool PACK>
__global__ void __launch_bounds__(256)
    pack3_kernel(Geometry3 g, Physics3 p, int q0, int m, double* __restrict__ dense,
                 T* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  const long long n = (long long)g.nx * g.ny * g.nz;
  const long long k = ((long long)z * g.ny + y) * g.nx + x;
  for (int j = 0; j < m; ++j) {
    const int q = q0 + j;
    const long long o = (long long)q * g.plane + src3(g, q, x, y, z);
    if (PACK)
      f[o] = (T)(dense[j * n + k] - p.s[q]);
    else
      dense[j * n + k] = (double)f[o] + p.s[q];
  }
}

// g_i += d_i on every node (change of the FP32 storage shift).
template <typename T>
__global__ void __launch_bounds__(256)
    reshift3_kernel(Geometry3 g, Physics3 d, T* __restrict__ f) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= g.nx) return;
  for (int q = 0; q < g.q; ++q) {
    const long long o = (long long)z * g.slab + (long long)y * g.pitch + (long long)q * g.plane + x;
    f[o] = (T)((double)f[o] + d.s[q]);
  }
}

}  // namespace

namespace {

inline dim3 grid_rows3(const Geometry3& g) { return dim3((g.nx + 255) / 256, g.ny, g.nz); }

}  // namespace

int blocks3(const Geometry3& g) {
  return ((g.nx + T3X - 1) / T3X) * ((g.ny + T3Y - 1) / T3Y) * ((g.nz + T3Z - 1) / T3Z);
}

namespace {

template <typename T, int Q>
void launch_init3_t(int scheme, const Geometry3& g, const Physics3& ph, const double* rho,
                    const double* ux, const double* uy, const double* uz, void* f, hipStream_t s) {
  if (scheme == STANDARD)
    hipLaunchKernelGGL((init3_kernel<T, STANDARD, Q>), grid_rows3(g), dim3(256), 0, s, g, ph, rho,
                       ux, uy, uz, (T*)f);
  else
    hipLaunchKernelGGL((init3_kernel<T, WELL_BALANCED, Q>), grid_rows3(g), dim3(256), 0, s, g, ph,
                       rho, ux, uy, uz, (T*)f);
}

}  // namespace

hipError_t launch_init3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                        const double* rho, const double* ux, const double* uy, const double* uz,
                        void* f, hipStream_t s) {
  if (scheme == STANDARD_EQF) scheme = STANDARD;  // same equilibrium
  if (g.q != Q3 && g.q != Q27) return hipErrorInvalidValue;
  if (storage == FP64)
    (g.q == Q3 ? launch_init3_t<double, Q3> : launch_init3_t<double, Q27>)(scheme, g, ph, rho, ux,
                                                                          uy, uz, f, s);
  else
    (g.q == Q3 ? launch_init3_t<float, Q3> : launch_init3_t<float, Q27>)(scheme, g, ph, rho, ux,
                                                                        uy, uz, f, s);
  return hipGetLastError();
}

hipError_t launch_pack3(int storage, const Geometry3& g, const Physics3& ph, const double* dense,
                        int q0, int m, void* f, hipStream_t s) {
  if (storage == FP64)
    hipLaunchKernelGGL((pack3_kernel<double, true>), grid_rows3(g), dim3(256), 0, s, g, ph, q0, m,
                       const_cast<double*>(dense), (double*)f);
  else
    hipLaunchKernelGGL((pack3_kernel<float, true>), grid_rows3(g), dim3(256), 0, s, g, ph, q0, m,
                       const_cast<double*>(dense), (float*)f);
  return hipGetLastError();
}

hipError_t launch_unpack3(int storage, const Geometry3& g, const Physics3& ph, const void* f,
                          int q0, int m, double* dense, hipStream_t s) {
  if (storage == FP64)
    hipLaunchKernelGGL((pack3_kernel<double, false>), grid_rows3(g), dim3(256), 0, s, g, ph, q0, m,
                       dense, const_cast<double*>((const double*)f));
  else
    hipLaunchKernelGGL((pack3_kernel<float, false>), grid_rows3(g), dim3(256), 0, s, g, ph, q0, m,
                       dense, const_cast<float*>((const float*)f));
  return hipGetLastError();
}

hipError_t launch_reshift3(int storage, const Geometry3& g, const Physics3& delta, void* f,
                           hipStream_t s) {
  if (storage == FP64)
    hipLaunchKernelGGL(reshift3_kernel<double>, grid_rows3(g), dim3(256), 0, s, g, delta,
                       (double*)f);
  else
    hipLaunchKernelGGL(reshift3_kernel<float>, grid_rows3(g), dim3(256), 0, s, g, delta,
                       (float*)f);
  return hipGetLastError();
}

Tiling3 make_tiling3(const Geometry3& g, int ty, int zc, int depth, int target) {
  Tiling3 t{};
  t.ty = ty;
  t.depth = depth;
  t.tiles_x = (g.nx + M3X - 1) / M3X;
  t.tiles_y = (g.ny + ty - 1) / ty;
  if (zc <= 0) {
    // about `target` blocks, chunks of at least 16 planes; but a small
    // lattice, whose step lasts about one block's march through its chunk,
    // gets shorter chunks (down to 2 planes) until there are about as many
    // blocks as compute units (32^3 FP64: 20 us per step instead of 75 us)
    const long long per = (long long)t.tiles_x * t.tiles_y;
    long long ch = (target + per - 1) / per;
    ch = std::max(1LL, std::min(ch, (long long)(g.nz + 15) / 16));
    constexpr long long kComputeUnits = 256;
    if (per * ch < kComputeUnits)
      ch = std::max(ch, std::min((kComputeUnits + per - 1) / per, (long long)(g.nz + 1) / 2));
    zc = (int)((g.nz + ch - 1) / ch);
  }
  t.zc = std::min(zc, g.nz);
  t.chunks = (g.nz + t.zc - 1) / t.zc;
  return t;
}

bool tiling3_supported(int q, int ty, int depth) {
  // D3Q27 in FP64 needs the register file and the accumulation registers of
  // a wave at 256 threads per block; 512 would spill to memory
  if (q == Q27) return ty == 8 && depth >= 1 && depth <= 2;
  return q == Q3 &&
         ((ty == 8 && depth >= 1 && depth <= 3) || (ty == 16 && depth >= 1 && depth <= 2));
}

long long blocks_of(const Tiling3& t) { return (long long)t.tiles_x * t.tiles_y * t.chunks; }

namespace {

template <typename T, int SCHEME, int TY, int D, int Q>
void launch_m3(const Geometry3& g, const Physics3& ph, const Tiling3& t, const T* in, T* out,
               long long nb, hipStream_t s) {
  hipLaunchKernelGGL((march3<T, SCHEME, TY, D, Q>), dim3((unsigned)nb), dim3(M3X * TY), 0, s, g,
                     ph, t, in, out);
}

template <typename T, int SCHEME, int Q>
hipError_t launch_march3(const Geometry3& g, const Physics3& ph, const Tiling3& t, const T* in,
                         T* out, hipStream_t s) {
  const long long nb = blocks_of(t);
  if (nb < 1 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  if (!tiling3_supported(Q, t.ty, t.depth)) return hipErrorInvalidValue;
  if (t.ty == 8 && t.depth == 1)
    launch_m3<T, SCHEME, 8, 0, Q>(g, ph, t, in, out, nb, s);
  else if (t.ty == 8 && t.depth == 2)
    launch_m3<T, SCHEME, 8, 1, Q>(g, ph, t, in, out, nb, s);
  else if constexpr (Q == Q3) {
    if (t.ty == 16 && t.depth == 1)
      launch_m3<T, SCHEME, 16, 0, Q>(g, ph, t, in, out, nb, s);
    else if (t.ty == 8 && t.depth == 3)
      launch_m3<T, SCHEME, 8, 2, Q>(g, ph, t, in, out, nb, s);
    else if (t.ty == 16 && t.depth == 2)
      launch_m3<T, SCHEME, 16, 1, Q>(g, ph, t, in, out, nb, s);
    else
      return hipErrorInvalidValue;
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T, int Q>
hipError_t launch_step3_t(int scheme, const Geometry3& g, const Physics3& ph, const Tiling3& t,
                          const void* fin, void* fout, hipStream_t s) {
  const auto* in = (const T*)fin;
  auto* out = (T*)fout;
  if (scheme == STANDARD) return launch_march3<T, STANDARD, Q>(g, ph, t, in, out, s);
  if (scheme == STANDARD_EQF) return launch_march3<T, STANDARD_EQF, Q>(g, ph, t, in, out, s);
  return launch_march3<T, WELL_BALANCED, Q>(g, ph, t, in, out, s);
}

template <typename T, int Q>
hipError_t launch_observe3_t(int scheme, const Geometry3& g, const Physics3& ph, const void* f,
                             double* rho, double* mu, const ObserveOut3& o, hipStream_t s) {
  const auto* in = (const Global<T>*)(const T*)f;
  hipLaunchKernelGGL((density3<T, Q>), grid_rows3(g), dim3(256), 0, s, g, ph, in, rho);
  hipLaunchKernelGGL((potential3<T, Q>), grid_rows3(g), dim3(256), 0, s, g, ph,
                     (const double*)rho, mu);
  const dim3 gc((g.nx + T3X - 1) / T3X, (g.ny + T3Y - 1) / T3Y, (g.nz + T3Z - 1) / T3Z);
  if (scheme != WELL_BALANCED)  // both standard forms: same force and velocity
    hipLaunchKernelGGL((observe3_kernel<T, STANDARD, Q>), gc, dim3(T3X * T3Y * T3Z), 0, s, g, in,
                       (const double*)rho, (const double*)mu, o);
  else
    hipLaunchKernelGGL((observe3_kernel<T, WELL_BALANCED, Q>), gc, dim3(T3X * T3Y * T3Z), 0, s, g,
                       in, (const double*)rho, (const double*)mu, o);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_step3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                        const Tiling3& t, const void* fin, void* fout, hipStream_t s) {
  const long long elem = storage == FP64 ? 8 : 4;
  if (g.slab * elem > 0xffffffffLL) return hipErrorInvalidValue;
  if (g.q == Q3)
    return storage == FP64 ? launch_step3_t<double, Q3>(scheme, g, ph, t, fin, fout, s)
                           : launch_step3_t<float, Q3>(scheme, g, ph, t, fin, fout, s);
  if (g.q == Q27)
    return storage == FP64 ? launch_step3_t<double, Q27>(scheme, g, ph, t, fin, fout, s)
                           : launch_step3_t<float, Q27>(scheme, g, ph, t, fin, fout, s);
  return hipErrorInvalidValue;
}

namespace {

template <typename T, int Q>
const void* batch3_fn(int scheme, int depth) {
  if (depth == 1) {
    if (scheme == STANDARD) return (const void*)march3_batch<T, STANDARD, 0, Q>;
    if (scheme == STANDARD_EQF) return (const void*)march3_batch<T, STANDARD_EQF, 0, Q>;
    return (const void*)march3_batch<T, WELL_BALANCED, 0, Q>;
  }
  if (depth == 2) {
    if (scheme == STANDARD) return (const void*)march3_batch<T, STANDARD, 1, Q>;
    if (scheme == STANDARD_EQF) return (const void*)march3_batch<T, STANDARD_EQF, 1, Q>;
    return (const void*)march3_batch<T, WELL_BALANCED, 1, Q>;
  }
  return nullptr;
}

}  // namespace

hipError_t launch_batch3(int storage, int scheme, int q, int depth, const BatchTable3* tab,
                         int tiles, int parity, hipStream_t s) {
  if (scheme != STANDARD && scheme != WELL_BALANCED && scheme != STANDARD_EQF) return hipErrorInvalidValue;
  const void* fn = nullptr;
  if (q == Q3)
    fn = storage == FP64 ? batch3_fn<double, Q3>(scheme, depth) : batch3_fn<float, Q3>(scheme, depth);
  else if (q == Q27)
    fn = storage == FP64 ? batch3_fn<double, Q27>(scheme, depth) : batch3_fn<float, Q27>(scheme, depth);
  if (!fn || tiles <= 0) return hipErrorInvalidValue;
  void* args[] = {(void*)&tab, (void*)&parity};
  return hipLaunchKernel(fn, dim3(tiles), dim3(M3X * kBatch3Ty), args, 0, s);
}

hipError_t launch_observe3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                           const void* f, double* rho, double* mu, const ObserveOut3& o,
                           hipStream_t s) {
  if (g.q == Q3)
    return storage == FP64 ? launch_observe3_t<double, Q3>(scheme, g, ph, f, rho, mu, o, s)
                           : launch_observe3_t<float, Q3>(scheme, g, ph, f, rho, mu, o, s);
  if (g.q == Q27)
    return storage == FP64 ? launch_observe3_t<double, Q27>(scheme, g, ph, f, rho, mu, o, s)
                           : launch_observe3_t<float, Q27>(scheme, g, ph, f, rho, mu, o, s);
  return hipErrorInvalidValue;
}

}  // namespace lbmk
