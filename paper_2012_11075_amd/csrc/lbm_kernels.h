// lbm_kernels.h -- internal interface between the host library (lbm_api.cpp)
// and the gfx950 kernels (lbm_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

constexpr int Q = 9;

// Geometry of one lattice's population storage: population q of node (x, y)
// is element q * plane + y * pitch + x (x fastest).  The library lays the
// nine population rows of a lattice row out contiguously (plane = row length
// rounded up to 32 elements, pitch = 9 * plane).
struct Geometry {
  int nx, ny, pitch;  // pitch: elements between lattice rows
  long long plane;    // elements between populations of one node
};

// Physical and storage constants of one lattice, in the step's arithmetic.
struct Physics {
  double omega;      // 1/tau
  double fpre;       // 1 - 1/(2 tau)
  double beta, kappa, rho_l, rho_v;
  double rho_ref;    // storage shift reference (0 for FP64)
  double geq_c[Q];   // feq_i(rho_ref, 0) - s_i: constant part of the shifted equilibrium,
                     // the same for every velocity of a shell
};

// Tiling of the marching step kernel.
struct Tiling {
  int block;   // threads per block (multiple of 64)
  int rows;    // output rows per block
  int strips;  // blocks across x: ceil(nx / block)
  int chunks;  // blocks along y: ceil(ny / rows)
  int depth;   // rows of populations in flight per thread (1..3)
  int blocks() const { return strips * chunks; }
};

// Per-block (per-tile) record of an observe pass, NPART doubles: max|u|,
// mass, kinetic energy E, non-finite flag, momentum x, y, z (z is 0 in 2-D),
// and one unused slot.
constexpr int NPART = 8;

// Node sums of one thread -> the block's NPART-double record at `out`:
// butterfly within each 64-lane wave, then the waves in order (a fixed
// summation order).  Every thread of the block must call it.
struct NodeSums {
  double umax = 0.0, mass = 0.0, ekin = 0.0, bad = 0.0, px = 0.0, py = 0.0, pz = 0.0;
};
template <int NW>
__device__ __forceinline__ void write_block_partials(NodeSums v, double* out) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v.umax = fmax(v.umax, __shfl_xor(v.umax, off));
    v.bad = fmax(v.bad, __shfl_xor(v.bad, off));
    v.mass += __shfl_xor(v.mass, off);
    v.ekin += __shfl_xor(v.ekin, off);
    v.px += __shfl_xor(v.px, off);
    v.py += __shfl_xor(v.py, off);
    v.pz += __shfl_xor(v.pz, off);
  }
  __shared__ double red[NW][NPART];
  const int t = threadIdx.x, wv = t >> 6;
  if ((t & 63) == 0) {
    red[wv][0] = v.umax;
    red[wv][1] = v.mass;
    red[wv][2] = v.ekin;
    red[wv][3] = v.bad;
    red[wv][4] = v.px;
    red[wv][5] = v.py;
    red[wv][6] = v.pz;
  }
  __syncthreads();
  if (t == 0) {
    double r[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int w = 0; w < NW; ++w) {
      r[0] = fmax(r[0], red[w][0]);
      r[3] = fmax(r[3], red[w][3]);
      r[1] += red[w][1];
      r[2] += red[w][2];
      r[4] += red[w][4];
      r[5] += red[w][5];
      r[6] += red[w][6];
    }
#pragma unroll
    for (int k = 0; k < NPART; ++k) out[k] = r[k];
  }
}

// Outputs of an observe pass (all optional).
struct ObserveOut {
  double* rho;
  double* ux;
  double* uy;
  double* mu;
  double* partials;  // NPART doubles per block (see NPART)
};

// STANDARD_EQF: the standard LBE (equilibrium Eq. 3, force Eq. 6) with the
// forcing term F_i = (c_i - u).F feq_i / cs2 rho named after Eq. (5) in
// place of Eq. (5); its observe and init passes are the standard ones.
enum Scheme { STANDARD = 0, WELL_BALANCED = 1, STANDARD_EQF = 2 };

// One lattice of a batched launch (lives in device memory).
struct BatchSlot {
  Geometry g;
  Physics ph;
  Tiling tl;
  void* buf[2];      // the two population copies
  double* partials;  // NPART doubles per tile, for observe launches
  int cur;           // buffer holding the state at parity 0
  int tile0;         // first work item of this slot in the concatenated list
};

// Device-resident table of one batched launch group: slots in order of
// tile0, total_tiles = sum of their tiles.
struct BatchTable {
  int nslots;
  int total_tiles;
  int pad[2];
  BatchSlot slot[1];  // nslots entries (allocated with room for the maximum)
};

inline size_t batch_table_bytes(int max_slots) {
  return sizeof(BatchTable) + (size_t)(max_slots > 1 ? max_slots - 1 : 0) * sizeof(BatchSlot);
}

enum Storage { FP64 = 0, FP32 = 1 };

// One step: populations fin -> fout (ping-pong buffers).
hipError_t launch_step(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const Tiling& t, const void* fin, void* fout, hipStream_t s);

// Two steps in one launch (central stencil): fin -> fout is the state two
// steps on, bit-identical to two launch_step calls.  Blocks of `block`
// threads (step2_block_supported) write strips of block - 6 columns by `rows`
// rows.
constexpr bool step2_block_supported(int block) { return block == 128 || block == 256; }
hipError_t launch_step2(int storage, int scheme, int block, const Geometry& g, const Physics& ph,
                        int rows, const void* fin, void* fout, hipStream_t s);

// Fields and per-block reduction partials of the state f.
hipError_t launch_observe(int storage, int scheme, const Geometry& g, const Physics& ph,
                          const Tiling& t, const void* f, const ObserveOut& o, hipStream_t s);

// Fixed-order finish of `count` per-tile records on the device, into the
// NPART doubles at `out`: the same order and compensated (Neumaier) sums as
// the host finish of lbm_observe, so the results are bit-identical.
hipError_t launch_finish_partials(const double* part, int count, double* out, hipStream_t s);

// f = feq(rho, u) - shift, from dense device fields (ux, uy may be null).
hipError_t launch_init(int storage, int scheme, const Geometry& g, const Physics& ph,
                       const double* rho, const double* ux, const double* uy, void* f,
                       hipStream_t s);

// Dense double planes [m][ny][nx] <-> storage planes q0 .. q0+m-1, removing
// (to storage) or adding back (from storage) the per-plane shift s[9]
// (a host array, or null for no shift).
hipError_t launch_pack(int storage, const Geometry& g, const double* shift, const double* dense,
                       int q0, int m, void* f, hipStream_t s);
hipError_t launch_unpack(int storage, const Geometry& g, const double* shift, const void* f,
                         int q0, int m, double* dense, hipStream_t s);

// The same for the window x0 .. x0+w-1, y0 .. y0+h-1 (periodic, 0 <= x0 < nx,
// 0 <= y0 < ny), as dense planes [m][h][w] of populations q0 .. q0+m-1.
hipError_t launch_unpack_window(int storage, const Geometry& g, const double* shift,
                                const void* f, int x0, int y0, int w, int h, int q0, int m,
                                double* dense, hipStream_t s);

// g_i += delta_i on every node (conversion of the FP32 storage shift).
hipError_t launch_reshift(int storage, const Geometry& g, const double* delta, void* f,
                          hipStream_t s);

// Batched step (or observe) of one launch group: one block per tile of the
// table's `tiles` work items (the group's total_tiles).  Block widths 64, 128
// and 256.
hipError_t launch_batch(int storage, int scheme, int block, int depth, bool observe,
                        const BatchTable* tab, int tiles, int parity, hipStream_t s);

// Two steps per launch of a launch group (central stencil, the kernel of
// launch_step2, block width 128 or 256), each slot's tiling holding
// step2_strips / chunks of its rows; one block per tile, as launch_batch.
inline int step2_strips(int nx, int block) {
  const int w = block - 6;
  return (nx + w - 1) / w;
}
hipError_t launch_batch2(int storage, int scheme, int block, const BatchTable* tab, int tiles,
                         int parity, hipStream_t s);

// Batched step of a launch group of force-stencil slots (block width
// kBatch4Block, depth 1..3): one block per tile, as launch_batch.  The
// variant's observe pass runs per slot (launch_observe4).
constexpr int kBatch4Block = 256;
hipError_t launch_batch4(int storage, int scheme, int depth, const BatchTable* tab, int tiles,
                         int parity, hipStream_t s);

// Force-stencil variant (FP64 or FP32-shifted storage): one step as one fused
// launch on the tiling `t` (block width 256 or 512, depth 1..3), and the
// observe pass of that variant in three launches (density into `rho`,
// chemical potential into `mu`, velocity into o.ux / o.uy; partials: one per
// block of stencil4_blocks(g)).  `rho` and `mu` are dense nx*ny doubles.
bool stencil4_block_supported(int block);
hipError_t launch_step4(int storage, int scheme, const Geometry& g, const Physics& ph,
                        const Tiling& t, const void* fin, void* fout, hipStream_t s);
hipError_t launch_observe4(int storage, int scheme, const Geometry& g, const Physics& ph,
                           const void* f, double* rho, double* mu, const ObserveOut& o,
                           hipStream_t s);
int stencil4_blocks(const Geometry& g);

// Block widths the kernels are instantiated for.
bool block_width_supported(int block);

}  // namespace lbmk
