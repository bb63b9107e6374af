// lbm_kernels3d.h -- internal interface between the host library
// (lbm_api.cpp) and the D3Q19 / D3Q27 kernels (lbm_kernels3d.hip).  Not
// part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_kernels.h"

namespace lbmk {

// Three-dimensional lattice, D3Q19 (q = 19) or D3Q27 (q = 27), populations
// f[z][y][q][x]: element (x, y, z, q) at z*slab + y*pitch + q*plane + x.
// D3Q27's velocities are D3Q19's followed by the 8 corner directions.
constexpr int Q3 = 19;
constexpr int Q27 = 27;
constexpr int QMAX3 = 27;
struct Geometry3 {
  int nx, ny, nz, q;
  long long plane, pitch, slab;
};

// Constants of the 3-D step.  FP32 storage holds g_i = f_i - s_i: rho_ref
// is the shift's reference density, c_i = feq_i(rho_ref, 0) - s_i of the
// scheme stepped (all zero, with rho_ref, for FP64 storage).
struct Physics3 {
  double omega, fpre, beta, kappa, rho_l, rho_v, rho0;
  double rho_ref;
  double c[QMAX3];  // first q entries used
  double s[QMAX3];
};

// Outputs of the 3-D observe pass (any field may be null).
struct ObserveOut3 {
  double *rho, *ux, *uy, *uz, *mu, *partials;
};

// Tiling of the fused step: blocks of M3X x ty threads, one node each, march
// along z through chunks of zc planes (tiles_x * tiles_y * chunks blocks),
// each thread with `depth` planes of populations in flight (the plane being
// summed and depth - 1 ahead).
constexpr int M3X = 32;
struct Tiling3 {
  int ty, zc, depth;
  int tiles_x, tiles_y, chunks;
};
// ty: 8 (depth 1..3 on D3Q19, 1..2 on D3Q27) or 16 (D3Q19 only, depth 1..2);
// zc <= 0 picks the chunk length for about `target` blocks.
Tiling3 make_tiling3(const Geometry3& g, int ty, int zc, int depth, int target);
bool tiling3_supported(int q, int ty, int depth);
long long blocks_of(const Tiling3& t);

// Three dimensions (g.q = 19 or 27, FP64 or FP32-shifted storage `storage`): init from
// dense fields (u may be null),
// pack/unpack m populations from q0 through a dense staging area, one step
// (one fused pass fin -> fout), and the observe pass (density into `rho`,
// chemical potential into `mu`, fields and partials: one per block of
// blocks3(g)).
hipError_t launch_init3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                        const double* rho, const double* ux, const double* uy, const double* uz,
                        void* f, hipStream_t s);
hipError_t launch_pack3(int storage, const Geometry3& g, const Physics3& ph, const double* dense,
                        int q0, int m, void* f, hipStream_t s);
hipError_t launch_unpack3(int storage, const Geometry3& g, const Physics3& ph, const void* f,
                          int q0, int m, double* dense, hipStream_t s);
// g_i += delta.s[i] on every node (change of the FP32 storage shift).
hipError_t launch_reshift3(int storage, const Geometry3& g, const Physics3& delta, void* f,
                           hipStream_t s);
hipError_t launch_step3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                        const Tiling3& t, const void* fin, void* fout, hipStream_t s);
hipError_t launch_observe3(int storage, int scheme, const Geometry3& g, const Physics3& ph,
                           const void* f, double* rho, double* mu, const ObserveOut3& o,
                           hipStream_t s);
int blocks3(const Geometry3& g);

// One 3-D lattice of a batched launch (device memory), and the table of one
// launch group: slots in order of tile0, total_tiles = sum of their tiles.
struct BatchSlot3 {
  Geometry3 g;
  Physics3 ph;
  Tiling3 tl;
  void* buf[2];  // the two population copies
  int cur;       // buffer holding the state at parity 0
  int tile0;     // first work item of this slot in the concatenated list
};
struct BatchTable3 {
  int nslots;
  int total_tiles;
  int pad[2];
  BatchSlot3 slot[1];  // nslots entries (allocated with room for the maximum)
};
inline size_t batch_table3_bytes(int max_slots) {
  return sizeof(BatchTable3) + (size_t)(max_slots > 1 ? max_slots - 1 : 0) * sizeof(BatchSlot3);
}
// Batched 3-D step of one launch group: tiles of 32 x kBatch3Ty nodes,
// depth 1 or 2, D3Q19 or D3Q27 (q), one block per tile.
constexpr int kBatch3Ty = 8;
hipError_t launch_batch3(int storage, int scheme, int q, int depth, const BatchTable3* tab,
                         int tiles, int parity, hipStream_t s);

}  // namespace lbmk
