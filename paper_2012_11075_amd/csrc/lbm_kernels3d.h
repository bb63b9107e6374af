// lbm_kernels3d.h -- internal interface between the host library
// (lbm_api.cpp) and the D3Q19 kernels (lbm_kernels3d.hip).  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include "lbm_kernels.h"

namespace lbmk {

// Three-dimensional lattice (D3Q19), populations f[z][y][q][x]: element
// (x, y, z, q) at z*slab + y*pitch + q*plane + x.
constexpr int Q3 = 19;
struct Geometry3 {
  int nx, ny, nz;
  long long plane, pitch, slab;
};

// Constants of the 3-D step (FP64, no storage shift).
struct Physics3 {
  double omega, fpre, beta, kappa, rho_l, rho_v, rho0;
};

// Outputs of the 3-D observe pass (any field may be null).
struct ObserveOut3 {
  double *rho, *ux, *uy, *uz, *mu, *partials;
};

// Three dimensions (D3Q19, FP64): init from dense fields (u may be null),
// pack/unpack m populations from q0 through a dense staging area, one step
// (density into `rho`, chemical potential into `mu`, collide-stream), and
// the observe pass (partials: one per block of blocks3(g)).
hipError_t launch_init3(int scheme, const Geometry3& g, const Physics3& ph, const double* rho,
                        const double* ux, const double* uy, const double* uz, void* f,
                        hipStream_t s);
hipError_t launch_pack3(const Geometry3& g, const double* dense, int q0, int m, void* f,
                        hipStream_t s);
hipError_t launch_unpack3(const Geometry3& g, const void* f, int q0, int m, double* dense,
                          hipStream_t s);
hipError_t launch_step3(int scheme, const Geometry3& g, const Physics3& ph, const void* fin,
                        void* fout, double* rho, double* mu, hipStream_t s);
hipError_t launch_observe3(int scheme, const Geometry3& g, const Physics3& ph, const void* f,
                           double* rho, double* mu, const ObserveOut3& o, hipStream_t s);
int blocks3(const Geometry3& g);

}  // namespace lbmk
