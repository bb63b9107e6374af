/*
 * lbm_oracle3d27.c -- TEST INFRASTRUCTURE, not product code.
 *
 * The oracle of the three-dimensional step on the D3Q27 lattice: the source
 * of lbm_oracle3d.c compiled with the 27-velocity set (functions orc27_*).
 * Eq. (24) and Eq. (26) of Z. Guo, arXiv:2012.11075, are written for general
 * dimension; the lattice changes only the velocities and weights, and with
 * them the weighted gradient and Laplacian and the term (|c_i|^2/cs2 - D)/2
 * of Eq. (26): -3/2 at rest, 0 on the axes, 3/2 on the edges and 3 at the
 * corners.
 */
#define ORC3_D3Q27 1
#include "lbm_oracle3d.c"
