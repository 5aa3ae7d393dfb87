// Tensor-product (sum-factorised) evaluation helpers shared by the set-up
// kernels (geometry, gradient contraction): one workgroup per element, every
// thread of the block calls them.
#pragma once

#include "internal.hpp"

namespace mfsem {

// Reference gradient (and value) of a nodal field at the Q^3 points by three
// 1D passes.  in: [P^3] nodal values, local index a + P (b + P c); B, D: [Q][P]
// basis and derivative at the points; t1: [2][P P Q], t2: [3][P Q Q]; outputs
// [Q^3] with point index k1 + Q (k2 + Q k3), each may be null.  Called by every
// thread of the block; ends with a barrier.
__device__ inline void sf_grad(const double* in, const double* B, const double* D, int P, int Q,
                        double* t1, double* t2, double* d0, double* d1, double* d2,
                        double* val) {
  const int P2Q = P * P * Q, PQ2 = P * Q * Q, Q2 = Q * Q, Q3 = Q2 * Q;
  // x: t1[0][c][b][k1] = sum_a B[k1][a] in[c][b][a], t1[1] with D
  for (int l = threadIdx.x; l < P2Q; l += blockDim.x) {
    const int k1 = l % Q, cb = l / Q;
    double sb = 0, sd = 0;
    for (int a = 0; a < P; ++a) {
      const double v = in[cb * P + a];
      sb += B[k1 * P + a] * v;
      sd += D[k1 * P + a] * v;
    }
    t1[l] = sb;
    t1[P2Q + l] = sd;
  }
  __syncthreads();
  // y: t2[0] = B_y t1[0], t2[1] = D_y t1[0], t2[2] = B_y t1[1], as [c][k2][k1]
  for (int l = threadIdx.x; l < PQ2; l += blockDim.x) {
    const int k1 = l % Q, k2 = (l / Q) % Q, c = l / Q2;
    double uu = 0, uy = 0, xd = 0;
    for (int b = 0; b < P; ++b) {
      const double vb = t1[(c * P + b) * Q + k1], vd = t1[P2Q + (c * P + b) * Q + k1];
      uu += B[k2 * P + b] * vb;
      uy += D[k2 * P + b] * vb;
      xd += B[k2 * P + b] * vd;
    }
    t2[l] = uu;
    t2[PQ2 + l] = uy;
    t2[2 * PQ2 + l] = xd;
  }
  __syncthreads();
  // z: d/dxi1 = B_z t2[2], d/dxi2 = B_z t2[1], d/dxi3 = D_z t2[0], value = B_z t2[0]
  for (int l = threadIdx.x; l < Q3; l += blockDim.x) {
    const int k12 = l % Q2, k3 = l / Q2;
    double g0 = 0, g1 = 0, g2 = 0, v = 0;
    for (int c = 0; c < P; ++c) {
      const double bz = B[k3 * P + c], dz = D[k3 * P + c];
      g0 += bz * t2[2 * PQ2 + c * Q2 + k12];
      g1 += bz * t2[PQ2 + c * Q2 + k12];
      g2 += dz * t2[c * Q2 + k12];
      v += bz * t2[c * Q2 + k12];
    }
    if (d0) d0[l] = g0;
    if (d1) d1[l] = g1;
    if (d2) d2[l] = g2;
    if (val) val[l] = v;
  }
  __syncthreads();
}


}  // namespace mfsem
