// Derivative of the operator with respect to each element's conductivities,
// contracted with two vectors: g[b][e][c] = w_b^T (dA/dsigma_{e,c}) u_b.
//
// A is linear in sigma_e = (sigma_l, sigma_t, sigma_n) (Section 2's diffusion
// tensor enters K linearly), so
//   g[e][c] = sum_k W_k |J_k| (T_c grad w)(x_k) . (grad u)(x_k)
// with T_l = f f^T, T_t = s s^T, T_n = n n^T (orthonormal fiber, sheet,
// normal), T_t = I - f f^T without a sheet, T_t = I without a fiber, and
// physical gradients grad = J^{-T} grad_ref.  This is the per-element
// contraction of the adjoint method: dL/dsigma = -lambda^T (dA/dsigma) u.
//
// One workgroup per element; the geometry is recomputed from the map nodes
// (as in the set-up kernel) and the reference gradients of u and w at each
// quadrature point are direct sums over the element's nodes staged in LDS.
// This runs once per gradient, not inside the solver loop.
#include "internal.hpp"

namespace mfsem {

namespace {

constexpr int GT = 256;
constexpr int MP = MFSEM_MAX_P + 1;
constexpr int MQ = MFSEM_MAX_P + 3;

struct GradArgs {
  int64_t n_elem, n_dof;
  int P, Pm, Q, batch;
  const int32_t* ed;
  const int32_t* map_ed;
  const double* xyz;
  const double* fiber;
  const double* sheet;
  const double* tab;
  int oB, oDb, oBm, oDm, ow;
  const double* u;
  const double* w;
  double* g;
};

__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < GT / 64; ++k) s += sh[k];
  return s;
}

__global__ __launch_bounds__(GT) void grad_kernel(GradArgs a) {
  __shared__ double sX[MP * MP * MP * 3];
  __shared__ double sF[MP * MP * MP * 3];
  __shared__ double sS[MP * MP * MP * 3];
  __shared__ double sU[MP * MP * MP], sW[MP * MP * MP];
  __shared__ double sB[MQ * MP], sDb[MQ * MP], sBm[MQ * MP], sDm[MQ * MP], sw[MQ];
  __shared__ double sh[GT / 64];

  const int64_t e = blockIdx.x;
  const int P = a.P, Pm = a.Pm, Q = a.Q;
  const int P3 = P * P * P, Pm3 = Pm * Pm * Pm, Q3 = Q * Q * Q;
  const int tid = threadIdx.x;
  for (int i = tid; i < Pm3; i += GT) {
    const int64_t gidx = a.map_ed[e * Pm3 + i];
    for (int r = 0; r < 3; ++r) {
      sX[i * 3 + r] = a.xyz[gidx * 3 + r];
      if (a.fiber) sF[i * 3 + r] = a.fiber[gidx * 3 + r];
      if (a.sheet) sS[i * 3 + r] = a.sheet[gidx * 3 + r];
    }
  }
  for (int i = tid; i < Q * P; i += GT) {
    sB[i] = a.tab[a.oB + i];
    sDb[i] = a.tab[a.oDb + i];
  }
  for (int i = tid; i < Q * Pm; i += GT) {
    sBm[i] = a.tab[a.oBm + i];
    sDm[i] = a.tab[a.oDm + i];
  }
  for (int i = tid; i < Q; i += GT) sw[i] = a.tab[a.ow + i];

  for (int bt = 0; bt < a.batch; ++bt) {
    __syncthreads();
    for (int i = tid; i < P3; i += GT) {
      const int64_t gidx = a.ed[e * P3 + i];
      sU[i] = a.u[(int64_t)bt * a.n_dof + gidx];
      sW[i] = a.w[(int64_t)bt * a.n_dof + gidx];
    }
    __syncthreads();
    double gl = 0, gt = 0, gn = 0;
    for (int k = tid; k < Q3; k += GT) {
      const int k1 = k % Q, k2 = (k / Q) % Q, k3 = k / (Q * Q);
      // map Jacobian, fiber and sheet at the point
      double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, f[3] = {0, 0, 0}, s[3] = {0, 0, 0};
      for (int c = 0; c < Pm; ++c)
        for (int b = 0; b < Pm; ++b)
          for (int aa = 0; aa < Pm; ++aa) {
            const double bx = sBm[k1 * Pm + aa], by = sBm[k2 * Pm + b], bz = sBm[k3 * Pm + c];
            const double dx = sDm[k1 * Pm + aa], dy = sDm[k2 * Pm + b], dz = sDm[k3 * Pm + c];
            const int i = aa + Pm * (b + Pm * c);
            const double g0 = dx * by * bz, g1 = bx * dy * bz, g2 = bx * by * dz, ph = bx * by * bz;
            for (int r = 0; r < 3; ++r) {
              J[r][0] += sX[i * 3 + r] * g0;
              J[r][1] += sX[i * 3 + r] * g1;
              J[r][2] += sX[i * 3 + r] * g2;
              if (a.fiber) f[r] += sF[i * 3 + r] * ph;
              if (a.sheet) s[r] += sS[i * 3 + r] * ph;
            }
          }
      // reference gradients of u and w
      double du[3] = {0, 0, 0}, dw[3] = {0, 0, 0};
      for (int c = 0; c < P; ++c)
        for (int b = 0; b < P; ++b)
          for (int aa = 0; aa < P; ++aa) {
            const double bx = sB[k1 * P + aa], by = sB[k2 * P + b], bz = sB[k3 * P + c];
            const double dx = sDb[k1 * P + aa], dy = sDb[k2 * P + b], dz = sDb[k3 * P + c];
            const int i = aa + P * (b + P * c);
            const double g0 = dx * by * bz, g1 = bx * dy * bz, g2 = bx * by * dz;
            du[0] += sU[i] * g0; du[1] += sU[i] * g1; du[2] += sU[i] * g2;
            dw[0] += sW[i] * g0; dw[1] += sW[i] * g1; dw[2] += sW[i] * g2;
          }
      const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      const double id = 1.0 / det;
      double Ji[3][3];
      Ji[0][0] = c00 * id;
      Ji[1][0] = c01 * id;
      Ji[2][0] = c02 * id;
      Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
      Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
      Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
      Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
      Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
      Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
      // physical gradients: grad = J^{-T} grad_ref, (grad)_r = sum_s Ji[s][r] ref_s
      double gu[3], gw[3];
      for (int r = 0; r < 3; ++r) {
        gu[r] = Ji[0][r] * du[0] + Ji[1][r] * du[1] + Ji[2][r] * du[2];
        gw[r] = Ji[0][r] * dw[0] + Ji[1][r] * dw[1] + Ji[2][r] * dw[2];
      }
      const double wj = sw[k1] * sw[k2] * sw[k3] * det;
      const double full = gu[0] * gw[0] + gu[1] * gw[1] + gu[2] * gw[2];
      if (!a.fiber) {
        gt += wj * full;
        continue;
      }
      const double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      const double fn[3] = {f[0] / fl, f[1] / fl, f[2] / fl};
      const double fu = fn[0] * gu[0] + fn[1] * gu[1] + fn[2] * gu[2];
      const double fw = fn[0] * gw[0] + fn[1] * gw[1] + fn[2] * gw[2];
      gl += wj * fu * fw;
      if (!a.sheet) {
        gt += wj * (full - fu * fw);
        continue;
      }
      const double d = s[0] * fn[0] + s[1] * fn[1] + s[2] * fn[2];
      double sn[3] = {s[0] - d * fn[0], s[1] - d * fn[1], s[2] - d * fn[2]};
      const double sl = sqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
      for (int r = 0; r < 3; ++r) sn[r] /= sl;
      const double nn[3] = {fn[1] * sn[2] - fn[2] * sn[1], fn[2] * sn[0] - fn[0] * sn[2],
                            fn[0] * sn[1] - fn[1] * sn[0]};
      const double su = sn[0] * gu[0] + sn[1] * gu[1] + sn[2] * gu[2];
      const double sw_ = sn[0] * gw[0] + sn[1] * gw[1] + sn[2] * gw[2];
      const double nu = nn[0] * gu[0] + nn[1] * gu[1] + nn[2] * gu[2];
      const double nw = nn[0] * gw[0] + nn[1] * gw[1] + nn[2] * gw[2];
      gt += wj * su * sw_;
      gn += wj * nu * nw;
    }
    gl = block_sum(gl, sh);
    gt = block_sum(gt, sh);
    gn = block_sum(gn, sh);
    if (tid == 0) {
      double* out = a.g + ((int64_t)bt * a.n_elem + e) * 3;
      out[0] = gl;
      out[1] = gt;
      out[2] = gn;
    }
  }
}

}  // namespace

void launch_grad_sigma(const mfsem_op& op, const double* u, const double* w, double* g,
                       hipStream_t s) {
  if (op.d.n_elem == 0) return;
  GradArgs a;
  a.n_elem = op.d.n_elem;
  a.n_dof = op.d.n_dof;
  a.P = op.P;
  a.Pm = op.Pm;
  a.Q = op.Q;
  a.batch = op.d.batch;
  a.ed = op.d.elem_dof;
  a.map_ed = op.d.map_elem_dof ? op.d.map_elem_dof : op.d.elem_dof;
  a.xyz = op.d.map_xyz;
  a.fiber = op.d.fiber;
  a.sheet = op.d.sheet;
  a.tab = op.tab64;
  a.oB = op.off.B;
  a.oDb = op.off.Db;
  a.oBm = op.off.Bm;
  a.oDm = op.off.Dm;
  a.ow = op.off.w;
  a.u = u;
  a.w = w;
  a.g = g;
  grad_kernel<<<dim3((unsigned)op.d.n_elem), GT, 0, s>>>(a);
  MFSEM_LAUNCH("grad_kernel");
}

}  // namespace mfsem
