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
// One workgroup per element.  The geometry is recomputed from the map nodes
// once per element, and the reference gradients of u and w of each batch
// member at the quadrature points come from three 1D passes (sum
// factorisation, Section 4.1) through LDS.  Per point the element keeps only
// what the contraction needs: with v = sqrt(W|J|) J^{-1} a for a unit
// direction a, (T_a grad w) . grad u = (v . grad_ref w)(v . grad_ref u), and
// the isotropic part is grad_ref w^T (W|J| J^{-1} J^{-T}) grad_ref u.  When the
// element's arrays do not fit the LDS budget (high p with Gauss points), a
// direct-sum kernel (one point per lane, sums over all nodes) is used instead.
#include "tensor.hpp"

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
  double scale;  // every output is multiplied by it
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
      out[0] = a.scale * gl;
      out[1] = a.scale * gt;
      out[2] = a.scale * gn;
    }
  }
}

// ---------------------------------------------------------------------------
constexpr int SFT = 256;
constexpr size_t SF_LDS_MAX = 64 * 1024;

__host__ __device__ inline size_t sf_lds_doubles(int P, int Pm, int Q) {
  const int PX = P > Pm ? P : Pm;
  const int P3 = P * P * P, Pm3 = Pm * Pm * Pm, Q3 = Q * Q * Q;
  return (size_t)2 * Q * P + 2 * Q * Pm + Q + (P3 > Pm3 ? P3 : Pm3) + 2 * PX * PX * Q +
         3 * PX * Q * Q + 15 * Q3 + SFT / 64;
}

__global__ __launch_bounds__(SFT) void grad_sf_kernel(GradArgs a) {
  extern __shared__ double lds[];
  const int P = a.P, Pm = a.Pm, Q = a.Q;
  const int PX = P > Pm ? P : Pm;
  const int P3 = P * P * P, Pm3 = Pm * Pm * Pm, Q3 = Q * Q * Q;
  double* sB = lds;
  double* sD = sB + Q * P;
  double* sBm = sD + Q * P;
  double* sDm = sBm + Q * Pm;
  double* sw = sDm + Q * Pm;
  double* fld = sw + Q;
  double* t1 = fld + (P3 > Pm3 ? P3 : Pm3);
  double* t2 = t1 + 2 * PX * PX * Q;
  double* geo = t2 + 3 * PX * Q * Q;  // [15][Q3]
  double* sh = geo + 15 * Q3;
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < Q * P; i += SFT) {
    sB[i] = a.tab[a.oB + i];
    sD[i] = a.tab[a.oDb + i];
  }
  for (int i = tid; i < Q * Pm; i += SFT) {
    sBm[i] = a.tab[a.oBm + i];
    sDm[i] = a.tab[a.oDm + i];
  }
  for (int i = tid; i < Q; i += SFT) sw[i] = a.tab[a.ow + i];

  // geometry: J[r][s] in slots 3r + s, fiber in 9..11, sheet in 12..14
  const int32_t* med = a.map_ed + e * Pm3;
  for (int r = 0; r < 3; ++r) {
    __syncthreads();
    for (int i = tid; i < Pm3; i += SFT) fld[i] = a.xyz[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, geo + (3 * r) * Q3, geo + (3 * r + 1) * Q3,
            geo + (3 * r + 2) * Q3, nullptr);
  }
  for (int r = 0; r < 3 && a.fiber; ++r) {
    for (int i = tid; i < Pm3; i += SFT) fld[i] = a.fiber[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, nullptr, nullptr, nullptr, geo + (9 + r) * Q3);
  }
  for (int r = 0; r < 3 && a.sheet; ++r) {
    for (int i = tid; i < Pm3; i += SFT) fld[i] = a.sheet[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, nullptr, nullptr, nullptr, geo + (12 + r) * Q3);
  }
  // per point, in place: slots 0..2 v_f, 3..5 v_s, 6..8 v_n (fiber and sheet);
  // 0..2 v_f and 3..8 H = W|J| J^{-1} J^{-T} (fiber only); 3..8 H (no fiber)
  for (int k = tid; k < Q3; k += SFT) {
    double J[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = geo[(3 * r + c) * Q3 + k];
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
    const int k1 = k % Q, k2 = (k / Q) % Q, k3 = k / (Q * Q);
    const double wj = sw[k1] * sw[k2] * sw[k3] * det;
    const double rw = sqrt(wj);
    // v[s] = sum_r Ji[s][r] a[r]: (J^{-T} grad_ref) . a = grad_ref . v
    auto put_v = [&](const double* dir, int slot) {
      for (int s_ = 0; s_ < 3; ++s_)
        geo[(slot + s_) * Q3 + k] =
            rw * (Ji[s_][0] * dir[0] + Ji[s_][1] * dir[1] + Ji[s_][2] * dir[2]);
    };
    if (a.fiber) {
      double f[3] = {geo[9 * Q3 + k], geo[10 * Q3 + k], geo[11 * Q3 + k]};
      const double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
      for (int r = 0; r < 3; ++r) f[r] /= fl;
      if (a.sheet) {
        double sv[3] = {geo[12 * Q3 + k], geo[13 * Q3 + k], geo[14 * Q3 + k]};
        const double d = sv[0] * f[0] + sv[1] * f[1] + sv[2] * f[2];
        for (int r = 0; r < 3; ++r) sv[r] -= d * f[r];
        const double sl = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
        for (int r = 0; r < 3; ++r) sv[r] /= sl;
        const double nv[3] = {f[1] * sv[2] - f[2] * sv[1], f[2] * sv[0] - f[0] * sv[2],
                              f[0] * sv[1] - f[1] * sv[0]};
        put_v(f, 0);
        put_v(sv, 3);
        put_v(nv, 6);
        continue;
      }
      put_v(f, 0);
    }
    // H[s][t] = W|J| sum_r Ji[s][r] Ji[t][r], symmetric (00 01 02 11 12 22)
    const int is[6] = {0, 0, 0, 1, 1, 2}, it[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; ++m)
      geo[(3 + m) * Q3 + k] = wj * (Ji[is[m]][0] * Ji[it[m]][0] + Ji[is[m]][1] * Ji[it[m]][1] +
                                    Ji[is[m]][2] * Ji[it[m]][2]);
  }
  // per member: reference gradients of u (slots 9..11) and w (12..14)
  for (int bt = 0; bt < a.batch; ++bt) {
    __syncthreads();
    for (int i = tid; i < P3; i += SFT) fld[i] = a.u[(int64_t)bt * a.n_dof + a.ed[e * P3 + i]];
    __syncthreads();
    sf_grad(fld, sB, sD, P, Q, t1, t2, geo + 9 * Q3, geo + 10 * Q3, geo + 11 * Q3, nullptr);
    for (int i = tid; i < P3; i += SFT) fld[i] = a.w[(int64_t)bt * a.n_dof + a.ed[e * P3 + i]];
    __syncthreads();
    sf_grad(fld, sB, sD, P, Q, t1, t2, geo + 12 * Q3, geo + 13 * Q3, geo + 14 * Q3, nullptr);
    double gl = 0, gt = 0, gn = 0;
    for (int k = tid; k < Q3; k += SFT) {
      const double du[3] = {geo[9 * Q3 + k], geo[10 * Q3 + k], geo[11 * Q3 + k]};
      const double dw[3] = {geo[12 * Q3 + k], geo[13 * Q3 + k], geo[14 * Q3 + k]};
      auto dotv = [&](int slot, const double* d) {
        return geo[slot * Q3 + k] * d[0] + geo[(slot + 1) * Q3 + k] * d[1] +
               geo[(slot + 2) * Q3 + k] * d[2];
      };
      if (a.fiber && a.sheet) {
        gl += dotv(0, du) * dotv(0, dw);
        gt += dotv(3, du) * dotv(3, dw);
        gn += dotv(6, du) * dotv(6, dw);
        continue;
      }
      const double h00 = geo[3 * Q3 + k], h01 = geo[4 * Q3 + k], h02 = geo[5 * Q3 + k];
      const double h11 = geo[6 * Q3 + k], h12 = geo[7 * Q3 + k], h22 = geo[8 * Q3 + k];
      const double full = du[0] * (h00 * dw[0] + h01 * dw[1] + h02 * dw[2]) +
                          du[1] * (h01 * dw[0] + h11 * dw[1] + h12 * dw[2]) +
                          du[2] * (h02 * dw[0] + h12 * dw[1] + h22 * dw[2]);
      if (a.fiber) {
        const double fuw = dotv(0, du) * dotv(0, dw);
        gl += fuw;
        gt += full - fuw;
      } else {
        gt += full;
      }
    }
    gl = block_sum(gl, sh);
    gt = block_sum(gt, sh);
    gn = block_sum(gn, sh);
    if (tid == 0) {
      double* out = a.g + ((int64_t)bt * a.n_elem + e) * 3;
      out[0] = a.scale * gl;
      out[1] = a.scale * gt;
      out[2] = a.scale * gn;
    }
  }
}

}  // namespace

void launch_grad_sigma(const mfsem_op& op, const double* u, const double* w, double scale,
                       double* g, hipStream_t s) {
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
  a.scale = scale;
  const size_t lds = sf_lds_doubles(a.P, a.Pm, a.Q) * sizeof(double);
  if (lds <= SF_LDS_MAX) {
    grad_sf_kernel<<<dim3((unsigned)op.d.n_elem), SFT, lds, s>>>(a);
    MFSEM_LAUNCH("grad_sf_kernel");
  } else {
    grad_kernel<<<dim3((unsigned)op.d.n_elem), GT, 0, s>>>(a);
    MFSEM_LAUNCH("grad_kernel");
  }
}

}  // namespace mfsem
