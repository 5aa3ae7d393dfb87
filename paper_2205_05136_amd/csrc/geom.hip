// Geometry and coefficient set-up (once per mesh, and per conductivity set).
//
// For every element and quadrature point xi_k (GLL for SEM-NI, Gauss for SEM,
// Section 3) this evaluates the isoparametric map's Jacobian
// J = sum_i X_i (grad phi_i)(xi_k)^T, checks det J > 0, interpolates and
// normalises the fiber (and sheet), forms the diffusion tensor of Section 2 and
// stores
//     G  = W_k |J| J^{-1} sigma J^{-T}   (6 symmetric entries)
//     WJ = W_k |J|
// which is what the operator kernels read ("the Jacobian ... is cached",
// Section 4; the diffusion tensor evaluated at every quadrature point,
// Section 4.2).  FP64 throughout; FP32 copies are rounded from the FP64 values.
//
// One workgroup per element: the element's map nodes, fibers and the 1D
// tables are staged in LDS; the Jacobian and the interpolated fiber come from
// 1D passes (sum factorisation), or, when the element's arrays exceed the LDS
// budget, from direct sums over the map nodes at each point.
#include "tensor.hpp"

namespace mfsem {

namespace {

constexpr int GEOM_THREADS = 256;
constexpr int MAXPM = MFSEM_MAX_P + 1;
constexpr int MAXQ = MFSEM_MAX_P + 3;

struct GeomArgs {
  int64_t n_elem;
  int Pm, Q, batch;
  const int32_t* map_elem_dof;
  const double* xyz;
  const double* fiber;
  const double* sheet;
  const double* tab;      // FP64 tables
  int oBm, oDm, ow;
  const double* sigma;    // [batch][n_elem][3] or null
  double s0, s1, s2;
  double* G64;            // [batch][n_elem][Q^3][6] or null
  double* WJ64;           // [n_elem][Q^3] or null
  float* G32;
  float* WJ32;
  double* idet64;         // [batch][n_elem] 1/det(sigma_e) or null
  float* idet32;
  unsigned long long* bad;
};

// Everything at one quadrature point once J, the interpolated fiber f and
// sheet s are known: det J > 0 check, J^{-1}, W|J|, the unit frame, and G for
// every batch member (FP64 and/or FP32 copies).
__device__ inline void finish_point(const GeomArgs& a, int64_t e, int k, int Q, int Q3,
                                    const double* sW, const double (&J)[3][3],
                                    const double (&f)[3], const double (&s)[3]) {
  const int k1 = k % Q, k2 = (k / Q) % Q, k3 = k / (Q * Q);
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  if (!(det > 0.0)) {
    atomicMin(a.bad, (unsigned long long)(e * Q3 + k));
    return;
  }
  const double id = 1.0 / det;
  // Jinv = adj(J) / det, adj(J)[r][s] = cofactor(J)[s][r]
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

  const double wj = sW[k1] * sW[k2] * sW[k3] * det;
  if (a.WJ64) a.WJ64[e * Q3 + k] = wj;
  if (a.WJ32) a.WJ32[e * Q3 + k] = (float)wj;

  // unit fiber / orthonormal sheet / normal
  double fn[3] = {0, 0, 0}, sn[3] = {0, 0, 0}, nn[3] = {0, 0, 0};
  if (a.fiber) {
    const double fl = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int r = 0; r < 3; ++r) fn[r] = f[r] / fl;
    if (a.sheet) {
      const double d = s[0] * fn[0] + s[1] * fn[1] + s[2] * fn[2];
      for (int r = 0; r < 3; ++r) sn[r] = s[r] - d * fn[r];
      const double sl = sqrt(sn[0] * sn[0] + sn[1] * sn[1] + sn[2] * sn[2]);
      for (int r = 0; r < 3; ++r) sn[r] /= sl;
      nn[0] = fn[1] * sn[2] - fn[2] * sn[1];
      nn[1] = fn[2] * sn[0] - fn[0] * sn[2];
      nn[2] = fn[0] * sn[1] - fn[1] * sn[0];
    }
  }
  for (int bt = 0; bt < a.batch; ++bt) {
    double sl = a.s0, st = a.s1, sv = a.s2;
    if (a.sigma) {
      const double* sp = a.sigma + ((int64_t)bt * a.n_elem + e) * 3;
      sl = sp[0]; st = sp[1]; sv = sp[2];
    }
    double S[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double v;
        if (!a.fiber) v = (r == c) ? st : 0.0;
        else if (!a.sheet) v = ((r == c) ? st : 0.0) + (sl - st) * fn[r] * fn[c];
        else v = sl * fn[r] * fn[c] + st * sn[r] * sn[c] + sv * nn[r] * nn[c];
        S[r][c] = v;
      }
    // T = Jinv * S ; G = T * Jinv^T
    double T[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c)
        T[r][c] = Ji[r][0] * S[0][c] + Ji[r][1] * S[1][c] + Ji[r][2] * S[2][c];
    double Gv[6];
    const int ir[6] = {0, 0, 0, 1, 1, 2}, is[6] = {0, 1, 2, 1, 2, 2};
    for (int m = 0; m < 6; ++m) {
      const int r = ir[m], c = is[m];
      Gv[m] = wj * (T[r][0] * Ji[c][0] + T[r][1] * Ji[c][1] + T[r][2] * Ji[c][2]);
    }
    const int64_t base = (((int64_t)bt * a.n_elem + e) * Q3 + k) * 6;
    for (int m = 0; m < 6; ++m) {
      if (a.G64) a.G64[base + m] = Gv[m];
      if (a.G32) a.G32[base + m] = (float)Gv[m];
    }
  }
}

// 1/det(sigma_e) per batch member (the eigenvalues of the tensor are (sigma_l,
// sigma_t, sigma_n) with a sheet, (sigma_l, sigma_t, sigma_t) with a fiber only,
// sigma_t (x3) without), counting the members whose det(sigma_e) <= 0.
__device__ inline void sigma_dets(const GeomArgs& a, int64_t e) {
  const int tid = threadIdx.x;
  for (int bt = tid; bt < a.batch; bt += blockDim.x) {
    double sl = a.s0, st = a.s1, sv = a.s2;
    if (a.sigma) {
      const double* sp = a.sigma + ((int64_t)bt * a.n_elem + e) * 3;
      sl = sp[0]; st = sp[1]; sv = sp[2];
    }
    const double dsig = !a.fiber ? st * st * st : (!a.sheet ? sl * st * st : sl * st * sv);
    if (!(dsig > 0.0) || !isfinite(1.0 / dsig)) atomicAdd(a.bad + 1, 1ull);
    if (a.idet64) a.idet64[(int64_t)bt * a.n_elem + e] = 1.0 / dsig;
    if (a.idet32) a.idet32[(int64_t)bt * a.n_elem + e] = (float)(1.0 / dsig);
  }
}

__global__ __launch_bounds__(GEOM_THREADS) void geom_kernel(GeomArgs a) {
  __shared__ double sX[MAXPM * MAXPM * MAXPM * 3];
  __shared__ double sF[MAXPM * MAXPM * MAXPM * 3];
  __shared__ double sS[MAXPM * MAXPM * MAXPM * 3];
  __shared__ double sBm[MAXQ * MAXPM], sDm[MAXQ * MAXPM], sW[MAXQ];

  const int64_t e = blockIdx.x;
  const int Pm = a.Pm, Q = a.Q;
  const int Pm3 = Pm * Pm * Pm, Q3 = Q * Q * Q;
  const int tid = threadIdx.x;

  for (int i = tid; i < Pm3; i += blockDim.x) {
    const int64_t g = a.map_elem_dof[e * Pm3 + i];
    for (int r = 0; r < 3; ++r) {
      sX[i * 3 + r] = a.xyz[g * 3 + r];
      if (a.fiber) sF[i * 3 + r] = a.fiber[g * 3 + r];
      if (a.sheet) sS[i * 3 + r] = a.sheet[g * 3 + r];
    }
  }
  for (int i = tid; i < Q * Pm; i += blockDim.x) {
    sBm[i] = a.tab[a.oBm + i];
    sDm[i] = a.tab[a.oDm + i];
  }
  for (int i = tid; i < Q; i += blockDim.x) sW[i] = a.tab[a.ow + i];
  sigma_dets(a, e);
  __syncthreads();

  for (int k = tid; k < Q3; k += blockDim.x) {
    const int k1 = k % Q, k2 = (k / Q) % Q, k3 = k / (Q * Q);
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    double f[3] = {0, 0, 0}, s[3] = {0, 0, 0};
    for (int c = 0; c < Pm; ++c) {
      const double bz = sBm[k3 * Pm + c], dz = sDm[k3 * Pm + c];
      for (int b = 0; b < Pm; ++b) {
        const double by = sBm[k2 * Pm + b], dy = sDm[k2 * Pm + b];
        for (int aa = 0; aa < Pm; ++aa) {
          const double bx = sBm[k1 * Pm + aa], dx = sDm[k1 * Pm + aa];
          const int i = aa + Pm * (b + Pm * c);
          const double g0 = dx * by * bz, g1 = bx * dy * bz, g2 = bx * by * dz;
          const double phi = bx * by * bz;
          for (int r = 0; r < 3; ++r) {
            const double X = sX[i * 3 + r];
            J[r][0] += X * g0;
            J[r][1] += X * g1;
            J[r][2] += X * g2;
            if (a.fiber) f[r] += sF[i * 3 + r] * phi;
            if (a.sheet) s[r] += sS[i * 3 + r] * phi;
          }
        }
      }
    }
    finish_point(a, e, k, Q, Q3, sW, J, f, s);
  }
}

// Sum-factorised variant: the Jacobian's nine entries and the fiber and sheet
// values at all points come from three 1D passes per nodal field (Section 4.1)
// instead of a sum over all map nodes per point; used while the element's
// arrays fit the LDS budget.
constexpr size_t GEOM_SF_LDS_MAX = 64 * 1024;

__host__ __device__ inline size_t geom_sf_doubles(int Pm, int Q) {
  return (size_t)2 * Q * Pm + Q + Pm * Pm * Pm + 2 * Pm * Pm * Q + 3 * Pm * Q * Q + 15 * Q * Q * Q;
}

__global__ __launch_bounds__(GEOM_THREADS) void geom_sf_kernel(GeomArgs a) {
  extern __shared__ double lds[];
  const int Pm = a.Pm, Q = a.Q;
  const int Pm3 = Pm * Pm * Pm, Q3 = Q * Q * Q;
  double* sBm = lds;
  double* sDm = sBm + Q * Pm;
  double* sW = sDm + Q * Pm;
  double* fld = sW + Q;
  double* t1 = fld + Pm3;
  double* t2 = t1 + 2 * Pm * Pm * Q;
  double* geo = t2 + 3 * Pm * Q * Q;  // [15][Q3]: J[r][c] at 3r + c, fiber 9..11, sheet 12..14
  const int64_t e = blockIdx.x;
  const int tid = threadIdx.x;
  for (int i = tid; i < Q * Pm; i += blockDim.x) {
    sBm[i] = a.tab[a.oBm + i];
    sDm[i] = a.tab[a.oDm + i];
  }
  for (int i = tid; i < Q; i += blockDim.x) sW[i] = a.tab[a.ow + i];
  sigma_dets(a, e);
  const int32_t* med = a.map_elem_dof + e * Pm3;
  for (int r = 0; r < 3; ++r) {
    __syncthreads();
    for (int i = tid; i < Pm3; i += blockDim.x) fld[i] = a.xyz[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, geo + (3 * r) * Q3, geo + (3 * r + 1) * Q3,
            geo + (3 * r + 2) * Q3, nullptr);
  }
  for (int r = 0; r < 3 && a.fiber; ++r) {
    for (int i = tid; i < Pm3; i += blockDim.x) fld[i] = a.fiber[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, nullptr, nullptr, nullptr, geo + (9 + r) * Q3);
  }
  for (int r = 0; r < 3 && a.sheet; ++r) {
    for (int i = tid; i < Pm3; i += blockDim.x) fld[i] = a.sheet[(int64_t)med[i] * 3 + r];
    __syncthreads();
    sf_grad(fld, sBm, sDm, Pm, Q, t1, t2, nullptr, nullptr, nullptr, geo + (12 + r) * Q3);
  }
  for (int k = tid; k < Q3; k += blockDim.x) {
    double J[3][3], f[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = geo[(3 * r + c) * Q3 + k];
    for (int r = 0; r < 3; ++r) {
      if (a.fiber) f[r] = geo[(9 + r) * Q3 + k];
      if (a.sheet) sv[r] = geo[(12 + r) * Q3 + k];
    }
    finish_point(a, e, k, Q, Q3, sW, J, f, sv);
  }
}

}  // namespace

void run_geometry(mfsem_op& op, hipStream_t s) {
  GeomArgs a;
  a.n_elem = op.d.n_elem;
  a.Pm = op.Pm;
  a.Q = op.Q;
  a.batch = op.d.batch;
  a.map_elem_dof = op.d.map_elem_dof ? op.d.map_elem_dof : op.d.elem_dof;
  a.xyz = op.d.map_xyz;
  a.fiber = op.d.fiber;
  a.sheet = op.d.sheet;
  a.tab = op.tab64;
  a.oBm = op.off.Bm;
  a.oDm = op.off.Dm;
  a.ow = op.off.w;
  a.sigma = op.sigma_copy;
  a.s0 = op.d.sigma_const[0];
  a.s1 = op.d.sigma_const[1];
  a.s2 = op.d.sigma_const[2];
  a.G64 = op.G64;
  a.WJ64 = op.WJ64;
  a.G32 = op.G32;
  a.WJ32 = op.WJ32;
  a.idet64 = op.idet64;
  a.idet32 = op.idet32;
  a.bad = op.bad;
  vfill<unsigned long long>(op.bad, 1, ~0ull, s);
  vfill<unsigned long long>(op.bad + 1, 2, 0ull, s);
  if (op.d.n_elem == 0) return;
  // one workgroup per element; the grid's x dimension holds up to 2^31-1
  const size_t lds = geom_sf_doubles(a.Pm, a.Q) * sizeof(double);
  if (lds <= GEOM_SF_LDS_MAX) {
    geom_sf_kernel<<<dim3((unsigned)op.d.n_elem), dim3(GEOM_THREADS), lds, s>>>(a);
    MFSEM_LAUNCH("geom_sf_kernel");
  } else {
    geom_kernel<<<dim3((unsigned)op.d.n_elem), dim3(GEOM_THREADS), 0, s>>>(a);
    MFSEM_LAUNCH("geom_kernel");
  }
}

}  // namespace mfsem
