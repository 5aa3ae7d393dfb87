// Matrix-free application of A = alpha*M + K(sigma) (Section 4: the local
// action of the operator recomputed cell by cell at each CG iteration, Alg. 1;
// Section 4.1: sum factorisation of the tensor-product basis).
//
// Per element, with the element's DOFs u gathered from the global vector:
//   reference gradient at each quadrature point by 1D contractions along the
//   three axes, flux = G * grad (G = W|J| J^{-1} sigma J^{-T}, precomputed),
//   mass term alpha * W|J| * u, then the transposed 1D contractions, and a
//   scatter-add of the element result into the global vector.
//
// SEM-NI (GLL, quadrature points = nodes): the interpolation is the identity
// and only the 1D derivative matrix D [P][P] is applied; the mass is diagonal.
// SEM (Gauss, Q points): values are first interpolated to the Gauss points with
// B [Q][P] (3 passes), differentiated there with the collocation matrix Dq
// [Q][Q] (3 passes), and the transposes are applied on the way back.
//
// Thread mapping: one lane per (i, j) pencil of the element's face tile, the
// third axis walked in registers; the first two axes go through LDS.  Several
// elements share a workgroup so the lanes of a wave64 stay busy.  The global
// sum is a hardware FP64/FP32 atomic add; y must be zero (or hold what is to be
// added to) beforehand.
#include "internal.hpp"
#include "rules.hpp"

namespace mfsem {

namespace {

constexpr int NT = 256;  // target lanes per workgroup

constexpr int round64(int n) { return ((n + 63) / 64) * 64; }

// ------------------------------------------------------------ SEM-NI ------
template <int P>
struct NiCfg {
  static constexpr int P2 = P * P, P3 = P2 * P;
  static constexpr int NE = (NT / P2) > 0 ? NT / P2 : 1;
  static constexpr int THREADS = round64(NE * P2);
};

template <typename T, int P, bool STIFF>
__global__ __launch_bounds__(NiCfg<P>::THREADS) void ax_ni_kernel(
    int64_t n_elem, int64_t n_dof, const int32_t* __restrict__ ed, const T* __restrict__ G,
    const T* __restrict__ WJ, const T* __restrict__ idet, T alpha, const T* __restrict__ Dtab,
    const T* __restrict__ wtab, const T* __restrict__ x, T* __restrict__ y) {
  using C = NiCfg<P>;
  constexpr int P2 = C::P2, P3 = C::P3, NE = C::NE;
  __shared__ T sD[P * P];
  __shared__ T sU[STIFF ? NE * P3 : 1];
  __shared__ T sV[STIFF ? NE * P3 : 1];

  const int tid = threadIdx.x;
  const int le = tid / P2, ab = tid % P2;
  const int ia = ab % P, ib = ab / P;
  const int64_t e = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NE + le;
  const bool active = (le < NE) && (e < n_elem);
  const int bt = blockIdx.y;
  x += (int64_t)bt * n_dof;
  y += (int64_t)bt * n_dof;

  if (STIFF)
    for (int i = tid; i < P * P; i += blockDim.x) sD[i] = Dtab[i];

  T u[P];
  int gi[P];
  if (!STIFF) {
    if (active) {
#pragma unroll
      for (int c = 0; c < P; ++c) gi[c] = ed[e * P3 + c * P2 + ab];
#pragma unroll
      for (int c = 0; c < P; ++c) atomic_add(&y[gi[c]], alpha * WJ[e * P3 + c * P2 + ab] * x[gi[c]]);
    }
    return;
  }
  // G (6 values per point, the dominant HBM stream) is loaded after the
  // derivative phase: loading it up front raises the register count and lowers
  // occupancy more than the overlap gains at moderate p.
  T g[P][6];
  if (active) {
#pragma unroll
    for (int c = 0; c < P; ++c) gi[c] = ed[e * P3 + c * P2 + ab];
#pragma unroll
    for (int c = 0; c < P; ++c) u[c] = x[gi[c]];
  }
  T* su = sU + le * P3;
  T* sv = sV + le * P3;
  if (active) {
#pragma unroll
    for (int c = 0; c < P; ++c) su[c * P2 + ab] = u[c];
  }
  __syncthreads();

  T ur[P], us[P], ut[P];
  if (active) {
    // this lane's rows of the 1D derivative matrix in registers; the
    // lane-uniform entries of the third direction are compile-time constants
    T dx[P], dy[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      dx[m] = sD[ia * P + m];
      dy[m] = sD[ib * P + m];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T r = 0, s = 0, t = 0;
#pragma unroll
      for (int m = 0; m < P; ++m) {
        r += dx[m] * su[c * P2 + ib * P + m];
        s += dy[m] * su[c * P2 + m * P + ia];
        t += T(rules::GllTables<P>::D.v[c * P + m]) * u[m];
      }
      ur[c] = r;
      us[c] = s;
      ut[c] = t;
    }
  }
  __syncthreads();

  T ft[P], out[P];
  if (active) {
    // mass weight W|J| = det(G) / (W^2 det(sigma)) when available, else stored
    const T* Ge = G + (((int64_t)bt * n_elem + e) * P3 + ab) * 6;
#pragma unroll
    for (int c = 0; c < P; ++c) load_g6(Ge + c * P2 * 6, g[c]);
    const T id = idet ? idet[(int64_t)bt * n_elem + e] : T(0);
    // 1/W^2 from the table entries 1/w^2 that follow the weights
    const T iw2ab = idet ? wtab[P + ia] * wtab[P + ib] : T(0);
#pragma unroll
    for (int c = 0; c < P; ++c) {
      const int q = c * P2 + ab;
      const T g00 = g[c][0], g01 = g[c][1], g02 = g[c][2];
      const T g11 = g[c][3], g12 = g[c][4], g22 = g[c][5];
      su[q] = g00 * ur[c] + g01 * us[c] + g02 * ut[c];
      sv[q] = g01 * ur[c] + g11 * us[c] + g12 * ut[c];
      ft[c] = g02 * ur[c] + g12 * us[c] + g22 * ut[c];
      T wj;
      if (idet) {
        const T dG = g00 * (g11 * g22 - g12 * g12) - g01 * (g01 * g22 - g12 * g02) +
                     g02 * (g01 * g12 - g11 * g02);
        wj = dG * (id * iw2ab) * wtab[P + c];
      } else {
        wj = WJ[e * P3 + q];
      }
      out[c] = alpha * wj * u[c];
    }
  }
  __syncthreads();

  if (active) {
    T dxt[P], dyt[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      dxt[m] = sD[m * P + ia];
      dyt[m] = sD[m * P + ib];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T v = out[c];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        v += dxt[m] * su[c * P2 + ib * P + m];
        v += dyt[m] * sv[c * P2 + m * P + ia];
        v += T(rules::GllTables<P>::D.v[m * P + c]) * ft[m];
      }
      atomic_add(&y[gi[c]], v);
    }
  }
}

// --------------------------------------------------------------- SEM -------
template <int P, int Q>
struct SemCfg {
  static constexpr int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  static constexpr int NE = (NT / Q2) > 0 ? NT / Q2 : 1;
  static constexpr int THREADS = round64(NE * Q2);
  static constexpr int L1 = (P3 > P * Q2) ? P3 : P * Q2;   // node values / [c][k2][k1]
  static constexpr int L2 = (P2 * Q > Q3) ? P2 * Q : Q3;   // [c][b][k1] / flux y
  static constexpr int L3 = Q3;                            // quad values / flux x
};

// Waves per SIMD the register budget must allow: 3 for the FP64 kernels from
// P = 6 with up to 9 Gauss points (at P = 8, Q = 9: 168 VGPRs and no spill,
// against 178 VGPRs and 2 waves unconstrained; the LDS of three 3-element
// workgroups fits a CU).
template <typename T, int P, int Q>
constexpr int sem_min_waves() { return (sizeof(T) == 8 && P >= 6 && Q <= 9) ? 3 : 1; }

// Structured lattices: the workgroup's NE elements are a brick along x, whose
// node lattice ((NE p + 1) x P x P nodes) is gathered once with coalesced rows
// (node numbers computed, no element-to-node index); each element's results go
// to its own node buffer and every lattice node sums its one or two
// contributions (two on an element boundary along x) before one global atomic
// per lattice node (the element form adds every element node with its own
// atomic).  Chosen per precision and degree by measurement on the 51M-DOF slab
// (q = p + 2): FP64 p = 2..6 4.64 / 2.98 / 2.19 / 1.85 / 1.73 -> 4.27 / 2.80 /
// 2.07 / 1.79 / 1.68 ms, but p = 7 1.72 -> 1.76 ms; FP32 p = 2..7 3.60 / 1.78 /
// 1.46 / 1.17 / 1.01 / 0.98 -> 2.11 / 1.42 / 1.11 / 0.96 / 0.91 / 0.96 ms.  Summing
// the lattice with LDS atomics instead measured the same in FP64 and up to 16%
// slower than the element form in FP32 (p = 7), whose LDS is the busier.
template <typename T, int P, int Q>
constexpr bool sem_lattice() { return sizeof(T) == 8 ? P <= 7 : true; }

template <typename T, int P, int Q, bool STIFF, bool LAT = false>
__global__ __launch_bounds__((SemCfg<P, Q>::THREADS), (sem_min_waves<T, P, Q>())) void ax_sem_kernel(
    int64_t n_elem, int64_t n_dof, const int32_t* __restrict__ ed, const T* __restrict__ G,
    const T* __restrict__ WJ, const T* __restrict__ idet, T alpha, const T* __restrict__ Btab,
    const T* __restrict__ Dqtab, const T* __restrict__ wtab, const T* __restrict__ x,
    T* __restrict__ y, int lnx, int lny) {
  using C = SemCfg<P, Q>;
  constexpr int P2 = C::P2, P3 = C::P3, Q2 = C::Q2, Q3 = C::Q3, NE = C::NE;
  // lane-uniform entries (z direction) are compile-time constants
  using R = rules::SemTables<P, Q>;
  __shared__ T sB[Q * P];
  __shared__ T sDq[Q * Q];
  __shared__ T s1[NE * C::L1];
  __shared__ T s2[NE * C::L2];
  __shared__ T s3[NE * C::L3];

  const int tid = threadIdx.x;
  const int le = tid / Q2, pq = tid % Q2;
  const int i = pq % Q, j = pq / Q;
  // LAT: a brick of NE elements along x of a structured lattice (see
  // sem_lattice), its node lattice of LX x P x P nodes gathered and written once
  constexpr int p = P - 1, LX = NE * p + 1, LN = LX * P2;
  int64_t e;
  bool active;
  int nex = 0;
  int64_t I0 = 0, J0 = 0, K0 = 0, NX = 0, NY = 0;
  if constexpr (LAT) {
    const int nbx = (lnx + NE - 1) / NE;
    const int brick = (int)xcd_block(blockIdx.x, gridDim.x);
    const int bxi = brick % nbx, byi = (brick / nbx) % lny, bzi = brick / (nbx * lny);
    nex = min(NE, lnx - bxi * NE);
    e = (int64_t)(bxi * NE + le) + (int64_t)lnx * (byi + (int64_t)lny * bzi);
    active = le < nex;
    NX = (int64_t)p * lnx + 1;
    NY = (int64_t)p * lny + 1;
    I0 = (int64_t)bxi * NE * p;
    J0 = (int64_t)byi * p;
    K0 = (int64_t)bzi * p;
  } else {
    e = (int64_t)xcd_block(blockIdx.x, gridDim.x) * NE + le;
    active = (le < NE) && (e < n_elem);
  }
  const bool node = active && i < P && j < P;  // lane owns node pencil (a=i, b=j)
  const bool rowb = active && j < P;           // lane owns (k1=i, b=j)
  const int bt = blockIdx.y;
  x += (int64_t)bt * n_dof;
  y += (int64_t)bt * n_dof;

  for (int t = tid; t < Q * P; t += blockDim.x) sB[t] = Btab[t];
  for (int t = tid; t < Q * Q; t += blockDim.x) sDq[t] = Dqtab[t];
  T* b1 = s1 + le * C::L1;
  T* b2 = s2 + le * C::L2;
  T* b3 = s3 + le * C::L3;

  if constexpr (LAT) {
    // the brick's node lattice into s3 (free until the z-interpolation)
    for (int n = tid; n < LN; n += blockDim.x) {
      const int ii = n % LX, jj = (n / LX) % P, kk = n / (LX * P);
      const bool in = ii <= nex * p;
      const T v = x[in ? (I0 + ii) + NX * ((J0 + jj) + NY * (K0 + kk)) : 0];
      s3[n] = in ? v : T(0);
    }
  } else if (node) {
#pragma unroll
    for (int c = 0; c < P; ++c) b1[c * P2 + j * P + i] = x[ed[e * P3 + c * P2 + j * P + i]];
  }
  __syncthreads();
  // x-interpolation: b2[c][b][k1] = sum_a B[k1][a] u[c][b][a]
  if (rowb) {
    const T* u = LAT ? s3 + le * p + LX * j : b1 + j * P;
    constexpr int CS = LAT ? LX * P : P2;
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T s = 0;
#pragma unroll
      for (int a = 0; a < P; ++a) s += sB[i * P + a] * u[c * CS + a];
      b2[c * P * Q + j * Q + i] = s;
    }
  }
  __syncthreads();
  // y-interpolation: b1[c][k2][k1] = sum_b B[k2][b] b2[c][b][k1]
  if (active) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < P; ++b) s += sB[j * P + b] * b2[c * P * Q + b * Q + i];
      b1[c * Q2 + j * Q + i] = s;
    }
  }
  __syncthreads();
  // z-interpolation into b3[k3][k2][k1] (the lane's own column is read back
  // from there, so the values need no registers between the phases)
  if (active) {
#pragma unroll
    for (int k = 0; k < Q; ++k) {
      T s = 0;
#pragma unroll
      for (int c = 0; c < P; ++c) s += T(R::B.v[k * P + c]) * b1[c * Q2 + j * Q + i];
      b3[k * Q2 + j * Q + i] = s;
    }
  }
  __syncthreads();

  T rq[Q];
  if (STIFF) {
    T dx[Q], dy[Q], dz[Q];
    if (active) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        T sx = 0, sy = 0, sz = 0;
#pragma unroll
        for (int m = 0; m < Q; ++m) {
          sx += sDq[i * Q + m] * b3[k * Q2 + j * Q + m];
          sy += sDq[j * Q + m] * b3[k * Q2 + m * Q + i];
          sz += T(R::Dq.v[k * Q + m]) * b3[m * Q2 + j * Q + i];
        }
        dx[k] = sx;
        dy[k] = sy;
        dz[k] = sz;
      }
    }
    __syncthreads();
    T fz[Q];
    if (active) {
      const T* Ge = G + ((int64_t)bt * n_elem + e) * 6 * Q3;
      // mass weight W|J| = det G / (W^2 det sigma) when det sigma > 0 (no W|J|
      // stream; wtab holds w and then 1/w^2), else the stored W|J|
      const T id = idet ? idet[(int64_t)bt * n_elem + e] : T(0);
      const T iw2ij = idet ? wtab[Q + i] * wtab[Q + j] : T(0);
      // one branch-free loop per mass source (MASS 1: W|J| from det G, 0: the
      // stored W|J|), so that the G loads of later planes are issued ahead of
      // the earlier planes' arithmetic; FP64 with P <= 4 keeps the choice in
      // the loop (MASS -1): there the hoisted loads cost a wave per SIMD
      // (p = 2, q = 4: 4.6 -> 5.8 ms on the 51M-DOF slab)
      auto flux = [&](auto mass_tag) {
        constexpr int MASS = decltype(mass_tag)::value;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
          const int q = k * Q2 + j * Q + i;
          T g6[6];
          load_g6(Ge + (int64_t)q * 6, g6);
          const T g00 = g6[0], g01 = g6[1], g02 = g6[2];
          const T g11 = g6[3], g12 = g6[4], g22 = g6[5];
          const T uk = b3[q];  // this lane's value, read before its flux overwrites it
          b3[q] = g00 * dx[k] + g01 * dy[k] + g02 * dz[k];
          b2[q] = g01 * dx[k] + g11 * dy[k] + g12 * dz[k];
          fz[k] = g02 * dx[k] + g12 * dy[k] + g22 * dz[k];
          T wj;
          if (MASS == 1 || (MASS == -1 && idet)) {
            const T dG = g00 * (g11 * g22 - g12 * g12) - g01 * (g01 * g22 - g12 * g02) +
                         g02 * (g01 * g12 - g11 * g02);
            wj = dG * (id * iw2ij) * T(R::iw2.v[k]);
          } else {
            wj = WJ[e * Q3 + q];
          }
          rq[k] = alpha * wj * uk;
        }
      };
      if constexpr (sizeof(T) == 8 && P <= 4) flux(std::integral_constant<int, -1>{});
      else if (idet) flux(std::integral_constant<int, 1>{});
      else flux(std::integral_constant<int, 0>{});
    }
    __syncthreads();
    if (active) {
#pragma unroll
      for (int k = 0; k < Q; ++k) {
        T v = rq[k];
#pragma unroll
        for (int m = 0; m < Q; ++m) {
          v += sDq[m * Q + i] * b3[k * Q2 + j * Q + m];
          v += sDq[m * Q + j] * b2[k * Q2 + m * Q + i];
          v += T(R::Dq.v[m * Q + k]) * fz[m];
        }
        rq[k] = v;
      }
    }
  } else {
    if (active) {
#pragma unroll
      for (int k = 0; k < Q; ++k)
        rq[k] = alpha * WJ[e * Q3 + k * Q2 + j * Q + i] * b3[k * Q2 + j * Q + i];
    }
  }
  // back to the nodes: z-pass from registers into b1[c][k2][k1]
  if (active) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) s += T(R::B.v[k * P + c]) * rq[k];
      b1[c * Q2 + j * Q + i] = s;
    }
  }
  __syncthreads();
  // y-pass: b2[c][b][k1] = sum_k2 B[k2][b] b1[c][k2][k1]
  if (rowb) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) s += sB[k * P + j] * b1[c * Q2 + k * Q + i];
      b2[c * P * Q + j * Q + i] = s;
    }
  }
  __syncthreads();
  // x-pass and scatter: v[c][b][a] = sum_k1 B[k1][a] b2[c][b][k1]
  if (node) {
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T s = 0;
#pragma unroll
      for (int k = 0; k < Q; ++k) s += sB[k * P + i] * b2[c * P * Q + j * Q + k];
      if constexpr (LAT)
        b1[c * P2 + j * P + i] = s;  // the element's node buffer (free after the y-pass)
      else
        atomic_add(&y[ed[e * P3 + c * P2 + j * P + i]], s);
    }
  }
  if constexpr (LAT) {
    __syncthreads();
    for (int n = tid; n < LN; n += blockDim.x) {
      const int ii = n % LX, jj = (n / LX) % P, kk = n / (LX * P);
      if (ii > nex * p) continue;
      // the node's contributions: its element, and the previous one on an
      // element boundary along x
      const int el = min(ii / p, nex - 1), a = ii - el * p;
      T sum = s1[el * C::L1 + kk * P2 + jj * P + a];
      if (a == 0 && el > 0) sum += s1[(el - 1) * C::L1 + kk * P2 + jj * P + p];
      atomic_add(y + (I0 + ii) + NX * ((J0 + jj) + NY * (K0 + kk)), sum);
    }
  }
}

// --------------------------------------------------------------- fills -----
template <typename T>
__global__ void zero_kernel(T* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) y[i] = T(0);
}

template <typename T>
void zero(T* y, int64_t n, hipStream_t s) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  zero_kernel<T><<<dim3((unsigned)blocks), dim3(256), 0, s>>>(y, n);
  MFSEM_LAUNCH("zero_kernel");
}

template <typename T>
const T* tables_of(const mfsem_op& op);
template <>
const double* tables_of<double>(const mfsem_op& op) { return op.tab64; }
template <>
const float* tables_of<float>(const mfsem_op& op) { return op.tab32; }
template <typename T>
const T* G_of(const mfsem_op& op);
template <>
const double* G_of<double>(const mfsem_op& op) { return op.G64; }
template <>
const float* G_of<float>(const mfsem_op& op) { return op.G32; }
template <typename T>
const T* WJ_of(const mfsem_op& op);
template <>
const double* WJ_of<double>(const mfsem_op& op) { return op.WJ64; }
template <>
const float* WJ_of<float>(const mfsem_op& op) { return op.WJ32; }

template <typename T>
const T* idet_of(const mfsem_op& op);
template <>
const double* idet_of<double>(const mfsem_op& op) { return op.idet64; }
template <>
const float* idet_of<float>(const mfsem_op& op) { return op.idet32; }

template <typename T, int P, bool STIFF>
void run_ni(const mfsem_op& op, const T* x, T* y, T alpha, hipStream_t s) {
  using C = NiCfg<P>;
  const unsigned nb = blocks_for(op.d.n_elem, C::NE);
  const T* tab = tables_of<T>(op);
  ax_ni_kernel<T, P, STIFF><<<dim3(nb, op.d.batch), dim3(C::THREADS), 0, s>>>(
      op.d.n_elem, op.d.n_dof, op.d.elem_dof, G_of<T>(op), WJ_of<T>(op),
      op.use_det ? idet_of<T>(op) : nullptr, alpha, tab + op.off.Db, tab + op.off.w, x, y);
  MFSEM_LAUNCH("ax_ni_kernel");
}

template <typename T, int P, int Q, bool STIFF>
void run_sem(const mfsem_op& op, const T* x, T* y, T alpha, hipStream_t s) {
  using C = SemCfg<P, Q>;
  const unsigned nb = blocks_for(op.d.n_elem, C::NE);
  const T* tab = tables_of<T>(op);
  if constexpr (STIFF && sem_lattice<T, P, Q>()) {
    if (op.structured) {
      const unsigned nbl = (unsigned)(((op.lat[0] + C::NE - 1) / C::NE) * (int64_t)op.lat[1] *
                                      op.lat[2]);
      ax_sem_kernel<T, P, Q, STIFF, true><<<dim3(nbl, op.d.batch), dim3(C::THREADS), 0, s>>>(
          op.d.n_elem, op.d.n_dof, op.d.elem_dof, G_of<T>(op), WJ_of<T>(op),
          op.use_det ? idet_of<T>(op) : nullptr, alpha, tab + op.off.B, tab + op.off.Dq,
          tab + op.off.w, x, y, op.lat[0], op.lat[1]);
      MFSEM_LAUNCH("ax_sem_kernel (lattice)");
      return;
    }
  }
  ax_sem_kernel<T, P, Q, STIFF><<<dim3(nb, op.d.batch), dim3(C::THREADS), 0, s>>>(
      op.d.n_elem, op.d.n_dof, op.d.elem_dof, G_of<T>(op), WJ_of<T>(op),
      op.use_det ? idet_of<T>(op) : nullptr, alpha, tab + op.off.B, tab + op.off.Dq,
      tab + op.off.w, x, y, 0, 0);
  MFSEM_LAUNCH("ax_sem_kernel");
}

template <typename T, bool STIFF>
void dispatch(const mfsem_op& op, const T* x, T* y, T alpha, hipStream_t s) {
  const int P = op.P, Q = op.Q;
  if (op.d.quad == MFSEM_GLL) {
    switch (P) {
      case 2: return run_ni<T, 2, STIFF>(op, x, y, alpha, s);
      case 3: return run_ni<T, 3, STIFF>(op, x, y, alpha, s);
      case 4: return run_ni<T, 4, STIFF>(op, x, y, alpha, s);
      case 5: return run_ni<T, 5, STIFF>(op, x, y, alpha, s);
      case 6: return run_ni<T, 6, STIFF>(op, x, y, alpha, s);
      case 7: return run_ni<T, 7, STIFF>(op, x, y, alpha, s);
      case 8: return run_ni<T, 8, STIFF>(op, x, y, alpha, s);
      case 9: return run_ni<T, 9, STIFF>(op, x, y, alpha, s);
    }
  } else {
#define MFSEM_SEM_CASE(PP)                                               \
  case PP:                                                               \
    if (Q == PP) return run_sem<T, PP, PP, STIFF>(op, x, y, alpha, s);   \
    if (Q == PP + 1) return run_sem<T, PP, PP + 1, STIFF>(op, x, y, alpha, s); \
    if (Q == PP + 2) return run_sem<T, PP, PP + 2, STIFF>(op, x, y, alpha, s); \
    break;
    switch (P) {
      MFSEM_SEM_CASE(2)
      MFSEM_SEM_CASE(3)
      MFSEM_SEM_CASE(4)
      MFSEM_SEM_CASE(5)
      MFSEM_SEM_CASE(6)
      MFSEM_SEM_CASE(7)
      MFSEM_SEM_CASE(8)
      MFSEM_SEM_CASE(9)
    }
#undef MFSEM_SEM_CASE
  }
  fail(MFSEM_EUNSUPPORTED, "no apply kernel for this (p, quadrature) pair");
}

// ------------------------------------------------------------ diagonal -----
// diag(A)_i = sum_e sum_k [alpha W|J| phi_i^2 + grad_ref(phi_i)^T G grad_ref(phi_i)],
// with phi_i = l_a l_b l_c and grad_ref = (l_a' l_b l_c, l_a l_b' l_c, l_a l_b l_c').
// Each of the seven stored fields F (alpha W|J| and the six entries of G) is
// weighted by a product of 1D factors, e.g. G00 by (l_a')^2 (l_b)^2 (l_c)^2 and
// G01 by 2 (l_a l_a')(l_b l_b')(l_c)^2, so its contribution is the separable
// contraction sum_k3 Z[k3][c] sum_k2 Y[k2][b] sum_k1 X[k1][a] F[k3][k2][k1],
// evaluated as three 1D passes (sum factorisation, Section 4.1) with X, Y, Z
// among BB = B^2, DD = D^2, BD = B D.  One workgroup per element and member.
constexpr int DIAG_THREADS = 256;
constexpr int MAXQ = MFSEM_MAX_P + 3, MAXP = MFSEM_MAX_P + 1;

template <typename T>
__global__ __launch_bounds__(DIAG_THREADS) void diag_kernel(
    int64_t n_elem, int64_t n_dof, int P, int Q, const int32_t* __restrict__ ed,
    const T* __restrict__ G, const T* __restrict__ WJ, T alpha, const T* __restrict__ Btab,
    const T* __restrict__ Dbtab, T* __restrict__ d) {
  __shared__ T sM[3][MAXQ * MAXP];  // BB, DD, BD
  __shared__ T sF[MAXQ * MAXQ * MAXQ];
  __shared__ T t1[MAXQ * MAXQ * MAXP];
  __shared__ T t2[MAXQ * MAXP * MAXP];
  const int64_t e = blockIdx.x;
  const int bt = blockIdx.y;
  const int P2 = P * P, P3 = P2 * P, Q2 = Q * Q, Q3 = Q2 * Q;
  const int tid = threadIdx.x;
  for (int t = tid; t < Q * P; t += blockDim.x) {
    const T b = Btab[t], dd = Dbtab[t];
    sM[0][t] = b * b;
    sM[1][t] = dd * dd;
    sM[2][t] = b * dd;
  }
  constexpr int MAXN = (MAXP * MAXP * MAXP + DIAG_THREADS - 1) / DIAG_THREADS;
  T acc[MAXN];
  for (int r = 0; r < MAXN; ++r) acc[r] = 0;
  const T* Ge = G + ((int64_t)bt * n_elem + e) * 6 * Q3;
  // field f: 0 = alpha*WJ, 1 = G00, 2 = G11, 3 = G22, 4 = G01, 5 = G02, 6 = G12,
  // with its 1D factors along x, y, z (0 = BB, 1 = DD, 2 = BD) and multiplicity
  const int gidx[7] = {-1, 0, 3, 5, 1, 2, 4};
  const int fx[7] = {0, 1, 0, 0, 2, 2, 0}, fy[7] = {0, 0, 1, 0, 2, 0, 2},
            fz[7] = {0, 0, 0, 1, 0, 2, 2};
  for (int f = 0; f < 7; ++f) {
    __syncthreads();
    for (int k = tid; k < Q3; k += blockDim.x)
      sF[k] = (f == 0) ? alpha * WJ[e * Q3 + k] : Ge[(int64_t)k * 6 + gidx[f]];
    __syncthreads();
    const T* X = sM[fx[f]];
    const T* Y = sM[fy[f]];
    const T* Z = sM[fz[f]];
    const T mult = f >= 4 ? T(2) : T(1);
    // x: t1[k3][k2][a] = sum_k1 X[k1][a] F[k3][k2][k1]
    for (int l = tid; l < Q2 * P; l += blockDim.x) {
      const int a = l % P, k23 = l / P;
      T s = 0;
      for (int k1 = 0; k1 < Q; ++k1) s += X[k1 * P + a] * sF[k23 * Q + k1];
      t1[l] = s;
    }
    __syncthreads();
    // y: t2[k3][b][a] = sum_k2 Y[k2][b] t1[k3][k2][a]
    for (int l = tid; l < Q * P2; l += blockDim.x) {
      const int a = l % P, b = (l / P) % P, k3 = l / P2;
      T s = 0;
      for (int k2 = 0; k2 < Q; ++k2) s += Y[k2 * P + b] * t1[(k3 * Q + k2) * P + a];
      t2[l] = s;
    }
    __syncthreads();
    // z: node (a, b, c) += mult sum_k3 Z[k3][c] t2[k3][b][a]
    for (int r = 0; r < MAXN; ++r) {
      const int l = tid + r * DIAG_THREADS;
      if (l >= P3) break;
      const int ab = l % P2, c = l / P2;
      T s = 0;
      for (int k3 = 0; k3 < Q; ++k3) s += Z[k3 * P + c] * t2[k3 * P2 + ab];
      acc[r] += mult * s;
    }
  }
  for (int r = 0; r < MAXN; ++r) {
    const int l = tid + r * DIAG_THREADS;
    if (l >= P3) break;
    atomic_add(&d[(int64_t)bt * n_dof + ed[e * P3 + l]], acc[r]);
  }
}

}  // namespace

template <typename T>
void launch_apply(const mfsem_op& op, const T* x, T* y, double alpha, bool stiffness,
                  hipStream_t s, bool accumulate) {
  if (!accumulate) zero<T>(y, op.d.n_dof * op.d.batch, s);
  if (op.d.n_elem == 0) return;
  // the GLL kernels read 1/w^2 right after the weights
  if (op.off.iw2 != op.off.w + op.Q) fail(MFSEM_EDEVICE, "table layout: 1/w^2 must follow w");
  if (stiffness && launch_brick<T>(op, G_of<T>(op), WJ_of<T>(op),
                                   op.use_det ? idet_of<T>(op) : nullptr, tables_of<T>(op), x, y,
                                   (T)alpha, s))
    return;
  if (stiffness) dispatch<T, true>(op, x, y, (T)alpha, s);
  else dispatch<T, false>(op, x, y, (T)alpha, s);
}

template <typename T>
void launch_diag(const mfsem_op& op, T* d, hipStream_t s) {
  zero<T>(d, op.d.n_dof * op.d.batch, s);
  if (op.d.n_elem == 0) return;
  const T* tab = tables_of<T>(op);
  diag_kernel<T><<<dim3((unsigned)op.d.n_elem, op.d.batch), dim3(DIAG_THREADS), 0, s>>>(
      op.d.n_elem, op.d.n_dof, op.P, op.Q, op.d.elem_dof, G_of<T>(op), WJ_of<T>(op),
      (T)op.alpha, tab + op.off.B, tab + op.off.Db, d);
  MFSEM_LAUNCH("diag_kernel");
}

template void launch_apply<double>(const mfsem_op&, const double*, double*, double, bool,
                                   hipStream_t, bool);
template void launch_apply<float>(const mfsem_op&, const float*, float*, double, bool,
                                  hipStream_t, bool);
template void launch_diag<double>(const mfsem_op&, double*, hipStream_t);
template void launch_diag<float>(const mfsem_op&, float*, hipStream_t);

}  // namespace mfsem
