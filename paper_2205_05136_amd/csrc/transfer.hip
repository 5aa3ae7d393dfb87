// Inter-level transfers of the geometric multigrid (Section 4.3: p-degree
// interpolation and restriction among octree meshes).
//
// Prolongation of a coarse function to a fine element is interpolation of
// the coarse element's nodal values at the fine nodes, applied as three 1D
// passes with I[i][a] = l^c_a(xi_i) (p-coarsening) or
// I_c[i][a] = l^c_a((xi_i + 2c - 1)/2) for the fine element's offset c in its
// octree parent (h-coarsening).  A node shared by several fine elements gets
// the same value from each of them (the 1D rows at element ends are exact
// unit vectors), so the result is written with plain stores.
// Restriction is the exact transpose: each fine element applies the
// transposed passes to w o r (w = 1/multiplicity of the fine node) and
// scatter-adds into the coarse vector.
#include "transfer.hpp"

namespace mfsem {

namespace {

constexpr int TT = 256;
constexpr int MP = MFSEM_MAX_P + 1;

template <typename T>
__global__ __launch_bounds__(TT) void prolong_kernel(TransferArgs<T> a, const T* __restrict__ xc,
                                                     T* __restrict__ xf) {
  __shared__ T sI[2 * MP * MP];
  __shared__ T u[MP * MP * MP], t1[MP * MP * MP], t2[MP * MP * MP];
  const int64_t e = blockIdx.x;
  const int bt = blockIdx.y;
  const int Pf = a.Pf, Pc = a.Pc, tid = threadIdx.x;
  const int64_t ec = a.parent ? a.parent[e] : e;
  const int ch = a.child ? a.child[e] : 0;
  xc += (int64_t)bt * a.nc;
  xf += (int64_t)bt * a.nf;
  for (int i = tid; i < 2 * Pf * Pc; i += TT) sI[i] = a.I[i];
  const int Pc3 = Pc * Pc * Pc;
  for (int l = tid; l < Pc3; l += TT) u[l] = xc[a.ed_c[ec * Pc3 + l]];
  __syncthreads();
  const T* Ix = sI + ((ch & 1) ? Pf * Pc : 0);
  const T* Iy = sI + ((ch & 2) ? Pf * Pc : 0);
  const T* Iz = sI + ((ch & 4) ? Pf * Pc : 0);
  // t1[c][b][i] = sum_a Ix[i][a] u[c][b][a]
  for (int l = tid; l < Pc * Pc * Pf; l += TT) {
    const int i = l % Pf, cb = l / Pf;
    T s = 0;
    for (int aa = 0; aa < Pc; ++aa) s += Ix[i * Pc + aa] * u[cb * Pc + aa];
    t1[l] = s;
  }
  __syncthreads();
  // t2[c][j][i] = sum_b Iy[j][b] t1[c][b][i]
  for (int l = tid; l < Pc * Pf * Pf; l += TT) {
    const int i = l % Pf, j = (l / Pf) % Pf, c = l / (Pf * Pf);
    T s = 0;
    for (int b = 0; b < Pc; ++b) s += Iy[j * Pc + b] * t1[(c * Pc + b) * Pf + i];
    t2[l] = s;
  }
  __syncthreads();
  const int Pf3 = Pf * Pf * Pf;
  for (int l = tid; l < Pf3; l += TT) {
    const int ij = l % (Pf * Pf), k = l / (Pf * Pf);
    T s = 0;
    for (int c = 0; c < Pc; ++c) s += Iz[k * Pc + c] * t2[c * Pf * Pf + ij];
    xf[a.ed_f[e * Pf3 + l]] = s;
  }
}

template <typename T>
__global__ __launch_bounds__(TT) void restrict_kernel(TransferArgs<T> a, const T* __restrict__ bf,
                                                      const T* __restrict__ tf,
                                                      const T* __restrict__ w,
                                                      T* __restrict__ rc) {
  __shared__ T sI[2 * MP * MP];
  __shared__ T r[MP * MP * MP], t2[MP * MP * MP], t1[MP * MP * MP];
  const int64_t e = blockIdx.x;
  const int bt = blockIdx.y;
  const int Pf = a.Pf, Pc = a.Pc, tid = threadIdx.x;
  const int64_t ec = a.parent ? a.parent[e] : e;
  const int ch = a.child ? a.child[e] : 0;
  bf += (int64_t)bt * a.nf;
  if (tf) tf += (int64_t)bt * a.nf;
  rc += (int64_t)bt * a.nc;
  for (int i = tid; i < 2 * Pf * Pc; i += TT) sI[i] = a.I[i];
  const int Pf3 = Pf * Pf * Pf;
  for (int l = tid; l < Pf3; l += TT) {
    const int64_t g = a.ed_f[e * Pf3 + l];
    r[l] = (tf ? bf[g] - tf[g] : bf[g]) * w[g];
  }
  __syncthreads();
  const T* Ix = sI + ((ch & 1) ? Pf * Pc : 0);
  const T* Iy = sI + ((ch & 2) ? Pf * Pc : 0);
  const T* Iz = sI + ((ch & 4) ? Pf * Pc : 0);
  // t2[c][j][i] = sum_k Iz[k][c] r[k][j][i]
  for (int l = tid; l < Pc * Pf * Pf; l += TT) {
    const int ij = l % (Pf * Pf), c = l / (Pf * Pf);
    T s = 0;
    for (int k = 0; k < Pf; ++k) s += Iz[k * Pc + c] * r[k * Pf * Pf + ij];
    t2[l] = s;
  }
  __syncthreads();
  // t1[c][b][i] = sum_j Iy[j][b] t2[c][j][i]
  for (int l = tid; l < Pc * Pc * Pf; l += TT) {
    const int i = l % Pf, b = (l / Pf) % Pc, c = l / (Pf * Pc);
    T s = 0;
    for (int j = 0; j < Pf; ++j) s += Iy[j * Pc + b] * t2[(c * Pf + j) * Pf + i];
    t1[l] = s;
  }
  __syncthreads();
  const int Pc3 = Pc * Pc * Pc;
  for (int l = tid; l < Pc3; l += TT) {
    const int aa = l % Pc, cb = l / Pc;
    T s = 0;
    for (int i = 0; i < Pf; ++i) s += Ix[i * Pc + aa] * t1[cb * Pf + i];
    atomic_add(&rc[a.ed_c[ec * Pc3 + l]], s);
  }
}

template <typename T>
__global__ void count_kernel(const int32_t* __restrict__ ed, int64_t n_elem, int P3,
                             T* __restrict__ cnt) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = n_elem * P3;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) atomic_add(&cnt[ed[i]], T(1));
}

}  // namespace

template <typename T>
void launch_prolong(const TransferArgs<T>& a, int batch, const T* xc, T* xf, hipStream_t s) {
  if (a.n_elem_f == 0) return;
  prolong_kernel<T><<<dim3((unsigned)a.n_elem_f, batch), TT, 0, s>>>(a, xc, xf);
  MFSEM_LAUNCH("prolong_kernel");
}

template <typename T>
void launch_restrict(const TransferArgs<T>& a, int batch, const T* bf, const T* tf, const T* w,
                     T* rc, hipStream_t s) {
  if (a.n_elem_f == 0) return;
  restrict_kernel<T><<<dim3((unsigned)a.n_elem_f, batch), TT, 0, s>>>(a, bf, tf, w, rc);
  MFSEM_LAUNCH("restrict_kernel");
}

template <typename T>
void launch_inv_multiplicity(const int32_t* ed, int64_t n_elem, int P3, int64_t n_dof, T* w,
                             hipStream_t s) {
  vfill<T>(w, n_dof, T(0), s);
  if (n_elem > 0) {
    int64_t blocks = (n_elem * P3 + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    count_kernel<T><<<(unsigned)blocks, 256, 0, s>>>(ed, n_elem, P3, w);
    MFSEM_LAUNCH("count_kernel");
  }
  vinvert<T>(w, n_dof, s);
}

// 1D interpolation matrices [2][Pf][Pc] (child 0 and 1; identical for p-transfers).
std::vector<double> transfer_matrices(int kind, int pf, int pc) {
  std::vector<double> xf, wf, xc, wc, L;
  gll_rule(pf, xf, wf);
  gll_rule(pc, xc, wc);
  const int Pf = pf + 1, Pc = pc + 1;
  std::vector<double> out(2 * Pf * Pc);
  for (int c = 0; c < 2; ++c) {
    std::vector<double> pts(Pf);
    for (int i = 0; i < Pf; ++i)
      pts[i] = (kind == MFSEM_TRANSFER_H) ? (xf[i] + 2.0 * c - 1.0) * 0.5 : xf[i];
    lagrange_matrices(xc, pts, &L, nullptr);
    for (int i = 0; i < Pf * Pc; ++i) out[c * Pf * Pc + i] = L[i];
  }
  return out;
}

template void launch_prolong<double>(const TransferArgs<double>&, int, const double*, double*,
                                     hipStream_t);
template void launch_prolong<float>(const TransferArgs<float>&, int, const float*, float*,
                                    hipStream_t);
template void launch_restrict<double>(const TransferArgs<double>&, int, const double*,
                                      const double*, const double*, double*, hipStream_t);
template void launch_restrict<float>(const TransferArgs<float>&, int, const float*, const float*,
                                     const float*, float*, hipStream_t);
template void launch_inv_multiplicity<double>(const int32_t*, int64_t, int, int64_t, double*,
                                              hipStream_t);
template void launch_inv_multiplicity<float>(const int32_t*, int64_t, int, int64_t, float*,
                                             hipStream_t);

}  // namespace mfsem
