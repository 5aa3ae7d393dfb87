// Inter-level transfers on structured lattices as three 1D passes.
//
// On a box the fine space's nodes form a tensor lattice, and the prolongation
// of Section 4.3 (interpolating the coarse function at the fine nodes, by
// degree for p-levels, by octree children for h-levels) is the tensor product
// of three 1D interpolations: fine node i along an axis lies in element
// e = min(i / p_f, n - 1) at local node a = i - e p_f, and takes
//     sum_b L[a][b] coarse[start(e) + b],
// with L the 1D element interpolation (the child's half for h-levels) and
// start(e) the first coarse node of the coarse element holding e.  A fine node
// on an element face gets the same value from both sides, so every fine node
// is written once.  Restriction is the exact transpose: for each coarse node,
// the sum over the fine nodes that reference it.  Each pass runs one thread per
// coarse element of a lattice line (lanes along x for the y and z passes, so
// their loads and stores are coalesced rows), reading each input value about
// once, without index arrays over elements, atomics or multiplicity weights.
#include "transfer_lattice.hpp"

#include <algorithm>

namespace mfsem {

namespace {

constexpr int LT = 256;

struct Dims {
  int ox, oy, oz;  // output lattice
  int ix, iy;      // input lattice (x and y extents; z follows from the pass)
};

// One 1D pass along axis AX, in element blocks.  Along the pass axis the fine
// lattice is ne coarse elements of F fine intervals each (F = p_f for a
// p-transfer, 2p for an h-transfer, the two children side by side), and the
// 1D interpolation of one coarse element is the dense matrix M [F+1][PC1]
// (row a: the coarse basis at the element's a-th fine node).  A fine node on
// a coarse element boundary belongs to the element on its right (the last one
// to the last element).  One thread per coarse element and line:
//   forward:    fine a (owned) = sum_b M[a][b] coarse(E p_c + b);
//   transposed: coarse b = sum over the element's owned fine a of M[a][b] fine,
//               and the left vertex b = 0 also gathers the previous element's
//               interior fine nodes with weights M[a][p_c];
// each thread writes only the nodes it owns, so every output is written once
// and no atomics are needed.  Each input value is read once by its element
// (twice for the transposed pass's interior nodes next to a vertex), instead
// of once per output that references it (up to 2 p_f + 1 times).
template <typename T, int AX, bool BWD, bool SUB, bool ACC, int PC1>
__global__ __launch_bounds__(LT) void lattice_elem_kernel(
    const T* __restrict__ in, const T* __restrict__ in2, T* __restrict__ out,
    T* __restrict__ zero, Dims d, int iz, int64_t n_in, int64_t n_out, ElemMat<T> m) {
  const int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x;
  const int ne = m.ne, F = m.F;
  // lines: the two axes other than AX, whose extents are the same in and out
  const int e0 = AX == 0 ? ne : d.ox;
  const int e1 = AX == 1 ? ne : d.oy;
  const int e2 = AX == 2 ? ne : d.oz;
  if (t >= (int64_t)e0 * e1 * e2) return;
  const int c0 = (int)(t % e0);
  const int c1 = (int)((t / e0) % e1);
  const int c2 = (int)(t / ((int64_t)e0 * e1));
  const int E = AX == 0 ? c0 : (AX == 1 ? c1 : c2);
  const int64_t bt = blockIdx.y;
  in += bt * n_in;
  if (SUB) in2 += bt * n_in;
  out += bt * n_out;
  if (zero) zero += bt * n_out;
  // strides of the input and output lattices, and the line's offset in each
  const int64_t isy = d.ix, isz = (int64_t)d.ix * d.iy;
  const int64_t osy = d.ox, osz = (int64_t)d.ox * d.oy;
  const int64_t ia = AX == 0 ? 1 : (AX == 1 ? isy : isz);
  const int64_t oa = AX == 0 ? 1 : (AX == 1 ? osy : osz);
  const int64_t ibase = (AX == 0 ? 0 : c0) + (AX == 1 ? 0 : c1 * isy) + (AX == 2 ? 0 : c2 * isz);
  const int64_t obase = (AX == 0 ? 0 : c0) + (AX == 1 ? 0 : c1 * osy) + (AX == 2 ? 0 : c2 * osz);
  constexpr int PC = PC1 - 1;
  const bool last = E == ne - 1;
  (void)iz;
  if (!BWD) {
    T cv[PC1];
#pragma unroll
    for (int b = 0; b < PC1; ++b) cv[b] = in[ibase + (int64_t)(E * PC + b) * ia];
    const int a_end = last ? F : F - 1;
    for (int a = 0; a <= a_end; ++a) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < PC1; ++b) s += m.M[a * PC1 + b] * cv[b];
      const int64_t o = obase + (int64_t)(E * F + a) * oa;
      out[o] = ACC ? out[o] + s : s;
      if (zero) zero[o] = T(0);
    }
  } else {
    T acc[PC1];
#pragma unroll
    for (int b = 0; b < PC1; ++b) acc[b] = 0;
    const int a_end = last ? F : F - 1;
    for (int a = 0; a <= a_end; ++a) {
      const int64_t k = ibase + (int64_t)(E * F + a) * ia;
      const T v = SUB ? in[k] - in2[k] : in[k];
#pragma unroll
      for (int b = 0; b < PC1; ++b) acc[b] += m.M[a * PC1 + b] * v;
    }
    if (E > 0) {
      for (int a = 1; a < F; ++a) {
        const int64_t k = ibase + (int64_t)((E - 1) * F + a) * ia;
        const T v = SUB ? in[k] - in2[k] : in[k];
        acc[0] += m.M[a * PC1 + PC] * v;
      }
    }
#pragma unroll
    for (int b = 0; b < PC1; ++b)
      if (b < PC || last) out[obase + (int64_t)(E * PC + b) * oa] = acc[b];
  }
}

template <typename T, int AX, bool BWD, bool SUB, bool ACC, int PC1>
void elem_pass_pc(const T* in, const T* in2, T* out, T* zero, const int od[3], const int id[3],
                  const ElemMat<T>& m, int batch, hipStream_t s) {
  const int64_t lines = AX == 0 ? (int64_t)od[1] * od[2]
                                : (AX == 1 ? (int64_t)od[0] * od[2] : (int64_t)od[0] * od[1]);
  const int64_t threads = lines * m.ne;
  if (threads == 0 || batch == 0) return;
  const Dims d{od[0], od[1], od[2], id[0], id[1]};
  const int64_t n_in = (int64_t)id[0] * id[1] * id[2];
  const int64_t n_out = (int64_t)od[0] * od[1] * od[2];
  const dim3 grid((unsigned)((threads + LT - 1) / LT), (unsigned)batch);
  lattice_elem_kernel<T, AX, BWD, SUB, ACC, PC1>
      <<<grid, LT, 0, s>>>(in, in2, out, zero, d, id[2], n_in, n_out, m);
  MFSEM_LAUNCH("lattice_elem_kernel");
}

template <typename T, int AX, bool BWD, bool SUB, bool ACC>
void elem_pass(const T* in, const T* in2, T* out, T* zero, const int od[3], const int id[3],
               const ElemMat<T>& m, int batch, hipStream_t s) {
  switch (m.pc1) {
#define MFSEM_ELEM_CASE(K) \
  case K: return elem_pass_pc<T, AX, BWD, SUB, ACC, K>(in, in2, out, zero, od, id, m, batch, s);
    MFSEM_ELEM_CASE(2)
    MFSEM_ELEM_CASE(3)
    MFSEM_ELEM_CASE(4)
    MFSEM_ELEM_CASE(5)
    MFSEM_ELEM_CASE(6)
    MFSEM_ELEM_CASE(7)
    MFSEM_ELEM_CASE(8)
    MFSEM_ELEM_CASE(9)
#undef MFSEM_ELEM_CASE
  }
  fail(MFSEM_EUNSUPPORTED, "lattice transfer: coarse degree beyond the element-block kernels");
}

__global__ void box_parents_check_kernel(int n0, int n1, int64_t n_elem,
                                         const int32_t* __restrict__ parent,
                                         const int8_t* __restrict__ child,
                                         unsigned long long* __restrict__ mismatch) {
  const int c0 = n0 / 2, c1 = n1 / 2;
  unsigned long long bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_elem;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ex = e % n0, ey = (e / n0) % n1, ez = e / ((int64_t)n0 * n1);
    const int64_t pe = ex / 2 + c0 * (ey / 2 + (int64_t)c1 * (ez / 2));
    const int ch = (int)((ex & 1) | ((ey & 1) << 1) | ((ez & 1) << 2));
    bad += (parent[e] != pe || child[e] != ch) ? 1 : 0;
  }
  if (bad) atomicAdd(mismatch, bad);
}

__global__ void parents_range_kernel(int64_t n_fine, int64_t n_coarse,
                                     const int32_t* __restrict__ parent,
                                     const int8_t* __restrict__ child,
                                     unsigned long long* __restrict__ bad) {
  unsigned long long cnt = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_fine;
       e += (int64_t)gridDim.x * blockDim.x)
    cnt += (parent[e] < 0 || parent[e] >= n_coarse || child[e] < 0 || child[e] > 7) ? 1 : 0;
  if (cnt) atomicAdd(bad, cnt);
}

// Node counts of one axis: fine and coarse lattices.
void axis_counts(int kind, int pf, int pc, int nf_elem, LatticeAxisHost& h) {
  h.nf = pf * nf_elem + 1;
  h.nc = pc * (kind == MFSEM_TRANSFER_H ? nf_elem / 2 : nf_elem) + 1;
}
}  // namespace

bool lattice_transfer_applies(const mfsem_op& fine, const mfsem_op& coarse, int kind) {
  if (kind != MFSEM_TRANSFER_P && kind != MFSEM_TRANSFER_H) return false;
  if (!fine.structured || !coarse.structured || fine.d.n_elem == 0) return false;
  for (int d = 0; d < 3; ++d) {
    if (kind == MFSEM_TRANSFER_P && fine.lat[d] != coarse.lat[d]) return false;
    if (kind == MFSEM_TRANSFER_H && fine.lat[d] != 2 * coarse.lat[d]) return false;
  }
  // the vectors are exactly the lattices
  auto nodes = [](const mfsem_op& op, int d) { return (int64_t)(op.P - 1) * op.lat[d] + 1; };
  if (fine.d.n_dof != nodes(fine, 0) * nodes(fine, 1) * nodes(fine, 2)) return false;
  if (coarse.d.n_dof != nodes(coarse, 0) * nodes(coarse, 1) * nodes(coarse, 2)) return false;
  // launch limits of the passes: z extents on grid.y, (x, y) planes in 32 bits
  return nodes(fine, 2) <= 65535 && nodes(fine, 0) * nodes(fine, 1) < ((int64_t)1 << 31) &&
         fine.d.batch <= 65535;
}

void lattice_transfer_layout(LatticeTransfer& t, const mfsem_op& fine, const mfsem_op& coarse,
                             int kind, int batch, size_t word, Arena& a) {
  const std::vector<double> I = transfer_matrices(kind, fine.P - 1, coarse.P - 1);
  for (int d = 0; d < 3; ++d) axis_counts(kind, fine.P - 1, coarse.P - 1, fine.lat[d], t.host[d]);
  {
    const int pf = fine.P - 1, Pf = fine.P, Pc = coarse.P;
    const bool hk = kind == MFSEM_TRANSFER_H;
    for (int d = 0; d < 3; ++d) {
      ElemMat<double>& m = t.em64[d];
      m.ne = coarse.lat[d];
      m.F = hk ? 2 * pf : pf;
      m.pc1 = Pc;
      for (int a = 0; a <= m.F; ++a) {
        const int child = (hk && a > pf) ? 1 : 0;
        const int af = a - child * pf;
        for (int b = 0; b < Pc; ++b)
          m.M[a * Pc + b] = I[(size_t)child * Pf * Pc + (size_t)af * Pc + b];
      }
      ElemMat<float>& f = t.em32[d];
      f.ne = m.ne;
      f.F = m.F;
      f.pc1 = m.pc1;
      for (int i = 0; i < (m.F + 1) * Pc; ++i) f.M[i] = (float)m.M[i];
    }
  }
  const int64_t nfx = t.host[0].nf, nfy = t.host[1].nf;
  const int64_t ncy = t.host[1].nc, ncz = t.host[2].nc;
  // both directions pass through (nfx, ncy, ncz) in s1 and (nfx, nfy, ncz) in s2
  t.s1 = a.take((size_t)(nfx * ncy * ncz) * batch * word);
  t.s2 = a.take((size_t)(nfx * nfy * ncz) * batch * word);
  t.word = word;
}

void launch_box_parents_check(const int32_t n_fine[3], const int32_t* parent,
                              const int8_t* child, unsigned long long* mismatch, hipStream_t s) {
  const int64_t ne = (int64_t)n_fine[0] * n_fine[1] * n_fine[2];
  if (ne == 0) return;
  int64_t blocks = (ne + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  box_parents_check_kernel<<<(unsigned)blocks, 256, 0, s>>>(n_fine[0], n_fine[1], ne, parent,
                                                           child, mismatch);
  MFSEM_LAUNCH("box_parents_check_kernel");
}

void launch_parents_range_check(int64_t n_fine, int64_t n_coarse, const int32_t* parent,
                                const int8_t* child, unsigned long long* bad, hipStream_t s) {
  if (n_fine == 0) return;
  int64_t blocks = (n_fine + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  parents_range_kernel<<<(unsigned)blocks, 256, 0, s>>>(n_fine, n_coarse, parent, child, bad);
  MFSEM_LAUNCH("parents_range_kernel");
}

// x pass, y pass, z pass: (ncx, ncy, ncz) -> (nfx, ncy, ncz) -> (nfx, nfy, ncz)
// -> (nfx, nfy, nfz)
template <typename T>
const ElemMat<T>& emat(const LatticeTransfer& t, int d);
template <>
const ElemMat<double>& emat<double>(const LatticeTransfer& t, int d) { return t.em64[d]; }
template <>
const ElemMat<float>& emat<float>(const LatticeTransfer& t, int d) { return t.em32[d]; }

// x pass, y pass, z pass: (ncx, ncy, ncz) -> (nfx, ncy, ncz) -> (nfx, nfy, ncz)
// -> (nfx, nfy, nfz)
template <typename T>
void lattice_prolong(const LatticeTransfer& t, int batch, const T* xc, T* xf, bool accumulate,
                     T* zero_f, hipStream_t s) {
  const LatticeAxisHost &hx = t.host[0], &hy = t.host[1], &hz = t.host[2];
  T* s1 = static_cast<T*>(t.s1);
  T* s2 = static_cast<T*>(t.s2);
  {
    const int id[3] = {hx.nc, hy.nc, hz.nc}, od[3] = {hx.nf, hy.nc, hz.nc};
    elem_pass<T, 0, false, false, false>(xc, nullptr, s1, nullptr, od, id, emat<T>(t, 0), batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nc, hz.nc}, od[3] = {hx.nf, hy.nf, hz.nc};
    elem_pass<T, 1, false, false, false>(s1, nullptr, s2, nullptr, od, id, emat<T>(t, 1), batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nf, hz.nc}, od[3] = {hx.nf, hy.nf, hz.nf};
    if (accumulate)
      elem_pass<T, 2, false, false, true>(s2, nullptr, xf, zero_f, od, id, emat<T>(t, 2), batch, s);
    else
      elem_pass<T, 2, false, false, false>(s2, nullptr, xf, zero_f, od, id, emat<T>(t, 2), batch,
                                           s);
  }
}

// transposed passes, z first: (nfx, nfy, nfz) -> (nfx, nfy, ncz) -> (nfx, ncy, ncz)
// -> (ncx, ncy, ncz)
template <typename T>
void lattice_restrict(const LatticeTransfer& t, int batch, const T* bf, const T* tf, T* rc,
                      hipStream_t s) {
  const LatticeAxisHost &hx = t.host[0], &hy = t.host[1], &hz = t.host[2];
  T* s1 = static_cast<T*>(t.s1);
  T* s2 = static_cast<T*>(t.s2);
  {
    const int id[3] = {hx.nf, hy.nf, hz.nf}, od[3] = {hx.nf, hy.nf, hz.nc};
    if (tf)
      elem_pass<T, 2, true, true, false>(bf, tf, s2, nullptr, od, id, emat<T>(t, 2), batch, s);
    else
      elem_pass<T, 2, true, false, false>(bf, nullptr, s2, nullptr, od, id, emat<T>(t, 2), batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nf, hz.nc}, od[3] = {hx.nf, hy.nc, hz.nc};
    elem_pass<T, 1, true, false, false>(s2, nullptr, s1, nullptr, od, id, emat<T>(t, 1), batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nc, hz.nc}, od[3] = {hx.nc, hy.nc, hz.nc};
    elem_pass<T, 0, true, false, false>(s1, nullptr, rc, nullptr, od, id, emat<T>(t, 0), batch, s);
  }
}

template void lattice_prolong<double>(const LatticeTransfer&, int, const double*, double*, bool,
                                      double*, hipStream_t);
template void lattice_prolong<float>(const LatticeTransfer&, int, const float*, float*, bool,
                                     float*, hipStream_t);
template void lattice_restrict<double>(const LatticeTransfer&, int, const double*, const double*,
                                       double*, hipStream_t);
template void lattice_restrict<float>(const LatticeTransfer&, int, const float*, const float*,
                                      float*, hipStream_t);

}  // namespace mfsem
