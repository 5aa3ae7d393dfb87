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
// the sum over the fine nodes that reference it.  Each pass streams a lattice
// with coalesced rows, without index arrays over elements, atomics or
// multiplicity weights.
#include "transfer_lattice.hpp"

#include <algorithm>
#include <utility>

namespace mfsem {

namespace {

constexpr int LT = 256;

struct Dims {
  int ox, oy, oz;  // output lattice
  int ix, iy;      // input lattice (x and y extents; z follows from the pass)
};

// One pass along axis AX.  Forward (!BWD): out(o) = sum_m coef[o][m] in(idx[o] + m);
// transposed: out(o) = sum_m coef[o][m] in(idx[o][m]); o is the output
// coordinate along AX and the other two coordinates are kept.  SUB reads
// in - in2; ACC adds into out; with zero, zero[out index] = 0 as well.
// Grid: x over the output's (x, y) plane, y over its z, z over the batch.
template <typename T, int AX, bool BWD, bool SUB, bool ACC>
__global__ __launch_bounds__(LT) void lattice_pass_kernel(
    const T* __restrict__ in, const T* __restrict__ in2, T* __restrict__ out, T* __restrict__ zero,
    Dims d, int64_t n_in, const int32_t* __restrict__ idx, const T* __restrict__ coef, int W) {
  const uint32_t plane = (uint32_t)d.ox * (uint32_t)d.oy;
  const uint32_t t = blockIdx.x * LT + threadIdx.x;
  if (t >= plane) return;
  const int z = blockIdx.y;
  const int64_t bt = blockIdx.z;
  const int x = (int)(t % (uint32_t)d.ox), y = (int)(t / (uint32_t)d.ox);
  const int o = AX == 0 ? x : (AX == 1 ? y : z);
  const int64_t sx = 1, sy = d.ix, sz = (int64_t)d.ix * d.iy;
  const int64_t sa = AX == 0 ? sx : (AX == 1 ? sy : sz);
  // input offset with the pass coordinate at 0
  const int64_t base = bt * n_in + (AX == 0 ? 0 : x) * sx + (AX == 1 ? 0 : (int64_t)y) * sy +
                       (AX == 2 ? 0 : (int64_t)z) * sz;
  const T* cf = coef + (int64_t)o * W;
  T s = 0;
  if (!BWD) {
    const int64_t k0 = base + (int64_t)idx[o] * sa;
    for (int m = 0; m < W; ++m) {
      const int64_t k = k0 + m * sa;
      s += cf[m] * (SUB ? in[k] - in2[k] : in[k]);
    }
  } else {
    const int32_t* id = idx + (int64_t)o * W;
    for (int m = 0; m < W; ++m) {
      const int64_t k = base + (int64_t)id[m] * sa;
      s += cf[m] * (SUB ? in[k] - in2[k] : in[k]);
    }
  }
  const int64_t g = bt * ((int64_t)plane * d.oz) + (int64_t)z * plane + t;
  out[g] = ACC ? out[g] + s : s;
  if (zero) zero[g] = T(0);
}

template <typename T, int AX, bool BWD, bool SUB, bool ACC>
void pass(const T* in, const T* in2, T* out, T* zero, const int od[3], const int id[3],
          const int32_t* idx, const void* coef, int W, int batch, hipStream_t s) {
  const int64_t plane = (int64_t)od[0] * od[1];
  if (plane == 0 || od[2] == 0 || batch == 0) return;
  const Dims d{od[0], od[1], od[2], id[0], id[1]};
  const int64_t n_in = (int64_t)id[0] * id[1] * id[2];
  const dim3 grid((unsigned)((plane + LT - 1) / LT), (unsigned)od[2], (unsigned)batch);
  lattice_pass_kernel<T, AX, BWD, SUB, ACC>
      <<<grid, LT, 0, s>>>(in, in2, out, zero, d, n_in, idx, static_cast<const T*>(coef), W);
  MFSEM_LAUNCH("lattice_pass_kernel");
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

// 1D tables of one axis: forward (per fine node: first coarse node and Pc
// coefficients) and transposed (per coarse node: fine nodes and coefficients).
void build_axis(int kind, int pf, int pc, int nf_elem, const std::vector<double>& I,
                LatticeAxisHost& h) {
  const int Pf = pf + 1, Pc = pc + 1;
  const bool hk = kind == MFSEM_TRANSFER_H;
  h.nf = pf * nf_elem + 1;
  h.nc = pc * (hk ? nf_elem / 2 : nf_elem) + 1;
  h.Wf = Pc;
  h.fstart.assign(h.nf, 0);
  h.fcoef.assign((size_t)h.nf * Pc, 0.0);
  std::vector<std::vector<std::pair<int, double>>> cols(h.nc);
  for (int i = 0; i < h.nf; ++i) {
    const int e = std::min(i / pf, nf_elem - 1), a = i - e * pf;
    const int child = hk ? (e & 1) : 0;
    const int ec = hk ? e / 2 : e;
    h.fstart[i] = ec * pc;
    for (int b = 0; b < Pc; ++b) {
      const double c = I[(size_t)child * Pf * Pc + (size_t)a * Pc + b];
      h.fcoef[(size_t)i * Pc + b] = c;
      if (c != 0.0) cols[ec * pc + b].push_back({i, c});  // exact zeros add nothing
    }
  }
  h.Wb = 1;
  for (const auto& c : cols) h.Wb = std::max<int>(h.Wb, (int)c.size());
  h.bidx.assign((size_t)h.nc * h.Wb, 0);
  h.bcoef.assign((size_t)h.nc * h.Wb, 0.0);
  for (int o = 0; o < h.nc; ++o)
    for (size_t k = 0; k < cols[o].size(); ++k) {
      h.bidx[(size_t)o * h.Wb + k] = cols[o][k].first;
      h.bcoef[(size_t)o * h.Wb + k] = cols[o][k].second;
    }
}

void upload(void* dst, const std::vector<double>& v, size_t word) {
  if (word == sizeof(double)) {
    MFSEM_HIP(hipMemcpy(dst, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice));
  } else {
    const std::vector<float> f(v.begin(), v.end());
    MFSEM_HIP(hipMemcpy(dst, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
  }
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
  for (int d = 0; d < 3; ++d) build_axis(kind, fine.P - 1, coarse.P - 1, fine.lat[d], I, t.host[d]);
  for (int d = 0; d < 3; ++d) {
    const LatticeAxisHost& h = t.host[d];
    t.fstart[d] = a.take_n<int32_t>(h.fstart.size());
    t.fcoef[d] = a.take(h.fcoef.size() * word);
    t.bidx[d] = a.take_n<int32_t>(h.bidx.size());
    t.bcoef[d] = a.take(h.bcoef.size() * word);
  }
  const int64_t nfx = t.host[0].nf, nfy = t.host[1].nf;
  const int64_t ncy = t.host[1].nc, ncz = t.host[2].nc;
  // both directions pass through (nfx, ncy, ncz) in s1 and (nfx, nfy, ncz) in s2
  t.s1 = a.take((size_t)(nfx * ncy * ncz) * batch * word);
  t.s2 = a.take((size_t)(nfx * nfy * ncz) * batch * word);
  t.word = word;
}

void lattice_transfer_upload(const LatticeTransfer& t) {
  for (int d = 0; d < 3; ++d) {
    const LatticeAxisHost& h = t.host[d];
    MFSEM_HIP(hipMemcpy(t.fstart[d], h.fstart.data(), h.fstart.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
    MFSEM_HIP(hipMemcpy(t.bidx[d], h.bidx.data(), h.bidx.size() * sizeof(int32_t),
                        hipMemcpyHostToDevice));
    upload(t.fcoef[d], h.fcoef, t.word);
    upload(t.bcoef[d], h.bcoef, t.word);
  }
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
void lattice_prolong(const LatticeTransfer& t, int batch, const T* xc, T* xf, bool accumulate,
                     T* zero_f, hipStream_t s) {
  const LatticeAxisHost &hx = t.host[0], &hy = t.host[1], &hz = t.host[2];
  T* s1 = static_cast<T*>(t.s1);
  T* s2 = static_cast<T*>(t.s2);
  {
    const int id[3] = {hx.nc, hy.nc, hz.nc}, od[3] = {hx.nf, hy.nc, hz.nc};
    pass<T, 0, false, false, false>(xc, nullptr, s1, nullptr, od, id, t.fstart[0], t.fcoef[0],
                                    hx.Wf, batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nc, hz.nc}, od[3] = {hx.nf, hy.nf, hz.nc};
    pass<T, 1, false, false, false>(s1, nullptr, s2, nullptr, od, id, t.fstart[1], t.fcoef[1],
                                    hy.Wf, batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nf, hz.nc}, od[3] = {hx.nf, hy.nf, hz.nf};
    if (accumulate)
      pass<T, 2, false, false, true>(s2, nullptr, xf, zero_f, od, id, t.fstart[2], t.fcoef[2],
                                     hz.Wf, batch, s);
    else
      pass<T, 2, false, false, false>(s2, nullptr, xf, zero_f, od, id, t.fstart[2], t.fcoef[2],
                                      hz.Wf, batch, s);
  }
}

// transposed passes, z first so that the pass over the full fine lattice
// reads its coefficient rows at a block-uniform coarse z:
// (nfx, nfy, nfz) -> (nfx, nfy, ncz) -> (nfx, ncy, ncz) -> (ncx, ncy, ncz)
template <typename T>
void lattice_restrict(const LatticeTransfer& t, int batch, const T* bf, const T* tf, T* rc,
                      hipStream_t s) {
  const LatticeAxisHost &hx = t.host[0], &hy = t.host[1], &hz = t.host[2];
  T* s1 = static_cast<T*>(t.s1);
  T* s2 = static_cast<T*>(t.s2);
  {
    const int id[3] = {hx.nf, hy.nf, hz.nf}, od[3] = {hx.nf, hy.nf, hz.nc};
    if (tf)
      pass<T, 2, true, true, false>(bf, tf, s2, nullptr, od, id, t.bidx[2], t.bcoef[2], hz.Wb,
                                    batch, s);
    else
      pass<T, 2, true, false, false>(bf, nullptr, s2, nullptr, od, id, t.bidx[2], t.bcoef[2],
                                     hz.Wb, batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nf, hz.nc}, od[3] = {hx.nf, hy.nc, hz.nc};
    pass<T, 1, true, false, false>(s2, nullptr, s1, nullptr, od, id, t.bidx[1], t.bcoef[1], hy.Wb,
                                   batch, s);
  }
  {
    const int id[3] = {hx.nf, hy.nc, hz.nc}, od[3] = {hx.nc, hy.nc, hz.nc};
    pass<T, 0, true, false, false>(s1, nullptr, rc, nullptr, od, id, t.bidx[0], t.bcoef[0], hx.Wb,
                                   batch, s);
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
