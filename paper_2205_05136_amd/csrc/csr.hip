// Matrix-based path: the assembled sparse matrix of A = alpha M + K in CSR and
// its product with a vector (the paper's matrix-based comparison: the global
// matrix assembled from the element matrices, Alg. 2, then sparse
// matrix-vector products inside CG, Section 4).
//
// Structured lattices only.  The pattern is the element connectivity: node
// (I, J, K) couples to every node of every element containing it, i.e. along
// each axis to [lo, hi] with
//     lo = I - (I mod p), hi = lo + p                  (I inside an element)
//     lo = max(I - p, 0), hi = min(I + p, N - 1)       (I on an element face)
// so a row holds rx * ry * rz entries (up to (2p+1)^3), in increasing global
// index.  Row offsets follow in closed form from the 1D prefix sums of r.
// Entries that vanish for GLL collocation (i and j in different rows of all
// three axes) stay in the pattern as zeros, as in a standard assembly of full
// element matrices.
//
// The coupled pattern keeps only the pairs that collocation can make non-zero:
// the nodes of that box that share at least one lattice coordinate with the
// row's node (every pair of them lies in a common element, and there the two
// share a local index, so one of the 1D derivative products is not a zero
// delta).  A row then holds rx ry rz - (rx-1)(ry-1)(rz-1) entries (on a
// 40 x 14 x 6 lattice 0.43 of the element pattern's at p = 4, 0.30 at p = 7),
// still in increasing global index, and its offset is the element pattern's
// minus the same prefix sums taken over the extents r - 1.
#include "internal.hpp"

namespace mfsem {

namespace {

struct Axis {
  int p;
  int64_t N;  // nodes along the axis
};

__host__ __device__ inline void axis_range(const Axis& a, int64_t I, int64_t& lo, int64_t& r) {
  if (I % a.p == 0) {
    lo = I - a.p > 0 ? I - a.p : 0;
    const int64_t hi = I + a.p < a.N - 1 ? I + a.p : a.N - 1;
    r = hi - lo + 1;
  } else {
    lo = I - I % a.p;
    r = a.p + 1;
  }
}

// sum of the row extents r(I') over I' < I (0 <= I <= N): interior nodes
// have p + 1, the two end nodes p + 1, the other multiples of p 2p + 1
__host__ __device__ inline int64_t axis_prefix(const Axis& a, int64_t I) {
  const int64_t m = (I + a.p - 1) / a.p;  // multiples of p in [0, I)
  const int64_t ends = (I > 0 ? 1 : 0) + (I > a.N - 1 ? 1 : 0);
  return (I - m) * (a.p + 1) + (m - ends) * (2 * a.p + 1) + ends * (a.p + 1);
}

// sum of r(I') - 1 over I' < I
__host__ __device__ inline int64_t axis_prefix1(const Axis& a, int64_t I) {
  return axis_prefix(a, I) - I;
}

struct Lattice {
  Axis x, y, z;
  int64_t Tx, Ty;  // axis_prefix(N) of x and y
  bool coupled;    // the coupled pattern (else the element pattern)
};

__host__ __device__ inline int64_t row_len(const Lattice& L, int64_t rx, int64_t ry, int64_t rz) {
  return L.coupled ? rx * ry * rz - (rx - 1) * (ry - 1) * (rz - 1) : rx * ry * rz;
}

__host__ __device__ inline int64_t row_start(const Lattice& L, int64_t I, int64_t J, int64_t K) {
  int64_t lo, ry, rz;
  axis_range(L.y, J, lo, ry);
  axis_range(L.z, K, lo, rz);
  const int64_t full = axis_prefix(L.z, K) * L.Tx * L.Ty +
                       rz * (axis_prefix(L.y, J) * L.Tx + ry * axis_prefix(L.x, I));
  if (!L.coupled) return full;
  const int64_t Tx1 = L.Tx - L.x.N, Ty1 = L.Ty - L.y.N;
  return full - (axis_prefix1(L.z, K) * Tx1 * Ty1 +
                 (rz - 1) * (axis_prefix1(L.y, J) * Tx1 + (ry - 1) * axis_prefix1(L.x, I)));
}

// slot of column node (Ic, Jc, Kc) in the row of node (I, J, K), whose box is
// [lx, lx + rx) x [ly, ly + ry) x [lz, lz + rz); in the coupled pattern the
// column must share a coordinate with the row (planes of the box other than
// K hold row J and the single node at I of every other row)
__host__ __device__ inline int64_t col_slot(const Lattice& L, int64_t I, int64_t J, int64_t K,
                                            int64_t lx, int64_t rx, int64_t ly, int64_t ry,
                                            int64_t lz, int64_t Ic, int64_t Jc, int64_t Kc) {
  if (!L.coupled) return ((Kc - lz) * ry + (Jc - ly)) * rx + (Ic - lx);
  const int64_t plane = rx + ry - 1;
  int64_t s = (Kc - lz) * plane + (K < Kc ? rx * ry - plane : 0);
  s += Kc == K ? (Jc - ly) * rx : (Jc - ly) + (J < Jc ? rx - 1 : 0);
  return s + (Kc == K || Jc == J ? Ic - lx : 0);
}

constexpr int CT = 256;  // threads per block; one wave of 64 lanes per row

// Row g of the pattern (its offset, and its columns t = lane, lane + nl, ...
// of the row's work: entries of the element pattern, x-rows of the box in the
// coupled one); the last row also writes row_ptr[n_rows].
__host__ __device__ inline void pattern_row(const Lattice& L, int64_t n_rows, int64_t g, int lane,
                                            int nl, int64_t* __restrict__ row_ptr,
                                            int32_t* __restrict__ col) {
  const int64_t NX = L.x.N, NY = L.y.N;
  const int64_t I = g % NX, J = (g / NX) % NY, K = g / (NX * NY);
  int64_t lx, rx, ly, ry, lz, rz;
  axis_range(L.x, I, lx, rx);
  axis_range(L.y, J, ly, ry);
  axis_range(L.z, K, lz, rz);
  const int64_t start = row_start(L, I, J, K);
  if (lane == 0) {
    row_ptr[g] = start;
    if (g == n_rows - 1) row_ptr[n_rows] = start + row_len(L, rx, ry, rz);
  }
  if (!L.coupled) {
    for (int64_t t = lane; t < rx * ry * rz; t += nl) {
      const int64_t ic = lx + t % rx, jc = ly + (t / rx) % ry, kc = lz + t / (rx * ry);
      col[start + t] = (int32_t)(ic + NX * (jc + NY * kc));
    }
  } else {
    // one lane per x-row of the box: all of it in row J or plane K, else the
    // node at I
    for (int64_t t = lane; t < ry * rz; t += nl) {
      const int64_t jc = ly + t % ry, kc = lz + t / ry;
      const bool whole = jc == J || kc == K;
      const int64_t at = start + col_slot(L, I, J, K, lx, rx, ly, ry, lz, whole ? lx : I, jc, kc);
      const int64_t base = NX * (jc + NY * kc);
      if (whole)
        for (int64_t a = 0; a < rx; ++a) col[at + a] = (int32_t)(lx + a + base);
      else
        col[at] = (int32_t)(I + base);
    }
  }
}

__global__ __launch_bounds__(CT) void csr_pattern_kernel(Lattice L, int64_t n_rows,
                                                         int64_t* __restrict__ row_ptr,
                                                         int32_t* __restrict__ col) {
  const int lane = threadIdx.x & 63;
  for (int64_t g = ((int64_t)blockIdx.x * CT + threadIdx.x) >> 6; g < n_rows;
       g += ((int64_t)gridDim.x * CT) >> 6)
    pattern_row(L, n_rows, g, lane, 64, row_ptr, col);
}

// One workgroup per element: every entry (i, j) of the element matrix
//   A_e[i][j] = alpha W|J|_i delta_ij + sum_q grad phi_i(q)^T G_q grad phi_j(q)
// from the stored G (GLL points = nodes, so grad phi_i is non-zero only at the
// points in the three lines through node i), added into the row of node i.
__global__ __launch_bounds__(CT) void csr_values_kernel(Lattice L, int P, const double* __restrict__ G,
                                                        const double* __restrict__ WJ, double alpha,
                                                        const double* __restrict__ Db,
                                                        int nex, int ney, double* __restrict__ val) {
  __shared__ double sD[(MFSEM_MAX_P + 1) * (MFSEM_MAX_P + 1)];
  const int64_t e = blockIdx.x;
  const int p = P - 1, P2 = P * P, P3 = P2 * P;
  for (int i = threadIdx.x; i < P2; i += CT) sD[i] = Db[i];
  __syncthreads();
  const int64_t ex = e % nex, ey = (e / nex) % ney, ez = e / ((int64_t)nex * ney);
  const double* Ge = G + e * P3 * 6;
  const int64_t NX = L.x.N, NY = L.y.N;
  auto Gc = [&](int qa, int qb, int qc, int comp) { return Ge[(qa + P * (qb + P * qc)) * 6 + comp]; };
  auto D = [&](int q, int m) { return sD[q * P + m]; };  // l_m'(x_q)
  for (int t = threadIdx.x; t < P3 * P3; t += CT) {
    const int i = t / P3, j = t % P3;
    const int ia = i % P, ib = (i / P) % P, ic = i / P2;
    const int ja = j % P, jb = (j / P) % P, jc = j / P2;
    const bool sa = ia == ja, sb = ib == jb, sc = ic == jc;
    if (!sa && !sb && !sc) continue;  // no common line: structurally zero
    double v = 0.0;
    if (sb && sc)
      for (int a = 0; a < P; ++a) v += D(a, ia) * D(a, ja) * Gc(a, ib, ic, 0);
    if (sa && sc)
      for (int b = 0; b < P; ++b) v += D(b, ib) * D(b, jb) * Gc(ia, b, ic, 3);
    if (sa && sb)
      for (int c = 0; c < P; ++c) v += D(c, ic) * D(c, jc) * Gc(ia, ib, c, 5);
    if (sc) {  // x-y couplings
      v += D(ja, ia) * D(ib, jb) * Gc(ja, ib, ic, 1);
      v += D(jb, ib) * D(ia, ja) * Gc(ia, jb, ic, 1);
    }
    if (sb) {  // x-z couplings
      v += D(ja, ia) * D(ic, jc) * Gc(ja, ib, ic, 2);
      v += D(jc, ic) * D(ia, ja) * Gc(ia, ib, jc, 2);
    }
    if (sa) {  // y-z couplings
      v += D(jb, ib) * D(ic, jc) * Gc(ia, jb, ic, 4);
      v += D(jc, ic) * D(ib, jb) * Gc(ia, ib, jc, 4);
    }
    if (i == j) v += alpha * WJ[e * P3 + i];
    // global node of i (row) and j (column), and the column's slot in the row
    const int64_t I = ex * p + ia, J = ey * p + ib, K = ez * p + ic;
    const int64_t Ic = ex * p + ja, Jc = ey * p + jb, Kc = ez * p + jc;
    int64_t lx, rx, ly, ry, lz, rz;
    axis_range(L.x, I, lx, rx);
    axis_range(L.y, J, ly, ry);
    axis_range(L.z, K, lz, rz);
    const int64_t pos =
        row_start(L, I, J, K) + col_slot(L, I, J, K, lx, rx, ly, ry, lz, Ic, Jc, Kc);
    (void)NX;
    (void)NY;
    atomic_add(&val[pos], v);
  }
}

// LPR lanes per row (a power of two dividing 64), so that 64 / LPR rows share a
// wave and their row-offset, column and x loads overlap; each lane keeps four
// independent partial sums so that several loads are in flight.  Measured on
// the c2 slab: 16 lanes are fastest up to ~200 entries per row (p <= 4), 32
// above; one wave per row is 12-38% slower, non-temporal loads 10-60% slower.
template <int LPR>
__global__ __launch_bounds__(CT) void csr_spmv_kernel(int64_t n_rows, const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ y) {
  const int lane = threadIdx.x & (LPR - 1);
  const int64_t rows_per_grid = ((int64_t)gridDim.x * CT) / LPR;
  for (int64_t g = ((int64_t)blockIdx.x * CT + threadIdx.x) / LPR; g < n_rows; g += rows_per_grid) {
    const int64_t a = row_ptr[g], b = row_ptr[g + 1];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t k = a + lane;
    for (; k + 3 * LPR < b; k += 4 * LPR) {
      const double v0 = val[k];
      const double v1 = val[k + LPR];
      const double v2 = val[k + 2 * LPR];
      const double v3 = val[k + 3 * LPR];
      const int32_t c0 = col[k];
      const int32_t c1 = col[k + LPR];
      const int32_t c2 = col[k + 2 * LPR];
      const int32_t c3 = col[k + 3 * LPR];
      s0 += v0 * x[c0];
      s1 += v1 * x[c1];
      s2 += v2 * x[c2];
      s3 += v3 * x[c3];
    }
    for (; k < b; k += LPR) s0 += val[k] * x[col[k]];
    double s = (s0 + s1) + (s2 + s3);
    for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_down(s, o, LPR);
    if (lane == 0) y[g] = s;
  }
}

Lattice lattice_of(const mfsem_op& op, bool coupled) {
  const int p = op.d.p;
  Lattice L;
  L.coupled = coupled;
  L.x = Axis{p, (int64_t)p * op.lat[0] + 1};
  L.y = Axis{p, (int64_t)p * op.lat[1] + 1};
  L.z = Axis{p, (int64_t)p * op.lat[2] + 1};
  L.Tx = axis_prefix(L.x, L.x.N);
  L.Ty = axis_prefix(L.y, L.y.N);
  return L;
}

unsigned row_blocks(int64_t rows, int lanes_per_row = 64) {
  int64_t b = (rows * lanes_per_row + CT - 1) / CT;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int64_t csr_nnz(const mfsem_op& op, bool coupled) {
  const Lattice L = lattice_of(op, coupled);
  const int64_t Tz = axis_prefix(L.z, L.z.N);
  const int64_t full = L.Tx * L.Ty * Tz;
  return coupled ? full - (L.Tx - L.x.N) * (L.Ty - L.y.N) * (Tz - L.z.N) : full;
}

void csr_assemble(const mfsem_op& op, bool coupled, int64_t* row_ptr, int32_t* col, double* val,
                  hipStream_t s) {
  const Lattice L = lattice_of(op, coupled);
  const int64_t n = op.d.n_dof, nnz = csr_nnz(op, coupled);
  csr_pattern_kernel<<<row_blocks(n), CT, 0, s>>>(L, n, row_ptr, col);
  MFSEM_LAUNCH("csr_pattern_kernel");
  vfill<double>(val, nnz, 0.0, s);
  if (op.d.n_elem == 0) return;
  csr_values_kernel<<<(unsigned)op.d.n_elem, CT, 0, s>>>(
      L, op.P, op.G64, op.WJ64, op.alpha, op.tab64 + op.off.Db, op.lat[0], op.lat[1], val);
  MFSEM_LAUNCH("csr_values_kernel");
}

void csr_spmv(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const double* val,
              const double* x, double* y, hipStream_t s) {
  if (n <= 0) return;
  const int64_t mean = nnz / n;  // lanes per row from the mean row length
  if (mean <= 256) {
    csr_spmv_kernel<16><<<row_blocks(n, 16), CT, 0, s>>>(n, row_ptr, col, val, x, y);
  } else {
    csr_spmv_kernel<32><<<row_blocks(n, 32), CT, 0, s>>>(n, row_ptr, col, val, x, y);
  }
  MFSEM_LAUNCH("csr_spmv_kernel");
}

}  // namespace mfsem
