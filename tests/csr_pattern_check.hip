// The CSR patterns of the assembled matrix (row offsets, columns, and the slot
// the values kernel adds each element-matrix entry into), run on the host with
// the same functions the kernels call, against brute-force enumeration.
#include "csr.hip"
#include <cstdio>
#include <vector>
#include <set>
using namespace mfsem;
int main() {
  int bad = 0;
  for (int p = 1; p <= 8; ++p)
    for (int nx = 1; nx <= 4; ++nx)
      for (int ny = 1; ny <= 3; ++ny)
        for (int nz = 1; nz <= 3; ++nz)
          for (int cp = 0; cp < 2; ++cp) {
            if (p > 4 && nx * ny * nz > 6) continue;
            mfsem_op op{};
            op.d.p = p;
            op.lat[0] = nx; op.lat[1] = ny; op.lat[2] = nz;
            const Lattice L = lattice_of(op, cp);
            const int64_t NX = L.x.N, NY = L.y.N, NZ = L.z.N, n = NX * NY * NZ;
            const int64_t nnz = csr_nnz(op, cp);
            std::vector<int64_t> rp(n + 1, -7);
            std::vector<int32_t> col(nnz + 16, -7);
            for (int64_t g = 0; g < n; ++g)
              for (int lane = 0; lane < 64; ++lane) pattern_row(L, n, g, lane, 64, rp.data(), col.data());
            // brute force: the rows' column sets
            int64_t at = 0;
            for (int64_t g = 0; g < n; ++g) {
              const int64_t I = g % NX, J = (g / NX) % NY, K = g / (NX * NY);
              std::vector<int64_t> want;
              for (int64_t kc = 0; kc < NZ; ++kc)
                for (int64_t jc = 0; jc < NY; ++jc)
                  for (int64_t ic = 0; ic < NX; ++ic) {
                    // share an element: along each axis in a common element interval
                    auto share = [&](int64_t a, int64_t b, int64_t N) {
                      for (int64_t e = 0; e * p < N - 1; ++e)
                        if (a >= e * p && a <= e * p + p && b >= e * p && b <= e * p + p) return true;
                      return N == 1;
                    };
                    if (!share(I, ic, NX) || !share(J, jc, NY) || !share(K, kc, NZ)) continue;
                    if (cp && ic != I && jc != J && kc != K) continue;
                    want.push_back(ic + NX * (jc + NY * kc));
                  }
              if (rp[g] != at) { if (bad++ < 10) printf("p%d %d%d%d cp%d row %ld start %ld want %ld\n", p, nx, ny, nz, cp, (long)g, (long)rp[g], (long)at); }
              for (size_t t = 0; t < want.size(); ++t)
                if (col[at + t] != want[t]) { if (bad++ < 10) printf("p%d cp%d row %ld col %zu %d want %ld\n", p, cp, (long)g, t, col[at + t], (long)want[t]); break; }
              at += want.size();
            }
            if (rp[n] != at || at != nnz) { if (bad++ < 10) printf("p%d %d%d%d cp%d end %ld nnz %ld want %ld\n", p, nx, ny, nz, cp, (long)rp[n], (long)nnz, (long)at); }
            for (int64_t t = nnz; t < nnz + 16; ++t) if (col[t] != -7) { bad++; printf("overrun\\n"); break; }
            // the values kernel's slot of every element pair (sharing a local index when coupled)
            const int P = p + 1;
            for (int64_t ez = 0; ez < nz; ++ez) for (int64_t ey = 0; ey < ny; ++ey) for (int64_t ex = 0; ex < nx; ++ex)
              for (int i = 0; i < P * P * P; ++i) for (int j = 0; j < P * P * P; ++j) {
                const int ia = i % P, ib = (i / P) % P, ic = i / (P * P);
                const int ja = j % P, jb = (j / P) % P, jc = j / (P * P);
                if (cp && ia != ja && ib != jb && ic != jc) continue;
                const int64_t I = ex * p + ia, J = ey * p + ib, K = ez * p + ic;
                const int64_t Ic = ex * p + ja, Jc = ey * p + jb, Kc = ez * p + jc;
                int64_t lx, rx, ly, ry, lz, rz;
                axis_range(L.x, I, lx, rx); axis_range(L.y, J, ly, ry); axis_range(L.z, K, lz, rz);
                const int64_t g = I + NX * (J + NY * K);
                const int64_t pos = row_start(L, I, J, K) + col_slot(L, I, J, K, lx, rx, ly, ry, lz, Ic, Jc, Kc);
                if (pos < rp[g] || pos >= rp[g + 1] || col[pos] != Ic + NX * (Jc + NY * Kc)) {
                  if (bad++ < 10) printf("slot p%d cp%d g %ld pos %ld\n", p, cp, (long)g, (long)pos);
                }
              }
          }
  // the c2 slab at p = 4 against the oracle's count of non-zeros
  mfsem_op op{}; op.d.p = 4; op.lat[0] = 40; op.lat[1] = 14; op.lat[2] = 6;
  printf("c2 p4: element %ld coupled %ld\n", (long)csr_nnz(op, false), (long)csr_nnz(op, true));
  printf("%s (%d mismatches)\n", bad ? "FAIL" : "OK", bad);
  return bad != 0;
}
