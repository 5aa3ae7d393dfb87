// Structured box meshes of degree p (Section 3: conforming hexahedral meshes
// and the continuous Q_p space with nodes at the GLL points of each element).
//
// Global node (I, J, K) of the (p n0 + 1) x (p n1 + 1) x (p n2 + 1) lattice has
// index I + NX (J + NY K); inside element (ex, ey, ez) local node (a, b, c) is
// global (p ex + a, p ey + b, p ez + c).  Coordinates put the GLL points on
// each element edge; an optional shear moves every node by the same
// d = amp * hx * sin(2 pi (x - x0)/Lx) in all three coordinates, and an
// optional fiber rotates in the xy-plane linearly with the undeformed z.
#include <cmath>
#include <vector>

#include "internal.hpp"

namespace mfsem {

namespace {

struct BoxArgs {
  int p, n0, n1, n2;
  double x0, y0, z0, Lx, Ly, Lz, amp, th0, th1;
  int fiber;
  double xi[MFSEM_MAX_P + 1];  // GLL points of degree p
};

__global__ void box_nodes_kernel(BoxArgs a, int64_t n_dof, double* __restrict__ xyz,
                                 double* __restrict__ fib) {
  const int64_t NX = (int64_t)a.p * a.n0 + 1, NY = (int64_t)a.p * a.n1 + 1;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; g < n_dof; g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t I = g % NX, r = g / NX, J = r % NY, K = r / NY;
    auto coord = [&](int64_t idx, int n, double o, double L) {
      int64_t e = idx / a.p;
      if (e >= n) e = n - 1;
      const int loc = (int)(idx - e * a.p);
      return o + (L / n) * ((double)e + 0.5 * (a.xi[loc] + 1.0));
    };
    const double x = coord(I, a.n0, a.x0, a.Lx);
    const double y = coord(J, a.n1, a.y0, a.Ly);
    const double z = coord(K, a.n2, a.z0, a.Lz);
    double d = 0.0;
    if (a.amp != 0.0) d = a.amp * (a.Lx / a.n0) * sin(2.0 * M_PI * (x - a.x0) / a.Lx);
    xyz[g * 3 + 0] = x + d;
    xyz[g * 3 + 1] = y + d;
    xyz[g * 3 + 2] = z + d;
    if (a.fiber) {
      const double th = a.th0 + (a.th1 - a.th0) * (z - a.z0) / a.Lz;
      fib[g * 3 + 0] = cos(th);
      fib[g * 3 + 1] = sin(th);
      fib[g * 3 + 2] = 0.0;
    }
  }
}

__global__ void box_elems_kernel(int p, int n0, int n1, int64_t n_elem, int32_t* __restrict__ ed) {
  const int P = p + 1, P3 = P * P * P;
  const int64_t NX = (int64_t)p * n0 + 1, NY = (int64_t)p * n1 + 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; t < n_elem * P3; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / P3;
    const int l = (int)(t % P3);
    const int aa = l % P, b = (l / P) % P, c = l / (P * P);
    const int64_t ex = e % n0, ey = (e / n0) % n1, ez = e / ((int64_t)n0 * n1);
    ed[t] = (int32_t)((p * ex + aa) + NX * ((p * ey + b) + NY * (p * ez + c)));
  }
}

__global__ void box_parent_kernel(int n0, int n1, int64_t n_elem, int32_t* __restrict__ parent,
                                  int8_t* __restrict__ child) {
  const int c0 = n0 / 2, c1 = n1 / 2;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; e < n_elem; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ex = e % n0, ey = (e / n0) % n1, ez = e / ((int64_t)n0 * n1);
    parent[e] = (int32_t)(ex / 2 + c0 * (ey / 2 + (int64_t)c1 * (ez / 2)));
    child[e] = (int8_t)((ex & 1) | ((ey & 1) << 1) | ((ez & 1) << 2));
  }
}

// Nodes of a derived mesh placed by the parent's isoparametric map (Section
// 4.3: the octree children of a coarse mesh and its lower-degree levels keep
// the parent's geometry).  New node g lies at lattice point loc[g] = I + M (J +
// M K) of element elem[g]'s M^3 reference lattice; with L[I][a] the degree-p
// Lagrange basis on the GLL nodes at the lattice's 1D points,
//   X = sum_{a,b,c} L[I][a] L[J][b] L[K][c] X_parent[elem_dof[e][a + P (b + P c)]],
// and the fiber the same way (the operator normalises it where it uses it).
// Out-of-range element, lattice or node indices give NaN (no access is made).
struct PlaceArgs {
  int P, M;                                              // parent nodes per axis, lattice points
  double L[(2 * MFSEM_MAX_P + 1) * (MFSEM_MAX_P + 1)];   // [M][P]
};

__global__ void place_nodes_kernel(PlaceArgs a, int64_t n_elem, const int32_t* __restrict__ ed,
                                   int64_t n_nodes, const double* __restrict__ xyz,
                                   const double* __restrict__ fib, int64_t n_new,
                                   const int32_t* __restrict__ elem, const int32_t* __restrict__ loc,
                                   double* __restrict__ xyz_out, double* __restrict__ fib_out) {
  const int P = a.P, M = a.M, P3 = P * P * P;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_new;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = elem[g];
    const int l = loc[g];
    bool ok = e >= 0 && e < n_elem && l >= 0 && l < M * M * M;
    double X[3] = {0, 0, 0}, F[3] = {0, 0, 0};
    if (ok) {
      const int I = l % M, J = (l / M) % M, K = l / (M * M);
      const int32_t* en = ed + e * P3;
      for (int c = 0; c < P && ok; ++c) {
        const double lc = a.L[K * P + c];
        for (int b = 0; b < P && ok; ++b) {
          const double lbc = a.L[J * P + b] * lc;
          for (int aa = 0; aa < P; ++aa) {
            const int64_t n = en[aa + P * (b + P * c)];
            if (n < 0 || n >= n_nodes) { ok = false; break; }
            const double w = a.L[I * P + aa] * lbc;
            X[0] += w * xyz[3 * n];
            X[1] += w * xyz[3 * n + 1];
            X[2] += w * xyz[3 * n + 2];
            if (fib) {
              F[0] += w * fib[3 * n];
              F[1] += w * fib[3 * n + 1];
              F[2] += w * fib[3 * n + 2];
            }
          }
        }
      }
    }
    const double nan = __builtin_nan("");
    for (int r = 0; r < 3; ++r) {
      xyz_out[3 * g + r] = ok ? X[r] : nan;
      if (fib_out) fib_out[3 * g + r] = ok ? F[r] : nan;
    }
  }
}

unsigned grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

void launch_box(const mfsem_box_desc& d, int64_t n_elem, int64_t n_dof, const double* xi_host,
                int32_t* ed, double* xyz, double* fib, hipStream_t s) {
  BoxArgs a;
  a.p = d.p;
  a.n0 = d.n[0];
  a.n1 = d.n[1];
  a.n2 = d.n[2];
  a.x0 = d.origin[0];
  a.y0 = d.origin[1];
  a.z0 = d.origin[2];
  a.Lx = d.length[0];
  a.Ly = d.length[1];
  a.Lz = d.length[2];
  a.amp = d.shear_amp;
  a.th0 = d.theta0;
  a.th1 = d.theta1;
  a.fiber = d.fiber;
  for (int i = 0; i <= d.p; ++i) a.xi[i] = xi_host[i];
  box_nodes_kernel<<<grid(n_dof), 256, 0, s>>>(a, n_dof, xyz, fib);
  MFSEM_LAUNCH("box_nodes_kernel");
  const int P3 = (d.p + 1) * (d.p + 1) * (d.p + 1);
  box_elems_kernel<<<grid(n_elem * P3), 256, 0, s>>>(d.p, d.n[0], d.n[1], n_elem, ed);
  MFSEM_LAUNCH("box_elems_kernel");
}

void launch_place_nodes(int p, int kind, int pc, int64_t n_elem, const int32_t* ed,
                        int64_t n_nodes, const double* xyz, const double* fib, int64_t n_new,
                        const int32_t* elem, const int32_t* loc, double* xyz_out,
                        double* fib_out, hipStream_t s) {
  std::vector<double> nodes, w, pts;
  gll_rule(p, nodes, w);
  if (kind == MFSEM_NODES_REFINE) {
    // the GLL points of the two halves of [-1, 1] (the children's nodes), 2p + 1 in all
    for (int i = 0; i < p; ++i) pts.push_back(0.5 * (nodes[i] - 1.0));
    for (int i = 0; i <= p; ++i) pts.push_back(0.5 * (nodes[i] + 1.0));
  } else {
    std::vector<double> wc;
    gll_rule(pc, pts, wc);
  }
  std::vector<double> L;
  lagrange_matrices(nodes, pts, &L, nullptr);
  PlaceArgs a;
  a.P = p + 1;
  a.M = (int)pts.size();
  for (size_t i = 0; i < L.size(); ++i) a.L[i] = L[i];
  if (n_new == 0) return;
  place_nodes_kernel<<<grid(n_new), 256, 0, s>>>(a, n_elem, ed, n_nodes, xyz, fib, n_new, elem,
                                                 loc, xyz_out, fib_out);
  MFSEM_LAUNCH("place_nodes_kernel");
}

void launch_box_parents(const int32_t n[3], int32_t* parent, int8_t* child, hipStream_t s) {
  const int64_t ne = (int64_t)n[0] * n[1] * n[2];
  box_parent_kernel<<<grid(ne), 256, 0, s>>>(n[0], n[1], ne, parent, child);
  MFSEM_LAUNCH("box_parent_kernel");
}

}  // namespace mfsem
