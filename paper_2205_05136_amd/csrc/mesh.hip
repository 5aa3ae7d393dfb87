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

void launch_box_parents(const int32_t n[3], int32_t* parent, int8_t* child, hipStream_t s) {
  const int64_t ne = (int64_t)n[0] * n[1] * n[2];
  box_parent_kernel<<<grid(ne), 256, 0, s>>>(n[0], n[1], ne, parent, child);
  MFSEM_LAUNCH("box_parent_kernel");
}

}  // namespace mfsem
