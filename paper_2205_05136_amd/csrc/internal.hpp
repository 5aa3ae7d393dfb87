// Internal declarations shared by the HIP translation units of libmfsem.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "mfsem.h"

namespace mfsem {

// node lattices of the placement kernel (mesh.hip)
enum { MFSEM_NODES_REFINE = 0, MFSEM_NODES_DEGREE = 1 };

// ---------------------------------------------------------------- errors ---
void set_error(const std::string& msg);
struct Error {
  mfsem_status code;
  std::string msg;
};
[[noreturn]] void fail(mfsem_status code, const std::string& msg);
void check_hip(hipError_t e, const char* what);
#define MFSEM_HIP(call) ::mfsem::check_hip((call), #call)
#define MFSEM_LAUNCH(what) ::mfsem::check_hip(hipGetLastError(), what)

// ------------------------------------------------------------- workspace ---
// Bump allocator over a caller-provided buffer.  With base == nullptr it only
// measures, so the same layout code sizes and carves a workspace.
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  void* take(size_t bytes) {
    used = (used + 255) & ~size_t(255);
    void* p = base ? base + used : nullptr;
    used += bytes;
    if (base && used > size) fail(MFSEM_EINVAL, "workspace too small");
    return p;
  }
  template <typename T>
  T* take_n(size_t n) { return static_cast<T*>(take(n * sizeof(T))); }
};

// ------------------------------------------------------------ 1D tables ---
// Host-side GLL / Gauss rules and Lagrange matrices used to build the device
// tables (geometry and operator kernels read them from device memory).
void gll_rule(int p, std::vector<double>& x, std::vector<double>& w);
void gauss_rule(int q, std::vector<double>& x, std::vector<double>& w);
// L[k*P + a] = l_a(x_k) and D[k*P + a] = l_a'(x_k) for nodes `nodes`.
void lagrange_matrices(const std::vector<double>& nodes, const std::vector<double>& x,
                       std::vector<double>* L, std::vector<double>* D);

// Device table layout (all row-major), in T = double or float:
//   B  [Q][P]  : nodal basis at the quadrature points (identity for GLL)
//   Db [Q][P]  : nodal basis derivative at the quadrature points
//   Dq [Q][Q]  : collocation derivative on the quadrature points (= Db for GLL)
//   Bm [Q][Pm] : map basis at the quadrature points
//   Dm [Q][Pm] : map basis derivative at the quadrature points
//   w  [Q]     : 1D quadrature weights
//   iw2 [Q]    : 1 / w^2 (the mass weight from det G needs 1/W^2, W = w_a w_b w_c)
struct TableOffsets {
  int B, Db, Dq, Bm, Dm, w, iw2, total;
};
TableOffsets table_offsets(int P, int Q, int Pm);
std::vector<double> build_tables(int p, int quad, int Q, int pm);

// --------------------------------------------------------- launch helpers ---
inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }
inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// Remaps a 1D grid so consecutive logical blocks land on the same XCD (the
// hardware dispatches workgroups round-robin over the 8 XCDs): neighbouring
// elements then share the XCD's L2 for their common nodes.
__device__ inline uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  constexpr uint32_t NX = 8;
  const uint32_t per = nblocks / NX, rem = nblocks % NX;
  const uint32_t x = bid % NX, k = bid / NX;
  // XCD x owns logical blocks [x*per + min(x,rem), ...)
  const uint32_t start = x * per + (x < rem ? x : rem);
  return start + k;
}

template <typename T>
__device__ inline void atomic_add(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// The six stored G entries of one quadrature point are contiguous
// (G[batch][elem][point][6]), 16-byte aligned in FP64: three 16-byte loads
// (three 8-byte loads in FP32) fetch a point, and the lanes of a wave that
// walk consecutive points read one contiguous span.
__device__ inline void load_g6(const double* p, double (&g)[6]) {
  const double2* q = reinterpret_cast<const double2*>(p);
  const double2 a = q[0], b = q[1], c = q[2];
  g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}
__device__ inline void load_g6(const float* p, float (&g)[6]) {
  const float2* q = reinterpret_cast<const float2*>(p);
  const float2 a = q[0], b = q[1], c = q[2];
  g[0] = a.x; g[1] = a.y; g[2] = b.x; g[3] = b.y; g[4] = c.x; g[5] = c.y;
}

}  // namespace mfsem

// ------------------------------------------------------------ op object ---
struct mfsem_op {
  mfsem_op_desc d;      // copy of the descriptor (pointers referenced)
  int P, Q, Pm;         // DOF nodes, quadrature points and map nodes per axis
  int64_t nq3;          // quadrature points per element
  double alpha;
  // device storage inside the caller's workspace
  double* G64 = nullptr;   // [batch][n_elem][Q^3][6]
  double* WJ64 = nullptr;  // [n_elem][Q^3]
  float* G32 = nullptr;
  float* WJ32 = nullptr;
  double* tab64 = nullptr; // 1D tables
  float* tab32 = nullptr;
  // 1/det(sigma_e) per member and element: the apply recovers W|J| at a point
  // from det G = (W|J|)^3 |J|^{-2} det(sigma) = W^3 |J| det(sigma), so the mass
  // term needs no stored W|J| (used when every det(sigma_e) > 0)
  double* idet64 = nullptr;  // [batch][n_elem]
  float* idet32 = nullptr;
  bool use_det = false;
  // structured lattice (elements per axis) when elem_dof follows the box numbering
  bool structured = false;
  int lat[3] = {0, 0, 0};
  // the FP64 stiffness apply rebuilds G from map_xyz, fiber and sigma
  bool otf = false;
  // [0]: first failing (element, point) of the geometry; [1]: elements with
  // det(sigma) <= 0; [2]: element nodes that differ from the structured numbering
  unsigned long long* bad = nullptr;
  double* sigma_copy = nullptr;       // [batch][n_elem][3] (kept for set_sigma / grad)
  mfsem::TableOffsets off;
  std::vector<double> tab_host;
  std::vector<float> tab_host32;
};

namespace mfsem {

// Layout of an operator's workspace (used for sizing and carving).
void op_layout(mfsem_op& op, Arena& a);
void run_geometry(mfsem_op& op, hipStream_t s);  // fills G/WJ and the bad flag

// y = A x, or y += A x with accumulate (the kernels add into y; without
// accumulate y is cleared first)
template <typename T>
void launch_apply(const mfsem_op& op, const T* x, T* y, double alpha, bool stiffness,
                  hipStream_t s, bool accumulate = false);
template <typename T>
void launch_diag(const mfsem_op& op, T* d, hipStream_t s);
// brick kernel on structured lattices, adding into y (returns false when it
// does not apply)
template <typename T>
bool launch_brick(const mfsem_op& op, const T* G, const T* WJ, const T* idet, const T* tab,
                  const T* x, T* y, T alpha, hipStream_t s);
void launch_lattice_check(const mfsem_op& op, unsigned long long* bad, hipStream_t s);
void launch_grad_sigma(const mfsem_op& op, const double* u, const double* w, double scale,
                       double* g, hipStream_t s);
// matrix-based path on structured lattices (csr.hip)
int64_t csr_nnz(const mfsem_op& op, bool coupled);
void csr_assemble(const mfsem_op& op, bool coupled, int64_t* row_ptr, int32_t* col, double* val,
                  hipStream_t s);
void csr_spmv(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col, const double* val,
              const double* x, double* y, hipStream_t s);

// vector kernels (vec.hip)
template <typename T>
void vfill(T* x, int64_t n, T v, hipStream_t s);
template <typename A, typename B>
void vcast(const A* x, B* y, int64_t n, hipStream_t s);

}  // namespace mfsem
