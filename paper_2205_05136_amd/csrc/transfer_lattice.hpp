// Inter-level transfers between structured lattices as three 1D passes.
#pragma once

#include <vector>

#include "transfer.hpp"

namespace mfsem {

// Node counts of the fine and coarse lattices along one axis.
struct LatticeAxisHost {
  int nf = 0, nc = 0;
};

// Dense 1D interpolation of one coarse element along an axis, [F+1][pc1]: row a
// is the coarse basis at the a-th fine node of the element (F = p_f fine
// intervals per coarse element for a p-transfer, 2p for an h-transfer), passed
// to the element-block kernels by value.
template <typename T>
struct ElemMat {
  int ne = 0, F = 0, pc1 = 0;  // coarse elements, fine intervals per element, coarse nodes per element
  T M[(2 * MFSEM_MAX_P + 1) * (MFSEM_MAX_P + 1)] = {};
};

struct LatticeTransfer {
  LatticeAxisHost host[3];
  ElemMat<double> em64[3];
  ElemMat<float> em32[3];
  void* s1 = nullptr;  // intermediate lattices of the passes
  void* s2 = nullptr;
  size_t word = sizeof(double);
};

// Both levels are structured lattices related by the transfer kind (the same
// lattice for p, the fine lattice twice the coarse one along every axis for h).
// For h the parent/child arrays must also follow the box convention, which
// the caller checks with launch_box_parents_check.
bool lattice_transfer_applies(const mfsem_op& fine, const mfsem_op& coarse, int kind);
// Builds the element matrices and carves the intermediate lattices out of the
// arena (null pointers when sizing).
void lattice_transfer_layout(LatticeTransfer& t, const mfsem_op& fine, const mfsem_op& coarse,
                             int kind, int batch, size_t word, Arena& a);
// Adds to *mismatch the fine elements whose parent/child differ from the box
// convention (parent = the element of (ex/2, ey/2, ez/2) on the coarse lattice,
// child bits = ex & 1, ey & 1, ez & 1).
void launch_box_parents_check(const int32_t n_fine[3], const int32_t* parent,
                              const int8_t* child, unsigned long long* mismatch, hipStream_t s);

// Adds to *bad the fine elements whose parent is outside [0, n_coarse) or whose
// child index is outside 0..7.
void launch_parents_range_check(int64_t n_fine, int64_t n_coarse, const int32_t* parent,
                                const int8_t* child, unsigned long long* bad, hipStream_t s);

// xf = P xc, or xf += P xc with accumulate; with zero_f, zero_f[i] = 0 at
// every fine node as well.
template <typename T>
void lattice_prolong(const LatticeTransfer& t, int batch, const T* xc, T* xf, bool accumulate,
                     T* zero_f, hipStream_t s);
// rc = P^T (bf - tf) (tf may be null); rc is overwritten.
template <typename T>
void lattice_restrict(const LatticeTransfer& t, int batch, const T* bf, const T* tf, T* rc,
                      hipStream_t s);

}  // namespace mfsem
