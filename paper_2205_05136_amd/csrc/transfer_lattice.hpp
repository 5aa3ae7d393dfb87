// Inter-level transfers between structured lattices as three 1D passes.
#pragma once

#include <vector>

#include "transfer.hpp"

namespace mfsem {

// 1D transfer along one axis: fine node i takes sum_b fcoef[i][b] coarse[fstart[i] + b]
// (Wf = Pc terms); the transpose, per coarse node o, is sum_k bcoef[o][k] fine[bidx[o][k]]
// (Wb terms, zero-padded).
struct LatticeAxisHost {
  int nf = 0, nc = 0;  // fine and coarse nodes along the axis
  int Wf = 0, Wb = 0;
  std::vector<int32_t> fstart, bidx;
  std::vector<double> fcoef, bcoef;
};

struct LatticeTransfer {
  LatticeAxisHost host[3];
  int32_t* fstart[3] = {nullptr, nullptr, nullptr};
  int32_t* bidx[3] = {nullptr, nullptr, nullptr};
  void* fcoef[3] = {nullptr, nullptr, nullptr};
  void* bcoef[3] = {nullptr, nullptr, nullptr};
  void* s1 = nullptr;  // intermediate lattices of the passes
  void* s2 = nullptr;
  size_t word = sizeof(double);
};

// Both levels are structured lattices related by the transfer kind (the same
// lattice for p, the fine lattice twice the coarse one along every axis for h).
// For h the parent/child arrays must also follow the box convention, which
// the caller checks with launch_box_parents_check.
bool lattice_transfer_applies(const mfsem_op& fine, const mfsem_op& coarse, int kind);
// Carves tables and intermediates out of the arena (null pointers when sizing).
void lattice_transfer_layout(LatticeTransfer& t, const mfsem_op& fine, const mfsem_op& coarse,
                             int kind, int batch, size_t word, Arena& a);
void lattice_transfer_upload(const LatticeTransfer& t);
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
