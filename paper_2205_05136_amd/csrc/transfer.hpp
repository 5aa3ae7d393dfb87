// Inter-level transfer kernels of the multigrid V-cycle.
#pragma once

#include "vec.hpp"

namespace mfsem {

template <typename T>
struct TransferArgs {
  int64_t n_elem_f;          // fine elements
  int Pf, Pc;                // nodes per axis, fine and coarse
  const int32_t* ed_f;       // [n_elem_f][Pf^3]
  const int32_t* ed_c;       // [n_elem_c][Pc^3]
  const int32_t* parent;     // [n_elem_f] or null (same element)
  const int8_t* child;       // [n_elem_f] or null
  const T* I;                // [2][Pf][Pc]
  int64_t nf, nc;            // DOFs per member, fine and coarse
};

// xf = P xc (plain stores; every fine DOF is written)
template <typename T>
void launch_prolong(const TransferArgs<T>& a, int batch, const T* xc, T* xf, hipStream_t s);
// rc += P^T ((bf - tf) o w)   (tf may be null); rc must be zeroed by the caller
template <typename T>
void launch_restrict(const TransferArgs<T>& a, int batch, const T* bf, const T* tf, const T* w,
                     T* rc, hipStream_t s);
// w = 1 / (number of elements containing each DOF)
template <typename T>
void launch_inv_multiplicity(const int32_t* ed, int64_t n_elem, int P3, int64_t n_dof, T* w,
                             hipStream_t s);
std::vector<double> transfer_matrices(int kind, int pf, int pc);

}  // namespace mfsem
