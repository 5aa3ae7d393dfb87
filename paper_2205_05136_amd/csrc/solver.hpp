// Multigrid hierarchy and (P)CG driver objects.
#pragma once

#include <vector>

#include "transfer_lattice.hpp"

struct mfsem_mg_level {
  const mfsem_op* op = nullptr;
  int64_t n = 0;               // DOFs per member
  int steps = 0;               // Chebyshev steps on this level
  void* dinv = nullptr;        // [batch][n]
  void* b = nullptr;           // right-hand side (levels > 0)
  void* x = nullptr;           // iterate (levels > 0)
  void* t = nullptr;           // A x
  void* d = nullptr;           // Chebyshev direction
  double* coef = nullptr;      // [steps][batch][2]
  std::vector<double> lam;     // [batch]
  // transfer to the next coarser level
  void* wmult = nullptr;       // [n] 1/multiplicity (element transfers)
  void* I = nullptr;           // [2][Pf][Pc] (element transfers)
  mfsem_transfer_desc tr{};
  // both levels structured lattices: the transfers run as 1D lattice passes
  bool lattice = false;
  mfsem::LatticeTransfer lt;
};

struct mfsem_mg {
  mfsem_mg_desc d;
  int batch = 1;
  int prec = MFSEM_F64;
  std::vector<mfsem_mg_level> lv;
  double* scratch = nullptr;   // reductions and coefficients during set-up
  // with d.graphs: the V-cycle's launches captured once per (r, z) pair and the
  // levels' alpha (a kernel argument), then replayed as one graph launch
  struct Graph {
    const void* r;
    void* z;
    std::vector<double> alpha;
    hipGraphExec_t exec;
  };
  mutable std::vector<Graph> graphs;
  mutable hipStream_t capture = nullptr;  // private stream the captures run on
  ~mfsem_mg();
};

namespace mfsem {
void mg_layout(mfsem_mg& mg, Arena& a);
void mg_setup(mfsem_mg& mg, hipStream_t s);
void mg_vcycle(const mfsem_mg& mg, const void* r, void* z, hipStream_t s);
void mg_transfer(const mfsem_mg& mg, int level, int direction, const void* in, void* out,
                 hipStream_t s);
size_t pcg_bytes(const mfsem_op& op, const mfsem_mg* mg);
mfsem_status pcg_solve(const mfsem_op& op, const mfsem_mg* mg, const double* b, double* x,
                       const mfsem_solve_opts& o, mfsem_solve_info* info, void* ws,
                       size_t ws_bytes, hipStream_t s);
}  // namespace mfsem
