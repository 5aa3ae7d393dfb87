// Geometric multigrid V-cycle with Chebyshev-Jacobi smoothing, and the (P)CG
// driver (Sections 4 and 4.3; smoother parameters from Section 5).
//
// Chebyshev smoothing of A x = b on [lo, hi] * lambda_max: k steps reduce the
// error by the degree-k Chebyshev polynomial of D^{-1} A scaled to 1 at zero.
// The three-term recurrence (theta = (l_hi + l_lo)/2, delta = (l_hi - l_lo)/2,
// s = theta/delta, rho_1 = 1/s; d = D^{-1}(b - A x0)/theta, then
// rho_j = 1/(2s - rho_{j-1}), d = rho_j rho_{j-1} d + (2 rho_j/delta) D^{-1}(b - A x),
// x += d) is applied here in its factored form: the same polynomial as k
// damped-Jacobi steps with weights 1/r over its roots r (cheb_coefficients),
// which gives the same iterate after the k steps with one vector less to read
// and write per step.  From x0 = 0 the first product with A is skipped.
// lambda_max per level comes from the Lanczos tridiagonal of a few
// Jacobi-preconditioned CG steps.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "solver.hpp"

namespace mfsem {

namespace {

template <typename T>
T* P_(void* p) { return static_cast<T*>(p); }

// Largest eigenvalue of a symmetric tridiagonal matrix by Sturm-sequence bisection.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // number of eigenvalues < x
    int c = 0;
    double q = a[0] - x;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
      const double qq = (q == 0.0) ? 1e-300 : q;
      q = a[i] - x - b[i - 1] * b[i - 1] / qq;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= m) hi = mid;  // all eigenvalues below mid
    else lo = mid;
  }
  return hi;
}

template <typename T>
void estimate_lambda(mfsem_mg& mg, mfsem_mg_level& L, int level, double* scratch_c,
                     hipStream_t s) {
  const int B = mg.batch;
  const int64_t n = L.n;
  // vectors: b, x, t, d of the level serve as r, z, q, p; a double buffer for v0
  T* r = P_<T>(L.b);
  T* z = P_<T>(L.x);
  T* q = P_<T>(L.t);
  T* p = P_<T>(L.d);
  const T* dinv = P_<T>(L.dinv);
  // seeded start vector (splitmix64 counter generator); for FP32 it is drawn
  // in FP64 into the level's x buffer (sized for doubles) and rounded
  const uint64_t seed = mg.d.eig_seed + 0x1000193ull * (uint64_t)level;
  if constexpr (sizeof(T) == sizeof(double)) {
    vrandom(reinterpret_cast<double*>(r), n * B, seed, s);
  } else {
    double* tmp = reinterpret_cast<double*>(z);
    vrandom(tmp, n * B, seed, s);
    vcast<double, float>(tmp, reinterpret_cast<float*>(r), n * B, s);
  }
  double* red = scratch_c;                 // [B][2]
  double* partial = scratch_c + 2 * B;     // [B][nblk][2]
  double* cdev = partial + 2 * (size_t)dot_blocks(n) * B;  // [B][2]
  std::vector<double> hc(2 * B), hred(2 * B), rz(B), alpha(B), beta(B);
  std::vector<std::vector<double>> al(B), be(B);
  vmul<T>(z, dinv, r, n, B, s);
  for (int b = 0; b < B; ++b) { hc[2 * b] = 0.0; hc[2 * b + 1] = 1.0; }
  MFSEM_HIP(hipMemcpy(cdev, hc.data(), 2 * B * sizeof(double), hipMemcpyHostToDevice));
  vlin<T>(p, z, n, B, cdev, s);
  vdot2<T, T>(r, z, nullptr, n, B, partial, red, s);
  MFSEM_HIP(hipMemcpyAsync(hred.data(), red, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
  MFSEM_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b) rz[b] = hred[2 * b];
  std::vector<int> live(B, 1);
  for (int it = 0; it < mg.d.eig_iters; ++it) {
    launch_apply<T>(*L.op, p, q, L.op->alpha, true, s);
    vdot2<T, T>(p, q, nullptr, n, B, partial, red, s);
    MFSEM_HIP(hipMemcpyAsync(hred.data(), red, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
    MFSEM_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b) {
      const double pq = hred[2 * b];
      if (!(pq > 0.0) || !(rz[b] > 0.0)) live[b] = 0;
      alpha[b] = live[b] ? rz[b] / pq : 0.0;
      hc[2 * b] = 1.0;
      hc[2 * b + 1] = -alpha[b];
    }
    MFSEM_HIP(hipMemcpy(cdev, hc.data(), 2 * B * sizeof(double), hipMemcpyHostToDevice));
    vlin<T>(r, q, n, B, cdev, s);
    vmul<T>(z, dinv, r, n, B, s);
    vdot2<T, T>(r, z, nullptr, n, B, partial, red, s);
    MFSEM_HIP(hipMemcpyAsync(hred.data(), red, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
    MFSEM_HIP(hipStreamSynchronize(s));
    for (int b = 0; b < B; ++b) {
      if (live[b]) {
        const double rzn = hred[2 * b];
        beta[b] = rzn / rz[b];
        al[b].push_back(alpha[b]);
        be[b].push_back(beta[b]);
        rz[b] = rzn;
        if (!(rzn > 0.0)) live[b] = 0;
      } else {
        beta[b] = 0.0;
      }
      hc[2 * b] = beta[b];
      hc[2 * b + 1] = 1.0;
    }
    MFSEM_HIP(hipMemcpy(cdev, hc.data(), 2 * B * sizeof(double), hipMemcpyHostToDevice));
    vlin<T>(p, z, n, B, cdev, s);
  }
  L.lam.assign(B, 0.0);
  for (int b = 0; b < B; ++b) {
    const int m = (int)al[b].size();
    if (m == 0) fail(MFSEM_EBREAKDOWN, "eigenvalue estimate: CG broke down at the first step");
    std::vector<double> da(m), off(m > 1 ? m - 1 : 0);
    for (int j = 0; j < m; ++j) {
      da[j] = 1.0 / al[b][j] + (j > 0 ? be[b][j - 1] / al[b][j - 1] : 0.0);
      if (j + 1 < m) off[j] = std::sqrt(be[b][j]) / al[b][j];
    }
    L.lam[b] = tridiag_max_eig(da, off);
  }
}

// The smoother applies the degree-k Chebyshev polynomial of the interval
// [lo, hi] to D^{-1} A, which equals the product of k damped-Jacobi steps
// x += w_j D^{-1} (b - A x) with w_j = 1 / r_j over the polynomial's roots
// r_j = theta + delta cos((2j+1) pi / (2k)).  After the k steps the iterate is
// the same as the three-term recurrence's; the steps carry no direction vector,
// so each reads x, b, A x and D^{-1} and writes x (two vectors fewer than the
// recurrence).  The roots are taken from the largest down: every partial
// product then stays within [-1, 1] on [0, hi] (no intermediate growth).
// coef[j][b] = (0, w_j).
void cheb_coefficients(const mfsem_mg& mg, const mfsem_mg_level& L, std::vector<double>& out) {
  const int B = mg.batch;
  const int k = L.steps;
  out.assign((size_t)k * B * 2, 0.0);
  for (int b = 0; b < B; ++b) {
    const double lmax = L.lam[b];
    const double lo = mg.d.lo_frac * lmax, hi = mg.d.hi_frac * lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo);
    for (int j = 0; j < k; ++j) {
      const double r = theta + delta * std::cos((2.0 * j + 1.0) * M_PI / (2.0 * k));
      out[((size_t)j * B + b) * 2] = 0.0;
      out[((size_t)j * B + b) * 2 + 1] = 1.0 / r;
    }
  }
}

template <typename T>
TransferArgs<T> transfer_args(const mfsem_mg& mg, int l) {
  const mfsem_mg_level& F = mg.lv[l];
  const mfsem_mg_level& C = mg.lv[l + 1];
  TransferArgs<T> a;
  a.n_elem_f = F.op->d.n_elem;
  a.Pf = F.op->P;
  a.Pc = C.op->P;
  a.ed_f = F.op->d.elem_dof;
  a.ed_c = C.op->d.elem_dof;
  a.parent = F.tr.kind == MFSEM_TRANSFER_H ? F.tr.parent : nullptr;
  a.child = F.tr.kind == MFSEM_TRANSFER_H ? F.tr.child : nullptr;
  a.I = P_<T>(F.I);
  a.nf = F.n;
  a.nc = C.n;
  return a;
}

// Chebyshev smoothing; the level's t is zero on entry and on exit (every
// product with A adds into it and the Chebyshev step clears it after reading).
// With clear_b the last step also clears b.
template <typename T>
void smooth(const mfsem_mg& mg, const mfsem_mg_level& L, T* b, T* x, bool from_zero,
            bool clear_b, hipStream_t s) {
  const int B = mg.batch;
  T* t = P_<T>(L.t);
  const T* dinv = P_<T>(L.dinv);
  for (int j = 0; j < L.steps; ++j) {
    const double* c = L.coef + (size_t)j * B * 2;
    const bool last = j + 1 == L.steps;
    if (j == 0 && from_zero) {
      vjacobi<T>(x, b, nullptr, dinv, L.n, B, c, true, false, clear_b && last, s);
    } else {
      launch_apply<T>(*L.op, x, t, L.op->alpha, true, s, true);
      vjacobi<T>(x, b, t, dinv, L.n, B, c, false, true, clear_b && last, s);
    }
  }
}

// V-cycle from x = 0.  Zero-on-consume invariant: between V-cycles every
// level's t, and the b of every level below the finest, hold zeros, so products
// with A and the restriction add into them without clearing launches; each
// buffer is cleared by the kernel that reads it last.  b of the finest level is
// the caller's and is never written.
template <typename T>
void vcycle(const mfsem_mg& mg, int l, T* b, T* x, hipStream_t s) {
  const mfsem_mg_level& L = mg.lv[l];
  const int B = mg.batch;
  const bool own_b = l > 0;
  if (l + 1 == (int)mg.lv.size()) {
    smooth<T>(mg, L, b, x, true, own_b, s);
    return;
  }
  const mfsem_mg_level& C = mg.lv[l + 1];
  smooth<T>(mg, L, b, x, true, false, s);
  T* t = P_<T>(L.t);
  launch_apply<T>(*L.op, x, t, L.op->alpha, true, s, true);
  if (L.lattice) {
    lattice_restrict<T>(L.lt, B, b, t, P_<T>(C.b), s);  // overwrites C.b
    vcycle<T>(mg, l + 1, P_<T>(C.b), P_<T>(C.x), s);
    lattice_prolong<T>(L.lt, B, P_<T>(C.x), x, true, t, s);  // x += P xc, t = 0
  } else {
    const TransferArgs<T> ta = transfer_args<T>(mg, l);
    launch_restrict<T>(ta, B, b, t, P_<T>(L.wmult), P_<T>(C.b), s);
    vcycle<T>(mg, l + 1, P_<T>(C.b), P_<T>(C.x), s);
    launch_prolong<T>(ta, B, P_<T>(C.x), t, s);  // overwrites t
    vaxpy<T>(x, t, L.n * B, true, s);
  }
  smooth<T>(mg, L, b, x, false, own_b, s);
}

}  // namespace

}  // namespace mfsem

mfsem_mg::~mfsem_mg() {
  for (auto& g : graphs) (void)hipGraphExecDestroy(g.exec);
  if (capture) (void)hipStreamDestroy(capture);
}

namespace mfsem {

void mg_layout(mfsem_mg& mg, Arena& a) {
  const size_t w = mg.prec == MFSEM_F64 ? sizeof(double) : sizeof(float);
  const int B = mg.batch;
  size_t scratch = 0;
  for (size_t l = 0; l < mg.lv.size(); ++l) {
    mfsem_mg_level& L = mg.lv[l];
    const size_t nb = (size_t)L.n * B;
    L.dinv = a.take(nb * w);
    L.t = a.take(nb * w);
    L.d = a.take(nb * w);
    // level 0 keeps its own b/x too: the eigenvalue estimate works in them
    L.b = a.take(nb * w);
    L.x = a.take(nb * std::max(w, sizeof(double)));
    L.coef = a.take_n<double>((size_t)std::max(1, L.steps) * B * 2);
    if (l + 1 < mg.lv.size()) {
      const mfsem_op& C = *mg.lv[l + 1].op;
      L.lattice = lattice_transfer_applies(*L.op, C, L.tr.kind);
      if (L.lattice) lattice_transfer_layout(L.lt, *L.op, C, L.tr.kind, B, w, a);
      // h-levels keep the element transfer's buffers: set-up falls back to it
      // when the parent/child arrays do not follow the box convention
      if (!L.lattice || L.tr.kind == MFSEM_TRANSFER_H) {
        L.wmult = a.take(L.n * w);
        L.I = a.take((size_t)2 * L.op->P * C.P * w);
      }
    }
    scratch = std::max(scratch, (size_t)(4 * B + 2 * (size_t)dot_blocks(L.n) * B));
  }
  mg.scratch = a.take_n<double>(scratch);
}

void mg_setup(mfsem_mg& mg, hipStream_t s) {
  const int B = mg.batch;
  const bool f64 = mg.prec == MFSEM_F64;
  for (size_t l = 0; l < mg.lv.size(); ++l) {
    mfsem_mg_level& L = mg.lv[l];
    if (f64) {
      launch_diag<double>(*L.op, P_<double>(L.dinv), s);
      vinvert<double>(P_<double>(L.dinv), L.n * B, s);
    } else {
      launch_diag<float>(*L.op, P_<float>(L.dinv), s);
      vinvert<float>(P_<float>(L.dinv), L.n * B, s);
    }
    if (l + 1 < mg.lv.size() && L.tr.kind == MFSEM_TRANSFER_H) {
      // parent/child arrays index the coarse elements and the child halves: an
      // out-of-range entry would make the transfer kernels read out of bounds
      auto* bad = reinterpret_cast<unsigned long long*>(mg.scratch);
      MFSEM_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), s));
      launch_parents_range_check(L.op->d.n_elem, mg.lv[l + 1].op->d.n_elem, L.tr.parent,
                                 L.tr.child, bad, s);
      unsigned long long nbad = 0;
      MFSEM_HIP(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, s));
      MFSEM_HIP(hipStreamSynchronize(s));
      if (nbad != 0)
        fail(MFSEM_EINVAL, "h-transfer of level " + std::to_string(l) + ": " +
                               std::to_string(nbad) + " parent/child entries out of range");
    }
    if (l + 1 < mg.lv.size() && L.lattice && L.tr.kind == MFSEM_TRANSFER_H) {
      auto* mismatch = reinterpret_cast<unsigned long long*>(mg.scratch);
      MFSEM_HIP(hipMemsetAsync(mismatch, 0, sizeof(unsigned long long), s));
      launch_box_parents_check(L.op->lat, L.tr.parent, L.tr.child, mismatch, s);
      unsigned long long bad = 0;
      MFSEM_HIP(hipMemcpyAsync(&bad, mismatch, sizeof(bad), hipMemcpyDeviceToHost, s));
      MFSEM_HIP(hipStreamSynchronize(s));
      L.lattice = bad == 0;
    }
    if (l + 1 < mg.lv.size() && !L.lattice) {
      const mfsem_op& F = *L.op;
      const int P3 = F.P * F.P * F.P;
      if (f64) launch_inv_multiplicity<double>(F.d.elem_dof, F.d.n_elem, P3, L.n, P_<double>(L.wmult), s);
      else launch_inv_multiplicity<float>(F.d.elem_dof, F.d.n_elem, P3, L.n, P_<float>(L.wmult), s);
      std::vector<double> I = transfer_matrices(L.tr.kind, F.P - 1, mg.lv[l + 1].op->P - 1);
      MFSEM_HIP(hipStreamSynchronize(s));
      if (f64) {
        MFSEM_HIP(hipMemcpy(L.I, I.data(), I.size() * sizeof(double), hipMemcpyHostToDevice));
      } else {
        std::vector<float> If(I.begin(), I.end());
        MFSEM_HIP(hipMemcpy(L.I, If.data(), If.size() * sizeof(float), hipMemcpyHostToDevice));
      }
    }
  }
  MFSEM_HIP(hipStreamSynchronize(s));
  for (size_t l = 0; l < mg.lv.size(); ++l) {
    mfsem_mg_level& L = mg.lv[l];
    if (mg.d.lambda_max) {
      L.lam.assign(mg.d.lambda_max + l * B, mg.d.lambda_max + (l + 1) * B);
    } else if (f64) {
      estimate_lambda<double>(mg, L, (int)l, mg.scratch, s);
    } else {
      estimate_lambda<float>(mg, L, (int)l, mg.scratch, s);
    }
    for (int b = 0; b < B; ++b)
      if (!(L.lam[b] > 0.0) || !std::isfinite(L.lam[b]))
        fail(MFSEM_EBREAKDOWN, "non-positive lambda_max on multigrid level " + std::to_string(l));
    std::vector<double> c;
    cheb_coefficients(mg, L, c);
    MFSEM_HIP(hipMemcpy(L.coef, c.data(), c.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  // establish the V-cycle's zero-on-consume invariant (the eigenvalue
  // estimate used these buffers as scratch)
  for (size_t l = 0; l < mg.lv.size(); ++l) {
    mfsem_mg_level& L = mg.lv[l];
    const int64_t nb = L.n * B;
    if (f64) {
      vfill<double>(P_<double>(L.t), nb, 0.0, s);
      if (l > 0) vfill<double>(P_<double>(L.b), nb, 0.0, s);
    } else {
      vfill<float>(P_<float>(L.t), nb, 0.0f, s);
      if (l > 0) vfill<float>(P_<float>(L.b), nb, 0.0f, s);
    }
  }
  MFSEM_HIP(hipStreamSynchronize(s));
}

template <typename T>
void transfer_t(const mfsem_mg& mg, int l, int direction, const T* in, T* out, hipStream_t s) {
  if (mg.lv[l].lattice) {
    if (direction == 0) lattice_prolong<T>(mg.lv[l].lt, mg.batch, in, out, false, nullptr, s);
    else lattice_restrict<T>(mg.lv[l].lt, mg.batch, in, nullptr, out, s);
    return;
  }
  const TransferArgs<T> ta = transfer_args<T>(mg, l);
  if (direction == 0) {
    launch_prolong<T>(ta, mg.batch, in, out, s);
  } else {
    vfill<T>(out, mg.lv[l + 1].n * mg.batch, T(0), s);
    launch_restrict<T>(ta, mg.batch, in, nullptr, P_<T>(mg.lv[l].wmult), out, s);
  }
}

void mg_transfer(const mfsem_mg& mg, int level, int direction, const void* in, void* out,
                 hipStream_t s) {
  if (mg.prec == MFSEM_F64)
    transfer_t<double>(mg, level, direction, static_cast<const double*>(in), static_cast<double*>(out), s);
  else
    transfer_t<float>(mg, level, direction, static_cast<const float*>(in), static_cast<float*>(out), s);
}

namespace {
void vcycle_launches(const mfsem_mg& mg, const void* r, void* z, hipStream_t s) {
  // r is only read: the finest level never clears its b
  void* b = const_cast<void*>(r);
  if (mg.prec == MFSEM_F64) vcycle<double>(mg, 0, static_cast<double*>(b), static_cast<double*>(z), s);
  else vcycle<float>(mg, 0, static_cast<float*>(b), static_cast<float*>(z), s);
}
constexpr size_t MAX_GRAPHS = 4;
}  // namespace

void mg_vcycle(const mfsem_mg& mg, const void* r, void* z, hipStream_t s) {
  if (!mg.d.graphs) {
    vcycle_launches(mg, r, z, s);
    return;
  }
  std::vector<double> alpha(mg.lv.size());
  for (size_t l = 0; l < mg.lv.size(); ++l) alpha[l] = mg.lv[l].op->alpha;
  for (const auto& g : mg.graphs)
    if (g.r == r && g.z == z && g.alpha == alpha) {
      MFSEM_HIP(hipGraphLaunch(g.exec, s));
      return;
    }
  // capture the launches on a private stream (the caller's may be the null
  // stream, which cannot be captured); nothing runs until the replay below
  if (!mg.capture) MFSEM_HIP(hipStreamCreateWithFlags(&mg.capture, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  MFSEM_HIP(hipStreamBeginCapture(mg.capture, hipStreamCaptureModeThreadLocal));
  try {
    vcycle_launches(mg, r, z, mg.capture);
  } catch (...) {
    (void)hipStreamEndCapture(mg.capture, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  MFSEM_HIP(hipStreamEndCapture(mg.capture, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  MFSEM_HIP(e);
  if (mg.graphs.size() >= MAX_GRAPHS) {
    (void)hipGraphExecDestroy(mg.graphs.front().exec);
    mg.graphs.erase(mg.graphs.begin());
  }
  mg.graphs.push_back({r, z, alpha, exec});
  MFSEM_HIP(hipGraphLaunch(exec, s));
}

// ------------------------------------------------------------------ PCG ---
namespace {

struct PcgWs {
  double *r, *z, *p, *q, *zo;
  float *r32, *z32;
  PcgScalars* sc;
  double *partial, *red;
};

PcgWs pcg_layout(const mfsem_op& op, const mfsem_mg* mg, bool flexible, Arena& a) {
  const size_t nb = (size_t)op.d.n_dof * op.d.batch;
  PcgWs w{};
  w.r = a.take_n<double>(nb);
  w.z = a.take_n<double>(nb);
  w.p = a.take_n<double>(nb);
  w.q = a.take_n<double>(nb);
  w.zo = a.take_n<double>(nb);  // the flexible variant's second z buffer
  (void)flexible;
  if (mg && mg->prec == MFSEM_F32) {
    w.r32 = a.take_n<float>(nb);
    w.z32 = a.take_n<float>(nb);
  }
  w.sc = a.take_n<PcgScalars>(op.d.batch);
  w.partial = a.take_n<double>(2 * (size_t)dot_blocks(op.d.n_dof) * op.d.batch);
  w.red = a.take_n<double>(2 * (size_t)op.d.batch);
  return w;
}

}  // namespace

size_t pcg_bytes(const mfsem_op& op, const mfsem_mg* mg) {
  Arena a;
  pcg_layout(op, mg, true, a);
  return a.used;
}

mfsem_status pcg_solve(const mfsem_op& op, const mfsem_mg* mg, const double* b, double* x,
                       const mfsem_solve_opts& o, mfsem_solve_info* info, void* ws,
                       size_t ws_bytes, hipStream_t s) {
  Arena a;
  a.base = static_cast<char*>(ws);
  a.size = ws_bytes;
  const PcgWs w = pcg_layout(op, mg, o.flexible != 0, a);
  const int B = op.d.batch;
  const int64_t n = op.d.n_dof;
  const size_t nb = (size_t)n * B;
  std::vector<PcgScalars> hs(B);
  for (int i = 0; i < B; ++i) {
    hs[i] = PcgScalars{};
    hs[i].active = 1;
    hs[i].flexible = o.flexible ? 1 : 0;
  }
  MFSEM_HIP(hipStreamSynchronize(s));
  MFSEM_HIP(hipMemcpy(w.sc, hs.data(), B * sizeof(PcgScalars), hipMemcpyHostToDevice));

  // With the FP32 V-cycle, r32 = (float)r is written by the kernels that
  // update r, and z stays in FP32: every read of z converts it exactly, so the
  // iteration equals the one with an FP64 copy of z, without the two casts.
  // The flexible variant keeps the previous z by alternating two z buffers
  // (the z_old buffer holds FP32 values in the mixed case).
  const bool mixed = mg && mg->prec == MFSEM_F32;
  double* z64[2] = {w.z, w.zo};
  float* z32[2] = {w.z32, reinterpret_cast<float*>(w.zo)};
  auto precondition = [&](int cur) {
    if (!mg) {
      MFSEM_HIP(hipMemcpyAsync(z64[cur], w.r, nb * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else if (!mixed) {
      mg_vcycle(*mg, w.r, z64[cur], s);
    } else {
      mg_vcycle(*mg, w.r32, z32[cur], s);
    }
  };
  auto fetch = [&]() {
    MFSEM_HIP(hipMemcpyAsync(hs.data(), w.sc, B * sizeof(PcgScalars), hipMemcpyDeviceToHost, s));
    MFSEM_HIP(hipStreamSynchronize(s));
  };

  // r = b - A x; q is left at zero, and every later q = A p adds into it
  // (the update of x and r clears it again)
  launch_apply<double>(op, x, w.q, op.alpha, true, s);
  vresidual(b, w.q, w.r, mixed ? w.r32 : nullptr, n, B, w.partial, w.red, true, w.sc, s);
  fetch();
  std::vector<double> tol(B);
  std::vector<char> done(B, 0);
  bool changed = false;
  int live = 0;
  for (int i = 0; i < B; ++i) {
    info[i] = mfsem_solve_info{};
    info[i].b_norm = std::sqrt(hs[i].bb);
    info[i].r0_norm = std::sqrt(hs[i].rr);
    info[i].r_norm = info[i].r0_norm;
    tol[i] = std::max(o.rtol * info[i].b_norm, o.atol);
    if (!std::isfinite(hs[i].rr)) info[i].status = MFSEM_ENONFINITE;
    if (info[i].status != MFSEM_OK || info[i].r0_norm <= tol[i]) {
      hs[i].active = 0;
      done[i] = 1;
      changed = true;
    }
    live += !done[i];
  }
  if (changed) MFSEM_HIP(hipMemcpy(w.sc, hs.data(), B * sizeof(PcgScalars), hipMemcpyHostToDevice));

  for (int it = 1; live > 0 && it <= o.max_it; ++it) {
    // z of this iteration, and the previous one for the flexible beta
    const int cur = o.flexible ? (it & 1) : 0;
    const bool use_old = o.flexible && it > 1;
    precondition(cur);
    const int rz_what = it == 1 ? PCG_SET_RZ_FIRST : PCG_SET_RZ;
    if (mixed) {
      vdot2<double, float>(w.r, z32[cur], use_old ? z32[cur ^ 1] : nullptr, n, B, w.partial,
                           w.red, s, w.sc, rz_what);
      vp<float>(w.p, z32[cur], n, B, w.sc, s);
    } else {
      vdot2<double, double>(w.r, z64[cur], use_old ? z64[cur ^ 1] : nullptr, n, B, w.partial,
                            w.red, s, w.sc, rz_what);
      vp<double>(w.p, z64[cur], n, B, w.sc, s);
    }
    launch_apply<double>(op, w.p, w.q, op.alpha, true, s, true);
    vdot2<double, double>(w.p, w.q, nullptr, n, B, w.partial, w.red, s, w.sc, PCG_SET_PQ);
    vxr(x, w.r, mixed ? w.r32 : nullptr, w.p, w.q, n, B, w.sc, w.partial, w.red, s);
    fetch();
    changed = false;
    live = 0;
    for (int i = 0; i < B; ++i) {
      if (done[i]) continue;
      info[i].iters = it;
      if (hs[i].flag != 0) {  // breakdown or non-finite found on the device
        info[i].status = hs[i].flag;
        done[i] = 1;
        continue;
      }
      info[i].r_norm = std::sqrt(hs[i].rr);
      if (!std::isfinite(hs[i].rr)) info[i].status = MFSEM_ENONFINITE;
      if (info[i].status != MFSEM_OK || info[i].r_norm <= tol[i]) {
        hs[i].active = 0;
        done[i] = 1;
        changed = true;
      }
      live += !done[i];
    }
    if (changed) MFSEM_HIP(hipMemcpy(w.sc, hs.data(), B * sizeof(PcgScalars), hipMemcpyHostToDevice));
  }
  mfsem_status worst = MFSEM_OK;
  for (int i = 0; i < B; ++i) {
    if (info[i].status == MFSEM_OK && info[i].r_norm > tol[i]) info[i].status = MFSEM_ENOCONV;
    if (info[i].status != MFSEM_OK && (worst == MFSEM_OK || info[i].status < worst))
      worst = (mfsem_status)info[i].status;
  }
  return worst;
}

}  // namespace mfsem
