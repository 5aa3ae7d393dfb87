// The C ABI of libmfsem: argument validation, error reporting and dispatch.
// No C++ exception crosses this boundary; every entry point returns a status.
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "solver.hpp"

namespace mfsem {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }

void fail(mfsem_status code, const std::string& msg) { throw Error{code, msg}; }

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess)
    fail(MFSEM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

namespace {
// Fixed device memory of mfsem_pcg_noalloc: the PCG work vectors, per-member
// scalars and reduction partials for callers that cannot allocate.  Every GPU
// the library runs on holds its own copy for the life of the process.  Host
// code never uses the array's name as an address (on the host it is a
// stand-in symbol): it takes each device's address from hipGetSymbolAddress,
// once per device, with that device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)MFSEM_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Device address of the scratch array on the calling thread's current device.
void* noalloc_scratch() {
  int dev = -1;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    fail(MFSEM_EDEVICE, "device index " + std::to_string(dev) + " beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    check_hip(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (ptr == nullptr) fail(MFSEM_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}
}  // namespace

void launch_box(const mfsem_box_desc& d, int64_t n_elem, int64_t n_dof, const double* xi_host,
                int32_t* ed, double* xyz, double* fib, hipStream_t s);
void launch_box_parents(const int32_t n[3], int32_t* parent, int8_t* child, hipStream_t s);
void launch_place_nodes(int p, int kind, int pc, int64_t n_elem, const int32_t* ed,
                        int64_t n_nodes, const double* xyz, const double* fib, int64_t n_new,
                        const int32_t* elem, const int32_t* loc, double* xyz_out,
                        double* fib_out, hipStream_t s);
void launch_ap(int64_t n, double dt, double chi, double cm, const mfsem_ap_params& prm,
               const double* V, double* w, const double* istim, const double* m, double* b,
               hipStream_t s);
void launch_ap_bdf2(int64_t n, double dt, double chi, double cm, const mfsem_ap_params& prm,
                    const double* V, const double* Vo, double* w, double* wo, const double* istim,
                    const double* m, double* b, hipStream_t s);
void launch_activation(int64_t n, double t, double dt, const double* V, const double* Vo,
                       double* act, double* rate, double v_cross, double* cross, hipStream_t s);
void launch_extrapolate(int64_t n, const double* v, const double* vo, double* out, hipStream_t s);

namespace {

template <typename F>
mfsem_status guarded(F&& f) {
  try {
    f();
    return MFSEM_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(std::string("internal error: ") + e.what());
    return MFSEM_EDEVICE;
  }
}

void require(bool ok, const std::string& msg) {
  if (!ok) fail(MFSEM_EINVAL, msg);
}
// literal messages build no std::string unless the check fails
void require(bool ok, const char* msg) {
  if (!ok) fail(MFSEM_EINVAL, msg);
}

void require_aligned(const void* p, size_t a, const char* what) {
  require((reinterpret_cast<uintptr_t>(p) % a) == 0,
          std::string(what) + " is not " + std::to_string(a) + "-byte aligned");
}

void box_counts(const mfsem_box_desc* b, int64_t* ne, int64_t* nd) {
  require(b != nullptr, "box descriptor is NULL");
  require(b->p >= 1 && b->p <= MFSEM_MAX_P, "box p must be in 1..MFSEM_MAX_P");
  for (int i = 0; i < 3; ++i) {
    require(b->n[i] >= 1, "box element counts must be >= 1");
    require(b->length[i] > 0.0 && std::isfinite(b->length[i]), "box lengths must be positive");
  }
  *ne = (int64_t)b->n[0] * b->n[1] * b->n[2];
  *nd = ((int64_t)b->p * b->n[0] + 1) * ((int64_t)b->p * b->n[1] + 1) * ((int64_t)b->p * b->n[2] + 1);
}

// The FP64 stiffness apply can rebuild G from the node lattice when the map
// nodes are the DOF nodes of a structured GLL lattice (points = nodes).
bool onthefly_eligible(const mfsem_op_desc* d) {
  const int mp = d->map_p == 0 ? d->p : d->map_p;
  return d->lattice[0] > 0 && d->quad == MFSEM_GLL && mp == d->p && d->p <= 6 &&
         (d->map_elem_dof == nullptr || d->map_elem_dof == d->elem_dof) &&
         d->n_map_nodes == d->n_dof && d->sheet == nullptr && d->store_f64;
}

void validate_op(const mfsem_op_desc* d) {
  require(d != nullptr, "operator descriptor is NULL");
  require(d->p >= 1 && d->p <= MFSEM_MAX_P, "p must be in 1..MFSEM_MAX_P");
  require(d->quad == MFSEM_GLL || d->quad == MFSEM_GAUSS, "quad must be MFSEM_GLL or MFSEM_GAUSS");
  const int q = d->nq1d == 0 ? d->p + 1 : d->nq1d;
  if (d->quad == MFSEM_GLL) require(q == d->p + 1, "GLL quadrature needs nq1d == p+1");
  else require(q >= d->p + 1 && q <= d->p + 3, "Gauss quadrature needs p+1 <= nq1d <= p+3");
  const int mp = d->map_p == 0 ? d->p : d->map_p;
  require(mp >= 1 && mp <= MFSEM_MAX_P, "map_p must be in 1..MFSEM_MAX_P");
  require(d->map_elem_dof != nullptr || mp == d->p, "map_elem_dof may be NULL only when map_p == p");
  require(d->n_elem >= 0 && d->n_dof >= 0, "negative sizes");
  require(d->n_dof <= INT32_MAX, "n_dof must fit in int32");
  require(d->n_elem <= INT32_MAX, "n_elem must fit in int32");
  require(d->n_elem == 0 || d->elem_dof != nullptr, "elem_dof is NULL");
  require(d->n_elem == 0 || d->map_xyz != nullptr, "map_xyz is NULL");
  require(d->sheet == nullptr || d->fiber != nullptr, "a sheet field needs a fiber field");
  require(d->batch >= 1 && d->batch <= 65535, "batch must be in 1..65535");
  require(d->alpha >= 0.0 && std::isfinite(d->alpha), "alpha must be finite and >= 0");
  require(d->store_f64 || d->store_f32, "store_f64 or store_f32 must be set");
  if (!d->sigma)
    for (int i = 0; i < 3; ++i)
      require(std::isfinite(d->sigma_const[i]), "sigma_const must be finite");
  if (d->lattice[0] || d->lattice[1] || d->lattice[2]) {
    require(d->lattice[0] > 0 && d->lattice[1] > 0 && d->lattice[2] > 0,
            "lattice counts must all be positive (or all zero)");
    require((int64_t)d->lattice[0] * d->lattice[1] * d->lattice[2] == d->n_elem,
            "lattice counts do not multiply to n_elem");
    const int64_t nd = ((int64_t)d->p * d->lattice[0] + 1) * ((int64_t)d->p * d->lattice[1] + 1) *
                       ((int64_t)d->p * d->lattice[2] + 1);
    require(nd == d->n_dof, "lattice counts do not give n_dof");
  }
  require(d->geometry >= MFSEM_GEOM_AUTO && d->geometry <= MFSEM_GEOM_ONTHEFLY,
          "geometry must be MFSEM_GEOM_AUTO, _STORED or _ONTHEFLY");
  if (d->geometry == MFSEM_GEOM_ONTHEFLY)
    require(onthefly_eligible(d),
            "on-the-fly geometry needs a structured lattice, GLL quadrature, p <= 6, the map on "
            "the DOF nodes (map_p == p, map_elem_dof NULL or elem_dof, n_map_nodes == n_dof), "
            "no sheet and store_f64");
}

void op_init(mfsem_op& op, const mfsem_op_desc* d) {
  op.d = *d;
  op.P = d->p + 1;
  op.Q = d->nq1d == 0 ? d->p + 1 : d->nq1d;
  op.d.nq1d = op.Q;
  op.d.map_p = d->map_p == 0 ? d->p : d->map_p;
  op.Pm = op.d.map_p + 1;
  op.nq3 = (int64_t)op.Q * op.Q * op.Q;
  op.alpha = d->alpha;
  op.off = table_offsets(op.P, op.Q, op.Pm);
  op.structured = d->lattice[0] > 0;
  for (int i = 0; i < 3; ++i) op.lat[i] = d->lattice[i];
  op.otf = d->geometry == MFSEM_GEOM_ONTHEFLY;  // validated as eligible
}

void check_op(const mfsem_op* op, int dtype) {
  require(op != nullptr, "operator is NULL");
  require(dtype == MFSEM_F64 || dtype == MFSEM_F32, "dtype must be MFSEM_F64 or MFSEM_F32");
  if (dtype == MFSEM_F64) require(op->G64 != nullptr, "operator has no FP64 geometry (store_f64 = 0)");
  else require(op->G32 != nullptr, "operator has no FP32 geometry (store_f32 = 0)");
}

// the vectors of an operator with DOFs must be given and distinct; with no
// DOFs (an empty mesh) they have no entries and may be NULL
void require_vectors(const mfsem_op& op, const void* x, const void* y) {
  if (op.d.n_dof == 0) return;
  require(x && y, "x or y is NULL");
  require(x != y, "x and y must not alias");
}

void read_bad_flag(mfsem_op& op, hipStream_t s) {
  unsigned long long flags[3] = {0, 0, 0};
  MFSEM_HIP(hipMemcpyAsync(flags, op.bad, sizeof(flags), hipMemcpyDeviceToHost, s));
  MFSEM_HIP(hipStreamSynchronize(s));
  op.use_det = flags[1] == 0;
  if (op.structured && flags[2] != 0)
    fail(MFSEM_EINVAL, "elem_dof does not follow the structured numbering of the given lattice (" +
                           std::to_string(flags[2]) + " element nodes differ)");
  const unsigned long long bad = flags[0];
  if (bad != ~0ull) {
    const unsigned long long e = bad / op.nq3, k = bad % op.nq3;
    fail(MFSEM_EGEOMETRY, "det J <= 0 in element " + std::to_string(e) + " at quadrature point " +
                              std::to_string(k));
  }
}

}  // namespace

void op_layout(mfsem_op& op, Arena& a) {
  const size_t ne = (size_t)op.d.n_elem, nq = (size_t)op.nq3, B = (size_t)op.d.batch;
  if (op.d.store_f64) {
    op.G64 = a.take_n<double>(B * ne * 6 * nq);
    op.WJ64 = a.take_n<double>(ne * nq);
  }
  if (op.d.store_f32) {
    op.G32 = a.take_n<float>(B * ne * 6 * nq);
    op.WJ32 = a.take_n<float>(ne * nq);
  }
  op.tab64 = a.take_n<double>(op.off.total);
  op.tab32 = a.take_n<float>(op.off.total);
  if (op.d.store_f64) op.idet64 = a.take_n<double>(B * ne);
  if (op.d.store_f32) op.idet32 = a.take_n<float>(B * ne);
  op.bad = a.take_n<unsigned long long>(3);
  op.sigma_copy = op.d.sigma ? a.take_n<double>(B * ne * 3) : nullptr;
}

}  // namespace mfsem

using namespace mfsem;

extern "C" {

int mfsem_abi_version(void) { return MFSEM_ABI_VERSION; }

const char* mfsem_last_error(void) { return mfsem::g_last_error.c_str(); }

mfsem_status mfsem_box_counts(const mfsem_box_desc* box, int64_t* n_elem, int64_t* n_dof) {
  return guarded([&] {
    require(n_elem && n_dof, "output pointers are NULL");
    box_counts(box, n_elem, n_dof);
  });
}

mfsem_status mfsem_box_generate(const mfsem_box_desc* box, int32_t* elem_dof, double* xyz,
                                double* fiber, void* stream) {
  return guarded([&] {
    int64_t ne, nd;
    box_counts(box, &ne, &nd);
    require(nd <= INT32_MAX, "box has more than INT32_MAX nodes");
    require(elem_dof && xyz, "elem_dof or xyz is NULL");
    require(!box->fiber || fiber, "fiber output is NULL but box->fiber is set");
    hipStream_t s = as_stream(stream);
    // GLL points of degree p for the node placement (passed by value)
    std::vector<double> xi, w;
    gll_rule(box->p, xi, w);
    launch_box(*box, ne, nd, xi.data(), elem_dof, xyz, fiber, s);
  });
}

mfsem_status mfsem_box_parents(const int32_t n_fine[3], int32_t* parent, int8_t* child,
                               void* stream) {
  return guarded([&] {
    require(n_fine && parent && child, "NULL argument");
    for (int i = 0; i < 3; ++i)
      require(n_fine[i] >= 2 && n_fine[i] % 2 == 0, "octree coarsening needs even counts >= 2");
    launch_box_parents(n_fine, parent, child, as_stream(stream));
  });
}

mfsem_status mfsem_op_workspace_bytes(const mfsem_op_desc* d, size_t* bytes) {
  return guarded([&] {
    require(bytes != nullptr, "bytes is NULL");
    validate_op(d);
    mfsem_op op;
    op_init(op, d);
    Arena a;
    op_layout(op, a);
    *bytes = a.used;
  });
}

mfsem_status mfsem_op_create(const mfsem_op_desc* d, void* ws, size_t ws_bytes, void* stream,
                             mfsem_op** out) {
  mfsem_op* op = nullptr;
  mfsem_status st = guarded([&] {
    require(out != nullptr, "out is NULL");
    validate_op(d);
    require(ws != nullptr, "workspace is NULL");
    require_aligned(ws, 256, "workspace");
    op = new mfsem_op();
    op_init(*op, d);
    Arena a;
    a.base = static_cast<char*>(ws);
    a.size = ws_bytes;
    op_layout(*op, a);
    hipStream_t s = as_stream(stream);
    op->tab_host = build_tables(op->d.p, op->d.quad, op->Q, op->d.map_p);
    op->tab_host32.assign(op->tab_host.begin(), op->tab_host.end());
    MFSEM_HIP(hipStreamSynchronize(s));
    MFSEM_HIP(hipMemcpy(op->tab64, op->tab_host.data(), op->tab_host.size() * sizeof(double),
                        hipMemcpyHostToDevice));
    MFSEM_HIP(hipMemcpy(op->tab32, op->tab_host32.data(), op->tab_host32.size() * sizeof(float),
                        hipMemcpyHostToDevice));
    if (d->sigma)
      MFSEM_HIP(hipMemcpyAsync(op->sigma_copy, d->sigma,
                               (size_t)d->batch * d->n_elem * 3 * sizeof(double),
                               hipMemcpyDeviceToDevice, s));
    run_geometry(*op, s);
    if (op->structured) launch_lattice_check(*op, op->bad + 2, s);
    read_bad_flag(*op, s);
    *out = op;
  });
  if (st != MFSEM_OK) delete op;
  return st;
}

mfsem_status mfsem_op_destroy(mfsem_op* op) {
  delete op;
  return MFSEM_OK;
}

mfsem_status mfsem_op_set_alpha(mfsem_op* op, double alpha) {
  return guarded([&] {
    require(op != nullptr, "operator is NULL");
    require(alpha >= 0.0 && std::isfinite(alpha), "alpha must be finite and >= 0");
    op->alpha = alpha;
    op->d.alpha = alpha;
  });
}

mfsem_status mfsem_op_set_sigma(mfsem_op* op, const double* sigma, void* stream) {
  return guarded([&] {
    require(op != nullptr && sigma != nullptr, "NULL argument");
    require(op->sigma_copy != nullptr, "operator was created without per-element sigma");
    hipStream_t s = as_stream(stream);
    MFSEM_HIP(hipMemcpyAsync(op->sigma_copy, sigma,
                             (size_t)op->d.batch * op->d.n_elem * 3 * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
    run_geometry(*op, s);
    read_bad_flag(*op, s);
  });
}

mfsem_status mfsem_op_apply(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                            void* stream) {
  return guarded([&] {
    check_op(op, dtype);
    require_vectors(*op, x, y);
    hipStream_t s = as_stream(stream);
    if (dtype == MFSEM_F64)
      launch_apply<double>(*op, static_cast<const double*>(x), static_cast<double*>(y), op->alpha, true, s);
    else
      launch_apply<float>(*op, static_cast<const float*>(x), static_cast<float*>(y), op->alpha, true, s);
  });
}

mfsem_status mfsem_op_apply_add(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                                void* stream) {
  return guarded([&] {
    check_op(op, dtype);
    require_vectors(*op, x, y);
    hipStream_t s = as_stream(stream);
    if (dtype == MFSEM_F64)
      launch_apply<double>(*op, static_cast<const double*>(x), static_cast<double*>(y), op->alpha, true, s, true);
    else
      launch_apply<float>(*op, static_cast<const float*>(x), static_cast<float*>(y), op->alpha, true, s, true);
  });
}

mfsem_status mfsem_op_apply_mass(const mfsem_op* op, int32_t dtype, const void* x, void* y,
                                 void* stream) {
  return guarded([&] {
    check_op(op, dtype);
    require_vectors(*op, x, y);
    hipStream_t s = as_stream(stream);
    if (dtype == MFSEM_F64)
      launch_apply<double>(*op, static_cast<const double*>(x), static_cast<double*>(y), 1.0, false, s);
    else
      launch_apply<float>(*op, static_cast<const float*>(x), static_cast<float*>(y), 1.0, false, s);
  });
}

mfsem_status mfsem_op_diagonal(const mfsem_op* op, int32_t dtype, void* d, void* stream) {
  return guarded([&] {
    check_op(op, dtype);
    require(d != nullptr || op->d.n_dof == 0, "d is NULL");
    hipStream_t s = as_stream(stream);
    if (dtype == MFSEM_F64) launch_diag<double>(*op, static_cast<double*>(d), s);
    else launch_diag<float>(*op, static_cast<float*>(d), s);
  });
}

mfsem_status mfsem_op_grad_sigma(const mfsem_op* op, const double* u, const double* w,
                                 double scale, double* g, void* stream) {
  return guarded([&] {
    require(op != nullptr, "operator is NULL");
    require(u && w && g, "NULL argument");
    require(std::isfinite(scale), "scale must be finite");
    launch_grad_sigma(*op, u, w, scale, g, as_stream(stream));
  });
}

// ----------------------------------------------------------- matrix-based ---
namespace {
void check_csr_op(const mfsem_op* op) {
  require(op != nullptr, "operator is NULL");
  if (!op->structured || op->d.quad != MFSEM_GLL || op->d.batch != 1 || op->G64 == nullptr)
    fail(MFSEM_EUNSUPPORTED,
         "the assembled matrix needs a structured GLL lattice, batch 1 and FP64 geometry");
}
void check_csr_pattern(int pattern) {
  require(pattern == MFSEM_CSR_ELEMENT || pattern == MFSEM_CSR_COUPLED,
          "pattern must be MFSEM_CSR_ELEMENT or MFSEM_CSR_COUPLED");
}
}  // namespace

mfsem_status mfsem_csr_nnz(const mfsem_op* op, int pattern, int64_t* nnz) {
  return guarded([&] {
    check_csr_op(op);
    check_csr_pattern(pattern);
    require(nnz != nullptr, "NULL argument");
    *nnz = csr_nnz(*op, pattern == MFSEM_CSR_COUPLED);
  });
}

mfsem_status mfsem_csr_assemble(const mfsem_op* op, int pattern, int64_t* row_ptr, int32_t* col,
                                double* val, void* stream) {
  return guarded([&] {
    check_csr_op(op);
    check_csr_pattern(pattern);
    require(row_ptr && col && val, "NULL argument");
    csr_assemble(*op, pattern == MFSEM_CSR_COUPLED, row_ptr, col, val, as_stream(stream));
  });
}

mfsem_status mfsem_csr_spmv(int64_t n_rows, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col, const double* val, const double* x, double* y,
                            void* stream) {
  return guarded([&] {
    require(n_rows >= 0 && nnz >= 0, "n_rows and nnz must be >= 0");
    require(n_rows == 0 || (row_ptr && col && val && x && y), "NULL argument");
    require(x != y, "x and y must not alias");
    csr_spmv(n_rows, nnz, row_ptr, col, val, x, y, as_stream(stream));
  });
}

// -------------------------------------------------------------- multigrid ---
namespace {

void mg_init(mfsem_mg& mg, const mfsem_mg_desc* d) {
  require(d != nullptr, "multigrid descriptor is NULL");
  require(d->n_levels >= 1 && d->n_levels <= 16, "n_levels must be in 1..16");
  require(d->ops != nullptr, "ops is NULL");
  require(d->n_levels == 1 || d->transfers != nullptr, "transfers is NULL");
  require(d->degree >= 1 && d->coarse_degree >= 1, "Chebyshev degrees must be >= 1");
  require(d->lo_frac > 0.0 && d->hi_frac > d->lo_frac, "need 0 < lo_frac < hi_frac");
  require(d->eig_iters >= 1 || d->lambda_max, "eig_iters must be >= 1");
  require(d->precision == MFSEM_F64 || d->precision == MFSEM_F32, "precision must be F64 or F32");
  require(d->graphs == 0 || d->graphs == 1, "graphs must be 0 or 1");
  mg.d = *d;
  mg.prec = d->precision;
  mg.batch = d->ops[0] ? d->ops[0]->d.batch : 1;
  mg.lv.assign(d->n_levels, mfsem_mg_level{});
  for (int l = 0; l < d->n_levels; ++l) {
    const mfsem_op* op = d->ops[l];
    check_op(op, d->precision);
    require(op->d.batch == mg.batch, "all levels need the same batch");
    mfsem_mg_level& L = mg.lv[l];
    L.op = op;
    L.n = op->d.n_dof;
    L.steps = (l + 1 == d->n_levels) ? d->coarse_degree : d->degree;
    if (l + 1 < d->n_levels) {
      L.tr = d->transfers[l];
      const mfsem_op* c = d->ops[l + 1];
      require(c != nullptr, "NULL level operator");
      if (L.tr.kind == MFSEM_TRANSFER_P) {
        require(c->d.n_elem == op->d.n_elem, "p-transfer levels need the same elements");
        require(c->P <= op->P, "p-transfer must not raise the degree");
      } else if (L.tr.kind == MFSEM_TRANSFER_H) {
        require(L.tr.parent && L.tr.child, "h-transfer needs parent and child arrays");
        require(c->P == op->P, "h-transfer keeps the degree");
      } else {
        fail(MFSEM_EINVAL, "unknown transfer kind");
      }
    }
  }
}

}  // namespace

mfsem_status mfsem_mg_workspace_bytes(const mfsem_mg_desc* d, size_t* bytes) {
  return guarded([&] {
    require(bytes != nullptr, "bytes is NULL");
    mfsem_mg mg;
    mg_init(mg, d);
    Arena a;
    mg_layout(mg, a);
    *bytes = a.used;
  });
}

mfsem_status mfsem_mg_create(const mfsem_mg_desc* d, void* ws, size_t ws_bytes, void* stream,
                             mfsem_mg** out) {
  mfsem_mg* mg = nullptr;
  mfsem_status st = guarded([&] {
    require(out != nullptr, "out is NULL");
    require(ws != nullptr, "workspace is NULL");
    require_aligned(ws, 256, "workspace");
    mg = new mfsem_mg();
    mg_init(*mg, d);
    mg->d.ops = nullptr;        // not kept: the levels hold the pointers
    mg->d.transfers = nullptr;
    mg->d.lambda_max = d->lambda_max;
    Arena a;
    a.base = static_cast<char*>(ws);
    a.size = ws_bytes;
    mg_layout(*mg, a);
    mg_setup(*mg, as_stream(stream));
    mg->d.lambda_max = nullptr;
    *out = mg;
  });
  if (st != MFSEM_OK) delete mg;
  return st;
}

mfsem_status mfsem_mg_destroy(mfsem_mg* mg) {
  delete mg;
  return MFSEM_OK;
}

mfsem_status mfsem_mg_vcycle(const mfsem_mg* mg, const void* r, void* z, void* stream) {
  return guarded([&] {
    require(mg && r && z, "NULL argument");
    require(r != z, "r and z must not alias");
    mg_vcycle(*mg, r, z, as_stream(stream));
  });
}

mfsem_status mfsem_mg_lambdas(const mfsem_mg* mg, double* lam) {
  return guarded([&] {
    require(mg && lam, "NULL argument");
    for (size_t l = 0; l < mg->lv.size(); ++l)
      for (int b = 0; b < mg->batch; ++b) lam[l * mg->batch + b] = mg->lv[l].lam[b];
  });
}

mfsem_status mfsem_mg_transfer(const mfsem_mg* mg, int32_t level, int32_t direction,
                               const void* in, void* out, void* stream) {
  return guarded([&] {
    require(mg && in && out, "NULL argument");
    require(in != out, "in and out must not alias");
    require(level >= 0 && level + 1 < (int)mg->lv.size(), "level out of range");
    require(direction == 0 || direction == 1, "direction must be 0 or 1");
    mg_transfer(*mg, level, direction, in, out, as_stream(stream));
  });
}

// --------------------------------------------------------- node placement ---
namespace {
mfsem_status place_nodes_entry(int kind, int32_t p, int64_t n_elem, const int32_t* elem_dof,
                               int64_t n_nodes, const double* xyz, const double* fiber,
                               int32_t pc, int64_t n_new, const int32_t* elem,
                               const int32_t* loc, double* xyz_new, double* fiber_new,
                               void* stream) {
  return guarded([&] {
    require(p >= 1 && p <= MFSEM_MAX_P, "p must be in 1..MFSEM_MAX_P");
    if (kind == MFSEM_NODES_DEGREE) require(pc >= 1 && pc <= MFSEM_MAX_P, "pc must be in 1..MFSEM_MAX_P");
    require(n_elem >= 0 && n_nodes >= 0 && n_new >= 0, "counts must be >= 0");
    require(n_new == 0 || (elem && loc && xyz_new), "NULL array");
    require(n_new == 0 || n_elem == 0 || (elem_dof && xyz), "NULL parent mesh array");
    require(fiber_new == nullptr || fiber != nullptr, "fiber_new needs a parent fiber");
    launch_place_nodes(p, kind, pc, n_elem, elem_dof, n_nodes, xyz, fiber, n_new, elem, loc,
                       xyz_new, fiber ? fiber_new : nullptr, as_stream(stream));
  });
}
}  // namespace

mfsem_status mfsem_mesh_refine_nodes(int32_t p, int64_t n_elem, const int32_t* elem_dof,
                                     int64_t n_nodes, const double* xyz, const double* fiber,
                                     int64_t n_new, const int32_t* elem, const int32_t* loc,
                                     double* xyz_new, double* fiber_new, void* stream) {
  return place_nodes_entry(MFSEM_NODES_REFINE, p, n_elem, elem_dof, n_nodes, xyz, fiber, 0,
                           n_new, elem, loc, xyz_new, fiber_new, stream);
}

mfsem_status mfsem_mesh_degree_nodes(int32_t p, int64_t n_elem, const int32_t* elem_dof,
                                     int64_t n_nodes, const double* xyz, const double* fiber,
                                     int32_t pc, int64_t n_new, const int32_t* elem,
                                     const int32_t* loc, double* xyz_new, double* fiber_new,
                                     void* stream) {
  return place_nodes_entry(MFSEM_NODES_DEGREE, p, n_elem, elem_dof, n_nodes, xyz, fiber, pc,
                           n_new, elem, loc, xyz_new, fiber_new, stream);
}

// -------------------------------------------------------------------- PCG ---
mfsem_status mfsem_pcg_workspace_bytes(const mfsem_op* op, const mfsem_mg* mg, size_t* bytes) {
  return guarded([&] {
    require(op && bytes, "NULL argument");
    *bytes = pcg_bytes(*op, mg);
  });
}

}  // extern "C"

namespace {
// (P)CG entry shared by mfsem_pcg and mfsem_pcg_noalloc: validation, then the
// solve in the workspace `ws` of ws_bytes (the caller's, or the scratch array).
mfsem_status pcg_entry(const mfsem_op* op, const mfsem_mg* mg, const double* b, double* x,
                       const mfsem_solve_opts* opts, mfsem_solve_info* info, void* ws,
                       size_t ws_bytes, bool noalloc, void* stream) {
  mfsem_status solve_status = MFSEM_OK;
  mfsem_status st = guarded([&] {
    check_op(op, MFSEM_F64);
    require(opts && info && (ws || noalloc), "NULL argument");
    require_vectors(*op, b, x);
    require(opts->max_it >= 1, "max_it must be >= 1");
    require(opts->rtol >= 0.0 && opts->atol >= 0.0 && (opts->rtol > 0.0 || opts->atol > 0.0),
            "need rtol > 0 or atol > 0");
    if (mg) {
      require(mg->lv[0].op->d.n_dof == op->d.n_dof && mg->batch == op->d.batch,
              "multigrid finest level does not match the operator");
    }
    const size_t need = pcg_bytes(*op, mg);
    if (noalloc) {
      if (need > ws_bytes)
        fail(MFSEM_EINVAL, "mfsem_pcg_noalloc: the solve needs " + std::to_string(need) +
                               " bytes of work space, more than the library's fixed " +
                               std::to_string(ws_bytes >> 20) +
                               " MiB scratch (n_dof * batch too large); use mfsem_pcg");
      ws = noalloc_scratch();
    } else {
      require_aligned(ws, 256, "workspace");
      require(ws_bytes >= need, "workspace too small");
    }
    solve_status = pcg_solve(*op, mg, b, x, *opts, info, ws, ws_bytes, as_stream(stream));
    if (solve_status != MFSEM_OK) {
      std::string m = "PCG did not converge for every batch member (worst status " +
                      std::to_string((int)solve_status) + ")";
      set_error(m);
    }
  });
  return st != MFSEM_OK ? st : solve_status;
}
}  // namespace

extern "C" {

mfsem_status mfsem_pcg(const mfsem_op* op, const mfsem_mg* mg, const double* b, double* x,
                       const mfsem_solve_opts* opts, mfsem_solve_info* info, void* ws,
                       size_t ws_bytes, void* stream) {
  return pcg_entry(op, mg, b, x, opts, info, ws, ws_bytes, false, stream);
}

mfsem_status mfsem_pcg_noalloc(const mfsem_op* op, const mfsem_mg* mg, const double* b,
                               double* x, const mfsem_solve_opts* opts, mfsem_solve_info* info,
                               void* stream) {
  return pcg_entry(op, mg, b, x, opts, info, nullptr, NOALLOC_SCRATCH_BYTES, true, stream);
}

// ----------------------------------------------------------------- ionic ---
mfsem_status mfsem_ap_imex_rhs(int64_t n, double dt, double chi, double cm,
                               const mfsem_ap_params* prm, const double* V, double* w,
                               const double* i_stim, const double* mass_diag, double* b,
                               void* stream) {
  return guarded([&] {
    require(n >= 0, "n must be >= 0");
    require(dt > 0.0 && chi > 0.0 && cm > 0.0, "dt, chi and cm must be positive");
    require(prm != nullptr, "params is NULL");
    require(prm->v_amp != 0.0 && prm->t_scale > 0.0, "v_amp != 0 and t_scale > 0 required");
    require(n == 0 || (V && w && mass_diag && b), "NULL array");
    launch_ap(n, dt, chi, cm, *prm, V, w, i_stim, mass_diag, b, as_stream(stream));
  });
}

mfsem_status mfsem_ap_bdf2_rhs(int64_t n, double dt, double chi, double cm,
                               const mfsem_ap_params* prm, const double* V, const double* V_old,
                               double* w, double* w_old, const double* i_stim,
                               const double* mass_diag, double* b, void* stream) {
  return guarded([&] {
    require(n >= 0, "n must be >= 0");
    require(dt > 0.0 && chi > 0.0 && cm > 0.0, "dt, chi and cm must be positive");
    require(prm != nullptr, "params is NULL");
    require(prm->v_amp != 0.0 && prm->t_scale > 0.0, "v_amp != 0 and t_scale > 0 required");
    require(n == 0 || (V && V_old && w && w_old && mass_diag && b), "NULL array");
    launch_ap_bdf2(n, dt, chi, cm, *prm, V, V_old, w, w_old, i_stim, mass_diag, b,
                   as_stream(stream));
  });
}

mfsem_status mfsem_activation_update(int64_t n, double t, double dt, const double* V,
                                     const double* V_old, double* act, double* rate,
                                     double v_cross, double* cross, void* stream) {
  return guarded([&] {
    require(n >= 0, "n must be >= 0");
    require(dt > 0.0 && std::isfinite(dt), "dt must be positive and finite");
    require(std::isfinite(t), "t must be finite");
    require((act == nullptr) == (rate == nullptr), "act and rate must both be given or both NULL");
    require(act != nullptr || cross != nullptr, "nothing to update (act, rate and cross are NULL)");
    require(cross == nullptr || std::isfinite(v_cross), "v_cross must be finite");
    require(n == 0 || (V && V_old), "NULL array");
    launch_activation(n, t, dt, V, V_old, act, rate, v_cross, cross, as_stream(stream));
  });
}

mfsem_status mfsem_extrapolate(int64_t n, const double* v, const double* v_old, double* out,
                               void* stream) {
  return guarded([&] {
    require(n >= 0, "n must be >= 0");
    require(n == 0 || (v && v_old && out), "NULL array");
    launch_extrapolate(n, v, v_old, out, as_stream(stream));
  });
}

}  // extern "C"
