// Vector kernels of the Krylov and multigrid drivers (the "CG steps" of
// Alg. 1 and the Chebyshev recurrence of the smoother, Section 4.3).
//
// Vectors are [batch][n]; per-member scalars live in device memory so that
// alpha, beta and the Chebyshev coefficients never make a host round trip.
// Dot products are two-stage and deterministic: fixed per-block partial sums
// accumulated in FP64 (also for FP32 vectors), then one block per member adds
// the partials in a fixed order.
#include "vec.hpp"

namespace mfsem {

namespace {

constexpr int VT = 256;

template <typename T>
__global__ void fill_kernel(T* __restrict__ x, int64_t n, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = v;
}

template <typename A, typename B>
__global__ void cast_kernel(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = (B)x[i];
}

__device__ inline double block_sum(double v, double* sh) {
  // wave64 reduction, then across the waves of the block
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) s += sh[w];
  return s;  // valid in thread 0
}

// partial[(bt*nblk + blk)*2 + {0,1}] = sum over the block's chunk of a*b and a*c
// (products and sums in FP64 whatever the storage types)
template <typename TA, typename TB>
__global__ __launch_bounds__(VT) void dot2_kernel(const TA* __restrict__ a,
                                                  const TB* __restrict__ b,
                                                  const TB* __restrict__ c, int64_t n,
                                                  double* __restrict__ partial) {
  __shared__ double sh[VT / 64];
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  double s0 = 0, s1 = 0;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    const double av = (double)a[off + i];
    s0 += av * (double)b[off + i];
    if (c) s1 += av * (double)c[off + i];
  }
  s0 = block_sum(s0, sh);
  s1 = c ? block_sum(s1, sh) : 0.0;
  if (threadIdx.x == 0) {
    const int64_t k = ((int64_t)bt * gridDim.x + blockIdx.x) * 2;
    partial[k] = s0;
    partial[k + 1] = s1;
  }
}

// Per-member scalar updates of (P)CG from the two reduced values of a dot.
__device__ void pcg_update(PcgScalars& s, double v0, double v1, int what) {
  switch (what) {
    case PCG_SET_RR_BB:  // after residual_kernel
      s.rr = v0;
      s.bb = v1;
      break;
    case PCG_SET_PQ:  // after dot(p, q)
      s.pq = v0;
      if (s.active && !(v0 > 0.0)) {
        s.active = 0;
        s.flag = (v0 == v0) ? MFSEM_EBREAKDOWN : MFSEM_ENONFINITE;
      }
      s.alpha = s.rz / v0;
      break;
    case PCG_SET_RR:  // after xr_kernel
      if (s.active) s.rr = v0;
      break;
    case PCG_SET_RZ_FIRST:  // after dot(r, z) on the first iteration
      s.rz = v0;
      s.beta = 0.0;
      if (s.active && !(v0 > 0.0)) {
        s.active = 0;
        s.flag = (v0 == v0) ? MFSEM_EBREAKDOWN : MFSEM_ENONFINITE;
      }
      break;
    case PCG_SET_RZ:  // dot(r, z) and dot(r, z_old): beta (flexible uses v0 - v1)
      if (s.active) {
        const double num = s.flexible ? v0 - v1 : v0;
        s.beta = num / s.rz;
        s.rz = v0;
        if (!(v0 > 0.0)) {
          s.active = 0;
          s.flag = (v0 == v0) ? MFSEM_EBREAKDOWN : MFSEM_ENONFINITE;
        }
      }
      break;
  }
}

// out[bt*2 + j] = sum of the partials of member bt; with sc, also the (P)CG
// scalar update `what` of member bt (saves a launch per dot product)
__global__ __launch_bounds__(VT) void reduce_kernel(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out, PcgScalars* sc,
                                                    int what) {
  __shared__ double sh[VT / 64];
  const int bt = blockIdx.x;
  double v[2];
  for (int j = 0; j < 2; ++j) {
    double s = 0;
    for (int i = threadIdx.x; i < nblk; i += VT) s += partial[((int64_t)bt * nblk + i) * 2 + j];
    s = block_sum(s, sh);
    v[j] = s;
    if (threadIdx.x == 0) out[bt * 2 + j] = s;
  }
  if (sc && threadIdx.x == 0) pcg_update(sc[bt], v[0], v[1], what);
}

// r = b - q ; partial sums of r.r and b.b; q is cleared after use (zero_q);
// r32 (may be null) receives r rounded to FP32
__global__ __launch_bounds__(VT) void residual_kernel(const double* __restrict__ b,
                                                      double* __restrict__ q,
                                                      double* __restrict__ r,
                                                      float* __restrict__ r32, int64_t n,
                                                      double* __restrict__ partial, int zero_q) {
  __shared__ double sh[VT / 64];
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  double s0 = 0, s1 = 0;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    const double bv = b[off + i];
    const double rv = q ? bv - q[off + i] : bv;
    if (q && zero_q) q[off + i] = 0.0;
    r[off + i] = rv;
    if (r32) r32[off + i] = (float)rv;
    s0 += rv * rv;
    s1 += bv * bv;
  }
  s0 = block_sum(s0, sh);
  s1 = block_sum(s1, sh);
  if (threadIdx.x == 0) {
    const int64_t k = ((int64_t)bt * gridDim.x + blockIdx.x) * 2;
    partial[k] = s0;
    partial[k + 1] = s1;
  }
}

// alpha = rz/pq; x += alpha p ; r -= alpha q ; partial r.r (finished members
// are left as they are); q is cleared for the next q = A p, which accumulates;
// r32 (may be null) receives the new r rounded to FP32
__global__ __launch_bounds__(VT) void xr_kernel(double* __restrict__ x, double* __restrict__ r,
                                                float* __restrict__ r32,
                                                const double* __restrict__ p,
                                                double* __restrict__ q, int64_t n,
                                                const PcgScalars* __restrict__ sc,
                                                double* __restrict__ partial) {
  __shared__ double sh[VT / 64];
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  const bool act = sc[bt].active != 0;
  const double al = sc[bt].alpha;
  double s0 = 0;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    if (act) {
      x[off + i] += al * p[off + i];
      const double rv = r[off + i] - al * q[off + i];
      r[off + i] = rv;
      if (r32) r32[off + i] = (float)rv;
      s0 += rv * rv;
    }
    q[off + i] = 0.0;
  }
  s0 = block_sum(s0, sh);
  if (threadIdx.x == 0) {
    const int64_t k = ((int64_t)bt * gridDim.x + blockIdx.x) * 2;
    partial[k] = s0;
    partial[k + 1] = 0.0;
  }
}

// p = z + beta p (beta = 0 on the first iteration via sc.beta)
template <typename TZ>
__global__ __launch_bounds__(VT) void p_kernel(double* __restrict__ p, const TZ* __restrict__ z,
                                               int64_t n, const PcgScalars* __restrict__ sc) {
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  if (!sc[bt].active) return;
  const double be = sc[bt].beta;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    p[off + i] = (be != 0.0) ? (double)z[off + i] + be * p[off + i] : (double)z[off + i];
}

// Damped-Jacobi step of the factored Chebyshev smoother:
// x = (overwrite ? 0 : x) + w dinv (b - t), w = coef[bt*2 + 1]; flags as for
// flags: 1 = overwrite x, 2 = clear t after use (the next A x accumulates into
// it), 4 = clear b after use (its last read in this V-cycle).
template <typename T>
__global__ __launch_bounds__(VT) void jacobi_kernel(T* __restrict__ x, T* __restrict__ b,
                                                    T* __restrict__ t, const T* __restrict__ dinv,
                                                    int64_t n, const double* __restrict__ coef,
                                                    int flags) {
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  const T w = (T)coef[bt * 2 + 1];
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT) {
    const T bv = b[off + i];
    const T r = t ? bv - t[off + i] : bv;
    const T dv = w * dinv[off + i] * r;
    x[off + i] = (flags & 1) ? dv : x[off + i] + dv;
    if (t && (flags & 2)) t[off + i] = T(0);
    if (flags & 4) b[off + i] = T(0);
  }
}

// y += x, then x = 0 when clear_x
template <typename T>
__global__ void axpy_kernel(T* __restrict__ y, T* __restrict__ x, int64_t n, int clear_x) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    y[i] += x[i];
    if (clear_x) x[i] = T(0);
  }
}

template <typename T>
__global__ void invert_kernel(T* __restrict__ x, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) x[i] = T(1) / x[i];
}

template <typename T>
__global__ __launch_bounds__(VT) void lin_kernel(T* __restrict__ y, const T* __restrict__ x,
                                                 int64_t n, const double* __restrict__ c) {
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  const T c0 = (T)c[bt * 2], c1 = (T)c[bt * 2 + 1];
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    y[off + i] = (c0 != T(0) ? c0 * y[off + i] : T(0)) + c1 * x[off + i];
}

template <typename T>
__global__ __launch_bounds__(VT) void mul_kernel(T* __restrict__ z, const T* __restrict__ w,
                                                 const T* __restrict__ r, int64_t n) {
  const int bt = blockIdx.y;
  const int64_t off = (int64_t)bt * n;
  for (int64_t i = (int64_t)blockIdx.x * VT + threadIdx.x; i < n; i += (int64_t)gridDim.x * VT)
    z[off + i] = w[off + i] * r[off + i];
}

// splitmix64 (Steele, Lea, Flood 2014) of a counter -> U[-1, 1)
__global__ void random_kernel(double* __restrict__ x, int64_t n, uint64_t seed) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    x[i] = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
  }
}

unsigned grid_for(int64_t n) {
  int64_t b = (n + VT - 1) / VT;
  if (b > 1024) b = 1024;
  if (b < 1) b = 1;
  return (unsigned)b;
}

// grid of the streaming kernels that write T: FP32 vectors need more lanes in
// flight than FP64 ones to keep the same bytes outstanding
template <typename T>
unsigned stream_grid(int64_t n) {
  constexpr int64_t cap = sizeof(T) <= 4 ? 4096 : 1024;
  int64_t b = (n + VT - 1) / VT;
  if (b > cap) b = cap;
  if (b < 1) b = 1;
  return (unsigned)b;
}

}  // namespace

int dot_blocks(int64_t n) { return (int)grid_for(n); }

template <typename T>
void vfill(T* x, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  fill_kernel<T><<<stream_grid<T>(n), VT, 0, s>>>(x, n, v);
  MFSEM_LAUNCH("fill_kernel");
}

template <typename A, typename B>
void vcast(const A* x, B* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  cast_kernel<A, B><<<stream_grid<B>(n), VT, 0, s>>>(x, y, n);
  MFSEM_LAUNCH("cast_kernel");
}

template <typename TA, typename TB>
void vdot2(const TA* a, const TB* b, const TB* c, int64_t n, int batch, double* partial,
           double* out, hipStream_t s, PcgScalars* sc, int what) {
  const unsigned nb = grid_for(n);
  dot2_kernel<TA, TB><<<dim3(nb, batch), VT, 0, s>>>(a, b, c, n, partial);
  MFSEM_LAUNCH("dot2_kernel");
  reduce_kernel<<<batch, VT, 0, s>>>(partial, (int)nb, out, sc, what);
  MFSEM_LAUNCH("reduce_kernel");
}

void vresidual(const double* b, double* q, double* r, float* r32, int64_t n, int batch,
               double* partial, double* out, bool zero_q, PcgScalars* sc, hipStream_t s) {
  const unsigned nb = grid_for(n);
  residual_kernel<<<dim3(nb, batch), VT, 0, s>>>(b, q, r, r32, n, partial, zero_q ? 1 : 0);
  MFSEM_LAUNCH("residual_kernel");
  reduce_kernel<<<batch, VT, 0, s>>>(partial, (int)nb, out, sc, PCG_SET_RR_BB);
  MFSEM_LAUNCH("reduce_kernel");
}

void vxr(double* x, double* r, float* r32, const double* p, double* q, int64_t n, int batch,
         PcgScalars* sc, double* partial, double* out, hipStream_t s) {
  const unsigned nb = grid_for(n);
  xr_kernel<<<dim3(nb, batch), VT, 0, s>>>(x, r, r32, p, q, n, sc, partial);
  MFSEM_LAUNCH("xr_kernel");
  reduce_kernel<<<batch, VT, 0, s>>>(partial, (int)nb, out, sc, PCG_SET_RR);
  MFSEM_LAUNCH("reduce_kernel");
}

template <typename TZ>
void vp(double* p, const TZ* z, int64_t n, int batch, const PcgScalars* sc, hipStream_t s) {
  p_kernel<TZ><<<dim3(grid_for(n), batch), VT, 0, s>>>(p, z, n, sc);
  MFSEM_LAUNCH("p_kernel");
}

template <typename T>
void vjacobi(T* x, T* b, T* t, const T* dinv, int64_t n, int batch, const double* coef,
             bool overwrite, bool clear_t, bool clear_b, hipStream_t s) {
  const int flags = (overwrite ? 1 : 0) | (clear_t ? 2 : 0) | (clear_b ? 4 : 0);
  jacobi_kernel<T><<<dim3(stream_grid<T>(n), batch), VT, 0, s>>>(x, b, t, dinv, n, coef, flags);
  MFSEM_LAUNCH("jacobi_kernel");
}

template <typename T>
void vaxpy(T* y, T* x, int64_t n, bool clear_x, hipStream_t s) {
  if (n <= 0) return;
  axpy_kernel<T><<<stream_grid<T>(n), VT, 0, s>>>(y, x, n, clear_x ? 1 : 0);
  MFSEM_LAUNCH("axpy_kernel");
}

template <typename T>
void vinvert(T* x, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  invert_kernel<T><<<stream_grid<T>(n), VT, 0, s>>>(x, n);
  MFSEM_LAUNCH("invert_kernel");
}

template <typename T>
void vlin(T* y, const T* x, int64_t n, int batch, const double* c, hipStream_t s) {
  lin_kernel<T><<<dim3(stream_grid<T>(n), batch), VT, 0, s>>>(y, x, n, c);
  MFSEM_LAUNCH("lin_kernel");
}

template <typename T>
void vmul(T* z, const T* w, const T* r, int64_t n, int batch, hipStream_t s) {
  mul_kernel<T><<<dim3(stream_grid<T>(n), batch), VT, 0, s>>>(z, w, r, n);
  MFSEM_LAUNCH("mul_kernel");
}

void vrandom(double* x, int64_t n, uint64_t seed, hipStream_t s) {
  if (n <= 0) return;
  random_kernel<<<grid_for(n), VT, 0, s>>>(x, n, seed);
  MFSEM_LAUNCH("random_kernel");
}

#define MFSEM_INST(T)                                                                        \
  template void vfill<T>(T*, int64_t, T, hipStream_t);                                       \
  template void vdot2<T, T>(const T*, const T*, const T*, int64_t, int, double*, double*,    \
                            hipStream_t, PcgScalars*, int);                                  \
  template void vp<T>(double*, const T*, int64_t, int, const PcgScalars*, hipStream_t);      \
  template void vaxpy<T>(T*, T*, int64_t, bool, hipStream_t);                                \
  template void vjacobi<T>(T*, T*, T*, const T*, int64_t, int, const double*, bool, bool,    \
                           bool, hipStream_t);                                               \
  template void vinvert<T>(T*, int64_t, hipStream_t);                                       \
  template void vlin<T>(T*, const T*, int64_t, int, const double*, hipStream_t);              \
  template void vmul<T>(T*, const T*, const T*, int64_t, int, hipStream_t);
MFSEM_INST(double)
MFSEM_INST(float)
#undef MFSEM_INST
template void vfill<unsigned long long>(unsigned long long*, int64_t, unsigned long long,
                                        hipStream_t);
template void vcast<double, float>(const double*, float*, int64_t, hipStream_t);
template void vcast<float, double>(const float*, double*, int64_t, hipStream_t);
template void vdot2<double, float>(const double*, const float*, const float*, int64_t, int,
                                   double*, double*, hipStream_t, PcgScalars*, int);

}  // namespace mfsem
