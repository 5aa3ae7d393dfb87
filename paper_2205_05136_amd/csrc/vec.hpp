// Vector kernels used by the Krylov and multigrid drivers.
#pragma once

#include "internal.hpp"

namespace mfsem {

// Per-member (P)CG scalars, kept in device memory.
struct PcgScalars {
  double rz, pq, rr, bb, alpha, beta;
  int32_t active, flag, flexible, pad;
};

enum { PCG_SET_RR_BB = 0, PCG_SET_PQ = 1, PCG_SET_RR = 2, PCG_SET_RZ_FIRST = 3, PCG_SET_RZ = 4 };

int dot_blocks(int64_t n);  // partial-sum blocks per member for vectors of length n

// out[bt*2 + {0,1}] = (a.b, a.c) per member (c may be null -> 0), in FP64; with
// sc, the reduction also applies the scalar update `what` to each member
template <typename TA, typename TB>
void vdot2(const TA* a, const TB* b, const TB* c, int64_t n, int batch, double* partial,
           double* out, hipStream_t s, PcgScalars* sc = nullptr, int what = 0);
// r = b - q (q may be null; cleared afterwards when zero_q), out = (r.r, b.b),
// then sc[bt].{rr, bb} = out when sc is given; r32 (may be null) = (float)r
void vresidual(const double* b, double* q, double* r, float* r32, int64_t n, int batch,
               double* partial, double* out, bool zero_q, PcgScalars* sc, hipStream_t s);
// x += alpha p, r -= alpha q with alpha from sc; q = 0; out[bt*2] = r.r and
// sc[bt].rr is updated for active members; r32 (may be null) = (float)r
void vxr(double* x, double* r, float* r32, const double* p, double* q, int64_t n, int batch,
         PcgScalars* sc, double* partial, double* out, hipStream_t s);
// p = z + beta p (p = z when beta == 0); z in FP64 or FP32
template <typename TZ>
void vp(double* p, const TZ* z, int64_t n, int batch, const PcgScalars* sc, hipStream_t s);
// x = (overwrite ? 0 : x) + w dinv (b - t) with w = coef[bt][1] (t may be
// null); clear_t / clear_b set t / b to zero after they are read
template <typename T>
void vjacobi(T* x, T* b, T* t, const T* dinv, int64_t n, int batch, const double* coef,
             bool overwrite, bool clear_t, bool clear_b, hipStream_t s);
// y += x, then x = 0 when clear_x
template <typename T>
void vaxpy(T* y, T* x, int64_t n, bool clear_x, hipStream_t s);
template <typename T>
void vinvert(T* x, int64_t n, hipStream_t s);
void vrandom(double* x, int64_t n, uint64_t seed, hipStream_t s);
// y = c[bt][0] y + c[bt][1] x   (c [batch][2] in device memory; y ignored when c0 == 0)
template <typename T>
void vlin(T* y, const T* x, int64_t n, int batch, const double* c, hipStream_t s);
// z = w o r
template <typename T>
void vmul(T* z, const T* w, const T* r, int64_t n, int batch, hipStream_t s);

}  // namespace mfsem
