// Pointwise ionic step and right-hand side of the full monodomain time loop
// (Alg. 1: the DOF-wise ionic loop and the right-hand side assembly; with
// SEM-NI the mass is diagonal, so the right-hand side is pointwise).
// First-order IMEX with the two-variable Aliev-Panfilov model standing in for
// the paper's ionic models: with u = (V - v_rest)/v_amp,
//   F = k u (1-u)(u-a) - u w,    G = (eps0 + mu1 w/(u+mu2)) (-w - k u (u-a-1)),
//   b = m * (chi cm/dt V + chi cm (v_amp/t_scale) F + I_stim),   w += dt/t_scale G.
#include "internal.hpp"

namespace mfsem {

namespace {

__global__ void ap_kernel(int64_t n, double dt, double chi, double cm, mfsem_ap_params prm,
                          const double* __restrict__ V, double* __restrict__ w,
                          const double* __restrict__ istim, const double* __restrict__ m,
                          double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double alpha = chi * cm / dt;
  const double fscale = chi * cm * (prm.v_amp / prm.t_scale);
  const double gscale = dt / prm.t_scale;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = V[i];
    const double u = (v - prm.v_rest) / prm.v_amp;
    const double wi = w[i];
    const double F = prm.k * u * (1.0 - u) * (u - prm.a) - u * wi;
    const double eps = prm.eps0 + prm.mu1 * wi / (u + prm.mu2);
    const double G = eps * (-wi - prm.k * u * (u - prm.a - 1.0));
    const double is = istim ? istim[i] : 0.0;
    b[i] = m[i] * (alpha * v + fscale * F + is);
    w[i] = wi + gscale * G;
  }
}

}  // namespace

void launch_ap(int64_t n, double dt, double chi, double cm, const mfsem_ap_params& prm,
               const double* V, double* w, const double* istim, const double* m, double* b,
               hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  ap_kernel<<<(unsigned)blocks, 256, 0, s>>>(n, dt, chi, cm, prm, V, w, istim, m, b);
  MFSEM_LAUNCH("ap_kernel");
}

}  // namespace mfsem
