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

// BDF2 step of the partitioned scheme (Section 3: the ionic and monodomain
// discretization), with the extrapolated potential V* = 2 V^n - V^{n-1}:
//   gating:  3 w^{n+1} - 4 w^n + w^{n-1} = (2 dt/t_scale) G(u*, w^{n+1}),
//            a quadratic in w^{n+1} (G is eps(u*, w) times a term linear in w):
//            with c = k u*(u*-a-1), r = mu1/(u*+mu2), h = 2 dt/t_scale,
//            h r w^2 + (3 + h (eps0 + r c)) w + (h eps0 c - 4 w^n + w^{n-1}) = 0,
//            solved by the root that tends to the linear solution as r -> 0;
//   b = m (chi cm/dt (4 V^n - V^{n-1})/2 + chi cm (v_amp/t_scale) F(u*, w^{n+1}) + I_stim),
// then w^{n-1} <- w^n, w^n <- w^{n+1}.
__global__ void ap_bdf2_kernel(int64_t n, double dt, double chi, double cm, mfsem_ap_params prm,
                               const double* __restrict__ V, const double* __restrict__ Vo,
                               double* __restrict__ w, double* __restrict__ wo,
                               const double* __restrict__ istim, const double* __restrict__ m,
                               double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double a1 = chi * cm / dt;
  const double fscale = chi * cm * (prm.v_amp / prm.t_scale);
  const double h = 2.0 * dt / prm.t_scale;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = V[i], vo = Vo[i];
    const double us = (2.0 * v - vo - prm.v_rest) / prm.v_amp;
    const double wn = w[i], wm = wo[i];
    const double c = prm.k * us * (us - prm.a - 1.0);
    const double r = prm.mu1 / (us + prm.mu2);
    const double qa = h * r, qb = 3.0 + h * (prm.eps0 + r * c), qc = h * prm.eps0 * c - 4.0 * wn + wm;
    // -2 qc / (qb + sqrt(qb^2 - 4 qa qc)) is the root continuous at qa = 0 (qb > 0)
    const double disc = fmax(qb * qb - 4.0 * qa * qc, 0.0);
    const double wnew = -2.0 * qc / (qb + sqrt(disc));
    const double F = prm.k * us * (1.0 - us) * (us - prm.a) - us * wnew;
    const double is = istim ? istim[i] : 0.0;
    b[i] = m[i] * (a1 * 0.5 * (4.0 * v - vo) + fscale * F + is);
    wo[i] = wn;
    w[i] = wnew;
  }
}

// Activation times (Section 5.1: the instant of the largest |du/dt| at each
// node) as a running maximum over the time loop.  V = V^{n+1} at time t and
// Vo = V^n at t - dt; the difference quotient |V - Vo|/dt estimates |du/dt| at
// the step's midpoint, so a step steeper than every earlier one (strictly:
// ties keep the earlier step) sets rate to it and act to t - dt/2.  With
// cross != NULL the first upward crossing of v_cross, interpolated linearly in
// [t - dt, t], is kept as well (a level crossing, not the activation time).
// One pass, 16 B read per node and 16-24 B read and (rarely) written.
template <bool CROSS>
__global__ void activation_kernel(int64_t n, double t, double dt, const double* __restrict__ V,
                                  const double* __restrict__ Vo, double* __restrict__ act,
                                  double* __restrict__ rate, double v_cross,
                                  double* __restrict__ cross) {
  const double t_mid = t - 0.5 * dt;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = V[i], vo = Vo[i];
    if (act) {
      const double q = fabs(v - vo) / dt;
      if (q > rate[i]) {
        rate[i] = q;
        act[i] = t_mid;
      }
    }
    if (CROSS && cross[i] < 0.0 && vo < v_cross && v >= v_cross)
      cross[i] = (t - dt) + dt * (v_cross - vo) / (v - vo);
  }
}

__global__ void extrapolate_kernel(int64_t n, const double* v, const double* vo, double* out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = 2.0 * v[i] - vo[i];
}

}  // namespace

void launch_extrapolate(int64_t n, const double* v, const double* vo, double* out, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  extrapolate_kernel<<<(unsigned)blocks, 256, 0, s>>>(n, v, vo, out);
  MFSEM_LAUNCH("extrapolate_kernel");
}

void launch_ap_bdf2(int64_t n, double dt, double chi, double cm, const mfsem_ap_params& prm,
                    const double* V, const double* Vo, double* w, double* wo, const double* istim,
                    const double* m, double* b, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  ap_bdf2_kernel<<<(unsigned)blocks, 256, 0, s>>>(n, dt, chi, cm, prm, V, Vo, w, wo, istim, m, b);
  MFSEM_LAUNCH("ap_bdf2_kernel");
}

void launch_activation(int64_t n, double t, double dt, const double* V, const double* Vo,
                       double* act, double* rate, double v_cross, double* cross, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (cross)
    activation_kernel<true><<<(unsigned)blocks, 256, 0, s>>>(n, t, dt, V, Vo, act, rate, v_cross,
                                                             cross);
  else
    activation_kernel<false><<<(unsigned)blocks, 256, 0, s>>>(n, t, dt, V, Vo, act, rate, v_cross,
                                                              cross);
  MFSEM_LAUNCH("activation_kernel");
}

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
