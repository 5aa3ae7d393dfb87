// SEM-NI apply on structured lattices, one workgroup per brick of elements.
//
// Same operator as ax_ni_kernel (Section 4.1's sum-factorised cell loop with
// the precomputed G = W|J| J^{-1} sigma J^{-T} and the diagonal GLL mass), for
// meshes whose element-to-node map is the structured box numbering.  A brick of
// BX x BY x BZ elements owns a (BX p + 1) x (BY p + 1) x (BZ p + 1) node lattice:
//   1. the lattice values of x are gathered once into LDS (rows of consecutive
//      global nodes, coalesced; node indices are computed, not loaded);
//   2. each lane takes one (a, b) pencil of one element and forms the reference
//      gradient at the pencil's P points straight from the LDS lattice;
//   3. the six G values per point are streamed from HBM and the fluxes of two
//      directions go to LDS, the third stays in registers;
//   4. the transposed 1D passes give each element node's result, which is added
//      into an LDS copy of the lattice (LDS atomics: nodes shared by elements of
//      the brick are summed on chip);
//   5. each lattice node of the brick is added into y with one global atomic.
// Compared with one gather and one scatter-add per element node, global reads of
// x and atomics drop from NE (p+1)^3 to (BX p+1)(BY p+1)(BZ p+1) per brick
// (1250 -> 1025 for the 10 x 1 x 1 bricks at p = 4), and no index array is read.
// On small meshes (a few thousand elements) one- and two-element bricks, which give the grid
// more waves, measured slower than these shapes: the extra global atomics on
// shared nodes cost more than the added parallelism gains.
#include "internal.hpp"
#include "rules.hpp"

namespace mfsem {

namespace {

constexpr int r64(int n) { return ((n + 63) / 64) * 64; }

// Brick shape per P = p+1.  The lanes (BX*BY*BZ*P^2) fill whole waves and the
// FP64 LDS footprint lets two to five workgroups share a CU; W is the number of
// waves per SIMD the register budget must allow (VGPRs <= 512/W).  Bricks are
// long along x, the fastest index of both the node lattice and the element
// order: the lattice rows a brick gathers are longer runs of consecutive nodes
// and its elements' G values are one contiguous run per (y, z) row (measured on
// the 51M-DOF slab against cube-like shapes: FP64 1-7% and FP32 3-12% faster).
// Their length keeps a workgroup near 256 lanes, so that several workgroups fit
// a CU at the register-limited occupancy: at p = 4 a 16-element brick (400
// lanes, 7 waves) left one workgroup per CU at 3 waves per SIMD, the 10-element
// brick (250 lanes) three; likewise 28 elements at p = 2 (against 32 x 2), 7 at
// p = 5 (against 8) and 5 at p = 6 (against 4, 196 lanes in 4 waves).  Measured
// FP64 on the 51M-DOF slab: p = 2 2.13 -> 1.92 ms, p = 4 1.30 -> 1.27 ms,
// p = 5 1.16 -> 1.14 ms, p = 6 1.23 -> 1.12 ms.
template <int P> struct BrickShape;
template <> struct BrickShape<2> { static constexpr int X = 32, Y = 2, Z = 1, W = 4; };
template <> struct BrickShape<3> { static constexpr int X = 28, Y = 1, Z = 1, W = 4; };
template <> struct BrickShape<4> { static constexpr int X = 16, Y = 1, Z = 1, W = 3; };
template <> struct BrickShape<5> { static constexpr int X = 10, Y = 1, Z = 1, W = 3; };
template <> struct BrickShape<6> { static constexpr int X = 7, Y = 1, Z = 1, W = 3; };
template <> struct BrickShape<7> { static constexpr int X = 5, Y = 1, Z = 1, W = 2; };
template <> struct BrickShape<8> { static constexpr int X = 2, Y = 1, Z = 2, W = 2; };
template <> struct BrickShape<9> { static constexpr int X = 2, Y = 1, Z = 1, W = 2; };

// z-rows of bricks per tile of the brick order (see the kernel), by measurement
// on the 51M-DOF slab: p = 7 (2 x 1 x 2 bricks) FP64 1.122 -> 1.063 ms with 4;
// p = 2 and 4 were slower with any tile (p = 4: 1.225 -> 1.242..1.268 ms).
template <int P>
constexpr int brick_z_tile() {
  return P == 8 ? 4 : 1;
}

// Loads in the order the kernel needs them (see the kernel), chosen per
// precision and degree by measurement on the 51M-DOF slab: FP64 p = 3 / 4 / 5
// 1.454 -> 1.448, 1.268 -> 1.237, 1.145 -> 1.128 ms, FP32 p = 5 / 6 / 7 0.585 ->
// 0.579, 0.549 -> 0.544, 0.558 -> 0.540 ms; slower at FP64 p = 2 (1.915 -> 1.930)
// and p = 7 (1.090 -> 1.136 ms); no change at FP64 p = 6 and FP32 p = 2..4.
template <typename T, int P>
constexpr bool brick_ordered_loads() {
  return sizeof(T) == 8 ? (P >= 4 && P <= 6) : (P >= 6);
}

template <int P>
struct BrickCfg {
  static constexpr int p = P - 1, P2 = P * P, P3 = P2 * P;
  static constexpr int BX = BrickShape<P>::X, BY = BrickShape<P>::Y, BZ = BrickShape<P>::Z;
  static constexpr int NE = BX * BY * BZ;
  static constexpr int LX = BX * p + 1, LY = BY * p + 1, LZ = BZ * p + 1;
  static constexpr int LN = LX * LY * LZ;
  static constexpr int THREADS = r64(NE * P2);
  static constexpr int WAVES = BrickShape<P>::W;
  // with on-the-fly geometry (FP64): the extra live values of the Jacobian fit
  // in the register budget of at most 2 waves per SIMD from P = 5 on
  static constexpr int WAVES_OTF = P >= 5 ? 2 : BrickShape<P>::W;
};

template <typename T>
__device__ inline void lds_add(T* p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// OTF: G and the mass weight are rebuilt at every point from the brick's node
// coordinates (staged in LDS, in the space the fluxes use later), the fiber at
// the point and the element's (sigma_l, sigma_t), instead of being read from
// the stored G: with C the cofactor matrix of J (J^{-1} = C^T / det J),
//   G = W |J| J^{-1} sigma J^{-T} = (W / det J) C^T sigma C,
//   sigma = sigma_t I + (sigma_l - sigma_t) f f^T / |f|^2,
// so G = (W / det J) (sigma_t C^T C + (sigma_l - sigma_t) v v^T / |f|^2), v = C^T f,
// and W |J| = W det J.  GLL points are the element's nodes, so J comes from the
// same 1D derivative rows as the gradient and f is the nodal fiber.
// G (6 values) and W|J| at point c of a lane's pencil from the LDS lattice
// coordinates cs [3][LN]; xk holds the coordinates along the pencil.
template <typename T, int P, int LX, int LY, int LN>
__device__ inline void otf_point(const T* cs, int o, int ia, int ib, int c, const T (&dx)[P],
                                 const T (&dy)[P], const T (&xk)[3][P],
                                 const T (&f)[3], bool has_fiber, T sl, T st, T W, T (&g)[6],
                                 T& wj) {
  T J[3][3];  // J[r][d] = d X_r / d xi_d
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int m = 0; m < P; ++m) {
      a0 += dx[m] * cs[r * LN + o - ia + m + LX * LY * c];
      a1 += dy[m] * cs[r * LN + o - LX * ib + LX * m + LX * LY * c];
      a2 += T(rules::GllTables<P>::D.v[c * P + m]) * xk[r][m];
    }
    J[r][0] = a0;
    J[r][1] = a1;
    J[r][2] = a2;
  }
  // cofactors C[r][d]
  const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const T c10 = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  const T c11 = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  const T c12 = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  const T c20 = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  const T c21 = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  const T c22 = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const T sc = W / det;
  T m00 = st * (c00 * c00 + c10 * c10 + c20 * c20);
  T m01 = st * (c00 * c01 + c10 * c11 + c20 * c21);
  T m02 = st * (c00 * c02 + c10 * c12 + c20 * c22);
  T m11 = st * (c01 * c01 + c11 * c11 + c21 * c21);
  T m12 = st * (c01 * c02 + c11 * c12 + c21 * c22);
  T m22 = st * (c02 * c02 + c12 * c12 + c22 * c22);
  if (has_fiber) {
    const T v0 = c00 * f[0] + c10 * f[1] + c20 * f[2];
    const T v1 = c01 * f[0] + c11 * f[1] + c21 * f[2];
    const T v2 = c02 * f[0] + c12 * f[1] + c22 * f[2];
    const T kf = (sl - st) / (f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    m00 += kf * v0 * v0;
    m01 += kf * v0 * v1;
    m02 += kf * v0 * v2;
    m11 += kf * v1 * v1;
    m12 += kf * v1 * v2;
    m22 += kf * v2 * v2;
  }
  g[0] = sc * m00;
  g[1] = sc * m01;
  g[2] = sc * m02;
  g[3] = sc * m11;
  g[4] = sc * m12;
  g[5] = sc * m22;
  wj = W * det;
}

template <typename T, int P, bool OTF>
__global__ __launch_bounds__(BrickCfg<P>::THREADS,
                             OTF ? BrickCfg<P>::WAVES_OTF : BrickCfg<P>::WAVES) void ax_brick_kernel(
    int nx, int ny, int nz, int64_t n_dof, const T* __restrict__ G, const T* __restrict__ WJ,
    const T* __restrict__ idet, const double* __restrict__ xyz, const double* __restrict__ fiber,
    const double* __restrict__ sig, double s_l, double s_t, T alpha, const T* __restrict__ Dtab,
    const T* __restrict__ wtab, const T* __restrict__ x, T* __restrict__ y) {
  using C = BrickCfg<P>;
  constexpr int p = C::p, P2 = C::P2, P3 = C::P3, NE = C::NE;
  constexpr int BX = C::BX, BY = C::BY, BZ = C::BZ, LX = C::LX, LY = C::LY, LN = C::LN;
  __shared__ T sD[P * P];
  __shared__ T sw[2 * P];  // w, then 1/w^2 (they follow each other in the tables)
  // FP32 sums the elements' contributions to a lattice node by gathering them
  // from the flux buffer (no LDS atomics: the FP32 kernel is bound by LDS
  // instructions, 6-15% faster); FP64 adds into an LDS lattice (faster there)
  constexpr bool GATHER = sizeof(T) == sizeof(float);
  __shared__ T xs[LN];
  __shared__ T ys[GATHER ? 1 : LN];
  __shared__ T F[NE * 2 * P3];
  __shared__ T cs[OTF ? 3 * LN : 1];  // OTF: lattice coordinates [3][LN]

  const int tid = threadIdx.x;
  const int nbx = (nx + BX - 1) / BX, nby = (ny + BY - 1) / BY, nbz = (nz + BZ - 1) / BZ;
  const int brick = (int)xcd_block(blockIdx.x, gridDim.x);
  // brick order: x fastest, then y, then z; with TZ > 1 the rows of bricks go
  // through tiles of TZ z-rows (z fastest within a tile, then y), so that
  // bricks sharing a z-face run close together in time on one XCD
  constexpr int TZ = brick_z_tile<P>();
  int bxi, byi, bzi;
  if constexpr (TZ == 1) {
    bxi = brick % nbx;
    byi = (brick / nbx) % nby;
    bzi = brick / (nbx * nby);
  } else {
    const int row = brick / nbx, ztile = row / (nby * TZ), rem = row - ztile * nby * TZ;
    const int nzt = min(TZ, nbz - ztile * TZ);
    bxi = brick % nbx;
    byi = rem / nzt;
    bzi = ztile * TZ + rem % nzt;
  }
  const int ex0 = bxi * BX, ey0 = byi * BY, ez0 = bzi * BZ;
  const int nex = min(BX, nx - ex0), ney = min(BY, ny - ey0), nez = min(BZ, nz - ez0);
  const int64_t NX = (int64_t)p * nx + 1, NY = (int64_t)p * ny + 1;
  const int64_t I0 = (int64_t)ex0 * p, J0 = (int64_t)ey0 * p, K0 = (int64_t)ez0 * p;
  const int bt = blockIdx.y;
  x += (int64_t)bt * n_dof;
  y += (int64_t)bt * n_dof;

  const int le = tid / P2, ab = tid % P2;
  const int ia = ab % P, ib = ab / P;
  const int lx = le % BX, ly = (le / BX) % BY, lz = le / (BX * BY);
  const bool active = le < NE && lx < nex && ly < ney && lz < nez;
  const int o = lx * p + LX * (ly * p + LY * lz * p) + ia + LX * ib;  // lattice index of (a, b, 0)
  const int64_t e = (int64_t)(ex0 + lx) + (int64_t)nx * ((ey0 + ly) + (int64_t)ny * (ez0 + lz));
  const int64_t ne_tot = (int64_t)nx * ny * nz;
  T* Fe = F + le * 2 * P3;

  // 1. issue every global load before any LDS traffic, so they are all in
  // flight together: the lattice values of x and the six G values of each of
  // the pencil's P points (the dominant HBM stream)
  // With ORD every load is issued unconditionally (out-of-range lanes read a
  // valid address and discard the value) and in the order the kernel needs
  // them: the small tables, the lattice of x, 1/det sigma, then G.  No load is
  // skipped on any path, so the wait before the LDS writes covers the tables and
  // x only and G stays in flight through the barrier and the first derivatives;
  // without ORD the table loads come last and that wait covers G too.
  constexpr bool ORD = brick_ordered_loads<T, P>();
  static_assert(!ORD || (C::THREADS >= P * P && C::THREADS >= 2 * P), "one table entry per lane");
  T dtv = 0, wtv = 0;
  if constexpr (ORD) {
    dtv = Dtab[tid < P * P ? tid : 0];
    wtv = wtab[tid < 2 * P ? tid : 0];
  }
  constexpr int NIT = (LN + C::THREADS - 1) / C::THREADS;
  T xv[NIT];
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int n = tid + it * C::THREADS;
    const int i = n % LX, j = (n / LX) % LY, k = n / (LX * LY);
    const bool in = n < LN && i <= nex * p && j <= ney * p && k <= nez * p;
    if constexpr (ORD) {
      const T v = x[in ? (I0 + i) + NX * ((J0 + j) + NY * (K0 + k)) : 0];
      xv[it] = in ? v : T(0);
    } else {
      xv[it] = in ? x[(I0 + i) + NX * ((J0 + j) + NY * (K0 + k))] : T(0);
    }
  }
  T g[P][6];
  T id = 0;
  // OTF: the lattice coordinates, the fiber at the pencil's points, sigma
  T cv[OTF ? 3 * NIT : 1];
  T fv[OTF ? P : 1][3];
  T sl = 0, st = 0;
  if constexpr (OTF) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int n = tid + it * C::THREADS;
      const int i = n % LX, j = (n / LX) % LY, k = n / (LX * LY);
      const bool in = n < LN && i <= nex * p && j <= ney * p && k <= nez * p;
      const double* src = xyz + 3 * ((I0 + i) + NX * ((J0 + j) + NY * (K0 + k)));
#pragma unroll
      for (int r = 0; r < 3; ++r) cv[3 * it + r] = in ? src[r] : T(0);
    }
    if (active) {
#pragma unroll
      for (int c = 0; c < P; ++c) {
        const int64_t node = (I0 + lx * p + ia) + NX * ((J0 + ly * p + ib) + NY * (K0 + lz * p + c));
#pragma unroll
        for (int r = 0; r < 3; ++r) fv[c][r] = fiber ? fiber[3 * node + r] : T(0);
      }
      if (sig) {
        sl = sig[((int64_t)bt * ne_tot + e) * 3];
        st = sig[((int64_t)bt * ne_tot + e) * 3 + 1];
      } else {
        sl = s_l;
        st = s_t;
      }
    }
  } else if constexpr (ORD) {
    const int64_t ec = active ? e : 0;
    const T iv = (idet ? idet : G)[(int64_t)bt * ne_tot + ec];
    const T* Ge = G + (((int64_t)bt * ne_tot + ec) * P3 + ab) * 6;
#pragma unroll
    for (int c = 0; c < P; ++c) load_g6(Ge + c * P2 * 6, g[c]);
    id = idet ? iv : T(0);
  } else if (active) {
    const T* Ge = G + (((int64_t)bt * ne_tot + e) * P3 + ab) * 6;
#pragma unroll
    for (int c = 0; c < P; ++c) load_g6(Ge + c * P2 * 6, g[c]);
    if (idet) id = idet[(int64_t)bt * ne_tot + e];
  }
  if constexpr (ORD) {
    if (tid < P * P) sD[tid] = dtv;
    if (tid < 2 * P) sw[tid] = wtv;
  } else {
    for (int i = tid; i < P * P; i += C::THREADS) sD[i] = Dtab[i];
    for (int i = tid; i < 2 * P; i += C::THREADS) sw[i] = wtab[i];
  }
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int n = tid + it * C::THREADS;
    if (n < LN) {
      xs[n] = xv[it];
      if constexpr (!GATHER) ys[n] = 0;
      if constexpr (OTF) {
#pragma unroll
        for (int r = 0; r < 3; ++r) cs[r * LN + n] = cv[3 * it + r];
      }
    }
  }
  __syncthreads();

  // this lane's rows of the 1D derivative matrix stay in registers; the
  // lane-uniform entries of the third direction are compile-time constants
  T dx[P], dy[P];
#pragma unroll
  for (int m = 0; m < P; ++m) {
    dx[m] = sD[ia * P + m];
    dy[m] = sD[ib * P + m];
  }
  const T wab = sw[ia] * sw[ib];
  const T iw2ab = sw[P + ia] * sw[P + ib];

  T u[P], ft[P], out[P];
  if (active) {
#pragma unroll
    for (int c = 0; c < P; ++c) u[c] = xs[o + LX * LY * c];
    T xk[OTF ? 3 : 1][P];  // OTF: coordinates along the pencil
    if constexpr (OTF) {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int m = 0; m < P; ++m) xk[r][m] = cs[r * LN + o + LX * LY * m];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T wjo = 0;
      if constexpr (OTF) otf_point<T, P, LX, LY, LN>(cs, o, ia, ib, c, dx, dy, xk, fv[c],
                                                    fiber != nullptr, sl, st, wab * sw[c], g[c], wjo);
      const T g00 = g[c][0], g01 = g[c][1], g02 = g[c][2];
      const T g11 = g[c][3], g12 = g[c][4], g22 = g[c][5];
      T r = 0, s = 0, t = 0;
#pragma unroll
      for (int m = 0; m < P; ++m) {
        r += dx[m] * xs[o - ia + m + LX * LY * c];
        s += dy[m] * xs[o - LX * ib + LX * m + LX * LY * c];
        t += T(rules::GllTables<P>::D.v[c * P + m]) * u[m];
      }
      const int q = c * P2 + ab;
      Fe[q] = g00 * r + g01 * s + g02 * t;
      Fe[P3 + q] = g01 * r + g11 * s + g12 * t;
      ft[c] = g02 * r + g12 * s + g22 * t;
      T wj;
      if constexpr (OTF) {
        wj = wjo;
      } else if (idet) {
        // W|J| = det G / (W^2 det sigma), with 1/W^2 from the table
        const T dG = g00 * (g11 * g22 - g12 * g12) - g01 * (g01 * g22 - g12 * g02) +
                     g02 * (g01 * g12 - g11 * g02);
        wj = dG * (id * iw2ab) * sw[P + c];
      } else {
        wj = WJ[e * P3 + q];
      }
      out[c] = alpha * wj * u[c];
    }
  }
  __syncthreads();
  // 4. transposed passes, summed into the LDS lattice
  if (active) {
    T dxt[P], dyt[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
      dxt[m] = sD[m * P + ia];
      dyt[m] = sD[m * P + ib];
    }
#pragma unroll
    for (int c = 0; c < P; ++c) {
      T v = out[c];
#pragma unroll
      for (int m = 0; m < P; ++m) {
        v += dxt[m] * Fe[c * P2 + ib * P + m];
        v += dyt[m] * Fe[P3 + c * P2 + m * P + ia];
        v += T(rules::GllTables<P>::D.v[m * P + c]) * ft[m];
      }
      if constexpr (GATHER) out[c] = v;
      else lds_add(&ys[o + LX * LY * c], v);
    }
  }
  __syncthreads();
  if constexpr (GATHER) {
    // each element's node results into the first half of its (consumed) flux space
    if (active) {
#pragma unroll
      for (int c = 0; c < P; ++c) Fe[c * P2 + ab] = out[c];
    }
    __syncthreads();
  }
  // 5. write back: every lattice node of the brick is added to y through the L2
  // atomic unit (y holds zero or the sum being accumulated into).  Plain stores
  // of the nodes no other brick touches, interleaved on the same cache lines
  // with other bricks' atomic adds, measured slower than atomics for all nodes.
  for (int n = tid; n < LN; n += blockDim.x) {
    const int i = n % LX, j = (n / LX) % LY, k = n / (LX * LY);
    if (i > nex * p || j > ney * p || k > nez * p) continue;
    T sum;
    if constexpr (GATHER) {
      // the node's contributions: one element per axis inside an element, two
      // on a face between elements of the brick (up to 8 in all)
      sum = 0;
      const int xi = i / p, yj = j / p, zk = k / p;
#pragma unroll
      for (int dz = 0; dz < 2; ++dz) {
        const int ez = zk - dz;
        if (ez < 0 || ez >= nez || (dz == 1 && k % p != 0)) continue;
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
          const int ey = yj - dy;
          if (ey < 0 || ey >= ney || (dy == 1 && j % p != 0)) continue;
#pragma unroll
          for (int dx = 0; dx < 2; ++dx) {
            const int ex = xi - dx;
            if (ex < 0 || ex >= nex || (dx == 1 && i % p != 0)) continue;
            sum += F[(ex + BX * (ey + BY * ez)) * 2 * P3 + (k - ez * p) * P2 + (j - ey * p) * P +
                     (i - ex * p)];
          }
        }
      }
    } else {
      sum = ys[n];
    }
    atomic_add(y + (I0 + i) + NX * ((J0 + j) + NY * (K0 + k)), sum);
  }
}

template <typename T, int P>
void run(const mfsem_op& op, const T* G, const T* WJ, const T* idet, const T* tab, const T* x,
         T* y, T alpha, hipStream_t s) {
  using C = BrickCfg<P>;
  const int nx = op.lat[0], ny = op.lat[1], nz = op.lat[2];
  const int64_t nb = (int64_t)((nx + C::BX - 1) / C::BX) * ((ny + C::BY - 1) / C::BY) *
                     ((nz + C::BZ - 1) / C::BZ);
  const dim3 grid((unsigned)nb, op.d.batch), block(C::THREADS);
  const double sl = op.d.sigma_const[0], st = op.d.sigma_const[1];
  // on-the-fly geometry up to P = 7: at P = 8 the coordinate lattice leaves
  // LDS for one workgroup per CU (the operator's eligibility check matches)
  if constexpr (sizeof(T) == sizeof(double) && P <= 7) {
    if (op.otf) {
      ax_brick_kernel<T, P, true><<<grid, block, 0, s>>>(
          nx, ny, nz, op.d.n_dof, nullptr, nullptr, nullptr, op.d.map_xyz, op.d.fiber,
          op.sigma_copy, sl, st, alpha, tab + op.off.Db, tab + op.off.w, x, y);
      MFSEM_LAUNCH("ax_brick_kernel (on-the-fly geometry)");
      return;
    }
  }
  ax_brick_kernel<T, P, false><<<grid, block, 0, s>>>(
      nx, ny, nz, op.d.n_dof, G, WJ, idet, nullptr, nullptr, nullptr, sl, st, alpha,
      tab + op.off.Db, tab + op.off.w, x, y);
  MFSEM_LAUNCH("ax_brick_kernel");
}

}  // namespace

template <typename T>
bool launch_brick(const mfsem_op& op, const T* G, const T* WJ, const T* idet, const T* tab,
                  const T* x, T* y, T alpha, hipStream_t s) {
  if (!op.structured || op.d.quad != MFSEM_GLL || op.d.n_elem == 0) return false;
  switch (op.P) {
    case 2: run<T, 2>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 3: run<T, 3>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 4: run<T, 4>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 5: run<T, 5>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 6: run<T, 6>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 7: run<T, 7>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 8: run<T, 8>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
    case 9: run<T, 9>(op, G, WJ, idet, tab, x, y, alpha, s); return true;
  }
  return false;
}

template bool launch_brick<double>(const mfsem_op&, const double*, const double*, const double*,
                                   const double*, const double*, double*, double, hipStream_t);
template bool launch_brick<float>(const mfsem_op&, const float*, const float*, const float*,
                                  const float*, const float*, float*, float, hipStream_t);

// ------------------------------------------------ structured-map check -------
namespace {
__global__ void lattice_check_kernel(const int32_t* __restrict__ ed, int p, int nx, int ny,
                                     int64_t n_elem, unsigned long long* bad) {
  const int P = p + 1, P3 = P * P * P;
  const int64_t NX = (int64_t)p * nx + 1, NY = (int64_t)p * ny + 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cnt = 0;
  for (; t < n_elem * P3; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = t / P3;
    const int l = (int)(t % P3);
    const int a = l % P, b = (l / P) % P, c = l / (P * P);
    const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / ((int64_t)nx * ny);
    const int64_t g = (p * ex + a) + NX * ((p * ey + b) + NY * (p * ez + c));
    if ((int64_t)ed[t] != g) ++cnt;
  }
  if (cnt) atomicAdd(bad, cnt);
}
}  // namespace

void launch_lattice_check(const mfsem_op& op, unsigned long long* bad, hipStream_t s) {
  int64_t blocks = (op.d.n_elem * op.P * op.P * op.P + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  lattice_check_kernel<<<(unsigned)blocks, 256, 0, s>>>(op.d.elem_dof, op.P - 1, op.lat[0],
                                                        op.lat[1], op.d.n_elem, bad);
  MFSEM_LAUNCH("lattice_check_kernel");
}

}  // namespace mfsem
