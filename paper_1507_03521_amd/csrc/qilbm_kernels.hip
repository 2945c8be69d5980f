// Forward kernels of the quasi-incompressible phase-field LBE step (Yang &
// Guo, Sec. III) for gfx950, and their host-side launchers.
//
// Memory: populations live in a "pull" layout: buffer slot (i, x) holds the
// post-collision population i produced at node x in the previous step, so
// the pre-collision population i at x is slot (i, x - c_i), or slot
// (opp(i), x) when x - c_i lies beyond a wall. Every kernel reads one buffer
// and writes the other; there are no in-place updates.
#include "qilbm_device.hpp"
#include "qilbm_internal.hpp"

namespace qilbm {

// ----------------------------------------------------------------- helpers
template <int P, int KOFF, int I>
__device__ __forceinline__ typename PrecT<P>::T pull_ld(const Pop<P>& in, int x, int y,
                                                        const Geom& g) {
  int plane;
  int64_t idx;
  pull_src<I>(x, y, g, plane, idx);
  return in.ld(KOFF + plane, idx);
}

template <int P, int KOFF, int I = 0>
__device__ __forceinline__ void pull9(const Pop<P>& in, int x, int y, const Geom& g,
                                      typename PrecT<P>::T v[9]) {
  if constexpr (I < 9) {
    v[I] = pull_ld<P, KOFF, I>(in, x, y, g);
    pull9<P, KOFF, I + 1>(in, x, y, g, v);
  }
}

template <typename T>
__device__ __forceinline__ void moments9(const T f[9], T& S, T& jx, T& jy) {
  S = f[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) S += f[i];
  jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
  jy = (f[2] - f[4]) + ((f[5] + f[6]) - (f[7] + f[8]));
}

template <typename T>
__device__ __forceinline__ T sum9(const T v[9]) {
  T s = v[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) s += v[i];
  return s;
}

template <typename T, typename F>
__device__ __forceinline__ void gather3x3(const F* fld, int x, int y, const Geom& g, T v[3][3]) {
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy) {
    const int64_t row = (int64_t)nbr_row(y + dy, g) * g.nx;
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) v[dy + 1][dx + 1] = T(fld[row + wrap_x(x + dx, g.nx)]);
  }
}

// -------------------------------------------------------- initial state
// f = 0 (u = 0, p = 0 => f^eq = 0) and g_i = H_i(phi0, mu0), computed in FP64
// and scattered into the pull layout (the slot each (i, x) is pulled from).
template <int P>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ phi0, Pop<P> out,
                                              Coef<double> c, Geom g) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  double v[3][3];
  gather3x3(phi0, x, y, g, v);
  double gx, gy, lap;
  stencil(v, gx, gy, lap);
  const double phi = v[1][1];
  const double mu = mu_bulk(phi, c) - c.kappa * lap;
  const double amu = c.alpha * mu;
  double h[9];
  h[0] = phi - (1.0 - 4.0 / 9.0) * amu;
#pragma unroll
  for (int i = 1; i < 9; ++i) h[i] = WGT(i) * amu;
  int plane;
  int64_t idx;
#define QILBM_SCATTER(I)                                                   \
  pull_src<I>(x, y, g, plane, idx);                                        \
  out.st(plane, idx, typename PrecT<P>::T(0));                             \
  out.st(9 + plane, idx, typename PrecT<P>::T(h[I]));
  QILBM_SCATTER(0) QILBM_SCATTER(1) QILBM_SCATTER(2) QILBM_SCATTER(3) QILBM_SCATTER(4)
  QILBM_SCATTER(5) QILBM_SCATTER(6) QILBM_SCATTER(7) QILBM_SCATTER(8)
#undef QILBM_SCATTER
}

// Canonical FP64 pre-collision state [9][ny][nx] -> pull layout.
template <int P>
__global__ __launch_bounds__(256) void k_from_canonical(const double* __restrict__ f,
                                                        const double* __restrict__ gg,
                                                        Pop<P> out, Geom g) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  int plane;
  int64_t idx;
  using T = typename PrecT<P>::T;
#define QILBM_SCATTER(I)                                                   \
  pull_src<I>(x, y, g, plane, idx);                                        \
  out.st(plane, idx, T(f[(int64_t)(I) * g.N + n]));                        \
  out.st(9 + plane, idx, T(gg[(int64_t)(I) * g.N + n]));
  QILBM_SCATTER(0) QILBM_SCATTER(1) QILBM_SCATTER(2) QILBM_SCATTER(3) QILBM_SCATTER(4)
  QILBM_SCATTER(5) QILBM_SCATTER(6) QILBM_SCATTER(7) QILBM_SCATTER(8)
#undef QILBM_SCATTER
}

// Pull layout -> canonical FP64 pre-collision state.
template <int P>
__global__ __launch_bounds__(256) void k_to_canonical(Pop<P> in, double* __restrict__ f,
                                                      double* __restrict__ gg, Geom g) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  using T = typename PrecT<P>::T;
  T a[9], b[9];
  pull9<P, 0>(in, x, y, g, a);
  pull9<P, 9>(in, x, y, g, b);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    f[(int64_t)i * g.N + n] = double(a[i]);
    gg[(int64_t)i * g.N + n] = double(b[i]);
  }
}

// ------------------------------------------------- unfused step (4 kernels)
// phi = sum_i g_i of the pulled populations.
template <int P>
__global__ __launch_bounds__(256) void k_phi(Pop<P> in, typename PrecT<P>::T* __restrict__ phi,
                                             Geom g) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  typename PrecT<P>::T v[9];
  pull9<P, 9>(in, x, y, g, v);
  phi[n] = sum9(v);
}

// mu = mu_bulk(phi) - kappa lap phi.
template <typename T>
__global__ __launch_bounds__(256) void k_mu(const T* __restrict__ phi, T* __restrict__ mu,
                                            Coef<T> c, Geom g) {
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  T v[3][3];
  gather3x3(phi, x, y, g, v);
  T gx, gy, lap;
  stencil(v, gx, gy, lap);
  mu[n] = mu_bulk(v[1][1], c) - c.kappa * lap;
}

// Node macroscopic state from pulled f and the phi, mu fields.
template <int P>
__device__ __forceinline__ void node_macro(const Pop<P>& in, const typename PrecT<P>::T* phi,
                                           const typename PrecT<P>::T* mu, int x, int y,
                                           const Coef<typename PrecT<P>::T>& c, const Geom& g,
                                           typename PrecT<P>::T f[9],
                                           Macro<typename PrecT<P>::T>& m) {
  using T = typename PrecT<P>::T;
  pull9<P, 0>(in, x, y, g, f);
  T S, jx, jy;
  moments9(f, S, jx, jy);
  T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu;
  gather3x3(phi, x, y, g, v);
  stencil(v, gphx, gphy, lapphi);
  const T ph = v[1][1];
  gather3x3(mu, x, y, g, v);
  stencil(v, gmux, gmuy, lapmu);
  macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, c, m);
}

// Pressure field (and, optionally, the FP64 moment outputs).
template <int P>
__global__ __launch_bounds__(256) void k_macro(Pop<P> in, const typename PrecT<P>::T* __restrict__ phi,
                                               const typename PrecT<P>::T* __restrict__ mu,
                                               typename PrecT<P>::T* __restrict__ p,
                                               MomentOut mo, Coef<typename PrecT<P>::T> c, Geom g) {
  using T = typename PrecT<P>::T;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  T f[9];
  Macro<T> m;
  node_macro<P>(in, phi, mu, x, y, c, g, f, m);
  if (p) p[n] = m.p;
  if (mo.phi) mo.phi[n] = double(m.phi);
  if (mo.rho) mo.rho[n] = double(m.rho);
  if (mo.ux) mo.ux[n] = double(m.ux);
  if (mo.uy) mo.uy[n] = double(m.uy);
  if (mo.p) mo.p[n] = double(m.p);
  if (mo.mu) mo.mu[n] = double(m.mu);
}

template <int P>
__device__ __forceinline__ void store_node(const Pop<P>& out, int64_t n,
                                           const typename PrecT<P>::T f[9],
                                           const typename PrecT<P>::T gg[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) out.st(i, n, f[i]);
#pragma unroll
  for (int i = 0; i < 9; ++i) out.st(9 + i, n, gg[i]);
}

// Collision with all fields materialised; post-collision values stay at
// their node (pull layout).
template <int P>
__global__ __launch_bounds__(256) void k_collide(Pop<P> in, Pop<P> out,
                                                 const typename PrecT<P>::T* __restrict__ phi,
                                                 const typename PrecT<P>::T* __restrict__ mu,
                                                 const typename PrecT<P>::T* __restrict__ p,
                                                 Coef<typename PrecT<P>::T> c, Geom g) {
  using T = typename PrecT<P>::T;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  T f[9], gg[9];
  Macro<T> m;
  node_macro<P>(in, phi, mu, x, y, c, g, f, m);
  pull9<P, 9>(in, x, y, g, gg);
  T v[3][3], dpx, dpy, lapp;
  gather3x3(p, x, y, g, v);
  stencil(v, dpx, dpy, lapp);
  collide_node(f, gg, m, dpx, dpy, c);
  store_node<P>(out, n, f, gg);
}

// ------------------------------------------------------- mass reduction
// Per-block FP64 partials of (sum phi, sum rho, sum rho ux, sum rho uy) over
// a fixed node-to-thread assignment, reduced with wave64 shuffles; a single
// block then adds the partials in a fixed order. Bitwise reproducible.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ void block_sum4(double a[4], double* out) {
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) a[k] = wave_sum(a[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) red[wave][k] = a[k];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    out[k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
  }
}

template <int P>
__global__ __launch_bounds__(256) void k_mass_partial(Pop<P> in,
                                                      const typename PrecT<P>::T* __restrict__ phi,
                                                      const typename PrecT<P>::T* __restrict__ mu,
                                                      double* __restrict__ part,
                                                      Coef<typename PrecT<P>::T> c, Geom g) {
  using T = typename PrecT<P>::T;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N;
       n += (int64_t)gridDim.x * 256) {
    const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
    T f[9];
    Macro<T> m;
    node_macro<P>(in, phi, mu, x, y, c, g, f, m);
    a[0] += double(m.phi);
    a[1] += double(m.rho);
    a[2] += double(m.rho) * double(m.ux);
    a[3] += double(m.rho) * double(m.uy);
  }
  block_sum4(a, part + 4 * blockIdx.x);
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nb,
                                                      int width, double* __restrict__ out) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] += k < width ? part[width * b + k] : 0.0;
  }
  block_sum4(a, out);
}

// ------------------------------------------------------ fused step kernel
// One pass over the lattice per time step. A workgroup owns a strip of
// FW columns (plus FH halo columns on each side) and a segment of rows, and
// sweeps the rows upwards keeping a ring of recent rows of phi, mu and p in
// LDS. In the iteration that brings in row r it
//   A: pulls g at row r and forms phi(r) (also on the halo columns),
//   B: forms mu(r-1) from the phi rows r-2..r,
//   C: pulls f at row r-2 and forms the force, velocity and pressure there,
//   D: collides row r-3, whose grad p now has all three p rows, and writes
//      both post-collision populations.
// The g values of a row are kept in registers from A to D (ring of four
// rows), the f values from C to D (ring of two), so each population is read
// once from memory and written once. Halo columns and the 3 rows of warm-up
// at each segment end are recomputed by neighbouring workgroups.
constexpr int FW = 256;
constexpr int FH = 3;
constexpr int FL = FW + 2 * FH;
constexpr int FT = FW + 64;

// Tiles handed out so that blocks that the hardware places on one XCD
// (consecutive blocks round-robin over 8 XCDs) get consecutive tiles, i.e.
// vertically adjacent segments of one strip share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  const int q = n >> 3, rem = n & 7, j = bid & 7, pos = bid >> 3;
  return j * q + (j < rem ? j : rem) + pos;
}

template <int P>
struct FusedCtx {
  using T = typename PrecT<P>::T;
  Pop<P> in, out;
  Coef<T> c;
  Geom g;
  int lc, x, wi, y0, y1;
  bool act;
};

template <typename T>
__device__ __forceinline__ void lds3x3(const T (*ring)[FL], int mask, int v, int ny, int walls,
                                       int lc, T out[3][3]) {
  const int vm = (walls && v == 0) ? v : v - 1;
  const int vp = (walls && v == ny - 1) ? v : v + 1;
  const T* a = ring[vm & mask];
  const T* b = ring[v & mask];
  const T* d = ring[vp & mask];
  out[0][0] = a[lc - 1]; out[0][1] = a[lc]; out[0][2] = a[lc + 1];
  out[1][0] = b[lc - 1]; out[1][1] = b[lc]; out[1][2] = b[lc + 1];
  out[2][0] = d[lc - 1]; out[2][1] = d[lc]; out[2][2] = d[lc + 1];
}

__device__ __forceinline__ int phys_row(int v, const Geom& g) {
  if (g.walls) return v;
  int r = v % g.ny;
  return r < 0 ? r + g.ny : r;
}

__device__ __forceinline__ bool row_ok(int v, const Geom& g) {
  return !g.walls || (v >= 0 && v < g.ny);
}

template <int P, int J>
__device__ __forceinline__ void fused_iter(const FusedCtx<P>& k, int r,
                                           typename PrecT<P>::T (&gb)[4][9],
                                           typename PrecT<P>::T (&fb)[2][9],
                                           typename PrecT<P>::T (*s_phi)[FL],
                                           typename PrecT<P>::T (*s_mu)[FL],
                                           typename PrecT<P>::T (*s_p)[FL]) {
  using T = typename PrecT<P>::T;
  const Geom& g = k.g;
  const int lc = k.lc;
  // A: phi at row r
  if (k.act && r < k.y1 + 3 && row_ok(r, g)) {
    pull9<P, 9>(k.in, k.x, phys_row(r, g), g, gb[J]);
    s_phi[r & 7][lc] = sum9(gb[J]);
  }
  __syncthreads();
  // B: mu at row r - 1
  const int b = r - 1;
  if (k.act && lc >= 1 && lc < k.wi + 5 && b >= k.y0 - 2 && b < k.y1 + 2 && row_ok(b, g)) {
    T v[3][3], gx, gy, lap;
    lds3x3<T>(s_phi, 7, b, g.ny, g.walls, lc, v);
    stencil(v, gx, gy, lap);
    s_mu[b & 3][lc] = mu_bulk(v[1][1], k.c) - k.c.kappa * lap;
  }
  __syncthreads();
  // C: force, velocity, pressure at row r - 2
  const int q = r - 2;
  if (k.act && lc >= 2 && lc < k.wi + 4 && q >= k.y0 - 1 && q < k.y1 + 1 && row_ok(q, g)) {
    pull9<P, 0>(k.in, k.x, phys_row(q, g), g, fb[J & 1]);
    T S, jx, jy;
    moments9(fb[J & 1], S, jx, jy);
    T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu;
    lds3x3<T>(s_phi, 7, q, g.ny, g.walls, lc, v);
    stencil(v, gphx, gphy, lapphi);
    const T ph = v[1][1];
    lds3x3<T>(s_mu, 3, q, g.ny, g.walls, lc, v);
    stencil(v, gmux, gmuy, lapmu);
    Macro<T> m;
    macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, k.c, m);
    s_p[q & 3][lc] = m.p;
  }
  __syncthreads();
  // D: collide row r - 3 and store
  const int cr = r - 3;
  if (k.act && lc >= FH && lc < k.wi + FH && cr >= k.y0 && cr < k.y1) {
    T* f = fb[(J + 1) & 1];
    T* gg = gb[(J + 1) & 3];
    T S, jx, jy;
    moments9(f, S, jx, jy);
    T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu, dpx, dpy, lapp;
    lds3x3<T>(s_phi, 7, cr, g.ny, g.walls, lc, v);
    stencil(v, gphx, gphy, lapphi);
    const T ph = v[1][1];
    lds3x3<T>(s_mu, 3, cr, g.ny, g.walls, lc, v);
    stencil(v, gmux, gmuy, lapmu);
    Macro<T> m;
    macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, k.c, m);
    lds3x3<T>(s_p, 3, cr, g.ny, g.walls, lc, v);
    stencil(v, dpx, dpy, lapp);
    collide_node(f, gg, m, dpx, dpy, k.c);
    store_node<P>(k.out, (int64_t)cr * g.nx + k.x, f, gg);
  }
}

template <int P>
__global__ __launch_bounds__(FT) void k_step_fused(Pop<P> in, Pop<P> out,
                                                   Coef<typename PrecT<P>::T> c, Geom g, int nseg,
                                                   int seg_len) {
  using T = typename PrecT<P>::T;
  __shared__ T s_phi[8][FL];
  __shared__ T s_mu[4][FL];
  __shared__ T s_p[4][FL];
  FusedCtx<P> k;
  k.in = in;
  k.out = out;
  k.c = c;
  k.g = g;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int strip = tile / nseg, seg = tile - strip * nseg;
  const int x0 = strip * FW;
  k.wi = min(FW, g.nx - x0);
  k.y0 = seg * seg_len;
  k.y1 = min(g.ny, k.y0 + seg_len);
  const int t = threadIdx.x;
  int lc = -1;
  if (t < FW) {
    lc = t < k.wi ? t + FH : -1;
  } else {
    const int j = t - FW;
    lc = j < FH ? j : (j < 2 * FH ? k.wi + j : -1);
  }
  k.lc = lc < 0 ? FH : lc;
  k.act = lc >= 0;
  k.x = wrap_x(x0 + k.lc - FH, g.nx);
  T gb[4][9];
  T fb[2][9];
  const int r0 = k.y0 - 3;
  const int nit = (k.y1 - k.y0) + 6;
  for (int it = 0; it < nit; it += 4) {
    fused_iter<P, 0>(k, r0 + it + 0, gb, fb, s_phi, s_mu, s_p);
    fused_iter<P, 1>(k, r0 + it + 1, gb, fb, s_phi, s_mu, s_p);
    fused_iter<P, 2>(k, r0 + it + 2, gb, fb, s_phi, s_mu, s_p);
    fused_iter<P, 3>(k, r0 + it + 3, gb, fb, s_phi, s_mu, s_p);
  }
}

// --------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <int P>
hipError_t launch_init(const double* phi0, void* pop, const Coef<double>& c, const Geom& g,
                       hipStream_t s) {
  Pop<P> o{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_init<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, phi0, o, c, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_from_canonical(const double* f, const double* gg, void* pop, const Geom& g,
                                 hipStream_t s) {
  Pop<P> o{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_from_canonical<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, f, gg, o, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_to_canonical(const void* pop, double* f, double* gg, const Geom& g,
                               hipStream_t s) {
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_to_canonical<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, f, gg, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_fields(const void* pop, void* phi, void* mu,
                         const Coef<typename PrecT<P>::T>& c, const Geom& g, hipStream_t s) {
  using T = typename PrecT<P>::T;
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_phi<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, (T*)phi, g);
  hipLaunchKernelGGL(k_mu<T>, dim3(nblk(g.N, 256)), dim3(256), 0, s, (const T*)phi, (T*)mu, c, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_macro(const void* pop, const void* phi, const void* mu, void* p,
                        const MomentOut& mo, const Coef<typename PrecT<P>::T>& c, const Geom& g,
                        hipStream_t s) {
  using T = typename PrecT<P>::T;
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_macro<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, (const T*)phi,
                     (const T*)mu, (T*)p, mo, c, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_step_unfused(const void* pin, void* pout, void* phi, void* mu, void* p,
                               const Coef<typename PrecT<P>::T>& c, const Geom& g,
                               hipStream_t s) {
  using T = typename PrecT<P>::T;
  hipError_t e = launch_fields<P>(pin, phi, mu, c, g, s);
  if (e != hipSuccess) return e;
  e = launch_macro<P>(pin, phi, mu, p, MomentOut{}, c, g, s);
  if (e != hipSuccess) return e;
  Pop<P> i{(char*)pin, g.Ns}, o{(char*)pout, g.Ns};
  hipLaunchKernelGGL(k_collide<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, o, (const T*)phi,
                     (const T*)mu, (const T*)p, c, g);
  return hipGetLastError();
}

FusedShape fused_shape(const Geom& g, int seg_rows) {
  FusedShape sh;
  sh.nstrips = (g.nx + FW - 1) / FW;
  if (seg_rows <= 0) {
    // about 2048 workgroups in flight: 8 per CU on 256 CUs, rows >= 16
    const int want = (2048 + sh.nstrips - 1) / sh.nstrips;
    seg_rows = (g.ny + want - 1) / want;
    if (seg_rows < 16) seg_rows = 16;
  }
  if (seg_rows > g.ny) seg_rows = g.ny;
  sh.seg_rows = seg_rows;
  sh.nseg = (g.ny + seg_rows - 1) / seg_rows;
  sh.threads = FT;
  return sh;
}

template <int P>
hipError_t launch_step_fused(const void* pin, void* pout, const Coef<typename PrecT<P>::T>& c,
                             const Geom& g, const FusedShape& sh, hipStream_t s) {
  Pop<P> i{(char*)pin, g.Ns}, o{(char*)pout, g.Ns};
  hipLaunchKernelGGL(k_step_fused<P>, dim3(sh.nstrips * sh.nseg), dim3(FT), 0, s, i, o, c, g,
                     sh.nseg, sh.seg_rows);
  return hipGetLastError();
}

template <int P>
hipError_t launch_mass(const void* pop, void* phi, void* mu, double* part, int nred, double* out,
                       const Coef<typename PrecT<P>::T>& c, const Geom& g, hipStream_t s) {
  using T = typename PrecT<P>::T;
  hipError_t e = launch_fields<P>(pop, phi, mu, c, g, s);
  if (e != hipSuccess) return e;
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_mass_partial<P>, dim3(nred), dim3(256), 0, s, i, (const T*)phi,
                     (const T*)mu, part, c, g);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, (const double*)part, nred, 4, out);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* part, int nb, int width, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, width, out);
  return hipGetLastError();
}

#define QILBM_INSTANTIATE(P)                                                                     \
  template hipError_t launch_init<P>(const double*, void*, const Coef<double>&, const Geom&,     \
                                     hipStream_t);                                               \
  template hipError_t launch_from_canonical<P>(const double*, const double*, void*, const Geom&, \
                                               hipStream_t);                                     \
  template hipError_t launch_to_canonical<P>(const void*, double*, double*, const Geom&,         \
                                             hipStream_t);                                       \
  template hipError_t launch_fields<P>(const void*, void*, void*,                                \
                                       const Coef<PrecT<P>::T>&, const Geom&, hipStream_t);      \
  template hipError_t launch_macro<P>(const void*, const void*, const void*, void*,              \
                                      const MomentOut&, const Coef<PrecT<P>::T>&, const Geom&,   \
                                      hipStream_t);                                              \
  template hipError_t launch_step_unfused<P>(const void*, void*, void*, void*, void*,            \
                                             const Coef<PrecT<P>::T>&, const Geom&, hipStream_t); \
  template hipError_t launch_step_fused<P>(const void*, void*, const Coef<PrecT<P>::T>&,         \
                                           const Geom&, const FusedShape&, hipStream_t);         \
  template hipError_t launch_mass<P>(const void*, void*, void*, double*, int, double*,           \
                                     const Coef<PrecT<P>::T>&, const Geom&, hipStream_t);

QILBM_INSTANTIATE(P_F64)
QILBM_INSTANTIATE(P_F32)
QILBM_INSTANTIATE(P_F16)

}  // namespace qilbm
