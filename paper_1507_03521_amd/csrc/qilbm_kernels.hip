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
  uint32_t idx;
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
  uint32_t idx;
  // H_i rounded once to the storage format (Q2.29 words exactly)
#define QILBM_SCATTER(I)                                                   \
  pull_src<I>(x, y, g, plane, idx);                                        \
  out.st_exact(plane, idx, 0.0);                                           \
  out.st_exact(9 + plane, idx, h[I]);
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
  uint32_t idx;
  // one rounding from binary64 to the storage format (Q2.29 g words exactly)
#define QILBM_SCATTER(I)                                                   \
  pull_src<I>(x, y, g, plane, idx);                                        \
  out.st_exact(plane, idx, f[(int64_t)(I) * g.N + n]);                     \
  out.st_exact(9 + plane, idx, gg[(int64_t)(I) * g.N + n]);
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
  int plane;
  uint32_t idx;
  // the stored values exactly (Q2.29 g words included)
#define QILBM_GATHER(I)                                                    \
  pull_src<I>(x, y, g, plane, idx);                                        \
  f[(int64_t)(I) * g.N + n] = in.ld_canon(plane, idx);                     \
  gg[(int64_t)(I) * g.N + n] = in.ld_canon(9 + plane, idx);
  QILBM_GATHER(0) QILBM_GATHER(1) QILBM_GATHER(2) QILBM_GATHER(3) QILBM_GATHER(4)
  QILBM_GATHER(5) QILBM_GATHER(6) QILBM_GATHER(7) QILBM_GATHER(8)
#undef QILBM_GATHER
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
                                           Macro<typename PrecT<P>::T>& m,
                                           typename PrecT<P>::T& S, typename PrecT<P>::T& jx,
                                           typename PrecT<P>::T& jy) {
  using T = typename PrecT<P>::T;
  pull9<P, 0>(in, x, y, g, f);
  moments9(f, S, jx, jy);
  T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu;
  gather3x3(phi, x, y, g, v);
  stencil(v, gphx, gphy, lapphi);
  const T ph = v[1][1];
  gather3x3(mu, x, y, g, v);
  stencil(v, gmux, gmuy, lapmu);
  macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, c, m);
}

// Pressure field (and, optionally, S = sum f and j = sum c f into three
// planes at sj, and the FP64 moment outputs).
template <int P>
__global__ __launch_bounds__(256) void k_macro(Pop<P> in, const typename PrecT<P>::T* __restrict__ phi,
                                               const typename PrecT<P>::T* __restrict__ mu,
                                               typename PrecT<P>::T* __restrict__ p,
                                               typename PrecT<P>::T* __restrict__ sj,
                                               MomentOut mo, Coef<typename PrecT<P>::T> c, Geom g) {
  using T = typename PrecT<P>::T;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  T f[9], S, jx, jy;
  Macro<T> m;
  node_macro<P>(in, phi, mu, x, y, c, g, f, m, S, jx, jy);
  if (p) p[n] = m.p;
  if (sj) {
    sj[n] = S;
    sj[g.Ns + n] = jx;
    sj[2 * g.Ns + n] = jy;
  }
  if (mo.phi) mo.phi[n] = double(m.phi);
  if (mo.rho) mo.rho[n] = double(m.rho);
  if (mo.ux) mo.ux[n] = double(m.ux);
  if (mo.uy) mo.uy[n] = double(m.uy);
  if (mo.p) mo.p[n] = double(m.p);
  if (mo.mu) mo.mu[n] = double(m.mu);
}

// Stores a node's post-collision populations. In the fixed-point modes g_0
// is written as phi_q - sum_{i>=1} q(g_i), phi_q being the exact Q2.29 sum
// of the node's pre-collision g, so the stored g of the node sum exactly to
// phi_q.
template <int P>
__device__ __forceinline__ void store_node(const Pop<P>& out, uint32_t n,
                                           const typename PrecT<P>::T f[9],
                                           const typename PrecT<P>::T gg[9], int32_t phi_q) {
#pragma unroll
  for (int i = 0; i < 9; ++i) out.st(i, n, f[i]);
  if constexpr (FixedG<P>::value) {
    int32_t rest = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) rest += out.st(9 + i, n, gg[i]);
    out.st_g0_q(n, phi_q - rest);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) out.st(9 + i, n, gg[i]);
  }
}

// Exact Q2.29 sum of the pulled g of node (x, y) (fixed-point modes).
template <int P, int I = 0>
__device__ __forceinline__ int32_t pull_phi_q(const Pop<P>& in, int x, int y, const Geom& g) {
  if constexpr (I < 9) {
    int plane;
    uint32_t idx;
    pull_src<I>(x, y, g, plane, idx);
    return in.ld_q(9 + plane, idx) + pull_phi_q<P, I + 1>(in, x, y, g);
  } else {
    return 0;
  }
}

// Exact binary64 sum of the pulled g of node (x, y).
template <int P, int I = 0>
__device__ __forceinline__ double pull_phi_exact(const Pop<P>& in, int x, int y, const Geom& g) {
  if constexpr (I < 9) {
    int plane;
    uint32_t idx;
    pull_src<I>(x, y, g, plane, idx);
    return in.ld_exact(9 + plane, idx) + pull_phi_exact<P, I + 1>(in, x, y, g);
  } else {
    return 0.0;
  }
}

// Collision with all fields materialised; post-collision values stay at
// their node (pull layout).
template <int P, bool TRT = false>
__global__ __launch_bounds__(256) void k_collide(Pop<P> in, Pop<P> out,
                                                 const typename PrecT<P>::T* __restrict__ phi,
                                                 const typename PrecT<P>::T* __restrict__ mu,
                                                 const typename PrecT<P>::T* __restrict__ p,
                                                 Coef<typename PrecT<P>::T> c, Geom g) {
  using T = typename PrecT<P>::T;
  const int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (n >= g.N) return;
  const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
  T f[9], gg[9], S, jx, jy;
  Macro<T> m;
  node_macro<P>(in, phi, mu, x, y, c, g, f, m, S, jx, jy);
  pull9<P, 9>(in, x, y, g, gg);
  T v[3][3], dpx, dpy, lapp;
  gather3x3(p, x, y, g, v);
  stencil(v, dpx, dpy, lapp);
  int32_t phi_q = 0;
  if constexpr (FixedG<P>::value) phi_q = pull_phi_q<P>(in, x, y, g);
  if constexpr (TRT) collide_node_trt(f, gg, m, dpx, dpy, c);
  else collide_node(f, gg, m, dpx, dpy, c);
  store_node<P>(out, (uint32_t)n, f, gg, phi_q);
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
                                                      Coef<typename PrecT<P>::T> c,
                                                      double rho_B, double drho, Geom g) {
  using T = typename PrecT<P>::T;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N;
       n += (int64_t)gridDim.x * 256) {
    const int y = (int)(n / g.nx), x = (int)(n - (int64_t)y * g.nx);
    T f[9], S, jx, jy;
    Macro<T> m;
    node_macro<P>(in, phi, mu, x, y, c, g, f, m, S, jx, jy);
    // phi and rho from the exact stored values and the binary64 density
    // parameters (so that the totals show the scheme's conservation rather
    // than the rounding of the compute type)
    const double ph = pull_phi_exact<P>(in, x, y, g);
    const double rho = rho_B + drho * ph;
    a[0] += ph;
    a[1] += rho;
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
// One pass over the lattice per time step. A workgroup of NT lanes owns a
// strip of at most NT - 2 FH columns plus FH halo columns on each side
// (lane lc <-> column x0 - FH + lc) and a segment of rows, and sweeps the
// rows in direction d (+1 or -1) keeping rings of recent rows of phi, mu,
// p and the node state in LDS. In the iteration that brings in row r it
//   A: forms phi(r) from the pulled g of row r (halo lanes included),
//   B: forms mu(r-d) from the phi rows r-2d..r,
//   C: forms force, velocity and pressure at row r-2d from its pulled f and
//      keeps them in LDS,
//   D: collides row r-3d, whose grad p now has all three p rows, and writes
//      both post-collision populations.
// The g values of a row stay in registers from A to D (ring of four rows),
// the f values from C to D (ring of two), so each population is read once
// from memory and written once. D first moves its row out of the rings and
// refills the freed slots with the loads of the next iteration (g of row
// r+d, f of row r-d), so their latency overlaps the collision, the stores
// and the barrier. Halo columns and the 3 rows of warm-up at each segment
// end are recomputed by the neighbouring workgroups.
constexpr int FH = 3;           // halo columns per side
constexpr int NM = 7;           // node values kept from C to D

// Population access of the fused kernel through buffer resources: one
// descriptor each for the f planes, the g_0 plane and the g_1..8 planes.
// The plane and row parts of an address are uniform over a wavefront and go
// into the scalar offset; the lane's column is one of three precomputed
// byte offsets (x - 1, x, x + 1). Loads beyond a descriptor's range return 0.
// Loads return the raw storage word (R), decoded only where the value is
// first used, so that a prefetched load is not waited for early.

template <int P> struct BufT;
template <> struct BufT<P_F64> { using F = double; using G0 = double; using GR = double; using R = double; };
// FP32: GR is the 64-bit word that holds f_i (low word, binary32) and g_i
// (high word, Q2.29), i = 0..8.
template <> struct BufT<P_F32> { using F = float; using G0 = int32_t; using GR = uint64_t; using R = uint64_t; };
// FP16 storage: F is the f_0 plane's binary16; GR the 32-bit word that holds
// f_i (low half) and g_i (high half), i >= 1.
template <> struct BufT<P_F16> { using F = __half; using G0 = int32_t; using GR = uint32_t; using R = uint32_t; };

// BIG: a group of population planes (f_0..8 or g_1..8) spans 4 GiB or more,
// beyond the 32-bit range of one descriptor (FP64: more than 2 GiB, see
// fused_big); every access then builds a
// descriptor for its own plane (scalar work only) and the scalar offset
// holds the row alone.
template <int P, bool BIG = false>
struct BufPop {
  using T = typename PrecT<P>::T;
  using F = typename BufT<P>::F;
  using G0 = typename BufT<P>::G0;
  using GR = typename BufT<P>::GR;
  using R = typename BufT<P>::R;
  // paired layouts: FP32 keeps (f_i, g_i) in one 64-bit word for i = 0..8,
  // FP16 storage in one 32-bit word for i = 1..8
  static constexpr bool PAIRED = P != P_F64;
  static constexpr int G_FIRST = P == P_F32 ? 0 : 1;   // first direction of the g group
  __amdgpu_buffer_rsrc_t rf, rg0, rgr;
  uint32_t pf, pg;     // plane strides (bytes) of the f and g (or pair) planes
  char *fp, *gp;       // first f plane and first g (or pair) plane

  __device__ __forceinline__ void init(const Pop<P>& p) {
    const int64_t Ns = p.Ns;
    char* b = p.base;
    char *f, *g0, *gr;
    if constexpr (P == P_F16) {
      f = b;
      g0 = b + 2 * Ns;
      gr = b + 6 * Ns;
    } else if constexpr (P == P_F32) {
      f = b;
      g0 = b;
      gr = b;
    } else {
      f = b;
      g0 = b + 9 * Ns * (int64_t)sizeof(T);
      gr = b + 10 * Ns * (int64_t)sizeof(T);
    }
    fp = f;
    gp = gr;
    pf = (uint32_t)(Ns * sizeof(F));
    pg = (uint32_t)(Ns * sizeof(GR));
    rg0 = __builtin_amdgcn_make_buffer_rsrc(g0, 0, (int)(Ns * sizeof(G0)), BUF_WORD3);
    if constexpr (!BIG) {
      rf = __builtin_amdgcn_make_buffer_rsrc(f, 0, (int)((P == P_F16 ? 1 : 9) * (int64_t)pf),
                                             BUF_WORD3);
      rgr = __builtin_amdgcn_make_buffer_rsrc(gr, 0, (int)((9 - G_FIRST) * (int64_t)pg), BUF_WORD3);
    }
  }
  template <typename S>
  __device__ __forceinline__ static R raw(S v) {
    if constexpr (sizeof(S) == 8) return v;
    else if constexpr (sizeof(S) == 4) return __builtin_bit_cast(uint32_t, v);
    else return (uint32_t)__builtin_bit_cast(uint16_t, v);
  }
  // descriptor and scalar offset of f_I / g_I (I >= 1) at element row elem_row
  template <int I>
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t f_rsrc() const {
    if constexpr (BIG) return __builtin_amdgcn_make_buffer_rsrc(fp + (int64_t)I * pf, 0, (int)pf, BUF_WORD3);
    else return rf;
  }
  template <int I>
  __device__ __forceinline__ uint32_t f_soff(uint32_t elem_row) const {
    return (BIG ? 0u : I * pf) + elem_row * (uint32_t)sizeof(F);
  }
  template <int I>
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t g_rsrc() const {
    if constexpr (BIG) return __builtin_amdgcn_make_buffer_rsrc(gp + (int64_t)(I - G_FIRST) * pg, 0, (int)pg, BUF_WORD3);
    else return rgr;
  }
  template <int I>
  __device__ __forceinline__ uint32_t g_soff(uint32_t elem_row) const {
    return (BIG ? 0u : (I - G_FIRST) * pg) + elem_row * (uint32_t)sizeof(GR);
  }
  // raw word of f_I (G = false) or g_I (G = true) at element (row, col[dx+1])
  template <bool G, int I>
  __device__ __forceinline__ R ld(uint32_t elem_row, const uint32_t col[3], int dx) const {
    if constexpr (P == P_F32 || (P == P_F16 && I >= 1)) {
      // the pair word of direction I (f_I low part, g_I high part)
      return buf_ld<GR>(g_rsrc<I>(), col[dx + 1] * (uint32_t)sizeof(GR), g_soff<I>(elem_row));
    } else if constexpr (!G) {
      return raw(buf_ld<F>(f_rsrc<I>(), col[dx + 1] * (uint32_t)sizeof(F), f_soff<I>(elem_row)));
    } else if constexpr (I == 0) {
      return raw(buf_ld<G0>(rg0, col[dx + 1] * (uint32_t)sizeof(G0),
                            elem_row * (uint32_t)sizeof(G0)));
    } else {
      return raw(buf_ld<GR>(g_rsrc<I>(), col[dx + 1] * (uint32_t)sizeof(GR), g_soff<I>(elem_row)));
    }
  }
  // decoded values of raw words
  template <int I>
  __device__ __forceinline__ static T val_f(R w) {
    if constexpr (P == P_F64) return w;
    else if constexpr (P == P_F32) return __builtin_bit_cast(float, (uint32_t)w);
    else return __half2float(__builtin_bit_cast(__half, (uint16_t)w)) * H_INV(I);
  }
  template <int I>
  __device__ __forceinline__ static T val_g(R w) {
    if constexpr (P == P_F64) return w;
    else if constexpr (P == P_F32) return float((int32_t)(uint32_t)(w >> 32)) * GQI;
    else if constexpr (I == 0) return float((int32_t)w) * GQI;
    else return __half2float(__builtin_bit_cast(__half, (uint16_t)(w >> 16))) * H_INV(I);
  }
  // Q2.29 contribution of a raw g word (fixed-point modes)
  template <int I>
  __device__ __forceinline__ static int32_t q_g(R w) {
    if constexpr (P == P_F32) return (int32_t)(uint32_t)(w >> 32);
    else if constexpr (I == 0) return (int32_t)w;
    else return q_half(__builtin_bit_cast(__half, (uint16_t)(w >> 16)), I);
  }
  // vb (stores): added to the lane's vector offset; 0x80000000 puts the
  // store beyond a descriptor of at most 2 GiB, where the hardware drops it
  template <int I>
  __device__ __forceinline__ void st_f(T v, uint32_t elem_row, uint32_t col,
                                       uint32_t vb = 0) const {
    F w;
    if constexpr (P == P_F16) w = __float2half_rn(v * H_SCALE(I));
    else w = v;
    buf_st<F>(w, f_rsrc<I>(), col * (uint32_t)sizeof(F) + vb, f_soff<I>(elem_row));
  }
  // stores g_I (I >= 1); returns its Q2.29 contribution in the fixed-point modes
  template <int I>
  __device__ __forceinline__ int32_t st_g(T v, uint32_t elem_row, uint32_t col,
                                          uint32_t vb = 0) const {
    const uint32_t so = g_soff<I>(elem_row);
    if constexpr (P == P_F64) {
      buf_st<GR>(v, g_rsrc<I>(), col * (uint32_t)sizeof(GR) + vb, so);
      return 0;
    } else if constexpr (P == P_F32) {
      const int32_t q = __float2int_rn(v * GQ);
      buf_st<GR>(q, g_rsrc<I>(), col * (uint32_t)sizeof(GR), so);
      return q;
    } else {
      const __half h = __float2half_rn(v * H_SCALE(I));
      buf_st<GR>(h, g_rsrc<I>(), col * (uint32_t)sizeof(GR), so);
      return q_half(h, I);
    }
  }
  // paired layouts: stores f_I and g_I as one word; returns the Q2.29
  // contribution of the stored g_I (FP32: I = 1..8; FP16 storage: I >= 1)
  template <int I>
  __device__ __forceinline__ int32_t st_pair(T fv, T gv, uint32_t elem_row, uint32_t col) const {
    if constexpr (P == P_F32) {
      const int32_t q = __float2int_rn(gv * GQ);
      st_pair_q<I>(fv, q, elem_row, col);
      return q;
    }
    const __half hf = __float2half_rn(fv * H_SCALE(I));
    const __half hg = __float2half_rn(gv * H_SCALE(I));
    const uint32_t w = (uint32_t)__builtin_bit_cast(uint16_t, hf) |
                       ((uint32_t)__builtin_bit_cast(uint16_t, hg) << 16);
    buf_st<GR>(w, g_rsrc<I>(), col * (uint32_t)sizeof(GR), g_soff<I>(elem_row));
    return q_half(hg, I);
  }
  // FP32: stores f_I and the Q2.29 word q of g_I as one 64-bit word
  template <int I>
  __device__ __forceinline__ void st_pair_q(T fv, int32_t q, uint32_t elem_row, uint32_t col) const {
    const uint64_t w = (uint64_t)__builtin_bit_cast(uint32_t, fv) | ((uint64_t)(uint32_t)q << 32);
    buf_st<GR>(w, g_rsrc<I>(), col * (uint32_t)sizeof(GR), g_soff<I>(elem_row));
  }
  __device__ __forceinline__ void st_g0(T v, int32_t q, uint32_t elem_row, uint32_t col,
                                        uint32_t vb = 0) const {
    if constexpr (P == P_F64) buf_st<G0>(v, rg0, col * (uint32_t)sizeof(G0) + vb, elem_row * (uint32_t)sizeof(G0));
    else buf_st<G0>(q, rg0, col * (uint32_t)sizeof(G0), elem_row * (uint32_t)sizeof(G0));
  }
};

// Pulls the nine pre-collision populations of row y (uniform over the
// workgroup) at this lane's column, as raw words. Off the wall rows every
// direction reads its plane at row y - c_iy (wrapped when periodic) and
// column x - c_ix; on a wall row the directions whose source lies beyond the
// wall read the opposite plane at the node itself (half-way bounce-back).
// WALL is 0 off the walls, -1 on the bottom row and +1 on the top row; the
// choice per direction is then fixed at compile time, so every offset stays
// scalar.
template <int P, bool BIG, bool G, int WALL, int I = 0>
__device__ __forceinline__ void pull_row_dirs(const BufPop<P, BIG>& B, const uint32_t rows[3],
                                              const uint32_t col[3],
                                              typename BufT<P>::R v[9]) {
  if constexpr (I < 9) {
    constexpr int cx = CXS(I), cy = CYS(I);
    if constexpr ((WALL == -1 && cy == 1) || (WALL == 1 && cy == -1))
      v[I] = B.template ld<G, OPP(I)>(rows[1], col, 0);
    else
      v[I] = B.template ld<G, I>(rows[1 - cy], col, -cx);
    pull_row_dirs<P, BIG, G, WALL, I + 1>(B, rows, col, v);
  }
}

template <int P, bool BIG>
struct FusedCtx {
  using T = typename PrecT<P>::T;
  BufPop<P, BIG> in, out;
  Coef<T> c;
  Geom g;
  int lc, x, wi, y0, y1;
  int d;               // sweep direction: +1 upwards, -1 downwards
  uint32_t col[3];     // element columns x - 1, x, x + 1 (wrapped)
  bool act;
  T* rec;              // record planes (phi, mu, p, S, jx, jy), or null
  // this lane stores (and records) row v: an interior column of the strip
  // and a row of the segment
  __device__ __forceinline__ bool owns(int v) const {
    return act && lc >= FH && lc < wi + FH && v >= y0 && v < y1;
  }
  __device__ __forceinline__ void record(int plane, int v, T val) const {
    rec[(int64_t)plane * g.Ns + (int64_t)v * g.nx + x] = val;
  }
};

// Pull row y (physical) of population set G.
template <int P, bool BIG, bool G>
__device__ __forceinline__ void pull_row(const FusedCtx<P, BIG>& k, int y, typename BufT<P>::R v[9]) {
  const Geom& g = k.g;
  const int nx = g.nx;
  int ym = y - 1, yp = y + 1;
  if (!g.walls) {
    ym = ym < 0 ? ym + g.ny : ym;
    yp = yp >= g.ny ? yp - g.ny : yp;
  }
  const uint32_t rows[3] = {(uint32_t)(ym * nx), (uint32_t)(y * nx), (uint32_t)(yp * nx)};
  if (g.walls && y == 0)
    pull_row_dirs<P, BIG, G, -1>(k.in, rows, k.col, v);
  else if (g.walls && y == g.ny - 1)
    pull_row_dirs<P, BIG, G, 1>(k.in, rows, k.col, v);
  else
    pull_row_dirs<P, BIG, G, 0>(k.in, rows, k.col, v);
}

// FP16 storage: the f_0 word of row y (direction 0 pulls from the node
// itself, walls included).
template <int P, bool BIG>
__device__ __forceinline__ typename BufT<P>::R pull_f0(const FusedCtx<P, BIG>& k, int y) {
  return k.in.template ld<false, 0>((uint32_t)(y * k.g.nx), k.col, 0);
}

template <int P, bool BIG, int I = 1>
__device__ __forceinline__ int32_t store_pairs(const FusedCtx<P, BIG>& k, uint32_t row,
                                               const typename PrecT<P>::T f[9],
                                               const typename PrecT<P>::T gg[9]) {
  if constexpr (I < 9) {
    const int32_t q = k.out.template st_pair<I>(f[I], gg[I], row, k.col[1]);
    return q + store_pairs<P, BIG, I + 1>(k, row, f, gg);
  } else {
    return 0;
  }
}

template <int P, bool BIG, int I = 1>
__device__ __forceinline__ int32_t store_g_rest(const FusedCtx<P, BIG>& k, uint32_t row,
                                              const typename PrecT<P>::T gg[9],
                                              uint32_t vb = 0) {
  if constexpr (I < 9) {
    const int32_t q = k.out.template st_g<I>(gg[I], row, k.col[1], vb);
    return q + store_g_rest<P, BIG, I + 1>(k, row, gg, vb);
  } else {
    return 0;
  }
}

template <int P, bool BIG, int I = 0>
__device__ __forceinline__ void store_f(const FusedCtx<P, BIG>& k, uint32_t row,
                                        const typename PrecT<P>::T f[9], uint32_t vb = 0) {
  if constexpr (I < 9) {
    k.out.template st_f<I>(f[I], row, k.col[1], vb);
    store_f<P, BIG, I + 1>(k, row, f, vb);
  }
}

// Stores a node's post-collision populations; in the fixed-point modes g_0
// closes the node's Q2.29 sum at phi_q exactly.
template <int P, bool BIG>
__device__ __forceinline__ void store_row(const FusedCtx<P, BIG>& k, uint32_t row,
                                          const typename PrecT<P>::T f[9],
                                          const typename PrecT<P>::T gg[9], int32_t phi_q,
                                          uint32_t vb = 0) {
  if constexpr (P == P_F16) {
    k.out.template st_f<0>(f[0], row, k.col[1]);
    const int32_t rest = store_pairs<P, BIG>(k, row, f, gg);
    k.out.st_g0(gg[0], phi_q - rest, row, k.col[1]);
  } else if constexpr (P == P_F32) {
    const int32_t rest = store_pairs<P, BIG>(k, row, f, gg);
    k.out.template st_pair_q<0>(f[0], phi_q - rest, row, k.col[1]);
  } else {
    store_f<P, BIG>(k, row, f, vb);
    const int32_t rest = store_g_rest<P, BIG>(k, row, gg, vb);
    k.out.st_g0(gg[0], phi_q - rest, row, k.col[1], vb);
  }
}

// Decodes raw words in place (R holds the bits of the compute-type value
// afterwards); for g also returns the exact Q2.29 sum.
template <int P, int I = 0>
__device__ __forceinline__ int32_t decode_g(typename BufT<P>::R w[9]) {
  if constexpr (I < 9) {
    int32_t q = 0;
    if constexpr (FixedG<P>::value) q = BufPop<P>::template q_g<I>(w[I]);
    const typename PrecT<P>::T v = BufPop<P>::template val_g<I>(w[I]);
    w[I] = BufPop<P>::raw(v);
    return q + decode_g<P, I + 1>(w);
  } else {
    return 0;
  }
}
template <int P, int I = 0>
__device__ __forceinline__ void decode_f(typename BufT<P>::R w[9]) {
  if constexpr (I < 9) {
    w[I] = BufPop<P>::raw(BufPop<P>::template val_f<I>(w[I]));
    decode_f<P, I + 1>(w);
  }
}
template <int P>
__device__ __forceinline__ typename PrecT<P>::T as_val(typename BufT<P>::R w) {
  if constexpr (P == P_F64) return w;
  else return __builtin_bit_cast(float, w);
}

// FP16 storage: exact Q2.29 sum of a pulled row's g (raw words left intact)
template <int P, int I = 0>
__device__ __forceinline__ int32_t qsum_g(const typename BufT<P>::R w[9]) {
  if constexpr (I < 9) return BufPop<P>::template q_g<I>(w[I]) + qsum_g<P, I + 1>(w);
  else return 0;
}
// FP16 storage: f (low halves, f_0 from its own word) and g (high halves,
// g_0 Q2.29) of a pulled row
template <int P, int I = 0>
__device__ __forceinline__ void unpack_row(const typename BufT<P>::R w[9],
                                           typename BufT<P>::R f0w, typename PrecT<P>::T f[9],
                                           typename PrecT<P>::T g[9]) {
  if constexpr (I < 9) {
    f[I] = BufPop<P>::template val_f<I>((I == 0 && P == P_F16) ? f0w : w[I]);
    g[I] = BufPop<P>::template val_g<I>(w[I]);
    unpack_row<P, I + 1>(w, f0w, f, g);
  }
}

template <typename T, int NT>
struct FusedLds {
  T phi[8][NT];
  int32_t phiq[8][NT];   // exact Q2.29 phi (fixed-point modes)
  T mu[4][NT];
  T p[4][NT];
  T node[2][NM][NT];   // ux, uy, Fx, Fy, drx, dry, D
};

__device__ __forceinline__ int phys_row(int v, const Geom& g) {
  if (g.walls) return v;
  int r = v % g.ny;
  return r < 0 ? r + g.ny : r;
}

__device__ __forceinline__ bool row_ok(int v, const Geom& g) {
  return !g.walls || (v >= 0 && v < g.ny);
}

// Row r needs phi (stage A) / row q needs F, u, p (stage C) on this lane.
template <int P, bool BIG>
__device__ __forceinline__ bool need_phi(const FusedCtx<P, BIG>& k, int r) {
  return k.act && r >= k.y0 - 3 && r < k.y1 + 3 && row_ok(r, k.g);
}
template <int P, bool BIG>
__device__ __forceinline__ bool need_p(const FusedCtx<P, BIG>& k, int q) {
  return k.act && k.lc >= 2 && k.lc < k.wi + 4 && q >= k.y0 - 1 && q < k.y1 + 1 && row_ok(q, k.g);
}

template <int P, bool BIG, bool REC, int J, int NT, bool TRT = false>
__device__ __forceinline__ void fused_iter(const FusedCtx<P, BIG>& k, int r,
                                           typename BufT<P>::R (&gb)[4][9],
                                           typename BufT<P>::R (&fb)[2][9],
                                           typename BufT<P>::R (&f0b)[4],
                                           FusedLds<typename PrecT<P>::T, NT>& L) {
  using T = typename PrecT<P>::T;
  // FP32 and FP16 storage load f and g of a row together (paired words): the
  // g ring then carries f too (FP16 storage: f0b the f_0 words); the f ring
  // fb is unused
  constexpr bool PAIR = BufPop<P>::PAIRED;
  const Geom& g = k.g;
  const int lc = k.lc;
  // A: phi at row r (its g was loaded by the previous iteration)
  if (need_phi(k, r)) {
    int32_t q;
    if constexpr (PAIR) q = qsum_g<P>(gb[J]);
    else q = decode_g<P>(gb[J]);
    T ph;
    if constexpr (FixedG<P>::value) {
      ph = T(q) * T(GQI);
      L.phiq[r & 7][lc] = q;
    } else {
      T v[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) v[i] = as_val<P>(gb[J][i]);
      ph = sum9(v);
    }
    L.phi[r & 7][lc] = ph;
    if constexpr (REC)
      if (k.owns(r)) k.record(0, r, ph);
  }
  __syncthreads();
  // B: mu at row r - d
  const int b = r - k.d;
  if (k.act && lc >= 1 && lc < k.wi + 5 && b >= k.y0 - 2 && b < k.y1 + 2 && row_ok(b, g)) {
    T v[3][3], gx, gy, lap;
    lds3x3<T, NT>(L.phi, 7, b, g.ny, g.walls, lc, v);
    stencil(v, gx, gy, lap);
    const T mu = mu_bulk(v[1][1], k.c) - k.c.kappa * lap;
    L.mu[b & 3][lc] = mu;
    if constexpr (REC)
      if (k.owns(b)) k.record(1, b, mu);
  }
  __syncthreads();
  // C: force, velocity, pressure at row r - 2d
  const int q = r - 2 * k.d;
  if (need_p(k, q)) {
    T fv[9];
    if constexpr (PAIR) {
      T gv[9];
      unpack_row<P>(gb[(J + 2) & 3], f0b[(J + 2) & 3], fv, gv);
    } else {
      decode_f<P>(fb[J & 1]);
#pragma unroll
      for (int i = 0; i < 9; ++i) fv[i] = as_val<P>(fb[J & 1][i]);
    }
    T S, jx, jy;
    moments9(fv, S, jx, jy);
    T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu;
    lds3x3<T, NT>(L.phi, 7, q, g.ny, g.walls, lc, v);
    stencil(v, gphx, gphy, lapphi);
    const T ph = v[1][1];
    lds3x3<T, NT>(L.mu, 3, q, g.ny, g.walls, lc, v);
    stencil(v, gmux, gmuy, lapmu);
    Macro<T> m;
    macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, k.c, m);
    L.p[q & 3][lc] = m.p;
    if constexpr (REC) {
      if (k.owns(q)) {
        k.record(2, q, m.p);
        k.record(3, q, S);
        k.record(4, q, jx);
        k.record(5, q, jy);
      }
    }
    T* nd = &L.node[q & 1][0][0];
    nd[0 * NT + lc] = m.ux;
    nd[1 * NT + lc] = m.uy;
    nd[2 * NT + lc] = m.Fx;
    nd[3 * NT + lc] = m.Fy;
    nd[4 * NT + lc] = m.drx;
    nd[5 * NT + lc] = m.dry;
    nd[6 * NT + lc] = m.D;
  }
  __syncthreads();
  // D: collide row r - 3d and store; meanwhile fetch the next iteration's rows
  const int cr = r - 3 * k.d;
  T f[9], gg[9];
  if constexpr (PAIR) {
    unpack_row<P>(gb[(J + 1) & 3], f0b[(J + 1) & 3], f, gg);
    // the converted values are formed here, before the next rows' loads
    // below reuse the registers of these words: otherwise the compiler
    // defers the conversions into the collision and copies the words aside
    // (FP16 storage: 0.317 -> 0.312 ms per step)
#pragma unroll
    for (int i = 0; i < 9; ++i) asm volatile("" ::"v"(f[i]), "v"(gg[i]));
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f[i] = as_val<P>(fb[(J + 1) & 1][i]);
      gg[i] = as_val<P>(gb[(J + 1) & 3][i]);
    }
  }
  if (need_phi(k, r + k.d)) {
    const int y = phys_row(r + k.d, g);
    pull_row<P, BIG, true>(k, y, gb[(J + 1) & 3]);
    if constexpr (P == P_F16) f0b[(J + 1) & 3] = pull_f0(k, y);
  }
  if constexpr (!PAIR)
    if (need_p(k, r - k.d)) pull_row<P, BIG, false>(k, phys_row(r - k.d, g), fb[(J + 1) & 1]);
  if (k.owns(cr)) {
    Macro<T> m;
    const T* nd = &L.node[cr & 1][0][0];
    m.phi = L.phi[cr & 7][lc];
    m.mu = L.mu[cr & 3][lc];
    m.rho = k.c.rho_B + k.c.drho * m.phi;
    m.ux = nd[0 * NT + lc];
    m.uy = nd[1 * NT + lc];
    m.Fx = nd[2 * NT + lc];
    m.Fy = nd[3 * NT + lc];
    m.drx = nd[4 * NT + lc];
    m.dry = nd[5 * NT + lc];
    m.D = nd[6 * NT + lc];
    T v[3][3], dpx, dpy, lapp;
    lds3x3<T, NT>(L.p, 3, cr, g.ny, g.walls, lc, v);
    m.p = v[1][1];
    stencil(v, dpx, dpy, lapp);
    const int32_t phi_q = FixedG<P>::value ? L.phiq[cr & 7][lc] : 0;
    if constexpr (TRT) collide_node_trt(f, gg, m, dpx, dpy, k.c);
    else collide_node(f, gg, m, dpx, dpy, k.c);
    store_row<P, BIG>(k, (uint32_t)(cr * g.nx), f, gg, phi_q);
  }
}

// Occupancy the register allocation targets (waves per SIMD): 4 for FP16
// storage (<= 128 VGPRs), 3 for FP32 (its 64-bit f/g words fill a larger
// register ring; 4 would spill), 2 for FP64.
template <int P> struct FusedWaves { static constexpr int value = 4; };
template <> struct FusedWaves<P_F32> { static constexpr int value = 3; };
template <> struct FusedWaves<P_F64> { static constexpr int value = 2; };

// Lanes per workgroup: 4 wavefronts (strips of up to 250 columns). Measured
// on MI355X at 2048 x 8192: 8 wavefronts were 3 % and 10 % slower for FP64
// and FP16 storage, and for FP32 with 64-bit words (its best, 31.8 GLUPS,
// is 256 lanes at 3 waves per SIMD; 512 lanes, which fit only one
// workgroup per CU at that register count, gave 28.7).
template <int P> struct FusedThreads { static constexpr int value = 256; };

template <int P, bool BIG, bool REC, bool TRT = false>
__global__ __launch_bounds__(FusedThreads<P>::value, FusedWaves<P>::value) void k_step_fused(Pop<P> in, Pop<P> out,
                                                   Coef<typename PrecT<P>::T> c, Geom g, int width,
                                                   int nstrips, int seg_len,
                                                   typename PrecT<P>::T* rec) {
  using T = typename PrecT<P>::T;
  constexpr int NT = FusedThreads<P>::value;
  __shared__ FusedLds<T, NT> L;
  FusedCtx<P, BIG> k;
  k.in.init(in);
  k.out.init(out);
  k.c = c;
  k.g = g;
  k.rec = rec;
  // tiles in row-band order: the strips of one segment are consecutive, so
  // they run together on one XCD and share their halo columns in its L2
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile / nstrips, strip = tile - seg * nstrips;
  const int x0 = strip * width;
  k.wi = min(width, g.nx - x0);
  k.y0 = seg * seg_len;
  k.y1 = min(g.ny, k.y0 + seg_len);
  // even segments sweep upwards, odd ones downwards: two neighbouring
  // segments then read the rows they both need (3 warm-up rows of g and
  // 1 of f beyond each end) at the same time, at the start or at the end of
  // their sweeps, and the second read hits L2
  k.d = (seg & 1) ? -1 : 1;
  const int t = threadIdx.x;
  k.act = t < k.wi + 2 * FH;
  k.lc = k.act ? t : FH;
  k.x = wrap_x(x0 + k.lc - FH, g.nx);
  k.col[0] = (uint32_t)wrap_x(k.x - 1, g.nx);
  k.col[1] = (uint32_t)k.x;
  k.col[2] = (uint32_t)wrap_x(k.x + 1, g.nx);
  typename BufT<P>::R gb[4][9];
  typename BufT<P>::R fb[2][9];
  typename BufT<P>::R f0b[4];
  const int r0 = k.d > 0 ? k.y0 - 3 : k.y1 + 2;
  const int nit = (k.y1 - k.y0) + 6;
  // prologue: g of the first row (the first f row is needed 2 iterations later
  // and is fetched by iteration 1)
  if (need_phi(k, r0)) {
    pull_row<P, BIG, true>(k, phys_row(r0, g), gb[0]);
    if constexpr (P == P_F16) f0b[0] = pull_f0(k, phys_row(r0, g));
  }
  for (int it = 0; it < nit; it += 4) {
    fused_iter<P, BIG, REC, 0, NT, TRT>(k, r0 + k.d * (it + 0), gb, fb, f0b, L);
    fused_iter<P, BIG, REC, 1, NT, TRT>(k, r0 + k.d * (it + 1), gb, fb, f0b, L);
    fused_iter<P, BIG, REC, 2, NT, TRT>(k, r0 + k.d * (it + 2), gb, fb, f0b, L);
    fused_iter<P, BIG, REC, 3, NT, TRT>(k, r0 + k.d * (it + 3), gb, fb, f0b, L);
  }
}

// --------------------------------------------- fused kernel, two steps a pass
// The pipeline above run twice within one sweep, so that a pass over the
// populations advances the lattice by two time steps. The first step's
// stages (A1..D1) load the populations from memory as above, but its
// collision puts the post-collision words into a three-row ring in LDS
// instead of memory; the second step's stages (A2..D2) pull from that ring
// and store to memory. The state between the two steps never leaves the
// chip: per two steps the populations are read once and written once. The
// ring holds the words a single FP32 or FP64 step would have written
// (binary32 f with Q2.29 g and the exact g_0 closure, or binary64), so a
// pass computes what two single steps compute; FP16 storage keeps its
// intermediate state in the FP32 format (MidP).
//
// Halo: the second collision at the owned columns needs the first step's
// output 4 columns (and rows) beyond them (its own stencils reach 3, the
// pull 1 more), and that output needs 3 more columns of the first step's
// stencils: FH2 = 7 halo columns per side and 7 warm-up rows per segment
// end. Stage s (A1 = 0, B1 = 1, ..., D1 = 3, A2 = 4, ..., D2 = 7) runs on
// lanes [s, wi + 14 - s) and rows [y0 - 7 + s, y1 + 7 - s).
//
// Iteration with A1 at row r (direction d), a barrier after each phase:
//   A: A1 phi(r) from the loaded words; A2 phi(r - 5d) from the words pulled
//      out of the ring (rows r - 6d .. r - 4d, put there by D1 in the three
//      previous iterations)
//   B: mu of rows r - d and r - 6d
//   C: force, velocity and pressure of rows r - 2d and r - 7d
//   D: D1 collides row r - 3d into the ring slot of row r - 6d (consumed in
//      A) and loads the words of row r + d; D2 collides row r - 8d and stores
//      it.
// The fourth barrier lets every LDS ring be four rows deep (three for the
// ring of words) and D read phi and mu of its row straight from the rings.
constexpr int FH2 = 7;

template <typename T, int NT>
struct StageRings {
  T phi[4][NT];
  T mu[4][NT];
  T p[4][NT];
};

// The storage words of one row at one lane, as loaded from memory or pulled
// from the ring: FP32 the nine (f_i, g_i) pair words; FP16 storage the g_0
// word and the eight pair words, plus the f_0 half; FP64 the nine f and the
// nine g values.
template <int P> struct Row {
  typename BufT<P>::R w[9];
  typename BufT<P>::R f0;
};
template <> struct Row<P_F64> {
  double f[9];
  double g[9];
};

// Three rows of the first step's output, direction-major.
template <int P, int NT> struct MidRing;
template <int NT> struct MidRing<P_F32, NT> {
  uint64_t w[3][9][NT];    // f_i (low word) and the Q2.29 g_i (high word)
};
template <int NT> struct MidRing<P_F16, NT> {
  uint32_t w[3][9][NT];    // [0]: Q2.29 g_0; [i >= 1]: f_i low half, g_i high half
  uint16_t f0[3][NT];      // binary16 f_0
};
template <int NT> struct MidRing<P_F64, NT> {
  double f[3][9][NT];
  double g[3][9][NT];
};

// Format of the state between the two steps: the storage format, except
// for FP16 storage, whose intermediate state stays in the FP32 format
// (binary32 f, Q2.29 g with the exact g_0 closure): the binary16
// conversions of a ring in the storage format made that kernel
// arithmetic-bound, and the state is rounded to binary16 once per pass.
template <int P> struct MidP { static constexpr int value = P; };
template <> struct MidP<P_F16> { static constexpr int value = P_F32; };

template <int P, int NT>
struct Fused2Lds {
  StageRings<typename PrecT<P>::T, NT> s1, s2;
  MidRing<MidP<P>::value, NT> mid;
};

template <int P, bool BIG>
__device__ __forceinline__ bool in_stage(const FusedCtx<P, BIG>& k, int v, int s) {
  return k.act && k.lc >= s && k.lc < k.wi + 2 * FH2 - s && v >= k.y0 - FH2 + s &&
         v < k.y1 + FH2 - s && row_ok(v, k.g);
}

// Record planes (phi, mu, p, S, jx, jy) of the state a step starts from, for
// the nodes this lane owns (interior column of the strip, row of the segment).
template <int P, bool BIG>
__device__ __forceinline__ void record2(const FusedCtx<P, BIG>& k, typename PrecT<P>::T* rec,
                                        int plane, int v, typename PrecT<P>::T val) {
  if (k.lc >= FH2 && k.lc < k.wi + FH2 && v >= k.y0 && v < k.y1)
    rec[(int64_t)plane * k.g.Ns + (int64_t)v * k.g.nx + k.x] = val;
}

// Storage words of a node's post-collision populations (fixed-point modes):
// what store_row writes, g_0 closing the node's Q2.29 sum at phi_q.
template <int P>
__device__ __forceinline__ void pack_row(const typename PrecT<P>::T f[9],
                                         const typename PrecT<P>::T gg[9], int32_t phi_q,
                                         typename BufT<P>::R w[9], typename BufT<P>::R& f0w) {
  int32_t rest = 0;
  if constexpr (P == P_F32) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int32_t q = __float2int_rn(gg[i] * GQ);
      rest += q;
      w[i] = (uint64_t)__builtin_bit_cast(uint32_t, f[i]) | ((uint64_t)(uint32_t)q << 32);
    }
    w[0] = (uint64_t)__builtin_bit_cast(uint32_t, f[0]) |
           ((uint64_t)(uint32_t)(phi_q - rest) << 32);
    f0w = 0;
  } else {
    f0w = (uint32_t)__builtin_bit_cast(uint16_t, __float2half_rn(f[0] * H_SCALE(0)));
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const __half hf = __float2half_rn(f[i] * H_SCALE(i));
      const __half hg = __float2half_rn(gg[i] * H_SCALE(i));
      rest += q_half(hg, i);
      w[i] = (uint32_t)__builtin_bit_cast(uint16_t, hf) |
             ((uint32_t)__builtin_bit_cast(uint16_t, hg) << 16);
    }
    w[0] = (uint32_t)(phi_q - rest);
  }
}

// Stores packed words of one node at (row, own column) (fixed-point modes).
template <int P, bool BIG, int I = 0>
__device__ __forceinline__ void store_words(const FusedCtx<P, BIG>& k, uint32_t row,
                                            const typename BufT<P>::R w[9],
                                            typename BufT<P>::R f0w) {
  using GR = typename BufT<P>::GR;
  if constexpr (I < 9) {
    const uint32_t col = k.col[1];
    if constexpr (P == P_F16 && I == 0) {
      buf_st<__half>(__builtin_bit_cast(__half, (uint16_t)f0w), k.out.template f_rsrc<0>(),
                     col * 2u, k.out.template f_soff<0>(row));
      buf_st<int32_t>((int32_t)w[0], k.out.rg0, col * 4u, row * 4u);
    } else {
      buf_st<GR>(w[I], k.out.template g_rsrc<I>(), col * (uint32_t)sizeof(GR),
                 k.out.template g_soff<I>(row));
    }
    store_words<P, BIG, I + 1>(k, row, w, f0w);
  }
}

// Row y's words from memory (pull streaming as in pull_row).
template <int P, bool BIG>
__device__ __forceinline__ void load_row(const FusedCtx<P, BIG>& k, int y, Row<P>& row) {
  if constexpr (P == P_F64) {
    pull_row<P, BIG, false>(k, y, row.f);
    pull_row<P, BIG, true>(k, y, row.g);
  } else {
    pull_row<P, BIG, true>(k, y, row.w);
    if constexpr (P == P_F16) row.f0 = pull_f0(k, y);
  }
}

// phi of a row (and, in the fixed-point modes, its exact Q2.29 sum q), as
// the one-step kernel forms it.
template <int P>
__device__ __forceinline__ typename PrecT<P>::T row_phi(const Row<P>& row, int32_t& q) {
  using T = typename PrecT<P>::T;
  if constexpr (P == P_F64) {
    q = 0;
    return sum9(row.g);
  } else {
    q = qsum_g<P>(row.w);
    return T(q) * T(GQI);
  }
}

template <int P>
__device__ __forceinline__ void row_unpack(const Row<P>& row, typename PrecT<P>::T f[9],
                                           typename PrecT<P>::T g[9]) {
  if constexpr (P == P_F64) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f[i] = row.f[i];
      g[i] = row.g[i];
    }
  } else {
    unpack_row<P>(row.w, row.f0, f, g);
  }
}

template <int P>
__device__ __forceinline__ void row_pack(const typename PrecT<P>::T f[9],
                                         const typename PrecT<P>::T g[9], int32_t phi_q,
                                         Row<P>& row) {
  if constexpr (P == P_F64) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      row.f[i] = f[i];
      row.g[i] = g[i];
    }
  } else {
    pack_row<P>(f, g, phi_q, row.w, row.f0);
  }
}

// Stores a node's post-collision populations to memory.
template <int P, bool BIG>
__device__ __forceinline__ void store_node2(const FusedCtx<P, BIG>& k, uint32_t rowoff,
                                            const typename PrecT<P>::T f[9],
                                            const typename PrecT<P>::T g[9], int32_t phi_q,
                                            uint32_t vb = 0) {
  if constexpr (P == P_F64) {
    store_row<P, BIG>(k, rowoff, f, g, 0, vb);
  } else {
    Row<P> o;
    pack_row<P>(f, g, phi_q, o.w, o.f0);
    store_words<P, BIG>(k, rowoff, o.w, o.f0);
  }
}

template <int P, int NT>
__device__ __forceinline__ void ring_put(MidRing<P, NT>& M, int s, int lc, const Row<P>& row) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    if constexpr (P == P_F64) {
      M.f[s][i][lc] = row.f[i];
      M.g[s][i][lc] = row.g[i];
    } else {
      M.w[s][i][lc] = row.w[i];
    }
  }
  if constexpr (P == P_F16) M.f0[s][lc] = (uint16_t)row.f0;
}

// Pulls row v's words out of the ring: sl[1 + dy] is the slot of row v + dy.
// The nine reads go straight (one lane address per ring row, direction and
// column as immediate offsets); on a wall row the directions that would come
// from beyond the wall are then read again as the row's own opposite
// populations (bounce-back, WALL as in pull_row_dirs), in a branch of their
// own, so that the wall cases do not turn every address into a select.
template <int P, int NT, int I = 0>
__device__ __forceinline__ void pull_mid_dirs(const MidRing<P, NT>& M, const int sl[3], int lc,
                                              Row<P>& row) {
  if constexpr (I < 9) {
    constexpr int cx = CXS(I), cy = CYS(I);
    const int s = sl[1 - cy];
    if constexpr (P == P_F64) {
      row.f[I] = (&M.f[s][I][lc - 1])[1 - cx];
      row.g[I] = (&M.g[s][I][lc - 1])[1 - cx];
    } else {
      row.w[I] = (&M.w[s][I][lc - 1])[1 - cx];
    }
    pull_mid_dirs<P, NT, I + 1>(M, sl, lc, row);
  }
}

template <int P, int NT, int WALL, int I = 0>
__device__ __forceinline__ void bounce_mid_dirs(const MidRing<P, NT>& M, int s1, int lc,
                                                Row<P>& row) {
  if constexpr (I < 9) {
    constexpr int cy = CYS(I);
    if constexpr ((WALL == -1 && cy == 1) || (WALL == 1 && cy == -1)) {
      if constexpr (P == P_F64) {
        row.f[I] = M.f[s1][OPP(I)][lc];
        row.g[I] = M.g[s1][OPP(I)][lc];
      } else {
        row.w[I] = M.w[s1][OPP(I)][lc];
      }
    }
    bounce_mid_dirs<P, NT, WALL, I + 1>(M, s1, lc, row);
  }
}

// FP64: one whole pull per wall case instead (measured 1.6 % faster there;
// the straight reads are faster for the 64-bit pair words).
template <int P, int NT, int WALL, int I = 0>
__device__ __forceinline__ void pull_mid_wall_dirs(const MidRing<P, NT>& M, const int sl[3],
                                                   int lc, Row<P>& row) {
  if constexpr (I < 9) {
    constexpr int cx = CXS(I), cy = CYS(I);
    constexpr bool bounce = (WALL == -1 && cy == 1) || (WALL == 1 && cy == -1);
    constexpr int src = bounce ? OPP(I) : I;
    const int s = bounce ? sl[1] : sl[1 - cy];
    const int l = bounce ? lc : lc - cx;
    row.f[I] = M.f[s][src][l];
    row.g[I] = M.g[s][src][l];
    pull_mid_wall_dirs<P, NT, WALL, I + 1>(M, sl, lc, row);
  }
}

template <int P, int NT>
__device__ __forceinline__ void pull_mid(const MidRing<P, NT>& M, const int sl[3], int v,
                                         const Geom& g, int lc, Row<P>& row) {
  if constexpr (P == P_F64) {
    if (g.walls && v == 0)
      pull_mid_wall_dirs<P, NT, -1>(M, sl, lc, row);
    else if (g.walls && v == g.ny - 1)
      pull_mid_wall_dirs<P, NT, 1>(M, sl, lc, row);
    else
      pull_mid_wall_dirs<P, NT, 0>(M, sl, lc, row);
  } else {
    pull_mid_dirs<P, NT>(M, sl, lc, row);
    if (g.walls && v == 0)
      bounce_mid_dirs<P, NT, -1>(M, sl[1], lc, row);
    else if (g.walls && v == g.ny - 1)
      bounce_mid_dirs<P, NT, 1>(M, sl[1], lc, row);
    if constexpr (P == P_F16) row.f0 = M.f0[sl[1]][lc];
  }
}

// Stage B of one pipeline: mu at row b.
template <typename T, int NT>
__device__ __forceinline__ T stage_mu(StageRings<T, NT>& S, int b, const Geom& g, int lc,
                                      const Coef<T>& c) {
  T v[3][3], gx, gy, lap;
  lds3x3<T, NT>(S.phi, 3, b, g.ny, g.walls, lc, v);
  stencil(v, gx, gy, lap);
  const T mu = mu_bulk(v[1][1], c) - c.kappa * lap;
  S.mu[b & 3][lc] = mu;
  return mu;
}

// Stage C of one pipeline: force, velocity and pressure at row q from its
// pulled populations; p into the ring, the rest into nd.
template <int P, int NT>
__device__ __forceinline__ void stage_macro(StageRings<typename PrecT<P>::T, NT>& S,
                                            const Row<P>& row, int q, const Geom& g, int lc,
                                            const Coef<typename PrecT<P>::T>& c,
                                            typename PrecT<P>::T nd[NM],
                                            typename PrecT<P>::T rv[4]) {
  using T = typename PrecT<P>::T;
  T fv[9], gv[9];
  row_unpack<P>(row, fv, gv);
  T Sm, jx, jy;
  moments9(fv, Sm, jx, jy);
  T v[3][3], gphx, gphy, lapphi, gmux, gmuy, lapmu;
  lds3x3<T, NT>(S.phi, 3, q, g.ny, g.walls, lc, v);
  stencil(v, gphx, gphy, lapphi);
  const T ph = v[1][1];
  lds3x3<T, NT>(S.mu, 3, q, g.ny, g.walls, lc, v);
  stencil(v, gmux, gmuy, lapmu);
  Macro<T> m;
  macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, Sm, jx, jy, c, m);
  S.p[q & 3][lc] = m.p;
  rv[0] = m.p;
  rv[1] = Sm;
  rv[2] = jx;
  rv[3] = jy;
  nd[0] = m.ux;
  nd[1] = m.uy;
  nd[2] = m.Fx;
  nd[3] = m.Fy;
  nd[4] = m.drx;
  nd[5] = m.dry;
  nd[6] = m.D;
}

// Stage D of one pipeline: collision of row cr (f, gg hold its pulled
// populations on entry, the post-collision ones on exit).
template <typename T, int NT, bool TRT = false>
__device__ __forceinline__ void stage_collide(const StageRings<T, NT>& S, int cr, const Geom& g,
                                              int lc, const Coef<T>& c, const T nd[NM], T f[9],
                                              T gg[9]) {
  Macro<T> m;
  m.phi = S.phi[cr & 3][lc];
  m.mu = S.mu[cr & 3][lc];
  m.rho = c.rho_B + c.drho * m.phi;
  m.ux = nd[0];
  m.uy = nd[1];
  m.Fx = nd[2];
  m.Fy = nd[3];
  m.drx = nd[4];
  m.dry = nd[5];
  m.D = nd[6];
  T v[3][3], dpx, dpy, lapp;
  lds3x3<T, NT>(S.p, 3, cr, g.ny, g.walls, lc, v);
  m.p = v[1][1];
  stencil(v, dpx, dpy, lapp);
  if constexpr (TRT) collide_node_trt(f, gg, m, dpx, dpy, c);
  else collide_node(f, gg, m, dpx, dpy, c);
}

template <int P, bool BIG, bool REC, int J, int NT, bool TRT = false>
__device__ __forceinline__ void fused2_iter(const FusedCtx<P, BIG>& k, int r, int s,
                                            Row<P> (&rb1)[4], Row<MidP<P>::value> (&rb2)[4],
                                            typename PrecT<P>::T (&nd1)[2][NM],
                                            typename PrecT<P>::T (&nd2)[2][NM],
                                            Fused2Lds<P, NT>& L, typename PrecT<P>::T* rec0,
                                            typename PrecT<P>::T* rec1) {
  using T = typename PrecT<P>::T;
  constexpr int P2 = MidP<P>::value;   // format of the ring and of rb2
  const Geom& g = k.g;
  const int lc = k.lc, d = k.d;
  const int r2 = r - 5 * d;
  int32_t q;
  T rv[4];
  // A
  if (in_stage(k, r, 0)) {
    const T ph = row_phi<P>(rb1[J], q);
    L.s1.phi[r & 3][lc] = ph;
    if constexpr (REC) record2(k, rec0, 0, r, ph);
  }
  if (in_stage(k, r2, 4)) {
    // slots of rows r2 - 1, r2, r2 + 1: the row D1 wrote i iterations ago
    // sits in slot (s - i) mod 3, and rows r2 - d, r2, r2 + d were written
    // 3, 2 and 1 iterations ago
    const int s1 = s == 0 ? 2 : s - 1, s2 = s == 2 ? 0 : s + 1;
    const int sl[3] = {d > 0 ? s : s1, s2, d > 0 ? s1 : s};
    pull_mid<P2, NT>(L.mid, sl, r2, g, lc, rb2[J]);
    const T ph = row_phi<P2>(rb2[J], q);
    L.s2.phi[r2 & 3][lc] = ph;
    if constexpr (REC) record2(k, rec1, 0, r2, ph);
  }
  __syncthreads();
  // B
  if (in_stage(k, r - d, 1)) {
    const T mu = stage_mu<T, NT>(L.s1, r - d, g, lc, k.c);
    if constexpr (REC) record2(k, rec0, 1, r - d, mu);
  }
  if (in_stage(k, r2 - d, 5)) {
    const T mu = stage_mu<T, NT>(L.s2, r2 - d, g, lc, k.c);
    if constexpr (REC) record2(k, rec1, 1, r2 - d, mu);
  }
  __syncthreads();
  // C
  if (in_stage(k, r - 2 * d, 2)) {
    stage_macro<P, NT>(L.s1, rb1[(J + 2) & 3], r - 2 * d, g, lc, k.c, nd1[J & 1], rv);
    if constexpr (REC) {
#pragma unroll
      for (int i = 0; i < 4; ++i) record2(k, rec0, 2 + i, r - 2 * d, rv[i]);
    }
  }
  if (in_stage(k, r2 - 2 * d, 6)) {
    stage_macro<P2, NT>(L.s2, rb2[(J + 2) & 3], r2 - 2 * d, g, lc, k.c, nd2[J & 1], rv);
    if constexpr (REC) {
#pragma unroll
      for (int i = 0; i < 4; ++i) record2(k, rec1, 2 + i, r2 - 2 * d, rv[i]);
    }
  }
  __syncthreads();
  // D1: row r - 3d into the ring; the words of row r + d into the freed slot
  {
    const int cr = r - 3 * d;
    T f[9], gg[9];
    int32_t phi_q;
    row_phi<P>(rb1[(J + 1) & 3], phi_q);
    row_unpack<P>(rb1[(J + 1) & 3], f, gg);
    // FP32 and FP16 storage issue the loads of row r + d before this
    // collision, to hide their latency behind it; FP64 after it, once the
    // row's words are dead: loading into registers still in use made the
    // compiler copy the whole 18-word row each iteration (0.85 -> 0.79 ms
    // per step), more than the latency costs there.
    if constexpr (P != P_F64)
      if (in_stage(k, r + d, 0)) load_row<P, BIG>(k, phys_row(r + d, g), rb1[(J + 1) & 3]);
    if (in_stage(k, cr, 3)) {
      stage_collide<T, NT, TRT>(L.s1, cr, g, lc, k.c, nd1[(J + 1) & 1], f, gg);
      Row<P2> o;
      row_pack<P2>(f, gg, phi_q, o);
      ring_put<P2, NT>(L.mid, s, lc, o);
    }
    if constexpr (P == P_F64)
      if (in_stage(k, r + d, 0)) load_row<P, BIG>(k, phys_row(r + d, g), rb1[(J + 1) & 3]);
  }
  // D2: row r - 8d to memory
  {
    const int cr = r2 - 3 * d;
    if constexpr (P == P_F64 && !BIG) {
      // Every lane issues the 18 stores; lanes and rows outside the stage
      // offset theirs 2 GiB beyond the descriptors (each spans at most
      // 2 GiB here, fused_big), where the hardware drops them. With the
      // stores under a branch the compiler's count of memory operations in
      // flight is merged from the path without them, and the next
      // iteration's wait for the loads of row r + d would also wait for
      // these stores (one wave per SIMD: nothing else covers it).
      const bool ok = in_stage(k, cr, 7);
      T f[9], gg[9];
      int32_t phi_q = 0;
      if (ok) {
        row_phi<P2>(rb2[(J + 1) & 3], phi_q);
        row_unpack<P2>(rb2[(J + 1) & 3], f, gg);
        stage_collide<T, NT, TRT>(L.s2, cr, g, lc, k.c, nd2[(J + 1) & 1], f, gg);
      }
      const int crs = cr >= 0 && cr < g.ny ? cr : 0;
      store_node2<P, BIG>(k, (uint32_t)(crs * g.nx), f, gg, phi_q, ok ? 0u : 0x80000000u);
    } else if (in_stage(k, cr, 7)) {
      T f[9], gg[9];
      int32_t phi_q;
      row_phi<P2>(rb2[(J + 1) & 3], phi_q);
      row_unpack<P2>(rb2[(J + 1) & 3], f, gg);
      stage_collide<T, NT, TRT>(L.s2, cr, g, lc, k.c, nd2[(J + 1) & 1], f, gg);
      store_node2<P, BIG>(k, (uint32_t)(cr * g.nx), f, gg, phi_q);
    }
  }
  __syncthreads();
}

// Resident workgroups per CU (waves per SIMD with 4-wave workgroups): two
// for FP32 and FP16 storage (LDS 78 KB / 53 KB, 245 / 216 VGPRs), one for
// FP64 (LDS 156 KB: the ring of 18 binary64 words per node is 108 KB).
template <int P> struct Fused2Waves { static constexpr int value = 2; };
template <> struct Fused2Waves<P_F64> { static constexpr int value = 1; };

// REC: also writes the records of the two states the pass starts from
// (rec0: the state read, rec1: the state after the first step).
template <int P, bool BIG, bool REC, bool TRT = false>
__global__ __launch_bounds__(256, Fused2Waves<P>::value) void k_step2_fused(
    Pop<P> in, Pop<P> out, Coef<typename PrecT<P>::T> c, Geom g, int width, int nstrips,
    int seg_len, typename PrecT<P>::T* rec0, typename PrecT<P>::T* rec1) {
  using T = typename PrecT<P>::T;
  constexpr int NT = 256;
  __shared__ Fused2Lds<P, NT> L;
  FusedCtx<P, BIG> k;
  k.in.init(in);
  k.out.init(out);
  k.c = c;
  k.g = g;
  k.rec = nullptr;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int seg = tile / nstrips, strip = tile - seg * nstrips;
  const int x0 = strip * width;
  k.wi = min(width, g.nx - x0);
  k.y0 = seg * seg_len;
  k.y1 = min(g.ny, k.y0 + seg_len);
  k.d = (seg & 1) ? -1 : 1;
  const int t = threadIdx.x;
  k.act = t < k.wi + 2 * FH2;
  k.lc = k.act ? t : FH2;
  // the halo reaches 7 columns beyond the strip: wrap with a full modulo
  // (lattices may be narrower than the halo)
  int xv = (x0 - FH2 + k.lc) % g.nx;
  k.x = xv < 0 ? xv + g.nx : xv;
  k.col[0] = (uint32_t)wrap_x(k.x - 1, g.nx);
  k.col[1] = (uint32_t)k.x;
  k.col[2] = (uint32_t)wrap_x(k.x + 1, g.nx);
  Row<P> rb1[4];
  Row<MidP<P>::value> rb2[4];
  T nd1[2][NM], nd2[2][NM];
  const int r0 = k.d > 0 ? k.y0 - FH2 : k.y1 + FH2 - 1;
  const int nit = (k.y1 - k.y0) + 2 * FH2 + 1;
  if (in_stage(k, r0, 0)) load_row<P, BIG>(k, phys_row(r0, g), rb1[0]);
  int s = 0;   // ring slot D1 writes in this iteration: iteration index mod 3
  for (int it = 0; it < nit; it += 4) {
    fused2_iter<P, BIG, REC, 0, NT, TRT>(k, r0 + k.d * (it + 0), s, rb1, rb2, nd1, nd2, L, rec0,
                                 rec1);
    s = s == 2 ? 0 : s + 1;
    fused2_iter<P, BIG, REC, 1, NT, TRT>(k, r0 + k.d * (it + 1), s, rb1, rb2, nd1, nd2, L, rec0,
                                 rec1);
    s = s == 2 ? 0 : s + 1;
    fused2_iter<P, BIG, REC, 2, NT, TRT>(k, r0 + k.d * (it + 2), s, rb1, rb2, nd1, nd2, L, rec0,
                                 rec1);
    s = s == 2 ? 0 : s + 1;
    fused2_iter<P, BIG, REC, 3, NT, TRT>(k, r0 + k.d * (it + 3), s, rb1, rb2, nd1, nd2, L, rec0,
                                 rec1);
    s = s == 2 ? 0 : s + 1;
  }
}

// --------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

__global__ __launch_bounds__(256) void k_zero_words(uint4* __restrict__ p, int64_t n16) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += (int64_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return hipSuccess;
  const unsigned grid = nblk(n16, 256) < 8192u ? nblk(n16, 256) : 8192u;
  hipLaunchKernelGGL(k_zero_words, dim3(grid), dim3(256), 0, s, (uint4*)p, n16);
  return hipGetLastError();
}

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
hipError_t launch_macro(const void* pop, const void* phi, const void* mu, void* p, void* sj,
                        const MomentOut& mo, const Coef<typename PrecT<P>::T>& c, const Geom& g,
                        hipStream_t s) {
  using T = typename PrecT<P>::T;
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_macro<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, (const T*)phi,
                     (const T*)mu, (T*)p, (T*)sj, mo, c, g);
  return hipGetLastError();
}

template <int P>
hipError_t launch_step_unfused(const void* pin, void* pout, void* phi, void* mu, void* p,
                               void* sj, const Coef<typename PrecT<P>::T>& c, const Geom& g,
                               hipStream_t s, bool trt) {
  using T = typename PrecT<P>::T;
  hipError_t e = launch_fields<P>(pin, phi, mu, c, g, s);
  if (e != hipSuccess) return e;
  e = launch_macro<P>(pin, phi, mu, p, sj, MomentOut{}, c, g, s);
  if (e != hipSuccess) return e;
  Pop<P> i{(char*)pin, g.Ns}, o{(char*)pout, g.Ns};
  if (trt)
    hipLaunchKernelGGL((k_collide<P, true>), dim3(nblk(g.N, 256)), dim3(256), 0, s, i, o,
                       (const T*)phi, (const T*)mu, (const T*)p, c, g);
  else
    hipLaunchKernelGGL(k_collide<P>, dim3(nblk(g.N, 256)), dim3(256), 0, s, i, o, (const T*)phi,
                       (const T*)mu, (const T*)p, c, g);
  return hipGetLastError();
}

template <int P>
FusedShape fused_shape(const Geom& g, int seg_rows, int resident) {
  constexpr int NT = FusedThreads<P>::value, FWMAX = NT - 2 * FH;
  FusedShape sh;
  // strips of equal width (at most FWMAX interior columns) so that every
  // workgroup carries the same work
  sh.nstrips = (g.nx + FWMAX - 1) / FWMAX;
  sh.width = (g.nx + sh.nstrips - 1) / sh.nstrips;
  if (seg_rows <= 0) {
    // about 2.25 workgroups per resident slot (CUs x workgroups per CU),
    // segments of 16..32 rows: measured best on MI355X for all three
    // precisions at 2048 x 8192 (longer segments leave the last wave of
    // workgroups too unbalanced, shorter ones recompute more warm-up rows)
    if (resident < 1) resident = 1024;
    const int total = (resident * 9 + 3) / 4;
    const int want = (total + sh.nstrips - 1) / sh.nstrips;
    seg_rows = (g.ny + want - 1) / want;
    if (seg_rows < 16) seg_rows = 16;
    if (seg_rows > 32) seg_rows = 32;
  }
  if (seg_rows > g.ny) seg_rows = g.ny;
  sh.seg_rows = seg_rows;
  sh.nseg = (g.ny + seg_rows - 1) / seg_rows;
  sh.threads = NT;
  return sh;
}

// FP64: also where a group spans more than 2 GiB, so that the two-step
// kernel's stores beyond the range of a group descriptor (2 GiB past the
// lane's offset) are dropped (the g_0 plane's descriptor is smaller still).
template <int P>
bool fused_big(const Geom& g) {
  const int64_t f_group = (P == P_F16 ? 1 : 9) * g.Ns * (int64_t)sizeof(typename BufT<P>::F);
  const int64_t g_group = (P == P_F32 ? 9 : 8) * g.Ns * (int64_t)sizeof(typename BufT<P>::GR);
  const int64_t lim = P == P_F64 ? ((int64_t)1 << 31) : (int64_t)UINT32_MAX;
  return f_group > lim || g_group > lim;
}

template <int P>
int fused_resident() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_fused<P, false, false>,
                                                   FusedThreads<P>::value, 0) != hipSuccess)
    return 0;
  return cus * (per_cu > 0 ? per_cu : 1);
}

template <int P, bool BIG, bool REC, bool TRT = false>
static void launch_fused_variant(const Pop<P>& i, const Pop<P>& o,
                                 const Coef<typename PrecT<P>::T>& c, const Geom& g,
                                 const FusedShape& sh, void* rec, hipStream_t s) {
  using T = typename PrecT<P>::T;
  hipLaunchKernelGGL((k_step_fused<P, BIG, REC, TRT>), dim3(sh.nstrips * sh.nseg),
                     dim3(sh.threads), 0, s, i, o, c, g, sh.width, sh.nstrips, sh.seg_rows,
                     (T*)rec);
}

template <int P>
hipError_t launch_step_fused(const void* pin, void* pout, const Coef<typename PrecT<P>::T>& c,
                             const Geom& g, const FusedShape& sh, void* rec, hipStream_t s,
                             bool trt) {
  Pop<P> i{(char*)pin, g.Ns}, o{(char*)pout, g.Ns};
  const bool big = fused_big<P>(g);
  if (trt) {
    if (rec) return hipErrorInvalidValue;       // no recording TRT variant
    if (big) launch_fused_variant<P, true, false, true>(i, o, c, g, sh, rec, s);
    else launch_fused_variant<P, false, false, true>(i, o, c, g, sh, rec, s);
  } else if (rec) {
    if (big) launch_fused_variant<P, true, true>(i, o, c, g, sh, rec, s);
    else launch_fused_variant<P, false, true>(i, o, c, g, sh, rec, s);
  } else {
    if (big) launch_fused_variant<P, true, false>(i, o, c, g, sh, rec, s);
    else launch_fused_variant<P, false, false>(i, o, c, g, sh, rec, s);
  }
  return hipGetLastError();
}

template <int P>
FusedShape fused2_shape(const Geom& g, int seg_rows, int resident) {
  constexpr int NT = 256, FWMAX = NT - 2 * FH2;
  FusedShape sh;
  sh.nstrips = (g.nx + FWMAX - 1) / FWMAX;
  sh.width = (g.nx + sh.nstrips - 1) / sh.nstrips;
  if (seg_rows <= 0) {
    // one round of workgroups: as many segments as resident slots allow,
    // since every segment end costs 7 warm-up rows of both steps
    if (resident < 1) resident = 512;
    int nseg = resident / sh.nstrips;
    if (nseg < 1) nseg = 1;
    seg_rows = (g.ny + nseg - 1) / nseg;
    if (seg_rows < 16) seg_rows = 16;
  }
  if (seg_rows > g.ny) seg_rows = g.ny;
  sh.seg_rows = seg_rows;
  sh.nseg = (g.ny + seg_rows - 1) / seg_rows;
  sh.threads = NT;
  return sh;
}

template <int P>
int fused2_resident() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step2_fused<P, false, false>, 256, 0) !=
      hipSuccess)
    return 0;
  return cus * (per_cu > 0 ? per_cu : 1);
}

template <int P, bool BIG, bool REC, bool TRT = false>
static void launch_fused2_variant(const Pop<P>& i, const Pop<P>& o,
                                  const Coef<typename PrecT<P>::T>& c, const Geom& g,
                                  const FusedShape& sh, void* rec0, void* rec1, hipStream_t s) {
  using T = typename PrecT<P>::T;
  hipLaunchKernelGGL((k_step2_fused<P, BIG, REC, TRT>), dim3(sh.nstrips * sh.nseg),
                     dim3(sh.threads), 0, s, i, o, c, g, sh.width, sh.nstrips, sh.seg_rows,
                     (T*)rec0, (T*)rec1);
}

template <int P>
hipError_t launch_step2_fused(const void* pin, void* pout, const Coef<typename PrecT<P>::T>& c,
                              const Geom& g, const FusedShape& sh, void* rec0, void* rec1,
                              hipStream_t s, bool trt) {
  Pop<P> i{(char*)pin, g.Ns}, o{(char*)pout, g.Ns};
  const bool big = fused_big<P>(g);
  if (trt) {
    if (rec0 || rec1) return hipErrorInvalidValue;   // no recording TRT variant
    if (big) launch_fused2_variant<P, true, false, true>(i, o, c, g, sh, nullptr, nullptr, s);
    else launch_fused2_variant<P, false, false, true>(i, o, c, g, sh, nullptr, nullptr, s);
  } else if (rec0 && rec1) {
    if (big) launch_fused2_variant<P, true, true>(i, o, c, g, sh, rec0, rec1, s);
    else launch_fused2_variant<P, false, true>(i, o, c, g, sh, rec0, rec1, s);
  } else {
    if (big) launch_fused2_variant<P, true, false>(i, o, c, g, sh, nullptr, nullptr, s);
    else launch_fused2_variant<P, false, false>(i, o, c, g, sh, nullptr, nullptr, s);
  }
  return hipGetLastError();
}

template <int P>
hipError_t launch_mass(const void* pop, void* phi, void* mu, double* part, int nred, double* out,
                       const Coef<typename PrecT<P>::T>& c, const Coef<double>& c64,
                       const Geom& g, hipStream_t s) {
  using T = typename PrecT<P>::T;
  hipError_t e = launch_fields<P>(pop, phi, mu, c, g, s);
  if (e != hipSuccess) return e;
  Pop<P> i{(char*)pop, g.Ns};
  hipLaunchKernelGGL(k_mass_partial<P>, dim3(nred), dim3(256), 0, s, i, (const T*)phi,
                     (const T*)mu, part, c, c64.rho_B, c64.drho, g);
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
  template hipError_t launch_macro<P>(const void*, const void*, const void*, void*, void*,     \
                                      const MomentOut&, const Coef<PrecT<P>::T>&, const Geom&,   \
                                      hipStream_t);                                              \
  template hipError_t launch_step_unfused<P>(const void*, void*, void*, void*, void*, void*,     \
                                             const Coef<PrecT<P>::T>&, const Geom&, hipStream_t,  \
                                             bool);                                               \
  template hipError_t launch_step_fused<P>(const void*, void*, const Coef<PrecT<P>::T>&,         \
                                           const Geom&, const FusedShape&, void*, hipStream_t,   \
                                           bool);                                                \
  template int fused_resident<P>();                                                              \
  template FusedShape fused_shape<P>(const Geom&, int, int);                                     \
  template bool fused_big<P>(const Geom&);                                                       \
  template FusedShape fused2_shape<P>(const Geom&, int, int);                                    \
  template int fused2_resident<P>();                                                             \
  template hipError_t launch_step2_fused<P>(const void*, void*, const Coef<PrecT<P>::T>&,        \
                                            const Geom&, const FusedShape&, void*, void*,        \
                                            hipStream_t, bool);                                  \
  template hipError_t launch_mass<P>(const void*, void*, void*, double*, int, double*,           \
                                     const Coef<PrecT<P>::T>&, const Coef<double>&, const Geom&,  \
                                     hipStream_t);

QILBM_INSTANTIATE(P_F64)
QILBM_INSTANTIATE(P_F32)
QILBM_INSTANTIATE(P_F16)

}  // namespace qilbm
