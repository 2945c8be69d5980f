// Three-dimensional (D3Q19) form of the quasi-incompressible phase-field LBE
// step (Yang & Guo, Sec. III, every term with three velocity components) for
// gfx950, and its C ABI (include/qilbm3d.h).
//
// The step runs as four node-per-thread kernels, like the unfused
// two-dimensional path: phi (the pulled g), mu (bulk part minus kappa times
// the 19-point Laplacian of phi), the pressure (moments of the pulled f,
// the stencils of phi and mu, force, velocity) with the collision of f,
// which needs no grad p, and the collision of g (grad p from the pressure
// field); or, in FP32, as one fused z-sweep kernel. Populations live in a pull
// layout: slot (i, x) holds the post-collision population i produced at x,
// so the pre-collision value at x is slot (i, x - c_i), or slot (opp(i), x)
// when x - c_i lies beyond a wall.
#include <math.h>
#include <new>
#include <type_traits>

#include "../../include/qilbm3d.h"
#include "qilbm_internal.hpp"

namespace qilbm3 {

using qilbm::Coef;
using qilbm::FixedG;
using qilbm::GQ;
using qilbm::GQI;
using qilbm::GQI_D;
using qilbm::P_F32;
using qilbm::P_F64;
using qilbm::PrecT;
using qilbm::mu_bulk;
using qilbm::recip;
using qilbm::fmad;
using qilbm::BUF_WORD3;
using qilbm::buf_ld;
using qilbm::buf_st;
using qilbm::xcd_tile;

// ------------------------------------------------------------------ lattice
// D3Q19 in the canonical order of the header: rest; the six axis vectors;
// the twelve vectors with two components +-1 (pairs of opposites).
__host__ __device__ constexpr int CX(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int CY(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int CZ(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr double W(int i) {
  return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// opposite directions are adjacent: (1,2), (3,4), ..., (17,18)
__host__ __device__ constexpr int OPP(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
static_assert(CX(OPP(13)) == -CX(13) && CY(OPP(17)) == -CY(17) && CZ(OPP(18)) == -CZ(18), "opp");
static_assert(CX(10) == -1 && CY(10) == 1 && CZ(14) == 1 && CX(14) == -1, "table");

struct Geom3 {
  int nx, ny, nz;
  int walls;     // 1: bounce-back walls below z = 0 and above z = nz - 1
  int64_t N;     // nx * ny * nz
  int64_t Ns;    // plane stride (elements)
};

template <typename T>
struct Coef3 {
  Coef<T> c;     // the two-dimensional coefficient set (gy holds gy, gx gx)
  T gz;
};

// Populations: FP64 38 binary64 planes (f_0..18, g_0..18); FP32 19 binary32
// planes of f, then 19 int32 planes of g in Q2.29.
template <int P>
struct Pop3 {
  char* base;
  int64_t Ns;
  using T = typename PrecT<P>::T;
  __device__ __forceinline__ T f(int i, uint32_t n) const {
    return reinterpret_cast<const T*>(base)[(int64_t)i * Ns + n];
  }
  __device__ __forceinline__ void set_f(int i, uint32_t n, T v) const {
    reinterpret_cast<T*>(base)[(int64_t)i * Ns + n] = v;
  }
  __device__ __forceinline__ int32_t gq(int i, uint32_t n) const {
    return reinterpret_cast<const int32_t*>(base + 19 * Ns * (int64_t)sizeof(T))[(int64_t)i * Ns + n];
  }
  __device__ __forceinline__ T g(int i, uint32_t n) const {
    if constexpr (P == P_F64)
      return reinterpret_cast<const double*>(base)[(int64_t)(19 + i) * Ns + n];
    else
      return float(gq(i, n)) * GQI;
  }
  __device__ __forceinline__ double g_exact(int i, uint32_t n) const {
    if constexpr (P == P_F64) return g(i, n);
    else return double(gq(i, n)) * GQI_D;
  }
  // stores g_i; returns its Q2.29 word in FP32 (0 in FP64)
  __device__ __forceinline__ int32_t set_g(int i, uint32_t n, T v) const {
    if constexpr (P == P_F64) {
      reinterpret_cast<double*>(base)[(int64_t)(19 + i) * Ns + n] = v;
      return 0;
    } else {
      const int32_t q = __float2int_rn(v * GQ);
      set_gq(i, n, q);
      return q;
    }
  }
  // stores g_i given in FP64: rounded once, to binary64 or to Q2.29
  __device__ __forceinline__ void set_g_d(int i, uint32_t n, double v) const {
    if constexpr (P == P_F64)
      reinterpret_cast<double*>(base)[(int64_t)(19 + i) * Ns + n] = v;
    else
      set_gq(i, n, __double2int_rn(v * 536870912.0));
  }
  __device__ __forceinline__ void set_gq(int i, uint32_t n, int32_t q) const {
    reinterpret_cast<int32_t*>(base + 19 * Ns * (int64_t)sizeof(T))[(int64_t)i * Ns + n] = q;
  }
};

inline int64_t pop3_bytes(int P, int64_t Ns) { return 38 * Ns * (P == P_F64 ? 8 : 4); }

// ------------------------------------------------------------- addressing
struct Node {
  int x, y, z;
  uint32_t n;
};

// Per-node addressing of the cold kernels (initial state, state transfer):
// N < 2^29, so the decomposition runs in 32-bit integer division.
__device__ __forceinline__ Node node_of(int64_t n, const Geom3& g) {
  Node k;
  k.n = (uint32_t)n;
  const uint32_t plane = (uint32_t)g.nx * (uint32_t)g.ny;
  const uint32_t z = k.n / plane, r = k.n - z * plane;
  const uint32_t y = r / (uint32_t)g.nx;
  k.z = (int)z;
  k.y = (int)y;
  k.x = (int)(r - y * (uint32_t)g.nx);
  return k;
}

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ uint32_t idx3(int x, int y, int z, const Geom3& g) {
  return (uint32_t)(((int64_t)z * g.ny + y) * g.nx + x);
}

// Pre-collision source of population i at node k: plane index and element.
template <int I>
__device__ __forceinline__ void pull_src(const Node& k, const Geom3& g, int& plane, uint32_t& e) {
  const int zs = k.z - CZ(I);
  if ((zs < 0 || zs >= g.nz) && g.walls) {
    plane = OPP(I);
    e = k.n;
    return;
  }
  plane = I;
  e = idx3(wrapi(k.x - CX(I), g.nx), wrapi(k.y - CY(I), g.ny), wrapi(zs, g.nz), g);
}

// Element of the stencil neighbour k + c: periodic, or the mirrored ghost
// plane (the boundary plane itself) beyond a wall.
__device__ __forceinline__ uint32_t nbr(const Node& k, int cx, int cy, int cz, const Geom3& g) {
  int z = k.z + cz;
  if (z < 0 || z >= g.nz) z = g.walls ? k.z : wrapi(z, g.nz);
  return idx3(wrapi(k.x + cx, g.nx), wrapi(k.y + cy, g.ny), z, g);
}

// Isotropic central gradient and Laplacian of a field at node k.
template <typename T, typename F, int I = 1>
__device__ __forceinline__ void stencil_acc(const F* psi, const Node& k, const Geom3& g, T c0,
                                            T& gx, T& gy, T& gz, T& lp) {
  if constexpr (I < 19) {
    const T v = T(psi[nbr(k, CX(I), CY(I), CZ(I), g)]);
    const T w = T(W(I));
    if constexpr (CX(I) != 0) gx += w * T(CX(I)) * v;
    if constexpr (CY(I) != 0) gy += w * T(CY(I)) * v;
    if constexpr (CZ(I) != 0) gz += w * T(CZ(I)) * v;
    lp += w * (v - c0);
    stencil_acc<T, F, I + 1>(psi, k, g, c0, gx, gy, gz, lp);
  }
}

template <typename T, typename F>
__device__ __forceinline__ void stencil3(const F* psi, const Node& k, const Geom3& g, T& gx,
                                         T& gy, T& gz, T& lp) {
  const T c0 = T(psi[k.n]);
  gx = gy = gz = lp = T(0);
  stencil_acc<T, F>(psi, k, g, c0, gx, gy, gz, lp);
  gx *= T(3);
  gy *= T(3);
  gz *= T(3);
  lp *= T(6);
}

// ------------------------------------------------------------- node algebra
template <typename T>
struct Node3 {
  T phi, rho, mu, p, D;
  T u[3], F[3], dr[3];
};

// Force, velocity and pressure (Sec. III moments with three components).
template <typename T>
__device__ __forceinline__ void macro3(T phi, T mu, const T gph[3], const T gmu[3], T lapmu,
                                       T S, const T j[3], const Coef3<T>& k, Node3<T>& m) {
  const Coef<T>& c = k.c;
  m.phi = phi;
  m.mu = mu;
  m.rho = c.rho_B + c.drho * phi;
  m.D = c.lam * lapmu;
  const T b = m.rho - c.rho_ref;
  const T gv[3] = {c.gx, c.gy, k.gz};
  const T inv = T(3) * recip(m.rho);
  T ud = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    m.dr[a] = c.drho * gph[a];
    m.F[a] = -phi * gmu[a] + b * gv[a];
    m.u[a] = (j[a] + m.F[a] * T(1.0 / 6.0)) * inv;
    ud += m.u[a] * m.dr[a];
  }
  m.p = S + T(1.0 / 6.0) * (ud - c.gamma * m.rho * m.D);
}

// c.(x, y, z) for a D3Q19 direction known at compile time (at most two
// nonzero components): signs and one sum, no products.
template <int CXV, int CYV, int CZV, typename T>
__device__ __forceinline__ T cdot3(T x, T y, T z) {
  static_assert(CXV == 0 || CYV == 0 || CZV == 0, "D3Q19: at most two nonzero components");
  if constexpr (CXV == 0) return qilbm::cdot<CYV, CZV>(y, z);
  else if constexpr (CYV == 0) return qilbm::cdot<CXV, CZV>(x, z);
  else return qilbm::cdot<CXV, CYV>(x, y);
}

// What every direction of one node's collision shares (three components):
// u, 1.5 |u|^2, F, grad rho / 3, grad p - F and their dot products with u.
template <typename T>
struct CollNode3 {
  T u[3], usq15;
  T F[3], uF;
  T d[3], ud;
  T q[3], uq;
};

template <typename T>
__device__ __forceinline__ CollNode3<T> coll_node3(const Node3<T>& m, const T dp[3]) {
  CollNode3<T> n;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    n.u[a] = m.u[a];
    n.F[a] = m.F[a];
    n.d[a] = m.dr[a] * T(1.0 / 3.0);
    n.q[a] = dp[a] - m.F[a];
  }
  n.usq15 = T(1.5) * fmad(m.u[2], m.u[2], fmad(m.u[1], m.u[1], m.u[0] * m.u[0]));
  n.uF = fmad(m.u[2], n.F[2], fmad(m.u[1], n.F[1], m.u[0] * n.F[0]));
  n.ud = fmad(m.u[2], n.d[2], fmad(m.u[1], n.d[1], m.u[0] * n.d[0]));
  n.uq = fmad(m.u[2], n.q[2], fmad(m.u[1], n.q[1], m.u[0] * n.q[0]));
  return n;
}

// Direction I: s = 3 c.u + 4.5 (c.u)^2 - 1.5 u^2, X = (c-u).(Gamma F +
// s grad rho / 3) = A + s (A + B), Y = Gamma (c-u).(grad p - F) = Q + s Q.
template <int I, typename T>
__device__ __forceinline__ void coll_dir3(const CollNode3<T>& n, T& s, T& X, T& Y) {
  T A, B, Q;
  if constexpr (I == 0) {
    s = -n.usq15;
    A = -n.uF;
    B = -n.ud;
    Q = -n.uq;
  } else {
    constexpr int cx = CX(I), cy = CY(I), cz = CZ(I);
    const T cu = cdot3<cx, cy, cz>(n.u[0], n.u[1], n.u[2]);
    s = fmad(cu, fmad(T(4.5), cu, T(3)), -n.usq15);
    A = cdot3<cx, cy, cz>(n.F[0], n.F[1], n.F[2]) - n.uF;
    B = cdot3<cx, cy, cz>(n.d[0], n.d[1], n.d[2]) - n.ud;
    Q = cdot3<cx, cy, cz>(n.q[0], n.q[1], n.q[2]) - n.uq;
  }
  X = fmad(s, A + B, A);
  Y = fmad(s, Q, Q);
}

// Relaxation factors of one weight class J (rest 1/3, axis 1/18, edge 1/36):
//   f* = (1 - 1/tau_f) f + w [p/tau_f + kf src1] + w rho/(3 tau_f) s + w kf X
//   g* = (1 - 1/tau_g) g + H/tau_g + w phi/tau_g s + w kg K Y,
// src1 = -rho gamma D / 3, K = -3 phi / rho, H_0 = phi - (1 - w_0) alpha mu,
// H_J = w_J alpha mu; formed just before the class's directions.
template <typename T>
struct CollF3 {
  T pf, rf, amu, ph, K, phi;
};

template <typename T>
struct CollK3 {
  T f0, fs, fx, g0, gs, gy;
};

template <typename T>
__device__ __forceinline__ CollF3<T> coll_f3(const Node3<T>& m, const Coef<T>& c) {
  CollF3<T> q;
  q.pf = fmad(m.p, c.inv_tau_f, -(m.rho * m.D) * (c.kf * c.gamma * T(1.0 / 3.0)));
  q.rf = m.rho * (c.inv_tau_f * T(1.0 / 3.0));
  q.amu = c.alpha * m.mu;
  q.ph = m.phi * c.inv_tau_g;
  q.K = -T(3) * m.phi * recip(m.rho);
  q.phi = m.phi;
  return q;
}

template <int J> __host__ __device__ constexpr double wclass3() {
  return J == 0 ? 1.0 / 3.0 : (J == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
}
template <int I> __host__ __device__ constexpr int wclass3_of() {
  return I == 0 ? 0 : (I <= 6 ? 1 : 2);
}

template <int J, typename T>
__device__ __forceinline__ CollK3<T> coll_k3(const CollF3<T>& q, const Coef<T>& c) {
  constexpr double wd = wclass3<J>();
  const T w = T(wd);
  CollK3<T> k;
  k.f0 = w * q.pf;
  k.fs = w * q.rf;
  k.fx = w * c.kf;
  k.gs = w * q.ph;
  k.gy = q.K * (w * c.kg);
  if constexpr (J == 0) k.g0 = fmad(-T(1.0 - wd), q.amu, q.phi) * c.inv_tau_g;
  else k.g0 = q.amu * (w * c.inv_tau_g);
  return k;
}

template <int I = 0, typename T>
__device__ __forceinline__ void collide3_dirs(T f[19], T gg[19], const CollNode3<T>& n,
                                              const CollF3<T>& q, CollK3<T> k,
                                              const Coef<T>& c, T af, T ag) {
  if constexpr (I < 19) {
    if constexpr (I == 0 || I == 1 || I == 7) k = coll_k3<wclass3_of<I>()>(q, c);
    T s, X, Y;
    coll_dir3<I>(n, s, X, Y);
    f[I] = fmad(af, f[I], fmad(k.fx, X, fmad(k.fs, s, k.f0)));
    gg[I] = fmad(ag, gg[I], fmad(k.gy, Y, fmad(k.gs, s, k.g0)));
    collide3_dirs<I + 1>(f, gg, n, q, k, c, af, ag);
  }
}

// BGK collisions of both populations with their sources (Sec. III):
// f^eq = w (p + rho s / 3), F_i = w (c-u).(Gamma F + s grad rho / 3)
// - w rho gamma D / 3, g^eq = H_i + w phi s, G_i = -3 (phi/rho) w Gamma
// (c-u).(grad p - F), x* = x - (x - x^eq)/tau + (1 - 1/(2 tau)) X_i, through
// the shared per-node and per-weight-class factors above.
template <typename T>
__device__ __forceinline__ void collide3(T f[19], T gg[19], const Node3<T>& m, const T dp[3],
                                         const Coef<T>& c) {
  const CollNode3<T> n = coll_node3(m, dp);
  const CollF3<T> q = coll_f3(m, c);
  collide3_dirs(f, gg, n, q, CollK3<T>{}, c, T(1) - c.inv_tau_f, T(1) - c.inv_tau_g);
}

template <int I = 0, typename T>
__device__ __forceinline__ void trt3_terms(T gg[19], T feq[19], T Fs[19], const CollNode3<T>& n,
                                           const CollF3<T>& q, CollK3<T> k, const Node3<T>& m,
                                           const Coef<T>& c, T src1, T ag) {
  if constexpr (I < 19) {
    if constexpr (I == 0 || I == 1 || I == 7) k = coll_k3<wclass3_of<I>()>(q, c);
    const T w = T(W(I));
    T s, X, Y;
    coll_dir3<I>(n, s, X, Y);
    feq[I] = w * fmad(m.rho * T(1.0 / 3.0), s, m.p);
    Fs[I] = w * (X + src1);
    gg[I] = fmad(ag, gg[I], fmad(k.gy, Y, fmad(k.gs, s, k.g0)));
    trt3_terms<I + 1>(gg, feq, Fs, n, q, k, m, c, src1, ag);
  }
}

// Two-relaxation-time variant of the f collision (g keeps BGK): f, f^eq and
// F_i split into parts even and odd under c_i -> -c_i (the D3Q19 opposite
// pairs); the even part relaxes with tau_f, the odd part with tau_-, each
// source part with its own 1 - 1/(2 tau) (Ginzburg, Verhaeghe and
// d'Humieres, 2008).
template <typename T>
__device__ __forceinline__ void collide3_trt(T f[19], T gg[19], const Node3<T>& m, const T dp[3],
                                             const Coef<T>& c) {
  const CollNode3<T> n = coll_node3(m, dp);
  const CollF3<T> q = coll_f3(m, c);
  const T src1 = -m.rho * c.gamma * m.D * T(1.0 / 3.0);
  T feq[19], Fs[19];
  trt3_terms(gg, feq, Fs, n, q, CollK3<T>{}, m, c, src1, T(1) - c.inv_tau_g);
  f[0] = f[0] - (f[0] - feq[0]) * c.inv_tau_f + c.kf * Fs[0];
#pragma unroll
  for (int i = 1; i < 19; i += 2) {           // (i, i + 1) are opposite
    const int o = i + 1;
    const T fp = T(0.5) * (f[i] + f[o]), fm = T(0.5) * (f[i] - f[o]);
    const T ep = T(0.5) * (feq[i] + feq[o]), em = T(0.5) * (feq[i] - feq[o]);
    const T sp = T(0.5) * (Fs[i] + Fs[o]), sm = T(0.5) * (Fs[i] - Fs[o]);
    const T dpl = c.kf * sp - (fp - ep) * c.inv_tau_f;
    const T dmi = c.km * sm - (fm - em) * c.inv_tau_m;
    f[i] = f[i] + dpl + dmi;
    f[o] = f[o] + dpl - dmi;
  }
}

__host__ __device__ constexpr bool opposite_pairs_adjacent() {
  for (int i = 1; i < 19; i += 2)
    if (CX(i + 1) != -CX(i) || CY(i + 1) != -CY(i) || CZ(i + 1) != -CZ(i)) return false;
  return true;
}
static_assert(opposite_pairs_adjacent(), "the pair loop assumes (i, i + 1) opposite");

// ------------------------------------------------------------------ kernels
#define QILBM3_FOR_NODES(n, g)                                                   \
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < (g).N;          \
       n += (int64_t)gridDim.x * 256)

template <int P>
__global__ __launch_bounds__(256) void k3_init(const double* __restrict__ phi0, Pop3<P> out,
                                               Coef3<double> k, Geom3 g) {
  QILBM3_FOR_NODES(n, g) {
    const Node nd = node_of(n, g);
    double gx, gy, gz, lp;
    stencil3<double, double>(phi0, nd, g, gx, gy, gz, lp);
    const double phi = phi0[n];
    const double mu = mu_bulk(phi, k.c) - k.c.kappa * lp;
    const double amu = k.c.alpha * mu;
    // pull layout: g_i pre-collision at x lives in slot (i, x - c_i) (or
    // (opp(i), x) beyond a wall); scatter each H_i to the slot it is pulled from
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const double h = i == 0 ? phi - (1.0 - 1.0 / 3.0) * amu : W(i) * amu;
      int zs = nd.z - CZ(i), plane = i;
      uint32_t e;
      if ((zs < 0 || zs >= g.nz) && g.walls) {
        plane = OPP(i);
        e = nd.n;
      } else {
        e = idx3(wrapi(nd.x - CX(i), g.nx), wrapi(nd.y - CY(i), g.ny), wrapi(zs, g.nz), g);
      }
      out.set_f(plane, e, typename PrecT<P>::T(0));
      out.set_g_d(plane, e, h);
    }
  }
}

// ------------------------------------------------------ row-wave kernels
// Work unit of the step kernels: one wave (64 lanes) takes 64 consecutive x
// of one (y, z) row. Everything that depends on y and z -- periodic wrap,
// the walls, the element index of the 3 x 3 neighbouring rows -- is then
// uniform across the wave and sits in scalar registers; a lane only holds
// its x and the wrapped x - 1, x + 1. Memory goes through buffer
// descriptors: the lane's byte offset in x (voffset) plus a scalar
// plane-and-row offset (soffset), so a neighbour access costs no vector
// address arithmetic and no integer division anywhere.
struct RowCtx {
  uint32_t rb[3][3];   // element index of (0, y + cy, z + cz), cy, cz in -1..1;
                       // beyond a wall z is clamped (mirrored ghost plane)
  bool below, above;   // walls: plane z - 1 / z + 1 lies beyond a wall
};

struct Lane {
  uint32_t xo[3];      // byte offsets of x - 1, x, x + 1 (wrapped)
  uint32_t x;
};

__device__ __forceinline__ RowCtx row_ctx(uint32_t y, uint32_t z, const Geom3& g) {
  RowCtx R;
  const uint32_t nx = g.nx, ny = g.ny, nz = g.nz;
  const bool wl = g.walls;
  const uint32_t ys[3] = {y == 0 ? ny - 1 : y - 1, y, y + 1 == ny ? 0 : y + 1};
  const uint32_t zs[3] = {z == 0 ? (wl ? 0 : nz - 1) : z - 1, z,
                          z + 1 == nz ? (wl ? z : 0) : z + 1};
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) R.rb[a][b] = (zs[b] * ny + ys[a]) * nx;
  R.below = wl && z == 0;
  R.above = wl && z + 1 == nz;
  return R;
}

template <int WS>
__device__ __forceinline__ Lane lane_of(uint32_t x, const Geom3& g) {
  Lane L;
  const uint32_t nx = g.nx;
  L.x = x;
  L.xo[0] = (x == 0 ? nx - 1 : x - 1) * WS;
  L.xo[1] = x * WS;
  L.xo[2] = (x + 1 == nx ? 0 : x + 1) * WS;
  return L;
}

// Rows are taken in blocks of RB x RB (y, z) rows, y fastest inside a block,
// so that the rows a stencil touches (y +- 1, z +- 1) are processed close
// together in time and their field values are still in L2.
constexpr uint32_t RB = 16;

__host__ __device__ inline uint32_t row_blocks(int n) { return ((uint32_t)n + RB - 1) / RB; }

// Waves over the padded block grid: 64-column chunks x (blocks of RB x RB rows).
__host__ __device__ inline uint32_t row_tasks(const Geom3& g, uint32_t nxc) {
  return nxc * row_blocks(g.ny) * row_blocks(g.nz) * RB * RB;
}

// Runs fn(row, lane) for every node, one (row, 64-column chunk) per wave;
// blocks are placed XCD-contiguously over the tasks. Waves on padding rows
// of the last blocks skip.
template <int WS, typename Fn>
__device__ __forceinline__ void for_rows(const Geom3& g, uint32_t nxc, Fn&& fn) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t nb = gridDim.x;
  const uint32_t b = (uint32_t)xcd_tile((int)blockIdx.x, (int)nb);
  const uint32_t ntask = row_tasks(g, nxc);
  const uint32_t nyb = row_blocks(g.ny);
  for (uint32_t t = (uint32_t)__builtin_amdgcn_readfirstlane((int)(b * 4 + (threadIdx.x >> 6)));
       t < ntask; t += nb * 4) {
    const uint32_t r = t / nxc, xc = t - r * nxc;
    const uint32_t blk = r / (RB * RB), w = r - blk * (RB * RB);
    const uint32_t bz = blk / nyb, by = blk - bz * nyb;
    const uint32_t y = by * RB + w % RB, z = bz * RB + w / RB;
    if (y >= (uint32_t)g.ny || z >= (uint32_t)g.nz) continue;
    const uint32_t x = xc * 64 + lane;
    if (x < (uint32_t)g.nx) fn(row_ctx(y, z, g), lane_of<WS>(x, g));
  }
}

// Equally spaced planes of words S; one descriptor for all of them when
// they span less than 4 GiB (BIG = false), else one per plane.
template <typename S, bool BIG>
struct Planes {
  char* base;
  uint32_t pb;                     // plane stride in bytes
  __amdgpu_buffer_rsrc_t all;
  __device__ __forceinline__ Planes(const void* b, int64_t Ns, int nplanes)
      : base((char*)b), pb((uint32_t)(Ns * (int64_t)sizeof(S))) {
    if constexpr (!BIG)
      all = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)((int64_t)nplanes * pb), BUF_WORD3);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(int plane) const {
    if constexpr (BIG)
      return __builtin_amdgcn_make_buffer_rsrc(base + (int64_t)plane * pb, 0, (int)pb, BUF_WORD3);
    else
      return all;
  }
  __device__ __forceinline__ uint32_t soff(int plane, uint32_t row) const {
    return (BIG ? 0u : (uint32_t)plane * pb) + row * (uint32_t)sizeof(S);
  }
  __device__ __forceinline__ S ld(int plane, uint32_t row, uint32_t vo) const {
    return buf_ld<S>(rsrc(plane), vo, soff(plane, row));
  }
  __device__ __forceinline__ void st(int plane, uint32_t row, uint32_t vo, S v) const {
    buf_st<S>(v, rsrc(plane), vo, soff(plane, row));
  }
  // byte offsets: sb (scalar, within the plane) and vb (per lane)
  __device__ __forceinline__ S ldb(int plane, uint32_t sb, uint32_t vb) const {
    return buf_ld<S>(rsrc(plane), vb, (BIG ? 0u : (uint32_t)plane * pb) + sb);
  }
  __device__ __forceinline__ void stb(int plane, uint32_t sb, uint32_t vb, S v) const {
    buf_st<S>(v, rsrc(plane), vb, (BIG ? 0u : (uint32_t)plane * pb) + sb);
  }
};

// The two population sets of a buffer: f (T) and g (T, or Q2.29 words).
template <int P, bool BIG>
struct PopView {
  using T = typename PrecT<P>::T;
  using GW = typename std::conditional<P == P_F64, double, int32_t>::type;
  Planes<T, BIG> f;
  Planes<GW, BIG> g;
  __device__ __forceinline__ explicit PopView(const Pop3<P>& p)
      : f(p.base, p.Ns, 19), g(p.base + 19 * p.Ns * (int64_t)sizeof(T), p.Ns, 19) {}
};

// Slot holding the pre-collision population i of the lane's node.
struct Src {
  int plane;
  uint32_t row, vo;
};

__device__ __forceinline__ Src pull_at(int i, const RowCtx& R, const Lane& L) {
  const int cz = CZ(i);
  const bool beyond = (cz == 1 && R.below) || (cz == -1 && R.above);
  Src s;
  s.plane = beyond ? OPP(i) : i;
  s.row = beyond ? R.rb[1][1] : R.rb[1 - CY(i)][1 - cz];
  s.vo = beyond ? L.xo[1] : L.xo[1 - CX(i)];
  return s;
}

// Isotropic gradient and Laplacian of a field (in direction order).
template <typename T>
__device__ __forceinline__ void stencil_r(const Planes<T, false>& F, const RowCtx& R,
                                          const Lane& L, T& c0, T& gx, T& gy, T& gz, T& lp) {
  c0 = F.ld(0, R.rb[1][1], L.xo[1]);
  gx = gy = gz = lp = T(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const T v = F.ld(0, R.rb[CY(i) + 1][CZ(i) + 1], L.xo[CX(i) + 1]);
    const T w = T(W(i));
    if (CX(i) != 0) gx += w * T(CX(i)) * v;
    if (CY(i) != 0) gy += w * T(CY(i)) * v;
    if (CZ(i) != 0) gz += w * T(CZ(i)) * v;
    lp += w * (v - c0);
  }
  gx *= T(3);
  gy *= T(3);
  gz *= T(3);
  lp *= T(6);
}

template <int P, bool BIG>
__global__ __launch_bounds__(256) void k3_phi(Pop3<P> in, typename PrecT<P>::T* __restrict__ phi,
                                              Geom3 g, uint32_t nxc) {
  using T = typename PrecT<P>::T;
  const PopView<P, BIG> v(in);
  const Planes<T, false> out(phi, g.Ns, 1);
  for_rows<sizeof(T)>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    if constexpr (FixedG<P>::value) {
      int32_t q = 0;
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const Src s = pull_at(i, R, L);
        q += v.g.ld(s.plane, s.row, s.vo);
      }
      out.st(0, R.rb[1][1], L.xo[1], T(q) * T(GQI));
    } else {
      T a = T(0);
#pragma unroll
      for (int i = 0; i < 19; ++i) {
        const Src s = pull_at(i, R, L);
        a += v.g.ld(s.plane, s.row, s.vo);
      }
      out.st(0, R.rb[1][1], L.xo[1], a);
    }
  });
}

// Pulled f of the lane's node and the node state from it and the phi, mu
// fields.
template <int P, bool BIG>
__device__ __forceinline__ void node_state_r(const PopView<P, BIG>& v,
                                             const Planes<typename PrecT<P>::T, false>& ph,
                                             const Planes<typename PrecT<P>::T, false>& mf,
                                             const RowCtx& R, const Lane& L,
                                             const Coef3<typename PrecT<P>::T>& k,
                                             typename PrecT<P>::T f[19],
                                             Node3<typename PrecT<P>::T>& m,
                                             typename PrecT<P>::T* jout = nullptr) {
  using T = typename PrecT<P>::T;
#pragma unroll
  for (int i = 0; i < 19; ++i) {
    const Src s = pull_at(i, R, L);
    f[i] = v.f.ld(s.plane, s.row, s.vo);
  }
  T S = f[0], j[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    S += f[i];
    if (CX(i) != 0) j[0] += T(CX(i)) * f[i];
    if (CY(i) != 0) j[1] += T(CY(i)) * f[i];
    if (CZ(i) != 0) j[2] += T(CZ(i)) * f[i];
  }
  T phi, mu, gph[3], gmu[3], lphi, lmu;
  stencil_r<T>(ph, R, L, phi, gph[0], gph[1], gph[2], lphi);
  stencil_r<T>(mf, R, L, mu, gmu[0], gmu[1], gmu[2], lmu);
  macro3<T>(phi, mu, gph, gmu, lmu, S, j, k, m);
  if (jout) {
    jout[0] = j[0];
    jout[1] = j[1];
    jout[2] = j[2];
  }
}

struct MomentOut3 {
  double *phi = nullptr, *rho = nullptr, *u[3] = {nullptr, nullptr, nullptr}, *p = nullptr,
         *mu = nullptr;
};

template <int P, bool BIG>
__global__ __launch_bounds__(256) void k3_macro(Pop3<P> in, const typename PrecT<P>::T* __restrict__ phi,
                                                const typename PrecT<P>::T* __restrict__ mu,
                                                typename PrecT<P>::T* __restrict__ p,
                                                MomentOut3 mo, Coef3<typename PrecT<P>::T> k,
                                                Geom3 g, uint32_t nxc) {
  using T = typename PrecT<P>::T;
  const PopView<P, BIG> v(in);
  const Planes<T, false> ph(phi, g.Ns, 1), mf(mu, g.Ns, 1), pf(p, g.Ns, 1);
  for_rows<sizeof(T)>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    T f[19];
    Node3<T> m;
    node_state_r<P, BIG>(v, ph, mf, R, L, k, f, m);
    if (p) pf.st(0, R.rb[1][1], L.xo[1], m.p);
    const uint32_t n = R.rb[1][1] + L.x;
    if (mo.phi) mo.phi[n] = double(m.phi);
    if (mo.rho) mo.rho[n] = double(m.rho);
    for (int a = 0; a < 3; ++a)
      if (mo.u[a]) mo.u[a][n] = double(m.u[a]);
    if (mo.p) mo.p[n] = double(m.p);
    if (mo.mu) mo.mu[n] = double(m.mu);
  });
}

// The collision in two kernels, so that each population set is pulled once:
// f's collision needs no grad p, so k3_pf collides f where it forms the
// pressure (and keeps j for k3_g); k3_g, after every p is written, pulls g
// and collides it with grad p and with u and F re-formed from j and the
// phi, mu stencils (the same arithmetic as in k3_pf; the pressure, which g
// does not use, is left out).
template <int P, bool BIG, bool TRT = false>
__global__ __launch_bounds__(256) void k3_pf(Pop3<P> in, Pop3<P> out,
                                             const typename PrecT<P>::T* __restrict__ phi,
                                             const typename PrecT<P>::T* __restrict__ mu,
                                             typename PrecT<P>::T* __restrict__ p,
                                             typename PrecT<P>::T* __restrict__ jx,
                                             typename PrecT<P>::T* __restrict__ jy,
                                             typename PrecT<P>::T* __restrict__ jz,
                                             Coef3<typename PrecT<P>::T> k, Geom3 g, uint32_t nxc) {
  using T = typename PrecT<P>::T;
  const PopView<P, BIG> v(in), w(out);
  const Planes<T, false> ph(phi, g.Ns, 1), mf(mu, g.Ns, 1), pf(p, g.Ns, 1);
  const Planes<T, false> jf[3] = {{jx, g.Ns, 1}, {jy, g.Ns, 1}, {jz, g.Ns, 1}};
  for_rows<sizeof(T)>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    T f[19], j[3];
    Node3<T> m;
    node_state_r<P, BIG>(v, ph, mf, R, L, k, f, m, j);
    const uint32_t row = R.rb[1][1], vo = L.xo[1];
    pf.st(0, row, vo, m.p);
#pragma unroll
    for (int a = 0; a < 3; ++a) jf[a].st(0, row, vo, j[a]);
    const T dp0[3] = {T(0), T(0), T(0)};
    T gd[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) gd[i] = T(0);
    if constexpr (TRT) collide3_trt<T>(f, gd, m, dp0, k.c);
    else collide3<T>(f, gd, m, dp0, k.c);
#pragma unroll
    for (int i = 0; i < 19; ++i) w.f.st(i, row, vo, f[i]);
  });
}

template <int P, bool BIG, bool TRT = false>
__global__ __launch_bounds__(256) void k3_g(Pop3<P> in, Pop3<P> out,
                                            const typename PrecT<P>::T* __restrict__ phi,
                                            const typename PrecT<P>::T* __restrict__ mu,
                                            const typename PrecT<P>::T* __restrict__ p,
                                            const typename PrecT<P>::T* __restrict__ jx,
                                            const typename PrecT<P>::T* __restrict__ jy,
                                            const typename PrecT<P>::T* __restrict__ jz,
                                            Coef3<typename PrecT<P>::T> k, Geom3 g, uint32_t nxc) {
  using T = typename PrecT<P>::T;
  const PopView<P, BIG> v(in), w(out);
  const Planes<T, false> ph(phi, g.Ns, 1), mf(mu, g.Ns, 1), pf(p, g.Ns, 1);
  const Planes<T, false> jf[3] = {{jx, g.Ns, 1}, {jy, g.Ns, 1}, {jz, g.Ns, 1}};
  for_rows<sizeof(T)>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    T gg[19];
    int32_t q = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const Src s = pull_at(i, R, L);
      if constexpr (FixedG<P>::value) {
        const int32_t word = v.g.ld(s.plane, s.row, s.vo);
        q += word;
        gg[i] = float(word) * GQI;
      } else {
        gg[i] = v.g.ld(s.plane, s.row, s.vo);
      }
    }
    const uint32_t row = R.rb[1][1], vo = L.xo[1];
    const T j[3] = {jf[0].ld(0, row, vo), jf[1].ld(0, row, vo), jf[2].ld(0, row, vo)};
    T phi, mu, gph[3], gmu[3], lphi, lmu;
    stencil_r<T>(ph, R, L, phi, gph[0], gph[1], gph[2], lphi);
    stencil_r<T>(mf, R, L, mu, gmu[0], gmu[1], gmu[2], lmu);
    Node3<T> m;
    macro3<T>(phi, mu, gph, gmu, lmu, T(0), j, k, m);
    T p0, dp[3], lapp;
    stencil_r<T>(pf, R, L, p0, dp[0], dp[1], dp[2], lapp);
    T fd[19];
#pragma unroll
    for (int i = 0; i < 19; ++i) fd[i] = T(0);
    if constexpr (TRT) collide3_trt<T>(fd, gg, m, dp, k.c);
    else collide3<T>(fd, gg, m, dp, k.c);
    if constexpr (FixedG<P>::value) {
      // g_0 closes the node's Q2.29 sum at the pulled total q
      int32_t rest = 0;
#pragma unroll
      for (int i = 1; i < 19; ++i) {
        const int32_t word = __float2int_rn(gg[i] * GQ);
        rest += word;
        w.g.st(i, row, vo, word);
      }
      w.g.st(0, row, vo, q - rest);
    } else {
#pragma unroll
      for (int i = 0; i < 19; ++i) w.g.st(i, row, vo, gg[i]);
    }
  });
}

// Q2.29 sum of the pulled g words of every node (the order parameter the
// fused FP32 step reads in its stage A).
template <bool BIG>
__global__ __launch_bounds__(256) void k3_phiq(Pop3<P_F32> in, int32_t* __restrict__ phiq, Geom3 g,
                                               uint32_t nxc) {
  const PopView<P_F32, BIG> v(in);
  for_rows<4>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    int32_t q = 0;
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const Src s = pull_at(i, R, L);
      q += v.g.ld(s.plane, s.row, s.vo);
    }
    phiq[R.rb[1][1] + L.x] = q;
  });
}

// ------------------------------------------------------ fused z-sweep step
// One kernel per time step. A workgroup owns a TX x TY tile of (x, y) and a
// segment [z0, z1) of planes and sweeps it in z. In the iteration that
// reaches plane a it
//   A: forms phi(a) from the pulled g over the tile plus 3 halo nodes,
//   B: forms mu(a-1) from the phi planes a-2..a over the tile plus 2,
//   C: forms the pressure p(a-2) from its pulled f and the phi, mu stencils
//      over the tile plus 1, and on the tile itself collides f (its
//      collision needs no grad p) and writes it,
//   D: collides g of plane a-3 of the tile (grad p from the p planes
//      a-4..a-2, u and F from the j that C kept in registers) and writes it.
// phi, mu and p live in LDS rings of 5, 4 and 3 planes; each population set
// is pulled from HBM once (f by C, g by D) and written once. Halo nodes and
// the 3 planes of warm-up at each segment end are
// recomputed by the neighbouring workgroups. Results equal those of the
// four-kernel path up to the rounding order of contracted multiply-adds.
// (The four kernels split the two collisions the same way.)
// Used for FP32 only, with stage A reading phi from the Q2.29 words that the
// previous step scattered (PHIQ below): pulling g there over the halo made
// the kernel read 453 B per node (those re-reads miss L2), against 252 with
// the scattered phi. In FP64 (no integer g; LDS rings for one 512-lane
// workgroup per CU, barrier-bound) the fused form was a quarter slower than
// the four kernels.
namespace fz {
// 64 x 16 columns on 512 lanes (two core nodes per lane): 79 KB of LDS,
// one workgroup (eight waves) per CU, 3 % faster than 64 x 8 columns on 256
// lanes (48 KB, three per CU): the ring of the pressure stage is 16 % of
// the tile instead of 29 %; 128 x 8 on 512 lanes 5 % slower
constexpr int TX = 64, TY = 16;
template <int H>
struct Reg {
  static constexpr int W = TX + 2 * H, HT = TY + 2 * H, A = W * HT;
};
constexpr int RPHI = 5, RMU = 4, RP = 3;
}  // namespace fz

template <int P>
struct FzThreads {
  static constexpr int value = 512;
};

// node rounds of stages C and D unrolled together (loads of several nodes
// in flight at once)
template <int P>
struct FzUnrollD {
  static constexpr int value = 2;
};

template <int P>
struct FzLds {
  using T = typename PrecT<P>::T;
  T phi[fz::RPHI][fz::Reg<3>::A];
  T mu[fz::RMU][fz::Reg<2>::A];
  T p[fz::RP][fz::Reg<1>::A];
};

// With the scattered order parameter: three planes of Q2.29 partial sums of
// the next step's phi over the core tile and a one-node ring around it (the
// targets of every word the tile's nodes stream).
template <int P>
struct FzLdsQ : FzLds<P> {
  int32_t acc[3][fz::Reg<1>::A];
};

struct Fz3Shape {
  int ntx, nty, nseg, seg;
};

__device__ __forceinline__ int wrapm(int v, int n) {
  while (v < 0) v += n;
  while (v >= n) v -= n;
  return v;
}

// Byte offsets of a node's x - 1, x, x + 1 and of its rows y - 1, y, y + 1
// (wrapped) within a plane.
struct XY {
  uint32_t xo[3], yo[3];
};

template <int WS>
__device__ __forceinline__ XY xy_of(int gx, int gy, const Geom3& g) {
  XY q;
  const int nx = g.nx, ny = g.ny;
  q.xo[0] = (uint32_t)(gx == 0 ? nx - 1 : gx - 1) * WS;
  q.xo[1] = (uint32_t)gx * WS;
  q.xo[2] = (uint32_t)(gx + 1 == nx ? 0 : gx + 1) * WS;
  q.yo[0] = (uint32_t)(gy == 0 ? ny - 1 : gy - 1) * (uint32_t)nx * WS;
  q.yo[1] = (uint32_t)gy * (uint32_t)nx * WS;
  q.yo[2] = (uint32_t)(gy + 1 == ny ? 0 : gy + 1) * (uint32_t)nx * WS;
  return q;
}

// Planes z - 1, z, z + 1 of global plane z as byte offsets (wrapped; at a
// wall the missing plane is flagged and never addressed).
struct ZP {
  uint32_t zo[3];
  bool below, above;
};

template <int WS>
__device__ __forceinline__ ZP zp_of(int z, const Geom3& g) {
  ZP Z;
  const uint32_t pl = (uint32_t)g.nx * (uint32_t)g.ny * WS;
  const int nz = g.nz;
  Z.zo[0] = (uint32_t)(z == 0 ? nz - 1 : z - 1) * pl;
  Z.zo[1] = (uint32_t)z * pl;
  Z.zo[2] = (uint32_t)(z + 1 == nz ? 0 : z + 1) * pl;
  Z.below = g.walls && z == 0;
  Z.above = g.walls && z + 1 == nz;
  return Z;
}

struct SrcB {
  int plane;
  uint32_t sb, vb;
};

// a[k] for k in 0..2 as selects (no private array when k is not a constant)
__device__ __forceinline__ uint32_t pick3(const uint32_t a[3], int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}

// Slot of the pre-collision population i of a node (pull; bounce-back
// from the node's own opposite slot beyond a wall).
__device__ __forceinline__ SrcB pull_b(int i, const ZP& Z, const XY& q) {
  const int cz = CZ(i);
  const bool beyond = (cz == 1 && Z.below) || (cz == -1 && Z.above);
  SrcB s;
  s.plane = beyond ? OPP(i) : i;
  s.sb = beyond ? Z.zo[1] : pick3(Z.zo, 1 - cz);
  s.vb = beyond ? q.yo[1] + q.xo[1] : pick3(q.yo, 1 - CY(i)) + pick3(q.xo, 1 - CX(i));
  return s;
}

// Isotropic gradient and Laplacian from three LDS planes of a region of
// row width RW, at index o (same accumulation order as stencil_r).
template <typename T, int RW>
__device__ __forceinline__ void lds_stencil(const T* pm, const T* p0, const T* pp, int o, T& c0,
                                            T& gx, T& gy, T& gz, T& lp) {
  c0 = p0[o];
  gx = gy = gz = lp = T(0);
#pragma unroll
  for (int i = 1; i < 19; ++i) {
    const T* pl = CZ(i) < 0 ? pm : (CZ(i) > 0 ? pp : p0);
    const T v = pl[o + CY(i) * RW + CX(i)];
    const T w = T(W(i));
    if (CX(i) != 0) gx += w * T(CX(i)) * v;
    if (CY(i) != 0) gy += w * T(CY(i)) * v;
    if (CZ(i) != 0) gz += w * T(CZ(i)) * v;
    lp += w * (v - c0);
  }
  gx *= T(3);
  gy *= T(3);
  gz *= T(3);
  lp *= T(6);
}

// mu = mu_bulk(phi) - kappa lap(phi) (Sec. II, the chemical potential) of a
// 64 x 4 column tile over a segment of MZ_ZS planes: the phi planes of the
// tile and the ring of nodes around it go through a ring of four LDS planes,
// so each phi value is read from memory about once instead of once per
// stencil neighbour. Beyond a wall the mirrored ghost plane is the wall plane
// itself; x, y and (without walls) z are periodic.
constexpr int MZ_TX = 64, MZ_TY = 4, MZ_W = MZ_TX + 2, MZ_A = MZ_W * (MZ_TY + 2), MZ_ZS = 32;

__host__ __device__ inline int mu_tiles_xy(const Geom3& g) {
  return ((g.nx + MZ_TX - 1) / MZ_TX) * ((g.ny + MZ_TY - 1) / MZ_TY);
}

template <typename T>
__global__ __launch_bounds__(256) void k3_mu(const T* __restrict__ phi, T* __restrict__ mu,
                                             Coef3<T> k, Geom3 g) {
  __shared__ T ring[4][MZ_A];
  const int ntx = (g.nx + MZ_TX - 1) / MZ_TX, nxy = mu_tiles_xy(g);
  const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int seg = b / nxy, txy = b - seg * nxy;
  const int ty = txy / ntx, tx = txy - ty * ntx;
  const int x0 = tx * MZ_TX, y0 = ty * MZ_TY;
  const int z0 = seg * MZ_ZS, z1 = min(g.nz, z0 + MZ_ZS);
  const int t = threadIdx.x, lx = t & 63, ly = t >> 6;
  const int x = x0 + lx, y = y0 + ly;
  const uint32_t nx = (uint32_t)g.nx, ny = (uint32_t)g.ny;
  // plane zz of the sweep (z0 - 1 .. z1) into its ring slot
  auto load_plane = [&](int zz) {
    int zp = zz;
    if (zp < 0) zp = g.walls ? 0 : zp + g.nz;
    else if (zp >= g.nz) zp = g.walls ? g.nz - 1 : zp - g.nz;
    T* dst = ring[zz & 3];
    for (int e = t; e < MZ_A; e += 256) {
      const int ey = e / MZ_W, ex = e - ey * MZ_W;
      // the halo can reach more than one period on narrow lattices
      const int gx = (x0 - 1 + ex + g.nx) % g.nx, gy = (y0 - 1 + ey + g.ny) % g.ny;
      dst[e] = phi[((uint32_t)zp * ny + (uint32_t)gy) * nx + (uint32_t)gx];
    }
  };
  load_plane(z0 - 1);
  load_plane(z0);
  // plane z + 1 goes into the slot of z - 3, which no lane reads after the
  // barrier of the iteration before: one barrier per plane
  for (int z = z0; z < z1; ++z) {
    load_plane(z + 1);
    __syncthreads();
    if (x < g.nx && y < g.ny) {
      T c0, gx, gy, gz, lp;
      lds_stencil<T, MZ_W>(ring[(z - 1) & 3], ring[z & 3], ring[(z + 1) & 3],
                           (ly + 1) * MZ_W + lx + 1, c0, gx, gy, gz, lp);
      mu[((uint32_t)z * ny + (uint32_t)y) * nx + (uint32_t)x] = mu_bulk(c0, k.c) - k.c.kappa * lp;
    }
  }
}

// PHIQ (FP32 only): stage A reads phi as the Q2.29 sum phiq_in of the
// pulled g words (formed by the previous step), and stage D scatters each
// post-collision g word to the node it streams to, accumulating the next
// step's sum into phiq_out (zero on entry): integer sums, so the order of
// the additions does not matter and the result equals the pulled sum
// exactly. Every target (core tile plus a one-node ring) accumulates in LDS
// (three planes, flushed with one atomic add per node once a plane has all
// its sources from this tile).
template <int P, bool BIG, bool PHIQ = false, bool TRT = false>
__global__ __launch_bounds__(FzThreads<P>::value) void k3_fused(Pop3<P> in, Pop3<P> out,
                                                                Coef3<typename PrecT<P>::T> k,
                                                                Geom3 g, Fz3Shape sh,
                                                                const int32_t* __restrict__ phiq_in,
                                                                int32_t* __restrict__ phiq_out) {
  using T = typename PrecT<P>::T;
  using namespace fz;
  constexpr int NT = FzThreads<P>::value;
  constexpr int WS = sizeof(T);
  using RA = Reg<3>;
  using RB = Reg<2>;
  using RC = Reg<1>;
  static_assert(!PHIQ || FixedG<P>::value, "scattered phi needs integer g words");
  __shared__ typename std::conditional<PHIQ, FzLdsQ<P>, FzLds<P>>::type L;

  const int ntiles = sh.ntx * sh.nty;
  const int b = xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const int tile = b % ntiles, sg = b / ntiles;
  const int x0 = (tile % sh.ntx) * TX, y0 = (tile / sh.ntx) * TY;
  const int z0 = sg * sh.seg;
  if (z0 >= g.nz) return;                  // whole workgroup, before any barrier
  const int z1 = min(z0 + sh.seg, g.nz);
  const int nz = g.nz;
  const bool wl = g.walls;
  const int vbase = z0 - 3;
  const PopView<P, BIG> v(in), w(out);
  const int tid = threadIdx.x;

  // ring slot of virtual plane zz as read by a stencil (clamped at walls)
  auto slot = [&](int zz, int R) {
    if (wl) zz = zz < 0 ? 0 : (zz >= nz ? nz - 1 : zz);
    return (zz - vbase) % R;
  };
  auto real = [&](int zz) { return wl ? (zz >= 0 && zz < nz) : true; };
  const uint32_t planeN = (uint32_t)g.nx * (uint32_t)g.ny;
  // adds the LDS partial sums of virtual plane zf to phiq_out and clears
  // them; region node (ly, lx) is global column (x0 - 1 + lx, y0 - 1 + ly),
  // wrapped (positions that wrap onto the same node add up there)
  auto flush = [&](int zf) {
    if constexpr (PHIQ) {
      int32_t* acc = L.acc[(zf - vbase) % 3];
      const bool ok = real(zf);
      const uint32_t zb = ok ? (uint32_t)wrapm(zf, nz) * planeN : 0u;
      for (int r = tid; r < RC::A; r += NT) {
        const int ly = r / RC::W, lx = r - ly * RC::W;
        const int32_t v = acc[r];
        acc[r] = 0;
        if (ok && v != 0) {
          const uint32_t X = (uint32_t)wrapm(x0 - 1 + lx, g.nx);
          const uint32_t Y = (uint32_t)wrapm(y0 - 1 + ly, g.ny);
          atomicAdd(&phiq_out[zb + Y * (uint32_t)g.nx + X], v);
        }
      }
    }
  };
  if constexpr (PHIQ) {
    for (int r = tid; r < 3 * RC::A; r += NT) (&L.acc[0][0])[r] = 0;
    __syncthreads();
  }

  const int niter = (z1 - z0) + 6;
  // j of the core nodes (two per lane): formed by stage C, used by stage D
  // one iteration later
  static_assert((TX * TY + NT - 1) / NT == 2, "two core nodes per lane");
  T jn[2][3] = {}, jd[2][3] = {};
  for (int it = 0; it < niter; ++it) {
    const int a = vbase + it;
    // A: phi(a) over the tile plus 3
    if (real(a)) {
      const ZP Z = zp_of<WS>(wrapm(a, nz), g);
      T* dst = L.phi[slot(a, RPHI)];
#pragma unroll
      for (int rr = 0; rr < (RA::A + NT - 1) / NT; ++rr) {
        const int r = tid + rr * NT;
        if (r >= RA::A) break;
        const int ly = r / RA::W, lx = r - ly * RA::W;
        if constexpr (PHIQ) {
          const uint32_t e = (uint32_t)wrapm(a, nz) * planeN +
                             (uint32_t)wrapm(y0 - 3 + ly, g.ny) * (uint32_t)g.nx +
                             (uint32_t)wrapm(x0 - 3 + lx, g.nx);
          dst[r] = T(phiq_in[e]) * T(GQI);
          continue;
        }
        const XY q = xy_of<WS>(wrapm(x0 - 3 + lx, g.nx), wrapm(y0 - 3 + ly, g.ny), g);
        if constexpr (FixedG<P>::value) {
          int32_t s = 0;
#pragma unroll
          for (int i = 0; i < 19; ++i) {
            const SrcB o = pull_b(i, Z, q);
            s += v.g.ldb(o.plane, o.sb, o.vb);
          }
          dst[r] = T(s) * T(GQI);
        } else {
          T s = T(0);
#pragma unroll
          for (int i = 0; i < 19; ++i) {
            const SrcB o = pull_b(i, Z, q);
            s += v.g.ldb(o.plane, o.sb, o.vb);
          }
          dst[r] = s;
        }
      }
    }
    __syncthreads();
    // B: mu(a-1) over the tile plus 2
    const int zb = a - 1;
    if (zb >= z0 - 2 && zb < z1 + 2 && real(zb)) {
      const T* pm = L.phi[slot(zb - 1, RPHI)];
      const T* p0 = L.phi[slot(zb, RPHI)];
      const T* pp = L.phi[slot(zb + 1, RPHI)];
      T* dst = L.mu[slot(zb, RMU)];
#pragma unroll
      for (int rr = 0; rr < (RB::A + NT - 1) / NT; ++rr) {
        const int r = tid + rr * NT;
        if (r >= RB::A) break;
        const int ly = r / RB::W, lx = r - ly * RB::W;
        T c0, gx, gy, gz, lp;
        lds_stencil<T, RA::W>(pm, p0, pp, (ly + 1) * RA::W + lx + 1, c0, gx, gy, gz, lp);
        dst[r] = mu_bulk(c0, k.c) - k.c.kappa * lp;
      }
    }
    __syncthreads();
    // C: p(a-2) over the tile plus 1; the core nodes of an owned plane also
    // collide f here (f's collision needs no grad p) and store it, so that f
    // is pulled once: the core nodes in stage D's lane mapping, whose j waits
    // in registers for D of the next iteration, then the one-node ring
    const int zc = a - 2;
    if (zc >= z0 - 1 && zc < z1 + 1 && real(zc)) {
      const ZP Z = zp_of<WS>(wrapm(zc, nz), g);
      const T* fm = L.phi[slot(zc - 1, RPHI)];
      const T* f0 = L.phi[slot(zc, RPHI)];
      const T* fp = L.phi[slot(zc + 1, RPHI)];
      const T* mm = L.mu[slot(zc - 1, RMU)];
      const T* m0 = L.mu[slot(zc, RMU)];
      const T* mp = L.mu[slot(zc + 1, RMU)];
      T* dst = L.p[slot(zc, RP)];
      const bool own = zc >= z0 && zc < z1;
      // pulled f of region node (ly, lx) (tile + 1 coordinates) and its state
      auto node_c = [&](int ly, int lx, T f[19], Node3<T>& m, T j[3], XY& q) {
        q = xy_of<WS>(wrapm(x0 - 1 + lx, g.nx), wrapm(y0 - 1 + ly, g.ny), g);
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          const SrcB o = pull_b(i, Z, q);
          f[i] = v.f.ldb(o.plane, o.sb, o.vb);
        }
        T S = f[0];
        j[0] = j[1] = j[2] = T(0);
#pragma unroll
        for (int i = 1; i < 19; ++i) {
          S += f[i];
          if (CX(i) != 0) j[0] += T(CX(i)) * f[i];
          if (CY(i) != 0) j[1] += T(CY(i)) * f[i];
          if (CZ(i) != 0) j[2] += T(CZ(i)) * f[i];
        }
        T phi, mu, gph[3], gmu[3], lphi, lmu;
        lds_stencil<T, RA::W>(fm, f0, fp, (ly + 2) * RA::W + lx + 2, phi, gph[0], gph[1], gph[2],
                              lphi);
        lds_stencil<T, RB::W>(mm, m0, mp, (ly + 1) * RB::W + lx + 1, mu, gmu[0], gmu[1], gmu[2],
                              lmu);
        macro3<T>(phi, mu, gph, gmu, lmu, S, j, k, m);
        dst[ly * RC::W + lx] = m.p;
      };
#pragma unroll FzUnrollD<P>::value
      for (int rr = 0; rr < (TX * TY + NT - 1) / NT; ++rr) {
        const int r = tid + rr * NT;
        const int ly = r / TX, lx = r - ly * TX;
        T f[19], j[3];
        Node3<T> m;
        XY q;
        node_c(ly + 1, lx + 1, f, m, j, q);
        jn[rr][0] = j[0];
        jn[rr][1] = j[1];
        jn[rr][2] = j[2];
        if (own && x0 + lx < g.nx && y0 + ly < g.ny) {
          const T dp0[3] = {T(0), T(0), T(0)};
          T gd[19];
#pragma unroll
          for (int i = 0; i < 19; ++i) gd[i] = T(0);
          if constexpr (TRT) collide3_trt<T>(f, gd, m, dp0, k.c);
          else collide3<T>(f, gd, m, dp0, k.c);
          const uint32_t sb = Z.zo[1], vb = q.yo[1] + q.xo[1];
#pragma unroll
          for (int i = 0; i < 19; ++i) w.f.stb(i, sb, vb, f[i]);
        }
      }
      constexpr int RING = RC::A - TX * TY;    // 2 (TX + 2) + 2 TY
      for (int r = tid; r < RING; r += NT) {
        int ly, lx;
        if (r < RC::W) {
          ly = 0;
          lx = r;
        } else if (r < 2 * RC::W) {
          ly = RC::HT - 1;
          lx = r - RC::W;
        } else {
          const int e = r - 2 * RC::W;
          ly = 1 + (e >> 1);
          lx = (e & 1) ? RC::W - 1 : 0;
        }
        T f[19], j[3];
        Node3<T> m;
        XY q;
        node_c(ly, lx, f, m, j, q);
      }
    }
    __syncthreads();
    // D: collide g of plane a-3 of the tile (grad p from the p planes
    // a-4..a-2; u and F from the j that stage C kept) and store it
    const int zd = a - 3;
    if (zd >= z0 && zd < z1) {
      const ZP Z = zp_of<WS>(zd, g);
      const T* fm = L.phi[slot(zd - 1, RPHI)];
      const T* f0 = L.phi[slot(zd, RPHI)];
      const T* fp = L.phi[slot(zd + 1, RPHI)];
      const T* mm = L.mu[slot(zd - 1, RMU)];
      const T* m0 = L.mu[slot(zd, RMU)];
      const T* mp = L.mu[slot(zd + 1, RMU)];
      const T* qm = L.p[slot(zd - 1, RP)];
      const T* q0 = L.p[slot(zd, RP)];
      const T* qp = L.p[slot(zd + 1, RP)];
#pragma unroll FzUnrollD<P>::value
      for (int rr = 0; rr < (TX * TY + NT - 1) / NT; ++rr) {
        const int r = tid + rr * NT;
        const int ly = r / TX, lx = r - ly * TX;
        const int X = x0 + lx, Y = y0 + ly;
        if (X >= g.nx || Y >= g.ny) continue;
        const XY q = xy_of<WS>(X, Y, g);
        T gg[19];
        int32_t qs = 0;
#pragma unroll
        for (int i = 0; i < 19; ++i) {
          const SrcB o = pull_b(i, Z, q);
          if constexpr (FixedG<P>::value) {
            const int32_t word = v.g.ldb(o.plane, o.sb, o.vb);
            qs += word;
            gg[i] = float(word) * GQI;
          } else {
            gg[i] = v.g.ldb(o.plane, o.sb, o.vb);
          }
        }
        T phi, mu, gph[3], gmu[3], lphi, lmu, p0, dp[3], lpp;
        lds_stencil<T, RA::W>(fm, f0, fp, (ly + 3) * RA::W + lx + 3, phi, gph[0], gph[1], gph[2],
                              lphi);
        lds_stencil<T, RB::W>(mm, m0, mp, (ly + 2) * RB::W + lx + 2, mu, gmu[0], gmu[1], gmu[2],
                              lmu);
        lds_stencil<T, RC::W>(qm, q0, qp, (ly + 1) * RC::W + lx + 1, p0, dp[0], dp[1], dp[2], lpp);
        // the node state as stage C formed it (u, F from the same j and
        // stencils; the pressure, which g does not use, left out)
        const T j[3] = {jd[rr][0], jd[rr][1], jd[rr][2]};
        Node3<T> m;
        macro3<T>(phi, mu, gph, gmu, lmu, T(0), j, k, m);
        T fd[19];
#pragma unroll
        for (int i = 0; i < 19; ++i) fd[i] = T(0);
        if constexpr (TRT) collide3_trt<T>(fd, gg, m, dp, k.c);
        else collide3<T>(fd, gg, m, dp, k.c);
        const uint32_t sb = Z.zo[1], vb = q.yo[1] + q.xo[1];
        if constexpr (FixedG<P>::value) {
          // g_0 closes the node's Q2.29 sum at the pulled total
          const int er = (ly + 1) * RC::W + lx + 1;    // the node in the ring region
          int32_t rest = 0;
#pragma unroll
          for (int i = 1; i < 19; ++i) {
            const int32_t word = __float2int_rn(gg[i] * GQ);
            rest += word;
            w.g.stb(i, sb, vb, word);
            if constexpr (PHIQ) {
              // the word streams to (X, Y, zd) + c_i, or back to this node
              // (as the opposite population) beyond a wall
              const int zt = zd + CZ(i);
              if (wl && (zt < 0 || zt >= nz))
                atomicAdd(&L.acc[(zd - vbase) % 3][er], word);
              else
                atomicAdd(&L.acc[(zt - vbase) % 3][er + CY(i) * RC::W + CX(i)], word);
            }
          }
          w.g.stb(0, sb, vb, qs - rest);
          if constexpr (PHIQ) atomicAdd(&L.acc[(zd - vbase) % 3][er], qs - rest);
        } else {
#pragma unroll
          for (int i = 0; i < 19; ++i) w.g.stb(i, sb, vb, gg[i]);
        }
      }
    }
    // stage C's j of this iteration's plane is stage D's in the next
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
      jd[rr][0] = jn[rr][0];
      jd[rr][1] = jn[rr][1];
      jd[rr][2] = jn[rr][2];
    }
    __syncthreads();
    if constexpr (PHIQ) {
      // plane zd - 1 now has the words of all its sources in this tile
      if (zd >= z0 && zd < z1) flush(zd - 1);
    }
  }
  if constexpr (PHIQ) {
    flush(z1 - 1);
    flush(z1);
  }
}

template <int P, int I = 0>
__device__ __forceinline__ void to_canonical_dirs(const Pop3<P>& in, const Node& k, const Geom3& g,
                                                  double* __restrict__ f, double* __restrict__ gg) {
  if constexpr (I < 19) {
    int plane;
    uint32_t e;
    pull_src<I>(k, g, plane, e);
    f[(int64_t)I * g.N + k.n] = double(in.f(plane, e));
    gg[(int64_t)I * g.N + k.n] = in.g_exact(plane, e);   // Q2.29 words exactly
    to_canonical_dirs<P, I + 1>(in, k, g, f, gg);
  }
}

template <int P>
__global__ __launch_bounds__(256) void k3_to_canonical(Pop3<P> in, double* __restrict__ f,
                                                       double* __restrict__ gg, Geom3 g) {
  QILBM3_FOR_NODES(n, g) to_canonical_dirs<P>(in, node_of(n, g), g, f, gg);
}

template <int P>
__global__ __launch_bounds__(256) void k3_from_canonical(const double* __restrict__ f,
                                                         const double* __restrict__ gg,
                                                         Pop3<P> out, Geom3 g) {
  using T = typename PrecT<P>::T;
  QILBM3_FOR_NODES(n, g) {
    const Node nd = node_of(n, g);
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const int zs = nd.z - CZ(i);
      int plane = i;
      uint32_t e;
      if ((zs < 0 || zs >= g.nz) && g.walls) {
        plane = OPP(i);
        e = nd.n;
      } else {
        e = idx3(wrapi(nd.x - CX(i), g.nx), wrapi(nd.y - CY(i), g.ny), wrapi(zs, g.nz), g);
      }
      out.set_f(plane, e, T(f[(int64_t)i * g.N + n]));
      out.set_g_d(plane, e, gg[(int64_t)i * g.N + n]);
    }
  }
}

// Per-block FP64 partials of (sum phi, sum rho, sum rho u) with phi and rho
// from the exact stored g; wave64 shuffles, fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <int P, bool BIG>
__global__ __launch_bounds__(256) void k3_mass_partial(Pop3<P> in,
                                                       const typename PrecT<P>::T* __restrict__ phi,
                                                       const typename PrecT<P>::T* __restrict__ mu,
                                                       double* __restrict__ part,
                                                       Coef3<typename PrecT<P>::T> k,
                                                       double rho_B, double drho, Geom3 g,
                                                       uint32_t nxc) {
  using T = typename PrecT<P>::T;
  const PopView<P, BIG> v(in);
  const Planes<T, false> ph(phi, g.Ns, 1), mf(mu, g.Ns, 1);
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for_rows<sizeof(T)>(g, nxc, [&](const RowCtx& R, const Lane& L) {
    T f[19];
    Node3<T> m;
    node_state_r<P, BIG>(v, ph, mf, R, L, k, f, m);
    double ex = 0.0;   // phi from the stored g, exactly
#pragma unroll
    for (int i = 0; i < 19; ++i) {
      const Src s = pull_at(i, R, L);
      if constexpr (FixedG<P>::value) ex += double(v.g.ld(s.plane, s.row, s.vo)) * GQI_D;
      else ex += v.g.ld(s.plane, s.row, s.vo);
    }
    a[0] += ex;
    a[1] += rho_B + drho * ex;       // binary64 density parameters
    for (int c = 0; c < 3; ++c) a[2 + c] += double(m.rho) * double(m.u[c]);
  });
  __shared__ double red[4][5];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 5; ++c) a[c] = wave_sum(a[c]);
  if (lane == 0)
    for (int c = 0; c < 5; ++c) red[wave][c] = a[c];
  __syncthreads();
  if (threadIdx.x < 5) {
    const int c = threadIdx.x;
    part[5 * blockIdx.x + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  }
}

// Final sum of nb rows of 5 partials by one workgroup, fixed order.
__global__ __launch_bounds__(256) void k3_sum5(const double* __restrict__ part, int nb,
                                               double* __restrict__ out) {
  double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += 256)
#pragma unroll
    for (int c = 0; c < 5; ++c) a[c] += part[5 * b + c];
  __shared__ double red[4][5];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 5; ++c) a[c] = wave_sum(a[c]);
  if (lane == 0)
    for (int c = 0; c < 5; ++c) red[wave][c] = a[c];
  __syncthreads();
  if (threadIdx.x < 5) {
    const int c = threadIdx.x;
    out[c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
  }
}

}  // namespace qilbm3

// ====================================================================== C ABI
using namespace qilbm3;

struct lbm3_ctx {
  lbm3_params prm;
  double beta, kappa, lam, alpha, gamma, drho;
  Geom3 geom;
  hipStream_t stream;
  char* pop[2];
  int cur;
  char* fields;      // phi, mu, p, jx, jy, jz (compute type, 8 bytes a node each)
  double* part;      // 5 per reduction block
  int nred;
  double* red_out;
  int64_t t;
  int resident;      // workgroups of the fused kernel resident at once (0: not yet known)
  int32_t* phiq[2];  // Q2.29 phi of the current state (FP32 fused step), double-buffered
  int qcur;          // phiq[qcur] belongs to pop[cur] when phiq_ok
  bool phiq_ok;
};

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

bool valid3(const lbm3_params* p) {
  if (!p) return false;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return false;
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  if (N > ((int64_t)1 << 29) - 4096) return false;
  const double v[] = {p->rho_A, p->rho_B, p->sigma, p->W, p->M, p->tau_f, p->tau_g,
                      p->gx,    p->gy,    p->gz,    p->rho_ref, p->trt_magic};
  for (double d : v)
    if (!isfinite(d)) return false;
  if (!(p->rho_A > 0.0) || !(p->rho_B > 0.0)) return false;
  if (!(p->sigma > 0.0) || !(p->W > 0.0) || !(p->M > 0.0)) return false;
  if (!(p->tau_f > 0.5) || !(p->tau_g > 0.5)) return false;
  if (p->bc != LBM_BC_PERIODIC && p->bc != 1) return false;
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32) return false;
  if (p->flags & ~(uint32_t)(LBM_FLAG_NO_GAMMA | LBM_FLAG_UNFUSED)) return false;
  if (!(p->trt_magic >= 0.0)) return false;
  return true;
}

Geom3 geom_of(const lbm3_params* p) {
  Geom3 g;
  g.nx = p->nx;
  g.ny = p->ny;
  g.nz = p->nz;
  g.walls = p->bc == 1;
  g.N = (int64_t)p->nx * p->ny * p->nz;
  g.Ns = qilbm::plane_stride(g.N);
  return g;
}

struct Layout3 {
  size_t pop0, pop1, fields, part, red, phiq, total;
  int nred;
};

Layout3 layout3(const lbm3_params* p) {
  const Geom3 g = geom_of(p);
  Layout3 L;
  const size_t pb = up((size_t)pop3_bytes(p->precision, g.Ns));
  L.nred = (int)((g.N + 255) / 256);
  if (L.nred > 2048) L.nred = 2048;
  L.pop0 = 0;
  L.pop1 = pb;
  L.fields = 2 * pb;
  L.part = L.fields + up(6 * (size_t)g.Ns * 8);   // phi, mu, p, j
  L.red = L.part + up((size_t)L.nred * 5 * 8);
  L.phiq = L.red + up(8 * 8);
  L.total = L.phiq + 2 * up((size_t)g.Ns * 4);
  return L;
}

template <typename T>
Coef3<T> coef3(const lbm3_ctx* c) {
  Coef3<T> k;
  k.c.beta4 = T(4.0 * c->beta);
  k.c.kappa = T(c->kappa);
  k.c.lam = T(c->lam);
  k.c.alpha = T(c->alpha);
  k.c.gamma = T(c->gamma);
  k.c.drho = T(c->drho);
  k.c.rho_B = T(c->prm.rho_B);
  k.c.rho_ref = T(c->prm.rho_ref);
  k.c.gx = T(c->prm.gx);
  k.c.gy = T(c->prm.gy);
  k.gz = T(c->prm.gz);
  k.c.inv_tau_f = T(1.0 / c->prm.tau_f);
  k.c.inv_tau_g = T(1.0 / c->prm.tau_g);
  k.c.kf = T(1.0 - 0.5 / c->prm.tau_f);
  k.c.kg = T(1.0 - 0.5 / c->prm.tau_g);
  const double tau_m =
      c->prm.trt_magic > 0.0 ? 0.5 + c->prm.trt_magic / (c->prm.tau_f - 0.5) : c->prm.tau_f;
  k.c.inv_tau_m = T(1.0 / tau_m);
  k.c.km = T(1.0 - 0.5 / tau_m);
  return k;
}

unsigned grid_of(int64_t N) {
  const int64_t b = (N + 255) / 256;
  return (unsigned)(b < 65536 ? b : 65536);
}

// Row-wave launches: ceil(nx / 64) chunks per row, four per workgroup.
uint32_t chunks_x(const Geom3& g) { return (uint32_t)((g.nx + 63) / 64); }

unsigned row_grid(const Geom3& g) {
  const int64_t tasks = (int64_t)row_tasks(g, chunks_x(g));
  const int64_t b = (tasks + 3) / 4;
  return (unsigned)(b < (1 << 24) ? b : (1 << 24));
}

// A population set spans more than 4 GiB - 1 bytes: one descriptor per plane.
template <int P>
bool big3(const Geom3& g) {
  return 19 * g.Ns * (int64_t)sizeof(typename PrecT<P>::T) > (int64_t)UINT32_MAX;
}

lbm_status st(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

template <int P>
hipError_t fields_p(lbm3_ctx* c) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  Pop3<P> in{c->pop[c->cur], g.Ns};
  T* phi = (T*)c->fields;
  T* mu = (T*)(c->fields + g.Ns * 8);
  const uint32_t nxc = chunks_x(g);
  if (big3<P>(g))
    hipLaunchKernelGGL((k3_phi<P, true>), dim3(row_grid(g)), dim3(256), 0, c->stream, in, phi, g,
                       nxc);
  else
    hipLaunchKernelGGL((k3_phi<P, false>), dim3(row_grid(g)), dim3(256), 0, c->stream, in, phi, g,
                       nxc);
  const int64_t mu_blocks = (int64_t)mu_tiles_xy(g) * ((g.nz + MZ_ZS - 1) / MZ_ZS);
  hipLaunchKernelGGL(k3_mu<T>, dim3((unsigned)mu_blocks), dim3(256), 0, c->stream,
                     (const T*)phi, mu, coef3<T>(c), g);
  return hipGetLastError();
}

template <int P, bool BIG>
void launch_macro(lbm3_ctx* c, typename PrecT<P>::T* p, const MomentOut3& mo) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  Pop3<P> in{c->pop[c->cur], g.Ns};
  hipLaunchKernelGGL((k3_macro<P, BIG>), dim3(row_grid(g)), dim3(256), 0, c->stream, in,
                     (const T*)c->fields, (const T*)(c->fields + g.Ns * 8), p, mo, coef3<T>(c), g,
                     chunks_x(g));
}

template <int P, bool BIG>
void launch_collide(lbm3_ctx* c) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  Pop3<P> in{c->pop[c->cur], g.Ns}, out{c->pop[c->cur ^ 1], g.Ns};
  T* phi = (T*)c->fields;
  T* mu = (T*)(c->fields + g.Ns * 8);
  T* p = (T*)(c->fields + 2 * g.Ns * 8);
  T* jx = (T*)(c->fields + 3 * g.Ns * 8);
  T* jy = (T*)(c->fields + 4 * g.Ns * 8);
  T* jz = (T*)(c->fields + 5 * g.Ns * 8);
  if (c->prm.trt_magic > 0.0) {
    hipLaunchKernelGGL((k3_pf<P, BIG, true>), dim3(row_grid(g)), dim3(256), 0, c->stream, in, out,
                       (const T*)phi, (const T*)mu, p, jx, jy, jz, coef3<T>(c), g, chunks_x(g));
    hipLaunchKernelGGL((k3_g<P, BIG, true>), dim3(row_grid(g)), dim3(256), 0, c->stream, in, out,
                       (const T*)phi, (const T*)mu, (const T*)p, (const T*)jx, (const T*)jy,
                       (const T*)jz, coef3<T>(c), g, chunks_x(g));
  } else {
    hipLaunchKernelGGL((k3_pf<P, BIG, false>), dim3(row_grid(g)), dim3(256), 0, c->stream, in,
                       out, (const T*)phi, (const T*)mu, p, jx, jy, jz, coef3<T>(c), g,
                       chunks_x(g));
    hipLaunchKernelGGL((k3_g<P, BIG, false>), dim3(row_grid(g)), dim3(256), 0, c->stream, in,
                       out, (const T*)phi, (const T*)mu, (const T*)p, (const T*)jx,
                       (const T*)jy, (const T*)jz, coef3<T>(c), g, chunks_x(g));
  }
}

// workgroups of the kernel that will run resident on the whole GPU at once
template <int P, bool TRT>
int fused_resident3() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k3_fused<P, false, true, TRT>,
                                                   FzThreads<P>::value, 0) != hipSuccess)
    return 0;
  return cus * (per_cu > 0 ? per_cu : 1);
}

// Tiles of TX x TY columns times z-segments, one round of workgroups.
Fz3Shape fused_shape3(const Geom3& g, int resident) {
  Fz3Shape sh;
  sh.ntx = (g.nx + fz::TX - 1) / fz::TX;
  sh.nty = (g.ny + fz::TY - 1) / fz::TY;
  const int ntiles = sh.ntx * sh.nty;
  int nseg = resident > ntiles ? resident / ntiles : 1;
  if (nseg > g.nz) nseg = g.nz;
  sh.seg = (g.nz + nseg - 1) / nseg;
  sh.nseg = (g.nz + sh.seg - 1) / sh.seg;
  return sh;
}

template <int P>
lbm_status step_fused_p(lbm3_ctx* c, int64_t n) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  if (c->resident == 0)
    c->resident = c->prm.trt_magic > 0.0 ? fused_resident3<P, true>() : fused_resident3<P, false>();
  if (c->resident <= 0) return LBM_EDEVICE;
  const Fz3Shape sh = fused_shape3(g, c->resident);
  const unsigned nblk = (unsigned)(sh.ntx * sh.nty * sh.nseg);
  const Coef3<T> k = coef3<T>(c);
  const bool big = big3<P>(g);
  const bool trt = c->prm.trt_magic > 0.0;
  if (n > 0 && !c->phiq_ok) {
    Pop3<P_F32> in{c->pop[c->cur], g.Ns};
    if (big)
      hipLaunchKernelGGL(k3_phiq<true>, dim3(row_grid(g)), dim3(256), 0, c->stream, in,
                         c->phiq[c->qcur], g, chunks_x(g));
    else
      hipLaunchKernelGGL(k3_phiq<false>, dim3(row_grid(g)), dim3(256), 0, c->stream, in,
                         c->phiq[c->qcur], g, chunks_x(g));
    if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
    c->phiq_ok = true;
  }
  for (int64_t s = 0; s < n; ++s) {
    Pop3<P> in{c->pop[c->cur], g.Ns}, out{c->pop[c->cur ^ 1], g.Ns};
    int32_t* qin = c->phiq[c->qcur];
    int32_t* qout = c->phiq[c->qcur ^ 1];
    if (qilbm::launch_zero(qout, (size_t)g.Ns * 4, c->stream) != hipSuccess) return LBM_EDEVICE;
    const dim3 grid(nblk), block(FzThreads<P>::value);
    if (big && trt)
      hipLaunchKernelGGL((k3_fused<P, true, true, true>), grid, block, 0, c->stream, in, out, k,
                         g, sh, (const int32_t*)qin, qout);
    else if (big)
      hipLaunchKernelGGL((k3_fused<P, true, true, false>), grid, block, 0, c->stream, in, out, k,
                         g, sh, (const int32_t*)qin, qout);
    else if (trt)
      hipLaunchKernelGGL((k3_fused<P, false, true, true>), grid, block, 0, c->stream, in, out, k,
                         g, sh, (const int32_t*)qin, qout);
    else
      hipLaunchKernelGGL((k3_fused<P, false, true, false>), grid, block, 0, c->stream, in, out, k,
                         g, sh, (const int32_t*)qin, qout);
    if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
    c->cur ^= 1;
    c->qcur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

template <int P>
lbm_status step_p(lbm3_ctx* c, int64_t n) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  if constexpr (P == P_F32)
    if (!(c->prm.flags & LBM_FLAG_UNFUSED)) return step_fused_p<P>(c, n);
  c->phiq_ok = false;
  const bool big = big3<P>(g);
  for (int64_t s = 0; s < n; ++s) {
    if (fields_p<P>(c) != hipSuccess) return LBM_EDEVICE;
    if (big)
      launch_collide<P, true>(c);
    else
      launch_collide<P, false>(c);
    if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
    c->cur ^= 1;
    c->t += 1;
  }
  return LBM_OK;
}

template <int P>
lbm_status moments_p(lbm3_ctx* c, const MomentOut3& mo) {
  if (fields_p<P>(c) != hipSuccess) return LBM_EDEVICE;
  if (big3<P>(c->geom))
    launch_macro<P, true>(c, nullptr, mo);
  else
    launch_macro<P, false>(c, nullptr, mo);
  return st(hipGetLastError());
}

template <int P>
lbm_status mass_p(lbm3_ctx* c) {
  using T = typename PrecT<P>::T;
  const Geom3& g = c->geom;
  if (fields_p<P>(c) != hipSuccess) return LBM_EDEVICE;
  Pop3<P> in{c->pop[c->cur], g.Ns};
  const T* phi = (const T*)c->fields;
  const T* mu = (const T*)(c->fields + g.Ns * 8);
  const Coef3<double> k64 = coef3<double>(c);
  if (big3<P>(g))
    hipLaunchKernelGGL((k3_mass_partial<P, true>), dim3(c->nred), dim3(256), 0, c->stream, in,
                       phi, mu, c->part, coef3<T>(c), k64.c.rho_B, k64.c.drho, g, chunks_x(g));
  else
    hipLaunchKernelGGL((k3_mass_partial<P, false>), dim3(c->nred), dim3(256), 0, c->stream, in,
                       phi, mu, c->part, coef3<T>(c), k64.c.rho_B, k64.c.drho, g, chunks_x(g));
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  hipLaunchKernelGGL(k3_sum5, dim3(1), dim3(256), 0, c->stream, (const double*)c->part, c->nred,
                     c->red_out);
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  return LBM_OK;
}

#define QILBM3_DISPATCH(prec, FN, ...) \
  ((prec) == LBM_FP64 ? FN<P_F64>(__VA_ARGS__) : FN<P_F32>(__VA_ARGS__))

}  // namespace

extern "C" {

size_t lbm3_workspace_bytes(const lbm3_params* params) {
  if (!valid3(params)) return 0;
  return layout3(params).total;
}

lbm_status lbm3_init(lbm3_ctx** out, const lbm3_params* params, void* ws, size_t bytes,
                     const double* phi0, void* stream) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if (!valid3(params) || !ws || !phi0) return LBM_EINVAL;
  if ((uintptr_t)ws % ALIGN != 0) return LBM_EINVAL;
  const Layout3 L = layout3(params);
  if (bytes < L.total) return LBM_ENOMEM;
  lbm3_ctx* c = new (std::nothrow) lbm3_ctx();
  if (!c) return LBM_ENOMEM;
  c->prm = *params;
  // Sec. II-III with phi_A = 1, phi_B = 0 (as for the two-dimensional step)
  c->beta = 12.0 * params->sigma / params->W;
  c->kappa = 1.5 * params->sigma * params->W;
  c->lam = params->M;
  c->alpha = params->M / ((params->tau_g - 0.5) / 3.0);
  c->gamma = (params->flags & LBM_FLAG_NO_GAMMA) ? 0.0 : params->rho_A / params->rho_B - 1.0;
  c->drho = params->rho_A - params->rho_B;
  c->geom = geom_of(params);
  c->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  c->pop[0] = base + L.pop0;
  c->pop[1] = base + L.pop1;
  c->cur = 0;
  c->fields = base + L.fields;
  c->part = (double*)(base + L.part);
  c->nred = L.nred;
  c->red_out = (double*)(base + L.red);
  c->t = 0;
  c->resident = 0;
  c->phiq[0] = (int32_t*)(base + L.phiq);
  c->phiq[1] = (int32_t*)(base + L.phiq + up((size_t)c->geom.Ns * 4));
  c->qcur = 0;
  c->phiq_ok = false;
  hipError_t e = qilbm::launch_zero(base, L.fields, c->stream);
  if (e == hipSuccess) {
    const Coef3<double> k = coef3<double>(c);
    if (params->precision == LBM_FP64)
      hipLaunchKernelGGL(k3_init<P_F64>, dim3(grid_of(c->geom.N)), dim3(256), 0, c->stream,
                         phi0, Pop3<P_F64>{c->pop[0], c->geom.Ns}, k, c->geom);
    else
      hipLaunchKernelGGL(k3_init<P_F32>, dim3(grid_of(c->geom.N)), dim3(256), 0, c->stream,
                         phi0, Pop3<P_F32>{c->pop[0], c->geom.Ns}, k, c->geom);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    delete c;
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm3_step(lbm3_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  return QILBM3_DISPATCH(c->prm.precision, step_p, c, nsteps);
}

lbm_status lbm3_moments(lbm3_ctx* c, double* phi, double* rho, double* ux, double* uy,
                        double* uz, double* p, double* mu) {
  if (!c) return LBM_EINVAL;
  MomentOut3 mo;
  mo.phi = phi;
  mo.rho = rho;
  mo.u[0] = ux;
  mo.u[1] = uy;
  mo.u[2] = uz;
  mo.p = p;
  mo.mu = mu;
  return QILBM3_DISPATCH(c->prm.precision, moments_p, c, mo);
}

lbm_status lbm3_mass(lbm3_ctx* c, double out[5]) {
  if (!c || !out) return LBM_EINVAL;
  lbm_status s = QILBM3_DISPATCH(c->prm.precision, mass_p, c);
  if (s != LBM_OK) return s;
  double tot[5];
  if (hipMemcpyAsync(tot, c->red_out, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream) !=
      hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return LBM_EDEVICE;
  for (int k = 0; k < 5; ++k) out[k] = tot[k];
  for (int k = 0; k < 5; ++k)
    if (!isfinite(out[k])) return LBM_EDIVERGED;
  return LBM_OK;
}

lbm_status lbm3_get_state(lbm3_ctx* c, double* f, double* g) {
  if (!c || !f || !g) return LBM_EINVAL;
  const Geom3& gm = c->geom;
  if (c->prm.precision == LBM_FP64)
    hipLaunchKernelGGL(k3_to_canonical<P_F64>, dim3(grid_of(gm.N)), dim3(256), 0, c->stream,
                       Pop3<P_F64>{c->pop[c->cur], gm.Ns}, f, g, gm);
  else
    hipLaunchKernelGGL(k3_to_canonical<P_F32>, dim3(grid_of(gm.N)), dim3(256), 0, c->stream,
                       Pop3<P_F32>{c->pop[c->cur], gm.Ns}, f, g, gm);
  return st(hipGetLastError());
}

lbm_status lbm3_set_state(lbm3_ctx* c, const double* f, const double* g) {
  if (!c || !f || !g) return LBM_EINVAL;
  const Geom3& gm = c->geom;
  c->phiq_ok = false;
  if (c->prm.precision == LBM_FP64)
    hipLaunchKernelGGL(k3_from_canonical<P_F64>, dim3(grid_of(gm.N)), dim3(256), 0, c->stream,
                       f, g, Pop3<P_F64>{c->pop[c->cur], gm.Ns}, gm);
  else
    hipLaunchKernelGGL(k3_from_canonical<P_F32>, dim3(grid_of(gm.N)), dim3(256), 0, c->stream,
                       f, g, Pop3<P_F32>{c->pop[c->cur], gm.Ns}, gm);
  return st(hipGetLastError());
}

int64_t lbm3_time(const lbm3_ctx* c) { return c ? c->t : -1; }

void lbm3_destroy(lbm3_ctx* c) { delete c; }

}  // extern "C"
