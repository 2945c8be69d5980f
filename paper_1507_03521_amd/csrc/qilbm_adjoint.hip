// Adjoint of one coupled step of the quasi-incompressible phase-field LBE
// (reverse mode; not part of the paper, which defines only the forward
// scheme of Sec. III). Each kernel is the transpose of one forward stage,
// taken in reverse order:
//
//   forward                                  adjoint
//   phi, S, j  <- populations                 gbar_i += phibar, fbar_i += Sbar + c_i.jbar
//   mu <- phi (bulk + lap)                    phibar += mubar bulk'(phi) + lap^T(-kappa mubar)
//   grad rho, grad mu, D <- stencils          grad^T, lap^T of their cotangents
//   F, u, p <- node values                    node-local transposes
//   grad p <- p                               pbar += grad^T(gradp_bar)
//   collision (BGK + F_i, G_i)                node-local Jacobian transpose
//   streaming (pull, bounce-back)             gather from the neighbour it fed
//
// The default adjoint step is one fused kernel (k_adj_fused, below) that
// sweeps the rows and applies these transposes in a pipeline; the three
// separate kernels remain for LBM_FLAG_UNFUSED (cross-checks).
//
// The adjoint populations are kept in the canonical pre-collision layout
// ([18][ny][nx], compute type). The forward step at t enters only through
// its record: phi, mu, p, S = sum f, jx, jy of the state s_t (planes of the
// compute type), written by the forward kernel itself (lbm_step_record) or
// recomputed here from a raw state. The direct (diagonal) part of the
// collision transpose, (1 - 1/tau) times the post-collision cotangent, is
// recomputed where it is added rather than stored. Cotangents of beta, kappa, lambda,
// alpha are summed in FP64 in a fixed block order (run-to-run reproducible)
// and turned into dL/dsigma and dL/dM at the end (beta, kappa are
// proportional to sigma at fixed W; lambda = M and alpha = M/(c_s^2 (tau_g - 1/2))).
#include <math.h>

#include "../../include/qilbm.h"
#include "qilbm_adjoint.hpp"
#include "qilbm_internal.hpp"

namespace qilbm {

namespace {

constexpr size_t ALIGN = 256;
inline size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

template <typename T>
struct AF {
  T* base;
  int64_t Ns;
  __device__ __forceinline__ T* operator[](int k) const { return base + (int64_t)k * Ns; }
};

// ------------------------------------------------------- node indexing
// Element offsets around node (x, y), all 32-bit (N < 2^29):
//   rs: rows y-1, y, y+1 as the forward stencils see them (periodic wrap or
//       the mirrored ghost row at a wall),
//   rt: the same rows for gathers, -1 where the row lies beyond a wall,
//   cl: columns x-1, x, x+1 (periodic).
struct NodeIdx {
  int n, x, y;
  int rs[3], rt[3], cl[3];
  bool lo, hi;   // bottom / top wall row
};

__device__ __forceinline__ NodeIdx node_idx(int n, const Geom& g) {
  NodeIdx k;
  k.n = n;
  k.y = (int)((unsigned)n / (unsigned)g.nx);
  k.x = n - k.y * g.nx;
  k.lo = g.walls && k.y == 0;
  k.hi = g.walls && k.y == g.ny - 1;
#pragma unroll
  for (int d = -1; d <= 1; ++d) {
    const int yy = k.y + d;
    const bool out = yy < 0 || yy >= g.ny;
    k.rs[d + 1] = nbr_row(yy, g) * g.nx;
    k.rt[d + 1] = (out && g.walls) ? -1 : k.rs[d + 1];
    k.cl[d + 1] = wrap_x(k.x + d, g.nx);
  }
  return k;
}

// 3x3 neighbourhood of a field as the forward stencils see it.
template <typename T>
__device__ __forceinline__ void load3x3(const T* psi, const NodeIdx& k, T v[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) v[a][b] = psi[k.rs[a] + k.cl[b]];
}

// ------------------------------------------------ transposed stencils
// grad psi(y) = 3 sum_i w_i c_i psi(nb(y, c_i)) and
// lap psi(y) = 6 sum_i w_i (psi(nb(y, c_i)) - psi(y)), with nb the periodic
// or mirrored neighbour. Their transposes, evaluated as gathers: node x
// collects from every (y, i) with nb(y, c_i) = x. Off the walls that is
// y = x - c_i; on a wall row the mirrored ghost adds y = x - (c_ix, 0) for
// the directions pointing into the wall.
template <typename T, bool GR, bool LP, int I>
__device__ __forceinline__ void gt_term(const T* vx, const T* vy, const T* ws, const NodeIdx& k,
                                        T& gacc, T& lacc) {
  constexpr int cx = CXS(I), cy = CYS(I);
  const T w3 = T(3.0 * WGT(I)), w6 = T(6.0 * WGT(I));
  const int r = k.rt[1 - cy];
  if (r >= 0) {
    const int m = r + k.cl[1 - cx];
    if constexpr (GR) gacc += w3 * cdot<cx, cy>(vx[m], vy[m]);
    if constexpr (LP) lacc += w6 * ws[m];
  }
  if ((cy == -1 && k.lo) || (cy == 1 && k.hi)) {
    const int m = k.rs[1] + k.cl[1 - cx];
    if constexpr (GR) gacc += w3 * cdot<cx, cy>(vx[m], vy[m]);
    if constexpr (LP) lacc += w6 * ws[m];
  }
}

// Returns grad^T(vx, vy)(x) (if GR) + lap^T(ws)(x) (if LP).
template <typename T, bool GR, bool LP>
__device__ __forceinline__ T stencil_T(const T* vx, const T* vy, const T* ws, const NodeIdx& k) {
  T gacc = T(0), lacc = T(0);
  gt_term<T, GR, LP, 1>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 2>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 3>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 4>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 5>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 6>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 7>(vx, vy, ws, k, gacc, lacc);
  gt_term<T, GR, LP, 8>(vx, vy, ws, k, gacc, lacc);
  if constexpr (LP) lacc -= T(10.0 / 3.0) * ws[k.n];
  return gacc + lacc;
}

// ----------------------------------------------- block partial accumulation
// Each block adds its FP64 partial to its own slot: the order of additions
// is fixed by the launch shape, so the totals are reproducible.
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ __forceinline__ void block_add(double v, int slot, double* acc_part) {
  __shared__ double red[4];     // one per wavefront of a workgroup of 64 to 256 lanes
  v = wsum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    double s = nw > 1 ? red[0] + red[1] : red[0];
    if (nw > 2) s += nw > 3 ? red[2] + red[3] : red[2];
    acc_part[4 * blockIdx.x + slot] += s;
  }
  __syncthreads();
}

// ----------------------------------------------------------------- kernels
__global__ __launch_bounds__(256) void k_fill_zero(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = 0.0;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_seed(const double* __restrict__ dphi, T* __restrict__ hat,
                                                  Geom g) {
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N;
       n += (int64_t)gridDim.x * 256) {
    const T v = T(dphi[n]);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      hat[(int64_t)i * g.Ns + n] = T(0);
      hat[(int64_t)(9 + i) * g.Ns + n] = v;
    }
  }
}

// Cotangent of the post-collision population i at x: the pre-collision
// population it becomes at t+1 is i at x + c_i, or opp(i) at x itself when
// x + c_i lies beyond a wall.
template <typename T, int I>
__device__ __forceinline__ T post_hat(const T* hat, int koff, const NodeIdx& k, int64_t Ns) {
  constexpr int cx = CXS(I), cy = CYS(I);
  const int r = k.rt[1 + cy];
  if (r < 0) return hat[(int64_t)(koff + OPP(I)) * Ns + k.n];
  return hat[(int64_t)(koff + I) * Ns + (r + k.cl[1 + cx])];
}

template <typename T, int I = 0>
__device__ __forceinline__ void post_hat9(const T* hat, int koff, const NodeIdx& k, int64_t Ns,
                                          T v[9]) {
  if constexpr (I < 9) {
    v[I] = post_hat<T, I>(hat, koff, k, Ns);
    post_hat9<T, I + 1>(hat, koff, k, Ns, v);
  }
}

// The f cotangents of the pre-collision state: the direct part fd_i plus the
// moment transposes Sbar + c_i.jbar, handed to store(i, value).
template <int I = 0, typename T, typename St>
__device__ __forceinline__ void fbar_out(const St& store, const T fd[9], T bS, T bjx, T bjy) {
  if constexpr (I < 9) {
    T v = fd[I] + bS;
    if constexpr (I != 0) v += cdot<CXS(I), CYS(I)>(bjx, bjy);
    store(I, v);
    fbar_out<I + 1>(store, fd, bS, bjx, bjy);
  }
}

// Transpose of collide_node at one node. Inputs: forward node state m,
// grad p, the populations' post-collision cotangents fh, gh. Outputs: the
// direct cotangents of the pre-collision populations (in fh, gh) and the
// cotangents of the node quantities the collision read.
template <typename T>
struct NodeBar {
  T p, rho, ux, uy, Fx, Fy, drx, dry, D, phi, mu, dpx, dpy, alpha;
};

// The collision in the form the forward kernels evaluate it (per node:
// u.F, u.(grad rho / 3), u.(grad p - F); per direction: s, A = (c-u).F,
// B = (c-u).grad rho / 3, Q = (c-u).(grad p - F), X = A + s (A + B),
// Y = Q + s Q;
//   f* = (1 - 1/tau_f) f + (1/tau_f) w (p + rho s / 3) + kf w (X + src1),
//   g* = (1 - 1/tau_g) g + (1/tau_g) (H + w phi s) + kg w K Y,
// src1 = -rho gamma D / 3, K = -3 phi / rho), transposed. With the weighted
// cotangents a = w fbar*, b = w gbar*:
//   sbar = a (rho/(3 tau_f) + kf (A + B)) + b (phi/tau_g + kg K Q),
//   Abar = kf a (1 + s), Bbar = kf a s, Qbar = kg K b (1 + s),
//   (c.u)bar = sbar (3 + 9 c.u), (1.5 u^2)bar = -sbar,
// and Abar, Bbar, Qbar go to F, grad rho, grad p - F through c - u. The
// sums over directions are carried per node and turned into the node
// cotangents once.
template <int I = 0, typename T>
__device__ __forceinline__ void coll_T_dirs(T fh[9], T gh[9], const CollNode<T>& n, T rp, T pp,
                                            T Kk, T kf, T af, T ag, T (&acc)[17]) {
  if constexpr (I < 9) {
    const T w = T(WGT(I));
    const T a = w * fh[I], b = w * gh[I];
    fh[I] = af * fh[I];
    gh[I] = ag * gh[I];
    T s, cu, A, B, Q;
    if constexpr (I == 0) {
      s = -n.usq15;
      cu = T(0);
      A = -n.uF;
      B = -n.ud;
      Q = -n.uq;
    } else {
      constexpr int cx = CXS(I), cy = CYS(I);
      cu = cdot<cx, cy>(n.ux, n.uy);
      s = fmad(cu, fmad(T(4.5), cu, T(3)), -n.usq15);
      A = cdot<cx, cy>(n.Fx, n.Fy) - n.uF;
      B = cdot<cx, cy>(n.dx, n.dy) - n.ud;
      Q = cdot<cx, cy>(n.qx, n.qy) - n.uq;
    }
    const T sbar = fmad(a, fmad(kf, A + B, rp), b * fmad(Kk, Q, pp));
    acc[0] += a;                       // sum a
    acc[1] = fmad(s, a, acc[1]);       // sum s a
    acc[2] = fmad(s, b, acc[2]);       // sum s b
    if constexpr (I != 0) acc[3] += b; // sum over i > 0 of b
    acc[4] = fmad(fmad(s, Q, Q), b, acc[4]);   // sum Y b
    const T Au = fmad(s, a, a), Bu = s * a, Qu = fmad(s, b, b);
    acc[5] += Au;
    acc[8] += Bu;
    acc[11] += Qu;
    if constexpr (I != 0) {
      constexpr int cx = CXS(I), cy = CYS(I);
      if constexpr (cx != 0) {
        acc[6] = cx > 0 ? acc[6] + Au : acc[6] - Au;
        acc[9] = cx > 0 ? acc[9] + Bu : acc[9] - Bu;
        acc[12] = cx > 0 ? acc[12] + Qu : acc[12] - Qu;
      }
      if constexpr (cy != 0) {
        acc[7] = cy > 0 ? acc[7] + Au : acc[7] - Au;
        acc[10] = cy > 0 ? acc[10] + Bu : acc[10] - Bu;
        acc[13] = cy > 0 ? acc[13] + Qu : acc[13] - Qu;
      }
      const T cbar = sbar * fmad(T(9), cu, T(3));
      if constexpr (cx != 0) acc[14] = cx > 0 ? acc[14] + cbar : acc[14] - cbar;
      if constexpr (cy != 0) acc[15] = cy > 0 ? acc[15] + cbar : acc[15] - cbar;
    }
    acc[16] += sbar;
    coll_T_dirs<I + 1>(fh, gh, n, rp, pp, Kk, kf, af, ag, acc);
  }
}

template <typename T>
__device__ __forceinline__ void collide_node_T(T fh[9], T gh[9], const Macro<T>& m, T dpx, T dpy,
                                               const Coef<T>& c, NodeBar<T>& nb) {
  const CollNode<T> n = coll_node(m, dpx, dpy);
  const T itf = c.inv_tau_f, itg = c.inv_tau_g;
  const T rinv = recip(m.rho);
  const T K = -T(3) * m.phi * rinv;
  const T Kk = K * c.kg;
  const T rp = m.rho * (itf * T(1.0 / 3.0));
  const T pp = m.phi * itg;
  const T b0 = gh[0];
  T acc[17];
#pragma unroll
  for (int j = 0; j < 17; ++j) acc[j] = T(0);
  coll_T_dirs(fh, gh, n, rp, pp, Kk, c.kf, T(1) - itf, T(1) - itg, acc);
  const T src1_bar = c.kf * acc[0];
  const T K_bar = c.kg * acc[4];
  // A, B, Q cotangents through c - u
  const T uF_bar = -c.kf * acc[5], ud_bar = -c.kf * acc[8], uq_bar = -Kk * acc[11];
  const T qx_bar = fmad(uq_bar, n.ux, Kk * acc[12]);
  const T qy_bar = fmad(uq_bar, n.uy, Kk * acc[13]);
  const T dx_bar = fmad(ud_bar, n.ux, c.kf * acc[9]);
  const T dy_bar = fmad(ud_bar, n.uy, c.kf * acc[10]);
  const T usq_bar = -acc[16];     // cotangent of 1.5 |u|^2
  nb.p = itf * acc[0];
  nb.rho = fmad(itf * T(1.0 / 3.0), acc[1],
                fmad(src1_bar, -c.gamma * m.D * T(1.0 / 3.0), K_bar * (T(3) * m.phi) * rinv * rinv));
  nb.D = -src1_bar * m.rho * c.gamma * T(1.0 / 3.0);
  nb.drx = dx_bar * T(1.0 / 3.0);
  nb.dry = dy_bar * T(1.0 / 3.0);
  // H_0 = phi - (1 - w_0) alpha mu, H_i = w_i alpha mu: (alpha mu)bar
  const T amu_bar = itg * fmad(-T(1.0 - 4.0 / 9.0), b0, acc[3]);
  nb.mu = c.alpha * amu_bar;
  nb.alpha = m.mu * amu_bar;
  nb.phi = fmad(itg, acc[2] + b0, -T(3) * K_bar * rinv);
  nb.dpx = qx_bar;
  nb.dpy = qy_bar;
  nb.Fx = fmad(uF_bar, n.ux, c.kf * acc[6]) - qx_bar;
  nb.Fy = fmad(uF_bar, n.uy, c.kf * acc[7]) - qy_bar;
  nb.ux = fmad(T(3) * n.ux, usq_bar,
               fmad(uq_bar, n.qx, fmad(ud_bar, n.dx, fmad(uF_bar, n.Fx, acc[14]))));
  nb.uy = fmad(T(3) * n.uy, usq_bar,
               fmad(uq_bar, n.qy, fmad(ud_bar, n.dy, fmad(uF_bar, n.Fy, acc[15]))));
}

// Forward node state from the record of step t (same arithmetic as the
// forward kernels). Record planes: 0 phi, 1 mu, 2 p, 3 S, 4 jx, 5 jy.
enum RecPlane : int { R_PHI = 0, R_MU, R_P, R_S, R_JX, R_JY, R_NPLANES };

template <typename T>
__device__ __forceinline__ void fwd_node(const T* rec, const NodeIdx& k, const Coef<T>& c,
                                         const Geom& g, Macro<T>& m, T& S, T& jx, T& jy,
                                         T& gmux, T& gmuy, T& lapmu) {
  S = rec[(int64_t)R_S * g.Ns + k.n];
  jx = rec[(int64_t)R_JX * g.Ns + k.n];
  jy = rec[(int64_t)R_JY * g.Ns + k.n];
  T v[3][3], gphx, gphy, lapphi;
  load3x3(rec + (int64_t)R_PHI * g.Ns, k, v);
  stencil(v, gphx, gphy, lapphi);
  const T ph = v[1][1];
  load3x3(rec + (int64_t)R_MU * g.Ns, k, v);
  stencil(v, gmux, gmuy, lapmu);
  macro_node(ph, v[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, c, m);
}

// AK1+2: collision transpose, then the transposes of grad p (gathered), the
// pressure, velocity, force, D, grad rho and rho definitions, fused. A block
// owns tiles of TX x 8 nodes; the collision transpose runs on the
// tile and a one-node ring around it (the ring only for its grad p
// cotangent, which the gather of the tile's nodes needs), keeping that
// cotangent in LDS and each interior node's other cotangents in registers
// of the thread that owns the node in both phases.
// Tile width: 32 columns (one interior node per thread) for FP32, whose
// register use then allows 3 waves per SIMD (measured 3 % faster than 64);
// 64 (two per thread) for FP64 (9 % faster than 32).
template <typename T> struct CmTile {
  static constexpr int TX = sizeof(T) == 8 ? 64 : 32, TY = 8;
  static constexpr int HX = TX + 2, HY = TY + 2;
  static constexpr int NI = TX * TY;            // interior nodes
  static constexpr int NPT = NI / 256;          // interior nodes per thread
  static constexpr int NH = HX * HY - NI;       // ring nodes
  static_assert(NI % 256 == 0 && NH <= 256, "whole interior nodes and one ring node per thread");
};

template <typename T>
struct CmLds {
  T dpx[CmTile<T>::HY][CmTile<T>::HX];
  T dpy[CmTile<T>::HY][CmTile<T>::HX];
};

// local position of ring node h: the full bottom and top rows, then the
// left and right columns of the interior rows
template <int HX, int HY>
__device__ __forceinline__ void ring_pos(int h, int& ly, int& lx) {
  if (h < HX) {
    ly = 0;
    lx = h;
  } else if (h < 2 * HX) {
    ly = HY - 1;
    lx = h - HX;
  } else {
    h -= 2 * HX;
    ly = 1 + (h >> 1);
    lx = (h & 1) ? HX - 1 : 0;
  }
}

// Node of local position (ly, lx) in the tile at (x0, y0): wrapped in x
// (and in y when periodic); false beyond a wall.
__device__ __forceinline__ bool cm_node(int x0, int y0, int ly, int lx, const Geom& g, int& n) {
  int y = y0 - 1 + ly, x = x0 - 1 + lx;
  if (g.walls) {
    if (y < 0 || y >= g.ny) return false;
  } else {
    y %= g.ny;
    if (y < 0) y += g.ny;
  }
  x %= g.nx;
  if (x < 0) x += g.nx;
  n = y * g.nx + x;
  return true;
}

// Collision transpose at node n; fd receives the direct part of the f
// cotangents, (1 - 1/tau_f) times the post-collision ones.
template <typename T>
__device__ __forceinline__ void collide_T_at(const T* rec, const T* hat, int n, const Coef<T>& c,
                                             const Geom& g, NodeBar<T>& nb, T fd[9]) {
  const NodeIdx k = node_idx(n, g);
  T S, jx, jy, gmux, gmuy, lapmu;
  Macro<T> m;
  fwd_node<T>(rec, k, c, g, m, S, jx, jy, gmux, gmuy, lapmu);
  T v[3][3], dpx, dpy, lapp;
  load3x3(rec + (int64_t)R_P * g.Ns, k, v);
  stencil(v, dpx, dpy, lapp);
  T gh[9];
  post_hat9<T>(hat, 0, k, g.Ns, fd);
  post_hat9<T>(hat, 9, k, g.Ns, gh);
  collide_node_T(fd, gh, m, dpx, dpy, c, nb);
}

// The grad p cotangent of node n alone: the only output of the collision
// transpose a ring node contributes. It comes from the G_i terms only, so
// the f cotangents and grad p itself are not needed; same operations, same
// order as in collide_node_T.
template <typename T>
__device__ __forceinline__ void gradp_cot_at(const T* rec, const T* hat, int n, const Coef<T>& c,
                                             const Geom& g, T& bx, T& by) {
  const NodeIdx k = node_idx(n, g);
  T S, jx, jy, gmux, gmuy, lapmu;
  Macro<T> m;
  fwd_node<T>(rec, k, c, g, m, S, jx, jy, gmux, gmuy, lapmu);
  T gh[9];
  post_hat9<T>(hat, 9, k, g.Ns, gh);
  T fh[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) fh[i] = T(0);
  // grad p enters the collision only through Q = (c-u).(grad p - F), and
  // its cotangent (c-u) Qbar does not depend on grad p itself: the grad p
  // cotangent of collide_node_T, computed here with zero f cotangents and
  // without grad p (whose value reaches only outputs not used)
  NodeBar<T> nb;
  collide_node_T(fh, gh, m, T(0), T(0), c, nb);
  bx = nb.dpx;
  by = nb.dpy;
}

// grad^T of the grad p cotangent at interior position (ly, lx), global row
// y, from the tile in LDS (same terms, same order as stencil_T).
template <typename T, int I>
__device__ __forceinline__ void gpT_term(const CmLds<T>& L, int ly, int lx, int y, const Geom& g,
                                         T& acc) {
  constexpr int cx = CXS(I), cy = CYS(I);
  const T w3 = T(3.0 * WGT(I));
  const int ys = y - cy;
  if (!g.walls || (ys >= 0 && ys < g.ny))
    acc += w3 * cdot<cx, cy>(L.dpx[ly - cy][lx - cx], L.dpy[ly - cy][lx - cx]);
  if (g.walls && ((cy == -1 && y == 0) || (cy == 1 && y == g.ny - 1)))
    acc += w3 * cdot<cx, cy>(L.dpx[ly][lx - cx], L.dpy[ly][lx - cx]);
}

template <typename T>
__device__ __forceinline__ T gradT_p(const CmLds<T>& L, int ly, int lx, int y, const Geom& g) {
  T acc = T(0);
  gpT_term<T, 1>(L, ly, lx, y, g, acc);
  gpT_term<T, 2>(L, ly, lx, y, g, acc);
  gpT_term<T, 3>(L, ly, lx, y, g, acc);
  gpT_term<T, 4>(L, ly, lx, y, g, acc);
  gpT_term<T, 5>(L, ly, lx, y, g, acc);
  gpT_term<T, 6>(L, ly, lx, y, g, acc);
  gpT_term<T, 7>(L, ly, lx, y, g, acc);
  gpT_term<T, 8>(L, ly, lx, y, g, acc);
  return acc;
}

// Transposes of the pressure, velocity, force, D, grad rho and rho
// definitions at node n given the full pressure cotangent b_p; then the
// node's f cotangents are complete: fd_i + Sbar + c_i.jbar into hat_out.
template <typename T>
__device__ __forceinline__ double macro_T_at(const T* rec, int n, const NodeBar<T>& nb, T b_p,
                                             const T fd[9], T* hat_out, AF<T> af,
                                             const Coef<T>& c, const Geom& g) {
  const NodeIdx k = node_idx(n, g);
  T S, jx, jy, gmux, gmuy, lapmu;
  Macro<T> m;
  fwd_node<T>(rec, k, c, g, m, S, jx, jy, gmux, gmuy, lapmu);
  T b_rho = nb.rho, b_ux = nb.ux, b_uy = nb.uy;
  T b_Fx = nb.Fx, b_Fy = nb.Fy, b_drx = nb.drx, b_dry = nb.dry;
  T b_D = nb.D, b_phi = nb.phi;
  // p = S + (ux drx + uy dry - gamma rho D) / 6
  const T b_S = b_p;
  b_ux += b_p * m.drx * T(1.0 / 6.0);
  b_uy += b_p * m.dry * T(1.0 / 6.0);
  b_drx += b_p * m.ux * T(1.0 / 6.0);
  b_dry += b_p * m.uy * T(1.0 / 6.0);
  b_rho -= b_p * c.gamma * m.D * T(1.0 / 6.0);
  b_D -= b_p * c.gamma * m.rho * T(1.0 / 6.0);
  // u = (j + F / 6) * inv, inv = 3 / rho
  const T inv = T(3) / m.rho;
  const T b_jx = b_ux * inv, b_jy = b_uy * inv;
  b_Fx += b_ux * inv * T(1.0 / 6.0);
  b_Fy += b_uy * inv * T(1.0 / 6.0);
  const T b_inv = b_ux * (jx + m.Fx * T(1.0 / 6.0)) + b_uy * (jy + m.Fy * T(1.0 / 6.0));
  b_rho -= b_inv * inv / m.rho;
  // F = -phi grad mu + (rho - rho_ref) g
  b_phi -= b_Fx * gmux + b_Fy * gmuy;
  const T b_gmux = -m.phi * b_Fx, b_gmuy = -m.phi * b_Fy;
  b_rho += b_Fx * c.gx + b_Fy * c.gy;
  // D = lambda lap mu; grad rho = drho grad phi; rho = rho_B + drho phi
  fbar_out(
      [&](int i, T v) { hat_out[(int64_t)i * g.Ns + n] = v; }, fd, b_S, b_jx, b_jy);
  af[A_GMUX][n] = b_gmux;
  af[A_GMUY][n] = b_gmuy;
  af[A_LMU][n] = c.lam * b_D;
  af[A_GPHX][n] = c.drho * b_drx;
  af[A_GPHY][n] = c.drho * b_dry;
  af[A_PHI2][n] = b_phi + c.drho * b_rho;
  af[A_MU1][n] = nb.mu;
  return double(b_D) * double(lapmu);   // lambda cotangent of this node
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj_cm(const T* __restrict__ rec,
                                                const T* __restrict__ hat, T* __restrict__ hat_out,
                                                AF<T> af, double* acc_part, Coef<T> c, Geom g) {
  using K = CmTile<T>;
  __shared__ CmLds<T> L;
  const int tx = (g.nx + K::TX - 1) / K::TX, ty = (g.ny + K::TY - 1) / K::TY;
  const int t = threadIdx.x;
  double alpha_acc = 0.0, lam_acc = 0.0;
  for (int tile = blockIdx.x; tile < tx * ty; tile += gridDim.x) {
    const int y0 = (tile / tx) * K::TY, x0 = (tile % tx) * K::TX;
    // phase 1: collision transpose on the interior nodes of this thread
    // (kept) and on at most one ring node (grad p cotangent only)
    NodeBar<T> nb[K::NPT];
    T fd[K::NPT][9];
    int own[K::NPT];
#pragma unroll
    for (int q = 0; q < K::NPT; ++q) {
      const int i = t + 256 * q;
      const int ly = 1 + i / K::TX, lx = 1 + i % K::TX;
      int n = -1;
      own[q] = -1;
      if (cm_node(x0, y0, ly, lx, g, n)) {
        collide_T_at<T>(rec, hat, n, c, g, nb[q], fd[q]);
        L.dpx[ly][lx] = nb[q].dpx;
        L.dpy[ly][lx] = nb[q].dpy;
        // the tile's own nodes (partial tiles hold wrapped copies beyond
        // nx or ny, which are only read as neighbours)
        if (x0 + lx - 1 < g.nx && y0 + ly - 1 < g.ny) {
          own[q] = n;
          alpha_acc += double(nb[q].alpha);
        }
      }
    }
    if (t < K::NH) {
      int ly, lx, n;
      ring_pos<K::HX, K::HY>(t, ly, lx);
      if (cm_node(x0, y0, ly, lx, g, n)) gradp_cot_at<T>(rec, hat, n, c, g, L.dpx[ly][lx], L.dpy[ly][lx]);
    }
    __syncthreads();
    // phase 2: full pressure cotangent and the macroscopic transposes
#pragma unroll
    for (int q = 0; q < K::NPT; ++q) {
      if (own[q] >= 0) {
        const int i = t + 256 * q;
        const int ly = 1 + i / K::TX, lx = 1 + i % K::TX;
        const T b_p = nb[q].p + gradT_p<T>(L, ly, lx, y0 + ly - 1, g);
        lam_acc += macro_T_at<T>(rec, own[q], nb[q], b_p, fd[q], hat_out, af, c, g);
      }
    }
    __syncthreads();
  }
  block_add(alpha_acc, AP_ALPHA, acc_part);
  block_add(lam_acc, AP_LAMBDA, acc_part);
}

// AK3: mu cotangent (node part + grad^T + lap^T), then the chemical
// potential mu = 4 beta (phi-1) phi (phi-1/2) - kappa lap phi.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_mu(const T* __restrict__ fphi, AF<T> af,
                                                double* acc_part, Coef<T> c, Geom g) {
  double beta_acc = 0.0, kappa_acc = 0.0;
  for (int n = blockIdx.x * 256 + threadIdx.x; n < (int)g.N; n += gridDim.x * 256) {
    const NodeIdx k = node_idx(n, g);
    const T b_mu = af[A_MU1][n] + stencil_T<T, true, true>(af[A_GMUX], af[A_GMUY], af[A_LMU], k);
    T v[3][3], gx, gy, lapphi;
    load3x3(fphi, k, v);
    stencil(v, gx, gy, lapphi);
    const T ph = v[1][1];
    const T dbulk = c.beta4 * (T(3) * ph * ph - T(3) * ph + T(0.5));
    af[A_PHI3][n] = af[A_PHI2][n] + b_mu * dbulk;
    af[A_LPHI][n] = -c.kappa * b_mu;
    beta_acc += double(b_mu) * 4.0 * double((ph - T(1)) * ph * (ph - T(0.5)));
    kappa_acc -= double(b_mu) * double(lapphi);
  }
  block_add(beta_acc, AP_BETA, acc_part);
  block_add(kappa_acc, AP_KAPPA, acc_part);
}

// AK4: phi cotangent (grad^T of grad phi's, lap^T of lap phi's), then the
// g cotangents gbar_i = direct + phibar, with the direct part (1 - 1/tau_g)
// times the post-collision cotangent gathered from hat again (the f
// cotangents are complete after AK1+2).
template <typename T>
__global__ __launch_bounds__(256) void k_adj_final(const T* __restrict__ hat, AF<T> af,
                                                   T* __restrict__ hat_out, Coef<T> c, Geom g) {
  for (int n = blockIdx.x * 256 + threadIdx.x; n < (int)g.N; n += gridDim.x * 256) {
    const NodeIdx k = node_idx(n, g);
    const T b_phi = af[A_PHI3][n] + stencil_T<T, true, true>(af[A_GPHX], af[A_GPHY], af[A_LPHI], k);
    T gh[9];
    post_hat9<T>(hat, 9, k, g.Ns, gh);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      hat_out[(int64_t)(9 + i) * g.Ns + n] = gh[i] * (T(1) - c.inv_tau_g) + b_phi;
  }
}

// Initial-state map transpose (FP64): s_0 = (0, H_i(phi0, mu0)),
// mu0 = 4 beta (phi0-1) phi0 (phi0-1/2) - kappa lap phi0.
template <typename T>
__global__ __launch_bounds__(256) void k_adj_init_local(const double* __restrict__ phi0,
                                                        const T* __restrict__ hat,
                                                        double* __restrict__ lphi_bar,
                                                        double* __restrict__ phi_bar,
                                                        double* acc_part, Coef<double> c, Geom g) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int n = blockIdx.x * 256 + threadIdx.x; n < (int)g.N; n += gridDim.x * 256) {
    const NodeIdx k = node_idx(n, g);
    double v[3][3], gx, gy, lap;
    load3x3(phi0, k, v);
    stencil(v, gx, gy, lap);
    const double ph = v[1][1];
    const double mu0 = mu_bulk(ph, c) - c.kappa * lap;
    double b_amu = -(1.0 - 4.0 / 9.0) * double(hat[(int64_t)9 * g.Ns + n]);
#pragma unroll
    for (int i = 1; i < 9; ++i) b_amu += WGT(i) * double(hat[(int64_t)(9 + i) * g.Ns + n]);
    const double b_mu = c.alpha * b_amu;
    acc[AP_ALPHA] += mu0 * b_amu;
    acc[AP_BETA] += b_mu * 4.0 * (ph - 1.0) * ph * (ph - 0.5);
    acc[AP_KAPPA] -= b_mu * lap;
    phi_bar[n] = double(hat[(int64_t)9 * g.Ns + n]) +
                 b_mu * c.beta4 * (3.0 * ph * ph - 3.0 * ph + 0.5);
    lphi_bar[n] = -c.kappa * b_mu;
  }
  block_add(acc[AP_BETA], AP_BETA, acc_part);
  block_add(acc[AP_KAPPA], AP_KAPPA, acc_part);
  block_add(acc[AP_ALPHA], AP_ALPHA, acc_part);
}

__global__ __launch_bounds__(256) void k_adj_init_final(const double* __restrict__ lphi_bar,
                                                        const double* __restrict__ phi_bar,
                                                        double* __restrict__ out, Geom g) {
  for (int n = blockIdx.x * 256 + threadIdx.x; n < (int)g.N; n += gridDim.x * 256) {
    const NodeIdx k = node_idx(n, g);
    out[n] = phi_bar[n] + stencil_T<double, false, true>(nullptr, nullptr, lphi_bar, k);
  }
}

// Canonical FP64 [9][N] pair <-> adjoint population planes [18][Ns].
template <typename T>
__global__ __launch_bounds__(256) void k_hat_from(const double* __restrict__ f,
                                                  const double* __restrict__ gg, T* __restrict__ hat,
                                                  Geom g) {
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N;
       n += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      hat[(int64_t)i * g.Ns + n] = T(f[(int64_t)i * g.N + n]);
      hat[(int64_t)(9 + i) * g.Ns + n] = T(gg[(int64_t)i * g.N + n]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_hat_to(const T* __restrict__ hat, double* __restrict__ f,
                                                double* __restrict__ gg, Geom g) {
  for (int64_t n = (int64_t)blockIdx.x * 256 + threadIdx.x; n < g.N;
       n += (int64_t)gridDim.x * 256) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f[(int64_t)i * g.N + n] = double(hat[(int64_t)i * g.Ns + n]);
      gg[(int64_t)i * g.N + n] = double(hat[(int64_t)(9 + i) * g.Ns + n]);
    }
  }
}

// ------------------------------------------------------ fused adjoint step
// The three kernels above in one sweep over the rows of a strip, the
// transposed stages in the order their dependencies allow (the forward
// kernel's pipeline run backwards). A workgroup of 256 lanes owns a strip of
// at most 248 columns plus 4 halo columns on each side (lane lc <-> column
// x0 - 4 + lc) and a segment of rows; the record rows and the cotangent
// fields that cross node boundaries live in LDS rings. In the iteration that
// brings in record row r (direction d):
//   0:  record row r (phi, mu, p, S, jx, jy) into the rings
//   A': collision transpose of row r - d (post-collision cotangents gathered
//       from the incoming cotangents, prefetched by the previous iteration);
//       grad p cotangent into LDS, the rest kept in registers
//   B': pressure cotangent of row r - 2d (grad^T of the grad p cotangents of
//       rows r - 3d .. r - d), the macroscopic transposes, f cotangents out;
//       grad mu, lambda D and grad phi cotangents into LDS
//   C': mu cotangent of row r - 3d (grad^T, lap^T), then mu(phi)
//   D': phi cotangent of row r - 4d (grad^T, lap^T), g cotangents out; the
//       gathers of row r's post-collision cotangents and the record row
//       r + d are issued here for the next iteration.
// Stage s (A' = 1 ... D' = 4) runs on lanes [s, wi + 8 - s) and rows
// [y0 - 4 + s, y1 + 4 - s); the record rows reach 4 beyond the segment.
constexpr int AH = 4;
#ifndef QILBM_ANT
#define QILBM_ANT 256
#endif
#ifndef QILBM_ADJ_WAVES32
#define QILBM_ADJ_WAVES32 2
#endif
constexpr int ANT = QILBM_ANT;

template <typename T>
struct AdjLds {
  T phi[8][ANT];             // record rows
  T mu[4][ANT];
  T p[4][ANT];
  T sj[4][3][ANT];           // S, jx, jy
  T gpx[4][ANT], gpy[4][ANT];                // grad p cotangent
  T gmx[4][ANT], gmy[4][ANT], lmu[4][ANT];   // grad mu cotangent, lambda x D cotangent
  T grx[4][ANT], gry[4][ANT];                // drho x grad rho cotangent (grad phi part)
  T lph[4][ANT];                             // -kappa x mu cotangent (lap phi part)
};

// Planes of T at a stride of Ns elements, through buffer resources: one
// descriptor for all planes, the plane and row in the scalar offset; BIG
// (the planes span 4 GiB or more): one descriptor per plane.
template <typename T, bool BIG>
struct PlaneArr {
  char* base;
  uint32_t ps;   // bytes between planes
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ void init(const T* p, int64_t Ns, int nplanes) {
    base = (char*)p;
    ps = (uint32_t)(Ns * (int64_t)sizeof(T));
    if constexpr (!BIG)
      r = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(nplanes * (int64_t)ps), BUF_WORD3);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t rs(int plane) const {
    if constexpr (BIG)
      return __builtin_amdgcn_make_buffer_rsrc(base + (int64_t)plane * ps, 0, (int)ps, BUF_WORD3);
    else
      return r;
  }
  __device__ __forceinline__ uint32_t so(int plane, uint32_t elem) const {
    return (BIG ? 0u : (uint32_t)plane * ps) + elem * (uint32_t)sizeof(T);
  }
  // element elem_row + col of plane
  __device__ __forceinline__ T ld(int plane, uint32_t elem_row, uint32_t col) const {
    return buf_ld<T>(rs(plane), col * (uint32_t)sizeof(T), so(plane, elem_row));
  }
  __device__ __forceinline__ void st(int plane, uint32_t elem_row, uint32_t col, T v) const {
    buf_st<T>(v, rs(plane), col * (uint32_t)sizeof(T), so(plane, elem_row));
  }
  // Element col of row elem_row / nx of plane, written only by lanes with
  // ok set. Every lane issues the store; the other lanes' offset lies 2 GiB
  // beyond the range of the descriptor, where the hardware drops a store.
  // No branch then separates the lanes that write from those that do not, so
  // the compiler's count of memory operations in flight stays exact across
  // the stores (with a branch it takes the path without them, and the next
  // wait for a load waits for the stores as well). The descriptors: not BIG,
  // one per group of 9 planes (the f and the g cotangents; under 2 GiB each
  // as the 18 planes span less than 4 GiB); BIG, one per plane and row.
  __device__ __forceinline__ void init_halves() {
    if constexpr (!BIG)
      for (int h = 0; h < 2; ++h)
        half[h] = __builtin_amdgcn_make_buffer_rsrc(base + (int64_t)(9 * h) * ps, 0,
                                                    (int)(9 * ps), BUF_WORD3);
  }
  __device__ __forceinline__ void st_if(bool ok, int plane, uint32_t elem_row, uint32_t col,
                                        uint32_t nx, T v) const {
    const uint32_t vo = col * (uint32_t)sizeof(T) + (ok ? 0u : 0x80000000u);
    if constexpr (!BIG) {
      buf_st<T>(v, half[plane >= 9], vo,
                (uint32_t)(plane % 9) * ps + elem_row * (uint32_t)sizeof(T));
    } else {
      const __amdgpu_buffer_rsrc_t rr = __builtin_amdgcn_make_buffer_rsrc(
          base + (int64_t)plane * ps + (int64_t)elem_row * sizeof(T), 0, (int)(nx * sizeof(T)),
          BUF_WORD3);
      buf_st<T>(v, rr, vo, 0u);
    }
  }
  __amdgpu_buffer_rsrc_t half[2];
};

template <typename T, bool BIG>
struct AdjCtx {
  PlaneArr<T, BIG> rec, hin, hout;
  Coef<T> c;
  Geom g;
  int lc, x, wi, y0, y1, d;
  int col[3];
  bool act;
  __device__ __forceinline__ bool in(int v, int s) const {
    return act && lc >= s && lc < wi + 2 * AH - s && v >= y0 - AH + s && v < y1 + AH - s &&
           (!g.walls || (v >= 0 && v < g.ny));
  }
  __device__ __forceinline__ bool owns(int v) const {
    return act && lc >= AH && lc < wi + AH && v >= y0 && v < y1;
  }
  // v if the tile owns row v, else its first row (a row of the lattice for
  // the descriptor of a store that no lane makes)
  __device__ __forceinline__ int own_row(int v) const { return v >= y0 && v < y1 ? v : y0; }
  // physical row of virtual row v (the halo reaches a few rows beyond the
  // lattice: a short uniform loop instead of a division)
  __device__ __forceinline__ int prow(int v) const {
    if (g.walls) return v;
    while (v < 0) v += g.ny;
    while (v >= g.ny) v -= g.ny;
    return v;
  }
  // +-1 on the bottom / top wall row, 0 elsewhere (uniform over the row)
  __device__ __forceinline__ int wall(int v) const {
    return !g.walls ? 0 : (v == 0 ? -1 : (v == g.ny - 1 ? 1 : 0));
  }
};

// Post-collision cotangents of row v at this lane's column, gathered from
// the incoming pre-collision cotangents (as post_hat: i at x + c_i, or
// opp(i) at x itself beyond a wall). WALL as AdjCtx::wall(v), so the choice
// per direction is made at compile time; ro[1 + dy]: element offset of row
// v + dy.
template <typename T, bool BIG, int WALL, int I = 0>
__device__ __forceinline__ void gather_post_w(const AdjCtx<T, BIG>& k, const uint32_t ro[3],
                                              int koff, T out[9]) {
  if constexpr (I < 9) {
    constexpr int cx = CXS(I), cy = CYS(I);
    constexpr bool bounce = (WALL == -1 && cy == -1) || (WALL == 1 && cy == 1);
    if constexpr (bounce)
      out[I] = k.hin.ld(koff + OPP(I), ro[1], k.col[1]);
    else
      out[I] = k.hin.ld(koff + I, ro[1 + cy], k.col[1 + cx]);
    gather_post_w<T, BIG, WALL, I + 1>(k, ro, koff, out);
  }
}

template <typename T, bool BIG>
__device__ __forceinline__ void gather_post(const AdjCtx<T, BIG>& k, int v, int koff, T out[9]) {
  const int w = k.wall(v);
  const uint32_t nx = (uint32_t)k.g.nx;
  const uint32_t ro[3] = {w == -1 ? 0u : (uint32_t)k.prow(v - 1) * nx, (uint32_t)k.prow(v) * nx,
                          w == 1 ? 0u : (uint32_t)k.prow(v + 1) * nx};
  if (w == -1)
    gather_post_w<T, BIG, -1>(k, ro, koff, out);
  else if (w == 1)
    gather_post_w<T, BIG, 1>(k, ro, koff, out);
  else
    gather_post_w<T, BIG, 0>(k, ro, koff, out);
}

// grad^T (vx, vy) (if GR) + lap^T ws (if LP) at row v, lane lc, from rings
// of four rows: the terms of stencil_T in the same order. On a wall row
// (WALL = -1 bottom, +1 top) the source row beyond the wall drops out and
// the mirrored ghost adds the row itself for the directions into the wall.
template <typename T, bool GR, bool LP, int WALL, int I>
__device__ __forceinline__ void gtl_term(const T (*vx)[ANT], const T (*vy)[ANT],
                                         const T (*ws)[ANT], int v, int lc, T& gacc, T& lacc) {
  constexpr int cx = CXS(I), cy = CYS(I);
  constexpr bool src = !((WALL == -1 && cy == 1) || (WALL == 1 && cy == -1));
  constexpr bool ghost = (WALL == -1 && cy == -1) || (WALL == 1 && cy == 1);
  const T w3 = T(3.0 * WGT(I)), w6 = T(6.0 * WGT(I));
  if constexpr (src) {
    const int ys = (v - cy) & 3;
    if constexpr (GR) gacc += w3 * cdot<cx, cy>(vx[ys][lc - cx], vy[ys][lc - cx]);
    if constexpr (LP) lacc += w6 * ws[ys][lc - cx];
  }
  if constexpr (ghost) {
    if constexpr (GR) gacc += w3 * cdot<cx, cy>(vx[v & 3][lc - cx], vy[v & 3][lc - cx]);
    if constexpr (LP) lacc += w6 * ws[v & 3][lc - cx];
  }
}

template <typename T, bool GR, bool LP, int WALL>
__device__ __forceinline__ T stencil_Tw(const T (*vx)[ANT], const T (*vy)[ANT],
                                        const T (*ws)[ANT], int v, int lc) {
  T gacc = T(0), lacc = T(0);
  gtl_term<T, GR, LP, WALL, 1>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 2>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 3>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 4>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 5>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 6>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 7>(vx, vy, ws, v, lc, gacc, lacc);
  gtl_term<T, GR, LP, WALL, 8>(vx, vy, ws, v, lc, gacc, lacc);
  if constexpr (LP) lacc -= T(10.0 / 3.0) * ws[v & 3][lc];
  return gacc + lacc;
}

template <typename T, bool GR, bool LP>
__device__ __forceinline__ T stencil_Tl(const T (*vx)[ANT], const T (*vy)[ANT],
                                        const T (*ws)[ANT], int v, int lc, int wall) {
  if (wall == -1) return stencil_Tw<T, GR, LP, -1>(vx, vy, ws, v, lc);
  if (wall == 1) return stencil_Tw<T, GR, LP, 1>(vx, vy, ws, v, lc);
  return stencil_Tw<T, GR, LP, 0>(vx, vy, ws, v, lc);
}

// Forward node state of row v at lane lc from the record rings (fwd_node).
template <typename T>
__device__ __forceinline__ void fwd_node_l(const AdjLds<T>& L, int v, int lc, const Coef<T>& c,
                                           const Geom& g, Macro<T>& m, T& S, T& jx, T& jy,
                                           T& gmux, T& gmuy, T& lapmu) {
  S = L.sj[v & 3][0][lc];
  jx = L.sj[v & 3][1][lc];
  jy = L.sj[v & 3][2][lc];
  T w[3][3], gphx, gphy, lapphi;
  lds3x3<T, ANT>(L.phi, 7, v, g.ny, g.walls, lc, w);
  stencil(w, gphx, gphy, lapphi);
  const T ph = w[1][1];
  lds3x3<T, ANT>(L.mu, 3, v, g.ny, g.walls, lc, w);
  stencil(w, gmux, gmuy, lapmu);
  macro_node(ph, w[1][1], gphx, gphy, gmux, gmuy, lapmu, S, jx, jy, c, m);
}

// Forward node state of a row as A' forms it, kept in registers for B' of the
// next iteration (the same row and lane: B' runs on a subset of A's rows and
// lanes).
template <typename T>
struct FwdState {
  Macro<T> m;
  T jx, jy, gmux, gmuy, lapmu;
};

// Whether the direct part of the g cotangents waits from A' to D' in
// registers (FP32) or is gathered again in D' (FP64, whose registers are
// full; the values are the same).
template <typename T> struct KeepGd { static constexpr bool value = sizeof(T) == 4; };

// Record row v (loaded into rrec) into the LDS rings.
template <typename T, bool BIG>
__device__ __forceinline__ void put_record(const AdjCtx<T, BIG>& k, int v, AdjLds<T>& L,
                                           const T (&rrec)[6]) {
  if (k.in(v, 0)) {
    const int lc = k.lc;
    L.phi[v & 7][lc] = rrec[R_PHI];
    L.mu[v & 3][lc] = rrec[R_MU];
    L.p[v & 3][lc] = rrec[R_P];
    L.sj[v & 3][0][lc] = rrec[R_S];
    L.sj[v & 3][1][lc] = rrec[R_JX];
    L.sj[v & 3][2][lc] = rrec[R_JY];
  }
}

template <typename T, bool BIG, int J>
__device__ __forceinline__ void adj_iter(const AdjCtx<T, BIG>& k, int r, AdjLds<T>& L, T (&rrec)[6],
                                         T (&hf)[9], T (&hg)[9], NodeBar<T> (&nbr)[2],
                                         FwdState<T> (&fst)[2],
                                         T (&fdr)[2][9], T (&gdr)[4][9], T (&p2)[2], T (&m1)[2],
                                         T (&p3)[2], double (&acc)[4]) {
  const Geom& g = k.g;
  const Coef<T>& c = k.c;
  const int lc = k.lc, d = k.d;
  const int a = r - d, b = r - 2 * d, cm = r - 3 * d, e = r - 4 * d;
  // (row r of the record is in the rings: put there at the end of the
  // previous iteration, or before the first)
  __syncthreads();
  // A': collision transpose of row a
  if (k.in(a, 1)) {
    FwdState<T>& fs = fst[J & 1];
    T S;
    fwd_node_l<T>(L, a, lc, c, g, fs.m, S, fs.jx, fs.jy, fs.gmux, fs.gmuy, fs.lapmu);
    T w[3][3], dpx, dpy, lapp;
    lds3x3<T, ANT>(L.p, 3, a, g.ny, g.walls, lc, w);
    stencil(w, dpx, dpy, lapp);
    collide_node_T(hf, hg, fs.m, dpx, dpy, c, nbr[J & 1]);
    // the direct part of the f cotangents, (1 - 1/tau_f) times the
    // post-collision ones, waits for B' in registers
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      fdr[J & 1][i] = hf[i];
      if constexpr (KeepGd<T>::value) gdr[J & 3][i] = hg[i];
    }
    L.gpx[a & 3][lc] = nbr[J & 1].dpx;
    L.gpy[a & 3][lc] = nbr[J & 1].dpy;
    if (k.owns(a)) acc[AP_ALPHA] += double(nbr[J & 1].alpha);
  }
  // The loads for the next iteration go out as soon as their registers are
  // free: a wait on the memory counter also waits for every store issued
  // before the load it needs, so a load issued behind the stores of D'
  // would wait for them. hf and hg are free once A' has kept what it needs.
  if (k.in(r, 1)) {
    gather_post<T>(k, r, 0, hf);
    gather_post<T>(k, r, 9, hg);
  }
  __syncthreads();
  // B': pressure cotangent and the macroscopic transposes of row b
  T o_S = T(0), o_jx = T(0), o_jy = T(0);
  if (k.in(b, 2)) {
    const NodeBar<T>& nb = nbr[(J + 1) & 1];
    const T b_p = nb.p + stencil_Tl<T, true, false>(L.gpx, L.gpy, nullptr, b, lc, k.wall(b));
    // the forward state of row b, formed by A' in the previous iteration
    const FwdState<T>& fs = fst[(J + 1) & 1];
    const Macro<T>& m = fs.m;
    const T jx = fs.jx, jy = fs.jy, gmux = fs.gmux, gmuy = fs.gmuy, lapmu = fs.lapmu;
    T b_rho = nb.rho, b_ux = nb.ux, b_uy = nb.uy;
    T b_Fx = nb.Fx, b_Fy = nb.Fy, b_drx = nb.drx, b_dry = nb.dry;
    T b_D = nb.D, b_phi = nb.phi;
    const T b_S = b_p;
    b_ux += b_p * m.drx * T(1.0 / 6.0);
    b_uy += b_p * m.dry * T(1.0 / 6.0);
    b_drx += b_p * m.ux * T(1.0 / 6.0);
    b_dry += b_p * m.uy * T(1.0 / 6.0);
    b_rho -= b_p * c.gamma * m.D * T(1.0 / 6.0);
    b_D -= b_p * c.gamma * m.rho * T(1.0 / 6.0);
    const T rinv = recip(m.rho);
    const T inv = T(3) * rinv;
    const T b_jx = b_ux * inv, b_jy = b_uy * inv;
    b_Fx += b_ux * inv * T(1.0 / 6.0);
    b_Fy += b_uy * inv * T(1.0 / 6.0);
    const T b_inv = b_ux * (jx + m.Fx * T(1.0 / 6.0)) + b_uy * (jy + m.Fy * T(1.0 / 6.0));
    b_rho -= b_inv * inv * rinv;
    b_phi -= b_Fx * gmux + b_Fy * gmuy;
    L.gmx[b & 3][lc] = -m.phi * b_Fx;
    L.gmy[b & 3][lc] = -m.phi * b_Fy;
    b_rho += b_Fx * c.gx + b_Fy * c.gy;
    L.lmu[b & 3][lc] = c.lam * b_D;
    L.grx[b & 3][lc] = c.drho * b_drx;
    L.gry[b & 3][lc] = c.drho * b_dry;
    p2[J & 1] = b_phi + c.drho * b_rho;
    m1[J & 1] = nb.mu;
    o_S = b_S;
    o_jx = b_jx;
    o_jy = b_jy;
    if (k.owns(b)) acc[AP_LAMBDA] += double(b_D) * double(lapmu);
  }
  {
    // the f cotangents of row b out, from every lane (st_if)
    const uint32_t ro = (uint32_t)(k.own_row(b) * g.nx);
    const bool ok = k.owns(b);
    fbar_out([&](int i, T v) { k.hout.st_if(ok, i, ro, (uint32_t)k.x, (uint32_t)g.nx, v); },
             fdr[(J + 1) & 1], o_S, o_jx, o_jy);
  }
  __syncthreads();
  T he[9] = {};
  if constexpr (!KeepGd<T>::value)
    if (k.owns(e)) gather_post<T>(k, e, 9, he);
  // the next record row (rrec is free: row r is in the rings)
  if (k.in(r + d, 0)) {
    const uint32_t ro = (uint32_t)(k.prow(r + d) * g.nx);
#pragma unroll
    for (int q = 0; q < 6; ++q) rrec[q] = k.rec.ld(q, ro, (uint32_t)k.x);
  }
  // C': mu cotangent of row cm, then mu(phi)
  if (k.in(cm, 3)) {
    const T b_mu = m1[(J + 1) & 1] + stencil_Tl<T, true, true>(L.gmx, L.gmy, L.lmu, cm, lc, k.wall(cm));
    T w[3][3], gx, gy, lapphi;
    lds3x3<T, ANT>(L.phi, 7, cm, g.ny, g.walls, lc, w);
    stencil(w, gx, gy, lapphi);
    const T ph = w[1][1];
    const T dbulk = c.beta4 * (T(3) * ph * ph - T(3) * ph + T(0.5));
    p3[J & 1] = p2[(J + 1) & 1] + b_mu * dbulk;
    L.lph[cm & 3][lc] = -c.kappa * b_mu;
    if (k.owns(cm)) {
      acc[AP_BETA] += double(b_mu) * 4.0 * double((ph - T(1)) * ph * (ph - T(0.5)));
      acc[AP_KAPPA] -= double(b_mu) * double(lapphi);
    }
  }
  __syncthreads();
  // D': phi cotangent of row e, g cotangents out
  {
    const bool ok = k.owns(e);
    T b_phi = T(0);
    if (ok)
      b_phi = p3[(J + 1) & 1] + stencil_Tl<T, true, true>(L.grx, L.gry, L.lph, e, lc, k.wall(e));
    const uint32_t ro = (uint32_t)(k.own_row(e) * g.nx);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      k.hout.st_if(ok, 9 + i, ro, (uint32_t)k.x, (uint32_t)g.nx,
                    (KeepGd<T>::value ? gdr[(J + 1) & 3][i] : he[i] * (T(1) - c.inv_tau_g)) +
                        b_phi);
  }
  // record row r + d into the rings for the next iteration (here rather than
  // at the top of the next one, so that its wait for the record loads is
  // counted in straight-line code and leaves D''s stores in flight)
  put_record(k, r + d, L, rrec);
}

template <typename T>
struct AdjWaves { static constexpr int value = sizeof(T) == 8 ? 1 : QILBM_ADJ_WAVES32; };

// BIG: the 18 cotangent planes span 4 GiB or more (one descriptor per plane).
template <typename T, bool BIG>
__global__ __launch_bounds__(ANT, AdjWaves<T>::value) void k_adj_fused(
    const T* __restrict__ rec, const T* __restrict__ hin, T* __restrict__ hout,
    double* acc_part, Coef<T> c, Geom g, int width, int nstrips, int seg_len, int ntiles) {
  __shared__ AdjLds<T> L;
  AdjCtx<T, BIG> k;
  k.rec.init(rec, g.Ns, 6);
  k.hin.init(hin, g.Ns, 18);
  k.hout.init(hout, g.Ns, 18);
  k.hout.init_halves();
  k.c = c;
  k.g = g;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  // the first round of tiles XCD-aware (xcd_tile permutes 0 .. gridDim - 1),
  // later rounds, if any, at a stride of gridDim
  for (int tile = xcd_tile(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
    const int seg = tile / nstrips, strip = tile - seg * nstrips;
    const int x0 = strip * width;
    k.wi = min(width, g.nx - x0);
    k.y0 = seg * seg_len;
    k.y1 = min(g.ny, k.y0 + seg_len);
    k.d = (seg & 1) ? -1 : 1;
    const int t = threadIdx.x;
    k.act = t < k.wi + 2 * AH;
    k.lc = k.act ? t : AH;
    int xv = (x0 - AH + k.lc) % g.nx;
    k.x = xv < 0 ? xv + g.nx : xv;
    k.col[0] = wrap_x(k.x - 1, g.nx);
    k.col[1] = k.x;
    k.col[2] = wrap_x(k.x + 1, g.nx);
    T rrec[6], hf[9], hg[9], fdr[2][9], gdr[4][9], p2[2], m1[2], p3[2];
    NodeBar<T> nbr[2];
    FwdState<T> fst[2];
    const int r0 = k.d > 0 ? k.y0 - AH : k.y1 + AH - 1;
    const int nit = (k.y1 - k.y0) + 2 * AH + 1;
    if (k.in(r0, 0)) {
      const uint32_t ro = (uint32_t)(k.prow(r0) * g.nx);
#pragma unroll
      for (int q = 0; q < 6; ++q) rrec[q] = k.rec.ld(q, ro, (uint32_t)k.x);
    }
    put_record(k, r0, L, rrec);
    for (int it = 0; it < nit; it += 4) {
      adj_iter<T, BIG, 0>(k, r0 + k.d * (it + 0), L, rrec, hf, hg, nbr, fst, fdr, gdr, p2, m1,
                            p3, acc);
      adj_iter<T, BIG, 1>(k, r0 + k.d * (it + 1), L, rrec, hf, hg, nbr, fst, fdr, gdr, p2, m1,
                            p3, acc);
      adj_iter<T, BIG, 2>(k, r0 + k.d * (it + 2), L, rrec, hf, hg, nbr, fst, fdr, gdr, p2, m1,
                            p3, acc);
      adj_iter<T, BIG, 3>(k, r0 + k.d * (it + 3), L, rrec, hf, hg, nbr, fst, fdr, gdr, p2, m1,
                            p3, acc);
    }
    __syncthreads();
  }
  block_add(acc[AP_BETA], AP_BETA, acc_part);
  block_add(acc[AP_KAPPA], AP_KAPPA, acc_part);
  block_add(acc[AP_LAMBDA], AP_LAMBDA, acc_part);
  block_add(acc[AP_ALPHA], AP_ALPHA, acc_part);
}

// ------------------------------------------------------------------ host
template <typename T>
Coef<T> coef_of(const CtxView& v) {
  const lbm_params* p = v.prm;
  Coef<T> k;
  k.beta4 = T(4.0 * v.beta);
  k.kappa = T(v.kappa);
  k.lam = T(v.lam);
  k.alpha = T(v.alpha);
  k.gamma = T(v.gamma);
  k.drho = T(v.drho);
  k.rho_B = T(p->rho_B);
  k.rho_ref = T(p->rho_ref);
  k.gx = T(p->gx);
  k.gy = T(p->gy);
  k.inv_tau_f = T(1.0 / p->tau_f);
  k.inv_tau_g = T(1.0 / p->tau_g);
  k.kf = T(1.0 - 0.5 / p->tau_f);
  k.kg = T(1.0 - 0.5 / p->tau_g);
  return k;
}

struct AdjLayout {
  size_t hat0, hat1, fld, afld, part, acc, total;
  int nred;
};

AdjLayout adj_layout(const lbm_params* p) {
  const int64_t N = (int64_t)p->nx * p->ny;
  const int64_t Ns = plane_stride(N);
  const size_t ts = p->precision == LBM_FP64 ? 8 : 4;
  AdjLayout L;
  L.nred = (int)((N + 255) / 256);
  if (L.nred > 2048) L.nred = 2048;
  const size_t pops = up(18 * (size_t)Ns * ts);
  L.hat0 = 0;
  L.hat1 = L.hat0 + pops;
  L.fld = L.hat1 + pops;
  // the field area holds a record (6 planes of the compute type) recomputed
  // from a raw state; the initial-state transpose uses two FP64 planes of it
  const size_t fb = up((size_t)Ns * (6 * ts > 16 ? 6 * ts : 16));
  L.afld = L.fld + fb;
  L.part = L.afld + up((size_t)A_NFIELDS * Ns * ts);
  L.acc = L.part + up((size_t)L.nred * 4 * 8);
  L.total = L.acc + up(8 * 8);
  return L;
}

// One adjoint step from the record of forward step t.
template <typename T>
lbm_status adj_core(const CtxView& v, const T* rec) {
  AdjointState& a = *v.adj;
  const Geom& g = v.geom;
  const Coef<T> k = coef_of<T>(v);
  AF<T> af{(T*)a.afld, g.Ns};
  const T* hin = (const T*)a.hat[a.cur];
  T* hout = (T*)a.hat[a.cur ^ 1];
  const dim3 grid(a.nred), blk(256);
  if (v.prm->flags & LBM_FLAG_UNFUSED) {
    hipLaunchKernelGGL(k_adj_cm<T>, grid, blk, 0, v.stream, rec, hin, hout, af, a.part, k, g);
    hipLaunchKernelGGL(k_adj_mu<T>, grid, blk, 0, v.stream, rec + (int64_t)R_PHI * g.Ns, af,
                       a.part, k, g);
    hipLaunchKernelGGL(k_adj_final<T>, grid, blk, 0, v.stream, hin, af, hout, k, g);
  } else {
    // strips of at most 248 columns; one round of workgroups (every segment
    // end recomputes 4 rows); at most nred workgroups, one partial slot each
    const int fw = ANT - 2 * AH;
    const int nstrips = (g.nx + fw - 1) / fw;
    const int width = (g.nx + nstrips - 1) / nstrips;
    if (a.resident <= 0) {
      int dev = 0, cus = 0, per_cu = 0;
      if (hipGetDevice(&dev) == hipSuccess &&
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
          hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_adj_fused<T, false>, ANT, 0) ==
              hipSuccess)
        a.resident = cus * (per_cu > 0 ? per_cu : 1);
      if (a.resident <= 0) a.resident = 256;
    }
    int nseg = a.resident / nstrips;
    if (nseg < 1) nseg = 1;
    int seg = (g.ny + nseg - 1) / nseg;
    if (seg < 16) seg = 16;
    if (seg > g.ny) seg = g.ny;
    nseg = (g.ny + seg - 1) / seg;
    const int ntiles = nstrips * nseg;
    const int nblk = ntiles < a.nred ? ntiles : a.nred;
    if (18 * g.Ns * (int64_t)sizeof(T) > (int64_t)UINT32_MAX)
      hipLaunchKernelGGL((k_adj_fused<T, true>), dim3(nblk), dim3(ANT), 0, v.stream, rec, hin,
                         hout, a.part, k, g, width, nstrips, seg, ntiles);
    else
      hipLaunchKernelGGL((k_adj_fused<T, false>), dim3(nblk), dim3(ANT), 0, v.stream, rec, hin,
                         hout, a.part, k, g, width, nstrips, seg, ntiles);
  }
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  a.cur ^= 1;
  return LBM_OK;
}

// One adjoint step from a raw forward state: its record is recomputed into
// the field area with the unfused forward kernels.
template <int P>
lbm_status adj_step_p(const CtxView& v, const void* fwd) {
  using T = typename PrecT<P>::T;
  AdjointState& a = *v.adj;
  const Geom& g = v.geom;
  const Coef<T> k = coef_of<T>(v);
  T* rec = (T*)a.fld;
  hipError_t e = launch_fields<P>(fwd, rec + R_PHI * g.Ns, rec + R_MU * g.Ns, k, g, v.stream);
  if (e != hipSuccess) return LBM_EDEVICE;
  e = launch_macro<P>(fwd, rec + R_PHI * g.Ns, rec + R_MU * g.Ns, rec + R_P * g.Ns,
                      rec + R_S * g.Ns, MomentOut{}, k, g, v.stream);
  if (e != hipSuccess) return LBM_EDEVICE;
  return adj_core<T>(v, rec);
}

template <typename T>
lbm_status adj_init_t(const CtxView& v, const double* phi0, double* dphi0, double out[2]) {
  AdjointState& a = *v.adj;
  const Geom& g = v.geom;
  const Coef<double> k = coef_of<double>(v);
  double* lphi = (double*)a.fld;
  double* phib = lphi + g.Ns;
  const dim3 grid(a.nred), blk(256);
  hipLaunchKernelGGL(k_adj_init_local<T>, grid, blk, 0, v.stream, phi0, (const T*)a.hat[a.cur],
                     lphi, phib, a.part, k, g);
  hipLaunchKernelGGL(k_adj_init_final, grid, blk, 0, v.stream, (const double*)lphi,
                     (const double*)phib, dphi0, g);
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  if (launch_sum_partials(a.part, a.nred, 4, a.acc + 4, v.stream) != hipSuccess)
    return LBM_EDEVICE;
  double tot[4];
  if (hipMemcpyAsync(tot, a.acc + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, v.stream) !=
      hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(v.stream) != hipSuccess) return LBM_EDEVICE;
  const lbm_params* p = v.prm;
  // beta, kappa proportional to sigma (W fixed); lambda = M, alpha proportional to M.
  out[0] = (tot[AP_BETA] * v.beta + tot[AP_KAPPA] * v.kappa) / p->sigma;
  out[1] = tot[AP_LAMBDA] + tot[AP_ALPHA] * v.alpha / p->M;
  return LBM_OK;
}

}  // namespace
}  // namespace qilbm

using namespace qilbm;

extern "C" {

// The adjoint transposes the BGK collisions only: contexts with the
// two-relaxation-time variant are refused.
size_t lbm_adjoint_workspace_bytes(const lbm_params* params) {
  if (!params || lbm_workspace_bytes(params) == 0 || params->trt_magic > 0.0) return 0;
  return adj_layout(params).total;
}

lbm_status lbm_adjoint_begin(lbm_ctx* ctx, void* ws, size_t bytes, const double* dL_dphi) {
  if (!ctx || !ws || !dL_dphi) return LBM_EINVAL;
  if ((uintptr_t)ws % ALIGN != 0) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  if (v.prm->trt_magic > 0.0) return LBM_EINVAL;
  const AdjLayout L = adj_layout(v.prm);
  if (bytes < L.total) return LBM_ENOMEM;
  AdjointState& a = *v.adj;
  a.ws = (char*)ws;
  a.bytes = bytes;
  a.hat[0] = a.ws + L.hat0;
  a.hat[1] = a.ws + L.hat1;
  a.cur = 0;
  a.fld = a.ws + L.fld;
  a.afld = a.ws + L.afld;
  a.part = (double*)(a.ws + L.part);
  a.acc = (double*)(a.ws + L.acc);
  a.nred = L.nred;
  a.active = true;
  return lbm_adjoint_seed(ctx, dL_dphi);
}

lbm_status lbm_adjoint_seed(lbm_ctx* ctx, const double* dL_dphi) {
  if (!ctx || !dL_dphi) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  AdjointState& a = *v.adj;
  if (!a.active) return LBM_ESTATE;
  a.cur = 0;
  const Geom& g = v.geom;
  hipLaunchKernelGGL(k_fill_zero, dim3(a.nred), dim3(256), 0, v.stream, a.part,
                     (int64_t)a.nred * 4);
  if (v.prm->precision == LBM_FP64)
    hipLaunchKernelGGL(k_adj_seed<double>, dim3(a.nred), dim3(256), 0, v.stream, dL_dphi,
                       (double*)a.hat[0], g);
  else
    hipLaunchKernelGGL(k_adj_seed<float>, dim3(a.nred), dim3(256), 0, v.stream, dL_dphi,
                       (float*)a.hat[0], g);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* fwd_state) {
  if (!ctx || !fwd_state) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  if (v.prm->trt_magic > 0.0) return LBM_EINVAL;
  if (!v.adj->active) return LBM_ESTATE;
  switch (v.prm->precision) {
    case LBM_FP64: return adj_step_p<P_F64>(v, fwd_state);
    case LBM_FP32: return adj_step_p<P_F32>(v, fwd_state);
    default: return adj_step_p<P_F16>(v, fwd_state);
  }
}

lbm_status lbm_adjoint_step_record(lbm_ctx* ctx, const void* record_dev) {
  if (!ctx || !record_dev) return LBM_EINVAL;
  if ((uintptr_t)record_dev % ALIGN != 0) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  if (v.prm->trt_magic > 0.0) return LBM_EINVAL;
  if (!v.adj->active) return LBM_ESTATE;
  if (v.prm->precision == LBM_FP64) return adj_core<double>(v, (const double*)record_dev);
  return adj_core<float>(v, (const float*)record_dev);
}

lbm_status lbm_adjoint_init(lbm_ctx* ctx, const double* phi0, double* dphi0, double out[2]) {
  if (!ctx || !phi0 || !dphi0 || !out) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  if (!v.adj->active) return LBM_ESTATE;
  if (v.prm->precision == LBM_FP64) return adj_init_t<double>(v, phi0, dphi0, out);
  return adj_init_t<float>(v, phi0, dphi0, out);
}

lbm_status lbm_adjoint_set(lbm_ctx* ctx, const double* fbar, const double* gbar) {
  if (!ctx || !fbar || !gbar) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  AdjointState& a = *v.adj;
  if (!a.active) return LBM_ESTATE;
  hipLaunchKernelGGL(k_fill_zero, dim3(a.nred), dim3(256), 0, v.stream, a.part,
                     (int64_t)a.nred * 4);
  if (v.prm->precision == LBM_FP64)
    hipLaunchKernelGGL(k_hat_from<double>, dim3(a.nred), dim3(256), 0, v.stream, fbar, gbar,
                       (double*)a.hat[a.cur], v.geom);
  else
    hipLaunchKernelGGL(k_hat_from<float>, dim3(a.nred), dim3(256), 0, v.stream, fbar, gbar,
                       (float*)a.hat[a.cur], v.geom);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_adjoint_get(lbm_ctx* ctx, double* fbar, double* gbar, double out[2]) {
  if (!ctx || !fbar || !gbar || !out) return LBM_EINVAL;
  CtxView v = ctx_view(ctx);
  AdjointState& a = *v.adj;
  if (!a.active) return LBM_ESTATE;
  if (v.prm->precision == LBM_FP64)
    hipLaunchKernelGGL(k_hat_to<double>, dim3(a.nred), dim3(256), 0, v.stream,
                       (const double*)a.hat[a.cur], fbar, gbar, v.geom);
  else
    hipLaunchKernelGGL(k_hat_to<float>, dim3(a.nred), dim3(256), 0, v.stream,
                       (const float*)a.hat[a.cur], fbar, gbar, v.geom);
  if (hipGetLastError() != hipSuccess) return LBM_EDEVICE;
  if (launch_sum_partials(a.part, a.nred, 4, a.acc + 4, v.stream) != hipSuccess)
    return LBM_EDEVICE;
  double tot[4];
  if (hipMemcpyAsync(tot, a.acc + 4, 4 * sizeof(double), hipMemcpyDeviceToHost, v.stream) !=
      hipSuccess)
    return LBM_EDEVICE;
  if (hipStreamSynchronize(v.stream) != hipSuccess) return LBM_EDEVICE;
  out[0] = (tot[AP_BETA] * v.beta + tot[AP_KAPPA] * v.kappa) / v.prm->sigma;
  out[1] = tot[AP_LAMBDA] + tot[AP_ALPHA] * v.alpha / v.prm->M;
  return LBM_OK;
}

}  // extern "C"
