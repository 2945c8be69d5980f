// Device-side building blocks of the quasi-incompressible phase-field LBE
// step (Yang & Guo, Sec. III) for gfx950: D2Q9 tables, derived
// coefficients, population storage formats, pull-streaming addressing with
// half-way bounce-back, the isotropic stencils and the per-node collision.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace qilbm {

// ------------------------------------------------------------------ lattice
// D2Q9 (Sec. III): c_0 = 0; c_1..4 axis-aligned at angles (i-1) pi/2;
// c_5..8 diagonal at (2i-1) pi/4. Weights 4/9, 1/9, 1/36; c_s^2 = 1/3.
__host__ __device__ constexpr int CXS(int i) {
  return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__host__ __device__ constexpr int CYS(int i) {
  return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__host__ __device__ constexpr int OPP(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) & 3) + 1 : ((i - 3) & 3) + 5);
}
__host__ __device__ constexpr double WGT(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
static_assert(OPP(1) == 3 && OPP(2) == 4 && OPP(3) == 1 && OPP(4) == 2, "opp");
static_assert(OPP(5) == 7 && OPP(6) == 8 && OPP(7) == 5 && OPP(8) == 6, "opp");

// ------------------------------------------------------------- coefficients
// Everything the step needs, derived on the host in FP64 (Sec. II-III) and
// rounded once to the compute type T.
template <typename T>
struct Coef {
  T beta4;      // 4 beta (bulk chemical potential 4 beta (phi-1) phi (phi-1/2))
  T kappa;      // gradient-energy coefficient
  T lam;        // mobility lambda
  T alpha;      // alpha of H_i
  T gamma;      // quasi-incompressibility coefficient (0 for the ablation)
  T drho;       // d rho / d phi
  T rho_B;      // density at phi = 0
  T rho_ref;    // reference density of the body force
  T gx, gy;     // gravity
  T inv_tau_f, inv_tau_g;
  T kf, kg;     // 1 - 1 / (2 tau)
  // two-relaxation-time collision of f (used by the TRT kernel variants):
  // 1 / tau_- and 1 - 1 / (2 tau_-) of the part odd under c_i -> -c_i
  T inv_tau_m, km;
};

struct Geom {
  int nx, ny;
  int walls;    // 1: bounce-back walls below row 0 and above row ny-1
  int64_t N;    // nx * ny
  int64_t Ns;   // plane stride in elements (N rounded up to 256)
};

// ----------------------------------------------------------- storage formats
enum Prec : int { P_F64 = 0, P_F32 = 1, P_F16 = 2 };

// Power-of-two scale of binary16 plane i (f_i and g_i, i >= 1; also f_0):
// 2^14 times the power of two nearest 1/w_i, so that populations of size
// ~ w_i * 1e-2 sit well inside the normal binary16 range.
__host__ __device__ constexpr float H_SCALE(int i) {
  return i == 0 ? 32768.0f : (i <= 4 ? 131072.0f : 524288.0f);
}
__host__ __device__ constexpr float H_INV(int i) {
  return i == 0 ? (1.0f / 32768.0f) : (i <= 4 ? (1.0f / 131072.0f) : (1.0f / 524288.0f));
}

template <int P> struct PrecT;
template <> struct PrecT<P_F64> { using T = double; };
template <> struct PrecT<P_F32> { using T = float; };
template <> struct PrecT<P_F16> { using T = float; };

// In the 32-bit and 16-bit storage modes the order-parameter populations g
// are kept in fixed point Q2.29 (int32: range +-4, step 2^-29): all nine in
// FP32 mode, g_0 (the O(1) one) in FP16-storage mode, whose g_1..8 stay
// scaled binary16. The collision writes g_0* = phi_q - sum_{i>=1} q(g_i*)
// with phi_q the exact integer sum of the node's pulled g, and streaming and
// bounce-back move the stored words unchanged, so the lattice total of phi
// is an exact integer invariant (the mass conservation of the model).
template <int P> struct FixedG { static constexpr bool value = P != P_F64; };
constexpr float GQ = 536870912.0f;            // 2^29
constexpr float GQI = 1.0f / 536870912.0f;
constexpr double GQI_D = 1.0 / 536870912.0;
constexpr double GQ_D = 536870912.0;
// Q2.29 contribution of a binary16 plane value: its value times 2^29, i.e.
// the stored half times 2^29 / H_SCALE(i), a power of two.
__host__ __device__ constexpr float HQ(int i) {
  return i == 0 ? 16384.0f : (i <= 4 ? 4096.0f : 1024.0f);
}
// The Q2.29 word of a stored binary16 g_i: the half times HQ(i), exact in
// binary32, truncated toward zero (a fraction remains only for halves below
// 1 / HQ(i), i.e. g below one Q2.29 step). Every kernel, and the host-side
// total of the tests, maps a half this one way, so g_0 = phi_q - sum of the
// other words keeps the lattice total an exact integer invariant; truncation
// is one conversion where rounding to nearest takes two.
__device__ __forceinline__ int32_t q_half(__half h, int i) {
  return (int32_t)(__half2float(h) * HQ(i));
}

// Bytes of one population buffer (18 planes).
__host__ __device__ inline int64_t pop_bytes(int P, int64_t Ns) {
  return P == P_F64 ? 18 * Ns * 8 : (P == P_F32 ? 18 * Ns * 4 : 17 * Ns * 2 + Ns * 4);
}

// Plane k in 0..17: f_0..f_8 are k = 0..8, g_0..g_8 are k = 9..17.
// f_i and g_i always move together (same pull source), so the 32-bit and
// 16-bit modes store them side by side and one access serves both:
// FP64: 18 binary64 planes. FP32: for i = 0..8 one plane of 64-bit words
// holding f_i (low word, binary32) and g_i (high word, Q2.29 int32). FP16
// storage: the f_0 plane (binary16), the g_0 plane (Q2.29 int32), then for
// i = 1..8 one plane of 32-bit words holding f_i (low half) and g_i (high
// half), both binary16.
// A plane's base address is uniform across the wavefront; the per-lane part
// is a 32-bit byte offset (lattices are capped so that it cannot overflow),
// which lets the compiler use scalar-base + 32-bit-offset addressing.
template <int P>
struct Pop {
  char* base;
  int64_t Ns;
  using T = typename PrecT<P>::T;

  template <typename S>
  __device__ __forceinline__ static S at(const char* plane, uint32_t idx) {
    return *reinterpret_cast<const S*>(plane + idx * (uint32_t)sizeof(S));
  }
  template <typename S>
  __device__ __forceinline__ static void put(char* plane, uint32_t idx, S v) {
    *reinterpret_cast<S*>(plane + idx * (uint32_t)sizeof(S)) = v;
  }
  // FP16 storage: address of the binary16 of plane k (k != 9) at idx
  __device__ __forceinline__ char* half_at(int k, uint32_t idx) const {
    if (k == 0) return base + idx * 2u;
    const int i = k < 9 ? k : k - 9;
    return base + 6 * Ns + (int64_t)(i - 1) * 4 * Ns + idx * 4u + (k < 9 ? 0 : 2);
  }
  __device__ __forceinline__ static __half half_ld(const char* a) {
    return *reinterpret_cast<const __half*>(a);
  }
  // FP32: address of the binary32 f_k (k < 9) or Q2.29 g_{k-9} word at idx
  __device__ __forceinline__ char* word_at(int k, uint32_t idx) const {
    const int i = k < 9 ? k : k - 9;
    return base + (int64_t)i * 8 * Ns + idx * 8u + (k < 9 ? 0 : 4);
  }
  __device__ __forceinline__ static int dir(int k) { return k < 9 ? k : k - 9; }

  // value of plane k at idx
  __device__ __forceinline__ T ld(int k, uint32_t idx) const {
    if constexpr (P == P_F64) {
      return at<double>(base + k * Ns * 8, idx);
    } else if constexpr (P == P_F32) {
      if (k < 9) return *reinterpret_cast<const float*>(word_at(k, idx));
      return float(*reinterpret_cast<const int32_t*>(word_at(k, idx))) * GQI;
    } else {
      if (k == 9) return float(at<int32_t>(base + 2 * Ns, idx)) * GQI;
      return __half2float(half_ld(half_at(k, idx))) * H_INV(dir(k));
    }
  }
  // value of plane k at idx in binary64: exact for f planes and FP64; for g
  // planes in the fixed-point modes the Q2.29 value, the quantity whose
  // lattice total the scheme conserves exactly
  __device__ __forceinline__ double ld_exact(int k, uint32_t idx) const {
    if constexpr (P == P_F64) {
      return at<double>(base + k * Ns * 8, idx);
    } else {
      if (k >= 9) return double(ld_q(k, idx)) * GQI_D;
      if constexpr (P == P_F32) return double(*reinterpret_cast<const float*>(word_at(k, idx)));
      else return double(__half2float(half_ld(half_at(k, idx)))) * double(H_INV(k));
    }
  }
  // value of plane k at idx in binary64 exactly as stored: binary16 halves
  // scaled back (not their Q2.29 contribution), Q2.29 words, binary32 f
  __device__ __forceinline__ double ld_canon(int k, uint32_t idx) const {
    if constexpr (P == P_F16) {
      if (k != 9) return double(__half2float(half_ld(half_at(k, idx)))) * double(H_INV(dir(k)));
    }
    return ld_exact(k, idx);
  }
  // Q2.29 contribution of g plane k (9..17) at idx (fixed-point modes only)
  __device__ __forceinline__ int32_t ld_q(int k, uint32_t idx) const {
    if constexpr (P == P_F32) {
      return *reinterpret_cast<const int32_t*>(word_at(k, idx));
    } else {
      if (k == 9) return at<int32_t>(base + 2 * Ns, idx);
      return q_half(half_ld(half_at(k, idx)), dir(k));
    }
  }
  // stores v into plane k; for g planes in the fixed-point modes returns the
  // Q2.29 contribution of what was stored (0 otherwise)
  __device__ __forceinline__ int32_t st(int k, uint32_t idx, T v) const {
    if constexpr (P == P_F64) {
      put<double>(base + k * Ns * 8, idx, v);
      return 0;
    } else if constexpr (P == P_F32) {
      if (k < 9) {
        *reinterpret_cast<float*>(word_at(k, idx)) = v;
        return 0;
      }
      const int32_t q = __float2int_rn(v * GQ);
      *reinterpret_cast<int32_t*>(word_at(k, idx)) = q;
      return q;
    } else {
      if (k == 9) {
        const int32_t q = __float2int_rn(v * GQ);
        put<int32_t>(base + 2 * Ns, idx, q);
        return q;
      }
      const __half h = __float2half_rn(v * H_SCALE(dir(k)));
      *reinterpret_cast<__half*>(half_at(k, idx)) = h;
      return k < 9 ? 0 : q_half(h, dir(k));
    }
  }
  // stores the binary64 value v into plane k with a single rounding to the
  // storage format: binary32 f, Q2.29 g words, binary16 (scaled) halves;
  // the inverse of ld_exact for values the format represents
  __device__ __forceinline__ void st_exact(int k, uint32_t idx, double v) const {
    if constexpr (P == P_F64) {
      put<double>(base + k * Ns * 8, idx, v);
    } else if constexpr (P == P_F32) {
      if (k < 9) *reinterpret_cast<float*>(word_at(k, idx)) = float(v);
      else *reinterpret_cast<int32_t*>(word_at(k, idx)) = __double2int_rn(v * GQ_D);
    } else {
      if (k == 9) {
        put<int32_t>(base + 2 * Ns, idx, __double2int_rn(v * GQ_D));
        return;
      }
      const _Float16 h = (_Float16)(v * double(H_SCALE(dir(k))));
      *reinterpret_cast<_Float16*>(half_at(k, idx)) = h;
    }
  }
  // stores the Q2.29 word q into g_0 (fixed-point modes)
  __device__ __forceinline__ void st_g0_q(uint32_t idx, int32_t q) const {
    if constexpr (P == P_F32) *reinterpret_cast<int32_t*>(word_at(9, idx)) = q;
    else if constexpr (P == P_F16) put<int32_t>(base + 2 * Ns, idx, q);
  }
};

// Buffer-resource access: a descriptor covers a byte range (loads beyond it
// return 0, stores beyond it are dropped); the uniform part of an address
// goes into the scalar offset, the lane's part into the vector offset.
constexpr int BUF_WORD3 = 0x00020000;
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

template <typename S>
__device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(S) == 8) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  } else if constexpr (sizeof(S) == 4) {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0));
  }
}
template <typename S>
__device__ __forceinline__ void buf_st(S v, __amdgpu_buffer_rsrc_t r, uint32_t voff,
                                       uint32_t soff) {
  if constexpr (sizeof(S) == 8) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
  } else if constexpr (sizeof(S) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
  } else {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, voff, soff, 0);
  }
}

// Tiles handed out so that blocks that the hardware places on one XCD
// (consecutive blocks round-robin over 8 XCDs) get consecutive tiles, i.e.
// neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int bid, int n) {
  const int q = n >> 3, rem = n & 7, j = bid & 7, pos = bid >> 3;
  return j * q + (j < rem ? j : rem) + pos;
}

// ------------------------------------------------------------- addressing
__device__ __forceinline__ int wrap_x(int x, int nx) {
  return x < 0 ? x + nx : (x >= nx ? x - nx : x);
}
// Row of the stencil neighbour: periodic wrap, or the mirrored boundary row
// (ghost rows psi(x,-1) = psi(x,0), psi(x,ny) = psi(x,ny-1)) at walls.
__device__ __forceinline__ int nbr_row(int y, const Geom& g) {
  if (y < 0) return g.walls ? 0 : y + g.ny;
  if (y >= g.ny) return g.walls ? g.ny - 1 : y - g.ny;
  return y;
}

// Pull streaming: the pre-collision population i at (x, y) is the
// post-collision population i of node (x - c_i, y - c_i,y); when that node
// lies beyond a wall it is the post-collision population opp(i) of (x, y)
// itself (half-way bounce-back). Returns plane offset (0..8) and index.
template <int I>
__device__ __forceinline__ void pull_src(int x, int y, const Geom& g, int& plane, uint32_t& idx) {
  constexpr int cx = CXS(I), cy = CYS(I);
  int ys = y - cy;
  if (ys < 0 || ys >= g.ny) {
    if (g.walls) { plane = OPP(I); idx = (uint32_t)(y * g.nx + x); return; }
    ys = ys < 0 ? ys + g.ny : ys - g.ny;
  }
  plane = I;
  idx = (uint32_t)(ys * g.nx + wrap_x(x - cx, g.nx));
}

// --------------------------------------------------------- per-node algebra
// Fused multiply-add in the compute type.
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

// 1/x: correctly rounded in FP64; the hardware reciprocal (1 ulp) in FP32.
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// Bulk part of mu: 4 beta (phi - phi_A)(phi - phi_B)(phi - (phi_A+phi_B)/2)
// with phi_A = 1, phi_B = 0 (Sec. II).
template <typename T>
__device__ __forceinline__ T mu_bulk(T phi, const Coef<T>& c) {
  // (phi - 1) phi (phi - 1/2) = phi (phi (phi - 3/2) + 1/2)
  return c.beta4 * (phi * fmad(phi, phi - T(1.5), T(0.5)));
}

// Isotropic central stencils on a 3x3 neighbourhood v[dy+1][dx+1]:
// grad = 3 sum_i w_i c_i v(c_i), lap = 6 sum_i w_i (v(c_i) - v(0)).
template <typename T>
__device__ __forceinline__ void stencil(const T v[3][3], T& gx, T& gy, T& lap) {
  // with w = 1/9 (axis), 1/36 (diagonal): 3 w = 1/3, 1/12 and 6 w = 2/3, 1/6
  const T ex = v[1][2] - v[1][0];
  const T ey = v[2][1] - v[0][1];
  const T d1 = v[2][2] - v[0][0];   // (1,1) - (-1,-1)
  const T d2 = v[0][2] - v[2][0];   // (1,-1) - (-1,1)
  gx = fmad(T(1.0 / 12.0), d1 + d2, T(1.0 / 3.0) * ex);
  gy = fmad(T(1.0 / 12.0), d1 - d2, T(1.0 / 3.0) * ey);
  const T sa = (v[1][2] + v[1][0]) + (v[2][1] + v[0][1]);
  const T sd = (v[2][2] + v[0][0]) + (v[0][2] + v[2][0]);
  lap = fmad(T(2.0 / 3.0), sa, fmad(T(1.0 / 6.0), sd, T(-10.0 / 3.0) * v[1][1]));
}

// The same stencil's 3x3 neighbourhood from a ring of rows in LDS: row v of
// the lattice sits in ring[v & mask], lane lc holds the lane's column (the
// neighbours at lc -+ 1); at a wall the mirrored ghost row is the row itself.
// walls is 0 or 1: the ghost-row shift as integer arithmetic stays in scalar
// registers (as a boolean select the compiler formed it per lane), and one
// lane address per row serves its three reads.
template <typename T, int NT>
__device__ __forceinline__ void lds3x3(const T (*ring)[NT], int mask, int v, int ny, int walls,
                                       int lc, T out[3][3]) {
  const int vm = v - 1 + (walls & (int)(v == 0));
  const int vp = v + 1 - (walls & (int)(v == ny - 1));
  const T* a = &ring[vm & mask][lc - 1];
  const T* b = &ring[v & mask][lc - 1];
  const T* d = &ring[vp & mask][lc - 1];
  out[0][0] = a[0]; out[0][1] = a[1]; out[0][2] = a[2];
  out[1][0] = b[0]; out[1][1] = b[1]; out[1][2] = b[2];
  out[2][0] = d[0]; out[2][1] = d[1]; out[2][2] = d[2];
}

// Macroscopic state of one node needed by the collision.
template <typename T>
struct Macro {
  T phi, rho, mu, ux, uy, p, Fx, Fy, drx, dry, D;
};

// Force F = -phi grad mu + (rho - rho_ref) g, velocity
// u = (j + F/6) / (rho/3), pressure p = S + (u.grad rho - gamma rho D)/6
// (Sec. III moments; Sec. II force).
template <typename T>
__device__ __forceinline__ void macro_node(T phi, T mu, T gphx, T gphy, T gmux, T gmuy,
                                           T lapmu, T S, T jx, T jy, const Coef<T>& c,
                                           Macro<T>& m) {
  m.phi = phi;
  m.mu = mu;
  m.rho = c.rho_B + c.drho * phi;
  m.drx = c.drho * gphx;
  m.dry = c.drho * gphy;
  m.D = c.lam * lapmu;
  const T b = m.rho - c.rho_ref;
  m.Fx = -phi * gmux + b * c.gx;
  m.Fy = -phi * gmuy + b * c.gy;
  const T inv = T(3) * recip(m.rho);
  m.ux = (jx + m.Fx * T(1.0 / 6.0)) * inv;
  m.uy = (jy + m.Fy * T(1.0 / 6.0)) * inv;
  m.p = S + T(1.0 / 6.0) * (m.ux * m.drx + m.uy * m.dry - c.gamma * m.rho * m.D);
}

// c.(x, y) for the direction (CX, CY) known at compile time: signs and
// sums only (a product with a zero component is not folded away in IEEE
// arithmetic, so the generic form would multiply).
template <int CX, int CY, typename T>
__device__ __forceinline__ T cdot(T x, T y) {
  static_assert(CX != 0 || CY != 0, "rest direction");
  if constexpr (CX == 0) return CY > 0 ? y : -y;
  else if constexpr (CY == 0) return CX > 0 ? x : -x;
  else if constexpr (CX > 0) return CY > 0 ? x + y : x - y;
  else return CY > 0 ? y - x : -(x + y);
}

// What every direction of one node's collision shares.
template <typename T>
struct CollNode {
  T ux, uy, usq15;     // u and 1.5 |u|^2
  T Fx, Fy, uF;        // F and u.F
  T dx, dy, ud;        // grad rho / 3 and u.(grad rho / 3)
  T qx, qy, uq;        // grad p - F and u.(grad p - F)
};

template <typename T>
__device__ __forceinline__ CollNode<T> coll_node(const Macro<T>& m, T dpx, T dpy) {
  CollNode<T> n;
  n.ux = m.ux;
  n.uy = m.uy;
  n.usq15 = T(1.5) * fmad(m.uy, m.uy, m.ux * m.ux);
  n.Fx = m.Fx;
  n.Fy = m.Fy;
  n.uF = fmad(m.uy, m.Fy, m.ux * m.Fx);
  n.dx = m.drx * T(1.0 / 3.0);
  n.dy = m.dry * T(1.0 / 3.0);
  n.ud = fmad(m.uy, n.dy, m.ux * n.dx);
  n.qx = dpx - m.Fx;
  n.qy = dpy - m.Fy;
  n.uq = fmad(m.uy, n.qy, m.ux * n.qx);
  return n;
}

// Direction I of the Sec. III algebra: s = 3 c.u + 4.5 (c.u)^2 - 1.5 u^2,
// X = (c - u).(Gamma F + s grad rho / 3) and Y = Gamma (c - u).(grad p - F)
// with Gamma = 1 + s, i.e. with A = (c-u).F, B = (c-u).grad rho / 3,
// Q = (c-u).(grad p - F): X = A + s (A + B), Y = Q + s Q.
template <int I, typename T>
__device__ __forceinline__ void coll_dir(const CollNode<T>& n, T& s, T& X, T& Y) {
  T A, B, Q;
  if constexpr (I == 0) {
    s = -n.usq15;
    A = -n.uF;
    B = -n.ud;
    Q = -n.uq;
  } else {
    constexpr int cx = CXS(I), cy = CYS(I);
    const T cu = cdot<cx, cy>(n.ux, n.uy);
    s = fmad(cu, fmad(T(4.5), cu, T(3)), -n.usq15);
    A = cdot<cx, cy>(n.Fx, n.Fy) - n.uF;
    B = cdot<cx, cy>(n.dx, n.dy) - n.ud;
    Q = cdot<cx, cy>(n.qx, n.qy) - n.uq;
  }
  X = fmad(s, A + B, A);
  Y = fmad(s, Q, Q);
}

// Per-node factors of the relaxation for one weight class j (rest, axis,
// diagonal; w_j = 4/9, 1/9, 1/36):
//   f* = (1 - 1/tau_f) f + w [p/tau_f + kf src1] + w rho/(3 tau_f) s + w kf X
//   g* = (1 - 1/tau_g) g + H/tau_g + w phi/tau_g s + w kg K Y
// with src1 = -rho gamma D / 3, K = -3 phi / rho, kf, kg = 1 - 1/(2 tau),
// H_0 = phi - (1 - w_0) alpha mu, H_j = w_j alpha mu (j > 0). They are
// formed just before the class's directions, so only one class's are live.
template <typename T>
struct CollNodeF {
  T pf, rf, amu, ph, K;    // p/tau_f + kf src1, rho/(3 tau_f), alpha mu, phi/tau_g, K
  T phi;
};

template <typename T>
__device__ __forceinline__ CollNodeF<T> coll_nodef(const Macro<T>& m, const Coef<T>& c) {
  CollNodeF<T> q;
  q.pf = fmad(m.p, c.inv_tau_f, -(m.rho * m.D) * (c.kf * c.gamma * T(1.0 / 3.0)));
  q.rf = m.rho * (c.inv_tau_f * T(1.0 / 3.0));
  q.amu = c.alpha * m.mu;
  q.ph = m.phi * c.inv_tau_g;
  q.K = -T(3) * m.phi * recip(m.rho);
  q.phi = m.phi;
  return q;
}

template <typename T>
struct CollClass {
  T f0, fs, fx;   // f: constant part, factor of s, factor of X
  T g0, gs, gy;   // g: constant part, factor of s, factor of Y
};

template <int J, typename T>
__device__ __forceinline__ CollClass<T> coll_class(const CollNodeF<T>& q, const Coef<T>& c) {
  constexpr double wd = J == 0 ? 4.0 / 9.0 : (J == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
  const T w = T(wd);
  CollClass<T> k;
  k.f0 = w * q.pf;
  k.fs = w * q.rf;
  k.fx = w * c.kf;
  k.gs = w * q.ph;
  k.gy = q.K * (w * c.kg);
  if constexpr (J == 0) k.g0 = fmad(-T(1.0 - wd), q.amu, q.phi) * c.inv_tau_g;
  else k.g0 = q.amu * (w * c.inv_tau_g);
  return k;
}

template <int I> __host__ __device__ constexpr int wclass() { return I == 0 ? 0 : (I <= 4 ? 1 : 2); }

template <int I = 0, typename T>
__device__ __forceinline__ void collide_dirs(T f[9], T g[9], const CollNode<T>& n,
                                             const CollNodeF<T>& q, CollClass<T> k,
                                             const Coef<T>& c, T af, T ag) {
  if constexpr (I < 9) {
    if constexpr (I == 0 || I == 1 || I == 5) k = coll_class<wclass<I>()>(q, c);
    T s, X, Y;
    coll_dir<I>(n, s, X, Y);
    f[I] = fmad(af, f[I], fmad(k.fx, X, fmad(k.fs, s, k.f0)));
    g[I] = fmad(ag, g[I], fmad(k.gy, Y, fmad(k.gs, s, k.g0)));
    collide_dirs<I + 1>(f, g, n, q, k, c, af, ag);
  }
}

// BGK collision of both populations with the source terms (Sec. III):
// s_i = 3 c.u + 4.5 (c.u)^2 - 1.5 u^2, Gamma_i = 1 + s_i,
// f^eq = w (p + rho s / 3), F_i = w (c-u).(Gamma F + s grad rho / 3) - w rho gamma D / 3,
// g^eq = H_i + w phi s, G_i = -3 (phi/rho) w Gamma (c-u).(grad p - F),
// x* = x - (x - x^eq)/tau + (1 - 1/(2 tau)) X_i,
// evaluated through the shared per-node and per-weight-class factors above.
template <typename T>
__device__ __forceinline__ void collide_node(T f[9], T g[9], const Macro<T>& m, T dpx, T dpy,
                                             const Coef<T>& c) {
  const CollNode<T> n = coll_node(m, dpx, dpy);
  const CollNodeF<T> q = coll_nodef(m, c);
  collide_dirs(f, g, n, q, CollClass<T>{}, c, T(1) - c.inv_tau_f, T(1) - c.inv_tau_g);
}

// Two-relaxation-time variant of the f collision (g keeps BGK): f, f^eq and
// F_i split into parts even and odd under c_i -> -c_i; the even part relaxes
// with tau_f, the odd part with tau_- (magic parameter
// (tau_f - 1/2)(tau_- - 1/2)), and each source part takes its own
// 1 - 1/(2 tau) (Ginzburg, Verhaeghe and d'Humieres, 2008). The rest
// population has no odd part.
template <int I = 0, typename T>
__device__ __forceinline__ void trt_terms(T g[9], T feq[9], T Fs[9], const CollNode<T>& n,
                                          const CollNodeF<T>& q, CollClass<T> k,
                                          const Macro<T>& m, const Coef<T>& c, T src1, T ag) {
  if constexpr (I < 9) {
    if constexpr (I == 0 || I == 1 || I == 5) k = coll_class<wclass<I>()>(q, c);
    const T w = T(WGT(I));
    T s, X, Y;
    coll_dir<I>(n, s, X, Y);
    feq[I] = w * fmad(m.rho * T(1.0 / 3.0), s, m.p);
    Fs[I] = w * (X + src1);
    g[I] = fmad(ag, g[I], fmad(k.gy, Y, fmad(k.gs, s, k.g0)));
    trt_terms<I + 1>(g, feq, Fs, n, q, k, m, c, src1, ag);
  }
}

template <typename T>
__device__ __forceinline__ void collide_node_trt(T f[9], T g[9], const Macro<T>& m, T dpx,
                                                 T dpy, const Coef<T>& c) {
  const CollNode<T> n = coll_node(m, dpx, dpy);
  const CollNodeF<T> q = coll_nodef(m, c);
  const T src1 = -m.rho * c.gamma * m.D * T(1.0 / 3.0);
  T feq[9], Fs[9];
  trt_terms(g, feq, Fs, n, q, CollClass<T>{}, m, c, src1, T(1) - c.inv_tau_g);
  f[0] = f[0] - (f[0] - feq[0]) * c.inv_tau_f + c.kf * Fs[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int o = OPP(i);
    if (o < i) continue;
    const T fp = T(0.5) * (f[i] + f[o]), fm = T(0.5) * (f[i] - f[o]);
    const T ep = T(0.5) * (feq[i] + feq[o]), em = T(0.5) * (feq[i] - feq[o]);
    const T sp = T(0.5) * (Fs[i] + Fs[o]), sm = T(0.5) * (Fs[i] - Fs[o]);
    const T dp = c.kf * sp - (fp - ep) * c.inv_tau_f;
    const T dm = c.km * sm - (fm - em) * c.inv_tau_m;
    f[i] = f[i] + dp + dm;
    f[o] = f[o] + dp - dm;
  }
}

}  // namespace qilbm
