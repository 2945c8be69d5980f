/*
 * qilbm3d.h -- C ABI of the three-dimensional (D3Q19) form of the
 * quasi-incompressible phase-field lattice Boltzmann step of Yang & Guo
 * (Sec. III). The paper states its scheme on D2Q9 and notes that the choice
 * is without loss of generality; here every term keeps its form with three
 * velocity components on the D3Q19 lattice (weights 1/3, 1/18, 1/36;
 * c_s^2 = 1/3), and the isotropic central differences use the same vectors
 * and weights: grad psi = 3 sum_i w_i c_i psi(x + c_i),
 * lap psi = 6 sum_i w_i (psi(x + c_i) - psi(x)).
 *
 * Conventions (otherwise as in qilbm.h, whose status codes, precision and
 * flag values this header reuses):
 *   Lattice: nx x ny x nz, node (x, y, z) at linear index (z*ny + y)*nx + x;
 *     periodic in x and y; in z periodic (LBM_BC_PERIODIC) or half-way
 *     bounce-back walls below plane 0 and above plane nz-1 (value 1, walls
 *     normal to z; stencils mirror the boundary plane into the ghost plane).
 *   Population sets [19][nz][ny][nx] in this direction order:
 *     0 (0,0,0); 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1)
 *     6 (0,0,-1); 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0)
 *     11 (1,0,1) 12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1)
 *     15 (0,1,1) 16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1).
 *   Precision: LBM_FP64 (binary64 populations) or LBM_FP32 (f binary32, g
 *     Q2.29 fixed point: int32 values in [-4, 4) at resolution 2^-29, so the
 *     lattice total of phi is an exact integer invariant); LBM_FP16_STORE is
 *     not offered in 3-D.
 *   Kernels: the populations in a pull layout. FP32 runs one fused kernel
 *     per step (a workgroup sweeps a 64 x 16 column tile along z, phi, mu
 *     and p in LDS plane rings; f collides where the pressure is formed, g
 *     a plane later, and the g collision scatters each g word to the node it
 *     streams to, accumulating the next step's phi as an exact Q2.29 sum in
 *     a workspace buffer); FP64, and FP32 with LBM_FLAG_UNFUSED, run four
 *     kernels per step (phi; mu; pressure with the collision of f; the
 *     collision of g), one wave per 64-node run of a row. The two FP32 paths agree to rounding
 *     order and hold the same exact phi total.
 *   Memory, streams, errors: as in qilbm.h (caller-owned device workspace,
 *     asynchronous calls on the context's stream except lbm3_mass).
 */
#ifndef QILBM3D_H
#define QILBM3D_H

#include <stddef.h>
#include <stdint.h>

#include "qilbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t nx, ny, nz;     /* lattice size; each >= 3, nx*ny*nz <= 2^29 - 4096 */
  double rho_A, rho_B;    /* densities of fluid A (phi = 1) and B (phi = 0)   */
  double sigma, W, M;     /* surface tension, interface width, mobility > 0   */
  double tau_f, tau_g;    /* relaxation times > 1/2                            */
  double gx, gy, gz;      /* gravity: F_b = (rho - rho_ref)(gx, gy, gz)        */
  double rho_ref;         /* reference density of the body force              */
  int32_t bc;             /* LBM_BC_PERIODIC, or 1 = walls normal to z         */
  int32_t precision;      /* LBM_FP64 or LBM_FP32                              */
  uint32_t flags;         /* LBM_FLAG_NO_GAMMA, LBM_FLAG_UNFUSED (others are
                             rejected)                                        */
  double trt_magic;       /* 0: the paper's BGK collision of f; > 0: the
                             two-relaxation-time collision of f with this
                             magic parameter, as lbm_params.trt_magic (the
                             D3Q19 opposite pairs). Finite, >= 0.             */
} lbm3_params;

typedef struct lbm3_ctx lbm3_ctx;

/* Device workspace bytes for these parameters (0 when invalid): two
 * population buffers, the phi/mu/p fields and the momentum j between the two
 * collision kernels of the four-kernel form, reduction partials and two
 * int32 buffers of the Q2.29 phi sums of the fused FP32 step. */
size_t lbm3_workspace_bytes(const lbm3_params* params);

/* Context at t = 0 from phi0_dev (FP64 [nz][ny][nx], device): f = 0 and
 * g_i = H_i(phi0, mu0) (u = 0, p = 0). workspace_dev: caller-owned, at least
 * lbm3_workspace_bytes bytes, 256-byte aligned, alive until lbm3_destroy.
 * stream: a hipStream_t (NULL = default). */
lbm_status lbm3_init(lbm3_ctx** out, const lbm3_params* params, void* workspace_dev,
                     size_t workspace_bytes, const double* phi0_dev, void* stream);

/* Advances nsteps >= 0 coupled time steps. Asynchronous. */
lbm_status lbm3_step(lbm3_ctx* ctx, int64_t nsteps);

/* phi, rho, u = (ux, uy, uz), p, mu at the current time as FP64
 * [nz][ny][nx] device arrays; NULL skips a field. Asynchronous. */
lbm_status lbm3_moments(lbm3_ctx* ctx, double* phi_dev, double* rho_dev, double* ux_dev,
                        double* uy_dev, double* uz_dev, double* p_dev, double* mu_dev);

/* FP64 totals (sum phi, sum rho, sum rho ux, sum rho uy, sum rho uz) into
 * out[5] (host), phi and rho from the exact stored values; fixed reduction
 * order. Synchronises the stream; LBM_EDIVERGED for a non-finite total. */
lbm_status lbm3_mass(lbm3_ctx* ctx, double out[5]);

/* Pre-collision populations in the canonical FP64 layout, f_dev and g_dev
 * each [19][nz][ny][nx] (device); set_state rounds to the storage
 * precision and keeps the time counter. Asynchronous. */
lbm_status lbm3_get_state(lbm3_ctx* ctx, double* f_dev, double* g_dev);
lbm_status lbm3_set_state(lbm3_ctx* ctx, const double* f_dev, const double* g_dev);

/* Steps taken since lbm3_init, or -1 for a null context. */
int64_t lbm3_time(const lbm3_ctx* ctx);

/* Releases the host context (not the caller's workspace). */
void lbm3_destroy(lbm3_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* QILBM3D_H */
