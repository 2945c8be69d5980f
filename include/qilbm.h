/*
 * qilbm.h -- C ABI of a gfx950 (AMD Instinct MI355X) implementation of the
 * quasi-incompressible phase-field lattice Boltzmann model of Yang & Guo,
 * "A lattice Boltzmann method for binary fluids based on mass-conserved
 * quasi-incompressible phase-field theory" (Sec. III, the two coupled LBEs).
 *
 * One coupled time step advances, on a D2Q9 lattice (dx = dt = 1):
 *   - the order-parameter LBE for g_i, whose moment phi = sum_i g_i obeys the
 *     Cahn-Hilliard equation with mobility lambda (Sec. III, g-LBE and its
 *     equilibrium H_i + w_i phi s_i(u) and source G_i);
 *   - the flow LBE for f_i, whose moments give the velocity u and the
 *     hydrodynamic pressure p (Sec. III, f-LBE with equilibrium
 *     w_i [p + c_s^2 rho s_i(u)] and source F_i carrying the force
 *     F = -phi grad mu + F_b and the divergence source
 *     -gamma div(lambda grad mu) of the quasi-incompressible model, Sec. II);
 *   - isotropic central finite differences (gradient, Laplacian) of phi,
 *     mu and p; mu = dpsi/dphi - kappa lap phi with the double-well psi
 *     (Sec. II).
 *
 * Conventions
 *   Lattice: nx columns (x, always periodic) by ny rows (y); node (x, y) has
 *     linear index y*nx + x. A population set is [9][ny][nx] (direction
 *     major), directions c_0 = (0,0), c_1..4 = (1,0),(0,1),(-1,0),(0,-1),
 *     c_5..8 = (1,1),(-1,1),(-1,-1),(1,-1).
 *   Order parameter: phi_A = 1 (fluid A), phi_B = 0 (fluid B).
 *   Coefficients derived by the library: beta = 12 sigma / W and
 *     kappa = 3 sigma W / 2 (from the interface-width and surface-tension
 *     relations of Sec. II), lambda = M, alpha = M / (c_s^2 (tau_g - 1/2))
 *     (Sec. III), gamma = (rho_A/rho_B - 1) (Sec. II with phi_B = 0).
 *   Boundaries: LBM_BC_PERIODIC (both axes) or LBM_BC_WALLS_Y (half-way
 *     bounce-back walls below row 0 and above row ny-1; stencils mirror the
 *     boundary row into the ghost row).
 *   Memory: every pointer marked _dev is device memory owned by the caller.
 *     The library never allocates or frees device memory; all state lives
 *     in the caller's workspace. The library owns only the host context and
 *     one static device array per GPU (the scratch of lbm_mass_noalloc).
 *   Streams: every call enqueues its work on the context's HIP stream and
 *     returns without synchronising, except lbm_mass, lbm_adjoint_init and
 *     lbm_adjoint_get (host outputs), which synchronise that stream.
 *   Errors: every function returns an lbm_status; arguments are validated
 *     before any device work, and nothing is enqueued when validation fails.
 *     Kernel-launch failures return LBM_EDEVICE. No exception or abort
 *     crosses the ABI.
 *   Threads: a context is bound to one stream and is not thread-safe.
 */
#ifndef QILBM_H
#define QILBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,     /* invalid argument (checked on the host)            */
  LBM_ENOMEM = -2,     /* workspace too small, host allocation failed       */
  LBM_EDEVICE = -3,    /* HIP error while enqueueing or synchronising       */
  LBM_EDIVERGED = -4,  /* non-finite total returned by lbm_mass             */
  LBM_ESTATE = -5      /* call not valid in the context's current state     */
} lbm_status;

typedef enum {
  LBM_FP64 = 0,        /* populations stored and computed in binary64       */
  LBM_FP32 = 1,        /* f stored as binary32, g as Q2.29 fixed point
                          (int32: values in [-4, 4) at resolution 2^-29, so
                          the lattice total of phi is an exact integer
                          invariant); arithmetic in binary32               */
  LBM_FP16_STORE = 2   /* f_0..8 and g_1..8 stored as binary16 scaled by a
                          power of two per direction, g_0 as Q2.29 int32;
                          arithmetic in binary32                            */
} lbm_precision;

typedef enum { LBM_BC_PERIODIC = 0, LBM_BC_WALLS_Y = 1 } lbm_bc;

/* lbm_params.flags */
#define LBM_FLAG_NO_GAMMA 1u  /* drop the gamma (quasi-incompressible) terms
                                 from F_i and p: the same LBE in the form of
                                 an incompressible model, for ablations    */
#define LBM_FLAG_UNFUSED  2u  /* run the step as four separate kernels that
                                 materialise phi, mu and p, and the adjoint
                                 step as three (same results up to
                                 rounding; used for cross-checks)           */

typedef struct {
  int32_t nx, ny;         /* lattice size; nx >= 3, ny >= 3,
                             nx * ny <= 2^29 - 4096                          */
  double rho_A, rho_B;    /* densities of fluid A (phi = 1) and B (phi = 0) */
  double sigma;           /* surface tension, > 0                            */
  double W;               /* interface width in lattice units, > 0          */
  double M;               /* mobility lambda of the Cahn-Hilliard eq., > 0  */
  double tau_f, tau_g;    /* relaxation times, > 1/2                         */
  double gx, gy;          /* gravity: body force F_b = (rho - rho_ref)(gx, gy) */
  double rho_ref;         /* reference density of the body force           */
  int32_t bc;             /* lbm_bc                                          */
  int32_t precision;      /* lbm_precision                                   */
  uint32_t flags;         /* LBM_FLAG_*                                      */
  double trt_magic;       /* 0: the paper's BGK collision of f. > 0: a
                             two-relaxation-time collision of f (a variant
                             beyond the paper, which cites generalisations
                             with several relaxation times but specifies
                             none): f, f^eq and F_i split into parts even and
                             odd under c_i -> -c_i; the even part relaxes with
                             tau_f, the odd part with tau_- = 1/2 + trt_magic /
                             (tau_f - 1/2), each source part with its own
                             1 - 1/(2 tau). g keeps BGK. 3/16 puts half-way
                             bounce-back walls exactly half-way for any tau_f.
                             With TRT, step records and the adjoint are
                             refused (LBM_EINVAL). Finite, >= 0.            */
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of device workspace lbm_init needs for these parameters (0 when
 * the parameters are invalid). The workspace holds two population buffers
 * in the storage precision, the phi/mu/p scratch fields and the reduction
 * partials. */
size_t lbm_workspace_bytes(const lbm_params* params);

/* Derived coefficients (beta, kappa, lambda, alpha, gamma, d rho/d phi) of
 * Sec. II-III for these parameters, into out[6] (host memory). */
lbm_status lbm_coefficients(const lbm_params* params, double out[6]);

/* Creates a context at t = 0 from the initial order parameter phi0_dev
 * (FP64, [ny][nx], device). The initial pre-collision state has u = 0 and
 * p = 0, hence f_i = f_i^eq = 0, and g_i = H_i(phi0, mu0) with
 * mu0 = mu(phi0) (Sec. III equilibria), so that sum_i g_i = phi0.
 * workspace_dev: caller-owned, at least lbm_workspace_bytes(params) bytes,
 * 256-byte aligned, kept alive until lbm_destroy; lbm_init zeroes its
 * population buffers (padding included, so raw snapshots of equal states
 * are equal byte for byte). stream: a hipStream_t (NULL = default stream).
 * On success *out receives the context. */
lbm_status lbm_init(lbm_ctx** out, const lbm_params* params,
                    void* workspace_dev, size_t workspace_bytes,
                    const double* phi0_dev, void* stream);

/* Advances nsteps >= 0 coupled time steps (Sec. III: moments, chemical
 * potential, force, velocity, pressure, both BGK collisions with their
 * source terms, streaming). Asynchronous. Every kernel launch reads one of
 * the context's two population buffers and writes the other, and the
 * context then switches to the other buffer (host-side state). A caller
 * that captures lbm_step in a HIP graph for repeated replay must capture an
 * even number of launches, so that each replay starts from the buffer the
 * previous one ended in: with one step per launch an even nsteps, with two
 * steps per launch (lbm_set_pass) a multiple of 4. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Macroscopic fields at the current time t (Sec. III moments): phi, rho,
 * u = (ux, uy), p and mu, each FP64 [ny][nx] device arrays; any pointer
 * may be NULL to skip that field. Asynchronous. */
lbm_status lbm_moments(lbm_ctx* ctx, double* phi_dev, double* rho_dev,
                       double* ux_dev, double* uy_dev, double* p_dev,
                       double* mu_dev);

/* Lattice totals at time t into out[4] (host): sum phi, sum rho,
 * sum rho ux, sum rho uy, accumulated in FP64 in a fixed order (run-to-run
 * bitwise reproducible). Synchronises the stream. Returns LBM_EDIVERGED
 * when a total is not finite (out is still written). The mass of the
 * quasi-incompressible model is conserved exactly by the scheme (Sec. II,
 * local mass conservation), so sum phi and sum rho are invariants. */
lbm_status lbm_mass(lbm_ctx* ctx, double out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the four
 * lbm_mass totals of a raw state, without a context or workspace, and
 * without allocating anything.
 * params: the parameters the state was made with (validated as for
 *   lbm_init; nx * ny must not exceed LBM_MASS_NOALLOC_MAX_NODES, else
 *   LBM_EINVAL).
 * state_dev: a raw state in the layout of lbm_save_raw for these parameters
 *   (lbm_state_bytes bytes, device memory, 256-byte aligned), read only.
 * out_dev: device memory for 4 doubles (8-byte aligned), written with sum
 *   phi, sum rho, sum rho ux, sum rho uy -- bit for bit the values lbm_mass
 *   reports for a context holding that state (same kernels, same order).
 * stream: a hipStream_t of the current device (NULL = default stream).
 * Asynchronous: no synchronisation, no host output, no divergence check
 * (the caller reads out_dev after the stream has run).
 * Scratch: the kernels keep their intermediate phi and mu fields and block
 * partials in one static device array of LBM_MASS_NOALLOC_SCRATCH_BYTES
 * (32 MiB + 64 KiB) per GPU, held from the first call on that GPU until the
 * process ends and looked up once per GPU. Every call on a GPU uses that
 * GPU's one array, whichever thread or stream makes it: calls whose work
 * overlaps on one GPU (concurrent streams, threads) race and give wrong
 * totals; serialise them. The array keeps the last call's contents, and
 * every call overwrites all of what it reads before reading it. */
#define LBM_MASS_NOALLOC_MAX_NODES (1 << 21)
#define LBM_MASS_NOALLOC_SCRATCH_BYTES (((size_t)2 << 24) + 65536)
lbm_status lbm_mass_noalloc(const lbm_params* params, const void* state_dev, double* out_dev,
                            void* stream);

/* Current pre-collision populations in canonical FP64 layout,
 * f_dev and g_dev each [9][ny][nx] (device), exactly as stored (binary32 f,
 * Q2.29 g words, scaled binary16 halves converted without rounding), so
 * lbm_set_state of the result restores the state bit for bit.
 * Asynchronous. */
lbm_status lbm_get_state(lbm_ctx* ctx, double* f_dev, double* g_dev);

/* Replaces the current pre-collision populations (canonical FP64 layout);
 * each value is rounded once, to nearest, to its storage format (binary32,
 * Q2.29 or scaled binary16). Keeps the time counter. */
lbm_status lbm_set_state(lbm_ctx* ctx, const double* f_dev, const double* g_dev);

/* Size in bytes of one step record (see lbm_step_record). */
size_t lbm_record_bytes(const lbm_ctx* ctx);

/* Advances one step exactly like lbm_step(ctx, 1) and also writes the
 * record of the state it started from: the forward quantities of Sec. III
 * that the step computed on the way -- planes phi, mu, p, S = sum_i f_i,
 * jx, jy = sum_i c_i f_i, in the compute type (binary64 for LBM_FP64,
 * binary32 otherwise), each plane lbm_record_bytes / 6 bytes apart, node
 * y * nx + x at element y * nx + x. record_dev: caller-owned device memory
 * of lbm_record_bytes bytes, 256-byte aligned. The record is the input of
 * lbm_adjoint_step_record and is a third of a raw state in size.
 * Asynchronous. */
lbm_status lbm_step_record(lbm_ctx* ctx, void* record_dev);

/* Advances nsteps steps like lbm_step and writes the record of the state
 * each step starts from: step k's into records[k] (records: a host array of
 * nsteps device pointers, each as for lbm_step_record). With two steps per
 * pass (lbm_set_pass) a pair of steps is one launch that writes both records,
 * so a checkpoint replay follows the same kernels as lbm_step. LBM_EINVAL for
 * nsteps < 0, a null array, or a null or misaligned record. Asynchronous. */
lbm_status lbm_step_records(lbm_ctx* ctx, int64_t nsteps, void* const* records);

/* Raw snapshot of the internal state buffer in the storage precision
 * (lbm_state_bytes bytes): exact save/restore for checkpointing.
 * lbm_load_raw also sets the time counter to t. Asynchronous. */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_save_raw(lbm_ctx* ctx, void* dst_dev);
lbm_status lbm_load_raw(lbm_ctx* ctx, const void* src_dev, int64_t t);

/* Time counter (number of steps taken since lbm_init). */
int64_t lbm_time(const lbm_ctx* ctx);

/* Rebinds the context to another HIP stream. */
lbm_status lbm_set_stream(lbm_ctx* ctx, void* stream);

/* Launch shape of the one-step fused kernel: rows per workgroup segment
 * (0 = automatic: about 2.25 workgroups per resident slot, 16..32 rows).
 * Results do not depend on it. */
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t seg_rows);

/* Current one-step fused launch shape into out[4] (host): column strips (of
 * equal width, at most 250 columns), segments per strip, rows per segment,
 * threads per workgroup. lbm_step_record always uses this kernel. */
lbm_status lbm_launch_info(const lbm_ctx* ctx, int32_t out[4]);

/* Time steps per pass of the fused kernel in lbm_step (temporal blocking,
 * an implementation choice; the scheme is Sec. III's step applied twice).
 * steps = 2 (the default for LBM_FP64 and LBM_FP32; available for
 * LBM_FP16_STORE, whose default is 1)
 * advances the lattice by two steps per launch: the first step's
 * post-collision words stay in on-chip memory and feed the second step, so
 * the populations cross HBM once per two steps; an odd last step of an
 * lbm_step call runs alone. The intermediate state is kept in the storage
 * format (FP16 storage: in the FP32 format, binary32 f and Q2.29 g, so the
 * state is rounded to binary16 once per pass), so results agree with
 * steps = 1 (one launch per step) to rounding: the two kernels evaluate the
 * same expressions, but the compiler may fuse multiply-adds differently in
 * each. The exact integer invariant of the stored g holds in both. seg_rows: rows per workgroup
 * segment of the two-step kernel (0 = automatic: one round of workgroups).
 * LBM_EINVAL for steps other than 1 and 2, or seg_rows < 0. Applies to lbm_step only (not lbm_step_record, not
 * LBM_FLAG_UNFUSED). */
lbm_status lbm_set_pass(lbm_ctx* ctx, int32_t steps, int32_t seg_rows);

/* Shape of the kernel lbm_step launches for a pair of steps, into out[5]
 * (host): steps per pass, column strips (at most 242 columns for two steps),
 * segments per strip, rows per segment, threads per workgroup. */
lbm_status lbm_pass_info(const lbm_ctx* ctx, int32_t out[5]);

/* ---------------------------------------------------------------- adjoint
 * Reverse-mode derivative of a loss L(phi_K) of the final order parameter
 * with respect to sigma, M and the initial phi0 (not in the paper: a
 * hand-written transpose of every stage of the step above). The caller
 * drives checkpoint-and-recompute: it restores a checkpoint with
 * lbm_load_raw, replays the segment with lbm_step_record keeping one
 * record per step, and hands the records to lbm_adjoint_step_record in
 * decreasing t (or hands raw states s_t to lbm_adjoint_step, which
 * recomputes the record). Parameter cotangents accumulate in FP64.
 *
 * lbm_adjoint_workspace_bytes: device bytes for the adjoint (two adjoint
 *   population sets, forward/adjoint scratch fields, FP64 partials).
 * lbm_adjoint_begin: binds the adjoint workspace and seeds the cotangent of
 *   the state at the final time: gbar_i = dL/dphi_K (all i), fbar = 0;
 *   clears the sigma/M accumulators. dL_dphi_dev: FP64 [ny][nx].
 * lbm_adjoint_seed: the same seeding with the workspace already bound (for
 *   another loss or another run with the same workspace).
 * lbm_adjoint_step: given the raw forward state s_t (layout of
 *   lbm_save_raw, storage precision of the context) replaces the cotangent
 *   of s_{t+1} by that of s_t = (d s_{t+1} / d s_t)^T applied to it, and
 *   adds (d s_{t+1} / d sigma)^T and (d s_{t+1} / d M)^T to the
 *   accumulators. Asynchronous.
 * lbm_adjoint_step_record: the same step given the record of forward step
 *   t written by lbm_step_record (256-byte aligned); no forward
 *   recomputation. Asynchronous.
 * lbm_adjoint_init: pulls the cotangent of s_0 back through the initial
 *   state map phi0 -> (f = 0, g = H_i(phi0, mu0)) given the same phi0_dev
 *   (FP64 [ny][nx], device) that lbm_init received: writes dL/dphi0 (FP64
 *   [ny][nx], device) and out[2] = (dL/dsigma, dL/dM) totals (host).
 *   Synchronises the stream.
 * The adjoint arithmetic runs in the compute type (FP64 for LBM_FP64,
 * FP32 otherwise); the parameter sums are FP64 and run-to-run reproducible.
 * lbm_adjoint_seed, lbm_adjoint_step, lbm_adjoint_step_record and
 * lbm_adjoint_init return LBM_ESTATE before lbm_adjoint_begin.
 */
size_t lbm_adjoint_workspace_bytes(const lbm_params* params);
lbm_status lbm_adjoint_begin(lbm_ctx* ctx, void* adj_workspace_dev,
                             size_t adj_workspace_bytes,
                             const double* dL_dphi_dev);
lbm_status lbm_adjoint_seed(lbm_ctx* ctx, const double* dL_dphi_dev);
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* fwd_state_dev);
lbm_status lbm_adjoint_step_record(lbm_ctx* ctx, const void* record_dev);
lbm_status lbm_adjoint_init(lbm_ctx* ctx, const double* phi0_dev, double* dL_dphi0_dev,
                            double out[2]);

/* Direct access to the adjoint state, for callers with a general state
 * cotangent and for per-step checks. lbm_adjoint_set replaces the current
 * cotangent of the pre-collision state by (fbar, gbar) (canonical FP64
 * [9][ny][nx] each, device) and clears the parameter accumulators.
 * lbm_adjoint_get copies the current cotangent out (same layout) and writes
 * out[2] = (dL/dsigma, dL/dM) accumulated by the adjoint steps so far
 * (without the initial-state map); synchronises the stream. Both return
 * LBM_ESTATE before lbm_adjoint_begin. */
lbm_status lbm_adjoint_set(lbm_ctx* ctx, const double* fbar_dev, const double* gbar_dev);
lbm_status lbm_adjoint_get(lbm_ctx* ctx, double* fbar_dev, double* gbar_dev, double out[2]);

/* Frees the host context (never the caller's device memory). NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* Static description of a status code. */
const char* lbm_strerror(lbm_status status);

/* Version of this interface: the layouts of lbm_params and lbm3_params
 * (read through the caller's pointer at the size the headers declare) and
 * every signature in qilbm.h and qilbm3d.h. It changes whenever one of them
 * does; a caller built against another value must not use the library (the
 * structs would be read past their end). lbm_abi_version returns the value
 * the library was built with. Host only: needs no GPU, enqueues nothing,
 * may be called before any other function. */
#define QILBM_ABI_VERSION 2
int32_t lbm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QILBM_H */
