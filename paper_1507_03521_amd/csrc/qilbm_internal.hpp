// Host-side declarations shared by the C-ABI layer and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "qilbm_device.hpp"

namespace qilbm {

// Stride (elements) between the planes of every per-node array: N rounded
// up to 256, plus a stagger of 2304 elements so that the planes a row
// touches at one column do not all start at the same offset modulo a large
// power of two (a power-of-two lattice would otherwise send all 18 plane
// streams to the same memory channels; the stagger is worth ~3 % at
// 2048 x 8192 on MI355X). The one definition used by every layout.
inline int64_t plane_stride(int64_t N) { return (N + 255) / 256 * 256 + 2304; }

// FP64 outputs of the moments kernel; NULL members are skipped.
struct MomentOut {
  double* phi = nullptr;
  double* rho = nullptr;
  double* ux = nullptr;
  double* uy = nullptr;
  double* p = nullptr;
  double* mu = nullptr;
};

// Launch shape of the fused step kernel.
struct FusedShape {
  int nstrips = 0, width = 0, nseg = 0, seg_rows = 0, threads = 0;
};

// Launch shape for seg_rows rows per segment (0: automatic, from the number
// of workgroups that can be resident at once, ``resident``).
template <int P>
FusedShape fused_shape(const Geom& g, int seg_rows, int resident);

// Workgroups of the fused kernel that the current device holds at once.
template <int P>
int fused_resident();

// True when a group of population planes spans more than 4 GiB - 1 bytes:
// the fused kernel then addresses every plane with its own descriptor.
template <int P>
bool fused_big(const Geom& g);

// Zeroes bytes (a multiple of 16, 16-byte aligned) of device memory with a
// kernel (no memset node, so the call may sit in a captured graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

template <int P>
hipError_t launch_init(const double* phi0, void* pop, const Coef<double>& c, const Geom& g,
                       hipStream_t s);
template <int P>
hipError_t launch_from_canonical(const double* f, const double* gg, void* pop, const Geom& g,
                                 hipStream_t s);
template <int P>
hipError_t launch_to_canonical(const void* pop, double* f, double* gg, const Geom& g,
                               hipStream_t s);
template <int P>
hipError_t launch_fields(const void* pop, void* phi, void* mu,
                         const Coef<typename PrecT<P>::T>& c, const Geom& g, hipStream_t s);
// Pressure into p and, when sj is not null, S = sum f, jx, jy into the three
// planes sj, sj + Ns, sj + 2 Ns (compute type); FP64 moments into mo.
template <int P>
hipError_t launch_macro(const void* pop, const void* phi, const void* mu, void* p, void* sj,
                        const MomentOut& mo, const Coef<typename PrecT<P>::T>& c, const Geom& g,
                        hipStream_t s);
template <int P>
hipError_t launch_step_unfused(const void* pin, void* pout, void* phi, void* mu, void* p,
                               void* sj, const Coef<typename PrecT<P>::T>& c, const Geom& g,
                               hipStream_t s, bool trt = false);
// One fused step; when rec is not null it also writes the forward quantities
// of the state it reads (the record: planes phi, mu, p, S, jx, jy of the
// compute type at stride Ns).
// trt selects the two-relaxation-time collision of f (no recording variant:
// rec must then be null).
template <int P>
hipError_t launch_step_fused(const void* pin, void* pout, const Coef<typename PrecT<P>::T>& c,
                             const Geom& g, const FusedShape& sh, void* rec, hipStream_t s,
                             bool trt = false);
// Two steps per launch: the state between the two steps stays on chip.
// With rec0 and rec1 not null it also writes the records of the state it
// reads (rec0) and of the state after the first step (rec1). Its shape, for
// seg_rows rows per segment (0: one round of workgroups).
template <int P>
FusedShape fused2_shape(const Geom& g, int seg_rows, int resident);
template <int P>
int fused2_resident();
template <int P>
hipError_t launch_step2_fused(const void* pin, void* pout, const Coef<typename PrecT<P>::T>& c,
                              const Geom& g, const FusedShape& sh, void* rec0, void* rec1,
                              hipStream_t s, bool trt = false);
template <int P>
hipError_t launch_mass(const void* pop, void* phi, void* mu, double* part, int nred, double* out,
                       const Coef<typename PrecT<P>::T>& c, const Coef<double>& c64,
                       const Geom& g, hipStream_t s);
hipError_t launch_sum_partials(const double* part, int nb, int width, double* out, hipStream_t s);

}  // namespace qilbm
