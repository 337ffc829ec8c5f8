// Host-side launchers of the DPD kernels (dpd_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dpd_device.hpp"

namespace dpd {

// Modes of the force pass: INIT stores f = F(x, vt; s = q) in place; FINISH
// adds integrate-2 in place; FUSED adds integrate-2 then integrate-1 and
// binning into state q+1; OBS writes per-tag observables only.
enum ForceMode : int { FORCE_INIT = 0, FORCE_FINISH = 1, FORCE_FUSED = 2, FORCE_OBS = 3 };

template <typename T>
hipError_t launch_force(const DevSys<T> &D, uint32_t q, int mode, int variant, hipStream_t st);
int force_variant_count();
// {BX, BY, BZ, threads per block, LDS neighbour capacity} of a variant.
void force_variant_shape(int variant, int out[5]);

template <typename T> hipError_t launch_begin(const DevSys<T> &D, uint32_t q, hipStream_t st);
template <typename T>
hipError_t launch_load(const DevSys<T> &D, uint32_t q, const double *x, const double *v,
                       const double *f, const uint8_t *type, hipStream_t st);
template <typename T>
hipError_t launch_gather(const DevSys<T> &D, uint32_t q, double *x, double *v, double *f,
                         int64_t *cell, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, int64_t m, uint32_t v, hipStream_t st);
hipError_t launch_noise(int precision_fp64, uint64_t seed, int64_t m, const uint32_t *ti,
                        const uint32_t *tj, const uint32_t *s, double *out, hipStream_t st);
hipError_t launch_u32_to_f64(const uint32_t *a, double *b, int64_t m, hipStream_t st);
hipError_t launch_reduce8(const double *const *in, int64_t m, int64_t chunk, int nblocks,
                          double *out, hipStream_t st);

}  // namespace dpd
