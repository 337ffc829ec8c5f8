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

// ---------------------------------------------------------------------------
// Replica batches (mixed precision, cubic cells).  Every resident replica is a
// whole system with its own box, parameters, seed and bonds; one launch of a
// batched kernel covers the work items of all of them.
// ---------------------------------------------------------------------------
struct BatchEnt {
    DevSys<float> D;
    int nbx, nby, nbz;  // bricks per axis (each at most the batch's brick extent)
    uint64_t thr;       // cutoff r^2 < 1 in squared brick-frame units
};

// A work item: (slot, brick) for the force pass, (slot, block of 256 cells)
// for begin.
struct BatchWork {
    uint32_t slot, item;
};

// Device view of a batch.  Per slot: t0 = resting state at the start of the
// current window, target = state at which the replica stops (t0 <= target;
// t0 == target for an idle or empty slot), status = {t0, error bits} after the
// window.  nwork = {force items, begin items, slots}.
struct BatchDev {
    const BatchEnt *tab;
    uint32_t *t0;
    const uint32_t *target;
    const BatchWork *wf, *wb;
    const int *nwork;
    uint32_t *status;
};

// Enqueues one window of K steps: begin for every replica that still has
// steps, K force passes (a replica's last step of the window, or its target
// step, ends in place), then the per-slot counter update.  Launch grids are
// the given capacities; surplus work-groups exit at once, so a captured window
// stays valid while the tables shrink or change within those capacities.
hipError_t launch_batch_window(const BatchDev &B, int variant, int K, int cap_force,
                               int cap_begin, int cap_slots, hipStream_t st);
hipError_t launch_noise(int precision_fp64, uint64_t seed, int64_t m, const uint32_t *ti,
                        const uint32_t *tj, const uint32_t *s, double *out, hipStream_t st);
hipError_t launch_u32_to_f64(const uint32_t *a, double *b, int64_t m, hipStream_t st);
hipError_t launch_reduce8(const double *const *in, int64_t m, int64_t chunk, int nblocks,
                          double *out, hipStream_t st);

}  // namespace dpd
