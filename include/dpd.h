/*
 * dpd.h - C ABI of the MI355X (gfx950) DPD step library.
 *
 * One call of dpd_step advances a periodic box of soft beads by Groot-style
 * dissipative particle dynamics as defined by Doi et al., "A portable code for
 * dissipative particle dynamics (DPD) simulations with additional specific
 * interactions" (arXiv 1804.06205):
 *   - the total force of Eq. (3): conservative F^C (Eq. 4), dissipative F^D and
 *     random F^R (the Groot-Warren forms the text after Eq. 5 refers to), and
 *     the bonded F^S of Eq. (8): harmonic springs (Eq. 6) and Morse terms
 *     (Eq. 7 and the standard form);
 *   - pairs taken straight from cells of edge rc = 1 rebuilt every step, with
 *     no stored neighbour list (design section of the paper);
 *   - Groot's modified velocity Verlet (Fig. 1):
 *       x <- x + dt v + dt^2 f / 2, wrap;  vt <- v + lambda dt f;
 *       f' <- F(x, vt; s);  v <- v + dt (f + f') / 2;  f <- f'.
 *
 * Units: masses 1, cutoff rc = 1.  Particles are named by their tag, the
 * index 0..n-1 of the arrays passed to dpd_create; every state array crossing
 * this ABI is in tag order, row-major (n, 3).
 *
 * The random force of pair (i, j) at force evaluation s (0 for the initial
 * force, k for the force at the end of step k) uses theta = sqrt(-2 ln u1)
 * cos(2 pi u2) from Philox4x32-10 with key = seed and counter
 * (min(tag_i, tag_j), max(tag_i, tag_j), s mod 2^32, 0), u1 = ((w0 >> 8) + 1)
 * 2^-24 and u2 = (w1 >> 8) 2^-24, so theta_ij = theta_ji and a run is
 * reproducible bit for bit.
 *
 * Memory: the library copies every host array at the call and never keeps a
 * caller pointer.  It owns all device memory it allocates and releases it in
 * dpd_destroy, where a system's device block (and a stream the library
 * created) is kept for reuse by later systems rather than returned to HIP:
 * hipFree waits for every stream of the device, so freeing while other
 * systems run would stall them.  At most 4 GiB of such blocks per device are
 * kept, and all of them are returned to HIP before an allocation fails.  Work
 * is enqueued on one HIP stream per system (the caller's, or one the library
 * creates); dpd_step returns after enqueueing.
 *
 * Errors: every int-returning call returns DPD_OK (0) or a negative code and
 * leaves a message for dpd_last_error() (per thread).  Device-side failures
 * (a cell or tile capacity exceeded, a non-finite value, a displacement over
 * half a box) are sticky: they surface at the next synchronising call
 * (dpd_sync, dpd_observables, dpd_get_state, dpd_get_cells) and every later
 * call on that system fails with the same code.
 *
 * Threading: one system must not be used from two threads at once; separate
 * systems are independent.
 */
#ifndef DPD_H
#define DPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DPD_ABI_VERSION 1

typedef struct dpd_system dpd_system;

enum dpd_status {
    DPD_OK = 0,
    DPD_EINVAL = -1,     /* bad argument: n < 2, non-finite input, gamma or sigma < 0,
                            dt <= 0, lambda outside [0, 1], bad type or precision     */
    DPD_ENOMEM = -2,     /* device or host allocation failed                          */
    DPD_EDEVICE = -3,    /* HIP runtime error, or no gfx950 device                     */
    DPD_ENUMERIC = -4,   /* non-finite state, or a displacement over half a box        */
    DPD_EBOX = -5,       /* some box edge below 3 cells (L < 3 rc)                     */
    DPD_ERANGE = -6,     /* bond tag out of range or i == j, or bond length >= L/2     */
    DPD_ESTATE = -7,     /* parameters or bonds changed after the first step, or a call
                            before dpd_set_params                                      */
    DPD_EBUSY = -8,      /* batch full or over its memory budget, or the system is
                            resident in a batch                                        */
    DPD_ECAPACITY = -9   /* a cell held more particles than its slots (local density far
                            above the box average); recreate with a larger cell_capacity */
};

enum dpd_precision {
    DPD_PREC_FP64 = 0,   /* FP64 throughout                                            */
    DPD_PREC_MIXED = 1   /* FP32 forces and velocities, FP64 positions                  */
};

enum dpd_bond_type {
    DPD_BOND_HARMONIC = 1,    /* Eq. (6): F_i = -C (r - r_e) e, U = C (r - r_e)^2 / 2  */
    DPD_BOND_MORSE_PAPER = 2, /* Eq. (7) with the alpha of Fig. 3a: E = exp(-alpha |r - r_e|),
                                 F_i = -2 alpha K E (1 - E) e (attractive on both sides of
                                 r_e), U = K (1 - E)^2 as Fig. 3a accumulates it          */
    DPD_BOND_MORSE = 3        /* standard Morse: E = exp(-alpha (r - r_e)),
                                 U = D [(1 - E)^2 - 1], F_i = -2 alpha D E (1 - E) e      */
};

/* Observables of the current state (FP64 sums; pressure per the virial of the
 * conservative and bonded forces, p = (2 KE + W) / (3 V)). */
typedef struct dpd_obs {
    int64_t step;        /* steps taken since the state's step counter was 0   */
    double time;         /* step * dt                                          */
    double ke;           /* sum |v|^2 / 2                                      */
    double kT;           /* 2 KE / (3N - 3)                                    */
    double u_pair;       /* sum over pairs r < 1 of a (1 - r)^2 / 2            */
    double u_bond;       /* bonded energy (Fig. 3a accumulates it as Ebond)    */
    double w_pair;       /* sum over pairs of d . F^C                          */
    double w_bond;       /* sum over bonds of d . F^S                          */
    double pressure;
    double momentum[3];  /* sum v                                              */
    int64_t npairs;      /* unordered pairs with r^2 < 1 (in the force precision) */
} dpd_obs;

/* Per-kernel timing of dpd_step_profiled, in milliseconds summed over launches. */
typedef struct dpd_kernel_times {
    double ms_begin;     /* integrate-1 + binning from the resting state       */
    double ms_fused;     /* pair + bond force, integrate-2, integrate-1, binning */
    double ms_finish;    /* pair + bond force, integrate-2                      */
    int64_t n_begin, n_fused, n_finish;  /* launch counts                       */
} dpd_kernel_times;

/* Library ABI version (DPD_ABI_VERSION). */
int dpd_version(void);

/* Message of the last failed call on this thread ("" if none).  Owned by the
 * library; valid until the next call on this thread. */
const char *dpd_last_error(void);

/*
 * Creates a system of n particles in a periodic box of edges L[0..2] (each
 * >= 3; cells per axis = floor(L), edge L / floor(L)).
 *   pos, vel   host arrays of n*3 doubles (tag order); positions are wrapped
 *              into [0, L) on entry.
 *   type       host array of n bytes, each < ntypes, or NULL (all 0).
 *   ntypes     1..16.
 *   seed       key of the pair noise stream.
 *   precision  DPD_PREC_FP64 or DPD_PREC_MIXED.
 *   hip_stream a hipStream_t to enqueue on, or NULL for a library-owned one.
 *   cell_capacity  slots per cell, or 0 for the default (32).
 * On success *out owns the system; the step counter is 0 and the force is
 * computed at the first step as F(x, v; s = 0).
 */
int dpd_create(dpd_system **out, const double L[3], int64_t n, const double *pos,
               const double *vel, const uint8_t *type, int ntypes, uint64_t seed,
               int precision, void *hip_stream, int cell_capacity);

/*
 * Sets the pair table and integrator parameters.  a_ij: ntypes*ntypes doubles,
 * row-major, must be symmetric (Eq. 4; Eq. 5 maps chi to a_ij on the caller's
 * side).  gamma, sigma >= 0 (sigma^2 = 2 gamma kT is not enforced); kT is only
 * reported back; dt > 0; lambda in [0, 1] (0.65 in the paper).  Allowed until
 * the first step.
 */
int dpd_set_params(dpd_system *sys, const double *a_ij, double gamma, double sigma, double kT,
                   double dt, double lambda);

/*
 * Adds nb bond records (Eq. 8; Fig. 3b's record [type, i, j, r_e, const,
 * const2]): btype[b] in dpd_bond_type, tags i[b] != j[b] in [0, n), r_e, k (C,
 * K_M or D) and alpha (ignored for harmonic).  Several records may sit on one
 * pair; they all add.  Bonds have no cutoff and use the minimum image.  May be
 * called several times before the first step.
 */
int dpd_add_bonds(dpd_system *sys, int64_t nb, const int32_t *btype, const int64_t *i,
                  const int64_t *j, const double *r_e, const double *k, const double *alpha);

/* Enqueues nsteps >= 0 steps on the system's stream and returns.  Any call,
 * nsteps = 0 included, freezes the parameters and bonds and enqueues the
 * initial force if it is not yet computed.  The step counter is limited to
 * 2^32 - 1 (it keys the noise as a 32-bit word): DPD_EINVAL if step + nsteps
 * would pass it. */
int dpd_step(dpd_system *sys, int64_t nsteps);

/* Like dpd_step, but synchronises and reports per-kernel device time. */
int dpd_step_profiled(dpd_system *sys, int64_t nsteps, dpd_kernel_times *out);

/* Waits for the system's stream; returns any sticky device error. */
int dpd_sync(dpd_system *sys);

/* Computes the observables of the current state (synchronises). */
int dpd_observables(dpd_system *sys, dpd_obs *out);

/* Copies the current state to host arrays of n*3 doubles in tag order (any
 * pointer may be NULL) and the step counter (may be NULL).  Synchronises. */
int dpd_get_state(dpd_system *sys, double *pos, double *vel, double *force, int64_t *step);

/* Replaces the state (pos and vel required; force NULL = recompute it as
 * F(x, v; s = step) at the next step) and the step counter (0 .. 2^32 - 1,
 * else DPD_EINVAL). */
int dpd_set_state(dpd_system *sys, const double *pos, const double *vel, const double *force,
                  int64_t step);

/* The current cell list: cell_of_tag[n] = linear cell (cz ny + cy) nx + cx of
 * each particle, count[ncells] = particles per cell.  Synchronises. */
int dpd_get_cells(dpd_system *sys, int64_t *cell_of_tag, int64_t *count);

/* Sizes of the system: out[0] = n, out[1] = ncells, out[2] = cell capacity,
 * out[3] = device bytes held, out[4..6] = cells per axis, out[7] = precision. */
int dpd_info(dpd_system *sys, int64_t out[8]);

/*
 * Autotuner.  The pair kernel runs on bricks of BX x BY x BZ cells with a
 * fixed work-group size and LDS tile; every variant computes bitwise the same
 * forces, so the choice only changes speed.
 *   dpd_variant_count()         number of variants.
 *   dpd_variant_shape(v, out)   out[0..4] = {BX, BY, BZ, threads, LDS capacity}.
 *   dpd_set_variant(sys, v)     use variant v (-1 = the library's default).
 *   dpd_autotune(sys, trials, &best, &ms)  times `trials` launches of every
 *       variant's fused step kernel on the current state, keeps the fastest and
 *       returns it with its mean time in ms.  The state is left unchanged
 *       (the trials write only the scratch layout of the next state).
 *       Synchronises.  Variants whose tile cannot hold the densest brick are
 *       skipped.  With the environment variable DPD_TUNE_CACHE naming a file,
 *       the choice is stored there per class of system (device architecture,
 *       precision, particle types, power-of-two class of the cell count,
 *       particles per cell, cubic or not, variant table), and a later call for
 *       a system of the same class, in any process, takes the stored variant
 *       and time without timing anything.
 * The variants differ in brick shape and in threads per brick: variants 5 and
 * 6 give each thread about two particles of the brick.
 */
int dpd_variant_count(void);
int dpd_variant_shape(int variant, int out[5]);
int dpd_set_variant(dpd_system *sys, int variant);
int dpd_autotune(dpd_system *sys, int trials, int *best_variant, double *best_ms);

/*
 * The pair noise theta_ij(s) of the random force (see the top of this file)
 * as the step kernels compute it, for m host triples (tag_i[k], tag_j[k],
 * s[k]) on the current device; precision selects the FP32 or FP64 Box-Muller.
 * Writes m doubles to theta (host).  For checking and for reproducing the
 * noise stream outside the library.  Synchronous.
 */
int dpd_pair_noise(uint64_t seed, int64_t m, const uint32_t *tag_i, const uint32_t *tag_j,
                   const uint32_t *s, int precision, double *theta);

/*
 * dpd_pair_noise for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernel and results (bit for bit), with the triples and results
 * staged in a fixed library-owned device array instead of memory allocated
 * per call.  No hipMalloc, hipFree or other allocating call.
 *   m          0 .. 262144 (2^18) triples, else DPD_EINVAL; other arguments and
 *              errors as dpd_pair_noise.  Synchronous.
 * The array (5 MiB per device: 2^18 x (3 u32 + 1 double)) is held by every
 * device the library runs on until the process ends and is shared by all
 * calls on that device: calls that overlap on one device (from several
 * threads) race, and must be serialised by the caller.
 */
int dpd_pair_noise_noalloc(uint64_t seed, int64_t m, const uint32_t *tag_i,
                           const uint32_t *tag_j, const uint32_t *s, int precision,
                           double *theta);

/* Frees the system once its stream is idle; its device memory is kept for
 * later systems (see Memory above).  NULL is ignored.  A system still resident
 * in a batch is retired from it first. */
void dpd_destroy(dpd_system *sys);

/* Device bytes that dpd_create (plus dpd_add_bonds with nbonds records) will
 * allocate for such a system; equals out[3] of dpd_info after the first step.
 * For admission decisions before a system is created. */
int dpd_footprint_bytes(const double L[3], int64_t n, int64_t nbonds, int precision,
                        int cell_capacity, int64_t *bytes);

/*
 * Replica batches.  A batch advances many independent resident systems
 * (replicas: each its own box, parameters, seed and bonds) together: every
 * pass of a step is one launch over the work items of all replicas, and a
 * window of K steps is one captured HIP graph, replayed while the set of
 * replicas stays the same.  Each replica follows exactly the trajectory
 * dpd_step would give it alone (bit for bit).  Batches hold mixed-precision
 * systems with cubic cells.
 *
 *   dpd_batch_create(out, budget_bytes, max_replicas, hip_stream, variant)
 *       budget_bytes  cap on the summed device bytes (dpd_info out[3]) of the
 *                     resident systems; max_replicas  number of slots (1..65536);
 *       hip_stream    stream for the batch's work (NULL = library-owned);
 *       variant       brick variant of the batched pair pass (-1 = 5x4x4).
 *   dpd_batch_admit(b, sys, nsteps, &slot)
 *       makes sys resident with a target of nsteps more steps.  Computes the
 *       initial force if needed and waits for the system's stream and the
 *       batch.  DPD_EBUSY if the budget or the slots would be exceeded.  While
 *       resident, every call on sys except dpd_info and dpd_destroy fails
 *       with DPD_EBUSY.
 *   dpd_batch_advance(b, K)
 *       enqueues one window: every resident replica advances min(K, steps
 *       left) steps.  Asynchronous.
 *   dpd_batch_poll(b, done, max_done, &ndone)
 *       waits for the enqueued windows, then lists (once each) the slots whose
 *       replica has reached its target or hit a device error (the error then
 *       surfaces on the system after retirement).
 *   dpd_batch_retire(b, slot)
 *       waits for the batch and hands the system back (usable as before, its
 *       step counter advanced); the slot and its bytes are freed.
 *   dpd_batch_autotune(b, K, &best_variant, &ms_per_step)
 *       runs one window of K steps with each brick variant (real steps: every
 *       variant gives the same trajectory), times each on the device and keeps
 *       the fastest; returns it and its time per step.  Best called once the
 *       batch holds a representative set of replicas.  Synchronises.
 *   dpd_batch_info(b, out[6])
 *       resident replicas, bytes used, budget, graph captures, windows, variant.
 *   dpd_batch_destroy(b)
 *       retires every resident replica and frees the batch.
 * Calls on one batch must not overlap (not thread-safe).
 */
typedef struct dpd_batch dpd_batch;

int dpd_batch_create(dpd_batch **out, int64_t budget_bytes, int max_replicas, void *hip_stream,
                     int variant);
int dpd_batch_admit(dpd_batch *b, dpd_system *sys, int64_t nsteps, int *slot);
int dpd_batch_advance(dpd_batch *b, int64_t K);
int dpd_batch_autotune(dpd_batch *b, int64_t K, int *best_variant, double *ms_per_step);
int dpd_batch_poll(dpd_batch *b, int *done, int max_done, int *ndone);
int dpd_batch_retire(dpd_batch *b, int slot);
int dpd_batch_info(dpd_batch *b, int64_t out[6]);
void dpd_batch_destroy(dpd_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* DPD_H */
