// Device-side building blocks of the DPD step for gfx950: records, the pair
// noise, binning and the pair / bond force terms.
//
// Method: Groot-style DPD as defined by Doi et al. (arXiv 1804.06205):
// Eq. (3) total force, Eq. (4) conservative repulsion, the Groot-Warren
// dissipative and random forces named after Eq. (5), bonds of Eqs. (6)-(8)
// and Fig. 3a, and the modified velocity Verlet of Fig. 1.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpd {

// ---------------------------------------------------------------------------
// Records kept per cell slot.  A cell owns `cap` consecutive slots; the first
// count[cell] of them are occupied, in arbitrary order (binning appends with
// atomics); kernels restore ascending tag order where summation order matters.
// ---------------------------------------------------------------------------

// Position of a particle inside its cell, as kept in pair records.
//  FP32 forces: a fixed-point offset, (x - c h) / h in units of 2^-29.  The
//    difference of two such offsets (plus a whole-cell shift) is an exact
//    integer, so a close pair's separation is rounded once, relative to its
//    own size, when it becomes a float; plain FP32 offsets would carry an
//    absolute error of ~6e-8 that near-coincident pairs turn into large force
//    errors.  The same integer difference read from either particle is
//    exactly negated, so F_ij = -F_ji holds bit for bit.
//  FP64: the offset x - c h itself.
template <typename T> struct Geo;
template <> struct Geo<float> {
    using P = int32_t;
    static constexpr double SCALE = 536870912.0;   // 2^29
    static constexpr int32_t ONE = 1 << 29;
    __device__ static __forceinline__ P encode(double x, int c, double h) {
        return (int32_t)rint((x - (double)c * h) / h * SCALE);
    }
    // encode(x, c, 1.0), without the divide.
    __device__ static __forceinline__ P encode_unit(double x, int c) {
        return (int32_t)rint((x - (double)c) * SCALE);
    }
    // Separation along one axis: a - b - s cells, in length units (hs = h / 2^29).
    __device__ static __forceinline__ float delta(P a, P b, int s, float hs) {
        return (float)(a - b - s * ONE) * hs;
    }
    __host__ __device__ static float hscale(double h) { return (float)(h / SCALE); }
};
template <> struct Geo<double> {
    using P = double;
    __device__ static __forceinline__ P encode(double x, int c, double h) {
        return x - (double)c * h;
    }
    __device__ static __forceinline__ P encode_unit(double x, int c) { return x - (double)c; }
    __device__ static __forceinline__ double delta(P a, P b, int s, double h) {
        return (a - b) - (double)s * h;
    }
    __host__ __device__ static double hscale(double h) { return h; }
};

// Pair record: what a neighbour needs (position inside its cell, predicted
// velocity vt, tag, type).
template <typename T> struct PRec;
template <> struct alignas(16) PRec<float> {
    int32_t ox, oy, oz;
    uint32_t tag;
    float vx, vy, vz;
    uint32_t type;
};
template <> struct alignas(16) PRec<double> {
    double ox, oy, oz;
    double vx, vy, vz;
    uint32_t tag, type;
    uint64_t pad;
};

// State record: FP64 position, velocity and force of the particle itself.
template <typename T> struct SRec;
template <> struct alignas(16) SRec<float> {
    double x, y, z;
    float vx, vy, vz;
    float fx, fy, fz;
};
template <> struct alignas(16) SRec<double> {
    double x, y, z;
    double vx, vy, vz;
    double fx, fy, fz;
    double pad;
};

// One end of a bond record, stored with the particle that owns it.  Bond
// terms are evaluated in FP64 in every precision mode.
template <typename T> struct BondEnt {
    uint32_t partner;   // tag of the other end
    int32_t type;       // 1 harmonic, 2 paper Morse, 3 standard Morse
    double r_e, k, alpha;
};

// Sticky device error bits.
enum : uint32_t {
    ERR_CELL_OVERFLOW = 1u,    // a cell got more than `cap` particles
    ERR_TILE_OVERFLOW = 2u,    // a brick's neighbourhood exceeded the tile buffer
    ERR_NONFINITE = 4u,        // non-finite position, velocity or force
    ERR_DISPLACEMENT = 8u,     // a step moved a particle by more than half a box
    ERR_INDEX = 16u            // an index outside its array (internal consistency)
};

// Everything a kernel needs about one system.  Passed by value.
template <typename T> struct DevSys {
    double L[3];        // box edges
    double h[3];        // cell edges, L / nc
    int nc[3];          // cells per axis
    int cap;            // slots per cell
    int64_t ncells;
    int64_t n;
    int ntypes;
    T dt, lambda, gamma, sigma_rdt;   // sigma_rdt = sigma / sqrt(dt)
    double dt_d, half_dt2_d;          // FP64 copies for the position update
    uint64_t seed;
    const T *a;                       // ntypes x ntypes repulsion table
    PRec<T> *P[2];                    // layouts, indexed by state parity
    SRec<T> *S[2];
    uint32_t *slot_of_tag[2];
    uint32_t *count[3];               // cell counts, indexed by state mod 3
    const uint32_t *bond_off;         // CSR over tags (n + 1) or null
    const BondEnt<T> *bonds;
    uint32_t *err;
    // Per-tag observables scratch (written by the observables pass).
    double *obs_u, *obs_w, *obs_ub, *obs_wb, *obs_ke, *obs_p;
    uint32_t *obs_np;
};

// Precision-generic math wrappers (float calls the f-suffixed functions).
__device__ __forceinline__ float t_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double t_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float t_exp(float x) { return expf(x); }
__device__ __forceinline__ double t_exp(double x) { return exp(x); }
__device__ __forceinline__ float t_abs(float x) { return fabsf(x); }
// 1 / sqrt(a) for a > 0 in FP64: the hardware estimate refined by two Newton
// steps, y <- y + y (1 - a y^2) / 2 (each doubles the correct bits; the
// result is within an ulp or two, without a square root and a divide).
__device__ __forceinline__ double rsqrt_nr(double a) {
    double y = __builtin_amdgcn_rsq(a);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double e = fma(-a * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}

// Reciprocal square root of a positive argument: the hardware v_rsq_f32
// (relative error below 1e-7, measured) for FP32; rsqrt_nr for FP64.
__device__ __forceinline__ float t_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double t_rsqrt(double x) { return rsqrt_nr(x); }
__device__ __forceinline__ float t_fma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double t_fma(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ double t_abs(double x) { return fabs(x); }

// ---------------------------------------------------------------------------
// Pair noise: Philox4x32-10 keyed by the seed, counter (min tag, max tag, s,
// 0), then Box-Muller on the first two words.
// ---------------------------------------------------------------------------

// 32x32 -> 64 product split into (hi, lo).
__device__ __forceinline__ void mulhilo(uint32_t a, uint32_t b, uint32_t &hi, uint32_t &lo) {
    const uint64_t p = (uint64_t)a * (uint64_t)b;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

// a ^ b ^ k in one VALU instruction: gfx950's three-input bitwise op with
// the XOR truth table 0x96 (the key k is wave-uniform, so it sits in a scalar
// register).  The compiler emits two XORs otherwise.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t k) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// Returns the first two output words of Philox4x32 with ten rounds.
__device__ __forceinline__ void philox_w01(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                           uint32_t k0, uint32_t k1, uint32_t &w0,
                                           uint32_t &w1) {
    constexpr uint32_t MA = 0xD2511F53u, MB = 0xCD9E8D57u;
    constexpr uint32_t WA = 0x9E3779B9u, WB = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint32_t hA, lA, hB, lB;
        mulhilo(MA, c0, hA, lA);
        mulhilo(MB, c2, hB, lB);
        const uint32_t n0 = xor3(hB, c1, k0);
        const uint32_t n2 = xor3(hA, c3, k1);
        c0 = n0;
        c1 = lB;
        c2 = n2;
        c3 = lA;
        k0 += WA;
        k1 += WB;
    }
    w0 = c0;
    w1 = c1;
}

template <typename T> __device__ __forceinline__ T box_muller(uint32_t w0, uint32_t w1);

// FP32: the hardware log2, square root and cosine (v_cos_f32 takes its
// argument in revolutions, so cos(2 pi u2) is one instruction).  Measured
// against FP64 over 4M draws the result is as accurate as the libm-style
// sequence (max error 7e-7 on |theta| <= 5.8, i.e. the FP32 rounding of theta).
template <> __device__ __forceinline__ float box_muller<float>(uint32_t w0, uint32_t w1) {
    const float u1 = (float)((w0 >> 8) + 1u) * 0x1.0p-24f;   // (0, 1]
    const float u2 = (float)(w1 >> 8) * 0x1.0p-24f;          // [0, 1)
    const float m2ln2 = -1.3862943611198906f;                // -2 ln 2
    return __builtin_amdgcn_sqrtf(m2ln2 * __builtin_amdgcn_logf(u1)) * __builtin_amdgcn_cosf(u2);
}

template <> __device__ __forceinline__ double box_muller<double>(uint32_t w0, uint32_t w1) {
    const double u1 = (double)((w0 >> 8) + 1u) * 0x1.0p-24;
    const double u2 = (double)(w1 >> 8) * 0x1.0p-24;
    return sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

template <typename T>
__device__ __forceinline__ T pair_theta(uint64_t seed, uint32_t ti, uint32_t tj, uint32_t s) {
    const uint32_t lo = min(ti, tj), hi = max(ti, tj);
    uint32_t w0, w1;
    philox_w01(lo, hi, s, 0u, (uint32_t)seed, (uint32_t)(seed >> 32), w0, w1);
    return box_muller<T>(w0, w1);
}

// ---------------------------------------------------------------------------
// Geometry.
// ---------------------------------------------------------------------------

// Periodic wrap of one coordinate: one shift, and a value that rounds onto L
// after the upward shift becomes 0.
__device__ __forceinline__ double wrap_coord(double x, double L) {
    if (x < 0.0) x += L;
    else if (x >= L) x -= L;
    if (x >= L) x = 0.0;
    return x;
}

// Cell coordinate floor(x / h) with an IEEE FP64 divide, clamped to [0, n-1].
__device__ __forceinline__ int cell_coord(double x, double h, int n) {
    int c = (int)floor(__ddiv_rn(x, h));
    c = c > n - 1 ? n - 1 : c;
    c = c < 0 ? 0 : c;
    return c;
}

// cell_coord(x, 1.0, n), without the divide.
__device__ __forceinline__ int cell_coord_unit(double x, int n) {
    int c = (int)floor(x);
    c = c > n - 1 ? n - 1 : c;
    c = c < 0 ? 0 : c;
    return c;
}

// Which of the three rotating count arrays belongs to state q + k (k = 0, 1,
// 2): (q + k) mod 3, taken without the 32-bit wrap of q + k (2^32 is not a
// multiple of 3).
__host__ __device__ __forceinline__ uint32_t count_index(uint32_t q, uint32_t k) {
    return (q % 3u + k) % 3u;
}

__device__ __forceinline__ int64_t cell_linear(int cx, int cy, int cz, const int nc[3]) {
    return ((int64_t)cz * nc[1] + cy) * nc[0] + cx;
}

__device__ __forceinline__ double min_image(double d, double L) {
    return d - L * rint(d / L);
}

// ---------------------------------------------------------------------------
// Bond term (Eqs. 6-8, Fig. 3a), in FP64.  d = x_i - x_j (minimum image),
// r2 = |d|^2.  Returns the coefficient c with F_i = c d; energy and virial
// through u, w.  Type 1 harmonic, C (r - r_e)^2 / 2 (r_e = 0: a spring of
// rest length zero, F = -C d); type 2 the paper's modified Morse,
// K (1 - e^{-alpha |r - r_e|})^2; type 3 the standard Morse, K ((1 -
// e^{-alpha (r - r_e)})^2 - 1).  A bond at r = 0 exerts no force except the
// zero-length spring.  One reciprocal square root serves every type and the
// two Morse forms share one exponential, so a wave whose lanes hold
// different types runs one short path and one exponential.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double bond_coef(int type, double r2, double r_e, double k,
                                            double alpha, double &u, double &w) {
    const double rinv = r2 > 0.0 ? rsqrt_nr(r2) : 0.0;
    const double r = r2 * rinv;
    const double x = r - r_e;
    double c;
    if (type == 1) {
        c = r_e == 0.0 ? -k : -k * x * rinv;
        u = 0.5 * k * x * x;
    } else {
        const double E = exp(-alpha * (type == 2 ? fabs(x) : x));
        const double omE = 1.0 - E;
        c = -2.0 * alpha * k * E * omE * rinv;
        u = k * (omE * omE - (type == 2 ? 0.0 : 1.0));
    }
    w = c * r2;
    return c;
}

}  // namespace dpd
