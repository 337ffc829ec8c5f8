// DPD oracle: TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of one step of Groot-style DPD as
// defined by Doi, Okuwaki, Naito, Saitou and Mochizuki, "A portable code for
// dissipative particle dynamics (DPD) simulations with additional specific
// interactions" (arXiv 1804.06205).  Only the test suite, the smoke check and
// the CPU-baseline leg of the benchmark load it.  It shares no code, header,
// table or helper with the HIP library and must never be called on the
// library's product path.
//
// Where the paper is silent (forms of F^D and F^R, the noise stream, the
// initial force, signs, binning tie-breaks) this file follows the readings
// listed in the design notes; each function names the passage it follows.
//
// Units: masses are 1 (paper, "Summary of DPD simulation": masses are made
// dimensionless), cutoff rc = 1 (Eq. 4 writes the cutoff as r < 1).
//
// Conventions for a pair (i, j): d = x_i - x_j under the minimum image,
// r = |d|, e = d / r points from j to i; a positive coefficient on e pushes i
// away from j; the force on j is minus the force on i.
//
// Status of pins: every function is pinned by a CPU test (closed forms,
// finite differences, brute force, invariants, statistics, an independent
// Philox implementation).  The pair noise stream is a reading, not a paper
// value: it is pinned by rocRAND's Philox4x32-10 (raw words) and statistics.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>

extern "C" {

// ---------------------------------------------------------------------------
// Noise: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) followed by Box-Muller.  The paper
// only says the random force is Gaussian thermal noise (text after Eq. 5);
// the counter layout (min tag, max tag, step, 0) makes theta_ij = theta_ji.
// ---------------------------------------------------------------------------

// One Philox-4x32 round: two 32x32->64 products of the even words with the
// round multipliers, then the odd words and the round key mix into the high
// halves, with the word order permuted.
static void philox_round(uint32_t x[4], const uint32_t k[2]) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ x[1] ^ k[0];
    const uint32_t y1 = lo1;
    const uint32_t y2 = hi0 ^ x[3] ^ k[1];
    const uint32_t y3 = lo0;
    x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
}

// Philox4x32 with 10 rounds; the key is bumped by the Weyl constants
// (golden ratio and sqrt(3) - 1, scaled to 32 bits) between rounds.
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t x[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(x, k);
    }
    std::memcpy(out, x, sizeof x);
}

// theta_ij(s): one standard normal per unordered pair per force evaluation s.
// u1 = ((w0 >> 8) + 1) 2^-24 in (0, 1], u2 = (w1 >> 8) 2^-24 in [0, 1),
// theta = sqrt(-2 ln u1) cos(2 pi u2).
double oracle_pair_noise(uint64_t seed, uint32_t tag_i, uint32_t tag_j, uint64_t s) {
    const uint32_t lo = tag_i < tag_j ? tag_i : tag_j;
    const uint32_t hi = tag_i < tag_j ? tag_j : tag_i;
    const uint32_t ctr[4] = {lo, hi, (uint32_t)(s & 0xFFFFFFFFu), 0u};
    const uint32_t key[2] = {(uint32_t)(seed & 0xFFFFFFFFu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    oracle_philox4x32_10(ctr, key, w);
    const double u1 = ((double)(w[0] >> 8) + 1.0) * std::ldexp(1.0, -24);
    const double u2 = (double)(w[1] >> 8) * std::ldexp(1.0, -24);
    const double pi = 3.14159265358979323846;
    return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * pi * u2);
}

// theta for m (tag_i, tag_j, s) triples; for statistical tests.
void oracle_pair_noise_batch(uint64_t seed, int64_t m, const uint32_t *ti, const uint32_t *tj,
                             const uint64_t *s, double *out) {
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < m; ++q) out[q] = oracle_pair_noise(seed, ti[q], tj[q], s[q]);
}

// ---------------------------------------------------------------------------
// Geometry.
// ---------------------------------------------------------------------------

// Minimum image of one component of x_i - x_j in a periodic box of edge L.
static double min_image(double d, double L) {
    return d - L * std::nearbyint(d / L);
}

// Periodic wrap ("boundary_check" in Fig. 1): one shift down or up, and a
// value that rounds onto L after the upward shift becomes 0.
double oracle_wrap(double x, double L) {
    if (x < 0.0) x += L;
    else if (x >= L) x -= L;
    if (x >= L) x = 0.0;
    return x;
}

// Number of cells along one edge: the cell edge equals the cutoff (design
// section of the paper), so n = floor(L / 1) and h = L / n >= 1.
static int64_t ncell_of(double L) { return (int64_t)std::floor(L); }

// Cell coordinate of x in [0, L): floor(x / h), clamped to n - 1.
static int64_t cell_coord(double x, double L) {
    const int64_t n = ncell_of(L);
    const double h = L / (double)n;
    int64_t c = (int64_t)std::floor(x / h);
    if (c > n - 1) c = n - 1;
    if (c < 0) c = 0;
    return c;
}

// ---------------------------------------------------------------------------
// Pair and bond terms.
// ---------------------------------------------------------------------------

// F^C + F^D + F^R on i from j (Eq. 3 without F^S; Eq. 4 for F^C; the
// Groot-Warren forms for F^D and F^R named in the text after Eq. 5):
//   w = 1 - r,  F_i = [ a w - gamma w^2 (e . dv) + sigma w theta / sqrt(dt) ] e.
// Also returns the pair energy a w^2 / 2 and the conservative virial d . F^C.
// Requires 0 < r^2 < 1.
static void pair_term(const double d[3], const double dv[3], double a, double gamma,
                      double sigma, double dt, double theta, double F[3],
                      double *U, double *W) {
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = std::sqrt(r2);
    const double e[3] = {d[0] / r, d[1] / r, d[2] / r};
    const double w = 1.0 - r;
    const double edv = e[0] * dv[0] + e[1] * dv[1] + e[2] * dv[2];
    const double fc = a * w;
    const double fd = -gamma * w * w * edv;
    const double fr = sigma * w * theta / std::sqrt(dt);
    const double coef = fc + fd + fr;
    for (int c = 0; c < 3; ++c) F[c] = coef * e[c];
    *U = 0.5 * a * w * w;
    *W = fc * r;
}

// Bonded force on i from one bond record (Eqs. 6-8, Fig. 3a).  x = r - r_e.
//  type 1, harmonic (Eq. 6): F_i = -C x e, U = C x^2 / 2 (Fig. 3a energy).
//  type 2, the paper's modified Morse (Eq. 7 with the alpha of Fig. 3a):
//          E = exp(-alpha |x|), F_i = -2 alpha K E (1 - E) e, U = K (1 - E)^2.
//  type 3, standard Morse: E = exp(-alpha x), U = D[(1 - E)^2 - 1],
//          F_i = -2 alpha D E (1 - E) e.
// No cutoff; r = 0 gives no force except for the harmonic spring with r_e = 0.
// Returns 0 on success, -1 for an unknown type.
int oracle_bond_term(int type, const double d[3], double r_e, double k, double alpha,
                     double F[3], double *U, double *W) {
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const double r = std::sqrt(r2);
    double coef_over_r = 0.0;  // F_i = coef_over_r * d
    double u = 0.0;
    if (type == 1) {
        const double x = r - r_e;
        if (r_e == 0.0) coef_over_r = -k;
        else if (r > 0.0) coef_over_r = -k * x / r;
        u = 0.5 * k * x * x;
    } else if (type == 2) {
        const double x = r - r_e;
        const double E = std::exp(-alpha * std::fabs(x));
        if (r > 0.0) coef_over_r = -2.0 * alpha * k * E * (1.0 - E) / r;
        u = k * (1.0 - E) * (1.0 - E);
    } else if (type == 3) {
        const double x = r - r_e;
        const double E = std::exp(-alpha * x);
        if (r > 0.0) coef_over_r = -2.0 * alpha * k * E * (1.0 - E) / r;
        u = k * ((1.0 - E) * (1.0 - E) - 1.0);
    } else {
        return -1;
    }
    for (int c = 0; c < 3; ++c) F[c] = coef_over_r * d[c];
    *U = u;
    *W = coef_over_r * r2;
    return 0;
}

// ---------------------------------------------------------------------------
// Binning (the per-step cell list of the design section and Fig. 1 step 3).
// ---------------------------------------------------------------------------

// cell_xyz[3i..3i+2] = per-axis cell coordinates; count[c] = particles in
// linear cell c = (cz ny + cy) nx + cx; start = exclusive prefix sum of count
// (ncells + 1 entries); order = tags sorted by (cell, tag).
void oracle_bin(int64_t n, const double L[3], const double *pos, int64_t *cell_xyz,
                int64_t *count, int64_t *start, int64_t *order) {
    const int64_t nx = ncell_of(L[0]), ny = ncell_of(L[1]), nz = ncell_of(L[2]);
    const int64_t ncells = nx * ny * nz;
    std::vector<int64_t> lin(n);
    for (int64_t c = 0; c < ncells; ++c) count[c] = 0;
    for (int64_t i = 0; i < n; ++i) {
        const int64_t cx = cell_coord(pos[3 * i + 0], L[0]);
        const int64_t cy = cell_coord(pos[3 * i + 1], L[1]);
        const int64_t cz = cell_coord(pos[3 * i + 2], L[2]);
        cell_xyz[3 * i + 0] = cx;
        cell_xyz[3 * i + 1] = cy;
        cell_xyz[3 * i + 2] = cz;
        lin[i] = (cz * ny + cy) * nx + cx;
        count[lin[i]] += 1;
    }
    start[0] = 0;
    for (int64_t c = 0; c < ncells; ++c) start[c + 1] = start[c] + count[c];
    // Tags are visited in increasing order, so each cell receives its members
    // in ascending tag order.
    std::vector<int64_t> fill(start, start + ncells);
    for (int64_t i = 0; i < n; ++i) order[fill[lin[i]]++] = i;
}

// ---------------------------------------------------------------------------
// Forces.
// ---------------------------------------------------------------------------

struct PairParams {
    double L[3];
    int ntypes;
    const double *a;
    double gamma, sigma, dt;
    uint64_t seed;
    uint64_t s;
};

// Adds the pair force on i from j if their minimum-image distance is below
// the cutoff (strict r^2 < 1, Eq. 4); returns 1 if the pair is in range.
static int add_pair(const PairParams &P, const double *pos, const double *vt,
                    const uint8_t *type, int64_t i, int64_t j, double Fi[3],
                    double *U, double *W) {
    double d[3], dv[3];
    for (int c = 0; c < 3; ++c) {
        d[c] = min_image(pos[3 * i + c] - pos[3 * j + c], P.L[c]);
        dv[c] = vt[3 * i + c] - vt[3 * j + c];
    }
    const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (!(r2 < 1.0)) return 0;
    // A coincident pair is in range but has no direction, hence no force.
    if (r2 == 0.0) return 1;
    const int ti = type ? type[i] : 0, tj = type ? type[j] : 0;
    const double a = P.a[ti * P.ntypes + tj];
    const double theta = oracle_pair_noise(P.seed, (uint32_t)i, (uint32_t)j, P.s);
    double F[3], u, w;
    pair_term(d, dv, a, P.gamma, P.sigma, P.dt, theta, F, &u, &w);
    for (int c = 0; c < 3; ++c) Fi[c] += F[c];
    *U += u;
    *W += w;
    return 1;
}

// Pair forces by brute force over all j != i (the plain definition of Eq. 3's
// sum restricted to r < 1).  Writes F (n*3); energy, virial and the number of
// unordered in-range pairs go to out3[0..2] if out3 is not NULL.
void oracle_pair_forces_brute(int64_t n, const double L[3], const double *pos,
                              const double *vt, const uint8_t *type, int ntypes,
                              const double *a, double gamma, double sigma, double dt,
                              uint64_t seed, uint64_t s, double *F, double *out3) {
    const PairParams P = {{L[0], L[1], L[2]}, ntypes, a, gamma, sigma, dt, seed, s};
    std::vector<double> Ui(n, 0.0), Wi(n, 0.0);
    std::vector<int64_t> Ni(n, 0);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double Fi[3] = {0.0, 0.0, 0.0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            Ni[i] += add_pair(P, pos, vt, type, i, j, Fi, &Ui[i], &Wi[i]);
        }
        for (int c = 0; c < 3; ++c) F[3 * i + c] = Fi[c];
    }
    if (out3) {
        double U = 0.0, W = 0.0;
        int64_t np2 = 0;
        for (int64_t i = 0; i < n; ++i) { U += Ui[i]; W += Wi[i]; np2 += Ni[i]; }
        out3[0] = 0.5 * U;
        out3[1] = 0.5 * W;
        out3[2] = 0.5 * (double)np2;
    }
}

// Pair forces through the cell list: particle i visits the 27 cells around
// its own (offsets -1..1 per axis, z slowest) and every particle in them.
// With at least 3 cells per axis these 27 cells are distinct, and they hold
// every particle within the cutoff, so the result equals the brute force.
// OpenMP over particles; every particle sums in a fixed order, so the result
// does not depend on the thread count.
void oracle_pair_forces(int64_t n, const double L[3], const double *pos, const double *vt,
                        const uint8_t *type, int ntypes, const double *a, double gamma,
                        double sigma, double dt, uint64_t seed, uint64_t s, double *F,
                        double *out3) {
    const PairParams P = {{L[0], L[1], L[2]}, ntypes, a, gamma, sigma, dt, seed, s};
    const int64_t nx = ncell_of(L[0]), ny = ncell_of(L[1]), nz = ncell_of(L[2]);
    const int64_t ncells = nx * ny * nz;
    std::vector<int64_t> cxyz(3 * n), count(ncells), start(ncells + 1), order(n);
    oracle_bin(n, L, pos, cxyz.data(), count.data(), start.data(), order.data());
    std::vector<double> Ui(n, 0.0), Wi(n, 0.0);
    std::vector<int64_t> Ni(n, 0);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double Fi[3] = {0.0, 0.0, 0.0};
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int64_t cx = (cxyz[3 * i + 0] + dx + nx) % nx;
                    const int64_t cy = (cxyz[3 * i + 1] + dy + ny) % ny;
                    const int64_t cz = (cxyz[3 * i + 2] + dz + nz) % nz;
                    const int64_t c = (cz * ny + cy) * nx + cx;
                    for (int64_t k = start[c]; k < start[c + 1]; ++k) {
                        const int64_t j = order[k];
                        if (j == i) continue;
                        Ni[i] += add_pair(P, pos, vt, type, i, j, Fi, &Ui[i], &Wi[i]);
                    }
                }
        for (int c = 0; c < 3; ++c) F[3 * i + c] = Fi[c];
    }
    if (out3) {
        double U = 0.0, W = 0.0;
        int64_t np2 = 0;
        for (int64_t i = 0; i < n; ++i) { U += Ui[i]; W += Wi[i]; np2 += Ni[i]; }
        out3[0] = 0.5 * U;
        out3[1] = 0.5 * W;
        out3[2] = 0.5 * (double)np2;
    }
}

// Bonded forces F^S (Eq. 8): every record adds its term to i and the opposite
// term to j; several records may sit on one pair (Fig. 3b lists a harmonic and
// a Morse record on the same 1-3 pair).  Adds into F; energy and virial go to
// out2[0..1] if out2 is not NULL.  Returns 0, or -1 on a bad record.
int oracle_bond_forces(int64_t n, const double L[3], const double *pos, int64_t nb,
                       const int32_t *btype, const int64_t *bi, const int64_t *bj,
                       const double *r_e, const double *k, const double *alpha,
                       double *F, double *out2) {
    double U = 0.0, W = 0.0;
    for (int64_t b = 0; b < nb; ++b) {
        const int64_t i = bi[b], j = bj[b];
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return -1;
        double d[3];
        for (int c = 0; c < 3; ++c) d[c] = min_image(pos[3 * i + c] - pos[3 * j + c], L[c]);
        double f[3], u, w;
        if (oracle_bond_term(btype[b], d, r_e[b], k[b], alpha[b], f, &u, &w) != 0) return -1;
        for (int c = 0; c < 3; ++c) {
            F[3 * i + c] += f[c];
            F[3 * j + c] -= f[c];
        }
        U += u;
        W += w;
    }
    if (out2) { out2[0] = U; out2[1] = W; }
    return 0;
}

// ---------------------------------------------------------------------------
// Time step (Fig. 1 with Groot's modified velocity Verlet).
// ---------------------------------------------------------------------------

// Scalar parameters, in this order: gamma, sigma, dt, lambda.
struct StepParams { double gamma, sigma, dt, lambda; };

static int total_force(int64_t n, const double L[3], const double *pos, const double *vt,
                       const uint8_t *type, int ntypes, const double *a, const StepParams &S,
                       uint64_t seed, uint64_t s, int64_t nb, const int32_t *btype,
                       const int64_t *bi, const int64_t *bj, const double *r_e,
                       const double *k, const double *alpha, double *F) {
    oracle_pair_forces(n, L, pos, vt, type, ntypes, a, S.gamma, S.sigma, S.dt, seed, s, F,
                       nullptr);
    return oracle_bond_forces(n, L, pos, nb, btype, bi, bj, r_e, k, alpha, F, nullptr);
}

// Total force f = F_pair(x, vt; s) + F_bond(x) at an arbitrary state; the
// initial force of a run is this with vt = v and s = 0.
int oracle_forces(int64_t n, const double L[3], const double *pos, const double *vt,
                  const uint8_t *type, int ntypes, const double *a, const double *sp,
                  uint64_t seed, uint64_t s, int64_t nb, const int32_t *btype,
                  const int64_t *bi, const int64_t *bj, const double *r_e, const double *k,
                  const double *alpha, double *F) {
    const StepParams S = {sp[0], sp[1], sp[2], sp[3]};
    return total_force(n, L, pos, vt, type, ntypes, a, S, seed, s, nb, btype, bi, bj, r_e, k,
                       alpha, F);
}

// Advances (pos, vel, force) by nsteps steps starting at step counter s0.
// force must hold the force of the current state (f = F(x, vt; s0)).
// Step k -> k+1, with s = k + 1 for the new force evaluation:
//   1. x <- x + dt v + dt^2 f / 2, then wrap (Fig. 1 step 1);
//   2. vt <- v + lambda dt f (Fig. 1 step 2; lambda = 0.65 in the paper);
//   3. bin (Fig. 1 step 3, inside the pair force);
//   4. f' <- F_pair(x, vt; s) + F_bond(x) (Fig. 1 step 4 plus the bonds);
//   5. v <- v + dt (f + f') / 2 (Fig. 1 step 5), then f <- f'.
// Returns 0, -1 on a bad bond record, -2 if a displacement exceeds half a box.
int oracle_run(int64_t n, const double L[3], double *pos, double *vel, double *force,
               const uint8_t *type, int ntypes, const double *a, const double *sp,
               uint64_t seed, uint64_t s0, int64_t nsteps, int64_t nb, const int32_t *btype,
               const int64_t *bi, const int64_t *bj, const double *r_e, const double *k,
               const double *alpha) {
    const StepParams S = {sp[0], sp[1], sp[2], sp[3]};
    const double dt = S.dt;
    std::vector<double> vt(3 * n), fnew(3 * n);
    for (int64_t step = 0; step < nsteps; ++step) {
        const uint64_t s = s0 + (uint64_t)step + 1;
        for (int64_t i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) {
                const int64_t q = 3 * i + c;
                const double disp = dt * vel[q] + 0.5 * dt * dt * force[q];
                if (!(std::fabs(disp) <= 0.5 * L[c])) return -2;
                pos[q] = oracle_wrap(pos[q] + disp, L[c]);
                vt[q] = vel[q] + S.lambda * dt * force[q];
            }
        std::fill(fnew.begin(), fnew.end(), 0.0);
        if (total_force(n, L, pos, vt.data(), type, ntypes, a, S, seed, s, nb, btype, bi, bj,
                        r_e, k, alpha, fnew.data()) != 0)
            return -1;
        for (int64_t q = 0; q < 3 * n; ++q) {
            vel[q] = vel[q] + 0.5 * dt * (force[q] + fnew[q]);
            force[q] = fnew[q];
        }
    }
    return 0;
}

// ---------------------------------------------------------------------------
// Observables.  The paper accumulates a bonded energy (Ebond, Fig. 3a); the
// temperature and pressure are the usual DPD estimators.
// ---------------------------------------------------------------------------

// out[0..13] = {KE, kT, U_pair, U_bond, W_pair, W_bond, pressure,
//               P_x, P_y, P_z, npairs, E_total, W_total, volume}
//   KE = sum |v|^2 / 2, kT = 2 KE / (3N - 3), p = (2 KE + W) / (3 V), where W is
//   the conservative plus bonded virial sum over pairs of d . F_i.
int oracle_observables(int64_t n, const double L[3], const double *pos, const double *vel,
                       const uint8_t *type, int ntypes, const double *a, int64_t nb,
                       const int32_t *btype, const int64_t *bi, const int64_t *bj,
                       const double *r_e, const double *k, const double *alpha, double *out) {
    double KE = 0.0, P[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            KE += 0.5 * vel[3 * i + c] * vel[3 * i + c];
            P[c] += vel[3 * i + c];
        }
    // Conservative energy and virial: gamma = sigma = 0 leaves only F^C.
    std::vector<double> F(3 * n, 0.0);
    double pr[3];
    oracle_pair_forces(n, L, pos, vel, type, ntypes, a, 0.0, 0.0, 1.0, 0, 0, F.data(), pr);
    double bo[2] = {0.0, 0.0};
    if (oracle_bond_forces(n, L, pos, nb, btype, bi, bj, r_e, k, alpha, F.data(), bo) != 0)
        return -1;
    const double V = L[0] * L[1] * L[2];
    const double W = pr[1] + bo[1];
    out[0] = KE;
    out[1] = 2.0 * KE / (3.0 * (double)n - 3.0);
    out[2] = pr[0];
    out[3] = bo[0];
    out[4] = pr[1];
    out[5] = bo[1];
    out[6] = (2.0 * KE + W) / (3.0 * V);
    out[7] = P[0];
    out[8] = P[1];
    out[9] = P[2];
    out[10] = pr[2];
    out[11] = KE + pr[0] + bo[0];
    out[12] = W;
    out[13] = V;
    return 0;
}

}  // extern "C"
