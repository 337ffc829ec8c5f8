// HIP kernels of the DPD step for gfx950 (CDNA4, 64-wide waves).
//
// One step of Fig. 1 (Groot's modified velocity Verlet) is split as
//   begin   : resting state q -> integrate-1 (drift, wrap, predictor) and
//             binning into the layout of state q+1;
//   fused   : forces of state q (pair sum over the 27 cells around each cell,
//             the design section's cell list with no neighbour list, plus
//             bonds), integrate-2 (Fig. 1 step 5), then integrate-1 and
//             binning of state q+1, all in one pass over the particles;
//   finish  : forces of state q and integrate-2, in place.
// dpd_step(n) runs begin, n-1 fused passes and one finish.
//
// Layouts.  Each state lives in a padded cell layout: cell g owns slots
// [g cap, (g+1) cap); count[g] of them are filled, in arbitrary order, by
// atomic appends.  Two layouts (state parity) and three count arrays (state
// mod 3) rotate, so a kernel reads one layout and writes the other while it
// zeroes the counts two states ahead.  Pair kernels restore ascending tag
// order inside each cell when they stage a neighbourhood in LDS, so every
// particle sums its pair forces in the same order on every run, whatever the
// storage order, and results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

#include "dpd_device.hpp"
#include "dpd_kernels.hpp"

namespace dpd {

constexpr int QCAP = 8;          // per-lane pending-pair queue depth (>= 5)
constexpr int MAXTYPES = 16;
// Wave priority in the fused step: a brick's first phases (cell counts and
// staging, chains of dependent memory round trips) issue ahead of other
// waves' candidate scans, so their round trips start sooner.
constexpr int PRIO_MEM = 3, PRIO_SCAN = 0;
constexpr int MAXCHUNK = 32;     // neighbourhood chunks per brick
// Pair rounds start once this fraction of a wave's lanes hold a pending pair.
#ifndef DPD_ROUND_NUM
#define DPD_ROUND_NUM 15
#define DPD_ROUND_DEN 16
#endif

enum : int { MODE_INIT = 0, MODE_FINISH = 1, MODE_FUSED = 2, MODE_OBS = 3 };

// Neighbour positions and tags staged in LDS.
template <typename T> struct alignas(16) LA { typename Geo<T>::P ox, oy, oz; uint32_t tag; };

__device__ __forceinline__ int wrapi(int c, int n) {
    c = c < 0 ? c + n : c;
    return c >= n ? c - n : c;
}

// Maximum of v over the wave.
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

// Exclusive prefix sums of a[0..ma) and b[0..mb) in place, in one pass
// (ma <= NT * IPTA, mb <= NT * IPTB); a[ma] and b[mb] get the totals.  Both
// totals must stay below 2^16: the two scans run as one, on a + b * 2^16.
// s_wave holds NT / 64 ints.  All threads of the block must call it.
template <int NT, int IPTA, int IPTB>
__device__ void block_scan2(int *a, int ma, int *b, int mb, int *s_wave) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    int va[IPTA], vb[IPTB];
    uint32_t sab = 0u;
#pragma unroll
    for (int k = 0; k < IPTA; ++k) {
        const int idx = tid * IPTA + k;
        va[k] = idx < ma ? a[idx] : 0;
        sab += (uint32_t)va[k];
    }
#pragma unroll
    for (int k = 0; k < IPTB; ++k) {
        const int idx = tid * IPTB + k;
        vb[k] = idx < mb ? b[idx] : 0;
        sab += (uint32_t)vb[k] << 16;
    }
    uint32_t iab = sab;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(iab, off, 64);
        if (lane >= off) iab += t;
    }
    if (lane == 63) s_wave[wid] = (int)iab;
    __syncthreads();
    uint32_t wab = 0u;
    for (int w = 0; w < wid; ++w) wab += (uint32_t)s_wave[w];
    const uint32_t rab = wab + iab - sab;
    int ra = (int)(rab & 0xFFFFu), rb = (int)(rab >> 16);
#pragma unroll
    for (int k = 0; k < IPTA; ++k) {
        const int idx = tid * IPTA + k;
        if (idx < ma) a[idx] = ra;
        ra += va[k];
    }
#pragma unroll
    for (int k = 0; k < IPTB; ++k) {
        const int idx = tid * IPTB + k;
        if (idx < mb) b[idx] = rb;
        rb += vb[k];
    }
    if (tid == NT - 1) {
        a[ma] = ra;
        b[mb] = rb;
    }
    __syncthreads();
}

// Exclusive prefix sums of a[0..ma) and b[0..mb) in place, in one pass
// (ma <= NT * IPTA, mb <= NT * IPTB); a[ma] and b[mb] get the totals.
// s_wave holds 2 * NT / 64 ints.  All threads of the block must call it.
// Used when a total may reach 2^16 (block_scan2 above packs both into one).
template <int NT, int IPTA, int IPTB>
__device__ void block_scan2_wide(int *a, int ma, int *b, int mb, int *s_wave) {
    constexpr int NW = NT / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    int va[IPTA], vb[IPTB];
    int sa = 0, sb = 0;
#pragma unroll
    for (int k = 0; k < IPTA; ++k) {
        const int idx = tid * IPTA + k;
        va[k] = idx < ma ? a[idx] : 0;
        sa += va[k];
    }
#pragma unroll
    for (int k = 0; k < IPTB; ++k) {
        const int idx = tid * IPTB + k;
        vb[k] = idx < mb ? b[idx] : 0;
        sb += vb[k];
    }
    int ia = sa, ib = sb;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ta = __shfl_up(ia, off, 64), tb = __shfl_up(ib, off, 64);
        if (lane >= off) {
            ia += ta;
            ib += tb;
        }
    }
    if (lane == 63) {
        s_wave[wid] = ia;
        s_wave[NW + wid] = ib;
    }
    __syncthreads();
    int wa = 0, wb = 0;
    for (int w = 0; w < wid; ++w) {
        wa += s_wave[w];
        wb += s_wave[NW + w];
    }
    int ra = wa + ia - sa, rb = wb + ib - sb;
#pragma unroll
    for (int k = 0; k < IPTA; ++k) {
        const int idx = tid * IPTA + k;
        if (idx < ma) a[idx] = ra;
        ra += va[k];
    }
#pragma unroll
    for (int k = 0; k < IPTB; ++k) {
        const int idx = tid * IPTB + k;
        if (idx < mb) b[idx] = rb;
        rb += vb[k];
    }
    if (tid == NT - 1) {
        a[ma] = ra;
        b[mb] = rb;
    }
    __syncthreads();
}

// Largest index c in [0, m) with a[c] <= u, for a non-decreasing a.
__device__ __forceinline__ int find_bin(const int *a, int m, int u) {
    int lo = 0, hi = m - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a[mid] <= u) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Work-group -> brick map that gives each XCD a contiguous range of bricks
// (work-groups are dealt to the 8 XCDs round robin), so the neighbourhood
// re-reads of adjacent bricks hit the same L2.
__device__ __forceinline__ int xcd_brick(int bid, int nb) {
    const int x = bid & 7, k = bid >> 3;
    const int per = nb >> 3, rem = nb & 7;
    return x * per + min(x, rem) + k;
}

// Integrate-1 (Fig. 1 steps 1-2) of one particle of state q and its append
// to the layout of state q + 1.  Shared by begin and fused so both round alike.
template <typename T>
__device__ __forceinline__ void drift_and_bin(const DevSys<T> &D, uint32_t q, double x,
                                              double y, double z, T vx, T vy, T vz, T fx,
                                              T fy, T fz, uint32_t tag, uint32_t type,
                                              bool bonded) {
    const double dx = D.dt_d * (double)vx + D.half_dt2_d * (double)fx;
    const double dy = D.dt_d * (double)vy + D.half_dt2_d * (double)fy;
    const double dz = D.dt_d * (double)vz + D.half_dt2_d * (double)fz;
    if (!(fabs(dx) <= 0.5 * D.L[0] && fabs(dy) <= 0.5 * D.L[1] && fabs(dz) <= 0.5 * D.L[2])) {
        atomicOr(D.err, (isfinite(dx) && isfinite(dy) && isfinite(dz)) ? ERR_DISPLACEMENT
                                                                       : ERR_NONFINITE);
        return;
    }
    x = wrap_coord(x + dx, D.L[0]);
    y = wrap_coord(y + dy, D.L[1]);
    z = wrap_coord(z + dz, D.L[2]);
    const T lt = D.lambda * D.dt;
    const T tx = vx + lt * fx, ty = vy + lt * fy, tz = vz + lt * fz;
    // Unit cells (integer box edges, the usual case): x / 1 = x exactly, so
    // the divides of the binning and the offset encoding drop out.
    const bool unit = D.h[0] == 1.0 && D.h[1] == 1.0 && D.h[2] == 1.0;
    const int cx = unit ? cell_coord_unit(x, D.nc[0]) : cell_coord(x, D.h[0], D.nc[0]);
    const int cy = unit ? cell_coord_unit(y, D.nc[1]) : cell_coord(y, D.h[1], D.nc[1]);
    const int cz = unit ? cell_coord_unit(z, D.nc[2]) : cell_coord(z, D.h[2], D.nc[2]);
    const int64_t g = cell_linear(cx, cy, cz, D.nc);
    const uint32_t k = atomicAdd(&D.count[count_index(q, 1u)][g], 1u);
    if (k >= (uint32_t)D.cap) {
        atomicOr(D.err, ERR_CELL_OVERFLOW);
        return;
    }
    const int64_t slot = g * D.cap + k;
    const uint32_t ln = (q + 1u) & 1u;
    PRec<T> p;
    p.ox = unit ? Geo<T>::encode_unit(x, cx) : Geo<T>::encode(x, cx, D.h[0]);
    p.oy = unit ? Geo<T>::encode_unit(y, cy) : Geo<T>::encode(y, cy, D.h[1]);
    p.oz = unit ? Geo<T>::encode_unit(z, cz) : Geo<T>::encode(z, cz, D.h[2]);
    p.tag = tag;
    p.vx = tx;
    p.vy = ty;
    p.vz = tz;
    p.type = type;
    D.P[ln][slot] = p;
    SRec<T> s;
    s.x = x;
    s.y = y;
    s.z = z;
    s.vx = vx;
    s.vy = vy;
    s.vz = vz;
    s.fx = fx;
    s.fy = fy;
    s.fz = fz;
    D.S[ln][slot] = s;
    // The tag -> slot map is read only to find bond partners; keep it for
    // bonded particles (a scattered 4-byte store costs a whole memory burst)
    // and rebuild it in full before any read-back.
    if (bonded) D.slot_of_tag[ln][tag] = (uint32_t)slot;
}

// ---------------------------------------------------------------------------
// Pair + bond force over one brick of BX x BY x BZ cells.
//
// The work-group stages the brick's neighbourhood (its cells plus one layer,
// periodic) in LDS with ascending tag order inside every cell.  Each lane owns
// one particle i and walks the 9 rows of 3 consecutive halo cells that hold
// its 27 neighbour cells, in a fixed order, so i adds its pair forces in the
// same order on every run.  In-range neighbours are queued per lane in LDS and
// the expensive pair term (Philox, Box-Muller, force) runs once 15 of every 16
// lanes hold a queued neighbour, which keeps the 64-wide wave busy although
// only ~15% of the candidates are within the cutoff.
//
// IGEO (mixed precision, cubic cells): LDS holds brick-frame fixed-point
// coordinates (cell offset + halo cell index, in units of 2^-29 cells, as
// u32), so a candidate's squared distance is an exact 64-bit integer and the
// cutoff test is three subtractions and three 32x32->64 multiply-adds.
// A lane walks its 9 rows back to back from a per-cell table of row ranges,
// so a wave's scan lasts as long as its longest lane's candidate list.
// Otherwise (FP64, or non-cubic cells) LDS holds cell-local offsets and the
// whole-cell shift of each neighbour is applied explicitly; the wave steps
// through the rows together.
// ---------------------------------------------------------------------------
struct alignas(16) LAI { uint32_t qx, qy, qz, tag; };

// Global cell of halo cell hc of the brick with origin (c0x, c0y, c0z).
template <int HX, int HY>
__device__ __forceinline__ int64_t halo_cell(int hc, int c0x, int c0y, int c0z, const int nc[3]) {
    const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
    return cell_linear(wrapi(c0x + hx - 1, nc[0]), wrapi(c0y + hy - 1, nc[1]),
                       wrapi(c0z + hz - 1, nc[2]), nc);
}

// Neighbour data staged in LDS for one brick: positions and tags (AT), the
// predicted velocity as three arrays and the type as bytes.
template <typename T, typename AT, int HCAP> struct Tile {
    AT *A;
    T *vx, *vy, *vz;
    uint8_t *type;
};

// Copies halo cells [c0, c1) into the tile at their offsets relative to cell
// c0 in ascending tag order inside every cell.  One thread per record: every
// record of the chunk is loaded at once (one memory round trip, however full
// the densest cell), its tag is parked in the tile's vx array, each record is
// ranked among its cell's tags (distinct) from there, and after a barrier it
// is stored at its rank.  Before that, one pass over the cells writes each
// record's cell into the tile's vy array, so a record finds its source slot
// from that and the cell's global index (s_gcell) with two LDS reads.  All
// threads of the block must call it; the tile's arrays are free on entry.
template <typename T, int HX, int HY, int NT, bool IGEO, typename AT, int HCAP>
__device__ __forceinline__ void stage_cells(const DevSys<T> &D, uint32_t lay,
                                            const int *s_hstart, const int32_t *s_gcell, int c0,
                                            int c1, const Tile<T, AT, HCAP> &tl) {
    constexpr int RPT = (HCAP + NT - 1) / NT;   // records per thread, at most
    const int cap = D.cap;
    const int off0 = s_hstart[c0];
    const int m = s_hstart[c1] - off0;           // <= HCAP (chunk planning)
    uint32_t *park = reinterpret_cast<uint32_t *>(tl.vx);
    uint16_t *rcell = reinterpret_cast<uint16_t *>(tl.vy);     // record -> halo cell
    for (int hc = c0 + (int)threadIdx.x; hc < c1; hc += NT) {
        const int lo = s_hstart[hc] - off0, hi = s_hstart[hc + 1] - off0;
        for (int k = lo; k < hi; ++k) rcell[k] = (uint16_t)hc;
    }
    __syncthreads();
    PRec<T> r[RPT];
    int hcell[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int t = (int)threadIdx.x + u * NT;
        hcell[u] = -1;
        if (t < m) {
            const int hc = rcell[t];
            hcell[u] = hc;
            r[u] = D.P[lay][(int64_t)s_gcell[hc] * cap + (t + off0 - s_hstart[hc])];
        }
    }
#pragma unroll
    for (int u = 0; u < RPT; ++u)
        if (hcell[u] >= 0) park[(int)threadIdx.x + u * NT] = r[u].tag;
    __syncthreads();
    int rank[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        rank[u] = 0;
        if (hcell[u] >= 0) {
            const int lo = s_hstart[hcell[u]] - off0, hi = s_hstart[hcell[u] + 1] - off0;
            int c = 0;
            for (int k = lo; k < hi; ++k) c += park[k] < r[u].tag ? 1 : 0;
            rank[u] = lo + c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        if (hcell[u] < 0) continue;
        const int hc = hcell[u];
        const PRec<T> &pr = r[u];
        AT a;
        if constexpr (IGEO) {
            a.qx = (uint32_t)pr.ox + ((uint32_t)(hc % HX) << 29);
            a.qy = (uint32_t)pr.oy + ((uint32_t)((hc / HX) % HY) << 29);
            a.qz = (uint32_t)pr.oz + ((uint32_t)(hc / (HX * HY)) << 29);
        } else {
            a.ox = pr.ox;
            a.oy = pr.oy;
            a.oz = pr.oz;
        }
        a.tag = pr.tag;
        const int j = rank[u];
        tl.A[j] = a;
        tl.vx[j] = pr.vx;
        tl.vy[j] = pr.vy;
        tl.vz[j] = pr.vz;
        tl.type[j] = (uint8_t)pr.type;
    }
}

// Forces of state q for brick b of an nbx x nby x nbz split of the box.  Each
// axis of n cells is cut into m near-equal runs (cell (k n) / m starts run k),
// each at most the compile-time extent, so no brick is a thin remainder.  fin
// (MODE_FUSED only) ends the step in place like MODE_FINISH instead of moving
// on to state q + 1; replicas of a batch use it for their last step of a window.
template <typename T, int BX, int BY, int BZ, int NT, int HCAP, int MODE, bool IGEO, bool BONDS>
__device__ __forceinline__ void force_brick(const DevSys<T> &D, uint32_t q, int b, int nbx,
                                            int nby, int nbz, uint64_t thr, bool fin) {
    constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;
    constexpr int NHC = HX * HY * HZ;
    constexpr int NOC = BX * BY * BZ;
    constexpr int IPT_H = (NHC + 1 + NT - 1) / NT;
    constexpr int IPT_O = (NOC + 1 + NT - 1) / NT;
    // Brick-frame fixed point: 2^29 units per cell (the pair records' own
    // scale, so every brick shape gives bitwise the same forces); the largest
    // coordinate, (halo extent) * 2^29, must fit in 32 bits.
    constexpr int HMAX = HX > HY ? (HX > HZ ? HX : HZ) : (HY > HZ ? HY : HZ);
    static_assert(!IGEO || HMAX <= 7, "brick too large for the u32 brick frame");
    // stage_cells keeps a u16 halo cell per record in vy before the tile is
    // filled.
    static_assert(NHC < 65536, "halo too large for the staging map");
    using AT = typename std::conditional<IGEO, LAI, LA<T>>::type;

    __shared__ int s_hstart[NHC + 1];
    __shared__ int32_t s_gcell[NHC];  // global cell of each halo cell (< 2^31 cells)
    __shared__ int s_ostart[NOC + 1];
    __shared__ int s_chunk[MAXCHUNK + 1];
    __shared__ int s_wave[2 * (NT / 64)];
    __shared__ int s_flag, s_nchunk;
    __shared__ T s_a[MAXTYPES * MAXTYPES];
    __shared__ AT s_A[HCAP + 4];     // + room for the 4-wide reads past a row's end
    __shared__ T s_vx[HCAP], s_vy[HCAP], s_vz[HCAP];
    __shared__ uint8_t s_t[HCAP];
    const Tile<T, AT, HCAP> tile{s_A, s_vx, s_vy, s_vz, s_t};
    // Per-lane queues of pending neighbours: LDS indices (u16) in the integer
    // frame; index plus whole-cell shift code (u32) otherwise.
    using QT = typename std::conditional<IGEO, uint16_t, uint32_t>::type;
    __shared__ QT s_q[QCAP * NT];
    // Integer frame: each own cell's candidate rows (see build_rows).
    __shared__ uint32_t s_rows[IGEO ? NOC * 10 : 1];

    const int tid = threadIdx.x;
    const uint32_t lay = q & 1u;
    const uint32_t *cnt = D.count[count_index(q, 0u)];
    const int cap = D.cap;

    // The sticky error word is read with the halo counts (no round trip of
    // its own); a brick of a failed system stops after that phase.
    if constexpr (IGEO && MODE == MODE_FUSED) __builtin_amdgcn_s_setprio(PRIO_MEM);
    if (tid == 0) s_flag = (int)*D.err;

    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int c0x = bx * D.nc[0] / nbx, c0y = by * D.nc[1] / nby, c0z = bz * D.nc[2] / nbz;
    const int ex = (bx + 1) * D.nc[0] / nbx - c0x, ey = (by + 1) * D.nc[1] / nby - c0y,
              ez = (bz + 1) * D.nc[2] / nbz - c0z;

    // Halo cells (own cells plus one layer, periodic) and their counts.
    for (int hc = tid; hc < NHC; hc += NT) {
        const int hx = hc % HX, hy = (hc / HX) % HY, hz = hc / (HX * HY);
        int c = 0;
        int32_t g = 0;
        if (hx <= ex + 1 && hy <= ey + 1 && hz <= ez + 1) {
            g = (int32_t)halo_cell<HX, HY>(hc, c0x, c0y, c0z, D.nc);
            c = (int)cnt[g];
            if (c > cap) {
                atomicOr(D.err, ERR_INDEX);
                c = cap;
            }
        }
        s_hstart[hc] = c;
        s_gcell[hc] = g;
        // Own cells (halo cells 1..B along each axis; those past a short
        // brick's extent hold no own particle).
        if (hx >= 1 && hx <= BX && hy >= 1 && hy <= BY && hz >= 1 && hz <= BZ)
            s_ostart[((hz - 1) * BY + (hy - 1)) * BX + (hx - 1)] =
                (hx <= ex && hy <= ey && hz <= ez) ? c : 0;
    }
    for (int i = tid; i < D.ntypes * D.ntypes; i += NT) s_a[i] = D.a[i];
    if (MODE == MODE_FUSED) {
        // Counts of state q+2 were last read for state q-1; clear this brick's.
        uint32_t *cz2 = D.count[count_index(q, 2u)];
        for (int oc = tid; oc < NOC; oc += NT) {
            const int ox = oc % BX, oy = (oc / BX) % BY, oz = oc / (BX * BY);
            if (ox < ex && oy < ey && oz < ez)
                cz2[cell_linear(c0x + ox, c0y + oy, c0z + oz, D.nc)] = 0u;
        }
    }
    __syncthreads();
    if (s_flag) return;
    // Halo counts are clamped to cap, so NHC * cap bounds both totals.
    if ((int64_t)NHC * cap < 65536)
        block_scan2<NT, IPT_H, IPT_O>(s_hstart, NHC, s_ostart, NOC, s_wave);
    else
        block_scan2_wide<NT, IPT_H, IPT_O>(s_hstart, NHC, s_ostart, NOC, s_wave);
    const int nown = s_ostart[NOC];
    // Chunks of whole halo cells that fit the LDS tile, in cell order: one
    // chunk unless the neighbourhood is unusually dense (then planned by one
    // thread).  A single cell over the tile, or more than MAXCHUNK chunks, is
    // a tile overflow.
    int nchunk = 1;
    if (s_hstart[NHC] > HCAP) {
    if (tid == 0) {
        int k = 0;
        bool over = false;
        s_chunk[0] = 0;
        if (s_hstart[NHC] > HCAP) {
            int base = 0;
            for (int hc = 0; hc < NHC; ++hc) {
                if (s_hstart[hc + 1] - s_hstart[hc] > HCAP) {
                    over = true;            // one cell larger than the tile
                    break;
                }
                if (s_hstart[hc + 1] - base > HCAP) {
                    if (k + 1 >= MAXCHUNK) {
                        over = true;
                        break;
                    }
                    s_chunk[++k] = hc;      // cell hc starts a new chunk
                    base = s_hstart[hc];
                }
            }
        }
        s_chunk[++k] = NHC;
        s_nchunk = k;
        s_flag = over ? 1 : 0;
        if (over) atomicOr(D.err, ERR_TILE_OVERFLOW);
    }
    __syncthreads();
    if (s_flag) return;
    nchunk = s_nchunk;
    }

    // Per-axis scale from offset units to length.
    const T hxT = (T)Geo<T>::hscale(D.h[0]), hyT = (T)Geo<T>::hscale(D.h[1]),
            hzT = (T)Geo<T>::hscale(D.h[2]);
    const T gamma = D.gamma, srdt = D.sigma_rdt;
    const int ntypes = D.ntypes;
    QT *myq = s_q + tid;
    // In-range test as one unsigned compare: r2 - 1 < thr - 1 also rejects
    // r2 = 0, i.e. i itself (in the observables pass, which counts coincident
    // pairs too, i is excluded by tag instead).
    const uint64_t thr1 = thr - 1u;
    // Integer frame: the nine candidate rows of every own cell (rows in
    // (dz, dy) order, each three halo cells along x) as LDS ranges of the
    // chunk [clo, chi): first | end << 16, then a zero entry.
    // Built once per brick, or per chunk when the neighbourhood is split.
    // One thread per own cell writes its ten entries (few threads, one pass).
    auto build_rows = [&](int clo, int chi, int off0) {
        if constexpr (IGEO) {
            for (int oc = tid; oc < NOC; oc += NT) {
                const int ox = oc % BX, oy = (oc / BX) % BY, oz = oc / (BX * BY);
                const int h0 = (oz * HY + oy) * HX + ox;
#pragma unroll
                for (int r = 0; r < 9; ++r) {
                    const int hr = h0 + (r / 3) * (HY * HX) + (r % 3) * HX;
                    const int r0 = max(hr, clo), r1 = min(hr + 3, chi);
                    int jb = 0, je = 0;
                    if (r0 < r1) {
                        jb = s_hstart[r0] - off0;
                        je = s_hstart[r1] - off0;
                    }
                    s_rows[oc * 10 + r] = (uint32_t)jb | ((uint32_t)je << 16);
                }
                s_rows[oc * 10 + 9] = 0u;
            }
        }
    };
    if constexpr (IGEO)
        if (nchunk == 1) build_rows(0, NHC, 0);

    for (int base = 0; base < nown; base += NT) {
        const int qi = base + tid;
        const bool have = qi < nown;
        int oxc = 0, oyc = 0, ozc = 0;
        int64_t slot = 0;
        PRec<T> pi;
        pi.ox = pi.oy = pi.oz = 0;
        pi.vx = pi.vy = pi.vz = (T)0;
        pi.tag = 0xFFFFFFFFu;
        pi.type = 0;
        if (have) {
            const int oc = find_bin(s_ostart, NOC, qi);
            oxc = oc % BX;
            oyc = (oc / BX) % BY;
            ozc = oc / (BX * BY);
            slot = (int64_t)s_gcell[((ozc + 1) * HY + (oyc + 1)) * HX + (oxc + 1)] * cap +
                   (qi - s_ostart[oc]);
            pi = D.P[lay][slot];
        }
        if (base == 0 && nchunk == 1) {
            // Stage the whole neighbourhood once; the own-particle load above
            // is already in flight.
            stage_cells<T, HX, HY, NT, IGEO, AT, HCAP>(D, lay, s_hstart, s_gcell, 0, NHC, tile);
            __syncthreads();
        }
        // Brick-frame coordinates of i (IGEO).
        uint32_t pqx = 0, pqy = 0, pqz = 0;
        if constexpr (IGEO) {
            pqx = (uint32_t)pi.ox + ((uint32_t)(oxc + 1) << 29);
            pqy = (uint32_t)pi.oy + ((uint32_t)(oyc + 1) << 29);
            pqz = (uint32_t)pi.oz + ((uint32_t)(ozc + 1) << 29);
        }
        const T *arow = s_a + (int)pi.type * ntypes;
        const T a00 = s_a[0];
        T fx = 0, fy = 0, fz = 0;
        double ou = 0.0, ow = 0.0;
        uint32_t onp = 0;
        uint32_t qh = 0, qt = 0;
        // Integer frame: a queue entry is a group of four consecutive
        // candidates, base index | hit mask << 12; `cur` is the group being
        // worked through; it is empty when its mask is (cur < 2^12), which
        // happens only while the queue is empty: a group goes straight to cur
        // when cur is empty, and cur is refilled from the queue as soon as it
        // runs out (the read's latency then hides behind the pair term).
        uint32_t cur = 0;
        // Lanes with a particle; pending pairs are processed once
        // DPD_ROUND_NUM / DPD_ROUND_DEN of them have one queued.
        const int nact = __popcll(__ballot(have));
        const int rth = max(1, (DPD_ROUND_NUM * nact) / DPD_ROUND_DEN);

        // Takes one pending neighbour per lane that has one (in candidate
        // order) and adds its force.
        auto process = [&]() __attribute__((always_inline)) {
            int j = -1;
            uint32_t e = 0;
            if constexpr (IGEO) {
                if (cur >= 0x1000u) {
                    j = (int)(cur & 0xFFFu) + __builtin_ctz(cur >> 12);
                    cur &= cur - 0x1000u;       // drop the lowest hit
                    if (cur < 0x1000u && qt != qh) {
                        cur = (uint32_t)myq[(qh % QCAP) * NT];
                        ++qh;
                    }
                }
            } else {
                if (qt != qh) {
                    e = (uint32_t)myq[(qh % QCAP) * NT];
                    ++qh;
                    j = (int)(e & 0xFFFFu);
                }
            }
            if (j >= 0) {
                const AT a = s_A[j];
                const T bvx = s_vx[j], bvy = s_vy[j], bvz = s_vz[j];

                T dx, dy, dz;
                if constexpr (IGEO) {
                    if (MODE != MODE_OBS) {
                        // Cubic cells: work in offset units (u = 2^-29 h) and
                        // rescale only r; e = d / r is unit-free.  r2 >= 1 u^2
                        // here (the scan rejected r = 0).
                        const T ux = (T)(int32_t)(pqx - a.qx);
                        const T uy = (T)(int32_t)(pqy - a.qy);
                        const T uz = (T)(int32_t)(pqz - a.qz);
                        const T u2 = t_fma(ux, ux, t_fma(uy, uy, uz * uz));
                        const T rinvu = t_rsqrt(u2);
                        const T r = u2 * rinvu * hxT;
                        const T w = (T)1 - r;
                        const T edv = t_fma(ux, pi.vx - bvx,
                                            t_fma(uy, pi.vy - bvy, uz * (pi.vz - bvz))) *
                                      rinvu;
                        const T th = pair_theta<T>(D.seed, pi.tag, a.tag, q);
                        // One particle type: a_ij is a constant (no per-pair
                        // type and table reads).
                        const T aij = ntypes == 1 ? a00 : arow[s_t[j]];
                        const T c = t_fma(srdt * w, th, w * t_fma(-gamma * w, edv, aij)) * rinvu;
                        fx = t_fma(c, ux, fx);
                        fy = t_fma(c, uy, fy);
                        fz = t_fma(c, uz, fz);
                        return;
                    }
                    dx = (T)(int32_t)(pqx - a.qx) * hxT;
                    dy = (T)(int32_t)(pqy - a.qy) * hyT;
                    dz = (T)(int32_t)(pqz - a.qz) * hzT;
                } else {
                    const int code = (int)(e >> 16);
                    const int sx = (code & 3) - 1, sy = ((code >> 2) & 3) - 1,
                              sz = ((code >> 4) & 3) - 1;
                    dx = Geo<T>::delta(pi.ox, a.ox, sx, hxT);
                    dy = Geo<T>::delta(pi.oy, a.oy, sy, hyT);
                    dz = Geo<T>::delta(pi.oz, a.oz, sz, hzT);
                }
                const T r2 = dx * dx + dy * dy + dz * dz;
                const T aij = arow[s_t[j]];
                if (MODE == MODE_OBS) {
                    ++onp;
                    if (r2 > (T)0) {
                        const T r = t_sqrt(r2);
                        const T w = (T)1 - r;
                        ou += (double)(aij * w * w);
                        ow += (double)(aij * w * r);
                    }
                } else if (r2 > (T)0) {
                    const T rinv = t_rsqrt(r2);
                    const T r = r2 * rinv;
                    const T w = (T)1 - r;
                    const T edv = (dx * (pi.vx - bvx) + dy * (pi.vy - bvy) +
                                   dz * (pi.vz - bvz)) * rinv;
                    const T th = pair_theta<T>(D.seed, pi.tag, a.tag, q);
                    const T c = (aij * w - gamma * w * w * edv + srdt * w * th) * rinv;
                    fx += c * dx;
                    fy += c * dy;
                    fz += c * dz;
                }
            }
        };

        for (int k = 0; k < nchunk; ++k) {
            const int clo = nchunk == 1 ? 0 : s_chunk[k];
            const int chi = nchunk == 1 ? NHC : s_chunk[k + 1];
            const int off0 = s_hstart[clo];
            if (nchunk > 1) {
                __syncthreads();
                stage_cells<T, HX, HY, NT, IGEO, AT, HCAP>(D, lay, s_hstart, s_gcell, clo, chi,
                                                          tile);
                if constexpr (IGEO) build_rows(clo, chi, off0);
                __syncthreads();
            }
            if constexpr (IGEO && MODE == MODE_FUSED) __builtin_amdgcn_s_setprio(PRIO_SCAN);
            // Candidate scan over rows of three consecutive halo cells (clipped
            // to the chunk), four candidates per step with the LDS reads issued
            // up front; the step writes the free queue slot whether or not it
            // found a pair, so it has no branches.  Before each step every
            // queue has room for what the step can add.
            if constexpr (IGEO) {
                // Each lane walks its own cell's nine rows back to back (the
                // next row's entry read one row ahead), so the wave runs for
                // its longest lane's total rather than each row's longest.
                // Candidate order per lane is unchanged: rows, then cells,
                // then LDS order.  A finished lane (ri past its cell's zero
                // entry) has t = je = 0: in-bounds reads, empty masks.
                const int oc = (ozc * BY + oyc) * BX + oxc;
                const int rend = oc * 10 + 9;
                int ri = have ? oc * 10 : rend;
                const uint32_t ent = s_rows[ri];
                ++ri;                       // next entry; past rend once the lane is done
                uint32_t nxt = s_rows[min(ri, rend)];
                int t = (int)(ent & 0xFFFFu), je = (int)(ent >> 16);
                // -1 held in a scalar register the compiler cannot see into:
                // it then stays the first multiply-add's addend instead of
                // being reassociated into a separate 64-bit add per candidate.
                uint64_t m1;
                asm("s_mov_b64 %0, -1" : "=s"(m1));
                // One step: four candidates of the lane's current row.
                auto scan_step = [&]() __attribute__((always_inline)) {
                    const AT *rowp = s_A + t;
                    AT a[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) a[u] = rowp[u];
                    uint32_t m = 0;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int32_t ddx = (int32_t)(pqx - a[u].qx);
                        const int32_t ddy = (int32_t)(pqy - a[u].qy);
                        const int32_t ddz = (int32_t)(pqz - a[u].qz);
                        // r^2 - 1 as an unsigned sum (each square < 2^62); the
                        // -1 rides on the first multiply-add.
                        const uint64_t r2m1 = (uint64_t)((int64_t)ddz * ddz) + m1 +
                                              (uint64_t)((int64_t)ddy * ddy) +
                                              (uint64_t)((int64_t)ddx * ddx);
                        bool hit;
                        // The observables pass counts coincident pairs too
                        // (r^2 = 0), excluding i by its tag.
                        if (MODE == MODE_OBS) hit = (r2m1 + 1u < thr) & (a[u].tag != pi.tag);
                        else hit = r2m1 < thr1;
                        m |= (hit ? 1u : 0u) << u;
                    }
                    // Up to three reads past the row's end (into later cells or
                    // the tile's padding) are dropped from the hit mask: by
                    // t + 4 - je, clamped at 0 (one subtraction with clamp); it
                    // is at most 4, as je >= t (a row starts at or before its
                    // end, and the lane moves on as soon as t reaches je).
                    const int tn = t + 4;
                    m &= 0xFu >> __builtin_elementwise_sub_sat((uint32_t)tn, (uint32_t)je);
                    const uint32_t entry = (uint32_t)t | (m << 12);
                    const bool direct = (m != 0u) & (cur < 0x1000u);
                    myq[(qt % QCAP) * NT] = (QT)entry;     // free slot, used or not
                    qt += ((m != 0u) & !direct) ? 1u : 0u;
                    cur = direct ? entry : cur;
                    t = tn;
                    if (t >= je) {
                        t = (int)(nxt & 0xFFFFu);
                        je = (int)(nxt >> 16);
                        ++ri;
                        nxt = s_rows[min(ri, rend)];
                    }
                    if (__popcll(__ballot(cur >= 0x1000u)) >= rth) process();
                    // Rounds until every queue has room (two per trip, for the
                    // same register-copy reason as the scan loop below).
                    while (__ballot(qt - qh >= (uint32_t)QCAP)) {
                        process();
                        if (!__ballot(qt - qh >= (uint32_t)QCAP)) break;
                        process();
                    }
                };
                // Two steps per trip: with one, the compiler copies the six
                // values a pair round updates (cur, qt, qh, f) between two
                // register sets on every step.
                while (__ballot(ri <= rend)) {
                    scan_step();
                    if (!__ballot(ri <= rend)) break;
                    scan_step();
                }
            } else {
                // Offsets frame: one queue entry per in-range candidate, with
                // its whole-cell shift code.
                for (int row = 0; row < 9; ++row) {
                    const int dyc = row % 3 - 1, dzc = row / 3 - 1;
                    int jb = 0, b1 = 0, b2 = 0, je = 0;
                    if (have) {
                        const int hr = ((ozc + 1 + dzc) * HY + (oyc + 1 + dyc)) * HX + oxc;
                        const int r0 = max(hr, clo), r1 = min(hr + 3, chi);
                        if (r0 < r1) {
                            jb = s_hstart[r0] - off0;
                            je = s_hstart[r1] - off0;
                        }
                        b1 = s_hstart[hr + 1] - off0;
                        b2 = s_hstart[hr + 2] - off0;
                    }
                    const int len = je - jb;
                    const uint32_t rowcode = (uint32_t)(((dyc + 1) << 2) | ((dzc + 1) << 4));
                    for (int t = 0; __ballot(t < len); t += 4) {
                        AT a[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) a[u] = s_A[min(jb + t + u, max(je - 1, 0))];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int j = jb + t + u;
                            const int sx = (j >= b1 ? 1 : 0) + (j >= b2 ? 1 : 0) - 1;
                            const T dx = Geo<T>::delta(pi.ox, a[u].ox, sx, hxT);
                            const T dy = Geo<T>::delta(pi.oy, a[u].oy, dyc, hyT);
                            const T dz = Geo<T>::delta(pi.oz, a[u].oz, dzc, hzT);
                            const bool hit = (dx * dx + dy * dy + dz * dz < (T)1) &
                                             (t + u < len) & (a[u].tag != pi.tag);
                            const uint32_t code = rowcode | (uint32_t)(sx + 1);
                            myq[(qt % QCAP) * NT] = (QT)((uint32_t)j | (code << 16));
                            qt += hit ? 1u : 0u;
                        }
                        if (__popcll(__ballot(qt != qh)) >= rth) process();
                        while (__ballot(qt - qh > (uint32_t)(QCAP - 4))) process();
                    }
                }
            }
            // Queue entries index this chunk's LDS contents: drain before the
            // next (two rounds per trip, as in the scan).
            while (__ballot(cur >= 0x1000u || qt != qh)) {
                process();
                if (!__ballot(cur >= 0x1000u || qt != qh)) break;
                process();
            }
        }

        // Bonds (Eq. 8): every record owned by this particle, in input order,
        // evaluated in FP64 (stiff Morse terms reach |F| ~ 1e2, where FP32
        // rounding alone would exceed the force tolerance).  Two schedules
        // with the same sums, chosen per wave:
        //  * few bonded lanes with several records each (chains in solvent):
        //    the wave's records, at most 64, are dealt one per lane, and each
        //    owner adds its terms in record order from the lanes that
        //    evaluated them, so no lane evaluates its records one by one;
        //  * otherwise (bonds spread over many lanes, or more than 64): each
        //    lane runs its own records, four at a time, their partners'
        //    slots and positions going out together.
        double oub = 0.0, owb = 0.0;
        double gbx = 0.0, gby = 0.0, gbz = 0.0;
        uint32_t nbond = 0;
        SRec<T> si{};
        if (have) si = D.S[lay][slot];
        if (BONDS && D.bond_off) {
            const int lane = (int)(threadIdx.x & 63u);
            uint32_t k0 = 0u;
            if (have) {
                k0 = D.bond_off[pi.tag];
                nbond = D.bond_off[pi.tag + 1] - k0;
            }
            uint32_t total = nbond, mx = nbond;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                total += (uint32_t)__shfl_xor(total, d);
                mx = max(mx, (uint32_t)__shfl_xor(mx, d));
            }
            if (total <= 64u && mx >= 3u) {
                // Exclusive prefix of the record counts over the wave.
                uint32_t incl = nbond;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t t = __shfl_up(incl, d);
                    if (lane >= d) incl += t;
                }
                const uint32_t pre = incl - nbond;
                // Record g = lane belongs to the last lane o whose prefix is
                // <= g (lanes without records share their successor's).
                const uint32_t g = (uint32_t)lane;
                int o = 0;
#pragma unroll
                for (int step = 32; step >= 1; step >>= 1)
                    if (__shfl(pre, o + step) <= g) o += step;
                const uint32_t kk = __shfl(k0, o) + (g - __shfl(pre, o));
                const double ox = __shfl(si.x, o), oy = __shfl(si.y, o), oz = __shfl(si.z, o);
                double tx = 0.0, ty = 0.0, tz = 0.0, tu = 0.0, tw = 0.0;
                if (g < total) {
                    const BondEnt<T> &be = D.bonds[kk];
                    uint32_t sj = D.slot_of_tag[lay][be.partner];
                    if ((int64_t)sj >= D.ncells * cap) {
                        atomicOr(D.err, ERR_INDEX);
                        sj = 0u;
                    }
                    const SRec<T> &pj = D.S[lay][sj];
                    const double ddx = min_image(ox - pj.x, D.L[0]);
                    const double ddy = min_image(oy - pj.y, D.L[1]);
                    const double ddz = min_image(oz - pj.z, D.L[2]);
                    double ub, wb;
                    const double c = bond_coef(be.type, ddx * ddx + ddy * ddy + ddz * ddz,
                                               be.r_e, be.k, be.alpha, ub, wb);
                    tx = c * ddx;
                    ty = c * ddy;
                    tz = c * ddz;
                    tu = 0.5 * ub;
                    tw = 0.5 * wb;
                }
                // The owner's record j was evaluated by lane pre + j.
                for (uint32_t j = 0; j < mx; ++j) {
                    const int sl = (int)((pre + j) & 63u);
                    const double vx = __shfl(tx, sl), vy = __shfl(ty, sl), vz = __shfl(tz, sl);
                    const double vu = __shfl(tu, sl), vw = __shfl(tw, sl);
                    if (j < nbond) {
                        gbx += vx;
                        gby += vy;
                        gbz += vz;
                        oub += vu;
                        owb += vw;
                    }
                }
            } else if (have) {
                const uint32_t k1 = k0 + nbond;
                for (uint32_t kb = k0; kb < k1; kb += 4u) {
                    const uint32_t nb = min(k1 - kb, 4u);
                    uint32_t sj[4];
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u)
                        sj[u] = u < nb ? D.bonds[kb + u].partner : 0u;
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u) {
                        if (u < nb) {
                            sj[u] = D.slot_of_tag[lay][sj[u]];
                            if ((int64_t)sj[u] >= D.ncells * cap) {
                                atomicOr(D.err, ERR_INDEX);
                                sj[u] = 0u;
                            }
                        }
                    }
                    double px[4], py[4], pz[4];
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u) {
                        const SRec<T> &pj = D.S[lay][u < nb ? sj[u] : sj[0]];
                        px[u] = pj.x;
                        py[u] = pj.y;
                        pz[u] = pj.z;
                    }
#pragma unroll
                    for (uint32_t u = 0; u < 4u; ++u) {
                        if (u >= nb) break;
                        const BondEnt<T> &be = D.bonds[kb + u];
                        const double ddx = min_image(si.x - px[u], D.L[0]);
                        const double ddy = min_image(si.y - py[u], D.L[1]);
                        const double ddz = min_image(si.z - pz[u], D.L[2]);
                        double ub, wb;
                        const double c = bond_coef(be.type, ddx * ddx + ddy * ddy + ddz * ddz,
                                                   be.r_e, be.k, be.alpha, ub, wb);
                        gbx += c * ddx;
                        gby += c * ddy;
                        gbz += c * ddz;
                        oub += 0.5 * ub;
                        owb += 0.5 * wb;
                    }
                }
            }
            fx = (T)((double)fx + gbx);
            fy = (T)((double)fy + gby);
            fz = (T)((double)fz + gbz);
        }
        if (!have) continue;

        if (MODE == MODE_OBS) {
            const uint32_t tg = pi.tag;
            D.obs_u[tg] = 0.25 * ou;
            D.obs_w[tg] = 0.5 * ow;
            D.obs_np[tg] = onp;
            D.obs_ub[tg] = oub;
            D.obs_wb[tg] = owb;
            D.obs_ke[tg] = 0.5 * ((double)si.vx * si.vx + (double)si.vy * si.vy +
                                  (double)si.vz * si.vz);
            D.obs_p[3 * tg + 0] = (double)si.vx;
            D.obs_p[3 * tg + 1] = (double)si.vy;
            D.obs_p[3 * tg + 2] = (double)si.vz;
            continue;
        }
        if (!(isfinite(fx) && isfinite(fy) && isfinite(fz))) atomicOr(D.err, ERR_NONFINITE);

        SRec<T> *sp = &D.S[lay][slot];
        if (MODE == MODE_INIT) {
            sp->fx = fx;
            sp->fy = fy;
            sp->fz = fz;
            continue;
        }
        // Integrate-2 (Fig. 1 step 5): v <- v + dt (f + f') / 2, f <- f'.
        const T hdt = (T)0.5 * D.dt;
        const T vx = si.vx + hdt * (si.fx + fx);
        const T vy = si.vy + hdt * (si.fy + fy);
        const T vz = si.vz + hdt * (si.fz + fz);
        if (MODE == MODE_FINISH || fin) {
            sp->vx = vx;
            sp->vy = vy;
            sp->vz = vz;
            sp->fx = fx;
            sp->fy = fy;
            sp->fz = fz;
        } else {
            drift_and_bin<T>(D, q, si.x, si.y, si.z, vx, vy, vz, fx, fy, fz, pi.tag, pi.type,
                             nbond > 0);
        }
    }
}

// Waves per SIMD the integer-frame pair kernels are register-budgeted for.
#ifndef DPD_WAVES_PER_EU
#define DPD_WAVES_PER_EU 4
#endif

// BONDS = false drops the bond terms from the code (systems without bonds).
template <typename T, int BX, int BY, int BZ, int NT, int HCAP, int MODE, bool IGEO,
          bool BONDS = true>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(IGEO ? DPD_WAVES_PER_EU : 1)))
void k_force(DevSys<T> D, uint32_t q, int nbx, int nby, int nbricks, uint64_t thr) {
    force_brick<T, BX, BY, BZ, NT, HCAP, MODE, IGEO, BONDS>(D, q, xcd_brick(blockIdx.x, nbricks),
                                                            nbx, nby, nbricks / (nbx * nby), thr,
                                                            false);
}

// begin: integrate-1 and binning of every particle of resting state q; one
// thread per cell g of layout q (a wave's appends then go to many different
// cells).  The cell's records are read four at a time, their loads issued
// together, rather than one round trip per record.
template <typename T>
__device__ __forceinline__ void begin_cell(const DevSys<T> &D, uint32_t q, int64_t g) {
    if (g >= D.ncells) return;
    const uint32_t lay = q & 1u;
    D.count[count_index(q, 2u)][g] = 0u;
    const uint32_t n = min(D.count[count_index(q, 0u)][g], (uint32_t)D.cap);
    for (uint32_t k0 = 0; k0 < n; k0 += 4u) {
        SRec<T> s[4];
        PRec<T> p[4];
#pragma unroll
        for (uint32_t u = 0; u < 4u; ++u) {
            if (k0 + u < n) {
                const int64_t slot = g * D.cap + k0 + u;
                s[u] = D.S[lay][slot];
                p[u] = D.P[lay][slot];
            }
        }
#pragma unroll
        for (uint32_t u = 0; u < 4u; ++u) {
            if (k0 + u >= n) break;
            const bool bonded =
                D.bond_off && D.bond_off[p[u].tag + 1] > D.bond_off[p[u].tag];
            drift_and_bin<T>(D, q, s[u].x, s[u].y, s[u].z, s[u].vx, s[u].vy, s[u].vz, s[u].fx,
                             s[u].fy, s[u].fz, p[u].tag, p[u].type, bonded);
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_begin(DevSys<T> D, uint32_t q) {
    begin_cell<T>(D, q, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched kernels.  Window step k of a replica with window start t0 computes
// the forces of state q = t0 + k + 1 (the state begin or the previous pass
// moved it to), exactly as dpd_step does, so a replica follows the same
// trajectory bit for bit whatever else shares the batch.
// ---------------------------------------------------------------------------
// The replica table is read in place (a copy would be indexed dynamically and
// land in scratch); it is never written during a window, which the restrict
// qualifier tells the compiler, so its fields stay uniform scalar loads.
template <int BX, int BY, int BZ, int NT, int HCAP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DPD_WAVES_PER_EU)))
void k_force_batch(const BatchEnt *__restrict__ tab, BatchDev B, uint32_t k, uint32_t last) {
    const int nw = B.nwork[0];
    if ((int)blockIdx.x >= nw) return;
    const BatchWork w = B.wf[xcd_brick(blockIdx.x, nw)];
    const uint32_t t0 = B.t0[w.slot], tgt = B.target[w.slot];
    if (tgt - t0 <= k) return;     // the replica reached its target earlier
    const uint32_t q = t0 + k + 1u;
    const BatchEnt &E = tab[w.slot];
    force_brick<float, BX, BY, BZ, NT, HCAP, MODE_FUSED, true, true>(
        E.D, q, (int)w.item, E.nbx, E.nby, E.nbz, E.thr, q == tgt || last != 0u);
}

__global__ __launch_bounds__(256) void k_begin_batch(const BatchEnt *__restrict__ tab,
                                                     BatchDev B) {
    if ((int)blockIdx.x >= B.nwork[1]) return;
    const BatchWork w = B.wb[blockIdx.x];
    const uint32_t t0 = B.t0[w.slot];
    if (t0 >= B.target[w.slot]) return;
    begin_cell<float>(tab[w.slot].D, t0, (int64_t)w.item * 256 + threadIdx.x);
}

__global__ __launch_bounds__(256) void k_end_batch(BatchDev B, uint32_t K) {
    const int slot = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (slot >= B.nwork[2]) return;
    const uint32_t t0 = B.t0[slot], tgt = B.target[slot];
    const uint32_t t = t0 + min(K, tgt - t0);
    const uint32_t *err = B.tab[slot].D.err;
    B.t0[slot] = t;
    B.status[2 * slot] = t;
    B.status[2 * slot + 1] = err ? *err : 0u;
}

// load: bins host-provided state (tag order) into the layout of state q.
// vt = v, so a following MODE_INIT pass computes F(x, v; s = q).
template <typename T>
__global__ __launch_bounds__(256) void k_load(DevSys<T> D, uint32_t q, const double *x,
                                              const double *v, const double *f,
                                              const uint8_t *type) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D.n) return;
    double px = wrap_coord(x[3 * i + 0], D.L[0]);
    double py = wrap_coord(x[3 * i + 1], D.L[1]);
    double pz = wrap_coord(x[3 * i + 2], D.L[2]);
    const int cx = cell_coord(px, D.h[0], D.nc[0]);
    const int cy = cell_coord(py, D.h[1], D.nc[1]);
    const int cz = cell_coord(pz, D.h[2], D.nc[2]);
    const int64_t g = cell_linear(cx, cy, cz, D.nc);
    const uint32_t k = atomicAdd(&D.count[count_index(q, 0u)][g], 1u);
    if (k >= (uint32_t)D.cap) {
        atomicOr(D.err, ERR_CELL_OVERFLOW);
        return;
    }
    const int64_t slot = g * D.cap + k;
    const uint32_t lay = q & 1u;
    PRec<T> p;
    p.ox = Geo<T>::encode(px, cx, D.h[0]);
    p.oy = Geo<T>::encode(py, cy, D.h[1]);
    p.oz = Geo<T>::encode(pz, cz, D.h[2]);
    p.tag = (uint32_t)i;
    p.vx = (T)v[3 * i + 0];
    p.vy = (T)v[3 * i + 1];
    p.vz = (T)v[3 * i + 2];
    p.type = type ? type[i] : 0u;
    D.P[lay][slot] = p;
    SRec<T> s;
    s.x = px;
    s.y = py;
    s.z = pz;
    s.vx = p.vx;
    s.vy = p.vy;
    s.vz = p.vz;
    s.fx = f ? (T)f[3 * i + 0] : (T)0;
    s.fy = f ? (T)f[3 * i + 1] : (T)0;
    s.fz = f ? (T)f[3 * i + 2] : (T)0;
    D.S[lay][slot] = s;
    D.slot_of_tag[lay][i] = (uint32_t)slot;
}

// gather: copies the state of layout q to tag-order FP64 arrays.
template <typename T>
__global__ __launch_bounds__(256) void k_gather(DevSys<T> D, uint32_t q, double *x, double *v,
                                                double *f, int64_t *cell) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= D.n) return;
    const uint32_t lay = q & 1u;
    uint32_t slot = D.slot_of_tag[lay][i];
    if ((int64_t)slot >= D.ncells * D.cap) {
        atomicOr(D.err, ERR_INDEX);
        slot = 0;
    }
    const SRec<T> s = D.S[lay][slot];
    x[3 * i + 0] = s.x;
    x[3 * i + 1] = s.y;
    x[3 * i + 2] = s.z;
    v[3 * i + 0] = (double)s.vx;
    v[3 * i + 1] = (double)s.vy;
    v[3 * i + 2] = (double)s.vz;
    f[3 * i + 0] = (double)s.fx;
    f[3 * i + 1] = (double)s.fy;
    f[3 * i + 2] = (double)s.fz;
    cell[i] = (int64_t)(slot / (uint32_t)D.cap);
}

// Rebuilds the full tag -> slot map of layout q (one thread per cell).
template <typename T>
__global__ __launch_bounds__(256) void k_slotmap(DevSys<T> D, uint32_t q) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= D.ncells) return;
    const uint32_t lay = q & 1u;
    const uint32_t n = min(D.count[count_index(q, 0u)][g], (uint32_t)D.cap);
    for (uint32_t k = 0; k < n; ++k) {
        const int64_t slot = g * D.cap + k;
        const uint32_t tag = D.P[lay][slot].tag;
        if ((int64_t)tag < D.n) D.slot_of_tag[lay][tag] = (uint32_t)slot;
        else atomicOr(D.err, ERR_INDEX);
    }
}

// theta_ij(s) for m triples, in the force precision T.
template <typename T>
__global__ __launch_bounds__(256) void k_noise(uint64_t seed, int64_t m, const uint32_t *ti,
                                               const uint32_t *tj, const uint32_t *s,
                                               double *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] = (double)pair_theta<T>(seed, ti[i], tj[i], s[i]);
}

hipError_t launch_noise(int precision_fp64, uint64_t seed, int64_t m, const uint32_t *ti,
                        const uint32_t *tj, const uint32_t *s, double *out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    const dim3 g((unsigned)((m + 255) / 256));
    if (precision_fp64)
        hipLaunchKernelGGL(k_noise<double>, g, dim3(256), 0, st, seed, m, ti, tj, s, out);
    else
        hipLaunchKernelGGL(k_noise<float>, g, dim3(256), 0, st, seed, m, ti, tj, s, out);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t m, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = v;
}

// Deterministic sums of K per-tag arrays: block b adds tags [b*chunk,
// (b+1)*chunk) in a fixed tree and writes out[b*K + k].
template <int K>
__global__ __launch_bounds__(256) void k_reduce(const double *const *in, int64_t m, int64_t chunk,
                                                double *out) {
    __shared__ double s[256];
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = min(lo + chunk, m);
    for (int k = 0; k < K; ++k) {
        double acc = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) acc += in[k][i];
        s[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) out[(int64_t)blockIdx.x * K + k] = s[0];
        __syncthreads();
    }
}

// Pair counts are integers; u32 -> double per tag before the reduction.
__global__ __launch_bounds__(256) void k_u32_to_f64(const uint32_t *a, double *b, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) b[i] = (double)a[i];
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------

template <typename T, int BX, int BY, int BZ, int NT, int HCAP, bool IGEO>
static hipError_t launch_force_g(const DevSys<T> &D, uint32_t q, int mode, hipStream_t st) {
    const int nbx = (D.nc[0] + BX - 1) / BX, nby = (D.nc[1] + BY - 1) / BY,
              nbz = (D.nc[2] + BZ - 1) / BZ;
    const int nb = nbx * nby * nbz;
    // Cutoff r^2 < 1 in squared fixed-point units: sum dq^2 < (2^29 / h)^2.
    const double lim = 536870912.0 / D.h[0];
    const uint64_t thr = (uint64_t)std::ceil(lim * lim);
    switch (mode) {
    case MODE_INIT:
        hipLaunchKernelGGL((k_force<T, BX, BY, BZ, NT, HCAP, MODE_INIT, IGEO>), dim3(nb), dim3(NT),
                           0, st, D, q, nbx, nby, nb, thr);
        break;
    case MODE_FINISH:
        hipLaunchKernelGGL((k_force<T, BX, BY, BZ, NT, HCAP, MODE_FINISH, IGEO>), dim3(nb),
                           dim3(NT), 0, st, D, q, nbx, nby, nb, thr);
        break;
    case MODE_FUSED:
        // The step kernel of mixed-precision cubic systems comes without bond
        // code for systems that have no bonds.
        if (IGEO && !D.bond_off)
            hipLaunchKernelGGL((k_force<T, BX, BY, BZ, NT, HCAP, MODE_FUSED, IGEO, !IGEO>),
                               dim3(nb), dim3(NT), 0, st, D, q, nbx, nby, nb, thr);
        else
            hipLaunchKernelGGL((k_force<T, BX, BY, BZ, NT, HCAP, MODE_FUSED, IGEO>), dim3(nb),
                               dim3(NT), 0, st, D, q, nbx, nby, nb, thr);
        break;
    default:
        hipLaunchKernelGGL((k_force<T, BX, BY, BZ, NT, HCAP, MODE_OBS, IGEO>), dim3(nb), dim3(NT),
                           0, st, D, q, nbx, nby, nb, thr);
        break;
    }
    return hipGetLastError();
}

// Mixed precision with cubic cells uses the integer brick frame.
template <typename T, int BX, int BY, int BZ, int NT, int HCAP>
static hipError_t launch_force_v(const DevSys<T> &D, uint32_t q, int mode, hipStream_t st) {
    if constexpr (std::is_same<T, float>::value) {
        if (D.h[0] == D.h[1] && D.h[0] == D.h[2])
            return launch_force_g<T, BX, BY, BZ, NT, HCAP, true>(D, q, mode, st);
    }
    return launch_force_g<T, BX, BY, BZ, NT, HCAP, false>(D, q, mode, st);
}

// Brick variants, selected by index: {BX, BY, BZ, threads, LDS capacity}.  The
// capacity sits ~5 standard deviations above a rho = 3 neighbourhood's mean;
// denser neighbourhoods are processed in chunks.  Variants 5 and 6 take a
// brick with half the threads (about two particles per thread, in two passes
// over the staged neighbourhood): smaller work-groups for small boxes.
#define DPD_VARIANTS(X)                                                                   \
    X(0, 4, 4, 4, 256, 800)                                                               \
    X(1, 5, 4, 4, 256, 896)                                                               \
    X(2, 5, 5, 4, 320, 1056)                                                              \
    X(3, 4, 4, 2, 128, 540)                                                               \
    X(4, 2, 2, 2, 64, 256)                                                                \
    X(5, 5, 4, 4, 128, 896)                                                               \
    X(6, 4, 4, 4, 128, 800)
constexpr int NVARIANTS = 7;

template <typename T>
hipError_t launch_force(const DevSys<T> &D, uint32_t q, int mode, int variant, hipStream_t st) {
    switch (variant) {
#define DPD_CASE(i, bx, by, bz, nt, hc)                                                   \
    case i: return launch_force_v<T, bx, by, bz, nt, hc>(D, q, mode, st);
        DPD_VARIANTS(DPD_CASE)
#undef DPD_CASE
    default: return hipErrorInvalidValue;
    }
}

int force_variant_count() { return NVARIANTS; }

void force_variant_shape(int variant, int out[5]) {
    static const int t[NVARIANTS][5] = {
#define DPD_ROW(i, bx, by, bz, nt, hc) {bx, by, bz, nt, hc},
        DPD_VARIANTS(DPD_ROW)
#undef DPD_ROW
    };
    for (int k = 0; k < 5; ++k) out[k] = t[variant][k];
}

template <int BX, int BY, int BZ, int NT, int HCAP>
static hipError_t launch_batch_v(const BatchDev &B, int K, int cap_force, int cap_begin,
                                 int cap_slots, hipStream_t st) {
    if (cap_begin > 0)
        hipLaunchKernelGGL(k_begin_batch, dim3(cap_begin), dim3(256), 0, st, B.tab, B);
    for (int k = 0; k < K && cap_force > 0; ++k)
        hipLaunchKernelGGL((k_force_batch<BX, BY, BZ, NT, HCAP>), dim3(cap_force), dim3(NT), 0, st,
                           B.tab, B, (uint32_t)k, (uint32_t)(k == K - 1));
    hipLaunchKernelGGL(k_end_batch, dim3((cap_slots + 255) / 256), dim3(256), 0, st, B,
                       (uint32_t)K);
    return hipGetLastError();
}

hipError_t launch_batch_window(const BatchDev &B, int variant, int K, int cap_force,
                               int cap_begin, int cap_slots, hipStream_t st) {
    if (K < 1 || cap_slots < 1) return hipErrorInvalidValue;
    switch (variant) {
#define DPD_CASE(i, bx, by, bz, nt, hc)                                                   \
    case i: return launch_batch_v<bx, by, bz, nt, hc>(B, K, cap_force, cap_begin, cap_slots, st);
        DPD_VARIANTS(DPD_CASE)
#undef DPD_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename T> hipError_t launch_begin(const DevSys<T> &D, uint32_t q, hipStream_t st) {
    const int64_t nb = (D.ncells + 255) / 256;
    hipLaunchKernelGGL(k_begin<T>, dim3((unsigned)nb), dim3(256), 0, st, D, q);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_load(const DevSys<T> &D, uint32_t q, const double *x, const double *v,
                       const double *f, const uint8_t *type, hipStream_t st) {
    const int64_t nb = (D.n + 255) / 256;
    hipLaunchKernelGGL(k_load<T>, dim3((unsigned)nb), dim3(256), 0, st, D, q, x, v, f, type);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const DevSys<T> &D, uint32_t q, double *x, double *v, double *f,
                         int64_t *cell, hipStream_t st) {
    const int64_t nc = (D.ncells + 255) / 256;
    hipLaunchKernelGGL(k_slotmap<T>, dim3((unsigned)nc), dim3(256), 0, st, D, q);
    const int64_t nb = (D.n + 255) / 256;
    hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)nb), dim3(256), 0, st, D, q, x, v, f, cell);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t m, uint32_t v, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, p, m, v);
    return hipGetLastError();
}

hipError_t launch_u32_to_f64(const uint32_t *a, double *b, int64_t m, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_u32_to_f64, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, st, a, b,
                       m);
    return hipGetLastError();
}

hipError_t launch_reduce8(const double *const *in, int64_t m, int64_t chunk, int nblocks,
                          double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce<8>, dim3(nblocks), dim3(256), 0, st, in, m, chunk, out);
    return hipGetLastError();
}

template hipError_t launch_force<float>(const DevSys<float> &, uint32_t, int, int, hipStream_t);
template hipError_t launch_force<double>(const DevSys<double> &, uint32_t, int, int, hipStream_t);
template hipError_t launch_begin<float>(const DevSys<float> &, uint32_t, hipStream_t);
template hipError_t launch_begin<double>(const DevSys<double> &, uint32_t, hipStream_t);
template hipError_t launch_load<float>(const DevSys<float> &, uint32_t, const double *,
                                       const double *, const double *, const uint8_t *,
                                       hipStream_t);
template hipError_t launch_load<double>(const DevSys<double> &, uint32_t, const double *,
                                        const double *, const double *, const uint8_t *,
                                        hipStream_t);
template hipError_t launch_gather<float>(const DevSys<float> &, uint32_t, double *, double *,
                                         double *, int64_t *, hipStream_t);
template hipError_t launch_gather<double>(const DevSys<double> &, uint32_t, double *, double *,
                                          double *, int64_t *, hipStream_t);

}  // namespace dpd
