// C ABI of the DPD step library (include/dpd.h): system lifetime, parameter
// and bond upload, the step schedule, state and observable read-back.
#include <hip/hip_runtime.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/dpd.h"
#include "dpd_device.hpp"
#include "dpd_kernels.hpp"

using namespace dpd;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_OK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(DPD_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

template <typename T> size_t prec_size() { return sizeof(T); }

// A system's device buffers live in one allocation (and its bond tables in a
// second one, made at the first step), each buffer at a 256-byte boundary.
enum Buf : int {
    B_P0, B_P1, B_S0, B_S1, B_SOT0, B_SOT1, B_CNT0, B_CNT1, B_CNT2, B_A, B_ERR, B_STAGE,
    B_CSTAGE, B_TYPE, B_OBS, B_OBSNP, B_OBSPTR, B_RED, B_NBUF
};

int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Largest state index: kernels take it as 32 bits (noise counter word 2, the
// layout parity and the count-array rotation modulo 3).
constexpr int64_t STEP_LIMIT = (int64_t)0xFFFFFFFF;

int red_blocks_for(int64_t n) { return (int)std::min<int64_t>(256, (n + 1023) / 1024); }

struct Layout {
    int64_t off[B_NBUF];
    int64_t total;
};

Layout system_layout(int prec, int64_t ncells, int64_t n, int cap) {
    const int64_t psz = prec == DPD_PREC_FP64 ? sizeof(PRec<double>) : sizeof(PRec<float>);
    const int64_t ssz = prec == DPD_PREC_FP64 ? sizeof(SRec<double>) : sizeof(SRec<float>);
    const int64_t slots = ncells * cap;
    int64_t size[B_NBUF];
    size[B_P0] = size[B_P1] = slots * psz;
    size[B_S0] = size[B_S1] = slots * ssz;
    size[B_SOT0] = size[B_SOT1] = n * (int64_t)sizeof(uint32_t);
    size[B_CNT0] = size[B_CNT1] = size[B_CNT2] = ncells * (int64_t)sizeof(uint32_t);
    size[B_A] = 256 * (int64_t)sizeof(double);
    size[B_ERR] = sizeof(uint32_t);
    size[B_STAGE] = 9 * n * (int64_t)sizeof(double);      // x, v, f in tag order
    size[B_CSTAGE] = n * (int64_t)sizeof(int64_t);
    size[B_TYPE] = n;
    size[B_OBS] = 9 * n * (int64_t)sizeof(double);        // per-tag observables
    size[B_OBSNP] = n * (int64_t)sizeof(uint32_t);
    size[B_OBSPTR] = 8 * (int64_t)sizeof(double *);
    size[B_RED] = (int64_t)red_blocks_for(n) * 8 * (int64_t)sizeof(double);
    Layout L;
    int64_t o = 0;
    for (int k = 0; k < B_NBUF; ++k) {
        L.off[k] = o;
        o += align256(size[k]);
    }
    L.total = o;
    return L;
}

int64_t bond_block_bytes(int64_t n, int64_t nb) {
    return align256((n + 1) * (int64_t)sizeof(uint32_t)) +
           align256(2 * nb * (int64_t)sizeof(BondEnt<double>));
}

// Device bytes dpd_create allocates for a system, plus what dpd_add_bonds
// adds at the first step for nb bond records.
int64_t footprint(int prec, const int nc[3], int64_t n, int64_t nb, int cap) {
    const int64_t ncells = (int64_t)nc[0] * nc[1] * nc[2];
    int64_t b = system_layout(prec, ncells, n, cap).total;
    if (nb > 0) b += bond_block_bytes(n, nb);
    return b;
}

}  // namespace

struct dpd_batch;

struct dpd_system {
    int prec = DPD_PREC_MIXED;
    int64_t n = 0;
    double L[3] = {0, 0, 0}, h[3] = {0, 0, 0};
    int nc[3] = {0, 0, 0};
    int64_t ncells = 0;
    int cap = 32;
    int ntypes = 1;
    uint64_t seed = 0;
    int dev = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;

    bool params_set = false;
    std::vector<double> a;
    double gamma = 0, sigma = 0, kT = 1, dt = 0, lambda = 0.65;

    std::vector<int32_t> btype;
    std::vector<int64_t> bi, bj;
    std::vector<double> bre, bk, balpha;
    bool frozen = false;

    // Device memory.
    void *P[2] = {nullptr, nullptr};
    void *S[2] = {nullptr, nullptr};
    uint32_t *slot_of_tag[2] = {nullptr, nullptr};
    uint32_t *count[3] = {nullptr, nullptr, nullptr};
    void *a_dev = nullptr;
    uint32_t *bond_off = nullptr;
    void *bonds = nullptr;
    uint32_t *err = nullptr;
    void *block = nullptr;          // the one allocation holding the buffers below
    void *bond_block = nullptr;     // bond CSR and records
    double *stage = nullptr;        // 9n doubles: x, v, f in tag order
    int64_t *cell_stage = nullptr;  // n
    uint8_t *type_dev = nullptr;
    double *obs = nullptr;          // 9n doubles: per-tag observables
    uint32_t *obs_np = nullptr;
    double **obs_ptrs = nullptr;    // 8 device pointers for the reduction
    double *red = nullptr;          // partial sums
    int red_blocks = 0;
    size_t bytes = 0;

    int64_t t = 0;                  // state index of the resting state
    bool force_valid = false;
    dpd_batch *batch = nullptr;     // the batch this system is resident in, if any
    int batch_slot = -1;
    int variant = 0;
    int sticky = DPD_OK;
    std::string sticky_msg;
};

namespace {

template <typename T> DevSys<T> make_dev(const dpd_system *s) {
    DevSys<T> D;
    std::memset(&D, 0, sizeof D);
    for (int k = 0; k < 3; ++k) {
        D.L[k] = s->L[k];
        D.h[k] = s->h[k];
        D.nc[k] = s->nc[k];
    }
    D.cap = s->cap;
    D.ncells = s->ncells;
    D.n = s->n;
    D.ntypes = s->ntypes;
    D.dt = (T)s->dt;
    D.lambda = (T)s->lambda;
    D.gamma = (T)s->gamma;
    D.sigma_rdt = s->dt > 0 ? (T)(s->sigma / std::sqrt(s->dt)) : (T)0;
    D.dt_d = s->dt;
    D.half_dt2_d = 0.5 * s->dt * s->dt;
    D.seed = s->seed;
    D.a = (const T *)s->a_dev;
    for (int k = 0; k < 2; ++k) {
        D.P[k] = (PRec<T> *)s->P[k];
        D.S[k] = (SRec<T> *)s->S[k];
        D.slot_of_tag[k] = s->slot_of_tag[k];
    }
    for (int k = 0; k < 3; ++k) D.count[k] = s->count[k];
    D.bond_off = s->bond_off;
    D.bonds = (const BondEnt<T> *)s->bonds;
    D.err = s->err;
    const int64_t n = s->n;
    D.obs_u = s->obs;
    D.obs_w = s->obs + n;
    D.obs_ub = s->obs + 2 * n;
    D.obs_wb = s->obs + 3 * n;
    D.obs_ke = s->obs + 4 * n;
    D.obs_p = s->obs + 6 * n;   // 3n, after the pair-count copy at 5n
    D.obs_np = s->obs_np;
    return D;
}

// ---------------------------------------------------------------------------
// Reuse across systems.  hipFree waits for every stream of the device (a
// batch window included), hipStreamCreate costs milliseconds, and pageable
// host copies are slow, all measured on MI355X; a serving loop creates and
// destroys systems while windows run.  So device blocks and streams of
// destroyed systems are kept for later systems (blocks by size class, at most
// REUSE_BYTES per device), and host arrays reach the device through one
// pinned staging buffer.
// ---------------------------------------------------------------------------
struct Reuse {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<void *>> blocks;   // (device, class)
    std::map<void *, std::pair<int, size_t>> live;                  // block -> (device, class)
    std::map<int, size_t> held;                                     // kept bytes per device
    std::map<int, std::vector<hipStream_t>> streams;
    std::mutex stage_mu;
    void *stage = nullptr;
    size_t stage_bytes = 0;
};
// Never destroyed: no HIP call may run from a static destructor at exit.
Reuse &reuse() {
    static Reuse *r = new Reuse();
    return *r;
}
constexpr size_t REUSE_BYTES = (size_t)4 << 30;
constexpr size_t REUSE_STREAMS = 64;
constexpr size_t STAGE_MAX = (size_t)256 << 20;

// Block size class: 4 KiB granules up to 64 KiB, then 16 classes per octave
// (at most 1/8 over the request).
size_t size_class(size_t b) {
    if (b <= ((size_t)64 << 10)) return (b + 4095) & ~(size_t)4095;
    size_t pw = 1;
    while (pw < b) pw <<= 1;
    const size_t step = pw / 16;
    return (b + step - 1) / step * step;
}

int dmalloc(dpd_system *s, void **p, size_t bytes) {
    Reuse &r = reuse();
    const size_t cls = size_class(bytes);
    *p = nullptr;
    {
        std::lock_guard<std::mutex> g(r.mu);
        auto it = r.blocks.find({s->dev, cls});
        if (it != r.blocks.end() && !it->second.empty()) {
            *p = it->second.back();
            it->second.pop_back();
            r.held[s->dev] -= cls;
            r.live[*p] = {s->dev, cls};
        }
    }
    if (!*p) {
        hipError_t e = hipMalloc(p, cls);
        if (e != hipSuccess) {
            // Give the kept blocks of this device back and try once more.
            std::vector<void *> drop;
            {
                std::lock_guard<std::mutex> g(r.mu);
                for (auto &kv : r.blocks)
                    if (kv.first.first == s->dev) {
                        drop.insert(drop.end(), kv.second.begin(), kv.second.end());
                        kv.second.clear();
                    }
                r.held[s->dev] = 0;
            }
            for (void *q : drop) (void)hipFree(q);
            e = hipMalloc(p, cls);
        }
        if (e != hipSuccess) {
            *p = nullptr;
            return fail(DPD_ENOMEM, "hipMalloc(%zu) failed: %s", cls, hipGetErrorString(e));
        }
        std::lock_guard<std::mutex> g(r.mu);
        r.live[*p] = {s->dev, cls};
    }
    s->bytes += bytes;
    return DPD_OK;
}

// Keeps a block that no device work refers to any more for a later system.
void dfree(void *p) {
    if (!p) return;
    Reuse &r = reuse();
    {
        std::lock_guard<std::mutex> g(r.mu);
        auto it = r.live.find(p);
        if (it != r.live.end()) {
            const auto key = it->second;
            r.live.erase(it);
            if (r.held[key.first] + key.second <= REUSE_BYTES) {
                r.blocks[key].push_back(p);
                r.held[key.first] += key.second;
                return;
            }
        }
    }
    (void)hipFree(p);
}

// The system's blocks go back once its stream is idle (a batch that held it
// has already waited for its windows when it let the system go).
void free_all(dpd_system *s) {
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    dfree(s->block);
    dfree(s->bond_block);
    s->block = s->bond_block = nullptr;
}

hipError_t stream_take(int dev, hipStream_t *st) {
    Reuse &r = reuse();
    {
        std::lock_guard<std::mutex> g(r.mu);
        auto &v = r.streams[dev];
        if (!v.empty()) {
            *st = v.back();
            v.pop_back();
            return hipSuccess;
        }
    }
    return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
}

// Returns a library-owned stream, once idle, for a later system.
void release_stream(dpd_system *s) {
    if (!s->own_stream || !s->stream) return;
    (void)hipStreamSynchronize(s->stream);
    Reuse &r = reuse();
    {
        std::lock_guard<std::mutex> g(r.mu);
        auto &v = r.streams[s->dev];
        if (v.size() < REUSE_STREAMS) {
            v.push_back(s->stream);
            s->stream = nullptr;
            return;
        }
    }
    (void)hipStreamDestroy(s->stream);
    s->stream = nullptr;
}

// Host -> device copy of caller memory through the pinned staging buffer;
// returns once the copy is complete (the buffer is reused by the next copy).
int h2d(void *dst, const void *src, size_t bytes, hipStream_t st) {
    if (bytes == 0) return DPD_OK;
    Reuse &r = reuse();
    std::lock_guard<std::mutex> g(r.stage_mu);
    if (bytes <= STAGE_MAX && r.stage_bytes < bytes) {
        if (r.stage) (void)hipHostFree(r.stage);
        r.stage = nullptr;
        r.stage_bytes = 0;
        size_t nb = (size_t)1 << 20;
        while (nb < bytes) nb <<= 1;
        if (hipHostMalloc(&r.stage, nb, hipHostMallocDefault) == hipSuccess) r.stage_bytes = nb;
        else r.stage = nullptr;
    }
    if (r.stage_bytes >= bytes) {
        std::memcpy(r.stage, src, bytes);
        HIP_OK(hipMemcpyAsync(dst, r.stage, bytes, hipMemcpyHostToDevice, st));
    } else {
        HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    }
    HIP_OK(hipStreamSynchronize(st));
    return DPD_OK;
}

// Reads the device error word; converts it to a sticky status.
int check_device(dpd_system *s) {
    if (s->sticky != DPD_OK) return fail(s->sticky, "%s", s->sticky_msg.c_str());
    HIP_OK(hipStreamSynchronize(s->stream));
    uint32_t e = 0;
    HIP_OK(hipMemcpy(&e, s->err, sizeof e, hipMemcpyDeviceToHost));
    if (e == 0) return DPD_OK;
    int code = DPD_EDEVICE;
    const char *what = "internal index error";
    if (e & ERR_CELL_OVERFLOW) {
        code = DPD_ECAPACITY;
        what = "a cell received more particles than its slots (raise cell_capacity)";
    } else if (e & ERR_TILE_OVERFLOW) {
        code = DPD_ECAPACITY;
        what = "a brick's neighbourhood exceeded the tile buffer (local density too high)";
    } else if (e & ERR_NONFINITE) {
        code = DPD_ENUMERIC;
        what = "non-finite position, velocity or force";
    } else if (e & ERR_DISPLACEMENT) {
        code = DPD_ENUMERIC;
        what = "a particle moved more than half a box in one step";
    }
    s->sticky = code;
    s->sticky_msg = std::string("device error: ") + what;
    return fail(code, "%s", s->sticky_msg.c_str());
}

template <typename T> int upload_params(dpd_system *s) {
    std::vector<T> a(s->a.begin(), s->a.end());
    if (int rc = h2d(s->a_dev, a.data(), a.size() * sizeof(T), s->stream)) return rc;
    // Bond CSR over tags: each record appears at both of its ends.
    const int64_t n = s->n, nb = (int64_t)s->btype.size();
    if (nb > 0) {
        std::vector<uint32_t> off(n + 1, 0);
        for (int64_t b = 0; b < nb; ++b) {
            off[s->bi[b] + 1]++;
            off[s->bj[b] + 1]++;
        }
        for (int64_t i = 0; i < n; ++i) off[i + 1] += off[i];
        std::vector<BondEnt<T>> ent(2 * nb);
        std::vector<uint32_t> fill(off.begin(), off.end() - 1);
        for (int64_t b = 0; b < nb; ++b) {
            BondEnt<T> e;
            e.type = s->btype[b];
            e.r_e = s->bre[b];
            e.k = s->bk[b];
            e.alpha = s->balpha[b];
            e.partner = (uint32_t)s->bj[b];
            ent[fill[s->bi[b]]++] = e;
            e.partner = (uint32_t)s->bi[b];
            ent[fill[s->bj[b]]++] = e;
        }
        static_assert(sizeof(BondEnt<T>) == sizeof(BondEnt<double>), "bond record size");
        if (dmalloc(s, &s->bond_block, (size_t)bond_block_bytes(n, nb))) return DPD_ENOMEM;
        s->bond_off = (uint32_t *)s->bond_block;
        s->bonds = (char *)s->bond_block + align256((n + 1) * (int64_t)sizeof(uint32_t));
        if (int rc = h2d(s->bond_off, off.data(), off.size() * sizeof(uint32_t), s->stream))
            return rc;
        if (int rc = h2d(s->bonds, ent.data(), ent.size() * sizeof(BondEnt<T>), s->stream))
            return rc;
    }
    return DPD_OK;
}

int freeze(dpd_system *s) {
    if (s->frozen) return DPD_OK;
    if (!s->params_set) return fail(DPD_ESTATE, "dpd_set_params must be called before stepping");
    int rc = s->prec == DPD_PREC_FP64 ? upload_params<double>(s) : upload_params<float>(s);
    if (rc) return rc;
    s->frozen = true;
    return DPD_OK;
}

template <typename T> int run_force(dpd_system *s, uint32_t q, int mode) {
    const DevSys<T> D = make_dev<T>(s);
    HIP_OK(launch_force<T>(D, q, mode, s->variant, s->stream));
    return DPD_OK;
}

int force(dpd_system *s, uint32_t q, int mode) {
    return s->prec == DPD_PREC_FP64 ? run_force<double>(s, q, mode) : run_force<float>(s, q, mode);
}

int begin(dpd_system *s, uint32_t q) {
    if (s->prec == DPD_PREC_FP64) HIP_OK(launch_begin<double>(make_dev<double>(s), q, s->stream));
    else HIP_OK(launch_begin<float>(make_dev<float>(s), q, s->stream));
    return DPD_OK;
}

int ensure_force(dpd_system *s) {
    if (s->force_valid) return DPD_OK;
    int rc = force(s, (uint32_t)s->t, FORCE_INIT);
    if (rc) return rc;
    s->force_valid = true;
    return DPD_OK;
}

// Uploads host state (tag order) and bins it as state t.
int load_state(dpd_system *s, const double *pos, const double *vel, const double *frc,
               int64_t t) {
    const int64_t n = s->n;
    if (int rc = h2d(s->stage, pos, 3 * n * sizeof(double), s->stream)) return rc;
    if (int rc = h2d(s->stage + 3 * n, vel, 3 * n * sizeof(double), s->stream)) return rc;
    if (frc)
        if (int rc = h2d(s->stage + 6 * n, frc, 3 * n * sizeof(double), s->stream)) return rc;
    for (int k = 0; k < 3; ++k) HIP_OK(launch_fill_u32(s->count[k], s->ncells, 0u, s->stream));
    const uint32_t q = (uint32_t)t;
    if (s->prec == DPD_PREC_FP64)
        HIP_OK(launch_load<double>(make_dev<double>(s), q, s->stage, s->stage + 3 * n,
                                   frc ? s->stage + 6 * n : nullptr, s->type_dev, s->stream));
    else
        HIP_OK(launch_load<float>(make_dev<float>(s), q, s->stage, s->stage + 3 * n,
                                  frc ? s->stage + 6 * n : nullptr, s->type_dev, s->stream));
    // The host arrays may be released by the caller after return.
    HIP_OK(hipStreamSynchronize(s->stream));
    s->t = t;
    s->force_valid = frc != nullptr;
    return DPD_OK;
}

int cells_default_variant(const dpd_system *s) {
    return s->ncells >= 64 * 1024 ? 0 : (s->ncells >= 8 * 1024 ? 3 : 4);
}

bool all_finite(const double *p, int64_t m) {
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int check_usable(dpd_system *s) {
    if (!s) return fail(DPD_EINVAL, "null system");
    if (s->batch) return fail(DPD_EBUSY, "the system is resident in a batch; retire it first");
    if (s->sticky != DPD_OK) return fail(s->sticky, "%s", s->sticky_msg.c_str());
    return DPD_OK;
}

// ---------------------------------------------------------------------------
// Autotuner cache.  With DPD_TUNE_CACHE naming a file, dpd_autotune keeps the
// brick variant it picked for each class of system there (a JSON object, one
// entry per line, rewritten through a temporary file and a rename), and a
// later call for the same class, in this process or another, takes the entry
// without timing anything.  The class: device architecture, precision,
// number of particle types, cell count (power-of-two size class), particles
// per cell (rounded), cubic or non-cubic cells, and a hash of the variant
// table, so entries of another table are not reused.
// ---------------------------------------------------------------------------
std::string tune_key(const dpd_system *s) {
    std::string arch = "unknown";
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, s->dev) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t c = arch.find(':');
        if (c != std::string::npos) arch.resize(c);
    }
    int lg = 0;
    while (((int64_t)1 << (lg + 1)) <= s->ncells) ++lg;
    const long dens = std::lround((double)s->n / (double)s->ncells);
    uint32_t h = 2166136261u;       // FNV-1a over the variant shapes
    for (int v = 0; v < force_variant_count(); ++v) {
        int sh[5];
        force_variant_shape(v, sh);
        for (int k = 0; k < 5; ++k) {
            h ^= (uint32_t)sh[k];
            h *= 16777619u;
        }
    }
    const bool cubic = s->h[0] == s->h[1] && s->h[0] == s->h[2];
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s|%s|types%d|cells2^%d|rho%ld|%s|table%08x", arch.c_str(),
                  s->prec == DPD_PREC_FP64 ? "fp64" : "mixed", s->ntypes, lg, dens,
                  cubic ? "cubic" : "noncubic", h);
    return buf;
}

// Entries of a cache file: key -> (variant, ms).  Lines that are not entries
// ("{", "}") or do not parse are skipped.
std::map<std::string, std::pair<int, double>> tune_read(const char *path) {
    std::map<std::string, std::pair<int, double>> m;
    FILE *f = std::fopen(path, "r");
    if (!f) return m;
    char line[1024];
    while (std::fgets(line, sizeof line, f)) {
        const char *q1 = std::strchr(line, '"');
        if (!q1) continue;
        const char *q2 = std::strchr(q1 + 1, '"');
        if (!q2) continue;
        int v = -1;
        double ms = 0.0;
        if (std::sscanf(q2 + 1, ": {\"variant\": %d, \"ms\": %lf", &v, &ms) == 2)
            m[std::string(q1 + 1, q2)] = {v, ms};
    }
    std::fclose(f);
    return m;
}

void tune_write(const char *path, const std::map<std::string, std::pair<int, double>> &m) {
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &e : m)
        std::fprintf(f, "\"%s\": {\"variant\": %d, \"ms\": %.17g}%s\n", e.first.c_str(),
                     e.second.first, e.second.second, ++k < m.size() ? "," : "");
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

int batch_detach(dpd_batch *b, int slot);

}  // namespace

extern "C" {

int dpd_version(void) { return DPD_ABI_VERSION; }

const char *dpd_last_error(void) { return g_err.c_str(); }

int dpd_create(dpd_system **out, const double L[3], int64_t n, const double *pos,
               const double *vel, const uint8_t *type, int ntypes, uint64_t seed, int precision,
               void *hip_stream, int cell_capacity) {
    g_err.clear();
    if (!out || !L || !pos || !vel) return fail(DPD_EINVAL, "null argument");
    *out = nullptr;
    if (n < 2) return fail(DPD_EINVAL, "need at least 2 particles, got %lld", (long long)n);
    if (n >= (int64_t)0xFFFFFFFF) return fail(DPD_EINVAL, "too many particles");
    if (precision != DPD_PREC_FP64 && precision != DPD_PREC_MIXED)
        return fail(DPD_EINVAL, "unknown precision %d", precision);
    if (ntypes < 1 || ntypes > 16) return fail(DPD_EINVAL, "ntypes must be in 1..16");
    if (cell_capacity < 0 || cell_capacity > 1024)
        return fail(DPD_EINVAL, "cell_capacity must be in 0..1024");
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(L[k])) return fail(DPD_EINVAL, "non-finite box");
        if (L[k] < 3.0) return fail(DPD_EBOX, "box edge %g is below 3 cutoffs", L[k]);
    }
    if (!all_finite(pos, 3 * n) || !all_finite(vel, 3 * n))
        return fail(DPD_EINVAL, "non-finite position or velocity");
    if (type)
        for (int64_t i = 0; i < n; ++i)
            if (type[i] >= ntypes) return fail(DPD_EINVAL, "type %d of particle %lld >= ntypes",
                                               (int)type[i], (long long)i);

    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(DPD_EDEVICE, "device %s is not gfx950", prop.gcnArchName);

    dpd_system *s = new (std::nothrow) dpd_system();
    if (!s) return fail(DPD_ENOMEM, "host allocation failed");
    s->dev = dev;
    s->prec = precision;
    s->n = n;
    s->ntypes = ntypes;
    s->seed = seed;
    s->cap = cell_capacity ? cell_capacity : 32;
    for (int k = 0; k < 3; ++k) {
        s->L[k] = L[k];
        s->nc[k] = (int)std::floor(L[k]);
        s->h[k] = L[k] / (double)s->nc[k];
    }
    s->ncells = (int64_t)s->nc[0] * s->nc[1] * s->nc[2];
    if (s->ncells * (int64_t)s->cap >= (int64_t)0xFFFFFFFF) {
        delete s;
        return fail(DPD_EINVAL, "cells x capacity exceeds 32-bit slot indices");
    }
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = stream_take(s->dev, &s->stream);
        if (e != hipSuccess) {
            delete s;
            return fail(DPD_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
        }
        s->own_stream = true;
    }
    const Layout lay = system_layout(precision, s->ncells, n, s->cap);
    int rc = dmalloc(s, &s->block, (size_t)lay.total);
    if (!rc) {
        char *base = (char *)s->block;
        auto at = [&](Buf k) { return (void *)(base + lay.off[k]); };
        s->P[0] = at(B_P0);
        s->P[1] = at(B_P1);
        s->S[0] = at(B_S0);
        s->S[1] = at(B_S1);
        s->slot_of_tag[0] = (uint32_t *)at(B_SOT0);
        s->slot_of_tag[1] = (uint32_t *)at(B_SOT1);
        s->count[0] = (uint32_t *)at(B_CNT0);
        s->count[1] = (uint32_t *)at(B_CNT1);
        s->count[2] = (uint32_t *)at(B_CNT2);
        s->a_dev = at(B_A);
        s->err = (uint32_t *)at(B_ERR);
        s->stage = (double *)at(B_STAGE);
        s->cell_stage = (int64_t *)at(B_CSTAGE);
        s->type_dev = (uint8_t *)at(B_TYPE);
        s->obs = (double *)at(B_OBS);
        s->obs_np = (uint32_t *)at(B_OBSNP);
        s->obs_ptrs = (double **)at(B_OBSPTR);
        s->red = (double *)at(B_RED);
    }
    s->red_blocks = red_blocks_for(n);
    if (rc) {
        free_all(s);
        release_stream(s);
        delete s;
        return rc;
    }
    auto setup = [&]() -> int {
        HIP_OK(hipMemsetAsync(s->err, 0, sizeof(uint32_t), s->stream));
        for (int k = 0; k < 2; ++k)
            HIP_OK(launch_fill_u32(s->slot_of_tag[k], n, 0u, s->stream));
        std::vector<uint8_t> tv(n, 0);
        if (type) std::memcpy(tv.data(), type, n);
        if (int rc = h2d(s->type_dev, tv.data(), n, s->stream)) return rc;
        double *ptrs[8] = {s->obs, s->obs + n, s->obs + 2 * n, s->obs + 3 * n, s->obs + 4 * n,
                           s->obs + 5 * n, s->obs + 6 * n, s->obs + 7 * n};
        if (int rc = h2d(s->obs_ptrs, ptrs, sizeof ptrs, s->stream)) return rc;
        return load_state(s, pos, vel, nullptr, 0);
    };
    rc = setup();
    if (rc == DPD_OK) rc = check_device(s);
    if (rc) {
        std::string msg = g_err;
        free_all(s);
        release_stream(s);
        delete s;
        return fail(rc, "%s", msg.c_str());
    }
    // Default brick: the largest one that still gives every CU work.
    s->variant = cells_default_variant(s);
    *out = s;
    return DPD_OK;
}

int dpd_set_params(dpd_system *s, const double *a_ij, double gamma, double sigma, double kT,
                   double dt, double lambda) {
    if (int rc = check_usable(s)) return rc;
    if (s->frozen) return fail(DPD_ESTATE, "parameters are frozen after the first step");
    if (!a_ij) return fail(DPD_EINVAL, "null a_ij");
    const int m = s->ntypes;
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            if (!std::isfinite(a_ij[i * m + j])) return fail(DPD_EINVAL, "non-finite a_ij");
            if (a_ij[i * m + j] != a_ij[j * m + i]) return fail(DPD_EINVAL, "a_ij not symmetric");
        }
    if (!(gamma >= 0) || !(sigma >= 0) || !std::isfinite(gamma) || !std::isfinite(sigma))
        return fail(DPD_EINVAL, "gamma and sigma must be finite and >= 0");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(DPD_EINVAL, "dt must be > 0");
    if (!(lambda >= 0 && lambda <= 1)) return fail(DPD_EINVAL, "lambda must be in [0, 1]");
    if (!std::isfinite(kT)) return fail(DPD_EINVAL, "non-finite kT");
    s->a.assign(a_ij, a_ij + m * m);
    s->gamma = gamma;
    s->sigma = sigma;
    s->kT = kT;
    s->dt = dt;
    s->lambda = lambda;
    s->params_set = true;
    return DPD_OK;
}

int dpd_add_bonds(dpd_system *s, int64_t nb, const int32_t *btype, const int64_t *i,
                  const int64_t *j, const double *r_e, const double *k, const double *alpha) {
    if (int rc = check_usable(s)) return rc;
    if (s->frozen) return fail(DPD_ESTATE, "bonds are frozen after the first step");
    if (nb < 0) return fail(DPD_EINVAL, "negative bond count");
    if (nb == 0) return DPD_OK;
    if (!btype || !i || !j || !r_e || !k || !alpha) return fail(DPD_EINVAL, "null bond array");
    // Validate against the current positions (minimum image needs r < L/2).
    std::vector<double> x(3 * s->n);
    HIP_OK(hipStreamSynchronize(s->stream));
    if (int rc = dpd_get_state(s, x.data(), nullptr, nullptr, nullptr)) return rc;
    for (int64_t b = 0; b < nb; ++b) {
        if (btype[b] < DPD_BOND_HARMONIC || btype[b] > DPD_BOND_MORSE)
            return fail(DPD_EINVAL, "bond %lld: unknown type %d", (long long)b, btype[b]);
        if (i[b] < 0 || j[b] < 0 || i[b] >= s->n || j[b] >= s->n || i[b] == j[b])
            return fail(DPD_ERANGE, "bond %lld: bad tags (%lld, %lld)", (long long)b,
                        (long long)i[b], (long long)j[b]);
        if (!std::isfinite(r_e[b]) || !std::isfinite(k[b]) || !std::isfinite(alpha[b]))
            return fail(DPD_EINVAL, "bond %lld: non-finite parameter", (long long)b);
        for (int c = 0; c < 3; ++c) {
            double d = x[3 * i[b] + c] - x[3 * j[b] + c];
            d -= s->L[c] * std::nearbyint(d / s->L[c]);
            if (std::fabs(d) >= 0.5 * s->L[c] - 1e-12)
                return fail(DPD_ERANGE, "bond %lld spans half the box", (long long)b);
        }
    }
    s->btype.insert(s->btype.end(), btype, btype + nb);
    s->bi.insert(s->bi.end(), i, i + nb);
    s->bj.insert(s->bj.end(), j, j + nb);
    s->bre.insert(s->bre.end(), r_e, r_e + nb);
    s->bk.insert(s->bk.end(), k, k + nb);
    s->balpha.insert(s->balpha.end(), alpha, alpha + nb);
    return DPD_OK;
}

static int step_impl(dpd_system *s, int64_t nsteps, dpd_kernel_times *tm) {
    if (int rc = check_usable(s)) return rc;
    if (nsteps < 0) return fail(DPD_EINVAL, "negative step count");
    // The noise counter and the layout/count rotation use the step index as
    // 32 bits; a run may not pass 2^32 - 1.
    if (nsteps > STEP_LIMIT - s->t)
        return fail(DPD_EINVAL, "step counter would pass 2^32 - 1 (at %lld, %lld more steps)",
                    (long long)s->t, (long long)nsteps);
    if (int rc = freeze(s)) return rc;
    if (int rc = ensure_force(s)) return rc;
    if (nsteps == 0) return DPD_OK;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (tm) {
        std::memset(tm, 0, sizeof *tm);
        HIP_OK(hipEventCreate(&ev[0]));
        HIP_OK(hipEventCreate(&ev[1]));
    }
    auto timed = [&](auto &&fn, double *acc, int64_t *cnt) -> int {
        if (tm) HIP_OK(hipEventRecord(ev[0], s->stream));
        if (int rc = fn()) return rc;
        if (tm) {
            HIP_OK(hipEventRecord(ev[1], s->stream));
            HIP_OK(hipEventSynchronize(ev[1]));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
            *acc += ms;
            ++*cnt;
        }
        return DPD_OK;
    };
    const uint32_t t0 = (uint32_t)s->t;
    int rc = timed([&] { return begin(s, t0); }, tm ? &tm->ms_begin : nullptr,
                   tm ? &tm->n_begin : nullptr);
    for (int64_t k = 1; k < nsteps && !rc; ++k)
        rc = timed([&] { return force(s, t0 + (uint32_t)k, FORCE_FUSED); },
                   tm ? &tm->ms_fused : nullptr, tm ? &tm->n_fused : nullptr);
    if (!rc)
        rc = timed([&] { return force(s, t0 + (uint32_t)nsteps, FORCE_FINISH); },
                   tm ? &tm->ms_finish : nullptr, tm ? &tm->n_finish : nullptr);
    if (tm) {
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    if (rc) return rc;
    s->t += nsteps;
    if (tm) return check_device(s);
    return DPD_OK;
}

int dpd_step(dpd_system *s, int64_t nsteps) { return step_impl(s, nsteps, nullptr); }

int dpd_step_profiled(dpd_system *s, int64_t nsteps, dpd_kernel_times *out) {
    if (!out) return fail(DPD_EINVAL, "null timing output");
    return step_impl(s, nsteps, out);
}

int dpd_sync(dpd_system *s) {
    if (!s) return fail(DPD_EINVAL, "null system");
    if (s->batch) return fail(DPD_EBUSY, "the system is resident in a batch; retire it first");
    return check_device(s);
}

int dpd_get_state(dpd_system *s, double *pos, double *vel, double *frc, int64_t *step) {
    if (int rc = check_usable(s)) return rc;
    if (frc) {
        // The force needs the parameters and the bond list, which freezes them.
        if (int rc = freeze(s)) return rc;
        if (int rc = ensure_force(s)) return rc;
    }
    const int64_t n = s->n;
    const uint32_t q = (uint32_t)s->t;
    if (s->prec == DPD_PREC_FP64)
        HIP_OK(launch_gather<double>(make_dev<double>(s), q, s->stage, s->stage + 3 * n,
                                     s->stage + 6 * n, s->cell_stage, s->stream));
    else
        HIP_OK(launch_gather<float>(make_dev<float>(s), q, s->stage, s->stage + 3 * n,
                                    s->stage + 6 * n, s->cell_stage, s->stream));
    if (int rc = check_device(s)) return rc;
    if (pos) HIP_OK(hipMemcpy(pos, s->stage, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (vel)
        HIP_OK(hipMemcpy(vel, s->stage + 3 * n, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    if (frc) {
        HIP_OK(hipMemcpy(frc, s->stage + 6 * n, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    }
    if (step) *step = s->t;
    return DPD_OK;
}

int dpd_set_state(dpd_system *s, const double *pos, const double *vel, const double *frc,
                  int64_t step) {
    if (int rc = check_usable(s)) return rc;
    if (!pos || !vel) return fail(DPD_EINVAL, "null position or velocity");
    if (step < 0) return fail(DPD_EINVAL, "negative step counter");
    if (step > STEP_LIMIT) return fail(DPD_EINVAL, "step counter above 2^32 - 1");
    if (!all_finite(pos, 3 * s->n) || !all_finite(vel, 3 * s->n) ||
        (frc && !all_finite(frc, 3 * s->n)))
        return fail(DPD_EINVAL, "non-finite state");
    if (int rc = load_state(s, pos, vel, frc, step)) return rc;
    return check_device(s);
}

int dpd_get_cells(dpd_system *s, int64_t *cell_of_tag, int64_t *count) {
    if (int rc = check_usable(s)) return rc;
    const int64_t n = s->n;
    const uint32_t q = (uint32_t)s->t;
    if (s->prec == DPD_PREC_FP64)
        HIP_OK(launch_gather<double>(make_dev<double>(s), q, s->stage, s->stage + 3 * n,
                                     s->stage + 6 * n, s->cell_stage, s->stream));
    else
        HIP_OK(launch_gather<float>(make_dev<float>(s), q, s->stage, s->stage + 3 * n,
                                    s->stage + 6 * n, s->cell_stage, s->stream));
    if (int rc = check_device(s)) return rc;
    if (cell_of_tag)
        HIP_OK(hipMemcpy(cell_of_tag, s->cell_stage, n * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (count) {
        std::vector<uint32_t> c(s->ncells);
        HIP_OK(hipMemcpy(c.data(), s->count[count_index((uint32_t)s->t, 0u)], s->ncells * sizeof(uint32_t),
                         hipMemcpyDeviceToHost));
        for (int64_t g = 0; g < s->ncells; ++g) count[g] = c[g];
    }
    return DPD_OK;
}

int dpd_observables(dpd_system *s, dpd_obs *out) {
    if (int rc = check_usable(s)) return rc;
    if (!out) return fail(DPD_EINVAL, "null output");
    if (int rc = freeze(s)) return rc;
    const int64_t n = s->n;
    if (int rc = force(s, (uint32_t)s->t, FORCE_OBS)) return rc;
    HIP_OK(launch_u32_to_f64(s->obs_np, s->obs + 5 * n, n, s->stream));
    const int64_t chunk = (n + s->red_blocks - 1) / s->red_blocks;
    HIP_OK(launch_reduce8((const double *const *)s->obs_ptrs, n, chunk, s->red_blocks, s->red,
                          s->stream));
    if (int rc = check_device(s)) return rc;
    std::vector<double> part((size_t)s->red_blocks * 8);
    HIP_OK(hipMemcpy(part.data(), s->red, part.size() * sizeof(double), hipMemcpyDeviceToHost));
    double tot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = 0; b < s->red_blocks; ++b)
        for (int k = 0; k < 8; ++k) tot[k] += part[(size_t)b * 8 + k];
    // obs layout: u, w, ub, wb, ke, npairs, px.. (interleaved 3n at 6n: summed as 2 arrays)
    out->step = s->t;
    out->time = (double)s->t * s->dt;
    out->u_pair = tot[0];
    out->w_pair = tot[1];
    out->u_bond = tot[2];
    out->w_bond = tot[3];
    out->ke = tot[4];
    out->npairs = (int64_t)std::llround(0.5 * tot[5]);
    out->kT = 2.0 * out->ke / (3.0 * (double)n - 3.0);
    const double V = s->L[0] * s->L[1] * s->L[2];
    out->pressure = (2.0 * out->ke + out->w_pair + out->w_bond) / (3.0 * V);
    // Momentum: per-tag (px, py, pz) interleaved over [6n, 9n).
    std::vector<double> p(3 * n);
    HIP_OK(hipMemcpy(p.data(), s->obs + 6 * n, 3 * n * sizeof(double), hipMemcpyDeviceToHost));
    double P[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) P[c] += p[3 * i + c];
    for (int c = 0; c < 3; ++c) out->momentum[c] = P[c];
    return DPD_OK;
}

int dpd_variant_count(void) { return force_variant_count(); }

int dpd_variant_shape(int variant, int out[5]) {
    if (!out || variant < 0 || variant >= force_variant_count())
        return fail(DPD_EINVAL, "bad variant %d", variant);
    force_variant_shape(variant, out);
    return DPD_OK;
}

int dpd_set_variant(dpd_system *s, int variant) {
    if (int rc = check_usable(s)) return rc;
    if (variant < -1 || variant >= force_variant_count())
        return fail(DPD_EINVAL, "bad variant %d", variant);
    s->variant = variant < 0 ? cells_default_variant(s) : variant;
    return DPD_OK;
}

int dpd_autotune(dpd_system *s, int trials, int *best_variant, double *best_ms) {
    if (int rc = check_usable(s)) return rc;
    if (trials < 1) return fail(DPD_EINVAL, "trials must be >= 1");
    const char *cache = std::getenv("DPD_TUNE_CACHE");
    std::string key;
    if (cache && *cache) {
        key = tune_key(s);
        const auto m = tune_read(cache);
        const auto it = m.find(key);
        if (it != m.end() && it->second.first >= 0 &&
            it->second.first < force_variant_count()) {
            s->variant = it->second.first;
            if (best_variant) *best_variant = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return DPD_OK;
        }
    }
    if (int rc = freeze(s)) return rc;
    if (int rc = ensure_force(s)) return rc;
    if (int rc = check_device(s)) return rc;
    const uint32_t q = (uint32_t)s->t;
    hipEvent_t ev[2];
    HIP_OK(hipEventCreate(&ev[0]));
    HIP_OK(hipEventCreate(&ev[1]));
    const int keep = s->variant;
    int best = -1;
    double best_t = 1e300;
    for (int v = 0; v < force_variant_count(); ++v) {
        s->variant = v;
        double tot = 0.0;
        bool ok = true;
        for (int k = 0; k <= trials && ok; ++k) {
            // The fused pass appends into the next state's counts: clear them.
            HIP_OK(launch_fill_u32(s->count[count_index(q, 1u)], s->ncells, 0u, s->stream));
            HIP_OK(hipEventRecord(ev[0], s->stream));
            if (int rc = force(s, q, FORCE_FUSED)) return rc;
            HIP_OK(hipEventRecord(ev[1], s->stream));
            HIP_OK(hipEventSynchronize(ev[1]));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, ev[0], ev[1]));
            uint32_t e = 0;
            HIP_OK(hipMemcpy(&e, s->err, sizeof e, hipMemcpyDeviceToHost));
            if (e) {
                // A tile too small for this state: skip the variant, clear the flag
                // (the trial wrote only scratch memory).
                ok = false;
                HIP_OK(hipMemsetAsync(s->err, 0, sizeof(uint32_t), s->stream));
                if (e & ~(uint32_t)ERR_TILE_OVERFLOW) {
                    s->variant = keep;
                    (void)hipEventDestroy(ev[0]);
                    (void)hipEventDestroy(ev[1]);
                    HIP_OK(hipStreamSynchronize(s->stream));
                    HIP_OK(hipMemcpy(s->err, &e, sizeof e, hipMemcpyHostToDevice));
                    return check_device(s);
                }
            }
            if (k > 0) tot += ms;
        }
        if (ok && tot / trials < best_t) {
            best_t = tot / trials;
            best = v;
        }
    }
    HIP_OK(launch_fill_u32(s->count[count_index(q, 1u)], s->ncells, 0u, s->stream));
    HIP_OK(hipStreamSynchronize(s->stream));
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (best < 0) {
        s->variant = keep;
        return fail(DPD_ECAPACITY, "no brick variant can hold this state's densest neighbourhood");
    }
    s->variant = best;
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    if (!key.empty()) {
        // A failed write leaves the choice in force for this system only.
        auto m = tune_read(cache);
        m[key] = {best, best_t};
        tune_write(cache, m);
    }
    return DPD_OK;
}

int dpd_pair_noise(uint64_t seed, int64_t m, const uint32_t *ti, const uint32_t *tj,
                   const uint32_t *sv, int precision, double *theta) {
    if (m < 0 || (m > 0 && (!ti || !tj || !sv || !theta))) return fail(DPD_EINVAL, "bad arrays");
    if (precision != DPD_PREC_FP64 && precision != DPD_PREC_MIXED)
        return fail(DPD_EINVAL, "unknown precision %d", precision);
    if (m == 0) return DPD_OK;
    uint32_t *d = nullptr;
    double *o = nullptr;
    HIP_OK(hipMalloc((void **)&d, 3 * m * sizeof(uint32_t)));
    hipError_t e = hipMalloc((void **)&o, m * sizeof(double));
    if (e != hipSuccess) {
        (void)hipFree(d);
        return fail(DPD_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    }
    auto run = [&]() -> int {
        HIP_OK(hipMemcpy(d, ti, m * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d + m, tj, m * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_OK(hipMemcpy(d + 2 * m, sv, m * sizeof(uint32_t), hipMemcpyHostToDevice));
        HIP_OK(launch_noise(precision == DPD_PREC_FP64, seed, m, d, d + m, d + 2 * m, o, nullptr));
        HIP_OK(hipDeviceSynchronize());
        HIP_OK(hipMemcpy(theta, o, m * sizeof(double), hipMemcpyDeviceToHost));
        return DPD_OK;
    };
    const int rc = run();
    (void)hipFree(d);
    (void)hipFree(o);
    return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// dpd_pair_noise without allocation: the triples and the results are staged
// in `scratch`, a fixed device array (each device holds its own copy for the
// life of the process).  Host code must never pass the array's name to a
// kernel or a copy: it stands for a host-side symbol; the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
// Layout: tag_i, tag_j, s (u32, NOISE_NA_MAX each), then theta (FP64).
// Nothing in it needs clearing: a call writes every element it reads.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t NOISE_NA_MAX = (int64_t)1 << 18;
constexpr size_t NOISE_NA_BYTES = (size_t)NOISE_NA_MAX * (3 * sizeof(uint32_t) + sizeof(double));
constexpr int NOISE_NA_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[NOISE_NA_BYTES];

namespace {
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[NOISE_NA_DEVICES] = {};

// Device address of `scratch` on the current device (looked up at the first
// call on that device).
int scratch_on_current_device(unsigned char **out) {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOISE_NA_DEVICES)
        return fail(DPD_EDEVICE, "device %d beyond the %d the library keeps scratch for", dev,
                    NOISE_NA_DEVICES);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(DPD_EDEVICE, "no device address for the scratch array");
        g_scratch_ptr[dev] = (unsigned char *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return DPD_OK;
}
}  // namespace

extern "C" {

int dpd_pair_noise_noalloc(uint64_t seed, int64_t m, const uint32_t *ti, const uint32_t *tj,
                           const uint32_t *sv, int precision, double *theta) {
    if (m < 0 || (m > 0 && (!ti || !tj || !sv || !theta))) return fail(DPD_EINVAL, "bad arrays");
    if (precision != DPD_PREC_FP64 && precision != DPD_PREC_MIXED)
        return fail(DPD_EINVAL, "unknown precision %d", precision);
    if (m > NOISE_NA_MAX)
        return fail(DPD_EINVAL, "%lld triples exceed the %lld this call can stage",
                    (long long)m, (long long)NOISE_NA_MAX);
    if (m == 0) return DPD_OK;
    unsigned char *base = nullptr;
    if (int rc = scratch_on_current_device(&base)) return rc;
    uint32_t *d = (uint32_t *)base;
    double *o = (double *)(base + 3 * NOISE_NA_MAX * sizeof(uint32_t));
    HIP_OK(hipMemcpy(d, ti, m * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d + NOISE_NA_MAX, tj, m * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d + 2 * NOISE_NA_MAX, sv, m * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIP_OK(launch_noise(precision == DPD_PREC_FP64, seed, m, d, d + NOISE_NA_MAX,
                        d + 2 * NOISE_NA_MAX, o, nullptr));
    // The copy back on the null stream follows the kernel.
    HIP_OK(hipMemcpy(theta, o, m * sizeof(double), hipMemcpyDeviceToHost));
    return DPD_OK;
}

int dpd_info(dpd_system *s, int64_t out[8]) {
    if (!s || !out) return fail(DPD_EINVAL, "null argument");
    out[0] = s->n;
    out[1] = s->ncells;
    out[2] = s->cap;
    out[3] = (int64_t)s->bytes;
    out[4] = s->nc[0];
    out[5] = s->nc[1];
    out[6] = s->nc[2];
    out[7] = s->prec;
    return DPD_OK;
}

void dpd_destroy(dpd_system *s) {
    if (!s) return;
    if (s->batch) (void)batch_detach(s->batch, s->batch_slot);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    free_all(s);
    release_stream(s);
    delete s;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Replica batches: many resident systems advanced by shared launches, one
// captured HIP graph per window of K steps.
// ---------------------------------------------------------------------------
struct dpd_batch {
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int64_t budget = 0, used = 0;
    int max_slots = 0;
    int variant = 4;
    int bx = 2, by = 2, bz = 2;

    std::vector<dpd_system *> sys;     // per slot (null = free)
    std::vector<uint32_t> t0, target;  // host mirror of the device counters
    std::vector<uint8_t> reported;
    std::vector<uint32_t> err;

    // Device tables (fixed addresses for the life of the batch, except the
    // work lists, which grow and then force a re-capture).
    BatchEnt *tab = nullptr;
    uint32_t *t0_dev = nullptr, *target_dev = nullptr, *status_dev = nullptr;
    int *nwork_dev = nullptr;
    BatchWork *wf = nullptr, *wb = nullptr;
    int cap_wf = 0, cap_wb = 0;

    // Pinned host staging.
    uint32_t *status_h = nullptr;
    BatchEnt *tab_h = nullptr;
    uint32_t *ctr_h = nullptr;           // t0 then target, 2 * max_slots
    int *nwork_h = nullptr;
    std::vector<BatchWork> wf_v, wb_v;
    BatchWork *wf_h = nullptr, *wb_h = nullptr;
    int cap_wf_h = 0, cap_wb_h = 0;

    bool dirty = true;        // host tables changed since the last upload
    bool inflight = false;    // a window was enqueued since the last refresh
    int n_force = 0, n_begin = 0;

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_K = 0, graph_wf = 0, graph_wb = 0;
    const BatchWork *graph_wf_ptr = nullptr, *graph_wb_ptr = nullptr;
    int64_t captures = 0, windows = 0;
    hipEvent_t done = nullptr;
};

namespace {

void batch_free(dpd_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    void *dptr[] = {b->tab, b->t0_dev, b->target_dev, b->status_dev, b->nwork_dev, b->wf, b->wb};
    for (void *p : dptr)
        if (p) (void)hipFree(p);
    void *hptr[] = {b->status_h, b->tab_h, b->ctr_h, b->nwork_h, b->wf_h, b->wb_h};
    for (void *p : hptr)
        if (p) (void)hipHostFree(p);
    if (b->done) (void)hipEventDestroy(b->done);
    if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

// Waits for enqueued windows and takes the device counters into the host mirror.
int batch_refresh(dpd_batch *b) {
    HIP_OK(hipStreamSynchronize(b->stream));
    if (!b->inflight) return DPD_OK;
    for (int k = 0; k < b->max_slots; ++k) {
        if (!b->sys[k]) continue;
        b->t0[k] = b->status_h[2 * k];
        b->err[k] = b->status_h[2 * k + 1];
        b->sys[k]->t = b->t0[k];
    }
    b->inflight = false;
    return DPD_OK;
}

template <typename P> int grow_pinned(P **p, int *cap, int need) {
    if (need <= *cap) return DPD_OK;
    int c = std::max(need, 2 * *cap);
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipHostMalloc((void **)p, (size_t)c * sizeof(P), hipHostMallocDefault);
    if (e != hipSuccess) return fail(DPD_ENOMEM, "hipHostMalloc failed: %s", hipGetErrorString(e));
    *cap = c;
    return DPD_OK;
}

template <typename P> int grow_device(P **p, int *cap, int need) {
    if (need <= *cap) return DPD_OK;
    int c = std::max(need, 2 * *cap);
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void **)p, (size_t)c * sizeof(P));
    if (e != hipSuccess) return fail(DPD_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
    *cap = c;
    return DPD_OK;
}

// Rebuilds the work lists and uploads every table (the stream is idle).
int batch_upload(dpd_batch *b) {
    b->wf_v.clear();
    b->wb_v.clear();
    for (int k = 0; k < b->max_slots; ++k) {
        dpd_system *s = b->sys[k];
        if (!s || b->t0[k] >= b->target[k]) continue;
        const int nbr = b->tab_h[k].nbx * b->tab_h[k].nby * b->tab_h[k].nbz;
        for (int i = 0; i < nbr; ++i) b->wf_v.push_back(BatchWork{(uint32_t)k, (uint32_t)i});
        const int nblk = (int)((s->ncells + 255) / 256);
        for (int i = 0; i < nblk; ++i) b->wb_v.push_back(BatchWork{(uint32_t)k, (uint32_t)i});
    }
    b->n_force = (int)b->wf_v.size();
    b->n_begin = (int)b->wb_v.size();
    if (int rc = grow_device(&b->wf, &b->cap_wf, std::max(1, b->n_force))) return rc;
    if (int rc = grow_device(&b->wb, &b->cap_wb, std::max(1, b->n_begin))) return rc;
    if (int rc = grow_pinned(&b->wf_h, &b->cap_wf_h, std::max(1, b->n_force))) return rc;
    if (int rc = grow_pinned(&b->wb_h, &b->cap_wb_h, std::max(1, b->n_begin))) return rc;
    std::copy(b->wf_v.begin(), b->wf_v.end(), b->wf_h);
    std::copy(b->wb_v.begin(), b->wb_v.end(), b->wb_h);
    for (int k = 0; k < b->max_slots; ++k) {
        b->ctr_h[k] = b->t0[k];
        b->ctr_h[b->max_slots + k] = b->target[k];
    }
    b->nwork_h[0] = b->n_force;
    b->nwork_h[1] = b->n_begin;
    b->nwork_h[2] = b->max_slots;
    const size_t ms = (size_t)b->max_slots;
    HIP_OK(hipMemcpyAsync(b->tab, b->tab_h, ms * sizeof(BatchEnt), hipMemcpyHostToDevice,
                          b->stream));
    HIP_OK(hipMemcpyAsync(b->t0_dev, b->ctr_h, ms * sizeof(uint32_t), hipMemcpyHostToDevice,
                          b->stream));
    HIP_OK(hipMemcpyAsync(b->target_dev, b->ctr_h + ms, ms * sizeof(uint32_t),
                          hipMemcpyHostToDevice, b->stream));
    HIP_OK(hipMemcpyAsync(b->nwork_dev, b->nwork_h, 3 * sizeof(int), hipMemcpyHostToDevice,
                          b->stream));
    if (b->n_force)
        HIP_OK(hipMemcpyAsync(b->wf, b->wf_h, (size_t)b->n_force * sizeof(BatchWork),
                              hipMemcpyHostToDevice, b->stream));
    if (b->n_begin)
        HIP_OK(hipMemcpyAsync(b->wb, b->wb_h, (size_t)b->n_begin * sizeof(BatchWork),
                              hipMemcpyHostToDevice, b->stream));
    // The pinned staging must not change before the copies are done.
    HIP_OK(hipStreamSynchronize(b->stream));
    b->dirty = false;
    return DPD_OK;
}

int batch_capture(dpd_batch *b, int K) {
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    BatchDev B;
    B.tab = b->tab;
    B.t0 = b->t0_dev;
    B.target = b->target_dev;
    B.wf = b->wf;
    B.wb = b->wb;
    B.nwork = b->nwork_dev;
    B.status = b->status_dev;
    HIP_OK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_batch_window(B, b->variant, K, b->cap_wf, b->cap_wb, b->max_slots,
                                       b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(DPD_EDEVICE, "capturing the batch window failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    HIP_OK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_K = K;
    b->graph_wf = b->cap_wf;
    b->graph_wb = b->cap_wb;
    b->graph_wf_ptr = b->wf;
    b->graph_wb_ptr = b->wb;
    ++b->captures;
    return DPD_OK;
}

void batch_split(dpd_batch *b, int slot);

int batch_detach(dpd_batch *b, int slot) {
    if (int rc = batch_refresh(b)) return rc;
    dpd_system *s = b->sys[slot];
    s->t = b->t0[slot];
    s->batch = nullptr;
    s->batch_slot = -1;
    b->used -= (int64_t)s->bytes;
    b->sys[slot] = nullptr;
    b->t0[slot] = b->target[slot] = 0;
    b->err[slot] = 0;
    b->reported[slot] = 0;
    std::memset(&b->tab_h[slot], 0, sizeof(BatchEnt));
    b->dirty = true;
    return DPD_OK;
}

}  // namespace

extern "C" {

int dpd_footprint_bytes(const double L[3], int64_t n, int64_t nbonds, int precision,
                        int cell_capacity, int64_t *bytes) {
    if (!L || !bytes) return fail(DPD_EINVAL, "null argument");
    if (n < 2 || nbonds < 0) return fail(DPD_EINVAL, "bad sizes");
    if (precision != DPD_PREC_FP64 && precision != DPD_PREC_MIXED)
        return fail(DPD_EINVAL, "unknown precision %d", precision);
    if (cell_capacity < 0 || cell_capacity > 1024)
        return fail(DPD_EINVAL, "cell_capacity must be in 0..1024");
    int nc[3];
    for (int k = 0; k < 3; ++k) {
        if (!std::isfinite(L[k]) || L[k] < 3.0) return fail(DPD_EBOX, "box edge below 3");
        nc[k] = (int)std::floor(L[k]);
    }
    *bytes = footprint(precision, nc, n, nbonds, cell_capacity ? cell_capacity : 32);
    return DPD_OK;
}

int dpd_batch_create(dpd_batch **out, int64_t budget_bytes, int max_replicas, void *hip_stream,
                     int variant) {
    g_err.clear();
    if (!out) return fail(DPD_EINVAL, "null argument");
    *out = nullptr;
    if (budget_bytes <= 0) return fail(DPD_EINVAL, "budget must be > 0");
    if (max_replicas < 1 || max_replicas > 65536)
        return fail(DPD_EINVAL, "max_replicas must be in 1..65536");
    if (variant < -1 || variant >= force_variant_count())
        return fail(DPD_EINVAL, "bad variant %d", variant);
    dpd_batch *b = new (std::nothrow) dpd_batch();
    if (!b) return fail(DPD_ENOMEM, "host allocation failed");
    b->budget = budget_bytes;
    b->max_slots = max_replicas;
    b->variant = variant < 0 ? 1 : variant;
    int shape[5];
    force_variant_shape(b->variant, shape);
    b->bx = shape[0];
    b->by = shape[1];
    b->bz = shape[2];
    const size_t ms = (size_t)max_replicas;
    b->sys.assign(ms, nullptr);
    b->t0.assign(ms, 0);
    b->target.assign(ms, 0);
    b->reported.assign(ms, 0);
    b->err.assign(ms, 0);
    auto setup = [&]() -> int {
        if (hip_stream) {
            b->stream = (hipStream_t)hip_stream;
        } else {
            HIP_OK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
            b->own_stream = true;
        }
        HIP_OK(hipMalloc((void **)&b->tab, ms * sizeof(BatchEnt)));
        HIP_OK(hipMalloc((void **)&b->t0_dev, ms * sizeof(uint32_t)));
        HIP_OK(hipMalloc((void **)&b->target_dev, ms * sizeof(uint32_t)));
        HIP_OK(hipMalloc((void **)&b->status_dev, 2 * ms * sizeof(uint32_t)));
        HIP_OK(hipMalloc((void **)&b->nwork_dev, 3 * sizeof(int)));
        HIP_OK(hipHostMalloc((void **)&b->status_h, 2 * ms * sizeof(uint32_t),
                             hipHostMallocDefault));
        HIP_OK(hipHostMalloc((void **)&b->tab_h, ms * sizeof(BatchEnt), hipHostMallocDefault));
        HIP_OK(hipHostMalloc((void **)&b->ctr_h, 2 * ms * sizeof(uint32_t), hipHostMallocDefault));
        HIP_OK(hipHostMalloc((void **)&b->nwork_h, 3 * sizeof(int), hipHostMallocDefault));
        std::memset(b->tab_h, 0, ms * sizeof(BatchEnt));
        std::memset(b->status_h, 0, 2 * ms * sizeof(uint32_t));
        HIP_OK(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
        return batch_upload(b);
    };
    if (int rc = setup()) {
        std::string msg = g_err;
        batch_free(b);
        delete b;
        return fail(rc, "%s", msg.c_str());
    }
    *out = b;
    return DPD_OK;
}

int dpd_batch_admit(dpd_batch *b, dpd_system *s, int64_t nsteps, int *slot) {
    if (!b || !s) return fail(DPD_EINVAL, "null argument");
    if (s->batch) return fail(DPD_EINVAL, "the system is already resident in a batch");
    if (int rc = check_usable(s)) return rc;
    if (nsteps < 0) return fail(DPD_EINVAL, "negative step count");
    if (s->prec != DPD_PREC_MIXED)
        return fail(DPD_EINVAL, "batches hold mixed-precision systems only");
    if (!(s->h[0] == s->h[1] && s->h[0] == s->h[2]))
        return fail(DPD_EINVAL, "batches need cubic cells (equal cell edges on all axes)");
    if (nsteps > STEP_LIMIT - s->t)
        return fail(DPD_EINVAL, "step counter would pass 2^32 - 1");
    if (int rc = freeze(s)) return rc;
    if (int rc = ensure_force(s)) return rc;
    if (int rc = check_device(s)) return rc;   // also waits for the system's own stream
    if (int rc = batch_refresh(b)) return rc;
    if (b->used + (int64_t)s->bytes > b->budget)
        return fail(DPD_EBUSY, "admitting %lld bytes would exceed the batch budget (%lld of %lld used)",
                    (long long)s->bytes, (long long)b->used, (long long)b->budget);
    int k = 0;
    while (k < b->max_slots && b->sys[k]) ++k;
    if (k == b->max_slots) return fail(DPD_EBUSY, "all %d batch slots are taken", b->max_slots);
    BatchEnt e;
    std::memset(&e, 0, sizeof e);
    e.D = make_dev<float>(s);
    const double lim = 536870912.0 / s->h[0];
    e.thr = (uint64_t)std::ceil(lim * lim);
    b->tab_h[k] = e;
    b->sys[k] = s;
    batch_split(b, k);
    b->t0[k] = (uint32_t)s->t;
    b->target[k] = (uint32_t)(s->t + nsteps);
    b->err[k] = 0;
    b->reported[k] = 0;
    b->used += (int64_t)s->bytes;
    s->batch = b;
    s->batch_slot = k;
    b->dirty = true;
    if (slot) *slot = k;
    return DPD_OK;
}

}  // extern "C"

namespace {

// Bricks of a replica in the batch's current brick shape.
void batch_split(dpd_batch *b, int slot) {
    const dpd_system *s = b->sys[slot];
    BatchEnt &e = b->tab_h[slot];
    e.nbx = (s->nc[0] + b->bx - 1) / b->bx;
    e.nby = (s->nc[1] + b->by - 1) / b->by;
    e.nbz = (s->nc[2] + b->bz - 1) / b->bz;
}

void batch_set_variant(dpd_batch *b, int variant) {
    int shape[5];
    force_variant_shape(variant, shape);
    b->variant = variant;
    b->bx = shape[0];
    b->by = shape[1];
    b->bz = shape[2];
    for (int k = 0; k < b->max_slots; ++k)
        if (b->sys[k]) batch_split(b, k);
    b->dirty = true;
    b->graph_K = 0;       // re-capture with the new kernels
}

int batch_advance(dpd_batch *b, int64_t K, float *ms) {
    if (!b) return fail(DPD_EINVAL, "null batch");
    if (K < 1 || K > 100000) return fail(DPD_EINVAL, "window length must be in 1..100000");
    if (b->dirty) {
        if (int rc = batch_refresh(b)) return rc;
        if (int rc = batch_upload(b)) return rc;
    }
    if (b->n_force == 0) return DPD_OK;   // nothing left to step
    if (!b->exec || b->graph_K != K || b->graph_wf != b->cap_wf || b->graph_wb != b->cap_wb ||
        b->graph_wf_ptr != b->wf || b->graph_wb_ptr != b->wb) {
        HIP_OK(hipStreamSynchronize(b->stream));
        if (int rc = batch_capture(b, (int)K)) return rc;
    }
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (ms) {
        HIP_OK(hipEventCreate(&ev[0]));
        HIP_OK(hipEventCreate(&ev[1]));
        HIP_OK(hipEventRecord(ev[0], b->stream));
    }
    HIP_OK(hipGraphLaunch(b->exec, b->stream));
    if (ms) HIP_OK(hipEventRecord(ev[1], b->stream));
    HIP_OK(hipMemcpyAsync(b->status_h, b->status_dev, 2 * (size_t)b->max_slots * sizeof(uint32_t),
                          hipMemcpyDeviceToHost, b->stream));
    HIP_OK(hipEventRecord(b->done, b->stream));
    b->inflight = true;
    ++b->windows;
    if (ms) {
        HIP_OK(hipEventSynchronize(ev[1]));
        HIP_OK(hipEventElapsedTime(ms, ev[0], ev[1]));
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
    }
    // Replicas that reach their target keep their (now idle) work items until
    // the next admission or retirement rebuilds the lists.
    return DPD_OK;
}

}  // namespace

extern "C" {

int dpd_batch_advance(dpd_batch *b, int64_t K) { return batch_advance(b, K, nullptr); }

int dpd_batch_autotune(dpd_batch *b, int64_t K, int *best_variant, double *best_ms) {
    if (!b) return fail(DPD_EINVAL, "null batch");
    if (K < 1 || K > 100000) return fail(DPD_EINVAL, "window length must be in 1..100000");
    int best = b->variant;
    double best_t = -1.0;
    for (int v = 0; v < force_variant_count(); ++v) {
        batch_set_variant(b, v);
        float ms = -1.0f;
        if (int rc = batch_advance(b, K, &ms)) return rc;
        if (ms < 0.0f) break;               // nothing left to step
        const double per = ms / (double)K;
        if (best_t < 0.0 || per < best_t) {
            best_t = per;
            best = v;
        }
    }
    batch_set_variant(b, best);
    if (best_variant) *best_variant = best;
    if (best_ms) *best_ms = best_t;
    return DPD_OK;
}

int dpd_batch_poll(dpd_batch *b, int *done, int max_done, int *ndone) {
    if (!b || !ndone || (max_done > 0 && !done)) return fail(DPD_EINVAL, "null argument");
    *ndone = 0;
    if (int rc = batch_refresh(b)) return rc;
    for (int k = 0; k < b->max_slots && *ndone < max_done; ++k) {
        if (!b->sys[k] || b->reported[k]) continue;
        if (b->t0[k] >= b->target[k] || b->err[k]) {
            b->reported[k] = 1;
            done[(*ndone)++] = k;
        }
    }
    return DPD_OK;
}

int dpd_batch_retire(dpd_batch *b, int slot) {
    if (!b) return fail(DPD_EINVAL, "null batch");
    if (slot < 0 || slot >= b->max_slots || !b->sys[slot])
        return fail(DPD_EINVAL, "slot %d holds no replica", slot);
    return batch_detach(b, slot);
}

int dpd_batch_info(dpd_batch *b, int64_t out[6]) {
    if (!b || !out) return fail(DPD_EINVAL, "null argument");
    int64_t res = 0;
    for (dpd_system *s : b->sys) res += s ? 1 : 0;
    out[0] = res;
    out[1] = b->used;
    out[2] = b->budget;
    out[3] = b->captures;
    out[4] = b->windows;
    out[5] = b->variant;
    return DPD_OK;
}

void dpd_batch_destroy(dpd_batch *b) {
    if (!b) return;
    for (int k = 0; k < b->max_slots; ++k)
        if (b->sys[k]) (void)batch_detach(b, k);
    (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
}

}  // extern "C"
