// api.cpp -- host runtime behind the C ABI of include/ginimds.h: contexts,
// argument validation, Gini weight tables, scratch management, descriptor
// upload, launch selection and the autotuner.  Every numeric step runs in the
// HIP kernels; the host only prepares tables of the weight function and
// decides what to launch.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ginimds.h"
#include "common.hpp"
#include "kernels.hpp"

using gmds::InstDesc;

namespace {

constexpr int kVersion = 10000;     // 1.0.0
constexpr int kRing = 16;           // descriptor upload slots
constexpr int64_t kMaxRankD = 1 << 20;
constexpr int kMaxDissimM = 4096;
constexpr int kErrCap = 512;        // longest error message, with its terminator

struct Slot {
    void* host = nullptr;   // pinned staging, made for the first upload too large for a kernel argument
    size_t hcap = 0;
    void* dev = nullptr;    // made for the whole ring at the first upload
    size_t dcap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
constexpr size_t kSlotBytes = 64 << 10;   // device bytes of an upload slot at first

struct TableKey {
    int d;
    std::vector<double> nus;
    bool operator<(const TableKey& o) const {
        if (d != o.d) return d < o.d;
        return nus < o.nus;
    }
};

struct TuneEntry {
    gini_solve_opts opts;
};

}  // namespace

// Streams (groups of instances) of a split batched solve.
constexpr int kSplitGroups = 2;

struct gini_ctx {
    int device = 0;
    bool ready = false;
    int cus = 0;
    std::string err;
    // scratch for tile partials (grown on demand)
    float* scratch = nullptr;
    size_t scratch_bytes = 0;
    // completion counters of the fused reductions: zero between launches
    uint32_t* cnt = nullptr;
    size_t cnt_cap = 0;      // words
    // persistent-solve control
    gmds::SolveCtl* ctl = nullptr;
    uint32_t* epochs = nullptr;
    size_t ctl_cap = 0;      // instances
    Slot ring[kRing];
    int ring_next = 0;
    std::map<TableKey, float*> tables;
    std::map<std::string, TuneEntry> tune;
    // kernel timing (gini_profile_enable)
    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[4];   // tile, reduce, persistent, dissim
    std::vector<hipEvent_t> ev_pool;
    int64_t spin_limit = 1000000000;   // ticks of the constant-rate device clock
    bool spin_override = false;
    // gini_select_nu: the folds' dissimilarities and the small result buffers
    float* sel = nullptr;
    size_t sel_bytes = 0;
    // gini_classical_mds: pinned landing slots for the Rayleigh-Ritz matrices
    // of the iterations in flight, and their events
    float* cm_pin = nullptr;
    float* cm_pin_dev = nullptr;     // the same memory as the device addresses it
    hipEvent_t cm_ev[4] = {};
    // the extra streams of a split batched solve, and the fork / join events
    hipStream_t side[kSplitGroups - 1] = {};
    hipEvent_t side_fork = nullptr, side_join[kSplitGroups - 1] = {};
};

namespace {

gini_status fail(gini_ctx* c, gini_status s, const char* fmt, ...) {
    char buf[kErrCap];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return s;
}

gini_status hip_fail(gini_ctx* c, hipError_t e, const char* where) {
    return fail(c, GINI_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define GINI_HIP(ctx, call)                                           \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);      \
    } while (0)

gini_status ensure_ready(gini_ctx* c) {
    if (c->ready) {
        GINI_HIP(c, hipSetDevice(c->device));
        return GINI_OK;
    }
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0) return fail(c, GINI_EDEVICE, "no HIP device available");
    if (c->device >= count) return fail(c, GINI_EINVAL, "device %d out of range (%d devices)", c->device, count);
    GINI_HIP(c, hipSetDevice(c->device));
    hipDeviceProp_t prop;
    GINI_HIP(c, hipGetDeviceProperties(&prop, c->device));
    c->cus = prop.multiProcessorCount;
    // the persistent solver's wait limit is counted in ticks of the device's
    // constant-rate clock: 10 s unless GINI_SPIN_LIMIT_TICKS overrides it
    int khz = 0;
    if (!c->spin_override && hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess &&
        khz > 0)
        c->spin_limit = (int64_t)khz * 1000 * 10;
    for (int i = 0; i < kRing; ++i) GINI_HIP(c, hipEventCreateWithFlags(&c->ring[i].done, hipEventDisableTiming));
    c->ready = true;
    return GINI_OK;
}

// Copy `bytes` from host to a device staging slot on `s`; returns the device
// pointer.  The slot is reused only after the work recorded on it has ended.
// Uploads of at most 3 KiB travel as the argument of a one-block kernel that
// stores them: the kernel's launch packet carries them, and no copy engine
// is involved (its latency is most of a small copy's cost).
constexpr int kArgBlobWords = 768;
struct ArgBlob {
    uint32_t w[kArgBlobWords];
};
__global__ void k_put_blob(ArgBlob b, uint32_t* dst, int nw) {
    for (int i = threadIdx.x; i < nw; i += blockDim.x) dst[i] = b.w[i];
}

gini_status upload(gini_ctx* c, const void* src, size_t bytes, hipStream_t s, void** dev, Slot** slot_out) {
    // the first upload allocates the device buffers of the whole ring, so
    // that later calls do not pay for them one slot at a time
    if (!c->ring[0].dev) {
        for (int i = 0; i < kRing; ++i) {
            if (hipMalloc(&c->ring[i].dev, kSlotBytes) != hipSuccess)
                return fail(c, GINI_ENOMEM, "upload slot allocation failed");
            c->ring[i].dcap = kSlotBytes;
        }
    }
    Slot& sl = c->ring[c->ring_next];
    c->ring_next = (c->ring_next + 1) % kRing;
    if (sl.used) GINI_HIP(c, hipEventSynchronize(sl.done));
    if (sl.dcap < bytes) {
        if (sl.dev) GINI_HIP(c, hipFree(sl.dev));
        sl.dev = nullptr;
        sl.dcap = 0;
        if (hipMalloc(&sl.dev, bytes) != hipSuccess) return fail(c, GINI_ENOMEM, "device staging allocation failed");
        sl.dcap = bytes;
    }
    if (bytes > sizeof(ArgBlob) && sl.hcap < bytes) {
        if (sl.host) GINI_HIP(c, hipHostFree(sl.host));
        sl.host = nullptr;
        sl.hcap = 0;
        const size_t cap = std::max<size_t>(bytes, 4096);
        if (hipHostMalloc(&sl.host, cap, hipHostMallocDefault) != hipSuccess)
            return fail(c, GINI_ENOMEM, "pinned staging allocation of %zu bytes failed", cap);
        sl.hcap = cap;
    }
    if (bytes <= sizeof(ArgBlob)) {
        ArgBlob b;
        const int nw = (int)((bytes + 3) / 4);
        if (nw > 0) b.w[nw - 1] = 0u;
        std::memcpy(b.w, src, bytes);
        hipLaunchKernelGGL(k_put_blob, dim3(1), dim3(256), 0, s, b, static_cast<uint32_t*>(sl.dev), nw);
        GINI_HIP(c, hipGetLastError());
    } else {
        std::memcpy(sl.host, src, bytes);
        GINI_HIP(c, hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s));
    }
    *dev = sl.dev;
    *slot_out = &sl;
    return GINI_OK;
}

gini_status slot_done(gini_ctx* c, Slot* sl, hipStream_t s) {
    GINI_HIP(c, hipEventRecord(sl->done, s));
    sl->used = true;
    return GINI_OK;
}

enum { kProfTile = 0, kProfReduce = 1, kProfPersistent = 2, kProfDissim = 3 };

hipEvent_t pool_event(gini_ctx* c) {
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

void prof_clear(gini_ctx* c) {
    for (auto& v : c->prof_ev) {
        for (auto& pr : v) {
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        v.clear();
    }
}

// Times launches while profiling is on.  A single-kernel launch takes
// timer(): the runtime stamps the two events at the kernel's own start and
// end, so no marker sits between consecutive kernels.  Otherwise (a call
// that enqueues several kernels) the events are recorded around the scope.
struct ProfScope {
    gini_ctx* c;
    int kind;
    hipStream_t s;
    bool stamped;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(gini_ctx* c_, int kind_, hipStream_t s_, bool stamped_ = false)
        : c(c_), kind(kind_), s(s_), stamped(stamped_) {
        if (!c->prof) return;
        a = pool_event(c);
        b = a ? pool_event(c) : nullptr;
        if (!b) {
            if (a) c->ev_pool.push_back(a);
            a = nullptr;
            return;
        }
        if (!stamped) (void)hipEventRecord(a, s);
    }
    gmds::LaunchTimer timer() const { return gmds::LaunchTimer{a, b}; }
    ~ProfScope() {
        if (!a) return;
        if (!stamped) (void)hipEventRecord(b, s);
        c->prof_ev[kind].emplace_back(a, b);
    }
};

// Every array argument must be memory a kernel on the context's GPU can use:
// device memory of that GPU, or managed memory.  Host memory, or a pointer
// HIP does not know, is refused here instead of faulting in a kernel.  Null
// entries are skipped (optional arguments; required ones are checked before).
gini_status check_dev(gini_ctx* c, std::initializer_list<std::pair<const void*, const char*>> ptrs) {
    for (const auto& pr : ptrs) {
        if (!pr.first) continue;
        hipPointerAttribute_t a{};
        const hipError_t e = hipPointerGetAttributes(&a, pr.first);
        if (e != hipSuccess) {
            (void)hipGetLastError();               // leave no error behind for the next call
            return fail(c, GINI_EINVAL, "%s is not memory allocated through HIP", pr.second);
        }
        if (a.type == hipMemoryTypeDevice) {
            if (a.device != c->device)
                return fail(c, GINI_EINVAL, "%s lives on device %d, the context on device %d", pr.second, a.device,
                            c->device);
        } else if (a.type != hipMemoryTypeManaged && a.type != hipMemoryTypeUnified) {
            return fail(c, GINI_EINVAL, "%s is host memory: pass device memory", pr.second);
        }
    }
    return GINI_OK;
}

gini_status check_dev_instances(gini_ctx* c, const gini_instance* inst, int32_t n_inst) {
    for (int k = 0; k < n_inst; ++k) {
        const gini_instance& I = inst[k];
        gini_status st = check_dev(c, {{I.Delta, "Delta"}, {I.Z, "Z"}, {I.sigma_hist, "sigma_hist"},
                                       {I.ks_hist, "ks_hist"}, {I.delta_sumsq, "delta_sumsq"},
                                       {I.delta_sum, "delta_sum"}});
        if (st != GINI_OK) return fail(c, st, "instance %d: %s", k, std::string(c->err).c_str());
    }
    return GINI_OK;
}

gini_status ensure_scratch(gini_ctx* c, size_t bytes) {
    if (bytes <= c->scratch_bytes) return GINI_OK;
    if (c->scratch) {
        GINI_HIP(c, hipDeviceSynchronize());
        GINI_HIP(c, hipFree(c->scratch));
        c->scratch = nullptr;
        c->scratch_bytes = 0;
    }
    size_t cap = std::max(bytes, c->scratch_bytes * 3 / 2);
    cap = (cap + 255) & ~size_t(255);
    if (hipMalloc(reinterpret_cast<void**>(&c->scratch), cap) != hipSuccess)
        return fail(c, GINI_ENOMEM, "scratch allocation of %zu bytes failed", cap);
    c->scratch_bytes = cap;
    return GINI_OK;
}

// Symmetric eigen-decomposition of a small q x q matrix A (row-major, FP64)
// by cyclic Jacobi rotations: A = W diag(lam) W^T, columns of W the vectors.
void jacobi_eig(int q, std::vector<double> A, std::vector<double>& lam, std::vector<double>& W) {
    W.assign((size_t)q * q, 0.0);
    for (int i = 0; i < q; ++i) W[(size_t)i * q + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < q; ++j) {
                tot += A[(size_t)i * q + j] * A[(size_t)i * q + j];
                if (i != j) off += A[(size_t)i * q + j] * A[(size_t)i * q + j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int pp = 0; pp < q - 1; ++pp)
            for (int qq = pp + 1; qq < q; ++qq) {
                const double apq = A[(size_t)pp * q + qq];
                if (apq == 0.0) continue;
                const double app = A[(size_t)pp * q + pp], aqq = A[(size_t)qq * q + qq];
                const double theta = 0.5 * (aqq - app) / apq;
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < q; ++k) {        // A <- J^T A J
                    const double akp = A[(size_t)k * q + pp], akq = A[(size_t)k * q + qq];
                    A[(size_t)k * q + pp] = cs * akp - sn * akq;
                    A[(size_t)k * q + qq] = sn * akp + cs * akq;
                }
                for (int k = 0; k < q; ++k) {
                    const double apk = A[(size_t)pp * q + k], aqk = A[(size_t)qq * q + k];
                    A[(size_t)pp * q + k] = cs * apk - sn * aqk;
                    A[(size_t)qq * q + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < q; ++k) {
                    const double wkp = W[(size_t)k * q + pp], wkq = W[(size_t)k * q + qq];
                    W[(size_t)k * q + pp] = cs * wkp - sn * wkq;
                    W[(size_t)k * q + qq] = sn * wkp + cs * wkq;
                }
            }
    }
    lam.resize(q);
    for (int i = 0; i < q; ++i) lam[i] = A[(size_t)i * q + i];
}

gini_status ensure_select(gini_ctx* c, size_t bytes) {
    if (bytes <= c->sel_bytes) return GINI_OK;
    if (c->sel) {
        GINI_HIP(c, hipFree(c->sel));
        c->sel = nullptr;
        c->sel_bytes = 0;
    }
    if (hipMalloc(reinterpret_cast<void**>(&c->sel), bytes) != hipSuccess)
        return fail(c, GINI_ENOMEM, "select workspace of %zu bytes failed", bytes);
    c->sel_bytes = bytes;
    return GINI_OK;
}

gini_status ensure_ctl(gini_ctx* c, size_t n_inst) {
    if (n_inst <= c->ctl_cap && c->ctl) return GINI_OK;
    if (c->ctl) {
        GINI_HIP(c, hipDeviceSynchronize());
        (void)hipFree(c->ctl);
        (void)hipFree(c->epochs);
        c->ctl = nullptr;
    }
    size_t cap = std::max<size_t>(n_inst, 64);
    if (hipMalloc(reinterpret_cast<void**>(&c->ctl), sizeof(gmds::SolveCtl)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&c->epochs), cap * sizeof(uint32_t)) != hipSuccess)
        return fail(c, GINI_ENOMEM, "solve control allocation failed");
    c->ctl_cap = cap;
    return GINI_OK;
}

// Counter words for the fused reductions.  They are zero when no launch is in
// flight (every launch leaves them as it found them); fresh memory is zeroed
// on the stream before first use.
gini_status ensure_counters(gini_ctx* c, size_t words, hipStream_t s) {
    if (words <= c->cnt_cap && c->cnt) return GINI_OK;
    if (c->cnt) {
        GINI_HIP(c, hipDeviceSynchronize());
        (void)hipFree(c->cnt);
        c->cnt = nullptr;
    }
    size_t cap = std::max<size_t>(words, 4096);
    if (hipMalloc(reinterpret_cast<void**>(&c->cnt), cap * sizeof(uint32_t)) != hipSuccess)
        return fail(c, GINI_ENOMEM, "counter allocation failed");
    c->cnt_cap = cap;
    GINI_HIP(c, gmds::launch_fill_u32(c->cnt, (int64_t)cap, 0u, s));
    return GINI_OK;
}

// W_{d,nu}[t] for t = 2..2d (index t-2): ((t-2)/(2d))^(nu-1) - ((2d-t)/(2d))^(nu-1),
// the weight a coordinate of doubled midrank t receives in the symmetrised
// generalised Gini pseudo-distance.  Built in FP64 as A[t] - A[2d+2-t] so that
// the FP32 table is exactly antisymmetric, W[2d+2-t] == -W[t].
double weight_part(int d, double nu, int t) { return std::pow((double)(t - 2) / (2.0 * d), nu - 1.0); }

void weight_table(int d, double nu, double* out) {
    for (int t = 2; t <= 2 * d; ++t) out[t - 2] = weight_part(d, nu, t) - weight_part(d, nu, 2 * d + 2 - t);
}

gini_status get_tables(gini_ctx* c, int d, const double* nu, int n_nu, hipStream_t s, float** dev) {
    TableKey key{d, std::vector<double>(nu, nu + n_nu)};
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
        *dev = it->second;
        return GINI_OK;
    }
    const int len = 2 * d - 1;
    std::vector<float> host((size_t)len * n_nu);
    std::vector<double> w(len);
    for (int k = 0; k < n_nu; ++k) {
        weight_table(d, nu[k], w.data());
        for (int i = 0; i < len; ++i) host[(size_t)k * len + i] = (float)w[i];
    }
    float* p = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&p), host.size() * sizeof(float)) != hipSuccess)
        return fail(c, GINI_ENOMEM, "weight table allocation failed");
    GINI_HIP(c, hipMemcpy(p, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice));
    c->tables[key] = p;
    *dev = p;
    (void)s;
    return GINI_OK;
}

bool bad_nu(double nu) { return !std::isfinite(nu) || !(nu > 1.0); }

gini_status check_latent(gini_ctx* c, int32_t p, double nu, int latent) {
    if (latent != GINI_LATENT_GINI && latent != GINI_LATENT_EUCLID)
        return fail(c, GINI_EINVAL, "latent must be GINI_LATENT_GINI or GINI_LATENT_EUCLID");
    if (p < 1 || p > gmds::kMaxP) return fail(c, GINI_EINVAL, "p = %d outside 1..%d", p, gmds::kMaxP);
    if (latent == GINI_LATENT_GINI && p < 2)
        return fail(c, GINI_EINVAL, "the Gini latent distance needs p >= 2 (it is identically 0 for p = 1)");
    if (latent == GINI_LATENT_GINI && bad_nu(nu)) return fail(c, GINI_EINVAL, "nu must be finite and > 1");
    return GINI_OK;
}

// Latent-space constants: (p/2) W_{p,nu}[t] and the default step factor
// c = |d delta / d u|^2 at a tie-free u.
void latent_consts(int p, double nu, int latent, InstDesc& D, double& c) {
    for (int i = 0; i < 2 * gmds::kMaxP - 1; ++i) D.wtab[i] = 0.f;
    D.c2 = 0.f;
    c = 1.0;
    if (latent == GINI_LATENT_GINI) {
        double w[2 * gmds::kMaxP - 1];
        weight_table(p, nu, w);
        for (int i = 0; i < 2 * p - 1; ++i) D.wtab[i] = (float)(0.5 * p * w[i]);
        if (p == 2) D.c2 = D.wtab[2];
        c = 0.0;
        for (int k = 1; k <= p; ++k) {
            const double a = 0.5 * p * w[2 * k - 2];
            c += a * a;
        }
    }
}

// Default tile when the caller leaves the choice to the library.  128 wins on
// MI355X from n ~ 1000 up (measured at n = 10^4: 256-wide tiles need twice the
// column registers and fall to 2-3 waves per SIMD); the autotuner also tries
// 64 and 256.
int pick_tile(int64_t n) {
    return n <= 512 ? 64 : 128;
}

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Fill the layout fields of one stress descriptor for tile size T; returns
// its number of work units.
int64_t layout(InstDesc& D, int T) {
    D.nb = cdiv(D.n, T);
    D.vec = (aligned16(D.Delta) && (D.ldd % 4) == 0) ? 1 : 0;
    return gmds::tri_count(D.nb) * gmds::units_per_tile(T, D.p);
}

// Scratch floats of one instance: row partials, column partials, per-wave
// stress partials and the stress slices of the reduction (two floats for
// each of up to kSigSlices slices; assign_partials lays them out in order).
size_t partial_floats(const InstDesc& D, int T, int pg) {
    const int64_t nt = gmds::tri_count(D.nb);
    const int64_t u = gmds::units_per_tile(T, D.p);
    return (size_t)nt * T * pg + (size_t)nt * u * T * pg + (size_t)nt * u * gmds::kStressWaves * 2 +
           2 * (size_t)gmds::kSigSlices;
}

void assign_partials(InstDesc& D, float* base, int T, int pg) {
    const int64_t nt = gmds::tri_count(D.nb);
    const int64_t u = gmds::units_per_tile(T, D.p);
    D.rowpart = base;
    D.colpart = base + (size_t)nt * T * pg;
    D.sigpart = D.colpart + (size_t)nt * u * T * pg;
    D.sigslice = D.sigpart + (size_t)nt * u * gmds::kStressWaves * 2;
}

// Argument checks of one stress evaluation (host only, no HIP call).
gini_status check_stress_args(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* Z, int32_t p,
                              int64_t ldz, double nu, gini_latent latent, float* gradZ, int64_t ldg,
                              float* out_sigma, bool grad, int loss, const float* dsum) {
    if (loss == GINI_LOSS_SAMMON && !dsum) return fail(c, GINI_EINVAL, "delta_sum must be non-null");
    if (!Delta || !Z) return fail(c, GINI_EINVAL, "Delta and Z must be non-null");
    if (n < 2) return fail(c, GINI_EINVAL, "n = %lld: need at least two points", (long long)n);
    if (ldd < n) return fail(c, GINI_EINVAL, "ldd = %lld < n = %lld", (long long)ldd, (long long)n);
    gini_status st = check_latent(c, p, nu, latent);
    if (st != GINI_OK) return st;
    if (ldz < p) return fail(c, GINI_EINVAL, "ldz = %lld < p = %d", (long long)ldz, p);
    if (grad) {
        if (!gradZ) return fail(c, GINI_EINVAL, "gradZ must be non-null");
        if (ldg < p) return fail(c, GINI_EINVAL, "ldg = %lld < p = %d", (long long)ldg, p);
    } else if (!out_sigma) {
        return fail(c, GINI_EINVAL, "out_sigma must be non-null");
    }
    if ((uint64_t)n > (uint64_t)1 << 31) return fail(c, GINI_EUNSUPPORTED, "n > 2^31 is not supported");
    return GINI_OK;
}

// Descriptor of one stress evaluation at tile T (everything but the scratch
// pointers); returns its number of work units.
int64_t stress_desc(InstDesc& D, const float* Delta, int64_t n, int64_t ldd, const float* Z, int32_t p,
                    int64_t ldz, double nu, gini_latent latent, const float* grad_out, float* gradZ, int64_t ldg,
                    float* out_sigma, int loss, const float* dsum, int T) {
    D = InstDesc{};
    D.Delta = Delta;
    D.Z = const_cast<float*>(Z);
    D.gradZ = gradZ;
    D.grad_out = grad_out;
    D.out_sigma = out_sigma;
    D.loss = loss;
    D.dsum = dsum;
    D.n = n;
    D.ldd = ldd;
    D.ldz = ldz;
    D.ldg = ldg;
    D.p = p;
    double cc;
    latent_consts(p, nu, latent, D, cc);
    D.tile_off = 0;
    D.red_off = 0;
    return layout(D, T);
}

gini_status stress_common(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* Z, int32_t p,
                          int64_t ldz, double nu, gini_latent latent, const float* grad_out, float* gradZ,
                          int64_t ldg, float* out_sigma, bool grad, int loss, const float* dsum, hipStream_t s) {
    if (!c) return GINI_EINVAL;
    c->err.clear();
    gini_status st = check_stress_args(c, Delta, n, ldd, Z, p, ldz, nu, latent, gradZ, ldg, out_sigma, grad, loss,
                                       dsum);
    if (st != GINI_OK) return st;
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{Delta, "Delta"}, {Z, "Z"}, {gradZ, "gradZ"}, {out_sigma, "out_sigma"}, {grad_out, "grad_out"},
                       {dsum, "delta_sum"}});
    if (st != GINI_OK) return st;
    const int T = pick_tile(n);
    InstDesc D;
    const int64_t nt = stress_desc(D, Delta, n, ldd, Z, p, ldz, nu, latent, grad_out, gradZ, ldg, out_sigma, loss,
                                   dsum, T);
    if (nt > (int64_t)0x7fffffff) return fail(c, GINI_EUNSUPPORTED, "too many tiles");
    const int pg = gmds::stored_components(p, latent);
    st = ensure_scratch(c, partial_floats(D, T, pg) * sizeof(float));
    if (st != GINI_OK) return st;
    assign_partials(D, c->scratch, T, pg);
    st = ensure_counters(c, 1, s);
    if (st != GINI_OK) return st;
    D.instcnt = c->cnt;
    const int64_t rblocks = gmds::reduce_block_count(D.n, D.nb, T, D.p);
    void* dd = nullptr;
    Slot* sl = nullptr;
    st = upload(c, &D, sizeof D, s, &dd, &sl);
    if (st != GINI_OK) return st;
    const InstDesc* ddp = static_cast<const InstDesc*>(dd);
    {
        ProfScope ps(c, kProfTile, s, true);
        GINI_HIP(c, gmds::launch_stress_units(ddp, 1, nt, 0, p, latent, T, grad, loss, s, ps.timer()));
    }
    {
        ProfScope ps(c, kProfReduce, s, true);
        GINI_HIP(c, gmds::launch_stress_reduce(ddp, 1, rblocks, 0, p, latent, T,
                                               grad ? gmds::kModeGrad : gmds::kModeSigma, 0, n, s, ps.timer()));
    }
    return slot_done(c, sl, s);
}

// ------------------------------------------------------------------ solve
struct Plan {
    std::vector<InstDesc> desc;     // in queue (LPT) order
    std::vector<int> order;         // desc[k] is caller instance order[k]
    std::vector<int64_t> prefix;    // work-unit prefix, n_inst + 1
    int64_t tiles = 0;              // work units per iteration
    int64_t rblocks = 0;            // reduction blocks per iteration
    int64_t maxn = 0;               // largest instance
    std::vector<int32_t> bmap;      // instance of every reduction block (batched launches)
    int p = 0, latent = 0, T = 0, loss = 0;
};

gini_status validate_instances(gini_ctx* c, const gini_instance* inst, int32_t n_inst) {
    if (!inst) return fail(c, GINI_EINVAL, "inst must be non-null");
    if (n_inst < 1 || n_inst > 65536) return fail(c, GINI_EINVAL, "n_inst = %d outside 1..65536", n_inst);
    for (int k = 0; k < n_inst; ++k) {
        const gini_instance& I = inst[k];
        if (!I.Delta || !I.Z) return fail(c, GINI_EINVAL, "instance %d: Delta and Z must be non-null", k);
        if (I.n < 2) return fail(c, GINI_EINVAL, "instance %d: n = %lld < 2", k, (long long)I.n);
        if ((uint64_t)I.n > (uint64_t)1 << 31) return fail(c, GINI_EUNSUPPORTED, "instance %d: n too large", k);
        if (I.ldd < I.n) return fail(c, GINI_EINVAL, "instance %d: ldd < n", k);
        if (I.ldz < I.p) return fail(c, GINI_EINVAL, "instance %d: ldz < p", k);
        if (I.loss != GINI_LOSS_RAW && I.loss != GINI_LOSS_SAMMON)
            return fail(c, GINI_EINVAL, "instance %d: unknown loss %d", k, (int)I.loss);
        if (I.loss == GINI_LOSS_SAMMON && !I.delta_sum)
            return fail(c, GINI_EINVAL, "instance %d: the Sammon loss needs delta_sum", k);
        if (I.loss == GINI_LOSS_SAMMON && !(I.eta > 0.f))
            return fail(c, GINI_EINVAL, "instance %d: the Sammon loss needs eta > 0 (see gini_sammon_step)", k);
        if (I.loss == GINI_LOSS_SAMMON && I.ks_hist)
            return fail(c, GINI_EINVAL, "instance %d: ks_hist is defined for the raw stress only", k);
        if (!std::isfinite(I.eta)) return fail(c, GINI_EINVAL, "instance %d: eta not finite", k);
        if (I.ks_hist && !I.delta_sumsq)
            return fail(c, GINI_EINVAL, "instance %d: ks_hist needs delta_sumsq", k);
        gini_status st = check_latent(c, I.p, I.nu, I.latent);
        if (st != GINI_OK) return fail(c, st, "instance %d: %s", k, c->err.c_str());
        if (I.p != inst[0].p || I.latent != inst[0].latent || I.loss != inst[0].loss)
            return fail(c, GINI_EUNSUPPORTED, "instance %d: all instances of one call must share p, latent and loss",
                        k);
    }
    for (int k = 0; k < n_inst; ++k)
        for (int l = k + 1; l < n_inst && n_inst <= 4096; ++l) {
            if (inst[k].Z == inst[l].Z) return fail(c, GINI_EINVAL, "instances %d and %d share Z", k, l);
            if (inst[k].sigma_hist && inst[k].sigma_hist == inst[l].sigma_hist)
                return fail(c, GINI_EINVAL, "instances %d and %d share sigma_hist", k, l);
            if (inst[k].ks_hist && inst[k].ks_hist == inst[l].ks_hist)
                return fail(c, GINI_EINVAL, "instances %d and %d share ks_hist", k, l);
        }
    return GINI_OK;
}

gini_status make_plan(gini_ctx* c, const gini_instance* inst, int32_t n_inst, int T, Plan& P, hipStream_t s,
                      bool caller_order = false) {
    P.p = inst[0].p;
    P.latent = inst[0].latent;
    P.loss = inst[0].loss;
    P.T = T;
    P.order.resize(n_inst);
    std::iota(P.order.begin(), P.order.end(), 0);
    // largest first (LPT), ties by caller order
    if (!caller_order)
        std::stable_sort(P.order.begin(), P.order.end(), [&](int a, int b) { return inst[a].n > inst[b].n; });
    const int pg = gmds::stored_components(P.p, P.latent);
    P.desc.resize(n_inst);
    P.prefix.assign(n_inst + 1, 0);
    size_t floats = 0;
    for (int k = 0; k < n_inst; ++k) {
        const gini_instance& I = inst[P.order[k]];
        InstDesc& D = P.desc[k];
        D = InstDesc{};
        D.Delta = I.Delta;
        D.Z = I.Z;
        D.sigma_hist = I.sigma_hist;
        D.dsumsq = I.delta_sumsq;
        D.ks_hist = I.ks_hist;
        D.dsum = I.delta_sum;
        D.loss = I.loss;
        D.n = I.n;
        D.ldd = I.ldd;
        D.ldz = I.ldz;
        D.p = I.p;
        double cc;
        latent_consts(I.p, I.nu, I.latent, D, cc);
        D.eta = I.eta > 0.f ? I.eta : (float)(1.0 / (2.0 * (double)I.n * cc));
        const int64_t nt = layout(D, T);
        D.tile_off = P.prefix[k];
        P.prefix[k + 1] = P.prefix[k] + nt;
        D.red_off = P.rblocks;
        P.rblocks += gmds::reduce_block_count(D.n, D.nb, T, D.p);
        P.maxn = std::max(P.maxn, D.n);
        floats += partial_floats(D, T, pg);
        floats = (floats + 63) & ~size_t(63);
    }
    P.tiles = P.prefix[n_inst];
    if (n_inst > 1) {
        P.bmap.resize(P.rblocks);
        for (int k = 0; k < n_inst; ++k) {
            const int64_t b1 = k + 1 < n_inst ? P.desc[k + 1].red_off : P.rblocks;
            for (int64_t b = P.desc[k].red_off; b < b1; ++b) P.bmap[b] = k;
        }
    }
    if (P.tiles > (int64_t)0x7fffffff) return fail(c, GINI_EUNSUPPORTED, "too many tiles in one solve");
    gini_status st = ensure_scratch(c, floats * sizeof(float));
    if (st != GINI_OK) return st;
    st = ensure_counters(c, (size_t)n_inst, s);
    if (st != GINI_OK) return st;
    size_t off = 0;
    for (int k = 0; k < n_inst; ++k) {
        assign_partials(P.desc[k], c->scratch + off, T, pg);
        off += partial_floats(P.desc[k], T, pg);
        off = (off + 63) & ~size_t(63);
        P.desc[k].instcnt = c->cnt + k;
    }
    return GINI_OK;
}

__global__ void k_reset_ctl(gmds::SolveCtl* ctl, uint32_t* ep, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ctl->head = 0ull;
        ctl->status = 0u;
    }
    if (i < n) ep[i] = 0u;
}

gini_status ensure_side(gini_ctx* c) {
    if (c->side_fork) return GINI_OK;
    for (int g = 0; g < kSplitGroups - 1; ++g) {
        GINI_HIP(c, hipEventCreateWithFlags(&c->side_join[g], hipEventDisableTiming));
        GINI_HIP(c, hipStreamCreateWithFlags(&c->side[g], hipStreamNonBlocking));
    }
    GINI_HIP(c, hipEventCreateWithFlags(&c->side_fork, hipEventDisableTiming));
    return GINI_OK;
}

// Batched descent in kSplitGroups groups of instances, one stream each.
// Instances are dealt largest first to the group with the least work so far
// (work = stress units per iteration); each group gets descriptors with its
// own unit and reduction-block numbering, and its launches alternate with the
// other groups' on the host, so that the GPU runs one group's reduction beside
// the others' stress units.  An instance's partials, counters and sums are
// those of the one-group launch, so the results are bitwise the same.
gini_status run_split(gini_ctx* c, Plan& P, int iters, int red_wg, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    constexpr int NG = kSplitGroups;
    const int n_inst = (int)P.desc.size();
    const int ng = std::min(NG, n_inst);
    struct Group {
        std::vector<InstDesc> desc;
        std::vector<int32_t> bmap;
        int64_t tiles = 0, rblocks = 0, maxn = 0;
    } G[NG];
    for (int k = 0; k < n_inst; ++k) {
        int gi = 0;
        for (int g = 1; g < ng; ++g)
            if (G[g].tiles < G[gi].tiles) gi = g;
        Group& g = G[gi];
        InstDesc d = P.desc[k];
        const int64_t units = P.prefix[k + 1] - P.prefix[k];
        const int64_t rb = (k + 1 < n_inst ? P.desc[k + 1].red_off : P.rblocks) - P.desc[k].red_off;
        d.tile_off = g.tiles;
        d.red_off = g.rblocks;
        g.bmap.insert(g.bmap.end(), (size_t)rb, (int32_t)g.desc.size());
        g.desc.push_back(d);
        g.tiles += units;
        g.rblocks += rb;
        g.maxn = std::max(g.maxn, d.n);
    }
    // one upload: the descriptor arrays, then the block maps
    size_t off[2 * NG];
    size_t bytes = 0;
    for (int g = 0; g < ng; ++g) {
        off[g] = bytes;
        bytes = (bytes + G[g].desc.size() * sizeof(InstDesc) + 15) & ~size_t(15);
    }
    for (int g = 0; g < ng; ++g) {
        off[NG + g] = bytes;
        bytes += G[g].bmap.size() * sizeof(int32_t);
    }
    std::vector<unsigned char> blob(bytes);
    for (int g = 0; g < ng; ++g) {
        std::memcpy(blob.data() + off[g], G[g].desc.data(), G[g].desc.size() * sizeof(InstDesc));
        std::memcpy(blob.data() + off[NG + g], G[g].bmap.data(), G[g].bmap.size() * sizeof(int32_t));
    }
    gini_status st = ensure_side(c);
    if (st != GINI_OK) return st;
    void* dd = nullptr;
    Slot* sl = nullptr;
    st = upload(c, blob.data(), blob.size(), s, &dd, &sl);
    if (st != GINI_OK) return st;
    auto at = [&](size_t o) { return static_cast<unsigned char*>(dd) + o; };
    hipStream_t str[NG];
    str[0] = s;
    for (int g = 1; g < NG; ++g) str[g] = c->side[g - 1];
    if (ev0) GINI_HIP(c, hipEventRecord(ev0, s));
    GINI_HIP(c, hipEventRecord(c->side_fork, s));
    for (int g = 1; g < ng; ++g) GINI_HIP(c, hipStreamWaitEvent(str[g], c->side_fork, 0));
    for (int it = 0; it < iters; ++it) {
        for (int g = 0; g < ng; ++g) {
            const InstDesc* ddp = reinterpret_cast<const InstDesc*>(at(off[g]));
            const int32_t* bmap = reinterpret_cast<const int32_t*>(at(off[NG + g]));
            const int ni = (int)G[g].desc.size();
            {
                ProfScope ps(c, kProfTile, str[g], true);
                GINI_HIP(c, gmds::launch_stress_units(ddp, ni, G[g].tiles, 0, P.p, P.latent, P.T, true, P.loss,
                                                      str[g], ps.timer(), (it & 1) != 0));
            }
            ProfScope ps(c, kProfReduce, str[g], true);
            GINI_HIP(c, gmds::launch_stress_reduce(ddp, ni, G[g].rblocks, 0, P.p, P.latent, P.T, gmds::kModeDescent,
                                                   it, G[g].maxn, str[g], ps.timer(), bmap, red_wg));
        }
    }
    for (int g = 1; g < ng; ++g) {
        GINI_HIP(c, hipEventRecord(c->side_join[g - 1], str[g]));
        GINI_HIP(c, hipStreamWaitEvent(s, c->side_join[g - 1], 0));
    }
    if (ev1) GINI_HIP(c, hipEventRecord(ev1, s));
    return slot_done(c, sl, s);
}

// ev0/ev1 (optional) are recorded right before the first and after the last
// kernel launch, so that their interval holds only the solve's GPU work.
gini_status run_plan(gini_ctx* c, Plan& P, int iters, int mode, int grid, hipStream_t s, hipEvent_t ev0 = nullptr,
                     hipEvent_t ev1 = nullptr, bool split = false) {
    const int n_inst = (int)P.desc.size();
    // grid: the persistent launch's workgroups, else the threads of a
    // reduction workgroup (0 = by instance size)
    if (mode == GINI_SOLVE_BATCHED && split && n_inst > 1) return run_split(c, P, iters, grid, s, ev0, ev1);
    // one upload: descriptors, then the tile prefix
    const size_t dbytes = (P.desc.size() * sizeof(InstDesc) + 15) & ~size_t(15);
    const size_t pbytes = P.prefix.size() * sizeof(int64_t);
    std::vector<unsigned char> blob(dbytes + pbytes + P.bmap.size() * sizeof(int32_t));
    std::memcpy(blob.data(), P.desc.data(), P.desc.size() * sizeof(InstDesc));
    std::memcpy(blob.data() + dbytes, P.prefix.data(), pbytes);
    if (!P.bmap.empty()) std::memcpy(blob.data() + dbytes + pbytes, P.bmap.data(), P.bmap.size() * sizeof(int32_t));
    void* dd = nullptr;
    Slot* sl = nullptr;
    gini_status st = upload(c, blob.data(), blob.size(), s, &dd, &sl);
    if (st != GINI_OK) return st;
    const InstDesc* ddp = static_cast<const InstDesc*>(dd);
    const int64_t* dprefix = reinterpret_cast<const int64_t*>(static_cast<unsigned char*>(dd) + dbytes);
    const int32_t* dbmap = P.bmap.empty() ? nullptr
                                          : reinterpret_cast<const int32_t*>(static_cast<unsigned char*>(dd) + dbytes +
                                                                             pbytes);
    if (mode == GINI_SOLVE_PERSISTENT) {
        st = ensure_ctl(c, n_inst);
        if (st != GINI_OK) return st;
    }
    if (ev0) GINI_HIP(c, hipEventRecord(ev0, s));
    if (mode == GINI_SOLVE_PLAIN) {
        for (int k = 0; k < n_inst; ++k) {
            const int64_t nu = P.prefix[k + 1] - P.prefix[k];
            for (int it = 0; it < iters; ++it) {
                {
                    ProfScope ps(c, kProfTile, s, true);
                    GINI_HIP(c, gmds::launch_stress_units(ddp + k, 1, nu, P.desc[k].tile_off, P.p, P.latent, P.T,
                                                          true, P.loss, s, ps.timer(), (it & 1) != 0));
                }
                ProfScope ps(c, kProfReduce, s, true);
                GINI_HIP(c, gmds::launch_stress_reduce(ddp + k, 1,
                                                       gmds::reduce_block_count(P.desc[k].n, P.desc[k].nb, P.T, P.p),
                                                       P.desc[k].red_off, P.p, P.latent, P.T, gmds::kModeDescent, it,
                                                       P.desc[k].n, s, ps.timer(), nullptr, grid));
            }
        }
    } else if (mode == GINI_SOLVE_BATCHED) {
        for (int it = 0; it < iters; ++it) {
            {
                ProfScope ps(c, kProfTile, s, true);
                GINI_HIP(c, gmds::launch_stress_units(ddp, n_inst, P.tiles, 0, P.p, P.latent, P.T, true, P.loss, s,
                                                      ps.timer(), (it & 1) != 0));
            }
            ProfScope ps(c, kProfReduce, s, true);
            GINI_HIP(c, gmds::launch_stress_reduce(ddp, n_inst, P.rblocks, 0, P.p, P.latent, P.T,
                                                   gmds::kModeDescent, it, P.maxn, s, ps.timer(), dbmap, grid));
        }
    } else {
        hipLaunchKernelGGL(k_reset_ctl, dim3((n_inst + 255) / 256), dim3(256), 0, s, c->ctl, c->epochs, n_inst);
        GINI_HIP(c, hipGetLastError());
        int g = grid;
        if (g <= 0) g = c->cus * gmds::persistent_max_blocks_per_cu(P.p, P.latent, P.T, P.loss);
        const int64_t cap = P.tiles * (int64_t)iters;
        if (g > cap) g = (int)std::max<int64_t>(1, cap);
        ProfScope ps(c, kProfPersistent, s, true);
        GINI_HIP(c, gmds::launch_solve_persistent(ddp, n_inst, dprefix, P.tiles, iters, P.p, P.latent, P.T, P.loss, g,
                                                  c->ctl, c->epochs, c->spin_limit, s, ps.timer()));
    }
    if (ev1) GINI_HIP(c, hipEventRecord(ev1, s));
    st = slot_done(c, sl, s);
    if (st != GINI_OK) return st;
    // the other modes return once their launches are enqueued; the
    // persistent launch is waited for, to report an abort
    if (mode == GINI_SOLVE_PERSISTENT) {
        GINI_HIP(c, hipStreamSynchronize(s));
        gmds::SolveCtl h{};
        GINI_HIP(c, hipMemcpy(&h, c->ctl, sizeof h, hipMemcpyDeviceToHost));
        if (h.status != gmds::kStatusOk) {
            // the aborted launch left completion counters mid-count: clear them
            GINI_HIP(c, gmds::launch_fill_u32(c->cnt, (int64_t)c->cnt_cap, 0u, s));
            GINI_HIP(c, hipStreamSynchronize(s));
            return fail(c, GINI_EDEVICE, "persistent solve aborted: a dependency wait exceeded its time limit");
        }
    }
    return GINI_OK;
}

int solve_mode(int flags) {
    if (flags & GINI_SOLVE_PLAIN) return GINI_SOLVE_PLAIN;
    if (flags & GINI_SOLVE_BATCHED) return GINI_SOLVE_BATCHED;
    return GINI_SOLVE_PERSISTENT;
}

std::string tune_key(const gini_instance* inst, int32_t n_inst) {
    std::vector<int64_t> ns(n_inst);
    for (int k = 0; k < n_inst; ++k) ns[k] = inst[k].n;
    std::sort(ns.begin(), ns.end());
    std::string key = std::to_string(n_inst) + ":" + std::to_string(inst[0].p) + ":" + std::to_string(inst[0].latent);
    uint64_t h = 1469598103934665603ull;
    for (int64_t v : ns) {
        h ^= (uint64_t)v;
        h *= 1099511628211ull;
    }
    return key + ":" + std::to_string(h);
}

gini_status solve_impl(gini_ctx* c, const gini_instance* inst, int32_t n_inst, const gini_solve_opts* o,
                       hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

gini_status autotune_impl(gini_ctx* c, const gini_instance* inst, int32_t n_inst, int32_t probe_iters,
                          gini_solve_opts* best, hipStream_t s) {
    if (probe_iters < 1) probe_iters = 20;
    struct ProfPause {
        gini_ctx* c;
        bool was;
        explicit ProfPause(gini_ctx* c_) : c(c_), was(c_->prof) { c->prof = false; }
        ~ProfPause() { c->prof = was; }
    } pause(c);
    // private copies of the configurations; histories are not recorded
    std::vector<gini_instance> tmp(inst, inst + n_inst);
    std::vector<float*> zcopy(n_inst, nullptr);
    gini_status st = GINI_OK;
    for (int k = 0; k < n_inst && st == GINI_OK; ++k) {
        const size_t bytes = (size_t)((inst[k].n - 1) * inst[k].ldz + inst[k].p) * sizeof(float);
        if (hipMalloc(reinterpret_cast<void**>(&zcopy[k]), bytes) != hipSuccess) {
            st = fail(c, GINI_ENOMEM, "autotune: configuration copy failed");
            break;
        }
        tmp[k].Z = zcopy[k];
        tmp[k].sigma_hist = nullptr;
        tmp[k].ks_hist = nullptr;
    }
    std::vector<gini_solve_opts> cand;
    int64_t maxn = 0;
    for (int k = 0; k < n_inst; ++k) maxn = std::max(maxn, inst[k].n);
    // Per tile size: the batched launches (one stream with the instances
    // largest first or in the caller's order, and two streams, for several
    // instances) with reduction workgroups of 256 and 1024 threads.
    // The persistent solver pays a device-scope release (a writeback of the
    // XCD's L2) per work unit; it can only win when an iteration is one wave
    // of workgroups or less and launch latency dominates, so it is tried only
    // there.
    for (int T : {64, 128, 256}) {
        if (T > 64 && maxn <= T / 2) continue;
        for (int rw : {256, 1024}) {
            cand.push_back({probe_iters, GINI_SOLVE_BATCHED, T, rw});
            if (n_inst > 1) {
                cand.push_back({probe_iters, GINI_SOLVE_BATCHED | GINI_SOLVE_SPLIT, T, rw});
                cand.push_back({probe_iters, GINI_SOLVE_BATCHED | GINI_SOLVE_CALLER_ORDER, T, rw});
            }
        }
        int64_t units = 0;
        for (int k = 0; k < n_inst; ++k) {
            const int64_t nb = (inst[k].n + T - 1) / T;
            units += gmds::tri_count(nb) * gmds::units_per_tile(T, inst[k].p);
        }
        if (units > c->cus) continue;
        int nb = gmds::persistent_max_blocks_per_cu(inst[0].p, inst[0].latent, T, inst[0].loss);
        for (int g : {1, 2, 4, 8}) {
            if (g > nb) break;
            cand.push_back({probe_iters, GINI_SOLVE_PERSISTENT, T, g * c->cus});
        }
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == GINI_OK) {
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            st = fail(c, GINI_EDEVICE, "autotune: event creation failed");
    }
    float best_ms = 1e30f;
    gini_solve_opts best_o{0, GINI_SOLVE_PERSISTENT, 0, 0};
    constexpr int kReps = 4;                                   // first run warms up; best of the rest
    for (size_t ci = 0; ci < cand.size() && st == GINI_OK; ++ci) {
        float cand_ms = 1e30f;
        for (int rep = 0; rep < kReps && st == GINI_OK; ++rep) {
            for (int k = 0; k < n_inst && st == GINI_OK; ++k) {
                const size_t bytes = (size_t)((inst[k].n - 1) * inst[k].ldz + inst[k].p) * sizeof(float);
                if (hipMemcpyAsync(zcopy[k], inst[k].Z, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
                    st = fail(c, GINI_EDEVICE, "autotune: copy failed");
            }
            if (st != GINI_OK) break;
            st = solve_impl(c, tmp.data(), n_inst, &cand[ci], s, e0, e1);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (st == GINI_OK && rep > 0 && ms < cand_ms) cand_ms = ms;
        }
        if (st == GINI_OK && cand_ms < best_ms) {
            best_ms = cand_ms;
            best_o = cand[ci];
        }
    }
    (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (float* z : zcopy)
        if (z) (void)hipFree(z);
    if (st != GINI_OK) return st;
    best_o.iters = 0;
    c->tune[tune_key(inst, n_inst)] = TuneEntry{best_o};
    *best = best_o;
    return GINI_OK;
}

gini_status solve_impl(gini_ctx* c, const gini_instance* inst, int32_t n_inst, const gini_solve_opts* o,
                       hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    gini_solve_opts opts = *o;
    if (opts.flags & GINI_SOLVE_AUTOTUNE) {
        const std::string key = tune_key(inst, n_inst);
        auto it = c->tune.find(key);
        gini_solve_opts t{};
        if (it == c->tune.end()) {
            gini_status st = autotune_impl(c, inst, n_inst, 20, &t, s);
            if (st != GINI_OK) return st;
        } else {
            t = it->second.opts;
        }
        opts.flags = (opts.flags & GINI_SOLVE_CHECK_FINITE) | t.flags;
        opts.tile = t.tile;
        opts.grid = t.grid;
    }
    int64_t maxn = 0;
    for (int k = 0; k < n_inst; ++k) maxn = std::max(maxn, inst[k].n);
    const int T = opts.tile > 0 ? opts.tile : pick_tile(maxn);
    Plan P;
    gini_status st = make_plan(c, inst, n_inst, T, P, s, (opts.flags & GINI_SOLVE_CALLER_ORDER) != 0);
    if (st != GINI_OK) return st;
    if (opts.iters == 0) return GINI_OK;
    st = run_plan(c, P, opts.iters, solve_mode(opts.flags), opts.grid, s, ev0, ev1,
                  (opts.flags & GINI_SOLVE_SPLIT) != 0);
    if (st != GINI_OK) return st;
    if (opts.flags & GINI_SOLVE_CHECK_FINITE) {
        GINI_HIP(c, hipStreamSynchronize(s));
        std::vector<float> h(opts.iters);
        for (int k = 0; k < n_inst; ++k) {
            if (!inst[k].sigma_hist) continue;
            GINI_HIP(c, hipMemcpy(h.data(), inst[k].sigma_hist, h.size() * sizeof(float), hipMemcpyDeviceToHost));
            for (float v : h)
                if (!std::isfinite(v)) return fail(c, GINI_ENOTFINITE, "instance %d: stress is not finite", k);
        }
    }
    return GINI_OK;
}

gini_status check_opts(gini_ctx* c, const gini_solve_opts* o) {
    if (!o) return fail(c, GINI_EINVAL, "opts must be non-null");
    if (o->iters < 0) return fail(c, GINI_EINVAL, "iters < 0");
    const int modes = o->flags & (GINI_SOLVE_PERSISTENT | GINI_SOLVE_PLAIN | GINI_SOLVE_BATCHED);
    if (modes & (modes - 1)) return fail(c, GINI_EINVAL, "choose one of PERSISTENT, PLAIN, BATCHED");
    if (o->flags & ~(GINI_SOLVE_PERSISTENT | GINI_SOLVE_PLAIN | GINI_SOLVE_BATCHED | GINI_SOLVE_AUTOTUNE |
                     GINI_SOLVE_CHECK_FINITE | GINI_SOLVE_SPLIT | GINI_SOLVE_CALLER_ORDER))
        return fail(c, GINI_EINVAL, "unknown solve flag");
    if ((o->flags & GINI_SOLVE_SPLIT) && !(o->flags & GINI_SOLVE_BATCHED))
        return fail(c, GINI_EINVAL, "SPLIT needs BATCHED");
    if (o->tile != 0 && o->tile != 64 && o->tile != 128 && o->tile != 256)
        return fail(c, GINI_EINVAL, "tile must be 0, 64, 128 or 256");
    if (o->grid < 0) return fail(c, GINI_EINVAL, "grid < 0");
    if ((o->flags & (GINI_SOLVE_PLAIN | GINI_SOLVE_BATCHED)) && o->grid != 0 && o->grid != 256 && o->grid != 1024)
        return fail(c, GINI_EINVAL, "grid of a plain or batched solve (threads per reduction workgroup) must be 0, "
                                    "256 or 1024");
    return GINI_OK;
}

// ------------------------------------------------------- no-allocation path
// gini_stress_bwd_static takes its scratch from one static device array per
// GPU: [0, 256) the descriptor, [256, 512) the stress-slice counter, then the
// tile partials of gini_stress_bwd's layout.  The array's address is looked
// up once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels.
constexpr size_t kStaticScratchBytes = GINI_STATIC_SCRATCH_BYTES;
constexpr size_t kStaticCounter = 256;
constexpr size_t kStaticHead = 512;
constexpr int kMaxStaticDevices = 64;
static_assert(sizeof(InstDesc) <= kStaticCounter, "the descriptor must fit its slot");

std::once_flag g_static_once[kMaxStaticDevices];
unsigned char* g_static_ptr[kMaxStaticDevices];
hipError_t g_static_status[kMaxStaticDevices];

// Writes the descriptor (a kernel argument) into its slot and clears the
// counter, so nothing the array kept from an earlier call is read.
__global__ void k_put_desc(InstDesc D, InstDesc* dst, uint32_t* cnt) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *dst = D;
        *cnt = 0u;
    }
}

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

gini_status static_scratch(gini_ctx* c, unsigned char** base) {
    const int dev = c->device;
    if (dev >= kMaxStaticDevices) return fail(c, GINI_EUNSUPPORTED, "device %d: static scratch for devices < %d only",
                                              dev, kMaxStaticDevices);
    GINI_HIP(c, hipSetDevice(dev));
    std::call_once(g_static_once[dev], [dev] {
        g_static_status[dev] = hipGetSymbolAddress(reinterpret_cast<void**>(&g_static_ptr[dev]), HIP_SYMBOL(scratch));
    });
    if (g_static_status[dev] != hipSuccess) return hip_fail(c, g_static_status[dev], "hipGetSymbolAddress(scratch)");
    *base = g_static_ptr[dev];
    return GINI_OK;
}

}  // namespace

// ======================================================================= C ABI
// A named range around every compute entry point, which rocprofv3
// --marker-trace shows around the entry point's launches (a call into the
// ROCTx library that returns at once when no tool is attached).
struct TraceRange {
    explicit TraceRange(const char* name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange&) = delete;
    TraceRange& operator=(const TraceRange&) = delete;
};

extern "C" {

gini_status gini_create(gini_ctx** ctx, int device) {
    if (!ctx) return GINI_EINVAL;
    *ctx = nullptr;
    if (device < 0) return GINI_EINVAL;
    gini_ctx* c = new (std::nothrow) gini_ctx();
    if (!c) return GINI_ENOMEM;
    c->device = device;
    c->err.reserve(kErrCap);   // fail() then never reallocates the message
    if (const char* v = std::getenv("GINI_SPIN_LIMIT_TICKS")) {
        const long long t = std::atoll(v);
        if (t > 0) {
            c->spin_limit = t;
            c->spin_override = true;
        }
    }
    *ctx = c;
    return GINI_OK;
}

void gini_destroy(gini_ctx* c) {
    if (!c) return;
    if (c->ready) {
        (void)hipSetDevice(c->device);
        (void)hipDeviceSynchronize();
        for (auto& kv : c->tables) (void)hipFree(kv.second);
        if (c->scratch) (void)hipFree(c->scratch);
        if (c->ctl) {
            (void)hipFree(c->ctl);
            (void)hipFree(c->epochs);
        }
        if (c->cnt) (void)hipFree(c->cnt);
        if (c->sel) (void)hipFree(c->sel);
        if (c->cm_pin) (void)hipHostFree(c->cm_pin);
        for (hipEvent_t e : c->cm_ev)
            if (e) (void)hipEventDestroy(e);
        if (c->side_fork) (void)hipEventDestroy(c->side_fork);
        for (int g = 0; g < kSplitGroups - 1; ++g) {
            if (c->side_join[g]) (void)hipEventDestroy(c->side_join[g]);
            if (c->side[g]) (void)hipStreamDestroy(c->side[g]);
        }
        prof_clear(c);
        for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
        for (auto& sl : c->ring) {
            if (sl.host) (void)hipHostFree(sl.host);
            if (sl.dev) (void)hipFree(sl.dev);
            if (sl.done) (void)hipEventDestroy(sl.done);
        }
    }
    delete c;
}

const char* gini_last_error(const gini_ctx* c) { return c ? c->err.c_str() : "null context"; }

const char* gini_status_string(gini_status s) {
    switch (s) {
        case GINI_OK: return "GINI_OK";
        case GINI_EINVAL: return "GINI_EINVAL";
        case GINI_ENOMEM: return "GINI_ENOMEM";
        case GINI_EDEVICE: return "GINI_EDEVICE";
        case GINI_ENOTFINITE: return "GINI_ENOTFINITE";
        case GINI_EUNSUPPORTED: return "GINI_EUNSUPPORTED";
    }
    return "unknown gini_status";
}

int gini_version(void) { return kVersion; }

gini_status gini_weight_table(int32_t d, double nu, float* W) {
    if (!W || d < 1 || d > 65536 || bad_nu(nu)) return GINI_EINVAL;
    std::vector<double> w(2 * (size_t)d - 1);
    weight_table(d, nu, w.data());
    for (size_t i = 0; i < w.size(); ++i) W[i] = (float)w[i];
    return GINI_OK;
}

gini_status gini_rank(gini_ctx* c, const float* V, int64_t rows, int32_t d, int64_t ldv, int32_t* twoR, int64_t ldr,
                      gini_stream_t stream) {
    TraceRange trace_range("gini_rank");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (rows < 0) return fail(c, GINI_EINVAL, "rows < 0");
    if (d < 1 || d > kMaxRankD) return fail(c, GINI_EINVAL, "d = %d outside 1..%lld", d, (long long)kMaxRankD);
    if (ldv < d || ldr < d) return fail(c, GINI_EINVAL, "leading dimensions must be >= d");
    if (rows > 0 && (!V || !twoR)) return fail(c, GINI_EINVAL, "V and twoR must be non-null");
    if (rows > (int64_t)0x7fffffff) return fail(c, GINI_EUNSUPPORTED, "rows > 2^31 - 1");
    if (rows == 0) return GINI_OK;
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{V, "V"}, {twoR, "twoR"}});
    if (st != GINI_OK) return st;
    const int64_t words = gmds::rank_scratch_words(rows, d);
    if (words > 0) {
        st = ensure_scratch(c, (size_t)words * sizeof(uint32_t));
        if (st != GINI_OK) return st;
    }
    GINI_HIP(c, gmds::launch_rank(V, rows, d, ldv, twoR, ldr, reinterpret_cast<uint32_t*>(c->scratch),
                                  reinterpret_cast<hipStream_t>(stream)));
    return GINI_OK;
}

gini_status gini_dissim(gini_ctx* c, const float* X, int64_t n, int32_t m, int64_t ldx, const double* nu, int32_t n_nu,
                        float* Delta, int64_t ldd, int64_t stride_nu, gini_stream_t stream) {
    TraceRange trace_range("gini_dissim");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (n < 1) return fail(c, GINI_EINVAL, "n = %lld < 1", (long long)n);
    if (m < 1 || m > kMaxDissimM) return fail(c, GINI_EINVAL, "m = %d outside 1..%d", m, kMaxDissimM);
    if (!X || !Delta || !nu) return fail(c, GINI_EINVAL, "X, nu and Delta must be non-null");
    if (ldx < m) return fail(c, GINI_EINVAL, "ldx = %lld < m = %d", (long long)ldx, m);
    if (ldd < n) return fail(c, GINI_EINVAL, "ldd = %lld < n = %lld", (long long)ldd, (long long)n);
    if (n_nu < 1 || n_nu > gmds::kMaxNu) return fail(c, GINI_EINVAL, "n_nu = %d outside 1..%d", n_nu, gmds::kMaxNu);
    for (int k = 0; k < n_nu; ++k)
        if (bad_nu(nu[k])) return fail(c, GINI_EINVAL, "nu[%d] must be finite and > 1", k);
    if (n_nu > 1 && stride_nu < n * ldd)
        return fail(c, GINI_EINVAL, "stride_nu = %lld < n*ldd", (long long)stride_nu);
    if (n > (int64_t)1 << 22) return fail(c, GINI_EUNSUPPORTED, "n > 2^22 is not supported");
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{X, "X"}, {Delta, "Delta"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float* w = nullptr;
    st = get_tables(c, m, nu, n_nu, s, &w);
    if (st != GINI_OK) return st;
    gmds::DissimArgs a{};
    a.X = X;
    a.Delta = Delta;
    a.wtab = w;
    a.n = n;
    a.ldx = ldx;
    a.ldd = ldd;
    a.stride_nu = n_nu > 1 ? stride_nu : 0;
    a.m = m;
    a.n_nu = n_nu;
    a.half_m = 0.5f * (float)m;
    a.lin = 1;
    for (int k = 0; k < n_nu; ++k) a.lin = a.lin && nu[k] == 2.0;
    a.vecx = (aligned16(X) && (ldx % 4) == 0) ? 1 : 0;
    ProfScope ps(c, kProfDissim, s);
    GINI_HIP(c, gmds::launch_dissim(a, s));
    return GINI_OK;
}

static gini_status sum_common(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, int32_t n_mat,
                              int64_t stride, float* out, int power, gini_stream_t stream) {
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!Delta || !out) return fail(c, GINI_EINVAL, "Delta and out must be non-null");
    if (n < 1) return fail(c, GINI_EINVAL, "n = %lld < 1", (long long)n);
    if (ldd < n) return fail(c, GINI_EINVAL, "ldd = %lld < n = %lld", (long long)ldd, (long long)n);
    if (n_mat < 1 || n_mat > 65535) return fail(c, GINI_EINVAL, "n_mat = %d outside 1..65535", n_mat);
    if (n_mat > 1 && stride < n * ldd) return fail(c, GINI_EINVAL, "stride = %lld < n*ldd", (long long)stride);
    if (n > (int64_t)1 << 31) return fail(c, GINI_EUNSUPPORTED, "n too large");
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{Delta, "Delta"}, {out, "out"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    st = ensure_scratch(c, (size_t)2 * n_mat * std::max<int64_t>(1, gmds::sumsq_blocks(n)) * sizeof(float));
    if (st != GINI_OK) return st;
    GINI_HIP(c, gmds::launch_sumsq(Delta, n, ldd, n_mat, n_mat > 1 ? stride : 0, c->scratch, out, power, s));
    return GINI_OK;
}

gini_status gini_sumsq(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, int32_t n_mat, int64_t stride,
                       float* out, gini_stream_t stream) {
    TraceRange trace_range("gini_sumsq");
    return sum_common(c, Delta, n, ldd, n_mat, stride, out, 2, stream);
}

gini_status gini_sum(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, int32_t n_mat, int64_t stride,
                     float* out, gini_stream_t stream) {
    TraceRange trace_range("gini_sum");
    return sum_common(c, Delta, n, ldd, n_mat, stride, out, 1, stream);
}

gini_status gini_sammon_step(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, int32_t p, double nu,
                             gini_latent latent, double* eta, gini_stream_t stream) {
    TraceRange trace_range("gini_sammon_step");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!Delta || !eta) return fail(c, GINI_EINVAL, "Delta and eta must be non-null");
    if (n < 2) return fail(c, GINI_EINVAL, "n = %lld: need at least two points", (long long)n);
    if (ldd < n) return fail(c, GINI_EINVAL, "ldd = %lld < n = %lld", (long long)ldd, (long long)n);
    gini_status st = check_latent(c, p, nu, latent);
    if (st != GINI_OK) return st;
    if (n > (int64_t)1 << 31) return fail(c, GINI_EUNSUPPORTED, "n too large");
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{Delta, "Delta"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // scratch: [sum hi, lo][max row sum][pad][sum partials][row-max partials]
    const size_t sq = (size_t)2 * std::max<int64_t>(1, gmds::sumsq_blocks(n));
    const size_t rb = (size_t)gmds::rowinv_blocks(n);
    st = ensure_scratch(c, (4 + sq + rb) * sizeof(float));
    if (st != GINI_OK) return st;
    float* out = c->scratch;
    GINI_HIP(c, gmds::launch_sumsq(Delta, n, ldd, 1, 0, c->scratch + 4, out, 1, s));
    GINI_HIP(c, gmds::launch_rowinv_max(Delta, n, ldd, c->scratch + 4 + sq, out + 2, s));
    float h[3];
    GINI_HIP(c, hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, s));
    GINI_HIP(c, hipStreamSynchronize(s));
    InstDesc D{};
    double cc;
    latent_consts(p, nu, latent, D, cc);
    const double S = (double)h[0] + (double)h[1];
    *eta = (h[2] > 0.f && cc > 0.0) ? S / (4.0 * cc * (double)h[2]) : 0.0;
    return GINI_OK;
}

gini_status gini_stress_fwd(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* Z, int32_t p,
                            int64_t ldz, double nu, gini_latent latent, float* out_sigma, gini_stream_t stream) {
    TraceRange trace_range("gini_stress_fwd");
    return stress_common(c, Delta, n, ldd, Z, p, ldz, nu, latent, nullptr, nullptr, p, out_sigma, false,
                         GINI_LOSS_RAW, nullptr, reinterpret_cast<hipStream_t>(stream));
}

gini_status gini_stress_bwd(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* Z, int32_t p,
                            int64_t ldz, double nu, gini_latent latent, const float* grad_out, float* gradZ,
                            int64_t ldg, float* out_sigma, gini_stream_t stream) {
    TraceRange trace_range("gini_stress_bwd");
    return stress_common(c, Delta, n, ldd, Z, p, ldz, nu, latent, grad_out, gradZ, ldg, out_sigma, true,
                         GINI_LOSS_RAW, nullptr, reinterpret_cast<hipStream_t>(stream));
}

gini_status gini_stress_bwd_static(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* Z,
                                   int32_t p, int64_t ldz, double nu, gini_latent latent, const float* grad_out,
                                   float* gradZ, int64_t ldg, float* out_sigma, gini_stream_t stream) {
    TraceRange trace_range("gini_stress_bwd_static");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    gini_status st = check_stress_args(c, Delta, n, ldd, Z, p, ldz, nu, latent, gradZ, ldg, out_sigma, true,
                                       GINI_LOSS_RAW, nullptr);
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int T = pick_tile(n);
    InstDesc D;
    const int64_t nt = stress_desc(D, Delta, n, ldd, Z, p, ldz, nu, latent, grad_out, gradZ, ldg, out_sigma,
                                   GINI_LOSS_RAW, nullptr, T);
    const int pg = gmds::stored_components(p, latent);
    const size_t need = kStaticHead + partial_floats(D, T, pg) * sizeof(float);
    if (nt > (int64_t)0x7fffffff || need > kStaticScratchBytes)
        return fail(c, GINI_EUNSUPPORTED,
                    "n = %lld, p = %d needs %zu bytes of scratch; the static array holds %zu "
                    "(gini_stress_bwd has no such limit)",
                    (long long)n, p, need, kStaticScratchBytes);
    unsigned char* base = nullptr;
    st = static_scratch(c, &base);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{Delta, "Delta"}, {Z, "Z"}, {gradZ, "gradZ"}, {out_sigma, "out_sigma"}, {grad_out, "grad_out"}});
    if (st != GINI_OK) return st;
    assign_partials(D, reinterpret_cast<float*>(base + kStaticHead), T, pg);
    D.instcnt = reinterpret_cast<uint32_t*>(base + kStaticCounter);
    InstDesc* dd = reinterpret_cast<InstDesc*>(base);
    hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(64), 0, s, D, dd, D.instcnt);
    GINI_HIP(c, hipGetLastError());
    GINI_HIP(c, gmds::launch_stress_units(dd, 1, nt, 0, p, latent, T, true, GINI_LOSS_RAW, s));
    GINI_HIP(c, gmds::launch_stress_reduce(dd, 1, gmds::reduce_block_count(D.n, D.nb, T, D.p), 0, p, latent, T,
                                           gmds::kModeGrad, 0, D.n, s));
    return GINI_OK;
}

gini_status gini_sammon_fwd(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* delta_sum,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent, float* out_sigma,
                            gini_stream_t stream) {
    TraceRange trace_range("gini_sammon_fwd");
    return stress_common(c, Delta, n, ldd, Z, p, ldz, nu, latent, nullptr, nullptr, p, out_sigma, false,
                         GINI_LOSS_SAMMON, delta_sum, reinterpret_cast<hipStream_t>(stream));
}

gini_status gini_sammon_bwd(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, const float* delta_sum,
                            const float* Z, int32_t p, int64_t ldz, double nu, gini_latent latent,
                            const float* grad_out, float* gradZ, int64_t ldg, float* out_sigma, gini_stream_t stream) {
    TraceRange trace_range("gini_sammon_bwd");
    return stress_common(c, Delta, n, ldd, Z, p, ldz, nu, latent, grad_out, gradZ, ldg, out_sigma, true,
                         GINI_LOSS_SAMMON, delta_sum, reinterpret_cast<hipStream_t>(stream));
}

gini_status gini_mds_solve(gini_ctx* c, const gini_instance* inst, int32_t n_inst, const gini_solve_opts* opts,
                           gini_stream_t stream) {
    TraceRange trace_range("gini_mds_solve");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    gini_status st = check_opts(c, opts);
    if (st != GINI_OK) return st;
    st = validate_instances(c, inst, n_inst);
    if (st != GINI_OK) return st;
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev_instances(c, inst, n_inst);
    if (st != GINI_OK) return st;
    return solve_impl(c, inst, n_inst, opts, reinterpret_cast<hipStream_t>(stream));
}

gini_status gini_profile_enable(gini_ctx* c, int enable) {
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (c->ready) {
        gini_status st = ensure_ready(c);
        if (st != GINI_OK) return st;
        for (auto& v : c->prof_ev)
            for (auto& pr : v) (void)hipEventSynchronize(pr.second);
    }
    prof_clear(c);
    c->prof = enable != 0;
    return GINI_OK;
}

gini_status gini_profile_read(gini_ctx* c, gini_profile* out) {
    if (!c || !out) return GINI_EINVAL;
    c->err.clear();
    std::memset(out, 0, sizeof *out);
    if (!c->ready) return GINI_OK;
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    int64_t* cnt[4] = {&out->tile_launches, &out->reduce_launches, &out->persistent_launches, &out->dissim_launches};
    double* ms[4] = {&out->tile_ms, &out->reduce_ms, &out->persistent_ms, &out->dissim_ms};
    for (int k = 0; k < 4; ++k) {
        for (auto& pr : c->prof_ev[k]) {
            GINI_HIP(c, hipEventSynchronize(pr.second));
            float t = 0.f;
            // a launcher that had nothing to launch leaves its stamped events
            // unrecorded: such a pair is skipped
            if (hipEventElapsedTime(&t, pr.first, pr.second) != hipSuccess) {
                (void)hipGetLastError();
                continue;
            }
            *ms[k] += t;
            *cnt[k] += 1;
        }
    }
    prof_clear(c);
    return GINI_OK;
}

gini_status gini_autotune(gini_ctx* c, const gini_instance* inst, int32_t n_inst, int32_t probe_iters,
                          gini_solve_opts* best, gini_stream_t stream) {
    TraceRange trace_range("gini_autotune");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!best) return fail(c, GINI_EINVAL, "best must be non-null");
    if (probe_iters < 1 || probe_iters > 1000) return fail(c, GINI_EINVAL, "probe_iters outside 1..1000");
    gini_status st = validate_instances(c, inst, n_inst);
    if (st != GINI_OK) return st;
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev_instances(c, inst, n_inst);
    if (st != GINI_OK) return st;
    const int keep = best->flags & GINI_SOLVE_CHECK_FINITE;
    st = autotune_impl(c, inst, n_inst, probe_iters, best, reinterpret_cast<hipStream_t>(stream));
    if (st == GINI_OK) best->flags |= keep;
    return st;
}

// Raw stress of every instance (no gradient) into out_sigma[2k], [2k+1]:
// one stress-tile launch and one stress-only reduction for the whole batch.
static gini_status eval_sigma_batch(gini_ctx* c, const gini_instance* inst, int n_inst, int T, float* out_sigma,
                                    hipStream_t s) {
    Plan P;
    gini_status st = make_plan(c, inst, n_inst, T, P, s);
    if (st != GINI_OK) return st;
    for (int k = 0; k < n_inst; ++k) P.desc[k].out_sigma = out_sigma + 2 * P.order[k];
    void* dd = nullptr;
    Slot* sl = nullptr;
    st = upload(c, P.desc.data(), P.desc.size() * sizeof(InstDesc), s, &dd, &sl);
    if (st != GINI_OK) return st;
    const InstDesc* ddp = static_cast<const InstDesc*>(dd);
    {
        ProfScope ps(c, kProfTile, s, true);
        GINI_HIP(c, gmds::launch_stress_units(ddp, n_inst, P.tiles, 0, P.p, P.latent, T, false, P.loss, s,
                                              ps.timer()));
    }
    {
        ProfScope ps(c, kProfReduce, s, true);
        GINI_HIP(c, gmds::launch_stress_reduce(ddp, n_inst, P.rblocks, 0, P.p, P.latent, T, gmds::kModeSigma, 0,
                                               P.maxn, s, ps.timer()));
    }
    return slot_done(c, sl, s);
}

gini_status gini_select_nu(gini_ctx* c, const float* X, int64_t n, int32_t m, int64_t ldx, const double* nu,
                           int32_t n_nu, const float* Z0, int64_t ldz0, const gini_select_opts* o, float* Z_out,
                           int64_t ldzo, int64_t stride_z, double* ks_mean, double* ks_fold, int32_t* best,
                           gini_stream_t stream) {
    TraceRange trace_range("gini_select_nu");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!o) return fail(c, GINI_EINVAL, "opts must be non-null");
    if (!X || !nu || !Z0 || !Z_out || !ks_mean || !best)
        return fail(c, GINI_EINVAL, "X, nu, Z0, Z_out, ks_mean and best must be non-null");
    if (m < 1 || m > kMaxDissimM) return fail(c, GINI_EINVAL, "m = %d outside 1..%d", m, kMaxDissimM);
    if (ldx < m) return fail(c, GINI_EINVAL, "ldx = %lld < m = %d", (long long)ldx, m);
    if (n_nu < 1 || n_nu > gmds::kMaxNu) return fail(c, GINI_EINVAL, "n_nu = %d outside 1..%d", n_nu, gmds::kMaxNu);
    for (int k = 0; k < n_nu; ++k)
        if (bad_nu(nu[k])) return fail(c, GINI_EINVAL, "nu[%d] must be finite and > 1", k);
    if (o->folds < 1 || n < 2 * (int64_t)o->folds)
        return fail(c, GINI_EINVAL, "folds = %d with n = %lld: every fold needs at least two rows", o->folds,
                    (long long)n);
    if (o->iters < 1) return fail(c, GINI_EINVAL, "iters = %d < 1", o->iters);
    if ((int64_t)n_nu * o->folds > 65536) return fail(c, GINI_EINVAL, "n_nu * folds > 65536");
    gini_status st = check_latent(c, o->p, nu[0], o->latent);
    if (st != GINI_OK) return st;
    const int p = o->p;
    if (ldz0 < p || ldzo < p) return fail(c, GINI_EINVAL, "ldz0 and ldzo must be >= p = %d", p);
    if (n_nu > 1 && stride_z < n * ldzo) return fail(c, GINI_EINVAL, "stride_z = %lld < n*ldzo", (long long)stride_z);
    if (n > (int64_t)1 << 22) return fail(c, GINI_EUNSUPPORTED, "n > 2^22 is not supported");
    gini_solve_opts so{o->iters, o->flags, o->tile, 0};
    st = check_opts(c, &so);
    if (st != GINI_OK) return st;
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{X, "X"}, {Z0, "Z0"}, {Z_out, "Z_out"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // workspace: per fold, n_nu stacked n_f x ld_f matrices (rows on 256 B);
    // then the normalisers and the Euclidean stresses, (hi, lo) per fit
    const int K = o->folds;
    const int nfit = n_nu * K;
    std::vector<int64_t> start(K + 1), ld(K);
    std::vector<size_t> off(K);
    size_t floats = 0;
    for (int f = 0; f <= K; ++f) start[f] = (int64_t)f * n / K;
    for (int f = 0; f < K; ++f) {
        const int64_t nf = start[f + 1] - start[f];
        ld[f] = (nf + 63) / 64 * 64;
        off[f] = floats;
        floats += (size_t)n_nu * nf * ld[f];
        floats = (floats + 63) & ~size_t(63);
    }
    const size_t sumsq_off = floats;
    const size_t sig_off = floats + 2 * (size_t)nfit;
    floats += 4 * (size_t)nfit;
    st = ensure_select(c, floats * sizeof(float));
    if (st != GINI_OK) return st;
    float* ws = c->sel;

    // 1. dissimilarities of every fold for every nu (one ranking per pair),
    //    and their normalisers
    for (int f = 0; f < K; ++f) {
        const int64_t nf = start[f + 1] - start[f];
        float* Df = ws + off[f];
        st = gini_dissim(c, X + start[f] * ldx, nf, m, ldx, nu, n_nu, Df, ld[f], nf * ld[f], stream);
        if (st != GINI_OK) return st;
        st = gini_sumsq(c, Df, nf, ld[f], n_nu, nf * ld[f], ws + sumsq_off + 2 * (size_t)f * n_nu, stream);
        if (st != GINI_OK) return st;
    }
    // 2. every configuration starts from Z0
    for (int k = 0; k < n_nu; ++k)
        GINI_HIP(c, hipMemcpy2DAsync(Z_out + (size_t)k * stride_z, (size_t)ldzo * sizeof(float), Z0,
                                     (size_t)ldz0 * sizeof(float), (size_t)p * sizeof(float), (size_t)n,
                                     hipMemcpyDeviceToDevice, s));
    // 3. all nu x folds fits in one batched descent
    std::vector<gini_instance> inst(nfit);
    int64_t maxn = 0;
    for (int k = 0; k < n_nu; ++k)
        for (int f = 0; f < K; ++f) {
            const int64_t nf = start[f + 1] - start[f];
            gini_instance& I = inst[k * K + f];
            I = gini_instance{};
            I.n = nf;
            I.p = p;
            I.Delta = ws + off[f] + (size_t)k * nf * ld[f];
            I.ldd = ld[f];
            I.Z = Z_out + (size_t)k * stride_z + (size_t)start[f] * ldzo;
            I.ldz = ldzo;
            I.nu = nu[k];
            I.latent = o->latent;
            maxn = std::max(maxn, nf);
        }
    st = solve_impl(c, inst.data(), nfit, &so, s);
    if (st != GINI_OK) return st;
    // 4. raw stress of every fit with the Euclidean latent distance
    for (auto& I : inst) I.latent = GINI_LATENT_EUCLID;
    st = eval_sigma_batch(c, inst.data(), nfit, pick_tile(maxn), ws + sig_off, s);
    if (st != GINI_OK) return st;
    // 5. KS per fit, mean over folds, argmin over nu
    std::vector<float> h(4 * (size_t)nfit);
    GINI_HIP(c, hipMemcpyAsync(h.data(), ws + sumsq_off, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    GINI_HIP(c, hipStreamSynchronize(s));
    int bi = 0;
    for (int k = 0; k < n_nu; ++k) {
        double acc = 0.0;
        for (int f = 0; f < K; ++f) {
            const size_t q = (size_t)f * n_nu + k;                    // normaliser order: fold-major
            const double den = (double)h[2 * q] + (double)h[2 * q + 1];
            const size_t r = 2 * (size_t)nfit + 2 * ((size_t)k * K + f);
            const double sig = (double)h[r] + (double)h[r + 1];
            const double ks = den > 0.0 ? std::sqrt(sig / den) : 0.0;
            if (ks_fold) ks_fold[(size_t)k * K + f] = ks;
            acc += ks;
        }
        ks_mean[k] = acc / K;
        if (!std::isfinite(ks_mean[k])) return fail(c, GINI_ENOTFINITE, "Kruskal stress of nu[%d] is not finite", k);
        if (ks_mean[k] < ks_mean[bi]) bi = k;
    }
    *best = bi;
    return GINI_OK;
}

gini_status gini_alternate_nu(gini_ctx* c, const float* X, int64_t n, int32_t m, int64_t ldx, const double* nu,
                              int32_t n_nu, const float* Z0, int64_t ldz0, const gini_alternate_opts* o,
                              float* Z_out, int64_t ldzo, int32_t* nu_hist, double* ks, int32_t* best,
                              gini_stream_t stream) {
    TraceRange trace_range("gini_alternate_nu");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!o) return fail(c, GINI_EINVAL, "opts must be non-null");
    if (!X || !nu || !Z0 || !Z_out || !nu_hist || !best)
        return fail(c, GINI_EINVAL, "X, nu, Z0, Z_out, nu_hist and best must be non-null");
    if (n < 2) return fail(c, GINI_EINVAL, "n = %lld < 2", (long long)n);
    if (m < 1 || m > kMaxDissimM) return fail(c, GINI_EINVAL, "m = %d outside 1..%d", m, kMaxDissimM);
    if (ldx < m) return fail(c, GINI_EINVAL, "ldx = %lld < m = %d", (long long)ldx, m);
    if (n_nu < 1 || n_nu > gmds::kMaxNu) return fail(c, GINI_EINVAL, "n_nu = %d outside 1..%d", n_nu, gmds::kMaxNu);
    for (int k = 0; k < n_nu; ++k)
        if (bad_nu(nu[k])) return fail(c, GINI_EINVAL, "nu[%d] must be finite and > 1", k);
    if (o->iters < 1) return fail(c, GINI_EINVAL, "iters = %d < 1", o->iters);
    if (o->rounds < 1) return fail(c, GINI_EINVAL, "rounds = %d < 1", o->rounds);
    if (o->init < 0 || o->init >= n_nu) return fail(c, GINI_EINVAL, "init = %d outside 0..%d", o->init, n_nu - 1);
    gini_status st = check_latent(c, o->p, nu[0], o->latent);
    if (st != GINI_OK) return st;
    const int p = o->p;
    if (ldz0 < p || ldzo < p) return fail(c, GINI_EINVAL, "ldz0 and ldzo must be >= p = %d", p);
    if (n > (int64_t)1 << 22) return fail(c, GINI_EUNSUPPORTED, "n > 2^22 is not supported");
    gini_solve_opts so{o->iters, o->flags, o->tile, 0};
    st = check_opts(c, &so);
    if (st != GINI_OK) return st;
    st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{X, "X"}, {Z0, "Z0"}, {Z_out, "Z_out"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);

    // workspace: the n_nu matrices, then per nu (sum, sum of squares, Euclidean stress) as (hi, lo)
    const int64_t ld = (n + 63) / 64 * 64;
    const size_t mat = (size_t)n * ld;
    const size_t aux = (size_t)n_nu * mat;
    st = ensure_select(c, (aux + 6 * (size_t)n_nu) * sizeof(float));
    if (st != GINI_OK) return st;
    float* ws = c->sel;
    float* dsum = ws + aux;
    float* dsq = dsum + 2 * (size_t)n_nu;
    float* sig = dsq + 2 * (size_t)n_nu;
    st = gini_dissim(c, X, n, m, ldx, nu, n_nu, ws, ld, (int64_t)mat, stream);
    if (st != GINI_OK) return st;
    st = gini_sum(c, ws, n, ld, n_nu, (int64_t)mat, dsum, stream);
    if (st != GINI_OK) return st;
    st = gini_sumsq(c, ws, n, ld, n_nu, (int64_t)mat, dsq, stream);
    if (st != GINI_OK) return st;
    GINI_HIP(c, hipMemcpy2DAsync(Z_out, (size_t)ldzo * sizeof(float), Z0, (size_t)ldz0 * sizeof(float),
                                 (size_t)p * sizeof(float), (size_t)n, hipMemcpyDeviceToDevice, s));
    std::vector<float> hsq(2 * (size_t)n_nu);
    GINI_HIP(c, hipMemcpyAsync(hsq.data(), dsq, hsq.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    GINI_HIP(c, hipStreamSynchronize(s));
    std::vector<double> eta(n_nu, 0.0);
    std::vector<gini_instance> ev(n_nu);
    for (int k = 0; k < n_nu; ++k) {
        gini_instance& I = ev[k];
        I = gini_instance{};
        I.n = n;
        I.p = p;
        I.Delta = ws + (size_t)k * mat;
        I.ldd = ld;
        I.Z = Z_out;
        I.ldz = ldzo;
        I.nu = nu[k];
        I.latent = GINI_LATENT_EUCLID;
    }
    int cur = o->init;
    std::vector<float> hs(2 * (size_t)n_nu);
    for (int t = 0; t < o->rounds; ++t) {
        // 1. Sammon fit at the current nu, warm-started
        if (eta[cur] <= 0.0) {
            st = gini_sammon_step(c, ws + (size_t)cur * mat, n, ld, p, nu[cur], o->latent, &eta[cur], stream);
            if (st != GINI_OK) return st;
            if (!(eta[cur] > 0.0)) return fail(c, GINI_EINVAL, "nu[%d]: every dissimilarity is zero", cur);
        }
        gini_instance fit{};
        fit.n = n;
        fit.p = p;
        fit.loss = GINI_LOSS_SAMMON;
        fit.Delta = ws + (size_t)cur * mat;
        fit.ldd = ld;
        fit.Z = Z_out;
        fit.ldz = ldzo;
        fit.nu = nu[cur];
        fit.latent = o->latent;
        fit.eta = (float)eta[cur];
        fit.delta_sum = dsum + 2 * (size_t)cur;
        st = solve_impl(c, &fit, 1, &so, s);
        if (st != GINI_OK) return st;
        nu_hist[t] = cur;
        // 2. Kruskal stress of the fit against every nu, Euclidean latent distance
        st = eval_sigma_batch(c, ev.data(), n_nu, pick_tile(n), sig, s);
        if (st != GINI_OK) return st;
        GINI_HIP(c, hipMemcpyAsync(hs.data(), sig, hs.size() * sizeof(float), hipMemcpyDeviceToHost, s));
        GINI_HIP(c, hipStreamSynchronize(s));
        // 3. move to the argmin
        int bi = 0;
        double bv = 0.0;
        for (int k = 0; k < n_nu; ++k) {
            const double den = (double)hsq[2 * k] + (double)hsq[2 * k + 1];
            const double v = den > 0.0 ? std::sqrt(((double)hs[2 * k] + (double)hs[2 * k + 1]) / den) : 0.0;
            if (!std::isfinite(v)) return fail(c, GINI_ENOTFINITE, "round %d: Kruskal stress of nu[%d] is not finite", t, k);
            if (ks) ks[(size_t)t * n_nu + k] = v;
            if (k == 0 || v < bv) {
                bv = v;
                bi = k;
            }
        }
        cur = bi;
    }
    *best = cur;
    return GINI_OK;
}

gini_status gini_classical_mds(gini_ctx* c, const float* Delta, int64_t n, int64_t ldd, int32_t p, int32_t max_iters,
                               double tol, float* Z, int64_t ldz, double* eigvals, int32_t* iters_done,
                               gini_stream_t stream) {
    TraceRange trace_range("gini_classical_mds");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!Delta || !Z) return fail(c, GINI_EINVAL, "Delta and Z must be non-null");
    if (n < 2) return fail(c, GINI_EINVAL, "n = %lld < 2", (long long)n);
    if (ldd < n) return fail(c, GINI_EINVAL, "ldd = %lld < n = %lld", (long long)ldd, (long long)n);
    if (p < 1 || p > gmds::kMaxCmdsQ || p > n - 1)
        return fail(c, GINI_EINVAL, "p = %d outside 1..min(%d, n-1)", p, gmds::kMaxCmdsQ);
    if (ldz < p) return fail(c, GINI_EINVAL, "ldz = %lld < p = %d", (long long)ldz, p);
    if (max_iters < 1) return fail(c, GINI_EINVAL, "max_iters = %d < 1", max_iters);
    if (!(tol >= 0.0)) return fail(c, GINI_EINVAL, "tol must be >= 0");
    if (n > (int64_t)1 << 31) return fail(c, GINI_EUNSUPPORTED, "n too large");
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{Delta, "Delta"}, {Z, "Z"}});
    if (st != GINI_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int q = (int)std::min<int64_t>({(int64_t)gmds::kMaxCmdsQ, (int64_t)p + 4, n - 1});
    const int Q = gmds::kMaxCmdsQ;
    constexpr int kSlots = 4;                  // Rayleigh-Ritz matrices in flight (ring)
    constexpr int kVRing = 3;                  // blocks V_t kept: the one being checked and two ahead
    // workspace: the V ring, Y = D^2 V in FP64 (two FP32 blocks Yp, Yh while
    // the start block is formed), then small buffers
    const size_t nq = ((size_t)n * q + 63) & ~size_t(63);
    const size_t small = 2 * (size_t)Q * Q * 2 + 2 * (size_t)Q * Q;
    const size_t partf = (size_t)std::max<int64_t>(gmds::gram_part_floats(), 2 * gmds::step_part_doubles());
    const size_t dsmall = 2 * ((size_t)Q * Q + Q);
    st = ensure_select(c, ((kVRing + 2) * nq + small + partf + dsmall + 64) * sizeof(float));
    if (st != GINI_OK) return st;
    if (!c->cm_pin) {
        if (hipHostMalloc(reinterpret_cast<void**>(&c->cm_pin), 2 * (size_t)Q * Q * kSlots * sizeof(float),
                          hipHostMallocDefault) != hipSuccess)
            return fail(c, GINI_ENOMEM, "pinned landing buffer of classical MDS failed");
        GINI_HIP(c, hipHostGetDevicePointer(reinterpret_cast<void**>(&c->cm_pin_dev), c->cm_pin, 0));
        for (auto& e : c->cm_ev) GINI_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    float* Vr[kVRing];
    for (int k = 0; k < kVRing; ++k) Vr[k] = c->sel + k * nq;
    double* Yd = reinterpret_cast<double*>(c->sel + kVRing * nq);
    float* Yp = c->sel + kVRing * nq;              // start only (the memory of Yd)
    float* Yh = Yp + nq;
    float* gout = Yh + nq;                         // column sums (hi, lo)
    float* gG = gout + 2 * (size_t)Q * Q;          // Gram matrix (hi, lo)
    float* Mdev = gG + 2 * (size_t)Q * Q;          // orthonormalising map, q x q
    float* Idev = Mdev + (size_t)Q * Q;            // identity, q x q
    float* part = Idev + (size_t)Q * Q;            // Gram partials (FP32 start, FP64 steps)
    double* Md = reinterpret_cast<double*>(part + partf);   // the step's map, q x q
    double* meand = Md + (size_t)Q * Q;                       // and its column means
    {
        std::vector<float> I((size_t)q * q, 0.f);
        for (int i = 0; i < q; ++i) I[(size_t)i * q + i] = 1.f;
        void* dI = nullptr;
        Slot* sl = nullptr;
        st = upload(c, I.data(), I.size() * sizeof(float), s, &dI, &sl);
        if (st != GINI_OK) return st;
        GINI_HIP(c, hipMemcpyAsync(Idev, dI, I.size() * sizeof(float), hipMemcpyDeviceToDevice, s));
        st = slot_done(c, sl, s);
        if (st != GINI_OK) return st;
    }
    // start: a fixed pseudo-random block, made on the device, centred and
    // orthonormalised (Cholesky of its Gram matrix, on the device)
    {
        GINI_HIP(c, gmds::launch_start_block(Yp, n * q, s));
        GINI_HIP(c, gmds::launch_gram(Yp, q, nullptr, 1, n, part, gout, s));
        GINI_HIP(c, gmds::launch_rowmat(Yp, q, gout, 1.f, Idev, q, n, Yh, q, s));
        GINI_HIP(c, gmds::launch_gram(Yh, q, Yh, q, n, part, gG, s));
        GINI_HIP(c, gmds::launch_chol_orth(gG, q, Mdev, s));
        GINI_HIP(c, gmds::launch_rowmat(Yh, q, nullptr, 1.f, Mdev, q, n, Vr[0], q, s));
    }
    // Step t on the device: Y = D^2 V_t in FP64 (one pass over Delta), then
    // from FP64 sums over the rows of Y and V_t the Rayleigh-Ritz matrix
    // T_t = V_t^T B V_t (stored into the pinned host ring), the Gram matrix of
    // B V_t = -1/2 H Y and V_{t+1} = (B V_t) R^-1 from its Cholesky factor.
    // The host checks step t while step t+1 runs, so the GPU never waits for
    // it; V_t stays in the ring until then.
    auto enqueue = [&](int t) -> gini_status {
        const float* V = Vr[t % kVRing];
        // T_t is stored by the step kernel straight into its pinned landing slot
        double* T = reinterpret_cast<double*>(c->cm_pin_dev + 2 * (size_t)Q * Q * (t % kSlots));
        GINI_HIP(c, gmds::launch_d2v(Delta, n, ldd, V, q, Yd, s, (t & 1) != 0));
        GINI_HIP(c, gmds::launch_subspace_step(Yd, V, q, n, reinterpret_cast<double*>(part), T, Md, meand,
                                               Vr[(t + 1) % kVRing], s));
        GINI_HIP(c, hipEventRecord(c->cm_ev[t % kSlots], s));
        return GINI_OK;
    };
    std::vector<double> lam, W, prev;
    int enq = 0, chk = 0;
    for (;;) {
        while (enq < max_iters && enq <= chk + 1) {
            st = enqueue(enq++);
            if (st != GINI_OK) return st;
        }
        GINI_HIP(c, hipEventSynchronize(c->cm_ev[chk % kSlots]));
        const double* g = reinterpret_cast<const double*>(c->cm_pin + 2 * (size_t)Q * Q * (chk % kSlots));
        std::vector<double> T(g, g + (size_t)q * q);
        for (int i = 0; i < q; ++i)
            for (int j = 0; j < i; ++j)
                T[(size_t)i * q + j] = T[(size_t)j * q + i] = 0.5 * (T[(size_t)i * q + j] + T[(size_t)j * q + i]);
        jacobi_eig(q, T, lam, W);
        std::vector<double> top(lam);
        std::sort(top.begin(), top.end(), std::greater<double>());
        top.resize(p);
        bool done = chk + 1 >= max_iters;
        if (!prev.empty()) {
            double scale = 0.0, diff = 0.0;
            for (int k = 0; k < p; ++k) {
                scale = std::max(scale, std::fabs(top[k]));
                diff = std::max(diff, std::fabs(top[k] - prev[k]));
            }
            done = done || diff <= tol * scale;
        }
        prev = top;
        if (done) break;
        ++chk;
    }
    // the p Ritz pairs of step chk with the largest eigenvalues: Z = V_chk W_p diag(sqrt(max(lam, 0)))
    std::vector<int> idx(q);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a2, int b2) { return lam[a2] > lam[b2]; });
    std::vector<float> M((size_t)q * p, 0.f);
    for (int k = 0; k < p; ++k) {
        const int j = idx[k];
        const double sc = std::sqrt(std::max(lam[j], 0.0));
        for (int i = 0; i < q; ++i) M[(size_t)i * p + k] = (float)(W[(size_t)i * q + j] * sc);
        if (eigvals) eigvals[k] = lam[j];
    }
    void* dM = nullptr;
    Slot* sl = nullptr;
    st = upload(c, M.data(), M.size() * sizeof(float), s, &dM, &sl);
    if (st != GINI_OK) return st;
    GINI_HIP(c, gmds::launch_rowmat(Vr[chk % kVRing], q, nullptr, 1.f, static_cast<const float*>(dM), p, n, Z, ldz,
                                    s));
    st = slot_done(c, sl, s);
    if (st != GINI_OK) return st;
    GINI_HIP(c, hipStreamSynchronize(s));
    if (iters_done) *iters_done = chk + 1;
    for (int k = 0; k < p; ++k)
        if (eigvals && !std::isfinite(eigvals[k])) return fail(c, GINI_ENOTFINITE, "eigenvalue %d is not finite", k);
    return GINI_OK;
}

gini_status gini_standardize(gini_ctx* c, const float* X, int64_t n, int32_t m, int64_t ldx, float* Y, int64_t ldy,
                             float* stats, gini_stream_t stream) {
    TraceRange trace_range("gini_standardize");
    if (!c) return GINI_EINVAL;
    c->err.clear();
    if (!X || !Y) return fail(c, GINI_EINVAL, "X and Y must be non-null");
    if (n < 1) return fail(c, GINI_EINVAL, "n = %lld < 1", (long long)n);
    if (m < 1) return fail(c, GINI_EINVAL, "m = %d < 1", m);
    if (ldx < m || ldy < m) return fail(c, GINI_EINVAL, "ldx and ldy must be >= m = %d", m);
    if (X == Y && ldx != ldy) return fail(c, GINI_EINVAL, "in place needs ldy == ldx");
    if (n > ((int64_t)1 << 32) - 1) return fail(c, GINI_EUNSUPPORTED, "n too large");
    if (m > 65535) return fail(c, GINI_EUNSUPPORTED, "m > 65535 is not supported");
    gini_status st = ensure_ready(c);
    if (st != GINI_OK) return st;
    st = check_dev(c, {{X, "X"}, {Y, "Y"}, {stats, "stats"}});
    if (st != GINI_OK) return st;
    GINI_HIP(c, gmds::launch_standardise(X, n, m, ldx, Y, ldy, stats, reinterpret_cast<hipStream_t>(stream)));
    return GINI_OK;
}

}  // extern "C"
